// nbr.hip -- GPU cell-list neighbour list (full list, periodic images, skin).
//
// The descriptor of atom i needs every (atom, image) entry within the cutoff
// (Sec. II B, Eqs. 3 and 6); the paper attributes the speed gap between its two
// MD interfaces to how this list is built (Sec. IV).  Here atoms of each
// structure are binned into cells of edge >= the list radius, and every atom
// scans the 27 cells around its own in *unwrapped* cell coordinates: each
// (cell, image shift) pair is visited at most once, so edges shorter than twice
// the cutoff are handled exactly (several images of one atom can be neighbours).
//
// Rows are deterministic: cells are sorted by atom index and scanned in a
// fixed order.  A row holds first the entries within R_a + skin (the angular
// candidates), then the remaining ones within max(R_r, R_a) + skin; both
// parts are ordered by (stencil cell, atom).  That order makes the reverse
// entry (j -> i, -s) of every (i -> j, s) findable by binary search, which the
// deterministic force gather uses instead of atomics.
#include "aenet_internal.h"

namespace aenet {

namespace {

__device__ inline double wrap_coord(double x, double L) {
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w = 0.0;
  return w;
}

__device__ inline bool skip(const NbrParams& p) { return p.cond && *p.cond == 0; }

__device__ inline void cell_coords(const BoxInfo& b, int cell, int c[3]) {
  int local = cell - b.cell_base;
  c[0] = local % b.nc[0];
  c[1] = (local / b.nc[0]) % b.nc[1];
  c[2] = local / (b.nc[0] * b.nc[1]);
}

__device__ inline int stencil_index(int ox, int oy, int oz) {
  return (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1);
}

__global__ void k_set_int(int* dst, int v) {
  if (threadIdx.x == 0) *dst = v;
}

__global__ void k_zero(NbrParams p) {
  if (skip(p)) return;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < p.n_cells) {
    p.cell_count[c] = 0;
    p.cell_fill[c] = 0;
  }
  if (c == 0) {
    p.maxcnt[0] = 0;
    p.maxcnt[1] = 0;
  }
}

__global__ void k_bin(NbrParams p) {
  if (skip(p)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  const BoxInfo b = p.boxes[p.seg[i]];
  int c[3];
  for (int a = 0; a < 3; ++a) {
    double x = p.pos[3 * (size_t)i + a];
    if (p.pbc[a]) {
      x = wrap_coord(x, b.L[a]);
      p.pos[3 * (size_t)i + a] = x;
    }
    p.pos_ref[3 * (size_t)i + a] = x;
    double fc = floor(x * (double)b.nc[a] / b.L[a]);
    fc = fmin(fmax(fc, 0.0), (double)(b.nc[a] - 1));
    c[a] = (int)fc;
  }
  int cell = b.cell_base + (c[2] * b.nc[1] + c[1]) * b.nc[0] + c[0];
  p.atom_cell[i] = cell;
  atomicAdd(&p.cell_count[cell], 1);
}

// exclusive scan of cell counts, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan(NbrParams p) {
  if (skip(p)) return;
  __shared__ int s[1024];
  const int n = p.n_cells;
  const int t = threadIdx.x;
  const int per = (n + 1023) / 1024;
  const int lo = min(t * per, n), hi = min(lo + per, n);
  int sum = 0;
  for (int k = lo; k < hi; ++k) sum += p.cell_count[k];
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  int run = t ? s[t - 1] : 0;
  for (int k = lo; k < hi; ++k) {
    p.cell_start[k] = run;
    run += p.cell_count[k];
  }
  if (t == 1023) p.cell_start[n] = s[1023];
}

__global__ void k_scatter(NbrParams p) {
  if (skip(p)) return;
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= p.n) return;
  int cell = p.atom_cell[i];
  int slot = atomicAdd(&p.cell_fill[cell], 1);
  p.cell_atoms[p.cell_start[cell] + slot] = i;
}

// the scatter order depends on atomics; sorting each cell makes rows deterministic
__global__ void k_sort_cells(NbrParams p) {
  if (skip(p)) return;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= p.n_cells) return;
  int* a = p.cell_atoms + p.cell_start[c];
  const int m = p.cell_count[c];
  for (int k = 1; k < m; ++k) {
    int v = a[k];
    int j = k - 1;
    while (j >= 0 && a[j] > v) {
      a[j + 1] = a[j];
      --j;
    }
    a[j + 1] = v;
  }
}

// one wavefront per atom
__global__ __launch_bounds__(256) void k_rows(NbrParams p) {
  if (skip(p)) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= p.n) return;  // uniform per wave
  const BoxInfo b = p.boxes[p.seg[i]];
  int ci[3];
  cell_coords(b, p.atom_cell[i], ci);
  const double xi0 = p.pos[3 * (size_t)i], xi1 = p.pos[3 * (size_t)i + 1], xi2 = p.pos[3 * (size_t)i + 2];
  uint32_t* row = p.nbr + (size_t)i * p.cap;
  int count = 0, count_ang = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int oz = -1; oz <= 1; ++oz)
      for (int oy = -1; oy <= 1; ++oy)
        for (int ox = -1; ox <= 1; ++ox) {
          const int o[3] = {ox, oy, oz};
          int w[3], s[3];
          bool out = false;
          for (int a = 0; a < 3; ++a) {
            int u = ci[a] + o[a];
            if (p.pbc[a]) {
              s[a] = u < 0 ? -1 : (u >= b.nc[a] ? 1 : 0);
              w[a] = u - s[a] * b.nc[a];
            } else {
              s[a] = 0;
              w[a] = u;
              out |= (u < 0 || u >= b.nc[a]);
            }
          }
          if (out) continue;
          const int cell = b.cell_base + (w[2] * b.nc[1] + w[1]) * b.nc[0] + w[0];
          const int start = p.cell_start[cell], cnt = p.cell_count[cell];
          const int code = (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1);
          // canonical orientation of the self-image pair: lexicographically positive shift
          const bool spos = s[2] > 0 || (s[2] == 0 && (s[1] > 0 || (s[1] == 0 && s[0] > 0)));
          for (int base = 0; base < cnt; base += 64) {
            const int k = base + lane;
            bool take = false;
            int q = 0;
            if (k < cnt) {
              q = p.cell_atoms[start + k];
              const bool self = (q == i) && code == 13;
              if (!self) {
                // displacement computed from the lower-index atom, so that the
                // entry and its reverse agree bit for bit on r^2
                const bool iq = (i < q) || (i == q && spos);
                const size_t ia = iq ? (size_t)i : (size_t)q;
                const size_t ib = iq ? (size_t)q : (size_t)i;
                const double sg = iq ? 1.0 : -1.0;
                double d0 = p.pos[3 * ib] + sg * (double)s[0] * b.L[0] - p.pos[3 * ia];
                double d1 = p.pos[3 * ib + 1] + sg * (double)s[1] * b.L[1] - p.pos[3 * ia + 1];
                double d2 = p.pos[3 * ib + 2] + sg * (double)s[2] * b.L[2] - p.pos[3 * ia + 2];
                double r2 = d0 * d0 + d1 * d1 + d2 * d2;
                if (r2 == 0.0) atomicOr(p.flags, kFlagOverlap);
                const bool ang = r2 < p.r_ang2;
                take = pass == 0 ? ang : (!ang && r2 < p.r_list2);
              }
            }
            const uint64_t m = __ballot(take);
            if (take) {
              const int at = count + __popcll(m & ((1ull << lane) - 1ull));
              if (at < p.cap) row[at] = (uint32_t)q | ((uint32_t)code << kImgBits);
            }
            count += __popcll(m);
          }
        }
    if (pass == 0) count_ang = count;
  }
  (void)xi0;
  (void)xi1;
  (void)xi2;
  if (lane == 0) {
    if (count > p.cap || count_ang > p.cap_ang) atomicOr(p.flags, kFlagOverflow);
    // clamp so that every later kernel stays inside the row even after an overflow
    const int nang = min(count_ang, min(p.cap_ang, p.cap));
    p.nnb[i] = max(min(count, p.cap), nang);
    p.nang[i] = nang;
    atomicMax(&p.maxcnt[0], count);
    atomicMax(&p.maxcnt[1], count_ang);
  }
}

__device__ inline uint32_t entry_key(const NbrParams& p, const BoxInfo& b, const int cc[3],
                                     uint32_t en) {
  const int x = (int)(en & kAtomMask);
  const int code = (int)(en >> kImgBits);
  const int s[3] = {code % 3 - 1, (code / 3) % 3 - 1, code / 9 - 1};
  int cx[3];
  cell_coords(b, p.atom_cell[x], cx);
  int o[3];
  for (int a = 0; a < 3; ++a) o[a] = cx[a] - cc[a] + s[a] * b.nc[a];
  return ((uint32_t)stencil_index(o[0], o[1], o[2]) << kImgBits) | (uint32_t)x;
}

// reverse entry of every row entry, one wavefront per atom
__global__ __launch_bounds__(256) void k_reverse(NbrParams p) {
  if (skip(p)) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= p.n) return;
  const BoxInfo b = p.boxes[p.seg[i]];
  int ci[3];
  cell_coords(b, p.atom_cell[i], ci);
  const int nn = p.nnb[i], na = p.nang[i];
  const uint32_t* row = p.nbr + (size_t)i * p.cap;
  for (int e = lane; e < nn; e += 64) {
    const uint32_t en = row[e];
    const int q = (int)(en & kAtomMask);
    const int code = (int)(en >> kImgBits);
    const int s[3] = {code % 3 - 1, (code / 3) % 3 - 1, code / 9 - 1};
    int cq[3];
    cell_coords(b, p.atom_cell[q], cq);
    int o[3];
    for (int a = 0; a < 3; ++a) o[a] = cq[a] - ci[a] + s[a] * b.nc[a];
    const uint32_t key = ((uint32_t)stencil_index(-o[0], -o[1], -o[2]) << kImgBits) | (uint32_t)i;
    const uint32_t* rq = p.nbr + (size_t)q * p.cap;
    int lo, hi;
    if (e < na) {
      lo = 0;
      hi = p.nang[q];
    } else {
      lo = p.nang[q];
      hi = p.nnb[q];
    }
    int found = -1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const uint32_t km = entry_key(p, b, cq, rq[mid]);
      if (km == key) {
        found = mid;
        break;
      }
      if (km < key) lo = mid + 1; else hi = mid;
    }
    if (found < 0) {
      atomicOr(p.flags, kFlagReverse);
      p.rev[(size_t)i * p.cap + e] = -1;
    } else {
      p.rev[(size_t)i * p.cap + e] = q * p.cap + found;
    }
  }
}

inline int blocks_for(int64_t n, int threads) { return (int)((n + threads - 1) / threads); }

}  // namespace

void launch_set_int(int* dst, int value, hipStream_t s) {
  hipLaunchKernelGGL(k_set_int, dim3(1), dim3(64), 0, s, dst, value);
}

void launch_build_neighbors(const NbrParams& p, hipStream_t s) {
  if (p.n <= 0) return;
  hipLaunchKernelGGL(k_zero, dim3(blocks_for(p.n_cells, 256)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_bin, dim3(blocks_for(p.n, 256)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, s, p);
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(p.n, 256)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_sort_cells, dim3(blocks_for(p.n_cells, 64)), dim3(64), 0, s, p);
  hipLaunchKernelGGL(k_rows, dim3(blocks_for(p.n, 4)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_reverse, dim3(blocks_for(p.n, 4)), dim3(256), 0, s, p);
}

}  // namespace aenet
