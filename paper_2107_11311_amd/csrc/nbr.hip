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
#include <climits>

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
  // Inside an MD chunk an overflowed build means the chunk is redone with
  // longer rows: later builds of the chunk are dropped (their request is
  // withdrawn, so the rest of this build skips too), which keeps the row
  // maxima that size the retry those of the build that overflowed.
  if (p.cond && (p.flags[0] & kFlagOverflow)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p.cond = 0;
    return;
  }
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < p.n_cells) {
    p.cell_count[c] = 0;
    p.cell_fill[c] = 0;
  }
  if (c == 0) {
    p.maxcnt[0] = 0;
    p.maxcnt[1] = 0;
    if (p.cond) atomicAdd(p.flags + 8, 1);  // builds triggered on the device (MD)
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

// The scatter order depends on atomics; sorting each cell by atom index makes
// the rows deterministic.  One block per cell: bitonic sort in LDS (cells of
// up to kSortMax atoms; larger ones, possible only for very thin non-periodic
// boxes, fall back to an insertion sort by one thread).
constexpr int kSortMax = 4096;

__global__ __launch_bounds__(256) void k_sort_cells(NbrParams p) {
  if (skip(p)) return;
  __shared__ int v[kSortMax];
  const int c = blockIdx.x;
  int* a = p.cell_atoms + p.cell_start[c];
  const int m = p.cell_count[c];
  if (m <= 1) return;
  if (m > kSortMax) {
    if (threadIdx.x == 0) {
      for (int k = 1; k < m; ++k) {
        int x = a[k];
        int j = k - 1;
        while (j >= 0 && a[j] > x) {
          a[j + 1] = a[j];
          --j;
        }
        a[j + 1] = x;
      }
    }
    return;
  }
  int pw = 2;
  while (pw < m) pw <<= 1;
  for (int k = threadIdx.x; k < pw; k += blockDim.x) v[k] = k < m ? a[k] : INT_MAX;
  __syncthreads();
  for (int size = 2; size <= pw; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int k = threadIdx.x; k < pw; k += blockDim.x) {
        const int partner = k ^ stride;
        if (partner > k) {
          const bool up = (k & size) == 0;
          const int x = v[k], y = v[partner];
          if ((x > y) == up) {
            v[k] = y;
            v[partner] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int k = threadIdx.x; k < m; k += blockDim.x) a[k] = v[k];
}

// One wavefront per atom.  The 27 stencil cells (unwrapped, so each
// (cell, image) pair appears once) are flattened into one candidate stream
// that the 64 lanes walk together; angular candidates go straight into the
// row, the remaining ones into a scratch row that is appended at the end.
__global__ __launch_bounds__(256) void k_rows(NbrParams p) {
  if (skip(p)) return;
  __shared__ int s_start[4][27], s_count[4][27], s_code[4][27], s_pref[4][28];
  extern __shared__ uint32_t s_rad[];  // per wave: radial-only entries, then their keys
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int i = blockIdx.x * (blockDim.x >> 6) + wv;
  const bool active = i < p.n;  // waves past the end stay for the barriers
  const BoxInfo b = p.boxes[active ? p.seg[i] : 0];
  int ci[3] = {0, 0, 0};
  if (active) cell_coords(b, p.atom_cell[i], ci);
  if (lane < 27) {
    // stencil cell `lane` = offset (lane%3-1, lane/3%3-1, lane/9-1), in unwrapped coordinates
    const int o[3] = {lane % 3 - 1, (lane / 3) % 3 - 1, lane / 9 - 1};
    int w[3], s[3];
    bool out = !active;
    for (int a = 0; a < 3; ++a) {
      const int u = ci[a] + o[a];
      if (p.pbc[a]) {
        s[a] = u < 0 ? -1 : (u >= b.nc[a] ? 1 : 0);
        w[a] = u - s[a] * b.nc[a];
      } else {
        s[a] = 0;
        w[a] = u;
        out |= (u < 0 || u >= b.nc[a]);
      }
    }
    const int cell = out ? 0 : b.cell_base + (w[2] * b.nc[1] + w[1]) * b.nc[0] + w[0];
    s_start[wv][lane] = out ? 0 : p.cell_start[cell];
    s_count[wv][lane] = out ? 0 : p.cell_count[cell];
    s_code[wv][lane] = (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1);
  }
  __syncthreads();
  if (lane == 0) {
    int run = 0;
    for (int k = 0; k < 27; ++k) {
      s_pref[wv][k] = run;
      run += s_count[wv][k];
    }
    s_pref[wv][27] = run;
  }
  __syncthreads();
  const int total = s_pref[wv][27];
  const size_t rbase = (size_t)(active ? i : 0) * p.cap;
  uint32_t* row = p.nbr + rbase;
  uint32_t* key = p.key + rbase;
  uint32_t* rad_e = s_rad + (size_t)wv * 2 * p.cap;
  uint32_t* rad_k = rad_e + p.cap;
  int cnt_a = 0, cnt_r = 0;
  int k_cell = 0;  // stencil cell of this lane's candidate (candidates advance monotonically)
  for (int base = 0; base < total; base += 64) {
    const int t = base + lane;
    bool ang = false, rad = false;
    uint32_t entry = 0, ekey = 0;
    if (t < total) {
      while (k_cell < 26 && t >= s_pref[wv][k_cell + 1]) ++k_cell;
      const int q = p.cell_atoms[s_start[wv][k_cell] + (t - s_pref[wv][k_cell])];
      const int code = s_code[wv][k_cell];
      const int s0 = code % 3 - 1, s1 = (code / 3) % 3 - 1, s2 = code / 9 - 1;
      const bool self = (q == i) && code == 13;
      if (!self) {
        // displacement computed from the lower-index atom, so that the entry
        // and its reverse agree bit for bit on r^2
        const bool spos = s2 > 0 || (s2 == 0 && (s1 > 0 || (s1 == 0 && s0 > 0)));
        const bool iq = (i < q) || (i == q && spos);
        const size_t ia = iq ? (size_t)i : (size_t)q;
        const size_t ib = iq ? (size_t)q : (size_t)i;
        const double sg = iq ? 1.0 : -1.0;
        const double d0 = p.pos[3 * ib] + sg * (double)s0 * b.L[0] - p.pos[3 * ia];
        const double d1 = p.pos[3 * ib + 1] + sg * (double)s1 * b.L[1] - p.pos[3 * ia + 1];
        const double d2 = p.pos[3 * ib + 2] + sg * (double)s2 * b.L[2] - p.pos[3 * ia + 2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (r2 == 0.0) atomicOr(p.flags, kFlagOverlap);
        ang = r2 < p.r_ang2;
        rad = !ang && r2 < p.r_list2;
        entry = (uint32_t)q | ((uint32_t)code << kImgBits);
        // search key of the entry: (stencil cell, atom); rows are sorted by it
        ekey = (uint32_t)q | ((uint32_t)k_cell << kImgBits);
      }
    }
    const uint64_t below = (1ull << lane) - 1ull;
    const uint64_t ma = __ballot(ang), mr = __ballot(rad);
    if (ang) {
      const int at = cnt_a + __popcll(ma & below);
      if (at < p.cap) {
        row[at] = entry;
        key[at] = ekey;
      }
    }
    if (rad) {
      const int at = cnt_r + __popcll(mr & below);
      if (at < p.cap) {
        rad_e[at] = entry;
        rad_k[at] = ekey;
      }
    }
    cnt_a += __popcll(ma);
    cnt_r += __popcll(mr);
  }
  __syncthreads();
  // append the radial-only entries after the angular ones
  for (int k = lane; k < cnt_r; k += 64) {
    const int at = cnt_a + k;
    if (at < p.cap && k < p.cap) {
      row[at] = rad_e[k];
      key[at] = rad_k[k];
    }
  }
  if (active && lane == 0) {
    const int count = cnt_a + cnt_r;
    if (count > p.cap || cnt_a > p.cap_ang) atomicOr(p.flags, kFlagOverflow);
    // clamp so that every later kernel stays inside the row even after an overflow
    const int nang = min(cnt_a, min(p.cap_ang, p.cap));
    p.nnb[i] = max(min(count, p.cap), nang);
    p.nang[i] = nang;
    // maxima for capacity planning; the plain read first keeps the atomics rare
    if (count > p.maxcnt[0]) atomicMax(&p.maxcnt[0], count);
    if (cnt_a > p.maxcnt[1]) atomicMax(&p.maxcnt[1], cnt_a);
  }
}

// reverse entry of every row entry, one wavefront per atom: the reverse of
// (i -> q) found in stencil cell k of i is (q -> i) in stencil cell 26 - k of q
__global__ __launch_bounds__(256) void k_reverse(NbrParams p) {
  if (skip(p)) return;
  const int lane = threadIdx.x & 63;
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (i >= p.n) return;
  const int nn = p.nnb[i], na = p.nang[i];
  const uint32_t* krow = p.key + (size_t)i * p.cap;
  for (int e = lane; e < nn; e += 64) {
    const uint32_t k = krow[e];
    const int q = (int)(k & kAtomMask);
    const uint32_t target = ((26u - (k >> kImgBits)) << kImgBits) | (uint32_t)i;
    const uint32_t* kq = p.key + (size_t)q * p.cap;
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
      const uint32_t km = kq[mid];
      if (km == target) {
        found = mid;
        break;
      }
      if (km < target) lo = mid + 1; else hi = mid;
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
  hipLaunchKernelGGL(k_sort_cells, dim3(p.n_cells), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_rows, dim3(blocks_for(p.n, 4)), dim3(256), (size_t)4 * 2 * p.cap * sizeof(uint32_t), s, p);
  hipLaunchKernelGGL(k_reverse, dim3(blocks_for(p.n, 4)), dim3(256), 0, s, p);
}

}  // namespace aenet
