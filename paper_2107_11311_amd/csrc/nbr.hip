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
// parts are ordered by (stencil cell, atom), and the row position where each
// stencil cell's entries start is kept per part (segs).  The reverse entry
// (j -> i, -s) of an entry (i -> j, s) found in stencil cell k of i lies in
// the segment of stencil cell 26 - k of j's row, where it is found by binary
// search on the atom index; the deterministic force gather uses these
// reverse entries instead of atomics.
//
// A build is binning (whose last block also scans the cell counts and
// resets them for the next build) and scatter into cells, then either the
// per-cell row kernel (cells of up to kCellAtomsMax atoms) or per-cell sort,
// per-atom rows and reverse entries.  In MD each kernel first checks the
// device flag of the step; with the per-cell row kernel the integrator bins
// the atoms into fixed-capacity cells as it moves them, and the row kernel is
// the only launch of the build.
#include <climits>

#include "aenet_internal.h"

namespace aenet {

namespace {

// the decision of this build, taken by the binning kernel: later kernels of
// the build follow it
__device__ inline bool skip(const NbrParams& p) { return p.cond && *p.go == 0; }

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

// Binning: wrap positions into the box (periodic axes), remember them as the
// reference of the skin test, count atoms per cell.  The last block to finish
// scans the counts into cell_start and zeroes the counters for the scatter
// and the next build.
__global__ __launch_bounds__(256) void k_bin(NbrParams p) {
  // In MD a build runs if the step asked for it, unless an earlier build of
  // the chunk overflowed (the chunk is then redone with longer rows, and the
  // row maxima that size the retry stay those of that build).  Every block
  // decides alike: nothing it reads is written before the later kernels.
  const bool go = !p.cond || (*p.cond != 0 && !(p.flags[0] & kFlagOverflow));
  if (blockIdx.x == 0 && threadIdx.x == 0 && p.cond) {
    *p.go = go ? 1 : 0;
    if (go) atomicAdd(p.flags + 8, 1);  // builds triggered on the device (MD)
  }
  if (!go) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < p.n) {
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
    const int cell = b.cell_base + (c[2] * b.nc[1] + c[1]) * b.nc[0] + c[0];
    p.atom_cell[i] = cell;
    atomicAdd(&p.cell_count[cell], 1);
  }
  // last block: exclusive scan of the counts
  __shared__ int last;
  __shared__ int s[256];
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) last = atomicAdd(p.ticket, 1) == (int)gridDim.x - 1;
  __syncthreads();
  if (!last) return;
  __threadfence();
  const int n = p.n_cells;
  const int t = threadIdx.x;
  const int per = (n + 255) / 256;
  const int lo = min(t * per, n), hi = min(lo + per, n);
  int sum = 0;
  for (int k = lo; k < hi; ++k)
    sum += __hip_atomic_load(&p.cell_count[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int v = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += v;
    __syncthreads();
  }
  int run = t ? s[t - 1] : 0;
  for (int k = lo; k < hi; ++k) {
    const int cnt = __hip_atomic_load(&p.cell_count[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    p.cell_start[k] = run;
    run += cnt;
    p.cell_count[k] = 0;
    p.cell_fill[k] = 0;
  }
  if (t == 255) p.cell_start[n] = s[255];
  if (t == 0) *p.ticket = 0;
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
  const int m = p.cell_start[c + 1] - p.cell_start[c];
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
  __shared__ int s_na[4][27], s_nr[4][27];  // accepted entries per stencil cell and row part
  extern __shared__ uint32_t s_rad[];        // per wave: the radial-only entries
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
    s_count[wv][lane] = out ? 0 : p.cell_start[cell + 1] - p.cell_start[cell];
    s_code[wv][lane] = (s[0] + 1) + 3 * (s[1] + 1) + 9 * (s[2] + 1);
    s_na[wv][lane] = 0;
    s_nr[wv][lane] = 0;
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
  uint32_t* row = p.nbr + (size_t)(active ? i : 0) * p.cap;
  uint32_t* rad_e = s_rad + (size_t)wv * p.cap;
  int cnt_a = 0, cnt_r = 0;
  if (total > 0) {  // (an inactive wave has no candidates)
    const double xi0 = p.pos[3 * (size_t)i], xi1 = p.pos[3 * (size_t)i + 1], xi2 = p.pos[3 * (size_t)i + 2];
    // Candidate t of the stream (clamped to it): its atom and stencil cell.
    // Each lane's candidates of the next two chunks are in flight while one
    // is tested (the atom index two chunks ahead, its position one chunk
    // ahead); stencil cells advance monotonically with t.
    int kf = 0;
    auto cand = [&](int t, int& kc) {
      const int tt = min(t, total - 1);
      while (kf < 26 && tt >= s_pref[wv][kf + 1]) ++kf;
      kc = kf;
      return p.cell_atoms[s_start[wv][kf] + (tt - s_pref[wv][kf])];
    };
    int k0, k1;
    int q0 = cand(lane, k0);
    int q1 = cand(lane + 64, k1);
    double x0[3] = {p.pos[3 * (size_t)q0], p.pos[3 * (size_t)q0 + 1], p.pos[3 * (size_t)q0 + 2]};
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      int k2;
      const int q2 = cand(t + 128, k2);
      const double x1[3] = {p.pos[3 * (size_t)q1], p.pos[3 * (size_t)q1 + 1], p.pos[3 * (size_t)q1 + 2]};
      const int q = q0, k_cell = k0;
      bool ang = false, rad = false;
      uint32_t entry = 0;
      const int code = s_code[wv][k_cell];
      const int s0 = code % 3 - 1, s1 = (code / 3) % 3 - 1, s2 = code / 9 - 1;
      const bool self = (q == i) && code == 13;
      if (t < total && !self) {
        // d = (x_q - x_i) + s L: the reverse entry's (x_i - x_q) - s L is its
        // exact negative (rounding is symmetric), so both agree bit for bit
        // on r^2
        const double d0 = (x0[0] - xi0) + (double)s0 * b.L[0];
        const double d1 = (x0[1] - xi1) + (double)s1 * b.L[1];
        const double d2 = (x0[2] - xi2) + (double)s2 * b.L[2];
        const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
        if (r2 == 0.0) atomicOr(p.flags, kFlagOverlap);
        ang = r2 < p.r_ang2;
        rad = !ang && r2 < p.r_list2;
        entry = (uint32_t)q | ((uint32_t)code << kImgBits);
      }
      const uint64_t below = (1ull << lane) - 1ull;
      const uint64_t ma = __ballot(ang), mr = __ballot(rad);
      if (ang) {
        const int at = cnt_a + __popcll(ma & below);
        if (at < p.cap) row[at] = entry;
        atomicAdd(&s_na[wv][k_cell], 1);
      }
      if (rad) {
        const int at = cnt_r + __popcll(mr & below);
        if (at < p.cap) rad_e[at] = entry;
        atomicAdd(&s_nr[wv][k_cell], 1);
      }
      cnt_a += __popcll(ma);
      cnt_r += __popcll(mr);
      q0 = q1;
      k0 = k1;
      q1 = q2;
      k1 = k2;
#pragma unroll
      for (int c = 0; c < 3; ++c) x0[c] = x1[c];
    }
  }
  __syncthreads();
  // append the radial-only entries after the angular ones
  for (int k = lane; k < cnt_r; k += 64) {
    const int at = cnt_a + k;
    if (at < p.cap && k < p.cap) row[at] = rad_e[k];
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
    // where each stencil cell's entries start in the two row parts (clamped
    // to the row like nnb / nang)
    uint16_t* sg = p.segs + (size_t)i * kSegWords;
    int ra = 0, rr = cnt_a;
    for (int k = 0; k < 27; ++k) {
      sg[k] = (uint16_t)min(ra, nang);
      sg[28 + k] = (uint16_t)min(rr, p.nnb[i]);
      ra += s_na[wv][k];
      rr += s_nr[wv][k];
    }
    sg[27] = (uint16_t)nang;
    sg[55] = (uint16_t)p.nnb[i];
  }
}

// Reverse entry of every row entry, one wavefront per atom: the reverse of
// (i -> q) found in stencil cell k of i is (q -> i) in stencil cell 26 - k of
// q, in the same row part (the r^2 of both agree bit for bit); it is found by
// binary search on the atom index inside that segment of q's row.
__global__ __launch_bounds__(256) void k_reverse(NbrParams p) {
  if (skip(p)) return;
  __shared__ uint16_t s_seg[4][kSegWords];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int i = blockIdx.x * (blockDim.x >> 6) + wv;
  const bool active = i < p.n;
  if (active && lane < kSegWords) s_seg[wv][lane] = p.segs[(size_t)i * kSegWords + lane];
  __syncthreads();
  if (!active) return;
  const int nn = p.nnb[i], na = p.nang[i];
  const uint32_t* row = p.nbr + (size_t)i * p.cap;
  int k = 0, part = 0;  // stencil cell and row part of this lane's entry (advance monotonically)
  for (int e = lane; e < nn; e += 64) {
    if (part == 0 && e >= na) {
      part = 1;
      k = 0;
    }
    const uint16_t* sg = s_seg[wv] + 28 * part;
    while (k < 26 && e >= sg[k + 1]) ++k;
    const int q = (int)(row[e] & kAtomMask);
    const uint16_t* sq = p.segs + (size_t)q * kSegWords + 28 * part;
    int lo = sq[26 - k], hi = sq[27 - k];
    const uint32_t* rq = p.nbr + (size_t)q * p.cap;
    int found = -1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      const int am = (int)(rq[mid] & kAtomMask);
      if (am == i) {
        found = mid;
        break;
      }
      if (am < i) lo = mid + 1; else hi = mid;
    }
    if (found < 0) {
      atomicOr(p.flags, kFlagReverse);
      p.rev[(size_t)i * p.cap + e] = -1;
    } else {
      p.rev[(size_t)i * p.cap + e] = q * p.cap + found;
    }
  }
}

// ------------------------------------------------------------------ per-cell rows
// One block per cell.  The atoms of the 27 stencil cells (the candidates of
// every atom of the central cell) are loaded into LDS once, ordered by
// (stencil cell, atom) there, and every central atom's row is built from
// LDS.  While doing so
// the block records, per candidate and row part, which central atoms accepted
// it (a bitmask).  The reverse of (i -> q) found in stencil cell k of i is
// (q -> i) in stencil cell 26 - k of q, whose segment of q's row holds
// exactly the central atoms that accepted q there, ordered by index: its
// position inside the segment is the number of set bits below i's.  The
// block stores that rank with k in rev (as kRevPending - (rank | k << 16));
// the force pass, which runs after every row is built, adds the segment start
// on its first use of the entry and stores the result back.
constexpr int kMaskWords = kCellAtomsMax / 32;

// (at most 80 scalar registers: measured, a version at 84-86 no longer fit two
// 1024-thread blocks on a CU and a third of the blocks started a round late)
__global__ __launch_bounds__(64 * kRowWaves) __attribute__((amdgpu_num_sgpr(80))) void k_rows_cell(NbrParams p) {
  if (p.binned) {
    // every step: clear this cell's count in the half the integrator fills next
    if (threadIdx.x == 0) p.bin_count[(size_t)(1 - p.bin_sel) * p.n_cells + blockIdx.x] = 0;
    if (*p.cond == 0) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(p.flags + 8, 1);  // builds triggered on the device
  } else if (skip(p)) {
    return;
  }
  extern __shared__ __align__(16) unsigned char smem[];
  const int tp = p.tp;
  // candidate positions in FP32 (x, y, z planes: unit-stride lanes): they
  // only decide list membership, where the skin leaves a margin far above
  // their rounding, and an entry's displacement stays the exact negative of
  // its reverse's
  float* s_pos = reinterpret_cast<float*>(smem);                            // [3][tp]
  uint32_t* s_key = reinterpret_cast<uint32_t*>(s_pos + 3 * (size_t)tp);      // [tp] atom | stencil cell << kImgBits
  uint32_t* s_mask = s_key + tp;                                              // [tp][2][kMaskWords]
  uint32_t* s_rad = s_mask + (size_t)tp * 2 * kMaskWords;                     // [waves][cap]
  __shared__ int s_start[27], s_cnt[27], s_code[27], s_pref[28];
  __shared__ float s_shift[27][3];                              // image shift s L of each stencil cell
  __shared__ int s_sa[kRowWaves][28], s_sr[kRowWaves][28];      // segment starts of the row being built
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int c = blockIdx.x;
  // the structure owning cell c
  int st = 0;
  while (st + 1 < p.n_struct && c >= p.boxes[st + 1].cell_base) ++st;
  const BoxInfo b = p.boxes[st];
  int ci[3];
  cell_coords(b, c, ci);
  if (tid < 27) {
    const int o[3] = {tid % 3 - 1, (tid / 3) % 3 - 1, tid / 9 - 1};
    int w[3], sh[3];
    bool out = false;
    for (int a = 0; a < 3; ++a) {
      const int u = ci[a] + o[a];
      if (p.pbc[a]) {
        sh[a] = u < 0 ? -1 : (u >= b.nc[a] ? 1 : 0);
        w[a] = u - sh[a] * b.nc[a];
      } else {
        sh[a] = 0;
        w[a] = u;
        out |= (u < 0 || u >= b.nc[a]);
      }
      s_shift[tid][a] = (float)((double)sh[a] * b.L[a]);
    }
    const int cell = out ? 0 : b.cell_base + (w[2] * b.nc[1] + w[1]) * b.nc[0] + w[0];
    if (p.binned) {
      s_start[tid] = cell * kCellAtomsMax;
      s_cnt[tid] = out ? 0 : p.bin_count[(size_t)p.bin_sel * p.n_cells + cell];
    } else {
      s_start[tid] = out ? 0 : p.cell_start[cell];
      s_cnt[tid] = out ? 0 : p.cell_start[cell + 1] - p.cell_start[cell];
    }
    s_code[tid] = (sh[0] + 1) + 3 * (sh[1] + 1) + 9 * (sh[2] + 1);
  }
  __syncthreads();
  if (tid == 0) {
    int run = 0;
    for (int k = 0; k < 27; ++k) {
      s_pref[k] = run;
      run += s_cnt[k];
    }
    s_pref[27] = run;
  }
  __syncthreads();
  const int total = s_pref[27];
  const int ncen = s_cnt[13];
  int cmax = 0;
  for (int k = 0; k < 27; ++k) cmax = max(cmax, s_cnt[k]);
  if (total > tp || cmax > kCellAtomsMax) {
    // does not fit: the host enlarges tp (or takes the per-atom kernels) and
    // builds again; nothing of this cell's rows is written
    if (tid == 0) {
      atomicOr(p.flags, kFlagOverflow);
      atomicMax(p.flags + 5, total);
      atomicMax(p.flags + 6, cmax);
    }
    return;
  }
  if (ncen == 0) return;
  // candidates: each stencil cell's atoms sorted by index (one wavefront per
  // cell, a bitonic network across its lanes; element j = lane + 64 h in
  // v[h], the second half only for cells of more than 64 atoms), so the
  // scatter's atomic order does not reach the rows
  const int* cell_src = p.binned ? p.bin_atoms : p.cell_atoms;
  for (int k = wv; k < 27; k += kRowWaves) {
    const int cnt = s_cnt[k];
    uint32_t v[2];
#pragma unroll
    for (int h = 0; h < 2; ++h)
      v[h] = lane + 64 * h < cnt ? (uint32_t)cell_src[s_start[k] + lane + 64 * h] : 0xffffffffu;
    if (cnt <= 64) {  // (uniform over the wavefront)
#pragma unroll
      for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          const uint32_t o = (uint32_t)__shfl_xor((int)v[0], stride, 64);
          const bool up = (lane & size) == 0, lower = (lane & stride) == 0;
          v[0] = (lower == up) ? min(v[0], o) : max(v[0], o);
        }
      }
    } else {
#pragma unroll
      for (int size = 2; size <= 128; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
          if (stride == 64) {  // elements j and j + 64 (size 128: ascending)
            const uint32_t lo = min(v[0], v[1]), hi = max(v[0], v[1]);
            v[0] = lo;
            v[1] = hi;
          } else {
            const bool lower = (lane & stride) == 0;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
              const uint32_t o = (uint32_t)__shfl_xor((int)v[h], stride, 64);
              const bool up = size == 128 || (((lane + 64 * h) & size) == 0);
              v[h] = (lower == up) ? min(v[h], o) : max(v[h], o);
            }
          }
        }
      }
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int j = lane + 64 * h;
      if (j < cnt) {
        const uint32_t a_ = v[h];
        const int t = s_pref[k] + j;
        s_key[t] = a_ | ((uint32_t)k << kImgBits);
        double x[3];
        for (int a = 0; a < 3; ++a) {
          x[a] = p.pos[3 * (size_t)a_ + a];
          // binned: the positions were last wrapped at the previous build; the
          // block of the atom's own cell stores the wrapped position and the
          // skin-test reference (other blocks may read either value: wrapping
          // is idempotent)
          if (p.binned && p.pbc[a]) x[a] = wrap_coord(x[a], b.L[a]);
          s_pos[(size_t)a * tp + t] = (float)x[a];
        }
        if (p.binned && k == 13) {
          for (int a = 0; a < 3; ++a) {
            p.pos[3 * (size_t)a_ + a] = x[a];
            p.pos_ref[3 * (size_t)a_ + a] = x[a];
          }
        }
      }
    }
  }
  for (int t = tid; t < total * 2 * kMaskWords; t += 64 * kRowWaves) s_mask[t] = 0u;
  __syncthreads();

  // rows of the central atoms (stencil cell 13, sorted by atom index), one
  // wavefront per atom; the radial-only entries are staged as (slot, stencil)
  const int c0 = s_pref[13];
  uint32_t* rad_t = s_rad + (size_t)wv * p.cap;
  // The FP32 radii carry a margin d well above the FP32 rounding of the
  // displacements (coordinates up to the largest box edge Lm lose at most
  // 2^-24 Lm each; d = max(2^-20 Lm, 5e-5 R)), so no pair within the list
  // radius in FP64 is left out and the skin keeps its guarantee; the few
  // pairs just beyond it that enter contribute nothing
  const double lm = fmax(b.L[0], fmax(b.L[1], b.L[2]));
  auto padded = [&](double r2) {
    const double r = sqrt(r2), d = fmax(0x1p-20 * lm, 5e-5 * r);
    return (float)((r + d) * (r + d));
  };
  const float r_ang2f = padded(p.r_ang2), r_list2f = padded(p.r_list2);
  for (int ai = wv; ai < ncen; ai += kRowWaves) {
    const int i = (int)(s_key[c0 + ai] & kAtomMask);
    const float xi0 = s_pos[c0 + ai], xi1 = s_pos[tp + c0 + ai], xi2 = s_pos[2 * tp + c0 + ai];
    uint32_t* row = p.nbr + (size_t)i * p.cap;
    int* slot = p.rev + (size_t)i * p.cap;  // (candidate slot, stencil cell) of each entry, then (rank, cell)
    int cnt_a = 0, cnt_r = 0;
    int k_cell = 0;
    uint32_t* mA = s_mask + (ai >> 5);
    const uint32_t mbit = 1u << (ai & 31);
    for (int base = 0; base < total; base += 64) {
      const int t = base + lane;
      const bool in = t < total;
      const int tt = in ? t : 0;
      const uint32_t key = s_key[tt];
      k_cell = (int)(key >> kImgBits);
      const int q = (int)(key & kAtomMask);
      const float qx = s_pos[tt], qy = s_pos[tp + tt], qz = s_pos[2 * tp + tt];
      // d = (x_q - x_i) + s: the reverse entry's (x_i - x_q) - s is its exact
      // negative (rounding is symmetric), so both agree bit for bit on r^2
      const float d0 = (qx - xi0) + s_shift[k_cell][0];
      const float d1 = (qy - xi1) + s_shift[k_cell][1];
      const float d2 = (qz - xi2) + s_shift[k_cell][2];
      const float r2 = d0 * d0 + d1 * d1 + d2 * d2;
      const bool self = q == i && k_cell == 13;
      const bool ok = in && !self;
      if (ok && r2 == 0.0f) {
        // coincident in FP32: overlapping only if coincident in FP64 too
        // (the atoms' wrapped coordinates and the cell's image shift)
        const int code = s_code[k_cell];
        double e2 = 0.0;
        for (int a = 0; a < 3; ++a) {
          double xq = p.pos[3 * (size_t)q + a], xa = p.pos[3 * (size_t)i + a];
          if (p.pbc[a]) {
            xq = wrap_coord(xq, b.L[a]);
            xa = wrap_coord(xa, b.L[a]);
          }
          const int sh = (a == 0 ? code % 3 : a == 1 ? (code / 3) % 3 : code / 9) - 1;
          const double d = (xq - xa) + (double)sh * b.L[a];
          e2 += d * d;
        }
        if (e2 == 0.0) atomicOr(p.flags, kFlagOverlap);
      }
      const bool ang = ok && r2 < r_ang2f;
      const bool rad = ok && !ang && r2 < r_list2f;
      const uint64_t below = (1ull << lane) - 1ull;
      const uint64_t ma = __ballot(ang), mr = __ballot(rad);
      const int pa = cnt_a + __popcll(ma & below), pr = cnt_r + __popcll(mr & below);
      // the first candidate of a stencil cell fixes where its entries start
      if (in && t == s_pref[k_cell]) {
        s_sa[wv][k_cell] = pa;
        s_sr[wv][k_cell] = pr;
      }
      if (ang) {
        if (pa < p.cap) {
          row[pa] = (uint32_t)q | ((uint32_t)s_code[k_cell] << kImgBits);
          slot[pa] = tt | (k_cell << 16);
        }
        atomicOr(mA + (2 * (size_t)tt) * kMaskWords, mbit);
      }
      if (rad) {
        if (pr < p.cap) rad_t[pr] = (uint32_t)tt | ((uint32_t)k_cell << 16);
        atomicOr(mA + (2 * (size_t)tt + 1) * kMaskWords, mbit);
      }
      cnt_a += __popcll(ma);
      cnt_r += __popcll(mr);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    // the radial-only entries after the angular ones
    for (int k = lane; k < cnt_r; k += 64) {
      const int at = cnt_a + k;
      if (at < p.cap && k < p.cap) {
        const uint32_t v = rad_t[k];
        row[at] = (s_key[v & 0xffffu] & kAtomMask) | ((uint32_t)s_code[v >> 16] << kImgBits);
        slot[at] = (int)v;
      }
    }
    const int nang = min(cnt_a, min(p.cap_ang, p.cap));
    const int nnb = max(min(cnt_a + cnt_r, p.cap), nang);
    if (lane < 28) {
      // stencil cells without candidates start where the next one does
      int sa = cnt_a, sr = cnt_r;
      for (int k = lane; k < 27; ++k)
        if (s_cnt[k] > 0) {
          sa = s_sa[wv][k];
          sr = s_sr[wv][k];
          break;
        }
      uint16_t* sg = p.segs + (size_t)i * kSegWords;
      sg[lane] = (uint16_t)(lane == 27 ? nang : min(sa, nang));
      sg[28 + lane] = (uint16_t)(lane == 27 ? nnb : min(cnt_a + sr, nnb));
    }
    if (lane == 0) {
      const int count = cnt_a + cnt_r;
      if (count > p.cap || cnt_a > p.cap_ang) atomicOr(p.flags, kFlagOverflow);
      p.nnb[i] = nnb;
      p.nang[i] = nang;
      if (count > p.maxcnt[0]) atomicMax(&p.maxcnt[0], count);
      if (cnt_a > p.maxcnt[1]) atomicMax(&p.maxcnt[1], cnt_a);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  __syncthreads();  // every central atom's acceptances are in the masks

  // ranks: position of i among the central atoms in the segment of q's row
  for (int ai = wv; ai < ncen; ai += kRowWaves) {
    const int i = (int)(s_key[c0 + ai] & kAtomMask);
    const int nn = p.nnb[i], na = p.nang[i];
    int* slot = p.rev + (size_t)i * p.cap;
    for (int e = lane; e < nn; e += 64) {
      const int v = slot[e];
      const int t = v & 0xffff, k = v >> 16;
      const uint32_t* m = s_mask + (2 * (size_t)t + (e < na ? 0 : 1)) * kMaskWords;
      int rank = 0;
#pragma unroll
      for (int w = 0; w < kMaskWords; ++w) {
        const int lo = 32 * w;
        const uint32_t below = ai >= lo + 32 ? 0xffffffffu : (ai <= lo ? 0u : ((1u << (ai - lo)) - 1u));
        rank += __popc(m[w] & below);
      }
      slot[e] = kRevPending - (rank | (k << 16));
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
  if (p.binned) {
    hipLaunchKernelGGL(k_rows_cell, dim3(p.n_cells), dim3(64 * kRowWaves), cell_rows_lds(p.tp, p.cap), s, p);
    return;
  }
  hipLaunchKernelGGL(k_bin, dim3(blocks_for(p.n, 256)), dim3(256), 0, s, p);
  hipLaunchKernelGGL(k_scatter, dim3(blocks_for(p.n, 256)), dim3(256), 0, s, p);
  if (p.tp > 0) {
    hipLaunchKernelGGL(k_rows_cell, dim3(p.n_cells), dim3(64 * kRowWaves), cell_rows_lds(p.tp, p.cap), s, p);
  } else {
    hipLaunchKernelGGL(k_sort_cells, dim3(p.n_cells), dim3(256), 0, s, p);
    hipLaunchKernelGGL(k_rows, dim3(blocks_for(p.n, 4)), dim3(256), (size_t)4 * p.cap * sizeof(uint32_t), s, p);
    hipLaunchKernelGGL(k_reverse, dim3(blocks_for(p.n, 4)), dim3(256), 0, s, p);
  }
}

}  // namespace aenet
