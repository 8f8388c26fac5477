// md.hip -- velocity-Verlet integrator (the propagation step of the MD cycle,
// Fig. 1), the deterministic force gather, permutations between the caller's
// atom order and the internal species-sorted order, deterministic reductions
// (total energy, Sec. II A, Eq. 2; kinetic energy) and the per-atom terms of
// the training loss.
#include "aenet_internal.h"

namespace aenet {

namespace {

constexpr double kKappa = 9648.533215665;  // (eV/amu) in A^2/ps^2

inline int nblk(int64_t n, int t) { return (int)((n + t - 1) / t); }

__device__ inline bool finite3(double a, double b, double c) {
  return isfinite(a) && isfinite(b) && isfinite(c);
}

__global__ void k_gather_in(int n, const int* perm, const double* src, double* dst, int* flags) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const size_t o = (size_t)perm[p];
  const double a = src[3 * o], b = src[3 * o + 1], c = src[3 * o + 2];
  if (!finite3(a, b, c)) atomicOr(flags, kFlagNonFinite);
  dst[3 * (size_t)p] = a;
  dst[3 * (size_t)p + 1] = b;
  dst[3 * (size_t)p + 2] = c;
}

__global__ void k_scatter_out(int n, const int* perm, const double* src3, double* dst3,
                              const double* src1, double* dst1) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const size_t o = (size_t)perm[p];
  if (dst3) {
    dst3[3 * o] = src3[3 * (size_t)p];
    dst3[3 * o + 1] = src3[3 * (size_t)p + 1];
    dst3[3 * o + 2] = src3[3 * (size_t)p + 2];
  }
  if (dst1) dst1[o] = src1[p];
}

// raises *differ if any caller-order position in src is not bitwise what
// k_md_outputs writes for the internal positions pos
__global__ void k_same_wrapped(int n, const int* perm, const double* pos, const int* seg,
                               const BoxInfo* boxes, int px, int py, int pz, const double* src,
                               int* differ) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const BoxInfo b = boxes[seg[p]];
  const int pb[3] = {px, py, pz};
  const size_t o = (size_t)perm[p];
  bool same = true;
  for (int a = 0; a < 3; ++a) {
    double x = pos[3 * (size_t)p + a];
    if (pb[a]) x = wrap_coord(x, b.L[a]);
    same = same && (src[3 * o + a] == x);
  }
  if (!same) atomicOr(differ, 1);
}

__global__ void k_copy3(int64_t m, const double* a, double* a2, const double* b, double* b2,
                        const double* c, double* c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= m) return;
  a2[k] = a[k];
  b2[k] = b[k];
  c2[k] = c[k];
}

// Put the atoms of the wavefront's lanes with `mine` set (atom i at position
// x) into their cell bins for the next build.  Lanes with the same cell take
// one atomic together (consecutive atoms mostly share a cell).  A bin holds
// kCellAtomsMax atoms; the count goes on beyond that and the build then
// reports the overflow.  Every lane of the wavefront calls it.
__device__ inline void bin_wave_cells(const DriftArgs& d, bool mine, int i, int cell) {
  const int lane = threadIdx.x & 63;
  uint64_t pending = __ballot(mine);
  while (pending) {
    const int leader = __ffsll((unsigned long long)pending) - 1;
    const int lc = __shfl(cell, leader, 64);
    const uint64_t same = __ballot(cell == lc) & pending;
    int base = 0;
    if (lane == leader) base = atomicAdd(&d.bin_count[lc], __popcll(same));
    base = __shfl(base, leader, 64);
    if ((same >> lane) & 1ull) {
      const int rank = base + __popcll(same & ((1ull << lane) - 1ull));
      if (rank < kCellAtomsMax) d.bin_atoms[(size_t)lc * kCellAtomsMax + rank] = i;
    }
    pending &= ~same;
  }
}
__device__ inline void bin_wave(const DriftArgs& d, bool mine, int i, const double x[3]) {
  bin_wave_cells(d, mine, i, mine ? cell_of(*d.box, d.pbc, x) : -1);
}

// F_q = sum_e dE_q/dd_e - sum over the entries (i -> q) of dE_i/dd: the first
// sum was formed by the force pass (Fself); the second is row q of pg, where
// the force pass stored the gradient of every contributing entry at the slot
// of its reverse entry, so this gather reads within one row: the slots of q's
// own contributing entries, listed by the forward pass.
//
// The kernel is a chain of dependent memory accesses, so everything it reads
// is requested before anything is written: the atom's state (lanes 0..2 of
// its group hold component 0..2), the first kGatherPre listed slots of every lane
// (in bounds whatever the count, a row has cap slots) and the box.  The
// count then only masks.
constexpr int kGatherLanes = 16;  // lanes per atom in the force gather
constexpr int kGatherPre = 8;     // listed slots per lane requested up front

template <typename R>
__global__ __launch_bounds__(256) void k_force_gather(int n, int cap, const int* nrad, const uint16_t* ridx,
                                                      const R* pg, const double* Fself, double* F,
                                                      double* vel, const double* inv_mass_k,
                                                      const int* species, double half_dt,
                                                      DriftArgs next) {
  constexpr int LPA = kGatherLanes;
  const int g = threadIdx.x / LPA, l = threadIdx.x % LPA;
  const int i = blockIdx.x * (blockDim.x / LPA) + g;
  const bool act = i < n;
  const int ic = act ? i : 0;
  const bool drift = next.pos != nullptr && vel != nullptr;
  const bool binning = drift && next.bin_count != nullptr;

  // ---- loads (addresses chosen without branches: a missing array reads a
  // harmless stand-in whose value is not used)
  const int a = l < 3 ? l : 0;
  const size_t k3 = 3 * (size_t)ic + a;
  const double* vel_in = vel ? vel : Fself;
  const double* pos_in = drift ? next.pos : Fself;
  const double* ref_in = drift ? next.pos_ref : Fself;
  const int* flag_in = drift ? next.rebuild_flag : nrad;
  const int* sp_in = vel ? species + ic : nrad + ic;
  const double fself = Fself[k3];
  const double v_old = vel_in[k3];
  const double x_old = pos_in[k3];
  const double x_ref = ref_in[k3];
  const int flag0 = *flag_in;
  const int sv = *sp_in;
  const int code = nrad[ic];
  const uint16_t* ri = ridx + (size_t)ic * cap;
  int ep[kGatherPre];
#pragma unroll
  for (int m = 0; m < kGatherPre; ++m) ep[m] = (int)ri[min(l + m * LPA, max(cap - 1, 0))];
  BoxInfo bx{};
  if (binning) bx = *next.box;
  const double im = *(vel ? inv_mass_k + sv : Fself + k3);
  const int nk = act ? (code & 0xffff) : 0;
  const R* row = pg + (size_t)ic * cap * 3;
  double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
  for (int m = 0; m < kGatherPre; ++m) {
    const bool use = l + m * LPA < nk;
    const int e = use ? ep[m] : 0;
    const R px = row[3 * e], py = row[3 * e + 1], pz = row[3 * e + 2];
    sx += use ? (double)px : 0.0;
    sy += use ? (double)py : 0.0;
    sz += use ? (double)pz : 0.0;
  }
  for (int k = l + kGatherPre * LPA; k < nk; k += LPA) {
    const int e = ri[k];
    sx += (double)row[3 * e];
    sy += (double)row[3 * e + 1];
    sz += (double)row[3 * e + 2];
  }
#pragma unroll
  for (int o = LPA / 2; o > 0; o >>= 1) {
    sx += __shfl_xor(sx, o, LPA);
    sy += __shfl_xor(sy, o, LPA);
    sz += __shfl_xor(sz, o, LPA);
  }

  // ---- stores
  if (next.pos && blockIdx.x == 0 && threadIdx.x == 0) {
    *next.clear_flag = 0;
    if (next.force_rebuild) *next.rebuild_flag = 1;
  }
  const double f = fself - (a == 0 ? sx : a == 1 ? sy : sz);
  double xn = 0.0, dd = 0.0;
  if (act && l < 3) {
    F[k3] = f;
    if (vel) {
      const double c = half_dt * im;
      double v = v_old + c * f;    // closing half kick of this step
      if (drift) {
        v = v + c * f;             // opening half kick of the next step
        xn = x_old + next.dt * v;
        next.pos[k3] = xn;
        dd = xn - x_ref;
      }
      vel[k3] = v;
    }
  }
  if (drift) {
    const double dd1 = __shfl(dd, 1, LPA), dd2 = __shfl(dd, 2, LPA);
    const double xn1 = __shfl(xn, 1, LPA), xn2 = __shfl(xn, 2, LPA);
    if (act && l == 0) {
      double d2 = dd * dd;
      d2 += dd1 * dd1;
      d2 += dd2 * dd2;
      if (!(d2 <= next.half_skin2) && flag0 == 0) *next.rebuild_flag = 1;
    }
    if (binning) {
      // the block's 16 atoms are binned by its first wavefront, so atoms of
      // one cell share one atomic across the block
      __shared__ int s_cell[256 / LPA];
      if (l == 0) {
        const double x3[3] = {xn, xn1, xn2};
        s_cell[g] = act ? cell_of(bx, next.pbc, x3) : -1;
      }
      __syncthreads();
      if (threadIdx.x < 64) {
        const int t = threadIdx.x;
        const bool mine = t < 256 / LPA && s_cell[t] >= 0;
        bin_wave_cells(next, mine, blockIdx.x * (blockDim.x / LPA) + t, mine ? s_cell[t] : -1);
      }
    }
  }
}

// first half kick + drift; flags a neighbour-list rebuild when an atom has
// moved more than skin/2 since the last build
__global__ void k_vv_drift(int n, double* vel, const double* F, const double* inv_mass_k,
                           const int* species, double half_dt, DriftArgs d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    *d.clear_flag = 0;
    if (d.force_rebuild) *d.rebuild_flag = 1;
  }
  double xn[3] = {0.0, 0.0, 0.0};
  if (i < n) {
    const double c = half_dt * inv_mass_k[species[i]];
    double d2 = 0.0;
    for (int a = 0; a < 3; ++a) {
      const size_t k = 3 * (size_t)i + a;
      const double v = vel[k] + c * F[k];
      vel[k] = v;
      const double x = d.pos[k] + d.dt * v;
      d.pos[k] = x;
      xn[a] = x;
      const double dd = x - d.pos_ref[k];
      d2 += dd * dd;
    }
    if (!(d2 <= d.half_skin2) && *d.rebuild_flag == 0) *d.rebuild_flag = 1;
  }
  if (d.bin_count) bin_wave(d, i < n, i, xn);
}

constexpr int kRedChunk = 2048;  // elements per partial sum (fixed: results depend only on n)

// row blockIdx.y of x ([rows][n]) into part[blockIdx.y * gridDim.x + blockIdx.x]
// block partial sums of x (or, with y, of (x - y)^2) over fixed chunks
__global__ __launch_bounds__(256) void k_partial_sum(int64_t n, const double* x, const double* y,
                                                     double* part) {
  __shared__ double s[256];
  x += (size_t)blockIdx.y * n;
  part += (size_t)blockIdx.y * gridDim.x;
  const int64_t base = (int64_t)blockIdx.x * kRedChunk;
  double acc = 0.0;
  for (int k = threadIdx.x; k < kRedChunk; k += 256) {
    const int64_t idx = base + k;
    if (idx < n) {
      const double v = y ? x[idx] - y[idx] : x[idx];
      acc += y ? v * v : v;
    }
  }
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

// row blockIdx.x of part ([rows][m]) into out[blockIdx.x]
__global__ __launch_bounds__(1024) void k_final_sum(int m, const double* part, double* out) {
  __shared__ double s[1024];
  part += (size_t)blockIdx.x * m;
  out += blockIdx.x;
  double acc = 0.0;
  for (int k = threadIdx.x; k < m; k += 1024) acc += part[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = s[0];
}

// The outputs of an MD call in two launches: every thread writes one atom's
// wrapped position, velocity and (if F_out) force to the caller's order, and
// the first m blocks form, per chunk of kRedChunk atoms, the partial sums of
// E_i (row 0) and of the kinetic energies (row 1) with the same chunks and
// tree as k_partial_sum; then k_final_sum2 adds each row's partials.  Nothing is
// written to the caller when the call's status words hold an error or a
// retry (flags[0]) or the state the call continued from was stale
// (flags[9]): the call is then redone or fails with its outputs untouched.
__device__ inline bool md_outputs_blocked(const int* flags) { return (flags[0] | flags[9]) != 0; }

__global__ __launch_bounds__(256) void k_md_outputs(int n, int m, const int* perm, const double* E,
                                                    const double* pos, const double* vel, const double* F,
                                                    const double* mass, const int* species, const int* seg,
                                                    const BoxInfo* boxes, int px, int py, int pz, const int* flags,
                                                    double* part, double* pos_out, double* vel_out,
                                                    double* F_out) {
  if (md_outputs_blocked(flags)) return;
  // the caller-order outputs: one atom per thread over the whole grid
  const int64_t q = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (q < n) {
    const int pb[3] = {px, py, pz};
    const size_t o = (size_t)perm[q];
    const BoxInfo b = boxes[seg[q]];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double x = pos[3 * q + a];
      if (pb[a]) x = wrap_coord(x, b.L[a]);
      pos_out[3 * o + a] = x;
      vel_out[3 * o + a] = vel[3 * q + a];
      if (F_out) F_out[3 * o + a] = F[3 * q + a];
    }
  }
  // the partial sums: block b < m takes chunk b
  if ((int)blockIdx.x >= m) return;
  __shared__ double s_e[256], s_k[256];
  const int64_t base = (int64_t)blockIdx.x * kRedChunk;
  double ae = 0.0, ak = 0.0;
  for (int k = threadIdx.x; k < kRedChunk; k += 256) {
    const int64_t p = base + k;
    if (p < n) {
      ae += E[p];
      const double vx = vel[3 * p], vy = vel[3 * p + 1], vz = vel[3 * p + 2];
      ak += 0.5 * mass[species[p]] * (vx * vx + vy * vy + vz * vz) / kKappa;
    }
  }
  s_e[threadIdx.x] = ae;
  s_k[threadIdx.x] = ak;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) {
      s_e[threadIdx.x] += s_e[threadIdx.x + o];
      s_k[threadIdx.x] += s_k[threadIdx.x + o];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s_e[0];
    part[m + blockIdx.x] = s_k[0];
  }
}

// rows 0 and 1 of part ([2][m]) into *out0 and *out1 (k_final_sum's tree)
__global__ __launch_bounds__(1024) void k_final_sum2(int m, const double* part, const int* flags, double* out0,
                                                     double* out1) {
  if (md_outputs_blocked(flags)) return;
  __shared__ double s[1024];
  part += (size_t)blockIdx.x * m;
  double acc = 0.0;
  for (int k = threadIdx.x; k < m; k += 1024) acc += part[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 512; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) *(blockIdx.x == 0 ? out0 : out1) = s[0];
}

__global__ __launch_bounds__(256) void k_segment_sum(const int64_t* off, const double* x, double* out) {
  __shared__ double s[256];
  const int64_t lo = off[blockIdx.x], hi = off[blockIdx.x + 1];
  double acc = 0.0;
  for (int64_t k = lo + threadIdx.x; k < hi; k += 256) acc += x[k];
  s[threadIdx.x] = acc;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

__global__ void k_copy(int64_t n, const double* src, double* dst) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[k];
}

__global__ void k_check_finite(int64_t n, const double* x, int* flags) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && !isfinite(x[k])) atomicOr(flags, kFlagNonFinite);
}

// per-atom loss terms in internal order; f_ref in the caller's order
// per-atom terms of the training cost and its adjoints: dC/dF (adj) and
// dC/dE_s of the atom's structure (eps_atom).  form 0: per-atom mean
// (1/B) sum_s [(dE_s/N_s)^2 + lambda_f/(3 N_s) sum |dF|^2]; form 1: Eq. 7's
// half sum 1/2 sum_s dE_s^2 + lambda_f/2 sum |dF|^2
__global__ void k_loss_atoms(int n, int n_struct, const int* seg, const int* perm, const double* F,
                             const double* f_ref, const double* e_struct, const double* e_ref,
                             const int64_t* seg_count, double lambda_f, int form, double* adj,
                             double* eps_atom, double* floss_atom) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int s = seg[p];
  const double Ns = (double)seg_count[s];
  const double B = (double)n_struct;
  const size_t o = (size_t)perm[p];
  double sq = 0.0;
  const double c = form == 0 ? 2.0 * lambda_f / (3.0 * Ns * B) : lambda_f;
  for (int a = 0; a < 3; ++a) {
    const double df = F[3 * (size_t)p + a] - f_ref[3 * o + a];
    adj[3 * (size_t)p + a] = c * df;
    sq += df * df;
  }
  const double de = e_struct[s] - e_ref[s];
  if (form == 0) {
    floss_atom[p] = lambda_f * sq / (3.0 * Ns * B);
    eps_atom[p] = 2.0 * de / (Ns * Ns * B);
  } else {
    floss_atom[p] = 0.5 * lambda_f * sq;
    eps_atom[p] = de;
  }
}

__global__ void k_loss_structs(int n_struct, const double* e_struct, const double* e_ref,
                               const int64_t* seg_count, int form, double* eloss) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n_struct) return;
  if (form == 0) {
    const double de = (e_struct[s] - e_ref[s]) / (double)seg_count[s];
    eloss[s] = de * de / (double)n_struct;
  } else {
    const double de = e_struct[s] - e_ref[s];
    eloss[s] = 0.5 * de * de;
  }
}

}  // namespace

void launch_gather_in(int n, const int* perm, const double* src, double* dst, int* flags,
                      hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_gather_in, dim3(nblk(n, 256)), dim3(256), 0, s, n, perm, src, dst, flags);
}

void launch_scatter_out(int n, const int* perm, const double* src3, double* dst3,
                        const double* src1, double* dst1, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_scatter_out, dim3(nblk(n, 256)), dim3(256), 0, s, n, perm, src3, dst3, src1, dst1);
}

void launch_same_wrapped(int n, const int* perm, const double* pos, const int* seg,
                         const BoxInfo* boxes, const int pbc[3], const double* src, int* differ,
                         hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_same_wrapped, dim3(nblk(n, 256)), dim3(256), 0, s, n, perm, pos, seg, boxes,
                       pbc[0], pbc[1], pbc[2], src, differ);
}

void launch_copy3(int64_t m, const double* a, double* a2, const double* b, double* b2,
                  const double* c, double* c2, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(k_copy3, dim3((unsigned)((m + 255) / 256)), dim3(256), 0, s, m, a, a2, b, b2, c, c2);
}

void launch_force_gather(int prec, int n, int cap, const int* nrad, const uint16_t* ridx, const void* pg,
                         const double* Fself, double* F, double* vel, const double* inv_mass_k,
                         const int* species, double half_dt, const DriftArgs& next,
                         hipStream_t s) {
  if (n <= 0) return;
  const dim3 grid(nblk(n, 256 / kGatherLanes)), block(256);
  if (prec == 0)
    hipLaunchKernelGGL(k_force_gather<double>, grid, block, 0, s, n, cap, nrad, ridx,
                       (const double*)pg, Fself, F, vel, inv_mass_k, species, half_dt, next);
  else
    hipLaunchKernelGGL(k_force_gather<float>, grid, block, 0, s, n, cap, nrad, ridx,
                       (const float*)pg, Fself, F, vel, inv_mass_k, species, half_dt, next);
}

void launch_vv_drift(int n, double* vel, const double* F, const double* inv_mass_k,
                     const int* species, double half_dt, const DriftArgs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_vv_drift, dim3(nblk(n > 0 ? n : 1, 256)), dim3(256), 0, s, n, vel, F,
                     inv_mass_k, species, half_dt, d);
}

int reduce_blocks(int64_t n) { return (int)((n + kRedChunk - 1) / kRedChunk); }

void launch_sum(int64_t n, const double* x, double* partials, double* out, hipStream_t s) {
  launch_sum_rows(1, n, x, partials, out, s);
}

void launch_sum_rows(int rows, int64_t n, const double* x, double* partials, double* out, hipStream_t s) {
  const int m = reduce_blocks(n);
  if (m > 0) hipLaunchKernelGGL(k_partial_sum, dim3(m, rows), dim3(256), 0, s, n, x, (const double*)nullptr,
                                partials);
  hipLaunchKernelGGL(k_final_sum, dim3(rows), dim3(1024), 0, s, m, partials, out);
}

__global__ void k_rms_finish(int64_t n, double* out) {
  if (threadIdx.x == 0) *out = n > 0 ? sqrt(*out / (double)n) : 0.0;
}

void launch_rms_diff(int64_t n, const double* x, const double* y, double* partials, double* out,
                     hipStream_t s) {
  const int m = reduce_blocks(n);
  if (m > 0) hipLaunchKernelGGL(k_partial_sum, dim3(m, 1), dim3(256), 0, s, n, x, y, partials);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(1024), 0, s, m, partials, out);
  hipLaunchKernelGGL(k_rms_finish, dim3(1), dim3(64), 0, s, n, out);
}

void launch_md_outputs(int n, const int* perm, const double* E, const double* pos, const double* vel,
                       const double* F, const double* mass, const int* species, const int* seg,
                       const BoxInfo* boxes, const int pbc[3], const int* flags, double* partials, double* e_pot,
                       double* e_kin, double* pos_out, double* vel_out, double* F_out, hipStream_t s) {
  const int m = reduce_blocks(n);
  const int grid = std::max(m, nblk(n, 256));
  if (m > 0)
    hipLaunchKernelGGL(k_md_outputs, dim3(grid), dim3(256), 0, s, n, m, perm, E, pos, vel, F, mass, species, seg,
                       boxes, pbc[0], pbc[1], pbc[2], flags, partials, pos_out, vel_out, F_out);
  hipLaunchKernelGGL(k_final_sum2, dim3(2), dim3(1024), 0, s, m, partials, flags, e_pot, e_kin);
}

void launch_segment_sum(int n_seg, const int64_t* seg_off, const double* x, double* out,
                        hipStream_t s) {
  if (n_seg > 0) hipLaunchKernelGGL(k_segment_sum, dim3(n_seg), dim3(256), 0, s, seg_off, x, out);
}

void launch_copy_f64(int64_t n, const double* src, double* dst, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_copy, dim3(nblk(n, 256)), dim3(256), 0, s, n, src, dst);
}

void launch_check_finite(int64_t n, const double* x, int* flags, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_check_finite, dim3(nblk(n, 256)), dim3(256), 0, s, n, x, flags);
}

void launch_loss_terms(int n, int n_struct, const int* seg, const int* perm, const double* F,
                       const double* f_ref, const double* e_struct, const double* e_ref,
                       const int64_t* seg_count, double lambda_f, int form, double* adj,
                       double* eps_atom, double* floss_atom, double* eloss_struct, hipStream_t s) {
  if (n > 0)
    hipLaunchKernelGGL(k_loss_atoms, dim3(nblk(n, 256)), dim3(256), 0, s, n, n_struct, seg, perm, F,
                       f_ref, e_struct, e_ref, seg_count, lambda_f, form, adj, eps_atom, floss_atom);
  if (n_struct > 0)
    hipLaunchKernelGGL(k_loss_structs, dim3(nblk(n_struct, 256)), dim3(256), 0, s, n_struct,
                       e_struct, e_ref, seg_count, form, eloss_struct);
}

}  // namespace aenet
