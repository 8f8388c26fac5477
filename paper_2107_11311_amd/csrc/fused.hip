// fused.hip -- descriptors (Sec. II B, Eqs. 3-6) and atomic networks
// (Sec. II A, Eqs. 1-2) of one 16-atom tile in one kernel.
//
// The 16 groups of 16 lanes of a 256-thread block compute the descriptor
// vectors of the tile's atoms straight into LDS, normalised as the network's
// input; after a block barrier the block's four wavefronts run the tile
// through the network (energies, and dE/dG for the force pass).  The
// descriptor vectors do not travel through HBM, one launch per step is
// saved, and the network's dependent MFMA/tanh chains overlap with the
// descriptor work of the other blocks on the CU.  The result is bitwise that
// of the separate descriptor and network kernels.
#include "desc_dev.h"
#include "mlp_dev.h"

namespace aenet {

namespace {

template <int PREC>
struct DescType {
  typedef float R;
};
template <>
struct DescType<0> {
  typedef double R;
};

constexpr int kFusedLanes = 16;  // lanes per atom: 16 atoms = one network tile per block

template <int PREC, int NR, int NA, int NL, bool NARROW>
__global__ __launch_bounds__(256, 3) void k_fwd_mlp(DescParams dp, MlpParams mp, int x0_off) {
  typedef typename Mt<PREC>::T T;
  typedef typename DescType<PREC>::R R;
  constexpr int LPA = kFusedLanes;
  extern __shared__ __align__(16) unsigned char smem[];
  const TileInfo ti = tile_info(mp, blockIdx.x);
  const int g = threadIdx.x / LPA, l = threadIdx.x % LPA;
  const int i = ti.first + g;
  const bool active = g < ti.count;
  const int w0 = mp.wp[0], D = mp.w[0];
  const MlpNet& net = mp.net[ti.species];
  const T* sh = reinterpret_cast<const T*>(net.shift);
  const T* sc = reinterpret_cast<const T*>(net.scale);
  T* X0 = reinterpret_cast<T*>(smem + x0_off);
  T* xrow = X0 + g * (w0 + 1);
  R* G = dp.G ? reinterpret_cast<R*>(dp.G) + (size_t)(active ? i : 0) * dp.ldG : nullptr;
  if (dp.prio) __builtin_amdgcn_s_setprio(3);
  desc_fwd_group<R, NR, NA, LPA>(dp, i, active, g, l, smem, [&](int c, R v) {
    xrow[c] = (T(v) - sh[c]) * sc[c];
    if (G) G[c] = v;
  });
  // padding columns, and the rows of a tile shorter than 16 atoms, are zero
  for (int c = l; c < w0; c += LPA)
    if (!active || c >= D) xrow[c] = T(0);
  // the network phase (its first loads are issued before its barrier); its
  // work buffers reuse the descriptor pass's LDS
  mlp_tile_n<PREC, NL, mlp_mkh<PREC, NARROW>()>(mp, ti, X0, reinterpret_cast<T*>(smem), threadIdx.x, dp.prio);
}

template <int PREC, int NR, int NA>
void launch_fused(const DescParams& dp, const MlpParams& mp, int n_tiles, size_t lds, int x0_off,
                  hipStream_t s) {
  DescParams q = dp;
  // the network's depth and hidden width select the kernel (see mlp_tile_n)
  const bool narrow = mlp_narrow(mp);
  auto go = [&](auto kernel) {
    q.prio = fits_one_round(reinterpret_cast<const void*>(kernel), 16 * kFusedLanes, lds, n_tiles);
    hipLaunchKernelGGL(kernel, dim3(n_tiles), dim3(16 * kFusedLanes), lds, s, q, mp, x0_off);
  };
  switch (mp.n_layers) {  // 1..kMaxLayers, checked when the model is set up
    case 1: go(k_fwd_mlp<PREC, NR, NA, 1, true>); break;
    case 2: narrow ? go(k_fwd_mlp<PREC, NR, NA, 2, true>) : go(k_fwd_mlp<PREC, NR, NA, 2, false>); break;
    case 3: narrow ? go(k_fwd_mlp<PREC, NR, NA, 3, true>) : go(k_fwd_mlp<PREC, NR, NA, 3, false>); break;
    default: narrow ? go(k_fwd_mlp<PREC, NR, NA, 4, true>) : go(k_fwd_mlp<PREC, NR, NA, 4, false>); break;
  }
}

template <int PREC>
bool dispatch_fused(int nr, int na, const DescParams& dp, const MlpParams& mp, int n_tiles, size_t lds,
                    int x0_off, hipStream_t s) {
#define AENET_CASE(A, B)                                              \
  if (nr == A && na == B) {                                           \
    launch_fused<PREC, A, B>(dp, mp, n_tiles, lds, x0_off, s);        \
    return true;                                                      \
  }
  AENET_ORDERS(AENET_CASE)
#undef AENET_CASE
  return false;
}

}  // namespace

namespace {

// LDS of the fused kernel: the descriptor pass's compaction buffers (later the
// network's work buffers) from 0, the normalised input tile from x0_off
size_t fused_lds(int prec, const DescParams& dp, const MlpParams& mp, size_t* x0_off) {
  const size_t el = prec == 0 ? sizeof(double) : sizeof(float);
  const size_t fwd_bytes = (size_t)16 * 5 * dp.cap_ang * el;
  const size_t work_bytes = mlp_work_elems(mp) * el;
  *x0_off = ((fwd_bytes > work_bytes ? fwd_bytes : work_bytes) + 15) / 16 * 16;
  return *x0_off + (size_t)16 * (mp.wp[0] + 1) * el;
}

}  // namespace

bool fwd_mlp_fits(int prec, const DescParams& dp, const MlpParams& mp) {
  // crowded angular shells take the 64-lane descriptor kernel instead
  if ((dp.ang_hint > 0 ? dp.ang_hint : dp.cap_ang) > 48) return false;
  size_t x0_off;
  return fused_lds(prec, dp, mp, &x0_off) <= 65536;
}

bool launch_fwd_mlp(int prec, int nr, int na, const DescParams& dp, const MlpParams& mp, int n_tiles,
                    hipStream_t s) {
  static_assert(kMlpWaves * 64 == 16 * kFusedLanes, "one network tile per block");
  if (!fwd_mlp_fits(prec, dp, mp)) return false;
  if (n_tiles <= 0) return true;
  size_t x0_off;
  const size_t lds = fused_lds(prec, dp, mp, &x0_off);
  if (prec == 0) return dispatch_fused<0>(nr, na, dp, mp, n_tiles, lds, (int)x0_off, s);
  if (prec == 1) return dispatch_fused<1>(nr, na, dp, mp, n_tiles, lds, (int)x0_off, s);
  return dispatch_fused<2>(nr, na, dp, mp, n_tiles, lds, (int)x0_off, s);
}

}  // namespace aenet
