// mlp_dev.h -- device code shared by the network kernels and the fused
// descriptor + network kernel: MFMA tiles of the per-species atomic networks
// (Sec. II A, Eqs. 1-2).
#pragma once
#include <hip/hip_bf16.h>

#include "aenet_internal.h"

namespace aenet {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int PREC>
struct Mt;
template <>
struct Mt<0> {
  typedef double T;    // compute / storage type
  typedef double B;    // packed operand element
  typedef v4d Acc;
  static constexpr int KS = 4;
  static constexpr int BV = 1;  // operand elements per lane per k-step
};
template <>
struct Mt<1> {
  typedef float T;
  typedef float B;
  typedef v4f Acc;
  static constexpr int KS = 4;
  static constexpr int BV = 1;
};
template <>
struct Mt<2> {
  typedef float T;
  typedef __bf16 B;
  typedef v4f Acc;
  static constexpr int KS = 32;
  static constexpr int BV = 8;
};

// row of accumulator element i of this lane (column is lane & 15)
template <int PREC>
__device__ inline int acc_row(int lane, int i) {
  return PREC == 0 ? (lane >> 4) + 4 * i : 4 * (lane >> 4) + i;
}

// The B operand of one 16-column output block held by one wavefront: K/KS
// k-steps of one packed element (FP64/FP32) or eight BF16 values per lane.
// BF16 also holds an optional second operand: the low parts of a layer kept
// as a BF16 pair (has_lo, wave-uniform).
// MK: k-steps the fragment can hold (the full kMaxWidth by default).
template <int PREC, int MK = kMaxWidth / Mt<PREC>::KS>
struct Frag {
  static constexpr int maxks = MK;
  typename Mt<PREC>::B b[MK][Mt<PREC>::BV];
  typename Mt<PREC>::B lo[PREC == 2 ? MK : 1][PREC == 2 ? 8 : 1];
  bool has_lo;
};

// issue the loads of output block nb's B operand (K/KS k-steps), and of its
// low parts if Blo is not NULL (BF16 only)
template <int PREC, int MK>
__device__ __forceinline__ void load_frag(Frag<PREC, MK>& f, const typename Mt<PREC>::B* Bp, const typename Mt<PREC>::B* Blo,
                                 int nb, int K, int lane) {
  typedef Mt<PREC> M;
  constexpr int MAXKS = MK;
  const int ksteps = K / M::KS;
  f.has_lo = PREC == 2 && Blo != nullptr;
  // every k-step slot is loaded, those past the layer's width with a copy of
  // its last k-step (unused): loads under a branch would make the wait for
  // this fragment, one stage later, also wait for the next stage's loads
  const typename Mt<PREC>::B* Bl = f.has_lo ? Blo : Bp;
#pragma unroll
  for (int ks = 0; ks < MAXKS; ++ks) {
    const int kc = min(ks, ksteps - 1);
    if constexpr (PREC == 2) {
      const size_t o = (((size_t)nb * ksteps + kc) * 64 + lane) * 8;
      const v8bf v = *reinterpret_cast<const v8bf*>(Bp + o);
      const v8bf w = *reinterpret_cast<const v8bf*>(Bl + o);
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        f.b[ks][t] = v[t];
        f.lo[ks][t] = w[t];
      }
    } else {
      f.b[ks][0] = Bp[((size_t)nb * ksteps + kc) * 64 + lane];
    }
  }
}

// one 16x16 output block: sum over K of A[16 x K] (LDS, row-major, row stride
// ld) times the B operand in f.  All A operands are loaded before the MFMA
// chain so their latencies overlap.
template <int PREC, int MK>
__device__ __forceinline__ typename Mt<PREC>::Acc mfma_frag(const typename Mt<PREC>::T* A, int ld, int K,
                                                    const Frag<PREC, MK>& f, int lane) {
  typedef Mt<PREC> M;
  typename M::Acc acc = {0, 0, 0, 0};
  const int ksteps = K / M::KS;
  const int r = lane & 15, kq = lane >> 4;
  if constexpr (PREC == 0 || PREC == 1) {
    typedef typename M::T T;
    constexpr int MAXKS = MK;
    T a[MAXKS];
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks) a[ks] = A[r * ld + min(ks, ksteps - 1) * 4 + kq];
    // two independent accumulation chains (even / odd k-steps) halve the
    // dependent MFMA latency
    typename M::Acc acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < MAXKS; ks += 2) {
      if (ks < ksteps) {
        if constexpr (PREC == 0)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], f.b[ks][0], acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks], f.b[ks][0], acc, 0, 0, 0);
      }
      if (ks + 1 < ksteps) {
        if constexpr (PREC == 0)
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks + 1], f.b[ks + 1][0], acc1, 0, 0, 0);
        else
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks + 1], f.b[ks + 1][0], acc1, 0, 0, 0);
      }
    }
    acc += acc1;
  } else {
    // BF16 weights; the FP32 activations (or deltas) enter as a compensated
    // pair hi + lo of BF16 values (lo = the rounding error of hi), two
    // products per k-step on the BF16 MFMA, FP32 accumulation; a layer held
    // as a weight pair adds the product of the activations' hi part with the
    // weights' lo part
    constexpr int MAXKS = MK;
    v8bf ah[MAXKS], al[MAXKS], bb[MAXKS], bl[MAXKS];
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks) {
      const float* ap = A + r * ld + min(ks, ksteps - 1) * 32 + 8 * kq;
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const __bf16 hi = (__bf16)ap[t];
        ah[ks][t] = hi;
        al[ks][t] = (__bf16)(ap[t] - (float)hi);
        bb[ks][t] = f.b[ks][t];
        bl[ks][t] = f.lo[ks][t];
      }
    }
    typename M::Acc acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks)
      if (ks < ksteps) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bb[ks], acc, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], bb[ks], acc1, 0, 0, 0);
      }
    if (f.has_lo) {
#pragma unroll
      for (int ks = 0; ks < MAXKS; ++ks)
        if (ks < ksteps) acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], bl[ks], acc1, 0, 0, 0);
    }
    acc += acc1;
  }
  return acc;
}

template <int PREC>
__device__ inline typename Mt<PREC>::Acc mfma_block(const typename Mt<PREC>::T* A, int ld, int K,
                                                     const typename Mt<PREC>::B* Bp, int nb,
                                                     int lane) {
  Frag<PREC> f;
  load_frag<PREC>(f, Bp, nullptr, nb, K, lane);
  return mfma_frag<PREC>(A, ld, K, f, lane);
}

// tanh z = 1 - 2 / (e^{2z} + 1) with z clamped to [-20, 20] (tanh is +-1 there
// to double precision); the reciprocal is the hardware estimate refined by two
// Newton steps.  The absolute error is a few units of 1e-16 (the relative
// error grows for |z| << 1, which the network's sums do not see).
__device__ inline double tanh_act(double z) {
  const double zc = fmin(fmax(z, -20.0), 20.0);
  const double d = exp(2.0 * zc) + 1.0;
  double y = __builtin_amdgcn_rcp(d);
  y = y * (2.0 - d * y);
  y = y * (2.0 - d * y);
  return 1.0 - 2.0 * y;
}
// single precision: e^{2z} = 2^{2 z log2(e)} and 1 / (e^{2z} + 1) from the
// hardware exp2 and reciprocal (about 1 ulp each), z clamped to [-10, 10]
__device__ inline float tanh_act(float z) {
  const float zc = fminf(fmaxf(z, -10.0f), 10.0f);
  const float e = __builtin_amdgcn_exp2f(zc * 2.88539008177792681f);
  return 1.0f - 2.0f * __builtin_amdgcn_rcpf(e + 1.0f);
}

template <typename T>
__device__ inline T act_fn(int act, T z) {
  return act == 1 ? tanh_act(z) : z;
}
template <typename T>
__device__ inline T act_d1(int act, T x) {
  return act == 1 ? T(1) - x * x : T(1);
}
template <typename T>
__device__ inline T act_d2(int act, T x) {
  return act == 1 ? T(-2) * x * (T(1) - x * x) : T(0);
}

struct TileInfo {
  int species, first, count;
};

__device__ __forceinline__ TileInfo tile_info(const MlpParams& p, int tile) {
  TileInfo t{0, 0, 0};
  int s = 0;
  while (s + 1 < p.n_species && tile >= p.tile_off[s + 1]) ++s;
  t.species = s;
  t.first = p.sp_off[s] + (tile - p.tile_off[s]) * 16;
  t.count = min(16, p.sp_off[s + 1] - t.first);
  return t;
}

// element offset of the activations of layer l when X_0..X_{L-1} are stored
// one after the other with row strides wp[l] + 1
__host__ __device__ __forceinline__ size_t act_offset(const MlpParams& p, int l) {
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += 16 * (size_t)(p.wp[k] + 1);
  return o;
}

// Layout of the activation buffers of a tile (elements of T): X_0 (the
// normalised input, row stride wp[0] + 1) is passed separately; X_l for
// l >= 1 at work + act_offset(l) - act_offset(1) (row stride wp[l] + 1, the
// odd stride spreads the 16 rows of an MFMA operand over the LDS banks), then
// two delta buffers of 16 x (kMaxWidth + 1).
__host__ __device__ inline size_t mlp_work_elems(const MlpParams& p) {
  return act_offset(p, p.n_layers) - act_offset(p, 1) + 2 * 16 * (kMaxWidth + 1);
}

constexpr int kMlpWaves = 4;  // wavefronts per tile

// The matrix products of a tile in order: the hidden layers 1..L-1 forward
// (stages 0..L-2), then, for the input gradient, layers L-1..1 backward.
// Stage s multiplies a 16 x K operand by the B operand of `Bp` (K x N).
struct MlpStage {
  const void* Bp;
  const void* Blo;  // low parts of a BF16 weight pair, or NULL
  int K, N;
};
__device__ __forceinline__ MlpStage mlp_stage(const MlpParams& p, const MlpNet& net, int s) {
  const int H = p.n_layers - 1;
  if (s < H) return MlpStage{net.wf[s + 1], s == 0 ? net.wf_lo : nullptr, p.wp[s], p.wp[s + 1]};
  const int l = H - (s - H);
  return MlpStage{net.wb[l], l == 1 ? net.wb_lo : nullptr, p.wp[l], p.wp[l - 1]};
}
__device__ __forceinline__ int mlp_n_stages(const MlpParams& p) { return (p.n_layers - 1) * (p.gG ? 2 : 1); }

// Issue wavefront `wave`'s B-operand loads of stage s (it owns the 16-column
// block nb = wave; a layer is at most kMaxWidth = 16 * kMlpWaves wide).
template <int PREC, int MK>
__device__ __forceinline__ void mlp_prefetch(const MlpParams& p, const MlpNet& net, int s, int wave, int lane,
                                    Frag<PREC, MK>& f) {
  if (s >= mlp_n_stages(p)) return;
  const MlpStage st = mlp_stage(p, net, s);
  typedef typename Mt<PREC>::B Bt;
  if (wave < st.N / 16)
    load_frag<PREC>(f, reinterpret_cast<const Bt*>(st.Bp), reinterpret_cast<const Bt*>(st.Blo), wave, st.K,
                    lane);
}

// Per-thread constants of a tile's network, loaded with the first B operand
// (before the tile barrier) so that no layer waits on a global load of its
// own: the bias of the thread's output column in each hidden layer, the
// output weights of the columns it reduces for the energy (k = (tid & 15) +
// 16 m), and the input scaling of its output column in the last backward
// stage.  Indices are clamped into the padded arrays; values past the true
// widths are not used.
template <int PREC>
struct MlpConsts {
  typename Mt<PREC>::T bias[kMaxLayers];
  typename Mt<PREC>::T wl[kMaxWidth / 16];
  typename Mt<PREC>::T sc;
  double blast;  // output-layer bias (parameters may be replaced on the device)
};
template <int PREC>
__device__ __forceinline__ void mlp_consts(const MlpParams& p, const MlpNet& net, int tid, MlpConsts<PREC>& c) {
  typedef typename Mt<PREC>::T T;
  const int col = (tid >> 6) * 16 + (tid & 15);
  const int L = p.n_layers;
  c.bias[0] = T(0);
#pragma unroll
  for (int l = 1; l < kMaxLayers; ++l)
    c.bias[l] = l < L ? reinterpret_cast<const T*>(net.bias[l])[min(col, p.wp[l] - 1)] : T(0);
  const T* wl = reinterpret_cast<const T*>(net.wlast);
  const int KL = p.wp[L - 1];
#pragma unroll
  for (int m = 0; m < kMaxWidth / 16; ++m) c.wl[m] = wl[min((tid & 15) + 16 * m, KL - 1)];
  c.sc = reinterpret_cast<const T*>(net.scale)[min(col, p.w[0] - 1)];
  c.blast = *net.blast;
}

// The network phase of a tile.  Stage 0 (the input layer) has its own
// fragment b0; the B operands of stages 1, 2, ... rotate through three
// fragments ring[(s - 1) mod 3].  Stages 0 and 1, and the per-thread
// constants, are loaded before the block barrier that starts the phase, and
// stage s + 2 while stage s multiplies, so that no stage waits for loads
// issued in the stage before.  Only stage 0 multiplies by the input width;
// the others by a hidden width, so the ring holds MKH k-steps (half the
// registers when every hidden layer is at most 32 wide).  NL = p.n_layers
// (weight layers) is a template parameter and every stage a template
// instance, so every fragment is a fixed register set.
//
// Hidden layers, energy and (if p.gG) input gradient of one 16-atom tile
// whose normalised input is in X0, by kMlpWaves wavefronts (tid < 64 *
// kMlpWaves): wavefront w computes the 16-column output block w of every
// layer, with a block barrier between layers.
// loads of stage S of a network of NL layers into its fragment (the stages
// as in mlp_stage; none past the last stage)
template <int PREC, int NL, int S, typename F>
__device__ __forceinline__ void mt_load_into(const MlpParams& p, const MlpNet& net, int wave, int lane, F& f) {
  constexpr int H = NL - 1;
  typedef typename Mt<PREC>::B Bt;
  if constexpr (S < 2 * H) {
    if (S >= H && !p.gG) return;
    const void* Bp;
    const void* Blo;
    int K, N;
    if constexpr (S < H) {
      Bp = net.wf[S + 1];
      Blo = S == 0 ? net.wf_lo : nullptr;
      K = p.wp[S];
      N = p.wp[S + 1];
    } else {
      constexpr int l = H - (S - H);
      Bp = net.wb[l];
      Blo = l == 1 ? net.wb_lo : nullptr;
      K = p.wp[l];
      N = p.wp[l - 1];
    }
    if (wave < N / 16)
      load_frag<PREC>(f, reinterpret_cast<const Bt*>(Bp), reinterpret_cast<const Bt*>(Blo), wave, K, lane);
  }
}
template <int PREC, int NL, int MKH, int S>
__device__ __forceinline__ void mt_load(const MlpParams& p, const MlpNet& net, int wave, int lane,
                                        Frag<PREC>& b0, Frag<PREC, MKH> (&ring)[3]) {
  if constexpr (S == 0)
    mt_load_into<PREC, NL, 0>(p, net, wave, lane, b0);
  else
    mt_load_into<PREC, NL, S>(p, net, wave, lane, ring[(S - 1) % 3]);
}
template <int PREC, int MKH, int S>
__device__ __forceinline__ typename Mt<PREC>::Acc mt_product(const typename Mt<PREC>::T* A, int ld, int K,
                                                             int lane, const Frag<PREC>& b0,
                                                             const Frag<PREC, MKH> (&ring)[3]) {
  if constexpr (S == 0)
    return mfma_frag<PREC>(A, ld, K, b0, lane);
  else
    return mfma_frag<PREC>(A, ld, K, ring[(S - 1) % 3], lane);
}

// everything one stage of a tile needs; X[l] = the activations of layer l
// (X[NL] = the first delta buffer)
template <int PREC, int NL>
struct MtState {
  typename Mt<PREC>::T* X[NL + 1];
  int tid, lane, wave;
  typename Mt<PREC>::T* Dcur;
  typename Mt<PREC>::T* Dnext;
};

// hidden layer l of NL (stage l - 1)
template <int PREC, int NL, int MKH, int l>
__device__ __forceinline__ void mt_forward(const MlpParams& p, const MlpNet& net, MtState<PREC, NL>& st,
                                           Frag<PREC>& b0, Frag<PREC, MKH> (&ring)[3],
                                           const MlpConsts<PREC>& kc) {
  typedef typename Mt<PREC>::T T;
  if constexpr (l <= NL - 1) {
    mt_load<PREC, NL, MKH, l + 1>(p, net, st.wave, st.lane, b0, ring);
    const T* Xin = st.X[l - 1];
    T* Y = st.X[l];
    const int K = p.wp[l - 1], N = p.wp[l];
    const int act = p.act[l - 1];
    if (st.wave < N / 16) {
      const auto acc = mt_product<PREC, MKH, l - 1>(Xin, K + 1, K, st.lane, b0, ring);
      const int col = st.wave * 16 + (st.lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = acc_row<PREC>(st.lane, i);
        Y[row * (N + 1) + col] = act_fn<T>(act, T(acc[i]) + kc.bias[l]);
      }
    }
    __syncthreads();
    mt_forward<PREC, NL, MKH, l + 1>(p, net, st, b0, ring, kc);
  }
}

// back-propagation through layer l of NL (stage 2 (NL - 1) - l)
template <int PREC, int NL, int MKH, int l>
__device__ __forceinline__ void mt_backward(const MlpParams& p, const TileInfo& ti, const MlpNet& net,
                                            MtState<PREC, NL>& st, Frag<PREC>& b0,
                                            Frag<PREC, MKH> (&ring)[3], const MlpConsts<PREC>& kc) {
  typedef typename Mt<PREC>::T T;
  constexpr int DLD = kMaxWidth + 1;
  if constexpr (l >= 1) {
    constexpr int S = 2 * (NL - 1) - l;
    mt_load<PREC, NL, MKH, S + 2>(p, net, st.wave, st.lane, b0, ring);
    const int K = p.wp[l], N = p.wp[l - 1];
    const T* Xp = st.X[l - 1];
    const int actp = l >= 2 ? p.act[l - 2] : 0;
    T* gout = reinterpret_cast<T*>(p.gG);
    if (st.wave < N / 16) {
      const auto acc = mt_product<PREC, MKH, S>(st.Dcur, DLD, K, st.lane, b0, ring);
      const int col = st.wave * 16 + (st.lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = acc_row<PREC>(st.lane, i);
        const T v = T(acc[i]);
        if (l >= 2) {
          st.Dnext[row * DLD + col] = v * act_d1<T>(actp, Xp[row * (N + 1) + col]);
        } else if (row < ti.count && col < p.w[0]) {
          gout[(size_t)(ti.first + row) * p.ldG + col] = v * kc.sc;
        }
      }
    }
    __syncthreads();
    T* t = st.Dcur;
    st.Dcur = st.Dnext;
    st.Dnext = t;
    mt_backward<PREC, NL, MKH, l - 1>(p, ti, net, st, b0, ring, kc);
  }
}

template <int PREC, int NL, int MKH>
__device__ __forceinline__ void mlp_tile_n(const MlpParams& p, const TileInfo& ti, typename Mt<PREC>::T* X0,
                                           typename Mt<PREC>::T* work, int tid, int prio) {
  typedef typename Mt<PREC>::T T;
  constexpr int NT = 64 * kMlpWaves;
  constexpr int L = NL, H = NL - 1;
  constexpr int DLD = kMaxWidth + 1;  // row stride of the delta buffers
  static_assert(16 * kMlpWaves == kMaxWidth, "one output block per wavefront and layer");
  const MlpNet& net = p.net[ti.species];
  MtState<PREC, NL> st;
  st.tid = tid;
  st.lane = tid & 63;
  st.wave = tid >> 6;
  st.X[0] = X0;
  {
    T* x = work;
#pragma unroll
    for (int l = 1; l <= NL; ++l) {
      st.X[l] = x;
      x += 16 * (size_t)(p.wp[l] + 1);
    }
  }
  Frag<PREC> b0;
  Frag<PREC, MKH> ring[3];
  MlpConsts<PREC> kc;
  mt_load<PREC, NL, MKH, 0>(p, net, st.wave, st.lane, b0, ring);
  mt_load<PREC, NL, MKH, 1>(p, net, st.wave, st.lane, b0, ring);
  mlp_consts<PREC>(p, net, tid, kc);
  __syncthreads();  // the tile's input is in X0
  if (prio) __builtin_amdgcn_s_setprio(0);
  mt_forward<PREC, NL, MKH, 1>(p, net, st, b0, ring, kc);

  // output layer and per-atom energy: 16 lanes per row, each summing every
  // 16th column, then a 16-lane tree; the same thread starts the
  // back-propagation to the input at those columns (the output layer is
  // linear; X_{L-1} was produced by the activation of layer L-1, none if
  // L == 1)
  const T* XL = st.X[L - 1];
  const int KL = p.wp[L - 1];
  T* D0 = st.X[L];
  {
    static_assert(NT == 256, "16 rows x 16 lanes");
    const int r = tid >> 4, c0 = tid & 15;
    T e = T(0);
    T x[kMaxWidth / 16];
#pragma unroll
    for (int m = 0; m < kMaxWidth / 16; ++m) {
      const int k = c0 + 16 * m;
      if (k < KL) {
        x[m] = XL[r * (KL + 1) + k];
        e += x[m] * kc.wl[m];
      }
    }
#pragma unroll
    for (int o = 8; o > 0; o >>= 1) e += __shfl_xor(e, o, 16);
    if (c0 == 0 && r < ti.count) p.E[ti.first + r] = (double)e + kc.blast + net.e_offset;
    if (!p.gG) return;
#pragma unroll
    for (int m = 0; m < kMaxWidth / 16; ++m) {
      const int k = c0 + 16 * m;
      if (k < KL) D0[r * DLD + k] = L >= 2 ? kc.wl[m] * act_d1<T>(p.act[L - 2], x[m]) : kc.wl[m];
    }
  }
  __syncthreads();
  st.Dcur = D0;
  st.Dnext = D0 + 16 * DLD;
  if constexpr (H == 0) {
    T* gout = reinterpret_cast<T*>(p.gG);
    const T* sc = reinterpret_cast<const T*>(net.scale);
    for (int idx = tid; idx < 16 * p.wp[0]; idx += NT) {
      const int r = idx / p.wp[0], c = idx % p.wp[0];
      if (r < ti.count && c < p.w[0]) gout[(size_t)(ti.first + r) * p.ldG + c] = st.Dcur[r * DLD + c] * sc[c];
    }
  } else {
    mt_backward<PREC, NL, MKH, H>(p, ti, net, st, b0, ring, kc);
  }
}

// k-steps of the ring fragments of mlp_tile_n: half the full width when every
// hidden layer of the network is at most 32 wide (NARROW, decided on the host)
template <int PREC, bool NARROW>
constexpr int mlp_mkh() {
  return (NARROW ? kMaxWidth / 2 : kMaxWidth) / Mt<PREC>::KS;
}
inline bool mlp_narrow(const MlpParams& p) {
  for (int l = 1; l < p.n_layers; ++l)
    if (p.wp[l] > kMaxWidth / 2) return false;
  return true;
}

}  // namespace

}  // namespace aenet
