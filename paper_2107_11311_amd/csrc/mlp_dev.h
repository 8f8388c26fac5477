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

// one 16x16 output block: sum over K of A[16 x K] (LDS, row-major, row stride
// ld) times the packed B operand block nb (K/KS k-steps).  All operands of the
// block are loaded before the MFMA chain so their latencies overlap.
template <int PREC>
__device__ inline typename Mt<PREC>::Acc mfma_block(const typename Mt<PREC>::T* A, int ld, int K,
                                                     const typename Mt<PREC>::B* Bp, int nb,
                                                     int lane) {
  typedef Mt<PREC> M;
  typename M::Acc acc = {0, 0, 0, 0};
  const int ksteps = K / M::KS;
  const int r = lane & 15, kq = lane >> 4;
  if constexpr (PREC == 0 || PREC == 1) {
    typedef typename M::T T;
    constexpr int MAXKS = kMaxWidth / 4;
    T a[MAXKS], b[MAXKS];
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks) {
      if (ks < ksteps) {
        a[ks] = A[r * ld + ks * 4 + kq];
        b[ks] = Bp[((size_t)nb * ksteps + ks) * 64 + lane];
      }
    }
    // two independent accumulation chains (even / odd k-steps) halve the
    // dependent MFMA latency
    typename M::Acc acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < MAXKS; ks += 2) {
      if (ks < ksteps) {
        if constexpr (PREC == 0)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], b[ks], acc, 0, 0, 0);
        else
          acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks], b[ks], acc, 0, 0, 0);
      }
      if (ks + 1 < ksteps) {
        if constexpr (PREC == 0)
          acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks + 1], b[ks + 1], acc1, 0, 0, 0);
        else
          acc1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ks + 1], b[ks + 1], acc1, 0, 0, 0);
      }
    }
    acc += acc1;
  } else {
    // BF16 weights; the FP32 activations (or deltas) enter as a compensated
    // pair hi + lo of BF16 values (lo = the rounding error of hi), two
    // products per k-step on the BF16 MFMA, FP32 accumulation
    constexpr int MAXKS = kMaxWidth / 32;
    v8bf ah[MAXKS], al[MAXKS], b[MAXKS];
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks) {
      if (ks < ksteps) {
        const float* ap = A + r * ld + ks * 32 + 8 * kq;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
          const __bf16 hi = (__bf16)ap[t];
          ah[ks][t] = hi;
          al[ks][t] = (__bf16)(ap[t] - (float)hi);
        }
        b[ks] = *reinterpret_cast<const v8bf*>(Bp + (((size_t)nb * ksteps + ks) * 64 + lane) * 8);
      }
    }
    typename M::Acc acc1 = {0, 0, 0, 0};
#pragma unroll
    for (int ks = 0; ks < MAXKS; ++ks)
      if (ks < ksteps) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[ks], b[ks], acc, 0, 0, 0);
        acc1 = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ks], b[ks], acc1, 0, 0, 0);
      }
    acc += acc1;
  }
  return acc;
}

template <typename T>
__device__ inline T act_fn(int act, T z) {
  return act == 1 ? tanh(z) : z;
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

__device__ inline TileInfo tile_info(const MlpParams& p, int tile) {
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
__host__ __device__ inline size_t act_offset(const MlpParams& p, int l) {
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

// Hidden layers, energy and (if p.gG) input gradient of one 16-atom tile
// whose normalised input is in X0, by kMlpWaves wavefronts (tid < 64 *
// kMlpWaves): the 16-column output blocks of every layer are dealt out over
// the waves, with a block barrier between layers.
template <int PREC>
__device__ inline void mlp_tile(const MlpParams& p, const TileInfo& ti, typename Mt<PREC>::T* X0,
                                typename Mt<PREC>::T* work, int tid) {
  typedef typename Mt<PREC>::T T;
  typedef typename Mt<PREC>::B Bt;
  constexpr int NT = 64 * kMlpWaves;
  const int lane = tid & 63, wave = tid >> 6;
  const MlpNet& net = p.net[ti.species];
  const int L = p.n_layers;
  constexpr int DLD = kMaxWidth + 1;  // row stride of the delta buffers
  const size_t base1 = act_offset(p, 1);
  auto X = [&](int l) { return l == 0 ? X0 : work + (act_offset(p, l) - base1); };
  T* D0 = work + (act_offset(p, L) - base1);
  T* D1 = D0 + 16 * DLD;

  // hidden layers
  for (int l = 1; l < L; ++l) {
    const T* Xin = X(l - 1);
    T* Y = X(l);
    const int K = p.wp[l - 1], N = p.wp[l];
    const Bt* Bp = reinterpret_cast<const Bt*>(net.wf[l]);
    const T* bias = reinterpret_cast<const T*>(net.bias[l]);
    const int act = p.act[l - 1];
    for (int nb = wave; nb < N / 16; nb += kMlpWaves) {
      auto acc = mfma_block<PREC>(Xin, K + 1, K, Bp, nb, lane);
      const int col = nb * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = acc_row<PREC>(lane, i);
        Y[row * (N + 1) + col] = act_fn<T>(act, T(acc[i]) + bias[col]);
      }
    }
    __syncthreads();
  }

  // output layer and per-atom energy
  const T* XL = X(L - 1);
  const int KL = p.wp[L - 1];
  const T* wl = reinterpret_cast<const T*>(net.wlast);
  if (tid < 16) {
    T e = T(0);
    for (int k = 0; k < KL; ++k) e += XL[tid * (KL + 1) + k] * wl[k];
    if (tid < ti.count) p.E[ti.first + tid] = (double)e + net.blast + net.e_offset;
  }
  if (!p.gG) return;

  // back-propagation to the input (the output layer is linear; X_{L-1} was
  // produced by the activation of layer L-1, none if L == 1)
  for (int idx = tid; idx < 16 * KL; idx += NT) {
    const int r = idx / KL, c = idx % KL;
    const T x = XL[r * (KL + 1) + c];
    D0[r * DLD + c] = L >= 2 ? wl[c] * act_d1<T>(p.act[L - 2], x) : wl[c];
  }
  __syncthreads();
  T* Dcur = D0;
  T* Dnext = D1;
  T* gout = reinterpret_cast<T*>(p.gG);
  const T* sc = reinterpret_cast<const T*>(net.scale);
  if (L == 1) {
    for (int idx = tid; idx < 16 * p.wp[0]; idx += NT) {
      const int r = idx / p.wp[0], c = idx % p.wp[0];
      if (r < ti.count && c < p.w[0]) gout[(size_t)(ti.first + r) * p.ldG + c] = Dcur[r * DLD + c] * sc[c];
    }
    return;
  }
  for (int l = L - 1; l >= 1; --l) {
    const int K = p.wp[l], N = p.wp[l - 1];
    const Bt* Bp = reinterpret_cast<const Bt*>(net.wb[l]);
    const T* Xp = X(l - 1);
    const int actp = l >= 2 ? p.act[l - 2] : 0;
    for (int nb = wave; nb < N / 16; nb += kMlpWaves) {
      auto acc = mfma_block<PREC>(Dcur, DLD, K, Bp, nb, lane);
      const int col = nb * 16 + (lane & 15);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = acc_row<PREC>(lane, i);
        const T v = T(acc[i]);
        if (l >= 2) {
          Dnext[row * DLD + col] = v * act_d1<T>(actp, Xp[row * (N + 1) + col]);
        } else if (row < ti.count && col < p.w[0]) {
          gout[(size_t)(ti.first + row) * p.ldG + col] = v * sc[col];
        }
      }
    }
    __syncthreads();
    T* t = Dcur;
    Dcur = Dnext;
    Dnext = t;
  }
}

}  // namespace

}  // namespace aenet
