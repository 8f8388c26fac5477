// mlp.hip -- per-species atomic networks (Sec. II A, Eqs. 1-2) as MFMA GEMMs.
//
// Atoms are stored species by species, so a tile of 16 consecutive atoms
// belongs to one species and one network.  A tile is one block:
//   X_0 = (G - shift) * scale            (normalised input, computed in T)
//   X_l = tanh(X_{l-1} W_l^T + b_l)      (hidden layers, MFMA, bias + tanh fused)
//   E   = X_{L-1} . w_L + b_L + e_offset (per-atom energy, VALU)
// and, for forces, back-propagates to the input:
//   D_{L-1} = w_L * f'(X_{L-1});  D_{l-1} = (D_l W_l) * f'(X_{l-1});  dE/dG = (D_1 W_1) * scale.
// Activations stay in LDS between layers.  Precisions: 0 = FP64 MFMA
// (16x16x4), 1 = FP32 MFMA (16x16x4), 2 = BF16 weights (rounded to nearest
// even) on the 16x16x32 BF16 MFMA with FP32 accumulation, the FP32
// activations entering as a hi + lo pair of BF16 values (tanh, biases and
// normalisation in FP32).
//
// The training kernel runs the same forward pass plus the tangent pass
// along u (the descriptor JVP) and the reverse pass of
//   phi = eps * E - (dE/dX_0 . u*scale)
// (double back-propagation), accumulating dphi/dW and dphi/db of the tile
// into an LDS copy of the species' parameters with MFMA outer products.
#include <type_traits>

#include "mlp_dev.h"

namespace aenet {

namespace {

// Forward and input-gradient pass of one 16-atom tile per block: the tile's
// descriptors are loaded and normalised into LDS, then mlp_tile (which holds
// the barrier).
template <int PREC, int NL, bool NARROW>
__global__ __launch_bounds__(64 * kMlpWaves) void k_mlp(MlpParams p) {
  typedef typename Mt<PREC>::T T;
  constexpr int NT = 64 * kMlpWaves;  // threads per tile
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int tid = threadIdx.x;
  const TileInfo ti = tile_info(p, blockIdx.x);
  const MlpNet& net = p.net[ti.species];
  {
    const T* G = reinterpret_cast<const T*>(p.G);
    const T* sh = reinterpret_cast<const T*>(net.shift);
    const T* sc = reinterpret_cast<const T*>(net.scale);
    const int w0 = p.wp[0], D = p.w[0];
    // all loads of the tile issued before any use (16 x w0 <= 16 x 64 elements)
    constexpr int IT = 16 * kMaxWidth / NT;
    T v[IT];
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + NT * it;
      const int r = idx / w0, c = idx % w0;
      v[it] = (idx < 16 * w0 && r < ti.count && c < D) ? G[(size_t)(ti.first + r) * p.ldG + c] : T(0);
    }
#pragma unroll
    for (int it = 0; it < IT; ++it) {
      const int idx = tid + NT * it;
      const int r = idx / w0, c = idx % w0;
      if (idx < 16 * w0) lds[r * (w0 + 1) + c] = (r < ti.count && c < D) ? (v[it] - sh[c]) * sc[c] : T(0);
    }
  }
  mlp_tile_n<PREC, NL, mlp_mkh<PREC, NARROW>()>(p, ti, lds, lds + act_offset(p, 1), tid, 0);
}

// ------------------------------------------------------------------ training
// LDS: X_l, Xd_l (tangent), Zd_l for l < L (16 x wp[l] each), two adjoint pairs
// (A, T) of 16 x 64, Zbar/Zdbar of 16 x 64, then the gradient accumulator of
// one species in the padded layout.
__host__ __device__ inline size_t train_param_count(const MlpParams& p) {
  size_t n = 0;
  for (int l = 1; l <= p.n_layers; ++l) {
    const int out = l == p.n_layers ? 1 : p.wp[l];
    n += (size_t)out * p.wp[l - 1] + out;
  }
  return n;
}

template <int PREC>
__global__ __launch_bounds__(64) void k_mlp_train(MlpParams p) {
  typedef typename Mt<PREC>::T T;
  typedef typename Mt<PREC>::B Bt;
  extern __shared__ __align__(16) unsigned char smem[];
  T* lds = reinterpret_cast<T*>(smem);
  const int lane = threadIdx.x;
  const int L = p.n_layers;
  const size_t act_sz = act_offset(p, L);
  T* X = lds;                 // X_l at act_offset(l)
  T* Xd = X + act_sz;         // tangents
  T* Zd = Xd + act_sz;        // tangent pre-activations
  T* Aa = Zd + act_sz;        // adjoint of X (16 x 64)
  T* Ta = Aa + 16 * kMaxWidth;  // adjoint of Xd
  T* Zb = Ta + 16 * kMaxWidth;
  T* Zdb = Zb + 16 * kMaxWidth;
  T* gacc = Zdb + 16 * kMaxWidth;
  const size_t npar = train_param_count(p);

  // block -> (species, tile range): blocks are dealt out per species
  int s = 0;
  int tiles_lo = 0, tiles_hi = 0;
  {
    int b0 = 0;
    for (int t = 0; t < p.n_species; ++t) {
      const int nt = p.tile_off[t + 1] - p.tile_off[t];
      const int nb = (nt + p.tiles_per_block - 1) / p.tiles_per_block;
      if ((int)blockIdx.x < b0 + nb) {
        s = t;
        tiles_lo = p.tile_off[t] + ((int)blockIdx.x - b0) * p.tiles_per_block;
        tiles_hi = min(tiles_lo + p.tiles_per_block, p.tile_off[t + 1]);
        break;
      }
      b0 += nb;
    }
  }
  const MlpNet& net = p.net[s];
  for (size_t k = lane; k < npar; k += 64) gacc[k] = T(0);
  __syncthreads();

  const T* sh = reinterpret_cast<const T*>(net.shift);
  const T* sc = reinterpret_cast<const T*>(net.scale);
  const T* wl = reinterpret_cast<const T*>(net.wlast);
  const T* Gm = reinterpret_cast<const T*>(p.G);
  const T* Um = reinterpret_cast<const T*>(p.U);
  const int w0 = p.wp[0], D = p.w[0];
  const int KL = p.wp[L - 1];

  for (int tile = tiles_lo; tile < tiles_hi; ++tile) {
    const TileInfo ti = tile_info(p, tile);
    {
      constexpr int IT = 16 * kMaxWidth / 64;
      T g[IT], u[IT];
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = lane + 64 * it;
        const int r = idx / w0, c = idx % w0;
        const bool in = idx < 16 * w0 && r < ti.count && c < D;
        const size_t o = (size_t)(ti.first + (in ? r : 0)) * p.ldG + (in ? c : 0);
        g[it] = in ? Gm[o] : T(0);
        u[it] = in ? Um[o] : T(0);
      }
#pragma unroll
      for (int it = 0; it < IT; ++it) {
        const int idx = lane + 64 * it;
        const int r = idx / w0, c = idx % w0;
        if (idx < 16 * w0) {
          const bool in = r < ti.count && c < D;
          X[idx] = in ? (g[it] - sh[c]) * sc[c] : T(0);
          Xd[idx] = in ? u[it] * sc[c] : T(0);
        }
      }
    }
    __syncthreads();
    // forward and tangent
    for (int l = 1; l < L; ++l) {
      const size_t oi = act_offset(p, l - 1), oo = act_offset(p, l);
      const int K = p.wp[l - 1], N = p.wp[l];
      const Bt* Bp = reinterpret_cast<const Bt*>(net.wf[l]);
      const T* bias = reinterpret_cast<const T*>(net.bias[l]);
      const int act = p.act[l - 1];
      for (int nb = 0; nb < N / 16; ++nb) {
        auto acc = mfma_block<PREC>(X + oi, K, K, Bp, nb, lane);
        auto accd = mfma_block<PREC>(Xd + oi, K, K, Bp, nb, lane);
        const int col = nb * 16 + (lane & 15);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int row = acc_row<PREC>(lane, i);
          const T x = act_fn<T>(act, T(acc[i]) + bias[col]);
          X[oo + row * N + col] = x;
          Zd[oo + row * N + col] = T(accd[i]);
          Xd[oo + row * N + col] = act_d1<T>(act, x) * T(accd[i]);
        }
      }
      __syncthreads();
    }
    // output layer: E = X_{L-1} . w + b ; dE/dw gets eps X - Xd, db gets eps
    {
      const size_t o = act_offset(p, L - 1);
      T* gW = gacc + (npar - 1 - KL);  // last layer block: W_L [1 x KL] then b_L
      for (int c = lane; c < KL; c += 64) {
        T acc = T(0);
        for (int r = 0; r < ti.count; ++r) {
          const T e = T(p.eps_atom[ti.first + r]);
          acc += e * X[o + r * KL + c] - Xd[o + r * KL + c];
        }
        gW[c] += acc;
      }
      if (lane == 0) {
        T acc = T(0);
        for (int r = 0; r < ti.count; ++r) acc += T(p.eps_atom[ti.first + r]);
        gacc[npar - 1] += acc;
      }
      for (int idx = lane; idx < 16 * KL; idx += 64) {
        const int r = idx / KL, c = idx % KL;
        const T e = r < ti.count ? T(p.eps_atom[ti.first + r]) : T(0);
        Aa[idx] = e * wl[c];
        Ta[idx] = r < ti.count ? -wl[c] : T(0);
      }
    }
    __syncthreads();
    // hidden layers, top down
    size_t goff = 0;
    size_t goffs[kMaxLayers + 1];
    for (int l = 1; l <= L; ++l) {
      goffs[l] = goff;
      const int out = l == L ? 1 : p.wp[l];
      goff += (size_t)out * p.wp[l - 1] + out;
    }
    for (int l = L - 1; l >= 1; --l) {
      const size_t oo = act_offset(p, l), oi = act_offset(p, l - 1);
      const int N = p.wp[l], K = p.wp[l - 1];
      const int act = p.act[l - 1];
      for (int idx = lane; idx < 16 * N; idx += 64) {
        const T x = X[oo + idx];
        const T d1 = act_d1<T>(act, x), d2 = act_d2<T>(act, x);
        Zb[idx] = Aa[idx] * d1 + Ta[idx] * d2 * Zd[oo + idx];
        Zdb[idx] = Ta[idx] * d1;
      }
      __syncthreads();
      // dW_l[q][k] += sum_r Zb[r][q] X[r][k] + Zdb[r][q] Xd[r][k]  (MFMA over the 16 rows)
      T* gW = gacc + goffs[l];
      T* gb = gW + (size_t)N * K;
      for (int mb = 0; mb < N / 16; ++mb) {
        for (int nb = 0; nb < K / 16; ++nb) {
          typename Mt<PREC>::Acc acc = {0, 0, 0, 0};
          if constexpr (PREC == 0) {
            for (int ks = 0; ks < 4; ++ks) {
              const int r = ks * 4 + (lane >> 4);
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Zb[r * N + mb * 16 + (lane & 15)],
                                                         X[oi + r * K + nb * 16 + (lane & 15)], acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Zdb[r * N + mb * 16 + (lane & 15)],
                                                         Xd[oi + r * K + nb * 16 + (lane & 15)], acc, 0, 0, 0);
            }
          } else {
            for (int ks = 0; ks < 4; ++ks) {
              const int r = ks * 4 + (lane >> 4);
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Zb[r * N + mb * 16 + (lane & 15)],
                                                         X[oi + r * K + nb * 16 + (lane & 15)], acc, 0, 0, 0);
              acc = __builtin_amdgcn_mfma_f32_16x16x4f32(Zdb[r * N + mb * 16 + (lane & 15)],
                                                         Xd[oi + r * K + nb * 16 + (lane & 15)], acc, 0, 0, 0);
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int q = mb * 16 + acc_row<PREC == 0 ? 0 : 1>(lane, i);
            const int k = nb * 16 + (lane & 15);
            gW[(size_t)q * K + k] += T(acc[i]);
          }
        }
      }
      for (int q = lane; q < N; q += 64) {
        T acc = T(0);
        for (int r = 0; r < 16; ++r) acc += Zb[r * N + q];
        gb[q] += acc;
      }
      __syncthreads();
      if (l > 1) {
        // adjoints of the layer below: A = Zb W_l, T = Zdb W_l
        const Bt* Bp = reinterpret_cast<const Bt*>(net.wb[l]);
        for (int nb = 0; nb < K / 16; ++nb) {
          auto acc = mfma_block<PREC>(Zb, N, N, Bp, nb, lane);
          auto accd = mfma_block<PREC>(Zdb, N, N, Bp, nb, lane);
          const int col = nb * 16 + (lane & 15);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int row = acc_row<PREC>(lane, i);
            Aa[row * K + col] = T(acc[i]);
            Ta[row * K + col] = T(accd[i]);
          }
        }
        __syncthreads();
      }
    }
  }
  __syncthreads();
  // write this block's partial gradient row (other species' sections zero)
  double* out = p.grad_part + (size_t)blockIdx.x * p.n_params_pad;
  for (int k = lane; k < p.n_params_pad; k += 64) out[k] = 0.0;
  __syncthreads();
  for (size_t k = lane; k < npar; k += 64) out[p.param_off[s] + k] = (double)gacc[k];
}

__global__ void k_grad_reduce(int n_blocks, int n, const double* part, double* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = 0.0;
  for (int b = 0; b < n_blocks; ++b) s += part[(size_t)b * n + k];
  out[k] = s;
}

}  // namespace

size_t mlp_lds_bytes(int prec, const MlpParams& p) {
  const size_t el = prec == 0 ? sizeof(double) : sizeof(float);
  return (act_offset(p, 1) + mlp_work_elems(p)) * el;
}

size_t mlp_train_lds_bytes(int prec, const MlpParams& p) {
  const size_t el = prec == 0 ? sizeof(double) : sizeof(float);
  return (3 * act_offset(p, p.n_layers) + 4 * 16 * kMaxWidth + train_param_count(p)) * el;
}

void launch_mlp(int prec, const MlpParams& p, int n_tiles, hipStream_t s) {
  if (n_tiles <= 0) return;
  const size_t lds = mlp_lds_bytes(prec, p);
  const dim3 block(64 * kMlpWaves);
  const bool narrow = mlp_narrow(p);
  auto go = [&](auto kernel) { hipLaunchKernelGGL(kernel, dim3(n_tiles), block, lds, s, p); };
  // the network's depth and hidden width select the kernel (see mlp_tile_n)
  auto by_shape = [&](auto prec_tag) {
    constexpr int P = decltype(prec_tag)::value;
    switch (p.n_layers) {  // 1..kMaxLayers, checked when the model is set up
      case 1: go(k_mlp<P, 1, true>); break;
      case 2: narrow ? go(k_mlp<P, 2, true>) : go(k_mlp<P, 2, false>); break;
      case 3: narrow ? go(k_mlp<P, 3, true>) : go(k_mlp<P, 3, false>); break;
      default: narrow ? go(k_mlp<P, 4, true>) : go(k_mlp<P, 4, false>); break;
    }
  };
  if (prec == 0)
    by_shape(std::integral_constant<int, 0>());
  else if (prec == 1)
    by_shape(std::integral_constant<int, 1>());
  else
    by_shape(std::integral_constant<int, 2>());
}

void launch_mlp_train(int prec, const MlpParams& p, int n_blocks, hipStream_t s) {
  if (n_blocks <= 0) return;
  const size_t lds = mlp_train_lds_bytes(prec, p);
  if (prec == 0)
    hipLaunchKernelGGL(k_mlp_train<0>, dim3(n_blocks), dim3(64), lds, s, p);
  else
    hipLaunchKernelGGL(k_mlp_train<1>, dim3(n_blocks), dim3(64), lds, s, p);
}

void launch_grad_reduce(int n_blocks, int n_params_pad, const double* part, double* out,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_grad_reduce, dim3((n_params_pad + 255) / 256), dim3(256), 0, s, n_blocks,
                     n_params_pad, part, out);
}

size_t pack_b_operand_count(int prec, int K, int N) {
  (void)prec;
  return (size_t)K * N;  // K, N already padded: every element lands in exactly one slot
}

// B is K x N (row-major, ldb), already zero padded to multiples of 32 / 16
void pack_b_operand(int prec, const double* B, int K, int N, int ldb, void* out, int part) {
  if (prec == 0 || prec == 1) {
    const int ksteps = K / 4;
    for (int nb = 0; nb < N / 16; ++nb)
      for (int ks = 0; ks < ksteps; ++ks)
        for (int lane = 0; lane < 64; ++lane) {
          const double v = B[(size_t)(ks * 4 + lane / 16) * ldb + nb * 16 + lane % 16];
          const size_t o = ((size_t)nb * ksteps + ks) * 64 + lane;
          if (prec == 0)
            reinterpret_cast<double*>(out)[o] = v;
          else
            reinterpret_cast<float*>(out)[o] = (float)v;
        }
  } else {
    const int ksteps = K / 32;
    for (int nb = 0; nb < N / 16; ++nb)
      for (int ks = 0; ks < ksteps; ++ks)
        for (int lane = 0; lane < 64; ++lane)
          for (int t = 0; t < 8; ++t) {
            const double v = B[(size_t)(ks * 32 + 8 * (lane / 16) + t) * ldb + nb * 16 + lane % 16];
            const size_t o = (((size_t)nb * ksteps + ks) * 64 + lane) * 8 + t;
            const __hip_bfloat16 hi = __float2bfloat16((float)v);
            reinterpret_cast<__hip_bfloat16*>(out)[o] =
                part == 0 ? hi : __float2bfloat16((float)(v - (double)__bfloat162float(hi)));
          }
  }
}

}  // namespace aenet
