// host.hip -- host runtime of the GPU library and the C ABI of
// include/aenet_gpu.h: model validation and packing, device memory, the
// caller-order <-> species-sorted internal order, neighbour-list capacity
// management and retries, and the call sequences of energy/forces, MD and
// the training-loss gradient.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/aenet_gpu.h"
#include "aenet_internal.h"

using namespace aenet;

namespace {

constexpr double kKappa = 9648.533215665;  // (eV/amu) in A^2/ps^2

struct DevMem {
  void* p = nullptr;
  size_t bytes = 0;
  DevMem() = default;
  DevMem(const DevMem&) = delete;
  DevMem& operator=(const DevMem&) = delete;
  ~DevMem() {
    if (p) (void)hipFree(p);
  }
  template <class T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};

int pad_to(int x, int m) { return (x + m - 1) / m * m; }

// Bump allocator over a fixed device region (the no-allocation entry point's
// workspace): buffers are handed out in call order, none is freed.
struct Arena {
  unsigned char* base = nullptr;
  size_t size = 0, used = 0;
};

}  // namespace

struct aenet_ctx {
  // model
  // nr, na, D: the model's descriptor orders and dimension; knr, kna, kD:
  // those of the compiled kernels that compute it (the smallest compiled
  // pair with knr >= nr and kna >= na).  The model's components are a subset
  // of the kernels' (same cutoffs, the lower orders of each block): colmap[k]
  // is the kernel column of model column k; the other kernel columns enter
  // the networks with input scale 0 and zero weights, so they add nothing.
  int S = 0, nr = 0, na = 0, D = 0, knr = 0, kna = 0, kD = 0, ldG = 0, prec = 0, device = 0;
  std::vector<int> colmap;                 // [D]
  double rr = 0, ra = 0, skin = 0, rlist = 0;
  double tw[kMaxSpecies] = {0}, mass[kMaxSpecies] = {0};
  bool have_mass = false;
  // Networks: L weight layers for every species.  w/wp are the kernels'
  // widths: the kernel descriptor dimension, then per hidden layer the
  // largest width of any species (a narrower species' extra units have zero
  // weights and bias: tanh(0) = 0 and nothing reads them), then 1.
  int L = 0;
  int w[kMaxLayers + 1] = {0}, wp[kMaxLayers + 1] = {0}, act[kMaxLayers] = {0};
  std::vector<int64_t> poff;               // [S + 1] first parameter of each species (API layout)
  int64_t nps_int = 0;                     // kernel-shape (unpadded) parameters per species
  std::vector<int> imap;                   // [S * nps_int] API parameter of each, -1: structural zero
  std::vector<double> params;              // [poff[S]] the parameters (API layout)
  std::vector<double> shift, scale;        // [S * kD] (kernel columns)
  double e_off[kMaxSpecies] = {0};
  int npad_species = 0;                    // padded parameters per species (training layout)
  hipStream_t stream = nullptr;
  std::string err;
  int rebuild_every = 50;
  aenet_stats stats{};

  DevMem netbuf;        // packed network operands
  DevMem d_blast;       // [kMaxSpecies] output-layer bias per species
  DevMem d_params;      // [poff[S]] the parameters (API layout), device copy
  DevMem d_packmap;     // [n_pack] netbuf element -> parameter index (FP64/FP32)
  DevMem d_blastsrc;    // [S] parameter index of each species' output bias
  int64_t n_pack = 0;
  int blast_src[kMaxSpecies] = {0};
  bool params_host_stale = false;  // d_params is newer than params (set on the device)
  int loss_form = 0;               // AENET_LOSS_*
  MlpParams mlp{};      // pointers into netbuf (species part); geometry filled per call
  DevMem d_pidx;        // API parameter index -> padded index

  // geometry
  int64_t n = 0;
  int n_struct = 0;
  std::vector<int32_t> species_cache;
  std::vector<int64_t> offsets_cache;
  std::vector<int> perm;
  int sp_off[kMaxSpecies + 1] = {0};
  std::vector<BoxInfo> boxes;
  int pbc[3] = {1, 1, 1};
  int n_cells = 0;
  int cap = 0, cap_ang = 0;
  int cap_user = 0, cap_ang_user = 0;  // capacities set by the caller (0: estimate)
  int tp = 0;  // candidate capacity of the per-cell row kernel (0: per-atom row kernels)
  // descriptor forward + networks in one kernel: on by default for the FP32
  // and BF16 networks; with FP64 descriptors all blocks of the water
  // workload run in one round and the network phase cannot overlap other
  // blocks' descriptor work, so two kernels are as fast
  bool fused = true;
  int ang_mean = 0;  // expected mean number of neighbours within R_a (densest structure)
  int ang_method = 0;  // AENET_ANGULAR_*: pair sums, factorised, or chosen by the shell size
  bool nbr_valid = false;
  // the cell counters and the build's block counter are zero (what a build
  // expects; every successful call leaves them so)
  bool counters_clean = false;
  // the device holds the end state of the last md_step call: internal
  // positions, forces at them, the neighbour rows and their reference
  // positions; anything else that uses the buffers clears it
  bool md_state = false;
  const double* md_pos_out = nullptr;  // the position buffer the last md_step call wrote
  // non-NULL during a no-allocation call: ensure() carves buffers from this
  // region instead of allocating
  Arena* arena = nullptr;

  DevMem d_perm, d_species, d_wq, d_seg, d_segoff, d_segcount, d_boxes;
  DevMem d_pos, d_pos_ref, d_vel, d_F, d_Fself, d_E, d_Eorig, d_G, d_gG, d_pg, d_U, d_adj, d_eps,
      d_tmp, d_red, d_scal, d_flags, d_mass, d_invmk;
  DevMem d_cell_count, d_cell_start, d_cell_fill, d_cell_atoms, d_atom_cell, d_nbr, d_segs, d_nnb, d_nang, d_rev;
  DevMem d_bin_count, d_bin_atoms;  // MD: cell bins filled by the integrator
  DevMem d_ridx, d_nrad;            // contributing entries, from the forward pass
  DevMem d_shA, d_gang;             // factorised angular descriptor: per-atom sums, entry gradients
  DevMem d_xmap;                    // [n_grid] atom of each force-pass block (-1: none)
  int n_grid = 0;
  DevMem d_judge;                   // partial sums of aenet_rms_diff_dev
  DevMem d_vir;                     // [9][n] per-atom virial, then its 9 sums
  bool want_vir = false;            // the next force pass also forms the virial
  DevMem d_build;  // [2] ints: decision of the current build, block counter
  DevMem d_save_pos, d_save_vel, d_save_F, d_estruct, d_gradpart, d_gradpad;
  DevMem h_pos, h_vel, h_F, h_E;  // device staging for the host-pointer entry points
  int* h_flags = nullptr;          // [16] pinned host copy of the status words

  // kernel timing
  bool profiling = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<int> ev_class;  // class of event pair k (events 2k, 2k+1)
  double prof_ms[AENET_K_COUNT] = {0};
  int64_t prof_n[AENET_K_COUNT] = {0};
};

namespace {

aenet_status fail(aenet_ctx* c, aenet_status code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIP_TRY(c, expr)                                                                     \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess)                                                                    \
      return fail(c, AENET_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));     \
  } while (0)

#define TRY(expr)                       \
  do {                                  \
    aenet_status st_ = (expr);          \
    if (st_ != AENET_OK) return st_;    \
  } while (0)

aenet_status ensure(aenet_ctx* c, DevMem& m, size_t bytes) {
  if (bytes == 0) bytes = 256;
  if (m.bytes >= bytes) return AENET_OK;
  if (c->arena) {
    // no-allocation call: a (larger) slice of the workspace; what the buffer
    // held before is not kept (every buffer is requested before it is filled)
    const size_t b = (bytes + 255) / 256 * 256;
    if (c->arena->used + b > c->arena->size)
      return fail(c, AENET_E_INVALID,
                  "the no-allocation workspace (" + std::to_string(c->arena->size) +
                      " bytes) is too small for this structure; use aenet_energy_forces_dev");
    m.p = c->arena->base + c->arena->used;
    m.bytes = b;
    c->arena->used += b;
    return AENET_OK;
  }
  if (m.p) {
    (void)hipFree(m.p);
    m.p = nullptr;
    m.bytes = 0;
  }
  size_t b = (bytes + bytes / 8 + 255) / 256 * 256;
  if (hipMalloc(&m.p, b) != hipSuccess) {
    (void)hipGetLastError();
    m.p = nullptr;
    return fail(c, AENET_E_OOM, "device allocation of " + std::to_string(b) + " bytes failed");
  }
  m.bytes = b;
  return AENET_OK;
}

size_t real_size(const aenet_ctx* c) { return c->prec == 0 ? sizeof(double) : sizeof(float); }
int desc_prec(const aenet_ctx* c) { return c->prec == 0 ? 0 : 1; }

// ------------------------------------------------------------------ network packing
// The per-precision network operands of every species in one device buffer
// (netbuf): per hidden layer the forward and backward MFMA B operands and the
// bias, then the output weights and the input shift and scale; the output
// bias of each species lives in d_blast.  For FP64/FP32 contexts a map from
// every netbuf element to the flat parameter it holds (-1: padding, zero;
// -2: input shift/scale, not a parameter) lets the device repack parameters
// that are already in device memory (aenet_set_params_dev).
aenet_status pack_networks(aenet_ctx* c) {
  const int S = c->S, L = c->L;
  const int prec = c->prec;
  const size_t el = real_size(c);
  const size_t bel = prec == 0 ? 8 : (prec == 1 ? 4 : 2);
  size_t total = 0;
  auto take = [&](size_t bytes) {
    size_t o = total;
    total += (bytes + 255) / 256 * 256;
    return o;
  };
  struct SpOff {
    size_t wf[kMaxLayers], wb[kMaxLayers], bias[kMaxLayers], wlast, shift, scale, wf_lo, wb_lo;
  };
  // BF16: the input layer as a hi + lo pair of BF16 operands
  const bool pair1 = prec == 2 && L >= 2;
  std::vector<SpOff> so(S);
  for (int s = 0; s < S; ++s) {
    for (int l = 1; l < L; ++l) {
      so[s].wf[l] = take(pack_b_operand_count(prec, c->wp[l - 1], c->wp[l]) * bel);
      so[s].wb[l] = take(pack_b_operand_count(prec, c->wp[l], c->wp[l - 1]) * bel);
      so[s].bias[l] = take((size_t)c->wp[l] * el);
    }
    if (pair1) {
      so[s].wf_lo = take(pack_b_operand_count(prec, c->wp[0], c->wp[1]) * bel);
      so[s].wb_lo = take(pack_b_operand_count(prec, c->wp[1], c->wp[0]) * bel);
    }
    so[s].wlast = take((size_t)c->wp[L - 1] * el);
    so[s].shift = take((size_t)c->ldG * el);
    so[s].scale = take((size_t)c->ldG * el);
  }
  // Fills the layout from per-species parameter values P(s, k), k indexing
  // the kernel-shape parameters (layer by layer W_l row-major, then b_l);
  // put(o, idx, v) stores element idx of the section at byte offset o,
  // packB(B, K, N, o, part) a B operand, blast(s, v) the output bias;
  // pad is the value of padded B-operand entries.
  auto fill = [&](auto P, auto put, auto packB, auto blast, double pad, double shift_scale_mark) {
    for (int s = 0; s < S; ++s) {
      size_t po = 0;
      for (int l = 1; l <= L; ++l) {
        const int in = c->w[l - 1], out = c->w[l];
        const size_t wo = po, bo = po + (size_t)out * in;
        po += (size_t)out * in + out;
        if (l < L) {
          const int Kp = c->wp[l - 1], Np = c->wp[l];
          std::vector<double> Bf((size_t)Kp * Np, pad), Bb((size_t)Np * Kp, pad);
          for (int q = 0; q < out; ++q)
            for (int k = 0; k < in; ++k) {
              Bf[(size_t)k * Np + q] = P(s, wo + (size_t)q * in + k);  // forward: B[k][n] = W[n][k]
              Bb[(size_t)q * Kp + k] = P(s, wo + (size_t)q * in + k);  // backward: B[k][n] = W[k][n]
            }
          packB(Bf.data(), Kp, Np, so[s].wf[l], 0);
          packB(Bb.data(), Np, Kp, so[s].wb[l], 0);
          if (pair1 && l == 1) {
            packB(Bf.data(), Kp, Np, so[s].wf_lo, 1);
            packB(Bb.data(), Np, Kp, so[s].wb_lo, 1);
          }
          for (int q = 0; q < out; ++q) put(so[s].bias[l], q, P(s, bo + q));
        } else {
          for (int k = 0; k < in; ++k) put(so[s].wlast, k, P(s, wo + k));
          blast(s, P(s, bo));
        }
      }
      for (int k = 0; k < c->kD; ++k) {
        put(so[s].shift, k, shift_scale_mark < 0 ? shift_scale_mark : c->shift[(size_t)s * c->kD + k]);
        put(so[s].scale, k, shift_scale_mark < 0 ? shift_scale_mark : c->scale[(size_t)s * c->kD + k]);
      }
    }
  };
  std::vector<unsigned char> host(total, 0);
  double blast_v[kMaxSpecies] = {0};
  auto api = [&](int s, size_t k) { return c->imap[(size_t)s * c->nps_int + k]; };
  fill([&](int s, size_t k) { return api(s, k) >= 0 ? c->params[api(s, k)] : 0.0; },
       [&](size_t o, int idx, double v) {
         if (el == 8)
           reinterpret_cast<double*>(host.data() + o)[idx] = v;
         else
           reinterpret_cast<float*>(host.data() + o)[idx] = (float)v;
       },
       [&](const double* B, int K, int N, size_t o, int part) {
         pack_b_operand(prec, B, K, N, N, host.data() + o, part);
       },
       [&](int s, double v) { blast_v[s] = v; }, 0.0, 0.0);
  TRY(ensure(c, c->netbuf, total));
  HIP_TRY(c, hipMemcpy(c->netbuf.p, host.data(), total, hipMemcpyHostToDevice));
  TRY(ensure(c, c->d_blast, kMaxSpecies * sizeof(double)));
  HIP_TRY(c, hipMemcpy(c->d_blast.p, blast_v, kMaxSpecies * sizeof(double), hipMemcpyHostToDevice));
  TRY(ensure(c, c->d_params, c->params.size() * sizeof(double)));
  HIP_TRY(c, hipMemcpy(c->d_params.p, c->params.data(), c->params.size() * sizeof(double),
                       hipMemcpyHostToDevice));
  if (prec != 2 && c->n_pack == 0) {
    // the element map (built once: the layout depends only on the shapes)
    std::vector<double> map(total / el, -1.0);
    fill([&](int s, size_t k) { return (double)api(s, k); },
         [&](size_t o, int idx, double v) { map[o / el + idx] = v; },
         [&](const double* B, int K, int N, size_t o, int) { pack_b_operand(0, B, K, N, N, map.data() + o / el); },
         [&](int s, double v) { c->blast_src[s] = (int)v; }, -1.0, -2.0);
    std::vector<int> imap(map.size());
    for (size_t k = 0; k < map.size(); ++k) imap[k] = (int)map[k];
    TRY(ensure(c, c->d_packmap, imap.size() * sizeof(int)));
    HIP_TRY(c, hipMemcpy(c->d_packmap.p, imap.data(), imap.size() * sizeof(int), hipMemcpyHostToDevice));
    TRY(ensure(c, c->d_blastsrc, kMaxSpecies * sizeof(int)));
    HIP_TRY(c, hipMemcpy(c->d_blastsrc.p, c->blast_src, kMaxSpecies * sizeof(int), hipMemcpyHostToDevice));
    c->n_pack = (int64_t)imap.size();
  }
  unsigned char* base = c->netbuf.as<unsigned char>();
  for (int s = 0; s < S; ++s) {
    MlpNet& nt = c->mlp.net[s];
    for (int l = 1; l < L; ++l) {
      nt.wf[l] = base + so[s].wf[l];
      nt.wb[l] = base + so[s].wb[l];
      nt.bias[l] = base + so[s].bias[l];
    }
    nt.wlast = base + so[s].wlast;
    nt.shift = base + so[s].shift;
    nt.scale = base + so[s].scale;
    nt.wf_lo = pair1 ? base + so[s].wf_lo : nullptr;
    nt.wb_lo = pair1 ? base + so[s].wb_lo : nullptr;
    nt.blast = c->d_blast.as<double>() + s;
    nt.e_offset = c->e_off[s];
  }
  return AENET_OK;
}

// ------------------------------------------------------------------ geometry
aenet_status prepare(aenet_ctx* c, int n_struct, const int64_t* offsets, const int32_t* species,
                     const double* boxes, const uint8_t* pbc, const double* pos_dev, hipStream_t st) {
  if (n_struct < 1 || !offsets || offsets[0] != 0) return fail(c, AENET_E_INVALID, "bad structure offsets");
  for (int s = 0; s < n_struct; ++s)
    if (offsets[s + 1] < offsets[s]) return fail(c, AENET_E_INVALID, "structure offsets must not decrease");
  const int64_t n = offsets[n_struct];
  if (n > kMaxAtoms || n > (int64_t)INT32_MAX / 4) return fail(c, AENET_E_INVALID, "too many atoms");
  if (n > 0 && !species) return fail(c, AENET_E_INVALID, "species is NULL");
  for (int64_t i = 0; i < n; ++i)
    if (species[i] < 0 || species[i] >= c->S)
      return fail(c, AENET_E_SPECIES, "species id " + std::to_string(species[i]) + " of atom " +
                                          std::to_string(i) + " outside 0.." + std::to_string(c->S - 1));
  int pb[3];
  for (int a = 0; a < 3; ++a) pb[a] = pbc ? (pbc[a] ? 1 : 0) : 1;
  // cell grids
  std::vector<BoxInfo> bx(n_struct);
  int64_t cells = 0;
  for (int s = 0; s < n_struct; ++s) {
    BoxInfo& b = bx[s];
    for (int a = 0; a < 3; ++a) {
      const double L = boxes[3 * s + a];
      if (!(L > 0.0) || !std::isfinite(L)) return fail(c, AENET_E_BOX, "box edges must be positive and finite");
      if (pb[a] && L < c->rlist)
        return fail(c, AENET_E_BOX, "periodic box edge " + std::to_string(L) +
                                        " A is shorter than the neighbour-list radius " +
                                        std::to_string(c->rlist) + " A");
      int nc = (int)std::min<double>(std::floor(L / c->rlist), 1024.0);
      while (nc > 1 && L / nc < c->rlist * (1.0 + 1e-12)) --nc;
      if (nc < 1) nc = 1;
      b.L[a] = L;
      b.nc[a] = nc;
    }
    b.cell_base = (int)cells;
    cells += (int64_t)b.nc[0] * b.nc[1] * b.nc[2];
    if (cells > (1 << 28)) return fail(c, AENET_E_INVALID, "too many neighbour cells");
  }
  const bool same = (n == c->n && n_struct == c->n_struct &&
                     c->offsets_cache.size() == (size_t)n_struct + 1 &&
                     std::equal(offsets, offsets + n_struct + 1, c->offsets_cache.begin()) &&
                     c->species_cache.size() == (size_t)n &&
                     (n == 0 || std::memcmp(species, c->species_cache.data(), n * sizeof(int32_t)) == 0));
  // same cell grids as the last call
  bool box_same = same && c->boxes.size() == (size_t)n_struct && c->d_boxes.p != nullptr;
  for (int a = 0; a < 3 && box_same; ++a) box_same = c->pbc[a] == pb[a];
  for (int s = 0; s < n_struct && box_same; ++s)
    for (int a = 0; a < 3; ++a)
      box_same = box_same && bx[s].L[a] == c->boxes[s].L[a] && bx[s].nc[a] == c->boxes[s].nc[a];
  if (!box_same) c->md_state = false;
  if (!same) {
    c->n = n;
    c->n_struct = n_struct;
    c->offsets_cache.assign(offsets, offsets + n_struct + 1);
    c->species_cache.assign(species, species + n);
    // internal order: by species (so that network tiles have one species), then
    // by structure, then spatially (Z-order of the neighbour cells of the
    // positions at this call) for cache locality of the neighbour gathers;
    // internal position p holds caller atom perm[p]
    std::vector<int> cnt(c->S + 1, 0);
    for (int64_t i = 0; i < n; ++i) cnt[species[i] + 1]++;
    for (int s = 0; s < c->S; ++s) cnt[s + 1] += cnt[s];
    for (int s = 0; s <= c->S; ++s) c->sp_off[s] = cnt[s];
    std::vector<uint64_t> zkey(n, 0);
    if (pos_dev && n > 0) {
      std::vector<double> ph((size_t)n * 3);
      // positions may still be in flight on the caller's stream (rare path: new species pattern)
      HIP_TRY(c, hipDeviceSynchronize());
      HIP_TRY(c, hipMemcpy(ph.data(), pos_dev, (size_t)n * 24, hipMemcpyDeviceToHost));
      for (int s = 0; s < n_struct; ++s) {
        const BoxInfo& b = bx[s];
        for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) {
          uint32_t cc[3];
          for (int a = 0; a < 3; ++a) {
            double x = ph[3 * i + a];
            double f = std::floor(x / b.L[a] * b.nc[a]);
            if (pb[a]) f -= b.nc[a] * std::floor(f / b.nc[a]);
            if (!(f >= 0)) f = 0;
            if (f > b.nc[a] - 1) f = b.nc[a] - 1;
            cc[a] = (uint32_t)f;
          }
          uint64_t z = 0;
          for (int bit = 0; bit < 10; ++bit)
            for (int a = 0; a < 3; ++a) z |= (uint64_t)((cc[a] >> bit) & 1u) << (3 * bit + a);
          zkey[i] = z;
        }
      }
    }
    std::vector<int> seg_orig(n);
    for (int s = 0; s < n_struct; ++s)
      for (int64_t i = offsets[s]; i < offsets[s + 1]; ++i) seg_orig[i] = s;
    c->perm.resize(n);
    for (int64_t i = 0; i < n; ++i) c->perm[i] = (int)i;
    std::stable_sort(c->perm.begin(), c->perm.end(), [&](int a, int b) {
      if (species[a] != species[b]) return species[a] < species[b];
      if (seg_orig[a] != seg_orig[b]) return seg_orig[a] < seg_orig[b];
      return zkey[a] < zkey[b];
    });
    std::vector<int> sp_int(n), seg_int(n);
    std::vector<double> wq(n);
    for (int64_t p = 0; p < n; ++p) {
      sp_int[p] = species[c->perm[p]];
      seg_int[p] = seg_orig[c->perm[p]];
      wq[p] = c->tw[sp_int[p]];
    }
    std::vector<int64_t> segcount(n_struct);
    for (int s = 0; s < n_struct; ++s) segcount[s] = offsets[s + 1] - offsets[s];
    const size_t nb = (size_t)std::max<int64_t>(n, 1);
    TRY(ensure(c, c->d_perm, nb * 4));
    TRY(ensure(c, c->d_species, nb * 4));
    TRY(ensure(c, c->d_wq, nb * 8));
    TRY(ensure(c, c->d_seg, nb * 4));
    TRY(ensure(c, c->d_segoff, (n_struct + 1) * 8));
    TRY(ensure(c, c->d_segcount, n_struct * 8));
    if (n > 0) {
      HIP_TRY(c, hipMemcpy(c->d_perm.p, c->perm.data(), n * 4, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(c->d_species.p, sp_int.data(), n * 4, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(c->d_wq.p, wq.data(), n * 8, hipMemcpyHostToDevice));
      HIP_TRY(c, hipMemcpy(c->d_seg.p, seg_int.data(), n * 4, hipMemcpyHostToDevice));
    }
    HIP_TRY(c, hipMemcpy(c->d_segoff.p, offsets, (n_struct + 1) * 8, hipMemcpyHostToDevice));
    HIP_TRY(c, hipMemcpy(c->d_segcount.p, segcount.data(), n_struct * 8, hipMemcpyHostToDevice));
    // XCD-aware order of the force pass's blocks (one atom each): the
    // hardware hands block k to XCD k mod 8, and XCD x is given the x-th
    // eighth of every species' atoms (a compact region in the Z-order), so
    // that the gradients the pass scatters to a region's neighbour rows meet
    // in that XCD's L2 and leave it as whole lines
    {
      std::vector<int> reg_n(8, 0);
      std::vector<int> xm;
      for (int pass = 0; pass < 2; ++pass) {
        std::vector<int> fill(8, 0);
        for (int s = 0; s < c->S; ++s) {
          const int a0 = c->sp_off[s], cs = c->sp_off[s + 1] - a0;
          for (int r = 0; r < cs; ++r) {
            const int x = (int)((int64_t)r * 8 / cs);
            if (pass == 0)
              ++reg_n[x];
            else
              xm[8 * (size_t)fill[x]++ + x] = a0 + r;
          }
        }
        if (pass == 0) xm.assign(8 * (size_t)std::max(1, *std::max_element(reg_n.begin(), reg_n.end())), -1);
      }
      c->n_grid = (int)xm.size();
      TRY(ensure(c, c->d_xmap, xm.size() * 4));
      HIP_TRY(c, hipMemcpy(c->d_xmap.p, xm.data(), xm.size() * 4, hipMemcpyHostToDevice));
    }
    c->nbr_valid = false;
    c->cap = 0;
  }
  for (int a = 0; a < 3; ++a) c->pbc[a] = pb[a];
  c->boxes = bx;
  c->n_cells = (int)cells;
  if (!box_same) {
    TRY(ensure(c, c->d_boxes, n_struct * sizeof(BoxInfo)));
    HIP_TRY(c, hipMemcpyAsync(c->d_boxes.p, c->boxes.data(), n_struct * sizeof(BoxInfo), hipMemcpyHostToDevice, st));
    HIP_TRY(c, hipStreamSynchronize(st));
  }
  // per-atom buffers
  const size_t nb = (size_t)std::max<int64_t>(n, 1);
  const size_t el = real_size(c);
  TRY(ensure(c, c->d_pos, nb * 24));
  TRY(ensure(c, c->d_pos_ref, nb * 24));
  if (!c->arena) TRY(ensure(c, c->d_vel, nb * 24));  // MD only
  TRY(ensure(c, c->d_F, nb * 24));
  TRY(ensure(c, c->d_Fself, nb * 24));
  TRY(ensure(c, c->d_E, nb * 8));
  TRY(ensure(c, c->d_Eorig, nb * 8));
  TRY(ensure(c, c->d_tmp, (nb + n_struct) * 8));
  TRY(ensure(c, c->d_G, nb * c->ldG * el));
  TRY(ensure(c, c->d_gG, nb * c->ldG * el));
  TRY(ensure(c, c->d_red, (size_t)(2 * reduce_blocks(n + n_struct) + 1) * 8));  // two rows of partials
  TRY(ensure(c, c->d_scal, 8 * 8));
  TRY(ensure(c, c->d_flags, 16 * 4));
  TRY(ensure(c, c->d_cell_count, (size_t)std::max(cells, (int64_t)1) * 4));
  TRY(ensure(c, c->d_cell_fill, (size_t)std::max(cells, (int64_t)1) * 4));
  TRY(ensure(c, c->d_cell_start, (size_t)(cells + 1) * 4));
  TRY(ensure(c, c->d_cell_atoms, nb * 4));
  TRY(ensure(c, c->d_atom_cell, nb * 4));
  TRY(ensure(c, c->d_nnb, nb * 4));
  TRY(ensure(c, c->d_nang, nb * 4));
  TRY(ensure(c, c->d_segs, nb * kSegWords * 2));
  TRY(ensure(c, c->d_build, 2 * 4));
  if (!box_same || !c->counters_clean) {
    // the binning kernel expects zero cell counters and block counter (each
    // build leaves them so for the next one)
    HIP_TRY(c, hipMemsetAsync(c->d_cell_count.p, 0, (size_t)std::max(cells, (int64_t)1) * 4, st));
    HIP_TRY(c, hipMemsetAsync(c->d_cell_fill.p, 0, (size_t)std::max(cells, (int64_t)1) * 4, st));
    HIP_TRY(c, hipMemsetAsync(c->d_build.p, 0, 2 * 4, st));
    // empty rows until a build writes them (a cell the per-cell row kernel
    // cannot hold leaves its atoms' rows unwritten until the retry)
    HIP_TRY(c, hipMemsetAsync(c->d_nnb.p, 0, nb * 4, st));
    HIP_TRY(c, hipMemsetAsync(c->d_nang.p, 0, nb * 4, st));
  }
  // cleared again by a successful end of the call
  c->counters_clean = false;
  // initial row capacities from the density of the densest structure
  if (c->cap == 0) {
    double est = 0.0, est_a = 0.0;
    const double ra = c->ra + c->skin;
    for (int s = 0; s < n_struct; ++s) {
      const double V = bx[s].L[0] * bx[s].L[1] * bx[s].L[2];
      const double rho = (double)(offsets[s + 1] - offsets[s]) / V;
      est = std::max(est, rho * 4.18879020478639 * c->rlist * c->rlist * c->rlist);
      est_a = std::max(est_a, rho * 4.18879020478639 * ra * ra * ra);
    }
    c->cap = pad_to((int)(est * 1.35) + 24, 16);
    double mean_a = 0.0;
    for (int s = 0; s < n_struct; ++s) {
      const double V = bx[s].L[0] * bx[s].L[1] * bx[s].L[2];
      const double rho = (double)(offsets[s + 1] - offsets[s]) / V;
      mean_a = std::max(mean_a, rho * 4.18879020478639 * c->ra * c->ra * c->ra);
    }
    c->ang_mean = (int)(mean_a + 0.5);
    c->cap_ang = std::min(c->cap, pad_to((int)(est_a * 1.3) + 8, 8));
    if (c->cap_user > 0) {
      c->cap = c->cap_user;
      c->cap_ang = c->cap_ang_user;
    }
    // rows by cell when the 27-cell neighbourhoods fit in LDS (grown, or
    // given up for the per-atom kernels, if a build finds otherwise)
    double per_cell = 0.0;
    for (int s = 0; s < n_struct; ++s) {
      const double ncell = (double)bx[s].nc[0] * bx[s].nc[1] * bx[s].nc[2];
      per_cell = std::max(per_cell, (double)(offsets[s + 1] - offsets[s]) / ncell);
    }
    c->tp = per_cell * 1.5 + 8 > kCellAtomsMax ? 0 : pad_to((int)(27.0 * per_cell * 1.2) + 64, 64);
    if (c->tp > 0 && cell_rows_lds(c->tp, c->cap) > 150 * 1024) c->tp = 0;
  }
  return AENET_OK;
}

aenet_status ensure_rows(aenet_ctx* c) {
  // row positions are stored in 16 bits (the forward pass's list for the force pass)
  if (c->cap > 65535) return fail(c, AENET_E_INVALID, "neighbour rows longer than 65535 entries");
  const size_t nb = (size_t)std::max<int64_t>(c->n, 1);
  TRY(ensure(c, c->d_nbr, nb * c->cap * 4));

  TRY(ensure(c, c->d_rev, nb * c->cap * 4));
  TRY(ensure(c, c->d_pg, nb * c->cap * 3 * real_size(c)));
  TRY(ensure(c, c->d_ridx, nb * c->cap * 2));
  TRY(ensure(c, c->d_nrad, nb * 4));
  return AENET_OK;
}

NbrParams nbr_params(aenet_ctx* c, int* cond) {
  NbrParams p{};
  p.n = (int)c->n;
  p.pos = c->d_pos.as<double>();
  p.pos_ref = c->d_pos_ref.as<double>();
  p.seg = c->d_seg.as<int>();
  p.boxes = c->d_boxes.as<BoxInfo>();
  p.n_struct = c->n_struct;
  for (int a = 0; a < 3; ++a) p.pbc[a] = c->pbc[a];
  p.n_cells = c->n_cells;
  p.tp = c->tp;
  p.r_list2 = c->rlist * c->rlist;
  p.r_ang2 = (c->ra + c->skin) * (c->ra + c->skin);
  p.cap = c->cap;
  p.cap_ang = c->cap_ang;
  p.cell_count = c->d_cell_count.as<int>();
  p.cell_start = c->d_cell_start.as<int>();
  p.cell_fill = c->d_cell_fill.as<int>();
  p.cell_atoms = c->d_cell_atoms.as<int>();
  p.atom_cell = c->d_atom_cell.as<int>();
  p.nbr = c->d_nbr.as<uint32_t>();
  p.segs = c->d_segs.as<uint16_t>();
  p.nnb = c->d_nnb.as<int>();
  p.nang = c->d_nang.as<int>();
  p.rev = c->d_rev.as<int>();
  p.flags = c->d_flags.as<int>();
  p.maxcnt = c->d_flags.as<int>() + 1;
  p.cond = cond;
  p.go = c->d_build.as<int>();
  p.ticket = c->d_build.as<int>() + 1;
  return p;
}

DescParams desc_params(aenet_ctx* c) {
  DescParams p{};
  p.n = (int)c->n;
  p.pos = c->d_pos.as<double>();
  p.species = c->d_species.as<int>();
  p.seg = c->d_seg.as<int>();
  p.boxes = c->d_boxes.as<BoxInfo>();
  p.nbr = c->d_nbr.as<uint32_t>();
  p.nnb = c->d_nnb.as<int>();
  p.nang = c->d_nang.as<int>();
  p.cap = c->cap;
  p.cap_ang = c->cap_ang;
  p.ang_hint = c->ang_mean;
  p.rr = c->rr;
  p.ra = c->ra;
  p.two_rr = 2.0 / c->rr;
  p.two_ra = 2.0 / c->ra;
  p.pi_rr = kPi / c->rr;
  p.pi_ra = kPi / c->ra;
  p.pi_2rr = 0.5 * kPi / c->rr;
  p.pi_2ra = 0.5 * kPi / c->ra;
  p.wq = c->d_wq.as<double>();
  for (int s = 0; s < kMaxSpecies; ++s) p.tw[s] = c->tw[s];
  p.n_species = c->S;
  p.weighted = c->S > 1;
  p.ldG = c->ldG;
  p.G = c->d_G.p;
  p.gG = c->d_gG.p;
  p.rev = c->d_rev.as<int>();
  p.segs = c->d_segs.as<uint16_t>();
  p.ridx = c->d_ridx.as<uint16_t>();
  p.nrad = c->d_nrad.as<int>();
  p.pg = c->d_pg.p;
  p.Fself = c->d_Fself.as<double>();
  p.vir = c->want_vir ? c->d_vir.as<double>() : nullptr;
  p.adj = c->d_adj.as<double>();
  p.U = c->d_U.p;
  p.flags = c->d_flags.as<int>();
  p.t1 = c->knr + 1;
  p.t2 = c->knr + c->kna + 2;
  p.shA = c->d_shA.p;
  p.xmap = c->d_xmap.as<int>();
  p.n_grid = c->n_grid;
  p.gang = c->d_gang.p;
  return p;
}

// The angular descriptor by its factorised form (angular.hip) where the
// expected angular shell is crowded (more than 48 neighbours within R_a: its
// cost grows with the shell size, the pair sum's with its square), or as the
// caller chose.
bool use_factorised(const aenet_ctx* c) {
  const bool ok = c->kna == 2 || c->kna == 3 || c->kna == 4 || c->kna == 6 || c->kna == 8;
  if (c->ang_method == AENET_ANGULAR_PAIRS || !ok) return false;
  if (c->ang_method == AENET_ANGULAR_FACTORISED) return true;
  return c->ang_mean > 48;
}

MlpParams mlp_params(aenet_ctx* c, bool want_grad) {
  MlpParams p = c->mlp;
  p.n_species = c->S;
  int t = 0;
  for (int s = 0; s <= c->S; ++s) p.sp_off[s] = c->sp_off[s];
  for (int s = 0; s < c->S; ++s) {
    p.tile_off[s] = t;
    t += (c->sp_off[s + 1] - c->sp_off[s] + 15) / 16;
  }
  p.tile_off[c->S] = t;
  p.G = c->d_G.p;
  p.gG = want_grad ? c->d_gG.p : nullptr;
  p.E = c->d_E.as<double>();
  return p;
}

int n_tiles(const MlpParams& p) { return p.tile_off[p.n_species]; }

// grow capacities from what the last build saw
aenet_status grow_caps(aenet_ctx* c, const int* hf) {
  // the per-cell row kernel: a neighbourhood or a cell larger than it holds
  if (c->tp > 0 && (hf[5] > c->tp || hf[6] > kCellAtomsMax)) {
    c->tp = hf[6] > kCellAtomsMax ? 0 : pad_to((int)(hf[5] * 1.15) + 64, 64);
    if (c->tp > 0 && cell_rows_lds(c->tp, c->cap) > 150 * 1024) c->tp = 0;
    c->stats.n_capacity_retries++;
    if (hf[1] <= c->cap && hf[2] <= c->cap_ang) return AENET_OK;
  }
  const int need = hf[1], need_a = hf[2];
  int cap = std::max(c->cap, pad_to((int)(need * 1.2) + 16, 16));
  int cap_a = std::max(c->cap_ang, pad_to((int)(need_a * 1.15) + 8, 8));
  if (cap_a > cap) cap = pad_to(cap_a, 16);
  if (cap_a > 700) return fail(c, AENET_E_INVALID, "angular neighbour shell too crowded (" + std::to_string(need_a) + " entries)");
  c->cap = cap;
  c->cap_ang = cap_a;
  if (c->tp > 0 && cell_rows_lds(c->tp, c->cap) > 150 * 1024) c->tp = 0;
  c->stats.n_capacity_retries++;
  return ensure_rows(c);
}

// the first `count` status words of d_flags, through the context's pinned
// buffer (a copy into pageable memory goes through the runtime's staging path)
aenet_status read_flags(aenet_ctx* c, hipStream_t s, int* hf, int count = 8) {
  HIP_TRY(c, hipMemcpyAsync(c->h_flags, c->d_flags.p, count * sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  std::memcpy(hf, c->h_flags, count * sizeof(int));
  return AENET_OK;
}

aenet_status flag_status(aenet_ctx* c, int f) {
  if (f & kFlagNonFinite) return fail(c, AENET_E_NONFINITE, "non-finite position or velocity");
  if (f & kFlagOverlap) return fail(c, AENET_E_OVERLAP, "two atoms (or an atom and an image) coincide");
  // a row truncated by a capacity overflow also leaves entries without a
  // reverse; the caller grows the rows and builds again
  if ((f & kFlagReverse) && !(f & kFlagOverflow))
    return fail(c, AENET_E_DEVICE, "internal error: neighbour list not symmetric");
  return AENET_OK;
}

// ------------------------------------------------------------------ kernel timing
void prof_begin(aenet_ctx* c, hipStream_t s, int cls) {
  if (!c->profiling) return;
  if (c->ev_used + 2 > c->ev_pool.size()) {
    for (int k = 0; k < 64; ++k) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        c->profiling = false;
        return;
      }
      c->ev_pool.push_back(e);
    }
  }
  (void)hipEventRecord(c->ev_pool[c->ev_used], s);
  c->ev_class.push_back(cls);
}

void prof_end(aenet_ctx* c, hipStream_t s) {
  // a begin is pending iff one more class than completed pairs was recorded
  if (!c->profiling || c->ev_class.size() != c->ev_used / 2 + 1) return;
  (void)hipEventRecord(c->ev_pool[c->ev_used + 1], s);
  c->ev_used += 2;
}

void prof_collect(aenet_ctx* c) {
  const size_t pairs = c->ev_used / 2;
  for (size_t k = 0; k < pairs; ++k) {
    float ms = 0.f;
    if (hipEventSynchronize(c->ev_pool[2 * k + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, c->ev_pool[2 * k], c->ev_pool[2 * k + 1]) == hipSuccess) {
      c->prof_ms[c->ev_class[k]] += ms;
      c->prof_n[c->ev_class[k]] += 1;
    }
    (void)hipGetLastError();
  }
  c->ev_used = 0;
  c->ev_class.clear();
}

// the neighbour build as one timed unit
void build_neighbors_timed(aenet_ctx* c, const NbrParams& p, hipStream_t s) {
  prof_begin(c, s, AENET_K_NEIGHBOR);
  launch_build_neighbors(p, s);
  prof_end(c, s);
}

// descriptors -> networks -> forces (internal order).  vel != NULL applies the closing half kick.
// keep_G: the descriptors are needed in HBM afterwards (training)
aenet_status compute(aenet_ctx* c, hipStream_t s, bool forces, double* vel, double half_dt,
                     const DriftArgs* next = nullptr, bool keep_G = false) {
  if (c->n == 0) return AENET_OK;
  const bool sh = use_factorised(c);
  if (sh) {
    const size_t el = real_size(c);
    TRY(ensure(c, c->d_shA, (size_t)c->n * 2 * ang_sh_terms(c->kna) * el));
    if (forces) TRY(ensure(c, c->d_gang, (size_t)c->n * c->cap_ang * 3 * el));
  }
  DescParams dp = desc_params(c);
  MlpParams mp = mlp_params(c, forces);
  if (sh) {
    prof_begin(c, s, AENET_K_DESC_FWD);
    launch_desc_fwd(desc_prec(c), c->knr, c->kna, dp, s, false);
    launch_ang_sh(true, desc_prec(c), c->kna, dp, s);
    prof_end(c, s);
    prof_begin(c, s, AENET_K_NETWORK);
    launch_mlp(c->prec, mp, n_tiles(mp), s);
    prof_end(c, s);
  } else if (c->fused && fwd_mlp_fits(c->prec, dp, mp)) {
    DescParams dq = dp;
    if (!keep_G) dq.G = nullptr;
    prof_begin(c, s, AENET_K_FWD_NETWORK);
    launch_fwd_mlp(c->prec, c->knr, c->kna, dq, mp, n_tiles(mp), s);
    prof_end(c, s);
  } else {
    prof_begin(c, s, AENET_K_DESC_FWD);
    launch_desc_fwd(desc_prec(c), c->knr, c->kna, dp, s);
    prof_end(c, s);
    prof_begin(c, s, AENET_K_NETWORK);
    launch_mlp(c->prec, mp, n_tiles(mp), s);
    prof_end(c, s);
  }
  if (forces) {
    prof_begin(c, s, AENET_K_DESC_BWD);
    if (sh) launch_ang_sh(false, desc_prec(c), c->kna, dp, s);
    launch_desc_bwd(desc_prec(c), c->knr, c->kna, dp, s, sh);
    prof_end(c, s);
    prof_begin(c, s, AENET_K_FORCE_GATHER);
    launch_force_gather(desc_prec(c), (int)c->n, c->cap, c->d_nrad.as<int>(), c->d_ridx.as<uint16_t>(), c->d_pg.p,
                        c->d_Fself.as<double>(), c->d_F.as<double>(), vel,
                        c->d_invmk.as<double>(), c->d_species.as<int>(), half_dt,
                        next ? *next : DriftArgs{}, s);
    prof_end(c, s);
  }
  HIP_TRY(c, hipGetLastError());
  return AENET_OK;
}

// forced build with capacity retries (positions already in d_pos)
aenet_status build_checked(aenet_ctx* c, hipStream_t s) {
  TRY(ensure_rows(c));
  for (int attempt = 0; attempt < 4; ++attempt) {
    // flags[0] keeps what the input gather found (non-finite input) on the
    // first attempt; a retry follows a clean flag word
    if (attempt == 0)
      HIP_TRY(c, hipMemsetAsync(c->d_flags.as<int>() + 1, 0, 7 * sizeof(int), s));
    else
      HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 8 * sizeof(int), s));
    build_neighbors_timed(c, nbr_params(c, nullptr), s);
    HIP_TRY(c, hipGetLastError());
    int hf[8];
    TRY(read_flags(c, s, hf));
    c->stats.n_rebuilds++;
    c->stats.max_neighbors = hf[1];
    c->stats.max_angular = hf[2];
    TRY(flag_status(c, hf[0]));
    if (!(hf[0] & kFlagOverflow)) {
      c->nbr_valid = true;
      c->stats.row_capacity = c->cap;
      c->stats.ang_capacity = c->cap_ang;
      return AENET_OK;
    }
    TRY(grow_caps(c, hf));
  }
  return fail(c, AENET_E_DEVICE, "neighbour capacity retries exhausted");
}

hipStream_t pick_stream(aenet_ctx* c, void* s) { return s ? (hipStream_t)s : c->stream; }

__global__ void k_take(int n, const int* idx, const double* src, double* dst) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = src[idx[k]];
}

void launch_take(int n, const int* idx, const double* src, double* dst, hipStream_t s) {
  if (n > 0) hipLaunchKernelGGL(k_take, dim3((n + 255) / 256), dim3(256), 0, s, n, idx, src, dst);
}

// parameters (device, API layout) -> the packed network operands: element k
// of netbuf holds parameter map[k] (-1: zero padding, -2: left as is), and
// blast[s] the output bias of species s; the same values the host packing
// writes (a float context rounds to nearest as the host conversion does)
template <class T>
__global__ void k_pack_params(int64_t n, const int* map, const double* P, T* out, int S,
                              const int* blast_src, double* blast) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < S) blast[k] = P[blast_src[k]];
  if (k >= n) return;
  const int src = map[k];
  if (src == -2) return;
  out[k] = src >= 0 ? (T)P[src] : T(0);
}

// flags[0] |= 1 if any of x[0..n) is not finite
__global__ void k_any_nonfinite(int64_t n, const double* x, int* flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n && !isfinite(x[k])) atomicOr(flag, 1);
}

// one Adam step (Kingma & Ba 2015) with bias corrections c1 = 1 - beta1^t,
// c2 = 1 - beta2^t: m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
// p -= lr (m / c1) / (sqrt(v / c2) + eps)
__global__ void k_adam(int64_t n, double* p, const double* g, double* m, double* v, double lr, double b1,
                       double b2, double eps, double c1, double c2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const double gk = g[k];
  const double mk = b1 * m[k] + (1.0 - b1) * gk;
  const double vk = b2 * v[k] + (1.0 - b2) * gk * gk;
  m[k] = mk;
  v[k] = vk;
  p[k] -= lr * (mk / c1) / (sqrt(vk / c2) + eps);
}

thread_local std::string g_setup_error;

// ------------------------------------------------------------------ no-allocation workspace
// The device memory of aenet_energy_forces_noalloc: one array per GPU,
// reserved when the library's code object is loaded onto that GPU and held
// until the process ends.  Host code never uses the symbol's name as an
// address: each device's address is looked up once (with that device
// current) and kept in g_scratch_addr.
constexpr size_t kScratchBytes = (size_t)AENET_NOALLOC_WORKSPACE_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {nullptr};

// address of this device's workspace (the device must be current); looked up
// on the first call for the device, NULL if the lookup fails
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_addr[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_addr[device] = ptr;
  }
  return g_scratch_addr[device];
}

aenet_status check_ctx(aenet_ctx* c) {
  if (!c) return AENET_E_INVALID;
  c->err.clear();
  HIP_TRY(c, hipSetDevice(c->device));
  return AENET_OK;
}

// energies/forces of a batch whose positions are on the device in caller order
// virial (device, 9 doubles, or NULL): the virial of the whole batch
aenet_status ef_core(aenet_ctx* c, int n_struct, const int64_t* offsets, const double* pos,
                     const int32_t* species, const double* boxes, const uint8_t* pbc,
                     double* e_struct, double* e_total, double* e_atom, double* forces,
                     hipStream_t s, double* virial = nullptr) {
  c->md_state = false;
  TRY(prepare(c, n_struct, offsets, species, boxes, pbc, pos, s));
  const int n = (int)c->n;
  if (n == 0) {
    if (e_total) HIP_TRY(c, hipMemsetAsync(e_total, 0, 8, s));
    if (e_struct) HIP_TRY(c, hipMemsetAsync(e_struct, 0, 8 * (size_t)n_struct, s));
    if (virial) HIP_TRY(c, hipMemsetAsync(virial, 0, 9 * 8, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    return AENET_OK;
  }
  HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 8 * sizeof(int), s));
  launch_gather_in(n, c->d_perm.as<int>(), pos, c->d_pos.as<double>(), c->d_flags.as<int>(), s);
  TRY(build_checked(c, s));
  if (virial) {
    TRY(ensure(c, c->d_vir, (size_t)9 * n * 8));
    TRY(ensure(c, c->d_red, (size_t)(9 * reduce_blocks(n) + 1) * 8));
  }
  c->want_vir = virial != nullptr;
  const aenet_status st = compute(c, s, forces != nullptr || virial != nullptr, nullptr, 0.0);
  c->want_vir = false;
  TRY(st);
  if (virial) launch_sum_rows(9, n, c->d_vir.as<double>(), c->d_red.as<double>(), virial, s);
  launch_scatter_out(n, c->d_perm.as<int>(), c->d_F.as<double>(), forces, c->d_E.as<double>(),
                     c->d_Eorig.as<double>(), s);
  if (e_atom) HIP_TRY(c, hipMemcpyAsync(e_atom, c->d_Eorig.p, (size_t)n * 8, hipMemcpyDeviceToDevice, s));
  if (e_total) launch_sum(n, c->d_Eorig.as<double>(), c->d_red.as<double>(), e_total, s);
  if (e_struct)
    launch_segment_sum(n_struct, c->d_segoff.as<int64_t>(), c->d_Eorig.as<double>(), e_struct, s);
  HIP_TRY(c, hipGetLastError());
  int hf[8];
  TRY(read_flags(c, s, hf));
  TRY(flag_status(c, hf[0]));
  c->counters_clean = true;
  return AENET_OK;
}

}  // namespace

// ====================================================================== C ABI

extern "C" {

aenet_status aenet_setup(const aenet_model* m, aenet_ctx** out) {
  if (!out) return AENET_E_INVALID;
  *out = nullptr;
  if (!m) return AENET_E_INVALID;
  aenet_ctx* c = new (std::nothrow) aenet_ctx();
  if (!c) return AENET_E_OOM;
  g_setup_error.clear();
  auto bad = [&](const std::string& msg) {
    g_setup_error = msg;
    delete c;
    return AENET_E_INVALID;
  };
  if (m->n_species < 1 || m->n_species > kMaxSpecies) return bad("n_species must be 1..8");
  if (m->radial_order < 0 || m->angular_order < 0) return bad("orders must be >= 0");
  if (!(m->radial_cutoff > 0) || !(m->angular_cutoff > 0)) return bad("cutoffs must be positive");
  if (!(m->skin >= 0) || !std::isfinite(m->skin)) return bad("skin must be >= 0");
  if (m->precision < 0 || m->precision > 2) return bad("unknown precision");
  if (!m->nets) return bad("nets is NULL");
  c->S = m->n_species;
  c->nr = m->radial_order;
  c->na = m->angular_order;
  c->rr = m->radial_cutoff;
  c->ra = m->angular_cutoff;
  c->skin = m->skin;
  c->rlist = std::max(c->rr, c->ra) + c->skin;
  c->prec = m->precision;
  c->fused = true;
  c->device = m->device;
  const int typed = c->nr + 1 + c->na + 1;
  c->D = c->S > 1 ? 2 * typed : typed;
  for (int s = 0; s < c->S; ++s) {
    if (c->S > 1 && !m->type_weight) return bad("type_weight is NULL");
    c->tw[s] = c->S > 1 ? m->type_weight[s] : 0.0;  // one species: no weighted half
    if (m->mass_amu) {
      if (!(m->mass_amu[s] > 0)) return bad("masses must be positive");
      c->mass[s] = m->mass_amu[s];
    }
  }
  c->have_mass = m->mass_amu != nullptr;
  // the compiled order pair that holds the model's descriptor: the one with
  // the smallest dimension (then the lowest angular order) among those that
  // reach both orders and whose descriptor the networks' input layer takes
  // (at most kMaxWidth components)
  {
    int pairs[2 * 64];
    const int np = std::min(desc_supported_list(pairs, 64), 64);
    int best = -1;
    for (int k = 0; k < np; ++k) {
      const int a = pairs[2 * k], b = pairs[2 * k + 1];
      if (a < c->nr || b < c->na || (c->S > 1 ? 2 : 1) * (a + b + 2) > kMaxWidth) continue;
      if (best < 0 || a + b < pairs[2 * best] + pairs[2 * best + 1] ||
          (a + b == pairs[2 * best] + pairs[2 * best + 1] && b < pairs[2 * best + 1]))
        best = k;
    }
    if (best < 0) {
      std::string list;
      for (int k = 0; k < np; ++k)
        list += (k ? ", " : "") + std::to_string(pairs[2 * k]) + "/" + std::to_string(pairs[2 * k + 1]);
      return bad("descriptor orders " + std::to_string(c->nr) + "/" + std::to_string(c->na) +
                 " exceed every compiled pair (" + list + ") whose descriptor dimension is at most " +
                 std::to_string(kMaxWidth) + " with " + std::to_string(c->S) + " species");
    }
    c->knr = pairs[2 * best];
    c->kna = pairs[2 * best + 1];
  }
  const int ktyped = c->knr + 1 + c->kna + 1;
  c->kD = c->S > 1 ? 2 * ktyped : ktyped;
  c->colmap.resize(c->D);
  for (int k = 0; k < c->D; ++k) {
    const int half = k / typed, r = k % typed;  // channel (typed, weighted) and place in it
    c->colmap[k] = half * ktyped + (r <= c->nr ? r : c->knr + 1 + (r - c->nr - 1));
  }
  // networks: every species has the same number of layers and activations;
  // the hidden widths may differ (the kernels use the largest of each layer)
  const aenet_net& n0 = m->nets[0];
  if (n0.n_layers < 1 || n0.n_layers > kMaxLayers) return bad("n_layers must be 1..4");
  c->L = n0.n_layers;
  for (int l = 0; l < c->L; ++l) {
    c->act[l] = n0.act[l];
    if (c->act[l] != AENET_ACT_LINEAR && c->act[l] != AENET_ACT_TANH) return bad("unknown activation");
  }
  if (c->act[c->L - 1] != AENET_ACT_LINEAR) return bad("the output layer must be linear");
  c->poff.assign(c->S + 1, 0);
  for (int s = 0; s < c->S; ++s) {
    const aenet_net& nt = m->nets[s];
    if (nt.n_layers != c->L) return bad("all species need the same number of layers");
    if (!nt.widths || !nt.act) return bad("widths or act is NULL");
    for (int l = 0; l < c->L; ++l)
      if (nt.act[l] != c->act[l]) return bad("all species need the same activations");
    for (int l = 0; l <= c->L; ++l)
      if (nt.widths[l] < 1 || nt.widths[l] > kMaxWidth) return bad("widths must be 1..64");
    if (nt.widths[0] != c->D) return bad("widths[0] must equal the descriptor dimension " + std::to_string(c->D));
    if (nt.widths[c->L] != 1) return bad("the last width must be 1");
    int64_t np = 0;
    for (int l = 1; l <= c->L; ++l) np += (int64_t)nt.widths[l] * (nt.widths[l - 1] + 1);
    c->poff[s + 1] = c->poff[s] + np;
  }
  c->w[0] = c->kD;
  c->w[c->L] = 1;
  for (int l = 1; l < c->L; ++l) {
    c->w[l] = 0;
    for (int s = 0; s < c->S; ++s) c->w[l] = std::max(c->w[l], m->nets[s].widths[l]);
  }
  for (int l = 0; l <= c->L; ++l) c->wp[l] = pad_to(c->w[l], kPad);
  c->ldG = c->wp[0];
  c->nps_int = 0;
  for (int l = 1; l <= c->L; ++l) c->nps_int += (int64_t)c->w[l] * (c->w[l - 1] + 1);
  c->params.assign((size_t)c->poff[c->S], 0.0);
  c->imap.assign((size_t)c->S * c->nps_int, -1);
  // input normalisation on the kernel columns: the model's columns take its
  // shift and scale, the others scale 0 (their input is exactly zero)
  c->shift.assign((size_t)c->S * c->kD, 0.0);
  c->scale.assign((size_t)c->S * c->kD, 0.0);
  for (int s = 0; s < c->S; ++s) {
    const aenet_net& nt = m->nets[s];
    if (!nt.W || !nt.b) return bad("missing weights");
    int64_t pa = c->poff[s];         // API index
    size_t ko = (size_t)s * c->nps_int;  // kernel-shape index of the layer
    for (int l = 1; l <= c->L; ++l) {
      const int in = nt.widths[l - 1], out = nt.widths[l], kin = c->w[l - 1];
      if (!nt.W[l - 1] || !nt.b[l - 1]) return bad("missing weights");
      for (int q = 0; q < out; ++q)
        for (int k = 0; k < in; ++k) {
          c->params[pa] = nt.W[l - 1][(size_t)q * in + k];
          c->imap[ko + (size_t)q * kin + (l == 1 ? c->colmap[k] : k)] = (int)pa;
          ++pa;
        }
      ko += (size_t)c->w[l] * kin;
      for (int q = 0; q < out; ++q) {
        c->params[pa] = nt.b[l - 1][q];
        c->imap[ko + q] = (int)pa;
        ++pa;
      }
      ko += c->w[l];
    }
    for (int k = 0; k < c->D; ++k) {
      c->shift[(size_t)s * c->kD + c->colmap[k]] = nt.in_shift ? nt.in_shift[k] : 0.0;
      c->scale[(size_t)s * c->kD + c->colmap[k]] = nt.in_scale ? nt.in_scale[k] : 1.0;
    }
    c->e_off[s] = nt.e_offset;
    for (int64_t k = c->poff[s]; k < c->poff[s + 1]; ++k)
      if (!std::isfinite(c->params[k])) return bad("non-finite network parameter");
  }
  // MLP shape
  c->mlp.n_layers = c->L;
  for (int l = 0; l <= c->L; ++l) {
    c->mlp.w[l] = c->w[l];
    c->mlp.wp[l] = c->wp[l];
  }
  for (int l = 0; l < c->L; ++l) c->mlp.act[l] = c->act[l];
  c->mlp.ldG = c->ldG;
  // padded training layout
  c->npad_species = 0;
  for (int l = 1; l <= c->L; ++l) {
    const int out = l == c->L ? 1 : c->wp[l];
    c->npad_species += out * c->wp[l - 1] + out;
  }
  if (hipSetDevice(c->device) != hipSuccess) {
    (void)hipGetLastError();
    g_setup_error = "hipSetDevice failed";
    delete c;
    return AENET_E_DEVICE;
  }
  if (hipStreamCreate(&c->stream) != hipSuccess) {
    (void)hipGetLastError();
    g_setup_error = "hipStreamCreate failed";
    delete c;
    return AENET_E_DEVICE;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&c->h_flags), 16 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    c->h_flags = nullptr;
    g_setup_error = "pinned host memory for the status words could not be allocated";
    aenet_destroy(c);
    return AENET_E_DEVICE;
  }
  // the device's no-allocation workspace (looked up once per device)
  if (!scratch_address(c->device)) {
    g_setup_error = "hipGetSymbolAddress of the no-allocation workspace failed";
    aenet_destroy(c);
    return AENET_E_DEVICE;
  }
  if (pack_networks(c) != AENET_OK) {
    g_setup_error = c->err;
    aenet_destroy(c);
    return AENET_E_DEVICE;
  }
  // masses (kappa / m per species) and the API -> padded parameter map
  double invmk[kMaxSpecies] = {0};
  for (int s = 0; s < c->S; ++s) invmk[s] = c->mass[s] > 0 ? kKappa / c->mass[s] : 0.0;
  std::vector<int> pidx(c->params.size());
  for (int s = 0; s < c->S; ++s) {
    size_t ko = (size_t)s * c->nps_int, go = 0;
    auto put = [&](int pad_index) {
      const int a = c->imap[ko++];
      if (a >= 0) pidx[a] = (int)((size_t)s * c->npad_species + pad_index);
    };
    for (int l = 1; l <= c->L; ++l) {
      const int in = c->w[l - 1], out = c->w[l];
      const int outp = l == c->L ? 1 : c->wp[l], inp = c->wp[l - 1];
      for (int q = 0; q < out; ++q)
        for (int k = 0; k < in; ++k) put((int)(go + (size_t)q * inp + k));
      for (int q = 0; q < out; ++q) put((int)(go + (size_t)outp * inp + q));
      go += (size_t)outp * inp + outp;
    }
  }
  if (ensure(c, c->d_mass, kMaxSpecies * 8) || ensure(c, c->d_invmk, kMaxSpecies * 8) ||
      ensure(c, c->d_pidx, pidx.size() * 4) ||
      hipMemcpy(c->d_mass.p, c->mass, kMaxSpecies * 8, hipMemcpyHostToDevice) ||
      hipMemcpy(c->d_invmk.p, invmk, kMaxSpecies * 8, hipMemcpyHostToDevice) ||
      hipMemcpy(c->d_pidx.p, pidx.data(), pidx.size() * 4, hipMemcpyHostToDevice)) {
    g_setup_error = "device buffers for the model could not be set up";
    aenet_destroy(c);
    return AENET_E_DEVICE;
  }
  c->stats.rebuild_every = c->rebuild_every;
  c->stats.deterministic = 1;
  *out = c;
  return AENET_OK;
}

void aenet_destroy(aenet_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipStreamDestroy(c->stream);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->h_flags) (void)hipHostFree(c->h_flags);
  delete c;
}

const char* aenet_last_error(const aenet_ctx* c) { return c ? c->err.c_str() : g_setup_error.c_str(); }

int aenet_descriptor_dim(const aenet_ctx* c) { return c ? c->D : -1; }

int64_t aenet_n_params(const aenet_ctx* c) { return c ? (int64_t)c->params.size() : -1; }

aenet_status aenet_get_params(aenet_ctx* c, double* params) {
  if (!c || !params) return AENET_E_INVALID;
  if (c->params_host_stale) {
    TRY(check_ctx(c));
    HIP_TRY(c, hipMemcpy(c->params.data(), c->d_params.p, c->params.size() * 8, hipMemcpyDeviceToHost));
    c->params_host_stale = false;
  }
  std::memcpy(params, c->params.data(), c->params.size() * 8);
  return AENET_OK;
}

aenet_status aenet_set_params_dev(aenet_ctx* c, const double* params, void* stream) {
  TRY(check_ctx(c));
  if (!params) return fail(c, AENET_E_INVALID, "params is NULL");
  if (c->prec == AENET_BF16 || c->n_pack == 0)
    return fail(c, AENET_E_INVALID, "parameters from device memory need an FP64 or FP32 context");
  hipStream_t s = pick_stream(c, stream);
  const int64_t np = (int64_t)c->params.size();
  TRY(ensure(c, c->d_flags, 16 * 4));
  int* flag = c->d_flags.as<int>() + 15;
  HIP_TRY(c, hipMemsetAsync(flag, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_any_nonfinite, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, np, params, flag);
  int bad = 0;
  HIP_TRY(c, hipMemcpyAsync(&bad, flag, sizeof(int), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (bad) return fail(c, AENET_E_NONFINITE, "non-finite parameter");
  c->md_state = false;  // the forces kept from the last MD call belong to the old parameters
  HIP_TRY(c, hipMemcpyAsync(c->d_params.p, params, np * 8, hipMemcpyDeviceToDevice, s));
  const int64_t n = std::max<int64_t>(c->n_pack, c->S);
  const dim3 grid((unsigned)((n + 255) / 256));
  if (c->prec == AENET_FP64)
    hipLaunchKernelGGL(k_pack_params<double>, grid, dim3(256), 0, s, c->n_pack, c->d_packmap.as<int>(),
                       c->d_params.as<double>(), c->netbuf.as<double>(), c->S, c->d_blastsrc.as<int>(),
                       c->d_blast.as<double>());
  else
    hipLaunchKernelGGL(k_pack_params<float>, grid, dim3(256), 0, s, c->n_pack, c->d_packmap.as<int>(),
                       c->d_params.as<double>(), c->netbuf.as<float>(), c->S, c->d_blastsrc.as<int>(),
                       c->d_blast.as<double>());
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(s));
  c->params_host_stale = true;
  return AENET_OK;
}

aenet_status aenet_adam_step_dev(int64_t n, double* params, const double* grad, double* m, double* v,
                                 double lr, double beta1, double beta2, double eps, int64_t step,
                                 void* stream) {
  if (n < 0 || (n > 0 && (!params || !grad || !m || !v)) || step < 1 || !(lr >= 0) ||
      !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return AENET_E_INVALID;
  if (n == 0) return AENET_OK;
  hipStream_t s = (hipStream_t)stream;
  const double c1 = 1.0 - std::pow(beta1, (double)step), c2 = 1.0 - std::pow(beta2, (double)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, params, grad, m, v, lr,
                     beta1, beta2, eps, c1, c2);
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess) {
    (void)hipGetLastError();
    return AENET_E_DEVICE;
  }
  return AENET_OK;
}

aenet_status aenet_rms_diff_dev(aenet_ctx* c, int64_t n, const double* a, const double* b, double* out,
                                void* stream) {
  TRY(check_ctx(c));
  if (n < 0 || !out || (n > 0 && (!a || !b))) return fail(c, AENET_E_INVALID, "bad arguments");
  hipStream_t s = pick_stream(c, stream);
  TRY(ensure(c, c->d_judge, (size_t)(reduce_blocks(n) + 1) * 8));
  launch_rms_diff(n, a, b, c->d_judge.as<double>(), out, s);
  HIP_TRY(c, hipGetLastError());
  HIP_TRY(c, hipStreamSynchronize(s));
  return AENET_OK;
}

aenet_status aenet_set_loss_form(aenet_ctx* c, int form) {
  if (!c || (form != AENET_LOSS_MEAN_PER_ATOM && form != AENET_LOSS_EQ7)) return AENET_E_INVALID;
  c->loss_form = form;
  return AENET_OK;
}

aenet_status aenet_set_params(aenet_ctx* c, const double* params) {
  TRY(check_ctx(c));
  if (!params) return fail(c, AENET_E_INVALID, "params is NULL");
  for (size_t k = 0; k < c->params.size(); ++k)
    if (!std::isfinite(params[k])) return fail(c, AENET_E_NONFINITE, "non-finite parameter");
  std::memcpy(c->params.data(), params, c->params.size() * 8);
  c->params_host_stale = false;
  c->md_state = false;  // the forces kept from the last MD call belong to the old parameters
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  return pack_networks(c);
}

int aenet_supported_orders(int* orders, int max_pairs) { return desc_supported_list(orders, max_pairs); }

aenet_status aenet_energy_forces_dev(aenet_ctx* c, int64_t n, const double* pos,
                                     const int32_t* species, const double box[3],
                                     const uint8_t pbc[3], double* e_total, double* e_atom,
                                     double* forces, void* stream) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && !pos)) return fail(c, AENET_E_INVALID, "bad arguments");
  const int64_t off[2] = {0, n};
  return ef_core(c, 1, off, pos, species, box, pbc, nullptr, e_total, e_atom, forces, pick_stream(c, stream));
}

aenet_status aenet_energy_forces_virial_dev(aenet_ctx* c, int64_t n, const double* pos,
                                            const int32_t* species, const double box[3],
                                            const uint8_t pbc[3], double* e_total, double* forces,
                                            double* virial, void* stream) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && !pos) || !virial) return fail(c, AENET_E_INVALID, "bad arguments");
  const int64_t off[2] = {0, n};
  return ef_core(c, 1, off, pos, species, box, pbc, nullptr, e_total, nullptr, forces, pick_stream(c, stream),
                 virial);
}

aenet_status aenet_energy_forces_batch_dev(aenet_ctx* c, int n_struct, const int64_t* offsets,
                                           const double* pos, const int32_t* species,
                                           const double* boxes, const uint8_t pbc[3],
                                           double* e_struct, double* e_atom, double* forces,
                                           void* stream) {
  TRY(check_ctx(c));
  if (n_struct < 1 || !offsets || !boxes) return fail(c, AENET_E_INVALID, "bad arguments");
  return ef_core(c, n_struct, offsets, pos, species, boxes, pbc, e_struct, nullptr, e_atom, forces,
                 pick_stream(c, stream));
}

aenet_status aenet_energy_forces_noalloc(aenet_ctx* c, int64_t n, const double* pos,
                                         const int32_t* species, const double box[3],
                                         const uint8_t pbc[3], double* e_total, double* e_atom,
                                         double* forces, void* stream) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && !pos)) return fail(c, AENET_E_INVALID, "bad arguments");
  void* ws = scratch_address(c->device);
  if (!ws) return fail(c, AENET_E_DEVICE, "no-allocation workspace unavailable on this device");
  // Every per-call device buffer of the context is swapped for a slice of
  // the workspace for the duration of the call and restored afterwards; the
  // context's own buffers (and the model's, allocated at set-up) are not
  // touched.  The workspace belongs to every context on this device, so
  // nothing the context remembers about its buffers' contents (atom order,
  // boxes, neighbour rows, cleared counters, MD state) carries into or out of
  // this call: set-up runs in full and the context forgets afterwards.
  DevMem* bufs[] = {&c->d_perm, &c->d_species, &c->d_wq, &c->d_seg, &c->d_segoff, &c->d_segcount,
                    &c->d_boxes, &c->d_pos, &c->d_pos_ref, &c->d_vel, &c->d_F, &c->d_Fself, &c->d_E,
                    &c->d_Eorig, &c->d_G, &c->d_gG, &c->d_U, &c->d_adj, &c->d_eps, &c->d_tmp, &c->d_red,
                    &c->d_scal, &c->d_flags, &c->d_cell_count, &c->d_cell_start, &c->d_cell_fill,
                    &c->d_cell_atoms, &c->d_atom_cell, &c->d_nbr, &c->d_segs, &c->d_nnb, &c->d_nang,
                    &c->d_rev, &c->d_ridx, &c->d_nrad, &c->d_vir, &c->d_build, &c->d_shA, &c->d_gang,
                    &c->d_pg, &c->d_xmap};
  constexpr int nbufs = (int)(sizeof(bufs) / sizeof(bufs[0]));
  struct Saved {
    void* p;
    size_t bytes;
  } saved[nbufs];
  auto forget = [&]() {
    c->n = -1;  // set-up treats the next call's species pattern as new
    c->species_cache.clear();
    c->offsets_cache.clear();
    c->boxes.clear();
    c->cap = 0;
    c->nbr_valid = false;
    c->md_state = false;
    c->counters_clean = false;
  };
  for (int k = 0; k < nbufs; ++k) {
    saved[k] = {bufs[k]->p, bufs[k]->bytes};
    bufs[k]->p = nullptr;
    bufs[k]->bytes = 0;
  }
  Arena arena;
  arena.base = static_cast<unsigned char*>(ws);
  arena.size = kScratchBytes;
  const bool prof = c->profiling;
  c->profiling = false;  // no event creation inside this call
  c->arena = &arena;
  forget();
  const int64_t off[2] = {0, n};
  const aenet_status st =
      ef_core(c, 1, off, pos, species, box, pbc, nullptr, e_total, e_atom, forces, pick_stream(c, stream));
  c->arena = nullptr;
  c->profiling = prof;
  forget();
  for (int k = 0; k < nbufs; ++k) {
    bufs[k]->p = saved[k].p;
    bufs[k]->bytes = saved[k].bytes;
  }
  return st;
}

namespace {
aenet_status ef_host(aenet_ctx* c, int64_t n, const double* pos, const int32_t* species,
                     const double box[3], const uint8_t pbc[3], double* e_total, double* e_atom,
                     double* forces, double* virial) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && !pos)) return fail(c, AENET_E_INVALID, "bad arguments");
  for (int64_t k = 0; k < 3 * n; ++k)
    if (!std::isfinite(pos[k])) return fail(c, AENET_E_NONFINITE, "non-finite position");
  const size_t nb = (size_t)std::max<int64_t>(n, 1);
  TRY(ensure(c, c->h_pos, nb * 24));
  TRY(ensure(c, c->h_F, nb * 24));
  TRY(ensure(c, c->h_E, (nb + 1 + 9) * 8));
  hipStream_t s = c->stream;
  if (n > 0) HIP_TRY(c, hipMemcpyAsync(c->h_pos.p, pos, n * 24, hipMemcpyHostToDevice, s));
  const int64_t off[2] = {0, n};
  double* dE = c->h_E.as<double>();
  TRY(ef_core(c, 1, off, c->h_pos.as<double>(), species, box, pbc, nullptr, dE + nb,
              e_atom ? dE : nullptr, forces ? c->h_F.as<double>() : nullptr, s,
              virial ? dE + nb + 1 : nullptr));
  double et = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&et, dE + nb, 8, hipMemcpyDeviceToHost, s));
  if (virial) HIP_TRY(c, hipMemcpyAsync(virial, dE + nb + 1, 9 * 8, hipMemcpyDeviceToHost, s));
  if (e_atom && n > 0) HIP_TRY(c, hipMemcpyAsync(e_atom, dE, n * 8, hipMemcpyDeviceToHost, s));
  if (forces && n > 0) HIP_TRY(c, hipMemcpyAsync(forces, c->h_F.p, n * 24, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (!std::isfinite(et)) return fail(c, AENET_E_NONFINITE, "non-finite energy");
  if (e_total) *e_total = et;
  return AENET_OK;
}
}  // namespace

aenet_status aenet_energy_forces(aenet_ctx* c, int64_t n, const double* pos,
                                 const int32_t* species, const double box[3],
                                 const uint8_t pbc[3], double* e_total, double* e_atom,
                                 double* forces) {
  return ef_host(c, n, pos, species, box, pbc, e_total, e_atom, forces, nullptr);
}

aenet_status aenet_energy_forces_virial(aenet_ctx* c, int64_t n, const double* pos,
                                        const int32_t* species, const double box[3],
                                        const uint8_t pbc[3], double* e_total, double* forces,
                                        double virial[9]) {
  if (c && !virial) return fail(c, AENET_E_INVALID, "virial is NULL");
  return ef_host(c, n, pos, species, box, pbc, e_total, nullptr, forces, virial);
}

aenet_status aenet_descriptors(aenet_ctx* c, int64_t n, const double* pos, const int32_t* species,
                               const double box[3], const uint8_t pbc[3], double* G) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && (!pos || !G))) return fail(c, AENET_E_INVALID, "bad arguments");
  const int64_t off[2] = {0, n};
  hipStream_t s = c->stream;
  if (n > 0) {
    TRY(ensure(c, c->h_pos, (size_t)n * 24));
    HIP_TRY(c, hipMemcpyAsync(c->h_pos.p, pos, n * 24, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipStreamSynchronize(s));
  }
  c->md_state = false;
  TRY(prepare(c, 1, off, species, box, pbc, n > 0 ? c->h_pos.as<double>() : nullptr, s));
  if (n == 0) return AENET_OK;
  HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 8 * sizeof(int), s));
  launch_gather_in((int)n, c->d_perm.as<int>(), c->h_pos.as<double>(), c->d_pos.as<double>(),
                   c->d_flags.as<int>(), s);
  TRY(build_checked(c, s));
  const bool sh = use_factorised(c);
  if (sh) TRY(ensure(c, c->d_shA, (size_t)n * 2 * ang_sh_terms(c->kna) * real_size(c)));
  DescParams dp = desc_params(c);
  launch_desc_fwd(desc_prec(c), c->knr, c->kna, dp, s, !sh);
  if (sh) launch_ang_sh(true, desc_prec(c), c->kna, dp, s);
  HIP_TRY(c, hipGetLastError());
  const size_t el = real_size(c);
  std::vector<unsigned char> buf((size_t)n * c->ldG * el);
  HIP_TRY(c, hipMemcpyAsync(buf.data(), c->d_G.p, buf.size(), hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  c->counters_clean = true;
  for (int64_t p = 0; p < n; ++p) {
    double* dst = G + (size_t)c->perm[p] * c->D;
    for (int k = 0; k < c->D; ++k) {
      const size_t at = (size_t)p * c->ldG + c->colmap[k];
      dst[k] = el == 8 ? reinterpret_cast<double*>(buf.data())[at] : (double)reinterpret_cast<float*>(buf.data())[at];
    }
  }
  return AENET_OK;
}

static aenet_status md_core(aenet_ctx* c, int64_t n, double* pos, double* vel, const int32_t* species,
                            const double box[3], const uint8_t pbc[3], double dt, int n_steps,
                            double* e_pot, double* e_kin, double* forces, hipStream_t s, bool may_speculate) {
  if (!c->have_mass) return fail(c, AENET_E_INVALID, "molecular dynamics needs mass_amu in the model");
  if (!(dt > 0) || n_steps < 0) return fail(c, AENET_E_INVALID, "dt must be > 0 and n_steps >= 0");
  const int64_t off[2] = {0, n};
  // prepare() clears md_state when the species pattern or the box changed
  TRY(prepare(c, 1, off, species, box, pbc, pos, s));
  bool resume = c->md_state;
  c->md_state = false;
  const int N = (int)n;
  if (N == 0) {
    if (e_pot) HIP_TRY(c, hipMemsetAsync(e_pot, 0, 8, s));
    if (e_kin) HIP_TRY(c, hipMemsetAsync(e_kin, 0, 8, s));
    HIP_TRY(c, hipStreamSynchronize(s));
    c->counters_clean = true;
    return AENET_OK;
  }
  TRY(ensure(c, c->d_save_pos, (size_t)N * 24));
  TRY(ensure(c, c->d_save_vel, (size_t)N * 24));
  TRY(ensure(c, c->d_save_F, (size_t)N * 24));
  int* flags = c->d_flags.as<int>();
  // flags: [0] status bits, [1..2] largest rows, [3..4] rebuild decisions by
  // step parity, [5..6] per-cell kernel needs, [8] device-triggered builds,
  // [9] positions differ from the kept state
  HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 16 * sizeof(int), s));
  launch_gather_in(N, c->d_perm.as<int>(), vel, c->d_vel.as<double>(), flags, s);
  // The start from the caller's positions: a list build and a force
  // evaluation.
  auto fresh_start = [&]() -> aenet_status {
    launch_gather_in(N, c->d_perm.as<int>(), pos, c->d_pos.as<double>(), flags, s);
    TRY(build_checked(c, s));
    return compute(c, s, true, nullptr, 0.0);
  };
  // Positions the caller hands back unchanged (bitwise what the last call
  // wrote) continue from the kept device state: its forces, rows and list
  // reference stay valid, so neither a build nor a force evaluation is
  // needed before the first step.  The comparison runs on the device.  When
  // the caller passes the very buffer the last call wrote (a device caller
  // stepping on in chunks) the call goes on as if it held, without waiting:
  // the result is read with the first chunk's status words, and if the state
  // was stale (flags[9]) that chunk, which wrote nothing to the caller, is
  // discarded and the call starts over from the caller's positions and
  // velocities.  Otherwise the result is read before the first step.
  bool speculative = resume && may_speculate && pos == c->md_pos_out;
  if (resume) {
    launch_same_wrapped(N, c->d_perm.as<int>(), c->d_pos.as<double>(), c->d_seg.as<int>(),
                        c->d_boxes.as<BoxInfo>(), c->pbc, pos, flags + 9, s);
    if (!speculative) {
      int hf[10];
      TRY(read_flags(c, s, hf, 10));
      if (hf[0] & kFlagNonFinite) return fail(c, AENET_E_NONFINITE, "non-finite position or velocity");
      if (hf[9] != 0) {
        HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 16 * sizeof(int), s));
        TRY(fresh_start());
      }
    }
  } else {
    TRY(fresh_start());
  }
  const double half_dt = 0.5 * dt;
  const double hs2 = 0.25 * c->skin * c->skin;
  const int K = std::max(1, c->rebuild_every);
  const int64_t nc = std::max<int64_t>(c->n_cells, 1);
  int dev_builds = 0;
  // outputs of the call, enqueued behind the last chunk so that its flag
  // read is the call's only wait
  auto outputs = [&]() {
    double* scal = c->d_scal.as<double>();
    launch_md_outputs(N, c->d_perm.as<int>(), c->d_E.as<double>(), c->d_pos.as<double>(), c->d_vel.as<double>(),
                      c->d_F.as<double>(), c->d_mass.as<double>(), c->d_species.as<int>(), c->d_seg.as<int>(),
                      c->d_boxes.as<BoxInfo>(), c->pbc, flags, c->d_red.as<double>(), e_pot ? e_pot : scal,
                      e_kin ? e_kin : scal + 1, pos, vel, forces, s);
  };
  int t = 0;  // steps done
  bool bins_clean = false;
  for (;;) {
    const int len = std::min(K - (t % K), n_steps - t);
    const bool last = t + len >= n_steps;
    // checkpoint for a capacity retry
    if (len > 0)
      launch_copy3(3 * (int64_t)N, c->d_pos.as<double>(), c->d_save_pos.as<double>(), c->d_vel.as<double>(),
                   c->d_save_vel.as<double>(), c->d_F.as<double>(), c->d_save_F.as<double>(), s);
    bool force_first = false;
    bool restart = false;
    for (int attempt = 0;; ++attempt) {
      // With the per-cell row kernel the integrator bins the atoms for the
      // next build as it moves them (two halves of counts by step parity:
      // the build of step t reads half t & 1 and clears the other, so after
      // the first chunk of a call the half the next drift fills is clear).
      const bool binned = c->tp > 0;
      if (binned && len > 0) {
        TRY(ensure(c, c->d_bin_count, (size_t)2 * nc * sizeof(int)));
        TRY(ensure(c, c->d_bin_atoms, (size_t)nc * kCellAtomsMax * sizeof(int)));
        if (!bins_clean) HIP_TRY(c, hipMemsetAsync(c->d_bin_count.p, 0, (size_t)2 * nc * sizeof(int), s));
        bins_clean = true;
      }
      // the opening half kick and drift of a step are fused into the force
      // gather of the step before it, except for the first step of a chunk
      auto drift_args = [&](int step, bool force) {
        DriftArgs d{};
        d.pos = c->d_pos.as<double>();
        d.pos_ref = c->d_pos_ref.as<double>();
        d.dt = dt;
        d.half_skin2 = hs2;
        d.rebuild_flag = flags + 3 + (step & 1);
        d.clear_flag = flags + 3 + ((step + 1) & 1);
        d.force_rebuild = force ? 1 : 0;
        if (binned) {
          d.bin_count = c->d_bin_count.as<int>() + (size_t)(step & 1) * nc;
          d.bin_atoms = c->d_bin_atoms.as<int>();
          d.box = c->d_boxes.as<BoxInfo>();
          for (int a = 0; a < 3; ++a) d.pbc[a] = c->pbc[a];
        }
        return d;
      };
      for (int k = 0; k < len; ++k) {
        const int step = t + k + 1;  // 1-based index of this step
        int* rb = flags + 3 + (step & 1);
        if (k == 0) {
          const int force = (step % K == 0) || force_first;
          prof_begin(c, s, AENET_K_INTEGRATE);
          launch_vv_drift(N, c->d_vel.as<double>(), c->d_F.as<double>(), c->d_invmk.as<double>(),
                          c->d_species.as<int>(), half_dt, drift_args(step, force != 0), s);
          prof_end(c, s);
        }
        NbrParams np = nbr_params(c, rb);
        if (binned) {
          np.binned = 1;
          np.bin_count = c->d_bin_count.as<int>();
          np.bin_atoms = c->d_bin_atoms.as<int>();
          np.bin_sel = step & 1;
        }
        build_neighbors_timed(c, np, s);
        if (k + 1 < len) {
          const DriftArgs next = drift_args(step + 1, (step + 1) % K == 0);
          TRY(compute(c, s, true, c->d_vel.as<double>(), half_dt, &next));
        } else {
          TRY(compute(c, s, true, c->d_vel.as<double>(), half_dt));
        }
      }
      if (last) outputs();
      HIP_TRY(c, hipGetLastError());
      int hf[10];
      TRY(read_flags(c, s, hf, 10));
      if (speculative) {
        speculative = false;
        if (hf[9] != 0) {
          HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 16 * sizeof(int), s));
          launch_gather_in(N, c->d_perm.as<int>(), vel, c->d_vel.as<double>(), flags, s);
          TRY(fresh_start());
          restart = true;
          break;
        }
      }
      // non-finite inputs (or a run that blew up) end the call whatever else
      // the chunk flagged: a capacity retry would clear the status word
      if (hf[0] & kFlagNonFinite) return fail(c, AENET_E_NONFINITE, "non-finite position or velocity");
      if (!(hf[0] & kFlagOverflow)) {
        TRY(flag_status(c, hf[0]));
        dev_builds = hf[8];
        break;
      }
      // truncated rows make the rest of the chunk meaningless, whatever else
      // it flagged: grow the rows and redo the chunk from its checkpoint
      if (attempt >= 3) return fail(c, AENET_E_DEVICE, "neighbour capacity retries exhausted");
      TRY(grow_caps(c, hf));
      launch_copy3(3 * (int64_t)N, c->d_save_pos.as<double>(), c->d_pos.as<double>(), c->d_save_vel.as<double>(),
                   c->d_vel.as<double>(), c->d_save_F.as<double>(), c->d_F.as<double>(), s);
      HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 8 * sizeof(int), s));
      bins_clean = false;
      force_first = true;
    }
    if (restart) {
      t = 0;
      bins_clean = false;
      continue;
    }
    t += len;
    if (t >= n_steps) break;
  }
  c->stats.n_rebuilds += dev_builds;
  c->counters_clean = true;
  c->md_state = true;
  c->md_pos_out = pos;
  return AENET_OK;
}

aenet_status aenet_md_step_dev(aenet_ctx* c, int64_t n, double* pos, double* vel,
                               const int32_t* species, const double box[3], const uint8_t pbc[3],
                               double dt_ps, int n_steps, double* e_pot, double* e_kin,
                               double* forces, void* stream) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && (!pos || !vel))) return fail(c, AENET_E_INVALID, "bad arguments");
  return md_core(c, n, pos, vel, species, box, pbc, dt_ps, n_steps, e_pot, e_kin, forces,
                 pick_stream(c, stream), true);
}

aenet_status aenet_md_step(aenet_ctx* c, int64_t n, double* pos, double* vel,
                           const int32_t* species, const double box[3], const uint8_t pbc[3],
                           double dt_ps, int n_steps, double* e_pot, double* e_kin,
                           double* forces) {
  TRY(check_ctx(c));
  if (n < 0 || !box || (n > 0 && (!pos || !vel))) return fail(c, AENET_E_INVALID, "bad arguments");
  for (int64_t k = 0; k < 3 * n; ++k)
    if (!std::isfinite(pos[k]) || !std::isfinite(vel[k]))
      return fail(c, AENET_E_NONFINITE, "non-finite position or velocity");
  const size_t nb = (size_t)std::max<int64_t>(n, 1);
  TRY(ensure(c, c->h_pos, nb * 24));
  TRY(ensure(c, c->h_vel, nb * 24));
  TRY(ensure(c, c->h_F, nb * 24));
  TRY(ensure(c, c->h_E, (nb + 2) * 8));
  hipStream_t s = c->stream;
  if (n > 0) {
    HIP_TRY(c, hipMemcpyAsync(c->h_pos.p, pos, n * 24, hipMemcpyHostToDevice, s));
    HIP_TRY(c, hipMemcpyAsync(c->h_vel.p, vel, n * 24, hipMemcpyHostToDevice, s));
  }
  double* dE = c->h_E.as<double>();
  TRY(md_core(c, n, c->h_pos.as<double>(), c->h_vel.as<double>(), species, box, pbc, dt_ps, n_steps,
              dE, dE + 1, forces ? c->h_F.as<double>() : nullptr, s, false));
  double e2[2] = {0, 0};
  HIP_TRY(c, hipMemcpyAsync(e2, dE, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  if (!std::isfinite(e2[0]) || !std::isfinite(e2[1])) return fail(c, AENET_E_NONFINITE, "non-finite energy");
  if (n > 0) {
    HIP_TRY(c, hipMemcpyAsync(pos, c->h_pos.p, n * 24, hipMemcpyDeviceToHost, s));
    HIP_TRY(c, hipMemcpyAsync(vel, c->h_vel.p, n * 24, hipMemcpyDeviceToHost, s));
    if (forces) HIP_TRY(c, hipMemcpyAsync(forces, c->h_F.p, n * 24, hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(c, hipStreamSynchronize(s));
  if (e_pot) *e_pot = e2[0];
  if (e_kin) *e_kin = e2[1];
  return AENET_OK;
}

aenet_status aenet_loss_grad_dev(aenet_ctx* c, int n_struct, const int64_t* offsets,
                                 const double* pos, const int32_t* species, const double* boxes,
                                 const uint8_t pbc[3], const double* e_ref, const double* f_ref,
                                 double lambda_f, double* loss, double* grad, void* stream) {
  TRY(check_ctx(c));
  if (c->prec == AENET_BF16) return fail(c, AENET_E_INVALID, "training needs an FP64 or FP32 context");
  if (n_struct < 1 || !offsets || !boxes || !e_ref || !f_ref || !loss || !grad || !(lambda_f >= 0))
    return fail(c, AENET_E_INVALID, "bad arguments");
  hipStream_t s = pick_stream(c, stream);
  c->md_state = false;
  TRY(prepare(c, n_struct, offsets, species, boxes, pbc, pos, s));
  const int n = (int)c->n;
  if (n == 0) return fail(c, AENET_E_INVALID, "empty batch");
  for (int b = 0; b < n_struct; ++b)
    if (offsets[b + 1] == offsets[b]) return fail(c, AENET_E_INVALID, "empty structure in batch");
  const size_t el = real_size(c);
  TRY(ensure(c, c->d_U, (size_t)n * c->ldG * el));
  TRY(ensure(c, c->d_adj, (size_t)n * 24));
  TRY(ensure(c, c->d_eps, (size_t)n * 8));
  TRY(ensure(c, c->d_estruct, (size_t)n_struct * 8));
  HIP_TRY(c, hipMemsetAsync(c->d_flags.p, 0, 8 * sizeof(int), s));
  launch_gather_in(n, c->d_perm.as<int>(), pos, c->d_pos.as<double>(), c->d_flags.as<int>(), s);
  TRY(build_checked(c, s));
  TRY(compute(c, s, true, nullptr, 0.0, nullptr, true));
  // structure energies (caller order makes every structure contiguous)
  launch_scatter_out(n, c->d_perm.as<int>(), nullptr, nullptr, c->d_E.as<double>(), c->d_Eorig.as<double>(), s);
  launch_segment_sum(n_struct, c->d_segoff.as<int64_t>(), c->d_Eorig.as<double>(), c->d_estruct.as<double>(), s);
  // loss terms: tmp[0..n) force part per atom, tmp[n..n+B) energy part per structure
  double* tmp = c->d_tmp.as<double>();
  launch_loss_terms(n, n_struct, c->d_seg.as<int>(), c->d_perm.as<int>(), c->d_F.as<double>(), f_ref,
                    c->d_estruct.as<double>(), e_ref, c->d_segcount.as<int64_t>(), lambda_f, c->loss_form,
                    c->d_adj.as<double>(), c->d_eps.as<double>(), tmp, tmp + n, s);
  launch_sum((int64_t)n + n_struct, tmp, c->d_red.as<double>(), loss, s);
  // descriptor JVP along the force adjoint, then double back-propagation
  DescParams dp = desc_params(c);
  launch_desc_jvp(desc_prec(c), c->knr, c->kna, dp, s);
  MlpParams mp = mlp_params(c, false);
  mp.U = c->d_U.p;
  mp.eps_atom = c->d_eps.as<double>();
  mp.tiles_per_block = 8;
  int nblocks = 0;
  for (int t = 0; t < c->S; ++t) {
    const int nt = mp.tile_off[t + 1] - mp.tile_off[t];
    nblocks += (nt + mp.tiles_per_block - 1) / mp.tiles_per_block;
  }
  const int npad = c->S * c->npad_species;
  mp.n_params_pad = npad;
  for (int t = 0; t < c->S; ++t) mp.param_off[t] = t * c->npad_species;
  TRY(ensure(c, c->d_gradpart, (size_t)std::max(nblocks, 1) * npad * 8));
  TRY(ensure(c, c->d_gradpad, (size_t)npad * 8));
  mp.grad_part = c->d_gradpart.as<double>();
  if (mlp_train_lds_bytes(c->prec, mp) > 160 * 1024) return fail(c, AENET_E_INVALID, "network too wide for the training kernel");
  launch_mlp_train(c->prec == 0 ? 0 : 1, mp, nblocks, s);
  launch_grad_reduce(nblocks, npad, c->d_gradpart.as<double>(), c->d_gradpad.as<double>(), s);
  // padded -> API layout
  launch_take((int)c->params.size(), c->d_pidx.as<int>(), c->d_gradpad.as<double>(), grad, s);
  HIP_TRY(c, hipGetLastError());
  int hf[8];
  TRY(read_flags(c, s, hf));
  TRY(flag_status(c, hf[0]));
  c->counters_clean = true;
  return AENET_OK;
}

aenet_status aenet_loss_grad(aenet_ctx* c, int n_struct, const int64_t* offsets, const double* pos,
                             const int32_t* species, const double* boxes, const uint8_t pbc[3],
                             const double* e_ref, const double* f_ref, double lambda_f, double* loss,
                             double* grad) {
  TRY(check_ctx(c));
  if (n_struct < 1 || !offsets || offsets[0] != 0 || !pos || !boxes || !e_ref || !f_ref || !loss || !grad)
    return fail(c, AENET_E_INVALID, "bad arguments");
  for (int b = 0; b < n_struct; ++b)
    if (offsets[b + 1] < offsets[b]) return fail(c, AENET_E_INVALID, "structure offsets must not decrease");
  const int64_t n = offsets[n_struct];
  if (n < 1) return fail(c, AENET_E_INVALID, "empty batch");
  for (int64_t k = 0; k < 3 * n; ++k)
    if (!std::isfinite(pos[k])) return fail(c, AENET_E_NONFINITE, "non-finite position");
  const size_t np = c->params.size();
  TRY(ensure(c, c->h_pos, (size_t)n * 24));
  TRY(ensure(c, c->h_F, (size_t)n * 24));
  TRY(ensure(c, c->h_E, ((size_t)n_struct + 1 + np) * 8));
  hipStream_t s = c->stream;
  double* dE = c->h_E.as<double>();
  HIP_TRY(c, hipMemcpyAsync(c->h_pos.p, pos, (size_t)n * 24, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(c->h_F.p, f_ref, (size_t)n * 24, hipMemcpyHostToDevice, s));
  HIP_TRY(c, hipMemcpyAsync(dE, e_ref, (size_t)n_struct * 8, hipMemcpyHostToDevice, s));
  TRY(aenet_loss_grad_dev(c, n_struct, offsets, c->h_pos.as<double>(), species, boxes, pbc, dE,
                          c->h_F.as<double>(), lambda_f, dE + n_struct, dE + n_struct + 1, s));
  double out = 0.0;
  HIP_TRY(c, hipMemcpyAsync(&out, dE + n_struct, 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipMemcpyAsync(grad, dE + n_struct + 1, np * 8, hipMemcpyDeviceToHost, s));
  HIP_TRY(c, hipStreamSynchronize(s));
  *loss = out;
  return AENET_OK;
}

aenet_status aenet_get_stats(const aenet_ctx* c, aenet_stats* out) {
  if (!c || !out) return AENET_E_INVALID;
  *out = c->stats;
  out->rebuild_every = c->rebuild_every;
  out->row_capacity = c->cap;
  out->ang_capacity = c->cap_ang;
  return AENET_OK;
}

aenet_status aenet_set_rebuild_every(aenet_ctx* c, int k) {
  if (!c || k < 1) return AENET_E_INVALID;
  c->rebuild_every = k;
  return AENET_OK;
}

aenet_status aenet_set_angular_method(aenet_ctx* c, int method) {
  TRY(check_ctx(c));
  if (method != AENET_ANGULAR_AUTO && method != AENET_ANGULAR_PAIRS && method != AENET_ANGULAR_FACTORISED)
    return fail(c, AENET_E_INVALID, "unknown angular method");
  c->ang_method = method;
  return AENET_OK;
}

aenet_status aenet_set_fused(aenet_ctx* c, int enable) {
  TRY(check_ctx(c));
  c->fused = enable != 0;
  return AENET_OK;
}

aenet_status aenet_set_capacity(aenet_ctx* c, int row_capacity, int ang_capacity) {
  TRY(check_ctx(c));
  if (row_capacity == 0 && ang_capacity == 0) {
    c->cap_user = c->cap_ang_user = 0;
  } else {
    if (ang_capacity < 1 || row_capacity < ang_capacity || ang_capacity > 700 || row_capacity > 4096)
      return fail(c, AENET_E_INVALID, "need 1 <= ang_capacity <= row_capacity, ang_capacity <= 700, row_capacity <= 4096");
    c->cap_user = row_capacity;
    c->cap_ang_user = ang_capacity;
  }
  c->cap = 0;  // applied at the next call's set-up
  c->nbr_valid = false;
  c->md_state = false;
  return AENET_OK;
}

aenet_status aenet_set_profiling(aenet_ctx* c, int enable) {
  TRY(check_ctx(c));
  HIP_TRY(c, hipStreamSynchronize(c->stream));
  prof_collect(c);
  c->profiling = enable != 0;
  return AENET_OK;
}

aenet_status aenet_get_kernel_times(aenet_ctx* c, double* ms, int64_t* launches) {
  TRY(check_ctx(c));
  if (!ms || !launches) return fail(c, AENET_E_INVALID, "bad arguments");
  prof_collect(c);
  for (int k = 0; k < AENET_K_COUNT; ++k) {
    ms[k] = c->prof_ms[k];
    launches[k] = c->prof_n[k];
    c->prof_ms[k] = 0.0;
    c->prof_n[k] = 0;
  }
  return AENET_OK;
}

}  // extern "C"

