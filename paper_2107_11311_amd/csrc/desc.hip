// desc.hip -- Chebyshev descriptor kernels (Sec. II B): forward (Eqs. 3-6),
// force back-propagation to per-entry displacement gradients, and the
// Jacobian-vector product used by the training gradient.
//
// Forward and JVP: a group of LPA lanes of one wavefront works on one centre
// atom; lanes stride over the atom's neighbour entries for the radial terms
// (Eq. 3), the entries within R_a are compacted into LDS (unit vector, f_c,
// species weight, ...) and lanes stride over the unordered pairs j < k for the
// angular terms (the ordered-pair sum of Eq. 6 is twice that).  Accumulators
// live in registers (orders are compile-time) and are summed over the group
// with cross-lane shuffles.  The force pass takes a wavefront per atom (see
// k_desc_bwd).  R is the arithmetic type (double, or float with the
// displacement taken in double).
#include <map>
#include <mutex>
#include <tuple>

#include "desc_dev.h"

namespace aenet {

namespace {
// ------------------------------------------------------------------ forward
template <typename R, int NR, int NA, int LPA, bool ANG>
__global__ __launch_bounds__(256, 3) void k_desc_fwd(DescParams p) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (p.prio) __builtin_amdgcn_s_setprio(3);
  const int apb = blockDim.x / LPA;
  const int g = threadIdx.x / LPA, l = threadIdx.x % LPA;
  const int i = blockIdx.x * apb + g;
  const bool active = i < p.n;
  R* G = reinterpret_cast<R*>(p.G) + (size_t)(active ? i : 0) * p.ldG;
  auto out = [&](int c, R v) { G[c] = v; };
  desc_fwd_group<R, NR, NA, LPA, decltype(out)&, ANG>(p, i, active, g, l, smem, out);
}

// ------------------------------------------------------------------ backward
// LDS of the force pass (elements of R): twelve arrays of cap_ang entries,
// the compaction index (cap_ang ints), then the per-species series
// coefficients
constexpr int kBwdArrays = 12;
template <typename R>
__host__ __device__ constexpr size_t bwd_coef_offset(int ca) {
  return (size_t)ca * kBwdArrays + ((size_t)ca * sizeof(int) + sizeof(R) - 1) / sizeof(R);
}

// dE_i / d d_e for every entry e of atom i, stored at the slot of the reverse
// entry (pg[rev(i, e)]) for the force gather; Fself[i] = sum_e dE_i / d d_e.
// One wavefront per atom (the atom index is uniform over the wave):
//   compaction of the entries within R_a into LDS (unit vector, f_c, f_c',
//     species weight, 1/r);
//   angular terms by rotation (below), the gradient of entry k kept in the
//     registers of the lane that owns k, so no atomics are needed;
//   radial terms, one entry per lane per iteration, adding the angular
//     gradient of the entry and writing pg.
// VIR: also the atom's virial -sum_e (dE_i/dd_e) d_e^T (a separate
// instance, so that the force pass of MD keeps its registers).
// AEXT: the angular part of every entry's gradient comes from p.gang (the
// factorised angular kernel), so the compaction and the pair loop are skipped.
template <typename R, int NR, int NA, bool VIR, bool AEXT>
__global__ __launch_bounds__(256, 5) void k_desc_bwd(DescParams p) {
  extern __shared__ __align__(16) unsigned char smem[];
  // one wavefront per block and atom (a block without an atom returns at
  // once), so every load below is unconditional (loads under a branch are
  // issued one after another, each waiting for the last)
  const int i = p.xmap[blockIdx.x];
  if (i < 0) return;
  const int l = threadIdx.x & 63;
  const int ca = p.cap_ang;
  R* ux = reinterpret_cast<R*>(smem);
  R* uy = ux + ca;
  R* uz = uy + ca;
  R* fs = uz + ca;
  R* fp = fs + ca;
  R* ws = fp + ca;
  R* ri = ws + ca;
  R* gx = ri + ca;
  R* gy = gx + ca;
  R* gz = gy + ca;
  R* s1a = gz + ca;  // crowded shells: the sums s1, s2 of each entry (below)
  R* s2a = s1a + ca;
  int* kidx = reinterpret_cast<int*>(reinterpret_cast<R*>(smem) + (size_t)ca * kBwdArrays);
  // radial series coefficients of each species s (NR + 1 per species); with
  // AEXT the angular arrays are not needed and the table starts the LDS
  R* s_c = reinterpret_cast<R*>(smem) + (AEXT ? 0 : bwd_coef_offset<R>(ca));

  const BoxInfo b = p.boxes[p.seg[i]];
  const double xi0 = p.pos[3 * (size_t)i];
  const double xi1 = p.pos[3 * (size_t)i + 1];
  const double xi2 = p.pos[3 * (size_t)i + 2];
  const uint32_t* row = p.nbr + (size_t)i * p.cap;
  const int na = p.nang[i];
  const double rr2 = p.rr * p.rr, ra2 = p.ra * p.ra;
  const R inv_rr2 = R(p.two_rr), pi_2rr = R(p.pi_2rr), pi_2ra = R(p.pi_2ra);
  const R* gG = reinterpret_cast<const R*>(p.gG) + (size_t)i * p.ldG;
  constexpr int T1 = NR + 1, T2 = NR + NA + 2;
  // the weighted channel's coefficients (read at the typed ones and unused
  // when the descriptor has no weighted channel)
  const R* gW = gG + (p.weighted ? T2 : 0);

  // compact the entries within R_a (lanes past the end reread the last one)
  int nv = 0;
  for (int base = 0; !AEXT && base < na; base += 64) {
    const int e = base + l;
    const NbrLoad nl = load_nbr(p, row[min(e, na - 1)]);
    double d0, d1, d2;
    nbr_disp(nl, b, xi0, xi1, xi2, d0, d1, d2);
    const bool valid = e < na && d0 * d0 + d1 * d1 + d2 * d2 < ra2;
    R r, vri, vf, vfp;
    len_inv<R>(R(d0) * R(d0) + R(d1) * R(d1) + R(d2) * R(d2), &r, &vri);
    const R vx = R(d0) * vri, vy = R(d1) * vri, vz = R(d2) * vri;
    cutoff_d<R>(r, pi_2ra, &vf, &vfp);
    const R vw = R(nl.w);
    const uint64_t m = __ballot(valid);
    const int at_ = nv + __popcll(m & ((1ull << l) - 1ull));
    if (valid) {
      ux[at_] = vx;
      uy[at_] = vy;
      uz[at_] = vz;
      fs[at_] = vf;
      fp[at_] = vfp;
      ws[at_] = vw;
      ri[at_] = vri;
    }
    if (e < na) kidx[e] = valid ? at_ : -1;
    nv += __popcll(m);
  }
  nv = __builtin_amdgcn_readfirstlane(nv);
  __syncthreads();

  // angular terms: d/dd_k of sum over ordered pairs = 2 x the unordered pairs
  if (!AEXT) {
    R ga[NA + 1], gw[NA + 1];
#pragma unroll
    for (int a = 0; a <= NA; ++a) {
      const R v = gW[T1 + a];
      ga[a] = gG[T1 + a];
      gw[a] = p.weighted ? v : R(0);
    }
    if (nv <= 64) {
      // Unordered pairs by rotation: the lane owning entry e takes at step t
      // the pair (e, (e + t) mod nv), adds the pair's terms to the sums of its
      // own entry and passes the partner's terms to the lane owning the
      // partner (a rotation by t).  Steps t = 1..floor(nv/2) visit every pair once (for
      // even nv the last step is taken by entries e < t only).  With nv <= 32
      // both halves of the wave hold all entries and share the steps: the
      // lower half takes t = 1..T1, the upper half the rest.
      const bool split = nv <= 32;
      const int half = split ? (l >> 5) : 0;
      const int e = split ? (l & 31) : l;
      const bool own = e < nv;
      const int T = nv >> 1;
      const int Tlo = split ? (T + 1) >> 1 : T;
      const int t0 = half ? Tlo : 0;
      const int cnt = half ? T - Tlo : Tlo;
      const int lane0 = half << 5;  // first lane of this half
      const int k = own ? e : 0;
      const R kx = ux[k], ky = uy[k], kz = uz[k], fk = fs[k], wk = ws[k];
      // With F(c) = sum_a (ga_a + w_j w_k gw_a) T_a(c), A = F, B = F' and
      // c = u_j . u_k, the pair (j, k) adds to dE/dd_k
      //   f_j [B f_k (u_j - c u_k) / r_k + A f_k' u_k],
      // so each lane sums V = sum_j B f_j u_j, s1 = sum_j B f_j c and
      // s2 = sum_j A f_j over its partners and forms the gradient once.
      R vx = 0, vy = 0, vz = 0, s1 = 0, s2 = 0;
      for (int st = 1; st <= Tlo; ++st) {
        const int t = t0 + st;
        const bool go = own && st <= cnt;
        int m = e + t;
        if (m >= nv) m -= nv;
        if (!go) m = k;
        const R wgt = (go && (2 * t != nv || e < t)) ? R(1) : R(0);
        const R jx = ux[m], jy = uy[m], jz = uz[m], fm = fs[m];
        const R c = jx * kx + jy * ky + jz * kz;
        R A, B;
        cheb_series_d<R, NA>(ga, gw, ws[m] * wk, c, &A, &B);
        A *= wgt;
        B *= wgt;
        // own side
        const R bj = B * fm;
        vx += bj * jx;
        vy += bj * jy;
        vz += bj * jz;
        s1 += bj * c;
        s2 += A * fm;
        // partner side, delivered by rotation: this lane receives from the
        // lane owning entry (e - t) mod nv in the same half
        const R bk = B * fk;
        int src = e - t;
        if (src < 0) src += nv;
        src = go ? lane0 + src : l;
        const R rx = __shfl(bk * kx, src, 64), ry = __shfl(bk * ky, src, 64), rz = __shfl(bk * kz, src, 64);
        const R r1 = __shfl(bk * c, src, 64), r2 = __shfl(A * fk, src, 64);
        if (go) {
          vx += rx;
          vy += ry;
          vz += rz;
          s1 += r1;
          s2 += r2;
        }
      }
      if (split) {
        vx += __shfl_xor(vx, 32, 64);
        vy += __shfl_xor(vy, 32, 64);
        vz += __shfl_xor(vz, 32, 64);
        s1 += __shfl_xor(s1, 32, 64);
        s2 += __shfl_xor(s2, 32, 64);
      }
      if (own && half == 0) {
        const R cb = R(2) * fk * ri[k], ca_ = R(2) * fp[k] * s2 - cb * s1;
        gx[e] = cb * vx + ca_ * kx;
        gy[e] = cb * vy + ca_ * ky;
        gz[e] = cb * vz + ca_ * kz;
      }
    } else {
      // Crowded shells: the same rotation over all nv entries, lane l taking
      // entries l, l + 64, ... in turn.  Its own entry's sums stay in
      // registers; the partner's are added into LDS (V into gx, gy, gz, s1
      // and s2 into s1a, s2a), in place: at a step t every entry is the
      // partner of exactly one entry, so the additions of one step never
      // meet; the steps are ordered by a fence (the lanes of the wavefront
      // exchange values through LDS).
      auto lds_step = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      };
      for (int k = l; k < nv; k += 64) gx[k] = gy[k] = gz[k] = s1a[k] = s2a[k] = R(0);
      __syncthreads();
      const int T = nv >> 1;
      for (int base = 0; base < nv; base += 64) {
        const int e = base + l;
        const bool own = e < nv;
        const int k = own ? e : 0;
        const R kx = ux[k], ky = uy[k], kz = uz[k], fk = fs[k], wk = ws[k];
        R vx = 0, vy = 0, vz = 0, s1 = 0, s2 = 0;
        for (int t = 1; t <= T; ++t) {
          int m = e + t;
          if (m >= nv) m -= nv;
          const bool go = own && (2 * t != nv || e < t);
          if (!own) m = k;
          const R wgt = go ? R(1) : R(0);
          const R jx = ux[m], jy = uy[m], jz = uz[m], fm = fs[m];
          const R c = jx * kx + jy * ky + jz * kz;
          R A, B;
          cheb_series_d<R, NA>(ga, gw, ws[m] * wk, c, &A, &B);
          A *= wgt;
          B *= wgt;
          const R bj = B * fm;
          vx += bj * jx;
          vy += bj * jy;
          vz += bj * jz;
          s1 += bj * c;
          s2 += A * fm;
          if (go) {
            const R bk = B * fk;
            gx[m] += bk * kx;
            gy[m] += bk * ky;
            gz[m] += bk * kz;
            s1a[m] += bk * c;
            s2a[m] += A * fk;
          }
          lds_step();
        }
        if (own) {
          gx[e] += vx;
          gy[e] += vy;
          gz[e] += vz;
          s1a[e] += s1;
          s2a[e] += s2;
        }
        lds_step();
      }
      __syncthreads();
      for (int k = l; k < nv; k += 64) {
        const R cb = R(2) * fs[k] * ri[k], ca_ = R(2) * fp[k] * s2a[k] - cb * s1a[k];
        const R vxk = gx[k], vyk = gy[k], vzk = gz[k];
        gx[k] = cb * vxk + ca_ * ux[k];
        gy[k] = cb * vyk + ca_ * uy[k];
        gz[k] = cb * vzk + ca_ * uz[k];
      }
    }
  }
  __syncthreads();

  // radial terms, plus the angular part of each entry, written per entry.
  // The coefficients of the series are combined per species into
  // c_a(s) = dE/dG_t,a + tw_s dE/dG_w,a in LDS (read by every lane for its
  // neighbour's species; kept in registers they would crowd out the scalar
  // registers the loop needs).
  for (int t = l; t < p.n_species * (NR + 1); t += 64) {
    const int sp = t / (NR + 1), a = t - sp * (NR + 1);
    const R w = p.weighted ? R(p.tw[sp]) : R(0);
    s_c[t] = gG[a] + w * gW[a];
  }
  __syncthreads();
  R* pg = reinterpret_cast<R*>(p.pg);
  int* rev = p.rev + (size_t)i * p.cap;
  const int n_slots = p.n * p.cap;
  double sx = 0.0, sy = 0.0, sz = 0.0;
  double w9[VIR ? 9 : 1] = {};
  // The reverse slot of entry e: on first use after a per-cell row build rev
  // holds (rank, stencil cell k) and the reverse entry (q -> i) is the rank-th
  // entry of the segment of stencil cell 26 - k in q's row part; resolved once
  // and stored back (-1: no slot, the list is flagged asymmetric).
  auto reverse_slot = [&](int e) {
    int dst = rev[e];
    if (dst <= kRevPending) {
      const int info = kRevPending - dst, rank = info & 0xffff, k = info >> 16;
      const int q = (int)(row[e] & kAtomMask);
      const uint16_t* sq = p.segs + (size_t)q * kSegWords + (e < na ? 0 : 28);
      const int at = k <= 26 ? (int)sq[26 - k] + rank : 0;
      const bool ok = k <= 26 && at < (int)sq[27 - k];
      dst = ok ? q * p.cap + at : -1;
      if (!ok) atomicOr(p.flags, kFlagReverse);
      rev[e] = dst;
    }
    return dst < n_slots ? dst : -1;
  };
  // The entries the forward pass listed (the contributing ones from the
  // front of ridx, then the margin ones from its back: nk in all), one per
  // lane per iteration with the next one's position loaded ahead; a slot past
  // the end repeats the last entry (an empty list reads row slot 0; the
  // clamps keep whatever it holds inside the arrays, and it is not used).
  // Their pg is stored at the reverse entry's slot, where the force gather of
  // the neighbour reads it.
  const uint16_t* ridx = p.ridx + (size_t)i * p.cap;
  const int nr_code = p.nrad[i];
  const int nkeep = nr_code & 0xffff;
  const int nk = nkeep + (nr_code >> 16);
  // (three dependent loads per entry: its row position, its row word, the
  // neighbour's position; each is issued one iteration before it is needed)
  auto entry = [&](int k) {
    const int kk = k < nk ? k : nk - 1;
    return min((int)ridx[kk < 0 ? 0 : kk < nkeep ? kk : p.cap - 1 - (kk - nkeep)], p.cap - 1);
  };
  auto word = [&](int e) { return row[e]; };
  int ea = entry(l), eb = entry(l + 64), ec = entry(l + 128);
  NbrLoad nx = load_nbr(p, word(ea));
  uint32_t wb = word(eb);
  for (int k = l; k - l < nk; k += 64) {
    const NbrLoad n1 = load_nbr(p, wb);
    wb = word(ec);
    const int ed = entry(k + 192);
    const int e = ea;
    ea = eb;
    eb = ec;
    ec = ed;
    const bool he = k < nk;
    double d0, d1, d2;
    nbr_disp(nx, b, xi0, xi1, xi2, d0, d1, d2);
    const R* cq = s_c + nx.sp * (NR + 1);
    nx = n1;
    // angular entries beyond R_r (R_a + skin > R_r) have no radial term
    const R mq = (he && d0 * d0 + d1 * d1 + d2 * d2 < rr2) ? R(1) : R(0);
    const R dx = R(d0), dy = R(d1), dz = R(d2);
    R r, ir;
    len_inv<R>(dx * dx + dy * dy + dz * dz, &r, &ir);
    const R x = r * inv_rr2 - R(1);
    R fc, fcp;
    cutoff_d<R>(r, pi_2rr, &fc, &fcp);
    // dE/dr = S'(x) (2/R_r) f_c + S(x) f_c' with S = sum_a c_a(s) T_a
    R S, dS;
    cheb_series_tab<R, NR>(cq, x, &S, &dS);
    const R sc = mq * (dS * inv_rr2 * fc + S * fcp) * ir;
    R px = sc * dx, py = sc * dy, pz = sc * dz;
    if (AEXT) {
      if (he && e < na) {
        const R* ga = reinterpret_cast<const R*>(p.gang) + ((size_t)i * p.cap_ang + e) * 3;
        px += ga[0];
        py += ga[1];
        pz += ga[2];
      }
    } else if (he && e < na) {
      const int ka = kidx[e];
      if (ka >= 0) {
        px += gx[ka];
        py += gy[ka];
        pz += gz[ka];
      }
    }
    if (he) {
      const int dst = reverse_slot(e);
      if (dst >= 0) {
        pg[3 * (size_t)dst] = px;
        pg[3 * (size_t)dst + 1] = py;
        pg[3 * (size_t)dst + 2] = pz;
      }
      sx += (double)px;
      sy += (double)py;
      sz += (double)pz;
      if constexpr (VIR) {
        const double g3[3] = {(double)px, (double)py, (double)pz}, d3[3] = {d0, d1, d2};
#pragma unroll
        for (int a = 0; a < 3; ++a)
#pragma unroll
          for (int c = 0; c < 3; ++c) w9[3 * a + c] -= g3[a] * d3[c];
      }
    }
  }
  // The other entries (the skin shell) store nothing: no gather reads their
  // slots.  (An entry that later moves inside R_r resolves its reverse slot
  // on that first use.)
  sx = group_sum<64>(sx);
  sy = group_sum<64>(sy);
  sz = group_sum<64>(sz);
  if constexpr (VIR) {
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const double v = group_sum<64>(w9[k]);
      if (l == 0) p.vir[(size_t)k * p.n + i] = v;
    }
  }
  if (l == 0) {
    p.Fself[3 * (size_t)i] = sx;
    p.Fself[3 * (size_t)i + 1] = sy;
    p.Fself[3 * (size_t)i + 2] = sz;
  }
}

// ------------------------------------------------------------------ JVP
// U_i = sum_e dG_i/dd_e . (adj_j(e) - adj_i)
template <typename R, int NR, int NA, int LPA>
__global__ __launch_bounds__(256) void k_desc_jvp(DescParams p) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int apb = blockDim.x / LPA;
  const int g = threadIdx.x / LPA, l = threadIdx.x % LPA;
  const int i = blockIdx.x * apb + g;
  const bool active = i < p.n;
  const int ca = p.cap_ang;
  R* ux = reinterpret_cast<R*>(smem) + (size_t)g * ca * 11;
  R* uy = ux + ca;
  R* uz = uy + ca;
  R* fs = uz + ca;   // f_c
  R* fd = fs + ca;   // f_c' (u . dd)   (time derivative of f_c)
  R* ws = fd + ca;
  R* ri = ws + ca;
  R* vx_ = ri + ca;  // dd
  R* vy_ = vx_ + ca;
  R* vz_ = vy_ + ca;
  R* pa = vz_ + ca;  // u . dd

  R rt[NR + 1], rw[NR + 1], at[NA + 1], aw[NA + 1];
#pragma unroll
  for (int a = 0; a <= NR; ++a) rt[a] = rw[a] = R(0);
#pragma unroll
  for (int a = 0; a <= NA; ++a) at[a] = aw[a] = R(0);

  const BoxInfo b = p.boxes[active ? p.seg[i] : 0];
  const double xi0 = active ? p.pos[3 * (size_t)i] : 0.0;
  const double xi1 = active ? p.pos[3 * (size_t)i + 1] : 0.0;
  const double xi2 = active ? p.pos[3 * (size_t)i + 2] : 0.0;
  const double ai0 = active ? p.adj[3 * (size_t)i] : 0.0;
  const double ai1 = active ? p.adj[3 * (size_t)i + 1] : 0.0;
  const double ai2 = active ? p.adj[3 * (size_t)i + 2] : 0.0;
  const uint32_t* row = p.nbr + (size_t)(active ? i : 0) * p.cap;
  const int nn = active ? p.nnb[i] : 0;
  const int na = active ? p.nang[i] : 0;
  const double rr2 = p.rr * p.rr, ra2 = p.ra * p.ra;
  const R inv_rr2 = R(p.two_rr), pi_rr = R(p.pi_rr), pi_ra = R(p.pi_ra);
  const R two_ra = R(p.two_ra);

  for (int e = l; e < nn; e += LPA) {
    double d0, d1, d2;
    const int q = entry_disp(p, b, xi0, xi1, xi2, row[e], d0, d1, d2);
    const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
    if (r2 < rr2) {
      const R dx = R(d0), dy = R(d1), dz = R(d2);
      R r, ir;
      len_inv<R>(dx * dx + dy * dy + dz * dz, &r, &ir);
      const R proj = (dx * R(p.adj[3 * (size_t)q] - ai0) + dy * R(p.adj[3 * (size_t)q + 1] - ai1) +
                      dz * R(p.adj[3 * (size_t)q + 2] - ai2)) * ir;
      const R x = r * inv_rr2 - R(1);
      R sn, cs;
      sincos_cut<R>(r, inv_rr2, &sn, &cs);
      const R fc = R(0.5) * (cs + R(1));
      const R fcp = R(-0.5) * pi_rr * sn;
      const R w = R(p.wq[q]);
      R t0 = R(1), t1 = x, u0 = R(1), u1 = R(2) * x;
      rt[0] += fcp * proj;
      rw[0] += w * fcp * proj;
#pragma unroll
      for (int a = 1; a <= NR; ++a) {
        const R dphi = (R(a) * u0 * inv_rr2 * fc + t1 * fcp) * proj;
        rt[a] += dphi;
        rw[a] += w * dphi;
        const R t2 = R(2) * x * t1 - t0;
        t0 = t1;
        t1 = t2;
        const R u2 = R(2) * x * u1 - u0;
        u0 = u1;
        u1 = u2;
      }
    }
  }

  int nv = 0;
  for (int base = 0; base < na; base += LPA) {
    const int e = base + l;
    bool valid = false;
    R vx = 0, vy = 0, vz = 0, vf = 0, vfd = 0, vw = 0, vri = 0, dx_ = 0, dy_ = 0, dz_ = 0, vpa = 0;
    if (e < na) {
      double d0, d1, d2;
      const int q = entry_disp(p, b, xi0, xi1, xi2, row[e], d0, d1, d2);
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      if (r2 < ra2) {
        valid = true;
        R r;
        len_inv<R>(R(d0) * R(d0) + R(d1) * R(d1) + R(d2) * R(d2), &r, &vri);
        vx = R(d0) * vri;
        vy = R(d1) * vri;
        vz = R(d2) * vri;
        dx_ = R(p.adj[3 * (size_t)q] - ai0);
        dy_ = R(p.adj[3 * (size_t)q + 1] - ai1);
        dz_ = R(p.adj[3 * (size_t)q + 2] - ai2);
        vpa = vx * dx_ + vy * dy_ + vz * dz_;
        R sn, cs;
        sincos_cut<R>(r, two_ra, &sn, &cs);
        vf = R(0.5) * (cs + R(1));
        vfd = R(-0.5) * pi_ra * sn * vpa;
        vw = R(p.wq[q]);
      }
    }
    const uint64_t m = group_ballot<LPA>(valid);
    if (valid) {
      const int at_ = nv + __popcll(m & ((1ull << l) - 1ull));
      ux[at_] = vx;
      uy[at_] = vy;
      uz[at_] = vz;
      fs[at_] = vf;
      fd[at_] = vfd;
      ws[at_] = vw;
      ri[at_] = vri;
      vx_[at_] = dx_;
      vy_[at_] = dy_;
      vz_[at_] = dz_;
      pa[at_] = vpa;
    }
    nv += __popcll(m);
  }
  __syncthreads();

  if (nv >= 2) {
    int j = 0, rem = l;
    while (j < nv - 1 && rem >= nv - 1 - j) {
      rem -= nv - 1 - j;
      ++j;
    }
    int k = j + 1 + rem;
    while (j < nv - 1) {
      const R c = ux[j] * ux[k] + uy[j] * uy[k] + uz[j] * uz[k];
      // dc = (u_k . dd_j - c u_j . dd_j)/r_j + (u_j . dd_k - c u_k . dd_k)/r_k
      const R dc = (ux[k] * vx_[j] + uy[k] * vy_[j] + uz[k] * vz_[j] - c * pa[j]) * ri[j] +
                   (ux[j] * vx_[k] + uy[j] * vy_[k] + uz[j] * vz_[k] - c * pa[k]) * ri[k];
      const R ff = fs[j] * fs[k];
      const R dff = fd[j] * fs[k] + fs[j] * fd[k];
      const R ww = ws[j] * ws[k];
      R t0 = R(1), t1 = c, u0 = R(1), u1 = R(2) * c;
      at[0] += dff;
      aw[0] += ww * dff;
#pragma unroll
      for (int a = 1; a <= NA; ++a) {
        const R v = R(a) * u0 * dc * ff + t1 * dff;
        at[a] += v;
        aw[a] += ww * v;
        const R t2 = R(2) * c * t1 - t0;
        t0 = t1;
        t1 = t2;
        const R u2 = R(2) * c * u1 - u0;
        u0 = u1;
        u1 = u2;
      }
      k += LPA;
      while (j < nv - 1 && k >= nv) {
        k = k - nv + j + 2;
        ++j;
      }
    }
  }

#pragma unroll
  for (int a = 0; a <= NR; ++a) {
    rt[a] = group_sum<LPA>(rt[a]);
    rw[a] = group_sum<LPA>(rw[a]);
  }
#pragma unroll
  for (int a = 0; a <= NA; ++a) {
    at[a] = group_sum<LPA>(at[a]) * R(2);
    aw[a] = group_sum<LPA>(aw[a]) * R(2);
  }
  if (active) {
    R* U = reinterpret_cast<R*>(p.U) + (size_t)i * p.ldG;
    constexpr int T1 = NR + 1, T2 = NR + NA + 2;
#pragma unroll
    for (int a = 0; a <= NR; ++a) {
      if (a % LPA == l) U[a] = rt[a];
      if (p.weighted && (T2 + a) % LPA == l) U[T2 + a] = rw[a];
    }
#pragma unroll
    for (int a = 0; a <= NA; ++a) {
      if ((T1 + a) % LPA == l) U[T1 + a] = at[a];
      if (p.weighted && (T2 + T1 + a) % LPA == l) U[T2 + T1 + a] = aw[a];
    }
  }
}

// ------------------------------------------------------------------ dispatch
enum Kind { FWD = 0, BWD = 1, JVP = 2 };

// LDS words (of type R) per angular entry, plus int words
constexpr int lds_words(int kind) { return kind == FWD ? 5 : (kind == BWD ? kBwdArrays : 11); }

template <typename R, int NR, int NA, int LPA>
void launch_kind(int kind, const DescParams& p, hipStream_t s, bool ang) {
  // atoms per block: as many as keep LDS <= 64 KiB and the block <= 256 lanes
  const size_t per_atom = (size_t)p.cap_ang * (lds_words(kind) * sizeof(R) + (kind == BWD ? sizeof(int) : 0));
  int apb = 256 / LPA;
  while (apb > 1 && (size_t)apb * per_atom > 65536) apb >>= 1;
  const size_t lds = (size_t)apb * per_atom;
  const int blocks = (p.n + apb - 1) / apb;
  const dim3 grid(blocks), block(apb * LPA);
  if (kind == FWD && ang) {
    DescParams q = p;
    q.prio = fits_one_round(reinterpret_cast<const void*>(&k_desc_fwd<R, NR, NA, LPA, true>), apb * LPA, lds,
                            blocks);
    hipLaunchKernelGGL((k_desc_fwd<R, NR, NA, LPA, true>), grid, block, lds, s, q);
  } else if (kind == FWD) {
    DescParams q = p;
    q.prio = 0;
    hipLaunchKernelGGL((k_desc_fwd<R, NR, NA, LPA, false>), grid, block, 0, s, q);
  } else {
    hipLaunchKernelGGL((k_desc_jvp<R, NR, NA, LPA>), grid, block, lds, s, p);
  }
}

// the force pass: one wavefront per atom and per block (single-wave blocks
// schedule with the finest grain: measured ~2 % faster than four per block)
template <typename R, int NR, int NA>
void launch_bwd(const DescParams& p, hipStream_t s, bool ext) {
  const size_t per_atom = ((ext ? 0 : bwd_coef_offset<R>(p.cap_ang)) + (size_t)p.n_species * (NR + 1)) * sizeof(R);
  if (p.vir && ext)
    hipLaunchKernelGGL((k_desc_bwd<R, NR, NA, true, true>), dim3(p.n_grid), dim3(64), per_atom, s, p);
  else if (p.vir)
    hipLaunchKernelGGL((k_desc_bwd<R, NR, NA, true, false>), dim3(p.n_grid), dim3(64), per_atom, s, p);
  else if (ext)
    hipLaunchKernelGGL((k_desc_bwd<R, NR, NA, false, true>), dim3(p.n_grid), dim3(64), per_atom, s, p);
  else
    hipLaunchKernelGGL((k_desc_bwd<R, NR, NA, false, false>), dim3(p.n_grid), dim3(64), per_atom, s, p);
}

template <typename R, int NR, int NA>
void launch_orders(int kind, const DescParams& p, hipStream_t s, bool flag) {
  // Lanes per atom from the expected number of angular neighbours within R_a:
  // narrow groups keep the cross-lane reductions short for sparse shells
  // (water: ~30), wide ones give crowded shells (dense amorphous: ~110)
  // enough lanes.  The force pass takes a wavefront per atom.
  if (kind == BWD) {
    launch_bwd<R, NR, NA>(p, s, flag);
    return;
  }
  // (the radial terms alone, flag false in the forward pass, take narrow groups)
  const int na = p.ang_hint > 0 ? p.ang_hint : p.cap_ang;
  if (na > 48 && (kind != FWD || flag))
    launch_kind<R, NR, NA, 64>(kind, p, s, kind != FWD || flag);
  else
    launch_kind<R, NR, NA, 16>(kind, p, s, kind != FWD || flag);
}

template <typename R>
bool dispatch(int kind, int nr, int na, const DescParams& p, hipStream_t s, bool flag) {
#define AENET_CASE(A, B)                       \
  if (nr == A && na == B) {                    \
    launch_orders<R, A, B>(kind, p, s, flag);  \
    return true;                               \
  }
  AENET_ORDERS(AENET_CASE)
#undef AENET_CASE
  return false;
}

void launch_any(int kind, int prec, int nr, int na, const DescParams& p, hipStream_t s, bool flag) {
  if (p.n <= 0) return;
  if (prec == 0)
    dispatch<double>(kind, nr, na, p, s, flag);
  else
    dispatch<float>(kind, nr, na, p, s, flag);
}

}  // namespace

bool fits_one_round(const void* kernel, int threads, size_t lds, int grid) {
  static std::mutex mu;
  static std::map<std::tuple<int, const void*, int, size_t>, int> cache;  // -> resident blocks per device
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  const auto key = std::make_tuple(dev, kernel, threads, lds);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int per_cu = 0, cus = 0;
    // (a failed query only switches the priorities off; its error is cleared)
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, lds) != hipSuccess) {
      per_cu = 0;
      (void)hipGetLastError();
    }
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) {
      cus = 0;
      (void)hipGetLastError();
    }
    it = cache.emplace(key, per_cu * cus).first;
  }
  return grid <= it->second;
}

int desc_supported_list(int* orders, int max_pairs) {
  int k = 0;
#define AENET_LIST(A, B)          \
  if (k < max_pairs && orders) {  \
    orders[2 * k] = A;            \
    orders[2 * k + 1] = B;        \
  }                               \
  ++k;
  AENET_ORDERS(AENET_LIST)
#undef AENET_LIST
  return k;
}

void launch_desc_fwd(int prec, int nr, int na, const DescParams& p, hipStream_t s, bool angular) {
  launch_any(FWD, prec, nr, na, p, s, angular);
}
void launch_desc_bwd(int prec, int nr, int na, const DescParams& p, hipStream_t s, bool ang_ext) {
  launch_any(BWD, prec, nr, na, p, s, ang_ext);
}
void launch_desc_jvp(int prec, int nr, int na, const DescParams& p, hipStream_t s) {
  launch_any(JVP, prec, nr, na, p, s, true);
}

}  // namespace aenet
