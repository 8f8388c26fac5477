// desc_dev.h -- device code shared by the descriptor kernels and the fused
// descriptor + network kernel: cross-lane reductions, the cosine cutoff
// (Eq. 5), neighbour loads, Chebyshev series, and the forward pass of one
// atom's descriptor (Eqs. 3-6).
#pragma once
#include "aenet_internal.h"

// (radial order, angular order) pairs compiled in; every descriptor kernel
// is instantiated for each pair.  A model of other orders runs on the
// smallest pair that reaches both of them (its descriptor is a subset of that
// pair's); the last two pairs are there to reach orders up to 24 / 12.
#define AENET_ORDERS(X) \
  X(10, 4)              \
  X(16, 8)              \
  X(18, 6)              \
  X(6, 2)               \
  X(5, 3)               \
  X(4, 2)               \
  X(20, 10)             \
  X(24, 12)

namespace aenet {

namespace {

template <int LPA, typename T>
__device__ inline T group_sum(T v) {
#pragma unroll
  for (int o = LPA / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, LPA);
  return v;
}

template <int LPA>
__device__ inline uint64_t group_ballot(bool pred) {
  const uint64_t m = __ballot(pred);
  if (LPA == 64) return m;
  const int g = (threadIdx.x & 63) / LPA;
  return (m >> (g * LPA)) & ((1ull << LPA) - 1ull);
}

// Reduce-scatter over a group of LPA lanes: on entry every lane holds N
// partial sums v[0..N) (N a power of two); on exit lane l holds the group sum
// of component rs_comp<LPA, N>(l, i) in v[i] for i < max(N / LPA, 1).  Each
// halving step sends the half the lane gives up to its partner, so about N
// values cross lanes instead of N log2(LPA) for a full butterfly.  When
// N < LPA the lanes that differ above bit log2(N) first add their vectors,
// and lanes l and l + N end with the same component.
template <int LPA, int N, typename T>
__device__ inline void group_reduce_scatter(T (&v)[N], int l) {
  if constexpr (LPA > N) {
#pragma unroll
    for (int mask = LPA / 2; mask >= N; mask >>= 1)
#pragma unroll
      for (int k = 0; k < N; ++k) v[k] += __shfl_xor(v[k], mask, LPA);
  }
  constexpr int W = LPA < N ? LPA : N;
#pragma unroll
  for (int mask = W / 2, h = N / 2; mask > 0; mask >>= 1, h >>= 1) {
    const bool up = (l & mask) != 0;
#pragma unroll
    for (int k = 0; k < h; ++k) {
      // the empty asm hides where lo and hi come from, so the selects stay
      // selects of values (not a load at a lane-dependent index, which would
      // put v in scratch memory)
      T lo = v[k], hi = v[k + h];
      asm volatile("" : "+v"(lo), "+v"(hi));
      const T send = up ? lo : hi;
      const T keep = up ? hi : lo;
      v[k] = keep + __shfl_xor(send, mask, LPA);
    }
  }
}

template <int LPA, int N>
__device__ inline int rs_comp(int l, int i) {
  constexpr int W = LPA < N ? LPA : N;
  return (N / W) * (l % W) + i;
}

constexpr int pow2_at_least(int x) { return x <= 1 ? 1 : 2 * pow2_at_least((x + 1) / 2); }

// r = |d| and 1/r from r2 = |d|^2 > 0: the hardware reciprocal square root
// estimate y refined by Newton's iteration for 1/sqrt, y <- y (3 - r2 y^2)/2,
// which squares the relative error at each step (two steps in double, one in
// float, leave a few units in the last place), then r = r2 y.
template <typename R>
__device__ inline void len_inv(R r2, R* r, R* ir);
template <>
__device__ inline void len_inv<double>(double r2, double* r, double* ir) {
  const double h = 0.5 * r2;
  double y = __builtin_amdgcn_rsq(r2);
  y = y * (1.5 - h * (y * y));
  y = y * (1.5 - h * (y * y));
  *ir = y;
  *r = r2 * y;
}
template <>
__device__ inline void len_inv<float>(float r2, float* r, float* ir) {
  float y = __builtin_amdgcn_rsqf(r2);
  y = y * (1.5f - 0.5f * r2 * (y * y));
  *ir = y;
  *r = r2 * y;
}

// Taylor coefficient of t^n in sin t (n odd) or cos t (n even): +-1/n!
constexpr double taylor_sc(int n) {
  double f = 1.0;
  for (int k = 2; k <= n; ++k) f /= k;
  return (n / 2) % 2 ? -f : f;
}

// sum_{k=0..K} taylor_sc(N0 + 2k) u^k by Horner's scheme (one fused
// multiply-add per term, coefficients fixed at compile time)
template <typename R, int N0, int K>
__device__ inline R taylor_poly(R u) {
  constexpr double c = taylor_sc(N0);
  if constexpr (K == 0)
    return R(c);
  else
    return taylor_poly<R, N0 + 2, K - 1>(u) * u + R(c);
}

// sin t and cos t for |t| <= pi/2 by their Taylor series in u = t^2; the
// first omitted term is below 2e-18 (double: terms to t^21 / t^22) or 7e-10
// (float: to t^13 / t^14).
template <typename R>
__device__ inline void sincos_halfpi(R t, R* s, R* c) {
  constexpr bool dbl = sizeof(R) == 8;
  const R u = t * t;
  const R ps = dbl ? taylor_poly<R, 3, 9>(u) : taylor_poly<R, 3, 5>(u);
  const R pc = dbl ? taylor_poly<R, 2, 10>(u) : taylor_poly<R, 2, 6>(u);
  *s = (t * u) * ps + t;
  *c = u * pc + R(1);
}

// sin and cos of pi r / R for 0 <= r < R (the cosine cutoff, Eq. 5): with
// x = 2r/R - 1 in [-1, 1) and t = pi x / 2, pi r / R = t + pi/2, so
// sin(pi r/R) = cos t and cos(pi r/R) = -sin t.
template <typename R>
__device__ inline void sincos_cut(R r, R two_over_R, R* sn, R* cs) {
  const R t = R(0.5 * kPi) * (r * two_over_R - R(1));
  R st, ct;
  sincos_halfpi<R>(t, &st, &ct);
  *sn = ct;
  *cs = -st;
}

// The cosine cutoff (Eq. 5) and its derivative for 0 <= r < R,
// f_c = (1 + cos(pi r/R))/2 and f_c' = -(pi/(2R)) sin(pi r/R), from sin and
// cos of psi = pi r/(2R) - pi/4 in [-pi/4, pi/4) (Taylor series to psi^15 /
// psi^16 in double, psi^9 / psi^10 in float; the first omitted term is below
// 5e-17 or 2e-9): pi r/R = 2 psi + pi/2 gives f_c = 1/2 - sin psi cos psi and
// f_c' = -(pi/(2R)) (cos psi - sin psi)(cos psi + sin psi).
template <typename R>
__device__ inline void cutoff_d(R r, R pi_2R, R* fc, R* dfc) {
  constexpr bool dbl = sizeof(R) == 8;
  const R psi = r * pi_2R - R(0.25 * kPi);
  const R u = psi * psi;
  const R ps = dbl ? taylor_poly<R, 3, 6>(u) : taylor_poly<R, 3, 3>(u);
  const R pc = dbl ? taylor_poly<R, 2, 7>(u) : taylor_poly<R, 2, 4>(u);
  const R sn = (psi * u) * ps + psi;
  const R cs = u * pc + R(1);
  *fc = R(0.5) - sn * cs;
  *dfc = -pi_2R * ((cs - sn) * (cs + sn));
}

// displacement d = r_j + s L - r_i of a packed entry (always in double)
__device__ inline int entry_disp(const DescParams& p, const BoxInfo& b, double xi0, double xi1,
                                 double xi2, uint32_t en, double& d0, double& d1, double& d2) {
  const int q = (int)(en & kAtomMask);
  const int code = (int)(en >> kImgBits);
  const double s0 = (double)(code % 3 - 1), s1 = (double)((code / 3) % 3 - 1), s2 = (double)(code / 9 - 1);
  d0 = p.pos[3 * (size_t)q] + s0 * b.L[0] - xi0;
  d1 = p.pos[3 * (size_t)q + 1] + s1 * b.L[1] - xi1;
  d2 = p.pos[3 * (size_t)q + 2] + s2 * b.L[2] - xi2;
  return q;
}

// A neighbour entry with its atom's position loaded (issued one loop
// iteration ahead of its use so the gather latency hides behind the
// arithmetic of the current iteration).
struct NbrLoad {
  int code, sp;       // image code; species of the neighbour atom
  double x, y, z, w;  // position and species weight of the neighbour atom
};

__device__ inline NbrLoad load_nbr(const DescParams& p, uint32_t word) {
  NbrLoad n;
  // clamped, so that a slot read past the end of a row (whose value is not
  // used) stays inside the arrays
  const int q = min((int)(word & kAtomMask), p.n - 1);
  n.code = (int)(word >> kImgBits);
  n.x = p.pos[3 * (size_t)q];
  n.y = p.pos[3 * (size_t)q + 1];
  n.z = p.pos[3 * (size_t)q + 2];
  n.w = p.wq[q];
  n.sp = p.species[q];
  return n;
}

__device__ inline void nbr_disp(const NbrLoad& n, const BoxInfo& b, double xi0, double xi1, double xi2,
                                double& d0, double& d1, double& d2) {
  d0 = n.x + (double)(n.code % 3 - 1) * b.L[0] - xi0;
  d1 = n.y + (double)((n.code / 3) % 3 - 1) * b.L[1] - xi1;
  d2 = n.z + (double)(n.code / 9 - 1) * b.L[2] - xi2;
}

// S(x) = sum_{a=0..N} c_a T_a(x) and S'(x) by Clenshaw's recurrence, with
// c_a = g[a] + w h[a] (the typed and weighted coefficients of one neighbour
// or pair combined on the fly): b_a = c_a + 2x b_{a+1} - b_{a+2} and its
// x-derivative b'_a = 2 b_{a+1} + 2x b'_{a+1} - b'_{a+2}, from
// b_{N+1} = b_{N+2} = 0; then S = c_0 + x b_1 - b_2, S' = b_1 + x b'_1 - b'_2.
// Five operations per order and only g, h live (instead of the values and
// derivatives of both channels kept by forward recurrences).
template <typename R, int N>
__device__ inline void cheb_series_d(const R (&g)[N + 1], const R (&h)[N + 1], R w, R x, R* S,
                                     R* dS) {
  static_assert(N >= 2, "series of order >= 2");
  const R x2 = x + x;
  // the steps a = N and N - 1 written out: b_N = c_N, b'_N = 0,
  // b_{N-1} = 2x c_N + c_{N-1}, b'_{N-1} = 2 c_N (no terms with the zero
  // starting values left for the hardware to multiply)
  R b2 = w * h[N] + g[N];
  R b1 = x2 * b2 + (w * h[N - 1] + g[N - 1]);
  R d2 = R(0);
  R d1 = R(2) * b2;
#pragma unroll
  for (int a = N - 2; a >= 1; --a) {
    // (w h_a - b2) + g_a: each operation reads at most one wave-uniform
    // coefficient, so none has to be copied out of the scalar registers
    const R bk = x2 * b1 + ((w * h[a] - b2) + g[a]);
    const R dk = x2 * d1 + (R(2) * b1 - d2);
    b2 = b1;
    b1 = bk;
    d2 = d1;
    d1 = dk;
  }
  *S = x * b1 + ((g[0] + w * h[0]) - b2);
  *dS = x * d1 + (b1 - d2);
}

// The same with the coefficients c_0..c_N read from c (LDS): four operations
// per order.
template <typename R, int N>
__device__ inline void cheb_series_tab(const R* c, R x, R* S, R* dS) {
  static_assert(N >= 2, "series of order >= 2");
  const R x2 = x + x;
  R b2 = c[N];
  R b1 = x2 * b2 + c[N - 1];
  R d2 = R(0);
  R d1 = R(2) * b2;
#pragma unroll
  for (int a = N - 2; a >= 1; --a) {
    const R bk = x2 * b1 + (c[a] - b2);
    const R dk = x2 * d1 + (R(2) * b1 - d2);
    b2 = b1;
    b1 = bk;
    d2 = d1;
    d1 = dk;
  }
  *S = x * b1 + (c[0] - b2);
  *dS = x * d1 + (b1 - d2);
}

// ------------------------------------------------------------------ forward
// Descriptor vector of atom i by group g (lanes l = 0..LPA-1) of the block;
// the group's compaction buffers are at smem + g * 5 * cap_ang elements.  Every
// group of the block must call it (it holds a block barrier).  The G
// components are handed to out(c, value) (c < D, one lane per component).
// ANG = false: the radial terms only (the angular components are handed out
// as zero, for the factorised angular kernel to overwrite).
template <typename R, int NR, int NA, int LPA, typename Out, bool ANG = true>
__device__ inline void desc_fwd_group(const DescParams& p, int i, bool active, int g, int l,
                                      unsigned char* smem, Out&& out) {
  R* ux = reinterpret_cast<R*>(smem) + (size_t)g * p.cap_ang * 5;
  R* uy = ux + p.cap_ang;
  R* uz = uy + p.cap_ang;
  R* fs = uz + p.cap_ang;
  R* ws = fs + p.cap_ang;

  R rt[NR + 1], rw[NR + 1], at[NA + 1], aw[NA + 1];
#pragma unroll
  for (int a = 0; a <= NR; ++a) rt[a] = rw[a] = R(0);
#pragma unroll
  for (int a = 0; a <= NA; ++a) at[a] = aw[a] = R(0);

  // an inactive group reads atom 0 and uses none of it (unconditional loads
  // are issued together; loads under a branch one after another)
  const int ic = active ? i : 0;
  const BoxInfo b = p.boxes[p.seg[ic]];
  const double xi0 = p.pos[3 * (size_t)ic];
  const double xi1 = p.pos[3 * (size_t)ic + 1];
  const double xi2 = p.pos[3 * (size_t)ic + 2];
  const uint32_t* row = p.nbr + (size_t)ic * p.cap;
  const int nn_ld = p.nnb[ic], na_ld = p.nang[ic];
  const int nn = active ? nn_ld : 0;
  const int na = active ? na_ld : 0;
  const double rr2 = p.rr * p.rr, ra2 = p.ra * p.ra;
  const R inv_rr2 = R(p.two_rr), pi_rr = R(p.pi_rr), pi_ra = R(p.pi_ra);
  const R two_ra = R(p.two_ra);

  // radial terms, Eq. 3.  Two entries per lane per iteration give two
  // independent recurrence chains; entries beyond R_r (skin) or past the end
  // of the row are computed with weight 0 instead of branching.
  // slots past the end of the row repeat its last entry (an empty row reads
  // slot 0, whatever it holds) and are given weight 0
  auto word = [&](int e) { return row[e < nn ? e : max(nn - 1, 0)]; };
  NbrLoad na_ = load_nbr(p, word(l)), nb_ = load_nbr(p, word(l + LPA));
  uint32_t wa1 = word(l + 2 * LPA), wb1 = word(l + 3 * LPA);
  // for the force pass and the gather: the contributing entries from the
  // front of ridx, the margin entries from the back (see DescParams)
  uint16_t* ridx = p.ridx + (size_t)ic * p.cap;
  const double rr2m = rr2 * (1.0 + 1e-9);
  int n_keep = 0, n_marg = 0;
  for (int e = l; e < nn; e += 2 * LPA) {
    const NbrLoad na1 = load_nbr(p, wa1), nb1 = load_nbr(p, wb1);
    const uint32_t wa2 = word(e + 4 * LPA), wb2 = word(e + 5 * LPA);
    const bool hb = e + LPA < nn;
    double a0, a1, a2, b0, b1, b2;
    nbr_disp(na_, b, xi0, xi1, xi2, a0, a1, a2);
    nbr_disp(nb_, b, xi0, xi1, xi2, b0, b1, b2);
    const R twa = R(na_.w), twb = R(nb_.w);
    na_ = na1;
    nb_ = nb1;
    wa1 = wa2;
    wb1 = wb2;
    const double ra2_ = a0 * a0 + a1 * a1 + a2 * a2, rb2_ = b0 * b0 + b1 * b1 + b2 * b2;
    const bool va = ra2_ < rr2;
    const bool vb = hb && (rb2_ < rr2);
    {
      const bool ka = va || e < na, kb = hb && (vb || e + LPA < na);
      const bool sa = !ka && ra2_ < rr2m, sb = hb && !kb && rb2_ < rr2m;
      const uint64_t ma = group_ballot<LPA>(ka), mb = group_ballot<LPA>(kb);
      const uint64_t za = group_ballot<LPA>(sa), zb = group_ballot<LPA>(sb);
      const uint64_t below = (1ull << l) - 1ull;
      if (ka) ridx[n_keep + __popcll(ma & below)] = (uint16_t)e;
      if (kb) ridx[n_keep + __popcll(ma) + __popcll(mb & below)] = (uint16_t)(e + LPA);
      if (sa) ridx[p.cap - 1 - (n_marg + __popcll(za & below))] = (uint16_t)e;
      if (sb) ridx[p.cap - 1 - (n_marg + __popcll(za) + __popcll(zb & below))] = (uint16_t)(e + LPA);
      n_keep += __popcll(ma) + __popcll(mb);
      n_marg += __popcll(za) + __popcll(zb);
    }
    R ra, rb, ira, irb;
    len_inv<R>(R(a0) * R(a0) + R(a1) * R(a1) + R(a2) * R(a2), &ra, &ira);
    len_inv<R>(R(b0) * R(b0) + R(b1) * R(b1) + R(b2) * R(b2), &rb, &irb);
    const R xa = ra * inv_rr2 - R(1), xb = rb * inv_rr2 - R(1);
    R sna, csa, snb, csb;
    sincos_cut<R>(ra, inv_rr2, &sna, &csa);
    sincos_cut<R>(rb, inv_rr2, &snb, &csb);
    const R fa = va ? R(0.5) * (csa + R(1)) : R(0);
    const R fb = vb ? R(0.5) * (csb + R(1)) : R(0);
    const R wa = twa * fa, wb = twb * fb;
    R ta0 = R(1), ta1 = xa, tb0 = R(1), tb1 = xb;
    rt[0] += fa + fb;
    rw[0] += wa + wb;
#pragma unroll
    for (int a = 1; a <= NR; ++a) {
      rt[a] += ta1 * fa + tb1 * fb;
      rw[a] += ta1 * wa + tb1 * wb;
      const R ta2 = R(2) * xa * ta1 - ta0;
      const R tb2 = R(2) * xb * tb1 - tb0;
      ta0 = ta1;
      ta1 = ta2;
      tb0 = tb1;
      tb1 = tb2;
    }
  }

  if (active && l == 0) p.nrad[i] = n_keep | (n_marg << 16);

  // With p.prio (set where every block of the grid is resident at once) the
  // wave priority falls phase by phase (radial 3, angular 2, reduction 1,
  // network 0): of the blocks sharing a CU, which all start together, the
  // ones behind get the issue slots, so they finish close together instead
  // of the last one running alone at the end.  (Where blocks arrive over
  // several rounds, new blocks would starve the old ones.)
  if (p.prio) __builtin_amdgcn_s_setprio(2);

  // compact the angular entries into LDS
  int nv = 0;
  for (int base = 0; ANG && base < na; base += LPA) {
    const int e = base + l;
    bool valid = false;
    R vx = 0, vy = 0, vz = 0, vf = 0, vw = 0;
    if (e < na) {
      double d0, d1, d2;
      const int q = entry_disp(p, b, xi0, xi1, xi2, row[e], d0, d1, d2);
      const double r2 = d0 * d0 + d1 * d1 + d2 * d2;
      if (r2 < ra2) {
        valid = true;
        R r, ir;
        len_inv<R>(R(d0) * R(d0) + R(d1) * R(d1) + R(d2) * R(d2), &r, &ir);
        vx = R(d0) * ir;
        vy = R(d1) * ir;
        vz = R(d2) * ir;
        R sn, cs;
        sincos_cut<R>(r, two_ra, &sn, &cs);
        vf = R(0.5) * (cs + R(1));
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
      ws[at_] = vw;
    }
    nv += __popcll(m);
  }
  if (ANG) __syncthreads();

  // angular terms, Eq. 6, over the unordered pairs {e, (e + t) mod nv},
  // t = 1..floor(nv/2) (for even nv the pairs at t = nv/2 are counted from
  // e < nv/2 only): the lane owning entry e (entries l, l + LPA, ...) keeps
  // it in registers and reads the partners from LDS, two steps per iteration
  // (the second with weight 0 past the last step)
  {
    const int T = nv >> 1;
    for (int e = l; e < nv; e += LPA) {
      const R kx = ux[e], ky = uy[e], kz = uz[e], fk = fs[e], wk = ws[e];
      int m = e;
      for (int t = 1; t <= T; t += 2) {
        const int ma = m + 1 == nv ? 0 : m + 1;
        const int mb = ma + 1 == nv ? 0 : ma + 1;
        m = mb;
        const bool hb = t + 1 <= T;
        const R ca = ux[ma] * kx + uy[ma] * ky + uz[ma] * kz;
        const R cb = ux[mb] * kx + uy[mb] * ky + uz[mb] * kz;
        const R fa = (2 * t != nv || e < t) ? fk * fs[ma] : R(0);
        const R fb = (hb && (2 * (t + 1) != nv || e < t + 1)) ? fk * fs[mb] : R(0);
        const R wa = wk * ws[ma] * fa, wb = wk * ws[mb] * fb;
        R ta0 = R(1), ta1 = ca, tb0 = R(1), tb1 = cb;
        at[0] += fa + fb;
        aw[0] += wa + wb;
#pragma unroll
        for (int a = 1; a <= NA; ++a) {
          at[a] += ta1 * fa + tb1 * fb;
          aw[a] += ta1 * wa + tb1 * wb;
          const R ta2 = R(2) * ca * ta1 - ta0;
          const R tb2 = R(2) * cb * tb1 - tb0;
          ta0 = ta1;
          ta1 = ta2;
          tb0 = tb1;
          tb1 = tb2;
        }
      }
    }
  }

  if (p.prio) __builtin_amdgcn_s_setprio(1);
  // G layout [rad_typ | ang_typ | rad_wt | ang_wt] (ordered angular pairs =
  // 2 x unordered).  Each half (typed, weighted) is packed into a vector of
  // NV = 2^k >= T2 partial sums and reduce-scattered over the group on its
  // own, so only one such vector is live at a time.
  constexpr int T1 = NR + 1, T2 = NR + NA + 2;
  constexpr int NV = pow2_at_least(T2);
  constexpr int PER = NV / LPA > 0 ? NV / LPA : 1;
  const bool writer = active && l < NV;
  {
    R v[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) v[a] = a <= NR ? rt[a] : (a < T2 ? R(2) * at[a - T1] : R(0));
    group_reduce_scatter<LPA, NV, R>(v, l);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = rs_comp<LPA, NV>(l, k);
      if (writer && c < T2) out(c, v[k]);
    }
  }
  if (p.weighted) {
    R v[NV];
#pragma unroll
    for (int a = 0; a < NV; ++a) v[a] = a <= NR ? rw[a] : (a < T2 ? R(2) * aw[a - T1] : R(0));
    group_reduce_scatter<LPA, NV, R>(v, l);
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int c = rs_comp<LPA, NV>(l, k);
      if (writer && c < T2) out(T2 + c, v[k]);
    }
  }
}

}  // namespace

}  // namespace aenet
