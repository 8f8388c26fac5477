// angular.hip -- the angular descriptor of Eq. 6 in factorised form, for
// crowded angular shells.
//
// Eq. 6 sums T_a(cos theta_jk) f_j f_k over ordered pairs of distinct
// neighbours j, k within R_a (and the same with w_j w_k in the weighted
// channel).  Writing T_a in Legendre polynomials, T_a = sum_l C[a][l] P_l, and
// P_l(u_j . u_k) by the addition theorem as a sum over products of functions
// of u_j and of u_k,
//   P_l(u_j . u_k) = sum_{m=0..l} N_lm [c_lm(u_j) c_lm(u_k) + s_lm(u_j) s_lm(u_k)],
//   c_lm + i s_lm = Q_lm(z) (x + i y)^m,  Q_lm = d^m P_l / dz^m,
//   N_lm = (2 - delta_m0) (l - m)! / (l + m)!,
// the pair sum becomes a sum over single neighbours:
//   sum_{j != k} P_l f_j f_k = sum_m N_lm (A_clm^2 + A_slm^2) - sum_j f_j^2,
//   A_clm = sum_j f_j c_lm(u_j),  A_slm = sum_j f_j s_lm(u_j)
// (the j = k terms are f_j^2 since P_l(1) = 1).  The weighted channel takes
// w_j f_j in place of f_j.  The result is Eq. 6 exactly, up to rounding; the
// cost per atom falls from O(n_a^2 (N_a + 1)) to O(n_a (N_a + 1)^2).
//
// A group of lanes per atom (4 or 8): the lanes walk the atom's angular
// entries (the front part of its neighbour row) in strides of the group, each
// keeping the (N_a + 1)^2 partial sums of both channels in its registers.
//   forward:  the sums (group sums by a reduce-scatter), then the
//             2 (N_a + 1) angular components of G; the sums are kept for the
//             force pass;
//   backward: dE/dA = 2 N_lm h_l A (h_l = sum_a C[a][l] dE/dG_ang,a), then per
//             entry j the gradient of the atom's energy with respect to its
//             displacement d_j, stored per row position for the force pass,
//             which adds the radial part and scatters.
// R is double, or float with the displacement taken in double.
#include "desc_dev.h"

namespace aenet {

namespace {

constexpr int kShMaxL = 8;

// T_a = sum_l C[a][l] P_l for a, l <= kShMaxL: T_a in powers of x by its
// recurrence, each power x^k in Legendre polynomials by
// x P_l = ((l + 1) P_{l+1} + l P_{l-1}) / (2l + 1)
struct ChebLeg {
  double c[kShMaxL + 1][kShMaxL + 1];
};
constexpr ChebLeg make_cheb_leg() {
  constexpr int M = kShMaxL + 1;
  double t[M][M] = {};  // t[a][k]: coefficient of x^k in T_a
  t[0][0] = 1.0;
  t[1][1] = 1.0;
  for (int a = 1; a + 1 < M; ++a)
    for (int k = 0; k < M; ++k) t[a + 1][k] = (k > 0 ? 2.0 * t[a][k - 1] : 0.0) - t[a - 1][k];
  double xl[M][M] = {};  // xl[k][l]: coefficient of P_l in x^k
  xl[0][0] = 1.0;
  for (int k = 0; k + 1 < M; ++k)
    for (int l = 0; l < M; ++l) {
      const double v = xl[k][l];
      if (l + 1 < M) xl[k + 1][l + 1] += v * (l + 1) / (2.0 * l + 1.0);
      if (l > 0) xl[k + 1][l - 1] += v * l / (2.0 * l + 1.0);
    }
  ChebLeg out = {};
  for (int a = 0; a < M; ++a)
    for (int l = 0; l < M; ++l) {
      double s = 0.0;
      for (int k = 0; k < M; ++k) s += t[a][k] * xl[k][l];
      out.c[a][l] = s;
    }
  return out;
}
constexpr ChebLeg kChebLeg = make_cheb_leg();

constexpr double sh_norm(int l, int m) {
  double r = m == 0 ? 1.0 : 2.0;
  for (int k = l - m + 1; k <= l + m; ++k) r /= (double)k;
  return r;
}

// Q_lm at its start of column m: Q_mm = (2m - 1)!!
constexpr double dfact(int m) {
  double r = 1.0;
  for (int k = 3; k <= 2 * m - 1; k += 2) r *= (double)k;
  return r;
}

// index of c_lm (m = 0..l) and s_lm (m = 1..l) among the (L+1)^2 functions
constexpr int ci(int l, int m) { return l * l + m; }
constexpr int si(int l, int m) { return l * l + l + m; }

// the displacement-independent part of one angular entry
template <typename R>
struct AngEntry {
  R x, y, z, r, ir, f, fp, w;
  bool valid;
};

template <typename R>
__device__ inline AngEntry<R> ang_entry(const NbrLoad& nl, const BoxInfo& b, double xi0, double xi1,
                                        double xi2, double ra2, R pi_2ra, bool in_row) {
  double d0, d1, d2;
  nbr_disp(nl, b, xi0, xi1, xi2, d0, d1, d2);
  AngEntry<R> a;
  a.valid = in_row && d0 * d0 + d1 * d1 + d2 * d2 < ra2;
  len_inv<R>(R(d0) * R(d0) + R(d1) * R(d1) + R(d2) * R(d2), &a.r, &a.ir);
  a.x = R(d0) * a.ir;
  a.y = R(d1) * a.ir;
  a.z = R(d2) * a.ir;
  R f, fp;
  cutoff_d<R>(a.r, pi_2ra, &f, &fp);
  a.f = a.valid ? f : R(0);
  a.fp = a.valid ? fp : R(0);
  a.w = R(nl.w);
  return a;
}

// The entries of one atom are spread over a group of LPA lanes (entry e on
// lane e mod LPA), so that the lanes of a group read neighbouring words of
// one row and store neighbouring gradients; every lane keeps the partial sums
// of its own entries.  A group's loop runs to the largest angular count of
// the wavefront (a slot past the atom's count is read clamped and weighs 0),
// so every load is unconditional and issued ahead of its use.  LPA per kernel
// and arithmetic type (measured on the 120k-atom Li/Si/O box, against one
// lane per atom): 4 for the FP64 forward pass (its 2 (N_a + 1)^2 sums fill
// the registers, which leaves no room for a wider group's reduction), 8 for
// the others (FP32 forward 455 -> 299 us, backward 1457 -> 942 us with the
// radial force pass; FP64 backward 1550 -> 1387 us).
template <typename R>
constexpr int sh_lanes(bool fwd) {
  return fwd && sizeof(R) == 8 ? 4 : 8;
}

// wavefront-uniform number of entry slots per lane: the largest count of
// the wavefront's atoms, in strides of LPA
template <int LPA>
__device__ inline int wave_strides(int na) {
  int m = na;
#pragma unroll
  for (int o = 32; o >= LPA; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  return __builtin_amdgcn_readfirstlane((m + LPA - 1) / LPA);
}

// forward: the sums of both channels over the atom's angular entries
template <typename R, int NA, int LPA>
__global__ __launch_bounds__(64) void k_ang_sh_fwd(DescParams p) {
  constexpr int NH = (NA + 1) * (NA + 1);
  // the sums: A (typed) at [0, NH), B (weighted) at [NH, 2 NH), the
  // diagonal sums D, Dw at 2 NH and 2 NH + 1, zero up to whole chunks of LPA
  constexpr int NV = 2 * NH + 2;
  constexpr int NC = (NV + LPA - 1) / LPA;
  static_assert(NA <= kShMaxL, "angular order above the factorised table");
  const int g = threadIdx.x / LPA, l = threadIdx.x % LPA;
  const int i0 = blockIdx.x * (64 / LPA) + g;
  const bool active = i0 < p.n;
  const int i = active ? i0 : p.n - 1;
  const BoxInfo b = p.boxes[p.seg[i]];
  const double xi0 = p.pos[3 * (size_t)i], xi1 = p.pos[3 * (size_t)i + 1], xi2 = p.pos[3 * (size_t)i + 2];
  const uint32_t* row = p.nbr + (size_t)i * p.cap;
  const int na = active ? p.nang[i] : 0;
  const double ra2 = p.ra * p.ra;
  const R pi_2ra = R(p.pi_2ra);
  R v[NC * LPA];
#pragma unroll
  for (int k = 0; k < NC * LPA; ++k) v[k] = R(0);
  const int last = na > 0 ? na - 1 : 0;
  const int ns = wave_strides<LPA>(na);
  // (the row word two strides ahead, the neighbour's position one stride)
  NbrLoad nx = load_nbr(p, row[min(l, last)]);
  uint32_t wnext = row[min(l + LPA, last)];
#pragma unroll 1
  for (int t = 0; t < ns; ++t) {
    const int e = l + t * LPA;
    const uint32_t wafter = row[min(e + 2 * LPA, last)];
    const NbrLoad nn = load_nbr(p, wnext);
    const AngEntry<R> a = ang_entry<R>(nx, b, xi0, xi1, xi2, ra2, pi_2ra, e < na);
    nx = nn;
    wnext = wafter;
    const R f = a.f, wf = a.w * a.f;
    v[2 * NH] += f * f;
    v[2 * NH + 1] += wf * wf;
    // (x + i y)^m and the columns Q_lm, l = m..NA, by the three-term
    // recurrence (l - m) Q_lm = (2l - 1) z Q_{l-1,m} - (l + m - 1) Q_{l-2,m}
    R wr = R(1), wi = R(0);
#pragma unroll
    for (int m = 0; m <= NA; ++m) {
      if (m > 0) {
        const R u = wr * a.x - wi * a.y;
        wi = wr * a.y + wi * a.x;
        wr = u;
      }
      R q2 = R(0), q1 = R(dfact(m));
#pragma unroll
      for (int k = m; k <= NA; ++k) {
        R q;
        if (k == m)
          q = q1;
        else
          q = (R(2 * k - 1) * a.z * q1 - R(k + m - 1) * q2) * R(1.0 / (k - m));
        if (k > m) {
          q2 = q1;
          q1 = q;
        }
        const R yc = q * wr;
        v[ci(k, m)] += f * yc;
        v[NH + ci(k, m)] += wf * yc;
        if (m > 0) {
          const R ys = q * wi;
          v[si(k, m)] += f * ys;
          v[NH + si(k, m)] += wf * ys;
        }
      }
    }
  }
  // group sums, LPA components at a time: lane l ends with component
  // c LPA + l of chunk c in own[c]
  R own[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    R t[LPA];
#pragma unroll
    for (int k = 0; k < LPA; ++k) t[k] = v[c * LPA + k];
    group_reduce_scatter<LPA, LPA, R>(t, l);
    own[c] = t[0];
  }
  // keep the sums for the force pass (lanes store neighbouring components)
  R* keep = reinterpret_cast<R*>(p.shA) + (size_t)i * 2 * NH;
#pragma unroll
  for (int c = 0; c < NC; ++c)
    if (active && c * LPA + l < 2 * NH) keep[c * LPA + l] = own[c];
  // S_l = sum_m N_lm (A_clm^2 + A_slm^2) - D per channel: each lane adds the
  // components it holds, then the group sums
  R S[NA + 1], Sw[NA + 1];
#pragma unroll
  for (int k = 0; k <= NA; ++k) S[k] = Sw[k] = R(0);
  R D = R(0), Dw = R(0);
#pragma unroll
  for (int k = 0; k <= NA; ++k)
#pragma unroll
    for (int m = 0; m <= k; ++m) {
      const R nlm = R(sh_norm(k, m));
#pragma unroll
      for (int h = 0; h < (m > 0 ? 2 : 1); ++h) {
        const int cc = h == 0 ? ci(k, m) : si(k, m);
        const R va = own[cc / LPA], vb = own[(NH + cc) / LPA];
        S[k] += l == cc % LPA ? nlm * va * va : R(0);
        Sw[k] += l == (NH + cc) % LPA ? nlm * vb * vb : R(0);
      }
    }
  D = l == (2 * NH) % LPA ? own[(2 * NH) / LPA] : R(0);
  Dw = l == (2 * NH + 1) % LPA ? own[(2 * NH + 1) / LPA] : R(0);
#pragma unroll
  for (int k = 0; k <= NA; ++k) {
    S[k] = group_sum<LPA>(S[k]);
    Sw[k] = group_sum<LPA>(Sw[k]);
  }
  D = group_sum<LPA>(D);
  Dw = group_sum<LPA>(Dw);
  // lane a mod LPA of the group writes component a of both halves
  R* G = reinterpret_cast<R*>(p.G) + (size_t)i * p.ldG;
  const int at = p.t1;         // first angular component, typed half
  const int aw = p.t1 + p.t2;  // first angular component, weighted half
#pragma unroll
  for (int a = 0; a <= NA; ++a) {
    R gt = R(0), gw = R(0);
#pragma unroll
    for (int k = 0; k <= a; ++k) {
      gt += R(kChebLeg.c[a][k]) * (S[k] - D);
      gw += R(kChebLeg.c[a][k]) * (Sw[k] - Dw);
    }
    if (active && l == a % LPA) {
      G[at + a] = gt;
      if (p.weighted) G[aw + a] = gw;
    }
  }
}

// backward: dE_i/dd_e of the angular part for every angular entry e of atom i
template <typename R, int NA, int LPA>
__global__ __launch_bounds__(64) void k_ang_sh_bwd(DescParams p) {
  constexpr int NH = (NA + 1) * (NA + 1);
  const int g = threadIdx.x / LPA, l = threadIdx.x % LPA;
  const int i0 = blockIdx.x * (64 / LPA) + g;
  const bool active = i0 < p.n;
  const int i = active ? i0 : p.n - 1;
  const BoxInfo b = p.boxes[p.seg[i]];
  const double xi0 = p.pos[3 * (size_t)i], xi1 = p.pos[3 * (size_t)i + 1], xi2 = p.pos[3 * (size_t)i + 2];
  const uint32_t* row = p.nbr + (size_t)i * p.cap;
  const int na = active ? p.nang[i] : 0;
  const double ra2 = p.ra * p.ra;
  const R pi_2ra = R(p.pi_2ra);
  // h_l = sum_a C[a][l] dE/dG_ang,a (both channels), H = sum_l h_l
  const R* gG = reinterpret_cast<const R*>(p.gG) + (size_t)i * p.ldG;
  R h[NA + 1], hw[NA + 1];
  R H = R(0), Hw = R(0);
  {
    R gt[NA + 1], gw[NA + 1];
#pragma unroll
    for (int a = 0; a <= NA; ++a) {
      gt[a] = gG[p.t1 + a];
      gw[a] = p.weighted ? gG[p.t1 + p.t2 + a] : R(0);
    }
#pragma unroll
    for (int k = 0; k <= NA; ++k) {
      R s = R(0), sw = R(0);
#pragma unroll
      for (int a = k; a <= NA; ++a) {
        s += R(kChebLeg.c[a][k]) * gt[a];
        sw += R(kChebLeg.c[a][k]) * gw[a];
      }
      h[k] = s;
      hw[k] = sw;
      H += s;
      Hw += sw;
    }
  }
  // coefficients of each function: qt = 2 N_lm h_l A_lm, qw = 2 N_lm hw_l B_lm;
  // an entry of weight w has q = qt + w qw (every lane of the group reads
  // the atom's sums)
  R qt[NH], qw[NH];
  {
    const R* keep = reinterpret_cast<const R*>(p.shA) + (size_t)i * 2 * NH;
#pragma unroll
    for (int k = 0; k <= NA; ++k)
#pragma unroll
      for (int m = 0; m <= k; ++m) {
        const R c2 = R(2.0 * sh_norm(k, m));
        qt[ci(k, m)] = c2 * h[k] * keep[ci(k, m)];
        qw[ci(k, m)] = c2 * hw[k] * keep[NH + ci(k, m)];
        if (m > 0) {
          qt[si(k, m)] = c2 * h[k] * keep[si(k, m)];
          qw[si(k, m)] = c2 * hw[k] * keep[NH + si(k, m)];
        }
      }
  }
  R* out = reinterpret_cast<R*>(p.gang) + (size_t)i * p.cap_ang * 3;
  const int last = na > 0 ? na - 1 : 0;
  const int ns = wave_strides<LPA>(na);
  // (the row word two strides ahead, the neighbour's position one stride)
  NbrLoad nx = load_nbr(p, row[min(l, last)]);
  uint32_t wnext = row[min(l + LPA, last)];
#pragma unroll 1
  for (int t = 0; t < ns; ++t) {
    const int e = l + t * LPA;
    const uint32_t wafter = row[min(e + 2 * LPA, last)];
    const NbrLoad nn = load_nbr(p, wnext);
    const AngEntry<R> a = ang_entry<R>(nx, b, xi0, xi1, xi2, ra2, pi_2ra, e < na);
    nx = nn;
    wnext = wafter;
    // V = sum q Y and the gradient G = sum q grad Y of the functions as
    // polynomials in (x, y, z): d/dx (x+iy)^m = m (x+iy)^(m-1),
    // d/dy (x+iy)^m = i m (x+iy)^(m-1), dQ_lm/dz = Q_l,m+1
    // V and the gradient are summed per column m (independent chains; one
    // chain through all (N_a + 1)^2 terms would serialise the column loop)
    R V = R(0), gx = R(0), gy = R(0), gz = R(0);
    R wr = R(1), wi = R(0), pr = R(0), pi = R(0);  // (x+iy)^m and (x+iy)^(m-1)
#pragma unroll
    for (int m = 0; m <= NA; ++m) {
      R Vm = R(0), gxm = R(0), gym = R(0), gzm = R(0);
      if (m > 0) {
        pr = wr;
        pi = wi;
        const R u = wr * a.x - wi * a.y;
        wi = wr * a.y + wi * a.x;
        wr = u;
      }
      // columns m and m + 1 of Q together
      R q2 = R(0), q1 = R(dfact(m));      // column m
      R u2 = R(0), u1 = R(dfact(m + 1));  // column m + 1
#pragma unroll
      for (int k = m; k <= NA; ++k) {
        R q;
        if (k == m)
          q = q1;
        else
          q = (R(2 * k - 1) * a.z * q1 - R(k + m - 1) * q2) * R(1.0 / (k - m));
        if (k > m) {
          q2 = q1;
          q1 = q;
        }
        R u = R(0);  // Q_k,m+1
        if (k == m + 1) {
          u = u1;
        } else if (k > m + 1) {
          u = (R(2 * k - 1) * a.z * u1 - R(k + m) * u2) * R(1.0 / (k - m - 1));
          u2 = u1;
          u1 = u;
        }
        const R qc = qt[ci(k, m)] + a.w * qw[ci(k, m)];
        const R qs = m > 0 ? qt[si(k, m)] + a.w * qw[si(k, m)] : R(0);
        const R cw = qc * wr + qs * wi;
        Vm += q * cw;
        gzm += u * cw;
        if (m > 0) {
          const R qm = q * R(m);
          gxm += qm * (qc * pr + qs * pi);
          gym += qm * (qs * pr - qc * pi);
        }
      }
      V += Vm;
      gx += gxm;
      gy += gym;
      gz += gzm;
    }
    // d/dd of f(r) Y(d/r) = f' Y u + (f / r) (grad Y - (u . grad Y) u),
    // minus the diagonal terms 2 f f' (H + w^2 Hw) u
    const R ug = a.x * gx + a.y * gy + a.z * gz;
    const R tr = a.f * a.ir;
    const R radial = a.fp * V - tr * ug - R(2) * a.f * a.fp * (H + a.w * a.w * Hw);
    const R ox = radial * a.x + tr * gx, oy = radial * a.y + tr * gy, oz = radial * a.z + tr * gz;
    if (e < na) {
      out[3 * e] = a.valid ? ox : R(0);
      out[3 * e + 1] = a.valid ? oy : R(0);
      out[3 * e + 2] = a.valid ? oz : R(0);
    }
  }
}

template <typename R, int NA>
void launch_na(bool fwd, const DescParams& p, hipStream_t s) {
  constexpr int lf = sh_lanes<R>(true), lb = sh_lanes<R>(false);
  if (fwd)
    hipLaunchKernelGGL((k_ang_sh_fwd<R, NA, lf>), dim3((p.n + 64 / lf - 1) / (64 / lf)), dim3(64), 0, s, p);
  else
    hipLaunchKernelGGL((k_ang_sh_bwd<R, NA, lb>), dim3((p.n + 64 / lb - 1) / (64 / lb)), dim3(64), 0, s, p);
}

template <typename R>
bool launch_r(bool fwd, int na, const DescParams& p, hipStream_t s) {
  switch (na) {
    case 2: launch_na<R, 2>(fwd, p, s); return true;
    case 3: launch_na<R, 3>(fwd, p, s); return true;
    case 4: launch_na<R, 4>(fwd, p, s); return true;
    case 6: launch_na<R, 6>(fwd, p, s); return true;
    case 8: launch_na<R, 8>(fwd, p, s); return true;
    default: return false;
  }
}

}  // namespace

size_t ang_sh_terms(int na) { return (size_t)(na + 1) * (na + 1); }

bool launch_ang_sh(bool fwd, int prec, int na, const DescParams& p, hipStream_t s) {
  if (p.n <= 0) return true;
  return prec == 0 ? launch_r<double>(fwd, na, p, s) : launch_r<float>(fwd, na, p, s);
}

}  // namespace aenet
