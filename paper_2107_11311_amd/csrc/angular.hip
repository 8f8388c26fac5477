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
// One lane per atom: the (N_a + 1)^2 sums of both channels live in its
// registers, and the lane walks the atom's angular entries (the front part of
// its neighbour row), one per iteration, the loads of the next two issued
// ahead.
//   forward:  the sums, then the 2 (N_a + 1) angular components of G; the
//             sums are kept for the force pass;
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

// forward: the sums of both channels over the atom's angular entries
template <typename R, int NA>
__global__ __launch_bounds__(64) void k_ang_sh_fwd(DescParams p) {
  constexpr int NH = (NA + 1) * (NA + 1);
  static_assert(NA <= kShMaxL, "angular order above the factorised table");
  const int i0 = blockIdx.x * 64 + threadIdx.x;
  const bool active = i0 < p.n;
  const int i = active ? i0 : p.n - 1;
  const BoxInfo b = p.boxes[p.seg[i]];
  const double xi0 = p.pos[3 * (size_t)i], xi1 = p.pos[3 * (size_t)i + 1], xi2 = p.pos[3 * (size_t)i + 2];
  const uint32_t* row = p.nbr + (size_t)i * p.cap;
  const int na = active ? p.nang[i] : 0;
  const double ra2 = p.ra * p.ra;
  const R pi_2ra = R(p.pi_2ra);
  R A[NH], B[NH];
#pragma unroll
  for (int k = 0; k < NH; ++k) A[k] = B[k] = R(0);
  R D = R(0), Dw = R(0);
  // The entries' two dependent loads (row word, then the neighbour's
  // position) run two and one entries ahead of their use, so that no
  // iteration waits on a load it issued itself; slots past the end repeat
  // the last entry (an empty row reads slot 0, whatever it holds, with
  // weight 0).
  const int last = na > 0 ? na - 1 : 0;
  NbrLoad nx = load_nbr(p, row[0]);
  uint32_t wnext = row[min(1, last)];
  for (int e = 0; e < na; ++e) {
    const uint32_t wafter = row[min(e + 2, last)];
    const NbrLoad nn = load_nbr(p, wnext);
    const AngEntry<R> a = ang_entry<R>(nx, b, xi0, xi1, xi2, ra2, pi_2ra, true);
    nx = nn;
    wnext = wafter;
    const R f = a.f, wf = a.w * a.f;
    D += f * f;
    Dw += wf * wf;
    // (x + i y)^m and the columns Q_lm, l = m..NA, by the three-term
    // recurrence (l - m) Q_lm = (2l - 1) z Q_{l-1,m} - (l + m - 1) Q_{l-2,m}
    R wr = R(1), wi = R(0);
#pragma unroll
    for (int m = 0; m <= NA; ++m) {
      if (m > 0) {
        const R t = wr * a.x - wi * a.y;
        wi = wr * a.y + wi * a.x;
        wr = t;
      }
      R q2 = R(0), q1 = R(dfact(m));
#pragma unroll
      for (int l = m; l <= NA; ++l) {
        R q;
        if (l == m)
          q = q1;
        else
          q = (R(2 * l - 1) * a.z * q1 - R(l + m - 1) * q2) * R(1.0 / (l - m));
        if (l > m) {
          q2 = q1;
          q1 = q;
        }
        const R yc = q * wr;
        A[ci(l, m)] += f * yc;
        B[ci(l, m)] += wf * yc;
        if (m > 0) {
          const R ys = q * wi;
          A[si(l, m)] += f * ys;
          B[si(l, m)] += wf * ys;
        }
      }
    }
  }
  if (!active) return;
  // keep the sums for the force pass
  R* keep = reinterpret_cast<R*>(p.shA) + (size_t)i * 2 * NH;
#pragma unroll
  for (int k = 0; k < NH; ++k) {
    keep[k] = A[k];
    keep[NH + k] = B[k];
  }
  R S[NA + 1], Sw[NA + 1];
#pragma unroll
  for (int l = 0; l <= NA; ++l) {
    R s = R(0), sw = R(0);
#pragma unroll
    for (int m = 0; m <= l; ++m) {
      const R nlm = R(sh_norm(l, m));
      R v = A[ci(l, m)] * A[ci(l, m)], vw = B[ci(l, m)] * B[ci(l, m)];
      if (m > 0) {
        v += A[si(l, m)] * A[si(l, m)];
        vw += B[si(l, m)] * B[si(l, m)];
      }
      s += nlm * v;
      sw += nlm * vw;
    }
    S[l] = s - D;
    Sw[l] = sw - Dw;
  }
  R* G = reinterpret_cast<R*>(p.G) + (size_t)i * p.ldG;
  const int at = p.t1;         // first angular component, typed half
  const int aw = p.t1 + p.t2;  // first angular component, weighted half
#pragma unroll
  for (int a = 0; a <= NA; ++a) {
    R g = R(0), gw = R(0);
#pragma unroll
    for (int l = 0; l <= a; ++l) {
      g += R(kChebLeg.c[a][l]) * S[l];
      gw += R(kChebLeg.c[a][l]) * Sw[l];
    }
    G[at + a] = g;
    if (p.weighted) G[aw + a] = gw;
  }
}

// backward: dE_i/dd_e of the angular part for every angular entry e of atom i
template <typename R, int NA>
__global__ __launch_bounds__(64) void k_ang_sh_bwd(DescParams p) {
  constexpr int NH = (NA + 1) * (NA + 1);
  const int i0 = blockIdx.x * 64 + threadIdx.x;
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
    R g[NA + 1], gw[NA + 1];
#pragma unroll
    for (int a = 0; a <= NA; ++a) {
      g[a] = gG[p.t1 + a];
      gw[a] = p.weighted ? gG[p.t1 + p.t2 + a] : R(0);
    }
#pragma unroll
    for (int l = 0; l <= NA; ++l) {
      R s = R(0), sw = R(0);
#pragma unroll
      for (int a = l; a <= NA; ++a) {
        s += R(kChebLeg.c[a][l]) * g[a];
        sw += R(kChebLeg.c[a][l]) * gw[a];
      }
      h[l] = s;
      hw[l] = sw;
      H += s;
      Hw += sw;
    }
  }
  // coefficients of each function: qt = 2 N_lm h_l A_lm, qw = 2 N_lm hw_l B_lm;
  // an entry of weight w has q = qt + w qw
  R qt[NH], qw[NH];
  {
    const R* keep = reinterpret_cast<const R*>(p.shA) + (size_t)i * 2 * NH;
#pragma unroll
    for (int l = 0; l <= NA; ++l)
#pragma unroll
      for (int m = 0; m <= l; ++m) {
        const R c2 = R(2.0 * sh_norm(l, m));
        qt[ci(l, m)] = c2 * h[l] * keep[ci(l, m)];
        qw[ci(l, m)] = c2 * hw[l] * keep[NH + ci(l, m)];
        if (m > 0) {
          qt[si(l, m)] = c2 * h[l] * keep[si(l, m)];
          qw[si(l, m)] = c2 * hw[l] * keep[NH + si(l, m)];
        }
      }
  }
  R* out = reinterpret_cast<R*>(p.gang) + (size_t)i * p.cap_ang * 3;
  // loads two and one entries ahead, as in the forward pass
  const int last = na > 0 ? na - 1 : 0;
  NbrLoad nx = load_nbr(p, row[0]);
  uint32_t wnext = row[min(1, last)];
  for (int e = 0; e < na; ++e) {
    const uint32_t wafter = row[min(e + 2, last)];
    const NbrLoad nn = load_nbr(p, wnext);
    const AngEntry<R> a = ang_entry<R>(nx, b, xi0, xi1, xi2, ra2, pi_2ra, true);
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
        const R t = wr * a.x - wi * a.y;
        wi = wr * a.y + wi * a.x;
        wr = t;
      }
      // columns m and m + 1 of Q together
      R q2 = R(0), q1 = R(dfact(m));      // column m
      R u2 = R(0), u1 = R(dfact(m + 1));  // column m + 1
#pragma unroll
      for (int l = m; l <= NA; ++l) {
        R q;
        if (l == m)
          q = q1;
        else
          q = (R(2 * l - 1) * a.z * q1 - R(l + m - 1) * q2) * R(1.0 / (l - m));
        if (l > m) {
          q2 = q1;
          q1 = q;
        }
        R u = R(0);  // Q_l,m+1
        if (l == m + 1) {
          u = u1;
        } else if (l > m + 1) {
          u = (R(2 * l - 1) * a.z * u1 - R(l + m) * u2) * R(1.0 / (l - m - 1));
          u2 = u1;
          u1 = u;
        }
        const R qc = qt[ci(l, m)] + a.w * qw[ci(l, m)];
        const R qs = m > 0 ? qt[si(l, m)] + a.w * qw[si(l, m)] : R(0);
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
    const R t = a.f * a.ir;
    const R radial = a.fp * V - t * ug - R(2) * a.f * a.fp * (H + a.w * a.w * Hw);
    const R ox = radial * a.x + t * gx, oy = radial * a.y + t * gy, oz = radial * a.z + t * gz;
    out[3 * e] = a.valid ? ox : R(0);
    out[3 * e + 1] = a.valid ? oy : R(0);
    out[3 * e + 2] = a.valid ? oz : R(0);
  }
}

template <typename R, int NA>
void launch_na(bool fwd, const DescParams& p, hipStream_t s) {
  const dim3 grid((p.n + 63) / 64), block(64);
  if (fwd)
    hipLaunchKernelGGL((k_ang_sh_fwd<R, NA>), grid, block, 0, s, p);
  else
    hipLaunchKernelGGL((k_ang_sh_bwd<R, NA>), grid, block, 0, s, p);
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
