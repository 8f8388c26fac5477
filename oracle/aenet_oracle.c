/*
 * aenet_oracle.c -- plain, slow FP64 CPU oracle of the Behler-Parrinello
 * ANN-potential energy, forces, molecular dynamics and training loss with the
 * Chebyshev descriptor of the paper (Chen, Morawietz, Mori, Markland, Artrith,
 * "AENET-LAMMPS and AENET-TINKER", arXiv:2107.11311, Sec. II).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU library links, includes or
 * calls this file.  Only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It is written for obviousness, not speed:
 * single-threaded, O(N^2) brute-force neighbour search, every sum taken in
 * the order of its definition.
 *
 * What is computed, and where the paper defines it:
 *   - feed-forward layer x^l = f(W^l x^{l-1} + b^l)           Sec. II A, Eq. 1
 *   - total energy as a sum of per-species atomic energies    Sec. II A, Eq. 2
 *   - radial Chebyshev coefficients c^pair_alpha              Sec. II B, Eq. 3
 *   - Chebyshev three-term recurrence                         Sec. II B, Eq. 4
 *   - cosine cutoff f_c                                       Sec. II B, Eq. 5
 *   - angular Chebyshev coefficients c^triple_alpha           Sec. II B, Eq. 6
 *   - training cost / back-propagated gradients               Sec. II C, Eq. 7
 *   - the MD cycle (coordinates -> E, F -> new coordinates)   Sec. III, Fig. 1
 *   - the virial (stress tensor of the whole system, which    Sec. III
 *     the earlier LAMMPS interface provides): minus the strain
 *     derivative of E, by the chain rule over the entries
 *
 * Readings where the paper is silent or loose (each also listed in the design
 * notes of the repository):
 *   - "order N" means alpha = 0..N (N+1 terms).
 *   - Eq. 6 sums over ordered pairs (j,k), j != k; the angular cutoff radius
 *     R_a is used for the angular set and its f_c, R_r for the radial terms;
 *     r_jk only defines the angle (no f_c(r_jk)).
 *   - species handling ("typed + weighted"): the typed channel gives every
 *     neighbour weight 1, the weighted channel weight w_{t(j)} (radial) and
 *     w_{t(j)} w_{t(k)} (angular).  G = [rad_typ | ang_typ | rad_wt | ang_wt];
 *     a single-species model keeps only the typed half.
 *   - a neighbour is an (atom, periodic image) pair with 0 < r < R (strict);
 *     r == 0 between distinct entries is an error (overlap).
 *   - T'_alpha = alpha U_{alpha-1} with the U recurrence (no division by sin).
 *   - energy+force loss for training (the paper's Eq. 7 is energy-only).
 *
 * Parity pins of every routine live in tests/test_oracle_*.py (closed forms,
 * invariances, finite differences, brute-force image sums, reversibility).
 */
#include "aenet_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* 1 eV/amu expressed in A^2/ps^2 (exact SI eV, CODATA-2018 atomic mass unit):
 * a = kappa * F / m turns eV/A and amu into A/ps^2. */
static const double KAPPA = 9648.533215665;

/* ------------------------------------------------------------------------- */
/* Chebyshev polynomials (Eq. 4) and the cosine cutoff (Eq. 5).              */
/* ------------------------------------------------------------------------- */

void orc_chebyshev(int order, double x, double* T, double* dT) {
  /* T_0 = 1, T_1 = x, T_{n+1} = 2 x T_n - T_{n-1}  (Eq. 4). */
  T[0] = 1.0;
  if (order >= 1) T[1] = x;
  for (int a = 1; a < order; ++a) T[a + 1] = 2.0 * x * T[a] - T[a - 1];
  if (!dT) return;
  /* dT_a/dx = a U_{a-1}(x); U_0 = 1, U_1 = 2x, U_{n+1} = 2x U_n - U_{n-1}. */
  double u_prev = 0.0; /* U_{-1} */
  double u = 1.0;      /* U_0 */
  dT[0] = 0.0;
  for (int a = 1; a <= order; ++a) {
    dT[a] = (double)a * u; /* u == U_{a-1} */
    double u_next = (a == 1) ? 2.0 * x : 2.0 * x * u - u_prev;
    u_prev = u;
    u = u_next;
  }
}

void orc_cutoff(double r, double rc, double* fc, double* dfc) {
  /* f_c(r) = (cos(pi r / R_c) + 1) / 2 for r <= R_c, 0 beyond (Eq. 5). */
  if (r <= rc) {
    *fc = 0.5 * (cos(M_PI * r / rc) + 1.0);
    if (dfc) *dfc = -0.5 * (M_PI / rc) * sin(M_PI * r / rc);
  } else {
    *fc = 0.0;
    if (dfc) *dfc = 0.0;
  }
}

int orc_descriptor_dim(int n_species, int radial_order, int angular_order) {
  int typed = (radial_order + 1) + (angular_order + 1);
  return n_species > 1 ? 2 * typed : typed;
}

/* ------------------------------------------------------------------------- */
/* Neighbour enumeration by brute force over atoms and periodic images.      */
/* ------------------------------------------------------------------------- */

typedef struct {
  int j;        /* neighbour atom */
  int s[3];     /* image shift */
  double d[3];  /* r_j + s*L - r_i */
  double r;     /* |d| */
} entry;

typedef struct {
  int n;
  int* start;   /* [n+1] */
  entry* e;     /* [start[n]] */
} nlist;

static double wrap1(double x, double L) {
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w = 0.0;
  return w;
}

static void wrap_positions(int n, const double* pos, const double* box, const int* pbc,
                           double* out) {
  for (int i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a)
      out[3 * i + a] = pbc[a] ? wrap1(pos[3 * i + a], box[a]) : pos[3 * i + a];
}

static void free_list(nlist* nl) {
  free(nl->start);
  free(nl->e);
  nl->start = NULL;
  nl->e = NULL;
}

/* All entries (j, s) != (i, 0) with |r_j + s L - r_i| < cutoff.  Images are
 * enumerated in [-ceil(cutoff/L)-1, ceil(cutoff/L)+1] on every periodic axis,
 * which contains every image closer than the cutoff for wrapped positions.
 * When every periodic edge is at least twice the cutoff, at most one image of
 * each atom can be closer than the cutoff, and only the nearest one (minimum
 * image) is examined. */
static int build_list(int n, const double* posw, const double* box, const int* pbc,
                      double cutoff, nlist* nl) {
  int smax[3];
  int minimg = 1;
  for (int a = 0; a < 3; ++a) {
    smax[a] = pbc[a] ? (int)ceil(cutoff / box[a]) + 1 : 0;
    if (pbc[a] && box[a] < 2.0 * cutoff) minimg = 0;
  }
  size_t cap = 1024, used = 0;
  nl->n = n;
  nl->start = (int*)malloc(sizeof(int) * (size_t)(n + 1));
  nl->e = (entry*)malloc(sizeof(entry) * cap);
  if (!nl->start || !nl->e) { free_list(nl); return ORC_E_NOMEM; }
  const double c2 = cutoff * cutoff;
  for (int i = 0; i < n; ++i) {
    nl->start[i] = (int)used;
    for (int j = 0; j < n; ++j) {
      int lo[3], hi[3];
      for (int a = 0; a < 3; ++a) { lo[a] = -smax[a]; hi[a] = smax[a]; }
      if (minimg) {
        if (j == i) continue;
        for (int a = 0; a < 3; ++a) {
          int s = 0;
          if (pbc[a]) {
            double dd = posw[3 * j + a] - posw[3 * i + a];
            if (dd > 0.5 * box[a]) s = -1;
            else if (dd < -0.5 * box[a]) s = 1;
          }
          lo[a] = hi[a] = s;
        }
      }
      for (int sx = lo[0]; sx <= hi[0]; ++sx)
        for (int sy = lo[1]; sy <= hi[1]; ++sy)
          for (int sz = lo[2]; sz <= hi[2]; ++sz) {
            if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
            double d[3];
            int s[3] = {sx, sy, sz};
            for (int a = 0; a < 3; ++a)
              d[a] = posw[3 * j + a] + (double)s[a] * box[a] - posw[3 * i + a];
            double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
            if (!(r2 < c2)) continue;
            if (r2 == 0.0) { free_list(nl); return ORC_E_OVERLAP; }
            if (used == cap) {
              cap *= 2;
              entry* ne = (entry*)realloc(nl->e, sizeof(entry) * cap);
              if (!ne) { free_list(nl); return ORC_E_NOMEM; }
              nl->e = ne;
            }
            entry* en = &nl->e[used++];
            en->j = j;
            for (int a = 0; a < 3; ++a) { en->s[a] = s[a]; en->d[a] = d[a]; }
            en->r = sqrt(r2);
          }
    }
  }
  nl->start[n] = (int)used;
  return ORC_OK;
}

int orc_neighbors(int n, const double* pos, const double* box, const int* pbc,
                  double cutoff, int cap, int* counts, int* nbr_j, int* nbr_shift) {
  if (n < 0 || cutoff <= 0.0) return ORC_E_INVALID;
  double* posw = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!posw) return ORC_E_NOMEM;
  wrap_positions(n, pos, box, pbc, posw);
  nlist nl;
  int st = build_list(n, posw, box, pbc, cutoff, &nl);
  free(posw);
  if (st) return st;
  int over = 0;
  for (int i = 0; i < n; ++i) {
    int c = nl.start[i + 1] - nl.start[i];
    counts[i] = c;
    if (c > cap) { over = 1; continue; }
    for (int k = 0; k < c; ++k) {
      const entry* en = &nl.e[nl.start[i] + k];
      nbr_j[(size_t)i * cap + k] = en->j;
      for (int a = 0; a < 3; ++a) nbr_shift[((size_t)i * cap + k) * 3 + a] = en->s[a];
    }
  }
  free_list(&nl);
  return over ? ORC_E_CAPACITY : ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Descriptor of one atom (Eqs. 3-6).                                        */
/* ------------------------------------------------------------------------- */

typedef struct {
  int D, nr, na, S;
  int off_rt, off_at, off_rw, off_aw; /* offsets of the four blocks (-1 = absent) */
} layout;

static layout make_layout(const orc_model* m) {
  layout L;
  L.nr = m->radial_order;
  L.na = m->angular_order;
  L.S = m->n_species;
  L.off_rt = 0;
  L.off_at = L.nr + 1;
  if (L.S > 1) {
    L.off_rw = L.off_at + L.na + 1;
    L.off_aw = L.off_rw + L.nr + 1;
  } else {
    L.off_rw = L.off_aw = -1;
  }
  L.D = orc_descriptor_dim(L.S, L.nr, L.na);
  return L;
}

static double wt(const orc_model* m, const int* species, int j) {
  return m->type_weight ? m->type_weight[species[j]] : 1.0;
}

/* G for atom i from its entries (any order). */
static void atom_descriptor(const orc_model* m, const layout* L, const entry* e, int ne,
                            const int* species, double* G, double* T) {
  for (int a = 0; a < L->D; ++a) G[a] = 0.0;
  const double Rr = m->radial_cutoff, Ra = m->angular_cutoff;
  /* radial: c_alpha = sum_j T_alpha(2 r_ij / R - 1) f_c(r_ij)  (Eq. 3) */
  for (int p = 0; p < ne; ++p) {
    if (!(e[p].r < Rr)) continue;
    double fc;
    orc_cutoff(e[p].r, Rr, &fc, NULL);
    orc_chebyshev(L->nr, 2.0 * e[p].r / Rr - 1.0, T, NULL);
    double w = wt(m, species, e[p].j);
    for (int a = 0; a <= L->nr; ++a) {
      G[L->off_rt + a] += T[a] * fc;
      if (L->S > 1) G[L->off_rw + a] += w * T[a] * fc;
    }
  }
  /* angular: c_alpha = sum_{j != k} T_alpha(cos theta_ijk) f_c(r_ij) f_c(r_ik)  (Eq. 6) */
  for (int p = 0; p < ne; ++p) {
    if (!(e[p].r < Ra)) continue;
    for (int q = 0; q < ne; ++q) {
      if (q == p || !(e[q].r < Ra)) continue;
      double fj, fk;
      orc_cutoff(e[p].r, Ra, &fj, NULL);
      orc_cutoff(e[q].r, Ra, &fk, NULL);
      double cth = (e[p].d[0] * e[q].d[0] + e[p].d[1] * e[q].d[1] + e[p].d[2] * e[q].d[2]) /
                   (e[p].r * e[q].r);
      orc_chebyshev(L->na, cth, T, NULL);
      double ww = wt(m, species, e[p].j) * wt(m, species, e[q].j);
      for (int a = 0; a <= L->na; ++a) {
        G[L->off_at + a] += T[a] * fj * fk;
        if (L->S > 1) G[L->off_aw + a] += ww * T[a] * fj * fk;
      }
    }
  }
}

/* ------------------------------------------------------------------------- */
/* Atomic network (Eq. 1) and its input gradient.                            */
/* ------------------------------------------------------------------------- */

int orc_net_nparams(const orc_net* net) {
  int np = 0;
  for (int l = 0; l < net->n_layers; ++l) np += net->widths[l + 1] * (net->widths[l] + 1);
  return np;
}

static int net_maxw(const orc_net* net) {
  int w = 0;
  for (int l = 0; l <= net->n_layers; ++l) if (net->widths[l] > w) w = net->widths[l];
  return w;
}

static double act_f(int act, double z) { return act == ORC_ACT_TANH ? tanh(z) : z; }
/* derivative expressed through the activation value x = f(z) */
static double act_d1(int act, double x) { return act == ORC_ACT_TANH ? 1.0 - x * x : 1.0; }
static double act_d2(int act, double x) {
  return act == ORC_ACT_TANH ? -2.0 * x * (1.0 - x * x) : 0.0;
}

/* Forward pass storing every layer's activations: xs[l] has widths[l] values
 * (xs[0] = normalised input).  Returns E. */
static double net_forward(const orc_net* net, const double* G, double** xs) {
  const int D = net->widths[0];
  for (int a = 0; a < D; ++a) {
    double s = net->shift ? net->shift[a] : 0.0;
    double c = net->scale ? net->scale[a] : 1.0;
    xs[0][a] = (G[a] - s) * c;
  }
  const double* p = net->params;
  for (int l = 0; l < net->n_layers; ++l) {
    int nin = net->widths[l], nout = net->widths[l + 1];
    const double* W = p;
    const double* b = p + (size_t)nout * nin;
    for (int o = 0; o < nout; ++o) {
      double z = b[o];
      for (int k = 0; k < nin; ++k) z += W[(size_t)o * nin + k] * xs[l][k];
      xs[l + 1][o] = act_f(net->act[l], z);
    }
    p = b + nout;
  }
  return xs[net->n_layers][0] + net->e_offset;
}

/* dE/dG by back-propagation through the stored activations. */
static void net_backward(const orc_net* net, double** xs, double* gbuf, double* gbuf2,
                         double* g) {
  const int Lw = net->n_layers;
  /* offsets of each layer's parameters */
  size_t off[64];
  size_t o = 0;
  for (int l = 0; l < Lw; ++l) { off[l] = o; o += (size_t)net->widths[l + 1] * (net->widths[l] + 1); }
  double* up = gbuf;   /* dE/dx_l */
  double* dn = gbuf2;
  up[0] = 1.0;
  for (int l = Lw - 1; l >= 0; --l) {
    int nin = net->widths[l], nout = net->widths[l + 1];
    const double* W = net->params + off[l];
    for (int k = 0; k < nin; ++k) dn[k] = 0.0;
    for (int q = 0; q < nout; ++q) {
      double dz = up[q] * act_d1(net->act[l], xs[l + 1][q]);
      for (int k = 0; k < nin; ++k) dn[k] += W[(size_t)q * nin + k] * dz;
    }
    double* t = up; up = dn; dn = t;
  }
  const int D = net->widths[0];
  for (int a = 0; a < D; ++a) g[a] = up[a] * (net->scale ? net->scale[a] : 1.0);
}

typedef struct {
  double** xs;
  double* b1;
  double* b2;
} net_ws;

static int ws_alloc(const orc_model* m, net_ws* w) {
  int maxw = 1, maxl = 1;
  for (int t = 0; t < m->n_species; ++t) {
    int q = net_maxw(&m->nets[t]);
    if (q > maxw) maxw = q;
    if (m->nets[t].n_layers > maxl) maxl = m->nets[t].n_layers;
  }
  w->xs = (double**)malloc(sizeof(double*) * (size_t)(maxl + 1));
  w->b1 = (double*)malloc(sizeof(double) * (size_t)maxw);
  w->b2 = (double*)malloc(sizeof(double) * (size_t)maxw);
  if (!w->xs || !w->b1 || !w->b2) return ORC_E_NOMEM;
  for (int l = 0; l <= maxl; ++l) {
    w->xs[l] = (double*)malloc(sizeof(double) * (size_t)maxw);
    if (!w->xs[l]) return ORC_E_NOMEM;
  }
  return ORC_OK;
}

static void ws_free(net_ws* w, const orc_model* m) {
  int maxl = 1;
  for (int t = 0; t < m->n_species; ++t) if (m->nets[t].n_layers > maxl) maxl = m->nets[t].n_layers;
  if (w->xs) for (int l = 0; l <= maxl; ++l) free(w->xs[l]);
  free(w->xs);
  free(w->b1);
  free(w->b2);
}

int orc_net_eval(const orc_net* net, const double* G, double* E, double* g) {
  int maxw = net_maxw(net);
  double** xs = (double**)malloc(sizeof(double*) * (size_t)(net->n_layers + 1));
  double* b1 = (double*)malloc(sizeof(double) * (size_t)maxw);
  double* b2 = (double*)malloc(sizeof(double) * (size_t)maxw);
  for (int l = 0; l <= net->n_layers; ++l) xs[l] = (double*)malloc(sizeof(double) * (size_t)maxw);
  *E = net_forward(net, G, xs);
  if (g) net_backward(net, xs, b1, b2, g);
  for (int l = 0; l <= net->n_layers; ++l) free(xs[l]);
  free(xs);
  free(b1);
  free(b2);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Energy and forces, pairwise chain rule.                                   */
/* ------------------------------------------------------------------------- */

static int check_model(const orc_model* m) {
  if (!m || m->n_species < 1 || m->radial_order < 0 || m->angular_order < 0) return ORC_E_INVALID;
  if (!(m->radial_cutoff > 0.0) || !(m->angular_cutoff > 0.0)) return ORC_E_INVALID;
  int D = orc_descriptor_dim(m->n_species, m->radial_order, m->angular_order);
  for (int t = 0; t < m->n_species; ++t) {
    const orc_net* nt = &m->nets[t];
    if (nt->n_layers < 1 || nt->n_layers > 60) return ORC_E_INVALID;
    if (nt->widths[0] != D || nt->widths[nt->n_layers] != 1) return ORC_E_INVALID;
  }
  return ORC_OK;
}

static double list_cutoff(const orc_model* m) {
  return m->radial_cutoff > m->angular_cutoff ? m->radial_cutoff : m->angular_cutoff;
}

/* Neumaier-compensated running sum. */
typedef struct { double s, c; } ksum;
static void ks_add(ksum* k, double x) {
  double t = k->s + x;
  if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x; else k->c += (x - t) + k->s;
  k->s = t;
}
static double ks_val(const ksum* k) { return k->s + k->c; }

/* Adds -dE_i/dr to forces for atom i, given g = dE_i/dG_i and its entries. */
/* F += the forces of E_i; if vir != NULL, vir[3a+b] -= (dE_i/dd)_a d_b over
 * every entry's gradient (the virial W = -dE/d(strain)). */
static void atom_forces(const orc_model* m, const layout* L, int i, const entry* e, int ne,
                        const int* species, const double* g, double* T, double* dT,
                        double* F, double* vir) {
  const double Rr = m->radial_cutoff, Ra = m->angular_cutoff;
  for (int p = 0; p < ne; ++p) {
    if (!(e[p].r < Rr)) continue;
    double fc, dfc;
    orc_cutoff(e[p].r, Rr, &fc, &dfc);
    orc_chebyshev(L->nr, 2.0 * e[p].r / Rr - 1.0, T, dT);
    double w = wt(m, species, e[p].j);
    double dEdr = 0.0;
    for (int a = 0; a <= L->nr; ++a) {
      double c = g[L->off_rt + a] + (L->S > 1 ? w * g[L->off_rw + a] : 0.0);
      dEdr += c * (dT[a] * (2.0 / Rr) * fc + T[a] * dfc);
    }
    for (int c = 0; c < 3; ++c) {
      double v = dEdr * e[p].d[c] / e[p].r; /* dE_i/dd */
      F[3 * i + c] += v;
      F[3 * e[p].j + c] -= v;
      if (vir)
        for (int b = 0; b < 3; ++b) vir[3 * c + b] -= v * e[p].d[b];
    }
  }
  for (int p = 0; p < ne; ++p) {
    if (!(e[p].r < Ra)) continue;
    for (int q = 0; q < ne; ++q) {
      if (q == p || !(e[q].r < Ra)) continue;
      double fj, dfj, fk, dfk;
      orc_cutoff(e[p].r, Ra, &fj, &dfj);
      orc_cutoff(e[q].r, Ra, &fk, &dfk);
      const double rj = e[p].r, rk = e[q].r;
      double cth = (e[p].d[0] * e[q].d[0] + e[p].d[1] * e[q].d[1] + e[p].d[2] * e[q].d[2]) / (rj * rk);
      orc_chebyshev(L->na, cth, T, dT);
      double ww = wt(m, species, e[p].j) * wt(m, species, e[q].j);
      double A = 0.0, B = 0.0;
      for (int a = 0; a <= L->na; ++a) {
        double c = g[L->off_at + a] + (L->S > 1 ? ww * g[L->off_aw + a] : 0.0);
        A += c * T[a];
        B += c * dT[a];
      }
      for (int c = 0; c < 3; ++c) {
        double dcos_dj = e[q].d[c] / (rj * rk) - cth * e[p].d[c] / (rj * rj);
        double dcos_dk = e[p].d[c] / (rj * rk) - cth * e[q].d[c] / (rk * rk);
        double vj = B * fj * fk * dcos_dj + A * dfj * fk * e[p].d[c] / rj;
        double vk = B * fj * fk * dcos_dk + A * fj * dfk * e[q].d[c] / rk;
        F[3 * i + c] += vj + vk;
        F[3 * e[p].j + c] -= vj;
        F[3 * e[q].j + c] -= vk;
        if (vir)
          for (int b = 0; b < 3; ++b) vir[3 * c + b] -= vj * e[p].d[b] + vk * e[q].d[b];
      }
    }
  }
}

typedef struct {
  double* posw;
  nlist nl;
  double* G;   /* [D] */
  double* g;   /* [D] */
  double* T;
  double* dT;
  net_ws ws;
} work;

static int work_init(const orc_model* m, int n, const double* pos, const double* box,
                     const int* pbc, work* w) {
  memset(w, 0, sizeof(*w));
  layout L = make_layout(m);
  int maxo = (m->radial_order > m->angular_order ? m->radial_order : m->angular_order) + 1;
  w->posw = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  w->G = (double*)malloc(sizeof(double) * (size_t)L.D);
  w->g = (double*)malloc(sizeof(double) * (size_t)L.D);
  w->T = (double*)malloc(sizeof(double) * (size_t)maxo);
  w->dT = (double*)malloc(sizeof(double) * (size_t)maxo);
  if (!w->posw || !w->G || !w->g || !w->T || !w->dT) return ORC_E_NOMEM;
  int st = ws_alloc(m, &w->ws);
  if (st) return st;
  wrap_positions(n, pos, box, pbc, w->posw);
  return build_list(n, w->posw, box, pbc, list_cutoff(m), &w->nl);
}

static void work_free(const orc_model* m, work* w) {
  free(w->posw);
  free_list(&w->nl);
  free(w->G);
  free(w->g);
  free(w->T);
  free(w->dT);
  ws_free(&w->ws, m);
}

static int check_species(const orc_model* m, int n, const int* species) {
  for (int i = 0; i < n; ++i)
    if (species[i] < 0 || species[i] >= m->n_species) return ORC_E_INVALID;
  return ORC_OK;
}

int orc_descriptors(const orc_model* m, int n, const double* pos, const int* species,
                    const double* box, const int* pbc, double* G) {
  int st = check_model(m);
  if (st) return st;
  if ((st = check_species(m, n, species))) return st;
  work w;
  st = work_init(m, n, pos, box, pbc, &w);
  if (st) { work_free(m, &w); return st; }
  layout L = make_layout(m);
  for (int i = 0; i < n; ++i)
    atom_descriptor(m, &L, &w.nl.e[w.nl.start[i]], w.nl.start[i + 1] - w.nl.start[i], species,
                    G + (size_t)i * L.D, w.T);
  work_free(m, &w);
  return ORC_OK;
}

int orc_energy_forces(const orc_model* m, int n, const double* pos, const int* species,
                      const double* box, const int* pbc, double* e_total, double* e_atom,
                      double* forces, double* Gout) {
  return orc_energy_forces_virial(m, n, pos, species, box, pbc, e_total, e_atom, forces, Gout, NULL);
}

int orc_energy_forces_virial(const orc_model* m, int n, const double* pos, const int* species,
                             const double* box, const int* pbc, double* e_total, double* e_atom,
                             double* forces, double* Gout, double* virial) {
  int st = check_model(m);
  if (st) return st;
  if ((st = check_species(m, n, species))) return st;
  work w;
  st = work_init(m, n, pos, box, pbc, &w);
  if (st) { work_free(m, &w); return st; }
  layout L = make_layout(m);
  double* fbuf = NULL;
  if (virial && !forces) {
    fbuf = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
    if (!fbuf) { work_free(m, &w); return ORC_E_NOMEM; }
    forces = fbuf;
  }
  if (virial) for (int k = 0; k < 9; ++k) virial[k] = 0.0;
  if (forces) for (int k = 0; k < 3 * n; ++k) forces[k] = 0.0;
  ksum E = {0.0, 0.0};
  for (int i = 0; i < n; ++i) {
    const entry* e = &w.nl.e[w.nl.start[i]];
    int ne = w.nl.start[i + 1] - w.nl.start[i];
    atom_descriptor(m, &L, e, ne, species, w.G, w.T);
    if (Gout) memcpy(Gout + (size_t)i * L.D, w.G, sizeof(double) * (size_t)L.D);
    const orc_net* net = &m->nets[species[i]];
    double Ei = net_forward(net, w.G, w.ws.xs);
    if (e_atom) e_atom[i] = Ei;
    ks_add(&E, Ei);
    if (forces) {
      net_backward(net, w.ws.xs, w.ws.b1, w.ws.b2, w.g);
      atom_forces(m, &L, i, e, ne, species, w.g, w.T, w.dT, forces, virial);
    }
  }
  if (e_total) *e_total = ks_val(&E);
  free(fbuf);
  work_free(m, &w);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Selected atoms of a large structure: E_m, F_m (and G_m) for the atoms in   */
/* sel only.  F_m = -sum_i dE_i/dr_m needs every atom i whose environment      */
/* contains m, i.e. m itself and its neighbours, each with its own list.       */
/* ------------------------------------------------------------------------- */

/* entries of atom i alone (brute force over all atoms and images) */
static int atom_list(int n, const double* posw, const double* box, const int* pbc, double cutoff,
                     int i, entry** out, int* count) {
  int smax[3];
  int minimg = 1;
  for (int a = 0; a < 3; ++a) {
    smax[a] = pbc[a] ? (int)ceil(cutoff / box[a]) + 1 : 0;
    if (pbc[a] && box[a] < 2.0 * cutoff) minimg = 0;
  }
  int cap = 256, used = 0;
  entry* e = (entry*)malloc(sizeof(entry) * (size_t)cap);
  if (!e) return ORC_E_NOMEM;
  const double c2 = cutoff * cutoff;
  for (int j = 0; j < n; ++j) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) { lo[a] = -smax[a]; hi[a] = smax[a]; }
    if (minimg) {
      if (j == i) continue;
      for (int a = 0; a < 3; ++a) {
        int s = 0;
        if (pbc[a]) {
          double dd = posw[3 * j + a] - posw[3 * i + a];
          if (dd > 0.5 * box[a]) s = -1;
          else if (dd < -0.5 * box[a]) s = 1;
        }
        lo[a] = hi[a] = s;
      }
    }
    for (int sx = lo[0]; sx <= hi[0]; ++sx)
      for (int sy = lo[1]; sy <= hi[1]; ++sy)
        for (int sz = lo[2]; sz <= hi[2]; ++sz) {
          if (j == i && sx == 0 && sy == 0 && sz == 0) continue;
          int s[3] = {sx, sy, sz};
          double d[3];
          for (int a = 0; a < 3; ++a) d[a] = posw[3 * j + a] + (double)s[a] * box[a] - posw[3 * i + a];
          double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
          if (!(r2 < c2)) continue;
          if (r2 == 0.0) { free(e); return ORC_E_OVERLAP; }
          if (used == cap) {
            cap *= 2;
            entry* ne = (entry*)realloc(e, sizeof(entry) * (size_t)cap);
            if (!ne) { free(e); return ORC_E_NOMEM; }
            e = ne;
          }
          e[used].j = j;
          for (int a = 0; a < 3; ++a) { e[used].s[a] = s[a]; e[used].d[a] = d[a]; }
          e[used].r = sqrt(r2);
          ++used;
        }
  }
  *out = e;
  *count = used;
  return ORC_OK;
}

int orc_energy_forces_subset(const orc_model* m, int n, const double* pos, const int* species,
                             const double* box, const int* pbc, int n_sel, const int* sel,
                             double* e_sel, double* f_sel, double* g_sel) {
  int st = check_model(m);
  if (st) return st;
  if ((st = check_species(m, n, species))) return st;
  layout L = make_layout(m);
  const double rc = list_cutoff(m);
  double* posw = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  double* F = (double*)calloc(3 * (size_t)(n > 0 ? n : 1), sizeof(double));
  int maxo = (m->radial_order > m->angular_order ? m->radial_order : m->angular_order) + 1;
  double* G = (double*)malloc(sizeof(double) * (size_t)L.D);
  double* g = (double*)malloc(sizeof(double) * (size_t)L.D);
  double* T = (double*)malloc(sizeof(double) * (size_t)maxo);
  double* dT = (double*)malloc(sizeof(double) * (size_t)maxo);
  net_ws ws;
  memset(&ws, 0, sizeof(ws));
  if (!posw || !F || !G || !g || !T || !dT || ws_alloc(m, &ws)) st = ORC_E_NOMEM;
  if (st == ORC_OK) wrap_positions(n, pos, box, pbc, posw);
  for (int q = 0; st == ORC_OK && q < n_sel; ++q) {
    const int mi = sel[q];
    if (mi < 0 || mi >= n) { st = ORC_E_INVALID; break; }
    entry* em = NULL;
    int nm = 0;
    st = atom_list(n, posw, box, pbc, rc, mi, &em, &nm);
    if (st) break;
    /* atoms whose environment holds mi: mi itself and every neighbour atom of mi
       (each atom once, whatever the number of its images) */
    int* who = (int*)malloc(sizeof(int) * (size_t)(nm + 1));
    int nw = 0;
    who[nw++] = mi;
    for (int p = 0; p < nm; ++p) {
      int seen = 0;
      for (int k = 0; k < nw; ++k) if (who[k] == em[p].j) { seen = 1; break; }
      if (!seen) who[nw++] = em[p].j;
    }
    for (int k = 0; k < 3 * n; ++k) F[k] = 0.0;
    for (int k = 0; st == ORC_OK && k < nw; ++k) {
      const int i = who[k];
      entry* ei = NULL;
      int ni = 0;
      st = atom_list(n, posw, box, pbc, rc, i, &ei, &ni);
      if (st) break;
      atom_descriptor(m, &L, ei, ni, species, G, T);
      const orc_net* net = &m->nets[species[i]];
      double Ei = net_forward(net, G, ws.xs);
      net_backward(net, ws.xs, ws.b1, ws.b2, g);
      atom_forces(m, &L, i, ei, ni, species, g, T, dT, F, NULL);
      if (i == mi) {
        if (e_sel) e_sel[q] = Ei;
        if (g_sel) memcpy(g_sel + (size_t)q * L.D, G, sizeof(double) * (size_t)L.D);
      }
      free(ei);
    }
    if (f_sel) for (int c = 0; c < 3; ++c) f_sel[3 * q + c] = F[3 * mi + c];
    free(who);
    free(em);
  }
  free(posw);
  free(F);
  free(G);
  free(g);
  free(T);
  free(dT);
  ws_free(&ws, m);
  return st;
}

/* ------------------------------------------------------------------------- */
/* Second formulation: Jacobians of the descriptor w.r.t. entry displacements. */
/* ------------------------------------------------------------------------- */

/* J[a*3*ne + 3*p + c] = dG_i[a] / dd_p[c] for the ne entries of atom i. */
static void entry_jacobian(const orc_model* m, const layout* L, const entry* e, int ne,
                           const int* species, double* J, double* T, double* dT) {
  const double Rr = m->radial_cutoff, Ra = m->angular_cutoff;
  const size_t stride = 3 * (size_t)ne;
  memset(J, 0, sizeof(double) * (size_t)L->D * stride);
  for (int p = 0; p < ne; ++p) {
    if (!(e[p].r < Rr)) continue;
    double fc, dfc;
    orc_cutoff(e[p].r, Rr, &fc, &dfc);
    orc_chebyshev(L->nr, 2.0 * e[p].r / Rr - 1.0, T, dT);
    double w = wt(m, species, e[p].j);
    for (int a = 0; a <= L->nr; ++a) {
      double dphi = dT[a] * (2.0 / Rr) * fc + T[a] * dfc;
      for (int c = 0; c < 3; ++c) {
        double v = dphi * e[p].d[c] / e[p].r;
        J[(size_t)(L->off_rt + a) * stride + 3 * p + c] += v;
        if (L->S > 1) J[(size_t)(L->off_rw + a) * stride + 3 * p + c] += w * v;
      }
    }
  }
  for (int p = 0; p < ne; ++p) {
    if (!(e[p].r < Ra)) continue;
    for (int q = 0; q < ne; ++q) {
      if (q == p || !(e[q].r < Ra)) continue;
      double fj, dfj, fk, dfk;
      orc_cutoff(e[p].r, Ra, &fj, &dfj);
      orc_cutoff(e[q].r, Ra, &fk, &dfk);
      const double rj = e[p].r, rk = e[q].r;
      double cth = (e[p].d[0] * e[q].d[0] + e[p].d[1] * e[q].d[1] + e[p].d[2] * e[q].d[2]) / (rj * rk);
      orc_chebyshev(L->na, cth, T, dT);
      double ww = wt(m, species, e[p].j) * wt(m, species, e[q].j);
      for (int a = 0; a <= L->na; ++a) {
        for (int c = 0; c < 3; ++c) {
          double dcos_dj = e[q].d[c] / (rj * rk) - cth * e[p].d[c] / (rj * rj);
          double dcos_dk = e[p].d[c] / (rj * rk) - cth * e[q].d[c] / (rk * rk);
          double vj = dT[a] * fj * fk * dcos_dj + T[a] * dfj * fk * e[p].d[c] / rj;
          double vk = dT[a] * fj * fk * dcos_dk + T[a] * fj * dfk * e[q].d[c] / rk;
          J[(size_t)(L->off_at + a) * stride + 3 * p + c] += vj;
          J[(size_t)(L->off_at + a) * stride + 3 * q + c] += vk;
          if (L->S > 1) {
            J[(size_t)(L->off_aw + a) * stride + 3 * p + c] += ww * vj;
            J[(size_t)(L->off_aw + a) * stride + 3 * q + c] += ww * vk;
          }
        }
      }
    }
  }
}

int orc_forces_dense(const orc_model* m, int n, const double* pos, const int* species,
                     const double* box, const int* pbc, double* forces) {
  int st = check_model(m);
  if (st) return st;
  if ((st = check_species(m, n, species))) return st;
  work w;
  st = work_init(m, n, pos, box, pbc, &w);
  if (st) { work_free(m, &w); return st; }
  layout L = make_layout(m);
  /* Dense Jacobian of G_i over all 3n coordinates. */
  double* Jd = (double*)malloc(sizeof(double) * (size_t)L.D * 3 * (size_t)n);
  int maxne = 0;
  for (int i = 0; i < n; ++i) {
    int ne = w.nl.start[i + 1] - w.nl.start[i];
    if (ne > maxne) maxne = ne;
  }
  double* Je = (double*)malloc(sizeof(double) * (size_t)L.D * 3 * (size_t)(maxne > 0 ? maxne : 1));
  if (!Jd || !Je) { free(Jd); free(Je); work_free(m, &w); return ORC_E_NOMEM; }
  for (int k = 0; k < 3 * n; ++k) forces[k] = 0.0;
  for (int i = 0; i < n; ++i) {
    const entry* e = &w.nl.e[w.nl.start[i]];
    int ne = w.nl.start[i + 1] - w.nl.start[i];
    atom_descriptor(m, &L, e, ne, species, w.G, w.T);
    const orc_net* net = &m->nets[species[i]];
    net_forward(net, w.G, w.ws.xs);
    net_backward(net, w.ws.xs, w.ws.b1, w.ws.b2, w.g);
    entry_jacobian(m, &L, e, ne, species, Je, w.T, w.dT);
    /* d_p = r_j + s L - r_i: dG/dr_j += dG/dd_p, dG/dr_i -= dG/dd_p. */
    memset(Jd, 0, sizeof(double) * (size_t)L.D * 3 * (size_t)n);
    for (int a = 0; a < L.D; ++a)
      for (int p = 0; p < ne; ++p)
        for (int c = 0; c < 3; ++c) {
          double v = Je[(size_t)a * 3 * ne + 3 * p + c];
          Jd[(size_t)a * 3 * n + 3 * e[p].j + c] += v;
          Jd[(size_t)a * 3 * n + 3 * i + c] -= v;
        }
    /* F -= J_i^T g_i */
    for (int k = 0; k < 3 * n; ++k) {
      double s = 0.0;
      for (int a = 0; a < L.D; ++a) s += Jd[(size_t)a * 3 * n + k] * w.g[a];
      forces[k] -= s;
    }
  }
  free(Jd);
  free(Je);
  work_free(m, &w);
  return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* Velocity Verlet (the propagation step of the MD cycle, Fig. 1).           */
/* ------------------------------------------------------------------------- */

int orc_md_vv(const orc_model* m, int n, double* pos, double* vel, const int* species,
              const double* masses, const double* box, const int* pbc, double dt,
              int n_steps, double* e_pot, double* e_kin, double* forces) {
  int st = check_model(m);
  if (st) return st;
  if ((st = check_species(m, n, species))) return st;
  double* F = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!F) return ORC_E_NOMEM;
  double E = 0.0;
  st = orc_energy_forces(m, n, pos, species, box, pbc, &E, NULL, F, NULL);
  for (int step = 0; st == ORC_OK && step < n_steps; ++step) {
    for (int i = 0; i < n; ++i) {
      double inv_m = KAPPA / masses[species[i]];
      for (int c = 0; c < 3; ++c) {
        vel[3 * i + c] += 0.5 * dt * inv_m * F[3 * i + c];
        pos[3 * i + c] += dt * vel[3 * i + c];
        if (pbc[c]) pos[3 * i + c] = wrap1(pos[3 * i + c], box[c]);
      }
    }
    st = orc_energy_forces(m, n, pos, species, box, pbc, &E, NULL, F, NULL);
    if (st) break;
    for (int i = 0; i < n; ++i) {
      double inv_m = KAPPA / masses[species[i]];
      for (int c = 0; c < 3; ++c) vel[3 * i + c] += 0.5 * dt * inv_m * F[3 * i + c];
    }
  }
  if (st == ORC_OK) {
    ksum K = {0.0, 0.0};
    for (int i = 0; i < n; ++i)
      for (int c = 0; c < 3; ++c)
        ks_add(&K, 0.5 * masses[species[i]] * vel[3 * i + c] * vel[3 * i + c] / KAPPA);
    if (e_pot) *e_pot = E;
    if (e_kin) *e_kin = ks_val(&K);
    if (forces) memcpy(forces, F, sizeof(double) * 3 * (size_t)n);
  }
  free(F);
  return st;
}

/* ------------------------------------------------------------------------- */
/* Energy+force loss and its parameter gradient (training, Sec. II C).       */
/* ------------------------------------------------------------------------- */

static int check_batch(const orc_model* m, int B, const int* offsets, const int* species) {
  if (B < 1 || offsets[0] != 0) return ORC_E_INVALID;
  for (int s = 0; s < B; ++s) if (offsets[s + 1] <= offsets[s]) return ORC_E_INVALID;
  return check_species(m, offsets[B], species);
}

int orc_loss(const orc_model* m, int B, const int* offsets, const double* pos,
             const int* species, const double* boxes, const int* pbc, const double* e_ref,
             const double* f_ref, double lambda_f, int form, double* loss) {
  int st = check_model(m);
  if (st) return st;
  if (form != 0 && form != 1) return ORC_E_INVALID;
  if ((st = check_batch(m, B, offsets, species))) return st;
  ksum C = {0.0, 0.0};
  for (int s = 0; s < B && st == ORC_OK; ++s) {
    int a0 = offsets[s], ns = offsets[s + 1] - offsets[s];
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)ns);
    double E;
    st = orc_energy_forces(m, ns, pos + 3 * (size_t)a0, species + a0, boxes + 3 * s, pbc, &E,
                           NULL, F, NULL);
    if (st == ORC_OK) {
      ksum fs = {0.0, 0.0};
      for (int k = 0; k < 3 * ns; ++k) {
        double df = F[k] - f_ref[3 * (size_t)a0 + k];
        ks_add(&fs, df * df);
      }
      if (form == 0) {
        double de = (E - e_ref[s]) / ns;
        ks_add(&C, de * de / B);
        ks_add(&C, lambda_f * ks_val(&fs) / (3.0 * ns) / B);
      } else {
        double de = E - e_ref[s];
        ks_add(&C, 0.5 * de * de);
        ks_add(&C, 0.5 * lambda_f * ks_val(&fs));
      }
    }
    free(F);
  }
  if (st == ORC_OK) *loss = ks_val(&C);
  return st;
}

/* Gradient of phi = eps*E - (dE/dx0 . udot) w.r.t. the parameters of one net,
 * accumulated into grad (params layout).  xs holds the forward activations and
 * udot = scale * u is the tangent of the network input. */
static void net_double_backprop(const orc_net* net, double** xs, const double* udot, double eps,
                                double* grad, double* scratch) {
  const int Lw = net->n_layers;
  int maxw = net_maxw(net);
  /* scratch: tangents xd[l] (Lw+1 rows), adjoints a, t and their next-layer copies */
  double* xd = scratch;                                 /* (Lw+1) * maxw */
  double* zd = xd + (size_t)(Lw + 1) * maxw;            /* (Lw+1) * maxw: zdot per layer */
  double* a = zd + (size_t)(Lw + 1) * maxw;             /* maxw */
  double* t = a + maxw;                                 /* maxw */
  double* a2 = t + maxw;
  double* t2 = a2 + maxw;
  size_t off[64];
  size_t o = 0;
  for (int l = 0; l < Lw; ++l) { off[l] = o; o += (size_t)net->widths[l + 1] * (net->widths[l] + 1); }
  /* tangent forward: zdot_l = W_l xdot_{l-1}, xdot_l = f'(z_l) zdot_l */
  for (int k = 0; k < net->widths[0]; ++k) xd[k] = udot[k];
  for (int l = 0; l < Lw; ++l) {
    int nin = net->widths[l], nout = net->widths[l + 1];
    const double* W = net->params + off[l];
    for (int q = 0; q < nout; ++q) {
      double z = 0.0;
      for (int k = 0; k < nin; ++k) z += W[(size_t)q * nin + k] * xd[(size_t)l * maxw + k];
      zd[(size_t)(l + 1) * maxw + q] = z;
      xd[(size_t)(l + 1) * maxw + q] = act_d1(net->act[l], xs[l + 1][q]) * z;
    }
  }
  /* reverse over (x, xdot): adjoints start at d phi/d x_L = eps, d phi/d xdot_L = -1 */
  a[0] = eps;
  t[0] = -1.0;
  for (int l = Lw - 1; l >= 0; --l) {
    int nin = net->widths[l], nout = net->widths[l + 1];
    const double* W = net->params + off[l];
    double* gW = grad + off[l];
    double* gb = gW + (size_t)nout * nin;
    for (int k = 0; k < nin; ++k) { a2[k] = 0.0; t2[k] = 0.0; }
    for (int q = 0; q < nout; ++q) {
      double x = xs[l + 1][q];
      double d1 = act_d1(net->act[l], x), d2 = act_d2(net->act[l], x);
      double zdot = zd[(size_t)(l + 1) * maxw + q];
      double zbar = a[q] * d1 + t[q] * d2 * zdot;
      double zdbar = t[q] * d1;
      for (int k = 0; k < nin; ++k) {
        gW[(size_t)q * nin + k] += zbar * xs[l][k] + zdbar * xd[(size_t)l * maxw + k];
        a2[k] += W[(size_t)q * nin + k] * zbar;
        t2[k] += W[(size_t)q * nin + k] * zdbar;
      }
      gb[q] += zbar;
    }
    for (int k = 0; k < nin; ++k) { a[k] = a2[k]; t[k] = t2[k]; }
  }
}

int orc_loss_grad(const orc_model* m, int B, const int* offsets, const double* pos,
                  const int* species, const double* boxes, const int* pbc,
                  const double* e_ref, const double* f_ref, double lambda_f, int form,
                  double* loss, double* grad) {
  int st = check_model(m);
  if (st) return st;
  if (form != 0 && form != 1) return ORC_E_INVALID;
  if ((st = check_batch(m, B, offsets, species))) return st;
  layout L = make_layout(m);
  size_t poff[64];
  size_t np = 0;
  int maxw = 1, maxl = 1;
  for (int t = 0; t < m->n_species; ++t) {
    poff[t] = np;
    np += (size_t)orc_net_nparams(&m->nets[t]);
    if (net_maxw(&m->nets[t]) > maxw) maxw = net_maxw(&m->nets[t]);
    if (m->nets[t].n_layers > maxl) maxl = m->nets[t].n_layers;
  }
  for (size_t k = 0; k < np; ++k) grad[k] = 0.0;
  double* scratch = (double*)malloc(sizeof(double) * ((size_t)(2 * (maxl + 1) + 4) * maxw));
  double* u = (double*)malloc(sizeof(double) * (size_t)L.D);
  double* ud = (double*)malloc(sizeof(double) * (size_t)L.D);
  if (!scratch || !u || !ud) { free(scratch); free(u); free(ud); return ORC_E_NOMEM; }
  ksum C = {0.0, 0.0};
  for (int s = 0; s < B && st == ORC_OK; ++s) {
    const int a0 = offsets[s], ns = offsets[s + 1] - offsets[s];
    const double* ps = pos + 3 * (size_t)a0;
    const int* sp = species + a0;
    double* F = (double*)malloc(sizeof(double) * 3 * (size_t)ns);
    double* adj = (double*)malloc(sizeof(double) * 3 * (size_t)ns);
    double E = 0.0;
    st = orc_energy_forces(m, ns, ps, sp, boxes + 3 * s, pbc, &E, NULL, F, NULL);
    if (st) { free(F); free(adj); break; }
    /* loss value and its adjoints w.r.t. E_s (eps) and F (adj) */
    ksum fs = {0.0, 0.0};
    for (int k = 0; k < 3 * ns; ++k) {
      double df = F[k] - f_ref[3 * (size_t)a0 + k];
      ks_add(&fs, df * df);
      adj[k] = form == 0 ? 2.0 * lambda_f * df / (3.0 * ns) / B : lambda_f * df;
    }
    double eps;
    if (form == 0) {
      double de = (E - e_ref[s]) / ns;
      ks_add(&C, de * de / B);
      ks_add(&C, lambda_f * ks_val(&fs) / (3.0 * ns) / B);
      eps = 2.0 * de / ns / B;
    } else {
      double de = E - e_ref[s];
      ks_add(&C, 0.5 * de * de);
      ks_add(&C, 0.5 * lambda_f * ks_val(&fs));
      eps = de;
    }
    /* per atom: u_i = J_i adj, then the double back-propagation */
    work w;
    st = work_init(m, ns, ps, boxes + 3 * s, pbc, &w);
    int maxne = 0;
    for (int i = 0; st == ORC_OK && i < ns; ++i)
      if (w.nl.start[i + 1] - w.nl.start[i] > maxne) maxne = w.nl.start[i + 1] - w.nl.start[i];
    double* Je = (double*)malloc(sizeof(double) * (size_t)L.D * 3 * (size_t)(maxne > 0 ? maxne : 1));
    if (!Je && st == ORC_OK) st = ORC_E_NOMEM;
    for (int i = 0; st == ORC_OK && i < ns; ++i) {
      const entry* e = &w.nl.e[w.nl.start[i]];
      int ne = w.nl.start[i + 1] - w.nl.start[i];
      atom_descriptor(m, &L, e, ne, sp, w.G, w.T);
      const orc_net* net = &m->nets[sp[i]];
      net_forward(net, w.G, w.ws.xs);
      entry_jacobian(m, &L, e, ne, sp, Je, w.T, w.dT);
      for (int a = 0; a < L.D; ++a) {
        double acc = 0.0;
        for (int p = 0; p < ne; ++p)
          for (int c = 0; c < 3; ++c)
            acc += Je[(size_t)a * 3 * ne + 3 * p + c] * (adj[3 * e[p].j + c] - adj[3 * i + c]);
        u[a] = acc;
        ud[a] = acc * (net->scale ? net->scale[a] : 1.0);
      }
      net_double_backprop(net, w.ws.xs, ud, eps, grad + poff[sp[i]], scratch);
    }
    free(Je);
    work_free(m, &w);
    free(F);
    free(adj);
  }
  free(scratch);
  free(u);
  free(ud);
  if (st == ORC_OK) *loss = ks_val(&C);
  return st;
}
