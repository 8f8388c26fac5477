/*
 * aenet_oracle.h -- interface of the FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This header belongs to the oracle and is used by
 * nothing but the oracle's own C file and its ctypes wrapper (oracle/__init__.py).
 * The GPU library has its own header (include/aenet_gpu.h); the two share no
 * code, constants or helpers.
 *
 * Units are metal units (eV, Angstrom, amu, ps), the unit system the paper's
 * LAMMPS input uses (Sec. III, LAMMPS example).  Positions are [n x 3]
 * row-major.  Boxes are orthorhombic, edge lengths box[3]; pbc[a] != 0 means
 * axis a is periodic.  All routines return 0 on success and a negative code on
 * error (ORC_E_*).
 */
#ifndef AENET_ORACLE_H
#define AENET_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_E_INVALID (-1)
#define ORC_E_OVERLAP (-4)
#define ORC_E_NOMEM (-7)
#define ORC_E_CAPACITY (-8)

#define ORC_ACT_LINEAR 0
#define ORC_ACT_TANH 1

/* One atomic network ANN_t (Eq. 1): n_layers weight layers, widths[0] = D,
 * widths[n_layers] = 1.  params holds, layer after layer, W[l] (row-major,
 * widths[l+1] x widths[l]) followed by b[l] (widths[l+1]).  The network input
 * is x0 = (G - shift) * scale (shift/scale may be NULL = 0 / 1). */
typedef struct {
  int n_layers;
  const int* widths;
  const int* act;
  const double* params;
  const double* shift;
  const double* scale;
  double e_offset;
} orc_net;

/* The whole potential: Chebyshev descriptor setup (Eqs. 3-6) plus one net per
 * species (Eq. 2).  type_weight[t] is the weight of species t in the
 * species-weighted descriptor channel (used only when n_species > 1). */
typedef struct {
  int n_species;
  const double* type_weight;
  int radial_order;
  double radial_cutoff;
  int angular_order;
  double angular_cutoff;
  const orc_net* nets;
} orc_model;

/* Building blocks, exposed for the tests. */
void orc_chebyshev(int order, double x, double* T, double* dT);
void orc_cutoff(double r, double rc, double* fc, double* dfc);
int orc_descriptor_dim(int n_species, int radial_order, int angular_order);
int orc_net_nparams(const orc_net* net);
/* E = ANN(x0(G)) and g = dE/dG for one atom. */
int orc_net_eval(const orc_net* net, const double* G, double* E, double* g);

/* Brute-force neighbour enumeration (all atom/image pairs with r < cutoff,
 * excluding the atom itself in the home cell).  Entry k of atom i is written to
 * nbr_j[i*cap + k] and nbr_shift[(i*cap + k)*3 + a], the displacement being
 * d = r_j + shift*box - r_i with positions wrapped into [0, box) on periodic
 * axes.  counts[i] receives the number of entries; ORC_E_CAPACITY if any row
 * exceeds cap (counts are still complete). */
int orc_neighbors(int n, const double* pos, const double* box, const int* pbc,
                  double cutoff, int cap, int* counts, int* nbr_j, int* nbr_shift);

/* Descriptors G [n x D] (layout rad_typ | ang_typ | rad_wt | ang_wt). */
int orc_descriptors(const orc_model* m, int n, const double* pos, const int* species,
                    const double* box, const int* pbc, double* G);

/* Energy and forces by the pairwise chain rule.  e_atom, forces, G may be NULL. */
int orc_energy_forces(const orc_model* m, int n, const double* pos, const int* species,
                      const double* box, const int* pbc, double* e_total, double* e_atom,
                      double* forces, double* G);

/* The same and the virial W [3 x 3] (row-major, eV): W_ab = -dE/d eps_ab for
 * the homogeneous strain r -> (1 + eps) r of positions and box, i.e.
 * W_ab = -sum_i sum_e (dE_i/dd_e)_a (d_e)_b over every neighbour entry e of
 * every atom i (d_e = r_j + image shift - r_i); the pressure of the
 * configuration is (N k T + tr W / 3) / V.  virial may be NULL. */
int orc_energy_forces_virial(const orc_model* m, int n, const double* pos, const int* species,
                             const double* box, const int* pbc, double* e_total, double* e_atom,
                             double* forces, double* G, double* virial);

/* E_m, F_m (and G_m if g_sel != NULL) of the n_sel atoms listed in sel only,
 * for structures too large for a full evaluation; e_sel [n_sel], f_sel
 * [n_sel x 3], g_sel [n_sel x D]. */
int orc_energy_forces_subset(const orc_model* m, int n, const double* pos, const int* species,
                             const double* box, const int* pbc, int n_sel, const int* sel,
                             double* e_sel, double* f_sel, double* g_sel);

/* Forces by the second formulation: dense Jacobians J_i = dG_i/dr, F = -sum J_i^T g_i.
 * Memory is O(n * D) per atom; meant for small systems. */
int orc_forces_dense(const orc_model* m, int n, const double* pos, const int* species,
                     const double* box, const int* pbc, double* forces);

/* Velocity Verlet (NVE) in metal units: n_steps steps of size dt (ps).  pos and
 * vel (A/ps) are updated in place, positions wrapped after every drift.
 * masses[t] in amu.  On return e_pot, e_kin (eV) and forces (may be NULL)
 * describe the final state. */
int orc_md_vv(const orc_model* m, int n, double* pos, double* vel, const int* species,
              const double* masses, const double* box, const int* pbc, double dt,
              int n_steps, double* e_pot, double* e_kin, double* forces);

/* Energy+force loss over a batch of B independent structures.  Structure s owns
 * atoms [offsets[s], offsets[s+1]) of pos/species/F_ref, box boxes[3s..3s+2] and
 * shares pbc.  Two forms:
 *   form 0 (per-atom mean):  C = (1/B) sum_s [((E_s-Eref_s)/N_s)^2
 *                                             + lambda_f/(3 N_s) sum_{i in s} |F_i-Fref_i|^2]
 *   form 1 (Eq. 7 as printed, Sec. II C: half the sum of squared energy errors,
 *           with an optional force term of the same kind):
 *                            C = 1/2 sum_s (E_s-Eref_s)^2 + lambda_f/2 sum_i |F_i-Fref_i|^2
 * orc_loss_grad also writes dC/dparams (concatenated over species, each in the
 * orc_net params layout) computed analytically by double back-propagation. */
int orc_loss(const orc_model* m, int n_struct, const int* offsets, const double* pos,
             const int* species, const double* boxes, const int* pbc, const double* e_ref,
             const double* f_ref, double lambda_f, int form, double* loss);
int orc_loss_grad(const orc_model* m, int n_struct, const int* offsets, const double* pos,
                  const int* species, const double* boxes, const int* pbc,
                  const double* e_ref, const double* f_ref, double lambda_f, int form,
                  double* loss, double* grad);

#ifdef __cplusplus
}
#endif
#endif
