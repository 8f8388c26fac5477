/*
 * aenet_gpu.h -- C ABI of the MI355X (gfx950) ANN-potential molecular-dynamics
 * library: Behler-Parrinello atomic neural networks on Chebyshev descriptors
 * (arXiv:2107.11311, Sec. II), with GPU neighbour lists, force
 * back-propagation, velocity-Verlet MD and the gradient of a training loss.
 *
 * Conventions shared by every call
 *   - Units are metal units: energies in eV, lengths in Angstrom, masses in
 *     amu, time in ps, velocities in A/ps, forces in eV/A (the unit system of
 *     the paper's LAMMPS example, Sec. III).
 *   - Positions, velocities and forces are [n x 3] row-major float64 arrays in
 *     the caller's atom order.  Species are int32 ids 0..S-1 in the order of
 *     the networks given to aenet_setup (one network per species, Sec. II A,
 *     Eq. 2).  Species arrays are always HOST memory, also in the _dev calls.
 *   - Boxes are orthorhombic: box[3] edge lengths (A), pbc[3] non-zero for a
 *     periodic axis.  On a periodic axis every edge must be at least the
 *     neighbour-list radius max(R_r, R_a) + skin (else AENET_E_BOX); images
 *     are handled exactly, also for edges shorter than twice the cutoff.  On a
 *     non-periodic axis atoms may lie anywhere.
 *   - "host" pointers are ordinary CPU memory; "_dev" calls take device
 *     pointers and a hipStream_t (passed as void*, NULL = default stream) and
 *     synchronise that stream before returning.
 *   - Every call returns an aenet_status.  On error the outputs are left
 *     untouched and aenet_last_error() describes the failure.  No call aborts
 *     or throws across the ABI.
 *   - Ownership: aenet_setup deep-copies the model; the caller may free its
 *     arrays afterwards.  Outputs are always caller-allocated.  A context is
 *     used by one host thread at a time.
 */
#ifndef AENET_GPU_H
#define AENET_GPU_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct aenet_ctx aenet_ctx;

typedef enum {
  AENET_OK = 0,
  AENET_E_INVALID = -1,   /* bad argument or unsupported model shape */
  AENET_E_SPECIES = -2,   /* species id outside 0..S-1 */
  AENET_E_BOX = -3,       /* periodic edge shorter than the neighbour-list radius */
  AENET_E_OVERLAP = -4,   /* two distinct atom/image entries at distance 0 */
  AENET_E_NONFINITE = -5, /* NaN/Inf in the inputs or the results */
  AENET_E_DEVICE = -6,    /* HIP runtime error */
  AENET_E_OOM = -7        /* device allocation failed */
} aenet_status;

/* Arithmetic of the hot path.  AENET_FP64: everything in float64.
 * AENET_FP32: descriptor terms and the networks in float32 (networks on FP32
 * MFMA), displacements, per-atom force sums, energies and the integrator in
 * float64.  AENET_BF16: as FP32, with the network weights rounded to
 * bfloat16 (round to nearest even) on BF16 MFMA with float32 accumulation,
 * except the input layer, whose weights are kept as a pair of bfloat16 values
 * (the weight rounded, and its rounding error rounded); the float32
 * activations and deltas enter the MFMA as such a pair too. */
typedef enum { AENET_FP64 = 0, AENET_FP32 = 1, AENET_BF16 = 2 } aenet_precision;

typedef enum { AENET_ACT_LINEAR = 0, AENET_ACT_TANH = 1 } aenet_act;

/* One atomic network ANN_t (Sec. II A, Eq. 1): x_l = f_l(W_l x_{l-1} + b_l),
 * x_0 = (G - in_shift) * in_scale, E_i = x_L + e_offset.  n_layers weight
 * layers (1..AENET_MAX_LAYERS), widths[0] = descriptor dimension D,
 * widths[n_layers] = 1, every width <= AENET_MAX_WIDTH.  W[l] is row-major
 * [widths[l+1] x widths[l]], b[l] has widths[l+1] entries.  in_shift/in_scale
 * may be NULL (0 / 1).  All species have the same number of layers and the
 * same activations; their hidden widths may differ (internally every species
 * runs at the largest width of each layer, the extra units with zero weights
 * and biases, which leaves every energy and force unchanged). */
#define AENET_MAX_LAYERS 4
#define AENET_MAX_WIDTH 64
typedef struct {
  int n_layers;
  const int* widths;
  const int* act;
  const double* const* W;
  const double* const* b;
  const double* in_shift;
  const double* in_scale;
  double e_offset;
} aenet_net;

/* The potential (Sec. II): Chebyshev radial expansion of order radial_order
 * within radial_cutoff (Eq. 3), angular expansion of order angular_order
 * within angular_cutoff (Eq. 6), cosine cutoff (Eq. 5).  Order N gives N+1
 * coefficients.  With S > 1 species the descriptor has a typed half (every
 * neighbour weight 1) and a species-weighted half (radial weight
 * type_weight[t_j], angular weight type_weight[t_j]*type_weight[t_k]):
 * G = [rad_typ (N_r+1) | ang_typ (N_a+1) | rad_wt (N_r+1) | ang_wt (N_a+1)],
 * D = 2(N_r+1) + 2(N_a+1); with S = 1 only the typed half (D = N_r+N_a+2).
 * The angular sum runs over ordered pairs of distinct neighbours.
 * Orders: any pair that some compiled pair (aenet_supported_orders) reaches
 * in both orders; the model then runs on the smallest such pair, whose
 * descriptor holds the model's as a subset (same cutoffs, the lower orders of
 * each block), with the other components entering the networks with zero
 * weight (exact, at that pair's cost).  The pair's descriptor dimension must
 * not exceed AENET_MAX_WIDTH (the networks' input layer): with S > 1 species
 * orders up to 20 / 10 are reached, with one species up to 24 / 12.  Other
 * orders give AENET_E_INVALID.  mass_amu is used by MD.
 * skin (A) enlarges the neighbour list so it is rebuilt only when an atom
 * has moved more than skin/2 (0 = rebuild every evaluation).  device is the
 * HIP device index. */
typedef struct {
  int n_species;
  const double* mass_amu;
  const double* type_weight;
  int radial_order;
  double radial_cutoff;
  int angular_order;
  double angular_cutoff;
  const aenet_net* nets;
  int precision;
  double skin;
  int device;
} aenet_model;

/* Creates a context for the model (validates, deep-copies, packs the
 * per-precision network operands).  Device buffers are allocated on first
 * use and grown as needed. */
aenet_status aenet_setup(const aenet_model* model, aenet_ctx** out);

/* Releases the context and all its device memory.  NULL is ignored. */
void aenet_destroy(aenet_ctx* ctx);

/* Message of the last failure on this context ("" if none); with ctx == NULL
 * the reason the calling thread's last aenet_setup failed.  Valid until the
 * next call on the context (or the next aenet_setup of the thread). */
const char* aenet_last_error(const aenet_ctx* ctx);

/* Descriptor dimension D of the model. */
int aenet_descriptor_dim(const aenet_ctx* ctx);

/* Number of trainable parameters: for every species in order, for every
 * layer, W[l] row-major then b[l] (in_shift/in_scale/e_offset excluded). */
int64_t aenet_n_params(const aenet_ctx* ctx);

/* Copies out / replaces the trainable parameters (flat layout above, host). */
aenet_status aenet_get_params(aenet_ctx* ctx, double* params);
aenet_status aenet_set_params(aenet_ctx* ctx, const double* params);

/* Writes into orders[2*k], orders[2*k+1] the (radial, angular) order pairs the
 * library was compiled for; returns their count (at most max_pairs written).
 * A model's orders (N_r, N_a) are accepted when some pair has both orders at
 * least as large. */
int aenet_supported_orders(int* orders, int max_pairs);

/* Total energy E = sum_i E_i (Sec. II A, Eq. 2), per-atom energies and forces
 * F = -dE/dr of one structure of n atoms.  e_atom and forces may be NULL. */
aenet_status aenet_energy_forces(aenet_ctx* ctx, int64_t n, const double* pos,
                                 const int32_t* species, const double box[3],
                                 const uint8_t pbc[3], double* e_total, double* e_atom,
                                 double* forces);

/* The same (host buffers) and the virial of the configuration, the stress
 * tensor of the whole system that the paper's earlier LAMMPS interface
 * provides (Sec. III): virial[3a+b] = W_ab = -dE/d eps_ab under the
 * homogeneous strain r -> (1 + eps) r of positions and box, formed as
 * -sum_i sum_e (dE_i/dd_e)_a (d_e)_b over every neighbour entry e of every
 * atom i (d_e = r_j + image shift - r_i), in eV; the pressure is
 * (N k T + (W_xx + W_yy + W_zz) / 3) / V.  Summed in a fixed order
 * (deterministic).  virial (9 doubles, row-major) must not be NULL; forces
 * may be NULL. */
aenet_status aenet_energy_forces_virial(aenet_ctx* ctx, int64_t n, const double* pos,
                                        const int32_t* species, const double box[3],
                                        const uint8_t pbc[3], double* e_total, double* forces,
                                        double virial[9]);

/* aenet_energy_forces_virial with device pointers (pos, e_total[1] or NULL,
 * forces or NULL, virial[9]) and a stream. */
aenet_status aenet_energy_forces_virial_dev(aenet_ctx* ctx, int64_t n, const double* pos,
                                            const int32_t* species, const double box[3],
                                            const uint8_t pbc[3], double* e_total, double* forces,
                                            double* virial, void* stream);

/* Same with device pointers (pos, e_total[1], e_atom, forces) and a stream. */
aenet_status aenet_energy_forces_dev(aenet_ctx* ctx, int64_t n, const double* pos,
                                     const int32_t* species, const double box[3],
                                     const uint8_t pbc[3], double* e_total, double* e_atom,
                                     double* forces, void* stream);

/* Independent structures evaluated in one launch: structure s owns atoms
 * [offsets[s], offsets[s+1]) (offsets: host, n_struct+1 entries, offsets[0]=0)
 * and box boxes[3s..3s+2]; pbc is shared.  e_struct[n_struct] (may be NULL),
 * e_atom and forces (may be NULL) in the caller's order.  Device pointers. */
aenet_status aenet_energy_forces_batch_dev(aenet_ctx* ctx, int n_struct, const int64_t* offsets,
                                           const double* pos, const int32_t* species,
                                           const double* boxes, const uint8_t pbc[3],
                                           double* e_struct, double* e_atom, double* forces,
                                           void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * results as aenet_energy_forces_dev (device pointers pos, e_total[1], e_atom,
 * forces, and a stream), computed by the same kernels, with every temporary
 * buffer (atom order, neighbour rows, per-entry gradients, descriptor
 * gradients, sums) carved from one fixed device array of
 * AENET_NOALLOC_WORKSPACE_BYTES per GPU instead of allocated.  The array is
 * reserved when the library is loaded onto a GPU and kept until the process
 * ends; the call itself allocates no device memory (the model's buffers were
 * allocated by aenet_setup).  A structure whose buffers do not fit returns
 * AENET_E_INVALID with the workspace size in the message (roughly 10,000 atoms
 * of water at a 6 A cutoff in FP64).  All contexts on one GPU share the array,
 * so calls that overlap in time on one GPU (different threads, or streams
 * not ordered with each other) race: the caller serialises them.  Nothing of
 * one call's workspace contents is reused by the next (every counter the
 * kernels need at zero is cleared by the call).  The context's own buffers
 * are not touched; a following aenet_md_step starts from its inputs. */
#define AENET_NOALLOC_WORKSPACE_BYTES (64u << 20)
aenet_status aenet_energy_forces_noalloc(aenet_ctx* ctx, int64_t n, const double* pos,
                                         const int32_t* species, const double box[3],
                                         const uint8_t pbc[3], double* e_total, double* e_atom,
                                         double* forces, void* stream);

/* Descriptor vectors G [n x D] (layout of aenet_model), host pointers. */
aenet_status aenet_descriptors(aenet_ctx* ctx, int64_t n, const double* pos,
                               const int32_t* species, const double box[3],
                               const uint8_t pbc[3], double* G);

/* Velocity-Verlet NVE molecular dynamics (the MD cycle of Fig. 1): n_steps
 * steps of dt_ps.  Each step: v += dt/2 F/m; r += dt v; (neighbour list
 * rebuilt when an atom moved more than skin/2 since the last build, and every
 * rebuild_every steps); F = F(r); v += dt/2 F/m.  pos and vel are read at
 * entry and overwritten at exit (positions wrapped into the box on periodic
 * axes).  The forces at the input positions are computed first, unless the
 * positions are bitwise those this context wrote at the end of its previous
 * md_step call, with the same species and box and no other call on the
 * context since that could change them (energy/force, descriptor or training
 * calls, new parameters or capacities): then the forces and neighbour list of
 * that call's end are taken over (the velocities are always read, so a
 * thermostat may rescale them between calls).  That comparison runs on the
 * device.  When aenet_md_step_dev is handed the very buffer its previous call
 * wrote, the call goes on as if the comparison held; if the positions
 * differ, the steps done meanwhile are discarded (nothing of them reaches
 * the outputs) and the call starts over from its inputs, so a caller that
 * edits that buffer between calls gets the same result at the cost of up to
 * rebuild_every discarded steps.  Otherwise the comparison is read before
 * the first step.  e_pot/e_kin (may be NULL) receive the final
 * potential and kinetic energy (eV); forces (may be NULL) the final forces.
 * On an error (a non-finite input, overlapping atoms, ...) pos, vel,
 * e_pot, e_kin and forces are left as they were.  State lives on the device
 * for the whole call. */
aenet_status aenet_md_step(aenet_ctx* ctx, int64_t n, double* pos, double* vel,
                           const int32_t* species, const double box[3], const uint8_t pbc[3],
                           double dt_ps, int n_steps, double* e_pot, double* e_kin,
                           double* forces);

/* Same with device pointers for pos, vel, e_pot[1], e_kin[1], forces. */
aenet_status aenet_md_step_dev(aenet_ctx* ctx, int64_t n, double* pos, double* vel,
                               const int32_t* species, const double box[3],
                               const uint8_t pbc[3], double dt_ps, int n_steps, double* e_pot,
                               double* e_kin, double* forces, void* stream);

/* Training loss over a batch of B structures and its gradient w.r.t. all
 * parameters (training, Sec. II C).  Two forms (aenet_set_loss_form):
 *   AENET_LOSS_MEAN_PER_ATOM (default):
 *     C = (1/B) sum_s [ ((E_s - e_ref_s)/N_s)^2 + lambda_f/(3 N_s) sum_{i in s} |F_i - f_ref_i|^2 ]
 *   AENET_LOSS_EQ7 (Eq. 7 as printed, half the sum of squared energy errors,
 *   with a force term of the same kind when lambda_f > 0):
 *     C = 1/2 sum_s (E_s - e_ref_s)^2 + lambda_f/2 sum_i |F_i - f_ref_i|^2
 * The gradient is obtained by double back-propagation (a descriptor
 * Jacobian-vector product followed by a reverse pass through the network and
 * its tangent).  Batch layout as aenet_energy_forces_batch_dev; e_ref [B],
 * f_ref [n x 3], loss [1], grad [aenet_n_params] are device pointers.
 * FP64 and FP32 contexts only. */
aenet_status aenet_loss_grad_dev(aenet_ctx* ctx, int n_struct, const int64_t* offsets,
                                 const double* pos, const int32_t* species, const double* boxes,
                                 const uint8_t pbc[3], const double* e_ref, const double* f_ref,
                                 double lambda_f, double* loss, double* grad, void* stream);

/* The same with host pointers (pos [n x 3], e_ref [B], f_ref [n x 3], loss
 * [1], grad [aenet_n_params]). */
aenet_status aenet_loss_grad(aenet_ctx* ctx, int n_struct, const int64_t* offsets,
                             const double* pos, const int32_t* species, const double* boxes,
                             const uint8_t pbc[3], const double* e_ref, const double* f_ref,
                             double lambda_f, double* loss, double* grad);

/* Root-mean-square difference sqrt(sum_k (a_k - b_k)^2 / n) of two float64
 * device arrays of n values (the force RMSE of a distilled network against
 * its teacher, 3 values per atom), summed in a fixed order; out is a device
 * pointer to one double.  Uses the context only for scratch memory. */
aenet_status aenet_rms_diff_dev(aenet_ctx* ctx, int64_t n, const double* a, const double* b, double* out,
                                void* stream);

/* Selects the loss form of the following aenet_loss_grad[_dev] calls. */
typedef enum { AENET_LOSS_MEAN_PER_ATOM = 0, AENET_LOSS_EQ7 = 1 } aenet_loss_form;
aenet_status aenet_set_loss_form(aenet_ctx* ctx, int form);

/* Replaces the parameters from DEVICE memory (flat layout of aenet_n_params,
 * float64), repacking the network operands on the device: training loops keep
 * parameters, gradients and optimiser state on the GPU with no host round
 * trip.  FP64 and FP32 contexts (AENET_E_INVALID for BF16); AENET_E_NONFINITE
 * (parameters unchanged) if any value is NaN/Inf.  aenet_get_params returns
 * the values set here. */
aenet_status aenet_set_params_dev(aenet_ctx* ctx, const double* params, void* stream);

/* One Adam step (Kingma and Ba, 2015) on n float64 device values:
 *   m = beta1 m + (1 - beta1) g;  v = beta2 v + (1 - beta2) g^2;
 *   p -= lr (m / (1 - beta1^step)) / (sqrt(v / (1 - beta2^step)) + eps)
 * step >= 1 counts the updates so far including this one.  Device pointers,
 * updated in place; synchronises the stream.  Context-free. */
aenet_status aenet_adam_step_dev(int64_t n, double* params, const double* grad, double* m, double* v,
                                 double lr, double beta1, double beta2, double eps, int64_t step,
                                 void* stream);

/* Tuning / diagnostics. */
typedef struct {
  int64_t n_rebuilds;     /* neighbour-list builds since setup */
  int64_t n_capacity_retries;
  int row_capacity;       /* neighbour entries reserved per atom */
  int ang_capacity;       /* angular entries reserved per atom */
  int max_neighbors;      /* largest row seen in the last build */
  int max_angular;        /* largest angular prefix seen in the last build */
  int rebuild_every;      /* forced rebuild interval of md_step (steps) */
  int deterministic;      /* 1: forces by deterministic gather (default) */
} aenet_stats;
aenet_status aenet_get_stats(const aenet_ctx* ctx, aenet_stats* out);
/* rebuild_every >= 1 (default 50). */
aenet_status aenet_set_rebuild_every(aenet_ctx* ctx, int rebuild_every);
/* Descriptor forward pass and networks in one kernel, per 16-atom tile
 * (enable = 1, where it applies: up to 48 expected angular neighbours and
 * 64 KiB of LDS per tile), or as two kernels (enable = 0).  The results are
 * bitwise the same.  Default: 1. */
aenet_status aenet_set_fused(aenet_ctx* ctx, int enable);
/* How the angular terms of Eq. 6 are evaluated.  AENET_ANGULAR_PAIRS: the
 * sum over pairs of angular neighbours as written (cost ~ n_a^2 per atom).
 * AENET_ANGULAR_FACTORISED: T_a expanded in Legendre polynomials and each
 * P_l(cos theta_jk) split by the addition theorem into products of functions
 * of u_j and of u_k, so the pair sum becomes squares of single sums over the
 * neighbours minus the j = k terms (cost ~ n_a (N_a + 1)^2 per atom; angular
 * orders 2, 3, 4, 6 and 8).  The results are the same up to rounding.
 * AENET_ANGULAR_AUTO (default): factorised when more than 48 neighbours are
 * expected within R_a. */
typedef enum {
  AENET_ANGULAR_AUTO = 0,
  AENET_ANGULAR_PAIRS = 1,
  AENET_ANGULAR_FACTORISED = 2
} aenet_angular_method;
aenet_status aenet_set_angular_method(aenet_ctx* ctx, int method);

/* Neighbour-row capacities used from the next call on: row_capacity entries
 * per atom within R_r + skin, ang_capacity of them within R_a + skin
 * (1 <= ang_capacity <= row_capacity, ang_capacity <= 700, row_capacity <=
 * 4096).  Rows grow by themselves when a build overflows them (the build, or
 * the MD chunk since the last checkpoint, is redone), so this only sets the
 * starting point: a caller who knows the densest environment avoids the
 * retry, and small values exercise it.  (0, 0) returns to the estimate from
 * the number density.  AENET_E_INVALID for other values. */
aenet_status aenet_set_capacity(aenet_ctx* ctx, int row_capacity, int ang_capacity);

/* Kernel timing (diagnostics).  While enabled, every launch of a hot-path
 * kernel is bracketed by HIP events on the stream it is launched on, and
 * aenet_get_kernel_times returns, per kernel class, the summed duration (ms)
 * and the launch count since the last call (then resets them).  Both arrays
 * have AENET_K_COUNT entries (host memory). */
typedef enum {
  AENET_K_NEIGHBOR = 0,     /* cell-list neighbour build (all its kernels) */
  AENET_K_DESC_FWD = 1,     /* descriptor forward, Eqs. 3-6 */
  AENET_K_NETWORK = 2,      /* atomic networks, Eq. 1 (+ input gradient) */
  AENET_K_DESC_BWD = 3,     /* force back-propagation to entry gradients */
  AENET_K_FORCE_GATHER = 4, /* deterministic force gather (+ closing half kick) */
  AENET_K_INTEGRATE = 5,    /* opening half kick + drift */
  AENET_K_FWD_NETWORK = 6,  /* descriptor forward and networks in one kernel */
  AENET_K_COUNT = 7
} aenet_kernel_class;
aenet_status aenet_set_profiling(aenet_ctx* ctx, int enable);
aenet_status aenet_get_kernel_times(aenet_ctx* ctx, double* ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif
