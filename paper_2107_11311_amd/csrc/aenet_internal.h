// aenet_internal.h -- declarations shared by the translation units of the
// GPU library (host runtime + kernels).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace aenet {

constexpr int kMaxSpecies = 8;
constexpr double kPi = 3.14159265358979323846;
constexpr int kMaxLayers = 4;  // weight layers
constexpr int kMaxWidth = 64;
constexpr int kPad = 32;       // every network width is padded to a multiple of this

// A neighbour entry packs the neighbour's internal atom index (low 27 bits)
// with its periodic-image code (high 5 bits): code = (sx+1) + 3(sy+1) + 9(sz+1)
// for an image shift s in {-1,0,1}^3, displacement d = r_j + s*L - r_i.
constexpr int kImgBits = 27;
constexpr uint32_t kAtomMask = (1u << kImgBits) - 1u;
constexpr int64_t kMaxAtoms = (int64_t)kAtomMask;

// device status flags (bitmask in ctx flags word)
constexpr int kFlagOverflow = 1;   // a neighbour row exceeded its capacity
constexpr int kFlagOverlap = 2;    // two distinct entries at distance 0
constexpr int kFlagReverse = 4;    // reverse entry not found (asymmetric list)
constexpr int kFlagNonFinite = 8;  // NaN/Inf in positions

struct BoxInfo {
  double L[3];
  int nc[3];      // cells per axis
  int cell_base;  // first global cell id of this structure
};

// x wrapped into [0, L); a wrapped value maps to itself exactly
__device__ inline double wrap_coord(double x, double L) {
  double w = x - L * floor(x / L);
  if (w >= L) w -= L;
  if (w < 0.0) w = 0.0;
  return w;
}

// global cell of a position (periodic axes wrapped first; non-finite or
// outside coordinates are clamped into the grid)
__device__ inline int cell_of(const BoxInfo& b, const int pbc[3], const double x[3]) {
  int c[3];
  for (int a = 0; a < 3; ++a) {
    const double w = pbc[a] ? wrap_coord(x[a], b.L[a]) : x[a];
    double fc = floor(w * (double)b.nc[a] / b.L[a]);
    fc = fmin(fmax(fc, 0.0), (double)(b.nc[a] - 1));
    c[a] = (int)fc;
  }
  return b.cell_base + (c[2] * b.nc[1] + c[1]) * b.nc[0] + c[0];
}

// ---------------------------------------------------------------- neighbour list
struct NbrParams {
  int n;                 // atoms
  double* pos;           // [n*3] internal order (wrapped in place by k_bin)
  double* pos_ref;       // [n*3] positions at the last build
  const int* seg;        // [n] structure id
  const BoxInfo* boxes;  // [n_struct]
  int n_struct;
  int pbc[3];
  int n_cells;
  int tp;                // candidates per cell neighbourhood held in LDS (power of
                         // two) by the per-cell row kernel; 0: per-atom kernels
  double r_list2;        // (max(R_r,R_a) + skin)^2
  double r_ang2;         // (R_a + skin)^2
  int cap, cap_ang;
  int* cell_count;       // [n_cells]
  int* cell_start;       // [n_cells+1]
  int* cell_fill;        // [n_cells]
  int* cell_atoms;       // [n]
  int* atom_cell;        // [n]
  uint32_t* nbr;         // [n*cap]
  uint16_t* segs;        // [n*kSegWords] row position where each stencil cell's
                         // entries start, per row part (see nbr.hip)
  int* nnb;              // [n]
  int* nang;             // [n]
  int* rev;              // [n*cap] global index of the reverse entry
  int* flags;
  int* maxcnt;           // [2] largest row, largest angular prefix
  int* cond;             // build only if *cond != 0 (NULL = always)
  int* go;               // [1] the decision of this build, for its later kernels
  int* ticket;           // [1] block counter of the binning kernel (0 between builds)
  // MD with the per-cell row kernel: the integrator has already put every
  // atom into a fixed-capacity cell bin (kCellAtomsMax slots), so the build is
  // the row kernel alone; it wraps the positions itself
  int binned;
  int* bin_count;        // [2][n_cells] atoms per cell, one half per step parity
  const int* bin_atoms;  // [n_cells][kCellAtomsMax]
  int bin_sel;           // half read by this build (the row kernel clears the other)
};
constexpr int kSegWords = 56;  // 2 row parts x 28 segment boundaries
constexpr int kRevPending = -2;  // rev values <= this are unresolved (rank, k)
constexpr int kCellAtomsMax = 128;  // atoms per cell the per-cell row kernel handles
constexpr int kRowWaves = 16;       // wavefronts per block of the per-cell row kernel
// LDS bytes of the per-cell row kernel for a candidate capacity tp: key,
// FP32 position and the two row parts' masks of every candidate, and each
// wavefront's staging row
inline size_t cell_rows_lds(int tp, int cap) {
  return (size_t)tp * (4 + 12 + 2 * (kCellAtomsMax / 32) * 4) + (size_t)kRowWaves * cap * 4;
}
void launch_build_neighbors(const NbrParams& p, hipStream_t s);
void launch_set_int(int* dst, int value, hipStream_t s);

// ---------------------------------------------------------------- descriptors
struct DescParams {
  int n;
  const double* pos;
  const int* species;
  const int* seg;
  const BoxInfo* boxes;
  const uint32_t* nbr;
  const int* nnb;
  const int* nang;
  int cap, cap_ang;
  int ang_hint;          // expected largest angular shell within R_a (tuning only)
  double rr, ra;
  // 2/R, pi/R and pi/(2R) of both cutoffs (computed once on the host)
  double two_rr, two_ra, pi_rr, pi_ra, pi_2rr, pi_2ra;
  const double* wq;      // [n] type weight of each atom's species (Sec. II B)
  double tw[kMaxSpecies];  // type weight per species
  int n_species;
  int weighted;          // n_species > 1
  int ldG;               // row stride of G / dE/dG
  void* G;               // [n x ldG] (float or double)
  const void* gG;        // dE/dG [n x ldG]
  int* rev;              // [n*cap] global index of the reverse entry, -1 if
                         // none, or kRevPending - (rank | k << 16) as left by
                         // the per-cell row build (resolved by the force pass)
  const uint16_t* segs;  // [n*kSegWords] segment starts of the rows
  // written by the forward pass, read by the force pass and the force
  // gather: per atom the row positions of the entries that contribute
  // (within R_r, or in the angular part; n_keep of them, from the front of
  // the atom's ridx row), and of those just beyond R_r (within a relative
  // margin of 1e-9 in r^2; n_margin of them, from the back), whose gradient
  // is zero but is still stored: the gather sums over its own n_keep entries,
  // and the reverse of each of them is among the stored ones even where the
  // two directions round r^2 differently.
  uint16_t* ridx;        // [n*cap]
  int* nrad;             // [n] n_keep | n_margin << 16
  int prio;              // set by the launcher: phase-wise wave priorities (see desc_dev.h)
  void* pg;              // [n*cap*3] dE_i/dd_e, stored at the slot of the
                         // reverse entry: pg[rev(i,e)] (see the force gather)
  double* Fself;         // [n*3]  sum_e dE_i/dd_e
  double* vir;           // [9][n] per-atom virial -sum_e (dE_i/dd_e)_a (d_e)_b
                         // (component 3a+b at vir[(3a+b) n + i]); NULL: none
  // factorised angular descriptor (angular.hip): t1 = N_r + 1 (first angular
  // component of G), t2 = N_r + N_a + 2 (offset of the weighted half);
  // shA [n x 2 (N_a+1)^2] the per-atom sums of the forward pass; gang
  // [n x cap_ang x 3] the angular part of dE_i/dd_e per angular row position
  int t1, t2;
  // the force pass's blocks: block k computes atom xmap[k] (-1: none); n_grid
  // blocks (the atoms in an XCD-aware order, see prepare())
  const int* xmap;
  int n_grid;
  void* shA;
  void* gang;
  const double* adj;     // [n*3] JVP direction (loss adjoint of the forces)
  void* U;               // [n x ldG] JVP output
  int* flags;
};
// prec: 0 = double arithmetic, 1 = float arithmetic
// true if `grid` blocks of the kernel are all resident at once on the current
// device (occupancy from the runtime, cached per kernel, block size and LDS)
bool fits_one_round(const void* kernel, int threads, size_t lds, int grid);
int desc_supported_list(int* orders, int max_pairs);
// angular: false = the radial terms only (the angular components of G are
// written as zero, for the factorised angular kernel to fill);
// ang_ext: the angular part of each entry's gradient is read from p.gang
void launch_desc_fwd(int prec, int nr, int na, const DescParams& p, hipStream_t s, bool angular = true);
void launch_desc_bwd(int prec, int nr, int na, const DescParams& p, hipStream_t s, bool ang_ext = false);
// factorised angular descriptor: fwd = the sums and G's angular components,
// else the angular entry gradients (p.gang); false if na is not compiled in
bool launch_ang_sh(bool fwd, int prec, int na, const DescParams& p, hipStream_t s);
size_t ang_sh_terms(int na);
void launch_desc_jvp(int prec, int nr, int na, const DescParams& p, hipStream_t s);

// ---------------------------------------------------------------- networks
struct MlpNet {          // device pointers of one species (compute type T = double/float)
  const void* wf[kMaxLayers];   // packed forward B operands, hidden layers 1..L-1
  const void* wb[kMaxLayers];   // packed backward B operands, layers 1..L-1
  const void* bias[kMaxLayers]; // biases of layers 1..L-1 (compute type, padded)
  const void* wlast;            // last layer weights (compute type, padded)
  const void* shift;            // [ldG] compute type (zero padded)
  const void* scale;            // [ldG] compute type (zero padded)
  const void* wfull[kMaxLayers + 1];  // plain row-major W_l (compute type) for training
  // BF16: layer 1 (the input layer) is held as a pair hi + lo of BF16
  // operands; these are the packed lo parts (NULL otherwise)
  const void* wf_lo;
  const void* wb_lo;
  const double* blast;           // output-layer bias (device, one double)
  double e_offset;
};
struct MlpParams {
  int n_species;
  int sp_off[kMaxSpecies + 1];    // internal atom ranges per species
  int tile_off[kMaxSpecies + 1];  // tile ranges per species (16 atoms per tile)
  int n_layers;                   // weight layers L (>= 1)
  int w[kMaxLayers + 1];          // true widths
  int wp[kMaxLayers + 1];         // padded widths (multiple of kPad)
  int act[kMaxLayers];
  int ldG;
  MlpNet net[kMaxSpecies];
  const void* G;
  void* gG;                       // dE/dG output (NULL: energies only)
  double* E;                      // [n] per-atom energies (internal order)
  // training (double back-propagation)
  const void* U;                  // [n x ldG] descriptor JVP u_i
  const double* eps_atom;         // [n] dC/dE for each atom (its structure's value)
  double* grad_part;              // [n_blocks x n_params_padded] per-block partial gradients
  int n_params_pad;               // stride of grad_part
  int param_off[kMaxSpecies];     // offset of each species inside a partial gradient row
  int tiles_per_block;
};
// prec: 0 fp64 (MFMA f64), 1 fp32 (MFMA f32), 2 bf16 operands (MFMA bf16, fp32 acc)
size_t mlp_lds_bytes(int prec, const MlpParams& p);
// descriptors and networks of every tile in one kernel (descriptors in double
// for prec 0, float otherwise); dp.G may be NULL (descriptors stay on chip).
// Returns false, launching nothing, where the fused kernel does not apply
// (crowded angular shells, LDS); the caller then runs the two kernels.
bool launch_fwd_mlp(int prec, int nr, int na, const DescParams& dp, const MlpParams& mp, int n_tiles,
                    hipStream_t s);
bool fwd_mlp_fits(int prec, const DescParams& dp, const MlpParams& mp);
void launch_mlp(int prec, const MlpParams& p, int n_tiles, hipStream_t s);
size_t mlp_train_lds_bytes(int prec, const MlpParams& p);
void launch_mlp_train(int prec, const MlpParams& p, int n_blocks, hipStream_t s);
// packs B operands for the MFMA layouts; returns element count (host side)
size_t pack_b_operand_count(int prec, int K, int N);
// part 0: the operand (BF16: rounded to nearest even); part 1 (BF16 only):
// the BF16 rounding of what part 0 leaves over
void pack_b_operand(int prec, const double* B, int K, int N, int ldb, void* out, int part = 0);

// ---------------------------------------------------------------- MD, reductions, gathers
void launch_gather_in(int n, const int* perm, const double* src, double* dst, int* flags,
                      hipStream_t s);
void launch_scatter_out(int n, const int* perm, const double* src3, double* dst3,
                        const double* src1, double* dst1, hipStream_t s);
// *differ |= 1 unless every caller-order position src[perm[p]] equals, bitwise,
// the wrapped internal position pos[p] (what launch_md_outputs writes)
void launch_same_wrapped(int n, const int* perm, const double* pos, const int* seg,
                         const BoxInfo* boxes, const int pbc[3], const double* src, int* differ,
                         hipStream_t s);
// a2 = a, b2 = b, c2 = c (m doubles each), one launch
void launch_copy3(int64_t m, const double* a, double* a2, const double* b, double* b2,
                  const double* c, double* c2, hipStream_t s);
// F_q = Fself_q - sum_{f < nnb[q]} pg[q, f] (pg holds at slot (q, f) the
// gradient of the entry whose reverse is (q, f)); prec of pg: 0 double,
// 1 float.  If vel != NULL also v += c*F/m.
// The opening half kick and drift of the next MD step, fused into the force
// gather of this one (pos == NULL: none): v += c F (again); r += dt v; the
// rebuild flag of the next step is raised when an atom moved more than
// skin/2 since the last build (or always if force_rebuild), and the flag of
// the step after it is cleared.
struct DriftArgs {
  double* pos;
  const double* pos_ref;
  double dt, half_skin2;
  int* rebuild_flag;
  int* clear_flag;
  int force_rebuild;
  // cell binning of the drifted positions for the next build (bin_count ==
  // NULL: none): bin_count is the half of the counts that build reads
  int* bin_count;
  int* bin_atoms;
  const BoxInfo* box;
  int pbc[3];
};
void launch_force_gather(int prec, int n, int cap, const int* nrad, const uint16_t* ridx, const void* pg,
                         const double* Fself, double* F, double* vel, const double* inv_mass_k,
                         const int* species, double half_dt, const DriftArgs& next,
                         hipStream_t s);
void launch_vv_drift(int n, double* vel, const double* F, const double* inv_mass_k,
                     const int* species, double half_dt, const DriftArgs& d, hipStream_t s);
// deterministic sums: out[0] = sum x ; partials has >= reduce_blocks(n) doubles
int reduce_blocks(int64_t n);
void launch_sum(int64_t n, const double* x, double* partials, double* out, hipStream_t s);
// rows independent sums of x [rows][n] into out[rows]; partials has >= rows *
// reduce_blocks(n) doubles; each row summed as launch_sum sums it
void launch_sum_rows(int rows, int64_t n, const double* x, double* partials, double* out, hipStream_t s);
// out = sqrt(sum_k (x_k - y_k)^2 / n), summed in a fixed order
void launch_rms_diff(int64_t n, const double* x, const double* y, double* partials, double* out,
                     hipStream_t s);
// the outputs of an MD call: E = sum E_i and the kinetic energy into *e_pot
// and *e_kin (partials: 2 * reduce_blocks(n) doubles), the wrapped positions,
// velocities and (F_out non-NULL) forces scattered to the caller's order;
// nothing is written if flags[0] or flags[9] is set when the kernels run
void launch_md_outputs(int n, const int* perm, const double* E, const double* pos, const double* vel,
                       const double* F, const double* mass, const int* species, const int* seg,
                       const BoxInfo* boxes, const int pbc[3], const int* flags, double* partials, double* e_pot,
                       double* e_kin, double* pos_out, double* vel_out, double* F_out, hipStream_t s);
void launch_segment_sum(int n_seg, const int64_t* seg_off, const double* x, double* out,
                        hipStream_t s);
void launch_copy_f64(int64_t n, const double* src, double* dst, hipStream_t s);
void launch_check_finite(int64_t n, const double* x, int* flags, hipStream_t s);

// training helpers
void launch_loss_terms(int n, int n_struct, const int* seg, const int* perm, const double* F,
                       const double* f_ref, const double* e_struct, const double* e_ref,
                       const int64_t* seg_count, double lambda_f, int form, double* adj,
                       double* eps_atom, double* floss_atom, double* eloss_struct, hipStream_t s);
void launch_grad_reduce(int n_blocks, int n_params_pad, const double* part, double* out,
                        hipStream_t s);

}  // namespace aenet
