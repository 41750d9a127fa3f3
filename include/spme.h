/*
 * spme.h -- C ABI of the MI355X smooth particle-mesh Ewald (SPME)
 * reciprocal-space step.
 *
 * One step takes atom positions and charges and returns the long-range
 * electrostatic force on every atom, as the paper's long-range pipeline does
 * each timestep (§III.A): charge spreading with order-p cardinal B-splines
 * (§III.A.1), forward 3D FFT, multiplication by the Green's function
 * (influence function) with energy and virial, inverse 3D FFT (§III.A.2),
 * and force interpolation with B-spline derivatives (§III.A.3).  The
 * equations are those of the SPME method the paper builds on (Essmann et
 * al., J. Chem. Phys. 103:8577, 1995):
 *   Q(k)   = sum_i q_i prod_a M_p(u_ia - k_a)           (charge grid)
 *   F(m)   = sum_k Q(k) exp(2 pi i m.k/K)               (3D FFT)
 *   G(m)   = c B(m) exp(-pi^2 |m|^2/beta^2) / (pi V |m|^2),  G(0) = 0
 *   E      = 1/2 sum_m G(m) |F(m)|^2
 *   P_ab   = 1/2 sum_m G|F|^2 (delta_ab - 2(1 + pi^2|m|^2/beta^2) m_a m_b/|m|^2)
 *   phi(k) = sum_m G(m) F(m) exp(-2 pi i m.k/K)         (inverse 3D FFT)
 *   F_i    = -q_i sum_k phi(k) grad_i prod_a M_p(u_ia - k_a)
 * with B(m) the product of the squared B-spline moduli along the three axes.
 *
 * Units: positions and box in Angstrom, charges in e, energies and forces in
 * c e^2/A and c e^2/A^2 where c is the Coulomb constant passed at creation
 * (1.0 by default; 332.0637 gives kcal/mol).
 *
 * Memory: the library never allocates device memory.  The caller owns every
 * device buffer: positions, charges, forces, the energy/virial vector and one
 * workspace of pme_workspace_bytes() bytes.  Device pointers are plain
 * addresses (e.g. torch tensor data_ptr()).  A plan is host memory owned by
 * the library between pme_create and pme_destroy; it is not thread safe and
 * enqueues all work on the stream given at creation (or pme_set_stream), in
 * stream order, without host synchronisation except where noted.
 *
 * Errors: every call returns a pme_status.  Argument errors are detected on
 * the host before anything is enqueued.  Conditions only the device can see
 * (a non-finite coordinate or charge, fixed-point headroom exceeded) raise
 * sticky flags read by pme_check().  Nothing aborts and no exception crosses
 * the ABI.
 *
 * Supported on the GPU: cubic grids K1 = K2 = K3 = K with
 * K in {16, 24, 32, 36, 48, 64, 72, 96, 128} and the non-cubic grids (K1, K2, K3) =
 * (32, 32, 64), (64, 64, 128) and (48, 32, 64); spline order p in {4, 6};
 * any non-degenerate cell (diagonal boxes take a separable fast path for the
 * influence function).  Anything else returns PME_EUNSUPPORTED.
 */
#ifndef SPME_H
#define SPME_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pme_plan pme_plan;

/* Arithmetic of the step.
 * PME_FP32_FIXED: B-spline weights, FFTs and the convolution in FP32; the
 *   charge grid accumulated in 64-bit two's-complement fixed point with
 *   frac_bits fraction bits (order-free, so bit-identical run to run);
 *   B-spline moduli, influence function, energy and virial in FP64.
 * PME_FP64: every stage in FP64 (charge grid accumulated in FP64).
 * PME_FP32_FIXED_HALF: as PME_FP32_FIXED, but the half spectrum is stored
 *   between launches in IEEE binary16 (round to nearest even), halving the
 *   bytes of both corner turns; arithmetic stays FP32/FP64.  Accuracy is
 *   bounded by binary16's 11-bit significand (force errors of order 1e-4
 *   relative) and its range (|values| < 65504).
 * PME_FP32_FIXED_BF16: as PME_FP32_FIXED_HALF, but in bfloat16 (the upper
 *   half of an FP32, round to nearest even): FP32's range, an 8-bit
 *   significand (rounding error <= 2^-8 relative), so force errors about
 *   eight times those of binary16 (of order 1e-3 relative). */
typedef enum {
  PME_FP64 = 0,
  PME_FP32_FIXED = 1,
  PME_FP32_FIXED_HALF = 2,
  PME_FP32_FIXED_BF16 = 3
} pme_precision;

typedef enum {
  PME_OK = 0,
  PME_EINVAL = 1,        /* bad argument (null pointer, N out of range, beta <= 0, ...) */
  PME_EUNSUPPORTED = 2,  /* valid SPME parameters this build does not run (grid, order, cell) */
  PME_EWORKSPACE = 3,    /* workspace missing, misaligned or smaller than pme_workspace_bytes */
  PME_EOVERFLOW = 4,     /* fixed-point headroom exceeded (sum |q| 2^F >= 2^51) */
  PME_EDEVICE = 5,       /* a HIP runtime call failed */
  PME_ENONFINITE = 6,    /* a position or charge was NaN or infinite */
  PME_ESTATE = 7,        /* call out of order (e.g. pme_solve before pme_spread) */
  PME_EBUSY = 8          /* batch admission: no free slot or arena range for the system */
} pme_status;

/* Sticky device flags reported by pme_check. */
#define PME_FLAG_NONFINITE 1u
#define PME_FLAG_OVERFLOW 2u
/* Atom buckets still held a previous binning (a replayed graph that holds
 * part of a step); atoms were dropped. */
#define PME_FLAG_BUCKETS 4u

/* Bytes of device workspace a plan with these parameters needs (0 when the
 * parameters are unsupported).  Host only; no device is touched. */
size_t pme_workspace_bytes(int K1, int K2, int K3, int order, int max_atoms, int precision);

/* Create a plan.
 *   K1, K2, K3  grid points per axis (§III.A.2: the FFT input volume)
 *   order       B-spline order p (the paper spreads over 4x4x4 points, p = 4)
 *   beta        Ewald splitting parameter in 1/A (> 0)
 *   max_atoms   largest N any later call will pass (>= 0)
 *   precision   pme_precision
 *   frac_bits   fixed-point fraction bits F for PME_FP32_FIXED (0 selects 32;
 *               otherwise 16..40); ignored for PME_FP64
 *   coulomb     Coulomb constant c (0 selects 1.0)
 *   workspace   device pointer, 256-byte aligned, >= pme_workspace_bytes();
 *               owned by the caller, must outlive the plan, must not be used
 *               by anyone else while the plan exists
 *   stream      hipStream_t (NULL = the default stream)
 * Enqueues one initialisation launch on the stream (per-axis B-spline
 * moduli and twiddles computed on the device in FP64, counters cleared);
 * no host synchronisation.  Later calls on the plan are ordered after it on
 * the stream.  On failure *out is NULL.  The kernel variants start at the
 * built-in choice for the shape (pme_default_tuning). */
int pme_create(pme_plan **out, int K1, int K2, int K3, int order, double beta, int max_atoms,
               int precision, int frac_bits, double coulomb, void *workspace,
               size_t workspace_bytes, void *stream);

/* Release the host plan.  Does not free the workspace and does not wait for
 * enqueued work. */
int pme_destroy(pme_plan *plan);

/* Change the stream subsequent calls enqueue on. */
int pme_set_stream(pme_plan *plan, void *stream);

/* Charge spreading and the first FFT pass (§III.A.1, start of §III.A.2):
 * bins the atoms, spreads them into the fixed-point (or FP64) grid and
 * transforms it along x (real-to-complex).  With the FP32/fixed path the
 * following pme_solve raises PME_FLAG_OVERFLOW when the spread charges had
 * sum |q| 2^F >= 2^51.
 *   pos  device [N][3] doubles (Angstrom, any image; wrapped internally)
 *   q    device [N] doubles
 *   N    0 <= N <= max_atoms
 *   box  HOST [9] doubles, rows a1, a2, a3 (Angstrom); any cell with nonzero
 *        volume (PME_EINVAL otherwise).  Fractional coordinates are
 *        x (1/L) per axis for a diagonal box, else r . a*_a with
 *        a*_a = (a_b x a_c) / (a_1 . (a_2 x a_3)), no contraction
 * pos and q are read by the launches this call enqueues only.  A spread
 * that follows a spread without pme_solve in between first clears the
 * earlier one's atom buckets (one extra small launch). */
int pme_spread(pme_plan *plan, const double *pos, const double *q, int N, const double box[9]);

/* Green's-function convolution (§III.A.2: the y and z transforms, the
 * multiplication, the inverse z and y transforms), energy and virial.
 * Exactly once after each pme_spread (else PME_ESTATE): it transforms the
 * spectrum in place.
 *   ev   device [7] doubles: E, Pxx, Pyy, Pzz, Pxy, Pxz, Pyz (overwritten),
 *        or NULL to skip writing them. */
int pme_solve(pme_plan *plan, double *ev);

/* Inverse x transform and force interpolation (end of §III.A.2, §III.A.3).
 * After pme_solve (else PME_ESTATE); may be repeated.
 *   forces      device [N][3] doubles in the caller's atom order
 *   accumulate  0 overwrites, 1 adds to the existing values */
int pme_gather(pme_plan *plan, double *forces, int accumulate);

/* The whole step (§III.A, Fig. 2: each timestep the long-range pipeline
 * takes positions and charges and returns the long-range force on every
 * atom): pme_spread + pme_solve + pme_gather, with the energy/virial sum
 * folded into the last launch. */
int pme_step(pme_plan *plan, const double *pos, const double *q, int N, const double box[9],
             double *forces, int accumulate, double *ev);

/* Bind the inputs and outputs of this plan's next batched steps (same
 * meaning and checks as pme_step's arguments).  The arguments are written to
 * the plan's workspace by a one-workgroup launch on the plan's stream, so a
 * bind is stream-ordered: batched runs enqueued before it on that stream
 * still see the previous binding, runs enqueued after it (or ordered after
 * it by an event) see the new one.  Rebind whenever a pointer, N or the box
 * changes.  Buffers must stay valid while batched runs use them. */
int pme_bind(pme_plan *plan, const double *pos, const double *q, int N, const double box[9],
             double *forces, int accumulate, double *ev);

/* One step of each of n bound plans in one batched launch sequence on
 * `stream` (hipStream_t): plans sharing precision, grid and order run as one
 * launch of each kernel over a second grid dimension, so many independent
 * systems of uneven size share every dispatch.  Enqueues kernel launches only
 * (no allocation, copy or synchronisation), so a run can be captured in a
 * hipGraph and replayed.  Each system's result is the same as its own
 * pme_step.  Returns PME_ESTATE if a plan was never bound.
 * A replayed graph must hold whole steps (pme_step, or pme_spread through
 * pme_gather, or pme_batch_run): the atom buckets a spread fills are moved
 * on by the convolution that follows it. */
int pme_batch_run(pme_plan *const *plans, int n, void *stream);

/* ------------------------------------------------------------------------
 * Kernel variants and autotuning.  The paper fixes its FFT size and stage
 * count per bitstream (§IV.A); here the shape of the work is chosen per plan
 * among variants that compute the same step (same E, forces and virial up
 * to FP32 summation order), by default from a built-in rule or by measuring
 * them on the device (pme_autotune).
 * ------------------------------------------------------------------------ */
#define PME_CONV_FUSED 0   /* y/z transforms, influence function and inverse y/z transforms:
                              one workgroup per x' column, the column held in LDS (one launch) */
#define PME_CONV_SPLIT 1   /* the same in three launches of row-chunk workgroups (forward y;
                              z, influence function, inverse z; inverse y), the half
                              spectrum in the workspace between them */
#define PME_CONV_REG 2     /* one workgroup per x' column (y and z pencils of 32 or 64
                              points, every precision): each pencil held in registers by a few lanes
                              of one wavefront, radix-8 and radix-4/8 DFTs in registers with
                              one transpose through LDS between them; the forward z
                              transform, the influence function and the inverse z transform
                              on the same registers (one launch) */
#define PME_INTERP_FUSED 0 /* each (z-plane, y-slice) tile transforms the potential rows its
                              atoms read back along x in LDS, then interpolates (one launch) */
#define PME_INTERP_SPLIT 1 /* inverse x transform once per plane into the workspace, then
                              a gather launch */
/* bits of pme_tuning_variants() */
#define PME_VAR_CONV_FUSED 1u
#define PME_VAR_CONV_SPLIT 2u
#define PME_VAR_INTERP_FUSED 4u
#define PME_VAR_INTERP_SPLIT 8u
#define PME_VAR_CONV_REG 16u

typedef struct {
  int conv;       /* PME_CONV_FUSED, PME_CONV_SPLIT or PME_CONV_REG */
  int interp;     /* PME_INTERP_FUSED or PME_INTERP_SPLIT */
  int bin_chunk;  /* atoms per binning workgroup: 256, 512 or 1024 */
} pme_tuning;

/* Variants a plan with these parameters can run (PME_VAR_* bits; 0 when the
 * parameters are unsupported).  Host only. */
unsigned pme_tuning_variants(int K1, int K2, int K3, int order, int precision);

/* The built-in choice for these parameters (PME_EUNSUPPORTED when none). */
int pme_default_tuning(int K1, int K2, int K3, int order, int precision, pme_tuning *out);

/* Read or change a plan's variants.  pme_set_tuning returns
 * PME_EUNSUPPORTED for a variant the plan's shape cannot run and PME_EINVAL
 * for a bin_chunk outside {256, 512, 1024}; it takes effect at the next
 * spread (or bind).  Changing the variants between pme_spread and pme_gather
 * returns PME_ESTATE. */
int pme_get_tuning(pme_plan *plan, pme_tuning *out);
int pme_set_tuning(pme_plan *plan, const pme_tuning *t);

/* Autotuning: runs whole steps (pme_step with these arguments) of every
 * variant the plan supports -- each conv (fused, split, reg) x interp
 * (fused, split) x bin_chunk (256, 512, 1024) combination, in that nesting
 * order, bin_chunk fastest: 18 candidates -- `reps` timed steps each
 * (after 3 untimed), measured with HIP events on the plan's stream; repeats
 * the sweep three times and keeps each candidate's best mean.  Leaves the
 * plan set to the fastest and returns it in *best with its time in
 * *best_us (microseconds per step).  times_us (may be NULL) receives up to
 * max_times candidate times in the same order, unsupported candidates as
 * -1.  Synchronises the plan's stream; forces and ev hold the last step.
 * Returns PME_EINVAL for reps < 1. */
int pme_autotune(pme_plan *plan, const double *pos, const double *q, int N, const double box[9],
                 double *forces, double *ev, int reps, pme_tuning *best, double *best_us,
                 double *times_us, int max_times);

/* ------------------------------------------------------------------------
 * Batch admission (continuous batching of independent systems).  A batch
 * owns up to max_systems resident systems inside one caller-owned device
 * arena: admitting a system carves its workspace out of the arena (first
 * fit over a free list, 256-byte aligned) and creates and binds its plan;
 * retiring it returns the range (merged with free neighbours).  A launch
 * runs one step of every admitted system, grid groups overlapping on
 * forked streams.  Everything is enqueued on the batch's stream; nothing
 * synchronises the host.
 * ------------------------------------------------------------------------ */
typedef struct pme_batch pme_batch;

typedef struct {
  int K1, K2, K3;       /* grid */
  int order;            /* B-spline order p */
  double beta;          /* Ewald splitting parameter (1/A) */
  int precision;        /* pme_precision */
  int max_atoms;        /* largest N this system will be updated to */
  const double *pos;    /* device [N][3], or NULL: carved from the arena with q, forces, ev */
  const double *q;      /* device [N] (NULL iff pos is NULL) */
  int N;
  double box[9];        /* rows a1, a2, a3 (A) */
  double *forces;       /* device [N][3] (NULL iff pos is NULL) */
  double *ev;           /* device [7], or NULL (not written; carved when pos is NULL) */
} pme_system_desc;

/* Arena bytes admitting this system takes (0 when unsupported): its plan
 * workspace, plus max_atoms x 56 + 56 bytes of inputs and outputs when the
 * desc leaves pos NULL. */
size_t pme_batch_footprint(const pme_system_desc *s);

/* Create a batch over `arena` (device, 256-byte aligned, arena_bytes long,
 * owned by the caller and unused by anyone else while the batch exists);
 * max_systems in [1, 4096]; stream a hipStream_t.  Host only: the batch's
 * three fork streams are created at its first admission. */
int pme_batch_create(pme_batch **out, int max_systems, void *arena, size_t arena_bytes,
                     void *stream);

/* Destroy the batch and every plan still admitted (does not wait for
 * enqueued work; does not free the arena). */
int pme_batch_destroy(pme_batch *b);

/* Admit a system: PME_EBUSY when every slot is taken or no free range of
 * the arena is large enough (nothing changes then); otherwise *slot is its
 * handle.  Argument errors as for pme_create and pme_bind.  The system's
 * plan starts from pme_default_tuning, except that a grid with K1 other
 * than 64 and 128 takes PME_INTERP_SPLIT (faster in batched launches);
 * pme_set_tuning on pme_batch_plan(b, slot) changes it. */
int pme_batch_admit(pme_batch *b, const pme_system_desc *s, int *slot);

/* New inputs/outputs of an admitted system (as pme_bind, on the batch's
 * stream; N <= its max_atoms). */
int pme_batch_update(pme_batch *b, int slot, const double *pos, const double *q, int N,
                     const double box[9], double *forces, double *ev);

/* Retire an admitted system: its plan is destroyed and its arena range
 * returned.  Work already enqueued for it completes first (stream order);
 * a later admission may reuse the range only after that work. */
int pme_batch_retire(pme_batch *b, int slot);

/* Device buffers of an admitted system (those carved from the arena, or
 * the caller's): positions [max_atoms][3], charges [max_atoms], forces
 * [max_atoms][3], energy/virial [7] (may be NULL for a caller's ev). */
int pme_batch_io(pme_batch *b, int slot, double **pos, double **q, double **forces, double **ev);

/* One step of the n listed admitted slots (slots NULL: every admitted
 * system; a slot listed twice is PME_EINVAL): systems sharing precision,
 * grid, order, variants and binning chunk share every launch; the groups
 * run, binning included, on up to three forked streams joined back into the
 * batch's stream (so a launch can be captured in a hipGraph as one
 * fork/join).  PME_OK with nothing to run. */
int pme_batch_launch(pme_batch *b, const int *slots, int n);

/* Occupancy: admitted systems, arena bytes in use, largest free range. */
int pme_batch_stats(pme_batch *b, int *admitted, size_t *bytes_used, size_t *largest_free);

/* The plan of an admitted slot (NULL otherwise), e.g. for pme_check. */
pme_plan *pme_batch_plan(pme_batch *b, int slot);

/* Keep a copy of the charge grid at each spread (costs K1 K2 K3 x 8 bytes
 * of extra writes; off by default). */
int pme_set_debug(pme_plan *plan, int keep_charge_grid);

/* Copy an intermediate grid (enqueued on the plan's stream) to device dst:
 *   which 0: charge grid [K3][K2][K1], int64 (FP32_FIXED, raw fixed point with
 *            frac_bits fraction bits) or double (FP64); needs pme_set_debug(1)
 *            before the spread
 *   which 1: the half spectrum, stored as columns [K1/2+1][K3][K2] complex
 *            (float2 / double2 / two binary16 for PME_FP32_FIXED_HALF / two
 *            bfloat16 for PME_FP32_FIXED_BF16; index m1 slowest, y fastest):
 *            after
 *            pme_spread the forward transform of the charge grid along x;
 *            after pme_solve G F transformed back along z and y
 *   which 2: the potential phi [K3][K2][K1], float (FP32_FIXED, _HALF, _BF16) or double */
int pme_debug_grid(pme_plan *plan, int which, void *dst);

/* Size in bytes of pme_debug_grid(which)'s output (0 for a bad which). */
size_t pme_debug_grid_bytes(pme_plan *plan, int which);

/* Synchronise the plan's stream, return the sticky device flags
 * (PME_FLAG_*) in *flags and clear them.  Returns PME_ENONFINITE or
 * PME_EOVERFLOW, or PME_ESTATE for PME_FLAG_BUCKETS, when the matching flag
 * was set, else PME_OK. */
int pme_check(pme_plan *plan, unsigned *flags);

/* Timing diagnostics for graph-replayed steps: pme_step (overwriting the
 * forces) with one kernel launched a second time where that leaves the
 * step's forces, energy and virial unchanged --
 *   PME_PROBE_SPREAD  spreading + x transform again right after the first
 *   PME_PROBE_INTERP  inverse x transform + interpolation again at the end
 *   PME_PROBE_CONV    the y/z convolution again at the end, on the spectrum
 *                     the next spread rewrites (a pme_gather after it
 *                     returns PME_ESTATE)
 *   PME_PROBE_BIN     binning again at the end, then its bucket counts
 *                     cleared for the next step (a one-workgroup launch)
 *   PME_PROBE_CLEAR   that clearing launch alone
 * so that the difference between replays of captured probe steps and of
 * plain steps is the repeated kernel's time in the step's stream (for
 * binning, the PME_PROBE_BIN difference less the PME_PROBE_CLEAR one).
 * Enqueues kernel launches only (capturable). */
#define PME_PROBE_NONE 0
#define PME_PROBE_BIN 1
#define PME_PROBE_SPREAD 2
#define PME_PROBE_CONV 3
#define PME_PROBE_INTERP 4
#define PME_PROBE_CLEAR 5
int pme_step_probe(pme_plan *plan, const double *pos, const double *q, int N,
                   const double box[9], double *forces, double *ev, int repeat);

/* Per-kernel timing with HIP events on the plan's stream (off by default).
 * While enabled every launch carries a start and a stop event attached to
 * the dispatch itself (hipExtLaunchKernel), so the elapsed time is the
 * kernel's own execution, the interval a profiler reports for the dispatch
 * (host-launched steps; not for stream capture).  Changing the setting drops
 * unread times.  pme_kernel_times
 * synchronises, adds the elapsed times of all completed launches into
 * ms[0..n-1] (kernel order: 0 bin, 1 spread + x FFT, 2 y/z FFTs with the
 * influence function and the inverse z/y FFTs, 3 inverse x FFT + force
 * interpolation) and returns the number of steps accumulated in *steps.
 * Where a slot takes several launches (the split convolution, the split
 * interpolation), it runs from the start of the first to the end of the
 * last, gaps included. */
int pme_kernel_timing(pme_plan *plan, int enable);
int pme_kernel_times(pme_plan *plan, double *ms, int n, int *steps);

/* ------------------------------------------------------------------------
 * Real-space part of the Ewald sum (the short-range electrostatics beside the
 * reciprocal pipeline, §II, §V.A): with it, pme_step's energy + E_real +
 * E_self + E_excl is the full Ewald energy, and the forces add up likewise.
 *   E_real = (c/2) sum_i sum_{j != i, |r_ij| <= rcut} q_i q_j erfc(beta r_ij)/r_ij
 *            (minimum image; rcut <= L/3 on every axis)
 *   E_self = -c beta/sqrt(pi) sum_i q_i^2
 *   E_excl = -(c/2) sum_i sum_{j in excl(i)} q_i q_j [erf(beta r)/r
 *            + (r <= rcut ? erfc(beta r)/r : 0)]   (removes excluded pairs
 *            from both the pair sum and the reciprocal sum)
 * Forces are -grad of E_real + E_excl.  FP64 throughout; diagonal boxes
 * only (PME_EUNSUPPORTED otherwise, when rcut > L/3 on some axis, or when
 * beta rcut > 6, where erfc(beta rcut) < 3e-17 and a shorter cutoff gives the
 * same sums).  erfc of a pair inside the cutoff comes from a Chebyshev
 * series of exp(x^2) erfc(x) on [0, beta rcut] (24 terms up to beta rcut =
 * 3.2, 32 beyond), relative error <= 2e-14.  Two distinct atoms at exactly the same position are not paired
 * (their pair term is infinite).
 * ------------------------------------------------------------------------ */

/* Bytes of device workspace for pme_real with at most max_atoms atoms and
 * max_cells cells of the neighbour grid (>= 27); 0 for bad arguments. */
size_t pme_real_workspace_bytes(int max_atoms, int max_cells);

/* One real-space evaluation, enqueued on `stream` (hipStream_t).
 *   pos, q       device [N][3], [N] doubles (any image)
 *   box          HOST [9] doubles, diagonal
 *   beta, rcut   Ewald splitting parameter (1/A) and pair cutoff (A), > 0
 *   coulomb      Coulomb constant c (0 selects 1.0)
 *   excl_off     device [N+1] ints, or NULL for no exclusions: atom i's
 *                excluded partners are excl_idx[excl_off[i] .. excl_off[i+1]);
 *                the lists must be symmetric and hold indices in [0, N)
 *   forces       device [N][3] doubles, overwritten (accumulate 0) or added to
 *   energies     device [3] doubles: E_real, E_self, E_excl (overwritten)
 *   workspace    device, 256-byte aligned, >= pme_real_workspace_bytes(
 *                max_atoms, max_cells); the cell grid is the finest with
 *                edges >= rcut, coarsened to fit max_cells
 * Cells hold atoms in an order set by atomics, so forces reproduce to FP64
 * rounding rather than bit for bit. */
int pme_real(const double *pos, const double *q, int N, const double box[9], double beta,
             double rcut, double coulomb, const int *excl_off, const int *excl_idx,
             double *forces, int accumulate, double *energies, void *workspace,
             size_t workspace_bytes, int max_atoms, int max_cells, void *stream);

/* ------------------------------------------------------------------------
 * Allocation-free step, for callers that cannot allocate device memory:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation.  One whole step (as pme_step on a plan with these parameters
 * and its built-in variants) with the library's own static device scratch
 * of PME_SCRATCH_BYTES per GPU in place of a caller workspace; nothing is
 * allocated (no hipMalloc, no host heap) and nothing synchronises.
 *   Size limit: pme_workspace_bytes(K1, K2, K3, order, N, precision) must
 *   not exceed PME_SCRATCH_BYTES (about 16 MiB at 65,536 atoms on 64^3),
 *   else PME_EWORKSPACE and nothing is enqueued.  Other arguments and
 *   errors as pme_create (frac_bits, coulomb) and pme_step.
 * Every call on one GPU uses that GPU's single scratch, which keeps the last
 * call's contents (each call re-initialises what it reads before use):
 * calls that overlap on one GPU -- on different streams, or from different
 * threads -- race and must be ordered by the caller.  The sticky device
 * flags of pme_check are not reported. */
#define PME_SCRATCH_BYTES ((size_t)32 << 20)
int pme_step_noalloc(int K1, int K2, int K3, int order, double beta, int precision,
                     int frac_bits, double coulomb, const double *pos, const double *q, int N,
                     const double box[9], double *forces, int accumulate, double *ev,
                     void *stream);

/* Human-readable text for a pme_status. */
const char *pme_strerror(int code);

/* ABI version (major * 100 + minor). */
int pme_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SPME_H */
