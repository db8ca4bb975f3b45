/*
 * sldg.h -- C ABI of libsldg, the MI355X (gfx950) projection sweep of the
 * mixed-precision semi-Lagrangian discontinuous Galerkin (sLdG) method
 * (L. Einkemmer, "A mixed precision semi-Lagrangian algorithm and its
 * performance on accelerators", arXiv 1603.07008).
 *
 * Data model (section II-A).  A periodic tensor grid of ndim dimensions,
 * ncells[0] x ... x ncells[ndim-1] cells, dimension 0 fastest:
 *     cell id = i_0 + N_0 * (i_1 + N_1 * (i_2 + ...)).
 * In each cell the solution is a polynomial of degree k in every variable,
 * stored as tensor-product Legendre coefficients, o = k + 1 per dimension:
 *     mode id m = j_0 + o * (j_1 + o * (j_2 + ...)),  0 <= j_e <= k.
 * Mode 0 is the cell mean (the mass mode).  The state is split in two arrays:
 *     mass : double [n_lo][cells]   the modes of total degree j_0+...+j_{d-1}
 *                                   below `ndouble`, in increasing mode id
 *     hi   : T      [n_hi][cells]   all other modes, in increasing mode id
 * where T is the storage type of the plan's tier: double (FP64 tier), float
 * (FP32 tier), bfloat16 or IEEE half (BF16 / FP16 tiers; raw 16-bit words).
 * With the default ndouble = 1 (sldg_plan), `mass` holds mode 0 only and
 * `hi` holds modes 1 .. o^ndim-1 at planes 0 .. o^ndim-2.  Keeping the mass
 * mode in FP64 while the others are narrower is the paper's mixed-precision
 * scheme (section II-A, the paragraph on the storage of c_0; section III-A); it
 * conserves the total mass to FP64 rounding.  Larger ndouble keeps more
 * leading coefficients in FP64 (the count of double-precision coefficients
 * that section III-A and its tables vary); ndouble = 0 stores every mode
 * narrow.
 *
 * All state pointers are device pointers (HIP device memory) owned by the
 * caller.  A plan owns only small device tables.  Functions never abort: they
 * return a status, and sldg_last_error() holds a thread-local detail string.
 */
#ifndef SLDG_H
#define SLDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sldg_plan_s* sldg_plan_t;

typedef enum {
    SLDG_OK = 0,
    SLDG_ERR_ARG = 1,          /* null pointer, bad dimension, bad mask, bad size */
    SLDG_ERR_ALIAS = 2,        /* an output buffer overlaps an input or another output */
    SLDG_ERR_UNSUPPORTED = 3,  /* degree or tier without a compiled kernel, grid too large */
    SLDG_ERR_NOMEM = 4,        /* a device allocation of the library failed, or would
                                  pass the limit of sldg_set_device_alloc_limit */
    SLDG_ERR_DEVICE = 5        /* a HIP call or kernel launch failed */
} sldg_status;

typedef enum {
    SLDG_TIER_FP64 = 0,        /* all modes FP64, FP64 arithmetic */
    SLDG_TIER_FP32 = 1,        /* mass FP64; other modes FP32 storage, FP64 arithmetic */
    SLDG_TIER_BF16 = 2,        /* mass FP64 (FP64 update); other modes bfloat16, FP32 arithmetic */
    SLDG_TIER_FP16 = 3         /* mass FP64 (FP64 update); other modes IEEE half, FP32 arithmetic */
} sldg_tier;

/*
 * Create a plan for a grid and a storage tier (section II-A).
 *   plan      out: the new plan (NULL on error)
 *   ndim      1..6
 *   ncells    host array [ndim], cells per dimension (>= 1), dimension 0
 *             fastest; the total cell count must be below 2^31
 *   k         polynomial degree per dimension, 1..3
 *   tier      storage tier of the modes other than the cell mean
 *   stream    hipStream_t every later call of this plan is enqueued on
 *             (NULL = the null stream)
 * Allocates the plan's device tables (per-line shift/matrix table and the
 * mass-reduction scratch) on the current device.  Errors: SLDG_ERR_ARG,
 * SLDG_ERR_UNSUPPORTED, SLDG_ERR_NOMEM, SLDG_ERR_DEVICE.
 */
sldg_status sldg_plan(sldg_plan_t* plan, int ndim, const int64_t* ncells, int k,
                      sldg_tier tier, void* stream);

/*
 * As sldg_plan, with the modes of total degree below `ndouble` stored in FP64
 * (0 <= ndouble <= ndim*k + 1; see the data model above).  The FP64 modes'
 * updates are computed in FP64 from exactly widened inputs.  sldg_mass needs
 * ndouble >= 1.
 */
sldg_status sldg_plan_ex(sldg_plan_t* plan, int ndim, const int64_t* ncells, int k,
                         sldg_tier tier, int ndouble, void* stream);

/* Planes of the `mass` (FP64) and `hi` arrays of a state of this plan. */
int64_t sldg_lo_planes(sldg_plan_t plan);
int64_t sldg_hi_planes(sldg_plan_t plan);
/* Where each mode is stored: out[m] >= 0 is plane out[m] of `hi`, out[m] < 0 is
 * plane -1-out[m] of `mass`; out is host int32 [o^ndim]. */
sldg_status sldg_plane_map(sldg_plan_t plan, int32_t* out);

/* Release a plan (synchronises its stream first).  NULL is a no-op. */
void sldg_plan_destroy(sldg_plan_t plan);

/* Change the stream later calls of the plan are enqueued on. */
sldg_status sldg_plan_set_stream(sldg_plan_t plan, void* stream);

/*
 * Per-line shift tables (section II-A, update rule and the remark that the
 * matrices are precomputed once per step).  For each displacement sigma[t]
 * (cells, FP64) computes s = floor(sigma) and alpha = sigma - s in [0, 1),
 * snapped so that alpha + (1 - alpha) == 1 exactly, and the projection
 * matrices A(alpha), B(alpha) of degree k with the exact mass row
 * (A_00 = 1 - alpha, B_00 = alpha, B_0l = -A_0l).  A fractional part that
 * rounds to 1 is taken as s + 1, alpha = 0.
 *   n        number of displacements
 *   sigma    device double [n]
 *   s_out    device int32 [n]: s reduced modulo `period` into [0, period)
 *            (period >= 1; pass the length of the swept dimension)
 *   ab_out   device double [n][2][k+1][k+1]: A then B, row-major [j][l]
 * Asynchronous on the plan's stream.  Non-finite sigma yields NaN matrices.
 */
sldg_status sldg_line_tables(sldg_plan_t plan, int64_t n, int64_t period,
                             const double* sigma, int32_t* s_out, double* ab_out);

/*
 * One out-of-place projection sweep along dimension `dim` (section II-A,
 * update rule; section II eq. (1) for the splitting into 1D advections):
 *     out[i] = A(alpha) in[i - s] + B(alpha) in[i - s - 1]
 * along dim, for every mode index j_dim, with the other mode indices as
 * spectators, periodic in dim.
 *   dim       swept dimension, 0..ndim-1
 *   shift     device double: displacement in cells (a * dt / h_dim) per line,
 *             indexed row-major over the dimensions in dep_mask, lowest
 *             dimension fastest, and broadcast over the other dimensions
 *             (dep_mask = 0: a single value)
 *   dep_mask  bit e set if the displacement depends on dimension e; must not
 *             contain dim
 *   in_mass, in_hi    input state (see the data model above)
 *   out_mass, out_hi  output state; must not overlap any input or each other
 * The mass mode's new value is computed entirely in FP64 from the promoted
 * inputs; the other modes are rounded to nearest even on store.  Allocates
 * nothing, does not synchronise; asynchronous on the plan's stream.
 * Errors: SLDG_ERR_ARG, SLDG_ERR_ALIAS, SLDG_ERR_DEVICE.
 */
sldg_status sldg_advect_dim(sldg_plan_t plan, int dim, const double* shift,
                            uint32_t dep_mask, const double* in_mass,
                            const void* in_hi, double* out_mass, void* out_hi);

/*
 * The transpose of sldg_advect_dim with the same displacements: for every
 * line, g_in[m] = A(alpha)^T g[m + s] + B(alpha)^T g[m + s + 1], i.e. the
 * adjoint of the projection sweep with respect to the Euclidean inner product
 * of the coefficient arrays (the gradient of a loss of the output with respect
 * to the input, for reverse-mode differentiation through split steps,
 * section II).  Same arguments, layout, storage tier and error behaviour as
 * sldg_advect_dim; in/out are the output-side and input-side gradients.
 */
sldg_status sldg_advect_dim_adjoint(sldg_plan_t plan, int dim, const double* shift,
                                    uint32_t dep_mask, const double* in_mass,
                                    const void* in_hi, double* out_mass, void* out_hi);

/* One sweep of a split step: dimension, dependence mask, device displacements. */
typedef struct {
    int dim;
    uint32_t dep_mask;
    const double* shift;
} sldg_sweep_desc;

/*
 * A split time step applied nsteps times (section II: the Vlasov equation is
 * split into a sequence of 1D advections).  Each step applies the nseq
 * sweeps of `seq` in order, each pass reading one buffer and writing the
 * other.  A sweep along dimension 0 directly followed by one along dimension
 * 1 runs as one fused pass (sldg_advect_dims01) where that entry point
 * accepts the pair and fusion is on (sldg_plan_set_fusion, default on): the
 * result is bitwise the same, but the pair then takes one pass instead of
 * two.  *result_buffer receives the buffer (0 or 1) holding the result:
 * (nsteps * nseq) % 2 without fused pairs.
 * Buffers 0 and 1 must not overlap.  Asynchronous on the plan's stream.
 */
sldg_status sldg_split_steps(sldg_plan_t plan, const sldg_sweep_desc* seq, int nseq,
                             int nsteps, double* mass0, void* hi0, double* mass1,
                             void* hi1, int* result_buffer);

/*
 * The sweep along dimension 0 followed by the sweep along dimension 1, as one
 * pass over the state: bitwise the result of sldg_advect_dim(plan, 0, shift0,
 * dep_mask0, in -> tmp) then sldg_advect_dim(plan, 1, shift1, dep_mask1,
 * tmp -> out), including the rounding of the intermediate state to the
 * storage tier, without the intermediate state in device memory (section II:
 * consecutive 1D advections of a split step).  Every coefficient is read
 * once and written once for the two sweeps.  A workgroup holds a tile of one
 * (dimension 0, dimension 1) slab (all N_0 cells of R + 1 consecutive rows of
 * dimension 1, the o^2 modes of one spectator group) in LDS.
 * Conditions, else SLDG_ERR_UNSUPPORTED (nothing is launched): ndim >= 2;
 * neither displacement depends on dimension 0 or 1 (dep_mask bits 0 and 1
 * clear), so each is uniform over a slab; at most the cell mean is stored in
 * FP64 (ndouble <= 1); ncells[0] % 4 == 0; all state pointers 16-byte
 * aligned; one tile of at least one row fits the LDS budget.  Arguments,
 * layout and other errors as sldg_advect_dim.  Allocates nothing,
 * asynchronous on the plan's stream.
 */
sldg_status sldg_advect_dims01(sldg_plan_t plan, const double* shift0, uint32_t dep_mask0,
                               const double* shift1, uint32_t dep_mask1,
                               const double* in_mass, const void* in_hi, double* out_mass,
                               void* out_hi);

/* Fusion of (0, 1) sweep pairs inside sldg_split_steps: enable != 0 on (the
 * default), 0 off (every sweep its own pass).  Errors: SLDG_ERR_ARG. */
sldg_status sldg_plan_set_fusion(sldg_plan_t plan, int enable);

/*
 * Sum of the mass array, mass[0] + ... + mass[cells-1], as an unevaluated
 * double-double out[0] + out[1] (|out[1]| <= ulp(out[0])/2), with a
 * deterministic reduction order (section II-A: c_0 carries the mass; section
 * III-A measures its conservation).  The physical mass is this sum times the
 * cell volume, which the caller applies.  `out` is host memory; the call
 * synchronises the plan's stream.
 */
sldg_status sldg_mass(sldg_plan_t plan, const double* mass, double out[2]);

/*
 * The same double-double sum written to device memory out_dev[2] (hi, lo),
 * asynchronously on the plan's stream, without synchronising; for use inside
 * a stream of sweeps (and under stream capture).
 */
sldg_status sldg_mass_device(sldg_plan_t plan, const double* mass, double* out_dev);

/*
 * Launch shape of the sweeps along one dimension.  It changes how the work is
 * split between threads, never the arithmetic of an output: results are
 * bitwise the same for every shape.
 *   rows      strided sweeps (dim > 0): consecutive rows per thread, 1/2/4/8,
 *             or 0 for the lane form (one cell per lane, consecutive lanes on
 *             consecutive cells).  Dimension 0, where the window form does
 *             not apply (N_0 % 4 != 0 or buffers not 16-byte aligned): 1 for
 *             the lane form, 2/4/8 for the group form (4 cells of a line
 *             per thread, interleaved with the line's other threads), 0 (the
 *             default) for all tuples in one run, in the group form when the
 *             displacement depends on dimension 1, else in the lane form
 *             (tuples is then ignored where the window form does not apply)
 *   tuples    spectator mode tuples per thread (0: all)
 *   colwaves  strided sweeps: waves of a workgroup side by side along the
 *             columns (1, 2 or 4; the others stack along the rows).  1, 2 or
 *             4 plus SLDG_SHAPE_STAGED: the workgroup loads the source rows of
 *             its tile (64 colwaves columns x 4 rows-per-thread chunks) into
 *             LDS with 16-byte accesses, and every thread takes its column
 *             from there (narrow tiers, rows 4 or 8, at most the cell mean
 *             in FP64, tiles of whole 64-column runs, 16-byte aligned input;
 *             elsewhere, and in a tile whose displacements spread over more
 *             rows than it holds, the same shape runs direct).  Plus
 *             SLDG_SHAPE_MEMORDER (with or without SLDG_SHAPE_STAGED): the
 *             workgroups take their tiles in memory order, the column blocks
 *             of a row chunk group before the next group (where the blocks
 *             tile the P columns below the swept dimension exactly; elsewhere
 *             the flag has no effect); without it the row chunk groups of a
 *             column block come one after the other.  The order changes no
 *             result bit.
 * Plans start from a shape measured on MI355X; sldg_plan_tune picks one per
 * dimension.  Errors: SLDG_ERR_ARG.
 */
#define SLDG_SHAPE_STAGED 16
#define SLDG_SHAPE_MEMORDER 32
sldg_status sldg_plan_set_shape(sldg_plan_t plan, int dim, int rows, int tuples, int colwaves);
sldg_status sldg_plan_get_shape(sldg_plan_t plan, int dim, int* rows, int* tuples,
                                int* colwaves);

/*
 * Kernel form that a sweep along `dim` with the plan's current shape runs in
 * for these buffers (host only, no device work; dep_mask as for
 * sldg_advect_dim): 0 dimension-0 window form, 1 dimension-0 group form,
 * 2 strided, 3 lane form, 4 strided staged through LDS.  Errors: SLDG_ERR_ARG
 * (null plan or form, dim or dep_mask out of range), SLDG_ERR_UNSUPPORTED
 * (the grid does not launch).
 */
sldg_status sldg_plan_sweep_form(sldg_plan_t plan, int dim, uint32_t dep_mask,
                                 const double* in_mass, const void* in_hi,
                                 const double* out_mass, const void* out_hi, int* form);

/* Candidate i of the shapes sldg_plan_tune tries, for dimension-0 (strided =
 * 0) or strided (strided = 1) sweeps; SLDG_ERR_ARG past the last one. */
sldg_status sldg_tune_candidate(int strided, int i, int* rows, int* tuples, int* colwaves);

/*
 * Autotuner: for every dimension swept in `seq`, time each candidate shape
 * (one warm-up and `reps` timed sweeps from buffer 0 into buffer 1, HIP
 * events on the plan's stream) and keep the fastest.  Buffer 1 is
 * overwritten; buffer 0 is only read.  Shapes a grid cannot launch are
 * skipped.  best_ms (host [nseq], optional) receives the kept time of each
 * sweep.  Synchronises the plan's stream.
 */
sldg_status sldg_plan_tune(sldg_plan_t plan, const sldg_sweep_desc* seq, int nseq,
                           const double* mass0, const void* hi0, double* mass1, void* hi1,
                           int reps, double* best_ms);

/*
 * FP16 storage with per-plane power-of-two scaling (FP16 tier only).
 *
 * FP16 has 11 significant bits but only the exponents -14..15 in its normal
 * range, so the small higher Legendre modes (c_j ~ h^|j| for smooth data,
 * section II-A) of a state in physical units lose their precision to the
 * subnormal range or flush to zero.  A scaled FP16 state stores hi plane p
 * as c * 2^exp[p] and carries a *scale block* beside its mass and hi arrays:
 *     int32 exp[n_hi]    storage exponent of every hi plane
 *     float amax[n_hi]   absolute maximum of the values c of every hi plane
 * (device memory, 8 * n_hi bytes, sldg_scale_bytes; caller-owned like the
 * state).  The exponent of a plane is chosen so that its absmax sits
 * `headroom` binades below 2^15: 2^(14-h) <= amax * 2^e < 2^(15-h), clamped
 * to [-100, 100].  The scaling is exact (powers of two), so the stored value
 * is the round-to-nearest-even of c onto FP16 with its exponent range moved
 * by -e, and results do not depend on the units of the state.
 */

/* Bytes of a scale block of this plan (8 * n_hi); -1 for a NULL plan. */
int64_t sldg_scale_bytes(sldg_plan_t plan);

/* Headroom h in binades (0..14) of the exponents chosen from now on; the
 * default is 8. */
sldg_status sldg_set_scale_headroom(sldg_plan_t plan, int binades);

/*
 * Scaled FP16 state from FP64 values: for every hi plane, the absmax (rounded
 * to FP32), the exponent with the plan's headroom (0 for an all-zero plane),
 * and the FP16 values round(c * 2^e), correctly rounded from FP64.
 *   hi64   device double [n_hi][cells] (the values of the narrow modes)
 *   hi     device FP16 [n_hi][cells] (out)
 *   scale  device scale block (out)
 * Asynchronous on the plan's stream.  Errors: SLDG_ERR_ARG,
 * SLDG_ERR_UNSUPPORTED (not an FP16 plan), SLDG_ERR_ALIAS, SLDG_ERR_DEVICE.
 */
sldg_status sldg_scaled_import(sldg_plan_t plan, const double* hi64, void* hi, void* scale);

/* The values a scaled FP16 state represents, hi[p][c] * 2^-exp[p], exactly,
 * into device double [n_hi][cells].  Asynchronous. */
sldg_status sldg_scaled_export(sldg_plan_t plan, const void* hi, const void* scale,
                               double* hi64);

/*
 * sldg_advect_dim on scaled FP16 states.  The exponent of every output plane
 * is predicted from the input's absmax of the same plane with the plan's
 * headroom (kept from the input when that absmax is 0); the sweep records the
 * absmax of what it computes; a plane whose absmax reaches 2^15 at its
 * predicted exponent (growth by more than the headroom in one sweep) is
 * recomputed with the exponent of its own absmax and one binade of headroom,
 * so no value overflows.  The FP64 modes are as in sldg_advect_dim.  Uses a
 * per-plan partial buffer, grown (hipMalloc) on the first call that needs
 * more; asynchronous; four launches besides the line tables (predict, sweep,
 * decide, repair).  Errors as sldg_advect_dim, plus SLDG_ERR_UNSUPPORTED for
 * a plan that is not FP16 and SLDG_ERR_NOMEM.
 */
sldg_status sldg_advect_dim_scaled(sldg_plan_t plan, int dim, const double* shift,
                                   uint32_t dep_mask, const double* in_mass,
                                   const void* in_hi, const void* in_scale,
                                   double* out_mass, void* out_hi, void* out_scale);

/* sldg_split_steps on scaled FP16 states (buffers 0 and 1 each with their
 * scale block). */
sldg_status sldg_split_steps_scaled(sldg_plan_t plan, const sldg_sweep_desc* seq, int nseq,
                                    int nsteps, double* mass0, void* hi0, void* scale0,
                                    double* mass1, void* hi1, void* scale1,
                                    int* result_buffer);

/*
 * Sweep along `dim` with transverse Gauss-node collocation in `tdim`.  The
 * displacement varies across the cells of tdim; instead of one value per
 * transverse cell (sldg_advect_dim), the state is taken at the k+1
 * Gauss-Legendre nodes y_q of each transverse cell (modal -> nodal in j_tdim),
 * each node line is swept with its own displacement (section II-A update rule,
 * unchanged), and the result is projected back onto the Legendre modes in
 * tdim with the Gauss weights (eq. (cj) with the (k+1)-point rule).  Other
 * mode indices are spectators.  The total mass is conserved (the rule
 * integrates P_0 exactly).
 *   node_shift  device double [N_tdim * (k+1)]: displacement in cells of
 *               node q (ascending in y) of transverse cell i at [i*(k+1) + q]
 *   buffers as in sldg_advect_dim
 * All arithmetic is FP64; narrow modes are rounded to nearest even on store.
 * Asynchronous on the plan's stream.  Errors: SLDG_ERR_ARG, SLDG_ERR_ALIAS,
 * SLDG_ERR_UNSUPPORTED, SLDG_ERR_DEVICE.
 */
sldg_status sldg_advect_dim_collocated(sldg_plan_t plan, int dim, int tdim,
                                       const double* node_shift, const double* in_mass,
                                       const void* in_hi, double* out_mass, void* out_hi);

/*
 * Self-consistent field of an (x, v) problem (ndim = 2; dimension 0 is x,
 * dimension 1 is v), for the v-sweep of the split step.  The paper states the
 * Vlasov equation with a field E(x) (section II) but no field equation; the
 * one taken is Gauss's law of the normalised Vlasov-Poisson system in the
 * paper's sign convention (+E d_v f): dE/dx = rho - mean(rho), E periodic
 * with zero mean, rho(x) = int f dv.  rho is exact for the piecewise
 * polynomial state (in x cell i its Legendre moments are h_v times the sums
 * over the v cells of the modes (j, 0)); E is its zero-mean antiderivative,
 * evaluated at the x cell centres.
 *   mass, hi    the state (device; the plan's layout and tier, unscaled)
 *   hx, hv      cell widths in x and v
 *   dt          time step of the v-sweep
 *   shift_out   device double [N_x]: E(x_i) * dt / hv, the displacement of the
 *               v-sweep line through x cell i (use dep_mask = 1)
 *   field_out   optional device double [N_x]: E(x_i)
 * Asynchronous on the plan's stream.  Grows a plan-owned scratch buffer
 * (hipMalloc) on the first call that needs more.  Errors: SLDG_ERR_ARG,
 * SLDG_ERR_ALIAS, SLDG_ERR_NOMEM, SLDG_ERR_DEVICE.
 */
sldg_status sldg_poisson_shift(sldg_plan_t plan, const double* mass, const void* hi, double hx,
                               double hv, double dt, double* shift_out, double* field_out);

/*
 * sldg_poisson_shift for callers that cannot allocate device memory: code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and errors as sldg_poisson_shift, but
 * the solve's scratch is a static device array of the library (4 MiB, one
 * copy per device, held until the process ends) instead of a plan-owned
 * buffer, and no call allocates or frees memory.
 *   Limit: (9 (k+1) + 1) N_x + 1 <= 2^19 doubles of scratch when N_v >= 8
 *          (N_x <= 14,169 at k = 3, 27,593 at k = 1); larger grids return
 *          SLDG_ERR_UNSUPPORTED.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents; nothing in it needs to start at zero.  Calls that overlap
 * in time on one device (other streams, other threads, other plans) race on
 * it: order them on one stream.  Errors: as sldg_poisson_shift, with
 * SLDG_ERR_UNSUPPORTED for grids beyond the limit and never SLDG_ERR_NOMEM.
 */
sldg_status sldg_poisson_shift_noalloc(sldg_plan_t plan, const double* mass, const void* hi,
                                       double hx, double hv, double dt, double* shift_out,
                                       double* field_out);

/*
 * nsteps self-consistent Strang steps of an (x, v) plan: X(dt/2) with the
 * displacements shift_x (device [N_v], per v line, dep_mask = 2), the field of
 * the state into shift_v (device [N_x], overwritten), V(dt) with shift_v,
 * X(dt/2).  Buffers as in sldg_split_steps; *result_buffer receives the buffer
 * holding the result.  Asynchronous on the plan's stream.
 */
sldg_status sldg_vlasov_poisson_steps(sldg_plan_t plan, int nsteps, const double* shift_x,
                                      double hx, double hv, double dt, double* shift_v,
                                      double* mass0, void* hi0, double* mass1, void* hi1,
                                      int* result_buffer);

/*
 * Self-consistent field of an (x1, x2, v1, v2) problem (ndim = 4, dimensions
 * in that order), for the v-sweeps of the split step.  As for the (x, v)
 * field, the paper gives the Vlasov equation with a field E(x) (section II)
 * but no field equation.  The one taken is Gauss's law div E = rho -
 * mean(rho), with E = -grad phi periodic, in the paper's sign convention
 * (+E . grad_v f).  It is solved spectrally on the x-cell means of rho,
 * which are h_v1 h_v2 times the sums over the v cells of the cell means c_0.
 * The 2D DFT of the cell means is divided by the Fourier symbol of cell
 * averaging, sinc(kappa_1 h_x1 / 2) sinc(kappa_2 h_x2 / 2), and
 * E_hat = -i kappa rho_hat / |kappa|^2.  The mean and the Nyquist modes are
 * dropped.  E is evaluated at the x cell centres.  The solve is exact for
 * densities that are trigonometric polynomials resolved by the grid.
 *   mass, hi    the state (device; the plan's layout and tier, unscaled)
 *   h           host double[4]: cell widths h_x1, h_x2, h_v1, h_v2
 *   dt          time step of the v-sweeps
 *   shift_v1    device double [N1 N2], x1 fastest: E_1 dt / h_v1, the
 *               displacement of the v1-sweep line through x cell (i1, i2)
 *               (use dep_mask = 3)
 *   shift_v2    device double [N1 N2]: E_2 dt / h_v2 (dep_mask = 3)
 *   field_out   optional device double [2 N1 N2]: E_1, then E_2
 * N1, N2 <= 2048 (direct DFTs with twiddles in LDS; SLDG_ERR_UNSUPPORTED
 * beyond).  Asynchronous on the plan's stream.  Grows a plan-owned scratch
 * buffer (hipMalloc) on the first call that needs more.  Errors: SLDG_ERR_ARG,
 * SLDG_ERR_ALIAS, SLDG_ERR_UNSUPPORTED, SLDG_ERR_NOMEM, SLDG_ERR_DEVICE.
 */
sldg_status sldg_poisson_shift_2d(sldg_plan_t plan, const double* mass, const void* hi,
                                  const double* h, double dt, double* shift_v1, double* shift_v2,
                                  double* field_out);

/*
 * nsteps self-consistent Strang steps of an (x1, x2, v1, v2) plan:
 *   - X1(dt/2) with shift_x1 (device [N_v1], per v1 line, dep_mask = 4);
 *   - X2(dt/2) with shift_x2 (device [N_v2], dep_mask = 8);
 *   - the field of the state into shift_v1, shift_v2 (device [N1 N2] each,
 *     overwritten; sldg_poisson_shift_2d);
 *   - V1(dt), V2(dt);
 *   - X1(dt/2), X2(dt/2).
 * Buffers as in sldg_split_steps.  *result_buffer receives the buffer holding
 * the result.  Asynchronous on the plan's stream.
 */
sldg_status sldg_vlasov_poisson_steps_2d2v(sldg_plan_t plan, int nsteps, const double* shift_x1,
                                           const double* shift_x2, const double* h, double dt,
                                           double* shift_v1, double* shift_v2, double* mass0,
                                           void* hi0, double* mass1, void* hi1,
                                           int* result_buffer);

/*
 * Kernel timing.  While enabled, every sweep kernel launch of the plan is
 * bracketed by a pair of HIP events recorded on the plan's stream (the line
 * table kernel is outside the pair), up to 4096 launches after enabling.
 * sldg_timing_enable(plan, 1) clears earlier records; (plan, 0) stops.
 * sldg_timing_read synchronises the plan's stream and returns, for launches
 * of the sweep along `dim` (dim = -1: along dimension 0; dim = -2: along
 * any dimension > 0; dim = -3: the fused (0, 1) passes), their count and the
 * sum of their durations in ms.
 */
sldg_status sldg_timing_enable(sldg_plan_t plan, int enable);
sldg_status sldg_timing_read(sldg_plan_t plan, int dim, int64_t* launches, double* total_ms);

/*
 * Plain device-to-device copy of `bytes` bytes (a multiple of 16, both
 * pointers 16-byte aligned) with one 16-byte load and store per thread, on
 * `stream`.  It measures the copy bandwidth the sweeps are compared with (the
 * paper lists copy-benchmark bandwidths beside the vendor figures, Table I)
 * and is the known-size kernel that hardware byte counters are scaled by.
 * Errors: SLDG_ERR_ARG (size or alignment), SLDG_ERR_ALIAS, SLDG_ERR_DEVICE.
 */
sldg_status sldg_device_copy(const void* src, void* dst, int64_t bytes, void* stream);

/*
 * Plane copy: nplanes planes of plane_bytes each (multiple of 16, 16-byte
 * aligned) copied with 16 bytes per thread, each thread copying the same
 * offset of planes_per_thread consecutive planes one after the other, as a
 * sweep thread walks the planes of its run of spectator tuples.  The
 * reference bandwidth of that access pattern, for the roofline.  Errors:
 * SLDG_ERR_ARG, SLDG_ERR_ALIAS, SLDG_ERR_DEVICE.
 */
sldg_status sldg_device_plane_copy(const void* src, void* dst, int64_t plane_bytes, int nplanes,
                                   int planes_per_thread, void* stream);

/* Bytes of one state's `hi` array for this plan, n_hi * cells * sizeof(T). */
int64_t sldg_hi_bytes(sldg_plan_t plan);

/*
 * Batches: many independent problems advanced together (each with its own
 * grid, degree and displacement fields; one storage tier and dimension count
 * for the whole batch).  Each sweep of a split step runs from one work list
 * of tiles of all problems, sorted by class (tile kind x degree); each class
 * is one launch of a kernel compiled for that class, and a split step can be
 * captured into one HIP graph.  The batch allocates its device tables and
 * work lists; the states are the caller's.
 */
typedef struct sldg_batch_s* sldg_batch_t;

/*   nprob   number of problems (>= 1); ndim: dimensions of every problem (1..6)
 *   ncells  host int64 [nprob * ndim]: problem p's extents at ncells[p*ndim ...],
 *           dimension 0 fastest, total per problem below 2^31
 *   k       host int [nprob]: degree of each problem (1..3)
 *   stream  hipStream_t of every later call (graph replay needs a non-null one) */
sldg_status sldg_batch_create(sldg_batch_t* batch, int nprob, int ndim, const int64_t* ncells,
                              const int* k, sldg_tier tier, void* stream);
/* Release (synchronises the stream first).  NULL is a no-op. */
void sldg_batch_destroy(sldg_batch_t batch);
/* Bind the two state buffers of every problem: host arrays [nprob] of device
 * pointers (layout of each problem as in sldg_advect_dim).  No buffer may
 * overlap another buffer of the same problem. */
sldg_status sldg_batch_bind(sldg_batch_t batch, double* const* mass0, void* const* hi0,
                            double* const* mass1, void* const* hi1);
/* The sweeps of one split step: sweep q runs along dims[q]; problem p uses
 * the dependence mask masks[q*nprob + p] and the device displacements
 * shifts[q*nprob + p] (as in sldg_advect_dim).  The per-line tables of every
 * sweep are computed now, once (section II-A: the matrices depend only on the
 * step); set the sequence again after changing displacements. */
sldg_status sldg_batch_set_sequence(sldg_batch_t batch, int nseq, const int* dims,
                                    const uint32_t* masks, const double* const* shifts);
/* nsteps split steps; sweep number q (over all steps) reads buffer q % 2 and
 * writes the other; *result_buffer receives the buffer holding the result.
 * use_graph != 0: each step is captured once (per starting buffer) into a
 * HIP graph and replayed. */
sldg_status sldg_batch_run(sldg_batch_t batch, int nsteps, int use_graph, int* result_buffer);
/* Launch-shape tuner: for every sweep of the sequence and every class of its
 * work list (tile kind: 0 dimension-0 window form, 1 dimension-0 group form,
 * 2 strided; x degree 1..3; class = 3 * kind + k - 1), times rows-per-thread
 * {2, 4, 8, 0} (strided sweeps; 0 the lane form, one cell per lane) or {4, 1}
 * (dimension 0: the group form, or with rows 1 the lane form; the window form
 * ignores rows) x
 * tuples-per-thread {1, 3, 9, all} on the bound data (reads buffer 0,
 * overwrites buffer 1) and keeps the fastest per class. */
sldg_status sldg_batch_tune(sldg_batch_t batch, int reps);
/* Set the launch shape of every class of sweep q (rows 2, 4 or 8; the lane
 * form: 1 along dimension 0, 0 along others; tuples 0 = all).  get: the shape of the class with the most tiles, and the tuned
 * time of the whole sweep (-1 if not tuned). */
sldg_status sldg_batch_get_tuning(sldg_batch_t batch, int q, int* rows, int* tuples, double* ms);
sldg_status sldg_batch_set_tuning(sldg_batch_t batch, int q, int rows, int tuples);
/* Shape, tuned time (ms, -1 if not tuned) and tile count of class `cls` (0..8)
 * of sweep q. */
sldg_status sldg_batch_get_class_tuning(sldg_batch_t batch, int q, int cls, int* rows,
                                        int* tuples, double* ms, int* nitems);
/* Set the launch shape of class `cls` of sweep q alone. */
sldg_status sldg_batch_set_class_tuning(sldg_batch_t batch, int q, int cls, int rows, int tuples);

/*
 * Device memory the library allocates for itself: plan tables, the scaled
 * FP16 partials, the field scratch and batch work lists (never the caller's
 * state buffers).  sldg_set_device_alloc_limit caps the bytes of these
 * allocations held at once, process-wide and over all devices; an allocation
 * that would pass the cap fails as if the device were out of memory, so the
 * call that needed it returns SLDG_ERR_NOMEM and leaves its plan or batch
 * usable (a plan is refused before any device call when its tables alone
 * pass the cap).  bytes = -1 removes the cap (the default); other negative
 * values give SLDG_ERR_ARG.  Allocations already held are kept when the cap
 * falls below them.  sldg_device_alloc_bytes returns the bytes held now.  A
 * robustness facility for callers that budget device memory, and the way
 * tests force the out-of-memory paths.
 */
sldg_status sldg_set_device_alloc_limit(int64_t bytes);
int64_t sldg_device_alloc_bytes(void);

const char* sldg_status_string(sldg_status s);
const char* sldg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SLDG_H */
