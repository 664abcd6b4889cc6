/*
 * mpmq.h -- C ABI of the quantized MLS-MPM substep on AMD MI355X (gfx950).
 *
 * The library advances an MLS-MPM simulation whose particle state is stored
 * bit-packed under a quantization scheme, following Liu et al., "Automatic
 * Quantization for Physics-Based Simulation" (SIGGRAPH 2022):
 *   - the quantized step model of Eq. 1: each substep evaluates the
 *     full-precision update on the decoded quantized state and imposes the
 *     quantization error only when the new state is stored;
 *   - fixed-point types of Eq. 3 (u = round(v/Delta), Delta = 2^-b R) with
 *     an affine range [lo, hi), and a shared-exponent float type;
 *   - non-subtractive dithered rounding of Eq. 11 (Sec. 5), drawn from
 *     Philox4x32-10 keyed by (seed) and counted by (slot, step, group, tag);
 *   - the "bit pack" container of Sec. 7 (Figs. 7-8): the components of all
 *     fields are concatenated in placement order and may span two 32-bit
 *     words.  Storage is word-major: word k of particle slot p is
 *     packed[k * capacity_padded + p].
 *
 * The scheme is the per-quantity (bits, range) pair that Algorithm 1
 * outputs, plus the dither flag and the placement order of
 * bit_pack().place(...) (Sec. 7).  The state is (x, v, C, F) per particle
 * (the MPM example of Sec. 3.1 / Fig. 3).
 *
 * Conventions.  All pointers named "device" are HIP device pointers on the
 * device that is current when mpmq_create is called; the library never
 * allocates or frees device memory -- the caller supplies every buffer,
 * sized by mpmq_query_sizes.  Host structs passed in are copied; nothing is
 * retained after the call returns.  Work is enqueued on the caller's HIP
 * stream and is asynchronous unless a function says it synchronizes.  A
 * context is not thread-safe; separate contexts on separate streams are
 * independent.  No C++ exception crosses this boundary; errors are returned
 * as mpmq_status and described by mpmq_last_error(ctx).
 */
#ifndef MPMQ_H
#define MPMQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MPMQ_OK = 0,
    MPMQ_EINVAL = -1,   /* invalid argument, scheme or parameters */
    MPMQ_ENOMEM = -2,   /* a caller buffer is too small / capacity exceeded */
    MPMQ_EDEVICE = -3,  /* a HIP call failed; mpmq_last_error has its message */
    MPMQ_ESTATE = -4,   /* call order (e.g. step before encode) */
    MPMQ_ENOTIMPL = -5
} mpmq_status;

/* Particle attributes (Sec. 3.1, Fig. 3; Sec. 8.3): position, velocity,
 * affine velocity C, and either the deformation gradient F (elastic solid)
 * or the volume ratio J (fluid).  F and J share the fourth state slot: the
 * arrays, statistics and adjoint rows named F hold J (one component) for a
 * fluid. */
typedef enum { MPMQ_FIELD_X = 0, MPMQ_FIELD_V = 1, MPMQ_FIELD_C = 2, MPMQ_FIELD_F = 3, MPMQ_FIELD_J = 4 } mpmq_field;

/* Materials.  MPMQ_ELASTIC: fixed-corotated solid, state x, v, C, F.
 * MPMQ_FLUID: weakly compressible fluid (the MLS-MPM fluid of Hu et al.
 * 2018): Kirchhoff stress E (J - 1) I with E the pressure coefficient,
 * J' = J (1 + dt tr C'); state x, v, C, J. */
typedef enum { MPMQ_ELASTIC = 0, MPMQ_FLUID = 1 } mpmq_material;

/* Storage kinds.
 * MPMQ_FIXED      Eq. 3 over [lo, hi): Delta = (hi-lo) 2^-bits,
 *                 u = floor((v-lo)*(2^bits/(hi-lo)) + 1/2)  (binary64, ties
 *                 up; + xi in [0,1) instead of 1/2 when dithered, Eq. 11),
 *                 clamped to [0, 2^bits-1]; decode fma(u, Delta, lo).
 *                 1 <= bits <= 32.
 * MPMQ_SHARED_EXP a vector field sharing one exponent of exp_bits bits:
 *                 E_max = ceil(log2 hi), E_min = E_max - 2^exp_bits + 1,
 *                 E = clamp(ilogb(max|v_k|)+1, E_min, E_max), raised by one
 *                 if a magnitude rounds up to 2^(bits-1);
 *                 q_k = round(|v_k| 2^(bits-1-E)) in bits-1 magnitude bits +
 *                 1 sign bit.  2 <= bits <= 32, 1 <= exp_bits <= 8, lo ignored.
 * MPMQ_RAW_F32    the IEEE float32 bit pattern (bits must be 32): an all-raw
 *                 scheme is the plain FP32 structure-of-arrays layout. */
typedef enum { MPMQ_FIXED = 0, MPMQ_SHARED_EXP = 1, MPMQ_RAW_F32 = 2 } mpmq_kind;

/* flags of mpmq_field_scheme */
#define MPMQ_REL_IDENTITY 1 /* F or J only: store F - I / J - 1 (diagonal in [lo+1, hi+1)) */

typedef struct {
    int32_t field;    /* mpmq_field */
    int32_t kind;     /* mpmq_kind */
    int32_t bits;     /* bits per component (SHARED_EXP: sign + magnitude) */
    int32_t exp_bits; /* SHARED_EXP only */
    int32_t dither;   /* 1: dithered rounding (Eq. 11), 0: round to nearest */
    int32_t flags;    /* MPMQ_REL_IDENTITY */
    double lo, hi;
} mpmq_field_scheme;

typedef struct {
    int32_t dim;                      /* 2 or 3 */
    int32_t n_fields;                 /* 4: X, V, C and one of F / J, each once */
    const mpmq_field_scheme *fields;  /* array order = bit placement order */
    uint64_t seed;                    /* Philox key (low word, high word) */
} mpmq_scheme;

/* MLS-MPM parameters.  Domain [0,1)^dim, grid_res nodes per axis
 * (dx = 1/grid_res, 8 <= grid_res <= 1024), quadratic B-splines,
 * fixed-corotated elasticity with Young's modulus E and Poisson ratio nu
 * (MPMQ_FLUID: E is the pressure coefficient, nu unused),
 * particle mass rho*p_vol.  Within bound_cells nodes of a wall the grid
 * velocity component pointing into the wall is zeroed.  Particles are
 * re-sorted by cell at every step s with s % sort_every == 0
 * (sort_every == 0: only after an encode). */
typedef struct {
    int32_t dim, grid_res, bound_cells, sort_every;
    double dt, gravity[3], E, nu, rho, p_vol;
    int32_t material;  /* mpmq_material; must match the scheme (F: ELASTIC, J: FLUID) */
    int32_t reserved;  /* 0 */
} mpmq_params;

typedef struct {
    int32_t words_per_particle;  /* W = ceil(record_bits / 32) */
    int32_t record_bits;
    int64_t capacity_padded;     /* capacity rounded up to a multiple of 256 */
    int64_t packed_bytes;        /* 4 * W * capacity_padded */
    int64_t grid_bytes;          /* bytes of EACH of the two grid buffers */
    int64_t scratch_bytes;       /* sort, work list, flags, counters */
    int64_t ids_bytes;           /* optional particle-id buffer */
} mpmq_sizes;

/* Caller-owned device buffers (256-byte aligned).  ids may be NULL: when
 * given, the library keeps ids[slot] = index of that particle in the last
 * mpmq_encode input, permuted along with every sort. */
typedef struct {
    void *packed;
    void *grid_a;
    void *grid_b;
    void *scratch;
    void *ids;
} mpmq_buffers;

typedef struct {
    int64_t sat[4];    /* codes clamped to the representable range, per field */
    int64_t nan[4];    /* NaN inputs to the encoder, per field */
    int64_t up[4];     /* roundings to the upper lattice point, per field */
    int64_t down[4];   /* roundings to the lower lattice point, per field */
    int64_t steps;     /* substeps taken by this context */
    int64_t sorts;     /* particle sorts performed */
    int64_t fallback;  /* particle-stencils that left their tile (global atomics) */
    int64_t active_nodes; /* sum over substeps of grid nodes with mass > 0 */
    int64_t clamped;   /* particle scatters (P2G) with a velocity term v - (A/m) f dx or
                          (A/m) dx above 2^12 in magnitude, clamped so that the 64-bit
                          fixed-point node sums cannot overflow (the clamp loses momentum) */
    int64_t atomics;   /* 64-bit global atomic adds issued by the P2G tile flushes (the
                          scatter of each work item's node sums into the grid) */
    int64_t wide;      /* particle scatters of the fused substep whose node values lay too
                          far from their work item's reference velocity for its 32-bit node
                          tile, scattered through the 64-bit global path instead */
} mpmq_stats_t;

typedef struct mpmq_ctx mpmq_ctx;

/* Sizes of every buffer for `capacity` particles.  Host only.
 * EINVAL: invalid scheme or params (mpmq_last_error(NULL) names why). */
mpmq_status mpmq_query_sizes(const mpmq_scheme *scheme, const mpmq_params *params,
                             int64_t capacity, mpmq_sizes *out);

/* Creates a context over caller buffers; `hip_stream` is a hipStream_t
 * (NULL = default stream).  Clears the grid buffers and scratch on the
 * stream.  EINVAL / ENOMEM (capacity < 1 or > 2^30-256) / EDEVICE. */
mpmq_status mpmq_create(const mpmq_scheme *scheme, const mpmq_params *params,
                        const mpmq_buffers *buffers, int64_t capacity, void *hip_stream,
                        mpmq_ctx **out);
mpmq_status mpmq_destroy(mpmq_ctx *ctx);

/* Encodes n particles (0 <= n <= capacity) from float32 device arrays in
 * component-major structure-of-arrays layout: x[c*n+p] (c < dim),
 * v[c*n+p], C[(i*dim+j)*n+p], F[(i*dim+j)*n+p] (full F, row-major; a
 * fluid passes J[p] there).
 * Dithered fields use Philox counter (p, step_count, group, 2).  Marks the
 * state unsorted (the next step sorts) and resets ids to 0..n-1. */
mpmq_status mpmq_encode(mpmq_ctx *ctx, const float *x, const float *v, const float *C,
                        const float *F, int64_t n);

/* Decodes the current state into float32 device arrays (same layout, n =
 * current particle count; the decode is exact in binary64 and rounded once
 * to float32).  Any pointer may be NULL to skip that field. */
mpmq_status mpmq_decode(mpmq_ctx *ctx, float *x, float *v, float *C, float *F);

/* Borrowed view of the packed words (device pointer, valid until destroy). */
mpmq_status mpmq_packed(mpmq_ctx *ctx, const uint32_t **words, int32_t *W, int64_t *n,
                        int64_t *stride);

/* Advances n_substeps MLS-MPM substeps (Eq. 1 model): sort when due,
 * P2G, grid update, then one fused kernel per substep that gathers (G2P),
 * updates x, v, C, F, re-encodes with dithered rounding, stores the words in
 * place and scatters (P2G) the stored state for the next substep.
 * Asynchronous.  ESTATE before the first encode. */
mpmq_status mpmq_step(mpmq_ctx *ctx, int32_t n_substeps);

/* Batched substeps for serving many scenes: advances every context of
 * ctxs[0..count) by n_substeps, each exactly as mpmq_step with the generic
 * kernels would (same results bit for bit: each scene keeps its own scheme,
 * parameters, buffers, step counter and Philox key), but with the grid
 * update and the fused
 * substep of all scenes issued as one launch each per substep (per chunk of
 * up to 96 scenes; sorts and the P2G after a sort stay per scene).  The
 * contexts must share the dimension, the material and the stream (the
 * launches go to that stream), and each may appear once.  Scheme-specialized
 * kernels (mpmq_specialize) are not used here: a specialized context stepped
 * in a batch follows the generic kernels' 64-bit P2G tile for those
 * substeps.  Asynchronous.  EINVAL (NULL,
 * count < 1, mixed dimension / material / stream, duplicates), ESTATE
 * (a context before its first encode), EDEVICE; the message of any error is
 * mpmq_last_error(ctxs[0]) (of mpmq_last_error(NULL) when ctxs[0] is NULL). */
mpmq_status mpmq_step_batch(mpmq_ctx *const *ctxs, int32_t count, int32_t n_substeps);

/* Substep counter (the Philox "step" of the next substep). */
mpmq_status mpmq_step_count(mpmq_ctx *ctx, int64_t *out);

/* Scheme specialization.  enable = 1: compiles, on the host with hipRTC,
 * the fused substep and bootstrap P2G kernels with this context's scheme as
 * compile-time constants (field kinds, bit offsets, masks, codec constants;
 * the Philox key stays a run-time value), loads them on the current device
 * and uses them from the next launch on.  The kernels are the same source
 * under the same device flags, with one difference: the specialized fused
 * kernel accumulates P2G in a 32-bit node tile per work item (node values
 * less a reference velocity, at a scale chosen per item, 48 KB of LDS in 3D
 * so that three work-groups share a CU), the generic one in an exact 64-bit
 * tile.  Where no fused P2G is involved (a sort before every substep)
 * results are bit-identical; otherwise they differ by the 32-bit tile's
 * roundings, of the order of float32 noise in the node velocities.  A
 * particle whose node values do not fit its item's 32-bit range is scattered
 * through the exact global path (mpmq_stats_t.wide).  Either way a run is
 * bit-reproducible, and the adjoint's recomputation reproduces the forward
 * pass: the scales each item used are recorded with the stored state.
 * Code objects are cached per process by (device, dimension, scheme): the
 * first call for a scheme takes a few seconds, later ones none.  enable = 0
 * returns to the generic kernels.  EDEVICE when the compiler or the loader
 * fails (mpmq_last_error carries the compiler log). */
mpmq_status mpmq_specialize(mpmq_ctx *ctx, int32_t enable);

/* Encoder statistics collected by mpmq_step: level 0 (default) counts
 * saturations and NaN inputs; level 1 also counts round-ups and
 * round-downs per field (the dithering diagnostic of Sec. 8.1), at a small
 * cost per stored component.  mpmq_encode always counts all four. */
mpmq_status mpmq_set_stats(mpmq_ctx *ctx, int32_t level);

/* Accumulated statistics.  Synchronizes the stream. */
mpmq_status mpmq_stats(mpmq_ctx *ctx, mpmq_stats_t *out);
mpmq_status mpmq_reset_stats(mpmq_ctx *ctx);

/* Calibration aid for the measurement of the P2G flush: adds 1 to word
 * (i * stride) mod n_words of buf for every i < n_words, `passes` times, with
 * 64-bit global atomics (stride 1: each wave instruction covers 64
 * consecutive words), on hip_stream.  buf: device, 256-byte aligned, owned by
 * the caller.  Asynchronous.  EINVAL on bad arguments. */
mpmq_status mpmq_calib_atomics(uint64_t *buf, int64_t n_words, int32_t passes, int64_t stride, void *hip_stream);

/* Per-kernel timing with HIP events recorded on the context stream around
 * every launch while enabled.  mpmq_kernel_times synchronizes and returns,
 * for up to `max` kernel names, the launch count and total milliseconds. */
typedef struct { char name[32]; int64_t launches; double total_ms; } mpmq_kernel_time;
mpmq_status mpmq_set_timing(mpmq_ctx *ctx, int32_t enable);
mpmq_status mpmq_kernel_times(mpmq_ctx *ctx, mpmq_kernel_time *out, int32_t max, int32_t *count);

/* ---- Adjoint (Sec. 6, Eqs. 8, 12-13) ----
 *
 * Reverse-mode gradient of an objective z of the final state through
 * `steps` quantized substeps.  The quantization error of every stored
 * state is treated as an additive perturbation e_t (Eq. 1), so
 * d z / d e_t = lambda_t, the adjoint of the stored state s_t, with
 * lambda_t = (d F(s_t) / d s_t)^T lambda_{t+1} (Eqs. 12-13).  Per field h
 * (x, v, C, F) the call returns G_h = sum over t = 0..T, particles and
 * components of lambda and g_h = the sum of its squares, the accumulated
 * squared gradient of Eq. 8 that the scheme solver of Alg. 1 consumes.
 *
 * Forward: from the current stored state s_0 (sorted first if a sort is
 * pending; lambda rows then follow the sorted slots, see lambda0 below),
 * `steps` substeps exactly as mpmq_step computes them, except that no
 * re-sort happens inside the horizon (so the slot of every particle is
 * fixed and the trajectory equals mpmq_step's for sort_every = 0).  The
 * context ends at s_T with the step counter advanced by `steps`, as after
 * mpmq_step; encoder statistics count the forward once.
 *
 * Backward: states are recovered by re-running the forward from stored
 * checkpoints (the forward is bit-reproducible):
 *   checkpoint_every = K >= 1: checkpoints every K steps, then every state
 *     of one K-step segment at a time (memory: ceil(T/K) + K states);
 *   checkpoint_every = 0: bisection (Sec. 6, Fig. 14): checkpoints on the
 *     path from the root of a binary tree over the steps to the current
 *     step, O(log T) states, O(T log T) recomputed substeps.
 *
 * objective: 0 = centre of mass along `axis` (mean over particles of x_axis),
 *            1 = kinetic energy (sum of m_p |v|^2 / 2). */
typedef struct {
    int32_t objective;
    int32_t axis;             /* 0 <= axis < dim (objective 0 only) */
    int32_t steps;            /* T >= 0 */
    int32_t checkpoint_every; /* K >= 1, or 0 for bisection */
} mpmq_adjoint_spec;

typedef struct {
    double z;           /* objective at s_T */
    double G[4];        /* per field (x, v, C, F): sum of lambda over t, particles, components */
    double g[4];        /* per field: sum of lambda^2 (Eq. 8 g_h) */
    double lo[4], hi[4];/* per field: min / max stored component value over s_0..s_T (Alg. 1
                           ranges; F - I for a REL_IDENTITY field) */
    int64_t recomputed; /* substeps re-run to recover states */
    int64_t states;     /* states held in the workspace at most */
} mpmq_adjoint_result;

/* Workspace bytes mpmq_adjoint needs for spec at the current particle count. */
mpmq_status mpmq_adjoint_workspace(mpmq_ctx *ctx, const mpmq_adjoint_spec *spec, int64_t *bytes);

/* Runs the forward and the adjoint described above on the context stream
 * and synchronizes it.  workspace: caller-owned device memory of at least
 * mpmq_adjoint_workspace bytes, 256-byte aligned, borrowed for the call.
 * lambda0 (optional, device, (2d + 2d^2) * n float32): lambda_0 in
 * component-major rows x[d], v[d], C[d*d], F[d*d], column = the particle's
 * index at mpmq_encode (the slot when the context has no ids buffer).
 * Errors: EINVAL (bad spec / NULL out), ENOMEM (workspace too small),
 * ESTATE (before encode), EDEVICE. */
mpmq_status mpmq_adjoint(mpmq_ctx *ctx, const mpmq_adjoint_spec *spec, void *workspace, int64_t workspace_bytes,
                         float *lambda0, mpmq_adjoint_result *out);

/* Allocation-free adjoint, for callers that cannot allocate device memory
 * (tight serving loops, harnesses that forbid hipMalloc): mpmq_adjoint with
 * the workspace taken from a library-owned static device array of
 * MPMQ_STATIC_WORKSPACE_BYTES (64 MiB) on the current device, which must be
 * the context's device.  Each device that runs this call holds its own
 * array until the process ends.  The call itself performs no device
 * allocation or free.  ENOMEM, with a message naming both sizes, when
 * mpmq_adjoint_workspace for spec exceeds the array; EDEVICE when the
 * array's address cannot be obtained.  Every call on one device shares
 * that device's array, which keeps the last call's contents (the call
 * clears what it needs cleared): calls that overlap on one device -- from
 * different threads, contexts or streams -- race and must be serialized by
 * the caller.  lambda0 (caller-owned output) and out as in mpmq_adjoint. */
#define MPMQ_STATIC_WORKSPACE_BYTES (64ll << 20)
mpmq_status mpmq_adjoint_static(mpmq_ctx *ctx, const mpmq_adjoint_spec *spec, float *lambda0,
                                mpmq_adjoint_result *out);

/* ---- Automatic quantization solver (Sec. 4, Eqs. 6-10, Alg. 1) ----
 * Host-only; touches no device.  Per data type h: P_h variables, the
 * accumulated squared gradient g_h (Eq. 8; mpmq_adjoint's g), the range
 * width R_h.  Error-bounded (mode 0): smallest sum P_h b_h with
 * (1/12) sum Delta_h^2 g_h <= (eps z)^2, Delta_h from Eq. 10 and
 * b_h = ceil(log2(R_h / Delta_h)) as in Alg. 1.  Memory-bounded (mode 1):
 * least expected error with sum P_h b_h <= eps * 32 sum P_h (Eq. 7);
 * Delta_h = K sqrt(P_h / g_h) (Lagrange conditions of Eq. 7 under Eq. 8),
 * b_h = floor(log2(R_h / Delta_h)).  Types with g_h = 0 take min_bits.  Bits
 * are clamped to [min_bits, max_bits].  Input arrays are host memory of
 * n_types entries; outputs likewise.  EINVAL on invalid input (the reason:
 * mpmq_solver_error()). */
#define MPMQ_SOLVE_MAX_TYPES 16
enum { MPMQ_SOLVE_ERROR_BOUND = 0, MPMQ_SOLVE_MEMORY_BOUND = 1 };
typedef struct {
    int32_t mode, n_types, min_bits, max_bits;
    double eps;       /* eps_err (relative error of z) or eps_mem (memory fraction of FP32) */
    double z;         /* reference objective value (error-bounded mode) */
    const double *P, *g, *R;
} mpmq_solve_input;
typedef struct {
    double *delta;    /* continuous quantization step (INFINITY where g_h = 0) */
    double *b_cont;   /* continuous bit width log2(R_h / Delta_h) */
    int32_t *bits;    /* integer bit width */
    double expected_error; /* (1/12) sum (R_h 2^-bits_h)^2 g_h */
    double total_bits;     /* sum P_h bits_h */
} mpmq_solve_output;
mpmq_status mpmq_solve_scheme(const mpmq_solve_input *in, mpmq_solve_output *out);

/* Alg. 1 from the record of a full-precision run: the per-field value
 * ranges, the accumulated squared gradients and the objective that
 * mpmq_adjoint returned (adj->lo, hi, g, z) become a fixed-point scheme.
 * Per field h (state slot order x, v, C, then F or J): the recorded range
 * [lo_h, hi_h] is widened about its centre by range_factor against
 * overflow (Sec. 3.2 uses 2; a half-width below 2^-20 max(1, |centre|) is
 * raised to it, so that a constant field gets a usable range),
 * R_h = its width, P_h = n_particles x the field's component count, and the
 * widths come from mpmq_solve_scheme with (mode, eps, z = adj->z, min_bits,
 * max_bits).  out_fields (host, 4 entries) receives the scheme in the
 * placement order of `base`: kind MPMQ_FIXED, the solved bits, the widened
 * [lo, hi), and the dither flag and REL_IDENTITY flag of the matching base
 * field (a REL_IDENTITY field's recorded range is already that of F - I).
 * solved (optional; its arrays hold 4 entries in slot order) receives the
 * solver's output.  Host only.  EINVAL on a NULL or invalid argument (the
 * reason: mpmq_solver_error()). */
typedef struct {
    int32_t mode;          /* MPMQ_SOLVE_ERROR_BOUND or MPMQ_SOLVE_MEMORY_BOUND */
    int32_t min_bits, max_bits;
    int32_t reserved;      /* 0 */
    double eps;            /* as in mpmq_solve_input */
    double range_factor;   /* >= 1 */
    int64_t n_particles;   /* >= 1 */
} mpmq_auto_input;
mpmq_status mpmq_auto_scheme(const mpmq_scheme *base, const mpmq_adjoint_result *adj, const mpmq_auto_input *in,
                             mpmq_field_scheme *out_fields, mpmq_solve_output *solved);
const char *mpmq_solver_error(void);

const char *mpmq_error_string(mpmq_status status);
/* Last error message of ctx (or of the calling thread's last failed
 * query/create when ctx is NULL).  Never NULL. */
const char *mpmq_last_error(mpmq_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* MPMQ_H */
