/*
 * orc.h -- FP64 CPU oracle for one MLS-MPM substep over bit-packed,
 * quantized particle state (Liu et al., "Automatic Quantization for
 * Physics-Based Simulation", SIGGRAPH 2022).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the GPU product path includes,
 * links or calls this code; only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark load it.  It shares no header, helper
 * or constant with the GPU library: every definition below is written
 * again here from the paper and from the readings listed with each
 * function.
 *
 * Precision: every quantity is computed in IEEE binary64 with fused
 * multiply-add only where a function says so (build with
 * -ffp-contract=off).
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Particle attributes quantized in the MPM examples of the paper
 * (Sec. 3.1, Fig. 3; Sec. 8.3): position, velocity, affine velocity C, and
 * either the deformation gradient F (elastic solid) or the volume ratio J
 * (fluid).  F and J share the fourth state slot: arrays passed for "F"
 * hold J (one row) for a fluid. */
enum { ORC_X = 0, ORC_V = 1, ORC_C = 2, ORC_F = 3, ORC_J = 4 };
/* Materials: fixed-corotated elastic solid (F), weakly compressible fluid (J)
 * with Kirchhoff stress E (J - 1) I, E the pressure coefficient. */
enum { ORC_ELASTIC = 0, ORC_FLUID = 1 };
/* Storage kinds: fixed point (Eq. 3), shared-exponent float, raw float32. */
enum { ORC_FIXED = 0, ORC_SHARED_EXP = 1, ORC_RAW_F32 = 2 };

typedef struct {
    int32_t field;        /* ORC_X .. ORC_J */
    int32_t kind;         /* ORC_FIXED / ORC_SHARED_EXP / ORC_RAW_F32 */
    int32_t bits;         /* bits per component (SHARED_EXP: sign + magnitude) */
    int32_t exp_bits;     /* SHARED_EXP only: width of the shared exponent */
    int32_t dither;       /* 1: Eq. 11 dithered rounding, 0: round to nearest */
    int32_t rel_identity; /* F only: store F - I instead of F */
    double lo, hi;        /* FIXED: value range [lo, hi); SHARED_EXP: |v| < hi */
} orc_field;

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t n_fields;     /* always 4; array order = bit placement order */
    orc_field f[4];
    uint64_t seed;        /* Philox key */
} orc_scheme;

typedef struct {
    int32_t dim, grid_res, bound_cells, sort_every;
    double dt, gravity[3], E, nu, rho, p_vol;
    int32_t material, pad;   /* ORC_ELASTIC / ORC_FLUID */
} orc_params;

/* Per-field statistics: saturations, NaN inputs, round-ups, round-downs. */
typedef struct { int64_t sat, nan, up, down; } orc_stat;

/* ---- layout / codec (codec.c) ---- */
int  orc_layout(const orc_scheme *s, int32_t *comp_offset, int32_t *field_offset,
                int32_t *total_bits, int32_t *W);
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
int  orc_encode(const orc_scheme *s, int64_t n, const float *x, const float *v,
                const float *C, const float *F, uint32_t step, uint32_t tag,
                uint32_t *words, orc_stat *stats);
int  orc_encode_f64(const orc_scheme *s, int64_t n, const double *x, const double *v,
                    const double *C, const double *F, uint32_t step, uint32_t tag,
                    uint32_t *words, orc_stat *stats);
int  orc_decode(const orc_scheme *s, int64_t n, const uint32_t *words,
                double *x, double *v, double *C, double *F);
int  orc_validate(const orc_scheme *s);

/* ---- MLS-MPM (mpm.c) ---- */
void orc_polar(int dim, const double *F, double *R);
void orc_kirchhoff(int dim, const double *F, double mu, double la, double *tau);
void orc_fluid_stress(int dim, double J, double E, double *tau);
int  orc_p2g(const orc_params *p, int64_t n, const double *x, const double *v,
             const double *C, const double *F, double *grid_m, double *grid_mom);
int  orc_grid_update(const orc_params *p, double *grid_m, double *grid_mom);
int  orc_g2p(const orc_params *p, int64_t n, const double *x, const double *F,
             const double *grid_v, double *x_new, double *v_new, double *C_new,
             double *F_new);
int  orc_sort_order(const orc_params *p, int64_t n, const double *x, int64_t *order);

/* ---- adjoint (adjoint.c): state = x[d][n], v[d][n], C[d*d][n], F[d*d][n]
 * (fluid: J[1][n] in place of F) ---- */
int  orc_step_exact(const orc_params *p, int64_t n, const double *in, double *out);
int  orc_step_vjp(const orc_params *p, int64_t n, const double *in, const double *lam_out,
                  double *lam_in);
int  orc_objective(const orc_params *p, int64_t n, const double *st, int objective, int axis,
                   double *z, double *lam);

typedef struct orc_sim orc_sim;
orc_sim *orc_sim_new(const orc_scheme *s, const orc_params *p, int64_t n,
                     const uint32_t *words);
int  orc_sim_step(orc_sim *sim, int32_t nsteps);
void orc_sim_words(const orc_sim *sim, uint32_t *out);
void orc_sim_ids(const orc_sim *sim, int64_t *out);
void orc_sim_stats(const orc_sim *sim, orc_stat *out);
int64_t orc_sim_step_count(const orc_sim *sim);
void orc_sim_free(orc_sim *sim);

#ifdef __cplusplus
}
#endif
#endif
