/*
 * adjoint.c -- oracle FP64 adjoint (vector-Jacobian product) of one MLS-MPM
 * substep, for the gradient computation of Sec. 6 (Eqs. 12-13) that feeds
 * the accumulated squared gradients g_h of Eq. 8.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * State layout: one array of n * (2d + 2d^2) doubles, x[d][n], v[d][n],
 * C[d*d][n], F[d*d][n] (component-major).  orc_step_exact maps a decoded
 * state s_t to the unquantized next state s'_{t+1} (the full-precision step
 * of Eq. 1); orc_step_vjp returns lam_t = (d s'_{t+1} / d s_t)^T lam_{t+1}.
 * The quantization is treated as an additive error (straight-through), so
 * the sensitivity of the objective to the error stored at step t is lam_t.
 *
 * Derivation notes (all written from the forward formulas of mpm.c):
 *  - weights w_ip = prod_a N(f_a + ...), d w / d x_pa = inv_dx N'_{o_a}(f_a)
 *    prod_{b != a} N_{o_b}(f_b); the base cell is locally constant;
 *  - grid: v_i = mom_i / m_i + dt g, components zeroed by the wall rule have
 *    zero derivative;
 *  - fixed-corotated stress tau = 2 mu (F - R) F^T + la J (J-1) I with the
 *    polar rotation R: dR = R Y, Y skew with S Y + Y S = skew(R^T dF -
 *    dF^T R) (F = R S).  In 3D, for symmetric S, S[y]x + [y]x S =
 *    [(tr S I - S) y]x; in 2D, S Y + Y S = tr(S) Y.
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

static void sym_polar(int dim, const double *F, double *R, double *S)
{
    orc_polar(dim, F, R);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double acc = 0.0;
            for (int k = 0; k < dim; ++k) acc += R[k * dim + i] * F[k * dim + j];
            S[i * dim + j] = acc;
        }
    /* symmetrize against round-off */
    for (int i = 0; i < dim; ++i)
        for (int j = i + 1; j < dim; ++j) {
            double a = 0.5 * (S[i * dim + j] + S[j * dim + i]);
            S[i * dim + j] = a;
            S[j * dim + i] = a;
        }
}

static double det_d(int dim, const double *F)
{
    if (dim == 2) return F[0] * F[3] - F[1] * F[2];
    return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
           F[2] * (F[3] * F[7] - F[4] * F[6]);
}

/* J F^{-T} (cofactor matrix) */
static void cofactor(int dim, const double *F, double *Cf)
{
    if (dim == 2) {
        Cf[0] = F[3]; Cf[1] = -F[2]; Cf[2] = -F[1]; Cf[3] = F[0];
        return;
    }
    Cf[0] = F[4] * F[8] - F[5] * F[7];
    Cf[1] = F[5] * F[6] - F[3] * F[8];
    Cf[2] = F[3] * F[7] - F[4] * F[6];
    Cf[3] = F[2] * F[7] - F[1] * F[8];
    Cf[4] = F[0] * F[8] - F[2] * F[6];
    Cf[5] = F[1] * F[6] - F[0] * F[7];
    Cf[6] = F[1] * F[5] - F[2] * F[4];
    Cf[7] = F[2] * F[3] - F[0] * F[5];
    Cf[8] = F[0] * F[4] - F[1] * F[3];
}

/* lamF += (d tau / d F)^T [lam_tau] for fixed-corotated elasticity */
static void stress_vjp(int dim, const double *F, double mu, double la, const double *lt, double *lamF)
{
    double R[9] = {0}, S[9] = {0}, Cf[9] = {0};
    sym_polar(dim, F, R, S);
    cofactor(dim, F, Cf);
    double J = det_d(dim, F);
    double tr_lt = 0.0;
    for (int i = 0; i < dim; ++i) tr_lt += lt[i * dim + i];
    /* terms without dR: 2mu lt F + 2mu lt^T (F - R) + la (2J - 1) tr(lt) cof(F) */
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double a = 0.0, b = 0.0;
            for (int k = 0; k < dim; ++k) {
                a += lt[i * dim + k] * F[k * dim + j];
                b += lt[k * dim + i] * (F[k * dim + j] - R[k * dim + j]);
            }
            lamF[i * dim + j] += 2.0 * mu * (a + b) + la * (2.0 * J - 1.0) * tr_lt * Cf[i * dim + j];
        }
    /* dR term: <lt, -2mu dR F^T> = -2mu <R^T lt F, Y>, Y = L^{-1}(skew(.)) */
    double M[9] = {0};
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double acc = 0.0;
            for (int k = 0; k < dim; ++k)
                for (int l = 0; l < dim; ++l) acc += R[k * dim + i] * lt[k * dim + l] * F[l * dim + j];
            M[i * dim + j] = acc;
        }
    double Y[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (dim == 2) {
        double b = 0.5 * (M[2] - M[1]); /* skew(M) = b [[0,-1],[1,0]] */
        double tr = S[0] + S[3];
        double y = (tr != 0.0) ? b / tr : 0.0;
        Y[1] = -y; Y[2] = y;
    } else {
        /* axial vector of skew(M): skew(M) = [b]x with b = (M21-M12, M02-M20, M10-M01)/2 */
        double b[3] = {0.5 * (M[7] - M[5]), 0.5 * (M[2] - M[6]), 0.5 * (M[3] - M[1])};
        double tr = S[0] + S[4] + S[8];
        double A[9];
        for (int i = 0; i < 9; ++i) A[i] = -S[i];
        A[0] += tr; A[4] += tr; A[8] += tr;
        /* solve A y = b (A = tr S I - S is SPD for S SPD) */
        double cof[9];
        cofactor(3, A, cof);
        double dA = det_d(3, A);
        double y[3] = {0, 0, 0};
        if (dA != 0.0)
            for (int i = 0; i < 3; ++i) y[i] = (cof[0 * 3 + i] * b[0] + cof[1 * 3 + i] * b[1] + cof[2 * 3 + i] * b[2]) / dA;
        /* [y]x */
        Y[1] = -y[2]; Y[2] = y[1];
        Y[3] = y[2]; Y[5] = -y[0];
        Y[6] = -y[1]; Y[7] = y[0];
    }
    /* lamF += -2mu * 2 R Y */
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double acc = 0.0;
            for (int k = 0; k < dim; ++k) acc += R[i * dim + k] * Y[k * dim + j];
            lamF[i * dim + j] += -4.0 * mu * acc;
        }
}

/* ---- shared stencil pieces ---- */
static void weights(const orc_params *p, const double *xp, int *base, double *fx, double w[3][3], double dw[3][3])
{
    double inv_dx = (double)p->grid_res;
    for (int a = 0; a < p->dim; ++a) {
        double xs = xp[a] * inv_dx;
        double b = floor(xs - 0.5);
        if (!(b >= 0.0)) b = 0.0;
        if (b > (double)(p->grid_res - 3)) b = (double)(p->grid_res - 3);
        base[a] = (int)b;
        double f = xs - b;
        fx[a] = f;
        w[a][0] = 0.5 * (1.5 - f) * (1.5 - f);
        w[a][1] = 0.75 - (f - 1.0) * (f - 1.0);
        w[a][2] = 0.5 * (f - 0.5) * (f - 0.5);
        dw[a][0] = -(1.5 - f) * inv_dx;
        dw[a][1] = -2.0 * (f - 1.0) * inv_dx;
        dw[a][2] = (f - 0.5) * inv_dx;
    }
}

static int64_t nidx(const orc_params *p, const int *ijk)
{
    int64_t n = p->grid_res;
    return p->dim == 2 ? (int64_t)ijk[1] * n + ijk[0] : ((int64_t)ijk[2] * n + ijk[1]) * n + ijk[0];
}

static int64_t nnodes(const orc_params *p)
{
    int64_t n = p->grid_res;
    return p->dim == 2 ? n * n : n * n * n;
}

/* rows of a state: x, v, C, then F (elastic) or J (fluid) */
static int nrows(const orc_params *p)
{
    int d = p->dim;
    return 2 * d + d * d + (p->material == ORC_FLUID ? 1 : d * d);
}

/* state pointers */
typedef struct { const double *x, *v, *C, *F; } cstate;
typedef struct { double *x, *v, *C, *F; } mstate;
static cstate cview(const double *s, int dim, int64_t n)
{
    cstate c = {s, s + dim * n, s + 2 * dim * n, s + (2 * dim + dim * dim) * n};
    return c;
}
static mstate mview(double *s, int dim, int64_t n)
{
    mstate c = {s, s + dim * n, s + 2 * dim * n, s + (2 * dim + dim * dim) * n};
    return c;
}

int orc_step_exact(const orc_params *p, int64_t n, const double *in, double *out)
{
    int dim = p->dim;
    int64_t nodes = nnodes(p);
    cstate s = cview(in, dim, n);
    mstate o = mview(out, dim, n);
    double *gm = calloc((size_t)nodes, sizeof(double));
    double *gmom = calloc((size_t)nodes * dim, sizeof(double));
    if (!gm || !gmom) { free(gm); free(gmom); return -1; }
    orc_p2g(p, n, s.x, s.v, s.C, s.F, gm, gmom);
    orc_grid_update(p, gm, gmom);
    orc_g2p(p, n, s.x, s.F, gmom, o.x, o.v, o.C, o.F);
    free(gm);
    free(gmom);
    return 0;
}

int orc_step_vjp(const orc_params *p, int64_t n, const double *in, const double *lam_out, double *lam_in)
{
    int dim = p->dim, D2 = dim * dim, nst = dim == 2 ? 9 : 27;
    int64_t nodes = nnodes(p);
    double inv_dx = (double)p->grid_res, dx = 1.0 / inv_dx, D = 4.0 * inv_dx * inv_dx;
    double mu = p->E / (2.0 * (1.0 + p->nu));
    double la = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
    double m = p->rho * p->p_vol;
    cstate s = cview(in, dim, n);
    cstate lo = cview(lam_out, dim, n);
    mstate li = mview(lam_in, dim, n);
    memset(lam_in, 0, sizeof(double) * (size_t)(n * nrows(p)));
    const int fluid = p->material == ORC_FLUID;
    /* forward grid (needed by both halves) */
    double *gm = calloc((size_t)nodes, sizeof(double));
    double *gmom = calloc((size_t)nodes * dim, sizeof(double));
    double *gv = malloc(sizeof(double) * (size_t)nodes * dim);
    double *lgv = calloc((size_t)nodes * dim, sizeof(double));   /* d z / d v_i */
    double *lmom = calloc((size_t)nodes * dim, sizeof(double));  /* d z / d mom_i */
    double *lm = calloc((size_t)nodes, sizeof(double));          /* d z / d m_i */
    if (!gm || !gmom || !gv || !lgv || !lmom || !lm) return -1;
    orc_p2g(p, n, s.x, s.v, s.C, s.F, gm, gmom);
    memcpy(gv, gmom, sizeof(double) * (size_t)nodes * dim);
    orc_grid_update(p, gm, gv);

    /* ---- G2P backward ---- */
    for (int64_t q = 0; q < n; ++q) {
        double xp[3], Fp[9], nC[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a < dim; ++a) xp[a] = s.x[a * n + q];
        if (!fluid)
            for (int c = 0; c < D2; ++c) Fp[c] = s.F[c * n + q];
        int base[3];
        double fx[3], w[3][3], dw[3][3];
        weights(p, xp, base, fx, w, dw);
        /* recompute C' (needed for the F' = (I + dt C') F adjoint) */
        for (int st = 0; st < nst; ++st) {
            int o[3] = {st % 3, (st / 3) % 3, st / 9}, ijk[3];
            double wt = 1.0, d[3];
            for (int a = 0; a < dim; ++a) { ijk[a] = base[a] + o[a]; wt *= w[a][o[a]]; d[a] = ((double)o[a] - fx[a]) * dx; }
            int64_t id = nidx(p, ijk);
            for (int a = 0; a < dim; ++a)
                for (int b = 0; b < dim; ++b) nC[a * dim + b] += D * wt * gv[a * nodes + id] * d[b];
        }
        double lx[3], lv[3], lC[9], lF[9];
        for (int a = 0; a < dim; ++a) { lx[a] = lo.x[a * n + q]; lv[a] = lo.v[a * n + q]; }
        for (int c = 0; c < D2; ++c) lC[c] = lo.C[c * n + q];
        if (fluid) {
            /* J' = J (1 + dt tr C') */
            double lJ = lo.F[q], tr = 0.0;
            for (int a = 0; a < dim; ++a) tr += nC[a * dim + a];
            li.F[q] += lJ * (1.0 + p->dt * tr);
            for (int a = 0; a < dim; ++a) lC[a * dim + a] += lJ * s.F[q] * p->dt;
        } else {
            for (int c = 0; c < D2; ++c) lF[c] = lo.F[c * n + q];
            /* F' = (I + dt C') F */
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) {
                    double aF = 0.0, aC = 0.0;
                    for (int k = 0; k < dim; ++k) {
                        double Mki = ((k == i) ? 1.0 : 0.0) + p->dt * nC[k * dim + i];
                        aF += Mki * lF[k * dim + j];                 /* (I + dt C')^T lF' */
                        aC += lF[i * dim + k] * Fp[j * dim + k];     /* lF' F^T */
                    }
                    li.F[(i * dim + j) * n + q] += aF;
                    lC[i * dim + j] += p->dt * aC;
                }
        }
        /* x' = x + dt v' */
        for (int a = 0; a < dim; ++a) { li.x[a * n + q] += lx[a]; lv[a] += p->dt * lx[a]; }
        /* v' = sum w v_i ; C' = D sum w v_i d^T, d = x_i - x_p */
        for (int st = 0; st < nst; ++st) {
            int o[3] = {st % 3, (st / 3) % 3, st / 9}, ijk[3];
            double wt = 1.0, d[3], gw[3];
            for (int a = 0; a < dim; ++a) { ijk[a] = base[a] + o[a]; wt *= w[a][o[a]]; d[a] = ((double)o[a] - fx[a]) * dx; }
            for (int a = 0; a < dim; ++a) {
                gw[a] = dw[a][o[a]];
                for (int b = 0; b < dim; ++b) if (b != a) gw[a] *= w[b][o[b]];
            }
            int64_t id = nidx(p, ijk);
            double lw = 0.0;
            for (int a = 0; a < dim; ++a) {
                double vi = gv[a * nodes + id];
                double ld = 0.0;
                for (int b = 0; b < dim; ++b) ld += lC[a * dim + b] * d[b];
                lgv[a * nodes + id] += wt * (lv[a] + D * ld);
                lw += lv[a] * vi + D * vi * ld;
                /* d / d x_p through d = x_i - x_p */
                for (int b = 0; b < dim; ++b) li.x[b * n + q] -= D * wt * lC[a * dim + b] * vi;
            }
            for (int a = 0; a < dim; ++a) li.x[a * n + q] += gw[a] * lw;
        }
    }

    /* ---- grid backward ---- */
    int gn = p->grid_res;
    for (int64_t id = 0; id < nodes; ++id) {
        if (!(gm[id] > 0.0)) continue;
        int ijk[3] = {(int)(id % gn), (int)((id / gn) % gn), (int)(id / ((int64_t)gn * gn))};
        for (int a = 0; a < dim; ++a) {
            double va = gmom[a * nodes + id] / gm[id] + p->dt * p->gravity[a];
            int masked = (ijk[a] < p->bound_cells && va < 0.0) || (ijk[a] >= gn - p->bound_cells && va > 0.0);
            if (masked) continue;
            double l = lgv[a * nodes + id];
            lmom[a * nodes + id] += l / gm[id];
            lm[id] -= l * gmom[a * nodes + id] / (gm[id] * gm[id]);
        }
    }

    /* ---- P2G backward ---- */
    for (int64_t q = 0; q < n; ++q) {
        double xp[3], vp[3], Cp[9], Fp[9], tau[9], A[9];
        for (int a = 0; a < dim; ++a) { xp[a] = s.x[a * n + q]; vp[a] = s.v[a * n + q]; }
        for (int c = 0; c < D2; ++c) Cp[c] = s.C[c * n + q];
        if (fluid) {
            orc_fluid_stress(dim, s.F[q], p->E, tau);
        } else {
            for (int c = 0; c < D2; ++c) Fp[c] = s.F[c * n + q];
            orc_kirchhoff(dim, Fp, mu, la, tau);
        }
        double sc = -p->dt * p->p_vol * D;
        for (int c = 0; c < D2; ++c) A[c] = sc * tau[c] + m * Cp[c];
        int base[3];
        double fx[3], w[3][3], dw[3][3];
        weights(p, xp, base, fx, w, dw);
        double lA[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int st = 0; st < nst; ++st) {
            int o[3] = {st % 3, (st / 3) % 3, st / 9}, ijk[3];
            double wt = 1.0, d[3], gw[3];
            for (int a = 0; a < dim; ++a) { ijk[a] = base[a] + o[a]; wt *= w[a][o[a]]; d[a] = ((double)o[a] - fx[a]) * dx; }
            for (int a = 0; a < dim; ++a) {
                gw[a] = dw[a][o[a]];
                for (int b = 0; b < dim; ++b) if (b != a) gw[a] *= w[b][o[b]];
            }
            int64_t id = nidx(p, ijk);
            double lw = lm[id] * m;
            for (int a = 0; a < dim; ++a) {
                double lmo = lmom[a * nodes + id];
                double Ad = 0.0;
                for (int b = 0; b < dim; ++b) Ad += A[a * dim + b] * d[b];
                lw += lmo * (m * vp[a] + Ad);
                li.v[a * n + q] += wt * m * lmo;
                for (int b = 0; b < dim; ++b) {
                    lA[a * dim + b] += wt * lmo * d[b];
                    li.x[b * n + q] -= wt * lmo * A[a * dim + b];
                }
            }
            for (int a = 0; a < dim; ++a) li.x[a * n + q] += gw[a] * lw;
        }
        /* A = sc tau(F) + m C */
        for (int c = 0; c < D2; ++c) li.C[c * n + q] += m * lA[c];
        double lt[9], lFp[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int c = 0; c < D2; ++c) lt[c] = sc * lA[c];
        if (fluid) {
            /* tau = E (J - 1) I */
            double tr = 0.0;
            for (int a = 0; a < dim; ++a) tr += lt[a * dim + a];
            li.F[q] += p->E * tr;
        } else {
            stress_vjp(dim, Fp, mu, la, lt, lFp);
            for (int c = 0; c < D2; ++c) li.F[c * n + q] += lFp[c];
        }
    }
    free(gm); free(gmom); free(gv); free(lgv); free(lmom); free(lm);
    return 0;
}

/* Objectives of the adjoint runs: 0 = centre of mass along `axis`,
 * 1 = kinetic energy.  Writes z and d z / d state. */
int orc_objective(const orc_params *p, int64_t n, const double *st, int objective, int axis, double *z,
                  double *lam)
{
    int dim = p->dim;
    double m = p->rho * p->p_vol;
    cstate s = cview(st, dim, n);
    memset(lam, 0, sizeof(double) * (size_t)(n * nrows(p)));
    mstate l = mview(lam, dim, n);
    double acc = 0.0;
    if (objective == 0) {
        for (int64_t q = 0; q < n; ++q) { acc += s.x[axis * n + q]; l.x[axis * n + q] = 1.0 / (double)n; }
        *z = acc / (double)n;
    } else {
        for (int64_t q = 0; q < n; ++q)
            for (int a = 0; a < dim; ++a) {
                double v = s.v[a * n + q];
                acc += 0.5 * m * v * v;
                l.v[a * n + q] = m * v;
            }
        *z = acc;
    }
    return 0;
}
