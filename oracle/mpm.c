/*
 * mpm.c -- oracle MLS-MPM substep (FP64) under the quantized-state model
 * of Eq. 1: the full-precision step acts on the decoded quantized state and
 * the error is imposed only when the new state is stored.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * The paper runs the MLS-MPM elastic simulator of Hu et al. 2018 (Sec. 8.1)
 * without printing its equations; this file writes out that method with
 * quadratic B-spline weights and fixed-corotated elasticity:
 *   P2G   base = floor(x/dx - 1/2), f = x/dx - base,
 *         w0 = (1.5-f)^2/2, w1 = 3/4-(f-1)^2, w2 = (f-1/2)^2/2 per axis,
 *         tau = 2 mu (F-R) F^T + lambda J (J-1) I      (Kirchhoff stress)
 *         A = -dt p_vol 4/dx^2 tau + m_p C
 *         node i += w (m_p v + A (x_i - x_p)),  m_i += w m_p
 *   grid  v_i = mom_i/m_i + dt g; within `bound_cells` nodes of a wall the
 *         velocity component pointing into that wall is zeroed
 *   G2P   v' = sum w v_i,  C' = 4/dx^2 sum w v_i (x_i - x_p)^T,
 *         x' = x + dt v',  F' = (I + dt C') F
 * Readings where the paper is silent: the base cell is clamped to
 * [0, n-3] per axis so the stencil stays inside the grid; the wall rule
 * above; the polar rotation of a reflected F (det F < 0) is the rotation
 * closest to it (sign of the smallest singular value flipped).
 *
 * Particle sort (not a step of the paper; it fixes which slot, and hence
 * which dither stream, each particle occupies): cells are grouped in
 * blocks of 8^3 (3D) or 16^2 (2D) cells; particles are ordered by
 * (block, rank of the particle among those of its cell in slot order,
 * cell within block, previous slot).
 */
#include "orc.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------- small dense linear algebra ---------------- */

static double det3(const double *A)
{
    return A[0] * (A[4] * A[8] - A[5] * A[7]) - A[1] * (A[3] * A[8] - A[5] * A[6]) +
           A[2] * (A[3] * A[7] - A[4] * A[6]);
}

/* Cyclic Jacobi eigen-decomposition of a symmetric 3x3 matrix:
 * A = V diag(lam) V^T, columns of V are eigenvectors. */
static void jacobi_eig3(const double *Ain, double *lam, double *V)
{
    double A[9];
    memcpy(A, Ain, sizeof(A));
    for (int i = 0; i < 9; ++i) V[i] = (i % 4 == 0) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 64; ++sweep) {
        double off = A[1] * A[1] + A[2] * A[2] + A[5] * A[5];
        double diag = A[0] * A[0] + A[4] * A[4] + A[8] * A[8];
        if (off <= 1e-40 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p) {
            for (int q = p + 1; q < 3; ++q) {
                double apq = A[p * 3 + q];
                if (apq == 0.0) continue;
                double app = A[p * 3 + p], aqq = A[q * 3 + q];
                double theta = (aqq - app) / (2.0 * apq);
                double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* A <- J^T A J with the rotation in the (p,q) plane */
                for (int k = 0; k < 3; ++k) {
                    double akp = A[k * 3 + p], akq = A[k * 3 + q];
                    A[k * 3 + p] = c * akp - s * akq;
                    A[k * 3 + q] = s * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {
                    double apk = A[p * 3 + k], aqk = A[q * 3 + k];
                    A[p * 3 + k] = c * apk - s * aqk;
                    A[q * 3 + k] = s * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {
                    double vkp = V[k * 3 + p], vkq = V[k * 3 + q];
                    V[k * 3 + p] = c * vkp - s * vkq;
                    V[k * 3 + q] = s * vkp + c * vkq;
                }
            }
        }
    }
    lam[0] = A[0]; lam[1] = A[4]; lam[2] = A[8];
}

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static void normalize3(double *a)
{
    double n = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
    if (n > 0) { a[0] /= n; a[1] /= n; a[2] /= n; }
}

/* Rotation factor of the polar decomposition F = R S (row-major). */
void orc_polar(int dim, const double *F, double *R)
{
    if (dim == 2) {
        double c = F[0] + F[3], s = F[2] - F[1];
        double r = sqrt(c * c + s * s);
        if (r == 0.0) { c = 1.0; s = 0.0; } else { c /= r; s /= r; }
        R[0] = c; R[1] = -s; R[2] = s; R[3] = c;
        return;
    }
    /* SVD through the eigen-decomposition of F^T F. */
    double FtF[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += F[k * 3 + i] * F[k * 3 + j];
            FtF[i * 3 + j] = acc;
        }
    double lam[3], V[9];
    jacobi_eig3(FtF, lam, V);
    /* order singular values descending */
    int idx[3] = {0, 1, 2};
    for (int a = 0; a < 3; ++a)
        for (int b = a + 1; b < 3; ++b)
            if (lam[idx[b]] > lam[idx[a]]) { int t = idx[a]; idx[a] = idx[b]; idx[b] = t; }
    double v[3][3], u[3][3], sig[3];
    for (int a = 0; a < 3; ++a) {
        sig[a] = sqrt(lam[idx[a]] > 0 ? lam[idx[a]] : 0.0);
        for (int k = 0; k < 3; ++k) v[a][k] = V[k * 3 + idx[a]];
    }
    /* make V a proper rotation */
    double vc[3];
    cross3(v[0], v[1], vc);
    if (vc[0] * v[2][0] + vc[1] * v[2][1] + vc[2] * v[2][2] < 0)
        for (int k = 0; k < 3; ++k) v[2][k] = -v[2][k];
    if (sig[0] == 0.0) {
        for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
        return;
    }
    for (int a = 0; a < 2; ++a)
        for (int k = 0; k < 3; ++k)
            u[a][k] = F[k * 3 + 0] * v[a][0] + F[k * 3 + 1] * v[a][1] + F[k * 3 + 2] * v[a][2];
    normalize3(u[0]);
    /* Gram-Schmidt u1 against u0; fall back to any orthogonal direction */
    double d = u[1][0] * u[0][0] + u[1][1] * u[0][1] + u[1][2] * u[0][2];
    for (int k = 0; k < 3; ++k) u[1][k] -= d * u[0][k];
    double n1 = sqrt(u[1][0] * u[1][0] + u[1][1] * u[1][1] + u[1][2] * u[1][2]);
    if (sig[1] <= 1e-300 || n1 <= 1e-12 * sig[0]) {
        double e[3] = {0, 0, 0};
        int m = 0;
        for (int k = 1; k < 3; ++k) if (fabs(u[0][k]) < fabs(u[0][m])) m = k;
        e[m] = 1.0;
        cross3(u[0], e, u[1]);
    }
    normalize3(u[1]);
    cross3(u[0], u[1], u[2]);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            R[i * 3 + j] = u[0][i] * v[0][j] + u[1][i] * v[1][j] + u[2][i] * v[2][j];
}

/* Kirchhoff stress of fixed-corotated elasticity,
 * psi = mu |F-R|^2 + lambda/2 (J-1)^2,  tau = dpsi/dF F^T. */
/* Weakly compressible fluid: Kirchhoff stress E (J - 1) I (E the pressure
 * coefficient; the MLS-MPM fluid of Hu et al. 2018). */
void orc_fluid_stress(int dim, double J, double E, double *tau)
{
    for (int i = 0; i < dim * dim; ++i) tau[i] = 0.0;
    for (int a = 0; a < dim; ++a) tau[a * dim + a] = E * (J - 1.0);
}

void orc_kirchhoff(int dim, const double *F, double mu, double la, double *tau)
{
    double R[9];
    orc_polar(dim, F, R);
    double J = (dim == 2) ? F[0] * F[3] - F[1] * F[2] : det3(F);
    for (int i = 0; i < dim; ++i)
        for (int j = 0; j < dim; ++j) {
            double acc = 0.0;
            for (int k = 0; k < dim; ++k) acc += (F[i * dim + k] - R[i * dim + k]) * F[j * dim + k];
            tau[i * dim + j] = 2.0 * mu * acc + ((i == j) ? la * J * (J - 1.0) : 0.0);
        }
}

/* ---------------- grid helpers ---------------- */

static int64_t node_count(const orc_params *p)
{
    int64_t n = p->grid_res;
    return p->dim == 2 ? n * n : n * n * n;
}

static int64_t node_index(const orc_params *p, const int *ijk)
{
    int64_t n = p->grid_res;
    return p->dim == 2 ? (int64_t)ijk[1] * n + ijk[0] : ((int64_t)ijk[2] * n + ijk[1]) * n + ijk[0];
}

/* base cell, fractional offset and quadratic B-spline weights of one particle */
static void stencil(const orc_params *p, const double *xp, int *base, double *fx, double w[3][3])
{
    double inv_dx = (double)p->grid_res;
    for (int a = 0; a < p->dim; ++a) {
        double xs = xp[a] * inv_dx;
        double b = floor(xs - 0.5);
        if (!(b >= 0.0)) b = 0.0; /* also maps NaN to 0 */
        if (b > (double)(p->grid_res - 3)) b = (double)(p->grid_res - 3);
        base[a] = (int)b;
        fx[a] = xs - b;
        double f = fx[a];
        w[a][0] = 0.5 * (1.5 - f) * (1.5 - f);
        w[a][1] = 0.75 - (f - 1.0) * (f - 1.0);
        w[a][2] = 0.5 * (f - 0.5) * (f - 0.5);
    }
}

/* SoA state: comp c of particle q at [c*n+q]. grid_mom: comp a of node i at [a*nodes+i]. */
int orc_p2g(const orc_params *p, int64_t n, const double *x, const double *v,
            const double *C, const double *F, double *grid_m, double *grid_mom)
{
    int dim = p->dim;
    int64_t nodes = node_count(p);
    double inv_dx = (double)p->grid_res, dx = 1.0 / inv_dx;
    double mu = p->E / (2.0 * (1.0 + p->nu));
    double la = p->E * p->nu / ((1.0 + p->nu) * (1.0 - 2.0 * p->nu));
    double p_mass = p->rho * p->p_vol;
    int nst = dim == 2 ? 9 : 27;
    for (int64_t q = 0; q < n; ++q) {
        double xp[3], vp[3], Cp[9], Fp[9], tau[9], A[9];
        for (int a = 0; a < dim; ++a) { xp[a] = x[a * n + q]; vp[a] = v[a * n + q]; }
        for (int c = 0; c < dim * dim; ++c) Cp[c] = C[c * n + q];
        int base[3];
        double fx[3], w[3][3];
        stencil(p, xp, base, fx, w);
        if (p->material == ORC_FLUID) {
            orc_fluid_stress(dim, F[q], p->E, tau);
        } else {
            for (int c = 0; c < dim * dim; ++c) Fp[c] = F[c * n + q];
            orc_kirchhoff(dim, Fp, mu, la, tau);
        }
        for (int c = 0; c < dim * dim; ++c)
            A[c] = -p->dt * p->p_vol * 4.0 * inv_dx * inv_dx * tau[c] + p_mass * Cp[c];
        for (int s = 0; s < nst; ++s) {
            int o[3] = {s % 3, (s / 3) % 3, s / 9};
            int ijk[3];
            double dpos[3], weight = 1.0;
            for (int a = 0; a < dim; ++a) {
                ijk[a] = base[a] + o[a];
                dpos[a] = ((double)o[a] - fx[a]) * dx;
                weight *= w[a][o[a]];
            }
            int64_t id = node_index(p, ijk);
            for (int a = 0; a < dim; ++a) {
                double ad = 0.0;
                for (int b = 0; b < dim; ++b) ad += A[a * dim + b] * dpos[b];
                grid_mom[a * nodes + id] += weight * (p_mass * vp[a] + ad);
            }
            grid_m[id] += weight * p_mass;
        }
    }
    return 0;
}

/* Converts momentum to velocity in place (grid_mom then holds v). */
int orc_grid_update(const orc_params *p, double *grid_m, double *grid_mom)
{
    int dim = p->dim, n = p->grid_res;
    int64_t nodes = node_count(p);
    for (int64_t id = 0; id < nodes; ++id) {
        int ijk[3] = {(int)(id % n), (int)((id / n) % n), (int)(id / ((int64_t)n * n))};
        if (grid_m[id] > 0.0) {
            for (int a = 0; a < dim; ++a) {
                double va = grid_mom[a * nodes + id] / grid_m[id] + p->dt * p->gravity[a];
                if (ijk[a] < p->bound_cells && va < 0.0) va = 0.0;
                if (ijk[a] >= n - p->bound_cells && va > 0.0) va = 0.0;
                grid_mom[a * nodes + id] = va;
            }
        } else {
            for (int a = 0; a < dim; ++a) grid_mom[a * nodes + id] = 0.0;
        }
    }
    return 0;
}

int orc_g2p(const orc_params *p, int64_t n, const double *x, const double *F,
            const double *grid_v, double *x_new, double *v_new, double *C_new, double *F_new)
{
    int dim = p->dim;
    int64_t nodes = node_count(p);
    double inv_dx = (double)p->grid_res, dx = 1.0 / inv_dx;
    int nst = dim == 2 ? 9 : 27;
    for (int64_t q = 0; q < n; ++q) {
        double xp[3], nv[3] = {0, 0, 0}, nC[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int a = 0; a < dim; ++a) xp[a] = x[a * n + q];
        int base[3];
        double fx[3], w[3][3];
        stencil(p, xp, base, fx, w);
        for (int s = 0; s < nst; ++s) {
            int o[3] = {s % 3, (s / 3) % 3, s / 9};
            int ijk[3];
            double dpos[3], weight = 1.0;
            for (int a = 0; a < dim; ++a) {
                ijk[a] = base[a] + o[a];
                dpos[a] = ((double)o[a] - fx[a]) * dx;
                weight *= w[a][o[a]];
            }
            int64_t id = node_index(p, ijk);
            for (int a = 0; a < dim; ++a) {
                double gv = grid_v[a * nodes + id];
                nv[a] += weight * gv;
                for (int b = 0; b < dim; ++b) nC[a * dim + b] += 4.0 * inv_dx * inv_dx * weight * gv * dpos[b];
            }
        }
        for (int a = 0; a < dim; ++a) {
            if (v_new) v_new[a * n + q] = nv[a];
            if (x_new) x_new[a * n + q] = xp[a] + p->dt * nv[a];
        }
        for (int c = 0; c < dim * dim; ++c)
            if (C_new) C_new[c * n + q] = nC[c];
        if (F_new && p->material == ORC_FLUID) {
            /* volume ratio: J' = J (1 + dt tr C') */
            double tr = 0.0;
            for (int a = 0; a < dim; ++a) tr += nC[a * dim + a];
            F_new[q] = F[q] * (1.0 + p->dt * tr);
        } else if (F_new) {
            for (int i = 0; i < dim; ++i)
                for (int j = 0; j < dim; ++j) {
                    double acc = 0.0;
                    for (int k = 0; k < dim; ++k) {
                        double Mik = ((i == k) ? 1.0 : 0.0) + p->dt * nC[i * dim + k];
                        acc += Mik * F[(k * dim + j) * n + q];
                    }
                    F_new[(i * dim + j) * n + q] = acc;
                }
        }
    }
    return 0;
}

/* ---------------- particle sort ---------------- */

typedef struct { int64_t block, rank, cell, slot; } sort_key;

static int cmp_key(const void *a, const void *b)
{
    const sort_key *x = (const sort_key *)a, *y = (const sort_key *)b;
    if (x->block != y->block) return x->block < y->block ? -1 : 1;
    if (x->rank != y->rank) return x->rank < y->rank ? -1 : 1;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return (x->slot > y->slot) - (x->slot < y->slot);
}

/* order[i] = slot whose particle moves to slot i. */
int orc_sort_order(const orc_params *p, int64_t n, const double *x, int64_t *order)
{
    int dim = p->dim, gn = p->grid_res;
    int B = dim == 3 ? 8 : 16;
    int64_t nb = (gn + B - 1) / B;
    int64_t ncell = dim == 3 ? (int64_t)gn * gn * gn : (int64_t)gn * gn;
    int32_t *count = (int32_t *)calloc((size_t)ncell, sizeof(int32_t));
    sort_key *keys = (sort_key *)malloc(sizeof(sort_key) * (size_t)(n > 0 ? n : 1));
    if (!count || !keys) { free(count); free(keys); return -1; }
    for (int64_t q = 0; q < n; ++q) {
        double xp[3];
        for (int a = 0; a < dim; ++a) xp[a] = x[a * n + q];
        int base[3] = {0, 0, 0};
        double fx[3], w[3][3];
        stencil(p, xp, base, fx, w);
        int64_t cell_lin = node_index(p, base);
        int64_t blk = 0;
        for (int a = dim - 1; a >= 0; --a) blk = blk * nb + base[a] / B;
        /* cell within the block, in tiles of 64 cells (4x4x4 in 3D, 8x8 in
         * 2D) taken in x-fastest order, cells x-fastest inside a tile */
        int64_t cib;
        if (dim == 3) {
            int cx = base[0] % B, cy = base[1] % B, cz = base[2] % B;
            cib = (((cz / 4) * 2 + cy / 4) * 2 + cx / 4) * 64 + ((cz % 4) * 4 + cy % 4) * 4 + cx % 4;
        } else {
            int cx = base[0] % B, cy = base[1] % B;
            cib = ((cy / 8) * 2 + cx / 8) * 64 + (cy % 8) * 8 + cx % 8;
        }
        keys[q].block = blk;
        keys[q].rank = count[cell_lin]++;
        keys[q].cell = cib;
        keys[q].slot = q;
    }
    qsort(keys, (size_t)n, sizeof(sort_key), cmp_key);
    for (int64_t i = 0; i < n; ++i) order[i] = keys[i].slot;
    free(count);
    free(keys);
    return 0;
}

/* ---------------- simulation driver ---------------- */

struct orc_sim {
    orc_scheme s;
    orc_params p;
    int64_t n;
    int32_t W;
    uint32_t *words;
    int64_t *ids;
    int64_t step;
    int sorted;
    int64_t sorted_at;
    orc_stat stats[4];
};

orc_sim *orc_sim_new(const orc_scheme *s, const orc_params *p, int64_t n, const uint32_t *words)
{
    int32_t W;
    if (orc_layout(s, 0, 0, 0, &W)) return 0;
    if (p->dim != s->dim || p->grid_res < 4) return 0;
    int has_j = 0;
    for (int i = 0; i < 4; ++i) has_j |= s->f[i].field == ORC_J;
    if (has_j != (p->material == ORC_FLUID)) return 0;
    orc_sim *sim = (orc_sim *)calloc(1, sizeof(orc_sim));
    sim->s = *s;
    sim->p = *p;
    sim->n = n;
    sim->W = W;
    sim->words = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(W * (n > 0 ? n : 1)));
    sim->ids = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    memcpy(sim->words, words, sizeof(uint32_t) * (size_t)(W * n));
    for (int64_t q = 0; q < n; ++q) sim->ids[q] = q;
    sim->step = 0;
    sim->sorted = 0;
    sim->sorted_at = -1;
    return sim;
}

static void sim_sort(orc_sim *sim, const double *x)
{
    int64_t n = sim->n;
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    orc_sort_order(&sim->p, n, x, order);
    uint32_t *nw = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(sim->W * (n > 0 ? n : 1)));
    int64_t *nid = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        for (int w = 0; w < sim->W; ++w) nw[(int64_t)w * n + i] = sim->words[(int64_t)w * n + order[i]];
        nid[i] = sim->ids[order[i]];
    }
    free(sim->words);
    free(sim->ids);
    sim->words = nw;
    sim->ids = nid;
    free(order);
}

int orc_sim_step(orc_sim *sim, int32_t nsteps)
{
    const orc_params *p = &sim->p;
    int dim = p->dim;
    int64_t n = sim->n, nodes = node_count(p);
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *x = malloc(sizeof(double) * nn * 3), *v = malloc(sizeof(double) * nn * 3);
    double *C = malloc(sizeof(double) * nn * 9), *F = malloc(sizeof(double) * nn * 9);
    double *x1 = malloc(sizeof(double) * nn * 3), *v1 = malloc(sizeof(double) * nn * 3);
    double *C1 = malloc(sizeof(double) * nn * 9), *F1 = malloc(sizeof(double) * nn * 9);
    double *gm = malloc(sizeof(double) * (size_t)nodes);
    double *gmom = malloc(sizeof(double) * (size_t)nodes * (size_t)dim);
    if (!x || !v || !C || !F || !x1 || !v1 || !C1 || !F1 || !gm || !gmom) return -1;
    for (int32_t it = 0; it < nsteps; ++it) {
        uint32_t s = (uint32_t)sim->step;
        orc_decode(&sim->s, n, sim->words, x, v, C, F);
        int S = p->sort_every;
        if (!sim->sorted || (S > 0 && (sim->step % S) == 0 && sim->sorted_at != sim->step)) {
            sim_sort(sim, x);
            sim->sorted = 1;
            sim->sorted_at = sim->step;
            orc_decode(&sim->s, n, sim->words, x, v, C, F);
        }
        memset(gm, 0, sizeof(double) * (size_t)nodes);
        memset(gmom, 0, sizeof(double) * (size_t)nodes * (size_t)dim);
        orc_p2g(p, n, x, v, C, F, gm, gmom);
        orc_grid_update(p, gm, gmom);
        orc_g2p(p, n, x, F, gmom, x1, v1, C1, F1);
        orc_encode_f64(&sim->s, n, x1, v1, C1, F1, s, 1u, sim->words, sim->stats);
        sim->step += 1;
    }
    free(x); free(v); free(C); free(F); free(x1); free(v1); free(C1); free(F1);
    free(gm); free(gmom);
    return 0;
}

void orc_sim_words(const orc_sim *sim, uint32_t *out)
{
    memcpy(out, sim->words, sizeof(uint32_t) * (size_t)(sim->W * sim->n));
}

void orc_sim_ids(const orc_sim *sim, int64_t *out)
{
    memcpy(out, sim->ids, sizeof(int64_t) * (size_t)sim->n);
}

void orc_sim_stats(const orc_sim *sim, orc_stat *out) { memcpy(out, sim->stats, sizeof(sim->stats)); }

int64_t orc_sim_step_count(const orc_sim *sim) { return sim->step; }

void orc_sim_free(orc_sim *sim)
{
    if (!sim) return;
    free(sim->words);
    free(sim->ids);
    free(sim);
}
