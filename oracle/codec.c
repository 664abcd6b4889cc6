/*
 * codec.c -- oracle bit-pack layout, fixed-point / shared-exponent /
 * raw-float32 codecs and the Philox4x32-10 counter generator.
 *
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Readings taken where the paper is silent (each one is also listed in the
 * design notes of the repository):
 *  - Record layout (Sec. 7, Figs. 7-8, "bit pack"): the components of the
 *    fields are concatenated in placement order, matrices row-major, a
 *    shared-exponent field stores its exponent first.  Component bit k sits
 *    at record bit o+k, LSB first; record bit g lives in word g/32, bit
 *    g%32.  Components may span two 32-bit words.  Storage is word-major:
 *    word k of particle p is words[k*n + p].
 *  - Fixed point (Eq. 3): Delta = (hi-lo) * 2^-b, u = round((v-lo)/Delta)
 *    over an affine range.  In binary64: t = (v - lo) * inv with
 *    inv = 2^b/(hi-lo) (two separate roundings), u = floor(t + 0.5)
 *    (ties round up); decoding is fma(u, Delta, lo).  Out-of-range codes
 *    saturate to [0, 2^b-1] and are counted.
 *  - Dither (Eq. 11): round(t + xi), xi ~ U(-1/2, 1/2), is floor(t + xi')
 *    with xi' ~ U(0,1); xi' = (r + 1/2) * 2^-16 for a 16-bit Philox draw r.
 *  - Philox counter = (slot, step, group, tag), key = seed.  Components are
 *    numbered in the canonical order x, v, C, F (matrices row-major,
 *    independent of the placement order): component k takes 16-bit half k%2
 *    of output word (k%8)/2 of group k/8.  A shared-exponent field draws for
 *    its magnitudes only.
 *  - Shared exponent (the custom float type mentioned with the hand-written
 *    scheme comparison, Sec. 8.1): E_max = ceil(log2 hi),
 *    E_min = E_max - 2^e + 1, E = clamp(ilogb(max|v_k|) + 1, E_min, E_max)
 *    (E_min for an all-zero vector), q_k = round(|v_k| * 2^(m-1-E)); if a
 *    q_k reaches 2^(m-1) the exponent is raised by one and the vector is
 *    rounded again.  Stored as E - E_min, then per component the magnitude
 *    in the low m-1 bits and the sign on top.
 */
#include "orc.h"
#include <math.h>
#include <string.h>

static int ncomp_of(int field, int dim)
{
    return (field == ORC_X || field == ORC_V) ? dim : field == ORC_J ? 1 : dim * dim;
}
/* state slot of a field: F and J share slot 3 */
static int slot_of(int field) { return field == ORC_J ? 3 : field; }
/* components of the scheme's slot-3 field */
static int nc3_of(const orc_scheme *s)
{
    for (int i = 0; i < 4; ++i)
        if (slot_of(s->f[i].field) == 3) return ncomp_of(s->f[i].field, s->dim);
    return s->dim * s->dim;
}

int orc_validate(const orc_scheme *s)
{
    if (s->dim != 2 && s->dim != 3) return -1;
    if (s->n_fields != 4) return -1;
    int seen[4] = {0, 0, 0, 0};
    int total = 0;
    for (int i = 0; i < 4; ++i) {
        const orc_field *f = &s->f[i];
        if (f->field < 0 || f->field > 4 || seen[slot_of(f->field)]) return -1;
        seen[slot_of(f->field)] = 1;
        int nc = ncomp_of(f->field, s->dim);
        if (f->rel_identity && f->field != ORC_F && f->field != ORC_J) return -1;
        if (f->kind == ORC_FIXED) {
            if (f->bits < 1 || f->bits > 32) return -1;
            if (!(f->hi > f->lo) || !isfinite(f->lo) || !isfinite(f->hi)) return -1;
            total += nc * f->bits;
        } else if (f->kind == ORC_SHARED_EXP) {
            if (f->bits < 2 || f->bits > 32) return -1;
            if (f->exp_bits < 1 || f->exp_bits > 8) return -1;
            if (!(f->hi > 0) || !isfinite(f->hi) || f->rel_identity) return -1;
            total += f->exp_bits + nc * f->bits;
        } else if (f->kind == ORC_RAW_F32) {
            if (f->bits != 32) return -1;
            total += nc * 32;
        } else {
            return -1;
        }
    }
    if (total > 32 * 32) return -1;
    return 0;
}

/* Bit offsets of every component (indexed field*9 + component) and of
 * every field's first bit (for SHARED_EXP: the exponent). */
int orc_layout(const orc_scheme *s, int32_t *comp_offset, int32_t *field_offset,
               int32_t *total_bits, int32_t *W)
{
    if (orc_validate(s)) return -1;
    int off = 0;
    for (int i = 0; i < 4; ++i) {
        const orc_field *f = &s->f[i];
        int nc = ncomp_of(f->field, s->dim);
        if (field_offset) field_offset[slot_of(f->field)] = off;
        if (f->kind == ORC_SHARED_EXP) off += f->exp_bits;
        for (int c = 0; c < nc; ++c) {
            if (comp_offset) comp_offset[slot_of(f->field) * 9 + c] = off;
            off += f->bits;
        }
    }
    if (total_bits) *total_bits = off;
    if (W) *W = (off + 31) / 32;
    return 0;
}

/* ---- Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) ---- */
static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    /* Multipliers and Weyl key increments as published with the method. */
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, c0, &hi0, &lo0);
        mulhilo32(M1, c2, &hi1, &lo1);
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 16-bit dither draws of one record: draws[k] for record component k. */
static void dither_draws(uint64_t seed, uint32_t slot, uint32_t step, uint32_t tag, int ncomp, double *draws)
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int j = 0; j * 8 < ncomp; ++j) {
        uint32_t ctr[4] = {slot, step, (uint32_t)j, tag};
        uint32_t out[4];
        orc_philox4x32_10(ctr, key, out);
        for (int i = 0; i < 8 && 8 * j + i < ncomp; ++i) {
            uint32_t word = out[i / 2];
            uint32_t r = (i % 2) ? (word >> 16) : (word & 0xFFFFu);
            draws[8 * j + i] = ((double)r + 0.5) / 65536.0;
        }
    }
}

/* ---- field codecs ---- */

/* smallest integer e with hi <= 2^e (hi > 0) */
static int ceil_log2(double hi)
{
    int ex;
    double m = frexp(hi, &ex); /* hi = m * 2^ex, m in [0.5, 1) */
    return (m == 0.5) ? ex - 1 : ex;
}

static void count_round(orc_stat *st, double t, uint32_t code)
{
    if (!st) return;
    if ((double)code > floor(t)) st->up++; else st->down++;
}

/* Fixed point, Eq. 3 (+ Eq. 11 when xi >= 0).  `val` is the quantity to
 * store (already relative to I for a REL_IDENTITY field). */
static uint32_t fixed_encode(const orc_field *f, double val, double xi, orc_stat *st)
{
    double range = f->hi - f->lo;
    double inv = ldexp(1.0, f->bits) / range;
    double maxc = ldexp(1.0, f->bits) - 1.0;
    double t = (val - f->lo) * inv;
    double s = t + (xi >= 0.0 ? xi : 0.5);
    if (isnan(s)) { if (st) st->nan++; return 0u; }
    double fl = floor(s);
    if (fl < 0.0) { if (st) st->sat++; return 0u; }
    if (fl > maxc) { if (st) st->sat++; return (uint32_t)maxc; }
    uint32_t code = (uint32_t)fl;
    count_round(st, t, code);
    return code;
}

static double fixed_decode(const orc_field *f, uint32_t code)
{
    double delta = ldexp(f->hi - f->lo, -f->bits);
    return fma((double)code, delta, f->lo);
}

static uint32_t f32_bits(float v) { uint32_t u; memcpy(&u, &v, 4); return u; }
static float bits_f32(uint32_t u) { float v; memcpy(&v, &u, 4); return v; }

/* Shared exponent: codes[0] = exponent code, codes[1..nc] = sign|magnitude. */
static void sexp_encode(const orc_field *f, int nc, const double *val, const double *xi,
                        uint32_t *codes, orc_stat *st)
{
    int m = f->bits, e = f->exp_bits;
    int Emax = ceil_log2(f->hi);
    int Emin = Emax - ((1 << e) - 1);
    double qmax = ldexp(1.0, m - 1) - 1.0;
    double a[9];
    double M = 0.0;
    for (int k = 0; k < nc; ++k) {
        double x = val[k];
        if (isnan(x)) { if (st) st->nan++; x = 0.0; }
        a[k] = fabs(x);
        if (a[k] > M) M = a[k];
    }
    int E;
    if (M == 0.0) E = Emin;
    else if (isinf(M)) E = Emax;
    else {
        E = ilogb(M) + 1;
        if (E < Emin) E = Emin;
        if (E > Emax) E = Emax;
    }
    double q[9], t[9];
    for (;;) {
        int overflow = 0;
        for (int k = 0; k < nc; ++k) {
            t[k] = ldexp(a[k], (m - 1) - E);
            q[k] = floor(t[k] + (xi ? xi[k] : 0.5));
            if (q[k] > qmax) overflow = 1;
        }
        if (overflow && E < Emax) { E += 1; continue; }
        break;
    }
    codes[0] = (uint32_t)(E - Emin);
    for (int k = 0; k < nc; ++k) {
        uint32_t qk;
        if (q[k] > qmax) { if (st) st->sat++; qk = (uint32_t)qmax; }
        else { qk = (uint32_t)q[k]; count_round(st, t[k], qk); }
        uint32_t sign = (val[k] < 0.0 && qk > 0) ? 1u : 0u;
        codes[1 + k] = qk | (sign << (m - 1));
    }
}

static void sexp_decode(const orc_field *f, int nc, const uint32_t *codes, double *out)
{
    int m = f->bits, e = f->exp_bits;
    int Emax = ceil_log2(f->hi);
    int Emin = Emax - ((1 << e) - 1);
    int E = (int)codes[0] + Emin;
    uint32_t magmask = (m - 1 == 32) ? 0xFFFFFFFFu : ((1u << (m - 1)) - 1u);
    for (int k = 0; k < nc; ++k) {
        uint32_t qk = codes[1 + k] & magmask;
        double mag = ldexp((double)qk, E - (m - 1));
        out[k] = ((codes[1 + k] >> (m - 1)) & 1u) ? -mag : mag;
    }
}

/* ---- bit packing (Sec. 7) ---- */
static void put_bits(uint32_t *rec, int off, int nbits, uint32_t code)
{
    /* record bits [off, off+nbits) <- code, LSB first; may touch two words */
    uint64_t mask = (nbits == 32) ? 0xFFFFFFFFull : ((1ull << nbits) - 1ull);
    uint64_t v = ((uint64_t)code & mask) << (off & 31);
    rec[off >> 5] |= (uint32_t)v;
    if ((off & 31) + nbits > 32) rec[(off >> 5) + 1] |= (uint32_t)(v >> 32);
}

static uint32_t get_bits(const uint32_t *rec, int off, int nbits)
{
    uint64_t lo = rec[off >> 5];
    uint64_t hi = ((off & 31) + nbits > 32) ? rec[(off >> 5) + 1] : 0u;
    uint64_t both = lo | (hi << 32);
    uint64_t mask = (nbits == 32) ? 0xFFFFFFFFull : ((1ull << nbits) - 1ull);
    return (uint32_t)((both >> (off & 31)) & mask);
}

/* Encode one particle.  vals[field][comp] are the attribute values (F is the
 * full deformation gradient; the codec subtracts I for REL_IDENTITY). */
static void encode_record(const orc_scheme *s, const double vals[4][9], uint32_t slot,
                          uint32_t step, uint32_t tag, uint32_t *rec, int W, orc_stat *stats)
{
    int dim = s->dim;
    memset(rec, 0, sizeof(uint32_t) * (size_t)W);
    int off = 0;
    double draws[32];
    dither_draws(s->seed, slot, step, tag, 2 * dim + dim * dim + nc3_of(s), draws);
    for (int i = 0; i < 4; ++i) {
        const orc_field *f = &s->f[i];
        int nc = ncomp_of(f->field, dim);
        int sl = slot_of(f->field);
        orc_stat *st = stats ? &stats[sl] : 0;
        /* canonical index of the field's first component: x, v, C, then F or J */
        int k = sl == ORC_X ? 0 : sl == ORC_V ? dim : sl == ORC_C ? 2 * dim : 2 * dim + dim * dim;
        double rel[9];
        for (int c = 0; c < nc; ++c) {
            double val = vals[sl][c];
            if (f->rel_identity && (c % (dim + 1) == 0)) val = val - 1.0;
            rel[c] = val;
        }
        if (f->kind == ORC_SHARED_EXP) {
            double xi[9];
            for (int c = 0; c < nc; ++c) xi[c] = draws[k + c];
            uint32_t codes[10];
            sexp_encode(f, nc, rel, f->dither ? xi : 0, codes, st);
            put_bits(rec, off, f->exp_bits, codes[0]);
            off += f->exp_bits;
            for (int c = 0; c < nc; ++c) { put_bits(rec, off, f->bits, codes[1 + c]); off += f->bits; }
        } else {
            for (int c = 0; c < nc; ++c) {
                uint32_t code;
                if (f->kind == ORC_RAW_F32) {
                    code = f32_bits((float)rel[c]);
                } else {
                    double xi = f->dither ? draws[k + c] : -1.0;
                    code = fixed_encode(f, rel[c], xi, st);
                }
                put_bits(rec, off, f->bits, code);
                off += f->bits;
            }
        }
    }
}

static void decode_record(const orc_scheme *s, const uint32_t *rec, double vals[4][9])
{
    int dim = s->dim;
    int off = 0;
    for (int i = 0; i < 4; ++i) {
        const orc_field *f = &s->f[i];
        int nc = ncomp_of(f->field, dim);
        double *out = vals[slot_of(f->field)];
        if (f->kind == ORC_SHARED_EXP) {
            uint32_t codes[10];
            codes[0] = get_bits(rec, off, f->exp_bits);
            off += f->exp_bits;
            for (int c = 0; c < nc; ++c) { codes[1 + c] = get_bits(rec, off, f->bits); off += f->bits; }
            sexp_decode(f, nc, codes, out);
        } else {
            for (int c = 0; c < nc; ++c) {
                uint32_t code = get_bits(rec, off, f->bits);
                off += f->bits;
                out[c] = (f->kind == ORC_RAW_F32) ? (double)bits_f32(code) : fixed_decode(f, code);
            }
        }
        if (f->rel_identity)
            for (int c = 0; c < nc; c += dim + 1) out[c] = out[c] + 1.0;
    }
}

/* ---- array entry points (component-major SoA: comp c of particle p at [c*n+p]) ---- */

static int encode_common(const orc_scheme *s, int64_t n, const float *xf, const float *vf,
                         const float *Cf, const float *Ff, const double *xd, const double *vd,
                         const double *Cd, const double *Fd, uint32_t step, uint32_t tag,
                         uint32_t *words, orc_stat *stats)
{
    int32_t W;
    if (orc_layout(s, 0, 0, 0, &W)) return -1;
    int dim = s->dim, nc3 = nc3_of(s);
    uint32_t rec[32];
    for (int64_t p = 0; p < n; ++p) {
        double vals[4][9];
        for (int c = 0; c < dim; ++c) {
            vals[ORC_X][c] = xf ? (double)xf[c * n + p] : xd[c * n + p];
            vals[ORC_V][c] = vf ? (double)vf[c * n + p] : vd[c * n + p];
        }
        for (int c = 0; c < dim * dim; ++c) vals[ORC_C][c] = Cf ? (double)Cf[c * n + p] : Cd[c * n + p];
        for (int c = 0; c < nc3; ++c) vals[ORC_F][c] = Ff ? (double)Ff[c * n + p] : Fd[c * n + p];
        encode_record(s, (const double(*)[9])vals, (uint32_t)p, step, tag, rec, W, stats);
        for (int w = 0; w < W; ++w) words[(int64_t)w * n + p] = rec[w];
    }
    return 0;
}

int orc_encode(const orc_scheme *s, int64_t n, const float *x, const float *v,
               const float *C, const float *F, uint32_t step, uint32_t tag,
               uint32_t *words, orc_stat *stats)
{
    return encode_common(s, n, x, v, C, F, 0, 0, 0, 0, step, tag, words, stats);
}

int orc_encode_f64(const orc_scheme *s, int64_t n, const double *x, const double *v,
                   const double *C, const double *F, uint32_t step, uint32_t tag,
                   uint32_t *words, orc_stat *stats)
{
    return encode_common(s, n, 0, 0, 0, 0, x, v, C, F, step, tag, words, stats);
}

int orc_decode(const orc_scheme *s, int64_t n, const uint32_t *words,
               double *x, double *v, double *C, double *F)
{
    int32_t W;
    if (orc_layout(s, 0, 0, 0, &W)) return -1;
    int dim = s->dim, nc3 = nc3_of(s);
    uint32_t rec[32];
    for (int64_t p = 0; p < n; ++p) {
        for (int w = 0; w < W; ++w) rec[w] = words[(int64_t)w * n + p];
        double vals[4][9];
        decode_record(s, rec, vals);
        for (int c = 0; c < dim; ++c) {
            if (x) x[c * n + p] = vals[ORC_X][c];
            if (v) v[c * n + p] = vals[ORC_V][c];
        }
        for (int c = 0; c < dim * dim; ++c)
            if (C) C[c * n + p] = vals[ORC_C][c];
        for (int c = 0; c < nc3; ++c)
            if (F) F[c * n + p] = vals[ORC_F][c];
    }
    return 0;
}
