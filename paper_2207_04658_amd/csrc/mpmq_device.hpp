// mpmq_device.hpp -- gfx950 device functions of the quantized MLS-MPM
// substep: bit-pack extraction/insertion, the three storage kinds, the
// Philox dither draws and the MLS-MPM stencil helpers.
#pragma once
#include "mpmq_internal.hpp"

namespace mpmq {

template <int N> using uvec = uint32_t __attribute__((ext_vector_type(N)));

enum { K_FIXED = 0, K_SEXP = 1, K_RAW = 2 };

// Makes a value opaque to the optimizer at this point, so that quantities
// derived from it are recomputed here instead of being hoisted out of the
// particle loop and kept live (the scheme constants and per-component row
// addresses would otherwise exhaust the scalar registers).
template <typename P> __device__ __forceinline__ P opaque(P v) {
    asm volatile("" : "+s"(v));
    return v;
}

// The scheme lives in device memory that no kernel writes; reading it
// through the constant address space keeps every field in scalar registers.
// A specialized build defines MPMQ_SCHEME_CONST (a DevScheme initializer):
// the kernels then read that compile-time constant instead, so kinds, bit
// offsets and codec constants fold into the code.  The Philox key is always
// read from the run-time copy (seed_ref), so one specialized build serves
// every seed.
typedef const __attribute__((address_space(4))) DevScheme *SchemeRef;
typedef const __attribute__((address_space(4))) DevField *FieldRef;
__device__ __forceinline__ SchemeRef seed_ref(const DevScheme *p) { return (SchemeRef)opaque(p); }
// The same holds for the simulation parameters (MPMQ_PARAMS_CONST, a
// DevParams initializer): a context's parameters never change.
// Float32 decode: with the scheme fixed at compile time, a field whose
// decoded values are all exact in float32 (DevField::f32dec) is decoded in
// float32 arithmetic, which then gives the same values as the binary64
// formula rounded once.
#ifdef MPMQ_SCHEME_CONST
constexpr bool kF32Decode = true;
#else
constexpr bool kF32Decode = false;
#endif
template <typename T> struct is_f32 { static constexpr bool value = false; };
template <> struct is_f32<float> { static constexpr bool value = true; };

// ... and for the row stride of the packed words (MPMQ_CAP_CONST): with a
// constant stride the row addresses need no registers.
#ifdef MPMQ_CAP_CONST
__device__ __forceinline__ int64_t cap_ref(int64_t) { return (int64_t)(MPMQ_CAP_CONST); }
#else
__device__ __forceinline__ int64_t cap_ref(int64_t c) { return c; }
#endif
#ifdef MPMQ_PARAMS_CONST
static constexpr DevParams kParamsConst = MPMQ_PARAMS_CONST;
__device__ __forceinline__ const DevParams &params_ref(const DevParams &) { return kParamsConst; }
#else
__device__ __forceinline__ const DevParams &params_ref(const DevParams &p) { return p; }
#endif
#ifdef MPMQ_SCHEME_CONST
static constexpr DevScheme kSchemeConst = MPMQ_SCHEME_CONST;
__device__ __forceinline__ SchemeRef scheme_ref(const DevScheme *) { return (SchemeRef)&kSchemeConst; }
#else
__device__ __forceinline__ SchemeRef scheme_ref(const DevScheme *p) { return (SchemeRef)opaque(p); }
#endif


// ---------------------------------------------------------------------------
// Field ids FID: 0 x, 1 v, 2 C, 3 F, 4 J.  F and J share state slot 3 (the
// scheme's f[3]).  Canonical component numbering x, v, C, then F or J
// (matrices row-major); it fixes the Philox draw of every component
// independently of the placement order.
// ---------------------------------------------------------------------------
template <int DIM, int FID> constexpr int ncomp() { return FID < 2 ? DIM : FID == 4 ? 1 : DIM * DIM; }
template <int FID> constexpr int slot_of() { return FID == 4 ? 3 : FID; }
template <int DIM, int FID> constexpr int canon0() {
    return FID == 0 ? 0 : FID == 1 ? DIM : FID == 2 ? 2 * DIM : 2 * DIM + DIM * DIM;
}
// material: 0 elastic (slot 3 holds F), 1 fluid (slot 3 holds J)
template <int MAT> constexpr int fid3() { return MAT ? 4 : 3; }
template <int DIM, int MAT> constexpr int nc3() { return MAT ? 1 : DIM * DIM; }

// ---------------------------------------------------------------------------
// Bit pack (Sec. 7, Figs. 7-8), word-major: word k of slot p is
// words[k * cap + p].  A component at record bit o is read from word o/32
// (and o/32 + 1 when it spans two words) at a wave-uniform row offset and a
// per-lane byte offset p4 = 4p, then rebuilt with one funnel shift:
// alignbit concatenates (hi:lo) and shifts right, the mask keeps `bits` bits.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t ld_row(const uint32_t *words, int64_t cap, int k, uint32_t p4) {
    const char *row = reinterpret_cast<const char *>(words + (int64_t)k * cap);
    return *reinterpret_cast<const uint32_t *>(row + p4);
}

// Where a decode reads the record from: the rows in global memory, or
// registers holding rows loaded ahead of time (r[k] = row k; a specialized
// build indexes it with compile-time constants only, so it stays in
// registers).
struct GlobalRows {
    const uint32_t *words;
    int64_t cap;
    uint32_t p4;
    __device__ __forceinline__ uint32_t row(int k) const { return ld_row(words, cap, k, p4); }
};
struct RegRows {
    const uint32_t *r;
    __device__ __forceinline__ uint32_t row(int k) const { return r[k]; }
};

template <typename Src>
__device__ __forceinline__ uint32_t get_comp(const Src &src, int o, int bits, uint32_t mask) {
    const int k = o >> 5, sh = o & 31;
    const uint32_t lo = src.row(k);
    uint32_t hi = 0u;
    if (sh + bits > 32) hi = src.row(k + 1);
    return __builtin_amdgcn_alignbit(hi, lo, (uint32_t)sh) & mask;
}
__device__ __forceinline__ uint32_t get_comp(const uint32_t *words, int64_t cap, uint32_t p4, int o, int bits,
                                             uint32_t mask) {
    return get_comp(GlobalRows{words, cap, p4}, o, bits, mask);
}

// Encoder output: codes arrive in placement order and are appended to a
// 64-bit accumulator; each completed word is stored at once (the fill level
// is wave-uniform, so the test is a scalar branch and no record is ever
// indexed in registers).
struct OutStream {
    uint32_t *words;
    int64_t cap;
    uint32_t p4;
    uint64_t acc;
    int nb, k;
    __device__ __forceinline__ void emit(uint32_t code, int bits) {
        // every code fits its width; with constant widths and positions this
        // lets the compiler keep the packing in 32-bit operations
        __builtin_assume((uint64_t)code < (1ull << bits));
        acc |= (uint64_t)code << nb;
        nb += bits;
        if (nb >= 32) {
            char *row = reinterpret_cast<char *>(words + (int64_t)k * cap);
            __builtin_nontemporal_store((uint32_t)acc, reinterpret_cast<uint32_t *>(row + p4));
            acc >>= 32;
            nb -= 32;
            ++k;
        }
    }
    __device__ __forceinline__ void finish() {
        if (nb > 0) {
            char *row = reinterpret_cast<char *>(words + (int64_t)k * cap);
            __builtin_nontemporal_store((uint32_t)acc, reinterpret_cast<uint32_t *>(row + p4));
        }
    }
};

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, key bumped by the
// Weyl constants between rounds.  Counter (slot, step, group, tag), key =
// seed.  Canonical component k takes 16 bits: half k%2 of word k/2 of the
// concatenated group outputs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t *out) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        // three-input XOR in one instruction (gfx950 v_bitop3_b32, table 0x96)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32((uint32_t)(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32((uint32_t)(p0 >> 32), c3, k1, 0x96);
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

// Dither draws, generated on demand one Philox group (8 components) at a
// time.  A field's components are consecutive canonical indices, so they
// span at most two groups: two cached groups (by group parity) serve every
// field without regenerating.  The group tags are wave-uniform.
struct Draws {
    uint32_t r[2][4];
    int tag[2];
    uint32_t slot, step, ptag, seed_lo, seed_hi;
    // s: the run-time scheme copy (seed_ref), which holds the key
    __device__ __forceinline__ void init(SchemeRef s, uint32_t slot_, uint32_t step_, uint32_t tag_) {
        tag[0] = tag[1] = -1;
        slot = slot_;
        step = step_;
        ptag = tag_;
        seed_lo = s->seed_lo;
        seed_hi = s->seed_hi;
    }
    // 16-bit draw of canonical component k (k is a compile-time index)
    __device__ __forceinline__ uint32_t draw16(int k) {
        const int g = k >> 3, b = g & 1;
        if (tag[b] != g) {
            philox10(slot, step, (uint32_t)g, ptag, seed_lo, seed_hi, r[b]);
            tag[b] = g;
        }
        const uint32_t w = r[b][(k >> 1) & 3];
        return (k & 1) ? (w >> 16) : (w & 0xffffu);
    }
};

// The dither offset xi' = h 2^-16 in (0,1) is kept as h = r16 + 1/2 (exact
// in binary64); the encoders add it as fma(h, 2^-16, t), which equals
// RN(t + xi') because h 2^-16 is exact.  Without dithering h = 2^15
// (xi' = 1/2, round to nearest).
constexpr double XI_SCALE = 1.0 / 65536.0, XI_HALF = 32768.0;
__device__ __forceinline__ double dither_h(Draws &d, int k) { return (double)d.draw16(k) + 0.5; }

// ---------------------------------------------------------------------------
// Encoder statistics kept per lane and flushed per work item:
// ud[f] = round-ups | round-downs << 16 (counted only when the RS template
// flag is set), sat / nan: 8 bits per field.
// ---------------------------------------------------------------------------
struct LaneStats {
    uint32_t ud[4];
    uint32_t sat, nan;
    __device__ void clear() { ud[0] = ud[1] = ud[2] = ud[3] = 0; sat = nan = 0; }
};

// Fixed point (Eq. 3, Eq. 11 when xi' = h 2^-16): binary64, no contraction,
// so the rounding sequence is exactly t = RN(RN(val - lo) * inv),
// s = RN(t + xi'), u = clamp(floor(s)).
template <bool RS>
__device__ __forceinline__ uint32_t enc_fixed(const FieldRef f, double val, double h, int fid,
                                              LaneStats &ls) {
#pragma clang fp contract(off)
    const double t = (val - f->lo) * f->inv;
    const double sv = fma(h, XI_SCALE, t);
    const double fl = floor(sv);
    if (RS) {
        // clamp to [0, maxc] (fmax takes a NaN to 0); a value the clamp
        // changed saturated.  Selects rather than branches: the counters are
        // per-lane.
        const bool nan = !(sv == sv), below = fl < 0.0, above = fl > f->maxc;
        const uint32_t code = (uint32_t)fmin(fmax(fl, 0.0), f->maxc);
        ls.nan += nan ? 1u << (8 * fid) : 0u;
        ls.sat += (below || above) ? 1u << (8 * fid) : 0u;
        ls.ud[fid] += (nan || below || above) ? 0u : (fl > floor(t)) ? 1u : 0x10000u;
        return code;
    }
    // fl in [0, maxc] holds for every lane unless the wave takes the branch:
    // as bit patterns, the non-negative doubles up to maxc are exactly those
    // not above maxc's (a negative value, -0, NaN or inf compares above), so
    // one unsigned compare decides, and the exact clamp and the counters run
    // only in a wave that holds an out-of-range value.
    uint32_t code = (uint32_t)fl;
    const uint64_t out = __ballot((uint64_t)__double_as_longlong(fl) >
                                  (uint64_t)__double_as_longlong(f->maxc));
    if (__builtin_expect(out != 0ull, 0)) {
        const bool nan = !(sv == sv), below = fl < 0.0, above = fl > f->maxc;
        code = (uint32_t)fmin(fmax(fl, 0.0), f->maxc);  // fmax takes a NaN to 0
        ls.nan += nan ? 1u << (8 * fid) : 0u;
        ls.sat += (below || above) ? 1u << (8 * fid) : 0u;
    }
    return code;
}

// Shared-exponent vector: E from the largest magnitude, raised by one if a
// magnitude rounds up to 2^(m-1); stored as E - E_min, then sign|magnitude.
template <int DIM, int FID, typename T, bool RS>
__device__ __forceinline__ void enc_sexp(const FieldRef f, const T *val, Draws &rnd, OutStream &os,
                                         LaneStats &ls, T *qv) {
#pragma clang fp contract(off)
    constexpr int NC = ncomp<DIM, FID>(), K0 = canon0<DIM, FID>();
    const int m1 = f->bits - 1;
    const double qmax = (double)f->mag_mask;
    double M = 0.0;
    uint64_t nan_lanes = 0ull;  // lanes of the wave with a NaN component
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double x = (double)val[c];
        if (RS) ls.nan += (x == x) ? 0u : 1u << (8 * slot_of<FID>());
        else nan_lanes |= __ballot(!(val[c] == val[c]));
        M = fmax(M, fabs(x));  // fmax ignores a NaN operand
    }
    int E;
    if (M == 0.0) E = f->emin;
    else if (isinf(M)) E = f->emax;
    else E = min(max(ilogb(M) + 1, f->emin), f->emax);
    // raise E while a magnitude rounds up to 2^(m-1) (at most once in exact
    // arithmetic; the loop keeps the definition literal); the rounded
    // magnitudes of the last pass are the codes
    double tq[NC], qq[NC];
    double qtop_end;
    for (;;) {
        double qtop = 0.0;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            double x = (double)val[c];
            x = fmax(fabs(x), 0.0);  // NaN -> 0
            const double h = f->dither ? dither_h(rnd, K0 + c) : XI_HALF;
            tq[c] = ldexp(x, m1 - E);
            qq[c] = floor(fma(h, XI_SCALE, tq[c]));
            qtop = fmax(qtop, qq[c]);
        }
        qtop_end = qtop;
        if (!(qtop > qmax && E < f->emax)) break;
        E += 1;
    }
    os.emit((uint32_t)(E - f->emin), f->exp_bits);
    // A magnitude can exceed qmax only where the loop above stopped at E_max
    // with qtop > qmax: without such a lane (and without a NaN) in the wave
    // the codes need neither the clamp nor the counters.
    bool slow = true;
    if (!RS) {
        slow = __ballot(qtop_end > qmax) != 0ull || nan_lanes != 0ull;
        if (__builtin_expect(slow, 0)) {
#pragma unroll
            for (int c = 0; c < NC; ++c)
                ls.nan += (val[c] == val[c]) ? 0u : 1u << (8 * slot_of<FID>());
        }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        const double t = tq[c];
        const double q = qq[c];
        uint32_t qc;
        if (RS || __builtin_expect(slow, 0)) {
            const bool above = q > qmax;
            qc = (uint32_t)fmin(q, qmax);  // q >= 0
            ls.sat += above ? 1u << (8 * slot_of<FID>()) : 0u;
            if (RS) ls.ud[slot_of<FID>()] += above ? 0u : (q > floor(t)) ? 1u : 0x10000u;
        } else {
            qc = (uint32_t)q;  // q <= qmax
        }
        const bool neg = (double)val[c] < 0.0 && qc > 0u;
        os.emit(qc | ((neg ? 1u : 0u) << m1), f->bits);
        if (kF32Decode && is_f32<T>::value && f->f32dec) {
            const float mag = ldexpf((float)qc, E - m1);
            qv[c] = (T)(neg ? -mag : mag);
        } else {
            const double mag = ldexp((double)qc, E - m1);
            qv[c] = (T)(neg ? -mag : mag);
        }
    }
}

// Encodes field FID (values are the full attribute; the identity is removed
// here for a REL_IDENTITY field), appends its codes to the stream and
// returns the decoded stored values in qv (Eq. 1: the next substep starts
// from these).  T is double for x and float for v, C, F.
template <int DIM, int FID, typename T, bool RS>
__device__ __forceinline__ void enc_field(const FieldRef f, const T *val, Draws &rnd, OutStream &os,
                                          LaneStats &ls, T *qv) {
#pragma clang fp contract(off)
    constexpr int NC = ncomp<DIM, FID>(), K0 = canon0<DIM, FID>();
    if (f->kind == K_FIXED) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const bool diag = f->rel && (c % (DIM + 1) == 0);
            const double rel = diag ? (double)val[c] - 1.0 : (double)val[c];
            const double h = f->dither ? dither_h(rnd, K0 + c) : XI_HALF;
            const uint32_t code = enc_fixed<RS>(f, rel, h, slot_of<FID>(), ls);
            os.emit(code, f->bits);
            if (kF32Decode && is_f32<T>::value && f->f32dec) {
                const float q = fmaf((float)code, (float)f->delta, (float)f->lo);
                qv[c] = (T)(diag ? q + 1.0f : q);
            } else {
                const double q = fma((double)code, f->delta, f->lo);
                qv[c] = (T)(diag ? q + 1.0 : q);
            }
        }
    } else if (f->kind == K_RAW) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const bool diag = f->rel && (c % (DIM + 1) == 0);
            const float fv = (float)(diag ? (double)val[c] - 1.0 : (double)val[c]);
            os.emit(__float_as_uint(fv), 32);
            qv[c] = (T)(diag ? (double)fv + 1.0 : (double)fv);
        }
    } else {
        enc_sexp<DIM, FID, T, RS>(f, val, rnd, os, ls, qv);  // REL_IDENTITY is rejected for this kind
    }
}

// Decodes field FID exactly in binary64 (identity added back for a
// REL_IDENTITY field) and rounds once to T.
template <int DIM, int FID, typename T, typename Src>
__device__ __forceinline__ void dec_field_src(const FieldRef f, const Src &src, T *out) {
#pragma clang fp contract(off)
    constexpr int NC = ncomp<DIM, FID>();
    if (f->kind == K_FIXED) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t u = get_comp(src, f->off + c * f->bits, f->bits, f->mask);
            const bool diag = f->rel && (c % (DIM + 1) == 0);
            if (kF32Decode && is_f32<T>::value && f->f32dec) {
                const float q = fmaf((float)u, (float)f->delta, (float)f->lo);
                out[c] = (T)(diag ? q + 1.0f : q);
            } else {
                const double q = fma((double)u, f->delta, f->lo);
                out[c] = (T)(diag ? q + 1.0 : q);
            }
        }
    } else if (f->kind == K_RAW) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double q = (double)__uint_as_float(get_comp(src, f->off + 32 * c, 32, 0xffffffffu));
            out[c] = (T)((f->rel && (c % (DIM + 1) == 0)) ? q + 1.0 : q);
        }
    } else {
        const int E = (int)get_comp(src, f->off, f->exp_bits, f->exp_mask) + f->emin;
        const int m1 = f->bits - 1;
        const int o0 = f->off + f->exp_bits;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t q = get_comp(src, o0 + c * f->bits, f->bits, f->mask);
            if (kF32Decode && is_f32<T>::value && f->f32dec) {
                const float mag = ldexpf((float)(q & f->mag_mask), E - m1);
                out[c] = (T)(((q >> m1) & 1u) ? -mag : mag);
            } else {
                const double mag = ldexp((double)(q & f->mag_mask), E - m1);
                out[c] = (T)(((q >> m1) & 1u) ? -mag : mag);
            }
        }
    }
}



template <int DIM, int FID, typename T>
__device__ __forceinline__ void dec_field(const FieldRef f, const uint32_t *words, int64_t cap, uint32_t p4,
                                          T *out) {
    dec_field_src<DIM, FID, T>(f, GlobalRows{words, cap, p4}, out);
}

#ifdef MPMQ_SCHEME_CONST
// Record rows (bit k: word row k) that the bits of a field of the
// compile-time scheme occupy.
constexpr uint32_t field_rows(const DevField &f, int nc) {
    const int nbits = f.kind == K_RAW ? 32 * nc : f.kind == K_SEXP ? f.exp_bits + nc * f.bits : nc * f.bits;
    uint32_t m = 0u;
    for (int k = f.off >> 5; k <= (f.off + nbits - 1) >> 5; ++k) m |= 1u << k;
    return m;
}
// Loads the rows of `mask` of slot p4 / 4 into r[] (compile-time indices).
template <uint32_t MASK>
__device__ __forceinline__ void load_rows(const uint32_t *words, int64_t cap, uint32_t p4, uint32_t *r) {
#pragma unroll
    for (int k = 0; k < MAX_WORDS; ++k)
        if (MASK & (1u << k)) r[k] = ld_row(words, cap, k, p4);
}
#endif

// Decodes the whole record (F3: F for a solid, J for a fluid).
template <int DIM, typename T, int MAT>
__device__ __forceinline__ void decode_all(const DevScheme *sp, const uint32_t *words, int64_t cap, uint32_t p4,
                                           double *xv, T *vv, T *Cv, T *F3) {
    SchemeRef s = scheme_ref(sp);
    dec_field<DIM, 0, double>(&s->f[0], words, cap, p4, xv);
    dec_field<DIM, 1, T>(&s->f[1], words, cap, p4, vv);
    dec_field<DIM, 2, T>(&s->f[2], words, cap, p4, Cv);
    dec_field<DIM, fid3<MAT>(), T>(&s->f[3], words, cap, p4, F3);
}

// Encodes all four fields in placement order; qx.. receive the stored values.
template <int DIM, bool RS, int MAT>
__device__ __forceinline__ void encode_record(const DevScheme *sp, const double *x, const float *v,
                                              const float *C, const float *F3, Draws &rnd, OutStream &os,
                                              LaneStats &ls, double *qx, float *qv, float *qC, float *qF3) {
    // with a run-time scheme the four fields are one loop (the field order is
    // data); with a compile-time scheme it unrolls and every word boundary of
    // the stream is known at compile time
#ifdef MPMQ_SCHEME_CONST
#pragma unroll
#else
#pragma unroll 1
#endif
    for (int slot = 0; slot < 4; ++slot) {
        SchemeRef s = scheme_ref(sp);
        const int fid = s->order[slot];
        if (fid == 0) enc_field<DIM, 0, double, RS>(&s->f[0], x, rnd, os, ls, qx);
        else if (fid == 1) enc_field<DIM, 1, float, RS>(&s->f[1], v, rnd, os, ls, qv);
        else if (fid == 2) enc_field<DIM, 2, float, RS>(&s->f[2], C, rnd, os, ls, qC);
        else enc_field<DIM, fid3<MAT>(), float, RS>(&s->f[3], F3, rnd, os, ls, qF3);
    }
    os.finish();
}

// ---------------------------------------------------------------------------
// MLS-MPM helpers (quadratic B-spline, fixed-corotated elasticity).
// ---------------------------------------------------------------------------

// After the grid update a node block's storage (BLK^DIM GNodes of 32 B)
// holds the blocks's node velocities and masses as float4, packed into its
// first half: node l of the block in float4 slot l.  Node index id ->
// float4 index in the grid buffer.  Tile loads then use whole cache lines.
template <int DIM>
__device__ __forceinline__ int64_t vel_slot(int64_t id) {
    return id + (id & ~(int64_t)(Geo<DIM>::CPB - 1));
}
template <int DIM>
__device__ __forceinline__ float4 node_vel(const GNode *__restrict__ grid, int64_t id) {
    return reinterpret_cast<const float4 *>(grid)[vel_slot<DIM>(id)];
}

// Block-major node index: node blocks of BLK^DIM nodes, nb blocks per axis.
template <int DIM>
__device__ __forceinline__ int64_t node_index(const int *ijk, int nb) {
    constexpr int B = Geo<DIM>::BLK, L = Geo<DIM>::LOG;
    if (DIM == 3) {
        const int64_t blk = ((int64_t)(ijk[2] >> L) * nb + (ijk[1] >> L)) * nb + (ijk[0] >> L);
        return (blk << (3 * L)) + (((ijk[2] & (B - 1)) * B + (ijk[1] & (B - 1))) * B + (ijk[0] & (B - 1)));
    } else {
        const int64_t blk = (int64_t)(ijk[1] >> L) * nb + (ijk[0] >> L);
        return (blk << (2 * L)) + ((ijk[1] & (B - 1)) * B + (ijk[0] & (B - 1)));
    }
}

template <int DIM>
__device__ __forceinline__ int64_t block_of(const int *ijk, int nb) {
    constexpr int L = Geo<DIM>::LOG;
    if (DIM == 3) return ((int64_t)(ijk[2] >> L) * nb + (ijk[1] >> L)) * nb + (ijk[0] >> L);
    return (int64_t)(ijk[1] >> L) * nb + (ijk[0] >> L);
}

// base = clamp(floor(x/dx - 1/2), 0, n-3), f = x/dx - base (binary64, exact
// for the decoded lattice values and power-of-two grids).
template <int DIM>
__device__ __forceinline__ void stencil_base(const double *xd, double inv_dx, int res, int *base,
                                             float *fx) {
#pragma clang fp contract(off)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const double xs = xd[a] * inv_dx;
        double b = floor(xs - 0.5);
        b = (b >= 0.0) ? b : 0.0;  // NaN -> 0
        b = fmin(b, (double)(res - 3));
        base[a] = (int)b;
        fx[a] = (float)(xs - b);
    }
}

__device__ __forceinline__ void bspline(float f, float *w) {
    const float a = 1.5f - f, b = f - 1.0f, c = f - 0.5f;
    w[0] = 0.5f * a * a;
    w[1] = 0.75f - b * b;
    w[2] = 0.5f * c * c;
}

// Rotation of the polar decomposition F = R S.
// 2D: closed form from the rotation angle of F.
// 3D: Newton iteration R <- (R + R^-T)/2 from R = F, until every lane of the
// wave has taken a step shorter than 1e-4 (at most 16 iterations).
__device__ __forceinline__ void polar2(const float *F, float *R) {
    float c = F[0] + F[3], s = F[2] - F[1];
    const float r2 = c * c + s * s;
    if (r2 > 0.0f) {
        const float ir = rsqrtf(r2);
        c *= ir;
        s *= ir;
    } else {
        c = 1.0f;
        s = 0.0f;
    }
    R[0] = c; R[1] = -s; R[2] = s; R[3] = c;
}

// One Jacobi rotation of the symmetric 3x3 matrix held as its six distinct
// entries a = (a00, a01, a02, a11, a12, a22), in the (P, Q) plane (R the
// third index; all compile-time constants, so everything stays in
// registers): the angle zeroes a_PQ (tan from theta = (a_QQ - a_PP) / 2 a_PQ,
// the smaller root); V <- V J accumulates the eigenvectors as columns.
template <int P, int Q>
__device__ __forceinline__ void jacobi_rot3(float *a, float *V) {
    constexpr int R = 3 - P - Q;
    constexpr int ix[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    const float apq = a[ix[P][Q]];
    if (apq == 0.0f) return;
    const float app = a[ix[P][P]], aqq = a[ix[Q][Q]];
    const float theta = (aqq - app) / (2.0f * apq);
    const float t = (theta >= 0.0f ? 1.0f : -1.0f) / (fabsf(theta) + sqrtf(theta * theta + 1.0f));
    const float c = 1.0f / sqrtf(t * t + 1.0f), s = t * c;
    const float arp = a[ix[R][P]], arq = a[ix[R][Q]];
    a[ix[P][P]] = app - t * apq;
    a[ix[Q][Q]] = aqq + t * apq;
    a[ix[P][Q]] = 0.0f;
    a[ix[R][P]] = c * arp - s * arq;
    a[ix[R][Q]] = s * arp + c * arq;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const float vkp = V[k * 3 + P], vkq = V[k * 3 + Q];
        V[k * 3 + P] = c * vkp - s * vkq;
        V[k * 3 + Q] = s * vkp + c * vkq;
    }
}

__device__ __forceinline__ void cross3f(const float *a, const float *b, float *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

__device__ __forceinline__ void normalize3f(float *a) {
    const float n2 = a[0] * a[0] + a[1] * a[1] + a[2] * a[2];
    if (n2 > 0.0f) {
        const float r = 1.0f / sqrtf(n2);
        a[0] *= r; a[1] *= r; a[2] *= r;
    }
}

// Swaps eigenpairs a < b (compile-time) when lam[b] > lam[a]; V's columns.
template <int A, int B>
__device__ __forceinline__ void order_pair(float *lam, float *V) {
    if (lam[B] > lam[A]) {
        const float t = lam[A]; lam[A] = lam[B]; lam[B] = t;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float u = V[k * 3 + A]; V[k * 3 + A] = V[k * 3 + B]; V[k * 3 + B] = u;
        }
    }
}

// Closest rotation to F from its singular value decomposition, for F that
// is inverted or nearly singular (there Newton's iteration below either
// converges to a reflection or not at all).  F^T F = V diag(sigma^2) V^T by
// cyclic Jacobi sweeps; the singular directions are ordered by decreasing
// sigma and V made a proper rotation (v_3 = v_1 x v_2); u_a = F v_a / sigma_a
// for the two largest (Gram-Schmidt), u_3 = u_1 x u_2; R = U V^T.  R is then
// the fixed-corotated model's rotation: det R = +1, with the reflection of an
// inverted F carried by the direction of its smallest singular value.
__device__ __forceinline__ void polar3_svd(const float *F, float *R) {
    float a[6], V[9] = {1.0f, 0.0f, 0.0f, 0.0f, 1.0f, 0.0f, 0.0f, 0.0f, 1.0f};
    {
        int k = 0;
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) a[k++] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
    }
    for (int sweep = 0; sweep < 12; ++sweep) {
        const float off = a[1] * a[1] + a[2] * a[2] + a[4] * a[4];
        const float diag = a[0] * a[0] + a[3] * a[3] + a[5] * a[5];
        if (!(off > 1e-14f * diag)) break;
        jacobi_rot3<0, 1>(a, V);
        jacobi_rot3<0, 2>(a, V);
        jacobi_rot3<1, 2>(a, V);
    }
    // eigenvalues with their eigenvector columns, by decreasing value
    float lam[3] = {a[0], a[3], a[5]};
    order_pair<0, 1>(lam, V);
    order_pair<0, 2>(lam, V);
    order_pair<1, 2>(lam, V);
    {
        const float v0[3] = {V[0], V[3], V[6]}, v1[3] = {V[1], V[4], V[7]};
        float v2[3];
        cross3f(v0, v1, v2);
        V[2] = v2[0]; V[5] = v2[1]; V[8] = v2[2];
    }
    const float s0 = sqrtf(fmaxf(lam[0], 0.0f)), s1 = sqrtf(fmaxf(lam[1], 0.0f));
    if (!(s0 > 0.0f)) {
#pragma unroll
        for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0f : 0.0f;
        return;
    }
    float u0[3], u1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        u0[k] = F[k * 3] * V[0] + F[k * 3 + 1] * V[3] + F[k * 3 + 2] * V[6];
        u1[k] = F[k * 3] * V[1] + F[k * 3 + 1] * V[4] + F[k * 3 + 2] * V[7];
    }
    normalize3f(u0);
    const float d = u1[0] * u0[0] + u1[1] * u0[1] + u1[2] * u0[2];
#pragma unroll
    for (int k = 0; k < 3; ++k) u1[k] -= d * u0[k];
    const float n1 = sqrtf(u1[0] * u1[0] + u1[1] * u1[1] + u1[2] * u1[2]);
    if (!(s1 > 1e-30f) || !(n1 > 1e-5f * s0)) {
        // rank one: any unit vector orthogonal to u_1 (from the axis least aligned with it)
        const float ax = fabsf(u0[0]), ay = fabsf(u0[1]), az = fabsf(u0[2]);
        float e[3] = {0.0f, 0.0f, 0.0f};
        if (ax <= ay && ax <= az) e[0] = 1.0f;
        else if (ay <= az) e[1] = 1.0f;
        else e[2] = 1.0f;
        cross3f(u0, e, u1);
    }
    normalize3f(u1);
    float u2[3];
    cross3f(u0, u1, u2);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) R[i * 3 + j] = u0[i] * V[j * 3] + u1[i] * V[j * 3 + 1] + u2[i] * V[j * 3 + 2];
}

// The SVD branch as a called function: a kernel near an occupancy step of
// its register count keeps the branch's registers out of its own allocation
// (the call is taken by the rare lanes only).
static __device__ __attribute__((noinline)) void polar3_svd_call(const float *F, float *R) { polar3_svd(F, R); }

// Newton's iteration R <- (R + R^-T) / 2 from R = F converges to the
// orthogonal polar factor, which is the closest rotation when det F > 0.
// Lanes where it does not deliver that rotation -- an inverted F (the limit
// is a reflection, det R = -1), a singular or degenerate F (a vanishing
// determinant on the way) or no convergence within 16 steps -- take the SVD
// above, after the iteration (which then holds no extra state).  OUTLINE:
// call the SVD instead of inlining it.
template <bool OUTLINE = false>
__device__ __forceinline__ void polar3(const float *F, float *R) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = F[i];
    bool bad = false;
    float d2 = 0.0f;
    for (int it = 0; it < 16; ++it) {
        // cofactor matrix = det * R^-T
        const float c00 = R[4] * R[8] - R[5] * R[7], c01 = R[5] * R[6] - R[3] * R[8],
                    c02 = R[3] * R[7] - R[4] * R[6];
        const float c10 = R[2] * R[7] - R[1] * R[8], c11 = R[0] * R[8] - R[2] * R[6],
                    c12 = R[1] * R[6] - R[0] * R[7];
        const float c20 = R[1] * R[5] - R[2] * R[4], c21 = R[2] * R[3] - R[0] * R[5],
                    c22 = R[0] * R[4] - R[1] * R[3];
        const float det = R[0] * c00 + R[1] * c01 + R[2] * c02;
        const bool ok = fabsf(det) > 1e-20f;
        bad |= !ok;
        // hardware reciprocal (1 ulp): the iteration absorbs its error
        const float hid = ok ? 0.5f * __builtin_amdgcn_rcpf(det) : 0.0f;
        // the Newton step d = (R^-T - R) / 2, added in place
        const float cf[9] = {c00, c01, c02, c10, c11, c12, c20, c21, c22};
        d2 = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const float d = fmaf(hid, cf[i], -0.5f * R[i]);
            d2 = fmaf(d, d, d2);
            R[i] += d;
        }
        // a lane with a vanishing determinant takes the SVD below whatever
        // its iterate (halved here, hid = 0): it no longer holds the loop
        d2 = ok ? d2 : 0.0f;
        // Newton's polar iteration converges quadratically: the error of the
        // new iterate is about |R_new - R|^2 / (2 sigma_min), at most 5e-8
        // once the squared step is under 1e-7 (for sigma_min near 1): the
        // float32 rounding of R's entries near 1, and below the rounding of
        // F - R, which the stress uses.  (A bound of 1e-8 costs a second
        // iteration for nearly every wave: strains of 1e-4, common, give a
        // first step of about 1e-4.)
        if (!__any(d2 > 1e-7f)) break;
    }
    const float detR = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                       R[2] * (R[3] * R[7] - R[4] * R[6]);
    bad |= !(detR > 0.5f) || d2 > 1e-7f;
    if (bad) {
        if constexpr (OUTLINE) polar3_svd_call(F, R);
        else polar3_svd(F, R);
    }
}

}  // namespace mpmq
