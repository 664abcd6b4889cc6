// mpmq_device.hpp -- gfx950 device functions of the quantized MLS-MPM
// substep: bit-pack extraction/insertion, the three storage kinds, the
// Philox dither draws and the MLS-MPM stencil helpers.
#pragma once
#include "mpmq_internal.hpp"

namespace mpmq {

template <int N> using uvec = uint32_t __attribute__((ext_vector_type(N)));

enum { K_FIXED = 0, K_SEXP = 1, K_RAW = 2 };

// ---------------------------------------------------------------------------
// Bit pack (Sec. 7, Figs. 7-8).  A record of W words lives in a register
// vector; a component is located by a wave-uniform descriptor, so the
// indexed register reads compile to uniform indexed moves (no scratch).  A
// component that spans two words is rebuilt with one funnel shift: alignbit
// concatenates (hi:lo) and shifts right, the mask keeps `bits` bits.
// ---------------------------------------------------------------------------
template <int WM>
__device__ __forceinline__ uint32_t get_code(const uvec<WM> &w, uint32_t desc, uint32_t mask) {
    const uint32_t k = desc & 0xffu, kh = (desc >> 8) & 0xffu, sh = (desc >> 16) & 0xffu;
    return __builtin_amdgcn_alignbit(w[kh], w[k], sh) & mask;
}

template <int WM>
__device__ __forceinline__ void put_code(uvec<WM> &w, uint32_t desc, uint32_t code) {
    const uint32_t k = desc & 0xffu, sh = (desc >> 16) & 0xffu;
    w[k] |= code << sh;
    if (desc >> 24) w[k + 1] |= code >> (32u - sh);  // spans => sh > 0
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two
// 32x32->64 multiplies with the published multipliers, key bumped by the
// Weyl constants between rounds.  Counter (slot, step, group, tag), key =
// seed.  Record component k takes 16 bits: half k%2 of word k/2 of the
// concatenated group outputs.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                         uint32_t k0, uint32_t k1, uint32_t *out) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

__device__ __forceinline__ uvec<16> dither_draws(const DevScheme &s, uint32_t slot, uint32_t step,
                                                 uint32_t tag) {
    uvec<16> r = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if ((s.dither_groups >> j) & 1u) {
            uint32_t o[4];
            philox10(slot, step, (uint32_t)j, tag, s.seed_lo, s.seed_hi, o);
            r[4 * j + 0] = o[0];
            r[4 * j + 1] = o[1];
            r[4 * j + 2] = o[2];
            r[4 * j + 3] = o[3];
        }
    }
    return r;
}

// xi' in (0,1): (r16 + 1/2) 2^-16, exact in binary64.
__device__ __forceinline__ double dither_xi(const uvec<16> &r, int k) {
    const uint32_t w = r[k >> 1];
    const uint32_t h = (k & 1) ? (w >> 16) : (w & 0xffffu);
    return ((double)h + 0.5) * (1.0 / 65536.0);
}

// ---------------------------------------------------------------------------
// Encoder statistics kept per lane and flushed per work item:
// ud[f] = round-ups | round-downs << 16, sat / nan: 8 bits per field.
// ---------------------------------------------------------------------------
struct LaneStats {
    uint32_t ud[4];
    uint32_t sat, nan;
    __device__ void clear() { ud[0] = ud[1] = ud[2] = ud[3] = 0; sat = nan = 0; }
};

// Fixed point (Eq. 3, Eq. 11 when r = xi): binary64, no contraction, so the
// rounding sequence is exactly t = RN(RN(val - lo) * inv), s = RN(t + r),
// u = clamp(floor(s)).
__device__ __forceinline__ uint32_t enc_fixed(const DevField &f, double val, double r, int fid,
                                              LaneStats &ls) {
#pragma clang fp contract(off)
    const double t = (val - f.lo) * f.inv;
    const double sv = t + r;
    const double fl = floor(sv);
    uint32_t code;
    if (!(sv == sv)) {
        code = 0u;
        ls.nan += 1u << (8 * fid);
    } else if (fl < 0.0) {
        code = 0u;
        ls.sat += 1u << (8 * fid);
    } else if (fl > f.maxc) {
        code = (uint32_t)f.maxc;
        ls.sat += 1u << (8 * fid);
    } else {
        code = (uint32_t)fl;
        ls.ud[fid] += (fl > floor(t)) ? 1u : 0x10000u;
    }
    return code;
}

// Shared-exponent vector: E from the largest magnitude, raised by one if a
// magnitude rounds up to 2^(m-1); then sign | magnitude per component.
template <int NC, int WM>
__device__ __forceinline__ void enc_sexp(const DevScheme &s, int fid, const double *val,
                                         const uvec<16> &rnd, uvec<WM> &w, LaneStats &ls) {
#pragma clang fp contract(off)
    const DevField &f = s.f[fid];
    const int m1 = f.bits - 1;
    const double qmax = (double)f.mag_mask;
    double a[NC];
    double M = 0.0;
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        double x = val[c];
        if (!(x == x)) {
            ls.nan += 1u << (8 * fid);
            x = 0.0;
        }
        a[c] = fabs(x);
        M = fmax(M, a[c]);
    }
    int E;
    if (M == 0.0) E = f.emin;
    else if (isinf(M)) E = f.emax;
    else E = min(max(ilogb(M) + 1, f.emin), f.emax);
    double q[NC], t[NC];
    bool over = true;
    while (over) {
        over = false;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            t[c] = ldexp(a[c], m1 - E);
            const double r = f.dither ? dither_xi(rnd, f.k0 + c) : 0.5;
            q[c] = floor(t[c] + r);
            over |= q[c] > qmax;
        }
        if (over && E < f.emax) E += 1;
        else over = false;
    }
    put_code(w, f.exp_desc, (uint32_t)(E - f.emin));
#pragma unroll
    for (int c = 0; c < NC; ++c) {
        uint32_t qc;
        if (q[c] > qmax) {
            qc = f.mag_mask;
            ls.sat += 1u << (8 * fid);
        } else {
            qc = (uint32_t)q[c];
            ls.ud[fid] += (q[c] > floor(t[c])) ? 1u : 0x10000u;
        }
        const uint32_t sign = (val[c] < 0.0 && qc > 0u) ? 1u : 0u;
        put_code(w, s.cdesc[fid][c], qc | (sign << m1));
    }
}

// Encode NC values of field `fid` into the record (values are the full
// attribute; the identity is removed here for a REL_IDENTITY field).
template <int DIM, int NC, int WM>
__device__ __forceinline__ void enc_field(const DevScheme &s, int fid, const double *val,
                                          const uvec<16> &rnd, uvec<WM> &w, LaneStats &ls) {
#pragma clang fp contract(off)
    const DevField &f = s.f[fid];
    double rel[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) rel[c] = (f.rel && (c % (DIM + 1) == 0)) ? val[c] - 1.0 : val[c];
    if (f.kind == K_FIXED) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const double r = f.dither ? dither_xi(rnd, f.k0 + c) : 0.5;
            put_code(w, s.cdesc[fid][c], enc_fixed(f, rel[c], r, fid, ls));
        }
    } else if (f.kind == K_RAW) {
#pragma unroll
        for (int c = 0; c < NC; ++c) put_code(w, s.cdesc[fid][c], __float_as_uint((float)rel[c]));
    } else {
        enc_sexp<NC>(s, fid, rel, rnd, w, ls);
    }
}

// Decode field `fid` exactly in binary64 (the identity added back for a
// REL_IDENTITY field).
template <int DIM, int NC, int WM>
__device__ __forceinline__ void dec_field(const DevScheme &s, int fid, const uvec<WM> &w, double *out) {
#pragma clang fp contract(off)
    const DevField &f = s.f[fid];
    if (f.kind == K_FIXED) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            out[c] = fma((double)get_code(w, s.cdesc[fid][c], s.cmask[fid][c]), f.delta, f.lo);
    } else if (f.kind == K_RAW) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
            out[c] = (double)__uint_as_float(get_code(w, s.cdesc[fid][c], s.cmask[fid][c]));
    } else {
        const int E = (int)get_code(w, f.exp_desc, f.exp_mask) + f.emin;
        const int m1 = f.bits - 1;
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const uint32_t q = get_code(w, s.cdesc[fid][c], s.cmask[fid][c]);
            const double mag = ldexp((double)(q & f.mag_mask), E - m1);
            out[c] = ((q >> m1) & 1u) ? -mag : mag;
        }
    }
    if (f.rel) {
#pragma unroll
        for (int c = 0; c < NC; c += DIM + 1) out[c] = out[c] + 1.0;
    }
}

// Loads the W words of slot p (word-major, stride cap) into a register record.
template <int WM>
__device__ __forceinline__ uvec<WM> load_record(const uint32_t *__restrict__ words, int W, int64_t cap,
                                                int64_t p) {
    uvec<WM> w = 0;
#pragma unroll
    for (int k = 0; k < WM; ++k)
        if (k < W) w[k] = __builtin_nontemporal_load(words + (int64_t)k * cap + p);
    return w;
}

template <int WM>
__device__ __forceinline__ void store_record(uint32_t *__restrict__ words, int W, int64_t cap, int64_t p,
                                             const uvec<WM> &w) {
#pragma unroll
    for (int k = 0; k < WM; ++k)
        if (k < W) __builtin_nontemporal_store(w[k], words + (int64_t)k * cap + p);
}

// ---------------------------------------------------------------------------
// MLS-MPM helpers (quadratic B-spline, fixed-corotated elasticity).
// ---------------------------------------------------------------------------

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
// 3D: Newton iteration R <- (R + R^-T)/2 from R = F, until all lanes of the
// wave have converged (at most 16 iterations); quadratic convergence near
// the identity.
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

__device__ __forceinline__ void polar3(const float *F, float *R) {
#pragma unroll
    for (int i = 0; i < 9; ++i) R[i] = F[i];
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
        const float hid = ok ? 0.5f / det : 0.0f;
        float Rn[9] = {0.5f * R[0] + hid * c00, 0.5f * R[1] + hid * c01, 0.5f * R[2] + hid * c02,
                       0.5f * R[3] + hid * c10, 0.5f * R[4] + hid * c11, 0.5f * R[5] + hid * c12,
                       0.5f * R[6] + hid * c20, 0.5f * R[7] + hid * c21, 0.5f * R[8] + hid * c22};
        float d2 = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const float d = Rn[i] - R[i];
            d2 += d * d;
            R[i] = ok ? Rn[i] : ((i % 4 == 0) ? 1.0f : 0.0f);
        }
        if (!__any(d2 > 1e-13f)) break;
    }
}

}  // namespace mpmq
