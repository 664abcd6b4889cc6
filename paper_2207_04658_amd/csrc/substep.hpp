// substep.hpp -- gfx950 device code of the fused substep and of the
// bootstrap P2G: integer fixed-point P2G into an LDS node tile, G2P from
// the tile, the per-particle update, the dithered encode and store.
// Compiled into libmpmq.so for any scheme read at run time (64-bit node
// tile), and (when a context asks for it) compiled again at run time with
// the context's scheme as a compile-time constant (32-bit node tile at
// per-item scales, three work-groups per CU).
#pragma once
#include "mpmq_device.hpp"

namespace mpmq {

// ---------------------------------------------------------------------------
// small utilities
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Wave-wide minimum / maximum (all 64 lanes active; the result is wave-
// uniform): DPP row shifts by 1, 2, 4, 8 leave each row's extreme in its lane
// 15, row broadcasts of lanes 15 and 31 carry them into lane 63, which is
// read back.  A source lane outside its row keeps the lane's own value.
template <bool MAX, int CTRL, int ROWS>
__device__ __forceinline__ float dpp_ext(float v) {
    const int o = __float_as_int(v);
    const float t = __int_as_float(__builtin_amdgcn_update_dpp(o, o, CTRL, ROWS, 0xf, false));
    return MAX ? fmaxf(v, t) : fminf(v, t);
}
template <bool MAX>
__device__ __forceinline__ float wave_ext(float v) {
    v = dpp_ext<MAX, 0x111, 0xf>(v);  // row_shr:1
    v = dpp_ext<MAX, 0x112, 0xf>(v);  // row_shr:2
    v = dpp_ext<MAX, 0x114, 0xf>(v);  // row_shr:4
    v = dpp_ext<MAX, 0x118, 0xf>(v);  // row_shr:8
    v = dpp_ext<MAX, 0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v = dpp_ext<MAX, 0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}
__device__ __forceinline__ float wave_min(float v) { return wave_ext<false>(v); }
__device__ __forceinline__ float wave_max(float v) { return wave_ext<true>(v); }
// A value equal in every lane, moved to scalar registers.
__device__ __forceinline__ int32_t uni(int32_t v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uni(float v) { return __int_as_float(uni(__float_as_int(v))); }

__device__ __forceinline__ void flush_stats(const LaneStats &ls, uint64_t *stats) {
    if (!__any((ls.ud[0] | ls.ud[1] | ls.ud[2] | ls.ud[3] | ls.sat | ls.nan) != 0u)) return;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const uint32_t up = wave_sum(ls.ud[f] & 0xffffu);
        const uint32_t dn = wave_sum(ls.ud[f] >> 16);
        const uint32_t sat = wave_sum((ls.sat >> (8 * f)) & 0xffu);
        const uint32_t nan = wave_sum((ls.nan >> (8 * f)) & 0xffu);
        if (__lane_id() == 0) {
            if (up) atomicAdd((unsigned long long *)&stats[ST_UP + f], (unsigned long long)up);
            if (dn) atomicAdd((unsigned long long *)&stats[ST_DOWN + f], (unsigned long long)dn);
            if (sat) atomicAdd((unsigned long long *)&stats[ST_SAT + f], (unsigned long long)sat);
            if (nan) atomicAdd((unsigned long long *)&stats[ST_NAN + f], (unsigned long long)nan);
        }
    }
}

__device__ __forceinline__ void add_stat(uint64_t *stats, int slot, uint32_t lane_value) {
    const uint32_t s = wave_sum(lane_value);
    if (__lane_id() == 0 && s) atomicAdd((unsigned long long *)&stats[slot], (unsigned long long)s);
}


// Fixed-point conversion: round(v * 2^32) as two's complement int64 for
// |v| < 2^19, via binary64: fma(w, x, 1.5*2^52) puts the rounded integer in
// the low mantissa bits (exponent field constant), the subtraction removes
// the offset.  w * x carries the 2^32 scale already.
__device__ __forceinline__ unsigned long long fixp(double w, double xs) {
    return (unsigned long long)__double_as_longlong(fma(w, xs, FIX_MAGIC)) - FIX_MAGIC_BITS;
}

// Raw fixed-point term of an LDS node tile: the bits of fma(w, x, 1.5 2^52),
// FIX_MAGIC_BITS + round(w x) for |w x| < 2^51 (x carries the fixed-point
// scale).  The 64-bit tile of the bootstrap P2G adds them without removing
// the offset: a node that received n terms holds n FIX_MAGIC_BITS + S
// (mod 2^64) in each of its four sums.  FIX_MAGIC_BITS = 2151 * 2^51, so
// n FIX_MAGIC_BITS mod 2^64 lies in the top 13 bits only; the mass sum S_m
// of at most 4096 terms (a work item) of at most 2^32 stays below 2^51, so
// the top 13 bits of the raw mass word are exactly that offset (tile_flush
// subtracts it from all four sums).  The low 32 bits of FIX_MAGIC_BITS are
// zero, so the low word of fixr(w, x) is round(w x) mod 2^32 (two's
// complement): the term of the fused kernel's 32-bit tile.
__device__ __forceinline__ unsigned long long fixr(double w, double xs) {
    return (unsigned long long)__double_as_longlong(fma(w, xs, FIX_MAGIC));
}
constexpr unsigned long long RAW_OFFSET_MASK = 0xFFF8000000000000ull;  // top 13 bits

// P2G straight into the grid buffer, for a particle whose stencil left its tile.
template <int DIM>
__device__ __forceinline__ void p2g_global(const DevParams &P, const int *base, const double (*w)[3],
                                           const double *q, const double (*ac)[DIM], GNode *__restrict__ gout,
                                           uint32_t *__restrict__ flags) {
    constexpr int NST = Geo<DIM>::NST;
#pragma unroll
    for (int s = 0; s < NST; ++s) {
        const int o[3] = {s % 3, (s / 3) % 3, s / 9};
        int ijk[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) ijk[a] = base[a] + o[a];
        // the same products, in the same order, as the tile path
        const double wr = (DIM == 3) ? w[2][o[2]] * w[1][o[1]] : w[1][o[1]];
        const double wt = wr * w[0][o[0]];
        unsigned long long *g = gout[node_index<DIM>(ijk, P.nb)].q;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double val = q[a];
#pragma unroll
            for (int b = 0; b < DIM; ++b) val += ac[b][a] * (double)o[b];
            atomicAdd(g + a, fixp(wt, val));
        }
        atomicAdd(g + 3, fixp(w[0][o[0]], wr * FIX_ONE));
        flags[block_of<DIM>(ijk, P.nb)] = 1u;
    }
}

// ---------------------------------------------------------------------------
// Node tile of the scheme-specialized fused kernel: 32-bit sums at a
// per-work-item scale (the generic build keeps the exact 64-bit tile).
//
// A work item's particles add, per node, w_i (v + (A/m)(x_i - x_p) - vref)
// in units of 2^-s (three momentum sums) and w_i in units of 2^-sm (the
// weight sum), each term rounded once, as 32-bit integers (LDS integer
// atomics: exact and order-independent).  vref (a multiple of 2^-(32 - sm),
// per item) centres the momentum sums on the item's velocities; the flush
// adds vref * (weight sum) back and shifts everything to the grid's 2^-32
// fixed point.  Bounds: a particle weight is at most 0.75^DIM, so a node's
// weight sum is below Wb = N_item * 0.75^DIM; sm is the largest exponent
// with Wb 2^sm < 2^32, and a particle enters the tile only if all its node
// values lie within lim 2^-s of vref with lim Wb < 2^31 (and its weights are
// B-spline weights, 0.5 <= f <= 1.5).  Then no node sum leaves the 32-bit
// range, and the rest go through the global 64-bit path (counted, ST_WIDE).
// s is the largest exponent at which the deviation the item's record of its
// last P2G predicts fits under lim (tile_scale, item_record).
// ---------------------------------------------------------------------------

// P2G of one particle from its decoded (quantized) state.  Node i receives,
// per unit particle mass, w_i (v + (A/m)(x_i - x_p)) and w_i (Eq. 1 with
// the MLS-MPM affine momentum), accumulated as exact fixed point: with
// AccT = unsigned long long as 64-bit sums at 2^-32 (raw terms, see fixr;
// the offset comes off at the flush), with AccT = uint32_t in the 32-bit
// tile above (the specialized fused kernel, and k_p2g replaying its
// scales).  Stencils outside the tile go to the grid directly (p2g_global).
// OUTLINE: the polar decomposition's rare SVD branch as a call (see polar3).
template <int DIM, int MAT, bool OUTLINE, typename AccT>
__device__ __forceinline__ void p2g_particle(const DevParams &P, const double *xd, const float *v,
                                             const float *C, const float *F, const int *origin,
                                             AccT *__restrict__ acc, GNode *__restrict__ gout,
                                             uint32_t *__restrict__ flags, uint32_t &fallback,
                                             uint32_t &clamped, uint32_t &wide, const bool tile_ok,
                                             const volatile TileScale &ts, float &rec) {
    constexpr bool T32 = sizeof(AccT) == 4;
    // the scales live in LDS (one copy per wave, written by the wave itself):
    // read here, so that they hold no registers across the particle loop
    float vref[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) vref[a] = ts.vref[a];
    constexpr int TB = Geo<DIM>::TB, TS = Geo<DIM>::TS, D2 = DIM * DIM;
    // |q|, |a_b| <= 2^12 keeps a node value q + sum_b a_b o_b below 2^15
    // (2^47 in fixed point), so a grid node sum of up to 2^16 contributions
    // stays inside int64.  A particle with a larger term is clamped and
    // counted (ST_CLAMP); the count sees finite values only: a NaN is
    // clamped too, and is counted by the encoder's NaN counter where it is
    // stored.
    constexpr float LIM = 4096.0f;
    int base[DIM];
    float fx[DIM];
    stencil_base<DIM>(xd, P.inv_dx_d, P.res, base, fx);
    double w[DIM][3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float wf[3];
        bspline(fx[a], wf);
        w[a][0] = wf[0];
        w[a][1] = wf[1];
        w[a][2] = wf[2];
    }
    // A / m_p = -4 dt / (rho dx^2) tau + C
    float Am[D2];
    if constexpr (MAT == 1) {
        // fluid: tau = pc (J - 1) I, J = F[0]
        const float t = P.stress_over_m * P.pc * (F[0] - 1.0f);
#pragma unroll
        for (int i = 0; i < D2; ++i) Am[i] = C[i] + ((i % (DIM + 1) == 0) ? t : 0.0f);
    } else {
        // fixed-corotated Kirchhoff stress tau = 2 mu (F - R) F^T + lambda J (J-1) I
        float R[D2];
        float J;
        if constexpr (DIM == 2) {
            polar2(F, R);
            J = F[0] * F[3] - F[1] * F[2];
        } else {
            polar3<OUTLINE>(F, R);
            J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
                F[2] * (F[3] * F[7] - F[4] * F[6]);
        }
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                float t = 0.0f;
#pragma unroll
                for (int k = 0; k < DIM; ++k) t += (F[i * DIM + k] - R[i * DIM + k]) * F[j * DIM + k];
                t = 2.0f * P.mu * t + ((i == j) ? P.la * J * (J - 1.0f) : 0.0f);
                Am[i * DIM + j] = P.stress_over_m * t + C[i * DIM + j];
            }
    }
    // node value = q + sum_b a_b o_b, q = v - (A/m) f dx, a_b = (A/m)[:, b] dx,
    // scaled by 2^32
    double q[DIM], ac[DIM][DIM];  // ac[b][a]
    float big = 0.0f;  // largest |term| before clamping
    float dev[DIM];    // bound of |node value - vref| over the stencil (32-bit tile)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float t = v[a], d = 0.0f;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const float ab0 = Am[a * DIM + b] * P.dx;
            big = fmaxf(big, fabsf(ab0));
            const float ab = fminf(fmaxf(ab0, -LIM), LIM);
            ac[b][a] = (double)ab * FIX_ONE;
            d += 2.0f * fabsf(ab);
            t -= ab * fx[b];
        }
        big = fmaxf(big, fabsf(t));
        const float tc = fminf(fmaxf(t, -LIM), LIM);
        q[a] = (double)tc * FIX_ONE;
        // 32-bit tile: the admission bound; 64-bit tile: an estimate of the
        // same bound about vref from v (|sum_b a_b f_b| <= 1.5 sum_b |a_b|)
        dev[a] = T32 ? d + fabsf(tc - vref[a]) : fabsf(v[a] - vref[a]) + 1.75f * d;
    }
    clamped += (big > LIM) ? 1u : 0u;
    bool stencil_in = tile_ok;
    int l[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        l[a] = base[a] - origin[a];
        stencil_in &= (l[a] >= 0) && (l[a] <= TB - 3);
    }
    // rec (the caller's running maximum, see tile_scale): the largest
    // deviation bound of a particle whose stencil is in the tile
#pragma unroll
    for (int a = 0; a < DIM; ++a) rec = fmaxf(rec, stencil_in ? dev[a] : 0.0f);
    bool in_tile = stencil_in;
    if constexpr (T32) {
        // admission to the 32-bit tile: |q + sum_b a_b o_b - vref| <= lim_v
        // for o_b in {0, 1, 2}, and B-spline weights (a clamped stencil base
        // at the grid edge, or a NaN position, gives others)
        bool fits = true;
        const float lim_v = ts.lim_v;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            fits &= dev[a] <= lim_v;  // false for a NaN
            fits &= fx[a] >= 0.5f && fx[a] <= 1.5f;
        }
        wide += (stencil_in && !fits) ? 1u : 0u;
        in_tile = stencil_in && fits;
    }
    if (in_tile) {
        const int l0 = (DIM == 3) ? (l[DIM - 1] * TB + l[1]) * TB + l[0] : l[1] * TB + l[0];
        // 32-bit tile: node values less vref (still scaled by 2^32) times
        // weights scaled by 2^(s - 32), weight sums at 2^sm; 64-bit tile:
        // 2^32 throughout.  A tile term is (AccT)fixr: the raw bits for the
        // 64-bit tile, the low word of the rounded value for the 32-bit one.
        if constexpr (T32) {
#pragma unroll
            for (int a = 0; a < DIM; ++a) q[a] -= (double)vref[a] * FIX_ONE;
        }
        const int ex = T32 ? ts.s - 32 : 0, sw = T32 ? ts.sm : 32;
        // node values stepped along each axis (q + sum_b a_b o_b by additions)
        if constexpr (DIM == 3) {
            // x weights at the two scales (exact: powers of two); a term's
            // weight is then w_z w_y (exact in binary64) times one of them
            double wxs[3], wxm[3];
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                wxs[ox] = ldexp(w[0][ox], ex);
                wxm[ox] = ldexp(w[0][ox], sw);
            }
            double vz[3] = {q[0], q[1], q[2]};
#pragma unroll
            for (int oz = 0; oz < 3; ++oz) {
                if (oz > 0)
#pragma unroll
                    for (int a = 0; a < 3; ++a) vz[a] += ac[2][a];
                double vzy[3] = {vz[0], vz[1], vz[2]};
#pragma unroll
                for (int oy = 0; oy < 3; ++oy) {
                    if (oy > 0)
#pragma unroll
                        for (int a = 0; a < 3; ++a) vzy[a] += ac[1][a];
                    const double wzy = w[2][oz] * w[1][oy];
                    double val[3] = {vzy[0], vzy[1], vzy[2]};
#pragma unroll
                    for (int ox = 0; ox < 3; ++ox) {
                        if (ox > 0)
#pragma unroll
                            for (int a = 0; a < 3; ++a) val[a] += ac[0][a];
                        const double wt = wzy * wxs[ox];
                        const int idx = l0 + (oz * TB + oy) * TB + ox;
#pragma unroll
                        for (int a = 0; a < 3; ++a) atomicAdd(&acc[a * TS + idx], (AccT)fixr(wt, val[a]));
                        atomicAdd(&acc[3 * TS + idx], (AccT)fixr(wxm[ox], wzy));
                    }
                }
            }
        } else {
            double vy[2] = {q[0], q[1]};
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                if (oy > 0)
#pragma unroll
                    for (int a = 0; a < 2; ++a) vy[a] += ac[1][a];
                const double ms = ldexp(w[1][oy], sw), wys = ldexp(w[1][oy], ex);  // exact (powers of two)
                double val[2] = {vy[0], vy[1]};
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    if (ox > 0)
#pragma unroll
                        for (int a = 0; a < 2; ++a) val[a] += ac[0][a];
                    const double wt = wys * w[0][ox];
                    const int idx = l0 + oy * TB + ox;
#pragma unroll
                    for (int a = 0; a < 2; ++a) atomicAdd(&acc[a * TS + idx], (AccT)fixr(wt, val[a]));
                    atomicAdd(&acc[3 * TS + idx], (AccT)fixr(w[0][ox], ms));
                }
            }
        }
    } else {
        fallback += (tile_ok && !stencil_in) ? 1u : 0u;
        p2g_global<DIM>(P, base, w, q, ac, gout, flags);
    }
}

// Work items with this many particles or fewer skip the node tiles: their
// particles gather and scatter straight from and to the grid buffers (a
// sparse scene gives items of a few particles, for which loading and
// flushing a whole tile costs more than the particles' own global accesses).
template <int DIM> constexpr int sparse_item() { return Geo<DIM>::TN / 48; }

// tile helpers ---------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void tile_origin(int block, int nb, int *origin) {
    constexpr int B = Geo<DIM>::BLK;
    origin[0] = (block % nb) * B - 1;
    if constexpr (DIM == 3) {
        origin[1] = ((block / nb) % nb) * B - 1;
        origin[2] = (block / (nb * nb)) * B - 1;
    } else {
        origin[1] = (block / nb) * B - 1;
    }
}

template <int DIM>
__device__ __forceinline__ bool tile_node(int t, const int *origin, int res, int *ijk) {
    constexpr int TB = Geo<DIM>::TB;
    ijk[0] = origin[0] + t % TB;
    if constexpr (DIM == 3) {
        ijk[1] = origin[1] + (t / TB) % TB;
        ijk[2] = origin[2] + t / (TB * TB);
    } else {
        ijk[1] = origin[1] + t / TB;
    }
    bool ok = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) ok &= (ijk[a] >= 0) && (ijk[a] < res);
    return ok;
}

// Adds the tile's non-zero node sums (raw sums less the offset of their
// terms, see fixr) to the grid with int64 atomics and flags
// the node blocks that received data.  A tile (origin = block corner - 1)
// overlaps 3 node blocks per axis: its first node layer lies in the block
// before, the next BLK in its own block, the rest in the block after.  The
// flags go through `touched` (LDS, 3^DIM entries, zero on entry and on
// return): one global store per touched block instead of one per node.
// Neighbour-block code of tile node t: (l == 0 ? 0 : l <= BLK ? 1 : 2) per
// axis, last axis most significant.
template <int DIM>
__device__ __forceinline__ int tile_block_code(const int *ijk, const int *origin) {
    constexpr int B = Geo<DIM>::BLK;
    int k = 0;
#pragma unroll
    for (int a = DIM - 1; a >= 0; --a) {
        const int l = ijk[a] - origin[a];  // 0 .. TB-1
        k = 3 * k + ((l == 0) ? 0 : (l <= B) ? 1 : 2);
    }
    return k;
}

// `table` (optional LDS scratch of TN words + TN bytes, free at the flush):
// the grid index and block code of every tile node are computed once, not
// once per component.
// natom counts the lane's global atomic adds.  AccT = uint32_t: the fused
// kernel's 32-bit tile at the scales of ts, widened here to 2^-32 (momentum
// deviation << (32 - s) plus vref * weight sum, weight sum << (32 - sm)).
template <int DIM, typename AccT>
__device__ __forceinline__ void tile_flush(const DevParams &P, const int *origin,
                                           const AccT *__restrict__ acc, GNode *__restrict__ gout,
                                           uint32_t *__restrict__ flags, uint32_t *touched, uint32_t &natom,
                                           uint32_t *__restrict__ table, const volatile TileScale &ts) {
    constexpr int TN = Geo<DIM>::TN, TS = Geo<DIM>::TS, TB = Geo<DIM>::TB, B = Geo<DIM>::BLK, L = Geo<DIM>::LOG;
    unsigned char *code = reinterpret_cast<unsigned char *>(table + TN);
    if (table) {
        // node index < 1024^3 fits 32 bits; 0xffffffff: outside the grid
        for (int t = threadIdx.x; t < TN; t += PWG) {
            int ijk[DIM];
            const bool ok = tile_node<DIM>(t, origin, P.res, ijk);
            table[t] = ok ? (uint32_t)node_index<DIM>(ijk, P.nb) : 0xffffffffu;
            code[t] = (unsigned char)tile_block_code<DIM>(ijk, origin);
        }
        __syncthreads();
    }
    // lane q takes component q % 4 of tile node q / 4: the four sums of a
    // node are adjacent in memory, so one wave-wide atomic instruction
    // covers whole cache lines (16 nodes) instead of 64 scattered words.
    // PWG is a multiple of 4, so a lane keeps its component c: the 32-bit
    // tile's shift and vref 2^(32 - sm) (exact, |k| <= 2^24) are per lane.
    static_assert(PWG % 4 == 0, "a lane keeps its tile component");
    int sh = 0;
    int32_t k = 0;
    if constexpr (sizeof(AccT) == 4) {
        const int c = threadIdx.x & 3, sm = ts.sm;
        sh = (c == 3) ? 32 - sm : 32 - ts.s;
        if (c < 3) k = (int32_t)ldexpf(ts.vref[c], 32 - sm);
    }
    for (int q = threadIdx.x; q < 4 * TN; q += PWG) {
        const int t = q >> 2, c = q & 3;
        unsigned long long sum;
        if constexpr (sizeof(AccT) == 4) {
            const uint32_t r = acc[c * TS + t];
            if (c == 3) {
                sum = (unsigned long long)r << sh;
            } else {
                const uint32_t wm = acc[3 * TS + t];
                if ((r | wm) == 0u) continue;  // no terms
                sum = ((unsigned long long)(long long)(int32_t)r << sh) +
                      (unsigned long long)((long long)k * (long long)wm);
            }
        } else {
            const unsigned long long raw = acc[c * TS + t];
            if (raw == 0ull) continue;  // no terms (a node with terms has a non-zero offset)
            sum = raw - (acc[3 * TS + t] & RAW_OFFSET_MASK);
        }
        if (sum != 0ull) {
            if (table) {
                const uint32_t id = table[t];
                if (id == 0xffffffffu) continue;  // never reached: contributions stay in-grid
                atomicAdd(gout[id].q + c, sum);
                ++natom;
                touched[code[t]] = 1u;
            } else {
                int ijk[DIM];
                if (!tile_node<DIM>(t, origin, P.res, ijk)) continue;  // never reached, as above
                atomicAdd(gout[node_index<DIM>(ijk, P.nb)].q + c, sum);
                ++natom;
                touched[tile_block_code<DIM>(ijk, origin)] = 1u;
            }
        }
    }
    static_assert(TB - 1 - B <= B, "a tile spans at most three blocks per axis");
    __syncthreads();
    constexpr int NB3 = (DIM == 3) ? 27 : 9;
    if (threadIdx.x < NB3) {
        if (touched[threadIdx.x]) {
            int k = threadIdx.x;
            int64_t blk = 0;
#pragma unroll
            for (int a = DIM - 1; a >= 0; --a) {
                int d = k;
#pragma unroll
                for (int e = 0; e < a; ++e) d /= 3;
                d = d % 3;
                blk = blk * P.nb + (((origin[a] + 1) >> L) + d - 1);
            }
            flags[blk] = 1u;
            touched[threadIdx.x] = 0u;
        }
    }
}

// A context's batch descriptor is never written by a kernel: read through
// the constant address space it stays in scalar registers.
typedef const __attribute__((address_space(4))) BatchDesc *BatchRef;
__device__ __forceinline__ BatchRef batch_ref(const BatchDesc *p) { return (BatchRef)p; }
// The simulation parameters of a descriptor, word by word (scalar loads).
__device__ __forceinline__ DevParams batch_params(BatchRef d) {
    static_assert(sizeof(DevParams) % 4 == 0, "DevParams is a whole number of words");
    typedef const __attribute__((address_space(4))) uint32_t *WordRef;
    const WordRef src = (WordRef)&d->P;
    uint32_t w[sizeof(DevParams) / 4];
#pragma unroll
    for (int k = 0; k < (int)(sizeof(DevParams) / 4); ++k) w[k] = src[k];
    DevParams out;
    __builtin_memcpy(&out, w, sizeof(DevParams));
    return out;
}

// Scene of work-group g in a batched launch (binary search over the
// scenes' first work-groups; the arguments are wave-uniform).
__device__ __forceinline__ int batch_scene(const BatchArgs &a, uint32_t g) {
    int lo = 0, hi = a.count - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.group_begin[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Work-item walk (a group takes one item or several, depending on the grid
// size).  Work-groups are dispatched round-robin over the
// 8 XCDs (each with its own L2), so work-group b runs on XCD b % 8; XCD x
// walks the contiguous range [x*chunk, (x+1)*chunk) of the block-ordered
// items, so spatially adjacent tiles (which share halo nodes) meet in the
// same L2.  The trip count depends only on blockIdx: uniform per group.
// ---------------------------------------------------------------------------
struct ItemWalk {
    uint32_t first, stride, end;
    __device__ ItemWalk(uint32_t nit) : ItemWalk(nit, blockIdx.x, gridDim.x) {}
    // group `bid` of `ngroups` (a multiple of 8, starting at a multiple of 8
    // of the launch, so that bid & 7 is still the XCD)
    __device__ ItemWalk(uint32_t nit, uint32_t bid, uint32_t ngroups) {
        const uint32_t x = bid & 7u, per = ngroups >> 3;
        const uint32_t chunk = (nit + 7u) >> 3;
        first = x * chunk + (bid >> 3);
        stride = per;
        end = min(nit, (x + 1u) * chunk);
    }
};

// Record of a work item's last P2G, read by its next fused substep:
// (v0, dev) with v0 the stored velocity of the item's first particle and
// dev a bound of |q + sum_b a_b o_b - v0| + 2 sum_b |a_b| over its
// particles whose stencil was in the tile: the largest bound about vref
// (per wave in red) plus |v0 - vref|.
template <int DIM>
__device__ __forceinline__ float4 item_record(const float *red, const volatile float *v0,
                                              const volatile TileScale &ts) {
    float r = red[0], sh = 0.0f;
    for (int w = 1; w < PWG / 64; ++w) r = fmaxf(r, red[w]);
#pragma unroll
    for (int a = 0; a < DIM; ++a) sh = fmaxf(sh, fabsf(v0[a] - ts.vref[a]));
    return make_float4(v0[0], v0[1], DIM == 3 ? v0[DIM - 1] : 0.0f, r + sh);
}

// Scales of the 32-bit node tile of a work item of n particles (see
// TileScale) from the item's record of its last P2G (rec, see item_record):
// vref is v0 rounded to a multiple of 2^-(32 - sm), and s the largest
// exponent at which the expected deviation fits under lim: 1.25 x the
// recorded bound (a quarter for growth) plus the rounding of vref, plus a
// floor for an item that moved uniformly at its last P2G (the record is then
// about zero, while this substep adds gravity, dvg = dt |g|, and the
// velocity's quantization, here 2^-6 |vref|).  Only the precision depends
// on this estimate: admission to the tile is checked per particle.
template <int DIM>
__device__ __forceinline__ TileScale tile_scale(int n, float4 rec, float dvg) {
    // binary32 throughout: wb is exact (n <= 4096), the bounds 2^32 - 2^13
    // and 2^31 - 2^13 are exact, sm is checked after the rounded division,
    // and lim_v keeps a 2^-20 margin over the rounding of lim
    constexpr float WMAX = (DIM == 3) ? 0.421875f : 0.5625f;  // largest particle weight, 0.75^DIM
    const float wb = (float)n * WMAX;
    int sm = min(32, ilogbf(4294959104.0f / wb));
    if (ldexpf(wb, sm) > 4294959104.0f) --sm;
    const float lim = 2147475456.0f / wb;
    // |vref| <= 2^(sm - 8) keeps |vref 2^(32 - sm)| <= 2^24 (vref exact in
    // binary32); a velocity beyond that (above 2^12 at least) only sends
    // particles to the global path.  A missing record (negative or NaN
    // bound) gives vref = 0 and a bound of 1 + |v0|.
    const float mlim = ldexpf(1.0f, sm - 8);
    const float v0[3] = {rec.x, rec.y, rec.z};
    const bool known = rec.w >= 0.0f;
    float vref[3] = {0.0f, 0.0f, 0.0f}, shift = 0.0f, mabs = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float m = known ? fminf(fmaxf(v0[a], -mlim), mlim) : 0.0f;  // (a NaN v0 gives -mlim)
        vref[a] = ldexpf(rintf(ldexpf(m, 32 - sm)), sm - 32);  // exact
        shift = fmaxf(shift, fabsf(v0[a] - vref[a]));
        mabs = fmaxf(mabs, fabsf(vref[a]));
    }
    const float dev = known ? 1.25f * (rec.w + shift) + 0x1p-6f * mabs + dvg + 0x1p-12f : 1.0f + shift;
    const int sx = max(0, min(32, ilogbf(lim / dev)));
    TileScale ts;
    ts.s = uni(sx);
    ts.sm = uni(sm);
    ts.lim_v = uni(ldexpf(lim, -sx) * (1.0f - 0x1p-20f));
#pragma unroll
    for (int a = 0; a < 3; ++a) ts.vref[a] = uni(vref[a]);
    return ts;
}

// ---------------------------------------------------------------------------
// P2G of a stored state outside the fused kernel.  iscale == nullptr: exact
// 64-bit tiles (after a sort or an encode); else the 32-bit tiles at the
// scales the fused kernel recorded when it scattered this same state, which
// reproduces its node sums bit for bit (same terms, same admission).  Either
// way each tiled item's record (irec, see tile_scale) is written for the
// next fused substep: in the replay exactly as the fused kernel wrote it, in
// the exact P2G from the estimate of p2g_particle about the velocity of the
// item's first particle.
// ---------------------------------------------------------------------------
template <int DIM, int MAT>
__global__ __launch_bounds__(PWG, PWG_WAVES_PER_EU) void k_p2g(const DevScheme *__restrict__ sch, DevParams Parg, const uint32_t *__restrict__ words,
                                            int64_t cap_arg, const WorkItem *__restrict__ items,
                                            const uint32_t *__restrict__ n_items, GNode *__restrict__ gout,
                                            uint32_t *__restrict__ flags, const TileScale *__restrict__ iscale,
                                            float4 *__restrict__ irec, uint64_t *stats) {
    const DevParams &P = params_ref(Parg);
    const int64_t cap = cap_ref(cap_arg);
    constexpr int TS = Geo<DIM>::TS, D2 = DIM * DIM, NW = PWG / 64;
    __shared__ __align__(16) unsigned long long acc[4 * TS];  // 64-bit tile, or the 32-bit tile in its first half
    uint32_t *acc32 = reinterpret_cast<uint32_t *>(acc);
    __shared__ uint32_t touched[27];
    __shared__ float red[NW];  // per wave: the record's deviation bound
    __shared__ TileScale tsw[NW];  // per wave: the item's tile scales
    volatile TileScale &ts = tsw[threadIdx.x >> 6];
    if (threadIdx.x < 27) touched[threadIdx.x] = 0u;
    const uint32_t nit = *n_items;
    uint32_t fallback = 0, clamped = 0, natom = 0, wide = 0;
    const ItemWalk walk(nit);
    for (uint32_t item = walk.first; item < walk.end; item += walk.stride) {
        const WorkItem it = items[item];
        const bool tiled = it.p1 - it.p0 > sparse_item<DIM>();  // uniform over the group
        const bool t32 = tiled && iscale != nullptr;
        // the item's first particle's velocity (every lane decodes it)
        float v0[DIM];
        dec_field<DIM, 1, float>(&scheme_ref(sch)->f[1], words, cap, (uint32_t)it.p0 * 4u, v0);
        if (__lane_id() == 0) {  // the previous item's reads of this wave's copy are done
            if (t32) {
                const TileScale g = iscale[item];
#pragma unroll
                for (int a = 0; a < 3; ++a) ts.vref[a] = g.vref[a];
                ts.lim_v = g.lim_v;
                ts.s = g.s;
                ts.sm = g.sm;
            } else {
#pragma unroll
                for (int a = 0; a < DIM; ++a) ts.vref[a] = v0[a];  // centre of the exact P2G's estimate
            }
        }
        int origin[DIM];
        tile_origin<DIM>(it.block, P.nb, origin);
        __syncthreads();
        if (tiled)
            for (int t = threadIdx.x; t < 4 * TS; t += PWG) acc[t] = 0ull;
        __syncthreads();
        float rec = 0.0f;
        for (int p = it.p0 + threadIdx.x; p < it.p1; p += PWG) {
            double xd[DIM];
            float v[DIM], C[D2], F[nc3<DIM, MAT>()];
            decode_all<DIM, float, MAT>(sch, words, cap, (uint32_t)p * 4u, xd, v, C, F);
            if (t32)
                p2g_particle<DIM, MAT, true>(P, xd, v, C, F, origin, acc32, gout, flags, fallback, clamped, wide,
                                             tiled, ts, rec);
            else
                p2g_particle<DIM, MAT, true>(P, xd, v, C, F, origin, acc, gout, flags, fallback, clamped, wide,
                                             tiled, ts, rec);
        }
        if (tiled) {
            rec = wave_max(rec);
            if (__lane_id() == 0) red[threadIdx.x >> 6] = rec;
        }
        __syncthreads();
        if (tiled && threadIdx.x == 0) irec[item] = item_record<DIM>(red, v0, ts);
        if (t32) tile_flush<DIM>(P, origin, acc32, gout, flags, touched, natom, nullptr, ts);
        else if (tiled) tile_flush<DIM>(P, origin, acc, gout, flags, touched, natom, nullptr, ts);
    }
    add_stat(stats, ST_FALLBACK, fallback);
    add_stat(stats, ST_CLAMP, clamped);
    add_stat(stats, ST_ATOMICS, natom);
    add_stat(stats, ST_WIDE, wide);
}


// ---------------------------------------------------------------------------
// fused substep: G2P -> update -> dithered encode + store -> P2G (next step)
// ---------------------------------------------------------------------------

// &p[i] as an opaque LDS address (p must point into LDS).  The G2P reads
// below take a base per component and stencil plane (or row, in 2D) and
// small constant offsets from it, which the paired LDS reads (ds_read2,
// offsets up to 255 words) reach from that one register; with the whole
// address visible the compiler would fold the component and plane into each
// pair's offset and, past 255 words, spend an address add per pair.
typedef const __attribute__((address_space(3))) float lds_f32;
__device__ __forceinline__ lds_f32 *lds_base(const float *p, int i) {
    lds_f32 *b = (lds_f32 *)p + i;
    asm volatile("" : "+v"(b));
    return b;
}

// G2P from the LDS tile, separable in the three axes:
// v' = sum_i w v_i and S_b = sum_i w (o_b - f_b) v_i, C' = 4/dx S, computed as
// S_b = sum_i w o_b v_i - f_b v' (o_b in {0, 1, 2}: the o_b = 0 terms drop out).
template <int DIM>
__device__ __forceinline__ void g2p_tile(const float *__restrict__ gv, int l0, const float (*wx)[3],
                                         const float *fx, float *nv, float (*S)[DIM]) {
    constexpr int TB = Geo<DIM>::TB, TN = Geo<DIM>::TN;
    float wo[DIM][3];  // o w_o
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        wo[a][0] = 0.0f;
        wo[a][1] = wx[a][1];
        wo[a][2] = 2.0f * wx[a][2];
    }
    if constexpr (DIM == 3) {
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
            float P00[3] = {0.f, 0.f, 0.f}, P01[3] = {0.f, 0.f, 0.f}, P10[3] = {0.f, 0.f, 0.f};
            lds_f32 *bz[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) bz[a] = lds_base(gv, a * TN + l0 + oz * TB * TB);
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                float R0[3] = {0.f, 0.f, 0.f}, R1[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float vi = bz[a][oy * TB + ox];
                        R0[a] += wx[0][ox] * vi;
                        if (ox > 0) R1[a] += wo[0][ox] * vi;
                    }
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    P00[a] += wx[1][oy] * R0[a];
                    if (oy > 0) P01[a] += wo[1][oy] * R0[a];
                    P10[a] += wx[1][oy] * R1[a];
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nv[a] += wx[2][oz] * P00[a];
                S[0][a] += wx[2][oz] * P10[a];
                S[1][a] += wx[2][oz] * P01[a];
                if (oz > 0) S[2][a] += wo[2][oz] * P00[a];
            }
        }
    } else {
        lds_f32 *bz[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) bz[a] = lds_base(gv, a * TN + l0);
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            float R0[2] = {0.f, 0.f}, R1[2] = {0.f, 0.f};
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float vi = bz[a][oy * TB + ox];
                    R0[a] += wx[0][ox] * vi;
                    if (ox > 0) R1[a] += wo[0][ox] * vi;
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                nv[a] += wx[1][oy] * R0[a];
                S[0][a] += wx[1][oy] * R1[a];
                if (oy > 0) S[1][a] += wo[1][oy] * R0[a];
            }
        }
    }
#pragma unroll
    for (int b = 0; b < DIM; ++b)
#pragma unroll
        for (int a = 0; a < DIM; ++a) S[b][a] -= fx[b] * nv[a];
}

// G2P straight from the grid buffer, for a particle whose stencil left its tile.
template <int DIM>
__device__ __forceinline__ void g2p_global(const GNode *__restrict__ gcur, int nb, const int *base,
                                                     const float (*wx)[3], const float (*wd)[3], float *nv,
                                                     float (*S)[DIM]) {
    constexpr int NST = Geo<DIM>::NST;
#pragma unroll
    for (int st = 0; st < NST; ++st) {
        const int o[3] = {st % 3, (st / 3) % 3, st / 9};
        int ijk[DIM];
        float w = 1.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            ijk[a] = base[a] + o[a];
            w *= wx[a][o[a]];
        }
        const float4 g = node_vel<DIM>(gcur, node_index<DIM>(ijk, nb));
        const float vi[3] = {g.x, g.y, g.z};
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            nv[a] += w * vi[a];
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                float wdb = 1.0f;
#pragma unroll
                for (int c = 0; c < DIM; ++c) wdb *= (c == b) ? wd[c][o[c]] : wx[c][o[c]];
                S[b][a] += wdb * vi[a];
            }
        }
    }
}


// Node tile of the fused kernel and its waves per SIMD.  The scheme-
// specialized build sums in the 32-bit tile at per-item scales (see
// TileScale): with the velocity tile that is 48 KB of LDS in 3D, so three
// work-groups share a CU, and the build fits the 168 VGPRs of three waves
// (its spills sit on the encoder's rare branches).  The generic build, which
// reads the scheme at run time, needs more registers than three waves allow
// and spills more under the 32-bit tile's bookkeeping: it keeps the exact
// 64-bit tile (76 KB) and two waves.  The two builds' node sums differ by the
// 32-bit tile's roundings; each is checked against the oracle.
#ifdef MPMQ_SCHEME_CONST
typedef uint32_t TileAcc;
constexpr int SUBSTEP_WAVES_PER_EU = 3;
#else
typedef unsigned long long TileAcc;
constexpr int SUBSTEP_WAVES_PER_EU = PWG_WAVES_PER_EU;
#endif

// The work items of one scene that a work-group takes (walk), each: the
// velocity tile from gcur, G2P, update, dithered encode and store in place,
// P2G of the stored state into the LDS accumulator tile, and its flush to
// gnxt.  gv / acc / touched: the group's LDS tiles (touched zero on entry).
template <int DIM, bool RS, int MAT>
__device__ __forceinline__ void substep_items(const DevScheme *__restrict__ sch, const DevParams &P, uint32_t *words,
                                              const int64_t cap, const WorkItem *__restrict__ items,
                                              const ItemWalk &walk, const GNode *__restrict__ gcur,
                                              GNode *__restrict__ gnxt, uint32_t *__restrict__ flags, uint32_t step,
                                              int do_p2g, int collect_stats, uint64_t *stats, float *gv,
                                              TileAcc *acc, uint32_t *touched, float *red,
                                              TileScale *__restrict__ iscale, float4 *__restrict__ irec,
                                              TileScale *tsw, float *v0s) {
    constexpr int TB = Geo<DIM>::TB, TN = Geo<DIM>::TN, TS = Geo<DIM>::TS, D2 = DIM * DIM;
    constexpr bool T32 = sizeof(TileAcc) == 4;
    uint32_t fallback = 0, clamped = 0, natom = 0, wide = 0;
    LaneStats ls;
    ls.clear();
    for (uint32_t item = walk.first; item < walk.end; item += walk.stride) {
        const WorkItem it = items[item];
        const bool tiled = it.p1 - it.p0 > sparse_item<DIM>();  // uniform over the group
        int origin[DIM];
        tile_origin<DIM>(it.block, P.nb, origin);
        __syncthreads();
        if (tiled) {
            for (int t = threadIdx.x; t < TN; t += PWG) {
                int ijk[DIM];
                float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
                if (tile_node<DIM>(t, origin, P.res, ijk))
                    g = node_vel<DIM>(gcur, node_index<DIM>(ijk, P.nb));
                gv[t] = g.x;
                gv[TN + t] = g.y;
                if constexpr (DIM == 3) gv[2 * TN + t] = g.z;
            }
            if (do_p2g) {
                static_assert((4 * TS * sizeof(TileAcc)) % sizeof(uint4) == 0, "tile clears in 16-byte stores");
                for (int t = threadIdx.x; t < 4 * TS * (int)sizeof(TileAcc) / (int)sizeof(uint4); t += PWG)
                    reinterpret_cast<uint4 *>(acc)[t] = make_uint4(0u, 0u, 0u, 0u);
            }
        }
        __syncthreads();
        volatile TileScale &ts = tsw[threadIdx.x >> 6];  // the wave's own copy
        if (T32 && tiled && do_p2g) {
            const float dvg = P.dt * fmaxf(fmaxf(fabsf(P.g[0]), fabsf(P.g[1])), fabsf(P.g[2]));
            const TileScale t = tile_scale<DIM>(it.p1 - it.p0, irec[item], dvg);
            if (__lane_id() == 0) {
#pragma unroll
                for (int a = 0; a < 3; ++a) ts.vref[a] = t.vref[a];
                ts.lim_v = t.lim_v;
                ts.s = t.s;
                ts.sm = t.sm;
            }
            if (threadIdx.x == 0) iscale[item] = t;  // for a later P2G of the same state (k_p2g)
        }
        float drec = 0.0f;  // the lane's part of the item's record (see item_record)
#ifdef MPMQ_SCHEME_CONST
        // the rows of x and of slot 3 (the only fields read from the old
        // state) of the next particle are loaded while this one is computed
        constexpr uint32_t RM = field_rows(kSchemeConst.f[0], DIM) | field_rows(kSchemeConst.f[3], nc3<DIM, MAT>());
        uint32_t rec[MAX_WORDS], nrec[MAX_WORDS];
        if (it.p0 + (int)threadIdx.x < it.p1) load_rows<RM>(words, cap, (uint32_t)(it.p0 + threadIdx.x) * 4u, nrec);
#endif
        for (int p = it.p0 + threadIdx.x; p < it.p1; p += PWG) {
            SchemeRef sp = scheme_ref(sch);
            const uint32_t p4 = (uint32_t)p * 4u;
            constexpr int N3 = nc3<DIM, MAT>();
            double xd[DIM];
            float F[N3];
#ifdef MPMQ_SCHEME_CONST
            // (every rec row is a register copy, so decoding waits for no load)
#pragma unroll
            for (int k = 0; k < MAX_WORDS; ++k)
                if (RM & (1u << k)) rec[k] = nrec[k];
            if (p + PWG < it.p1) load_rows<RM>(words, cap, p4 + 4u * PWG, nrec);
            dec_field_src<DIM, 0, double>(&sp->f[0], RegRows{rec}, xd);
            dec_field_src<DIM, fid3<MAT>(), float>(&sp->f[3], RegRows{rec}, F);
#else
            dec_field<DIM, 0, double>(&sp->f[0], words, cap, p4, xd);
            dec_field<DIM, fid3<MAT>(), float>(&sp->f[3], words, cap, p4, F);
#endif
            int base[DIM];
            float fx[DIM], wx[DIM][3];
            stencil_base<DIM>(xd, P.inv_dx_d, P.res, base, fx);
            bool in_tile = tiled;
            int l[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                bspline(fx[a], wx[a]);
                l[a] = base[a] - origin[a];
                in_tile &= (l[a] >= 0) && (l[a] <= TB - 3);
            }
            float nv[DIM], S[DIM][DIM];  // S[b][a]
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                nv[a] = 0.0f;
#pragma unroll
                for (int b = 0; b < DIM; ++b) S[b][a] = 0.0f;
            }
            if (in_tile) {
                const int l0 = (DIM == 3) ? (l[DIM - 1] * TB + l[1]) * TB + l[0] : l[1] * TB + l[0];
                g2p_tile<DIM>(gv, l0, wx, fx, nv, S);
            } else {
                fallback += tiled ? 1u : 0u;
                float wd[DIM][3];  // w (o - f)
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int o = 0; o < 3; ++o) wd[a][o] = wx[a][o] * ((float)o - fx[a]);
                g2p_global<DIM>(gcur, P.nb, base, wx, wd, nv, S);
            }
            // update: x' = x + dt v' (binary64), C' = 4/dx S, F' = (I + dt C') F
            // (fluid: J' = J (1 + dt tr C'))
            double xn[DIM];
            float Cn[D2], Fn[N3];
            {
#pragma clang fp contract(off)
#pragma unroll
                for (int a = 0; a < DIM; ++a) xn[a] = xd[a] + P.dt_d * (double)nv[a];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Cn[a * DIM + b] = 4.0f * P.inv_dx * S[b][a];
            if constexpr (MAT == 1) {
                float tr = 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) tr += Cn[a * DIM + a];
                Fn[0] = F[0] * (1.0f + P.dt * tr);
            } else {
#pragma unroll
                for (int i = 0; i < DIM; ++i)
#pragma unroll
                    for (int j = 0; j < DIM; ++j) {
                        float t = F[i * DIM + j];
#pragma unroll
                        for (int k = 0; k < DIM; ++k) t += P.dt * Cn[i * DIM + k] * F[k * DIM + j];
                        Fn[i * DIM + j] = t;
                    }
            }
            // dithered encode (Eq. 11), streamed in place in placement order
            Draws rnd;
            rnd.init(seed_ref(sch), (uint32_t)p, step, 1u);
            OutStream os{words, cap, p4, 0ull, 0, 0};
            double qx[DIM];
            float qv[DIM], qC[D2], qF[N3];
            encode_record<DIM, RS, MAT>(sch, xn, nv, Cn, Fn, rnd, os, ls, qx, qv, qC, qF);
            if (T32 && p == it.p0)  // lane 0: the stored velocity of the item's first particle
#pragma unroll
                for (int a = 0; a < DIM; ++a) v0s[a] = qv[a];
            // P2G of the stored (quantized) state for the next substep (Eq. 1)
            if (do_p2g)
                p2g_particle<DIM, MAT, false>(P, qx, qv, qC, qF, origin, acc, gnxt, flags, fallback, clamped, wide,
                                              tiled, ts, drec);
        }
        // the item's record for the next substep
        if (T32 && do_p2g && tiled) {
            drec = wave_max(drec);
            if (__lane_id() == 0) red[threadIdx.x >> 6] = drec;
        }
        __syncthreads();
        if (T32 && do_p2g && tiled && threadIdx.x == 0) irec[item] = item_record<DIM>(red, v0s, ts);
        // the velocity tile is free now: it holds the flush's node table
        static_assert(DIM * TN * sizeof(float) >= TN * (sizeof(uint32_t) + 1), "node table fits the velocity tile");
        if (do_p2g && tiled)
            tile_flush<DIM>(P, origin, acc, gnxt, flags, touched, natom, reinterpret_cast<uint32_t *>(gv), ts);
        if (collect_stats) {
            flush_stats(ls, stats);
            ls.clear();
        }
    }
    add_stat(stats, ST_FALLBACK, fallback);
    add_stat(stats, ST_CLAMP, clamped);
    add_stat(stats, ST_ATOMICS, natom);
    add_stat(stats, ST_WIDE, wide);
}


template <int DIM, bool RS, int MAT>
__global__ __launch_bounds__(PWG, SUBSTEP_WAVES_PER_EU) void k_substep(const DevScheme *__restrict__ sch, DevParams Parg, uint32_t *words,
                                                int64_t cap_arg, const WorkItem *__restrict__ items,
                                                const uint32_t *__restrict__ n_items,
                                                const GNode *__restrict__ gcur, GNode *__restrict__ gnxt,
                                                uint32_t *__restrict__ flags, TileScale *__restrict__ iscale,
                                                float4 *__restrict__ irec, uint32_t step, int do_p2g,
                                                int collect_stats, uint64_t *stats) {
    constexpr int TN = Geo<DIM>::TN, TS = Geo<DIM>::TS;
    __shared__ float gv[DIM * TN];
    __shared__ __align__(16) TileAcc acc[4 * TS];
    __shared__ uint32_t touched[27];
    __shared__ float red[PWG / 64];  // per wave: the item record's deviation bound
    __shared__ TileScale tsw[PWG / 64];  // per wave: the item's tile scales
    __shared__ float v0s[3];  // the stored velocity of the item's first particle
    if (threadIdx.x < 27) touched[threadIdx.x] = 0u;
    const ItemWalk walk(*n_items);
    substep_items<DIM, RS, MAT>(sch, params_ref(Parg), words, cap_ref(cap_arg), items, walk, gcur, gnxt, flags,
                                step, do_p2g, collect_stats, stats, gv, acc, touched, red, iscale, irec, tsw, v0s);
}

// Batched substep of several scenes (serving): work-group g belongs to the
// scene i with group_begin[i] <= g < group_begin[i + 1] and walks that
// scene's work items as the per-scene launch would (same arithmetic, the
// scene's own scheme, parameters, buffers, step and Philox key).
template <int DIM, bool RS, int MAT>
__global__ __launch_bounds__(PWG, SUBSTEP_WAVES_PER_EU) void k_substep_batch(const BatchArgs args) {
    constexpr int TN = Geo<DIM>::TN, TS = Geo<DIM>::TS;
    __shared__ float gv[DIM * TN];
    __shared__ __align__(16) TileAcc acc[4 * TS];
    __shared__ uint32_t touched[27];
    __shared__ float red[PWG / 64];  // per wave: the item record's deviation bound
    __shared__ TileScale tsw[PWG / 64];  // per wave: the item's tile scales
    __shared__ float v0s[3];  // the stored velocity of the item's first particle
    if (threadIdx.x < 27) touched[threadIdx.x] = 0u;
    const int i = batch_scene(args, blockIdx.x);
    const BatchRef d = batch_ref(args.desc[i]);
    const DevParams P = batch_params(d);
    const uint32_t g0 = args.group_begin[i];
    const ItemWalk walk(*d->n_items, blockIdx.x - g0, args.group_begin[i + 1] - g0);
    const uint32_t step = args.step[i];
    substep_items<DIM, RS, MAT>(d->scheme, P, d->words, d->cap, d->items, walk, d->grid[step & 1],
                                d->grid[(step & 1) ^ 1], d->flags[(step & 1) ^ 1], step, args.mode[i] & 1,
                                (args.mode[i] >> 1) & 1, d->stats, gv, acc, touched, red, d->iscale, d->irec, tsw,
                                v0s);
}


}  // namespace mpmq
