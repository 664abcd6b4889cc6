// kernels.hip -- gfx950 kernels of the quantized MLS-MPM substep.
//
// Data layout in HBM:
//   packed state  uint32 words[W][cap]          word-major SoA, coalesced
//   grid          GNode node[nblocks][BLK^dim], 32 B: int64 fixed-point
//                 momentum xyz + mass during P2G, float4 velocity|mass after
//                 the grid update; block-major; two buffers (this step's P2G
//                 target and the previous one), plus one "touched" flag per
//                 node block each
//   work items    (block, p0, p1): a sorted block's particles, split in
//                 chunks of at most item_cap
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

__device__ __forceinline__ void flush_stats(const LaneStats &ls, uint64_t *stats) {
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

__global__ void k_fill_u32(uint32_t *p, uint32_t value, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

__global__ void k_gather_u32(const uint32_t *__restrict__ in, const uint32_t *__restrict__ perm,
                             uint32_t *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[perm[i]];
}

__global__ void k_copy_u32(const uint32_t *__restrict__ in, uint32_t *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = in[i];
}

static int grid_for(int64_t n, int per_block = 256) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (g > 65536 * 4) g = 65536 * 4;
    return (int)g;
}

// ---------------------------------------------------------------------------
// encode / decode (float32 SoA <-> packed words)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(WG) void k_encode(const DevScheme *__restrict__ sch, const float *__restrict__ x,
                                               const float *__restrict__ v, const float *__restrict__ C,
                                               const float *__restrict__ F, int64_t n, int64_t cap,
                                               uint32_t *words, uint32_t *__restrict__ ids,
                                               uint32_t step, uint32_t tag, uint64_t *stats) {
    constexpr int D2 = DIM * DIM;
    LaneStats ls;
    ls.clear();
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (p < n) {
        double xv[DIM], qx[DIM];
        float vv[DIM], Cv[D2], Fv[D2], qv[DIM], qC[D2], qF[D2];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            xv[c] = (double)x[c * n + p];
            vv[c] = v[c * n + p];
        }
#pragma unroll
        for (int c = 0; c < D2; ++c) {
            Cv[c] = C[c * n + p];
            Fv[c] = F[c * n + p];
        }
        Draws rnd;
        rnd.init(scheme_ref(sch), (uint32_t)p, step, tag);
        OutStream os{words, cap, (uint32_t)p * 4u, 0ull, 0, 0};
        encode_record<DIM, true>(sch, xv, vv, Cv, Fv, rnd, os, ls, qx, qv, qC, qF);
        if (ids) ids[p] = (uint32_t)p;
    }
    flush_stats(ls, stats);
}

template <int DIM, typename T>
__device__ __forceinline__ void decode_all(const DevScheme *sp, const uint32_t *words, int64_t cap, uint32_t p4,
                                           double *xv, T *vv, T *Cv, T *Fv) {
    SchemeRef s = scheme_ref(sp);
    dec_field<DIM, 0, double>(&s->f[0], words, cap, p4, xv);
    dec_field<DIM, 1, T>(&s->f[1], words, cap, p4, vv);
    dec_field<DIM, 2, T>(&s->f[2], words, cap, p4, Cv);
    dec_field<DIM, 3, T>(&s->f[3], words, cap, p4, Fv);
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_decode(const DevScheme *__restrict__ sch, const uint32_t *__restrict__ words, int64_t n,
                                               int64_t cap, float *__restrict__ x, float *__restrict__ v,
                                               float *__restrict__ C, float *__restrict__ F) {
    constexpr int D2 = DIM * DIM;
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (p >= n) return;
    double xv[DIM], vv[DIM], Cv[D2], Fv[D2];
    decode_all<DIM, double>(sch, words, cap, (uint32_t)p * 4u, xv, vv, Cv, Fv);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        if (x) x[c * n + p] = (float)xv[c];
        if (v) v[c * n + p] = (float)vv[c];
    }
#pragma unroll
    for (int c = 0; c < D2; ++c) {
        if (C) C[c * n + p] = (float)Cv[c];
        if (F) F[c * n + p] = (float)Fv[c];
    }
}

// ---------------------------------------------------------------------------
// particle sort by cell
// key = block * BLK^dim + cell-in-block of the (clamped) base cell (tiled)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(WG) void k_sort_keys(const DevScheme *__restrict__ sch, DevParams P, const uint32_t *__restrict__ words,
                                                  int64_t n, int64_t cap, uint32_t *__restrict__ keys,
                                                  uint32_t *__restrict__ vals, uint32_t *__restrict__ cell_count) {
    constexpr int B = Geo<DIM>::BLK, L = Geo<DIM>::LOG;
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (p >= n) return;
    double xv[DIM];
    dec_field<DIM, 0, double>(&scheme_ref(sch)->f[0], words, cap, (uint32_t)p * 4u, xv);
    int base[DIM];
    float fx[DIM];
    stencil_base<DIM>(xv, P.inv_dx_d, P.res, base, fx);
    uint32_t blk = 0;
#pragma unroll
    for (int a = DIM - 1; a >= 0; --a) blk = blk * (uint32_t)P.nb + (uint32_t)(base[a] >> L);
    // cell within the block in tiles of 64 cells (4x4x4 / 8x8), so that the
    // 64 lanes of a wave hold a compact tile: its LDS node addresses then
    // fall in distinct banks for the G2P reads and the P2G atomics
    uint32_t cib;
    if constexpr (DIM == 3) {
        const uint32_t cx = base[0] & 7, cy = base[1] & 7, cz = base[2] & 7;
        cib = ((((cz >> 2) * 2 + (cy >> 2)) * 2 + (cx >> 2)) << 6) + (((cz & 3) * 4 + (cy & 3)) << 2) + (cx & 3);
    } else {
        const uint32_t cx = base[0] & 15, cy = base[1] & 15;
        cib = ((((cy >> 3) * 2) + (cx >> 3)) << 6) + ((cy & 7) << 3) + (cx & 7);
    }
    const uint32_t key = blk * (uint32_t)Geo<DIM>::CPB + cib;
    keys[p] = key;
    vals[p] = (uint32_t)p;
    atomicAdd(&cell_count[key], 1u);
}

// ---- exclusive scan (uint32), tiles of 4096 ----
constexpr int SCAN_TILE = 4096;

__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *total) {
    __shared__ uint32_t wsum[WG / 64];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t t = __shfl_up(incl, o, 64);
        if (lane >= o) incl += t;
    }
    if (lane == 63) wsum[wv] = incl;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) {
        if (i < wv) off += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return off + incl - v;
}

__global__ __launch_bounds__(WG) void k_scan_reduce(const uint32_t *__restrict__ data, int64_t n,
                                                    uint32_t *__restrict__ partial) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 16;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i)
        if (base + i < n) s += data[base + i];
    uint32_t tot;
    block_exclusive_scan(s, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

__global__ __launch_bounds__(WG) void k_scan_down(uint32_t *__restrict__ data, int64_t n,
                                                  const uint32_t *__restrict__ partial_scanned) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + threadIdx.x * 16;
    uint32_t vals[16];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        vals[i] = (base + i < n) ? data[base + i] : 0u;
        s += vals[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot) + partial_scanned[blockIdx.x];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (base + i < n) data[base + i] = run;
        run += vals[i];
    }
}

// single work-group scan for n <= SCAN_TILE
__global__ __launch_bounds__(WG) void k_scan_single(uint32_t *__restrict__ data, int64_t n) {
    const int64_t base = threadIdx.x * 16;
    uint32_t vals[16];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        vals[i] = (base + i < n) ? data[base + i] : 0u;
        s += vals[i];
    }
    uint32_t tot;
    uint32_t run = block_exclusive_scan(s, &tot);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        if (base + i < n) data[base + i] = run;
        run += vals[i];
    }
}

// ---- stable LSD radix sort pass, 8-bit digits, tiles of 4096 ----
constexpr int RADIX_TILE = 4096;

__global__ __launch_bounds__(WG) void k_radix_hist(const uint32_t *__restrict__ keys, int64_t n, int shift,
                                                   uint32_t *__restrict__ hist, int64_t ntiles) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
#pragma unroll 4
    for (int r = 0; r < RADIX_TILE / WG; ++r) {
        const int64_t e = base + r * WG + threadIdx.x;
        if (e < n) atomicAdd(&h[(keys[e] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(WG) void k_radix_scatter(const uint32_t *__restrict__ kin,
                                                      const uint32_t *__restrict__ vin,
                                                      uint32_t *__restrict__ kout, uint32_t *__restrict__ vout,
                                                      int64_t n, int shift, const uint32_t *__restrict__ offs,
                                                      int64_t ntiles) {
    __shared__ uint32_t run[256];
    __shared__ uint32_t wcnt[WG / 64][256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    run[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) wcnt[i][threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RADIX_TILE;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < RADIX_TILE / WG; ++r) {
        const int64_t e = base + r * WG + threadIdx.x;
        const bool valid = e < n;
        uint32_t key = 0, val = 0, dig = 0;
        if (valid) {
            key = kin[e];
            val = vin[e];
            dig = (key >> shift) & 255u;
        }
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t bm = __ballot(bit);
            match &= bit ? bm : ~bm;
        }
        const uint32_t rank = __popcll(match & lt);
        const bool leader = valid && ((match >> lane) == 1ull);
        if (leader) wcnt[wv][dig] = __popcll(match);
        __syncthreads();
        if (valid) {
            uint32_t pos = run[dig] + rank;
            for (int i = 0; i < wv; ++i) pos += wcnt[i][dig];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int i = 0; i < WG / 64; ++i) {
            add += wcnt[i][threadIdx.x];
            wcnt[i][threadIdx.x] = 0;
        }
        run[threadIdx.x] += add;
        __syncthreads();
    }
}

// ---- layered placement within each block ----
// For block b with cells c (CPB of them, counts n_c, cell starts s_c in the
// cell-sorted order): the particle of rank r in cell c goes to
// block_start + sum_{r' < r} #{c': n_c' > r'} + #{c' < c : n_c' > r}.
template <int DIM>
__global__ __launch_bounds__(WG) void k_layer(const uint32_t *__restrict__ cell_start,
                                              const uint32_t *__restrict__ sorted_vals, int64_t nblocks,
                                              uint32_t *__restrict__ perm, uint32_t *__restrict__ block_items,
                                              int item_cap) {
    constexpr int CPB = Geo<DIM>::CPB, PER = CPB / WG;
    __shared__ uint32_t smax[WG / 64];
    const int64_t b = blockIdx.x;
    const uint32_t bstart = cell_start[b * CPB];
    const uint32_t bend = cell_start[(b + 1) * CPB];
    if (threadIdx.x == 0) block_items[b] = (bend - bstart + item_cap - 1) / item_cap;
    if (b == 0 && threadIdx.x == 0) block_items[nblocks] = 0u;
    if (bend == bstart) return;
    uint32_t cnt[PER], cst[PER];
    uint32_t mx = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
        const int c = threadIdx.x * PER + i;
        cst[i] = cell_start[b * CPB + c];
        cnt[i] = cell_start[b * CPB + c + 1] - cst[i];
        mx = max(mx, cnt[i]);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    uint32_t layers = 0;
#pragma unroll
    for (int i = 0; i < WG / 64; ++i) layers = max(layers, smax[i]);
    uint32_t off = bstart;
    for (uint32_t r = 0; r < layers; ++r) {
        uint32_t mine = 0;
#pragma unroll
        for (int i = 0; i < PER; ++i) mine += (cnt[i] > r) ? 1u : 0u;
        uint32_t tot;
        uint32_t pos = off + block_exclusive_scan(mine, &tot);
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            if (cnt[i] > r) {
                perm[pos] = sorted_vals[cst[i] + r];
                ++pos;
            }
        }
        off += tot;
    }
}

__global__ __launch_bounds__(WG) void k_items(const uint32_t *__restrict__ cell_start,
                                              const uint32_t *__restrict__ item_off, int64_t nblocks, int cpb,
                                              int item_cap, WorkItem *__restrict__ items,
                                              uint32_t *__restrict__ n_items) {
    const int64_t b = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (b == nblocks) *n_items = item_off[nblocks];
    if (b >= nblocks) return;
    const uint32_t s0 = cell_start[b * cpb], s1 = cell_start[(b + 1) * cpb];
    uint32_t o = item_off[b];
    for (uint32_t p = s0; p < s1; p += (uint32_t)item_cap, ++o) {
        WorkItem it;
        it.block = (int32_t)b;
        it.p0 = (int32_t)p;
        it.p1 = (int32_t)min(p + (uint32_t)item_cap, s1);
        it.pad = 0;
        items[o] = it;
    }
}

// Fixed-point conversion: round(v * 2^32) as two's complement int64 for
// |v| < 2^19, via binary64: fma(w, x, 1.5*2^52) puts the rounded integer in
// the low mantissa bits (exponent field constant), the subtraction removes
// the offset.  w * x carries the 2^32 scale already.
__device__ __forceinline__ unsigned long long fixp(double w, double xs) {
    return (unsigned long long)__double_as_longlong(fma(w, xs, FIX_MAGIC)) - FIX_MAGIC_BITS;
}

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
        double wt = 1.0;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            ijk[a] = base[a] + o[a];
            wt *= w[a][o[a]];
        }
        unsigned long long *g = gout[node_index<DIM>(ijk, P.nb)].q;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            double val = q[a];
#pragma unroll
            for (int b = 0; b < DIM; ++b) val += ac[b][a] * (double)o[b];
            atomicAdd(g + a, fixp(wt, val));
        }
        atomicAdd(g + 3, fixp(wt, FIX_ONE));
        flags[block_of<DIM>(ijk, P.nb)] = 1u;
    }
}

// ---------------------------------------------------------------------------
// P2G of one particle from its decoded (quantized) state.  Node i receives,
// per unit particle mass, w_i (v + (A/m)(x_i - x_p)) and w_i, accumulated as
// exact 64-bit fixed point (LDS integer atomics: float LDS atomics are an
// order of magnitude slower on this part, and integer sums are
// order-independent).
// ---------------------------------------------------------------------------
template <int DIM>
__device__ __forceinline__ void p2g_particle(const DevParams &P, const double *xd, const float *v,
                                             const float *C, const float *F, const int *origin,
                                             unsigned long long *__restrict__ acc, GNode *__restrict__ gout,
                                             uint32_t *__restrict__ flags, uint32_t &fallback) {
    constexpr int TB = Geo<DIM>::TB, TN = Geo<DIM>::TN, D2 = DIM * DIM;
    constexpr float LIM = 4096.0f;  // |q|, |a_b| <= 2^12 keeps every term below 2^19
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
    // fixed-corotated Kirchhoff stress tau = 2 mu (F - R) F^T + lambda J (J-1) I
    float R[D2];
    float J;
    if constexpr (DIM == 2) {
        polar2(F, R);
        J = F[0] * F[3] - F[1] * F[2];
    } else {
        polar3(F, R);
        J = F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
            F[2] * (F[3] * F[7] - F[4] * F[6]);
    }
    // A / m_p = -4 dt / (rho dx^2) tau + C
    float Am[D2];
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
    // node value = w (q + sum_b a_b o_b), q = v - (A/m) f dx, a_b = (A/m)[:, b] dx, scaled by 2^32
    double q[DIM], ac[DIM][DIM];  // ac[b][a]
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float t = v[a];
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            const float ab = fminf(fmaxf(Am[a * DIM + b] * P.dx, -LIM), LIM);
            ac[b][a] = (double)ab * FIX_ONE;
            t -= ab * fx[b];
        }
        q[a] = (double)fminf(fmaxf(t, -LIM), LIM) * FIX_ONE;
    }
    bool in_tile = true;
    int l[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        l[a] = base[a] - origin[a];
        in_tile &= (l[a] >= 0) && (l[a] <= TB - 3);
    }
    if (in_tile) {
        const int l0 = (DIM == 3) ? (l[DIM - 1] * TB + l[1]) * TB + l[0] : l[1] * TB + l[0];
        // node values stepped along each axis (q + sum_b a_b o_b by additions)
        if constexpr (DIM == 3) {
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
                        const double wt = wzy * w[0][ox];
                        const int idx = l0 + (oz * TB + oy) * TB + ox;
#pragma unroll
                        for (int a = 0; a < 3; ++a) atomicAdd(&acc[a * TN + idx], fixp(wt, val[a]));
                        atomicAdd(&acc[3 * TN + idx], fixp(wt, FIX_ONE));
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
                double val[2] = {vy[0], vy[1]};
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    if (ox > 0)
#pragma unroll
                        for (int a = 0; a < 2; ++a) val[a] += ac[0][a];
                    const double wt = w[1][oy] * w[0][ox];
                    const int idx = l0 + oy * TB + ox;
#pragma unroll
                    for (int a = 0; a < 2; ++a) atomicAdd(&acc[a * TN + idx], fixp(wt, val[a]));
                    atomicAdd(&acc[3 * TN + idx], fixp(wt, FIX_ONE));
                }
            }
        }
    } else {
        fallback += 1;
        p2g_global<DIM>(P, base, w, q, ac, gout, flags);
    }
}

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

template <int DIM>
__device__ __forceinline__ void tile_flush(const DevParams &P, const int *origin,
                                           const unsigned long long *__restrict__ acc, GNode *__restrict__ gout,
                                           uint32_t *__restrict__ flags) {
    constexpr int TN = Geo<DIM>::TN;
    for (int t = threadIdx.x; t < TN; t += WG) {
        const unsigned long long a0 = acc[t], a1 = acc[TN + t], a2 = acc[2 * TN + t], m = acc[3 * TN + t];
        if ((a0 | a1 | a2 | m) != 0ull) {
            int ijk[DIM];
            if (!tile_node<DIM>(t, origin, P.res, ijk)) continue;  // never reached: contributions stay in-grid
            unsigned long long *g = gout[node_index<DIM>(ijk, P.nb)].q;
            atomicAdd(g + 0, a0);
            atomicAdd(g + 1, a1);
            if (DIM == 3) atomicAdd(g + 2, a2);
            atomicAdd(g + 3, m);
            flags[block_of<DIM>(ijk, P.nb)] = 1u;
        }
    }
}

// ---------------------------------------------------------------------------
// Persistent work-item walk.  Work-groups are dispatched round-robin over the
// 8 XCDs (each with its own L2), so work-group b runs on XCD b % 8; XCD x
// walks the contiguous range [x*chunk, (x+1)*chunk) of the block-ordered
// items, so spatially adjacent tiles (which share halo nodes) meet in the
// same L2.  The trip count depends only on blockIdx: uniform per group.
// ---------------------------------------------------------------------------
struct ItemWalk {
    uint32_t first, stride, end;
    __device__ ItemWalk(uint32_t nit) {
        const uint32_t x = blockIdx.x & 7u, per = gridDim.x >> 3;
        const uint32_t chunk = (nit + 7u) >> 3;
        first = x * chunk + (blockIdx.x >> 3);
        stride = per;
        end = min(nit, (x + 1u) * chunk);
    }
};

// ---------------------------------------------------------------------------
// bootstrap P2G from the packed state (after a sort or an encode)
// ---------------------------------------------------------------------------
template <int DIM>
__global__ __launch_bounds__(WG) void k_p2g(const DevScheme *__restrict__ sch, DevParams P, const uint32_t *__restrict__ words,
                                            int64_t cap, const WorkItem *__restrict__ items,
                                            const uint32_t *__restrict__ n_items, GNode *__restrict__ gout,
                                            uint32_t *__restrict__ flags, uint64_t *stats) {
    constexpr int TN = Geo<DIM>::TN, D2 = DIM * DIM;
    __shared__ unsigned long long acc[4 * TN];
    const uint32_t nit = *n_items;
    uint32_t fallback = 0;
    const ItemWalk walk(nit);
    for (uint32_t item = walk.first; item < walk.end; item += walk.stride) {
        const WorkItem it = items[item];
        int origin[DIM];
        tile_origin<DIM>(it.block, P.nb, origin);
        __syncthreads();
        for (int t = threadIdx.x; t < 4 * TN; t += WG) acc[t] = 0ull;
        __syncthreads();
        for (int p = it.p0 + threadIdx.x; p < it.p1; p += WG) {
            double xd[DIM];
            float v[DIM], C[D2], F[D2];
            decode_all<DIM, float>(sch, words, cap, (uint32_t)p * 4u, xd, v, C, F);
            p2g_particle<DIM>(P, xd, v, C, F, origin, acc, gout, flags, fallback);
        }
        __syncthreads();
        tile_flush<DIM>(P, origin, acc, gout, flags);
    }
    add_stat(stats, ST_FALLBACK, fallback);
}

// ---------------------------------------------------------------------------
// grid update: fixed-point sums -> velocity (mom/m + dt g, wall rule) in
// place; clears the other buffer's touched blocks
// ---------------------------------------------------------------------------
__device__ __forceinline__ double from_fix(unsigned long long v) { return (double)(long long)v; }

template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_update(DevParams P, GNode *__restrict__ gcur,
                                                    GNode *__restrict__ gnxt, uint32_t *__restrict__ fcur,
                                                    uint32_t *__restrict__ fnxt, int64_t nblocks, uint64_t *stats) {
    constexpr int B = Geo<DIM>::BLK, CPB = Geo<DIM>::CPB, L = Geo<DIM>::LOG;
    const int64_t b = blockIdx.x;
    const bool tc = fcur[b] != 0u, tn = fnxt[b] != 0u;
    if (!tc && !tn) return;
    int bc[3] = {0, 0, 0};
    bc[0] = (int)(b % P.nb);
    if constexpr (DIM == 3) {
        bc[1] = (int)((b / P.nb) % P.nb);
        bc[2] = (int)(b / ((int64_t)P.nb * P.nb));
    } else {
        bc[1] = (int)(b / P.nb);
    }
    uint32_t active = 0;
    for (int l = threadIdx.x; l < CPB; l += WG) {
        const int64_t idx = (b << (DIM * L)) + l;
        if (tc) {
            const GNode g = gcur[idx];
            const double m = from_fix(g.q[3]);
            float vel[3] = {0.0f, 0.0f, 0.0f};
            if (m > 0.0) {
                ++active;
                int ijk[3];
                ijk[0] = bc[0] * B + (l & (B - 1));
                ijk[1] = bc[1] * B + ((l >> L) & (B - 1));
                ijk[2] = (DIM == 3) ? bc[2] * B + (l >> (2 * L)) : 0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    float va = (float)(from_fix(g.q[a]) / m) + P.dt * P.g[a];
                    if (ijk[a] < P.bound && va < 0.0f) va = 0.0f;
                    if (ijk[a] >= P.res - P.bound && va > 0.0f) va = 0.0f;
                    vel[a] = va;
                }
            }
            const float mass = m > 0.0 ? (float)(m * (1.0 / FIX_ONE)) * P.p_mass : 0.0f;
            reinterpret_cast<float4 *>(gcur + idx)[0] = make_float4(vel[0], vel[1], vel[2], mass);
        }
        if (tn) {
            ulonglong4 z;
            z.x = z.y = z.z = z.w = 0ull;
            reinterpret_cast<ulonglong4 *>(gnxt + idx)[0] = z;
        }
    }
    if (tn && threadIdx.x == 0) fnxt[b] = 0u;
    add_stat(stats, ST_ACTIVE, active);
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_clear_touched(GNode *__restrict__ g, uint32_t *__restrict__ flags,
                                                      int64_t nblocks) {
    constexpr int CPB = Geo<DIM>::CPB, L = Geo<DIM>::LOG;
    const int64_t b = blockIdx.x;
    if (flags[b] == 0u) return;
    for (int l = threadIdx.x; l < CPB; l += WG) {
        ulonglong4 z;
        z.x = z.y = z.z = z.w = 0ull;
        reinterpret_cast<ulonglong4 *>(g + (b << (DIM * L)) + l)[0] = z;
    }
    if (threadIdx.x == 0) flags[b] = 0u;
}

// ---------------------------------------------------------------------------
// fused substep: G2P -> update -> dithered encode + store -> P2G (next step)
// ---------------------------------------------------------------------------

// G2P from the LDS tile, separable in the three axes:
// v' = sum_i w v_i and S_b = sum_i w (o_b - f_b) v_i, C' = 4/dx S.
template <int DIM>
__device__ __forceinline__ void g2p_tile(const float *__restrict__ gv, int l0, const float (*wx)[3],
                                         const float (*wd)[3], float *nv, float (*S)[DIM]) {
    constexpr int TB = Geo<DIM>::TB, TN = Geo<DIM>::TN;
    if constexpr (DIM == 3) {
#pragma unroll
        for (int oz = 0; oz < 3; ++oz) {
            float P00[3] = {0.f, 0.f, 0.f}, P01[3] = {0.f, 0.f, 0.f}, P10[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int oy = 0; oy < 3; ++oy) {
                float R0[3] = {0.f, 0.f, 0.f}, R1[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int ox = 0; ox < 3; ++ox) {
                    const int idx = l0 + (oz * TB + oy) * TB + ox;
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const float vi = gv[a * TN + idx];
                        R0[a] += wx[0][ox] * vi;
                        R1[a] += wd[0][ox] * vi;
                    }
                }
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    P00[a] += wx[1][oy] * R0[a];
                    P01[a] += wd[1][oy] * R0[a];
                    P10[a] += wx[1][oy] * R1[a];
                }
            }
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                nv[a] += wx[2][oz] * P00[a];
                S[0][a] += wx[2][oz] * P10[a];
                S[1][a] += wx[2][oz] * P01[a];
                S[2][a] += wd[2][oz] * P00[a];
            }
        }
    } else {
#pragma unroll
        for (int oy = 0; oy < 3; ++oy) {
            float R0[2] = {0.f, 0.f}, R1[2] = {0.f, 0.f};
#pragma unroll
            for (int ox = 0; ox < 3; ++ox) {
                const int idx = l0 + oy * TB + ox;
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const float vi = gv[a * TN + idx];
                    R0[a] += wx[0][ox] * vi;
                    R1[a] += wd[0][ox] * vi;
                }
            }
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                nv[a] += wx[1][oy] * R0[a];
                S[0][a] += wx[1][oy] * R1[a];
                S[1][a] += wd[1][oy] * R0[a];
            }
        }
    }
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
        const float4 g = reinterpret_cast<const float4 *>(gcur + node_index<DIM>(ijk, nb))[0];
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

template <int DIM, bool RS>
__global__ __launch_bounds__(WG, 2) void k_substep(const DevScheme *__restrict__ sch, DevParams P, uint32_t *words,
                                                int64_t cap, const WorkItem *__restrict__ items,
                                                const uint32_t *__restrict__ n_items,
                                                const GNode *__restrict__ gcur, GNode *__restrict__ gnxt,
                                                uint32_t *__restrict__ flags, uint32_t step, int do_p2g,
                                                int collect_stats, uint64_t *stats) {
    constexpr int TB = Geo<DIM>::TB, TN = Geo<DIM>::TN, D2 = DIM * DIM;
    __shared__ float gv[DIM * TN];
    __shared__ unsigned long long acc[4 * TN];
    const uint32_t nit = *n_items;
    uint32_t fallback = 0;
    LaneStats ls;
    ls.clear();
    const ItemWalk walk(nit);
    for (uint32_t item = walk.first; item < walk.end; item += walk.stride) {
        const WorkItem it = items[item];
        int origin[DIM];
        tile_origin<DIM>(it.block, P.nb, origin);
        __syncthreads();
        for (int t = threadIdx.x; t < TN; t += WG) {
            int ijk[DIM];
            float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (tile_node<DIM>(t, origin, P.res, ijk))
                g = reinterpret_cast<const float4 *>(gcur + node_index<DIM>(ijk, P.nb))[0];
            gv[t] = g.x;
            gv[TN + t] = g.y;
            if constexpr (DIM == 3) gv[2 * TN + t] = g.z;
        }
        if (do_p2g)
            for (int t = threadIdx.x; t < 4 * TN; t += WG) acc[t] = 0ull;
        __syncthreads();
        for (int p = it.p0 + threadIdx.x; p < it.p1; p += WG) {
            SchemeRef sp = scheme_ref(sch);
            const uint32_t p4 = (uint32_t)p * 4u;
            double xd[DIM];
            float F[D2];
            dec_field<DIM, 0, double>(&sp->f[0], words, cap, p4, xd);
            dec_field<DIM, 3, float>(&sp->f[3], words, cap, p4, F);
            int base[DIM];
            float fx[DIM], wx[DIM][3], wd[DIM][3];
            stencil_base<DIM>(xd, P.inv_dx_d, P.res, base, fx);
            bool in_tile = true;
            int l[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                bspline(fx[a], wx[a]);
#pragma unroll
                for (int o = 0; o < 3; ++o) wd[a][o] = wx[a][o] * ((float)o - fx[a]);
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
                g2p_tile<DIM>(gv, l0, wx, wd, nv, S);
            } else {
                fallback += 1;
                g2p_global<DIM>(gcur, P.nb, base, wx, wd, nv, S);
            }
            // update: x' = x + dt v' (binary64), C' = 4/dx S, F' = (I + dt C') F
            double xn[DIM];
            float Cn[D2], Fn[D2];
            {
#pragma clang fp contract(off)
#pragma unroll
                for (int a = 0; a < DIM; ++a) xn[a] = xd[a] + P.dt_d * (double)nv[a];
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b = 0; b < DIM; ++b) Cn[a * DIM + b] = 4.0f * P.inv_dx * S[b][a];
#pragma unroll
            for (int i = 0; i < DIM; ++i)
#pragma unroll
                for (int j = 0; j < DIM; ++j) {
                    float t = F[i * DIM + j];
#pragma unroll
                    for (int k = 0; k < DIM; ++k) t += P.dt * Cn[i * DIM + k] * F[k * DIM + j];
                    Fn[i * DIM + j] = t;
                }
            // dithered encode (Eq. 11), streamed in place in placement order
            Draws rnd;
            rnd.init(sp, (uint32_t)p, step, 1u);
            OutStream os{words, cap, p4, 0ull, 0, 0};
            double qx[DIM];
            float qv[DIM], qC[D2], qF[D2];
            encode_record<DIM, RS>(sch, xn, nv, Cn, Fn, rnd, os, ls, qx, qv, qC, qF);
            // P2G of the stored (quantized) state for the next substep (Eq. 1)
            if (do_p2g) p2g_particle<DIM>(P, qx, qv, qC, qF, origin, acc, gnxt, flags, fallback);
        }
        __syncthreads();
        if (do_p2g) tile_flush<DIM>(P, origin, acc, gnxt, flags);
        if (collect_stats) {
            flush_stats(ls, stats);
            ls.clear();
        }
    }
    add_stat(stats, ST_FALLBACK, fallback);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
#define MPMQ_DISPATCH(dim, wm, KERNEL, GRID, ...)                                                \
    do {                                                                                          \
        (void)(wm);                                                                               \
        if ((dim) == 3) hipLaunchKernelGGL((KERNEL<3>), GRID, dim3(WG), 0, st, __VA_ARGS__);      \
        else hipLaunchKernelGGL((KERNEL<2>), GRID, dim3(WG), 0, st, __VA_ARGS__);                 \
    } while (0)

#define MPMQ_DISPATCH2(dim, KERNEL, FLAG, GRID, ...)                                                \
    do {                                                                                            \
        if ((dim) == 3) hipLaunchKernelGGL((KERNEL<3, FLAG>), GRID, dim3(WG), 0, st, __VA_ARGS__);  \
        else hipLaunchKernelGGL((KERNEL<2, FLAG>), GRID, dim3(WG), 0, st, __VA_ARGS__);             \
    } while (0)

static dim3 pgrid(int64_t n) { return dim3((unsigned)((n + WG - 1) / WG)); }

hipError_t launch_encode(int dim, int wm, const DevScheme *s, const float *x, const float *v, const float *C,
                         const float *F, int64_t n, int64_t cap, uint32_t *words, uint32_t *ids, uint32_t step,
                         uint32_t tag, uint64_t *stats, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    MPMQ_DISPATCH(dim, wm, k_encode, pgrid(n), s, x, v, C, F, n, cap, words, ids, step, tag, stats);
    return hipGetLastError();
}

hipError_t launch_decode(int dim, int wm, const DevScheme *s, const uint32_t *words, int64_t n, int64_t cap,
                         float *x, float *v, float *C, float *F, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    MPMQ_DISPATCH(dim, wm, k_decode, pgrid(n), s, words, n, cap, x, v, C, F);
    return hipGetLastError();
}

hipError_t launch_sort_keys(int dim, int wm, const DevScheme *s, const DevParams &p, const uint32_t *words,
                            int64_t n, int64_t cap, uint32_t *keys, uint32_t *vals, uint32_t *cell_count,
                            hipStream_t st) {
    if (n <= 0) return hipSuccess;
    MPMQ_DISPATCH(dim, wm, k_sort_keys, pgrid(n), s, p, words, n, cap, keys, vals, cell_count);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n)), dim3(256), 0, st, p, value, n);
    return hipGetLastError();
}

hipError_t launch_gather_u32(const uint32_t *in, const uint32_t *perm, uint32_t *out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(n)), dim3(256), 0, st, in, perm, out, n);
    return hipGetLastError();
}

hipError_t launch_copy_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_u32, dim3(grid_for(n)), dim3(256), 0, st, in, out, n);
    return hipGetLastError();
}

// Exclusive scan in place; tmp holds the partial sums of every level.
hipError_t launch_scan(uint32_t *data, int64_t n, uint32_t *tmp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (n <= SCAN_TILE) {
        hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(WG), 0, st, data, n);
        return hipGetLastError();
    }
    const int64_t tiles = (n + SCAN_TILE - 1) / SCAN_TILE;
    hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)tiles), dim3(WG), 0, st, data, n, tmp);
    hipError_t e = launch_scan(tmp, tiles, tmp + tiles, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_scan_down, dim3((unsigned)tiles), dim3(WG), 0, st, data, n, tmp);
    return hipGetLastError();
}

hipError_t launch_radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout, int64_t n,
                             int shift, uint32_t *hist, uint32_t *scan_tmp, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int64_t tiles = (n + RADIX_TILE - 1) / RADIX_TILE;
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)tiles), dim3(WG), 0, st, kin, n, shift, hist, tiles);
    hipError_t e = launch_scan(hist, 256 * tiles, scan_tmp, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)tiles), dim3(WG), 0, st, kin, vin, kout, vout, n, shift,
                       hist, tiles);
    return hipGetLastError();
}

hipError_t launch_layer(int dim, const uint32_t *cell_start, const uint32_t *sorted_vals, int64_t nblocks,
                        uint32_t *perm, uint32_t *block_items, int item_cap, hipStream_t st) {
    if (dim == 3)
        hipLaunchKernelGGL(k_layer<3>, dim3((unsigned)nblocks), dim3(WG), 0, st, cell_start, sorted_vals, nblocks,
                           perm, block_items, item_cap);
    else
        hipLaunchKernelGGL(k_layer<2>, dim3((unsigned)nblocks), dim3(WG), 0, st, cell_start, sorted_vals, nblocks,
                           perm, block_items, item_cap);
    return hipGetLastError();
}

hipError_t launch_items(const uint32_t *cell_start, const uint32_t *item_off, int64_t nblocks, int cpb,
                        int item_cap, WorkItem *items, uint32_t *n_items, hipStream_t st) {
    hipLaunchKernelGGL(k_items, pgrid(nblocks + 1), dim3(WG), 0, st, cell_start, item_off, nblocks, cpb, item_cap,
                       items, n_items);
    return hipGetLastError();
}

hipError_t launch_p2g(int dim, int wm, const DevScheme *s, const DevParams &p, const uint32_t *words, int64_t cap,
                      const WorkItem *items, const uint32_t *n_items, int grid, GNode *gout, uint32_t *flags_out,
                      uint64_t *stats, hipStream_t st) {
    MPMQ_DISPATCH(dim, wm, k_p2g, dim3(grid), s, p, words, cap, items, n_items, gout, flags_out, stats);
    return hipGetLastError();
}

hipError_t launch_grid_update(int dim, const DevParams &p, GNode *gcur, GNode *gnxt, uint32_t *flags_cur,
                              uint32_t *flags_nxt, int64_t nblocks, uint64_t *stats, hipStream_t st) {
    if (dim == 3)
        hipLaunchKernelGGL(k_grid_update<3>, dim3((unsigned)nblocks), dim3(WG), 0, st, p, gcur, gnxt, flags_cur,
                           flags_nxt, nblocks, stats);
    else
        hipLaunchKernelGGL(k_grid_update<2>, dim3((unsigned)nblocks), dim3(WG), 0, st, p, gcur, gnxt, flags_cur,
                           flags_nxt, nblocks, stats);
    return hipGetLastError();
}

hipError_t launch_clear_touched(int dim, GNode *g, uint32_t *flags, int64_t nblocks, hipStream_t st) {
    if (dim == 3)
        hipLaunchKernelGGL(k_clear_touched<3>, dim3((unsigned)nblocks), dim3(WG), 0, st, g, flags, nblocks);
    else
        hipLaunchKernelGGL(k_clear_touched<2>, dim3((unsigned)nblocks), dim3(WG), 0, st, g, flags, nblocks);
    return hipGetLastError();
}

hipError_t launch_substep(int dim, int wm, const DevScheme *s, const DevParams &p, uint32_t *words, int64_t cap,
                          const WorkItem *items, const uint32_t *n_items, int grid, const GNode *gcur,
                          GNode *gnxt, uint32_t *flags_nxt, uint32_t step, int do_p2g, int collect_stats,
                          int round_stats, uint64_t *stats, hipStream_t st) {
    if (round_stats)
        MPMQ_DISPATCH2(dim, k_substep, true, dim3(grid), s, p, words, cap, items, n_items, gcur, gnxt, flags_nxt,
                       step, do_p2g, collect_stats, stats);
    else
        MPMQ_DISPATCH2(dim, k_substep, false, dim3(grid), s, p, words, cap, items, n_items, gcur, gnxt, flags_nxt,
                       step, do_p2g, collect_stats, stats);
    return hipGetLastError();
}

}  // namespace mpmq
