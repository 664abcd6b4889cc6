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
#include "substep.hpp"

namespace mpmq {

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
// Grid-stride over particles; statistics are summed per lane in 32-bit
// counters and flushed once per work-group (per-wave flushes of a few shared
// counters would serialize in the L2).
template <int DIM, int MAT>
__global__ __launch_bounds__(WG) void k_encode(const DevScheme *__restrict__ sch, const float *__restrict__ x,
                                               const float *__restrict__ v, const float *__restrict__ C,
                                               const float *__restrict__ F, int64_t n, int64_t cap,
                                               uint32_t *words, uint32_t *__restrict__ ids,
                                               uint32_t step, uint32_t tag, uint64_t *stats) {
    constexpr int D2 = DIM * DIM, N3 = nc3<DIM, MAT>();
    uint32_t cnt[16];  // up[4], down[4], sat[4], nan[4]
#pragma unroll
    for (int i = 0; i < 16; ++i) cnt[i] = 0u;
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < n; p += (int64_t)gridDim.x * WG) {
        LaneStats ls;
        ls.clear();
        double xv[DIM], qx[DIM];
        float vv[DIM], Cv[D2], Fv[N3], qv[DIM], qC[D2], qF[N3];
#pragma unroll
        for (int c = 0; c < DIM; ++c) {
            xv[c] = (double)x[c * n + p];
            vv[c] = v[c * n + p];
        }
#pragma unroll
        for (int c = 0; c < D2; ++c) Cv[c] = C[c * n + p];
#pragma unroll
        for (int c = 0; c < N3; ++c) Fv[c] = F[c * n + p];
        Draws rnd;
        rnd.init(seed_ref(sch), (uint32_t)p, step, tag);
        OutStream os{words, cap, (uint32_t)p * 4u, 0ull, 0, 0};
        encode_record<DIM, true, MAT>(sch, xv, vv, Cv, Fv, rnd, os, ls, qx, qv, qC, qF);
        if (ids) ids[p] = (uint32_t)p;
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            cnt[f] += ls.ud[f] & 0xffffu;
            cnt[4 + f] += ls.ud[f] >> 16;
            cnt[8 + f] += (ls.sat >> (8 * f)) & 0xffu;
            cnt[12 + f] += (ls.nan >> (8 * f)) & 0xffu;
        }
    }
    __shared__ uint32_t part[WG / 64][16];
#pragma unroll
    for (int i = 0; i < 16; ++i) {
        const uint32_t w = wave_sum(cnt[i]);
        if (__lane_id() == 0) part[threadIdx.x >> 6][i] = w;
    }
    __syncthreads();
    if (threadIdx.x < 16) {
        uint32_t tot = 0;
#pragma unroll
        for (int k = 0; k < WG / 64; ++k) tot += part[k][threadIdx.x];
        const int f = threadIdx.x & 3, kind = threadIdx.x >> 2;
        const int slot = kind == 0 ? ST_UP : kind == 1 ? ST_DOWN : kind == 2 ? ST_SAT : ST_NAN;
        if (tot) atomicAdd((unsigned long long *)&stats[slot + f], (unsigned long long)tot);
    }
}


template <int DIM, int MAT>
__global__ __launch_bounds__(WG) void k_decode(const DevScheme *__restrict__ sch, const uint32_t *__restrict__ words, int64_t n,
                                               int64_t cap, float *__restrict__ x, float *__restrict__ v,
                                               float *__restrict__ C, float *__restrict__ F) {
    constexpr int D2 = DIM * DIM, N3 = nc3<DIM, MAT>();
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (p >= n) return;
    double xv[DIM], vv[DIM], Cv[D2], Fv[N3];
    decode_all<DIM, double, MAT>(sch, words, cap, (uint32_t)p * 4u, xv, vv, Cv, Fv);
#pragma unroll
    for (int c = 0; c < DIM; ++c) {
        if (x) x[c * n + p] = (float)xv[c];
        if (v) v[c * n + p] = (float)vv[c];
    }
#pragma unroll
    for (int c = 0; c < D2; ++c)
        if (C) C[c * n + p] = (float)Cv[c];
#pragma unroll
    for (int c = 0; c < N3; ++c)
        if (F) F[c * n + p] = (float)Fv[c];
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

// ---------------------------------------------------------------------------
// grid update: fixed-point sums -> velocity (mom/m + dt g, wall rule) in
// place; clears the other buffer's touched blocks
// ---------------------------------------------------------------------------
__device__ __forceinline__ double from_fix(unsigned long long v) { return (double)(long long)v; }

// Persistent: work-group g of ngroups walks node blocks g, g + ngroups, ...;
// a block flagged in fcur gets its fixed-point sums turned into float4
// (v, m) in place, a block flagged in fnxt is cleared for the next P2G.  One
// count atomic per work-group.
template <int DIM>
__device__ __forceinline__ void grid_update_blocks(const DevParams &P, GNode *__restrict__ gcur,
                                                   GNode *__restrict__ gnxt, uint32_t *__restrict__ fcur,
                                                   uint32_t *__restrict__ fnxt, int64_t nblocks, uint64_t *stats,
                                                   uint32_t g, uint32_t ngroups) {
    constexpr int B = Geo<DIM>::BLK, CPB = Geo<DIM>::CPB, L = Geo<DIM>::LOG;
    static_assert(CPB % WG == 0, "a node block is a whole number of work-group passes");
    uint32_t active = 0;
    for (int64_t b = g; b < nblocks; b += ngroups) {
        const bool tc = fcur[b] != 0u, tn = fnxt[b] != 0u;
        // every wave has read fnxt[b] before thread 0 resets it below (the
        // waves of a group do not run in lockstep)
        __syncthreads();
        if (!tc && !tn) continue;
        int bc[3] = {0, 0, 0};
        bc[0] = (int)(b % P.nb);
        if constexpr (DIM == 3) {
            bc[1] = (int)((b / P.nb) % P.nb);
            bc[2] = (int)(b / ((int64_t)P.nb * P.nb));
        } else {
            bc[1] = (int)(b / P.nb);
        }
        if (tc) {
            // all loads of the block first (CPB / WG nodes per thread)
            GNode g[CPB / WG];
#pragma unroll
            for (int r = 0; r < CPB / WG; ++r) g[r] = gcur[(b << (DIM * L)) + threadIdx.x + r * WG];
            // the packed velocities overwrite the first half of the block
            __syncthreads();
#pragma unroll
            for (int r = 0; r < CPB / WG; ++r) {
                const int l = threadIdx.x + r * WG;
                const double m = from_fix(g[r].q[3]);
                float vel[3] = {0.0f, 0.0f, 0.0f};
                if (m > 0.0) {
                    ++active;
                    int ijk[3];
                    ijk[0] = bc[0] * B + (l & (B - 1));
                    ijk[1] = bc[1] * B + ((l >> L) & (B - 1));
                    ijk[2] = (DIM == 3) ? bc[2] * B + (l >> (2 * L)) : 0;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) {
                        float va = (float)(from_fix(g[r].q[a]) / m) + P.dt * P.g[a];
                        if (ijk[a] < P.bound && va < 0.0f) va = 0.0f;
                        if (ijk[a] >= P.res - P.bound && va > 0.0f) va = 0.0f;
                        vel[a] = va;
                    }
                }
                const float mass = m > 0.0 ? (float)(m * (1.0 / FIX_ONE)) * P.p_mass : 0.0f;
                reinterpret_cast<float4 *>(gcur)[vel_slot<DIM>((b << (DIM * L)) + l)] =
                    make_float4(vel[0], vel[1], vel[2], mass);
            }
        }
        if (tn) {
            ulonglong4 z;
            z.x = z.y = z.z = z.w = 0ull;
#pragma unroll
            for (int r = 0; r < CPB / WG; ++r)
                reinterpret_cast<ulonglong4 *>(gnxt + (b << (DIM * L)) + threadIdx.x + r * WG)[0] = z;
            if (threadIdx.x == 0) fnxt[b] = 0u;
        }
    }
    // one atomic per work-group, spread over ST_ACTIVE_SLOTS counters: a
    // single counter hit by every wave serializes in the L2
    __shared__ uint32_t wsum[WG / 64];
    const uint32_t ws = wave_sum(active);
    if (__lane_id() == 0) wsum[threadIdx.x >> 6] = ws;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
#pragma unroll
        for (int i = 0; i < WG / 64; ++i) tot += wsum[i];
        if (tot)
            atomicAdd((unsigned long long *)&stats[ST_ACTIVE + (g % ST_ACTIVE_SLOTS)], (unsigned long long)tot);
    }
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_update(DevParams P, GNode *__restrict__ gcur,
                                                    GNode *__restrict__ gnxt, uint32_t *__restrict__ fcur,
                                                    uint32_t *__restrict__ fnxt, int64_t nblocks, uint64_t *stats) {
    grid_update_blocks<DIM>(P, gcur, gnxt, fcur, fnxt, nblocks, stats, blockIdx.x, gridDim.x);
}

// Batched grid update: work-group g serves the scene whose group range holds
// it (see k_substep_batch), with that scene's grids for its step.
template <int DIM>
__global__ __launch_bounds__(WG) void k_grid_update_batch(const BatchArgs args) {
    const int i = batch_scene(args, blockIdx.x);
    const BatchRef d = batch_ref(args.desc[i]);
    const DevParams P = batch_params(d);
    const uint32_t g0 = args.group_begin[i], cur = args.step[i] & 1u;
    grid_update_blocks<DIM>(P, d->grid[cur], d->grid[cur ^ 1u], d->flags[cur], d->flags[cur ^ 1u], d->nblocks,
                            d->stats, blockIdx.x - g0, args.group_begin[i + 1] - g0);
}

template <int DIM>
__global__ __launch_bounds__(WG) void k_clear_touched(GNode *__restrict__ g, uint32_t *__restrict__ flags,
                                                      int64_t nblocks) {
    constexpr int CPB = Geo<DIM>::CPB, L = Geo<DIM>::LOG;
    const int64_t b = blockIdx.x;
    const bool touched = flags[b] != 0u;
    __syncthreads();  // every wave has read the flag before thread 0 resets it
    if (!touched) return;
    for (int l = threadIdx.x; l < CPB; l += WG) {
        ulonglong4 z;
        z.x = z.y = z.z = z.w = 0ull;
        reinterpret_cast<ulonglong4 *>(g + (b << (DIM * L)) + l)[0] = z;
    }
    if (threadIdx.x == 0) flags[b] = 0u;
}

// Calibration of 64-bit global atomic throughput: every thread adds 1 to
// word (i * stride) mod n for its indices i, `passes` times (stride 1: each
// wave instruction covers 64 consecutive words).
__global__ __launch_bounds__(WG) void k_calib_atomics(unsigned long long *__restrict__ buf, int64_t n, int passes,
                                                      int64_t stride) {
    const int64_t nthreads = (int64_t)gridDim.x * WG;
    for (int r = 0; r < passes; ++r)
        for (int64_t i = (int64_t)blockIdx.x * WG + threadIdx.x; i < n; i += nthreads)
            atomicAdd(buf + (i * stride) % n, 1ull);
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

// dimension x material, work-group of NT threads
#define MPMQ_DISPATCH_MB(dim, mat, KERNEL, GRID, NT, ...)                                               \
    do {                                                                                               \
        if ((dim) == 3 && (mat)) hipLaunchKernelGGL((KERNEL<3, 1>), GRID, dim3(NT), 0, st, __VA_ARGS__);  \
        else if ((dim) == 3) hipLaunchKernelGGL((KERNEL<3, 0>), GRID, dim3(NT), 0, st, __VA_ARGS__);      \
        else if (mat) hipLaunchKernelGGL((KERNEL<2, 1>), GRID, dim3(NT), 0, st, __VA_ARGS__);             \
        else hipLaunchKernelGGL((KERNEL<2, 0>), GRID, dim3(NT), 0, st, __VA_ARGS__);                      \
    } while (0)
#define MPMQ_DISPATCH_M(dim, mat, KERNEL, GRID, ...) MPMQ_DISPATCH_MB(dim, mat, KERNEL, GRID, WG, __VA_ARGS__)

// dimension x flag x material (particle-tile kernels)
#define MPMQ_DISPATCH2(dim, mat, KERNEL, FLAG, GRID, ...)                                                    \
    do {                                                                                                    \
        if ((dim) == 3 && (mat)) hipLaunchKernelGGL((KERNEL<3, FLAG, 1>), GRID, dim3(PWG), 0, st, __VA_ARGS__); \
        else if ((dim) == 3) hipLaunchKernelGGL((KERNEL<3, FLAG, 0>), GRID, dim3(PWG), 0, st, __VA_ARGS__);     \
        else if (mat) hipLaunchKernelGGL((KERNEL<2, FLAG, 1>), GRID, dim3(PWG), 0, st, __VA_ARGS__);            \
        else hipLaunchKernelGGL((KERNEL<2, FLAG, 0>), GRID, dim3(PWG), 0, st, __VA_ARGS__);                     \
    } while (0)

static dim3 pgrid(int64_t n) { return dim3((unsigned)((n + WG - 1) / WG)); }

hipError_t launch_encode(int dim, int mat, const DevScheme *s, const float *x, const float *v, const float *C,
                         const float *F, int64_t n, int64_t cap, uint32_t *words, uint32_t *ids, uint32_t step,
                         uint32_t tag, uint64_t *stats, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const dim3 g((unsigned)std::min<int64_t>((n + WG - 1) / WG, 4096));
    MPMQ_DISPATCH_M(dim, mat, k_encode, g, s, x, v, C, F, n, cap, words, ids, step, tag, stats);
    return hipGetLastError();
}

hipError_t launch_decode(int dim, int mat, const DevScheme *s, const uint32_t *words, int64_t n, int64_t cap,
                         float *x, float *v, float *C, float *F, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    MPMQ_DISPATCH_M(dim, mat, k_decode, pgrid(n), s, words, n, cap, x, v, C, F);
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

hipError_t launch_p2g(int dim, int mat, const DevScheme *s, const DevParams &p, const uint32_t *words, int64_t cap,
                      const WorkItem *items, const uint32_t *n_items, int grid, GNode *gout, uint32_t *flags_out,
                      const TileScale *iscale, float4 *irec, uint64_t *stats, hipStream_t st, const JitKernels *jit) {
    if (jit && jit->p2g) {
        DevParams pv = p;
        void *args[] = {(void *)&s, &pv, (void *)&words, &cap, (void *)&items, (void *)&n_items, &gout, &flags_out,
                        (void *)&iscale, &irec, &stats};
        return hipModuleLaunchKernel(jit->p2g, (unsigned)grid, 1, 1, PWG, 1, 1, 0, st, args, nullptr);
    }
    MPMQ_DISPATCH_MB(dim, mat, k_p2g, dim3(grid), PWG, s, p, words, cap, items, n_items, gout, flags_out, iscale,
                     irec, stats);
    return hipGetLastError();
}

hipError_t launch_grid_update(int dim, const DevParams &p, GNode *gcur, GNode *gnxt, uint32_t *flags_cur,
                              uint32_t *flags_nxt, int64_t nblocks, uint64_t *stats, hipStream_t st) {
    const dim3 grid((unsigned)std::min<int64_t>(nblocks, 4096));
    if (dim == 3)
        hipLaunchKernelGGL(k_grid_update<3>, grid, dim3(WG), 0, st, p, gcur, gnxt, flags_cur, flags_nxt, nblocks,
                           stats);
    else
        hipLaunchKernelGGL(k_grid_update<2>, grid, dim3(WG), 0, st, p, gcur, gnxt, flags_cur, flags_nxt, nblocks,
                           stats);
    return hipGetLastError();
}

hipError_t launch_calib_atomics(unsigned long long *buf, int64_t n, int passes, int64_t stride, hipStream_t st) {
    const dim3 grid((unsigned)std::min<int64_t>((n + WG - 1) / WG, 65536));
    hipLaunchKernelGGL(k_calib_atomics, grid, dim3(WG), 0, st, buf, n, passes, stride);
    return hipGetLastError();
}

hipError_t launch_grid_update_batch(int dim, const BatchArgs &a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    const dim3 grid(a.group_begin[a.count]);
    if (dim == 3) hipLaunchKernelGGL(k_grid_update_batch<3>, grid, dim3(WG), 0, st, a);
    else hipLaunchKernelGGL(k_grid_update_batch<2>, grid, dim3(WG), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_substep_batch(int dim, int mat, int round_stats, const BatchArgs &a, hipStream_t st) {
    if (a.count <= 0) return hipSuccess;
    const dim3 grid(a.group_begin[a.count]);
    if (round_stats) MPMQ_DISPATCH2(dim, mat, k_substep_batch, true, grid, a);
    else MPMQ_DISPATCH2(dim, mat, k_substep_batch, false, grid, a);
    return hipGetLastError();
}

hipError_t launch_clear_touched(int dim, GNode *g, uint32_t *flags, int64_t nblocks, hipStream_t st) {
    if (dim == 3)
        hipLaunchKernelGGL(k_clear_touched<3>, dim3((unsigned)nblocks), dim3(WG), 0, st, g, flags, nblocks);
    else
        hipLaunchKernelGGL(k_clear_touched<2>, dim3((unsigned)nblocks), dim3(WG), 0, st, g, flags, nblocks);
    return hipGetLastError();
}

hipError_t launch_substep(int dim, int mat, const DevScheme *s, const DevParams &p, uint32_t *words, int64_t cap,
                          const WorkItem *items, const uint32_t *n_items, int grid, const GNode *gcur,
                          GNode *gnxt, uint32_t *flags_nxt, TileScale *iscale, float4 *irec, uint32_t step,
                          int do_p2g, int collect_stats, int round_stats, uint64_t *stats, hipStream_t st,
                          const JitKernels *jit) {
    if (jit && jit->substep[round_stats ? 1 : 0]) {
        DevParams pv = p;
        void *args[] = {(void *)&s, &pv, &words, &cap, (void *)&items, (void *)&n_items, (void *)&gcur, &gnxt,
                        &flags_nxt, &iscale, &irec, &step, &do_p2g, &collect_stats, &stats};
        return hipModuleLaunchKernel(jit->substep[round_stats ? 1 : 0], (unsigned)grid, 1, 1, PWG, 1, 1, 0, st, args,
                                     nullptr);
    }
    if (round_stats)
        MPMQ_DISPATCH2(dim, mat, k_substep, true, dim3(grid), s, p, words, cap, items, n_items, gcur, gnxt, flags_nxt,
                       iscale, irec, step, do_p2g, collect_stats, stats);
    else
        MPMQ_DISPATCH2(dim, mat, k_substep, false, dim3(grid), s, p, words, cap, items, n_items, gcur, gnxt, flags_nxt,
                       iscale, irec, step, do_p2g, collect_stats, stats);
    return hipGetLastError();
}

}  // namespace mpmq
