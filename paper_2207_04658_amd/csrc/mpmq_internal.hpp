// mpmq_internal.hpp -- descriptors shared by the host runtime and the gfx950
// kernels of the quantized MLS-MPM library (not part of the public ABI).
#pragma once
#ifndef __HIPCC_RTC__
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string>
#else
// runtime compilation (hipRTC): the HIP runtime header is implicit
using __hip_internal::int32_t;
using __hip_internal::int64_t;
using __hip_internal::uint16_t;
using __hip_internal::uint32_t;
using __hip_internal::uint64_t;
#endif

namespace mpmq {

// Sort / tile geometry.  Particles are sorted by cell and grouped by blocks of
// BLK^dim cells; each work item covers one block's particles (or a chunk of
// them) and stages a (BLK+4)^dim node tile in LDS (one node of margin on
// each side beyond the 3-node stencil reach, so particles that drifted by up
// to one cell since the sort stay inside the tile).
template <int DIM> struct Geo;
// TS: stride of the four component arrays of the LDS accumulator tile, TN + 8
// nodes, so that the flush's lanes (16 nodes x 4 components per wave) spread
// over all 64 LDS banks.
template <> struct Geo<3> {
    static constexpr int BLK = 8, LOG = 3, CPB = 512, TB = 12, TN = 1728, TS = 1736, NST = 27;
};
template <> struct Geo<2> {
    static constexpr int BLK = 16, LOG = 4, CPB = 256, TB = 20, TN = 400, TS = 408, NST = 9;
};

constexpr int WG = 256;          // threads per work-group of the particle kernels
// Threads per work-group of the particle-tile kernels (bootstrap P2G and the
// fused substep).  In 3D a group stages 76 KB of node tile in LDS, so two
// groups share a CU's 160 KB: two waves per SIMD, up to 256 VGPRs per lane.
// (384-thread groups, three waves per SIMD, measured 25 % slower on the
// 3e8-particle workload.)
constexpr int PWG = 256;
constexpr int PWG_WAVES_PER_EU = 2;
constexpr int MAX_WORDS = 32;    // record <= 1024 bits

// One field's codec constants (indexed by field id x=0, v=1, C=2, F=3).
struct DevField {
    int32_t kind, bits, exp_bits, dither;
    int32_t rel, off, emin, emax;        // off: first record bit (SHARED_EXP: exponent)
    uint32_t mask, exp_mask, mag_mask;
    uint32_t f32dec;                     // 1: every decoded value is exact in float32 (see compile_scheme)
    double lo, delta, inv, maxc;         // FIXED: range start, step, 2^b/(hi-lo), 2^b-1
};

struct DevScheme {
    int32_t dim, W;
    uint32_t seed_lo, seed_hi;
    uint32_t dither_groups;              // bit j: Philox group j (canonical comps 8j..8j+7) is needed
    int32_t order[4];                    // placement order of the state slots (F and J: slot 3)
    int32_t mat;                         // 0 elastic (slot 3 = F), 1 fluid (slot 3 = J)
    int32_t pad[2];
    DevField f[4];
};

// Grid node.  During P2G: exact fixed-point sums (two's complement int64,
// 2^-32 resolution) of momentum and mass per unit particle mass; integer
// addition is associative, so the sums do not depend on the order of the
// atomics.  After the grid update the first 16 bytes hold the float
// velocity and mass (float4).
struct alignas(32) GNode {
    unsigned long long q[4];
};
constexpr double FIX_ONE = 4294967296.0;          // 2^32
constexpr double FIX_MAGIC = 6755399441055744.0;  // 1.5 * 2^52
constexpr unsigned long long FIX_MAGIC_BITS = 0x4338000000000000ull;

struct DevParams {
    int32_t dim, res, bound, nb;         // nb: node blocks per axis
    float dt, inv_dx, dx, mu, la, p_mass, stress_over_m, pc;  // pc: fluid pressure coefficient
    float g[3], pad2;
    double dt_d, inv_dx_d;
};

// Statistics slots (uint64) in scratch.  ST_CLAMP: particles whose P2G
// terms were clamped to the fixed-point range (see p2g_particle);
// ST_ATOMICS: 64-bit global atomic adds issued by the P2G tile flushes;
// ST_WIDE: particles of the fused kernel whose P2G terms did not fit their
// work item's 32-bit node tile (scattered through the 64-bit global path).
enum {
    ST_SAT = 0, ST_NAN = 4, ST_UP = 8, ST_DOWN = 12, ST_FALLBACK = 16, ST_ACTIVE = 17, ST_ACTIVE_SLOTS = 7,
    ST_CLAMP = 24, ST_ATOMICS = 25, ST_WIDE = 26, ST_COUNT = 27
};

// Device scratch layout (byte offsets, all 256-aligned).
struct Scratch {
    int64_t keys, vals, keys2, vals2;    // radix sort (Ncap each)
    int64_t cells;                       // ncells + 1 counts -> exclusive starts
    int64_t scan_tmp;                    // scan partial sums (all levels)
    int64_t hist;                        // radix histogram, 256 * tiles
    int64_t block_items;                 // nblocks + 1 item counts -> offsets
    int64_t items;                       // int4 work items
    int64_t iscale;                      // TileScale per work item (P2G tile scales of the stored state)
    int64_t irec;                        // float4 per work item: record of its last P2G (tile_scale)
    int64_t flags;                       // 2 * nblocks uint32 touched flags
    int64_t stats;                       // ST_COUNT uint64
    int64_t misc;                        // 64 uint32 (n_items, ...)
    int64_t scheme;                      // device copy of the DevScheme
    int64_t batch;                       // the context's BatchDesc
    int64_t total;
    int64_t ncells, nblocks, max_items, hist_entries, scan_tmp_entries;
};

struct WorkItem { int32_t block, p0, p1, pad; };

// Scales of a work item's 32-bit P2G node tile (see substep.hpp): node
// values are summed less vref in units of 2^-s, weights in units of 2^-sm,
// and a particle enters the tile only if its node values lie within lim_v
// of vref.  The fused kernel records the scales each item used in a table
// (one entry per work item) so that a later P2G of the same stored state
// (the adjoint's recomputation from a checkpoint, a grid rebuilt after the
// adjoint) reproduces its sums bit for bit.
struct TileScale {
    float vref[3];     // reference velocity, a multiple of 2^-(32 - sm), |vref| 2^(32 - sm) <= 2^24
    float lim_v;       // admission bound of |node value - vref| (velocity units)
    int32_t s, sm;     // exponents of the momentum and weight scales
};

// Batched launches (serving): a context's buffers and parameters, kept in its
// scratch in device memory, and the per-launch table of scenes.
struct BatchDesc {
    const DevScheme *scheme;
    uint32_t *words;
    int64_t cap;
    const WorkItem *items;
    const uint32_t *n_items;
    GNode *grid[2];
    uint32_t *flags[2];
    uint64_t *stats;
    TileScale *iscale;
    float4 *irec;
    int64_t nblocks;
    DevParams P;
};
constexpr int MAX_BATCH = 96;  // scenes per batched launch (the table is a kernel argument)
struct BatchArgs {
    int32_t count, pad;
    uint32_t group_begin[MAX_BATCH + 1];  // first work-group of each scene; [count] = total
    const BatchDesc *desc[MAX_BATCH];
    uint32_t step[MAX_BATCH];             // the scene's substep index (Philox step; grid G[step & 1])
    uint32_t mode[MAX_BATCH];             // bit 0: scatter the stored state (P2G); bit 1: flush encoder counters
};

#ifndef __HIPCC_RTC__
// ---- launchers (kernels.hip) ----

hipError_t launch_encode(int dim, int mat, const DevScheme *s, const float *x, const float *v,
                         const float *C, const float *F, int64_t n, int64_t cap, uint32_t *words,
                         uint32_t *ids, uint32_t step, uint32_t tag, uint64_t *stats, hipStream_t st);
hipError_t launch_decode(int dim, int mat, const DevScheme *s, const uint32_t *words, int64_t n,
                         int64_t cap, float *x, float *v, float *C, float *F, hipStream_t st);
hipError_t launch_sort_keys(int dim, int wm, const DevScheme *s, const DevParams &p,
                            const uint32_t *words, int64_t n, int64_t cap, uint32_t *keys,
                            uint32_t *vals, uint32_t *cell_count, hipStream_t st);
hipError_t launch_fill_u32(uint32_t *p, uint32_t value, int64_t n, hipStream_t st);
hipError_t launch_scan(uint32_t *data, int64_t n, uint32_t *tmp, hipStream_t st);
hipError_t launch_radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                             int64_t n, int shift, uint32_t *hist, uint32_t *scan_tmp, hipStream_t st);
hipError_t launch_layer(int dim, const uint32_t *cell_start, const uint32_t *sorted_vals,
                        int64_t nblocks, uint32_t *perm, uint32_t *block_items, int item_cap,
                        hipStream_t st);
hipError_t launch_items(const uint32_t *cell_start, const uint32_t *block_items_scanned,
                        int64_t nblocks, int cpb, int item_cap, WorkItem *items, uint32_t *n_items,
                        hipStream_t st);
hipError_t launch_gather_u32(const uint32_t *in, const uint32_t *perm, uint32_t *out, int64_t n,
                             hipStream_t st);
hipError_t launch_copy_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t st);
hipError_t launch_calib_atomics(unsigned long long *buf, int64_t n, int passes, int64_t stride, hipStream_t st);
// Kernels compiled at run time with a context's scheme as constants
// (jit.hip); null entries fall back to the generic kernels.
struct JitKernels {
    hipFunction_t substep[2];  // k_substep<dim, RS = false / true>
    hipFunction_t p2g;         // k_p2g<dim>
};
// Compiles (once per process, scheme and device) and loads the specialized
// kernels for the current device.  Returns false with a message on failure.
bool jit_kernels(int dim, const DevScheme &ds, const DevParams &dp, int64_t cap, JitKernels *out, std::string *err);

// iscale: null for an exact 64-bit P2G (after a sort or an encode), else the
// scales the fused kernel recorded when it scattered this state.
// irec: receives each tiled work item's record (for the next fused substep).
hipError_t launch_p2g(int dim, int mat, const DevScheme *s, const DevParams &p, const uint32_t *words,
                      int64_t cap, const WorkItem *items, const uint32_t *n_items, int grid,
                      GNode *gout, uint32_t *flags_out, const TileScale *iscale, float4 *irec,
                      uint64_t *stats, hipStream_t st, const JitKernels *jit = nullptr);
hipError_t launch_grid_update(int dim, const DevParams &p, GNode *gcur, GNode *gnxt,
                              uint32_t *flags_cur, uint32_t *flags_nxt, int64_t nblocks,
                              uint64_t *stats, hipStream_t st);
hipError_t launch_clear_touched(int dim, GNode *g, uint32_t *flags, int64_t nblocks, hipStream_t st);
// Batched grid update / fused substep of a.count scenes of one dimension and
// material (group_begin counts the launch's work-groups per scene).
hipError_t launch_grid_update_batch(int dim, const BatchArgs &a, hipStream_t st);
hipError_t launch_substep_batch(int dim, int mat, int round_stats, const BatchArgs &a, hipStream_t st);
// iscale: receives the tile scales of every work item that scatters (do_p2g);
// irec: each item's record of its last P2G, read and rewritten.
hipError_t launch_substep(int dim, int mat, const DevScheme *s, const DevParams &p, uint32_t *words,
                          int64_t cap, const WorkItem *items, const uint32_t *n_items, int grid,
                          const GNode *gcur, GNode *gnxt, uint32_t *flags_nxt, TileScale *iscale,
                          float4 *irec, uint32_t step, int do_p2g, int collect_stats, int round_stats,
                          uint64_t *stats, hipStream_t st, const JitKernels *jit = nullptr);

// Adjoint (adjoint.hip).  lam buffers: float32 rows x[d], v[d], C[d*d],
// then F[d*d] (elastic) or J (fluid) of n each; nadj: one float4 per grid node; acc: binary64 z, G[4],
// g[4]; rng: uint32 order keys min[4], max[4].
hipError_t launch_adj_objective(int dim, int mat, const DevScheme *s, const DevParams &P, const uint32_t *words, int64_t cap,
                                int64_t n, int objective, int axis, float *lam, double *acc, hipStream_t st);
// items / n_items / item_grid / item_cap: the work items of the last sort and
// their particle limit (the adjoint's G2P backward accumulates node adjoints
// per item tile; its P2G backward gathers them from per-item tiles)
hipError_t launch_adj_step(int dim, int mat, const DevScheme *s, const DevParams &P, const uint32_t *words, int64_t cap,
                           int64_t n, const WorkItem *items, const uint32_t *n_items, int item_grid, int item_cap,
                           const GNode *grid, int64_t nodes, const float *lin, float *lout, float4 *nadj,
                           hipStream_t st);
// The adjoint's per-field reductions add into ADJ_SLOTS copies of their
// accumulators (work-group b into copy b % ADJ_SLOTS; the host combines
// them): device-wide atomics on one address serialize, and a few hundred
// groups on one copy cost more than the reduction itself.
constexpr int ADJ_SLOTS = 64;
// acc[0]: objective z; acc[1 + 8 s + k]: copy s of the sums of lambda
// (k = field) and of lambda^2 (k = 4 + field).
constexpr int ADJ_ACC_DOUBLES = 1 + 8 * ADJ_SLOTS;
hipError_t launch_adj_reduce(int dim, int mat, const float *lam, int64_t n, double *acc, hipStream_t st);
// rng[4 s + f]: copy s of the minimum key of field f; rng[4 ADJ_SLOTS + 4 s + f]:
// of its maximum key
hipError_t launch_adj_range(int dim, int mat, const DevScheme *s, const uint32_t *words, int64_t cap, int64_t n, uint32_t *rng,
                            hipStream_t st);
hipError_t launch_adj_unpermute(const float *lam, const uint32_t *ids, int64_t n, int rows, float *out,
                                hipStream_t st);

#endif  // __HIPCC_RTC__

}  // namespace mpmq
