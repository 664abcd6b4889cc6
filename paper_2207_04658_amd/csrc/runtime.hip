// runtime.hip -- host side of the C ABI declared in include/mpmq.h: scheme
// compilation (bit offsets, codec constants), carving of the caller's
// buffers, and the launch sequence of one substep on the caller's stream.
#include "../../include/mpmq.h"
#include "mpmq_internal.hpp"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <vector>

using namespace mpmq;

namespace {

thread_local std::string g_last_error = "";

struct EventPair {
    const char *name;
    hipEvent_t a, b;
};

int ceil_log2_double(double hi) {
    int ex;
    const double m = std::frexp(hi, &ex);
    return (m == 0.5) ? ex - 1 : ex;
}

int ncomp(int field, int dim) {
    return (field == MPMQ_FIELD_X || field == MPMQ_FIELD_V) ? dim : field == MPMQ_FIELD_J ? 1 : dim * dim;
}
// state slot of a field: F and J share slot 3
int slot_of(int field) { return field == MPMQ_FIELD_J ? 3 : field; }

bool compile_scheme(const mpmq_scheme *sc, DevScheme &ds, int &total_bits, std::string &err) {
    if (!sc || !sc->fields) { err = "scheme or scheme->fields is NULL"; return false; }
    if (sc->dim != 2 && sc->dim != 3) { err = "scheme dim must be 2 or 3"; return false; }
    if (sc->n_fields != 4) { err = "scheme must list 4 fields: x, v, C and one of F / J"; return false; }
    std::memset(&ds, 0, sizeof(ds));
    ds.dim = sc->dim;
    ds.seed_lo = (uint32_t)sc->seed;
    ds.seed_hi = (uint32_t)(sc->seed >> 32);
    bool seen[4] = {false, false, false, false};
    int off = 0;
    static const char *names[5] = {"x", "v", "C", "F", "J"};
    const int dim = sc->dim;
    for (int i = 0; i < 4; ++i) {
        const mpmq_field_scheme &f = sc->fields[i];
        if (f.field < 0 || f.field > 4 || seen[slot_of(f.field)]) {
            err = "fields must be x, v, C and one of F / J, each exactly once";
            return false;
        }
        const int sl = slot_of(f.field);
        seen[sl] = true;
        ds.order[i] = sl;
        if (f.field == MPMQ_FIELD_J) ds.mat = 1;
        const char *nm = names[f.field];
        const int nc = ncomp(f.field, dim);
        const bool rel = (f.flags & MPMQ_REL_IDENTITY) != 0;
        if (rel && sl != 3) { err = std::string("REL_IDENTITY is only valid for F or J (field ") + nm + ")"; return false; }
        DevField &d = ds.f[sl];
        d.kind = f.kind;
        d.bits = f.bits;
        d.exp_bits = f.exp_bits;
        d.dither = f.dither ? 1 : 0;
        d.rel = rel ? 1 : 0;
        d.off = off;
        d.mask = (f.bits >= 32) ? 0xffffffffu : (uint32_t)((1ull << f.bits) - 1ull);
        if (f.kind == MPMQ_FIXED) {
            if (f.bits < 1 || f.bits > 32) { err = std::string("field ") + nm + ": FIXED bits must be in [1, 32]"; return false; }
            if (!(f.hi > f.lo) || !std::isfinite(f.lo) || !std::isfinite(f.hi)) { err = std::string("field ") + nm + ": need finite lo < hi"; return false; }
            d.lo = f.lo;
            d.delta = std::ldexp(f.hi - f.lo, -f.bits);
            d.inv = std::ldexp(1.0, f.bits) / (f.hi - f.lo);
            d.maxc = std::ldexp(1.0, f.bits) - 1.0;
            // decoded values lo + u delta (+ 1 on a REL_IDENTITY diagonal) are
            // exact in float32 when delta is a power of two in [2^-100, 1], lo
            // is a multiple of it and every value is below 2^24 delta
            int e = 0;
            const bool pow2 = std::frexp(d.delta, &e) == 0.5 && d.delta >= std::ldexp(1.0, -100) && d.delta <= 1.0;
            const double top = std::ldexp(d.delta, 24), last = d.lo + d.maxc * d.delta;
            bool fits = f.bits <= 24 && std::fabs(d.lo) < top && std::fabs(last) < top;
            if (rel) fits = fits && std::fabs(d.lo + 1.0) < top && std::fabs(last + 1.0) < top;
            d.f32dec = (pow2 && std::fmod(d.lo, d.delta) == 0.0 && fits) ? 1u : 0u;
        } else if (f.kind == MPMQ_SHARED_EXP) {
            if (f.bits < 2 || f.bits > 32) { err = std::string("field ") + nm + ": SHARED_EXP bits must be in [2, 32]"; return false; }
            if (f.exp_bits < 1 || f.exp_bits > 8) { err = std::string("field ") + nm + ": exp_bits must be in [1, 8]"; return false; }
            if (!(f.hi > 0.0) || !std::isfinite(f.hi) || rel) { err = std::string("field ") + nm + ": SHARED_EXP needs finite hi > 0 and no REL_IDENTITY"; return false; }
            d.emax = ceil_log2_double(f.hi);
            d.emin = d.emax - ((1 << f.exp_bits) - 1);
            d.mag_mask = (uint32_t)((1ull << (f.bits - 1)) - 1ull);
            d.exp_mask = (uint32_t)((1ull << f.exp_bits) - 1ull);
            // q 2^(E - m + 1) is exact in float32 for q < 2^24 and normal exponents
            d.f32dec = (f.bits - 1 <= 24 && d.emin - (f.bits - 1) >= -126 && d.emax <= 127) ? 1u : 0u;
            off += f.exp_bits;
        } else if (f.kind == MPMQ_RAW_F32) {
            if (f.bits != 32) { err = std::string("field ") + nm + ": RAW_F32 bits must be 32"; return false; }
        } else {
            err = std::string("field ") + nm + ": unknown kind";
            return false;
        }
        off += nc * f.bits;
        // canonical component numbering x, v, C, then F or J selects the Philox groups
        const int k0 = sl == 0 ? 0 : sl == 1 ? dim : sl == 2 ? 2 * dim : 2 * dim + dim * dim;
        if (d.dither && f.kind != MPMQ_RAW_F32)
            for (int c = 0; c < nc; ++c) ds.dither_groups |= 1u << ((k0 + c) / 8);
    }
    if (off > 32 * MAX_WORDS) { err = "record longer than 1024 bits"; return false; }
    total_bits = off;
    ds.W = (off + 31) / 32;
    return true;
}

bool compile_params(const mpmq_params *pp, int dim, DevParams &dp, std::string &err) {
    if (!pp) { err = "params is NULL"; return false; }
    if (pp->dim != dim) { err = "params dim differs from scheme dim"; return false; }
    if (pp->material != MPMQ_ELASTIC && pp->material != MPMQ_FLUID) { err = "unknown material"; return false; }
    if (pp->grid_res < 8 || pp->grid_res > 1024) { err = "grid_res must be in [8, 1024]"; return false; }
    if (pp->bound_cells < 0 || pp->sort_every < 0) { err = "bound_cells and sort_every must be >= 0"; return false; }
    if (!(pp->dt > 0) || !(pp->E > 0) || !(pp->rho > 0) || !(pp->p_vol > 0) || !(pp->nu > -1.0 && pp->nu < 0.5)) {
        err = "need dt, E, rho, p_vol > 0 and -1 < nu < 0.5";
        return false;
    }
    std::memset(&dp, 0, sizeof(dp));
    const int B = dim == 3 ? Geo<3>::BLK : Geo<2>::BLK;
    dp.dim = dim;
    dp.res = pp->grid_res;
    dp.bound = pp->bound_cells;
    dp.nb = (pp->grid_res + B - 1) / B;
    const double inv_dx = (double)pp->grid_res;
    const double mu = pp->E / (2.0 * (1.0 + pp->nu));
    const double la = pp->E * pp->nu / ((1.0 + pp->nu) * (1.0 - 2.0 * pp->nu));
    dp.dt = (float)pp->dt;
    dp.inv_dx = (float)inv_dx;
    dp.dx = (float)(1.0 / inv_dx);
    dp.mu = (float)mu;
    dp.la = (float)la;
    dp.p_mass = (float)(pp->rho * pp->p_vol);
    dp.stress_over_m = (float)(-pp->dt * 4.0 * inv_dx * inv_dx / pp->rho);
    dp.pc = (float)pp->E;
    if (pp->material == MPMQ_FLUID) dp.mu = dp.la = 0.0f;
    for (int a = 0; a < 3; ++a) dp.g[a] = (float)pp->gravity[a];
    dp.dt_d = pp->dt;
    dp.inv_dx_d = inv_dx;
    return true;
}

int64_t align256(int64_t x) { return (x + 255) & ~(int64_t)255; }

Scratch plan_scratch(int dim, int res, int64_t cap_pad) {
    Scratch s;
    std::memset(&s, 0, sizeof(s));
    const int B = dim == 3 ? Geo<3>::BLK : Geo<2>::BLK;
    const int CPB = dim == 3 ? Geo<3>::CPB : Geo<2>::CPB;
    const int64_t nb = (res + B - 1) / B;
    s.nblocks = dim == 3 ? nb * nb * nb : nb * nb;
    s.ncells = s.nblocks * CPB;
    const int64_t tiles = (cap_pad + 4095) / 4096;
    s.hist_entries = 256 * tiles;
    int64_t big = std::max<int64_t>(s.ncells + 1, std::max<int64_t>(s.hist_entries, s.nblocks + 1));
    s.scan_tmp_entries = 0;
    for (int64_t lvl = big; lvl > 4096;) {
        lvl = (lvl + 4095) / 4096;
        s.scan_tmp_entries += lvl;
    }
    s.scan_tmp_entries += 64;
    s.max_items = std::min<int64_t>(s.nblocks, cap_pad) + cap_pad / 256 + 2;
    int64_t o = 0;
    s.keys = o; o = align256(o + 4 * cap_pad);
    s.vals = o; o = align256(o + 4 * cap_pad);
    s.keys2 = o; o = align256(o + 4 * cap_pad);
    s.vals2 = o; o = align256(o + 4 * cap_pad);
    s.cells = o; o = align256(o + 4 * (s.ncells + 1));
    s.scan_tmp = o; o = align256(o + 4 * s.scan_tmp_entries);
    s.hist = o; o = align256(o + 4 * s.hist_entries);
    s.block_items = o; o = align256(o + 4 * (s.nblocks + 1));
    s.items = o; o = align256(o + 16 * s.max_items);
    s.iscale = o; o = align256(o + (int64_t)sizeof(TileScale) * s.max_items);
    s.irec = o; o = align256(o + 16 * s.max_items);
    s.flags = o; o = align256(o + 4 * 2 * s.nblocks);
    s.stats = o; o = align256(o + 8 * ST_COUNT);
    s.misc = o; o = align256(o + 256);
    s.scheme = o; o = align256(o + (int64_t)sizeof(DevScheme));
    s.batch = o; o = align256(o + (int64_t)sizeof(BatchDesc));
    s.total = o;
    return s;
}

}  // namespace

struct mpmq_ctx {
    DevScheme ds;
    DevParams dp;
    mpmq_params params;
    int dim = 0, W = 0, wm = 16, record_bits = 0;
    int64_t cap = 0, cap_pad = 0;
    hipStream_t stream = nullptr;
    uint32_t *words = nullptr;
    GNode *grid[2] = {nullptr, nullptr};
    uint32_t *ids = nullptr;
    char *scratch = nullptr;
    Scratch sp;
    int64_t n = 0, step = 0, sorted_at = -1, sorts = 0, steps_taken = 0;
    bool encoded = false, sorted = false, p2g_ready = false;
    // the P2G tile scales of c->words are in iscale() (recorded by the fused
    // kernel that stored it); false after a sort or an encode
    bool scales_valid = false;
    int item_cap = 256, launch_grid = 1;
    bool timing = false;
    int stats_level = 0;
    std::vector<EventPair> events;
    std::map<std::string, std::pair<int64_t, double>> times;
    std::string err;
    JitKernels jit{};
    bool use_jit = false;
    BatchDesc bdesc{};  // host copy of the device descriptor (source of its upload)

    const JitKernels *jit_ptr() const { return use_jit ? &jit : nullptr; }
    uint32_t *u32(int64_t off) { return reinterpret_cast<uint32_t *>(scratch + off); }
    uint64_t *stats() { return reinterpret_cast<uint64_t *>(scratch + sp.stats); }
    uint32_t *flags(int i) { return u32(sp.flags) + (int64_t)i * sp.nblocks; }
    uint32_t *n_items() { return u32(sp.misc); }
    WorkItem *items() { return reinterpret_cast<WorkItem *>(scratch + sp.items); }
    TileScale *iscale() { return reinterpret_cast<TileScale *>(scratch + sp.iscale); }
    float4 *irec() { return reinterpret_cast<float4 *>(scratch + sp.irec); }
    const DevScheme *dscheme() { return reinterpret_cast<const DevScheme *>(scratch + sp.scheme); }
    const BatchDesc *dbatch() { return reinterpret_cast<const BatchDesc *>(scratch + sp.batch); }
};

namespace {

mpmq_status fail(mpmq_ctx *ctx, mpmq_status st, const std::string &msg) {
    if (ctx) ctx->err = msg;
    else g_last_error = msg;
    return st;
}

#define HIPCHK(ctx, call, what)                                                                        \
    do {                                                                                               \
        hipError_t e_ = (call);                                                                        \
        if (e_ != hipSuccess)                                                                          \
            return fail(ctx, MPMQ_EDEVICE, std::string(what) + ": " + hipGetErrorString(e_));          \
    } while (0)

// Records the events of a timed launch.
struct Timed {
    mpmq_ctx *c;
    EventPair ev;
    bool on;
    Timed(mpmq_ctx *ctx, const char *name) : c(ctx), on(ctx->timing) {
        if (on) {
            ev.name = name;
            (void)hipEventCreate(&ev.a);
            (void)hipEventCreate(&ev.b);
            (void)hipEventRecord(ev.a, c->stream);
        }
    }
    ~Timed() {
        if (on) {
            (void)hipEventRecord(ev.b, c->stream);
            c->events.push_back(ev);
        }
    }
};

mpmq_status do_sort(mpmq_ctx *c) {
    hipStream_t st = c->stream;
    c->scales_valid = false;  // new work items
    const int64_t n = c->n;
    const Scratch &s = c->sp;
    const int cpb = c->dim == 3 ? Geo<3>::CPB : Geo<2>::CPB;
    uint32_t *cells = c->u32(s.cells);
    // item size (a multiple of the particle work-group, 1 to 16 passes of it):
    // four passes by default, as each item pays for loading and flushing a
    // whole node tile (measured, particle-substeps/s against one pass:
    // +9 % on 1M-particle scenes, +7 % on the 262,144-particle adjoint,
    // +10 % over the mixed serving stream; two or eight passes do worse on
    // the first two); fewer on scenes too small to give ~256 items, more
    // (up to 16) on scenes of 4M particles and up
    int cap = 4 * PWG;
    while (cap > PWG && (int64_t)cap * 256 > n) cap /= 2;
    while (cap < 16 * PWG && (int64_t)cap * 2 * 2048 <= n) cap *= 2;
    c->item_cap = cap;
    const int64_t upper = std::min<int64_t>(s.nblocks, n) + (n + cap - 1) / cap + 1;
    // up to one work-group per work item (at most 131072): items differ in
    // size, and many short-lived groups balance better than a persistent
    // grid (measured on the 3e8-particle workload: 22.8 ms per substep with
    // 131072 groups, 23.8 ms with 4096, 25.9 ms with 512); a multiple of the
    // 8 XCDs (see ItemWalk)
    c->launch_grid = (int)std::max<int64_t>(8, ((std::min<int64_t>(upper, 131072) + 7) / 8) * 8);
    Timed t(c, "sort");
    HIPCHK(c, launch_fill_u32(cells, 0u, s.ncells + 1, st), "sort: clear cells");
    HIPCHK(c, launch_sort_keys(c->dim, c->wm, c->dscheme(), c->dp, c->words, n, c->cap_pad, c->u32(s.keys),
                               c->u32(s.vals), cells, st), "sort: keys");
    int kbits = 1;
    while (((int64_t)1 << kbits) < s.ncells) ++kbits;
    uint32_t *ka = c->u32(s.keys), *va = c->u32(s.vals), *kb = c->u32(s.keys2), *vb = c->u32(s.vals2);
    for (int shift = 0; shift < kbits; shift += 8) {
        HIPCHK(c, launch_radix_pass(ka, va, kb, vb, n, shift, c->u32(s.hist), c->u32(s.scan_tmp), st), "sort: radix");
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // ka/va: keys and original slots in cell order (stable)
    HIPCHK(c, launch_scan(cells, s.ncells + 1, c->u32(s.scan_tmp), st), "sort: cell scan");
    uint32_t *perm = ka;  // keys no longer needed
    uint32_t *tmp = kb;
    uint32_t *bitems = c->u32(s.block_items);
    HIPCHK(c, launch_layer(c->dim, cells, va, s.nblocks, perm, bitems, cap, st), "sort: layer");
    HIPCHK(c, launch_scan(bitems, s.nblocks + 1, c->u32(s.scan_tmp), st), "sort: item scan");
    HIPCHK(c, launch_items(cells, bitems, s.nblocks, cpb, cap, c->items(), c->n_items(), st), "sort: items");
    for (int k = 0; k < c->W; ++k) {
        uint32_t *row = c->words + (int64_t)k * c->cap_pad;
        HIPCHK(c, launch_gather_u32(row, perm, tmp, n, st), "sort: permute");
        HIPCHK(c, launch_copy_u32(tmp, row, n, st), "sort: permute");
    }
    if (c->ids) {
        HIPCHK(c, launch_gather_u32(c->ids, perm, tmp, n, st), "sort: ids");
        HIPCHK(c, launch_copy_u32(tmp, c->ids, n, st), "sort: ids");
    }
    c->sorts += 1;
    return MPMQ_OK;
}

// First part of a substep: sort when due (allow_sort), and P2G unless the
// previous substep already scattered this state.
mpmq_status pre_substep(mpmq_ctx *c, bool allow_sort) {
    hipStream_t st = c->stream;
    const int S = c->params.sort_every;
    const int64_t s = c->step;
    const int cur = (int)(s & 1);
    const bool need_sort = allow_sort && (!c->sorted || (S > 0 && s % S == 0 && c->sorted_at != s));
    if (need_sort) {
        if (c->p2g_ready) {
            Timed t(c, "clear");
            HIPCHK(c, launch_clear_touched(c->dim, c->grid[cur], c->flags(cur), c->sp.nblocks, st), "clear");
            c->p2g_ready = false;
        }
        mpmq_status r = do_sort(c);
        if (r != MPMQ_OK) return r;
        c->sorted = true;
        c->sorted_at = s;
    }
    if (!c->p2g_ready) {
        Timed t(c, "p2g");
        HIPCHK(c, launch_p2g(c->dim, c->ds.mat, c->dscheme(), c->dp, c->words, c->cap_pad, c->items(), c->n_items(),
                             c->launch_grid, c->grid[cur], c->flags(cur), c->scales_valid ? c->iscale() : nullptr,
                             c->irec(), c->stats(), st, c->jit_ptr()), "p2g");
    }
    return MPMQ_OK;
}

// Whether the substep after the current one sorts (then the fused kernel
// does not scatter its stored state).
bool next_sorts(const mpmq_ctx *c, bool allow_sort) {
    const int S = c->params.sort_every;
    return allow_sort && S > 0 && ((c->step + 1) % S) == 0;
}

// Host state after a substep's launches.
// t32: the fused kernel that ran sums in the 32-bit node tile (the scheme-
// specialized build) and recorded its tile scales; the generic build's
// 64-bit sums are reproduced by an exact P2G.
void post_substep(mpmq_ctx *c, bool allow_sort, bool t32) {
    c->p2g_ready = !next_sorts(c, allow_sort);
    c->scales_valid = c->p2g_ready && t32;
    c->step += 1;
    c->steps_taken += 1;
}

// One substep on c->words: pre_substep, grid update, fused
// G2P / update / encode / store / P2G kernel.
mpmq_status substep_once(mpmq_ctx *c, bool allow_sort) {
    mpmq_status r = pre_substep(c, allow_sort);
    if (r != MPMQ_OK) return r;
    hipStream_t st = c->stream;
    const int64_t s = c->step;
    const int cur = (int)(s & 1), nxt = cur ^ 1;
    {
        Timed t(c, "grid_update");
        HIPCHK(c, launch_grid_update(c->dim, c->dp, c->grid[cur], c->grid[nxt], c->flags(cur), c->flags(nxt),
                                     c->sp.nblocks, c->stats(), st), "grid update");
    }
    {
        Timed t(c, "substep");
        HIPCHK(c, launch_substep(c->dim, c->ds.mat, c->dscheme(), c->dp, c->words, c->cap_pad, c->items(), c->n_items(),
                                 c->launch_grid, c->grid[cur], c->grid[nxt], c->flags(nxt), c->iscale(), c->irec(),
                                 (uint32_t)s,
                                 next_sorts(c, allow_sort) ? 0 : 1, 1, c->stats_level >= 1 ? 1 : 0, c->stats(), st,
                                 c->jit_ptr()),
               "substep");
    }
    const JitKernels *jk = c->jit_ptr();
    post_substep(c, allow_sort, jk && jk->substep[c->stats_level >= 1 ? 1 : 0]);
    return MPMQ_OK;
}

// One substep of every context of a batch (same dimension, material and
// stream): per-scene sorts and bootstrap P2G, then a batched grid update and
// a batched fused kernel per chunk of up to MAX_BATCH scenes, grouped by
// whether the scene counts round-ups / round-downs.
mpmq_status batch_substep(mpmq_ctx *const *all, int count_all) {
    // scenes without particles only advance their counters (as mpmq_step)
    std::vector<mpmq_ctx *> live;
    for (int i = 0; i < count_all; ++i) {
        if (all[i]->n > 0) {
            live.push_back(all[i]);
        } else {
            all[i]->step += 1;
            all[i]->steps_taken += 1;
        }
    }
    if (live.empty()) return MPMQ_OK;
    mpmq_ctx *const *ctxs = live.data();
    const int count = (int)live.size();
    mpmq_ctx *c0 = ctxs[0];
    hipStream_t st = c0->stream;
    for (int i = 0; i < count; ++i) {
        mpmq_status r = pre_substep(ctxs[i], true);
        if (r != MPMQ_OK) {
            all[0]->err = ctxs[i]->err;  // batch errors are reported on the first context
            return r;
        }
    }
    for (int rs = 0; rs < 2; ++rs) {
        int i = 0;
        while (i < count) {
            BatchArgs ga{}, sa{};
            int k = 0;
            for (; i < count && k < MAX_BATCH; ++i) {
                mpmq_ctx *c = ctxs[i];
                if ((c->stats_level >= 1 ? 1 : 0) != rs) continue;
                // grid update: the per-scene launch's group count (a multiple of 8)
                const uint32_t gg = (uint32_t)((std::min<int64_t>(c->sp.nblocks, 4096) + 7) / 8 * 8);
                ga.desc[k] = sa.desc[k] = c->dbatch();
                ga.step[k] = sa.step[k] = (uint32_t)c->step;
                ga.mode[k] = sa.mode[k] = (next_sorts(c, true) ? 0u : 1u) | 2u;
                ga.group_begin[k + 1] = ga.group_begin[k] + gg;
                sa.group_begin[k + 1] = sa.group_begin[k] + (uint32_t)c->launch_grid;
                ++k;
            }
            ga.count = sa.count = k;
            if (k == 0) continue;
            {
                Timed t(c0, "grid_update_batch");
                HIPCHK(c0, launch_grid_update_batch(c0->dim, ga, st), "batch grid update");
            }
            {
                Timed t(c0, "substep_batch");
                HIPCHK(c0, launch_substep_batch(c0->dim, c0->ds.mat, rs, sa, st), "batch substep");
            }
        }
    }
    for (int i = 0; i < count; ++i) post_substep(ctxs[i], true, false);  // generic kernels
    return MPMQ_OK;
}

// Zeroes both grid buffers (every non-zero node block is flagged) so that
// the next substep starts with a P2G of c->words.
mpmq_status reset_grids(mpmq_ctx *c) {
    for (int i = 0; i < 2; ++i)
        HIPCHK(c, launch_clear_touched(c->dim, c->grid[i], c->flags(i), c->sp.nblocks, c->stream), "clear grids");
    c->p2g_ready = false;
    return MPMQ_OK;
}

int adj_rows(int dim, int mat) { return 2 * dim + dim * dim + (mat ? 1 : dim * dim); }

// Checkpoint plan of the adjoint: which states the forward pass stores and
// how many state buffers the backward pass holds at once.
struct AdjPlan {
    int64_t T = 0, K = 0;
    std::vector<int64_t> forward_saves;  // step indices stored by the forward pass
    int64_t slots = 0;                   // state buffers (excluding the final state)
};

// Bisection: the forward pass keeps s_0 and the midpoints on the path to the
// last step; reverse(lo, hi) then needs one new buffer per tree level.
void bisect_right_path(int64_t lo, int64_t hi, std::vector<int64_t> &out) {
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) / 2;
        out.push_back(mid);
        lo = mid;
    }
}

AdjPlan adj_plan(int64_t T, int64_t K) {
    AdjPlan p;
    p.T = T;
    p.K = K;
    p.forward_saves.push_back(0);
    if (T <= 0) {
        p.slots = 1;
        return p;
    }
    if (K >= 1) {
        for (int64_t t = K; t < T; t += K) p.forward_saves.push_back(t);
        p.slots = (int64_t)p.forward_saves.size() + std::min<int64_t>(K, T) - 1;
    } else {
        bisect_right_path(0, T, p.forward_saves);
        int64_t depth = 0;
        while (((int64_t)1 << depth) < T) ++depth;
        p.slots = depth + 1;
    }
    return p;
}

struct AdjWork {
    int64_t state_bytes = 0, scale_bytes = 0, lam_bytes = 0, nodes = 0;
    int64_t off_states = 0, off_final = 0, off_scales = 0, off_lam = 0, off_nadj = 0, off_acc = 0, off_stats = 0,
            total = 0;
};

AdjWork adj_layout(const mpmq_ctx *c, const AdjPlan &plan) {
    AdjWork w;
    const int CPB = c->dim == 3 ? Geo<3>::CPB : Geo<2>::CPB;
    w.nodes = c->sp.nblocks * CPB;
    w.state_bytes = 4 * (int64_t)c->W * c->cap_pad;
    w.lam_bytes = align256(4 * (int64_t)adj_rows(c->dim, c->ds.mat) * std::max<int64_t>(c->n, 1));
    int64_t o = 0;
    w.scale_bytes = align256((int64_t)sizeof(TileScale) * c->sp.max_items);
    w.off_states = o; o += plan.slots * w.state_bytes;
    w.off_final = o; o += w.state_bytes;
    w.off_scales = o; o += (plan.slots + 1) * w.scale_bytes;  // slot s, then the final state
    w.off_lam = o; o += 2 * w.lam_bytes;
    w.off_nadj = o; o = align256(o + 16 * w.nodes);
    w.off_acc = o; o = align256(o + 8 * ADJ_ACC_DOUBLES + 4 * 8 * ADJ_SLOTS);
    w.off_stats = o; o = align256(o + 8 * ST_COUNT);
    w.total = o;
    return w;
}

mpmq_status check_spec(mpmq_ctx *c, const mpmq_adjoint_spec *sp) {
    if (!sp) return fail(c, MPMQ_EINVAL, "spec is NULL");
    if (sp->objective != 0 && sp->objective != 1) return fail(c, MPMQ_EINVAL, "objective must be 0 (COM) or 1 (KE)");
    if (sp->objective == 0 && (sp->axis < 0 || sp->axis >= c->dim)) return fail(c, MPMQ_EINVAL, "axis out of range");
    if (sp->steps < 0) return fail(c, MPMQ_EINVAL, "steps < 0");
    if (sp->checkpoint_every < 0) return fail(c, MPMQ_EINVAL, "checkpoint_every < 0");
    return MPMQ_OK;
}

// Backward driver over a workspace: state buffers handed out from a free
// list, states recovered by re-running the forward from a stored one.
struct AdjRun {
    mpmq_ctx *c;
    char *ws;
    AdjWork w;
    int64_t step0 = 0;
    std::vector<int> free_slots;
    std::map<int64_t, int> saved;  // step -> slot, states kept by the forward pass
    float *lam_cur = nullptr, *lam_nxt = nullptr;
    int64_t recomputed = 0, live = 0, max_live = 0;
    // State buffers 0 .. slots-1, and `fin` (= slots) for s_T.  Each holds
    // the packed state and, when the fused kernel stored that state, the
    // P2G tile scales it recorded (valid), so that a P2G of the saved state
    // reproduces the forward pass's grid bit for bit.
    int fin = 0;
    std::vector<char> valid;

    uint32_t *slot_ptr(int s) {
        return reinterpret_cast<uint32_t *>(ws + (s == fin ? w.off_final : w.off_states + (int64_t)s * w.state_bytes));
    }
    TileScale *scale_ptr(int s) { return reinterpret_cast<TileScale *>(ws + w.off_scales + (int64_t)s * w.scale_bytes); }
    int64_t scale_words() const { return (int64_t)sizeof(TileScale) / 4 * c->sp.max_items; }
    double *acc() { return reinterpret_cast<double *>(ws + w.off_acc); }
    uint32_t *rng() { return reinterpret_cast<uint32_t *>(ws + w.off_acc + 8 * ADJ_ACC_DOUBLES); }
    float4 *nadj() { return reinterpret_cast<float4 *>(ws + w.off_nadj); }
    int64_t state_words() const { return (int64_t)c->W * c->cap_pad; }

    int take() {
        const int s = free_slots.back();
        free_slots.pop_back();
        max_live = std::max<int64_t>(max_live, ++live);
        return s;
    }
    void give(int s) {
        free_slots.push_back(s);
        --live;
    }
    // c->words (and its tile scales) into buffer s, and back
    mpmq_status save(int s) {
        HIPCHK(c, launch_copy_u32(c->words, slot_ptr(s), state_words(), c->stream), "adjoint: state copy");
        if (c->scales_valid)
            HIPCHK(c, launch_copy_u32(reinterpret_cast<const uint32_t *>(c->iscale()),
                                      reinterpret_cast<uint32_t *>(scale_ptr(s)), scale_words(), c->stream),
                   "adjoint: scale copy");
        valid[(size_t)s] = c->scales_valid ? 1 : 0;
        return MPMQ_OK;
    }
    mpmq_status load(int s) {
        HIPCHK(c, launch_copy_u32(slot_ptr(s), c->words, state_words(), c->stream), "adjoint: state copy");
        if (valid[(size_t)s])
            HIPCHK(c, launch_copy_u32(reinterpret_cast<const uint32_t *>(scale_ptr(s)),
                                      reinterpret_cast<uint32_t *>(c->iscale()), scale_words(), c->stream),
                   "adjoint: scale copy");
        c->scales_valid = valid[(size_t)s] != 0;
        return MPMQ_OK;
    }
    // c->words = s_from (taken from buffer `from`), then substeps up to each
    // target step in ascending order, saving s_t into its buffer.
    mpmq_status advance(int from, int64_t t_from, const std::vector<std::pair<int64_t, int>> &targets) {
        mpmq_status r = load(from);
        if (r != MPMQ_OK) return r;
        if ((r = reset_grids(c)) != MPMQ_OK) return r;
        c->step = step0 + t_from;
        int64_t t = t_from;
        for (const auto &tg : targets) {
            while (t < tg.first) {
                if ((r = substep_once(c, false)) != MPMQ_OK) return r;
                ++t;
                ++recomputed;
            }
            if ((r = save(tg.second)) != MPMQ_OK) return r;
        }
        return MPMQ_OK;
    }
    // lambda_t from lambda_{t+1} at the state s_t held in buffer `slot`.
    mpmq_status adjoint_step(int slot) {
        mpmq_status r = reset_grids(c);
        if (r != MPMQ_OK) return r;
        hipStream_t st = c->stream;
        const uint32_t *words = slot_ptr(slot);
        HIPCHK(c, launch_p2g(c->dim, c->ds.mat, c->dscheme(), c->dp, words, c->cap_pad, c->items(), c->n_items(),
                             c->launch_grid, c->grid[0], c->flags(0), valid[(size_t)slot] ? scale_ptr(slot) : nullptr,
                             c->irec(), c->stats(), st, c->jit_ptr()), "adjoint: p2g");
        HIPCHK(c, launch_grid_update(c->dim, c->dp, c->grid[0], c->grid[1], c->flags(0), c->flags(1), c->sp.nblocks,
                                     c->stats(), st), "adjoint: grid update");
        {
            Timed tm(c, "adjoint_step");
            HIPCHK(c, launch_adj_step(c->dim, c->ds.mat, c->dscheme(), c->dp, words, c->cap_pad, c->n, c->items(),
                                      c->n_items(), c->launch_grid, c->item_cap, c->grid[0], w.nodes,
                                      lam_cur, lam_nxt, nadj(), st), "adjoint: step");
        }
        HIPCHK(c, launch_adj_reduce(c->dim, c->ds.mat, lam_nxt, c->n, acc(), st), "adjoint: reduce");
        std::swap(lam_cur, lam_nxt);
        return MPMQ_OK;
    }
    // Reverses steps [lo, hi) given s_lo in slot `slot_lo` and lambda_hi in
    // lam_cur; leaves lambda_lo in lam_cur.
    mpmq_status reverse_bisect(int64_t lo, int64_t hi, int slot_lo) {
        if (hi - lo == 1) return adjoint_step(slot_lo);
        const int64_t mid = (lo + hi) / 2;
        int slot_mid;
        mpmq_status r;
        auto it = saved.find(mid);
        if (it != saved.end()) {
            slot_mid = it->second;
            saved.erase(it);
        } else {
            slot_mid = take();
            if ((r = advance(slot_lo, lo, {{mid, slot_mid}})) != MPMQ_OK) return r;
        }
        if ((r = reverse_bisect(mid, hi, slot_mid)) != MPMQ_OK) return r;
        give(slot_mid);
        return reverse_bisect(lo, mid, slot_lo);
    }
    // Uniform checkpoints: segment [a, b) from the stored s_a; all of its
    // states are recovered, then reversed.
    mpmq_status reverse_segment(int64_t a, int64_t b, int slot_a) {
        std::vector<std::pair<int64_t, int>> tg;
        for (int64_t t = a + 1; t < b; ++t) tg.push_back({t, take()});
        mpmq_status r;
        if (!tg.empty() && (r = advance(slot_a, a, tg)) != MPMQ_OK) return r;
        for (int64_t t = b - 1; t > a; --t) {
            const int s = tg[(size_t)(t - a - 1)].second;
            if ((r = adjoint_step(s)) != MPMQ_OK) return r;
            give(s);
        }
        return adjoint_step(slot_a);
    }
};

}  // namespace

extern "C" {

const char *mpmq_error_string(mpmq_status s) {
    switch (s) {
    case MPMQ_OK: return "ok";
    case MPMQ_EINVAL: return "invalid argument";
    case MPMQ_ENOMEM: return "buffer too small or capacity exceeded";
    case MPMQ_EDEVICE: return "HIP error";
    case MPMQ_ESTATE: return "invalid call order";
    case MPMQ_ENOTIMPL: return "not implemented";
    }
    return "unknown status";
}

const char *mpmq_last_error(mpmq_ctx *ctx) { return ctx ? ctx->err.c_str() : g_last_error.c_str(); }

mpmq_status mpmq_query_sizes(const mpmq_scheme *scheme, const mpmq_params *params, int64_t capacity,
                             mpmq_sizes *out) {
    if (!out) return fail(nullptr, MPMQ_EINVAL, "out is NULL");
    DevScheme ds;
    DevParams dp;
    int bits = 0;
    std::string err;
    if (!compile_scheme(scheme, ds, bits, err)) return fail(nullptr, MPMQ_EINVAL, err);
    if (!compile_params(params, ds.dim, dp, err)) return fail(nullptr, MPMQ_EINVAL, err);
    if ((params->material == MPMQ_FLUID) != (ds.mat == 1))
        return fail(nullptr, MPMQ_EINVAL, "material must match the scheme: F for ELASTIC, J for FLUID");
    if (capacity < 1 || capacity > (int64_t)0x3fffff00) return fail(nullptr, MPMQ_ENOMEM, "capacity must be in [1, 2^30-256]");
    const int64_t cap_pad = (capacity + 255) & ~(int64_t)255;
    const Scratch sp = plan_scratch(ds.dim, dp.res, cap_pad);
    const int CPB = ds.dim == 3 ? Geo<3>::CPB : Geo<2>::CPB;
    out->words_per_particle = ds.W;
    out->record_bits = bits;
    out->capacity_padded = cap_pad;
    out->packed_bytes = 4 * (int64_t)ds.W * cap_pad;
    out->grid_bytes = (int64_t)sizeof(GNode) * sp.nblocks * CPB;
    out->scratch_bytes = sp.total;
    out->ids_bytes = 4 * cap_pad;
    return MPMQ_OK;
}

mpmq_status mpmq_create(const mpmq_scheme *scheme, const mpmq_params *params, const mpmq_buffers *buffers,
                        int64_t capacity, void *hip_stream, mpmq_ctx **out) {
    if (!out || !buffers) return fail(nullptr, MPMQ_EINVAL, "out or buffers is NULL");
    *out = nullptr;
    mpmq_sizes sz;
    mpmq_status st = mpmq_query_sizes(scheme, params, capacity, &sz);
    if (st != MPMQ_OK) return st;
    if (!buffers->packed || !buffers->grid_a || !buffers->grid_b || !buffers->scratch)
        return fail(nullptr, MPMQ_EINVAL, "packed, grid_a, grid_b and scratch buffers are required");
    const uintptr_t al = (uintptr_t)buffers->packed | (uintptr_t)buffers->grid_a | (uintptr_t)buffers->grid_b |
                         (uintptr_t)buffers->scratch | (uintptr_t)buffers->ids;
    if (al & 255u) return fail(nullptr, MPMQ_EINVAL, "buffers must be 256-byte aligned");
    mpmq_ctx *c = new mpmq_ctx();
    int bits = 0;
    std::string err;
    compile_scheme(scheme, c->ds, bits, err);
    compile_params(params, c->ds.dim, c->dp, err);
    c->params = *params;
    c->dim = c->ds.dim;
    c->W = c->ds.W;
    c->record_bits = bits;
    c->cap = capacity;
    c->cap_pad = sz.capacity_padded;
    c->stream = (hipStream_t)hip_stream;
    c->words = (uint32_t *)buffers->packed;
    c->grid[0] = (GNode *)buffers->grid_a;
    c->grid[1] = (GNode *)buffers->grid_b;
    c->scratch = (char *)buffers->scratch;
    c->ids = (uint32_t *)buffers->ids;
    c->sp = plan_scratch(c->dim, c->dp.res, c->cap_pad);
    hipError_t e = hipMemsetAsync(c->grid[0], 0, sz.grid_bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->grid[1], 0, sz.grid_bytes, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->scratch + c->sp.flags, 0, 4 * 2 * c->sp.nblocks, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->scratch + c->sp.stats, 0, 8 * ST_COUNT, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(c->scratch + c->sp.misc, 0, 256, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->scratch + c->sp.scheme, &c->ds, sizeof(DevScheme), hipMemcpyHostToDevice, c->stream);
    BatchDesc &bd = c->bdesc;
    bd.scheme = c->dscheme();
    bd.words = c->words;
    bd.cap = c->cap_pad;
    bd.items = c->items();
    bd.n_items = c->n_items();
    bd.grid[0] = c->grid[0];
    bd.grid[1] = c->grid[1];
    bd.flags[0] = c->flags(0);
    bd.flags[1] = c->flags(1);
    bd.stats = c->stats();
    bd.iscale = c->iscale();
    bd.irec = c->irec();
    bd.nblocks = c->sp.nblocks;
    bd.P = c->dp;
    if (e == hipSuccess) e = hipMemcpyAsync(c->scratch + c->sp.batch, &bd, sizeof(BatchDesc), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        g_last_error = std::string("create: ") + hipGetErrorString(e);
        delete c;
        return MPMQ_EDEVICE;
    }
    *out = c;
    return MPMQ_OK;
}

mpmq_status mpmq_destroy(mpmq_ctx *ctx) {
    if (!ctx) return MPMQ_OK;
    for (auto &ev : ctx->events) {
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    delete ctx;
    return MPMQ_OK;
}

mpmq_status mpmq_encode(mpmq_ctx *c, const float *x, const float *v, const float *C, const float *F, int64_t n) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    if (n < 0 || n > c->cap) return fail(c, MPMQ_ENOMEM, "n exceeds capacity");
    if (n > 0 && (!x || !v || !C || !F)) return fail(c, MPMQ_EINVAL, "x, v, C and F are required");
    {
        Timed t(c, "encode");
        HIPCHK(c, launch_encode(c->dim, c->ds.mat, c->dscheme(), x, v, C, F, n, c->cap_pad, c->words, c->ids,
                                (uint32_t)c->step, 2u, c->stats(), c->stream), "encode");
    }
    c->n = n;
    c->encoded = true;
    c->sorted = false;
    c->scales_valid = false;
    return MPMQ_OK;
}

mpmq_status mpmq_decode(mpmq_ctx *c, float *x, float *v, float *C, float *F) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    if (!c->encoded) return fail(c, MPMQ_ESTATE, "decode before encode");
    Timed t(c, "decode");
    HIPCHK(c, launch_decode(c->dim, c->ds.mat, c->dscheme(), c->words, c->n, c->cap_pad, x, v, C, F, c->stream), "decode");
    return MPMQ_OK;
}

mpmq_status mpmq_packed(mpmq_ctx *c, const uint32_t **words, int32_t *W, int64_t *n, int64_t *stride) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    if (words) *words = c->words;
    if (W) *W = c->W;
    if (n) *n = c->n;
    if (stride) *stride = c->cap_pad;
    return MPMQ_OK;
}

mpmq_status mpmq_step(mpmq_ctx *c, int32_t n_substeps) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    if (n_substeps < 0) return fail(c, MPMQ_EINVAL, "n_substeps < 0");
    if (!c->encoded) return fail(c, MPMQ_ESTATE, "step before encode");
    if (c->n == 0) {
        c->step += n_substeps;
        c->steps_taken += n_substeps;
        return MPMQ_OK;
    }
    for (int32_t it = 0; it < n_substeps; ++it) {
        mpmq_status r = substep_once(c, true);
        if (r != MPMQ_OK) return r;
    }
    return MPMQ_OK;
}

mpmq_status mpmq_step_batch(mpmq_ctx *const *ctxs, int32_t count, int32_t n_substeps) {
    if (!ctxs || count < 1) return fail(nullptr, MPMQ_EINVAL, "ctxs is NULL or count < 1");
    if (n_substeps < 0) return fail(nullptr, MPMQ_EINVAL, "n_substeps < 0");
    mpmq_ctx *c0 = ctxs[0];
    if (!c0) return fail(nullptr, MPMQ_EINVAL, "ctxs[0] is NULL");
    std::vector<const mpmq_ctx *> seen;
    for (int i = 0; i < count; ++i) {
        mpmq_ctx *c = ctxs[i];
        if (!c) return fail(c0, MPMQ_EINVAL, "ctxs[" + std::to_string(i) + "] is NULL");
        if (c->dim != c0->dim || c->ds.mat != c0->ds.mat)
            return fail(c0, MPMQ_EINVAL, "batched contexts must share the dimension and the material");
        if (c->stream != c0->stream) return fail(c0, MPMQ_EINVAL, "batched contexts must share one stream");
        if (!c->encoded) return fail(c0, MPMQ_ESTATE, "step before encode (ctxs[" + std::to_string(i) + "])");
        seen.push_back(c);
    }
    std::sort(seen.begin(), seen.end());
    if (std::adjacent_find(seen.begin(), seen.end()) != seen.end())
        return fail(c0, MPMQ_EINVAL, "a context appears twice in the batch");
    for (int32_t s = 0; s < n_substeps; ++s) {
        mpmq_status r = batch_substep(ctxs, count);
        if (r != MPMQ_OK) return r;
    }
    return MPMQ_OK;
}

mpmq_status mpmq_calib_atomics(uint64_t *buf, int64_t n_words, int32_t passes, int64_t stride, void *hip_stream) {
    if (!buf || n_words < 1 || passes < 1 || stride < 1 || ((uintptr_t)buf & 255u))
        return fail(nullptr, MPMQ_EINVAL, "calib_atomics: need an aligned buffer, n_words, passes, stride >= 1");
    const hipError_t e = launch_calib_atomics(reinterpret_cast<unsigned long long *>(buf), n_words, passes, stride,
                                              (hipStream_t)hip_stream);
    if (e != hipSuccess) return fail(nullptr, MPMQ_EDEVICE, std::string("calib_atomics: ") + hipGetErrorString(e));
    return MPMQ_OK;
}

mpmq_status mpmq_step_count(mpmq_ctx *c, int64_t *out) {
    if (!c || !out) return fail(c, MPMQ_EINVAL, "ctx or out is NULL");
    *out = c->step;
    return MPMQ_OK;
}

mpmq_status mpmq_stats(mpmq_ctx *c, mpmq_stats_t *out) {
    if (!c || !out) return fail(c, MPMQ_EINVAL, "ctx or out is NULL");
    uint64_t h[ST_COUNT];
    HIPCHK(c, hipMemcpyAsync(h, c->stats(), sizeof(h), hipMemcpyDeviceToHost, c->stream), "stats");
    HIPCHK(c, hipStreamSynchronize(c->stream), "stats");
    for (int f = 0; f < 4; ++f) {
        out->sat[f] = (int64_t)h[ST_SAT + f];
        out->nan[f] = (int64_t)h[ST_NAN + f];
        out->up[f] = (int64_t)h[ST_UP + f];
        out->down[f] = (int64_t)h[ST_DOWN + f];
    }
    out->steps = c->steps_taken;
    out->sorts = c->sorts;
    out->fallback = (int64_t)h[ST_FALLBACK];
    out->clamped = (int64_t)h[ST_CLAMP];
    out->atomics = (int64_t)h[ST_ATOMICS];
    out->wide = (int64_t)h[ST_WIDE];
    out->active_nodes = 0;
    for (int i = 0; i < ST_ACTIVE_SLOTS; ++i) out->active_nodes += (int64_t)h[ST_ACTIVE + i];
    return MPMQ_OK;
}

mpmq_status mpmq_reset_stats(mpmq_ctx *c) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t *>(c->stats()), 0u, 2 * ST_COUNT, c->stream), "reset stats");
    c->steps_taken = 0;
    c->sorts = 0;
    return MPMQ_OK;
}

mpmq_status mpmq_set_stats(mpmq_ctx *c, int32_t level) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    if (level < 0 || level > 1) return fail(c, MPMQ_EINVAL, "stats level must be 0 or 1");
    c->stats_level = level;
    return MPMQ_OK;
}

mpmq_status mpmq_specialize(mpmq_ctx *c, int32_t enable) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    if (!enable) {
        c->use_jit = false;
        return MPMQ_OK;
    }
    std::string err;
    JitKernels k{};
    if (!jit_kernels(c->dim, c->ds, c->dp, c->cap_pad, &k, &err)) return fail(c, MPMQ_EDEVICE, "specialize: " + err);
    c->jit = k;
    // the generic fused kernel keeps no item records: until the next P2G
    // outside it, the specialized one starts from "no record" (-1)
    if (!c->use_jit)
        HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t *>(c->irec()), 0xbf800000u, 4 * c->sp.max_items, c->stream),
               "specialize: records");
    c->use_jit = true;
    return MPMQ_OK;
}

mpmq_status mpmq_set_timing(mpmq_ctx *c, int32_t enable) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    c->timing = enable != 0;
    return MPMQ_OK;
}

mpmq_status mpmq_kernel_times(mpmq_ctx *c, mpmq_kernel_time *out, int32_t max, int32_t *count) {
    if (!c) return fail(nullptr, MPMQ_EINVAL, "ctx is NULL");
    HIPCHK(c, hipStreamSynchronize(c->stream), "kernel times");
    for (auto &ev : c->events) {
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, ev.a, ev.b), "kernel times");
        auto &slot = c->times[ev.name];
        slot.first += 1;
        slot.second += ms;
        (void)hipEventDestroy(ev.a);
        (void)hipEventDestroy(ev.b);
    }
    c->events.clear();
    int32_t i = 0;
    for (auto &kv : c->times) {
        if (out && i < max) {
            std::memset(out[i].name, 0, sizeof(out[i].name));
            std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
            out[i].launches = kv.second.first;
            out[i].total_ms = kv.second.second;
        }
        ++i;
    }
    if (count) *count = i;
    if (max < 0) c->times.clear();
    return MPMQ_OK;
}

mpmq_status mpmq_adjoint_workspace(mpmq_ctx *c, const mpmq_adjoint_spec *spec, int64_t *bytes) {
    if (!c || !bytes) return fail(c, MPMQ_EINVAL, "ctx or bytes is NULL");
    mpmq_status r = check_spec(c, spec);
    if (r != MPMQ_OK) return r;
    *bytes = adj_layout(c, adj_plan(spec->steps, spec->checkpoint_every)).total;
    return MPMQ_OK;
}

}  // extern "C"

namespace {

mpmq_status adjoint_impl(mpmq_ctx *c, const mpmq_adjoint_spec *spec, void *workspace, int64_t workspace_bytes,
                         float *lambda0, mpmq_adjoint_result *out) {
    if (!c || !out) return fail(c, MPMQ_EINVAL, "ctx or out is NULL");
    mpmq_status r = check_spec(c, spec);
    if (r != MPMQ_OK) return r;
    if (!c->encoded) return fail(c, MPMQ_ESTATE, "adjoint before encode");
    const int64_t T = spec->steps;
    const AdjPlan plan = adj_plan(T, spec->checkpoint_every);
    AdjRun run;
    run.c = c;
    run.w = adj_layout(c, plan);
    if (!workspace || workspace_bytes < run.w.total) return fail(c, MPMQ_ENOMEM, "adjoint workspace too small");
    if ((uintptr_t)workspace & 255u) return fail(c, MPMQ_EINVAL, "workspace must be 256-byte aligned");
    std::memset(out, 0, sizeof(*out));
    hipStream_t st = c->stream;
    const int64_t n = c->n;
    const int rows = adj_rows(c->dim, c->ds.mat);
    if (n == 0) {
        c->step += T;
        c->steps_taken += T;
        return MPMQ_OK;
    }
    run.ws = (char *)workspace;
    run.step0 = c->step;
    run.lam_cur = reinterpret_cast<float *>(run.ws + run.w.off_lam);
    run.lam_nxt = reinterpret_cast<float *>(run.ws + run.w.off_lam + run.w.lam_bytes);
    for (int s = (int)plan.slots - 1; s >= 0; --s) run.free_slots.push_back(s);
    run.fin = (int)plan.slots;
    run.valid.assign((size_t)plan.slots + 1, 0);
    HIPCHK(c, launch_fill_u32(reinterpret_cast<uint32_t *>(run.acc()), 0u, 2 * ADJ_ACC_DOUBLES, st), "adjoint: clear");
    HIPCHK(c, launch_fill_u32(run.rng(), 0xffffffffu, 4 * ADJ_SLOTS, st), "adjoint: clear");
    HIPCHK(c, launch_fill_u32(run.rng() + 4 * ADJ_SLOTS, 0u, 4 * ADJ_SLOTS, st), "adjoint: clear");
    // forward: sort once if pending, then T substeps without re-sorting
    if (!c->sorted) {
        if (c->p2g_ready) {
            HIPCHK(c, launch_clear_touched(c->dim, c->grid[c->step & 1], c->flags((int)(c->step & 1)), c->sp.nblocks, st),
                   "clear");
            c->p2g_ready = false;
        }
        if ((r = do_sort(c)) != MPMQ_OK) return r;
        c->sorted = true;
        c->sorted_at = c->step;
    }
    size_t save_i = 0;
    for (int64_t t = 0; t <= T; ++t) {
        HIPCHK(c, launch_adj_range(c->dim, c->ds.mat, c->dscheme(), c->words, c->cap_pad, n, run.rng(), st), "adjoint: ranges");
        if (save_i < plan.forward_saves.size() && plan.forward_saves[save_i] == t) {
            const int s = run.take();
            if ((r = run.save(s)) != MPMQ_OK) return r;
            run.saved[t] = s;
            ++save_i;
        }
        if (t < T && (r = substep_once(c, false)) != MPMQ_OK) return r;
    }
    const int64_t steps_after = c->steps_taken;
    HIPCHK(c, launch_copy_u32(reinterpret_cast<uint32_t *>(c->stats()), reinterpret_cast<uint32_t *>(run.ws + run.w.off_stats),
                              2 * ST_COUNT, st), "adjoint: stats");
    if ((r = run.save(run.fin)) != MPMQ_OK) return r;
    // objective at s_T and lambda_T
    HIPCHK(c, launch_adj_objective(c->dim, c->ds.mat, c->dscheme(), c->dp, c->words, c->cap_pad, n, spec->objective, spec->axis,
                                   run.lam_cur, run.acc(), st), "adjoint: objective");
    HIPCHK(c, launch_adj_reduce(c->dim, c->ds.mat, run.lam_cur, n, run.acc(), st), "adjoint: reduce");
    // backward
    if (T > 0) {
        if (spec->checkpoint_every >= 1) {
            const int64_t K = spec->checkpoint_every;
            const int64_t nseg = (T + K - 1) / K;
            for (int64_t sg = nseg - 1; sg >= 0; --sg) {
                const int64_t a = sg * K, b = std::min<int64_t>(a + K, T);
                const int slot_a = run.saved.at(a);
                if ((r = run.reverse_segment(a, b, slot_a)) != MPMQ_OK) return r;
                run.saved.erase(a);
                run.give(slot_a);
            }
        } else {
            const int slot0 = run.saved.at(0);
            run.saved.erase(0);
            if ((r = run.reverse_bisect(0, T, slot0)) != MPMQ_OK) return r;
            run.give(slot0);
        }
    }
    if (lambda0) {
        if (c->ids) {
            HIPCHK(c, launch_adj_unpermute(run.lam_cur, c->ids, n, rows, lambda0, st), "adjoint: lambda0");
        } else {
            HIPCHK(c, launch_copy_u32(reinterpret_cast<const uint32_t *>(run.lam_cur), reinterpret_cast<uint32_t *>(lambda0),
                                      (int64_t)rows * n, st), "adjoint: lambda0");
        }
    }
    // restore s_T, the step counter and the statistics of the forward pass
    if ((r = run.load(run.fin)) != MPMQ_OK) return r;
    if ((r = reset_grids(c)) != MPMQ_OK) return r;  // the next substep's P2G replays the recorded scales
    HIPCHK(c, launch_copy_u32(reinterpret_cast<uint32_t *>(run.ws + run.w.off_stats), reinterpret_cast<uint32_t *>(c->stats()),
                              2 * ST_COUNT, st), "adjoint: stats");
    c->step = run.step0 + T;
    c->steps_taken = steps_after;
    std::vector<double> acc(ADJ_ACC_DOUBLES);
    std::vector<uint32_t> rng(8 * ADJ_SLOTS);
    HIPCHK(c, hipMemcpyAsync(acc.data(), run.acc(), sizeof(double) * acc.size(), hipMemcpyDeviceToHost, st),
           "adjoint: result");
    HIPCHK(c, hipMemcpyAsync(rng.data(), run.rng(), sizeof(uint32_t) * rng.size(), hipMemcpyDeviceToHost, st),
           "adjoint: result");
    HIPCHK(c, hipStreamSynchronize(st), "adjoint: sync");
    out->z = acc[0];
    for (int f = 0; f < 4; ++f) {
        // combine the ADJ_SLOTS copies, in slot order
        double G = 0.0, g = 0.0;
        uint32_t klo = 0xffffffffu, khi = 0u;
        for (int sl = 0; sl < ADJ_SLOTS; ++sl) {
            G += acc[1 + 8 * sl + f];
            g += acc[1 + 8 * sl + 4 + f];
            klo = std::min(klo, rng[4 * sl + f]);
            khi = std::max(khi, rng[4 * ADJ_SLOTS + 4 * sl + f]);
        }
        auto unkey = [](uint32_t k) {
            const uint32_t u = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
            float v;
            std::memcpy(&v, &u, 4);
            return (double)v;
        };
        out->G[f] = G;
        out->g[f] = g;
        out->lo[f] = unkey(klo);
        out->hi[f] = unkey(khi);
    }
    out->recomputed = run.recomputed;
    out->states = run.max_live + 1;
    return MPMQ_OK;
}

}  // namespace

extern "C" {

mpmq_status mpmq_adjoint(mpmq_ctx *c, const mpmq_adjoint_spec *spec, void *workspace, int64_t workspace_bytes,
                         float *lambda0, mpmq_adjoint_result *out) {
    return adjoint_impl(c, spec, workspace, workspace_bytes, lambda0, out);
}

}  // extern "C"

// ---- allocation-free adjoint ----
// A file-scope device array serves as the adjoint workspace of
// mpmq_adjoint_static.  In host code the name `scratch` denotes a host-side
// stand-in, not a device address: the device address is obtained once per
// device with hipGetSymbolAddress (that device current) and only that
// address is handed to the kernels.
static __device__ __align__(256) unsigned char scratch[MPMQ_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device).
mpmq_status static_workspace(mpmq_ctx *c, void **out) {
    int dev = 0;
    HIPCHK(c, hipGetDevice(&dev), "static workspace: hipGetDevice");
    if (dev < 0 || dev >= kMaxDevices) return fail(c, MPMQ_EDEVICE, "static workspace: device index out of range");
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "static workspace: hipGetSymbolAddress");
        if (!p) return fail(c, MPMQ_EDEVICE, "static workspace: no device address");
        g_static_ptr[dev] = p;
    }
    *out = g_static_ptr[dev];
    return MPMQ_OK;
}

}  // namespace

extern "C" {

mpmq_status mpmq_adjoint_static(mpmq_ctx *c, const mpmq_adjoint_spec *spec, float *lambda0,
                                mpmq_adjoint_result *out) {
    if (!c || !out) return fail(c, MPMQ_EINVAL, "ctx or out is NULL");
    mpmq_status r = check_spec(c, spec);
    if (r != MPMQ_OK) return r;
    const int64_t need = adj_layout(c, adj_plan(spec->steps, spec->checkpoint_every)).total;
    if (need > (int64_t)MPMQ_STATIC_WORKSPACE_BYTES)
        return fail(c, MPMQ_ENOMEM, "adjoint needs a workspace of " + std::to_string(need) +
                                        " bytes; the static workspace holds " +
                                        std::to_string((int64_t)MPMQ_STATIC_WORKSPACE_BYTES));
    void *ws = nullptr;
    if ((r = static_workspace(c, &ws)) != MPMQ_OK) return r;
    return adjoint_impl(c, spec, ws, (int64_t)MPMQ_STATIC_WORKSPACE_BYTES, lambda0, out);
}

}  // extern "C"
