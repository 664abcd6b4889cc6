// solver.hip -- host-only: the automatic quantization solver (Sec. 4,
// Eqs. 6-10, Alg. 1).  Given, per data type h, the number of variables P_h,
// the accumulated squared gradient g_h of Eq. 8 and the range width R_h, it
// returns the quantization step Delta_h and the bit width b_h.
//
//   error-bounded:  Delta_h = sqrt(12 P_h (eps z)^2 / (g_h sum P)),
//                   b_h = ceil(log2(R_h / Delta_h))            (Eq. 10, Alg. 1)
//   memory-bounded: minimize (1/12) sum Delta_h^2 g_h subject to
//                   sum P_h b_h <= eps M, M = 32 sum P (Eq. 7).  Lagrange:
//                   Delta_h = K sqrt(P_h / g_h) with K set by the active
//                   constraint; b_h = floor(log2(R_h / Delta_h)) so that the
//                   bound holds for the integer widths.
// Types with g_h = 0 take min_bits (and leave the memory budget first).
#include "../../include/mpmq.h"

#include <cmath>
#include <string>

namespace {
thread_local std::string g_solver_error;
}

extern "C" const char *mpmq_solver_error(void) { return g_solver_error.c_str(); }

extern "C" mpmq_status mpmq_solve_scheme(const mpmq_solve_input *in, mpmq_solve_output *out) {
    auto bad = [](const char *m) {
        g_solver_error = m;
        return MPMQ_EINVAL;
    };
    if (!in || !out) return bad("in or out is NULL");
    const int H = in->n_types;
    if (H < 1 || H > MPMQ_SOLVE_MAX_TYPES) return bad("n_types must be in [1, 16]");
    if (in->min_bits < 1 || in->max_bits > 32 || in->min_bits > in->max_bits) return bad("need 1 <= min_bits <= max_bits <= 32");
    if (!(in->eps > 0.0) || !std::isfinite(in->eps)) return bad("eps must be finite and > 0");
    if (in->mode != MPMQ_SOLVE_ERROR_BOUND && in->mode != MPMQ_SOLVE_MEMORY_BOUND) return bad("unknown mode");
    for (int h = 0; h < H; ++h) {
        if (!(in->P[h] > 0.0) || !std::isfinite(in->P[h])) return bad("P_h must be finite and > 0");
        if (!(in->R[h] > 0.0) || !std::isfinite(in->R[h])) return bad("R_h must be finite and > 0");
        if (!(in->g[h] >= 0.0) || !std::isfinite(in->g[h])) return bad("g_h must be finite and >= 0");
    }
    double sumP = 0.0;
    for (int h = 0; h < H; ++h) sumP += in->P[h];
    auto clampb = [&](double b) {
        if (b < in->min_bits) return in->min_bits;
        if (b > in->max_bits) return in->max_bits;
        return (int32_t)b;
    };
    for (int h = 0; h < H; ++h) {
        out->delta[h] = INFINITY;
        out->b_cont[h] = -INFINITY;
        out->bits[h] = in->min_bits;
    }
    if (in->mode == MPMQ_SOLVE_ERROR_BOUND) {
        const double t = in->eps * in->z;
        if (!(t * t > 0.0) || !std::isfinite(t)) return bad("error-bounded mode needs a finite z != 0");
        for (int h = 0; h < H; ++h) {
            if (!(in->g[h] > 0.0)) continue;
            const double d = std::sqrt(12.0 * in->P[h] * t * t / (in->g[h] * sumP));
            const double b = std::log2(in->R[h] / d);
            out->delta[h] = d;
            out->b_cont[h] = b;
            out->bits[h] = clampb(std::ceil(b));
        }
    } else {
        double budget = in->eps * 32.0 * sumP, live_P = 0.0, acc_R = 0.0, acc_Pg = 0.0;
        for (int h = 0; h < H; ++h) {
            if (in->g[h] > 0.0) {
                live_P += in->P[h];
                acc_R += in->P[h] * std::log2(in->R[h]);
                acc_Pg += in->P[h] * std::log2(in->P[h] / in->g[h]);
            } else {
                budget -= in->P[h] * in->min_bits;
            }
        }
        if (live_P > 0.0) {
            const double log2K = (acc_R - 0.5 * acc_Pg - budget) / live_P;
            for (int h = 0; h < H; ++h) {
                if (!(in->g[h] > 0.0)) continue;
                const double d = std::exp2(log2K) * std::sqrt(in->P[h] / in->g[h]);
                const double b = std::log2(in->R[h] / d);
                out->delta[h] = d;
                out->b_cont[h] = b;
                out->bits[h] = clampb(std::floor(b));
            }
        }
    }
    double e = 0.0, mem = 0.0;
    for (int h = 0; h < H; ++h) {
        const double d = std::ldexp(in->R[h], -out->bits[h]);
        e += d * d * in->g[h];
        mem += in->P[h] * out->bits[h];
    }
    out->expected_error = e / 12.0;
    out->total_bits = mem;
    return MPMQ_OK;
}

// Alg. 1 from a recorded run (see mpmq_auto_scheme in mpmq.h): ranges
// widened about their centre (Sec. 3.2), P_h = particles x components,
// then the closed-form widths above.
extern "C" mpmq_status mpmq_auto_scheme(const mpmq_scheme *base, const mpmq_adjoint_result *adj,
                                        const mpmq_auto_input *in, mpmq_field_scheme *out_fields,
                                        mpmq_solve_output *solved) {
    auto bad = [](const char *m) {
        g_solver_error = m;
        return MPMQ_EINVAL;
    };
    if (!base || !base->fields || !adj || !in || !out_fields) return bad("base, adj, in and out_fields are required");
    if (base->dim != 2 && base->dim != 3) return bad("base scheme dim must be 2 or 3");
    if (base->n_fields != 4) return bad("base scheme must list 4 fields");
    if (in->n_particles < 1) return bad("n_particles must be >= 1");
    if (!(in->range_factor >= 1.0) || !std::isfinite(in->range_factor)) return bad("range_factor must be finite and >= 1");
    const int dim = base->dim;
    // slot of each base field (F and J share slot 3), each slot once
    int slot_field[4] = {-1, -1, -1, -1};
    for (int i = 0; i < 4; ++i) {
        const int f = base->fields[i].field;
        if (f < MPMQ_FIELD_X || f > MPMQ_FIELD_J) return bad("unknown field in base scheme");
        const int sl = f == MPMQ_FIELD_J ? 3 : f;
        if (slot_field[sl] >= 0) return bad("base scheme lists a field twice");
        slot_field[sl] = i;
    }
    double P[4], g[4], R[4], lo[4], hi[4];
    for (int sl = 0; sl < 4; ++sl) {
        const int f = base->fields[slot_field[sl]].field;
        const int nc = (f == MPMQ_FIELD_X || f == MPMQ_FIELD_V) ? dim : f == MPMQ_FIELD_J ? 1 : dim * dim;
        if (!std::isfinite(adj->lo[sl]) || !std::isfinite(adj->hi[sl]) || adj->hi[sl] < adj->lo[sl])
            return bad("recorded ranges must be finite with lo <= hi");
        const double mid = 0.5 * (adj->lo[sl] + adj->hi[sl]);
        // a constant field (zero recorded width) gets +-2^-20 max(1, |centre|)
        const double half = std::fmax(0.5 * (adj->hi[sl] - adj->lo[sl]) * in->range_factor,
                                      std::ldexp(std::fmax(1.0, std::fabs(mid)), -20));
        lo[sl] = mid - half;
        hi[sl] = mid + half;
        P[sl] = (double)in->n_particles * nc;
        g[sl] = adj->g[sl];
        R[sl] = hi[sl] - lo[sl];
    }
    double delta[4], bcont[4];
    int32_t bits[4];
    mpmq_solve_output o{delta, bcont, bits, 0.0, 0.0};
    const mpmq_solve_input si{in->mode, 4, in->min_bits, in->max_bits, in->eps, adj->z, P, g, R};
    const mpmq_status st = mpmq_solve_scheme(&si, &o);
    if (st != MPMQ_OK) return st;
    for (int sl = 0; sl < 4; ++sl) {
        const int i = slot_field[sl];
        const mpmq_field_scheme &b = base->fields[i];
        mpmq_field_scheme &f = out_fields[i];
        f.field = b.field;
        f.kind = MPMQ_FIXED;
        f.bits = bits[sl];
        f.exp_bits = 0;
        f.dither = b.dither;
        f.flags = b.flags & MPMQ_REL_IDENTITY;
        f.lo = lo[sl];
        f.hi = hi[sl];
        if (solved) {
            if (solved->delta) solved->delta[sl] = delta[sl];
            if (solved->b_cont) solved->b_cont[sl] = bcont[sl];
            if (solved->bits) solved->bits[sl] = bits[sl];
        }
    }
    if (solved) {
        solved->expected_error = o.expected_error;
        solved->total_bits = o.total_bits;
    }
    return MPMQ_OK;
}
