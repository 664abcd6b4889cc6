// adjoint.hip -- gfx950 adjoint kernels of the quantized MLS-MPM substep
// (Sec. 6, Eqs. 12-13): lambda_t = (d s'_{t+1} / d s_t)^T lambda_{t+1}, with
// the quantization error treated as an additive perturbation of the stored
// state (straight-through), so d z / d e_t = lambda_t.  Their sums over
// steps, particles and components give the per-field sensitivities G_h and
// the accumulated squared gradients g_h of Eq. 8.
//
// Adjoint state layout: float32 SoA, L = 2d + 2d^2 rows of n:
// x[d], v[d], C[d*d], F[d*d].  Node adjoints: float4 per node (the grid's
// block-major node order).
#include "substep.hpp"  // tile helpers, work-item walk (includes mpmq_device.hpp)

namespace mpmq {

// waves per SIMD the G2P backward is built for (caps its registers)
constexpr int ADJ_WAVES_PER_EU = 2;

template <int DIM, int MAT> constexpr int LROWS() { return 2 * DIM + DIM * DIM + nc3<DIM, MAT>(); }

// d w / d x_a for a node with offsets o: inv_dx N'_{o_a}(f_a) prod_{b!=a} N_{o_b}(f_b)
__device__ __forceinline__ void bspline_d(float f, float inv_dx, float *dw) {
    dw[0] = -(1.5f - f) * inv_dx;
    dw[1] = -2.0f * (f - 1.0f) * inv_dx;
    dw[2] = (f - 0.5f) * inv_dx;
}

template <int DIM>
__device__ __forceinline__ float det_f(const float *F) {
    if constexpr (DIM == 2) return F[0] * F[3] - F[1] * F[2];
    else
        return F[0] * (F[4] * F[8] - F[5] * F[7]) - F[1] * (F[3] * F[8] - F[5] * F[6]) +
               F[2] * (F[3] * F[7] - F[4] * F[6]);
}

template <int DIM>
__device__ __forceinline__ void cofactor_f(const float *F, float *Cf) {
    if constexpr (DIM == 2) {
        Cf[0] = F[3]; Cf[1] = -F[2]; Cf[2] = -F[1]; Cf[3] = F[0];
    } else {
        Cf[0] = F[4] * F[8] - F[5] * F[7];
        Cf[1] = F[5] * F[6] - F[3] * F[8];
        Cf[2] = F[3] * F[7] - F[4] * F[6];
        Cf[3] = F[2] * F[7] - F[1] * F[8];
        Cf[4] = F[0] * F[8] - F[2] * F[6];
        Cf[5] = F[1] * F[6] - F[0] * F[7];
        Cf[6] = F[1] * F[5] - F[2] * F[4];
        Cf[7] = F[2] * F[3] - F[0] * F[5];
        Cf[8] = F[0] * F[4] - F[1] * F[3];
    }
}

// lamF += (d tau / d F)^T [lt] for tau = 2 mu (F - R) F^T + la J (J-1) I.
// dR = R Y with Y skew solving S Y + Y S = skew(R^T dF - dF^T R), F = R S;
// the adjoint of the dR term is -4 mu R Y' with S Y' + Y' S = skew(R^T lt F)
// (3D: S[y]x + [y]x S = [(tr S I - S) y]x; 2D: S Y + Y S = tr(S) Y).
template <int DIM>
__device__ __forceinline__ void stress_vjp(const DevParams &P, const float *F, const float *lt, float *lamF) {
    constexpr int D2 = DIM * DIM;
    float R[D2], S[D2], Cf[D2];
    if constexpr (DIM == 2) polar2(F, R);
    else polar3<true>(F, R);
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) a += R[k * DIM + i] * F[k * DIM + j];
            S[i * DIM + j] = a;
        }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = i + 1; j < DIM; ++j) {
            const float a = 0.5f * (S[i * DIM + j] + S[j * DIM + i]);
            S[i * DIM + j] = a;
            S[j * DIM + i] = a;
        }
    cofactor_f<DIM>(F, Cf);
    const float J = det_f<DIM>(F);
    float tr_lt = 0.0f;
#pragma unroll
    for (int i = 0; i < DIM; ++i) tr_lt += lt[i * DIM + i];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            float a = 0.0f, b = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) {
                a += lt[i * DIM + k] * F[k * DIM + j];
                b += lt[k * DIM + i] * (F[k * DIM + j] - R[k * DIM + j]);
            }
            lamF[i * DIM + j] += 2.0f * P.mu * (a + b) + P.la * (2.0f * J - 1.0f) * tr_lt * Cf[i * DIM + j];
        }
    float M[D2];
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k)
#pragma unroll
                for (int l = 0; l < DIM; ++l) a += R[k * DIM + i] * lt[k * DIM + l] * F[l * DIM + j];
            M[i * DIM + j] = a;
        }
    float Y[D2];
#pragma unroll
    for (int i = 0; i < D2; ++i) Y[i] = 0.0f;
    if constexpr (DIM == 2) {
        const float b = 0.5f * (M[2] - M[1]);
        const float tr = S[0] + S[3];
        const float y = (tr != 0.0f) ? b / tr : 0.0f;
        Y[1] = -y;
        Y[2] = y;
    } else {
        const float b[3] = {0.5f * (M[7] - M[5]), 0.5f * (M[2] - M[6]), 0.5f * (M[3] - M[1])};
        const float tr = S[0] + S[4] + S[8];
        float A[9];
#pragma unroll
        for (int i = 0; i < 9; ++i) A[i] = -S[i];
        A[0] += tr;
        A[4] += tr;
        A[8] += tr;
        float cof[9];
        cofactor_f<3>(A, cof);
        const float dA = det_f<3>(A);
        float y[3] = {0.0f, 0.0f, 0.0f};
        if (dA != 0.0f) {
#pragma unroll
            for (int i = 0; i < 3; ++i) y[i] = (cof[i] * b[0] + cof[3 + i] * b[1] + cof[6 + i] * b[2]) / dA;
        }
        Y[1] = -y[2]; Y[2] = y[1];
        Y[3] = y[2]; Y[5] = -y[0];
        Y[6] = -y[1]; Y[7] = y[0];
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
        for (int j = 0; j < DIM; ++j) {
            float a = 0.0f;
#pragma unroll
            for (int k = 0; k < DIM; ++k) a += R[i * DIM + k] * Y[k * DIM + j];
            lamF[i * DIM + j] += -4.0f * P.mu * a;
        }
}

template <int DIM>
__device__ __forceinline__ void stencil_all(const DevParams &P, const double *xd, int *base, float *fx,
                                            float (*w)[3], float (*dw)[3]) {
    stencil_base<DIM>(xd, P.inv_dx_d, P.res, base, fx);
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        bspline(fx[a], w[a]);
        bspline_d(fx[a], P.inv_dx, dw[a]);
    }
}

// lambda_t contributions that reach the node adjoints: lambda_v' and
// lambda_C' of particle p, with the VJP of F' = (I + dt C') F (fluid:
// J' = J (1 + dt tr C')) added to lambda_C' and that of x' = x + dt v' to
// lambda_v'.  Also returns lambda_x' and lambda_F' as read.
template <int DIM, int MAT>
__device__ __forceinline__ void adj_lambda_in(const DevParams &P, const float *__restrict__ lin, int64_t n,
                                              int64_t p, const float *F, float *lx, float *lv, float *lC,
                                              float *lF) {
    constexpr int D2 = DIM * DIM, N3 = nc3<DIM, MAT>();
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lx[a] = lin[a * n + p];
        lv[a] = lin[(DIM + a) * n + p];
    }
#pragma unroll
    for (int c = 0; c < D2; ++c) lC[c] = lin[(2 * DIM + c) * n + p];
#pragma unroll
    for (int c = 0; c < N3; ++c) lF[c] = lin[(2 * DIM + D2 + c) * n + p];
    if constexpr (MAT == 1) {
#pragma unroll
        for (int a = 0; a < DIM; ++a) lC[a * DIM + a] += lF[0] * F[0] * P.dt;
    } else {
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                float aC = 0.0f;
#pragma unroll
                for (int k = 0; k < DIM; ++k) aC += lF[i * DIM + k] * F[j * DIM + k];
                lC[i * DIM + j] += P.dt * aC;
            }
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) lv[a] += P.dt * lx[a];
}

// Bound on |w (lambda_v'_a + D sum_b lambda_C'_ab d_b)| over the stencil of a
// particle: w <= 1 and |d_b| <= 1.5 dx, so D |d_b| <= 6 / dx.
template <int DIM>
__device__ __forceinline__ float adj_node_bound(const DevParams &P, const float *lv, const float *lC) {
    float bmax = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        float sc = 0.0f;
#pragma unroll
        for (int b = 0; b < DIM; ++b) sc += fabsf(lC[a * DIM + b]);
        const float b = fabsf(lv[a]) + 6.0f * P.inv_dx * sc;
        bmax = (b > bmax || b != b) ? b : bmax;  // NaN propagates
    }
    return bmax;
}

// Fixed-point scale of the node-adjoint tile: contributions of magnitude
// below 2^e (e from the item's bound) map to integers below 2^46, so sums
// over up to 2^16 particles stay below 2^62 and the magic-number rounding of
// fixp (exact for |value| < 2^51) applies.
constexpr int ADJ_FIX_BITS = 46;

// Node adjoints of one particle's G2P: for each stencil node, lambda_v_i
// gains w (lambda_v' + D lambda_C' d), and the particle's lambda_x gains the
// weight-gradient and dpos terms.  TILE: node velocities come from the LDS
// tile `gv` and the node adjoints go to the LDS tile `tacc` (both with
// corner offset l0): as integers of scale `fs` when FIX, else as floats;
// otherwise both go straight to the grid buffers.
template <int DIM, bool TILE, bool FIX>
__device__ __forceinline__ void adj_g2p_nodes(const DevParams &P, const int *base, const float *fx,
                                              const float (*w)[3], const float (*dw)[3], const float *lv,
                                              const float *lC, const GNode *__restrict__ grid,
                                              const float *gv, int l0, unsigned long long *tacc, double fs,
                                              float4 *__restrict__ nadj, float *ox) {
    constexpr int NST = Geo<DIM>::NST, TB = Geo<DIM>::TB, TN = Geo<DIM>::TN;
    const float D = 4.0f * P.inv_dx * P.inv_dx;
#pragma unroll
    for (int st = 0; st < NST; ++st) {
        const int o[3] = {st % 3, (st / 3) % 3, st / 9};
        float wt = 1.0f, d[DIM], gw[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            wt *= w[a][o[a]];
            d[a] = ((float)o[a] - fx[a]) * P.dx;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            gw[a] = dw[a][o[a]];
#pragma unroll
            for (int b = 0; b < DIM; ++b)
                if (b != a) gw[a] *= w[b][o[b]];
        }
        float vi[3] = {0.0f, 0.0f, 0.0f};
        int lt = 0;
        float *na = nullptr;
        if constexpr (TILE) {
            lt = l0 + ((DIM == 3) ? (o[2] * TB + o[1]) * TB + o[0] : o[1] * TB + o[0]);
#pragma unroll
            for (int a = 0; a < DIM; ++a) vi[a] = gv[a * TN + lt];
        } else {
            int ijk[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) ijk[a] = base[a] + o[a];
            const int64_t id = node_index<DIM>(ijk, P.nb);
            const float4 g = node_vel<DIM>(grid, id);
            vi[0] = g.x;
            vi[1] = g.y;
            vi[2] = g.z;
            na = reinterpret_cast<float *>(nadj + id);
        }
        float lw = 0.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            float ld = 0.0f;
#pragma unroll
            for (int b = 0; b < DIM; ++b) ld += lC[a * DIM + b] * d[b];
            const float c = wt * (lv[a] + D * ld);
            if constexpr (TILE && FIX) atomicAdd(&tacc[a * TN + lt], fixp((double)c, fs));
            else if constexpr (TILE) atomicAdd(reinterpret_cast<float *>(tacc) + a * TN + lt, c);
            else unsafeAtomicAdd(na + a, c);
            lw += lv[a] * vi[a] + D * vi[a] * ld;
#pragma unroll
            for (int b = 0; b < DIM; ++b) ox[b] -= D * wt * lC[a * DIM + b] * vi[a];
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) ox[a] += gw[a] * lw;
    }
}

// G2P backward of particle p: from lambda_{t+1} (of x', v', C', F') to the
// partial lambda_t of x and F, and the node adjoints lambda_v_i.  A particle
// whose stencil lies in the item's tile (corner `origin`) reads node
// velocities from the LDS tile `gv` and adds its node adjoints into the LDS
// tile `tacc` (3 x TN; integers of scale `fs` when `fix`, else floats); any
// other reads and adds the grid buffers.
template <int DIM, int MAT>
__device__ __forceinline__ void adj_g2p_particle(const DevScheme *__restrict__ sch, const DevParams &P,
                                                 const uint32_t *__restrict__ words, int64_t cap, int64_t n,
                                                 int64_t p, const GNode *__restrict__ grid,
                                                 const float *__restrict__ lin, float *__restrict__ lout,
                                                 float4 *__restrict__ nadj, const float *gv,
                                                 unsigned long long *tacc, bool fix, double fs,
                                                 const int *origin) {
    constexpr int D2 = DIM * DIM, N3 = nc3<DIM, MAT>();
    constexpr int TB = Geo<DIM>::TB;
    SchemeRef s = scheme_ref(sch);
    const uint32_t p4 = (uint32_t)p * 4u;
    double xd[DIM];
    float F[N3];
    dec_field<DIM, 0, double>(&s->f[0], words, cap, p4, xd);
    dec_field<DIM, fid3<MAT>(), float>(&s->f[3], words, cap, p4, F);
    int base[DIM];
    float fx[DIM], w[DIM][3], dw[DIM][3];
    stencil_all<DIM>(P, xd, base, fx, w, dw);
    bool in_tile = true;
    int l0 = 0;
#pragma unroll
    for (int a = DIM - 1; a >= 0; --a) {
        const int la = base[a] - origin[a];
        in_tile &= (la >= 0) && (la <= TB - 3);
        l0 = l0 * TB + la;
    }
    // recompute C' for the F' adjoint, as the forward G2P forms it
    float nv[DIM], S[DIM][DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        nv[a] = 0.0f;
#pragma unroll
        for (int b = 0; b < DIM; ++b) S[b][a] = 0.0f;
    }
    if (in_tile) {
        g2p_tile<DIM>(gv, l0, w, fx, nv, S);
    } else {
        float wd[DIM][3];  // w (o - f)
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int o = 0; o < 3; ++o) wd[a][o] = w[a][o] * ((float)o - fx[a]);
        g2p_global<DIM>(grid, P.nb, base, w, wd, nv, S);
    }
    float Cn[D2];
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int b = 0; b < DIM; ++b) Cn[a * DIM + b] = 4.0f * P.inv_dx * S[b][a];
    float lx[DIM], lv[DIM], lC[D2], lF[N3], oF[N3];
    adj_lambda_in<DIM, MAT>(P, lin, n, p, F, lx, lv, lC, lF);
    if constexpr (MAT == 1) {
        float tr = 0.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) tr += Cn[a * DIM + a];
        oF[0] = lF[0] * (1.0f + P.dt * tr);
    } else {
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                float aF = 0.0f;
#pragma unroll
                for (int k = 0; k < DIM; ++k)
                    aF += (((k == i) ? 1.0f : 0.0f) + P.dt * Cn[k * DIM + i]) * lF[k * DIM + j];
                oF[i * DIM + j] = aF;
            }
    }
    float ox[DIM];
#pragma unroll
    for (int a = 0; a < DIM; ++a) ox[a] = lx[a];
    if (in_tile) {
        if (fix) adj_g2p_nodes<DIM, true, true>(P, base, fx, w, dw, lv, lC, grid, gv, l0, tacc, fs, nadj, ox);
        else adj_g2p_nodes<DIM, true, false>(P, base, fx, w, dw, lv, lC, grid, gv, l0, tacc, fs, nadj, ox);
    } else {
        adj_g2p_nodes<DIM, false, false>(P, base, fx, w, dw, lv, lC, grid, gv, l0, tacc, fs, nadj, ox);
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lout[a * n + p] = ox[a];
        lout[(DIM + a) * n + p] = 0.0f;
    }
#pragma unroll
    for (int c = 0; c < D2; ++c) lout[(2 * DIM + c) * n + p] = 0.0f;
#pragma unroll
    for (int c = 0; c < N3; ++c) lout[(2 * DIM + D2 + c) * n + p] = oF[c];
}

// Per work item (the forward's sort): the item's node velocities are staged
// in an LDS tile; node adjoints of its particles accumulate in a second LDS
// tile, as 64-bit fixed point whose scale comes from a bound over the item's
// particles (exact, order-independent sums; LDS integer atomics are much
// cheaper than float ones), or as floats when that bound is not finite.  The
// tile is then added to `nadj` with one float atomic per non-zero node
// component.
template <int DIM, int MAT>
__global__ __launch_bounds__(WG, ADJ_WAVES_PER_EU) void k_adj_g2p(const DevScheme *__restrict__ sch, DevParams P,
                                                const uint32_t *__restrict__ words, int64_t cap, int64_t n,
                                                const WorkItem *__restrict__ items,
                                                const uint32_t *__restrict__ n_items,
                                                const GNode *__restrict__ grid, const float *__restrict__ lin,
                                                float *__restrict__ lout, float4 *__restrict__ nadj) {
    constexpr int TN = Geo<DIM>::TN, D2 = DIM * DIM, N3 = nc3<DIM, MAT>();
    __shared__ float gv[DIM * TN];
    __shared__ unsigned long long tacc[3 * TN];
    __shared__ uint32_t sbound;
    const uint32_t nit = *n_items;
    const ItemWalk walk(nit);
    for (uint32_t item = walk.first; item < walk.end; item += walk.stride) {
        const WorkItem it = items[item];
        int origin[DIM];
        tile_origin<DIM>(it.block, P.nb, origin);
        __syncthreads();
        if (threadIdx.x == 0) sbound = 0u;
        for (int t = threadIdx.x; t < TN; t += WG) {
            int ijk[DIM];
            float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (tile_node<DIM>(t, origin, P.res, ijk)) g = node_vel<DIM>(grid, node_index<DIM>(ijk, P.nb));
            gv[t] = g.x;
            gv[TN + t] = g.y;
            if constexpr (DIM == 3) gv[2 * TN + t] = g.z;
        }
        for (int t = threadIdx.x; t < 3 * TN; t += WG) tacc[t] = 0ull;
        __syncthreads();
        {
            // bound of the item's node-adjoint contributions (non-negative
            // floats order as their bit patterns; NaN and inf sort above)
            SchemeRef s = scheme_ref(sch);
            float bmax = 0.0f;
            for (int64_t p = it.p0 + threadIdx.x; p < it.p1; p += WG) {
                float F[N3], lx[DIM], lv[DIM], lC[D2], lF[N3];
                dec_field<DIM, fid3<MAT>(), float>(&s->f[3], words, cap, (uint32_t)p * 4u, F);
                adj_lambda_in<DIM, MAT>(P, lin, n, p, F, lx, lv, lC, lF);
                const float b = adj_node_bound<DIM>(P, lv, lC);
                bmax = (b > bmax || b != b) ? b : bmax;
            }
            atomicMax(&sbound, __float_as_uint(bmax) & 0x7fffffffu);
        }
        __syncthreads();
        const uint32_t bb = sbound;
        const bool fix = bb < 0x7f800000u;
        int e = 0;
        (void)frexpf(__uint_as_float(bb), &e);
        const double fs = fix ? ldexp(1.0, ADJ_FIX_BITS - e) : 1.0;
        const double inv_fs = fix ? ldexp(1.0, e - ADJ_FIX_BITS) : 1.0;
        for (int64_t p = it.p0 + threadIdx.x; p < it.p1; p += WG)
            adj_g2p_particle<DIM, MAT>(sch, P, words, cap, n, p, grid, lin, lout, nadj, gv, tacc, fix, fs, origin);
        __syncthreads();
        // lanes take (node, component) pairs: adjacent lanes, adjacent words
        for (int q = threadIdx.x; q < 4 * TN; q += WG) {
            const int t = q >> 2, c = q & 3;
            if (c >= DIM) continue;
            float v;
            if (fix) {
                const unsigned long long u = tacc[c * TN + t];
                if (u == 0ull) continue;
                v = (float)((double)(long long)u * inv_fs);
            } else {
                v = reinterpret_cast<const float *>(tacc)[c * TN + t];
                if (v == 0.0f) continue;
            }
            int ijk[DIM];
            if (!tile_node<DIM>(t, origin, P.res, ijk)) continue;  // never reached: stencils stay in-grid
            unsafeAtomicAdd(reinterpret_cast<float *>(nadj + node_index<DIM>(ijk, P.nb)) + c, v);
        }
    }
}

// Grid backward: v_i = mom_i / m_i + dt g (components zeroed by the wall
// rule carry no derivative).  In place: (lambda_v, -) -> (lambda_mom, lambda_m).
template <int DIM>
__global__ __launch_bounds__(WG) void k_adj_grid(DevParams P, const GNode *__restrict__ grid,
                                                 float4 *__restrict__ nadj, int64_t nodes) {
    constexpr int B = Geo<DIM>::BLK, L = Geo<DIM>::LOG;
    const int64_t id = (int64_t)blockIdx.x * WG + threadIdx.x;
    if (id >= nodes) return;
    const float4 g = node_vel<DIM>(grid, id);
    const float4 la = nadj[id];
    float out[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    const float m = g.w;  // physical node mass (0: no particle touched it)
    if (m > 0.0f) {
        const int64_t blk = id >> (DIM * L);
        const int l = (int)(id & ((1 << (DIM * L)) - 1));
        int ijk[3];
        ijk[0] = (int)(blk % P.nb) * B + (l & (B - 1));
        if constexpr (DIM == 3) {
            ijk[1] = (int)((blk / P.nb) % P.nb) * B + ((l >> L) & (B - 1));
            ijk[2] = (int)(blk / ((int64_t)P.nb * P.nb)) * B + (l >> (2 * L));
        } else {
            ijk[1] = (int)(blk / P.nb) * B + (l >> L);
        }
        const float vi[3] = {g.x, g.y, g.z}, lv[3] = {la.x, la.y, la.z};
        float lm = 0.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const bool wall = (ijk[a] < P.bound || ijk[a] >= P.res - P.bound) && vi[a] == 0.0f;
            if (wall) continue;
            out[a] = lv[a] / m;
            lm -= lv[a] * (vi[a] - P.dt * P.g[a]) / m;
        }
        out[3] = lm;
    }
    nadj[id] = make_float4(out[0], out[1], out[2], out[3]);
}

// Gathers of one particle's P2G backward over its stencil: lambda_x,
// lambda_v and lambda_A from the node adjoints (lambda_mom_i, lambda_m_i).
// TILE: node adjoints come from the LDS tile `nt` (corner offset l0), else
// from the grid-wide array.
template <int DIM, bool TILE>
__device__ __forceinline__ void adj_p2g_nodes(const DevParams &P, const int *base, const float *fx,
                                              const float (*w)[3], const float (*dw)[3], const float *v,
                                              const float *A, const float4 *__restrict__ nadj, const float4 *nt,
                                              int l0, float *lx, float *lv, float *lA) {
    constexpr int NST = Geo<DIM>::NST, TB = Geo<DIM>::TB;
    const float m = P.p_mass;
#pragma unroll
    for (int st = 0; st < NST; ++st) {
        const int o[3] = {st % 3, (st / 3) % 3, st / 9};
        float wt = 1.0f, d[DIM], gw[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            wt *= w[a][o[a]];
            d[a] = ((float)o[a] - fx[a]) * P.dx;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            gw[a] = dw[a][o[a]];
#pragma unroll
            for (int b = 0; b < DIM; ++b)
                if (b != a) gw[a] *= w[b][o[b]];
        }
        float4 la;
        if constexpr (TILE) {
            la = nt[l0 + ((DIM == 3) ? (o[2] * TB + o[1]) * TB + o[0] : o[1] * TB + o[0])];
        } else {
            int ijk[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) ijk[a] = base[a] + o[a];
            la = nadj[node_index<DIM>(ijk, P.nb)];
        }
        const float lmo[3] = {la.x, la.y, la.z};
        float lw = la.w * m;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            float Ad = 0.0f;
#pragma unroll
            for (int b = 0; b < DIM; ++b) Ad += A[a * DIM + b] * d[b];
            lw += lmo[a] * (m * v[a] + Ad);
            lv[a] += wt * m * lmo[a];
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                lA[a * DIM + b] += wt * lmo[a] * d[b];
                lx[b] -= wt * lmo[a] * A[a * DIM + b];
            }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) lx[a] += gw[a] * lw;
    }
}

// P2G backward of particle p: gathers (lambda_mom_i, lambda_m_i) and adds the
// partial lambda_t of x, v, C and F (stress through its VJP).  A particle
// whose stencil lies in the item's tile (corner `origin`) reads the node
// adjoints from the LDS tile `nt`.
template <int DIM, int MAT>
__device__ __forceinline__ void adj_p2g_particle(const DevScheme *__restrict__ sch, const DevParams &P,
                                                 const uint32_t *__restrict__ words, int64_t cap, int64_t n,
                                                 int64_t p, const float4 *__restrict__ nadj, const float4 *nt,
                                                 const int *origin, float *__restrict__ lout) {
    constexpr int D2 = DIM * DIM, N3 = nc3<DIM, MAT>(), TB = Geo<DIM>::TB;
    SchemeRef s = scheme_ref(sch);
    const uint32_t p4 = (uint32_t)p * 4u;
    double xd[DIM];
    float v[DIM], C[D2], F[N3];
    dec_field<DIM, 0, double>(&s->f[0], words, cap, p4, xd);
    dec_field<DIM, 1, float>(&s->f[1], words, cap, p4, v);
    dec_field<DIM, 2, float>(&s->f[2], words, cap, p4, C);
    dec_field<DIM, fid3<MAT>(), float>(&s->f[3], words, cap, p4, F);
    int base[DIM];
    float fx[DIM], w[DIM][3], dw[DIM][3];
    stencil_all<DIM>(P, xd, base, fx, w, dw);
    // A = -dt V D tau + m C  (physical units: p_mass * (stress_over_m tau + C))
    float A[D2];
    if constexpr (MAT == 1) {
        const float t = P.pc * (F[0] - 1.0f);  // fluid: tau = pc (J - 1) I
#pragma unroll
        for (int i = 0; i < D2; ++i) A[i] = P.p_mass * (((i % (DIM + 1) == 0) ? P.stress_over_m * t : 0.0f) + C[i]);
    } else {
        float R[D2];
        if constexpr (DIM == 2) polar2(F, R);
        else polar3<true>(F, R);
        const float J = det_f<DIM>(F);
#pragma unroll
        for (int i = 0; i < DIM; ++i)
#pragma unroll
            for (int j = 0; j < DIM; ++j) {
                float t = 0.0f;
#pragma unroll
                for (int k = 0; k < DIM; ++k) t += (F[i * DIM + k] - R[i * DIM + k]) * F[j * DIM + k];
                t = 2.0f * P.mu * t + ((i == j) ? P.la * J * (J - 1.0f) : 0.0f);
                A[i * DIM + j] = P.p_mass * (P.stress_over_m * t + C[i * DIM + j]);
            }
    }
    const float m = P.p_mass;
    float lx[DIM], lv[DIM], lA[D2];
#pragma unroll
    for (int a = 0; a < DIM; ++a) lx[a] = lv[a] = 0.0f;
#pragma unroll
    for (int c = 0; c < D2; ++c) lA[c] = 0.0f;
    bool in_tile = true;
    int l0 = 0;
#pragma unroll
    for (int a = DIM - 1; a >= 0; --a) {
        const int la = base[a] - origin[a];
        in_tile &= (la >= 0) && (la <= TB - 3);
        l0 = l0 * TB + la;
    }
    if (in_tile) adj_p2g_nodes<DIM, true>(P, base, fx, w, dw, v, A, nadj, nt, l0, lx, lv, lA);
    else adj_p2g_nodes<DIM, false>(P, base, fx, w, dw, v, A, nadj, nt, l0, lx, lv, lA);

    // A = p_mass stress_over_m tau + p_mass C
    float lt[D2], lF[N3];
#pragma unroll
    for (int c = 0; c < D2; ++c) lt[c] = P.p_mass * P.stress_over_m * lA[c];
#pragma unroll
    for (int c = 0; c < N3; ++c) lF[c] = 0.0f;
    if constexpr (MAT == 1) {
        float tr = 0.0f;  // tau = pc (J - 1) I
#pragma unroll
        for (int a = 0; a < DIM; ++a) tr += lt[a * DIM + a];
        lF[0] = P.pc * tr;
    } else {
        stress_vjp<DIM>(P, F, lt, lF);
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        lout[a * n + p] += lx[a];
        lout[(DIM + a) * n + p] += lv[a];
    }
#pragma unroll
    for (int c = 0; c < D2; ++c) lout[(2 * DIM + c) * n + p] += m * lA[c];
#pragma unroll
    for (int c = 0; c < N3; ++c) lout[(2 * DIM + D2 + c) * n + p] += lF[c];
}

// Per slice of a work item (`slices` per item, slice k taking the item's
// particles k WG, (k + slices) WG, ...; groups of different slices of one item
// load the same tile): the node adjoints of the item's tile are staged in
// LDS (zero outside the grid), then each particle gathers from them.  The
// gather has no accumulation tile to flush, so it splits items into
// work-group-sized slices: more groups in flight on small scenes.
template <int DIM, int MAT>
__global__ __launch_bounds__(WG, ADJ_WAVES_PER_EU) void k_adj_p2g(const DevScheme *__restrict__ sch, DevParams P,
                                                const uint32_t *__restrict__ words, int64_t cap, int64_t n,
                                                const WorkItem *__restrict__ items,
                                                const uint32_t *__restrict__ n_items, int slices,
                                                const float4 *__restrict__ nadj, float *__restrict__ lout) {
    constexpr int TN = Geo<DIM>::TN;
    __shared__ float4 nt[TN];
    const uint32_t nit = *n_items;
    const ItemWalk walk(nit * (uint32_t)slices);
    for (uint32_t vit = walk.first; vit < walk.end; vit += walk.stride) {
        const uint32_t item = vit / (uint32_t)slices, slice = vit % (uint32_t)slices;
        const WorkItem it = items[item];
        int origin[DIM];
        tile_origin<DIM>(it.block, P.nb, origin);
        __syncthreads();
        for (int t = threadIdx.x; t < TN; t += WG) {
            int ijk[DIM];
            float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            if (tile_node<DIM>(t, origin, P.res, ijk)) g = nadj[node_index<DIM>(ijk, P.nb)];
            nt[t] = g;
        }
        __syncthreads();
        for (int64_t p = it.p0 + (int64_t)slice * WG + threadIdx.x; p < it.p1; p += (int64_t)slices * WG)
            adj_p2g_particle<DIM, MAT>(sch, P, words, cap, n, p, nadj, nt, origin, lout);
    }
}

// Objective at the final state: 0 = centre of mass along `axis`, 1 = kinetic
// energy.  Writes lambda_T and accumulates z (binary64) into acc[0].
template <int DIM, int MAT>
__global__ __launch_bounds__(WG) void k_adj_objective(const DevScheme *__restrict__ sch, DevParams P,
                                                      const uint32_t *__restrict__ words, int64_t cap, int64_t n,
                                                      int objective, int axis, float *__restrict__ lout,
                                                      double *__restrict__ acc) {
    constexpr int LR = LROWS<DIM, MAT>();
    const int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x;
    double zc = 0.0;
    if (p < n) {
        SchemeRef s = scheme_ref(sch);
        const uint32_t p4 = (uint32_t)p * 4u;
#pragma unroll
        for (int r = 0; r < LR; ++r) lout[r * n + p] = 0.0f;
        if (objective == 0) {
            double xd[DIM];
            dec_field<DIM, 0, double>(&s->f[0], words, cap, p4, xd);
            zc = xd[axis] / (double)n;
            lout[axis * n + p] = 1.0f / (float)n;
        } else {
            double vd[DIM];
            dec_field<DIM, 1, double>(&s->f[1], words, cap, p4, vd);
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                zc += 0.5 * (double)P.p_mass * vd[a] * vd[a];
                lout[(DIM + a) * n + p] = P.p_mass * (float)vd[a];
            }
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) zc += __shfl_xor(zc, o, 64);
    if (__lane_id() == 0 && zc != 0.0) atomicAdd(acc, zc);
}

// G[f] += sum lambda, g[f] += sum lambda^2 over the rows of field f.
template <int DIM, int MAT>
__global__ __launch_bounds__(WG) void k_adj_reduce(const float *__restrict__ lam, int64_t n,
                                                   double *__restrict__ acc) {
    constexpr int LR = LROWS<DIM, MAT>();
    double G[4] = {0, 0, 0, 0}, g[4] = {0, 0, 0, 0};
    // grid-stride (a few hundred groups), then wave and group sums: one
    // atomic per sum and group (atomics on one address serialize in the L2)
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < n; p += (int64_t)gridDim.x * WG) {
#pragma unroll
        for (int r = 0; r < LR; ++r) {
            const int f = r < DIM ? 0 : r < 2 * DIM ? 1 : r < 2 * DIM + DIM * DIM ? 2 : 3;
            const double l = (double)lam[r * n + p];
            G[f] += l;
            g[f] += l * l;
        }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            G[f] += __shfl_xor(G[f], o, 64);
            g[f] += __shfl_xor(g[f], o, 64);
        }
    }
    __shared__ double part[WG / 64][8];
    if (__lane_id() == 0) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            part[threadIdx.x >> 6][f] = G[f];
            part[threadIdx.x >> 6][4 + f] = g[f];
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < WG / 64; ++w) t += part[w][threadIdx.x];
        // copy b % ADJ_SLOTS of the sums (k < 4) and sums of squares (k >= 4)
        atomicAdd(acc + 1 + 8 * (blockIdx.x % ADJ_SLOTS) + threadIdx.x, t);
    }
}

__global__ void k_zero_f4(float4 *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

// Order-preserving map of float32 to uint32 (for atomic min / max).
__device__ __forceinline__ uint32_t ord_key(float f) {
    const uint32_t u = __float_as_uint(f);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}

// Per-field minimum and maximum of the stored (decoded) values, F - I for a
// REL_IDENTITY F:
// rng[f] = min key, rng[4 + f] = max key (ord_key order).
template <int DIM, int MAT>
__global__ __launch_bounds__(WG) void k_adj_range(const DevScheme *__restrict__ sch, const uint32_t *__restrict__ words,
                                                  int64_t cap, int64_t n, uint32_t *__restrict__ rng) {
    constexpr int D2 = DIM * DIM, N3 = nc3<DIM, MAT>();
    uint32_t lo[4] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0xffffffffu}, hi[4] = {0u, 0u, 0u, 0u};
    for (int64_t p = (int64_t)blockIdx.x * WG + threadIdx.x; p < n; p += (int64_t)gridDim.x * WG) {
        SchemeRef s = scheme_ref(sch);
        const uint32_t p4 = (uint32_t)p * 4u;
        double xd[DIM];
        float v[DIM], C[D2], F[N3];
        dec_field<DIM, 0, double>(&s->f[0], words, cap, p4, xd);
        dec_field<DIM, 1, float>(&s->f[1], words, cap, p4, v);
        dec_field<DIM, 2, float>(&s->f[2], words, cap, p4, C);
        dec_field<DIM, fid3<MAT>(), float>(&s->f[3], words, cap, p4, F);
        if (s->f[3].rel) {
#pragma unroll
            for (int c = 0; c < N3; c += DIM + 1) F[c] -= 1.0f;
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            const uint32_t kx = ord_key((float)xd[a]), kv = ord_key(v[a]);
            lo[0] = min(lo[0], kx); hi[0] = max(hi[0], kx);
            lo[1] = min(lo[1], kv); hi[1] = max(hi[1], kv);
        }
#pragma unroll
        for (int c = 0; c < D2; ++c) {
            const uint32_t kc = ord_key(C[c]);
            lo[2] = min(lo[2], kc); hi[2] = max(hi[2], kc);
        }
#pragma unroll
        for (int c = 0; c < N3; ++c) {
            const uint32_t kf = ord_key(F[c]);
            lo[3] = min(lo[3], kf); hi[3] = max(hi[3], kf);
        }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            lo[f] = min(lo[f], (uint32_t)__shfl_xor((int)lo[f], o, 64));
            hi[f] = max(hi[f], (uint32_t)__shfl_xor((int)hi[f], o, 64));
        }
    }
    __shared__ uint32_t part[WG / 64][8];
    if (__lane_id() == 0) {
#pragma unroll
        for (int f = 0; f < 4; ++f) {
            part[threadIdx.x >> 6][f] = lo[f];
            part[threadIdx.x >> 6][4 + f] = hi[f];
        }
    }
    __syncthreads();
    if (threadIdx.x < 8) {
        uint32_t t = part[0][threadIdx.x];
#pragma unroll
        for (int w = 1; w < WG / 64; ++w) t = (threadIdx.x < 4) ? min(t, part[w][threadIdx.x]) : max(t, part[w][threadIdx.x]);
        const uint32_t slot = 4u * (blockIdx.x % ADJ_SLOTS);
        if (threadIdx.x < 4) atomicMin(rng + slot + threadIdx.x, t);
        else atomicMax(rng + 4 * ADJ_SLOTS + slot + (threadIdx.x - 4), t);
    }
}

// out[r * n + ids[p]] = lam[r * n + p]: rows back into the order of the
// particles at encode time.
__global__ void k_adj_unpermute(const float *__restrict__ lam, const uint32_t *__restrict__ ids, int64_t n,
                                int rows, float *__restrict__ out) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int64_t q = ids[p];
    if (q >= n) return;
    for (int r = 0; r < rows; ++r) out[r * n + q] = lam[r * n + p];
}

static dim3 agrid(int64_t n) { return dim3((unsigned)((n + WG - 1) / WG)); }
// reductions: at most 1024 groups (grid-stride), one atomic per group and
// sum, into ADJ_SLOTS copies
static dim3 rgrid(int64_t n) { return dim3((unsigned)std::min<int64_t>((n + WG - 1) / WG, 1024)); }

#define MPMQ_ADJ_DISPATCH(KERNEL, GRID, ...)                                                              \
    do {                                                                                                 \
        if (dim == 3 && mat) hipLaunchKernelGGL((KERNEL<3, 1>), GRID, dim3(WG), 0, st, __VA_ARGS__);     \
        else if (dim == 3) hipLaunchKernelGGL((KERNEL<3, 0>), GRID, dim3(WG), 0, st, __VA_ARGS__);       \
        else if (mat) hipLaunchKernelGGL((KERNEL<2, 1>), GRID, dim3(WG), 0, st, __VA_ARGS__);            \
        else hipLaunchKernelGGL((KERNEL<2, 0>), GRID, dim3(WG), 0, st, __VA_ARGS__);                     \
    } while (0)

hipError_t launch_adj_objective(int dim, int mat, const DevScheme *s, const DevParams &P, const uint32_t *words,
                                int64_t cap, int64_t n, int objective, int axis, float *lam, double *acc,
                                hipStream_t st) {
    MPMQ_ADJ_DISPATCH(k_adj_objective, agrid(n), s, P, words, cap, n, objective, axis, lam, acc);
    return hipGetLastError();
}

hipError_t launch_adj_step(int dim, int mat, const DevScheme *s, const DevParams &P, const uint32_t *words,
                           int64_t cap, int64_t n, const WorkItem *items, const uint32_t *n_items, int item_grid,
                           int item_cap,
                           const GNode *grid, int64_t nodes, const float *lin, float *lout, float4 *nadj,
                           hipStream_t st) {
    hipLaunchKernelGGL(k_zero_f4, dim3((unsigned)std::min<int64_t>((nodes + 255) / 256, 65536)), dim3(256), 0, st,
                       nadj, nodes);
    MPMQ_ADJ_DISPATCH(k_adj_g2p, dim3((unsigned)item_grid), s, P, words, cap, n, items, n_items, grid, lin, lout,
                      nadj);
    if (dim == 3) hipLaunchKernelGGL(k_adj_grid<3>, agrid(nodes), dim3(WG), 0, st, P, grid, nadj, nodes);
    else hipLaunchKernelGGL(k_adj_grid<2>, agrid(nodes), dim3(WG), 0, st, P, grid, nadj, nodes);
    // one group per work-group pass of an item (a multiple of the 8 XCDs)
    const int slices = std::max(1, item_cap / WG);
    const int p2g_grid = (int)std::min<int64_t>((int64_t)item_grid * slices, 131072);
    MPMQ_ADJ_DISPATCH(k_adj_p2g, dim3((unsigned)p2g_grid), s, P, words, cap, n, items, n_items, slices, nadj,
                      lout);
    return hipGetLastError();
}

hipError_t launch_adj_reduce(int dim, int mat, const float *lam, int64_t n, double *acc, hipStream_t st) {
    MPMQ_ADJ_DISPATCH(k_adj_reduce, rgrid(n), lam, n, acc);
    return hipGetLastError();
}

hipError_t launch_adj_range(int dim, int mat, const DevScheme *s, const uint32_t *words, int64_t cap, int64_t n,
                            uint32_t *rng, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    MPMQ_ADJ_DISPATCH(k_adj_range, rgrid(n), s, words, cap, n, rng);
    return hipGetLastError();
}

hipError_t launch_adj_unpermute(const float *lam, const uint32_t *ids, int64_t n, int rows, float *out,
                                hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_unpermute, agrid(n), dim3(WG), 0, st, lam, ids, n, rows, out);
    return hipGetLastError();
}

}  // namespace mpmq
