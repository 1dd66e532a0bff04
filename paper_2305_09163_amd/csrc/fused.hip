// Fused right-hand side: one launch per Runge-Kutta stage evaluates the whole
// semi-discrete operator of eq. (fvmdis) (Sec. 3.1) for a block of cells and
// writes the stage result, so the state is read once and written once.
//
// Work decomposition (3D).  A workgroup of 16 x 16 threads owns a 16 x 16
// column of cells in (x, y) and marches through a chunk of z planes:
//   - z: each thread keeps the primitives of planes k-1 .. k+3 of its own
//     column in registers, reconstructs cell k+1 (WENO5, both faces) and
//     solves the Riemann problem at face k+1/2 (Sec. 3.2, 3.2.1); the flux of
//     face k-1/2 is carried over from the previous plane;
//   - x and y: plane k (with 3-cell halos) is converted to primitives into
//     LDS once; every cell of the tile plus one halo cell per side is
//     reconstructed once per direction (both face values from one stencil),
//     the pair values go to LDS, and the HLLC flux of every face of the tile
//     is computed once and shared by the two cells that own the face;
//   - each thread then forms its cell's flux differences plus the
//     alpha1 div(u) source and the SSP-RK3 stage combination.
// 2D uses the same tile without the z march; 1D uses a 256-cell row.
// With ROUTE = true every (cell, direction) is first classified by the learned
// indicator of mlp.h (whole wavefronts at a time) and a smooth one takes the
// linear fifth-order stencil for every variable instead of WENO5.
#include <type_traits>

#include "internal.h"
#include "mlp.h"

namespace mfc {
namespace {

template <int NDIM>
struct Shape {
    static constexpr int TX = NDIM == 1 ? 256 : 16;
    static constexpr int TY = NDIM == 1 ? 1 : 16;
    static constexpr int NT = TX * TY;
    static constexpr int NV = 4 + NDIM;
    static constexpr int PX = TX + 2 * NG;
    static constexpr int PY = NDIM >= 2 ? TY + 2 * NG : 1;
    static constexpr int OY = NDIM >= 2 ? NG : 0;   // LDS row of the tile's first row
    static constexpr int NPX = (TX + 2) * TY;       // x reconstructions (cells -1 .. TX)
    static constexpr int NFX = (TX + 1) * TY;       // x faces
    static constexpr int NPY = NDIM >= 2 ? TX * (TY + 2) : 0;
    static constexpr int NFY = NDIM >= 2 ? TX * (TY + 1) : 0;
    static constexpr int NP = NPX > NPY ? NPX : NPY;
    static constexpr int NF = NFX > NFY ? NFX : NFY;
    static constexpr int NHALO = 2 * NG * TY + (NDIM >= 2 ? 2 * NG * TX : 0);
};

constexpr int kLZ = 16;  // z planes per workgroup

// Load one cell and convert it to primitives.  Returns true if the cell is
// non-physical AND is one the method reads (interior or ghost face slab: at
// most one coordinate outside the interior).  Lanes past a ragged grid edge
// may load edge/corner ghost cells, which are never written; their values
// only feed lanes whose results are discarded, so they must not raise the
// flag either.
template <int NDIM, class T>
__device__ __forceinline__ bool load_prim(const Grid &g, const T *__restrict__ q, int i, int j, int k, T *w)
{
    constexpr int NV = 4 + NDIM;
    const int64_t c = (int64_t)(k + g.off[2]) * g.stride[2] + (int64_t)(j + g.off[1]) * g.stride[1] + (i + g.off[0]);
    T qc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + c];
    const bool bad = cons_to_prim<NDIM, T>(g, qc, w);
    const int outside = (i < 0 || i >= g.n[0]) + (j < 0 || j >= g.n[1]) + (k < 0 || k >= g.n[2]);
    return bad && outside <= 1;
}

// Reconstruct one 5-cell stencil for all variables: order ORDER (5 WENO5,
// 3 WENO3, 1 first order), or the linear fifth-order stencil when lin is set.
template <int ORDER, int NV, class T>
__device__ __forceinline__ void recon_regs(const T (&zw)[5][NV], T eps, bool lin, T *plus, T *minus,
                                           const double *cf = nullptr)
{
#pragma unroll
    for (int v = 0; v < NV; v++) {
        if (lin) linear5_pair<T>(zw[0][v], zw[1][v], zw[2][v], zw[3][v], zw[4][v], plus[v], minus[v]);
        else recon_cell<ORDER, T>(cf, zw[0][v], zw[1][v], zw[2][v], zw[3][v], zw[4][v], eps, plus[v], minus[v]);
    }
}

// The learned indicator's decision for a stencil held in registers (all lanes
// of the wavefront must call).
template <int NDIM, class T>
__device__ __forceinline__ bool route_regs(const mlp::Params &P, uint16_t *scratch, const T (&zw)[5][4 + NDIM],
                                           T sqrt_eps, float logit_tau, int lane)
{
    T av[5], rv[5], pv[5];
#pragma unroll
    for (int j = 0; j < 5; j++) {
        av[j] = zw[j][3 + NDIM];
        rv[j] = zw[j][0] + zw[j][1];
        pv[j] = zw[j][2 + NDIM];
    }
    uint16_t f[16];
    mlp::features<T>(av, rv, pv, sqrt_eps, f);
    return mlp::smooth_wave(P, scratch, f, logit_tau, lane);
}

template <int NDIM, class T, bool ROUTE, int ORDER, bool STRETCH>
__global__ void __launch_bounds__(Shape<NDIM>::NT, 2)
    k_fused(Grid g, const T *__restrict__ q, const T *q0, T *out, int mode, double dt,
            const double *__restrict__ dt_dev, int *__restrict__ flag, int lz, const float *__restrict__ mlpw,
            float logit_tau, T sqrt_eps)
{
    using S = Shape<NDIM>;
    constexpr int NV = S::NV, A = 3 + NDIM, E = 2 + NDIM, TX = S::TX, TY = S::TY, NT = S::NT, OY = S::OY;
    __shared__ T s_plane[NV][S::PY][S::PX];
    __shared__ T s_pair[2 * NV][S::NP];
    __shared__ __align__(16) T s_flux[NV + 1][S::NF];
    // feature exchange area of the routed reconstruction (64 x 16 bf16 per
    // wavefront): inside the flux array when it is large enough, since no
    // thread reads the fluxes while reconstructions are formed
    constexpr int kFeat = (NT / 64) * 64 * 16;
    constexpr bool kInFlux = sizeof(T) * (NV + 1) * S::NF >= sizeof(uint16_t) * kFeat;
    __shared__ __align__(16) typename std::conditional<ROUTE, mlp::Params, char>::type s_mlp;
    __shared__ __align__(16) uint16_t s_feat_own[(ROUTE && !kInFlux) ? kFeat : 1];
    uint16_t *scratch = (kInFlux ? (uint16_t *)&s_flux[0][0] : s_feat_own) + (threadIdx.x / 64) * 64 * 16;
    const int lane = threadIdx.x % 64;
    if constexpr (ROUTE) {
        mlp::stage_params(s_mlp, nullptr, mlpw, threadIdx.x, NT);
        __syncthreads();
    }
    const T eps = T(g.eps), idx = T(g.inv_dx[0]), idy = T(g.inv_dx[1]), idz = T(g.inv_dx[2]);

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    const int x0 = blockIdx.x * TX, y0 = blockIdx.y * TY;
    const int z0 = NDIM == 3 ? (int)blockIdx.z * lz : 0;
    const int z1 = NDIM == 3 ? min(z0 + lz, g.n[2]) : 1;
    const int xmax = g.n[0] + NG - 1;                  // last readable cell (ghost)
    const int ymax = NDIM >= 2 ? g.n[1] + NG - 1 : 0;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool own = gx < g.n[0] && gy < g.n[1];
    const int cx = min(gx, xmax), cy = min(gy, ymax);  // clamped: out-of-grid lanes read real cells
    bool bad = false;

    // ---- z march state (3D): primitives of planes k-1 .. k+3 of this column,
    // the reconstruction of cell k at its + face, the flux at face k-1/2.
    T zw[5][NV];
    T pk[NV];
    T Fz[NV + 1];
    if constexpr (NDIM == 3) {
#pragma unroll
        for (int p = 0; p < 5; p++) bad |= load_prim<NDIM, T>(g, q, cx, cy, z0 - 3 + p, zw[p]);
        T plus_prev[NV], mk[NV], dummy[NV];
        bool lin = false;
        if constexpr (ROUTE) lin = route_regs<NDIM, T>(s_mlp, scratch, zw, sqrt_eps, logit_tau, lane);
        recon_regs<ORDER, NV, T>(zw, eps, lin, plus_prev, dummy, STRETCH ? coef_row(g, 2, z0 - 1) : nullptr);
#pragma unroll
        for (int p = 0; p < 4; p++)
#pragma unroll
            for (int v = 0; v < NV; v++) zw[p][v] = zw[p + 1][v];
        bad |= load_prim<NDIM, T>(g, q, cx, cy, z0 + 2, zw[4]);
        if constexpr (ROUTE) lin = route_regs<NDIM, T>(s_mlp, scratch, zw, sqrt_eps, logit_tau, lane);
        recon_regs<ORDER, NV, T>(zw, eps, lin, pk, mk, STRETCH ? coef_row(g, 2, z0) : nullptr);
        bad |= hllc<NDIM, (NDIM == 3 ? 2 : 0), T>(g, plus_prev, mk, Fz, Fz[NV]) && own;
    }

    const T hdt = T(mode ? (dt_dev ? *dt_dev : dt) : 0.0);
    const T ca = T(mode == 1 ? 0.0 : (mode == 2 ? 0.75 : 1.0 / 3.0));
    const T cb = T(mode == 1 ? 1.0 : (mode == 2 ? 0.25 : 2.0 / 3.0));

    for (int k = z0; k < z1; k++) {
        T wk[NV];
        T Fzn[NV + 1];
        if constexpr (NDIM == 3) {
#pragma unroll
            for (int p = 0; p < 4; p++)
#pragma unroll
                for (int v = 0; v < NV; v++) zw[p][v] = zw[p + 1][v];
            bad |= load_prim<NDIM, T>(g, q, cx, cy, k + 3, zw[4]);
            T pn[NV], mn[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) wk[v] = zw[1][v];
            bool lin = false;
            if constexpr (ROUTE) lin = route_regs<NDIM, T>(s_mlp, scratch, zw, sqrt_eps, logit_tau, lane);
            recon_regs<ORDER, NV, T>(zw, eps, lin, pn, mn, STRETCH ? coef_row(g, 2, k + 1) : nullptr);
            bad |= hllc<NDIM, (NDIM == 3 ? 2 : 0), T>(g, pk, mn, Fzn, Fzn[NV]) && own;
#pragma unroll
            for (int v = 0; v < NV; v++) pk[v] = pn[v];
        } else {
            bad |= load_prim<NDIM, T>(g, q, cx, cy, 0, wk);
        }

        // ---- plane k into LDS: own cell, then the x and y halos
#pragma unroll
        for (int v = 0; v < NV; v++) s_plane[v][ty + OY][tx + NG] = wk[v];
        for (int h = tid; h < S::NHALO; h += NT) {
            int li, lj;
            if (h < 2 * NG * TY) {
                const int col = h % (2 * NG), row = h / (2 * NG);
                li = col < NG ? col : TX + col;
                lj = row + OY;
            } else {
                const int h2 = h - 2 * NG * TY;
                const int col = h2 % TX, r = h2 / TX;
                li = col + NG;
                lj = r < NG ? r : TY + r;
            }
            const int gi = min(x0 + li - NG, xmax), gj = min(y0 + lj - OY, ymax);
            T w[NV];
            bad |= load_prim<NDIM, T>(g, q, gi, gj, k, w);
#pragma unroll
            for (int v = 0; v < NV; v++) s_plane[v][lj][li] = w[v];
        }
        __syncthreads();

        // ---- x: reconstruct cells -1 .. TX of every row
        if constexpr (ROUTE) {
            for (int p0 = 0; p0 < S::NPX; p0 += NT) {  // uniform trip count: whole wavefronts classify
                const int p = p0 + tid;
                const bool valid = p < S::NPX;
                const int pc = valid ? p : S::NPX - 1;
                const int lj = pc / (TX + 2) + OY, c = pc % (TX + 2);
                bool lin = false;
                if (__ballot(valid))
                    lin = mlp::smooth_stencil<T>(s_mlp, scratch, &s_plane[A][lj][c], &s_plane[0][lj][c],
                                                 &s_plane[1][lj][c], &s_plane[E][lj][c], 1, sqrt_eps, logit_tau,
                                                 lane);
                if (valid) {
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        const T *s = &s_plane[v][lj][c];
                        if (lin) linear5_pair<T>(s[0], s[1], s[2], s[3], s[4], s_pair[v][p], s_pair[NV + v][p]);
                        else recon_pair<ORDER, T>(s[0], s[1], s[2], s[3], s[4], eps, s_pair[v][p], s_pair[NV + v][p]);
                    }
                }
            }
        } else {
            for (int p = tid; p < S::NPX; p += NT) {
                const int row = p / (TX + 2), c = p % (TX + 2);
                const int lj = row + OY;
                const double *cf = STRETCH ? coef_row(g, 0, x0 + c - 1) : nullptr;
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T *s = &s_plane[v][lj][c];
                    recon_cell<ORDER, T>(cf, s[0], s[1], s[2], s[3], s[4], eps, s_pair[v][p], s_pair[NV + v][p]);
                }
            }
        }
        __syncthreads();
        // ---- x faces: face fi sits between tile cells fi-1 and fi
        for (int f = tid; f < S::NFX; f += NT) {
            const int row = f / (TX + 1), fi = f % (TX + 1);
            const int pl = row * (TX + 2) + fi;
            T wL[NV], wR[NV], F[NV], uf;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wL[v] = s_pair[v][pl];
                wR[v] = s_pair[NV + v][pl + 1];
            }
            const bool b = hllc<NDIM, 0, T>(g, wL, wR, F, uf);
            bad |= b && (y0 + row < g.n[1]) && (x0 + fi <= g.n[0]);
#pragma unroll
            for (int v = 0; v < NV; v++) s_flux[v][f] = F[v];
            s_flux[NV][f] = uf;
        }
        __syncthreads();
        T L[NV], divu;
        {
            const int f = ty * (TX + 1) + tx;
            const T ix = STRETCH ? T(inv_width(g, 0, gx)) : idx;
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] = (s_flux[v][f] - s_flux[v][f + 1]) * ix;
            divu = (s_flux[NV][f + 1] - s_flux[NV][f]) * ix;
        }

        if constexpr (NDIM >= 2) {
            // ---- y: reconstruct rows -1 .. TY of every column
            if constexpr (ROUTE) {
                if constexpr (kInFlux) __syncthreads();  // x fluxes are read above before the area is reused
                for (int p0 = 0; p0 < S::NPY; p0 += NT) {
                    const int p = p0 + tid;
                    const bool valid = p < S::NPY;
                    const int pc = valid ? p : S::NPY - 1;
                    const int li = pc % TX + NG, r = pc / TX;
                    bool lin = false;
                    if (__ballot(valid))
                        lin = mlp::smooth_stencil<T>(s_mlp, scratch, &s_plane[A][r][li], &s_plane[0][r][li],
                                                     &s_plane[1][r][li], &s_plane[E][r][li], S::PX, sqrt_eps,
                                                     logit_tau, lane);
                    if (valid) {
#pragma unroll
                        for (int v = 0; v < NV; v++) {
                            if (lin)
                                linear5_pair<T>(s_plane[v][r][li], s_plane[v][r + 1][li], s_plane[v][r + 2][li],
                                                s_plane[v][r + 3][li], s_plane[v][r + 4][li], s_pair[v][p],
                                                s_pair[NV + v][p]);
                            else
                                recon_pair<ORDER, T>(s_plane[v][r][li], s_plane[v][r + 1][li], s_plane[v][r + 2][li],
                                           s_plane[v][r + 3][li], s_plane[v][r + 4][li], eps, s_pair[v][p],
                                           s_pair[NV + v][p]);
                        }
                    }
                }
            } else {
                for (int p = tid; p < S::NPY; p += NT) {
                    const int c = p % TX, r = p / TX;
                    const int li = c + NG;
                    const double *cf = STRETCH ? coef_row(g, 1, y0 + r - 1) : nullptr;
#pragma unroll
                    for (int v = 0; v < NV; v++)
                        recon_cell<ORDER, T>(cf, s_plane[v][r][li], s_plane[v][r + 1][li], s_plane[v][r + 2][li],
                                             s_plane[v][r + 3][li], s_plane[v][r + 4][li], eps, s_pair[v][p],
                                             s_pair[NV + v][p]);
                }
            }
            __syncthreads();
            for (int f = tid; f < S::NFY; f += NT) {
                const int c = f % TX, fr = f / TX;
                const int pl = fr * TX + c;
                T wL[NV], wR[NV], F[NV], uf;
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    wL[v] = s_pair[v][pl];
                    wR[v] = s_pair[NV + v][pl + TX];
                }
                const bool b = hllc<NDIM, (NDIM >= 2 ? 1 : 0), T>(g, wL, wR, F, uf);
                bad |= b && (x0 + c < g.n[0]) && (y0 + fr <= g.n[1]);
#pragma unroll
                for (int v = 0; v < NV; v++) s_flux[v][f] = F[v];
                s_flux[NV][f] = uf;
            }
            __syncthreads();
            const int f = ty * TX + tx;
            const T iy = STRETCH ? T(inv_width(g, 1, gy)) : idy;
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] += (s_flux[v][f] - s_flux[v][f + TX]) * iy;
            divu += (s_flux[NV][f + TX] - s_flux[NV][f]) * iy;
        }
        if constexpr (NDIM == 3) {
            const T iz = STRETCH ? T(inv_width(g, 2, k)) : idz;
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] += (Fz[v] - Fzn[v]) * iz;
            divu += (Fzn[NV] - Fz[NV]) * iz;
#pragma unroll
            for (int v = 0; v <= NV; v++) Fz[v] = Fzn[v];
        }
        L[A] += alpha_source<T>(g, wk[A], wk[E]) * divu;

        if (own) {
            const int64_t c = (int64_t)(k + g.off[2]) * g.stride[2] + (int64_t)(gy + g.off[1]) * g.stride[1] +
                              (gx + g.off[0]);
            if (mode == 0) {
#pragma unroll
                for (int v = 0; v < NV; v++) out[v * g.vstride + c] = L[v];
            } else {
                // every operand before the first store (out may alias q0)
                T a0[NV], a1[NV];
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    a0[v] = q0[v * g.vstride + c];
                    a1[v] = q[v * g.vstride + c];
                }
#pragma unroll
                for (int v = 0; v < NV; v++) out[v * g.vstride + c] = ca * a0[v] + cb * (a1[v] + hdt * L[v]);
            }
        }
    }
    if (bad) atomicOr(flag, 1);
}

template <int NDIM, class T, bool ROUTE, int ORDER, bool STRETCH>
int rhs_fused(mfc_grid *h, const T *q, const T *q0, T *out, int mode, double dt, const double *dt_dev, hipStream_t s)
{
    using S = Shape<NDIM>;
    const Grid &g = h->g;
    dim3 grid((g.n[0] + S::TX - 1) / S::TX, NDIM >= 2 ? (g.n[1] + S::TY - 1) / S::TY : 1,
              NDIM == 3 ? (g.n[2] + kLZ - 1) / kLZ : 1);
    const T se = T(__builtin_sqrt(g.eps));
    timing_begin(h, s);
    hipLaunchKernelGGL((k_fused<NDIM, T, ROUTE, ORDER, STRETCH>), grid, dim3(S::NT), 0, s, g, q, q0, out, mode, dt, dt_dev, h->flag, kLZ,
                       h->mlp, h->logit_tau, se);
    timing_end(h, s);
    return hip_status(hipGetLastError(), "fused right-hand side launch");
}

template <class T, bool ROUTE, int ORDER, bool STRETCH = false>
int rhs_fused_t(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt, const double *dt_dev,
                hipStream_t s)
{
    const T *a = (const T *)q, *b = (const T *)q0;
    T *o = (T *)out;
    switch (h->g.ndim) {
    case 1: return rhs_fused<1, T, ROUTE, ORDER, STRETCH>(h, a, b, o, mode, dt, dt_dev, s);
    case 2: return rhs_fused<2, T, ROUTE, ORDER, STRETCH>(h, a, b, o, mode, dt, dt_dev, s);
    default: return rhs_fused<3, T, ROUTE, ORDER, STRETCH>(h, a, b, o, mode, dt, dt_dev, s);
    }
}

}  // namespace

int launch_rhs_fused(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt,
                     const double *dt_dev, hipStream_t s)
{
    const bool learned = h->desc.recon == MFC_RECON_LEARNED;
    if (learned && !h->mlp) return fail(MFC_E_ARG, "MFC_RECON_LEARNED needs mfc_set_indicator first");
    const bool f32 = h->desc.precision == MFC_FP32_MIXED;
    if (h->g.stretched) {   // WENO5 or first order (validated at init)
        if (h->desc.recon == MFC_RECON_FIRST_ORDER)
            return f32 ? rhs_fused_t<float, false, 1, true>(h, q, q0, out, mode, dt, dt_dev, s)
                       : rhs_fused_t<double, false, 1, true>(h, q, q0, out, mode, dt, dt_dev, s);
        return f32 ? rhs_fused_t<float, false, 5, true>(h, q, q0, out, mode, dt, dt_dev, s)
                   : rhs_fused_t<double, false, 5, true>(h, q, q0, out, mode, dt, dt_dev, s);
    }
    switch (h->desc.recon) {
    case MFC_RECON_LEARNED:
        return f32 ? rhs_fused_t<float, true, 5>(h, q, q0, out, mode, dt, dt_dev, s)
                   : rhs_fused_t<double, true, 5>(h, q, q0, out, mode, dt, dt_dev, s);
    case MFC_RECON_WENO3:
        return f32 ? rhs_fused_t<float, false, 3>(h, q, q0, out, mode, dt, dt_dev, s)
                   : rhs_fused_t<double, false, 3>(h, q, q0, out, mode, dt, dt_dev, s);
    case MFC_RECON_FIRST_ORDER:
        return f32 ? rhs_fused_t<float, false, 1>(h, q, q0, out, mode, dt, dt_dev, s)
                   : rhs_fused_t<double, false, 1>(h, q, q0, out, mode, dt, dt_dev, s);
    default:
        return f32 ? rhs_fused_t<float, false, 5>(h, q, q0, out, mode, dt, dt_dev, s)
                   : rhs_fused_t<double, false, 5>(h, q, q0, out, mode, dt, dt_dev, s);
    }
}

}  // namespace mfc
