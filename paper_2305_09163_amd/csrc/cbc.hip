// Characteristic-based non-reflecting boundaries (Sec. 3.3: the paper's
// characteristic boundary conditions, in the time-dependent form of
// Thompson): a post-pass over the boundary cells of every face marked
// MFC_BC_CHARACTERISTIC, run after the stage kernel of any path.
//
// For each boundary cell it takes the finite-volume terms normal to the face
// (the two HLLC fluxes of the cell along that dimension, its share of
// alpha1 div(u)): kept by the split stage kernels, recomputed here for the
// fused and staged paths.  It replaces them by the characteristic form: wave
// amplitudes L1 = (u-c)(p_x - rho c u_x), L5 = (u+c)(p_x + rho c u_x),
// L_k = u((alpha_k rho_k)_x - alpha_k rho_k p_x/(rho c^2)), L_t = u (u_t)_x,
// L_a = u (alpha1)_x from second-order one-sided differences into the
// domain, with every amplitude whose wave enters the domain set to zero;
// p_t = -(L5+L1)/2, u_t = -(L5-L1)/(2 rho c), (alpha_k rho_k)_t = -L_k -
// alpha_k rho_k (L5+L1)/(2 rho c^2), (u_t)_t = -L_t, (alpha1)_t = -L_a,
// carried to the conservative rows through the mixture EOS.  The stage
// result gets the difference times the stage's weight of dt (or, for a bare
// right-hand side, the difference itself).  Neighbours past a face are read
// through the boundary rule (the adjacent interior cell), so the ghost
// cells need not be filled.
#include "charbc.h"
#include "internal.h"

namespace mfc {
namespace {

// 64-thread blocks spread the few boundary cells over every CU; the pass is
// latency-bound, so each cell's two normal fluxes go to two lanes.
#ifndef MFC_CBC_THREADS
#define MFC_CBC_THREADS 64
#endif
#ifndef MFC_CBC_WAVES
#define MFC_CBC_WAVES 2
#endif
constexpr int kCbcThreads = MFC_CBC_THREADS;

// The characteristic faces of a grid: bit f of `mask` is set when face f
// (x-, x+, y-, y+, z-, z+) is characteristic; start[f] is the index of the
// face's first boundary cell in the one launch that covers them all (two
// lanes per cell), start[6] the number of cells.
struct CbcFaces {
    int mask;
    int64_t start[7];
};

// Index into the four distinct cells of a boundary stencil: cells b - 3 ..
// b + 3 along D with the non-periodic boundary rule (indices clamped into
// the interior) are, for the low face (b = 0), cell 0 four times and then
// cells 1, 2, 3; for the high face (b = n - 1) the mirror image.  W[k] holds
// cell b + k s (s = +1 low face, -1 high face), so stencil cell o is W[at(o)].
template <int SIDE>
__device__ constexpr int at(int o)
{
    return SIDE == 0 ? (o <= 3 ? 0 : o - 3) : (o >= 3 ? 0 : 3 - o);
}

// Change of the stage derivative of boundary cell c (c[D] = its boundary
// index) from the characteristic face SIDE of dimension D: the
// characteristic rate minus the finite-volume terms normal to the face.
// STORED: those terms were kept by the split stage kernels (Grid::cbc_fv);
// otherwise they are recomputed here, the cell's two normal fluxes on the
// two lanes of a pair.
template <int NDIM, int D, int SIDE, class T, int ORDER, bool STORED>
__device__ __forceinline__ bool face_delta(const Grid &g, int c[3], const T *__restrict__ q, T delta[4 + NDIM],
                                           int half)
{
    constexpr int NV = 4 + NDIM, A = 3 + NDIM, E = 2 + NDIM;
    constexpr int sg = SIDE == 0 ? 1 : -1;
    const int n = g.n[D];
    const int b = SIDE == 0 ? 0 : n - 1;
    const T idx = T(inv_width(g, D, b));   // 1/dx_D, or 1/width of the boundary cell on non-uniform cells
    bool bad = false;

    T W[4][NV];
#pragma unroll
    for (int k = 0; k < (STORED ? 3 : 4); k++) {   // the stored terms need only the one-sided stencil
        c[D] = min(max(b + k * sg, 0), n - 1);   // n = 3: the third neighbour is clamped
        const int64_t off = (int64_t)(c[2] + g.off[2]) * g.stride[2] + (int64_t)(c[1] + g.off[1]) * g.stride[1] +
                            (c[0] + g.off[0]);
        T qc[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + off];
        bad |= cons_to_prim<NDIM, T>(g, qc, W[k]);
    }
    c[D] = b;

    T fv[NV];
    if constexpr (STORED) {
        constexpr int F = 2 * D + SIDE;
        const int c1 = D == 0 ? c[1] : c[0], n1 = D == 0 ? g.n[1] : g.n[0], c2 = D == 2 ? c[1] : c[2];
        const T *src = (const T *)g.cbc_fv + g.cbc_off[F] + 8 * ((int64_t)c1 + (int64_t)n1 * c2);
#pragma unroll
        for (int v = 0; v < NV; v++) fv[v] = src[v];
        fv[A] += W[0][A] * src[7];   // the normal part of alpha1 div(u)
    } else {
    // finite-volume terms normal to the face.  The two lanes of a pair
    // compute one flux each on the same instruction stream, lane 0 the flux
    // at b-1/2 (left state: cell b-1 reconstructed from stencil cells 0..4,
    // right state: cell b from 1..5), lane 1 the flux at b+1/2 (cells b from
    // 1..5 and b+1 from 2..6), and exchange them.
    // On non-uniform cells the two cells of the face reconstruct with their
    // own WENO5 coefficients (cells b - 1 + half and b + half).
    constexpr int i0 = at<SIDE>(0), i1 = at<SIDE>(1), i2 = at<SIDE>(2), i3 = at<SIDE>(3), i4 = at<SIDE>(4),
                  i5 = at<SIDE>(5), i6 = at<SIDE>(6);
    const double *cl = coef_row(g, D, b - 1 + half), *cr = coef_row(g, D, b + half);
    T lft[NV], rgt[NV], dummy;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const T s0 = half ? W[i1][v] : W[i0][v], s1 = half ? W[i2][v] : W[i1][v], s2 = half ? W[i3][v] : W[i2][v],
                s3 = half ? W[i4][v] : W[i3][v], s4 = half ? W[i5][v] : W[i4][v], s5 = half ? W[i6][v] : W[i5][v];
        recon_cell<ORDER, T>(cl, s0, s1, s2, s3, s4, T(g.eps), lft[v], dummy);
        recon_cell<ORDER, T>(cr, s1, s2, s3, s4, s5, T(g.eps), dummy, rgt[v]);
    }
    T F[NV], uf;
    bad |= hllc<NDIM, D, T>(g, lft, rgt, F, uf);
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const T other = __shfl_xor(F[v], 1);
        fv[v] = (half ? other - F[v] : F[v] - other) * idx;
    }
    const T uother = __shfl_xor(uf, 1);
    fv[A] += W[0][A] * ((half ? uf - uother : uother - uf) * idx);
    }

    // characteristic form on the boundary cell
    T rate[NV];
    bad |= char_rate<NDIM, D, SIDE, T>(g, W[0], W[1], W[2], idx, one_sided<T>(g, D, SIDE), rate);
#pragma unroll
    for (int v = 0; v < NV; v++) delta[v] += rate[v] - fv[v];
    return bad;
}

// One lane (STORED) or two lanes per (characteristic face, boundary cell of
// it).  A cell on several characteristic faces (an edge or corner) belongs
// to the first of them, whose lanes add the changes of all of them in face
// order: every cell is written by one lane, once, in a fixed order.
// smax_partial (the split path's last stage of a step followed by another of
// the same run): the pass also reduces max_d (|u_d| + c) of the cells it
// writes, as the z kernel does for the others, one maximum per workgroup.
template <int NDIM, class T, int ORDER, bool STORED>
__device__ __forceinline__ double cbc_cell(const Grid &g, const CbcFaces &F, const T *__restrict__ q, T *out, int mode,
                                           double dt, const double *__restrict__ dt_dev, bool reduce, int64_t gt,
                                           bool &bad);

template <int NDIM, class T, int ORDER, bool STORED>
__global__ void __launch_bounds__(kCbcThreads, MFC_CBC_WAVES)
    k_cbc(Grid g, CbcFaces F, const T *__restrict__ q, T *out, int mode, double dt, const double *__restrict__ dt_dev,
          int *__restrict__ flag, double *__restrict__ smax_partial)
{
    bool bad = false;
    const int64_t gt = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double smax = cbc_cell<NDIM, T, ORDER, STORED>(g, F, q, out, mode, dt, dt_dev, smax_partial != nullptr, gt, bad);
    if (smax_partial) {   // every lane of the workgroup (one wavefront) takes part
        static_assert(kCbcThreads == 64, "one wavefront per workgroup");
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) smax = __builtin_fmax(smax, __shfl_xor(smax, o, 64));
        if (threadIdx.x == 0) smax_partial[blockIdx.x] = smax;
    }
    if (bad) atomicOr(flag, 1);
}

template <int NDIM, class T, int ORDER, bool STORED>
__device__ __forceinline__ double cbc_cell(const Grid &g, const CbcFaces &F, const T *__restrict__ q, T *out, int mode,
                                           double dt, const double *__restrict__ dt_dev, bool reduce, int64_t gt,
                                           bool &bad)
{
    constexpr int NV = 4 + NDIM;
    const int64_t t = STORED ? gt : gt >> 1;   // the cell; both lanes of a pair leave or stay together
    const int half = STORED ? 1 : (int)(gt & 1);
    if (t >= F.start[6]) return 0.0;
    int my = -1;
    int64_t first = 0;
#pragma unroll
    for (int f = 0; f < 2 * NDIM; f++)
        if (((F.mask >> f) & 1) && t >= F.start[f]) {
            my = f;
            first = F.start[f];
        }
    if (my < 0) return 0.0;
    const int D = my >> 1;
    const int nD = D == 0 ? g.n[0] : (D == 1 ? g.n[1] : g.n[2]);
    const int b = (my & 1) ? nD - 1 : 0;
    const int n1 = D == 0 ? g.n[1] : g.n[0];
    const int64_t local = t - first;
    const int a = (int)(local % n1), a2 = (int)(local / n1);
    int c[3];
    c[0] = D == 0 ? b : a;
    c[1] = D == 0 ? a : (D == 1 ? b : a2);
    c[2] = D == 2 ? b : a2;
    int on = 0;   // bit f: the cell lies on characteristic face f
#pragma unroll
    for (int f = 0; f < 2 * NDIM; f++)
        if (((F.mask >> f) & 1) && c[f >> 1] == ((f & 1) ? g.n[f >> 1] - 1 : 0)) on |= 1 << f;
    if (on & ((1 << my) - 1)) return 0.0;   // an earlier face owns this cell

    T delta[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) delta[v] = T(0);
    if (on & 1) bad |= face_delta<NDIM, 0, 0, T, ORDER, STORED>(g, c, q, delta, half);
    if (on & 2) bad |= face_delta<NDIM, 0, 1, T, ORDER, STORED>(g, c, q, delta, half);
    if constexpr (NDIM >= 2) {
        if (on & 4) bad |= face_delta<NDIM, 1, 0, T, ORDER, STORED>(g, c, q, delta, half);
        if (on & 8) bad |= face_delta<NDIM, 1, 1, T, ORDER, STORED>(g, c, q, delta, half);
    }
    if constexpr (NDIM == 3) {
        if (on & 16) bad |= face_delta<NDIM, 2, 0, T, ORDER, STORED>(g, c, q, delta, half);
        if (on & 32) bad |= face_delta<NDIM, 2, 1, T, ORDER, STORED>(g, c, q, delta, half);
    }

    const int64_t off = (int64_t)(c[2] + g.off[2]) * g.stride[2] + (int64_t)(c[1] + g.off[1]) * g.stride[1] +
                        (c[0] + g.off[0]);
    const T w_dt = mode == 0 ? T(1) : T((mode == 1 ? 1.0 : (mode == 2 ? 0.25 : 2.0 / 3.0)) * (dt_dev ? *dt_dev : dt));
    double smax = 0.0;
    if (half) {
        T r[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) {
            r[v] = out[v * g.vstride + off] + w_dt * delta[v];
            out[v * g.vstride + off] = r[v];
        }
        if (reduce) {   // as the x+y pass of a first stage forms it from the stored values
            T w[NV];
            cons_to_prim<NDIM, T>(g, r, w);
            double Gam, Pi;
            mixture<double>(g, double(w[NV - 1]), Gam, Pi);
            const double cs = sqrtT(sound2<double>(Gam, Pi, double(w[0]) + double(w[1]), double(w[NV - 2])));
#pragma unroll
            for (int d = 0; d < NDIM; d++) {
                const double a = __builtin_fabs(double(w[2 + d])) + cs;
                smax = __builtin_fmax(smax, g.stretched ? a * inv_width(g, d, c[d]) : a);
            }
        }
    }
    return smax;
}

template <class T, int ORDER>
void launch_t(mfc_grid *h, const void *q, void *out, int mode, double dt, const double *dt_dev, hipStream_t s,
              double *smax_partial)
{
    const Grid &g = h->g;
    CbcFaces F{};
    int64_t total = 0;
    // the split path (3D) applies the x and y faces inside its x+y kernel
    // and keeps the normal terms of the z faces' cells; the other paths
    // recompute them here for every face
    const bool stored = g.cbc_mask != 0;
    for (int f = 0; f < 6; f++) {
        F.start[f] = total;
        if (f >= 2 * g.ndim || g.bc[f] != MFC_BC_CHARACTERISTIC || (stored && f < 4)) continue;
        const int d = f >> 1;
        F.mask |= 1 << f;
        // inactive dimensions have n = 1
        total += (int64_t)(d == 0 ? g.n[1] : g.n[0]) * (d == 2 ? g.n[1] : g.n[2]);
    }
    F.start[6] = total;
    if (F.mask == 0) return;
    const int lanes = stored ? 1 : 2;
    const dim3 grid((unsigned)((lanes * total + kCbcThreads - 1) / kCbcThreads));
    const T *a = (const T *)q;
    T *o = (T *)out;
    switch (g.ndim) {
    case 1:
        hipLaunchKernelGGL((k_cbc<1, T, ORDER, false>), grid, dim3(kCbcThreads), 0, s, g, F, a, o, mode, dt, dt_dev,
                           h->flag, nullptr);
        break;
    case 2:
        hipLaunchKernelGGL((k_cbc<2, T, ORDER, false>), grid, dim3(kCbcThreads), 0, s, g, F, a, o, mode, dt, dt_dev,
                           h->flag, nullptr);
        break;
    default:
        if (stored)
            hipLaunchKernelGGL((k_cbc<3, T, ORDER, true>), grid, dim3(kCbcThreads), 0, s, g, F, a, o, mode, dt,
                               dt_dev, h->flag, smax_partial);
        else
            hipLaunchKernelGGL((k_cbc<3, T, ORDER, false>), grid, dim3(kCbcThreads), 0, s, g, F, a, o, mode, dt,
                               dt_dev, h->flag, nullptr);
    }
}

}  // namespace

int64_t cbc_stored_blocks(const Grid &g)
{
    int64_t total = 0;
    for (int f = 4; f < 6; f++)
        if (g.ndim == 3 && g.bc[f] == MFC_BC_CHARACTERISTIC) total += (int64_t)g.n[0] * g.n[1];
    return (total + kCbcThreads - 1) / kCbcThreads;
}

bool has_cbc(const mfc_grid *h)
{
    for (int f = 0; f < 2 * h->g.ndim; f++)
        if (h->g.bc[f] == MFC_BC_CHARACTERISTIC) return true;
    return false;
}

int launch_cbc(mfc_grid *h, const void *q, void *out, int mode, double dt, const double *dt_dev, hipStream_t s,
               double *smax_partial)
{
    const bool f32 = h->desc.precision == MFC_FP32_MIXED;
    double *sp = smax_partial;
    switch (h->g.order) {
    case 3:
        f32 ? launch_t<float, 3>(h, q, out, mode, dt, dt_dev, s, sp) : launch_t<double, 3>(h, q, out, mode, dt, dt_dev, s, sp);
        break;
    case 1:
        f32 ? launch_t<float, 1>(h, q, out, mode, dt, dt_dev, s, sp) : launch_t<double, 1>(h, q, out, mode, dt, dt_dev, s, sp);
        break;
    default:
        f32 ? launch_t<float, 5>(h, q, out, mode, dt, dt_dev, s, sp) : launch_t<double, 5>(h, q, out, mode, dt, dt_dev, s, sp);
    }
    return hip_status(hipGetLastError(), "characteristic boundary launch");
}

}  // namespace mfc
