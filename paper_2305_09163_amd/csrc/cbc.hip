// Characteristic-based non-reflecting boundaries (Sec. 3.3: the paper's
// characteristic boundary conditions, in the time-dependent form of
// Thompson): a post-pass over the boundary cells of every face marked
// MFC_BC_CHARACTERISTIC, run after the stage kernel of any path.
//
// For each boundary cell it recomputes the finite-volume terms normal to
// the face (the two HLLC fluxes of the cell along that dimension, its share
// of alpha1 div(u)) and replaces them by the characteristic form: wave
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
#include "internal.h"

namespace mfc {
namespace {

constexpr int kCbcThreads = 256;

template <int NDIM, int D, class T, int ORDER>
__global__ void __launch_bounds__(kCbcThreads)
    k_cbc(Grid g, int side, const T *__restrict__ q, T *out, int mode, double dt, const double *__restrict__ dt_dev,
          int *__restrict__ flag)
{
    constexpr int NV = 4 + NDIM, A = 3 + NDIM, E = 2 + NDIM;
    constexpr int O1 = D == 0 ? 1 : 0, O2 = D == 2 ? 1 : 2;
    const int n1 = O1 < NDIM ? g.n[O1] : 1, n2 = O2 < NDIM ? g.n[O2] : 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n1 * n2) return;
    int c[3] = {0, 0, 0};
    c[O1] = t % n1;
    c[O2] = t / n1;
    const int n = g.n[D];
    const int b = side == 0 ? 0 : n - 1, sg = side == 0 ? 1 : -1;
    const T idx = T(g.inv_dx[D]);
    bool bad = false;

    // primitives of cells b-3 .. b+3 along D (clamped into the interior:
    // the non-periodic boundary rule)
    T w[7][NV];
#pragma unroll
    for (int o = 0; o < 7; o++) {
        c[D] = min(max(b - 3 + o, 0), n - 1);
        const int64_t off = (int64_t)(c[2] + g.off[2]) * g.stride[2] + (int64_t)(c[1] + g.off[1]) * g.stride[1] +
                            (c[0] + g.off[0]);
        T qc[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + off];
        bad |= cons_to_prim<NDIM, T>(g, qc, w[o]);
    }

    // finite-volume terms normal to the face: fluxes at b-1/2 and b+1/2
    T pl[NV], mb[NV], pb[NV], mr[NV], dummy[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        recon_pair<ORDER, T>(w[0][v], w[1][v], w[2][v], w[3][v], w[4][v], T(g.eps), pl[v], dummy[v]);
        recon_pair<ORDER, T>(w[1][v], w[2][v], w[3][v], w[4][v], w[5][v], T(g.eps), pb[v], mb[v]);
        recon_pair<ORDER, T>(w[2][v], w[3][v], w[4][v], w[5][v], w[6][v], T(g.eps), dummy[v], mr[v]);
    }
    T Flo[NV], Fhi[NV], ulo, uhi;
    bad |= hllc<NDIM, D, T>(g, pl, mb, Flo, ulo);
    bad |= hllc<NDIM, D, T>(g, pb, mr, Fhi, uhi);
    T fv[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) fv[v] = (Flo[v] - Fhi[v]) * idx;
    fv[A] += w[3][A] * ((uhi - ulo) * idx);

    // characteristic form on the boundary cell
    const T *wb = w[3];
    T dw[NV];
#pragma unroll
    for (int v = 0; v < NV; v++)
        dw[v] = T(sg) * (T(-3) * wb[v] + T(4) * w[3 + sg][v] - w[3 + 2 * sg][v]) * (T(0.5) * idx);
    T Gam, Pi;
    mixture<T>(g, wb[A], Gam, Pi);
    const T rho = wb[0] + wb[1], p = wb[E], un = wb[2 + D];
    const T c2 = sound2<T>(Gam, Pi, rho, p), cs = sqrtT(c2);
    bad |= nonphysical<T>(rho, c2);
    auto enters = [&](T lam) { return side == 0 ? lam > T(0) : lam < T(0); };
    const T lam1 = un - cs, lam5 = un + cs;
    const T L1 = enters(lam1) ? T(0) : lam1 * (dw[E] - rho * cs * dw[2 + D]);
    const T L5 = enters(lam5) ? T(0) : lam5 * (dw[E] + rho * cs * dw[2 + D]);
    const bool in_m = enters(un);
    const T irc2 = rcp(rho * c2), S = T(0.5) * (L5 + L1);
    T rkt[2];
#pragma unroll
    for (int k = 0; k < 2; k++) rkt[k] = -(in_m ? T(0) : un * (dw[k] - wb[k] * irc2 * dw[E])) - wb[k] * irc2 * S;
    T ut[NDIM];
#pragma unroll
    for (int m = 0; m < NDIM; m++) ut[m] = m == D ? -(L5 - L1) * rcp(T(2) * rho * cs) : (in_m ? T(0) : -un * dw[2 + m]);
    const T pt = -S, at = in_m ? T(0) : -un * dw[A];
    const T rhot = rkt[0] + rkt[1];
    T dq[NV], u2 = T(0), uut = T(0);
    dq[0] = rkt[0];
    dq[1] = rkt[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) {
        dq[2 + m] = wb[2 + m] * rhot + rho * ut[m];
        u2 += wb[2 + m] * wb[2 + m];
        uut += wb[2 + m] * ut[m];
    }
    dq[E] = Gam * pt + (T(g.g1 - g.g2) * p + T(g.h1 - g.h2)) * at + T(0.5) * u2 * rhot + rho * uut;
    dq[A] = at;

    // replace the normal finite-volume terms of the stage result
    c[D] = b;
    const int64_t off = (int64_t)(c[2] + g.off[2]) * g.stride[2] + (int64_t)(c[1] + g.off[1]) * g.stride[1] +
                        (c[0] + g.off[0]);
    const T w_dt = mode == 0 ? T(1) : T((mode == 1 ? 1.0 : (mode == 2 ? 0.25 : 2.0 / 3.0)) * (dt_dev ? *dt_dev : dt));
#pragma unroll
    for (int v = 0; v < NV; v++) out[v * g.vstride + off] += w_dt * (dq[v] - fv[v]);
    if (bad) atomicOr(flag, 1);
}

template <int NDIM, class T, int ORDER>
void launch_faces(mfc_grid *h, const T *q, T *out, int mode, double dt, const double *dt_dev, hipStream_t s)
{
    const Grid &g = h->g;
    for (int d = 0; d < NDIM; d++)
        for (int side = 0; side < 2; side++) {
            if (g.bc[2 * d + side] != MFC_BC_CHARACTERISTIC) continue;
            const int n1 = d == 0 ? g.n[1] : g.n[0], n2 = d == 2 ? g.n[1] : g.n[2];
            const dim3 grid((unsigned)((int64_t)n1 * n2 + kCbcThreads - 1) / kCbcThreads);
            if (d == 0)
                hipLaunchKernelGGL((k_cbc<NDIM, 0, T, ORDER>), grid, dim3(kCbcThreads), 0, s, g, side, q, out, mode,
                                   dt, dt_dev, h->flag);
            else if (d == 1)
                hipLaunchKernelGGL((k_cbc<NDIM, (NDIM >= 2 ? 1 : 0), T, ORDER>), grid, dim3(kCbcThreads), 0, s, g,
                                   side, q, out, mode, dt, dt_dev, h->flag);
            else
                hipLaunchKernelGGL((k_cbc<NDIM, (NDIM == 3 ? 2 : 0), T, ORDER>), grid, dim3(kCbcThreads), 0, s, g,
                                   side, q, out, mode, dt, dt_dev, h->flag);
        }
}

template <class T, int ORDER>
void launch_t(mfc_grid *h, const void *q, void *out, int mode, double dt, const double *dt_dev, hipStream_t s)
{
    const T *a = (const T *)q;
    T *o = (T *)out;
    switch (h->g.ndim) {
    case 1: launch_faces<1, T, ORDER>(h, a, o, mode, dt, dt_dev, s); break;
    case 2: launch_faces<2, T, ORDER>(h, a, o, mode, dt, dt_dev, s); break;
    default: launch_faces<3, T, ORDER>(h, a, o, mode, dt, dt_dev, s);
    }
}

}  // namespace

bool has_cbc(const mfc_grid *h)
{
    for (int f = 0; f < 2 * h->g.ndim; f++)
        if (h->g.bc[f] == MFC_BC_CHARACTERISTIC) return true;
    return false;
}

int launch_cbc(mfc_grid *h, const void *q, void *out, int mode, double dt, const double *dt_dev, hipStream_t s)
{
    const bool f32 = h->desc.precision == MFC_FP32_MIXED;
    switch (h->g.order) {
    case 3:
        f32 ? launch_t<float, 3>(h, q, out, mode, dt, dt_dev, s) : launch_t<double, 3>(h, q, out, mode, dt, dt_dev, s);
        break;
    case 1:
        f32 ? launch_t<float, 1>(h, q, out, mode, dt, dt_dev, s) : launch_t<double, 1>(h, q, out, mode, dt, dt_dev, s);
        break;
    default:
        f32 ? launch_t<float, 5>(h, q, out, mode, dt, dt_dev, s) : launch_t<double, 5>(h, q, out, mode, dt, dt_dev, s);
    }
    return hip_status(hipGetLastError(), "characteristic boundary launch");
}

}  // namespace mfc
