// Characteristic (non-reflecting) boundary rates of Sec. 3.3, in
// Thompson's time-dependent form for the two-fluid system: shared by the
// boundary post-pass (cbc.hip) and the split stage kernels, which apply it
// to the boundary cells they hold.
#pragma once

#include "physics.h"

namespace mfc {

// Weights of the one-sided derivative at the boundary cell of a
// characteristic face on a non-uniform dimension (Grid::cbc_cf), in the
// arithmetic's type; `on` is false on a uniform dimension.
template <class T>
struct OneSided {
    T c[3];
    bool on;
};
template <class T>
__device__ __forceinline__ OneSided<T> one_sided(const Grid &g, int d, int side)
{
    OneSided<T> o;
    o.on = g.wcoef[d] != nullptr;
#pragma unroll
    for (int t = 0; t < 3; t++) o.c[t] = T(g.cbc_cf[2 * d + side][t]);
    return o;
}

// Rates of the conservative rows of a boundary cell on the characteristic
// face SIDE (0: low, 1: high) normal to dimension D, from the primitives of
// the boundary cell W0 and of the next two cells into the domain W1, W2
// (uniform cells: idx = 1/dx_D; non-uniform: the weights os).  Wave amplitudes L1 = (u-c)(p_x - rho c u_x),
// L5 = (u+c)(p_x + rho c u_x), L_k = u((alpha_k rho_k)_x - alpha_k rho_k
// p_x/(rho c^2)), L_t = u (u_t)_x, L_a = u (alpha1)_x from second-order
// one-sided differences into the domain, every amplitude whose wave enters
// the domain set to zero; p_t = -(L5+L1)/2, u_t = -(L5-L1)/(2 rho c),
// (alpha_k rho_k)_t = -L_k - alpha_k rho_k (L5+L1)/(2 rho c^2),
// (u_t)_t = -L_t, (alpha1)_t = -L_a, carried to the conservative rows
// through the mixture EOS.  Returns true if the cell is non-physical.
template <int NDIM, int D, int SIDE, class T>
__device__ __forceinline__ bool char_rate(const Grid &g, const T *W0, const T *W1, const T *W2, T idx,
                                          const OneSided<T> &os, T *rate)
{
    constexpr int NV = 4 + NDIM, A = 3 + NDIM, E = 2 + NDIM;
    constexpr int sg = SIDE == 0 ? 1 : -1;
    bool bad = false;
    const T *wb = W0;
    T dw[NV];
#pragma unroll
    for (int v = 0; v < NV; v++)
        dw[v] = os.on ? fmaT(os.c[2], W2[v], fmaT(os.c[1], W1[v], os.c[0] * wb[v]))
                      : T(sg) * (T(-3) * wb[v] + T(4) * W1[v] - W2[v]) * (T(0.5) * idx);
    T Gam, Pi;
    mixture<T>(g, wb[A], Gam, Pi);
    const T rho = wb[0] + wb[1], p = wb[E], un = wb[2 + D];
    const T c2 = sound2<T>(Gam, Pi, rho, p), cs = sqrtT(c2);
    bad |= nonphysical<T>(rho, c2);
    // a wave enters through the low face when it moves to +x, through the
    // high face when it moves to -x
    auto enters = [](T lam) { return SIDE == 0 ? lam > T(0) : lam < T(0); };
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
    const T pt = -S, at_ = in_m ? T(0) : -un * dw[A];
    const T rhot = rkt[0] + rkt[1];
    T u2 = T(0), uut = T(0);
    rate[0] = rkt[0];
    rate[1] = rkt[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) {
        rate[2 + m] = wb[2 + m] * rhot + rho * ut[m];
        u2 += wb[2 + m] * wb[2 + m];
        uut += wb[2 + m] * ut[m];
    }
    rate[E] = Gam * pt + (T(g.g1 - g.g2) * p + T(g.h1 - g.h2)) * at_ + T(0.5) * u2 * rhot + rho * uut;
    rate[A] = at_;
    return bad;
}

}  // namespace mfc
