// Device building blocks of the five-equation right-hand side: mixture
// stiffened-gas EOS, WENO5-JS reconstruction and the HLLC flux.
//
// Everything here is inlined into the kernels; the state ordering is
// [a1r1, a2r2, mom_1..mom_NDIM, rhoE, alpha1] (conservative) and
// [a1r1, a2r2, u_1..u_NDIM, p, alpha1] (primitive).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mfc {

constexpr int NG = 3;  // ghost layers: WENO5 reads 2 cells past the face cell

// Grid geometry and material constants passed by value to every kernel.
struct Grid {
    int ndim;
    int n[3];         // interior cells (1 on inactive dims)
    int p[3];         // padded extents
    int off[3];       // ghost offset per dim (NG or 0)
    int64_t stride[3];  // element strides of x, y, z (1, px, px*py)
    int64_t vstride;  // stride between variables (px*py*pz)
    double inv_dx[3];
    double dxmin;
    // mixture EOS coefficients: Gamma = a1*g1 + (1-a1)*g2, Pi = a1*h1 + (1-a1)*h2
    double g1, g2, h1, h2;
    double eps;       // WENO epsilon
};

// ---------------------------------------------------------------- reciprocal
// Correctly-rounded-in-practice double reciprocal: hardware estimate refined
// by two Newton-Raphson steps (r <- r + r (1 - x r)), each doubling the
// number of correct bits.  Used where a full IEEE division sequence would be
// the dominant cost; inputs are normal, finite and nonzero on physical states.
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    return r;
}

// ------------------------------------------------------------------- EOS
__device__ __forceinline__ void mixture(const Grid &g, double a1, double &Gam, double &Pi)
{
    double a2 = 1.0 - a1;
    Gam = a1 * g.g1 + a2 * g.g2;
    Pi = a1 * g.h1 + a2 * g.h2;
}

// Frozen mixture sound speed squared, c^2 = ((Gamma + 1) p + Pi) / (Gamma rho).
__device__ __forceinline__ double sound2(double Gam, double Pi, double rho, double p)
{
    return ((Gam + 1.0) * p + Pi) / (Gam * rho);
}

__device__ __forceinline__ bool nonphysical(double rho, double c2)
{
    return !(rho > 0.0) || !(c2 > 0.0) || !__builtin_isfinite(rho) || !__builtin_isfinite(c2);
}

// Conservative -> primitive for one cell; returns true if non-physical.
template <int NDIM>
__device__ __forceinline__ bool cons_to_prim(const Grid &g, const double *q, double *w)
{
    constexpr int E = 2 + NDIM, A = 3 + NDIM;
    double rho = q[0] + q[1];
    double ir = 1.0 / rho;
    double Gam, Pi;
    mixture(g, q[A], Gam, Pi);
    double ke = 0.0;
    w[0] = q[0];
    w[1] = q[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) {
        w[2 + m] = q[2 + m] * ir;
        ke += q[2 + m] * w[2 + m];
    }
    w[E] = (q[E] - 0.5 * ke - Pi) / Gam;
    w[A] = q[A];
    return nonphysical(rho, sound2(Gam, Pi, rho, w[E]));
}

template <int NDIM>
__device__ __forceinline__ void prim_to_cons(const Grid &g, const double *w, double *q)
{
    constexpr int E = 2 + NDIM, A = 3 + NDIM;
    double rho = w[0] + w[1];
    double Gam, Pi;
    mixture(g, w[A], Gam, Pi);
    double u2 = 0.0;
    q[0] = w[0];
    q[1] = w[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) {
        q[2 + m] = rho * w[2 + m];
        u2 += w[2 + m] * w[2 + m];
    }
    q[E] = Gam * w[E] + Pi + 0.5 * rho * u2;
    q[A] = w[A];
}

// ----------------------------------------------------------------- WENO5-JS
// Both reconstructions a cell contributes, from its 5-cell stencil
// (vm2, vm1, v0, vp1, vp2): `plus` at its right face x_{i+1/2} (the left
// state of that face) and `minus` at its left face x_{i-1/2}.  The two share
// the divided differences and the smoothness indicators.  The nonlinear
// weights a_r = d_r/(eps + beta_r)^2 are normalised through common
// denominators, a_r ~ d_r prod_{s != r} (eps + beta_s)^2, so that one
// reciprocal serves both faces; the result is written as v0 plus a weighted
// sum of candidate increments, which reproduces constants exactly.
__device__ __forceinline__ void weno5_pair(double vm2, double vm1, double v0, double vp1, double vp2,
                                           double eps, double &plus, double &minus)
{
    const double dm2 = vm1 - vm2, dm1 = v0 - vm1, d0 = vp1 - v0, d1 = vp2 - vp1;
    const double b0 = (10.0 / 3.0) * dm1 * dm1 - (11.0 / 3.0) * dm1 * dm2 + (4.0 / 3.0) * dm2 * dm2;
    const double b1 = (4.0 / 3.0) * d0 * d0 - (5.0 / 3.0) * d0 * dm1 + (4.0 / 3.0) * dm1 * dm1;
    const double b2 = (10.0 / 3.0) * d0 * d0 - (11.0 / 3.0) * d0 * d1 + (4.0 / 3.0) * d1 * d1;
    const double e0 = eps + b0, e1 = eps + b1, e2 = eps + b2;
    const double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
    const double m0 = s1 * s2, m1 = s0 * s2, m2 = s0 * s1;
    // candidate increments at x_{i+1/2} and x_{i-1/2}
    const double cp0 = (5.0 / 6.0) * dm1 - (1.0 / 3.0) * dm2;
    const double cp1 = (1.0 / 3.0) * d0 + (1.0 / 6.0) * dm1;
    const double cp2 = (2.0 / 3.0) * d0 - (1.0 / 6.0) * d1;
    const double cm0 = (1.0 / 6.0) * dm2 - (2.0 / 3.0) * dm1;
    const double cm1 = -(1.0 / 3.0) * dm1 - (1.0 / 6.0) * d0;
    const double cm2 = (1.0 / 3.0) * d1 - (5.0 / 6.0) * d0;
    const double ap0 = 0.1 * m0, ap1 = 0.6 * m1, ap2 = 0.3 * m2;
    const double am0 = 0.3 * m0, am1 = 0.6 * m1, am2 = 0.1 * m2;
    const double sp = ap0 + ap1 + ap2, sm = am0 + am1 + am2;
    const double np = ap0 * cp0 + ap1 * cp1 + ap2 * cp2;
    const double nm = am0 * cm0 + am1 * cm1 + am2 * cm2;
    const double r = rcp(sp * sm);
    plus = v0 + np * (sm * r);
    minus = v0 + nm * (sp * r);
}

// ------------------------------------------------------------------- HLLC
// HLLC flux through a face normal to DIR between primitive states wL and wR
// (NV = 4 + NDIM values each).  F[0 .. NV-2]: flux of the conserved rows;
// F[NV-1]: alpha1_face * u_face; uf: face normal velocity.  Davis wave-speed
// estimates, Toro's contact speed s* (= u*), star states scaled by
// xi = (s_K - u_K)/(s_K - s*).  The region of the fan at x/t = 0 is picked
// exactly as in the case table: s_L >= 0 -> L, s_R <= 0 -> R, otherwise L*
// if s* >= 0 and R* if not; alpha1 jumps only across the contact.
// Returns true if either side is non-physical.
template <int NDIM, int DIR>
__device__ __forceinline__ bool hllc(const Grid &g, const double *wL, const double *wR, double *F, double &uf)
{
    constexpr int NV = 4 + NDIM, E = 2 + NDIM, A = 3 + NDIM;
    const double rhoL = wL[0] + wL[1], rhoR = wR[0] + wR[1];
    const double uL = wL[2 + DIR], uR = wR[2 + DIR];
    const double pL = wL[E], pR = wR[E];
    double GL, PL, GR, PR;
    mixture(g, wL[A], GL, PL);
    mixture(g, wR[A], GR, PR);
    const double c2L = sound2(GL, PL, rhoL, pL), c2R = sound2(GR, PR, rhoR, pR);
    const bool bad = nonphysical(rhoL, c2L) || nonphysical(rhoR, c2R);
    const double cL = __builtin_sqrt(c2L), cR = __builtin_sqrt(c2R);
    const double sL = __builtin_fmin(uL - cL, uR - cR);
    const double sR = __builtin_fmax(uL + cL, uR + cR);
    const double mL = rhoL * (sL - uL), mR = rhoR * (sR - uR);
    const double sS = (pR - pL + mL * uL - mR * uR) / (mL - mR);

    const bool super_L = sL >= 0.0, super_R = sR <= 0.0;
    const bool useL = super_L || (!super_R && sS >= 0.0);
    const bool star = !super_L && !super_R;

    // the side whose state (plain or starred) is the fan at x/t = 0
    double w[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) w[v] = useL ? wL[v] : wR[v];
    const double rho = useL ? rhoL : rhoR;
    const double Gam = useL ? GL : GR, Pi = useL ? PL : PR;
    const double sK = useL ? sL : sR;
    const double un = w[2 + DIR], p = w[E];
    double u2 = 0.0;
#pragma unroll
    for (int m = 0; m < NDIM; m++) u2 += w[2 + m] * w[2 + m];
    const double En = Gam * p + Pi + 0.5 * rho * u2;

    // physical flux of that side
    F[0] = w[0] * un;
    F[1] = w[1] * un;
#pragma unroll
    for (int m = 0; m < NDIM; m++) F[2 + m] = rho * w[2 + m] * un + (m == DIR ? p : 0.0);
    F[E] = (En + p) * un;

    // star correction s_K (q*_K - q_K), with xi - 1 = (s* - u)/(s_K - s*)
    const double sku = sK - un;
    const double ism = 1.0 / (sK - sS);
    const double xim1 = (sS - un) * ism;
    const double xi = sku * ism;
    double dq[NV - 1];
    dq[0] = xim1 * w[0];
    dq[1] = xim1 * w[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) dq[2 + m] = (m == DIR) ? rho * (xi * sS - un) : xim1 * rho * w[2 + m];
    dq[E] = xim1 * En + xi * (sS - un) * (rho * sS + p / sku);
#pragma unroll
    for (int v = 0; v < NV - 1; v++) F[v] = star ? F[v] + sK * dq[v] : F[v];

    uf = star ? sS : un;
    F[A] = w[A] * uf;
    return bad;
}

}  // namespace mfc
