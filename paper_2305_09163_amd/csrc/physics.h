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
    return __builtin_fma(Gam + 1.0, p, Pi) * rcp(Gam * rho);
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
    double ir = rcp(rho);
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
    const double iG = rcp(Gam);
    w[E] = (q[E] - 0.5 * ke - Pi) * iG;
    w[A] = q[A];
    // c^2 = ((Gamma + 1) p + Pi) / (Gamma rho): its sign and finiteness
    // without the division
    const double num = __builtin_fma(Gam + 1.0, w[E], Pi);
    return !(rho > 0.0) || !(num * iG > 0.0) || !__builtin_isfinite(rho) || !__builtin_isfinite(num * iG * ir);
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
// the divided differences a = v0 - vm1, b = vm1 - vm2, c = vp1 - v0,
// d = vp2 - vp1 and the smoothness indicators.
//
// Arithmetic, equal to the Jiang-Shu definitions up to rounding:
//   - every smoothness indicator is scaled by 3, with eps scaled alike
//     (3 beta_0 = a (10a - 11b) + 4b^2, 3 beta_1 = c (4c - 5a) + 4a^2,
//     3 beta_2 = c (10c - 11d) + 4d^2); the weights depend only on ratios of
//     (eps + beta_r)^2, so the common factor cancels;
//   - a_r = d_r/(eps + beta_r)^2 is normalised through common denominators,
//     a_r ~ d_r prod_{s != r} (eps + beta_s)^2, with the ideal weights scaled
//     by 10 (1, 6, 3 and 3, 6, 1), so one reciprocal serves both faces;
//   - the candidates enter as increments over v0 scaled by 6
//     (6 (p_r - v0) at x_{i+1/2}: 5a - 2b, 2c + a, 4c - d; at x_{i-1/2}:
//     b - 4a, -(2a + c), 2d - 5c), which reproduces constants exactly.
__device__ __forceinline__ void weno5_pair(double vm2, double vm1, double v0, double vp1, double vp2,
                                           double eps, double &plus, double &minus)
{
    const double b = vm1 - vm2, a = v0 - vm1, c = vp1 - v0, d = vp2 - vp1;
    const double e3 = 3.0 * eps;
    const double e0 = __builtin_fma(a, __builtin_fma(10.0, a, -11.0 * b), __builtin_fma(4.0 * b, b, e3));
    const double e1 = __builtin_fma(c, __builtin_fma(4.0, c, -5.0 * a), __builtin_fma(4.0 * a, a, e3));
    const double e2 = __builtin_fma(c, __builtin_fma(10.0, c, -11.0 * d), __builtin_fma(4.0 * d, d, e3));
    const double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2;
    const double m0 = s1 * s2, m1 = 6.0 * (s0 * s2), m2 = s0 * s1;  // m1 carries the ideal weight 6
    const double sp = __builtin_fma(3.0, m2, m0 + m1);                // weights 1, 6, 3
    const double sm = __builtin_fma(3.0, m0, m1 + m2);                // weights 3, 6, 1
    const double np = __builtin_fma(3.0 * m2, __builtin_fma(4.0, c, -d),
                                    __builtin_fma(m1, __builtin_fma(2.0, c, a), m0 * __builtin_fma(5.0, a, -2.0 * b)));
    const double nm = __builtin_fma(m2, __builtin_fma(2.0, d, -5.0 * c),
                                    __builtin_fma(m1, -__builtin_fma(2.0, a, c), 3.0 * m0 * __builtin_fma(-4.0, a, b)));
    const double r = rcp(6.0 * (sp * sm));
    plus = __builtin_fma(np, sm * r, v0);
    minus = __builtin_fma(nm, sp * r, v0);
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
    const double sS = (pR - pL + mL * uL - mR * uR) * rcp(mL - mR);

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
    const double ism = rcp(sK - sS);
    const double xim1 = (sS - un) * ism;
    const double xi = sku * ism;
    double dq[NV - 1];
    dq[0] = xim1 * w[0];
    dq[1] = xim1 * w[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) dq[2 + m] = (m == DIR) ? rho * (xi * sS - un) : xim1 * rho * w[2 + m];
    // xi (s* - u)(rho s* + p/(s_K - u)) = (s* - u)(xi rho s* + p/(s_K - s*))
    dq[E] = xim1 * En + (sS - un) * __builtin_fma(xi * rho, sS, p * ism);
#pragma unroll
    for (int v = 0; v < NV - 1; v++) F[v] = star ? F[v] + sK * dq[v] : F[v];

    uf = star ? sS : un;
    F[A] = w[A] * uf;
    return bad;
}

}  // namespace mfc
