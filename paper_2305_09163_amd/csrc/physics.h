// Device building blocks of the five-equation right-hand side: mixture
// stiffened-gas EOS, WENO5-JS reconstruction and the HLLC flux.
//
// Everything here is inlined into the kernels; the state ordering is
// [a1r1, a2r2, mom_1..mom_NDIM, rhoE, alpha1] (conservative) and
// [a1r1, a2r2, u_1..u_NDIM, p, alpha1] (primitive).
//
// Two precisions share the code, selected by the storage type T:
//   double  everything in FP64;
//   float   FP32 storage, reconstruction and Riemann solve, except the
//           mixture pressure recovery p = (rho E - rho|u|^2/2 - Pi)/Gamma and
//           the HLLC contact speed s*, which are evaluated in FP64 because
//           both cancel large terms (Pi ~ 8e8 Pa in water against p ~ 1e5).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "../../include/mfc.h"   // MFC_BC_* (boundary kinds)

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
    int bc[6];        // boundary kind per face (x-, x+, y-, y+, z-, z+): MFC_BC_*
    int order;        // reconstruction of the staged path: 5 WENO5, 3 WENO3, 1 first order
    // Kapila alpha1 equation (kapila != 0): rho_k c_k^2 = zg[k] p + zp[k]
    int kapila;
    double zg[2], zp[2];  // gamma_k and gamma_k pi_k
    // non-uniform cells (device tables; null on a uniform dimension):
    // wcoef[d][(i + 1) * kStretchCoef ...] the WENO5 coefficients of cell i
    // (-1 <= i <= n_d), winv[d][i] = 1 / width of interior cell i
    int stretched;
    const double *wcoef[3];
    const double *winv[3];
    // characteristic faces on the split path: bit f of cbc_mask marks face f
    // (x-, x+, y-, y+, z-, z+); the x+y kernel applies the x and y faces to
    // their boundary cells itself, the z kernel stores the finite-volume
    // terms normal to a z face of its boundary cells (7 flux differences,
    // then the normal part of div(u)) at cbc_fv + cbc_off[f] + 8 (x + nx y),
    // in the storage type, for the boundary pass
    int cbc_mask;
    void *cbc_fv;
    int64_t cbc_off[6];
    // characteristic face f on a non-uniform dimension: weights of the
    // boundary cell and of the next two cells into the domain in the
    // second-order one-sided derivative at the boundary cell's centre
    double cbc_cf[6][3];
};
constexpr int kStretchCoef = 42;

// Store the normal finite-volume terms of a boundary cell of characteristic
// face F (the split kernels; read back by the boundary post-pass).
template <int F, class T>
__device__ __forceinline__ void store_normal_terms(const Grid &g, int c1, int n1, int c2, const T *L, T divu)
{
    T *dst = (T *)g.cbc_fv + g.cbc_off[F] + 8 * ((int64_t)c1 + (int64_t)n1 * c2);
#pragma unroll
    for (int v = 0; v < 7; v++) dst[v] = L[v];
    dst[7] = divu;
}

// Interior cell whose value the ghost position i (-NG <= i < n + NG) holds
// after the ghost fill of Sec. 3.3: the adjacent interior cell
// (extrapolation) or the cell one period away (periodic).  The split and
// batched kernels read every neighbour through this map and never read a
// ghost cell, which gives the values a filled ghost layer holds, bit for
// bit, with no fill pass.
__device__ __forceinline__ int bc_cell(int i, int n, int lo, int hi)
{
    if (i < 0) return lo == MFC_BC_PERIODIC ? i + n : 0;
    if (i >= n) return hi == MFC_BC_PERIODIC ? i - n : n - 1;
    return i;
}

// ---------------------------------------------------------------- reciprocal
// Double reciprocal: the hardware estimate (about 24 correct bits) refined by
// Newton-Raphson steps r <- r + r (1 - x r), each doubling the number of
// correct bits.  One step leaves at most 11 ulp (2.4e-15 relative) over
// 4M random inputs spanning 2^-300 .. 2^300 on gfx950; a second step gives
// the correctly rounded reciprocal on all of them and costs two FMAs per
// reciprocal (about 1.4 % of the FP64 benchmark step).  Used where a full
// IEEE division sequence would be the dominant cost; inputs are normal,
// finite and nonzero on physical states.
#ifndef MFC_RCP_STEPS
#define MFC_RCP_STEPS 1
#endif
__device__ __forceinline__ double rcp(double x)
{
    double r = __builtin_amdgcn_rcp(x);
    double e = __builtin_fma(-x, r, 1.0);
    r = __builtin_fma(r, e, r);
    if (MFC_RCP_STEPS > 1) {
        e = __builtin_fma(-x, r, 1.0);
        r = __builtin_fma(r, e, r);
    }
    return r;
}
// Single reciprocal: the hardware instruction (1 ulp).
__device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
// Square roots of sound speeds squared (positive, normal and finite on
// physical states; on others the cell has been flagged non-physical and the
// value is not used).  Double: the hardware reciprocal square root r ~
// 1/sqrt(a) refined by the coupled Newton-Raphson iteration for
// s ~ sqrt(a), h ~ 1/(2 sqrt(a)) (one step on (s, h), then two
// corrections s <- s + h (a - s^2)): the refinement of the full sqrt()
// sequence without its rescaling of arguments below 2^-767 and its
// handling of 0 and infinity, half its instructions.  Single: the hardware
// square root (1 ulp), as in the FP32 reciprocals.
__device__ __forceinline__ double sqrtT(double a)
{
    const double r = __builtin_amdgcn_rsq(a);
    double s = a * r, h = 0.5 * r;
    const double e = __builtin_fma(-h, s, 0.5);
    s = __builtin_fma(s, e, s);
    h = __builtin_fma(h, e, h);
    double d = __builtin_fma(-s, s, a);
    s = __builtin_fma(d, h, s);
    d = __builtin_fma(-s, s, a);
    return __builtin_fma(d, h, s);
}
__device__ __forceinline__ float sqrtT(float a) { return __builtin_amdgcn_sqrtf(a); }
__device__ __forceinline__ double fminT(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float fminT(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double fmaxT(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float fmaxT(float a, float b) { return __builtin_fmaxf(a, b); }

// ------------------------------------------------------------------- EOS
// Gamma and Pi of the mixture, affine in alpha1 (alpha2 = 1 - alpha1):
// Gamma = g2 + alpha1 (g1 - g2), Pi = h2 + alpha1 (h1 - h2), one FMA each
// (the differences are constants of the grid).
template <class T>
__device__ __forceinline__ void mixture(const Grid &g, T a1, T &Gam, T &Pi)
{
    Gam = fmaT(a1, T(g.g1 - g.g2), T(g.g2));
    Pi = fmaT(a1, T(g.h1 - g.h2), T(g.h2));
}

// Frozen mixture sound speed squared, c^2 = ((Gamma + 1) p + Pi) / (Gamma rho).
template <class T>
__device__ __forceinline__ T sound2(T Gam, T Pi, T rho, T p)
{
    return fmaT(Gam + T(1), p, Pi) * rcp(Gam * rho);
}

template <class T>
__device__ __forceinline__ bool nonphysical(T rho, T c2)
{
    return !(rho > T(0)) || !(c2 > T(0)) || !__builtin_isfinite(rho) || !__builtin_isfinite(c2);
}

// Conservative -> primitive for one cell; returns true if non-physical
// (rho <= 0, c^2 <= 0 or non-finite).  For float storage the pressure is
// recovered in FP64 from the stored (float) energy, momenta and fractions.
template <int NDIM, class T>
__device__ __forceinline__ bool cons_to_prim(const Grid &g, const T *q, T *w)
{
    constexpr int E = 2 + NDIM, A = 3 + NDIM;
    const T rho = q[0] + q[1];
    const T ir = rcp(rho);
    w[0] = q[0];
    w[1] = q[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) w[2 + m] = q[2 + m] * ir;
    w[A] = q[A];
    double ke = 0.0;
#pragma unroll
    for (int m = 0; m < NDIM; m++) ke += double(q[2 + m]) * double(w[2 + m]);
    double Gam, Pi;
    mixture<double>(g, double(q[A]), Gam, Pi);
    // the FP32 form stores p as float: the hardware estimate of 1/Gamma
    // (about 24 correct bits) is as accurate as that rounding
    const double iG = std::is_same<T, float>::value ? __builtin_amdgcn_rcp(Gam) : rcp(Gam);
    const double p = (double(q[E]) - 0.5 * ke - Pi) * iG;
    w[E] = T(p);
    // c^2 = ((Gamma + 1) p + Pi) / (Gamma rho): its sign and finiteness
    // without the division
    const double num = __builtin_fma(Gam + 1.0, p, Pi);
    const double dr = double(rho), di = double(ir);
    return !(dr > 0.0) || !(num * iG > 0.0) || !__builtin_isfinite(dr) || !__builtin_isfinite(num * iG * di);
}

// Primitive -> conservative for one cell (energy assembled in FP64).
template <int NDIM, class T>
__device__ __forceinline__ void prim_to_cons(const Grid &g, const T *w, T *q)
{
    constexpr int E = 2 + NDIM, A = 3 + NDIM;
    const double rho = double(w[0]) + double(w[1]);
    double Gam, Pi;
    mixture<double>(g, double(w[A]), Gam, Pi);
    double u2 = 0.0;
    q[0] = w[0];
    q[1] = w[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) {
        q[2 + m] = T(rho * double(w[2 + m]));
        u2 += double(w[2 + m]) * double(w[2 + m]);
    }
    q[E] = T(Gam * double(w[E]) + Pi + 0.5 * rho * u2);
    q[A] = w[A];
}

// --------------------------------------------------------- Kapila source
// Coefficient h of the alpha1 row's non-conservative term h div(u)
// (eq. fvmdis with h(q) of eq. fvm negated): alpha1 for the Allaire model,
// alpha1 + K for the Kapila model (Sec. 2.1), with
//   K = (Z2 - Z1) / (Z2/alpha2 + Z1/alpha1),  Z_k = rho_k c_k^2 = gamma_k (p + pi_k)
// for stiffened-gas phases at the common pressure p; K = 0 where a volume
// fraction is not positive.
template <class T>
__device__ __forceinline__ T alpha_source(const Grid &g, T alpha1, T p)
{
    if (!g.kapila) return alpha1;
    const T alpha2 = T(1) - alpha1;
    if (!(alpha1 > T(0)) || !(alpha2 > T(0))) return alpha1;
    const T z1 = fmaT(T(g.zg[0]), p, T(g.zp[0])), z2 = fmaT(T(g.zg[1]), p, T(g.zp[1]));
    return alpha1 + (z2 - z1) / (z2 / alpha2 + z1 / alpha1);
}

// ----------------------------------------------------------------- WENO5-JS
// Both reconstructions a cell contributes, from its 5-cell stencil
// (vm2, vm1, v0, vp1, vp2): `plus` at its right face x_{i+1/2} (the left
// state of that face) and `minus` at its left face x_{i-1/2}.  The two share
// the divided differences a = v0 - vm1, b = vm1 - vm2, c = vp1 - v0,
// d = vp2 - vp1 and the smoothness indicators.
//
// Arithmetic, equal to the Jiang-Shu definitions up to rounding:
//   - every smoothness indicator is scaled by 3/4, with eps scaled alike
//     (3/4 beta_0 = a (2.5a - 2.75b) + b^2, 3/4 beta_1 = c (c - 1.25a) + a^2,
//     3/4 beta_2 = c (2.5c - 2.75d) + d^2: no product by a constant is left
//     in the squares); the weights depend only on ratios of (eps + beta_r)^2,
//     so the common factor cancels;
//   - the candidates enter as increments over v0 scaled by 6
//     (6 (p_r - v0) at x_{i+1/2}: 5a - 2b, 2c + a, 4c - d; at x_{i-1/2}:
//     b - 4a, -(2a + c), 2d - 5c), which reproduces constants exactly.
//   - FP64: a_r = d_r/(eps + beta_r)^2 is normalised through common
//     denominators, a_r ~ d_r prod_{s != r} (eps + beta_s)^2, so one
//     reciprocal serves both faces;
//   - FP32: (eps + beta)^2 can exceed the float range across strong jumps,
//     so the weights use the ratio form a_r ~ d_r ((eps + beta_min)/(eps + beta_r))^2,
//     every term of which lies in [0, d_r].
// Ideal weights are scaled by 10: (1, 6, 3) at x_{i+1/2}, (3, 6, 1) at x_{i-1/2}.
__device__ __forceinline__ void weno5_pair(double vm2, double vm1, double v0, double vp1, double vp2,
                                           double eps, double &plus, double &minus)
{
    const double b = vm1 - vm2, a = v0 - vm1, c = vp1 - v0, d = vp2 - vp1;
    const double e3 = 0.75 * eps;
    const double e0 = __builtin_fma(a, __builtin_fma(2.5, a, -2.75 * b), __builtin_fma(b, b, e3));
    const double e1 = __builtin_fma(c, __builtin_fma(-1.25, a, c), __builtin_fma(a, a, e3));
    const double e2 = __builtin_fma(c, __builtin_fma(2.5, c, -2.75 * d), __builtin_fma(d, d, e3));
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

__device__ __forceinline__ void weno5_pair(float vm2, float vm1, float v0, float vp1, float vp2, float eps,
                                           float &plus, float &minus)
{
    const float b = vm1 - vm2, a = v0 - vm1, c = vp1 - v0, d = vp2 - vp1;
    const float e3 = 0.75f * eps;
    const float e0 = __builtin_fmaf(a, __builtin_fmaf(2.5f, a, -2.75f * b), __builtin_fmaf(b, b, e3));
    const float e1 = __builtin_fmaf(c, __builtin_fmaf(-1.25f, a, c), __builtin_fmaf(a, a, e3));
    const float e2 = __builtin_fmaf(c, __builtin_fmaf(2.5f, c, -2.75f * d), __builtin_fmaf(d, d, e3));
    const float emin = __builtin_fminf(e0, __builtin_fminf(e1, e2));
    const float t0 = emin * rcp(e0), t1 = emin * rcp(e1), t2 = emin * rcp(e2);
    const float m0 = t0 * t0, m1 = 6.0f * (t1 * t1), m2 = t2 * t2;
    const float sp = __builtin_fmaf(3.0f, m2, m0 + m1);
    const float sm = __builtin_fmaf(3.0f, m0, m1 + m2);
    const float np = __builtin_fmaf(3.0f * m2, __builtin_fmaf(4.0f, c, -d),
                                   __builtin_fmaf(m1, __builtin_fmaf(2.0f, c, a), m0 * __builtin_fmaf(5.0f, a, -2.0f * b)));
    const float nm = __builtin_fmaf(m2, __builtin_fmaf(2.0f, d, -5.0f * c),
                                   __builtin_fmaf(m1, -__builtin_fmaf(2.0f, a, c), 3.0f * m0 * __builtin_fmaf(-4.0f, a, b)));
    const float r = rcp(6.0f * (sp * sm));
    plus = __builtin_fmaf(np, sm * r, v0);
    minus = __builtin_fmaf(nm, sp * r, v0);
}

// WENO3-JS from (vm1, v0, vp1): candidates at x_{i+1/2} v0 + a/2 and
// v0 + c/2 (a = v0 - vm1, c = vp1 - v0) with ideal weights 1/3, 2/3; at
// x_{i-1/2} v0 - a/2 and v0 - c/2 with 2/3, 1/3; beta_0 = a^2, beta_1 = c^2.
// FP64 through common denominators (one reciprocal for both faces), FP32 in
// the ratio form (terms in [0, 1]) as for WENO5.
__device__ __forceinline__ void weno3_pair(double vm1, double v0, double vp1, double eps, double &plus,
                                           double &minus)
{
    const double a = v0 - vm1, c = vp1 - v0;
    const double e0 = __builtin_fma(a, a, eps), e1 = __builtin_fma(c, c, eps);
    const double s0 = e0 * e0, s1 = e1 * e1;   // (eps + beta_r)^2
    const double dp = __builtin_fma(2.0, s0, s1), dm = __builtin_fma(2.0, s1, s0);
    const double r = rcp(2.0 * (dp * dm));
    plus = __builtin_fma(__builtin_fma(2.0 * s0, c, s1 * a), dm * r, v0);
    minus = __builtin_fma(-__builtin_fma(s0, c, 2.0 * s1 * a), dp * r, v0);
}

__device__ __forceinline__ void weno3_pair(float vm1, float v0, float vp1, float eps, float &plus, float &minus)
{
    const float a = v0 - vm1, c = vp1 - v0;
    const float e0 = __builtin_fmaf(a, a, eps), e1 = __builtin_fmaf(c, c, eps);
    const float emin = __builtin_fminf(e0, e1);
    const float t0 = emin * rcp(e0), t1 = emin * rcp(e1);
    const float m0 = t0 * t0, m1 = t1 * t1;    // proportional to 1/(eps + beta_r)^2
    const float dp = __builtin_fmaf(2.0f, m1, m0), dm = __builtin_fmaf(2.0f, m0, m1);
    plus = __builtin_fmaf(__builtin_fmaf(2.0f * m1, c, m0 * a), rcp(2.0f * dp), v0);
    minus = __builtin_fmaf(-__builtin_fmaf(m1, c, 2.0f * m0 * a), rcp(2.0f * dm), v0);
}

// Both face values of a cell for reconstruction order ORDER from its 5-cell
// stencil: 5 WENO5-JS, 3 WENO3-JS (inner three cells), 1 first order (the
// cell value).
template <int ORDER, class T>
__device__ __forceinline__ void recon_pair(T vm2, T vm1, T v0, T vp1, T vp2, T eps, T &plus, T &minus)
{
    static_assert(ORDER == 5 || ORDER == 3 || ORDER == 1, "reconstruction order 5, 3 or 1");
    if constexpr (ORDER == 5) {
        weno5_pair(vm2, vm1, v0, vp1, vp2, eps, plus, minus);
    } else if constexpr (ORDER == 3) {
        weno3_pair(vm1, v0, vp1, eps, plus, minus);
    } else {
        plus = v0;
        minus = v0;
    }
}

// WENO5 on non-uniform cells from the 42 coefficients of the cell (layout in
// stretch.hip): candidates, a1 and a2 of each stencil are linear in its
// three values, beta_r = a1^2 + (13/3) a2^2, ideal weights per face.  FP64
// directly, FP32 in the ratio form (weights relative to the smallest
// (eps + beta)).  CF is the row in memory, or a copy of it in registers
// (one load per cell for all its variables).
template <class T, class CF>
__device__ __forceinline__ void weno5_nonuniform_pair(const CF &cf, T vm2, T vm1, T v0, T vp1, T vp2, T eps, T &plus,
                                                      T &minus)
{
    const T s[5] = {vm2, vm1, v0, vp1, vp2};
    T pp[3], pm[3], e[3];
#pragma unroll
    for (int r = 0; r < 3; r++) {
        T a1 = T(0), a2 = T(0);
        pp[r] = pm[r] = T(0);
#pragma unroll
        for (int j = 0; j < 3; j++) {
            pp[r] = fmaT(T(cf[3 * r + j]), s[r + j], pp[r]);
            pm[r] = fmaT(T(cf[9 + 3 * r + j]), s[r + j], pm[r]);
            a1 = fmaT(T(cf[18 + 3 * r + j]), s[r + j], a1);
            a2 = fmaT(T(cf[27 + 3 * r + j]), s[r + j], a2);
        }
        e[r] = eps + fmaT(a1, a1, T(13.0 / 3.0) * a2 * a2);
    }
    T wp[3], wm[3], sp = T(0), sm = T(0);
    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const T inv = rcp(e[r] * e[r]);
            wp[r] = T(cf[36 + r]) * inv;
            wm[r] = T(cf[39 + r]) * inv;
        }
    } else {
        const T emin = __builtin_fminf(e[0], __builtin_fminf(e[1], e[2]));
#pragma unroll
        for (int r = 0; r < 3; r++) {
            const T t = emin * rcp(e[r]);
            wp[r] = T(cf[36 + r]) * (t * t);
            wm[r] = T(cf[39 + r]) * (t * t);
        }
    }
    T np = T(0), nm = T(0);
#pragma unroll
    for (int r = 0; r < 3; r++) {
        sp += wp[r];
        sm += wm[r];
        np = fmaT(wp[r], pp[r], np);
        nm = fmaT(wm[r], pm[r], nm);
    }
    plus = np * rcp(sp);
    minus = nm * rcp(sm);
}

// Reconstruction along one direction for a cell whose coefficient row is cf
// (non-null on a non-uniform dimension, where ORDER 5 takes the non-uniform
// WENO5 and first order needs no coefficients).
template <int ORDER, class T>
__device__ __forceinline__ void recon_cell(const double *cf, T vm2, T vm1, T v0, T vp1, T vp2, T eps, T &plus,
                                           T &minus)
{
    if (ORDER == 5 && cf) weno5_nonuniform_pair<T>(cf, vm2, vm1, v0, vp1, vp2, eps, plus, minus);
    else recon_pair<ORDER, T>(vm2, vm1, v0, vp1, vp2, eps, plus, minus);
}

// The coefficient row of a cell copied into registers, in the arithmetic's
// type (a uniform dimension has none: the flag is false).
template <class T>
struct CoefRegs {
    T c[kStretchCoef];
    bool on;
    __device__ __forceinline__ T operator[](int i) const { return c[i]; }
};
template <class T>
__device__ __forceinline__ void load_coefs(const double *__restrict__ cf, CoefRegs<T> &r)
{
    r.on = cf != nullptr;
    if (r.on) {
#pragma unroll
        for (int i = 0; i < kStretchCoef; i++) r.c[i] = T(cf[i]);
    }
}
template <int ORDER, class T>
__device__ __forceinline__ void recon_cell(const CoefRegs<T> &cf, T vm2, T vm1, T v0, T vp1, T vp2, T eps, T &plus,
                                           T &minus)
{
    if (ORDER == 5 && cf.on) weno5_nonuniform_pair<T>(cf, vm2, vm1, v0, vp1, vp2, eps, plus, minus);
    else recon_pair<ORDER, T>(vm2, vm1, v0, vp1, vp2, eps, plus, minus);
}

// Coefficient row of cell i (-1 <= i <= n_d, clamped for lanes past a ragged
// edge, whose results are discarded) along d on a non-uniform dimension.
__device__ __forceinline__ const double *coef_row(const Grid &g, int d, int i)
{
    if (!g.wcoef[d]) return nullptr;
    i = i < -1 ? -1 : (i > g.n[d] ? g.n[d] : i);
    return g.wcoef[d] + (int64_t)(i + 1) * kStretchCoef;
}

// Inverse width of interior cell i along d (clamped like coef_row).
__device__ __forceinline__ double inv_width(const Grid &g, int d, int i)
{
    if (!g.winv[d]) return g.inv_dx[d];
    i = i < 0 ? 0 : (i >= g.n[d] ? g.n[d] - 1 : i);
    return g.winv[d][i];
}

// The linear fifth-order upwind reconstruction (the ideal-weight limit of
// WENO5 on smooth data), in the same increments over v0:
//   60 (plus - v0)  = 11a - 2b + 24c - 3d,
//   60 (minus - v0) = 3b - 24a - 11c + 2d.
template <class T>
__device__ __forceinline__ void linear5_pair(T vm2, T vm1, T v0, T vp1, T vp2, T &plus, T &minus)
{
    const T b = vm1 - vm2, a = v0 - vm1, c = vp1 - v0, d = vp2 - vp1;
    const T k = T(1.0 / 60.0);
    plus = fmaT(fmaT(T(11), a, fmaT(T(24), c, fmaT(T(-2), b, T(-3) * d))), k, v0);
    minus = fmaT(fmaT(T(-24), a, fmaT(T(-11), c, fmaT(T(3), b, T(2) * d))), k, v0);
}

// The contact speed s* of the HLLC solver from the two sides' values.
// FP64 for both storage types: numerator and denominator cancel at material
// interfaces (equal pressures, opposite wave speeds).
template <class T>
__device__ __forceinline__ T contact_speed(T pL, T pR, T mL, T mR, T uL, T uR)
{
    if constexpr (std::is_same<T, double>::value) {
        return (pR - pL + mL * uL - mR * uR) * rcp(mL - mR);
    } else {
        const double num = double(pR) - double(pL) + double(mL) * double(uL) - double(mR) * double(uR);
        // rounded to float: the estimate of the reciprocal (about 24 bits) suffices
        return T(num * __builtin_amdgcn_rcp(double(mL) - double(mR)));
    }
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
template <int NDIM, int DIR, class T>
__device__ __forceinline__ bool hllc(const Grid &g, const T *wL, const T *wR, T *F, T &uf)
{
    constexpr int NV = 4 + NDIM, E = 2 + NDIM, A = 3 + NDIM;
    const T rhoL = wL[0] + wL[1], rhoR = wR[0] + wR[1];
    const T uL = wL[2 + DIR], uR = wR[2 + DIR];
    const T pL = wL[E], pR = wR[E];
    T GL, PL, GR, PR;
    mixture<T>(g, wL[A], GL, PL);
    mixture<T>(g, wR[A], GR, PR);
    const T c2L = sound2<T>(GL, PL, rhoL, pL), c2R = sound2<T>(GR, PR, rhoR, pR);
    const bool bad = nonphysical<T>(rhoL, c2L) || nonphysical<T>(rhoR, c2R);
    const T cL = sqrtT(c2L), cR = sqrtT(c2R);
    const T sL = fminT(uL - cL, uR - cR);
    const T sR = fmaxT(uL + cL, uR + cR);
    const T mL = rhoL * (sL - uL), mR = rhoR * (sR - uR);
    const T sS = contact_speed<T>(pL, pR, mL, mR, uL, uR);

    const bool super_L = sL >= T(0), super_R = sR <= T(0);
    const bool useL = super_L || (!super_R && sS >= T(0));
    const bool star = !super_L && !super_R;

    // the side whose state (plain or starred) is the fan at x/t = 0
    T w[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) w[v] = useL ? wL[v] : wR[v];
    const T rho = useL ? rhoL : rhoR;
    const T Gam = useL ? GL : GR, Pi = useL ? PL : PR;
    const T sK = useL ? sL : sR;
    const T un = w[2 + DIR], p = w[E];
    T u2 = T(0);
#pragma unroll
    for (int m = 0; m < NDIM; m++) u2 += w[2 + m] * w[2 + m];
    const T En = Gam * p + Pi + T(0.5) * rho * u2;

    // physical flux of that side
    const T mn = rho * un;   // normal mass flux
    F[0] = w[0] * un;
    F[1] = w[1] * un;
#pragma unroll
    for (int m = 0; m < NDIM; m++) F[2 + m] = (m == DIR) ? fmaT(mn, un, p) : mn * w[2 + m];
    F[E] = (En + p) * un;

    // star correction s_K (q*_K - q_K), with xi - 1 = (s* - u)/(s_K - s*)
    const T ism = rcp(sK - sS);
    const T xim1 = (sS - un) * ism;
    const T xi = (sK - un) * ism;
    T dq[NV - 1];
    const T xr = xim1 * rho;
    dq[0] = xim1 * w[0];
    dq[1] = xim1 * w[1];
#pragma unroll
    for (int m = 0; m < NDIM; m++) dq[2 + m] = (m == DIR) ? rho * fmaT(xi, sS, -un) : xr * w[2 + m];
    // xi (s* - u)(rho s* + p/(s_K - u)) = (s* - u)(xi rho s* + p/(s_K - s*))
    dq[E] = xim1 * En + (sS - un) * fmaT(xi * rho, sS, p * ism);
#pragma unroll
    for (int v = 0; v < NV - 1; v++) F[v] = star ? F[v] + sK * dq[v] : F[v];

    uf = star ? sS : un;
    F[A] = w[A] * uf;
    return bad;
}

}  // namespace mfc
