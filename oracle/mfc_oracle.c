/*
 * Plain, slow, FP64 CPU oracle for the finite-volume right-hand side of the
 * two-fluid five-equation diffuse-interface model with stiffened-gas
 * equations of state, as the paper states it:
 *
 *   - governing equations: Sec. 2.1 (two partial densities, mixture momentum,
 *     total energy, volume-fraction advection), in the Allaire form where the
 *     K div(u) term of the Kapila model is dropped;
 *   - stiffened-gas EOS: Sec. 2.1, eq. (soe), applied per fluid and mixed
 *     with volume-fraction weights (the printed equation omits the kinetic
 *     energy; total energy here is internal plus kinetic);
 *   - semi-discrete finite-volume form: Sec. 3.1, eqs. (fvm) and (fvmdis),
 *     with the face-velocity divergence that follows (fvmdis);
 *   - WENO5-JS reconstruction of primitive variables: Sec. 3.2 and the WENO5
 *     listing of Sec. 4.2 (divided differences, candidate polynomials,
 *     smoothness indicators, nonlinear weights), uniform-grid Jiang-Shu
 *     coefficients;
 *   - HLLC approximate Riemann solver: Sec. 3.2.1 (three waves s_L, s*, s_R,
 *     four-case state and flux, s* equal to the contact velocity u*);
 *   - boundary buffers of WENO width: Sec. 3.3 (extrapolation or periodic);
 *   - TVD (SSP) third-order Runge-Kutta: Sec. 3.4;
 *   - CFL-limited time step: Sec. 1.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU path is
 * checked against.  It shares no code, header, table or constant with the GPU
 * library and must never be linked into it.  Only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark load it.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fast-math): every
 * operation below is an IEEE double operation in source order.
 *
 * State layout (shared with the GPU path by specification, not by code):
 * q[v][z][y][x], x fastest, 3 ghost cells per side on active dimensions and
 * none on inactive ones.  nvar = 4 + ndim, ordered
 *   [alpha1*rho1, alpha2*rho2, rho*u_1 .. rho*u_ndim, rho*E, alpha1].
 * The primitive vector has the same ordering with velocities in place of
 * momenta and pressure in place of total energy:
 *   [alpha1*rho1, alpha2*rho2, u_1 .. u_ndim, p, alpha1].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_OK 0
#define ORA_E_ARG (-1)
#define ORA_E_NOMEM (-2)
#define ORA_E_NONPHYSICAL (-4)

#define NG 3   /* ghost layers per side: half the WENO5 stencil plus one */
#define MAXV 7 /* 4 + ndim with ndim <= 3 */

typedef struct {
    int ndim;           /* 1, 2 or 3                                     */
    int n[3];           /* interior cells per dimension (1 if inactive)   */
    double dx[3];       /* uniform cell width per active dimension        */
    double gamma[2];    /* stiffened-gas gamma of fluids 1 and 2          */
    double pi_inf[2];   /* stiffened-gas pi_infinity of fluids 1 and 2    */
    int bc[6];          /* x-,x+,y-,y+,z-,z+: 0 extrapolation, 1 periodic,
                           2 characteristic non-reflecting (ghosts filled
                           as for extrapolation; the boundary cell's normal
                           terms take the characteristic form)            */
    double weno_eps;    /* WENO5-JS epsilon                               */
    int recon;          /* 0 WENO5 everywhere; 1 the linear fifth-order
                           stencil everywhere; 2 per (cell, direction) as
                           `smooth` says; 3 WENO3 everywhere; 4 first
                           order (cell values) everywhere                  */
    const unsigned char *smooth; /* recon 2: smooth[d * padded cells + c]
                           != 0 selects the linear stencil for every
                           variable of padded cell c along direction d    */
    int model;          /* 0 Allaire (alpha1 equation without K div(u));
                           1 Kapila (with K div(u))                       */
    const double *faces[3]; /* non-uniform grid: faces[d][0 .. n_d] are the
                           n_d + 1 interior face coordinates along d (NULL:
                           uniform cells of width dx[d])                   */
} ora_grid;

int ora_nvar(int ndim) { return 4 + ndim; }

static int64_t pad(const ora_grid *g, int d) { return d < g->ndim ? g->n[d] + 2 * NG : 1; }
static int off(const ora_grid *g, int d) { return d < g->ndim ? NG : 0; }

/* Linear index of variable v at interior-relative cell (i, j, k); negative
 * or >= n indices address ghost cells. */
static int64_t at(const ora_grid *g, int v, int i, int j, int k)
{
    return (((int64_t)v * pad(g, 2) + (k + off(g, 2))) * pad(g, 1) + (j + off(g, 1))) * pad(g, 0)
           + (i + off(g, 0));
}

int64_t ora_padded_cells(const ora_grid *g) { return pad(g, 0) * pad(g, 1) * pad(g, 2); }

/* Width of cell i (-NG <= i < n + NG) along dimension d.  Ghost cells take
 * the width of the interior cell whose value the ghost fill copies there:
 * mirrored for extrapolation (cell -1 <- 0, -2 <- 1, n <- n-1, ...),
 * one period away for periodic boundaries. */
double ora_cell_width(const ora_grid *g, int d, int i)
{
    if (!g->faces[d]) return g->dx[d];
    int n = g->n[d];
    if (i < 0) i = g->bc[2 * d] == 1 ? i + n : -1 - i;
    else if (i >= n) i = g->bc[2 * d + 1] == 1 ? i - n : 2 * n - 1 - i;
    return g->faces[d][i + 1] - g->faces[d][i];
}

/* ---------------------------------------------------------------------- */
/* Equation of state (Sec. 2.1, eq. soe)                                    */
/* ---------------------------------------------------------------------- */

/* Each fluid obeys rho_k e_k = p/(gamma_k - 1) + gamma_k pi_k/(gamma_k - 1).
 * With pressure equilibrium the mixture internal energy is
 * rho e = Gamma p + Pi, with Gamma = sum_k alpha_k/(gamma_k - 1) and
 * Pi = sum_k alpha_k gamma_k pi_k/(gamma_k - 1), alpha2 = 1 - alpha1. */
void ora_mixture(const ora_grid *g, double alpha1, double *Gamma, double *Pi)
{
    double alpha2 = 1.0 - alpha1;
    double g1 = 1.0 / (g->gamma[0] - 1.0);
    double g2 = 1.0 / (g->gamma[1] - 1.0);
    double h1 = g->gamma[0] * g->pi_inf[0] / (g->gamma[0] - 1.0);
    double h2 = g->gamma[1] * g->pi_inf[1] / (g->gamma[1] - 1.0);
    *Gamma = alpha1 * g1 + alpha2 * g2;
    *Pi = alpha1 * h1 + alpha2 * h2;
}

/* Frozen sound speed squared of the mixture: the mixture is itself a
 * stiffened gas with gamma_m = 1 + 1/Gamma and pi_m = Pi/(Gamma + 1), so
 * c^2 = gamma_m (p + pi_m)/rho = ((Gamma + 1) p + Pi)/(Gamma rho). */
double ora_sound_speed2(const ora_grid *g, double rho, double p, double alpha1)
{
    double Gamma, Pi;
    ora_mixture(g, alpha1, &Gamma, &Pi);
    return ((Gamma + 1.0) * p + Pi) / (Gamma * rho);
}

/* K of the Kapila model's volume-fraction equation (Sec. 2.1):
 *   K = (rho2 c2^2 - rho1 c1^2) / (rho2 c2^2/alpha2 + rho1 c1^2/alpha1),
 * (the paper prints rho1 c2^2 in the second denominator term; the model's
 * derivation, equal phase pressure rates under compression, needs
 * rho1 c1^2), with the phase densities rho_k = (alpha_k rho_k)/alpha_k and
 * the stiffened-gas phase sound speeds c_k^2 = gamma_k (p + pi_k)/rho_k at
 * the common pressure p.  w is one cell's primitive vector.  K is 0 where a
 * volume fraction is not positive (the pure-phase limit). */
double ora_kapila_K(const ora_grid *g, const double *w)
{
    int nv = ora_nvar(g->ndim);
    double alpha1 = w[nv - 1], alpha2 = 1.0 - alpha1, p = w[nv - 2];
    if (!(alpha1 > 0.0) || !(alpha2 > 0.0))
        return 0.0;
    double rho1 = w[0] / alpha1, rho2 = w[1] / alpha2;
    double c1sq = g->gamma[0] * (p + g->pi_inf[0]) / rho1;
    double c2sq = g->gamma[1] * (p + g->pi_inf[1]) / rho2;
    double z1 = rho1 * c1sq, z2 = rho2 * c2sq;
    return (z2 - z1) / (z2 / alpha2 + z1 / alpha1);
}

static int nonphysical(double rho, double c2)
{
    return !(rho > 0.0) || !(c2 > 0.0) || !isfinite(rho) || !isfinite(c2);
}

/* Primitive -> conservative for one cell (nv values each). */
void ora_prim_to_cons(const ora_grid *g, const double *w, double *q)
{
    int nd = g->ndim, nv = 4 + nd;
    double rho = w[0] + w[1];
    double Gamma, Pi, u2 = 0.0;
    ora_mixture(g, w[nv - 1], &Gamma, &Pi);
    q[0] = w[0];
    q[1] = w[1];
    for (int m = 0; m < nd; m++) {
        q[2 + m] = rho * w[2 + m];
        u2 += w[2 + m] * w[2 + m];
    }
    q[2 + nd] = Gamma * w[2 + nd] + Pi + 0.5 * rho * u2;
    q[nv - 1] = w[nv - 1];
}

/* Conservative -> primitive for one cell.  Returns ORA_E_NONPHYSICAL when
 * rho <= 0, c^2 <= 0 or a value is not finite (the values are still
 * written). */
int ora_cons_to_prim(const ora_grid *g, const double *q, double *w)
{
    int nd = g->ndim, nv = 4 + nd;
    double rho = q[0] + q[1];
    double Gamma, Pi, ke = 0.0;
    ora_mixture(g, q[nv - 1], &Gamma, &Pi);
    w[0] = q[0];
    w[1] = q[1];
    for (int m = 0; m < nd; m++) {
        w[2 + m] = q[2 + m] / rho;
        ke += 0.5 * q[2 + m] * w[2 + m];
    }
    w[2 + nd] = (q[2 + nd] - ke - Pi) / Gamma;
    w[nv - 1] = q[nv - 1];
    double c2 = ((Gamma + 1.0) * w[2 + nd] + Pi) / (Gamma * rho);
    return nonphysical(rho, c2) ? ORA_E_NONPHYSICAL : ORA_OK;
}

/* ---------------------------------------------------------------------- */
/* WENO5-JS reconstruction (Sec. 3.2; listing of Sec. 4.2)                   */
/* ---------------------------------------------------------------------- */

/* From the five cell averages s[0..4] = v_{i-2} .. v_{i+2} of cell i:
 *   *at_plus  = reconstructed value at face x_{i+1/2} (left state there),
 *   *at_minus = reconstructed value at face x_{i-1/2} (right state there),
 *   *maxdev   = max over r and both faces of |omega_r - d_r| (may be NULL).
 *
 * As in the listing, the candidate values are written with the divided
 * differences dvd(q) = v_{i+q+1} - v_{i+q}, q = -2..1, and the smoothness
 * indicators are quadratic forms in them.  Coefficients are the uniform-grid
 * Jiang-Shu values (three candidate stencils r = 0, 1, 2, ideal weights
 * 1/10, 6/10, 3/10 at x_{i+1/2} and their mirror 3/10, 6/10, 1/10 at
 * x_{i-1/2}); the nonlinear weights are alpha_r = d_r/(eps + beta_r)^2,
 * omega_r = alpha_r/sum(alpha). */
void ora_weno5(const double *s, double eps, double *at_plus, double *at_minus, double *maxdev)
{
    double vi = s[2];
    double dm2 = s[1] - s[0]; /* dvd(-2) = v_{i-1} - v_{i-2} */
    double dm1 = s[2] - s[1]; /* dvd(-1) = v_i     - v_{i-1} */
    double d0 = s[3] - s[2];  /* dvd(0)  = v_{i+1} - v_i     */
    double d1 = s[4] - s[3];  /* dvd(1)  = v_{i+2} - v_{i+1} */

    /* candidate values at x_{i+1/2} */
    double pp[3], pm[3], beta[3];
    pp[0] = vi + (5.0 / 6.0) * dm1 - (1.0 / 3.0) * dm2;
    pp[1] = vi + (1.0 / 3.0) * d0 + (1.0 / 6.0) * dm1;
    pp[2] = vi + (2.0 / 3.0) * d0 - (1.0 / 6.0) * d1;
    /* candidate values at x_{i-1/2} */
    pm[0] = vi - (2.0 / 3.0) * dm1 + (1.0 / 6.0) * dm2;
    pm[1] = vi - (1.0 / 3.0) * dm1 - (1.0 / 6.0) * d0;
    pm[2] = vi - (5.0 / 6.0) * d0 + (1.0 / 3.0) * d1;

    /* smoothness indicators: 13/12 (second difference)^2 + 1/4 (one-sided
     * first-derivative estimate)^2, written in divided differences */
    beta[0] = (10.0 / 3.0) * dm1 * dm1 - (11.0 / 3.0) * dm1 * dm2 + (4.0 / 3.0) * dm2 * dm2;
    beta[1] = (4.0 / 3.0) * d0 * d0 - (5.0 / 3.0) * d0 * dm1 + (4.0 / 3.0) * dm1 * dm1;
    beta[2] = (10.0 / 3.0) * d0 * d0 - (11.0 / 3.0) * d0 * d1 + (4.0 / 3.0) * d1 * d1;

    static const double dplus[3] = {0.1, 0.6, 0.3};
    static const double dminus[3] = {0.3, 0.6, 0.1};
    double ap[3], am[3], sp = 0.0, sm = 0.0;
    for (int r = 0; r < 3; r++) {
        double den = (eps + beta[r]) * (eps + beta[r]);
        ap[r] = dplus[r] / den;
        am[r] = dminus[r] / den;
        sp += ap[r];
        sm += am[r];
    }
    double vp = 0.0, vm = 0.0, dev = 0.0;
    for (int r = 0; r < 3; r++) {
        double wp = ap[r] / sp, wm = am[r] / sm;
        vp += wp * pp[r];
        vm += wm * pm[r];
        if (fabs(wp - dplus[r]) > dev) dev = fabs(wp - dplus[r]);
        if (fabs(wm - dminus[r]) > dev) dev = fabs(wm - dminus[r]);
    }
    *at_plus = vp;
    *at_minus = vm;
    if (maxdev) *maxdev = dev;
}

/* WENO5 on non-uniform cells (Sec. 3.2 with cell widths Delta x_i).  For
 * cell i the candidate polynomial p_r (degree 2) is the one whose averages
 * over the three cells of stencil r ({i-2+r .. i+r}) equal the data; the
 * face values are p_r(x_{i+1/2}) and p_r(x_{i-1/2}); the smoothness
 * indicator is beta_r = sum_{l=1,2} Delta x_i^{2l-1} int_{I_i} (d^l p_r/dx^l)^2,
 * which for p_r = a0 + a1 xi + a2 xi^2, xi = (x - x_i)/Delta x_i, is
 * a1^2 + (13/3) a2^2; the ideal weights d_r are those for which
 * sum_r d_r p_r(face) equals the face value of the degree-4 polynomial
 * whose averages over all five cells equal the data.  Everything is linear
 * in the data: the coefficients below are computed once per cell from the
 * widths by solving the cell-average systems in xi. */
typedef struct {
    double plus[3][3], minus[3][3]; /* p_r(x_{i+1/2}), p_r(x_{i-1/2}) on stencil r's cells */
    double a1[3][3], a2[3][3];      /* a1, a2 of p_r on stencil r's cells                */
    double dplus[3], dminus[3];     /* ideal weights                                    */
} ora_weno_coef;

/* Solve the m x m system A x = b (m <= 5) by Gaussian elimination with
 * partial pivoting; A and b are overwritten. */
static void solve_small(int m, double A[5][5], double *b, double *x)
{
    for (int c = 0; c < m; c++) {
        int piv = c;
        for (int r = c + 1; r < m; r++)
            if (fabs(A[r][c]) > fabs(A[piv][c])) piv = r;
        for (int k = 0; k < m; k++) {
            double t = A[c][k]; A[c][k] = A[piv][k]; A[piv][k] = t;
        }
        double t = b[c]; b[c] = b[piv]; b[piv] = t;
        for (int r = c + 1; r < m; r++) {
            double f = A[r][c] / A[c][c];
            for (int k = c; k < m; k++) A[r][k] -= f * A[c][k];
            b[r] -= f * b[c];
        }
    }
    for (int r = m - 1; r >= 0; r--) {
        double acc = b[r];
        for (int k = r + 1; k < m; k++) acc -= A[r][k] * x[k];
        x[r] = acc / A[r][r];
    }
}

/* Polynomial coefficients (in xi about cell i, scaled by h_i) of the degree
 * m-1 polynomial whose averages over the m consecutive cells starting at
 * cell offset `first` (relative to i) equal e_j: coef[j][k] is the xi^k
 * coefficient for unit data on the j-th of those cells.  w[t] is the width
 * of cell i - 2 + t, t = 0..4. */
static void average_inverse(const double *w, int first, int m, double coef[5][5])
{
    /* cell edges in xi: cell i spans [-1/2, 1/2] */
    double edge[6];
    edge[2] = -0.5;
    for (int t = 2; t < 5; t++) edge[t + 1] = edge[t] + w[t] / w[2];
    for (int t = 2; t > 0; t--) edge[t - 1] = edge[t] - w[t - 1] / w[2];
    for (int j = 0; j < m; j++) {
        double A[5][5], b[5], x[5];
        for (int r = 0; r < m; r++) {
            int t = first + 2 + r;          /* cell index within w[] */
            double lo = edge[t], hi = edge[t + 1];
            for (int k = 0; k < m; k++)
                A[r][k] = (pow(hi, k + 1) - pow(lo, k + 1)) / ((k + 1) * (hi - lo));
            b[r] = r == j ? 1.0 : 0.0;
        }
        solve_small(m, A, b, x);
        for (int k = 0; k < m; k++) coef[j][k] = x[k];
    }
}

static double poly_at(const double *c, int m, double xi)
{
    double v = 0.0;
    for (int k = m - 1; k >= 0; k--) v = v * xi + c[k];
    return v;
}

/* Coefficients for cell i from the widths w[0..4] of cells i-2 .. i+2. */
void ora_weno_coef_nonuniform(const double *w, ora_weno_coef *cf)
{
    double q5[5][5], q3[5][5];
    average_inverse(w, -2, 5, q5);
    double qplus[5], qminus[5];
    for (int j = 0; j < 5; j++) {
        qplus[j] = poly_at(q5[j], 5, 0.5);
        qminus[j] = poly_at(q5[j], 5, -0.5);
    }
    for (int r = 0; r < 3; r++) {
        average_inverse(w, r - 2, 3, q3);
        for (int j = 0; j < 3; j++) {
            cf->plus[r][j] = poly_at(q3[j], 3, 0.5);
            cf->minus[r][j] = poly_at(q3[j], 3, -0.5);
            cf->a1[r][j] = q3[j][1];
            cf->a2[r][j] = q3[j][2];
        }
    }
    /* sum_r d_r p_r = q on every datum: the outermost cells appear in one
     * stencil each (r = 0 holds cell i-2, r = 2 holds cell i+2), and the
     * weights sum to one */
    cf->dplus[0] = qplus[0] / cf->plus[0][0];
    cf->dplus[2] = qplus[4] / cf->plus[2][2];
    cf->dplus[1] = 1.0 - cf->dplus[0] - cf->dplus[2];
    cf->dminus[0] = qminus[0] / cf->minus[0][0];
    cf->dminus[2] = qminus[4] / cf->minus[2][2];
    cf->dminus[1] = 1.0 - cf->dminus[0] - cf->dminus[2];
}

/* Smoothness indicator of stencil r for the values s[0..4]. */
static double beta_nonuniform(const ora_weno_coef *cf, int r, const double *s)
{
    double a1 = 0.0, a2 = 0.0;
    for (int j = 0; j < 3; j++) {
        a1 += cf->a1[r][j] * s[r + j];
        a2 += cf->a2[r][j] * s[r + j];
    }
    return a1 * a1 + (13.0 / 3.0) * a2 * a2;
}

/* Non-uniform WENO5 of the five values s[0..4] (cells i-2 .. i+2). */
void ora_weno5_nonuniform(const ora_weno_coef *cf, const double *s, double eps, double *at_plus,
                          double *at_minus)
{
    double ap[3], am[3], pp[3], pm[3], sp = 0.0, sm = 0.0;
    for (int r = 0; r < 3; r++) {
        pp[r] = pm[r] = 0.0;
        for (int j = 0; j < 3; j++) {
            pp[r] += cf->plus[r][j] * s[r + j];
            pm[r] += cf->minus[r][j] * s[r + j];
        }
        double beta = beta_nonuniform(cf, r, s);
        double den = (eps + beta) * (eps + beta);
        ap[r] = cf->dplus[r] / den;
        am[r] = cf->dminus[r] / den;
        sp += ap[r];
        sm += am[r];
    }
    double vp = 0.0, vm = 0.0;
    for (int r = 0; r < 3; r++) {
        vp += ap[r] / sp * pp[r];
        vm += am[r] / sm * pm[r];
    }
    *at_plus = vp;
    *at_minus = vm;
}

/* One cell's non-uniform WENO5 from the widths w[0..4] and values s[0..4]
 * of cells i-2 .. i+2, and its three smoothness indicators (test access). */
void ora_weno5_nonuniform_cell(const double *w, const double *s, double eps, double *at_plus, double *at_minus)
{
    ora_weno_coef cf;
    ora_weno_coef_nonuniform(w, &cf);
    ora_weno5_nonuniform(&cf, s, eps, at_plus, at_minus);
}

void ora_weno5_nonuniform_betas(const double *w, const double *s, double *beta)
{
    ora_weno_coef cf;
    ora_weno_coef_nonuniform(w, &cf);
    for (int r = 0; r < 3; r++) beta[r] = beta_nonuniform(&cf, r, s);
}

/* WENO3-JS reconstruction (Sec. 3.2, the third-order variant: k = 2
 * candidate stencils).  From s[0..2] = v_{i-1}, v_i, v_{i+1}:
 *   candidates at x_{i+1/2}: (-v_{i-1} + 3 v_i)/2 on {i-1, i} and
 *   (v_i + v_{i+1})/2 on {i, i+1}, ideal weights 1/3 and 2/3;
 *   at x_{i-1/2} the mirror: (v_{i-1} + v_i)/2 and (3 v_i - v_{i+1})/2,
 *   ideal weights 2/3 and 1/3;
 *   smoothness indicators beta_0 = (v_i - v_{i-1})^2, beta_1 = (v_{i+1} - v_i)^2,
 *   nonlinear weights alpha_r = d_r/(eps + beta_r)^2, omega_r = alpha_r/sum(alpha). */
void ora_weno3(const double *s, double eps, double *at_plus, double *at_minus)
{
    double pp[2], pm[2], beta[2];
    pp[0] = (-s[0] + 3.0 * s[1]) / 2.0;
    pp[1] = (s[1] + s[2]) / 2.0;
    pm[0] = (s[0] + s[1]) / 2.0;
    pm[1] = (3.0 * s[1] - s[2]) / 2.0;
    beta[0] = (s[1] - s[0]) * (s[1] - s[0]);
    beta[1] = (s[2] - s[1]) * (s[2] - s[1]);
    static const double dplus[2] = {1.0 / 3.0, 2.0 / 3.0};
    static const double dminus[2] = {2.0 / 3.0, 1.0 / 3.0};
    double ap[2], am[2], sp = 0.0, sm = 0.0;
    for (int r = 0; r < 2; r++) {
        double den = (eps + beta[r]) * (eps + beta[r]);
        ap[r] = dplus[r] / den;
        am[r] = dminus[r] / den;
        sp += ap[r];
        sm += am[r];
    }
    *at_plus = (ap[0] * pp[0] + ap[1] * pp[1]) / sp;
    *at_minus = (am[0] * pm[0] + am[1] * pm[1]) / sm;
}

/* The linear fifth-order upwind reconstruction: the same candidates with
 * the ideal weights, i.e. the limit of WENO5 on smooth data. */
void ora_linear5(const double *s, double *at_plus, double *at_minus)
{
    *at_plus = (2.0 * s[0] - 13.0 * s[1] + 47.0 * s[2] + 27.0 * s[3] - 3.0 * s[4]) / 60.0;
    *at_minus = (-3.0 * s[0] + 27.0 * s[1] + 47.0 * s[2] - 13.0 * s[3] + 2.0 * s[4]) / 60.0;
}

/* ---------------------------------------------------------------------- */
/* HLLC approximate Riemann solver (Sec. 3.2.1)                            */
/* ---------------------------------------------------------------------- */

/* Physical flux normal to dimension dir of primitive state w with
 * conservative state q: F = (a1r1 u_n, a2r2 u_n, rho u u_n + p e_n,
 * (rhoE + p) u_n); the alpha1 slot is left to the caller. */
static void physical_flux(const ora_grid *g, int dir, const double *w, const double *q, double *F)
{
    int nd = g->ndim;
    double un = w[2 + dir], p = w[2 + nd];
    F[0] = q[0] * un;
    F[1] = q[1] * un;
    for (int m = 0; m < nd; m++) F[2 + m] = q[2 + m] * un + (m == dir ? p : 0.0);
    F[2 + nd] = (q[2 + nd] + p) * un;
}

/* Flux through a face normal to dimension dir between primitive states wL
 * (left side) and wR (right side).  On return F[0 .. nv-2] hold the HLLC
 * flux of the conserved rows, F[nv-1] holds alpha1_upwind * u_face (the
 * conservative part of the alpha1 advection), and *uface holds the face
 * normal velocity used by the div(u) term of eq. (fvmdis).
 *
 * Wave speeds: direct (Davis) estimates s_L = min(uL - cL, uR - cR),
 * s_R = max(uL + cL, uR + cR).  Contact speed: Toro's expression that
 * follows from equal normal velocity and pressure on both sides of the
 * contact, s* = u*.  Star states: q*_K = xi_K (a1r1_K, a2r2_K, rho_K s* e_n
 * + rho_K u_t,K, rhoE_K + (s* - u_K)(rho_K s* + p_K/(s_K - u_K))) with
 * xi_K = (s_K - u_K)/(s_K - s*).  Face velocity and face volume fraction:
 * those of the Riemann fan at x/t = 0.  The four regions L, L*, R*, R are
 * chosen as in the paper's case table (s_L >= 0: L; s_L < 0 <= s*: L*;
 * s* < 0 < s_R: R*; s_R <= 0: R); the normal velocity is u_L, s*, s* or u_R,
 * and alpha1 is alpha1_L in L and L* and alpha1_R in R* and R, since the
 * volume fraction jumps only across the contact. */
int ora_hllc(const ora_grid *g, int dir, const double *wL, const double *wR, double *F, double *uface)
{
    int nd = g->ndim, nv = 4 + nd, E = 2 + nd;
    double qL[MAXV], qR[MAXV], FL[MAXV], FR[MAXV];
    ora_prim_to_cons(g, wL, qL);
    ora_prim_to_cons(g, wR, qR);
    physical_flux(g, dir, wL, qL, FL);
    physical_flux(g, dir, wR, qR, FR);

    double rhoL = wL[0] + wL[1], rhoR = wR[0] + wR[1];
    double uL = wL[2 + dir], uR = wR[2 + dir];
    double pL = wL[E], pR = wR[E];
    double c2L = ora_sound_speed2(g, rhoL, pL, wL[nv - 1]);
    double c2R = ora_sound_speed2(g, rhoR, pR, wR[nv - 1]);
    int bad = nonphysical(rhoL, c2L) || nonphysical(rhoR, c2R);
    double cL = sqrt(c2L), cR = sqrt(c2R);

    double sL = fmin(uL - cL, uR - cR);
    double sR = fmax(uL + cL, uR + cR);
    double sS = (pR - pL + rhoL * uL * (sL - uL) - rhoR * uR * (sR - uR))
                / (rhoL * (sL - uL) - rhoR * (sR - uR));

    double alpha_face;
    if (sL >= 0.0) {
        for (int v = 0; v < nv - 1; v++) F[v] = FL[v];
        *uface = uL;
        alpha_face = wL[nv - 1];
    } else if (sR <= 0.0) {
        for (int v = 0; v < nv - 1; v++) F[v] = FR[v];
        *uface = uR;
        alpha_face = wR[nv - 1];
    } else {
        /* subsonic: the face lies between s_L and s_R */
        const double *w = sS >= 0.0 ? wL : wR;
        const double *q = sS >= 0.0 ? qL : qR;
        const double *Fk = sS >= 0.0 ? FL : FR;
        double sK = sS >= 0.0 ? sL : sR;
        double rho = w[0] + w[1], un = w[2 + dir], p = w[E];
        double xi = (sK - un) / (sK - sS);
        double qs[MAXV];
        qs[0] = xi * q[0];
        qs[1] = xi * q[1];
        for (int m = 0; m < nd; m++) qs[2 + m] = xi * (m == dir ? rho * sS : rho * w[2 + m]);
        qs[E] = xi * (q[E] + (sS - un) * (rho * sS + p / (sK - un)));
        for (int v = 0; v < nv - 1; v++) F[v] = Fk[v] + sK * (qs[v] - q[v]);
        *uface = sS;
        alpha_face = w[nv - 1];
    }
    F[nv - 1] = alpha_face * (*uface);
    return bad ? ORA_E_NONPHYSICAL : ORA_OK;
}

/* ---------------------------------------------------------------------- */
/* Boundary buffers (Sec. 3.3)                                             */
/* ---------------------------------------------------------------------- */

/* Fill NG ghost layers on each side of every active dimension, for the
 * face slabs only (cells whose other coordinates are interior); edges and
 * corners are never read by the dimension-by-dimension sweeps.
 * bc 0 (extrapolation): copy the adjacent interior cell.
 * bc 1 (periodic): copy the cell one period away. */
int ora_fill_ghosts(const ora_grid *g, double *q)
{
    int nv = 4 + g->ndim;
    for (int d = 0; d < g->ndim; d++) {
        int n = g->n[d];
        int na = d == 0 ? g->n[1] : g->n[0];   /* the two other dimensions */
        int nb = d == 2 ? g->n[1] : g->n[2];
        for (int v = 0; v < nv; v++)
            for (int b = 0; b < nb; b++)
                for (int a = 0; a < na; a++)
                    for (int l = 1; l <= NG; l++) {
                        int lo = -l, hi = n - 1 + l;
                        int slo = g->bc[2 * d] == 1 ? n - l : 0;
                        int shi = g->bc[2 * d + 1] == 1 ? l - 1 : n - 1;
                        int c[3], s[3];
                        /* place (a, b) on the two non-d dimensions */
                        int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
                        c[o1] = a; c[o2] = b; s[o1] = a; s[o2] = b;
                        c[d] = lo; s[d] = slo;
                        q[at(g, v, c[0], c[1], c[2])] = q[at(g, v, s[0], s[1], s[2])];
                        c[d] = hi; s[d] = shi;
                        q[at(g, v, c[0], c[1], c[2])] = q[at(g, v, s[0], s[1], s[2])];
                    }
    }
    return ORA_OK;
}

/* ---------------------------------------------------------------------- */
/* Characteristic boundary condition (Sec. 3.3)                             */
/* ---------------------------------------------------------------------- */

/* Characteristic-based, non-reflecting treatment of a boundary cell along
 * dimension d (the paper uses characteristic boundary conditions after
 * Thompson, time-dependent form).  In the primitive variables the terms
 * normal to the boundary are written with the wave amplitudes of the
 * one-dimensional system:
 *   L1 = (u - c)(p_x - rho c u_x),  L5 = (u + c)(p_x + rho c u_x),
 *   L_k = u ((alpha_k rho_k)_x - alpha_k rho_k p_x/(rho c^2))   (k = 1, 2),
 *   L_t = u (u_t)_x for each tangential velocity,  L_a = u (alpha1)_x,
 * with c the mixture sound speed and u the normal velocity; an amplitude
 * whose wave travels into the domain is set to zero (no incoming wave),
 * the others use the one-sided derivative dwdx of the caller.  Then
 *   p_t = -(L5 + L1)/2,  u_t = -(L5 - L1)/(2 rho c),
 *   (alpha_k rho_k)_t = -L_k - alpha_k rho_k (L5 + L1)/(2 rho c^2),
 *   (u_t)_t = -L_t,  (alpha1)_t = -L_a,
 * converted to the conservative rows through rho E = Gamma(alpha1) p +
 * Pi(alpha1) + rho |u|^2/2.  side 0: boundary at the low end (the domain
 * lies at larger coordinates), side 1: at the high end.  dqdt receives the
 * normal-direction time derivative of the conservative rows. */
void ora_cbc_cell(const ora_grid *g, int d, int side, const double *w, const double *dwdx, double *dqdt)
{
    int nd = g->ndim, nv = 4 + nd;
    double rho = w[0] + w[1], p = w[nv - 2], alpha1 = w[nv - 1], un = w[2 + d];
    double c2 = ora_sound_speed2(g, rho, p, alpha1), c = sqrt(c2);
    double lam1 = un - c, lam5 = un + c, lamm = un;
    #define ENTERS(l) (side == 0 ? (l) > 0.0 : (l) < 0.0)
    double dp = dwdx[nv - 2], du = dwdx[2 + d];
    double L1 = ENTERS(lam1) ? 0.0 : lam1 * (dp - rho * c * du);
    double L5 = ENTERS(lam5) ? 0.0 : lam5 * (dp + rho * c * du);
    double Lk[2], Lt[3], La;
    for (int k = 0; k < 2; k++) Lk[k] = ENTERS(lamm) ? 0.0 : lamm * (dwdx[k] - w[k] / (rho * c2) * dp);
    for (int m = 0; m < nd; m++) Lt[m] = ENTERS(lamm) ? 0.0 : lamm * dwdx[2 + m];
    La = ENTERS(lamm) ? 0.0 : lamm * dwdx[nv - 1];
    #undef ENTERS
    /* primitive time derivatives */
    double pt = -0.5 * (L5 + L1);
    double ut[3];
    for (int m = 0; m < nd; m++) ut[m] = m == d ? -(L5 - L1) / (2.0 * rho * c) : -Lt[m];
    double rkt[2];
    for (int k = 0; k < 2; k++) rkt[k] = -Lk[k] - w[k] / (rho * c2) * 0.5 * (L5 + L1);
    double at = -La;
    /* conservative rows */
    double Gamma, Pi, G1, P1, G0, P0;
    ora_mixture(g, alpha1, &Gamma, &Pi);
    ora_mixture(g, 1.0, &G1, &P1);   /* Gamma and Pi are affine in alpha1: their */
    ora_mixture(g, 0.0, &G0, &P0);   /* derivatives are the pure-fluid differences */
    double rhot = rkt[0] + rkt[1], u2 = 0.0, uut = 0.0;
    dqdt[0] = rkt[0];
    dqdt[1] = rkt[1];
    for (int m = 0; m < nd; m++) {
        dqdt[2 + m] = w[2 + m] * rhot + rho * ut[m];
        u2 += w[2 + m] * w[2 + m];
        uut += w[2 + m] * ut[m];
    }
    dqdt[2 + nd] = Gamma * pt + ((G1 - G0) * p + (P1 - P0)) * at + 0.5 * u2 * rhot + rho * uut;
    dqdt[nv - 1] = at;
}

/* Coefficients c[0..2] of the second-order one-sided derivative along d at
 * the centre of the boundary cell of face `side` (0 low, 1 high), applied to
 * the values of that cell and of the next two cells into the domain: the
 * derivative at x0 of the quadratic through (x_t, f_t), t = 0, 1, 2, where
 * x_t are the centres of cells b, b + s, b + 2s (b = 0, s = +1 on the low
 * face; b = n - 1, s = -1 on the high face).  On the non-uniform cells of
 * the structured mesh (Sec. 4.1) the centres come from the face
 * coordinates; on uniform cells this is s (-3, 4, -1) / (2 dx). */
void ora_one_sided_coef(const ora_grid *g, int d, int side, double c[3])
{
    int n = g->n[d], s = side == 0 ? 1 : -1, b = side == 0 ? 0 : n - 1;
    double x[3];
    for (int t = 0; t < 3; t++) {
        int i = b + s * t;
        x[t] = g->faces[d] ? 0.5 * (g->faces[d][i] + g->faces[d][i + 1]) : (i + 0.5) * g->dx[d];
    }
    c[0] = 1.0 / (x[0] - x[1]) + 1.0 / (x[0] - x[2]);
    c[1] = (x[0] - x[2]) / ((x[1] - x[0]) * (x[1] - x[2]));
    c[2] = (x[0] - x[1]) / ((x[2] - x[0]) * (x[2] - x[1]));
}

/* ---------------------------------------------------------------------- */
/* Right-hand side (Sec. 3.1, eq. fvmdis)                                   */
/* ---------------------------------------------------------------------- */

/* dq/dt on interior cells of q (ghost cells must already be filled):
 *   rows other than alpha1: sum_d (F_{-1/2} - F_{+1/2})/dx_d;
 *   alpha1 row: the same flux difference of alpha1 u plus
 *               alpha1_cell * div(u), div(u) = sum_d (u_{+1/2} - u_{-1/2})/dx_d,
 * i.e. eq. (fvm) with s = 0 and h = -alpha1 on the alpha1 row, which is
 * the Allaire model's u . grad(alpha1) = div(alpha1 u) - alpha1 div(u);
 * with model 1 (Kapila) the alpha1 row carries (alpha1 + K)_cell div(u),
 * i.e. h = -(alpha1 + K), from u . grad(alpha1) = K div(u).
 * Ghost entries of rhs are not written. */
/* Threads of the OpenMP build (1 in the plain build, where the pragmas
 * below are ignored).  Every parallel loop writes disjoint cells, so the
 * two builds give bitwise the same results. */
int ora_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int ora_rhs(const ora_grid *g, const double *q, double *rhs)
{
    int nd = g->ndim, nv = 4 + nd;
    int64_t ncell = ora_padded_cells(g);
    int nx = g->n[0], ny = g->n[1], nz = g->n[2];
    int status = ORA_OK;
    double *w = malloc(sizeof(double) * ncell * nv);
    double *divu = calloc(ncell, sizeof(double));
    int nmax = nx > ny ? nx : ny;
    if (nz > nmax) nmax = nz;
    if (!w || !divu) {
        free(w); free(divu);
        return ORA_E_NOMEM;
    }

    /* conservative -> primitive on every cell the sweeps read: interior
     * cells and the ghost face slabs (at most one coordinate outside) */
    int lo[3], hi[3];
    for (int d = 0; d < 3; d++) {
        lo[d] = d < nd ? -NG : 0;
        hi[d] = d < nd ? g->n[d] + NG : 1;
    }
    #pragma omp parallel for reduction(min : status) schedule(static)
    for (int k = lo[2]; k < hi[2]; k++)
        for (int j = lo[1]; j < hi[1]; j++)
            for (int i = lo[0]; i < hi[0]; i++) {
                int outside = (i < 0 || i >= nx) + (j < 0 || j >= ny) + (k < 0 || k >= nz);
                if (outside > 1) continue;
                double qc[MAXV], wc[MAXV];
                for (int v = 0; v < nv; v++) qc[v] = q[at(g, v, i, j, k)];
                if (ora_cons_to_prim(g, qc, wc) != ORA_OK) status = ORA_E_NONPHYSICAL;
                for (int v = 0; v < nv; v++) w[at(g, v, i, j, k)] = wc[v];
            }

    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++)
                for (int v = 0; v < nv; v++) rhs[at(g, v, i, j, k)] = 0.0;

    for (int d = 0; d < nd; d++) {
        int n = g->n[d];
        int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
        int n1 = o1 < nd ? g->n[o1] : 1, n2 = o2 < nd ? g->n[o2] : 1;
        /* non-uniform cells: WENO5 coefficients of every cell -1 .. n along d */
        ora_weno_coef *cf = NULL;
        if (g->faces[d]) {
            if (g->recon != 0 && g->recon != 4) {
                status = ORA_E_ARG;   /* non-uniform cells take WENO5 or first order */
                break;
            }
            cf = malloc(sizeof(ora_weno_coef) * (n + 2));
            if (!cf) {
                status = ORA_E_NOMEM;
                break;
            }
            for (int cell = -1; cell <= n; cell++) {
                double wd[5];
                for (int t = 0; t < 5; t++) wd[t] = ora_cell_width(g, d, cell - 2 + t);
                ora_weno_coef_nonuniform(wd, &cf[cell + 1]);
            }
        }
        int pencil_status = ORA_OK;
        #pragma omp parallel
        {
        /* per-pencil work: reconstructed values at both faces of each
         * cell, and fluxes at the faces (one set per thread) */
        int mine = ORA_OK;
        double *rp = malloc(sizeof(double) * (nmax + 2) * nv);
        double *rm = malloc(sizeof(double) * (nmax + 2) * nv);
        double *Ff = malloc(sizeof(double) * (nmax + 1) * nv);
        double *uf = malloc(sizeof(double) * (nmax + 1));
        if (!rp || !rm || !Ff || !uf) mine = ORA_E_NOMEM;
        #pragma omp for schedule(static)
        for (int b = 0; b < n2; b++)
            for (int a = 0; a < n1; a++) {
                if (mine == ORA_E_NOMEM) continue;
                int c[3];
                c[o1] = a;
                c[o2] = b;
                /* reconstruction: cells -1 .. n along d */
                for (int cell = -1; cell <= n; cell++)
                    for (int v = 0; v < nv; v++) {
                        double s[5];
                        for (int t = 0; t < 5; t++) {
                            c[d] = cell - 2 + t;
                            s[t] = w[at(g, v, c[0], c[1], c[2])];
                        }
                        int lin = g->recon == 1;
                        if (g->recon == 2) {
                            c[d] = cell;
                            lin = g->smooth[(int64_t)d * ora_padded_cells(g) + at(g, 0, c[0], c[1], c[2])] != 0;
                        }
                        double *pl = &rp[(cell + 1) * nv + v], *mi = &rm[(cell + 1) * nv + v];
                        if (cf && g->recon == 0)
                            ora_weno5_nonuniform(&cf[cell + 1], s, g->weno_eps, pl, mi);
                        else if (g->recon == 3)
                            ora_weno3(&s[1], g->weno_eps, pl, mi);
                        else if (g->recon == 4)
                            *pl = *mi = s[2]; /* first order: the cell value at both faces */
                        else if (lin)
                            ora_linear5(s, pl, mi);
                        else
                            ora_weno5(s, g->weno_eps, pl, mi, NULL);
                    }
                /* Riemann problems at faces f - 1/2, f = 0 .. n: left state
                 * from cell f-1 (its + face), right state from cell f */
                for (int f = 0; f <= n; f++) {
                    if (ora_hllc(g, d, &rp[f * nv], &rm[(f + 1) * nv], &Ff[f * nv], &uf[f]) != ORA_OK)
                        mine = ORA_E_NONPHYSICAL;
                }
                /* flux differences and the divergence of the face velocity */
                for (int cell = 0; cell < n; cell++) {
                    double inv_dx = 1.0 / ora_cell_width(g, d, cell);
                    int side = cell == 0 && g->bc[2 * d] == 2 ? 0 : (cell == n - 1 && g->bc[2 * d + 1] == 2 ? 1 : -1);
                    if (side >= 0) {
                        /* characteristic boundary cell: second-order one-sided
                         * derivative of the primitives into the domain (on
                         * non-uniform cells, that of the quadratic through
                         * the three cell centres) */
                        double wc[MAXV], dw[MAXV], dq[MAXV], cs[3];
                        int sg = side == 0 ? 1 : -1;
                        if (g->faces[d]) ora_one_sided_coef(g, d, side, cs);
                        for (int v = 0; v < nv; v++) {
                            double f[3];
                            for (int t = 0; t < 3; t++) {
                                c[d] = cell + sg * t;
                                f[t] = w[at(g, v, c[0], c[1], c[2])];
                            }
                            wc[v] = f[0];
                            if (g->faces[d])
                                dw[v] = cs[0] * f[0] + cs[1] * f[1] + cs[2] * f[2];
                            else
                                dw[v] = sg * (-3.0 * f[0] + 4.0 * f[1] - f[2]) * 0.5 * inv_dx;
                        }
                        c[d] = cell;
                        ora_cbc_cell(g, d, side, wc, dw, dq);
                        for (int v = 0; v < nv; v++) rhs[at(g, v, c[0], c[1], c[2])] += dq[v];
                        continue;   /* no flux difference, no d-part of div(u) */
                    }
                    c[d] = cell;
                    for (int v = 0; v < nv; v++)
                        rhs[at(g, v, c[0], c[1], c[2])] += (Ff[cell * nv + v] - Ff[(cell + 1) * nv + v]) * inv_dx;
                    divu[at(g, 0, c[0], c[1], c[2])] += (uf[cell + 1] - uf[cell]) * inv_dx;
                }
            }
        free(rp); free(rm); free(Ff); free(uf);
        #pragma omp critical
        if (mine < pencil_status) pencil_status = mine;
        }
        if (pencil_status < status) status = pencil_status;
        free(cf);
        if (status == ORA_E_NOMEM) break;
    }
    /* non-conservative source: -h div(u) with h = -alpha1 (Allaire) or
     * h = -(alpha1 + K) (Kapila) on the alpha1 row */
    #pragma omp parallel for schedule(static)
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                double h = w[at(g, nv - 1, i, j, k)];
                if (g->model == 1) {
                    double wc[MAXV];
                    for (int v = 0; v < nv; v++)
                        wc[v] = w[at(g, v, i, j, k)];
                    h += ora_kapila_K(g, wc);
                }
                rhs[at(g, nv - 1, i, j, k)] += h * divu[at(g, 0, i, j, k)];
            }

    free(w); free(divu);
    return status;
}

/* ---------------------------------------------------------------------- */
/* Time stepping (Sec. 3.4) and the CFL time step                           */
/* ---------------------------------------------------------------------- */

/* Stage combinations of the third-order TVD (SSP) Runge-Kutta scheme of
 * Gottlieb and Shu, Shu-Osher form, over count values:
 *   stage 1: out = q0 + dt L
 *   stage 2: out = 3/4 q0 + 1/4 (qs + dt L)
 *   stage 3: out = 1/3 q0 + 2/3 (qs + dt L)                               */
int ora_rk3_combine(int stage, int64_t count, const double *q0, const double *qs, const double *L,
                    double dt, double *out)
{
    for (int64_t t = 0; t < count; t++) {
        if (stage == 1) out[t] = q0[t] + dt * L[t];
        else if (stage == 2) out[t] = 0.75 * q0[t] + 0.25 * (qs[t] + dt * L[t]);
        else if (stage == 3) out[t] = (1.0 / 3.0) * q0[t] + (2.0 / 3.0) * (qs[t] + dt * L[t]);
        else return ORA_E_ARG;
    }
    return ORA_OK;
}

/* Largest signal speed over interior cells: max over cells of
 * max_d (|u_d| + c).  Returns ORA_E_NONPHYSICAL if a cell is non-physical. */
int ora_max_wavespeed(const ora_grid *g, const double *q, double *smax)
{
    int nd = g->ndim, nv = 4 + nd, status = ORA_OK;
    double s = 0.0;
    for (int k = 0; k < g->n[2]; k++)
        for (int j = 0; j < g->n[1]; j++)
            for (int i = 0; i < g->n[0]; i++) {
                double qc[MAXV], wc[MAXV];
                for (int v = 0; v < nv; v++) qc[v] = q[at(g, v, i, j, k)];
                if (ora_cons_to_prim(g, qc, wc) != ORA_OK) status = ORA_E_NONPHYSICAL;
                double c = sqrt(ora_sound_speed2(g, wc[0] + wc[1], wc[2 + nd], wc[nv - 1]));
                for (int d = 0; d < nd; d++) {
                    double sd = fabs(wc[2 + d]) + c;
                    if (sd > s) s = sd;
                }
            }
    *smax = s;
    return status;
}

/* One SSP-RK3 step of size dt, in place on q (interior cells are advanced;
 * ghost cells are refilled before every right-hand side). */
int ora_rk3_step(const ora_grid *g, double *q, double dt)
{
    int nv = 4 + g->ndim;
    int64_t count = ora_padded_cells(g) * nv;
    double *q0 = malloc(sizeof(double) * count);
    double *qs = malloc(sizeof(double) * count);
    double *L = calloc(count, sizeof(double));
    int status = ORA_OK;
    if (!q0 || !qs || !L) {
        free(q0); free(qs); free(L);
        return ORA_E_NOMEM;
    }
    memcpy(q0, q, sizeof(double) * count);
    memcpy(qs, q, sizeof(double) * count);
    for (int stage = 1; stage <= 3; stage++) {
        ora_fill_ghosts(g, qs);
        if (ora_rhs(g, qs, L) != ORA_OK) status = ORA_E_NONPHYSICAL;
        /* ghost entries of L are zero and q0/qs ghost values are discarded
         * by the next fill, so combining whole arrays touches interior
         * results only where it matters */
        ora_rk3_combine(stage, count, q0, qs, L, dt, stage == 3 ? q : qs);
    }
    free(q0); free(qs); free(L);
    return status;
}

/* The CFL step on non-uniform cells: cfl times the smallest, over interior
 * cells and dimensions, of Delta x_d(cell) / (|u_d| + c). */
int ora_cfl_dt_nonuniform(const ora_grid *g, const double *q, double cfl, double *dt)
{
    int nd = g->ndim, nv = 4 + nd, status = ORA_OK;
    double m = INFINITY;
    for (int k = 0; k < g->n[2]; k++)
        for (int j = 0; j < g->n[1]; j++)
            for (int i = 0; i < g->n[0]; i++) {
                double qc[MAXV], wc[MAXV];
                for (int v = 0; v < nv; v++) qc[v] = q[at(g, v, i, j, k)];
                if (ora_cons_to_prim(g, qc, wc) != ORA_OK) status = ORA_E_NONPHYSICAL;
                double c = sqrt(ora_sound_speed2(g, wc[0] + wc[1], wc[2 + nd], wc[nv - 1]));
                int idx[3] = {i, j, k};
                for (int d = 0; d < nd; d++) {
                    double r = ora_cell_width(g, d, idx[d]) / (fabs(wc[2 + d]) + c);
                    if (r < m) m = r;
                }
            }
    *dt = cfl * m;
    return status;
}

static int nonuniform(const ora_grid *g)
{
    return g->faces[0] || g->faces[1] || g->faces[2];
}

/* nsteps steps; dt = cfl * min_d dx_d / smax(q^n) if cfl > 0 (on
 * non-uniform cells cfl * min over cells and d of Delta x_d/(|u_d| + c)),
 * else dt_fixed.  *t_out receives the total time advanced. */
int ora_run(const ora_grid *g, double *q, int nsteps, double cfl, double dt_fixed, double *t_out)
{
    double t = 0.0, dxmin = g->dx[0];
    for (int d = 1; d < g->ndim; d++)
        if (g->dx[d] < dxmin) dxmin = g->dx[d];
    int status = ORA_OK;
    for (int s = 0; s < nsteps && status == ORA_OK; s++) {
        double dt = dt_fixed;
        if (cfl > 0.0 && nonuniform(g)) {
            status = ora_cfl_dt_nonuniform(g, q, cfl, &dt);
            if (status != ORA_OK) break;
        } else if (cfl > 0.0) {
            double smax;
            status = ora_max_wavespeed(g, q, &smax);
            if (status != ORA_OK) break;
            dt = cfl * dxmin / smax;
        }
        status = ora_rk3_step(g, q, dt);
        t += dt;
    }
    if (t_out) *t_out = t;
    return status;
}

/* ---------------------------------------------------------------------- */
/* Whole-array conversions (every padded cell)                              */
/* ---------------------------------------------------------------------- */

/* Primitive -> conservative on every cell of a padded array (v-major). */
int ora_prim_to_cons_field(const ora_grid *g, const double *w, double *q)
{
    int nv = 4 + g->ndim;
    int64_t ncell = ora_padded_cells(g);
    for (int64_t c = 0; c < ncell; c++) {
        double wc[MAXV], qc[MAXV];
        for (int v = 0; v < nv; v++) wc[v] = w[v * ncell + c];
        ora_prim_to_cons(g, wc, qc);
        for (int v = 0; v < nv; v++) q[v * ncell + c] = qc[v];
    }
    return ORA_OK;
}

/* Conservative -> primitive on every cell of a padded array (v-major). */
int ora_cons_to_prim_field(const ora_grid *g, const double *q, double *w)
{
    int nv = 4 + g->ndim, status = ORA_OK;
    int64_t ncell = ora_padded_cells(g);
    for (int64_t c = 0; c < ncell; c++) {
        double qc[MAXV], wc[MAXV];
        for (int v = 0; v < nv; v++) qc[v] = q[v * ncell + c];
        if (ora_cons_to_prim(g, qc, wc) != ORA_OK) status = ORA_E_NONPHYSICAL;
        for (int v = 0; v < nv; v++) w[v * ncell + c] = wc[v];
    }
    return status;
}
