// Non-uniform (stretched) grids (Sec. 4.1: structured meshes with
// non-uniform spacing, refined locally by hyperbolic-tangent stretching):
// host-side construction of the per-cell WENO5 coefficients and inverse
// widths read by the fused kernel.
//
// For cell i of width h_i, with xi = (x - x_i)/h_i, the candidate p_r of
// stencil r (cells i-2+r .. i+r) is the derivative of the cubic that
// interpolates the primitive function V(xi) = int v dxi at the four faces of
// the stencil (so that p_r has the data as its cell averages); the 5-cell
// quartic q is built the same way from six faces.  Per cell and direction
// the table holds, for r = 0, 1, 2 and the stencil's cells j = 0, 1, 2:
//   [0, 9)    p_r(xi = 1/2)  coefficients   (x_{i+1/2} value)
//   [9, 18)   p_r(xi = -1/2) coefficients   (x_{i-1/2} value)
//   [18, 27)  d p_r/d xi at 0               (a1)
//   [27, 36)  (d^2 p_r/d xi^2)/2 at 0        (a2)
//   [36, 39)  ideal weights at x_{i+1/2}, [39, 42) at x_{i-1/2},
// where sum_r d_r p_r reproduces q at the face; the smoothness indicator
// sum_l h^{2l-1} int_{I_i} (p_r^(l))^2 is then a1^2 + (13/3) a2^2.
#include <cmath>
#include <vector>

#include "internal.h"

namespace mfc {

namespace {

// Width of cell i (-NG <= i < n + NG): ghost cells repeat the widths of
// the interior cells the ghost fill copies into them (mirror image for
// extrapolation, one period away for periodic boundaries).
double ghost_width(const double *faces, int n, int bc_lo, int bc_hi, int i)
{
    if (i < 0) i = bc_lo == MFC_BC_PERIODIC ? n + i : -i - 1;
    else if (i >= n) i = bc_hi == MFC_BC_PERIODIC ? i - n : 2 * n - 1 - i;
    return faces[i + 1] - faces[i];
}

// Monomial coefficients (degree m-1, lowest first) of the Lagrange basis
// polynomial ell_k on nodes X[0 .. m-1].
void lagrange_basis(const double *X, int m, int k, double *c)
{
    for (int t = 0; t < m; t++) c[t] = 0.0;
    c[0] = 1.0;
    int deg = 0;
    for (int q = 0; q < m; q++) {
        if (q == k) continue;
        const double den = X[k] - X[q];
        // multiply by (xi - X[q]) / den
        for (int t = deg + 1; t >= 0; t--) {
            const double hi = t > 0 ? c[t - 1] : 0.0;
            const double lo = t <= deg ? c[t] * X[q] : 0.0;
            c[t] = (hi - lo) / den;
        }
        deg++;
    }
}

// Monomial coefficients of the polynomial p of degree m-1 with average v_j
// over cell j of the m cells between the m+1 faces X (in xi units): for
// unit data on cell j, coef[j][t].
void reconstruction_basis(const double *X, int m, double coef[5][5])
{
    // V(X_k) = sum_{l < k} (X_{l+1} - X_l) v_l;  p = V' = sum_k V(X_k) ell_k'
    double dl[6][6];
    for (int k = 0; k <= m; k++) {
        double c[6];
        lagrange_basis(X, m + 1, k, c);
        for (int t = 0; t < m; t++) dl[k][t] = (t + 1) * c[t + 1];   // derivative
    }
    for (int j = 0; j < m; j++)
        for (int t = 0; t < m; t++) {
            double s = 0.0;
            for (int k = j + 1; k <= m; k++) s += dl[k][t];
            coef[j][t] = (X[j + 1] - X[j]) * s;
        }
}

double horner(const double *c, int m, double x)
{
    double v = 0.0;
    for (int t = m - 1; t >= 0; t--) v = v * x + c[t];
    return v;
}

// The 42 coefficients of cell i from the widths of cells i-2 .. i+2.
void cell_coefficients(const double *w, double *out)
{
    // faces of cells i-2 .. i+2 in xi units (cell i = [-1/2, 1/2])
    double X[6];
    X[2] = -0.5;
    X[3] = 0.5;
    X[4] = X[3] + w[3] / w[2];
    X[5] = X[4] + w[4] / w[2];
    X[1] = X[2] - w[1] / w[2];
    X[0] = X[1] - w[0] / w[2];
    double q[5][5], pr[5][5];
    reconstruction_basis(X, 5, q);
    for (int r = 0; r < 3; r++) {
        reconstruction_basis(X + r, 3, pr);
        for (int j = 0; j < 3; j++) {
            out[3 * r + j] = horner(pr[j], 3, 0.5);
            out[9 + 3 * r + j] = horner(pr[j], 3, -0.5);
            out[18 + 3 * r + j] = pr[j][1];
            out[27 + 3 * r + j] = pr[j][2];
        }
    }
    // cell i-2 appears only in stencil 0, cell i+2 only in stencil 2
    const double qp0 = horner(q[0], 5, 0.5), qp4 = horner(q[4], 5, 0.5);
    const double qm0 = horner(q[0], 5, -0.5), qm4 = horner(q[4], 5, -0.5);
    out[36] = qp0 / out[0];
    out[38] = qp4 / out[8];
    out[37] = 1.0 - out[36] - out[38];
    out[39] = qm0 / out[9];
    out[41] = qm4 / out[17];
    out[40] = 1.0 - out[39] - out[41];
}

}  // namespace

int build_stretch_tables(mfc_grid *h, const mfc_grid_desc *d)
{
    for (int dim = 0; dim < d->ndim; dim++) {
        if (!d->faces[dim]) continue;
        const int n = d->n[dim];
        const double *f = d->faces[dim];
        std::vector<double> tab((size_t)(n + 2) * kStretchCoef), inv(n);
        for (int c = -1; c <= n; c++) {
            double w[5];
            for (int t = 0; t < 5; t++)
                w[t] = ghost_width(f, n, d->bc[2 * dim], d->bc[2 * dim + 1], c - 2 + t);
            cell_coefficients(w, &tab[(size_t)(c + 1) * kStretchCoef]);
        }
        for (int c = 0; c < n; c++) inv[c] = 1.0 / (f[c + 1] - f[c]);
        double *dt = nullptr, *di = nullptr;
        if (hipMalloc((void **)&dt, tab.size() * sizeof(double)) != hipSuccess ||
            hipMalloc((void **)&di, inv.size() * sizeof(double)) != hipSuccess) {
            if (dt) (void)hipFree(dt);
            return fail(MFC_E_NOMEM, "stretched-grid tables");
        }
        if (hipMemcpy(dt, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(di, inv.data(), inv.size() * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
            (void)hipFree(dt);
            (void)hipFree(di);
            return fail(MFC_E_HIP, "stretched-grid table upload");
        }
        h->g.wcoef[dim] = dt;
        h->g.winv[dim] = di;
    }
    return MFC_OK;
}

void free_stretch_tables(mfc_grid *h)
{
    for (int dim = 0; dim < 3; dim++) {
        if (h->g.wcoef[dim]) (void)hipFree((void *)h->g.wcoef[dim]);
        if (h->g.winv[dim]) (void)hipFree((void *)h->g.winv[dim]);
        h->g.wcoef[dim] = h->g.winv[dim] = nullptr;
    }
}

}  // namespace mfc
