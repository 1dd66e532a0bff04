// Staged right-hand side: the method's steps as separate passes over HBM,
// in the order the paper's solver runs them (Sec. 3.1-3.2.1):
//   1. conservative -> primitive on interior cells and ghost face slabs;
//   2. per direction, WENO5 reconstruction of every cell's two face values;
//   3. per direction, the HLLC flux and face velocity at every face;
//   4. per interior cell, flux differences + alpha1 div(u), then either the
//      plain right-hand side or an SSP-RK3 stage combination.
// Simple and easy to check; the fused kernel is the fast path.
#include "internal.h"

namespace mfc {
namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ int64_t cell_offset(const Grid &g, int i, int j, int k)
{
    return (int64_t)(k + g.off[2]) * g.stride[2] + (int64_t)(j + g.off[1]) * g.stride[1] + (i + g.off[0]);
}

// Decompose a linear index over a box [lo, lo + ext) of interior-relative cells.
__device__ __forceinline__ void box_index(int64_t t, const int lo[3], const int ext[3], int &i, int &j, int &k)
{
    i = lo[0] + (int)(t % ext[0]);
    int64_t r = t / ext[0];
    j = lo[1] + (int)(r % ext[1]);
    k = lo[2] + (int)(r / ext[1]);
}

struct Box {
    int lo[3];
    int ext[3];
    __host__ __device__ int64_t count() const { return (int64_t)ext[0] * ext[1] * ext[2]; }
};

template <int NDIM>
__global__ void __launch_bounds__(kThreads) k_prim(Grid g, const double *__restrict__ q, double *__restrict__ w,
                                                   int *__restrict__ flag, Box b)
{
    constexpr int NV = 4 + NDIM;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.count()) return;
    int i, j, k;
    box_index(t, b.lo, b.ext, i, j, k);
    int outside = (i < 0 || i >= g.n[0]) + (j < 0 || j >= g.n[1]) + (k < 0 || k >= g.n[2]);
    if (outside > 1) return;  // edges and corners are never read
    int64_t c = cell_offset(g, i, j, k);
    double qc[NV], wc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + c];
    if (cons_to_prim<NDIM>(g, qc, wc)) atomicOr(flag, 1);
#pragma unroll
    for (int v = 0; v < NV; v++) w[v * g.vstride + c] = wc[v];
}

template <int NDIM, int DIR>
__global__ void __launch_bounds__(kThreads) k_recon(Grid g, const double *__restrict__ w, double *__restrict__ rp,
                                                    double *__restrict__ rm, Box b)
{
    constexpr int NV = 4 + NDIM;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.count()) return;
    int i, j, k;
    box_index(t, b.lo, b.ext, i, j, k);
    int64_t c = cell_offset(g, i, j, k);
    int64_t s = g.stride[DIR];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const double *x = w + v * g.vstride + c;
        double plus, minus;
        switch (g.order) {
        case 3: recon_pair<3, double>(x[-2 * s], x[-s], x[0], x[s], x[2 * s], g.eps, plus, minus); break;
        case 1: recon_pair<1, double>(x[-2 * s], x[-s], x[0], x[s], x[2 * s], g.eps, plus, minus); break;
        default: recon_pair<5, double>(x[-2 * s], x[-s], x[0], x[s], x[2 * s], g.eps, plus, minus);
        }
        rp[v * g.vstride + c] = plus;
        rm[v * g.vstride + c] = minus;
    }
}

// Face f - 1/2 (between cells f-1 and f along DIR) is stored at cell f.
template <int NDIM, int DIR>
__global__ void __launch_bounds__(kThreads) k_riemann(Grid g, const double *__restrict__ rp,
                                                      const double *__restrict__ rm, double *__restrict__ F,
                                                      int *__restrict__ flag, Box b)
{
    constexpr int NV = 4 + NDIM;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.count()) return;
    int i, j, k;
    box_index(t, b.lo, b.ext, i, j, k);
    int64_t c = cell_offset(g, i, j, k);
    int64_t s = g.stride[DIR];
    double wL[NV], wR[NV], f[NV], uf;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        wL[v] = rp[v * g.vstride + c - s];
        wR[v] = rm[v * g.vstride + c];
    }
    if (hllc<NDIM, DIR>(g, wL, wR, f, uf)) atomicOr(flag, 1);
#pragma unroll
    for (int v = 0; v < NV; v++) F[v * g.vstride + c] = f[v];
    F[NV * g.vstride + c] = uf;
}

template <int NDIM>
__global__ void __launch_bounds__(kThreads) k_update(Grid g, const double *__restrict__ faces,
                                                     const double *__restrict__ w, const double *__restrict__ q,
                                                     const double *q0, double *out,  // may alias (last stage)
                                                     int mode, double dt, const double *__restrict__ dt_dev, Box b)
{
    constexpr int NV = 4 + NDIM, A = 3 + NDIM;
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= b.count()) return;
    int i, j, k;
    box_index(t, b.lo, b.ext, i, j, k);
    int64_t c = cell_offset(g, i, j, k);
    double L[NV], divu = 0.0;
#pragma unroll
    for (int v = 0; v < NV; v++) L[v] = 0.0;
#pragma unroll
    for (int d = 0; d < NDIM; d++) {
        const double *F = faces + (int64_t)d * (NV + 1) * g.vstride;
        int64_t s = g.stride[d];
#pragma unroll
        for (int v = 0; v < NV; v++) L[v] += (F[v * g.vstride + c] - F[v * g.vstride + c + s]) * g.inv_dx[d];
        divu += (F[NV * g.vstride + c + s] - F[NV * g.vstride + c]) * g.inv_dx[d];
    }
    L[A] += alpha_source<double>(g, w[A * g.vstride + c], w[(A - 1) * g.vstride + c]) * divu;
    if (mode == 0) {
#pragma unroll
        for (int v = 0; v < NV; v++) out[v * g.vstride + c] = L[v];
        return;
    }
    const double h = dt_dev ? *dt_dev : dt;
    const double a = mode == 1 ? 0.0 : (mode == 2 ? 0.75 : 1.0 / 3.0);
    const double bb = mode == 1 ? 1.0 : (mode == 2 ? 0.25 : 2.0 / 3.0);
    // every operand before the first store (out may alias q0)
    double a0[NV], a1[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) {
        a0[v] = q0[v * g.vstride + c];
        a1[v] = q[v * g.vstride + c];
    }
#pragma unroll
    for (int v = 0; v < NV; v++) out[v * g.vstride + c] = a * a0[v] + bb * (a1[v] + h * L[v]);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

template <int NDIM, int DIR>
int recon_riemann(mfc_grid *h, hipStream_t s)
{
    const Grid &g = h->g;
    Box rb{{0, 0, 0}, {g.n[0], g.n[1], g.n[2]}};
    rb.lo[DIR] = -1;
    rb.ext[DIR] = g.n[DIR] + 2;
    hipLaunchKernelGGL((k_recon<NDIM, DIR>), dim3(blocks_for(rb.count())), dim3(kThreads), 0, s, g, h->prim, h->recp,
                       h->recm, rb);
    Box fb{{0, 0, 0}, {g.n[0], g.n[1], g.n[2]}};
    fb.ext[DIR] = g.n[DIR] + 1;
    double *F = h->faces + (int64_t)DIR * (h->nvar + 1) * g.vstride;
    hipLaunchKernelGGL((k_riemann<NDIM, DIR>), dim3(blocks_for(fb.count())), dim3(kThreads), 0, s, g, h->recp,
                       h->recm, F, h->flag, fb);
    return MFC_OK;
}

template <int NDIM>
int rhs_staged(mfc_grid *h, const double *q, const double *q0, double *out, int mode, double dt,
               const double *dt_dev, hipStream_t s)
{
    const Grid &g = h->g;
    Box pb{{0, 0, 0}, {g.p[0], g.p[1], g.p[2]}};
    for (int d = 0; d < NDIM; d++) pb.lo[d] = -NG;
    timing_begin(h, s);  // the staged passes are timed together
    hipLaunchKernelGGL((k_prim<NDIM>), dim3(blocks_for(pb.count())), dim3(kThreads), 0, s, g, q, h->prim, h->flag,
                       pb);
    recon_riemann<NDIM, 0>(h, s);
    if (NDIM > 1) recon_riemann<NDIM, (NDIM > 1 ? 1 : 0)>(h, s);
    if (NDIM > 2) recon_riemann<NDIM, (NDIM > 2 ? 2 : 0)>(h, s);
    Box ub{{0, 0, 0}, {g.n[0], g.n[1], g.n[2]}};
    hipLaunchKernelGGL((k_update<NDIM>), dim3(blocks_for(ub.count())), dim3(kThreads), 0, s, g, h->faces, h->prim,
                       q, q0, out, mode, dt, dt_dev, ub);
    timing_end(h, s);
    return hip_status(hipGetLastError(), "staged right-hand side launch");
}

}  // namespace

int launch_rhs_staged(mfc_grid *h, const void *qv, const void *q0v, void *outv, int mode, double dt,
                      const double *dt_dev, hipStream_t s)
{
    if (h->desc.precision != MFC_FP64) return fail(MFC_E_UNSUPPORTED, "the staged path is FP64 only");
    const double *q = (const double *)qv, *q0 = (const double *)q0v;
    double *out = (double *)outv;
    switch (h->g.ndim) {
    case 1: return rhs_staged<1>(h, q, q0, out, mode, dt, dt_dev, s);
    case 2: return rhs_staged<2>(h, q, q0, out, mode, dt, dt_dev, s);
    default: return rhs_staged<3>(h, q, q0, out, mode, dt, dt_dev, s);
    }
}

}  // namespace mfc
