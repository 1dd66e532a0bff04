// C ABI of the library (declared in include/mfc.h): argument validation,
// scratch ownership, the small kernels around the right-hand side (ghost
// fill, EOS conversions, the CFL reduction, the time-step bookkeeping) and
// the SSP-RK3 driver.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>

#include "internal.h"

namespace mfc {

static thread_local char g_detail[512] = "";

// The detail of a failure is formatted into a fixed thread-local buffer (no
// heap allocation on the error paths).
int fail(int status, const char *detail)
{
    std::snprintf(g_detail, sizeof g_detail, "%s", detail);
    return status;
}

int fail(int status, const std::string &detail) { return fail(status, detail.c_str()); }

int hip_status(hipError_t e, const char *what)
{
    if (e == hipSuccess) return MFC_OK;
    std::snprintf(g_detail, sizeof g_detail, "%s: %s", what, hipGetErrorString(e));
    return e == hipErrorOutOfMemory ? MFC_E_NOMEM : MFC_E_HIP;
}

void timing_begin(mfc_grid *h, hipStream_t s, int slot)
{
    if (!h->timing || h->timing_skip) return;
    auto &ev = h->ev[slot];
    if (h->ev_used[slot] + 2 > ev.size()) {
        for (int t = 0; t < 64; t++) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            ev.push_back(e);
        }
    }
    (void)hipEventRecord(ev[h->ev_used[slot]], s);
}

void timing_end(mfc_grid *h, hipStream_t s, int slot)
{
    if (!h->timing || h->timing_skip || h->ev_used[slot] + 2 > h->ev[slot].size()) return;
    (void)hipEventRecord(h->ev[slot][h->ev_used[slot] + 1], s);
    h->ev_used[slot] += 2;
}

void set_kapila(Grid &g, const mfc_grid_desc &d)
{
    g.kapila = d.model == MFC_MODEL_KAPILA;
    for (int k = 0; k < 2; k++) {
        g.zg[k] = d.gamma[k];
        g.zp[k] = d.gamma[k] * d.pi_inf[k];
    }
}

void make_grid(const mfc_grid_desc &desc, Grid &g)
{
    g = Grid{};
    g.ndim = desc.ndim;
    for (int d = 0; d < 3; d++) {
        bool act = d < desc.ndim;
        g.n[d] = act ? desc.n[d] : 1;
        g.off[d] = act ? NG : 0;
        g.p[d] = act ? desc.n[d] + 2 * NG : 1;
        g.inv_dx[d] = act ? desc.n[d] / (desc.hi[d] - desc.lo[d]) : 0.0;
        g.bc[2 * d] = act ? desc.bc[2 * d] : MFC_BC_EXTRAP;
        g.bc[2 * d + 1] = act ? desc.bc[2 * d + 1] : MFC_BC_EXTRAP;
    }
    g.dxmin = 1e300;
    for (int d = 0; d < desc.ndim; d++) g.dxmin = std::fmin(g.dxmin, (desc.hi[d] - desc.lo[d]) / desc.n[d]);
    g.stride[0] = 1;
    g.stride[1] = g.p[0];
    g.stride[2] = (int64_t)g.p[0] * g.p[1];
    g.vstride = (int64_t)g.p[0] * g.p[1] * g.p[2];
    g.g1 = 1.0 / (desc.gamma[0] - 1.0);
    g.g2 = 1.0 / (desc.gamma[1] - 1.0);
    g.h1 = desc.gamma[0] * desc.pi_inf[0] / (desc.gamma[0] - 1.0);
    g.h2 = desc.gamma[1] * desc.pi_inf[1] / (desc.gamma[1] - 1.0);
    g.eps = desc.weno_eps;
    set_kapila(g, desc);
    g.order = desc.recon == MFC_RECON_WENO3 ? 3 : (desc.recon == MFC_RECON_FIRST_ORDER ? 1 : 5);
    g.stretched = 0;
    for (int d = 0; d < desc.ndim; d++) g.stretched |= desc.faces[d] != nullptr;
    if (g.stretched) g.dxmin = 1.0;   // the reduction then returns max (|u_d| + c)/dx_d
    // one-sided derivative at the boundary cell of a non-uniform dimension
    // (characteristic faces, Sec. 3.3): that of the quadratic through the
    // centres x0 (the boundary cell), x1, x2 (the next two into the domain);
    // with h1 = x1 - x0, h2 = x2 - x0 the weights of f1 and f2 are
    // h2 / (h1 (h2 - h1)) and -h1 / (h2 (h2 - h1)), and f0 takes minus
    // their sum (constants have no derivative)
    for (int d = 0; d < desc.ndim; d++) {
        const double *f = desc.faces[d];
        if (!f) continue;
        for (int side = 0; side < 2; side++) {
            const int n = desc.n[d], b = side ? n - 1 : 0, s = side ? -1 : 1;
            auto centre = [&](int i) { return 0.5 * (f[i] + f[i + 1]); };
            const double h1 = centre(b + s) - centre(b), h2 = centre(b + 2 * s) - centre(b);
            double *c = g.cbc_cf[2 * d + side];
            c[1] = h2 / (h1 * (h2 - h1));
            c[2] = -h1 / (h2 * (h2 - h1));
            c[0] = -(c[1] + c[2]);
        }
    }
}

namespace {

constexpr int kThreads = 256;

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

// ------------------------------------------------------------ ghost fill
// One thread per (variable, ghost layer, side, face-slab cell) of every
// active dimension: the slabs of dimension d take the thread range
// [start[d], start[d + 1]).
template <class T>
__global__ void __launch_bounds__(kThreads) k_ghosts(Grid g, T *__restrict__ q, int nv, int64_t s1, int64_t s2,
                                                     int64_t s3)
{
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= s3) return;
    const int d = t < s1 ? 0 : (t < s2 ? 1 : 2);
    t -= d == 0 ? 0 : (d == 1 ? s1 : s2);
    const int bc_lo = g.bc[2 * d], bc_hi = g.bc[2 * d + 1];
    int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
    int n1 = g.n[o1], n2 = g.n[o2], n = g.n[d];
    int64_t per_var = (int64_t)2 * NG * n1 * n2;
    int v = (int)(t / per_var);
    int64_t r = t % per_var;
    int a, b, l, side;
    if (d == 0) {
        // x slabs are 3 cells wide: let consecutive threads take the
        // consecutive ghost cells of a row (x = -3, -2, -1 and n .. n+2)
        const int u = (int)(r % NG);
        r /= NG;
        side = (int)(r % 2);
        r /= 2;
        a = (int)(r % n1);
        b = (int)(r / n1);
        l = side == 0 ? NG - u : 1 + u;
    } else {
        // y and z slabs: consecutive threads take consecutive x
        a = (int)(r % n1);
        r /= n1;
        b = (int)(r % n2);
        r /= n2;
        l = 1 + (int)(r % NG);
        side = (int)(r / NG);
    }
    int c[3], src[3];
    c[o1] = src[o1] = a;
    c[o2] = src[o2] = b;
    if (side == 0) {
        c[d] = -l;
        src[d] = bc_lo == MFC_BC_PERIODIC ? n - l : 0;
    } else {
        c[d] = n - 1 + l;
        src[d] = bc_hi == MFC_BC_PERIODIC ? l - 1 : n - 1;
    }
    auto off = [&](const int *x) {
        return (int64_t)(x[2] + g.off[2]) * g.stride[2] + (int64_t)(x[1] + g.off[1]) * g.stride[1] + (x[0] + g.off[0]);
    };
    q[v * g.vstride + off(c)] = q[v * g.vstride + off(src)];
}

// ------------------------------------------------------ EOS conversions
template <int NDIM, class T>
__global__ void __launch_bounds__(kThreads) k_p2c(Grid g, const T *__restrict__ w, T *__restrict__ q)
{
    constexpr int NV = 4 + NDIM;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.vstride) return;
    T wc[NV], qc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) wc[v] = w[v * g.vstride + c];
    prim_to_cons<NDIM, T>(g, wc, qc);
#pragma unroll
    for (int v = 0; v < NV; v++) q[v * g.vstride + c] = qc[v];
}

template <int NDIM, class T>
__global__ void __launch_bounds__(kThreads) k_c2p(Grid g, const T *__restrict__ q, T *__restrict__ w,
                                                  int *__restrict__ flag)
{
    constexpr int NV = 4 + NDIM;
    int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= g.vstride) return;
    T qc[NV], wc[NV];
#pragma unroll
    for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + c];
    if (cons_to_prim<NDIM, T>(g, qc, wc)) atomicOr(flag, 1);
#pragma unroll
    for (int v = 0; v < NV; v++) w[v * g.vstride + c] = wc[v];
}

// -------------------------------------------------- CFL wave-speed reduction
// Per-block maxima of max_d (|u_d| + c) over interior cells (grid-stride),
// reduced within each wavefront by butterfly shuffles and across the block
// through LDS.  Maxima are exact and order-independent.
template <int NDIM, class T>
__global__ void __launch_bounds__(kReduceThreads) k_wavespeed(Grid g, const T *__restrict__ q,
                                                              double *__restrict__ partial, int *__restrict__ flag)
{
    constexpr int NV = 4 + NDIM, E = 2 + NDIM, A = 3 + NDIM;
    __shared__ double red[kReduceThreads / 64];
    double smax = 0.0;
    const int64_t total = (int64_t)g.n[0] * g.n[1] * g.n[2];
    bool bad = false;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        int i = (int)(t % g.n[0]);
        int64_t r = t / g.n[0];
        int j = (int)(r % g.n[1]);
        int k = (int)(r / g.n[1]);
        int64_t c = (int64_t)(k + g.off[2]) * g.stride[2] + (int64_t)(j + g.off[1]) * g.stride[1] + (i + g.off[0]);
        T qc[NV], wc[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + c];
        bad |= cons_to_prim<NDIM, T>(g, qc, wc);
        double Gam, Pi;
        mixture<double>(g, double(wc[A]), Gam, Pi);
        double cs = sqrtT(sound2<double>(Gam, Pi, double(wc[0]) + double(wc[1]), double(wc[E])));
        if (g.stretched) {
            // non-uniform cells: the largest (|u_d| + c)/dx_d (the CFL step is cfl over it)
            const int idx[3] = {i, j, k};
#pragma unroll
            for (int d = 0; d < NDIM; d++) {
                const double iw = g.winv[d] ? g.winv[d][idx[d]] : g.inv_dx[d];
                smax = __builtin_fmax(smax, (__builtin_fabs(double(wc[2 + d])) + cs) * iw);
            }
        } else {
#pragma unroll
            for (int d = 0; d < NDIM; d++) smax = __builtin_fmax(smax, __builtin_fabs(double(wc[2 + d])) + cs);
        }
    }
    if (bad) atomicOr(flag, 2);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) smax = __builtin_fmax(smax, __shfl_xor(smax, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kReduceThreads / 64; w++) m = __builtin_fmax(m, red[w]);
        partial[blockIdx.x] = m;
    }
}

// One block: reduce the partial maxima, then set the step size and advance
// the accumulated time.  scalars = [smax, dt, t].
__global__ void __launch_bounds__(kReduceThreads) k_step_begin(const double *__restrict__ partial, int nblocks,
                                                               double cfl, double dt_fixed, double dxmin,
                                                               double *__restrict__ scalars)
{
    __shared__ double red[kReduceThreads / 64];
    double m = 0.0;
    if (partial)
        for (int b = threadIdx.x; b < nblocks; b += blockDim.x) m = __builtin_fmax(m, partial[b]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = __builtin_fmax(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = red[0];
        for (int w = 1; w < kReduceThreads / 64; w++) s = __builtin_fmax(s, red[w]);
        double dt = dt_fixed;
        if (partial) {
            scalars[0] = s;
            if (cfl > 0.0) dt = cfl * dxmin / s;
        }
        scalars[1] = dt;
        scalars[2] += dt;
    }
}

// The step size the last step took (scalars[1]) into the caller's device
// word (mfc_rk3_step's dt_used_dev).
__global__ void k_copy_dt(const double *__restrict__ scalars, double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *out = scalars[1];
}

__global__ void k_set_scalars(double *scalars, int *flag, int what)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        if (what & 1) {
            scalars[0] = scalars[1] = scalars[2] = scalars[3] = 0.0;
        }
        if (what & 2) *flag = 0;
    }
}

// ---------------------------------------------------------------- helpers
int validate(const mfc_grid_desc *d)
{
    if (!d) return fail(MFC_E_ARG, "desc is NULL");
    if (d->ndim < 1 || d->ndim > 3) return fail(MFC_E_ARG, "ndim must be 1, 2 or 3");
    if (d->num_fluids != 2) return fail(MFC_E_UNSUPPORTED, "num_fluids must be 2");
    for (int k = 0; k < d->ndim; k++) {
        if (d->n[k] < 3) return fail(MFC_E_ARG, "n must be >= 3 on active dimensions");
        if (d->n[k] > (1 << 20)) return fail(MFC_E_ARG, "n too large");
        if (!(d->hi[k] > d->lo[k]) || !std::isfinite(d->hi[k] - d->lo[k])) return fail(MFC_E_ARG, "hi must exceed lo");
        int a = d->bc[2 * k], b = d->bc[2 * k + 1];
        auto known = [](int x) { return x == MFC_BC_EXTRAP || x == MFC_BC_PERIODIC || x == MFC_BC_CHARACTERISTIC; };
        if (!known(a) || !known(b)) return fail(MFC_E_ARG, "unknown boundary condition");
        if (a == MFC_BC_CHARACTERISTIC || b == MFC_BC_CHARACTERISTIC) {
            if (d->model != MFC_MODEL_ALLAIRE)
                return fail(MFC_E_UNSUPPORTED, "characteristic boundaries take the Allaire model");
            // the boundary pass of the other kernels recomputes the normal
            // terms with WENO5, the split kernels keep their own (routed) ones
            if (d->recon == MFC_RECON_LEARNED && d->kernel != MFC_KERNEL_SPLIT)
                return fail(MFC_E_UNSUPPORTED, "characteristic boundaries with the learned routing need the split kernel");
        }
        if ((a == MFC_BC_PERIODIC) != (b == MFC_BC_PERIODIC))
            return fail(MFC_E_ARG, "periodic must be set on both faces of a dimension");
    }
    for (int f = 0; f < 2; f++) {
        if (!(d->gamma[f] > 1.0) || !std::isfinite(d->gamma[f])) return fail(MFC_E_ARG, "gamma must be > 1");
        if (!(d->pi_inf[f] >= 0.0) || !std::isfinite(d->pi_inf[f])) return fail(MFC_E_ARG, "pi_inf must be >= 0");
    }
    if (!(d->weno_eps > 0.0)) return fail(MFC_E_ARG, "weno_eps must be > 0");
    if (d->precision != MFC_FP64 && d->precision != MFC_FP32_MIXED) return fail(MFC_E_ARG, "unknown precision");
    if (d->recon != MFC_RECON_WENO5 && d->recon != MFC_RECON_LEARNED && d->recon != MFC_RECON_WENO3 &&
        d->recon != MFC_RECON_FIRST_ORDER)
        return fail(MFC_E_ARG, "unknown recon");
    if (d->model != MFC_MODEL_ALLAIRE && d->model != MFC_MODEL_KAPILA) return fail(MFC_E_ARG, "unknown model");
    if (d->kernel != MFC_KERNEL_FUSED && d->kernel != MFC_KERNEL_STAGED && d->kernel != MFC_KERNEL_SPLIT)
        return fail(MFC_E_ARG, "unknown kernel");
    if (d->precision == MFC_FP32_MIXED && d->kernel == MFC_KERNEL_STAGED)
        return fail(MFC_E_UNSUPPORTED, "the staged path is FP64 only");
    if (d->kernel == MFC_KERNEL_SPLIT && d->ndim != 3) return fail(MFC_E_UNSUPPORTED, "the split path is 3D only");
    if (d->recon == MFC_RECON_LEARNED && d->kernel == MFC_KERNEL_STAGED)
        return fail(MFC_E_UNSUPPORTED, "the staged path reconstructs with WENO5 only");
    for (int k = 0; k < d->ndim; k++) {
        const double *f = d->faces[k];
        if (!f) continue;
        if (d->kernel == MFC_KERNEL_STAGED)
            return fail(MFC_E_UNSUPPORTED, "non-uniform cells need the fused or the split kernel");
        if (d->recon != MFC_RECON_WENO5 && d->recon != MFC_RECON_FIRST_ORDER)
            return fail(MFC_E_UNSUPPORTED, "non-uniform cells take WENO5 or first order");
        for (int i = 0; i < d->n[k]; i++)
            if (!(f[i + 1] > f[i]) || !std::isfinite(f[i]) || !std::isfinite(f[i + 1]))
                return fail(MFC_E_ARG, "face coordinates must be finite and strictly increasing");
    }
    return MFC_OK;
}

bool bad_handle(const mfc_grid *h) { return h == nullptr; }

int set_device(mfc_grid *h)
{
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess) return fail(MFC_E_HIP, "hipGetDevice failed");
    if (cur != h->device) return fail(MFC_E_ARG, "handle belongs to another device than the current one");
    return MFC_OK;
}

template <class F>
int by_ndim(int ndim, F f)
{
    switch (ndim) {
    case 1: return f(std::integral_constant<int, 1>{});
    case 2: return f(std::integral_constant<int, 2>{});
    default: return f(std::integral_constant<int, 3>{});
    }
}

int rhs_dispatch(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt,
                 const double *dt_dev, hipStream_t s, double cfl = 0.0, double *zmax = nullptr)
{
    int st;
    if (h->desc.kernel == MFC_KERNEL_STAGED) st = launch_rhs_staged(h, q, q0, out, mode, dt, dt_dev, s);
    else if (h->desc.kernel == MFC_KERNEL_SPLIT) st = launch_rhs_split(h, q, q0, out, mode, dt, dt_dev, s, cfl, zmax);
    else st = launch_rhs_fused(h, q, q0, out, mode, dt, dt_dev, s);
    // with characteristic faces, a wave-speed-reducing last stage leaves the
    // z faces' cells to the boundary pass, whose maxima follow the z kernel's
    if (st == MFC_OK && has_cbc(h))
        st = launch_cbc(h, q, out, mode, dt, dt_dev, s,
                        zmax ? zmax + split_z_partials(h->g, h->desc.precision == MFC_FP32_MIXED) : nullptr);
    return st;
}

bool is_fp32(const mfc_grid *h) { return h->desc.precision == MFC_FP32_MIXED; }

template <class T>
void fill_ghosts_t(mfc_grid *h, T *q, hipStream_t s)
{
    const Grid &g = h->g;
    int64_t start[4] = {0, 0, 0, 0};
    for (int d = 0; d < 3; d++) {
        int o1 = d == 0 ? 1 : 0, o2 = d == 2 ? 1 : 2;
        start[d + 1] = start[d] + (d < g.ndim ? (int64_t)2 * NG * g.n[o1] * g.n[o2] * h->nvar : 0);
    }
    hipLaunchKernelGGL((k_ghosts<T>), dim3(blocks_for(start[3])), dim3(kThreads), 0, s, g, q, h->nvar, start[1],
                       start[2], start[3]);
}

}  // namespace

void launch_step_begin(mfc_grid *h, const double *partial, int nblocks, double cfl, double dt, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_begin, dim3(1), dim3(kReduceThreads), 0, s, partial, nblocks, cfl, dt, h->g.dxmin,
                       h->scalars);
}

namespace {

int fill_ghosts(mfc_grid *h, void *q, hipStream_t s)
{
    if (is_fp32(h)) fill_ghosts_t<float>(h, (float *)q, s);
    else fill_ghosts_t<double>(h, (double *)q, s);
    return hip_status(hipGetLastError(), "ghost fill launch");
}

template <class T>
void wavespeed_t(mfc_grid *h, const T *q, hipStream_t s)
{
    by_ndim(h->g.ndim, [&](auto nd) {
        hipLaunchKernelGGL((k_wavespeed<decltype(nd)::value, T>), dim3(kReduceBlocks), dim3(kReduceThreads), 0, s,
                           h->g, q, h->partial, h->flag);
        return 0;
    });
}

int wavespeed(mfc_grid *h, const void *q, hipStream_t s)
{
    if (is_fp32(h)) wavespeed_t<float>(h, (const float *)q, s);
    else wavespeed_t<double>(h, (const double *)q, s);
    return hip_status(hipGetLastError(), "wave-speed launch");
}

int64_t elem_bytes(const mfc_grid *h) { return is_fp32(h) ? 4 : 8; }
int64_t state_bytes(const mfc_grid *h) { return (int64_t)h->nvar * h->cells_padded * elem_bytes(h); }

}  // namespace

int validate_desc(const mfc_grid_desc *d) { return validate(d); }

}  // namespace mfc

using namespace mfc;

extern "C" {

const char *mfc_strerror(int status)
{
    switch (status) {
    case MFC_OK: return "ok";
    case MFC_E_ARG: return "invalid argument";
    case MFC_E_NOMEM: return "out of device memory";
    case MFC_E_HIP: return "HIP runtime error";
    case MFC_E_NONPHYSICAL: return "non-physical state (rho <= 0, c^2 <= 0 or non-finite)";
    case MFC_E_UNSUPPORTED: return "unsupported configuration";
    default: return "unknown status";
    }
}

const char *mfc_last_error_detail(void) { return g_detail; }

int mfc_free_grid(mfc_grid *h)
{
    if (!h) return MFC_OK;
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)h->stage_a, (void *)h->stage_b, (void *)h->prim, (void *)h->recp, (void *)h->recm,
                    (void *)h->faces, (void *)h->lxy, (void *)h->partial, (void *)h->scalars, (void *)h->flag,
                    (void *)h->mlp, h->cbc_fv})
        if (p) (void)hipFree(p);
    for (auto &ev : h->ev)
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    free_stretch_tables(h);
    delete h;
    return MFC_OK;
}

int mfc_init_grid(const mfc_grid_desc *desc, mfc_grid **out)
{
    if (!out) return fail(MFC_E_ARG, "out is NULL");
    *out = nullptr;
    int st = validate(desc);
    if (st != MFC_OK) return st;
    mfc_grid *h = new (std::nothrow) mfc_grid();
    if (!h) return fail(MFC_E_NOMEM, "host allocation failed");
    h->desc = *desc;
    Grid &g = h->g;
    make_grid(*desc, g);
    h->nvar = 4 + desc->ndim;
    for (int d = desc->ndim; d < 3; d++) {
        h->desc.n[d] = 1;
        h->desc.bc[2 * d] = h->desc.bc[2 * d + 1] = MFC_BC_EXTRAP;
    }
    for (int d = 0; d < 3; d++) h->desc.faces[d] = nullptr;   // the caller's arrays are not kept
    h->cells_padded = g.vstride;
    h->cells = (int64_t)g.n[0] * g.n[1] * g.n[2];
    if (hipGetDevice(&h->device) != hipSuccess ||
        hipDeviceGetAttribute(&h->cu_count, hipDeviceAttributeMultiprocessorCount, h->device) != hipSuccess ||
        h->cu_count <= 0) {
        delete h;
        return fail(MFC_E_HIP, "device query failed");
    }

    if (g.stretched && (st = build_stretch_tables(h, desc)) != MFC_OK) {
        free_stretch_tables(h);
        delete h;
        return st;
    }
    int64_t sb = state_bytes(h);
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, int64_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, (size_t)bytes);
    };
    alloc(&h->stage_a, sb);
    alloc(&h->stage_b, sb);
    if (desc->kernel == MFC_KERNEL_STAGED) {
        alloc((void **)&h->prim, sb);
        alloc((void **)&h->recp, sb);
        alloc((void **)&h->recm, sb);
        alloc((void **)&h->faces, (int64_t)3 * (h->nvar + 1) * h->cells_padded * 8);
    }
    if (desc->kernel == MFC_KERNEL_SPLIT) {
        alloc((void **)&h->lxy, (int64_t)h->nvar * h->cells_padded * elem_bytes(h));
        // characteristic faces: the x+y kernel applies the x and y faces
        // itself; the z kernel keeps the normal terms of the z faces' cells
        // (8 values per cell) for the boundary pass
        int64_t words = 0;
        for (int f = 0; f < 2 * g.ndim; f++) {
            if (g.bc[f] != MFC_BC_CHARACTERISTIC) continue;
            g.cbc_mask |= 1 << f;
            if (f < 4) continue;
            g.cbc_off[f] = words;
            words += 8 * (int64_t)g.n[0] * g.n[1];
        }
        if (words) alloc(&h->cbc_fv, words * elem_bytes(h));
        g.cbc_fv = h->cbc_fv;
    }
    h->partial_len = std::max<int64_t>(
        kReduceBlocks,
        desc->ndim == 3 ? std::max(split_xy_blocks(g), split_z_partials(g, is_fp32(h)) + cbc_stored_blocks(g)) : 0);
    alloc((void **)&h->partial, h->partial_len * 8);
    alloc((void **)&h->scalars, 4 * 8);
    alloc((void **)&h->flag, 8);
    if (e != hipSuccess) {
        mfc_free_grid(h);
        return hip_status(e, "scratch allocation");
    }
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, 0, h->scalars, h->flag, 3);
    e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mfc_free_grid(h);
        return hip_status(e, "initialisation");
    }
    *out = h;
    return MFC_OK;
}

int mfc_state_layout(const mfc_grid *h, int64_t *nvar, int64_t padded[3], int64_t *elem_bytes)
{
    if (bad_handle(h)) return fail(MFC_E_ARG, "handle is NULL");
    if (nvar) *nvar = h->nvar;
    if (padded)
        for (int d = 0; d < 3; d++) padded[d] = h->g.p[d];
    if (elem_bytes) *elem_bytes = mfc::elem_bytes(h);
    return MFC_OK;
}

int mfc_prim_to_cons(mfc_grid *h, const void *w, void *q, void *stream)
{
    if (bad_handle(h) || !w || !q) return fail(MFC_E_ARG, "null argument");
    if (w == q) return fail(MFC_E_ARG, "w and q must be distinct");
    int st = set_device(h);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    by_ndim(h->g.ndim, [&](auto nd) {
        constexpr int ND = decltype(nd)::value;
        if (is_fp32(h))
            hipLaunchKernelGGL((k_p2c<ND, float>), dim3(blocks_for(h->cells_padded)), dim3(kThreads), 0, s, h->g,
                               (const float *)w, (float *)q);
        else
            hipLaunchKernelGGL((k_p2c<ND, double>), dim3(blocks_for(h->cells_padded)), dim3(kThreads), 0, s, h->g,
                               (const double *)w, (double *)q);
        return 0;
    });
    return hip_status(hipGetLastError(), "prim_to_cons launch");
}

int mfc_cons_to_prim(mfc_grid *h, const void *q, void *w, void *stream)
{
    if (bad_handle(h) || !w || !q) return fail(MFC_E_ARG, "null argument");
    if (w == q) return fail(MFC_E_ARG, "w and q must be distinct");
    int st = set_device(h);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    by_ndim(h->g.ndim, [&](auto nd) {
        constexpr int ND = decltype(nd)::value;
        if (is_fp32(h))
            hipLaunchKernelGGL((k_c2p<ND, float>), dim3(blocks_for(h->cells_padded)), dim3(kThreads), 0, s, h->g,
                               (const float *)q, (float *)w, h->flag);
        else
            hipLaunchKernelGGL((k_c2p<ND, double>), dim3(blocks_for(h->cells_padded)), dim3(kThreads), 0, s, h->g,
                               (const double *)q, (double *)w, h->flag);
        return 0;
    });
    return hip_status(hipGetLastError(), "cons_to_prim launch");
}

int mfc_fill_ghosts(mfc_grid *h, void *q, void *stream)
{
    if (bad_handle(h) || !q) return fail(MFC_E_ARG, "null argument");
    int st = set_device(h);
    if (st) return st;
    return fill_ghosts(h, q, (hipStream_t)stream);
}

int mfc_rhs(mfc_grid *h, const void *q, void *rhs, void *stream)
{
    if (bad_handle(h) || !q || !rhs) return fail(MFC_E_ARG, "null argument");
    if (q == rhs) return fail(MFC_E_ARG, "q and rhs must be distinct");
    int st = set_device(h);
    if (st) return st;
    return rhs_dispatch(h, q, nullptr, rhs, 0, 0.0, nullptr, (hipStream_t)stream);
}

int mfc_max_wavespeed(mfc_grid *h, const void *q, double *smax_host, void *stream)
{
    if (bad_handle(h) || !q || !smax_host) return fail(MFC_E_ARG, "null argument");
    int st = set_device(h);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    st = wavespeed(h, q, s);
    if (st) return st;
    double *partial = (double *)std::malloc(kReduceBlocks * sizeof(double));
    int flag = 0;
    hipError_t e = hipMemcpyAsync(partial, h->partial, kReduceBlocks * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        std::free(partial);
        return hip_status(e, "wave-speed readback");
    }
    double m = 0.0;
    for (int b = 0; b < kReduceBlocks; b++) m = std::fmax(m, partial[b]);
    std::free(partial);
    *smax_host = m;
    if (flag & 2) {
        hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, h->scalars, h->flag, 2);
        return fail(MFC_E_NONPHYSICAL, "non-physical interior cell in the wave-speed reduction");
    }
    return MFC_OK;
}

namespace {

// Split path, CFL steps of one run: the z pass of a step's last stage can
// reduce the wave speeds of q^{n+1} as it writes it (the x+y pass of the
// next step's first stage would reduce the same values to the same
// maxima), so that the next step's size is known before its first stage and
// that stage's x+y pass forms its part of the combination.  With
// characteristic faces the boundary pass, which changes the z faces' cells
// after the z pass, reduces those cells itself.
bool carries_wavespeed(const mfc_grid *h, double cfl)
{
    return cfl > 0.0 && h->desc.kernel == MFC_KERNEL_SPLIT;
}

// Number of wave-speed maxima a carrying last stage leaves in h->partial.
int64_t carried_partials(const mfc_grid *h)
{
    return split_z_partials(h->g, is_fp32(h)) + (has_cbc(h) ? cbc_stored_blocks(h->g) : 0);
}

// One SSP-RK3 step.  carried_in: the wave-speed partials of q^n are in
// h->partial (written by the previous step's last stage); carry_out: have
// this step's last stage write those of q^{n+1}.
int rk3_step_launches(mfc_grid *h, void *q, double cfl, double dt, double *dt_used_dev, hipStream_t s,
                      bool carried_in, bool carry_out);

int rk3_step(mfc_grid *h, void *q, double cfl, double dt, double *dt_used_dev, hipStream_t s, bool carried_in,
             bool carry_out)
{
    // with a timing stride, only every stride-th step's launches are timed
    h->timing_skip = h->timing && (h->timing_step++ % h->timing_stride) != 0;
    const int st = rk3_step_launches(h, q, cfl, dt, dt_used_dev, s, carried_in, carry_out);
    h->timing_skip = false;
    return st;
}

int rk3_step_launches(mfc_grid *h, void *q, double cfl, double dt, double *dt_used_dev, hipStream_t s,
                      bool carried_in, bool carry_out)
{
    int st = MFC_OK;
    void *A = h->stage_a, *B = h->stage_b;
    const double *dt_dev = h->scalars + 1;
    // the split kernels read boundary neighbours through the boundary
    // condition itself (the values a ghost fill writes) and need no fill
    const bool fill = h->desc.kernel != MFC_KERNEL_SPLIT;
    if (fill && (st = fill_ghosts(h, q, s))) return st;
    if (carried_in) {
        launch_step_begin(h, h->partial, (int)carried_partials(h), cfl, 0.0, s);
        if ((st = rhs_dispatch(h, q, q, A, 1, 0.0, dt_dev, s))) return st;
    } else if (h->desc.kernel == MFC_KERNEL_SPLIT && cfl > 0.0) {
        // the x+y pass of the first stage reduces the wave speeds of q^n and
        // the step size is set before its z pass, the first to use it
        if ((st = rhs_dispatch(h, q, q, A, 1, 0.0, dt_dev, s, cfl))) return st;
    } else {
        if (cfl > 0.0) {
            if ((st = wavespeed(h, q, s))) return st;
            launch_step_begin(h, h->partial, kReduceBlocks, cfl, 0.0, s);
        } else {
            launch_step_begin(h, nullptr, 0, 0.0, dt, s);
        }
        if ((st = rhs_dispatch(h, q, q, A, 1, 0.0, dt_dev, s))) return st;
    }
    if (fill && (st = fill_ghosts(h, A, s))) return st;
    if ((st = rhs_dispatch(h, A, q, B, 2, 0.0, dt_dev, s))) return st;
    if (fill && (st = fill_ghosts(h, B, s))) return st;
    if ((st = rhs_dispatch(h, B, q, q, 3, 0.0, dt_dev, s, 0.0, carry_out ? h->partial : nullptr))) return st;
    if (dt_used_dev) hipLaunchKernelGGL(k_copy_dt, dim3(1), dim3(64), 0, s, h->scalars, dt_used_dev);
    return hip_status(hipGetLastError(), "rk3 step launch");
}

int check_step_args(mfc_grid *h, const void *q, double cfl, double dt)
{
    if (bad_handle(h) || !q) return fail(MFC_E_ARG, "null argument");
    if (!(cfl > 0.0) && !(dt > 0.0)) return fail(MFC_E_ARG, "need cfl > 0 or dt > 0");
    if (!std::isfinite(cfl) || !std::isfinite(dt)) return fail(MFC_E_ARG, "cfl and dt must be finite");
    return set_device(h);
}

}  // namespace

int mfc_rk3_step(mfc_grid *h, void *q, double cfl, double dt, double *dt_used_dev, void *stream)
{
    int st = check_step_args(h, q, cfl, dt);
    if (st) return st;
    return rk3_step(h, q, cfl, dt, dt_used_dev, (hipStream_t)stream, false, false);
}

int mfc_run(mfc_grid *h, void *q, int nsteps, double cfl, double dt, void *stream)
{
    if (nsteps < 0) return fail(MFC_E_ARG, "nsteps must be >= 0");
    if (nsteps == 0) return MFC_OK;
    int st = check_step_args(h, q, cfl, dt);
    if (st) return st;
    const bool carry = carries_wavespeed(h, cfl);
    for (int n = 0; n < nsteps && st == MFC_OK; n++)
        st = rk3_step(h, q, cfl, dt, nullptr, (hipStream_t)stream, carry && n > 0, carry && n + 1 < nsteps);
    return st;
}

int mfc_time(mfc_grid *h, double *t_host, double *last_dt_host, void *stream)
{
    if (bad_handle(h)) return fail(MFC_E_ARG, "handle is NULL");
    int st = set_device(h);
    if (st) return st;
    double sc[4];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(sc, h->scalars, sizeof sc, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "time readback");
    if (t_host) *t_host = sc[2];
    if (last_dt_host) *last_dt_host = sc[1];
    return MFC_OK;
}

int mfc_reset_time(mfc_grid *h, void *stream)
{
    if (bad_handle(h)) return fail(MFC_E_ARG, "handle is NULL");
    int st = set_device(h);
    if (st) return st;
    hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, (hipStream_t)stream, h->scalars, h->flag, 1);
    return hip_status(hipGetLastError(), "reset time");
}

int mfc_check(mfc_grid *h, void *stream)
{
    if (bad_handle(h)) return fail(MFC_E_ARG, "handle is NULL");
    int st = set_device(h);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    int flag = 0;
    hipError_t e = hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "flag readback");
    if (flag) {
        hipLaunchKernelGGL(k_set_scalars, dim3(1), dim3(64), 0, s, h->scalars, h->flag, 2);
        return fail(MFC_E_NONPHYSICAL, "a kernel met a non-physical cell");
    }
    return MFC_OK;
}

int mfc_set_kernel_timing(mfc_grid *h, int enable)
{
    if (bad_handle(h)) return fail(MFC_E_ARG, "handle is NULL");
    if (enable < 0) return fail(MFC_E_ARG, "enable must be >= 0");
    h->timing = enable != 0;   // what was recorded stays until mfc_kernel_time reads it
    h->timing_stride = enable > 1 ? enable : 1;
    h->timing_step = 0;
    return MFC_OK;
}

int mfc_kernel_time(mfc_grid *h, int slot, double *ms_total, int64_t *launches)
{
    if (bad_handle(h) || !ms_total || !launches) return fail(MFC_E_ARG, "null argument");
    if (slot < 0 || slot > 1) return fail(MFC_E_ARG, "slot must be 0 or 1");
    const auto &ev = h->ev[slot];
    double total = 0.0;
    for (size_t p = 0; p + 1 < h->ev_used[slot]; p += 2) {
        hipError_t e = hipEventSynchronize(ev[p + 1]);
        if (e != hipSuccess) return hip_status(e, "event sync");
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, ev[p], ev[p + 1]);
        if (e != hipSuccess) return hip_status(e, "event elapsed time");
        total += ms;
    }
    *ms_total = total;
    *launches = (int64_t)(h->ev_used[slot] / 2);
    h->ev_used[slot] = 0;
    return MFC_OK;
}

}  // extern "C"
