// Learned smoothness indicator (project extension beside Sec. 3.2): harvest
// of training samples from a solver state, training of the perceptron of
// mlp.h with the project's own bf16 matrix-core forward and backward kernels
// (FP32 master weights, mean binary cross-entropy, Adam), batched inference,
// and the handle call that installs a trained network for the routed
// reconstruction.
//
//   k_harvest     one thread per interior (cell, direction): the 15 inputs
//                 and the label "every variable keeps its WENO5 weights
//                 within 0.01 of the ideal ones on both faces";
//   k_mlp_grad    forward + backward over a batch; each wavefront walks
//                 16-sample tiles, keeps the weight-gradient tiles in MFMA
//                 accumulators and the bias/W3 gradients in registers; a
//                 workgroup writes one partial sum of all 1601 gradients and
//                 the loss;
//   k_mlp_reduce  sums the partials in a fixed order (deterministic);
//   k_adam        one thread per parameter;
//   k_mlp_infer   P(smooth) of a list of samples.
#include <cmath>
#include <new>

#include "internal.h"
#include "mlp.h"

struct mfc_trainer {
    int64_t max_batch = 0;
    int blocks = 0;
    int device = 0;
    float *w = nullptr, *m = nullptr, *v = nullptr;  // master weights, Adam moments
    float *grad = nullptr;                           // [NPARAM + 1]: gradients, loss
    float *partial = nullptr;                        // [blocks][NPARAM + 1]
    int64_t step = 0;                                // Adam steps taken
    bool have_grad = false;
};

namespace mfc {
namespace {

using namespace mlp;
constexpr int kThreads = 256, kWaves = kThreads / 64;
constexpr int NP1 = NPARAM + 1;

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Largest |omega_r - d_r| of WENO5-JS over the three stencils and both faces
// of the 5-cell stencil s (the weights of Sec. 3.2 with the Jiang-Shu
// smoothness indicators, written in the divided differences of the stencil).
__device__ double weno_deviation(const double *s, double eps)
{
#pragma clang fp contract(off)
    const double dm2 = s[1] - s[0], dm1 = s[2] - s[1], d0 = s[3] - s[2], d1 = s[4] - s[3];
    double beta[3];
    beta[0] = (10.0 / 3.0) * dm1 * dm1 - (11.0 / 3.0) * dm1 * dm2 + (4.0 / 3.0) * dm2 * dm2;
    beta[1] = (4.0 / 3.0) * d0 * d0 - (5.0 / 3.0) * d0 * dm1 + (4.0 / 3.0) * dm1 * dm1;
    beta[2] = (10.0 / 3.0) * d0 * d0 - (11.0 / 3.0) * d0 * d1 + (4.0 / 3.0) * d1 * d1;
    const double dp[3] = {0.1, 0.6, 0.3}, dmn[3] = {0.3, 0.6, 0.1};
    double ap[3], am[3], sp = 0.0, sm = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        const double e = (eps + beta[r]) * (eps + beta[r]);
        ap[r] = dp[r] / e;
        am[r] = dmn[r] / e;
        sp += ap[r];
        sm += am[r];
    }
    double dev = 0.0;
#pragma unroll
    for (int r = 0; r < 3; r++) {
        dev = fmax(dev, fabs(ap[r] / sp - dp[r]));
        dev = fmax(dev, fabs(am[r] / sm - dmn[r]));
    }
    return dev;
}

template <int NDIM>
__global__ void __launch_bounds__(kThreads)
    k_harvest(Grid g, const double *__restrict__ q, uint16_t *__restrict__ X, uint8_t *__restrict__ Y,
              double *__restrict__ D, double sqrt_eps, double threshold, int64_t cells)
{
    constexpr int NV = 4 + NDIM;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cells * NDIM) return;
    const int d = (int)(t / cells);
    const int64_t c = t % cells;
    int ijk[3] = {(int)(c % g.n[0]), (int)((c / g.n[0]) % g.n[1]), (int)(c / ((int64_t)g.n[0] * g.n[1]))};
    double w[5][NV];
#pragma unroll
    for (int p = 0; p < 5; p++) {
        int a[3] = {ijk[0], ijk[1], ijk[2]};
        a[d] += p - 2;
        const int64_t o = (int64_t)(a[2] + g.off[2]) * g.stride[2] + (int64_t)(a[1] + g.off[1]) * g.stride[1] +
                          (a[0] + g.off[0]);
        double qc[NV];
#pragma unroll
        for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + o];
        (void)cons_to_prim<NDIM, double>(g, qc, w[p]);
    }
    double al[5], rh[5], pr[5];
#pragma unroll
    for (int p = 0; p < 5; p++) {
        al[p] = w[p][NV - 1];
        rh[p] = w[p][0] + w[p][1];
        pr[p] = w[p][NV - 2];
    }
    uint16_t f[16];
    features<double>(al, rh, pr, sqrt_eps, f);
    uint4 *xo = (uint4 *)(X + t * 16);
    const uint32_t *f32 = (const uint32_t *)f;
    xo[0] = make_uint4(f32[0], f32[1], f32[2], f32[3]);
    xo[1] = make_uint4(f32[4], f32[5], f32[6], f32[7]);
    double dev = 0.0;
#pragma unroll
    for (int v = 0; v < NV; v++) {
        const double s[5] = {w[0][v], w[1][v], w[2][v], w[3][v], w[4][v]};
        dev = fmax(dev, weno_deviation(s, g.eps));
    }
    Y[t] = dev < threshold ? 1 : 0;
    if (D) D[t] = dev;
}

__global__ void __launch_bounds__(kThreads)
    k_mlp_grad(const float *__restrict__ w, const uint16_t *__restrict__ X, const uint8_t *__restrict__ Y,
               const int *__restrict__ index, int64_t batch, float inv_n, float *__restrict__ partial)
{
    __shared__ __align__(16) Params P;
    __shared__ __align__(16) ParamsT PT;
    __shared__ __align__(16) uint16_t sx[kWaves][16 * 16];   // X tile [sample][feature]
    __shared__ __align__(16) uint16_t sh1[kWaves][16 * NH];  // H1 tile [sample][unit]
    __shared__ __align__(16) uint16_t sd2[kWaves][16 * NH];  // dZ2 tile
    __shared__ __align__(16) uint16_t sd1[kWaves][16 * NH];  // dZ1 tile
    __shared__ float red[kWaves][NP1];
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, g = lane >> 4, s = lane & 15;
    stage_params(P, &PT, w, tid, kThreads);
    __syncthreads();

    f4 aw1[2], aw2[2][2];
#pragma unroll
    for (int b = 0; b < 2; b++) {
        aw1[b] = f4{0.f, 0.f, 0.f, 0.f};
        aw2[b][0] = aw2[b][1] = f4{0.f, 0.f, 0.f, 0.f};
    }
    float dw3[8], db2[8], db1[8], db3 = 0.f, loss = 0.f;
#pragma unroll
    for (int q = 0; q < 8; q++) dw3[q] = db2[q] = db1[q] = 0.f;

    const int64_t ntiles = (batch + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
        const int64_t smp = tile * 16 + s;
        const bool valid = smp < batch;
        const int64_t row = valid ? (index ? (int64_t)index[smp] : smp) : 0;
        s4 xb = *(const s4 *)(X + row * 16 + 4 * g);
        if (!valid) xb = s4{0, 0, 0, 0};
        Fwd F;
        forward_tile(P, xb, lane, F);
        const float y = valid ? float(Y[row]) : 0.f;
        const float prob = 1.0f / (1.0f + __expf(-F.z));
        const float dz = valid ? (prob - y) * inv_n : 0.f;
        if (g == 0) {
            db3 += dz;
            if (valid) loss += fmaxf(F.z, 0.f) - F.z * y + log1pf(__expf(-fabsf(F.z)));
        }
        float dz2[8];
        uint16_t dz2_bits[8];
        bf8 dz2b;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int u = 16 * (q / 4) + 4 * g + (q % 4);
            dw3[q] += dz * F.h2[q];
            dz2[q] = P.w3[u] * dz * gelu_grad(F.z2[q]);
            db2[q] += dz2[q];
            dz2_bits[q] = bf16_bits(dz2[q]);
            dz2b[q] = as_bf16(dz2_bits[q]);
        }
        float dz1[8];
#pragma unroll
        for (int b = 0; b < 2; b++) {
            f4 c = f4{0.f, 0.f, 0.f, 0.f};
            c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(PT.a2t[b][lane], dz2b, c, 0, 0, 0);
#pragma unroll
            for (int t = 0; t < 4; t++) {
                dz1[4 * b + t] = c[t] * gelu_grad(F.z1[4 * b + t]);
                db1[4 * b + t] += dz1[4 * b + t];
            }
        }
        // stage the tiles [sample][unit] for the sample-contracted products
        *(s4 *)&sx[wave][s * 16 + 4 * g] = xb;
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int u = unit(g, q);
            sh1[wave][s * NH + u] = F.h1_bits[q];
            sd2[wave][s * NH + u] = dz2_bits[q];
            sd1[wave][s * NH + u] = bf16_bits(dz1[q]);
        }
        wave_sync();
        // dW1 [16 f x 32 u] += X^T dZ1, dW2 [32 in x 32 out] += H1^T dZ2 (k = samples)
        s4 ax;
#pragma unroll
        for (int t = 0; t < 4; t++) ax[t] = (short)sx[wave][(4 * g + t) * 16 + s];
#pragma unroll
        for (int bu = 0; bu < 2; bu++) {
            s4 bz;
#pragma unroll
            for (int t = 0; t < 4; t++) bz[t] = (short)sd1[wave][(4 * g + t) * NH + 16 * bu + s];
            aw1[bu] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ax, bz, aw1[bu], 0, 0, 0);
        }
#pragma unroll
        for (int bi = 0; bi < 2; bi++) {
            s4 ah;
#pragma unroll
            for (int t = 0; t < 4; t++) ah[t] = (short)sh1[wave][(4 * g + t) * NH + 16 * bi + s];
#pragma unroll
            for (int bo = 0; bo < 2; bo++) {
                s4 bz;
#pragma unroll
                for (int t = 0; t < 4; t++) bz[t] = (short)sd2[wave][(4 * g + t) * NH + 16 * bo + s];
                aw2[bi][bo] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(ah, bz, aw2[bi][bo], 0, 0, 0);
            }
        }
        wave_sync();
    }

    // wavefront partials -> red[wave][flat index]
    float *r = red[wave];
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int t = 0; t < 4; t++) {
            const int f = 4 * g + t;
            if (f < NIN) r[OW1 + f * NH + 16 * b + s] = aw1[b][t];
#pragma unroll
            for (int bo = 0; bo < 2; bo++) r[OW2 + (16 * b + 4 * g + t) * NH + 16 * bo + s] = aw2[b][bo][t];
        }
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            dw3[q] += __shfl_xor(dw3[q], o, 64);
            db2[q] += __shfl_xor(db2[q], o, 64);
            db1[q] += __shfl_xor(db1[q], o, 64);
        }
        db3 += __shfl_xor(db3, o, 64);
        loss += __shfl_xor(loss, o, 64);
    }
    if (s == 0) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int u = 16 * (q / 4) + 4 * g + (q % 4);
            r[OW3 + u] = dw3[q];
            r[OB2 + u] = db2[q];
            r[OB1 + u] = db1[q];
        }
        if (g == 0) {
            r[OB3] = db3;
            r[NPARAM] = loss;
        }
    }
    __syncthreads();
    for (int e = tid; e < NP1; e += kThreads)
        partial[(int64_t)blockIdx.x * NP1 + e] = (red[0][e] + red[1][e]) + (red[2][e] + red[3][e]);
}

__global__ void k_mlp_reduce(const float *__restrict__ partial, int blocks, float *__restrict__ out, float inv_n)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NP1) return;
    float acc = 0.f;
    for (int b = 0; b < blocks; b++) acc += partial[(int64_t)b * NP1 + e];
    out[e] = e == NPARAM ? acc * inv_n : acc;   // the loss is a mean
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v,
                       const float *__restrict__ grad, float lr, float b1, float b2, float c1, float c2, float eps)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= NPARAM) return;
    const float gr = grad[e];
    const float mm = b1 * m[e] + (1.0f - b1) * gr;
    const float vv = b2 * v[e] + (1.0f - b2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    w[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

__global__ void __launch_bounds__(kThreads)
    k_mlp_infer(const float *__restrict__ w, const uint16_t *__restrict__ X, int64_t n, float *__restrict__ prob)
{
    __shared__ __align__(16) Params P;
    const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64, g = lane >> 4, s = lane & 15;
    stage_params(P, nullptr, w, tid, kThreads);
    __syncthreads();
    const int64_t ntiles = (n + 15) / 16;
    for (int64_t tile = (int64_t)blockIdx.x * kWaves + wave; tile < ntiles; tile += (int64_t)gridDim.x * kWaves) {
        const int64_t smp = tile * 16 + s;
        s4 xb = smp < n ? *(const s4 *)(X + smp * 16 + 4 * g) : s4{0, 0, 0, 0};
        const float z = logit_tile(P, xb, lane);
        if (g == 0 && smp < n) prob[smp] = 1.0f / (1.0f + __expf(-z));
    }
}

}  // namespace
}  // namespace mfc

using namespace mfc;

extern "C" {

int mfc_harvest(mfc_grid *h, void *q, uint16_t *features, uint8_t *labels, double *maxdev, void *stream)
{
    if (!h || !q || !features || !labels) return fail(MFC_E_ARG, "null argument");
    if (h->desc.precision != MFC_FP64) return fail(MFC_E_UNSUPPORTED, "harvest reads FP64 states");
    if (h->g.stretched) return fail(MFC_E_UNSUPPORTED, "harvest labels uniform-grid WENO5 weights");
    int st = mfc_fill_ghosts(h, q, stream);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = h->cells * h->g.ndim;
    const unsigned blocks = (unsigned)((n + kThreads - 1) / kThreads);
    const double se = std::sqrt(h->g.eps);
    const double *qd = (const double *)q;
    switch (h->g.ndim) {
    case 1: hipLaunchKernelGGL(k_harvest<1>, dim3(blocks), dim3(kThreads), 0, s, h->g, qd, features, labels, maxdev, se, 0.01, h->cells); break;
    case 2: hipLaunchKernelGGL(k_harvest<2>, dim3(blocks), dim3(kThreads), 0, s, h->g, qd, features, labels, maxdev, se, 0.01, h->cells); break;
    default: hipLaunchKernelGGL(k_harvest<3>, dim3(blocks), dim3(kThreads), 0, s, h->g, qd, features, labels, maxdev, se, 0.01, h->cells); break;
    }
    return hip_status(hipGetLastError(), "harvest launch");
}

int mfc_trainer_free(mfc_trainer *t)
{
    if (!t) return MFC_OK;
    (void)hipDeviceSynchronize();
    for (void *p : {(void *)t->w, (void *)t->m, (void *)t->v, (void *)t->grad, (void *)t->partial})
        if (p) (void)hipFree(p);
    delete t;
    return MFC_OK;
}

int mfc_trainer_init(int64_t max_batch, mfc_trainer **out)
{
    if (!out) return fail(MFC_E_ARG, "out is NULL");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (int64_t(1) << 31)) return fail(MFC_E_ARG, "max_batch must be in [1, 2^31]");
    mfc_trainer *t = new (std::nothrow) mfc_trainer();
    if (!t) return fail(MFC_E_NOMEM, "host allocation failed");
    t->max_batch = max_batch;
    int cu = 0;
    if (hipGetDevice(&t->device) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, t->device) != hipSuccess || cu <= 0) {
        delete t;
        return fail(MFC_E_HIP, "device query failed");
    }
    const int64_t tiles = (max_batch + 15) / 16;
    t->blocks = (int)std::min<int64_t>((tiles + kWaves - 1) / kWaves, (int64_t)2 * cu);
    hipError_t e = hipSuccess;
    auto alloc = [&](float **p, size_t n) {
        if (e == hipSuccess) e = hipMalloc((void **)p, n * sizeof(float));
    };
    alloc(&t->w, NPARAM);
    alloc(&t->m, NPARAM);
    alloc(&t->v, NPARAM);
    alloc(&t->grad, NP1);
    alloc(&t->partial, (size_t)t->blocks * NP1);
    if (e == hipSuccess) e = hipMemset(t->w, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemset(t->m, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemset(t->v, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        mfc_trainer_free(t);
        return fail(MFC_E_NOMEM, "trainer allocation failed");
    }
    *out = t;
    return MFC_OK;
}

int mfc_trainer_set_params(mfc_trainer *t, const float *params_host)
{
    if (!t || !params_host) return fail(MFC_E_ARG, "null argument");
    hipError_t e = hipMemcpy(t->w, params_host, NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(t->m, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemset(t->v, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    t->step = 0;
    t->have_grad = false;
    return hip_status(e, "trainer parameter upload");
}

int mfc_trainer_get_params(mfc_trainer *t, float *params_host)
{
    if (!t || !params_host) return fail(MFC_E_ARG, "null argument");
    return hip_status(hipMemcpy(params_host, t->w, NPARAM * sizeof(float), hipMemcpyDeviceToHost),
                      "trainer parameter download");
}

int mfc_trainer_grad(mfc_trainer *t, const uint16_t *features, const uint8_t *labels, const int32_t *index,
                     int64_t batch, void *stream)
{
    if (!t || !features || !labels) return fail(MFC_E_ARG, "null argument");
    if (batch < 1 || batch > t->max_batch) return fail(MFC_E_ARG, "batch must be in [1, max_batch]");
    hipStream_t s = (hipStream_t)stream;
    const float inv_n = (float)(1.0 / (double)batch);
    hipLaunchKernelGGL(k_mlp_grad, dim3(t->blocks), dim3(kThreads), 0, s, t->w, features, labels, index, batch, inv_n,
                       t->partial);
    hipLaunchKernelGGL(k_mlp_reduce, dim3((NP1 + 255) / 256), dim3(256), 0, s, t->partial, t->blocks, t->grad, inv_n);
    t->have_grad = true;
    return hip_status(hipGetLastError(), "gradient launch");
}

int mfc_trainer_read_grad(mfc_trainer *t, float *grad_host, float *loss_host, void *stream)
{
    if (!t || !grad_host) return fail(MFC_E_ARG, "null argument");
    if (!t->have_grad) return fail(MFC_E_ARG, "no gradient computed yet");
    float buf[NP1];
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(buf, t->grad, sizeof(buf), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "gradient download");
    for (int i = 0; i < NPARAM; i++) grad_host[i] = buf[i];
    if (loss_host) *loss_host = buf[NPARAM];
    return MFC_OK;
}

int mfc_trainer_adam(mfc_trainer *t, float lr, float beta1, float beta2, float eps, void *stream)
{
    if (!t) return fail(MFC_E_ARG, "null argument");
    if (!t->have_grad) return fail(MFC_E_ARG, "no gradient computed yet");
    if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
        return fail(MFC_E_ARG, "bad Adam hyper-parameters");
    t->step++;
    const float c1 = (float)(1.0 - std::pow((double)beta1, (double)t->step));
    const float c2 = (float)(1.0 - std::pow((double)beta2, (double)t->step));
    hipLaunchKernelGGL(k_adam, dim3((NPARAM + 255) / 256), dim3(256), 0, (hipStream_t)stream, t->w, t->m, t->v, t->grad,
                       lr, beta1, beta2, c1, c2, eps);
    return hip_status(hipGetLastError(), "Adam launch");
}

int mfc_trainer_infer(mfc_trainer *t, const uint16_t *features, int64_t n, float *prob, void *stream)
{
    if (!t || !features || !prob) return fail(MFC_E_ARG, "null argument");
    if (n < 1) return fail(MFC_E_ARG, "n must be >= 1");
    const int64_t tiles = (n + 15) / 16;
    const unsigned blocks = (unsigned)std::min<int64_t>((tiles + kWaves - 1) / kWaves, 4096);
    hipLaunchKernelGGL(k_mlp_infer, dim3(blocks), dim3(kThreads), 0, (hipStream_t)stream, t->w, features, n, prob);
    return hip_status(hipGetLastError(), "inference launch");
}

int mfc_set_indicator(mfc_grid *h, const float *params_host, double tau)
{
    if (!h || !params_host) return fail(MFC_E_ARG, "null argument");
    if (!std::isfinite(tau)) return fail(MFC_E_ARG, "tau must be finite");
    for (int i = 0; i < NPARAM; i++)
        if (!std::isfinite(params_host[i])) return fail(MFC_E_ARG, "non-finite network parameter");
    hipError_t e = hipSuccess;
    if (!h->mlp) e = hipMalloc((void **)&h->mlp, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemcpy(h->mlp, params_host, NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_status(e, "indicator upload");
    // P > tau  <=>  logit > log(tau / (1 - tau))
    h->logit_tau = tau <= 0.0 ? -INFINITY : (tau >= 1.0 ? INFINITY : (float)std::log(tau / (1.0 - tau)));
    return MFC_OK;
}

}  // extern "C"
