// Batched ensembles of independent 2D runs (uneven grid sizes) advanced
// together: every kernel of an SSP-RK3 step (Sec. 3.4) covers all runs at
// once, so one step of the whole ensemble is five launches (four when the
// previous step of the same run call supplied the wave speeds), which
// mfc_batch_run captures once into a HIP graph and replays.
//
//   k_batch_wavespeed  per-run maxima of max_d(|u_d| + c)
//   k_batch_dt         per-run time step from the CFL number (Sec. 1)
//   k_batch_stage      the right-hand side of eq. (fvmdis) (Sec. 3.1-3.2.1)
//                      and the stage combination; a persistent kernel: a
//                      fixed set of workgroups walks the flat list of
//                      (run, tile) work items, 16 x 16 (or autotuned) tiles
//                      of the LDS-staged x/y sweep.  It reads neighbours
//                      past a domain face through the boundary rule
//                      (bc_cell: the values a ghost fill would write, bit
//                      for bit), so no ghost fill runs; in the last stage
//                      of a step followed by another of the same call it
//                      also reduces the wave speeds of the state it writes,
//                      for that step's size.
// Runs differ only through their descriptors (sizes, strides, dx, fluids,
// boundaries), so a run advanced in the batch and the same run advanced
// alone by the single-grid path execute the same arithmetic.
#include <cmath>
#include <map>
#include <new>

#include "charbc.h"
#include "internal.h"

namespace mfc {
namespace {

constexpr int kBT = 256;          // threads per workgroup
constexpr int kWsBlocks = 8;      // wave-speed workgroups per run
constexpr int kXcds = 8;          // accelerator complex dies of the MI355X

template <class T>
struct RunDev {
    Grid g;
    T *q;          // caller's state (step input and output)
    T *a, *b;      // stage registers q^(1), q^(2)
    int tiles_x;   // for the stage kernel's tile decode (set per tile shape)
};

// ------------------------------------------------------------ wave speed
template <class T>
__global__ void __launch_bounds__(kBT) k_batch_wavespeed(const RunDev<T> *__restrict__ runs, double *__restrict__ partial,
                                                         int *__restrict__ flag)
{
    __shared__ double red[kBT / 64];
    const int run = blockIdx.x / kWsBlocks, part = blockIdx.x % kWsBlocks;
    const RunDev<T> &R = runs[run];
    const Grid &g = R.g;
    const int64_t total = (int64_t)g.n[0] * g.n[1];
    double smax = 0.0;
    bool bad = false;
    for (int64_t t = (int64_t)part * kBT + threadIdx.x; t < total; t += (int64_t)kWsBlocks * kBT) {
        const int i = (int)(t % g.n[0]), j = (int)(t / g.n[0]);
        const int64_t c = (int64_t)(j + NG) * g.stride[1] + (i + NG);
        T qc[6], wc[6];
#pragma unroll
        for (int v = 0; v < 6; v++) qc[v] = R.q[v * g.vstride + c];
        bad |= cons_to_prim<2, T>(g, qc, wc);
        double Gam, Pi;
        mixture<double>(g, double(wc[5]), Gam, Pi);
        const double cs = sqrtT(sound2<double>(Gam, Pi, double(wc[0]) + double(wc[1]), double(wc[4])));
        smax = __builtin_fmax(smax, __builtin_fmax(__builtin_fabs(double(wc[2])), __builtin_fabs(double(wc[3]))) + cs);
    }
    if (bad) atomicOr(flag, 2);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) smax = __builtin_fmax(smax, __shfl_xor(smax, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = smax;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = red[0];
        for (int w = 1; w < kBT / 64; w++) m = __builtin_fmax(m, red[w]);
        partial[blockIdx.x] = m;
    }
}

// Per-run step size and accumulated time: scal[3 r + 0..2] = smax, dt, t.
// The maximum comes from the wave-speed partials, or (carried) from the
// maxima the previous step's last stage accumulated in cmax, kept as the
// bit patterns of non-negative doubles (which order as integers); either
// way cmax is cleared for the next accumulation.
__global__ void k_batch_dt(const double *__restrict__ partial, unsigned long long *__restrict__ cmax,
                           double *__restrict__ scal, const double *__restrict__ dxmin, int nrun, double cfl,
                           int carried)
{
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nrun) return;
    double m = 0.0;
    if (carried) {
        m = __longlong_as_double((long long)cmax[r]);
    } else {
        for (int b = 0; b < kWsBlocks; b++) m = __builtin_fmax(m, partial[r * kWsBlocks + b]);
    }
    cmax[r] = 0ull;
    const double dt = cfl * dxmin[r] / m;
    scal[3 * r + 0] = m;
    scal[3 * r + 1] = dt;
    scal[3 * r + 2] += dt;
}

// ------------------------------------------------------------------ stage
// One (run, tile) work item: the 2D right-hand side of a TX x TY tile and its
// stage combination, with the plane and the face values staged in LDS.
template <int TX, int TY, class T>
struct Tile2 {
    static constexpr int NV = 6, PX = TX + 2 * NG, PY = TY + 2 * NG;
    static constexpr int NPX = (TX + 2) * TY, NFX = (TX + 1) * TY;
    static constexpr int NPY = TX * (TY + 2), NFY = TX * (TY + 1);
    static constexpr int NP = NPX > NPY ? NPX : NPY, NF = NFX > NFY ? NFX : NFY;
    static constexpr int NHALO = 2 * NG * (TX + TY);
};

template <class T>
__device__ __forceinline__ bool load6(const Grid &g, const T *__restrict__ q, int i, int j, T *w)
{
    const int64_t c = (int64_t)(j + NG) * g.stride[1] + (i + NG);
    T qc[6];
#pragma unroll
    for (int v = 0; v < 6; v++) qc[v] = q[v * g.vstride + c];
    const bool bad = cons_to_prim<2, T>(g, qc, w);
    const int outside = (i < 0 || i >= g.n[0]) + (j < 0 || j >= g.n[1]);
    return bad && outside <= 1;
}

// Characteristic rates (charbc.h, Sec. 3.3) of the boundary cell at tile
// position (r, c) on face SIDE of dimension D, from the cell and the next
// two cells into the domain in the tile's LDS plane.
template <int D, int SIDE, class T, int PY, int PX>
__device__ __forceinline__ bool tile_char_rate(const Grid &g, const T (&pl)[6][PY][PX], int r, int c, T inv_dx,
                                               T *rate)
{
    constexpr int sg = SIDE == 0 ? 1 : -1;
    T W[3][6];
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
        for (int v = 0; v < 6; v++) W[j][v] = D == 0 ? pl[v][r][c + sg * j] : pl[v][r + sg * j][c];
    return char_rate<2, D, SIDE, T>(g, W[0], W[1], W[2], inv_dx, one_sided<T>(g, D, SIDE), rate);
}

// LDS of a tile (plane, face-value pairs, fluxes): the FP64 64 x 4 tile
// (88 KB) fits one workgroup per CU, every other shape at least two
template <int TX, int TY, class T>
constexpr int kBatchWaves =
    sizeof(T) * (6 * Tile2<TX, TY, T>::PY * Tile2<TX, TY, T>::PX + 12 * Tile2<TX, TY, T>::NP + 7 * Tile2<TX, TY, T>::NF) >
            80 * 1024 ? 1 : 2;

template <int TX, int TY, class T>
__global__ void __launch_bounds__(kBT, (kBatchWaves<TX, TY, T>))
    k_batch_stage(const RunDev<T> *__restrict__ runs, const int *__restrict__ item_run, const int *__restrict__ item_tile,
                  int nitems, const double *__restrict__ scal, int stage, int xcd, int *__restrict__ flag,
                  unsigned long long *__restrict__ cmax)
{
    using S = Tile2<TX, TY, T>;
    constexpr int NV = 6, A = 5, E = 4;
    static_assert(TX * TY == kBT, "one cell per thread");
    __shared__ T s_plane[NV][S::PY][S::PX];
    __shared__ T s_pair[2 * NV][S::NP];
    __shared__ T s_flux[NV + 1][S::NF];
    const int tid = threadIdx.x, tx = tid % TX, ty = tid / TX;
    const T ca = T(stage == 1 ? 0.0 : (stage == 2 ? 0.75 : 1.0 / 3.0));
    const T cb = T(stage == 1 ? 1.0 : (stage == 2 ? 0.25 : 2.0 / 3.0));
    bool bad = false;

    // Work items: round-robin over the workgroups, or (xcd != 0) contiguous
    // runs of items per XCD, so that neighbouring tiles, which read each
    // other's halo cells, are served by the same L2.  Workgroups are dealt to
    // the 8 XCDs round-robin by index; the grid is a multiple of 8.
    int it0 = blockIdx.x, it1 = nitems, istep = gridDim.x;
    if (xcd) {
        const int x = blockIdx.x % kXcds, per = gridDim.x / kXcds;
        it0 = (int)((int64_t)x * nitems / kXcds) + blockIdx.x / kXcds;
        it1 = (int)((int64_t)(x + 1) * nitems / kXcds);
        istep = per;
    }
    for (int it = it0; it < it1; it += istep) {
        const int run = item_run[it], tile = item_tile[it];
        const RunDev<T> &R = runs[run];
        const Grid &g = R.g;
        const T *q = stage == 1 ? R.q : (stage == 2 ? R.a : R.b);
        T *out = stage == 1 ? R.a : (stage == 2 ? R.b : R.q);
        const T *q0 = R.q;
        const T hdt = T(scal[3 * run + 1]);
        const T eps = T(g.eps), idx = T(g.inv_dx[0]), idy = T(g.inv_dx[1]);
        const int x0 = (tile % R.tiles_x) * TX, y0 = (tile / R.tiles_x) * TY;
        const int xmax = g.n[0] + NG - 1, ymax = g.n[1] + NG - 1;
        const int gx = x0 + tx, gy = y0 + ty;
        const bool own = gx < g.n[0] && gy < g.n[1];
        // cell (i, j) of the tile's window through the boundary rule (cells
        // past a ragged tile edge load a duplicate whose results are dropped)
        auto bx = [&](int i) { return bc_cell(min(i, xmax), g.n[0], g.bc[0], g.bc[1]); };
        auto by = [&](int j) { return bc_cell(min(j, ymax), g.n[1], g.bc[2], g.bc[3]); };
        T wk[NV];
        bad |= load6<T>(g, q, bx(gx), by(gy), wk);
#pragma unroll
        for (int v = 0; v < NV; v++) s_plane[v][ty + NG][tx + NG] = wk[v];
        for (int h = tid; h < S::NHALO; h += kBT) {
            int li, lj;
            if (h < 2 * NG * TY) {
                const int c = h % (2 * NG), row = h / (2 * NG);
                li = c < NG ? c : TX + c;
                lj = row + NG;
            } else {
                const int h2 = h - 2 * NG * TY;
                const int c = h2 % TX, r = h2 / TX;
                li = c + NG;
                lj = r < NG ? r : TY + r;
            }
            T w[NV];
            bad |= load6<T>(g, q, bx(x0 + li - NG), by(y0 + lj - NG), w);
#pragma unroll
            for (int v = 0; v < NV; v++) s_plane[v][lj][li] = w[v];
        }
        __syncthreads();
        for (int p = tid; p < S::NPX; p += kBT) {
            const int row = p / (TX + 2), c = p % (TX + 2);
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const T *s = &s_plane[v][row + NG][c];
                weno5_pair(s[0], s[1], s[2], s[3], s[4], eps, s_pair[v][p], s_pair[NV + v][p]);
            }
        }
        __syncthreads();
        for (int f = tid; f < S::NFX; f += kBT) {
            const int row = f / (TX + 1), fi = f % (TX + 1);
            const int pl = row * (TX + 2) + fi;
            T wL[NV], wR[NV], F[NV], uf;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wL[v] = s_pair[v][pl];
                wR[v] = s_pair[NV + v][pl + 1];
            }
            const bool b = hllc<2, 0, T>(g, wL, wR, F, uf);
            bad |= b && (y0 + row < g.n[1]) && (x0 + fi <= g.n[0]);
#pragma unroll
            for (int v = 0; v < NV; v++) s_flux[v][f] = F[v];
            s_flux[NV][f] = uf;
        }
        __syncthreads();
        T L[NV], divu;
        {
            const int f = ty * (TX + 1) + tx;
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] = (s_flux[v][f] - s_flux[v][f + 1]) * idx;
            divu = (s_flux[NV][f + 1] - s_flux[NV][f]) * idx;
        }
        // Characteristic faces (Sec. 3.3): the boundary cell of such a face
        // takes the characteristic rates in place of its terms normal to it.
        // The rates of x faces are taken here, while s_plane is this item's
        // for every thread, and put in place of the x terms after the y
        // sweep; every other cell sums its terms exactly as the single-grid
        // kernel does.
        const int xside = !own ? -1
                               : (gx == 0 && g.bc[0] == MFC_BC_CHARACTERISTIC)
                                     ? 0
                                     : ((gx == g.n[0] - 1 && g.bc[1] == MFC_BC_CHARACTERISTIC) ? 1 : -1);
        const int yside = !own ? -1
                               : (gy == 0 && g.bc[2] == MFC_BC_CHARACTERISTIC)
                                     ? 0
                                     : ((gy == g.n[1] - 1 && g.bc[3] == MFC_BC_CHARACTERISTIC) ? 1 : -1);
        T xrate[NV];
        if (xside == 0) bad |= tile_char_rate<0, 0>(g, s_plane, ty + NG, tx + NG, idx, xrate);
        else if (xside == 1) bad |= tile_char_rate<0, 1>(g, s_plane, ty + NG, tx + NG, idx, xrate);
        for (int p = tid; p < S::NPY; p += kBT) {
            const int c = p % TX, r = p / TX;
            const int li = c + NG;
#pragma unroll
            for (int v = 0; v < NV; v++)
                weno5_pair(s_plane[v][r][li], s_plane[v][r + 1][li], s_plane[v][r + 2][li], s_plane[v][r + 3][li],
                           s_plane[v][r + 4][li], eps, s_pair[v][p], s_pair[NV + v][p]);
        }
        __syncthreads();
        for (int f = tid; f < S::NFY; f += kBT) {
            const int c = f % TX, fr = f / TX;
            const int pl = fr * TX + c;
            T wL[NV], wR[NV], F[NV], uf;
#pragma unroll
            for (int v = 0; v < NV; v++) {
                wL[v] = s_pair[v][pl];
                wR[v] = s_pair[NV + v][pl + TX];
            }
            const bool b = hllc<2, 1, T>(g, wL, wR, F, uf);
            bad |= b && (x0 + c < g.n[0]) && (y0 + fr <= g.n[1]);
#pragma unroll
            for (int v = 0; v < NV; v++) s_flux[v][f] = F[v];
            s_flux[NV][f] = uf;
        }
        __syncthreads();
        {
            const int f = ty * TX + tx;
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] += (s_flux[v][f] - s_flux[v][f + TX]) * idy;
            divu += (s_flux[NV][f + TX] - s_flux[NV][f]) * idy;
        }
        if (xside >= 0 || yside >= 0) {   // boundary cells of characteristic faces
            // the y terms again (the x ones: the sum minus them), each
            // replaced by the face's rates where the cell is on such a face
            // (s_plane stays this item's until the barrier at the end of it)
            const int f = ty * TX + tx;
            T yt[NV], rate[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) yt[v] = (s_flux[v][f] - s_flux[v][f + TX]) * idy;
            const T dy = (s_flux[NV][f + TX] - s_flux[NV][f]) * idy;
            if (yside == 0) bad |= tile_char_rate<1, 0>(g, s_plane, ty + NG, tx + NG, idy, rate);
            else if (yside == 1) bad |= tile_char_rate<1, 1>(g, s_plane, ty + NG, tx + NG, idy, rate);
#pragma unroll
            for (int v = 0; v < NV; v++) {
                const T xs = xside >= 0 ? xrate[v] : L[v] - yt[v];
                L[v] = xs + (yside >= 0 ? rate[v] : yt[v]);
            }
            divu = (xside >= 0 ? T(0) : divu - dy) + (yside >= 0 ? T(0) : dy);
        }
        L[A] += alpha_source<T>(g, wk[A], wk[E]) * divu;
        double smax_item = 0.0;
        if (own) {
            const int64_t c = (int64_t)(gy + NG) * g.stride[1] + (gx + NG);
            // every operand before the first store (out may alias q0)
            T a0[NV], a1[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                a0[v] = q0[v * g.vstride + c];
                a1[v] = q[v * g.vstride + c];
            }
            T r[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) {
                r[v] = ca * a0[v] + cb * (a1[v] + hdt * L[v]);
                out[v * g.vstride + c] = r[v];
            }
            if (cmax) {   // max_d |u_d| + c of the stored state, as k_batch_wavespeed forms it
                T wr[NV];
                cons_to_prim<2, T>(g, r, wr);
                double Gam, Pi;
                mixture<double>(g, double(wr[5]), Gam, Pi);
                const double cs = sqrtT(sound2<double>(Gam, Pi, double(wr[0]) + double(wr[1]), double(wr[4])));
                smax_item = __builtin_fmax(__builtin_fabs(double(wr[2])), __builtin_fabs(double(wr[3]))) + cs;
            }
        }
        if (cmax) {   // wavefront maximum of the item, one atomic per wavefront
            double m = smax_item;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) m = __builtin_fmax(m, __shfl_xor(m, o, 64));
            if ((tid & 63) == 0) atomicMax(&cmax[run], (unsigned long long)__double_as_longlong(m));
        }
        // the next item overwrites s_plane only after every thread passed the
        // barrier above; s_pair and s_flux after two more
        __syncthreads();
    }
    if (bad) atomicOr(flag, 1);
}

__global__ void k_batch_reset(double *scal, int n3, int *flag)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n3) scal[i] = 0.0;
    if (i == 0) *flag = 0;
}

}  // namespace
}  // namespace mfc

using namespace mfc;

// Tile shapes the stage kernel is instantiated for, and workgroups per CU of
// the persistent stage launch; the autotuner searches their product with the
// XCD mapping on and off.
static const int kShapes[][2] = {{16, 16}, {32, 8}, {64, 4}};
constexpr int kNumShapes = 3;
static const int kGroupsPerCu[] = {1, 2, 4};
constexpr int kNumGroups = 3;
constexpr int kMaxGraphSteps = 64;  // steps captured in one graph

struct mfc_batch {
    int nrun = 0;
    int precision = MFC_FP32_MIXED;
    int device = 0;
    int cu_count = 0;
    mfc_batch_tune tune{0, 1, 1};
    std::vector<mfc_grid_desc> desc;
    std::vector<Grid> grids;
    std::vector<void *> stage;        // 2 per run
    void *runs = nullptr;             // RunDev<T>[nrun] (device)
    int64_t cells = 0;
    int *items[kNumShapes][2] = {};   // item_run, item_tile per shape (device)
    int nitems[kNumShapes] = {};
    double *partial = nullptr;        // [nrun * kWsBlocks]
    unsigned long long *cmax = nullptr;  // [nrun] carried wave-speed maxima (bit patterns)
    double *scal = nullptr;           // [3 * nrun]
    double *dxmin = nullptr;          // [nrun]
    int *flag = nullptr;
    std::vector<void *> bound_q;      // q pointers the device descriptors hold
    int bound_shape = -1;
    hipGraphExec_t graph = nullptr;
    double graph_cfl = 0.0;
    int graph_steps = 0;
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;  // recorded stage launches
    double ms = 0.0;
    int64_t launches = 0;
};

namespace {

size_t elem(const mfc_batch *b) { return b->precision == MFC_FP32_MIXED ? 4 : 8; }

void drop_graph(mfc_batch *b)
{
    if (b->graph) {
        (void)hipGraphExecDestroy(b->graph);
        b->graph = nullptr;
    }
}

template <class T>
int upload_runs(mfc_batch *b, void *const *q)
{
    std::vector<RunDev<T>> h(b->nrun);
    const int tx = kShapes[b->tune.shape][0];
    for (int r = 0; r < b->nrun; r++) {
        h[r].g = b->grids[r];
        h[r].q = (T *)q[r];
        h[r].a = (T *)b->stage[2 * r];
        h[r].b = (T *)b->stage[2 * r + 1];
        h[r].tiles_x = (b->grids[r].n[0] + tx - 1) / tx;
    }
    // earlier steps may still read the descriptors
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(b->runs, h.data(), sizeof(RunDev<T>) * b->nrun, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        b->bound_q.clear();
        return hip_status(e, "batch descriptor upload");
    }
    b->bound_q.assign(q, q + b->nrun);
    b->bound_shape = b->tune.shape;
    return MFC_OK;
}

int bind(mfc_batch *b, void *const *q)
{
    for (int r = 0; r < b->nrun; r++)
        if (!q[r]) return fail(MFC_E_ARG, "null state pointer in the batch");
    bool same = b->bound_q.size() == (size_t)b->nrun && b->bound_shape == b->tune.shape;
    for (int r = 0; same && r < b->nrun; r++) same = b->bound_q[r] == q[r];
    if (same) return MFC_OK;
    drop_graph(b);
    return b->precision == MFC_FP32_MIXED ? upload_runs<float>(b, q) : upload_runs<double>(b, q);
}

unsigned stage_groups(const mfc_batch *b)
{
    const int64_t want = (int64_t)kGroupsPerCu[b->tune.groups] * b->cu_count;
    const int64_t n = std::min<int64_t>(want, b->nitems[b->tune.shape]);
    return (unsigned)((n + kXcds - 1) / kXcds * kXcds);
}

template <class T>
void launch_stage(mfc_batch *b, int st, hipStream_t s, unsigned long long *cmax = nullptr)
{
    const RunDev<T> *runs = (const RunDev<T> *)b->runs;
    const int sh = b->tune.shape, nitems = b->nitems[sh], xcd = b->tune.xcd;
    const int *ir = b->items[sh][0], *it = b->items[sh][1];
    const dim3 grid(stage_groups(b)), block(kBT);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (b->timing && hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess)
        (void)hipEventRecord(e0, s);
    if (sh == 0)
        hipLaunchKernelGGL((k_batch_stage<16, 16, T>), grid, block, 0, s, runs, ir, it, nitems, b->scal, st, xcd, b->flag, cmax);
    else if (sh == 1)
        hipLaunchKernelGGL((k_batch_stage<32, 8, T>), grid, block, 0, s, runs, ir, it, nitems, b->scal, st, xcd, b->flag, cmax);
    else
        hipLaunchKernelGGL((k_batch_stage<64, 4, T>), grid, block, 0, s, runs, ir, it, nitems, b->scal, st, xcd, b->flag, cmax);
    if (e1) {
        (void)hipEventRecord(e1, s);
        b->ev.emplace_back(e0, e1);
    } else if (e0) {
        (void)hipEventDestroy(e0);
    }
}

// One step of every run.  carried_in: the per-run maxima of this step's
// input were accumulated in cmax by the previous step's last stage;
// carry_out: have this step's last stage accumulate those of its output.
template <class T>
int enqueue_step(mfc_batch *b, double cfl, hipStream_t s, bool carried_in, bool carry_out)
{
    const RunDev<T> *runs = (const RunDev<T> *)b->runs;
    if (!carried_in)
        hipLaunchKernelGGL((k_batch_wavespeed<T>), dim3(b->nrun * kWsBlocks), dim3(kBT), 0, s, runs, b->partial,
                           b->flag);
    hipLaunchKernelGGL(k_batch_dt, dim3((b->nrun + 63) / 64), dim3(64), 0, s, b->partial, b->cmax, b->scal, b->dxmin,
                       b->nrun, cfl, carried_in ? 1 : 0);
    launch_stage<T>(b, 1, s);
    launch_stage<T>(b, 2, s);
    launch_stage<T>(b, 3, s, carry_out ? b->cmax : nullptr);
    return hip_status(hipGetLastError(), "batch step launch");
}

int enqueue(mfc_batch *b, double cfl, hipStream_t s, bool carried_in = false, bool carry_out = false)
{
    return b->precision == MFC_FP32_MIXED ? enqueue_step<float>(b, cfl, s, carried_in, carry_out)
                                          : enqueue_step<double>(b, cfl, s, carried_in, carry_out);
}

// n steps as one sequence: the first reduces its wave speeds itself, every
// other takes them from its predecessor's last stage.
int enqueue_steps(mfc_batch *b, int n, double cfl, hipStream_t s)
{
    int st = MFC_OK;
    for (int k = 0; k < n && st == MFC_OK; k++) st = enqueue(b, cfl, s, k > 0, k + 1 < n);
    return st;
}

int collect_timing(mfc_batch *b)
{
    for (auto &p : b->ev) {
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(p.second);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, p.first, p.second);
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
        if (e != hipSuccess) {
            b->ev.clear();
            return hip_status(e, "batch kernel timing");
        }
        b->ms += ms;
        b->launches++;
    }
    b->ev.clear();
    return MFC_OK;
}

}  // namespace

extern "C" {

int mfc_batch_free(mfc_batch *b)
{
    if (!b) return MFC_OK;
    (void)hipDeviceSynchronize();
    (void)collect_timing(b);
    drop_graph(b);
    for (void *p : b->stage)
        if (p) (void)hipFree(p);
    for (int sh = 0; sh < kNumShapes; sh++)
        for (int k = 0; k < 2; k++)
            if (b->items[sh][k]) (void)hipFree(b->items[sh][k]);
    for (void *p : {b->runs, (void *)b->cmax, (void *)b->partial, (void *)b->scal, (void *)b->dxmin, (void *)b->flag})
        if (p) (void)hipFree(p);
    delete b;
    return MFC_OK;
}

int mfc_batch_init(const mfc_grid_desc *descs, int count, mfc_batch **out)
{
    if (!out) return fail(MFC_E_ARG, "out is NULL");
    *out = nullptr;
    if (!descs || count <= 0 || count > 4096) return fail(MFC_E_ARG, "need 1..4096 descriptors");
    const int prec = descs[0].precision;
    for (int r = 0; r < count; r++) {
        const mfc_grid_desc &d = descs[r];
        if (d.ndim != 2) return fail(MFC_E_UNSUPPORTED, "batched runs must be 2D");
        if (d.precision != prec) return fail(MFC_E_ARG, "all runs of a batch share one precision");
        if (d.precision != MFC_FP64 && d.precision != MFC_FP32_MIXED) return fail(MFC_E_ARG, "unknown precision");
        if (d.num_fluids != 2) return fail(MFC_E_UNSUPPORTED, "num_fluids must be 2");
        if (d.recon != MFC_RECON_WENO5) return fail(MFC_E_UNSUPPORTED, "batched runs use WENO5");
        if (d.model != MFC_MODEL_ALLAIRE && d.model != MFC_MODEL_KAPILA) return fail(MFC_E_ARG, "unknown model");
        if (d.faces[0] || d.faces[1]) return fail(MFC_E_UNSUPPORTED, "batched runs use uniform cells");
        for (int k = 0; k < 2; k++) {
            if (d.n[k] < 3 || d.n[k] > (1 << 15)) return fail(MFC_E_ARG, "n must be in [3, 32768]");
            if (!(d.hi[k] > d.lo[k])) return fail(MFC_E_ARG, "hi must exceed lo");
            const int a = d.bc[2 * k], c = d.bc[2 * k + 1];
            auto known = [](int x) { return x == MFC_BC_EXTRAP || x == MFC_BC_PERIODIC || x == MFC_BC_CHARACTERISTIC; };
            if (!known(a) || !known(c) || ((a == MFC_BC_PERIODIC) != (c == MFC_BC_PERIODIC)))
                return fail(MFC_E_ARG, "bad boundary conditions");
            if ((a == MFC_BC_CHARACTERISTIC || c == MFC_BC_CHARACTERISTIC) && d.model != MFC_MODEL_ALLAIRE)
                return fail(MFC_E_UNSUPPORTED, "characteristic boundaries take the Allaire model");
        }
        for (int f = 0; f < 2; f++)
            if (!(d.gamma[f] > 1.0) || !(d.pi_inf[f] >= 0.0)) return fail(MFC_E_ARG, "bad fluid parameters");
        if (!(d.weno_eps > 0.0)) return fail(MFC_E_ARG, "weno_eps must be > 0");
    }
    mfc_batch *b = new (std::nothrow) mfc_batch();
    if (!b) return fail(MFC_E_NOMEM, "host allocation failed");
    b->nrun = count;
    b->precision = prec;
    b->desc.assign(descs, descs + count);
    if (hipGetDevice(&b->device) != hipSuccess ||
        hipDeviceGetAttribute(&b->cu_count, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess ||
        b->cu_count <= 0) {
        delete b;
        return fail(MFC_E_HIP, "device query failed");
    }
    std::vector<double> dxmin(count);
    for (int r = 0; r < count; r++) {
        const mfc_grid_desc &d = descs[r];
        Grid g{};
        g.ndim = 2;
        g.n[0] = d.n[0];
        g.n[1] = d.n[1];
        g.n[2] = 1;
        g.p[0] = d.n[0] + 2 * NG;
        g.p[1] = d.n[1] + 2 * NG;
        g.p[2] = 1;
        g.off[0] = g.off[1] = NG;
        g.off[2] = 0;
        for (int f = 0; f < 6; f++) g.bc[f] = f < 4 ? d.bc[f] : MFC_BC_EXTRAP;   // read by index (bc_cell)
        g.stride[0] = 1;
        g.stride[1] = g.p[0];
        g.stride[2] = (int64_t)g.p[0] * g.p[1];
        g.vstride = g.stride[2];
        for (int k = 0; k < 2; k++) g.inv_dx[k] = d.n[k] / (d.hi[k] - d.lo[k]);
        g.inv_dx[2] = 0.0;
        // the same expressions, in the same order, as the single-grid handle
        g.dxmin = 1e300;
        for (int k = 0; k < 2; k++) g.dxmin = std::fmin(g.dxmin, (d.hi[k] - d.lo[k]) / d.n[k]);
        g.g1 = 1.0 / (d.gamma[0] - 1.0);
        g.g2 = 1.0 / (d.gamma[1] - 1.0);
        g.h1 = d.gamma[0] * d.pi_inf[0] / (d.gamma[0] - 1.0);
        g.h2 = d.gamma[1] * d.pi_inf[1] / (d.gamma[1] - 1.0);
        g.eps = d.weno_eps;
        set_kapila(g, d);
        g.order = 5;
        g.stretched = 0;
        for (int k = 0; k < 3; k++) g.wcoef[k] = g.winv[k] = nullptr;
        b->grids.push_back(g);
        dxmin[r] = g.dxmin;
        b->cells += (int64_t)g.n[0] * g.n[1];
    }
    hipError_t e = hipSuccess;
    auto alloc = [&](void **p, size_t bytes) {
        if (e == hipSuccess) e = hipMalloc(p, bytes);
    };
    b->stage.assign(2 * count, nullptr);
    for (int r = 0; r < count; r++)
        for (int k = 0; k < 2; k++) alloc(&b->stage[2 * r + k], (size_t)6 * b->grids[r].vstride * elem(b));
    alloc(&b->runs, sizeof(RunDev<double>) * count);
    alloc((void **)&b->cmax, sizeof(unsigned long long) * count);
    alloc((void **)&b->partial, sizeof(double) * count * kWsBlocks);
    alloc((void **)&b->scal, sizeof(double) * 3 * count);
    alloc((void **)&b->dxmin, sizeof(double) * count);
    alloc((void **)&b->flag, sizeof(int) * 2);
    for (int sh = 0; sh < kNumShapes && e == hipSuccess; sh++) {
        std::vector<int> ir, it;
        for (int r = 0; r < count; r++) {
            const int tx = (b->grids[r].n[0] + kShapes[sh][0] - 1) / kShapes[sh][0];
            const int ty = (b->grids[r].n[1] + kShapes[sh][1] - 1) / kShapes[sh][1];
            for (int t = 0; t < tx * ty; t++) {
                ir.push_back(r);
                it.push_back(t);
            }
        }
        b->nitems[sh] = (int)ir.size();
        alloc((void **)&b->items[sh][0], sizeof(int) * ir.size());
        alloc((void **)&b->items[sh][1], sizeof(int) * it.size());
        if (e == hipSuccess) e = hipMemcpy(b->items[sh][0], ir.data(), sizeof(int) * ir.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(b->items[sh][1], it.data(), sizeof(int) * it.size(), hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(b->cmax, 0, sizeof(unsigned long long) * count);   // set-up, not a graph node
    if (e == hipSuccess) e = hipMemcpy(b->dxmin, dxmin.data(), sizeof(double) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_batch_reset, dim3((3 * count + 255) / 256), dim3(256), 0, 0, b->scal, 3 * count, b->flag);
        e = hipDeviceSynchronize();
    }
    if (e != hipSuccess) {
        mfc_batch_free(b);
        return e == hipErrorOutOfMemory ? fail(MFC_E_NOMEM, "batch device allocation failed")
                                        : hip_status(e, "batch set-up");
    }
    *out = b;
    return MFC_OK;
}

int mfc_batch_layout(const mfc_batch *b, int run, int64_t *nvar, int64_t padded[3], int64_t *elem_bytes)
{
    if (!b || !nvar || !padded || !elem_bytes) return fail(MFC_E_ARG, "null argument");
    if (run < 0 || run >= b->nrun) return fail(MFC_E_ARG, "run index out of range");
    *nvar = 6;
    padded[0] = b->grids[run].p[0];
    padded[1] = b->grids[run].p[1];
    padded[2] = 1;
    *elem_bytes = (int64_t)elem(b);
    return MFC_OK;
}

int mfc_batch_set_tune(mfc_batch *b, const mfc_batch_tune *t)
{
    if (!b || !t) return fail(MFC_E_ARG, "null argument");
    if (t->shape < 0 || t->shape >= kNumShapes) return fail(MFC_E_ARG, "unknown tile shape");
    if (t->groups < 0 || t->groups >= kNumGroups) return fail(MFC_E_ARG, "unknown workgroup count");
    if (t->xcd != 0 && t->xcd != 1) return fail(MFC_E_ARG, "xcd must be 0 or 1");
    if (t->shape != b->tune.shape || t->groups != b->tune.groups || t->xcd != b->tune.xcd) drop_graph(b);
    b->tune = *t;
    return MFC_OK;
}

int mfc_batch_get_tune(const mfc_batch *b, mfc_batch_tune *t)
{
    if (!b || !t) return fail(MFC_E_ARG, "null argument");
    *t = b->tune;
    return MFC_OK;
}

int mfc_batch_step(mfc_batch *b, void *const *q, double cfl, void *stream)
{
    if (!b || !q) return fail(MFC_E_ARG, "null argument");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(MFC_E_ARG, "cfl must be > 0");
    int st = bind(b, q);
    if (st) return st;
    return enqueue_steps(b, 1, cfl, (hipStream_t)stream);
}

int mfc_batch_run(mfc_batch *b, void *const *q, int nsteps, double cfl, int use_graph, void *stream)
{
    if (!b || !q) return fail(MFC_E_ARG, "null argument");
    if (nsteps < 0) return fail(MFC_E_ARG, "nsteps must be >= 0");
    if (!(cfl > 0.0) || !std::isfinite(cfl)) return fail(MFC_E_ARG, "cfl must be > 0");
    int st = bind(b, q);
    if (st) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!use_graph || b->timing) return enqueue_steps(b, nsteps, cfl, s);
    const int chunk = std::min(nsteps, kMaxGraphSteps);
    if (chunk == 0) return MFC_OK;
    if (!b->graph || b->graph_cfl != cfl || b->graph_steps != chunk) {
        drop_graph(b);
        // capture `chunk` steps of the whole ensemble on a private stream
        hipStream_t cs;
        hipError_t e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (e != hipSuccess) return hip_status(e, "capture stream");
        hipGraph_t graph = nullptr;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e == hipSuccess) {
            st = enqueue_steps(b, chunk, cfl, cs);   // each replay starts from its own wave speeds
            e = hipStreamEndCapture(cs, &graph);
        }
        if (e == hipSuccess && st == MFC_OK) e = hipGraphInstantiate(&b->graph, graph, nullptr, nullptr, 0);
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (st) return st;
        if (e != hipSuccess) {
            b->graph = nullptr;
            return hip_status(e, "graph capture");
        }
        b->graph_cfl = cfl;
        b->graph_steps = chunk;
    }
    int done = 0;
    for (; done + chunk <= nsteps; done += chunk) {
        hipError_t e = hipGraphLaunch(b->graph, s);
        if (e != hipSuccess) return hip_status(e, "graph launch");
    }
    return enqueue_steps(b, nsteps - done, cfl, s);
}

int mfc_batch_autotune(mfc_batch *b, void *const *q, int reps, mfc_batch_tune *best, double *ms_table, void *stream)
{
    if (!b || !q) return fail(MFC_E_ARG, "null argument");
    if (reps < 1 || reps > 1000) return fail(MFC_E_ARG, "reps must be in [1, 1000]");
    hipStream_t s = (hipStream_t)stream;
    const mfc_batch_tune keep = b->tune;
    const bool keep_timing = b->timing;
    int st = collect_timing(b);
    if (st) return st;
    const double keep_ms = b->ms;
    const int64_t keep_launches = b->launches;
    b->timing = true;
    double best_ms = 1e300;
    mfc_batch_tune arg = keep;
    // Stage 1 reads the step input and writes the first stage register only,
    // so timing it leaves the states and the accumulated times untouched.
    for (int sh = 0; sh < kNumShapes && st == MFC_OK; sh++)
        for (int gr = 0; gr < kNumGroups && st == MFC_OK; gr++)
            for (int x = 0; x < 2 && st == MFC_OK; x++) {
                b->tune = mfc_batch_tune{sh, gr, x};
                if ((st = bind(b, q))) break;
                b->timing = false;
                if (b->precision == MFC_FP32_MIXED) launch_stage<float>(b, 1, s);  // warm-up
                else launch_stage<double>(b, 1, s);
                b->timing = true;
                b->ms = 0.0;
                b->launches = 0;
                for (int r = 0; r < reps; r++) {
                    if (b->precision == MFC_FP32_MIXED) launch_stage<float>(b, 1, s);
                    else launch_stage<double>(b, 1, s);
                }
                if ((st = hip_status(hipGetLastError(), "autotune launch"))) break;
                if ((st = collect_timing(b))) break;
                const double ms = b->ms / reps;
                if (ms_table) ms_table[(sh * kNumGroups + gr) * 2 + x] = ms;
                if (ms < best_ms) {
                    best_ms = ms;
                    arg = b->tune;
                }
            }
    b->timing = keep_timing;
    b->ms = keep_ms;
    b->launches = keep_launches;
    b->tune = st ? keep : arg;
    drop_graph(b);
    if (st) return st;
    if (best) *best = arg;
    return MFC_OK;
}

int mfc_batch_set_timing(mfc_batch *b, int enable)
{
    if (!b) return fail(MFC_E_ARG, "null argument");
    b->timing = enable != 0;
    return MFC_OK;
}

int mfc_batch_kernel_time(mfc_batch *b, double *ms_total, int64_t *launches)
{
    if (!b || !ms_total || !launches) return fail(MFC_E_ARG, "null argument");
    int st = collect_timing(b);
    if (st) return st;
    *ms_total = b->ms;
    *launches = b->launches;
    b->ms = 0.0;
    b->launches = 0;
    return MFC_OK;
}

int mfc_batch_cells(const mfc_batch *b, int64_t *cells, int *nrun)
{
    if (!b || !cells || !nrun) return fail(MFC_E_ARG, "null argument");
    *cells = b->cells;
    *nrun = b->nrun;
    return MFC_OK;
}

int mfc_batch_time(mfc_batch *b, double *t_host, void *stream)
{
    if (!b || !t_host) return fail(MFC_E_ARG, "null argument");
    std::vector<double> sc(3 * b->nrun);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(sc.data(), b->scal, sizeof(double) * sc.size(), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "batch time readback");
    for (int r = 0; r < b->nrun; r++) t_host[r] = sc[3 * r + 2];
    return MFC_OK;
}

int mfc_batch_check(mfc_batch *b, void *stream)
{
    if (!b) return fail(MFC_E_ARG, "null argument");
    int flag = 0;
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(&flag, b->flag, sizeof(int), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_status(e, "batch flag readback");
    if (flag) {
        hipLaunchKernelGGL(k_batch_reset, dim3(1), dim3(64), 0, s, b->scal, 0, b->flag);
        return fail(MFC_E_NONPHYSICAL, "a batched run met a non-physical cell");
    }
    return MFC_OK;
}

}  // extern "C"
