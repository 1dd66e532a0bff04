// Split right-hand side (3D): two launches per Runge-Kutta stage.
//
//   k_xy  x and y directions of eq. (fvmdis) (Sec. 3.1): a workgroup of
//         256 threads owns a 16 x 13 tile of an x-y plane and walks four
//         planes; each plane (with 3-cell halos) is converted to primitives
//         into LDS once, every cell of the tile plus one halo cell per side is
//         reconstructed once per direction (WENO5, both face values from one
//         stencil, Sec. 3.2), the HLLC flux of every face (Sec. 3.2.1) is
//         computed once and shared by the two cells of the face.  Per cell
//         it forms the x+y flux differences plus the x+y share of the
//         alpha1 div(u) source (eq. fvmdis) and writes 7 values: that x+y
//         part L_xy itself, or, when the stage's dt is already known (every
//         stage after the first, and the first with a given dt), the x+y
//         part of the SSP-RK3 combination (Sec. 3.4),
//         ca q^n + cb (q + dt L_xy).
//   k_z   z direction plus the rest of the stage update: one thread per
//         (x, y) column marches through a chunk of planes with the
//         primitives of five planes at hand (four in a per-thread LDS ring,
//         the newest in registers), reconstructs each cell once (both
//         faces) and solves each z face once, forms the z flux differences
//         and the z share of the source, and writes the stage result: the
//         x+y part plus cb dt L_z (or L_xy + L_z for a bare right-hand side,
//         q + dt (L_xy + L_z) in a first stage whose dt is set between the
//         two launches from the x+y pass's wave-speed maxima).  In the last
//         stage of a step followed by another of the same run it also
//         reduces the wave speeds of the state it writes, which sets the
//         next step's dt before that step starts.
//
// Neither kernel carries the other's state, so each fits its registers
// without spilling; the price is one round trip of 7 values per cell through
// HBM, and with the combination folded into the x+y pass the z pass reads
// neither q^n nor its own stage input a second time.  Both kernels are
// instantiated for FP64 and for the FP32 storage form
// (T = float; the x+y part is kept in the same type), and with the routed
// reconstruction (ROUTE = true): every (cell, direction) is first classified by
// the learned indicator of mlp.h, a whole wavefront at a time, and a smooth
// one takes the linear fifth-order stencil for every variable instead of
// WENO5.  ORDER selects the reconstruction otherwise (5 WENO5, 3 WENO3,
// 1 first order; the routed variant is always 5).
#include <type_traits>

#include "charbc.h"
#include "internal.h"
#include "mlp.h"

namespace mfc {
namespace {

// k_xy tile (cells) and workgroup (threads).  The thread count is fixed at
// 256 and may exceed the tile, so that every phase takes a single pass: one
// thread per reconstruction and direction, the same thread then solving the
// face on the reconstruction's + side with its own + value kept in
// registers, so that only the - values pass through LDS.  With a 16 x 13 tile
// the FP64 kernel's LDS (primitives, - values, face fluxes: 51.8 KB) admits
// three workgroups per CU; 16 x 14 needs 54.8 KB and admits two.  Four
// planes per workgroup (more workgroups) measured faster than 8 or 16.
#ifndef MFC_XY_TX
#define MFC_XY_TX 16
#endif
#ifndef MFC_XY_TY
#define MFC_XY_TY 13
#endif
#ifndef MFC_XY_PLANES
#define MFC_XY_PLANES 4
#endif
constexpr int TX = MFC_XY_TX, TY = MFC_XY_TY, NT = 256, NOWN = TX * TY;
static_assert(NOWN <= NT, "one thread per tile cell");
// Halo width of the reconstruction of order ORDER: WENO5 reads two cells
// past the face cell (3-cell halos); WENO3 one (2-cell halos, which first
// order shares: its face problem still needs the neighbour past the face,
// and the z pass keeps three planes so that the updated cell is in the
// window).  OFF is where the stencil of the cell at plane index h starts,
// relative to h - (H - 1): 0 for WENO5 and WENO3, 1 for first order.
template <int ORDER>
constexpr int kHalo = ORDER == 5 ? 3 : 2;
template <int ORDER>
constexpr int kOff = kHalo<ORDER> - 1 - (ORDER - 1) / 2;
static_assert(kHalo<5> <= NG && kHalo<3> <= NG, "halos fit the ghost layers");
constexpr int NPX = (TX + 2) * TY;  // x reconstructions: cells -1 .. TX of every row
constexpr int NPY = TX * (TY + 2);  // y reconstructions: rows -1 .. TY of every column
static_assert(NPX <= NT && NPY <= NT, "one reconstruction per thread and direction");
constexpr int NP = NPX > NPY ? NPX : NPY;
// A face is indexed by the reconstruction on its low side: x face p lies
// between reconstructions p and p + 1 of a row (p % (TX + 2) <= TX), y face p
// between reconstructions p and p + TX (p / TX <= TY).
constexpr int NFX = (TX + 2) * (TY - 1) + TX + 1;
constexpr int NFY = TX * (TY + 1);
constexpr int NF = NFX > NFY ? NFX : NFY;
constexpr int kPlanesXY = MFC_XY_PLANES;  // planes per k_xy workgroup
#ifndef MFC_Z_Y
#define MFC_Z_Y 4
#endif
constexpr int kZX = 64, kZY = MFC_Z_Y;  // k_z workgroup: 64 x 4 columns
#ifndef MFC_Z_LZ64
#define MFC_Z_LZ64 16
#endif
#ifndef MFC_Z_LZ32
#define MFC_Z_LZ32 16
#endif
// planes per k_z column chunk (the march re-reads 6 halo planes per chunk)
template <class T>
constexpr int kLZ = sizeof(T) == 8 ? MFC_Z_LZ64 : MFC_Z_LZ32;

#ifndef MFC_XCD
#define MFC_XCD 1
#endif

// Logical tile of this workgroup.  Workgroup ids are handed to the eight XCDs
// round-robin (id % 8), and each XCD has its own L2; renumbering the tiles so
// that XCD j receives the j-th contiguous range of tiles (x fastest, then y,
// then z) keeps tiles that read each other's halo cells in one L2.  The map
// is a bijection for any grid size, so correctness never depends on it.
__device__ __forceinline__ void tile_of_block(int &bx, int &by, int &bz)
{
    const int gxn = gridDim.x, gyn = gridDim.y;
    int lin = blockIdx.x + gxn * (blockIdx.y + gyn * blockIdx.z);
    if (MFC_XCD) {
        const int n = gxn * gyn * gridDim.z, x = lin % 8, base = n / 8, extra = n % 8;
        lin = x * base + min(x, extra) + lin / 8;
    }
    bx = lin % gxn;
    by = (lin / gxn) % gyn;
    bz = lin / (gxn * gyn);
}

__device__ __forceinline__ int64_t offset(const Grid &g, int i, int j, int k)
{
    return (int64_t)(k + g.off[2]) * g.stride[2] + (int64_t)(j + g.off[1]) * g.stride[1] + (i + g.off[0]);
}

// Both face values of a cell from the ORDER values of its stencil, starting
// at st with stride s (WENO5, WENO3 or first order, Sec. 3.2).
template <int ORDER, class T>
__device__ __forceinline__ void recon_at(const T *st, int s, T eps, T &plus, T &minus)
{
    if constexpr (ORDER == 5) {
        weno5_pair(st[0], st[s], st[2 * s], st[3 * s], st[4 * s], eps, plus, minus);
    } else if constexpr (ORDER == 3) {
        weno3_pair(st[0], st[s], st[2 * s], eps, plus, minus);
    } else {
        plus = st[0];
        minus = st[0];
    }
}

// Characteristic rates (charbc.h) of the boundary cell at plane position
// (r, c) of an LDS plane tile, on face SIDE of dimension D (0: x, 1: y),
// from the cell and the next two cells into the domain.
template <int D, int SIDE, class T, int PY, int PX>
__device__ __forceinline__ bool plane_char_rate(const Grid &g, const T (&pl)[7][PY][PX], int r, int c, T inv_dx,
                                                T *rate)
{
    constexpr int sg = SIDE == 0 ? 1 : -1;
    T W[3][7];
#pragma unroll
    for (int j = 0; j < 3; j++)
#pragma unroll
        for (int v = 0; v < 7; v++) W[j][v] = D == 0 ? pl[v][r][c + sg * j] : pl[v][r + sg * j][c];
    return char_rate<3, D, SIDE, T>(g, W[0], W[1], W[2], inv_dx, one_sided<T>(g, D, SIDE), rate);
}

// A load of data the x+y pass reads once (q^n for its part of the stage
// combination), marked non-temporal so that it does not evict the halo
// cells that neighbouring tiles read from L2 (FP64: 1.2 % faster measured;
// MFC_XY_NT=0 turns it off).
#ifndef MFC_XY_NT
#define MFC_XY_NT 1
#endif
template <class T>
__device__ __forceinline__ T ld_once(const T *p)
{
    if constexpr (MFC_XY_NT != 0) return __builtin_nontemporal_load(p);
    else return *p;
}

// Load and convert cell (i, j, bc_cell(k)) of a column (i, j interior).
template <class T>
__device__ __forceinline__ void load_cons_z(const Grid &g, const T *__restrict__ q, int i, int j, int k, T *qc)
{
    const int64_t c = offset(g, i, j, bc_cell(k, g.n[2], g.bc[4], g.bc[5]));
#pragma unroll
    for (int v = 0; v < 7; v++) qc[v] = q[v * g.vstride + c];
}
template <class T>
__device__ __forceinline__ bool load_prim_z(const Grid &g, const T *__restrict__ q, int i, int j, int k, T *w)
{
    T qc[7];
    load_cons_z<T>(g, q, i, j, k, qc);
    return cons_to_prim<3, T>(g, qc, w);
}

// Feature exchange area of the routed reconstruction: 64 samples x 16 bf16
// per wavefront.  It lives in the flux array, which no thread reads while
// reconstructions are formed, when that array is large enough.
constexpr int kFeatWords = (NT / 64) * 64 * 16;

template <class T, bool ROUTE>
struct RouteLds {
    static constexpr bool in_flux = sizeof(T) * (7 + 1) * NF >= sizeof(uint16_t) * kFeatWords;
    using P = typename std::conditional<ROUTE, mlp::Params, char>::type;
    static constexpr int own_words = (ROUTE && !in_flux) ? kFeatWords : 1;
};

// When smax_partial is not null (the first stage of a CFL step whose wave
// speeds no earlier launch reduced) the kernel also reduces max_d (|u_d| + c)
// over its interior cells, the quantity of the CFL condition (Sec. 1), and
// writes one maximum per workgroup: the step size is then set between this
// launch and the z pass, which is the first to use it.
#ifndef MFC_XY_WAVES32
#define MFC_XY_WAVES32 5
#endif
// the routed variant's LDS (network, feature exchange) admits two workgroups per CU
// non-uniform cells read the tile's coefficient rows from LDS: the FP64
// kernel then fits two workgroups per CU, the FP32 one four
// the FP32 kernel with characteristic faces runs four workgroups per CU (at
// five its boundary rates spill 14 registers; 1.5 % faster measured)
template <class T, bool ROUTE, bool STRETCH = false, bool KEEP = false>
constexpr int kXYWaves = ROUTE ? 2
                               : (STRETCH ? (sizeof(T) == 8 ? 2 : 4)
                                          : (sizeof(T) == 8 ? 3 : (KEEP ? 4 : MFC_XY_WAVES32)));

// The x+y pass holds the stage input of its part of the stage combination
// in registers from the start of each plane and loads q^n late in it
// (FP64, measured faster), or loads both at its end (FP32, whose five
// wavefronts per SIMD leave no registers for them).
#ifndef MFC_XY_HOLD64
#define MFC_XY_HOLD64 1
#endif
template <class T>
constexpr bool kHoldFold = sizeof(T) == 8 ? MFC_XY_HOLD64 : 0;

template <class T, bool ROUTE, int ORDER, bool STRETCH, bool KEEP>
__global__ void __launch_bounds__(NT, (kXYWaves<T, ROUTE, STRETCH, KEEP>))
    k_xy(Grid g, const T *__restrict__ q, const T *q0, T *__restrict__ lxy, int *__restrict__ flag,
         const float *__restrict__ mlpw, float logit_tau, T sqrt_eps, double *__restrict__ smax_partial,
         int mode, int fold, double dt, const double *__restrict__ dt_dev)
{
    constexpr int NV = 7;
    // plane tile with halos of this order's width H; a stencil of ORDER
    // values of the cell at plane column (row) h starts at h - (H - 1) + OFF
    constexpr int H = kHalo<ORDER>, OFF = kOff<ORDER>;
    constexpr int PX = TX + 2 * H, PY = TY + 2 * H, NHALO = 2 * H * (TX + TY);
    using R = RouteLds<T, ROUTE>;
    __shared__ T s_plane[NV][PY][PX];
    __shared__ T s_minus[NV][NP];                    // - face value of every reconstruction
    __shared__ __align__(16) T s_flux[NV + 1][NF];   // flux and face velocity of every face
    __shared__ __align__(16) typename R::P s_mlp;
    __shared__ __align__(16) uint16_t s_feat_own[R::own_words];
    const T eps = T(g.eps);
    // stage combination ca q^n + cb (q + dt L) of the SSP-RK3 stage `mode`
    // (1, 2, 3), formed here for the x+y part when `fold` is set
    const T hdt = T(fold ? (dt_dev ? *dt_dev : dt) : 0.0);
    const T ca = T(mode == 2 ? 0.75 : (mode == 3 ? 1.0 / 3.0 : 0.0));
    const T cb = T(mode == 2 ? 0.25 : (mode == 3 ? 2.0 / 3.0 : 1.0));
    const int lane = threadIdx.x % 64;
    uint16_t *scratch = (R::in_flux ? (uint16_t *)&s_flux[0][0] : s_feat_own) + (threadIdx.x / 64) * 64 * 16;
    if constexpr (ROUTE) mlp::stage_params(s_mlp, nullptr, mlpw, threadIdx.x, NT);  // visible after the first barrier

    const int tid = threadIdx.x;
    const int tx = tid % TX, ty = tid / TX;
    int bx, by, bz;
    tile_of_block(bx, by, bz);
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * kPlanesXY, z1 = min(z0 + kPlanesXY, g.n[2]);
    const int xmax = g.n[0] + H - 1, ymax = g.n[1] + H - 1;
    const int gx = x0 + tx, gy = y0 + ty;
    const bool cell = tid < NOWN;                       // this thread has a tile cell
    const bool own = cell && gx < g.n[0] && gy < g.n[1];
    bool bad = false;
    double smax = 0.0;
    // Each thread loads the conservative values of its own cell and of at
    // most one halo cell of the next plane while the current plane is being
    // processed, so the HBM latency of a plane overlaps a plane of work.
    static_assert(NHALO <= NT, "one halo cell per thread");
    const bool halo = tid < NHALO;
    int hli = 0, hlj = 0;
    if (tid < 2 * H * TY) {
        const int c = tid % (2 * H), row = tid / (2 * H);
        hli = c < H ? c : TX + c;
        hlj = row + H;
    } else {
        const int h2 = tid - 2 * H * TY;
        const int c = h2 % TX, r = h2 / TX;
        hli = c + H;
        hlj = r < H ? r : TY + r;
    }
    // cells past a ragged tile edge load a duplicate whose results are discarded
    const int ox = bc_cell(min(gx, xmax), g.n[0], g.bc[0], g.bc[1]);
    const int oy = bc_cell(min(gy, ymax), g.n[1], g.bc[2], g.bc[3]);
    const int hx = bc_cell(min(x0 + hli - H, xmax), g.n[0], g.bc[0], g.bc[1]);
    const int hy = bc_cell(min(y0 + hlj - H, ymax), g.n[1], g.bc[2], g.bc[3]);
    T qo[NV], qh[NV];
    auto fetch = [&](int k) {
        if (cell) {
            const int64_t c = offset(g, ox, oy, k);
#pragma unroll
            for (int v = 0; v < NV; v++) qo[v] = q[v * g.vstride + c];
        }
        if (halo) {
            const int64_t c = offset(g, hx, hy, k);
#pragma unroll
            for (int v = 0; v < NV; v++) qh[v] = q[v * g.vstride + c];
        }
    };
    fetch(z0);
    // non-uniform cells: the WENO5 coefficient rows of the tile's x cells
    // (-1 .. TX) and y cells (-1 .. TY), in the arithmetic's type, in LDS
    // for every plane (in registers they spill or cost occupancy); visible
    // after the first barrier below
    constexpr bool kLdsCoef = STRETCH && ORDER == 5;
    __shared__ T s_cx[kLdsCoef ? (TX + 2) * kStretchCoef : 1];
    __shared__ T s_cy[kLdsCoef ? (TY + 2) * kStretchCoef : 1];
    if constexpr (kLdsCoef) {
        const bool ux = g.wcoef[0] != nullptr, uy = g.wcoef[1] != nullptr;
        for (int i = tid; i < (TX + 2) * kStretchCoef; i += NT) {
            const int c = i / kStretchCoef, j = i % kStretchCoef;
            s_cx[i] = ux ? T(coef_row(g, 0, x0 - 1 + c)[j]) : T(0);
        }
        for (int i = tid; i < (TY + 2) * kStretchCoef; i += NT) {
            const int r = i / kStretchCoef, j = i % kStretchCoef;
            s_cy[i] = uy ? T(coef_row(g, 1, y0 - 1 + r)[j]) : T(0);
        }
    }

    for (int k = z0; k < z1; k++) {
        // ---- plane k (own cell + x/y halos) into LDS as primitives
        {
            if (cell) {
                T w[NV];
                bad |= cons_to_prim<3, T>(g, qo, w);
#pragma unroll
                for (int v = 0; v < NV; v++) s_plane[v][ty + H][tx + H] = w[v];
                if (smax_partial && own) {
                    double Gam, Pi;
                    mixture<double>(g, double(w[6]), Gam, Pi);
                    const double cs = sqrtT(sound2<double>(Gam, Pi, double(w[0]) + double(w[1]), double(w[5])));
                    if constexpr (STRETCH) {   // non-uniform cells: the largest (|u_d| + c)/dx_d
                        const int ci[3] = {gx, gy, k};
#pragma unroll
                        for (int d = 0; d < 3; d++)
                            smax = __builtin_fmax(smax, (__builtin_fabs(double(w[2 + d])) + cs) * inv_width(g, d, ci[d]));
                    } else {
#pragma unroll
                        for (int d = 0; d < 3; d++) smax = __builtin_fmax(smax, __builtin_fabs(double(w[2 + d])) + cs);
                    }
                }
            }
            if (halo) {
                T w[NV];
                bad |= cons_to_prim<3, T>(g, qh, w);
#pragma unroll
                for (int v = 0; v < NV; v++) s_plane[v][hlj][hli] = w[v];
            }
        }
        __syncthreads();
        // operands of the x+y part of the stage combination: the cell's
        // stage input, copied here before the next plane's fetch replaces it
        // and held in registers to the end of the plane, and q^n, loaded
        // late in the plane (written after the x sweep below; the compiler
        // issues the loads after the last barrier, shortly before their use)
        // so that its traffic does not coincide with the fetch (issued with
        // the fetch, stages 2 and 3 took 5-7 us more).  The copy is kept
        // ahead of the loads that follow it (the empty asm): placed after
        // them, its wait for the fetched values was also a wait for those
        // loads.
        T qc[NV], q0c[NV];
        if (kHoldFold<T> && fold && own) {
#pragma unroll
            for (int v = 0; v < NV; v++) {
                qc[v] = qo[v];
                __asm__ volatile("" : "+v"(qc[v]));
            }
        }
        if (k + 1 < z1) fetch(k + 1);

        // ---- x: thread p reconstructs cell p % (TX + 2) - 1 of row p / (TX + 2)
        // and solves the face on its + side
        T wP[NV];  // + face values of this thread's reconstruction
        {
            const int p = tid;
            const bool valid = p < NPX;
            const int pc = valid ? p : NPX - 1;
            const int row = pc / (TX + 2), c = pc % (TX + 2);
            bool lin = false;
            if constexpr (ROUTE) {  // whole wavefronts classify together
                if (__ballot(valid))
                    lin = mlp::smooth_stencil<T>(s_mlp, scratch, &s_plane[6][row + H][c], &s_plane[0][row + H][c],
                                                 &s_plane[1][row + H][c], &s_plane[5][row + H][c], 1, sqrt_eps,
                                                 logit_tau, lane);
            }
            if (valid) {
                const T *cl = kLdsCoef && g.wcoef[0] ? &s_cx[c * kStretchCoef] : nullptr;
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    const T *st = &s_plane[v][row + H][c + OFF];
                    if (ROUTE && lin) linear5_pair<T>(st[0], st[1], st[2], st[3], st[4], wP[v], s_minus[v][p]);
                    else if (kLdsCoef && cl) weno5_nonuniform_pair<T>(cl, st[0], st[1], st[2], st[3], st[4], eps, wP[v], s_minus[v][p]);
                    else recon_at<ORDER, T>(st, 1, eps, wP[v], s_minus[v][p]);
                }
            }
        }
        __syncthreads();
        {
            const int p = tid, row = p / (TX + 2), c = p % (TX + 2);
            if (p < NPX && c <= TX) {
                T wR[NV], F[NV], uf;
#pragma unroll
                for (int v = 0; v < NV; v++) wR[v] = s_minus[v][p + 1];
                const bool b = hllc<3, 0, T>(g, wP, wR, F, uf);
                bad |= b && (y0 + row < g.n[1]) && (x0 + c <= g.n[0]);
#pragma unroll
                for (int v = 0; v < NV; v++) s_flux[v][p] = F[v];
                s_flux[NV][p] = uf;
            }
        }
        __syncthreads();
        const T idx = STRETCH ? T(inv_width(g, 0, gx)) : T(g.inv_dx[0]);
        const T idy = STRETCH ? T(inv_width(g, 1, gy)) : T(g.inv_dx[1]);
        T L[NV], divu;
        if (cell) {
            const int f = ty * (TX + 2) + tx;
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] = (s_flux[v][f] - s_flux[v][f + 1]) * idx;
            divu = (s_flux[NV][f + 1] - s_flux[NV][f]) * idx;
            if (KEEP && (g.cbc_mask & 3) && own) {
                // the boundary cell of a characteristic x face takes the
                // characteristic rates in place of its x terms (Sec. 3.3),
                // from itself and the next two cells into the domain
                if (gx == 0 && (g.cbc_mask & 1)) {
                    bad |= plane_char_rate<0, 0>(g, s_plane, ty + H, tx + H, idx, L);
                    divu = T(0);
                } else if (gx == g.n[0] - 1 && (g.cbc_mask & 2)) {
                    bad |= plane_char_rate<0, 1>(g, s_plane, ty + H, tx + H, idx, L);
                    divu = T(0);
                }
            }
        }
        // ---- y: thread p reconstructs row p / TX - 1 of column p % TX and
        // solves the face on its + side
        if (kHoldFold<T> && fold && own && mode != 1) {   // q^n of the combination (see above)
            const int64_t c = offset(g, gx, gy, k);
#pragma unroll
            for (int v = 0; v < NV; v++) q0c[v] = ld_once(&q0[v * g.vstride + c]);
        }
        if constexpr (ROUTE && R::in_flux) __syncthreads();  // the x fluxes above are read before the area is reused
        {
            const int p = tid;
            const bool valid = p < NPY;
            const int pc = valid ? p : NPY - 1;
            const int li = pc % TX + H, r = pc / TX;
            bool lin = false;
            if constexpr (ROUTE) {
                if (__ballot(valid))
                    lin = mlp::smooth_stencil<T>(s_mlp, scratch, &s_plane[6][r][li], &s_plane[0][r][li],
                                                 &s_plane[1][r][li], &s_plane[5][r][li], PX, sqrt_eps, logit_tau,
                                                 lane);
            }
            if (valid) {
                const T *cl = kLdsCoef && g.wcoef[1] ? &s_cy[r * kStretchCoef] : nullptr;
#pragma unroll
                for (int v = 0; v < NV; v++) {
                    if (ROUTE && lin)
                        linear5_pair<T>(s_plane[v][r][li], s_plane[v][r + 1][li], s_plane[v][r + 2][li],
                                        s_plane[v][r + 3][li], s_plane[v][r + 4][li], wP[v], s_minus[v][p]);
                    else if (kLdsCoef && cl)
                        weno5_nonuniform_pair<T>(cl, s_plane[v][r][li], s_plane[v][r + 1][li], s_plane[v][r + 2][li],
                                                 s_plane[v][r + 3][li], s_plane[v][r + 4][li], eps, wP[v], s_minus[v][p]);
                    else
                        recon_at<ORDER, T>(&s_plane[v][r + OFF][li], PX, eps, wP[v], s_minus[v][p]);
                }
            }
        }
        __syncthreads();
        {
            const int p = tid, c = p % TX, r = p / TX;
            if (p < NPY && r <= TY) {
                T wR[NV], F[NV], uf;
#pragma unroll
                for (int v = 0; v < NV; v++) wR[v] = s_minus[v][p + TX];
                const bool b = hllc<3, 1, T>(g, wP, wR, F, uf);
                bad |= b && (x0 + c < g.n[0]) && (y0 + r <= g.n[1]);
#pragma unroll
                for (int v = 0; v < NV; v++) s_flux[v][p] = F[v];
                s_flux[NV][p] = uf;
            }
        }
        __syncthreads();
        if (cell) {
            const int f = ty * TX + tx;
            T Ly[NV];
#pragma unroll
            for (int v = 0; v < NV; v++) Ly[v] = (s_flux[v][f] - s_flux[v][f + TX]) * idy;
            T dy = (s_flux[NV][f + TX] - s_flux[NV][f]) * idy;
            if (KEEP && (g.cbc_mask & 12) && own) {   // characteristic y faces, as for x
                if (gy == 0 && (g.cbc_mask & 4)) {
                    bad |= plane_char_rate<1, 0>(g, s_plane, ty + H, tx + H, idy, Ly);
                    dy = T(0);
                } else if (gy == g.n[1] - 1 && (g.cbc_mask & 8)) {
                    bad |= plane_char_rate<1, 1>(g, s_plane, ty + H, tx + H, idy, Ly);
                    dy = T(0);
                }
            }
#pragma unroll
            for (int v = 0; v < NV; v++) L[v] += Ly[v];
            divu += dy;
        }
        if (own) {
            const int64_t c = offset(g, gx, gy, k);
            // the x+y share of the alpha1 row's source, from the cell's own
            // primitives (only this thread writes its cell's LDS slots)
            L[NV - 1] += alpha_source<T>(g, s_plane[NV - 1][ty + H][tx + H], s_plane[NV - 2][ty + H][tx + H]) * divu;
            if (fold) {
                if constexpr (!kHoldFold<T>) {   // loaded here instead (registers are scarcer)
#pragma unroll
                    for (int v = 0; v < NV; v++) qc[v] = q[v * g.vstride + c];
                    if (mode != 1) {
#pragma unroll
                        for (int v = 0; v < NV; v++) q0c[v] = q0[v * g.vstride + c];
                    }
                }
                if (mode != 1) {
#pragma unroll
                    for (int v = 0; v < NV; v++) lxy[v * g.vstride + c] = ca * q0c[v] + cb * (qc[v] + hdt * L[v]);
                } else {
#pragma unroll
                    for (int v = 0; v < NV; v++) lxy[v * g.vstride + c] = qc[v] + hdt * L[v];
                }
            } else {
#pragma unroll
                for (int v = 0; v < NV; v++) lxy[v * g.vstride + c] = L[v];
            }
        }
        // The next plane overwrites s_plane, s_minus and s_flux only after
        // zero, one and two more barriers.  s_plane is last read before the
        // y-face barrier, except by the characteristic rate of a y face's
        // boundary cells above, which reads the next two rows (other
        // threads' slots): a workgroup whose tile has such cells waits here
        // (the condition is the same for all its threads).
        if (KEEP && (g.cbc_mask & 12) &&
            (((g.cbc_mask & 4) && y0 == 0) || ((g.cbc_mask & 8) && y0 + TY >= g.n[1])))
            __syncthreads();
    }
    if (smax_partial) {
        // workgroup maximum: wavefront butterflies, then one value per wavefront
        __shared__ double s_red[NT / 64];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) smax = __builtin_fmax(smax, __shfl_xor(smax, o, 64));
        if (lane == 0) s_red[tid / 64] = smax;
        __syncthreads();
        if (tid == 0) {
            double m = s_red[0];
#pragma unroll
            for (int w = 1; w < NT / 64; w++) m = __builtin_fmax(m, s_red[w]);
            smax_partial[((int64_t)blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x] = m;
        }
    }
    if (bad) atomicOr(flag, 1);
}

// z direction + stage update.  Threads of a workgroup own a 64 x 4 block of
// columns (64 consecutive x per wavefront: coalesced plane loads) and march
// through kLZ planes, starting two planes early to reconstruct cell z0-1 and
// solve face z0-1/2 without writing.  Of the five planes of a column's
// reconstruction window, the kRing oldest are kept in a per-thread ring in
// LDS (each thread touches only its own slots: no barriers) and the others in
// registers, which leaves the registers to the reconstruction and the
// Riemann solve (the FP64 kernel spilled with the whole window in registers).
#ifndef MFC_Z_WAVES64
#define MFC_Z_WAVES64 2
#endif
#ifndef MFC_Z_WAVES32
#define MFC_Z_WAVES32 3
#endif
#ifndef MFC_Z_RING
#define MFC_Z_RING 4
#endif
#ifndef MFC_Z_EARLY64
#define MFC_Z_EARLY64 1
#endif
#ifndef MFC_Z_EARLY32
#define MFC_Z_EARLY32 1
#endif
#ifndef MFC_Z_RING_ROUTE
#define MFC_Z_RING_ROUTE 1
#endif
// odd z chunks marched downward (see k_z)
#ifndef MFC_Z_ALT
#define MFC_Z_ALT 1
#endif

template <class T>
constexpr int kZWaves = sizeof(T) == 8 ? MFC_Z_WAVES64 : MFC_Z_WAVES32;
// FP64 with characteristic faces, and the FP64 variant that re-reads its
// stage input, load them late: the z-face terms or the second stage-input
// read leave no registers for them (15 and 20 spilled otherwise)
template <class T, bool KEEP, bool REREAD>
constexpr bool kZEarly = sizeof(T) == 8 ? (MFC_Z_EARLY64 && !KEEP && !REREAD) : MFC_Z_EARLY32;
// the routed variant keeps LDS for the network and its feature exchange
template <bool ROUTE>
constexpr int kRing = ROUTE ? MFC_Z_RING_ROUTE : MFC_Z_RING;
static_assert(kRing<false> >= 1 && kRing<false> <= 4 && kRing<true> >= 1 && kRing<true> <= 4,
              "one to four planes in the ring");

// REREAD: the first stage of a CFL step, whose x+y pass could not form its
// part of the stage combination (dt unknown then): out = q + dt (L_xy + L_z),
// reading the stage input again.  Otherwise out = (x+y part) + s L_z with
// s = cb dt (a folded stage) or 1 (a bare right-hand side).
// SMAX (the last stage of a step followed by another CFL step in the same
// run): the kernel also reduces the wave speeds of the state it writes, the
// next step's q^n, exactly as the x+y pass of a first stage does from the
// stored values (the same conversion in the same arithmetic, so the same
// maxima), one partial maximum per wavefront in smax_partial.
template <class T, bool ROUTE, int ORDER, bool STRETCH, bool KEEP, bool REREAD, bool SMAX = false>
__global__ void __launch_bounds__(kZX * kZY, kZWaves<T>)
    k_z(Grid g, const T *__restrict__ q, T *__restrict__ out, const T *__restrict__ lxy, int mode, double dt,
        const double *__restrict__ dt_dev, int *__restrict__ flag, const float *__restrict__ mlpw, float logit_tau,
        T sqrt_eps, double *__restrict__ smax_partial)
{
    static_assert(!(SMAX && REREAD), "the wave speeds are reduced in a step's last stage");
    // window of W = 2H - 1 planes; the kRing oldest in the LDS ring
    constexpr int H = kHalo<ORDER>, OFF = kOff<ORDER>, W = 2 * H - 1;
    constexpr int kRing = mfc::kRing<ROUTE> < W - 1 ? mfc::kRing<ROUTE> : W - 1, kZReg = W - kRing;
    constexpr int NV = 7, A = 6, NZT = kZX * kZY;
    const T eps = T(g.eps), idz_u = T(g.inv_dx[2]);
    int bx, by, bz;
    tile_of_block(bx, by, bz);
    int gx = bx * kZX + threadIdx.x % kZX;
    int gy = by * kZY + threadIdx.x / kZX;
    const bool own = gx < g.n[0] && gy < g.n[1];
    __shared__ __align__(16) typename std::conditional<ROUTE, mlp::Params, char>::type s_mlp;
    __shared__ __align__(16) uint16_t s_feat[ROUTE ? NZT * 16 : 1];
    __shared__ T s_ring[kRing][NV][NZT];
    if constexpr (ROUTE || SMAX) {
        // every lane of a wavefront takes part in the classification or the
        // reduction: lanes past a ragged edge march a duplicate of the last
        // column (their maxima are those of that column)
        if constexpr (ROUTE) {
            mlp::stage_params(s_mlp, nullptr, mlpw, threadIdx.x, NZT);
            __syncthreads();
        }
        gx = min(gx, g.n[0] - 1);
        gy = min(gy, g.n[1] - 1);
    } else if (!own) {
        return;   // no barriers in this variant
    }
    double smax = 0.0;
    uint16_t *scratch = s_feat + (ROUTE ? (threadIdx.x / 64) * 64 * 16 : 0);
    const int lane = threadIdx.x % 64, t = threadIdx.x;
    const int z0 = bz * kLZ<T>, z1 = min(z0 + kLZ<T>, g.n[2]);
    const T hdt = T(mode ? (dt_dev ? *dt_dev : dt) : 0.0);
    const T cb = T(mode == 2 ? 0.25 : (mode == 3 ? 2.0 / 3.0 : 1.0));
    const T sz = mode ? cb * hdt : T(1);   // weight of L_z in the result
    bool bad = false;

    // The chunk is marched upward (S = +1) or downward (S = -1), alternately
    // from chunk to chunk, so that two neighbouring chunks read the planes
    // they share at about the same time (both at the end of their marches,
    // or both at the start), while those planes are still in L2.  A cell's
    // arithmetic is the same either way: the reconstruction of a cell from
    // its five planes in increasing z, each face solved once with its lower
    // cell on the left.
    //
    // At step k (the cell updated), the window holds the W planes around
    // cell k + S: planes k + S - (H - 1) .. k + S + (H - 1) (for WENO5
    // k - 1 .. k + 3 if S = +1, k - 3 .. k + 1 if S = -1).  Window position
    // i (0 = oldest plane, W - 1 = the newest, plane k + S H) is ring slot
    // rs[i] for i < kRing, else zr[i - kRing]; window index j (0 = lowest z)
    // is position j (S = +1) or W - 1 - j (S = -1).
    int rs[kRing];
    T zr[kZReg][NV];
    T ck[NV];      // cell k at its face toward the march: + face (S = +1), - face (S = -1)
    T Fz[NV + 1];  // flux and face velocity at the face of cell k behind the march
    auto march = [&](auto dir) {
        constexpr int S = decltype(dir)::value;
        auto win = [&](int j, int v) -> T {
            const int i = S > 0 ? j : W - 1 - j;
            return i < kRing ? s_ring[rs[i]][v][t] : zr[i - kRing][v];
        };
        const int kfirst = S > 0 ? z0 - 2 : z1 + 1;
        // the W - 1 oldest planes of the first window: plane kfirst + S + S (i - (H - 1))
#pragma unroll
        for (int i = 0; i < kRing; i++) {
            rs[i] = i;
            bad |= load_prim_z<T>(g, q, gx, gy, kfirst + S * (i + 2 - H), zr[kZReg - 1]);
#pragma unroll
            for (int v = 0; v < NV; v++) s_ring[i][v][t] = zr[kZReg - 1][v];
        }
#pragma unroll
        for (int i = kRing; i < W - 1; i++) bad |= load_prim_z<T>(g, q, gx, gy, kfirst + S * (i + 2 - H), zr[i - kRing]);

        const int steps = z1 - z0 + 2;
        for (int st = 0; st < steps; st++) {
            const int k = kfirst + S * st;
            bad |= load_prim_z<T>(g, q, gx, gy, k + H * S, zr[kZReg - 1]);
            // the operands of the stage update of cell k are loaded before the
            // reconstruction so that their latency overlaps it (FP64: 3-5 us
            // per launch faster measured, although the wave-speed-reducing
            // variant then spills a few registers)
            T lx[NV], qb[NV];
            auto load_update = [&](int64_t c) {
#pragma unroll
                for (int v = 0; v < NV; v++) lx[v] = lxy[v * g.vstride + c];
                if constexpr (REREAD) {
#pragma unroll
                    for (int v = 0; v < NV; v++) qb[v] = q[v * g.vstride + c];
                }
            };
            const bool upd = st >= 2 && own;   // cell k is in the chunk
            if constexpr (kZEarly<T, KEEP, REREAD>) {
                if (upd) load_update(offset(g, gx, gy, k));
            }
            T pn[NV], mn[NV], Fzn[NV + 1];
            bool lin = false;
            if constexpr (ROUTE) {
                T av[5], rv[5], pv[5];
#pragma unroll
                for (int j = 0; j < 5; j++) {
                    av[j] = win(j, A);
                    rv[j] = win(j, 0) + win(j, 1);
                    pv[j] = win(j, 5);
                }
                uint16_t f[16];
                mlp::features<T>(av, rv, pv, sqrt_eps, f);
                lin = mlp::smooth_wave(s_mlp, scratch, f, logit_tau, lane);
            }
            CoefRegs<T> cf;   // cell k + S of this window
            if constexpr (STRETCH && ORDER == 5) load_coefs<T>(coef_row(g, 2, k + S), cf);
#pragma unroll
            for (int v = 0; v < NV; v++) {
                T st[ORDER];   // the stencil of cell k + S, lowest z first
#pragma unroll
                for (int j = 0; j < ORDER; j++) st[j] = win(OFF + j, v);
                if constexpr (ORDER == 5) {
                    if (ROUTE && lin) linear5_pair<T>(st[0], st[1], st[2], st[3], st[4], pn[v], mn[v]);
                    else if (STRETCH) recon_cell<ORDER, T>(cf, st[0], st[1], st[2], st[3], st[4], eps, pn[v], mn[v]);
                    else recon_at<ORDER, T>(st, 1, eps, pn[v], mn[v]);
                } else {
                    recon_at<ORDER, T>(st, 1, eps, pn[v], mn[v]);
                }
            }
            // the face between cells k and k + S (the first step's is not needed)
            if (st >= 1) {
                if constexpr (S > 0) bad |= hllc<3, 2, T>(g, ck, mn, Fzn, Fzn[NV]);
                else bad |= hllc<3, 2, T>(g, pn, ck, Fzn, Fzn[NV]);
            }
            // The face's values as rounded, before any use: a value that
            // ends in a product (alpha1 u_face, u_face itself) would
            // otherwise be fused into the flux difference of this step's
            // cell but enter the next cell's difference rounded, and the
            // face would not cancel between the two (a uniform state would
            // not give a zero right-hand side).
#pragma unroll
            for (int v = 0; v <= NV; v++) __asm__ volatile("" : "+v"(Fzn[v]));
#pragma unroll
            for (int v = 0; v < NV; v++) ck[v] = S > 0 ? pn[v] : mn[v];
            if (upd) {
                const int64_t c = offset(g, gx, gy, k);
                const T idz = STRETCH ? T(inv_width(g, 2, k)) : idz_u;
                // fluxes at k - 1/2 and k + 1/2
                const T *Flo = S > 0 ? Fz : Fzn, *Fhi = S > 0 ? Fzn : Fz;
                T L[NV], divu;
                if (KEEP && (g.cbc_mask & 48)) {   // characteristic z faces keep the boundary cells' z terms
                    T Lz[NV];
#pragma unroll
                    for (int v = 0; v < NV; v++) Lz[v] = (Flo[v] - Fhi[v]) * idz;
                    const T dz = (Fhi[NV] - Flo[NV]) * idz;
                    if (k == 0 && (g.cbc_mask & 16)) store_normal_terms<4, T>(g, gx, g.n[0], gy, Lz, dz);
                    if (k == g.n[2] - 1 && (g.cbc_mask & 32)) store_normal_terms<5, T>(g, gx, g.n[0], gy, Lz, dz);
                }
                // every operand before the first store (here when they are
                // not loaded early)
                if constexpr (!kZEarly<T, KEEP, REREAD>) load_update(c);
#pragma unroll
                for (int v = 0; v < NV; v++) L[v] = (Flo[v] - Fhi[v]) * idz;
                divu = (Fhi[NV] - Flo[NV]) * idz;
                L[A] += alpha_source<T>(g, win(H - 1 - S, A), win(H - 1 - S, A - 1)) * divu;   // the z share of the source
                if constexpr (REREAD) {
#pragma unroll
                    for (int v = 0; v < NV; v++) out[v * g.vstride + c] = qb[v] + hdt * (lx[v] + L[v]);
                } else {
                    T r[NV];
#pragma unroll
                    for (int v = 0; v < NV; v++) {
                        r[v] = lx[v] + sz * L[v];
                        out[v * g.vstride + c] = r[v];
                    }
                    // |u_d| + c of the stored state (non-uniform cells: over dx_d);
                    // the cells of characteristic z faces are left to the
                    // boundary pass, which changes them after this kernel
                    const bool zface = KEEP && ((k == 0 && (g.cbc_mask & 16)) || (k == g.n[2] - 1 && (g.cbc_mask & 32)));
                    if (SMAX && !zface) {
                        T w[NV];
                        cons_to_prim<3, T>(g, r, w);
                        double Gam, Pi;
                        mixture<double>(g, double(w[6]), Gam, Pi);
                        const double cs = sqrtT(sound2<double>(Gam, Pi, double(w[0]) + double(w[1]), double(w[5])));
                        const int ci[3] = {gx, gy, k};
#pragma unroll
                        for (int d = 0; d < 3; d++) {
                            const double a = __builtin_fabs(double(w[2 + d])) + cs;
                            smax = __builtin_fmax(smax, STRETCH ? a * inv_width(g, d, ci[d]) : a);
                        }
                    }
                }
            }
#pragma unroll
            for (int v = 0; v <= NV; v++) Fz[v] = Fzn[v];
            // shift the window: the oldest plane in registers replaces the
            // oldest plane of the ring
#pragma unroll
            for (int v = 0; v < NV; v++) {
                s_ring[rs[0]][v][t] = zr[0][v];
#pragma unroll
                for (int j = 0; j + 1 < kZReg; j++) zr[j][v] = zr[j + 1][v];
            }
            const int r = rs[0];
#pragma unroll
            for (int j = 0; j + 1 < kRing; j++) rs[j] = rs[j + 1];
            rs[kRing - 1] = r;
        }
    };
    if (MFC_Z_ALT && (bz & 1)) march(std::integral_constant<int, -1>{});
    else march(std::integral_constant<int, 1>{});
    if constexpr (SMAX) {   // wavefront maximum, one partial per wavefront
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) smax = __builtin_fmax(smax, __shfl_xor(smax, o, 64));
        if (lane == 0)
            smax_partial[((int64_t)(blockIdx.z * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x) * kZY + t / 64] = smax;
    }
    if (bad) atomicOr(flag, 1);
}

dim3 xy_grid(const Grid &g)
{
    return dim3((g.n[0] + TX - 1) / TX, (g.n[1] + TY - 1) / TY, (g.n[2] + kPlanesXY - 1) / kPlanesXY);
}

template <class T, bool ROUTE, int ORDER, bool STRETCH = false, bool KEEP = false>
int rhs_split(mfc_grid *h, const T *q, const T *q0, T *out, int mode, double dt, const double *dt_dev, hipStream_t s,
              double cfl, double *zmax)
{
    const Grid &g = h->g;
    const dim3 gxy = xy_grid(g);
    dim3 gz((g.n[0] + kZX - 1) / kZX, (g.n[1] + kZY - 1) / kZY, (g.n[2] + kLZ<T> - 1) / kLZ<T>);
    T *lxy = (T *)h->lxy;
    const T se = T(__builtin_sqrt(g.eps));
    double *partial = cfl > 0.0 ? h->partial : nullptr;
    // the x+y pass forms its part of the stage combination whenever the
    // stage's dt is known before it runs (not in a first stage whose dt is
    // set from that pass's own wave-speed maxima)
    const int fold = mode != 0 && !partial;
    timing_begin(h, s);
    hipLaunchKernelGGL((k_xy<T, ROUTE, ORDER, STRETCH, KEEP>), gxy, dim3(NT), 0, s, g, q, q0, lxy, h->flag, h->mlp,
                       h->logit_tau, se, partial, mode, fold, dt, dt_dev);
    timing_end(h, s);
    if (partial) launch_step_begin(h, partial, (int)split_xy_blocks(g), cfl, 0.0, s);
    timing_begin(h, s, 1);
    bool done = false;
    if (zmax && mode != 0 && fold) {
        hipLaunchKernelGGL((k_z<T, ROUTE, ORDER, STRETCH, KEEP, false, true>), gz, dim3(kZX * kZY), 0, s, g, q, out,
                           lxy, mode, dt, dt_dev, h->flag, h->mlp, h->logit_tau, se, zmax);
        done = true;
    }
    if (done) {
    } else if (mode != 0 && !fold) {
        hipLaunchKernelGGL((k_z<T, ROUTE, ORDER, STRETCH, KEEP, true>), gz, dim3(kZX * kZY), 0, s, g, q, out, lxy, mode,
                           dt, dt_dev, h->flag, h->mlp, h->logit_tau, se, nullptr);
    } else {
        hipLaunchKernelGGL((k_z<T, ROUTE, ORDER, STRETCH, KEEP, false>), gz, dim3(kZX * kZY), 0, s, g, q, out, lxy, mode,
                           dt, dt_dev, h->flag, h->mlp, h->logit_tau, se, nullptr);
    }
    timing_end(h, s, 1);
    return hip_status(hipGetLastError(), "split right-hand side launch");
}

// The right-hand side (mode 0) on a grid with no handle: uniform cells,
// extrapolated or periodic boundaries, WENO5, WENO3 or first order; the x+y
// part goes to the caller's `lxy` (nvar arrays of the padded grid) and
// non-physical cells set *flag.
template <class T, int ORDER>
int rhs_split_raw(const Grid &g, const T *q, T *out, T *lxy, int *flag, hipStream_t s)
{
    const dim3 gxy = xy_grid(g);
    const dim3 gz((g.n[0] + kZX - 1) / kZX, (g.n[1] + kZY - 1) / kZY, (g.n[2] + kLZ<T> - 1) / kLZ<T>);
    const T se = T(__builtin_sqrt(g.eps));
    hipLaunchKernelGGL((k_xy<T, false, ORDER, false, false>), gxy, dim3(NT), 0, s, g, q, q, lxy, flag, nullptr, 0.f,
                       se, nullptr, 0, 0, 0.0, nullptr);
    hipLaunchKernelGGL((k_z<T, false, ORDER, false, false, false>), gz, dim3(kZX * kZY), 0, s, g, q, out, lxy, 0, 0.0,
                       nullptr, flag, nullptr, 0.f, se, nullptr);
    return hip_status(hipGetLastError(), "split right-hand side launch");
}

}  // namespace

int launch_rhs_split_raw(const Grid &g, bool fp32, const void *q, void *out, void *lxy, int *flag, hipStream_t s)
{
    if (g.ndim != 3 || g.stretched || g.cbc_mask) return fail(MFC_E_UNSUPPORTED, "3D uniform cells only");
    if (fp32) {
        const float *fq = (const float *)q;
        float *fo = (float *)out, *fl = (float *)lxy;
        if (g.order == 3) return rhs_split_raw<float, 3>(g, fq, fo, fl, flag, s);
        if (g.order == 1) return rhs_split_raw<float, 1>(g, fq, fo, fl, flag, s);
        return rhs_split_raw<float, 5>(g, fq, fo, fl, flag, s);
    }
    const double *dq = (const double *)q;
    double *dout = (double *)out, *dl = (double *)lxy;
    if (g.order == 3) return rhs_split_raw<double, 3>(g, dq, dout, dl, flag, s);
    if (g.order == 1) return rhs_split_raw<double, 1>(g, dq, dout, dl, flag, s);
    return rhs_split_raw<double, 5>(g, dq, dout, dl, flag, s);
}

int64_t split_xy_blocks(const Grid &g)
{
    const dim3 b = xy_grid(g);
    return (int64_t)b.x * b.y * b.z;
}

int64_t split_z_partials(const Grid &g, bool fp32)
{
    const int lz = fp32 ? kLZ<float> : kLZ<double>;
    return (int64_t)((g.n[0] + kZX - 1) / kZX) * ((g.n[1] + kZY - 1) / kZY) * ((g.n[2] + lz - 1) / lz) * kZY;
}

int launch_rhs_split(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt,
                     const double *dt_dev, hipStream_t s, double cfl, double *zmax)
{
    if (h->g.ndim != 3) return fail(MFC_E_UNSUPPORTED, "the split path is 3D only");
    const bool learned = h->desc.recon == MFC_RECON_LEARNED;
    if (learned && !h->mlp) return fail(MFC_E_ARG, "MFC_RECON_LEARNED needs mfc_set_indicator first");
    const float *fq = (const float *)q, *fq0 = (const float *)q0;
    const double *dq = (const double *)q, *dq0 = (const double *)q0;
    float *fo = (float *)out;
    double *dout = (double *)out;
    const bool f32 = h->desc.precision == MFC_FP32_MIXED;
    if (h->g.stretched && h->g.cbc_mask) {   // non-uniform cells with characteristic faces
        if (h->desc.recon == MFC_RECON_FIRST_ORDER)
            return f32 ? rhs_split<float, false, 1, true, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                       : rhs_split<double, false, 1, true, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
        return f32 ? rhs_split<float, false, 5, true, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, false, 5, true, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    }
    if (h->g.stretched) {   // non-uniform cells: WENO5 or first order (checked at init)
        if (h->desc.recon == MFC_RECON_FIRST_ORDER)
            return f32 ? rhs_split<float, false, 1, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                       : rhs_split<double, false, 1, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
        return f32 ? rhs_split<float, false, 5, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, false, 5, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    }
    if (h->g.cbc_mask) {   // characteristic faces (WENO5, WENO3, first order or routed; checked at init)
        if (learned)
            return f32 ? rhs_split<float, true, 5, false, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                       : rhs_split<double, true, 5, false, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
        if (h->desc.recon == MFC_RECON_WENO3)
            return f32 ? rhs_split<float, false, 3, false, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                       : rhs_split<double, false, 3, false, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
        if (h->desc.recon == MFC_RECON_FIRST_ORDER)
            return f32 ? rhs_split<float, false, 1, false, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                       : rhs_split<double, false, 1, false, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
        return f32 ? rhs_split<float, false, 5, false, true>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, false, 5, false, true>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    }
    switch (h->desc.recon) {
    case MFC_RECON_LEARNED:
        return f32 ? rhs_split<float, true, 5>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, true, 5>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    case MFC_RECON_WENO3:
        return f32 ? rhs_split<float, false, 3>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, false, 3>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    case MFC_RECON_FIRST_ORDER:
        return f32 ? rhs_split<float, false, 1>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, false, 1>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    default:
        return f32 ? rhs_split<float, false, 5>(h, fq, fq0, fo, mode, dt, dt_dev, s, cfl, zmax)
                   : rhs_split<double, false, 5>(h, dq, dq0, dout, mode, dt, dt_dev, s, cfl, zmax);
    }
}

}  // namespace mfc
