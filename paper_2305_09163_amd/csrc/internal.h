// Internal declarations shared by the library's translation units: the grid
// handle, kernel launchers and status helpers.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/mfc.h"
#include "physics.h"

struct mfc_grid {
    mfc_grid_desc desc;
    mfc::Grid g;           // device-side geometry/material constants
    int nvar;
    int64_t cells_padded;  // px * py * pz
    int64_t cells;         // interior cells
    int device;
    int cu_count;          // compute units of the device (resident-workgroup sizing)

    // scratch owned by the handle (device memory)
    void *stage_a = nullptr;   // RK stage state q^(1)
    void *stage_b = nullptr;   // RK stage state q^(2)
    double *prim = nullptr;    // staged path: primitive state (padded layout)
    double *recp = nullptr;    // staged path: reconstruction at x_{i+1/2}, per cell
    double *recm = nullptr;    // staged path: reconstruction at x_{i-1/2}, per cell
    double *faces = nullptr;   // staged path: 3 directions x (nvar + 1) face arrays
    double *lxy = nullptr;     // split path: x+y part of each cell's right-hand side or stage result, nvar arrays
    void *cbc_fv = nullptr;    // split path: normal terms of characteristic boundary cells
    double *partial = nullptr; // per-block maxima of the wave-speed reduction
    int64_t partial_len = 0;   // its length (the larger of the two producers' grids)
    double *scalars = nullptr; // [0] smax, [1] dt, [2] t, [3] spare
    int *flag = nullptr;       // non-physical flag
    float *mlp = nullptr;      // learned indicator parameters (FP32, flat order of mlp.h)
    float logit_tau = 0.0f;    // routing threshold on the indicator's logit

    // kernel timing, per slot (0: main right-hand-side kernel, 1: z kernel);
    // stride N records the launches of every N-th step (timing_step counts
    // the steps since timing was enabled; timing_skip is set for the others)
    bool timing = false;
    int timing_stride = 1;
    int64_t timing_step = 0;
    bool timing_skip = false;
    std::vector<hipEvent_t> ev[2];  // pairs (start, stop)
    size_t ev_used[2] = {0, 0};
};

namespace mfc {

constexpr int kReduceBlocks = 1024;
constexpr int kReduceThreads = 256;

// status helpers
int fail(int status, const char *detail);
int fail(int status, const std::string &detail);
// Kapila coefficients of a grid from its descriptor (model, gamma, pi_inf)
void set_kapila(Grid &g, const mfc_grid_desc &d);
// The kernels' geometry and material constants of a validated descriptor
// (host only; no device tables: non-uniform and characteristic-boundary
// fields are left empty)
void make_grid(const mfc_grid_desc &d, Grid &g);
// Checks of mfc_init_grid on a descriptor (MFC_OK or the failure status)
int validate_desc(const mfc_grid_desc *d);
// Device tables of a non-uniform grid (stretch.hip): built at init from the
// descriptor's face coordinates, released with the handle.
int build_stretch_tables(mfc_grid *h, const mfc_grid_desc *d);
// Characteristic boundaries (cbc.hip): whether a face has one, and the
// post-pass that replaces the boundary cells' normal terms in `out` (the
// right-hand side for mode 0, else the stage result of that mode).
// smax_partial non-null (the split path's last stage of a step followed by
// another of the same run): the pass also writes the wave-speed maxima of the
// cells it changes, cbc_stored_blocks(g) of them.
bool has_cbc(const mfc_grid *h);
int launch_cbc(mfc_grid *h, const void *q, void *out, int mode, double dt, const double *dt_dev, hipStream_t s,
               double *smax_partial = nullptr);
// Workgroups of the split path's boundary pass (the z faces' cells).
int64_t cbc_stored_blocks(const Grid &g);
void free_stretch_tables(mfc_grid *h);
int hip_status(hipError_t e, const char *what);

// kernel timing: bracket one launch of the dominant kernel
void timing_begin(mfc_grid *h, hipStream_t s, int slot = 0);
void timing_end(mfc_grid *h, hipStream_t s, int slot = 0);

// Launchers.  `q` has ghosts filled.  mode 0: out = rhs; mode s = 1, 2, 3:
// out = a_s q0 + b_s (q + dt rhs) with the SSP-RK3 stage coefficients.
// dt is *dt_dev if dt_dev is non-null, else dt.  Arrays hold double for
// MFC_FP64 and float for MFC_FP32_MIXED.
int launch_rhs_staged(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt,
                      const double *dt_dev, hipStream_t s);
int launch_rhs_fused(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt,
                     const double *dt_dev, hipStream_t s);
// Split path: cfl > 0 reduces the wave speeds of q in the x+y pass and sets
// the step size before the z pass (the first stage of a CFL step); zmax
// non-null (a last stage) has the z pass reduce the wave speeds of the state
// it writes into zmax, split_z_partials(g) maxima for the next step.
int launch_rhs_split(mfc_grid *h, const void *q, const void *q0, void *out, int mode, double dt,
                     const double *dt_dev, hipStream_t s, double cfl = 0.0, double *zmax = nullptr);

// Split right-hand side (mode 0) without a handle: 3D uniform cells,
// WENO5/WENO3/first order as g.order says, no learned routing and no
// characteristic faces; lxy holds nvar arrays of the padded grid in the
// storage type.
int launch_rhs_split_raw(const Grid &g, bool fp32, const void *q, void *out, void *lxy, int *flag, hipStream_t s);

// Split path: number of x+y workgroups of one launch (each writes one
// wave-speed partial when the step size is computed inside the launch).
int64_t split_xy_blocks(const Grid &g);
// Split path: number of wave-speed partials the z pass writes (one per wavefront).
int64_t split_z_partials(const Grid &g, bool fp32);

// Reduce nblocks partial maxima, set the step size (cfl > 0: from the
// maxima; else dt) and advance the accumulated time, on the device.
void launch_step_begin(mfc_grid *h, const double *partial, int nblocks, double cfl, double dt, hipStream_t s);

}  // namespace mfc
