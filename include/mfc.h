/*
 * mfc.h - C ABI of the MI355X (gfx950) right-hand side of the two-fluid
 * five-equation diffuse-interface model.
 *
 * The operations are those of the paper's numerical method:
 *   - governing equations (Sec. 2.1): partial densities alpha1 rho1 and
 *     alpha2 rho2, mixture momentum, total energy, and the volume fraction
 *     alpha1 advected with the non-conservative alpha1 div(u) term; the
 *     Allaire form (K div(u) dropped, the default) or the Kapila form
 *     (u . grad(alpha1) = K div(u), MFC_MODEL_KAPILA);
 *   - stiffened-gas EOS per fluid (Sec. 2.1, eq. soe) mixed at pressure
 *     equilibrium: rho E = Gamma p + Pi + rho |u|^2/2 with
 *     Gamma = sum alpha_k/(gamma_k - 1), Pi = sum alpha_k gamma_k pi_k/(gamma_k - 1);
 *   - finite-volume semi-discretisation (Sec. 3.1, eqs. fvm and fvmdis);
 *   - WENO5-JS reconstruction of primitive variables (Sec. 3.2);
 *   - HLLC fluxes and face velocities (Sec. 3.2.1);
 *   - boundary buffers (Sec. 3.3), third-order TVD Runge-Kutta (Sec. 3.4)
 *     and the CFL time step (Sec. 1).
 *
 * Data layout.  A state is nvar = 4 + ndim arrays, variable-major, each
 * x-fastest over the padded grid (px, py, pz) = n + 6 on active dimensions
 * (3 ghost cells per side) and 1 on inactive ones:
 *     element (v, k, j, i) at offset ((v * pz + k) * py + j) * px + i.
 * Conservative ordering: [alpha1 rho1, alpha2 rho2, rho u_1 .. rho u_ndim,
 * rho E, alpha1].  Primitive ordering: [alpha1 rho1, alpha2 rho2,
 * u_1 .. u_ndim, p, alpha1].  Element type is double for MFC_FP64 and float
 * for MFC_FP32_MIXED.
 *
 * Ownership.  State arrays (q, rhs, w) are device memory owned by the
 * caller; the library never frees them and never keeps a pointer past the
 * call.  The grid handle owns all scratch memory from mfc_init_grid to
 * mfc_free_grid.  Work is enqueued on the caller's stream (a hipStream_t
 * passed as void*, NULL = the null stream); only calls documented as
 * synchronising wait for it.  A handle must not be used from two host
 * threads or two streams at once.
 *
 * Errors.  Every call returns MFC_OK (0) or a negative code; arguments are
 * validated on the host before anything is enqueued, and no exception
 * crosses the ABI.  mfc_strerror gives a message; mfc_last_error_detail gives
 * the detail of the last failure on the calling thread.
 */
#ifndef MFC_H
#define MFC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MFC_OK = 0,
    MFC_E_ARG = -1,          /* invalid argument (null pointer, bad size, bad value) */
    MFC_E_NOMEM = -2,        /* device allocation failed                              */
    MFC_E_HIP = -3,          /* a HIP runtime call or kernel launch failed            */
    MFC_E_NONPHYSICAL = -4,  /* a cell had rho <= 0, c^2 <= 0 or a non-finite value   */
    MFC_E_UNSUPPORTED = -5   /* valid request the library does not implement         */
};

/* Boundary condition per face.  EXTRAP: ghost cells copy the adjacent
 * interior cell; PERIODIC: the cell one period away (both faces of a
 * dimension); CHARACTERISTIC: non-reflecting characteristic boundary
 * (Sec. 3.3, Thompson's time-dependent form): ghost cells as for EXTRAP,
 * and on each boundary cell the finite-volume terms normal to the face are
 * replaced by the characteristic form of the one-dimensional system, with
 * wave amplitudes from second-order one-sided differences of the primitives
 * (on non-uniform cells, the derivative of the quadratic through the
 * boundary cell's centre and the next two) and every amplitude whose wave
 * enters the domain set to zero (Allaire model; with the learned routing on
 * the split kernel only). */
enum { MFC_BC_EXTRAP = 0, MFC_BC_PERIODIC = 1, MFC_BC_CHARACTERISTIC = 2 };
enum { MFC_FP64 = 0, MFC_FP32_MIXED = 1 };
/* Reconstruction of the primitive variables at the faces (Sec. 3.2):
 * WENO5-JS (the default), the learned routing between WENO5 and its linear
 * fifth-order stencil (see mfc_set_indicator), WENO3-JS (two candidate
 * stencils, ideal weights 1/3, 2/3 and their mirror, beta_r the squared
 * one-sided differences, alpha_r = d_r/(eps + beta_r)^2), or first order
 * (the cell value at both faces).  All of them read the same 3-cell ghost
 * layers. */
enum { MFC_RECON_WENO5 = 0, MFC_RECON_LEARNED = 1, MFC_RECON_WENO3 = 2, MFC_RECON_FIRST_ORDER = 3 };

/* Volume-fraction equation (Sec. 2.1).  Allaire: d(alpha1)/dt + u . grad(alpha1)
 * = 0, i.e. the alpha1 row of eq. (fvmdis) carries alpha1_cell div(u).
 * Kapila: d(alpha1)/dt + u . grad(alpha1) = K div(u) with
 * K = (rho2 c2^2 - rho1 c1^2) / (rho2 c2^2/alpha2 + rho1 c1^2/alpha1) and
 * rho_k c_k^2 = gamma_k (p + pi_k) at the cell's pressure (the paper's
 * rho1 c2^2 in the denominator read as rho1 c1^2), so the alpha1 row carries
 * (alpha1 + K)_cell div(u); K = 0 where alpha1 or alpha2 is not positive.
 * The Kapila form can lose positivity of alpha at strong material
 * interfaces (the paper notes its numerical instability); such cells are
 * reported like any non-physical state. */
enum { MFC_MODEL_ALLAIRE = 0, MFC_MODEL_KAPILA = 1 };

/* Kernel implementation of the right-hand side. */
enum {
    MFC_KERNEL_FUSED = 0,   /* one fused pass per stage (default)                    */
    MFC_KERNEL_STAGED = 1,  /* separate reconstruction / Riemann / update passes      */
    MFC_KERNEL_SPLIT = 2    /* 3D: an x+y pass and a z + stage-update pass per stage  */
};

typedef struct mfc_grid mfc_grid;

typedef struct {
    int ndim;            /* 1, 2 or 3                                              */
    int n[3];            /* interior cells per dimension; >= 3 on active dims,
                            ignored (treated as 1) on inactive ones                */
    double lo[3], hi[3]; /* uniform grid: dx_d = (hi_d - lo_d) / n_d > 0           */
    int num_fluids;      /* must be 2                                              */
    double gamma[2];     /* stiffened-gas gamma of fluid 1 and 2, > 1              */
    double pi_inf[2];    /* stiffened-gas pi_infinity (Pa), >= 0                   */
    int bc[6];           /* per face x-, x+, y-, y+, z-, z+: MFC_BC_*; periodic
                            must be set on both faces of a dimension               */
    int precision;       /* MFC_FP64 or MFC_FP32_MIXED                             */
    int recon;           /* MFC_RECON_*: WENO5, WENO3 or FIRST_ORDER (every kernel),
                            or LEARNED (fused and split kernels; needs
                            mfc_set_indicator before any right-hand side)          */
    double weno_eps;     /* WENO5-JS epsilon, > 0 (1e-6 in the paper's setting)    */
    int kernel;          /* MFC_KERNEL_*                                           */
    int model;           /* MFC_MODEL_ALLAIRE or MFC_MODEL_KAPILA                  */
    const double *faces[3];  /* non-uniform cells (Sec. 4.1): host array of the
                            n_d + 1 strictly increasing interior face coordinates
                            along d, copied at mfc_init_grid (lo/hi of that
                            dimension are then ignored); NULL for uniform cells.
                            Supported by MFC_KERNEL_FUSED and (3D)
                            MFC_KERNEL_SPLIT with MFC_RECON_WENO5
                            (WENO5 with per-cell coefficients from the widths)
                            or MFC_RECON_FIRST_ORDER; ghost cells take the widths
                            of the cells the ghost fill copies into them.
                            With any non-uniform dimension the CFL step is
                            cfl / max over cells and d of (|u_d| + c)/dx_d(cell),
                            and mfc_max_wavespeed returns that maximum (1/s). */
} mfc_grid_desc;

/* Create a grid handle from *desc (validated; see mfc_grid_desc) and
 * allocate its device scratch on the current HIP device.  The grid is the
 * Cartesian finite-volume mesh of Sec. 3.1 (cell averages on uniform cells,
 * or on the non-uniform cells of Sec. 4.1), with the two stiffened-gas
 * fluids of Sec. 2.1 (eq. soe) and the boundary buffers of Sec. 3.3.
 * Returns MFC_E_ARG, MFC_E_UNSUPPORTED or MFC_E_NOMEM on failure, with *out
 * set to NULL. */
int mfc_init_grid(const mfc_grid_desc *desc, mfc_grid **out);

/* Release the handle and its scratch (waits for work the handle enqueued). */
int mfc_free_grid(mfc_grid *g);

/* Shape of a state array on this grid: *nvar, padded[0..2] = (px, py, pz)
 * and the element size in bytes (8 or 4).  Host-only, never fails on a valid
 * handle. */
int mfc_state_layout(const mfc_grid *g, int64_t *nvar, int64_t padded[3], int64_t *elem_bytes);

/* Primitive -> conservative on every padded cell (EOS of Sec. 2.1): w and q
 * are distinct device arrays of the state layout. */
int mfc_prim_to_cons(mfc_grid *g, const void *w, void *q, void *stream);

/* Conservative -> primitive on every padded cell (non-physical cells set the
 * handle's flag, see mfc_check). */
int mfc_cons_to_prim(mfc_grid *g, const void *q, void *w, void *stream);

/* Fill the 3 ghost layers of every active face slab of q in place
 * (Sec. 3.3): extrapolation copies the adjacent interior cell, periodic the
 * cell one period away.  Edge and corner ghost cells are not written (the
 * dimension-by-dimension sweeps never read them). */
int mfc_fill_ghosts(mfc_grid *g, void *q, void *stream);

/* rhs = dq/dt of eq. (fvmdis) on interior cells, from q whose ghost cells are
 * filled: for every row the flux difference sum_d (F_{-1/2} - F_{+1/2})/dx_d
 * of the HLLC fluxes between WENO5 reconstructions of the primitives, plus
 * alpha1 div(u) (face-velocity divergence) on the alpha1 row.  Ghost
 * entries of rhs are not written.  q and rhs must not overlap.
 * MFC_KERNEL_SPLIT reads no ghost cell: it takes every neighbour past a face
 * from the interior cell the ghost fill would copy there (the boundary
 * condition applied by index), so its result is the one for filled ghosts
 * whatever the ghost cells of q hold. */
int mfc_rhs(mfc_grid *g, const void *q, void *rhs, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops, harnesses that forbid hipMalloc): the right-hand
 * side of mfc_rhs with MFC_KERNEL_SPLIT, from a descriptor and no grid handle.
 * desc is validated as by mfc_init_grid and must describe a 3D grid of
 * uniform cells with extrapolated or periodic faces and WENO5, WENO3 or
 * first-order reconstruction (desc->kernel is ignored); q and rhs are device
 * arrays of that grid's state layout in its precision, as for mfc_rhs (rhs
 * ghost entries are not written; q's ghost cells are not read).  flag_dev is
 * a caller-owned device int that the kernels set nonzero if a cell is
 * non-physical; it is not cleared.  The one scratch buffer, the x+y part of
 * every cell (nvar x padded cells x element size), lives in a 64 MiB device
 * array that the library holds on every GPU it runs on until the process
 * ends; grids needing more return MFC_E_ARG before anything is enqueued.
 * Nothing is allocated.  Calls on the same GPU share that array: calls that
 * overlap in time on one GPU (two streams, two host threads) race and give
 * undefined results. */
int mfc_rhs_noalloc(const mfc_grid_desc *desc, const void *q, void *rhs, int *flag_dev, void *stream);

/* Largest signal speed max_cells max_d (|u_d| + c) over interior cells, the
 * quantity that bounds the explicit step through the CFL condition (Sec. 1;
 * c the frozen mixture sound speed of the stiffened-gas mixture, Sec. 2.1)
 * (ghosts not read); on a grid with non-uniform cells the largest
 * (|u_d| + c)/dx_d(cell) instead (1/s).  Synchronises the stream and writes
 * *smax_host.  Returns MFC_E_NONPHYSICAL if an interior cell is
 * non-physical. */
int mfc_max_wavespeed(mfc_grid *g, const void *q, double *smax_host, void *stream);

/* One third-order TVD (SSP) Runge-Kutta step in place on q (Sec. 3.4:
 * q1 = q + dt L(q), q2 = 3/4 q + 1/4 (q1 + dt L(q1)),
 * q^{n+1} = 1/3 q + 2/3 (q2 + dt L(q2)), L the right-hand side of eq.
 * (fvmdis) as in mfc_rhs), ghost fill
 * before every right-hand side (MFC_KERNEL_SPLIT applies the boundary
 * conditions by index instead, with the same result, and leaves the ghost
 * cells of q as they were).  If cfl > 0 the step size is
 * cfl * min_d dx_d / max_wavespeed(q^n), computed on the device with no host
 * synchronisation; otherwise dt (> 0) is used.  The step size taken and the
 * accumulated time are kept on the device (mfc_time); if dt_used_dev is not
 * NULL, the step size taken is also written, on the stream and with no host
 * synchronisation, to that caller-owned device double. */
int mfc_rk3_step(mfc_grid *g, void *q, double cfl, double dt, double *dt_used_dev, void *stream);

/* nsteps SSP-RK3 steps as by mfc_rk3_step (dt_used_dev NULL), enqueued back
 * to back.  MFC_KERNEL_SPLIT with cfl > 0: the z pass of each step's last
 * stage also reduces the wave speeds of the state it writes (the next step's
 * q^n; with characteristic z faces, the boundary pass reduces those faces'
 * cells after it has changed them), so the next step's size is set before
 * its first stage, whose x+y pass then forms its part of the stage
 * combination (q + dt L_xy, the z pass adding dt L_z) instead of the z pass
 * reading q^n again.  The step sizes are those of single mfc_rk3_step calls
 * on the same states, bit for bit; the states agree to rounding. */
int mfc_run(mfc_grid *g, void *q, int nsteps, double cfl, double dt, void *stream);

/* Synchronise and read the accumulated simulated time and the last step
 * size (either pointer may be NULL).  mfc_reset_time sets both to 0. */
int mfc_time(mfc_grid *g, double *t_host, double *last_dt_host, void *stream);
int mfc_reset_time(mfc_grid *g, void *stream);

/* Synchronise, return MFC_E_NONPHYSICAL if any kernel of this handle met a
 * non-physical cell since the last check, and clear the flag. */
int mfc_check(mfc_grid *g, void *stream);

/* Kernel timing: while enabled, launches of the right-hand-side kernels are
 * bracketed by HIP events on the launch stream.  Slot 0 is the main
 * right-hand-side kernel (the fused kernel, the x+y kernel of the split
 * path, or the whole staged sequence); slot 1 is the z + stage-update kernel
 * of the split path.  enable = 0 stops the recording and keeps what was
 * recorded; enable = 1 times every launch; enable = N > 1 times every
 * launch of mfc_rhs and those of every N-th SSP-RK3 step of mfc_rk3_step and
 * mfc_run, counted from this call (the first step is timed), so that a
 * sample of a long run is timed without events between all its launches.
 * enable < 0 gives MFC_E_ARG.  mfc_kernel_time synchronises, returns the
 * summed duration (ms) and number of timed launches of that slot since the
 * last call for it, and resets them.  slot outside [0, 1] gives MFC_E_ARG. */
int mfc_set_kernel_timing(mfc_grid *g, int enable);
int mfc_kernel_time(mfc_grid *g, int slot, double *ms_total, int64_t *launches);

/* ------------------------------------------------------------------------
 * Learned smoothness indicator (project extension beside the WENO5
 * reconstruction of Sec. 3.2).  For every (cell, direction) a perceptron
 * 15 -> 32 -> 32 -> 1 (GELU, logistic output) reads the 5-cell stencils of
 * alpha1, rho = a1r1 + a2r2 and p, each as (v_j - v_centre) /
 * max(max_j |v_j - v_centre|, sqrt(weno_eps)), and gives P(smooth).  With
 * MFC_RECON_LEARNED, a (cell, direction) with P(smooth) > tau takes the
 * linear fifth-order stencil (the ideal-weight limit of WENO5) for every
 * variable and both faces; all others take WENO5.  Products run on bf16
 * matrix cores: their operands (inputs, W1, W2, hidden activations and,
 * in training, the back-propagated dZ2 and dZ1) are rounded to bf16
 * (nearest, ties to even), sums and all element-wise work are FP32.
 *
 * Parameters are 1601 floats in the flat order W1[15][32] (input-major),
 * b1[32], W2[32][32] (input-major), b2[32], W3[32], b3.  Features are
 * 16 bf16 values per sample (uint16_t bit patterns; the 16th is 0).
 * ------------------------------------------------------------------------ */
typedef struct mfc_trainer mfc_trainer;

/* Install a network (1601 host floats, copied) and the routing threshold
 * tau for the handle's MFC_RECON_LEARNED right-hand sides.  tau <= 0 routes
 * every reconstruction to the linear stencil, tau >= 1 none.  MFC_E_ARG on
 * non-finite parameters or tau. */
int mfc_set_indicator(mfc_grid *g, const float *params_host, double tau);

/* Training samples from an FP64 state q (device, the handle's layout; its
 * ghost cells are refilled first, as mfc_fill_ghosts): for every interior
 * (cell, direction), ordered direction-major then z, y, x, the 16 features
 * (features[16 * sample ..], device) and the label (labels[sample], device):
 * 1 when every variable's WENO5 weights stay within 0.01 of the ideal
 * weights (max over the three stencils and both faces of |omega_r - d_r|)
 * and 0 otherwise.  maxdev (nullable, device, doubles) receives that largest
 * deviation.  Arrays hold ndim * cells samples.  MFC_E_UNSUPPORTED for an
 * FP32 handle. */
int mfc_harvest(mfc_grid *g, void *q, uint16_t *features, uint8_t *labels, double *maxdev, void *stream);

/* A trainer owns FP32 master weights, Adam moments and gradient scratch for
 * batches of up to max_batch samples (1 .. 2^31).  Weights start at 0:
 * set them with mfc_trainer_set_params (which also clears the moments and
 * the step count). */
int mfc_trainer_init(int64_t max_batch, mfc_trainer **out);
int mfc_trainer_free(mfc_trainer *t);
int mfc_trainer_set_params(mfc_trainer *t, const float *params_host);   /* synchronises */
int mfc_trainer_get_params(mfc_trainer *t, float *params_host);         /* synchronises */

/* Gradient of the mean binary cross-entropy over `batch` samples (1 ..
 * max_batch) of device arrays features / labels, sample i being
 * index[i] (device int32, nullable: sample i is i).  The gradient and the
 * mean loss stay on the device (deterministic: a fixed reduction order). */
int mfc_trainer_grad(mfc_trainer *t, const uint16_t *features, const uint8_t *labels, const int32_t *index,
                     int64_t batch, void *stream);

/* Synchronise and copy the last gradient (1601 floats) and mean loss
 * (nullable) to the host. */
int mfc_trainer_read_grad(mfc_trainer *t, float *grad_host, float *loss_host, void *stream);

/* One Adam step on the master weights with the last gradient:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * w -= lr (m / (1 - b1^k)) / (sqrt(v / (1 - b2^k)) + eps), k = steps taken. */
int mfc_trainer_adam(mfc_trainer *t, float lr, float beta1, float beta2, float eps, void *stream);

/* P(smooth) of n samples (device features -> device floats). */
int mfc_trainer_infer(mfc_trainer *t, const uint16_t *features, int64_t n, float *prob, void *stream);

/* ------------------------------------------------------------------------
 * Batched ensembles (project extension beside the method of Sec. 3).  Many
 * independent 2D runs, each with its own grid size, fluids and boundaries,
 * advanced together: every kernel of an SSP-RK3 step (Sec. 3.4) covers all
 * runs, each run takes its own CFL step size (Sec. 1) on the device, and the
 * right-hand side of every run is the one mfc_rhs defines.  A run advanced in
 * a batch gives the same bits as the same run advanced alone with
 * mfc_rk3_step (MFC_KERNEL_FUSED, same precision and cfl), except a run with
 * characteristic faces, which the batch's stage kernel applies itself and
 * the single-grid kernels in a boundary pass: the same scheme, rounded in
 * another order.
 *
 * State arrays stay owned by the caller: run r is a device array of the 2D
 * state layout above (nvar 6, padded (n[0] + 6, n[1] + 6, 1)).  The batch
 * owns two stage registers per run, the per-run step sizes and times, and
 * the captured graph.  A batch must not be used from two host threads or
 * two streams at once.
 * ------------------------------------------------------------------------ */
typedef struct mfc_batch mfc_batch;

/* Launch configuration of the batched right-hand-side kernel:
 *   shape  tile of one work item: 0 = 16 x 16, 1 = 32 x 8, 2 = 64 x 4 cells;
 *   groups persistent workgroups per compute unit: 0 = 1, 1 = 2, 2 = 4;
 *   xcd    1 = give each XCD a contiguous range of work items (neighbouring
 *          tiles share one L2), 0 = deal items round-robin. */
typedef struct {
    int shape;
    int groups;
    int xcd;
} mfc_batch_tune;

/* Create a batch of count (1..4096) runs from descs[0..count-1]: every
 * descriptor must have ndim 2, num_fluids 2, recon MFC_RECON_WENO5 and the
 * same precision; n[0], n[1] in [3, 32768]; other fields as for
 * mfc_init_grid (kernel is ignored).  Allocates the stage registers on the
 * current device.  MFC_E_ARG / MFC_E_UNSUPPORTED / MFC_E_NOMEM with *out
 * set to NULL on failure.  The initial configuration is {0, 1, 1}. */
int mfc_batch_init(const mfc_grid_desc *descs, int count, mfc_batch **out);

/* Release the batch (waits for the device). */
int mfc_batch_free(mfc_batch *b);

/* State layout of run `run` (host only): nvar, padded sizes, element size. */
int mfc_batch_layout(const mfc_batch *b, int run, int64_t *nvar, int64_t padded[3], int64_t *elem_bytes);

/* Total interior cells and number of runs (host only). */
int mfc_batch_cells(const mfc_batch *b, int64_t *cells, int *nrun);

/* One SSP-RK3 step of every run in place on q[0..count-1] (device arrays of
 * the run layouts).  Neighbours past a domain face are taken through the
 * run's boundary conditions (the values a ghost fill would write, bit for
 * bit): ghost cells are neither read nor written.  Step size per run:
 * cfl * min_d dx_d / (max wave speed of that run), on the device. */
int mfc_batch_step(mfc_batch *b, void *const *q, double cfl, void *stream);

/* nsteps steps.  Within the call each step's size comes from the wave
 * speeds the previous step's last stage reduced over the state it wrote
 * (the first step, and the first of each graph replay, reduce their own):
 * the same sizes and states, bit for bit, as nsteps mfc_batch_step calls.
 * With use_graph != 0, steps are replayed from a HIP graph that captures up
 * to 64 steps of the whole ensemble; it is captured on the first call and
 * reused while q, cfl, the chunk length and the configuration stay the
 * same.  Kernel timing (mfc_batch_set_timing) turns graph replay off. */
int mfc_batch_run(mfc_batch *b, void *const *q, int nsteps, double cfl, int use_graph, void *stream);

/* Choose the launch configuration: time the first-stage kernel (which reads
 * q and writes only a stage register, so states and times are unchanged;
 * ghost cells of q are refilled) reps (1..1000) times for each of the
 * 3 x 3 x 2 configurations, keep the fastest and return it in *best.
 * ms_table (nullable, 18 doubles) receives the mean time of configuration
 * (shape, groups, xcd) at index (shape * 3 + groups) * 2 + xcd.
 * Synchronises. */
int mfc_batch_autotune(mfc_batch *b, void *const *q, int reps, mfc_batch_tune *best, double *ms_table, void *stream);
int mfc_batch_set_tune(mfc_batch *b, const mfc_batch_tune *t);
int mfc_batch_get_tune(const mfc_batch *b, mfc_batch_tune *t);

/* Kernel timing of the batched right-hand-side launches (HIP events on the
 * launch stream), as mfc_set_kernel_timing / mfc_kernel_time. */
int mfc_batch_set_timing(mfc_batch *b, int enable);
int mfc_batch_kernel_time(mfc_batch *b, double *ms_total, int64_t *launches);

/* Synchronise and read the accumulated simulated time of every run into
 * t_host[0..count-1]. */
int mfc_batch_time(mfc_batch *b, double *t_host, void *stream);

/* Synchronise; MFC_E_NONPHYSICAL if any run met a non-physical cell since
 * the last check (the flag is then cleared). */
int mfc_batch_check(mfc_batch *b, void *stream);

/* Message for a status code (static storage). */
const char *mfc_strerror(int status);

/* Detail of the last failing call on this thread (static per thread). */
const char *mfc_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* MFC_H */
