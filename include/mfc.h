/*
 * mfc.h - C ABI of the MI355X (gfx950) right-hand side of the two-fluid
 * five-equation diffuse-interface model.
 *
 * The operations are those of the paper's numerical method:
 *   - governing equations (Sec. 2.1): partial densities alpha1 rho1 and
 *     alpha2 rho2, mixture momentum, total energy, and the volume fraction
 *     alpha1 advected with the non-conservative alpha1 div(u) term (Allaire
 *     form: the K div(u) term of the Kapila model is dropped);
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
    MFC_E_UNSUPPORTED = -5   /* valid request this build does not implement          */
};

enum { MFC_BC_EXTRAP = 0, MFC_BC_PERIODIC = 1 };
enum { MFC_FP64 = 0, MFC_FP32_MIXED = 1 };
enum { MFC_RECON_WENO5 = 0, MFC_RECON_LEARNED = 1 };

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
    int recon;           /* MFC_RECON_WENO5 (MFC_RECON_LEARNED: see mfc_set_indicator) */
    double weno_eps;     /* WENO5-JS epsilon, > 0 (1e-6 in the paper's setting)    */
    int kernel;          /* MFC_KERNEL_*                                           */
} mfc_grid_desc;

/* Create a grid handle from *desc (validated; see mfc_grid_desc) and
 * allocate its device scratch on the current HIP device.
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
 * entries of rhs are not written.  q and rhs must not overlap. */
int mfc_rhs(mfc_grid *g, const void *q, void *rhs, void *stream);

/* Largest signal speed max_cells max_d (|u_d| + c) over interior cells
 * (ghosts not read).  Synchronises the stream and writes *smax_host.
 * Returns MFC_E_NONPHYSICAL if an interior cell is non-physical. */
int mfc_max_wavespeed(mfc_grid *g, const void *q, double *smax_host, void *stream);

/* One third-order TVD (SSP) Runge-Kutta step in place on q, ghost fill
 * before every right-hand side.  If cfl > 0 the step size is
 * cfl * min_d dx_d / max_wavespeed(q^n), computed on the device with no host
 * synchronisation; otherwise dt (> 0) is used.  The step size taken and the
 * accumulated time are kept on the device (mfc_time). */
int mfc_rk3_step(mfc_grid *g, void *q, double cfl, double dt, void *stream);

/* nsteps calls of mfc_rk3_step, enqueued back to back. */
int mfc_run(mfc_grid *g, void *q, int nsteps, double cfl, double dt, void *stream);

/* Synchronise and read the accumulated simulated time and the last step
 * size (either pointer may be NULL).  mfc_reset_time sets both to 0. */
int mfc_time(mfc_grid *g, double *t_host, double *last_dt_host, void *stream);
int mfc_reset_time(mfc_grid *g, void *stream);

/* Synchronise, return MFC_E_NONPHYSICAL if any kernel of this handle met a
 * non-physical cell since the last check, and clear the flag. */
int mfc_check(mfc_grid *g, void *stream);

/* Kernel timing: while enabled, every launch of the right-hand-side kernels
 * is bracketed by HIP events on the launch stream.  Slot 0 is the main
 * right-hand-side kernel (the fused kernel, the x+y kernel of the split
 * path, or the whole staged sequence); slot 1 is the z + stage-update kernel
 * of the split path.  mfc_kernel_time synchronises, returns the summed
 * duration (ms) and number of launches of that slot since the last call for
 * it, and resets them.  slot outside [0, 1] gives MFC_E_ARG. */
int mfc_set_kernel_timing(mfc_grid *g, int enable);
int mfc_kernel_time(mfc_grid *g, int slot, double *ms_total, int64_t *launches);

/* Message for a status code (static storage). */
const char *mfc_strerror(int status);

/* Detail of the last failing call on this thread (static per thread). */
const char *mfc_last_error_detail(void);

#ifdef __cplusplus
}
#endif

#endif /* MFC_H */
