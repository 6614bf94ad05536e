/*
 * wenomhd.h -- C ABI of the MI355X (gfx950) WENO5 constrained-transport ideal
 * MHD step of Donnert et al., "WENO-Wombat" (arXiv:1812.04278).
 *
 * Method: per direction, the finite-difference WENO5 flux of Sect. 2.2
 * (eq. FWENO, Jiang-Shu or WENO-Z weights) computed in characteristic fields
 * with the eigenvectors of Appendix A at the face, Lax-Friedrichs split; its
 * conservative divergence (eq. num); the CT transport fluxes (eq. fct1-fct6),
 * corner fluxes (eq. ox1-ox3) and the face-field update of Sect. 2.3; a
 * Runge-Kutta stage in increment form (SSP-RK3 at CFL 0.4, or the classical
 * RK4 of Sect. 2.1 at CFL 0.8); the adjoint (vector-Jacobian products) of the
 * right-hand side and of a step.
 *
 * Grid: nx * ny * nz zones, one zone size h for every direction (Sect. 2.3
 * divides every difference by the same Delta x), periodic in each direction
 * unless wm_config.walls marks it: then the box has reflecting, perfectly
 * conducting walls at both ends of that axis (the reflecting boundaries of the
 * paper's test problems, Sect. 4): ghost zones mirror the interior (normal
 * momentum and normal field odd, the rest even), the corner fluxes on wall
 * edges vanish and the normal face field on the wall faces is zero -- the last
 * face of bface along a walled axis (index n-1) is the upper wall face and
 * must hold 0; the lower wall face is implicit.
 * Every array is structure-of-arrays, [component][z][y][x] with x contiguous,
 * in device memory of the GPU that is current when the patch is created, and
 * double precision -- except the bound state (hydro, bface, bcell) and the
 * stage states of wm_step_record, which hold floats when the configuration's
 * precision is WM_MIXED_F32STATE.  Conventions of the field components:
 *   hydro  [5][nz][ny][nx]  rho, m_x, m_y, m_z, E            (zone centred)
 *   bface  [3][nz][ny][nx]  b_x at (i+1/2, j, k), b_y at (i, j+1/2, k),
 *                           b_z at (i, j, k+1/2)              (face centred)
 *   bcell  [3][nz][ny][nx]  zone B, the fourth-order interpolation of bface
 *                           (Sect. 2.3); written by the library, never read
 *                           as an input to a step
 *   A_edge [3][nz][ny][nx]  A_x at (i, j+1/2, k+1/2), A_y at (i+1/2, j, k+1/2),
 *                           A_z at (i+1/2, j+1/2, k)  (Sect. 4.1 placement)
 *
 * Ownership: the caller owns every buffer (state, scratch, outputs).  The
 * library never allocates device memory: it launches kernels on the caller's
 * stream and only allocates the small host-side patch object.  A patch is used
 * by one host thread and one stream at a time; calls are stream ordered.
 *
 * Errors: every call returns a wm_status and never aborts.  Argument errors
 * are detected synchronously (nothing is launched); launch failures return
 * WM_ERR_HIP.  Physical failures (rho <= 0, P <= 0, non-finite values) are
 * not checked inside a step; wm_diagnostics counts them and then returns
 * WM_ERR_UNPHYSICAL.  wm_last_error() gives a message for the last failure on
 * the calling thread.
 */
#ifndef WENOMHD_H
#define WENOMHD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  WM_OK = 0,
  WM_ERR_ARG = -1,          /* invalid argument or unsupported option       */
  WM_ERR_HIP = -2,          /* a HIP runtime call or a launch failed        */
  WM_ERR_UNPHYSICAL = -3,   /* diagnostics found rho<=0, P<=0 or NaN/Inf    */
  WM_ERR_STATE = -4         /* call out of order (e.g. step before binding) */
} wm_status;

typedef enum {
  WM_FP64 = 0,              /* everything in double precision                */
  WM_MIXED = 1,             /* FP64 state, pressure recovery, eigenvector
                               renormalisation and central flux; FP32
                               characteristic projections, WENO weights and
                               split fluxes                                   */
  WM_MIXED_F32STATE = 2     /* the WM_MIXED arithmetic with the state (hydro,
                               bface, bcell), the stage states, the RK
                               accumulator and the face fluxes stored in FP32
                               (float arrays); increments and divergences are
                               formed in FP64 before rounding to the state    */
} wm_precision;

typedef enum {
  WM_WENO_JS = 0,           /* Jiang-Shu weights, Sect. 2.2                  */
  WM_WENO_Z = 1,            /* WENO-Z weights, Sect. 2.2 (reading: the
                               bracket (tau_5/(eps_Z + IS_k))^2)              */
  WM_WENO_Z_PRINTED = 2     /* WENO-Z weights as Sect. 2.2 prints them,
                               d_k (1 + tau_5/(eps_Z + IS_k)^2): not invariant
                               under a scaling of the data (the term has the
                               dimension of 1/IS); like WENO-Z in every call,
                               the adjoint included                           */
} wm_weights;

typedef enum {
  WM_SSPRK3 = 0,            /* three-stage SSP-RK3 (Shu-Osher), CFL 0.4       */
  WM_RK4 = 1                /* the classical four-stage RK4 of Sect. 2.1, for
                               which the paper uses CFL 0.8                   */
} wm_integrator;

typedef struct {
  int nx, ny, nz;           /* zones per direction, each >= 1                */
  double h;                 /* zone size (> 0)                               */
  double gamma;             /* adiabatic index (> 1)                         */
  double cfl;               /* Courant number for wm_compute_dt (> 0)        */
  double eps_weno;          /* WENO epsilon, 1e-6 in the paper               */
  double eps_B;             /* degeneracy threshold, 1e-30 in the paper      */
  double eps_Z;             /* WENO-Z epsilon, 1e-40 in the paper; at least
                               1e-50 (the weights are formed with (eps_Z +
                               IS_k)^6 in FP64, which also bounds the
                               smoothness indicators there to ~1e50)          */
  int weights;              /* wm_weights                                    */
  int precision;            /* wm_precision                                  */
  int integrator;           /* wm_integrator                                 */
  int walls[3];             /* per axis x, y, z: 0 periodic, 1 reflecting
                               conducting walls (that axis needs >= 3 zones;
                               no adjoint)                                    */
  double rho_floor;         /* opt-in density floor, 0 = off: after every
                               stage a density below it is raised to it (the
                               momentum kept)                                 */
  double p_floor;           /* opt-in gas-pressure floor, 0 = off: then a
                               pressure below it is raised to it by adding
                               internal energy; floors need WM_SSPRK3 and
                               have no adjoint                                */
} wm_config;

typedef struct {
  double max_divb;          /* max over zones of |div_h b| (eq. divb)        */
  double mass;              /* sum of rho over zones                         */
  double mom[3];            /* sums of m_x, m_y, m_z                         */
  double energy;            /* sum of E                                      */
  double bflux[3];          /* sums of b_x, b_y, b_z over all faces          */
  double min_rho;           /* minimum density                               */
  double min_p;             /* minimum gas pressure (eq. P, zone B)          */
  long long n_unphysical;   /* zones with rho<=0, P<=0 or non-finite values  */
  long long n_floored;      /* floor activations (a density and a pressure
                               activation count separately) since the state
                               was bound, initialised or refreshed            */
} wm_diag;

typedef struct wm_patch wm_patch;   /* opaque; owns no device memory */

/* Fills cfg with the paper's constants (gamma 5/3, eps 1e-6, eps_B 1e-30,
 * eps_Z 1e-40, Jiang-Shu, FP64) and SSP-RK3 at CFL 0.4 for a periodic n^3 box
 * of length 1 without floors (for WM_RK4 the paper's Courant number is 0.8). */
void wm_config_default(wm_config* cfg, int n);

/* Bytes of device scratch a patch with this configuration needs: the stage
 * state, the RK accumulator, the face fluxes of the three sweeps and the
 * reduction buffers.  Returns 0 for an invalid configuration. */
size_t wm_scratch_bytes(const wm_config* cfg);

/* Creates a patch.  `hip_stream` is a hipStream_t (NULL = default stream);
 * `scratch` is a device buffer of at least wm_scratch_bytes(cfg) bytes,
 * 256-byte aligned, owned by the caller and reserved for this patch. */
wm_status wm_patch_create(const wm_config* cfg, void* hip_stream, void* scratch,
                          size_t scratch_bytes, wm_patch** out);
wm_status wm_patch_destroy(wm_patch* p);

/* Binds the caller's state arrays (layouts above; element type double, or
 * float for WM_MIXED_F32STATE).  hydro and bface are read and advanced in
 * place by the last stage of wm_rk_stage (2 for SSP-RK3, 3 for RK4) and by
 * wm_step; bcell is written. */
wm_status wm_bind_state(wm_patch* p, void* hydro, void* bface, void* bcell);

/* Initial state from primitive fields and an edge vector potential
 * (Sect. 4.1): b = B0 + curl_h A by first-order differences (div_h b = 0),
 * zone B by the fourth-order interpolation of Sect. 2.3, m = rho v and
 * E = P0/(gamma-1) + (rho v^2 + B^2)/2 (eq. P).  With walls, the normal face
 * field on the wall faces is set to zero (give A with no tangential component
 * on the wall edges to keep div_h b = 0 there).  rho [nz][ny][nx],
 * v [3][nz][ny][nx], A_edge [3][nz][ny][nx]: device arrays; B0 a host array. */
wm_status wm_init_from_potential(wm_patch* p, const double* rho, const double* v,
                                 const double* A_edge, double P0, const double B0[3]);

/* Recomputes zone B of the bound state from its face field (the fourth-order
 * interpolation of Sect. 2.3), for callers that wrote bface themselves. */
wm_status wm_refresh_zone_field(wm_patch* p);

/* Time step of eq. (cfl) at equality: dt = cfl h / sum_d max(|v_d| + c_fast^d),
 * from the bound state.  The result stays in device memory for the stages; if
 * dt_host is non-NULL the stream is synchronised and dt copied there.  A NaN
 * in the state, or a fast speed that is not real (negative pressure), gives a
 * NaN dt. */
wm_status wm_compute_dt(wm_patch* p, double* dt_host);

/* One Runge-Kutta stage in increment form, k_s the right-hand side at the
 * stage state (stage 0: the bound state U^n).  WM_SSPRK3, stages 0..2:
 * stage 0 writes k0 and U1 = U^n + dt k0 into scratch; stage 1 writes k0+k1
 * and U2 = U^n + dt/4 (k0+k1); stage 2 writes U^{n+1} = U^n + dt/6 (k0+k1+4 k2)
 * into the bound state.  WM_RK4, stages 0..3 (Sect. 2.1): U1 = U^n + dt/2 k0,
 * U2 = U^n + dt/2 k1, U3 = U^n + dt k2 into scratch with the accumulator
 * k0 + 2 k1 + 2 k2, and stage 3 writes U^{n+1} = U^n + dt/6 (k0 + 2 k1 +
 * 2 k2 + k3) into the bound state (the paper's q_save sum).  Each stage ends
 * with zone B re-interpolated from the new face field.  Stages run in order
 * (WM_ERR_STATE otherwise).  dt_host NULL: the device dt of the last
 * wm_compute_dt. */
wm_status wm_rk_stage(wm_patch* p, int stage, const double* dt_host);

/* The dt of wm_compute_dt followed by the stages of the configured integrator
 * (three for WM_SSPRK3, four for WM_RK4).  The maxima of eq. (cfl) are taken
 * from the zones the first stage's sweeps already evaluate, so the step reads
 * the state once less; dt, and so the step, are bitwise those of
 * wm_compute_dt followed by wm_rk_stage.  The first stage's accumulator
 * scratch holds the partial maxima meanwhile.  If dt_used is non-NULL the
 * stream is synchronised and the dt of the step is returned there. */
wm_status wm_step(wm_patch* p, double* dt_used);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): wm_step on
 * the caller's state arrays (hydro, bface, bcell: the layouts above, element
 * type double, or float for WM_MIXED_F32STATE) without a patch and without
 * caller scratch.  The step's scratch is a 64 MiB device array inside the
 * library, one per GPU, created when the library's code is loaded onto that
 * GPU and held until the process ends; its device address is looked up once
 * per device, on the first call with that device current.  Configurations
 * whose wm_scratch_bytes exceeds 64 MiB are rejected with WM_ERR_ARG before
 * any device work (FP64 up to about 200,000 zones, e.g. 58^3; the FP32 state
 * up to about 400,000, e.g. 73^3).  No device or host memory is allocated:
 * only kernels are launched on hip_stream (plus, when dt_used is non-NULL, one
 * copy of dt to the host and a stream synchronisation).  The step keeps no
 * state between calls (every scratch value is written before it is read), but
 * all calls on one GPU share the array: calls that overlap in time on the same
 * GPU (other streams or host threads) race and give wrong results. */
wm_status wm_step_static(const wm_config* cfg, void* hip_stream, void* hydro, void* bface, void* bcell,
                         double* dt_used);

/* Diagnostics of the bound state (synchronises the stream).  Returns
 * WM_ERR_UNPHYSICAL (with *out filled) when n_unphysical > 0. */
wm_status wm_diagnostics(wm_patch* p, wm_diag* out);

/* Direction-resolved output of one sweep of the bound state, for testing the
 * rows of the step separately.  out [9][nz][ny][nx] (device): components
 * 0..6 the WENO interface flux on the forward face along `axis` in the sweep
 * frame (rho, m_n, m_t1, m_t2, B_t1, B_t2, E), with (n, t1, t2) = (x, y, z),
 * (y, z, x), (z, x, y) for axis 0, 1, 2; components 7, 8 the CT transport
 * fluxes T^n_t1, T^n_t2 of eq. (fct1)-(fct6). */
wm_status wm_debug_sweep(wm_patch* p, int axis, void* out);

/* Testing switch (on != 0): the sweep addresses its loads and stores with
 * 64-bit pointers, the path it otherwise takes only for arrays of 4 GiB and
 * more (raw buffer accesses with 32-bit offsets below that).  The arithmetic is
 * the same, so results are bitwise equal either way.  WM_ERR_ARG for a null
 * patch. */
wm_status wm_debug_wide_addressing(wm_patch* p, int on);

/* Right-hand side dU/dt of the bound state: out [8][nz][ny][nx] (device) =
 * d(rho, m_x, m_y, m_z, E)/dt from the flux divergence (eq. num) and
 * d(b_x, b_y, b_z)/dt from the corner fluxes (Sect. 2.3). */
wm_status wm_debug_rhs(wm_patch* p, void* out);

/* ---- adjoint (vector-Jacobian products), FP64 ----------------------------
 * The differentiated map is the step with a given dt (dt is held fixed: its
 * dependence on the state through eq. (cfl) is not differentiated).  At the
 * non-smooth points of the scheme the derivative of the branch the forward
 * pass takes is used (max: the larger argument, ties the first; |x|: sign(x);
 * clamps and the degenerate constants of Appendix A: zero).  Cotangent arrays
 * have the layout of the state: lam_hydro [5][nz][ny][nx] (rho, m, E),
 * lam_bface [3][nz][ny][nx].  The adjoint needs every grid size >= 3. */

/* Bytes of device scratch the adjoint calls need (caller-owned, 256-aligned,
 * reserved for one patch at a time; more for WM_RK4, whose step adjoint holds
 * a third stage state).  0 for an invalid configuration.
 * The adjoint calls linearise the FP64 method with the patch's weights
 * (Jiang-Shu or WENO-Z) and integrator (grid sizes below 3: WM_ERR_ARG).  On a
 * mixed-precision patch they give the FP64 linearisation at the states passed
 * in (stage states recomputed by the adjoint itself come from the patch's own
 * precision).  On a WM_MIXED_F32STATE patch the state arguments (U^n, the
 * stage states, the state of wm_rhs_vjp) are float arrays like the patch's
 * state: they are widened to FP64 on load, and the FP64 method is linearised
 * at the widened states; cotangents are double arrays in every mode. */
size_t wm_adjoint_scratch_bytes(const wm_config* cfg);

/* lam_out = (dL/dU)^T lam_k for the semi-discrete right-hand side L of the
 * state U = (hydro, bface) (eq. num, eq. ox1-ox3 and the b equations of
 * Sect. 2.3).  lam_k, lam_out: [8][nz][ny][nx] device arrays (rho, m_x, m_y,
 * m_z, E, b_x, b_y, b_z); lam_out is overwritten. */
wm_status wm_rhs_vjp(wm_patch* p, void* adj_scratch, const void* hydro, const void* bface, const void* lam_k,
                     void* lam_out);

/* Adjoint of one step U^{n+1} = Phi(U^n; dt) of the patch's integrator
 * (increment form, dt held fixed): lam_hydro [5][..], lam_bface [3][..] hold
 * dJ/dU^{n+1} on entry and dJ/dU^n on return.  SSP-RK3: U1_stage, U2_stage are
 * the step's two intermediate stage states as wm_step_record stores them
 * ([8][..]: hydro then face b), or both NULL to recompute them from U^n into
 * adj_scratch.  WM_RK4 (Sect. 2.1): both must be NULL (the three stage states
 * are recomputed; WM_ERR_ARG otherwise).  Recomputing them uses the forward
 * scratch of the patch: with NULL stage states the call returns WM_ERR_STATE
 * while a step of wm_rk_stage is in progress. */
wm_status wm_adjoint_step(wm_patch* p, void* adj_scratch, const void* Un_hydro, const void* Un_bface,
                          const void* U1_stage, const void* U2_stage, double dt, void* lam_hydro, void* lam_bface);

/* One SSP-RK3 step of the bound state with the given dt (as wm_rk_stage
 * 0, 1, 2), also copying the two intermediate stage states to U1_out and
 * U2_out ([8][nz][ny][nx] device arrays each: rho, m_x, m_y, m_z, E, b_x, b_y,
 * b_z), for a later wm_adjoint_step.  A WM_RK4 patch returns WM_ERR_ARG. */
wm_status wm_step_record(wm_patch* p, double dt, void* U1_out, void* U2_out);

/* lam_bface += transpose of the zone interpolation B = interp4(b) applied to
 * lam_bcell ([3][nz][ny][nx]): the cotangent of a loss on zone B. */
wm_status wm_zone_field_vjp(wm_patch* p, const void* lam_bcell, void* lam_bface);

/* Adjoint of wm_init_from_potential with respect to A_edge and v (rho, P0
 * and B0 held fixed): given dJ/d(hydro, bface) of the initial state, writes
 * g_A = dJ/dA_edge [3][..] and g_v = dJ/dv [3][..] (device arrays). */
wm_status wm_init_adjoint(wm_patch* p, void* adj_scratch, const double* rho, const double* v, const double* A_edge,
                          const double B0[3], const void* lam_hydro, const void* lam_bface, double* g_A,
                          double* g_v);

/* Kernel timing with HIP events recorded on the patch's stream around every
 * launch (for measurement; adds two event records per launch).  enable = 1
 * starts a session (discarding earlier records), 0 stops it.  Records up to
 * 8192 launches per session; later launches are not timed. */
wm_status wm_profile(wm_patch* p, int enable);

/* Synchronises the stream and reports the session: out[2*c] = number of
 * launches and out[2*c+1] = summed milliseconds of kernel class c, with
 * c = 0 sweeps, 1 update (divergence + CT + RK), 2 zone-B interpolation,
 * 3 time-step reduction, 4 other (adjoint kernels).  n_out must be >= 10. */
wm_status wm_profile_report(wm_patch* p, double* out, int n_out);

/* Message of the last failed call on this thread ("" if none). */
const char* wm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* WENOMHD_H */
