/*
 * dgsem.h -- C ABI of the MI355X (gfx950) DGSEM Navier-Stokes library.
 *
 * The library evaluates the discontinuous Galerkin spectral element time
 * derivative of the compressible Navier-Stokes equations on curved,
 * unstructured hexahedral meshes with periodic connectivity, and advances it
 * with a low-storage Runge-Kutta scheme (five or fourteen stages).
 * Paper: Kurz, Kempf et al., GALAEXI (arXiv 2404.12703):
 *   equations           Sec. 2.1, Eqs. nse, eos_p, eos_T
 *   mapping, metrics    Sec. 2.2 "Mapping the Equations" (curl form)
 *   operator            Sec. 2.2 Eq. dgsem; Table tab:dg_routines; App. A
 *   BR1 lifting         Sec. 2.2 "Second-Order Equations", Eq. lifting
 *   split form          Sec. 2.2 "Nonlinear Stability" (Pirozzoli's two-point flux)
 *   viscosity law       Sec. 2.1 Eq. sutherland
 *   time integration    Sec. 2.2 "Time integration" (Carpenter-Kennedy 4(5);
 *                       Niegemann et al.'s fourteen stages)
 *   shock capturing     Sec. 2.3 (convex DG/FV-subcell blend, a-priori indicator)
 *   dissipation rates   Sec. 5.2 (solenoidal and dilatational, from the lifted gradients)
 *   throughput metric   Sec. 4.2 (PID); memory per DOF Sec. 4.3
 *
 * Conventions shared by every entry point
 *   - All functions are extern "C"; no exception crosses the ABI.  They return
 *     a dg_status (0 = DG_OK, negative = error) and leave a message for
 *     dg_last_error() (thread-local, valid until the next call on that thread).
 *   - Host arrays passed in are copied before the call returns; the caller may
 *     free them at once.
 *   - Device memory is owned by the caller: the workspace (and the server's
 *     arena) is allocated by the caller and must outlive the object that uses
 *     it.  The library never allocates or frees device memory itself.
 *   - Work is enqueued asynchronously on the caller's HIP stream (hipStream_t
 *     passed as void*; NULL = the default stream).  Only calls that return host
 *     data (get_state to host, rhs to host, alpha, integrals, stable_dt,
 *     synchronize, and the server's run/fetch) synchronise with that stream.
 *   - State layout: conservative variables U = (rho, rho u, rho v, rho w, rho e)
 *     as double[5][n_elems][(N+1)^3]; the node index is i + (N+1)(j + (N+1) k)
 *     with i fastest along the element's first reference axis.
 *   - Local faces: 0 xi-, 1 xi+, 2 eta-, 3 eta+, 4 zeta-, 5 zeta+.  Face
 *     coordinates (p, q) run along the two other reference axes in increasing
 *     order (xi faces: (j,k); eta faces: (i,k); zeta faces: (i,j)).
 */
#ifndef DGSEM_H
#define DGSEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define DG_ABI_VERSION 2

typedef int32_t dg_status;
enum {
  DG_OK = 0,
  DG_EINVAL = -1,     /* bad argument or parameter                               */
  DG_EMESH = -2,      /* mesh rejected: asymmetric neighbours, J <= 0, faces not watertight */
  DG_ENOMEM = -3,     /* workspace or arena too small                            */
  DG_EDEVICE = -4,    /* a HIP call failed                                       */
  DG_ENONFINITE = -5, /* the state holds NaN or Inf                              */
  DG_EBUSY = -6,      /* request can never fit the server's memory budget        */
  DG_ESTATE = -7      /* object unusable after an earlier device error, or wrong call order */
};

/* Problem parameters.  gamma, R, Pr, mu: perfect gas; heat conductivity
 * lambda = gamma R mu(T) / ((gamma - 1) Pr) (Sec. 2.1), mu constant or by
 * Sutherland's law. */
typedef struct dg_params {
  int32_t abi_version;     /* must be DG_ABI_VERSION                                   */
  int32_t N;               /* polynomial degree, 1 <= N <= 9 (see below for the cap)   */
  int32_t nodes;           /* 0 Gauss-Legendre, 1 Gauss-Lobatto (required by shock capturing and the split form) */
  int32_t riemann;         /* 0 local Lax-Friedrichs, 1 Roe (no entropy fix)           */
  int32_t precision;       /* 0 FP64; 1 mixed: FP32 fluxes and contractions, FP64 state, RK, setup */
  int32_t viscous;         /* 0 Euler, 1 Navier-Stokes with BR1 lifting                */
  int32_t source;          /* 0 none, 1 manufactured-solution source of Sec. 5.1 (see below) */
  int32_t shock_capturing; /* 1: per-element DG/FV blend with the modal indicator (2 <= N <= 7) */
  int32_t check_finite;    /* 1: dg_advance checks the state after every step and reports the first non-finite one */
  int32_t reserved;
  double gamma, R, Pr, mu; /* mu: the constant viscosity, or mu(T_ref) under Sutherland's law */
  double alpha_max, alpha_min; /* blending clip: alpha < alpha_min -> 0, > 1-alpha_min -> 1, then min(alpha, alpha_max);
                                  0 <= alpha_min < 1/2, 0 <= alpha_max <= 1 */
  double ind_a, ind_c, ind_s;  /* threshold T = ind_a 10^(-ind_c (N+1)^(1/4)); alpha = 1/(1+exp(-ind_s/T (E-T))) */
  /* ---- since ABI version 2 ---- */
  int32_t volume_flux;     /* 0 standard weak-form volume integral (Eq. dgsem);
                              1 split form with Pirozzoli's kinetic-energy-preserving two-point flux
                                (Sec. 2.2 "Nonlinear Stability"; Gauss-Lobatto nodes only) */
  int32_t viscosity_law;   /* 0 constant mu; 1 Sutherland (Sec. 2.1 Eq. sutherland):
                              mu(T) = mu 1.4042 (T/T_ref)^(3/2) / (T/T_ref + 0.4042) */
  int32_t time_scheme;     /* 0 five-stage Carpenter-Kennedy 4(5); 1 fourteen-stage fourth-order
                              scheme of Niegemann, Diehl and Busch (both 2N-storage, Sec. 2.2 "Time integration") */
  int32_t alpha_smooth;    /* 0: alpha is the element's own indicator value, local to the element (Sec. 2.3);
                              1: raised to half the largest face neighbour's value, then alpha < alpha_min -> 0
                                 and min(alpha, alpha_max) (Hennemann's smoothing, not in the paper) */
  double T_ref;            /* Sutherland reference temperature (> 0 when viscosity_law = 1) */
  double p_ref;            /* mixed precision only: background pressure taken out of the FP32
                              arithmetic (the energy is carried as rho e - p_ref/(gamma-1));
                              0 = none.  Ignored in FP64. */
} dg_params;
/* The degree cap: one workgroup holds one element's (N+1)^3 tile and its face
 * arrays in LDS (at N = 9 the FP64 volume sweep takes 138 KB of the 160 KB of
 * a CU); N >= 10 would need a tile split across workgroups. */
/* source = 1: rho = 2 + 0.1 sin(pi(x+y+z-t)), u = v = w = 1, p = rho is an exact
 * solution once 0.1 pi cos(pi(x+y+z-t)) (2, 3, 3, 3, 2(3 gamma-2)/(gamma-1)) is added. */

/* Mesh.  Geometry nodes on the Gauss-Lobatto points of degree n_geo of every
 * element; the curl-form metric terms are computed from them.  Each element
 * face names its neighbour element, the neighbour's local face and an
 * orientation code mapping own face coordinates (p,q) to the neighbour's:
 * (a,b) = bit0 ? (q,p) : (p,q);  p' = bit1 ? N-a : a;  q' = bit2 ? N-b : b.
 * Periodic meshes list the periodic partner as the neighbour. */
typedef struct dg_mesh {
  int64_t n_elems;           /* >= 1, with n_elems (N+1)^3 < 2^31 and 6 n_elems (N+1)^2 < 2^31 */
  int32_t n_geo;             /* 1 <= n_geo <= N                                       */
  int32_t reserved;
  const double *x_geo;       /* host [n_elems][3][(n_geo+1)^3], i fastest             */
  const int64_t *nbr_elem;   /* host [n_elems][6]                                     */
  const int8_t *nbr_face;    /* host [n_elems][6], 0..5                               */
  const int8_t *nbr_orient;  /* host [n_elems][6], 0..7                               */
} dg_mesh;

typedef struct dg_solver dg_solver;

/* ABI version compiled into the library. */
int32_t dg_abi_version(void);

/* Bytes of device workspace one solver needs (Sec. 4.3 reports the paper's
 * memory per DOF; this is ours).  Sizes all state, metric, trace and scratch
 * arrays for n_elems elements.  DG_EINVAL on bad parameters or an n_elems
 * outside the range dg_mesh states. */
dg_status dg_workspace_bytes(const dg_params *p, int64_t n_elems, size_t *bytes);

/* Set up a solver: nodes and weights, D-hat and l-hat (Sec. 2.2 Eq. dgsem),
 * curl-form metrics and face normals (Sec. 2.2), connectivity checks, upload
 * into d_workspace (device, ws_bytes >= dg_workspace_bytes).  On success *out
 * holds a solver bound to hip_stream; the state is zero and t = 0.
 * DG_EMESH names the offending element and face; DG_ENOMEM if ws_bytes is short. */
dg_status dg_create(const dg_params *p, const dg_mesh *m, void *d_workspace, size_t ws_bytes,
                    void *hip_stream, dg_solver **out);

/* Load the state U ([5][E][(N+1)^3] doubles; host memory if on_device == 0,
 * else device memory) and set the time to t: the initial condition of the
 * semi-discrete system (Sec. 2.2, Eq. dgsem, integrated in time as in
 * "Time integration").  The RK register restarts: the next step's first
 * stage ignores what it held (A_1 = 0), so a state restored after a failure
 * steps cleanly.  Host copies synchronise the stream. */
dg_status dg_set_state(dg_solver *s, const double *U, int32_t on_device, double t);

/* Copy the state out (host: synchronises the stream) and return the time.
 * Time stepping keeps every array on the device; the host reads the solution
 * back for analysis only (Sec. 3, design principles). */
dg_status dg_get_state(dg_solver *s, double *U, int32_t on_device, double *t);

/* Stable time step of the current state: min over nodes of
 * cfl * 2/((2N+1) sum_i (|u.Ja^i| + c|Ja^i|)/J) and, if viscous,
 * dfl * 4/((N+1)^4 nu sum_i (|Ja^i|/J)^2), nu = max(4/3, gamma/Pr) mu/rho.
 * The paper does not give a formula; this is an estimate from the 1-D spectra. */
dg_status dg_stable_dt(dg_solver *s, double cfl, double dfl, double *dt);

/* Advance n_steps steps of size dt with the low-storage RK scheme of
 * time_scheme (Sec. 2.2 "Time integration"); each stage evaluates the full
 * operator: ProlongToFace, BR1 lifting, FillFlux, VolInt, SurfInt, ApplyJac,
 * optional FV blending (Sec. 2.3), then du = A_s du + dt R; U = U + B_s du.
 * Asynchronous.  With check_finite the state is checked on the device after
 * every step and the call synchronises after each check: at the first
 * non-finite step it stops, leaves that step's state and time in the solver,
 * names the step in dg_last_error and returns DG_ENONFINITE. */
dg_status dg_advance(dg_solver *s, int32_t n_steps, double dt);

/* One evaluation of the time derivative R(U, t) (Eq. dgsem) into Ut
 * ([5][E][(N+1)^3]; host if on_device == 0, which synchronises).  The state is unchanged. */
dg_status dg_rhs(dg_solver *s, double t, double *Ut, int32_t on_device);

/* Blending factors alpha of the last evaluation, one per element (host, [E]). */
dg_status dg_alpha(dg_solver *s, double *alpha_host);

/* Freeze alpha per element (host [E], copied) instead of the indicator;
 * NULL returns to the indicator.  A test hook for Sec. 2.3's blend. */
dg_status dg_set_alpha(dg_solver *s, const double *alpha_host);

/* Quadrature integrals of the state: out[0..4] = sum w J U (mass, momentum,
 * energy), out[5] = kinetic energy sum w J rho|u|^2/2 / |Omega| (Sec. 5.2 with
 * rho0 = U0 = 1), out[6] = |Omega| = sum w J. */
dg_status dg_integrals(dg_solver *s, double out[7]);

/* Dissipation rates of Sec. 5.2 of the current state, from the BR1-lifted
 * gradients g of one volume sweep (state and RK register unchanged):
 * out[0] = eps_S = (1/|Omega|) sum w J mu(T) |curl u|^2 (solenoidal),
 * out[1] = eps_D = (4/(3|Omega|)) sum w J mu(T) (div u)^2 (dilatational),
 * |Omega| = sum w J; with rho0 = U0 = L = 1 the paper's mu(T)/(mu0 Re) is
 * mu(T).  Per-element partial sums are reduced in a fixed order on the host
 * (synchronises).  DG_EINVAL without the viscous operator. */
dg_status dg_dissipation(dg_solver *s, double out[2]);

/* dg_dissipation for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same kernels and the same result, but the per-element partial sums go
 * to a file-scope device array of the library (6 MiB per GPU, held until the
 * process ends) instead of the solver's workspace.  At most 262144 elements
 * (DG_EINVAL above); the solver's workspace must be on the current device.
 * The first call on a device looks the array's address up once.  Every call
 * on a GPU shares that GPU's array: calls that overlap on one GPU race.
 * Makes no hipMalloc/hipFree call; synchronises the solver's stream. */
dg_status dg_dissipation_noalloc(dg_solver *s, double out[2]);

/* Wait for all work the solver enqueued on its stream (the host side of the
 * asynchronous stage launches of Sec. 3.2). */
dg_status dg_synchronize(dg_solver *s);

/* Message of the last failing call on this thread ("" if none). */
const char *dg_last_error(void);

/* Release host-side objects.  Never frees caller memory. */
void dg_destroy(dg_solver *s);

/* Per-kernel timing of dg_advance with HIP events recorded on the solver's
 * stream around every launch (off by default; adds events, not syncs).
 * dg_profile_read returns, for kernel k in 0..n-1 (0 trace, 1 lift, 2 rhs+update),
 * the summed milliseconds and launch counts since the last enable, then resets. */
dg_status dg_profile_enable(dg_solver *s, int32_t on);
dg_status dg_profile_read(dg_solver *s, int32_t n, double *ms, int64_t *launches);

/* -------------------------------------------------------------------------
 * Serving: many independent solves share one GPU.  Requests are admitted in
 * arrival order while the arena budget and the slot table allow; every tick
 * runs one RK stage for every active request, with one launch per kernel and
 * per polynomial degree covering all active requests of that degree; finished
 * requests are copied out and their memory is released.  The paper schedules
 * one solve over concurrent streams (Sec. 3.2); this batches many.
 * ------------------------------------------------------------------------- */
typedef struct dg_server dg_server;

enum { DG_REQ_QUEUED = 0, DG_REQ_RUNNING = 1, DG_REQ_DONE = 2, DG_REQ_FAILED = 3 };

typedef struct dg_timing {
  double t_arrival; /* given at submit (seconds on the server clock)      */
  double t_admit;   /* server clock (seconds since the first dg_server_run) when admitted */
  double t_done;    /* server clock when the result was copied out        */
  int32_t state;    /* DG_REQ_*                                           */
  int32_t reserved;
} dg_timing;

/* Create a server over a caller-owned device arena (d_arena, arena_bytes);
 * at most hbm_budget bytes of it are used at once and at most max_active
 * requests run together.  Work goes on hip_stream; uploads on
 * hip_copy_stream (may equal hip_stream).  The server allocates its pinned
 * host memory here, once: descriptor mirrors and 16 staging slots of 16 MiB
 * through which finished states are copied out in chunks. */
dg_status dg_server_create(void *d_arena, size_t arena_bytes, size_t hbm_budget, int32_t max_active,
                           void *hip_stream, void *hip_copy_stream, dg_server **out);

/* Queue one solve: parameters, mesh, initial state (host [5][E][(N+1)^3]),
 * n_steps of size dt.  dt < 0 asks for the stable step of dg_stable_dt with
 * CFL = DFL = -dt on the initial state, evaluated in FP64 on the host when
 * the request is prepared.  All host data is copied.  t_arrival: finite
 * seconds >= 0 on the server clock, which starts at the first dg_server_run
 * call (so a
 * stream can be submitted up front); the request becomes eligible for
 * admission once the server clock passes it.  Once a request has arrived, a
 * thread of the server builds its geometry and metrics while the serving loop
 * runs, reusing those of an identical mesh and set-up seen before (up to
 * 4 GiB of them are kept in host memory); a mesh that fails those checks ends
 * DG_REQ_FAILED.  DG_EBUSY if it can never fit the budget. */
dg_status dg_server_submit(dg_server *sv, const dg_params *p, const dg_mesh *m, const double *U0_host,
                           int32_t n_steps, double dt, double t_arrival, int64_t *req_id);

/* Drive the loop: admit -> one stage tick -> retire, up to max_ticks ticks
 * (<= 0: until every submitted request is done or failed). */
dg_status dg_server_run(dg_server *sv, int32_t max_ticks);

/* State of a request (DG_REQ_*). */
dg_status dg_server_poll(dg_server *sv, int64_t req_id, int32_t *state);

/* Copy a finished request's state ([5][E][(N+1)^3] doubles) and timing to the host. */
dg_status dg_server_fetch(dg_server *sv, int64_t req_id, double *U_host, dg_timing *timing);

/* Loop statistics since creation: out[0] ticks, out[1] mean active requests
 * per tick, host seconds spent in out[2] admission (set-up uploads), out[3]
 * tick issue (launches and descriptor copies, out[5] included), out[4]
 * retirement, out[5] waiting for the GPU to free a descriptor slot, out[6]
 * waiting with nothing to run; out[7] bytes uploaded at admission; out[8]
 * geometry blocks uploaded and out[9] admissions that found their mesh's
 * geometry resident (the arena keeps each mesh's read-only metrics, normals
 * and connectivity after its last request, shared by the requests of that
 * mesh, until the memory is needed). */
dg_status dg_server_stats(dg_server *sv, double out[10]);

void dg_server_destroy(dg_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* DGSEM_H */
