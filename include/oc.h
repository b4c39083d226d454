/*
 * oc.h -- C ABI of the MI355X (gfx950) hot path of the Oceananigans
 * nonhydrostatic ocean model (Wagner et al., arXiv 2502.14148).
 *
 * The library computes, on one GPU, the per-time-step loop of the
 * NonhydrostaticModel on a staggered Arakawa C-grid:
 *   - tendencies of u, v, w and the tracers: flux-form WENO5-Z advection
 *     (reconstruction subsection and momentum-advection subsection of the
 *     finite-volume appendix), f-plane Coriolis, linear-EOS buoyancy,
 *     constant-coefficient Laplacian closure and a prescribed top tracer flux
 *     (nonhydrostatic momentum and tracer equations);
 *   - low-storage RK3 substages (rk3 equation of the time-discretisation
 *     appendix);
 *   - the pressure correction: an FFT/DCT eigenfunction solve of the
 *     discrete Poisson equation and the projection of the predictor velocity
 *     (pressure-correction appendix, pressure-poisson equation).
 *
 * Conventions
 *   Grid: cells i = 0..nx-1 (x fastest), j, k likewise.  Face i is the left
 *   face of cell i.  u lives at (F,C,C), v at (C,F,C), w at (C,C,F), tracers
 *   and pressure at (C,C,C).  x and y are periodic; z is periodic or bounded
 *   by impenetrable, free-slip, no-flux walls (then w has nz+1 faces and the
 *   wall faces hold 0).
 *   Memory: all large device memory is BORROWED.  The caller allocates one
 *   device workspace of oc_model_workspace_size() bytes (e.g. a torch tensor)
 *   and keeps it alive until oc_model_destroy().  The library owns only small
 *   host metadata.
 *   Streams: every call that touches the GPU is enqueued asynchronously on
 *   the hipStream_t passed as `void* stream` (NULL = the null stream).
 *   Calls on one model must not overlap from several threads.
 *   Errors: every function returns OC_OK (0) or a negative OC_ERR_* code;
 *   oc_last_error() returns a per-thread message.  Arguments are validated
 *   before anything is enqueued; on error nothing is enqueued and no state
 *   changes.  Device-side faults surface at the next synchronising call.
 */
#ifndef OC_H
#define OC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  OC_OK = 0,
  OC_ERR_ARG = -1,          /* null pointer or out-of-range scalar        */
  OC_ERR_SHAPE = -2,        /* array shape does not match the grid        */
  OC_ERR_DTYPE = -3,        /* unsupported element type                   */
  OC_ERR_DEVICE = -4,       /* HIP runtime error                          */
  OC_ERR_UNSUPPORTED = -5,  /* configuration not supported by the kernels */
  OC_ERR_NONFINITE = -6     /* a NaN/Inf was detected in the state        */
};

enum { OC_PERIODIC = 0, OC_BOUNDED = 1 };
enum { OC_RECTILINEAR = 0, OC_LATLON = 1 };
enum { OC_NONHYDROSTATIC = 0, OC_HYDROSTATIC = 1 };
enum { OC_FP64 = 0, OC_FP32_MIXED = 1 };
enum {
  OC_ADV_NONE = 0,
  OC_ADV_WENO5Z = 1,
  OC_ADV_WENO5_LINEAR = 2,
  OC_ADV_WENO7Z = 3,
  OC_ADV_WENO7_LINEAR = 4,
  OC_ADV_WENO9Z = 5,
  OC_ADV_WENO9_LINEAR = 6
};
enum { OC_F32 = 0, OC_F64 = 1 };
enum { OC_LES_NONE = 0, OC_LES_SMAGORINSKY = 1, OC_LES_AMD = 2 };
/* Field identifiers: velocities, then tracers 0..ntracers-1; the
 * hydrostatic model adds its 2D barotropic fields (FP64): free surface eta
 * at cell centres (shape (1, ny, nx)), transports U at x faces (1, ny, nx)
 * and V at y faces (1, ny + 1, nx), the slow forcing Gbar of U and V (same
 * shapes as U and V), and the kinematic surface stress tau / rho_0
 * (m^2 s^-2) at u points (OC_TAUX, (1, ny, nx)) and v points (OC_TAUY,
 * (1, ny + 1, nx)), the surface momentum flux of the baroclinic step.  In the
 * hydrostatic model v has ny + 1 rows (y faces, walls included) and w is
 * diagnostic: it can be read (nz + 1 faces) but not set. */
enum { OC_U = 0, OC_V = 1, OC_W = 2, OC_TRACER0 = 3 };
enum { OC_ETA = 16, OC_UBT = 17, OC_VBT = 18, OC_GUBT = 19, OC_GVBT = 20, OC_TAUX = 21,
       OC_TAUY = 22 };
#define OC_MAX_TRACERS 4
#define OC_NDIAG 12

/* Grid: RectilinearGrid or LatitudeLongitudeGrid of the library subsection.
 *   OC_RECTILINEAR: domain [x0, x0+lx) x [y0, y0+ly) x [z0, z0+lz) in meters;
 *     x and y periodic and uniformly spaced, z per topology_z.  z is uniform,
 *     or stretched when z_faces is given: nz + 1 strictly increasing face
 *     positions (host array, copied at oc_grid_create) from z0 to z0 + lz,
 *     cells between consecutive faces, centres at the midpoints
 *     (one-dimensional staggered-grid listing of the finite-volume
 *     appendix).  Stretched z needs topology_z = OC_BOUNDED and 8 <= nz <=
 *     256; its pressure solve is the mixed FFT(x, y) - tridiagonal(z) one
 *     (pressure-correction appendix).
 *   OC_LATLON (thin spherical shell of `radius`): x0, lx are the longitude
 *     start and extent in degrees (periodic, lx = 360), y0, ly the latitude
 *     start and extent in degrees (walls at both ends), z0, lz in meters
 *     (walls at both ends). */
typedef struct {
  int32_t nx, ny, nz;       /* cells */
  int32_t topology_z;       /* OC_PERIODIC or OC_BOUNDED */
  double x0, lx;
  double y0, ly;
  double z0, lz;
  int32_t coord;            /* OC_RECTILINEAR or OC_LATLON */
  double radius;            /* OC_LATLON: sphere radius in meters */
  const double* z_faces;    /* OC_RECTILINEAR, bounded z: NULL (uniform) or
                               nz + 1 face positions (see above) */
} oc_grid_desc;

/* Model physics (NonhydrostaticModel arguments of the equations section). */
typedef struct {
  int32_t kind;             /* OC_NONHYDROSTATIC (rectilinear grid) or
                               OC_HYDROSTATIC (lat-lon grid, split-explicit
                               free surface; each field with its
                               three-cell halos under 2^32 bytes, else
                               OC_ERR_UNSUPPORTED) */
  int32_t precision;        /* OC_FP64: everything in FP64.  OC_FP32_MIXED:
                               state, tendencies and the stencil arithmetic in
                               FP32; divergence, Poisson solve and projection
                               arithmetic in FP64.  With buoyancy, FP32 keeps T
                               and S as anomalies about (t_ref, s_ref) (the
                               ABI always exchanges full values) */
  int32_t advection;        /* OC_ADV_*: WENO-Z of order 5, 7 or 9 (r shifted
                               order-r stencils, r = 3, 4, 5; reconstruction
                               subsection), the ideal-weight limit of each,
                               or none.  Momentum's advecting velocity is the
                               centred reconstruction one order lower (4, 6,
                               8).  Orders 7 and 9 widen the halo to 4 and 5
                               cells and are nonhydrostatic-only; ensembles
                               take WENO5-Z */
  double weno_eps;          /* WENO-Z regulariser (> 0) */
  int32_t weno_q;           /* WENO-Z exponent; only 2 is supported */
  int32_t ntracers;         /* 1..OC_MAX_TRACERS */
  int32_t buoyancy;         /* 1: tracers 0, 1 are T, S and b = g(alpha(T-T0) - beta(S-S0)) */
  double f;                 /* f-plane Coriolis parameter */
  double g, alpha, beta, t_ref, s_ref;
  double nu, kappa;         /* constant viscosity, diffusivity */
  double top_flux[OC_MAX_TRACERS]; /* upward tracer flux through the top wall */
  double depth;             /* OC_HYDROSTATIC: resting depth H (flat bottom) */
  double omega;             /* OC_HYDROSTATIC: planetary rotation rate */
  int32_t closure;          /* 1: reserve workspace for a learned closure
                               (oc_model_set_closure) */
  int32_t implicit_z;       /* OC_NONHYDROSTATIC with bounded z: 1 treats the
                               vertical part of the nu and kappa diffusion
                               implicitly (vertically implicit time
                               discretisation of the time-stepping appendix):
                               it leaves the tendencies, and after each RK3
                               combine every field solves
                               (1 - dt_eff d/dz K d/dz) X = X~ column by
                               column, dt_eff = (gamma_m - zeta_m) dt, before
                               the pressure correction */
  int32_t les;              /* OC_NONHYDROSTATIC: an eddy-viscosity LES closure
                               added to the constant nu, kappa (closure
                               paragraph of the nonhydrostatic model section):
                               OC_LES_SMAGORINSKY, nu_e = (C Delta)^2 |S|
                               sqrt(max(0, 1 - C_b N^2/|S|^2)), |S|^2 =
                               2 S_ij S_ij, Delta = (dx dy dz_c)^(1/3),
                               kappa_e = nu_e / Pr; or OC_LES_AMD (anisotropic
                               minimum dissipation), nu_e = max(0, -C sum_k
                               Delta_k^2 d_k u_i d_k u_j S_ij / |grad u|^2) and
                               per tracer kappa_e = max(0, -C sum_k Delta_k^2
                               d_k u_i d_k c d_i c / |grad c|^2).  The closure
                               adds d_j(2 nu_e S_ij) to G_u_i and
                               d_i(kappa_e d_i c) to G_c (stresses on the C-grid
                               edges, viscosities averaged from the centres; no
                               flux through walls).  Not with closure = 1. */
  double les_c;             /* C (C_s for Smagorinsky-Lilly, e.g. 0.16; the
                               AMD constant, e.g. 1/12); > 0 */
  double les_cb;            /* Smagorinsky-Lilly: C_b of the stratification
                               factor (>= 0; N^2 from the T, S buoyancy) */
  double les_pr;            /* Smagorinsky-Lilly: turbulent Prandtl number (> 0) */
  int32_t immersed;         /* OC_NONHYDROSTATIC on a uniform rectilinear grid:
                               1 reserves a grid-fitted immersed boundary
                               (immersed-boundary grid of the paper's examples;
                               set the immersed cells with oc_set_immersed).
                               Faces next to an immersed cell are closed: zero
                               velocity and velocity tendency, no diffusive
                               tracer flux, no top flux into an immersed top
                               cell.  The pressure then solves the Poisson
                               equation on the fluid cells with no flux through
                               closed faces by conjugate gradients
                               preconditioned with the FFT solver of the whole
                               box applied to the masked residual (pressure
                               solver for irregular domains of the
                               pressure-correction appendix); gauge: zero mean
                               over the fluid cells.  WENO5 or no advection; not
                               with implicit_z, les or closure */
  double cg_tol;            /* immersed: relative residual at which the
                               iteration stops (> 0, e.g. 1e-13 in FP64) */
  int32_t cg_maxiter;       /* immersed: at most this many iterations (1..10000) */
} oc_model_desc;

typedef struct oc_grid oc_grid;
typedef struct oc_model oc_model;

/* Per-thread message of the last failing call ("" if none). */
const char* oc_last_error(void);

/* Validate `d` and create a grid handle (host memory only).  Rectilinear
 * grids (for the nonhydrostatic model's FFT solver) support lengths 8, 16,
 * 32, 64, 96, 128, 256 in x, y, z with ny even; lat-lon grids any nx, ny,
 * nz >= 8 with nx, ny multiples of 8.  Errors: OC_ERR_ARG, OC_ERR_UNSUPPORTED. */
int oc_grid_create(const oc_grid_desc* d, oc_grid** out);
int oc_grid_destroy(oc_grid* g);

/* Bytes of device workspace a model needs (state x2, tendencies, spectrum,
 * pressure, tables, reduction scratch). */
int oc_model_workspace_size(const oc_grid* g, const oc_model_desc* m, uint64_t* bytes);

/* Create a model on the current HIP device.  `workspace` is a device pointer
 * (256-byte aligned) of at least oc_model_workspace_size() bytes, borrowed
 * for the model's lifetime.  Uploads small tables synchronously and zeroes
 * the state.  Errors: OC_ERR_ARG, OC_ERR_UNSUPPORTED, OC_ERR_DEVICE. */
int oc_model_create(const oc_grid* g, const oc_model_desc* m, void* workspace,
                    uint64_t workspace_bytes, oc_model** out);
int oc_model_destroy(oc_model* m);

/* Copy interior values of `field` in (set) or out (get).  `buf` holds
 * shape[0] x shape[1] x shape[2] = (nz_f, ny, nx) elements, x fastest, of
 * type `dtype` (OC_F32 / OC_F64), in device memory if on_device else host
 * memory; nz_f = nz + 1 for w with walls, nz otherwise.  Values are
 * converted to the model precision; oc_set_state then refills the halos
 * (and sets w = 0 on walls).  Host copies synchronise the stream.  The
 * state refers to the current time level (after the last completed step). */
int oc_set_state(oc_model* m, int32_t field, const void* buf, int32_t dtype,
                 int32_t on_device, const int64_t shape[3], void* stream);
int oc_get_state(oc_model* m, int32_t field, void* buf, int32_t dtype,
                 int32_t on_device, const int64_t shape[3], void* stream);

/* Tendencies G of all prognostic fields from the current state, excluding
 * the nonhydrostatic pressure gradient (momentum-tendency-definition
 * equation); read them with oc_get_tendency (same layout as oc_get_state;
 * wall faces of G_w are 0). */
int oc_tendencies(oc_model* m, void* stream);
int oc_get_tendency(oc_model* m, int32_t field, void* buf, int32_t dtype,
                    int32_t on_device, const int64_t shape[3], void* stream);

/* Pressure correction of the current velocity as a predictor:
 * rhs = div(u)/dt_eff, solve lap p = rhs (mean-zero p), u -= dt_eff grad p
 * at interior faces, halos refilled.  Errors: OC_ERR_ARG if dt_eff <= 0.
 * oc_get_pressure copies the p of the model's last solve (this call, or the
 * last substage of oc_rk3_step / oc_ensemble_step) to buf: FP64, shape
 * (nz, ny, nx).  Without an immersed boundary the solve keeps p only as its
 * x-spectrum (the projection transforms it on the fly), and the first
 * oc_get_pressure after a solve enqueues the inverse x transform on
 * `stream` before the copy; with on_device = 0 it waits for the copy. */
int oc_pressure_solve(oc_model* m, double dt_eff, void* stream);
int oc_get_pressure(oc_model* m, double* buf, int32_t on_device, void* stream);

/* Advance nsteps full RK3 steps of size dt: per substage m the fused
 * tendency + RK3 combine X~ = X + dt(gamma_m G^m - zeta_m G^{m-1}),
 * with implicit_z the implicit vertical diffusion over dt_eff, then the
 * pressure correction with dt_eff = (gamma_m - zeta_m) dt. */
int oc_rk3_step(oc_model* m, double dt, int32_t nsteps, void* stream);

/* One implicit vertical-diffusion solve of the current state (the step that
 * oc_rk3_step applies after each combine when implicit_z is set; tracer- and
 * predictor-velocity time-discretisation equations): every column of u, v
 * and the tracers solves (1 - dt_eff d/dz K d/dz) X^new = X with no
 * diffusive flux through the walls (K = nu for u, v; kappa for tracers),
 * and w on the interior faces with w = 0 on the walls (K = nu); second-order
 * operator on the (stretched) z grid; halos refilled.  Tridiagonal
 * elimination with factors precomputed in FP64 per (dt_eff, K).  Needs a
 * nonhydrostatic model with bounded z.  Errors: OC_ERR_ARG (dt_eff <= 0),
 * OC_ERR_UNSUPPORTED. */
int oc_implicit_vertical_diffusion(oc_model* m, double dt_eff, void* stream);

/* Immersed cells of a model created with immersed = 1 (grid-fitted
 * immersed boundary; see oc_model_desc.immersed).  solid: HOST array of
 * nz * ny * nx bytes, x fastest, nonzero = immersed (the library copies it;
 * the caller keeps ownership).  All cells are fluid until the first call.
 * The call also zeroes the velocities of the current state on the faces it
 * closes and refills their halos; so does every later oc_set_state of u, v
 * or w on such a model.  Synchronous with respect to the host.
 * Errors: OC_ERR_ARG (NULL arguments), OC_ERR_UNSUPPORTED (immersed = 0, or
 * no fluid cell left). */
int oc_set_immersed(oc_model* m, const uint8_t* solid, void* stream);

/* Conjugate-gradient statistics of the last pressure solve of an immersed
 * model: iterations taken and the final relative residual |r| / |b| (host
 * outputs; synchronises the stream).  Errors: OC_ERR_ARG, OC_ERR_UNSUPPORTED
 * (immersed = 0). */
int oc_pressure_stats(oc_model* m, int32_t* iterations, double* rel_residual, void* stream);

/* Per-kernel-class timing with HIP events recorded on the model's stream
 * around every launch (classes: OC_PROF_*).  oc_profile(m, 1) clears the
 * counters and starts recording, oc_profile(m, 0) stops.  oc_profile_read
 * synchronises on the recorded events and writes OC_NPROF totals: ms (host
 * double array) and launches (host int64 array). */
enum {
  OC_PROF_TENDENCY = 0, OC_PROF_FFT_X_FWD = 1, OC_PROF_FFT_Y_FWD = 2, OC_PROF_Z_SOLVE = 3,
  OC_PROF_FFT_Y_INV = 4, OC_PROF_FFT_X_INV = 5, OC_PROF_PROJECT = 6, OC_PROF_HALO = 7,
  OC_PROF_CLOSURE = 8, OC_PROF_HYDRO_DIAG = 9, OC_PROF_HYDRO_TEND = 10, OC_PROF_BAROTROPIC = 11,
  OC_PROF_IMPLICIT_Z = 12, OC_PROF_LES = 13, OC_PROF_CG = 14
};
#define OC_NPROF 15
int oc_profile(oc_model* m, int32_t enable);
int oc_profile_read(oc_model* m, double* ms, int64_t* launches);
/* Restrict the event recording to the classes whose bit (1 << OC_PROF_*) is
 * set in `classes` (a model starts with all of them): a run that times only
 * one kernel class records two events per launch of that class and none
 * around the others.  Bits at or above OC_NPROF: OC_ERR_ARG. */
int oc_profile_classes(oc_model* m, uint32_t classes);

/* Split-explicit barotropic mode of the hydrostatic model (hydrostatic
 * time-discretisation appendix): M forward-backward substeps of length
 * dt / N of the FP64 free surface eta and transports (U, V) under the frozen
 * slow forcing Gbar,
 *     eta <- eta - dtau div_h(U, V);  (U, V) <- (U, V) - dtau (g H grad_h eta - Gbar),
 * accumulating etabar = sum a_n eta^n and (Ubar, Vbar) = sum a_n (U, V)^n
 * over n = 1..M; then the correction of the baroclinic velocity,
 * u <- u + (Ubar - sum_k dz u) / H (v likewise at interior y faces), and the
 * restart eta = etabar, (U, V) = (Ubar, Vbar).  `a` is a host array of M
 * weights (the filter is the caller's choice).  Linear free surface (H
 * fixed), no Coriolis in the substeps.  Errors: OC_ERR_UNSUPPORTED for a
 * nonhydrostatic model, OC_ERR_ARG for N < 1, M < 1, M > 4096 or NULL a. */
int oc_free_surface_substeps(oc_model* m, double dt, int32_t N, int32_t M, const double* a,
                             void* stream);

/* nsteps baroclinic steps of the hydrostatic model (hydrostatic-model
 * subsection; hydrostatic time-discretisation appendix).  Per step:
 *   1. column scans: w from the floor up (dw/dz = -div_h u_h, w = 0 on the
 *      floor), the hydrostatic pressure gradient from dp/dz = b with p = 0
 *      at the surface, and the vertical vorticity at cell corners;
 *   2. tendencies G^n of u, v, T, S: WENO vector-invariant momentum
 *      advection, f = 2 Omega sin(latitude) Coriolis, hydrostatic pressure
 *      gradient, vertical viscosity with the surface stress OC_TAUX/OC_TAUY,
 *      flux-form WENO tracer advection on the shell's metrics, vertical
 *      diffusion; the QAB2 predictor X~ = X + dt [(3/2 + chi) G^n -
 *      (1/2 + chi) G^{n-1}] with chi = 0.1, and Gbar = sum_k dz [...] of u, v
 *      in FP64;
 *   3. the split-explicit barotropic substeps, correction and restart of
 *      oc_free_surface_substeps with the same N, M, a.
 * The first step after model creation or after oc_set_state of a 3D field
 * is an Euler step (chi = -1/2).  State precision per the model descriptor;
 * eta, U, V, Gbar FP64.  After the call G (oc_get_tendency) holds G^n of
 * the last step and w (oc_get_state, OC_W) the diagnosed velocity of the new
 * state.  Errors: OC_ERR_UNSUPPORTED for a nonhydrostatic model, OC_ERR_ARG
 * for dt <= 0, N < 1, M < 1, M > 4096, nsteps < 0, a NULL or non-finite a,
 * OC_ERR_DEVICE on a HIP failure. */
int oc_hydrostatic_step(oc_model* m, double dt, int32_t N, int32_t M, const double* a,
                        int32_t nsteps, void* stream);

/* ---- Ensembles: many nonhydrostatic models stepped together ----
 * The paper's case for GPUs is the throughput of many moderate-size
 * simulations (introduction; ensembles for parameter studies).  An ensemble
 * borrows existing models (created, filled and read with the calls above;
 * they must outlive it) and advances all of them by the RK3 step of
 * oc_rk3_step with one dt: per substage one fused tendency + RK3 launch over
 * every member's column tiles, and per class of members with equal grids one
 * launch per Poisson pass.  Results equal those of oc_rk3_step on each
 * member.  Members: nonhydrostatic, WENO5-Z, tracers T and S, no learned
 * closure, uniform grids without implicit vertical diffusion, one
 * precision, nx and ny multiples of 8.
 * Flags: OC_ENS_TUNE times the candidate launch configurations (column tile
 * 32x8, 16x8 or 8x8; one workgroup per tile or a persistent grid draining an
 * atomic work queue; k-chunk length) at creation and keeps the fastest, as
 * oc_autotune with no cache does.  OC_ENS_GRAPH captures one RK3 step per
 * buffer parity as a HIP graph on the first call (again when dt or the
 * launch configuration changes) and replays it.
 * Workspace: caller-owned device memory of oc_ensemble_workspace_size bytes
 * (member tables, work list, Poisson pointer tables). */
typedef struct oc_ensemble oc_ensemble;
enum { OC_ENS_TUNE = 1, OC_ENS_GRAPH = 2 };
/* Errors: OC_ERR_ARG (NULL, count outside 1..4096, repeated member, mixed
 * precision), OC_ERR_UNSUPPORTED (a member outside the list above). */
int oc_ensemble_workspace_size(oc_model* const* members, int32_t count, uint64_t* bytes);
int oc_ensemble_create(oc_model* const* members, int32_t count, void* workspace, uint64_t bytes,
                       int32_t flags, oc_ensemble** out);
/* nsteps RK3 steps of every member on `stream`; afterwards each member's
 * state is read as usual.  A member stepped on its own in between is picked
 * up where it stands.  Errors: OC_ERR_ARG for dt <= 0 or nsteps < 0,
 * OC_ERR_DEVICE on a HIP failure. */
int oc_ensemble_step(oc_ensemble* e, double dt, int32_t nsteps, void* stream);
/* The launch configuration in use: out[0] tile (0: 32x8, 1: 16x8, 2: 8x8),
 * out[1] persistent grid (0/1), out[2] workgroups of the persistent grid,
 * out[3] k-chunk divisor, out[4] 0 default / 1 timed / 2 from the cache /
 * 3 set by oc_ensemble_set_tuning, out[5] work items per launch; *ms
 * (optional) the timed launch. */
int oc_ensemble_tuning(const oc_ensemble* e, int32_t* out, double* ms);
/* The project's autotuner (the batching form of the build: tile shapes of
 * the fused tendency launch picked by measurement).  Synchronous: waits for
 * the device, then times every candidate (column tile 32x8, 16x8, 8x8; flat
 * or persistent grid; k-chunk divisor 256, 1024, 4096) on substage-1
 * launches that read the members' current states and write only buffers
 * that the next step overwrites, and keeps the fastest.  cache_path (host
 * string, may be NULL): a JSON-lines file, one object per choice,
 * {"key": arch|precision|sizes, "tile": t, "persistent": p, "kc_div": k,
 * "ms": x}; a line with this ensemble's key is used instead of timing (the
 * last such line wins), and a timed choice is appended.  An unreadable or
 * unwritable file is treated as absent.  Captured graphs are dropped and
 * recaptured on the next step.  Errors: OC_ERR_ARG (NULL ensemble),
 * OC_ERR_DEVICE. */
int oc_autotune(oc_ensemble* e, const char* cache_path);
/* Force a launch configuration (host array of 3): tuning[0] tile (0: 32x8,
 * 1: 16x8, 2: 8x8), tuning[1] persistent grid (0/1), tuning[2] k-chunk
 * divisor (>= 1: a member's k chunk is nz * tiles / divisor levels, clamped
 * to 4..64).  Synchronous like oc_autotune; results do not depend on the
 * configuration.  Errors: OC_ERR_ARG (values outside these ranges, or a tile
 * that does not divide some member's nx and ny). */
int oc_ensemble_set_tuning(oc_ensemble* e, const int32_t* tuning);
int oc_ensemble_destroy(oc_ensemble* e);

/* ---- Learned subgrid closure (an MLP trained on coarse-grained fluxes) ----
 * The network maps the standardised 5x5x5 neighbourhood of (u, v, w, b) of a
 * coarse cell (500 values, variable-major, offsets (dk, dj, di) in C order)
 * through two 256-wide exact-erf GELU layers to 4 standardised vertical
 * subgrid fluxes (tau_uw, tau_vw, tau_ww, J_bw).  GEMMs use BF16 operands
 * with FP32 accumulation (MFMA); master weights and Adam state are FP32.
 * Parameters are packed FP32: W1 (256 x 500, row = output) | b1 (256) |
 * W2 (256 x 256) | b2 | W3 (4 x 256) | b3 (4): OC_MLP_NPARAM values.
 * The paper names trainable parameterizations as a goal (introduction,
 * conclusions); coarse-graining follows its integral-preserving regridding
 * (finite-volume appendix). */
#define OC_MLP_NPARAM 195076
typedef struct oc_mlp oc_mlp;

/* Device workspace for batches up to max_batch (a multiple of 32). */
int oc_mlp_workspace_size(int32_t max_batch, uint64_t* bytes);
/* Create on the current device over a borrowed, 256-byte aligned device
 * workspace; parameters start at zero. */
int oc_mlp_create(int32_t max_batch, void* workspace, uint64_t bytes, oc_mlp** out);
int oc_mlp_destroy(oc_mlp* m);
/* Upload (host FP32, OC_MLP_NPARAM values; OC_ERR_NONFINITE on NaN/Inf)
 * and reset the optimiser; synchronous. */
int oc_mlp_set_params(oc_mlp* m, const float* params, void* stream);
int oc_mlp_get_params(oc_mlp* m, float* params, void* stream);
/* y (device, batch x 4 FP32) = MLP(x) for x (device, batch x 500 FP32);
 * batch a multiple of 32 up to max_batch. */
int oc_mlp_forward(oc_mlp* m, const float* x, int32_t batch, float* y, void* stream);
/* Gradients of the mean squared error mean((y - target)^2) over the batch
 * (target: device, batch x 4) into grad (device, OC_MLP_NPARAM FP32, packed
 * like the parameters); *loss (host, optional) receives the loss,
 * synchronising the stream. */
int oc_mlp_gradients(oc_mlp* m, const float* x, const float* target, int32_t batch, float* grad,
                     double* loss, void* stream);
/* One Adam step (beta = 0.9, 0.999, eps = 1e-8) with learning rate lr on
 * the same loss; *loss (optional) as above. */
int oc_mlp_train_step(oc_mlp* m, const float* x, const float* target, int32_t batch, float lr,
                      double* loss, void* stream);

/* Attach (net != NULL) or detach (net == NULL) the learned closure of a
 * nonhydrostatic model created with closure = 1 (walls in z, uniform
 * spacing; tracers 0, 1 = T, S).  Every substage then gathers the standardised features of all
 * cells, runs the network (the model's cell count must be a multiple of 32
 * and at most the network's max_batch) and adds the flux divergence of the
 * predicted vertical fluxes -d/dz(F) to G: u and v take F at their (x or y
 * face, z face) edges as the mean of the four adjacent centres, T the mean
 * of the two centres about a z face (as J_b / (g alpha)), w the difference
 * of tau_ww across its face; wall fluxes are zero, so column integrals are
 * conserved.  stats (host, 16 doubles): input mean and std of (u, v, w, b),
 * output mean and std of (tau_uw, tau_vw, tau_ww, J_b).  The model's
 * constant-diffusivity closure stays on.  A network whose parameters are not
 * all finite is refused with OC_ERR_NONFINITE and the model keeps running
 * without it (the diffusive fallback).  The network must outlive the
 * attachment. */
int oc_model_set_closure(oc_model* m, oc_mlp* net, const double* stats, void* stream);

/* The network input of every cell of the model's current state: x (device,
 * FP32, ncell x 500, cells in (k, j, i) order, x fastest), standardised with
 * stats[0..7] (input means and standard deviations of u, v, w, b; stats as
 * for oc_model_set_closure, the output half unused).  For training data.
 * Errors: OC_ERR_UNSUPPORTED without walls in z, with stretched z or
 * without T, S buoyancy. */
int oc_closure_features(oc_model* m, const double* stats, float* x, void* stream);

/* Coarse-graining (the regridding paragraph of the finite-volume appendix:
 * volume- and area-weighted averages that preserve integrals and the
 * discrete divergence): the state of `coarse` becomes the average of the
 * current state of `fine`, refined by one integer factor r in x, y and z
 * over the same domain: centred fields over r^3 cells, u (v, w) over the r^2
 * fine faces on each coarse face; halos refilled.  fluxes (device, FP32,
 * (4, nz, ny, nx) of the coarse grid, may be NULL) receives the vertical
 * subgrid fluxes <q w> - <q><w> over each r^3 box, q = u, v, w, b, with the
 * velocities first averaged to the fine cell centres (physical units).
 * Sums in FP64.  Errors: OC_ERR_UNSUPPORTED (not wall-bounded, stretched
 * z, no T, S buoyancy), OC_ERR_SHAPE (grids not related by one factor), OC_ERR_ARG
 * (different precision, domain or tracer storage). */
int oc_coarse_grain(oc_model* fine, oc_model* coarse, float* fluxes, void* stream);

/* FP64 diagnostics of the current state of a nonhydrostatic model, with
 * every sum taken in one fixed order (deterministic), synchronous; out (host)
 * receives OC_NDIAG doubles:
 *   [0] max|div u| * min(spacing) (the discrete divergence of the
 *       pressure-correction method, dimensionless once divided by max|u|),
 *   [1] max|u|, [2] max|v|, [3] max|w|,
 *   [4..7] volume integrals of tracers 0..3 (0 if absent): the sum of cell
 *       value times cell volume, the finite-volume integral,
 *   [8..10] volume integrals of u, v, w over their own control volumes
 *       (u, v: the cell's volume; w: dx dy times the spacing of the centres
 *       either side of the face),
 *   [11] the advective CFL rate max(max|u|/dx, max|v|/dy, max|w|/dz_min) in
 *       1/s; the CFL number of a step dt is dt times it.
 * Errors: OC_ERR_NONFINITE if any state value is NaN or Inf (the values are
 * still written), OC_ERR_UNSUPPORTED for a hydrostatic model. */
int oc_diagnostics(oc_model* m, double* out, void* stream);

/* For callers that cannot allocate device memory or wait for the device
 * (code under HIP graph capture, tight serving loops): the values of
 * oc_diagnostics, computed and finished on the device, written
 * asynchronously on `stream` to out (device memory, OC_NDIAG + 1 doubles:
 * out[0 .. OC_NDIAG-1] as oc_diagnostics, out[OC_NDIAG] the number of
 * non-finite state values, which the caller checks instead of an error
 * code).  Partial sums go to a library-held device array of 256 levels x 12
 * doubles (24 KiB) per GPU, kept until the process ends; every call on that
 * GPU shares it, so calls that overlap on one GPU race.  Nothing is
 * allocated, copied to the host or waited for; sums are taken level by level
 * in a fixed order (maxima and the count equal oc_diagnostics', sums agree to
 * rounding).  Errors: OC_ERR_ARG (NULL), OC_ERR_UNSUPPORTED (hydrostatic
 * model), OC_ERR_SHAPE (more than 256 levels), OC_ERR_DEVICE. */
int oc_diagnostics_noalloc(oc_model* m, double* out, void* stream);

/* Synchronise `stream` and report what the device has done since the last
 * check: OC_ERR_DEVICE for a HIP error (message from the runtime), then, for
 * a nonhydrostatic model, OC_ERR_NONFINITE if the current state holds a NaN
 * or Inf (the NaN guard of oc_diagnostics).  OC_OK otherwise. */
int oc_sync_check(oc_model* m, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* OC_H */
