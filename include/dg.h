/*
 * dg.h -- C ABI of the MI355X (gfx950) nodal discontinuous Galerkin solver
 * core for the 3-D compressible Euler equations on a periodic Cartesian
 * hexahedral mesh, with its five-stage fourth-order low-storage Runge-Kutta
 * stage update.
 *
 * Method: Kirby & Mavriplis, "GPU-Accelerated Discontinuous Galerkin Methods:
 * 30x Speedup on 345 Billion Unknowns".
 *   - Equations: Eq. (1) conservation form, Eq. (2) state Q and flux columns
 *     F^1..F^3 (total enthalpy H = E + p/rho), Eq. (3) ideal-gas closure.
 *   - Discretisation: Section II-B, Eq. (4)-(5) weak form, Eq. (6)-(7) nodal
 *     Lagrange basis through N = p+1 Gauss-Legendre points per direction,
 *     collocated quadrature (Section I), Lax-Friedrichs face flux.
 *   - Time integration: Sections II-B, IV, V: five-stage fourth-order
 *     low-storage explicit Runge-Kutta (LSERK45).
 *   - Volume term sum-factorised along 1-D lines: Section IV, Listing 1.
 *
 * Conventions that hold for every entry point:
 *   Layout.  Every state-sized array is a DEVICE pointer to
 *     5 * E * N^3 doubles, E = nx*ny*nz, in the order
 *     [field][ez][ey][ex][k][j][i]: fields rho, rho u, rho v, rho w, rho E;
 *     element index ex fastest among elements; node index i (x direction)
 *     fastest inside an element.  Element (ex,ey,ez) covers
 *     [ex hx,(ex+1)hx] x [ey hy,(ey+1)hy] x [ez hz,(ez+1)hz], h_d = L_d/n_d;
 *     node (i,j,k) sits at the Gauss-Legendre points (xi_i, xi_j, xi_k) of
 *     that box.  Neighbours are periodic.
 *   Alignment.  State arrays must be 8-byte aligned, as any array of doubles
 *     is (DG_EINVAL otherwise): the kernels read them in 8- and 16-byte pieces.
 *   Ownership.  The caller owns every array and the workspace (allocated by
 *     PyTorch or hipMalloc); the library owns only the context.  The library
 *     performs no device allocation.
 *   Streams.  Every call runs asynchronously on the context's stream (default
 *     stream 0 until dg_set_stream) except those marked SYNCHRONISING, which
 *     wait for their own result.  A context is not thread-safe.
 *   Errors.  Functions return DG_OK (0) or a negative DG_E* code and set a
 *     thread-local message readable with dg_last_error().  Argument errors are
 *     detected before any launch and leave every array untouched.  A failed
 *     launch returns DG_EHIP.  Faults inside kernels surface at the next
 *     synchronising call.  The hot path does no physical checks: a
 *     non-physical state propagates NaN/Inf.
 *   Aliasing.  Q must not overlap R, res or gQ (DG_EALIAS).
 *   Degrees.  p = 0..7 (N = 1..8).
 */
#ifndef DG_H
#define DG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_ctx dg_ctx;

enum {
  DG_OK = 0,
  DG_EINVAL = -1,        /* bad argument (NULL, size, range) */
  DG_EUNSUPPORTED = -2,  /* valid request outside what the library supports */
  DG_EHIP = -3,          /* HIP runtime error (launch, copy, sync) */
  DG_EALIAS = -4,        /* forbidden overlap between arrays */
  DG_ENONPHYSICAL = -5,  /* dg_check_state found rho<=0, p<=0 or NaN/Inf */
  DG_EWORKSPACE = -6     /* no workspace set, or too small */
};

enum {
  DG_FP64 = 0,       /* all arithmetic in FP64 */
  DG_FP32_MFMA = 1   /* tensor-product contractions on FP32 matrix cores,
                        RK accumulation and all state in FP64 */
};

/* Create a context for an nx*ny*nz periodic mesh of degree p (0..7) and
 * ratio of specific heats gamma (> 1; Eq. (3) uses 1.4).  The domain is
 * [0,1]^3 until dg_set_domain.  Returns NULL on error (dg_last_error()).
 * Builds the Gauss-Legendre rule, the 1-D differentiation matrix and the
 * face interpolation weights on the host (Section II-B, Eqs. (6)-(7)). */
dg_ctx* dg_create(int nx, int ny, int nz, int p, double gamma);

/* Destroy a context (NULL is allowed).  Does not free caller memory. */
void dg_destroy(dg_ctx* ctx);

/* Message of the last error on the calling thread ("" if none). */
const char* dg_last_error(void);

/* Domain lengths Lx, Ly, Lz (> 0); element sizes h_d = L_d / n_d. */
int dg_set_domain(dg_ctx* ctx, double Lx, double Ly, double Lz);

/* HIP stream (hipStream_t passed as void*; NULL = default stream) on which
 * every later call of this context is enqueued. */
int dg_set_stream(dg_ctx* ctx, void* hip_stream);

/* Arithmetic of the RHS contractions: DG_FP64 (default) or DG_FP32_MFMA.
 * DG_EUNSUPPORTED if the mode is not available for this p. */
int dg_set_precision(dg_ctx* ctx, int mode);

/* Viscous terms (Navier-Stokes).  The paper's CPU code has a viscous
 * formulation (Section III, Fig. 2) that the paper does not print; the one
 * built here: constant dynamic viscosity mu >= 0, Stokes' hypothesis,
 * Fourier conduction with conductivity mu gamma / ((gamma - 1) Pr) (gas
 * constant 1: T = p / rho), discretised by Bassi & Rebay's first scheme on
 * the same collocated basis: the gradients of (u, v, w, T) are weak
 * derivatives of their nodal interpolants with central face means, the
 * viscous flux is evaluated at the nodes and enters Eq. (5) beside the
 * inviscid flux with the central mean of both sides' traces.  mu = 0
 * (default) is the Euler equations.  With mu > 0: dg_rhs, dg_rk_stage,
 * dg_rk_step(s) and dg_rk_graph_steps (which then launches directly) add
 * the viscous terms in FP64 (the inviscid part follows dg_set_precision);
 * dg_workspace_bytes grows by 17 N^3 E doubles, so set the viscosity before
 * the workspace; the adjoint calls and dg_rk_steps_noalloc return
 * DG_EUNSUPPORTED.  DG_EINVAL for mu < 0, Pr <= 0 or non-finite values. */
int dg_set_viscosity(dg_ctx* ctx, double mu, double prandtl);

/* Volume term of the inviscid flux.  DG_VOLUME_STANDARD (default): the weak
 * form of Eq. (5) with the volume integral of the flux at the collocated
 * nodes.  DG_VOLUME_KEP: a kinetic-energy-preserving split form (the paper
 * cites such flux schemes of its authors' framework, reference list, without
 * printing one): flux differencing with Kennedy & Gruber's two-point flux
 * ({rho}{u_d}, {rho}{u_d}{u_k} + {p} delta_kd, {rho}{u_d}{e} + {p}{u_d}, {.}
 * the mean of two states, e = E / rho) along every d-line, whose
 * Gauss-Legendre nodes are coupled with the two face traces by the
 * hybridised summation-by-parts operator; the faces keep the local
 * Lax-Friedrichs flux.  With the central two-point flux the form is the
 * standard one.  The split form is FP64 only (DG_EUNSUPPORTED with
 * DG_FP32_MFMA, in either order of the two calls); dg_rhs, dg_rk_stage,
 * dg_rk_step(s), dg_rk_graph_steps (launching directly) and the viscous
 * terms follow it; the adjoint calls and dg_rk_steps_noalloc return
 * DG_EUNSUPPORTED while it is set. */
enum { DG_VOLUME_STANDARD = 0, DG_VOLUME_KEP = 1 };
int dg_set_volume_form(dg_ctx* ctx, int form);

/* Tuning options (dg_set_option).
 * DG_OPT_EXCHANGE: how an FP64 stage obtains its neighbours' face traces.
 *   DG_EXCHANGE_NEIGHBOUR (default): interpolated in the launch itself from
 *   the neighbour elements' state (read through the caches); the state is
 *   ping-ponged between the caller's Q and a workspace buffer, so a call
 *   with an odd number of stages ends with one device-to-device copy.
 *   DG_EXCHANGE_TRACES: every launch writes the face traces of its updated
 *   state to a workspace buffer that the next launch reads.
 *   Both give bitwise identical results.
 * The remaining options change only the order in which the neighbour-read
 * stage visits elements; the results are bitwise the same for every
 * setting.
 * DG_OPT_ORDER: the stage kernel works on blocks of consecutive elements of
 *   one x-row.  DG_ORDER_LINEAR visits them in index order;
 *   DG_ORDER_PENCIL visits pencils of PENCIL_X x PENCIL_Z elements (x by z)
 *   swept along y, so that every neighbour of an element is visited shortly
 *   before or after it and is still in L2.  Needs no condition on the mesh
 *   (ragged pencils and rows are handled).
 * DG_OPT_PENCIL_X: elements of a pencil along x (rounded up to the
 *   kernel's block of elements; 0 = the whole row).
 * DG_OPT_PENCIL_Z: element planes of a pencil along z (>= 1).
 * DG_OPT_XCD_REMAP: 1 gives each of the 8 XCDs of the MI355X (each with
 *   its own L2) a contiguous part of the visiting order; 0 leaves the
 *   hardware's round-robin spread of workgroups over the XCDs.
 * DG_OPT_VISC_FUSED: with viscosity set (FP64, standard volume form), 1
 *   forms the inviscid rate inside the viscous-flux launch from the
 *   neighbour loads that launch makes anyway; 0 gives it a launch of its
 *   own (the neighbour-read kernel).  Bitwise the same results.
 * Defaults (read back with dg_get_option): DG_EXCHANGE_NEIGHBOUR,
 * DG_ORDER_PENCIL with 16 x 8 pencils, DG_OPT_XCD_REMAP 1 and
 * DG_OPT_VISC_FUSED 1, the fastest setting measured on the Taylor-Green
 * workloads at p = 3, 4 and 6. */
enum {
  DG_OPT_EXCHANGE = 1,
  DG_OPT_XCD_REMAP = 2,
  DG_OPT_ORDER = 3,
  DG_OPT_PENCIL_X = 4,
  DG_OPT_PENCIL_Z = 5,
  DG_OPT_BATCH_LAUNCH = 6,  /* batched meshes only (dg_batch_set_option) */
  DG_OPT_VISC_FUSED = 7
};
enum { DG_EXCHANGE_TRACES = 0, DG_EXCHANGE_NEIGHBOUR = 1 };
enum { DG_ORDER_LINEAR = 0, DG_ORDER_PENCIL = 1 };
enum { DG_BATCH_PERSISTENT = 0, DG_BATCH_PER_DEGREE = 1 };
/* DG_EINVAL for an unknown key or a value out of range. */
int dg_set_option(dg_ctx* ctx, int key, int value);
/* Current value of an option into *value. */
int dg_get_option(const dg_ctx* ctx, int key, int* value);

/* Bytes of device workspace that the compute calls need (the second state
 * buffer of the neighbour-read exchange, the face-trace ping-pong buffers,
 * reduction partials and the adjoint's two state-sized buffers).  Depends
 * on the mesh and p. */
size_t dg_workspace_bytes(const dg_ctx* ctx);

/* Hand the context a caller-owned device workspace of at least
 * dg_workspace_bytes() bytes, 256-byte aligned.  The caller keeps it alive
 * until the context is destroyed or another workspace is set.
 * DG_EWORKSPACE if too small, DG_EINVAL if NULL or misaligned. */
int dg_set_workspace(dg_ctx* ctx, void* dptr, size_t bytes);

/* Number of solution nodes E*N^3 (the paper's DOF count, Section V);
 * every state array holds 5 times this many doubles.  -1 on NULL ctx. */
int64_t dg_num_dof(const dg_ctx* ctx);

/* Host helper: the N = p+1 point Gauss-Legendre nodes (ascending) and
 * weights on [-1,1] used by the library (Section II-B).  xi and w are HOST
 * arrays of N doubles. */
int dg_quadrature(int p, double* xi, double* w);

/* R = dQ/dt, the right-hand side of Eq. (5) solved for the time derivative:
 * R = M^{-1} (volume term - surface term) per element, with the local
 * Lax-Friedrichs flux lambda = max(|u_n-|+c-, |u_n+|+c+) at every face point.
 * Q (read) and R (written) are device arrays in the layout above. */
int dg_rhs(dg_ctx* ctx, const double* Q, double* R);

/* One LSERK45 stage s (0..4) in place (Sections IV-V):
 *   res <- a_s res + dt R(Q)   (s = 0 overwrites res: a_0 = 0)
 *   Q   <- Q + b_s res
 * with the Carpenter-Kennedy (5,4) 2N-storage coefficients.  Q and res are
 * device arrays in the layout above; res is read only for s > 0. */
int dg_rk_stage(dg_ctx* ctx, int s, double* Q, double* res, double dt);

/* One LSERK45 time step (five stages) in place. */
int dg_rk_step(dg_ctx* ctx, double* Q, double* res, double dt);

/* nsteps >= 0 LSERK45 time steps in place (the paper's benchmark advances a
 * fixed number of steps, Section V).  Bit-identical to nsteps calls of
 * dg_rk_step. */
int dg_rk_steps(dg_ctx* ctx, double* Q, double* res, double dt, int nsteps);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * nsteps LSERK45 steps as dg_rk_steps, bitwise the same result, with the
 * second state buffer of the neighbour-read ping-pong taken from a
 * library-held static device buffer of DG_NOALLOC_MAX_BYTES (128 MiB, one
 * per GPU, held until the process ends) instead of the workspace.  Needs no
 * workspace (none need be set) and calls no allocating routine; the stages
 * always use the neighbour-read exchange (bitwise equal to the trace-buffer
 * one) and are never timed by dg_set_timing.  DG_EUNSUPPORTED if the state
 * (5 E N^3 doubles) exceeds DG_NOALLOC_MAX_BYTES.  Every call on one GPU
 * shares that buffer: calls that overlap on one GPU (other streams, other
 * threads, other contexts) race and must be serialised by the caller.  The
 * buffer holds nothing between calls that a later call relies on. */
#define DG_NOALLOC_MAX_BYTES ((size_t)128 << 20)
int dg_rk_steps_noalloc(dg_ctx* ctx, double* Q, double* res, double dt, int nsteps);

/* As dg_rk_steps (bitwise the same result), with each step's five stage
 * launches captured once in a HIP graph (one per ping-pong parity of the
 * neighbour-read exchange) and replayed nsteps times on an internal stream
 * that is ordered after, and before, the context's stream by events.  The
 * graphs are kept while Q, res, dt and the context's settings stay the
 * same, and rebuilt otherwise.  Launches inside the graphs are not seen by
 * dg_set_timing.  With DG_EXCHANGE_TRACES it runs as dg_rk_steps. */
int dg_rk_graph_steps(dg_ctx* ctx, double* Q, double* res, double dt, int nsteps);

/* Vector-Jacobian product of the right-hand side: gQ = (dR/dQ)^T gR at Q,
 * FP64, overwriting gQ.  At the kinks of max and |.| in the face flux the
 * branch taken by the forward evaluation is differentiated (ties: the -
 * side's wave speed; |x| has derivative +1 at x >= 0).  Q, gR (read) and gQ
 * (written) are device arrays in the layout above; gQ must not alias Q or gR. */
int dg_rhs_vjp(dg_ctx* ctx, const double* Q, const double* gR, double* gQ);

/* Reverse of LSERK45 stage s (0..4) for checkpointed gradients through
 * time stepping.  Qs is the state that stage s started from; on entry gQ and
 * gres hold the adjoints of the stage's outputs (Q, res), on return the
 * adjoints of its inputs:
 *   g = gres + b_s gQ;   gQ <- gQ + dt (dR/dQ at Qs)^T g;   gres <- a_s g
 * (a_0 = 0: the input res of stage 0 has zero adjoint).  Device arrays in the
 * layout above; gQ and gres must not overlap each other or Qs. */
int dg_rk_stage_vjp(dg_ctx* ctx, int s, const double* Qs, double* gQ, double* gres, double dt);

/* Gradient of the integrated kinetic energy (out[5] of dg_integrals) with
 * respect to every nodal value of Q, written to gQ (overwritten):
 * d/d rho = -|u|^2/2 Jw, d/d(rho u_d) = u_d Jw, d/d(rho E) = 0, with Jw the
 * weight J w_i w_j w_k of the node in the collocated Gauss-Legendre rule of
 * Section II-B.  Not in the paper: the adjoint of the objective that the
 * differentiation extension uses (dg_rhs_vjp, dg_rk_stage_vjp).  Q (read) and
 * gQ (written) are device arrays in the layout above; gQ must not overlap Q. */
int dg_kinetic_energy_grad(dg_ctx* ctx, const double* Q, double* gQ);

/* SYNCHRONISING.  Domain integrals by the nodal Gauss-Legendre rule:
 * out[0..4] = integral of the five conserved fields, out[5] = integral of
 * the kinetic energy |rho u|^2/(2 rho).  The conserved integrals are the
 * quantities whose rate of change Eq. (1) states in conservation form (zero
 * on a periodic mesh, as the weak form of Eq. (5) keeps discretely); the
 * rule is the collocated Gauss-Legendre quadrature of Section II-B, exact for
 * the nodal polynomial.  out is a HOST array of 6 doubles.  Summation order
 * is fixed (bitwise reproducible). */
int dg_integrals(dg_ctx* ctx, const double* Q, double out[6]);

/* SYNCHRONISING.  *out = max over nodes of sum_d (|u_d| + c)/h_d, built
 * from the wave speed |u_n| + c of the Lax-Friedrichs flux (Section II-B)
 * with the sound speed c = sqrt(gamma p / rho) of the closure Eq. (3)
 * (units 1/time; a CFL time step is CFL/((2p+1) * *out), a rule the paper
 * does not state).  out is HOST. */
int dg_max_wavespeed(dg_ctx* ctx, const double* Q, double* out);

/* SYNCHRONISING.  DG_OK if every node has finite values, rho > 0 and
 * p > 0 (p from Eq. (3)); DG_ENONPHYSICAL otherwise.  The paper's scheme has
 * no limiter, so the check is opt-in and never part of the hot path. */
int dg_check_state(dg_ctx* ctx, const double* Q);

/* Not in the paper: accuracy check of the reciprocal and square root that
 * the flux kernels use (1/rho at every node and face point, the sound speed
 * sqrt(gamma p / rho) of the Lax-Friedrichs wave speed, Section II-B).  For
 * i < n: r[i] = 1/x[i], s[i] = sqrt(x[i]) computed exactly as inside the
 * kernels.  x, r, s are DEVICE arrays of n doubles that must not overlap;
 * the launch is enqueued on hip_stream (NULL = default stream). */
int dg_recip_sqrt(const double* x, double* r, double* s, int64_t n, void* hip_stream);

/* ---- batched independent meshes ---------------------------------------
 * Not in the paper: an extension of its hot path to many small problems on
 * one GPU (the per-mesh arithmetic is that of Section II-B and Sections
 * IV-V, unchanged).  Many independent periodic meshes of uneven size and degree advanced
 * together: per RK stage one launch per degree present (or one persistent
 * launch, DG_OPT_BATCH_LAUNCH) over a work list of (mesh, element block)
 * items, with a per-degree code path and per-degree elements-per-workgroup
 * tile (dg_batch_set_tile).  The arithmetic on every
 * element is the one of the single-mesh entry points above, so each mesh's
 * result is bitwise that of a single-mesh context on the same state.
 * State layout: one device array holding the meshes back to back; mesh i
 * occupies doubles [dg_batch_offset(b, i), dg_batch_offset(b, i + 1)) in the
 * single-mesh layout [field][ez][ey][ex][k][j][i]. */
typedef struct dg_batch dg_batch;

/* count >= 1 meshes; n[3i..3i+2] = (nx, ny, nz) and p[i] (1..5) of mesh i,
 * L[3i..3i+2] its domain lengths (HOST arrays).  NULL on error. */
dg_batch* dg_batch_create(int count, const int* n, const int* p, const double* L, double gamma);
void dg_batch_destroy(dg_batch* b);
int dg_batch_set_stream(dg_batch* b, void* hip_stream);
/* FP64 (default) or FP32 matrix-core contractions for every mesh. */
int dg_batch_set_precision(dg_batch* b, int mode);
/* Elements per workgroup for degree p (values the library provides: see
 * dg_batch_tile_options); changes the work list, so call it before
 * dg_batch_set_workspace. */
int dg_batch_set_tile(dg_batch* b, int p, int epb);
/* Launch form and the order in which the launches walk the work list; the
 * results are bitwise the same for every setting.  Keys as for
 * dg_set_option:
 * DG_OPT_XCD_REMAP 1: with one launch per degree, each XCD of the MI355X
 *   takes a contiguous part of the degree's items; with the persistent
 *   launch, every degree group of the work list is cut into 8 contiguous
 *   parts of equal node count and XCD x gets part x of each group, so that
 *   every XCD runs the same mix of degrees.  Either way the items that run
 *   at the same time on one XCD are neighbours in the list and share its
 *   L2; 0 (default) leaves the round-robin spread of workgroups.
 * DG_OPT_ORDER: items of a mesh row by row (DG_ORDER_LINEAR) or in
 *   pencils of DG_OPT_PENCIL_X elements (0 = the whole row) by
 *   DG_OPT_PENCIL_Z planes swept along y (DG_ORDER_PENCIL, default, 16 x 8),
 *   which lists an item's y- and z-neighbours close to it.
 * DG_OPT_BATCH_LAUNCH: DG_BATCH_PER_DEGREE (default) runs a stage as one
 *   launch per degree present over that degree's items (one workgroup per
 *   item, each (degree, tile) variant its own kernel and register
 *   allocation; with DG_OPT_XCD_REMAP each XCD takes a contiguous part of
 *   the degree's items); DG_BATCH_PERSISTENT as one persistent launch over
 *   the whole work list with every variant in one kernel (the register
 *   allocation of the largest variant for all).
 * The work list is rebuilt (and re-uploaded, SYNCHRONISING, when a
 * workspace is set); DG_EINVAL for an unknown key or a value out of range. */
int dg_batch_set_option(dg_batch* b, int key, int value);
int dg_batch_get_option(const dg_batch* b, int key, int* value);
/* Up to max tile sizes available for degree p into out[]; returns count. */
int dg_batch_tile_options(int p, int* out, int max);
/* Doubles before mesh i's block (i = count gives the total length). */
int64_t dg_batch_offset(const dg_batch* b, int i);
size_t dg_batch_workspace_bytes(const dg_batch* b);
/* Caller-owned device workspace (256-byte aligned).  SYNCHRONISING: copies
 * the per-mesh tables and the work list into it. */
int dg_batch_set_workspace(dg_batch* b, void* dptr, size_t bytes);
/* Per-mesh time steps dt[count] (HOST).  SYNCHRONISING (copied to the
 * workspace, where the captured graphs read them). */
int dg_batch_set_dt(dg_batch* b, const double* dt);
/* R = dQ/dt of every mesh. */
int dg_batch_rhs(dg_batch* b, const double* Q, double* R);
/* nsteps LSERK45 steps of every mesh with its own dt (per stage the
 * launches of DG_OPT_BATCH_LAUNCH); the state alternates between Q and a
 * workspace buffer (an odd nsteps ends with one device-to-device copy back
 * into Q). */
int dg_batch_rk_steps(dg_batch* b, double* Q, double* res, int nsteps);
/* Same result as dg_batch_rk_steps, with the launches of a step's five
 * stages replayed from HIP graphs (captured on first use for this (Q, res) pair and
 * step parity; recaptured when the pointers change). */
int dg_batch_graph_steps(dg_batch* b, double* Q, double* res, int nsteps);

/* ---- Variable degree per element, optionally refined cells ---------------
 * The hp-adaptive setting that the paper names (Sections I and III: degree
 * and element size adapted element by element) on the periodic Cartesian
 * mesh of nx x ny x nz cells, each cell one element or, refined once, eight
 * elements of half its size.  Every element e has its own degree p_e in
 * 0..7 and the scheme of Section II-B (Eq. (5), collocated Gauss-Legendre
 * basis, local Lax-Friedrichs flux) on it.  A face whose two elements
 * differ in degree or size is integrated on a mortar: the tensor
 * Gauss-Legendre rule of max(p, q) + 1 points per tangential direction on
 * the smaller of the two faces (where a refined cell meets an unrefined
 * one, a fine element's face: a quarter of the coarse face, a hanging
 * face), where both elements' traces are evaluated and the flux is formed
 * once for both sides (conservative; where the two sides match it is the
 * single-degree scheme, bitwise).  Per RK stage one launch for the faces
 * between degrees, one for the hanging faces (each face's flux projected
 * onto both sides), then one launch per (degree, element size) present.
 * Elements are numbered cell by cell, c = (cz ny + cy) nx + cx; a refined
 * cell's children in the order (kz, ky, kx), kx fastest (child (kx, ky, kz)
 * spans [cx + kx/2, cx + (kx+1)/2] h_x, ...).
 * State layout: Q[f * T + off[e] + (k N_e + j) N_e + i], field f = rho, rho u,
 * rho v, rho w, rho E, T = dg_varp_num_dof, off[e] = dg_varp_offset(v, e):
 * the elements' [N_e]^3 blocks back to back in element order, the node
 * index i fastest.  Arrays are device pointers, FP64, 8-byte aligned; Q
 * must not overlap R or res (DG_EALIAS). */
typedef struct dg_varp dg_varp;

/* No refinement: E = nx ny nz elements, e = (ez ny + ey) nx + ex.
 * nx, ny, nz >= 1; degrees[E] (HOST, element order as above) each in 0..7
 * (DG_EUNSUPPORTED otherwise); L[3] (HOST) the domain lengths.  NULL on
 * error (dg_last_error). */
dg_varp* dg_varp_create(int nx, int ny, int nz, const int* degrees, const double* L, double gamma);
/* refine[nx ny nz] (HOST, cell order) each 0 or 1 (DG_EINVAL otherwise):
 * E = nx ny nz + 7 (number of refined cells) elements; degrees[E] (HOST,
 * element order) each in 0..7; at most 2^31-1 elements, and where any
 * cell is refined at most 2^31-1 cells of the twice finer mesh
 * (DG_EUNSUPPORTED).  NULL on error. */
dg_varp* dg_varp_create_refined(int nx, int ny, int nz, const int* refine, const int* degrees, const double* L,
                                double gamma);
void dg_varp_destroy(dg_varp* v);
int dg_varp_set_stream(dg_varp* v, void* hip_stream);
/* Total nodes T (the DOF count), -1 for NULL. */
int64_t dg_varp_num_dof(const dg_varp* v);
/* Number of elements E, -1 for NULL. */
int64_t dg_varp_num_elements(const dg_varp* v);
/* First node of element e (e = E gives T); -1 out of range. */
int64_t dg_varp_offset(const dg_varp* v, int64_t e);
size_t dg_varp_workspace_bytes(const dg_varp* v);
/* Caller-owned device workspace (256-byte aligned): mortar tables, face
 * table, offsets, element lists, the face-flux buffer, the face-trace buffer
 * (the elements' traces on those faces, which each stage of
 * dg_varp_rk_steps writes for the next) and the second state buffer of the
 * ping-pong.  Calls on one context share it: they must not overlap.
 * SYNCHRONISING (uploads the tables). */
int dg_varp_set_workspace(dg_varp* v, void* dptr, size_t bytes);
/* R = dQ/dt. */
int dg_varp_rhs(dg_varp* v, const double* Q, double* R);
/* nsteps LSERK45 steps (Sections IV-V) of size dt; res is the 2N register
 * (its input is ignored: the first stage does not read it).  The state
 * alternates between Q and a workspace buffer; an odd nsteps ends with one
 * device-to-device copy back into Q. */
int dg_varp_rk_steps(dg_varp* v, double* Q, double* res, double dt, int nsteps);
/* Not in the paper: measurement support.  While on, every launch is
 * bracketed by HIP events (switching on clears the record). */
int dg_varp_set_timing(dg_varp* v, int on);
/* Slots of dg_varp_timing_read. */
#define DG_VARP_TIMING_SLOTS 26
/* SYNCHRONISING.  ms[3 p + mode], count[3 p + mode] (HOST arrays of
 * DG_VARP_TIMING_SLOTS): summed milliseconds and launches of degree p's
 * kernel (both element sizes), mode 0 right-hand side, 1 RK stages 2..5,
 * 2 the first RK stage; ms[24], count[24] the kernel of the faces between
 * degrees, ms[25], count[25] the hanging-face kernel.  Clears the record. */
int dg_varp_timing_read(dg_varp* v, double* ms, int64_t* count);

/* Not in the paper: measurement support.  Opt-in per-launch timing for
 * benchmarks.  While on, the context brackets
 * every kernel it launches with HIP events on its stream (a few microseconds
 * of overhead per launch).  Kinds: 0 face-trace kernel, 1 RK stage kernel of
 * stages 2..5, 2 RHS kernel (also the inviscid rate of a viscous stage),
 * 3 adjoint kernels, 4 reductions, 5 RK stage kernel of the first stage
 * (whose coefficient a is zero, so it writes the residual without reading
 * it), 6 the two viscous kernels of a right-hand side or stage (timed
 * together).  Switching on clears the record; at most 65536 launches are
 * recorded. */
int dg_set_timing(dg_ctx* ctx, int on);

/* SYNCHRONISING.  Summed milliseconds ms[k] and launch counts count[k] for
 * the seven kinds above since timing was switched on.  HOST arrays of 7. */
int dg_timing_read(dg_ctx* ctx, double ms[7], int64_t count[7]);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
