/*
 * lmfr.h -- C ABI of the MI355X (gfx950) implementation of the implicit
 * Weiss-Smith-preconditioned flux reconstruction (FR/CPR) method for low-Mach
 * compressible Navier-Stokes flow on static or deforming quadrilateral meshes
 * (Wang & Yu, arXiv:1903.06304).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Unknowns are the primitive variables q^p = (p, u, v, T) (paper Sec. 2.2) at
 *    (p+1)^2 Gauss-Legendre solution points per quadrilateral element.
 *  - State-sized arrays are DEVICE pointers owned by the caller, FP64, layout
 *    [4][n_elem][Np], var-major, Np = (order+1)^2, solution point (i, j) at index
 *    i + (order+1)*j, i along xi.  Residual rows are the conservation equations
 *    (mass, x-momentum, y-momentum, energy) in the units of dq^c/dt.
 *  - Element faces: 0 (xi=-1), 1 (xi=+1), 2 (eta=-1), 3 (eta=+1).  Face point k
 *    runs along the face (eta index on faces 0/1, xi index on faces 2/3).
 *  - Geometry: isoparametric Gauss-Lobatto nodes of degree geom_order, node (a, b)
 *    at a + (geom_order+1)*b, arrays [2][n_elem][(geom_order+1)^2] (x then y).
 *  - `stream` is a hipStream_t (NULL = the default stream).  All calls are
 *    asynchronous on it unless stated otherwise.
 *  - No exceptions cross the ABI: every call returns an fr_status; the text of
 *    the last failure on the calling thread is returned by fr_last_error().
 *  - Memory: a context allocates its tables and the residual / JVP / VJP workspaces in
 *    fr_create.  fr_reserve (fr_batch_reserve for a batch) allocates everything the
 *    factor, apply, step and steady-solve paths use, for Krylov dimensions up to a stated
 *    maximum and an inverse stored at up to a stated precision; after it those calls
 *    allocate no device memory (a step that captures its GMRES cycle still builds the
 *    graph on its first call, in the runtime's own memory).  Without fr_reserve the first
 *    factor allocates the blocks and the inverse at its precision, and the first step with
 *    a larger Krylov dimension its workspace; residual, JVP, VJP and apply never allocate.
 */
#ifndef LMFR_H
#define LMFR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fr_ctx_s* fr_ctx;
typedef struct fr_batch_s* fr_batch;

typedef enum {
    FR_OK = 0,
    FR_EINVAL = -1,        /* invalid argument (null pointer, size, range) */
    FR_EHIP = -2,          /* HIP runtime error (text in fr_last_error) */
    FR_ENOMEM = -3,        /* device allocation failed */
    FR_ENONFINITE = -4,    /* NaN/Inf met in a residual or Krylov norm */
    FR_ENOCONV = -5,       /* Newton or GMRES did not reach its tolerance */
    FR_EUNSUPPORTED = -6   /* order or geometry outside what is built */
} fr_status;

typedef enum { FR_FP64 = 0, FR_FP32 = 1, FR_BF16 = 2 } fr_prec;

/* Boundary faces (paper Sec. "Boundary Conditions"): a negative h_nbr entry in
 * fr_create marks a face on the domain boundary and names its condition.  The state
 * beyond the face, formed from the own trace, enters the same common flux (preconditioned
 * Rusanov + BR2) as an interior neighbour's trace:
 *   FR_BC_FARFIELD      the free stream q^inf of fr_set_farfield, uniform (zero gradient);
 *   FR_BC_SLIP_WALL     the mirror image across the wall, velocity relative to the face's
 *                       grid velocity (a symmetry plane: gradients mirrored too);
 *   FR_BC_NOSLIP_WALL   adiabatic no-slip wall moving with the grid: velocity
 *                       2 v_g - v, same p and T, same velocity gradient, temperature
 *                       gradient mirrored (no heat flux through the wall).
 * The BR2 lifting beyond a boundary face uses the own |J|. */
typedef enum { FR_BC_FARFIELD = -1, FR_BC_SLIP_WALL = -2, FR_BC_NOSLIP_WALL = -3 } fr_bc;

/* Physical and discretisation parameters (paper Sec. 2.1 non-dimensionalisation:
 * R = 1/(gamma mach_ref^2), Cp = 1/((gamma-1) mach_ref^2), k = mu Cp / prandtl;
 * Sec. 2.2 Eq. (eps_nonmove)/(eps_move): eps = min(1, max(kappa mach_inf, Ma))). */
typedef struct {
    int32_t order;        /* solution degree p, 1..4 */
    int32_t geom_order;   /* degree of the geometry nodes, 1..4 */
    int32_t n_elem;
    int32_t viscous;      /* 0: Euler, 1: Navier-Stokes (BR2 viscous fluxes) */
    int32_t moving;       /* 1: grid velocities present (deforming / moving mesh) */
    double gamma, mach_ref, reynolds, prandtl, mu, kappa, mach_inf;
} fr_params;

/* Options of one BDF2 dual-time step (paper Sec. 3.2, Eq. unsteady_pre_discretized_3). */
typedef struct {
    double dt;            /* physical time step */
    double inv_dtau;      /* 1/dtau of the pseudo-time term (paper: dtau = 1e20) */
    double tol_pseudo;    /* stop when Res_m / Res_0 <= tol_pseudo (mass-row 2-norm) */
    double tol_res;       /* GMRES relative tolerance ||b - A x|| <= tol_res ||b|| */
    double tol_abs;       /* also stop when Res_m <= tol_abs (round-off floor) */
    int32_t krylov;       /* restart length m, 1..156 */
    int32_t max_lin_it;   /* GMRES iteration cap per Newton step */
    int32_t max_newton;   /* Newton (pseudo-time) iteration cap */
    int32_t jac_lag;      /* refresh the block-Jacobi blocks when m % jac_lag == 0 */
    int32_t prec;         /* fr_prec of the stored preconditioner blocks */
} fr_step_opts;

typedef struct {
    int32_t newton_its, gmres_its, converged;
    double res0, res_final;
} fr_step_stats;

/* Options of a steady solve by pseudo-transient continuation (paper Sec. 3.2,
 * Eq. steady_pre_discretized_1, with the pseudo-time step of Eq. SER).  The paper's
 * defaults: dtau0 = dtau_min = 0.01, dtau_max = 1e20, r_ser = 2. */
typedef struct {
    double dtau0;         /* pseudo-time step of the first iteration */
    double dtau_min, dtau_max;   /* SER bounds of the pseudo-time step */
    double r_ser;         /* SER exponent: dtau_m = dtau_{m-1} (Res_{m-1}/Res_m)^r_ser, clipped */
    double tol_pseudo;    /* stop when Res_m / Res_0 <= tol_pseudo (continuity-row 2-norm of R) */
    double tol_res;       /* GMRES relative tolerance of each linear solve */
    double tol_abs;       /* also stop when Res_m <= tol_abs (round-off floor) */
    int32_t krylov;       /* restart length m, 1..156 (paper: 150 for steady problems) */
    int32_t max_lin_it;   /* GMRES iteration cap per pseudo-time step */
    int32_t max_steps;    /* pseudo-time step cap */
    int32_t jac_lag;      /* refresh the block-Jacobi blocks when m % jac_lag == 0 (paper: 1) */
    int32_t prec;         /* fr_prec of the stored preconditioner blocks */
    double reject_growth; /* step rejection, not part of the paper's method (0 = off, the paper's
                             SER): a step after which Res is not finite or exceeds reject_growth
                             times the Res before it is undone and retried from the same state
                             with dtau / 10 (no SER update, no clipping, for that retry); undone
                             steps count towards max_steps */
} fr_steady_opts;

typedef struct {
    int32_t steps, gmres_its, converged;
    double res0, res_final;
    double dtau_final;    /* pseudo-time step of the last step taken */
    int32_t rejected;     /* steps undone by step rejection */
} fr_steady_stats;

/* Create a context for one mesh.  h_nbr/h_nbr_face/h_flip are HOST arrays [n_elem][4]:
 * neighbour element, neighbour's local face and point-order reversal (NULL = none)
 * across each face.  An interior face must be listed from both sides; a boundary face
 * has an fr_bc code in h_nbr (its h_nbr_face and h_flip entries are ignored).  A mesh
 * with far-field faces needs fr_set_farfield before any evaluation.
 * Returns FR_EUNSUPPORTED for order or geom_order outside 1..4, FR_EINVAL for a
 * table that is out of range or not symmetric, and for meshes past the size limits of
 * the kernels' 32-bit offsets: n_elem < 2^27, 4 n_elem (p+1)^2 < 2^31 state entries and
 * 8 n_elem max((p+1)^2, 4(p+1)) < 2^32 bytes per solution- or flux-point field. */
fr_status fr_create(const fr_params* prm, const int32_t* h_nbr, const int32_t* h_nbr_face,
                    const int8_t* h_flip, fr_ctx* out);

/* Free-stream primitive state (p, u, v, T) beyond the far-field faces (paper Sec.
 * "Boundary Conditions": q^{p,b} = q^{p,inf}).  h_qinf: HOST array [4].  Synchronous
 * (a blocking copy): call it while no work of this context is in flight.  Every solver
 * that holds the context (its own, batches) sees the new state.  FR_EINVAL for a
 * non-finite entry or p, T <= 0. */
fr_status fr_set_farfield(fr_ctx ctx, const double* h_qinf);

/* Geometry of the mesh at the time level where the residual is evaluated (paper
 * Sec. 2.3, metrics of the map x(xi, eta, t) and grid velocity v_g = dx/dt):
 * xg, vg are DEVICE arrays [2][n_elem][(geom_order+1)^2]; vg NULL for static meshes
 * (required when the context was created with moving = 1).  Computes and keeps the
 * metric terms at solution and flux points; the face vector of each interface is
 * computed once, from its owner side, and shared by both sides.  Also flags the affine
 * elements (constant metrics); reading the flags back synchronises `stream`. */
fr_status fr_set_geometry(fr_ctx ctx, const double* xg, const double* vg, void* stream);

/* Number of elements the last fr_set_geometry found affine: every metric term constant
 * over the element to 1e-10 of its scale, and no boundary face.  Where the neighbour across a face is affine,
 * the kernels form its gradient trace from its state traces (the chain rule applied to
 * the traced reference derivatives, the same values to rounding) instead of tracing its
 * pointwise gradient.  *n_affine is HOST; synchronises `stream`. */
fr_status fr_affine_elements(fr_ctx ctx, int32_t* n_affine, void* stream);

/* R(q): the FR/CPR residual of paper Eq. (cpr_ns) with the moving-mesh terms of
 * Eq. (unsteady_pre_mov_pdomain), preconditioned Rusanov common flux (Eq. Rosanov),
 * BR2 common gradient and Radau correction functions.  q, R: [4][E][Np]. */
fr_status fr_residual(fr_ctx ctx, const double* q, double* R, void* stream);

/* Exact Jacobian-vector product Jv = (dR/dq^p) v (forward tangent of the residual);
 * R_or_null receives R(q) when non-NULL.  All arrays [4][E][Np]. */
fr_status fr_jvp(fr_ctx ctx, const double* q, const double* v, double* Jv, double* R_or_null,
                 void* stream);

/* Vector-Jacobian product JTw = (dR/dq^p)^T w (reverse / adjoint of the residual),
 * gather-formulated and deterministic.  All arrays [4][E][Np]. */
fr_status fr_vjp(fr_ctx ctx, const double* q, const double* w, double* JTw, void* stream);

/* fr_vjp for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): the same kernels and results, bit for
 * bit, with the two side buffers of the adjoint (face traces and face adjoints,
 * E * 4 * 10 * (order+1) doubles each) in a 32 MiB array that the library holds on each
 * device for the life of the process, instead of context memory.  Meshes above that
 * (E * (order+1) > 52428) get FR_EINVAL.  Calls that overlap on one device share the
 * array and race; the current device must be the context's.  Allocates nothing. */
fr_status fr_vjp_noalloc(fr_ctx ctx, const double* q, const double* w, double* JTw, void* stream);

/* Operator of the BDF2 Newton system, paper Eq. (unsteady_pre_discretized_3):
 * Av = inv_dtau Gamma v + c_time M v - (dR/dq) v, pointwise Gamma and M at q. */
fr_status fr_bdf_operator(fr_ctx ctx, const double* q, const double* v, double c_time,
                          double inv_dtau, double* Av, void* stream);

/* Element-block-Jacobi preconditioner (paper Sec. 4, parallel set-up: block Jacobi over
 * the element blocks): P_e = inv_dtau Gamma_e + c_time M_e - dR_e/dq_e,
 * the true diagonal block of the Newton operator (own-state dependence through the
 * faces included), assembled on the device in FP64, inverted by Gauss-Jordan elimination
 * with partial pivoting and stored as an explicit inverse in precision `prec`.  The apply
 * reads the stored inverse and accumulates in FP64.
 * c_time = 3/(2 dt) for BDF2, 1/dt for BDF1.  Kept in the context for the apply. */
fr_status fr_block_jacobi_factor(fr_ctx ctx, const double* q, double c_time, double inv_dtau,
                                 int32_t prec, void* stream);

/* z = P^-1 r with the last factored blocks; r, z [4][E][Np] (may not alias).  With the
 * option "preconditioner" = 1 (2), P is the symmetric (forward) block Gauss-Seidel
 * preconditioner of the operator the last fr_block_jacobi_factor linearised (its q, c_time and inv_dtau; a later
 * fr_bdf_operator with "operator_packs" replaces that linearisation). */
fr_status fr_block_jacobi_apply(fr_ctx ctx, const double* r, double* z, void* stream);

/* Copy the stored inverse of the last fr_block_jacobi_factor, widened exactly to FP64, to
 * the DEVICE array inv [E][4Np][4Np], row-major (row = v*Np + s), so that z_e = inv_e r_e
 * is what fr_block_jacobi_apply computes with block Jacobi.  Element order always (a factor
 * under the Gauss-Seidel option stores the blocks in colour order internally; the values
 * are the same).  FR_EINVAL before a factor. */
fr_status fr_get_inverse(fr_ctx ctx, double* inv, void* stream);

/* Allocate now every device workspace of fr_block_jacobi_factor, fr_block_jacobi_apply,
 * fr_bdf_operator, fr_bdf2_step and fr_steady_solve for Krylov dimensions up to krylov_max
 * (1..156) and an inverse stored at up to the width of `prec` (FR_FP64 covers every
 * precision): those calls then allocate no device memory, which keeps them usable where
 * allocation is not allowed.  FR_EINVAL for arguments out of range, FR_ENOMEM. */
fr_status fr_reserve(fr_ctx ctx, int32_t krylov_max, int32_t prec);

/* Copy the assembled (unfactored) FP64 blocks of the last fr_block_jacobi_factor to
 * the DEVICE array blk [E][4Np][4Np], row-major (row = v*Np + s).  Only available
 * when the context keeps them (fr_block_jacobi_factor with keep = 1 via fr_set_option). */
fr_status fr_get_blocks(fr_ctx ctx, double* blk, void* stream);

/* One BDF2 dual-time Newton step (BDF1 when q_nm1 is NULL): q holds q^n on entry and
 * q^{n+1} on return.  Newton starts from q^n (paper Sec. 3.2); each Newton step solves
 * the Eq. (unsteady_pre_discretized_3) system with restarted, right-preconditioned
 * FP64 GMRES and the element-block-Jacobi preconditioner (refreshed every jac_lag steps).
 * Synchronises once per GMRES restart cycle and Newton step.  h_stats: HOST,
 * may be NULL.  Returns FR_ENOCONV (state still updated) when max_newton is reached. */
fr_status fr_bdf2_step(fr_ctx ctx, double* q, const double* q_nm1, const fr_step_opts* opts,
                       fr_step_stats* h_stats, void* stream);

/* Steady solve by pseudo-transient continuation (paper Sec. 3.2): from q (DEVICE
 * [4][E][Np], updated in place), repeat (Gamma^m/dtau_m - dR/dq^m) dq = R^m, q += dq,
 * with dtau_m from the SER rule (Eq. SER; dtau0 at m = 0, then the previous step times
 * (Res_{m-1}/Res_m)^r_ser, clipped to [dtau_min, dtau_max]), until Res_m/Res_0 <=
 * tol_pseudo or Res_m <= tol_abs.  Each linear system is solved by the same restarted
 * right-preconditioned FP64 GMRES and element-block-Jacobi preconditioner as the BDF2
 * step.  Synchronises once per GMRES restart cycle and pseudo-time step.  h_stats: HOST,
 * may be NULL.  Returns FR_ENOCONV (state still updated) when max_steps is reached. */
fr_status fr_steady_solve(fr_ctx ctx, double* q, const fr_steady_opts* opts, fr_steady_stats* h_stats,
                          void* stream);

/* Options: "keep_blocks" (0/1: keep the FP64 blocks for fr_get_blocks), "graph" (0/1:
 * replay each GMRES restart cycle from a captured hipGraph, default 1), "gram_schmidt"
 * (1: classical Gram-Schmidt, one orthogonalisation pass per Arnoldi step, the default;
 * 2: with one re-orthogonalisation pass), "fused_gram_schmidt" (0/1, default 1: with two
 * passes, the first pass's update and the second pass's dot products share one read of
 * the basis, up to 32 basis vectors; same results bit for bit), "operator_packs" (0/1: fr_bdf_operator first
 * stores the values its nonlinear point functions need at q, then applies the operator
 * on tangents only -- the form the BDF2 step uses inside GMRES; fr_block_jacobi_factor
 * assembles its block columns the same way; same results to rounding), "preconditioner"
 * (0: element-block Jacobi, the default; 1: symmetric block Gauss-Seidel over the
 * elements in colour order, P = (D + L) D^-1 (D + U) with D the element blocks and L / U
 * the couplings of the Newton operator to elements of lower / higher colour -- colours
 * from fr_create, the smallest colour no face neighbour has, in element order; each
 * application costs 2 (K - 1) operator passes for K colours, each over the elements of
 * one colour (on even periodic meshes two passes over half the elements each), and
 * 2 - 1/K block applies; 2: forward block Gauss-Seidel in the same colour order, P = D + L,
 * the forward half of that sweep: K - 1 operator passes over one colour each and one
 * block apply; used by fr_block_jacobi_apply and the GMRES of the BDF2 and steady solves),
 * and a manual launch shape of the fused kernels (what fr_autotune chooses): "tile_lanes" (0 =
 * default, 64, 128, 256; dual-number modes cap it at 128), "tile_grid" (0 = one
 * workgroup per tile, else the persistent grid size), "tile_xcd" (1 = each XCD walks a
 * contiguous eighth of the tiles, 0 = round robin). */
fr_status fr_set_option(fr_ctx ctx, const char* name, int64_t value);

/* Choose the launch shape (workgroup width: elements per workgroup, persistent grid
 * size, tile order across XCDs) of the residual, JVP and Newton-operator kernels by timing the candidates on the
 * device with a free-stream state; block-column assembly takes the Newton operator's
 * shape.  cache_path (may be NULL): text file of earlier choices keyed by GPU
 * architecture, order, viscous/moving flags, mode and element-count bucket; entries
 * found there are used without timing, new ones are appended.  Synchronises `stream`.
 * The choice affects speed only: every shape computes the same values bit for bit. */
fr_status fr_autotune(fr_ctx ctx, const char* cache_path, void* stream);

/* ---------------------------------------------------------------------------------
 * Batches: many independent cases (meshes of different sizes and orders, different
 * Mach and Reynolds numbers, static or deforming) advanced together.  Every launch of
 * the hot path covers all cases: cases of one (order, viscous, moving) kind share one
 * persistent launch of the fused residual kernel over a ragged tile list, and the
 * Krylov kernels reduce per case over one concatenated vector.  Each case keeps its
 * own Newton and GMRES convergence through per-case flags on the device; each GMRES
 * restart cycle of the whole batch is one captured hipGraph replay. */

/* Create a batch over n contexts (each created and given its geometry as usual; the
 * batch does not own them and they must outlive it).  A context may appear once. */
fr_status fr_batch_create(const fr_ctx* ctxs, int32_t n, fr_batch* out);
void fr_batch_destroy(fr_batch batch);

/* Layout of the batch's concatenated state vectors: *n_total entries; case c's
 * [4][E_c][Np_c] array starts at offsets[c] (HOST array [n], may be NULL); the gaps
 * between cases are padding the kernels neither read into results nor write. */
fr_status fr_batch_layout(fr_batch batch, int64_t* n_total, int64_t* offsets);

/* Residual / JVP of every case on concatenated DEVICE arrays laid out as reported by
 * fr_batch_layout (q, v in; R, Jv out; padding of the outputs is left untouched). */
fr_status fr_batch_residual(fr_batch batch, const double* q, double* R, void* stream);
fr_status fr_batch_jvp(fr_batch batch, const double* q, const double* v, double* Jv, void* stream);

/* One BDF2 (BDF1 where q_nm1[c] is NULL or q_nm1 itself is NULL) dual-time step of
 * every case: q[c] (DEVICE, [4][E_c][Np_c]) holds q^n on entry and q^{n+1} on return.
 * opts[c]: per-case dt, inv_dtau and tolerances; krylov, max_lin_it, max_newton,
 * jac_lag and prec must agree across the batch.  h_stats: HOST [n] or NULL.  Cases
 * that converge leave the iteration while the others continue.  Synchronises once per
 * GMRES restart cycle and Newton iteration.  Returns FR_ENONFINITE or FR_ENOCONV when
 * a case failed (fr_last_error names the first); the other cases are still advanced. */
fr_status fr_batch_bdf2_step(fr_batch batch, double* const* q, const double* const* q_nm1,
                             const fr_step_opts* opts, fr_step_stats* h_stats, void* stream);

/* Steady solve of every case (paper Sec. 3.2, as fr_steady_solve): q[c] DEVICE
 * [4][E_c][Np_c], updated in place; opts[c] per-case pseudo-time steps and tolerances;
 * krylov, max_lin_it, max_steps, jac_lag and prec must agree across the batch.  Each case
 * keeps its own SER step and convergence.  h_stats: HOST [n] or NULL. */
fr_status fr_batch_steady_solve(fr_batch batch, double* const* q, const fr_steady_opts* opts,
                                fr_steady_stats* h_stats, void* stream);

/* fr_reserve for a batch: every workspace of its step and steady-solve paths. */
fr_status fr_batch_reserve(fr_batch batch, int32_t krylov_max, int32_t prec);

/* Options: "graph", "gram_schmidt", "preconditioner" and the "tile_*" launch-shape
 * options, as for a context. */
fr_status fr_batch_set_option(fr_batch batch, const char* name, int64_t value);

/* fr_autotune for every launch group of the batch. */
fr_status fr_batch_autotune(fr_batch batch, const char* cache_path, void* stream);

const char* fr_last_error(void);
void fr_destroy(fr_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* LMFR_H */
