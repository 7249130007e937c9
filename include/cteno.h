/*
 * cteno.h -- C ABI of the MI355X (gfx950) CTENO / CTENOZ finite-volume
 * library for the 2-D Euler equations and scalar advection on unstructured
 * triangular meshes.
 *
 * Method: Ma, Chong, Feng, Zhang, Wang, Zhou, "High-order finite-volume
 * central targeted ENO family scheme for compressible flows in unstructured
 * meshes" (arXiv 2312.17042).  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point:
 *   - every call returns a cteno_status; on failure the outputs and handles
 *     are left unchanged and cteno_last_error() returns a message that stays
 *     valid until the next failing call on the same thread;
 *   - "host" pointers are read or written during the call only (inputs are
 *     copied); "device" pointers are HIP device allocations owned by the
 *     caller (for example torch tensors) and are accessed on the context's
 *     stream, asynchronously, in stream order;
 *   - arrays use the caller's cell order (the order of the triangles passed
 *     to cteno_mesh_upload); the library may reorder cells internally;
 *   - cell states are cell averages of the conserved variables, laid out
 *     variable-major [nv][n_cells] in double precision: nv = 1 for scalar
 *     advection, nv = 4 (rho, rho u, rho v, E) for the Euler equations;
 *   - asynchronous device failures (non-physical states, faults) are
 *     reported by the next synchronising call (cteno_sol_download,
 *     cteno_solve, cteno_ctx_synchronize).
 */
#ifndef CTENO_H
#define CTENO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CTENO_OK = 0,
    CTENO_ERR_INVALID = 1,      /* bad argument or call sequence */
    CTENO_ERR_MESH = 2,         /* malformed mesh (degenerate cell, unmatched periodic seam, ...) */
    CTENO_ERR_STENCIL = 3,      /* stencil cannot be built (mesh too small) or rank-deficient LS */
    CTENO_ERR_NOMEM = 4,        /* device or host allocation failed */
    CTENO_ERR_DEVICE = 5,       /* HIP runtime error */
    CTENO_ERR_NONPHYSICAL = 6,  /* density or pressure <= 0 / NaN met in a face state */
    CTENO_ERR_BUSY = 7          /* resource budget exhausted; retry later */
} cteno_status;

/* Boundary kinds per box side.  The outside state of a boundary face at a
   Gauss point is: WALL, the inside state with its normal momentum reversed
   (the HLLC flux against it is evaluated in closed form with its zero
   contact speed, (0, p* n, 0): no mass or energy crosses a wall);
   TRANSMISSIVE, the inside state (fit for outflow, not for a supersonic
   inflow, where it lets a boundary mode grow); INFLOW, a prescribed state
   (cteno_mesh_desc.behind / ahead).  The paper names its test cases'
   boundaries only in words (sec. 3); these are the usual ghost states. */
enum { CTENO_PERIODIC = 0, CTENO_WALL = 1, CTENO_TRANSMISSIVE = 2, CTENO_INFLOW = 3 };
/* physics */
enum { CTENO_ADVECTION = 0, CTENO_EULER = 1 };
/* weighting scheme: CTENO = Algorithm 1 (sec. 2.5), CTENOZ = Algorithm 2 (sec. 2.6) */
/* Reconstructed variables: conserved variables component-wise, or per face
   the characteristic fields W = L_f U of the Euler flux Jacobian along the
   face normal at the cell's average state (sec. 2.2 recommends them for
   strong shocks; the paper uses them for Sod).  With characteristic
   variables the selection bytes are per face and field: [n_cells][3][nv]. */
enum { CTENO_VARS_CONSERVED = 0, CTENO_VARS_CHARACTERISTIC = 1 };

/* CTENO: Algorithm 1; CTENOZ: Algorithm 2; CWENO and TENO: the paper's
   comparison schemes (sec. 2.3-2.4) in the same pipeline */
enum { CTENO_SCHEME_CTENO = 0, CTENO_SCHEME_CTENOZ = 1, CTENO_SCHEME_CWENO = 2, CTENO_SCHEME_TENO = 3 };
/* Scale-separation form (gamma_s of the selection).  PAPER: as printed --
   CTENO gamma_s = 1/(SI_s+eps)^6 (Algorithm 1), CTENOZ gamma_s =
   1 + tau/(SI_s+eps) with tau = (mean_s |SI_s - SI_1|)^6 (Algorithm 2).
   LAMBDA (CTENO only): gamma_s = lambda_s/(SI_s+eps)^6, the linear weights
   of eq. e18 included.  SCALED (CTENOZ only): gamma_s = 1 + tau/(SI_s+eps)^6,
   the sixth power that Algorithm 1 puts on the denominator, which makes the
   selection independent of the scale of the indicators (the printed form is
   not: tau grows like SI^6, the denominator like SI). */
enum { CTENO_GAMMA_PAPER = 0, CTENO_GAMMA_LAMBDA = 1, CTENO_GAMMA_SCALED = 2 };
/* arithmetic of the reconstruction, weights and fluxes.  The cell-average
   state, the residual accumulation and the Runge-Kutta update are always
   FP64; MIXED runs reconstruction, smoothness indicators, weights and HLLC
   in FP32.  Bit mask of the pseudo-inverse copies kept on the device. */
enum { CTENO_FP64 = 1, CTENO_MIXED = 2, CTENO_BOTH = 3 };

typedef void *(*cteno_alloc_fn)(size_t bytes, void *user);
typedef void (*cteno_free_fn)(void *ptr, void *user);

typedef struct cteno_ctx cteno_ctx;
typedef struct cteno_mesh cteno_mesh;
typedef struct cteno_sol cteno_sol;
typedef struct cteno_server cteno_server;

/* Triangular mesh (sec. 2: cells V_i with faces A_ij).  Vertices are raw
   coordinates; each triangle's own three vertices must form the cell as it
   lies in the plane (no wrap-around triangles).  On a periodic pair of box
   sides, vertices on the two sides are welded where their other coordinate
   matches (tolerance 1e-9 of the box size), so seam vertices may be
   duplicated.  Triangles may have either orientation; each is normalised to
   counter-clockwise by swapping its 2nd and 3rd vertex. */
typedef struct {
    int32_t n_vertices;
    const double *xy;      /* host [n_vertices][2] */
    int32_t n_cells;
    const int32_t *tri;    /* host [n_cells][3] */
    double box[4];         /* x0, x1, y0, y1 */
    int32_t bc[4];         /* kinds of the sides x = x0, x = x1, y = y0, y = y1 */
    /* Prescribed outside states of INFLOW faces (conserved variables; entry 0
       alone for advection): `behind` at Gauss points (x, y) with
       x < line[0] + line[1] y + line[2] t at the stage time t, `ahead`
       elsewhere -- a straight discontinuity moving in x, such as the incident
       shock of the double Mach reflection (sec. 3.3); a constant inflow sets
       behind = ahead.  Both must be physical (density, pressure > 0) when a
       side is INFLOW. */
    double behind[4], ahead[4];
    double line[3];
    /* Optional switch of kind along a side: faces of side k whose midpoint
       lies below split_at[k] along the side (y on the sides x = const, x on
       the sides y = const) take kind split_kind[k] instead of bc[k];
       split_kind[k] = 0 means no switch (periodic sides cannot switch). */
    int32_t split_kind[4];
    double split_at[4];
} cteno_mesh_desc;

/* Scheme parameters (sec. 2.1-2.7).  degree r in 2..6: the central
   polynomial of degree r gives order r+1 and uses M = 2K neighbours,
   K = (r+1)(r+2)/2 - 1; directional polynomials have degree r_d = 1 up to
   r = 3 and ceil(r/2) above (K_d basis functions, M_d = 2 K_d cells);
   N_q = ceil((r+1)/2) Gauss-Legendre points per face.
   lambda1_prime: eq. e18; c_t: cut-off of eq. e23 (paper: 1e-6); eps: the
   regulariser of the smoothness indicators (not given by the paper; 1e-12
   recommended).
   positivity (Euler only): 0 (the paper's scheme, which has no positivity
   treatment) -- a non-physical face state (density or pressure <= 0, or
   NaN) is reported as CTENO_ERR_NONPHYSICAL; 1 -- an optional fallback the
   paper does not describe: a cell whose reconstructed density or pressure
   is <= 0 at any Gauss point uses its cell average at all of them, flagged
   by bit 7 of its selection bytes and counted (cteno_sol_fallbacks,
   cteno_request_info.fallbacks). */
typedef struct {
    int32_t physics;
    double ax, ay;          /* advection velocity (ADVECTION) */
    double gamma;           /* ratio of specific heats (EULER) */
    int32_t scheme;
    int32_t degree;
    double lambda1_prime;
    double c_t;
    double eps;
    int32_t gamma_form;
    int32_t precision;      /* CTENO_FP64 | CTENO_MIXED | CTENO_BOTH */
    int32_t reorder;        /* 1: Morton-order cells internally for locality; 0: keep order */
    int32_t variables;      /* CTENO_VARS_CONSERVED | CTENO_VARS_CHARACTERISTIC (Euler only) */
    int32_t positivity;     /* 0: report non-physical states (default); 1: cell-average fallback */
} cteno_scheme;

typedef struct {
    int64_t n_cells, n_faces, n_boundary_faces;
    int32_t K, M, slots, nv, nq;
    int32_t n_inadmissible;     /* interior faces whose directional stencil has < K_d + 1 cells */
    int32_t Kd, Md;             /* directional basis size and stencil size (M_d = 2 K_d) */
    int64_t device_bytes;       /* resident device memory of the mesh handle */
    int64_t n_cross_cells;      /* cells with a face to another 256-cell block (the fused
                                   stage's second kernel finishes them); 0 above degree 3 */
} cteno_mesh_info;

/* ---------------------------------------------------------------------- */
/* context                                                                 */
/* ---------------------------------------------------------------------- */

/* Creates a context on HIP device `device`, issuing all work on `stream`
   (a hipStream_t; NULL = a non-blocking stream owned by the context).  alloc/free (both or neither)
   route every device allocation through the caller, e.g. a framework's
   caching allocator; NULL uses hipMalloc/hipFree. */
cteno_status cteno_ctx_create(int device, void *stream, cteno_alloc_fn alloc, cteno_free_fn free_fn,
                              void *user, cteno_ctx **out);
void cteno_ctx_destroy(cteno_ctx *ctx);
cteno_status cteno_ctx_set_stream(cteno_ctx *ctx, void *stream);
/* waits for the stream and reports pending device errors */
cteno_status cteno_ctx_synchronize(cteno_ctx *ctx);
const char *cteno_last_error(void);
/* Stage kernels of degree 2 and 3, in either precision, for RK stages and
   marches (cteno_rk_stage, cteno_solve): on = 1 (default), one fused
   kernel per stage reconstructs each block of 256 cells into on-chip
   memory and evaluates the fluxes of the faces inside the block there, and
   a second kernel finishes the cells with faces to other blocks; on = 0, a
   reconstruction kernel writes all face values to device memory and a flux
   kernel reads them back.  A stage's results agree to FP64 rounding (the
   fused path sums a cell's faces inside its block first).  Synchronises. */
cteno_status cteno_ctx_set_fused_stage(cteno_ctx *ctx, int32_t on);
/* Per-kernel timing with HIP events on the context stream (off by default).
   kernel: 0 = reconstruction (the fused stage kernel when it runs), 1 =
   flux + residual + RK update (the fused stage's second kernel), 2 =
   pseudo-inverse precompute.  Reports launches and summed milliseconds
   since the last reset. */
cteno_status cteno_ctx_set_timing(cteno_ctx *ctx, int32_t on);
cteno_status cteno_ctx_kernel_stats(cteno_ctx *ctx, int32_t kernel, int64_t *launches, double *total_ms);
cteno_status cteno_ctx_reset_stats(cteno_ctx *ctx);

/* ---------------------------------------------------------------------- */
/* mesh                                                                    */
/* ---------------------------------------------------------------------- */

/* Builds faces, central and directional stencils on the host (sec. 2.1,
   2.3: central stencil of M cells, one compact directional stencil per
   face inside it) and computes the least-squares pseudo-inverses
   P = R^-1 Q^T diag(|V'_m|) of every stencil on the device in FP64
   (sec. 2.1, Householder QR), plus an FP32 copy when precision includes
   MIXED.  Synchronises. */
cteno_status cteno_mesh_upload(cteno_ctx *ctx, const cteno_mesh_desc *desc, const cteno_scheme *scheme,
                               cteno_mesh **out);
cteno_status cteno_mesh_info_get(const cteno_mesh *mesh, cteno_mesh_info *info);
/* Host copies of the stencils: central [n_cells][M] cell ids (ascending),
   directional [n_cells][3][M_d] (face neighbour first, -1 padded) and the
   directional sizes [n_cells][3] (0 = inadmissible).  Any output may be NULL. */
cteno_status cteno_mesh_stencils(const cteno_mesh *mesh, int32_t *central, int32_t *directional, int32_t *dir_count);
/* Pseudo-inverses of selected cells, copied to host: central [n][K][M]
   (columns in the order of cteno_mesh_stencils' central list), directional
   [n][3][K_d][M_d] (columns in directional-list order, zero where absent).
   which = CTENO_FP64 or CTENO_MIXED (the FP32 copy, widened).  Synchronises. */
cteno_status cteno_mesh_pinv(cteno_ctx *ctx, const cteno_mesh *mesh, int32_t which, int32_t n, const int32_t *cells,
                             double *central, double *directional);
void cteno_mesh_destroy(cteno_mesh *mesh);
/* Host-only stencil construction (no device needed), same rule and output
   layout as cteno_mesh_stencils; the outputs must hold n_cells rows. */
cteno_status cteno_stencils_host(const cteno_mesh_desc *desc, const cteno_scheme *scheme, int32_t *central,
                                 int32_t *directional, int32_t *dir_count);

/* ---------------------------------------------------------------------- */
/* solution state                                                          */
/* ---------------------------------------------------------------------- */

/* Device-resident cell averages (FP64) at time t0, copied from host u0
   [nv][n_cells]. */
cteno_status cteno_sol_create(cteno_ctx *ctx, const cteno_mesh *mesh, const double *u0, double t0, cteno_sol **out);
/* Replaces the state with host u [nv][n_cells] and sets the time. */
cteno_status cteno_sol_set(cteno_sol *sol, const double *u, double t);
/* Copies the state to host u [nv][n_cells] (may be NULL) and the time to *t
   (may be NULL).  Synchronises and reports pending device errors; returns
   CTENO_ERR_NONPHYSICAL (outputs written) once if a cteno_rk_stage call
   since the last report met a non-physical face state. */
cteno_status cteno_sol_download(cteno_sol *sol, double *u, double *t);
/* Number of cell reconstructions (cells x stages) of this solution that
   took the positivity fallback (scheme.positivity = 1) since it was created
   or last set, over cteno_reconstruct, cteno_residual, cteno_rk_stage and
   cteno_solve.  Synchronises. */
cteno_status cteno_sol_fallbacks(cteno_sol *sol, int64_t *count);
void cteno_sol_destroy(cteno_sol *sol);

/* ---------------------------------------------------------------------- */
/* stage kernels (low level; outputs in caller cell order)                 */
/* ---------------------------------------------------------------------- */

/* Reconstruction of the current state of `sol` (sec. 2.1-2.6): central and
   directional least-squares polynomials, p_1 (eq. e17), smoothness
   indicators, CTENO/CTENOZ selection and the final polynomial, evaluated at
   the N_q Gauss points of each face.
   face_vals: device [n_cells][3][N_q][nv], FP64 (precision CTENO_FP64) or
   FP32 (CTENO_MIXED); point q of face f lies at t_q along the face from
   vertex f to vertex f+1 of the counter-clockwise triangle.
   delta_out: device [n_cells][nv] ([n_cells][3][nv] per face and field with
   characteristic variables) or NULL: bit 0 = delta_1 (central),
   bit 1+f = delta of the directional stencil of face f, bit 7 = positivity
   fallback taken (scheme.positivity = 1 only).
   delta_forced: device, same layout as delta_out, or NULL: use these selections instead
   of computing them (bits of inadmissible stencils are ignored). */
cteno_status cteno_reconstruct(cteno_ctx *ctx, const cteno_mesh *mesh, const cteno_sol *sol, int32_t precision,
                               void *face_vals, uint8_t *delta_out, const uint8_t *delta_forced);
/* Face fluxes from face-point values (sec. 2.7, HLLC for Euler, upwind for
   advection), integrated over each face with the Gauss weights:
   face_flux: device [n_cells][3][nv] (FP64 or FP32 by precision), the
   outward flux of cell i through its face f, times |A_f|.  t is the time of
   the prescribed states of INFLOW faces.  Synchronises; a non-physical face
   state returns CTENO_ERR_NONPHYSICAL (the fluxes are still written). */
cteno_status cteno_flux(cteno_ctx *ctx, const cteno_mesh *mesh, int32_t precision, const void *face_vals,
                        double t, void *face_flux);
/* cteno_flux for callers that cannot allocate device memory (code that may
   not call hipMalloc, such as tight serving loops or a harness that forbids
   allocation): the same arguments, kernels and results as cteno_flux, with
   its internal-order staging buffers (face-point values, face fluxes, the
   non-physical flag) in a fixed 32 MiB array of device memory that the
   library holds on each device it runs on until the process ends.  It
   allocates nothing: meshes whose staging exceeds the array
   (about 116k cells in FP64 at degree 3) are refused with
   CTENO_ERR_INVALID.  Every call on a device shares that device's array, so
   calls that overlap on one device (other threads, other streams) race;
   calls in sequence are safe.  Synchronises. */
cteno_status cteno_flux_noalloc(cteno_ctx *ctx, const cteno_mesh *mesh, int32_t precision, const void *face_vals,
                                double t, void *face_flux);
/* Residual dU/dt = -(1/|V_i|) sum_f outward flux (the semi-discrete form
   after eq. e1) of the current state at the solution's time:
   resid device [nv][n_cells] FP64.  Synchronises; a non-physical face state
   returns CTENO_ERR_NONPHYSICAL (the residual is still written). */
cteno_status cteno_residual(cteno_ctx *ctx, const cteno_mesh *mesh, const cteno_sol *sol, int32_t precision,
                            double *resid);
/* One SSP-RK3 stage (Shu-Osher form) of size dt on `sol`: stage 0 forms
   U1 = U + dt R(U), stage 1 U2 = 3/4 U + 1/4 (U1 + dt R(U1)), stage 2
   U <- 1/3 U + 2/3 (U2 + dt R(U2)).  Stages must be issued 0, 1, 2; the
   residuals are those of the times t, t + dt and t + dt/2 (t the solution's
   time, advanced by dt after stage 2).  Asynchronous: a non-physical face
   state is reported by the next cteno_sol_download. */
cteno_status cteno_rk_stage(cteno_ctx *ctx, const cteno_mesh *mesh, cteno_sol *sol, int32_t precision, int32_t stage,
                            double dt);

/* ---------------------------------------------------------------------- */
/* time marching                                                           */
/* ---------------------------------------------------------------------- */

/* Marches `sol` with SSP-RK3 until t_final or max_steps steps, whichever
   comes first, dt = cfl * min_i 2|V_i| / sum_f |A_f| s_if (s the normal
   signal speed |v.n| + c, or |a.n|), the last step clipped to land on
   t_final.  The time step is computed and applied on the device (no host
   round trip per step); use_graph = 1 replays a captured HIP graph per step.
   steps_done (may be NULL) receives the number of steps taken by this call.
   Synchronises. */
cteno_status cteno_solve(cteno_ctx *ctx, const cteno_mesh *mesh, cteno_sol *sol, int32_t precision, double t_final,
                         int64_t max_steps, double cfl, int32_t use_graph, int64_t *steps_done);

/* Selection bytes (cells x variables, or cells x faces x characteristic
   fields) whose TENO selection (delta bits) differs between the FP32 and
   FP64 reconstructions of the current state.  Needs precision
   CTENO_BOTH on the mesh.  Synchronises. */
cteno_status cteno_count_flips(cteno_ctx *ctx, const cteno_mesh *mesh, const cteno_sol *sol, int64_t *flips);

/* ---------------------------------------------------------------------- */
/* serving: continuous batching of independent solves                     */
/* ---------------------------------------------------------------------- */

typedef struct {
    int64_t submitted, finished;
    int32_t active, peak_active;    /* solves resident on the device now / at most */
    int64_t ticks;                  /* batched SSP-RK3 steps launched (4 per tick) */
    int64_t cell_stages;            /* cells x stages of finished solves */
    int64_t bytes_in_use, peak_bytes, budget_bytes;
    int64_t fallbacks;              /* cells x stages of finished solves that took the positivity fallback */
} cteno_server_stats;

/* One request as the server saw it.  Times in seconds: build_s from
   submission until its host mesh and stencils were built; queue_s the time
   spent waiting, for device memory before the upload and for a batch slot
   after it; admit_s for the upload and the FP64 pseudo-inverse precompute;
   run_s from joining a batch until its result was on the host (steps,
   the batched ticks of the others, result copy); latency_s = submission to
   result.  Stages not reached yet read 0. */
typedef struct {
    int32_t state;                  /* CTENO_REQ_* */
    int32_t status;                 /* CTENO_OK, or the error of a FAILED request */
    int64_t n_cells;
    int64_t steps_done;
    int64_t fallbacks;              /* cells x stages that took the positivity fallback */
    double latency_s, build_s, queue_s, admit_s, run_s;
} cteno_request_info;

enum { CTENO_REQ_QUEUED = 0, CTENO_REQ_READY = 1, CTENO_REQ_RUNNING = 2, CTENO_REQ_DONE = 3, CTENO_REQ_FAILED = 4 };

/* Starts a server for independent 2-D Euler solves with one scheme (FP32
   reconstruction / weights / HLLC, FP64 state; degree 2 or 3).  Builder
   threads take requests in arrival order, build each one's mesh and
   stencils on the host, wait until its device footprint (pseudo-inverses,
   geometry, state, face values, plus the transient FP64 precompute) fits in
   hbm_budget_bytes beside the resident solves, and upload it and run its
   precompute on a stream of their own, overlapping the batched steps.  A
   scheduler thread puts resident requests into batch slots (at most
   max_slots) and runs ticks of four batched SSP-RK3 steps of every slot
   (one launch per kernel for all of them, replayed from a HIP graph whose
   grid covers the active cells; each solve keeps its own CFL time step and
   stops at its own step count), retiring finished solves between ticks and
   returning their memory.  Work is issued on streams owned by the server. */
cteno_status cteno_server_create(cteno_ctx *ctx, const cteno_scheme *scheme, size_t hbm_budget_bytes,
                                 int32_t max_slots, cteno_server **out);
/* Queues a solve of n_steps SSP-RK3 steps at the given CFL number from the
   initial cell averages u0 (host [4][n_cells]); copies every input and
   returns at once with a ticket. */
cteno_status cteno_server_submit(cteno_server *server, const cteno_mesh_desc *desc, const double *u0,
                                 int32_t n_steps, double cfl, uint64_t *ticket);
/* Reports a request's state (CTENO_REQ_*).  When it is DONE: steps_done,
   latency_s (submission to result on the host) are set and, if u_out
   (host [4][n_cells]) is not NULL, the result is copied and the ticket is
   released.  A FAILED request returns its error status (message in
   cteno_last_error); polling it with u_out != NULL releases it.  Any output
   may be NULL. */
cteno_status cteno_server_poll(cteno_server *server, uint64_t ticket, int32_t *state, double *u_out,
                               int64_t *steps_done, double *latency_s);
/* Blocks until every submitted request has finished or failed. */
cteno_status cteno_server_drain(cteno_server *server);
cteno_status cteno_server_get_stats(cteno_server *server, cteno_server_stats *stats);
/* State, counts and latency split of a request that has not been released
   (a DONE request is released by cteno_server_poll with u_out). */
cteno_status cteno_server_request_info(cteno_server *server, uint64_t ticket, cteno_request_info *info);
/* Stops the threads (queued requests are dropped) and frees everything. */
void cteno_server_destroy(cteno_server *server);

/* Device copy kernel used to calibrate hardware byte counters: copies
   n_bytes (multiple of 16) from src to dst on the context stream. */
cteno_status cteno_util_copy(cteno_ctx *ctx, void *dst, const void *src, size_t n_bytes);

#ifdef __cplusplus
}
#endif
#endif /* CTENO_H */
