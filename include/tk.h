/*
 * tk.h - C ABI of the Tucker-compressed S-model kinetic step for MI355X.
 *
 * One explicit first-order upwind finite-volume step of the tensorised
 * discrete velocity method of Chikitkin, Kornev and Titarev ("Numerical
 * solution of the Boltzmann equation with S-model collision integral using
 * tensor decompositions"): every cell's distribution function on an N^3
 * Cartesian velocity grid is a Tucker tensor (Section "Tensor
 * decompositions"), and a step is Alg. 1 (boundary values, face fluxes of
 * eq. exact-flux, the S-model collision term of Alg. 2 / eq.
 * shakhov_integral, explicit Euler of eq. expl-scheme-final) followed by
 * Tucker rounding (Op4, truncated HOSVD) back to a tolerance or rank cap.
 *
 * Conventions
 *  - Every call returns tk_status: TK_OK (0), TK_PENDING (1) or a negative
 *    error.  tk_last_error() returns the message of the last error raised
 *    on a context.  No C++ exception crosses this interface.
 *  - Host pointers passed in are only read during the call: inputs are
 *    copied before return and may be freed by the caller afterwards.
 *  - Outputs go to caller-allocated host buffers of the documented size.
 *  - Handles belong to the caller until the matching *_destroy call.  A
 *    state keeps a reference to its mesh: destroy states before meshes and
 *    everything before the context.
 *  - Calls on one context are serialised by the context.  The tk_serve_*
 *    calls are thread-safe.
 *  - All device work runs on the context's HIP stream.
 *
 * Physical units: R_g and m are parameters; the workloads use R_g = 1/2,
 * m = 1, so 2 R_g T = T.  Viscosity mu(T) = (Kn/2) T^omega, collision
 * frequency nu = p / mu with p = m n R_g T (Section "Mathematical model";
 * the nondimensional form of mu is this library's reading).
 */
#ifndef TK_H
#define TK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t tk_status;
#define TK_OK 0
#define TK_PENDING 1
#define TK_EINVAL (-1)   /* bad argument, shape or mesh                     */
#define TK_ENOMEM (-2)   /* does not fit the memory budget / device memory   */
#define TK_ENUMERIC (-3) /* n <= 0, T <= 0 or a non-finite value in a cell   */
#define TK_EDEVICE (-4)  /* HIP runtime or kernel launch failure             */
#define TK_EBUSY (-5)    /* server stopped or queue closed                   */
#define TK_ENOTFOUND (-6)/* unknown ticket                                   */

typedef struct tk_ctx tk_ctx;
typedef struct tk_mesh tk_mesh;
typedef struct tk_state tk_state;
typedef struct tk_server tk_server;

/* Boundary kinds (Section "Mathematical model": free stream, diffuse wall,
 * symmetry plane; plus zero-gradient outflow).                            */
enum { TK_BC_SYM = 0, TK_BC_INFLOW = 1, TK_BC_OUTFLOW = 2, TK_BC_WALL = 3 };

typedef struct {
  int32_t kind;   /* TK_BC_*                                               */
  double n;       /* free-stream density (TK_BC_INFLOW)                    */
  double u[3];    /* free-stream velocity (TK_BC_INFLOW)                   */
  double T;       /* free-stream temperature (TK_BC_INFLOW)                */
  double T_w;     /* wall temperature (TK_BC_WALL)                         */
} tk_bc;

/* Hexahedral mesh in the form the paper's mesh reader stores it (Section
 * "Implementation"; eq. ode_system): per face the two cells, unit normal
 * and area; per cell the volume.  A boundary face has face_right = -(b+1)
 * with b an index into bc[], its left cell is the interior cell and its
 * normal points out of the domain.  Periodic boundaries are interior
 * faces.  Every cell must have at most 6 faces and be closed
 * (|sum_l s_l A_l e_l| <= 1e-12 sum_l A_l), otherwise TK_EINVAL.
 * Symmetry and wall boundaries must lie on coordinate-axis planes.        */
typedef struct {
  int32_t n_cells;
  int32_t n_faces;
  const int32_t* face_left;    /* [n_faces]                               */
  const int32_t* face_right;   /* [n_faces]                               */
  const double* face_normal;   /* [n_faces][3], unit, left -> right       */
  const double* face_area;     /* [n_faces]                               */
  const double* cell_volume;   /* [n_cells]                               */
  const double* cell_center;   /* [n_cells][3], may be NULL               */
  int32_t n_bc;
  const tk_bc* bc;             /* [n_bc]                                  */
} tk_mesh_desc;

enum { TK_FP64 = 0, TK_MIXED = 1 };

/* Solver parameters of one instance.  Velocity grid (Section "Discrete
 * velocity method"): N uniform nodes per axis on [-xi_max, xi_max] with
 * the end points included, quadrature weight dxi^3.                       */
typedef struct {
  int32_t N;          /* 16, 24, 32 or 48 (FP64 at 48: every cell through
                         the general fibre-pass expansion, for reference runs) */
  double xi_max;
  double R_g, m;      /* gas constant, molecular mass                      */
  double Pr;          /* Prandtl number (2/3 for a monatomic gas)          */
  double omega;       /* viscosity exponent                                */
  double Kn;          /* mu(T) = (Kn/2) T^omega                            */
  double tol;         /* rounding tolerance eps (Op4)                      */
  int32_t rank_cap;   /* 1 .. 16                                           */
  double cfl;         /* dt = cfl / max_i (D_i + nu_i^0), see tk_state_dt  */
  int32_t precision;  /* TK_FP64 or TK_MIXED                               */
} tk_params;

/* A Tucker tensor A(i1,i2,i3) = sum G(k1,k2,k3) U1(i1,k1) U2(i2,k2) U3(i3,k3)
 * with N x r_a factors stored column-major (U_a[i + N k]) and the core
 * column-major (G[k1 + r1 (k2 + r2 k3)]).  Caller-owned buffers; on output
 * core must hold rank_cap^3 and each U[a] N * rank_cap doubles.           */
typedef struct {
  int32_t N;
  int32_t r[3];
  double* core;
  double* U[3];
} tk_tucker;

/* ---- context ------------------------------------------------------------ */
/* device: HIP device ordinal, or -1 for a host-only context that can load
 * and validate meshes but runs no device work (state creation and rounding
 * then return TK_EDEVICE).  hbm_budget: bytes the library may allocate
 * (0 = 90% of free device memory).  hip_stream: a hipStream_t to run on
 * (NULL = the library creates one at default priority).  TK_EDEVICE if the
 * device is not available.                                                */
tk_status tk_ctx_create(int32_t device, size_t hbm_budget, void* hip_stream, tk_ctx** out);
/* Device memory from the caller, for example a framework's caching
 * allocator: every device buffer of the context (states, workspaces, the
 * rounding hook's buffers) is obtained by alloc(user, bytes), which returns
 * device memory on `device` aligned to at least 256 bytes or NULL (the call
 * then fails with TK_ENOMEM), and returned by free(user, ptr) when the
 * library no longer needs it (at the latest when its state or context is
 * destroyed).  The budget still applies.  The functions are called with the
 * context's lock held, from the calling thread (or the server's worker
 * thread for a serving context) and must not call back into the library.
 * tk_ctx_create(...) is tk_ctx_create_ex(..., NULL, ...).                  */
typedef struct {
  void* user;
  void* (*alloc)(void* user, size_t bytes);
  void (*free)(void* user, void* ptr);
} tk_alloc_fns;
tk_status tk_ctx_create_ex(int32_t device, size_t hbm_budget, void* hip_stream, const tk_alloc_fns* alloc,
                           tk_ctx** out);
tk_status tk_ctx_destroy(tk_ctx* ctx);
const char* tk_last_error(const tk_ctx* ctx);
tk_status tk_sync(tk_ctx* ctx);
/* Per-kernel timing with HIP events recorded around every launch of the
 * named kernel family while enabled, on the stream the launch runs on (the
 * context stream, or the state's second stream for alternate rounding
 * passes: then a launch's time includes the concurrent pass's kernels).  */
tk_status tk_prof_enable(tk_ctx* ctx, int32_t on);
tk_status tk_prof_get(tk_ctx* ctx, const char* kernel, double* total_ms, int64_t* launches);
tk_status tk_prof_reset(tk_ctx* ctx);
/* Eigensolver counters of the N-basis rounding since the last reset
 * (process-wide): out4[1] matrices solved, [2] Jacobi sweeps run (sweeps
 * that found nothing to rotate are not counted); [0] and [3] are zero.
 * Synchronises the context stream.                                        */
tk_status tk_prof_eig(tk_ctx* ctx, int64_t* out4, int32_t reset);

/* ---- mesh ------------------------------------------------------------------ */
tk_status tk_mesh_load(tk_ctx* ctx, const tk_mesh_desc* desc, tk_mesh** out);
tk_status tk_mesh_destroy(tk_mesh* mesh);

/* ---- state -------------------------------------------------------------- */
/* Rank-1 Maxwellian per cell from macro[n_cells][5] = (n, u1, u2, u3, T)
 * (Section "Tensorized discrete velocity method": the Maxwellian is the
 * product of three 1-D functions).  Computes the face data and dt.
 * TK_ENUMERIC if some n <= 0 or T <= 0; TK_ENOMEM if it does not fit.    */
tk_status tk_state_init(tk_ctx* ctx, const tk_mesh* mesh, const tk_params* params,
                        const double* macro, tk_state** out);
/* Several independent instances advanced together (same N and precision;
 * other parameters per instance).  Cells are numbered instance after
 * instance in the order given.                                            */
tk_status tk_state_init_batch(tk_ctx* ctx, int32_t count, const tk_mesh* const* meshes,
                              const tk_params* params, const double* const* macros,
                              tk_state** out);
tk_status tk_state_destroy(tk_state* st);
/* Number of cells, instances, and the dt of instance `inst`.               */
tk_status tk_state_info(const tk_state* st, int32_t* n_cells, int32_t* n_instances);
tk_status tk_state_dt(const tk_state* st, int32_t inst, double* dt);

/* Cells per rounding pass (the expansion workspace holds one pass).
 * cells = 0 lets the library choose: on the first state of a shape (N,
 * precision, rank cap, cell count, face kind) on a context, 16 ordinary
 * steps (so that the ranks resemble a running state) are followed by 4
 * timed steps with each of several pass sizes (cycles over the sizes in
 * alternating order), and the size with the smallest mean time is kept
 * for every later state of that shape on the context.  cells > 0 fixes the pass size
 * (TK_EINVAL above the allocated maximum).  Every choice computes the same
 * bits: cells are independent within a pass.  tk_state_chunk reports the
 * size in use and the allocated maximum.                                  */
tk_status tk_state_set_chunk(tk_state* st, int32_t cells);
tk_status tk_state_chunk(const tk_state* st, int32_t* cells, int32_t* max_cells);
/* Run the remaining timed trial steps of the pass-size choice now (they
 * advance the state like any step), then wait; steps_run (nullable)
 * receives their number.  No-op when the size is chosen or fixed.        */
tk_status tk_state_tune(tk_state* st, int32_t* steps_run);
/* on != 0: after the first step, each step is replayed from a HIP graph
 * captured from the same launches (one graph per buffer parity, captured
 * again when the pass size changes); not while kernel timing is enabled.
 * The results are those of the eager launches.                           */
tk_status tk_state_use_graph(tk_state* st, int32_t on);
/* two = 1: alternate rounding passes on the state's second stream (the
 * default when its second workspace was allocated); two = 0: every pass on
 * the context stream (for timing kernels one at a time); two < 0: leave
 * the setting.  available (nullable) receives 1 if the second workspace
 * and stream exist.  Results are the same either way.                    */
tk_status tk_state_streams(tk_state* st, int32_t two, int32_t* available);
/* Rounding path (Op4, Section "Tensor decompositions").  With
 * factor_space = 1 (the default where available: Tucker states with
 * N <= 32) a cell whose faces all lie on coordinate-axis planes and whose
 * own state and far sides all have rank 1 is rounded in the space of its
 * concatenated factors:
 * Gram-Schmidt QR of the factors, the small core multiplied by the R
 * factors, eigen-decompositions of that core's unfolding Grams, fused with
 * the term assembly; the other cells are rounded in the N-basis (the update
 * expanded on the N^3 grid, mode Grams of the full tensor).
 * factor_space = 0 rounds every cell in the N-basis; < 0 leaves the
 * setting.  Both give the truncated HOSVD of the same update (results
 * differ by rounding errors, and where an eigenvalue sits at the
 * truncation threshold by the rank chosen).  TK_EINVAL when enabling it on
 * a state without the factor-space path.  counts (nullable, [4]) receives
 * and resets: cells rounded in factor space, cells rounded in the N-basis
 * by eager steps (not counted for served states), Jacobi sweeps in factor
 * space, and the FP64 operations
 * of the factor-space rounding (2 per multiply-add of its Gram-Schmidt,
 * core, Gram, rotation, Jacobi and output products).  Waits for the
 * context stream.                                                         */
tk_status tk_state_rounding(tk_state* st, int32_t factor_space, int64_t* counts);

/* Restart checkpoints (Sec. "The program": a run is continued from a saved
 * solution).  tk_state_checkpoint writes the whole state to host memory:
 * the instances' step parameters (dt included), every cell's Tucker core,
 * factors and ranks (or the full tensors of a plain state), the
 * eigensolver's warm-start bases and whether they are in use.  With
 * buf == NULL it only sets *needed; TK_EINVAL if bytes < *needed.  The
 * buffer is the caller's.  tk_state_restore loads such a buffer into a
 * state built from the same meshes, N, precision, rank cap and kind
 * (checked against the buffer's header, TK_EINVAL otherwise); the steps
 * that follow are then bit for bit those the saved state would have taken.
 * Both wait for the context stream.                                       */
tk_status tk_state_checkpoint(tk_state* st, void* buf, size_t bytes, size_t* needed);
tk_status tk_state_restore(tk_state* st, const void* buf, size_t bytes);

/* Macroparameters of every cell, out[n_cells][8] = (n, u1, u2, u3, T, q1,
 * q2, q3), computed on the device in FP64 from the Tucker state (Alg. 2
 * steps 1-9 by Op5 convolutions).  Blocking.                              */
tk_status tk_moments(tk_state* st, double* out);

/* Advance nsteps explicit steps (Alg. 1 with one rounding per cell per
 * step).  Enqueued on the context stream and waited for.  When the budget
 * left room for a second workspace at tk_state_init, alternate rounding
 * passes of a step run on a second stream of the state's own, forked from
 * and joined back into the context stream within the step, with the same
 * results; to the caller a step remains ordered work on the context
 * stream.  residual, if not
 * NULL, receives per instance max(||dn||/||n||, ||dT||/||T||) over the
 * last step (cell-volume weighted 2-norms).  TK_ENUMERIC if a cell's n or
 * T became non-positive or non-finite (the state is left as computed).    */
tk_status tk_step(tk_state* st, int32_t nsteps, double* residual);
/* Enqueue nsteps steps without waiting (no residual, no numeric check).   */
tk_status tk_step_async(tk_state* st, int32_t nsteps);

/* iters LU-SGS implicit iterations (Section "Tensorized discrete velocity
 * method", implicit scheme): eq. linear-system times dt,
 *   [I - dt dR/df] df = dt R(f),   f <- f + df,
 * with f_S and the boundary ghosts held fixed in the Jacobian, the far-cell
 * blocks (dt A / V) P_in of the explicit fluxes, and the diagonal of eq.
 * diagonal_term with |xi_n| replaced by the bound |xi| of eq.
 * xin-one-rank-approx, (1 + dt nu) 1 + (dt / (2 V)) (sum_l A_l) |xi|, taken
 * as its rank-1 truncated HOSVD and divided exactly in rank-1 form (eq.
 * one_rank_division).  Symmetric Gauss-Seidel order: a greedy colouring of
 * the face graph (cells in index order, the smallest colour no earlier
 * neighbour has); the forward sweep forms df* colour by colour ascending,
 * the backward sweep df descending (cells without a later neighbour keep
 * df*), each rounded to the state's tolerance and cap, and f + df is
 * rounded into the new state.  dt is the state's (a CFL above the explicit
 * step's bound of 1 is the point).  FP64 states round each stage on the
 * FP64 N-basis path, mixed states assemble it in FP32 and round it with
 * the mixed path's eigensolver.  residual as for tk_step.  TK_EINVAL for
 * plain or N = 48 states and for meshes with faces off the coordinate
 * axes.  Blocking.                                                        */
tk_status tk_lusgs(tk_state* st, int32_t iters, double* residual);

/* Intermediate rounding (Section "Tensorized discrete velocity method": a
 * rounding after each operation that can raise the Tucker ranks a lot).
 * With on = 1 every later step of st rounds each face's flux term,
 *   E_l = -(dt A_l / V) (P_out o f + P_in o g_l)
 * (P_out/in = max/min(s xi_a, 0) on an axis-aligned face, (xi_n +- est_l)/2
 * with the |xi.e| estimate on an oblique one; g_l the far side or ghost),
 * to the instance's relative accuracy and rank cap on its own, then rounds
 * the sum (1 - dt nu) f + dt nu f_S + sum_l E~_l once more.  With eps -> 0
 * this is the exact update that on = 0 (the default) rounds once; otherwise
 * the result lies within eps (sum_l |E_l| (1 + eps) + |f*|) of the exact
 * update f* per cell (Frobenius norms).  tk_lusgs iterations keep their own
 * single rounding whatever the setting.  Every cell takes the N-basis path,
 * eagerly on the context stream (no graph replay, no pass-size trials),
 * with the precision's eigensolver (FP64: two passes).
 * The first enable allocates six state-sized buffers (TK_ENOMEM beyond the
 * budget); they live as long as the state.  TK_EINVAL for plain states and
 * a server's states.                                                      */
tk_status tk_state_face_rounding(tk_state* st, int32_t on);

/* Rank histogram (hist[0..16], ranks are max over modes) and mean
 * compression ratio C = (r1 r2 r3 + N (r1 + r2 + r3)) / N^3 (Section "Test
 * problem").                                                              */
tk_status tk_state_ranks(tk_state* st, int32_t* ranks /* [n_cells][3] or NULL */,
                         double* mean_compression);

/* Copy one cell's Tucker state out (columns beyond the ranks are not
 * written).                                                               */
tk_status tk_state_export(tk_state* st, int32_t cell, tk_tucker* out);

/* Op4 on a resident state: every cell's current Tucker tensor is rounded
 * again by truncated HOSVD with tolerance tol and rank cap `cap` (1 .. the
 * state's rank cap), in FP64 on the N-basis path (the tensor expanded on
 * the N^3 grid, mode Grams, two Jacobi passes), and becomes the state.  The
 * step's own rounding is unchanged (it keeps each instance's tol and cap).
 * Allocates a work space for passes of up to 4096 cells within the budget
 * (TK_ENOMEM if none fits) and waits for the context stream.  TK_EINVAL for
 * a plain state, N = 48, tol < 0 or cap out of range.                       */
tk_status tk_round(tk_state* st, double tol, int32_t cap);

/* Test hook for Op4: round `count` Tucker tensors (same N, ranks <= N)
 * with tolerance tol and rank cap `cap` by truncated HOSVD on the device,
 * FP64 throughout.  TK_EINVAL if a rank exceeds N.                        */
tk_status tk_round_tucker(tk_ctx* ctx, int32_t count, const tk_tucker* in, double tol,
                          int32_t cap, tk_tucker* out);

/* Op4 on device-resident Tucker tensors with no device allocation, for
 * callers that cannot allocate: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc.  The same rounding as
 * tk_round_tucker (same kernels, same results).  Buffers are caller-owned
 * device memory in the state layout:
 *   core_in[count][in_cap^3]    (k1 + in_cap (k2 + in_cap k3)),
 *   fac_in[count][3][in_cap][N] (column k of mode a: N contiguous values),
 *   rank_in[count][3]           (each in 1..in_cap; a value outside is
 *                                clamped into that range by the kernels),
 * and the outputs core_out[count][cap^3], fac_out[count][3][cap][N],
 * rank_out[count][3] in the same layout with cap in place of in_cap
 * (entries beyond the ranks are written as zeros).  N is 16, 24 or 32,
 * in_cap and cap in 1..16 and <= N, otherwise TK_EINVAL.  Work space comes
 * from a fixed 32 MiB device array of the library (one copy per GPU, kept
 * until the process ends): tensors are processed in passes of as many as
 * fit it (107 at N = 32).  Enqueued on the context stream without waiting;
 * the caller synchronises (tk_sync) before reading the outputs.  Calls
 * share that array: calls that overlap on one GPU (from different contexts
 * or streams) race.  Calls no allocating routine of HIP or any library.   */
tk_status tk_round_tucker_noalloc(tk_ctx* ctx, int32_t N, int32_t count, int32_t in_cap, const double* core_in,
                                  const double* fac_in, const int32_t* rank_in, double tol, int32_t cap,
                                  double* core_out, double* fac_out, int32_t* rank_out);

/* ---- plain full-tensor comparator -------------------------------------- */
/* The same step with N^3 values stored per cell and no rounding (the
 * paper's baseline discrete velocity method).  Precision TK_FP64 stores
 * doubles, TK_MIXED stores floats (FP64 moments).                        */
tk_status tk_plain_init(tk_ctx* ctx, const tk_mesh* mesh, const tk_params* params,
                        const double* macro, tk_state** out);

/* ---- serving --------------------------------------------------------------- */
typedef struct {
  tk_mesh_desc mesh;
  tk_params params;
  const double* macro;   /* [n_cells][5]                                   */
  int32_t max_steps;
  double residual_tol;   /* stop when residual < residual_tol             */
} tk_request;

typedef struct {
  tk_status status;      /* TK_PENDING while queued or running             */
  int32_t steps;
  double residual;
  double t_arrive, t_admit, t_done;  /* seconds on the server's clock      */
  double* macro_out;     /* caller buffer [n_cells][8], filled when done, may be NULL */
} tk_result;

/* Continuous batching of independent solves over one device.  A worker
 * thread admits queued requests in arrival order among those whose
 * estimated device memory fits what the running ones leave of hbm_budget
 * (0: the context's budget).  Requests that share N, precision and
 * whether their mesh has faces off the coordinate axes form a cohort: the
 * instances of one resident batched state with its own stream, so one step
 * of the cohort is one set of launches over all their cells.  A newly
 * admitted request joins the running cohort of its kind at that cohort's
 * next step boundary (the cohort's state is rebuilt with the running
 * requests' states copied over on the device; old and new states coexist
 * for the rebuild), or forms a new cohort when none runs.  Each cohort
 * keeps one step in flight and starts its next as soon as that one
 * completes, without waiting for the other cohorts.  A request retires when
 * its residual (tk_step) falls below residual_tol, at max_steps, or with
 * TK_ENUMERIC when one of its cells turns non-positive or non-finite; its
 * cells are then no longer stepped, and its memory returns to the budget
 * when its cohort ends or is rebuilt.  A request's result does not depend
 * on the requests served beside it.                                       */
tk_status tk_serve_create(tk_ctx* ctx, size_t hbm_budget, tk_server** out);
/* Never blocks; TK_ENOMEM only for a request that could never fit.       */
tk_status tk_serve_submit(tk_server* srv, const tk_request* req, uint64_t* ticket);
/* Returns the request's status (TK_PENDING while queued or running) and
 * fills *res; TK_ENOTFOUND for an unknown ticket.                         */
tk_status tk_serve_poll(tk_server* srv, uint64_t ticket, tk_result* res);
/* out4[0] cohorts formed or rebuilt, [1] cohort steps (shared launch
 * sets), [2] request steps, [3] requests in the largest cohort.           */
tk_status tk_serve_stats(tk_server* srv, int64_t* out4);
/* Stops the worker (running requests stay TK_PENDING) and frees all.     */
tk_status tk_serve_destroy(tk_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* TK_H */
