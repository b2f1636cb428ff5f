/*
 * emg.h -- C ABI of the MI355X (gfx950) geometric-multigrid solver for the
 * node-based finite-difference elasticity operator of Runnels, Agrawal,
 * Zhang and Almgren, "Massively parallel finite difference elasticity using
 * block-structured adaptive mesh refinement with a geometric multigrid
 * solver" (arXiv 2001.04789).
 *
 * Conventions shared by every entry point
 *   - Every function returns an emg_status; EMG_OK (0) on success.  On error
 *     emg_last_error() returns a message (thread-local, valid until the next
 *     call on the same thread).  No C++ exception crosses this boundary.
 *   - Grids are node based.  Axis a has n[a] nodes including both ends,
 *     spacing h[a] = (hi[a] - lo[a]) / (n[a] - 1).  A periodic axis stores
 *     n[a] - 1 unique nodes (node n[a]-1 is node 0); every other axis stores
 *     n[a].  m[a] below is that stored count (m[2] = 1 in 2D).
 *   - Fields are dense structure-of-arrays, component-major:
 *     field[comp][z][y][x] over the stored nodes, x fastest, no padding.
 *   - A pointer argument is a host pointer unless the call's `on_device`
 *     flag is set (then it is a device pointer on the problem's GPU, e.g. a
 *     torch tensor's data_ptr()).  The library copies what it is given; the
 *     caller keeps ownership of every buffer it passes.  A device buffer must
 *     hold its final contents when the call is made: the problem's stream
 *     does not wait on the caller's streams (synchronize the producing
 *     stream first, or hand the library that stream with emg_set_stream).
 *     Calls that write device buffers have finished writing them when they
 *     return.
 *   - Each problem owns its device memory and one HIP stream (created at
 *     default priority); all of its work runs on that stream.  Calls on one
 *     problem must not overlap; different problems may be used from
 *     different threads.
 */
#ifndef EMG_H
#define EMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  EMG_OK = 0,
  EMG_EINVAL = -1,     /* bad argument, size, layout or boundary-condition combination */
  EMG_ENOMEM = -2,     /* device allocation failed or HBM budget exceeded */
  EMG_EDEVICE = -3,    /* a HIP call failed */
  EMG_ENOTCONV = -4,   /* cycle cap reached; the last iterate and stats are still returned */
  EMG_EDIVERGED = -5,  /* residual norm became NaN or Inf */
  EMG_ESTATE = -6,     /* call order, e.g. solve before the moduli are set */
  EMG_EBUSY = -7       /* the problem, or the device's allocation-free scratch, is in use by a
                          call on another thread; nothing was done */
} emg_status;

/* Face boundary types (Sec. 2.1, eqs. elastic_b1, elastic_b2 and
 * elastic_b3; periodic faces of representative volume elements, Sec. 1).
 * Face f = 2*axis + side (side 0 = low end, 1 = high end).  Both faces of an
 * axis are periodic or neither is.  A node on a Dirichlet face has the
 * Dirichlet row; otherwise a node on a Neumann face has the Neumann row
 * (normal derivative of each displacement component, 3-point one-sided,
 * summed over its Neumann faces); otherwise a node on traction faces has the
 * sum over those faces of the traction rows. */
typedef enum { EMG_BC_DIRICHLET = 0, EMG_BC_TRACTION = 1, EMG_BC_PERIODIC = 2, EMG_BC_NEUMANN = 3 } emg_bc_type;

/* Stored moduli per node (Sec. 2.1.1 reduced constants; Sec. 4.3 Voigt form):
 *   EMG_MOD_ISO:   2 components, lambda then mu.
 *   EMG_MOD_ANISO: upper triangle, row-major, of the symmetric Voigt matrix:
 *                  21 components in 3D (Voigt order 11,22,33,23,31,12),
 *                  6 in 2D plane strain (order 11,22,12). */
typedef enum { EMG_MOD_ISO = 0, EMG_MOD_ANISO = 1 } emg_moduli_kind;

typedef enum { EMG_FP64 = 0, EMG_MIXED = 1 } emg_precision;

/* Multigrid cycle (Sec. 3.1).  EMG_VCYCLE: nu1 sweeps, residual,
 * restriction, coarse correction by one V-cycle from zero, interpolation,
 * nu2 sweeps.  EMG_FCYCLE: the same, with the coarse correction given by an
 * F-cycle from zero followed by a V-cycle from its result (level k below the
 * finest is then smoothed k + 1 times per cycle). */
typedef enum { EMG_VCYCLE = 0, EMG_FCYCLE = 1 } emg_cycle;

typedef struct emg_ctx emg_ctx;
typedef struct emg_problem emg_problem;

typedef struct {
  int dim;          /* 2 (plane strain) or 3 */
  int64_t n[3];     /* nodes per axis including both ends; n[2] = 1 in 2D */
  double lo[3], hi[3];
  int bc[6];        /* emg_bc_type per face; faces 4,5 are ignored in 2D */
  int kind;         /* emg_moduli_kind */
} emg_domain;

typedef struct {
  double rtol;       /* stop when ||r||_2 / ||r_0||_2 <= rtol (default 1e-10); the norm runs over
                        non-Dirichlet rows, r_0 is the residual of the Dirichlet lift */
  int max_cycles;    /* cap on V-cycles, default 200.  EMG_MIXED: each refinement step runs
                        inner_cycles FP32 V-cycles, so the cap is rounded up to whole steps; after
                        an FP64 fallback every FP64 V-cycle counts one against what is left */
  int precision;     /* EMG_FP64: V-cycles in FP64.  EMG_MIXED: FP64 residual and update around
                        one FP32 V-cycle per iteration, FP64 coarsest solve */
  int nu1, nu2;      /* damped-Jacobi sweeps before / after the coarse correction (default 2, 2) */
  double omega;      /* Jacobi damping (default 2/3) */
  int warm_start;    /* 1: start from the current displacement instead of the Dirichlet lift */
  int check_every;   /* V-cycles (EMG_FP64) or refinement steps (EMG_MIXED) per device-side launch
                        between host convergence reads (default 4); those after convergence inside
                        a launch are skipped on the device */
  int use_graph;     /* 1 (default): replay captured HIP graphs; 0: launch kernels eagerly */
  int cycle;         /* emg_cycle (default EMG_VCYCLE); emg_solve_batch and the server take
                        EMG_VCYCLE only (EMG_EINVAL otherwise) */
  int stall_iters;   /* EMG_MIXED in emg_solve: if the FP64 residual norm has not fallen below
                        stall_factor times its value at the start of a window of stall_iters
                        refinement steps (not V-cycles), the solve continues with FP64 cycles from the
                        current iterate (emg_solve_stats.fp64_fallback = 1).  Default 24; 0 turns
                        the test off; read at host convergence reads (every check_every) */
  double stall_factor; /* in (0, 1); default 0.5 */
  int inner_cycles;  /* EMG_MIXED only (EMG_EINVAL for FP64 or refined levels if not 1; also
                        taken by emg_solve_batch and the server):
                        FP32 cycles per FP64 refinement step, 1..4 (default 1).  Each step
                        computes one FP64 residual and applies one correction; the cycles
                        after the first continue the FP32 correction from its iterate.  The
                        convergence test runs once per step, so emg_solve_stats.cycles is a
                        multiple of inner_cycles (until an FP64 fallback) and max_cycles is
                        rounded up to one */
} emg_solve_opts;

typedef struct {
  int cycles;          /* V-cycles (or refinement iterations) applied to the returned solution */
  int converged;       /* 1 if rel_res <= rtol */
  double rel_res;      /* final ||r|| / ||r_0|| (FP64 residual) */
  double conv_factor;  /* geometric mean reduction per cycle */
  double solve_seconds;/* wall time of the cycle loop (lift to tolerance) */
  double setup_seconds;/* wall time of hierarchy setup and right-hand-side assembly in this call */
  int64_t dofs;        /* d x stored nodes not on a Dirichlet face */
  int fp64_fallback;   /* 1 if a mixed-precision solve stalled and finished with FP64 cycles */
} emg_solve_stats;

const char *emg_last_error(void);
void emg_default_opts(emg_solve_opts *opts);

/* Context: binds a HIP device and an HBM budget (0 = no limit) checked at
 * problem creation against the problem's device footprint.  Destroying a
 * context that still has live problems or servers defers the release to the
 * last of them; no new problem or server can be created on it meanwhile. */
emg_status emg_ctx_create(int hip_device, size_t hbm_budget_bytes, emg_ctx **out);
emg_status emg_ctx_destroy(emg_ctx *ctx);

/* Problem on one node grid.  Builds the multigrid hierarchy (levels 0, -1,
 * -2, ... of Sec. 3.1): all axes halve together while every non-periodic
 * axis has an even cell count >= 8 and every periodic axis an even stored
 * node count >= 8; the coarsest level is solved exactly in FP64.
 * EMG_EINVAL for: dim not 2/3, an axis with fewer than 5 nodes, mismatched
 * periodic faces, no Dirichlet face (rigid-body null space), fewer than two
 * levels, a coarsest level with more than 1536 unknowns, or 2^29 or more
 * stored nodes (the interior kernels use 32-bit node offsets).  The device
 * footprint is allocated here (EMG_ENOMEM if it exceeds the budget). */
emg_status emg_problem_create(emg_ctx *ctx, const emg_domain *dom, emg_problem **out);
emg_status emg_problem_destroy(emg_problem *p);
/* Replace the problem's stream (a hipStream_t, e.g. torch's current stream
 * on ROCm).  NULL restores the problem's own stream. */
emg_status emg_set_stream(emg_problem *p, void *hip_stream);
/* Bytes of device memory the problem holds. */
emg_status emg_footprint(const emg_problem *p, size_t *bytes);

/* Inputs of Sec. 2.1 eq. elastic_int: moduli C (layout per emg_moduli_kind),
 * eigenstrain eps0 (tensor components, not engineering shears, Voigt order,
 * 6 in 3D / 3 in 2D; NULL = 0), body force b (d components; NULL = 0). */
emg_status emg_set_moduli(emg_problem *p, const double *C, int on_device);
emg_status emg_set_eigenstrain(emg_problem *p, const double *eps0, int on_device);
emg_status emg_set_body_force(emg_problem *p, const double *b, int on_device);
/* Face data: d components over the face's stored nodes, laid out like a
 * field whose normal axis has extent 1.  Prescribed displacement u0 on a
 * Dirichlet face (eq. elastic_b1), prescribed traction t0 on a traction face
 * (eq. elastic_b2), prescribed normal derivative du0_i = (du_i/dx_j) n_j on a
 * Neumann face (eq. elastic_b3; n the outward normal).  NULL = 0.  At a node
 * on several Dirichlet faces the lowest-numbered face supplies u0; at a node
 * on several Neumann faces the row and its right-hand side sum over them. */
emg_status emg_set_face(emg_problem *p, int face, const double *values, int on_device);

/* Solve D_H(u) = -(D(0) + b) with the boundary operators (Sec. 2.1.1) by
 * correction-scheme V-cycles (Sec. 3.1) to opts->rtol.  Blocking.
 * EMG_ENOTCONV / EMG_EDIVERGED still leave the last iterate readable. */
emg_status emg_solve(emg_problem *p, const emg_solve_opts *opts, emg_solve_stats *stats);

/* Outputs on level 0: displacement (d components) and the assembled
 * right-hand side (d components).  Stress sigma = C (grad u - eps0) (Sec. 4.3)
 * in Voigt order (6 in 3D: 11,22,33,23,31,12; 3 in 2D: 11,22,12) on `level`:
 * 0 = the base grid (6 or 3 components over its stored nodes; central
 * differences inside, 3-point one-sided on non-periodic faces); k >= 1 = the
 * refined level k after a solve (over its bounding array, extents of
 * emg_amr_level_shape), from its displacement with the interpolated ghosts
 * and the moduli of the solve (covered nodes averaged from level k+1);
 * values are the stress of the composite solution at valid nodes (central
 * differences: their neighbours are valid or ghosts); at other nodes they
 * are not defined.  EMG_EINVAL for a level that does not exist. */
emg_status emg_get_displacement(emg_problem *p, double *u, int on_device);
emg_status emg_set_displacement(emg_problem *p, const double *u, int on_device);
emg_status emg_get_stress(emg_problem *p, int level, double *sigma, int on_device);
/* Von Mises stress sqrt(3/2 S_ij S_ij), S the deviator of the stress that
 * emg_get_stress returns (Sec. 4.3), one value per stored node of level 0.
 * 3D problems only (EMG_EINVAL in 2D: plane strain does not store the moduli
 * that give sigma_33).  svm: N doubles, host or device (on_device). */
emg_status emg_get_von_mises(emg_problem *p, double *svm, int on_device);
emg_status emg_get_rhs(emg_problem *p, double *f, int on_device);

/* ---- level-wise steps of the cycle, for verification and timing ----
 * Level 0 is the input grid, level l the l-th coarsening.  All vector
 * arguments are DEVICE pointers with d components in the level's layout;
 * `precision` selects double (EMG_FP64) or float (EMG_MIXED) vectors and
 * moduli.  Setup (coarsened moduli, coarsest inverse) runs on first use. */
emg_status emg_num_levels(emg_problem *p, int *levels);
/* Stencil pass used on a level (introspection, e.g. for tests and profiles):
 * *chunks > 0 if stencil passes of that level in that precision (EMG_FP64
 * for FP64 passes, EMG_MIXED for the FP32 ones) run the z-marching kernel
 * (3D levels, isotropic or anisotropic, large enough to give every CU its
 * resident workgroups), with that many plane runs per column; 0 if they run
 * the tile kernel. */
emg_status emg_level_zmarch(emg_problem *p, int level, int precision, int *chunks);
emg_status emg_level_shape(emg_problem *p, int level, int64_t m[3], double h[3]);
/* moduli of a level (FP64, layout of emg_set_moduli), device pointer out */
emg_status emg_level_moduli(emg_problem *p, int level, double *C_dev);
/* out = D_H u on every row (interior, traction, Dirichlet rows u) */
emg_status emg_level_apply(emg_problem *p, int level, int precision, const void *u, void *out);
/* out = f - D_H u */
emg_status emg_level_residual(emg_problem *p, int level, int precision, const void *u, const void *f, void *out);
/* one damped Jacobi sweep: out = u + omega (f - D_H u) / diag; Dirichlet rows out = f */
emg_status emg_level_jacobi(emg_problem *p, int level, int precision, double omega, const void *u,
                            const void *f, void *out);
/* full-weighting restriction of a fine residual on `level` to level+1 */
emg_status emg_level_restrict(emg_problem *p, int level, int precision, const void *r_fine, void *f_coarse);
/* u_fine (on `level`) += interpolation of e_coarse (on level+1); Dirichlet rows untouched */
emg_status emg_level_prolong_add(emg_problem *p, int level, int precision, const void *e_coarse, void *u_fine);
/* exact FP64 solve on the coarsest level: e = A^-1 f, A^-1 the dense inverse built at setup by
 * blocked Gauss-Jordan elimination with partial pivoting (the bottom of the cycle is not specified
 * by the paper; a direct FP64 solve keeps it exact in both precisions) */
emg_status emg_level_bottom_solve(emg_problem *p, int precision, const void *f, void *e);

/* ---- ragged batches ----
 * Solve n independent problems (any sizes, both moduli kinds, same context
 * and dimension) together: every step of the cycle is one launch per
 * (dimension, moduli kind) group whose workgroups walk a device work list of
 * (problem, level, tiles) entries, captured once as a HIP graph and replayed
 * until every problem has converged; a converged problem's entries are
 * skipped.  Each problem's arithmetic is that of emg_solve, so its result is
 * bit-identical alone and in the batch.  Runs on probs[0]'s stream.  stats
 * (n entries, may be NULL) get per-problem cycles/residuals; solve_seconds is
 * the batch's wall time.  Refined (AMR) problems and warm starts are rejected. */
emg_status emg_solve_batch(emg_problem **probs, int n, const emg_solve_opts *opts, emg_solve_stats *stats);

/* Allocation-free variant of emg_solve_batch, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same problems, options, arithmetic and
 * results (bit for bit) as emg_solve_batch; what differs:
 *   - the batch's device work lists live in a fixed array of
 *     EMG_NOALLOC_SCRATCH_BYTES per GPU, held by the library from the first
 *     emg_ctx_create on that GPU until the process ends; no call allocates
 *     or frees device memory, and no HIP graph is instantiated (the cycle
 *     steps are launched directly, opts->use_graph is ignored);
 *   - every problem must already hold its hierarchy: solved (emg_solve or
 *     emg_solve_batch) since its moduli were last set, and for EMG_MIXED
 *     solved once in mixed precision, else EMG_ESTATE.  New face data,
 *     eigenstrain or body force need no allocation;
 *   - a batch whose work lists need more than EMG_NOALLOC_SCRATCH_BYTES
 *     (about 100 lists of the problems of one kind; several hundred small
 *     problems) is rejected with EMG_EINVAL before anything runs;
 *   - calls on one GPU share its array: the call is blocking and holds the
 *     array until it returns, and a call that finds it held by another
 *     thread returns EMG_EBUSY at once (the array keeps the last call's
 *     lists; each call rewrites what it reads). */
#define EMG_NOALLOC_SCRATCH_BYTES ((size_t)8 << 20)
emg_status emg_solve_batch_noalloc(emg_problem **probs, int n, const emg_solve_opts *opts, emg_solve_stats *stats);

/* ---- serving: continuous batching of independent solves ----
 * A server owns a preparation thread and a scheduler thread, each with its own
 * stream.  Submitted requests wait in a FIFO queue; the preparation thread
 * takes them in order once the request's device footprint fits the context's
 * HBM budget (idle resident hierarchies are freed to make room) and builds
 * hierarchy, right-hand side and lift while the GPU runs the current batch;
 * at every cycle boundary the scheduler moves prepared requests into free
 * slots (at most max_slots active), runs one batched launch sequence (as
 * emg_solve_batch) over all active requests for opts->check_every cycles,
 * and retires converged ones:
 * the displacement is copied to u_out and the problem's device memory stays
 * resident for the next request with the same domain.  Requests that arrive
 * while others are on the GPU therefore join the running batch, and each
 * result is bit-identical to its emg_solve result.  Host inputs are copied at
 * submit; with EMG_REQ_DEVICE every array (inputs and u_out) is a device
 * pointer that is borrowed, not copied, and must stay valid and unchanged
 * until the ticket is done.  u_out must stay valid until the ticket is done.
 * Times are seconds on the server's steady clock (emg_server_now).  Ticket
 * records are kept until the server is destroyed.  Calls are thread-safe. */
typedef struct emg_server emg_server;
#define EMG_REQ_DEVICE 1
typedef struct {
  emg_domain dom;
  const double *C, *eps0, *body;   /* arrays as for emg_set_moduli / _eigenstrain / _body_force (eps0, body may be NULL) */
  const double *face[6];           /* face data as for emg_set_face (NULL = 0) */
  double *u_out;                   /* buffer for the displacement (d components, as emg_get_displacement), or NULL */
  int flags;                       /* 0: host arrays; EMG_REQ_DEVICE: device arrays */
} emg_request;
typedef struct {
  int done;
  emg_status status;               /* EMG_OK, EMG_ENOTCONV, EMG_EDIVERGED, or the admission error */
  emg_solve_stats stats;           /* setup_seconds = preparation, solve_seconds = prepared to completion */
  double t_submit, t_admit, t_ready, t_done;   /* queued, preparation started, prepared, result copied out */
} emg_ticket_info;
emg_status emg_server_create(emg_ctx *ctx, int max_slots, const emg_solve_opts *opts, emg_server **out);
emg_status emg_server_submit(emg_server *s, const emg_request *req, uint64_t *ticket);
emg_status emg_server_poll(emg_server *s, uint64_t ticket, emg_ticket_info *info);
emg_status emg_server_wait(emg_server *s, uint64_t ticket, emg_ticket_info *info);
emg_status emg_server_now(emg_server *s, double *t);
/* Finishes every submitted request, then frees the server and its resident hierarchies. */
emg_status emg_server_destroy(emg_server *s);

/* ---- block-structured AMR with reflux-free coarse/fine coupling (Sec. 3.2, App. A) ----
 * Refined level k >= 1 (ratio 2, spacing h_{k-1}/2) is a list of boxes of
 * nodes of its own index space (inclusive bounds, every bound even so box
 * corners fall on coarse nodes; Sec. 1 block-structured hierarchy, Fig.
 * "hierarchy").  Its valid nodes are the union of the boxes; boxes may touch
 * or overlap (shared nodes are simply valid).  Every box grown by two coarse
 * cells must consist of valid nodes of level k-1 (for k = 1: lie inside the
 * base grid, off its boundary, on non-periodic axes).  Level-k fields are
 * laid out over the bounding box [lo, hi] of the list grown by one node per
 * side: extents m[a] = hi[a] - lo[a] + 3, [comp][z][y][x]; nodes of that
 * array that are not valid are ghosts (next to valid nodes) or unused, and
 * input fields must hold finite values there, moduli positive definite
 * (EMG_EINVAL for bounds that break these rules or a bounding array of 2^29
 * or more nodes).  Composite system solved by emg_solve (EMG_FP64: composite
 * cycles in FP64; EMG_MIXED: FP64 state, composite residual, convergence test
 * and update around an FP32 composite correction cycle):
 *   - unknowns: valid nodes of every refined level plus the coarser nodes not
 *     covered by valid nodes of the next level; a covered coarse node takes
 *     the coincident fine value (App. A, phi_c2 = phi_f4);
 *   - fine nodes that are not valid take the bi/trilinear interpolation of
 *     the next coarser level (App. A, phi_f3 = (phi_c1 + phi_c2)/2);
 *   - fine valid rows use the fine operator, uncovered coarse rows the coarse
 *     operator; moduli and eigenstrain of covered coarse nodes are replaced by
 *     the full-weighting average of the finer level (Sec. 1: coarse levels
 *     are updated from fine levels by averaging).
 * The relative residual is the 2-norm over all composite rows.  With a warm
 * start the reference norm is the warm iterate's own residual.  After a solve
 * emg_get_displacement returns the base grid (covered nodes injected) and
 * emg_amr_get_displacement a level's array: valid nodes and their ghosts
 * (interpolated); the cycle only works on the 64 x 4 tiles of the array that
 * hold such nodes, and the other nodes keep what was last written there (0
 * after emg_set_level_boxes). */
typedef struct {
  int64_t lo[3], hi[3];   /* inclusive node box in its level's index space (2D: lo[2] = hi[2] = 0) */
} emg_box;
/* Adds refined level `level` as the union of boxes[0..nbox-1] (copied).
 * Levels are added in order: `level` must be the number of refined levels
 * so far plus one (EMG_ESTATE otherwise); nbox >= 1.  Drops the problem's
 * hierarchy and graphs (moduli of the new level must be set before a solve). */
emg_status emg_set_level_boxes(emg_problem *p, int level, const emg_box *boxes, int nbox);
/* One-box form of emg_set_level_boxes for the next level. */
emg_status emg_amr_add_level(emg_problem *p, const int64_t lo[3], const int64_t hi[3]);
/* Valid-node mask of refined level `level` over its bounding array (1 byte
 * per node, layout [z][y][x]; NULL to skip) and the number of valid nodes. */
emg_status emg_amr_level_valid(emg_problem *p, int level, unsigned char *mask, int64_t *nvalid);
emg_status emg_amr_num_levels(emg_problem *p, int *levels);
emg_status emg_amr_level_shape(emg_problem *p, int level, int64_t m[3]);
emg_status emg_amr_set_moduli(emg_problem *p, int level, const double *C, int on_device);
emg_status emg_amr_set_eigenstrain(emg_problem *p, int level, const double *eps0, int on_device);
emg_status emg_amr_set_body_force(emg_problem *p, int level, const double *b, int on_device);
emg_status emg_amr_get_displacement(emg_problem *p, int level, double *u, int on_device);
emg_status emg_amr_set_displacement(emg_problem *p, int level, const double *u, int on_device);
/* Composite residual of the current state on one level (0 = base grid; rows
 * that are not composite rows are left as computed, callers mask them) into
 * the device buffer r_dev; *norm (if non-NULL) = 2-norm over all composite rows. */
emg_status emg_amr_residual(emg_problem *p, int level, double *r_dev, double *norm);

/* Average duration in milliseconds of one launch of a cycle kernel on the
 * problem's stream: `reps` back-to-back launches in the launch configuration
 * the solve uses are captured into one HIP graph (as the solve's cycles are),
 * replayed once untimed and once between two HIP events.  kernel: 0 = Jacobi
 * sweep, 1 = residual, 2 = interpolation from level+1 onto the level with the
 * correction added, 3 = full-weighting restriction from the level to level+1
 * (fused with level+1's zero-start sweep where the cycle fuses them).
 * EMG_EINVAL for reps < 1, an unknown kernel or a missing coarser level. */
emg_status emg_kernel_time(emg_problem *p, int kernel, int level, int precision, int reps, double *avg_ms);

/* ---- autotuner ----
 * Picks, by measurement instead of the cost model, how the steps of the
 * cycle of Sec. 3.1 are launched on each level; the operations themselves are
 * unchanged (launch configurations, not steps of the method).  For every
 * multigrid level, in `precision` (EMG_FP64: FP64 passes, EMG_MIXED: the FP32
 * ones): the Jacobi sweep with the tile kernel in tiles of 64 x 4, 64 x 2,
 * 128 x 2 and 32 x 8 nodes and, on 3D levels wide enough (at least
 * 64 x 4 interior nodes per plane and 8 planes), with the z-marching pass at
 * every chunk count leaving at least 8 planes per chunk; and, on levels with a
 * coarser one, the restriction from the level and the interpolation onto it in
 * the same four tile shapes.  Each variant is timed as `reps` launches
 * captured into a graph (best of two replays), and the fastest of each kind is
 * recorded in a process-wide table keyed by device architecture, precision,
 * level extents, periodic axes and moduli kind.  Every later plan of any
 * problem with such a level takes the recorded choices (emg_solve; batched
 * and served solves take the z-marching choice and keep 64 x 4 tiles);
 * emg_level_zmarch and emg_level_tiles report them.  All variants compute the
 * same values node by node; the norm partials of a level-0 sweep are summed
 * per tile, so a different tile shape can change the convergence test's
 * last bits (never the iterates).  Levels already in the table are skipped
 * unless `retune` is nonzero.  The problem's recorded solve graphs are
 * dropped (re-recorded at the next solve); graphs of servers already running
 * keep their plans.  If the environment variable EMG_TUNE_CACHE names a file,
 * the table is read from it at first use and rewritten after each call that
 * measured a level: a JSON object of
 * "arch/fp64|fp32/m0xm1xm2/p<mask>[/iso][/r|/i]" -> value, mask bit a set for
 * a periodic axis a; for the stencil pass the value is the chunks per column
 * of the z-marching pass (> 0), 0 for the tile kernel in 64 x 4 tiles, or
 * -1, -2, -3 for the tile kernel in 64 x 2, 128 x 2, 32 x 8 tiles; for the
 * restriction ("/r") and interpolation ("/i") it is the tile shape 0..3 in
 * that order; entries out of range for their level are ignored.  Problems
 * with at least two levels below level 0 of at most 1024 nodes each also get
 * "<level 0 key>/tail" (see emg_tail_levels): the V(2,2) correction on those levels timed
 * as one fused launch and as a launch per pass, the value being their count
 * if fused was faster, else 0.  *tuned (optional) receives the number of
 * levels measured.  EMG_EINVAL for reps
 * outside 1..1000 or when the cache file cannot be written (the table itself
 * is updated). */
emg_status emg_autotune(emg_problem *p, int precision, int reps, int retune, int *tuned);
/* Launch shapes a level uses in `precision`: tile shape of the tile kernel
 * (0 = 64 x 4, 1 = 64 x 2, 2 = 128 x 2, 3 = 32 x 8; 0 when the level runs the
 * z-marching pass), of the restriction from the level and of the
 * interpolation onto it (-1 on the coarsest level).  Outputs may be NULL. */
emg_status emg_level_tiles(emg_problem *p, int level, int precision, int *stencil, int *restriction,
                           int *interpolation);
/* Empties the process-wide table; the EMG_TUNE_CACHE file, if any, is read
 * again at the next lookup. */
emg_status emg_autotune_reset(void);
/* Fused coarse tail (multigrid level sequence, Sec. 3.1): the cycle on the
 * smallest levels -- zero-start sweep, sweeps, residual, restriction, bottom
 * solve, interpolation and sweeps of each of them, in the order the cycle
 * visits them -- can run as ONE launch of one workgroup per problem instead
 * of a launch per pass, with the same values node for node (bit-identical
 * solves).  *levels receives how many levels, counted from the coarsest, the
 * cycles of `precision` (EMG_FP64, EMG_MIXED: the FP32 cycles) fuse that way;
 * 0 (every pass its own launch) unless the table holds an entry
 * "arch/fp64|fp32/m0xm1xm2/p<mask>[/iso]/tail" -> count keyed by level 0
 * (see emg_autotune, which times the fused and the separate launches of the
 * levels below level 0 with at most 1024 nodes each and records the faster;
 * EMG_TUNE_CACHE).  Counts beyond the levels below level 0 are clipped to
 * them.  It applies to emg_solve, batched and served solves; graphs recorded
 * before a change keep their plans. */
emg_status emg_tail_levels(emg_problem *p, int precision, int *levels);

#ifdef __cplusplus
}
#endif
#endif /* EMG_H */
