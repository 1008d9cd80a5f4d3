/*
 * pp.h - C ABI of the MI355X pressure-Poisson tree-code library.
 *
 * The library evaluates the free-space Green's-function solution of the 2-D
 * pressure Poisson equation (Verma et al., "Computing the force distribution on
 * the surface of complex, deforming geometries using vortex methods and
 * Brinkman penalization", Appendix A):
 *
 *     P(t_j) = sum_i G(t_j, s_i) f(s_i) h^2,      G(x, x') = (1/2pi) ln|x - x'|
 *
 * (eq. greenSum with the kernel of eq. green2D) for sources f on a uniform
 * Cartesian grid and arbitrary target points: grid nodes (the full-field
 * evaluation of Sec. 3.3), body-surface points (Sec. 2.3.1) or lifted-surface
 * points (Sec. 2.3.2).  The sum is evaluated with a quadtree and multipole /
 * local expansions (eq. alphaK, eq. pressTruncated, eq. expandedShift) plus a
 * direct near field, all in hand-written HIP kernels for gfx950.
 *
 * Conventions shared by all entry points
 * --------------------------------------
 * - Grid: f is ny*nx doubles, row-major (f[j*nx + i]); node (i, j) lies at
 *   (x0 + (i + 1/2) h, y0 + (j + 1/2) h).  Nodes with f == 0 are skipped.
 *   Limits: 1 <= nx, ny <= 65536 and nx*ny < 2^31.
 * - Root square (grid): anchored at (x0, y0), side 2^k h with 2^k >= max(nx,
 *   ny).  Every target must lie inside it (half-open), else PP_ERR_DOMAIN.
 * - Scattered sources (pp_solve_points): n points (sx, sy) with weights w =
 *   f h^2 given per source, so each source may carry its own cell area (the
 *   paper allows h to vary from source to source).  Sources with w == 0 are
 *   skipped.  The root square is anchored at the lower-left corner of the
 *   bounding box of the weighted sources and the targets, with finest cells
 *   of the power-of-two side u for which 2^15 u first exceeds the box's
 *   extent; no target can lie outside it.
 * - Pointers: every input and output may be host memory or device memory of
 *   the context's device (detected with hipPointerGetAttributes).  The caller
 *   owns all buffers; inputs are only read; p_out (m doubles, the caller's
 *   target order) is written only when the call returns PP_OK.
 * - Streams: work is enqueued on `hip_stream` (a hipStream_t, or NULL for the
 *   default stream) and the call returns after it has completed.
 * - Self-interaction (a target that coincides exactly, in FP64, with a grid
 *   node x0 + (i + 1/2) h; the paper does not treat it): PP_SELF_SKIP drops the
 *   node, PP_SELF_CELLAVG adds w (ln h - kappa) / 2pi, the mean of the kernel
 *   over the node's h x h cell (kappa = 3/2 - pi/4 + ln(2)/2).  Scattered
 *   sources that coincide exactly with a target are dropped (PP_SELF_SKIP is
 *   the only mode there).  In PP_MIXED, a grid target within 2^-20 h of a node
 *   is treated exactly (its FP64 term is restored); scattered points closer
 *   than FP32 resolves (about 1e-7 of their leaf's side) are not, and their
 *   pair is evaluated at that resolution.
 * - Errors: functions never throw; they return a pp_status and leave a message
 *   for pp_last_error().  PP_ERR_DEVICE poisons the context (destroy it).
 * - Threads: a context serves one host thread at a time.
 */
#ifndef PP_H_
#define PP_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pp_ctx pp_ctx;
typedef int32_t pp_status;

enum {
  PP_OK = 0,
  PP_ERR_ARG = -1,     /* null pointer, bad size, non-finite input, bad parameter */
  PP_ERR_DOMAIN = -2,  /* a target lies outside the root square */
  PP_ERR_NOMEM = -3,   /* the solve would exceed the context's device-memory budget */
  PP_ERR_DEVICE = -4,  /* a HIP call failed; the context is unusable */
  PP_ERR_LIMIT = -5,   /* the tree exceeded an internal limit (the largest traversal frontier, cell capacity) */
  PP_ERR_TIMEOUT = -6, /* pp_server_wait: the request did not finish in time (ticket stays valid) */
  PP_ERR_CANCELLED = -7, /* pp_server_wait: the request was cancelled before it started */
  PP_ERR_BUSY = -8     /* pp_server_cancel: the request has already started (or finished) */
};

enum { PP_FP64 = 0, PP_MIXED = 1 };            /* MIXED: P2P and L2P/M2P in FP32 (Kahan), expansions FP64 */
enum { PP_SELF_SKIP = 0, PP_SELF_CELLAVG = 1 };
enum { PP_METHOD_FMM = 0, PP_METHOD_TREECODE = 1 };

/*
 * Parameters of the tree-code (Appendix A):
 *   p         expansion order: p terms after the log term (eq. pressTruncated), 1..20
 *   theta     acceptance: target cell A and source cell B interact through
 *             expansions when (r_A + r_B) < theta * d, r = half-diagonal, d =
 *             centre distance (the paper's "sufficiently large distances");
 *             read as round(1000 theta)/1000, 0 < theta < 1
 *   leaf_max  a cell is split while it holds more than leaf_max sources or
 *             more than leaf_max targets (1..4096)
 *   precision PP_FP64 or PP_MIXED
 *   self_mode PP_SELF_SKIP or PP_SELF_CELLAVG
 *   method    PP_METHOD_FMM (default, 0): multipoles shifted into local
 *             expansions (M2L, L2L, L2P) with the dual-tree acceptance above.
 *             PP_METHOD_TREECODE: the paper's own tree-code - every target
 *             leaf evaluates the multipoles of the groups it accepts directly
 *             at its targets (eq. pressTruncated, M2P; no local expansions),
 *             with acceptance s_B / d < theta, s_B the side of group B and d
 *             the distance from the leaf's square to B's centre.
 */
typedef struct {
  int32_t p;
  double theta;
  int32_t leaf_max;
  int32_t precision;
  int32_t self_mode;
  int32_t method;
} pp_params;

/* Per-solve statistics of the last successful call on a context. */
typedef struct {
  int32_t depth;          /* deepest tree level */
  int32_t ncells;         /* cells in the tree */
  int32_t nsrc_leaves;    /* leaves holding sources */
  int32_t ntgt_leaves;    /* leaves holding targets */
  int64_t nsources;       /* sources with a nonzero weight */
  int64_t ntargets;
  int64_t n_m2l;          /* M2L (cell, cell) pairs; tree-code: M2P (leaf, cell) pairs */
  int64_t n_p2p_lists;    /* P2P (leaf, leaf) pairs */
  int64_t n_p2p_pairs;    /* P2P (target, source) interactions */
  double ms_total;        /* wall time of the call on the host, ms */
  /* GPU time per phase (HIP events on the call's stream), filled only while
   * profiling is enabled with pp_set_profiling; indices PP_PHASE_*. */
  double ms_phase[12];
} pp_stats;

enum {
  PP_PHASE_INGEST = 0,   /* input staging, source weights in Morton order */
  PP_PHASE_SORT = 1,     /* target keys and radix sort */
  PP_PHASE_TREE = 2,     /* quadtree levels */
  PP_PHASE_LISTS = 3,    /* cell lists, interaction lists, near-field work items */
  PP_PHASE_PACK = 4,     /* per-leaf source records and target offsets */
  PP_PHASE_P2M = 5,
  PP_PHASE_M2M = 6,      /* bottom-up recursion, three levels per launch */
  PP_PHASE_M2L = 7,      /* tree-code: M2P */
  PP_PHASE_L2L = 8,      /* final locals: own M2L plus exact shifts of every ancestor's */
  PP_PHASE_L2P = 9,
  PP_PHASE_P2P = 10,
  PP_PHASE_FINALIZE = 11
};

/* Create a context on HIP device `device`.  hbm_budget_bytes bounds the
 * device memory the context may hold (0 = no bound).  *out receives the
 * context; returns PP_ERR_DEVICE if the device cannot be used. */
pp_status pp_create(int32_t device, uint64_t hbm_budget_bytes, pp_ctx** out);
void pp_destroy(pp_ctx* ctx);

/* Tree-code solve (P2M, M2M, M2L, L2L, L2P, P2P) of eq. greenSum for grid
 * sources f at the m targets (tx, ty).  Writes P to p_out[0..m).  A traversal
 * frontier or interaction list that outgrows its working capacity makes the
 * call raise that capacity for the context and repeat the solve by itself;
 * PP_ERR_LIMIT only if the largest frontier capacity (2048 source cells per
 * level on the way down, a stack of 4096 at the target cell) is exceeded. */
pp_status pp_solve_grid(pp_ctx* ctx, int32_t nx, int32_t ny, double x0, double y0, double h, const double* f,
                        int64_t m, const double* tx, const double* ty, const pp_params* params, double* p_out,
                        void* hip_stream);

/* For callers that cannot allocate device memory (code being captured into a
 * HIP graph, tight serving loops, harnesses that forbid allocation): the same
 * solve as pp_solve_grid, with every intermediate array taken from a fixed
 * workspace of 256 MiB that the library holds on each GPU it runs on (a
 * static device array, alive until the process ends), so the call itself
 * allocates nothing.  f, tx, ty and p_out must be device memory (else
 * PP_ERR_ARG; there are no staging copies).  A solve whose arrays do not fit
 * in the workspace returns PP_ERR_NOMEM before anything is enqueued (the 512^2
 * vortex workload with 264,192 targets needs about 80 MiB; grids up to 1024^2
 * with a few thousand targets fit).  All calls on one GPU share the
 * workspace, which keeps the last call's contents: calls that overlap on one
 * GPU (from several threads or contexts) race and must be serialised by the
 * caller.  The call runs on hip_stream alone (no second stream, no graph
 * replay), returns after completion like pp_solve_grid, gives bitwise the
 * same result, and keeps no tree for pp_solve_grid_resident. */
pp_status pp_solve_grid_noalloc(pp_ctx* ctx, int32_t nx, int32_t ny, double x0, double y0, double h,
                                const double* f, int64_t m, const double* tx, const double* ty,
                                const pp_params* params, double* p_out, void* hip_stream);

/* Resident solve: the pressure is recomputed every time step on the same
 * grid (Sec. 2.2: the source f changes with the flow, the grid does not), so
 * the quadtree, its interaction lists and the target sort of the last
 * successful pp_solve_grid on this context are kept and reused.  f (nx*ny,
 * the grid of that call) brings new values; tx, ty (m points, the count of
 * that call) may move as long as each target stays in the finest cell (side
 * h) it was sorted into.  Only the weights, the expansions, the near field
 * and the finalize step run: no ingest, sort, tree build or list build.  f
 * may be zero where it was nonzero (the node keeps its place with weight 0),
 * but must be zero wherever it was zero: both this and the targets' cells are
 * checked on the device, and a mismatch returns PP_ERR_ARG with p_out
 * untouched (the retained tree stays usable).  Parameters, precision and
 * method are those of the retained call.  PP_ERR_ARG also when the last call
 * on the context was not a successful pp_solve_grid (pp_solve_points,
 * pp_direct_*, a failure, and a context without a solve keep no tree).  The
 * result is bitwise that of pp_solve_grid on the same inputs whenever f has
 * the same nonzero nodes. */
pp_status pp_solve_grid_resident(pp_ctx* ctx, const double* f, const double* tx, const double* ty, double* p_out,
                                 void* hip_stream);

/* Several solves of one grid geometry at once (Appendix A's sum for each,
 * eq. greenSum): request r has its own source f[r] (nx*ny), m[r] targets
 * (tx[r], ty[r]) and output p_out[r]; nx, ny, x0, y0, h and params are
 * shared.  The requests are solved as one forest in one set of launches: each
 * request's grid occupies its own cell of a few extra top levels (4^levels >=
 * nreq), cells above that level are always split and no interaction crosses
 * between requests, so each request's tree, lists and arithmetic are those of
 * its lone pp_solve_grid, and p_out[r] is bitwise that solve's result.  For
 * serving many requests of one shape (the launches and their latency are
 * shared).  nreq 1..16 (1 is pp_solve_grid); every pointer device memory
 * (else PP_ERR_ARG); grids of 33 to 65536 nodes a side with the forest at
 * most 65536 nodes wide; multipole method only (PP_ERR_ARG otherwise); a
 * request may have no targets.  Keeps no tree for pp_solve_grid_resident. */
pp_status pp_solve_grid_batch(pp_ctx* ctx, int32_t nreq, int32_t nx, int32_t ny, double x0, double y0, double h,
                              const double* const* f, const int64_t* m, const double* const* tx,
                              const double* const* ty, const pp_params* params, double* const* p_out,
                              void* hip_stream);

/* All-pairs direct sum of eq. greenSum on the GPU (no expansions): the
 * baseline the tree-code is measured against.  Uses params->precision,
 * params->self_mode and params->leaf_max (tiling); p and theta are ignored. */
pp_status pp_direct_grid(pp_ctx* ctx, int32_t nx, int32_t ny, double x0, double y0, double h, const double* f,
                         int64_t m, const double* tx, const double* ty, const pp_params* params, double* p_out,
                         void* hip_stream);

/* Tree-code solve of eq. greenSum for n scattered sources (sx, sy) with
 * weights w (w_i = f_i h_i^2) at the m targets (tx, ty): the same passes as
 * pp_solve_grid.  Writes P to p_out[0..m).  params->self_mode must be
 * PP_SELF_SKIP (else PP_ERR_ARG). */
pp_status pp_solve_points(pp_ctx* ctx, int64_t n, const double* sx, const double* sy, const double* w, int64_t m,
                          const double* tx, const double* ty, const pp_params* params, double* p_out,
                          void* hip_stream);

/* All-pairs direct sum for scattered sources on the GPU (the baseline of
 * pp_solve_points); as pp_direct_grid otherwise. */
pp_status pp_direct_points(pp_ctx* ctx, int64_t n, const double* sx, const double* sy, const double* w, int64_t m,
                           const double* tx, const double* ty, const pp_params* params, double* p_out,
                           void* hip_stream);

/*
 * Pressure forces on body surfaces (Sec. 2.3.1): for every surface panel j
 * with pressure p[j] (e.g. the output of a solve at the panel points), unit
 * outward normal (nx[j], ny[j]) and length ds[j], the pointwise force
 * dF_j = -p_j n_j ds_j (eq. Fpress); for every body s, the panels
 * [seg_start[s], seg_start[s+1]) of one closed surface, the net force
 * F = sum_j dF_j (eq. FpressNet), the drag F . U / |U| along the free stream
 * U = (ux, uy) and the coefficient 2 drag / (rho |U|^2 area) (eq. CdP).
 * seg_start has nseg + 1 entries, starts at 0, ends at m and does not
 * decrease (host memory); the sums are compensated and in a fixed order.
 * dfx/dfy (m doubles, may be NULL) and out (nseg entries) may be host or
 * device memory.  Errors: PP_ERR_ARG for bad sizes, offsets, |U|, rho or area.
 */
typedef struct {
  double fx, fy;  /* net pressure force */
  double drag;    /* F . U / |U| */
  double cd;      /* 2 drag / (rho |U|^2 area) */
} pp_force;
pp_status pp_surface_forces(pp_ctx* ctx, int64_t m, const double* p, const double* nx, const double* ny,
                            const double* ds, int32_t nseg, const int64_t* seg_start, double ux, double uy, double rho,
                            double area, double* dfx, double* dfy, pp_force* out, void* hip_stream);

/*
 * Pressure source from a gridded velocity (eq. PoissonFinal): at every node of
 * the nx x ny grid (spacing h, row-major like f)
 *   f = -rho (grad u^T : grad u) + rho lambda div(chi (u_s - u))
 * with grad u^T : grad u = u_x^2 + 2 u_y v_x + v_y^2.  Derivatives: central
 * differences inside, second-order one-sided differences on the first and last
 * row/column.  chi, us, vs (the smoothed solid indicator and the solid's
 * velocity, node fields) may all be NULL, which drops the penalisation term.
 * f_out (nx*ny) may be host or device memory and can be passed to
 * pp_solve_grid.  Errors: PP_ERR_ARG for bad sizes or h, or non-finite output.
 */
pp_status pp_pressure_source(pp_ctx* ctx, int32_t nx, int32_t ny, double h, const double* u, const double* v,
                             double rho, double lambda, const double* chi, const double* us, const double* vs,
                             double* f_out, void* hip_stream);

/*
 * Viscous forces on body surfaces (Sec. 2.3.2): for every panel j with lifted
 * point (lx[j], ly[j]) (the surface point moved outward along the normal,
 * typically by 2h), unit outward normal (nx[j], ny[j]) and length ds[j], the
 * velocity gradient of the grid node nearest to the lifted point gives
 * D = (grad u + grad u^T)/2 and the force dF_j = 2 mu D n_j ds_j (eq. Fvisc);
 * per body (segments as in pp_surface_forces) the net force (eq. FviscNet),
 * drag and coefficient (eq. CdNu).  The grid is the one of pp_solve_grid
 * (node (i, j) at x0 + (i + 1/2) h); the nearest node of a point is the
 * centre of the cell holding it, clamped to the grid.
 */
pp_status pp_viscous_forces(pp_ctx* ctx, int32_t nx, int32_t ny, double x0, double y0, double h, const double* u,
                            const double* v, int64_t m, const double* lx, const double* ly, const double* pnx,
                            const double* pny, const double* ds, int32_t nseg, const int64_t* seg_start, double mu,
                            double ux, double uy, double rho, double area, double* dfx, double* dfy, pp_force* out,
                            void* hip_stream);

pp_status pp_get_stats(const pp_ctx* ctx, pp_stats* out);

/* GPU timing of later calls: 0 off; 1 HIP events between all phases
 * (ms_phase[]; every phase then runs on the call's stream, one after the
 * other, and launches are not replayed from graphs); 16 + phase (PP_PHASE_*)
 * HIP events around that phase's launches only, on the stream they run on,
 * in the schedule of an untimed call (ms_phase[phase]; the launches of the
 * second segment are issued one by one, and the first segment is replayed
 * from its graph unless the timed phase is in it: ingest, sort or tree);
 * 2 is 16 + PP_PHASE_P2P, the near-field launch.
 * Events add no synchronisation beyond the
 * call's own.  Outside mode 1 the near field runs on a second stream owned by
 * the context, concurrently with the expansions on the call's stream, which
 * waits for it before the finalize step; the mode-2 events are recorded on
 * that second stream.  Repeated calls with device-resident grid input of
 * unchanged shape and pointers replay the launches of their two segments from
 * captured HIP graphs. */
pp_status pp_set_profiling(pp_ctx* ctx, int32_t on);

/*
 * Introspection of the last successful solve on a context, for testing: copy
 * one of its device arrays to host memory.  `what` selects the array (below);
 * dst receives min(capacity, length) elements; *length (may be NULL) receives
 * the full element count.  Element types: int32 unless noted.
 */
enum {
  PP_ARR_SRC_KEY = 0,    /* uint32 Morton key per source, in key order */
  PP_ARR_SRC_INDEX = 1,  /* per source: packed node index i | (j << 16) (grid), caller index (points) */
  PP_ARR_TGT_KEY = 2,    /* uint32 key per target, sorted */
  PP_ARR_TGT_PERM = 3,   /* caller index of each sorted target */
  PP_ARR_CELL_LEVEL = 4,
  PP_ARR_CELL_IX = 5,
  PP_ARR_CELL_IY = 6,
  PP_ARR_CELL_SB = 7,
  PP_ARR_CELL_SE = 8,
  PP_ARR_CELL_TB = 9,
  PP_ARR_CELL_TE = 10,
  PP_ARR_CELL_CHILD = 11, /* first child or -1 */
  PP_ARR_CELL_NCHILD = 12,
  PP_ARR_CELL_PARENT = 13,
  PP_ARR_M2L_OFF = 14,    /* per cell: begin of its M2L source list (tree-code: M2P list of a target leaf) */
  PP_ARR_M2L_CNT = 15,    /* per cell: length */
  PP_ARR_M2L_SRC = 16,
  PP_ARR_P2P_OFF = 17,
  PP_ARR_P2P_CNT = 18,
  PP_ARR_P2P_SRC = 19,
  PP_ARR_MULTIPOLE = 20,  /* double, per cell (p+1) complex: scaled a'_k = a_k / s^k */
  PP_ARR_LOCAL = 21,      /* double, per cell (p+1) complex: scaled L'_l = L_l s^l (not in the tree-code) */
  PP_ARR_FAR = 22,        /* double per sorted target: the far field times 2pi (L2P, or the M2P sum) */
  PP_ARR_NEAR = 23,       /* double [parts][sorted target]: partial sums over near sources of w ln r */
  PP_ARR_LEAF_WNEAR = 24, /* not stored (the near weights are folded into PP_ARR_NEAR): PP_ERR_ARG */
  PP_ARR_TGT_LEAF = 25    /* leaf cell of each sorted target */
};
pp_status pp_debug_copy(const pp_ctx* ctx, int32_t what, void* dst, int64_t capacity, int64_t* length);

const char* pp_status_string(pp_status s);
const char* pp_last_error(const pp_ctx* ctx);

/*
 * Serving: a persistent pool of solve slots fed from a FIFO of requests
 * (continuous batching of independent solves on one GPU).  Each slot owns a
 * context (device buffers stay resident between requests), a HIP stream and a
 * host thread.  The head of the queue is admitted as soon as a slot is free,
 * the estimated device footprints of the requests in flight plus its own fit
 * in hbm_budget_bytes, and their work (grid nodes plus targets) fits in
 * work_budget_points (0 = no bound for either; a request always runs when
 * nothing else is in flight).  The memory counted is that of every slot: the
 * buffers an idle slot keeps resident from its last request, or the larger of
 * those and the footprint of the request a busy slot runs; a slot whose
 * resident buffers leave the total above the budget after a request releases
 * them (so once every request has finished, the slots hold at most the
 * budget).  The work bound keeps large requests from
 * sharing the GPU with each other, which would stretch all of their
 * latencies, while small ones still overlap.  Requests admitted together run
 * concurrently and their kernels overlap on the device.  A request's result
 * is bitwise the result of pp_solve_grid on the same inputs: slots share
 * nothing.
 *
 * Fused launches (max_batch > 1): when a slot admits the head of the queue it
 * also takes, in queue order, up to max_batch - 1 more queued requests of the
 * same shape (nx, ny, x0, y0, h and parameters; multipole method; every input
 * and output in device memory) while the memory bound leaves room, and solves
 * them together with pp_solve_grid_batch: one set of launches for all of them,
 * each result still bitwise its pp_solve_grid result.  The batch counts as its
 * head's work for the work bound (its time grows far more slowly than its
 * work).  Should the
 * batched call fail, its requests are solved one by one, so each gets its own
 * status.  The requests of a batch start and finish together.
 *
 * Ownership: host inputs (f, tx, ty) are copied at submission; device inputs
 * and p_out must stay valid until pp_server_wait has returned for the ticket.
 * All server functions are thread-safe.
 */
typedef struct pp_server pp_server;
typedef struct {
  int32_t device;
  int32_t max_slots;          /* concurrent solves, 1..64 */
  uint64_t hbm_budget_bytes;  /* admission bound on in-flight footprints (0 = none) */
  uint64_t work_budget_points; /* admission bound on in-flight nx*ny + m (0 = none) */
  int32_t max_batch;          /* requests fused into one launch set, 0 or 1 = none, up to 16 */
} pp_server_cfg;
typedef struct {              /* the arguments of pp_solve_grid */
  int32_t nx, ny;
  double x0, y0, h;
  const double* f;
  int64_t m;
  const double* tx;
  const double* ty;
  pp_params params;
  double* p_out;
} pp_request;
typedef struct {
  pp_status status;           /* the solve's own status */
  int32_t slot;               /* slot that ran it */
  double queue_us;            /* submission to start */
  double run_us;              /* start to completion */
  double total_us;            /* submission to completion */
  double start_us, end_us;    /* start and completion, microseconds since pp_server_create */
} pp_ticket_info;

pp_status pp_server_create(const pp_server_cfg* cfg, pp_server** out);
/* Queue one solve; *ticket identifies it for pp_server_wait. */
pp_status pp_server_submit(pp_server* s, const pp_request* req, uint64_t* ticket);
/* Block until the ticket's solve has finished (timeout_us < 0: no limit);
 * returns its status (PP_ERR_TIMEOUT leaves the ticket valid) and releases
 * the ticket; info (may be NULL) receives its timings. */
pp_status pp_server_wait(pp_server* s, uint64_t ticket, int64_t timeout_us, pp_ticket_info* info);
/* Withdraw a request that has not started: returns PP_OK and its wait then
 * returns PP_ERR_CANCELLED (p_out untouched); PP_ERR_BUSY if it has already
 * started or finished (wait for it as usual); PP_ERR_ARG for an unknown
 * ticket. */
pp_status pp_server_cancel(pp_server* s, uint64_t ticket);
/* Finish every queued request, then stop the slots and free their memory. */
pp_status pp_server_destroy(pp_server* s);
const char* pp_server_last_error(const pp_server* s);
/* Device bytes the server's slots hold right now (their resident buffers). */
uint64_t pp_server_device_bytes(pp_server* s);
/* Device bytes a request of this shape may use (the admission estimate). */
uint64_t pp_footprint_estimate(int32_t nx, int32_t ny, int64_t m, int32_t p, int32_t leaf_max);

#ifdef __cplusplus
}
#endif

#endif /* PP_H_ */
