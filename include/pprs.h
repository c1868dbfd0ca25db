/*
 * pprs — prefix-scan registration of micrograph series on AMD Instinct MI355X (gfx950).
 *
 * The method (Copik 2017): every frame f_i of a series is aligned to f_0 by an inclusive
 * prefix scan whose binary operator is a pairwise non-rigid registration. Function A (end of
 * the "Image registration for electron microscopy" section) registers a template to a
 * reference by a multilevel gradient flow on -NCC + Dirichlet energy; function B (section
 * "Registration for series of images") composes two deformations and refines the composition
 * with A; the series registration (definition "Image series registration") runs A on all
 * neighbour pairs, then scans them with B (section "Prefix sum for registration problem").
 *
 * Conventions shared by every entry point:
 *  - Frames are float32, row-major [H][W], with H == W and either H == 2^L (pixels; the grid
 *    gets one replicated row and column) or H == 2^L + 1 (grid nodes). 2 <= L <= 10.
 *  - A displacement u = phi - id is float32 [2][H][W]: plane 0 is the x (column) component,
 *    plane 1 the y (row) component, in pixels of the finest level. phi maps reference
 *    coordinates to template coordinates: template(x + u(x)) ~ reference(x).
 *  - Unless a comment says "host", pointers are device pointers in the context's device
 *    memory. The caller owns every array it passes; the library never frees them.
 *  - Calls are ordered on the context's stream and return after the work has completed.
 *  - No call throws; each returns a pprs_status. pprs_last_error() describes the last
 *    non-OK status of the calling thread.
 *  - A context is not thread-safe: calls on one context must not overlap.
 */
#ifndef PPRS_H
#define PPRS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PPRS_OK = 0,
  PPRS_NOT_CONVERGED = 1, /* warning: some level hit iter_max; the result is valid */
  PPRS_EINVAL = -1,       /* bad size, null pointer, bad parameter, constant reference */
  PPRS_ENOMEM = -2,       /* device allocation failed */
  PPRS_EHIP = -3,         /* a HIP runtime call failed */
  PPRS_EINDEX = -4,       /* scan operands do not share their middle frame */
  PPRS_ESTATE = -5,       /* context used after a fatal error, or wrong device */
  PPRS_ENAN = -6          /* a registration produced a non-finite energy */
} pprs_status;

enum {
  PPRS_SCAN_SEQUENTIAL = 0,   /* algorithm "serial" of the Prefix sum chapter */
  PPRS_SCAN_BRENT_KUNG = 1,   /* algorithm "brent_kung" (work-efficient, 2 log2 M - 1 levels) */
  PPRS_SCAN_KOGGE_STONE = 2,  /* algorithm "kogge_stone" (log2 M levels, M log2 M - M + 1 ops) */
  PPRS_SCAN_SKLANSKY = 3,     /* algorithm "sklansky" (log2 M levels, M/2 log2 M ops) */
  PPRS_SCAN_GENERAL = 4,      /* general strategy of the distributed chapter with P workers
                                 (pprs_params.scan_workers): serial scans inside P chunks, a
                                 Brent-Kung scan over the chunk ends, then every other element
                                 of each later chunk combined with the end of the one before */
  PPRS_SCAN_BLELLOCH = 5,     /* algorithm "blelloch": exclusive up/down sweep with the identity
                                 element (2 log2 N levels, 2(N-1) operator applications of which
                                 those with the identity cost nothing) */
  PPRS_SCAN_REDUCE_THEN_SCAN = 6 /* the distributed chapter's alternative strategy with P workers:
                                 each chunk reduced, a scan over the P totals, each chunk
                                 rescanned serially from the total before it */
};

/* Instructions of a scan program (pprs_scan_program). */
enum { PPRS_SCAN_OP_COMBINE = 0, PPRS_SCAN_OP_MOVE = 1, PPRS_SCAN_OP_CLEAR = 2 };

/* NONCONV: some level hit iter_max. NAN: a non-finite energy. FALLBACK: the warm start's
   guess was rejected and the registration ran cold. NET_START: a B application started from
   the network's guess for its pair instead of the composition (lower energy on level 7). */
enum { PPRS_FLAG_NONCONV = 1, PPRS_FLAG_NAN = 2, PPRS_FLAG_FALLBACK = 4, PPRS_FLAG_NET_START = 8 };

#define PPRS_MAX_LEVELS 16

/* Parameters of operator A. The paper leaves lambda, the metric, the line-search details,
   eps and iter_max to the user; pprs_default_params() fills the values this library uses. */
typedef struct {
  int levels;           /* number of grid levels m1 - m0 + 1 (multilevel section); 1..L */
  double lambda;        /* weight of the Dirichlet regulariser (energy E[phi]) */
  double beta;          /* metric A = S1 (x) S1, S1 = M1 + (beta h)^2 K1 (gradient flow) */
  double armijo_sigma;  /* Armijo constant, 0 < sigma < 1 (the paper uses 0.5) */
  int ladder_k;         /* one line-search pass tries 2K+1 steps top * 2^-j, j = 0..2K */
  double step_cap;      /* tau_max = step_cap * h / max|d| (largest step in cells) */
  double tau_min_rel;   /* line search gives up when top < tau_min_rel * tau_max */
  double eps;           /* stop a level when E_k - E_{k+1} < eps (stopping criteria) */
  int iter_max;         /* accepted steps per level (stopping criteria) */
  int scan;             /* PPRS_SCAN_* schedule of the series step */
  int scan_workers;     /* P of PPRS_SCAN_GENERAL and PPRS_SCAN_REDUCE_THEN_SCAN (0:
                           ceil(sqrt(M)); at most M); ignored by the other schedules */
  int warm_start;       /* 1: start neighbour registrations (and, past level 7, B applications)
                           from the context's network (pprs_set_warm_start) where one is set,
                           with the cold start as fallback; 0: cold even where one is set */
  int force_fallback;   /* test switch: 1 rejects every network prediction, so each warm
                           registration takes the fallback (PPRS_FLAG_FALLBACK) */
} pprs_params;

/* Statistics of one A or B application. Level index 0 is the coarsest level. */
typedef struct {
  int iters[PPRS_MAX_LEVELS];   /* accepted gradient-flow steps per level (0 for levels a
                                   warm start skipped) */
  int passes[PPRS_MAX_LEVELS];  /* line-search passes per level */
  double energy;                /* final energy at the finest level */
  double ncc;                   /* final NCC at the finest level */
  int flags;                    /* PPRS_FLAG_* */
  float ms;                     /* time the registration took (ms): the batch's time for the
                                   pair calls; in a series, from the slot-pool poll that started
                                   it to the poll that retired it (host clock) */
} pprs_pair_stats;

typedef struct {
  int n_ops_a;            /* neighbour registrations (preprocessing) */
  int n_ops_b;            /* B applications of the scan */
  int n_scan_levels;      /* batches of mutually independent B applications */
  int flags_or;           /* OR of all pair flags */
  double ms_total;        /* wall time of the call on the device (ms) */
  double ms_prepare;      /* frame pyramids and normalisation */
  double ms_preprocess;   /* the warm start's network predictions (0 when cold) */
  double ms_scan;         /* all A and B applications (they overlap in the slot pool) */
  long long node_steps;   /* sum over ops and levels of accepted steps x grid nodes */
  long long node_passes;  /* sum over ops and levels of line-search passes x grid nodes */
} pprs_series_stats;

typedef struct pprs_ctx pprs_ctx;

/* Fills *p with the library defaults (levels = 4, scan = Brent-Kung). Host pointer. */
void pprs_default_params(pprs_params* p);

/* Creates a context on HIP device `device`. `stream` is a hipStream_t to order work on, or
   NULL for a blocking stream the context creates and owns (ordered with the legacy default
   stream, as work the caller issues there). The stream must not be the legacy default stream
   itself: the series step loop is replayed from a captured graph. The context allocates its
   device workspace lazily and keeps it until pprs_destroy. */
pprs_status pprs_create(pprs_ctx** ctx, int device, void* stream);
void pprs_destroy(pprs_ctx* ctx);

/* Thread-local description of the last non-OK status; never NULL. */
const char* pprs_last_error(void);

/* Workspace of pprs_prefix_register_series (definition "Image series registration": the N-1
   neighbour registrations and the scan's B applications, all in one slot pool) on a context
   with the default pool shape and no warm start: *bytes (host) receives the device memory the
   call keeps in its context for N frames of H x W with these params. Makes no HIP call.
   PPRS_EINVAL for bad sizes or params. The figure is the sum of the context's buffers, each
   sized for this call alone; a context that already holds larger buffers keeps them. */
pprs_status pprs_workspace_query(int N, int H, int W, const pprs_params* params, size_t* bytes);
/* Allocates on ctx the workspace pprs_workspace_query describes (for ctx's pool shape), so that
   a later pprs_prefix_register_series call of that size allocates nothing more. */
pprs_status pprs_reserve_workspace(pprs_ctx* ctx, int N, int H, int W, const pprs_params* params);
/* Device memory (bytes) ctx holds right now in its workspace buffers (host pointer). */
pprs_status pprs_workspace_bytes(pprs_ctx* ctx, size_t* bytes);

/* Function A: registers f_tmpl to f_ref (reference f_i, template f_k: f_k o phi ~ f_i).
   f_ref, f_tmpl: [H][W]. u_init: [2][H][W] initial guess (NULL = identity); it is restricted
   to the coarsest level only, as the multilevel algorithm prescribes. u_out: [2][H][W].
   stats: host pointer, may be NULL. Returns PPRS_NOT_CONVERGED when some level hit iter_max,
   PPRS_EINVAL when the reference is constant on some level. */
pprs_status pprs_register_pair(pprs_ctx* ctx, const float* f_ref, const float* f_tmpl, int H,
                               int W, const float* u_init, float* u_out,
                               const pprs_params* params, pprs_pair_stats* stats);

/* pprs_register_pair for callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the same registration and
   the same result bits, with every working buffer carved from a fixed scratch array in the
   library (PPRS_SCRATCH_BYTES = 40 MiB per device, held until the process ends) instead of the
   context's workspace. It calls no hipMalloc, hipFree or other allocating routine. Frames up to
   512 x 512 (513 x 513 nodes) fit at any level count; larger frames are PPRS_EINVAL. The
   caller still passes ctx (its stream and launch shape), the inputs and the output. All calls
   on one device share that device's scratch and it keeps the last call's contents (whatever
   must start at zero is cleared by the call): calls that overlap on one device, from any
   context or thread, race and must not be made. Synchronous on ctx's stream. */
pprs_status pprs_register_pair_noalloc(pprs_ctx* ctx, const float* f_ref, const float* f_tmpl,
                                       int H, int W, const float* u_init, float* u_out,
                                       const pprs_params* params, pprs_pair_stats* stats);

/* Function A over a batch: for p < P registers frames[tmpl[p]] to frames[ref[p]] (as
   pprs_register_pair with the identity start, or the learned warm start when it is enabled on
   ctx). frames: device [N][H][W]; ref, tmpl: host arrays of P indices in [0, N);
   u_out: device [P][2][H][W] in pixels; stats: host array of P entries or NULL. The pairs run
   as batches of up to 512 concurrent registrations; each result is independent of the batch it
   ran in. Returns PPRS_EINVAL for an index out of range or a constant reference frame,
   PPRS_NOT_CONVERGED when some registration hit iter_max. */
pprs_status pprs_register_pairs(pprs_ctx* ctx, const float* frames, int N, int H, int W,
                                const int* ref, const int* tmpl, int P, float* u_out,
                                const pprs_params* params, pprs_pair_stats* stats);

/* Rigid variant of pprs_register_pairs (definition "Rigid transformation"): phi(x) =
   R(alpha) x + t with R(alpha) the rotation by alpha about the pixel origin (row 0, column 0)
   and t in pixels, found by the same multilevel gradient flow on the three parameters:
   energy -NCC (no regulariser), steepest descent in (alpha, t) with the Armijo ladder and the
   stopping rules of the displacement-field flow, the parameters carried from level to level.
   f_ref[k] is approximated by f_tmpl[k] o phi_k. p_init (host, 3 per pair: alpha, t0, t1;
   NULL = identity) and p_out (host, 3 per pair) use radians and pixels; frames, ref, tmpl and
   stats as for pprs_register_pairs. */
pprs_status pprs_register_pairs_rigid(pprs_ctx* ctx, const float* frames, int N, int H, int W,
                                      const int* ref, const int* tmpl, int P,
                                      const double* p_init, double* p_out,
                                      const pprs_params* params, pprs_pair_stats* stats);

/* Rigid series (definition "Image series registration" with the rigid operator): p_out
   (host, 3 per frame) receives phi_0i as (alpha, t0, t1) in radians and pixels, p_out[0] = 0.
   The N-1 neighbour registrations run as one batch, then each level of the params->scan
   schedule as one batch, every B application started from the composition of its operands'
   maps (alpha = alpha_ij + alpha_jk, t = R(alpha_jk) t_ij + t_jk). stats (host, may be NULL):
   op counts, flags and times (ms_prepare: pyramids; ms_scan: A and B applications). */
pprs_status pprs_prefix_register_series_rigid(pprs_ctx* ctx, const float* frames, int N, int H,
                                              int W, double* p_out, const pprs_params* params,
                                              pprs_series_stats* stats);

/* Composition of deformations (section "Registration for series of images"):
   (phi_jk o phi_ij)(x) = phi_jk(phi_ij(x)), i.e. u_ik(x) = u_ij(x) + u_jk(x + u_ij(x)) with
   u_jk interpolated bilinearly and clamped to the domain. All [2][H][W]; u_ik may alias u_ij
   or u_jk. */
pprs_status pprs_compose_deformations(pprs_ctx* ctx, const float* u_ij, const float* u_jk,
                                      float* u_ik, int H, int W);

/* Series registration (definition "Image series registration"): frames [N][H][W];
   u_out [N][2][H][W] receives u_out[0] = 0 and u_out[i] = phi_{0,i}, so that
   f_i o phi_{0,i} ~ f_0. The neighbour registrations and the scan's B applications run in one
   pool of concurrent registrations (pprs_set_pool), each B application as soon as its inputs
   exist. stats and op_stats are host pointers and
   may be NULL; op_stats receives N-1 A entries followed by the B entries in schedule order,
   so it needs N-1 + n_ops entries (n_ops from pprs_scan_plan for M = N-1: at most 2(N-1) for
   the sequential and Brent-Kung schedules, about (N-1) log2(N-1) for the others). */
pprs_status pprs_prefix_register_series(pprs_ctx* ctx, const float* frames, int N, int H,
                                        int W, float* u_out, const pprs_params* params,
                                        pprs_series_stats* stats, pprs_pair_stats* op_stats);

/* Execution of pprs_prefix_register_series: all its operator applications (the N-1 neighbour
   registrations and every B application) run in one pool of `slots` concurrent registrations
   (0 = 512). An application starts as soon as the applications producing its two inputs have
   finished and a slot is free (in schedule order); the host retires finished registrations and
   starts new ones every `group_steps` steps (0 = 16). Results do not depend on either value.
   Returns PPRS_EINVAL for values out of range (slots > 65536, group_steps > 1024). */
pprs_status pprs_set_pool(pprs_ctx* ctx, int slots, int group_steps);

/* Decision log of later calls on ctx (test and diagnosis): log is a device buffer of rows of
   `cap` bytes (caller-owned, NULL disables). Row r belongs to the call's r-th registration (the
   pair index of pprs_register_pair(s)(_rigid); in a series the N-1 neighbour registrations, then
   the B applications in schedule order, as op_stats; in a multi-series call the pool's op
   order). Byte k of a row is the ladder position J of the registration's k-th accepted step
   (levels in order, coarsest first): the accepted step was top 2^-J, top the first step of that
   iteration's line search (Armijo with widening, section "Gradient flow"); 255 stands for 255
   or more. Steps beyond cap are not logged; the library never clears the buffer. Together with
   the per-level step counts of the stats this is every decision a registration took. */
pprs_status pprs_set_decision_log(pprs_ctx* ctx, unsigned char* log, int cap);

/* Metric solve d = A^-1 G, A = S1 (x) S1 (section "Gradient flow"). EXACT (default): two
   passes of line solves (columns, then rows). WINDOW: one windowed pass per step where beta
   allows it (the LU recurrences of S1 contract so fast that a 64x64 tile plus a halo of 16 or 24
   nodes reproduces the line solves to FP32 resolution; beta up to about 1.4), else EXACT. WINDOW
   moves 16 instead of 40 bytes per node but, VALU-latency bound, runs slower on gfx950. The two
   differ by FP32 rounding only. PPRS_EINVAL for another mode. */
#define PPRS_METRIC_EXACT 0
#define PPRS_METRIC_WINDOW 1
pprs_status pprs_set_metric_solve(pprs_ctx* ctx, int mode);

/* Launch shape of the registration kernels; 0 selects the default. Every value only changes
   how work is spread over the GPU, never a result (each tile's partial sums and each slot's
   decisions are the same for any shape): the autotuner (paper_1712_02533_amd.autotune) times
   candidates and keeps the fastest. */
typedef struct {
  int pool_slots;    /* concurrent registrations of a series (default 512, at most 65536) */
  int pool_group;    /* steps between polls of the slot pool (default 16, at most 1024) */
  int grid_energy;   /* workgroups of the energy kernels (default 8192) */
  int grid_grad;     /* workgroups of the gradient kernel (default 8192) */
  int grid_smooth;   /* workgroups of the metric-solve kernels (default 8192) */
  int grid_prolong;  /* unused: the prolongations run inside the gradient launch */
  int tile_grad;     /* gradient tile shape: 0 = default (64x8), 1 = 64x8, 2 = 128x4,
                        3 = 64x16, 4 = 32x16 nodes */
  int smooth_lines;  /* columns per workgroup of the column solves: 8, 16 (default) or 32 */
  int ladder_rungs;  /* step sizes evaluated per line-search pass: 1, 2, 3, 5 or 7; 0 = one
                        group of 2K+1. The ladder is walked step by step in the same order
                        (groups of 2K+1, a group below tau_min_rel tau_max not begun) whatever
                        the value, so the accepted steps are the same. */
} pprs_tuning;

/* Reads / replaces the launch shape of ctx (host struct). PPRS_EINVAL for out-of-range
   values. */
pprs_status pprs_get_tuning(pprs_ctx* ctx, pprs_tuning* t);
pprs_status pprs_set_tuning(pprs_ctx* ctx, const pprs_tuning* t);

/* Several independent series in one run (segmented scan): series j has N[j] frames of
   side[j] x side[j] (each 2^L or 2^L+1, L may differ between series) at frames[j] (device) and
   receives u_out[j] ([N[j]][2][side][side], as pprs_prefix_register_series). All neighbour
   registrations and B applications of all series share one slot pool (pprs_set_pool), so a
   short series does not wait for a long one and no series waits at another's scan levels.
   params apply to every series; levels (host, S entries, or NULL for params->levels) gives
   each series' level count (<= its L). stats (S entries) and latency_ms (S entries: from the
   start of the call to the series' last result) are host arrays or NULL. Each series' result
   equals its pprs_prefix_register_series result bit for bit. The warm start, when enabled,
   applies to every series with m0 <= 7 <= L. Host arrays: frames, N, side, levels, u_out. */
pprs_status pprs_register_series_batch(pprs_ctx* ctx, int S, const float* const* frames,
                                       const int* N, const int* side, const int* levels,
                                       float* const* u_out, const pprs_params* params,
                                       pprs_series_stats* stats, double* latency_ms);
/* The same segmented scan (one inclusive scan per series, the segmented form of the Prefix
   sum chapter) with per-series heights and widths: series j has N[j] frames of H[j] x W[j]
   (H[j] == W[j] required) and params->levels levels. Equivalent to pprs_register_series_batch
   with side = H, levels = NULL and latency_ms = NULL. Host arrays: frames, N, H, W, u_out. */
pprs_status pprs_prefix_register_series_batch(pprs_ctx* ctx, int S, const float* const* frames,
                                              const int* N, const int* H, const int* W,
                                              float* const* u_out, const pprs_params* params,
                                              pprs_series_stats* stats);

/* Series averaging (Introduction; image series registration): the aligned frames f_i o phi_0i
   averaged into one image, avg(x) = 1/N sum_i f_i(x + u_i(x)), the consumer of the scan output.
   frames [N][H][W] and u [N][2][H][W] (pixels, as pprs_prefix_register_series writes them,
   u[0] = 0) are device pointers; avg [H][W] (device) receives the mean. Frames are sampled
   bilinearly on the pixel grid, positions clamped to [0, W-1] x [0, H-1]; the sum runs in FP64
   in frame order. Any H, W >= 2. Synchronous on the context stream. */
pprs_status pprs_series_average(pprs_ctx* ctx, const float* frames, const float* u, int N, int H,
                                int W, float* avg);

/* The series averaging procedure (Introduction; section "Registration for series of images":
   the scan's result improved by further rounds against the series mean). Each of `passes`
   rounds averages the aligned frames as pprs_series_average does, then registers every frame
   f_i, i >= 1, to that average with operator A (reference = average, template = f_i), started
   from its current u_i restricted to the coarsest level; u_0 is left as given (the identity
   for a scan result), which keeps the result in f_0's coordinates.
   frames [N][H][W] (device, square, side 2^L or 2^L+1) and u [N][2][H][W] (device, pixels,
   read and overwritten in place) as pprs_prefix_register_series writes them; passes >= 0.
   avg (device [H][W], may be NULL) receives the average of the final alignment. stats (host,
   may be NULL) receives passes x (N-1) records, pass-major, frame 1 first. With a decision log
   set, registration r of pass q logs to row q * (N-1) + r. A reference (average) constant on
   some level is PPRS_EINVAL; a non-finite energy is PPRS_ENAN, with u still written.
   Synchronous on the context stream. */
pprs_status pprs_series_average_refine(pprs_ctx* ctx, const float* frames, int N, int H, int W,
                                       float* u, int passes, const pprs_params* params,
                                       float* avg, pprs_pair_stats* stats);

/* Host-only: the scan schedule over M = N-1 elements (PPRS_SCAN_*: the Prefix sum chapter's
   algorithms "serial", "brent_kung", "kogge_stone" and "sklansky", and the distributed
   chapter's general strategy).
   ops (host, capacity `cap` triples) receives (left, right, level) per B application in
   execution order: x[right] <- x[left] (.) x[right], each operand taken as it stands at that
   point of the list. Within a level no op reads an element an earlier op of the level wrote,
   so the ops of a level are independent (Kogge-Stone lists a level right to left for this: its
   ops read the previous level's values, the double buffering of the paper's description).
   Writes the op count and level count. Returns PPRS_EINVAL for bad arguments or a too small
   capacity (then *n_ops holds the needed count). Makes no HIP call. */
pprs_status pprs_scan_plan(int kind, int M, int* ops, int cap, int* n_ops, int* n_levels);
/* pprs_scan_plan with the worker count P of PPRS_SCAN_GENERAL (0: ceil(sqrt(M)); clipped to
   M; P < 0 is PPRS_EINVAL). pprs_scan_plan(kind, ...) is pprs_scan_plan_p(kind, M, 0, ...).
   The Blelloch and reduce-then-scan schedules need scratch elements and the identity and are
   PPRS_EINVAL here: they exist as programs only. */
pprs_status pprs_scan_plan_p(int kind, int M, int P, int* ops, int cap, int* n_ops,
                             int* n_levels);
/* Host-only: any schedule (PPRS_SCAN_*, P as for pprs_scan_plan_p) as a program over
   *n_elems elements (the M scan elements first, then scratch elements that start as the
   identity element). prog (host, capacity `cap` instructions of 5 ints) receives
   (code, a, b, dst, level), executed in list order: PPRS_SCAN_OP_COMBINE x[dst] <- x[a] (.)
   x[b], PPRS_SCAN_OP_MOVE x[dst] <- x[a], PPRS_SCAN_OP_CLEAR x[dst] <- identity. A combine
   with the identity is a copy of the other operand; the others are operator applications
   (*n_reg of them). Combines sharing a level are mutually independent. At the end x[m] holds
   x_0 (.) ... (.) x_m for m < M. The plan schedules are the programs of their combines
   (dst = right). PPRS_EINVAL for bad arguments or a too small capacity (then *n_instr holds
   the needed count). Makes no HIP call. */
pprs_status pprs_scan_program(int kind, int M, int P, int* prog, int cap, int* n_instr,
                              int* n_levels, int* n_elems, int* n_reg);

/* Kernel timing (HIP events around the launches of each kernel kind on the context stream).
   Enabling costs a few microseconds per launch. Kinds are listed by pprs_kernel_name(). */
pprs_status pprs_set_kernel_timing(pprs_ctx* ctx, int enable);
/* Host arrays of `cap` entries: total ms, launch count, algorithmic bytes per kind since the
   last reset. Returns the number of kinds in *n_kinds. */
pprs_status pprs_get_kernel_timing(pprs_ctx* ctx, double* ms, long long* launches,
                                   double* bytes, int cap, int* n_kinds, int reset);
const char* pprs_kernel_name(int kind);

/* ---- Learned warm start (not in the paper: a small BF16 CNN predicts the level-7
   displacement of a frame pair; the gradient flow then refines levels 7..L) ------------------ */

typedef struct pprs_cnn pprs_cnn;

/* Creates the network on `device`, ordered on `stream` (NULL = the default stream), with
   He-normal weights drawn from `seed`. Inputs are [B][128][128][2] float32 (channel 0 the
   reference, 1 the template: level-7 frames normalised to mean 0, sigma 1), outputs
   [B][128][128][2] float32 displacements in level-7 cells (x then y). */
pprs_status pprs_cnn_create(pprs_cnn** cnn, int device, void* stream, unsigned long long seed);
void pprs_cnn_destroy(pprs_cnn* cnn);
const char* pprs_cnn_last_error(void);
/* Number of float32 parameters (FP32 master weights, layer by layer: weights then bias). */
size_t pprs_cnn_param_count(const pprs_cnn* cnn);
/* Host buffers of pprs_cnn_param_count floats. set also resets the optimiser state. */
pprs_status pprs_cnn_set_params(pprs_cnn* cnn, const float* host, size_t count);
pprs_status pprs_cnn_get_params(pprs_cnn* cnn, float* host, size_t count);
/* Loads the parameters from a weights-only blob (host memory, `bytes` long) in the safetensors
   layout: an 8-byte little-endian header length, a JSON header naming each tensor's dtype,
   shape and byte range, then the data. The blob must hold one F32 tensor named "params" (or a
   single F32 tensor) of pprs_cnn_param_count elements, the layout pprs_cnn_get_params returns.
   Nothing in the blob is executed; a malformed header, another dtype or size, or a byte range
   outside the blob is PPRS_EINVAL and leaves the weights unchanged. Resets the optimiser. */
pprs_status pprs_cnn_load(pprs_cnn* cnn, const void* blob, size_t bytes);
/* Inference on B samples (device pointers). */
pprs_status pprs_cnn_forward(pprs_cnn* cnn, const float* x, int B, float* y);
/* Mean squared error over the interior (a border of `margin` pixels left out) and its gradient
   with respect to every parameter; grad_host (host, may be NULL) receives it. */
pprs_status pprs_cnn_gradients(pprs_cnn* cnn, const float* x, const float* target, int B,
                               int margin, double* loss, float* grad_host);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) with learning rate lr on that loss. */
pprs_status pprs_cnn_train_step(pprs_cnn* cnn, const float* x, const float* target, int B,
                                int margin, float lr, double* loss);

/* Network inputs for P frame pairs of a series: frames [N][H][W] as in
   pprs_prefix_register_series (side >= 128); ref and tmpl are host arrays of P frame indices;
   out [P][128][128][2]. */
pprs_status pprs_pair_inputs(pprs_ctx* ctx, const float* frames, int N, int H, int W,
                             const int* ref, const int* tmpl, int P, float* out);
/* Network targets: displacements u [P][2][H][W] (pixels) restricted to level 7 and expressed in
   level-7 cells, out [P][128][128][2]. */
pprs_status pprs_level7_targets(pprs_ctx* ctx, const float* u, int P, int H, int W, float* out);
/* Warm-start modes. REFINE: the prediction, restricted to the coarsest level, replaces the
   identity as the initial guess and every level runs (B applications are unchanged).
   SKIP: the neighbour registrations start on level 7 from the prediction and B applications
   on level 7 from the composition; the coarser levels are skipped. */
#define PPRS_WARM_REFINE 0
#define PPRS_WARM_SKIP 1

/* Enables (cnn != NULL) or disables the warm start for later pprs_prefix_register_series and
   pprs_register_pairs calls on ctx (it needs levels m0 <= 7 <= L). A prediction that is not
   finite or exceeds max_cells level-7 cells is rejected: that pair runs the cold start and its
   stats carry PPRS_FLAG_FALLBACK. ctx keeps the pointer: cnn must outlive its use. Returns
   PPRS_EINVAL for max_cells <= 0, an unknown mode or a network on another device. */
pprs_status pprs_set_warm_start(pprs_ctx* ctx, pprs_cnn* cnn, double max_cells, int mode);
/* Restricts the warm start to series whose side is 2^L (or 2^L + 1) for the bits L set in
   level_mask (default: all), e.g. the sides the network was trained on. */
pprs_status pprs_set_warm_sides(pprs_ctx* ctx, unsigned level_mask);

#ifdef __cplusplus
}
#endif

#endif /* PPRS_H */
