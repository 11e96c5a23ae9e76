/*
 * opf.h - C ABI of the MI355X (gfx950) proximal message-passing solver for
 * contingency-constrained DC optimal power flow.
 *
 * Method: Degleris, El Gamal, Rajagopal, "GPU Accelerated Security
 * Constrained Optimal Power Flow" (arXiv 2410.17203).  The problem is the
 * contingency-constrained OPF of Section 2.3 on the device-node model of
 * Section 2; the iteration is the message-passing form of ADMM of Section
 * 3.2 with the stopping rule of Section 3.3 (eq. converge) and the adaptive
 * penalty of Section 3.5.
 *
 * Conventions for every function:
 *   - the return value is an opf_status; nothing is thrown and nothing
 *     exits across this boundary; opf_last_error() describes a failure;
 *   - all host arrays passed in are owned by the caller and only read
 *     during the call (they are copied);
 *   - device memory is never allocated by the library: the caller passes
 *     one workspace (any device allocation, e.g. a PyTorch tensor) whose
 *     size opf_workspace_size() reports; the library borrows it until
 *     opf_destroy(); the one exception is the fixed 64 MiB array per GPU
 *     behind opf_load_network_static, part of the library's image;
 *   - all device work is enqueued on the stream given in opf_options and
 *     is asynchronous unless a function says it synchronises;
 *   - a context is not thread-safe; use one context per stream.  Distinct
 *     contexts may be driven from distinct host threads at once (graph
 *     capture is thread-local; the only global state is the per-thread
 *     text of opf_last_error(NULL) and the fixed array's bookkeeping,
 *     which is locked).
 */
#ifndef OPF_H
#define OPF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct opf_ctx opf_ctx;

typedef enum {
  OPF_OK = 0,
  OPF_NOT_CONVERGED = 1,   /* informational: max_iter reached first      */
  OPF_E_INVALID = -1,      /* bad argument or bad network data           */
  OPF_E_OOM = -2,          /* workspace smaller than required            */
  OPF_E_HIP = -3,          /* a HIP runtime call failed                  */
  OPF_E_STATE = -4,        /* call out of order (e.g. iterate before load) */
  OPF_E_NUMERIC = -5       /* a residual became NaN or infinite          */
} opf_status;

typedef enum { OPF_F64 = 0, OPF_F32 = 1, OPF_BF16 = 2 } opf_dtype;

/* Solver options.  Defaults (opf_default_options) follow Section 5.2:
 * rho_p = rho_theta = 1, mu = 2, gamma = 1.1 every 10 iterations, no
 * over-relaxation; 10 inner iterations for time-coupled devices (Section 4.5). */
typedef struct {
  int32_t state_dtype;        /* OPF_F64 or OPF_F32: storage and arithmetic of the
                                 iterate; norms and the objective are always FP64 */
  int32_t dual_dtype;         /* storage of the line phase duals: equal to
                                 state_dtype, or OPF_BF16 with an F32 state      */
  double rho_p, rho_theta;    /* initial penalties (Section 3.2)                 */
  double mu, gamma;           /* adaptive penalty rule (Section 3.5)             */
  int32_t adapt_every;        /* iterations between penalty updates; 0 = fixed   */
  double eps;                 /* tolerance of eq. converge on the RMS residuals  */
  int32_t eps_relative;       /* 1: eps is scaled by the RMS load demand         */
  int32_t max_iter, min_iter; /* iteration limits of opf_solve                   */
  int32_t block_iters;        /* iterations per captured graph block in opf_solve */
  int32_t check_every;        /* residuals every check_every iterations; must
                                 divide adapt_every                              */
  int32_t inner_iters;        /* inner ADMM iterations of the time-coupled prox  */
  double inner_omega_scale;   /* inner penalty omega = scale * (K+1) rho_p       */
  int32_t polish_fp64;        /* F32 state: opf_solve switches the iterate to
                                 FP64 once the residual is within polish_factor
                                 of the tolerance                                */
  double polish_factor;       /* [1.2] switch point, as a multiple of eps        */
  int32_t use_graphs;         /* 1: opf_solve replays captured graph blocks      */
  void* hip_stream;           /* hipStream_t for all work; NULL = null stream    */
  int32_t sweep_tiles;        /* sweep over clusters of consecutive nodes
                                 (-1 default, or 1) whenever every node has
                                 at most 128 lines and 128 devices, else node
                                 rows; 0: node rows always */
} opf_options;

/* Fills *opt with the defaults above (F64 state, eps = 1e-3 relative,
 * max_iter 10000, block_iters 50, check_every 1, polish on at 1.2 eps,
 * graphs on). */
void opf_default_options(opf_options* opt);

/* One network (Section 2): nodes 0..N-1, T periods, K contingencies.
 * Line l joins terminal 1 at node line_from[l] to terminal 2 at line_to[l];
 * its flow into the to node is susceptance * (phase_from - phase_to)
 * (Section 2.1, AC line).  Contingency k in 1..K zeroes the capacity and
 * susceptance of line outage[k-1] (Section 2.3, N-1 example); an outage of
 * -1 leaves the network unchanged.  Per-period arrays are row-major
 * [device][t].  Loads store demand d >= 0 and inject -d.  gen_ramp[g] <= 0
 * or infinite means no ramp limit; otherwise |p_{t+1} - p_t| <= gen_ramp[g]
 * for T > 1.  Battery parameters are power P, duration (energy = dur * P),
 * charge efficiency eta in (0, 1] and discharge cost alpha >= 0 (Section
 * 2.1, battery).  Every node needs at least one terminal.  Host arrays,
 * caller-owned, copied by opf_load_network.
 * line_kind (optional, NULL = every line is an AC line): 0 = AC line, 1 = DC
 * link (HVDC line, Section 2.1): p1 + p2 = 0 and |p2| <= cap with no phase
 * relation between its terminals, so its susceptance is ignored.  Its prox
 * takes the clipped midpoint (z2 - z1)/2 of the two power targets as the
 * flow and leaves both phases at their targets; an outaged DC link carries
 * no power.
 * General per-contingency line parameters (optional, Section 2.3: in
 * contingency k the lines may take parameters x_kl other than the base ones):
 * entry i gives line chg_line[i] the susceptance chg_sus[i] and capacity
 * chg_cap[i] in contingency chg_k[i] (1..K).  sus = 0 takes an AC line out
 * (no power, both phases free: a second outage of an N-k contingency); sus > 0
 * with any cap >= 0 models emergency ratings or switched series devices; for a
 * DC link only the capacity applies.  A (contingency, line) pair appears at
 * most once and never repeats that contingency's outage[] line.  n_chg = 0
 * (the arrays may be NULL): the N-1 outages only.
 * The adjoint (opf_tape_forward, opf_adjoint) covers DC links and changes:
 * the derivative with respect to line_cap[l] collects the contingencies in
 * which line l keeps its own capacity (not those a change rerates or where
 * it is out). */
typedef struct {
  int32_t N, T, K;
  int32_t L;
  const int32_t *line_from, *line_to;
  const double *line_sus, *line_cap;      /* sus > 0 (AC lines), cap >= 0    */
  const int32_t* outage;                  /* K entries, distinct or -1       */
  int32_t G;
  const int32_t* gen_node;
  const double *gen_c2, *gen_c1;          /* c2 >= 0; c2 = 0 is a linear cost, and
                                             pmin < pmax <= 0 with c1 = the
                                             curtailment cost is a curtailable
                                             load (Section 2.1)               */
  const double *gen_pmin, *gen_pmax;      /* G*T, pmin <= pmax               */
  const double* gen_ramp;                 /* G                               */
  int32_t D;
  const int32_t* load_node;
  const double* load_d;                   /* D*T                             */
  int32_t B;
  const int32_t* bat_node;
  const double *bat_P, *bat_dur, *bat_eta, *bat_alpha;
  const int32_t* line_kind;               /* L entries of 0 or 1, or NULL    */
  int32_t n_chg;                          /* per-contingency changes         */
  const int32_t *chg_k, *chg_line;
  const double *chg_sus, *chg_cap;
} opf_network;

/* Residual record of one iteration (Section 3.3).  Norms are 2-norms over
 * all terminal copies of all contingencies and periods; rms_* divide by
 * sqrt(2 J T (K+1)); dual norms include the penalty factor. */
typedef struct {
  int64_t iter;                 /* iterations completed                      */
  double primal_p, primal_theta; /* ||pbar||, ||theta tilde||                */
  double dual_p, dual_theta;    /* rho_p ||d ptilde||, rho_theta ||d thetabar|| */
  double rms_primal, rms_dual;
  double threshold;             /* effective eps                             */
  double objective;             /* sum of generator and battery costs        */
  double rho_p, rho_theta;      /* penalties used by this iteration          */
  int32_t converged;
  int32_t precision;            /* opf_dtype of the iterate                  */
} opf_resid;

/* Creates a context.  *out receives the handle; opt is copied. */
opf_status opf_create(const opf_options* opt, opf_ctx** out);

/* Device bytes the workspace must provide for net (validates net). */
opf_status opf_workspace_size(opf_ctx* ctx, const opf_network* net, size_t* bytes);

/* Validates and copies the network into the workspace (d_workspace: device
 * pointer, 256-byte aligned, at least opf_workspace_size bytes) and resets
 * the iterate to the all-zero start of Section 3.4.  Synchronises the
 * stream.  Invalid data returns OPF_E_INVALID and leaves ctx unchanged.
 * Before anything is changed, the tables derived from the network (see
 * opf_check_network) are bounds-checked on the host. */
opf_status opf_load_network(opf_ctx* ctx, const opf_network* net,
                            void* d_workspace, size_t bytes);

/* Host-only check of a network, with no device and no context: the data
 * checks of opf_load_network under opt (NULL: opf_default_options), then
 * every index of the tables the kernels read through, against the range
 * each kernel assumes: the node CSR over line terminals (the per-terminal
 * incidence of Section 4.3: each terminal's line, end and far node) and
 * over devices, the node clusters of the tiled sweep with their line
 * tables and per-terminal line slots, and the ramp generator, DC link and
 * per-contingency change indices.  opf_load_network and opf_load_batch run the same check.
 * tiled (may be NULL) receives 1 when the clusters of the tiled sweep exist
 * (no node has more lines or devices than a cluster holds), else 0.
 * Returns OPF_OK or OPF_E_INVALID, the reason in opf_last_error(NULL) (kept
 * per thread). */
opf_status opf_check_network(const opf_network* net, const opf_options* opt, int32_t* tiled);

/* For callers that cannot allocate device memory (code under stream
 * capture, tight serving loops, harnesses that forbid allocation): as
 * opf_load_network, but the workspace is a fixed array of 64 MiB
 * (67,108,864 bytes) that the library holds on each GPU it runs on until
 * the process ends, so the caller allocates nothing.  The call itself
 * allocates no device or pinned memory (the context's pinned readback
 * buffers come from opf_create).  Networks whose opf_workspace_size exceeds
 * 64 MiB return OPF_E_OOM and leave ctx unchanged; invalid data returns
 * OPF_E_INVALID.  One context per GPU holds the array at a time: a later
 * opf_load_network_static on the same device, from any context, waits for
 * the holder's stream, takes the array over and leaves the previous holder
 * unloaded (its calls then return OPF_E_STATE).  Calls of two contexts on
 * one GPU that overlap in time race on the array.  The array keeps the
 * last instance's contents; the load clears what must start at zero.
 * Zero-copy views (opf_state_layout offsets) are relative to the array and
 * not usable from the caller's memory.  A later opf_load_network or
 * opf_load_batch on the context releases the array.  Synchronises. */
opf_status opf_load_network_static(opf_ctx* ctx, const opf_network* net);

/* Batched form (several independent instances of uneven size in one context;
 * the paper solves its planning scenarios as one batch in Section 5.6): the
 * workspace holds all of them and every phase of an iteration is one launch
 * over a work list spanning all instances.  Each instance keeps its own penalties, counters
 * and convergence flag; converged instances are skipped.  FP64 polishing is
 * not applied to batches.  Instance indices follow the order of nets. */
opf_status opf_workspace_size_batch(opf_ctx* ctx, const opf_network* nets, int32_t count,
                                    size_t* bytes);
opf_status opf_load_batch(opf_ctx* ctx, const opf_network* nets, int32_t count,
                          void* d_workspace, size_t bytes);

/* Number of loaded instances (0 before a load). */
opf_status opf_num_instances(opf_ctx* ctx, int32_t* count);

/* Resets every instance to the all-zero start and the initial penalties. */
opf_status opf_reset(opf_ctx* ctx);

/* Enqueues n_iters message-passing iterations (Section 3.2 steps 1-3 plus
 * residuals and the adaptive penalty).  Asynchronous.  Iterations after
 * convergence or max_iter are skipped on the device. */
opf_status opf_iterate(opf_ctx* ctx, int32_t n_iters);

/* Iterates until eq. converge holds (for every instance) or max_iter;
 * synchronises.  Returns OPF_OK or OPF_NOT_CONVERGED and instance 0's last
 * residual record in *out.  In a batch, each instance stops on its own; at
 * each block of block_iters iterations the stopped instances leave the work
 * lists (their iterates stay as they stopped), which are whole again when
 * opf_solve returns. */
opf_status opf_solve(opf_ctx* ctx, opf_resid* out);

/* Synchronises the stream and returns the last residual record (of
 * instance 0, or of instance i for the _i form). */
opf_status opf_residuals(opf_ctx* ctx, opf_resid* out);
opf_status opf_residuals_i(opf_ctx* ctx, int32_t instance, opf_resid* out);

/* Copies up to max records of the residual history (oldest first, at most
 * the last 4096 iterations) into out; *n receives the count.  Synchronises. */
opf_status opf_residual_history(opf_ctx* ctx, opf_resid* out, int32_t max, int32_t* n);
opf_status opf_residual_history_i(opf_ctx* ctx, int32_t instance, opf_resid* out, int32_t max,
                                  int32_t* n);

/* Fields of the iterate in the paper's layout (Section 4.1), FP64. */
typedef enum {
  OPF_FIELD_P = 0,      /* line flow p2 into the to node    [K+1][L][T] */
  OPF_FIELD_TH1 = 1,    /* line phase at terminal 1         [K+1][L][T] */
  OPF_FIELD_TH2 = 2,    /* line phase at terminal 2         [K+1][L][T] */
  OPF_FIELD_V1 = 3,     /* scaled phase dual, terminal 1    [K+1][L][T] */
  OPF_FIELD_V2 = 4,     /* scaled phase dual, terminal 2    [K+1][L][T] */
  OPF_FIELD_U = 5,      /* scaled power dual (node-constant) [K+1][N][T] */
  OPF_FIELD_PBAR = 6,   /* node average power               [K+1][N][T] */
  OPF_FIELD_THBAR = 7,  /* node average phase               [K+1][N][T] */
  OPF_FIELD_PNC = 8,    /* generator, load, battery power   [G+D+B][T]  */
  OPF_FIELD_THNC = 9,   /* their phases                     [G+D+B][T]  */
  OPF_FIELD_VNC = 10    /* their phase duals averaged over k [G+D+B][T] */
} opf_field;

/* Number of doubles in a field (of instance 0, or of instance i). */
opf_status opf_field_size(opf_ctx* ctx, int32_t field, size_t* count);
opf_status opf_field_size_i(opf_ctx* ctx, int32_t instance, int32_t field, size_t* count);

/* Writes one field of the current iterate, as FP64 in the layout above,
 * to the device buffer d_dst (count doubles).  Enqueued on the stream. */
opf_status opf_get_field(opf_ctx* ctx, int32_t field, double* d_dst, size_t count);
opf_status opf_get_field_i(opf_ctx* ctx, int32_t instance, int32_t field, double* d_dst,
                           size_t count);

/* Enables (1) or disables (0) per-kernel HIP-event timing of subsequent
 * opf_iterate calls; enabling clears the accumulated times. */
opf_status opf_set_timing(opf_ctx* ctx, int32_t enable);

/* Kernel classes timed by opf_set_timing. */
typedef enum {
  OPF_KERNEL_DEVICES = 0,   /* generator, load, battery prox (step 2)   */
  OPF_KERNEL_SWEEP = 1,     /* line prox, node averages, price update
                               (steps 1 and 3, fused)                   */
  OPF_KERNEL_FINALIZE = 2,  /* residual norms, stopping, penalty        */
  OPF_KERNEL_RESCALE = 3,   /* dual rescale after a penalty change      */
  OPF_KERNEL_COUNT = 4
} opf_kernel;

/* Synchronises and returns, per kernel class, the summed milliseconds and
 * the launch count since timing was enabled (arrays of OPF_KERNEL_COUNT). */
opf_status opf_kernel_times(opf_ctx* ctx, double* ms, int64_t* launches);

/* Algorithmic device bytes one launch of a kernel class moves for the
 * loaded network and current precision (used for roofline reporting). */
opf_status opf_kernel_bytes(opf_ctx* ctx, int32_t kernel, double* bytes);

/* Launch configuration chosen by opf_autotune. */
typedef struct {
  int32_t lanes_shift;   /* lanes per (period, node) row: natural count << shift */
  double grid_factor;    /* sweep grid as a multiple of the resident blocks     */
  double ms_per_iter;    /* measured time of one iteration with this choice     */
  int32_t from_cache;    /* 1 if read from cache_path instead of measured       */
  int32_t tiled;         /* sweep over node clusters: 1 on, 0 node rows, -1 by size */
  int32_t tile_groups;   /* period groups per work item of the tiled sweep (a
                            group is the periods that share one pass: several
                            where one pass holds all of a period's
                            contingencies, else one)                         */
} opf_tuning;

/* Times `trials` iterations for each candidate launch configuration of the
 * loaded instance(s), for one instance or a batch: the node-row sweep with
 * lanes per row halved/natural/doubled x sweep grid 0.5/1/2 times the
 * resident blocks, and, where every instance has clusters, the tiled sweep
 * with 1, 2, 4 or 8 period groups per work item x grid 0.5/1/2 (untuned
 * defaults: 1 for one instance, 4 for a batch); keeps the
 * fastest and resets the iterate to the zero start.  With cache_path
 * non-NULL, a result for the same device, precision and instance shapes is
 * read from that text file (one line per result: key, lanes shift, grid
 * factor, tiled, groups, ms) instead of being measured, and new results
 * are appended to it.  Synchronises. */
opf_status opf_autotune(opf_ctx* ctx, int32_t trials, const char* cache_path, opf_tuning* out);

/* ---- The iterate: layout, export and import (warm start, Section 3.4) ------ */

/* Where the current iterate of one instance lives in the workspace (byte
 * offsets from the workspace start; valid until the next iteration, which
 * flips the double buffer).  Line arrays P (flow at the to end), Tm (mean of
 * the two terminal phases), V1, V2 (scaled phase duals before this
 * iteration's update) are [T][chunk][L][w] and node arrays U (scaled price),
 * W (= pbar + U) and TB (thetabar) are [T][chunk][N][w]: the K+1
 * contingencies, padded to Kpp (a multiple of 4), are split into chunks of
 * `chunk` (32), chunk c holding contingencies c*chunk .. c*chunk + w - 1 with
 * w = min(chunk, Kpp - c*chunk), so element (t, i, k) is at
 * (t * Kpp + c*chunk) * count + i * w + (k - c*chunk), c = k / chunk.  Td ([T][Kpp])
 * is the half phase difference of each contingency's outaged line; Hd
 * ([T][chunk][Ldc][w], the chunked layout over the Ldc DC links in line
 * order) holds the half phase difference (theta1 - theta2)/2 of every DC
 * link, whose Tm is the mean phase as for AC lines; Tz ([T][Zc]) that of the
 * Zc lines taken out by changes (sus = 0), in the order of the change list;
 * device
 * arrays pnc, thnc, vbar (contingency mean of the phase duals) are
 * [G+D+B][T].  Element types: state_dtype for all but V1, V2 (dual_dtype).
 * Synchronises. */
typedef struct {
  int32_t N, T, K, Kpp, L, Jnc;
  int32_t state_dtype, dual_dtype;
  int32_t chunk;          /* contingencies per chunk */
  size_t P, Tm, V1, V2, Td, U, W, TB, pnc, thnc, vbar;
  int32_t Ldc;            /* DC links */
  size_t Hd;
  int32_t Zc;             /* lines taken out by changes */
  size_t Tz;
} opf_layout;
opf_status opf_state_layout(opf_ctx* ctx, int32_t instance, opf_layout* out);

/* Bytes of an exported iterate (single instance, FP32 or FP64 duals). */
opf_status opf_state_size(opf_ctx* ctx, size_t* bytes);

/* Copies the whole iterate (line, node and device state, inner ADMM state of
 * ramp generators and batteries) and the current penalties into dst (host
 * or device memory, >= opf_state_size bytes).  Synchronises. */
opf_status opf_get_state(opf_ctx* ctx, void* dst, size_t bytes);

/* Warm start (Section 3.4): replaces the iterate with one exported by
 * opf_get_state from a network of the same structure (the same sizes, line
 * ends and kinds, outages, changed pairs and device nodes; the data, e.g.
 * loads, costs or capacities, may differ), continues with its penalties, and
 * restarts the iteration count at 0.  The message-passing form needs scaled
 * prices with u constant over each node's terminals and v summing to zero at
 * each node: the first holds by construction (one price per node), the
 * second for any iterate of a run on the same structure, which a
 * fingerprint in the blob enforces.  The exported precision must be one
 * this context holds.  Rejects foreign or mismatched blobs with
 * OPF_E_INVALID before changing anything.  Synchronises. */
opf_status opf_set_state(opf_ctx* ctx, const void* src, size_t bytes);

/* ---- Derivatives through unrolled iterations (Section 4.4, sensitivities
 * of Section 5.5) ------------------------------------------------------------
 * The iteration map is piecewise linear in the iterate and in the data, so
 * the derivative of the iterate after n iterations with respect to the load
 * demand, the line capacities and the generator upper limits is a product of
 * per-iteration Jacobians.  The library computes its transpose-vector product
 * (reverse mode) with hand-written kernels: the forward run stores the
 * penalty schedule (held fixed, as a constant of the map) and checkpoints
 * of the iterate every checkpoint_every iterations; the reverse pass
 * recomputes each segment from its checkpoint, keeping every iterate of the
 * segment, and walks it backwards.  At a clip whose argument equals a bound
 * the derivative passes the argument through.  One instance, FP64 or FP32
 * iterate with FP32 or FP64 duals (not BF16), inner_iters <= 32. */

/* Bytes of device memory the tape of an n_iters run needs, for the loaded
 * network and the active precision: ceil(n/C) checkpoints, C - 1 segment
 * snapshots and the final iterate (iterate snapshots), the penalty history,
 * the clip masks of every time-coupled prox of every iteration (two 32-bit
 * words per bound, lane and slot of each ramp generator and battery), and
 * the adjoint arrays.  C = 1 keeps every iterate: the adjoint then recomputes
 * nothing. */
opf_status opf_tape_workspace_size(opf_ctx* ctx, int32_t n_iters, int32_t checkpoint_every,
                                   size_t* bytes);

/* Resets the iterate to the zero start and runs exactly n_iters iterations
 * (no stop on convergence or max_iter; the adaptive penalty runs as
 * configured), recording the tape in d_tape (caller-owned device memory,
 * 256-byte aligned, >= opf_tape_workspace_size bytes, borrowed until the next
 * opf_tape_forward, opf_load_network or opf_destroy).  Afterwards the iterate,
 * residuals and fields are those after n_iters iterations.  Synchronises. */
opf_status opf_tape_forward(opf_ctx* ctx, int32_t n_iters, int32_t checkpoint_every,
                            void* d_tape, size_t bytes);

/* As opf_tape_forward, but continuing from the current iterate (e.g. after
 * opf_set_state: the warm-started solves of gradient-based planning, Section
 * 5.6) and stopping by the options' rule (eps) once at least min_iters and
 * at most max_iters iterations have run; the iterations run are the tape and
 * their count is written to *n_run.  The iterate it starts from is a
 * constant of the derivative.  d_tape must hold opf_tape_workspace_size(ctx,
 * max_iters, checkpoint_every) bytes.  Synchronises. */
opf_status opf_tape_forward_warm(opf_ctx* ctx, int32_t min_iters, int32_t max_iters,
                                 int32_t checkpoint_every, void* d_tape, size_t bytes,
                                 int32_t* n_run);

/* Reverse pass over the recorded run.  Cotangent: d_cot_power (device,
 * [G+D+B][T] doubles, generator/load/battery order, or NULL for zero) on the
 * final device powers, plus cot_objective times the objective of the final
 * iterate (generator cost + battery alpha * discharge).  Writes (device,
 * doubles; any may be NULL): d_grad_load [D][T], derivative with respect to
 * the load demand d; d_grad_cap [L], with respect to the line capacities;
 * d_grad_pmax [G][T], with respect to the generator upper limits.  The
 * iterate is left as opf_tape_forward left it.  Synchronises. */
opf_status opf_adjoint(opf_ctx* ctx, const double* d_cot_power, double cot_objective,
                       double* d_grad_load, double* d_grad_cap, double* d_grad_pmax);

/* Text of the last failure on ctx (or of opf_create when ctx is NULL). */
const char* opf_last_error(opf_ctx* ctx);

/* Releases host resources and captured graphs; the workspace is the
 * caller's to free afterwards.  Synchronises the stream. */
void opf_destroy(opf_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* OPF_H */
