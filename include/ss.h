/*
 * ss.h -- C interface of libss, the MI355X (gfx950) double-double hot path of
 * collective-coordinate optimisation for stealthy hyperuniform point patterns
 * (Morse, Kim, Steinhardt, Torquato, arXiv:2304.09139).
 *
 * Problem (paper, "Definitions"): N points in a periodic hypercubic box of side
 * L in R^d; wavevectors k = 2 pi n / L with integer n and 0 < |k| <= K;
 * n~(k) = sum_j exp(-i k.r_j) (Eq. ntilde), S(k) = |n~(k)|^2 / N
 * (Eq. structurefactor), S_max = max over the exclusion region (Eq. smax), and
 * the energy of Eq. energy with its structure-independent term dropped, whose
 * minimisation drives S(k) -> 0 inside the exclusion region.
 *
 * Conventions used by every entry point:
 *  - Double-double (dd) arrays store a hi plane followed by a lo plane; the
 *    value is hi + lo.
 *  - Positions are FRACTIONAL coordinates u = r / L as double[2][d][N]
 *    (pos[a*N + j] = hi of u_{j,a}, pos[(d + a)*N + j] = lo).  They need not
 *    lie in [0, 1) (the energy is periodic) but must satisfy |u| < 2^20.
 *  - The wavevector set is the half set H(R2) = { n in Z^d : 0 < |n|^2 <= R2,
 *    first nonzero component > 0 }: by the inversion symmetry S(k) = S(-k)
 *    only M of the 2M nonzero vectors in the ball are independent ("Definitions",
 *    the paragraph defining chi).  Its canonical order is ascending |n|^2, ties by
 *    ascending lexicographic order of (n_1, ..., n_d).
 *  - Weights v_k are the dimensionless v~(k) / (eps0 L^d): v = 1 for the
 *    Heaviside potential of the "Simulations" section.  With them
 *        Phi = sum_{n in H} v_n |n~(k_n)|^2
 *    which equals the paper's Phi / eps0 (the full +-k sum of Eq. energy folds
 *    onto the half set).
 *  - n~ outputs are double[4][M] = (C.hi, C.lo, S.hi, S.lo) in canonical
 *    order, with C = sum_j cos(k.r_j), S = sum_j sin(k.r_j), n~ = C - i S.
 *  - Device pointers are caller-owned (e.g. PyTorch tensors); the library
 *    never frees them.  `stream` is a hipStream_t passed as void*; NULL means
 *    the default stream.  Calls marked "async" only enqueue work on `stream`.
 *  - Return codes: SS_OK (0), SS_PENDING (> 0, informative) or a negative
 *    error.  Nothing aborts or throws across this interface.  HIP failures map
 *    to SS_EHIP with detail in ss_last_error(); a fault inside an async launch
 *    surfaces at the next synchronising call.
 *  - Results are bitwise reproducible: every reduction has a fixed order and
 *    launch shapes depend only on (d, N, M).
 */
#ifndef SS_H
#define SS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  SS_OK = 0,
  SS_PENDING = 1,
  SS_EINVAL = -1,    /* invalid argument (sizes, NULL pointers, workspace too small) */
  SS_ENOMEM = -2,    /* device allocation failed                                       */
  SS_EHIP = -3,      /* HIP runtime error                                              */
  SS_ENOTFOUND = -4, /* unknown ticket                                                 */
  SS_ESTATE = -5,    /* call not valid in the current state                            */
  SS_ENUMERIC = -6   /* non-finite value met                                           */
};

typedef struct ss_ctx ss_ctx;

/* A problem instance.  M must equal the size of H(R2) (ss_count).
 * vkind: 0 -> v = 1 (v_dev ignored, may be NULL);
 *        1 -> v = (1 - |k|/K)^2 with K^2 = (R2 + 1/2) (2 pi / L)^2, a weight
 *             table that the caller fills with ss_weights;
 *        2 -> an arbitrary positive caller table v_dev. */
typedef struct {
  int32_t d;     /* 1..4 */
  int64_t N;     /* particles, >= 1 */
  int64_t R2;    /* cutoff: |n|^2 <= R2, i.e. K = 2 pi sqrt(R2) / L */
  int64_t M;     /* |H(R2)| */
  double L;      /* box side, > 0 */
  int32_t vkind; /* see above */
} ss_problem;

/* Create a context on HIP device `device` (the device is made current).  The
 * context owns only its cached wavevector plans and a private stream for
 * building them.  Returns SS_OK and *out, or SS_EINVAL / SS_EHIP. */
int ss_create(int device, ss_ctx** out);

/* Release the context and its plans.  NULL is accepted. */
int ss_destroy(ss_ctx* ctx);

/* Build id of this library: the first 16 hex digits of the SHA-256 of the
 * sources it was compiled from (HIP sources and headers, and this header), so
 * that a caller can check that a binary matches its source tree.  Static
 * string; "unknown" if the build did not define it. */
const char* ss_build_id(void);

/* Static description of a return code. */
const char* ss_strerror(int code);

/* Detail of the last error seen by this context ("" if none); the string lives
 * until the next call on the context. */
const char* ss_last_error(ss_ctx* ctx);

/* Size of the half set H(R2): M.  Host only, pure.  SS_EINVAL for d outside
 * 1..4 or R2 < 1. (The paper's count of M independent constraints,
 * "Definitions", the paragraph defining chi.) */
int ss_count(int d, int64_t R2, int64_t* M);

/* Cutoff from the constraint fraction chi = M / (d (N - 1)) (same paragraph):
 * the largest squared radius R2 that some lattice vector attains and whose
 * count M(R2) does not exceed chi d (N - 1).  Host only, pure.  SS_EINVAL for
 * d outside 1..4, N < 2, chi outside (0, 1/2) (the disordered regime the paper
 * restricts to), or when no shell fits. */
int ss_cutoff(int d, int64_t N, double chi, int64_t* R2, int64_t* M);

/* Enumerate H(R2) in canonical order into n_dev (int32[M][d], device memory of
 * `capacity` vectors) with integer GPU kernels; also caches the plan the
 * energy kernels use for this (d, R2).  Pass n_dev = NULL for a size query.
 * Synchronising.  *M receives |H(R2)|; SS_EINVAL if capacity < M. */
int ss_wavevectors(ss_ctx* ctx, int d, int64_t R2, int32_t* n_dev, int64_t capacity, int64_t* M, void* stream);

/* Fill v_dev (double[2][M], device) with the weights of prob->vkind (0 or 1)
 * for the canonical list n_dev (from ss_wavevectors).  Async. */
int ss_weights(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, double* v_dev, void* stream);

/* Workspace bytes needed by ss_energy_grad (op = 0) or ss_minimize (op = 1)
 * for this problem.  Builds the wavevector plan if needed (synchronising). */
int ss_workspace_size(ss_ctx* ctx, const ss_problem* prob, int op, size_t* bytes);

/* One evaluation of the energy and its gradient (the two O(MN) sums of the
 * "Simulations" section):
 *   phi_dev[2]   <- Phi = sum_{n in H} v_n (C_n^2 + S_n^2)          (Eq. energy)
 *   smax_dev[2]  <- S_max = max_n (C_n^2 + S_n^2) / N (or NULL)      (Eq. smax)
 *   grad_dev     <- dPhi/dr_{j,a} = (4 pi / L) sum_n v_n n_a (S_n c_jn - C_n s_jn)
 *                   as double[2][d][N] (or NULL to skip the gradient pass);
 *                   this is -F_j of Eq. force
 *   nk_dev       <- n~ as double[4][M] in canonical order (or NULL)
 * where c_jn, s_jn = cos, sin of k_n.r_j.  n_dev is the canonical list from
 * ss_wavevectors for (d, R2); v_dev is double[2][M] (see vkind).  ws is device
 * scratch of at least ss_workspace_size(op = 0) bytes (dominated by the phase
 * table, 32 d (R + 1) N bytes with R = floor(sqrt(R2))).  Async; SS_EINVAL on
 * bad sizes, NULL required pointers, a short workspace, or a cutoff whose
 * per-particle table 32 d (R + 1) bytes exceeds 64 KB (d = 1: R > 2047;
 * d = 3: R > 681; d = 4: R > 511; d = 2 has no such limit: from R = 48 on it
 * stages 32 table rows per particle whatever R is). */
int ss_energy_grad(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                   const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev, double* nk_dev,
                   void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * evaluation of ss_energy_grad with the same arguments, layouts, kernels and
 * results bit for bit, minus the workspace -- it runs in the library's own
 * static device array of ss_static_scratch_bytes() bytes (32 MiB; one per GPU,
 * held until the process ends).  It calls no hipMalloc, hipFree or other
 * allocating routine.  The problem must have been prepared beforehand by
 * ss_workspace_size(op = 0) on the same context (that call builds and caches
 * the wavevector plan, schedules and chunk bounds); otherwise SS_ESTATE.
 * SS_ENOMEM (nothing launched) when the problem's workspace,
 * ss_workspace_size(op = 0), exceeds the scratch size.  Every call on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (two streams, two
 * contexts or two threads at once) race and give wrong results: serialise
 * them.  Async, like ss_energy_grad; nothing in the array needs clearing
 * between calls (every value read is written earlier in the same call). */
int ss_energy_grad_static(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                          const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev, double* nk_dev,
                          void* stream);
size_t ss_static_scratch_bytes(void);

/* The same evaluation with the two pair passes in plain FP64 (the first stage
 * of a staged quench; see ss_min_opts.precision).  Same arguments, layouts and
 * errors as ss_energy_grad; every output low word is zero.  Each term of a
 * sum is a product of at most d + 8 (n~ pass) or d + run length (gradient
 * pass) table entries of relative error <= 2^-53, so |C_k error| and
 * |S_k error| are bounded by about (d + 10) N 2^-53. */
int ss_energy_grad_fp64(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                        const double* pos_dev, double* phi_dev, double* smax_dev, double* grad_dev, double* nk_dev,
                        void* ws, size_t ws_bytes, void* stream);

/* Progress lines for long runs (off by default): with seconds > 0, ss_minimize
 * prints its stage, iteration, evaluations, Phi and S_max to stderr at most
 * this often, and ss_minimize_batch the number of configurations still
 * running.  0 turns them off; SS_EINVAL for a negative or non-finite value. */
int ss_set_progress(ss_ctx* ctx, double seconds);

/* Per-kernel timing for measurement (off by default).  `mask` selects the
 * kernels: bit 0 the n~(k) pass (kernel 0), bit 1 the gradient pass (kernel 1),
 * bit 2 the phase-table kernel (kernel 2); 0 turns timing off.  Every launch of
 * a selected kernel (single or batched) is bracketed by hipEvents recorded on
 * the caller's stream.  ss_profile_read synchronises on the recorded events and
 * returns the number of launches, their summed duration in milliseconds and
 * (if work != NULL) the summed work they covered: particle-wavevector pairs
 * M N for the two passes (summed over the configurations listed in a batched
 * launch), table entries d (R + 1) N for the table; reset != 0 then forgets
 * them.  SS_EINVAL for a mask outside 0..7 or an unknown kernel. */
int ss_profile_enable(ss_ctx* ctx, int mask);
int ss_profile_read(ss_ctx* ctx, int kernel, int reset, int64_t* launches, double* total_ms, double* work);

/* Options of the L-BFGS quench (ss_minimize).  The paper quenches with FIRE
 * until Phi is as small as the precision allows ("Simulations" section); this
 * library uses limited-memory BFGS with these rules:
 *  - converged when S_max <= s_floor;
 *  - direction -H g by the two-loop recursion over the last `history` pairs
 *    (1..16), H0 = (s.y / y.y) I of the newest pair; with no pairs, or when
 *    that is not a descent direction, the history is cleared and the step is
 *    -g * min(step_cap * N^(-1/d) / max|g|, 2 Phi / g.g): at most step_cap of
 *    the mean spacing, and no longer than the step to the minimum of the
 *    isotropic quadratic through (Phi, g) with minimum value 0 (a ground state
 *    has Phi = 0);
 *  - Armijo backtracking from alpha = 1 by halving: accept when
 *    Phi(x + alpha p) <= Phi(x) + c1 alpha g.p; after max_halvings halvings a
 *    failure is recorded, the history cleared and x kept;
 *  - a pair (s, y) = (x_new - x, g_new - g) is kept only when s.y > 0;
 *  - stalled when min Phi over the last stall_window iterations exceeds
 *    stall_ratio * min Phi over the stall_window before, or after max_ls_fail
 *    consecutive failures; stops after max_iter iterations in all.
 * Precision (the paper's point is that the last decades of S(k) need more than
 * FP64, "Simulations"): 0 evaluates every energy and gradient in double-double;
 * 1 in plain FP64 (the same sums with FP64 products and additions; S_max below
 * about 1e-25 is then rounding noise); 2 is staged: FP64 until that stage stops
 * (stalled, S_max <= max(s_floor, fp64_floor), its first line-search failure --
 * past that point FP64 rounding noise decides the Armijo test -- or the
 * iteration cap), then
 * double-double from the FP64 stage's positions with the energy and gradient
 * re-evaluated, the stall window restarted and the kept (s, y) pairs carried
 * over (a steepest-descent restart with the capped step is far too long this
 * close to a minimum).  The minimiser's own vectors and dot products are
 * double-double in every mode.
 * Method 1 is FIRE, the paper's minimiser ("Simulations"; Bitzek, Koskinen,
 * Gaehler, Moseler, Gumbsch, PRL 97, 170201 (2006)) with its published
 * parameters: unit masses, F = -g; per step P = F.v; if P > 0 the velocity is
 * mixed, v <- (1 - a) v + a |v| F/|F|, and after more than N_min = 5
 * consecutive such steps dt <- min(1.1 dt, dt_max) and a <- 0.99 a; if P <= 0
 * then dt <- dt / 2, v <- 0, a <- 0.1; then v <- v + dt F, x <- x + dt v.
 * dt0^2 max|g(x0)| = step_cap N^(-1/d), dt_max = 10 dt0.  history, c1,
 * max_halvings and max_ls_fail do not apply; the stopping rules are the same
 * (FIRE's energy is not monotone, so a longer stall_window suits it).
 * fault_iter is a failure-injection hook for testing that a configuration
 * whose energy turns non-finite ends on its own (status 3) while every other
 * configuration of a batch or server runs on unaffected: when > 0, the first
 * trial point of iteration fault_iter (counted from 1 within the running
 * stage) gets a NaN coordinate.  0 disables it; production runs leave it 0. */
typedef struct {
  int32_t history;      /* 1..16 (8 is typical)                 */
  int64_t max_iter;     /* >= 0                                 */
  double s_floor;       /* stated S(k) floor                    */
  int32_t stall_window; /* >= 1, e.g. 50                         */
  double stall_ratio;   /* e.g. 0.99                            */
  double c1;            /* Armijo constant (0, 1)               */
  double step_cap;      /* > 0, e.g. 1e-2                       */
  int32_t max_halvings; /* >= 0                                 */
  int32_t max_ls_fail;  /* >= 1                                 */
  int32_t precision;    /* 0 double-double, 1 FP64, 2 staged    */
  double fp64_floor;    /* >= 0: S_max floor of the FP64 stage (e.g. 1e-24) */
  int32_t method;       /* 0 L-BFGS, 1 FIRE                     */
  int64_t fault_iter;   /* failure injection, 0 = off (see above) */
} ss_min_opts;

/* status: 0 converged (S_max <= s_floor), 1 stalled, 2 iteration cap,
 * 3 non-finite energy (of the last stage run).  iters and evals count every
 * stage; iters_fp64 and evals_fp64 are the parts done in FP64. */
typedef struct {
  int32_t status;
  int64_t iters, evals, grad_evals;
  double phi[2], smax[2];
  double seconds;
  int64_t iters_fp64, evals_fp64;
} ss_min_result;

/* Quench pos_dev (double[2][d][N] fractional coordinates, updated in place and
 * not wrapped into the unit cell) with the rules of ss_min_opts, every vector
 * kept in device memory.  ws must hold ss_workspace_size(op = 1) bytes.
 * Synchronising: returns when the run ends, with *out filled.  Returns SS_OK,
 * SS_ENUMERIC if the energy is not finite (status 3), or an error. */
int ss_minimize(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev, double* pos_dev,
                const ss_min_opts* opts, ss_min_result* out, void* ws, size_t ws_bytes, void* stream);

/* ---- Batches of independent quenches -------------------------------------
 * The paper's production runs are many independent quenches from Poisson
 * starts ("Simulations"); small configurations leave most of the GPU idle and
 * are bound by launch latency when run one at a time.  A batch runs many
 * quenches together: every kernel of an L-BFGS step is ONE launch whose blocks
 * cover all configurations still running; configurations that stop leave the
 * work lists at the next compaction.
 *
 * Tile shapes of the batched launches (particles per n~(k) work unit,
 * wavevectors per gradient block) come from the context's tile table, looked up
 * by (d, N, M) only: a configuration's reduction order -- and therefore its
 * result, bit for bit -- is the same in every batch, alone or mixed with
 * others.  (It may differ in the last bits from ss_minimize's result, whose
 * launch shape is sized to fill the device with one configuration.) */

/* One entry of the tile table: used for problems with d == this d (0 = any d),
 * N <= max_N and M <= max_M; the first matching entry wins, and problems that
 * match none use nk_chunk = max(64, ceil(N / 256)), grad_k = 1024. */
typedef struct {
  int32_t d;
  int64_t max_N, max_M;
  int64_t nk_chunk; /* particles per n~(k) unit, >= 1 (rounded up to the LDS tile) */
  int64_t grad_k;   /* wavevectors per gradient block, >= 1                        */
} ss_tile;

/* Replace the context's tile table by `count` entries (count = 0 clears it).
 * Changing the table changes later batched results in their last bits; set it
 * once, before the first batch.  SS_EINVAL for NULL with count > 0 or an entry
 * with a non-positive size. */
int ss_set_tiles(ss_ctx* ctx, const ss_tile* tiles, int count);

/* The tile shape a problem would get (matching entry or the default). */
int ss_get_tile(ss_ctx* ctx, const ss_problem* prob, ss_tile* out);

/* Workspace bytes for ss_minimize_batch over `count` problems with per-problem
 * options opts[i] (the history length sets the memory of each). */
int ss_batch_workspace_size(ss_ctx* ctx, int count, const ss_problem* probs, const ss_min_opts* opts,
                            size_t* bytes);

/* Quench `count` configurations together.  probs[i], opts[i] as for
 * ss_minimize; pos_dev[i] (double[2][d_i][N_i], fractional) is updated in
 * place; v_dev[i] is the weight table double[2][M_i] for vkind != 0 (v_dev may
 * be NULL when every vkind is 0).  The wavevector sets are built internally
 * from (d_i, R2_i).  ws: ss_batch_workspace_size bytes of device memory.
 * Batched quenches run L-BFGS or FIRE (method 0 or 1, mixed freely) at any
 * precision; a staged configuration switches to double-double on its own when
 * its FP64 stage stops.  A FIRE configuration takes the same steps as under
 * ss_minimize (its time step is derived on the device from max|g(x0)| with the
 * same IEEE operations).
 * Synchronising: returns when every quench has stopped, with out[i] filled;
 * out[i].seconds is the time from the call until the library saw quench i
 * stop.  Returns SS_OK (individual non-finite energies show as status 3), or an
 * error (SS_EINVAL for count < 1, NULL arrays, an invalid problem or options,
 * or a short workspace). */
int ss_minimize_batch(ss_ctx* ctx, int count, const ss_problem* probs, const double* const* v_dev,
                      double* const* pos_dev, const ss_min_opts* opts, ss_min_result* out, void* ws,
                      size_t ws_bytes, void* stream);

/* ---- Serving: continuous batching of quench requests ----------------------
 * A server on a context runs a worker thread with its own HIP stream that
 * keeps one batched minimiser step in flight over every configuration it is
 * running.  Requests wait in submission order; at step boundaries the worker
 * walks the queue and admits every request for which there are a free slot and
 * room in the caller's device arena (first fit), so a request too large for
 * the space free now does not hold back smaller ones behind it -- until 16
 * admissions have overtaken it, after which nothing else is admitted ahead of
 * it.  Admitted requests get their starting evaluation and join the work
 * lists; stopped configurations are copied out and their slot and arena space
 * reused.  Launch shapes come from the tile table by (d, N, M) alone, so a
 * request's result is bitwise the same whatever else is being served and equal
 * to ss_minimize_batch's result for it.  ss_submit and ss_poll may be called
 * from any thread.  Do not change the tile table while a server runs. */

/* One quench request.  The starting positions are copied by ss_submit, or,
 * with pos_host NULL, drawn by ss_uniform_positions from seed (a Poisson start,
 * the paper's initial condition). */
typedef struct {
  int32_t d;               /* 1..4                                                     */
  int64_t N;               /* particles                                                */
  int64_t R2;              /* cutoff |n|^2 <= R2 (ss_cutoff gives it from chi)          */
  double L;                /* box side                                                 */
  int32_t vkind;           /* 0: v = 1; 1: v = (1 - |k|/K)^2, computed by the library   */
  const double* pos_host;  /* double[2][d][N] fractional starting positions (host), or NULL */
  uint64_t seed;           /* the start's seed when pos_host is NULL                   */
  ss_min_opts opts;        /* minimiser options (L-BFGS or FIRE; any precision)        */
} ss_request;

/* Independent uniform fractional positions in [0, 1)^d (the paper's Poisson
 * initial condition, "Simulations") as double[2][d][N] (host): coordinate
 * (a, j) is the exact 106-bit dyadic u = A 2^-53 + B 2^-106, A and B the top 53
 * bits of outputs 2 (a N + j) + 1 and 2 (a N + j) + 2 of the SplitMix64
 * sequence (Steele, Lea and Flood, OOPSLA 2014) started at seed, stored as
 * hi = u rounded to nearest and lo = u - hi (exact).  Host only, pure.
 * SS_EINVAL for d outside 1..4, N < 1 or a NULL output. */
int ss_uniform_positions(int d, int64_t N, uint64_t seed, double* pos_host_out);

/* Start the server.  arena_dev: caller-owned device memory that holds every
 * running configuration's workspace (ss_batch_workspace_size of a single
 * problem gives the order of magnitude; ss_submit refuses a request larger
 * than the whole arena with SS_ENOMEM); max_slots: the most
 * configurations run at once (1..65536).  The server also allocates its
 * descriptor arrays and work lists (a few MB).  SS_ESTATE if one already runs
 * on this context. */
int ss_server_start(ss_ctx* ctx, void* arena_dev, size_t arena_bytes, int max_slots);

/* Queue one request; *ticket identifies it for ss_poll.  Non-blocking apart
 * from building the wavevector plan of a new (d, R2) on first use.  SS_EINVAL
 * for an invalid request (shape, vkind, options, non-finite positions),
 * SS_ENOMEM for a request whose workspace, positions and weights exceed the
 * whole arena (detail in ss_last_error), SS_ESTATE without a running server or
 * while it stops, or the server's error after a failure. */
int ss_submit(ss_ctx* ctx, const ss_request* req, uint64_t* ticket);

/* SS_PENDING while the request is queued or running.  When it is done: fills
 * *out (seconds = from ss_submit until the result was copied out), copies the
 * final positions to pos_host_out (double[2][d][N], if not NULL), forgets the
 * ticket and returns SS_OK (the quench's own outcome is out->status: a
 * configuration whose energy turned non-finite ends with status 3 and the
 * others run on).  SS_ENOTFOUND for an unknown or already collected ticket; a
 * request failed by a server error returns that error. */
int ss_poll(ss_ctx* ctx, uint64_t ticket, ss_min_result* out, double* pos_host_out);

/* Counters of a running server (a snapshot). */
typedef struct {
  int64_t submitted;   /* requests accepted by ss_submit                              */
  int64_t admitted;    /* requests that have started running                           */
  int64_t completed;   /* results ready (collected or not)                             */
  int64_t queued;      /* waiting now                                                  */
  int64_t running;     /* configurations in the batched steps now                      */
  int64_t max_running; /* the most configurations running at once so far               */
  int64_t steps;       /* batched minimiser steps launched                             */
  int64_t overtaking;  /* admissions that went ahead of an older request still waiting */
} ss_server_counters;

/* Fill *out with the server's counters.  SS_ESTATE without a running server. */
int ss_server_stats(ss_ctx* ctx, ss_server_counters* out);

/* Stop accepting requests, finish every queued and running one, stop the
 * worker and release the server; results not yet collected with ss_poll are
 * dropped.  Returns the server's error, if any (SS_OK if none runs).
 * ss_destroy stops a running server. */
int ss_server_stop(ss_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* SS_H */
