// ss_min.h -- device-resident minimiser state and the per-configuration
// descriptors of the batched launches (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ss_internal.h"

namespace ss {

constexpr int kMaxHistory = 16;
constexpr int kMaxWindow = 256;
constexpr int kDotBlocks = 120;
constexpr int kMaxDots = 2 + 2 * kMaxHistory;  // 34
constexpr int kMaxComb = 1 + 2 * kMaxHistory;  // 33

// control state of one quench (device memory)
struct MinState {
  int32_t running;    // 1 while the quench continues; every kernel of a tick reads it
  int32_t status;     // 0 converged, 1 stalled, 2 iteration cap, 3 non-finite (valid once running == 0)
  int32_t phase;      // 0: a new direction is needed; 1: a trial step is pending
  int32_t new_dir;    // 1 when this tick computed a new direction
  int32_t accepted;   // 1 when this tick accepted its trial
  int32_t halvings, ls_fail, k, spare;
  int32_t slot[kMaxHistory];  // history slots, oldest first
  int32_t ncoef;
  int32_t coef_vec[kMaxComb];  // 0: g, 1 + s: S[s], kMaxHistory + 2 + s: Y[s]
  int64_t iter, evals;
  double alpha;
  double f[2], smax[2], ft[2], smaxt[2], gp[2];
  double coef[kMaxComb][2];
  double SY[kMaxHistory][kMaxHistory][2];  // s_i . y_j for i <= j (upper triangle R)
  double YY[kMaxHistory][kMaxHistory][2];
  double dir_dots[kMaxDots][2];    // s_i.g (k), y_i.g (k), g.g, max|g|
  double trial_dots[kMaxDots][2];  // s.y, y.y, s_i.y (k), y.y_i (k) of the fresh pair
  double fhist[2 * kMaxWindow][2];
  // FIRE (method 1): time step, its cap, the mixing parameter, consecutive P > 0 steps
  double fdt, fdt_max, fa;
  int32_t npos, fire_reset;
  double fcv[2], fcg[2];  // this step's velocity mixing coefficients
  int64_t fault_iter;     // > 0: the trial of this iteration gets a NaN (failure injection)
};

struct MinParams {
  int32_t m, W, max_halvings, max_ls_fail;
  int64_t max_iter;
  double s_floor, stall_ratio, c1, step;  // step = step_cap * N^(-1/d)
  int64_t fault_iter;                     // failure injection (ss_min_opts), 0 = off
  int32_t method;                         // 0 L-BFGS, 1 FIRE
};

// the vectors of one quench
struct VecSet {
  double* x;  // positions (the caller's buffer)
  double* g;
  double* xt;
  double* gt;
  double* p;
  double* S[kMaxHistory + 1];
  double* Y[kMaxHistory + 1];
};

// One block of a batched launch: configuration `slot`, block `idx` of that
// configuration's own grid for the kernel (flattened).
struct BUnit {
  int32_t slot;
  int32_t idx;
};

// What the batched energy/gradient kernels need of one configuration.
struct EvalSlot {
  int32_t d, R1, Q, pt;
  int64_t N, M, nsegs, combine_blocks, pblocks;
  double L;
  const Span* segs;
  const NkUnit* units;
  const int32_t* rows_of;
  const int32_t* k_of_slot;
  const Span* runs;
  const int32_t* chunk_begin;
  const int32_t* canon_of_lex;
  const double* v;  // weights [2][M] canonical, or nullptr for v = 1
  SlotOffsets so;
  double* tab;
  double* part;
  double* csw;
  double* gpart;
  double* blk;
  const double* pos[2];    // evaluation points: the iterate x and the trial xt
  double* grad[2];         // their gradients g and gt (fractional coordinates)
  double* phi;             // Phi and S_max of the iterate (the starting evaluation)
  double* smax;
  const int32_t* running;  // the minimiser's running word
  // the tiled d = 2 n(k) pass (nk2 != 0), in both precisions, instead of the
  // piece pass above
  int32_t nk2, R, t2_nrows;
  int64_t t2_chunk;
  const int32_t* t2_tiles;
  const int32_t* t2_lexinfo;
  const int32_t* t2_rows_of;
  const int32_t* t2_ident;
};

// What the batched minimiser kernels need of one configuration.
struct MinSlot {
  VecSet V;
  MinState* S;
  MinParams P;
  double* partial;  // [kMaxDots][dot_blocks][2]
  const double* eblk;  // per-block energy partials of the trial evaluation
  int64_t neblk;
  int64_t nv;
  int32_t dot_blocks;
  int32_t keep;  // the start keeps the kept (s, y) pairs (a change of precision)
};

// per-configuration status gathered for the host after every batched step
struct SlotFlags {
  int32_t running, status;
  int64_t iter, evals;
};

}  // namespace ss
