// ss_lbfgs.hip -- device-resident L-BFGS quench of the stealthy energy.
//
// The paper quenches with FIRE ("Simulations" section) until Phi reaches the
// smallest value the precision allows; this library minimises with L-BFGS and
// an Armijo backtracking line search.  Everything lives on the device: the
// positions, gradients and the (s, y) history as double-double [2][d N] planes,
// and the minimiser's control state (iteration, line-search step, history
// products, stopping tests) in a small struct in device memory.  One "tick" is a
// fixed sequence of launches that advances the state machine by one trial
// evaluation; the host enqueues ticks a few ahead and polls a status word copied
// to pinned memory, so no blocking synchronisation sits inside the loop.
//
// Rules (the CPU oracle's minimiser implements the same rules independently):
//  * converged when S_max <= s_floor;
//  * direction p = -H g, H the L-BFGS matrix of the kept pairs with
//    H0 = (s.y / y.y) I of the newest pair, evaluated with the compact
//    representation of Byrd, Nocedal & Schnabel (Math. Prog. 63, 1994,
//    Thm 2.2), algebraically identical to the two-loop recursion of Nocedal &
//    Wright (Alg. 7.4) that the oracle uses; when the history is empty or
//    g.p >= 0, the history is cleared and
//    p = -g min(step_cap N^(-1/d) / max|g|, 2 Phi / g.g): at most step_cap of the
//    mean spacing, and no longer than the step to the minimum (value 0, a
//    ground state) of the isotropic quadratic through (Phi, g);
//  * Armijo backtracking from alpha = 1 by halving, accept when
//    Phi(x + alpha p) <= Phi(x) + c1 alpha g.p; after max_halvings halvings a
//    failure is recorded, the history cleared and x kept;
//  * a pair (s, y) = (x_new - x, g_new - g) is kept only when s.y > 0, the
//    oldest being dropped beyond `history` pairs;
//  * stalled when min Phi over the last W iterations exceeds stall_ratio x min
//    Phi over the W before, or after max_ls_fail consecutive failures; stops
//    after max_iter iterations.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <stdio.h>

#include <chrono>
#include <vector>

#include "ss.h"
#include "ss_dd.h"
#include "ss_internal.h"
#include "ss_min.h"
#include "ss_reduce.h"

namespace ss {

int prepare(ss_ctx* ctx, const ss_problem* p, Plan** pl, LaunchCfg* cfg);
int energy_grad_impl(ss_ctx* ctx, const ss_problem* p, Plan* pl, const LaunchCfg& c, const double* v_dev,
                     const double* pos, double* phi, double* smax, double* grad, double* nk, char* ws,
                     hipStream_t st, double* kmax, const int* active, bool fp64);

__device__ __forceinline__ dd ld(const double* a) { return dd{a[0], a[1]}; }
__device__ __forceinline__ void st(double* a, dd v) {
  a[0] = v.h;
  a[1] = v.l;
}
__device__ __forceinline__ dd shfl_xor_dd(dd v, int m) {
  return dd{__shfl_xor(v.h, m, 64), __shfl_xor(v.l, m, 64)};
}
__device__ __forceinline__ dd shfl_dd(dd v, int src) { return dd{__shfl(v.h, src, 64), __shfl(v.l, src, 64)}; }

__device__ __forceinline__ const double* vec_of(const VecSet& V, int code) {
  if (code == 0) return V.g;
  if (code <= kMaxHistory + 1) return V.S[code - 1];
  return V.Y[code - kMaxHistory - 2];
}

__device__ __forceinline__ dd vload(const double* p, int64_t nv, int64_t i) { return dd{p[i], p[nv + i]}; }

// ---------------------------------------------------------------------------
// the direction (run by the one block that finishes the direction products, on
// its LDS copy of the state; wave 0 works, row i on lane i < k).  Compact form
// with H0 = gamma I:
//   H g = gamma g + S top - gamma Y z,  R z = u,  R^T top = D z + gamma (Y^T Y z - w)
// with u = S^T g, w = Y^T g, R the upper triangle of S^T Y and D its diagonal.
// The triangular solves run column by column; the loops run over the k kept
// pairs only (short code: the kernel is a single block, so its time is mostly
// instruction fetch when unrolled over the maximum history).
// ---------------------------------------------------------------------------
__device__ void direction_logic(MinState& S, const MinParams& P, int i) {
  if (i >= 64) return;
  const int k = S.k;
  const dd gg = ld(S.dir_dots[2 * k]);
  const dd gmax = ld(S.dir_dots[2 * k + 1]);
  bool use_sd = (k == 0);
  dd gp{0.0, 0.0};
  if (!use_sd) {
    const bool mine = i < k;
    const dd u = mine ? ld(S.dir_dots[i]) : dd{0.0, 0.0};
    const dd w = mine ? ld(S.dir_dots[k + i]) : dd{0.0, 0.0};
    const dd gamma = dd_div(ld(S.SY[k - 1][k - 1]), ld(S.YY[k - 1][k - 1]));
    const dd diag = mine ? ld(S.SY[i][i]) : dd{1.0, 0.0};
    const dd rdiag = dd_div(dd{1.0, 0.0}, diag);  // all lanes at once, off the serial chain
    // back substitution R z = u (rows i < j updated with z_j)
    dd acc = u, zi{0.0, 0.0};
#pragma unroll 1
    for (int j = k - 1; j >= 0; --j) {
      if (i == j) zi = dd_mul(acc, rdiag);
      const dd zj = shfl_dd(zi, j);
      if (i < j) acc = dd_sub(acc, dd_mul(ld(S.SY[i][j]), zj));
    }
    // rhs_i = D_i z_i + gamma (sum_j YY_ij z_j - w_i)
    dd t{0.0, 0.0};
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
      const dd zj = shfl_dd(zi, j);
      if (mine) t = dd_add(t, dd_mul(ld(S.YY[i][j]), zj));
    }
    const dd rhs = dd_add(dd_mul(diag, zi), dd_mul(gamma, dd_sub(t, w)));
    // forward substitution R^T top = rhs (rows i > j updated with top_j)
    dd topi{0.0, 0.0};
    acc = rhs;
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
      if (i == j) topi = dd_mul(acc, rdiag);
      const dd tj = shfl_dd(topi, j);
      if (i > j && mine) acc = dd_sub(acc, dd_mul(ld(S.SY[j][i]), tj));
    }
    const dd cs = dd_neg(topi);       // on S[slot_i]
    const dd cy = dd_mul(gamma, zi);  // on Y[slot_i]
    if (mine) {
      st(S.coef[1 + i], cs);
      st(S.coef[1 + k + i], cy);
      S.coef_vec[1 + i] = 1 + S.slot[i];
      S.coef_vec[1 + k + i] = kMaxHistory + 2 + S.slot[i];
    }
    // g.p = sum coef * (vector . g) in a fixed order
    gp = dd_mul(dd_neg(gamma), gg);
#pragma unroll 1
    for (int j = 0; j < k; ++j) {
      gp = dd_add(gp, dd_mul(shfl_dd(cs, j), ld(S.dir_dots[j])));
      gp = dd_add(gp, dd_mul(shfl_dd(cy, j), ld(S.dir_dots[k + j])));
    }
    if (i == 0) {
      st(S.coef[0], dd_neg(gamma));
      S.coef_vec[0] = 0;
    }
    if (!(gp.h < 0.0 || (gp.h == 0.0 && gp.l < 0.0))) use_sd = true;
  }
  if (i != 0) return;
  if (use_sd) {
    S.k = 0;
    if (gmax.h == 0.0) {  // stationary point
      S.status = 0;
      S.running = 0;
      S.new_dir = 0;
      return;
    }
    // at most step_cap of the mean spacing, and at most 2 Phi / g.g: the energy's
    // minimum is 0, and there the line along -g meets the minimum of the
    // isotropic quadratic through (Phi, g)
    dd scale = dd_div(dd{P.step, 0.0}, gmax);
    const dd polyak = dd_div(dd_mul_d(ld(S.f), 2.0), gg);
    if (dd_less(polyak, scale)) scale = polyak;
    if (scale.h == 0.0) {  // Phi = 0: a ground state
      S.status = 0;
      S.running = 0;
      S.new_dir = 0;
      return;
    }
    st(S.coef[0], dd_neg(scale));
    S.coef_vec[0] = 0;
    S.ncoef = 1;
    gp = dd_neg(dd_mul(scale, gg));
  } else {
    S.ncoef = 1 + 2 * k;
  }
  st(S.gp, gp);
  S.alpha = 1.0;
  S.halvings = 0;
  S.phase = 1;
  S.new_dir = 1;
  // the candidate pair goes to a slot no kept pair uses
  int spare = 0;
  for (;; ++spare) {
    bool used = false;
    for (int h = 0; h < S.k; ++h) used |= (S.slot[h] == spare);
    if (!used) break;
  }
  S.spare = spare;
}

// p <- sum_c coef_c v_c (accurate dd sums in c order) when a new direction was
// made this tick; then xt <- x + alpha p (alpha a power of two)
__device__ __forceinline__ void step_body(const VecSet& V, const MinState* S_, int64_t nv, int64_t bx) {
  const MinState& S = *S_;
  if (!S.running) return;
  __shared__ double s_ch[kMaxComb], s_cl[kMaxComb];
  __shared__ const double* s_v[kMaxComb];
  const int nd = S.new_dir;
  const int nc = S.ncoef;
  if (nd && threadIdx.x < nc) {
    s_ch[threadIdx.x] = S.coef[threadIdx.x][0];
    s_cl[threadIdx.x] = S.coef[threadIdx.x][1];
    s_v[threadIdx.x] = vec_of(V, S.coef_vec[threadIdx.x]);
  }
  __syncthreads();
  const int64_t i = bx * kThreads + threadIdx.x;
  if (i >= nv) return;
  dd p;
  if (nd) {
    dd acc{0.0, 0.0};
    for (int c = 0; c < nc; ++c) acc = dd_add(acc, dd_mul(dd{s_ch[c], s_cl[c]}, vload(s_v[c], nv, i)));
    V.p[i] = acc.h;
    V.p[nv + i] = acc.l;
    p = acc;
  } else {
    p = vload(V.p, nv, i);
  }
  const double a = S.alpha;
  dd r = dd_add(vload(V.x, nv, i), dd{a * p.h, a * p.l});
  // failure injection: the first trial of iteration fault_iter gets a NaN
  if (i == 0 && S.fault_iter > 0 && S.iter + 1 == S.fault_iter && S.halvings == 0) r.h = __builtin_nan("");
  V.xt[i] = r.h;
  V.xt[nv + i] = r.l;
}

__global__ void __launch_bounds__(kThreads) k_step(VecSet V, const MinState* S_, int64_t nv) {
  step_body(V, S_, nv, blockIdx.x);
}

// gradient with respect to the fractional coordinates: g <- L * dPhi/dr
__global__ void __launch_bounds__(kThreads) k_times_L(double* __restrict__ g, int64_t nv, double L,
                                                      const int* __restrict__ active) {
  if (active && *active == 0) return;
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nv) return;
  const dd r = dd_mul_d(dd{g[i], g[nv + i]}, L);
  g[i] = r.h;
  g[nv + i] = r.l;
}

// start-of-iteration tests (the top of the loop in the rules above) for
// iteration `it` with energy f and S_max smax; all 64 lanes of one wave call it
// (they scan the stall window in parallel), lane 0 writes the state
__device__ void top_of_iteration(MinState& S, const MinParams& P, int lane, int64_t it, dd f, dd smax) {
  const int W = P.W;
  int status = -1;
  if (!(smax.h > P.s_floor || (smax.h == P.s_floor && smax.l > 0.0))) status = 0;
  else if (it >= P.max_iter) status = 2;
  else if (it >= 2 * (int64_t)W) {
    dd recent = f, older{INFINITY, 0.0};
    for (int64_t q = it - 2 * W + 1 + lane; q < it; q += 64) {
      const dd v = ld(S.fhist[q % (2 * W)]);
      if (q > it - W) {
        if (dd_less(v, recent)) recent = v;
      } else if (dd_less(v, older)) {
        older = v;
      }
    }
    for (int m = 32; m > 0; m >>= 1) {
      const dd r = shfl_xor_dd(recent, m), o = shfl_xor_dd(older, m);
      if (dd_less(r, recent)) recent = r;
      if (dd_less(o, older)) older = o;
    }
    if (dd_less(dd_mul_d(older, P.stall_ratio), recent)) status = 1;
  }
  if (lane == 0) {
    st(S.fhist[it % (2 * W)], f);
    if (status >= 0) {
      S.status = status;
      S.running = 0;
    }
  }
}

// after the starting evaluation (f, smax set): finite check and the tests
// keep != 0: the kept (s, y) pairs survive (a change of evaluation precision)
__device__ __forceinline__ void init_body(MinState* S_, const MinParams& P, int keep) {
  MinState& S = *S_;
  const int lane = threadIdx.x;
  if (lane == 0) {
    S.iter = 0;
    S.evals = 1;
    if (!keep) S.k = 0;
    S.phase = 0;
    S.new_dir = 0;
    S.accepted = 0;
    S.ls_fail = 0;
    S.halvings = 0;
    S.spare = 0;
    S.alpha = 1.0;
    S.running = 1;
    S.status = 2;
    S.fault_iter = P.fault_iter;
  }
  const dd f = ld(S.f), smax = ld(S.smax);  // written by the previous kernel
  if (!isfinite(f.h)) {
    if (lane == 0) {
      S.status = 3;
      S.running = 0;
    }
    return;
  }
  top_of_iteration(S, P, lane, 0, f, smax);
}

__global__ void __launch_bounds__(64) k_init(MinState* S_, MinParams P, int keep) { init_body(S_, P, keep); }

// the Armijo test and its consequences (run by the one block that finishes the trial
// products; all threads call it for the barriers, wave 0 does the work).  Lane 0
// takes the decisions and hands them to the other lanes through LDS.
__device__ void decide_logic(MinState& S, const MinParams& P, int i) {
  __shared__ int s_push, s_drop, s_acc, s_top, s_run;
  __shared__ long long s_it;
  __shared__ double s_f[2], s_sm[2];
  const int k = S.k;
  if (i == 0) {
    S.evals += 1;
    const dd f = ld(S.f), ft = ld(S.ft);
    const double alpha = S.alpha;
    const dd bound = dd_add(f, dd_mul(dd_mul_d(dd{alpha, 0.0}, P.c1), ld(S.gp)));
    int push = 0, drop = 0, acc = 0, top = 0, run = 1;
    int64_t it = S.iter;
    dd fn = f, smn = ld(S.smax);
    if (!dd_less(bound, ft)) {  // accepted
      acc = 1;
      S.ls_fail = 0;
      if (S.trial_dots[0][0] > 0.0) {
        push = 1;
        drop = (k == P.m) ? 1 : 0;
      }
      fn = ft;
      smn = ld(S.smaxt);
      st(S.f, fn);
      st(S.smax, smn);
      it += 1;
      S.iter = it;
      S.phase = 0;
      top = 1;
      if (!isfinite(fn.h)) {
        S.status = 3;
        S.running = 0;
        run = 0;
        top = 0;
      }
    } else {
      S.alpha = alpha * 0.5;
      const int h = S.halvings + 1;
      S.halvings = h;
      if (h > P.max_halvings) {  // line-search failure: keep x, clear the history
        const int lf = S.ls_fail + 1;
        S.ls_fail = lf;
        S.k = 0;
        it += 1;
        S.iter = it;
        S.phase = 0;
        top = 1;
        if (lf >= P.max_ls_fail) {
          st(S.fhist[it % (2 * P.W)], fn);
          S.status = 1;
          S.running = 0;
          run = 0;
          top = 0;
        }
      }
    }
    S.accepted = acc;
    s_push = push;
    s_drop = drop;
    s_acc = acc;
    s_top = top;
    s_run = run;
    s_it = it;
    s_f[0] = fn.h;
    s_f[1] = fn.l;
    s_sm[0] = smn.h;
    s_sm[1] = smn.l;
  }
  __syncthreads();
  if (s_push) {
    // drop the oldest pair when full, then append the fresh pair as the newest
    // column of the upper triangle of S^T Y and row/column of Y^T Y
    const int first = s_drop;
    const int kept = k - first;
    const bool mine = i < k;
    const dd colsy = mine ? ld(S.trial_dots[2 + i]) : dd{0.0, 0.0};
    const dd colyy = mine ? ld(S.trial_dots[2 + k + i]) : dd{0.0, 0.0};
    if (first) {
      // shift both matrices up and left by one: thread (r, c) moves element
      // (r, c), 1 <= r, c < k, to (r - 1, c - 1)
      static_assert(kMaxHistory * kMaxHistory <= kThreads, "one thread per matrix element");
      const int r = i / kMaxHistory, c = i % kMaxHistory;
      const bool mv = i < kMaxHistory * kMaxHistory && r >= 1 && c >= 1 && r < k && c < k;
      const dd esy = mv ? ld(S.SY[r][c]) : dd{0.0, 0.0};
      const dd eyy = mv ? ld(S.YY[r][c]) : dd{0.0, 0.0};
      __syncthreads();
      if (mv) {
        st(S.SY[r - 1][c - 1], esy);
        st(S.YY[r - 1][c - 1], eyy);
      }
    }
    __syncthreads();
    if (i >= first && mine) {
      st(S.SY[i - first][kept], colsy);
      st(S.YY[i - first][kept], colyy);
      st(S.YY[kept][i - first], colyy);
    }
    if (i == 0) {
      st(S.SY[kept][kept], ld(S.trial_dots[0]));
      st(S.YY[kept][kept], ld(S.trial_dots[1]));
      for (int h = first; h < k; ++h) S.slot[h - first] = S.slot[h];
      S.slot[kept] = S.spare;
      S.k = kept + 1;
    }
  }
  __syncthreads();
  if (i >= 64) return;
  if (s_top && s_run) top_of_iteration(S, P, i, s_it, dd{s_f[0], s_f[1]}, dd{s_sm[0], s_sm[1]});
}

// ---------------------------------------------------------------------------
// fixed-order multi-dot products.  Block (x, q) reduces element range x of
// product q (strided sequential sums per lane, xor butterfly per wave, waves in
// order) into one partial; k_dots_final sums the partials in range order.
// mode 0: direction products (operands from the history); mode 1: the trial
// pair s = xt - x, y = gt - g (computed on the fly; blocks of product 0 also
// write it to S[spare], Y[spare]) against the history.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void dots_body(const VecSet& V, MinState* S_, int mode, int64_t nv,
                                          double* __restrict__ partial, int bx, int q, int G) {
  MinState& S = *S_;
  if (!S.running) return;
  if (mode == 0 && S.phase != 0) return;
  __shared__ double s_h[kThreads / 64], s_l[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int k = S.k;
  const int n = 2 * k + 2;
  const int64_t per = (nv + G - 1) / G;
  const int64_t i0 = (int64_t)bx * per;
  const int64_t i1 = i0 + per < nv ? i0 + per : nv;
  const int spare = S.spare;
  if (mode == 1 && q == 0) {
    double* so = V.S[spare];
    double* yo = V.Y[spare];
    for (int64_t i = i0 + tid; i < i1; i += kThreads) {
      const dd a = dd_sub(vload(V.xt, nv, i), vload(V.x, nv, i));
      const dd b = dd_sub(vload(V.gt, nv, i), vload(V.g, nv, i));
      so[i] = a.h;
      so[nv + i] = a.l;
      yo[i] = b.h;
      yo[nv + i] = b.l;
    }
  }
  const bool isdot = !(mode == 0 && q == 2 * k + 1);
  dd acc{0.0, 0.0};
  if (q < n) {
    // operand codes: fa / fb = 1 fresh s, 2 fresh y, 0 the pointer pa / pb
    const double* pa = nullptr;
    const double* pb = nullptr;
    int fa = 0, fb = 0;
    if (mode == 0) {
      pb = V.g;
      if (q < k) pa = V.S[S.slot[q]];
      else if (q < 2 * k) pa = V.Y[S.slot[q - k]];
      else pa = V.g;  // g.g, and max|g| for q = 2k + 1
    } else {
      if (q == 0) {
        fa = 1;
        fb = 2;
      } else if (q == 1) {
        fa = 2;
        fb = 2;
      } else if (q < 2 + k) {
        pa = V.S[S.slot[q - 2]];
        fb = 2;
      } else {
        fa = 2;
        pb = V.Y[S.slot[q - 2 - k]];
      }
    }
    for (int64_t i = i0 + tid; i < i1; i += kThreads) {
      dd x;
      if (fa == 1) x = dd_sub(vload(V.xt, nv, i), vload(V.x, nv, i));
      else if (fa == 2) x = dd_sub(vload(V.gt, nv, i), vload(V.g, nv, i));
      else x = vload(pa, nv, i);
      if (!isdot) {
        const dd ax = x.h < 0.0 ? dd_neg(x) : x;
        if (dd_less(acc, ax)) acc = ax;
        continue;
      }
      const dd y = fb == 2 ? dd_sub(vload(V.gt, nv, i), vload(V.g, nv, i)) : vload(pb, nv, i);
      acc = dd_add(acc, dd_mul(x, y));
    }
    for (int mm = 32; mm > 0; mm >>= 1) {
      const dd o = shfl_xor_dd(acc, mm);
      acc = isdot ? dd_add(acc, o) : (dd_less(acc, o) ? o : acc);
    }
    if (lane == 0) {
      s_h[wave] = acc.h;
      s_l[wave] = acc.l;
    }
  }
  __syncthreads();
  if (tid == 0 && q < n) {
    dd r{s_h[0], s_l[0]};
    for (int w = 1; w < kThreads / 64; ++w) {
      const dd o{s_h[w], s_l[w]};
      r = isdot ? dd_add(r, o) : (dd_less(r, o) ? o : r);
    }
    partial[((int64_t)q * G + bx) * 2] = r.h;
    partial[((int64_t)q * G + bx) * 2 + 1] = r.l;
  }
}

__global__ void __launch_bounds__(kThreads) k_dots(VecSet V, MinState* S_, int mode, int64_t nv,
                                                   double* __restrict__ partial) {
  dots_body(V, S_, mode, nv, partial, blockIdx.x, blockIdx.y, gridDim.x);
}

// one block: each product's range partials summed in range order (kSubs
// sub-ranges in parallel, then the sub-range sums in order), then the
// direction (mode 0) or the Armijo decision (mode 1)
// The block works on a copy of the state in LDS: one parallel load of the whole
// state instead of the chain of dependent global loads that its decisions make,
// and one parallel store of it at the end.
__device__ __forceinline__ void dots_final_body(MinState* S_, const MinParams& P, int mode, int G,
                                                const double* __restrict__ partial, const double* __restrict__ eblk,
                                                int64_t neblk) {
  static_assert(sizeof(MinState) % sizeof(double) == 0, "state copied as 8-byte words");
  constexpr int kWords = (int)(sizeof(MinState) / sizeof(double));
  __shared__ MinState S;
  const int tid = threadIdx.x;
  {
    const double* src = reinterpret_cast<const double*>(S_);
    double* dst = reinterpret_cast<double*>(&S);
    for (int w = tid; w < kWords; w += kThreads) dst[w] = src[w];
  }
  __syncthreads();
  if (!S.running) return;
  if (mode == 0 && S.phase != 0) return;
  if (mode == 1) {
    // the trial's Phi and S_max from the per-block partials of the energy pass
    dd phi, sm;
    double kk;
    reduce_energy_partials(eblk, neblk, &phi, &sm, &kk);
    if (tid == 0) {
      S.ft[0] = phi.h;
      S.ft[1] = phi.l;
      S.smaxt[0] = sm.h;
      S.smaxt[1] = sm.l;
    }
    __syncthreads();
  }
  const int k = S.k;
  const int n = 2 * k + 2;
  constexpr int kSubs = 7;
  __shared__ double s_ph[kSubs][kMaxDots], s_pl[kSubs][kMaxDots];
  {
    const int qq = tid / kSubs, r = tid % kSubs;
    if (qq < n) {
      const bool dotq = !(mode == 0 && qq == 2 * k + 1);
      const int per_r = (G + kSubs - 1) / kSubs;
      const int b0 = r * per_r, b1 = b0 + per_r < G ? b0 + per_r : G;
      dd acc2{0.0, 0.0};
      for (int blk = b0; blk < b1; ++blk) {
        const dd o{partial[((int64_t)qq * G + blk) * 2], partial[((int64_t)qq * G + blk) * 2 + 1]};
        acc2 = dotq ? dd_add(acc2, o) : (dd_less(acc2, o) ? o : acc2);
      }
      s_ph[r][qq] = acc2.h;
      s_pl[r][qq] = acc2.l;
    }
  }
  __syncthreads();
  if (tid < n) {
    const bool dotq = !(mode == 0 && tid == 2 * k + 1);
    dd r{s_ph[0][tid], s_pl[0][tid]};
    for (int q2 = 1; q2 < kSubs; ++q2) {
      const dd o{s_ph[q2][tid], s_pl[q2][tid]};
      r = dotq ? dd_add(r, o) : (dd_less(r, o) ? o : r);
    }
    st(mode == 0 ? S.dir_dots[tid] : S.trial_dots[tid], r);
  }
  __syncthreads();  // the products written above are read by other threads below
  if (mode == 0) direction_logic(S, P, tid);
  else decide_logic(S, P, tid);
  __syncthreads();
  {
    const double* src = reinterpret_cast<const double*>(&S);
    double* dst = reinterpret_cast<double*>(S_);
    for (int w = tid; w < kWords; w += kThreads) dst[w] = src[w];
  }
}

__global__ void __launch_bounds__(kThreads) k_dots_final(MinState* S_, MinParams P, int mode, int G,
                                                         const double* __restrict__ partial,
                                                         const double* __restrict__ eblk, int64_t neblk) {
  dots_final_body(S_, P, mode, G, partial, eblk, neblk);
}

// ---------------------------------------------------------------------------
// FIRE (the paper's minimiser; Bitzek et al., PRL 97, 170201 (2006)), unit
// masses, F = -g, velocities in V.p.  One step: P = F.v; if P > 0 the velocity
// is mixed, v <- (1 - a) v + a |v| F / |F|, and after more than N_min = 5
// consecutive such steps dt <- min(1.1 dt, dt_max), a <- 0.99 a; otherwise
// dt <- dt / 2, v <- 0, a <- 0.1; then v <- v + dt F, x <- x + dt v and the
// energy and gradient at the new x.  dt0^2 max|g(x0)| = step_cap N^(-1/d) and
// dt_max = 10 dt0 are set by the host; dt and a are IEEE doubles.
// ---------------------------------------------------------------------------
constexpr int kFireDots = 3;  // g.v, g.g, v.v

__device__ __forceinline__ void fire_dots_body(const VecSet& V, const MinState* S_, int64_t nv,
                                               double* __restrict__ partial, int bx, int q, int G) {
  if (!S_->running) return;
  __shared__ double s_h[kThreads / 64], s_l[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t per = (nv + G - 1) / G;
  const int64_t i0 = (int64_t)bx * per;
  const int64_t i1 = i0 + per < nv ? i0 + per : nv;
  const double* a = q == 2 ? V.p : V.g;
  const double* b = q == 1 ? V.g : V.p;
  dd acc{0.0, 0.0};
  for (int64_t i = i0 + tid; i < i1; i += kThreads) acc = dd_add(acc, dd_mul(vload(a, nv, i), vload(b, nv, i)));
  for (int m = 32; m > 0; m >>= 1) acc = dd_add(acc, shfl_xor_dd(acc, m));
  if (lane == 0) {
    s_h[wave] = acc.h;
    s_l[wave] = acc.l;
  }
  __syncthreads();
  if (tid == 0) {
    dd r{s_h[0], s_l[0]};
    for (int w = 1; w < kThreads / 64; ++w) r = dd_add(r, dd{s_h[w], s_l[w]});
    partial[((int64_t)q * G + bx) * 2] = r.h;
    partial[((int64_t)q * G + bx) * 2 + 1] = r.l;
  }
}

__global__ void __launch_bounds__(kThreads) k_fire_dots(VecSet V, const MinState* S_, int64_t nv,
                                                        double* __restrict__ partial) {
  fire_dots_body(V, S_, nv, partial, blockIdx.x, blockIdx.y, gridDim.x);
}

// one block: the three products in range order, then the FIRE decisions
// (every thread of the block calls it; wave 0 works)
__device__ __forceinline__ void fire_final_body(MinState* S_, int G, const double* __restrict__ partial) {
  MinState& S = *S_;
  if (!S.running) return;
  const int tid = threadIdx.x;
  __shared__ double s_d[kFireDots][2];
  if (tid < kFireDots) {
    dd r{0.0, 0.0};
    for (int b = 0; b < G; ++b) r = dd_add(r, dd{partial[((int64_t)tid * G + b) * 2], partial[((int64_t)tid * G + b) * 2 + 1]});
    s_d[tid][0] = r.h;
    s_d[tid][1] = r.l;
  }
  __syncthreads();
  if (tid != 0) return;
  if (S.fdt == 0.0) {  // g = 0 at the start: a stationary point
    S.status = 0;
    S.running = 0;
    return;
  }
  const dd gv{s_d[0][0], s_d[0][1]}, gg{s_d[1][0], s_d[1][1]}, vv{s_d[2][0], s_d[2][1]};
  const dd P = dd_neg(gv);
  if (P.h > 0.0 || (P.h == 0.0 && P.l > 0.0)) {
    const double a = S.fa;
    const dd cg = dd_mul_d(dd_div(dd_sqrt(vv), dd_sqrt(gg)), a);
    st(S.fcv, dd{1.0 - a, 0.0});
    st(S.fcg, cg);
    S.fire_reset = 0;
    S.npos += 1;
    if (S.npos > 5) {
      const double up = S.fdt * 1.1;
      S.fdt = up < S.fdt_max ? up : S.fdt_max;
      S.fa = a * 0.99;
    }
  } else {
    S.fdt = S.fdt * 0.5;
    S.fire_reset = 1;
    S.fa = 0.1;
    S.npos = 0;
  }
}

__global__ void __launch_bounds__(64) k_fire_final(MinState* S_, int G, const double* __restrict__ partial) {
  fire_final_body(S_, G, partial);
}

// v <- mix(v, g); v <- v - dt g; x_new <- x + dt v, written to x (single
// quenches evaluate in place) or to xt (batched quenches, accepted afterwards)
__device__ __forceinline__ void fire_step_body(const VecSet& V, const MinState* S_, int64_t nv, int64_t i,
                                               double* __restrict__ xnew) {
  const MinState& S = *S_;
  if (!S.running) return;
  if (i >= nv) return;
  const double dt = S.fdt;
  const dd g = vload(V.g, nv, i);
  dd v{0.0, 0.0};
  if (!S.fire_reset) v = dd_sub(dd_mul(ld(S.fcv), vload(V.p, nv, i)), dd_mul(ld(S.fcg), g));
  v = dd_sub(v, dd_mul_d(g, dt));
  dd x = dd_add(vload(V.x, nv, i), dd_mul_d(v, dt));
  // failure injection: the step of iteration fault_iter gets a NaN
  if (i == 0 && S.fault_iter > 0 && S.iter + 1 == S.fault_iter) x.h = __builtin_nan("");
  V.p[i] = v.h;
  V.p[nv + i] = v.l;
  xnew[i] = x.h;
  xnew[nv + i] = x.l;
}

__global__ void __launch_bounds__(kThreads) k_fire_step(VecSet V, const MinState* S_, int64_t nv) {
  fire_step_body(V, S_, nv, (int64_t)blockIdx.x * kThreads + threadIdx.x, V.x);
}

// after the evaluation at the new x: Phi and S_max from the energy pass's block
// partials, the finite check and the start-of-iteration tests (every thread of
// a kThreads block calls it); accept != 0 marks the step for the batched
// acceptance copy x <- xt, g <- gt
__device__ __forceinline__ void fire_top_body(MinState* S_, const MinParams& P, const double* __restrict__ eblk,
                                              int64_t neblk, int accept) {
  MinState& S = *S_;
  if (!S.running) return;
  dd phi, sm;
  double kk;
  reduce_energy_partials(eblk, neblk, &phi, &sm, &kk);
  const int tid = threadIdx.x;
  if (tid >= 64) return;
  const int64_t it = S.iter + 1;
  if (tid == 0) {
    S.iter = it;
    S.evals += 1;
    st(S.f, phi);
    st(S.smax, sm);
    S.accepted = accept;
  }
  if (!isfinite(phi.h)) {
    if (tid == 0) {
      S.status = 3;
      S.running = 0;
    }
    return;
  }
  top_of_iteration(S, P, tid, it, phi, sm);
}

__global__ void __launch_bounds__(kThreads) k_fire_top(MinState* S_, MinParams P, const double* __restrict__ eblk,
                                                       int64_t neblk) {
  fire_top_body(S_, P, eblk, neblk, 0);
}

// FIRE start: dt0 from the host, v = 0, a = 0.1
__global__ void __launch_bounds__(kThreads) k_fire_init(VecSet V, MinState* S_, int64_t nv, double dt0) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < nv) {
    V.p[i] = 0.0;
    V.p[nv + i] = 0.0;
  }
  if (i == 0) {
    MinState& S = *S_;
    S.fdt = dt0;
    S.fdt_max = 10.0 * dt0;
    S.fa = 0.1;
    S.npos = 0;
    S.fire_reset = 0;
  }
}

// max |g_i| over the vector (one block, fixed order) for the initial step
__global__ void __launch_bounds__(kThreads) k_gmax(const double* __restrict__ g, int64_t nv, double* __restrict__ out) {
  __shared__ double s_h[kThreads], s_l[kThreads];
  const int tid = threadIdx.x;
  dd m{0.0, 0.0};
  for (int64_t i = tid; i < nv; i += kThreads) {
    dd x = vload(g, nv, i);
    if (x.h < 0.0) x = dd_neg(x);
    if (dd_less(m, x)) m = x;
  }
  s_h[tid] = m.h;
  s_l[tid] = m.l;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const dd a{s_h[tid], s_l[tid]}, b{s_h[tid + w], s_l[tid + w]};
      if (dd_less(a, b)) {
        s_h[tid] = b.h;
        s_l[tid] = b.l;
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    out[0] = s_h[0];
    out[1] = s_l[0];
  }
}

// progress record of a quench: running, iteration, evaluations, Phi.hi, S_max.hi
struct Progress {
  int32_t running, pad;
  int64_t iter, evals;
  double f, smax;
};

__global__ void k_progress(const MinState* S_, Progress* out) {
  if (threadIdx.x != 0) return;
  const MinState& S = *S_;
  out->running = S.running;
  out->pad = 0;
  out->iter = S.iter;
  out->evals = S.evals;
  out->f = S.f[0];
  out->smax = S.smax[0];
}

// x <- xt, g <- gt after an accepted trial
__device__ __forceinline__ void accept_body(const VecSet& V, const MinState* S_, int64_t nv, int64_t bx) {
  if (!S_->accepted) return;
  const int64_t i = bx * kThreads + threadIdx.x;
  if (i >= nv) return;
  V.x[i] = V.xt[i];
  V.x[nv + i] = V.xt[nv + i];
  V.g[i] = V.gt[i];
  V.g[nv + i] = V.gt[nv + i];
}

__global__ void __launch_bounds__(kThreads) k_accept(VecSet V, const MinState* S_, int64_t nv) {
  accept_body(V, S_, nv, blockIdx.x);
}

// ---------------------------------------------------------------------------
// batched minimiser kernels: the same bodies over many configurations (see the
// batched energy kernels for the unit convention)
// ---------------------------------------------------------------------------
// A FIRE configuration (P.method 1) maps its step onto the same launches: the
// direction products compute g.v, g.g, v.v (the first 3 of the G (2m + 2)
// units), the direction block takes the FIRE decisions, the step writes the new
// positions to xt, the trial evaluation is the step's evaluation, the decision
// block runs the stopping tests and always accepts, and the acceptance copies
// xt, gt to x, g -- the same arithmetic as a single FIRE quench.
__global__ void __launch_bounds__(kThreads) kb_dots(const MinSlot* __restrict__ ms, const BUnit* __restrict__ units,
                                                    int mode) {
  const BUnit u = units[blockIdx.x];
  const MinSlot& C = ms[u.slot];
  const int G = C.dot_blocks;
  if (C.P.method == 1) {
    if (mode == 0 && u.idx / G < kFireDots) fire_dots_body(C.V, C.S, C.nv, C.partial, u.idx % G, u.idx / G, G);
    return;
  }
  dots_body(C.V, C.S, mode, C.nv, C.partial, u.idx % G, u.idx / G, G);
}

__global__ void __launch_bounds__(kThreads) kb_dots_final(const MinSlot* __restrict__ ms,
                                                          const int32_t* __restrict__ list, int mode) {
  const MinSlot& C = ms[list[blockIdx.x]];
  if (C.P.method == 1) {
    if (mode == 0) fire_final_body(C.S, C.dot_blocks, C.partial);
    else fire_top_body(C.S, C.P, C.eblk, C.neblk, 1);
    return;
  }
  dots_final_body(C.S, C.P, mode, C.dot_blocks, C.partial, C.eblk, C.neblk);
}

__global__ void __launch_bounds__(kThreads) kb_step(const MinSlot* __restrict__ ms, const BUnit* __restrict__ units) {
  const BUnit u = units[blockIdx.x];
  const MinSlot& C = ms[u.slot];
  if (C.P.method == 1) {
    fire_step_body(C.V, C.S, C.nv, (int64_t)u.idx * kThreads + threadIdx.x, C.V.xt);
    return;
  }
  step_body(C.V, C.S, C.nv, u.idx);
}

__global__ void __launch_bounds__(kThreads) kb_accept(const MinSlot* __restrict__ ms,
                                                      const BUnit* __restrict__ units) {
  const BUnit u = units[blockIdx.x];
  const MinSlot& C = ms[u.slot];
  accept_body(C.V, C.S, C.nv, u.idx);
}

// FIRE start of a batched configuration (one 64-thread block): v = 0, a = 0.1
// and dt0 = sqrt(step / max|g(x0)|) (dt_max = 10 dt0), the same IEEE
// operations the single quench does on the host
__device__ __forceinline__ void fire_init_block(const MinSlot& C) {
  const int tid = threadIdx.x;
  __shared__ double s_h[64], s_l[64];
  dd m{0.0, 0.0};
  for (int64_t i = tid; i < C.nv; i += 64) {
    C.V.p[i] = 0.0;
    C.V.p[C.nv + i] = 0.0;
    dd x = vload(C.V.g, C.nv, i);
    if (x.h < 0.0) x = dd_neg(x);
    if (dd_less(m, x)) m = x;
  }
  s_h[tid] = m.h;
  s_l[tid] = m.l;
  __syncthreads();
  if (tid != 0) return;
  for (int w = 1; w < 64; ++w)
    if (dd_less(m, dd{s_h[w], s_l[w]})) m = dd{s_h[w], s_l[w]};
  MinState& S = *C.S;
  const double dt0 = m.h > 0.0 ? sqrt(C.P.step / m.h) : 0.0;
  S.fdt = dt0;
  S.fdt_max = 10.0 * dt0;
  S.fa = 0.1;
  S.npos = 0;
  S.fire_reset = 0;
}

__global__ void __launch_bounds__(64) kb_init(const MinSlot* __restrict__ ms, const int32_t* __restrict__ list) {
  const MinSlot& C = ms[list[blockIdx.x]];
  init_body(C.S, C.P, C.keep);
  if (C.P.method == 1) {
    __syncthreads();
    fire_init_block(C);
  }
}

// status of each listed configuration, gathered for one copy to the host
__global__ void __launch_bounds__(kThreads) kb_flags(const MinSlot* __restrict__ ms, const int32_t* __restrict__ list,
                                                     int64_t n, SlotFlags* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int32_t s = list[i];
  const MinState& S = *ms[s].S;
  SlotFlags f;
  f.running = S.running;
  f.status = S.status;
  f.iter = S.iter;
  f.evals = S.evals;
  out[s] = f;
}

hipError_t launch_batch_dots(const MinSlot* ms, const BUnit* units, int64_t n, int mode, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_dots, dim3((unsigned)n), dim3(kThreads), 0, st, ms, units, mode);
  return hipGetLastError();
}
hipError_t launch_batch_dots_final(const MinSlot* ms, const int32_t* list, int64_t n, int mode, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_dots_final, dim3((unsigned)n), dim3(kThreads), 0, st, ms, list, mode);
  return hipGetLastError();
}
hipError_t launch_batch_step(const MinSlot* ms, const BUnit* units, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_step, dim3((unsigned)n), dim3(kThreads), 0, st, ms, units);
  return hipGetLastError();
}
hipError_t launch_batch_accept(const MinSlot* ms, const BUnit* units, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_accept, dim3((unsigned)n), dim3(kThreads), 0, st, ms, units);
  return hipGetLastError();
}
hipError_t launch_batch_init(const MinSlot* ms, const int32_t* list, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_init, dim3((unsigned)n), dim3(64), 0, st, ms, list);
  return hipGetLastError();
}
hipError_t launch_batch_flags(const MinSlot* ms, const int32_t* list, int64_t n, SlotFlags* out, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(kb_flags, dim3((unsigned)((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, ms, list, n,
                       out);
  return hipGetLastError();
}

namespace {

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t lbfgs_bytes(int64_t nv) {
  const size_t vec = al256(sizeof(double) * 2 * (size_t)nv);
  return vec * (4 + 2 * (kMaxHistory + 1)) + al256(sizeof(MinState)) +
         al256(sizeof(double) * 2 * kMaxDots * kDotBlocks + 64) + 256;
}

struct Layout {
  VecSet V;
  MinState* state;
  double* partial;
};

void carve(char* base, int64_t nv, double* x, Layout* L) {
  const size_t vec = al256(sizeof(double) * 2 * (size_t)nv);
  size_t off = 0;
  auto take = [&](size_t n) {
    char* p = base + off;
    off += n;
    return p;
  };
  L->V.x = x;
  L->V.g = (double*)take(vec);
  L->V.xt = (double*)take(vec);
  L->V.gt = (double*)take(vec);
  L->V.p = (double*)take(vec);
  for (int i = 0; i <= kMaxHistory; ++i) L->V.S[i] = (double*)take(vec);
  for (int i = 0; i <= kMaxHistory; ++i) L->V.Y[i] = (double*)take(vec);
  L->state = (MinState*)take(al256(sizeof(MinState)));
  L->partial = (double*)take(al256(sizeof(double) * 2 * kMaxDots * kDotBlocks + 64));
}

}  // namespace

size_t minimize_extra_bytes(int64_t nv) { return lbfgs_bytes(nv); }

bool min_opts_valid(const ss_min_opts* op) {
  return op && op->history >= 1 && op->history <= kMaxHistory && op->max_iter >= 0 && op->stall_window >= 1 &&
         op->stall_window <= kMaxWindow && op->max_halvings >= 0 && op->max_ls_fail >= 1 && op->step_cap > 0.0 &&
         op->c1 > 0.0 && op->c1 < 1.0 && op->stall_ratio > 0.0 && op->precision >= 0 && op->precision <= 2 &&
         op->fp64_floor >= 0.0 && op->method >= 0 && op->method <= 1 && op->fault_iter >= 0;
}

MinParams min_params(const ss_min_opts* op, const ss_problem* prob) {
  MinParams P;
  P.m = op->history;
  P.W = op->stall_window;
  P.max_halvings = op->max_halvings;
  P.max_ls_fail = op->max_ls_fail;
  P.max_iter = op->max_iter;
  P.s_floor = op->s_floor;
  P.stall_ratio = op->stall_ratio;
  P.c1 = op->c1;
  P.step = op->step_cap * pow((double)prob->N, -1.0 / (double)prob->d);
  P.fault_iter = op->fault_iter;
  P.method = op->method;
  return P;
}

}  // namespace ss

using namespace ss;

extern "C" int ss_minimize(ss_ctx* ctx, const ss_problem* prob, const int32_t* n_dev, const double* v_dev,
                           double* pos_dev, const ss_min_opts* op, ss_min_result* out, void* ws, size_t ws_bytes,
                           void* stream) {
  if (!ctx) return SS_EINVAL;
  Plan* pl = nullptr;
  LaunchCfg c;
  int rc = prepare(ctx, prob, &pl, &c);
  if (rc) return rc;
  if (!n_dev || !pos_dev || !op || !out || !ws) {
    ctx->last_error = "NULL required pointer";
    return SS_EINVAL;
  }
  if (prob->vkind != 0 && !v_dev) {
    ctx->last_error = "vkind != 0 needs v_dev";
    return SS_EINVAL;
  }
  if (!min_opts_valid(op)) {
    ctx->last_error = "invalid minimiser options";
    return SS_EINVAL;
  }
  const int64_t nv = (int64_t)prob->d * prob->N;
  if (ws_bytes < c.total + minimize_extra_bytes(nv)) {
    ctx->last_error = "workspace too small";
    return SS_EINVAL;
  }
  const auto t0 = std::chrono::steady_clock::now();
  hipStream_t st = (hipStream_t)stream;
  char* ews = (char*)ws;
  Layout Lay;
  carve(ews + c.total, nv, pos_dev, &Lay);
  VecSet& V = Lay.V;
  MinState* S = Lay.state;
  const int blocks_nv = (int)((nv + kThreads - 1) / kThreads);
  const int dot_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (nv + 1023) / 1024));
  const double L = prob->L;
  int err = SS_OK;
  auto ok = [&](hipError_t e, const char* what) {
    if (e != hipSuccess && err == SS_OK) {
      ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
      err = e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EHIP;
    }
    return err == SS_OK;
  };
  const int* running = &S->running;
  bool fp64 = false;
  auto eval = [&](const double* x, double* phi, double* smax, double* g, const int* active) -> bool {
    int e = energy_grad_impl(ctx, prob, pl, c, v_dev, x, phi, smax, g, nullptr, ews, st, nullptr, active, fp64);
    if (e) {
      if (err == SS_OK) err = e;
      return false;
    }
    if (L != 1.0) {
      hipLaunchKernelGGL(k_times_L, dim3(blocks_nv), dim3(kThreads), 0, st, g, nv, L, active);
      ok(hipGetLastError(), "k_times_L");
    }
    return err == SS_OK;
  };

  // ticks, enqueued kDepth ahead; the status word of each tick is copied to
  // pinned memory and read once that tick's event has completed
  constexpr int kDepth = 3;
  // per tick: the running word (and, with progress lines on, a Progress record)
  const double progress = ctx->progress_interval;
  Progress* prog_dev = (Progress*)(Lay.partial + 2 * kMaxDots * kDotBlocks);  // spare room of the dot partials
  Progress* prog_host = nullptr;
  int32_t* flags = nullptr;
  hipEvent_t ev[kDepth] = {};
  if (!ok(hipHostMalloc((void**)&flags, sizeof(int32_t) * kDepth, hipHostMallocDefault), "hipHostMalloc")) return err;
  if (progress > 0.0 &&
      !ok(hipHostMalloc((void**)&prog_host, sizeof(Progress) * kDepth, hipHostMallocDefault), "hipHostMalloc")) {
    hipHostFree(flags);
    return err;
  }
  auto last_print = std::chrono::steady_clock::now();
  int has_prog[kDepth] = {};
  bool prog_pending = false;
  for (int q = 0; q < kDepth && err == SS_OK; ++q) ok(hipEventCreateWithFlags(&ev[q], hipEventDisableTiming), "event");

  // one stage: a fresh start (history cleared) from the current positions
  const bool fire = op->method == 1;
  auto run_stage = [&](const MinParams& P, int keep) {
    prog_pending = false;
    for (int& h : has_prog) h = 0;
    if (!eval(pos_dev, S->f, S->smax, V.g, nullptr)) return;
    hipLaunchKernelGGL(k_init, dim3(1), dim3(64), 0, st, S, P, keep);
    ok(hipGetLastError(), "k_init");
    if (fire) {  // the initial step from max|g(x0)| (one read-back)
      double* gm = Lay.partial;
      hipLaunchKernelGGL(k_gmax, dim3(1), dim3(kThreads), 0, st, V.g, nv, gm);
      double hg[2] = {0.0, 0.0};
      if (!ok(hipMemcpyAsync(hg, gm, sizeof(hg), hipMemcpyDeviceToHost, st), "gmax copy") ||
          !ok(hipStreamSynchronize(st), "gmax sync"))
        return;
      const double dt0 = hg[0] > 0.0 ? sqrt(P.step / hg[0]) : 0.0;
      hipLaunchKernelGGL(k_fire_init, dim3(blocks_nv), dim3(kThreads), 0, st, V, S, nv, dt0);
      ok(hipGetLastError(), "k_fire_init");
    }
    int64_t tick = 0;
    while (err == SS_OK) {
      if (fire) {
        hipLaunchKernelGGL(k_fire_dots, dim3(dot_blocks, kFireDots), dim3(kThreads), 0, st, V, S, nv, Lay.partial);
        hipLaunchKernelGGL(k_fire_final, dim3(1), dim3(64), 0, st, S, dot_blocks, Lay.partial);
        hipLaunchKernelGGL(k_fire_step, dim3(blocks_nv), dim3(kThreads), 0, st, V, S, nv);
        if (!ok(hipGetLastError(), "FIRE step kernels")) break;
        if (!eval(V.x, nullptr, nullptr, V.g, running)) break;
        hipLaunchKernelGGL(k_fire_top, dim3(1), dim3(kThreads), 0, st, S, P, (const double*)(ews + c.off_blk),
                           c.combine_blocks);
        if (!ok(hipGetLastError(), "FIRE tests")) break;
      } else {
      hipLaunchKernelGGL(k_dots, dim3(dot_blocks, 2 * P.m + 2), dim3(kThreads), 0, st, V, S, 0, nv, Lay.partial);
      hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(kThreads), 0, st, S, P, 0, dot_blocks, Lay.partial, nullptr,
                         (int64_t)0);
      hipLaunchKernelGGL(k_step, dim3(blocks_nv), dim3(kThreads), 0, st, V, S, nv);
      if (!ok(hipGetLastError(), "direction kernels")) break;
      if (!eval(V.xt, nullptr, nullptr, V.gt, running)) break;  // Phi_t, S_max_t: reduced in k_dots_final
      hipLaunchKernelGGL(k_dots, dim3(dot_blocks, 2 * P.m + 2), dim3(kThreads), 0, st, V, S, 1, nv, Lay.partial);
      hipLaunchKernelGGL(k_dots_final, dim3(1), dim3(kThreads), 0, st, S, P, 1, dot_blocks, Lay.partial,
                         (const double*)(ews + c.off_blk), c.combine_blocks);
      hipLaunchKernelGGL(k_accept, dim3(blocks_nv), dim3(kThreads), 0, st, V, S, nv);
      if (!ok(hipGetLastError(), "decision kernels")) break;
      }
      const int q = (int)(tick % kDepth);
      if (!ok(hipMemcpyAsync(flags + q, running, sizeof(int32_t), hipMemcpyDeviceToHost, st), "flag copy")) break;
      // a progress record only on a tick enqueued once the interval has passed
      has_prog[q] = 0;
      if (prog_host && !prog_pending &&
          std::chrono::duration<double>(std::chrono::steady_clock::now() - last_print).count() >= progress) {
        hipLaunchKernelGGL(k_progress, dim3(1), dim3(64), 0, st, S, prog_dev);
        if (!ok(hipMemcpyAsync(prog_host + q, prog_dev, sizeof(Progress), hipMemcpyDeviceToHost, st),
                "progress copy"))
          break;
        has_prog[q] = 1;
        prog_pending = true;
      }
      if (!ok(hipEventRecord(ev[q], st), "event record")) break;
      ++tick;
      if (tick >= kDepth) {
        const int w = (int)(tick % kDepth);  // the oldest tick in flight
        if (!ok(hipEventSynchronize(ev[w]), "event sync")) break;
        if (has_prog[w]) {
          const auto now = std::chrono::steady_clock::now();
          const Progress& pr = prog_host[w];
          fprintf(stderr, "[ss_minimize] %s iter %lld evals %lld Phi %.6e S_max %.6e t %.1fs\n",
                  fp64 ? "fp64" : "dd", (long long)pr.iter, (long long)pr.evals, pr.f, pr.smax,
                  std::chrono::duration<double>(now - t0).count());
          fflush(stderr);
          last_print = now;
          has_prog[w] = 0;
          prog_pending = false;
        }
        if (flags[w] == 0) break;
      }
    }
    ok(hipStreamSynchronize(st), "stage sync");
  };

  // stages: FP64 only, double-double only, or FP64 until it stops (stall, its
  // own floor or the cap) and then double-double from there, keeping the
  // kept (s, y) pairs: a restart from steepest descent with the capped step
  // would need far more halvings than allowed this close to a minimum
  MinState hs;
  int64_t iters_fp64 = 0, evals_fp64 = 0, evals = 0, iters = 0;
  const int prec = op->precision;
  for (int stage = (prec == 0 ? 1 : 0); stage < (prec == 1 ? 1 : 2) && err == SS_OK; ++stage) {
    fp64 = stage == 0;
    MinParams P = min_params(op, prob);
    if (fp64 && prec == 2) {
      // the FP64 stage ends at its own floor or at its first line-search
      // failure: from there on the FP64 energy's rounding noise decides the
      // Armijo test and further FP64 steps are wasted
      P.s_floor = std::max(op->s_floor, op->fp64_floor);
      P.max_ls_fail = 1;
    }
    P.max_iter = std::max<int64_t>(0, op->max_iter - iters);
    run_stage(P, (prec == 2 && stage == 1) ? 1 : 0);
    if (err == SS_OK) ok(hipMemcpy(&hs, S, sizeof(MinState), hipMemcpyDeviceToHost), "state copy");
    if (err != SS_OK) break;
    iters += hs.iter;
    evals += hs.evals;
    if (fp64) {
      iters_fp64 = hs.iter;
      evals_fp64 = hs.evals;
    }
    if (hs.status == 3) break;  // non-finite: no second stage
  }
  for (int q = 0; q < kDepth; ++q)
    if (ev[q]) hipEventDestroy(ev[q]);
  hipHostFree(flags);
  if (prog_host) hipHostFree(prog_host);
  if (err != SS_OK) return err;
  out->status = hs.status;
  out->iters = iters;
  out->evals = evals;
  out->grad_evals = evals;
  out->iters_fp64 = iters_fp64;
  out->evals_fp64 = evals_fp64;
  out->phi[0] = hs.f[0];
  out->phi[1] = hs.f[1];
  out->smax[0] = hs.smax[0];
  out->smax[1] = hs.smax[1];
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (hs.status == 3) {
    ctx->last_error = "non-finite energy";
    return SS_ENUMERIC;
  }
  return SS_OK;
}
