// ss_lbfgs.hip -- device-resident L-BFGS quench of the stealthy energy.
//
// The paper quenches with FIRE ("Simulations" section) until Phi reaches the
// smallest value the precision allows; this library minimises with the
// limited-memory BFGS two-loop recursion (Nocedal & Wright, Numerical
// Optimization, 2nd ed., Alg. 7.4) with an Armijo backtracking line search.
// Every vector (positions, gradients, the (s, y) history) lives in device memory
// as double-double [2][d N] planes; dot products are double-double with a fixed
// reduction order.  The host only reads a few scalars per iteration to take the
// line-search and stopping decisions.
//
// Rules (shared with the CPU oracle's minimiser, which implements the same
// rules independently):
//  * stop "converged" when S_max <= s_floor;
//  * direction p = -H g with H0 = (s.y / y.y) I of the newest pair; when the
//    history is empty or g.p >= 0, reset the history and take the
//    steepest-descent step p = -g * step_cap * N^(-1/d) / max|g|;
//  * Armijo backtracking from alpha = 1 by halving, accept when
//    Phi(x + alpha p) <= Phi(x) + c1 alpha g.p; after max_halvings halvings
//    record a failure, reset the history and keep x;
//  * keep the pair (s, y) = (x_new - x, g_new - g) only when s.y > 0;
//  * stop "stalled" when min Phi over the last W iterations exceeds
//    stall_ratio * min Phi over the W before, or after max_ls_fail
//    consecutive failures; stop at max_iter.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <chrono>
#include <vector>

#include "ss.h"
#include "ss_dd.h"
#include "ss_internal.h"

namespace ss {

int prepare(ss_ctx* ctx, const ss_problem* p, Plan** pl, LaunchCfg* cfg);
int energy_grad_impl(ss_ctx* ctx, const ss_problem* p, Plan* pl, const LaunchCfg& c, const double* v_dev,
                     const double* pos, double* phi, double* smax, double* grad, double* nk, char* ws,
                     hipStream_t st, double* kmax);

constexpr int kMaxHistory = 16;
constexpr int kDotBlocks = 240;

// ---------------------------------------------------------------------------
// vector kernels on dd planes [2][nv]
// ---------------------------------------------------------------------------

// Fixed-order dot product a.b: each block reduces a fixed contiguous range
// (thread-strided sequential sums, then a tree); the last block to finish
// combines the block partials in block order and applies `op`:
//   0: out = dot    1: out = s0 * dot    2: out = s1 - s0 * dot
//   3: out = s0 / dot    4: out = dot, out2 = 1 / dot
// For op 5 the kernel computes max_i |a_i| instead and out = c / max.
__global__ void __launch_bounds__(kThreads) k_dot(const double* __restrict__ a, const double* __restrict__ b,
                                                  int64_t nv, double* __restrict__ partial,
                                                  unsigned int* __restrict__ counter, int op,
                                                  const double* __restrict__ s0, const double* __restrict__ s1,
                                                  double c, double* __restrict__ out, double* __restrict__ out2) {
  __shared__ double sh[kThreads], sl[kThreads];
  __shared__ bool is_last;
  const int tid = threadIdx.x;
  const int64_t per = (nv + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * per;
  const int64_t i1 = i0 + per < nv ? i0 + per : nv;
  dd acc{0.0, 0.0};
  for (int64_t i = i0 + tid; i < i1; i += kThreads) {
    const dd x{a[i], a[nv + i]};
    if (op == 5) {
      const dd ax = x.h < 0.0 ? dd_neg(x) : x;
      if (dd_less(acc, ax)) acc = ax;
    } else {
      acc = dd_add(acc, dd_mul(x, dd{b[i], b[nv + i]}));
    }
  }
  sh[tid] = acc.h;
  sl[tid] = acc.l;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const dd x{sh[tid], sl[tid]}, y{sh[tid + w], sl[tid + w]};
      const dd r = op == 5 ? (dd_less(x, y) ? y : x) : dd_add(x, y);
      sh[tid] = r.h;
      sl[tid] = r.l;
    }
    __syncthreads();
  }
  if (tid == 0) {
    partial[2 * blockIdx.x] = sh[0];
    partial[2 * blockIdx.x + 1] = sl[0];
    __threadfence();
    const unsigned int prev = atomicAdd(counter, 1u);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  if (!is_last) return;
  __threadfence();
  if (tid == 0) {
    dd r{0.0, 0.0};
    for (unsigned int q = 0; q < gridDim.x; ++q) {
      const dd y{partial[2 * q], partial[2 * q + 1]};
      r = op == 5 ? (dd_less(r, y) ? y : r) : dd_add(r, y);
    }
    dd res = r;
    if (op == 1) res = dd_mul(dd{s0[0], s0[1]}, r);
    else if (op == 2) res = dd_sub(dd{s1[0], s1[1]}, dd_mul(dd{s0[0], s0[1]}, r));
    else if (op == 3) res = dd_div(dd{s0[0], s0[1]}, r);
    else if (op == 5) res = r.h > 0.0 ? dd_div(dd{c, 0.0}, r) : dd{0.0, 0.0};
    out[0] = res.h;
    out[1] = res.l;
    if (op == 4 && out2) {
      const dd inv = r.h > 0.0 ? dd_div(dd{1.0, 0.0}, r) : dd{0.0, 0.0};
      out2[0] = inv.h;
      out2[1] = inv.l;
    }
    *counter = 0u;  // ready for the next reduction
  }
}

// y <- y + sgn * coef * x, coef a device dd scalar
__global__ void __launch_bounds__(kThreads) k_axpy(double* __restrict__ y, const double* __restrict__ x, int64_t nv,
                                                   const double* __restrict__ coef, double sgn) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nv) return;
  const dd c{sgn * coef[0], sgn * coef[1]};
  const dd r = dd_add(dd{y[i], y[nv + i]}, dd_mul(c, dd{x[i], x[nv + i]}));
  y[i] = r.h;
  y[nv + i] = r.l;
}

// y <- sgn * coef * x (coef a device dd scalar); x may alias y
__global__ void __launch_bounds__(kThreads) k_scale(double* y, const double* x, int64_t nv,
                                                    const double* __restrict__ coef, double sgn) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nv) return;
  const dd c{sgn * coef[0], sgn * coef[1]};
  const dd r = dd_mul(c, dd{x[i], x[nv + i]});
  y[i] = r.h;
  y[nv + i] = r.l;
}

// z <- x + alpha * p (alpha an exact power of two)
__global__ void __launch_bounds__(kThreads) k_step(double* __restrict__ z, const double* __restrict__ x,
                                                   const double* __restrict__ p, int64_t nv, double alpha) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nv) return;
  const dd r = dd_add(dd{x[i], x[nv + i]}, dd{alpha * p[i], alpha * p[nv + i]});
  z[i] = r.h;
  z[nv + i] = r.l;
}

// s <- xt - x, y <- gt - g
__global__ void __launch_bounds__(kThreads) k_pair(double* __restrict__ s, double* __restrict__ y,
                                                   const double* __restrict__ xt, const double* __restrict__ x,
                                                   const double* __restrict__ gt, const double* __restrict__ g,
                                                   int64_t nv) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nv) return;
  const dd a = dd_sub(dd{xt[i], xt[nv + i]}, dd{x[i], x[nv + i]});
  const dd b = dd_sub(dd{gt[i], gt[nv + i]}, dd{g[i], g[nv + i]});
  s[i] = a.h;
  s[nv + i] = a.l;
  y[i] = b.h;
  y[nv + i] = b.l;
}

// gradient with respect to the fractional coordinates: g <- L * dPhi/dr
__global__ void __launch_bounds__(kThreads) k_times_L(double* __restrict__ g, int64_t nv, double L) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= nv) return;
  const dd r = dd_mul_d(dd{g[i], g[nv + i]}, L);
  g[i] = r.h;
  g[nv + i] = r.l;
}

__global__ void k_zero_u32(unsigned int* p) { *p = 0u; }

// ---------------------------------------------------------------------------
// host double-double helpers (the line-search and stall decisions)
// ---------------------------------------------------------------------------
namespace {

struct hdd {
  double h, l;
};

inline hdd h_two_sum(double a, double b) {
  const double s = a + b;
  const double bb = s - a;
  return hdd{s, (a - (s - bb)) + (b - bb)};
}
inline hdd h_fast(double a, double b) {
  const double s = a + b;
  return hdd{s, b - (s - a)};
}
inline hdd h_add(hdd a, hdd b) {
  hdd s = h_two_sum(a.h, b.h);
  hdd t = h_two_sum(a.l, b.l);
  s.l += t.h;
  s = h_fast(s.h, s.l);
  s.l += t.l;
  return h_fast(s.h, s.l);
}
inline hdd h_mul_d(hdd a, double b) {
  const double p = a.h * b;
  double e = fma(a.h, b, -p);
  e = fma(a.l, b, e);
  return h_fast(p, e);
}
inline hdd h_mul(hdd a, hdd b) {
  const double p = a.h * b.h;
  double e = fma(a.h, b.h, -p);
  double t = a.l * b.l;
  t = fma(a.h, b.l, t);
  t = fma(a.l, b.h, t);
  e += t;
  return h_fast(p, e);
}
inline bool h_less(hdd a, hdd b) { return a.h < b.h || (a.h == b.h && a.l < b.l); }

struct Vecs {
  int64_t nv;
  double *g, *xt, *gt, *p, *q;
  double* S[kMaxHistory + 1];
  double* Y[kMaxHistory + 1];
  double* scal;  // device scalars (dd pairs), see Slot*
  double* partial;
  unsigned int* counter;
  size_t bytes;
};

// device scalar slots (each a dd = 2 doubles)
enum {
  kPhi = 0, kSmax, kPhiT, kSmaxT, kSy, kGp, kGamma, kYY, kTmp, kCoef, kKmax,
  kRho = 16, kAlpha = kRho + kMaxHistory + 1, kSyH = kAlpha + kMaxHistory + 1,
  kNumScal = kSyH + kMaxHistory + 1
};

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

size_t lbfgs_bytes(int64_t nv) {
  const size_t vec = al256(sizeof(double) * 2 * (size_t)nv);
  return vec * (5 + 2 * (kMaxHistory + 1)) + al256(sizeof(double) * 2 * kNumScal) +
         al256(sizeof(double) * 2 * kDotBlocks) + 256;
}

void carve(char* base, int64_t nv, Vecs* v) {
  const size_t vec = al256(sizeof(double) * 2 * (size_t)nv);
  size_t off = 0;
  v->nv = nv;
  auto take = [&](size_t n) {
    char* p = base + off;
    off += n;
    return p;
  };
  v->g = (double*)take(vec);
  v->xt = (double*)take(vec);
  v->gt = (double*)take(vec);
  v->p = (double*)take(vec);
  v->q = (double*)take(vec);
  for (int i = 0; i <= kMaxHistory; ++i) v->S[i] = (double*)take(vec);
  for (int i = 0; i <= kMaxHistory; ++i) v->Y[i] = (double*)take(vec);
  v->scal = (double*)take(al256(sizeof(double) * 2 * kNumScal));
  v->partial = (double*)take(al256(sizeof(double) * 2 * kDotBlocks));
  v->counter = (unsigned int*)take(256);
  v->bytes = off;
}

}  // namespace

size_t minimize_extra_bytes(int64_t nv) { return lbfgs_bytes(nv); }

}  // namespace ss

using namespace ss;

namespace {

struct Runner {
  ss_ctx* ctx;
  hipStream_t st;
  Vecs v;
  int blocks_nv;
  int dot_blocks;
  int err = SS_OK;

  bool ok(hipError_t e, const char* what) {
    if (e != hipSuccess && err == SS_OK) {
      ctx->last_error = std::string(what) + ": " + hipGetErrorString(e);
      err = e == hipErrorOutOfMemory ? SS_ENOMEM : SS_EHIP;
    }
    return err == SS_OK;
  }
  double* sc(int slot) { return v.scal + 2 * slot; }
  void dot(const double* a, const double* b, int op, int out, const double* s0 = nullptr,
           const double* s1 = nullptr, double c = 0.0, double* out2 = nullptr) {
    hipLaunchKernelGGL(k_dot, dim3(dot_blocks), dim3(kThreads), 0, st, a, b, v.nv, v.partial, v.counter, op, s0, s1,
                       c, sc(out), out2);
    ok(hipGetLastError(), "k_dot");
  }
  void axpy(double* y, const double* x, const double* coef, double sgn) {
    hipLaunchKernelGGL(k_axpy, dim3(blocks_nv), dim3(kThreads), 0, st, y, x, v.nv, coef, sgn);
    ok(hipGetLastError(), "k_axpy");
  }
  void scale(double* y, const double* x, const double* coef, double sgn) {
    hipLaunchKernelGGL(k_scale, dim3(blocks_nv), dim3(kThreads), 0, st, y, x, v.nv, coef, sgn);
    ok(hipGetLastError(), "k_scale");
  }
  bool fetch(int slot, int count, double* host) {
    if (!ok(hipMemcpyAsync(host, sc(slot), sizeof(double) * 2 * count, hipMemcpyDeviceToHost, st), "fetch")) return false;
    return ok(hipStreamSynchronize(st), "sync");
  }
};

}  // namespace

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
  if (op->history < 1 || op->history > kMaxHistory || op->max_iter < 0 || op->stall_window < 1 ||
      op->max_halvings < 0 || op->max_ls_fail < 1 || !(op->step_cap > 0.0) || !(op->c1 > 0.0 && op->c1 < 1.0)) {
    ctx->last_error = "invalid minimiser options";
    return SS_EINVAL;
  }
  const int64_t nv = (int64_t)prob->d * prob->N;
  if (ws_bytes < c.total + minimize_extra_bytes(nv)) {
    ctx->last_error = "workspace too small";
    return SS_EINVAL;
  }
  const auto t0 = std::chrono::steady_clock::now();
  char* ews = (char*)ws;
  Runner R{ctx, (hipStream_t)stream, {}, (int)((nv + kThreads - 1) / kThreads), 1};
  carve(ews + c.total, nv, &R.v);
  R.dot_blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kDotBlocks, (nv + 1023) / 1024));
  const int m = op->history;
  const double L = prob->L;
  Vecs& V = R.v;
  hipStream_t st = R.st;
  hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, st, V.counter);
  R.ok(hipGetLastError(), "k_zero_u32");

  auto eval = [&](const double* x, int phi_slot, double* g) -> bool {
    int e = energy_grad_impl(ctx, prob, pl, c, v_dev, x, R.sc(phi_slot), R.sc(phi_slot + 1), g, nullptr, ews, st,
                             nullptr);
    if (e) {
      if (R.err == SS_OK) R.err = e;
      return false;
    }
    if (g && L != 1.0) {
      hipLaunchKernelGGL(k_times_L, dim3(R.blocks_nv), dim3(kThreads), 0, st, g, nv, L);
      R.ok(hipGetLastError(), "k_times_L");
    }
    return R.err == SS_OK;
  };

  double hbuf[8];
  int64_t evals = 0, gevals = 0;
  if (!eval(pos_dev, kPhi, V.g) || !R.fetch(kPhi, 2, hbuf)) return R.err;
  ++evals;
  ++gevals;
  hdd f{hbuf[0], hbuf[1]}, smax{hbuf[2], hbuf[3]};
  if (!std::isfinite(f.h)) {
    out->status = 3;
    out->iters = 0;
    out->evals = evals;
    out->grad_evals = gevals;
    out->phi[0] = f.h;
    out->phi[1] = f.l;
    out->smax[0] = smax.h;
    out->smax[1] = smax.l;
    out->seconds = 0.0;
    ctx->last_error = "non-finite energy at the starting positions";
    return SS_ENUMERIC;
  }
  const double nmean = pow((double)prob->N, -1.0 / (double)prob->d);
  std::vector<int> ring;  // slots, oldest first
  std::vector<int> free_slots;
  for (int i = 0; i <= m; ++i) free_slots.push_back(m - i);
  std::vector<hdd> fhist;
  const int64_t W = op->stall_window;
  int ls_fail = 0;
  int status = 2;
  int64_t it = 0;
  for (;;) {
    fhist.push_back(f);
    if (!(smax.h > op->s_floor || (smax.h == op->s_floor && smax.l > 0.0))) {
      status = 0;
      break;
    }
    if (it >= op->max_iter) {
      status = 2;
      break;
    }
    if (it >= 2 * W) {
      hdd recent = fhist[it], older = fhist[it - W];
      for (int64_t i = it - W + 1; i <= it; ++i)
        if (h_less(fhist[i], recent)) recent = fhist[i];
      for (int64_t i = it - 2 * W + 1; i <= it - W; ++i)
        if (h_less(fhist[i], older)) older = fhist[i];
      if (h_less(h_mul_d(older, op->stall_ratio), recent)) {
        status = 1;
        break;
      }
    }
    bool use_sd = ring.empty();
    hdd gp{0.0, 0.0};
    if (!use_sd) {
      // two-loop recursion on q = g
      R.ok(hipMemcpyAsync(V.q, V.g, sizeof(double) * 2 * nv, hipMemcpyDeviceToDevice, st), "copy q");
      for (int h = (int)ring.size() - 1; h >= 0; --h) {
        const int s = ring[h];
        R.dot(V.S[s], V.q, 1, kAlpha + s, R.sc(kRho + s));       // alpha_s = rho_s s.q
        R.axpy(V.q, V.Y[s], R.sc(kAlpha + s), -1.0);             // q -= alpha_s y_s
      }
      const int nw = ring.back();
      R.dot(V.Y[nw], V.Y[nw], 3, kGamma, R.sc(kSyH + nw));       // gamma = s.y / y.y
      R.scale(V.q, V.q, R.sc(kGamma), 1.0);
      for (size_t h = 0; h < ring.size(); ++h) {
        const int s = ring[h];
        R.dot(V.Y[s], V.q, 2, kCoef, R.sc(kRho + s), R.sc(kAlpha + s));  // alpha_s - rho_s y.r
        R.axpy(V.q, V.S[s], R.sc(kCoef), 1.0);
      }
      R.dot(V.g, V.q, 0, kGp);                                   // g.q = -g.p
      if (!R.fetch(kGp, 1, hbuf)) return R.err;
      gp = hdd{-hbuf[0], -hbuf[1]};
      if (!(gp.h < 0.0 || (gp.h == 0.0 && gp.l < 0.0))) use_sd = true;
      else std::swap(V.p, V.q);  // p = -q is applied in the step (sign folded below)
    }
    double dir_sign = -1.0;  // p_dev holds -p for the two-loop direction
    if (use_sd) {
      for (int s : ring) free_slots.push_back(s);
      ring.clear();
      R.dot(V.g, V.g, 5, kTmp, nullptr, nullptr, op->step_cap * nmean);  // scale = step / max|g|
      R.scale(V.p, V.g, R.sc(kTmp), 1.0);                                  // p_dev = scale g = -p
      R.dot(V.g, V.p, 0, kGp);
      if (!R.fetch(kGp, 1, hbuf)) return R.err;
      gp = hdd{-hbuf[0], -hbuf[1]};
      if (gp.h == 0.0) {
        status = 0;
        break;
      }
    }
    // Armijo backtracking; each trial also computes the gradient and the
    // candidate pair into the spare history slot
    const int spare = free_slots.back();
    double alpha = 1.0;
    bool accepted = false;
    hdd ft{0, 0}, smt{0, 0}, sy{0, 0};
    for (int hcount = 0; hcount <= op->max_halvings; ++hcount) {
      hipLaunchKernelGGL(k_step, dim3(R.blocks_nv), dim3(kThreads), 0, st, V.xt, pos_dev, V.p, nv, dir_sign * alpha);
      R.ok(hipGetLastError(), "k_step");
      if (!eval(V.xt, kPhiT, V.gt)) return R.err;
      ++evals;
      ++gevals;
      hipLaunchKernelGGL(k_pair, dim3(R.blocks_nv), dim3(kThreads), 0, st, V.S[spare], V.Y[spare], V.xt, pos_dev,
                         V.gt, V.g, nv);
      R.ok(hipGetLastError(), "k_pair");
      R.dot(V.S[spare], V.Y[spare], 4, kSyH + spare, nullptr, nullptr, 0.0, R.sc(kRho + spare));
      R.ok(hipMemcpyAsync(R.sc(kSy), R.sc(kSyH + spare), 2 * sizeof(double), hipMemcpyDeviceToDevice, st),
           "copy sy");
      if (!R.fetch(kPhiT, 3, hbuf)) return R.err;  // PhiT, SmaxT, Sy in one read
      ft = hdd{hbuf[0], hbuf[1]};
      smt = hdd{hbuf[2], hbuf[3]};
      sy = hdd{hbuf[4], hbuf[5]};
      const hdd bound = h_add(f, h_mul(h_mul_d(hdd{alpha, 0.0}, op->c1), gp));
      if (!h_less(bound, ft)) {
        accepted = true;
        break;
      }
      alpha *= 0.5;
    }
    ++it;
    if (!accepted) {
      ++ls_fail;
      for (int s : ring) free_slots.push_back(s);
      ring.clear();
      if (ls_fail >= op->max_ls_fail) {
        fhist.push_back(f);
        status = 1;
        break;
      }
      continue;
    }
    ls_fail = 0;
    if (sy.h > 0.0) {
      free_slots.pop_back();
      ring.push_back(spare);
      if ((int)ring.size() > m) {
        free_slots.push_back(ring.front());
        ring.erase(ring.begin());
      }
    }
    R.ok(hipMemcpyAsync(pos_dev, V.xt, sizeof(double) * 2 * nv, hipMemcpyDeviceToDevice, st), "copy x");
    std::swap(V.g, V.gt);
    R.ok(hipMemcpyAsync(R.sc(kPhi), R.sc(kPhiT), 4 * sizeof(double), hipMemcpyDeviceToDevice, st), "copy phi");
    f = ft;
    smax = smt;
    if (!std::isfinite(f.h)) {
      status = 3;
      break;
    }
  }
  if (!R.ok(hipStreamSynchronize(st), "final sync")) return R.err;
  out->status = status;
  out->iters = it;
  out->evals = evals;
  out->grad_evals = gevals;
  out->phi[0] = f.h;
  out->phi[1] = f.l;
  out->smax[0] = smax.h;
  out->smax[1] = smax.l;
  out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  return status == 3 ? SS_ENUMERIC : SS_OK;
}
