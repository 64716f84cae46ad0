// ss_reduce.h -- the fixed-order, single-block reduction of the energy pass's
// per-block partials (Phi and S_max with the wavevector that attains it).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ss_dd.h"
#include "ss_internal.h"

namespace ss {

// One block of kThreads threads; every thread must call it.  blk[b * 5 + (0..4)]
// = Phi.hi, Phi.lo, Smax.hi, Smax.lo, k of the maximum.  Thread t first sums
// blocks t, t + kThreads, ... in order, then a tree over the threads; ties of
// S_max go to the smaller k.  The result is in phi / smax / kmax of thread 0.
__device__ inline void reduce_energy_partials(const double* __restrict__ blk, int64_t nblk, dd* phi_out,
                                              dd* smax_out, double* kmax_out) {
  __shared__ double s_ph[kThreads], s_pl[kThreads], s_mh[kThreads], s_ml[kThreads], s_mk[kThreads];
  const int tid = threadIdx.x;
  dd phi{0.0, 0.0}, sk{-1.0, 0.0};
  double kk = 1e300;
  for (int64_t b = tid; b < nblk; b += kThreads) {
    const double* q = blk + b * 5;
    phi = dd_add(phi, dd{q[0], q[1]});
    const dd y{q[2], q[3]};
    if (dd_less(sk, y) || (!dd_less(y, sk) && q[4] < kk)) {
      sk = y;
      kk = q[4];
    }
  }
  s_ph[tid] = phi.h;
  s_pl[tid] = phi.l;
  s_mh[tid] = sk.h;
  s_ml[tid] = sk.l;
  s_mk[tid] = kk;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const dd a = dd_add(dd{s_ph[tid], s_pl[tid]}, dd{s_ph[tid + w], s_pl[tid + w]});
      s_ph[tid] = a.h;
      s_pl[tid] = a.l;
      const dd x{s_mh[tid], s_ml[tid]}, y{s_mh[tid + w], s_ml[tid + w]};
      if (dd_less(x, y) || (!dd_less(y, x) && s_mk[tid + w] < s_mk[tid])) {
        s_mh[tid] = y.h;
        s_ml[tid] = y.l;
        s_mk[tid] = s_mk[tid + w];
      }
    }
    __syncthreads();
  }
  *phi_out = dd{s_ph[0], s_pl[0]};
  *smax_out = dd{s_mh[0], s_ml[0]};
  *kmax_out = s_mk[0];
  __syncthreads();  // the shared arrays may be reused by the caller's next call
}

}  // namespace ss
