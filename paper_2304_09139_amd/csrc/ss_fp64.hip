// ss_fp64.hip -- the two pair passes in plain FP64 arithmetic, for the first
// stage of a staged quench.
//
// The paper's point is that the last decades of S(k) need double-double; the
// early part of a quench from a Poisson start does not.  These kernels compute
// the same sums as the double-double passes (n~(k), Phi, S_max and the
// gradient, by the same factorisation exp(2 pi i n.u) = prod_a z_a^{n_a} over
// the same runs and pieces) with FP64 products and sums: about a fifth of the
// operations per pair.  The phase table is the double-double one; only its
// high words are read.  Results are written in the double-double layouts with
// zero low words, so the minimiser is unchanged.
//
// Error: every table entry carries a relative error <= 2^-53; a term is a
// product of at most D of them in the n(k) pass (the prefix entries and one
// z^t) and of D - 1 + len in the gradient pass (len the run length), so
// |term error| <= (D + len + 1) 2^-53 with len = 1 in the n(k) pass, and the
// N-term sums add N rounding errors of their own.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ss_dd.h"
#include "ss_internal.h"
#include "ss_min.h"

namespace ss {

struct c64 {
  double re, im;
};

__device__ __forceinline__ c64 cmul64(c64 a, c64 b) {
  return c64{__builtin_fma(a.re, b.re, -(a.im * b.im)), __builtin_fma(a.re, b.im, a.im * b.re)};
}

// entry z_a^m (high words) of a particle table staged in LDS as [a][m][re, im]
__device__ __forceinline__ c64 lds64_entry(const double* tp, int R1, int a, int m) {
  const int mm = m < 0 ? -m : m;
  const double* e = tp + (a * R1 + mm) * 2;
  return c64{e[0], m < 0 ? -e[1] : e[1]};
}

// the staged particles of one tile, every lane taking the L exponents of the
// wave's widest piece (terms past a lane's own piece are not stored): per
// particle the prefix product b, then b z^t and b conj(z^t) into accumulators
// 2i and 2i + 1 (the pieces, accumulators and slots of the double-double pass)
template <int D, int L>
__device__ __forceinline__ void nk64_tile(const double* __restrict__ lds, int np, int epp, int R1, const Span& sg,
                                          double (&cr)[kSegLen], double (&ci)[kSegLen]) {
  const int t0 = sg.n[D - 1];
#pragma unroll 1
  for (int p = 0; p < np; ++p) {
    const double* tp = lds + p * epp;
    c64 b{1.0, 0.0};
    if constexpr (D > 1) {
      b = lds64_entry(tp, R1, 0, sg.n[0]);
#pragma unroll
      for (int a = 1; a < D - 1; ++a) b = cmul64(b, lds64_entry(tp, R1, a, sg.n[a]));
    }
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const int m = t0 + i < R1 ? t0 + i : R1 - 1;
      const double* e = tp + ((D - 1) * R1 + m) * 2;
      const double ur = e[0], ui = e[1];
      const double ii = b.im * ui, ri = b.re * ui, ir = b.im * ur;
      cr[2 * i] += __builtin_fma(b.re, ur, -ii);
      ci[2 * i] += __builtin_fma(b.re, ui, ir);
      cr[2 * i + 1] += __builtin_fma(b.re, ur, ii);
      ci[2 * i + 1] += __builtin_fma(b.im, ur, -ri);
    }
  }
}

// n~(k) partials in FP64: part[(row * 2 + c) * M + slot], c = (C, S), slot order
template <int D, int PT>
__device__ __forceinline__ void nk64_body(const Span* __restrict__ segs, int64_t nseg, const NkUnit u,
                                          const double* __restrict__ tab, int64_t N, int R1,
                                          double* __restrict__ part, int64_t M, const SlotOffsets& so,
                                          double* __restrict__ lds) {
  const int tid = threadIdx.x;
  const int64_t s = (int64_t)u.block * kNkPieces + tid;
  const Span sg = segs[s < nseg ? s : nseg - 1];
  const int len = s < nseg ? sg.len : 0;
  const int epp = D * R1 * 2;  // doubles per particle
  bool plus = true;  // the prefix-zero column
#pragma unroll
  for (int a = 0; a < D - 1; ++a) plus = plus && sg.n[a] == 0;
  const bool zero = !plus && sg.n[D - 1] == 0;
  const int nt = plus ? len : (len + 1) / 2;  // exponents of this lane's piece
  double cr[kSegLen], ci[kSegLen];
#pragma unroll
  for (int t = 0; t < kSegLen; ++t) cr[t] = ci[t] = 0.0;
  // the widest piece of the wave, in a scalar register, selects the unrolled loop
  int wmax = nt;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o));
  const int wl = __builtin_amdgcn_readfirstlane(wmax);
  for (int64_t tile = u.j0; tile < u.j1; tile += PT) {
    const int np = (int)((u.j1 - tile) < PT ? (u.j1 - tile) : PT);
    __syncthreads();
    for (int i = tid; i < epp * PT; i += kThreads) {
      const int p = i % PT;
      const int ec = i / PT;  // (a R1 + m) * 2 + part; part 0 = re.hi (row 0), 1 = im.hi (row 2)
      const int64_t row = (int64_t)(ec >> 1) * 4 + 2 * (ec & 1);
      lds[p * epp + ec] = p < np ? tab[row * N + tile + p] : 0.0;
    }
    __syncthreads();
    switch (wl) {
      case 4:
        if constexpr (kSegLen >= 8) nk64_tile<D, 4>(lds, np, epp, R1, sg, cr, ci);
        break;
      case 3: nk64_tile<D, 3>(lds, np, epp, R1, sg, cr, ci); break;
      case 2: nk64_tile<D, 2>(lds, np, epp, R1, sg, cr, ci); break;
      case 1: nk64_tile<D, 1>(lds, np, epp, R1, sg, cr, ci); break;
      default: break;
    }
  }
  double* out = part + (int64_t)u.row * 2 * M;
#pragma unroll
  for (int t = 0; t < kSegLen; ++t) {
    if (t < len) {
      const int64_t slot = so.off[t] + s;
      constexpr int kLast = kSegLen - 1;
      const int q1 = t + 1 < kLast ? t + 1 : kLast, q2 = 2 * t < kLast ? 2 * t : kLast;
      double vr = cr[t], vi = ci[t];
      if (zero && t >= 1) vr = cr[q1], vi = ci[q1];
      if (plus) vr = cr[q2], vi = ci[q2];
      out[slot] = vr;
      out[M + slot] = vi;
    }
  }
}

template <int D, int PT>
__global__ void __launch_bounds__(kThreads) k_nk64(const Span* __restrict__ segs, int64_t nseg,
                                                   const NkUnit* __restrict__ units, const double* __restrict__ tab,
                                                   int64_t N, int R1, double* __restrict__ part, int64_t M,
                                                   const SlotOffsets so, const int* __restrict__ active) {
  if (active && *active == 0) return;
  extern __shared__ double lds[];  // [PT][D][R1][2]
  nk64_body<D, PT>(segs, nseg, units[blockIdx.x], tab, N, R1, part, M, so, lds);
}

// combine the FP64 partials (fixed order); n~ (dd layout, zero low words) in
// canonical order, (v C, v S) in walk order as csw[2][M], and per-block Phi and
// S_max partials in the double-double block layout
__device__ __forceinline__ void combine64_body(const double* __restrict__ part, const int32_t* __restrict__ rows_of,
                                               const int32_t* __restrict__ k_of_slot, int64_t M, int64_t N,
                                               const int32_t* __restrict__ canon_of_lex,
                                               const double* __restrict__ v, double* __restrict__ nk_out,
                                               double* __restrict__ csw, double* __restrict__ blk, int64_t bidx) {
  constexpr int kCombG = kThreads / kCombK;
  __shared__ double s_c[kCombG][2][kCombK];
  __shared__ double s_ph[kCombK], s_mh[kCombK];
  __shared__ int64_t s_mk[kCombK];
  const int tid = threadIdx.x, q = tid % kCombK, g = tid / kCombK;
  const int64_t i = bidx * kCombK + q;
  double C = 0.0, S = 0.0;
  if (i < M) {
    const int64_t P = rows_of[i];
    for (int64_t p = g; p < P; p += kCombG) {
      const double* r = part + p * 2 * M;
      C += r[i];
      S += r[M + i];
    }
  }
  s_c[g][0][q] = C;
  s_c[g][1][q] = S;
  __syncthreads();
  for (int w = kCombG / 2; w > 0; w >>= 1) {
    if (g < w) {
      s_c[g][0][q] += s_c[g + w][0][q];
      s_c[g][1][q] += s_c[g + w][1][q];
    }
    __syncthreads();
  }
  if (g == 0) {
    C = s_c[0][0][q];
    S = s_c[0][1][q];
    double phi = 0.0, sk = -1.0;
    int64_t kc = INT64_MAX;
    if (i < M) {
      const int64_t k = k_of_slot[i];
      kc = canon_of_lex[k];
      if (nk_out) {
        nk_out[kc] = C;
        nk_out[M + kc] = 0.0;
        nk_out[2 * M + kc] = S;
        nk_out[3 * M + kc] = 0.0;
      }
      const double w = v ? v[kc] + v[M + kc] : 1.0;
      csw[k] = w * C;
      csw[M + k] = w * S;
      const double mag = __builtin_fma(C, C, S * S);
      phi = w * mag;
      sk = mag / (double)N;
    }
    s_ph[q] = phi;
    s_mh[q] = sk;
    s_mk[q] = kc;
  }
  __syncthreads();
  for (int w = kCombK / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s_ph[tid] += s_ph[tid + w];
      if (s_mh[tid + w] > s_mh[tid] || (s_mh[tid + w] == s_mh[tid] && s_mk[tid + w] < s_mk[tid])) {
        s_mh[tid] = s_mh[tid + w];
        s_mk[tid] = s_mk[tid + w];
      }
    }
    __syncthreads();
  }
  if (tid == 0) {
    double* b = blk + bidx * 5;
    b[0] = s_ph[0];
    b[1] = 0.0;
    b[2] = s_mh[0];
    b[3] = 0.0;
    b[4] = (double)s_mk[0];
  }
}

__global__ void __launch_bounds__(kThreads) k_nk_combine64(const double* __restrict__ part,
                                                           const int32_t* __restrict__ rows_of,
                                                           const int32_t* __restrict__ k_of_slot, int64_t M,
                                                           int64_t N, const int32_t* __restrict__ canon_of_lex,
                                                           const double* __restrict__ v, double* __restrict__ nk_out,
                                                           double* __restrict__ csw, double* __restrict__ blk,
                                                           const int* __restrict__ active) {
  if (active && *active == 0) return;
  combine64_body(part, rows_of, k_of_slot, M, N, canon_of_lex, v, nk_out, csw, blk, blockIdx.x);
}

// table entry (high words) of particle j from the global table
__device__ __forceinline__ c64 tab64_entry(const double* __restrict__ tab, int64_t N, int R1, int a, int m, int64_t j) {
  const int mm = m < 0 ? -m : m;
  const double* e = tab + ((int64_t)(a * R1 + mm) * 4) * N + j;
  return c64{e[0], m < 0 ? -e[2 * N] : e[2 * N]};
}

// gradient partials in FP64: gpart[(q * D + a) * N + j]
template <int D>
__device__ __forceinline__ void grad64_body(const Span* __restrict__ runs, const int32_t* __restrict__ chunk_begin,
                                            const double* __restrict__ tab, const double* __restrict__ csw,
                                            int64_t N, int R1, int64_t M, double* __restrict__ gpart, int64_t pblock,
                                            int q) {
  __shared__ double s_g[kWaves][D][64];
  const int tid = threadIdx.x, lane = tid & 63;
  // the wave index is uniform across the wave: in a scalar register the run
  // bounds, the run records and the per-wavevector (vC, vS) become scalar loads
  // and the wavevector loop is a scalar loop
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t j = pblock * 64 + lane;
  const int64_t jj = j < N ? j : N - 1;
  const int r0 = chunk_begin[kWaves * q + wave], r1 = chunk_begin[kWaves * q + wave + 1];
  const c64 z = tab64_entry(tab, N, R1, D - 1, 1, jj);
  double g[D];
#pragma unroll
  for (int a = 0; a < D; ++a) g[a] = 0.0;
  for (int r = r0; r < r1; ++r) {
    const Span run = runs[r];
    c64 w = tab64_entry(tab, N, R1, D - 1, run.n[D - 1], jj);
#pragma unroll
    for (int a = 0; a < D - 1; ++a) w = cmul64(w, tab64_entry(tab, N, R1, a, run.n[a], jj));
    double q0 = 0.0, qd = 0.0;
    double nd = (double)run.n[D - 1];
    const double* cp = csw + run.k0;
#pragma unroll 2
    for (int t = 0; t < run.len; ++t) {
      const double qs = __builtin_fma(cp[M + t], w.re, -(cp[t] * w.im));  // v (S c - C s)
      q0 += qs;
      qd = __builtin_fma(nd, qs, qd);
      nd += 1.0;
      w = cmul64(w, z);
    }
#pragma unroll
    for (int a = 0; a < D - 1; ++a) g[a] = __builtin_fma((double)run.n[a], q0, g[a]);
    g[D - 1] += qd;
  }
#pragma unroll
  for (int a = 0; a < D; ++a) s_g[wave][a][lane] = g[a];
  __syncthreads();
  if (wave == 0 && j < N) {  // ((w0 + w2) + (w1 + w3))
#pragma unroll
    for (int a = 0; a < D; ++a)
      gpart[((int64_t)q * D + a) * N + j] =
          (s_g[0][a][lane] + s_g[2][a][lane]) + (s_g[1][a][lane] + s_g[3][a][lane]);
  }
}

template <int D>
__global__ void __launch_bounds__(kThreads) k_grad64(const Span* __restrict__ runs,
                                                     const int32_t* __restrict__ chunk_begin,
                                                     const double* __restrict__ tab, const double* __restrict__ csw,
                                                     int64_t N, int R1, int64_t M, double* __restrict__ gpart,
                                                     const int* __restrict__ active) {
  if (active && *active == 0) return;
  grad64_body<D>(runs, chunk_begin, tab, csw, N, R1, M, gpart, blockIdx.x, blockIdx.y);
}

// sum the Q FP64 partials in order, scale by 4 pi / L (and by L with times_L),
// store in the dd layout with zero low words
__device__ __forceinline__ void gcomb64_body(const double* __restrict__ gpart, int Q, int d, int64_t N, double L,
                                             bool times_L, double* __restrict__ grad, int64_t i) {
  const int64_t DN = (int64_t)d * N;
  if (i >= DN) return;
  double g = 0.0;
  for (int q = 0; q < Q; ++q) g += gpart[(int64_t)q * DN + i];
  const dd tp = two_pi_dd();
  g *= 2.0 * tp.h / L;
  if (times_L) g *= L;
  grad[i] = g;
  grad[DN + i] = 0.0;
}

__global__ void __launch_bounds__(kThreads) k_grad_combine64(const double* __restrict__ gpart, int Q, int d,
                                                             int64_t N, double L, int times_L,
                                                             double* __restrict__ grad,
                                                             const int* __restrict__ active) {
  if (active && *active == 0) return;
  gcomb64_body(gpart, Q, d, N, L, times_L != 0, grad, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

// ---------------------------------------------------------------------------
// the tiled d = 2 n~(k) pass in FP64: the double-double tiled pass with the high
// words of the two staged table slices, FP64 complex products and sums;
// part[(row * 2 + c) * M + walk position]
// ---------------------------------------------------------------------------
constexpr int kT2f = 16;
constexpr int kT2fPitch = kT2f * 2 + 2;  // doubles per staged particle (pad: no bank conflicts)

__device__ __forceinline__ void nk2_64_body(const int32_t* __restrict__ tiles, const int32_t* __restrict__ lexinfo,
                                            int R, const double* __restrict__ tab, int64_t N, int R1, int64_t chunk,
                                            int tile, int row, double* __restrict__ part, int64_t M) {
  __shared__ double s0[kT2f * kT2fPitch], s1[kT2f * kT2fPitch];  // [particle][row][re, im]
  const int tid = threadIdx.x;
  const int a0 = tiles[2 * tile], b0 = tiles[2 * tile + 1];
  const int i0 = tid / kT2f, i1 = tid % kT2f;
  const int n0 = a0 + i0, n1 = b0 + i1;
  int64_t pos = -1;
  if (n0 <= R) {
    const int off = lexinfo[3 * n0], lo = lexinfo[3 * n0 + 1], hi = lexinfo[3 * n0 + 2];
    if (n1 >= lo && n1 <= hi) pos = off + (n1 - lo);
  }
  const bool mine = pos >= 0;
  const bool neg = n1 < 0;
  double cr = 0.0, ci = 0.0;
  const int64_t j0 = (int64_t)row * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  // 2 slices x 16 rows x (re.hi, im.hi) x 16 particles, particle fastest; the
  // next chunk's values are loaded into registers while the current one is used
  constexpr int kQ = (2 * kT2f * 2 * kT2f) / kThreads;
  double pre[kQ];
  auto fetch = [&](int64_t tj) {
    const int np = (int)((j1 - tj) < kT2f ? (j1 - tj) : kT2f);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int idx = tid + kThreads * q;
      const int p = idx % kT2f, c2 = (idx / kT2f) % 2, r = (idx / (2 * kT2f)) % kT2f, ax = idx / (2 * kT2f * kT2f);
      const int m = ax == 0 ? a0 + r : (b0 + r < 0 ? -(b0 + r) : b0 + r);
      pre[q] = (p < np && m <= R) ? tab[((int64_t)(ax * R1 + m) * 4 + 2 * c2) * N + tj + p] : 0.0;
    }
  };
  if (j0 < j1) fetch(j0);
  for (int64_t tj = j0; tj < j1; tj += kT2f) {
    const int np = (int)((j1 - tj) < kT2f ? (j1 - tj) : kT2f);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int idx = tid + kThreads * q;
      const int p = idx % kT2f, c2 = (idx / kT2f) % 2, r = (idx / (2 * kT2f)) % kT2f, ax = idx / (2 * kT2f * kT2f);
      (ax == 0 ? s0 : s1)[p * kT2fPitch + r * 2 + c2] = pre[q];
    }
    __syncthreads();
    if (tj + kT2f < j1) fetch(tj + kT2f);
    if (mine) {
#pragma unroll 4
      for (int p = 0; p < np; ++p) {
        const double* e0 = s0 + p * kT2fPitch + i0 * 2;
        const double* e1 = s1 + p * kT2fPitch + i1 * 2;
        const c64 w = cmul64(c64{e0[0], e0[1]}, c64{e1[0], neg ? -e1[1] : e1[1]});
        cr += w.re;
        ci += w.im;
      }
    }
  }
  if (mine) {
    double* out = part + (int64_t)row * 2 * M;
    out[pos] = cr;
    out[M + pos] = ci;
  }
}

__global__ void __launch_bounds__(kThreads) k_nk2_64(const int32_t* __restrict__ tiles,
                                                     const int32_t* __restrict__ lexinfo, int R,
                                                     const double* __restrict__ tab, int64_t N, int R1,
                                                     int64_t chunk, int nrows, double* __restrict__ part, int64_t M,
                                                     const int* __restrict__ active) {
  if (active && *active == 0) return;
  nk2_64_body(tiles, lexinfo, R, tab, N, R1, chunk, (int)(blockIdx.x / nrows), (int)(blockIdx.x % nrows), part, M);
}

// ---------------------------------------------------------------------------
// batched FP64 launches (the FP64 stage of staged quenches in a batch): the
// same bodies over the blocks of many configurations, as in the double-double
// batched kernels
// ---------------------------------------------------------------------------
template <int D, int PT>
__global__ void __launch_bounds__(kThreads) kb_nk64(const EvalSlot* __restrict__ es, const BUnit* __restrict__ units,
                                                    int gate) {
  extern __shared__ double lds[];
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  nk64_body<D, PT>(E.segs, E.nsegs, E.units[u.idx], E.tab, E.N, E.R1, E.part, E.M, E.so, lds);
}

__global__ void __launch_bounds__(kThreads) kb_nk2_64(const EvalSlot* __restrict__ es,
                                                      const BUnit* __restrict__ units, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  nk2_64_body(E.t2_tiles, E.t2_lexinfo, E.R, E.tab, E.N, E.R1, E.t2_chunk, u.idx / E.t2_nrows, u.idx % E.t2_nrows,
              E.part, E.M);
}

__global__ void __launch_bounds__(kThreads) kb_combine64(const EvalSlot* __restrict__ es,
                                                         const BUnit* __restrict__ units, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  combine64_body(E.part, E.nk2 ? E.t2_rows_of : E.rows_of, E.nk2 ? E.t2_ident : E.k_of_slot, E.M, E.N,
                 E.canon_of_lex, E.v, nullptr, E.csw, E.blk, u.idx);
}

template <int D>
__global__ void __launch_bounds__(kThreads) kb_grad64(const EvalSlot* __restrict__ es,
                                                      const BUnit* __restrict__ units, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  grad64_body<D>(E.runs, E.chunk_begin, E.tab, E.csw, E.N, E.R1, E.M, E.gpart, u.idx % E.pblocks,
                 (int)(u.idx / E.pblocks));
}

__global__ void __launch_bounds__(kThreads) kb_gcomb64(const EvalSlot* __restrict__ es,
                                                       const BUnit* __restrict__ units, int which, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  gcomb64_body(E.gpart, E.Q, E.d, E.N, E.L, E.L != 1.0, E.grad[which], (int64_t)u.idx * kThreads + threadIdx.x);
}

// ---------------------------------------------------------------------------
// launch helpers
// ---------------------------------------------------------------------------
template <int D, int PT>
static void launch_nk64_t(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units, int64_t nunits,
                          const double* tab, double* part, const SlotOffsets& so, hipStream_t st, const int* active) {
  const size_t lds = (size_t)PT * D * c.R1 * 2 * sizeof(double);
  hipLaunchKernelGGL((k_nk64<D, PT>), dim3((unsigned)nunits), dim3(kThreads), lds, st, segs, nseg, units, tab, c.N,
                     c.R1, part, c.M, so, active);
}

template <int D>
static void launch_nk64_d(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units, int64_t nunits,
                          const double* tab, double* part, const SlotOffsets& so, hipStream_t st, const int* active) {
  switch (c.pt) {
    case 16: launch_nk64_t<D, 16>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
    case 4: launch_nk64_t<D, 4>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
    default: launch_nk64_t<D, 1>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
  }
}

hipError_t launch_nk64(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units, int64_t nunits,
                       const double* tab, double* part, const SlotOffsets& so, hipStream_t st, const int* active) {
  switch (c.d) {
    case 1: launch_nk64_d<1>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
    case 2: launch_nk64_d<2>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
    case 3: launch_nk64_d<3>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
    default: launch_nk64_d<4>(c, segs, nseg, units, nunits, tab, part, so, st, active); break;
  }
  return hipGetLastError();
}

hipError_t launch_nk_combine64(const LaunchCfg& c, const double* part, const int32_t* rows_of,
                               const int32_t* k_of_slot, const int32_t* canon_of_lex, const double* v,
                               double* nk_out, double* csw, double* blk, hipStream_t st, const int* active) {
  hipLaunchKernelGGL(k_nk_combine64, dim3((unsigned)c.combine_blocks), dim3(kThreads), 0, st, part, rows_of,
                     k_of_slot, c.M, c.N, canon_of_lex, v, nk_out, csw, blk, active);
  return hipGetLastError();
}

hipError_t launch_grad64(const LaunchCfg& c, const Span* runs, const int32_t* chunk_begin, const double* tab,
                         const double* csw, double* gpart, hipStream_t st, const int* active) {
  const dim3 grid((unsigned)((c.N + 63) / 64), (unsigned)c.Q);
  switch (c.d) {
    case 1: hipLaunchKernelGGL((k_grad64<1>), grid, dim3(kThreads), 0, st, runs, chunk_begin, tab, csw, c.N, c.R1, c.M, gpart, active); break;
    case 2: hipLaunchKernelGGL((k_grad64<2>), grid, dim3(kThreads), 0, st, runs, chunk_begin, tab, csw, c.N, c.R1, c.M, gpart, active); break;
    case 3: hipLaunchKernelGGL((k_grad64<3>), grid, dim3(kThreads), 0, st, runs, chunk_begin, tab, csw, c.N, c.R1, c.M, gpart, active); break;
    default: hipLaunchKernelGGL((k_grad64<4>), grid, dim3(kThreads), 0, st, runs, chunk_begin, tab, csw, c.N, c.R1, c.M, gpart, active); break;
  }
  return hipGetLastError();
}

hipError_t launch_grad_combine64(const LaunchCfg& c, const double* gpart, double L, bool times_L, double* grad,
                                 hipStream_t st, const int* active) {
  const int64_t DN = (int64_t)c.d * c.N;
  hipLaunchKernelGGL(k_grad_combine64, dim3((unsigned)((DN + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                     gpart, c.Q, c.d, c.N, L, times_L ? 1 : 0, grad, active);
  return hipGetLastError();
}

hipError_t launch_batch_nk64(int d, int pt, int R1max, const EvalSlot* es, const BUnit* units, int64_t n, int gate,
                             hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const dim3 g((unsigned)n), b(kThreads);
#define SS_NK64(DD, P) \
  hipLaunchKernelGGL((kb_nk64<DD, P>), g, b, (size_t)P * DD * R1max * 2 * sizeof(double), st, es, units, gate)
  switch (d * 100 + pt) {
    case 116: SS_NK64(1, 16); break;
    case 104: SS_NK64(1, 4); break;
    case 101: SS_NK64(1, 1); break;
    case 216: SS_NK64(2, 16); break;
    case 204: SS_NK64(2, 4); break;
    case 201: SS_NK64(2, 1); break;
    case 316: SS_NK64(3, 16); break;
    case 304: SS_NK64(3, 4); break;
    case 301: SS_NK64(3, 1); break;
    case 416: SS_NK64(4, 16); break;
    case 404: SS_NK64(4, 4); break;
    default: SS_NK64(4, 1); break;
  }
#undef SS_NK64
  return hipGetLastError();
}

hipError_t launch_batch_nk2_64(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_nk2_64, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate);
  return hipGetLastError();
}

hipError_t launch_nk2_64(const int32_t* tiles, int64_t ntiles, const int32_t* lexinfo, int R, const double* tab,
                         int64_t N, int R1, int64_t chunk, int nrows, double* part, int64_t M, hipStream_t st,
                         const int* active) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nk2_64, dim3((unsigned)(ntiles * nrows)), dim3(kThreads), 0, st, tiles, lexinfo, R, tab, N,
                     R1, chunk, nrows, part, M, active);
  return hipGetLastError();
}

hipError_t launch_batch_combine64(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_combine64, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate);
  return hipGetLastError();
}

hipError_t launch_batch_grad64(int d, const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (d) {
    case 1: hipLaunchKernelGGL((kb_grad64<1>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
    case 2: hipLaunchKernelGGL((kb_grad64<2>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
    case 3: hipLaunchKernelGGL((kb_grad64<3>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
    default: hipLaunchKernelGGL((kb_grad64<4>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_gcomb64(const EvalSlot* es, const BUnit* units, int64_t n, int which, int gate,
                                hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_gcomb64, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, which, gate);
  return hipGetLastError();
}

}  // namespace ss
