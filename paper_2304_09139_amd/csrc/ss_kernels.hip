// ss_kernels.hip -- the double-double hot path on gfx950.
//
// Paper: Morse, Kim, Steinhardt, Torquato, "Generating large disordered
// stealthy hyperuniform systems with ultra-high accuracy ..." (arXiv:2304.09139).
//
// The energy needs, for every wavevector k = 2 pi n / L of the half set H and
// every particle j, the factor exp(i k.r_j) (Eq. ntilde and Eq. force; the
// "Simulations" paragraph counts both O(MN) sums as the whole cost).  With
// fractional coordinates u = r / L the factor is a product over axes,
//     exp(2 pi i n.u_j) = prod_a z_{j,a}^{n_a},   z_{j,a}^m = exp(2 pi i m u_{j,a}),
// so the kernels never form n.u per pair:
//   * k_table      builds z_{j,a}^m for m = 0..R by an exact reduction of
//                  m u mod 1 and a double-double sin/cos (the only
//                  transcendental work, O(d R N));
//   * k_nk         runs the n~(k) reduction.  Each lane owns a piece of one
//                  column (fixed n_0..n_{d-2}): up to kSegLen / 2 exponents t
//                  of the last axis and, where the column is symmetric, their
//                  negatives.  Per particle of a chunk whose tables are staged
//                  in LDS it forms the prefix b = prod z_a^{n_a} once and, for
//                  each t, b z^t and b conj(z^t) from four shared real products;
//   * k_nk2        (d = 2, large cutoffs) computes a 16 x 16 tile of
//                  wavevectors as products of two staged 16-row table slices;
//   * k_nk_combine sums the chunk partials in a fixed order with the accurate
//                  dd addition and forms v C, v S, Phi and S_max per block;
//   * k_grad       is the transposed gradient pass: each lane owns one particle
//                  and all lanes walk the same wavevector runs (uniform data),
//                  one complex product and a dd dot product per pair.
// All reductions have a fixed order: results are bitwise reproducible.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ss_dd.h"
#include "ss_internal.h"
#include "ss_min.h"
#include "ss_reduce.h"

namespace ss {

// ---------------------------------------------------------------------------
// table of z^m = exp(2 pi i m u) per particle and axis
// layout: tab[((a * R1 + m) * 4 + c) * N + j], c = (re.hi, re.lo, im.hi, im.lo)
// ---------------------------------------------------------------------------
__device__ __forceinline__ void table_body(const double* __restrict__ pos, int d, int64_t N, int R1,
                                           double* __restrict__ tab, int64_t idx) {
  // thread (a, group of kTabRun exponents m0 .. m0 + kTabRun - 1, particle j):
  // z^m0 and z by the exact reduction and the dd sin/cos, then z^m = z^(m-1) z
  const int groups = (R1 + kTabRun - 1) / kTabRun;
  const int64_t total = (int64_t)d * groups * N;
  if (idx >= total) return;
  const int64_t j = idx % N;
  const int64_t ag = idx / N;
  const int m0 = (int)(ag % groups) * kTabRun;
  const int a = (int)(ag / groups);
  const double uh = pos[(int64_t)a * N + j];
  const double ul = pos[(int64_t)(d + a) * N + j];
  cdd w, z;
  expi2pi2(phase_of((double)m0, uh, ul), phase_of(1.0, uh, ul), w, z);
  for (int t = 0; t < kTabRun && m0 + t < R1; ++t) {
    if (t > 0) w = cmul(w, z);
    double rh, rl, ih, il;
    fast_two_sum(w.rh, w.rl, rh, rl);
    fast_two_sum(w.ih, w.il, ih, il);
    const int64_t base = ((int64_t)(a * R1 + m0 + t) * 4) * N + j;
    tab[base] = rh;
    tab[base + N] = rl;
    tab[base + 2 * N] = ih;
    tab[base + 3 * N] = il;
  }
}

__global__ void __launch_bounds__(kThreads) k_table(const double* __restrict__ pos, int d, int64_t N, int R1,
                                                    double* __restrict__ tab, const int* __restrict__ active) {
  if (active && *active == 0) return;
  table_body(pos, d, N, R1, tab, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

// entry z_a^m of the particle table staged in LDS ([a][m][c] per particle),
// conjugated for negative exponents (z^-m = conj z^m for |z| = 1)
__device__ __forceinline__ cdd lds_entry(const double* tp, int R1, int a, int m) {
  const int mm = m < 0 ? -m : m;
  const double* e = tp + (a * R1 + mm) * 4;
  cdd z{e[0], e[1], e[2], e[3]};
  if (m < 0) z = cconj(z);
  return z;
}

// ---------------------------------------------------------------------------
// n~(k) partial sums.  One block per unit (a block of kNkPieces pieces, one per
// lane, over a particle range [j0, j1)); the particle tables of the range are
// staged through LDS PT particles at a time and every lane evaluates its piece
// over every staged particle.
// part[((row * 4) + c) * M + slot], c = (C.hi, C.lo, S.hi, S.lo), slot order.
//
// A piece is one column of H (a fixed prefix n_0 .. n_{d-2}) and exponents
// t = t0 .. t0 + L - 1 of its last axis (L <= kSegLen / 2).  Where the prefix is
// nonzero the column takes every last component in [-h, h], and the lane also
// takes the negatives -t: with b = prod_{a < d-1} z_a^{n_a} and u = z_{d-1}^t
// from the table, the two factors are b u and b conj(u), which share their four
// real products (cmul_pm).  Accumulators 2i and 2i + 1 hold t0 + i and -(t0 + i).
// Stored index i of the piece (slot off[i] + lane) holds accumulator
//   i      where t0 > 0,
//   0, i + 1 (i >= 1) where t0 = 0 (accumulator 1, "-0", repeats t = 0),
//   2 i    in the prefix-zero column (0, .., 0, t), t >= 1, whose negatives
//          are outside H.
// ---------------------------------------------------------------------------
// the staged particles of one tile for a wave whose widest piece spans L
// exponents: every lane takes L exponents (lanes with narrower pieces compute
// terms they never store; exponents past R are clamped into the table), fully
// unrolled with no per-lane branches
template <int D, int L>
__device__ __forceinline__ void nk_tile(const double* __restrict__ lds, int np, int epp, int R1, const Span& sg,
                                        double (&crh)[kSegLen], double (&crl)[kSegLen], double (&cih)[kSegLen],
                                        double (&cil)[kSegLen]) {
  const int t0 = sg.n[D - 1];
#pragma unroll 1
  for (int p = 0; p < np; ++p) {
    const double* tp = lds + p * epp;
    cdd b{1.0, 0.0, 0.0, 0.0};
    if constexpr (D > 1) {
      b = lds_entry(tp, R1, 0, sg.n[0]);
#pragma unroll
      for (int a = 1; a < D - 1; ++a) b = cmul(b, lds_entry(tp, R1, a, sg.n[a]));
    }
    // the entries z^t are read one exponent ahead of their products
    auto uent = [&](int i) {
      const int m = t0 + i < R1 ? t0 + i : R1 - 1;
      const double* e = tp + ((D - 1) * R1 + m) * 4;
      return cdd{e[0], e[1], e[2], e[3]};
    };
    cdd un = uent(0);
#pragma unroll
    for (int i = 0; i < L; ++i) {
      const cdd u = un;
      if (i + 1 < L) un = uent(i + 1);
      cdd wp, wm;
      cmul_pm(b, u, wp, wm);
      lazy_acc(crh[2 * i], crl[2 * i], wp.rh, wp.rl);
      lazy_acc(cih[2 * i], cil[2 * i], wp.ih, wp.il);
      lazy_acc(crh[2 * i + 1], crl[2 * i + 1], wm.rh, wm.rl);
      lazy_acc(cih[2 * i + 1], cil[2 * i + 1], wm.ih, wm.il);
    }
  }
}

// a unit's particle tiles and stores for a wave whose widest piece spans L
// exponents: the whole loop is instantiated per L, so that no accumulator is
// merged across the widths (waves of a block may take different L: each runs
// the same tiles and so the same barriers)
template <int D, int PT, int L>
__device__ __forceinline__ void nk_unit(const Span& sg, int64_t s, int len, bool plus, bool zero, const NkUnit u,
                                        const double* __restrict__ tab, int64_t N, int R1,
                                        double* __restrict__ part, int64_t M, const SlotOffsets& so,
                                        double* __restrict__ lds) {
  const int tid = threadIdx.x;
  const int epp = D * R1 * 4;  // doubles per particle
  double crh[kSegLen], crl[kSegLen], cih[kSegLen], cil[kSegLen];
#pragma unroll
  for (int t = 0; t < kSegLen; ++t) crh[t] = crl[t] = cih[t] = cil[t] = 0.0;
  const int64_t j0 = u.j0;
  const int64_t j1 = u.j1;
  for (int64_t tile = j0; tile < j1; tile += PT) {
    const int np = (int)((j1 - tile) < PT ? (j1 - tile) : PT);
    __syncthreads();
    for (int i = tid; i < epp * PT; i += kThreads) {
      const int p = i % PT;
      const int ec = i / PT;
      lds[p * epp + ec] = p < np ? tab[(int64_t)ec * N + tile + p] : 0.0;
    }
    __syncthreads();
    if constexpr (L > 0) nk_tile<D, L>(lds, np, epp, R1, sg, crh, crl, cih, cil);
#pragma unroll
    for (int t = 0; t < 2 * L; ++t) {
      renorm(crh[t], crl[t]);
      renorm(cih[t], cil[t]);
    }
  }
  // slot order: for each stored index the lanes of a wave write consecutive slots
  double* out = part + (int64_t)u.row * 4 * M;
#pragma unroll
  for (int t = 0; t < 2 * L; ++t) {
    if (t < len) {
      constexpr int kLast = 2 * L - 1 > 0 ? 2 * L - 1 : 0;
      const int q1 = t + 1 < kLast ? t + 1 : kLast, q2 = 2 * t < kLast ? 2 * t : kLast;
      double vrh = crh[t], vrl = crl[t], vih = cih[t], vil = cil[t];
      if (zero && t >= 1) vrh = crh[q1], vrl = crl[q1], vih = cih[q1], vil = cil[q1];
      if (plus) vrh = crh[q2], vrl = crl[q2], vih = cih[q2], vil = cil[q2];
      const int64_t slot = so.off[t] + s;
      out[slot] = vrh;
      out[M + slot] = vrl;
      out[2 * M + slot] = vih;
      out[3 * M + slot] = vil;
    }
  }
}

template <int D, int PT>
__device__ __forceinline__ void nk_body(const Span* __restrict__ segs, int64_t nseg, const NkUnit u,
                                        const double* __restrict__ tab, int64_t N, int R1,
                                        double* __restrict__ part, int64_t M, const SlotOffsets& so,
                                        double* __restrict__ lds) {
  const int tid = threadIdx.x;
  const int64_t s = (int64_t)u.block * kNkPieces + tid;
  const Span sg = segs[s < nseg ? s : nseg - 1];
  const int len = s < nseg ? sg.len : 0;
  bool plus = true;  // the prefix-zero column
#pragma unroll
  for (int a = 0; a < D - 1; ++a) plus = plus && sg.n[a] == 0;
  const bool zero = !plus && sg.n[D - 1] == 0;
  const int nt = plus ? len : (len + 1) / 2;  // exponents of this lane's piece
  // the widest piece of the wave, in a scalar register, selects the unit's loop
  int wmax = nt;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) wmax = max(wmax, __shfl_xor(wmax, o));
  const int wl = __builtin_amdgcn_readfirstlane(wmax);
  static_assert(kSegLen == 8, "the unit loops below cover widths 0 .. 4");
  switch (wl) {
    case 4: nk_unit<D, PT, 4>(sg, s, len, plus, zero, u, tab, N, R1, part, M, so, lds); break;
    case 3: nk_unit<D, PT, 3>(sg, s, len, plus, zero, u, tab, N, R1, part, M, so, lds); break;
    case 2: nk_unit<D, PT, 2>(sg, s, len, plus, zero, u, tab, N, R1, part, M, so, lds); break;
    case 1: nk_unit<D, PT, 1>(sg, s, len, plus, zero, u, tab, N, R1, part, M, so, lds); break;
    default: nk_unit<D, PT, 0>(sg, s, len, plus, zero, u, tab, N, R1, part, M, so, lds); break;
  }
}

template <int D, int PT>
__global__ void __launch_bounds__(kThreads, 3) k_nk(const Span* __restrict__ segs, int64_t nseg,
                                                 const NkUnit* __restrict__ units, const double* __restrict__ tab,
                                                 int64_t N, int R1, double* __restrict__ part, int64_t M,
                                                 const SlotOffsets so, const int* __restrict__ active) {
  if (active && *active == 0) return;
  extern __shared__ double lds[];  // [PT][D][R1][4]
  nk_body<D, PT>(segs, nseg, units[blockIdx.x], tab, N, R1, part, M, so, lds);
}

// ---------------------------------------------------------------------------
// n~(k) partial sums for d = 2 at large cutoffs, as a product of two table
// slices.  With the phase table, exp(2 pi i n.u_j) = z0_j^{n0} z1_j^{n1}, so a
// 16 x 16 tile of wavevectors (n0 in [a0, a0 + 16), n1 in [b0, b0 + 16)) over a
// particle chunk needs only 16 + 16 table rows per particle: the block stages
// them for 16 particles at a time (coalesced: 16 consecutive particles per row
// and component) and thread (i0, i1) adds z0^{n0} z1^{n1} -- one complex
// product per pair, no walk and no prefix products.  Thread t takes
// i0 = t / 16, i1 = t % 16; threads whose (n0, n1) is not in H idle.
// lexinfo[3 n0 + (0, 1, 2)] = walk position of (n0, lo), lo, hi: the n1 of H in
// row n0 are lo .. hi.  part[(row * 4 + c) * M + walk position].
// ---------------------------------------------------------------------------
constexpr int kT2 = 16;                 // tile side and particles per staged chunk
constexpr int kT2Pitch = kT2 * 4 + 2;   // doubles per staged particle (pad: no bank conflicts)

__device__ __forceinline__ void nk2_body(const int32_t* __restrict__ tiles, const int32_t* __restrict__ lexinfo,
                                         int R, const double* __restrict__ tab, int64_t N, int R1, int64_t chunk,
                                         int tile, int row, double* __restrict__ part, int64_t M) {
  __shared__ double s0[kT2 * kT2Pitch], s1[kT2 * kT2Pitch];  // [particle][row][re.h, re.l, im.h, im.l]
  const int tid = threadIdx.x;
  const int a0 = tiles[2 * tile], b0 = tiles[2 * tile + 1];
  const int i0 = tid / kT2, i1 = tid % kT2;
  const int n0 = a0 + i0, n1 = b0 + i1;
  int64_t pos = -1;
  if (n0 <= R) {
    const int off = lexinfo[3 * n0], lo = lexinfo[3 * n0 + 1], hi = lexinfo[3 * n0 + 2];
    if (n1 >= lo && n1 <= hi) pos = off + (n1 - lo);
  }
  const bool mine = pos >= 0;
  const bool neg = n1 < 0;
  double crh = 0.0, crl = 0.0, cih = 0.0, cil = 0.0;
  const int64_t j0 = (int64_t)row * chunk;
  const int64_t j1 = j0 + chunk < N ? j0 + chunk : N;
  // 2 slices x 16 rows x 4 components x 16 particles, particle fastest; the
  // next chunk's values are loaded into registers while the current one is used
  constexpr int kQ = (2 * kT2 * 4 * kT2) / kThreads;
  double pre[kQ];
  auto fetch = [&](int64_t tj) {
    const int np = (int)((j1 - tj) < kT2 ? (j1 - tj) : kT2);
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int idx = tid + kThreads * q;
      const int p = idx % kT2, c = (idx / kT2) % 4, r = (idx / (4 * kT2)) % kT2, ax = idx / (4 * kT2 * kT2);
      const int m = ax == 0 ? a0 + r : (b0 + r < 0 ? -(b0 + r) : b0 + r);
      pre[q] = (p < np && m <= R) ? tab[((int64_t)(ax * R1 + m) * 4 + c) * N + tj + p] : 0.0;
    }
  };
  if (j0 < j1) fetch(j0);
  for (int64_t tj = j0; tj < j1; tj += kT2) {
    const int np = (int)((j1 - tj) < kT2 ? (j1 - tj) : kT2);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kQ; ++q) {
      const int idx = tid + kThreads * q;
      const int p = idx % kT2, c = (idx / kT2) % 4, r = (idx / (4 * kT2)) % kT2, ax = idx / (4 * kT2 * kT2);
      (ax == 0 ? s0 : s1)[p * kT2Pitch + r * 4 + c] = pre[q];
    }
    __syncthreads();
    if (tj + kT2 < j1) fetch(tj + kT2);
    if (mine) {
#pragma unroll 4
      for (int p = 0; p < np; ++p) {
        const double* e0 = s0 + p * kT2Pitch + i0 * 4;
        const double* e1 = s1 + p * kT2Pitch + i1 * 4;
        cdd z1{e1[0], e1[1], e1[2], e1[3]};
        if (neg) z1 = cconj(z1);
        const cdd w = cmul(cdd{e0[0], e0[1], e0[2], e0[3]}, z1);
        lazy_acc(crh, crl, w.rh, w.rl);
        lazy_acc(cih, cil, w.ih, w.il);
      }
      renorm(crh, crl);
      renorm(cih, cil);
    }
  }
  if (mine) {
    double* out = part + (int64_t)row * 4 * M;
    out[pos] = crh;
    out[M + pos] = crl;
    out[2 * M + pos] = cih;
    out[3 * M + pos] = cil;
  }
}

__global__ void __launch_bounds__(kThreads) k_nk2(const int32_t* __restrict__ tiles,
                                                  const int32_t* __restrict__ lexinfo, int R,
                                                  const double* __restrict__ tab, int64_t N, int R1, int64_t chunk,
                                                  int nrows, double* __restrict__ part, int64_t M,
                                                  const int* __restrict__ active) {
  if (active && *active == 0) return;
  nk2_body(tiles, lexinfo, R, tab, N, R1, chunk, (int)(blockIdx.x / nrows), (int)(blockIdx.x % nrows), part, M);
}

// ---------------------------------------------------------------------------
// combine the P chunk partials per wavevector (fixed order, accurate dd sums);
// write n~ in canonical order, (v C, v S) in walk order, and per-block Phi and
// S_max partials.  Block b covers slots b kCombK .. (b + 1) kCombK - 1 (reads of
// consecutive slots are contiguous).  blk[b * 5 + (0..4)] = Phi.hi, Phi.lo,
// Smax.hi, Smax.lo, canonical index of the maximum
// ---------------------------------------------------------------------------
__device__ __forceinline__ void combine_body(const double* __restrict__ part, const int32_t* __restrict__ rows_of,
                                             const int32_t* __restrict__ k_of_slot, int64_t M, int64_t N,
                                             const int32_t* __restrict__ canon_of_lex, const double* __restrict__ v,
                                             double* __restrict__ nk_out, double* __restrict__ csw,
                                             double* __restrict__ blk, int64_t bidx) {
  // thread (q, g): slot i = bidx * kCombK + q; partial group g sums rows
  // g, g + kCombG, ...; the groups are then added pairwise in a fixed tree
  constexpr int kCombG = kThreads / kCombK;
  __shared__ double s_c[kCombG][4][kCombK];
  __shared__ double s_ph[kCombK], s_pl[kCombK], s_mh[kCombK], s_ml[kCombK];
  __shared__ int64_t s_mk[kCombK];
  const int tid = threadIdx.x, q = tid % kCombK, g = tid / kCombK;
  const int64_t i = bidx * kCombK + q;
  dd C{0.0, 0.0}, S{0.0, 0.0};
  if (i < M) {
    const int64_t P = rows_of[i];
    for (int64_t p = g; p < P; p += kCombG) {
      const double* r = part + p * 4 * M;
      C = dd_add(C, dd{r[i], r[M + i]});
      S = dd_add(S, dd{r[2 * M + i], r[3 * M + i]});
    }
  }
  s_c[g][0][q] = C.h;
  s_c[g][1][q] = C.l;
  s_c[g][2][q] = S.h;
  s_c[g][3][q] = S.l;
  __syncthreads();
  for (int w = kCombG / 2; w > 0; w >>= 1) {
    if (g < w) {
      const dd c = dd_add(dd{s_c[g][0][q], s_c[g][1][q]}, dd{s_c[g + w][0][q], s_c[g + w][1][q]});
      const dd sn = dd_add(dd{s_c[g][2][q], s_c[g][3][q]}, dd{s_c[g + w][2][q], s_c[g + w][3][q]});
      s_c[g][0][q] = c.h;
      s_c[g][1][q] = c.l;
      s_c[g][2][q] = sn.h;
      s_c[g][3][q] = sn.l;
    }
    __syncthreads();
  }
  if (g == 0) {
    C = dd{s_c[0][0][q], s_c[0][1][q]};
    S = dd{s_c[0][2][q], s_c[0][3][q]};
    dd phi{0.0, 0.0}, sk{-1.0, 0.0};
    int64_t kc = INT64_MAX;
    if (i < M) {
      const int64_t k = k_of_slot[i];
      kc = canon_of_lex[k];
      if (nk_out) {
        nk_out[kc] = C.h;
        nk_out[M + kc] = C.l;
        nk_out[2 * M + kc] = S.h;
        nk_out[3 * M + kc] = S.l;
      }
      const dd w = v ? dd{v[kc], v[M + kc]} : dd{1.0, 0.0};
      const dd Cw = v ? dd_mul(w, C) : C;
      const dd Sw = v ? dd_mul(w, S) : S;
      csw[k] = Cw.h;
      csw[M + k] = Cw.l;
      csw[2 * M + k] = Sw.h;
      csw[3 * M + k] = Sw.l;
      const dd mag = dd_add(dd_mul(C, C), dd_mul(S, S));
      phi = v ? dd_mul(w, mag) : mag;
      sk = dd_div_d(mag, (double)N);
    }
    s_ph[q] = phi.h;
    s_pl[q] = phi.l;
    s_mh[q] = sk.h;
    s_ml[q] = sk.l;
    s_mk[q] = kc;
  }
  __syncthreads();
  for (int w = kCombK / 2; w > 0; w >>= 1) {
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
  if (tid == 0) {
    double* b = blk + bidx * 5;
    b[0] = s_ph[0];
    b[1] = s_pl[0];
    b[2] = s_mh[0];
    b[3] = s_ml[0];
    b[4] = (double)s_mk[0];
  }
}

__global__ void __launch_bounds__(kThreads) k_nk_combine(const double* __restrict__ part,
                                                         const int32_t* __restrict__ rows_of,
                                                         const int32_t* __restrict__ k_of_slot, int64_t M,
                                                         int64_t N, const int32_t* __restrict__ canon_of_lex,
                                                         const double* __restrict__ v, double* __restrict__ nk_out,
                                                         double* __restrict__ csw, double* __restrict__ blk,
                                                         const int* __restrict__ active) {
  if (active && *active == 0) return;
  combine_body(part, rows_of, k_of_slot, M, N, canon_of_lex, v, nk_out, csw, blk, blockIdx.x);
}

// single block: fixed-order reduction of the per-block partials
__global__ void __launch_bounds__(kThreads) k_final(const double* __restrict__ blk, int64_t nblk,
                                                    double* __restrict__ phi_out, double* __restrict__ smax_out,
                                                    double* __restrict__ kmax_out,
                                                    const int* __restrict__ active) {
  if (active && *active == 0) return;
  dd phi, sm;
  double kk;
  reduce_energy_partials(blk, nblk, &phi, &sm, &kk);
  if (threadIdx.x == 0) {
    phi_out[0] = phi.h;
    phi_out[1] = phi.l;
    smax_out[0] = sm.h;
    smax_out[1] = sm.l;
    if (kmax_out) kmax_out[0] = kk;
  }
}

// ---------------------------------------------------------------------------
// gradient partials.  grid = (particle blocks, wavevector chunks).
// gpart[((q * 2 + plane) * D + a) * N + j]
// ---------------------------------------------------------------------------
__device__ __forceinline__ cdd tab_entry(const double* __restrict__ tab, int64_t N, int R1, int a, int m, int64_t j) {
  const int mm = m < 0 ? -m : m;
  const double* e = tab + ((int64_t)(a * R1 + mm) * 4) * N + j;
  cdd z{e[0], e[N], e[2 * N], e[3 * N]};
  if (m < 0) z = cconj(z);
  return z;
}

template <int D>
__device__ __forceinline__ void grad_body(const Span* __restrict__ runs, const int32_t* __restrict__ chunk_begin,
                                          const double* __restrict__ tab, const double* __restrict__ csw,
                                          int64_t N, int R1, int64_t M, double* __restrict__ gpart, int64_t pblock,
                                          int q) {
  __shared__ double s_g[kWaves][2 * D][64];
  const int tid = threadIdx.x, lane = tid & 63;
  // the wave index is uniform across the wave: in a scalar register the run
  // bounds, the run records and the per-wavevector (vC, vS) become scalar loads
  // and the wavevector loop is a scalar loop
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t j = pblock * 64 + lane;
  const int64_t jj = j < N ? j : N - 1;
  const int r0 = chunk_begin[kWaves * q + wave], r1 = chunk_begin[kWaves * q + wave + 1];
  const cdd z = tab_entry(tab, N, R1, D - 1, 1, jj);
  double gh[D], gl[D];
#pragma unroll
  for (int a = 0; a < D; ++a) gh[a] = gl[a] = 0.0;

  for (int r = r0; r < r1; ++r) {
    const Span run = runs[r];
    cdd w = tab_entry(tab, N, R1, D - 1, run.n[D - 1], jj);
#pragma unroll
    for (int a = 0; a < D - 1; ++a) w = cmul(w, tab_entry(tab, N, R1, a, run.n[a], jj));
    // q_t = v (S c - C s) along the run; P = sum_t q_t and the sum of the prefix
    // sums PP = sum_t P_t give sum_t (n0 + t) q_t = (n0 + len) P - PP without a
    // product per pair
    double q0h = 0.0, q0l = 0.0, pph = 0.0, ppl = 0.0;
    const double* cp = csw + run.k0;
#pragma unroll 2
    for (int t = 0; t < run.len; ++t) {
      const double Ch = cp[t], Cl = cp[M + t], Sh = cp[2 * M + t], Sl = cp[3 * M + t];
      double qs, qt;
      lazy_dot2m(Sh, Sl, w.rh, w.rl, Ch, Cl, w.ih, w.il, qs, qt);  // v (S c - C s)
      lazy_acc(q0h, q0l, qs, qt);
      lazy_acc(pph, ppl, q0h, q0l);
      w = cmul(w, z);
    }
    renorm(q0h, q0l);
    renorm(pph, ppl);
    double qdh, qdl;
    {
      const double nl = (double)(run.n[D - 1] + run.len);
      double p = nl * q0h;
      double e = __builtin_fma(nl, q0h, -p);
      e = __builtin_fma(nl, q0l, e);
      const dd r = dd_sub(dd_norm(p, e), dd{pph, ppl});
      qdh = r.h;
      qdl = r.l;
    }
#pragma unroll
    for (int a = 0; a < D - 1; ++a) {
      const double na = (double)run.n[a];
      double p = na * q0h;
      double e = __builtin_fma(na, q0h, -p);
      e = __builtin_fma(na, q0l, e);
      lazy_acc(gh[a], gl[a], p, e);
      renorm(gh[a], gl[a]);
    }
    lazy_acc(gh[D - 1], gl[D - 1], qdh, qdl);
    renorm(gh[D - 1], gl[D - 1]);
  }
#pragma unroll
  for (int a = 0; a < D; ++a) {
    s_g[wave][2 * a][lane] = gh[a];
    s_g[wave][2 * a + 1][lane] = gl[a];
  }
  __syncthreads();
  if (wave == 0 && j < N) {  // ((w0 + w2) + (w1 + w3))
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const dd x02 = dd_add(dd{s_g[0][2 * a][lane], s_g[0][2 * a + 1][lane]},
                            dd{s_g[2][2 * a][lane], s_g[2][2 * a + 1][lane]});
      const dd x13 = dd_add(dd{s_g[1][2 * a][lane], s_g[1][2 * a + 1][lane]},
                            dd{s_g[3][2 * a][lane], s_g[3][2 * a + 1][lane]});
      const dd g = dd_add(x02, x13);
      gpart[((int64_t)(q * 2 + 0) * D + a) * N + j] = g.h;
      gpart[((int64_t)(q * 2 + 1) * D + a) * N + j] = g.l;
    }
  }
}

template <int D>
__global__ void __launch_bounds__(kThreads, 5) k_grad(const Span* __restrict__ runs,
                                                   const int32_t* __restrict__ chunk_begin,
                                                   const double* __restrict__ tab, const double* __restrict__ csw,
                                                   int64_t N, int R1, int64_t M, double* __restrict__ gpart, int Q,
                                                   const int* __restrict__ active) {
  if (active && *active == 0) return;
  // XCD-aware order: workgroups go to the 8 XCDs round-robin by linear index,
  // so block b runs on XCD b % 8; it takes particle block 8 k' + (b % 8) with
  // k = b / 8 = k' Q + q, i.e. every chunk q of one particle block runs on the
  // same XCD and the particle tables are fetched into one L2 only
  const int64_t b = blockIdx.x;
  const int64_t k = b / kXcds;
  const int64_t pblock = (k / Q) * kXcds + (b % kXcds);
  const int q = (int)(k % Q);
  if (pblock * 64 >= N) return;
  grad_body<D>(runs, chunk_begin, tab, csw, N, R1, M, gpart, pblock, q);
}

// sum the Q gradient partials (fixed order) and scale by 4 pi / L:
// dPhi/dr_{j,a} = (4 pi / L) sum_k v_k n_{k,a} (S_k c_jk - C_k s_jk); with
// times_L the result is then multiplied by L (the gradient with respect to the
// fractional coordinates, as the minimiser uses it)
__device__ __forceinline__ void gcomb_body(const double* __restrict__ gpart, int Q, int d, int64_t N, double L,
                                           bool times_L, double* __restrict__ grad, int64_t i) {
  const int64_t DN = (int64_t)d * N;
  if (i >= DN) return;
  dd g{0.0, 0.0};
  for (int q = 0; q < Q; ++q) g = dd_add(g, dd{gpart[(int64_t)(q * 2) * DN + i], gpart[(int64_t)(q * 2 + 1) * DN + i]});
  const dd tp = two_pi_dd();
  const dd scale = dd_div_d(dd{2.0 * tp.h, 2.0 * tp.l}, L);
  g = dd_mul(g, scale);
  if (times_L) g = dd_mul_d(g, L);
  grad[i] = g.h;
  grad[DN + i] = g.l;
}

__global__ void __launch_bounds__(kThreads) k_grad_combine(const double* __restrict__ gpart, int Q, int d, int64_t N,
                                                           double L, double* __restrict__ grad,
                                                           const int* __restrict__ active) {
  if (active && *active == 0) return;
  gcomb_body(gpart, Q, d, N, L, false, grad, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

// ---------------------------------------------------------------------------
// batched launches: one grid covers the blocks of many configurations; block
// b runs block units[b].idx of configuration units[b].slot's own grid, with the
// same arithmetic and order as the single-configuration kernels, so a
// configuration's results do not depend on what else is in the batch.  With
// gate != 0 the blocks of a configuration whose quench has stopped exit at once.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kThreads) kb_table(const EvalSlot* __restrict__ es,
                                                     const BUnit* __restrict__ units, int which, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  table_body(E.pos[which], E.d, E.N, E.R1, E.tab, (int64_t)u.idx * kThreads + threadIdx.x);
}

template <int D, int PT>
__global__ void __launch_bounds__(kThreads, 3) kb_nk(const EvalSlot* __restrict__ es, const BUnit* __restrict__ units,
                                                  int gate) {
  extern __shared__ double lds[];  // [PT][D][R1][4], sized for the largest R1 of the launch
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  nk_body<D, PT>(E.segs, E.nsegs, E.units[u.idx], E.tab, E.N, E.R1, E.part, E.M, E.so, lds);
}

// the tiled d = 2 pass (configurations with E.nk2): unit idx = tile * rows + row
__global__ void __launch_bounds__(kThreads) kb_nk2(const EvalSlot* __restrict__ es, const BUnit* __restrict__ units,
                                                   int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  nk2_body(E.t2_tiles, E.t2_lexinfo, E.R, E.tab, E.N, E.R1, E.t2_chunk, u.idx / E.t2_nrows, u.idx % E.t2_nrows,
           E.part, E.M);
}

// double-double partials: of the tiled pass (by walk position) or of the piece walk
__global__ void __launch_bounds__(kThreads) kb_combine(const EvalSlot* __restrict__ es,
                                                       const BUnit* __restrict__ units, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  combine_body(E.part, E.nk2 ? E.t2_rows_of : E.rows_of, E.nk2 ? E.t2_ident : E.k_of_slot, E.M, E.N,
               E.canon_of_lex, E.v, nullptr, E.csw, E.blk, u.idx);
}

// one block per listed configuration: Phi and S_max of the iterate
__global__ void __launch_bounds__(kThreads) kb_final(const EvalSlot* __restrict__ es,
                                                     const int32_t* __restrict__ list) {
  const EvalSlot& E = es[list[blockIdx.x]];
  dd phi, sm;
  double kk;
  reduce_energy_partials(E.blk, E.combine_blocks, &phi, &sm, &kk);
  if (threadIdx.x == 0) {
    E.phi[0] = phi.h;
    E.phi[1] = phi.l;
    E.smax[0] = sm.h;
    E.smax[1] = sm.l;
  }
}

template <int D>
__global__ void __launch_bounds__(kThreads) kb_grad(const EvalSlot* __restrict__ es, const BUnit* __restrict__ units,
                                                    int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  const int64_t pblock = u.idx % E.pblocks;
  const int q = (int)(u.idx / E.pblocks);
  grad_body<D>(E.runs, E.chunk_begin, E.tab, E.csw, E.N, E.R1, E.M, E.gpart, pblock, q);
}

__global__ void __launch_bounds__(kThreads) kb_gcomb(const EvalSlot* __restrict__ es,
                                                     const BUnit* __restrict__ units, int which, int gate) {
  const BUnit u = units[blockIdx.x];
  const EvalSlot& E = es[u.slot];
  if (gate && *E.running == 0) return;
  gcomb_body(E.gpart, E.Q, E.d, E.N, E.L, E.L != 1.0, E.grad[which], (int64_t)u.idx * kThreads + threadIdx.x);
}

// ---------------------------------------------------------------------------
// wavevector enumeration (integer, bit-exact)
// candidates are the lexicographically ordered grid [-R, R]^d
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool candidate(int64_t idx, int d, int R, int64_t R2, int32_t* n, int64_t* shell) {
  const int64_t side = 2 * R + 1;
  int64_t rem = idx, s = 0;
  for (int a = d - 1; a >= 0; --a) {
    n[a] = (int32_t)(rem % side) - R;
    rem /= side;
  }
  int first = 0;
  for (int a = 0; a < d; ++a) {
    s += (int64_t)n[a] * n[a];
    if (first == 0 && n[a] != 0) first = n[a] > 0 ? 1 : -1;
  }
  *shell = s;
  return s <= R2 && first > 0;  // half set: first nonzero component positive
}

constexpr int kEnumPer = 1024;  // candidates per block

__global__ void __launch_bounds__(kThreads) k_enum_count(int64_t total, int d, int R, int64_t R2,
                                                         int32_t* __restrict__ bcount) {
  __shared__ int s_cnt;
  if (threadIdx.x == 0) s_cnt = 0;
  __syncthreads();
  int c = 0;
  int32_t n[4];
  int64_t sh;
  const int64_t base = (int64_t)blockIdx.x * kEnumPer;
  for (int i = threadIdx.x; i < kEnumPer; i += kThreads) {
    const int64_t idx = base + i;
    if (idx < total && candidate(idx, d, R, R2, n, &sh)) ++c;
  }
  atomicAdd(&s_cnt, c);  // integer: order-independent
  __syncthreads();
  if (threadIdx.x == 0) bcount[blockIdx.x] = s_cnt;
}

__global__ void k_enum_scan(const int32_t* __restrict__ bcount, int64_t nb, int32_t* __restrict__ bofs,
                            int64_t* __restrict__ total_out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    int64_t acc = 0;
    for (int64_t b = 0; b < nb; ++b) {
      bofs[b] = (int32_t)acc;
      acc += bcount[b];
    }
    *total_out = acc;
  }
}

// stable scatter in lexicographic order; key = (|n|^2 << 32) | lex position
__global__ void __launch_bounds__(kThreads) k_enum_scatter(int64_t total, int d, int R, int64_t R2,
                                                           const int32_t* __restrict__ bofs,
                                                           int32_t* __restrict__ lex_n, uint64_t* __restrict__ keys) {
  __shared__ int s_flag[kEnumPer];
  __shared__ int s_pos[kEnumPer];
  const int64_t base = (int64_t)blockIdx.x * kEnumPer;
  int32_t n[4];
  int64_t sh;
  for (int i = threadIdx.x; i < kEnumPer; i += kThreads) {
    const int64_t idx = base + i;
    s_flag[i] = (idx < total && candidate(idx, d, R, R2, n, &sh)) ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {  // exclusive scan of the block's flags (1024 entries)
    int acc = 0;
    for (int i = 0; i < kEnumPer; ++i) {
      s_pos[i] = acc;
      acc += s_flag[i];
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kEnumPer; i += kThreads) {
    if (!s_flag[i]) continue;
    const int64_t idx = base + i;
    candidate(idx, d, R, R2, n, &sh);
    const int64_t pos = (int64_t)bofs[blockIdx.x] + s_pos[i];
    for (int a = 0; a < d; ++a) lex_n[pos * d + a] = n[a];
    keys[pos] = ((uint64_t)sh << 32) | (uint64_t)pos;
  }
}

__global__ void __launch_bounds__(kThreads) k_fill_keys(uint64_t* __restrict__ keys, int64_t from, int64_t to) {
  const int64_t i = from + (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i < to) keys[i] = ~(uint64_t)0;
}

// one compare-exchange stage of a bitonic sort (keys are unique)
__global__ void __launch_bounds__(kThreads) k_bitonic(uint64_t* __restrict__ keys, int64_t n, int64_t j, int64_t k) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= n) return;
  const int64_t l = i ^ j;
  if (l > i) {
    const uint64_t a = keys[i], b = keys[l];
    const bool up = (i & k) == 0;
    if ((up && a > b) || (!up && a < b)) {
      keys[i] = b;
      keys[l] = a;
    }
  }
}

__global__ void __launch_bounds__(kThreads) k_enum_canon(const uint64_t* __restrict__ keys, int64_t M, int d,
                                                         const int32_t* __restrict__ lex_n,
                                                         int32_t* __restrict__ canon_n,
                                                         int32_t* __restrict__ canon_of_lex) {
  const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (i >= M) return;
  const int64_t lp = (int64_t)(keys[i] & 0xffffffffull);
  for (int a = 0; a < d; ++a) canon_n[i * d + a] = lex_n[lp * d + a];
  canon_of_lex[lp] = (int32_t)i;
}

// v_k = (1 - |k|/K)^2 with K^2 = (R2 + 1/2)(2 pi/L)^2, written without
// cancellation as ((K^2 - |n|^2) / (K^2 (1 + |n|/K)))^2 in units of (2 pi/L)
__global__ void __launch_bounds__(kThreads) k_weights(const int32_t* __restrict__ n, int64_t M, int d, int64_t R2,
                                                      int vkind, double* __restrict__ v) {
  const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (k >= M) return;
  dd w{1.0, 0.0};
  if (vkind == 1) {
    int64_t s = 0;
    for (int a = 0; a < d; ++a) s += (int64_t)n[k * d + a] * n[k * d + a];
    const double K2 = (double)R2 + 0.5;
    const dd root = dd_sqrt(dd_div(dd{(double)s, 0.0}, dd{K2, 0.0}));
    const dd den = dd_mul_d(dd_add(dd{1.0, 0.0}, root), K2);
    const dd om = dd_div(dd{K2 - (double)s, 0.0}, den);
    w = dd_mul(om, om);
  }
  v[k] = w.h;
  v[M + k] = w.l;
}

// ---------------------------------------------------------------------------
// host-side launch helpers
// ---------------------------------------------------------------------------
hipError_t launch_table(const double* pos, int d, int64_t N, int R1, double* tab, hipStream_t st,
                        const int* active) {
  const int64_t total = (int64_t)d * ((R1 + kTabRun - 1) / kTabRun) * N;
  const int64_t blocks = (total + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(k_table, dim3((unsigned)blocks), dim3(kThreads), 0, st, pos, d, N, R1, tab, active);
  return hipGetLastError();
}

template <int D, int PT>
static hipError_t launch_nk_t(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units,
                              int64_t nunits, const double* tab, double* part, const SlotOffsets& so, hipStream_t st,
                              const int* active) {
  const size_t lds = (size_t)PT * D * c.R1 * 4 * sizeof(double);
  hipLaunchKernelGGL((k_nk<D, PT>), dim3((unsigned)nunits), dim3(kThreads), lds, st, segs, nseg, units, tab, c.N,
                     c.R1, part, c.M, so, active);
  return hipGetLastError();
}

template <int D>
static hipError_t launch_nk_d(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units,
                              int64_t nunits, const double* tab, double* part, const SlotOffsets& so, hipStream_t st,
                              const int* active) {
  switch (c.pt) {
    case 16: return launch_nk_t<D, 16>(c, segs, nseg, units, nunits, tab, part, so, st, active);
    case 4: return launch_nk_t<D, 4>(c, segs, nseg, units, nunits, tab, part, so, st, active);
    default: return launch_nk_t<D, 1>(c, segs, nseg, units, nunits, tab, part, so, st, active);
  }
}

hipError_t launch_nk(const LaunchCfg& c, const Span* segs, int64_t nseg, const NkUnit* units, int64_t nunits,
                     const double* tab, double* part, const SlotOffsets& so, hipStream_t st, const int* active) {
  switch (c.d) {
    case 1: return launch_nk_d<1>(c, segs, nseg, units, nunits, tab, part, so, st, active);
    case 2: return launch_nk_d<2>(c, segs, nseg, units, nunits, tab, part, so, st, active);
    case 3: return launch_nk_d<3>(c, segs, nseg, units, nunits, tab, part, so, st, active);
    default: return launch_nk_d<4>(c, segs, nseg, units, nunits, tab, part, so, st, active);
  }
}

hipError_t launch_batch_nk2(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_nk2, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate);
  return hipGetLastError();
}

hipError_t launch_nk2(const int32_t* tiles, int64_t ntiles, const int32_t* lexinfo, int R, const double* tab,
                      int64_t N, int R1, int64_t chunk, int nrows, double* part, int64_t M, hipStream_t st,
                      const int* active) {
  if (ntiles <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_nk2, dim3((unsigned)(ntiles * nrows)), dim3(kThreads), 0, st, tiles, lexinfo, R, tab, N, R1,
                     chunk, nrows, part, M, active);
  return hipGetLastError();
}

int nk2_blocks_per_cu() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_nk2, kThreads, 0) != hipSuccess) b = 1;
  return b > 0 ? b : 1;
}

hipError_t launch_nk_combine(const LaunchCfg& c, const double* part, const int32_t* rows_of,
                             const int32_t* k_of_slot, const int32_t* canon_of_lex, const double* v, double* nk_out,
                             double* csw, double* blk, hipStream_t st, const int* active) {
  hipLaunchKernelGGL(k_nk_combine, dim3((unsigned)c.combine_blocks), dim3(kThreads), 0, st, part, rows_of, k_of_slot,
                     c.M, c.N, canon_of_lex, v, nk_out, csw, blk, active);
  return hipGetLastError();
}

hipError_t launch_final(const LaunchCfg& c, const double* blk, double* phi, double* smax, double* kmax, hipStream_t st,
                        const int* active) {
  hipLaunchKernelGGL(k_final, dim3(1), dim3(kThreads), 0, st, blk, c.combine_blocks, phi, smax, kmax, active);
  return hipGetLastError();
}

template <int D>
static hipError_t launch_grad_d(const LaunchCfg& c, const Span* runs, const int32_t* chunk_begin, const double* tab,
                                const double* csw, double* gpart, hipStream_t st, const int* active) {
  // particle blocks padded to a multiple of the XCD count (the padding exits)
  const int64_t pblocks = ((c.N + 63) / 64 + kXcds - 1) / kXcds * kXcds;
  hipLaunchKernelGGL((k_grad<D>), dim3((unsigned)(pblocks * c.Q)), dim3(kThreads), 0, st, runs, chunk_begin, tab,
                     csw, c.N, c.R1, c.M, gpart, c.Q, active);
  return hipGetLastError();
}

hipError_t launch_grad(const LaunchCfg& c, const Span* runs, const int32_t* chunk_begin, const double* tab,
                       const double* csw, double* gpart, hipStream_t st, const int* active) {
  switch (c.d) {
    case 1: return launch_grad_d<1>(c, runs, chunk_begin, tab, csw, gpart, st, active);
    case 2: return launch_grad_d<2>(c, runs, chunk_begin, tab, csw, gpart, st, active);
    case 3: return launch_grad_d<3>(c, runs, chunk_begin, tab, csw, gpart, st, active);
    default: return launch_grad_d<4>(c, runs, chunk_begin, tab, csw, gpart, st, active);
  }
}

hipError_t launch_grad_combine(const LaunchCfg& c, const double* gpart, double L, double* grad, hipStream_t st,
                               const int* active) {
  const int64_t DN = (int64_t)c.d * c.N;
  hipLaunchKernelGGL(k_grad_combine, dim3((unsigned)((DN + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, gpart,
                     c.Q, c.d, c.N, L, grad, active);
  return hipGetLastError();
}

// batched launch helpers (n = number of units; nothing is launched for n = 0)
hipError_t launch_batch_table(const EvalSlot* es, const BUnit* units, int64_t n, int which, int gate,
                              hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_table, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, which, gate);
  return hipGetLastError();
}

template <int D>
static hipError_t launch_batch_nk_d(int pt, int R1max, const EvalSlot* es, const BUnit* units, int64_t n, int gate,
                                    hipStream_t st) {
  const size_t lds = (size_t)pt * D * R1max * 4 * sizeof(double);
  switch (pt) {
    case 16: hipLaunchKernelGGL((kb_nk<D, 16>), dim3((unsigned)n), dim3(kThreads), lds, st, es, units, gate); break;
    case 4: hipLaunchKernelGGL((kb_nk<D, 4>), dim3((unsigned)n), dim3(kThreads), lds, st, es, units, gate); break;
    default: hipLaunchKernelGGL((kb_nk<D, 1>), dim3((unsigned)n), dim3(kThreads), lds, st, es, units, gate); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_nk(int d, int pt, int R1max, const EvalSlot* es, const BUnit* units, int64_t n, int gate,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (d) {
    case 1: return launch_batch_nk_d<1>(pt, R1max, es, units, n, gate, st);
    case 2: return launch_batch_nk_d<2>(pt, R1max, es, units, n, gate, st);
    case 3: return launch_batch_nk_d<3>(pt, R1max, es, units, n, gate, st);
    default: return launch_batch_nk_d<4>(pt, R1max, es, units, n, gate, st);
  }
}

hipError_t launch_batch_combine(const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_combine, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate);
  return hipGetLastError();
}

hipError_t launch_batch_final(const EvalSlot* es, const int32_t* list, int64_t n, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_final, dim3((unsigned)n), dim3(kThreads), 0, st, es, list);
  return hipGetLastError();
}

hipError_t launch_batch_grad(int d, const EvalSlot* es, const BUnit* units, int64_t n, int gate, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  switch (d) {
    case 1: hipLaunchKernelGGL((kb_grad<1>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
    case 2: hipLaunchKernelGGL((kb_grad<2>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
    case 3: hipLaunchKernelGGL((kb_grad<3>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
    default: hipLaunchKernelGGL((kb_grad<4>), dim3((unsigned)n), dim3(kThreads), 0, st, es, units, gate); break;
  }
  return hipGetLastError();
}

hipError_t launch_batch_gcomb(const EvalSlot* es, const BUnit* units, int64_t n, int which, int gate,
                              hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(kb_gcomb, dim3((unsigned)n), dim3(kThreads), 0, st, es, units, which, gate);
  return hipGetLastError();
}

// resident blocks per CU of the two pair kernels (for grid sizing in whole rounds)
template <int D>
static int grad_bpc_d() {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_grad<D>, kThreads, 0) != hipSuccess) b = 1;
  return b > 0 ? b : 1;
}
int grad_blocks_per_cu(int d) {
  switch (d) {
    case 1: return grad_bpc_d<1>();
    case 2: return grad_bpc_d<2>();
    case 3: return grad_bpc_d<3>();
    default: return grad_bpc_d<4>();
  }
}
template <int D, int PT>
static int nk_bpc_t(size_t lds) {
  int b = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k_nk<D, PT>, kThreads, lds) != hipSuccess) b = 1;
  return b > 0 ? b : 1;
}
template <int D>
static int nk_bpc_d(int pt, int R1) {
  const size_t lds = (size_t)pt * D * R1 * 4 * sizeof(double);
  switch (pt) {
    case 16: return nk_bpc_t<D, 16>(lds);
    case 4: return nk_bpc_t<D, 4>(lds);
    default: return nk_bpc_t<D, 1>(lds);
  }
}
int nk_blocks_per_cu(int d, int pt, int R1) {
  switch (d) {
    case 1: return nk_bpc_d<1>(pt, R1);
    case 2: return nk_bpc_d<2>(pt, R1);
    case 3: return nk_bpc_d<3>(pt, R1);
    default: return nk_bpc_d<4>(pt, R1);
  }
}

hipError_t launch_weights(const int32_t* n, int64_t M, int d, int64_t R2, int vkind, double* v, hipStream_t st) {
  hipLaunchKernelGGL(k_weights, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, n, M, d, R2,
                     vkind, v);
  return hipGetLastError();
}

// Enumerate H(R2): lexicographic list + canonical list + lex -> canonical map.
// Device buffers are allocated here; M is returned (a synchronising call).  The
// scratch buffers are freed on every path; on failure the plan's lists are left
// for the caller's plan release (which frees whatever is non-null).
hipError_t enumerate(int d, int64_t R2, int R, hipStream_t st, Plan* pl) {
  int64_t side = 2 * R + 1, total = 1;
  for (int a = 0; a < d; ++a) total *= side;
  const int64_t nb = (total + kEnumPer - 1) / kEnumPer;
  int32_t *bcount = nullptr, *bofs = nullptr;
  int64_t* dM = nullptr;
  uint64_t* keys = nullptr;
  hipError_t e = hipSuccess;
  int64_t M = 0, P2 = 1;
  unsigned sb = 0;
  if ((e = hipMalloc(&bcount, sizeof(int32_t) * nb)) != hipSuccess) goto done;
  if ((e = hipMalloc(&bofs, sizeof(int32_t) * nb)) != hipSuccess) goto done;
  if ((e = hipMalloc(&dM, sizeof(int64_t))) != hipSuccess) goto done;
  hipLaunchKernelGGL(k_enum_count, dim3((unsigned)nb), dim3(kThreads), 0, st, total, d, R, R2, bcount);
  hipLaunchKernelGGL(k_enum_scan, dim3(1), dim3(1), 0, st, bcount, nb, bofs, dM);
  if ((e = hipMemcpyAsync(&M, dM, sizeof(int64_t), hipMemcpyDeviceToHost, st)) != hipSuccess) goto done;
  if ((e = hipStreamSynchronize(st)) != hipSuccess) goto done;
  pl->M = M;
  while (P2 < M) P2 <<= 1;
  if ((e = hipMalloc(&keys, sizeof(uint64_t) * P2)) != hipSuccess) goto done;
  if ((e = hipMalloc(&pl->lex_n, sizeof(int32_t) * M * d)) != hipSuccess) goto done;
  if ((e = hipMalloc(&pl->canon_n, sizeof(int32_t) * M * d)) != hipSuccess) goto done;
  if ((e = hipMalloc(&pl->canon_of_lex, sizeof(int32_t) * M)) != hipSuccess) goto done;
  hipLaunchKernelGGL(k_enum_scatter, dim3((unsigned)nb), dim3(kThreads), 0, st, total, d, R, R2, bofs, pl->lex_n,
                     keys);
  if (P2 > M)
    hipLaunchKernelGGL(k_fill_keys, dim3((unsigned)((P2 - M + kThreads - 1) / kThreads)), dim3(kThreads), 0, st,
                       keys, M, P2);
  sb = (unsigned)((P2 + kThreads - 1) / kThreads);
  for (int64_t k = 2; k <= P2; k <<= 1)
    for (int64_t j = k >> 1; j > 0; j >>= 1) hipLaunchKernelGGL(k_bitonic, dim3(sb), dim3(kThreads), 0, st, keys, P2, j, k);
  hipLaunchKernelGGL(k_enum_canon, dim3((unsigned)((M + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, keys, M, d,
                     pl->lex_n, pl->canon_n, pl->canon_of_lex);
  if ((e = hipGetLastError()) != hipSuccess) goto done;
  e = hipStreamSynchronize(st);
done:
  // a launch may still be queued after an early failure: wait before freeing
  if (e != hipSuccess) (void)hipStreamSynchronize(st);
  if (keys) (void)hipFree(keys);
  if (bcount) (void)hipFree(bcount);
  if (bofs) (void)hipFree(bofs);
  if (dM) (void)hipFree(dM);
  return e;
}

}  // namespace ss
