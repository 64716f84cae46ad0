// ss_dd.h -- double-double arithmetic on the gfx950 FP64 vector ALUs.
//
// A double-double (dd) value is hi + lo.  The primitives are the published
// error-free transformations: TwoSum (Knuth), Fast2Sum and TwoProduct with FMA
// (Dekker 1971), and the accurate double-word sum and product of Joldes,
// Muller and Popescu (ACM TOMS 44, 2017).  The paper computes its whole
// minimisation in double-double ("Simulations" section); these are this
// library's own implementation of those algorithms.
//
// Two families are provided:
//  * normalised operations (|lo| <= ulp(hi)/2) for everything whose relative
//    accuracy matters (reductions of the partial sums, Phi, the minimiser);
//  * "lazy" operations for the pair loops.  Their operands are O(1) complex
//    numbers of unit modulus (or O(1) multiples of them), so only absolute
//    error matters there; they skip the final renormalisation, which keeps
//    hi + lo accurate to a few 2^-106 in absolute terms while saving the
//    Fast2Sum of every product.  The pair loops renormalise their
//    accumulators at block boundaries.
//
// All code must be compiled with -ffp-contract=off: a contracted TwoSum is no
// longer error-free.
#pragma once
#include <hip/hip_runtime.h>

namespace ss {

struct dd {
  double h, l;
};

// complex double-double: re = (rh, rl), im = (ih, il)
struct cdd {
  double rh, rl, ih, il;
};

__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__device__ __forceinline__ void fast_two_sum(double a, double b, double& s, double& e) {
  s = a + b;
  e = b - (s - a);
}

__device__ __forceinline__ void two_prod(double a, double b, double& p, double& e) {
  p = a * b;
  e = __builtin_fma(a, b, -p);
}

__device__ __forceinline__ dd dd_norm(double h, double l) {
  dd r;
  fast_two_sum(h, l, r.h, r.l);
  return r;
}

// accurate sum of two dd values (relative error <= 3 * 2^-106)
__device__ __forceinline__ dd dd_add(dd a, dd b) {
  double sh, sl, th, tl, vh, vl;
  two_sum(a.h, b.h, sh, sl);
  two_sum(a.l, b.l, th, tl);
  sl += th;
  fast_two_sum(sh, sl, vh, vl);
  vl += tl;
  dd r;
  fast_two_sum(vh, vl, r.h, r.l);
  return r;
}

__device__ __forceinline__ dd dd_neg(dd a) { return dd{-a.h, -a.l}; }
__device__ __forceinline__ dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

// dd * dd (relative error <= 4 * 2^-106)
__device__ __forceinline__ dd dd_mul(dd a, dd b) {
  double p, e;
  two_prod(a.h, b.h, p, e);
  double t = a.l * b.l;
  t = __builtin_fma(a.h, b.l, t);
  t = __builtin_fma(a.l, b.h, t);
  e += t;
  return dd_norm(p, e);
}

// dd * double
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
  double p, e;
  two_prod(a.h, b, p, e);
  e = __builtin_fma(a.l, b, e);
  return dd_norm(p, e);
}

// dd / double by long division (two quotient digits)
__device__ __forceinline__ dd dd_div_d(dd a, double b) {
  double q1 = a.h / b;
  double p, pe;
  two_prod(q1, b, p, pe);
  double r = ((a.h - p) - pe) + a.l;
  double q2 = r / b;
  return dd_norm(q1, q2);
}

// dd / dd by long division (three quotient digits)
__device__ __forceinline__ dd dd_div(dd a, dd b) {
  double q1 = a.h / b.h;
  dd r = dd_sub(a, dd_mul_d(b, q1));
  double q2 = r.h / b.h;
  r = dd_sub(r, dd_mul_d(b, q2));
  double q3 = r.h / b.h;
  dd q = dd_norm(q1, q2);
  return dd_add(q, dd{q3, 0.0});
}

__device__ __forceinline__ dd dd_sqrt(dd a) {
  if (!(a.h > 0.0)) return dd{0.0, 0.0};
  double y = __builtin_sqrt(a.h);
  double p, e;
  two_prod(y, y, p, e);
  dd r = dd_sub(a, dd{p, e});
  return dd_norm(y, r.h / (2.0 * y));
}

__device__ __forceinline__ bool dd_less(dd a, dd b) { return a.h < b.h || (a.h == b.h && a.l < b.l); }

// ---------------------------------------------------------------------------
// lazy complex arithmetic for the pair loops
// ---------------------------------------------------------------------------

// x*y - z*w with dd inputs (x,y,z,w given as hi/lo), result unnormalised (s, t)
__device__ __forceinline__ void lazy_dot2m(double xh, double xl, double yh, double yl, double zh, double zl,
                                           double wh, double wl, double& s, double& t) {
  double p1 = xh * yh;
  double e1 = __builtin_fma(xh, yh, -p1);
  double p2 = zh * wh;
  double e2 = __builtin_fma(zh, wh, -p2);
  two_sum(p1, -p2, s, t);
  t += e1 - e2;
  t = __builtin_fma(xh, yl, t);
  t = __builtin_fma(xl, yh, t);
  t = __builtin_fma(-zh, wl, t);
  t = __builtin_fma(-zl, wh, t);
}

// x*y + z*w, result unnormalised (s, t)
__device__ __forceinline__ void lazy_dot2p(double xh, double xl, double yh, double yl, double zh, double zl,
                                           double wh, double wl, double& s, double& t) {
  double p1 = xh * yh;
  double e1 = __builtin_fma(xh, yh, -p1);
  double p2 = zh * wh;
  double e2 = __builtin_fma(zh, wh, -p2);
  two_sum(p1, p2, s, t);
  t += e1 + e2;
  t = __builtin_fma(xh, yl, t);
  t = __builtin_fma(xl, yh, t);
  t = __builtin_fma(zh, wl, t);
  t = __builtin_fma(zl, wh, t);
}

// a * b for complex dd of modulus O(1)
__device__ __forceinline__ cdd cmul(const cdd& a, const cdd& b) {
  cdd r;
  lazy_dot2m(a.rh, a.rl, b.rh, b.rl, a.ih, a.il, b.ih, b.il, r.rh, r.rl);
  lazy_dot2p(a.rh, a.rl, b.ih, b.il, a.ih, a.il, b.rh, b.rl, r.ih, r.il);
  return r;
}

__device__ __forceinline__ cdd cconj(const cdd& a) { return cdd{a.rh, a.rl, -a.ih, -a.il}; }

// accumulator: acc += (xh, xl) without renormalising acc (8 ops)
__device__ __forceinline__ void lazy_acc(double& ah, double& al, double xh, double xl) {
  double s, e;
  two_sum(ah, xh, s, e);
  ah = s;
  al += e + xl;
}

__device__ __forceinline__ void renorm(double& h, double& l) {
  double s, e;
  fast_two_sum(h, l, s, e);
  h = s;
  l = e;
}

// ---------------------------------------------------------------------------
// exp(2 pi i m u) for an integer m and a dd coordinate u
// ---------------------------------------------------------------------------

// 2 pi: leading double and the rounded remainder
__device__ __forceinline__ dd two_pi_dd() { return dd{0x1.921fb54442d18p+2, 0x1.1a62633145c07p-52}; }

// frac(m u) in [-1/2, 1/2]: the products are split exactly (TwoProduct), the
// integer part of the leading product is removed exactly, and the rest is
// summed into a double-double.
__device__ __forceinline__ dd phase_of(double m, double uh, double ul) {
  double p, pe, q, qe;
  two_prod(m, uh, p, pe);
  two_prod(m, ul, q, qe);
  double r = __builtin_rint(p);
  p -= r;  // exact
  double s1, e1, s2, e2;
  two_sum(p, pe, s1, e1);
  two_sum(s1, q, s2, e2);
  double lo = (e1 + e2) + qe;
  dd t = dd_norm(s2, lo);
  if (t.h > 0.5) {
    t = dd_norm(t.h - 1.0, t.l);
  } else if (t.h < -0.5) {
    t = dd_norm(t.h + 1.0, t.l);
  }
  return t;
}

// sin and cos of a small dd angle x (|x| <= pi/16) by the nested Taylor form
// sin x = x (1 - x^2/(2.3) (1 - x^2/(4.5) (1 - ...))) through x^19 and
// cos x = 1 - x^2/(1.2) (1 - x^2/(3.4) (1 - ...)) through x^20.
__device__ __forceinline__ void sincos_small(dd x, dd& s, dd& c) {
  dd x2 = dd_mul(x, x);
  dd ps{1.0, 0.0};
#pragma unroll 1
  for (int k = 9; k >= 1; --k) {  // factors (2k)(2k+1)
    dd t = dd_div_d(dd_mul(x2, ps), (double)((2 * k) * (2 * k + 1)));
    ps = dd_sub(dd{1.0, 0.0}, t);
  }
  s = dd_mul(x, ps);
  dd pc{1.0, 0.0};
#pragma unroll 1
  for (int k = 10; k >= 1; --k) {  // factors (2k-1)(2k)
    dd t = dd_div_d(dd_mul(x2, pc), (double)((2 * k - 1) * (2 * k)));
    pc = dd_sub(dd{1.0, 0.0}, t);
  }
  c = pc;
}

// (cos 2 pi t, sin 2 pi t) for t in [-1/2, 1/2]: exact quarter-turn reduction,
// then the angle is quartered, the small-angle series evaluated, and the angle
// doubled twice (sin 2y = 2 sin y cos y, cos 2y = 1 - 2 sin^2 y).
__device__ __forceinline__ cdd expi2pi(dd t) {
  double q = __builtin_rint(4.0 * t.h);
  dd r = dd_norm(t.h - 0.25 * q, t.l);  // exact by Sterbenz
  dd th = dd_mul(two_pi_dd(), r);
  dd y{0.25 * th.h, 0.25 * th.l};
  dd s, c;
  sincos_small(y, s, c);
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    dd s2 = dd_mul(s, c);
    s2 = dd{2.0 * s2.h, 2.0 * s2.l};
    dd ss = dd_mul(s, s);
    c = dd_sub(dd{1.0, 0.0}, dd{2.0 * ss.h, 2.0 * ss.l});
    s = s2;
  }
  int qi = ((int)q) & 3;
  cdd z;
  if (qi == 0) {
    z = cdd{c.h, c.l, s.h, s.l};
  } else if (qi == 1) {
    z = cdd{-s.h, -s.l, c.h, c.l};
  } else if (qi == 2) {
    z = cdd{-c.h, -c.l, -s.h, -s.l};
  } else {
    z = cdd{s.h, s.l, -c.h, -c.l};
  }
  return z;
}

}  // namespace ss
