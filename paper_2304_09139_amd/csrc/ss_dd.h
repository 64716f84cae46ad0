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

// plus = b u and minus = b conj(u) for complex dd of modulus O(1).  The two
// products share the four real products br ur, bi ui, br ui, bi ur (4
// operations each: the high product, its rounding error by FMA and the two
// cross terms); each component is then one TwoSum of two of them plus the
// error terms (8).  48 operations for the pair against 64 for two cmul.
__device__ __forceinline__ void cmul_pm(const cdd& b, const cdd& u, cdd& plus, cdd& minus) {
  const double p1 = b.rh * u.rh;
  double e1 = __builtin_fma(b.rh, u.rh, -p1);
  e1 = __builtin_fma(b.rh, u.rl, e1);
  e1 = __builtin_fma(b.rl, u.rh, e1);
  const double p2 = b.ih * u.ih;
  double e2 = __builtin_fma(b.ih, u.ih, -p2);
  e2 = __builtin_fma(b.ih, u.il, e2);
  e2 = __builtin_fma(b.il, u.ih, e2);
  const double p3 = b.rh * u.ih;
  double e3 = __builtin_fma(b.rh, u.ih, -p3);
  e3 = __builtin_fma(b.rh, u.il, e3);
  e3 = __builtin_fma(b.rl, u.ih, e3);
  const double p4 = b.ih * u.rh;
  double e4 = __builtin_fma(b.ih, u.rh, -p4);
  e4 = __builtin_fma(b.ih, u.rl, e4);
  e4 = __builtin_fma(b.il, u.rh, e4);
  two_sum(p1, -p2, plus.rh, plus.rl);  // re(b u) = br ur - bi ui
  plus.rl += e1 - e2;
  two_sum(p3, p4, plus.ih, plus.il);  // im(b u) = br ui + bi ur
  plus.il += e3 + e4;
  two_sum(p1, p2, minus.rh, minus.rl);  // re(b conj u) = br ur + bi ui
  minus.rl += e1 + e2;
  two_sum(p4, -p3, minus.ih, minus.il);  // im(b conj u) = bi ur - br ui
  minus.il += e4 - e3;
}

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

// sin and cos of two small dd angles x0, x1 (|x| <= pi/16) by the nested
// Taylor form sin x = x (1 - x^2/(2.3) (1 - x^2/(4.5) (1 - ...))) through x^19
// and cos x = 1 - x^2/(1.2) (1 - x^2/(3.4) (1 - ...)) through x^20.  The four
// recurrences share one loop so that their dependent chains interleave.
__device__ __forceinline__ void sincos_small2(dd x0, dd x1, dd& s0, dd& c0, dd& s1, dd& c1) {
  const dd a2 = dd_mul(x0, x0), b2 = dd_mul(x1, x1);
  dd ps0{1.0, 0.0}, ps1{1.0, 0.0}, pc0{1.0, 0.0}, pc1{1.0, 0.0};
#pragma unroll 1
  for (int k = 10; k >= 1; --k) {
    if (k <= 9) {  // sine factors (2k)(2k+1), k = 9 .. 1
      const double fs = (double)((2 * k) * (2 * k + 1));
      ps0 = dd_sub(dd{1.0, 0.0}, dd_div_d(dd_mul(a2, ps0), fs));
      ps1 = dd_sub(dd{1.0, 0.0}, dd_div_d(dd_mul(b2, ps1), fs));
    }
    const double fc = (double)((2 * k - 1) * (2 * k));  // cosine factors, k = 10 .. 1
    pc0 = dd_sub(dd{1.0, 0.0}, dd_div_d(dd_mul(a2, pc0), fc));
    pc1 = dd_sub(dd{1.0, 0.0}, dd_div_d(dd_mul(b2, pc1), fc));
  }
  s0 = dd_mul(x0, ps0);
  s1 = dd_mul(x1, ps1);
  c0 = pc0;
  c1 = pc1;
}

// quarter-turn reduction of t in [-1/2, 1/2]: t = q/4 + r exactly (Sterbenz),
// and the quartered angle y = 2 pi r / 4
__device__ __forceinline__ dd quarter_angle(dd t, double& q) {
  q = __builtin_rint(4.0 * t.h);
  const dd r = dd_norm(t.h - 0.25 * q, t.l);
  const dd th = dd_mul(two_pi_dd(), r);
  return dd{0.25 * th.h, 0.25 * th.l};
}

// the angle doubled twice (sin 2y = 2 sin y cos y, cos 2y = 1 - 2 sin^2 y), then
// the quarter turns q restored
__device__ __forceinline__ cdd unquarter(dd s, dd c, double q) {
#pragma unroll
  for (int i = 0; i < 2; ++i) {
    dd s2 = dd_mul(s, c);
    s2 = dd{2.0 * s2.h, 2.0 * s2.l};
    dd ss = dd_mul(s, s);
    c = dd_sub(dd{1.0, 0.0}, dd{2.0 * ss.h, 2.0 * ss.l});
    s = s2;
  }
  const int qi = ((int)q) & 3;
  if (qi == 0) return cdd{c.h, c.l, s.h, s.l};
  if (qi == 1) return cdd{-s.h, -s.l, c.h, c.l};
  if (qi == 2) return cdd{-c.h, -c.l, -s.h, -s.l};
  return cdd{s.h, s.l, -c.h, -c.l};
}

// (cos 2 pi t, sin 2 pi t) for two phases t0, t1 in [-1/2, 1/2]: exact
// quarter-turn reduction, the small-angle series on the quartered angle, and
// two angle doublings
__device__ __forceinline__ void expi2pi2(dd t0, dd t1, cdd& z0, cdd& z1) {
  double q0, q1;
  const dd y0 = quarter_angle(t0, q0), y1 = quarter_angle(t1, q1);
  dd s0, c0, s1, c1;
  sincos_small2(y0, y1, s0, c0, s1, c1);
  z0 = unquarter(s0, c0, q0);
  z1 = unquarter(s1, c1, q1);
}

}  // namespace ss
