/*
 * ss_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU implementation of what the stealthy
 * hyperuniform collective-coordinate hot path computes (Morse, Kim,
 * Steinhardt, Torquato, arXiv:2304.09139).  It exists so that the GPU path can
 * be checked against an independent computation.  Only the test-suite, the
 * smoke check and the CPU-baseline leg of the benchmark may load it; the
 * product library never links, calls or falls back to it.  It shares no code,
 * header, table or constant generator with the GPU path.
 *
 * Everything is double-double (dd): a value is hi + lo with |lo| <= ulp(hi)/2,
 * the precision the paper uses for its whole minimisation (abstract;
 * "Simulations" section, the pyCudaPack paragraph).  The dd primitives follow
 * the published error-free transformations: TwoSum (Knuth), Fast2Sum and
 * TwoProduct (Dekker 1971, here with FMA), and the accurate double-word
 * algorithms of Joldes, Muller and Popescu (ACM TOMS 44, 2017).
 *
 * Must be compiled with -ffp-contract=off and without fast-math: a contracted
 * or reassociated TwoSum silently degrades to plain double.
 *
 * Parity pins (see tests/test_oracle_*.py): dd primitives against exact
 * rationals; phase reduction against exact rationals; sin/cos against 256-bit
 * mpmath; wavevector counts against sum-of-squares counts; energy, n(k) and
 * gradient against a single particle, two particles, an m x m lattice,
 * translation/inversion/permutation invariance, Poisson mean S(k)=1, 256-bit
 * brute force and 256-bit central differences; L-BFGS against an independent
 * 256-bit implementation of the same rules.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------- */
/* double-double primitives                                                   */
/* ------------------------------------------------------------------------- */

typedef struct { double hi, lo; } dd;

/* Knuth's TwoSum: s + e == a + b exactly. */
static inline dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    dd r = {s, e};
    return r;
}

/* Dekker's Fast2Sum, valid when |a| >= |b| (or a == 0). */
static inline dd fast_two_sum(double a, double b) {
    double s = a + b;
    double e = b - (s - a);
    dd r = {s, e};
    return r;
}

/* TwoProduct with FMA: p + e == a * b exactly. */
static inline dd two_prod(double a, double b) {
    double p = a * b;
    double e = fma(a, b, -p);
    dd r = {p, e};
    return r;
}

static inline dd dd_make(double hi, double lo) { return fast_two_sum(hi, lo); }
static inline dd dd_from(double x) { dd r = {x, 0.0}; return r; }
static inline dd dd_neg(dd a) { dd r = {-a.hi, -a.lo}; return r; }

/* AccurateDWPlusDW (Joldes-Muller-Popescu 2017, relative error <= 3u^2). */
static inline dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    dd t = two_sum(a.lo, b.lo);
    double c = s.lo + t.hi;
    dd v = fast_two_sum(s.hi, c);
    double w = t.lo + v.lo;
    return fast_two_sum(v.hi, w);
}
static inline dd dd_sub(dd a, dd b) { return dd_add(a, dd_neg(b)); }

/* DWTimesDW3 (Joldes-Muller-Popescu 2017, relative error <= 4u^2). */
static inline dd dd_mul(dd a, dd b) {
    dd c = two_prod(a.hi, b.hi);
    double tl0 = a.lo * b.lo;
    double tl1 = fma(a.hi, b.lo, tl0);
    double cl2 = fma(a.lo, b.hi, tl1);
    double cl3 = c.lo + cl2;
    return fast_two_sum(c.hi, cl3);
}

/* DWTimesFP3 (relative error <= 2u^2). */
static inline dd dd_mul_d(dd a, double b) {
    dd c = two_prod(a.hi, b);
    double cl3 = fma(a.lo, b, c.lo);
    return fast_two_sum(c.hi, cl3);
}

/* Long division by a double: q1 = a/b, remainder exactly, second quotient digit. */
static inline dd dd_div_d(dd a, double b) {
    double q1 = a.hi / b;
    dd p = two_prod(q1, b);
    double r = ((a.hi - p.hi) - p.lo) + a.lo;
    double q2 = r / b;
    return fast_two_sum(q1, q2);
}

/* Long division a / b with three quotient digits. */
static inline dd dd_div(dd a, dd b) {
    double q1 = a.hi / b.hi;
    dd r = dd_sub(a, dd_mul_d(b, q1));
    double q2 = r.hi / b.hi;
    r = dd_sub(r, dd_mul_d(b, q2));
    double q3 = r.hi / b.hi;
    dd q = fast_two_sum(q1, q2);
    return dd_add(q, dd_from(q3));
}

/* One Newton step on the double square root (Karp-Markstein form). */
static inline dd dd_sqrt(dd a) {
    if (a.hi <= 0.0) return dd_from(0.0);
    double y = sqrt(a.hi);
    dd r = dd_sub(a, two_prod(y, y));
    double corr = r.hi / (2.0 * y);
    return fast_two_sum(y, corr);
}

static inline int dd_lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }
static inline int dd_gt(dd a, dd b) { return dd_lt(b, a); }

/* 2*pi and pi as double-double: the correctly rounded leading double of 2*pi
 * plus the correctly rounded remainder. */
static const dd TWO_PI = {0x1.921fb54442d18p+2, 0x1.1a62633145c07p-52};

/* ------------------------------------------------------------------------- */
/* exact reduction of n . u modulo 1                                          */
/* ------------------------------------------------------------------------- */

/* Grow-Expansion (Shewchuk 1997) with zero elimination: e[0..m) is a
 * nonoverlapping expansion ordered by increasing magnitude; add x exactly. */
static int grow_expansion(double* e, int m, double x) {
    double q = x;
    int k = 0;
    for (int i = 0; i < m; i++) {
        dd t = two_sum(q, e[i]);
        q = t.hi;
        if (t.lo != 0.0) e[k++] = t.lo;
    }
    if (q != 0.0 || k == 0) e[k++] = q;
    return k;
}

static double expansion_approx(const double* e, int m) {
    double s = 0.0;
    for (int i = 0; i < m; i++) s += e[i];
    return s;
}

/* t = frac(sum_a n_a (hi_a + lo_a)) in [-1/2, 1/2] (to within one rounding of
 * the final double-double), with the integer part removed exactly. */
static dd phase_exact(int d, const int32_t* n, const double* uhi, const double* ulo) {
    double e[64];
    int m = 0;
    for (int a = 0; a < d; a++) {
        double na = (double)n[a];
        dd p = two_prod(na, uhi[a]);
        dd q = two_prod(na, ulo[a]);
        double terms[4] = {p.hi, p.lo, q.hi, q.lo};
        for (int i = 0; i < 4; i++) {
            double x = terms[i];
            double r = nearbyint(x);
            m = grow_expansion(e, m, r);        /* integer part kept exactly ... */
            m = grow_expansion(e, m, x - r);    /* ... x - rint(x) is exact      */
        }
    }
    /* remove the (exact, integer) total integer part */
    double r = nearbyint(expansion_approx(e, m));
    m = grow_expansion(e, m, -r);
    double approx = expansion_approx(e, m);
    if (approx > 0.5) m = grow_expansion(e, m, -1.0);
    else if (approx < -0.5) m = grow_expansion(e, m, 1.0);
    /* round to double-double: leading double, then the exact remainder */
    double hi = expansion_approx(e, m);
    m = grow_expansion(e, m, -hi);
    double lo = expansion_approx(e, m);
    return fast_two_sum(hi, lo);
}

/* ------------------------------------------------------------------------- */
/* cos(2 pi t), sin(2 pi t) in double-double                                  */
/* ------------------------------------------------------------------------- */

#define NFACT 32
static dd INV_FACT[NFACT]; /* 1/k! */

__attribute__((constructor)) static void init_inv_fact(void) {
    INV_FACT[0] = dd_from(1.0);
    for (int k = 1; k < NFACT; k++) INV_FACT[k] = dd_div_d(INV_FACT[k - 1], (double)k);
}

/* Quadrant reduction by the exact symmetry 2*pi*t = q*pi/2 + theta with
 * |theta| <= pi/4, then the Taylor series of sin (through theta^27) and cos
 * (through theta^28), each evaluated by Horner's rule in theta^2. */
static void sincos2pi(dd t, dd* c_out, dd* s_out) {
    double q = nearbyint(4.0 * t.hi);
    dd r = fast_two_sum(t.hi - 0.25 * q, t.lo); /* exact by Sterbenz */
    dd th = dd_mul(TWO_PI, r);
    dd th2 = dd_mul(th, th);
    /* sin: theta * sum_{k=0}^{13} (-1)^k theta^{2k} / (2k+1)! */
    dd ps = dd_from(0.0);
    for (int k = 13; k >= 0; k--) {
        dd coef = INV_FACT[2 * k + 1];
        if (k & 1) coef = dd_neg(coef);
        ps = dd_add(dd_mul(ps, th2), coef);
    }
    dd sn = dd_mul(ps, th);
    /* cos: sum_{k=0}^{14} (-1)^k theta^{2k} / (2k)! */
    dd pc = dd_from(0.0);
    for (int k = 14; k >= 0; k--) {
        dd coef = INV_FACT[2 * k];
        if (k & 1) coef = dd_neg(coef);
        pc = dd_add(dd_mul(pc, th2), coef);
    }
    dd cs = pc;
    int qi = ((int)q) & 3;
    switch (qi) {
    case 0: *c_out = cs; *s_out = sn; break;
    case 1: *c_out = dd_neg(sn); *s_out = cs; break;
    case 2: *c_out = dd_neg(cs); *s_out = dd_neg(sn); break;
    default: *c_out = sn; *s_out = dd_neg(cs); break;
    }
}

/* ------------------------------------------------------------------------- */
/* exported primitives (for pinning tests)                                   */
/* ------------------------------------------------------------------------- */

void or_dd_add(const double* a, const double* b, double* r) { dd x = dd_add((dd){a[0], a[1]}, (dd){b[0], b[1]}); r[0] = x.hi; r[1] = x.lo; }
void or_dd_mul(const double* a, const double* b, double* r) { dd x = dd_mul((dd){a[0], a[1]}, (dd){b[0], b[1]}); r[0] = x.hi; r[1] = x.lo; }
void or_dd_div(const double* a, const double* b, double* r) { dd x = dd_div((dd){a[0], a[1]}, (dd){b[0], b[1]}); r[0] = x.hi; r[1] = x.lo; }
void or_dd_sqrt(const double* a, double* r) { dd x = dd_sqrt((dd){a[0], a[1]}); r[0] = x.hi; r[1] = x.lo; }

void or_phase(int d, const int32_t* n, const double* uhi, const double* ulo, double* t) {
    dd x = phase_exact(d, n, uhi, ulo);
    t[0] = x.hi; t[1] = x.lo;
}

void or_sincos2pi(const double* t, double* c, double* s) {
    dd cc, ss;
    sincos2pi((dd){t[0], t[1]}, &cc, &ss);
    c[0] = cc.hi; c[1] = cc.lo; s[0] = ss.hi; s[1] = ss.lo;
}

void or_two_pi(double* r) { r[0] = TWO_PI.hi; r[1] = TWO_PI.lo; }

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
void or_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------- */
/* wavevectors: the half set H(R2) and the cutoff                             */
/* ------------------------------------------------------------------------- */

/* n is in the half set when its first nonzero component is positive; the
 * inversion symmetry S(k) = S(-k) leaves M independent vectors out of the 2M
 * nonzero vectors inside the cutoff ("Definitions", the paragraph defining chi). */
static int in_half_space(int d, const int64_t* n) {
    for (int a = 0; a < d; a++) {
        if (n[a] > 0) return 1;
        if (n[a] < 0) return 0;
    }
    return 0; /* the origin */
}

/* counts[s] (s = 0..R2) = number of half-set vectors with |n|^2 == s */
static int shell_counts(int d, int64_t R2, int64_t* counts) {
    int64_t R = (int64_t)floor(sqrt((double)R2));
    while ((R + 1) * (R + 1) <= R2) R++;
    while (R * R > R2) R--;
    for (int64_t s = 0; s <= R2; s++) counts[s] = 0;
    int64_t side = 2 * R + 1, total = 1;
    for (int a = 0; a < d; a++) total *= side;
    int64_t n[4];
    for (int64_t idx = 0; idx < total; idx++) {
        int64_t rem = idx, s = 0;
        for (int a = d - 1; a >= 0; a--) { n[a] = rem % side - R; rem /= side; }
        for (int a = 0; a < d; a++) s += n[a] * n[a];
        if (s <= R2 && in_half_space(d, n)) counts[s]++;
    }
    return 0;
}

int64_t or_count(int d, int64_t R2) {
    if (d < 1 || d > 4 || R2 < 0) return -1;
    int64_t* c = (int64_t*)malloc(sizeof(int64_t) * (size_t)(R2 + 1));
    if (!c) return -1;
    shell_counts(d, R2, c);
    int64_t M = 0;
    for (int64_t s = 0; s <= R2; s++) M += c[s];
    free(c);
    return M;
}

/* Cutoff from the constraint fraction chi = M / (d (N - 1)): the largest
 * realised squared radius R2 whose half-set count does not exceed
 * chi * d * (N - 1).  Returns 0 on success, -1 on invalid input. */
int or_cutoff(int d, int64_t N, double chi, int64_t* R2_out, int64_t* M_out) {
    if (d < 1 || d > 4 || N < 2 || !(chi > 0.0) || !(chi < 0.5)) return -1;
    double T = chi * (double)d * (double)(N - 1);
    if (T < 1.0) return -1;
    for (int64_t R = 1;; R++) {
        int64_t R2max = R * R;
        int64_t* c = (int64_t*)malloc(sizeof(int64_t) * (size_t)(R2max + 1));
        if (!c) return -1;
        shell_counts(d, R2max, c);
        int64_t cum = 0, best_R2 = -1, best_M = 0;
        int exceeded = 0;
        for (int64_t s = 1; s <= R2max; s++) {
            if (c[s] == 0) continue;
            if ((double)(cum + c[s]) > T) { exceeded = 1; break; }
            cum += c[s];
            best_R2 = s;
            best_M = cum;
        }
        free(c);
        if (exceeded) {
            if (best_R2 < 0) return -1;
            *R2_out = best_R2;
            *M_out = best_M;
            return 0;
        }
    }
}

typedef struct { int64_t shell, lex; int32_t n[4]; } wv_rec;

static int wv_cmp(const void* pa, const void* pb) {
    const wv_rec* a = (const wv_rec*)pa;
    const wv_rec* b = (const wv_rec*)pb;
    if (a->shell != b->shell) return a->shell < b->shell ? -1 : 1;
    if (a->lex != b->lex) return a->lex < b->lex ? -1 : 1;
    return 0;
}

/* The half set H(R2) ordered by ascending |n|^2, ties by ascending
 * lexicographic order of (n_1, ..., n_d).  Writes min(M, cap) vectors. */
int or_wavevectors(int d, int64_t R2, int32_t* out, int64_t cap, int64_t* M_out) {
    if (d < 1 || d > 4 || R2 < 1) return -1;
    int64_t R = (int64_t)floor(sqrt((double)R2));
    while ((R + 1) * (R + 1) <= R2) R++;
    while (R * R > R2) R--;
    int64_t side = 2 * R + 1, total = 1;
    for (int a = 0; a < d; a++) total *= side;
    int64_t M = or_count(d, R2);
    *M_out = M;
    if (!out) return 0;
    wv_rec* recs = (wv_rec*)malloc(sizeof(wv_rec) * (size_t)(M > 0 ? M : 1));
    if (!recs) return -1;
    int64_t k = 0, n[4];
    for (int64_t idx = 0; idx < total; idx++) {  /* idx increases with lex order */
        int64_t rem = idx, s = 0;
        for (int a = d - 1; a >= 0; a--) { n[a] = rem % side - R; rem /= side; }
        for (int a = 0; a < d; a++) s += n[a] * n[a];
        if (s <= R2 && in_half_space(d, n)) {
            recs[k].shell = s;
            recs[k].lex = idx;
            for (int a = 0; a < 4; a++) recs[k].n[a] = a < d ? (int32_t)n[a] : 0;
            k++;
        }
    }
    qsort(recs, (size_t)k, sizeof(wv_rec), wv_cmp);
    for (int64_t i = 0; i < k && i < cap; i++)
        for (int a = 0; a < d; a++) out[i * d + a] = recs[i].n[a];
    free(recs);
    return 0;
}

/* Weights v_k (dimensionless: the paper's v~(k) / (eps0 L^d)).
 * vkind 0: the Heaviside form of the "Simulations" section, v = 1 inside.
 * vkind 1: v = (1 - |k|/K)^2 with K^2 = (R2 + 1/2) (2 pi / L)^2, which keeps
 *          exactly the same integer set and every weight positive. */
int or_weights(int d, int64_t M, const int32_t* n, int64_t R2, int vkind, double* v) {
    for (int64_t k = 0; k < M; k++) {
        dd w;
        if (vkind == 0) {
            w = dd_from(1.0);
        } else if (vkind == 1) {
            int64_t s = 0;
            for (int a = 0; a < d; a++) s += (int64_t)n[k * d + a] * n[k * d + a];
            /* 1 - |k|/K = (K^2 - |k|^2) / (K^2 (1 + |k|/K)): no cancellation, and
             * K^2 - |k|^2 = R2 + 1/2 - s is exact */
            double K2 = (double)R2 + 0.5;
            dd ratio = dd_div(dd_from((double)s), dd_from(K2));
            dd denom = dd_mul_d(dd_add(dd_from(1.0), dd_sqrt(ratio)), K2);
            dd one_minus = dd_div(dd_from(K2 - (double)s), denom);
            w = dd_mul(one_minus, one_minus);
        } else {
            return -1;
        }
        v[k] = w.hi;
        v[M + k] = w.lo;
    }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* collective density, energy, structure factor, gradient                    */
/* ------------------------------------------------------------------------- */

static inline dd weight_at(const double* v, int64_t M, int64_t k) {
    if (!v) return dd_from(1.0);
    dd w = {v[k], v[M + k]};
    return w;
}

/* n~(k) = sum_j exp(-i k.r_j) = C_k - i S_k with C_k = sum_j cos(2 pi t_jk),
 * S_k = sum_j sin(2 pi t_jk), t_jk = n_k . u_j mod 1 (Eq. ntilde).  The sum
 * runs over j in ascending order with the accurate dd addition.
 * Computes k in [k0, k1) into nk[4][M] = (C.hi, C.lo, S.hi, S.lo). */
void or_nk(int d, int64_t N, int64_t M, const int32_t* n, const double* pos,
           double* nk, int64_t k0, int64_t k1) {
    #pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = k0; k < k1; k++) {
        dd C = dd_from(0.0), S = dd_from(0.0);
        double uh[4], ul[4];
        for (int64_t j = 0; j < N; j++) {
            for (int a = 0; a < d; a++) { uh[a] = pos[a * N + j]; ul[a] = pos[(int64_t)d * N + a * N + j]; }
            dd t = phase_exact(d, n + k * d, uh, ul);
            dd c, s;
            sincos2pi(t, &c, &s);
            C = dd_add(C, c);
            S = dd_add(S, s);
        }
        nk[k] = C.hi; nk[M + k] = C.lo; nk[2 * M + k] = S.hi; nk[3 * M + k] = S.lo;
    }
}

/* Phi = sum_{k in H} v_k (C_k^2 + S_k^2), summed in k order.  This equals the
 * paper's Phi / eps0 (Eq. energy with the structure-independent term dropped):
 * N/(2 v_F) sum over the full +-k set of v~ S(k) = sum over H of v |n~|^2.
 * S(k) = |n~(k)|^2 / N (Eq. structurefactor); S_max = max over H (Eq. smax). */
void or_energy_from_nk(int64_t N, int64_t M, const double* v, const double* nk,
                       double* phi, double* smax, int64_t* kmax, double* sk /*[2][M] or NULL*/) {
    dd P = dd_from(0.0), best = dd_from(-1.0);
    int64_t bk = -1;
    for (int64_t k = 0; k < M; k++) {
        dd C = {nk[k], nk[M + k]}, S = {nk[2 * M + k], nk[3 * M + k]};
        dd mag = dd_add(dd_mul(C, C), dd_mul(S, S));
        P = dd_add(P, dd_mul(weight_at(v, M, k), mag));
        dd Sk = dd_div_d(mag, (double)N);
        if (sk) { sk[k] = Sk.hi; sk[M + k] = Sk.lo; }
        if (dd_gt(Sk, best)) { best = Sk; bk = k; }
    }
    phi[0] = P.hi; phi[1] = P.lo;
    if (smax) { smax[0] = best.hi; smax[1] = best.lo; }
    if (kmax) *kmax = bk;
}

/* dPhi/dr_{j,a} = (4 pi / L) sum_{k in H} v_k n_{k,a} (S_k c_jk - C_k s_jk):
 * minus the force of Eq. force, whose sum over the full +-k set folds into
 * twice the sum over the half set H.  Summed over k in ascending order.
 * Writes g[js_idx][a][2] for the particles listed in js (all if js == NULL). */
void or_grad(int d, int64_t N, int64_t M, double L, const int32_t* n, const double* v,
             const double* pos, const double* nk, const int64_t* js, int64_t nj, double* g) {
    dd four_pi_over_L = dd_div_d(dd_mul_d(TWO_PI, 2.0), L);
    int64_t cnt = js ? nj : N;
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t q = 0; q < cnt; q++) {
        int64_t j = js ? js[q] : q;
        double uh[4], ul[4];
        for (int a = 0; a < d; a++) { uh[a] = pos[a * N + j]; ul[a] = pos[(int64_t)d * N + a * N + j]; }
        dd acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (int64_t k = 0; k < M; k++) {
            dd t = phase_exact(d, n + k * d, uh, ul);
            dd c, s;
            sincos2pi(t, &c, &s);
            dd C = {nk[k], nk[M + k]}, S = {nk[2 * M + k], nk[3 * M + k]};
            dd term = dd_sub(dd_mul(S, c), dd_mul(C, s));
            term = dd_mul(weight_at(v, M, k), term);
            for (int a = 0; a < d; a++)
                acc[a] = dd_add(acc[a], dd_mul_d(term, (double)n[k * d + a]));
        }
        for (int a = 0; a < d; a++) {
            dd ga = dd_mul(acc[a], four_pi_over_L);
            g[(q * d + a) * 2 + 0] = ga.hi;
            g[(q * d + a) * 2 + 1] = ga.lo;
        }
    }
}

/* Full evaluation: n~, Phi, S_max and (optionally) the gradient in the
 * [2][d][N] hi/lo plane layout.  Returns 0. */
int or_energy_grad(int d, int64_t N, int64_t M, double L, const int32_t* n, const double* v,
                   const double* pos, double* phi, double* smax, double* grad, double* nk_out) {
    double* nk = nk_out ? nk_out : (double*)malloc(sizeof(double) * 4 * (size_t)M);
    if (!nk) return -1;
    or_nk(d, N, M, n, pos, nk, 0, M);
    or_energy_from_nk(N, M, v, nk, phi, smax, NULL, NULL);
    if (grad) {
        double* g = (double*)malloc(sizeof(double) * 2 * (size_t)d * (size_t)N);
        if (!g) { if (!nk_out) free(nk); return -1; }
        or_grad(d, N, M, L, n, v, pos, nk, NULL, 0, g);
        for (int64_t j = 0; j < N; j++)
            for (int a = 0; a < d; a++) {
                grad[a * N + j] = g[(j * d + a) * 2 + 0];
                grad[(int64_t)d * N + a * N + j] = g[(j * d + a) * 2 + 1];
            }
        free(g);
    }
    if (!nk_out) free(nk);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* L-BFGS (the minimiser; the paper quenches with FIRE, this path uses the     */
/* limited-memory BFGS two-loop recursion of Nocedal & Wright, Alg. 7.4)      */
/* ------------------------------------------------------------------------- */

typedef struct {
    int history;          /* m, number of (s, y) pairs kept                      */
    int64_t max_iter;     /* iteration cap                                        */
    double s_floor;       /* converged when S_max <= s_floor                      */
    int stall_window;     /* W: stalled when min Phi over the last W iterations   */
    double stall_ratio;   /*    exceeds stall_ratio * min Phi over the W before   */
    double c1;            /* Armijo constant                                      */
    double step_cap;      /* first/reset step moves at most step_cap * N^(-1/d)   */
    int max_halvings;     /* line-search halvings before a failure is recorded    */
    int max_ls_fail;      /* consecutive failures that end the run as stalled     */
    int method;           /* 0 L-BFGS, 1 FIRE                                     */
} or_lbfgs_opts;

typedef struct {
    int status;           /* 0 converged, 1 stalled, 2 iteration cap */
    int64_t iters, evals, grad_evals;
    double phi[2], smax[2];
} or_lbfgs_result;

/* objective: 0 = stealthy energy; 1 = quadratic 1/2 sum w_i (x_i - c_i)^2 (test) */
typedef struct {
    int kind;
    int d; int64_t N, M; double L;
    const int32_t* n; const double* v;
    const double* qw; const double* qc; /* quadratic weights / centres, dd [2][n] */
    double* nk;   /* scratch [4][M] */
    double* pos;  /* scratch [2][d][N] */
    double* grad; /* scratch [2][d][N] */
} objective;

static void obj_eval(objective* o, int64_t nv, const dd* x, dd* f, dd* smax, dd* g) {
    if (o->kind == 1) {
        dd F = dd_from(0.0);
        for (int64_t i = 0; i < nv; i++) {
            dd w = {o->qw[i], o->qw[nv + i]}, c = {o->qc[i], o->qc[nv + i]};
            dd r = dd_sub(x[i], c);
            dd wr = dd_mul(w, r);
            F = dd_add(F, dd_mul(wr, r));
            if (g) g[i] = wr;
        }
        *f = dd_mul_d(F, 0.5);
        *smax = *f;
        return;
    }
    int64_t N = o->N;
    int d = o->d;
    for (int64_t i = 0; i < nv; i++) { o->pos[i] = x[i].hi; o->pos[nv + i] = x[i].lo; }
    or_nk(d, N, o->M, o->n, o->pos, o->nk, 0, o->M);
    double phi[2], sm[2];
    or_energy_from_nk(N, o->M, o->v, o->nk, phi, sm, NULL, NULL);
    f->hi = phi[0]; f->lo = phi[1];
    smax->hi = sm[0]; smax->lo = sm[1];
    if (g) {
        double* gg = (double*)malloc(sizeof(double) * 2 * (size_t)nv);
        or_grad(d, N, o->M, o->L, o->n, o->v, o->pos, o->nk, NULL, 0, gg);
        /* gradient with respect to the fractional coordinates: L * dPhi/dr */
        for (int64_t j = 0; j < N; j++)
            for (int a = 0; a < d; a++) {
                dd ga = {gg[(j * d + a) * 2 + 0], gg[(j * d + a) * 2 + 1]};
                g[a * N + j] = dd_mul_d(ga, o->L);
            }
        free(gg);
    }
}

static dd vdot(int64_t nv, const dd* a, const dd* b) {
    dd s = dd_from(0.0);
    for (int64_t i = 0; i < nv; i++) s = dd_add(s, dd_mul(a[i], b[i]));
    return s;
}

static int lbfgs_run(objective* o, int64_t nv, dd* x, const or_lbfgs_opts* op,
                     or_lbfgs_result* res, double* phi_trace, int64_t trace_cap) {
    int m = op->history;
    dd* g = (dd*)calloc((size_t)nv, sizeof(dd));
    dd* p = (dd*)calloc((size_t)nv, sizeof(dd));
    dd* xt = (dd*)calloc((size_t)nv, sizeof(dd));
    dd* gt = (dd*)calloc((size_t)nv, sizeof(dd));
    dd* q = (dd*)calloc((size_t)nv, sizeof(dd));
    /* m ring slots plus one spare that receives each candidate pair, so a pair
     * rejected by the s.y > 0 test never overwrites a kept one */
    dd* S = (dd*)calloc((size_t)nv * (size_t)(m + 1), sizeof(dd));
    dd* Y = (dd*)calloc((size_t)nv * (size_t)(m + 1), sizeof(dd));
    dd* rho = (dd*)calloc((size_t)(m + 1), sizeof(dd));
    dd* alpha = (dd*)calloc((size_t)(m + 1), sizeof(dd));
    int* ring = (int*)calloc((size_t)(m + 1), sizeof(int)); /* ring[0..hn) = slots, oldest first */
    int64_t W = op->stall_window;
    dd* fhist = (dd*)calloc((size_t)(op->max_iter + 2), sizeof(dd));
    if (!g || !p || !xt || !gt || !q || !S || !Y || !rho || !alpha || !fhist || !ring) return -1;
    int hn = 0;
    int ls_fail = 0;
    double nmean = pow((double)o->N, -1.0 / (double)(o->d > 0 ? o->d : 1));
    if (o->kind == 1) nmean = 1.0;
    dd f, smax, ft, smt;
    obj_eval(o, nv, x, &f, &smax, g);
    res->evals = 1; res->grad_evals = 1;
    int64_t it = 0;
    int status = 2;
    for (;;) {
        if (phi_trace && it < trace_cap) { phi_trace[2 * it] = f.hi; phi_trace[2 * it + 1] = f.lo; }
        fhist[it] = f;
        if (!dd_gt(smax, dd_from(op->s_floor))) { status = 0; break; }
        if (it >= op->max_iter) { status = 2; break; }
        if (it >= 2 * W) {
            dd recent = fhist[it], older = fhist[it - W];
            for (int64_t i = it - W + 1; i <= it; i++) if (dd_lt(fhist[i], recent)) recent = fhist[i];
            for (int64_t i = it - 2 * W + 1; i <= it - W; i++) if (dd_lt(fhist[i], older)) older = fhist[i];
            if (dd_gt(recent, dd_mul_d(older, op->stall_ratio))) { status = 1; break; }
        }
        /* search direction: two-loop recursion, H0 = gamma I */
        int use_sd = (hn == 0);
        dd gp = dd_from(0.0);
        if (!use_sd) {
            for (int64_t i = 0; i < nv; i++) q[i] = g[i];
            for (int h = hn - 1; h >= 0; h--) {
                int slot = ring[h];
                alpha[slot] = dd_mul(rho[slot], vdot(nv, S + (int64_t)slot * nv, q));
                for (int64_t i = 0; i < nv; i++) q[i] = dd_sub(q[i], dd_mul(alpha[slot], Y[(int64_t)slot * nv + i]));
            }
            int newest = ring[hn - 1];
            dd sy = vdot(nv, S + (int64_t)newest * nv, Y + (int64_t)newest * nv);
            dd yy = vdot(nv, Y + (int64_t)newest * nv, Y + (int64_t)newest * nv);
            dd gamma = dd_div(sy, yy);
            for (int64_t i = 0; i < nv; i++) q[i] = dd_mul(gamma, q[i]);
            for (int h = 0; h < hn; h++) {
                int slot = ring[h];
                dd beta = dd_mul(rho[slot], vdot(nv, Y + (int64_t)slot * nv, q));
                dd coef = dd_sub(alpha[slot], beta);
                for (int64_t i = 0; i < nv; i++) q[i] = dd_add(q[i], dd_mul(coef, S[(int64_t)slot * nv + i]));
            }
            for (int64_t i = 0; i < nv; i++) p[i] = dd_neg(q[i]);
            gp = vdot(nv, g, p);
            if (!dd_lt(gp, dd_from(0.0))) use_sd = 1;
        }
        if (use_sd) {
            hn = 0;
            dd gmax = dd_from(0.0); /* max_i |g_i|, compared in double-double */
            for (int64_t i = 0; i < nv; i++) {
                dd ag = g[i].hi < 0.0 ? dd_neg(g[i]) : g[i];
                if (dd_gt(ag, gmax)) gmax = ag;
            }
            if (gmax.hi == 0.0) { status = 0; break; }
            dd scale = dd_div(dd_from(op->step_cap * nmean), gmax);
            /* the minimum of the energy is 0 (a ground state), so the step is also
             * bounded by 2 f / g.g, where the line along -g meets the minimum of
             * the isotropic quadratic through (f, g) */
            dd polyak = dd_div(dd_mul_d(f, 2.0), vdot(nv, g, g));
            if (dd_lt(polyak, scale)) scale = polyak;
            if (scale.hi == 0.0) { status = 0; break; }
            for (int64_t i = 0; i < nv; i++) p[i] = dd_neg(dd_mul(g[i], scale));
            gp = vdot(nv, g, p);
        }
        /* Armijo backtracking from alpha = 1 */
        dd a = dd_from(1.0);
        int accepted = 0;
        for (int hcount = 0; hcount <= op->max_halvings; hcount++) {
            for (int64_t i = 0; i < nv; i++) xt[i] = dd_add(x[i], dd_mul(a, p[i]));
            obj_eval(o, nv, xt, &ft, &smt, NULL);
            res->evals++;
            dd bound = dd_add(f, dd_mul(dd_mul_d(a, op->c1), gp));
            if (!dd_gt(ft, bound)) { accepted = 1; break; }
            a = dd_mul_d(a, 0.5);
        }
        it++;
        if (!accepted) {
            ls_fail++;
            hn = 0;
            if (ls_fail >= op->max_ls_fail) { fhist[it] = f; status = 1; break; }
            continue;
        }
        ls_fail = 0;
        obj_eval(o, nv, xt, &ft, &smt, gt);
        res->grad_evals++;
        /* candidate pair s = x_new - x, y = g_new - g in a slot no kept pair uses */
        int slot = 0;
        for (;; slot++) {
            int used = 0;
            for (int h = 0; h < hn; h++) if (ring[h] == slot) used = 1;
            if (!used) break;
        }
        dd* s_new = S + (int64_t)slot * nv;
        dd* y_new = Y + (int64_t)slot * nv;
        for (int64_t i = 0; i < nv; i++) { s_new[i] = dd_sub(xt[i], x[i]); y_new[i] = dd_sub(gt[i], g[i]); }
        dd sy = vdot(nv, s_new, y_new);
        if (dd_gt(sy, dd_from(0.0))) {   /* keep it; drop the oldest beyond m */
            rho[slot] = dd_div(dd_from(1.0), sy);
            if (hn == m) { for (int h = 1; h < m; h++) ring[h - 1] = ring[h]; hn--; }
            ring[hn++] = slot;
        }
        for (int64_t i = 0; i < nv; i++) { x[i] = xt[i]; g[i] = gt[i]; }
        f = ft; smax = smt;
    }
    res->status = status;
    res->iters = it;
    res->phi[0] = f.hi; res->phi[1] = f.lo;
    res->smax[0] = smax.hi; res->smax[1] = smax.lo;
    free(g); free(p); free(xt); free(gt); free(q); free(S); free(Y); free(rho); free(alpha); free(fhist); free(ring);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* FIRE, the paper's minimiser ("Simulations"; Bitzek, Koskinen, Gaehler,      */
/* Moseler and Gumbsch, Phys. Rev. Lett. 97, 170201 (2006)).  Unit masses,      */
/* force F = -g.  Each iteration: P = F.v; the velocity is mixed towards the   */
/* force direction, v <- (1 - a) v + a |v| F/|F|; if P > 0 the count of        */
/* consecutive uphill-free steps grows and, once it exceeds N_min, the step    */
/* grows (dt <- min(f_inc dt, dt_max)) and a shrinks (a <- f_a a); if P <= 0    */
/* the step shrinks (dt <- f_dec dt), the system is frozen (v <- 0) and         */
/* a <- a_start.  Then one semi-implicit Euler step: v <- v + dt F,             */
/* x <- x + dt v, and a new evaluation.  The published parameters are used:    */
/* N_min 5, f_inc 1.1, f_dec 0.5, a_start 0.1, f_a 0.99, dt_max = 10 dt0;       */
/* dt0^2 max|g(x0)| = step_cap N^(-1/d).  The stopping rules are the L-BFGS     */
/* ones (floor, stall window, cap).                                             */
/* ------------------------------------------------------------------------- */
static int fire_run(objective* o, int64_t nv, dd* x, const or_lbfgs_opts* op,
                    or_lbfgs_result* res, double* phi_trace, int64_t trace_cap) {
    const int n_min = 5;
    const double f_inc = 1.1, f_dec = 0.5, a_start = 0.1, f_a = 0.99;
    dd* g = (dd*)calloc((size_t)nv, sizeof(dd));
    dd* v = (dd*)calloc((size_t)nv, sizeof(dd));
    dd* fhist = (dd*)calloc((size_t)(op->max_iter + 2), sizeof(dd));
    if (!g || !v || !fhist) return -1;
    double nmean = pow((double)o->N, -1.0 / (double)(o->d > 0 ? o->d : 1));
    if (o->kind == 1) nmean = 1.0;
    const int64_t W = op->stall_window;
    dd f, smax;
    obj_eval(o, nv, x, &f, &smax, g);
    res->evals = 1; res->grad_evals = 1;
    /* initial step from the largest gradient component (compared in dd) */
    dd gmax = dd_from(0.0);
    for (int64_t i = 0; i < nv; i++) {
        dd ag = g[i].hi < 0.0 ? dd_neg(g[i]) : g[i];
        if (dd_gt(ag, gmax)) gmax = ag;
    }
    double dt = gmax.hi > 0.0 ? sqrt(op->step_cap * nmean / gmax.hi) : 0.0;
    const double dt_max = 10.0 * dt;
    double a = a_start;
    int npos = 0;
    int64_t it = 0;
    int status = 2;
    for (;;) {
        if (phi_trace && it < trace_cap) { phi_trace[2 * it] = f.hi; phi_trace[2 * it + 1] = f.lo; }
        fhist[it] = f;
        if (!dd_gt(smax, dd_from(op->s_floor))) { status = 0; break; }
        if (it >= op->max_iter) { status = 2; break; }
        if (it >= 2 * W) {
            dd recent = fhist[it], older = fhist[it - W];
            for (int64_t i = it - W + 1; i <= it; i++) if (dd_lt(fhist[i], recent)) recent = fhist[i];
            for (int64_t i = it - 2 * W + 1; i <= it - W; i++) if (dd_lt(fhist[i], older)) older = fhist[i];
            if (dd_gt(recent, dd_mul_d(older, op->stall_ratio))) { status = 1; break; }
        }
        if (dt == 0.0) { status = 0; break; }  /* g = 0 at the start: a stationary point */
        /* P = F.v = -(g.v) */
        dd P = dd_neg(vdot(nv, g, v));
        if (dd_gt(P, dd_from(0.0))) {
            dd vn = dd_sqrt(vdot(nv, v, v));
            dd gn = dd_sqrt(vdot(nv, g, g));
            dd cg = dd_mul_d(dd_div(vn, gn), a);          /* a |v| / |F| */
            dd cv = dd_from(1.0 - a);
            for (int64_t i = 0; i < nv; i++) v[i] = dd_sub(dd_mul(cv, v[i]), dd_mul(cg, g[i]));
            npos++;
            if (npos > n_min) {
                dt = fmin(dt * f_inc, dt_max);
                a = a * f_a;
            }
        } else {
            dt = dt * f_dec;
            for (int64_t i = 0; i < nv; i++) v[i] = dd_from(0.0);
            a = a_start;
            npos = 0;
        }
        for (int64_t i = 0; i < nv; i++) {
            v[i] = dd_sub(v[i], dd_mul_d(g[i], dt));
            x[i] = dd_add(x[i], dd_mul_d(v[i], dt));
        }
        obj_eval(o, nv, x, &f, &smax, g);
        res->evals++; res->grad_evals++;
        it++;
        if (!(f.hi == f.hi) || f.hi > 1e300) { status = 3; break; }
    }
    res->status = status;
    res->iters = it;
    res->phi[0] = f.hi; res->phi[1] = f.lo;
    res->smax[0] = smax.hi; res->smax[1] = smax.lo;
    free(g); free(v); free(fhist);
    return 0;
}

/* Minimise the stealthy energy from the positions in pos ([2][d][N],
 * fractional, updated in place; not wrapped into the unit cell). */
int or_minimize(int d, int64_t N, int64_t M, double L, const int32_t* n, const double* v,
                double* pos, const or_lbfgs_opts* op, or_lbfgs_result* res,
                double* phi_trace, int64_t trace_cap) {
    int64_t nv = (int64_t)d * N;
    objective o;
    memset(&o, 0, sizeof(o));
    o.kind = 0; o.d = d; o.N = N; o.M = M; o.L = L; o.n = n; o.v = v;
    o.nk = (double*)malloc(sizeof(double) * 4 * (size_t)M);
    o.pos = (double*)malloc(sizeof(double) * 2 * (size_t)nv);
    dd* x = (dd*)malloc(sizeof(dd) * (size_t)nv);
    if (!o.nk || !o.pos || !x) return -1;
    for (int64_t i = 0; i < nv; i++) { x[i].hi = pos[i]; x[i].lo = pos[nv + i]; }
    int rc = op->method == 1 ? fire_run(&o, nv, x, op, res, phi_trace, trace_cap)
                             : lbfgs_run(&o, nv, x, op, res, phi_trace, trace_cap);
    for (int64_t i = 0; i < nv; i++) { pos[i] = x[i].hi; pos[nv + i] = x[i].lo; }
    free(o.nk); free(o.pos); free(x);
    return rc;
}

/* The same minimiser on a separable quadratic (test objective). */
int or_minimize_quadratic(int64_t nv, const double* w, const double* c, double* x_io,
                          const or_lbfgs_opts* op, or_lbfgs_result* res,
                          double* phi_trace, int64_t trace_cap) {
    objective o;
    memset(&o, 0, sizeof(o));
    o.kind = 1; o.d = 1; o.N = nv; o.qw = w; o.qc = c;
    dd* x = (dd*)malloc(sizeof(dd) * (size_t)nv);
    if (!x) return -1;
    for (int64_t i = 0; i < nv; i++) { x[i].hi = x_io[i]; x[i].lo = x_io[nv + i]; }
    int rc = op->method == 1 ? fire_run(&o, nv, x, op, res, phi_trace, trace_cap)
                             : lbfgs_run(&o, nv, x, op, res, phi_trace, trace_cap);
    for (int64_t i = 0; i < nv; i++) { x_io[i] = x[i].hi; x_io[nv + i] = x[i].lo; }
    free(x);
    return rc;
}
