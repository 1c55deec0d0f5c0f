// tables.hpp - the arithmetic of the 1D-integral tables (Algorithm 1 step 1,
// eq. Gten_sep), used by the device kernel in tables.hip:
//   J_p(k) = 2 int_0^{b} y^p exp(-a y^2) cos(2 pi k y / L) dy,  p in {0, 2},
// by the 15-point Gauss-Kronrod rule on equal panels of [0, b].
//
// At high k these integrals are ~k^2 smaller than their integrands, and the
// kernel spectrum sums them with cancellation between Gaussians, so every
// quantity is carried in double-double (~1e-19 and better): the node and its
// phase q = y / L, the node weight h w exp(-a y^2), the cosine of the
// exactly reduced phase (a 256-entry table of cos and sin plus short Taylor
// series), the products and the sums.  Only the final table entry is
// rounded to double.
#pragma once
#include <cmath>

#ifdef __HIPCC__
#define PSP_HD __host__ __device__ __forceinline__
#else
#define PSP_HD inline
#endif

namespace psp {

struct dd {
    double hi, lo;
};

PSP_HD dd dd_two_sum(double a, double b) {
    const double s = a + b;
    const double bb = s - a;
    return dd{s, (a - (s - bb)) + (b - bb)};
}
PSP_HD dd dd_quick(double a, double b) {   // |a| >= |b|
    const double s = a + b;
    return dd{s, b - (s - a)};
}
PSP_HD dd dd_two_prod(double a, double b) {
    const double p = a * b;
    return dd{p, fma(a, b, -p)};
}
PSP_HD dd dd_neg(dd a) { return dd{-a.hi, -a.lo}; }
// sum with both parts compensated (exact to ~2^-104 also under cancellation)
PSP_HD dd dd_add(dd a, dd b) {
    dd s = dd_two_sum(a.hi, b.hi);
    const dd t = dd_two_sum(a.lo, b.lo);
    s.lo += t.hi;
    s = dd_quick(s.hi, s.lo);
    s.lo += t.lo;
    return dd_quick(s.hi, s.lo);
}
PSP_HD dd dd_mul(dd a, dd b) {
    const dd p = dd_two_prod(a.hi, b.hi);
    return dd_quick(p.hi, p.lo + (a.hi * b.lo + a.lo * b.hi));
}
PSP_HD dd dd_mul_d(dd a, double b) {
    const dd p = dd_two_prod(a.hi, b);
    return dd_quick(p.hi, p.lo + a.lo * b);
}
PSP_HD dd dd_div_d(dd a, double b) {
    const double q1 = a.hi / b;
    const dd p = dd_two_prod(q1, b);
    const double q2 = ((a.hi - p.hi) - p.lo + a.lo) / b;
    return dd_quick(q1, q2);
}

// the Gauss-Kronrod 7/15 rule on [-1, 1]: nodes x_0 > ... > x_7 = 0 and
// Kronrod weights, double-double; the rule is symmetric.  2 pi and ln 2.
struct TabRule {
    double x_hi[8], x_lo[8], w_hi[8], w_lo[8];
    double two_pi_hi, two_pi_lo, ln2_hi, ln2_lo;
};

// cos and sin of 2 pi j / TAB_TRIG, j = 0..TAB_TRIG/2, double-double
constexpr int TAB_TRIG = 256;
struct TabTrig {
    double c_hi, c_lo, s_hi, s_lo;
};

// one Gaussian of the sum: exponent a, panel width dy = b / panels as a
// double-double (a rounded dy would move the end of the interval by an ulp,
// which for a nearly flat Gaussian is a ~1e-16 error in integrals of size
// ~1e-6); closed != 0: a (L/2)^2 is large enough for the full-line closed
// forms
struct TabJob {
    double a, dy_hi, dy_lo;
    int panels, closed;
};

// exp(-t) for 0 <= t < ~700: t = m ln 2 + r, |r| <= ln 2 / 2, Taylor
// series of exp(-r) to r^20 / 20! (< 1e-25) by Horner's rule, scaled by 2^-m
PSP_HD dd dd_exp_neg(dd t, const TabRule &rl) {
    const double m = rint(t.hi / rl.ln2_hi);
    const dd r = dd_add(t, dd_neg(dd_mul_d(dd{rl.ln2_hi, rl.ln2_lo}, m)));
    const dd x = dd_neg(r);
    dd acc{1.0, 0.0};
    for (int i = 20; i >= 1; --i) acc = dd_add(dd{1.0, 0.0}, dd_div_d(dd_mul(x, acc), (double)i));
    const int e = -(int)m;
    return dd{ldexp(acc.hi, e), ldexp(acc.lo, e)};
}

// the full-line closed forms at xi = 2 pi k / L (two_pi_l: 2 pi / L):
//   J0 = sqrt(pi/a) exp(-xi^2/(4a)),  J2 = J0 (2a - xi^2) / (4a^2),
// with xi^2, the exponent and 2a - xi^2 (which cancels near the zero of J2)
// in double-double
PSP_HD void tab_closed(double a, dd two_pi_l, int k, const TabRule &rl, double *j0, double *j2) {
    const dd xi = dd_mul_d(two_pi_l, (double)k);
    const dd xi2 = dd_mul(xi, xi);
    const dd e = dd_exp_neg(dd_div_d(xi2, 4.0 * a), rl);
    const double j = sqrt(3.14159265358979323846 / a) * (e.hi + e.lo);
    const dd d = dd_add(dd{2.0 * a, 0.0}, dd_neg(xi2));
    *j0 = j;
    *j2 = j * ((d.hi + d.lo) / (4.0 * a * a));
}

// node idx < 15 * panels (panel idx / 15, position idx % 15 as in the
// rule's order: c - hw x_j for j < 8, c + hw x_{14-j} after): its phase
// y / L and its weights for p = 0 and p = 2
PSP_HD void tab_node(const TabRule &rl, const TabJob &jb, dd inv_l, int idx, dd *q, dd *g0, dd *g2) {
    const int i = idx / 15, j = idx % 15;
    const int m = j < 8 ? j : 14 - j;
    const double sg = j < 8 ? -0.5 : 0.5;
    // y = dy (i + 1/2 + x/2): the node of panel i
    const dd t = dd_add(dd{i + 0.5, 0.0}, dd{sg * rl.x_hi[m], sg * rl.x_lo[m]});
    const dd dy{jb.dy_hi, jb.dy_lo};
    const dd y = dd_mul(t, dy);
    *q = dd_mul(y, inv_l);
    const dd y2 = dd_mul(y, y);
    const dd e = dd_exp_neg(dd_mul_d(y2, jb.a), rl);
    *g0 = dd_mul(dd_mul(dd{rl.w_hi[m], rl.w_lo[m]}, dd_mul_d(dy, 0.5)), e);
    *g2 = dd_mul(*g0, y2);
}

// cos(2 pi k q): the phase k q reduced exactly to f in [-1/2, 1/2], then
// f = j / TAB_TRIG + r with |r| <= 1 / (2 TAB_TRIG): the table's cos and sin
// of 2 pi j / TAB_TRIG times Taylor series of cos and sin of x = 2 pi r
// (|x| < 0.0123; the dropped terms are below 1e-22)
PSP_HD dd tab_cos(const TabRule &rl, const TabTrig *trig, int k, dd q) {
    const dd p = dd_mul_d(q, (double)k);
    const double mi = rint(p.hi);
    const dd f = dd_two_sum(p.hi - mi, p.lo);           // p.hi - mi is exact
    const double jd = rint(f.hi * (double)TAB_TRIG);
    const dd rf = dd_two_sum(f.hi - jd / TAB_TRIG, f.lo);  // exact difference
    const dd x = dd_mul(rf, dd{rl.two_pi_hi, rl.two_pi_lo});
    const double x2 = x.hi * x.hi;
    const dd h2 = dd_mul_d(dd_mul(x, x), 0.5);
    const double ct = x2 * x2 * (1.0 / 24.0 - x2 * (1.0 / 720.0 - x2 * (1.0 / 40320.0)));
    const double st = -x.hi * x2 * (1.0 / 6.0 - x2 * (1.0 / 120.0 - x2 * (1.0 / 5040.0)));
    const dd cx = dd_add(dd_add(dd{1.0, 0.0}, dd_neg(h2)), dd{ct, 0.0});
    const dd sx = dd_add(x, dd{st, 0.0});
    const int j = (int)jd;
    const TabTrig T = trig[j < 0 ? -j : j];
    const double sg = j < 0 ? -1.0 : 1.0;
    const dd a = dd_mul(dd{T.c_hi, T.c_lo}, cx);
    const dd b = dd_mul(dd{sg * T.s_hi, sg * T.s_lo}, sx);
    return dd_add(a, dd_neg(b));
}

}  // namespace psp
