// tables.hip - S1 on the device: the 1D integrals of the separable kernel
// transform (eq. Gten_sep, Algorithm 1 step 1),
//   J0_s(k) = int_{-L/2}^{L/2} exp(-a_s y^2) cos(2 pi k y / L) dy,
//   J2_s(k) = int_{-L/2}^{L/2} y^2 exp(-a_s y^2) cos(2 pi k y / L) dy,
// s < R, k = 0..n, written straight into the device tables the spectrum
// build (S2) reads.
//  * a (L/2)^2 >= 50: beyond L/2 the Gaussian is below e^-50 of its mass and
//    the full-line closed forms hold,
//      J0 = sqrt(pi/a) e^{-xi^2/(4a)},  J2 = J0 (2a - xi^2) / (4a^2),
//    with xi = 2 pi k / L;
//  * otherwise the 15-point Gauss-Kronrod rule on equal panels of [0, b],
//    b = min(L/2, 8.6/sqrt(a)) (beyond 8.6/sqrt(a) the integrand is below
//    e^-74 of its peak), panels no wider than half a cosine period at k = n
//    (the rule's error there is ~1e-18 of the integrand) or half the
//    Gaussian's width; all of it in double-double (tables.hpp).
// One workgroup of TAB_W waves per (s, block of 64 wavenumbers): wave w takes
// the w-th contiguous share of the nodes, stages 64 of them at a time in LDS
// (phase, weights) and every lane sums its wavenumber over them in order;
// the waves' partial sums are then added in wave order, so the tables are
// deterministic.
#include <algorithm>
#include <cmath>
#include <vector>

#include "host_common.hpp"
#include "tables.hpp"

namespace psp {

constexpr int TAB_K = 64;   // wavenumbers per workgroup (one per lane)
constexpr int TAB_W = 8;    // waves per workgroup, each over its share of the nodes

__global__ void __launch_bounds__(TAB_K * TAB_W)
k_tables(const TabJob *__restrict__ jobs, const TabTrig *__restrict__ trig_g, TabRule rule, dd inv_l,
         dd two_pi_l, int n, double *__restrict__ J0, double *__restrict__ J2) {
    __shared__ TabTrig trig[TAB_TRIG / 2 + 1];
    __shared__ dd sq[TAB_W][TAB_K], sg0[TAB_W][TAB_K], sg2[TAB_W][TAB_K];
    __shared__ dd p0[TAB_W][TAB_K], p2[TAB_W][TAB_K];
    const int s = blockIdx.y;
    const int lane = threadIdx.x % TAB_K, w = threadIdx.x / TAB_K;
    const int k = blockIdx.x * TAB_K + lane;
    const TabJob jb = jobs[s];
    double *j0 = J0 + (size_t)s * (n + 1), *j2 = J2 + (size_t)s * (n + 1);
    if (jb.closed) {                                  // uniform over the workgroup
        if (w == 0 && k <= n) tab_closed(jb.a, two_pi_l, k, rule, &j0[k], &j2[k]);
        return;
    }
    for (int i = threadIdx.x; i <= TAB_TRIG / 2; i += TAB_K * TAB_W) trig[i] = trig_g[i];
    // wave w: nodes [w * share, (w + 1) * share), in blocks of TAB_K; every
    // wave runs the same number of blocks, so the barriers stay uniform
    const int nodes = 15 * jb.panels;
    const int share = (nodes + TAB_W - 1) / TAB_W;
    const int lo = w * share, hi = min(nodes, lo + share);
    dd s0{0.0, 0.0}, s2{0.0, 0.0};
    for (int base = 0; base < share; base += TAB_K) {
        const int idx = lo + base + lane;
        if (idx < hi) tab_node(rule, jb, inv_l, idx, &sq[w][lane], &sg0[w][lane], &sg2[w][lane]);
        __syncthreads();
        const int cnt = max(0, min(TAB_K, hi - (lo + base)));
        if (k <= n) {
            for (int i = 0; i < cnt; ++i) {
                const dd c = tab_cos(rule, trig, k, sq[w][i]);
                s0 = dd_add(s0, dd_mul(sg0[w][i], c));
                s2 = dd_add(s2, dd_mul(sg2[w][i], c));
            }
        }
        __syncthreads();
    }
    p0[w][lane] = s0;
    p2[w][lane] = s2;
    __syncthreads();
    if (w == 0 && k <= n) {
        dd t0 = p0[0][lane], t2 = p2[0][lane];
        for (int v = 1; v < TAB_W; ++v) {
            t0 = dd_add(t0, p0[v][lane]);
            t2 = dd_add(t2, p2[v][lane]);
        }
        j0[k] = 2.0 * (t0.hi + t0.lo);
        j2[k] = 2.0 * (t2.hi + t2.lo);
    }
}

// Gauss-Kronrod 7/15 nodes (x_0 > ... > x_7 = 0) and Kronrod weights on
// [-1, 1] (checked against the rule recomputed in 50-digit arithmetic:
// exact for polynomials of degree <= 22 to 1e-30)
typedef long double ld;
static const ld kXgk[8] = {
    0.991455371120812639206854697526329L, 0.949107912342758524526189684047851L,
    0.864864423359769072789712788640926L, 0.741531185599394439863864773280788L,
    0.586087235467691130294144838258729598L, 0.405845151377397166906606412076961L,
    0.207784955007898467600689403773245L, 0.000000000000000000000000000000000L};
static const ld kWgk[8] = {
    0.022935322010529224963732008058970L, 0.063092092629978553290700663189204L,
    0.104790010322250183839876322541518L, 0.140653259715525918745189590510238L,
    0.169004726639267902826583426598550L, 0.190350578064785409913256402421014L,
    0.204432940075298892414161999234649L, 0.209482141084727828012999174891714L};

static void split(ld v, double *hi, double *lo) {
    *hi = (double)v;
    *lo = (double)(v - (ld)*hi);
}

TabRule table_rule() {
    TabRule r;
    for (int i = 0; i < 8; ++i) {
        split(kXgk[i], &r.x_hi[i], &r.x_lo[i]);
        split(kWgk[i], &r.w_hi[i], &r.w_lo[i]);
    }
    split(6.283185307179586476925286766559005768L, &r.two_pi_hi, &r.two_pi_lo);
    split(0.693147180559945309417232121458176568L, &r.ln2_hi, &r.ln2_lo);
    return r;
}

std::vector<TabTrig> table_trig() {
    std::vector<TabTrig> t(TAB_TRIG / 2 + 1);
    const ld two_pi = 6.283185307179586476925286766559005768L;
    for (int j = 0; j <= TAB_TRIG / 2; ++j) {
        const ld a = two_pi * (ld)j / (ld)TAB_TRIG;
        split(cosl(a), &t[j].c_hi, &t[j].c_lo);
        split(sinl(a), &t[j].s_hi, &t[j].s_lo);
    }
    return t;
}

std::vector<TabJob> table_jobs(const std::vector<double> &alpha, int n, double L) {
    std::vector<TabJob> jobs(alpha.size());
    const double half = 0.5 * L;
    for (size_t s = 0; s < alpha.size(); ++s) {
        const double a = alpha[s];
        TabJob &jb = jobs[s];
        jb.a = a;
        if (a * half * half >= 50.0) {
            jb.closed = 1;
            jb.panels = 0;
            jb.dy_hi = jb.dy_lo = 0.0;
            continue;
        }
        jb.closed = 0;
        const double b = std::min(half, 8.6 / std::sqrt(a));
        double w0 = std::min(b, 0.5 / std::sqrt(a));
        if (n > 0) w0 = std::min(w0, L / (2.0 * n));
        jb.panels = std::max(1, (int)std::ceil(b / w0 - 1e-12));
        const dd dy = dd_div_d(dd{b, 0.0}, (double)jb.panels);
        jb.dy_hi = dy.hi;
        jb.dy_lo = dy.lo;
    }
    return jobs;
}

hipError_t launch_tables(const std::vector<TabJob> &jobs, const std::vector<TabTrig> &trig, int n, double L,
                         double *J0, double *J2, TabJob *jobs_dev, TabTrig *trig_dev, hipStream_t st) {
    const int R = (int)jobs.size();
    hipError_t e = hipMemcpyAsync(jobs_dev, jobs.data(), sizeof(TabJob) * R, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(trig_dev, trig.data(), sizeof(TabTrig) * trig.size(), hipMemcpyHostToDevice, st);
    if (e != hipSuccess) return e;
    dd inv_l{1.0 / L, 0.0};
    inv_l.lo = (double)((1.0L - (ld)L * (ld)inv_l.hi) / (ld)L);
    dd two_pi_l;
    split(6.283185307179586476925286766559005768L / (ld)L, &two_pi_l.hi, &two_pi_l.lo);
    dim3 grid((n + 1 + TAB_K - 1) / TAB_K, R);
    hipLaunchKernelGGL(k_tables, grid, dim3(TAB_K * TAB_W), 0, st, jobs_dev, trig_dev, table_rule(), inv_l, two_pi_l,
                       n, J0, J2);
    return hipGetLastError();
}

}  // namespace psp
