/*
 * naive_fft.c - the oracle's own discrete Fourier transform, in plain C.
 *
 * TEST INFRASTRUCTURE.  Only the oracle (oracle/psp_oracle.py) loads this
 * file's library; it shares no code with the GPU library.
 *
 * What it computes: along one axis of a C-ordered 3D complex array, every
 * line x[0..N) is replaced by its unnormalised DFT
 *     X[k] = sum_{j<N} x[j] exp(sign * 2 pi i j k / N),   k < N,
 * for N a product of 2s and 3s (the padded lengths of the method's zero
 * padding by a factor 2, Section 2).  The algorithm is the textbook
 * recursive decimation in time: while N is even, split the inputs into the
 * even and odd samples, otherwise into the three residue classes mod 3;
 * transform each class (length M = N/p) and combine
 *     X[k] = sum_{r<p} W_N^{r k} Y_r[k mod M],   W_N = exp(sign 2 pi i / N).
 * No pruning, no blocking: the same operation count for every line.  The
 * twiddles are cos and sin of sign * 2 pi m / N0 in double precision (N0 the
 * line length), taken from one table of m < N0: a sub-transform of length
 * N = N0 / s uses entry (e mod N) * s for W_N^e, the same angle.
 *
 * Lines are independent, so they are spread over OpenMP threads; each line
 * is copied to a contiguous buffer, transformed and copied back.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double re, im;
} cpx;

static int is_2_3_smooth(long N) {
    if (N < 1) return 0;
    while (N % 2 == 0) N /= 2;
    while (N % 3 == 0) N /= 3;
    return N == 1;
}

/* out[k] = sum_j x[j * xs] W^{jk} for k < N; tw[m * step] = W_N^m.
 * out and work each hold N values; work is scratch. */
static void dft_rec(const cpx *x, long xs, long N, const cpx *tw, long step, cpx *out, cpx *work) {
    if (N == 1) {
        out[0] = x[0];
        return;
    }
    const long p = (N % 2 == 0) ? 2 : 3;
    const long M = N / p;
    /* sub-transform r of the samples x[r], x[r + p], ... into work[r M ..),
     * with out[r M ..) as its scratch */
    for (long r = 0; r < p; ++r) dft_rec(x + r * xs, xs * p, M, tw, step * p, work + r * M, out + r * M);
    /* e[r] = (r k) mod N and kk = k mod M, advanced with k (no division) */
    long e[3] = {0, 0, 0}, kk = 0;
    for (long k = 0; k < N; ++k) {
        double re = 0.0, im = 0.0;
        for (long r = 0; r < p; ++r) {
            const cpx w = tw[e[r] * step];
            const cpx y = work[r * M + kk];
            re += w.re * y.re - w.im * y.im;
            im += w.re * y.im + w.im * y.re;
            e[r] += r;
            if (e[r] >= N) e[r] -= N;
        }
        out[k].re = re;
        out[k].im = im;
        if (++kk == M) kk = 0;
    }
}

/* Threads of the following transforms (OpenMP); t <= 0 keeps the default
 * (OMP_NUM_THREADS or the core count).  Returns the count now in force. */
int oracle_set_threads(int t) {
    if (t > 0) omp_set_num_threads(t);
    return omp_get_max_threads();
}

/* DFT along `axis` (0, 1 or 2) of the C-ordered array a[d0][d1][d2] of
 * interleaved (re, im) doubles, in place.  sign = -1 forward, +1 inverse
 * (no scaling).  Returns 0, or -1 for a length that is not a product of 2s
 * and 3s or another bad argument, -2 if memory runs out. */
int oracle_fft_axis(double *a, long d0, long d1, long d2, int axis, int sign) {
    const long dims[3] = {d0, d1, d2};
    if (!a || axis < 0 || axis > 2 || (sign != 1 && sign != -1)) return -1;
    if (d0 < 1 || d1 < 1 || d2 < 1) return -1;
    const long N = dims[axis];
    if (!is_2_3_smooth(N)) return -1;
    long inner = 1;                     /* stride of the axis, in elements */
    for (int q = axis + 1; q < 3; ++q) inner *= dims[q];
    const long lines = d0 * d1 * d2 / N;
    cpx *tw = (cpx *)malloc(sizeof(cpx) * N);
    if (!tw) return -2;
    for (long m = 0; m < N; ++m) {
        const double ang = sign * 2.0 * M_PI * (double)m / (double)N;
        tw[m].re = cos(ang);
        tw[m].im = sin(ang);
    }
    cpx *data = (cpx *)a;
    int failed = 0;
#pragma omp parallel
    {
        cpx *buf = (cpx *)malloc(sizeof(cpx) * 3 * N);
        if (!buf) {
#pragma omp atomic write
            failed = 1;
        }
#pragma omp for schedule(static)
        for (long q = 0; q < lines; ++q) {
            if (!buf) continue;
            /* line q: outer index q / inner, inner index q % inner */
            cpx *line = data + (q / inner) * N * inner + (q % inner);
            cpx *x = buf, *out = buf + N, *work = buf + 2 * N;
            for (long j = 0; j < N; ++j) x[j] = line[j * inner];
            dft_rec(x, 1, N, tw, 1, out, work);
            for (long k = 0; k < N; ++k) line[k * inner] = out[k];
        }
        free(buf);
    }
    free(tw);
    return failed ? -2 : 0;
}
