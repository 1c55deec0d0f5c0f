/*
 * The oracle's C FFT (oracle/naive_fft.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: every axis of small arrays with lengths 2^a 3^b
 * (and a rejected length), against the DFT sum written out.  Exits 0 when
 * every transform is within 1e-12 of the sum.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_fft_axis(double *a, long d0, long d1, long d2, int axis, int sign);
int oracle_set_threads(int t);

int main(void) {
    const long lens[] = {1, 2, 3, 4, 6, 9, 12, 18, 27, 36, 64};
    int failures = 0;
    oracle_set_threads(2);
    for (unsigned li = 0; li < sizeof(lens) / sizeof(lens[0]); ++li) {
        for (int axis = 0; axis < 3; ++axis) {
            long d[3] = {2, 3, 2};
            d[axis] = lens[li];
            const long total = d[0] * d[1] * d[2];
            double *a = malloc(sizeof(double) * 2 * total), *b = malloc(sizeof(double) * 2 * total);
            for (long i = 0; i < 2 * total; ++i) a[i] = b[i] = sin(0.7 * i + axis) + 0.1 * i;
            if (oracle_fft_axis(a, d[0], d[1], d[2], axis, -1) != 0) ++failures;
            long inner = 1;
            for (int q = axis + 1; q < 3; ++q) inner *= d[q];
            const long N = d[axis];
            for (long line = 0; line < total / N; ++line) {
                const long base = (line / inner) * N * inner + line % inner;
                for (long k = 0; k < N; ++k) {
                    double re = 0, im = 0;
                    for (long j = 0; j < N; ++j) {
                        const double ang = -2.0 * M_PI * (double)((j * k) % N) / (double)N;
                        const double xr = b[2 * (base + j * inner)], xi = b[2 * (base + j * inner) + 1];
                        re += xr * cos(ang) - xi * sin(ang);
                        im += xr * sin(ang) + xi * cos(ang);
                    }
                    const double *y = a + 2 * (base + k * inner);
                    if (fabs(y[0] - re) > 1e-12 * (1 + fabs(re)) || fabs(y[1] - im) > 1e-12 * (1 + fabs(im))) ++failures;
                }
            }
            free(a);
            free(b);
        }
    }
    double z[2 * 10] = {0};
    if (oracle_fft_axis(z, 1, 1, 10, 2, -1) != -1) ++failures;     /* length 10: rejected */
    printf("oracle_fft_driver: %d failures\n", failures);
    return failures ? 1 : 0;
}
