/* Host sanitizer driver for the C oracle: every exported routine on small
 * and degenerate inputs (n = 1 .. 9, zero and diagonal matrices, 1-D to 3-D
 * lattices), built with AddressSanitizer and UndefinedBehaviorSanitizer by
 * tests/test_sanitize.py.  Any out-of-bounds access, leak or undefined
 * operation aborts the program; the few value checks catch gross failures
 * only (the oracle's pins test its results). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

void oracle_kinetic_1d(int N, double *T, double *T_imag);
int oracle_assemble(int ndim, const int *dims, const double *U, const double *Delta, double mu, double *Hout);
int oracle_zheev_jacobi(int n, double *Aio, double *W, double *Zout, double tol, int max_sweeps);
void oracle_zhetrd(int n, double *Aio, double *d, double *eio, double *tau);
int oracle_tridiag_ql(int n, double *d, double *e_in, double *Y);
int oracle_zheev_hqr(int n, const double *Ain, double *W, double *Zout, double *td, double *te);
int oracle_dstev(int n, const double *d_in, const double *e_in, double *W, double *Y);
int64_t oracle_sturm_count(int64_t n, const double *d, const double *e, double sigma);
double oracle_bisect(int64_t n, const double *d, const double *e, int64_t k);

static unsigned long long rs = 88172645463325252ull;
static double rnd(void) {
    rs ^= rs << 13; rs ^= rs >> 7; rs ^= rs << 17;
    return (double)(rs >> 11) / 9007199254740992.0 - 0.5;
}

static void herm(int n, double *A, int kind) {
    for (int j = 0; j < n; ++j)
        for (int i = j; i < n; ++i) {
            double re = kind == 0 ? rnd() : 0.0, im = (kind == 0 && i != j) ? rnd() : 0.0;
            if (kind == 1 && i == j) re = (double)(i % 3);  /* diagonal, repeated values */
            A[2 * (i + (size_t)j * n)] = re; A[2 * (i + (size_t)j * n) + 1] = im;
            A[2 * (j + (size_t)i * n)] = re; A[2 * (j + (size_t)i * n) + 1] = -im;
        }
}

static int sorted(int n, const double *W) {
    for (int i = 1; i < n; ++i) if (!(W[i - 1] <= W[i])) return 0;
    return 1;
}

int main(void) {
    int bad = 0;
    for (int N = 1; N <= 7; ++N) {
        double *T = malloc(sizeof(double) * N * N), *Ti = malloc(sizeof(double) * N * N);
        oracle_kinetic_1d(N, T, Ti);
        oracle_kinetic_1d(N, T, NULL);
        free(T); free(Ti);
    }
    const int lat[][4] = {{1, 1, 0, 0}, {1, 5, 0, 0}, {2, 3, 2, 0}, {3, 2, 2, 3}, {3, 1, 1, 1}};
    for (size_t L = 0; L < sizeof(lat) / sizeof(lat[0]); ++L) {
        const int nd = lat[L][0];
        int ns = 1;
        for (int d = 0; d < nd; ++d) ns *= lat[L][1 + d];
        const int n = 2 * ns;
        double *U = malloc(sizeof(double) * ns), *D = malloc(sizeof(double) * 2 * ns);
        for (int i = 0; i < ns; ++i) { U[i] = rnd(); D[2 * i] = rnd(); D[2 * i + 1] = rnd(); }
        double *H = malloc(sizeof(double) * 2 * (size_t)n * n), *W = malloc(sizeof(double) * n);
        double *Z = malloc(sizeof(double) * 2 * (size_t)n * n);
        if (oracle_assemble(nd, &lat[L][1], U, D, 0.3, H) != 0) bad |= 1;
        if (oracle_zheev_hqr(n, H, W, Z, NULL, NULL) != 0 || !sorted(n, W)) bad |= 2;
        free(U); free(D); free(H); free(W); free(Z);
    }
    {
        int dims[1] = {4};
        double U[4] = {0}, D[8] = {0}, H[2 * 8 * 8];
        if (oracle_assemble(0, dims, U, D, 0.0, H) == 0) bad |= 4;  /* ndim outside 1..3 refused */
    }
    for (int n = 1; n <= 9; ++n)
        for (int kind = 0; kind < 3; ++kind) {
            double *A = malloc(sizeof(double) * 2 * n * n), *B = malloc(sizeof(double) * 2 * n * n);
            double *W = malloc(sizeof(double) * n), *W2 = malloc(sizeof(double) * n);
            double *Z = malloc(sizeof(double) * 2 * n * n), *td = malloc(sizeof(double) * n);
            double *te = malloc(sizeof(double) * n), *tau = malloc(sizeof(double) * n);
            double *d = malloc(sizeof(double) * n), *e = malloc(sizeof(double) * 2 * n);
            double *Y = malloc(sizeof(double) * n * n);
            herm(n, A, kind);
            memcpy(B, A, sizeof(double) * 2 * n * n);
            /* returns the sweep count, or -1 without convergence; Z is required */
            if (oracle_zheev_jacobi(n, B, W, Z, 1e-15, 100) < 0 || !sorted(n, W)) bad |= 8;
            if (oracle_zheev_hqr(n, A, W2, Z, td, te) != 0 || !sorted(n, W2)) bad |= 16;
            if (oracle_zheev_hqr(n, A, W2, NULL, NULL, NULL) != 0) bad |= 16;
            for (int i = 0; i < n; ++i) if (fabs(W[i] - W2[i]) > 1e-10) bad |= 32;
            memcpy(B, A, sizeof(double) * 2 * n * n);
            oracle_zhetrd(n, B, d, e, tau);
            memcpy(d, td, sizeof(double) * n);
            for (int i = 0; i + 1 < n; ++i) e[i] = te[i];
            if (oracle_dstev(n, d, e, W, Y) != 0 || !sorted(n, W)) bad |= 64;
            if (oracle_dstev(n, d, e, W, NULL) != 0) bad |= 64;
            for (int64_t k = 0; k < n; ++k) {
                const double x = oracle_bisect(n, d, e, k);
                if (fabs(x - W[k]) > 1e-9 * (1.0 + fabs(W[k]))) bad |= 128;
            }
            if (oracle_sturm_count(n, d, e, 1e300) != n || oracle_sturm_count(n, d, e, -1e300) != 0) bad |= 256;
            double *dq = malloc(sizeof(double) * n), *eq = malloc(sizeof(double) * n);
            memcpy(dq, d, sizeof(double) * n);
            memcpy(eq, e, sizeof(double) * n);
            if (oracle_tridiag_ql(n, dq, eq, NULL) != 0) bad |= 512;
            free(dq); free(eq);
            free(A); free(B); free(W); free(W2); free(Z); free(td); free(te); free(tau); free(d); free(e); free(Y);
        }
    if (oracle_tridiag_ql(0, NULL, NULL, NULL) != 0) bad |= 1024;
    printf("sanitize_oracle: %s (flags %d)\n", bad ? "FAILED" : "ok", bad);
    return bad ? 1 : 0;
}
