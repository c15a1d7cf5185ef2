/*
 * CPU oracle for the dense BdG eigenproblem (test infrastructure only).
 *
 * Plain, slow, FP64 implementations of what the GPU path computes, written
 * from the definitions in the paper and from textbook algorithms:
 *
 *   - oracle_kinetic_1d / oracle_assemble: the quasiparticle Hamiltonian of
 *     the static BdG/SLDA eigenproblem (paper eq. stHpsi with eq. TDSLDA's
 *     block structure) on the periodic spectral grid of "Numerical setup and
 *     implementation": the kinetic term is F^-1 (k^2/2) F with momenta
 *     k = 2 pi n / N, n = -N/2 .. N/2-1, evaluated here as the direct Fourier
 *     sum over those momenta (no closed form, no FFT).
 *   - oracle_zheev_jacobi: complex cyclic Jacobi (Golub & Van Loan, Matrix
 *     Computations, sec. 8.5), the plain definition of a Hermitian
 *     eigendecomposition Z^H Z = I, H Z = Z W.
 *   - oracle_zhetrd + oracle_tridiag_ql + oracle_zheev_hqr: unblocked
 *     Householder reduction to a real tridiagonal (phase-scaled) followed by
 *     implicit QL with a Wilkinson-type shift (G&VL sec. 8.3), optional
 *     eigenvector accumulation and back-transformation.  The QL iteration is
 *     the classical formulation of Bowdler, Martin, Reinsch and Wilkinson's
 *     tql2 (Numer. Math. 11, 1968; Handbook for Automatic Computation II,
 *     1971): implicit shifted QL sweeps with plane rotations chasing from the
 *     bottom of each unreduced block, and the same underflow split.
 *   - oracle_sturm_count / oracle_bisect: Sturm-sequence counts and bisection
 *     on a real symmetric tridiagonal (G&VL sec. 8.4).
 *
 * Storage: complex numbers interleaved (re, im) as double pairs; matrices
 * column-major with leading dimension n.  Nothing here is shared with the GPU
 * library.  Only tests, the smoke check and the CPU-baseline leg of the
 * benchmark may call this code.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { double re, im; } cplx;

static inline cplx c_make(double r, double i) { cplx z = {r, i}; return z; }
static inline cplx c_add(cplx a, cplx b) { return c_make(a.re + b.re, a.im + b.im); }
static inline cplx c_sub(cplx a, cplx b) { return c_make(a.re - b.re, a.im - b.im); }
static inline cplx c_mul(cplx a, cplx b) { return c_make(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static inline cplx c_conj(cplx a) { return c_make(a.re, -a.im); }
static inline cplx c_scale(cplx a, double s) { return c_make(a.re * s, a.im * s); }
static inline double c_abs2(cplx a) { return a.re * a.re + a.im * a.im; }
static inline double c_abs(cplx a) { return hypot(a.re, a.im); }
/* conj(a) * b */
static inline cplx c_cmul(cplx a, cplx b) { return c_make(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re); }

#define AT(A, n, i, j) ((A)[(size_t)(j) * (size_t)(n) + (size_t)(i)])

/* Test builds compile this file with -DORACLE_MUTANT=k (k > 0) to plant one
   plausible mistake and check that the pins in the test-suite catch it.  The
   default build (0) has none. */
#ifndef ORACLE_MUTANT
#define ORACLE_MUTANT 0
#endif

/* ------------------------------------------------------------------------ */
/* Kinetic operator: T_ab = (1/N) sum_k (k^2/2) exp(i k (a-b)), k = 2 pi n/N, */
/* n = -N/2 .. N/2-1.  The imaginary part (from the unpaired -N/2 mode) is   */
/* returned so that callers can check it vanishes.                            */
/* ------------------------------------------------------------------------ */
void oracle_kinetic_1d(int N, double *T, double *T_imag)
{
    for (int a = 0; a < N; ++a)
        for (int b = 0; b < N; ++b) {
            double sr = 0.0, si = 0.0;
#if ORACLE_MUTANT == 1
            for (int n = 0; n < N; ++n) {
#else
            for (int n = -N / 2; n <= N / 2 - 1 + (N % 2); ++n) {
#endif
                double k = 2.0 * M_PI * (double)n / (double)N;
                double ph = k * (double)(a - b);
                sr += 0.5 * k * k * cos(ph);
                si += 0.5 * k * k * sin(ph);
            }
            T[(size_t)b * N + a] = sr / (double)N;
            if (T_imag) T_imag[(size_t)b * N + a] = si / (double)N;
        }
}

/*
 * H = [[h, diag(Delta)], [diag(conj Delta), -conj(h)]], h = sum_d T_d + diag(U - mu),
 * with site index r = x + Nx (y + Ny z) and the u-block first.
 * H is n x n complex, n = 2 * prod(dims), column-major (interleaved re/im).
 */
int oracle_assemble(int ndim, const int *dims, const double *U, const double *Delta,
                    double mu, double *Hout)
{
    if (ndim < 1 || ndim > 3) return -1;
    int N[3] = {1, 1, 1};
    for (int d = 0; d < ndim; ++d) N[d] = dims[d];
    const int64_t ns = (int64_t)N[0] * N[1] * N[2];
    const int64_t n = 2 * ns;
    cplx *H = (cplx *)Hout;
    memset(H, 0, sizeof(cplx) * (size_t)n * (size_t)n);
    double *T[3] = {0, 0, 0};
    for (int d = 0; d < ndim; ++d) {
        T[d] = (double *)malloc(sizeof(double) * (size_t)N[d] * N[d]);
        oracle_kinetic_1d(N[d], T[d], NULL);
    }
    /* single-particle h (complex in general; real here) */
    for (int64_t r = 0; r < ns; ++r) {
        int x = (int)(r % N[0]), y = (int)((r / N[0]) % N[1]), z = (int)(r / ((int64_t)N[0] * N[1]));
        for (int64_t s = 0; s < ns; ++s) {
            int xs = (int)(s % N[0]), ys = (int)((s / N[0]) % N[1]), zs = (int)(s / ((int64_t)N[0] * N[1]));
            double h = 0.0;
            if (y == ys && z == zs) h += T[0][(size_t)xs * N[0] + x];
            if (ndim > 1 && x == xs && z == zs) h += T[1][(size_t)ys * N[1] + y];
            if (ndim > 2 && x == xs && y == ys) h += T[2][(size_t)zs * N[2] + z];
#if ORACLE_MUTANT == 3
            if (r == s) h += U[r];
#else
            if (r == s) h += U[r] - mu;
#endif
            /* u-u block: h ; v-v block: -conj(h) */
            AT(H, n, r, s) = c_make(h, 0.0);
#if ORACLE_MUTANT == 2
            AT(H, n, ns + r, ns + s) = c_make(h, 0.0);
#else
            AT(H, n, ns + r, ns + s) = c_make(-h, 0.0);
#endif
        }
        cplx D = c_make(Delta[2 * r], Delta[2 * r + 1]);
        AT(H, n, r, ns + r) = D;           /* upper-right: Delta      */
#if ORACLE_MUTANT == 4
        AT(H, n, ns + r, r) = D;
#else
        AT(H, n, ns + r, r) = c_conj(D);   /* lower-left: conj(Delta) */
#endif
    }
    for (int d = 0; d < ndim; ++d) free(T[d]);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Complex cyclic Jacobi.  A (n x n Hermitian, full storage) is destroyed.   */
/* Returns the number of sweeps, or -1 if not converged.                     */
/* ------------------------------------------------------------------------ */
static void sort_eig(int n, double *W, cplx *Z /* may be NULL */)
{
    /* selection sort on W with column swaps of Z (n is small here) */
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j) if (W[j] < W[k]) k = j;
        if (k != i) {
            double t = W[i]; W[i] = W[k]; W[k] = t;
            if (Z)
                for (int r = 0; r < n; ++r) {
                    cplx tz = AT(Z, n, r, i); AT(Z, n, r, i) = AT(Z, n, r, k); AT(Z, n, r, k) = tz;
                }
        }
    }
}

int oracle_zheev_jacobi(int n, double *Aio, double *W, double *Zout, double tol, int max_sweeps)
{
    cplx *A = (cplx *)Aio, *Z = (cplx *)Zout;
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) AT(Z, n, i, j) = c_make(i == j ? 1.0 : 0.0, 0.0);
    double fro2 = 0.0;
    for (size_t k = 0; k < (size_t)n * n; ++k) fro2 += c_abs2(A[k]);
    /* An entry is negligible when it is below tol * sqrt(|a_pp a_qq|) (the
       relative criterion of Demmel & Veselic) or below tol^2 * ||A||_F;
       the iteration stops after a sweep without any rotation. */
    const double floor_abs = tol * tol * sqrt(fro2) + 1e-300;
    int sweep;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        long nrot = 0;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                cplx b = AT(A, n, p, q);
                double r = c_abs(b);
                double app = AT(A, n, p, p).re, aqq = AT(A, n, q, q).re;
                if (r <= floor_abs || r <= tol * sqrt(fabs(app * aqq))) continue;
                ++nrot;
                /* phase e = b / |b| turns the block into [[app, r],[r, aqq]]  */
                cplx e = c_scale(b, 1.0 / r);
                double tau = (aqq - app) / (2.0 * r);
                double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double c = 1.0 / sqrt(1.0 + t * t), s = t * c;
                /* G = diag(1, conj e) * [[c, s], [-s, c]]  (acts on columns p, q) */
#if ORACLE_MUTANT == 7
                cplx ge = e;
#else
                cplx ge = c_conj(e);
#endif
                cplx g_pp = c_make(c, 0.0), g_pq = c_make(s, 0.0);
                cplx g_qp = c_scale(ge, -s), g_qq = c_scale(ge, c);
                /* columns p, q of G^H A G for rows k != p, q equal those of A G;
                   rows p, q follow by Hermitian symmetry */
                for (int k = 0; k < n; ++k) {
                    if (k == p || k == q) continue;
                    cplx akp = AT(A, n, k, p), akq = AT(A, n, k, q);
                    cplx np_ = c_add(c_mul(akp, g_pp), c_mul(akq, g_qp));
                    cplx nq_ = c_add(c_mul(akp, g_pq), c_mul(akq, g_qq));
                    AT(A, n, k, p) = np_;
                    AT(A, n, k, q) = nq_;
                    AT(A, n, p, k) = c_conj(np_);
                    AT(A, n, q, k) = c_conj(nq_);
                }
                AT(A, n, p, p) = c_make(app - t * r, 0.0);
                AT(A, n, q, q) = c_make(aqq + t * r, 0.0);
                AT(A, n, p, q) = c_make(0.0, 0.0);
                AT(A, n, q, p) = c_make(0.0, 0.0);
                /* Z <- Z G */
                for (int k = 0; k < n; ++k) {
                    cplx zkp = AT(Z, n, k, p), zkq = AT(Z, n, k, q);
                    AT(Z, n, k, p) = c_add(c_mul(zkp, g_pp), c_mul(zkq, g_qp));
                    AT(Z, n, k, q) = c_add(c_mul(zkp, g_pq), c_mul(zkq, g_qq));
                }
            }
        if (nrot == 0) break;
    }
    for (int i = 0; i < n; ++i) W[i] = AT(A, n, i, i).re;
    sort_eig(n, W, Z);
    return sweep < max_sweeps ? sweep : -1;
}

/* ------------------------------------------------------------------------ */
/* Householder reduction of a Hermitian matrix to tridiagonal form.          */
/* A (full storage) is overwritten: reflector k is stored in A[k+1:, k]      */
/* (unnormalised, first entry explicit), tau[k] its real scale, so that      */
/* H_k = I - tau_k v_k v_k^H.  d (n) real diagonal, e (n-1) complex sub-     */
/* diagonal (interleaved).                                                   */
/* ------------------------------------------------------------------------ */
void oracle_zhetrd(int n, double *Aio, double *d, double *eio, double *tau)
{
    cplx *A = (cplx *)Aio, *e = (cplx *)eio;
    cplx *p = (cplx *)malloc(sizeof(cplx) * (size_t)(n > 0 ? n : 1));
    for (int k = 0; k < n - 1; ++k) {
        const int L = n - k - 1;
        cplx *x = &AT(A, n, k + 1, k);
        double xn2 = 0.0;
        for (int i = 0; i < L; ++i) xn2 += c_abs2(x[i]);
        double xn = sqrt(xn2);
        cplx alpha = x[0];
        double aa = c_abs(alpha);
        double tail2 = xn2 - c_abs2(alpha);
        if (xn == 0.0 || (L == 1) || tail2 <= 0.0) {
            /* nothing to eliminate below the subdiagonal */
            tau[k] = 0.0;
            e[k] = alpha;
            continue;
        }
        cplx sgn = aa > 0.0 ? c_scale(alpha, 1.0 / aa) : c_make(1.0, 0.0);
        cplx beta = c_scale(sgn, -xn);
        x[0] = c_sub(alpha, beta);
        double vn2 = 2.0 * xn * (xn + aa);
        double t = 2.0 / vn2;
        tau[k] = t;
        e[k] = beta;
        /* p = t * A22 v */
        cplx *A22 = &AT(A, n, k + 1, k + 1);
        #pragma omp parallel for schedule(static)
        for (int i = 0; i < L; ++i) {
            double sr = 0.0, si = 0.0;
            for (int j = 0; j < L; ++j) {
                cplx a = A22[(size_t)j * n + i];
                sr += a.re * x[j].re - a.im * x[j].im;
                si += a.re * x[j].im + a.im * x[j].re;
            }
            p[i] = c_make(t * sr, t * si);
        }
        /* K = (t/2) v^H p ; w = p - K v */
        double Kr = 0.0, Ki = 0.0;
        for (int i = 0; i < L; ++i) {
            cplx q = c_cmul(x[i], p[i]);
            Kr += q.re; Ki += q.im;
        }
        cplx K = c_make(0.5 * t * Kr, 0.5 * t * Ki);
#if ORACLE_MUTANT != 5
        for (int i = 0; i < L; ++i) p[i] = c_sub(p[i], c_mul(K, x[i]));
#endif
        /* A22 -= v w^H + w v^H */
        #pragma omp parallel for schedule(static)
        for (int j = 0; j < L; ++j) {
            cplx wj = c_conj(p[j]), vj = c_conj(x[j]);
            for (int i = 0; i < L; ++i) {
                cplx upd = c_add(c_mul(x[i], wj), c_mul(p[i], vj));
                A22[(size_t)j * n + i] = c_sub(A22[(size_t)j * n + i], upd);
            }
        }
    }
    for (int k = 0; k < n; ++k) d[k] = AT(A, n, k, k).re;
    free(p);
}

/* ------------------------------------------------------------------------ */
/* Implicit QL on a real symmetric tridiagonal (d: n, e: n-1, e[i] couples   */
/* i and i+1).  If Y != NULL it is an n x n row-major-by-column array        */
/* (column-major, leading dim n) that is post-multiplied by the rotations.   */
/* On exit d holds the (unsorted) eigenvalues.  Returns 0 or -1 (no conv.).  */
/* ------------------------------------------------------------------------ */
int oracle_tridiag_ql(int n, double *d, double *e_in, double *Y)
{
    if (n <= 0) return 0;
    double *e = (double *)calloc((size_t)n, sizeof(double));
    for (int i = 0; i < n - 1; ++i) e[i] = e_in[i];
    double *cs = (double *)malloc(sizeof(double) * 2 * (size_t)n);
    int rc = 0;
    for (int l = 0; l < n; ++l) {
        int iter = 0;
        for (;;) {
            int m;
            for (m = l; m < n - 1; ++m) {
                double dd = fabs(d[m]) + fabs(d[m + 1]);
                if (fabs(e[m]) <= 1e-300 || fabs(e[m]) <= 2.2e-16 * dd) break;
            }
            if (m == l) break;
            if (++iter > 60) { rc = -1; break; }
            /* shift from the leading 2x2 of the active block (eigenvalue of
               [[d_l, e_l],[e_l, d_l+1]] closer to d_l) */
            double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
            double r = hypot(g, 1.0);
            g = d[m] - d[l] + e[l] / (g + (g >= 0.0 ? r : -r));
            double s = 1.0, c = 1.0, p = 0.0;
            int i, nrot = 0, early = 0;
            for (i = m - 1; i >= l; --i) {
                double f = s * e[i], b = c * e[i];
                r = hypot(f, g);
                e[i + 1] = r;
                if (r == 0.0) {           /* underflow: split and restart */
                    d[i + 1] -= p;
                    e[m] = 0.0;
                    early = 1;
                    break;
                }
                s = f / r;
                c = g / r;
                g = d[i + 1] - p;
                r = (d[i] - g) * s + 2.0 * c * b;
                p = s * r;
                d[i + 1] = g + p;
                g = c * r - b;
                cs[2 * nrot] = c; cs[2 * nrot + 1] = s; ++nrot;
            }
            if (Y && nrot > 0) {
                /* rotation j acts on columns (m-1-j, m-j) */
                #pragma omp parallel for schedule(static)
                for (int row = 0; row < n; ++row) {
                    for (int j = 0; j < nrot; ++j) {
                        int col = m - 1 - j;
                        double cc = cs[2 * j], ss = cs[2 * j + 1];
                        double *y0 = &Y[(size_t)col * n + row];
                        double *y1 = &Y[(size_t)(col + 1) * n + row];
                        double f = *y1;
#if ORACLE_MUTANT == 6
                        *y1 = -ss * (*y0) + cc * f;
#else
                        *y1 = ss * (*y0) + cc * f;
#endif
                        *y0 = cc * (*y0) - ss * f;
                    }
                }
            }
            if (early) continue;
            d[l] -= p;
            e[l] = g;
            e[m] = 0.0;
        }
        if (rc) break;
    }
    free(e);
    free(cs);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Full Hermitian eigensolver via Householder + phase scaling + QL.          */
/* A is copied (not destroyed).  If Z != NULL, eigenvectors are returned.    */
/* The real tridiagonal (d, |e|) can be returned through td/te (may be NULL).*/
/* ------------------------------------------------------------------------ */
int oracle_zheev_hqr(int n, const double *Ain, double *W, double *Zout, double *td, double *te)
{
    cplx *A = (cplx *)malloc(sizeof(cplx) * (size_t)n * n);
    memcpy(A, Ain, sizeof(cplx) * (size_t)n * n);
    double *d = (double *)malloc(sizeof(double) * n);
    cplx *e = (cplx *)calloc((size_t)(n > 1 ? n - 1 : 1), sizeof(cplx));
    double *er = (double *)calloc((size_t)(n > 1 ? n - 1 : 1), sizeof(double));
    double *tau = (double *)calloc((size_t)n, sizeof(double));
    cplx *ph = (cplx *)malloc(sizeof(cplx) * n);
    oracle_zhetrd(n, (double *)A, d, (double *)e, tau);
    /* phase scaling: ph_0 = 1, ph_{k+1} = ph_k e_k / |e_k| makes the
       off-diagonal real and non-negative */
    ph[0] = c_make(1.0, 0.0);
    for (int k = 0; k < n - 1; ++k) {
        double a = c_abs(e[k]);
        er[k] = a;
        ph[k + 1] = a > 0.0 ? c_mul(ph[k], c_scale(e[k], 1.0 / a)) : ph[k];
    }
    if (td) memcpy(td, d, sizeof(double) * n);
    if (te && n > 1) memcpy(te, er, sizeof(double) * (n - 1));
    double *Y = NULL;
    if (Zout) {
        Y = (double *)calloc((size_t)n * n, sizeof(double));
        for (int i = 0; i < n; ++i) Y[(size_t)i * n + i] = 1.0;
    }
    int rc = oracle_tridiag_ql(n, d, er, Y);
    for (int i = 0; i < n; ++i) W[i] = d[i];
    if (Zout) {
        cplx *Z = (cplx *)Zout;
        /* Z = D Y */
        for (int j = 0; j < n; ++j)
            for (int i = 0; i < n; ++i) AT(Z, n, i, j) = c_scale(ph[i], Y[(size_t)j * n + i]);
        /* Z <- H_0 H_1 ... H_{n-2} Z */
        for (int k = n - 2; k >= 0; --k) {
            if (tau[k] == 0.0) continue;
            const int L = n - k - 1;
            const cplx *v = &AT(A, n, k + 1, k);
            #pragma omp parallel for schedule(static)
            for (int j = 0; j < n; ++j) {
                cplx *z = &AT(Z, n, k + 1, j);
                double sr = 0.0, si = 0.0;
                for (int i = 0; i < L; ++i) {
                    cplx q = c_cmul(v[i], z[i]);
                    sr += q.re; si += q.im;
                }
                cplx s = c_make(tau[k] * sr, tau[k] * si);
                for (int i = 0; i < L; ++i) z[i] = c_sub(z[i], c_mul(v[i], s));
            }
        }
        sort_eig(n, W, Z);
        free(Y);
    } else {
        sort_eig(n, W, NULL);
    }
    free(A); free(d); free(e); free(er); free(tau); free(ph);
    return rc;
}

/* Real symmetric tridiagonal eigensolver (values, optionally vectors in Y,  */
/* column-major n x n), sorted ascending.                                    */
int oracle_dstev(int n, const double *d_in, const double *e_in, double *W, double *Y)
{
    double *d = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
    memcpy(d, d_in, sizeof(double) * n);
    if (Y) {
        memset(Y, 0, sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; ++i) Y[(size_t)i * n + i] = 1.0;
    }
    int rc = oracle_tridiag_ql(n, d, (double *)e_in, Y);
    /* sort with column swaps */
    for (int i = 0; i < n - 1; ++i) {
        int k = i;
        for (int j = i + 1; j < n; ++j) if (d[j] < d[k]) k = j;
        if (k != i) {
            double t = d[i]; d[i] = d[k]; d[k] = t;
            if (Y)
                for (int r = 0; r < n; ++r) {
                    double ty = Y[(size_t)i * n + r];
                    Y[(size_t)i * n + r] = Y[(size_t)k * n + r];
                    Y[(size_t)k * n + r] = ty;
                }
        }
    }
    memcpy(W, d, sizeof(double) * n);
    free(d);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Sturm count: number of eigenvalues of the tridiagonal (d, e) below sigma. */
/* ------------------------------------------------------------------------ */
int64_t oracle_sturm_count(int64_t n, const double *d, const double *e, double sigma)
{
    int64_t cnt = 0;
    double q = 1.0;
    for (int64_t i = 0; i < n; ++i) {
#if ORACLE_MUTANT == 8
        double off = (i > 0 && i < n - 1) ? e[i] * e[i] : 0.0;
#else
        double off = (i > 0) ? e[i - 1] * e[i - 1] : 0.0;
#endif
        q = (d[i] - sigma) - (i > 0 ? off / q : 0.0);
        if (q == 0.0) q = -1e-300;  /* treat an exact zero pivot as negative */
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

/* k-th smallest eigenvalue (0-based) by bisection on Sturm counts. */
double oracle_bisect(int64_t n, const double *d, const double *e, int64_t k)
{
    double lo = 0.0, hi = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + (i < n - 1 ? fabs(e[i]) : 0.0);
        double a = d[i] - r, b = d[i] + r;
        if (i == 0 || a < lo) lo = a;
        if (i == 0 || b > hi) hi = b;
    }
    double span = hi - lo;
    lo -= 1e-14 * span + 1e-300; hi += 1e-14 * span + 1e-300;
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (oracle_sturm_count(n, d, e, mid) > k) hi = mid; else lo = mid;
    }
    return 0.5 * (lo + hi);
}
