// FP64 eigenpair refinement (the precision extension of the hot path: the
// reduction stages run in FP32 and accuracy is recovered here).
//
// Ogita & Aishima, "Iterative refinement for symmetric eigenvalue
// decomposition" (2018), written for complex Hermitian H and refining only the
// window columns W of the full basis X (n x n):
//   R = I[:, W] - X^H X_W,   S = X^H (H X_W)      (window block Hermitian-symmetrised)
//   lam_j = s_jj / (1 - r_jj)                    (j in W; the rest keep their values)
//   E_ij  = (s_ij + lam_j r_ij) / (lam_j - lam_i)  for well-separated pairs,  r_ij / 2 else
//   X_W  <- X_W + X E
// All products are FP64 on the matrix cores (HEMM from the lower triangle of
// H, ZGEMMs for X^H and X E).
//
// Close pairs and clusters.  The published test |lam_i - lam_j| <= delta uses
// one global delta = 2 (||S - diag|| + ||H|| ||R||), which from an FP32 basis
// of order 10^4 exceeds the mean level spacing; a pair is taken as close here
// when its first-order coefficient would not be small,
// |s_ij + lam_j r_ij| >= TAU |lam_j - lam_i|.  The r_ij / 2 branch never
// resolves mixing inside a group of close eigenvalues, so the connected
// components of close window pairs (at most CMAX members; larger ones are cut,
// and close pairs across a cut keep r_ij / 2) get an FP64 Rayleigh-Ritz step
// (part II of the method, clustered eigenvalues, 2019):
//   L = I + R_JJ / 2,  M = L S_JJ L = Q diag(mu) Q^H  (complex Jacobi in LDS)
//   E[:, J] <- (I_W + E)[:, J] Q - I_W[:, J],  lam_J <- mu
#include <math.h>

#include <algorithm>
#include <cstdio>
#include <numeric>
#include <vector>

#include "gemm.h"
#include "refine.h"

namespace bdg {
namespace {

__global__ void cast_c64_c128(int64_t rows, int64_t cols, const float *__restrict__ src, int64_t lds,
                              double *__restrict__ dst, int64_t ldd) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float2 v = *(const float2 *)(src + 2 * (i + j * lds));
        *(double2 *)(dst + 2 * (i + j * ldd)) = make_double2(v.x, v.y);
    }
}

__global__ void cast_c128_c64(int64_t rows, int64_t cols, const double *__restrict__ src,
                              int64_t lds, float *__restrict__ dst, int64_t ldd) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = *(const double2 *)(src + 2 * (i + j * lds));
        *(float2 *)(dst + 2 * (i + j * ldd)) = make_float2((float)v.x, (float)v.y);
    }
}

// column (half - 1 - j) = (-conj(v), conj(u)) of column (half + j), [u; v] split at n/2
template <typename T>
__global__ void mirror_cols(int64_t n, int64_t half, T *__restrict__ X, int64_t ld) {
    const int64_t j = blockIdx.y;
    const int64_t ns = n / 2;
    const T *src = X + 2 * (half + j) * ld;
    T *dst = X + 2 * (half - 1 - j) * ld;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * blockDim.x) {
        const T ur = src[2 * r], ui = src[2 * r + 1];
        const T vr = src[2 * (ns + r)], vi = src[2 * (ns + r) + 1];
        dst[2 * r] = -vr;
        dst[2 * r + 1] = vi;
        dst[2 * (ns + r)] = ur;
        dst[2 * (ns + r) + 1] = -ui;
    }
}

// column dst0 + k <- (-conj(v), conj(u)) of column src0 - k, k < count
template <typename T>
__global__ void mirror_map(int64_t n, T *__restrict__ X, int64_t ld, int64_t dst0, int64_t src0) {
    const int64_t k = blockIdx.y;
    const int64_t ns = n / 2;
    const T *src = X + 2 * (src0 - k) * ld;
    T *dst = X + 2 * (dst0 + k) * ld;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * blockDim.x) {
        const T ur = src[2 * r], ui = src[2 * r + 1];
        const T vr = src[2 * (ns + r)], vi = src[2 * (ns + r) + 1];
        dst[2 * r] = -vr;
        dst[2 * r + 1] = vi;
        dst[2 * (ns + r)] = ur;
        dst[2 * (ns + r) + 1] = -ui;
    }
}

// R[i0 + j, j] += 1 ;  window block of R and S made Hermitian; lam_j = s_jj/(1 - r_jj)
__global__ void window_block(int64_t m, int64_t i0, double *__restrict__ R, double *__restrict__ S,
                             int64_t ld, double *__restrict__ lamW) {
    const int64_t j = blockIdx.x;  // column of the block
    for (int64_t i = threadIdx.x; i <= j; i += blockDim.x) {
        // pair (i, j) and (j, i) of the m x m block at rows i0..
        double *rij = R + 2 * ((i0 + i) + j * ld), *rji = R + 2 * ((i0 + j) + i * ld);
        double *sij = S + 2 * ((i0 + i) + j * ld), *sji = S + 2 * ((i0 + j) + i * ld);
        if (i == j) {
            const double r = 1.0 + rij[0];  // identity added here
            rij[0] = r;
            rij[1] = 0.0;
            sij[1] = 0.0;
            lamW[j] = sij[0] / (1.0 - r);
        } else {
            const double ar = 0.5 * (rij[0] + rji[0]), ai = 0.5 * (rij[1] - rji[1]);
            rij[0] = ar; rij[1] = ai; rji[0] = ar; rji[1] = -ai;
            const double br = 0.5 * (sij[0] + sji[0]), bi = 0.5 * (sij[1] - sji[1]);
            sij[0] = br; sij[1] = bi; sji[0] = br; sji[1] = -bi;
        }
    }
}

constexpr double TAU = 1e-3;

// Close pairs (a, b), a > b, of the window (both orientations tested), appended
// to pairs[] (capacity cap; count keeps counting past it).
__global__ void close_pairs(int64_t m, int64_t i0, const double *__restrict__ S, const double *__restrict__ R,
                            int64_t ld, const double *__restrict__ lamW, int2 *__restrict__ pairs, int cap,
                            int *__restrict__ count) {
    const int64_t b = blockIdx.y;
    const double lb = lamW[b];
    for (int64_t a = b + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < m;
         a += (int64_t)gridDim.x * blockDim.x) {
        const double la = lamW[a];
        const int64_t ab = 2 * ((i0 + a) + b * ld), ba = 2 * ((i0 + b) + a * ld);
        // row a, column b: s_ab + lam_b r_ab against lam_b - lam_a; and the transpose
        const double n1 = hypot(S[ab] + lb * R[ab], S[ab + 1] + lb * R[ab + 1]);
        const double n2 = hypot(S[ba] + la * R[ba], S[ba + 1] + la * R[ba + 1]);
        const double gap = fabs(lb - la);
        if (n1 >= TAU * gap || n2 >= TAU * gap) {
            const int k = atomicAdd(count, 1);
            if (k < cap) pairs[k] = make_int2((int)a, (int)b);
        }
    }
}

// E (in place of S): off-window rows use lam_all, window rows use lamW.
// r_ij / 2 on the diagonal, for close pairs, and inside a cluster (cid: cluster
// of each window column, -1 none; null when there are none); the first-order
// quotient elsewhere.
// emax: per block, max over (i, j) off the window diagonal of
// max(|r_ij|, |s_ij + lam_j r_ij| / normH), the step's defect in residual units
// (|E_ij| itself is large for well-separated but very close pairs whose
// mixing no longer matters); rows outside the window are columns of the
// unrefined basis, whose overlap with a converged column stays at the level of
// their own error, so there only the residual part counts
__global__ void build_E(int64_t n, int64_t m, int64_t i0, double *__restrict__ S,
                        const double *__restrict__ R, int64_t ld, const double *__restrict__ lam_all,
                        const double *__restrict__ lamW, const int *__restrict__ cid, double inv_normH,
                        double *__restrict__ emax) {
    __shared__ double red[4];
    const int64_t j = blockIdx.y;
    const double lj = lamW[j];
    const int cj = cid ? cid[j] : -1;
    double mx = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const bool inw = i >= i0 && i < i0 + m;
        const double li = inw ? lamW[i - i0] : lam_all[i];
        const double sr = S[2 * (i + j * ld)], si = S[2 * (i + j * ld) + 1];
        const double rr = R[2 * (i + j * ld)], ri = R[2 * (i + j * ld) + 1];
        const double dif = lj - li;
        const double nr = sr + lj * rr, ni = si + lj * ri;
        const bool diag = i == i0 + j;
        const bool same = inw && cj >= 0 && cid[i - i0] == cj;
        double er, ei;
        if (diag || same || hypot(nr, ni) >= TAU * fabs(dif)) {
            er = 0.5 * rr;
            ei = 0.5 * ri;
        } else {
            er = nr / dif;
            ei = ni / dif;
        }
        S[2 * (i + j * ld)] = er;
        S[2 * (i + j * ld) + 1] = ei;
        if (!diag) {
            const double dn = (fabs(nr) + fabs(ni)) * inv_normH;
            mx = fmax(mx, inw ? fmax(fabs(rr) + fabs(ri), dn) : dn);
        }
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        emax[blockIdx.y * gridDim.x + blockIdx.x] = v;
    }
}

constexpr int CMAX = 48;
constexpr int CLD = CMAX + 1;  // LDS row pitch (complex entries)

// c x c complex products in LDS: C = A B (all CLD-pitched, row-major [row][col])
__device__ void lds_cmatmul(int c, const double2 *A, const double2 *B, double2 *C) {
    for (int e = threadIdx.x; e < c * c; e += blockDim.x) {
        const int r = e / c, q = e % c;
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < c; ++k) {
            const double2 a = A[r * CLD + k], b = B[k * CLD + q];
            sr += a.x * b.x - a.y * b.y;
            si += a.x * b.y + a.y * b.x;
        }
        C[r * CLD + q] = make_double2(sr, si);
    }
}

// One block per cluster: M = L S_JJ L (L = I + R_JJ / 2), Hermitian Jacobi
// M = Q diag(mu) Q^H, mu ascending.  cidx lists each cluster's window columns in
// ascending order of their current eigenvalue; Q goes to qbuf (column-major
// c x c at qoff[b]), mu to mu[cidx], max_{k != l} |M_kl| / normH to cmax[b].
__global__ void __launch_bounds__(256) cluster_eig(int64_t i0, const int *__restrict__ cidx,
                                                   const int *__restrict__ coff,
                                                   const int64_t *__restrict__ qoff,
                                                   const double *__restrict__ S,
                                                   const double *__restrict__ R, int64_t ld,
                                                   double normH, double *__restrict__ qbuf,
                                                   double *__restrict__ mu, double *__restrict__ cmax) {
    __shared__ double2 A0[CMAX * CLD], A1[CMAX * CLD], A2[CMAX * CLD];
    __shared__ double rot[4];
    __shared__ int flag, perm[CMAX];
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int *J = cidx + coff[b];
    const int c = coff[b + 1] - coff[b];
    // A0 = S_JJ, A1 = L
    for (int e = threadIdx.x; e < c * c; e += blockDim.x) {
        const int r = e / c, q = e % c;
        const int64_t off = 2 * ((i0 + J[r]) + (int64_t)J[q] * ld);
        A0[r * CLD + q] = make_double2(S[off], S[off + 1]);
        A1[r * CLD + q] = make_double2((r == q ? 1.0 : 0.0) + 0.5 * R[off], 0.5 * R[off + 1]);
    }
    __syncthreads();
    lds_cmatmul(c, A0, A1, A2);  // T = S L
    __syncthreads();
    lds_cmatmul(c, A1, A2, A0);  // M = L T
    __syncthreads();
    // Hermitian part; Q = I in A1
    double mx = 0.0;
    for (int e = threadIdx.x; e < c * c; e += blockDim.x) {
        const int r = e / c, q = e % c;
        if (r < q) {
            const double2 u = A0[r * CLD + q], v = A0[q * CLD + r];
            const double2 h = make_double2(0.5 * (u.x + v.x), 0.5 * (u.y - v.y));
            A0[r * CLD + q] = h;
            A0[q * CLD + r] = make_double2(h.x, -h.y);
            mx = fmax(mx, sqrt(h.x * h.x + h.y * h.y));
        } else if (r == q) {
            A0[r * CLD + r].y = 0.0;
        }
        A1[r * CLD + q] = make_double2(r == q ? 1.0 : 0.0, 0.0);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) cmax[b] = fmax(fmax(red[0], red[1]), fmax(red[2], red[3])) / normH;
    // cyclic Jacobi with complex rotations G = [[cs, sn e], [-sn conj(e), cs]] on (p, q)
    for (int sweep = 0; sweep < 30; ++sweep) {
        if (threadIdx.x == 0) flag = 0;
        __syncthreads();
        for (int p = 0; p < c - 1; ++p) {
            for (int q = p + 1; q < c; ++q) {
                if (threadIdx.x == 0) {
                    const double2 bpq = A0[p * CLD + q];
                    const double ab = sqrt(bpq.x * bpq.x + bpq.y * bpq.y);
                    const double a = A0[p * CLD + p].x, d = A0[q * CLD + q].x;
                    if (ab == 0.0 || ab < 1e-17 * (fabs(a) + fabs(d))) {
                        rot[0] = 1.0;
                        rot[1] = 0.0;
                    } else {
                        const double z = (d - a) / (2.0 * ab);
                        const double t = fabs(z) < 1e150 ? (z >= 0.0 ? 1.0 : -1.0) / (fabs(z) + sqrt(1.0 + z * z))
                                                         : 0.5 / z;
                        const double cs = 1.0 / sqrt(1.0 + t * t);
                        rot[0] = cs;
                        rot[1] = t * cs;
                        rot[2] = bpq.x / ab;
                        rot[3] = bpq.y / ab;
                        flag = 1;
                    }
                }
                __syncthreads();
                const double cs = rot[0], sn = rot[1];
                if (sn != 0.0) {
                    const double er = rot[2], ei = rot[3];
                    const int k = threadIdx.x;
                    if (k < c) {
                        // columns p, q of M and Q: [x_p, x_q] G
                        double2 *cols[2] = {A0, A1};
                        for (int w = 0; w < 2; ++w) {
                            double2 *X = cols[w];
                            const double2 xp = X[k * CLD + p], xq = X[k * CLD + q];
                            // xp' = cs xp - sn conj(e) xq ; xq' = sn e xp + cs xq
                            X[k * CLD + p] = make_double2(cs * xp.x - sn * (er * xq.x + ei * xq.y),
                                                          cs * xp.y - sn * (er * xq.y - ei * xq.x));
                            X[k * CLD + q] = make_double2(sn * (er * xp.x - ei * xp.y) + cs * xq.x,
                                                          sn * (er * xp.y + ei * xp.x) + cs * xq.y);
                        }
                    }
                    __syncthreads();
                    if (k < c) {
                        // rows p, q of M: G^H [y_p; y_q]
                        const double2 yp = A0[p * CLD + k], yq = A0[q * CLD + k];
                        // yp' = cs yp - sn e yq ; yq' = sn conj(e) yp + cs yq
                        A0[p * CLD + k] = make_double2(cs * yp.x - sn * (er * yq.x - ei * yq.y),
                                                       cs * yp.y - sn * (er * yq.y + ei * yq.x));
                        A0[q * CLD + k] = make_double2(sn * (er * yp.x + ei * yp.y) + cs * yq.x,
                                                       sn * (er * yp.y - ei * yp.x) + cs * yq.y);
                    }
                    __syncthreads();
                    if (threadIdx.x == 0) {
                        A0[p * CLD + q] = make_double2(0.0, 0.0);
                        A0[q * CLD + p] = make_double2(0.0, 0.0);
                        A0[p * CLD + p].y = 0.0;
                        A0[q * CLD + q].y = 0.0;
                    }
                }
                __syncthreads();
            }
        }
        if (flag == 0) break;
        __syncthreads();
    }
    // ascending order of the eigenvalues
    if (threadIdx.x == 0) {
        for (int k = 0; k < c; ++k) perm[k] = k;
        for (int k = 0; k < c; ++k) {
            int best = k;
            for (int l = k + 1; l < c; ++l)
                if (A0[perm[l] * CLD + perm[l]].x < A0[perm[best] * CLD + perm[best]].x) best = l;
            const int t = perm[k];
            perm[k] = perm[best];
            perm[best] = t;
        }
    }
    __syncthreads();
    double *Qo = qbuf + 2 * qoff[b];
    for (int e = threadIdx.x; e < c * c; e += blockDim.x) {
        const int r = e % c, l = e / c;  // column-major output
        const double2 v = A1[r * CLD + perm[l]];
        Qo[2 * e] = v.x;
        Qo[2 * e + 1] = v.y;
    }
    for (int l = threadIdx.x; l < c; l += blockDim.x) mu[J[l]] = A0[perm[l] * CLD + perm[l]].x;
}

// E[:, J] <- (I_W + E)[:, J] Q - I_W[:, J] for rows of a 64-row tile; lam_J <- mu
__global__ void __launch_bounds__(64) cluster_apply(int64_t n, int64_t i0, const int *__restrict__ cidx,
                                                    const int *__restrict__ coff,
                                                    const int64_t *__restrict__ qoff,
                                                    const double *__restrict__ qbuf, double *__restrict__ E,
                                                    int64_t ld, const double *__restrict__ mu,
                                                    double *__restrict__ lamW) {
    __shared__ double2 Qs[CMAX * CMAX];
    __shared__ double2 e[64 * CLD];
    __shared__ int Js[CMAX];
    const int b = blockIdx.y;
    const int *J = cidx + coff[b];
    const int c = coff[b + 1] - coff[b];
    const double *Q = qbuf + 2 * qoff[b];
    for (int t = threadIdx.x; t < c * c; t += 64) Qs[t] = make_double2(Q[2 * t], Q[2 * t + 1]);
    for (int t = threadIdx.x; t < c; t += 64) Js[t] = J[t];
    __syncthreads();
    if (blockIdx.x == 0)
        for (int t = threadIdx.x; t < c; t += 64) lamW[Js[t]] = mu[Js[t]];
    const int64_t i = (int64_t)blockIdx.x * 64 + threadIdx.x;
    if (i >= n) return;
    const int64_t wrow = i - i0;  // this row's window column, if any
    double2 *er = e + threadIdx.x * CLD;
    for (int k = 0; k < c; ++k) {
        const int64_t off = 2 * (i + (int64_t)Js[k] * ld);
        er[k] = make_double2(E[off] + (wrow == Js[k] ? 1.0 : 0.0), E[off + 1]);
    }
    for (int l = 0; l < c; ++l) {
        double sr = 0.0, si = 0.0;
        for (int k = 0; k < c; ++k) {
            const double2 a = er[k], q = Qs[k + l * c];
            sr += a.x * q.x - a.y * q.y;
            si += a.x * q.y + a.y * q.x;
        }
        const int64_t off = 2 * (i + (int64_t)Js[l] * ld);
        E[off] = sr - (wrow == Js[l] ? 1.0 : 0.0);
        E[off + 1] = si;
    }
}

__global__ void copy_c128(int64_t rows, const double *__restrict__ src, int64_t lds,
                          double *__restrict__ dst, int64_t ldd) {
    const int64_t j = blockIdx.y;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x)
        *(double2 *)(dst + 2 * (i + j * ldd)) = *(const double2 *)(src + 2 * (i + j * lds));
}

__global__ void max_abs_diff(int64_t m, const double *__restrict__ a, const double *__restrict__ b,
                             double *__restrict__ out) {
    __shared__ double red[16];
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) mx = fmax(mx, fabs(a[i] - (b ? b[i] : 0.0)));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) v = fmax(v, red[q]);
        out[0] = v;
    }
}

unsigned gx(int64_t rows) {
    int64_t g = (rows + 255) / 256;
    return (unsigned)(g > 64 ? 64 : (g < 1 ? 1 : g));
}

}  // namespace

int cast_c64_to_c128(int64_t rows, int64_t cols, const float *src, int64_t lds, double *dst,
                     int64_t ldd, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    hipLaunchKernelGGL(cast_c64_c128, dim3(gx(rows), (unsigned)cols), dim3(256), 0, s, rows, cols, src,
                       lds, dst, ldd);
    BDG_CHECK_LAUNCH();
    return 0;
}

int cast_c128_to_c64(int64_t rows, int64_t cols, const double *src, int64_t lds, float *dst,
                     int64_t ldd, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return 0;
    hipLaunchKernelGGL(cast_c128_c64, dim3(gx(rows), (unsigned)cols), dim3(256), 0, s, rows, cols, src,
                       lds, dst, ldd);
    BDG_CHECK_LAUNCH();
    return 0;
}

int mirror_half(int64_t n, double *X, int64_t ld, hipStream_t s) {
    const int64_t half = n / 2;
    if (half <= 0) return 0;
    hipLaunchKernelGGL((mirror_cols<double>), dim3(gx(half), (unsigned)half), dim3(256), 0, s, n, half, X,
                       ld);
    BDG_CHECK_LAUNCH();
    return 0;
}

int mirror_half(int64_t n, float *X, int64_t ld, hipStream_t s) {
    const int64_t half = n / 2;
    if (half <= 0) return 0;
    hipLaunchKernelGGL((mirror_cols<float>), dim3(gx(half), (unsigned)half), dim3(256), 0, s, n, half, X,
                       ld);
    BDG_CHECK_LAUNCH();
    return 0;
}

int mirror_columns(int64_t n, double *X, int64_t ld, int64_t dst0, int64_t src0, int64_t count,
                   hipStream_t s) {
    if (count <= 0) return 0;
    hipLaunchKernelGGL((mirror_map<double>), dim3(gx(n / 2), (unsigned)count), dim3(256), 0, s, n, X, ld,
                       dst0, src0);
    BDG_CHECK_LAUNCH();
    return 0;
}

namespace {

// Workspace of refine_window, carved in this order.
struct RefineLayout {
    size_t B1, B2, lamW, lamP, tmp, emax, qbuf, mu, cidx, coff, qoff, cmax, cid, pairs, count, total;
    RefineLayout(int64_t n, int64_t m) {
        size_t o = 0;
        auto take = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
        B1 = take(16 * (size_t)n * m);
        B2 = take(16 * (size_t)n * m);
        lamW = take(8 * (size_t)m);
        lamP = take(8 * (size_t)m);
        tmp = take(64);
        emax = take(8 * (size_t)m * 64 + 64);
        qbuf = take(16 * (size_t)CMAX * m);
        mu = take(8 * (size_t)m);
        cidx = take(4 * (size_t)m);
        coff = take(4 * (size_t)(m + 2));
        qoff = take(8 * (size_t)(m + 2));
        cmax = take(8 * (size_t)(m + 2));
        cid = take(4 * (size_t)m);
        pairs = take(8 * (size_t)cap(m));
        count = take(64);
        total = o;
    }
    static int cap(int64_t m) { return (int)(4 * m + 4096); }
};

// Connected components (>= 2 members) of the close pairs, members in ascending
// order of lam, components cut into pieces of at most CMAX.  Fills the flat
// member list, offsets, Q offsets and the cluster id of every column (-1 none);
// returns the number of clusters.
int find_clusters(const std::vector<double> &lam, const std::vector<int2> &pairs, std::vector<int> &idx,
                  std::vector<int> &off, std::vector<int64_t> &qo, std::vector<int> &cid) {
    const int m = (int)lam.size();
    std::vector<int> parent((size_t)m);
    std::iota(parent.begin(), parent.end(), 0);
    auto root = [&](int a) {
        while (parent[a] != a) {
            parent[a] = parent[parent[a]];
            a = parent[a];
        }
        return a;
    };
    for (const int2 &p : pairs) {
        const int ra = root(p.x), rb = root(p.y);
        if (ra != rb) parent[ra] = rb;
    }
    std::vector<int> order((size_t)m);
    std::iota(order.begin(), order.end(), 0);
    // group by root, ascending lam inside a group, groups by their lowest lam
    std::vector<int> r((size_t)m);
    for (int a = 0; a < m; ++a) r[a] = root(a);
    std::vector<double> glo((size_t)m, 0.0);
    std::vector<int> gsize((size_t)m, 0);
    for (int a = 0; a < m; ++a) {
        if (gsize[r[a]] == 0 || lam[a] < glo[r[a]]) glo[r[a]] = lam[a];
        ++gsize[r[a]];
    }
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        if (r[a] != r[b]) return glo[r[a]] < glo[r[b]] || (glo[r[a]] == glo[r[b]] && r[a] < r[b]);
        return lam[a] < lam[b];
    });
    idx.clear();
    off.assign(1, 0);
    qo.assign(1, 0);
    cid.assign((size_t)m, -1);
    for (int k = 0; k < m;) {
        int e = k;
        while (e < m && r[order[e]] == r[order[k]]) ++e;
        for (int a = k; e - a >= 2; a += CMAX) {
            const int c = std::min(CMAX, e - a);
            if (c < 2) break;
            const int id = (int)off.size() - 1;
            for (int t = 0; t < c; ++t) {
                idx.push_back(order[a + t]);
                cid[order[a + t]] = id;
            }
            off.push_back((int)idx.size());
            qo.push_back(qo.back() + (int64_t)c * c);
        }
        k = e;
    }
    return (int)off.size() - 1;
}

}  // namespace

size_t refine_workspace(int64_t n, int64_t m) { return RefineLayout(n, m).total + 256; }

// X: full FP64 basis n x n (ld ldx), lam_all[n] its approximate eigenvalues;
// window columns [i0, i0+m) are refined in place; W receives lam_W.
int refine_window(int64_t n, const double *H, int64_t ldh, double *X, int64_t ldx,
                  const double *lam_all, int64_t i0, int64_t m, double normH, int iters, double tol,
                  double *W, void *work, hipStream_t s, double *eig_shift, double *last_corr,
                  int *iters_done, int *close0, int *ccols0) {
    if (m <= 0) return 0;
    const RefineLayout L(n, m);
    char *base = (char *)work;
    double *B1 = (double *)(base + L.B1);
    double *B2 = (double *)(base + L.B2);
    double *lamW = (double *)(base + L.lamW);
    double *lamP = (double *)(base + L.lamP);
    double *tmp = (double *)(base + L.tmp);
    double *emax = (double *)(base + L.emax);
    double *qbuf = (double *)(base + L.qbuf);
    double *mu = (double *)(base + L.mu);
    int *cidx = (int *)(base + L.cidx);
    int *coff = (int *)(base + L.coff);
    int64_t *qoff = (int64_t *)(base + L.qoff);
    double *cmax = (double *)(base + L.cmax);
    int *cid = (int *)(base + L.cid);
    int2 *pairs = (int2 *)(base + L.pairs);
    int *count = (int *)(base + L.count);
    const int cap = RefineLayout::cap(m);
    std::vector<double> lam_h((size_t)m);
    std::vector<int2> pairs_h;
    std::vector<int> idx_h, off_h, cid_h;
    std::vector<int64_t> qo_h;
    double *XW = X + 2 * i0 * ldx;
    const double hn = normH > 0.0 ? normH : 1.0;
    BDG_HIP(hipMemcpyAsync(lamP, lam_all + i0, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    double shift = 0.0;
    for (int it = 0; it < iters; ++it) {
        // B1 = H X_W (Hermitian H from its lower triangle)
        GemmArgs g1{n, m, n, 1.0, 0.0, 0.0, 0.0, H, ldh, XW, ldx, B1, n, GEMM_HEMM_L, 1, nullptr};
        BDG_TRY((gemm<double, true>('N', 'N', g1, s)));
        // B2 = S = X^H B1
        GemmArgs g2{n, m, n, 1.0, 0.0, 0.0, 0.0, X, ldx, B1, n, B2, n, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<double, true>('C', 'N', g2, s)));
        // B1 = -X^H X_W   (identity added on the window block)
        GemmArgs g3{n, m, n, -1.0, 0.0, 0.0, 0.0, X, ldx, XW, ldx, B1, n, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<double, true>('C', 'N', g3, s)));
        hipLaunchKernelGGL(window_block, dim3((unsigned)m), dim3(256), 0, s, m, i0, B1, B2, n, lamW);
        BDG_CHECK_LAUNCH();
        // close pairs of the window -> clusters
        BDG_HIP(hipMemsetAsync(count, 0, 4, s));
        if (m >= 2) {
            hipLaunchKernelGGL(close_pairs, dim3(gx(m), (unsigned)(m - 1)), dim3(256), 0, s, m, i0, B2, B1, n,
                               lamW, pairs, cap, count);
            BDG_CHECK_LAUNCH();
        }
        int npairs = 0;
        BDG_HIP(hipMemcpyAsync(&npairs, count, 4, hipMemcpyDeviceToHost, s));
        BDG_HIP(hipMemcpyAsync(lam_h.data(), lamW, 8 * (size_t)m, hipMemcpyDeviceToHost, s));
        BDG_HIP(hipStreamSynchronize(s));
        pairs_h.resize((size_t)std::min(npairs, cap));
        if (!pairs_h.empty()) {
            BDG_HIP(hipMemcpyAsync(pairs_h.data(), pairs, 8 * pairs_h.size(), hipMemcpyDeviceToHost, s));
            BDG_HIP(hipStreamSynchronize(s));
        }
        const int ncl = find_clusters(lam_h, pairs_h, idx_h, off_h, qo_h, cid_h);
        if (ncl > 0) {
            BDG_HIP(hipMemcpyAsync(cidx, idx_h.data(), 4 * idx_h.size(), hipMemcpyHostToDevice, s));
            BDG_HIP(hipMemcpyAsync(coff, off_h.data(), 4 * off_h.size(), hipMemcpyHostToDevice, s));
            BDG_HIP(hipMemcpyAsync(qoff, qo_h.data(), 8 * qo_h.size(), hipMemcpyHostToDevice, s));
            BDG_HIP(hipMemcpyAsync(cid, cid_h.data(), 4 * cid_h.size(), hipMemcpyHostToDevice, s));
            // reads S and R before build_E turns S into E
            hipLaunchKernelGGL(cluster_eig, dim3((unsigned)ncl), dim3(256), 0, s, i0, cidx, coff, qoff, B2, B1,
                               n, hn, qbuf, mu, cmax);
            BDG_CHECK_LAUNCH();
        }
        hipLaunchKernelGGL(build_E, dim3(gx(n), (unsigned)m), dim3(256), 0, s, n, m, i0, B2, B1, n, lam_all,
                           lamW, ncl > 0 ? (const int *)cid : (const int *)nullptr, 1.0 / hn, emax);
        BDG_CHECK_LAUNCH();
        hipLaunchKernelGGL(max_abs_diff, dim3(1), dim3(1024), 0, s, (int64_t)gx(n) * m, emax,
                           (const double *)nullptr, tmp + 1);
        BDG_CHECK_LAUNCH();
        if (ncl > 0) {
            hipLaunchKernelGGL(cluster_apply, dim3((unsigned)((n + 63) / 64), (unsigned)ncl), dim3(64), 0, s, n,
                               i0, cidx, coff, qoff, qbuf, B2, n, mu, lamW);
            BDG_CHECK_LAUNCH();
            hipLaunchKernelGGL(max_abs_diff, dim3(1), dim3(1024), 0, s, (int64_t)ncl, cmax,
                               (const double *)nullptr, tmp + 2);
            BDG_CHECK_LAUNCH();
        } else {
            BDG_HIP(hipMemsetAsync(tmp + 2, 0, 8, s));
        }
        if (it == 0) {
            if (close0) *close0 = npairs;
            if (ccols0) *ccols0 = (int)idx_h.size();
        }
        // B1 = X_W ; B1 += X E ; X_W = B1
        hipLaunchKernelGGL(copy_c128, dim3(gx(n), (unsigned)m), dim3(256), 0, s, n, XW, ldx, B1, n);
        BDG_CHECK_LAUNCH();
        GemmArgs g4{n, m, n, 1.0, 0.0, 1.0, 0.0, X, ldx, B2, n, B1, n, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<double, true>('N', 'N', g4, s)));
        hipLaunchKernelGGL(copy_c128, dim3(gx(n), (unsigned)m), dim3(256), 0, s, n, B1, n, XW, ldx);
        BDG_CHECK_LAUNCH();
        hipLaunchKernelGGL(max_abs_diff, dim3(1), dim3(1024), 0, s, m, lamW, lamP, tmp);
        BDG_CHECK_LAUNCH();
        double h[3] = {0.0, 0.0, 0.0};
        BDG_HIP(hipMemcpyAsync(h, tmp, 24, hipMemcpyDeviceToHost, s));
        BDG_HIP(hipMemcpyAsync(lamP, lamW, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
        BDG_HIP(hipStreamSynchronize(s));
        if (it == 0) shift = h[0];
        const double corr = std::max(h[1], h[2]);
        if (last_corr) *last_corr = corr;
        if (iters_done) *iters_done = it + 1;
        if (verbose()) {
            fprintf(stderr, "[bdg] refinement step %d: defect %.3e, %d close pairs, %d clustered columns\n",
                    it + 1, corr, npairs, (int)idx_h.size());
            fflush(stderr);
        }
        // the defect shrinks quadratically; stop once it (and the in-cluster
        // coupling) is at rounding level
        if (corr < tol) break;
    }
    BDG_HIP(hipMemcpyAsync(W, lamW, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    if (eig_shift) *eig_shift = shift;
    return 0;
}

}  // namespace bdg
