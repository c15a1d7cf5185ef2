// FP64 eigenpair refinement (the precision extension of the hot path: the
// reduction stages run in FP32 and accuracy is recovered here).
//
// Ogita & Aishima, "Iterative refinement for symmetric eigenvalue
// decomposition" (2018), written for complex Hermitian H and refining only the
// window columns W of the full basis X (n x n):
//   R = I[:, W] - X^H X_W,   S = X^H (H X_W)      (window block Hermitian-symmetrised)
//   lam_j = s_jj / (1 - r_jj)                    (j in W; the rest keep their values)
//   delta = 2 (||S_WW - diag lam||_2 + ||H||_2 ||R||_2)
//   E_ij  = (s_ij + lam_j r_ij) / (lam_j - lam_i)  if |lam_j - lam_i| > delta,  r_ij / 2 else
//   X_W  <- X_W + X E
// All products are FP64 on the matrix cores (HEMM from the lower triangle of
// H, ZGEMMs for X^H and X E); the 2-norms are power-iteration estimates.
#include <math.h>

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

// y = (A - D) x  (rows x cols, ld; D = diag(dsub) placed at rows roff.. if dsub)
__global__ void gemv_n(int64_t rows, int64_t cols, const double *__restrict__ A, int64_t ld,
                       int64_t roff, const double *__restrict__ dsub, const double *__restrict__ x,
                       double *__restrict__ y) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows;
         i += (int64_t)gridDim.x * blockDim.x) {
        double sr = 0.0, si = 0.0;
        for (int64_t j = 0; j < cols; ++j) {
            double ar = A[2 * ((roff + i) + j * ld)], ai = A[2 * ((roff + i) + j * ld) + 1];
            if (dsub && i == j) ar -= dsub[j];
            const double xr = x[2 * j], xi = x[2 * j + 1];
            sr += ar * xr - ai * xi;
            si += ar * xi + ai * xr;
        }
        y[2 * i] = sr;
        y[2 * i + 1] = si;
    }
}

// x = (A - D)^H y  (workgroup per column)
__global__ void gemv_c(int64_t rows, int64_t cols, const double *__restrict__ A, int64_t ld,
                       int64_t roff, const double *__restrict__ dsub, const double *__restrict__ y,
                       double *__restrict__ x) {
    __shared__ double red[2][8];
    const int64_t j = blockIdx.x;
    double sr = 0.0, si = 0.0;
    for (int64_t i = threadIdx.x; i < rows; i += blockDim.x) {
        double ar = A[2 * ((roff + i) + j * ld)], ai = A[2 * ((roff + i) + j * ld) + 1];
        if (dsub && i == j) ar -= dsub[j];
        const double yr = y[2 * i], yi = y[2 * i + 1];
        sr += ar * yr + ai * yi;  // conj(a) y
        si += ar * yi - ai * yr;
    }
    sr = wave_sum(sr);
    si = wave_sum(si);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[0][w] = sr; red[1][w] = si; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) { a += red[0][q]; b += red[1][q]; }
        x[2 * j] = a;
        x[2 * j + 1] = b;
    }
}

__global__ void vec_norm2(int64_t len, const double *__restrict__ v, double *__restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < len; i += blockDim.x) s += v[2 * i] * v[2 * i] + v[2 * i + 1] * v[2 * i + 1];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s;
}

__global__ void vec_scale(int64_t len, double *__restrict__ v, const double *__restrict__ nrm2) {
    const double inv = nrm2[0] > 0.0 ? 1.0 / sqrt(nrm2[0]) : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * len;
         i += (int64_t)gridDim.x * blockDim.x)
        v[i] *= inv;
}

__global__ void vec_init(int64_t len, double *__restrict__ v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
         i += (int64_t)gridDim.x * blockDim.x) {
        // deterministic, not orthogonal to anything in particular
        v[2 * i] = 1.0 + 0.001 * (double)((i * 7919) % 101);
        v[2 * i + 1] = 0.0005 * (double)((i * 104729) % 97);
    }
}

// E (in place of S): off-window rows use lam_all, window rows use lamW
__global__ void build_E(int64_t n, int64_t m, int64_t i0, double *__restrict__ S,
                        const double *__restrict__ R, int64_t ld, const double *__restrict__ lam_all,
                        const double *__restrict__ lamW, double delta) {
    const int64_t j = blockIdx.y;
    const double lj = lamW[j];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double li = (i >= i0 && i < i0 + m) ? lamW[i - i0] : lam_all[i];
        const double sr = S[2 * (i + j * ld)], si = S[2 * (i + j * ld) + 1];
        const double rr = R[2 * (i + j * ld)], ri = R[2 * (i + j * ld) + 1];
        const double dif = lj - li;
        double er, ei;
        if (fabs(dif) > delta) {
            er = (sr + lj * rr) / dif;
            ei = (si + lj * ri) / dif;
        } else {
            er = 0.5 * rr;
            ei = 0.5 * ri;
        }
        S[2 * (i + j * ld)] = er;
        S[2 * (i + j * ld) + 1] = ei;
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
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) mx = fmax(mx, fabs(a[i] - b[i]));
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

// ||A - D||_2 estimate by power iteration on (A - D)^H (A - D)
int norm2_est(int64_t rows, int64_t cols, const double *A, int64_t ld, int64_t roff,
              const double *dsub, double *vx, double *vy, double *tmp, int iters, hipStream_t s,
              double *out) {
    hipLaunchKernelGGL(vec_init, dim3(gx(cols)), dim3(256), 0, s, cols, vx);
    hipLaunchKernelGGL(vec_norm2, dim3(1), dim3(1024), 0, s, cols, vx, tmp);
    hipLaunchKernelGGL(vec_scale, dim3(gx(cols)), dim3(256), 0, s, cols, vx, tmp);
    for (int it = 0; it < iters; ++it) {
        hipLaunchKernelGGL(gemv_n, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, s, rows, cols, A, ld,
                           roff, dsub, vx, vy);
        hipLaunchKernelGGL(gemv_c, dim3((unsigned)cols), dim3(256), 0, s, rows, cols, A, ld, roff, dsub, vy,
                           vx);
        hipLaunchKernelGGL(vec_norm2, dim3(1), dim3(1024), 0, s, cols, vx, tmp);
        hipLaunchKernelGGL(vec_scale, dim3(gx(cols)), dim3(256), 0, s, cols, vx, tmp);
    }
    BDG_CHECK_LAUNCH();
    double h = 0.0;
    BDG_HIP(hipMemcpyAsync(&h, tmp, 8, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    *out = sqrt(sqrt(h));  // ||(A-D)^H (A-D) x|| with ||x|| = 1 -> sigma^2
    return 0;
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

size_t refine_workspace(int64_t n, int64_t m) {
    const size_t big = 16 * (size_t)n * (size_t)m;
    return 2 * ((big + 255) / 256 * 256) + 16 * (size_t)(n + m) * 4 + 8 * (size_t)m * 2 + 4096;
}

// X: full FP64 basis n x n (ld ldx), lam_all[n] its approximate eigenvalues;
// window columns [i0, i0+m) are refined in place; W receives lam_W.
int refine_window(int64_t n, const double *H, int64_t ldh, double *X, int64_t ldx,
                  const double *lam_all, int64_t i0, int64_t m, double normH, int iters,
                  double *W, void *work, hipStream_t s, double *eig_shift, double *last_corr) {
    if (m <= 0) return 0;
    char *wp = (char *)work;
    auto take = [&](size_t bytes) {
        char *p = wp;
        wp += (bytes + 255) / 256 * 256;
        return (double *)p;
    };
    double *B1 = take(16 * (size_t)n * m);
    double *B2 = take(16 * (size_t)n * m);
    double *vx = take(16 * (size_t)(n + m));
    double *vy = take(16 * (size_t)(n + m));
    double *lamW = take(8 * (size_t)m);
    double *lamP = take(8 * (size_t)m);
    double *tmp = take(64);
    double *XW = X + 2 * i0 * ldx;
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
        // delta = 2 (||S_WW - diag lam||_2 + ||H||_2 ||R||_2)
        double nS = 0.0, nR = 0.0;
        BDG_TRY(norm2_est(m, m, B2, n, i0, lamW, vx, vy, tmp, 8, s, &nS));
        BDG_TRY(norm2_est(n, m, B1, n, 0, nullptr, vx, vy, tmp, 8, s, &nR));
        const double delta = 2.0 * 2.0 * (nS + normH * nR);  // x2: power iteration bounds from below
        hipLaunchKernelGGL(build_E, dim3(gx(n), (unsigned)m), dim3(256), 0, s, n, m, i0, B2, B1, n, lam_all,
                           lamW, delta);
        BDG_CHECK_LAUNCH();
        // B1 = X_W ; B1 += X E ; X_W = B1
        hipLaunchKernelGGL(copy_c128, dim3(gx(n), (unsigned)m), dim3(256), 0, s, n, XW, ldx, B1, n);
        BDG_CHECK_LAUNCH();
        GemmArgs g4{n, m, n, 1.0, 0.0, 1.0, 0.0, X, ldx, B2, n, B1, n, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<double, true>('N', 'N', g4, s)));
        hipLaunchKernelGGL(copy_c128, dim3(gx(n), (unsigned)m), dim3(256), 0, s, n, B1, n, XW, ldx);
        BDG_CHECK_LAUNCH();
        hipLaunchKernelGGL(max_abs_diff, dim3(1), dim3(1024), 0, s, m, lamW, lamP, tmp);
        BDG_CHECK_LAUNCH();
        double h = 0.0;
        BDG_HIP(hipMemcpyAsync(&h, tmp, 8, hipMemcpyDeviceToHost, s));
        BDG_HIP(hipMemcpyAsync(lamP, lamW, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
        BDG_HIP(hipStreamSynchronize(s));
        if (it == 0) shift = h;
        if (last_corr) *last_corr = h;
    }
    BDG_HIP(hipMemcpyAsync(W, lamW, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    if (eig_shift) *eig_shift = shift;
    return 0;
}

}  // namespace bdg
