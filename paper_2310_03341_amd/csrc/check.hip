// FP64 accuracy check of eigenpairs: residual norms ||H z_j - w_j z_j|| and the
// Gram defect max |Z^H Z - I|, both computed with the MFMA GEMM in FP64.
#include "gemm.h"
#include "solver.h"

namespace bdg {
namespace {

// R = HZ (n x m, ld n) -> out[j] = ||R[:, j] - w_j Z[:, j]||_2
__global__ void resid_cols(int64_t n, int64_t m, const double *__restrict__ R,
                           const double *__restrict__ W, const double *__restrict__ Z, int64_t ldz,
                           double *__restrict__ out) {
    __shared__ double red[16];
    const int64_t j = blockIdx.x;
    if (j >= m) return;
    const double w = W[j];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double rr = R[2 * (i + j * n)] - w * Z[2 * (i + j * ldz)];
        const double ri = R[2 * (i + j * n) + 1] - w * Z[2 * (i + j * ldz) + 1];
        s += rr * rr + ri * ri;
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[j] = sqrt(s);
}

// G = Z^H Z (m x m) -> per-column max |G - I|
__global__ void gram_cols(int64_t m, const double *__restrict__ G, double *__restrict__ out) {
    __shared__ double red[16];
    const int64_t j = blockIdx.x;
    if (j >= m) return;
    double mx = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
        const double re = G[2 * (i + j * m)] - (i == j ? 1.0 : 0.0);
        const double im = G[2 * (i + j * m) + 1];
        mx = fmax(mx, sqrt(re * re + im * im));
    }
    // block max via shuffles
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) red[w] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double r = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r = fmax(r, red[i]);
        out[j] = r;
    }
}

__global__ void max_reduce(int64_t m, const double *__restrict__ v, const double *__restrict__ W,
                           double *__restrict__ out) {
    __shared__ double red[32];
    double mx = 0.0, wm = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
        mx = fmax(mx, v[i]);
        if (W) wm = fmax(wm, fabs(W[i]));
    }
    for (int o = 32; o > 0; o >>= 1) {
        mx = fmax(mx, __shfl_xor(mx, o, 64));
        wm = fmax(wm, __shfl_xor(wm, o, 64));
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) { red[w] = mx; red[16 + w] = wm; }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, b = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) { a = fmax(a, red[i]); b = fmax(b, red[16 + i]); }
        out[0] = a;
        out[1] = b;
    }
}

}  // namespace

int check_pairs(int64_t n, const double *H, int64_t ldh, int64_t m, const double *W,
                const double *Z, int64_t ldz, double *max_resid, double *gram_defect, void *work,
                hipStream_t s) {
    if (m == 0) {
        *max_resid = 0.0;
        *gram_defect = 0.0;
        return 0;
    }
    // work layout: R (n x m complex) | G (m x m complex) | 8 doubles of results
    double *R = (double *)work;
    double *G = R + 2 * n * m;
    double *res = G + 2 * m * m;
    GemmArgs g1{n, m, n, 1.0, 0.0, 0.0, 0.0, H, ldh, Z, ldz, R, n, GEMM_FULL, 1, nullptr};
    BDG_TRY((gemm<double, true>('N', 'N', g1, s)));
    double *rn = G;  // m residual norms (G not formed yet)
    hipLaunchKernelGGL(resid_cols, dim3((unsigned)m), dim3(256), 0, s, n, m, R, W, Z, ldz, rn);
    BDG_CHECK_LAUNCH();
    hipLaunchKernelGGL(max_reduce, dim3(1), dim3(1024), 0, s, m, rn, W, res);
    BDG_CHECK_LAUNCH();
    GemmArgs g2{m, m, n, 1.0, 0.0, 0.0, 0.0, Z, ldz, Z, ldz, G, m, GEMM_FULL, 1, nullptr};
    BDG_TRY((gemm<double, true>('C', 'N', g2, s)));
    double *gc = R;  // m per-column maxima (R no longer needed; 2nm >= m)
    hipLaunchKernelGGL(gram_cols, dim3((unsigned)m), dim3(256), 0, s, m, G, gc);
    BDG_CHECK_LAUNCH();
    hipLaunchKernelGGL(max_reduce, dim3(1), dim3(1024), 0, s, m, gc, (const double *)nullptr, res + 2);
    BDG_CHECK_LAUNCH();
    double h[4];
    BDG_HIP(hipMemcpyAsync(h, res, sizeof(h), hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    *max_resid = h[1] > 0.0 ? h[0] / h[1] : h[0];
    *gram_defect = h[2];
    return 0;
}

}  // namespace bdg
