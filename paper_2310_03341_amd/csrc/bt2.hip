// Back-transformation 2: eigenvectors of the real tridiagonal -> eigenvectors
// of the band matrix ("the subsequent back transformation of the eigenvectors
// also requires two stages", paper sec. "Performance of the Matrix
// Diagonalization Algorithm").
//
// Z <- Q2 D Y: D = diag(ph) undoes the phase scaling that made the
// tridiagonal real, Q2 = H_{0,0} H_{0,1} ... (generation order of stage 2).
//
// Reflectors of the same task index t from nbk consecutive sweeps S form one
// block G(S, t) = H_{s0,t} ... H_{s0+nbk-1,t} = I - V T V^H (V a
// parallelogram, (b + nbk - 1) x nbk).  Within the sweeps of S, reflectors of
// different t commute in the order G(S, T-1) ... G(S, 0) (rows of H_{s,t} end
// before those of H_{s',t'} start whenever s' > s and t' > t, and
// H_{s',t'} precedes H_{s,t} in generation order whenever s' < s, t' < t, with
// disjoint rows); so  Z <- Q2 Z  applies, for S from last to first, G(S, 0),
// G(S, 1), ... in that order.  Columns of Z are independent: each workgroup
// owns a slab of columns and streams all blocks through LDS.
#include "gemm.h"
#include "stages.h"

namespace bdg {
namespace {

constexpr int NBK = 16;     // sweeps per block
constexpr int BMAX = 64;
constexpr int HMAX = BMAX + NBK - 1;
constexpr int SLAB = 16;    // columns of Z per workgroup

// Phase vector: ph_0 = 1, ph_{i+1} = ph_i e_i / |e_i| (renormalised); |e| out.
__global__ void phases_kernel(int64_t n, const double *__restrict__ e_cplx, double *__restrict__ ph,
                              double *__restrict__ e_abs) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double pr = 1.0, pi = 0.0;
    ph[0] = 1.0;
    ph[1] = 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        const double er = e_cplx[2 * i], ei = e_cplx[2 * i + 1];
        const double a = hypot(er, ei);
        e_abs[i] = a;
        if (a > 0.0) {
            const double ur = er / a, ui = ei / a;
            const double nr = pr * ur - pi * ui, ni = pr * ui + pi * ur;
            const double nn = hypot(nr, ni);
            pr = nr / nn;
            pi = ni / nn;
        }
        ph[2 * (i + 1)] = pr;
        ph[2 * (i + 1) + 1] = pi;
    }
}

// Z[:, j] = ph .* Y[:, i0 + j]  (Y real, ld n)
__global__ void scale_phase(int64_t n, int64_t m, const double *__restrict__ Y, int64_t i0,
                            const double *__restrict__ ph, double *__restrict__ Z, int64_t ldz) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double y = Y[i + (i0 + j) * n];
        Z[2 * (i + j * ldz)] = ph[2 * i] * y;
        Z[2 * (i + j * ldz) + 1] = ph[2 * i + 1] * y;
    }
}

// T factor of every block G(S, t): forward column-wise recurrence from
// V^H V over the parallelogram and the scales tau.  One workgroup per block.
__global__ __launch_bounds__(256) void bt2_tfactors(int64_t n, int b, const double *__restrict__ V2,
                                                    const double *__restrict__ tau2,
                                                    const int64_t *__restrict__ voff, int64_t nsb,
                                                    int64_t tmax, double *__restrict__ TF) {
    __shared__ double2 Vs[HMAX * NBK];
    __shared__ double2 Gs[NBK * NBK];
    __shared__ double2 Ts[NBK * NBK];
    __shared__ double ts[NBK];
    const int64_t blk = blockIdx.x;
    const int64_t S = blk / tmax, t = blk % tmax;
    const int64_t s0 = S * NBK;
    const int tid = threadIdx.x;
    const int64_t nsw = n - 2;
    // parallelogram: column j holds reflector (s0 + j, t) at rows j .. j + b - 1
    for (int e = tid; e < HMAX * NBK; e += blockDim.x) {
        const int r = e % HMAX, j = e / HMAX;
        const int64_t s = s0 + j;
        double2 v = make_double2(0.0, 0.0);
        if (s < nsw && t < (n - 2 - s) / b + 1) {
            const int o = r - j;
            if (o >= 0 && o < b) v = *(const double2 *)(V2 + 2 * ((voff[s] + t) * b + o));
        }
        Vs[r + j * HMAX] = v;
    }
    if (tid < NBK) {
        const int64_t s = s0 + tid;
        ts[tid] = (s < nsw && t < (n - 2 - s) / b + 1) ? tau2[voff[s] + t] : 0.0;
    }
    __syncthreads();
    // G = V^H V
    {
        const int i = tid % NBK, j = tid / NBK;  // 256 = 16 x 16
        double gr = 0.0, gi = 0.0;
        for (int r = 0; r < HMAX; ++r) {
            const double2 a = Vs[r + i * HMAX], c = Vs[r + j * HMAX];
            gr += a.x * c.x + a.y * c.y;
            gi += a.x * c.y - a.y * c.x;
        }
        Gs[i + j * NBK] = make_double2(gr, gi);
        Ts[i + j * NBK] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int j = 0; j < NBK; ++j) {
        const double tj = ts[j];
        if (tid < j) {
            double sr = 0.0, si = 0.0;
            for (int l = tid; l < j; ++l) {
                const double2 a = Ts[tid + l * NBK], g = Gs[l + j * NBK];
                sr += a.x * g.x - a.y * g.y;
                si += a.x * g.y + a.y * g.x;
            }
            Ts[tid + j * NBK] = make_double2(-tj * sr, -tj * si);
        }
        if (tid == j) Ts[j + j * NBK] = make_double2(tj, 0.0);
        __syncthreads();
    }
    {
        const int i = tid % NBK, j = tid / NBK;
        *(double2 *)(TF + 2 * (blk * NBK * NBK + i + j * NBK)) = Ts[i + j * NBK];
    }
}

// Apply every block to a slab of SLAB columns.  256 threads = 16 columns x 16 lanes.
__global__ __launch_bounds__(256) void bt2_apply(int64_t n, int b, int64_t m,
                                                 const double *__restrict__ V2,
                                                 const int64_t *__restrict__ voff, int64_t nsb,
                                                 int64_t tmax, const double *__restrict__ TF,
                                                 double *__restrict__ Z, int64_t ldz) {
    __shared__ double2 Vs[HMAX * NBK];
    __shared__ double2 Ts[NBK * NBK];
    __shared__ double2 Zs[HMAX * SLAB];
    __shared__ double2 Ws[NBK * SLAB];
    __shared__ double2 W2[NBK * SLAB];
    const int tid = threadIdx.x;
    const int64_t j0 = (int64_t)blockIdx.x * SLAB;
    const int ncol = (int)min((int64_t)SLAB, m - j0);
    const int64_t nsw = n - 2;
    for (int64_t S = nsb - 1; S >= 0; --S) {
        const int64_t s0 = S * NBK;
        const int64_t T0 = (n - 2 - s0) / b + 1;  // tasks of the first sweep (the most)
        for (int64_t t = 0; t < T0; ++t) {
            const int64_t rs = s0 + 1 + t * b;
            if (rs >= n) break;
            const int h = (int)min((int64_t)HMAX, n - rs);
            __syncthreads();
            for (int e = tid; e < HMAX * NBK; e += blockDim.x) {
                const int r = e % HMAX, j = e / HMAX;
                const int64_t s = s0 + j;
                double2 v = make_double2(0.0, 0.0);
                if (s < nsw && t < (n - 2 - s) / b + 1 && r < h) {
                    const int o = r - j;
                    if (o >= 0 && o < b) v = *(const double2 *)(V2 + 2 * ((voff[s] + t) * b + o));
                }
                Vs[r + j * HMAX] = v;
            }
            {
                const int i = tid % NBK, j = tid / NBK;
                Ts[i + j * NBK] = *(const double2 *)(TF + 2 * ((S * tmax + t) * NBK * NBK + i + j * NBK));
            }
            for (int e = tid; e < HMAX * SLAB; e += blockDim.x) {
                const int r = e % HMAX, c = e / HMAX;
                double2 z = make_double2(0.0, 0.0);
                if (r < h && c < ncol) z = *(const double2 *)(Z + 2 * ((rs + r) + (j0 + c) * ldz));
                Zs[r + c * HMAX] = z;
            }
            __syncthreads();
            // W = V^H Z  (NBK x SLAB)
            {
                const int i = tid % NBK, c = tid / NBK;
                double wr = 0.0, wi = 0.0;
                for (int r = 0; r < h; ++r) {
                    const double2 v = Vs[r + i * HMAX], z = Zs[r + c * HMAX];
                    wr += v.x * z.x + v.y * z.y;
                    wi += v.x * z.y - v.y * z.x;
                }
                Ws[i + c * NBK] = make_double2(wr, wi);
            }
            __syncthreads();
            // W2 = T W
            {
                const int i = tid % NBK, c = tid / NBK;
                double wr = 0.0, wi = 0.0;
                for (int l = i; l < NBK; ++l) {
                    const double2 a = Ts[i + l * NBK], w = Ws[l + c * NBK];
                    wr += a.x * w.x - a.y * w.y;
                    wi += a.x * w.y + a.y * w.x;
                }
                W2[i + c * NBK] = make_double2(wr, wi);
            }
            __syncthreads();
            // Z -= V W2
            for (int e = tid; e < h * SLAB; e += blockDim.x) {
                const int r = e % h, c = e / h;
                if (c >= ncol) continue;
                double zr = Zs[r + c * HMAX].x, zi = Zs[r + c * HMAX].y;
                for (int l = 0; l < NBK; ++l) {
                    const double2 v = Vs[r + l * HMAX], w = W2[l + c * NBK];
                    zr -= v.x * w.x - v.y * w.y;
                    zi -= v.x * w.y + v.y * w.x;
                }
                *(double2 *)(Z + 2 * ((rs + r) + (j0 + c) * ldz)) = make_double2(zr, zi);
            }
        }
    }
}

}  // namespace

int64_t bt2_nblocks(int64_t n, int b) {
    const int64_t nsw = n - 2;
    if (nsw <= 0) return 0;
    const int64_t nsb = (nsw + NBK - 1) / NBK;
    const int64_t tmax = (n - 2) / b + 1;
    return nsb * tmax;
}

size_t bt2_workspace(int64_t n, int b) { return 16 * (size_t)bt2_nblocks(n, b) * NBK * NBK + 256; }

int phases(int64_t n, const double *e_cplx, double *ph, double *e_abs, hipStream_t s) {
    hipLaunchKernelGGL(phases_kernel, dim3(1), dim3(64), 0, s, n, e_cplx, ph, e_abs);
    BDG_CHECK_LAUNCH();
    return 0;
}

int phase_scale(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, double *Z,
                int64_t ldz, hipStream_t s) {
    if (m <= 0) return 0;
    hipLaunchKernelGGL(scale_phase, dim3((unsigned)m), dim3(256), 0, s, n, m, Y, i0, ph, Z, ldz);
    BDG_CHECK_LAUNCH();
    return 0;
}

int bt2(int64_t n, int b, int64_t m, const double *V2, const double *tau2, const int64_t *voff,
        double *Z, int64_t ldz, void *work, hipStream_t s) {
    if (n < 3 || m <= 0) return 0;
    if (b > BMAX) return BDG_ERR_NOT_IMPLEMENTED;
    const int64_t nsw = n - 2;
    const int64_t nsb = (nsw + NBK - 1) / NBK;
    const int64_t tmax = (n - 2) / b + 1;
    double *TF = (double *)work;
    hipLaunchKernelGGL(bt2_tfactors, dim3((unsigned)(nsb * tmax)), dim3(256), 0, s, n, b, V2, tau2, voff,
                       nsb, tmax, TF);
    BDG_CHECK_LAUNCH();
    hipLaunchKernelGGL(bt2_apply, dim3((unsigned)((m + SLAB - 1) / SLAB)), dim3(256), 0, s, n, b, m, V2,
                       voff, nsb, tmax, TF, Z, ldz);
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace bdg
