// FP64 matrix products emulated on the INT8 matrix cores (Ozaki, Ogita, Oishi
// and Rump, Numer. Algorithms 59 (2012), error-free splitting of the factors;
// Ootomo, Ozaki and Yokota, IJHPCA 2024, the integer form on 8-bit units).
//
// For C = op(A) op(B) (real, or complex through the real embedding
// [[Ar, -Ai], [Ai, Ar]] [[Br], [Bi]], which keeps one scale per row of A and
// per column of B for both parts):
//   1. each row r of op(A) gets the exponent e_r with max |A_r.| < 2^(e_r - 1),
//      each column c of op(B) e_c likewise;
//   2. X = round(A_rk 2^(7 S - e_r)) is cut into S balanced base-128 digits,
//      X = sum_i d_i 128^(S - i): d_2 .. d_S in [-64, 63], d_1 within +-65,
//      stored as S int8 slices (rows of op(A), columns of op(B) with k
//      contiguous, K padded to the 64-deep MFMA step);
//   3. C_rc = 2^(e_r + e_c) sum_{t=2}^{S+1} 128^-t sum_{i+j=t} (D^A_i D^B_j)_rc,
//      every D^A_i D^B_j exact in int32 on v_mfma_i32_16x16x64_i8; the pairs of
//      one t are summed in int32 over one 64-deep step (|sum| <= S 64 65^2 <
//      2^22) and then converted to FP64 and added with their power-of-two
//      weight, so nothing overflows whatever K is.  Dropping i + j > S + 1 and the rounding in step 2
//      bound the error by 2^(e_r + e_c) K (128^-S + (S + 1) 65^2 128^-(S+2)).
// S = 8 gives FP64-level accuracy against the row and column scales
// (2^-56 per term); S = 36 pair products per step.
#include <math.h>

#include "gemm.h"
#include "solver.h"

namespace bdg {
namespace {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int OT = 64;     // output tile (rows and columns) of one workgroup
constexpr int OK = 64;     // K step (one MFMA depth)
constexpr int LP = 80;     // LDS row pitch in bytes (64 + 16: no bank conflicts for 16-byte lane reads)

// element (r, k) of a line view of the column-major X: X[r + k ld] (trans =
// false) or X[k + r ld] (trans = true), conjugated when conj
template <bool CX>
__device__ __forceinline__ void opel(const double *X, int64_t ld, bool trans, bool conj, int64_t r, int64_t k,
                                     double &re, double &im) {
    const int64_t idx = trans ? k + r * ld : r + k * ld;
    if constexpr (CX) {
        const double2 v = *(const double2 *)(X + 2 * idx);
        re = v.x;
        im = conj ? -v.y : v.y;
    } else {
        re = X[idx];
        im = 0.0;
    }
}

// exponent e of each line (rows of op(A), or columns of op(B) seen as rows of
// op(B)^T) with max |re|, |im| < 2^(e - 1); 0 for an all-zero line.  One
// workgroup per line.
template <bool CX>
__global__ __launch_bounds__(256) void line_exponents(const double *X, int64_t ld, bool trans, int64_t len,
                                                      int *e) {
    __shared__ double red[4];
    const int64_t r = blockIdx.x;
    double mx = 0.0;
    for (int64_t k = threadIdx.x; k < len; k += blockDim.x) {
        double re, im;
        opel<CX>(X, ld, trans, false, r, k, re, im);
        mx = fmax(mx, fmax(fabs(re), fabs(im)));
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
        int ex = 0;
        if (m > 0.0) {
            (void)frexp(m, &ex);  // m < 2^ex
            ex += 1;
        }
        e[r] = ex;
    }
}

// S digit slices of the (embedded) rows: out[i][row][k], row < rows_p, k < Kp.
// Complex embedding (CX): for the left factor, embedded row r < M is
// [re(r, :), -im(r, :)], row M + r is [im(r, :), re(r, :)]; for the right
// factor (embedded "row" = column c of op(B)) it is [re(:, c), im(:, c)].
// Rows and k beyond the data are zero.  Tiles of 64 x 64 through LDS so that
// both the reads of X and the writes of the slices are coalesced.
template <bool CX, int S>
__global__ __launch_bounds__(256) void make_slices(const double *X, int64_t ld, bool trans, bool conj, bool left,
                                                   int64_t M, int64_t K, const int *__restrict__ e, int64_t rows_p,
                                                   int64_t Kp, signed char *__restrict__ out) {
    __shared__ double tile[64][65];
    const int64_t rows = CX && left ? 2 * M : M;
    const int64_t Ke = CX ? 2 * K : K;
    const int64_t r0 = (int64_t)blockIdx.y * 64, k0 = (int64_t)blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    // load: the source index runs fastest along k for a transposed view, along
    // r otherwise
    for (int q = ty; q < 64; q += 4) {
        const int64_t r = trans ? r0 + q : r0 + tx, k = trans ? k0 + tx : k0 + q;
        const int64_t rr = CX && left && r >= M ? r - M : r;       // source row of op(X)
        const int64_t kk = CX && k >= K ? k - K : k;               // source k
        double re = 0.0, im = 0.0;
        if (r < rows && k < Ke) opel<CX>(X, ld, trans, conj, rr, kk, re, im);
        double v;
        if (!CX) v = re;
        else if (!left) v = k < K ? re : im;                       // [re; im]
        else if (r < M) v = k < K ? re : -im;                      // [re, -im]
        else v = k < K ? im : re;                                  // [im, re]
        const int lr = trans ? q : tx, lk = trans ? tx : q;
        tile[lr][lk] = v;
    }
    __syncthreads();
    for (int q = ty; q < 64; q += 4) {
        const int64_t r = r0 + q, k = k0 + tx;
        if (r >= rows_p || k >= Kp) continue;
        const int64_t er = CX && left && r >= M ? r - M : r;
        const int ex = (r < rows) ? e[er] : 0;
        const double x = tile[q][tx];
        // X = round(x 2^(7 S - e)), |X| <= 2^(7 S - 1)
        long long X = (long long)rint(ldexp(x, 7 * S - ex));
        signed char dg[S];
#pragma unroll
        for (int i = S - 1; i >= 1; --i) {
            long long d = ((X + 64) & 127) - 64;  // balanced digit in [-64, 63]
            dg[i] = (signed char)d;
            X = (X - d) / 128;
        }
        dg[0] = (signed char)X;
#pragma unroll
        for (int i = 0; i < S; ++i) out[((int64_t)i * rows_p + r) * Kp + k] = dg[i];
    }
}

// R[r][c] = 2^(e_r + e_c) sum_t 128^-t sum_{i+j=t} (A_i B_j^T)[r][c], one 64 x 64
// tile per workgroup, four waves of 2 x 2 MFMA 16 x 16 blocks.  Lane l holds
// row l % 16 of the A block and column l % 16 of the B block, k = 16 (l / 16)
// + q for its 16 bytes; accumulator element q of lane l is row 4 (l / 16) + q.
template <int S>
__global__ __launch_bounds__(256) void ozaki_kernel(int64_t Mr, int64_t N, int64_t rows_p, int64_t cols_p,
                                                    int64_t Kp, const signed char *__restrict__ SA,
                                                    const signed char *__restrict__ SB,
                                                    const int *__restrict__ ea, const int *__restrict__ eb,
                                                    int64_t M_half, double *__restrict__ R, int64_t ldr) {
    __shared__ __attribute__((aligned(16))) signed char As[S][OT * LP];
    __shared__ __attribute__((aligned(16))) signed char Bs[S][OT * LP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t r0 = (int64_t)blockIdx.y * OT, c0 = (int64_t)blockIdx.x * OT;
    const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
    double facc[2][2][4];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int q = 0; q < 4; ++q) facc[a][b][q] = 0.0;
    for (int64_t k0 = 0; k0 < Kp; k0 += OK) {
        __syncthreads();
        // stage the S slices of both 64 x 64 tiles: 16 bytes per thread per row chunk
        for (int e = tid; e < S * OT * 4; e += 256) {
            const int i = e / (OT * 4), rem = e % (OT * 4), row = rem >> 2, ch = rem & 3;
            const v4i va = *(const v4i *)(SA + ((int64_t)i * rows_p + r0 + row) * Kp + k0 + 16 * ch);
            const v4i vb = *(const v4i *)(SB + ((int64_t)i * cols_p + c0 + row) * Kp + k0 + 16 * ch);
            *(v4i *)(&As[i][row * LP + 16 * ch]) = va;
            *(v4i *)(&Bs[i][row * LP + 16 * ch]) = vb;
        }
        __syncthreads();
        v4i a[S][2], b[S][2];
#pragma unroll
        for (int i = 0; i < S; ++i)
#pragma unroll
            for (int x = 0; x < 2; ++x) {
                a[i][x] = *(const v4i *)(&As[i][(wr + 16 * x + (lane & 15)) * LP + 16 * (lane >> 4)]);
                b[i][x] = *(const v4i *)(&Bs[i][(wc + 16 * x + (lane & 15)) * LP + 16 * (lane >> 4)]);
            }
#pragma unroll
        for (int t = S + 1; t >= 2; --t) {
            v4i acc[2][2];
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y) acc[x][y] = v4i{0, 0, 0, 0};
#pragma unroll
            for (int i = 1; i <= S; ++i) {
                const int j = t - i;
                if (j < 1 || j > S) continue;
#pragma unroll
                for (int x = 0; x < 2; ++x)
#pragma unroll
                    for (int y = 0; y < 2; ++y)
                        acc[x][y] = __builtin_amdgcn_mfma_i32_16x16x64_i8(a[i - 1][x], b[j - 1][y], acc[x][y], 0, 0, 0);
            }
            const double w = ldexp(1.0, -7 * t);
#pragma unroll
            for (int x = 0; x < 2; ++x)
#pragma unroll
                for (int y = 0; y < 2; ++y)
#pragma unroll
                    for (int q = 0; q < 4; ++q) facc[x][y][q] += w * (double)acc[x][y][q];
        }
    }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t r = r0 + wr + 16 * x + 4 * (lane >> 4) + q;
                const int64_t c = c0 + wc + 16 * y + (lane & 15);
                if (r < Mr && c < N) {
                    const int er = ea[M_half > 0 && r >= M_half ? r - M_half : r];
                    R[r + c * ldr] = ldexp(facc[x][y][q], er + eb[c]);
                }
            }
}

// C = alpha (R_re + i R_im) + beta C (complex; R rows M .. 2M-1 the imaginary
// part) or C = alpha R + beta C (real)
template <bool CX>
__global__ void ozaki_epilogue(int64_t M, int64_t N, const double *__restrict__ R, int64_t ldr, double ar,
                               double ai, double br, double bi, double *C, int64_t ldc) {
    const int64_t c = blockIdx.y;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < M; r += (int64_t)gridDim.x * blockDim.x) {
        if constexpr (CX) {
            const double xr = R[r + c * ldr], xi = R[M + r + c * ldr];
            double2 *p = (double2 *)(C + 2 * (r + c * ldc));
            double2 v = make_double2(ar * xr - ai * xi, ar * xi + ai * xr);
            if (br != 0.0 || bi != 0.0) {
                const double2 o = *p;
                v.x += br * o.x - bi * o.y;
                v.y += br * o.y + bi * o.x;
            }
            *p = v;
        } else {
            double v = ar * R[r + c * ldr];
            if (br != 0.0) v += br * C[r + c * ldc];
            C[r + c * ldc] = v;
        }
    }
}

int64_t rup(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct OzLayout {
    int64_t Mr, rows_p, cols_p, Kp;
    size_t off_SA, off_SB, off_ea, off_eb, off_R, total;
};

OzLayout oz_layout(bool cx, int64_t M, int64_t N, int64_t K, int S) {
    OzLayout L;
    L.Mr = cx ? 2 * M : M;
    L.rows_p = rup(L.Mr, OT);
    L.cols_p = rup(N, OT);
    L.Kp = rup(cx ? 2 * K : K, OK);
    size_t o = 0;
    auto put = [&](size_t b) { size_t r = o; o += (b + 255) / 256 * 256; return r; };
    L.off_SA = put((size_t)S * L.rows_p * L.Kp);
    L.off_SB = put((size_t)S * L.cols_p * L.Kp);
    L.off_ea = put(4 * (size_t)std::max<int64_t>(M, 1));
    L.off_eb = put(4 * (size_t)std::max<int64_t>(N, 1));
    L.off_R = put(8 * (size_t)L.Mr * N);
    L.total = o + 256;
    return L;
}

template <bool CX, int S>
int ozaki_t(char opA, char opB, int64_t M, int64_t N, int64_t K, const double *alpha, const double *A,
            int64_t lda, const double *B, int64_t ldb, const double *beta, double *C, int64_t ldc, void *work,
            hipStream_t s) {
    const OzLayout L = oz_layout(CX, M, N, K, S);
    char *base = (char *)work;
    signed char *SA = (signed char *)(base + L.off_SA);
    signed char *SB = (signed char *)(base + L.off_SB);
    int *ea = (int *)(base + L.off_ea);
    int *eb = (int *)(base + L.off_eb);
    double *R = (double *)(base + L.off_R);
    // lines of the left factor: rows r of op(A), element k = A[r + k lda] for
    // op N, conj(A[k + r lda]) for op C; lines of the right factor: columns c
    // of op(B), element k = B[k + c ldb] for op N, conj(B[c + k ldb]) for op C
    const bool ca = opA == 'C' || opA == 'c' || opA == 'T' || opA == 't';
    const bool cb = opB == 'C' || opB == 'c' || opB == 'T' || opB == 't';
    hipLaunchKernelGGL((line_exponents<CX>), dim3((unsigned)M), dim3(256), 0, s, A, lda, ca, K, ea);
    hipLaunchKernelGGL((line_exponents<CX>), dim3((unsigned)N), dim3(256), 0, s, B, ldb, !cb, K, eb);
    BDG_CHECK_LAUNCH();
    {
        const dim3 ga((unsigned)(L.Kp / 64), (unsigned)(L.rows_p / 64));
        hipLaunchKernelGGL((make_slices<CX, S>), ga, dim3(256), 0, s, A, lda, ca, ca, true, M, K, ea, L.rows_p, L.Kp,
                           SA);
        const dim3 gb((unsigned)(L.Kp / 64), (unsigned)(L.cols_p / 64));
        hipLaunchKernelGGL((make_slices<CX, S>), gb, dim3(256), 0, s, B, ldb, !cb, cb, false, N, K, eb, L.cols_p,
                           L.Kp, SB);
        BDG_CHECK_LAUNCH();
    }
    const dim3 grid((unsigned)(L.cols_p / OT), (unsigned)(L.rows_p / OT));
    hipLaunchKernelGGL((ozaki_kernel<S>), grid, dim3(256), 0, s, L.Mr, N, L.rows_p, L.cols_p, L.Kp, SA, SB, ea, eb,
                       CX ? M : (int64_t)0, R, L.Mr);
    BDG_CHECK_LAUNCH();
    const unsigned gx = (unsigned)std::min<int64_t>(64, (M + 255) / 256);
    hipLaunchKernelGGL((ozaki_epilogue<CX>), dim3(gx, (unsigned)N), dim3(256), 0, s, M, N, R, L.Mr, alpha[0],
                       CX ? alpha[1] : 0.0, beta[0], CX ? beta[1] : 0.0, C, ldc);
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace

size_t ozaki_workspace(bool cx, int64_t M, int64_t N, int64_t K, int S) { return oz_layout(cx, M, N, K, S).total; }

int ozaki_gemm(bool cx, int S, char opA, char opB, int64_t M, int64_t N, int64_t K, const double *alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb, const double *beta, double *C,
               int64_t ldc, void *work, hipStream_t s) {
    if (M <= 0 || N <= 0) return 0;
#define BDG_OZ(SV)                                                                                          \
    case SV:                                                                                                \
        return cx ? ozaki_t<true, SV>(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, s)     \
                  : ozaki_t<false, SV>(opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work, s);
    switch (S) {
        BDG_OZ(3)
        BDG_OZ(4)
        BDG_OZ(5)
        BDG_OZ(6)
        BDG_OZ(7)
        BDG_OZ(8)
        default:
            set_error("ozaki gemm: slices must be 3..8");
            return BDG_ERR_NOT_IMPLEMENTED;
    }
#undef BDG_OZ
}

}  // namespace bdg
