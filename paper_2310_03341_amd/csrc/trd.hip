// One-stage FP64 eigensolver: dense -> real tridiagonal in one Householder
// reduction, tridiagonal divide and conquer, one back-transformation.  The
// paper benchmarks ELPA's one-stage solver on real symmetric matrices and
// states that the complex Hermitian problem takes about twice as long (sec.
// "Performance of the Matrix Diagonalization Algorithm"); this path gives both
// element types (real = symmetric, complex = Hermitian) next to the two-stage
// solver of bdg_eigh.
//
// Reduction (lower triangle, panels of NB columns).  Column c of panel k gets
// H_c = I - tau v v^H with H_c^H A[c+1:, c] = (beta, 0, ..., 0), beta real:
//   alpha = A[c+1, c], beta = -sign(Re alpha) ||A[c+1:, c]||,
//   tau = (beta - alpha) / beta,  v = (1, A[c+2:, c] / (alpha - beta)).
// The two-sided update H^H A H = A - v w^H - w v^H uses
//   w = tau y - (|tau|^2 / 2)(v^H y) v,  y = A v,
// and inside a panel the matrix is not updated: column c first receives the
// earlier reflectors of the panel, and y = A v - V (W^H v) - W (V^H v) (the
// delayed update of the blocked Householder tridiagonalisation).  After the
// panel, A[k+NB:, k+NB:] -= [V W] [W V]^H on the lower tiles (MFMA GEMM).
// y = A v is the memory-bound half of the flops: every column reads the
// lower triangle of the trailing matrix once (tiles of 64 x 64; each tile adds
// its product to its row block and its adjoint product to its column block,
// in partial sums that a second kernel adds in a fixed order).
//
// Back-transformation: Z = H_0 H_1 ... Y, panel by panel in reverse order with
// the compact WY form Q_p = I - V_p T_p V_p^H, T_p = (diag(1/tau) +
// strictly-upper(V_p^H V_p))^-1 (zero rows and columns where tau = 0).
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "gemm.h"
#include "solver.h"
#include "stages.h"

namespace bdg {
namespace {

constexpr int NB = 64;    // panel width
constexpr int HT = 64;    // hemv tile
constexpr int HCH = 8;    // tiles per hemv workgroup along a tile column
constexpr int CB = 256;   // threads of the column kernels

// element access: complex interleaved (re, im) or real
template <bool CX>
__device__ __forceinline__ zd eld(const double *p, int64_t i) {
    if constexpr (CX) {
        const double2 v = *(const double2 *)(p + 2 * i);
        return mk(v.x, v.y);
    } else {
        return mk(p[i], 0.0);
    }
}
template <bool CX>
__device__ __forceinline__ void est(double *p, int64_t i, zd v) {
    if constexpr (CX) *(double2 *)(p + 2 * i) = make_double2(v.re, v.im);
    else p[i] = v.re;
}
// a * conj(b) and the complex multiply-add helpers
__device__ __forceinline__ zd mulc(zd a, zd b) { return mk(a.re * b.re + a.im * b.im, a.im * b.re - a.re * b.im); }

__device__ inline double block_sum(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += red[i];
    return s;
}

// Column c (panel column j, panel start k): apply the panel's earlier
// reflectors, A[r, c] -= sum_{i<j} V[r,i] conj(W[c,i]) + W[r,i] conj(V[c,i])
// for rows r >= c; partial sums of |A[r, c]|^2 over r >= c + 2.
template <bool CX>
__global__ __launch_bounds__(CB) void col_update(int64_t n, int64_t c, int j, double *A, int64_t lda,
                                                 const double *__restrict__ VW, int64_t ldw,
                                                 double *__restrict__ part) {
    __shared__ double red[4];
    __shared__ double2 vc[NB], wc[NB];  // conj(W[c, i]), conj(V[c, i])
    for (int i = threadIdx.x; i < j; i += blockDim.x) {
        const zd v = eld<CX>(VW, c + (int64_t)i * ldw), w = eld<CX>(VW, c + (int64_t)(NB + i) * ldw);
        wc[i] = make_double2(w.re, -w.im);
        vc[i] = make_double2(v.re, -v.im);
    }
    __syncthreads();
    const int64_t r = c + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double nrm = 0.0;
    if (r < n) {
        zd a = eld<CX>(A, r + c * lda);
        for (int i = 0; i < j; ++i) {
            const zd v = eld<CX>(VW, r + (int64_t)i * ldw), w = eld<CX>(VW, r + (int64_t)(NB + i) * ldw);
            const zd cw = mk(wc[i].x, wc[i].y), cv = mk(vc[i].x, vc[i].y);
            a = csub(a, cadd(cmul(v, cw), cmul(w, cv)));
        }
        est<CX>(A, r + c * lda, a);
        if (r >= c + 2) nrm = cabs2(a);
    }
    nrm = block_sum(nrm, red);
    if (threadIdx.x == 0) part[blockIdx.x] = nrm;
}

// Reflector of column c: d[c], e[c] = beta, tau[c], scal = 1 / (alpha - beta)
// (0 when no reflection is needed).  One block.
template <bool CX>
__global__ void reflector(int64_t n, int64_t c, const double *A, int64_t lda, const double *__restrict__ part,
                          int nparts, double *d, double *e, double *tau, double *scal) {
    __shared__ double red[4];
    double s = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x != 0) return;
    d[c] = eld<CX>(A, c + c * lda).re;
    const zd al = eld<CX>(A, c + 1 + c * lda);
    double tr = 0.0, ti = 0.0, sr = 0.0, si = 0.0, beta = al.re;
    if (!(s == 0.0 && al.im == 0.0)) {
        const double nrm = sqrt(al.re * al.re + al.im * al.im + s);
        beta = al.re >= 0.0 ? -nrm : nrm;
        tr = (beta - al.re) / beta;
        ti = -al.im / beta;
        // 1 / (alpha - beta)
        const double xr = al.re - beta, xi = al.im, q = xr * xr + xi * xi;
        sr = xr / q;
        si = -xi / q;
    }
    e[c] = beta;
    tau[2 * c] = tr;
    tau[2 * c + 1] = ti;
    scal[0] = sr;
    scal[1] = si;
}

// v = (1, A[c+2:, c] scal) stored in A (with zeros on rows k+1 .. c of column
// c, so that the panel's V is explicit) and in the panel buffers.
template <bool CX>
__global__ __launch_bounds__(CB) void scale_v(int64_t n, int64_t c, int64_t k, int j, double *A, int64_t lda,
                                              const double *__restrict__ scal, double *VW, double *WV,
                                              int64_t ldw) {
    const zd s = mk(scal[0], scal[1]);
    for (int64_t r = k + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        zd v;
        if (r <= c) v = mk(0.0, 0.0);
        else if (r == c + 1) v = mk(1.0, 0.0);
        else v = cmul(eld<CX>(A, r + c * lda), s);
        est<CX>(A, r + c * lda, v);
        est<CX>(VW, r + (int64_t)j * ldw, v);
        est<CX>(WV, r + (int64_t)(NB + j) * ldw, v);
    }
}

// u[i] = W[:, i]^H v and u[NB + i] = V[:, i]^H v over rows c+1 .. n-1, i < j
// (block i of 2j: the first j use W, the next j use V).
template <bool CX>
__global__ __launch_bounds__(CB) void panel_dots(int64_t n, int64_t c, int j, const double *__restrict__ VW,
                                                 int64_t ldw, double *__restrict__ u) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int i = b < j ? b : b - j;
    const double *X = VW + (CX ? 2 : 1) * (int64_t)(b < j ? NB + i : i) * ldw;
    const double *v = VW + (CX ? 2 : 1) * (int64_t)j * ldw;
    double sr = 0.0, si = 0.0;
    for (int64_t r = c + 1 + threadIdx.x; r < n; r += blockDim.x) {
        const zd p = cjmul(eld<CX>(X, r), eld<CX>(v, r));
        sr += p.re;
        si += p.im;
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red);
    if (threadIdx.x == 0) {
        const int o = b < j ? i : NB + i;
        u[2 * o] = sr;
        u[2 * o + 1] = si;
    }
}

// Partial products of y = B v for the Hermitian trailing block B (order mt,
// lower triangle valid).  Workgroup (J, q): tiles I = J + q HCH .. (up to HCH
// of them) of tile column J.  P1[J][row] += B_IJ v_J for the rows of tile I;
// P2[J][q][col] = sum over its tiles of B_IJ^H v_I for the columns of tile J.
// On the diagonal tile only the strictly lower part adds its adjoint and the
// diagonal adds once.  512 threads: lane r is row r of a tile (coalesced
// column reads), wave cq holds columns 8 cq .. 8 cq + 7.  The tile loop has no
// barrier: each thread keeps its part of the row sums of every tile in LDS
// slots of its own, which one barrier at the end reduces over the eight
// waves; the column sums are reduced over the lanes of each wave by DPP
// moves.  With about 120 registers, two workgroups share a CU and hide the
// latency of each other's loads.
constexpr int HW = 8;           // waves of hemv_tiles
constexpr int HC = HT / HW;     // columns per thread
template <bool CX>
__global__ __launch_bounds__(64 * HW, 4) void hemv_tiles(int64_t mt, const double *__restrict__ B, int64_t ldb,
                                                      const double *__restrict__ v, double *__restrict__ P1,
                                                      double *__restrict__ P2, int maxq) {
    const int J = blockIdx.x, q = blockIdx.y;
    const int nt = (int)((mt + HT - 1) / HT);
    const int I0 = J + q * HCH;
    if (I0 >= nt) return;
    const int I1 = std::min(nt, I0 + HCH);
    const int r = threadIdx.x & 63, cq = threadIdx.x >> 6;
    __shared__ double2 rs[HCH][HW][HT];  // row-sum partials: tile, wave, row
    zd vJ[HC], acc2[HC];
    const int64_t c0 = (int64_t)J * HT + cq * HC;
#pragma unroll
    for (int s = 0; s < HC; ++s) {
        vJ[s] = c0 + s < mt ? eld<CX>(v, c0 + s) : mk(0.0, 0.0);
        acc2[s] = mk(0.0, 0.0);
    }
#pragma unroll
    for (int u = 0; u < HCH; ++u) {
        const int I = I0 + u;
        if (I >= I1) break;
        const int64_t row = (int64_t)I * HT + r;
        const bool rok = row < mt;
        const zd vI = rok ? eld<CX>(v, row) : mk(0.0, 0.0);
        zd bv[HC];
#pragma unroll
        for (int s = 0; s < HC; ++s) {
            const int64_t col = c0 + s;
            const bool ok = rok & (col < mt) & ((I != J) | (row >= col));
            // unconditional load from entry 0 outside, so the loads overlap
            const zd b = eld<CX>(B, ok ? row + col * ldb : 0);
            bv[s] = ok ? b : mk(0.0, 0.0);
        }
        zd s1 = mk(0.0, 0.0);
#pragma unroll
        for (int s = 0; s < HC; ++s) {
            const int64_t col = c0 + s;
            zd b = bv[s];
            if (I == J && row == col) b.im = 0.0;  // Hermitian diagonal is real
            s1 = cadd(s1, cmul(b, vJ[s]));
            if (I != J || row > col) acc2[s] = cadd(acc2[s], cjmul(b, vI));
        }
        rs[u][cq][r] = make_double2(s1.re, s1.im);
    }
    // column sums over the 64 rows (lanes) of this wave's columns
#pragma unroll
    for (int s = 0; s < HC; ++s) {
        const double xr = wave_sum_last(acc2[s].re), xi = wave_sum_last(acc2[s].im);
        if (r == 63 && c0 + s < mt) est<CX>(P2, ((int64_t)J * maxq + q) * HT + cq * HC + s, mk(xr, xi));
    }
    __syncthreads();
    // row sums: thread (u, r) of the first HCH x 64 adds the eight waves' parts
    for (int e = threadIdx.x; e < HCH * HT; e += 64 * HW) {
        const int u = e / HT, rr = e % HT;
        const int64_t row = (int64_t)(I0 + u) * HT + rr;
        if (I0 + u >= I1 || row >= mt) continue;
        double xr = 0.0, xi = 0.0;
#pragma unroll
        for (int w = 0; w < HW; ++w) {
            xr += rs[u][w][rr].x;
            xi += rs[u][w][rr].y;
        }
        est<CX>(P1, (int64_t)J * mt + row, mk(xr, xi));
    }
}

// w = tau (y - V u1 - W u2) over rows c+1 .. n-1, with y summed from the hemv
// partials; partial sums of w^H v.  Rows <= c of W's column are zero.
// Workgroup: the 64 rows of tile I (lane = row); its eight waves split the
// terms of y (tile columns J, chunks q and delayed-update columns i, each
// wave every eighth), then one barrier and wave 0 finishes the rows.
template <bool CX>
__global__ __launch_bounds__(64 * HW) void finish_w(int64_t n, int64_t c, int j, const double *__restrict__ tau,
                                                    const double *__restrict__ u, double *VW, int64_t ldw,
                                                    const double *__restrict__ P1, const double *__restrict__ P2,
                                                    int maxq, double *__restrict__ part) {
    __shared__ double2 us[2 * NB];
    __shared__ double2 ys[HW][HT];
    for (int i = threadIdx.x; i < 2 * NB; i += blockDim.x) us[i] = make_double2(u[2 * i], u[2 * i + 1]);
    __syncthreads();
    const int64_t mt = n - c - 1;
    const int I = blockIdx.x, lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t idx = (int64_t)I * HT + lane;  // 0 .. mt-1
    const int nt = (int)((mt + HT - 1) / HT);
    zd y = mk(0.0, 0.0);
    if (idx < mt) {
        const int64_t r = c + 1 + idx;
        for (int J = wv; J <= I; J += HW) y = cadd(y, eld<CX>(P1, (int64_t)J * mt + idx));
        const int nq = (nt - I + HCH - 1) / HCH;
        for (int q = wv; q < nq; q += HW) y = cadd(y, eld<CX>(P2, ((int64_t)I * maxq + q) * HT + lane));
        for (int i = wv; i < j; i += HW) {
            const zd v = eld<CX>(VW, r + (int64_t)i * ldw), w = eld<CX>(VW, r + (int64_t)(NB + i) * ldw);
            y = csub(y, cadd(cmul(v, mk(us[i].x, us[i].y)), cmul(w, mk(us[NB + i].x, us[NB + i].y))));
        }
    }
    ys[wv][lane] = make_double2(y.re, y.im);
    __syncthreads();
    if (wv != 0) return;
    double pr = 0.0, pi = 0.0;
    if (idx < mt) {
        const int64_t r = c + 1 + idx;
        zd ysum = mk(0.0, 0.0);
#pragma unroll
        for (int w = 0; w < HW; ++w) ysum = cadd(ysum, mk(ys[w][lane].x, ys[w][lane].y));
        const zd w = cmul(mk(tau[2 * c], tau[2 * c + 1]), ysum);
        est<CX>(VW, r + (int64_t)(NB + j) * ldw, w);
        const zd p = cjmul(w, eld<CX>(VW, r + (int64_t)j * ldw));
        pr = p.re;
        pi = p.im;
    }
    pr = wave_sum_last(pr);
    pi = wave_sum_last(pi);
    if (lane == 63) {
        part[2 * blockIdx.x] = pr;
        part[2 * blockIdx.x + 1] = pi;
    }
}

// w += alpha v, alpha = -tau (w^H v) / 2; rows <= c set to zero; copies into WV.
template <bool CX>
__global__ __launch_bounds__(CB) void fix_w(int64_t n, int64_t c, int64_t k, int j, const double *__restrict__ tau,
                                            const double *__restrict__ part, int nparts, double *VW, double *WV,
                                            int64_t ldw) {
    __shared__ double red[4];
    __shared__ double al[2];
    double sr = 0.0, si = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) {
        sr += part[2 * i];
        si += part[2 * i + 1];
    }
    sr = block_sum(sr, red);
    si = block_sum(si, red);
    if (threadIdx.x == 0) {
        const zd a = cmul(mk(tau[2 * c], tau[2 * c + 1]), mk(sr, si));
        al[0] = -0.5 * a.re;
        al[1] = -0.5 * a.im;
    }
    __syncthreads();
    const zd a = mk(al[0], al[1]);
    for (int64_t r = k + 1 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * blockDim.x) {
        zd w = mk(0.0, 0.0);
        if (r > c) w = cadd(eld<CX>(VW, r + (int64_t)(NB + j) * ldw), cmul(a, eld<CX>(VW, r + (int64_t)j * ldw)));
        est<CX>(VW, r + (int64_t)(NB + j) * ldw, w);
        est<CX>(WV, r + (int64_t)j * ldw, w);
    }
}

// d[n-1] (and d[0] for n = 1) from the updated diagonal
template <bool CX>
__global__ void last_diag(int64_t n, const double *A, int64_t lda, double *d) {
    if (threadIdx.x == 0 && blockIdx.x == 0) d[n - 1] = eld<CX>(A, (n - 1) + (n - 1) * lda).re;
}

// T = (diag(1/tau) + strictly-upper(G))^-1 for G = V^H V (nb x nb, ld nb),
// column by column by back substitution; zero tau gives a zero row and column.
template <bool CX>
__global__ void tfactor(int nb, const double *__restrict__ G, const double *__restrict__ tau, double *T) {
    __shared__ double2 Ts[NB * NB];
    __shared__ double2 Gs[NB * NB];
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) {
        const zd g = eld<CX>(G, e);
        Gs[e] = make_double2(g.re, g.im);
        Ts[e] = make_double2(0.0, 0.0);
    }
    __syncthreads();
    const int cidx = threadIdx.x;
    if (cidx < nb) {
        const zd tc = mk(tau[2 * cidx], tau[2 * cidx + 1]);
        Ts[cidx + cidx * nb] = make_double2(tc.re, tc.im);
        for (int i = cidx - 1; i >= 0; --i) {
            zd s = mk(0.0, 0.0);
            for (int k = i + 1; k <= cidx; ++k)
                s = cadd(s, cmul(mk(Gs[i + k * nb].x, Gs[i + k * nb].y), mk(Ts[k + cidx * nb].x, Ts[k + cidx * nb].y)));
            const zd ti = mk(tau[2 * i], tau[2 * i + 1]);
            const zd x = cmul(ti, s);
            Ts[i + cidx * nb] = make_double2(-x.re, -x.im);
        }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < nb * nb; e += blockDim.x) est<CX>(T, e, mk(Ts[e].x, Ts[e].y));
}

// Z[:, j] = Y[:, i0 + j] (real Y, ld n) widened to the element type
template <bool CX>
__global__ void widen_cols(int64_t n, const double *__restrict__ Y, int64_t i0, double *Z, int64_t ldz) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) est<CX>(Z, i + j * ldz, mk(Y[i + (i0 + j) * n], 0.0));
}

size_t al256(size_t x) { return (x + 255) / 256 * 256; }

struct L1 {
    int64_t np, nt, maxq, nparts;
    size_t off_d, off_e, off_tau, off_scal, off_part, off_u, off_VW, off_WV, off_P1, off_P2, off_G, off_T,
        off_Wv, off_Q, off_sc, total;
};

L1 layout1(int64_t n, bool cx, int64_t zcols) {
    L1 L;
    const size_t es = cx ? 16 : 8;
    L.np = n >= 2 ? (n - 1 + NB - 1) / NB : 0;
    L.nt = (n + HT - 1) / HT;
    L.maxq = (L.nt + HCH - 1) / HCH;
    L.nparts = (n + HT - 1) / HT + 1;  // >= (n + CB - 1) / CB + 1 as well
    size_t o = 0;
    auto put = [&](size_t b) { size_t r = o; o += al256(b); return r; };
    L.off_d = put(8 * (size_t)n);
    L.off_e = put(8 * (size_t)n);
    L.off_tau = put(16 * (size_t)n);
    L.off_scal = put(16);
    L.off_part = put(16 * (size_t)L.nparts);
    L.off_u = put(16 * 2 * NB);
    L.off_VW = put(es * (size_t)n * 2 * NB);
    L.off_WV = put(es * (size_t)n * 2 * NB);
    L.off_P1 = put(es * (size_t)(L.nt + 1) * n);
    L.off_P2 = put(es * (size_t)(L.nt + 1) * L.maxq * HT);
    L.off_G = put(es * NB * NB);
    L.off_T = put(es * (size_t)(L.np + 1) * NB * NB);
    L.off_Wv = put(8 * (size_t)n);
    L.off_Q = put(8 * (size_t)n * n);
    // stage scratch: D&C, then the back-transformation's two NB x zcols products
    L.off_sc = put(std::max(stedc_workspace(n), 2 * es * (size_t)NB * std::max<int64_t>(zcols, 1)));
    L.total = o + 256;
    return L;
}

template <bool CX>
int trd_t(int64_t n, double *A, int64_t lda, const L1 &L, char *base, hipStream_t s) {
    double *d = (double *)(base + L.off_d);
    double *e = (double *)(base + L.off_e);
    double *tau = (double *)(base + L.off_tau);
    double *scal = (double *)(base + L.off_scal);
    double *part = (double *)(base + L.off_part);
    double *u = (double *)(base + L.off_u);
    double *VW = (double *)(base + L.off_VW);
    double *WV = (double *)(base + L.off_WV);
    double *P1 = (double *)(base + L.off_P1);
    double *P2 = (double *)(base + L.off_P2);
    double *G = (double *)(base + L.off_G);
    double *T = (double *)(base + L.off_T);
    const int64_t ldw = n;
    const int ew = CX ? 2 : 1;
    BDG_HIP(hipMemsetAsync(u, 0, 16 * 2 * NB, s));
    for (int64_t p = 0; p < L.np; ++p) {
        const int64_t k = p * NB;
        const int nb = (int)std::min<int64_t>(NB, n - 1 - k);
        BDG_HIP(hipMemsetAsync(VW, 0, 8 * ew * (size_t)n * 2 * NB, s));
        BDG_HIP(hipMemsetAsync(WV, 0, 8 * ew * (size_t)n * 2 * NB, s));
        for (int j = 0; j < nb; ++j) {
            const int64_t c = k + j;
            const int64_t rows = n - c;
            const int nparts = (int)((rows + CB - 1) / CB);
            hipLaunchKernelGGL((col_update<CX>), dim3(nparts), dim3(CB), 0, s, n, c, j, A, lda, VW, ldw, part);
            hipLaunchKernelGGL((reflector<CX>), dim3(1), dim3(CB), 0, s, n, c, A, lda, part, nparts, d, e, tau,
                               scal);
            const int64_t rs = n - (k + 1);
            const unsigned gs = (unsigned)std::min<int64_t>(1024, (rs + CB - 1) / CB);
            hipLaunchKernelGGL((scale_v<CX>), dim3(gs), dim3(CB), 0, s, n, c, k, j, A, lda, scal, VW, WV, ldw);
            if (j > 0)
                hipLaunchKernelGGL((panel_dots<CX>), dim3(2 * j), dim3(CB), 0, s, n, c, j, VW, ldw, u);
            const int64_t mt = n - c - 1;
            const int nt = (int)((mt + HT - 1) / HT);
            const int maxq = (nt + HCH - 1) / HCH;
            hipLaunchKernelGGL((hemv_tiles<CX>), dim3(nt, maxq), dim3(64 * HW), 0, s, mt,
                               A + ew * ((c + 1) + (c + 1) * lda), lda, VW + ew * ((c + 1) + (int64_t)j * ldw),
                               P1, P2, maxq);
            const int nw = nt;  // one workgroup per 64-row tile
            hipLaunchKernelGGL((finish_w<CX>), dim3(nw), dim3(64 * HW), 0, s, n, c, j, tau, u, VW, ldw, P1, P2,
                               maxq, part);
            hipLaunchKernelGGL((fix_w<CX>), dim3(gs), dim3(CB), 0, s, n, c, k, j, tau, part, nw, VW, WV, ldw);
            BDG_CHECK_LAUNCH();
        }
        // T factor of the panel: G = V^H V over rows k+1 .. n-1
        {
            const int64_t mr = n - k - 1;
            GemmArgs g{nb, nb, mr, 1.0, 0.0, 0.0, 0.0, VW + ew * (k + 1), ldw, VW + ew * (k + 1), ldw, G, nb,
                       GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<double, CX>('C', 'N', g, s)));
            hipLaunchKernelGGL((tfactor<CX>), dim3(1), dim3(NB), 0, s, nb, G, tau + 2 * k, T + ew * p * NB * NB);
            BDG_CHECK_LAUNCH();
        }
        // trailing update A[k+nb:, k+nb:] -= [V W] [W V]^H, lower tiles
        const int64_t k2 = k + nb;
        if (k2 < n) {
            const int64_t mr = n - k2;
            // the buffers hold NB columns of V, then NB of W: pass K = 2 NB
            // (the unused columns are zero)
            GemmArgs g{mr, mr, 2 * NB, -1.0, 0.0, 1.0, 0.0, VW + ew * k2, ldw, WV + ew * k2, ldw,
                       A + ew * (k2 + k2 * lda), lda, GEMM_LOWER, 1, nullptr};
            BDG_TRY((gemm<double, CX>('N', 'C', g, s)));
        }
    }
    hipLaunchKernelGGL((last_diag<CX>), dim3(1), dim3(64), 0, s, n, A, lda, d);
    BDG_CHECK_LAUNCH();
    return 0;
}

// Z <- Q Z with the reflectors left in A (explicit unit lower trapezoids)
template <bool CX>
int trd_back_t(int64_t n, int64_t m, const double *A, int64_t lda, const L1 &L, char *base, double *Z,
               int64_t ldz, hipStream_t s) {
    const int ew = CX ? 2 : 1;
    const double *T = (const double *)(base + L.off_T);
    double *W1 = (double *)(base + L.off_sc);
    double *W2 = W1 + ew * (size_t)NB * m;
    for (int64_t p = L.np - 1; p >= 0; --p) {
        const int64_t k = p * NB;
        const int nb = (int)std::min<int64_t>(NB, n - 1 - k);
        const int64_t mr = n - k - 1;
        const double *V = A + ew * ((k + 1) + k * lda);
        double *Zs = Z + ew * (k + 1);
        {   // W1 = V^H Z
            GemmArgs g{nb, m, mr, 1.0, 0.0, 0.0, 0.0, V, lda, Zs, ldz, W1, nb, GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<double, CX>('C', 'N', g, s)));
        }
        {   // W2 = T W1
            GemmArgs g{nb, m, nb, 1.0, 0.0, 0.0, 0.0, T + ew * p * NB * NB, nb, W1, nb, W2, nb, GEMM_FULL, 1,
                       nullptr};
            BDG_TRY((gemm<double, CX>('N', 'N', g, s)));
        }
        {   // Z -= V W2
            GemmArgs g{mr, m, nb, -1.0, 0.0, 1.0, 0.0, V, lda, W2, nb, Zs, ldz, GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<double, CX>('N', 'N', g, s)));
        }
    }
    return 0;
}

}  // namespace

size_t eigh1_workspace(int64_t n, bool cx, int64_t zcols) { return layout1(n, cx, zcols).total; }

int eigh1(int64_t n, bool cx, double *A, int64_t lda, double emin, double emax, double *W, double *Z,
          int64_t ldz, int64_t zcols, int64_t *m_out, void *work, bdg_err_report *report, hipStream_t s) {
    const L1 L = layout1(n, cx, zcols);
    char *base = (char *)work;
    double *d = (double *)(base + L.off_d);
    double *e = (double *)(base + L.off_e);
    double *Wv = (double *)(base + L.off_Wv);
    double *Q = (double *)(base + L.off_Q);
    void *sc = base + L.off_sc;
    hipEvent_t ev[5];
    for (int i = 0; i < 5; ++i) BDG_HIP(hipEventCreate(&ev[i]));
    struct Guard {
        hipEvent_t *e;
        ~Guard() {
            for (int i = 0; i < 5; ++i) (void)hipEventDestroy(e[i]);
        }
    } guard{ev};
    BDG_HIP(hipEventRecord(ev[0], s));
    if (cx) BDG_TRY(trd_t<true>(n, A, lda, L, base, s));
    else BDG_TRY(trd_t<false>(n, A, lda, L, base, s));
    BDG_HIP(hipEventRecord(ev[1], s));
    BDG_TRY(stedc(n, d, e, Wv, Q, n, sc, s, 32));
    BDG_HIP(hipEventRecord(ev[2], s));
    std::vector<double> wh((size_t)n);
    BDG_HIP(hipMemcpyAsync(wh.data(), Wv, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    const int64_t i0 = std::lower_bound(wh.begin(), wh.end(), emin) - wh.begin();
    const int64_t i1 = std::upper_bound(wh.begin(), wh.end(), emax) - wh.begin();
    const int64_t m = std::max<int64_t>(0, i1 - i0);
    *m_out = m;
    if (m > zcols) {
        set_error("bdg_eigh1: %lld eigenpairs in the window exceed zcols = %lld", (long long)m, (long long)zcols);
        return BDG_ERR_WORKSPACE;
    }
    if (m > 0) {
        BDG_HIP(hipMemcpyAsync(W, Wv + i0, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
        if (cx) hipLaunchKernelGGL((widen_cols<true>), dim3((unsigned)m), dim3(256), 0, s, n, Q, i0, Z, ldz);
        else hipLaunchKernelGGL((widen_cols<false>), dim3((unsigned)m), dim3(256), 0, s, n, Q, i0, Z, ldz);
        BDG_CHECK_LAUNCH();
    }
    BDG_HIP(hipEventRecord(ev[3], s));
    if (m > 0) {
        if (cx) BDG_TRY(trd_back_t<true>(n, m, A, lda, L, base, Z, ldz, s));
        else BDG_TRY(trd_back_t<false>(n, m, A, lda, L, base, Z, ldz, s));
    }
    BDG_HIP(hipEventRecord(ev[4], s));
    BDG_HIP(hipStreamSynchronize(s));
    if (report) {
        memset(report, 0, sizeof(*report));
        float t = 0.f;
        auto ms = [&](int a, int b) { return hipEventElapsedTime(&t, ev[a], ev[b]) == hipSuccess ? (double)t : 0.0; };
        report->stage_ms[0] = ms(0, 1);  // tridiagonalisation
        report->stage_ms[2] = ms(1, 2);  // divide and conquer
        report->stage_ms[6] = ms(2, 3);  // window
        report->stage_ms[4] = ms(3, 4);  // back-transformation
        report->stage_ms[7] = ms(0, 4);
    }
    return 0;
}

}  // namespace bdg
