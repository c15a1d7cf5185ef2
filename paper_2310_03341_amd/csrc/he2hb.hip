// Stage 1 of the two-stage reduction: Hermitian dense -> Hermitian band.
//
// First step of the 2-stage solver ("first transforming the dense matrix in a
// banded matrix", paper sec. "Performance of the Matrix Diagonalization
// Algorithm").  For each panel of b columns starting at k:
//   P = A[k+b:n, k:k+b] = Q R          (Householder QR, Q = I - V T V^H)
//   A22 = A[k+b:n, k+b:n] <- Q^H A22 Q = A22 - V W^H - W V^H,
//   with X = A22 V T, W = X - 1/2 V (T^H V^H X).
// R lands on the b-th sub-diagonal band; V (unit lower trapezoidal, stored
// explicitly with its zeros and ones) stays in A's panel for the
// back-transformation; T is kept per panel.
//
// The panel QR runs one column per launch over many workgroups (each owns a
// chunk of rows); a launch applies reflector j and, in the same pass, forms
// the partial norms and inner products that define reflector j+1.  All the
// O(n^3) work (HEMM, HER2K and small GEMMs) goes through the MFMA tile kernel.
#include <mutex>

#include "gemm.h"
#include "stages.h"

namespace bdg {

// One non-blocking side stream per device (default priority), created on first
// use and kept for the life of the process: stage 1's look-ahead panels, and
// the phase scan that runs beside the divide and conquer.
hipStream_t side_stream() {
    static std::mutex mu;
    static hipStream_t st[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!st[dev] && hipStreamCreateWithFlags(&st[dev], hipStreamNonBlocking) != hipSuccess) st[dev] = nullptr;
    return st[dev];
}

namespace {

constexpr int PQ_ROWS = 256;  // rows per workgroup in the panel kernels

struct Events {
    hipEvent_t upd = nullptr, panel = nullptr;
    bool ok = false;
    Events() {
        ok = hipEventCreateWithFlags(&upd, hipEventDisableTiming) == hipSuccess &&
             hipEventCreateWithFlags(&panel, hipEventDisableTiming) == hipSuccess;
    }
    ~Events() {
        if (upd) (void)hipEventDestroy(upd);
        if (panel) (void)hipEventDestroy(panel);
    }
};
constexpr int MAXB = 64;      // largest supported band
constexpr int PCH = 32;       // panel columns per load batch in a column step

// Partials layout per workgroup: [0..nb) complex s_c, [nb] (tail2, 0).
template <typename F>
__device__ inline void reduce_partials(const F *__restrict__ part, int G, int nb,
                                       F *__restrict__ s_sh /* 2*(nb+1) */) {
    // 4 threads per column (256 threads)
    typedef typename v2t<F>::type CV;
    __shared__ F tmp[4][2 * (MAXB + 1)];
    const int t = threadIdx.x;
    for (int col = t & 63; col <= nb; col += 64) {
        const int g0 = t >> 6;
        F re = 0.0, im = 0.0;
        // eight loads in flight per round (entry of workgroup 0 past the end,
        // dropped by the select), so the sum does not wait on each in turn
        for (int gb = g0; gb < G; gb += 32) {
            CV v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int g = gb + 4 * u;
                v[u] = ld2<F>(part + (size_t)(g < G ? g : 0) * 2 * (nb + 1) + 2 * col);
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (gb + 4 * u < G) {
                    re += v[u].x;
                    im += v[u].y;
                }
        }
        tmp[g0][2 * col] = re;
        tmp[g0][2 * col + 1] = im;
    }
    __syncthreads();
    for (int col = t; col <= nb; col += blockDim.x) {
        F re = 0.0, im = 0.0;
        for (int g = 0; g < 4; ++g) {
            re += tmp[g][2 * col];
            im += tmp[g][2 * col + 1];
        }
        s_sh[2 * col] = re;
        s_sh[2 * col + 1] = im;
    }
    __syncthreads();
}

// One column step of the panel QR.
//   j >= 0: apply reflector j (from partials in part_in / row_in) to the panel.
//   j+1 < ncol: write partials for column j+1 to part_out / row_out.
template <typename F>
__global__ __launch_bounds__(256) void panel_step(F *__restrict__ P, int64_t ld, int64_t mr,
                                                  int nb, int j, int ncol,
                                                  const F *__restrict__ part_in,
                                                  const F *__restrict__ row_in,
                                                  F *__restrict__ part_out,
                                                  F *__restrict__ row_out,
                                                  F *__restrict__ tau, int G) {
    typedef typename v2t<F>::type CV;
    __shared__ F s_sh[2 * (MAXB + 1)];
    __shared__ F wc[2 * MAXB];
    __shared__ F red[4][2 * (MAXB + 1)];
    __shared__ F sc[6];  // u0inv (re, im), tau, beta (re, im), active
    const int t = threadIdx.x;
    const int64_t r = (int64_t)blockIdx.x * PQ_ROWS + t;  // panel row of this thread
    const bool have = r < mr;

    if (j >= 0) {
        reduce_partials<F>(part_in, G, nb, s_sh);
        if (t == 0) {
            const F ar = row_in[2 * j], ai = row_in[2 * j + 1];
            const F tail2 = s_sh[2 * nb];
            const F aa = sqrt(ar * ar + ai * ai);
            if (tail2 == 0.0) {
                sc[0] = 0.0; sc[1] = 0.0; sc[2] = 0.0; sc[3] = ar; sc[4] = ai; sc[5] = 0.0;
            } else {
                const F xn = sqrt(aa * aa + tail2);
                F sr = 1.0, si = 0.0;
                if (aa > 0.0) { sr = ar / aa; si = ai / aa; }
                const F br = -sr * xn, bi = -si * xn;
                // u0 = alpha - beta = sgn (|alpha| + xn); 1/u0 = conj(sgn) / (|alpha| + xn)
                const F den = aa + xn;
                sc[0] = sr / den;
                sc[1] = -si / den;
                sc[2] = den / xn;  // tau
                sc[3] = br;
                sc[4] = bi;
                sc[5] = 1.0;
            }
        }
        __syncthreads();
    }
    const F tj = j >= 0 ? sc[2] : 0.0;
    const F ur = j >= 0 ? sc[0] : 0.0, ui = j >= 0 ? sc[1] : 0.0;
    const bool upd = j >= 0 && sc[5] != 0.0;  // uniform: a reflector to apply
    if (j >= 0 && blockIdx.x == 0 && t == 0) tau[j] = tj;
    if (upd) {
        // w_c = (s_c - conj(beta) P[j,c]) / conj(u0), scaled by tau: tw_c = tau * w_c
        const F br = sc[3], bi = sc[4];
        for (int c = j + 1 + t; c < nb; c += blockDim.x) {
            const F sr = s_sh[2 * c], si = s_sh[2 * c + 1];
            const F pr = row_in[2 * c], pi = row_in[2 * c + 1];
            // s - conj(beta) * p
            const F nr = sr - (br * pr + bi * pi);
            const F ni = si - (br * pi - bi * pr);
            // / conj(u0) == * conj(1/u0)   (1/conj(u0) = conj(1/u0))
            const F cr = ur, ci = -ui;
            wc[2 * c] = tj * (nr * cr - ni * ci);
            wc[2 * c + 1] = tj * (nr * ci + ni * cr);
        }
        __syncthreads();
    }
    const int jn = j + 1;
    const bool part = jn < ncol;  // uniform: partials for column jn wanted
    if (!upd && !part) return;
    // One pass over this thread's panel row: apply reflector j to columns
    // > j, then form the partials of column jn from the updated values while
    // they are still in registers.
    const bool rowupd = upd && have && r >= j;
    const bool in = part && have && r >= jn;
    F vr = 0.0, vi = 0.0;
    if (rowupd) {
        // v_r: 1 at r == j, x_r / u0 below
        F *pj = P + 2 * (r + (int64_t)j * ld);
        if (r == j) {
            vr = 1.0;
            pj[0] = sc[3];
            pj[1] = sc[4];
        } else {
            const F xr = pj[0], xi = pj[1];
            vr = xr * ur - xi * ui;
            vi = xr * ui + xi * ur;
            pj[0] = vr;
            pj[1] = vi;
        }
    }
    const bool need = rowupd || in;
    const int w = t >> 6, l = t & 63;
    F xr = 0.0, xi = 0.0;
    // columns in chunks of PCH: all loads of a chunk are issued first
    for (int c0 = jn; c0 < nb; c0 += PCH) {
        CV pv[PCH];
#pragma unroll
        for (int q = 0; q < PCH; ++q) {
            const int c = c0 + q;
            pv[q] = (need && c < nb) ? ld2<F>(P + 2 * (r + (int64_t)c * ld)) : mk2<F>(0.0, 0.0);
        }
        if (rowupd) {
#pragma unroll
            for (int q = 0; q < PCH; ++q) {
                const int c = c0 + q;
                if (c >= nb) break;
                const F wr = wc[2 * c], wi = wc[2 * c + 1];
                pv[q] = mk2<F>(pv[q].x - (vr * wr - vi * wi), pv[q].y - (vr * wi + vi * wr));
                st2<F>(P + 2 * (r + (int64_t)c * ld), pv[q]);
            }
        }
        if (part) {
            if (c0 == jn) {
                // column jn itself: x, and tail2 over r > jn
                xr = in ? pv[0].x : 0.0;
                xi = in ? pv[0].y : 0.0;
                F t2 = (in && r > jn) ? xr * xr + xi * xi : 0.0;
                t2 = wave_sum_last(t2);
                if (l == 63) { red[w][2 * nb] = t2; red[w][2 * nb + 1] = 0.0; }
            }
#pragma unroll
            for (int q = 0; q < PCH; ++q) {
                const int c = c0 + q;
                if (c >= nb) break;
                if (c == jn) continue;
                // conj(x) * p
                F sr = xr * pv[q].x + xi * pv[q].y, si = xr * pv[q].y - xi * pv[q].x;
                sr = wave_sum_last(sr);
                si = wave_sum_last(si);
                if (l == 63) { red[w][2 * c] = sr; red[w][2 * c + 1] = si; }
            }
        }
    }
    if (part) {
        __syncthreads();
        for (int c = t; c <= nb; c += blockDim.x) {
            F sr = 0.0, si = 0.0;
            if (c > jn) {
                for (int q = 0; q < 4; ++q) { sr += red[q][2 * c]; si += red[q][2 * c + 1]; }
            }
            part_out[(size_t)blockIdx.x * 2 * (nb + 1) + 2 * c] = sr;
            part_out[(size_t)blockIdx.x * 2 * (nb + 1) + 2 * c + 1] = si;
        }
        // the pivot row jn, copied by the workgroup that owns it (one thread per column)
        const int64_t rb = (int64_t)blockIdx.x * PQ_ROWS;
        if (jn >= rb && jn < rb + PQ_ROWS && t < nb)
            st2<F>(row_out + 2 * t, ld2<F>(P + 2 * (jn + (int64_t)t * ld)));
    }
}

// Copy the finished band columns [k, k+nb) into lower band storage AB: the
// diagonal block (rows < k+b) and R (rows k+b .. k+b+c of column k+c).
template <typename F>
__global__ void panel_band(const F *__restrict__ A, int64_t lda, int64_t n, int64_t k, int b,
                           F *__restrict__ AB, int64_t ldab) {
    const int c = blockIdx.y;
    const int64_t j = k + c;
    for (int64_t d = threadIdx.x; d < ldab; d += blockDim.x) {
        const int64_t i = j + d;
        F re = 0.0, im = 0.0;
        if (i < n && (i < k + b || i - (k + b) <= c)) {
            re = A[2 * (i + j * lda)];
            im = A[2 * (i + j * lda) + 1];
        }
        AB[2 * (d + j * ldab)] = re;
        AB[2 * (d + j * ldab) + 1] = im;
    }
}

// Write V explicitly (zeros above, ones on the diagonal) into the panel, into
// VW[:, 0:nb] and into WV[:, nb:2nb].
template <typename F>
__global__ void panel_explicit_v(F *__restrict__ A, int64_t lda, int64_t k, int b, int nb,
                                 int64_t mr, F *__restrict__ VW, F *__restrict__ WV,
                                 int64_t ldw) {
    const int c = blockIdx.y;
    const int64_t j = k + c;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < mr;
         r += (int64_t)gridDim.x * blockDim.x) {
        F *p = A + 2 * ((k + b + r) + j * lda);
        F vr, vi;
        if (r < c) { vr = 0.0; vi = 0.0; }
        else if (r == c) { vr = 1.0; vi = 0.0; }
        else { vr = p[0]; vi = p[1]; }
        p[0] = vr;
        p[1] = vi;
        VW[2 * (r + (int64_t)c * ldw)] = vr;
        VW[2 * (r + (int64_t)c * ldw) + 1] = vi;
        WV[2 * (r + (int64_t)(nb + c) * ldw)] = vr;
        WV[2 * (r + (int64_t)(nb + c) * ldw) + 1] = vi;
    }
}

// Band columns that need no reduction: copy lower band of A.
template <typename F>
__global__ void band_copy_tail(const F *__restrict__ A, int64_t lda, int64_t n, int64_t j0,
                               F *__restrict__ AB, int64_t ldab) {
    const int64_t j = j0 + blockIdx.y;
    for (int64_t d = threadIdx.x; d < ldab; d += blockDim.x) {
        const int64_t i = j + d;
        F re = 0.0, im = 0.0;
        if (i < n) {
            re = A[2 * (i + j * lda)];
            im = A[2 * (i + j * lda) + 1];
        }
        AB[2 * (d + j * ldab)] = re;
        AB[2 * (d + j * ldab) + 1] = im;
    }
}

// T from G = V^H V and tau: T[j][j] = tau_j, T[0:j, j] = -tau_j T[0:j,0:j] G[0:j, j].
// One workgroup; T upper triangular nb x nb (ld nb), zeros below.
template <typename F>
__global__ void tfactor(int nb, const F *__restrict__ G, const F *__restrict__ tau,
                        F *__restrict__ T) {
    __shared__ F Ts[2 * MAXB * MAXB];
    __shared__ F Gs[2 * MAXB * MAXB];
    __shared__ F taus[MAXB];
    const int t = threadIdx.x;
    for (int e = t; e < nb * nb; e += blockDim.x) {
        Ts[2 * e] = 0.0; Ts[2 * e + 1] = 0.0;
        Gs[2 * e] = G[2 * e]; Gs[2 * e + 1] = G[2 * e + 1];
    }
    for (int e = t; e < nb; e += blockDim.x) taus[e] = tau[e];
    __syncthreads();
    // T is the inverse of U = diag(1 / tau) + (strictly upper part of G), G =
    // V^H V: the same matrix the forward column recurrence builds.  Each quad
    // of lanes solves one column by back substitution,
    //   T[c, c] = tau_c,  T[i, c] = -tau_i sum_{k = i+1 .. c} G[i, k] T[k, c],
    // the four lanes taking every fourth k; the columns proceed independently
    // with no block barrier per step (a quad's lanes are in one wave, whose
    // LDS accesses complete in order).  A zero tau gives a zero row and
    // column, as in the recurrence.
    {
        const int c = t >> 2, q = t & 3;
        if (c < nb) {
            if (q == 0) {
                Ts[2 * (c + c * nb)] = taus[c];
                Ts[2 * (c + c * nb) + 1] = 0.0;
            }
            for (int i = c - 1; i >= 0; --i) {
                F sr = 0.0, si = 0.0;
                for (int k = i + 1 + q; k <= c; k += 4) {
                    const F gr = Gs[2 * (i + k * nb)], gi = Gs[2 * (i + k * nb) + 1];
                    const F xr = Ts[2 * (k + c * nb)], xi = Ts[2 * (k + c * nb) + 1];
                    sr += gr * xr - gi * xi;
                    si += gr * xi + gi * xr;
                }
                sr = quad_sum(sr);
                si = quad_sum(si);
                if (q == 0) {
                    const F ti = taus[i];
                    Ts[2 * (i + c * nb)] = -ti * sr;
                    Ts[2 * (i + c * nb) + 1] = -ti * si;
                }
            }
        }
    }
    __syncthreads();
    for (int e = t; e < nb * nb; e += blockDim.x) { T[2 * e] = Ts[2 * e]; T[2 * e + 1] = Ts[2 * e + 1]; }
}

template <typename F>
__global__ void copy_cols(const F *__restrict__ src, int64_t lds, F *__restrict__ dst,
                          int64_t ldd, int64_t rows) {
    const int c = blockIdx.y;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x) {
        dst[2 * (r + c * ldd)] = src[2 * (r + c * lds)];
        dst[2 * (r + c * ldd) + 1] = src[2 * (r + c * lds) + 1];
    }
}

int splitk_for(int64_t tiles, int64_t K) {
    // aim for >= 4096 workgroups (sixteen per CU, so the last round is
    // short), chunks of at least 512 along K
    int64_t s = (4096 + tiles - 1) / tiles;
    const int64_t kmax = (K + 511) / 512;
    if (s > kmax) s = kmax;
    if (s < 1) s = 1;
    if (s > 64) s = 64;
    return (int)s;
}

}  // namespace

// Most K chunks splitk_for gives a product whose K is at most n: the
// split-K partial buffers are sized for it.
static int64_t max_splits(int64_t n) { return std::max<int64_t>(1, std::min<int64_t>(64, (n + 511) / 512)); }

size_t he2hb_workspace(int64_t n, int b) {
    const size_t z = 16;
    size_t w = 0;
    w += z * (size_t)n * 2 * b * 2;              // VW, WV
    w += z * (size_t)n * b;                       // Y
    w += z * (size_t)b * b * 3;                   // G, S, M
    w += z * max_splits(n) * (size_t)n * b;      // split-K partials (upper bound)
    w += z * 2 * ((size_t)(n / PQ_ROWS + 2) * (b + 1) + b) * 2;  // panel partials + rows
    w += 8 * (size_t)b;                           // tau
    w += 4096;
    return w;
}

template <typename F>
int he2hb_t(int64_t n, F *A, int64_t lda, int b, F *AB, int64_t ldab, F *T1,
            void *work, hipStream_t s) {
    if (b < 1 || b > MAXB) {
        set_error("he2hb: band %d outside [1, %d]", b, MAXB);
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    if (ldab < 2 * b + 2) {
        set_error("he2hb: ldab %lld < 2b+2", (long long)ldab);
        return BDG_ERR_WORKSPACE;
    }
    char *wp = (char *)work;
    auto take = [&](size_t bytes) {
        char *p = wp;
        wp += (bytes + 255) / 256 * 256;
        return (F *)p;
    };
    const int64_t ldw = n;
    F *VW = take(16 * (size_t)n * 2 * b);
    F *WV = take(16 * (size_t)n * 2 * b);
    F *Y = take(16 * (size_t)n * b);
    F *Gm = take(16 * (size_t)b * b);
    F *Sm = take(16 * (size_t)b * b);
    F *Mm = take(16 * (size_t)b * b);
    F *part = take(16 * max_splits(n) * (size_t)n * b);
    const int64_t Gmax = n / PQ_ROWS + 2;
    F *ppart[2], *prow[2];
    ppart[0] = take(16 * (size_t)Gmax * (b + 1));
    ppart[1] = take(16 * (size_t)Gmax * (b + 1));
    prow[0] = take(16 * (size_t)b);
    prow[1] = take(16 * (size_t)b);
    F *tau = take(8 * (size_t)b);

    // QR of the panel below the band at column k (one launch per column)
    auto factor_panel = [&](int64_t kp, hipStream_t st) -> int {
        const int64_t mrp = n - kp - b;
        F *Pp = A + 2 * ((kp + b) + kp * lda);
        const int ncolp = (int)(mrp < b ? mrp : b);
        const int Gp = (int)((mrp + PQ_ROWS - 1) / PQ_ROWS);
        BDG_HIP(hipMemsetAsync(tau, 0, 8 * (size_t)b, st));
        for (int j = -1; j < ncolp; ++j) {
            const int ib = (j + 2) & 1;   // buffer read by step j
            const int ob = (j + 3) & 1;   // buffer written for column j+1
            hipLaunchKernelGGL((panel_step<F>), dim3(Gp), dim3(256), 0, st, Pp, lda, mrp, b, j, ncolp,
                               ppart[ib], prow[ib], ppart[ob], prow[ob], tau, Gp);
            BDG_CHECK_LAUNCH();
        }
        return 0;
    };
    // Look-ahead: once the trailing update has reached the next panel's
    // columns, that panel is factored on a second stream while the rest of
    // the trailing matrix is updated on the caller's stream (disjoint
    // columns).  Its reflectors, tau and T are consumed on the caller's
    // stream after an event wait.
    hipStream_t s2 = side_stream();
    Events ev;
    if (!s2 || !ev.ok) {
        set_error("he2hb: could not create the look-ahead stream or events");
        return BDG_ERR_HIP;
    }

    int64_t k = 0;
    int p = 0;
    if (k + b + 1 < n) BDG_TRY(factor_panel(0, s));
    for (; k + b + 1 < n; k += b, ++p) {
        const int nb = b;
        const int64_t mr = n - k - b;
        if (p > 0) BDG_HIP(hipStreamWaitEvent(s, ev.panel, 0));
        // band columns, then explicit V (overwrites R in A)
        hipLaunchKernelGGL((panel_band<F>), dim3(1, nb), dim3(256), 0, s, A, lda, n, k, b, AB, ldab);
        BDG_CHECK_LAUNCH();
        {
            int64_t gx = (mr + 255) / 256;
            if (gx > 16) gx = 16;
            hipLaunchKernelGGL((panel_explicit_v<F>), dim3((unsigned)gx, nb), dim3(256), 0, s, A, lda,
                               k, b, nb, mr, VW, WV, ldw);
            BDG_CHECK_LAUNCH();
        }
        F *T = T1 + 2 * (size_t)p * b * b;
        // G = V^H V
        {
            GemmArgs g{nb, nb, mr, 1.0, 0.0, 0.0, 0.0, VW, ldw, VW, ldw, Gm, nb, GEMM_FULL,
                       splitk_for(1, mr), part};
            BDG_TRY((gemm<F, true>('C', 'N', g, s)));
        }
        hipLaunchKernelGGL((tfactor<F>), dim3(1), dim3(256), 0, s, nb, Gm, tau, T);
        BDG_CHECK_LAUNCH();
        // Y = A22 V  (A22 Hermitian, lower triangle valid)
        F *A22 = A + 2 * ((k + b) + (k + b) * lda);
        {
            const int64_t tiles = (mr + 63) / 64;
            GemmArgs g{mr, nb, mr, 1.0, 0.0, 0.0, 0.0, A22, lda, VW, ldw, Y, ldw, GEMM_HEMM_L,
                       splitk_for(tiles, mr), part};
            BDG_TRY((gemm<F, true>('N', 'N', g, s)));
        }
        // X = Y T  -> VW[:, nb:2nb]
        F *X = VW + 2 * (size_t)nb * ldw;
        {
            GemmArgs g{mr, nb, nb, 1.0, 0.0, 0.0, 0.0, Y, ldw, T, nb, X, ldw, GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<F, true>('N', 'N', g, s)));
        }
        // S = V^H X
        {
            GemmArgs g{nb, nb, mr, 1.0, 0.0, 0.0, 0.0, VW, ldw, X, ldw, Sm, nb, GEMM_FULL,
                       splitk_for(1, mr), part};
            BDG_TRY((gemm<F, true>('C', 'N', g, s)));
        }
        // M = T^H S
        {
            GemmArgs g{nb, nb, nb, 1.0, 0.0, 0.0, 0.0, T, nb, Sm, nb, Mm, nb, GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<F, true>('C', 'N', g, s)));
        }
        // W = X - 1/2 V M  (in place in X)
        {
            GemmArgs g{mr, nb, nb, -0.5, 0.0, 1.0, 0.0, VW, ldw, Mm, nb, X, ldw, GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<F, true>('N', 'N', g, s)));
        }
        // WV[:, 0:nb] = W
        {
            dim3 grid((unsigned)(((mr + 255) / 256) > 16 ? 16 : (mr + 255) / 256), nb);
            hipLaunchKernelGGL((copy_cols<F>), grid, dim3(256), 0, s, X, ldw, WV, ldw, mr);
            BDG_CHECK_LAUNCH();
        }
        // A22 -= [V W] [W V]^H   (lower tiles)
        const bool ahead = lookahead() && (k + b) + b + 1 < n && mr > nb;
        if (ahead) {
            // the next panel's columns first (all rows), then that panel's QR
            // on the side stream, then the rest of A22
            GemmArgs ga{mr, nb, 2 * (int64_t)nb, -1.0, 0.0, 1.0, 0.0, VW, ldw, WV, ldw, A22, lda,
                        GEMM_FULL, 1, nullptr};
            BDG_TRY((gemm<F, true>('N', 'C', ga, s)));
            BDG_HIP(hipEventRecord(ev.upd, s));
            BDG_HIP(hipStreamWaitEvent(s2, ev.upd, 0));
            BDG_TRY(factor_panel(k + b, s2));
            BDG_HIP(hipEventRecord(ev.panel, s2));
            const int64_t mr2 = mr - nb;
            GemmArgs gb{mr2, mr2, 2 * (int64_t)nb, -1.0, 0.0, 1.0, 0.0, VW + 2 * nb, ldw, WV + 2 * nb, ldw,
                        A22 + 2 * (nb + (int64_t)nb * lda), lda, GEMM_LOWER, 1, nullptr};
            BDG_TRY((gemm<F, true>('N', 'C', gb, s)));
        } else {
            GemmArgs g{mr, mr, 2 * (int64_t)nb, -1.0, 0.0, 1.0, 0.0, VW, ldw, WV, ldw, A22, lda,
                       GEMM_LOWER, 1, nullptr};
            BDG_TRY((gemm<F, true>('N', 'C', g, s)));
            // the next panel (if any) is factored in order on this stream
            if ((k + b) + b + 1 < n) BDG_TRY(factor_panel(k + b, s));
        }
    }
    // remaining columns are already inside the band
    if (k < n) {
        dim3 grid(1, (unsigned)(n - k));
        hipLaunchKernelGGL((band_copy_tail<F>), grid, dim3(256), 0, s, A, lda, n, k, AB, ldab);
        BDG_CHECK_LAUNCH();
    }
    return 0;
}

int he2hb_panels(int64_t n, int b) {
    int p = 0;
    for (int64_t k = 0; k + b + 1 < n; k += b) ++p;
    return p;
}

}  // namespace bdg

namespace bdg {

// Back-transformation 1: Z <- Q1 Z = Q_0 Q_1 ... Q_last Z, Q_p = I - V_p T_p V_p^H
// acting on rows k_p + b .. n-1; V_p explicit in A's panel p.
//
// BT1_GROUP consecutive panels are applied as one block reflector
// Q_p0 ... Q_p0+g-1 = I - V T V^H, V = [V_p0 ... V_p0+g-1] (each shifted down by
// b rows per panel, zeros above), T from the recurrence
// T = [[T_a, -T_a (V_a^H V_c) T_c], [0, T_c]], so the three products per
// group have inner dimension g b instead of b.
constexpr int BT1_GROUP = 8;

template <typename F>
__global__ void bt1_gather_v(const F *__restrict__ A, int64_t lda, int64_t k0, int b, int64_t R,
                             F *__restrict__ Vg) {
    const int c = blockIdx.y;  // column of the group's V
    const int64_t j0 = (int64_t)(c / b) * b;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < R;
         r += (int64_t)gridDim.x * blockDim.x) {
        F vr = 0.0, vi = 0.0;
        if (r >= j0) {
            const F *p = A + 2 * ((k0 + b + r) + (k0 + c) * lda);
            vr = p[0];
            vi = p[1];
        }
        Vg[2 * (r + (int64_t)c * R)] = vr;
        Vg[2 * (r + (int64_t)c * R) + 1] = vi;
    }
}

// Tg (gb x gb) = block diagonal of the panels' T factors, zeros elsewhere
template <typename F>
__global__ void bt1_tinit(int gb, int b, const F *__restrict__ T1p, F *__restrict__ Tg) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < gb * gb; e += gridDim.x * blockDim.x) {
        const int i = e % gb, j = e / gb;
        F vr = 0.0, vi = 0.0;
        if (i / b == j / b) {
            const F *t = T1p + 2 * ((size_t)(i / b) * b * b + (i % b) + (size_t)(j % b) * b);
            vr = t[0];
            vi = t[1];
        }
        Tg[2 * e] = vr;
        Tg[2 * e + 1] = vi;
    }
}

template <typename F>
int bt1_t(int64_t n, int64_t m, const F *A, int64_t lda, int b, const F *T1, F *Z,
          int64_t ldz, void *work, hipStream_t s) {
    const int np = he2hb_panels(n, b);
    if (np == 0 || m <= 0) return 0;
    const int gmax = BT1_GROUP * b;
    F *W1 = (F *)work;                              // gb x m
    F *W2 = W1 + 2 * (size_t)gmax * m;              // gb x m
    F *G = W2 + 2 * (size_t)gmax * m;               // gb x gb
    F *Tg = G + 2 * (size_t)gmax * gmax;            // gb x gb
    F *X = Tg + 2 * (size_t)gmax * gmax;            // gb x b
    F *Vg = X + 2 * (size_t)gmax * b;               // R x gb
    F *Pk = Vg + 2 * (size_t)n * gmax;              // split-K partials of G (<= max_splits(n) gb x gb)
    const int ngroups = (np + BT1_GROUP - 1) / BT1_GROUP;
    for (int q = ngroups - 1; q >= 0; --q) {
        const int p0 = q * BT1_GROUP;
        const int g = std::min(BT1_GROUP, np - p0);
        const int gb = g * b;
        const int64_t k0 = (int64_t)p0 * b;
        const int64_t R = n - k0 - b;
        F *Zs = Z + 2 * (k0 + b);
        const unsigned gx = (unsigned)std::min<int64_t>((R + 255) / 256, 64);
        hipLaunchKernelGGL((bt1_gather_v<F>), dim3(gx, (unsigned)gb), dim3(256), 0, s, A, lda, k0, b, R, Vg);
        hipLaunchKernelGGL((bt1_tinit<F>), dim3((unsigned)((gb * gb + 255) / 256)), dim3(256), 0, s, gb, b,
                           T1 + 2 * (size_t)p0 * b * b, Tg);
        BDG_CHECK_LAUNCH();
        if (g > 1) {
            // only (gb / 64)^2 output tiles over a long K: split K to fill the chip
            const int64_t tg = (gb + 63) / 64;
            const int skg = splitk_for(tg * tg, R);
            GemmArgs gg{gb, gb, R, 1.0, 0.0, 0.0, 0.0, Vg, R, Vg, R, G, gb, GEMM_FULL, skg,
                        skg > 1 ? Pk : nullptr};
            BDG_TRY((gemm<F, true>('C', 'N', gg, s)));
            for (int c = 1; c < g; ++c) {
                const int cb = c * b;
                // X = G[0:cb, cb:cb+b] T_cc ;  T[0:cb, cb:cb+b] = -T[0:cb, 0:cb] X
                GemmArgs gx1{cb, b, b, 1.0, 0.0, 0.0, 0.0, G + 2 * (size_t)cb * gb, gb,
                             Tg + 2 * (cb + (size_t)cb * gb), gb, X, gmax, GEMM_FULL, 1, nullptr};
                BDG_TRY((gemm<F, true>('N', 'N', gx1, s)));
                GemmArgs gx2{cb, b, cb, -1.0, 0.0, 0.0, 0.0, Tg, gb, X, gmax, Tg + 2 * (size_t)cb * gb, gb,
                             GEMM_FULL, 1, nullptr};
                BDG_TRY((gemm<F, true>('N', 'N', gx2, s)));
            }
        }
        GemmArgs g1{gb, m, R, 1.0, 0.0, 0.0, 0.0, Vg, R, Zs, ldz, W1, gb, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<F, true>('C', 'N', g1, s)));
        GemmArgs g2{gb, m, gb, 1.0, 0.0, 0.0, 0.0, Tg, gb, W1, gb, W2, gb, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<F, true>('N', 'N', g2, s)));
        GemmArgs g3{R, m, gb, -1.0, 0.0, 1.0, 0.0, Vg, R, W2, gb, Zs, ldz, GEMM_FULL, 1, nullptr};
        BDG_TRY((gemm<F, true>('N', 'N', g3, s)));
    }
    return 0;
}

size_t bt1_workspace(int64_t n, int64_t m, int b) {
    const size_t gb = (size_t)BT1_GROUP * b;
    return 16 * (2 * gb * (size_t)m + 2 * gb * gb + gb * (size_t)b + gb * (size_t)n + max_splits(n) * gb * gb) +
           1024;
}

}  // namespace bdg

namespace bdg {

int he2hb(int64_t n, double *A, int64_t lda, int b, double *AB, int64_t ldab, double *T1,
          void *work, hipStream_t s) {
    return he2hb_t<double>(n, A, lda, b, AB, ldab, T1, work, s);
}
int he2hb(int64_t n, float *A, int64_t lda, int b, float *AB, int64_t ldab, float *T1,
          void *work, hipStream_t s) {
    return he2hb_t<float>(n, A, lda, b, AB, ldab, T1, work, s);
}
int bt1(int64_t n, int64_t m, const double *A, int64_t lda, int b, const double *T1, double *Z,
        int64_t ldz, void *work, hipStream_t s) {
    return bt1_t<double>(n, m, A, lda, b, T1, Z, ldz, work, s);
}
int bt1(int64_t n, int64_t m, const float *A, int64_t lda, int b, const float *T1, float *Z,
        int64_t ldz, void *work, hipStream_t s) {
    return bt1_t<float>(n, m, A, lda, b, T1, Z, ldz, work, s);
}

}  // namespace bdg
