// Stage 2 of the two-stage reduction: Hermitian band -> real tridiagonal.
//
// Second step of the 2-stage solver ("then transforming the banded matrix
// into a tridiagonal form", paper sec. "Performance of the Matrix
// Diagonalization Algorithm"), by bulge chasing.  Sweep s removes column s
// below the sub-diagonal; its task t works on the index range
//   C = [r0 - b, r0), R = [r0, min(n, r0 + b)),  r0 = s + 1 + t b:
//   t = 0 : reflector H_0 on rows s+1.. zeroes A[s+2:s+1+b, s]; two-sided on A[R, R].
//   t >= 1: A[R, C] <- A[R, C] H_{t-1} (creates the bulge); reflector H_t zeroes
//           A[r0+1:, r0-b] (first bulge column); A[R, C] <- H_t^H A[R, C];
//           two-sided on A[R, R].
// Consecutive sweeps lag by two tasks: task t of sweep s+1 reads and writes
// entries with row and column <= i* = s+1+(t+1)b, which task t+1 of sweep s
// finished, while task t+2 of sweep s only touches rows >= i* + b.  One launch
// executes every (s, t) with t = g - 2 s, so the kernel boundary orders the
// dependent tasks and no in-kernel waits are needed.
//
// The band lives in lower band storage AB[(i - j) + j ldab] (ldab >= 2b + 2
// holds the bulge).  Reflector (s, t) is stored with v_0 = 1 (length b, zero
// padded) at V2 + b * (voff[s] + t), its scale at tau2[voff[s] + t].  On exit
// d = real diag, e = complex sub-diagonal (phase scaled later).
#include "stages.h"

namespace bdg {
namespace {

constexpr int BMAX = 64;
constexpr int LDS = BMAX + 1;
constexpr int LAG = 2;  // task t of sweep s runs in step t + LAG s


// Offset of sweep s's first reflector, sum over s' < s of T_s' with
// T_s = (n - 2 - s) / b + 1, in closed form: with m = n - 2 and
// P(N) = sum_{j <= N} floor(j / b), it is s + P(m) - P(m - s).  Computed in
// the kernel so that loading the previous reflector waits on no other load.
__host__ __device__ inline int64_t sweep_offset(int64_t n, int b, int64_t s) {
    auto P = [b](int64_t N) {
        const int64_t q = N / b, r = N - q * b;
        return (int64_t)b * q * (q - 1) / 2 + q * (r + 1);
    };
    return s + P(n - 2) - P(n - 2 - s);
}

// Sum over each group of G consecutive lanes (G = 4, 8 or 16), to all of them.
template <int G, typename T>
__device__ inline T group_sum(T v) {
    v = dpp_fold<0xB1, 0xf>(v);                   // quad_perm [1, 0, 3, 2]
    v = dpp_fold<0x4E, 0xf>(v);                   // quad_perm [2, 3, 0, 1]
    if (G >= 8) v = dpp_fold<0x141, 0xf>(v);      // row_half_mirror
    if (G == 16) v = dpp_fold<0x140, 0xf>(v);     // row_mirror
    return v;
}

// One task per workgroup of NT threads; BT (16, 32 or 64) bounds the band
// width b so that every loop has a fixed trip count.  All global loads are
// issued at once, the reflector scalars are computed by every thread (no
// broadcast step), and the task takes four block barriers.  A task is a chain
// of dependent latencies (loads, two matrix-vector products, the update and
// its stores) that no other task can hide: at band 64, 512 threads (eight
// elements each) take 10 % less time per step than 256, and 1024 threads
// take 4 % more than 256.
template <typename F, int BT, int NT>
__global__ __launch_bounds__(NT) void hb2st_step(int64_t n, int b, F *__restrict__ AB, int64_t ldab,
                                                 F *__restrict__ V2, F *__restrict__ tau2, int64_t g,
                                                 int64_t s_lo) {
    typedef typename v2t<F>::type CV;
    constexpr int NE = BT * BT / NT;  // matrix elements per thread
    constexpr int NW = NT / 64;       // waves
    constexpr int TPR = NT / 64;      // threads per row in the matrix-vector products
    static_assert(NE >= 1 && BT % TPR == 0 && (TPR == 4 || TPR == 8 || TPR == 16), "hb2st: tile shape");
    constexpr int LD = BT + 1;
    // The Hermitian block D is handled through its stored lower triangle only:
    // entry p of the triangle lies in column pair j = p / (BT + 1) (columns j
    // and BT - 1 - j, BT + 1 entries together), so consecutive p are
    // consecutive rows of one column.
    constexpr int ND = BT / 2 * (BT + 1);
    constexpr int NED = (ND + NT - 1) / NT;
    __shared__ CV Bs[BT * LD];
    __shared__ CV Ds[BT * LD];
    __shared__ CV vp[BT], xv[BT], vn[BT], yv[BT], pv[BT], wb[BT];
    __shared__ F red[NW][4];
    const int64_t s = s_lo + blockIdx.x;
    const int64_t t = g - LAG * s;
    if (s > n - 3 || t < 0) return;
    const int64_t Ts = (n - 2 - s) / b + 1;
    if (t >= Ts) return;
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int64_t r0 = s + 1 + t * b;
    const int Lr = (int)min((int64_t)b, n - r0);
    const int64_t ridx = sweep_offset(n, b, s) + t;
    const int64_t c0 = r0 - b;
    const CV zero = mk2<F>(0.0, 0.0);

    // ---- phase 0: B = A[R, C] (t > 0), D = A[R, R] (full Hermitian), the
    // previous reflector (t > 0) or the column being removed (t = 0).
    // Unconditional loads (entry 0 outside the block), zeroed by select.
    CV rb[NE], rd[NED];
    auto dpos = [](int p, int &r, int &c) {
        const int j = p / (BT + 1), k = p - j * (BT + 1);
        if (k < BT - j) {
            c = j;
            r = j + k;
        } else {
            c = BT - 1 - j;
            r = c + (k - (BT - j));
        }
    };
    F tp = 0.0;
    {
        unsigned okb = 0, okd = 0;
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + NT * i;
            const int r = e % BT, c = e / BT;
            const bool ob = (t > 0) & (r < Lr) & (c < b);
            const int64_t offb = ob ? 2 * ((b + r - c) + (c0 + c) * ldab) : 0;
            rb[i] = ld2<F>(AB + offb);
            okb |= (unsigned)ob << i;
        }
#pragma unroll
        for (int i = 0; i < NED; ++i) {
            const int p = tid + NT * i;
            int r, c;
            dpos(p < ND ? p : 0, r, c);
            const bool od = (p < ND) & (r < Lr);
            const int64_t offd = od ? 2 * ((r - c) + (r0 + c) * ldab) : 0;
            rd[i] = ld2<F>(AB + offd);
            okd |= (unsigned)od << i;
        }
        const bool ov = (t > 0) & (tid < b);
        const bool ox = (t == 0) & (tid < Lr);
        const CV pv0 = ld2<F>(V2 + (ov ? 2 * ((ridx - 1) * b + tid) : 0));
        const CV xc0 = ld2<F>(AB + (ox ? 2 * ((1 + tid) + s * ldab) : 0));
        const F tp0 = tau2[t > 0 ? ridx - 1 : 0];
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + NT * i;
            const int r = e % BT, c = e / BT;
            if (!((okb >> i) & 1u)) rb[i] = zero;
            Bs[r + c * LD] = rb[i];
        }
#pragma unroll
        for (int i = 0; i < NED; ++i) {
            const int p = tid + NT * i;
            if (p >= ND) break;
            int r, c;
            dpos(p, r, c);
            if (!((okd >> i) & 1u)) rd[i] = zero;
            Ds[r + c * LD] = rd[i];
            if (r > c) Ds[c + r * LD] = mk2<F>(rd[i].x, -rd[i].y);  // upper: conj of the lower entry
        }
        if (tid < BT) {
            vp[tid] = sel2(ov, pv0, zero);
            xv[tid] = sel2(ox, xc0, zero);
        }
        tp = t > 0 ? tp0 : (F)0.0;
    }
    __syncthreads();

    // ---- phase 1: y = tp B vp and the first bulge column x = B[:, 0] - y
    // (vp_0 = 1) for t > 0; quads of threads per row.
    const int qr = tid / TPR, q = tid % TPR;
    CV yr = zero, xr = zero;
    {
        F sr = 0.0, si = 0.0;
        if (qr < BT) {
#pragma unroll
            for (int j = 0; j < BT / TPR; ++j) {
                const int c = q + TPR * j;
                const CV a = Bs[qr + c * LD], v = vp[c];
                sr += a.x * v.x - a.y * v.y;
                si += a.x * v.y + a.y * v.x;
            }
        }
        sr = group_sum<TPR>(sr);
        si = group_sum<TPR>(si);
        F n2 = 0.0;
        if (qr < BT) {
            yr = mk2<F>(tp * sr, tp * si);
            if (t > 0) {
                const CV a = Bs[qr];
                xr = sel2(qr < Lr, mk2<F>(a.x - yr.x, a.y - yr.y), zero);
            } else {
                xr = xv[qr];
            }
            if (q == 0 && qr > 0) n2 = xr.x * xr.x + xr.y * xr.y;
        }
        n2 = wave_sum_last(n2);
        if (qr < BT && q == 0) {
            yv[qr] = yr;
            if (t > 0) xv[qr] = xr;  // for t = 0, xv already holds x (read above)
        }
        if (l == 63) red[w][0] = n2;
    }
    __syncthreads();

    // ---- phase 2: reflector H = I - tau v v^H with H^H x = beta e_0 (every
    // thread computes the scalars), v = x / u_0 with v_0 = 1.
    F tj, ur, ui;
    CV beta;
    {
        F tail2 = 0.0;
#pragma unroll
        for (int k = 0; k < NW; ++k) tail2 += red[k][0];
        const CV x0 = xv[0];
        const F aa = sqrt(x0.x * x0.x + x0.y * x0.y);
        if (tail2 == 0.0) {
            tj = 0.0; ur = 0.0; ui = 0.0;
            beta = x0;
        } else {
            const F xn = sqrt(aa * aa + tail2);
            F sgr = 1.0, sgi = 0.0;
            if (aa > 0.0) { sgr = x0.x / aa; sgi = x0.y / aa; }
            const F den = aa + xn;
            ur = sgr / den;  // 1/u0 = conj(sgn)/(|a| + |x|)
            ui = -sgi / den;
            tj = den / xn;
            beta = mk2<F>(-sgr * xn, -sgi * xn);
        }
    }
    if (qr < BT && q == 0) {
        CV v;
        if (qr == 0) v = mk2<F>(1.0, 0.0);
        else if (qr < Lr && tj != 0.0) v = mk2<F>(xr.x * ur - xr.y * ui, xr.x * ui + xr.y * ur);
        else v = zero;
        vn[qr] = v;
        if (qr < b) st2<F>(V2 + 2 * (ridx * b + qr), v);
    }
    if (tid == 0) tau2[ridx] = tj;
    __syncthreads();
    if (tj == 0.0) {
        // H = I: only the right update of B remains (t > 0)
        if (t > 0) {
#pragma unroll
            for (int i = 0; i < NE; ++i) {
                const int e = tid + NT * i;
                const int r = e % BT, c = e / BT;
                if (r >= Lr || c >= b) continue;
                CV a = rb[i];
                const CV vpc = vp[c], y = yv[r];
                a.x -= y.x * vpc.x + y.y * vpc.y;
                a.y -= y.y * vpc.x - y.x * vpc.y;
                st2<F>(AB + 2 * ((b + r - c) + (c0 + c) * ldab), a);
            }
        }
        return;
    }

    // ---- phase 3: p = tau D v (rows), wB = v^H B (columns, t > 0),
    // K = (tau/2) v^H p and gamma = v^H y.
    {
        F pr = 0.0, pi = 0.0, wr = 0.0, wi = 0.0;
        if (qr < BT) {
#pragma unroll
            for (int j = 0; j < BT / TPR; ++j) {
                const int c = q + TPR * j;
                const CV a = Ds[qr + c * LD], v = vn[c];
                pr += a.x * v.x - a.y * v.y;
                pi += a.x * v.y + a.y * v.x;
            }
            if (t > 0) {
#pragma unroll
                for (int j = 0; j < BT / TPR; ++j) {
                    const int r = q + TPR * j;
                    const CV v = vn[r], a = Bs[r + qr * LD];
                    wr += v.x * a.x + v.y * a.y;
                    wi += v.x * a.y - v.y * a.x;
                }
            }
        }
        pr = group_sum<TPR>(pr);
        pi = group_sum<TPR>(pi);
        wr = group_sum<TPR>(wr);
        wi = group_sum<TPR>(wi);
        F kr = 0.0, ki = 0.0, gr = 0.0, gi = 0.0;
        if (qr < BT && q == 0) {
            const CV p = mk2<F>(tj * pr, tj * pi);
            pv[qr] = p;
            wb[qr] = mk2<F>(wr, wi);
            const CV v = vn[qr];
            kr = v.x * p.x + v.y * p.y;
            ki = v.x * p.y - v.y * p.x;
            gr = v.x * yr.x + v.y * yr.y;
            gi = v.x * yr.y - v.y * yr.x;
        }
        kr = wave_sum_last(kr);
        ki = wave_sum_last(ki);
        gr = wave_sum_last(gr);
        gi = wave_sum_last(gi);
        if (l == 63) { red[w][0] = kr; red[w][1] = ki; red[w][2] = gr; red[w][3] = gi; }
    }
    __syncthreads();

    // ---- phase 4: write B (t > 0) or the removed column (t = 0), and D
    F Kr = 0.0, Ki = 0.0, gmr = 0.0, gmi = 0.0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        Kr += red[k][0];
        Ki += red[k][1];
        gmr += red[k][2];
        gmi += red[k][3];
    }
    Kr *= 0.5 * tj;
    Ki *= 0.5 * tj;
    if (t > 0) {
#pragma unroll
        for (int i = 0; i < NE; ++i) {
            const int e = tid + NT * i;
            const int r = e % BT, c = e / BT;
            if (r >= Lr || c >= b) continue;
            CV a;
            if (c == 0) {
                a = sel2(r == 0, beta, zero);
            } else {
                a = rb[i];
                const CV vpc = vp[c], y = yv[r];
                // right update: - y conj(vp_c)
                a.x -= y.x * vpc.x + y.y * vpc.y;
                a.y -= y.y * vpc.x - y.x * vpc.y;
                // left update: - tau v_r (wB_c - gamma conj(vp_c)),  gamma = v^H y (y holds tp)
                const CV wbc = wb[c];
                const F qre = wbc.x - (gmr * vpc.x + gmi * vpc.y);
                const F qim = wbc.y - (gmi * vpc.x - gmr * vpc.y);
                const CV v = vn[r];
                a.x -= tj * (v.x * qre - v.y * qim);
                a.y -= tj * (v.x * qim + v.y * qre);
            }
            st2<F>(AB + 2 * ((b + r - c) + (c0 + c) * ldab), a);
        }
    } else if (tid < Lr) {
        st2<F>(AB + 2 * ((1 + tid) + s * ldab), sel2(tid == 0, beta, zero));
    }
#pragma unroll
    for (int i = 0; i < NED; ++i) {
        const int p = tid + NT * i;
        if (p >= ND) break;
        int r, c;
        dpos(p, r, c);
        if (r >= Lr) continue;
        const CV vr = vn[r], vc = vn[c], pr = pv[r], pc = pv[c];
        const CV wr = mk2<F>(pr.x - (Kr * vr.x - Ki * vr.y), pr.y - (Kr * vr.y + Ki * vr.x));
        const CV wc = mk2<F>(pc.x - (Kr * vc.x - Ki * vc.y), pc.y - (Kr * vc.y + Ki * vc.x));
        CV a = rd[i];
        a.x -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
        a.y -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
        if (r == c) a.y = 0.0;
        st2<F>(AB + 2 * ((r - c) + (r0 + c) * ldab), a);
    }
}

template <typename F>
__global__ void hb2st_extract(int64_t n, const F *__restrict__ AB, int64_t ldab,
                              double *__restrict__ d, double *__restrict__ e_cplx) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        d[i] = AB[2 * (i * ldab)];
        if (i + 1 < n) {
            e_cplx[2 * i] = AB[2 * (1 + i * ldab)];
            e_cplx[2 * i + 1] = AB[2 * (1 + i * ldab) + 1];
        }
    }
}

}  // namespace

int64_t hb2st_nrefl(int64_t n, int b) {
    int64_t tot = 0;
    for (int64_t s = 0; s <= n - 3; ++s) tot += (n - 2 - s) / b + 1;
    return tot;
}

void hb2st_offsets(int64_t n, int b, int64_t *voff_host) {
    int64_t tot = 0;
    for (int64_t s = 0; s <= n - 3; ++s) {
        voff_host[s] = tot;
        tot += (n - 2 - s) / b + 1;
    }
}

template <typename F>
int hb2st_t(int64_t n, int b, F *AB, int64_t ldab, F *V2, F *tau2, double *d, double *e_cplx,
            hipStream_t s) {
    if (b > BMAX) {
        set_error("hb2st: band %d > %d", b, BMAX);
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    if (n >= 3) {
        const int64_t nsw = n - 2;  // sweeps 0 .. n-3
        const int64_t T0 = (n - 2) / b + 1;
        const int64_t gmax = LAG * (nsw - 1) + T0;  // last step index + 1 upper bound
        int64_t s_lo = 0;
        for (int64_t g = 0; g < gmax; ++g) {
            // smallest sweep still active at step g: g - LAG s < T_s
            while (s_lo < nsw && g - LAG * s_lo >= (n - 2 - s_lo) / b + 1) ++s_lo;
            if (s_lo >= nsw) break;
            int64_t s_hi = g / LAG;
            if (s_hi > nsw - 1) s_hi = nsw - 1;
            if (s_hi < s_lo) continue;
            const dim3 grid((unsigned)(s_hi - s_lo + 1));
            if (b <= 16)
                hipLaunchKernelGGL((hb2st_step<F, 16, 256>), grid, dim3(256), 0, s, n, b, AB, ldab, V2, tau2, g, s_lo);
            else if (b <= 32)
                hipLaunchKernelGGL((hb2st_step<F, 32, 256>), grid, dim3(256), 0, s, n, b, AB, ldab, V2, tau2, g, s_lo);
            else
                hipLaunchKernelGGL((hb2st_step<F, 64, 512>), grid, dim3(512), 0, s, n, b, AB, ldab, V2, tau2, g, s_lo);
        }
        BDG_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL((hb2st_extract<F>), dim3((unsigned)((n + 255) / 256 > 1024 ? 1024 : (n + 255) / 256)),
                       dim3(256), 0, s, n, AB, ldab, d, e_cplx);
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace bdg

namespace bdg {

int hb2st(int64_t n, int b, double *AB, int64_t ldab, double *V2, double *tau2, double *d,
          double *e_cplx, hipStream_t s) {
    return hb2st_t<double>(n, b, AB, ldab, V2, tau2, d, e_cplx, s);
}
int hb2st(int64_t n, int b, float *AB, int64_t ldab, float *V2, float *tau2, double *d,
          double *e_cplx, hipStream_t s) {
    return hb2st_t<float>(n, b, AB, ldab, V2, tau2, d, e_cplx, s);
}

}  // namespace bdg
