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


template <typename F>
__global__ __launch_bounds__(256) void hb2st_step(int64_t n, int b, F *__restrict__ AB,
                                                  int64_t ldab, F *__restrict__ V2,
                                                  F *__restrict__ tau2,
                                                  const int64_t *__restrict__ voff, int64_t g,
                                                  int64_t s_lo) {
    typedef typename v2t<F>::type CV;
    __shared__ CV Bs[BMAX * LDS];
    __shared__ CV Ds[BMAX * LDS];
    __shared__ CV vp[BMAX], vn[BMAX], yv[BMAX], pv[BMAX], wb[BMAX];
    __shared__ F red[4][4];
    __shared__ F sc[8];
    const int64_t s = s_lo + blockIdx.x;
    const int64_t t = g - LAG * s;
    if (s > n - 3 || t < 0) return;
    const int64_t Ts = (n - 2 - s) / b + 1;
    if (t >= Ts) return;
    const int tid = threadIdx.x;
    const int w = tid >> 6, l = tid & 63;
    const int64_t r0 = s + 1 + t * b;
    const int Lr = (int)min((int64_t)b, n - r0);
    const int64_t ridx = voff[s] + t;
    const int64_t c0 = r0 - b;
    F tp = 0.0;

    // ---- phase 0: load B = A[R, C] (t > 0), D = A[R, R] (full Hermitian), previous v.
    // Fixed trip counts (64 x 64 tiles, 16 elements per thread) so that all
    // global loads are issued before their LDS stores.
    {
        CV rb[16], rd[16];
        // unconditional loads (entry 0 outside the block), zeroed by select:
        // guarded loads compile to branch + load + wait and run one by one
        unsigned okb = 0, okd = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            const int r = e & 63, c = e >> 6;
            const bool ob = (t > 0) & (r < Lr) & (c < b);
            const bool od = (r < Lr) & (c < Lr);
            const int64_t offb = ob ? 2 * ((b + r - c) + (c0 + c) * ldab) : 0;
            const int64_t offd = od ? 2 * (r >= c ? (r - c) + (r0 + c) * ldab : (c - r) + (r0 + r) * ldab) : 0;
            rb[i] = ld2<F>(AB + offb);
            rd[i] = ld2<F>(AB + offd);
            okb |= (unsigned)ob << i;
            okd |= (unsigned)od << i;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            const int r = e & 63, c = e >> 6;
            if (!((okb >> i) & 1u)) rb[i] = mk2<F>(0.0, 0.0);
            if (!((okd >> i) & 1u)) rd[i] = mk2<F>(0.0, 0.0);
            else if (r < c) rd[i].y = -rd[i].y;  // upper entry: conj of the stored lower one
        }
        if (t > 0) {
            if (tid < b) vp[tid] = ld2<F>(V2 + 2 * ((ridx - 1) * b + tid));
            tp = tau2[ridx - 1];
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            const int r = e & 63, c = e >> 6;
            Bs[r + c * LDS] = rb[i];
            Ds[r + c * LDS] = rd[i];
        }
    }
    __syncthreads();

    // ---- phase 1: y = tp * B vp  (row sums, 4 threads per row)
    if (t > 0) {
        for (int base = 0; base < Lr * 4; base += blockDim.x) {
            const int e = base + tid;
            const int r = e >> 2, q = e & 3;
            F yr = 0.0, yi = 0.0;
            if (r < Lr && tp != 0.0) {
                for (int c = q; c < b; c += 4) {
                    const CV a = Bs[r + c * LDS], v = vp[c];
                    yr += a.x * v.x - a.y * v.y;
                    yi += a.x * v.y + a.y * v.x;
                }
            }
            yr += __shfl_xor(yr, 1, 64); yi += __shfl_xor(yi, 1, 64);
            yr += __shfl_xor(yr, 2, 64); yi += __shfl_xor(yi, 2, 64);
            if (r < Lr && q == 0) yv[r] = mk2<F>(tp * yr, tp * yi);
        }
        __syncthreads();
    }

    // ---- phase 2: x (first bulge column after the right update), reflector
    {
        F t2 = 0.0;
        for (int r = tid; r < Lr; r += blockDim.x) {
            CV x;
            if (t > 0) {
                const CV a = Bs[r], y = yv[r];
                x = mk2<F>(a.x - y.x, a.y - y.y);  // vp_0 = 1
            } else {
                x = ld2<F>(AB + 2 * ((1 + r) + s * ldab));
            }
            vn[r] = x;
            if (r > 0) t2 += x.x * x.x + x.y * x.y;
        }
        t2 = wave_sum(t2);
        if (l == 0) red[w][0] = t2;
        __syncthreads();
        if (tid == 0) {
            const F tail2 = red[0][0] + red[1][0] + red[2][0] + red[3][0];
            const F ar = vn[0].x, ai = vn[0].y;
            const F aa = sqrt(ar * ar + ai * ai);
            if (tail2 == 0.0) {
                sc[0] = 0.0; sc[1] = 0.0; sc[2] = 0.0; sc[3] = ar; sc[4] = ai;
            } else {
                const F xn = sqrt(aa * aa + tail2);
                F sr = 1.0, si = 0.0;
                if (aa > 0.0) { sr = ar / aa; si = ai / aa; }
                const F den = aa + xn;
                sc[0] = sr / den;     // 1/u0 = conj(sgn)/(|a| + |x|)
                sc[1] = -si / den;
                sc[2] = den / xn;     // tau
                sc[3] = -sr * xn;     // beta
                sc[4] = -si * xn;
            }
        }
        __syncthreads();
    }
    const F tj = sc[2];
    const CV beta = mk2<F>(sc[3], sc[4]);
    {
        const F ur = sc[0], ui = sc[1];
        CV vr0 = mk2<F>(0.0, 0.0);
        if (tid < b) {
            CV v;
            if (tid == 0) v = mk2<F>(1.0, 0.0);
            else if (tid < Lr && tj != 0.0) {
                const CV x = vn[tid];
                v = mk2<F>(x.x * ur - x.y * ui, x.x * ui + x.y * ur);
            } else v = mk2<F>(0.0, 0.0);
            vr0 = v;
            st2<F>(V2 + 2 * (ridx * b + tid), v);
        }
        if (tid == 0) tau2[ridx] = tj;
        __syncthreads();
        if (tid < b) vn[tid] = vr0;
        __syncthreads();
    }

    // ---- phase 3: wB = v^H B (column sums, original B), gamma = v^H y, p = tau D v
    if (tj != 0.0) {
        if (t > 0) {
            for (int base = 0; base < b * 4; base += blockDim.x) {
                const int e = base + tid;
                const int c = e >> 2, q = e & 3;
                F sr = 0.0, si = 0.0;
                if (c < b) {
                    for (int r = q; r < Lr; r += 4) {
                        const CV v = vn[r], a = Bs[r + c * LDS];
                        sr += v.x * a.x + v.y * a.y;
                        si += v.x * a.y - v.y * a.x;
                    }
                }
                sr += __shfl_xor(sr, 1, 64); si += __shfl_xor(si, 1, 64);
                sr += __shfl_xor(sr, 2, 64); si += __shfl_xor(si, 2, 64);
                if (c < b && q == 0) wb[c] = mk2<F>(sr, si);
            }
        }
        for (int base = 0; base < Lr * 4; base += blockDim.x) {
            const int e = base + tid;
            const int r = e >> 2, q = e & 3;
            F pr = 0.0, pi = 0.0;
            if (r < Lr) {
                for (int c = q; c < Lr; c += 4) {
                    const CV a = Ds[r + c * LDS], v = vn[c];
                    pr += a.x * v.x - a.y * v.y;
                    pi += a.x * v.y + a.y * v.x;
                }
            }
            pr += __shfl_xor(pr, 1, 64); pi += __shfl_xor(pi, 1, 64);
            pr += __shfl_xor(pr, 2, 64); pi += __shfl_xor(pi, 2, 64);
            if (r < Lr && q == 0) pv[r] = mk2<F>(tj * pr, tj * pi);
        }
        __syncthreads();
        // K = (tau/2) v^H p  and  gamma = v^H y
        F kr = 0.0, ki = 0.0, gr = 0.0, gi = 0.0;
        for (int r = tid; r < Lr; r += blockDim.x) {
            const CV v = vn[r], p = pv[r];
            kr += v.x * p.x + v.y * p.y;
            ki += v.x * p.y - v.y * p.x;
            if (t > 0) {
                const CV y = yv[r];
                gr += v.x * y.x + v.y * y.y;
                gi += v.x * y.y - v.y * y.x;
            }
        }
        kr = wave_sum(kr); ki = wave_sum(ki); gr = wave_sum(gr); gi = wave_sum(gi);
        if (l == 0) { red[w][0] = kr; red[w][1] = ki; red[w][2] = gr; red[w][3] = gi; }
        __syncthreads();
        if (tid == 0) {
            sc[5] = 0.5 * tj * (red[0][0] + red[1][0] + red[2][0] + red[3][0]);
            sc[6] = 0.5 * tj * (red[0][1] + red[1][1] + red[2][1] + red[3][1]);
            sc[7] = 0.0;
            red[0][2] = red[0][2] + red[1][2] + red[2][2] + red[3][2];
            red[0][3] = red[0][3] + red[1][3] + red[2][3] + red[3][3];
        }
        __syncthreads();
    }

    // ---- phase 4: write B and D
    if (t > 0) {
        const F gmr = red[0][2], gmi = red[0][3];
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            const int r = e & 63, c = e >> 6;
            if (r >= Lr || c >= b) continue;
            CV a;
            if (c == 0) {
                a = (tj == 0.0) ? mk2<F>(vn[0].x * 0 + Bs[r].x - yv[r].x, Bs[r].y - yv[r].y)
                                : (r == 0 ? beta : mk2<F>(0.0, 0.0));
            } else {
                a = Bs[r + c * LDS];
                const CV vpc = vp[c], y = yv[r];
                // right update: - y conj(vp_c)
                a.x -= y.x * vpc.x + y.y * vpc.y;
                a.y -= y.y * vpc.x - y.x * vpc.y;
                if (tj != 0.0) {
                    // left update: - tau v_r (wB_c - gamma conj(vp_c)),  gamma = v^H y (y holds tp)
                    const CV wbc = wb[c];
                    const F qr = wbc.x - (gmr * vpc.x + gmi * vpc.y);
                    const F qi = wbc.y - (gmi * vpc.x - gmr * vpc.y);
                    const CV v = vn[r];
                    a.x -= tj * (v.x * qr - v.y * qi);
                    a.y -= tj * (v.x * qi + v.y * qr);
                }
            }
            st2<F>(AB + 2 * ((b + r - c) + (c0 + c) * ldab), a);
        }
    } else {
        for (int r = tid; r < Lr; r += blockDim.x) {
            const CV a = (tj == 0.0) ? vn[r] : (r == 0 ? beta : mk2<F>(0.0, 0.0));
            // when tj == 0 the column is unchanged (vn was overwritten by v; reload)
            if (tj == 0.0) continue;
            st2<F>(AB + 2 * ((1 + r) + s * ldab), a);
        }
    }
    if (tj != 0.0) {
        const F Kr = sc[5], Ki = sc[6];
#pragma unroll 4
        for (int i = 0; i < 16; ++i) {
            const int e = tid + 256 * i;
            const int r = e & 63, c = e >> 6;
            if (r >= Lr || c >= Lr || r < c) continue;
            const CV vr = vn[r], vc = vn[c], pr = pv[r], pc = pv[c];
            const CV wr = mk2<F>(pr.x - (Kr * vr.x - Ki * vr.y), pr.y - (Kr * vr.y + Ki * vr.x));
            const CV wc = mk2<F>(pc.x - (Kr * vc.x - Ki * vc.y), pc.y - (Kr * vc.y + Ki * vc.x));
            CV a = Ds[r + c * LDS];
            a.x -= (vr.x * wc.x + vr.y * wc.y) + (wr.x * vc.x + wr.y * vc.y);
            a.y -= (vr.y * wc.x - vr.x * wc.y) + (wr.y * vc.x - wr.x * vc.y);
            if (r == c) a.y = 0.0;
            st2<F>(AB + 2 * ((r - c) + (r0 + c) * ldab), a);
        }
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
int hb2st_t(int64_t n, int b, F *AB, int64_t ldab, F *V2, F *tau2, const int64_t *voff_dev,
            double *d, double *e_cplx, hipStream_t s) {
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
            hipLaunchKernelGGL((hb2st_step<F>), dim3((unsigned)(s_hi - s_lo + 1)), dim3(256), 0, s, n, b,
                               AB, ldab, V2, tau2, voff_dev, g, s_lo);
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

int hb2st(int64_t n, int b, double *AB, int64_t ldab, double *V2, double *tau2,
          const int64_t *voff_dev, double *d, double *e_cplx, hipStream_t s) {
    return hb2st_t<double>(n, b, AB, ldab, V2, tau2, voff_dev, d, e_cplx, s);
}
int hb2st(int64_t n, int b, float *AB, int64_t ldab, float *V2, float *tau2,
          const int64_t *voff_dev, double *d, double *e_cplx, hipStream_t s) {
    return hb2st_t<float>(n, b, AB, ldab, V2, tau2, voff_dev, d, e_cplx, s);
}

}  // namespace bdg
