// Tridiagonal eigensolver: divide and conquer in FP64 (third step of the
// solver, "diagonalizing this tridiagonal form", paper sec. "Performance of
// the Matrix Diagonalization Algorithm").
//
// Method (Cuppen 1981; deflation as in Dongarra & Sorensen 1987; eigenvectors
// by the Gu & Eisenstat 1995 recomputation of z):
//   * tear T at the midpoint m of every node: T = diag(T1', T2') + rho w w^T,
//     rho = |e_{m-1}|, w = e_{m-1} + sign(e_{m-1}) e_m, T1'/T2' lose rho on
//     the touching diagonal entries;
//   * leaves (<= 32) are solved by parallel cyclic Jacobi in one workgroup;
//   * a merge solves D + rho z z^T: z from the last row of Q1 and first row of
//     Q2, deflation of small z_i and of close pairs (Givens rotation), the
//     secular equation 1 + rho sum z_i^2/(d_i - lambda) = 0 for the rest (one
//     thread per root; bracketed iteration on a two-pole rational model,
//     Bunch, Nielsen & Sorensen 1978, with bisection as the safeguard), the
//     Loewner formula for z-hat, and the eigenvector DGEMM on MFMA.
// Roots are kept as (origin pole, offset) so that d_i - lambda_j is formed
// without cancellation.
#include "gemm.h"
#include "stages.h"

#include <math.h>
#include <mutex>
#include <vector>

namespace bdg {
namespace {

constexpr int LEAFMAX = 32;
constexpr double EPS = 1.1102230246251565e-16;  // unit roundoff 2^-53

// ---------------------------------------------------------------- tearing
__global__ void tear_kernel(const double *__restrict__ e, const int64_t *__restrict__ splits, int ns,
                            double *__restrict__ dt) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    const int64_t m = splits[i];
    const double rho = fabs(e[m - 1]);
    dt[m - 1] -= rho;
    dt[m] -= rho;
}

// ---------------------------------------------------------------- leaves
__global__ __launch_bounds__(64) void leaf_jacobi(const double *__restrict__ dt,
                                                  const double *__restrict__ e,
                                                  const int64_t *__restrict__ starts, int64_t ldq,
                                                  double *__restrict__ Q, double *__restrict__ lam) {
    __shared__ double A[LEAFMAX][LEAFMAX + 1];
    __shared__ double V[LEAFMAX][LEAFMAX + 1];
    __shared__ double rc[LEAFMAX / 2], rs[LEAFMAX / 2];
    __shared__ int rp[LEAFMAX / 2], rq[LEAFMAX / 2];
    __shared__ int nrot;
    __shared__ double ev[LEAFMAX];
    const int t = threadIdx.x;
    const int64_t a = starts[blockIdx.x], c = starts[blockIdx.x + 1];
    const int L = (int)(c - a);
    const int Lp = L + (L & 1);
    for (int idx = t; idx < LEAFMAX * LEAFMAX; idx += 64) {
        const int i = idx % LEAFMAX, j = idx / LEAFMAX;
        double v = 0.0;
        if (i < L && j < L) {
            if (i == j) v = dt[a + i];
            else if (i == j + 1) v = e[a + j];
            else if (j == i + 1) v = e[a + i];
        }
        A[i][j] = v;
        V[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 40; ++sweep) {
        // an entry is negligible below EPS * sqrt(|a_pp a_qq|) (relative
        // criterion); the iteration stops after a sweep without rotations
        if (t == 0) nrot = 0;
        __syncthreads();
        for (int r = 0; r < Lp - 1; ++r) {
            if (t < Lp / 2) {
                int p, q;
                if (t == 0) { p = Lp - 1; q = r; }
                else { p = (r + t) % (Lp - 1); q = (r - t + (Lp - 1)) % (Lp - 1); }
                if (p > q) { const int tmp = p; p = q; q = tmp; }
                double cc = 1.0, ss = 0.0;
                if (q < L) {
                    const double apq = A[p][q];
                    if (fabs(apq) > 1e-300 && fabs(apq) > EPS * sqrt(fabs(A[p][p] * A[q][q]))) {
                        atomicAdd(&nrot, 1);
                        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                        const double tt = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        cc = 1.0 / sqrt(1.0 + tt * tt);
                        ss = tt * cc;
                    }
                }
                rp[t] = p; rq[t] = q; rc[t] = cc; rs[t] = ss;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (int idx = t; idx < (Lp / 2) * L; idx += 64) {
                const int k = idx / L, i = idx % L;
                const int p = rp[k], q = rq[k];
                if (q >= L) continue;
                const double cc = rc[k], ss = rs[k];
                const double ap = A[i][p], aq = A[i][q];
                A[i][p] = cc * ap - ss * aq;
                A[i][q] = ss * ap + cc * aq;
                const double vp = V[i][p], vq = V[i][q];
                V[i][p] = cc * vp - ss * vq;
                V[i][q] = ss * vp + cc * vq;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (int idx = t; idx < (Lp / 2) * L; idx += 64) {
                const int k = idx / L, i = idx % L;
                const int p = rp[k], q = rq[k];
                if (q >= L) continue;
                const double cc = rc[k], ss = rs[k];
                const double ap = A[p][i], aq = A[q][i];
                A[p][i] = cc * ap - ss * aq;
                A[q][i] = ss * ap + cc * aq;
            }
            __syncthreads();
        }
        const bool done = (nrot == 0);
        __syncthreads();
        if (done) break;
    }
    // sort eigenvalues ascending (ties by index) and write Q block, lam
    if (t < L) ev[t] = A[t][t];
    __syncthreads();
    if (t < L) {
        const double v = ev[t];
        int rank = 0;
        for (int j = 0; j < L; ++j) rank += (ev[j] < v) || (ev[j] == v && j < t);
        lam[a + rank] = v;
        for (int i = 0; i < L; ++i) Q[(a + i) + (a + rank) * ldq] = V[i][t];
    }
}

// ---------------------------------------------------------------- merge scratch
struct MergeScratch {
    double *z;      // K, block column order
    double *Ds;     // K, sorted D
    int *sidx;      // K, block column of sorted position
    int *nd;        // K, nondeflated block columns (sorted order)
    double *Dnd;    // K
    double *znd;    // K
    int *dfi;       // K, deflated block columns (sorted by value)
    double *Ddf;    // K
    int *rotp;      // K rotation pairs
    int *rotq;
    double *rotc;
    double *rots;
    int *orig;      // k, origin pole of each root
    double *tau;    // k
    double *zhat;   // k
    int *posnd;     // k final positions
    int *posdf;     // K - k
    double *lamnd;  // k
    int *ctop;      // nondeflated columns touching the top half, and their rows in U
    int *rtop;
    int *cbot;      // ... touching the bottom half
    int *rbot;
    int *info;      // [0]=k [1]=ndef [2]=nrot [4]=k_top [5]=k_bot (one block per merge)
    int *err;       // secular iteration did not converge (shared by all merges)
};

// The merges of one tree level cover disjoint column ranges [a, a + K): each
// takes the slice of every K-sized array that starts at a, its own info block
// and rho slot.
MergeScratch slice(const MergeScratch &m, int64_t a, int *info) {
    MergeScratch r = m;
    r.z += a; r.Ds += a; r.sidx += a; r.nd += a; r.Dnd += a; r.znd += a; r.dfi += a; r.Ddf += a;
    r.rotp += a; r.rotq += a; r.rotc += a; r.rots += a; r.orig += a; r.tau += a; r.zhat += a;
    r.posnd += a; r.posdf += a; r.lamnd += a; r.ctop += a; r.rtop += a; r.cbot += a; r.rbot += a;
    r.info = info;
    return r;
}

// z, sorted order and deflation (one workgroup).  The rank merge, the gathers
// and the final split of the kept columns by half run on all threads; the
// deflation scan itself is serial (each test depends on the rotations before
// it) and runs on thread 0 over chunks of sorted positions that the block
// stages in LDS, so the scan never waits on global memory.
constexpr int DCH = 2048;   // sorted positions staged per chunk
constexpr int DWIN = 1024;  // tail of the deflated list mirrored in LDS (power of two)
__global__ __launch_bounds__(1024) void merge_deflate(int64_t K, int64_t n1, double rho_in, double sgn,
                                                      const double *__restrict__ Qblk, int64_t ldq,
                                                      const double *__restrict__ lam, MergeScratch m,
                                                      double *__restrict__ rho_out) {
    __shared__ double red[32];
    __shared__ double sD[DCH], sZ[DCH];
    __shared__ int sJ[DCH];
    __shared__ double wD[DWIN];
    __shared__ int wI[DWIN];
    __shared__ int wcnt[2][16];
    __shared__ int shk[3];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const double inv_sqrt2 = 0.70710678118654752440;
    // z from last row of Q1 / first row of Q2
    for (int64_t i = t; i < K; i += blockDim.x) {
        double zi;
        if (i < n1) zi = Qblk[(n1 - 1) + i * ldq];
        else zi = sgn * Qblk[n1 + i * ldq];
        m.z[i] = zi * inv_sqrt2;
    }
    // merge the two sorted lists by rank
    for (int64_t i = t; i < K; i += blockDim.x) {
        const double v = lam[i];
        int64_t lo, hi, base;
        if (i < n1) {  // count second-list entries < v
            lo = n1; hi = K;
            while (lo < hi) { const int64_t md = (lo + hi) >> 1; if (lam[md] < v) lo = md + 1; else hi = md; }
            base = i + (lo - n1);
        } else {       // count first-list entries <= v
            lo = 0; hi = n1;
            while (lo < hi) { const int64_t md = (lo + hi) >> 1; if (lam[md] <= v) lo = md + 1; else hi = md; }
            base = (i - n1) + lo;
        }
        m.sidx[base] = (int)i;
        m.Ds[base] = v;
    }
    // tolerance: 8 eps max(max|D|, rho)
    double mx = 0.0;
    for (int64_t i = t; i < K; i += blockDim.x) mx = fmax(mx, fabs(lam[i]));
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (lane == 0) red[w] = mx;
    __syncthreads();
    double dmax = 0.0;
    for (int q = 0; q < (int)(blockDim.x >> 6); ++q) dmax = fmax(dmax, red[q]);
    const double rho = 2.0 * rho_in;
    const double tol = 8.0 * 2.0 * EPS * fmax(dmax, rho);

    // scan state (thread 0): pending column pj with value Dpj, weight zpj and
    // the halves mpj its column is nonzero in (1 top, 2 bottom)
    int k = 0, ndef = 0, nrot = 0, pj = -1, mpj = 0;
    double Dpj = 0.0, zpj = 0.0;
    // deflated list, kept sorted by insertion (values arrive nearly sorted);
    // written through to global memory, its last DWIN entries also in LDS
    auto put_def = [&](int p, double v, int col) {
        if (p > ndef - DWIN) { wD[p & (DWIN - 1)] = v; wI[p & (DWIN - 1)] = col; }
        m.Ddf[p] = v;
        m.dfi[p] = col;
    };
    auto add_def = [&](int col, double val) {
        int p = ndef;
        while (p > 0) {
            const bool inl = p - 1 > ndef - DWIN;
            const double prev = inl ? wD[(p - 1) & (DWIN - 1)] : m.Ddf[p - 1];
            if (!(prev > val)) break;
            put_def(p, prev, inl ? wI[(p - 1) & (DWIN - 1)] : m.dfi[p - 1]);
            --p;
        }
        put_def(p, val, col);
        ++ndef;
    };
    // kept column: its half mask goes to posnd, which merge_place overwrites later
    auto emit = [&]() {
        m.nd[k] = pj; m.Dnd[k] = Dpj; m.znd[k] = zpj; m.posnd[k] = mpj; ++k;
    };
    for (int64_t c0 = 0; c0 < K; c0 += DCH) {
        const int cn = (int)((K - c0) < DCH ? (K - c0) : DCH);
        for (int q = t; q < cn; q += blockDim.x) {
            const int j = m.sidx[c0 + q];
            sJ[q] = j;
            sD[q] = m.Ds[c0 + q];
            sZ[q] = m.z[j];
        }
        __syncthreads();
        if (t == 0) {
            for (int q = 0; q < cn; ++q) {
                const int j = sJ[q];
                const double Dj = sD[q], zj = sZ[q];
                const int mj = j < n1 ? 1 : 2;
                if (rho * fabs(zj) <= tol) {
                    add_def(j, Dj);
                    continue;
                }
                if (pj < 0) { pj = j; Dpj = Dj; zpj = zj; mpj = mj; continue; }
                // rotation test |(Dj - Dpj) c s| <= tol with c = zj/r, s = -zpj/r
                const double r2 = zj * zj + zpj * zpj;
                if (fabs((Dj - Dpj) * zj * zpj) <= tol * r2) {
                    // rotate (pj, j): z_pj -> 0, z_j -> r
                    const double r = sqrt(r2);
                    const double cc = zj / r, ss = -zpj / r;
                    m.rotp[nrot] = pj; m.rotq[nrot] = j; m.rotc[nrot] = cc; m.rots[nrot] = ss; ++nrot;
                    const double newp = Dpj * cc * cc + Dj * ss * ss;
                    const double newj = Dpj * ss * ss + Dj * cc * cc;
                    add_def(pj, newp);
                    pj = j; Dpj = newj; zpj = r; mpj |= mj;
                } else {
                    emit();
                    pj = j; Dpj = Dj; zpj = zj; mpj = mj;
                }
            }
            if (c0 + cn == K) {
                if (pj >= 0) emit();
                shk[0] = k; shk[1] = ndef; shk[2] = nrot;
            }
        }
        __syncthreads();
    }
    // kept columns of each half (order preserved) for the split eigenvector product
    const int kk = K > 0 ? shk[0] : 0;
    int bt = 0, bb = 0;
    for (int c0 = 0; c0 < kk; c0 += (int)blockDim.x) {
        const int i = c0 + t;
        const int mk = i < kk ? m.posnd[i] : 0;
        const unsigned long long vt = __ballot(mk & 1), vb = __ballot(mk & 2);
        const unsigned long long below = (1ull << lane) - 1ull;
        if (lane == 0) { wcnt[0][w] = __popcll(vt); wcnt[1][w] = __popcll(vb); }
        __syncthreads();
        int ot = bt + __popcll(vt & below), ob = bb + __popcll(vb & below);
        for (int q = 0; q < (int)(blockDim.x >> 6); ++q) {
            if (q < w) { ot += wcnt[0][q]; ob += wcnt[1][q]; }
            bt += wcnt[0][q];
            bb += wcnt[1][q];
        }
        if (mk) {
            const int col = m.nd[i];
            if (mk & 1) { m.ctop[ot] = col; m.rtop[ot] = i; }
            if (mk & 2) { m.cbot[ob] = col; m.rbot[ob] = i; }
        }
        __syncthreads();
    }
    if (t == 0) {
        m.info[4] = bt;
        m.info[5] = bb;
        m.info[0] = kk;
        m.info[1] = K > 0 ? shk[1] : 0;
        m.info[2] = K > 0 ? shk[2] : 0;
        *rho_out = rho;
    }
}

// Apply the deflation rotations to the block columns (thread per row).
__global__ void merge_rotate(int64_t K, double *__restrict__ Qblk, int64_t ldq, MergeScratch m) {
    const int nrot = m.info[2];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < K;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int r = 0; r < nrot; ++r) {
            double *qp = Qblk + i + (int64_t)m.rotp[r] * ldq;
            double *qq = Qblk + i + (int64_t)m.rotq[r] * ldq;
            const double cc = m.rotc[r], ss = m.rots[r];
            const double x = *qp, y = *qq;
            *qp = cc * x + ss * y;
            *qq = cc * y - ss * x;
        }
    }
}

// Secular equation, one wavefront per root j of D + rho z z^T (rho > 0): the
// 64 lanes split every sum over the poles (wave reductions, fixed order), and
// all lanes then take the same step, so the control flow stays uniform.
__global__ __launch_bounds__(256) void merge_secular(const double *__restrict__ rho_p, MergeScratch m) {
    const int k = m.info[0];
    const int lane = threadIdx.x & 63;
    const int j = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (j >= k) return;  // the whole wave
    const double rho = *rho_p;
    const double *D = m.Dnd;
    const double *z = m.znd;
    int o;
    double lo, hi;  // bracket for tau relative to D[o]
    if (j < k - 1) {
        const double gap = D[j + 1] - D[j];
        const double mid = 0.5 * gap;
        double f = 0.0;
        for (int i = lane; i < k; i += 64) f += rho * z[i] * z[i] / ((D[i] - D[j]) - mid);
        f = 1.0 + wave_sum(f);
        if (f >= 0.0) { o = j; lo = 0.0; hi = mid; }
        else { o = j + 1; lo = -mid; hi = 0.0; }
    } else {
        double ztz = 0.0;
        for (int i = lane; i < k; i += 64) ztz += z[i] * z[i];
        ztz = wave_sum(ztz);
        o = j;
        lo = 0.0;
        hi = rho * ztz;
    }
    const double Do = D[o];
    double tau = 0.5 * (lo + hi);
    bool conv = false;
    for (int it = 0; it < 100; ++it) {
        double psi = 0.0, dpsi = 0.0, phi = 0.0, dphi = 0.0, aerr = 0.0;
        for (int i = lane; i < k; i += 64) {
            const double del = (D[i] - Do) - tau;
            const double q = z[i] / del;
            const double term = rho * z[i] * q;
            if (i <= j) { psi += term; dpsi += rho * q * q; }
            else { phi += term; dphi += rho * q * q; }
            aerr += fabs(term);
        }
        psi = wave_sum(psi);
        dpsi = wave_sum(dpsi);
        phi = wave_sum(phi);
        dphi = wave_sum(dphi);
        aerr = wave_sum(aerr);
        const double f = 1.0 + psi + phi;
        if (fabs(f) <= 8.0 * EPS * (1.0 + aerr) * (double)(k < 8 ? 8 : k) / 8.0 * 4.0) { conv = true; break; }
        if (f < 0.0) lo = tau; else hi = tau;
        if (hi - lo <= 2.0 * EPS * fmax(fabs(lo), fabs(hi))) { conv = true; break; }
        // two-pole rational model through (psi, dpsi) at the left pole and (phi, dphi) at the right
        const double p1 = (D[j] - Do) - tau;  // left pole offset (<= 0 side)
        double eta;
        bool ok = false;
        if (j < k - 1) {
            const double p2 = (D[j + 1] - Do) - tau;
            const double b = dpsi * p1 * p1, a = psi - b / p1;
            const double dd = dphi * p2 * p2, cc = phi - dd / p2;
            const double A0 = 1.0 + a + cc;
            const double B = A0 * (p1 + p2) + b + dd;
            const double C = p1 * p2 * f;
            const double disc = B * B - 4.0 * A0 * C;
            if (disc >= 0.0) {
                const double sq = sqrt(disc);
                const double den = B + (B >= 0.0 ? sq : -sq);
                if (den != 0.0) { eta = 2.0 * C / den; ok = true; }
            }
        } else {
            const double b = dpsi * p1 * p1, a = psi - b / p1;
            if (1.0 + a != 0.0) { eta = p1 + b / (1.0 + a); ok = true; }
        }
        double tn = ok ? tau + eta : 0.5 * (lo + hi);
        if (!(tn > lo && tn < hi)) tn = 0.5 * (lo + hi);
        if (tn == tau) { conv = true; break; }
        tau = tn;
    }
    if (lane != 0) return;
    if (!conv) atomicOr(m.err, 1);
    m.orig[j] = o;
    m.tau[j] = tau;
    m.lamnd[j] = Do + tau;
}

// z-hat by the Loewner formula, one wavefront per i: every factor of the
// product except lambda_{k-1}/rho lies in (0, 1) by interlacing, so the
// lanes' partial products cannot overflow.
__global__ __launch_bounds__(256) void merge_zhat(const double *__restrict__ rho_p, MergeScratch m) {
    const int k = m.info[0];
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= k) return;  // the whole wave
    const double rho = *rho_p;
    const double *D = m.Dnd;
    const double Di = D[i];
    // lambda_j - D_i = (D[o_j] - D_i) + tau_j
    auto lmd = [&](int jj) { return (D[m.orig[jj]] - Di) + m.tau[jj]; };
    double prod = 1.0;
    for (int jj = lane; jj < k; jj += 64) {
        if (jj < i) prod *= lmd(jj) / (D[jj] - Di);
        else if (jj > i) prod *= lmd(jj - 1) / (D[jj] - Di);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) prod *= __shfl_xor(prod, o, 64);
    if (lane != 0) return;
    prod *= lmd(k - 1) / rho;
    double zh = sqrt(fabs(prod));
    if (m.znd[i] < 0.0) zh = -zh;
    m.zhat[i] = zh;
}

// U[:, j] = zhat / (D - lambda_j), normalised (workgroup per column).
__global__ __launch_bounds__(256) void merge_vectors(MergeScratch m, double *__restrict__ U) {
    __shared__ double red[8];
    const int k = m.info[0];
    const int j = blockIdx.x;
    if (j >= k) return;
    const double *D = m.Dnd;
    const double Do = D[m.orig[j]], tj = m.tau[j];
    double s = 0.0;
    for (int i = threadIdx.x; i < k; i += blockDim.x) {
        const double u = m.zhat[i] / ((D[i] - Do) - tj);
        U[i + (int64_t)j * k] = u;
        s += u * u;
    }
    s = block_sum(s, red);
    const double inv = 1.0 / sqrt(s);
    for (int i = threadIdx.x; i < k; i += blockDim.x) U[i + (int64_t)j * k] *= inv;
}

// Final positions (merge nondeflated roots with deflated values), copy the
// deflated columns and all eigenvalues into the next level's buffers.
__global__ void merge_place(int64_t K, const double *__restrict__ Qblk, int64_t ldq,
                            double *__restrict__ Qnext, double *__restrict__ lam_next, MergeScratch m) {
    const int k = m.info[0], ndef = m.info[1];
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < k + ndef;
         s += (int64_t)gridDim.x * blockDim.x) {
        if (s < k) {
            const double v = m.lamnd[s];
            int lo = 0, hi = ndef;  // deflated values < v
            while (lo < hi) { const int md = (lo + hi) >> 1; if (m.Ddf[md] < v) lo = md + 1; else hi = md; }
            const int pos = (int)s + lo;
            m.posnd[s] = pos;
            lam_next[pos] = v;
        } else {
            const int q = (int)(s - k);
            const double v = m.Ddf[q];
            int lo = 0, hi = k;  // roots <= v
            while (lo < hi) { const int md = (lo + hi) >> 1; if (m.lamnd[md] <= v) lo = md + 1; else hi = md; }
            const int pos = q + lo;
            m.posdf[q] = pos;
            lam_next[pos] = v;
        }
    }
}

__global__ void copy_deflated(int64_t K, const double *__restrict__ Qblk, int64_t ldq,
                              double *__restrict__ Qnext, MergeScratch m) {
    const int ndef = m.info[1];
    const int q = blockIdx.x;
    if (q >= ndef) return;
    const double *src = Qblk + (int64_t)m.dfi[q] * ldq;
    double *dst = Qnext + (int64_t)m.posdf[q] * ldq;
    for (int64_t i = threadIdx.x; i < K; i += blockDim.x) dst[i] = src[i];
}

struct Node { int64_t a, m, c; };

constexpr int MERGE_STREAMS = 4;

// MERGE_STREAMS non-blocking streams per device (default priority), created
// on first use and kept for the life of the process.
hipStream_t *merge_streams() {
    static std::mutex mu;
    static hipStream_t st[64][MERGE_STREAMS];
    static bool made[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> lock(mu);
    if (!made[dev]) {
        for (int q = 0; q < MERGE_STREAMS; ++q)
            if (hipStreamCreateWithFlags(&st[dev][q], hipStreamNonBlocking) != hipSuccess) return nullptr;
        made[dev] = true;
    }
    return st[dev];
}

struct StreamEvents {
    hipEvent_t main = nullptr, side[MERGE_STREAMS] = {};
    bool ok = false;
    StreamEvents() {
        ok = hipEventCreateWithFlags(&main, hipEventDisableTiming) == hipSuccess;
        for (int q = 0; q < MERGE_STREAMS; ++q)
            ok = ok && hipEventCreateWithFlags(&side[q], hipEventDisableTiming) == hipSuccess;
    }
    ~StreamEvents() {
        if (main) (void)hipEventDestroy(main);
        for (int q = 0; q < MERGE_STREAMS; ++q)
            if (side[q]) (void)hipEventDestroy(side[q]);
    }
};

// Between a fork and its join the merge streams may still run kernels on the
// caller's workspace: an early error return drains them first.
struct MergeDrain {
    hipStream_t *st;
    bool armed = false;
    explicit MergeDrain(hipStream_t *s) : st(s) {}
    ~MergeDrain() {
        if (armed)
            for (int q = 0; q < MERGE_STREAMS; ++q) (void)hipStreamSynchronize(st[q]);
    }
};

}  // namespace

size_t stedc_workspace(int64_t n) {
    size_t w = 0;
    w += 8 * (size_t)n * n;       // second Q buffer
    w += 8 * (size_t)n * n;       // U
    w += 8 * (size_t)n * 4;       // dt, lam a/b, spare
    w += (size_t)n * (8 * 12 + 4 * 20);  // merge scratch
    w += 8 * (size_t)n + 4096;    // splits, starts, rho, info
    w += 48 * (size_t)n;          // per-merge info blocks and rho slots
    return w;
}

int stedc(int64_t n, const double *d, const double *e, double *lam_out, double *Q_out, int64_t ldq,
          void *work, hipStream_t s, int leaf) {
    if (leaf <= 0 || leaf > LEAFMAX) leaf = LEAFMAX;
    if (ldq != n) {
        set_error("stedc: ldq must equal n");
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    char *wp = (char *)work;
    auto take = [&](size_t bytes) {
        char *p = wp;
        wp += (bytes + 255) / 256 * 256;
        return (void *)p;
    };
    double *Qalt = (double *)take(8 * (size_t)n * n);
    double *U = (double *)take(8 * (size_t)n * n);
    double *dt = (double *)take(8 * (size_t)n);
    double *lamA = (double *)take(8 * (size_t)n);
    double *lamB = (double *)take(8 * (size_t)n);
    MergeScratch ms;
    ms.z = (double *)take(8 * (size_t)n);
    ms.Ds = (double *)take(8 * (size_t)n);
    ms.sidx = (int *)take(4 * (size_t)n);
    ms.nd = (int *)take(4 * (size_t)n);
    ms.Dnd = (double *)take(8 * (size_t)n);
    ms.znd = (double *)take(8 * (size_t)n);
    ms.dfi = (int *)take(4 * (size_t)n);
    ms.Ddf = (double *)take(8 * (size_t)n);
    ms.rotp = (int *)take(4 * (size_t)n);
    ms.rotq = (int *)take(4 * (size_t)n);
    ms.rotc = (double *)take(8 * (size_t)n);
    ms.rots = (double *)take(8 * (size_t)n);
    ms.orig = (int *)take(4 * (size_t)n);
    ms.tau = (double *)take(8 * (size_t)n);
    ms.zhat = (double *)take(8 * (size_t)n);
    ms.posnd = (int *)take(4 * (size_t)n);
    ms.posdf = (int *)take(4 * (size_t)n);
    ms.lamnd = (double *)take(8 * (size_t)n);
    ms.ctop = (int *)take(4 * (size_t)n);
    ms.rtop = (int *)take(4 * (size_t)n);
    ms.cbot = (int *)take(4 * (size_t)n);
    ms.rbot = (int *)take(4 * (size_t)n);
    // per merge of a level (at most n / 2 merges): an info block of 8 ints
    // and a rho slot; plus the shared error flag
    int *info_all = (int *)take(32 * (size_t)n + 64);
    double *rho_all = (double *)take(8 * (size_t)n + 64);
    ms.err = (int *)take(64);
    ms.info = info_all;

    // tree: split every node at its midpoint down to a common depth
    int depth = 0;
    while ((n + ((int64_t)1 << depth) - 1) >> depth > leaf) ++depth;
    std::vector<std::vector<Node>> levels(depth + 1);
    std::vector<int64_t> starts;
    std::vector<int64_t> splits;
    {
        std::vector<std::pair<int64_t, int64_t>> cur{{0, n}};
        for (int lv = 0; lv < depth; ++lv) {
            std::vector<std::pair<int64_t, int64_t>> nxt;
            for (auto &r : cur) {
                const int64_t a = r.first, c = r.second, mm = a + (c - a) / 2;
                levels[depth - lv].push_back(Node{a, mm, c});
                splits.push_back(mm);
                nxt.push_back({a, mm});
                nxt.push_back({mm, c});
            }
            cur.swap(nxt);
        }
        for (auto &r : cur) starts.push_back(r.first);
        starts.push_back(n);
    }
    // device copies of the split and start lists
    const size_t nst = starts.size(), nsp = splits.size();
    int64_t *dsplit = (int64_t *)take(8 * (nsp + 1));
    int64_t *dstart = (int64_t *)take(8 * (nst + 1));
    if (nsp) BDG_HIP(hipMemcpyAsync(dsplit, splits.data(), 8 * nsp, hipMemcpyHostToDevice, s));
    BDG_HIP(hipMemcpyAsync(dstart, starts.data(), 8 * nst, hipMemcpyHostToDevice, s));
    BDG_HIP(hipMemcpyAsync(dt, d, 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (nsp) {
        hipLaunchKernelGGL(tear_kernel, dim3((unsigned)((nsp + 255) / 256)), dim3(256), 0, s, e, dsplit,
                           (int)nsp, dt);
        BDG_CHECK_LAUNCH();
    }
    // buffers: level h writes buf[h % 2]; the top level (depth) must land in Q_out
    double *Qbuf[2], *Lbuf[2];
    Qbuf[depth % 2] = Q_out;
    Qbuf[(depth + 1) % 2] = Qalt;
    Lbuf[depth % 2] = lamA;
    Lbuf[(depth + 1) % 2] = lamB;
    BDG_HIP(hipMemsetAsync(Q_out, 0, 8 * (size_t)n * n, s));
    if (depth > 0) BDG_HIP(hipMemsetAsync(Qalt, 0, 8 * (size_t)n * n, s));
    BDG_HIP(hipMemsetAsync(ms.err, 0, sizeof(int), s));
    hipLaunchKernelGGL(leaf_jacobi, dim3((unsigned)(nst - 1)), dim3(64), 0, s, dt, e, dstart, n, Qbuf[0],
                       Lbuf[0]);
    BDG_CHECK_LAUNCH();
    std::vector<double> eh((size_t)(n > 1 ? n - 1 : 1));
    if (n > 1) {
        BDG_HIP(hipMemcpyAsync(eh.data(), e, 8 * (size_t)(n - 1), hipMemcpyDeviceToHost, s));
        BDG_HIP(hipStreamSynchronize(s));
    }
    // The merges of one level are independent (disjoint columns of Q, scratch
    // slices, U blocks): they run on MERGE_STREAMS streams in two phases,
    // deflation for all of them, one copy of their sizes to the host, then
    // the rest, so a level costs one host round trip instead of one per merge.
    hipStream_t *mst = merge_streams();
    if (!mst) {
        set_error("stedc: could not create the merge streams");
        return BDG_ERR_HIP;
    }
    StreamEvents evs;
    if (!evs.ok) {
        set_error("stedc: could not create events");
        return BDG_ERR_HIP;
    }
    MergeDrain drain(mst);
    auto fork = [&]() -> int {
        BDG_HIP(hipEventRecord(evs.main, s));
        drain.armed = true;
        for (int q = 0; q < MERGE_STREAMS; ++q) BDG_HIP(hipStreamWaitEvent(mst[q], evs.main, 0));
        return 0;
    };
    auto join = [&]() -> int {
        for (int q = 0; q < MERGE_STREAMS; ++q) {
            BDG_HIP(hipEventRecord(evs.side[q], mst[q]));
            BDG_HIP(hipStreamWaitEvent(s, evs.side[q], 0));
        }
        drain.armed = false;
        return 0;
    };
    std::vector<int> infoh;
    for (int h = 1; h <= depth; ++h) {
        double *Qc = Qbuf[(h - 1) % 2], *Qn = Qbuf[h % 2];
        double *Lc = Lbuf[(h - 1) % 2], *Ln = Lbuf[h % 2];
        const std::vector<Node> &lv = levels[h];
        const int nm = (int)lv.size();
        BDG_TRY(fork());
        for (int i = 0; i < nm; ++i) {
            const Node &nd = lv[i];
            const int64_t K = nd.c - nd.a, n1 = nd.m - nd.a;
            const double ev = eh[nd.m - 1];
            const double rho = fabs(ev), sg = ev >= 0.0 ? 1.0 : -1.0;
            const MergeScratch mi = slice(ms, nd.a, info_all + 8 * i);
            hipLaunchKernelGGL(merge_deflate, dim3(1), dim3(1024), 0, mst[i % MERGE_STREAMS], K, n1, rho, sg,
                               Qc + nd.a + nd.a * n, n, Lc + nd.a, mi, rho_all + i);
            BDG_CHECK_LAUNCH();
        }
        BDG_TRY(join());
        infoh.resize((size_t)8 * nm);
        BDG_HIP(hipMemcpyAsync(infoh.data(), info_all, 32 * (size_t)nm, hipMemcpyDeviceToHost, s));
        BDG_HIP(hipStreamSynchronize(s));
        BDG_TRY(fork());
        for (int i = 0; i < nm; ++i) {
            const Node &nd = lv[i];
            hipStream_t q = mst[i % MERGE_STREAMS];
            const int64_t K = nd.c - nd.a, n1 = nd.m - nd.a;
            const int *inf = infoh.data() + 8 * i;
            const int k = inf[0], ndef = inf[1], nrot = inf[2], ktop = inf[4], kbot = inf[5];
            const MergeScratch mi = slice(ms, nd.a, info_all + 8 * i);
            double *rho_d = rho_all + i;
            double *Ui = U + nd.a * n;  // k x k with ld k inside columns [a, a + K) of U
            double *Qblk = Qc + nd.a + nd.a * n;
            double *Qnb = Qn + nd.a + nd.a * n;
            if (nrot > 0) {
                hipLaunchKernelGGL(merge_rotate, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, q, K, Qblk, n, mi);
                BDG_CHECK_LAUNCH();
            }
            if (k > 0) {
                hipLaunchKernelGGL(merge_secular, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, q, rho_d, mi);
                BDG_CHECK_LAUNCH();
                hipLaunchKernelGGL(merge_zhat, dim3((unsigned)((k + 3) / 4)), dim3(256), 0, q, rho_d, mi);
                BDG_CHECK_LAUNCH();
                hipLaunchKernelGGL(merge_vectors, dim3((unsigned)k), dim3(256), 0, q, mi, Ui);
                BDG_CHECK_LAUNCH();
            }
            hipLaunchKernelGGL(merge_place, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, q, K, Qblk, n, Qnb,
                               Ln + nd.a, mi);
            BDG_CHECK_LAUNCH();
            if (ndef > 0) {
                hipLaunchKernelGGL(copy_deflated, dim3((unsigned)ndef), dim3(256), 0, q, K, Qblk, n, Qnb, mi);
                BDG_CHECK_LAUNCH();
            }
            if (k > 0) {
                // top rows use the columns nonzero there, bottom rows likewise
                GemmArgs gt{n1, k, ktop, 1.0, 0.0, 0.0, 0.0, Qblk, n, Ui, k, Qnb, n, GEMM_FULL, 1, nullptr};
                gt.acol = mi.ctop;
                gt.brow = mi.rtop;
                gt.ccol = mi.posnd;
                BDG_TRY((gemm<double, false>('N', 'N', gt, q)));
                GemmArgs gb{K - n1, k, kbot, 1.0, 0.0, 0.0, 0.0, Qblk + n1, n, Ui, k, Qnb + n1, n, GEMM_FULL, 1,
                            nullptr};
                gb.acol = mi.cbot;
                gb.brow = mi.rbot;
                gb.ccol = mi.posnd;
                BDG_TRY((gemm<double, false>('N', 'N', gb, q)));
            }
        }
        BDG_TRY(join());
    }
    BDG_HIP(hipMemcpyAsync(lam_out, Lbuf[depth % 2], 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
    int errh = 0;
    BDG_HIP(hipMemcpyAsync(&errh, ms.err, sizeof(int), hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    if (errh) {
        set_error("stedc: secular equation did not converge");
        return BDG_ERR_NOCONV;
    }
    return 0;
}

}  // namespace bdg
