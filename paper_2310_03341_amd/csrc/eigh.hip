// bdg_eigh driver: dense Hermitian -> band -> real tridiagonal -> divide and
// conquer -> window selection -> back-transformations (the 2-stage solver of
// the paper's diagonalisation section, with the energy window of the density
// sums, "Methods").
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <vector>

#include "refine.h"
#include "solver.h"
#include "stages.h"

namespace bdg {
namespace {

constexpr int DEFAULT_BAND = 64;

struct Layout {
    int b;
    int64_t ldab, np, nrefl;
    size_t off_AB, off_T1, off_V2, off_tau2, off_voff, off_d, off_ec, off_ea, off_ph, off_Y, off_W2,
        off_flag, off_scratch, scratch, total;
};

size_t al(size_t x) { return (x + 255) / 256 * 256; }

Layout layout(int64_t n, const bdg_opts *o) {
    Layout L;
    L.b = (o && o->band > 0) ? o->band : DEFAULT_BAND;
    if (L.b > 64) L.b = 64;
    if (n <= 2) L.b = 1;
    L.ldab = 2 * L.b + 2;
    L.np = he2hb_panels(n, L.b);
    L.nrefl = hb2st_nrefl(n, L.b);
    size_t o_ = 0;
    auto put = [&](size_t bytes) { size_t r = o_; o_ += al(bytes); return r; };
    L.off_AB = put(16 * (size_t)L.ldab * n);
    L.off_T1 = put(16 * (size_t)(L.np + 1) * L.b * L.b);
    L.off_V2 = put(16 * (size_t)(L.nrefl + 1) * L.b);
    L.off_tau2 = put(8 * (size_t)(L.nrefl + 1));
    L.off_voff = put(8 * (size_t)(n + 1));
    L.off_d = put(8 * (size_t)n);
    L.off_ec = put(16 * (size_t)n);
    L.off_ea = put(8 * (size_t)n);
    L.off_ph = put(16 * (size_t)n);
    L.off_Y = put(8 * (size_t)n * n);
    L.off_W2 = put(8 * (size_t)n);
    L.off_flag = put(256);
    // scratch shared by the stages (they run one after another)
    size_t sc = he2hb_workspace(n, L.b);
    sc = std::max(sc, stedc_workspace(n));
    sc = std::max(sc, bt2_workspace(n, L.b));
    sc = std::max(sc, bt1_workspace(n, n, L.b));
    L.off_scratch = put(sc);
    L.scratch = sc;
    L.total = o_ + 256;
    return L;
}

__global__ void nonfinite_lower(int64_t n, const double *__restrict__ A, int64_t lda, int *flag) {
    const int64_t j = blockIdx.x;
    int bad = 0;
    for (int64_t i = j + threadIdx.x; i < n; i += blockDim.x) {
        const double re = A[2 * (i + j * lda)], im = A[2 * (i + j * lda) + 1];
        if (!isfinite(re) || !isfinite(im)) bad = 1;
    }
    if (bad) atomicOr(flag, 1);
}

// The phase scan (one thread, sequential over the sub-diagonal) runs on the
// side stream beside the divide and conquer: it reads the complex sub-diagonal
// and writes the phase vector, which only the phase scaling after the D&C
// reads; the D&C itself needs |e| only (phase_abs, on the caller's stream).
struct SideScan {
    hipEvent_t ready = nullptr, done = nullptr;
    ~SideScan() {
        if (ready) (void)hipEventDestroy(ready);
        if (done) (void)hipEventDestroy(done);
    }
    int start(int64_t n, const double *ec, double *ph, hipStream_t s) {
        hipStream_t s2 = side_stream();
        if (!s2 || hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&done, hipEventDisableTiming) != hipSuccess) {
            if (done) (void)hipEventDestroy(done);
            done = nullptr;
            return phase_scan(n, ec, ph, s);  // in order on the caller's stream
        }
        BDG_HIP(hipEventRecord(ready, s));
        BDG_HIP(hipStreamWaitEvent(s2, ready, 0));
        BDG_TRY(phase_scan(n, ec, ph, s2));
        BDG_HIP(hipEventRecord(done, s2));
        return 0;
    }
    // the caller's stream waits for the scan
    int join(hipStream_t s) {
        if (done) BDG_HIP(hipStreamWaitEvent(s, done, 0));
        return 0;
    }
};

struct Timer {
    hipStream_t s;
    hipEvent_t ev[12];
    bool ok = false;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    explicit Timer(hipStream_t st) : s(st) {
        ok = true;
        for (int i = 0; i < 12; ++i)
            if (hipEventCreate(&ev[i]) != hipSuccess) ok = false;
    }
    ~Timer() {
        for (int i = 0; i < 12; ++i) (void)hipEventDestroy(ev[i]);
    }
    // what: stage just finished; with BDG_VERBOSE set, waits for it and prints
    // the elapsed wall time to stderr (long solves report their own progress)
    void mark(int i, const char *what = nullptr) {
        if (ok) (void)hipEventRecord(ev[i], s);
        if (what && verbose()) {
            (void)hipStreamSynchronize(s);
            const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            fprintf(stderr, "[bdg] %s done, %.2f s\n", what, sec);
            fflush(stderr);
        }
    }
    double ms(int a, int b) {
        float t = 0.f;
        if (!ok || hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0.0;
        return (double)t;
    }
};

}  // namespace

struct MLayout {
    int b;
    int64_t ldab, np, nrefl, mcap;
    size_t off_AB, off_T1, off_V2, off_tau2, off_voff, off_d, off_ec, off_ea, off_ph, off_W2,
        off_lam, off_flag, off_R1, off_R2, off_R3, r3_bytes, total;
};

// Window columns the refinement buffers are sized for: max_pairs (0 = n) plus
// room for the guard band around the window (see eigh_mixed).
int64_t refine_capacity(int64_t n, const bdg_opts *o) {
    const int64_t mp = (o && o->max_pairs > 0) ? o->max_pairs : n;
    return std::min<int64_t>(n, mp + mp / 64 + 64);
}

// Mixed-precision workspace.  While the FP32 stages run:
//   R1 = A32 (n x n complex64, holds the stage-1 reflectors for BT1),
//   R2 = Y (n x n f64 tridiagonal eigenvectors), overwritten in place by the
//        FP32 basis X32 (n x n complex64: the same 8-byte elements),
//   R3 = stage scratch (D&C buffers, BT2 block factors and row-major Z, ...).
// Once the basis is complete:
//   R3 = X64, the FP64 basis (n x n complex128),
//   R1 + R2 (+ a tail when needed) = refinement buffers for mcap columns.
MLayout mlayout(int64_t n, const bdg_opts *o) {
    MLayout L;
    L.b = (o && o->band > 0) ? o->band : DEFAULT_BAND;
    if (L.b > 64) L.b = 64;
    if (n <= 2) L.b = 1;
    L.ldab = 2 * L.b + 2;
    L.np = he2hb_panels(n, L.b);
    L.nrefl = hb2st_nrefl(n, L.b);
    L.mcap = refine_capacity(n, o);
    size_t o_ = 0;
    auto put = [&](size_t bytes) { size_t r = o_; o_ += al(bytes); return r; };
    const size_t nn = (size_t)n * n;
    L.off_AB = put(8 * (size_t)L.ldab * n);
    L.off_T1 = put(8 * (size_t)(L.np + 1) * L.b * L.b);
    L.off_V2 = put(8 * (size_t)(L.nrefl + 1) * L.b);
    L.off_tau2 = put(4 * (size_t)(L.nrefl + 1));
    L.off_voff = put(8 * (size_t)(n + 1));
    L.off_d = put(8 * (size_t)n);
    L.off_ec = put(16 * (size_t)n);
    L.off_ea = put(8 * (size_t)n);
    L.off_ph = put(16 * (size_t)n);
    L.off_W2 = put(8 * (size_t)n);
    L.off_lam = put(8 * (size_t)n);
    L.off_flag = put(256);
    L.off_R1 = put(8 * nn);
    L.off_R2 = put(8 * nn);
    const size_t rw = refine_workspace(n, L.mcap);
    const size_t span = o_ - L.off_R1;
    if (rw > span) put(rw - span);
    size_t sc = std::max(he2hb_workspace(n, L.b), stedc_workspace(n));
    sc = std::max(sc, bt2_workspace(n, L.b));
    sc = std::max(sc, bt1_workspace(n, n, L.b));
    L.r3_bytes = std::max(sc, 16 * nn);
    L.off_R3 = put(L.r3_bytes);
    L.total = o_ + 256;
    return L;
}

int eigh_workspace(int64_t n, const bdg_opts *opts, size_t *bytes) {
    if (opts && opts->precision != BDG_FP64 && opts->precision != BDG_FP32_REFINED) {
        set_error("bdg_eigh: unknown precision %d", opts->precision);
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    *bytes = (opts && opts->precision == BDG_FP32_REFINED) ? mlayout(n, opts).total : layout(n, opts).total;
    return 0;
}

__global__ void neg_reverse(int64_t half, const double *__restrict__ W, double *__restrict__ lam) {
    // lam[half - 1 - j] = -W[half + j], lam[half + j] = W[half + j]
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < half;
         j += (int64_t)gridDim.x * blockDim.x) {
        const double w = W[half + j];
        lam[half - 1 - j] = -w;
        lam[half + j] = w;
    }
}

// Z[:, j] = X[:, src[j]] for src[j] >= 0, and the particle-hole partner
// (-conj(v), conj(u)) of X[:, -src[j] - 1] otherwise ([u; v] split at n/2).
__global__ void gather_columns_ph(int64_t n, const double *__restrict__ X, int64_t ldx,
                                  const int64_t *__restrict__ src, double *__restrict__ Z, int64_t ldz) {
    const int64_t j = blockIdx.x;
    const int64_t c = src[j];
    double *dst = Z + 2 * j * ldz;
    if (c >= 0) {
        const double *x = X + 2 * c * ldx;
        for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
            dst[2 * i] = x[2 * i];
            dst[2 * i + 1] = x[2 * i + 1];
        }
    } else {
        const double *x = X + 2 * (-c - 1) * ldx;
        const int64_t ns = n / 2;
        for (int64_t r = threadIdx.x; r < ns; r += blockDim.x) {
            const double ur = x[2 * r], ui = x[2 * r + 1];
            const double vr = x[2 * (ns + r)], vi = x[2 * (ns + r) + 1];
            dst[2 * r] = -vr;
            dst[2 * r + 1] = vi;
            dst[2 * (ns + r)] = ur;
            dst[2 * (ns + r) + 1] = -ui;
        }
    }
}

// Relative width of the guard band around the window, in units of ||H||_2:
// the window is taken on refined eigenvalues, and the FP32 stages place an
// eigenvalue within a few 1e-6 ||H||_2 of its FP64 value at the sizes of this
// library, so every eigenvalue that may end up inside the window is refined.
constexpr double WINDOW_GUARD = 1e-4;

int eigh_mixed(int64_t n, double *A, int64_t lda, double emin, double emax, double *W, double *Z,
               int64_t ldz, int64_t zcols, int64_t *m_out, const bdg_opts *opts, void *work,
               bdg_err_report *report, hipStream_t s) {
    const MLayout L = mlayout(n, opts);
    const int b = L.b;
    char *base = (char *)work;
    float *AB = (float *)(base + L.off_AB);
    float *T1 = (float *)(base + L.off_T1);
    float *V2 = (float *)(base + L.off_V2);
    float *tau2 = (float *)(base + L.off_tau2);
    int64_t *voff = (int64_t *)(base + L.off_voff);
    double *d = (double *)(base + L.off_d);
    double *ec = (double *)(base + L.off_ec);
    double *ea = (double *)(base + L.off_ea);
    double *ph = (double *)(base + L.off_ph);
    double *W2 = (double *)(base + L.off_W2);
    double *lam = (double *)(base + L.off_lam);
    int *flag = (int *)(base + L.off_flag);
    float *A32 = (float *)(base + L.off_R1);
    double *Y = (double *)(base + L.off_R2);
    float *X32 = (float *)(base + L.off_R2);  // overwrites Y in place
    void *scratch = base + L.off_R3;
    double *X64 = (double *)(base + L.off_R3);  // once the stage scratch is dead
    void *rscratch = base + L.off_R1;           // R1 + R2 (+ tail) once A32 and X32 are dead
    const int leaf = (opts && opts->dc_leaf > 0) ? opts->dc_leaf : 32;
    const bool ph_mirror = opts && opts->ph_mirror && (n % 2 == 0);
    // refine_max_iter: 0 = default (4), < 0 = no refinement (the FP32 result)
    const int iters = (opts && opts->refine_max_iter != 0) ? std::max(opts->refine_max_iter, 0) : 4;
    const double rtol = (opts && opts->refine_tol > 0.0) ? opts->refine_tol : 1e-14;

    Timer tm(s);
    tm.mark(0);
    BDG_HIP(hipMemsetAsync(flag, 0, 4, s));
    hipLaunchKernelGGL(nonfinite_lower, dim3((unsigned)n), dim3(256), 0, s, n, A, lda, flag);
    BDG_CHECK_LAUNCH();
    int hflag = 0;
    BDG_HIP(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    if (hflag) {
        set_error("bdg_eigh: the input matrix holds NaN or Inf");
        return BDG_ERR_NONFINITE;
    }
    BDG_TRY(cast_c128_to_c64(n, n, A, lda, A32, n, s));
    tm.mark(1, "input check + cast to FP32");
    BDG_TRY(he2hb(n, A32, n, b, AB, L.ldab, T1, scratch, s));
    tm.mark(2, "he2hb");
    if (n >= 3) {
        std::vector<int64_t> vh((size_t)(n - 2));
        hb2st_offsets(n, b, vh.data());
        BDG_HIP(hipMemcpyAsync(voff, vh.data(), 8 * (size_t)(n - 2), hipMemcpyHostToDevice, s));
        BDG_HIP(hipStreamSynchronize(s));
    }
    BDG_TRY(hb2st(n, b, AB, L.ldab, V2, tau2, d, ec, s));
    BDG_TRY(phase_abs(n, ec, ea, s));
    SideScan scan;
    BDG_TRY(scan.start(n, ec, ph, s));
    tm.mark(3, "hb2st");
    {
        const int rc = stedc(n, d, ea, W2, Y, n, scratch, s, leaf);
        BDG_TRY(scan.join(s));
        BDG_TRY(rc);
    }
    tm.mark(4, "stedc");
    // FP32 basis: all columns, or the E >= 0 half and its particle-hole partners
    const int64_t c0 = ph_mirror ? n / 2 : 0;
    const int64_t nc = n - c0;
    // row-major route for the back-transformation 2 as in the FP64 driver
    const size_t tf_bytes = al(bt2_workspace(n, b));
    const bool rm = n >= 3 && nc > 0 && bt2_rowmajor_ok(b) && tf_bytes + 8 * (size_t)n * nc <= L.r3_bytes;
    float *Zrm = (float *)((char *)scratch + tf_bytes);
    if (rm) BDG_TRY(phase_scale_rm(n, nc, Y, c0, ph, Zrm, nc, s));
    else BDG_TRY(phase_scale(n, nc, Y, c0, ph, X32 + 2 * c0 * n, n, s));  // in place over Y
    tm.mark(5, "phase scaling");
    BDG_TRY(bt2_prepare(n, b, V2, tau2, voff, scratch, s));
    tm.mark(10);
    if (rm) BDG_TRY(bt2_apply_blocks_rm(n, b, nc, V2, voff, Zrm, nc, scratch, s));
    else BDG_TRY(bt2_apply_blocks(n, b, nc, V2, voff, X32 + 2 * c0 * n, n, scratch, s));
    tm.mark(11);
    if (rm) BDG_TRY(rm_to_cm(n, nc, Zrm, nc, X32 + 2 * c0 * n, n, s));
    tm.mark(6, "bt2");
    BDG_TRY(bt1(n, nc, A32, n, b, T1, X32 + 2 * c0 * n, n, scratch, s));
    if (ph_mirror) {
        BDG_TRY(mirror_half(n, X32, n, s));
        hipLaunchKernelGGL(neg_reverse, dim3(64), dim3(256), 0, s, n / 2, W2, lam);
        BDG_CHECK_LAUNCH();
    } else {
        BDG_HIP(hipMemcpyAsync(lam, W2, 8 * (size_t)n, hipMemcpyDeviceToDevice, s));
    }
    // the stage scratch is dead: the FP64 basis takes its place
    BDG_TRY(cast_c64_to_c128(n, n, X32, n, X64, n, s));
    tm.mark(7, "bt1");
    // Refine every eigenvalue that may belong to the window: the FP32 values
    // widened by a guard band; the window itself is cut on refined values.
    std::vector<double> wh((size_t)n);
    BDG_HIP(hipMemcpyAsync(wh.data(), lam, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    double normH = 0.0;
    for (double v : wh) normH = std::max(normH, std::fabs(v));
    const double guard = WINDOW_GUARD * normH;
    const int64_t i0 = std::lower_bound(wh.begin(), wh.end(), emin - guard) - wh.begin();
    const int64_t i1 = std::upper_bound(wh.begin(), wh.end(), emax + guard) - wh.begin();
    // with the mirror, a window that holds the partner of every E < 0 pair only
    // needs its E >= 0 half refined; the E < 0 half is rebuilt from it
    const int64_t h = n / 2;
    const bool mir = ph_mirror && i0 < h && i1 > h && n - i0 <= i1;
    const int64_t r0 = mir ? h : i0;
    const int64_t mr = i1 > r0 ? i1 - r0 : 0;
    if (mr > L.mcap) {
        set_error("bdg_eigh: %lld eigenpairs to refine exceed the workspace's %lld (set opts.max_pairs)",
                  (long long)mr, (long long)L.mcap);
        *m_out = mr;
        return BDG_ERR_WORKSPACE;
    }
    double shift = 0.0, corr = 0.0;
    int done = 0, close0 = 0, ccols = 0;
    if (iters > 0 && mr > 0) {
        BDG_TRY(refine_window(n, A, lda, X64, n, lam, r0, mr, normH, iters, rtol, W, rscratch, s, &shift, &corr,
                              &done, &close0, &ccols));
    } else if (mr > 0) {  // refinement switched off: the FP32 result, widened
        BDG_HIP(hipMemcpyAsync(W, lam + r0, 8 * (size_t)mr, hipMemcpyDeviceToDevice, s));
    }
    tm.mark(8, "refinement");
    // Cut the window on the refined eigenvalues and put it in ascending order
    // (a pair closer than the FP32 basis could separate, refined column by
    // column, can converge with its two columns swapped).  Codes of the source
    // columns: c >= 0 copies X64 column c, -c - 1 takes its partner (-v*, u*).
    std::vector<double> wr((size_t)mr);
    if (mr > 0) {
        BDG_HIP(hipMemcpyAsync(wr.data(), W, 8 * (size_t)mr, hipMemcpyDeviceToHost, s));
        BDG_HIP(hipStreamSynchronize(s));
    }
    std::vector<std::pair<double, int64_t>> sel;
    sel.reserve((size_t)(mir ? 2 * mr : mr));
    for (int64_t k = 0; k < mr; ++k) {
        const double w = wr[k];
        if (w >= emin && w <= emax) sel.emplace_back(w, r0 + k);
        if (mir && -w >= emin && -w <= emax) sel.emplace_back(-w, -(r0 + k) - 1);
    }
    std::stable_sort(sel.begin(), sel.end(),
                     [](const std::pair<double, int64_t> &a, const std::pair<double, int64_t> &c) {
                         return a.first < c.first;
                     });
    const int64_t m = (int64_t)sel.size();
    *m_out = m;
    if (m > zcols) {
        set_error("bdg_eigh: %lld eigenpairs in the window exceed zcols=%lld", (long long)m, (long long)zcols);
        return BDG_ERR_WORKSPACE;
    }
    if (m > 0) {
        std::vector<double> ws((size_t)m);
        std::vector<int64_t> src((size_t)m);
        for (int64_t j = 0; j < m; ++j) {
            ws[j] = sel[j].first;
            src[j] = sel[j].second;
        }
        int64_t *srcd = (int64_t *)rscratch;  // the refinement buffers are dead
        BDG_HIP(hipMemcpyAsync(srcd, src.data(), 8 * (size_t)m, hipMemcpyHostToDevice, s));
        BDG_HIP(hipMemcpyAsync(W, ws.data(), 8 * (size_t)m, hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(gather_columns_ph, dim3((unsigned)m), dim3(256), 0, s, n, X64, n, srcd, Z, ldz);
        BDG_CHECK_LAUNCH();
        BDG_HIP(hipStreamSynchronize(s));  // the host vectors go out of scope
    }
    tm.mark(9, "window");
    BDG_HIP(hipStreamSynchronize(s));
    if (report) {
        memset(report, 0, sizeof(*report));
        report->stage_ms[0] = tm.ms(1, 2);
        report->stage_ms[1] = tm.ms(2, 3);
        report->stage_ms[2] = tm.ms(3, 4);
        report->stage_ms[3] = tm.ms(5, 6);
        report->stage_ms[4] = tm.ms(6, 7);
        report->stage_ms[5] = tm.ms(7, 8);
        report->stage_ms[6] = tm.ms(4, 5) + tm.ms(8, 9);
        report->stage_ms[7] = tm.ms(0, 9);
        report->eig_shift_max = shift;
        report->refine_iters = done;
        report->max_resid = corr;  // last defect (the residual itself is measured by bdg_check)
        report->bt2_kernel_ms = tm.ms(10, 11);
        report->refine_close_pairs = close0;
        report->refine_cluster_cols = ccols;
    }
    if (iters > 0 && mr > 0 && corr >= std::sqrt(rtol)) {
        set_error("bdg_eigh: refinement stopped after %d steps with defect %.3e", done, corr);
        return BDG_ERR_REFINE_TOL;
    }
    return 0;
}

int eigh(int64_t n, double *A, int64_t lda, double emin, double emax, double *W, double *Z,
         int64_t ldz, int64_t zcols, int64_t *m_out, const bdg_opts *opts, void *work,
         size_t work_bytes, bdg_err_report *report, hipStream_t s) {
    (void)work_bytes;
    if (opts && opts->precision == BDG_FP32_REFINED)
        return eigh_mixed(n, A, lda, emin, emax, W, Z, ldz, zcols, m_out, opts, work, report, s);
    if (opts && opts->precision != BDG_FP64) {
        set_error("bdg_eigh: unknown precision %d", opts->precision);
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    const Layout L = layout(n, opts);
    const int b = L.b;
    char *base = (char *)work;
    double *AB = (double *)(base + L.off_AB);
    double *T1 = (double *)(base + L.off_T1);
    double *V2 = (double *)(base + L.off_V2);
    double *tau2 = (double *)(base + L.off_tau2);
    int64_t *voff = (int64_t *)(base + L.off_voff);
    double *d = (double *)(base + L.off_d);
    double *ec = (double *)(base + L.off_ec);
    double *ea = (double *)(base + L.off_ea);
    double *ph = (double *)(base + L.off_ph);
    double *Y = (double *)(base + L.off_Y);
    double *W2 = (double *)(base + L.off_W2);
    int *flag = (int *)(base + L.off_flag);
    void *scratch = base + L.off_scratch;
    const int leaf = (opts && opts->dc_leaf > 0) ? opts->dc_leaf : 32;

    Timer tm(s);
    tm.mark(0);
    // reject NaN/Inf before touching anything
    BDG_HIP(hipMemsetAsync(flag, 0, 4, s));
    hipLaunchKernelGGL(nonfinite_lower, dim3((unsigned)n), dim3(256), 0, s, n, A, lda, flag);
    BDG_CHECK_LAUNCH();
    int hflag = 0;
    BDG_HIP(hipMemcpyAsync(&hflag, flag, 4, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    if (hflag) {
        set_error("bdg_eigh: the input matrix holds NaN or Inf");
        return BDG_ERR_NONFINITE;
    }
    tm.mark(1, "input check");
    // ---- stage 1: dense -> band
    BDG_TRY(he2hb(n, A, lda, b, AB, L.ldab, T1, scratch, s));
    tm.mark(2, "he2hb");
    // ---- stage 2: band -> tridiagonal
    if (n >= 3) {
        std::vector<int64_t> vh((size_t)(n - 2));
        hb2st_offsets(n, b, vh.data());
        BDG_HIP(hipMemcpyAsync(voff, vh.data(), 8 * (size_t)(n - 2), hipMemcpyHostToDevice, s));
        BDG_HIP(hipStreamSynchronize(s));  // vh goes out of scope
    }
    BDG_TRY(hb2st(n, b, AB, L.ldab, V2, tau2, d, ec, s));
    BDG_TRY(phase_abs(n, ec, ea, s));
    SideScan scan;
    BDG_TRY(scan.start(n, ec, ph, s));
    tm.mark(3, "hb2st");
    // ---- tridiagonal divide and conquer
    {
        const int rc = stedc(n, d, ea, W2, Y, n, scratch, s, leaf);
        BDG_TRY(scan.join(s));
        BDG_TRY(rc);
    }
    tm.mark(4, "stedc");
    // ---- window
    std::vector<double> wh((size_t)n);
    BDG_HIP(hipMemcpyAsync(wh.data(), W2, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    const int64_t i0 = std::lower_bound(wh.begin(), wh.end(), emin) - wh.begin();
    const int64_t i1 = std::upper_bound(wh.begin(), wh.end(), emax) - wh.begin();
    const int64_t m = i1 > i0 ? i1 - i0 : 0;
    *m_out = m;
    if (m > zcols) {
        set_error("bdg_eigh: %lld eigenpairs in the window exceed zcols=%lld", (long long)m,
                  (long long)zcols);
        return BDG_ERR_WORKSPACE;
    }
    BDG_HIP(hipMemcpyAsync(W, W2 + i0, 8 * (size_t)m, hipMemcpyDeviceToDevice, s));
    // Particle-hole mirror: when the window straddles E = 0 and every negative
    // eigenvalue's partner n-1-i lies inside it, only the E > 0 columns are
    // back-transformed and the others are built as (-v^*, u^*).
    const int64_t h = n / 2;
    int64_t bt_lo = i0, bt_hi = i1;
    bool mirror = false;
    if (opts && opts->ph_mirror && (n % 2 == 0) && i0 < h && i1 > h && n - i0 <= i1) {
        mirror = true;
        bt_lo = h;
    }
    const int64_t mb = bt_hi - bt_lo;
    double *Zb = Z + 2 * (bt_lo - i0) * ldz;
    // back-transformation 2 on a row-major copy of Z when the scratch holds it
    // after the block T factors (rows of a block are then contiguous)
    const size_t tf_bytes = al(bt2_workspace(n, b));
    const bool rm = n >= 3 && mb > 0 && bt2_rowmajor_ok(b) && tf_bytes + 16 * (size_t)n * mb <= L.scratch;
    double *Zrm = (double *)((char *)scratch + tf_bytes);
    if (rm) BDG_TRY(phase_scale_rm(n, mb, Y, bt_lo, ph, Zrm, mb, s));
    else BDG_TRY(phase_scale(n, mb, Y, bt_lo, ph, Zb, ldz, s));
    tm.mark(5, "window + phase scaling");
    // ---- back-transformation 2 (band <- tridiagonal), then 1 (dense <- band)
    BDG_TRY(bt2_prepare(n, b, V2, tau2, voff, scratch, s));
    tm.mark(8);
    if (rm) BDG_TRY(bt2_apply_blocks_rm(n, b, mb, V2, voff, Zrm, mb, scratch, s));
    else BDG_TRY(bt2_apply_blocks(n, b, mb, V2, voff, Zb, ldz, scratch, s));
    tm.mark(9);
    if (rm) BDG_TRY(rm_to_cm(n, mb, Zrm, mb, Zb, ldz, s));
    tm.mark(6, "bt2");
    BDG_TRY(bt1(n, mb, A, lda, b, T1, Zb, ldz, scratch, s));
    if (mirror) BDG_TRY(mirror_columns(n, Z, ldz, 0, (n - 1 - i0) - i0, h - i0, s));
    tm.mark(7, "bt1");
    BDG_HIP(hipStreamSynchronize(s));
    if (report) {
        memset(report, 0, sizeof(*report));
        report->stage_ms[0] = tm.ms(1, 2);
        report->stage_ms[1] = tm.ms(2, 3);
        report->stage_ms[2] = tm.ms(3, 4);
        report->stage_ms[3] = tm.ms(5, 6);
        report->stage_ms[4] = tm.ms(6, 7);
        report->stage_ms[5] = 0.0;
        report->stage_ms[6] = tm.ms(4, 5);
        report->stage_ms[7] = tm.ms(0, 7);
        report->bt2_kernel_ms = tm.ms(8, 9);
    }
    return 0;
}

// bdg_refine: refinement of columns [i0, i0 + m) of the basis X.
int refine_pairs(int64_t n, const double *H, int64_t ldh, const double *lam, double *X, int64_t ldx,
                 int64_t i0, int64_t m, double *W, const bdg_opts *opts, void *work,
                 bdg_err_report *report, hipStream_t s) {
    const int iters = (opts && opts->refine_max_iter > 0) ? opts->refine_max_iter : 4;
    const double rtol = (opts && opts->refine_tol > 0.0) ? opts->refine_tol : 1e-14;
    Timer tm(s);
    tm.mark(0);
    // ||H||_2 from the eigenvalues of the whole basis
    std::vector<double> wh((size_t)n);
    BDG_HIP(hipMemcpyAsync(wh.data(), lam, 8 * (size_t)n, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    double normH = 0.0;
    for (double v : wh) {
        if (!std::isfinite(v)) {
            set_error("bdg_refine: lam holds NaN or Inf");
            return BDG_ERR_NONFINITE;
        }
        normH = std::max(normH, std::fabs(v));
    }
    double shift = 0.0, corr = 0.0;
    int done = 0, close0 = 0, ccols = 0;
    if (m > 0)
        BDG_TRY(refine_window(n, H, ldh, X, ldx, lam, i0, m, normH, iters, rtol, W, work, s, &shift, &corr, &done,
                              &close0, &ccols));
    tm.mark(1);
    BDG_HIP(hipStreamSynchronize(s));
    if (report) {
        memset(report, 0, sizeof(*report));
        report->stage_ms[5] = report->stage_ms[7] = tm.ms(0, 1);
        report->eig_shift_max = shift;
        report->refine_iters = done;
        report->max_resid = corr;
        report->refine_close_pairs = close0;
        report->refine_cluster_cols = ccols;
    }
    if (m > 0 && corr >= std::sqrt(rtol)) {
        set_error("bdg_refine: stopped after %d steps with defect %.3e", done, corr);
        return BDG_ERR_REFINE_TOL;
    }
    return 0;
}

}  // namespace bdg
