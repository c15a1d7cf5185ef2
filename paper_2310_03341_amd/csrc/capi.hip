// C-ABI entry points of libbdg.so (declared in include/bdg.h).
#include <math.h>
#include <stdlib.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include "common.h"
#include "gemm.h"
#include "net.h"
#include "refine.h"
#include "solver.h"

namespace bdg {

static thread_local char g_err[512] = "no error";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

bool verbose() {
    static const bool v = [] {
        const char *e = getenv("BDG_VERBOSE");
        return e && e[0] && e[0] != '0';
    }();
    return v;
}

bool lookahead() {
    static const bool v = [] {
        const char *e = getenv("BDG_NO_LOOKAHEAD");
        return !(e && e[0] && e[0] != '0');
    }();
    return v;
}

int hip_fail(hipError_t e, const char *what, const char *file, int line) {
    set_error("HIP error %d (%s) in %s at %s:%d", (int)e, hipGetErrorString(e), what, file, line);
    return BDG_ERR_HIP;
}

}  // namespace bdg

using namespace bdg;

extern "C" {

const char *bdg_last_error(void) { return bdg::g_err; }

const char *bdg_version(void) { return "bdg-mi355x 0.1 (gfx950)"; }

int bdg_assemble(const bdg_lattice *lat, const double *U, const double *Delta, double mu,
                 double *H, int64_t ldh, bdg_stream_t stream) {
    if (!lat || lat->ndim < 1 || lat->ndim > 3) {
        set_error("bdg_assemble: lattice must have ndim in 1..3");
        return -1;
    }
    int64_t ns = 1;
    for (int d = 0; d < lat->ndim; ++d) {
        const int N = lat->dims[d];
        if (N < 2 || (N & 1) || N > 64) {
            set_error("bdg_assemble: dims[%d]=%d must be even and in [2, 64]", d, N);
            return -1;
        }
        ns *= N;
    }
    if (!U) { set_error("bdg_assemble: U is NULL"); return -2; }
    if (!Delta) { set_error("bdg_assemble: Delta is NULL"); return -3; }
    if (!H) { set_error("bdg_assemble: H is NULL"); return -5; }
    if (ldh < 2 * ns) { set_error("bdg_assemble: ldh=%lld < n=%lld", (long long)ldh, (long long)(2 * ns)); return -6; }
    return bdg::assemble(lat, U, Delta, mu, H, ldh, (hipStream_t)stream);
}

// op 'T' (transpose without conjugation) only for real products, where it is 'C'
static int check_gemm_args(char opA, char opB, int64_t M, int64_t N, int64_t K, const void *A,
                           int64_t lda, const void *B, int64_t ldb, void *C, int64_t ldc, bool real) {
    auto okop = [real](char o) {
        return o == 'N' || o == 'n' || o == 'C' || o == 'c' || (real && (o == 'T' || o == 't'));
    };
    if (!okop(opA)) { set_error("gemm: bad opA"); return -1; }
    if (!okop(opB)) { set_error("gemm: bad opB"); return -2; }
    if (M < 0) return -3;
    if (N < 0) return -4;
    if (K < 0) return -5;
    const bool na = (opA == 'N' || opA == 'n'), nb = (opB == 'N' || opB == 'n');
    if (M && N && K && !A) return -7;
    if (lda < (na ? (M > 0 ? M : 1) : (K > 0 ? K : 1))) { set_error("gemm: lda too small"); return -8; }
    if (M && N && K && !B) return -9;
    if (ldb < (nb ? (K > 0 ? K : 1) : (N > 0 ? N : 1))) { set_error("gemm: ldb too small"); return -10; }
    if (M && N && !C) return -12;
    if (ldc < (M > 0 ? M : 1)) { set_error("gemm: ldc too small"); return -13; }
    return 0;
}

int bdg_zgemm(char opA, char opB, int64_t M, int64_t N, int64_t K, const double *alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, const double *beta,
              double *C, int64_t ldc, bdg_stream_t stream) {
    BDG_TRY(check_gemm_args(opA, opB, M, N, K, A, lda, B, ldb, C, ldc, false));
    GemmArgs g{M, N, K, alpha[0], alpha[1], beta[0], beta[1], A, lda, B, ldb, C, ldc, GEMM_FULL, 1, nullptr};
    return gemm<double, true>(opA, opB, g, (hipStream_t)stream);
}

int bdg_cgemm(char opA, char opB, int64_t M, int64_t N, int64_t K, const float *alpha,
              const float *A, int64_t lda, const float *B, int64_t ldb, const float *beta,
              float *C, int64_t ldc, bdg_stream_t stream) {
    BDG_TRY(check_gemm_args(opA, opB, M, N, K, A, lda, B, ldb, C, ldc, false));
    GemmArgs g{M, N, K, alpha[0], alpha[1], beta[0], beta[1], A, lda, B, ldb, C, ldc, GEMM_FULL, 1, nullptr};
    return gemm<float, true>(opA, opB, g, (hipStream_t)stream);
}

int bdg_dgemm(char opA, char opB, int64_t M, int64_t N, int64_t K, double alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
              double *C, int64_t ldc, bdg_stream_t stream) {
    BDG_TRY(check_gemm_args(opA, opB, M, N, K, A, lda, B, ldb, C, ldc, true));
    GemmArgs g{M, N, K, alpha, 0.0, beta, 0.0, A, lda, B, ldb, C, ldc, GEMM_FULL, 1, nullptr};
    return gemm<double, false>(opA, opB, g, (hipStream_t)stream);
}

int bdg_check(int64_t n, const double *H, int64_t ldh, int64_t m, const double *W,
              const double *Z, int64_t ldz, double *max_resid, double *gram_defect, void *work,
              size_t work_bytes, bdg_stream_t stream) {
    if (n < 1) return -1;
    if (!H) return -2;
    if (ldh < n) return -3;
    if (m < 0 || m > n) return -4;
    if (m > 0 && !W) return -5;
    if (m > 0 && !Z) return -6;
    if (ldz < n) return -7;
    if (!max_resid) return -8;
    if (!gram_defect) return -9;
    const size_t need = 16 * ((size_t)n * m + (size_t)m * m) + 64;
    if (work_bytes < need || !work) {
        set_error("bdg_check: workspace %zu < %zu bytes", work_bytes, need);
        return BDG_ERR_WORKSPACE;
    }
    return bdg::check_pairs(n, H, ldh, m, W, Z, ldz, max_resid, gram_defect, work, (hipStream_t)stream);
}

}  // extern "C"

extern "C" {

int bdg_eigh_workspace(int64_t n, const bdg_opts *opts, size_t *bytes) {
    if (n < 1) { set_error("bdg_eigh_workspace: n must be >= 1"); return -1; }
    if (!bytes) return -3;
    return bdg::eigh_workspace(n, opts, bytes);
}

int bdg_eigh(int64_t n, double *A, int64_t lda, double emin, double emax, double *W, double *Z,
             int64_t ldz, int64_t zcols, int64_t *m, const bdg_opts *opts, void *work,
             size_t work_bytes, bdg_err_report *report, bdg_stream_t stream) {
    if (n < 1) { set_error("bdg_eigh: n must be >= 1"); return -1; }
    if (!A) return -2;
    if (lda < n) { set_error("bdg_eigh: lda < n"); return -3; }
    if (!(emin <= emax)) { set_error("bdg_eigh: emin > emax or NaN"); return -4; }
    if (!W) return -6;
    if (!Z) return -7;
    if (ldz < n) { set_error("bdg_eigh: ldz < n"); return -8; }
    if (zcols < 0) return -9;
    if (!m) return -10;
    size_t need = 0;
    BDG_TRY(bdg::eigh_workspace(n, opts, &need));
    if (!work || work_bytes < need) {
        set_error("bdg_eigh: workspace %zu < %zu bytes", work_bytes, need);
        return BDG_ERR_WORKSPACE;
    }
    return bdg::eigh(n, A, lda, emin, emax, W, Z, ldz, zcols, m, opts, work, work_bytes, report,
                     (hipStream_t)stream);
}

int bdg_gemm_int8_workspace(int32_t cplx, int64_t M, int64_t N, int64_t K, int32_t slices, size_t *bytes) {
    if (cplx != 0 && cplx != 1) return -1;
    if (M < 0 || N < 0 || K < 0) return -2;
    if (slices < 3 || slices > 8) return -5;
    if (!bytes) return -6;
    *bytes = bdg::ozaki_workspace(cplx == 1, M, N, K, slices);
    return 0;
}

int bdg_gemm_int8(int32_t cplx, int32_t slices, char opA, char opB, int64_t M, int64_t N, int64_t K,
                  const double *alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                  const double *beta, double *C, int64_t ldc, void *work, size_t work_bytes,
                  bdg_stream_t stream) {
    if (cplx != 0 && cplx != 1) return -1;
    if (slices < 3 || slices > 8) {
        set_error("bdg_gemm_int8: slices must be 3..8");
        return -2;
    }
    BDG_TRY(check_gemm_args(opA, opB, M, N, K, A, lda, B, ldb, C, ldc, cplx == 0));
    if (!alpha || !beta) return -8;
    if (M == 0 || N == 0) return 0;
    if (!work || work_bytes < bdg::ozaki_workspace(cplx == 1, M, N, K, slices)) {
        set_error("bdg_gemm_int8: workspace too small");
        return BDG_ERR_WORKSPACE;
    }
    return bdg::ozaki_gemm(cplx == 1, slices, opA, opB, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, work,
                           (hipStream_t)stream);
}

int bdg_eigh1_workspace(int64_t n, int32_t real, int64_t zcols, size_t *bytes) {
    if (n < 1) return -1;
    if (real != 0 && real != 1) return -2;
    if (zcols < 0) return -3;
    if (!bytes) return -4;
    *bytes = bdg::eigh1_workspace(n, real == 0, zcols);
    return 0;
}

int bdg_eigh1(int64_t n, int32_t real, double *A, int64_t lda, double emin, double emax, double *W,
              double *Z, int64_t ldz, int64_t zcols, int64_t *m, void *work, size_t work_bytes,
              bdg_err_report *report, bdg_stream_t stream) {
    if (n < 1) return -1;
    if (real != 0 && real != 1) return -2;
    if (!A) return -3;
    if (lda < n) return -4;
    if (!(emin <= emax)) return -5;
    if (!W) return -7;
    if (!Z) return -8;
    if (ldz < n) return -9;
    if (zcols < 0) return -10;
    if (!m) return -11;
    if (!work || work_bytes < bdg::eigh1_workspace(n, real == 0, zcols)) {
        set_error("bdg_eigh1: workspace too small");
        return BDG_ERR_WORKSPACE;
    }
    return bdg::eigh1(n, real == 0, A, lda, emin, emax, W, Z, ldz, zcols, m, work, report,
                      (hipStream_t)stream);
}

int bdg_refine_workspace(int64_t n, int64_t m, size_t *bytes) {
    if (n < 1) { set_error("bdg_refine_workspace: n must be >= 1"); return -1; }
    if (m < 0 || m > n) { set_error("bdg_refine_workspace: m must be in [0, n]"); return -2; }
    if (!bytes) return -3;
    *bytes = bdg::refine_workspace(n, m);
    return 0;
}

int bdg_refine(int64_t n, const double *H, int64_t ldh, const double *lam, double *X, int64_t ldx,
               int64_t i0, int64_t m, double *W, const bdg_opts *opts, void *work, size_t work_bytes,
               bdg_err_report *report, bdg_stream_t stream) {
    if (n < 1) { set_error("bdg_refine: n must be >= 1"); return -1; }
    if (!H) return -2;
    if (ldh < n) { set_error("bdg_refine: ldh < n"); return -3; }
    if (!lam) return -4;
    if (!X) return -5;
    if (ldx < n) { set_error("bdg_refine: ldx < n"); return -6; }
    if (i0 < 0 || i0 > n) { set_error("bdg_refine: i0 must be in [0, n]"); return -7; }
    if (m < 0 || i0 + m > n) { set_error("bdg_refine: need 0 <= m and i0 + m <= n"); return -8; }
    if (m > 0 && !W) return -9;
    if (opts && opts->refine_max_iter < 0) { set_error("bdg_refine: refine_max_iter < 0"); return -10; }
    const size_t need = bdg::refine_workspace(n, m);
    if (m > 0 && (!work || work_bytes < need)) {
        set_error("bdg_refine: workspace %zu < %zu bytes", work_bytes, need);
        return BDG_ERR_WORKSPACE;
    }
    return bdg::refine_pairs(n, H, ldh, lam, X, ldx, i0, m, W, opts, work, report, (hipStream_t)stream);
}

}  // extern "C"

// ---------------------------------------------------------------- stage hooks
#include <vector>
#include "stages.h"

extern "C" {

int bdg_stage_workspace(int stage, int64_t n, int band, int64_t m, size_t *bytes) {
    if (!bytes) return -5;
    switch (stage) {
        case 1: *bytes = bdg::he2hb_workspace(n, band); return 0;
        case 2: *bytes = 0; return 0;
        case 3: *bytes = bdg::stedc_workspace(n); return 0;
        case 4:  // phases, T factors, and the row-major copy of Z when the band allows that route
            *bytes = bdg::bt2_workspace(n, band) + 16 * (size_t)n + 8 * (size_t)n + 1024 +
                     (bdg::bt2_rowmajor_ok(band) ? 16 * (size_t)n * (size_t)(m > 0 ? m : 0) : 0);
            return 0;
        case 5: *bytes = bdg::bt1_workspace(n, m, band); return 0;
        default: set_error("bdg_stage_workspace: unknown stage %d", stage); return -1;
    }
}

int64_t bdg_stage_nrefl(int64_t n, int band) { return bdg::hb2st_nrefl(n, band); }

int bdg_stage_he2hb(int64_t n, double *A, int64_t lda, int band, double *AB, int64_t ldab,
                    double *T1, void *work, size_t work_bytes, bdg_stream_t stream) {
    if (n < 1) return -1;
    if (work_bytes < bdg::he2hb_workspace(n, band)) return BDG_ERR_WORKSPACE;
    return bdg::he2hb(n, A, lda, band, AB, ldab, T1, work, (hipStream_t)stream);
}

int bdg_stage_hb2st(int64_t n, int band, double *AB, int64_t ldab, double *d, double *e,
                    double *V2, double *tau2, int64_t *voff, bdg_stream_t stream) {
    if (n < 1) return -1;
    hipStream_t s = (hipStream_t)stream;
    if (n >= 3) {
        std::vector<int64_t> vh((size_t)(n - 2));
        bdg::hb2st_offsets(n, band, vh.data());
        BDG_HIP(hipMemcpyAsync(voff, vh.data(), 8 * (size_t)(n - 2), hipMemcpyHostToDevice, s));
        BDG_HIP(hipStreamSynchronize(s));
    }
    return bdg::hb2st(n, band, AB, ldab, V2, tau2, d, e, s);
}

int bdg_stage_stedc(int64_t n, const double *d, const double *e, double *W, double *Q, int leaf,
                    void *work, size_t work_bytes, bdg_stream_t stream) {
    if (n < 1) return -1;
    if (work_bytes < bdg::stedc_workspace(n)) return BDG_ERR_WORKSPACE;
    return bdg::stedc(n, d, e, W, Q, n, work, (hipStream_t)stream, leaf);
}

int bdg_stage_bt2(int64_t n, int band, int64_t m, const double *e, const double *Y, int64_t i0,
                  const double *V2, const double *tau2, const int64_t *voff, double *Z,
                  int64_t ldz, void *work, size_t work_bytes, bdg_stream_t stream) {
    // workspace of stage 4: with the row-major copy of Z when the band allows
    // it; a workspace without room for that copy takes the column-major route
    size_t need = 0;
    bdg_stage_workspace(4, n, band, m, &need);
    const size_t zrm = bdg::bt2_rowmajor_ok(band) ? 16 * (size_t)n * (size_t)(m > 0 ? m : 0) : 0;
    if (work_bytes < need - zrm) return BDG_ERR_WORKSPACE;
    const bool rm = zrm > 0 && work_bytes >= need;
    hipStream_t s = (hipStream_t)stream;
    char *w = (char *)work;
    auto al = [](size_t x) { return (x + 255) / 256 * 256; };
    double *ph = (double *)w;
    double *ea = (double *)(w + al(16 * (size_t)n));
    void *rest = w + al(16 * (size_t)n) + al(8 * (size_t)n);
    BDG_TRY(bdg::phases(n, e, ph, ea, s));
    if (!rm || n < 3 || m <= 0) {
        BDG_TRY(bdg::phase_scale(n, m, Y, i0, ph, Z, ldz, s));
        return bdg::bt2(n, band, m, V2, tau2, voff, Z, ldz, rest, s);
    }
    // row-major route: Zrm after the T factors
    double *Zrm = (double *)((char *)rest + (bdg::bt2_workspace(n, band) + 255) / 256 * 256);
    BDG_TRY(bdg::phase_scale_rm(n, m, Y, i0, ph, Zrm, m, s));
    BDG_TRY(bdg::bt2_prepare(n, band, V2, tau2, voff, rest, s));
    BDG_TRY(bdg::bt2_apply_blocks_rm(n, band, m, V2, voff, Zrm, m, rest, s));
    return bdg::rm_to_cm(n, m, Zrm, m, Z, ldz, s);
}

int bdg_stage_zgemm(int mode, int splitk, char opA, char opB, int64_t M, int64_t N, int64_t K,
                    const double *alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                    const double *beta, double *C, int64_t ldc, void *work, size_t work_bytes,
                    bdg_stream_t stream) {
    if (mode < GEMM_FULL || mode > GEMM_HEMM_L) { set_error("bdg_stage_zgemm: unknown mode %d", mode); return -1; }
    if (splitk < 1 || splitk > 64) { set_error("bdg_stage_zgemm: splitk must be in [1, 64]"); return -2; }
    BDG_TRY(check_gemm_args(opA, opB, M, N, K, A, lda, B, ldb, C, ldc, false));
    const bool na = (opA == 'N' || opA == 'n');
    if (mode == GEMM_LOWER && (!na || M != N || splitk > 1)) {
        set_error("bdg_stage_zgemm: lower-tile mode needs opA = 'N', M == N and splitk == 1");
        return -1;
    }
    if (mode == GEMM_HEMM_L && (!na || M != K)) {
        set_error("bdg_stage_zgemm: HEMM mode needs opA = 'N' and M == K");
        return -1;
    }
    const size_t need = splitk > 1 ? 16 * gemm_split_elems(M, N, splitk) : 0;
    if (need && (!work || work_bytes < need)) {
        set_error("bdg_stage_zgemm: workspace %zu < %zu bytes", work_bytes, need);
        return BDG_ERR_WORKSPACE;
    }
    GemmArgs g{M, N, K, alpha[0], alpha[1], beta[0], beta[1], A, lda, B, ldb, C, ldc, mode, splitk,
               splitk > 1 ? work : nullptr};
    return gemm<double, true>(opA, opB, g, (hipStream_t)stream);
}

int bdg_stage_bt1(int64_t n, int64_t m, const double *A, int64_t lda, int band, const double *T1,
                  double *Z, int64_t ldz, void *work, size_t work_bytes, bdg_stream_t stream) {
    if (work_bytes < bdg::bt1_workspace(n, m, band)) return BDG_ERR_WORKSPACE;
    return bdg::bt1(n, m, A, lda, band, T1, Z, ldz, work, (hipStream_t)stream);
}

}  // extern "C"

extern "C" {

static int lattice_ok(const bdg_lattice *lat, const char *fn) {
    if (!lat || lat->ndim < 1 || lat->ndim > 3) {
        set_error("%s: lattice must have ndim in 1..3", fn);
        return -1;
    }
    for (int d = 0; d < lat->ndim; ++d) {
        const int N = lat->dims[d];
        if (N < 2 || (N & 1) || N > 64) {
            set_error("%s: dims[%d]=%d must be even and in [2, 64]", fn, d, N);
            return -1;
        }
    }
    return 0;
}

int bdg_scf_workspace(const bdg_lattice *lat, size_t *bytes) {
    BDG_TRY(lattice_ok(lat, "bdg_scf_workspace"));
    if (!bytes) return -2;
    *bytes = bdg::scf_workspace(lat);
    return 0;
}

int bdg_scf_step(const bdg_lattice *lat, const double *Vext, const double *theta, double mu,
                 const bdg_scf_params *params, double *U, double *absDelta, double *density,
                 double *nu_abs, double *change, int64_t *m, void *work, size_t work_bytes,
                 bdg_stream_t stream) {
    BDG_TRY(lattice_ok(lat, "bdg_scf_step"));
    if (!Vext) return -2;
    if (!theta) return -3;
    if (!params || !(params->Ec > 0.0) || !(params->alpha > 0.0 && params->alpha <= 1.0) ||
        !(params->T >= 0.0) || (params->regularize != 0 && params->regularize != 1)) {
        set_error("bdg_scf_step: params must have Ec > 0, 0 < alpha <= 1, T >= 0 and regularize 0 or 1");
        return -5;
    }
    if (params->regularize && (lat->ndim != 3 || !(params->g > 0.0))) {
        set_error("bdg_scf_step: the cut-off regularisation needs a 3-D lattice and g > 0");
        return -5;
    }
    if (!U) return -6;
    if (!absDelta) return -7;
    if (!change) return -10;
    if (!m) return -11;
    if (!work || work_bytes < bdg::scf_workspace(lat)) {
        set_error("bdg_scf_step: workspace too small");
        return BDG_ERR_WORKSPACE;
    }
    return bdg::scf_step(lat, Vext, theta, mu, params, U, absDelta, density, nu_abs, change, m, work,
                         (hipStream_t)stream);
}

int bdg_td_workspace(const bdg_lattice *lat, int64_t m, size_t *bytes) {
    BDG_TRY(lattice_ok(lat, "bdg_td_workspace"));
    if (m < 1) return -2;
    if (!bytes) return -3;
    *bytes = bdg::td_workspace(lat, m);
    return 0;
}

int bdg_td_evolve(const bdg_lattice *lat, const double *Vext, double mu, const bdg_td_params *params,
                  int64_t m, double *Phi, int64_t ldphi, double dt, int64_t nsteps, const double *U0,
                  const double *Delta0, void *work, size_t work_bytes, bdg_stream_t stream) {
    BDG_TRY(lattice_ok(lat, "bdg_td_evolve"));
    int64_t ns = 1;
    for (int d = 0; d < lat->ndim; ++d) ns *= lat->dims[d];
    if (ns > bdg::td_max_sites()) {
        set_error("bdg_td_evolve: %lld sites, at most %lld (a state's u and v are staged in LDS)",
                  (long long)ns, (long long)bdg::td_max_sites());
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    if (!params || (params->self_consistent != 0 && params->self_consistent != 1) ||
        (params->resume != 0 && params->resume != 1)) {
        set_error("bdg_td_evolve: params must be given, self_consistent and resume 0 or 1");
        return -4;
    }
    if (params->self_consistent && !Vext) return -2;
    if (m < 1) return -5;
    if (!Phi) return -6;
    if (ldphi < 2 * ns) return -7;
    if (!(dt > 0.0) || !isfinite(dt)) return -8;
    if (nsteps < 0) return -9;
    if (!params->self_consistent && !U0) return -10;
    if (!params->self_consistent && !Delta0) return -11;
    if (!work || work_bytes < bdg::td_workspace(lat, m)) {
        set_error("bdg_td_evolve: workspace too small");
        return BDG_ERR_WORKSPACE;
    }
    return bdg::td_evolve(lat, Vext, mu, params, m, Phi, ldphi, dt, nsteps, U0, Delta0, work,
                          (hipStream_t)stream);
}

int bdg_regrid(const bdg_lattice *src, const double *f, const bdg_lattice *dst, double *g, double scale,
               bdg_stream_t stream) {
    BDG_TRY(lattice_ok(src, "bdg_regrid"));
    if (!f) return -2;
    if (lattice_ok(dst, "bdg_regrid") || dst->ndim != src->ndim) {
        set_error("bdg_regrid: the target lattice must be valid and have the source's ndim");
        return -3;
    }
    if (!g) return -4;
    return bdg::regrid(src, f, dst, g, scale, (hipStream_t)stream);
}

}  // extern "C"

extern "C" {

static int net_shape_ok(const bdg_net_shape *sh) {
    if (!sh || sh->channels < 1 || sh->channels > 64 || sh->ny < 3 || sh->nx < 3 || sh->batch < 1) {
        set_error("net: shape must have 1 <= channels <= 64, ny, nx >= 3, batch >= 1");
        return -1;
    }
    return 0;
}

int64_t bdg_net_nparams(const bdg_net_shape *shape) {
    if (net_shape_ok(shape)) return -1;
    return bdg::net_layout(shape).nparams;
}

int bdg_net_workspace(const bdg_net_shape *shape, size_t *bytes) {
    BDG_TRY(net_shape_ok(shape));
    if (!bytes) return -2;
    *bytes = bdg::net_layout(shape).total;
    return 0;
}

int bdg_net_forward(const bdg_net_shape *shape, const float *params, const double *Vext,
                    const double *theta, double mu, float *y, void *work, size_t work_bytes,
                    bdg_stream_t stream) {
    BDG_TRY(net_shape_ok(shape));
    if (!params) return -2;
    if (!Vext) return -3;
    if (!theta) return -4;
    if (!y) return -6;
    if (!work || work_bytes < bdg::net_layout(shape).total) return BDG_ERR_WORKSPACE;
    return bdg::net_forward(shape, params, Vext, theta, mu, y, work, (hipStream_t)stream);
}

int bdg_net_forward_noalloc(const bdg_net_shape *shape, const float *params, const double *Vext,
                            const double *theta, double mu, float *y, bdg_stream_t stream) {
    BDG_TRY(net_shape_ok(shape));
    if (!params) return -2;
    if (!Vext) return -3;
    if (!theta) return -4;
    if (!y) return -6;
    return bdg::net_forward_noalloc(shape, params, Vext, theta, mu, y, (hipStream_t)stream);
}

int bdg_net_backward(const bdg_net_shape *shape, const float *params, const double *Vext,
                     const double *theta, double mu, const float *target, float *grads,
                     float *loss, void *work, size_t work_bytes, bdg_stream_t stream) {
    BDG_TRY(net_shape_ok(shape));
    if (!params) return -2;
    if (!Vext) return -3;
    if (!theta) return -4;
    if (!target) return -6;
    if (!grads) return -7;
    if (!loss) return -8;
    if (!work || work_bytes < bdg::net_layout(shape).total) return BDG_ERR_WORKSPACE;
    return bdg::net_backward(shape, params, Vext, theta, mu, target, grads, loss, work,
                             (hipStream_t)stream);
}

int bdg_net_start_fields(const bdg_net_shape *shape, const float *y, int32_t sample, const double *Vext,
                         double *U, double *absDelta, bdg_stream_t stream) {
    BDG_TRY(net_shape_ok(shape));
    if (!y) return -2;
    if (sample < 0 || sample >= shape->batch) return -3;
    if (!Vext) return -4;
    if (!U) return -5;
    if (!absDelta) return -6;
    return bdg::net_start_fields(shape, y, sample, Vext, U, absDelta, (hipStream_t)stream);
}

int bdg_net_adam_step(int64_t nparams, float *params, const float *grads, float *m, float *v,
                      int32_t t, float lr, bdg_stream_t stream) {
    if (nparams < 1) return -1;
    if (!params || !grads || !m || !v) return -2;
    if (t < 1) return -6;
    return bdg::net_adam(nparams, params, grads, m, v, t, lr, (hipStream_t)stream);
}

}  // extern "C"
