// Refinement and precision-conversion helpers of the mixed-precision solver.
#pragma once
#include "common.h"

namespace bdg {

int cast_c64_to_c128(int64_t rows, int64_t cols, const float *src, int64_t lds, double *dst,
                     int64_t ldd, hipStream_t s);
int cast_c128_to_c64(int64_t rows, int64_t cols, const double *src, int64_t lds, float *dst,
                     int64_t ldd, hipStream_t s);
// columns [0, n/2) <- particle-hole partners (-v^*, u^*) of columns [n/2, n) (reversed)
int mirror_half(int64_t n, double *X, int64_t ld, hipStream_t s);
int mirror_half(int64_t n, float *X, int64_t ld, hipStream_t s);
// columns dst0 + k <- particle-hole partner of column src0 - k (k < count)
int mirror_columns(int64_t n, double *X, int64_t ld, int64_t dst0, int64_t src0, int64_t count,
                   hipStream_t s);
size_t refine_workspace(int64_t n, int64_t m);
// Up to `iters` steps; stops early once the step's defect, max over (i, j) off
// the window diagonal of max(|r_ij|, |s_ij + lam_j r_ij| / normH) (only the
// second term on rows outside the window), and the in-cluster coupling
// max |M_kl| / normH are both < tol.  delta0: the
// first step's delta; nclusters: columns in clusters at the last step.
int refine_window(int64_t n, const double *H, int64_t ldh, double *X, int64_t ldx,
                  const double *lam_all, int64_t i0, int64_t m, double normH, int iters, double tol,
                  double *W, void *work, hipStream_t s, double *eig_shift, double *last_corr,
                  int *iters_done, int *close0, int *ccols0);

}  // namespace bdg
