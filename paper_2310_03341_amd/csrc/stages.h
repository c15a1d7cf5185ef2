// Internal interfaces of the solver stages.
#pragma once
#include "common.h"

namespace bdg {

// Stage 1: A (lower triangle) -> band AB (lower band storage, ldab >= 2b+2),
// V1 explicit in A's panels, T1 = [panels][b x b].
size_t he2hb_workspace(int64_t n, int b);
int he2hb(int64_t n, double *A, int64_t lda, int b, double *AB, int64_t ldab, double *T1,
          void *work, hipStream_t s);
int he2hb(int64_t n, float *A, int64_t lda, int b, float *AB, int64_t ldab, float *T1,
          void *work, hipStream_t s);
int he2hb_panels(int64_t n, int b);

// Back-transformation 1: Z <- Q1 Z.
size_t bt1_workspace(int64_t n, int64_t m, int b);
int bt1(int64_t n, int64_t m, const double *A, int64_t lda, int b, const double *T1, double *Z,
        int64_t ldz, void *work, hipStream_t s);
int bt1(int64_t n, int64_t m, const float *A, int64_t lda, int b, const float *T1, float *Z,
        int64_t ldz, void *work, hipStream_t s);

}  // namespace bdg

namespace bdg {

// Stage 2: band -> real tridiagonal (d real, e complex before phase scaling).
int64_t hb2st_nrefl(int64_t n, int b);
void hb2st_offsets(int64_t n, int b, int64_t *voff_host);
// Reflector (s, t) lands at V2 + b (voff[s] + t), voff as hb2st_offsets gives.
int hb2st(int64_t n, int b, double *AB, int64_t ldab, double *V2, double *tau2, double *d,
          double *e_cplx, hipStream_t s);
int hb2st(int64_t n, int b, float *AB, int64_t ldab, float *V2, float *tau2, double *d,
          double *e_cplx, hipStream_t s);

// Tridiagonal divide and conquer (FP64): eigenvalues ascending, Q (ld n).
size_t stedc_workspace(int64_t n);
int stedc(int64_t n, const double *d, const double *e, double *lam_out, double *Q_out, int64_t ldq,
          void *work, hipStream_t s, int leaf);

// The library's side stream on the current device (nullptr if it cannot be created).
hipStream_t side_stream();

// Phase scaling of the complex sub-diagonal and back-transformation 2.
// phases = phase_abs (|e|, what the divide and conquer needs) + phase_scan
// (the phase vector, needed only by the scaling after it).
int phases(int64_t n, const double *e_cplx, double *ph, double *e_abs, hipStream_t s);
int phase_abs(int64_t n, const double *e_cplx, double *e_abs, hipStream_t s);
int phase_scan(int64_t n, const double *e_cplx, double *ph, hipStream_t s);
int phase_scale(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, double *Z,
                int64_t ldz, hipStream_t s);
int phase_scale(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, float *Z,
                int64_t ldz, hipStream_t s);
int64_t bt2_nblocks(int64_t n, int b);
// block T factors (into work), then the application to Z (same work)
int bt2_prepare(int64_t n, int b, const double *V2, const double *tau2, const int64_t *voff,
                void *work, hipStream_t s);
int bt2_prepare(int64_t n, int b, const float *V2, const float *tau2, const int64_t *voff,
                void *work, hipStream_t s);
int bt2_apply_blocks(int64_t n, int b, int64_t m, const double *V2, const int64_t *voff, double *Z,
                     int64_t ldz, void *work, hipStream_t s);
int bt2_apply_blocks(int64_t n, int b, int64_t m, const float *V2, const int64_t *voff, float *Z,
                     int64_t ldz, void *work, hipStream_t s);
size_t bt2_workspace(int64_t n, int b);
// Row-major route for the back-transformation 2 (band widths that are a
// multiple of 16): Zrm [n x m], row stride ldr >= m, built from Y with the
// phase scaling, transformed in place, then copied to column-major Z.
bool bt2_rowmajor_ok(int b);
int phase_scale_rm(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, double *Zrm,
                   int64_t ldr, hipStream_t s);
int phase_scale_rm(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, float *Zrm,
                   int64_t ldr, hipStream_t s);
int bt2_apply_blocks_rm(int64_t n, int b, int64_t m, const double *V2, const int64_t *voff, double *Zrm,
                        int64_t ldr, void *work, hipStream_t s);
int bt2_apply_blocks_rm(int64_t n, int b, int64_t m, const float *V2, const int64_t *voff, float *Zrm,
                        int64_t ldr, void *work, hipStream_t s);
int rm_to_cm(int64_t n, int64_t m, const double *Zrm, int64_t ldr, double *Z, int64_t ldz, hipStream_t s);
int rm_to_cm(int64_t n, int64_t m, const float *Zrm, int64_t ldr, float *Z, int64_t ldz, hipStream_t s);
int bt2(int64_t n, int b, int64_t m, const double *V2, const double *tau2, const int64_t *voff,
        double *Z, int64_t ldz, void *work, hipStream_t s);
int bt2(int64_t n, int b, int64_t m, const float *V2, const float *tau2, const int64_t *voff,
        float *Z, int64_t ldz, void *work, hipStream_t s);

}  // namespace bdg
