// Internal interfaces between the C-ABI layer and the solver stages.
#pragma once
#include "common.h"

namespace bdg {

int assemble(const bdg_lattice *lat, const double *U, const double *Delta, double mu, double *H,
             int64_t ldh, hipStream_t s);

int check_pairs(int64_t n, const double *H, int64_t ldh, int64_t m, const double *W,
                const double *Z, int64_t ldz, double *max_resid, double *gram_defect, void *work,
                hipStream_t s);

}  // namespace bdg

namespace bdg {

int eigh_workspace(int64_t n, const bdg_opts *opts, size_t *bytes);
int eigh(int64_t n, double *A, int64_t lda, double emin, double emax, double *W, double *Z,
         int64_t ldz, int64_t zcols, int64_t *m, const bdg_opts *opts, void *work,
         size_t work_bytes, bdg_err_report *report, hipStream_t s);
size_t ozaki_workspace(bool cx, int64_t M, int64_t N, int64_t K, int S);
int ozaki_gemm(bool cx, int S, char opA, char opB, int64_t M, int64_t N, int64_t K, const double *alpha,
               const double *A, int64_t lda, const double *B, int64_t ldb, const double *beta, double *C,
               int64_t ldc, void *work, hipStream_t s);
size_t eigh1_workspace(int64_t n, bool cx, int64_t zcols);
int eigh1(int64_t n, bool cx, double *A, int64_t lda, double emin, double emax, double *W, double *Z,
          int64_t ldz, int64_t zcols, int64_t *m_out, void *work, bdg_err_report *report, hipStream_t s);
int refine_pairs(int64_t n, const double *H, int64_t ldh, const double *lam, double *X, int64_t ldx,
                 int64_t i0, int64_t m, double *W, const bdg_opts *opts, void *work,
                 bdg_err_report *report, hipStream_t s);

}  // namespace bdg

namespace bdg {

size_t scf_workspace(const bdg_lattice *lat);
int scf_step(const bdg_lattice *lat, const double *Vext, const double *theta, double mu,
             const bdg_scf_params *p, double *U, double *absDelta, double *density, double *nu_abs,
             double *change, int64_t *m_out, void *work, hipStream_t s);
int regrid(const bdg_lattice *src, const double *f, const bdg_lattice *dst, double *g, double scale,
           hipStream_t s);
size_t td_workspace(const bdg_lattice *lat, int64_t m);
int64_t td_max_sites();
int td_evolve(const bdg_lattice *lat, const double *Vext, double mu, const bdg_td_params *p, int64_t m,
              double *Phi, int64_t ldphi, double dt, int64_t nsteps, const double *U0, const double *D0,
              void *work, hipStream_t s);

}  // namespace bdg
