// MFMA tile GEMM for gfx950: C = alpha op(A) op(B) + beta C.
//
// One 256-thread workgroup computes a 64x64 tile of C; its four waves each own
// a 32x32 quarter made of 2x2 MFMA 16x16 blocks.  Operand tiles are staged in
// LDS (double-buffered through registers); complex products use four real
// MFMAs per block (re*re, -im*im, re*im, im*re).  Modes:
//   GEMM_FULL   every tile of C
//   GEMM_LOWER  only tiles (I, J) with I >= J (Hermitian rank-2k updates)
//   GEMM_HEMM_L A is Hermitian and only its lower triangle is valid; tiles of A
//               above the diagonal are read conjugate-transposed from below it
#pragma once
#include "common.h"

namespace bdg {

enum { GEMM_FULL = 0, GEMM_LOWER = 1, GEMM_HEMM_L = 2 };

struct GemmArgs {
    int64_t M, N, K;
    double alpha_re, alpha_im, beta_re, beta_im;
    const void *A;
    int64_t lda;
    const void *B;
    int64_t ldb;
    void *C;
    int64_t ldc;
    int mode;        // GEMM_*
    int splitk;      // >1: partial sums to `part`, then reduced into C
    void *part;      // device scratch: splitk * M * N elements (used when splitk > 1)
    const int *acol = nullptr;  // opA='N' only: column k of A is A[:, acol[k]]
    const int *ccol = nullptr;  // column j of C is C[:, ccol[j]]
    const int *brow = nullptr;  // opB='N' only: row k of B is B[brow[k], :]
};

// T = double/float, cplx = complex (interleaved) or real elements.
template <typename T, bool CPLX>
int gemm(char opA, char opB, const GemmArgs &g, hipStream_t s);

// Scratch elements needed by a split-K launch.
inline size_t gemm_split_elems(int64_t M, int64_t N, int splitk) {
    return splitk > 1 ? (size_t)splitk * (size_t)M * (size_t)N : 0;
}

}  // namespace bdg
