"""Oracle: FP64 matrix products emulated with exact integer products of
8-bit slices (Ozaki, Ogita, Oishi & Rump, "Error-free transformations of
matrix multiplication by using fast routines of matrix multiplication and its
applications", Numer. Algorithms 59 (2012); the integer form of Ootomo, Ozaki
& Yokota, "DGEMM on integer matrix multiplication unit", IJHPCA 2024).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The plain definition of what the emulated product reaches is the matrix
product itself; this module writes the scheme's steps out so that the GPU
kernel can be compared with the same truncation, and the pins compare both
with exact rational products.

Steps, for C = A B with A (M x K), B (K x N) real FP64:
  1. Row scales of A: e_r with max_k |A_rk| < 2^(e_r - 1); column scales e_c of
     B likewise.  Then x = A_rk / 2^e_r lies in (-1/2, 1/2).
  2. X = round(x 2^(7 s)), an integer with |X| <= 2^(7 s - 1), written in
     balanced base 128: X = sum_{i=1..s} d_i 128^(s-i), the digits d_2 .. d_s
     in [-64, 63] and the leading digit d_1 what remains (|d_1| <= 65), so
     that x = sum_i d_i 128^(-i) up to the rounding of step 2.
  3. C_rc ~ 2^(e_r + e_c) sum_{i + j <= s + 1} 128^-(i+j) (D^A_i D^B_j)_rc,
     each D^A_i D^B_j an exact integer product of 8-bit matrices (|entries|
     <= 65, so a K-term sum stays below 2^31 for K < 2^18).  The dropped pairs
     (i + j > s + 1) and the rounding of step 2 bound the error:
       |C_rc - (A B)_rc| <= 2^(e_r + e_c) K (128^-s + (s + 1) 65^2 128^-(s+2))
     (each rounding error at most 128^-s / 2 against a factor below 1/2 in
     modulus, each dropped digit product at most 65^2 128^-t, at most s of
     them for every t >= s + 2, and sum_{t >= s+2} s 128^-t < (s+1) 128^-(s+2)).
Complex products use the real embedding [[Ar, -Ai], [Ai, Ar]] [[Br], [Bi]] =
[[Cr], [Ci]]: one real product of order 2M x 2K x N, whose row scales are
shared by the real and imaginary parts of a row of A and whose column scales
by both parts of a column of B.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def scales(A: np.ndarray, axis: int) -> np.ndarray:
    """e with max |A| along `axis` < 2^(e - 1) (0 for an all-zero line)."""
    mx = np.max(np.abs(A), axis=axis)
    e = np.zeros(mx.shape, dtype=np.int64)
    nz = mx > 0
    e[nz] = np.frexp(mx[nz])[1] + 1          # mx < 2^frexp_exp
    return e


def digits(x: np.ndarray, s: int) -> np.ndarray:
    """Balanced base-128 digits d_1 .. d_s (most significant first) of
    round(x 2^(7 s)) for |x| < 1/2 (the leading one within +-65); returns an
    int64 array [s, ...]."""
    X = np.rint(np.ldexp(x, 7 * s)).astype(np.int64)
    out = np.zeros((s,) + x.shape, dtype=np.int64)
    for i in range(s - 1, 0, -1):
        d = ((X + 64) % 128) - 64
        out[i] = d
        X = (X - d) // 128
    out[0] = X
    assert np.all(np.abs(X) <= 65)
    return out


def split_rows(A: np.ndarray, s: int):
    e = scales(A, 1)
    return digits(np.ldexp(A, -e[:, None]), s), e


def split_cols(B: np.ndarray, s: int):
    e = scales(B, 0)
    return digits(np.ldexp(B, -e[None, :]), s), e


def gemm_real(A: np.ndarray, B: np.ndarray, s: int) -> np.ndarray:
    """The emulated product of step 3 (integer products exact in int64, the
    weighted sum in FP64 by increasing significance)."""
    DA, ea = split_rows(A, s)
    DB, eb = split_cols(B, s)
    acc = np.zeros((A.shape[0], B.shape[1]))
    for t in range(s + 1, 1, -1):
        P = np.zeros_like(acc, dtype=np.int64)
        for i in range(1, t):
            j = t - i
            if 1 <= i <= s and 1 <= j <= s:
                P += DA[i - 1] @ DB[j - 1]
        acc += np.ldexp(P.astype(np.float64), -7 * t)
    return np.ldexp(acc, ea[:, None] + eb[None, :])


def gemm_complex(A: np.ndarray, B: np.ndarray, s: int) -> np.ndarray:
    M = A.shape[0]
    Ae = np.block([[A.real, -A.imag], [A.imag, A.real]])
    Be = np.vstack([B.real, B.imag])
    Ce = gemm_real(Ae, Be, s)
    return Ce[:M] + 1j * Ce[M:]


def error_bound(A: np.ndarray, B: np.ndarray, s: int) -> np.ndarray:
    """Entrywise bound of step 3 on |C - A B| (real A, B)."""
    ea, eb = scales(A, 1), scales(B, 0)
    K = A.shape[1]
    per = K * (128.0 ** -s + (s + 1) * 65.0 ** 2 * 128.0 ** -(s + 2))
    return np.ldexp(np.full((A.shape[0], B.shape[1]), per), ea[:, None] + eb[None, :])


def exact_product(A: np.ndarray, B: np.ndarray):
    """A B in exact rational arithmetic (small matrices only)."""
    M, K = A.shape
    N = B.shape[1]
    Af = [[Fraction(float(A[i, k])) for k in range(K)] for i in range(M)]
    Bf = [[Fraction(float(B[k, j])) for j in range(N)] for k in range(K)]
    return [[sum(Af[i][k] * Bf[k][j] for k in range(K)) for j in range(N)] for i in range(M)]
