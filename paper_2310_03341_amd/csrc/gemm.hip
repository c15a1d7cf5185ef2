// MFMA tile GEMM kernels (see gemm.h for the layout and modes).
#include "gemm.h"

#include <math.h>
#include <stdlib.h>

namespace bdg {
namespace {

constexpr int NT = 256;

// WB: 16x16 MFMA blocks per wave along M and along N; the workgroup's four
// waves form a 2 x 2 grid, so a tile of C is 32 WB x 32 WB.
template <typename T, bool CPLX, int WB = 2>
struct Cfg {
    static constexpr int EW = CPLX ? 2 : 1;       // scalars per element
    static constexpr int BM = 32 * WB;            // tile rows (and columns)
    static constexpr int BK = (CPLX || WB > 2) ? 16 : 32;  // k-depth of one LDS tile
    static constexpr int LDS_LD = BM + 1;         // elements per k-row in LDS
    static constexpr int TILE_ELEMS = BK * BM;    // elements of one operand tile
    static constexpr int PER_THREAD = TILE_ELEMS / NT;
};

// Load one operand tile (MN x BK elements) from global memory into registers.
//   KFAST = false: element (i, k) at P[(r0 + i) + (k0 + k) * ld]  (contiguous in i)
//   KFAST = true : element (i, k) at P[(k0 + k) + (r0 + i) * ld]  (contiguous in k)
// Out-of-range elements are zero.  HEMM_DIAG: lower-Hermitian select for the
// diagonal tile (i-fast layout only).
template <typename T, bool CPLX, int WB, bool KFAST, bool CONJ>
__device__ inline void load_tile(const T *__restrict__ P, int64_t ld, int64_t r0, int64_t k0,
                                 int64_t MN, int64_t K, typename v2t<T>::type (&v)[Cfg<T, CPLX, WB>::PER_THREAD],
                                 unsigned &okm, unsigned &cjm, bool hemm_diag,
                                 const int *__restrict__ kmap = nullptr) {
    typedef Cfg<T, CPLX, WB> C;
    constexpr int PT = C::PER_THREAD;
    const int t = threadIdx.x;
    // all loads of the tile are issued before any is used: unconditional (from
    // element 0 outside the range) and zeroed by select afterwards.  A guarded
    // load compiles to branch + load + wait, which would serialise them.
    int64_t gi[PT], gk[PT], kk[PT];
    bool ok[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        int i, k;
        if (KFAST) {
            k = t % C::BK;
            i = t / C::BK + (NT / C::BK) * j;
        } else {
            i = t % C::BM;
            k = t / C::BM + (NT / C::BM) * j;
        }
        gi[j] = r0 + i;
        gk[j] = k0 + k;
        ok[j] = (gi[j] < MN) & (gk[j] < K);
        kk[j] = ok[j] ? gk[j] : 0;
    }
    if (kmap) {
#pragma unroll
        for (int j = 0; j < PT; ++j) kk[j] = kmap[kk[j]];
    }
    bool cj[PT];
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        int64_t off;
        cj[j] = CONJ;
        if (KFAST) {
            off = kk[j] + gi[j] * ld;
        } else if (hemm_diag && gk[j] > gi[j]) {
            off = gk[j] + gi[j] * ld;  // upper element of a Hermitian tile: conj of lower
            cj[j] = true;
        } else {
            off = gi[j] + kk[j] * ld;
        }
        off = ok[j] ? off : 0;
        if (CPLX) {
            v[j] = *(const typename v2t<T>::type *)(P + 2 * off);
        } else {
            v[j].x = P[off];
            v[j].y = 0;
        }
    }
    // the values are only selected when they go to LDS (store_tile), so the
    // products of the current tile run while these loads are in flight
    okm = 0;
    cjm = 0;
#pragma unroll
    for (int j = 0; j < PT; ++j) {
        okm |= (unsigned)ok[j] << j;
        cjm |= (unsigned)cj[j] << j;
    }
}

template <typename T, bool CPLX, int WB, bool KFAST>
__device__ inline void store_tile(T *__restrict__ S, const typename v2t<T>::type (&v)[Cfg<T, CPLX, WB>::PER_THREAD],
                                  unsigned okm, unsigned cjm) {
    typedef Cfg<T, CPLX, WB> C;
    const int t = threadIdx.x;
    T reg[C::PER_THREAD][2];
#pragma unroll
    for (int j = 0; j < C::PER_THREAD; ++j) {
        const bool ok = (okm >> j) & 1u, cj = (cjm >> j) & 1u;
        reg[j][0] = ok ? v[j].x : (T)0;
        reg[j][1] = (ok && CPLX) ? (cj ? -v[j].y : v[j].y) : (T)0;
    }
#pragma unroll
    for (int j = 0; j < C::PER_THREAD; ++j) {
        int i, k;
        if (KFAST) {
            k = t % C::BK;
            i = t / C::BK + (NT / C::BK) * j;
        } else {
            i = t % C::BM;
            k = t / C::BM + (NT / C::BM) * j;
        }
        const int idx = k * C::LDS_LD + i;
        if (CPLX) {
            S[2 * idx] = reg[j][0];
            S[2 * idx + 1] = reg[j][1];
        } else {
            S[idx] = reg[j][0];
        }
    }
}

// Direct global -> LDS operand tiles (complex FP64, 64 x 16 elements per
// tile).  One wave instruction moves 64 elements of 16 bytes to 64
// consecutive LDS slots (lane l to slot base + l, the slot base in M0; checked
// on gfx950 by an in-bounds probe), so the tile never passes through vector
// registers.  Layouts, in elements:
//   i-fast operands (column i contiguous in memory: A 'N', B 'C'):
//     (i, k) at k * 64 + i, one instruction per k row;
//   k-fast operands (k contiguous: A 'C', B 'N'): (i, k) at i * 16 + (k ^ (i & 15)),
//     one instruction per four i rows; the XOR places the 16 rows that one
//     MFMA operand read touches at one k in 16 different bank groups.
// Elements outside the matrix are loaded from row or column 0 (any valid
// address): rows beyond M or N only reach outputs that are never stored,
// and K beyond the end is masked when the tile is read.
__device__ inline int dslot(bool kfast, int i, int k) { return kfast ? i * 16 + (k ^ (i & 15)) : k * 64 + i; }

__device__ inline void direct_tile(const double *__restrict__ P, int64_t ld, int64_t r0, int64_t MN, int64_t k0,
                                   int64_t K, bool kfast, double *lds_tile, int wave, int lane) {
    const unsigned lbase = (unsigned)(size_t)(__attribute__((address_space(3))) void *)lds_tile;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int q = wave + 4 * u;  // instruction q of 16
        int i, k;
        if (kfast) {
            i = 4 * q + (lane >> 4);
            k = (lane & 15) ^ (i & 15);
        } else {
            i = lane;
            k = q;
        }
        int64_t gi = r0 + i, gk = k0 + k;
        gi = gi < MN ? gi : 0;
        gk = gk < K ? gk : 0;
        const double *src = P + 2 * (kfast ? gk + gi * ld : gi + gk * ld);
        const unsigned m0v = __builtin_amdgcn_readfirstlane(lbase + 1024u * (unsigned)q);
        asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                     :: "v"(src), "s"(m0v) : "memory", "m0");
    }
}

__device__ inline void wait_vm_direct() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// opA: false = 'N', true = 'C'.  opB likewise.
template <typename T, bool CPLX, bool CA, bool CB, int MODE, int WB, bool DIRECT>
__global__ __launch_bounds__(NT, 2) void gemm_kernel(GemmArgs g, int64_t kchunk) {
    typedef Cfg<T, CPLX, WB> C;
    typedef typename acc4<T>::type A4;
    constexpr int EW = C::EW;
    constexpr int BM = C::BM, BN = C::BM, WT = 16 * WB;  // tile, and each wave's share of it
    static_assert(WB == 2 || (WB == 4 && !CPLX && MODE == GEMM_FULL), "large tiles: real, full mode");
    static_assert(!DIRECT || (sizeof(T) == 8 && CPLX && WB == 2), "direct tiles: complex FP64");
    __shared__ T As[2][C::BK * C::LDS_LD * EW];
    __shared__ T Bs[2][C::BK * C::LDS_LD * EW];

    const T *__restrict__ A = (const T *)g.A;
    const T *__restrict__ B = (const T *)g.B;
    T *__restrict__ Cm = (T *)g.C;

    int64_t tI, tJ;
    if (MODE == GEMM_LOWER) {
        const int64_t L = blockIdx.x;
        int64_t I = (int64_t)((sqrt(8.0 * (double)L + 1.0) - 1.0) * 0.5);
        while (I * (I + 1) / 2 > L) --I;
        while ((I + 1) * (I + 2) / 2 <= L) ++I;
        tI = I;
        tJ = L - I * (I + 1) / 2;
    } else {
        tI = blockIdx.x;
        tJ = blockIdx.y;
    }
    const int64_t m0 = tI * BM, n0 = tJ * BN;
    const int64_t kbeg = (int64_t)blockIdx.z * kchunk;
    const int64_t kend = min(g.K, kbeg + kchunk);

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int wm = wave & 1, wn = wave >> 1;

    // complex: three real products per complex one (Gauss' form),
    // P1 = sum ar br, P2 = sum ai bi, P3 = sum (ar + ai)(br + bi);
    // Re = P1 - P2, Im = P3 - P1 - P2 (formed after the k loop).  Real: P1 only.
    A4 accR[WB][WB], accI[CPLX ? WB : 1][CPLX ? WB : 1], acc3[CPLX ? WB : 1][CPLX ? WB : 1];
#pragma unroll
    for (int a = 0; a < WB; ++a)
#pragma unroll
        for (int b = 0; b < WB; ++b) accR[a][b] = A4{0, 0, 0, 0};
    if (CPLX) {
#pragma unroll
        for (int a = 0; a < (CPLX ? WB : 1); ++a)
#pragma unroll
            for (int b = 0; b < (CPLX ? WB : 1); ++b) {
                accI[a][b] = A4{0, 0, 0, 0};
                acc3[a][b] = A4{0, 0, 0, 0};
            }
    }

    typename v2t<T>::type ra[C::PER_THREAD], rb[C::PER_THREAD];
    unsigned aok = 0, acj = 0, bok = 0, bcj = 0;

    // A operand: 'N' -> i-fast, 'C' -> k-fast.  HEMM_L: per tile choice.
    auto loadA = [&](int64_t k0) {
        if (MODE == GEMM_HEMM_L) {
            // block column of A holding k0 (tiles aligned to BM)
            if (k0 + C::BK <= m0) {
                load_tile<T, CPLX, WB, false, false>(A, g.lda, m0, k0, g.M, kend, ra, aok, acj, false);
            } else if (k0 >= m0 + BM) {
                load_tile<T, CPLX, WB, true, true>(A, g.lda, m0, k0, g.M, kend, ra, aok, acj, false);
            } else {
                load_tile<T, CPLX, WB, false, false>(A, g.lda, m0, k0, g.M, kend, ra, aok, acj, true);
            }
        } else if (CA) {
            load_tile<T, CPLX, WB, true, true>(A, g.lda, m0, k0, g.M, kend, ra, aok, acj, false);
        } else {
            load_tile<T, CPLX, WB, false, false>(A, g.lda, m0, k0, g.M, kend, ra, aok, acj, false, g.acol);
        }
    };
    auto storeA = [&](int buf, int64_t k0) {
        bool kf;
        if (MODE == GEMM_HEMM_L) kf = (k0 >= m0 + BM);
        else kf = CA;
        if (kf) store_tile<T, CPLX, WB, true>(As[buf], ra, aok, acj);
        else store_tile<T, CPLX, WB, false>(As[buf], ra, aok, acj);
    };
    // B operand: 'N' -> k-fast (B stored K x N), 'C' -> i-fast (B stored N x K).
    auto loadB = [&](int64_t k0) {
        if (CB) load_tile<T, CPLX, WB, false, true>(B, g.ldb, n0, k0, g.N, kend, rb, bok, bcj, false);
        else load_tile<T, CPLX, WB, true, false>(B, g.ldb, n0, k0, g.N, kend, rb, bok, bcj, false, g.brow);
    };
    auto storeB = [&](int buf) {
        if (CB) store_tile<T, CPLX, WB, false>(Bs[buf], rb, bok, bcj);
        else store_tile<T, CPLX, WB, true>(Bs[buf], rb, bok, bcj);
    };

    // C entry (row block a, column block b, element q) of this lane: offset and
    // whether it lies inside the matrix (split-K partials excluded)
    auto c_off = [&](int a, int b, int q, bool &ok) -> int64_t {
        const int64_t col = n0 + wn * WT + b * 16 + (lane & 15);
        const int64_t row = m0 + wm * WT + a * 16 + mfma_row((T)0, lane, q);
        ok = (row < g.M) & (col < g.N);
        return ok ? row + (g.ccol ? (int64_t)g.ccol[col] : col) * g.ldc : 0;
    };
    constexpr bool CEARLY = DIRECT && MODE != GEMM_HEMM_L;  // HEMM tiles have no registers to spare
    const bool c_early = CEARLY && g.splitk <= 1 && !((T)g.beta_re == (T)0 && (T)g.beta_im == (T)0);
    typename v2t<T>::type preC[CEARLY ? WB : 1][CEARLY ? WB : 1][4];
    if constexpr (DIRECT) {
        // operand layouts: A 'C' and B 'N' are k-fast.  HEMM_L: A tiles below
        // the diagonal block are i-fast, above it k-fast and conjugated (the
        // stored lower triangle read transposed); the four tiles of the
        // diagonal block go through registers (load_tile picks each element
        // from the stored triangle) and are stored i-fast, conjugation done.
        constexpr bool kfB = !CB;
        auto a_layout = [&](int64_t k0, bool &kf, bool &cj) {
            if (MODE == GEMM_HEMM_L) {
                kf = k0 >= m0 + BM;
                cj = kf;
            } else {
                kf = CA;
                cj = CA;
            }
        };
        auto compute_direct = [&](int buf, int64_t k0, bool tail) {
            bool kfA, cjA;
            a_layout(k0, kfA, cjA);
            const double2 *as = (const double2 *)As[buf];
            const double2 *bs = (const double2 *)Bs[buf];
#pragma unroll
            for (int kk = 0; kk < C::BK; kk += 4) {
                const int kr = kk + (lane >> 4);
                const bool kin = !tail || (k0 + kr < kend);
                T are[WB], aim[WB], bre[WB], bim[WB];
#pragma unroll
                for (int a = 0; a < WB; ++a) {
                    const double2 v = as[dslot(kfA, wm * WT + a * 16 + (lane & 15), kr)];
                    are[a] = kin ? v.x : 0.0;
                    aim[a] = kin ? (cjA ? -v.y : v.y) : 0.0;
                }
#pragma unroll
                for (int b = 0; b < WB; ++b) {
                    const double2 v = bs[dslot(kfB, wn * WT + b * 16 + (lane & 15), kr)];
                    bre[b] = kin ? v.x : 0.0;
                    bim[b] = kin ? (CB ? -v.y : v.y) : 0.0;
                }
                T as2[WB], bs2[WB];
#pragma unroll
                for (int a = 0; a < WB; ++a) as2[a] = are[a] + aim[a];
#pragma unroll
                for (int b = 0; b < WB; ++b) bs2[b] = bre[b] + bim[b];
#pragma unroll
                for (int a = 0; a < WB; ++a)
#pragma unroll
                    for (int b = 0; b < WB; ++b) accR[a][b] = mfma16(are[a], bre[b], accR[a][b]);
#pragma unroll
                for (int a = 0; a < WB; ++a)
#pragma unroll
                    for (int b = 0; b < WB; ++b)
                        accI[CPLX ? a : 0][CPLX ? b : 0] = mfma16(aim[a], bim[b], accI[CPLX ? a : 0][CPLX ? b : 0]);
#pragma unroll
                for (int a = 0; a < WB; ++a)
#pragma unroll
                    for (int b = 0; b < WB; ++b)
                        acc3[CPLX ? a : 0][CPLX ? b : 0] = mfma16(as2[a], bs2[b], acc3[CPLX ? a : 0][CPLX ? b : 0]);
            }
        };
        bool stagedA = false;  // a diagonal-block A tile waits in ra for its LDS store
        auto issue = [&](int buf, int64_t k0) {
            if (MODE == GEMM_HEMM_L && k0 + C::BK > m0 && k0 < m0 + BM) {
                load_tile<T, CPLX, WB, false, false>(A, g.lda, m0, k0, g.M, kend, ra, aok, acj, true);
                stagedA = true;
            } else {
                bool kfA, cjA;
                a_layout(k0, kfA, cjA);
                direct_tile((const double *)A, g.lda, m0, g.M, k0, kend, kfA, (double *)As[buf], wave, lane);
            }
            direct_tile((const double *)B, g.ldb, n0, g.N, k0, kend, kfB, (double *)Bs[buf], wave, lane);
        };
        auto store_staged = [&](int buf) {
            if (MODE != GEMM_HEMM_L || !stagedA) return;
            stagedA = false;
            double2 *dst = (double2 *)As[buf];
            const int t = threadIdx.x;
#pragma unroll
            for (int j = 0; j < C::PER_THREAD; ++j) {
                const int i = t % C::BM, k = t / C::BM + (NT / C::BM) * j;  // load_tile's i-fast assignment
                const bool ok = (aok >> j) & 1u, cj = (acj >> j) & 1u;
                dst[k * 64 + i] = make_double2(ok ? ra[j].x : 0.0, ok ? (cj ? -ra[j].y : ra[j].y) : 0.0);
            }
        };
        if (kbeg < kend) {
            // full K tiles in the loop, a partial last tile after it
            const int64_t kfull = kbeg + (kend - kbeg) / C::BK * C::BK;
            issue(0, kbeg);
            store_staged(0);
            wait_vm_direct();
            __syncthreads();
            // C (beta != 0) is read now, so that its latency passes behind the first K tile
            if (c_early) {
#pragma unroll
                for (int a = 0; a < WB; ++a)
#pragma unroll
                    for (int b = 0; b < WB; ++b)
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            bool ok;
                            const int64_t off = c_off(a, b, q, ok);
                            preC[CEARLY ? a : 0][CEARLY ? b : 0][q] = ld2<T>(Cm + 2 * off);
                        }
            }
            int buf = 0;
            int64_t k0 = kbeg;
            for (; k0 < kfull; k0 += C::BK) {
                const int64_t kn = k0 + C::BK;
                const bool more = kn < kend;
                // the other buffer was last read before the barrier that ended the previous step
                if (more) issue(buf ^ 1, kn);
                compute_direct(buf, k0, false);
                if (more) {
                    store_staged(buf ^ 1);
                    wait_vm_direct();
                }
                __syncthreads();
                buf ^= 1;
            }
            if (k0 < kend) compute_direct(buf, k0, true);
        }
    } else {
        if (kbeg < kend) {
            loadA(kbeg);
            loadB(kbeg);
            storeA(0, kbeg);
            storeB(0);
            __syncthreads();
            int buf = 0;
            for (int64_t k0 = kbeg; k0 < kend; k0 += C::BK) {
                const int64_t kn = k0 + C::BK;
                const bool more = kn < kend;
                if (more) {
                    loadA(kn);
                    loadB(kn);
                }
                const T *as = As[buf];
                const T *bs = Bs[buf];
    #pragma unroll
                for (int kk = 0; kk < C::BK; kk += 4) {
                    const int kr = kk + (lane >> 4);
                    T are[WB], aim[WB], bre[WB], bim[WB];
    #pragma unroll
                    for (int a = 0; a < WB; ++a) {
                        const int idx = kr * C::LDS_LD + wm * WT + a * 16 + (lane & 15);
                        if (CPLX) {
                            are[a] = as[2 * idx];
                            aim[a] = as[2 * idx + 1];
                        } else {
                            are[a] = as[idx];
                            aim[a] = 0;
                        }
                    }
    #pragma unroll
                    for (int b = 0; b < WB; ++b) {
                        const int idx = kr * C::LDS_LD + wn * WT + b * 16 + (lane & 15);
                        if (CPLX) {
                            bre[b] = bs[2 * idx];
                            bim[b] = bs[2 * idx + 1];
                        } else {
                            bre[b] = bs[idx];
                            bim[b] = 0;
                        }
                    }
    #pragma unroll
                    for (int a = 0; a < WB; ++a)
    #pragma unroll
                        for (int b = 0; b < WB; ++b) accR[a][b] = mfma16(are[a], bre[b], accR[a][b]);
                    if (CPLX) {
                        T as2[WB], bs2[WB];
    #pragma unroll
                        for (int a = 0; a < WB; ++a) as2[a] = are[a] + aim[a];
    #pragma unroll
                        for (int b = 0; b < WB; ++b) bs2[b] = bre[b] + bim[b];
    #pragma unroll
                        for (int a = 0; a < (CPLX ? WB : 1); ++a)
    #pragma unroll
                            for (int b = 0; b < (CPLX ? WB : 1); ++b) accI[a][b] = mfma16(aim[a], bim[b], accI[a][b]);
    #pragma unroll
                        for (int a = 0; a < (CPLX ? WB : 1); ++a)
    #pragma unroll
                            for (int b = 0; b < (CPLX ? WB : 1); ++b) acc3[a][b] = mfma16(as2[a], bs2[b], acc3[a][b]);
                    }
                }
                if (more) {
                    storeA(buf ^ 1, kn);
                    storeB(buf ^ 1);
                }
                __syncthreads();
                buf ^= 1;
            }
        }
    }

    if (CPLX) {
#pragma unroll
        for (int a = 0; a < (CPLX ? WB : 1); ++a)
#pragma unroll
            for (int b = 0; b < (CPLX ? WB : 1); ++b) {
                const A4 p1 = accR[a][b], p2 = accI[a][b];
                accR[a][b] = p1 - p2;
                accI[a][b] = acc3[a][b] - p1 - p2;
            }
    }
    // epilogue, one row of blocks at a time: its 4 WB entries of C are read
    // (when beta != 0) in one batch before any of them is written
    const bool to_part = g.splitk > 1;
    T *__restrict__ P = (T *)g.part;
    const T ar = (T)g.alpha_re, ai = (T)g.alpha_im, br = (T)g.beta_re, bi = (T)g.beta_im;
    const bool beta0 = (br == (T)0 && bi == (T)0);
#pragma unroll
    for (int a = 0; a < WB; ++a) {
        int64_t coff[WB][4];
        bool cok[WB][4];
#pragma unroll
        for (int b = 0; b < WB; ++b) {
            const int64_t col = n0 + wn * WT + b * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int64_t row = m0 + wm * WT + a * 16 + mfma_row((T)0, lane, q);
                const bool ok = (row < g.M) & (col < g.N);
                cok[b][q] = ok;
                if (to_part) coff[b][q] = (int64_t)blockIdx.z * g.M * g.N + row + col * g.M;
                else coff[b][q] = ok ? row + (g.ccol ? (int64_t)g.ccol[col] : col) * g.ldc : 0;
            }
        }
        T oldr[WB][4], oldi[WB][4];
        if (CEARLY && c_early) {
#pragma unroll
            for (int b = 0; b < WB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    oldr[b][q] = preC[CEARLY ? a : 0][CEARLY ? b : 0][q].x;
                    oldi[b][q] = preC[CEARLY ? a : 0][CEARLY ? b : 0][q].y;
                }
        } else if (!to_part && !beta0) {
#pragma unroll
            for (int b = 0; b < WB; ++b)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (CPLX) {
                        const typename v2t<T>::type v = ld2<T>(Cm + 2 * coff[b][q]);
                        oldr[b][q] = v.x;
                        oldi[b][q] = v.y;
                    } else {
                        oldr[b][q] = Cm[coff[b][q]];
                        oldi[b][q] = 0;
                    }
                }
        }
#pragma unroll
        for (int b = 0; b < WB; ++b) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (!cok[b][q]) continue;
                const T vr = accR[a][b][q], vi = CPLX ? accI[CPLX ? a : 0][CPLX ? b : 0][q] : (T)0;
                const int64_t off = coff[b][q];
                if (to_part) {
                    if (CPLX) {
                        P[2 * off] = vr;
                        P[2 * off + 1] = vi;
                    } else {
                        P[off] = vr;
                    }
                    continue;
                }
                if (CPLX) {
                    T cr = ar * vr - ai * vi, ci = ar * vi + ai * vr;
                    if (!beta0) {
                        const T orr = oldr[b][q], oi = oldi[b][q];
                        cr += br * orr - bi * oi;
                        ci += br * oi + bi * orr;
                    }
                    st2<T>(Cm + 2 * off, mk2<T>(cr, ci));
                } else {
                    T cr = ar * vr;
                    if (!beta0) cr += br * oldr[b][q];
                    Cm[off] = cr;
                }
            }
        }
    }
}

template <typename T, bool CPLX>
__global__ void splitk_reduce(GemmArgs g) {
    const int64_t total = g.M * g.N;
    const T *__restrict__ P = (const T *)g.part;
    T *__restrict__ Cm = (T *)g.C;
    const T ar = (T)g.alpha_re, ai = (T)g.alpha_im, br = (T)g.beta_re, bi = (T)g.beta_im;
    const bool beta0 = (br == (T)0 && bi == (T)0);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e % g.M, col = e / g.M;
        T vr = 0, vi = 0;
        for (int z = 0; z < g.splitk; ++z) {
            const int64_t off = (int64_t)z * total + e;
            if (CPLX) {
                vr += P[2 * off];
                vi += P[2 * off + 1];
            } else {
                vr += P[off];
            }
        }
        const int64_t off = row + (g.ccol ? (int64_t)g.ccol[col] : col) * g.ldc;
        if (CPLX) {
            T cr = ar * vr - ai * vi, ci = ar * vi + ai * vr;
            if (!beta0) {
                const T orr = Cm[2 * off], oi = Cm[2 * off + 1];
                cr += br * orr - bi * oi;
                ci += br * oi + bi * orr;
            }
            Cm[2 * off] = cr;
            Cm[2 * off + 1] = ci;
        } else {
            T cr = ar * vr;
            if (!beta0) cr += br * Cm[off];
            Cm[off] = cr;
        }
    }
}

template <typename T, bool CPLX, bool CA, bool CB, int MODE, int WB = 2>
int launch(const GemmArgs &g, hipStream_t s) {
    typedef Cfg<T, CPLX, WB> C;
    const int64_t tm = (g.M + C::BM - 1) / C::BM, tn = (g.N + C::BM - 1) / C::BM;
    int splitk = g.splitk > 1 ? g.splitk : 1;
    int64_t kchunk = g.K;
    if (splitk > 1) {
        kchunk = (g.K + splitk - 1) / splitk;
        kchunk = (kchunk + C::BK - 1) / C::BK * C::BK;
        splitk = (int)((g.K + kchunk - 1) / kchunk);
    }
    if (kchunk <= 0) kchunk = C::BK;
    if (MODE == GEMM_LOWER && splitk > 1) {
        // the reduction writes every entry of C, the lower-tile product only
        // the tiles on and below the diagonal
        set_error("gemm: the lower-tile mode does not split K");
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    GemmArgs h = g;
    h.splitk = splitk;
    dim3 grid;
    if (MODE == GEMM_LOWER) {
        grid = dim3((unsigned)(tm * (tm + 1) / 2), 1, splitk);
    } else {
        grid = dim3((unsigned)tm, (unsigned)tn, splitk);
    }
    if (tm <= 0 || tn <= 0) return 0;
    // complex FP64 tiles without index maps load straight into LDS
    constexpr bool DIRECT_OK = sizeof(T) == 8 && CPLX && WB == 2;
    static const bool direct_env = [] {
        const char *v = getenv("BDG_GEMM_DIRECT");
        return !(v && v[0] == '0');
    }();
    if (DIRECT_OK && direct_env && !g.acol && !g.brow)
        hipLaunchKernelGGL((gemm_kernel<T, CPLX, CA, CB, MODE, WB, DIRECT_OK>), grid, dim3(NT), 0, s, h, kchunk);
    else
        hipLaunchKernelGGL((gemm_kernel<T, CPLX, CA, CB, MODE, WB, false>), grid, dim3(NT), 0, s, h, kchunk);
    BDG_CHECK_LAUNCH();
    if (splitk > 1) {
        const int64_t total = g.M * g.N;
        int64_t blocks = (total + 255) / 256;
        if (blocks > 4096) blocks = 4096;
        hipLaunchKernelGGL((splitk_reduce<T, CPLX>), dim3((unsigned)blocks), dim3(256), 0, s, h);
        BDG_CHECK_LAUNCH();
    }
    return 0;
}

}  // namespace

template <typename T, bool CPLX>
int gemm(char opA, char opB, const GemmArgs &g, hipStream_t s) {
    if (g.M <= 0 || g.N <= 0) return 0;
    const bool ca = (opA == 'C' || opA == 'c' || opA == 'T' || opA == 't');
    const bool cb = (opB == 'C' || opB == 'c' || opB == 'T' || opB == 't');
    if (g.mode == GEMM_HEMM_L) {
        if (cb) return launch<T, CPLX, false, true, GEMM_HEMM_L>(g, s);
        return launch<T, CPLX, false, false, GEMM_HEMM_L>(g, s);
    }
    if (g.mode == GEMM_LOWER) {
        if (!ca && cb) return launch<T, CPLX, false, true, GEMM_LOWER>(g, s);
        if (!ca && !cb) return launch<T, CPLX, false, false, GEMM_LOWER>(g, s);
        set_error("gemm: lower mode supports opA='N' only");
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    // real products with room for them: 128 x 128 tiles (twice the reuse of
    // every operand element loaded)
    const bool big = !CPLX && g.M >= 256 && g.N >= 256;
    if (ca) {
        if (cb) return big ? launch<T, CPLX, true, true, GEMM_FULL, CPLX ? 2 : 4>(g, s)
                           : launch<T, CPLX, true, true, GEMM_FULL>(g, s);
        return big ? launch<T, CPLX, true, false, GEMM_FULL, CPLX ? 2 : 4>(g, s)
                   : launch<T, CPLX, true, false, GEMM_FULL>(g, s);
    }
    if (cb) return big ? launch<T, CPLX, false, true, GEMM_FULL, CPLX ? 2 : 4>(g, s)
                       : launch<T, CPLX, false, true, GEMM_FULL>(g, s);
    return big ? launch<T, CPLX, false, false, GEMM_FULL, CPLX ? 2 : 4>(g, s)
               : launch<T, CPLX, false, false, GEMM_FULL>(g, s);
}

template int gemm<double, true>(char, char, const GemmArgs &, hipStream_t);
template int gemm<float, true>(char, char, const GemmArgs &, hipStream_t);
template int gemm<double, false>(char, char, const GemmArgs &, hipStream_t);
template int gemm<float, false>(char, char, const GemmArgs &, hipStream_t);

}  // namespace bdg
