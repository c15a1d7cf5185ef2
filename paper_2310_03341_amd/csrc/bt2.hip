// Back-transformation 2: eigenvectors of the real tridiagonal -> eigenvectors
// of the band matrix ("the subsequent back transformation of the eigenvectors
// also requires two stages", paper sec. "Performance of the Matrix
// Diagonalization Algorithm").
//
// Z <- Q2 D Y: D = diag(ph) undoes the phase scaling that made the
// tridiagonal real, Q2 = H_{0,0} H_{0,1} ... (generation order of stage 2).
//
// Reflectors of the same task index t from nbk consecutive sweeps S form one
// block G(S, t) = H_{s0,t} ... H_{s0+nbk-1,t} = I - V T V^H (V a
// parallelogram, (b + nbk - 1) x nbk).  Within the sweeps of S, reflectors of
// different t commute in the order G(S, T-1) ... G(S, 0) (rows of H_{s,t} end
// before those of H_{s',t'} start whenever s' > s and t' > t, and
// H_{s',t'} precedes H_{s,t} in generation order whenever s' < s, t' < t, with
// disjoint rows); so  Z <- Q2 Z  applies, for S from last to first, G(S, 0),
// G(S, 1), ... in that order.  Columns of Z are independent: each workgroup
// owns a slab of columns and streams all blocks through LDS.
#include "gemm.h"
#include <stdlib.h>
#include <type_traits>
#include "stages.h"

namespace bdg {
namespace {

constexpr int NBK = 32;     // sweeps per block
constexpr int BMAX = 64;
constexpr int HMAX = BMAX + NBK - 1;
constexpr int HT = 6;       // 16-row tiles covering HMAX (<= 96 rows)
constexpr int VLD = 97;     // LDS leading dimension of V (padding avoids bank conflicts)
constexpr int SLAB = 64;    // columns of Z per workgroup (16 per wave)

// |e_i| of the complex sub-diagonal, one thread per entry (the same hypot as
// the phase scan).
__global__ void abs_kernel(int64_t n, const double *__restrict__ e_cplx, double *__restrict__ e_abs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i + 1 < n) e_abs[i] = hypot(e_cplx[2 * i], e_cplx[2 * i + 1]);
}

// Phase vector: ph_0 = 1, ph_{i+1} = ph_i e_i / |e_i| (renormalised); |e| out
// unless e_abs is null.
__global__ void phases_kernel(int64_t n, const double *__restrict__ e_cplx, double *__restrict__ ph,
                              double *__restrict__ e_abs) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    double pr = 1.0, pi = 0.0;
    ph[0] = 1.0;
    ph[1] = 0.0;
    for (int64_t i = 0; i + 1 < n; ++i) {
        const double er = e_cplx[2 * i], ei = e_cplx[2 * i + 1];
        const double a = hypot(er, ei);
        if (e_abs) e_abs[i] = a;
        if (a > 0.0) {
            const double ur = er / a, ui = ei / a;
            const double nr = pr * ur - pi * ui, ni = pr * ui + pi * ur;
            const double nn = hypot(nr, ni);
            pr = nr / nn;
            pi = ni / nn;
        }
        ph[2 * (i + 1)] = pr;
        ph[2 * (i + 1) + 1] = pi;
    }
}

// Z[:, j] = ph .* Y[:, i0 + j]  (Y real, ld n).  Each element is read once and
// written once at its own position, so a complex64 Z may overwrite Y in place
// (Z = Y + i0 n elements, ldz = n: both are 8-byte elements); Y and Z are not
// declared restrict for that reason.
template <typename F>
__global__ void scale_phase(int64_t n, int64_t m, const double *Y, int64_t i0,
                            const double *__restrict__ ph, F *Z, int64_t ldz) {
    const int64_t j = blockIdx.x;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const double y = Y[i + (i0 + j) * n];
        Z[2 * (i + j * ldz)] = (F)(ph[2 * i] * y);
        Z[2 * (i + j * ldz) + 1] = (F)(ph[2 * i + 1] * y);
    }
}

// Row-major copy with the phase scaling folded in:
// Zrm[r ldr + j] = ph[r] Y[r + (i0 + j) n]  (Y real, ld n); 32 x 32 tiles through LDS.
template <typename F>
__global__ __launch_bounds__(256) void scale_phase_rm(int64_t n, int64_t m, const double *__restrict__ Y,
                                                      int64_t i0, const double *__restrict__ ph,
                                                      F *__restrict__ Zrm, int64_t ldr) {
    __shared__ double tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {  // row r0 + tx of column j0 + k
        const int64_t r = r0 + tx, j = j0 + k;
        tile[k][tx] = (r < n && j < m) ? Y[r + (i0 + j) * n] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {  // column j0 + tx of row r0 + k
        const int64_t r = r0 + k, j = j0 + tx;
        if (r < n && j < m) {
            const double y = tile[tx][k];
            st2<F>(Zrm + 2 * (r * ldr + j), mk2<F>((F)(ph[2 * r] * y), (F)(ph[2 * r + 1] * y)));
        }
    }
}

// Z[r + j ldz] = Zrm[r ldr + j]; 32 x 32 tiles through LDS.
template <typename F>
__global__ __launch_bounds__(256) void rm_to_cm_kernel(int64_t n, int64_t m, const F *__restrict__ Zrm,
                                                       int64_t ldr, F *__restrict__ Z, int64_t ldz) {
    typedef typename v2t<F>::type CV;
    __shared__ CV tile[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int k = ty; k < 32; k += 8) {  // column j0 + tx of row r0 + k
        const int64_t r = r0 + k, j = j0 + tx;
        tile[k][tx] = (r < n && j < m) ? ld2<F>(Zrm + 2 * (r * ldr + j)) : mk2<F>(0.0, 0.0);
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {  // row r0 + tx of column j0 + k
        const int64_t r = r0 + tx, j = j0 + k;
        if (r < n && j < m) st2<F>(Z + 2 * (r + j * ldz), tile[tx][k]);
    }
}

// T factor of every block G(S, t), the compact-WY factor of its reflectors,
// from V^H V over the parallelogram and the scales tau.  One workgroup per block.
template <typename F>
__global__ __launch_bounds__(256) void bt2_tfactors(int64_t n, int b, const F *__restrict__ V2,
                                                    const F *__restrict__ tau2,
                                                    const int64_t *__restrict__ voff, int64_t nsb,
                                                    int64_t tmax, F *__restrict__ TF) {
    typedef typename v2t<F>::type CV;
    __shared__ CV Vs[VLD * NBK];
    __shared__ CV Gs[NBK * NBK];
    __shared__ CV Ts[NBK * NBK];
    __shared__ F ts[NBK];
    const int64_t blk = blockIdx.x;
    const int64_t S = blk / tmax, t = blk % tmax;
    const int64_t s0 = S * NBK;
    const int tid = threadIdx.x;
    const int64_t nsw = n - 2;
    // the first sweep of the block has the most tasks: when it has none at
    // step t, no sweep of the block has, and T is zero
    if (s0 >= nsw || t >= (n - 2 - s0) / b + 1) {
        for (int e = tid; e < NBK * NBK; e += blockDim.x)
            st2<F>(TF + 2 * (blk * NBK * NBK + e), mk2<F>(0.0, 0.0));
        return;
    }
    // parallelogram: column j holds reflector (s0 + j, t) at rows j .. j + b - 1
    for (int e = tid; e < HT * 16 * NBK; e += blockDim.x) {
        const int r = e % (HT * 16), j = e / (HT * 16);
        const int64_t sw = s0 + j;
        CV v = mk2<F>(0.0, 0.0);
        if (sw < nsw && t < (n - 2 - sw) / b + 1) {
            const int o = r - j;
            if (o >= 0 && o < b) v = ld2<F>(V2 + 2 * ((voff[sw] + t) * b + o));
        }
        Vs[r + j * VLD] = v;
    }
    if (tid < NBK) {
        const int64_t sw = s0 + tid;
        ts[tid] = (sw < nsw && t < (n - 2 - sw) / b + 1) ? tau2[voff[sw] + t] : 0.0;
    }
    __syncthreads();
    // G = V^H V (only the strictly upper part is used)
    for (int e = tid; e < NBK * NBK; e += blockDim.x) {
        const int i = e % NBK, j = e / NBK;
        F gr = 0.0, gi = 0.0;
        if (i < j) {
            for (int r = j; r < i + b && r < HT * 16; ++r) {
                const CV a = Vs[r + i * VLD], c = Vs[r + j * VLD];
                gr += a.x * c.x + a.y * c.y;
                gi += a.x * c.y - a.y * c.x;
            }
        }
        Gs[e] = mk2<F>(gr, gi);
        Ts[e] = mk2<F>(0.0, 0.0);
    }
    __syncthreads();
    // T is the inverse of U = diag(1 / tau) + (strictly upper part of G): each
    // quad of lanes solves one column by back substitution,
    //   T[c, c] = tau_c,  T[i, c] = -tau_i sum_{k = i+1 .. c} G[i, k] T[k, c],
    // the four lanes taking every fourth k (a quad's lanes are in one wave,
    // whose LDS accesses complete in order, so no block barrier per step).
    // A zero tau gives a zero row and column.
    {
        const int c = tid >> 2, q = tid & 3;
        if (c < NBK) {
            if (q == 0) Ts[c + c * NBK] = mk2<F>(ts[c], 0.0);
            for (int i = c - 1; i >= 0; --i) {
                F sr = 0.0, si = 0.0;
                for (int k = i + 1 + q; k <= c; k += 4) {
                    const CV g = Gs[i + k * NBK], x = Ts[k + c * NBK];
                    sr += g.x * x.x - g.y * x.y;
                    si += g.x * x.y + g.y * x.x;
                }
                sr = quad_sum(sr);
                si = quad_sum(si);
                if (q == 0) Ts[i + c * NBK] = mk2<F>(-ts[i] * sr, -ts[i] * si);
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < NBK * NBK; e += blockDim.x)
        st2<F>(TF + 2 * (blk * NBK * NBK + e), Ts[e]);
}

// One 16-row tile of the Z window (rows rs + 16 rt + ...) in accumulator layout.
template <typename F>
__device__ __forceinline__ void load_tile(const F *__restrict__ Z, int64_t ldz, int64_t rs, int rt, int lane,
                                          int h, bool colok, int64_t col, typename acc4<F>::type &zr,
                                          typename acc4<F>::type &zi) {
    typedef typename v2t<F>::type CV;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        // unconditional load (entry 0 outside the matrix) so that all loads of
        // a window are in flight together
        const int row = rt * 16 + mfma_row((F)0, lane, q);
        const bool ok = (row < h) & colok;
        const CV z = ld2<F>(Z + (int64_t)ok * (2 * ((rs + row) + col * ldz)));
        zr[q] = ok ? z.x : (F)0;
        zi[q] = ok ? z.y : (F)0;
    }
}

template <typename F>
__device__ __forceinline__ void store_tile(F *__restrict__ Z, int64_t ldz, int64_t rs, int rt, int lane, int h,
                                           bool colok, int64_t col, const typename acc4<F>::type &zr,
                                           const typename acc4<F>::type &zi) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int row = rt * 16 + mfma_row((F)0, lane, q);
        if (row < h && colok) st2<F>(Z + 2 * ((rs + row) + col * ldz), mk2<F>(zr[q], zi[q]));
    }
}

// Apply every block to a slab of SLAB columns on the FP64 matrix cores.
// Each wave keeps its 96 x 16 window of Z in MFMA accumulator layout
// (element r of lane l = row (l/16) + 4 r of a 16-row tile, column l%16).
// The same registers serve as the B operand of the next product with the k
// index permuted accordingly (a sum over k does not depend on its order).
//   W  = V^H Z   (32 x 16)     W2 = T W     Z -= V W2
// Tiles of the parallelogram V that are zero by construction are skipped.
template <typename F, int BB, int OCC>
__global__ __launch_bounds__(256, OCC) void bt2_apply(int64_t n, int b_rt, int64_t m,
                                                 const F *__restrict__ V2,
                                                 const int64_t *__restrict__ voff, int64_t nsb,
                                                 int64_t tmax, const F *__restrict__ TF,
                                                 F *__restrict__ Z, int64_t ldz) {
    typedef typename v2t<F>::type CV;
    typedef typename acc4<F>::type A4;
    // BB > 0: the band width is a compile-time constant, so the tile-skip tests
    // fold and the product loops become straight-line code
    const int b = BB > 0 ? BB : b_rt;
    __shared__ CV Vs[VLD * NBK];
    __shared__ CV Ts[NBK * NBK];
    __shared__ int64_t vb[NBK];  // reflector base of each sweep of the block
    __shared__ int64_t vt[NBK];  // task count of each sweep (0 beyond the last sweep)
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int64_t j0 = (int64_t)blockIdx.x * SLAB;
    const int64_t col = j0 + wave * 16 + li;  // this lane's column of Z
    const bool colok = col < m;
    const int64_t nsw = n - 2;
    for (int64_t S = nsb - 1; S >= 0; --S) {
        const int64_t s0 = S * NBK;
        const int64_t T0 = (n - 2 - s0) / b + 1;
        __syncthreads();
        if (tid < NBK) {
            const int64_t sw = s0 + tid;
            vb[tid] = sw < nsw ? voff[sw] : 0;
            vt[tid] = sw < nsw ? (n - 2 - sw) / b + 1 : 0;
        }
        for (int64_t t = 0; t < T0; ++t) {
            const int64_t rs = s0 + 1 + t * b;
            if (rs >= n) break;
            const int h = (int)min((int64_t)(HT * 16), n - rs);
            __syncthreads();
            {
                CV rt4[NBK * NBK / 256];
#pragma unroll
                for (int i = 0; i < NBK * NBK / 256; ++i)
                    rt4[i] = ld2<F>(TF + 2 * ((S * tmax + t) * NBK * NBK + tid + 256 * i));
                // parallelogram: 96 x 32 entries, 12 per thread, loads issued first
                CV rv[HT * 16 * NBK / 256];
#pragma unroll
                for (int i = 0; i < HT * 16 * NBK / 256; ++i) {
                    // unconditional loads (from entry 0 when outside the
                    // parallelogram) so that all of them are in flight at once
                    const int e = tid + 256 * i;
                    const int r = e % (HT * 16), j = e / (HT * 16);
                    const int o = r - j;
                    const int64_t vbj = vb[j], vtj = vt[j];
                    const bool ok = (r < h) & (o >= 0) & (o < b) & (t < vtj);
                    const CV v = ld2<F>(V2 + (int64_t)ok * (2 * ((vbj + t) * b + o)));
                    rv[i] = ok ? v : mk2<F>(0.0, 0.0);
                }
#pragma unroll
                for (int i = 0; i < HT * 16 * NBK / 256; ++i) {
                    const int e = tid + 256 * i;
                    const int r = e % (HT * 16), j = e / (HT * 16);
                    Vs[r + j * VLD] = rv[i];
                }
#pragma unroll
                for (int i = 0; i < NBK * NBK / 256; ++i) Ts[tid + 256 * i] = rt4[i];
            }
            // Z window in accumulator layout
            A4 zr[HT], zi[HT];
#pragma unroll
            for (int rt = 0; rt < HT; ++rt) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = rt * 16 + mfma_row((F)0, lane, q);
                    const bool ok = row < h && colok;
                    const CV z = ld2<F>(Z + (ok ? 2 * ((rs + row) + col * ldz) : 0));
                    zr[rt][q] = ok ? z.x : (F)0;
                    zi[rt][q] = ok ? z.y : (F)0;
                }
            }
            __syncthreads();
            // W = V^H Z
            A4 wr[2], wi[2];
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                wr[it] = A4{0, 0, 0, 0};
                wi[it] = A4{0, 0, 0, 0};
#pragma unroll
                for (int kt = 0; kt < HT; ++kt) {
                    if (16 * kt + 15 < 16 * it || 16 * kt > 16 * it + 14 + b) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const CV v = Vs[(16 * kt + mfma_row((F)0, lane, q)) + (16 * it + li) * VLD];
                        wr[it] = mfma16(v.x, zr[kt][q], wr[it]);
                        wi[it] = mfma16(v.x, zi[kt][q], wi[it]);
                        wr[it] = mfma16(v.y, zi[kt][q], wr[it]);
                        wi[it] = mfma16(-v.y, zr[kt][q], wi[it]);
                    }
                }
            }
            // W2 = T W   (T upper triangular), stored negated
            A4 ur[2], ui[2];
#pragma unroll
            for (int it = 0; it < 2; ++it) {
                ur[it] = A4{0, 0, 0, 0};
                ui[it] = A4{0, 0, 0, 0};
#pragma unroll
                for (int kt = it; kt < 2; ++kt) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const CV tv = Ts[(16 * it + li) + (16 * kt + mfma_row((F)0, lane, q)) * NBK];
                        ur[it] = mfma16(tv.x, wr[kt][q], ur[it]);
                        ui[it] = mfma16(tv.x, wi[kt][q], ui[it]);
                        ur[it] = mfma16(-tv.y, wi[kt][q], ur[it]);
                        ui[it] = mfma16(tv.y, wr[kt][q], ui[it]);
                    }
                }
                ur[it] = -ur[it];
                ui[it] = -ui[it];
            }
            // Z += V (-W2)
#pragma unroll
            for (int rt = 0; rt < HT; ++rt) {
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) {
                    if (16 * rt + 15 < 16 * kt || 16 * rt > 16 * kt + 14 + b) continue;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const CV v = Vs[(16 * rt + li) + (16 * kt + mfma_row((F)0, lane, q)) * VLD];
                        zr[rt] = mfma16(v.x, ur[kt][q], zr[rt]);
                        zi[rt] = mfma16(v.x, ui[kt][q], zi[rt]);
                        zr[rt] = mfma16(-v.y, ui[kt][q], zr[rt]);
                        zi[rt] = mfma16(v.y, ur[kt][q], zi[rt]);
                    }
                }
            }
#pragma unroll
            for (int rt = 0; rt < HT; ++rt) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int row = rt * 16 + mfma_row((F)0, lane, q);
                    if (row < h && colok)
                        st2<F>(Z + 2 * ((rs + row) + col * ldz), mk2<F>(zr[rt][q], zi[rt][q]));
                }
            }
        }
    }
}

// Copy cnt complex entries from global memory to LDS with direct loads
// (no registers): lane l of each instruction fills the next 16 bytes (FP64)
// or 4 bytes (FP32) after the wave-uniform LDS base.  One wave.  Issued as
// inline assembly so that the compiler does not make the next LDS read wait
// for these loads (it cannot tell that they fill the other buffer); the
// caller waits for them (vmcnt) before the barrier that publishes the data.
template <typename F>
__device__ inline void wave_copy_to_lds(const F *g, typename v2t<F>::type *l, int cnt, int lane) {
    const unsigned lbase = (unsigned)(size_t)(__attribute__((address_space(3))) void *)l;
    if constexpr (sizeof(F) == 8) {
        for (int base = 0; base < cnt; base += 64) {
            const unsigned m0v = __builtin_amdgcn_readfirstlane(lbase + 16u * (unsigned)base);
            if (base + lane < cnt)
                asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dwordx4 %0, off"
                             :: "v"(g + 2 * (base + lane)), "s"(m0v) : "memory", "m0");
        }
    } else {
        for (int base = 0; base < 2 * cnt; base += 64) {
            const unsigned m0v = __builtin_amdgcn_readfirstlane(lbase + 4u * (unsigned)base);
            if (base + lane < 2 * cnt)
                asm volatile("s_mov_b32 m0, %1\n\ts_nop 0\n\tglobal_load_lds_dword %0, off"
                             :: "v"(g + base + lane), "s"(m0v) : "memory", "m0");
        }
    }
}

// Wait for every vector memory operation of this wave.
__device__ inline void wait_vm_all() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Pipelined variant (b a multiple of 16, SHIFT = b / 16 tiles; Z column-major
// with leading dimension ldz, or row-major (RM) with row stride ldz): while
// the matrix cores work on block t, the loads for block t + 1 are in flight:
// its V and T go straight to the other half of a double LDS buffer, and its
// SHIFT new Z tiles (rows the current block does not touch) to registers; the
// window rows shared by consecutive blocks stay in registers.
template <typename F, int SHIFT, bool RM>
__global__ __launch_bounds__(256, 1) void bt2_apply_pipe(int64_t n, int b_rt, int64_t m,
                                                         const F *__restrict__ V2,
                                                         const int64_t *__restrict__ voff, int64_t nsb,
                                                         int64_t tmax, const F *__restrict__ TF,
                                                         F *__restrict__ Z, int64_t ldz) {
    typedef typename v2t<F>::type CV;
    typedef typename acc4<F>::type A4;
    constexpr int b = 16 * SHIFT;  // the launcher guarantees b_rt == 16 SHIFT
    (void)b_rt;
    __shared__ CV Vs[2][VLD * NBK];
    __shared__ CV Ts[2][NBK * NBK];
    __shared__ int64_t vb[NBK];
    __shared__ int64_t vt[NBK];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15;
    const int64_t j0 = (int64_t)blockIdx.x * SLAB;
    const int64_t col = j0 + wave * 16 + li;
    const bool colok = col < m;
    const int64_t nsw = n - 2;
    const CV zero = mk2<F>(0.0, 0.0);
    // Column j of the V parallelogram of block (S, t) is reflector (s0 + j, t),
    // rows j .. j + b - 1 (stored zero-padded past the matrix end); nothing
    // ever writes the rows outside that range, which stay zero from the start.
    // T is the block's 32 x 32 factor, contiguous.  Wave w fills columns
    // w, w + 4, ... and a quarter of T.
    for (int i = tid; i < 2 * VLD * NBK; i += 256) (&Vs[0][0])[i] = zero;
    auto fetch = [&](int64_t S, int64_t t, int bufn) {
#pragma unroll
        for (int k = 0; k < NBK / 4; ++k) {
            const int j = wave + 4 * k;
            CV *dst = &Vs[bufn][j + j * VLD];
            if (t < vt[j]) wave_copy_to_lds<F>(V2 + 2 * (vb[j] + t) * b, dst, b, lane);
            else if (lane < b) dst[lane] = zero;  // no such reflector
        }
        constexpr int TQ = NBK * NBK / 4;
        wave_copy_to_lds<F>(TF + 2 * ((S * tmax + t) * NBK * NBK + wave * TQ), &Ts[bufn][wave * TQ], TQ, lane);
    };
    // complex offset of Z entry (row, this lane's column)
    // Z entry (row, this lane's column) = zl[row * rstr]: zl holds the lane's
    // column, rstr is the row stride; the four rows a lane holds in a tile
    // differ by per-lane constants, so an address costs one add of a uniform
    // row offset (no 64-bit multiply per element).
    const int64_t rstr = RM ? ldz : 1;
    const F *zl = Z + 2 * (RM ? col : col * ldz);
    int64_t lrow[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) lrow[q] = 2 * (int64_t)mfma_row((F)0, lane, q) * rstr;
    // raw loads of one Z tile (rows outside the matrix read the lane's row 0 of
    // the tile block and are zeroed later); ok bits for its 4 entries in zmask
    auto fetch_tile = [&](int64_t rs1, int rtl, int h1, CV *raw, unsigned &zmask, int bit0) {
        const F *base = zl + 2 * (rs1 + rtl * 16) * rstr;  // uniform part
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rtl * 16 + mfma_row((F)0, lane, q);
            const bool ok = (row < h1) & colok;
            raw[q] = ld2<F>(ok ? base + lrow[q] : Z);
            zmask |= (unsigned)ok << (bit0 + q);
        }
    };
    auto put_tile = [&](int64_t rs1, int rtl, int h1, const A4 &tr, const A4 &ti) {
        F *base = (F *)zl + 2 * (rs1 + rtl * 16) * rstr;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int row = rtl * 16 + mfma_row((F)0, lane, q);
            if (row < h1 && colok) st2<F>(base + lrow[q], mk2<F>(tr[q], ti[q]));
        }
    };
    // Tiles that lie wholly inside the matrix (every window but the last of
    // each sweep block, when the workgroup's 64 columns exist): a wave-uniform
    // base address plus this lane's 32-bit byte offset, so each load or store
    // costs one instruction with a scalar base and no bounds selects.  The
    // offsets stay below 2^32 for every n the workspace can hold.
    const bool cols_full = j0 + SLAB <= m;
    uint32_t lofs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
        lofs[q] = (uint32_t)sizeof(CV) *
                  (uint32_t)(RM ? (int64_t)mfma_row((F)0, lane, q) * ldz + (wave * 16 + li)
                                : (int64_t)mfma_row((F)0, lane, q) + (int64_t)(wave * 16 + li) * ldz);
    auto tile_base = [&](int64_t row0) {
        return (char *)Z + sizeof(CV) * (RM ? row0 * ldz + j0 : row0 + j0 * ldz);
    };
    auto fetch_tile_full = [&](int64_t rs1, int rtl, CV *raw) {
        const char *base = tile_base(rs1 + rtl * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) raw[q] = ld2<F>((const F *)(base + lofs[q]));
    };
    auto put_tile_full = [&](int64_t rs1, int rtl, const A4 &tr, const A4 &ti) {
        char *base = tile_base(rs1 + rtl * 16);
#pragma unroll
        for (int q = 0; q < 4; ++q) st2<F>((F *)(base + lofs[q]), mk2<F>(tr[q], ti[q]));
    };
    for (int64_t S = nsb - 1; S >= 0; --S) {
        const int64_t s0 = S * NBK;
        const int64_t T0 = (n - 2 - s0) / b + 1;
        if (s0 + 1 >= n) continue;
        __syncthreads();
        if (tid < NBK) {
            const int64_t sw = s0 + tid;
            vb[tid] = sw < nsw ? voff[sw] : 0;
            vt[tid] = sw < nsw ? (n - 2 - sw) / b + 1 : 0;
        }
        __syncthreads();
        A4 zr[HT], zi[HT];
        {
            const int h0 = (int)min((int64_t)(HT * 16), n - (s0 + 1));
            fetch(S, 0, 0);
            CV raw[HT][4];
            unsigned zm = 0;
#pragma unroll
            for (int rtl = 0; rtl < HT; ++rtl) fetch_tile(s0 + 1, rtl, h0, raw[rtl], zm, 4 * rtl);
            wait_vm_all();
#pragma unroll
            for (int rtl = 0; rtl < HT; ++rtl) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const bool ok = (zm >> (4 * rtl + q)) & 1u;
                    zr[rtl][q] = ok ? raw[rtl][q].x : (F)0;
                    zi[rtl][q] = ok ? raw[rtl][q].y : (F)0;
                }
            }
        }
        __syncthreads();
        for (int64_t t = 0; t < T0; ++t) {
            const int64_t rs = s0 + 1 + t * b;
            const int h = (int)min((int64_t)(HT * 16), n - rs);
            const int buf = (int)(t & 1);
            const bool more = t + 1 < T0 && rs + b < n;
            CV zraw[SHIFT][4];
            unsigned zmask = 0;
            if (more) {
                // the other buffer was last read in block t - 1, before the
                // barrier that closed it
                fetch(S, t + 1, buf ^ 1);
            }
            const CV *V = Vs[buf];
            const CV *T = Ts[buf];
            // The three complex products use three real MFMAs each (Gauss'
            // form: for (a + ib)(c + id), ac, bd and (a + b)(c + d)) instead of
            // four.  Each product is a fixed sequence of steps whose LDS
            // operands are read one step ahead into a second register set;
            // the scheduling barriers keep those reads ahead of the previous
            // step's MFMAs, so LDS latency hides behind them (one wave per SIMD).
            //
            // W = V^H Z:  Re = P1 + P2, Im = P3 + P1 - P2 with
            // P1 = sum vr zr, P2 = sum vi zi, P3 = sum (vr + vi)(zi - zr);
            // step (kt, q) reads V rows 16 kt + .. for column tiles it = 0, 1.
            auto wvalid = [](int kt, int it) { return !(16 * kt + 15 < 16 * it || 16 * kt > 16 * it + 14 + b); };
            A4 wr[2], wi[2];
            {
                A4 p1[2], p2[2], p3[2];
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    p1[it] = A4{0, 0, 0, 0};
                    p2[it] = A4{0, 0, 0, 0};
                    p3[it] = A4{0, 0, 0, 0};
                }
                constexpr int NS = HT * 4;
                CV vc[2], vn[2];
                auto wload = [&](int st, CV *dst) {
                    const int kt = st >> 2, q = st & 3;
#pragma unroll
                    for (int it = 0; it < 2; ++it)
                        if (wvalid(kt, it)) dst[it] = V[(16 * kt + mfma_row((F)0, lane, q)) + (16 * it + li) * VLD];
                };
                wload(0, vc);
#pragma unroll
                for (int st = 0; st < NS; ++st) {
                    if (st + 1 < NS) wload(st + 1, vn);
                    __builtin_amdgcn_sched_barrier(0);
                    const int kt = st >> 2, q = st & 3;
                    const F d = zi[kt][q] - zr[kt][q];
#pragma unroll
                    for (int it = 0; it < 2; ++it) {
                        if (!wvalid(kt, it)) continue;
                        p1[it] = mfma16(vc[it].x, zr[kt][q], p1[it]);
                        p2[it] = mfma16(vc[it].y, zi[kt][q], p2[it]);
                        p3[it] = mfma16(vc[it].x + vc[it].y, d, p3[it]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    vc[0] = vn[0];
                    vc[1] = vn[1];
                }
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    wr[it] = p1[it] + p2[it];
                    wi[it] = p3[it] + p1[it] - p2[it];
                }
            }
            // The SHIFT Z tiles block t + 1 adds to the window are loaded
            // now, behind this block's W = V^H Z: issued at the start of the
            // block, right after the previous block's stores and beside the
            // V/T loads, the same loads made the launch 2.7 % slower.
            const bool nfull = cols_full && n - (rs + b) >= HT * 16;  // window of block t + 1 inside
            if (more) {
                if (nfull) {
#pragma unroll
                    for (int k = 0; k < SHIFT; ++k) fetch_tile_full(rs + b, HT - SHIFT + k, zraw[k]);
                } else {
                    const int h1 = (int)min((int64_t)(HT * 16), n - (rs + b));
#pragma unroll
                    for (int k = 0; k < SHIFT; ++k) fetch_tile(rs + b, HT - SHIFT + k, h1, zraw[k], zmask, 4 * k);
                }
            }
            // W2 = T W (T upper triangular), stored negated:
            // Re = Q1 - Q2, Im = Q3 - Q1 - Q2, Q1 = sum tr wr, Q2 = sum ti wi,
            // Q3 = sum (tr + ti)(wr + wi); steps (it, kt >= it, q).
            A4 ur[2], ui[2];
            {
                A4 sw[2];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) sw[kt] = wr[kt] + wi[kt];
                A4 q1[2], q2[2], q3[2];
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    q1[it] = A4{0, 0, 0, 0};
                    q2[it] = A4{0, 0, 0, 0};
                    q3[it] = A4{0, 0, 0, 0};
                }
                // step st: (it, kt, q) = (0, 0, st) for st < 4, (0, 1, st - 4) for st < 8, (1, 1, st - 8)
                auto tload = [&](int st) {
                    const int it = st >= 8 ? 1 : 0, kt = st >= 4 ? 1 : 0, q = st & 3;
                    return T[(16 * it + li) + (16 * kt + mfma_row((F)0, lane, q)) * NBK];
                };
                CV tc = tload(0), tn;
#pragma unroll
                for (int st = 0; st < 12; ++st) {
                    if (st + 1 < 12) tn = tload(st + 1);
                    __builtin_amdgcn_sched_barrier(0);
                    const int it = st >= 8 ? 1 : 0, kt = st >= 4 ? 1 : 0, q = st & 3;
                    q1[it] = mfma16(tc.x, wr[kt][q], q1[it]);
                    q2[it] = mfma16(tc.y, wi[kt][q], q2[it]);
                    q3[it] = mfma16(tc.x + tc.y, sw[kt][q], q3[it]);
                    __builtin_amdgcn_sched_barrier(0);
                    tc = tn;
                }
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    ur[it] = q2[it] - q1[it];
                    ui[it] = q1[it] + q2[it] - q3[it];
                }
            }
            // Z += V (-W2): per row tile, Re += Q1 - Q2, Im += Q3 - Q1 - Q2 with
            // Q1 = sum vr ur, Q2 = sum vi ui, Q3 = sum (vr + vi)(ur + ui);
            // steps (rtl, kt, q) over the tiles the parallelogram meets.
            {
                A4 su[2];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) su[kt] = ur[kt] + ui[kt];
                constexpr int NS = HT * 8;
                auto uvalid = [&](int st) { return wvalid(st >> 3, (st >> 2) & 1); };
                auto uload = [&](int st) {
                    const int rtl = st >> 3, kt = (st >> 2) & 1, q = st & 3;
                    return V[(16 * rtl + li) + (16 * kt + mfma_row((F)0, lane, q)) * VLD];
                };
                // first valid step, and the valid step after each one
                auto nextv = [&](int st) {
                    int x = st + 1;
                    while (x < NS && !uvalid(x)) ++x;
                    return x;
                };
                // two accumulator sets by row-tile parity: tile rtl - 1 is
                // folded into Z while the MFMAs of tile rtl run
                A4 acc[2][3];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[p][c] = A4{0, 0, 0, 0};
                auto fold = [&](int rtl) {
                    A4 *a = acc[rtl & 1];
                    zr[rtl] += a[0] - a[1];
                    zi[rtl] += a[2] - a[0] - a[1];
                    a[0] = A4{0, 0, 0, 0};
                    a[1] = A4{0, 0, 0, 0};
                    a[2] = A4{0, 0, 0, 0};
                };
                CV uc = uload(nextv(-1)), un;
                int last_rtl = -1;
#pragma unroll
                for (int st = 0; st < NS; ++st) {
                    if (!uvalid(st)) continue;
                    const int nx = nextv(st);
                    if (nx < NS) un = uload(nx);
                    __builtin_amdgcn_sched_barrier(0);
                    const int rtl = st >> 3, kt = (st >> 2) & 1, q = st & 3;
                    A4 *a = acc[rtl & 1];
                    a[0] = mfma16(uc.x, ur[kt][q], a[0]);
                    a[1] = mfma16(uc.y, ui[kt][q], a[1]);
                    a[2] = mfma16(uc.x + uc.y, su[kt][q], a[2]);
                    if (rtl != last_rtl) {  // first step of row tile rtl
                        if (last_rtl >= 0) fold(last_rtl);
                        last_rtl = rtl;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    uc = un;
                }
                fold(last_rtl);
            }
            if (more) {
                // Consume every prefetched value (the direct LDS loads were
                // issued before them) ahead of the first store of this block:
                // stores share the load counter, and a wait placed after
                // (predicated) stores would also wait for them to reach memory.
                A4 inr[SHIFT], ini[SHIFT];
#pragma unroll
                for (int k = 0; k < SHIFT; ++k) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const bool ok = nfull || ((zmask >> (4 * k + q)) & 1u);
                        F a = ok ? zraw[k][q].x : (F)0, c = ok ? zraw[k][q].y : (F)0;
                        // pins the selects (and the wait for the loads) here
                        asm volatile("" : "+v"(a), "+v"(c)::"memory");
                        inr[k][q] = a;
                        ini[k][q] = c;
                    }
                }
                wait_vm_all();  // the direct LDS loads of block t + 1 (nothing else is pending)
                if (cols_full && h == HT * 16) {
#pragma unroll
                    for (int k = 0; k < SHIFT; ++k) put_tile_full(rs, k, zr[k], zi[k]);
                } else {
#pragma unroll
                    for (int k = 0; k < SHIFT; ++k) put_tile(rs, k, h, zr[k], zi[k]);
                }
#pragma unroll
                for (int k = 0; k + SHIFT < HT; ++k) {
                    zr[k] = zr[k + SHIFT];
                    zi[k] = zi[k + SHIFT];
                }
#pragma unroll
                for (int k = 0; k < SHIFT; ++k) {
                    zr[HT - SHIFT + k] = inr[k];
                    zi[HT - SHIFT + k] = ini[k];
                }
                __syncthreads();
            } else {
#pragma unroll
                for (int k = 0; k < HT; ++k) put_tile(rs, k, h, zr[k], zi[k]);
                break;
            }
        }
    }
}

// Steps (row tile rt, column tile kt, k slice q) of the update product
// Z += V (-W2) that meet the V parallelogram of band width B, and for each step
// the next such step: next[st + 1] for st = -1 .. HT * 8 - 1 (HT * 8 when none
// is left).  Built at compile time: a search loop in the unrolled product
// stays a run-time loop of scalar compares and branches.
template <int B>
struct UpdSteps {
    static constexpr int NS = HT * 8;
    int next[NS + 1];
    static constexpr bool valid(int st) {
        const int rt = st >> 3, kt = (st >> 2) & 1;
        return !(16 * rt + 15 < 16 * kt || 16 * rt > 16 * kt + 14 + B);
    }
    constexpr UpdSteps() : next{} {
        int nx = NS;
        for (int st = NS - 1; st >= -1; --st) {
            next[st + 1] = nx;
            if (st >= 0 && valid(st)) nx = st;
        }
    }
};

// Sixteen zero bytes that Z entries outside the matrix are loaded from, and a
// sink their stores go to, so a tile load or store is always the same four
// instructions (no branch, no select).
__device__ __align__(16) double kZeroPad[2] = {0.0, 0.0};
__device__ __align__(16) double kSinkPad[2];

// Band width 64 (SHIFT = 4) variant of the pipelined kernel.  The window's
// six 16-row tiles live in a ring of six register slots: logical tile i of
// block t is slot (4 t + i) mod 6, so the four tiles a block hands back are
// the slots that receive the four tiles the next block adds.  Each outgoing
// tile is stored right after its last update and its slot is refilled at
// once with the next window's tile, straight from memory: no registers hold
// prefetched tiles, and nothing is copied at the end of a block step.  The
// slot map repeats every three blocks, so the block loop is unrolled by three
// with the map as a compile-time constant.  The window is kept as (real,
// imaginary) scalars, which the two halves of a 16-byte load fill in place.
// Lane offsets within a tile are 32-bit: the launcher uses this kernel only
// when 16 rows and 64 columns of Z span less than 2^31 bytes.
//
// Counter discipline: the V/T fetch for block t + 1 is issued at the start
// of block t and followed by exactly 32 vector memory instructions (four
// tiles stored and four loaded, four instructions each, whichever path a tile
// takes), so waiting until at most 32 are outstanding waits for the fetch
// alone.  The next block's first reads of the refilled slots are counted by
// the compiler, which does not see the fetch issued after them; its counts
// then wait for a few more of the older accesses, never for the fetch.
template <typename F, bool RM>
__global__ __launch_bounds__(256, 1) void bt2_apply_ring(int64_t n, int64_t m, const F *__restrict__ V2,
                                                         const int64_t *__restrict__ voff, int64_t nsb,
                                                         int64_t tmax, const F *__restrict__ TF,
                                                         F *__restrict__ Z, int64_t ldz) {
    typedef typename v2t<F>::type CV;
    typedef typename acc4<F>::type A4;
    constexpr int SHIFT = 4, b = 64;
    static_assert(HT == 6 && HT * 16 >= b + NBK - 1, "a ring of six tiles covers the window");
    __shared__ CV Vs[2][VLD * NBK];
    __shared__ CV Ts[2][NBK * NBK];
    __shared__ int64_t vb[NBK];
    __shared__ int64_t vt[NBK];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15;
    const int64_t j0 = (int64_t)blockIdx.x * SLAB;
    const int64_t col = j0 + wave * 16 + li;
    const bool colok = col < m;
    const int64_t nsw = n - 2;
    const CV zero = mk2<F>(0.0, 0.0);
    for (int i = tid; i < 2 * VLD * NBK; i += 256) (&Vs[0][0])[i] = zero;
    auto fetch = [&](int64_t S, int64_t t, int bufn) {
#pragma unroll
        for (int k = 0; k < NBK / 4; ++k) {
            const int j = wave + 4 * k;
            CV *dst = &Vs[bufn][j + j * VLD];
            if (t < vt[j]) wave_copy_to_lds<F>(V2 + 2 * (vb[j] + t) * b, dst, b, lane);
            else if (lane < b) dst[lane] = zero;  // no such reflector
        }
        constexpr int TQ = NBK * NBK / 4;
        wave_copy_to_lds<F>(TF + 2 * ((S * tmax + t) * NBK * NBK + wave * TQ), &Ts[bufn][wave * TQ], TQ, lane);
    };
    // tile addresses: inside the matrix, a wave-uniform base plus this lane's
    // 32-bit byte offset; otherwise per element, with the zero pad and the sink
    const int64_t rstr = RM ? ldz : 1;
    const F *zl = Z + 2 * (RM ? col : col * ldz);
    int64_t lrow[4];
    uint32_t lofs[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        lrow[q] = 2 * (int64_t)mfma_row((F)0, lane, q) * rstr;
        lofs[q] = (uint32_t)sizeof(CV) *
                  (uint32_t)(RM ? (int64_t)mfma_row((F)0, lane, q) * ldz + (wave * 16 + li)
                                : (int64_t)mfma_row((F)0, lane, q) + (int64_t)(wave * 16 + li) * ldz);
    }
    const bool cols_full = j0 + SLAB <= m;
    auto tile_base = [&](int64_t row0) {
        return (char *)Z + sizeof(CV) * (RM ? row0 * ldz + j0 : row0 + j0 * ldz);
    };
    // the ring: logical tile i of block t in slot (4 t + i) mod 6, entry q of a
    // lane's column as (real, imaginary) scalars
    F zx[HT][4], zy[HT][4];
    auto load_tile = [&](int64_t rs1, int rtl, int h1, bool full, int slot) __attribute__((always_inline)) {
        if (full) {
            const char *base = tile_base(rs1 + rtl * 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const CV v = ld2<F>((const F *)(base + lofs[q]));
                zx[slot][q] = v.x;
                zy[slot][q] = v.y;
            }
        } else {
            const F *base = zl + 2 * (rs1 + rtl * 16) * rstr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = rtl * 16 + mfma_row((F)0, lane, q);
                const bool ok = (row < h1) & colok;
                const CV v = ld2<F>(ok ? base + lrow[q] : (const F *)kZeroPad);
                zx[slot][q] = v.x;
                zy[slot][q] = v.y;
            }
        }
    };
    auto store_tile = [&](int64_t rs1, int rtl, int h1, bool full, int slot) __attribute__((always_inline)) {
        if (full) {
            char *base = tile_base(rs1 + rtl * 16);
#pragma unroll
            for (int q = 0; q < 4; ++q) st2<F>((F *)(base + lofs[q]), mk2<F>(zx[slot][q], zy[slot][q]));
        } else {
            F *base = (F *)zl + 2 * (rs1 + rtl * 16) * rstr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int row = rtl * 16 + mfma_row((F)0, lane, q);
                const bool ok = (row < h1) & colok;
                st2<F>(ok ? base + lrow[q] : (F *)kSinkPad, mk2<F>(zx[slot][q], zy[slot][q]));
            }
        }
    };
    auto wvalid = [](int kt, int it) { return !(16 * kt + 15 < 16 * it || 16 * kt > 16 * it + 14 + b); };
    for (int64_t S = nsb - 1; S >= 0; --S) {
        const int64_t s0 = S * NBK;
        const int64_t T0 = (n - 2 - s0) / b + 1;
        if (s0 + 1 >= n) continue;
        __syncthreads();
        if (tid < NBK) {
            const int64_t sw = s0 + tid;
            vb[tid] = sw < nsw ? voff[sw] : 0;
            vt[tid] = sw < nsw ? (n - 2 - sw) / b + 1 : 0;
        }
        __syncthreads();
        {
            const int h0 = (int)min((int64_t)(HT * 16), n - (s0 + 1));
            fetch(S, 0, 0);
#pragma unroll
            for (int i = 0; i < HT; ++i) load_tile(s0 + 1, i, h0, cols_full && h0 == HT * 16, i);
            wait_vm_all();
        }
        __syncthreads();
        // one block step with the slot map of phase P; false after the last block
        // (inlined: the ring must stay in registers)
        auto block = [&](int64_t t, auto Pc) __attribute__((always_inline)) -> bool {
            constexpr int P = decltype(Pc)::value;
            auto sl = [](int i) { return (4 * P + i) % HT; };
            const int64_t rs = s0 + 1 + t * b;
            const int h = (int)min((int64_t)(HT * 16), n - rs);
            const int buf = (int)(t & 1);
            const bool more = t + 1 < T0 && rs + b < n;
            const bool full = cols_full && h == HT * 16;
            const bool nfull = cols_full && n - (rs + b) >= HT * 16;
            const int h1 = (int)min((int64_t)(HT * 16), n - (rs + b));
            const CV *V = Vs[buf];
            const CV *T = Ts[buf];
            // V and T of block t + 1 into the other buffer (last read in block
            // t - 1, before the barrier that closed it)
            if (more) fetch(S, t + 1, buf ^ 1);
            // W = V^H Z in Gauss' three-product form (as in the kernel above)
            A4 wr[2], wi[2];
            {
                A4 p1[2], p2[2], p3[2];
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    p1[it] = A4{0, 0, 0, 0};
                    p2[it] = A4{0, 0, 0, 0};
                    p3[it] = A4{0, 0, 0, 0};
                }
                constexpr int NS = HT * 4;
                CV vc[2], vn[2];
                auto wload = [&](int st, CV *dst) {
                    const int kt = st >> 2, q = st & 3;
#pragma unroll
                    for (int it = 0; it < 2; ++it)
                        if (wvalid(kt, it)) dst[it] = V[(16 * kt + mfma_row((F)0, lane, q)) + (16 * it + li) * VLD];
                };
                wload(0, vc);
#pragma unroll
                for (int st = 0; st < NS; ++st) {
                    if (st + 1 < NS) wload(st + 1, vn);
                    __builtin_amdgcn_sched_barrier(0);
                    const int kt = st >> 2, q = st & 3;
                    const F zre = zx[sl(kt)][q], zim = zy[sl(kt)][q];
                    const F d = zim - zre;
#pragma unroll
                    for (int it = 0; it < 2; ++it) {
                        if (!wvalid(kt, it)) continue;
                        p1[it] = mfma16(vc[it].x, zre, p1[it]);
                        p2[it] = mfma16(vc[it].y, zim, p2[it]);
                        p3[it] = mfma16(vc[it].x + vc[it].y, d, p3[it]);
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    vc[0] = vn[0];
                    vc[1] = vn[1];
                }
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    wr[it] = p1[it] + p2[it];
                    wi[it] = p3[it] + p1[it] - p2[it];
                }
            }
            // W2 = T W, stored negated
            A4 ur[2], ui[2];
            {
                A4 sw[2];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) sw[kt] = wr[kt] + wi[kt];
                A4 q1[2], q2[2], q3[2];
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    q1[it] = A4{0, 0, 0, 0};
                    q2[it] = A4{0, 0, 0, 0};
                    q3[it] = A4{0, 0, 0, 0};
                }
                auto tload = [&](int st) {
                    const int it = st >= 8 ? 1 : 0, kt = st >= 4 ? 1 : 0, q = st & 3;
                    return T[(16 * it + li) + (16 * kt + mfma_row((F)0, lane, q)) * NBK];
                };
                CV tc = tload(0), tn;
#pragma unroll
                for (int st = 0; st < 12; ++st) {
                    if (st + 1 < 12) tn = tload(st + 1);
                    __builtin_amdgcn_sched_barrier(0);
                    const int it = st >= 8 ? 1 : 0, kt = st >= 4 ? 1 : 0, q = st & 3;
                    q1[it] = mfma16(tc.x, wr[kt][q], q1[it]);
                    q2[it] = mfma16(tc.y, wi[kt][q], q2[it]);
                    q3[it] = mfma16(tc.x + tc.y, sw[kt][q], q3[it]);
                    __builtin_amdgcn_sched_barrier(0);
                    tc = tn;
                }
#pragma unroll
                for (int it = 0; it < 2; ++it) {
                    ur[it] = q2[it] - q1[it];
                    ui[it] = q1[it] + q2[it] - q3[it];
                }
            }
            // Z += V (-W2); each outgoing tile is stored after its last fold
            // and its slot refilled with the next window's tile
            {
                A4 su[2];
#pragma unroll
                for (int kt = 0; kt < 2; ++kt) su[kt] = ur[kt] + ui[kt];
                constexpr int NS = HT * 8;
                auto uvalid = [&](int st) { return wvalid(st >> 3, (st >> 2) & 1); };
                constexpr UpdSteps<b> usteps{};
                auto nextv = [&](int st) { return usteps.next[st + 1]; };
                auto uload = [&](int st) {
                    const int rtl = st >> 3, kt = (st >> 2) & 1, q = st & 3;
                    return V[(16 * rtl + li) + (16 * kt + mfma_row((F)0, lane, q)) * VLD];
                };
                A4 acc[2][3];
#pragma unroll
                for (int p = 0; p < 2; ++p)
#pragma unroll
                    for (int c = 0; c < 3; ++c) acc[p][c] = A4{0, 0, 0, 0};
                auto fold = [&](int rtl) __attribute__((always_inline)) {
                    A4 *a = acc[rtl & 1];
                    const int slot = sl(rtl);
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        zx[slot][q] += a[0][q] - a[1][q];
                        zy[slot][q] += a[2][q] - a[0][q] - a[1][q];
                    }
                    a[0] = A4{0, 0, 0, 0};
                    a[1] = A4{0, 0, 0, 0};
                    a[2] = A4{0, 0, 0, 0};
                    if (rtl < SHIFT) {
                        store_tile(rs, rtl, h, full, slot);
                        if (more) load_tile(rs + b, rtl + HT - SHIFT, h1, nfull, slot);
                    }
                };
                CV uc = uload(nextv(-1)), un;
                int last_rtl = -1;
#pragma unroll
                for (int st = 0; st < NS; ++st) {
                    if (!uvalid(st)) continue;
                    const int nx = nextv(st);
                    if (nx < NS) un = uload(nx);
                    __builtin_amdgcn_sched_barrier(0);
                    const int rtl = st >> 3, kt = (st >> 2) & 1, q = st & 3;
                    A4 *a = acc[rtl & 1];
                    a[0] = mfma16(uc.x, ur[kt][q], a[0]);
                    a[1] = mfma16(uc.y, ui[kt][q], a[1]);
                    a[2] = mfma16(uc.x + uc.y, su[kt][q], a[2]);
                    if (rtl != last_rtl) {  // first step of row tile rtl
                        if (last_rtl >= 0) fold(last_rtl);
                        last_rtl = rtl;
                    }
                    __builtin_amdgcn_sched_barrier(0);
                    uc = un;
                }
                fold(last_rtl);
            }
            if (more) {
                // the V/T fetch is older than the 32 tile accesses after it
                asm volatile("s_waitcnt vmcnt(32)" ::: "memory");
                __syncthreads();
                return true;
            }
#pragma unroll
            for (int i = SHIFT; i < HT; ++i) store_tile(rs, i, h, full, sl(i));
            return false;
        };
        for (int64_t t = 0;; t += 3) {
            if (!block(t, std::integral_constant<int, 0>{})) break;
            if (!block(t + 1, std::integral_constant<int, 1>{})) break;
            if (!block(t + 2, std::integral_constant<int, 2>{})) break;
        }
    }
}

}  // namespace

bool bt2_rowmajor_ok(int b) { return b >= 16 && b <= BMAX && b % 16 == 0; }

int64_t bt2_nblocks(int64_t n, int b) {
    const int64_t nsw = n - 2;
    if (nsw <= 0) return 0;
    const int64_t nsb = (nsw + NBK - 1) / NBK;
    const int64_t tmax = (n - 2) / b + 1;
    return nsb * tmax;
}

size_t bt2_workspace(int64_t n, int b) { return 16 * (size_t)bt2_nblocks(n, b) * NBK * NBK + 256; }

int phases(int64_t n, const double *e_cplx, double *ph, double *e_abs, hipStream_t s) {
    hipLaunchKernelGGL(phases_kernel, dim3(1), dim3(64), 0, s, n, e_cplx, ph, e_abs);
    BDG_CHECK_LAUNCH();
    return 0;
}

int phase_abs(int64_t n, const double *e_cplx, double *e_abs, hipStream_t s) {
    if (n < 2) return 0;
    hipLaunchKernelGGL(abs_kernel, dim3((unsigned)((n - 1 + 255) / 256)), dim3(256), 0, s, n, e_cplx, e_abs);
    BDG_CHECK_LAUNCH();
    return 0;
}

int phase_scan(int64_t n, const double *e_cplx, double *ph, hipStream_t s) {
    hipLaunchKernelGGL(phases_kernel, dim3(1), dim3(64), 0, s, n, e_cplx, ph, (double *)nullptr);
    BDG_CHECK_LAUNCH();
    return 0;
}

template <typename F>
int phase_scale_t(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, F *Z,
                  int64_t ldz, hipStream_t s) {
    if (m <= 0) return 0;
    hipLaunchKernelGGL((scale_phase<F>), dim3((unsigned)m), dim3(256), 0, s, n, m, Y, i0, ph, Z, ldz);
    BDG_CHECK_LAUNCH();
    return 0;
}

template <typename F>
int phase_scale_rm_t(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, F *Zrm,
                     int64_t ldr, hipStream_t s) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL((scale_phase_rm<F>), dim3((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32)), dim3(256),
                       0, s, n, m, Y, i0, ph, Zrm, ldr);
    BDG_CHECK_LAUNCH();
    return 0;
}

template <typename F>
int rm_to_cm_t(int64_t n, int64_t m, const F *Zrm, int64_t ldr, F *Z, int64_t ldz, hipStream_t s) {
    if (m <= 0 || n <= 0) return 0;
    hipLaunchKernelGGL((rm_to_cm_kernel<F>), dim3((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32)), dim3(256),
                       0, s, n, m, Zrm, ldr, Z, ldz);
    BDG_CHECK_LAUNCH();
    return 0;
}

template <typename F>
int bt2_prepare_t(int64_t n, int b, const F *V2, const F *tau2, const int64_t *voff, void *work,
                  hipStream_t s) {
    if (n < 3) return 0;
    if (b > BMAX) return BDG_ERR_NOT_IMPLEMENTED;
    const int64_t nsw = n - 2;
    const int64_t nsb = (nsw + NBK - 1) / NBK;
    const int64_t tmax = (n - 2) / b + 1;
    hipLaunchKernelGGL((bt2_tfactors<F>), dim3((unsigned)(nsb * tmax)), dim3(256), 0, s, n, b, V2, tau2,
                       voff, nsb, tmax, (F *)work);
    BDG_CHECK_LAUNCH();
    return 0;
}

template <typename F>
int bt2_apply_t(int64_t n, int b, int64_t m, const F *V2, const int64_t *voff, F *Z, int64_t ldz,
                void *work, hipStream_t s, bool rm = false) {
    if (n < 3 || m <= 0) return 0;
    if (b > BMAX) return BDG_ERR_NOT_IMPLEMENTED;
    const int64_t nsw = n - 2;
    const int64_t nsb = (nsw + NBK - 1) / NBK;
    const int64_t tmax = (n - 2) / b + 1;
    const dim3 grid((unsigned)((m + SLAB - 1) / SLAB));
    const F *TFw = (const F *)work;
    // band widths that are a multiple of 16 (the default 64): the pipelined
    // kernel, one workgroup per CU (more slabs than CUs run in rounds, still
    // ahead of two-per-CU occupancy: 23.7 s for the generic kernel at 384
    // slabs of the 32x32x24 workload against an estimated 2 x 10.3 s);
    // other widths: the generic kernel, two workgroups per CU
    // Z row-major (rm, row stride ldz): the pipelined kernel only
    if (rm && !bt2_rowmajor_ok(b)) {
        set_error("bt2: a row-major Z needs a band width that is a multiple of 16");
        return BDG_ERR_NOT_IMPLEMENTED;
    }
#define BDG_BT2_PIPE(SH)                                                                                     \
    if (rm) hipLaunchKernelGGL((bt2_apply_pipe<F, SH, true>), grid, dim3(256), 0, s, n, b, m, V2, voff, nsb, \
                               tmax, TFw, Z, ldz);                                                           \
    else hipLaunchKernelGGL((bt2_apply_pipe<F, SH, false>), grid, dim3(256), 0, s, n, b, m, V2, voff, nsb,   \
                            tmax, TFw, Z, ldz);
    // band 64: the ring-window kernel (BDG_BT2_RING=0 selects the pipelined one)
    static const bool ring_env = [] {
        const char *v = getenv("BDG_BT2_RING");
        return !(v && v[0] == '0');
    }();
    switch (b % 16 == 0 ? b / 16 : 0) {
        case 1: BDG_BT2_PIPE(1) break;
        case 2: BDG_BT2_PIPE(2) break;
        case 3: BDG_BT2_PIPE(3) break;
        case 4:
            if (!ring_env || (int64_t)sizeof(F) * 2 * (16 + SLAB * ldz) >= ((int64_t)1 << 31)) {
                BDG_BT2_PIPE(4)
            } else if (rm) {
                hipLaunchKernelGGL((bt2_apply_ring<F, true>), grid, dim3(256), 0, s, n, m, V2, voff, nsb, tmax, TFw, Z, ldz);
            } else {
                hipLaunchKernelGGL((bt2_apply_ring<F, false>), grid, dim3(256), 0, s, n, m, V2, voff, nsb, tmax, TFw, Z, ldz);
            }
            break;
        default: hipLaunchKernelGGL((bt2_apply<F, 0, 2>), grid, dim3(256), 0, s, n, b, m, V2, voff, nsb, tmax, TFw, Z, ldz); break;
    }
#undef BDG_BT2_PIPE
    BDG_CHECK_LAUNCH();
    return 0;
}

template <typename F>
int bt2_t(int64_t n, int b, int64_t m, const F *V2, const F *tau2, const int64_t *voff, F *Z,
          int64_t ldz, void *work, hipStream_t s) {
    if (n < 3 || m <= 0) return 0;
    BDG_TRY(bt2_prepare_t<F>(n, b, V2, tau2, voff, work, s));
    return bt2_apply_t<F>(n, b, m, V2, voff, Z, ldz, work, s);
}

}  // namespace bdg

namespace bdg {

int phase_scale(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, double *Z,
                int64_t ldz, hipStream_t s) {
    return phase_scale_t<double>(n, m, Y, i0, ph, Z, ldz, s);
}
int phase_scale(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, float *Z,
                int64_t ldz, hipStream_t s) {
    return phase_scale_t<float>(n, m, Y, i0, ph, Z, ldz, s);
}
int bt2(int64_t n, int b, int64_t m, const double *V2, const double *tau2, const int64_t *voff,
        double *Z, int64_t ldz, void *work, hipStream_t s) {
    return bt2_t<double>(n, b, m, V2, tau2, voff, Z, ldz, work, s);
}
int bt2(int64_t n, int b, int64_t m, const float *V2, const float *tau2, const int64_t *voff,
        float *Z, int64_t ldz, void *work, hipStream_t s) {
    return bt2_t<float>(n, b, m, V2, tau2, voff, Z, ldz, work, s);
}

}  // namespace bdg

namespace bdg {

int bt2_prepare(int64_t n, int b, const double *V2, const double *tau2, const int64_t *voff,
                void *work, hipStream_t s) {
    return bt2_prepare_t<double>(n, b, V2, tau2, voff, work, s);
}
int bt2_prepare(int64_t n, int b, const float *V2, const float *tau2, const int64_t *voff,
                void *work, hipStream_t s) {
    return bt2_prepare_t<float>(n, b, V2, tau2, voff, work, s);
}
int bt2_apply_blocks(int64_t n, int b, int64_t m, const double *V2, const int64_t *voff, double *Z,
                     int64_t ldz, void *work, hipStream_t s) {
    return bt2_apply_t<double>(n, b, m, V2, voff, Z, ldz, work, s);
}
int bt2_apply_blocks(int64_t n, int b, int64_t m, const float *V2, const int64_t *voff, float *Z,
                     int64_t ldz, void *work, hipStream_t s) {
    return bt2_apply_t<float>(n, b, m, V2, voff, Z, ldz, work, s);
}

}  // namespace bdg

namespace bdg {

int phase_scale_rm(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, double *Zrm,
                   int64_t ldr, hipStream_t s) {
    return phase_scale_rm_t<double>(n, m, Y, i0, ph, Zrm, ldr, s);
}
int phase_scale_rm(int64_t n, int64_t m, const double *Y, int64_t i0, const double *ph, float *Zrm,
                   int64_t ldr, hipStream_t s) {
    return phase_scale_rm_t<float>(n, m, Y, i0, ph, Zrm, ldr, s);
}
int bt2_apply_blocks_rm(int64_t n, int b, int64_t m, const double *V2, const int64_t *voff, double *Zrm,
                        int64_t ldr, void *work, hipStream_t s) {
    return bt2_apply_t<double>(n, b, m, V2, voff, Zrm, ldr, work, s, true);
}
int bt2_apply_blocks_rm(int64_t n, int b, int64_t m, const float *V2, const int64_t *voff, float *Zrm,
                        int64_t ldr, void *work, hipStream_t s) {
    return bt2_apply_t<float>(n, b, m, V2, voff, Zrm, ldr, work, s, true);
}
int rm_to_cm(int64_t n, int64_t m, const double *Zrm, int64_t ldr, double *Z, int64_t ldz, hipStream_t s) {
    return rm_to_cm_t<double>(n, m, Zrm, ldr, Z, ldz, s);
}
int rm_to_cm(int64_t n, int64_t m, const float *Zrm, int64_t ldr, float *Z, int64_t ldz, hipStream_t s) {
    return rm_to_cm_t<float>(n, m, Zrm, ldr, Z, ldz, s);
}

}  // namespace bdg
