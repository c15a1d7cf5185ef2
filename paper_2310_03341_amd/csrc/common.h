// Shared device/host helpers of the BdG eigensolver library (gfx950 only).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "../../include/bdg.h"

namespace bdg {

typedef double __attribute__((ext_vector_type(4))) d4;
typedef float __attribute__((ext_vector_type(4))) f4;

// Interleaved complex scalar used on both host and device.
template <typename T>
struct cx {
    T re, im;
};
typedef cx<double> zd;
typedef cx<float> cf;

template <typename T>
__host__ __device__ inline cx<T> mk(T r, T i) { cx<T> z; z.re = r; z.im = i; return z; }
template <typename T>
__host__ __device__ inline cx<T> cadd(cx<T> a, cx<T> b) { return mk(a.re + b.re, a.im + b.im); }
template <typename T>
__host__ __device__ inline cx<T> csub(cx<T> a, cx<T> b) { return mk(a.re - b.re, a.im - b.im); }
template <typename T>
__host__ __device__ inline cx<T> cmul(cx<T> a, cx<T> b) { return mk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
// conj(a) * b
template <typename T>
__host__ __device__ inline cx<T> cjmul(cx<T> a, cx<T> b) { return mk(a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re); }
template <typename T>
__host__ __device__ inline cx<T> cconj(cx<T> a) { return mk(a.re, -a.im); }
template <typename T>
__host__ __device__ inline cx<T> cscale(cx<T> a, T s) { return mk(a.re * s, a.im * s); }
template <typename T>
__host__ __device__ inline T cabs2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// MFMA 16x16x4 (one block).  Operand lane layout: lane l supplies A[l%16][l/16]
// and B[l/16][l%16].  Accumulator element r of lane l holds D[row][l%16] with
// row = (l/16) + 4 r for the f64 instruction and row = 4 (l/16) + r for the
// f32 one (measured on gfx950; see mfma_row).
__device__ inline d4 mfma16(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mfma16(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ inline int mfma_row(double, int lane, int r) { return (lane >> 4) + 4 * r; }
__device__ inline int mfma_row(float, int lane, int r) { return 4 * (lane >> 4) + r; }
template <typename T> struct acc4;
template <> struct acc4<double> { typedef d4 type; };
template <> struct acc4<float> { typedef f4 type; };

// Two-component vector of a real type (interleaved complex element).
template <typename T> struct v2t;
template <> struct v2t<double> { typedef double2 type; };
template <> struct v2t<float> { typedef float2 type; };
template <typename T>
__host__ __device__ inline typename v2t<T>::type mk2(T x, T y) {
    typename v2t<T>::type v;
    v.x = x;
    v.y = y;
    return v;
}
// 16-byte (8-byte for float) loads and stores of one complex element through
// the native vector type: a copy of the HIP vector struct is a memcpy that
// keeps arrays of such values out of registers.
template <typename T> struct nv2;
template <> struct nv2<double> { typedef double __attribute__((ext_vector_type(2))) type; };
template <> struct nv2<float> { typedef float __attribute__((ext_vector_type(2))) type; };
template <typename T>
__device__ inline typename v2t<T>::type ld2(const T *p) {
    const typename nv2<T>::type v = *(const typename nv2<T>::type *)p;
    return mk2<T>(v.x, v.y);
}
template <typename T>
__device__ inline void st2(T *p, typename v2t<T>::type v) {
    typename nv2<T>::type w;
    w.x = v.x;
    w.y = v.y;
    *(typename nv2<T>::type *)p = w;
}

// c ? a : b per component (a select of whole structs goes through memory)
template <typename V>
__device__ inline V sel2(bool c, V a, V b) {
    V r;
    r.x = c ? a.x : b.x;
    r.y = c ? a.y : b.y;
    return r;
}

// Wave-level reductions (64 lanes).
template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Wave sum through DPP lane moves (no LDS round trips); the total is valid
// in lane 63 only.  Pairs, quads, half rows, rows (mirrors), then the row
// broadcasts 15 and 31 fold rows 0 + 1 into 1, 2 + 3 into 3, and 1 into 3.
template <int CTRL, int ROWMASK>
__device__ inline double dpp_fold(double v) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)bits, CTRL, ROWMASK, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(bits >> 32), CTRL, ROWMASK, 0xf, false);
    return v + __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
template <int CTRL, int ROWMASK>
__device__ inline float dpp_fold(float v) {
    const int t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWMASK, 0xf, false);
    return v + __int_as_float(t);
}
template <typename T>
__device__ inline T wave_sum_last(T v) {
    v = dpp_fold<0xB1, 0xf>(v);   // quad_perm [1, 0, 3, 2]
    v = dpp_fold<0x4E, 0xf>(v);   // quad_perm [2, 3, 0, 1]
    v = dpp_fold<0x141, 0xf>(v);  // row_half_mirror
    v = dpp_fold<0x140, 0xf>(v);  // row_mirror
    v = dpp_fold<0x142, 0xa>(v);  // row_bcast:15 into rows 1, 3
    v = dpp_fold<0x143, 0xc>(v);  // row_bcast:31 into rows 2, 3
    return v;
}

// Sum over each group of 4 consecutive lanes, to all 4 (DPP quad permutes).
template <typename T>
__device__ inline T quad_sum(T v) {
    v = dpp_fold<0xB1, 0xf>(v);  // quad_perm [1, 0, 3, 2]
    v = dpp_fold<0x4E, 0xf>(v);  // quad_perm [2, 3, 0, 1]
    return v;
}

// Block-level sum over blockDim.x threads (multiple of 64), result to all.
template <typename T>
__device__ inline T block_sum(T v, T* red /* >= blockDim.x/64 */) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    T s = 0;
    const int nw = blockDim.x >> 6;
    for (int i = 0; i < nw; ++i) s += red[i];
    __syncthreads();
    return s;
}

}  // namespace bdg

// ---- host-side error plumbing -------------------------------------------------
namespace bdg {
void set_error(const char* fmt, ...);
// true when the environment sets BDG_VERBOSE (progress lines on stderr)
bool verbose();
// false when the environment sets BDG_NO_LOOKAHEAD (stage 1 on one stream)
bool lookahead();
int hip_fail(hipError_t e, const char* what, const char* file, int line);
}  // namespace bdg

#define BDG_HIP(call)                                                               \
    do {                                                                            \
        hipError_t _e = (call);                                                     \
        if (_e != hipSuccess) return bdg::hip_fail(_e, #call, __FILE__, __LINE__);  \
    } while (0)

#define BDG_CHECK_LAUNCH() BDG_HIP(hipGetLastError())

#define BDG_TRY(call)                 \
    do {                              \
        int _rc = (call);             \
        if (_rc != 0) return _rc;     \
    } while (0)
