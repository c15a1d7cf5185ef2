// Start-field network of the learned SCF start: 4 periodic 3x3 conv layers,
// FP32 master weights, BF16 activations, BF16 MFMA with FP32 accumulation.
//
//   x0 = (Vext - mu, cos theta, sin theta);  x_{l+1} = relu(conv(x_l));  y = conv(x3)
//   y[0] = U - Vext, y[1] = |Delta|  (the starting fields of the SLDA iteration)
//
// conv is an implicit GEMM: M = output channels, N = pixels, K = 9 x input
// channels gathered on the fly with periodic wrap-around (the lattice is a
// torus).  The data gradient is the same product with the transposed,
// spatially flipped weights; weight and bias gradients are FP32 reductions.
#include <math.h>

#include <mutex>

#include "net.h"

namespace bdg {
namespace {

typedef short __attribute__((ext_vector_type(4))) s4;

__device__ inline unsigned short f2bf(float f) {
    unsigned int u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
    return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

// MFMA 16x16x16 bf16: lane l supplies A[l%16][4(l/16)+q] and B[4(l/16)+q][l%16],
// q = 0..3; the f32 accumulator holds D[4(l/16)+r][l%16].
__device__ inline f4 mfma_bf16(s4 a, s4 b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// out[b, o, p] = act(bias[o] + sum_k Wk[o, k] in[b, c(k), p + d(k)]),  k = 9 c + 3 dy + dx
// grid: (ceil(P / 64), batch), block 256: wave w -> pixels p0 + 16 w .. +15, all o.
__global__ __launch_bounds__(256) void conv_mfma(int Cin, int Cout, int Ny, int Nx,
                                                const unsigned short *__restrict__ in,
                                                const unsigned short *__restrict__ Wk,
                                                const float *__restrict__ bias, int relu,
                                                unsigned short *__restrict__ out_bf,
                                                float *__restrict__ out_f) {
    const int P = Ny * Nx;
    const int K = 9 * Cin;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int b = blockIdx.y;
    const int p = blockIdx.x * 64 + wave * 16 + (lane & 15);
    const int py = p / Nx, px = p % Nx;
    const bool pok = p < P;
    const unsigned short *inb = in + (size_t)b * Cin * P;
    const int Mt = (Cout + 15) / 16;
    f4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        s4 bv;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int k = k0 + 4 * (lane >> 4) + q;
            unsigned short v = 0;
            if (pok && k < K) {
                const int c = k / 9, r = k % 9, dy = r / 3, dx = r % 3;
                int yy = py + dy - 1, xx = px + dx - 1;
                yy += (yy < 0) ? Ny : 0; yy -= (yy >= Ny) ? Ny : 0;
                xx += (xx < 0) ? Nx : 0; xx -= (xx >= Nx) ? Nx : 0;
                v = inb[(size_t)c * P + yy * Nx + xx];
            }
            bv[q] = (short)v;
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            if (t >= Mt) break;
            s4 av;
            const int o = t * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int k = k0 + 4 * (lane >> 4) + q;
                av[q] = (short)((o < Cout && k < K) ? Wk[(size_t)o * K + k] : 0);
            }
            acc[t] = mfma_bf16(av, bv, acc[t]);
        }
    }
    if (!pok) return;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        if (t >= Mt) break;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int o = t * 16 + 4 * (lane >> 4) + r;
            if (o >= Cout) continue;
            float v = acc[t][r] + (bias ? bias[o] : 0.f);
            if (relu) v = fmaxf(v, 0.f);
            const size_t idx = ((size_t)b * Cout + o) * P + p;
            if (out_bf) out_bf[idx] = f2bf(v);
            if (out_f) out_f[idx] = v;
        }
    }
}

// x0 = (Vext - mu, cos theta, sin theta) in bf16
__global__ void features_kernel(int batch, int P, const double *__restrict__ Vext,
                                const double *__restrict__ theta, double mu,
                                unsigned short *__restrict__ x0) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < batch * P; i += gridDim.x * blockDim.x) {
        const int b = i / P, p = i % P;
        double sn, cs;
        sincos(theta[i], &sn, &cs);
        x0[((size_t)b * 3 + 0) * P + p] = f2bf((float)(Vext[i] - mu));
        x0[((size_t)b * 3 + 1) * P + p] = f2bf((float)cs);
        x0[((size_t)b * 3 + 2) * P + p] = f2bf((float)sn);
    }
}

// bf16 copies of the weights: forward Wk[o][c*9+d] and data-gradient Wt[c][o*9+(8-d)]
__global__ void weights_bf16(int Cin, int Cout, const float *__restrict__ W,
                             unsigned short *__restrict__ Wk, unsigned short *__restrict__ Wt) {
    const int total = Cout * Cin * 9;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int o = i / (Cin * 9), rem = i % (Cin * 9), c = rem / 9, d = rem % 9;
        const unsigned short h = f2bf(W[i]);
        Wk[i] = h;
        if (Wt) Wt[(size_t)c * (Cout * 9) + o * 9 + (8 - d)] = h;
    }
}

// loss partials and output gradient g = 2 (y - t) / N (fp32 and bf16 copies)
__global__ void mse_kernel(int total, const float *__restrict__ y, const float *__restrict__ t,
                           float *__restrict__ g, unsigned short *__restrict__ gbf,
                           float *__restrict__ part) {
    __shared__ float red[16];
    float s = 0.f;
    const float inv = 2.f / (float)total;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const float d = y[i] - t[i];
        s += d * d;
        g[i] = inv * d;
        gbf[i] = f2bf(inv * d);
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void sum_partials(int n, const float *__restrict__ part, float scale, float *__restrict__ out) {
    __shared__ float red[16];
    float s = 0.f;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += part[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) out[0] = s * scale;
}

// g_in = g_out_conv * (h > 0)  (relu backward), fp32 and bf16
__global__ void relu_back(int total, const float *__restrict__ gx, const unsigned short *__restrict__ h,
                          float *__restrict__ g, unsigned short *__restrict__ gbf) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const float v = (bf2f(h[i]) > 0.f) ? gx[i] : 0.f;
        g[i] = v;
        gbf[i] = f2bf(v);
    }
}

// dW[o][c][d] = sum_{b,p} g[b,o,p] x[b,c,p+d];  grid (Cin, Cout), block 256
__global__ __launch_bounds__(256) void conv_wgrad(int batch, int Cin, int Cout, int Ny, int Nx,
                                                  const float *__restrict__ g,
                                                  const unsigned short *__restrict__ x,
                                                  float *__restrict__ dW) {
    __shared__ float red[9][4];
    const int c = blockIdx.x, o = blockIdx.y;
    const int P = Ny * Nx;
    float acc[9];
#pragma unroll
    for (int d = 0; d < 9; ++d) acc[d] = 0.f;
    for (int i = threadIdx.x; i < batch * P; i += blockDim.x) {
        const int b = i / P, p = i % P;
        const float gv = g[((size_t)b * Cout + o) * P + p];
        if (gv == 0.f) continue;
        const int py = p / Nx, px = p % Nx;
        const unsigned short *xb = x + ((size_t)b * Cin + c) * P;
#pragma unroll
        for (int d = 0; d < 9; ++d) {
            int yy = py + d / 3 - 1, xx = px + d % 3 - 1;
            yy += (yy < 0) ? Ny : 0; yy -= (yy >= Ny) ? Ny : 0;
            xx += (xx < 0) ? Nx : 0; xx -= (xx >= Nx) ? Nx : 0;
            acc[d] += gv * bf2f(xb[yy * Nx + xx]);
        }
    }
#pragma unroll
    for (int d = 0; d < 9; ++d) {
        const float v = wave_sum(acc[d]);
        if ((threadIdx.x & 63) == 0) red[d][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 9) {
        const int d = threadIdx.x;
        dW[((size_t)o * Cin + c) * 9 + d] = red[d][0] + red[d][1] + red[d][2] + red[d][3];
    }
}

__global__ void conv_bgrad(int batch, int Cout, int P, const float *__restrict__ g, float *__restrict__ db) {
    __shared__ float red[16];
    const int o = blockIdx.x;
    float s = 0.f;
    for (int i = threadIdx.x; i < batch * P; i += blockDim.x) {
        const int b = i / P, p = i % P;
        s += g[((size_t)b * Cout + o) * P + p];
    }
    s = block_sum(s, red);
    if (threadIdx.x == 0) db[o] = s;
}

__global__ void adam_kernel(int64_t np, float *__restrict__ p, const float *__restrict__ g,
                            float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2,
                            float eps, float c1, float c2) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np;
         i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// start fields of the SCF from the network output of one sample:
// U = Vext + y[0], |Delta| = max(y[1], 0)
__global__ void start_fields_kernel(int64_t P, const float *__restrict__ y, const double *__restrict__ Vext,
                                   double *__restrict__ U, double *__restrict__ D) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < P; p += (int64_t)gridDim.x * blockDim.x) {
        U[p] = Vext[p] + (double)y[p];
        D[p] = fmax((double)y[P + p], 0.0);
    }
}

unsigned blocks_for(int64_t total) {
    int64_t g = (total + 255) / 256;
    return (unsigned)(g > 2048 ? 2048 : (g < 1 ? 1 : g));
}

}  // namespace

NetLayout net_layout(const bdg_net_shape *sh, bool forward_only) {
    NetLayout L;
    const int C = sh->channels;
    const int64_t P = (int64_t)sh->ny * sh->nx;
    const int64_t B = sh->batch;
    const int cin[4] = {3, C, C, C}, cout[4] = {C, C, C, 2};
    int64_t off = 0;
    for (int l = 0; l < 4; ++l) {
        L.w_off[l] = off;
        off += (int64_t)cout[l] * cin[l] * 9;
        L.b_off[l] = off;
        off += cout[l];
        L.cin[l] = cin[l];
        L.cout[l] = cout[l];
    }
    L.nparams = off;
    size_t o = 0;
    auto put = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
    for (int l = 0; l < 4; ++l) L.wk[l] = put(2 * (size_t)cout[l] * cin[l] * 9);
    for (int l = 0; l < 4; ++l) L.act[l] = put(2 * (size_t)B * cin[l] * P);  // inputs of layer l (bf16)
    if (forward_only) {
        // what a forward pass into a caller-given output touches: the BF16
        // weights and the layer inputs; the backward buffers are left out
        for (int l = 0; l < 4; ++l) L.wt[l] = 0;
        L.y = L.g32 = L.gbf = L.gx32 = L.part = 0;
        L.total = o;
        return L;
    }
    for (int l = 0; l < 4; ++l) L.wt[l] = put(2 * (size_t)cout[l] * cin[l] * 9);
    L.y = put(4 * (size_t)B * 2 * P);
    L.g32 = put(4 * (size_t)B * C * P);
    L.gbf = put(2 * (size_t)B * C * P);
    L.gx32 = put(4 * (size_t)B * C * P);
    L.part = put(4 * 4096);
    L.total = o;
    return L;
}

int net_forward(const bdg_net_shape *sh, const float *params, const double *Vext, const double *theta,
                double mu, float *y_out, void *work, hipStream_t s) {
    // with a caller-given output only the forward part of the layout is used;
    // its offsets are the same in both layouts
    const NetLayout L = net_layout(sh, y_out != nullptr);
    char *w = (char *)work;
    const int64_t P = (int64_t)sh->ny * sh->nx;
    const int B = sh->batch;
    for (int l = 0; l < 4; ++l) {
        hipLaunchKernelGGL(weights_bf16, dim3(blocks_for((int64_t)L.cout[l] * L.cin[l] * 9)), dim3(256), 0, s,
                           L.cin[l], L.cout[l], params + L.w_off[l], (unsigned short *)(w + L.wk[l]),
                           (unsigned short *)nullptr);
    }
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for(B * P)), dim3(256), 0, s, B, (int)P, Vext, theta, mu,
                       (unsigned short *)(w + L.act[0]));
    for (int l = 0; l < 4; ++l) {
        const bool last = (l == 3);
        hipLaunchKernelGGL(conv_mfma, dim3((unsigned)((P + 63) / 64), B), dim3(256), 0, s, L.cin[l], L.cout[l],
                           sh->ny, sh->nx, (const unsigned short *)(w + L.act[l]),
                           (const unsigned short *)(w + L.wk[l]), params + L.b_off[l], last ? 0 : 1,
                           last ? (unsigned short *)nullptr : (unsigned short *)(w + L.act[l + 1]),
                           last ? (y_out ? y_out : (float *)(w + L.y)) : (float *)nullptr);
    }
    BDG_CHECK_LAUNCH();
    return 0;
}

int net_backward(const bdg_net_shape *sh, const float *params, const double *Vext, const double *theta,
                 double mu, const float *target, float *grads, float *loss, void *work, hipStream_t s) {
    const NetLayout L = net_layout(sh);
    char *w = (char *)work;
    const int64_t P = (int64_t)sh->ny * sh->nx;
    const int B = sh->batch;
    float *y = (float *)(w + L.y);
    BDG_TRY(net_forward(sh, params, Vext, theta, mu, y, work, s));
    for (int l = 0; l < 4; ++l)
        hipLaunchKernelGGL(weights_bf16, dim3(blocks_for((int64_t)L.cout[l] * L.cin[l] * 9)), dim3(256), 0, s,
                           L.cin[l], L.cout[l], params + L.w_off[l], (unsigned short *)(w + L.wk[l]),
                           (unsigned short *)(w + L.wt[l]));
    float *g32 = (float *)(w + L.g32);
    unsigned short *gbf = (unsigned short *)(w + L.gbf);
    float *gx32 = (float *)(w + L.gx32);
    float *part = (float *)(w + L.part);
    const int total = B * 2 * (int)P;
    const unsigned nb = blocks_for(total) > 1024 ? 1024 : blocks_for(total);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, s, total, y, target, g32, gbf, part);
    hipLaunchKernelGGL(sum_partials, dim3(1), dim3(1024), 0, s, (int)nb, part, 1.f / (float)total, loss);
    for (int l = 3; l >= 0; --l) {
        // gradient of layer l's output is in g32/gbf (B x cout[l] x P)
        hipLaunchKernelGGL(conv_wgrad, dim3(L.cin[l], L.cout[l]), dim3(256), 0, s, B, L.cin[l], L.cout[l],
                           sh->ny, sh->nx, g32, (const unsigned short *)(w + L.act[l]),
                           grads + L.w_off[l]);
        hipLaunchKernelGGL(conv_bgrad, dim3(L.cout[l]), dim3(256), 0, s, B, L.cout[l], (int)P, g32,
                           grads + L.b_off[l]);
        if (l == 0) break;
        // data gradient through the conv, then through the relu of layer l-1
        hipLaunchKernelGGL(conv_mfma, dim3((unsigned)((P + 63) / 64), B), dim3(256), 0, s, L.cout[l], L.cin[l],
                           sh->ny, sh->nx, gbf, (const unsigned short *)(w + L.wt[l]), (const float *)nullptr,
                           0, (unsigned short *)nullptr, gx32);
        hipLaunchKernelGGL(relu_back, dim3(blocks_for((int64_t)B * L.cin[l] * P)), dim3(256), 0, s,
                           (int)(B * L.cin[l] * P), gx32, (const unsigned short *)(w + L.act[l]), g32, gbf);
    }
    BDG_CHECK_LAUNCH();
    return 0;
}

int net_start_fields(const bdg_net_shape *sh, const float *y, int sample, const double *Vext, double *U, double *D,
                     hipStream_t s) {
    const int64_t P = (int64_t)sh->ny * sh->nx;
    hipLaunchKernelGGL(start_fields_kernel, dim3(blocks_for(P)), dim3(256), 0, s, P, y + (int64_t)sample * 2 * P, Vext,
                       U, D);
    BDG_CHECK_LAUNCH();
    return 0;
}

int net_adam(int64_t np, float *params, const float *grads, float *m, float *v, int t, float lr,
             hipStream_t s) {
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3(blocks_for(np)), dim3(256), 0, s, np, params, grads, m, v, lr, b1, b2,
                       eps, c1, c2);
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace bdg

namespace bdg {

// ---------------------------------------------------------------------------
// Forward pass without a caller workspace, for callers that cannot allocate
// device memory (code under stream capture, tight inference loops).  The
// scratch is one file-scope device array per GPU, held until the process
// ends; every call on a GPU reuses it, so calls that overlap on one GPU race.
// A forward pass writes every scratch byte it later reads (BF16 weights, then
// each layer's input), so nothing has to be cleared between calls.
namespace {

constexpr size_t NET_SCRATCH_BYTES = size_t(32) << 20;  // 32 MiB
__device__ __align__(256) unsigned char net_scratch[NET_SCRATCH_BYTES];

constexpr int NET_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NET_MAX_DEVICES] = {};

// Device address of this GPU's scratch array (the host-side name of a
// __device__ variable is not a device address; the runtime resolves the
// address once per device, with that device current).
int scratch_for_current_device(void **out) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice", __FILE__, __LINE__);
    if (dev < 0 || dev >= NET_MAX_DEVICES) {
        set_error("net_forward_noalloc: device %d beyond the %d supported", dev, NET_MAX_DEVICES);
        return BDG_ERR_NOT_IMPLEMENTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(net_scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(net_scratch)", __FILE__, __LINE__);
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

}  // namespace

size_t net_scratch_capacity() { return NET_SCRATCH_BYTES; }

int net_forward_noalloc(const bdg_net_shape *sh, const float *params, const double *Vext, const double *theta,
                        double mu, float *y_out, hipStream_t s) {
    const size_t need = net_layout(sh, true).total;
    if (need > NET_SCRATCH_BYTES) {
        set_error("bdg_net_forward_noalloc: the shape needs %zu scratch bytes, more than the %zu available "
                  "(use bdg_net_forward with a workspace)", need, NET_SCRATCH_BYTES);
        return BDG_ERR_WORKSPACE;
    }
    void *scratch = nullptr;
    BDG_TRY(scratch_for_current_device(&scratch));
    return net_forward(sh, params, Vext, theta, mu, y_out, scratch, s);
}

}  // namespace bdg
