// Time evolution of the quasiparticle wavefunctions, eq. (TDSLDA):
//   i d/dt phi_j = H(t) phi_j,  H = [[h, Delta], [Delta^*, -h^*]],  h = -nabla^2/2 + U - mu,
// with the mean fields recomputed from the evolved states at every evaluation
// (zero-temperature occupations of the time-dependent runs, eq. densities2):
//   n = 2 sum_j |v_j|^2,  nu = sum_j u_j v_j^*,  U = Vext + B eps_F(n),  Delta = g nu,
// or held at given (U0, Delta0) when the evolution is not self-consistent.
//
// Integrator (sec. "Performance of the Time Evolution Algorithm"): fifth-order
// Adams-Bashforth-Moulton predictor-corrector with two evaluations of H per
// step, f = -i H[phi] phi, f_k = f(phi_k):
//   phi*      = phi_k + dt (1901 f_k - 2774 f_{k-1} + 2616 f_{k-2} - 1274 f_{k-3} + 251 f_{k-4}) / 720
//   phi_{k+1} = phi_k + dt (251 f(phi*) + 646 f_k - 264 f_{k-1} + 106 f_{k-2} - 19 f_{k-3}) / 720
// The first four steps (history not yet filled) take classical RK4.
//
// Kernels, all bound by HBM traffic of the n x m state arrays:
//  * td_combine: out = sum_i c_i X_i over up to eight state arrays, with the
//    density partials of `out` summed in the same pass (one read of every
//    input, one write);
//  * td_fields: the partials -> n, nu -> U, Delta on the lattice;
//  * td_apply: F = -i H X, one workgroup per state: the state's u and v sit in
//    LDS (up to 4096 sites, 128 KB), the kinetic term is the periodic spectral
//    second derivative, a circulant matrix along each axis, applied on 2 x 2
//    site blocks so that every LDS value read feeds two outputs.  The paper
//    applies the same operator with FFTs; on lattices of at most 64 points
//    per axis the circulant product is as cheap and needs no transposes.
// A step moves 18 state arrays through HBM (predictor 6 in / 1 out, two
// evaluations 1 in / 1 out each, corrector 6 in / 1 out).
#include <math.h>
#include <stdlib.h>

#include "solver.h"

namespace bdg {
namespace {

constexpr int TD_JSPLIT = 32;
constexpr int TD_MAXK = 8;

struct Comb {
    const double *X[TD_MAXK];
    int64_t ld[TD_MAXK];
    double c[TD_MAXK];
    int K;
};

// out[:, j] = sum_i c_i X_i[:, j] for the m states (rows u then v, complex);
// part[s][r] = (sum |v|^2, re sum u v^*, im sum u v^*) of `out` over slice s of
// the states.  out may be one of the inputs (each entry is read before it is
// written by the same thread); out == nullptr computes the partials only of X_0.
__global__ __launch_bounds__(256) void td_combine(int64_t ns, int64_t m, Comb cb, double *out, int64_t ldo,
                                                  double *__restrict__ part) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    if (r >= ns) return;
    const int64_t per = (m + TD_JSPLIT - 1) / TD_JSPLIT;
    const int64_t j0 = sl * per, j1 = min(m, j0 + per);
    double nn = 0.0, vr = 0.0, vi = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        double ur = 0.0, ui = 0.0, wr = 0.0, wi = 0.0;
        for (int i = 0; i < cb.K; ++i) {
            const double2 a = *(const double2 *)(cb.X[i] + 2 * (r + j * cb.ld[i]));
            const double2 b = *(const double2 *)(cb.X[i] + 2 * (ns + r + j * cb.ld[i]));
            ur += cb.c[i] * a.x;
            ui += cb.c[i] * a.y;
            wr += cb.c[i] * b.x;
            wi += cb.c[i] * b.y;
        }
        if (out) {
            *(double2 *)(out + 2 * (r + j * ldo)) = make_double2(ur, ui);
            *(double2 *)(out + 2 * (ns + r + j * ldo)) = make_double2(wr, wi);
        }
        nn += wr * wr + wi * wi;
        vr += ur * wr + ui * wi;  // u conj(v)
        vi += ui * wr - ur * wi;
    }
    if (part) {
        double *q = part + 3 * (sl * ns + r);
        q[0] = nn;
        q[1] = vr;
        q[2] = vi;
    }
}

__device__ inline double td_fermi_energy(double n, int ndim) {
    n = fmax(n, 0.0);
    if (ndim == 2) return M_PI * n;
    if (ndim == 3) return 0.5 * cbrt(3.0 * M_PI * M_PI * n) * cbrt(3.0 * M_PI * M_PI * n);
    const double kf = 0.5 * M_PI * n;
    return 0.5 * kf * kf;
}

// U = Vext + B eps_F(n), Delta = g nu from the partial sums
__global__ void td_fields(int64_t ns, int ndim, const double *__restrict__ part, const double *__restrict__ Vext,
                          double B, double g, double *__restrict__ U, double *__restrict__ D) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * blockDim.x) {
        double nn = 0.0, vr = 0.0, vi = 0.0;
        for (int s = 0; s < TD_JSPLIT; ++s) {
            const double *q = part + 3 * (s * ns + r);
            nn += q[0];
            vr += q[1];
            vi += q[2];
        }
        U[r] = Vext[r] + B * td_fermi_energy(2.0 * nn, ndim);
        D[2 * r] = g * vr;
        D[2 * r + 1] = g * vi;
    }
}

// F[:, j] = -i H X[:, j]; one workgroup per state, u and v of the state in LDS.
// Sites are taken in BY x 2 blocks (y, x): BY = 2 on 2-D and 3-D lattices, 1
// on a 1-D one (a compile-time constant, so the accumulators stay in
// registers).  Circulant coefficients t(x - k) are walked down the table as k
// goes up (t(-1) = t(N - 1)).
template <int MAXS, int BY, int NT>
__global__ __launch_bounds__(NT) void td_apply(int ndim, int Nx, int Ny, int Nz, const double *__restrict__ X,
                                               int64_t ldx, const double *__restrict__ U,
                                               const double *__restrict__ D, double mu, double *__restrict__ F,
                                               int64_t ldf) {
    __shared__ double2 sh[2 * MAXS];  // u: [0, ns), v: [ns, 2 ns); the launcher checks ns <= MAXS
    __shared__ double tab[3][64];
    const int ns = Nx * Ny * Nz;
    const int64_t j = blockIdx.x;
    for (int d = 0; d < 3; ++d) {
        const int Nd = d == 0 ? Nx : (d == 1 ? Ny : Nz);
        for (int k = threadIdx.x; k < Nd; k += blockDim.x) {
            double v;
            const double pn = M_PI / (double)Nd;
            if (k == 0) {
                v = M_PI * M_PI * ((double)Nd * Nd + 2.0) / (6.0 * (double)Nd * Nd);
            } else {
                const double sn = sin(pn * (double)k);
                v = ((k & 1) ? -1.0 : 1.0) * pn * pn / (sn * sn);
            }
            tab[d][k] = (d < ndim) ? v : 0.0;
        }
    }
    const double2 *col = (const double2 *)(X + 2 * j * ldx);
    // fixed trip count (2 ns <= 2 MAXS): every load is issued before the first store
#pragma unroll
    for (int it = 0; it < 2 * MAXS / NT; ++it) {
        const int i = threadIdx.x + it * NT;
        if (i < 2 * ns) sh[i] = col[i];
    }
    __syncthreads();
    const int bx = Nx / 2, by = Ny / BY;
    const int nb = bx * by * Nz;
    double2 *fcol = (double2 *)(F + 2 * j * ldf);
    for (int b = threadIdx.x; b < nb; b += NT) {
        const int x0 = 2 * (b % bx);
        const int y0 = BY * ((b / bx) % by);
        const int z = b / (bx * by);
        double ar[2][BY][2], ai[2][BY][2];  // [component u/v][yy][xx]
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int yy = 0; yy < BY; ++yy)
#pragma unroll
                for (int xx = 0; xx < 2; ++xx) ar[c][yy][xx] = ai[c][yy][xx] = 0.0;
#pragma unroll
        for (int c = 0; c < 2; ++c) {
            const double2 *s = sh + c * ns;
            // along x: out(x0 + xx, y0 + yy) += t(x0 + xx - k) s(k, y0 + yy)
            {
                const double2 *line = s + Nx * (y0 + Ny * z);
                int d0 = x0;  // (x0 - k) mod Nx at k = 0
                for (int k = 0; k < Nx; ++k) {
                    const int d1 = d0 + 1 == Nx ? 0 : d0 + 1;
                    const double t0 = tab[0][d0], t1 = tab[0][d1];
#pragma unroll
                    for (int yy = 0; yy < BY; ++yy) {
                        const double2 a = line[k + Nx * yy];
                        ar[c][yy][0] += t0 * a.x;
                        ai[c][yy][0] += t0 * a.y;
                        ar[c][yy][1] += t1 * a.x;
                        ai[c][yy][1] += t1 * a.y;
                    }
                    d0 = d0 == 0 ? Nx - 1 : d0 - 1;
                }
            }
            if (BY == 2) {
                // along y: out(x0 + xx, y0 + yy) += t(y0 + yy - k) s(x0 + xx, k)
                const double2 *plane = s + Nx * Ny * z + x0;
                int d0 = y0;
                for (int k = 0; k < Ny; ++k) {
                    const int d1 = d0 + 1 == Ny ? 0 : d0 + 1;
                    const double t0 = tab[1][d0], t1 = tab[1][d1];
                    const double2 a0 = plane[Nx * k], a1 = plane[Nx * k + 1];
                    ar[c][0][0] += t0 * a0.x;
                    ai[c][0][0] += t0 * a0.y;
                    ar[c][0][1] += t0 * a1.x;
                    ai[c][0][1] += t0 * a1.y;
                    ar[c][BY - 1][0] += t1 * a0.x;
                    ai[c][BY - 1][0] += t1 * a0.y;
                    ar[c][BY - 1][1] += t1 * a1.x;
                    ai[c][BY - 1][1] += t1 * a1.y;
                    d0 = d0 == 0 ? Ny - 1 : d0 - 1;
                }
            }
            if (ndim > 2) {
                // along z: out(x, y, z) += t(z - k) s(x, y, k)
                const double2 *colz = s + x0 + Nx * y0;
                int d0 = z;
                for (int k = 0; k < Nz; ++k) {
                    const double t0 = tab[2][d0];
#pragma unroll
                    for (int yy = 0; yy < BY; ++yy) {
                        const double2 a0 = colz[Nx * (yy + Ny * k)], a1 = colz[Nx * (yy + Ny * k) + 1];
                        ar[c][yy][0] += t0 * a0.x;
                        ai[c][yy][0] += t0 * a0.y;
                        ar[c][yy][1] += t0 * a1.x;
                        ai[c][yy][1] += t0 * a1.y;
                    }
                    d0 = d0 == 0 ? Nz - 1 : d0 - 1;
                }
            }
        }
#pragma unroll
        for (int yy = 0; yy < BY; ++yy) {
#pragma unroll
            for (int xx = 0; xx < 2; ++xx) {
                const int r = x0 + xx + Nx * (y0 + yy + Ny * z);
                const double2 u = sh[r], v = sh[ns + r];
                const double w = U[r] - mu;
                const double2 dl = *(const double2 *)(D + 2 * r);
                // top = T u + (U - mu) u + Delta v;  bottom = Delta^* u - T v - (U - mu) v
                const double tr = ar[0][yy][xx] + w * u.x + (dl.x * v.x - dl.y * v.y);
                const double ti = ai[0][yy][xx] + w * u.y + (dl.x * v.y + dl.y * v.x);
                const double br = (dl.x * u.x + dl.y * u.y) - ar[1][yy][xx] - w * v.x;
                const double bi = (dl.x * u.y - dl.y * u.x) - ai[1][yy][xx] - w * v.y;
                // f = -i (a + i b) = b - i a
                fcol[r] = make_double2(ti, -tr);
                fcol[ns + r] = make_double2(bi, -br);
            }
        }
    }
}

// The same F = -i H X with the kinetic term on the matrix cores, for 2-D
// lattices whose sides are multiples of 16 and the 16 x 16 x 16 lattice.  The
// circulant product along x and along y of one z plane is a 16 x 16 tile
// product: D[x][y] = sum_x' t(x - x') s[x'][y] + sum_y' s[x][y'] t(y - y'),
// i.e. T_x S and S T_y with T symmetric (v_mfma_f64_16x16x4, real tables,
// real and imaginary parts of s as two products).  Along z the tile is
// oriented [z][x] for one y: D[z][x] = sum_z' t(z - z') s[x][y][z'].  One
// component (u, then v) at a time sits in LDS with the x stride padded by
// one element (the tile operands then hit distinct banks); the x and y terms
// go to an LDS result buffer, the z term is added into it, and the epilogue
// adds the local terms with the other component read from global memory.
// 1024 threads: the per-state chain of loads, products and stores is latency
// bound, and more waves shorten it (0.31 ms per application at 16^3 against
// 0.36 ms with 512 threads and 0.35 ms for the general kernel).
constexpr int TD_MFMA_LDS = 4352;  // padded sites: (Nx + 1) Ny Nz <= 4352
constexpr int TD_MFMA_NT = 1024;
__global__ __launch_bounds__(TD_MFMA_NT) void td_apply_mfma(int ndim, int Nx, int Ny, int Nz,
                                                            const double *__restrict__ X, int64_t ldx,
                                                            const double *__restrict__ U,
                                                            const double *__restrict__ D, double mu,
                                                            double *__restrict__ F, int64_t ldf) {
    constexpr int NTH = TD_MFMA_NT, NW = NTH / 64;
    __shared__ double2 S[TD_MFMA_LDS];
    __shared__ double2 O[TD_MFMA_LDS];
    __shared__ double tab[3][64];
    const int ns = Nx * Ny * Nz;
    const int px = Nx + 1, pxy = (Nx + 1) * Ny;  // padded strides
    const int64_t j = blockIdx.x;
    for (int d = 0; d < 3; ++d) {
        const int Nd = d == 0 ? Nx : (d == 1 ? Ny : Nz);
        for (int k = threadIdx.x; k < Nd; k += blockDim.x) {
            double v;
            const double pn = M_PI / (double)Nd;
            if (k == 0) {
                v = M_PI * M_PI * ((double)Nd * Nd + 2.0) / (6.0 * (double)Nd * Nd);
            } else {
                const double sn = sin(pn * (double)k);
                v = ((k & 1) ? -1.0 : 1.0) * pn * pn / (sn * sn);
            }
            tab[d][k] = (d < ndim) ? v : 0.0;
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int lr = lane & 15, lk = lane >> 4;
    const double2 *col = (const double2 *)(X + 2 * j * ldx);
    double2 *fcol = (double2 *)(F + 2 * j * ldf);
    const int txb = Nx / 16, tyb = Ny / 16;
    for (int c = 0; c < 2; ++c) {
        // fixed trip count (ns <= 4096): every load is issued before the first store
#pragma unroll
        for (int it = 0; it < 4096 / NTH; ++it) {
            const int r = threadIdx.x + it * NTH;
            if (r < ns) {
                const int x = r % Nx, y = (r / Nx) % Ny, z = r / (Nx * Ny);
                S[x + px * y + pxy * z] = col[c * ns + r];
            }
        }
        __syncthreads();
        // x and y terms, tiles [x][y] of one plane z
        const int nA = txb * tyb * Nz;
        for (int tile = wv; tile < nA; tile += NW) {
            const int bx = tile % txb, by = (tile / txb) % tyb, z = tile / (txb * tyb);
            d4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
            const int xo = bx * 16 + lr, yo = by * 16 + lr;
            for (int k0 = 0; k0 < Nx; k0 += 4) {
                const int xp = k0 + lk;
                const int dd = xo - xp < 0 ? xo - xp + Nx : xo - xp;
                const double a = tab[0][dd];
                const double2 b = S[xp + px * yo + pxy * z];
                ar = mfma16(a, b.x, ar);
                ai = mfma16(a, b.y, ai);
            }
            for (int k0 = 0; k0 < Ny; k0 += 4) {
                const int yp = k0 + lk;
                const int dd = yo - yp < 0 ? yo - yp + Ny : yo - yp;
                const double bt = tab[1][dd];
                const double2 a = S[xo + px * yp + pxy * z];
                ar = mfma16(a.x, bt, ar);
                ai = mfma16(a.y, bt, ai);
            }
#pragma unroll
            for (int q = 0; q < 4; ++q) O[(bx * 16 + lk + 4 * q) + px * yo + pxy * z] = make_double2(ar[q], ai[q]);
        }
        if (ndim == 3) {
            __syncthreads();
            // z term, tiles [z][x] of one y (Nz == 16)
            const int nB = Ny * txb;
            for (int tile = wv; tile < nB; tile += NW) {
                const int bx = tile % txb, y = tile / txb;
                d4 ar = {0, 0, 0, 0}, ai = {0, 0, 0, 0};
                const int xo = bx * 16 + lr;
                for (int k0 = 0; k0 < Nz; k0 += 4) {
                    const int zp = k0 + lk;
                    const int dd = lr - zp < 0 ? lr - zp + Nz : lr - zp;
                    const double a = tab[2][dd];
                    const double2 b = S[xo + px * y + pxy * zp];
                    ar = mfma16(a, b.x, ar);
                    ai = mfma16(a, b.y, ai);
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    double2 &o = O[xo + px * y + pxy * (lk + 4 * q)];
                    o.x += ar[q];
                    o.y += ai[q];
                }
            }
        }
        __syncthreads();
#pragma unroll
        for (int it = 0; it < 4096 / NTH; ++it) {
            const int r = threadIdx.x + it * NTH;
            if (r >= ns) break;
            const int x = r % Nx, y = (r / Nx) % Ny, z = r / (Nx * Ny);
            const int li = x + px * y + pxy * z;
            const double2 kin = O[li], self = S[li], other = col[(1 - c) * ns + r];
            const double w = U[r] - mu;
            const double2 dl = *(const double2 *)(D + 2 * r);
            if (c == 0) {
                // top = T u + (U - mu) u + Delta v;  f = -i top
                const double tr = kin.x + w * self.x + (dl.x * other.x - dl.y * other.y);
                const double ti = kin.y + w * self.y + (dl.x * other.y + dl.y * other.x);
                fcol[r] = make_double2(ti, -tr);
            } else {
                // bottom = Delta^* u - T v - (U - mu) v
                const double br = (dl.x * other.x + dl.y * other.y) - kin.x - w * self.x;
                const double bi = (dl.x * other.y - dl.y * other.x) - kin.y - w * self.y;
                fcol[ns + r] = make_double2(bi, -br);
            }
        }
        __syncthreads();
    }
}

// Resume state kept at the head of the workspace: [count of valid history
// entries, ring position of f_k].
__global__ void td_set_header(int64_t *hdr, int64_t count, int64_t head) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        hdr[0] = count;
        hdr[1] = head;
    }
}

struct TdLayout {
    size_t hdr, arr[8], part, U, D, total;
};

TdLayout td_layout(int64_t ns, int64_t m) {
    TdLayout L;
    const size_t sa = 16 * (size_t)(2 * ns) * (size_t)m;
    size_t o = 0;
    auto put = [&](size_t bytes) { size_t r = o; o += (bytes + 255) / 256 * 256; return r; };
    L.hdr = put(64);
    for (int i = 0; i < 8; ++i) L.arr[i] = put(sa);
    L.part = put(24 * (size_t)ns * TD_JSPLIT);
    L.U = put(8 * (size_t)ns);
    L.D = put(16 * (size_t)ns);
    L.total = o;
    return L;
}

}  // namespace

size_t td_workspace(const bdg_lattice *lat, int64_t m) {
    int64_t ns = 1;
    for (int d = 0; d < lat->ndim; ++d) ns *= lat->dims[d];
    return td_layout(ns, m).total;
}

int64_t td_max_sites() { return 4096; }

int td_evolve(const bdg_lattice *lat, const double *Vext, double mu, const bdg_td_params *p, int64_t m,
              double *Phi, int64_t ldphi, double dt, int64_t nsteps, const double *U0, const double *D0,
              void *work, hipStream_t s) {
    int dims[3] = {1, 1, 1};
    int64_t ns = 1;
    for (int d = 0; d < lat->ndim; ++d) {
        dims[d] = lat->dims[d];
        ns *= dims[d];
    }
    const int64_t n = 2 * ns;
    const TdLayout L = td_layout(ns, m);
    char *base = (char *)work;
    int64_t *hdr = (int64_t *)(base + L.hdr);
    double *A[8];
    for (int i = 0; i < 8; ++i) A[i] = (double *)(base + L.arr[i]);
    double *hist[5] = {A[0], A[1], A[2], A[3], A[4]};
    double *tmp = A[5], *kb = A[6], *acc = A[7];
    double *part = (double *)(base + L.part);
    double *Uw = (double *)(base + L.U);
    double *Dw = (double *)(base + L.D);
    const bool sc = p->self_consistent != 0;
    const double *Uf = sc ? Uw : U0;
    const double *Df = sc ? Dw : D0;
    const dim3 cgrid((unsigned)((ns + 255) / 256), TD_JSPLIT);
    const unsigned fgrid = (unsigned)((ns + 255) / 256 > 1024 ? 1024 : (ns + 255) / 256);

    // out = sum c_i X_i (+ partials, + fields when self-consistent)
    auto combine = [&](int K, const double *const *X, const int64_t *ld, const double *c, double *out, int64_t ldo,
                       bool fields) -> int {
        Comb cb;
        cb.K = K;
        for (int i = 0; i < TD_MAXK; ++i) {
            cb.X[i] = i < K ? X[i] : nullptr;
            cb.ld[i] = i < K ? ld[i] : 0;
            cb.c[i] = i < K ? c[i] : 0.0;
        }
        const bool dens = fields && sc;
        hipLaunchKernelGGL(td_combine, cgrid, dim3(256), 0, s, ns, m, cb, out, ldo, dens ? part : (double *)nullptr);
        if (dens)
            hipLaunchKernelGGL(td_fields, dim3(fgrid), dim3(256), 0, s, ns, lat->ndim, part, Vext, p->B, p->g, Uw,
                               Dw);
        BDG_CHECK_LAUNCH();
        return 0;
    };
    // the matrix-core kinetic term: 2-D sides that are multiples of 16, or 16^3
    static const bool mfma_env = [] {
        const char *v = getenv("BDG_TD_MFMA");
        return !(v && v[0] == '0');
    }();
    const bool mfma_ok = mfma_env && ((lat->ndim == 2 && dims[0] % 16 == 0 && dims[1] % 16 == 0 &&
                                       (dims[0] + 1) * dims[1] <= TD_MFMA_LDS) ||
                                      (lat->ndim == 3 && dims[0] == 16 && dims[1] == 16 && dims[2] == 16));
    auto apply = [&](const double *X, int64_t ldx, double *Fo) -> int {
#define BDG_TD_APPLY(MS, BYV, NTV)                                                                       \
    hipLaunchKernelGGL((td_apply<MS, BYV, NTV>), dim3((unsigned)m), dim3(NTV), 0, s, lat->ndim, dims[0], dims[1], \
                       dims[2], X, ldx, Uf, Df, mu, Fo, n)
        // matrix-core form where the lattice allows it; otherwise LDS sized
        // for the lattice, 1024 threads (16 waves) hiding the LDS latency
        // when one state fills the CU's LDS
        if (mfma_ok) {
            hipLaunchKernelGGL(td_apply_mfma, dim3((unsigned)m), dim3(TD_MFMA_NT), 0, s, lat->ndim, dims[0], dims[1],
                               dims[2], X, ldx, Uf, Df, mu, Fo, n);
        } else if (lat->ndim == 1) {
            if (ns <= 1024) BDG_TD_APPLY(1024, 1, 256);
            else BDG_TD_APPLY(4096, 1, 1024);
        } else {
            if (ns <= 1024) BDG_TD_APPLY(1024, 2, 256);
            else BDG_TD_APPLY(4096, 2, 1024);
        }
#undef BDG_TD_APPLY
        BDG_CHECK_LAUNCH();
        return 0;
    };

    int64_t count = 0, head = 0;  // valid history entries, ring slot of f_k
    if (p->resume) {
        int64_t h[2];
        BDG_HIP(hipMemcpyAsync(h, hdr, sizeof(h), hipMemcpyDeviceToHost, s));
        BDG_HIP(hipStreamSynchronize(s));
        count = h[0];
        head = h[1];
        if (count < 1 || count > 5 || head < 0 || head > 4) {
            set_error("bdg_td_evolve: resume requested but the workspace holds no history");
            return BDG_ERR_WORKSPACE;
        }
    }
    auto slot = [&](int back) { return hist[((head - back) % 5 + 5) % 5]; };  // f_{k - back}
    if (count == 0) {
        // f_0 = f(phi_0), with the fields of phi_0 when they follow the states
        if (sc) {
            const double *X[1] = {Phi};
            const int64_t ld[1] = {ldphi};
            const double c[1] = {1.0};
            BDG_TRY(combine(1, X, ld, c, nullptr, 0, true));
        }
        head = 0;
        BDG_TRY(apply(Phi, ldphi, hist[0]));
        count = 1;
    }
    for (int64_t step = 0; step < nsteps; ++step) {
        const double *f0 = slot(0);
        if (count < 5) {
            // classical RK4: k1 = f_k;  acc = k1 + 2 k2 + 2 k3 (+ k4 folded into the update)
            {
                const double *X[2] = {Phi, f0};
                const int64_t ld[2] = {ldphi, n};
                const double c[2] = {1.0, 0.5 * dt};
                BDG_TRY(combine(2, X, ld, c, tmp, n, true));
                BDG_TRY(apply(tmp, n, kb));  // k2
            }
            {
                const double *X[2] = {f0, kb};
                const int64_t ld[2] = {n, n};
                const double c[2] = {1.0, 2.0};
                BDG_TRY(combine(2, X, ld, c, acc, n, false));
            }
            {
                const double *X[2] = {Phi, kb};
                const int64_t ld[2] = {ldphi, n};
                const double c[2] = {1.0, 0.5 * dt};
                BDG_TRY(combine(2, X, ld, c, tmp, n, true));
                BDG_TRY(apply(tmp, n, kb));  // k3
            }
            {
                const double *X[2] = {acc, kb};
                const int64_t ld[2] = {n, n};
                const double c[2] = {1.0, 2.0};
                BDG_TRY(combine(2, X, ld, c, acc, n, false));
            }
            {
                const double *X[2] = {Phi, kb};
                const int64_t ld[2] = {ldphi, n};
                const double c[2] = {1.0, dt};
                BDG_TRY(combine(2, X, ld, c, tmp, n, true));
                BDG_TRY(apply(tmp, n, kb));  // k4
            }
            {
                const double *X[3] = {Phi, acc, kb};
                const int64_t ld[3] = {ldphi, n, n};
                const double c[3] = {1.0, dt / 6.0, dt / 6.0};
                BDG_TRY(combine(3, X, ld, c, Phi, ldphi, true));
            }
        } else {
            // predictor, evaluation, corrector
            static const double ab[5] = {1901.0 / 720.0, -2774.0 / 720.0, 2616.0 / 720.0, -1274.0 / 720.0,
                                         251.0 / 720.0};
            static const double am[5] = {251.0 / 720.0, 646.0 / 720.0, -264.0 / 720.0, 106.0 / 720.0,
                                         -19.0 / 720.0};
            {
                const double *X[6] = {Phi, slot(0), slot(1), slot(2), slot(3), slot(4)};
                const int64_t ld[6] = {ldphi, n, n, n, n, n};
                double c[6] = {1.0};
                for (int i = 0; i < 5; ++i) c[i + 1] = dt * ab[i];
                BDG_TRY(combine(6, X, ld, c, tmp, n, true));
                BDG_TRY(apply(tmp, n, kb));  // f(phi*)
            }
            {
                const double *X[6] = {Phi, kb, slot(0), slot(1), slot(2), slot(3)};
                const int64_t ld[6] = {ldphi, n, n, n, n, n};
                double c[6] = {1.0};
                for (int i = 0; i < 5; ++i) c[i + 1] = dt * am[i];
                BDG_TRY(combine(6, X, ld, c, Phi, ldphi, true));
            }
        }
        // f_{k+1} = f(phi_{k+1}) into the ring (over f_{k-4} once the ring is full)
        head = (head + 1) % 5;
        BDG_TRY(apply(Phi, ldphi, hist[head]));
        if (count < 5) ++count;
    }
    hipLaunchKernelGGL(td_set_header, dim3(1), dim3(64), 0, s, hdr, count, head);
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace bdg
