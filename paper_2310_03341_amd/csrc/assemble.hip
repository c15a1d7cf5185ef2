// Dense BdG matrix assembly (eq. stHpsi with the block form of eq. TDSLDA).
//
// h(r, r') = sum_d t_d(x_d - x'_d) prod_{e != d} delta(x_e, x'_e) + (U(r) - mu) delta(r, r'),
// where t_N(m) is the matrix of F^-1 (k^2/2) F on the periodic grid with
// momenta k = 2 pi n / N, n = -N/2 .. N/2-1 ("Numerical setup and
// implementation").  For even N that operator has the closed form
//   t(0) = pi^2 (N^2 + 2) / (6 N^2),  t(m) = (-1)^m pi^2 / (N^2 sin^2(pi m / N)),
// (the periodic spectral second-derivative matrix, halved, at unit spacing).
// H = [[h, diag Delta], [diag conj(Delta), -conj(h)]]; h is real here.
//
// The kernel is bound by the 16 n^2 bytes it writes: one workgroup per column
// j, threads stride down the rows so that stores are coalesced.
#include "common.h"

#include <math.h>

namespace bdg {
namespace {

__global__ __launch_bounds__(256) void assemble_kernel(int ndim, int Nx, int Ny, int Nz,
                                                       const double *__restrict__ U,
                                                       const double *__restrict__ Delta, double mu,
                                                       double *__restrict__ H, int64_t ldh) {
    __shared__ double tab[3][64];
    for (int d = 0; d < 3; ++d) {
        const int Nd = d == 0 ? Nx : (d == 1 ? Ny : Nz);
        for (int m = threadIdx.x; m < Nd; m += blockDim.x) {
            double v;
            const double pn = M_PI / (double)Nd;
            if (m == 0) {
                v = M_PI * M_PI * ((double)Nd * Nd + 2.0) / (6.0 * (double)Nd * Nd);
            } else {
                const double sn = sin(pn * (double)m);
                v = ((m & 1) ? -1.0 : 1.0) * pn * pn / (sn * sn);
            }
            tab[d][m] = (d < ndim) ? v : 0.0;
        }
    }
    __syncthreads();
    const double *tx = tab[0], *ty = tab[1], *tz = tab[2];
    const int64_t ns = (int64_t)Nx * Ny * Nz;
    const int64_t n = 2 * ns;
    const int64_t j = blockIdx.x;
    const int64_t sj = j < ns ? j : j - ns;
    const bool jv = j >= ns;
    const int xj = (int)(sj % Nx), yj = (int)((sj / Nx) % Ny), zj = (int)(sj / ((int64_t)Nx * Ny));
    double2 *col = (double2 *)(H + 2 * j * ldh);
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const bool iv = i >= ns;
        const int64_t si = iv ? i - ns : i;
        double re = 0.0, im = 0.0;
        if (iv == jv) {
            const int xi = (int)(si % Nx), yi = (int)((si / Nx) % Ny), zi = (int)(si / ((int64_t)Nx * Ny));
            double h = 0.0;
            if (yi == yj && zi == zj) {
                int dm = xi - xj;
                if (dm < 0) dm = -dm;
                h += tx[dm];
            }
            if (ndim > 1 && xi == xj && zi == zj) {
                int dm = yi - yj;
                if (dm < 0) dm = -dm;
                h += ty[dm];
            }
            if (ndim > 2 && xi == xj && yi == yj) {
                int dm = zi - zj;
                if (dm < 0) dm = -dm;
                h += tz[dm];
            }
            if (si == sj) h += U[si] - mu;
            re = iv ? -h : h;
        } else if (si == sj) {
            re = Delta[2 * si];
            im = iv ? -Delta[2 * si + 1] : Delta[2 * si + 1];  // lower-left: conj(Delta)
        }
        col[i] = make_double2(re, im);
    }
}

}  // namespace

int assemble(const bdg_lattice *lat, const double *U, const double *Delta, double mu, double *H,
             int64_t ldh, hipStream_t s) {
    int N[3] = {1, 1, 1};
    for (int d = 0; d < lat->ndim; ++d) N[d] = lat->dims[d];
    const int64_t ns = (int64_t)N[0] * N[1] * N[2];
    const int64_t n = 2 * ns;
    hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)n), dim3(256), 0, s, lat->ndim, N[0], N[1],
                       N[2], U, Delta, mu, H, ldh);
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace bdg
