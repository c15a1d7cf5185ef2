// One step of the static SLDA self-consistency on the GPU ("Methods" of the
// paper; the iteration that the multigrid runs repeat "through a series of
// diagonalizations", sec. "Performance of the Matrix Diagonalization
// Algorithm").
//
//   Delta(r) = |Delta(r)| exp(i theta(r))          (fixed phase, only |Delta| iterates)
//   H        = BdG matrix of (U, Delta, mu)         (bdg_assemble)
//   (E, Z)   = eigenpairs with 0 < E < Ec           (bdg_eigh, window)
//   n(r)     = 2 sum |v_n(r)|^2,  nu(r) = sum u_n(r) v_n(r)^*   (T = 0, eq. densities2)
//   U'       = Vext + B eps_F(n),  |Delta|' = g |nu|
//   U, |Delta| <- (1 - alpha) old + alpha new;  change = max(|U' - U|, ||Delta|' - |Delta||)
//
// The density sums read Z once (HBM bound, 16 n m bytes); every sum runs on
// the device, the host only receives the change norm and the window count.
#include <math.h>

#include "solver.h"

namespace bdg {
namespace {

constexpr int JSPLIT = 32;

__global__ void delta_from_phase(int64_t ns, const double *__restrict__ absD,
                                 const double *__restrict__ theta, double *__restrict__ D) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * blockDim.x) {
        double sn, cs;
        sincos(theta[r], &sn, &cs);
        D[2 * r] = absD[r] * cs;
        D[2 * r + 1] = absD[r] * sn;
    }
}

// partial sums over a slice of the columns: part[s][r] = (n, nu.re, nu.im)
__global__ void density_partials(int64_t ns, int64_t m, const double *__restrict__ Z, int64_t ldz,
                                 double *__restrict__ part) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    if (r >= ns) return;
    const int64_t per = (m + JSPLIT - 1) / JSPLIT;
    const int64_t j0 = sl * per, j1 = min(m, j0 + per);
    double nn = 0.0, vr = 0.0, vi = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double2 u = *(const double2 *)(Z + 2 * (r + j * ldz));
        const double2 v = *(const double2 *)(Z + 2 * (ns + r + j * ldz));
        nn += v.x * v.x + v.y * v.y;
        vr += u.x * v.x + u.y * v.y;  // u conj(v)
        vi += u.y * v.x - u.x * v.y;
    }
    double *p = part + 3 * (sl * ns + r);
    p[0] = nn;
    p[1] = vr;
    p[2] = vi;
}

__device__ inline double fermi_energy(double n, int ndim) {
    n = fmax(n, 0.0);
    if (ndim == 2) return M_PI * n;
    if (ndim == 3) return 0.5 * cbrt(3.0 * M_PI * M_PI * n) * cbrt(3.0 * M_PI * M_PI * n);
    const double kf = 0.5 * M_PI * n;
    return 0.5 * kf * kf;
}

__global__ void scf_update(int64_t ns, int ndim, const double *__restrict__ part,
                           const double *__restrict__ Vext, bdg_scf_params p, double *__restrict__ U,
                           double *__restrict__ absD, double *__restrict__ dens,
                           double *__restrict__ nuabs, double *__restrict__ chg) {
    __shared__ double red[16];
    double mx = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < ns;
         r += (int64_t)gridDim.x * blockDim.x) {
        double nn = 0.0, vr = 0.0, vi = 0.0;
        for (int s = 0; s < JSPLIT; ++s) {
            const double *q = part + 3 * (s * ns + r);
            nn += q[0];
            vr += q[1];
            vi += q[2];
        }
        nn *= 2.0;
        const double na = sqrt(vr * vr + vi * vi);
        const double Un = Vext[r] + p.B * fermi_energy(nn, ndim);
        const double Dn = p.g * na;
        mx = fmax(mx, fmax(fabs(Un - U[r]), fabs(Dn - absD[r])));
        U[r] = (1.0 - p.alpha) * U[r] + p.alpha * Un;
        absD[r] = (1.0 - p.alpha) * absD[r] + p.alpha * Dn;
        if (dens) dens[r] = nn;
        if (nuabs) nuabs[r] = na;
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) v = fmax(v, red[i]);
        chg[blockIdx.x] = v;
    }
}

size_t al(size_t x) { return (x + 255) / 256 * 256; }

struct ScfLayout {
    size_t H, eig, W, Z, D, part, chg, total;
    size_t eig_bytes;
};

ScfLayout scf_layout(int64_t ns) {
    const int64_t n = 2 * ns;
    ScfLayout L;
    size_t o = 0;
    size_t eb = 0;
    eigh_workspace(n, nullptr, &eb);
    L.eig_bytes = eb;
    L.H = o; o += al(16 * (size_t)n * n);
    L.eig = o; o += al(eb);
    L.W = o; o += al(8 * (size_t)n);
    L.Z = o; o += al(16 * (size_t)n * n);
    L.D = o; o += al(16 * (size_t)ns);
    L.part = o; o += al(24 * (size_t)ns * JSPLIT);
    L.chg = o; o += al(8 * 1024);
    L.total = o;
    return L;
}

}  // namespace

size_t scf_workspace(const bdg_lattice *lat) {
    int64_t ns = 1;
    for (int d = 0; d < lat->ndim; ++d) ns *= lat->dims[d];
    return scf_layout(ns).total;
}

int scf_step(const bdg_lattice *lat, const double *Vext, const double *theta, double mu,
             const bdg_scf_params *p, double *U, double *absDelta, double *density, double *nu_abs,
             double *change, int64_t *m_out, void *work, hipStream_t s) {
    int64_t ns = 1;
    for (int d = 0; d < lat->ndim; ++d) ns *= lat->dims[d];
    const int64_t n = 2 * ns;
    const ScfLayout L = scf_layout(ns);
    char *base = (char *)work;
    double *H = (double *)(base + L.H);
    void *ew = base + L.eig;
    double *W = (double *)(base + L.W);
    double *Z = (double *)(base + L.Z);
    double *D = (double *)(base + L.D);
    double *part = (double *)(base + L.part);
    double *chg = (double *)(base + L.chg);
    const unsigned gs = (unsigned)((ns + 255) / 256 > 1024 ? 1024 : (ns + 255) / 256);
    hipLaunchKernelGGL(delta_from_phase, dim3(gs), dim3(256), 0, s, ns, absDelta, theta, D);
    BDG_CHECK_LAUNCH();
    BDG_TRY(assemble(lat, U, D, mu, H, n, s));
    int64_t m = 0;
    // window 0 < E < Ec: the smallest positive double excludes E = 0 exactly
    BDG_TRY(eigh(n, H, n, 4.9406564584124654e-324, p->Ec, W, Z, n, n, &m, nullptr, ew,
                 L.eig_bytes, nullptr, s));
    *m_out = m;
    if (m > 0) {
        hipLaunchKernelGGL(density_partials, dim3((unsigned)((ns + 255) / 256), JSPLIT), dim3(256), 0, s,
                           ns, m, Z, n, part);
        BDG_CHECK_LAUNCH();
    } else {
        BDG_HIP(hipMemsetAsync(part, 0, 24 * (size_t)ns * JSPLIT, s));
    }
    hipLaunchKernelGGL(scf_update, dim3(gs), dim3(256), 0, s, ns, lat->ndim, part, Vext, *p, U, absDelta,
                       density, nu_abs, chg);
    BDG_CHECK_LAUNCH();
    double hc[1024];
    BDG_HIP(hipMemcpyAsync(hc, chg, 8 * (size_t)gs, hipMemcpyDeviceToHost, s));
    BDG_HIP(hipStreamSynchronize(s));
    double c = 0.0;
    for (unsigned i = 0; i < gs; ++i) c = c > hc[i] ? c : hc[i];
    *change = c;
    return 0;
}

}  // namespace bdg
