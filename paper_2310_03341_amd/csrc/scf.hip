// One step of the static SLDA self-consistency on the GPU ("Methods" of the
// paper; the iteration that the multigrid runs repeat "through a series of
// diagonalizations", sec. "Performance of the Matrix Diagonalization
// Algorithm").
//
//   Delta(r) = |Delta(r)| exp(i theta(r))          (fixed phase, only |Delta| iterates)
//   H        = BdG matrix of (U, Delta, mu)         (bdg_assemble)
//   (E, Z)   = eigenpairs with 0 < E < Ec           (bdg_eigh, window)
//   n(r)     = 2 sum (|v_n|^2 f_T(-E_n) + |u_n|^2 f_T(E_n)),
//   nu(r)    = sum u_n v_n^* (f_T(-E_n) - f_T(E_n))      (eq. densities2, f_T = 1/(1 + e^{E/T}))
//   U'       = Vext + B eps_F(n),  |Delta|' = g_eff |nu|,
//   g_eff    = g, or 1/(1/g + Lambda_c(r)) with the cut-off regularisation (3-D):
//              Lambda_c = (k_c - (k_0/2) ln((k_c+k_0)/(k_c-k_0))) / 2 pi^2,
//              k_c^2/2 = Ec + mu - U(r), k_0^2/2 = mu - U(r)   ("Density functional
//              theory for superfluid fermions"; for mu < U the pole-free form
//              (k_c - kappa atan(k_c/kappa)) / 2 pi^2, kappa^2 = -k_0^2)
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

// f_T(E) = 1 / (1 + exp(E/T)); T = 0: the step (1/2 at E = 0)
__device__ inline double fermi_fn(double E, double T) {
    if (T == 0.0) return E < 0.0 ? 1.0 : (E > 0.0 ? 0.0 : 0.5);
    const double x = E / T;
    const double q = exp(-fabs(x));  // never overflows
    return x > 0.0 ? q / (1.0 + q) : 1.0 / (1.0 + q);
}

// occupation weights of the window states: occ[2j] = f_T(-E_j), occ[2j+1] = f_T(E_j)
__global__ void occupations(int64_t m, const double *__restrict__ W, double T, double *__restrict__ occ) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += (int64_t)gridDim.x * blockDim.x) {
        occ[2 * j] = fermi_fn(-W[j], T);
        occ[2 * j + 1] = fermi_fn(W[j], T);
    }
}

// partial sums over a slice of the columns: part[s][r] = (n/2, nu.re, nu.im)
__global__ void density_partials(int64_t ns, int64_t m, const double *__restrict__ Z, int64_t ldz,
                                 const double *__restrict__ occ, double *__restrict__ part) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int sl = blockIdx.y;
    if (r >= ns) return;
    const int64_t per = (m + JSPLIT - 1) / JSPLIT;
    const int64_t j0 = sl * per, j1 = min(m, j0 + per);
    double nn = 0.0, vr = 0.0, vi = 0.0;
    for (int64_t j = j0; j < j1; ++j) {
        const double2 u = *(const double2 *)(Z + 2 * (r + j * ldz));
        const double2 v = *(const double2 *)(Z + 2 * (ns + r + j * ldz));
        const double fp = occ[2 * j], fm = occ[2 * j + 1], fd = fp - fm;
        nn += (v.x * v.x + v.y * v.y) * fp + (u.x * u.x + u.y * u.y) * fm;
        vr += (u.x * v.x + u.y * v.y) * fd;  // u conj(v)
        vi += (u.y * v.x - u.x * v.y) * fd;
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

// Lambda_c of the cut-off regularisation (3-D, hbar = m = 1) from k_c^2, k_0^2
__device__ inline double lambda_c(double kc2, double k02) {
    if (kc2 <= 0.0) return 0.0;  // no state below the cut-off
    const double kc = sqrt(kc2);
    double v;
    if (k02 > 0.0) {
        const double k0 = sqrt(k02);
        v = kc - 0.5 * k0 * log((kc + k0) / (kc - k0));
    } else if (k02 < 0.0) {
        const double ka = sqrt(-k02);
        v = kc - ka * atan(kc / ka);
    } else {
        v = kc;
    }
    return v / (2.0 * M_PI * M_PI);
}

__global__ void scf_update(int64_t ns, int ndim, const double *__restrict__ part,
                           const double *__restrict__ Vext, double mu, bdg_scf_params p, double *__restrict__ U,
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
        const double geff =
            p.regularize ? 1.0 / (1.0 / p.g + lambda_c(2.0 * (p.Ec + mu - U[r]), 2.0 * (mu - U[r]))) : p.g;
        const double Dn = geff * na;
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
    size_t H, eig, W, Z, D, part, occ, chg, total;
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
    L.occ = o; o += al(16 * (size_t)n);
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
    double *occ = (double *)(base + L.occ);
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
        hipLaunchKernelGGL(occupations, dim3((unsigned)((m + 255) / 256 > 1024 ? 1024 : (m + 255) / 256)),
                           dim3(256), 0, s, m, W, p->T, occ);
        hipLaunchKernelGGL(density_partials, dim3((unsigned)((ns + 255) / 256), JSPLIT), dim3(256), 0, s,
                           ns, m, Z, n, occ, part);
        BDG_CHECK_LAUNCH();
    } else {
        BDG_HIP(hipMemsetAsync(part, 0, 24 * (size_t)ns * JSPLIT, s));
    }
    hipLaunchKernelGGL(scf_update, dim3(gs), dim3(256), 0, s, ns, lat->ndim, part, Vext, mu, *p, U, absDelta,
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

// ---------------------------------------------------------------------------
// Moving fields between the levels of the multigrid start ("Performance of the
// Matrix Diagonalization Algorithm": coarser lattices start the finer ones).
//
// To a finer lattice: trigonometric interpolation of the periodic samples,
// separable over the axes.  Along an axis with N_c coarse and N_f fine sites,
// fine site x sits at xi = x N_c / N_f coarse spacings, and with h = N_c / 2
// and the Nyquist coefficient split evenly between -h and +h
//   P(xi, j) = (1/N_c) (1 + 2 sum_{k=1}^{h-1} cos(k t) + cos(h t)),  t = 2 pi (xi - j) / N_c
//            = (1/N_c) (sin((h - 1/2) t) / sin(t / 2) + cos(h t))      (Dirichlet kernel),
// and P = 1 (0) where xi falls on coarse site j (another coarse site).
// To a coarser lattice (each fine size a multiple s of the coarse one):
// injection, g(x) = f(s x).  Either way the result is multiplied by `scale`.
__device__ inline double interp_weight(int64_t xf, int Nf, int j, int Nc) {
    // xi - j = (xf Nc - j Nf) / Nf exactly in integers
    const int64_t num = xf * (int64_t)Nc - (int64_t)j * Nf;
    if (num % Nf == 0) return (num / Nf) % Nc == 0 ? 1.0 : 0.0;
    const int h = Nc / 2;
    const double t = 2.0 * M_PI * ((double)num / (double)Nf) / (double)Nc;
    return (sin((h - 0.5) * t) / sin(0.5 * t) + cos(h * t)) / (double)Nc;
}

__global__ void interp_kernel(int nd, int cx, int cy, int cz, int fx, int fy, int fz,
                              const double *__restrict__ f, double scale, double *__restrict__ g) {
    const int64_t nf = (int64_t)fx * fy * fz;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nf;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(r % fx), y = (int)((r / fx) % fy), z = (int)(r / ((int64_t)fx * fy));
        double acc = 0.0;
        for (int k = 0; k < cz; ++k) {
            const double wz = nd > 2 ? interp_weight(z, fz, k, cz) : 1.0;
            if (wz == 0.0) continue;
            double accy = 0.0;
            for (int j = 0; j < cy; ++j) {
                const double wy = nd > 1 ? interp_weight(y, fy, j, cy) : 1.0;
                if (wy == 0.0) continue;
                const double *row = f + ((int64_t)k * cy + j) * cx;
                double accx = 0.0;
                for (int i = 0; i < cx; ++i) accx += interp_weight(x, fx, i, cx) * row[i];
                accy += wy * accx;
            }
            acc += wz * accy;
        }
        g[r] = scale * acc;
    }
}

__global__ void inject_kernel(int cx, int cy, int cz, int sx, int sy, int sz, int fx, int fy,
                              const double *__restrict__ f, double scale, double *__restrict__ g) {
    const int64_t nc = (int64_t)cx * cy * cz;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < nc;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int x = (int)(r % cx), y = (int)((r / cx) % cy), z = (int)(r / ((int64_t)cx * cy));
        g[r] = scale * f[(int64_t)x * sx + (int64_t)fx * ((int64_t)y * sy + (int64_t)fy * z * sz)];
    }
}

int regrid(const bdg_lattice *src, const double *f, const bdg_lattice *dst, double *g, double scale,
           hipStream_t s) {
    int sd[3] = {1, 1, 1}, dd[3] = {1, 1, 1};
    for (int d = 0; d < src->ndim; ++d) {
        sd[d] = src->dims[d];
        dd[d] = dst->dims[d];
    }
    bool finer = true, coarser = true;
    for (int d = 0; d < 3; ++d) {
        finer &= dd[d] >= sd[d];
        coarser &= dd[d] <= sd[d] && sd[d] % dd[d] == 0;
    }
    int64_t nd = (int64_t)dd[0] * dd[1] * dd[2];
    const unsigned gs = (unsigned)((nd + 255) / 256 > 2048 ? 2048 : (nd + 255) / 256);
    if (finer) {
        hipLaunchKernelGGL(interp_kernel, dim3(gs), dim3(256), 0, s, src->ndim, sd[0], sd[1], sd[2], dd[0], dd[1],
                           dd[2], f, scale, g);
    } else if (coarser) {
        hipLaunchKernelGGL(inject_kernel, dim3(gs), dim3(256), 0, s, dd[0], dd[1], dd[2], sd[0] / dd[0],
                           sd[1] / dd[1], sd[2] / dd[2], sd[0], sd[1], f, scale, g);
    } else {
        set_error("bdg_regrid: the target lattice must be finer along every axis, or coarser by an integer "
                  "factor along every axis");
        return -3;
    }
    BDG_CHECK_LAUNCH();
    return 0;
}

}  // namespace bdg
