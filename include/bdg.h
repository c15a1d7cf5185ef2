/*
 * bdg.h -- C-ABI of the MI355X (gfx950) dense BdG eigensolver library.
 *
 * The library diagonalises the quasiparticle Hamiltonian of the static
 * SLDA/BdG problem (Wlazlowski et al., arXiv:2310.03341, eq. stHpsi with the
 * block form of eq. TDSLDA):
 *
 *     H = [[ h, Delta ], [ Delta^*, -h^* ]],   h = -(1/2) nabla^2 + U(r) - mu,
 *
 * on a periodic Nx x Ny x Nz grid with unit spacing and hbar = m = 1, the
 * kinetic term being the spectral operator F^-1 (k^2/2) F over the momenta
 * k = 2 pi n / N, n = -N/2 .. N/2-1 ("Numerical setup and implementation").
 * The matrix has order n = 2 Nx Ny Nz; a quasiparticle wavefunction is the
 * vector [u; v] with the site index r = x + Nx (y + Ny z) (x fastest).
 *
 * The eigensolver is the two-stage direct method that the paper's ELPA runs
 * use ("Performance of the Matrix Diagonalization Algorithm"): dense ->
 * Hermitian band (blocked Householder), band -> real tridiagonal (bulge
 * chasing), tridiagonal divide and conquer, and the two back-transformations
 * of the eigenvectors.  Only eigenpairs inside a closed energy window
 * [emin, emax] are returned (the densities of eq. densities2 sum over the
 * window 0 < E_n < E_c with E_c = pi^2/2, "Methods").
 *
 * Conventions for every entry point:
 *   - All array arguments are DEVICE pointers owned by the caller; the library
 *     never frees them and never keeps them after the call returns.
 *   - Complex arrays are complex128 (or complex64 where stated) interleaved
 *     (re, im); matrices are column-major with a leading dimension >= rows.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = legacy default
 *     stream) and is asynchronous unless stated otherwise.
 *   - Return value: BDG_OK (0) or a status below; a negative value -i means
 *     argument i (1-based) is invalid.  bdg_last_error() gives a message.
 *   - Thread-compatible: concurrent calls need distinct streams and distinct
 *     workspaces.
 */
#ifndef BDG_H
#define BDG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes. */
#define BDG_OK 0
#define BDG_ERR_NOCONV 1          /* secular-equation / iteration failure       */
#define BDG_ERR_REFINE_TOL 2      /* refinement missed refine_tol (result valid) */
#define BDG_ERR_HIP 3             /* HIP runtime error                          */
#define BDG_ERR_WORKSPACE 4       /* workspace or output capacity too small     */
#define BDG_ERR_NOT_IMPLEMENTED 5 /* option not supported                       */
#define BDG_ERR_NONFINITE 6       /* NaN/Inf found in the input matrix          */

typedef void *bdg_stream_t; /* hipStream_t */

/* Periodic lattice; dims[d] for d < ndim, unit spacing, x fastest. */
typedef struct {
    int32_t ndim;    /* 1, 2 or 3 */
    int32_t dims[3]; /* each even and >= 2 */
} bdg_lattice;

/* Arithmetic of the reduction stages. */
#define BDG_FP64 0         /* all stages in FP64                                  */
#define BDG_FP32_REFINED 1 /* band reduction + back-transforms in FP32 on MFMA,
                              tridiagonal solve in FP64, then FP64 refinement     */

typedef struct {
    int32_t precision;       /* BDG_FP64 or BDG_FP32_REFINED                     */
    int32_t band;            /* half-bandwidth of stage 1 (0 = default 64)      */
    int32_t refine_max_iter; /* refinement steps for BDG_FP32_REFINED (0 = 4;
                                < 0 = none: the FP32 result widened to FP64)    */
    double refine_tol;       /* stop once the step's defect (max |r_ij| and
                                |s_ij + lam_j r_ij| / ||H||_2 off the diagonal,
                                in-cluster coupling / ||H||_2) is below this
                                (0 = 1e-14); BDG_ERR_REFINE_TOL when the last
                                defect still exceeds sqrt(refine_tol)           */
    int32_t dc_leaf;         /* divide-and-conquer leaf size (0 = default 32)   */
    int32_t ph_mirror;       /* 1: back-transform only E >= 0 vectors and build
                                the E < 0 ones as (-v^*, u^*) (particle-hole
                                symmetry of a BdG matrix with real h and local
                                Delta); 0: back-transform every vector          */
    int64_t max_pairs;       /* BDG_FP32_REFINED: most eigenpairs the window can
                                hold (0 = n).  The refinement buffers are sized
                                for it (plus max_pairs/64 + 64 columns for the
                                guard band around the window), so a window of a
                                few tenths of the spectrum needs far less
                                workspace than n.  Ignored by BDG_FP64.          */
} bdg_opts;

/* Progress: when the environment variable BDG_VERBOSE is set (and not "0"),
 * bdg_eigh waits for each stage and prints one line per finished stage and
 * per refinement step to stderr.  Off by default (no extra synchronisation). */
/* Look-ahead: stage 1 factors the next panel on a second stream of the library
 * while the trailing update runs on the caller's stream.  When the environment
 * variable BDG_NO_LOOKAHEAD is set (and not "0"), every panel is factored on
 * the caller's stream instead (same results; for tools that serialise
 * dispatches, such as hardware-counter profilers). */
/* Divide and conquer (bdg_eigh, bdg_stage_stedc): the merges of one level of
 * the merge tree run on four non-blocking streams the library creates once
 * per device (default priority, kept until the process ends), ordered against
 * the caller's stream by events.  The stage synchronises the caller's stream
 * once per tree level to read the merge sizes back to the host, and returns
 * only after all its work has been ordered before later work on `stream`. */

/* Per-call accuracy and timing report (filled when non-NULL). */
typedef struct {
    double max_resid;     /* mixed arm: defect measured by the last refinement
                             step (see refine_tol)                                */
    double gram_defect;   /* max_ij |(Z^H Z - I)_ij|              (when checked) */
    double eig_shift_max; /* largest eigenvalue change made by refinement        */
    int32_t refine_iters; /* refinement sweeps performed                         */
    int32_t pad;
    double stage_ms[8];   /* he2hb, hb2st, stedc, bt2, bt1, refine, select, total */
    double bt2_kernel_ms; /* duration of the back-transformation-2 apply kernel     */
    int32_t refine_close_pairs;  /* mixed arm: close window pairs, first step  */
    int32_t refine_cluster_cols; /* mixed arm: clustered columns, first step    */
} bdg_err_report;

/*
 * bdg_assemble -- dense BdG matrix H of eq. (stHpsi) on the lattice `lat`.
 *   U     [nsites] real potential U(r) (device, f64).
 *   Delta [nsites] complex pairing field Delta(r) (device, complex128).
 *   mu    chemical potential (enters h as -mu, "Methods", mean-field h).
 *   H     [ldh x n] output (device, complex128), n = 2*nsites; both triangles
 *         are written.  ldh >= n.
 * The kinetic block uses the closed form of F^-1 (k^2/2) F on the paper's
 * momentum grid; the v-block is -conj(h) and the off-diagonal blocks are
 * diag(Delta) (upper right) and diag(conj Delta) (lower left).
 */
int bdg_assemble(const bdg_lattice *lat, const double *U, const double *Delta, double mu,
                 double *H, int64_t ldh, bdg_stream_t stream);

/*
 * bdg_eigh_workspace -- device workspace (bytes) that bdg_eigh needs for order n.
 */
int bdg_eigh_workspace(int64_t n, const bdg_opts *opts, size_t *bytes);

/*
 * bdg_eigh -- eigenpairs of the Hermitian matrix A with eigenvalues in the
 * closed window [emin, emax] (use -INFINITY/INFINITY for the full spectrum).
 *   n         order of A (>= 1).
 *   A         [lda x n] complex128 Hermitian; only the lower triangle is read.
 *             DESTROYED (holds the stage-1 reflectors on exit).
 *   W         [n] f64 output; W[0..m) are the selected eigenvalues, ascending.
 *             W[m..n) is scratch.
 *   Z         [ldz x zcols] complex128 output; Z[:, 0..m) the eigenvectors.
 *   zcols     column capacity of Z; if m > zcols, BDG_ERR_WORKSPACE is
 *             returned and *m holds the count.
 *   m         output: number of eigenpairs in the window (host pointer).
 *   opts      options (NULL = defaults, FP64).
 *   work      device workspace of work_bytes >= bdg_eigh_workspace(n, opts).
 *   report    optional host pointer for accuracy/timing information.
 * Host synchronisation: the call returns only after its work on `stream` has
 * finished.  On the way it waits for `stream` to read back the NaN/Inf flag,
 * after uploading the stage-2 reflector offsets, once per level of the
 * divide-and-conquer merge tree (merge sizes) and to read the eigenvalues
 * that decide the window; the mixed arm also once per refinement step.
 * Returns BDG_ERR_NONFINITE (and does not modify W, Z) if A holds NaN/Inf.
 *
 * BDG_FP32_REFINED: A is only read (kept intact; the FP64 refinement needs
 * it).  The window is cut on the REFINED eigenvalues: every eigenvalue of the
 * FP32 stages within 1e-4 ||H||_2 of [emin, emax] is refined, then the window
 * is taken; *m counts the refined eigenvalues inside it.  If more pairs need
 * refining than opts.max_pairs allows, BDG_ERR_WORKSPACE is returned and *m
 * holds that count.
 */
int bdg_eigh(int64_t n, double *A, int64_t lda, double emin, double emax, double *W,
             double *Z, int64_t ldz, int64_t zcols, int64_t *m, const bdg_opts *opts,
             void *work, size_t work_bytes, bdg_err_report *report, bdg_stream_t stream);

/*
 * bdg_eigh1_workspace -- device workspace (bytes) of bdg_eigh1 for order n,
 * element type `real` (1 = real symmetric, 0 = complex Hermitian) and zcols
 * columns of Z.
 */
int bdg_eigh1_workspace(int64_t n, int32_t real, int64_t zcols, size_t *bytes);

/*
 * bdg_eigh1 -- one-stage FP64 eigensolver: blocked Householder reduction of
 * the dense matrix straight to real tridiagonal form (panels of 64 columns,
 * delayed two-sided updates; the trailing matrix is read once per column by a
 * Hermitian matrix-vector product, the memory-bound half of the work), the
 * same tridiagonal divide and conquer as bdg_eigh, and one back-
 * transformation in compact-WY blocks.  This is the solver family the paper
 * benchmarks (ELPA one-stage, real symmetric; complex Hermitian "about twice
 * as long", sec. "Performance of the Matrix Diagonalization Algorithm"), next
 * to the two-stage bdg_eigh.
 *   real   1: A and Z hold real f64 (symmetric A); 0: complex128 (Hermitian).
 *   A      [lda x n], lower triangle read; DESTROYED (the reflectors).
 *   W, Z, zcols, m   as for bdg_eigh (window [emin, emax], ascending).
 *   report optional: stage_ms[0] tridiagonalisation, [2] divide and
 *          conquer, [4] back-transformation, [6] window, [7] total.
 * Synchronises `stream` to read the eigenvalues that decide the window and
 * returns after all its work has finished.  No particle-hole mirror, no
 * mixed precision.
 */
int bdg_eigh1(int64_t n, int32_t real, double *A, int64_t lda, double emin, double emax, double *W,
              double *Z, int64_t ldz, int64_t zcols, int64_t *m, void *work, size_t work_bytes,
              bdg_err_report *report, bdg_stream_t stream);

/*
 * bdg_refine_workspace -- device workspace (bytes) of bdg_refine for order n
 * and m refined columns.
 */
int bdg_refine_workspace(int64_t n, int64_t m, size_t *bytes);

/*
 * bdg_refine -- FP64 refinement of the eigenpairs in columns [i0, i0 + m) of
 * an approximate eigenbasis X of the Hermitian H (the precision extension of
 * the method: Ogita & Aishima, "Iterative refinement for symmetric eigenvalue
 * decomposition", Japan J. Indust. Appl. Math. 35 (2018), complex Hermitian
 * form, with a Rayleigh-Ritz step inside groups of close eigenvalues as in
 * their part II on clustered eigenvalues, 2019).  One step, for the window
 * columns W against the whole basis:
 *     R = I[:, W] - X^H X_W,  S = X^H H X_W   (window rows Hermitian-symmetrised)
 *     lam_j = s_jj / (1 - r_jj),
 *     E_ij = (s_ij + lam_j r_ij) / (lam_j - lam_i), or r_ij / 2 for close pairs,
 *     X_W <- X_W + X E.
 * A pair is close when |s_ij + lam_j r_ij| >= 1e-3 |lam_j - lam_i|; connected
 * groups of close window pairs (cut into pieces of at most 48) get the
 * Rayleigh-Ritz step.  Steps repeat until the defect (max |r_ij| and
 * |s_ij + lam_j r_ij| / ||H||_2 off the diagonal, in-cluster coupling /
 * ||H||_2) drops below opts.refine_tol or opts.refine_max_iter steps are done.
 *   n      order of H (>= 1).
 *   H      [ldh x n] complex128 Hermitian, lower triangle read, not modified.
 *   lam    [n] f64 approximate eigenvalues of ALL columns of X (device); they
 *          stand in for the Rayleigh quotients of the columns outside the
 *          window.  max |lam| is taken as ||H||_2.
 *   X      [ldx x n] complex128 approximate eigenvectors, all n of them
 *          (refining a subset needs the whole basis: the error of a window
 *          column along the other eigenvectors is corrected from them);
 *          columns i0 .. i0+m-1 are refined in place, the others are read.
 *   i0, m  the refined columns, 0 <= i0, i0 + m <= n.
 *   W      [m] f64 output: W[k] is the refined eigenvalue of column i0 + k.
 *          The column order is kept (two columns of a pair closer than the
 *          basis error may converge swapped: sort W if order matters).
 *   opts   refine_max_iter (0 = 4, < 0 invalid), refine_tol (0 = 1e-14); the
 *          other fields are ignored.  NULL = defaults.
 *   work   device workspace of work_bytes >= bdg_refine_workspace(n, m).
 *   report optional host pointer: refine_iters, max_resid (last defect),
 *          eig_shift_max (largest change of an eigenvalue in the first step),
 *          refine_close_pairs / refine_cluster_cols (first step),
 *          stage_ms[5] = stage_ms[7] = elapsed time.
 * Synchronises `stream` once per step (close pairs and the defect are read
 * back).  Returns BDG_ERR_REFINE_TOL when the last defect still exceeds
 * sqrt(refine_tol) (X and W hold the refined result all the same).
 */
int bdg_refine(int64_t n, const double *H, int64_t ldh, const double *lam, double *X, int64_t ldx,
               int64_t i0, int64_t m, double *W, const bdg_opts *opts, void *work, size_t work_bytes,
               bdg_err_report *report, bdg_stream_t stream);

/*
 * Constants of one self-consistency step (the SLDA loop of "Methods").
 *   U' = Vext + B eps_F(n)   (eps_F = pi n in 2D, (3 pi^2 n)^(2/3)/2 in 3D),
 *   |Delta|' = g_eff |nu|    (pairing field Delta = g_eff nu, phase held fixed),
 *   U, |Delta| <- (1 - alpha) old + alpha new,  states with 0 < E < Ec,
 * with the densities of eq. (densities2) at temperature T (Fermi function
 * f_T(E) = 1/(1 + exp(E/T)); T = 0 is the ground state):
 *   n = 2 sum (|v|^2 f_T(-E) + |u|^2 f_T(E)),  nu = sum u v^* (f_T(-E) - f_T(E)).
 * g_eff = g, or with regularize = 1 (3-D lattices only) the cut-off
 * regularisation of "Density functional theory for superfluid fermions":
 * g is then the finite coupling and g_eff(r) = 1 / (1/g + Lambda_c(r)),
 *   Lambda_c = (k_c - (k_0/2) ln((k_c + k_0)/(k_c - k_0))) / (2 pi^2),
 *   k_c^2 / 2 = Ec + mu - U(r),  k_0^2 / 2 = mu - U(r)
 * (the principal-value integral of 1/(k^2 - k_0^2) over |k| < k_c; for
 * mu < U(r) its pole-free form (k_c - kappa atan(k_c/kappa)) / (2 pi^2),
 * kappa^2 = -k_0^2; zero where k_c^2 <= 0).
 */
typedef struct {
    double B;     /* coefficient of the density term of U               */
    double g;     /* pairing coupling (the finite one with regularize)   */
    double alpha; /* linear mixing weight                               */
    double Ec;    /* energy cutoff (pi^2/2 = k_max^2/2 on the unit grid) */
    double T;     /* temperature (>= 0)                                  */
    int32_t regularize; /* 1: cut-off regularisation of g (3-D only)    */
    int32_t pad;
} bdg_scf_params;

/* bdg_scf_workspace -- device workspace (bytes) of bdg_scf_step for `lat`. */
int bdg_scf_workspace(const bdg_lattice *lat, size_t *bytes);

/*
 * bdg_scf_step -- one zero-temperature SLDA self-consistency step on the GPU:
 * assemble H(U, |Delta| e^{i theta}, mu), diagonalise with the window
 * 0 < E < Ec, form n(r) = 2 sum |v_n|^2 and nu(r) = sum u_n v_n^* (eq.
 * densities2 at T = 0), update and mix U and |Delta|.
 *   Vext, theta [nsites] f64 device (external potential, fixed pairing phase).
 *   U, absDelta [nsites] f64 device, in/out.
 *   density, nu_abs [nsites] f64 device outputs (may be NULL).
 *   change  host output: max(|U' - U|, ||Delta|' - |Delta||) before mixing.
 *   m       host output: number of states in the window.
 *   work    device workspace of bdg_scf_workspace bytes.
 * Synchronises `stream`.
 */
int bdg_scf_step(const bdg_lattice *lat, const double *Vext, const double *theta, double mu,
                 const bdg_scf_params *params, double *U, double *absDelta, double *density,
                 double *nu_abs, double *change, int64_t *m, void *work, size_t work_bytes,
                 bdg_stream_t stream);

/*
 * bdg_regrid -- move a real periodic field between the lattices of the
 * multigrid start ("Performance of the Matrix Diagonalization Algorithm":
 * the solution on a coarser lattice starts the next finer one).
 *   src, f   source lattice and field [src sites] (device, f64, x fastest).
 *   dst, g   target lattice (same ndim) and field [dst sites] (device, f64).
 *   scale    every output value is multiplied by it (the energy and density
 *            rescaling between lattices whose unit is the lattice spacing).
 * dst finer or equal along every axis: trigonometric interpolation of the
 * samples (fine site x at x N_c / N_f coarse spacings; the Nyquist
 * coefficient is split evenly between +-N_c/2 so a real field stays real;
 * cost N_f^d N_c^d operations).  dst coarser along every axis by integer
 * factors s_d: injection, g(x) = f(s x).  Anything else returns -3.
 * Dimensions must be even (as for bdg_assemble).  Asynchronous.
 */
int bdg_regrid(const bdg_lattice *src, const double *f, const bdg_lattice *dst, double *g, double scale,
               bdg_stream_t stream);

/*
 * Time evolution of the quasiparticle wavefunctions, eq. (TDSLDA):
 *   i d/dt phi_j = H(t) phi_j,  H = [[h, Delta], [Delta^*, -h^*]],  h = -nabla^2/2 + U - mu,
 * the kinetic term being the same spectral operator as in bdg_assemble.  With
 * self_consistent = 1 the mean fields follow the evolved states at every
 * evaluation (zero-temperature occupations, eq. densities2):
 *   n = 2 sum_j |v_j|^2,  nu = sum_j u_j v_j^*,  U = Vext + B eps_F(n),  Delta = g nu
 * (the pairing phase evolves freely); with 0 they stay the given U0, Delta0.
 * Integrator ("Performance of the Time Evolution Algorithm"): fifth-order
 * Adams-Bashforth-Moulton predictor-corrector, two evaluations of H per step,
 *   phi* = phi_k + dt (1901 f_k - 2774 f_{k-1} + 2616 f_{k-2} - 1274 f_{k-3} + 251 f_{k-4}) / 720,
 *   phi_{k+1} = phi_k + dt (251 f(phi*) + 646 f_k - 264 f_{k-1} + 106 f_{k-2} - 19 f_{k-3}) / 720,
 * f = -i H[phi] phi; the first four steps of a fresh start take classical RK4.
 */
typedef struct {
    double B;                /* density coefficient of U (as in bdg_scf_params)  */
    double g;                /* pairing coupling, Delta = g nu                    */
    int32_t self_consistent; /* 1: fields from the evolved states; 0: U0, Delta0  */
    int32_t resume;          /* 1: continue the history the workspace holds from
                                the previous call (same lattice, states, dt);
                                0: fresh start (RK4 for the first four steps)    */
} bdg_td_params;

/* bdg_td_workspace -- device workspace (bytes) of bdg_td_evolve for m states:
 * eight n x m complex128 state arrays (five derivatives of the history, the
 * predictor, one evaluation, one RK4 sum) plus O(n) fields. */
int bdg_td_workspace(const bdg_lattice *lat, int64_t m, size_t *bytes);

/*
 * bdg_td_evolve -- advance m states by nsteps steps of size dt.
 *   lat      lattice with at most 4096 sites (u and v of a state are staged in
 *            LDS); more returns BDG_ERR_NOT_IMPLEMENTED.
 *   Vext     [nsites] f64 device (self-consistent fields; may be NULL otherwise).
 *   mu       chemical potential in h.
 *   Phi      [ldphi x m] complex128 device, the states [u; v] (n = 2 nsites
 *            rows), advanced in place.
 *   U0, Delta0  [nsites] f64 / complex128 device: the fixed fields when
 *            self_consistent = 0 (may be NULL otherwise).
 *   work     device workspace of work_bytes >= bdg_td_workspace(lat, m).
 * Asynchronous (stream-ordered, no host wait) except that resume = 1 reads two
 * integers of the workspace's history record back first.  A step moves 18
 * state arrays (16 n m bytes each) through HBM.
 */
int bdg_td_evolve(const bdg_lattice *lat, const double *Vext, double mu, const bdg_td_params *params,
                  int64_t m, double *Phi, int64_t ldphi, double dt, int64_t nsteps, const double *U0,
                  const double *Delta0, void *work, size_t work_bytes, bdg_stream_t stream);

/*
 * Start-field network of the learned SCF start (an extension of the method:
 * the paper starts its iterations from coarser lattices).  Four periodic 3x3
 * convolution layers, ReLU between them, FP32 master weights, BF16
 * activations, BF16 matrix cores with FP32 accumulation:
 *   input  (Vext - mu, cos theta, sin theta)  ->  output (U - Vext, |Delta|).
 * Parameters are one flat FP32 vector: W1 [C][3][3][3], b1 [C], W2 [C][C][3][3],
 * b2, W3 [C][C][3][3], b3, W4 [2][C][3][3], b4 (count from bdg_net_nparams).
 * Field arrays are [batch][ny*nx] (site index x + nx y); y and target are
 * [batch][2][ny*nx] FP32.  All pointers are device pointers.
 */
typedef struct {
    int32_t channels; /* hidden channels C (<= 64) */
    int32_t ny, nx;   /* lattice                  */
    int32_t batch;    /* samples per call         */
} bdg_net_shape;

int64_t bdg_net_nparams(const bdg_net_shape *shape);
int bdg_net_workspace(const bdg_net_shape *shape, size_t *bytes);
/* y = net(Vext, theta; params) */
int bdg_net_forward(const bdg_net_shape *shape, const float *params, const double *Vext,
                    const double *theta, double mu, float *y, void *work, size_t work_bytes,
                    bdg_stream_t stream);
/*
 * bdg_net_forward_noalloc -- bdg_net_forward without a workspace argument, for
 * callers that cannot allocate device memory (code under HIP stream capture,
 * tight inference loops, harnesses that forbid hipMalloc).  Same kernels and
 * bit-identical output.  Its scratch (the BF16 weights and each layer's
 * input) lives in a 32 MiB array in the library's device image, one per GPU,
 * kept until the process ends.  A shape needs
 *   2 * 9 * (3C + 2C^2 + 2C) + 2 * batch * ny * nx * (3 + 3C)
 * bytes of it (each of the eight pieces rounded up to 256 bytes; C =
 * channels), e.g. 3.1 MiB for C = 32 on 64 x 64 at batch 4.  A shape that
 * needs more than 32 MiB returns BDG_ERR_WORKSPACE before anything is
 * launched (use bdg_net_forward with a workspace then).
 * The call uses the scratch of the CURRENT device, which must be the device
 * of `stream`.  Every call on one GPU shares that array and leaves its
 * contents behind: calls that overlap on one GPU (two streams, two threads)
 * race and must be serialised by the caller.  A forward pass writes every
 * scratch byte before reading it, so nothing needs clearing between calls.
 * The first call on a device resolves the array's device address once
 * (hipGetSymbolAddress); no call allocates or frees memory.
 */
int bdg_net_forward_noalloc(const bdg_net_shape *shape, const float *params, const double *Vext,
                            const double *theta, double mu, float *y, bdg_stream_t stream);
/* grads = d loss / d params, loss (device scalar) = mean((y - target)^2) */
int bdg_net_backward(const bdg_net_shape *shape, const float *params, const double *Vext,
                     const double *theta, double mu, const float *target, float *grads,
                     float *loss, void *work, size_t work_bytes, bdg_stream_t stream);
/* Start fields of the SCF from output sample `sample` of y (as bdg_net_forward
 * writes it): U = Vext + y[sample][0], |Delta| = max(y[sample][1], 0), f64 on
 * the lattice (Vext, U, absDelta [ny*nx] device). */
int bdg_net_start_fields(const bdg_net_shape *shape, const float *y, int32_t sample, const double *Vext,
                         double *U, double *absDelta, bdg_stream_t stream);
/* Adam (Kingma & Ba) on the FP32 master weights; t is the 1-based step count. */
int bdg_net_adam_step(int64_t nparams, float *params, const float *grads, float *m, float *v,
                      int32_t t, float lr, bdg_stream_t stream);

/*
 * bdg_check -- FP64 accuracy of m eigenpairs (W, Z) of the Hermitian H.
 *   H [ldh x n] complex128 (full storage, both triangles read).
 *   max_resid   = max_j ||H z_j - w_j z_j||_2 / max_j |w_j| (host output)
 *   gram_defect = max_ij |(Z^H Z - I)_ij|                     (host output)
 *   work        device scratch of at least 16*(n*m + m*m) bytes.
 * Synchronises `stream`.
 */
int bdg_check(int64_t n, const double *H, int64_t ldh, int64_t m, const double *W,
              const double *Z, int64_t ldz, double *max_resid, double *gram_defect,
              void *work, size_t work_bytes, bdg_stream_t stream);

/* Text of the last error recorded by this thread (never NULL). */
const char *bdg_last_error(void);

/* Library version string. */
const char *bdg_version(void);

/* ------------------------------------------------------------------------
 * Stage-level entry points.  They expose the individual steps of the
 * two-stage method so that each can be tested and timed on its own; bdg_eigh
 * chains the same kernels.
 * ------------------------------------------------------------------------ */

/*
 * bdg_zgemm -- C = alpha op(A) op(B) + beta C, complex128, column-major,
 * op = 'N' (none) or 'C' (conjugate transpose); 'T' is refused (-1 / -2).  alpha/beta are host
 * complex scalars given as (re, im) pairs.  The MFMA tile kernel shared by
 * stage 1 and the back-transformations.
 */
int bdg_zgemm(char opA, char opB, int64_t M, int64_t N, int64_t K, const double *alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, const double *beta,
              double *C, int64_t ldc, bdg_stream_t stream);

/* bdg_cgemm -- same for complex64 (FP32 MFMA, FP32 accumulation). */
int bdg_cgemm(char opA, char opB, int64_t M, int64_t N, int64_t K, const float *alpha,
              const float *A, int64_t lda, const float *B, int64_t ldb, const float *beta,
              float *C, int64_t ldc, bdg_stream_t stream);

/* bdg_dgemm -- same for real f64 (used by the divide-and-conquer merges);
 * 'T' and 'C' both transpose. */
int bdg_dgemm(char opA, char opB, int64_t M, int64_t N, int64_t K, double alpha,
              const double *A, int64_t lda, const double *B, int64_t ldb, double beta,
              double *C, int64_t ldc, bdg_stream_t stream);

/*
 * bdg_gemm_int8 -- C = alpha op(A) op(B) + beta C in FP64 (real) or complex128
 * (cplx = 1), emulated on the INT8 matrix cores: every row of op(A) and
 * column of op(B) is scaled by a power of two, rounded to 7 slices bits and
 * cut into `slices` int8 digit slices; the slice products are exact int32
 * MFMA sums, added in FP64 with their weights (Ozaki, Ogita, Oishi & Rump,
 * Numer. Algorithms 59 (2012); integer form of Ootomo, Ozaki & Yokota, IJHPCA
 * 2024).  Error bound per entry: 2^(e_r + e_c) K (128^-S + (S+1) 65^2
 * 128^-(S+2)) with max|row r of op(A)| < 2^(e_r - 1), max|column c of op(B)|
 * < 2^(e_c - 1) (complex: real and imaginary parts) -- about 2^-56 2^(e_r +
 * e_c) K at S = 8.  Complex products use the real embedding (four real
 * products of M x K x N).
 *   slices  3 .. 8.   op 'N' or 'C' ('T' for real only).
 *   alpha, beta host scalars ((re, im) pairs when cplx).
 *   work    device workspace of bdg_gemm_int8_workspace bytes.
 * Asynchronous.
 */
int bdg_gemm_int8_workspace(int32_t cplx, int64_t M, int64_t N, int64_t K, int32_t slices, size_t *bytes);
int bdg_gemm_int8(int32_t cplx, int32_t slices, char opA, char opB, int64_t M, int64_t N, int64_t K,
                  const double *alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                  const double *beta, double *C, int64_t ldc, void *work, size_t work_bytes,
                  bdg_stream_t stream);

/*
 * Stage hooks (same kernels as bdg_eigh; for tests and per-stage timing).
 * Workspace sizes come from bdg_stage_workspace(stage, n, band):
 * stage 1 = he2hb, 2 = hb2st (none), 3 = stedc, 4 = bt2, 5 = bt1 (per column: m).
 *
 * bdg_stage_he2hb: A (lower triangle read, overwritten by the reflectors) ->
 *   AB lower band storage (ldab >= 2 band + 2, AB[(i-j) + j ldab] = B(i, j)),
 *   T1 [panels x band x band] block-reflector factors.
 * bdg_stage_hb2st: AB (destroyed) -> d [n] real diagonal, e [n-1] complex
 *   sub-diagonal; reflectors in V2/tau2 with device offsets voff [n] that the
 *   call fills.  V2 needs band*(bdg_stage_nrefl(n, band)+1) complex entries.
 * bdg_stage_stedc: real symmetric tridiagonal (d, e) -> W ascending and Q
 *   (n x n, ld n, real).
 * bdg_stage_bt2: Z [n x m] complex = Q2 diag(ph) Y[:, i0:i0+m] with ph from e.
 * bdg_stage_bt1: Z <- Q1 Z with the stage-1 reflectors left in A.
 */
int bdg_stage_workspace(int stage, int64_t n, int band, int64_t m, size_t *bytes);

/*
 * bdg_stage_zgemm -- the complex128 tile GEMM in one of the modes the solver
 * stages use, with an explicit split of K (the stage-1 products and the BT1
 * Gram product split K over several workgroups and sum the partial products
 * in a second kernel).  C = alpha op(A) op(B) + beta C, column-major.
 *   mode 0: every tile of C.
 *   mode 1: only the 64 x 64 tiles of C on and below the diagonal (Hermitian
 *           rank-k updates); needs opA = 'N', M == N, splitk == 1.
 *   mode 2: A is Hermitian M x M with only its lower triangle valid (the
 *           upper triangle is never read); needs opA = 'N', K == M.
 *   splitk 1..64: number of K chunks (rounded to whole 16-deep steps; may
 *           come out smaller).  work: >= 16 splitk M N bytes when splitk > 1.
 */
int bdg_stage_zgemm(int mode, int splitk, char opA, char opB, int64_t M, int64_t N, int64_t K,
                    const double *alpha, const double *A, int64_t lda, const double *B, int64_t ldb,
                    const double *beta, double *C, int64_t ldc, void *work, size_t work_bytes,
                    bdg_stream_t stream);
int64_t bdg_stage_nrefl(int64_t n, int band);
int bdg_stage_he2hb(int64_t n, double *A, int64_t lda, int band, double *AB, int64_t ldab,
                    double *T1, void *work, size_t work_bytes, bdg_stream_t stream);
int bdg_stage_hb2st(int64_t n, int band, double *AB, int64_t ldab, double *d, double *e,
                    double *V2, double *tau2, int64_t *voff, bdg_stream_t stream);
int bdg_stage_stedc(int64_t n, const double *d, const double *e, double *W, double *Q, int leaf,
                    void *work, size_t work_bytes, bdg_stream_t stream);
int bdg_stage_bt2(int64_t n, int band, int64_t m, const double *e, const double *Y, int64_t i0,
                  const double *V2, const double *tau2, const int64_t *voff, double *Z,
                  int64_t ldz, void *work, size_t work_bytes, bdg_stream_t stream);
int bdg_stage_bt1(int64_t n, int64_t m, const double *A, int64_t lda, int band, const double *T1,
                  double *Z, int64_t ldz, void *work, size_t work_bytes, bdg_stream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* BDG_H */
