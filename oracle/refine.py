"""Oracle: Ogita-Aishima iterative refinement of Hermitian eigenpairs (FP64).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Refinement recovers FP64 accuracy from eigenvectors computed in a lower
precision (the precision extension of the hot path; the paper's own
diagonalisations are FP64 throughout).  One step, following Ogita & Aishima,
"Iterative refinement for symmetric eigenvalue decomposition", Japan J.
Indust. Appl. Math. 35 (2018), written for complex Hermitian H:

    R = I - X^H X,  S = X^H H X          (both Hermitian-symmetrised)
    lam_i = s_ii / (1 - r_ii)
    delta = 2 (||S - diag(lam)||_2 + ||H||_2 ||R||_2)
    E_ij  = (s_ij + lam_j r_ij) / (lam_j - lam_i)  if |lam_i - lam_j| > delta
          = r_ij / 2                               otherwise
    X <- X + X E

(the complex case follows from E + E^H = R and S + E^H Lam + Lam E = Lam, as in
the real case).  The window variant refines only the columns W of X against
the full basis X: R[:, W] = I[:, W] - X^H X_W, S[:, W] = X^H (H X_W).

Clusters (Ogita & Aishima, part II: clustered eigenvalues, Japan J. Indust.
Appl. Math. 36 (2019)).  The r_ij / 2 branch only re-orthonormalises a group of
close eigenvalues; it never resolves the mixing inside the group.  So each
cluster also gets a Rayleigh-Ritz step in FP64: with L = I + R_JJ / 2
(first-order Loewdin orthonormalisation of the cluster columns),
M = L S_JJ L = Q diag(mu) Q^H, the cluster columns become X (I + E)[:, J] Q and
their eigenvalues mu.

Which pairs are close (rule "pair", the one the GPU path uses): the published
criterion |lam_i - lam_j| <= delta uses one global delta, and from an FP32
basis of order 10^4 delta exceeds the mean level spacing, so its chains of
close eigenvalues join most of the spectrum.  Here a pair is close when its
first-order coefficient would not be small, |s_ij + lam_j r_ij| >= tau
|lam_j - lam_i| with tau = 1e-3 (this includes lam_i = lam_j); clusters are the
connected components of close pairs inside the window; close pairs with a row
outside the window take r_ij / 2 without Rayleigh-Ritz.  Rule "delta" is the
published criterion (clusters = chains of sorted eigenvalues with gaps <= delta).
"""
from __future__ import annotations

import numpy as np

TAU = 1e-3


def _herm(M):
    return 0.5 * (M + M.conj().T)


def clusters(lam: np.ndarray, delta: float):
    """Index arrays of the chains (>= 2 members) of sorted lam with gaps <= delta,
    each in ascending order of lam."""
    order = np.argsort(lam, kind="stable")
    out, start = [], 0
    for k in range(1, order.size + 1):
        if k == order.size or lam[order[k]] - lam[order[k - 1]] > delta:
            if k - start >= 2:
                out.append(order[start:k])
            start = k
    return out


def components(m: int, pairs, lam: np.ndarray):
    """Connected components (>= 2 members) of the graph on 0..m-1 with the given
    edges, each in ascending order of lam."""
    parent = list(range(m))

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    for a, b in pairs:
        ra, rb = root(int(a)), root(int(b))
        if ra != rb:
            parent[ra] = rb
    groups = {}
    for a in range(m):
        groups.setdefault(root(a), []).append(a)
    out = [np.array(sorted(g, key=lambda t: (lam[t], t))) for g in groups.values() if len(g) >= 2]
    out.sort(key=lambda J: (lam[J[0]], J[0]))
    return out


def _correction(S, R, lam_rows, lam_W, win_rows, rule, delta, tau=TAU):
    """E for the rows of S, R (n x m) and the clusters of the window.

    win_rows[k] is the row of window column k."""
    n, m = S.shape
    diff = lam_W[None, :] - lam_rows[:, None]        # lam_j - lam_i
    num = S + lam_W[None, :] * R
    if rule == "delta":
        near = np.abs(diff) <= delta
        cl = clusters(lam_W, delta)
    else:
        near = np.abs(num) >= tau * np.abs(diff)
        Wn = near[win_rows, :]
        a, b = np.nonzero(np.triu(Wn | Wn.T, 1))
        cl = components(m, zip(a, b), lam_W)
        same = np.zeros((m, m), dtype=bool)
        for J in cl:
            same[np.ix_(J, J)] = True
        same[np.arange(m), np.arange(m)] = True
        near[win_rows, :] = same
    with np.errstate(divide="ignore", invalid="ignore"):
        E = np.where(near, R / 2.0, num / np.where(near, 1.0, diff))
    return E, cl


def _cluster_rr(E, I_W, Rw, Sw, lam_W, cl):
    """Rayleigh-Ritz inside each cluster: E[:, J] <- (I_W + E)[:, J] Q - I_W[:, J]."""
    for J in cl:
        L = np.eye(J.size) + Rw[np.ix_(J, J)] / 2.0
        M = _herm(L @ Sw[np.ix_(J, J)] @ L)
        mu, Q = np.linalg.eigh(M)
        E[:, J] = (I_W[:, J] + E[:, J]) @ Q - I_W[:, J]
        lam_W[J] = mu


def oa_step(H: np.ndarray, X: np.ndarray, normH: float | None = None, cluster_rr: bool = True,
            rule: str = "pair"):
    """One full Ogita-Aishima step on all columns; returns (X_new, lam)."""
    n = X.shape[1]
    R = _herm(np.eye(n) - X.conj().T @ X)
    S = _herm(X.conj().T @ (H @ X))
    lam = np.real(np.diag(S)) / (1.0 - np.real(np.diag(R)))
    delta = None
    if rule == "delta":
        if normH is None:
            normH = np.abs(np.linalg.eigvalsh(H)).max()
        delta = 2.0 * (np.linalg.norm(S - np.diag(lam), 2) + normH * np.linalg.norm(R, 2))
    E, cl = _correction(S, R, lam, lam, np.arange(n), rule, delta)
    if cluster_rr:
        _cluster_rr(E, np.eye(n), R, S, lam, cl)
    return X + X @ E, lam


def oa_step_window(H: np.ndarray, X: np.ndarray, lam0: np.ndarray, cols: np.ndarray, normH: float,
                   cluster_rr: bool = True, rule: str = "pair", return_clusters: bool = False):
    """Refine columns `cols` of the full basis X; returns (X_W_new, lam_W),
    and the clusters (index arrays into the window) if return_clusters.

    lam0 are the approximate eigenvalues that came with X; outside the window
    they stand in for the Rayleigh quotients in the denominators (their error
    only enters the small off-window coefficients at second order)."""
    XW = X[:, cols]
    n = X.shape[1]
    I_W = np.zeros((n, cols.size))
    I_W[cols, np.arange(cols.size)] = 1.0
    R = I_W - X.conj().T @ XW
    S = X.conj().T @ (H @ XW)
    # Hermitian symmetrisation of the square block on the window rows
    Rw = _herm(R[cols, :])
    Sw = _herm(S[cols, :])
    R[cols, :] = Rw
    S[cols, :] = Sw
    lam_all = np.array(lam0, dtype=np.float64, copy=True)
    lam_W = np.real(np.diag(Sw)) / (1.0 - np.real(np.diag(Rw)))
    lam_all[cols] = lam_W
    delta = None
    if rule == "delta":
        delta = 2.0 * (np.linalg.norm(Sw - np.diag(lam_W), 2) + normH * np.linalg.norm(R, 2))
    E, cl = _correction(S, R, lam_all, lam_W, cols, rule, delta)
    if cluster_rr:
        _cluster_rr(E, I_W, Rw, Sw, lam_W, cl)
    if return_clusters:
        return XW + X @ E, lam_W, cl
    return XW + X @ E, lam_W


def ph_mirror(Xp: np.ndarray) -> np.ndarray:
    """Particle-hole partners (-v^*, u^*) of the columns [u; v] of Xp."""
    ns = Xp.shape[0] // 2
    u, v = Xp[:ns], Xp[ns:]
    return np.vstack([-v.conj(), u.conj()])


def accuracy(H: np.ndarray, W: np.ndarray, Z: np.ndarray):
    """(max_j ||H z_j - w_j z_j|| / ||H||_2, max |Z^H Z - I|)."""
    normH = np.abs(np.linalg.eigvalsh(H)).max()
    res = np.linalg.norm(H @ Z - Z * W, axis=0).max() / normH
    gram = np.abs(Z.conj().T @ Z - np.eye(Z.shape[1])).max()
    return res, gram
