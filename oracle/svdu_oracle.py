"""CPU oracle for the rank-1 SVD update -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this module. The product path never calls it and it
shares no code with the HIP path.

Plain, slow, fp64 numpy. It follows the paper (Gandhi & Rajgor, "Updating
Singular Value Decomposition for Rank One Matrix Perturbation") step by step:

* Section 3 / Appendix A: the Gram expansions of A^ A^T and A^T A^ and the 2x2
  symmetric splits (equations AAT3Rank11, U+D+U+T, V+D+V+T).
* Section 6.1 (Algorithm "Update SVD of rank-1 modified matrix"), Steps 1-8,
  in the literal form: b~ = U S V^T b and a~ = V S^T U^T a are formed
  explicitly and every projected vector is re-projected with the current
  basis (RankOneUpdate Step 1).
* Section 6.2 (RankOneUpdate), Steps 1-7: projection, the secular equation
  (equation GolubEigenvalUpdate), the Cauchy eigenvector matrix
  C~ = diag(a_bar) C diag(|c_i|)^-1 (equation CTildeFinalForm1) and the
  product U C~ (equation UCTildeProduct), done here as a dense matmul.

Readings where the paper is silent (each also recorded in the design notes):

* Deflation (Section 3.1 names the cases but no rule): components with
  |z_j| <= 8 u sqrt(N) |z| are dropped (their basis vector is kept with its old
  eigenvalue); exactly repeated poles are merged into one pole, whose weight is
  the norm of the group's z, and a Householder reflection supplies the group's
  remaining eigenvectors. Close but distinct poles are not merged.
* The secular roots are stored relative to their nearer pole, (k_i, tau_i) with
  mu_i = d_k + tau_i, and found by bisection in tau (Golub's function is
  monotone between consecutive poles). Negative rho is handled by reflecting
  the poles.
* The eigenvector weights are recomputed from the roots (the Loewner formula of
  Gu & Eisenstat, not in the paper) so that C~ is orthogonal to working
  precision.
* Step 8 takes Sigma^ from the left side; the signs of the right singular
  vectors are paired with the left ones by s_i = sign(u_i^T A^ v_i), which the
  paper leaves out.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

U64 = 2.0 ** -53          # unit roundoff of IEEE double
BISECT_MAX = 400          # bisection halvings per root (never reached in practice)


# ---------------------------------------------------------------------------
# Algorithm Steps 2-3 / Appendix A: Schur decomposition of [[beta, 1], [1, 0]].
# ---------------------------------------------------------------------------
def gram_split(beta: float):
    """Eigen-decomposition [[beta, 1], [1, 0]] = Q diag(rho_plus, rho_minus) Q^T.

    The eigenvalues are the roots of r^2 - beta r - 1 = 0; their product is -1,
    which gives the smaller-magnitude one without cancellation. The eigenvector
    of eigenvalue r is proportional to (r, 1).
    """
    s = np.hypot(beta, 2.0)
    if beta >= 0.0:
        rp = 0.5 * (beta + s)
        rm = -1.0 / rp
    else:
        rm = 0.5 * (beta - s)
        rp = -1.0 / rm
    qp = np.array([rp, 1.0]) / np.hypot(rp, 1.0)
    qm = np.array([rm, 1.0]) / np.hypot(rm, 1.0)
    return rp, rm, np.column_stack([qp, qm])


# ---------------------------------------------------------------------------
# Deflation (Section 3.1 cases (1) and (3)).
# ---------------------------------------------------------------------------
@dataclass
class Deflation:
    tol: float
    tiny: np.ndarray        # bool, per sorted position
    cluster: np.ndarray     # int, cluster id per sorted position (-1 for tiny)
    first: np.ndarray       # int, first sorted position of each cluster
    members: list           # list of arrays of sorted positions per cluster
    g: np.ndarray           # representative pole per cluster (ascending)
    W: np.ndarray           # weight = norm of the cluster's z


def deflate(lam: np.ndarray, z: np.ndarray, rho: float) -> Deflation:
    """Deflation decisions for D + rho z z^T with lam sorted ascending.

    Case (1), a zero component: |z_j| <= 8 u sqrt(N) |z|, the level of the
    rounding noise that a projection z = X^T v leaves in a component that is
    zero in exact arithmetic. The basis vector is kept with its eigenvalue.
    Case (3), a repeated eigenvalue: poles that are exactly equal merge into one
    pole whose weight is the norm of their z entries. Poles that are merely
    close stay separate: the pole-relative roots resolve them, and moving a
    pole by an absolute tolerance would spoil the small eigenvalues.
    """
    N = lam.shape[0]
    znorm = float(np.sqrt(np.sum(z * z)))
    tol = 8.0 * U64 * np.sqrt(max(N, 1)) * znorm
    tiny = np.abs(z) <= tol
    cluster = np.full(N, -1, dtype=np.int64)
    first, members = [], []
    start_val = None
    for j in range(N):
        if tiny[j]:
            continue
        if start_val is None or lam[j] != start_val:
            start_val = lam[j]
            first.append(j)
            members.append([])
        cluster[j] = len(first) - 1
        members[-1].append(j)
    members = [np.asarray(mm, dtype=np.int64) for mm in members]
    first = np.asarray(first, dtype=np.int64)
    g = lam[first] if len(first) else np.zeros(0)
    W = np.array([np.sqrt(np.sum(z[mm] ** 2)) for mm in members]) if members else np.zeros(0)
    return Deflation(tol=tol, tiny=tiny, cluster=cluster, first=first, members=members, g=g, W=W)


# ---------------------------------------------------------------------------
# RankOneUpdate Step 2: roots of w(mu) = 1 + rho sum z_k^2 / (d_k - mu).
# ---------------------------------------------------------------------------
def secular_f(g, W2, rho, org, tau):
    """Golub's secular function at mu = g[org] + tau, with pole differences
    formed as (g_k - g_org) - tau. Vectorised over roots; returns shape (r,)."""
    delta = (g[None, :] - g[org][:, None]) - tau[:, None]
    return 1.0 + rho * np.sum(W2[None, :] / delta, axis=1)


def _secular_positive(g, W2, rho, idx):
    """Roots with index idx for rho > 0 (poles ascending, all weights > 0)."""
    K = g.shape[0]
    idx = np.asarray(idx, dtype=np.int64)
    org = idx.copy()
    lo = np.zeros(idx.shape[0])
    hi = np.zeros(idx.shape[0])
    inner = idx < K - 1
    if np.any(inner):
        ii = idx[inner]
        half = 0.5 * (g[ii + 1] - g[ii])
        fmid = secular_f(g, W2, rho, ii, half)
        left = fmid >= 0.0       # root in (g_i, g_i + half]: origin at g_i
        o = np.where(left, ii, ii + 1)
        org[inner] = o
        lo[inner] = np.where(left, 0.0, -half)
        hi[inner] = np.where(left, half, 0.0)
    last = ~inner
    if np.any(last):
        org[last] = K - 1
        lo[last] = 0.0
        hi[last] = rho * np.sum(W2)
    active = np.ones(idx.shape[0], dtype=bool)
    for _ in range(BISECT_MAX):
        width = hi - lo
        active &= width > 2.0 * U64 * np.maximum(np.abs(lo), np.abs(hi))
        if not np.any(active):
            break
        a = np.nonzero(active)[0]
        mid = 0.5 * (lo[a] + hi[a])
        f = secular_f(g, W2, rho, org[a], mid)
        neg = f < 0.0
        lo[a] = np.where(neg, mid, lo[a])
        hi[a] = np.where(neg, hi[a], mid)
    return org, 0.5 * (lo + hi)


def secular_roots(g, W, rho, idx=None, chunk=256):
    """All (or the selected) roots of the secular equation, pole-relative.

    g: distinct poles ascending; W: weights (only W^2 enters); rho != 0.
    Returns (org, tau) with mu_i = g[org_i] + tau_i, roots ascending in i.
    For rho < 0 the poles are reflected, d -> -reverse(d), and mapped back.
    """
    K = g.shape[0]
    if idx is None:
        idx = np.arange(K)
    idx = np.asarray(idx, dtype=np.int64)
    W2 = W * W
    if rho > 0:
        gg, ww, rr, ii = g, W2, rho, idx
    else:
        gg, ww, rr, ii = -g[::-1], W2[::-1], -rho, K - 1 - idx
    org = np.empty(ii.shape[0], dtype=np.int64)
    tau = np.empty(ii.shape[0])
    for s in range(0, ii.shape[0], chunk):
        o, t = _secular_positive(gg, ww, rr, ii[s:s + chunk])
        org[s:s + chunk] = o
        tau[s:s + chunk] = t
    if rho < 0:
        org = K - 1 - org
        tau = -tau
    return org, tau


# ---------------------------------------------------------------------------
# Eigenvector weights from the roots (Loewner / Gu-Eisenstat).
# ---------------------------------------------------------------------------
def loewner_weights(g, org, tau, rho):
    """|w_hat_j| with prod_i (mu_i - g_j) / (rho prod_{k != j} (g_k - g_j)).

    The product is taken as K ratios that each lie in (0, 1]: for rho > 0 the
    roots interlace g_1 < mu_1 < g_2 < ... < g_K < mu_K, and root i is paired
    with pole i (i < j) or pole i+1 (i >= j); the last root pairs with rho.
    rho < 0 is reduced to rho > 0 by reflection.
    """
    K = g.shape[0]
    if rho < 0:
        gr = -g[::-1]
        o = K - 1 - org[::-1]
        t = -tau[::-1]
        return loewner_weights(gr, o, t, -rho)[::-1]
    if K == 0:
        return np.zeros(0)
    # mu_i - g_j = (g_org(i) - g_j) + tau_i, matrix [i, j]
    mu_minus_g = (g[org][:, None] - g[None, :]) + tau[:, None]
    i = np.arange(K)[:, None]
    j = np.arange(K)[None, :]
    ratio = np.empty((K, K))
    # roots 0..K-2 pair with pole i (when i < j) or pole i+1 (when i >= j)
    pair = np.where(i < j, i, i + 1)[: K - 1]
    ratio[: K - 1] = mu_minus_g[: K - 1] / (g[pair] - g[None, :])
    # the last root pairs with rho
    ratio[K - 1] = mu_minus_g[K - 1] / rho
    return np.sqrt(np.prod(ratio, axis=0))


# ---------------------------------------------------------------------------
# RankOneUpdate (Section 6.2).
# ---------------------------------------------------------------------------
@dataclass
class StageResult:
    X: np.ndarray          # updated basis, columns sorted by ascending eigenvalue
    lam: np.ndarray        # eigenvalues ascending
    flags: np.ndarray      # int8 per input column: 0 live, 1 tiny z, 2 merged pole
    K: int                 # number of secular roots
    org: np.ndarray        # root origin pole (index into g)
    tau: np.ndarray        # root offset from its origin pole
    g: np.ndarray          # distinct live poles, ascending
    W: np.ndarray          # their weights
    zhat: np.ndarray       # Loewner weights (per live pole)
    z: np.ndarray          # projected vector (input column order)


def cauchy_eigvecs(lam_s, z_s, rho, defl: Deflation, org, tau, what):
    """Columns of C~ (sorted-pole row order) and their eigenvalues.

    Live column i: entries what_j / ((g(j) - g_org) - tau_i), j over the rows
    of live clusters, normalised to unit length (equation CTildeFinalForm1).
    Deflated columns: unit vectors for tiny-z rows; Householder columns for the
    non-leading members of merged clusters.
    """
    N = lam_s.shape[0]
    K = defl.g.shape[0]
    cols, vals, kinds, keys = [], [], [], []
    # live columns
    rows_live = np.nonzero(~defl.tiny)[0]
    cl = defl.cluster[rows_live]
    zeta = what[cl] * z_s[rows_live] / defl.W[cl]      # per-row weight, sign of z
    for i in range(K):
        delta = (defl.g[cl] - defl.g[org[i]]) - tau[i]
        c = np.zeros(N)
        c[rows_live] = zeta / delta
        s = np.max(np.abs(c))
        c /= s * np.sqrt(np.sum((c / s) ** 2)) if s > 0 else 1.0
        cols.append(c)
        vals.append(defl.g[org[i]] + tau[i])
        kinds.append(0)
        keys.append(i)
    # deflated columns: tiny rows
    for j in np.nonzero(defl.tiny)[0]:
        c = np.zeros(N)
        c[j] = 1.0
        cols.append(c)
        vals.append(lam_s[j])
        kinds.append(1)
        keys.append(j)
    # deflated columns: merged clusters (Householder H v = -s e_first)
    for mm in defl.members:
        if mm.shape[0] < 2:
            continue
        v = z_s[mm] / np.sqrt(np.sum(z_s[mm] ** 2))
        sgn = 1.0 if v[0] >= 0 else -1.0
        u = v.copy()
        u[0] += sgn
        H = np.eye(mm.shape[0]) - 2.0 * np.outer(u, u) / (u @ u)
        for t in range(1, mm.shape[0]):
            c = np.zeros(N)
            c[mm] = H[:, t]
            cols.append(c)
            vals.append(lam_s[mm[t]])
            kinds.append(1)
            keys.append(mm[t])
    C = np.column_stack(cols) if cols else np.zeros((N, 0))
    vals = np.asarray(vals)
    order = np.lexsort((np.asarray(keys), np.asarray(kinds), vals))
    return C[:, order], vals[order]


def rank_one_update(X: np.ndarray, lam: np.ndarray, v: np.ndarray, rho: float) -> StageResult:
    """RankOneUpdate(X, v, D, rho): eigen-decomposition of X diag(lam) X^T + rho v v^T.

    X has orthonormal columns with eigenvalues lam (any order). Returns the new
    basis X C~ and eigenvalues, both ascending.
    """
    return rank_one_update_z(X, lam, X.T @ v, rho)   # Step 1: a_bar = X^T v


def rank_one_update_z(X: np.ndarray, lam: np.ndarray, z: np.ndarray, rho: float) -> StageResult:
    """RankOneUpdate Steps 2-7 for a given projection z = a_bar (Step 1 done)."""
    N = lam.shape[0]
    order = np.argsort(lam, kind="stable")
    lam_s, z_s = lam[order], z[order]
    defl = deflate(lam_s, z_s, rho)
    K = defl.g.shape[0]
    if K:
        org, tau = secular_roots(defl.g, defl.W, rho)          # Step 2
        what = loewner_weights(defl.g, org, tau, rho)
    else:
        org = np.zeros(0, dtype=np.int64)
        tau = np.zeros(0)
        what = np.zeros(0)
    C, vals = cauchy_eigvecs(lam_s, z_s, rho, defl, org, tau, what)   # Steps 3, 5, 7
    Xn = X[:, order] @ C                             # Steps 4, 6: U_1 C, column-scaled
    flags_s = np.zeros(N, dtype=np.int8)
    flags_s[defl.tiny] = 1
    for mm in defl.members:
        flags_s[mm[1:]] = 2
    flags = np.empty(N, dtype=np.int8)
    flags[order] = flags_s
    return StageResult(X=Xn, lam=vals, flags=flags, K=K, org=org, tau=tau, g=defl.g,
                       W=defl.W, zhat=what, z=z)


# ---------------------------------------------------------------------------
# Algorithm of Section 6.1.
# ---------------------------------------------------------------------------
@dataclass
class UpdateResult:
    U: np.ndarray          # m x m, columns by descending singular value
    sigma: np.ndarray      # m, descending
    V: np.ndarray          # n x n; columns m..n-1 span the null space of A^
    lam_v: np.ndarray      # n eigenvalues of A^T A^, descending
    stages: list           # StageResult for L+, L-, R+, R-
    rho: tuple             # (rho1, rho2, rho3, rho4)
    signs: np.ndarray      # applied to the first m columns of V


def svd_rank1_update(U, sigma, V, a, b, pair_signs: bool = True) -> UpdateResult:
    """SVD of A^ = U diag(sigma) V^T + a b^T, m <= n, sigma descending."""
    U = np.asarray(U, dtype=np.float64)
    V = np.asarray(V, dtype=np.float64)
    sigma = np.asarray(sigma, dtype=np.float64)
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m, n = U.shape[0], V.shape[0]
    if not (1 <= m <= n) or sigma.shape[0] != m:
        raise ValueError("need 1 <= m <= n and len(sigma) == m")
    # Step 1
    Vtb = V.T @ b
    btil = U @ (sigma * Vtb[:m])                     # U Sigma V^T b
    atil = V[:, :m] @ (sigma * (U.T @ a))            # V Sigma^T U^T a
    beta = float(b @ b)
    alpha = float(a @ a)
    Du = sigma ** 2
    Dv = np.concatenate([sigma ** 2, np.zeros(n - m)])
    # Steps 2-3
    r1, r2, Qu = gram_split(beta)
    a1 = Qu[0, 0] * a + Qu[1, 0] * btil
    b1 = Qu[0, 1] * a + Qu[1, 1] * btil
    r3, r4, Qv = gram_split(alpha)
    a2 = Qv[0, 0] * b + Qv[1, 0] * atil
    b2 = Qv[0, 1] * b + Qv[1, 1] * atil
    # Steps 4-7
    s1 = rank_one_update(U, Du, a1, r1)
    s2 = rank_one_update(s1.X, s1.lam, b1, r2)
    s3 = rank_one_update(V, Dv, a2, r3)
    s4 = rank_one_update(s3.X, s3.lam, b2, r4)
    # Step 8: descending order, Sigma_n = sqrt(D_n)
    Un = s2.X[:, ::-1].copy()
    Dn = s2.lam[::-1]
    Vn = s4.X[:, ::-1].copy()
    Dvn = s4.lam[::-1]
    sig = np.sqrt(np.maximum(Dn, 0.0))
    signs = np.ones(m)
    if pair_signs:
        Ahat = (U * sigma[None, :]) @ V[:, :m].T + np.outer(a, b)
        d = np.einsum("ij,ij->j", Un, Ahat @ Vn[:, :m])
        signs = np.where(d < 0.0, -1.0, 1.0)
        Vn[:, :m] *= signs[None, :]
    return UpdateResult(U=Un, sigma=sig, V=Vn, lam_v=Dvn, stages=[s1, s2, s3, s4],
                        rho=(r1, r2, r3, r4), signs=signs)


# ---------------------------------------------------------------------------
# Rank-k update (Section 8, Conclusion: the extension to rank k), as k rank-1
# updates applied in order.
# ---------------------------------------------------------------------------
def svd_rankk_update(U, sigma, V, A, B) -> UpdateResult:
    """SVD of U diag(sigma) V^T + sum_j A[j]^T B[j] (row j of A and B is the
    pair a_j, b_j): the rank-1 update of Section 6.1 applied to a_0 b_0^T, then
    to a_1 b_1^T on its result, and so on. Returns the last update's result."""
    A = np.atleast_2d(np.asarray(A, dtype=np.float64))
    B = np.atleast_2d(np.asarray(B, dtype=np.float64))
    if A.shape[0] != B.shape[0] or A.shape[0] < 1:
        raise ValueError("A and B need the same k >= 1 rows")
    r = None
    for a, b in zip(A, B):
        r = svd_rank1_update(U, sigma, V, a, b)
        U, sigma, V = r.U, r.sigma, r.V
    return r


# ---------------------------------------------------------------------------
# Checks used by the tests (plain definitions).
# ---------------------------------------------------------------------------
def dense_ahat(U, sigma, V, a, b):
    m = U.shape[0]
    return (U * sigma[None, :]) @ V[:, :m].T + np.outer(a, b)


def recon_error(Ahat, Uh, sh, Vh):
    """|U^ S^ V^^T - A^|_F / |A^|_F."""
    m = Uh.shape[0]
    R = (Uh * sh[None, :]) @ Vh[:, :m].T - Ahat
    return float(np.linalg.norm(R) / np.linalg.norm(Ahat))


def paper_error(Ahat, Uh, sh, Vh):
    """Error measure of the paper's Section 7: max |(A^ - U^ S^ V^^T) / max sigma^|."""
    m = Uh.shape[0]
    R = Ahat - (Uh * sh[None, :]) @ Vh[:, :m].T
    return float(np.max(np.abs(R)) / np.max(sh))


def orth_error(Q):
    return float(np.max(np.abs(Q.T @ Q - np.eye(Q.shape[1])))) if Q.size else 0.0
