"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each check is a closed form, an
invariant, a library routine on a special case, brute force on a tiny input,
or a bound the paper prints. The planted-mistake tests at the end show that a
plausible error in the oracle fails at least one pin.
"""
import os

import numpy as np
import pytest

import oracle as O
import oracle.svdu_oracle as OS
import synth_inputs as S

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# 2x2 split (Algorithm Steps 2-3, Appendix A)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("beta", [0.0, 1.0, -3.0, 1e-8, 1e8, 2.5])
def test_gram_split_closed_form(beta):
    rp, rm, Q = O.gram_split(beta)
    # r^2 - beta r - 1 = 0 for both roots: product -1, sum beta
    assert abs(rp * rm + 1.0) <= 4e-16
    assert abs((rp + rm) - beta) <= 4e-16 * max(1.0, abs(beta))
    assert rp > 0 > rm
    assert np.max(np.abs(Q.T @ Q - np.eye(2))) <= 4e-16
    M = np.array([[beta, 1.0], [1.0, 0.0]])
    assert np.max(np.abs(Q @ np.diag([rp, rm]) @ Q.T - M)) <= 4e-16 * max(1.0, abs(beta))


def test_gram_split_reproduces_three_rank_one_terms():
    rng = np.random.default_rng(3)
    a, bt = rng.standard_normal(7), rng.standard_normal(7)
    beta = 0.37
    rp, rm, Q = O.gram_split(beta)
    a1 = Q[0, 0] * a + Q[1, 0] * bt
    b1 = Q[0, 1] * a + Q[1, 1] * bt
    lhs = beta * np.outer(a, a) + np.outer(a, bt) + np.outer(bt, a)
    rhs = rp * np.outer(a1, a1) + rm * np.outer(b1, b1)
    assert np.max(np.abs(lhs - rhs)) <= 1e-14


# ---------------------------------------------------------------------------
# Secular equation (equation GolubEigenvalUpdate, RankOneUpdate Step 2)
# ---------------------------------------------------------------------------
def _roots(d, z, rho):
    # module attributes, so that the planted-mistake tests below reach them
    defl = OS.deflate(d, z, rho)
    org, tau = OS.secular_roots(defl.g, defl.W, rho)
    return defl, org, tau


@pytest.mark.parametrize("rho", [0.7, -0.7, 3.0, -0.05])
def test_secular_2x2_closed_form(rho):
    d = np.array([0.3, 1.1])
    z = np.array([0.6, -0.8])
    _, org, tau = _roots(d, z, rho)
    M = np.diag(d) + rho * np.outer(z, z)
    T, D = M[0, 0] + M[1, 1], M[0, 0] * M[1, 1] - M[0, 1] ** 2
    disc = np.sqrt(T * T - 4 * D)
    big = 0.5 * (T + disc) if T >= 0 else 0.5 * (T - disc)
    closed = np.sort([big, D / big])
    mu = d[org] + tau
    assert np.max(np.abs(mu - closed)) <= 2e-16 * np.max(np.abs(closed)) * 4


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("rho_sign", [1.0, -1.0])
def test_secular_matches_library_eigvalsh(seed, rho_sign):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 64))
    d = np.sort(rng.uniform(0.0, 5.0, N))
    z = rng.standard_normal(N) / np.sqrt(N)
    rho = rho_sign * rng.uniform(0.1, 3.0)
    defl, org, tau = _roots(d, z, rho)
    assert defl.g.shape[0] == N
    mu = d[org] + tau
    M = np.diag(d) + rho * np.outer(z, z)
    ref = np.linalg.eigvalsh(M)
    assert np.max(np.abs(mu - ref)) <= 1e-14 * np.max(np.abs(ref))
    # trace: sum mu = sum d + rho |z|^2
    assert abs(np.sum(mu) - (np.sum(d) + rho * z @ z)) <= 1e-13 * np.sum(np.abs(d))
    # interlacing
    if rho > 0:
        assert np.all(mu > d) and np.all(mu[:-1] < d[1:])
    else:
        assert np.all(mu < d) and np.all(mu[1:] > d[:-1])


def test_secular_residual_is_at_rounding_level():
    rng = np.random.default_rng(11)
    N = 200
    d = np.sort(rng.uniform(0.0, 1.0, N))
    z = rng.standard_normal(N) / np.sqrt(N)
    for rho in (0.5, -0.5):
        defl, org, tau = _roots(d, z, rho)
        W2 = defl.W ** 2
        delta = (defl.g[None, :] - defl.g[org][:, None]) - tau[:, None]
        f = 1.0 + rho * np.sum(W2[None, :] / delta, axis=1)
        scale = 1.0 + abs(rho) * np.sum(W2[None, :] / np.abs(delta), axis=1)
        assert np.max(np.abs(f) / scale) <= 64 * N * O.U64


def test_secular_resolves_poles_one_part_in_1e11_apart():
    d = np.array([1e-12, 1e-12 * (1 + 2e-11), 1e-6, 0.5, 0.5 * (1 + 2e-11), 1.0])
    z = np.array([0.3, 0.2, 0.1, 0.5, 0.4, 0.2])
    for rho in (1.0, -0.3):
        defl, org, tau = _roots(d, z, rho)
        mu = defl.g[org] + tau
        if rho > 0:
            assert np.all(mu > d) and np.all(mu[:-1] < d[1:])
        else:
            assert np.all(mu < d) and np.all(mu[1:] > d[:-1])


# ---------------------------------------------------------------------------
# Eigenvectors: Loewner weights, C~ orthogonal (equation CTildeFinalForm1),
# and Appendix B's 2x2 worked form.
# ---------------------------------------------------------------------------
def test_loewner_weights_equal_z_on_well_conditioned_data():
    rng = np.random.default_rng(5)
    N = 40
    d = np.arange(N, dtype=float)
    z = rng.uniform(0.5, 1.0, N) * rng.choice([-1, 1], N)
    for rho in (0.8, -0.8):
        defl, org, tau = _roots(d, z, rho)
        what = O.loewner_weights(defl.g, org, tau, rho)
        assert np.max(np.abs(what - np.abs(z)) / np.abs(z)) <= 1e-12


@pytest.mark.parametrize("rho", [0.9, -0.9])
def test_stage_eigvecs_orthogonal_and_eigen_residual(rho):
    rng = np.random.default_rng(7)
    N = 60
    d = np.sort(rng.uniform(0, 2, N))
    d[10] = d[11] = d[12]        # an exactly repeated pole (merge deflation)
    v = rng.standard_normal(N) / np.sqrt(N)
    v[30] = 0.0                  # an exact zero (tiny deflation)
    st = OS.rank_one_update(np.eye(N), d, v, rho)
    C = st.X
    assert np.max(np.abs(C.T @ C - np.eye(N))) <= 1e-14
    M = np.diag(d) + rho * np.outer(v, v)
    R = M @ C - C * st.lam[None, :]
    assert np.max(np.abs(R)) <= 1e-14 * np.max(np.abs(M))
    assert st.flags[30] == 1
    assert sorted(st.flags[10:13].tolist()) == [0, 2, 2]


@pytest.mark.parametrize("rho", [0.9, -0.9])
def test_stage_zero_block_cluster(rho):
    """A block of 30 exactly equal zero poles, as the right-hand eigen-updates
    carry when n > m. One root leaves the block; the other 29 eigenvectors keep
    eigenvalue 0, vanish outside the block's rows and are orthogonal to z on
    them (they span the complement of z within the block)."""
    rng = np.random.default_rng(9)
    N, W = 70, 30
    d = np.sort(np.concatenate([np.zeros(W), rng.uniform(0.5, 2.0, N - W)]))
    v = rng.standard_normal(N) / np.sqrt(N)
    st = OS.rank_one_update(np.eye(N), d, v, rho)
    C = st.X
    assert np.max(np.abs(C.T @ C - np.eye(N))) <= 1e-14
    M = np.diag(d) + rho * np.outer(v, v)
    assert np.max(np.abs(M @ C - C * st.lam[None, :])) <= 1e-14 * np.max(np.abs(M))
    assert np.count_nonzero(st.flags == 2) == W - 1
    zero = st.lam == 0.0
    assert np.count_nonzero(zero) == W - 1
    Cz = C[:, zero]
    assert np.all(Cz[W:, :] == 0.0)
    assert np.max(np.abs(v[:W] @ Cz[:W, :])) <= 1e-15


def test_appendix_b_two_by_two_eigenvector_form():
    """Appendix B: for a 2x2 problem the i-th eigenvector is proportional to
    [a1 / (mu_i - lam_1), a2 / (mu_i - lam_2)]. Worked case: D = diag(1, 2),
    a_bar = (1, 1) / sqrt(2), rho = 1, so B = [[1.5, 0.5], [0.5, 2.5]] with
    eigenvalues 2 -+ sqrt(1/2)."""
    lam = np.array([1.0, 2.0])
    abar = np.array([1.0, 1.0]) / np.sqrt(2.0)
    st = O.rank_one_update(np.eye(2), lam, abar, 1.0)
    mu_closed = np.array([2.0 - np.sqrt(0.5), 2.0 + np.sqrt(0.5)])
    assert np.max(np.abs(st.lam - mu_closed)) <= 4e-16 * 4
    for i in range(2):
        c = abar / (mu_closed[i] - lam)
        c /= np.linalg.norm(c)
        got = st.X[:, i]
        assert min(np.max(np.abs(got - c)), np.max(np.abs(got + c))) <= 1e-15


# ---------------------------------------------------------------------------
# Whole update (Algorithm of Section 6.1)
# ---------------------------------------------------------------------------
def _invariants(P, r):
    Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
    m, n = P.m, P.n
    out = dict(recon=O.recon_error(Ah, r.U, r.sigma, r.V), orthU=O.orth_error(r.U),
               orthV=O.orth_error(r.V))
    # Frobenius identity: |A^|_F^2 = |S|^2 + 2 p^T S q + |a|^2 |b|^2
    p, q = P.U.T @ P.a, P.V.T @ P.b
    fro = np.sum(P.sigma ** 2) + 2 * p @ (P.sigma * q[:m]) + (P.a @ P.a) * (P.b @ P.b)
    out["fro"] = abs(np.sum(r.sigma ** 2) - fro) / fro
    # rank-one interlacing: s^_{i+1} <= s_i and s_{i+1} <= s^_i
    tol = 1e-13 * max(r.sigma[0], P.sigma[0])
    out["interlace"] = bool(np.all(r.sigma[1:] <= P.sigma[:-1] + tol) and
                            np.all(P.sigma[1:] <= r.sigma[:-1] + tol))
    out["null"] = float(np.max(np.abs(Ah @ r.V[:, m:]))) / r.sigma[0] if n > m else 0.0
    return out


CASES = [
    (8, 8, "uniform", {}), (5, 9, "uniform", {}), (1, 1, "uniform", {}), (1, 6, "uniform", {}),
    (33, 33, "geometric", {}), (48, 64, "uniform", {}), (64, 64, "clustered", {}),
    (64, 64, "clustered", dict(zero_frac=0.05, zero_q=True)), (40, 40, "zero", {}),
]


@pytest.mark.parametrize("m,n,kind,kw", CASES)
def test_whole_update_invariants(m, n, kind, kw):
    for seed in range(3):
        P = S.make_problem(m, n, kind, seed=seed, **kw)
        r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
        inv = _invariants(P, r)
        assert inv["recon"] <= 1e-12, inv
        assert inv["orthU"] <= 1e-12 and inv["orthV"] <= 1e-12, inv
        assert inv["fro"] <= 1e-13, inv
        assert inv["interlace"], inv
        assert inv["null"] <= 1e-12, inv


def test_jacobi_svd_matches_library_svd():
    rng = np.random.default_rng(0)
    for (m, n) in [(1, 1), (3, 7), (16, 16), (30, 45)]:
        A = rng.standard_normal((m, n))
        U, s, W = O.jacobi_svd(A)
        ref = np.linalg.svd(A, compute_uv=False)
        assert np.max(np.abs(s - ref)) <= 1e-13 * ref[0]
        assert np.max(np.abs((U * s[None, :]) @ W.T - A)) <= 1e-13 * ref[0]
        assert np.max(np.abs(U.T @ U - np.eye(m))) <= 1e-13


def _align(X, Y):
    s = np.sign(np.sum(X * Y, axis=0))
    s[s == 0] = 1
    return Y * s[None, :]


@pytest.mark.parametrize("m,n,kind", [(12, 12, "uniform"), (20, 31, "uniform"), (64, 64, "geometric"),
                                      (48, 48, "clustered")])
def test_whole_update_matches_jacobi_svd(m, n, kind):
    for seed in range(4):
        P = S.make_problem(m, n, kind, seed=seed)
        r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
        Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
        Uj, sj, Wj = O.jacobi_svd(Ah)
        assert np.max(np.abs(r.sigma - sj)) <= 1e-13 * sj[0]
        # singular vectors are unique up to sign where the values are separated
        gap = np.full(m, np.inf)
        if m > 1:
            dif = np.abs(np.diff(sj))
            gap[:-1] = dif
            gap[1:] = np.minimum(gap[1:], dif)
        ok = (gap / sj[0] >= 1e-4) & (sj / sj[0] >= 1e-6)
        Ua = _align(r.U, Uj)
        Va = _align(r.V[:, :m], Wj)
        assert np.max(np.abs(Ua - r.U)[:, ok]) <= 1e-10
        assert np.max(np.abs(Va - r.V[:, :m])[:, ok]) <= 1e-10


def test_config_one_matches_jacobi_svd():
    """m = n = 256, sigma ~ U[0.1, 10], a, b ~ N(0, 1/n): the oracle agrees with
    the hand-written Jacobi SVD of the explicit A^."""
    P = S.make_problem(256, 256, "uniform", seed=0)
    r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
    Uj, sj, Wj = O.jacobi_svd(Ah)
    assert np.max(np.abs(r.sigma - sj)) <= 1e-13 * sj[0]
    assert O.recon_error(Ah, r.U, r.sigma, r.V) <= 1e-12


# ---------------------------------------------------------------------------
# Special cases with closed-form answers
# ---------------------------------------------------------------------------
def test_zero_update_leaves_factors_unchanged():
    P = S.make_problem(20, 27, "uniform", seed=1)
    for a, b in [(np.zeros(20), P.b), (P.a, np.zeros(27))]:
        r = O.svd_rank1_update(P.U, P.sigma, P.V, a, b)
        assert np.max(np.abs(r.sigma - P.sigma)) <= 1e-14 * P.sigma[0]
        assert np.max(np.abs(np.abs(np.sum(r.U * P.U, axis=0)) - 1)) <= 1e-13


def test_update_along_a_singular_pair_moves_one_value():
    P = S.make_problem(16, 20, "uniform", seed=2)
    k, gam, dlt = 5, 0.7, -1.3
    a, b = gam * P.U[:, k], dlt * P.V[:, k]
    r = O.svd_rank1_update(P.U, P.sigma, P.V, a, b)
    expect = P.sigma.copy()
    expect[k] = abs(P.sigma[k] + gam * dlt)
    expect = np.sort(expect)[::-1]
    assert np.max(np.abs(r.sigma - expect)) <= 1e-14 * expect[0]


def test_zero_sigma_gives_the_outer_product():
    P = S.make_problem(9, 13, "zero", seed=3)
    r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    na, nb = np.linalg.norm(P.a), np.linalg.norm(P.b)
    assert abs(r.sigma[0] - na * nb) <= 1e-15 * na * nb * 4
    assert np.max(np.abs(r.sigma[1:])) <= 1e-15
    s = np.sign(r.U[:, 0] @ P.a)
    assert np.max(np.abs(s * r.U[:, 0] - P.a / na)) <= 1e-14
    assert np.max(np.abs(s * r.V[:, 0] - P.b / nb)) <= 1e-14


def test_one_by_one():
    r = O.svd_rank1_update(np.array([[1.0]]), np.array([2.0]), np.array([[-1.0]]),
                           np.array([0.5]), np.array([3.0]))
    # A = 1 * 2 * (-1) = -2, A^ = -2 + 1.5 = -0.5; the Gram route passes
    # through eigenvalues of size ~|A|^2 = 4, so a few ulps of 4 is the bound.
    assert abs(r.sigma[0] - 0.5) <= 16 * O.U64 * 4
    assert abs(r.U[0, 0] * r.sigma[0] * r.V[0, 0] - (-0.5)) <= 16 * O.U64 * 4


def test_zeroed_projections_preserve_singular_triplets():
    """With p_i = q_i = 0 the update never touches (sigma_i, u_i, v_i): the
    component deflates in all four eigen-updates."""
    P = S.make_problem(64, 64, "clustered", seed=4, zero_frac=0.05, zero_q=True)
    r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    for i in P.meta["zeroed"]:
        j = int(np.argmin(np.abs(r.sigma - P.sigma[i])))
        assert abs(r.sigma[j] - P.sigma[i]) <= 1e-15 * P.sigma[0]
        assert abs(abs(r.U[:, j] @ P.U[:, i]) - 1) <= 1e-13
        for st in r.stages:
            assert st.flags[st.flags == 1].size >= len(P.meta["zeroed"])


# ---------------------------------------------------------------------------
# Deflation threshold and scale (Section 3.1 case (1)): the secular equation
# 1 + rho sum z_k^2 / (d_k - mu) = 0 is unchanged by d -> S d, z -> sqrt(S) z,
# mu -> S mu, so the decisions must be unchanged and the roots exactly scaled.
# S = 2^-600 keeps every quantity normal, so the scaled arithmetic is exact.
# ---------------------------------------------------------------------------
def _scaled_pair():
    rng = np.random.default_rng(600)
    N = 60
    d = np.sort(rng.uniform(0.1, 2.0, N))
    z = rng.standard_normal(N)
    z[[3, 17, 40]] = [1e-17, -3e-18, 2e-16]     # below 8 u sqrt(N) |z| ~ 6.6e-15
    z[[9, 25]] = [1e-13, -2e-13]                # above it
    return d, z


def test_deflation_decisions_and_roots_invariant_under_scaling():
    d, z = _scaled_pair()
    rho = 0.8
    S, sS = 2.0 ** -600, 2.0 ** -300
    r1 = OS.deflate(d, z, rho)
    r2 = OS.deflate(d * S, z * sS, rho)
    assert np.array_equal(r1.tiny, r2.tiny)
    assert np.array_equal(np.nonzero(r1.tiny)[0], [3, 17, 40])
    assert np.array_equal(r1.cluster, r2.cluster)
    o1, t1 = OS.secular_roots(r1.g, r1.W, rho)
    o2, t2 = OS.secular_roots(r2.g, r2.W, rho)
    assert np.array_equal(o1, o2)
    assert np.array_equal(t1 * S, t2)          # bitwise: every step scales exactly
    st1 = OS.rank_one_update_z(np.eye(60), d, z, rho)
    st2 = OS.rank_one_update_z(np.eye(60), d * S, z * sS, rho)
    assert np.array_equal(st1.flags, st2.flags)
    assert np.array_equal(st1.lam * S, st2.lam)


def test_planted_absolute_deflation_threshold_fails(monkeypatch):
    """A threshold that forgets the |z| factor drops every component of the
    scaled problem, which the scale pin catches."""
    import inspect
    src = inspect.getsource(OS.deflate)
    good = "tol = 8.0 * U64 * np.sqrt(max(N, 1)) * znorm"
    assert good in src
    ns = dict(vars(OS))
    exec(src.replace(good, "tol = 8.0 * U64 * np.sqrt(max(N, 1))"), ns)
    monkeypatch.setattr(OS, "deflate", ns["deflate"])
    with pytest.raises(AssertionError):
        test_deflation_decisions_and_roots_invariant_under_scaling()


# ---------------------------------------------------------------------------
# The paper's error measure (Section 7, eq. error) on a hand-computed case.
# ---------------------------------------------------------------------------
def test_paper_error_hand_computed():
    # A^ is 2 x 3; U^ = I, S^ = diag(2, 1), V^ = I, so U^ S^ V^[:, :2]^T =
    # [[2, 0, 0], [0, 1, 0]] and A^ minus it is [[-1, 2, 0], [0, 0, 0]]:
    # max |.| = 2, divided by max sigma^ = 2 gives 1.
    Ah = np.array([[1.0, 2.0, 0.0], [0.0, 1.0, 0.0]])
    assert O.paper_error(Ah, np.eye(2), np.array([2.0, 1.0]), np.eye(3)) == 1.0
    # scaling sigma^ and A^ by 4 leaves the measure unchanged
    assert O.paper_error(4 * Ah, np.eye(2), np.array([8.0, 4.0]), np.eye(3)) == 1.0
    # an exact factorisation gives 0
    assert O.paper_error(np.array([[2.0, 0, 0], [0, 1.0, 0]]), np.eye(2), np.array([2.0, 1.0]), np.eye(3)) == 0.0


# ---------------------------------------------------------------------------
# The paper's Table 2: an upper bound for any correct implementation.
# ---------------------------------------------------------------------------
def test_error_far_below_paper_table_two():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "paper_table2_error.txt"))
            if l.strip() and not l.startswith("#")]
    for n_str, err_str in rows:
        n, paper = int(n_str), float(err_str)
        P, A = S.paper_random_square(n, 1.0, 9.0, seed=n)
        r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
        Ah = A + np.outer(P.a, P.b)
        err = O.paper_error(Ah, r.U, r.sigma, r.V)
        assert err < paper
        assert err <= 1e-13


# ---------------------------------------------------------------------------
# Planted mistakes: each plausible slip in the oracle must fail a pin.
# ---------------------------------------------------------------------------
def _recon_of(P):
    r = OS.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    return O.recon_error(O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b), r.U, r.sigma, r.V)


def test_planted_unpaired_signs_fail(monkeypatch):
    P = S.make_problem(24, 24, "uniform", seed=1)
    r = OS.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b, pair_signs=False)
    assert O.recon_error(O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b), r.U, r.sigma, r.V) > 1e-3


def test_planted_wrong_split_sign_fails(monkeypatch):
    real = OS.gram_split

    def bad(beta):
        rp, rm, Q = real(beta)
        return rp, -rm, Q          # dropped sign of the negative eigenvalue
    monkeypatch.setattr(OS, "gram_split", bad)
    assert _recon_of(S.make_problem(24, 24, "uniform", seed=1)) > 1e-3


def test_planted_root_origin_off_by_one_fails(monkeypatch):
    real = OS.secular_roots

    def bad(g, W, rho, idx=None, chunk=256):
        org, tau = real(g, W, rho, idx, chunk)
        return np.minimum(org + 1, g.shape[0] - 1), tau
    monkeypatch.setattr(OS, "secular_roots", bad)
    with pytest.raises(AssertionError):
        test_secular_matches_library_eigvalsh(0, 1.0)


def test_planted_transposed_projection_fails(monkeypatch):
    real = OS.rank_one_update

    def bad(X, lam, v, rho):
        return real(X.T.copy(), lam, v, rho) if X.shape[0] == X.shape[1] else real(X, lam, v, rho)
    monkeypatch.setattr(OS, "rank_one_update", bad)
    assert _recon_of(S.make_problem(24, 24, "uniform", seed=1)) > 1e-3


def test_planted_dropped_rank_one_term_fails(monkeypatch):
    real = OS.gram_split

    def bad(beta):
        return real(0.0)           # forgets beta a a^T
    monkeypatch.setattr(OS, "gram_split", bad)
    assert _recon_of(S.make_problem(24, 24, "uniform", seed=1)) > 1e-3


def test_planted_missing_column_norm_fails(monkeypatch):
    def bad_norm(*args, **kw):
        C, vals = real_cev(*args, **kw)
        return C * 1.01, vals
    real_cev = OS.cauchy_eigvecs
    monkeypatch.setattr(OS, "cauchy_eigvecs", bad_norm)
    with pytest.raises(AssertionError):
        test_stage_eigvecs_orthogonal_and_eigen_residual(0.9)


def test_planted_householder_column_off_by_one_fails(monkeypatch):
    """The merged cluster's deflated columns taken as reflection columns 0..k-2
    instead of 1..k-1: column 0 is parallel to z, so the zero-block pin fails."""
    import inspect
    src = inspect.getsource(OS.cauchy_eigvecs)
    good = "for t in range(1, mm.shape[0]):"
    assert good in src
    ns = dict(vars(OS))
    exec(src.replace(good, "for t in range(0, mm.shape[0] - 1):"), ns)
    monkeypatch.setattr(OS, "cauchy_eigvecs", ns["cauchy_eigvecs"])
    with pytest.raises(AssertionError):
        test_stage_zero_block_cluster(0.9)



# ---------------------------------------------------------------------------
# Rank-k update (the Conclusion's extension), as k rank-1 updates in order
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,k", [(12, 12, 2), (20, 31, 3), (40, 40, 5)])
def test_rankk_update_matches_jacobi_svd_of_the_sum(m, n, k):
    """Against brute force: the one-sided Jacobi SVD of the explicit
    U S V^T + sum_j a_j b_j^T."""
    P = S.make_problem(m, n, "uniform", seed=m + k)
    rng = np.random.default_rng(m * k)
    A = rng.standard_normal((k, m)) / np.sqrt(n)
    B = rng.standard_normal((k, n)) / np.sqrt(n)
    r = O.svd_rankk_update(P.U, P.sigma, P.V, A, B)
    Ah = (P.U * P.sigma[None, :]) @ P.V[:, :m].T + A.T @ B
    _, sj, _ = O.jacobi_svd(Ah)
    assert np.max(np.abs(r.sigma - sj)) <= 1e-13 * sj[0]
    assert O.recon_error(Ah, r.U, r.sigma, r.V) <= 1e-13
    assert O.orth_error(r.U) <= 1e-13 and O.orth_error(r.V) <= 1e-13


def test_rankk_with_one_pair_is_the_rank1_update():
    P = S.make_problem(16, 20, "uniform", seed=3)
    r1 = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    rk = O.svd_rankk_update(P.U, P.sigma, P.V, P.a[None, :], P.b[None, :])
    assert np.array_equal(r1.sigma, rk.sigma) and np.array_equal(r1.U, rk.U) and np.array_equal(r1.V, rk.V)


def test_planted_rankk_skipping_the_last_pair_fails():
    """A composition that drops one pair misses the Jacobi SVD of the sum."""
    orig = OS.svd_rankk_update

    def dropped(U, sigma, V, A, B):
        return orig(U, sigma, V, A[:-1], B[:-1])
    P = S.make_problem(12, 12, "uniform", seed=5)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((3, 12)) / np.sqrt(12)
    B = rng.standard_normal((3, 12)) / np.sqrt(12)
    Ah = (P.U * P.sigma[None, :]) @ P.V.T + A.T @ B
    _, sj, _ = O.jacobi_svd(Ah)
    r = dropped(P.U, P.sigma, P.V, A, B)
    assert np.max(np.abs(r.sigma - sj)) > 1e-6 * sj[0]
