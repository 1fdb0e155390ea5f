"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances (fp64 everywhere):
  * secular roots: both sides solve to full precision, so the pole-relative
    offsets agree to |tau_gpu - tau_oracle| <= 64 K u |tau| + 4 u |mu|;
  * eigenvalues / singular values: |d sigma_i| <= 1e-13 sigma_max;
  * vectors: sign-aligned columns agree to 1e-9 where the eigenvalue gap is
    at least 1e-4 of the largest eigenvalue (elsewhere only invariants);
  * reconstruction |U^ S^ V^^T - A^|_F / |A^|_F <= 1e-12, orthogonality
    max |Q^T Q - I| <= 1e-12;
  * deflation flags: bit-exact (both sides decide in fp64 on the same rule),
    except which member of an exactly repeated pole group stays live.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _align_cols(ref, got):
    s = np.sign(np.sum(ref * got, axis=0))
    s[s == 0] = 1.0
    return got * s[None, :]


def _separated(vals, rel=1e-4):
    v = np.asarray(vals)
    gap = np.full(v.shape[0], np.inf)
    if v.shape[0] > 1:
        d = np.abs(np.diff(v))
        gap[:-1] = d
        gap[1:] = np.minimum(gap[1:], d)
    return gap >= rel * max(np.max(np.abs(v)), 1e-300)


def _flags_match(fg, fo, lam):
    """Deflation flags agree; among exactly equal poles which member stays live
    is a free choice, so such groups are compared as multisets."""
    fg, fo, lam = np.asarray(fg), np.asarray(fo), np.asarray(lam)
    for v in np.unique(lam):
        grp = lam == v
        if np.sum(grp) == 1:
            if fg[grp][0] != fo[grp][0]:
                return False
        elif sorted(fg[grp].tolist()) != sorted(fo[grp].tolist()):
            return False
    return True


# ---------------------------------------------------------------------------
# secular roots
# ---------------------------------------------------------------------------
def _secular_case(K, rho, kind, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        d = np.sort(rng.uniform(0.0, 5.0, K))
    elif kind == "geometric":
        d = np.sort(10.0 ** (-12.0 * np.arange(K) / K))
    else:  # close pairs one part in 1e11 apart
        base = np.sort(rng.uniform(0.1, 1.0, (K + 1) // 2))
        d = np.sort(np.concatenate([base, base * (1 + 2e-11)]))[:K]
    z = rng.standard_normal(K) / np.sqrt(K)
    return d, z, rho


@pytest.mark.parametrize("K", [1, 2, 3, 17, 64, 65, 257, 1000])
@pytest.mark.parametrize("rho", [0.8, -0.8])
@pytest.mark.parametrize("kind", ["uniform", "geometric", "pairs"])
def test_secular_roots_match_oracle(lib, K, rho, kind):
    d, z, rho = _secular_case(K, rho, kind, seed=K)
    org_g, tau_g, its = lib.secular(dev(d), dev(z), rho)
    org_g, tau_g = host(org_g).astype(np.int64), host(tau_g)
    defl = O.deflate(d, z, rho)
    assert defl.g.shape[0] == K
    org_o, tau_o = O.secular_roots(defl.g, defl.W, rho)
    mu_g = d[org_g] + tau_g
    mu_o = d[org_o] + tau_o
    # both roots lie in the same interval and agree to the stated bound
    same = org_g == org_o
    tol = 64 * K * U64 * np.abs(tau_o) + 4 * U64 * np.abs(mu_o)
    assert np.all(np.abs(tau_g - tau_o)[same] <= tol[same])
    assert np.all(np.abs(mu_g - mu_o)[~same] <= 4 * U64 * np.abs(mu_o)[~same] + 64 * K * U64 * np.abs(tau_o)[~same])
    assert int(host(its).max()) < 60


def test_secular_full_size_sampled_roots(lib):
    """8192 poles from the headline spectrum (sigma^2, sigma ~ U[1e-3, 1]); the
    oracle bisects 96 sampled roots one by one."""
    K = 8192
    rng = np.random.default_rng(8192)
    d = np.sort(rng.uniform(1e-3, 1.0, K) ** 2)
    z = rng.standard_normal(K) / np.sqrt(K)
    for rho in (2.6, -0.38):
        org_g, tau_g, its = lib.secular(dev(d), dev(z), rho)
        org_g, tau_g = host(org_g).astype(np.int64), host(tau_g)
        idx = np.unique(np.concatenate([[0, 1, K - 2, K - 1], rng.choice(K, 92, replace=False)]))
        org_o, tau_o = O.secular_roots(d, np.abs(z), rho, idx=idx)
        assert np.all(org_g[idx] == org_o)
        tol = 64 * K * U64 * np.abs(tau_o) + 4 * U64 * np.abs(d[org_o] + tau_o)
        assert np.all(np.abs(tau_g[idx] - tau_o) <= tol)


# Power-of-two scales that put every pole difference below 2^-1000, the range
# where the kernels' fast reciprocal gives way to the exact one (and the column
# norms to their scaled form). Scaling poles by S and z by sqrt(S) is exact and
# scales every root by S, so the unscaled oracle stays the reference.
TINY_S, TINY_R = 2.0 ** -1004, 2.0 ** -502


def _spaced_poles(K, hi, rng):
    """Poles at least hi / (2K) apart, so that the scaled gaps stay normal numbers."""
    return (np.arange(K) + 0.5 * rng.uniform(size=K)) * hi / K


@pytest.mark.parametrize("K", [64, 1000, 2100])
@pytest.mark.parametrize("rho", [0.8, -0.8])
def test_secular_roots_below_reciprocal_range(lib, K, rho):
    """One root per lane (K <= 2048) and one per wave (K = 2100) on the
    exact-reciprocal path: roots equal 2^-1004 times the oracle's roots of the
    unscaled problem."""
    rng = np.random.default_rng(K + 7)
    d = _spaced_poles(K, 5.0, rng)
    z = rng.choice([-1.0, 1.0], K) * rng.uniform(0.5, 1.5, K) / np.sqrt(K)
    org_g, tau_g, its = lib.secular(dev(d * TINY_S), dev(z * TINY_R), rho)
    org_g, tau_g = host(org_g).astype(np.int64), host(tau_g) / TINY_S
    defl = O.deflate(d, z, rho)
    assert defl.g.shape[0] == K
    org_o, tau_o = O.secular_roots(defl.g, defl.W, rho)
    mu_g, mu_o = d[org_g] + tau_g, d[org_o] + tau_o
    same = org_g == org_o
    tol = 64 * K * U64 * np.abs(tau_o) + 4 * U64 * np.abs(mu_o)
    assert np.all(np.abs(tau_g - tau_o)[same] <= tol[same])
    assert np.all(np.abs(mu_g - mu_o)[~same] <= tol[~same])
    assert int(host(its).max()) < 60


# ---------------------------------------------------------------------------
# one eigen-update
# ---------------------------------------------------------------------------
def _eig_case(R, N, rho, seed, repeat=False, zeros=False):
    rng = np.random.default_rng(seed)
    lam = np.sort(rng.uniform(0.0, 3.0, N))
    z = rng.standard_normal(N) / np.sqrt(N)
    if repeat and N >= 8:
        lam[3:6] = lam[3]                  # three exactly equal poles
        lam[:2] = 0.0                      # and a zero pair
        lam = np.sort(lam)
    if zeros and N >= 8:
        z[[1, N // 2, N - 1]] = 0.0
    X = rng.standard_normal((R, N))
    return X, lam, z, rho


@pytest.mark.parametrize("R,N", [(1, 1), (5, 3), (64, 64), (130, 129), (300, 257), (128, 384)])
@pytest.mark.parametrize("rho", [0.9, -0.6])
@pytest.mark.parametrize("variant", ["plain", "repeat", "zeros"])
def test_eig_update_matches_oracle(lib, R, N, rho, variant):
    X, lam, z, rho = _eig_case(R, N, rho, seed=R * 1000 + N, repeat=variant == "repeat",
                               zeros=variant == "zeros")
    Xo, lo, fl = lib.eig_update(dev(X), dev(lam), dev(z), rho)
    Xo, lo, fl = host(Xo), host(lo), host(fl)
    st = O.rank_one_update_z(X, lam, z, rho)
    assert np.array_equal(fl, st.flags)
    scale = max(np.max(np.abs(lam)), 1.0)
    assert np.max(np.abs(lo - st.lam)) <= 1e-13 * scale
    # C~ of the GPU, recovered through the product with an identity block
    Ci, lci, _ = lib.eig_update(dev(np.eye(N)), dev(lam), dev(z), rho)
    Ci = host(Ci)
    assert np.max(np.abs(Ci.T @ Ci - np.eye(N))) <= 1e-13
    M = np.diag(lam) + rho * np.outer(z, z)
    assert np.max(np.abs(M @ Ci - Ci * host(lci)[None, :])) <= 1e-13 * np.max(np.abs(M))
    # the product itself: X C~ against X times the oracle's C~, column by column
    ok = _separated(st.lam)
    Xa = _align_cols(st.X, Xo)
    err = np.max(np.abs(Xa - st.X)[:, ok]) if np.any(ok) else 0.0
    assert err <= 1e-9 * max(1.0, np.max(np.abs(X)))
    # the product is exactly X times the GPU's own C~ (same kernels) to rounding
    assert np.max(np.abs(Xo - X @ Ci)) <= 1e-12 * max(1.0, np.max(np.abs(X))) * np.sqrt(N)


@pytest.mark.parametrize("R,N", [(64, 300), (40, 2100)])
@pytest.mark.parametrize("rho", [0.9, -0.6])
def test_eig_update_below_reciprocal_range(lib, R, N, rho):
    """Poles scaled by 2^-1004 and z by 2^-502: the secular sums, Loewner
    weights, column norms (scaled form) and product tiles (general entry) all
    meet differences below 2^-1000. Eigenvalues are 2^-1004 times the oracle's
    on the unscaled problem; eigenvector products are the same."""
    rng = np.random.default_rng(N + 11)
    lam = _spaced_poles(N, 3.0, rng)
    z = rng.standard_normal(N) / np.sqrt(N)
    X = rng.standard_normal((R, N))
    Xo, lo, fl = lib.eig_update(dev(X), dev(lam * TINY_S), dev(z * TINY_R), rho)
    Xo, lo, fl = host(Xo), host(lo) / TINY_S, host(fl)
    st = O.rank_one_update_z(X, lam, z, rho)
    assert np.array_equal(fl, st.flags)
    assert np.max(np.abs(lo - st.lam)) <= 1e-13 * np.max(np.abs(lam))
    ok = _separated(st.lam)
    Xa = _align_cols(st.X, Xo)
    assert np.any(ok)
    assert np.max(np.abs(Xa - st.X)[:, ok]) <= 1e-9 * np.max(np.abs(X))


@pytest.mark.parametrize("shape", [-1, 3])
@pytest.mark.parametrize("rho", [0.9, -0.6])
def test_eig_update_wide_cluster_copy_columns(lib, shape, rho):
    """1200 equal poles: 1199 deflated columns of one Householder reflection.
    Whole 64-column chunks of them are written as copies plus the reflection,
    without MFMA work (with the 64 x 64 tile the member rows pass through LDS
    in two chunks). C~ recovered from the identity must be orthogonal with the
    new eigenvalues on its diagonal, X C~ must equal X times it, and on
    separated eigenvalues X times the oracle's C~."""
    R, N, W = 200, 1500, 1200
    rng = np.random.default_rng(31)
    lam = np.sort(np.concatenate([np.zeros(W), rng.uniform(0.5, 3.0, N - W)]))
    z = rng.standard_normal(N) / np.sqrt(N)
    X = rng.standard_normal((R, N))
    old = lib.set_option(lib.SVDU_OPT_TILE_SHAPE, shape)
    try:
        Xo, lo, fl = lib.eig_update(dev(X), dev(lam), dev(z), rho)
        Ci, lci, _ = lib.eig_update(dev(np.eye(N)), dev(lam), dev(z), rho)
    finally:
        lib.set_option(lib.SVDU_OPT_TILE_SHAPE, old)
    Xo, lo, fl, Ci, lci = host(Xo), host(lo), host(fl), host(Ci), host(lci)
    st = O.rank_one_update_z(X, lam, z, rho)
    assert np.count_nonzero(st.flags == 2) == W - 1
    assert np.array_equal(fl, st.flags)
    assert np.max(np.abs(lo - st.lam)) <= 1e-13 * 3.0
    assert np.max(np.abs(Ci.T @ Ci - np.eye(N))) <= 1e-13
    M = np.diag(lam) + rho * np.outer(z, z)
    assert np.max(np.abs(M @ Ci - Ci * lci[None, :])) <= 1e-13 * np.max(np.abs(M))
    assert np.max(np.abs(Xo - X @ Ci)) <= 1e-12 * np.max(np.abs(X)) * np.sqrt(N)
    ok = _separated(st.lam)
    assert np.any(ok)
    Xa = _align_cols(st.X, Xo)
    assert np.max(np.abs(Xa - st.X)[:, ok]) <= 1e-9 * np.max(np.abs(X))


# ---------------------------------------------------------------------------
# the whole update
# ---------------------------------------------------------------------------
UPDATE_CASES = [
    (1, 1, "uniform", {}), (1, 5, "uniform", {}), (3, 3, "uniform", {}), (16, 16, "uniform", {}),
    (100, 173, "uniform", {}), (256, 256, "uniform", {}), (300, 457, "uniform", {}),
    (512, 512, "geometric", {}), (512, 512, "clustered", dict(zero_frac=0.05)),
    (512, 512, "clustered", dict(zero_frac=0.05, zero_q=True)), (40, 40, "zero", {}), (129, 130, "uniform", {}),
]


def _gpu_update(lib, P, **kw):
    Uo, so, Vo, defl = lib.rank1_update(dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b), **kw)
    return host(Uo), host(so), host(Vo), host(defl)


@pytest.mark.parametrize("m,n,kind,kw", UPDATE_CASES)
def test_rank1_update_matches_oracle(lib, m, n, kind, kw):
    for seed in (0, 1):
        P = S.make_problem(m, n, kind, seed=seed, **kw)
        Ug, sg, Vg, fg = _gpu_update(lib, P)
        r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
        Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
        smax = max(r.sigma[0], 1e-300)
        assert np.max(np.abs(sg - r.sigma)) <= 1e-13 * smax
        assert O.recon_error(Ah, Ug, sg, Vg) <= 1e-12
        assert O.orth_error(Ug) <= 1e-12 and O.orth_error(Vg) <= 1e-12
        if n > m:
            assert np.max(np.abs(Ah @ Vg[:, m:])) <= 1e-12 * smax
        lam_in = [P.sigma ** 2, r.stages[0].lam, np.concatenate([P.sigma ** 2, np.zeros(n - m)]),
                  r.stages[2].lam]
        for k, st in enumerate(r.stages):
            assert _flags_match(fg[k, :st.flags.shape[0]], st.flags, lam_in[k]), k
        ok = _separated(r.sigma ** 2) & (r.sigma >= 1e-6 * smax)
        Ua = _align_cols(r.U, Ug)
        assert np.max(np.abs(Ua - r.U)[:, ok], initial=0.0) <= 1e-9
        # V^ carries the same signs as U^ (pairing), so align it with U's signs
        su = np.sign(np.sum(r.U * Ug, axis=0))
        Va = Vg[:, :m] * su[None, :]
        assert np.max(np.abs(Va - r.V[:, :m])[:, ok], initial=0.0) <= 1e-9


def test_rank1_update_preserves_zeroed_triplets(lib):
    P = S.make_problem(512, 512, "clustered", seed=3, zero_frac=0.05, zero_q=True)
    Ug, sg, Vg, fg = _gpu_update(lib, P)
    for i in P.meta["zeroed"]:
        j = int(np.argmin(np.abs(sg - P.sigma[i])))
        assert abs(sg[j] - P.sigma[i]) <= 1e-15 * P.sigma[0]
        assert abs(abs(Ug[:, j] @ P.U[:, i]) - 1) <= 1e-13
        assert abs(abs(Vg[:, j] @ P.V[:, i]) - 1) <= 1e-13
    assert np.all(np.sum(fg == 1, axis=1) >= len(P.meta["zeroed"]))


def _full_size_checks(m, n, Ug, sg, Vg, U, sig, V, a, b):
    """Invariants at any size, computed with plain torch fp64 on the device."""
    Ah = (U * sig[None, :]) @ V[:, :m].T + torch.outer(a, b)
    R = (Ug * sg[None, :]) @ Vg[:, :m].T - Ah
    recon = (torch.linalg.norm(R) / torch.linalg.norm(Ah)).item()
    I_m = torch.eye(m, dtype=torch.float64, device=Ug.device)
    orthU = torch.max(torch.abs(Ug.T @ Ug - I_m)).item()
    I_n = torch.eye(n, dtype=torch.float64, device=Ug.device)
    orthV = torch.max(torch.abs(Vg.T @ Vg - I_n)).item()
    p, q = U.T @ a, V.T @ b
    fro = (torch.sum(sig ** 2) + 2 * p @ (sig * q[:m]) + (a @ a) * (b @ b)).item()
    fro_err = abs(torch.sum(sg ** 2).item() - fro) / fro
    tol = 1e-13 * max(sg[0].item(), sig[0].item())
    inter = bool(torch.all(sg[1:] <= sig[:-1] + tol).item() and torch.all(sig[1:] <= sg[:-1] + tol).item())
    return recon, orthU, orthV, fro_err, inter


@pytest.mark.parametrize("m,n,kind", [(4096, 4096, "geometric"), (4096, 8192, "uniform01"),
                                      (8192, 8192, "uniform01")])
def test_rank1_update_full_size_invariants(lib, m, n, kind):
    """Headline sizes in the launch configuration the benchmark times."""
    torch.manual_seed(0)
    U = S.haar_torch(m, seed=11, device="cuda")
    V = S.haar_torch(n, seed=12, device="cuda")
    rng = np.random.default_rng(13)
    if kind == "geometric":
        sig = S.sigma_geometric(m)
    else:
        sig = S.sigma_uniform(m, 1e-3, 1.0, rng)
    a = rng.standard_normal(m) / np.sqrt(n)
    b = rng.standard_normal(n) / np.sqrt(n)
    sig_t, a_t, b_t = dev(sig), dev(a), dev(b)
    Ug, sg, Vg, _ = lib.rank1_update(U, sig_t, V, a_t, b_t)
    recon, orthU, orthV, fro_err, inter = _full_size_checks(m, n, Ug, sg, Vg, U, sig_t, V, a_t, b_t)
    assert recon <= 1e-12, recon
    assert orthU <= 1e-12 and orthV <= 1e-12, (orthU, orthV)
    assert fro_err <= 1e-12, fro_err
    assert inter


# ---------------------------------------------------------------------------
# device status, determinism, streams
# ---------------------------------------------------------------------------
def test_device_status_codes(lib):
    P = S.make_problem(32, 40, "uniform", seed=5)
    a = P.a.copy()
    a[3] = np.nan
    with pytest.raises(lib.SvduError) as e:
        lib.rank1_update(dev(P.U), dev(P.sigma), dev(P.V), dev(a), dev(P.b))
    assert e.value.code == lib.SVDU_ENONFINITE
    s = P.sigma.copy()
    s[[4, 5]] = s[[5, 4]]
    with pytest.raises(lib.SvduError) as e:
        lib.rank1_update(dev(P.U), dev(s), dev(P.V), dev(P.a), dev(P.b))
    assert e.value.code == lib.SVDU_EBADSIGMA
    old = lib.set_option(lib.SVDU_OPT_SECULAR_MAXIT, 1)
    try:
        with pytest.raises(lib.SvduError) as e:
            lib.rank1_update(dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))
        assert e.value.code == lib.SVDU_ENOCONV
    finally:
        lib.set_option(lib.SVDU_OPT_SECULAR_MAXIT, old)
    lib.rank1_update(dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))   # clean again


def test_bitwise_deterministic_and_stream_ordered(lib):
    P = S.make_problem(300, 457, "uniform", seed=9)
    r1 = lib.rank1_update(dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        U, sg, V, a, b = dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)
        r2 = lib.rank1_update(U, sg, V, a, b, stream=s)
    s.synchronize()
    for x, y in zip(r1, r2):
        assert torch.equal(x, y)


# ---------------------------------------------------------------------------
# precision form (split FP32 products): same roots, flags and sigma as FP64;
# vectors within the FP32-accumulation error
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("m,n,kind", [(256, 256, "uniform"), (300, 457, "uniform"), (512, 512, "geometric")])
def test_split32_negative_result_keeps_roots_and_reports_its_error(lib, m, n, kind):
    """The split-FP32 form, kept as a measured negative result: it cannot meet
    the precision form's 1e-10 bound (its FP32 accumulation floors at about
    1e-7), so this checks what it delivers. The precision form that meets the
    bound, the exact-slice INT8 form, is tested at 1e-10 in test_gpu_int8.py."""
    P = S.make_problem(m, n, kind, seed=4)
    args = (dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b))
    U64_, s64, V64, f64 = lib.rank1_update(*args)
    U32, s32, V32, f32 = lib.rank1_update(*args, precision=lib.SVDU_PREC_SPLIT32)
    assert torch.equal(s64, s32)            # no form touches roots ...
    assert torch.equal(f64, f32)            # ... or deflation decisions
    Ug, Vg, sg = host(U32), host(V32), host(s32)
    Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
    recon = O.recon_error(Ah, Ug, sg, Vg)
    orth = max(O.orth_error(Ug), O.orth_error(Vg))
    # FP32 accumulation limits this form to about 1e-7 (the 1e-10 target is not
    # reachable this way); the bound checked here is what it delivers
    assert recon <= 5e-6 and orth <= 5e-6, (recon, orth)
    assert np.max(np.abs(np.linalg.norm(Ug, axis=0) - 1)) <= 1e-14   # the FP64 renormalisation sweep
    print(f"split32 m={m} n={n} {kind}: recon {recon:.2e} orth {orth:.2e}")


# ---------------------------------------------------------------------------
# FMM path of the product: matches the direct sum (the definition, here the
# oracle's dense X C~) to <= 1e-9 at eps = 1e-10
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("N,kind", [(2, "uniform"), (5, "uniform"), (17, "geometric"), (33, "uniform"),
                                    (257, "uniform"), (1000, "geometric"), (1000, "uniform"), (3000, "geometric")])
@pytest.mark.parametrize("rho", [0.9, -0.6])
@pytest.mark.parametrize("variant", ["plain", "repeat_zeros", "isolated_top", "isolated_bottom"])
def test_fmm_product_matches_direct_sum(lib, N, kind, rho, variant):
    rng = np.random.default_rng(N)
    R = 200
    lam = np.sort(rng.uniform(0, 3, N)) if kind == "uniform" else np.sort(10.0 ** (-12.0 * rng.uniform(0, 1, N)))
    z = rng.standard_normal(N) / np.sqrt(N)
    if variant == "repeat_zeros":
        a = min(5, N - 1)
        lam[a:a + 4] = lam[a]
        lam = np.sort(lam)
        z[[min(2, N - 1), N // 3]] = 0.0
    elif variant == "isolated_top":        # one pole far above the others, as a level's extreme root
        lam[-1] = lam[-1] + 2.0 * (lam[-1] - lam[0])
    elif variant == "isolated_bottom":
        lam[0] = lam[0] - 2.0 * (lam[-1] - lam[0])
    X = rng.standard_normal((R, N))
    Xf, lf, ff = lib.eig_update(dev(X), dev(lam), dev(z), rho, path=lib.SVDU_PATH_FMM, eps=1e-10)
    Xd, ld, fd = lib.eig_update(dev(X), dev(lam), dev(z), rho)
    assert torch.equal(lf, ld) and torch.equal(ff, fd)      # same roots and deflation as the direct path
    st = O.rank_one_update_z(X, lam, z, rho)                  # oracle: dense C~ and matmul
    scale = np.max(np.abs(st.X))
    err_oracle = np.max(np.abs(_align_cols(st.X, host(Xf)) - st.X)[:, _separated(st.lam)], initial=0.0)
    err_direct = np.max(np.abs(host(Xf) - host(Xd)))
    assert err_direct <= 1e-9 * scale, err_direct
    assert err_oracle <= 1e-9 * scale, err_oracle


@pytest.mark.parametrize("m,n,kind,kw", [(300, 457, "uniform", {}), (512, 512, "clustered",
                                                                      dict(zero_frac=0.05, zero_q=True)),
                                         (4096, 4096, "geometric", {}), (8192, 8192, "uniform01", {})])
def test_fmm_update_matches_direct_update(lib, m, n, kind, kw):
    """Direct vs FMM at eps = 1e-10 on the whole update (the geometric 4096 case
    is the direct-vs-FMM workload; 8192 with sigma ~ U[1e-3, 1] is the benchmark's,
    whose second level has an isolated extreme pole)."""
    if m >= 4096:
        U = S.haar_torch(m, seed=21, device="cuda")
        V = S.haar_torch(n, seed=22, device="cuda")
        rng = np.random.default_rng(23)
        sig = dev(S.sigma_geometric(m) if kind == "geometric" else S.sigma_uniform(m, 1e-3, 1.0, rng))
        a, b = dev(rng.standard_normal(m) / np.sqrt(n)), dev(rng.standard_normal(n) / np.sqrt(n))
    else:
        P = S.make_problem(m, n, kind, seed=7, **kw)
        U, sig, V, a, b = dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)
    Ud, sd, Vd, fd = lib.rank1_update(U, sig, V, a, b)
    Uf, sf, Vf, ff = lib.rank1_update(U, sig, V, a, b, path=lib.SVDU_PATH_FMM, eps=1e-10)
    assert torch.equal(sd, sf) and torch.equal(fd, ff)
    assert (Uf - Ud).abs().max().item() <= 1e-9
    assert (Vf - Vd).abs().max().item() <= 1e-9
    recon, orthU, orthV, fro_err, inter = _full_size_checks(m, n, Uf, sf, Vf, U, sig, V, a, b)
    assert recon <= 1e-9 and orthU <= 1e-9 and orthV <= 1e-9, (recon, orthU, orthV)
