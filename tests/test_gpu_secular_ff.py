"""GPU parity of the far-field form of the secular solve (SVDU_OPT_SECULAR_FMM).

Each leaf of 64 consecutive poles takes the sums over poles at least one leaf
width away from Chebyshev interpolants at 32 points sampled once per
eigen-update; the iterates sum the near poles directly, and the extreme root
beyond the last pole takes the direct sums. The interpolants' error is at
rounding level (tests/test_secular_farfield_cpu.py), so the roots are held to
the bound of the direct form against the oracle:
  |tau_gpu - tau_oracle| <= 64 K u |tau| + 4 u |mu|   (same origin pole),
and whole updates to the bounds of tests/test_gpu_parity.py.

Contexts: `ffctx` takes the far field at every order (mode 2), so that small
orders and leaf edges are tested; `dctx` the direct sums (mode 0); the default
(mode 1) takes the far field above order 2048 only.
"""
import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def host(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def ffctx(lib):
    ctx = lib.Context()
    ctx.set_option(lib.SVDU_OPT_SECULAR_FMM, 2)
    yield ctx
    ctx.close()


@pytest.fixture(scope="module")
def dctx(lib):
    ctx = lib.Context()
    ctx.set_option(lib.SVDU_OPT_SECULAR_FMM, 0)
    yield ctx
    ctx.close()


def _poles(K, kind, rng):
    if kind == "uniform":
        return np.sort(rng.uniform(0.0, 5.0, K))
    if kind == "geometric":
        return np.sort(10.0 ** (-12.0 * np.arange(K) / K))
    if kind == "pairs":     # close pairs one part in 1e11 apart
        base = np.sort(rng.uniform(0.1, 1.0, (K + 1) // 2))
        return np.sort(np.concatenate([base, base * (1 + 2e-11)]))[:K]
    if kind == "top_outlier":
        # the spectrum after an update with rho > 0: the top pole far above the
        # rest (with rho < 0 the reflected problem sees it as its first pole)
        d = np.sort(rng.uniform(0.0, 1.0, K))
        d[-1] = 4.0
        return d
    # a tight cluster of most poles inside a wide spread: near ranges of the
    # cluster's neighbours cover most poles
    nc = (3 * K) // 4
    cl = 1.0 + 1e-9 * (np.arange(nc) + 0.5 * rng.uniform(0.0, 1.0, nc)) / max(nc, 1)   # distinct doubles
    return np.sort(np.concatenate([cl, rng.uniform(0.0, 10.0, K - nc)]))


def _check_roots(d, z, rho, org_g, tau_g):
    K = d.shape[0]
    org_g, tau_g = host(org_g).astype(np.int64), host(tau_g)
    defl = O.deflate(d, z, rho)
    assert defl.g.shape[0] == K
    org_o, tau_o = O.secular_roots(defl.g, defl.W, rho)
    mu_g, mu_o = d[org_g] + tau_g, d[org_o] + tau_o
    same = org_g == org_o
    tol = 64 * K * U64 * np.abs(tau_o) + 4 * U64 * np.abs(mu_o)
    assert np.all(np.abs(tau_g - tau_o)[same] <= tol[same])
    assert np.all(np.abs(mu_g - mu_o)[~same] <= tol[~same])


@pytest.mark.parametrize("K", [1, 2, 63, 64, 65, 200, 1000, 3000])
@pytest.mark.parametrize("rho", [0.8, -0.8])
@pytest.mark.parametrize("kind", ["uniform", "geometric", "pairs", "cluster", "top_outlier"])
def test_far_field_roots_match_oracle(lib, ffctx, K, rho, kind):
    rng = np.random.default_rng(K + 100)
    d = _poles(K, kind, rng)
    z = rng.standard_normal(K) / np.sqrt(K)
    org_g, tau_g, its = lib.secular(dev(d), dev(z), rho, ctx=ffctx)
    _check_roots(d, z, rho, org_g, tau_g)
    assert int(host(its).max()) < 60


@pytest.mark.parametrize("rho", [1e6, -1e6])
def test_far_field_wide_last_leaf(lib, ffctx, rho):
    """A large |rho| puts the extreme root far beyond the poles: the last
    leaf's interval then spans them all and its roots sum everything directly."""
    K = 700
    rng = np.random.default_rng(7)
    d = np.sort(rng.uniform(0.0, 1.0, K))
    z = rng.standard_normal(K) / np.sqrt(K)
    org_g, tau_g, _ = lib.secular(dev(d), dev(z), rho, ctx=ffctx)
    _check_roots(d, z, rho, org_g, tau_g)


@pytest.mark.parametrize("K", [64, 1000, 2100])
def test_far_field_scaled_units(lib, ffctx, K):
    """Poles scaled by 2^-1004 (the secular iteration's scaled units and the
    exact reciprocals): roots equal 2^-1004 times the unscaled oracle's."""
    s, r = 2.0 ** -1004, 2.0 ** -502
    rng = np.random.default_rng(K + 7)
    d = (np.arange(K) + 0.5 * rng.uniform(size=K)) * 5.0 / K
    z = rng.choice([-1.0, 1.0], K) * rng.uniform(0.5, 1.5, K) / np.sqrt(K)
    for rho in (0.8, -0.8):
        org_g, tau_g, _ = lib.secular(dev(d * s), dev(z * r), rho, ctx=ffctx)
        _check_roots(d, z, rho, org_g, tau_g / s)


def test_far_field_full_size_sampled_roots(lib, dctx):
    """8192 poles of the headline spectrum (the default context takes the far
    field at this order): 96 sampled roots against the oracle, and every root
    against the direct sums."""
    K = 8192
    rng = np.random.default_rng(8192)
    d = np.sort(rng.uniform(1e-3, 1.0, K) ** 2)
    z = rng.standard_normal(K) / np.sqrt(K)
    for rho in (2.6, -0.38):
        org_f, tau_f, its_f = lib.secular(dev(d), dev(z), rho)
        org_d, tau_d, its_d = lib.secular(dev(d), dev(z), rho, ctx=dctx)
        org_f, tau_f = host(org_f).astype(np.int64), host(tau_f)
        org_d, tau_d = host(org_d).astype(np.int64), host(tau_d)
        idx = np.unique(np.concatenate([[0, 1, K - 2, K - 1], rng.choice(K, 92, replace=False)]))
        org_o, tau_o = O.secular_roots(d, np.abs(z), rho, idx=idx)
        assert np.all(org_f[idx] == org_o)
        tol = 64 * K * U64 * np.abs(tau_o) + 4 * U64 * np.abs(d[org_o] + tau_o)
        assert np.all(np.abs(tau_f[idx] - tau_o) <= tol)
        # all roots: the same origins and offsets to a few units of rounding
        assert np.array_equal(org_f, org_d)
        assert np.all(np.abs(tau_f - tau_d) <= 64 * U64 * (np.abs(tau_d) + np.abs(d[org_d])))
        assert abs(float(host(its_f).mean()) - float(host(its_d).mean())) < 0.5


def _separated(vals, rel=1e-4):
    v = np.asarray(vals)
    gap = np.full(v.shape[0], np.inf)
    d = np.abs(np.diff(v))
    gap[:-1] = d
    gap[1:] = np.minimum(gap[1:], d)
    return gap >= rel * max(np.max(np.abs(v)), 1e-300)


@pytest.mark.parametrize("m,n,kind,kw", [(300, 300, "uniform", {}), (512, 700, "geometric", {}),
                                         (513, 513, "clustered", dict(zero_frac=0.05, zero_q=True))])
@pytest.mark.parametrize("path", ["direct", "fmm"])
def test_far_field_update_matches_oracle(lib, ffctx, m, n, kind, kw, path):
    P = S.make_problem(m, n, kind, seed=m + n, **kw)
    p = lib.SVDU_PATH_FMM if path == "fmm" else lib.SVDU_PATH_DIRECT
    Ug, sg, Vg, fg = lib.rank1_update(dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b), path=p,
                                      ctx=ffctx)
    Ug, sg, Vg = host(Ug), host(sg), host(Vg)
    r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
    smax = max(r.sigma[0], 1e-300)
    assert np.max(np.abs(sg - r.sigma)) <= 1e-13 * smax
    assert O.recon_error(Ah, Ug, sg, Vg) <= 1e-12
    assert O.orth_error(Ug) <= 1e-12 and O.orth_error(Vg) <= 1e-12
    ok = _separated(r.sigma ** 2) & (r.sigma >= 1e-6 * smax)
    su = np.sign(np.sum(r.U * Ug, axis=0))
    su[su == 0] = 1.0
    assert np.max(np.abs(Ug * su[None, :] - r.U)[:, ok], initial=0.0) <= 1e-9
    assert np.max(np.abs(Vg[:, :m] * su[None, :] - r.V[:, :m])[:, ok], initial=0.0) <= 1e-9


@pytest.mark.parametrize("K", [700, 2048, 2049, 3000])
def test_default_mode_splits_at_order_2048(lib, ffctx, dctx, K):
    """The default takes the direct sums up to order 2048 and the far field
    above it: bitwise equal to mode 0 below, to mode 2 above."""
    rng = np.random.default_rng(K)
    d, z = dev(np.sort(rng.uniform(0.0, 3.0, K))), dev(rng.standard_normal(K) / np.sqrt(K))
    o1, t1, _ = lib.secular(d, z, 0.7)
    o0, t0, _ = lib.secular(d, z, 0.7, ctx=dctx)
    o2, t2, _ = lib.secular(d, z, 0.7, ctx=ffctx)
    ref = (o0, t0) if K <= 2048 else (o2, t2)
    assert torch.equal(o1, ref[0]) and torch.equal(t1, ref[1])


def test_far_field_update_8192_against_direct_sums(lib, dctx):
    """The headline workload: the far-field form (the default at this order)
    against the direct sums of the same path, on the device (the oracle
    comparison at this size is in tests/test_gpu_configs.py)."""
    m = n = 8192
    U = S.haar_torch(m, seed=71, device="cuda")
    V = S.haar_torch(n, seed=72, device="cuda")
    rng = np.random.default_rng(73)
    sig = dev(S.sigma_uniform(m, 1e-3, 1.0, rng))
    a = dev(rng.standard_normal(m) / np.sqrt(n))
    b = dev(rng.standard_normal(n) / np.sqrt(n))
    Ud, sd, Vd, fd = lib.rank1_update(U, sig, V, a, b, ctx=dctx)
    Uf, sf, Vf, ff = lib.rank1_update(U, sig, V, a, b)
    assert torch.equal(fd, ff)
    assert float((sf - sd).abs().max()) <= 1e-13 * float(sd[0])
    assert float((Uf - Ud).abs().max()) <= 1e-9 and float((Vf - Vd).abs().max()) <= 1e-9
