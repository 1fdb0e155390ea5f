"""The far-field interpolants of the secular solve's far-field form, on the CPU.

The far-field form (SVDU_OPT_SECULAR_FMM) splits the poles into leaves of 64
consecutive poles. Leaf l's interval T runs from its first pole to the next
leaf's first pole (the last leaf: to the last pole; leaf 0 from the second
pole: the extreme root beyond the last pole and the root between the first two
poles take the direct sums). Poles at least |T| from T are far: those below T enter psi and those
above it phi for every root of the leaf. The four far sums psi, psi', phi, phi'
are sampled at 32 Chebyshev points of the first kind on T and interpolated in
the barycentric form. This file restates that construction in numpy and
measures it against the far sums taken directly in extended precision at
points across T.

For a singularity one width |T| from T the Bernstein ellipse parameter is
3 + sqrt 8, so the truncation error is about (3 + sqrt 8)^-32 ~ 4e-25 times a
modest constant. What remains is rounding: the barycentric form keeps it at a
few units of FP64 (bounded here by 2e-15 relative to the sum of the terms'
magnitudes), where the coefficient form (DCT, then Clenshaw) loses about p
units; the second test shows both.
"""
import numpy as np
import pytest

LEAF, P = 64, 32


def _leaf(d, k0):
    K = d.shape[0]
    lo = d[max(k0, 1)]
    wd = d[min(k0 + LEAF, K - 1)] - lo
    off = d - lo
    kl = int(np.argmax(off > -wd))                    # first near pole
    kr = int(np.nonzero(off < 2 * wd)[0][-1])         # last near pole
    return lo, wd, kl, kr


def _far_sums(d, w, lo, xo, kl, kr, dtype):
    """psi, psi', phi, phi' over the far poles at x = lo + xo (offsets from lo),
    and the sums of their terms' magnitudes."""
    d, w = d.astype(dtype), w.astype(dtype)
    lo, xo = dtype(lo), np.asarray(xo, dtype=dtype)
    out, mag = [], []
    for sl in (slice(0, kl), slice(kr + 1, None)):
        den = (d[sl][None, :] - lo) - xo[:, None]
        out.append(np.sum(w[sl][None, :] / den, axis=1))
        out.append(np.sum(w[sl][None, :] / den ** 2, axis=1))
        mag.append(np.sum(np.abs(w[sl][None, :] / den), axis=1))
        mag.append(np.sum(w[sl][None, :] / den ** 2, axis=1))
    return out, mag


def _cospi_frac(k, n):
    """cos(pi k / n) for integers k, n with the argument reduced exactly first
    (as cospi does): a rounded pi times a large k would cost digits."""
    k = np.mod(k, 2 * n)
    return np.cos(np.pi * k / n)


def _nodes():
    return _cospi_frac(2 * np.arange(P) + 1, 2 * P)


def _cheb_coef(f):
    q = np.arange(P)
    c = np.array([np.sum(f * _cospi_frac(j * (2 * q + 1), 2 * P)) for j in range(P)]) * (2.0 / P)
    c[0] *= 0.5
    return c


def _clenshaw(c, t):
    b1 = np.zeros_like(t)
    b2 = np.zeros_like(t)
    for j in range(P - 1, 0, -1):
        b1, b2 = 2 * t * b1 - b2 + c[j], b1
    return t * b1 - b2 + c[0]


def _bary(f, t):
    """Barycentric interpolation from the values f at the first-kind points."""
    tq = _nodes()
    q = np.arange(P)
    lam = np.where(q % 2 == 1, -1.0, 1.0) * _cospi_frac(2 * q + 1 - P, 2 * P)   # sin((2q+1) pi / 2P)
    D = t[:, None] - tq[None, :]
    hit = np.abs(D) < 2.0 ** -60           # at a point: that point's value
    D[hit] = 1.0
    r = lam[None, :] / D
    out = np.sum(r * f[None, :], axis=1) / np.sum(r, axis=1)
    rows, cols = np.nonzero(hit)
    out[rows] = f[cols]
    return out


def _spectrum(kind, K, rng):
    if kind == "uniform":
        return np.sort(rng.uniform(1e-3, 1.0, K) ** 2)
    if kind == "geometric":
        return np.sort(10.0 ** (-12.0 * np.arange(K) / K))
    if kind == "pairs":
        base = np.sort(rng.uniform(0.1, 1.0, K // 2))
        return np.sort(np.concatenate([base, base * (1 + 2e-11)]))
    if kind == "first_outlier":   # reflected spectrum after an update with rho > 0
        d = np.sort(rng.uniform(0.0, 1.0, K))
        d[0] = -3.0
        return d
    nc = (3 * K) // 4
    cl = 1.0 + 1e-9 * (np.arange(nc) + 0.5 * rng.uniform(0.0, 1.0, nc)) / nc
    return np.sort(np.concatenate([cl, rng.uniform(0, 10, K - nc)]))


def _leaf_errors(kind, rng, form):
    K = 4096
    d = _spectrum(kind, K, rng)
    w = (rng.standard_normal(K) / np.sqrt(K)) ** 2
    rho = 0.8
    leaves = sorted(set([0, 1, K // LEAF // 2, K // LEAF - 2, K // LEAF - 1] +
                        list(rng.integers(0, K // LEAF, 3))))
    worst = 0.0
    for leaf in leaves:
        k0 = leaf * LEAF
        lo, wd, kl, kr = _leaf(d, k0)
        # the near range holds the leaf and the next pole; far poles are >= |T| away
        assert kl <= max(k0, 1) and kr >= min(k0 + LEAF, K - 1)
        assert np.all(lo - d[:kl] >= wd * (1 - 1e-15))
        assert np.all(d[kr + 1:] - (lo + wd) >= wd * (1 - 1e-15))
        h = 0.5 * wd
        node_vals, _ = _far_sums(d, w, lo, h * (1 + _nodes()), kl, kr, np.float64)
        xo = np.concatenate([[0.0, wd, h * (1 + _nodes()[5])], rng.uniform(0.0, wd, 60)])
        t = (xo - h) / h
        ref, mag = _far_sums(d, w, lo, xo, kl, kr, np.longdouble)
        for a in range(4):
            got = _bary(node_vals[a], t) if form == "bary" else _clenshaw(_cheb_coef(node_vals[a]), t)
            err = np.abs(got - ref[a].astype(np.float64))
            m = mag[a].astype(np.float64)
            worst = max(worst, float(np.max(np.where(m > 0, err / np.maximum(m, 1e-300), 0.0))))
    return worst


@pytest.mark.parametrize("kind", ["uniform", "geometric", "pairs", "cluster", "first_outlier"])
def test_far_field_interpolants_are_at_rounding_level(kind):
    assert _leaf_errors(kind, np.random.default_rng(11), "bary") <= 2e-15


def test_barycentric_form_rounds_less_than_the_coefficient_form():
    bary = _leaf_errors("uniform", np.random.default_rng(5), "bary")
    coef = _leaf_errors("uniform", np.random.default_rng(5), "coef")
    assert bary < 0.6 * coef


def test_far_field_interpolant_error_falls_with_the_order():
    """The construction's convergence rate itself: order p = 4 ... 16 against
    the predicted (3 + sqrt 8)^-p (worst case, a pole exactly one width away)."""
    rng = np.random.default_rng(3)
    # one leaf [0, 1] with far poles starting exactly one width below it
    far = -1.0 - np.sort(rng.uniform(0.0, 3.0, 200))
    far[-1] = -1.0
    wts = rng.uniform(0.5, 1.5, 200)
    x = np.linspace(0.0, 1.0, 101)
    exact = np.array([np.sum(wts / (far - xi)) for xi in x])
    errs = []
    for p in (4, 8, 12, 16):
        tq = np.cos(np.pi * (2 * np.arange(p) + 1) / (2 * p))
        f = np.array([np.sum(wts / (far - 0.5 * (1 + tt))) for tt in tq])
        q = np.arange(p)
        c = np.array([np.sum(f * np.cos(np.pi * j * (2 * q + 1) / (2 * p))) for j in range(p)]) * (2.0 / p)
        c[0] *= 0.5
        t = 2 * x - 1
        Tm = np.cos(np.outer(np.arccos(np.clip(t, -1, 1)), np.arange(p)))
        errs.append(np.max(np.abs(Tm @ c - exact)) / np.max(np.abs(exact)))
    rate = 3 + np.sqrt(8)
    for p, e in zip((4, 8, 12, 16), errs):
        assert e <= 10.0 * rate ** -p, (p, e)
    assert errs[-1] < errs[0] * 1e-6
