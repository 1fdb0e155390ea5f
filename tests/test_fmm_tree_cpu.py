"""The FMM tree on the CPU alone (no GPU): coverage and admissibility.

The host tree of the FMM product (paper_1707_08369_amd/csrc/fmm_tree.h; the
paper's Section 5 and Appendix D, with the adaptive per-box geometry described
there) is compiled with g++ under AddressSanitizer together with
tests/fmm_tree_check.cpp, and run on pole/root sets of the shapes the library
meets: uniform, geometric over 12 decades, 1e-11 pairs, exact repeats removed,
an isolated extreme pole above or below the rest (the second eigen-update of a
side, whose poles are the first one's roots), and both signs of rho. Every
non-empty pair of leaves must be covered exactly once, every M2L pair must be
admissible, every point must lie in its leaf, and every directly evaluated root
must see every leaf once. The roots of the smaller cases are true secular roots
from the oracle; the 8192-pole cases use interlacing roots of the same layout.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle.svdu_oracle as OS

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "fmm_tree_check.cpp")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("fmmtree") / "fmm_tree_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", SRC, "-o",
           exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, cases, p=15):
    text = []
    for g, mu in cases:
        text.append(f"{len(g)} {p}")
        text.append(" ".join(repr(float(x)) for x in g))
        text.append(" ".join(repr(float(x)) for x in mu))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe], input="\n".join(text) + "\n", capture_output=True, text=True, env=env, timeout=600)
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.strip().splitlines()
    assert len(lines) == len(cases), (r.stdout, r.stderr[-2000:])
    for l in lines:
        assert l.startswith("ok"), l
    assert r.returncode == 0
    return [list(map(int, l.split()[1:])) for l in lines]


def _true_roots(d, z, rho):
    defl = OS.deflate(d, z, rho)
    org, tau = OS.secular_roots(defl.g, defl.W, rho)
    return defl.g, defl.g[org] + tau


def _spectrum(kind, K, rng):
    if kind == "uniform":
        return np.sort(rng.uniform(1e-6, 1.0, K))
    if kind == "geometric":
        return np.sort(10.0 ** (-12.0 * np.arange(K) / K))
    if kind == "pairs":
        d = np.sort(rng.uniform(1e-3, 1.0, K))
        h = K // 2
        d[1:2 * h:2] = d[0:2 * h:2] * (1 + 1e-11)
        return np.sort(d)
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["uniform", "geometric", "pairs"])
@pytest.mark.parametrize("rho", [1.6, -0.6])
def test_tree_covers_true_secular_roots(checker, kind, rho):
    rng = np.random.default_rng(11)
    cases = []
    for K in (2, 5, 17, 33, 100, 700):
        d = _spectrum(kind, K, rng)
        z = rng.standard_normal(K) / np.sqrt(K)
        cases.append(_true_roots(d, z, rho))
    _run(checker, cases)


@pytest.mark.parametrize("rho", [1.6, -0.6])
def test_tree_on_two_levels_with_isolated_pole(checker, rho):
    """Second eigen-update of a side: its poles are the first one's roots, so
    the first update's extreme root becomes a pole far from the rest."""
    rng = np.random.default_rng(5)
    K = 1500
    d = np.sort(rng.uniform(1e-6, 1.0, K))
    z = rng.standard_normal(K) / np.sqrt(K) * 1.1
    g1, mu1 = _true_roots(d, z, rho)
    z2 = rng.standard_normal(mu1.shape[0]) / np.sqrt(K) * 1.1
    g2, mu2 = _true_roots(np.sort(mu1), z2, -1.0 / rho)   # the first update's roots are the poles
    res = _run(checker, [(g1, mu1), (g2, mu2)])
    assert res[1][3] >= 0, "the extreme pole of the second update is kept out of the boxes"


def _interlaced(g, rng, above):
    """Roots interlacing poles g (ascending): one per gap, and the extreme one
    beyond the last pole (above) or before the first (below)."""
    K = g.shape[0]
    th = rng.uniform(0.05, 0.95, K)
    mu = np.empty(K)
    if above:
        mu[:-1] = g[:-1] + th[:-1] * np.diff(g)
        mu[-1] = g[-1] + 0.3
    else:
        mu[1:] = g[:-1] + th[1:] * np.diff(g)
        mu[0] = g[0] - 0.3
    return mu


@pytest.mark.parametrize("kind", ["uniform", "geometric", "pairs"])
def test_tree_at_8192_with_isolated_poles(checker, kind):
    """The headline order, including an isolated extreme pole above (as the
    second left eigen-update at m = n = 8192 sees it: 1.77 against <= 1.0) and
    one below."""
    rng = np.random.default_rng(8192)
    cases = []
    for above in (True, False):
        g = _spectrum(kind, 8192, rng)
        cases.append((g, _interlaced(g, rng, above)))
        gi = g.copy()
        if above:
            gi[-1] = 1.77
        else:
            gi[0] = -0.77
        gi = np.sort(gi)
        cases.append((gi, _interlaced(gi, rng, not above)))
    res = _run(checker, cases)
    assert any(r[3] >= 0 for r in res)
