"""GPU tests of the rank-k update (svdu_rankk_update): k rank-1 updates in
one call, against the oracle's k rank-1 updates in order (the Conclusion's
extension), at the workloads' sizes."""
import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


def host(t):
    return t.detach().cpu().numpy()


def _separated(vals, rel=1e-4):
    v = np.asarray(vals)
    gap = np.full(v.shape, np.inf)
    d = np.abs(np.diff(v))
    gap[:-1] = np.minimum(gap[:-1], d)
    gap[1:] = np.minimum(gap[1:], d)
    return gap > rel * max(np.max(np.abs(v)), 1e-300)


def _pairs(m, n, k, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((k, m)) / np.sqrt(n), rng.standard_normal((k, n)) / np.sqrt(n)


@pytest.mark.parametrize("m,n,k,prec", [(1, 1, 2, 0), (16, 16, 1, 0), (100, 173, 3, 0), (256, 256, 4, 0),
                                        (300, 457, 5, 0), (256, 256, 3, 2)])
def test_rankk_matches_oracle(lib, m, n, k, prec):
    P = S.make_problem(m, n, "uniform", seed=m + k)
    A, B = _pairs(m, n, k, seed=m * k + 1)
    Ug, sg, Vg = (host(t) for t in lib.rankk_update(dev(P.U), dev(P.sigma), dev(P.V), dev(A), dev(B),
                                                     precision=prec))
    r = O.svd_rankk_update(P.U, P.sigma, P.V, A, B)
    Ah = (P.U * P.sigma[None, :]) @ P.V[:, :m].T + A.T @ B
    smax = r.sigma[0]
    assert np.max(np.abs(sg - r.sigma)) <= 1e-13 * smax * k
    assert O.recon_error(Ah, Ug, sg, Vg) <= 1e-12 * k
    assert O.orth_error(Ug) <= 1e-12 * k and O.orth_error(Vg) <= 1e-12 * k
    ok = _separated(r.sigma ** 2) & (r.sigma >= 1e-6 * smax)
    su = np.sign(np.sum(r.U * Ug, axis=0))
    su[su == 0] = 1.0
    assert np.max(np.abs(Ug * su[None, :] - r.U)[:, ok], initial=0.0) <= 1e-9
    assert np.max(np.abs(Vg[:, :m] * su[None, :] - r.V[:, :m])[:, ok], initial=0.0) <= 1e-9


def test_rankk_is_the_sequence_of_rank1_calls(lib):
    """Bitwise: the same kernels in the same order as k svdu_rank1_update calls."""
    m, n, k = 130, 200, 3
    P = S.make_problem(m, n, "uniform", seed=8)
    A, B = _pairs(m, n, k, seed=9)
    cur = (dev(P.U), dev(P.sigma), dev(P.V))
    for j in range(k):
        cur = lib.rank1_update(*cur, dev(A[j]), dev(B[j]), want_defl=False)[:3]
    got = lib.rankk_update(dev(P.U), dev(P.sigma), dev(P.V), dev(A), dev(B))
    assert all(torch.equal(x, y) for x, y in zip(got, cur))


def test_rankk_full_size_invariants(lib):
    m = n = 4096
    k = 2
    U = S.haar_torch(m, seed=81, device="cuda")
    V = S.haar_torch(n, seed=82, device="cuda")
    rng = np.random.default_rng(83)
    sig = dev(S.sigma_geometric(m))
    A, B = _pairs(m, n, k, seed=84)
    At, Bt = dev(A), dev(B)
    Ug, sg, Vg = lib.rankk_update(U, sig, V, At, Bt)
    Ah = (U * sig[None, :]) @ V[:, :m].T + At.T @ Bt
    recon = ((Ug * sg[None, :]) @ Vg[:, :m].T - Ah).norm().item() / Ah.norm().item()
    I = torch.eye(m, dtype=torch.float64, device="cuda")
    assert recon <= 1e-12, recon
    assert (Ug.T @ Ug - I).abs().max().item() <= 1e-12 and (Vg.T @ Vg - I).abs().max().item() <= 1e-12
    # Frobenius identity of the sum
    fro = Ah.norm().item() ** 2
    assert abs((sg ** 2).sum().item() - fro) <= 1e-12 * fro


def test_rankk_reports_a_device_error_of_any_update(lib):
    m, n, k = 32, 40, 3
    P = S.make_problem(m, n, "uniform", seed=10)
    A, B = _pairs(m, n, k, seed=11)
    A[1, 5] = np.nan          # only the second update sees it
    with pytest.raises(lib.SvduError) as e:
        lib.rankk_update(dev(P.U), dev(P.sigma), dev(P.V), dev(A), dev(B))
    assert e.value.code == lib.SVDU_ENONFINITE
