"""GPU tests of the exact-slice INT8 precision form (SVDU_PREC_SLICED_INT8):
the products X C~ run as INT8 slice products with exact INT32 accumulation.
Roots, deflation, weights and signs are the FP64 ones, so sigma^ and the flags
must be bitwise those of the FP64 path; the vectors must meet the stated bound
of the precision form, reconstruction and orthogonality error <= 1e-10 against
the inputs, and match the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle as O
import synth_inputs as S

pytestmark = pytest.mark.gpu

BOUND = 1e-10          # the precision form's stated bound (recon, orth)


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


def _align_cols(ref, got):
    s = np.sign(np.sum(ref * got, axis=0))
    s[s == 0] = 1.0
    return got * s[None, :]


CASES = [(1, 1, "uniform", {}), (3, 3, "uniform", {}), (16, 16, "uniform", {}), (100, 173, "uniform", {}),
         (129, 130, "uniform", {}), (256, 256, "uniform", {}), (300, 457, "uniform", {}),
         (512, 512, "geometric", {}), (512, 512, "clustered", dict(zero_frac=0.05)),
         (512, 512, "clustered", dict(zero_frac=0.05, zero_q=True)), (40, 40, "zero", {})]


@pytest.mark.parametrize("m,n,kind,kw", CASES)
def test_int8_form_matches_oracle_and_fp64_roots(lib, m, n, kind, kw):
    P = S.make_problem(m, n, kind, seed=7, **kw)
    args = [dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)]
    Uf, sf, Vf, ff = lib.rank1_update(*args)
    Ui, si, Vi, fi = lib.rank1_update(*args, precision=lib.SVDU_PREC_SLICED_INT8)
    # the form touches only the products
    assert torch.equal(si, sf) and torch.equal(fi, ff)
    Ug, sg, Vg = host(Ui), host(si), host(Vi)
    r = O.svd_rank1_update(P.U, P.sigma, P.V, P.a, P.b)
    Ah = O.dense_ahat(P.U, P.sigma, P.V, P.a, P.b)
    smax = max(r.sigma[0], 1e-300)
    assert np.max(np.abs(sg - r.sigma)) <= 1e-13 * smax
    assert O.recon_error(Ah, Ug, sg, Vg) <= BOUND
    assert O.orth_error(Ug) <= BOUND and O.orth_error(Vg) <= BOUND
    if n > m:
        assert np.max(np.abs(Ah @ Vg[:, m:])) <= BOUND * smax
    ok = _separated(r.sigma ** 2) & (r.sigma >= 1e-6 * smax)
    Ua = _align_cols(r.U, Ug)
    assert np.max(np.abs(Ua - r.U)[:, ok], initial=0.0) <= 1e-9
    su = np.sign(np.sum(r.U * Ug, axis=0))
    Va = Vg[:, :m] * su[None, :]
    assert np.max(np.abs(Va - r.V[:, :m])[:, ok], initial=0.0) <= 1e-9
    # against the FP64 path's vectors, element by element, in the columns whose
    # singular value is well separated (inside a close cluster any rotation of
    # the basis is as correct)
    Uf_h, Vf_h = host(Uf), host(Vf)
    assert np.max(np.abs(Ug - Uf_h)[:, ok], initial=0.0) <= 1e-11
    assert np.max(np.abs(Vg[:, :m] - Vf_h[:, :m])[:, ok], initial=0.0) <= 1e-11


@pytest.mark.parametrize("slices", [6, 7, 8])
def test_int8_slices_option(lib, slices):
    """More slices, smaller error; every setting within the bound; the option
    lives in the context."""
    P = S.make_problem(384, 512, "uniform", seed=9, lo=1e-3, hi=1.0)
    args = [dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)]
    ref = lib.rank1_update(*args, want_defl=False)
    ctx = lib.Context()
    try:
        assert ctx.set_option(lib.SVDU_OPT_SLICES, slices) == 7
        Ui, si, Vi, _ = lib.rank1_update(*args, precision=lib.SVDU_PREC_SLICED_INT8, ctx=ctx, want_defl=False)
    finally:
        ctx.close()
    assert torch.equal(si, ref[1])
    ok = torch.as_tensor(_separated(host(si) ** 2), device="cuda")
    err = max(float((Ui - ref[0])[:, ok].abs().max()), float((Vi[:, :384] - ref[2][:, :384])[:, ok].abs().max()))
    # the slicing error is about 2^(1 - 7 S) relative to the largest entry
    assert err <= {6: 2e-11, 7: 2e-13, 8: 5e-15}[slices], err


def test_int8_option_range(lib):
    ctx = lib.Context()
    try:
        assert ctx.set_option(lib.SVDU_OPT_SLICES, 5) == lib.SVDU_EINVAL
        assert ctx.set_option(lib.SVDU_OPT_SLICES, 9) == lib.SVDU_EINVAL
        assert ctx.set_option(lib.SVDU_OPT_SLICES, 8) == 7
    finally:
        ctx.close()


def test_int8_deterministic_and_batched_bitwise(lib):
    items = []
    for k, (m, n) in enumerate([(64, 64), (200, 333), (130, 130), (17, 40)]):
        P = S.make_problem(m, n, "uniform", seed=20 + k)
        items.append((dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)))
    single = [lib.rank1_update(*it, precision=lib.SVDU_PREC_SLICED_INT8, want_defl=False)[:3] for it in items]
    again = [lib.rank1_update(*it, precision=lib.SVDU_PREC_SLICED_INT8, want_defl=False)[:3] for it in items]
    for a, b in zip(single, again):
        assert all(torch.equal(x, y) for x, y in zip(a, b))
    for graph in (False, True):
        outs = lib.rank1_update_batched(items, precision=lib.SVDU_PREC_SLICED_INT8, use_graph=graph)
        for a, b in zip(single, outs):
            assert all(torch.equal(x, y) for x, y in zip(a, b))


def _recon_orth_gpu(U, s, V, a, b, Uo, so, Vo):
    m = U.shape[0]
    Ah = (U * s[None, :]) @ V[:, :m].T + torch.outer(a, b)
    rec = ((Uo * so[None, :]) @ Vo[:, :m].T - Ah).norm().item() / Ah.norm().item()
    ou = (Uo.T @ Uo - torch.eye(m, dtype=Uo.dtype, device=Uo.device)).abs().max().item()
    ov = (Vo.T @ Vo - torch.eye(Vo.shape[0], dtype=Vo.dtype, device=Vo.device)).abs().max().item()
    return rec, ou, ov


@pytest.mark.parametrize("m,n", [(4096, 8192), (8192, 8192)])
def test_int8_form_full_size_within_bound(lib, m, n):
    """The precision-form configurations at their full sizes: sigma ~ U[1e-3, 1],
    Haar U and V; reconstruction and orthogonality <= 1e-10, sigma^ bitwise the
    FP64 path's."""
    rng = S.rng_for(31 + m)
    U = S.haar_torch(m, seed=41 + m, device="cuda")
    V = S.haar_torch(n, seed=42 + n, device="cuda")
    s = dev(S.sigma_uniform(m, 1e-3, 1.0, rng))
    a = dev(rng.standard_normal(m) / np.sqrt(n))
    b = dev(rng.standard_normal(n) / np.sqrt(n))
    Uf, sf, Vf, ff = lib.rank1_update(U, s, V, a, b)
    Ui, si, Vi, fi = lib.rank1_update(U, s, V, a, b, precision=lib.SVDU_PREC_SLICED_INT8)
    assert torch.equal(si, sf) and torch.equal(fi, ff)
    rec, ou, ov = _recon_orth_gpu(U, s, V, a, b, Ui, si, Vi)
    assert rec <= BOUND and ou <= BOUND and ov <= BOUND, (rec, ou, ov)
    ok = torch.as_tensor(_separated(host(sf) ** 2), device="cuda")
    assert float((Ui - Uf)[:, ok].abs().max()) <= 1e-11
    assert float((Vi[:, :m] - Vf[:, :m])[:, ok].abs().max()) <= 1e-11
