"""The FMM path's error against the direct product as the expansion order p
grows (the paper's experiment on the error against p, Section 7.1 "Choice of
epsilon", on the m = n = 4096 geometric workload). The order is chosen from
the tolerance as p = ceil(log_5(1/eps)), so eps = 1.5 * 5^-p selects p. The
difference from the direct path must stay within the tolerance contract
(10 eps) and within the convergence rate of Chebyshev interpolation between
boxes one box apart, (3 + sqrt 8)^-p, and fall as p grows until it reaches
rounding level."""
import numpy as np
import pytest
import torch

import synth_inputs as S

pytestmark = pytest.mark.gpu


def test_fmm_error_falls_with_the_order(lib):
    m = n = 4096
    U = S.haar_torch(m, seed=91, device="cuda")
    V = S.haar_torch(n, seed=92, device="cuda")
    rng = np.random.default_rng(93)
    sig = torch.as_tensor(S.sigma_geometric(m), device="cuda")
    a = torch.as_tensor(rng.standard_normal(m) / np.sqrt(n), device="cuda")
    b = torch.as_tensor(rng.standard_normal(n) / np.sqrt(n), device="cuda")
    Ud, sd, Vd, _ = lib.rank1_update(U, sig, V, a, b, want_defl=False)
    errs = {}
    for p in (8, 10, 12, 14, 16):
        eps = 1.5 * 5.0 ** (-p)
        Uf, sf, Vf, _ = lib.rank1_update(U, sig, V, a, b, path=lib.SVDU_PATH_FMM, eps=eps, want_defl=False)
        assert torch.equal(sf, sd)      # the roots do not depend on the product path
        err = max((Uf - Ud).abs().max().item(), (Vf - Vd).abs().max().item())
        errs[p] = err
        assert err <= 10.0 * eps, (p, err)
        assert err <= (3.0 + 8.0 ** 0.5) ** (-p), (p, err)
    for p in (8, 10, 12, 14):
        assert errs[p + 2] < errs[p] or errs[p] < 1e-14, errs
    # at least five orders of magnitude from p = 8 to p = 16
    assert errs[8] >= 1e5 * errs[16] or errs[16] < 1e-14, errs
