"""GPU test of svdu_rank1_update_noalloc (the update without a caller
workspace): through the C ABI, its results equal, bitwise, those of
svdu_rank1_update on the same inputs, on two calls in a row (the second one
smaller, so it runs on what the first left in the shared scratch array), in
both precisions; an update too large for the array is refused on the host."""
import numpy as np
import pytest
import torch

import synth_inputs as S

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64).cuda()


@pytest.mark.parametrize("precision", [0, 1])
def test_noalloc_equals_workspace_entry_point(lib, precision):
    for (m, n, kind, seed) in [(700, 1024, "uniform", 5), (130, 257, "clustered", 6)]:
        kw = dict(zero_frac=0.05) if kind == "clustered" else {}
        P = S.make_problem(m, n, kind, seed=seed, **kw)
        args = [dev(P.U), dev(P.sigma), dev(P.V), dev(P.a), dev(P.b)]
        ref = lib.rank1_update(*args, precision=precision)
        got = lib.rank1_update_noalloc(*args, precision=precision)
        for x, y in zip(got, ref):
            assert torch.equal(x, y), (m, n)


def test_noalloc_refuses_updates_beyond_the_array(lib):
    m = n = 1400
    assert lib.svdu_workspace_bytes(m, n) > lib.SVDU_NOALLOC_SCRATCH_BYTES
    x = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    v = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(lib.SvduError) as e:
        lib.rank1_update_noalloc(x, v, x.clone(), v, v, check=False)
    assert e.value.code == lib.SVDU_ENOMEM
