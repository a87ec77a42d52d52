"""The allocation-free entry point sop_ramp_run_static against sop_ramp_run:
the same particles and moments on two calls in a row, the second smaller."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

KSP, KBT = 40.0, 4.14
XI = KBT / 1.5e-9
RF = 1e-8


def test_static_matches_workspace_entry_point():
    import torch
    import paper_1003_1148_amd as P
    assert torch.cuda.is_available()
    mom = torch.full((2,), float("nan"), dtype=torch.float64, device="cuda")
    for M, order, n in ((300_001, 1, 400), (1_000, 2, 250)):
        rp = P.ramp_params(RF, XI, KSP, KBT, 25.0, order=order, seed=99, stream=1)
        x0 = np.linspace(-0.05, 0.05, M)
        a = torch.zeros((M, 2), dtype=torch.float32, device="cuda")
        a[:, 0] = torch.as_tensor(x0.astype(np.float32))
        b = a.clone()
        ref = P.ramp_run(rp, a, 0, n)
        P.ramp_run_static(rp, b, 0, n, moments_out=mom)
        torch.cuda.synchronize()
        assert torch.equal(a, b)
        got = mom.cpu().numpy()
        assert got[0] == ref[0] and got[1] == ref[1]
        # against the positions themselves
        v = b.cpu().numpy().astype(np.float64)
        X = v[:, 0] + v[:, 1]
        assert got[0] == pytest.approx(X.mean(), rel=1e-12, abs=1e-15)
