"""Precision study on the 250,000-residue fibre: compensated FP32 positions
and FP32 forces against the FP64 oracle where the coordinates are largest.

The far end of the fibre (its last 20 subunits, |x| up to 1.8e4 A, where
the FP32 spacing of a coordinate is 2e-3 A, far above the thermal step's
rounding budget) runs 1,000 steps on the GPU and in the oracle from the same
start and Philox stream. Every 100 steps the test records the L2 force error
of the GPU forces against the oracle's on the same coordinates, and the RMS
and largest coordinate difference between the two trajectories.
"""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config

from parity import force_errors, force_gate_scale

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-5
TRAJ_TOL = 1e-4


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_1003_1148_amd as P
    P.lib()
    return P


def tail_of(s, n):
    """The last n residues of a single-trajectory system (whole chains)."""
    from synth.structures import System
    a = s.n_res - n
    keep_b = (s.bonds >= a).all(1)
    keep_n = (s.natives >= a).all(1)
    return System(s.name + f"-last{n}", s.x[a:].copy(), np.array([0, n], np.int64),
                  s.stream_ids.copy(), s.chain_id[a:].copy(), s.bonds[keep_b] - a,
                  s.bond_r0[keep_b], s.natives[keep_n] - a, s.native_r0[keep_n], None, [], None,
                  s.steps)


def test_fibre_end_force_error_and_drift(P, orc):
    s = tail_of(make_config("c4"), 20 * 250)
    assert np.abs(s.x[:, 0]).max() > 1.4e4
    p = RunParams()
    c = P.from_system(s, p)
    o = orc.OracleSystem(s, p)
    xo = s.x.copy()
    rows = []
    for k in range(1, 11):
        c.step(100)
        xo, _, _, st = o.run(xo, 100, step0=100 * (k - 1))
        assert st == 0
        xg = c.get_coordinates()
        F, _, _ = c.compute_forces()
        pairs = o.pairlist(xg)
        Fo, _, _, st = o.forces(xg, step=100 * k, pairs=pairs)
        assert st == 0
        S = force_gate_scale(o, xg, step=100 * k, pairs=pairs)
        ferr, ew, _, zero_ok = force_errors(F, Fo, S)
        assert zero_ok
        d = np.linalg.norm(xg - xo, axis=1)
        rows.append((100 * k, ferr, ew, float(np.sqrt((d * d).mean())), float(d.max())))
    log("step  force_rel_err  max_res_err/(S+0.05K)  rms_dx_A  max_dx_A")
    for r in rows:
        log(f"{r[0]:5d}  {r[1]:.3e}  {r[2]:.3e}  {r[3]:.3e}  {r[4]:.3e}")
    assert all(r[1] <= FORCE_TOL and r[2] <= FORCE_TOL for r in rows)
    assert rows[1][4] <= TRAJ_TOL          # 200 steps
    assert rows[-1][4] <= 10 * TRAJ_TOL    # 1,000 steps: still far below the FP32 spacing
