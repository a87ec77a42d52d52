"""The plain schedule at protein density (Table I's HK97 row: about 140 list
pairs per residue): a seeded globule of 4,800 residues at 116 A^3 per
residue, over 100 list pairs per residue.  Its tiles stage more partners
than one LDS window holds on every tile size, so the kernels take the
windowed path.  Bars as elsewhere: bit-exact lists, element-wise forces,
200-step trajectories; no list or staging overflow."""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config

from parity import TRAJ_TOL, assert_forces, oracle_reference

pytestmark = pytest.mark.gpu


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


@pytest.fixture(scope="module")
def dense():
    return make_config("dense")


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_dense_list_forces_and_trajectory(P, orc, dense, tile):
    s = dense
    p = RunParams()
    o = orc.OracleSystem(s, p)
    c = P.from_system(s, p, tile=tile, graph_steps=2)
    c.build_pairlist()
    got = c.get_pairlist()
    ref = o.pairlist(s.x)
    log(f"  tile {tile}: {len(ref) / s.n_res:.1f} list pairs per residue")
    assert len(ref) / s.n_res >= 100.0
    assert np.array_equal(got, ref)
    rng = np.random.default_rng(tile)
    x = s.x + 0.1 * rng.standard_normal(s.x.shape)
    d = P.from_system(s, p, tile=tile, coordinates=x)
    F, _, _ = d.compute_forces()
    Fo, _, _, S, _ = oracle_reference(o, x)
    assert_forces(F, Fo, S, f"dense tile {tile}")
    d.close()
    c.step(200)
    xg = c.get_coordinates()
    xo, _, _, st = o.run(s.x, 200)
    assert st == 0
    dx = float(np.linalg.norm(xg - xo, axis=1).max())
    log(f"  tile {tile}: 200-step max |dx| {dx:.3e} A")
    assert dx <= TRAJ_TOL
    c.build_pairlist()
    assert np.array_equal(c.get_pairlist(), o.pairlist(xg))
    c.close()
