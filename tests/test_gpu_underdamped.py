"""The underdamped (BAOAB) integrator of the plain schedule against the FP64
oracle: positions and velocities after 200 steps of the 56-residue chain
and of the pulled globule (a fixed residue and a cantilever), both force
modes, graph replays against direct launches, and the velocity round trip."""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config

from parity import TRAJ_TOL

pytestmark = pytest.mark.gpu

MASS = 1.0
ZETA = 0.5   # an underdamped friction: zeta h / m = 0.04 per step


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


@pytest.mark.parametrize("name,mode", [("c0", "particle"), ("c1", "particle"), ("c1", "pair")])
def test_underdamped_matches_the_oracle(P, orc, name, mode):
    s = make_config(name)
    p = RunParams(zeta=ZETA)
    rng = np.random.default_rng(3)
    v0 = 0.3 * rng.standard_normal(s.x.shape)
    if s.fixed is not None:
        v0[s.fixed.astype(bool)] = 0.0
    c = P.from_system(s, p, graph_steps=2)
    c.set_force_mode(mode)
    c.set_integrator("underdamped", MASS)
    c.set_velocities(v0)
    c.step(200)
    xg, vg = c.get_coordinates(), c.get_velocities()
    o = orc.OracleSystem(s, p)
    xo, vo, st = o.run_underdamped(s.x, v0, 200, MASS)
    assert st == 0
    dx = float(np.linalg.norm(xg - xo, axis=1).max())
    dv = float(np.linalg.norm(vg - vo, axis=1).max())
    vs = float(np.linalg.norm(vo, axis=1).max())
    log(f"  underdamped {name} ({mode}): max |dx| {dx:.3e} A, max |dv| {dv:.3e} (|v| up to {vs:.2f})")
    assert dx <= TRAJ_TOL
    assert dv <= 1e-4 * vs
    c.close()


def test_underdamped_graphs_equal_direct_launches(P):
    s = make_config("c1")
    p = RunParams(zeta=ZETA)
    a = P.from_system(s, p, graph_steps=1)
    b = P.from_system(s, p, graph_steps=0)
    for c in (a, b):
        c.set_integrator("underdamped", MASS)
    for n in (1, 9, 30, 11, 29):
        a.step(n)
        b.step(n)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    assert np.array_equal(a.get_velocities(), b.get_velocities())
    a.close()
    b.close()


def test_velocities_round_trip_and_overdamped_default(P):
    s = make_config("c0")
    p = RunParams(zeta=ZETA)
    c = P.from_system(s, p)
    c.set_integrator("underdamped", 2.0)
    v = np.random.default_rng(1).standard_normal(s.x.shape)
    c.set_velocities(v)
    got = c.get_velocities()
    assert np.allclose(got, v.astype(np.float32), rtol=0, atol=0)
    c.set_coordinates(s.x)   # new coordinates zero the velocities
    assert not c.get_velocities().any()
    with pytest.raises(P.SopError):
        c.set_integrator("underdamped", 0.0)
    c.close()
