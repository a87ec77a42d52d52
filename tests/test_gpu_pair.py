"""The pair-based force evaluation of the plain schedule (Algorithm 4: each
pair once, +df / -df accumulated with hardware float atomics; Algorithm 5's
gathering folded into the update kernel) against the FP64 oracle, with the
same bars as the particle-based one.  The order of the atomic additions is
not fixed, so runs agree with each other to rounding, not bit for bit."""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config

from parity import TRAJ_TOL, assert_energies, assert_forces, oracle_reference

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


_CACHE = {}


def cfg(name):
    if name not in _CACHE:
        _CACHE[name] = make_config(name)
    return _CACHE[name]


def perturbed(s, sd=0.15, seed=1):
    rng = np.random.default_rng(seed)
    return s.x + sd * rng.standard_normal(s.x.shape)


@pytest.mark.parametrize("name,tile", [("c0", 64), ("c1", 64), ("c1", 128), ("c1", 256), ("c2", 64)])
def test_pair_forces_and_energies(P, orc, name, tile):
    s = cfg(name)
    x = perturbed(s)
    c = P.from_system(s, RunParams(), coordinates=x, tile=tile)
    c.set_force_mode("pair")
    assert c.get_force_mode() == "pair"
    c.set_step(321)
    F, E, fe = c.compute_forces()
    o = orc.OracleSystem(s, RunParams())
    Fo, Eo, feo, S, Em = oracle_reference(o, x, step=321)
    assert_forces(F, Fo, S, f"pair {name} tile {tile}")
    assert_energies(E, Eo, Em, s.res_offsets, f"pair {name} tile {tile}")
    assert np.allclose(fe, feo, rtol=1e-5, atol=1e-12)
    c.close()


@pytest.mark.parametrize("name", ["c0", "c1"])
def test_pair_trajectory_200_steps(P, orc, name):
    s = cfg(name)
    p = RunParams()
    c = P.from_system(s, p, graph_steps=2, energy_every=10)
    c.set_force_mode("pair")
    c.step(200)
    xg = c.get_coordinates()
    Eg, estep = c.get_energies()
    o = orc.OracleSystem(s, p)
    x190, _, _, st = o.run(s.x, 190)
    assert st == 0
    xo, Eo, _, st = o.run(x190, 10, step0=190, energy_every=10)
    assert st == 0
    d = float(np.linalg.norm(xg - xo, axis=1).max())
    log(f"  pair {name}: 200-step max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL
    assert estep == 190
    _, Em = o.force_scale(x190, step=190)
    assert_energies(Eg, Eo[0], Em, s.res_offsets, f"pair {name} step 190")
    c.close()


def test_pair_and_particle_agree_and_switch(P):
    """Switching the mode mid-run is allowed (graphs are recaptured); the two
    modes' trajectories agree to rounding."""
    s = cfg("c1")
    p = RunParams()
    a = P.from_system(s, p, graph_steps=1)
    b = P.from_system(s, p, graph_steps=1)
    b.set_force_mode("pair")
    a.step(50)
    b.step(50)
    b.set_force_mode("particle")
    a.step(50)
    b.step(50)
    d = float(np.linalg.norm(a.get_coordinates() - b.get_coordinates(), axis=1).max())
    log(f"  particle vs pair then particle: max |dx| {d:.3e} A")
    assert d < 1e-5
    a.close()
    b.close()


def test_autotune_includes_the_pair_mode(P, tmp_path):
    s = cfg("c0")
    c = P.from_system(s, RunParams())
    path = str(tmp_path / "tune.txt")
    c.autotune(budget_ms=60.0, cache_path=path)
    mode, tile = c.get_force_mode(), c.get_tile()
    with open(path) as f:
        line = f.read().split()
    assert int(line[-2]) == tile and int(line[-1]) == (1 if mode == "pair" else 0)
    d = P.from_system(s, RunParams())
    d.autotune(budget_ms=60.0, cache_path=path)   # read back from the cache
    assert (d.get_force_mode(), d.get_tile()) == (mode, tile)
    c.close()
    d.close()
