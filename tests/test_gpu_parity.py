"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: Philox words and pair lists bit-exact; forces within a relative L2
error of 1e-5 and, residue by residue, within 1e-5 of the oracle's force
scale S_i (tests/parity.py); energies term by term within 1e-5 of the
oracle's magnitude sums; 200-step trajectories within 1e-4 A per residue;
graph replays, repeated runs and checkpoint/resume bit-identical.
"""
import math
import sys

import numpy as np
import pytest

from synth import RunParams, make_config
from synth.structures import Tip

from parity import assert_energies, assert_forces, oracle_reference

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


_CACHE = {}


def cfg(name):
    if name not in _CACHE:
        if name == "c3s":
            _CACHE[name] = make_config("c3", n_traj=96)
        elif name == "c2cap":
            _CACHE[name] = cap_of(make_config("c2"), 80 * 250)
        else:
            _CACHE[name] = make_config(name)
    return _CACHE[name]


def cap_of(s, n):
    """The first n residues of a single-trajectory system (whole chains)."""
    from synth.structures import System
    keep_b = (s.bonds < n).all(1)
    keep_n = (s.natives < n).all(1)
    fixed = None if s.fixed is None else s.fixed[:n].copy()
    return System(s.name + f"-first{n}", s.x[:n].copy(), np.array([0, n], np.int64),
                  s.stream_ids.copy(), s.chain_id[:n].copy(), s.bonds[keep_b], s.bond_r0[keep_b],
                  s.natives[keep_n], s.native_r0[keep_n], fixed, [], s.tip, s.steps)


def perturbed(s, sd=0.15, seed=1):
    """Start coordinates displaced by N(0, sd^2) per axis; sd = 0.15 A keeps
    every FENE bond of the largest workload well inside |r - r0| < R0."""
    rng = np.random.default_rng(seed)
    return s.x + sd * rng.standard_normal(s.x.shape)


def ctx_for(P, s, p=None, x=None, **kw):
    p = p or RunParams()
    return P.from_system(s, p, coordinates=x, **kw)


# --------------------------------------------------------------------------
# random numbers
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0", "c3s"])
def test_philox_words_bit_exact(P, orc, name):
    s = cfg(name)
    p = RunParams(seed=0xA5A5F00D12345678)
    log(f"noise {name} n={s.n_res}")
    c = ctx_for(P, s, p)
    rng = np.random.default_rng(0)
    rows = rng.choice(s.n_res, size=min(400, s.n_res), replace=False)
    for step in [0, 7, 2**32 + 5]:
        w, g = c.sample_noise(step)
        for i in rows:
            t = int(np.searchsorted(s.res_offsets, i, side="right") - 1)
            local = i - s.res_offsets[t]
            ctr = np.array([local, s.stream_ids[t], step & 0xFFFFFFFF, step >> 32], np.uint32)
            key = np.array([p.seed & 0xFFFFFFFF, p.seed >> 32], np.uint32)
            assert np.array_equal(w[i], orc.philox(ctr, key)), (i, step)
            ref = orc.gauss3(p.seed, local, s.stream_ids[t], step)
            assert np.allclose(g[i], ref, rtol=0, atol=4e-6), (i, step, g[i], ref)


def test_free_particle_msd_on_gpu(P):
    m, n = 40000, 10
    rng = np.random.default_rng(21)
    from synth.structures import System
    x = rng.uniform(-1e4, 1e4, size=(m, 3))
    s = System("free", x, np.arange(m + 1, dtype=np.int64), np.arange(m, dtype=np.uint32),
               np.zeros(m, np.int32), np.zeros((0, 2), np.int32), np.zeros(0),
               np.zeros((0, 2), np.int32), np.zeros(0))
    p = RunParams(r_list=1e-3)
    c = ctx_for(P, s, p)
    c.step(n)
    x1 = c.get_coordinates()
    msd = ((x1 - x) ** 2).sum(1).mean()
    expect = 6.0 * p.kBT / p.zeta * n * p.h
    assert abs(msd / expect - 1.0) < 4.5 * math.sqrt(2.0 / 3.0) / math.sqrt(m)


# --------------------------------------------------------------------------
# pair lists
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3s", "c4"])
def test_pairlist_bit_exact(P, orc, name):
    s = cfg(name)
    log(f"pairlist {name} n={s.n_res}")
    c = ctx_for(P, s)
    c.build_pairlist()
    got = c.get_pairlist()
    ref = orc.OracleSystem(s, RunParams()).pairlist(s.x)
    assert got.shape == ref.shape
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_pairlist_all_tile_sizes(P, orc, tile):
    s = cfg("c1")
    x = perturbed(s, 0.5, seed=tile)   # the list build evaluates no bond terms
    c = ctx_for(P, s, x=x, tile=tile)
    c.build_pairlist()
    ref = orc.OracleSystem(s, RunParams()).pairlist(x)
    assert np.array_equal(c.get_pairlist(), ref)


def test_pairlist_after_dynamics(P, orc):
    s = cfg("c1")
    c = ctx_for(P, s)
    c.step(137)
    x = c.get_coordinates()
    c.build_pairlist()
    ref = orc.OracleSystem(s, RunParams()).pairlist(x)
    assert np.array_equal(c.get_pairlist(), ref)


# --------------------------------------------------------------------------
# forces and energies
# --------------------------------------------------------------------------

@pytest.mark.parametrize("start", ["perturbed", "native"])
@pytest.mark.parametrize("name", ["c0", "c1", "c2", "c3s", "c4"])
def test_forces_and_energies(P, orc, name, start):
    """At a perturbed start and at the generated (native) structure, where the
    bonded and native terms vanish and the list pairs carry the force."""
    s = cfg(name)
    x = perturbed(s) if start == "perturbed" else s.x.copy()
    log(f"forces {name} ({start}) n={s.n_res}")
    c = ctx_for(P, s, x=x)
    c.set_step(1234)
    F, E, fe = c.compute_forces()
    o = orc.OracleSystem(s, RunParams())
    Fo, Eo, feo, S, Em = oracle_reference(o, x, step=1234)
    assert_forces(F, Fo, S, f"{name} {start}")
    assert_energies(E, Eo, Em, s.res_offsets, f"{name} {start}")
    assert np.allclose(fe, feo, rtol=1e-5, atol=1e-9)


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_forces_all_tile_sizes(P, orc, tile):
    s = cfg("c1")
    x = perturbed(s, seed=2)
    c = ctx_for(P, s, x=x, tile=tile)
    F, E, _ = c.compute_forces()
    Fo, Eo, _, S, Em = oracle_reference(orc.OracleSystem(s, RunParams()), x)
    assert_forces(F, Fo, S, f"tile {tile}")
    assert_energies(E, Eo, Em, s.res_offsets, f"tile {tile}")


def test_newton_third_law_on_gpu(P):
    s = cfg("c2")
    s2 = cap_of(s, s.n_res)
    s2.tip = None
    s2.fixed = None
    c = ctx_for(P, s2, x=perturbed(s2))
    F, _, _ = c.compute_forces()
    assert np.abs(F.sum(0)).max() < 2e-5 * np.abs(F).sum()


# --------------------------------------------------------------------------
# trajectories
# --------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0", "c1", "c2cap"])
def test_trajectory_200_steps(P, orc, name):
    s = cfg(name)
    p = RunParams()
    log(f"trajectory {name} n={s.n_res}")
    c = ctx_for(P, s, p, energy_every=10)
    c.step(200)
    xg = c.get_coordinates()
    Eg, estep = c.get_energies()
    o = orc.OracleSystem(s, p)
    x190, _, _, st = o.run(s.x, 190)
    assert st == 0
    xo, Eo, _, st = o.run(x190, 10, step0=190, energy_every=10)
    assert st == 0
    d = np.linalg.norm(xg - xo, axis=1).max()
    log(f"  max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL
    assert estep == 190
    _, Em = o.force_scale(x190, step=190)
    assert_energies(Eg, Eo[0], Em, s.res_offsets, f"{name} step 190")


@pytest.mark.parametrize("tile", [128, 256])
def test_trajectory_other_tile_sizes(P, orc, tile):
    """The wider tiles split a residue's work over two lanes (128) or keep
    it in one (256), so their noise draws and external terms take other
    paths than the default tile's."""
    s = cfg("c1")
    p = RunParams()
    c = ctx_for(P, s, p, tile=tile, energy_every=10)
    c.step(100)
    o = orc.OracleSystem(s, p)
    x90, _, _, st = o.run(s.x, 90)
    assert st == 0
    xo, Eo, _, st = o.run(x90, 10, step0=90, energy_every=10)
    assert st == 0
    d = float(np.linalg.norm(c.get_coordinates() - xo, axis=1).max())
    log(f"  tile {tile}: 100-step max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL
    Eg, estep = c.get_energies()
    assert estep == 90
    _, Em = o.force_scale(x90, step=90)
    assert_energies(Eg, Eo[0], Em, s.res_offsets, f"tile {tile} step 90")


def test_graph_replay_equals_direct_launches(P):
    s = cfg("c1")
    a = ctx_for(P, s, graph_steps=1, energy_every=20)
    b = ctx_for(P, s, graph_steps=0, energy_every=20)
    for n in [3, 7, 40, 5]:     # crosses period boundaries in both orders
        a.step(n)
        b.step(n)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    Ea, sa = a.get_energies()
    Eb, sb = b.get_energies()
    assert sa == sb == 40
    assert np.array_equal(Ea, Eb)


def test_graph_span_change_and_energy_alignment(P):
    """Changing the graph span drops the captured graphs, and a graph never
    starts where a record step would fall inside it: with 2-period graphs and
    energies every 20 steps, steps [10, 40] from 0 record step 40, exactly as
    kernel-by-kernel launches do."""
    s = cfg("c1")
    a = ctx_for(P, s, graph_steps=1, energy_every=20)
    b = ctx_for(P, s, graph_steps=0, energy_every=20)
    a.step(20)
    b.step(20)
    a.set_graph_steps(2)
    for n in [10, 40]:
        a.step(n)
        b.step(n)
    assert a.get_step() == b.get_step() == 70
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    Ea, sa = a.get_energies()
    Eb, sb = b.get_energies()
    assert sa == sb == 60
    assert np.array_equal(Ea, Eb)


@pytest.mark.parametrize("graph_steps", [1, 0])
def test_energy_records_do_not_change_the_trajectory(P, graph_steps):
    """Record steps run the step kernel's energy variant; its forces and
    update have the same bits as those of the plain variant."""
    s = cfg("c2cap")
    a = ctx_for(P, s, graph_steps=graph_steps, energy_every=0)
    b = ctx_for(P, s, graph_steps=graph_steps, energy_every=10)
    a.step(60)
    b.step(60)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    assert b.get_energies()[1] == 50


def test_runs_are_bit_reproducible(P):
    s = cfg("c2cap")
    xs = []
    for _ in range(2):
        c = ctx_for(P, s)
        c.step(60)
        xs.append(c.get_coordinates())
        c.close()
    assert np.array_equal(xs[0], xs[1])


def test_resume_at_period_boundary_is_exact(P):
    s = cfg("c1")
    a = ctx_for(P, s)
    a.step(40)
    xa = a.get_coordinates()
    b = ctx_for(P, s)
    b.step(20)
    mid = b.get_coordinates()
    c = ctx_for(P, s, x=mid)
    c.set_step(20)
    c.step(20)
    assert np.array_equal(c.get_coordinates(), xa)


def test_fixed_residue_and_cantilever(P, orc):
    s = cfg("c1")
    c = ctx_for(P, s, energy_every=10)
    x0 = c.get_coordinates()
    c.step(30)
    x = c.get_coordinates()
    assert np.array_equal(x[0], x0[0])
    assert not np.array_equal(x[1], x0[1])
    fe = c.get_external_force()
    _, _, feo, _ = orc.OracleSystem(s, RunParams()).run(s.x, 30, energy_every=10)
    assert np.allclose(fe, feo[-1], rtol=1e-4, atol=1e-6)


# --------------------------------------------------------------------------
# error paths, forced from the host
# --------------------------------------------------------------------------

def test_stretched_bond_is_reported(P):
    s = cfg("c0")
    x = s.x.copy()
    b = x[10] - x[9]
    x[10:] += 2.5 * b / np.linalg.norm(b)   # bond 9-10 stretched past R0
    c = ctx_for(P, s, x=x)
    with pytest.raises(P.SopError) as e:
        c.compute_forces()
    assert e.value.name == "SOP_E_FENE"
    c.set_coordinates(s.x)            # clears the sticky error
    c.compute_forces()


def test_list_overflow_is_reported(P):
    s = cfg("c1")
    c = ctx_for(P, s, RunParams(list_capacity=16))
    c.build_pairlist()
    with pytest.raises(P.SopError) as e:
        c.synchronize()
    assert e.value.name == "SOP_E_LIST_OVERFLOW"


def test_tip_contact_is_reported(P):
    s = make_config("c0")
    s.tip = Tip(5.0, 1.0, 1.0, s.x[3].copy(), np.zeros(3))
    c = ctx_for(P, s)
    with pytest.raises(P.SopError) as e:
        c.compute_forces()
    assert e.value.name == "SOP_E_TIP"


def test_coincident_residues_are_reported(P):
    from synth.structures import System
    x = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [5.0, 0.0, 0.0]])
    s = System("coincident", x, np.array([0, 3], np.int64), np.zeros(1, np.uint32),
               np.zeros(3, np.int32), np.zeros((0, 2), np.int32), np.zeros(0),
               np.zeros((0, 2), np.int32), np.zeros(0))
    c = ctx_for(P, s)
    c.step(1)
    with pytest.raises(P.SopError) as e:
        c.synchronize()
    assert e.value.name == "SOP_E_NONFINITE"
    with pytest.raises(P.SopError):
        c.set_coordinates(np.full_like(x, np.nan))   # rejected on the host


def test_step_timing_leaves_the_state(P):
    """Timing runs the kernels on a copy of the state and restores it."""
    s = cfg("c1")
    a = ctx_for(P, s)
    a.step(20)
    x0 = a.get_coordinates()
    k_ms, search_ms, filter_ms = a.step_timed(40)
    assert k_ms > 0.0 and search_ms > filter_ms > 0.0
    assert a.get_step() == 20
    assert np.array_equal(a.get_coordinates(), x0)
    a.step(10)
    b = ctx_for(P, s)
    b.step(30)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
