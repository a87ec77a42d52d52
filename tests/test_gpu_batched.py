"""The batched ensemble schedule (one persistent launch over packs of whole
trajectories) against the FP64 oracle, plus its schedule invariances."""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config

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


@pytest.fixture(scope="module")
def ens():
    """48 trajectories of 50-500 residues (the ensemble's first 48 chains),
    with a cantilever on the last residue of trajectory 3 and residue 0 of
    trajectory 5 fixed."""
    from synth.structures import Pull
    s = make_config("c3", n_traj=48)
    t = 3
    last = int(s.res_offsets[t + 1] - 1)
    s.pulls = [Pull(t, last, 0.5, s.x[last] + np.array([0.5, 0.0, 0.0]), np.array([0.01, 0.0, 0.0]))]
    fixed = np.zeros(s.n_res, np.uint8)
    fixed[s.res_offsets[5]] = 1
    s.fixed = fixed
    return s


def ctx(P, s, x=None, wg=0, steps=50, energy_every=0, graph=1, p=None):
    return P.from_system(s, p or RunParams(), coordinates=x, schedule="batched",
                         batch=(wg, steps), energy_every=energy_every, graph_steps=graph)


def perturbed(s, sd=0.15, seed=1):
    rng = np.random.default_rng(seed)
    return s.x + sd * rng.standard_normal(s.x.shape)


def test_batched_pairlist_bit_exact(P, orc, ens):
    x = perturbed(ens)
    c = ctx(P, ens, x=x)
    c.build_pairlist()
    ref = orc.OracleSystem(ens, RunParams()).pairlist(x)
    assert np.array_equal(c.get_pairlist(), ref)


@pytest.mark.parametrize("start", ["perturbed", "native"])
def test_batched_forces_and_energies(P, orc, ens, start):
    x = perturbed(ens) if start == "perturbed" else ens.x.copy()
    c = ctx(P, ens, x=x)
    c.set_step(77)
    F, E, fe = c.compute_forces()
    Fo, Eo, feo, S, Em = oracle_reference(orc.OracleSystem(ens, RunParams()), x, step=77)
    assert_forces(F, Fo, S, f"batched {start}")
    assert_energies(E, Eo, Em, ens.res_offsets, f"batched {start}")
    assert np.allclose(fe, feo, rtol=1e-5, atol=1e-9)


def test_batched_trajectory_200_steps(P, orc, ens):
    p = RunParams()
    c = ctx(P, ens, energy_every=10, steps=30)    # launches that straddle list periods
    c.step(200)
    xg = c.get_coordinates()
    Eg, estep = c.get_energies()
    o = orc.OracleSystem(ens, p)
    x190, _, _, st = o.run(ens.x, 190)
    assert st == 0
    xo, Eo, feo, st = o.run(x190, 10, step0=190, energy_every=10)
    assert st == 0
    d = float(np.linalg.norm(xg - xo, axis=1).max())
    log(f"batched 200-step max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL
    assert estep == 190
    _, Em = o.force_scale(x190, step=190)
    assert_energies(Eg, Eo[0], Em, ens.res_offsets, "batched step 190")
    assert np.allclose(c.get_external_force(), feo[0], rtol=1e-4, atol=1e-9)
    assert np.array_equal(xg[ens.res_offsets[5]], c_first(P, ens)[ens.res_offsets[5]])


def far_ensemble(ens):
    """The ensemble with every trajectory moved 5e3-1e4 A from the origin in
    a seeded direction (the cantilever's anchor with it), where a
    coordinate's single-precision spacing is about 1e-3 A."""
    import copy
    s = copy.deepcopy(ens)
    rng = np.random.default_rng(17)
    for t in range(len(s.res_offsets) - 1):
        v = rng.standard_normal(3)
        v *= 1.0e4 * (0.5 + 0.5 * rng.random()) / np.linalg.norm(v)
        s.x[s.res_offsets[t]:s.res_offsets[t + 1]] += v
        for pl in s.pulls:
            if pl.traj == t:
                pl.anchor0 = pl.anchor0 + v
    return s


def test_batched_far_from_the_origin(P, orc, ens):
    """Forces element by element and a 200-step trajectory with every
    trajectory about 1e4 A out: the list pairs take the low parts too."""
    s = far_ensemble(ens)
    log(f"far ensemble: |x| up to {np.abs(s.x).max():.0f} A")
    x = perturbed(s)
    c = ctx(P, s, x=x)
    F, E, _ = c.compute_forces()
    o = orc.OracleSystem(s, RunParams())
    Fo, Eo, _, S, Em = oracle_reference(o, x)
    assert_forces(F, Fo, S, "batched far")
    assert_energies(E, Eo, Em, s.res_offsets, "batched far")
    c.close()
    c = ctx(P, s, steps=50)
    c.step(200)
    xg = c.get_coordinates()
    xo, _, _, st = o.run(s.x, 200)
    assert st == 0
    d = float(np.linalg.norm(xg - xo, axis=1).max())
    log(f"batched far 200-step max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL


def c_first(P, ens):
    return ctx(P, ens).get_coordinates()


def test_batched_results_do_not_depend_on_the_schedule(P, ens):
    """Packing and steps per launch change only how work maps to the GPU."""
    runs = []
    for wg, k, graph in [(512, 100, 1), (1024, 20, 1), (1024, 7, 0)]:
        c = ctx(P, ens, wg=wg, steps=k, graph=graph, energy_every=20)
        c.step(140)
        runs.append((c.get_coordinates(), c.get_energies()[0]))
        c.close()
    for x, E in runs[1:]:
        assert np.array_equal(x, runs[0][0])
        assert np.array_equal(E, runs[0][1])


@pytest.mark.parametrize("graph", [1, 0])
def test_energy_records_do_not_change_the_trajectory(P, ens, graph):
    """Launches without energy records run a kernel of their own; its forces
    and updates have the same bits as those of the recording kernel."""
    a = ctx(P, ens, steps=20, graph=graph, energy_every=0)
    b = ctx(P, ens, steps=20, graph=graph, energy_every=40)
    a.step(120)
    b.step(120)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    assert b.get_energies()[1] == 80
    a.close()
    b.close()


def test_batched_energy_interval_change(P, ens):
    """A new energy interval drops the captured launch graphs: energies and
    their step equal those of launches made without graphs."""
    a = ctx(P, ens, steps=20, graph=1, energy_every=20)
    b = ctx(P, ens, steps=20, graph=0, energy_every=20)
    a.step(40)
    b.step(40)
    for c in (a, b):
        c.set_energy_interval(10)
        c.step(30)
    Ea, sa = a.get_energies()
    Eb, sb = b.get_energies()
    assert sa == sb == 60
    assert np.array_equal(Ea, Eb)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    a.close()
    b.close()


def test_batched_resume_is_exact(P, ens):
    a = ctx(P, ens)
    a.step(60)
    b = ctx(P, ens)
    b.step(30)
    c = ctx(P, ens, x=b.get_coordinates())
    c.set_step(30)
    c.step(30)
    assert np.array_equal(a.get_coordinates(), c.get_coordinates())


def test_autotune_keeps_state_and_uses_cache(P, ens, tmp_path):
    cache = str(tmp_path / "tune.txt")
    a = ctx(P, ens)
    x0 = a.get_coordinates()
    a.autotune(budget_ms=100.0, cache_path=cache)
    assert np.array_equal(a.get_coordinates(), x0)
    assert a.get_step() == 0
    choice = a.get_batch()
    a.step(40)
    b = ctx(P, ens)
    b.step(40)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    # a second context picks the cached choice without timing
    c = ctx(P, ens, wg=1024, steps=7)
    c.autotune(budget_ms=100.0, cache_path=cache)
    assert c.get_batch() == choice
    with open(cache) as f:
        assert len(f.read().strip().splitlines()) == 1


def test_plain_autotune_keeps_state(P):
    s = make_config("c1")
    c = P.from_system(s, RunParams())
    x0 = c.get_coordinates()
    c.autotune(budget_ms=50.0)
    assert np.array_equal(c.get_coordinates(), x0)
    assert c.get_tile() in (64, 128, 256)
    c.step(20)
    c.synchronize()


def test_batched_matches_plain_to_tolerance(P, ens):
    a = ctx(P, ens)
    b = P.from_system(ens, RunParams())
    a.step(100)
    b.step(100)
    d = float(np.linalg.norm(a.get_coordinates() - b.get_coordinates(), axis=1).max())
    assert d <= TRAJ_TOL


@pytest.fixture(scope="module")
def dense():
    """Three compact 120-residue globules whose native contacts reach 12 A:
    about 22 bonded/native entries per residue, more than the batched kernel
    keeps in LDS (8 per slot on average), so the entries past that capacity
    are read from global memory."""
    from synth.structures import System, globule, topology_from_chains
    chains = [[globule(120, seed)] for seed in (11, 12, 13)]
    x, offs, cid, b, br0, nn, nr0 = topology_from_chains(chains, native_cutoff=12.0)
    return System("dense natives", x, offs, np.arange(3, dtype=np.uint32), cid, b, br0, nn, nr0)


def test_batched_dense_topology(P, orc, dense):
    ntop = np.bincount(np.concatenate([dense.bonds.ravel(), dense.natives.ravel()]),
                       minlength=dense.n_res)
    assert ntop.mean() > 16  # well past the LDS share of a pack
    x = perturbed(dense, sd=0.1, seed=4)
    o = orc.OracleSystem(dense, RunParams())
    for wg in (256, 512):
        c = ctx(P, dense, x=x, wg=wg)
        c.build_pairlist()
        assert np.array_equal(c.get_pairlist(), o.pairlist(x))
        c.set_step(5)
        F, E, fe = c.compute_forces()
        Fo, Eo, feo, S, Em = oracle_reference(o, x, step=5)
        assert_forces(F, Fo, S, f"dense topology, {wg}-slot packs")
        assert_energies(E, Eo, Em, dense.res_offsets, f"dense topology, {wg}-slot packs")
        c.close()
    # trajectories against the oracle, and the same bits for both packings
    runs = []
    for wg, k in [(256, 30), (512, 7)]:
        c = ctx(P, dense, wg=wg, steps=k)
        c.step(100)
        runs.append(c.get_coordinates())
        c.close()
    assert np.array_equal(runs[0], runs[1])
    xo, _, _, st = o.run(dense.x, 100)
    assert st == 0
    d = float(np.linalg.norm(runs[0] - xo, axis=1).max())
    log(f"dense topology 100-step max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL


def ffd_pack_count(lengths, wg):
    """First-fit decreasing (ties by index), the packing the library states."""
    room = []
    for L in sorted(lengths, key=lambda v: -v):
        for k in range(len(room)):
            if room[k] >= L:
                room[k] -= L
                break
        else:
            room.append(wg - L)
    return len(room)


def test_batched_packs_first_fit_decreasing(P, ens):
    lengths = np.diff(ens.res_offsets).tolist()
    for wg in (512, 1024):
        c = ctx(P, ens, wg=wg)
        w, k, n_packs = c.get_batch()
        assert w == wg
        assert n_packs == ffd_pack_count(lengths, wg)
        c.close()


def test_batched_list_overflow_is_reported(P, ens):
    """Rows longer than the list capacity stop at the capacity (the sums
    read only that far) and raise the overflow error at the next sync."""
    c = ctx(P, ens, p=RunParams(list_capacity=16))
    c.step(20)
    with pytest.raises(P.SopError) as e:
        c.synchronize()
    assert e.value.name == "SOP_E_LIST_OVERFLOW"
    c.close()


def test_equipartition_matches_the_oracle(P, orc):
    """The virial temperature of 24 free 56-residue chains (independent noise
    streams) on the batched schedule against the oracle's on the same
    ensemble, 4,000 steps after the start and over 4,000 more: the two agree
    to 1e-4 (same noise, same starts; the trajectories stay within about
    1e-6 A of each other), and both lie within 8% of the bath's 300 K (the
    slowest modes and the O(h) bias of the first-order scheme)."""
    from synth.structures import _system
    base = make_config("c0")
    m = 24
    s = _system("c0 x 24", [[base.x.copy()] for _ in range(m)])
    p = RunParams()
    kB = p.kBT / 300.0
    burn, every, n_rec = 4000, 10, 400
    c = ctx(P, s, steps=every, energy_every=every)
    c.step(burn)
    Wg = []
    for _ in range(n_rec):
        c.step(every)
        E, _ = c.get_energies()
        Wg.append(E[:, 4].copy())
    Wg = np.array(Wg)                        # (records, chains)
    o = orc.OracleSystem(s, p)
    _, Eo, _, st = o.run_par(s.x, burn + every * n_rec, energy_every=every)
    assert st == 0
    Wo = Eo[burn // every:, :, 4]            # records at steps burn .. burn + every (n_rec - 1)
    assert Wo.shape == Wg.shape
    Tg = P.virial_temperature(Wg.ravel(), base.n_res, kB)
    To = P.virial_temperature(Wo.ravel(), base.n_res, kB)
    log(f"virial temperature: GPU {Tg:.3f} K, oracle {To:.3f} K")
    assert abs(Tg - To) <= 1e-4 * To
    assert abs(Tg - 300.0) <= 0.08 * 300.0 and abs(To - 300.0) <= 0.08 * 300.0
    c.close()
