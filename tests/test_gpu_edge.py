"""Edge cases of the input shape, on both schedules, against the FP64 oracle.

One system holds the degenerate and ragged trajectories the method allows:
empty trajectories (no residues), a single free residue, a bonded pair,
chains just below, at and above one 64-residue tile, a trajectory of three
chains (one of them a single residue, so that natives cross chains and a
tile starts inside a trajectory), and a 1,024-residue chain, the longest a
batched workgroup holds. Pair lists must be bit-exact, forces within 1e-5
(L2 and residue by residue against the oracle's force scale), 60-step trajectories (six list rebuilds) within 1e-4 A, and the
energies of the empty trajectories exactly zero.
"""
import sys

import numpy as np
import pytest

from synth import RunParams
from synth.structures import _system, saw_batch

from parity import assert_energies, assert_forces, oracle_reference

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-5
TRAJ_TOL = 1e-4
LENGTHS = [1, 0, 2, 3, 5, 63, 64, 65, 129, 0, "3 chains", 1024]


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
def edge():
    rng = np.random.default_rng(17)
    sizes = [n for n in LENGTHS if isinstance(n, int) and n > 0] + [40, 1, 30]
    walks = iter(saw_batch(np.array(sizes), rng))
    trajs = []
    for n in LENGTHS:
        if n == "3 chains":
            continue
        trajs.append([next(walks)] if n else [])
    a, b, c = next(walks), next(walks), next(walks)
    # three chains of one trajectory, moved along random directions from the
    # first one until they are 4 A clear of it: close enough to share natives
    for k, w in ((1, b), (2, c)):
        placed = [a] if k == 1 else [a, b]
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        w = w - w.mean(0) + a.mean(0)
        while min(np.linalg.norm(w[:, None] - q[None], axis=2).min() for q in placed) < 4.0:
            w = w + 0.5 * u
        b, c = (w, c) if k == 1 else (b, w)
    trajs.insert(LENGTHS.index("3 chains"), [a, b, c])
    trajs = [[w - w.mean(0) for w in t] if len(t) == 1 else t for t in trajs]
    s = _system("edge cases", trajs)
    x = s.x + 0.1 * np.random.default_rng(5).standard_normal(s.x.shape)
    return s, x


def ctx(P, s, x, schedule, p=None, energy_every=0):
    batch = (0, 20) if schedule == "batched" else None
    return P.from_system(s, p or RunParams(), coordinates=x, schedule=schedule, batch=batch,
                         energy_every=energy_every)


def test_edge_system_shape(edge):
    s, _ = edge
    n = np.diff(s.res_offsets)
    assert list(n[:10]) == [1, 0, 2, 3, 5, 63, 64, 65, 129, 0]
    assert n[-1] == 1024 and n[-2] == 71
    t = len(n) - 2  # the three-chain trajectory has natives between its chains
    lo, hi = s.res_offsets[t], s.res_offsets[t + 1]
    inside = (s.natives[:, 0] >= lo) & (s.natives[:, 1] < hi)
    cross = s.chain_id[s.natives[inside, 0]] != s.chain_id[s.natives[inside, 1]]
    assert cross.any()


@pytest.mark.parametrize("schedule", ["plain", "batched"])
def test_edge_pairlist_and_forces(P, orc, edge, schedule):
    s, x = edge
    log(f"edge cases, {schedule}: n={s.n_res}, {s.n_traj} trajectories")
    c = ctx(P, s, x, schedule)
    c.build_pairlist()
    o = orc.OracleSystem(s, RunParams())
    assert np.array_equal(c.get_pairlist(), o.pairlist(x))
    F, E, _ = c.compute_forces()
    Fo, Eo, _, S, Em = oracle_reference(o, x)
    assert_forces(F, Fo, S, f"edge {schedule}")
    assert_energies(E, Eo, Em, s.res_offsets, f"edge {schedule}")
    assert np.all(F[s.res_offsets[0]] == 0.0)  # the single residue feels nothing
    empty = np.nonzero(np.diff(s.res_offsets) == 0)[0]
    assert np.all(E[empty] == 0.0) and np.all(Eo[empty] == 0.0)


@pytest.mark.parametrize("schedule", ["plain", "batched"])
def test_edge_trajectory_60_steps(P, orc, edge, schedule):
    s, x = edge
    p = RunParams()
    c = ctx(P, s, x, schedule, p, energy_every=20)
    c.step(60)
    xg = c.get_coordinates()
    Eg, estep = c.get_energies()
    o = orc.OracleSystem(s, p)
    x40, _, _, st = o.run(x, 40)
    assert st == 0
    xo, Eo, _, st = o.run(x40, 20, step0=40, energy_every=20)
    assert st == 0
    d = np.linalg.norm(xg - xo, axis=1)
    log(f"  {schedule}: 60-step max |dx| {d.max():.3e} A")
    assert d.max() <= TRAJ_TOL
    assert estep == 40
    empty = np.nonzero(np.diff(s.res_offsets) == 0)[0]
    assert np.all(Eg[empty] == 0.0)
    _, Em = o.force_scale(x40, step=40)
    assert_energies(Eg, Eo[0], Em, s.res_offsets, f"edge {schedule} step 40")
