"""The Verlet skin of the plain schedule: the cell-grid search runs at
r_list + skin only when a residue has moved more than skin/2 since the last
search, and each rebuild filters those rows to r_list.  The filtered list
must equal the oracle's list of all pairs closer than r_list (bit-exact, as
sorted sets) at every rebuild, whatever the skin, and the trajectories must
not depend on the skin beyond summation order."""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config

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
def c1():
    return make_config("c1")


@pytest.mark.parametrize("skin", [0.0, 0.1, 1.0, 4.0])
def test_list_equals_all_pairs_at_every_rebuild(P, orc, c1, skin):
    """30 list periods of the pulled globule; after each, the list the next
    period uses (a rebuild in cadence, so the skin is filtered unless the
    displacement check asked for a new search) equals the oracle's."""
    p = RunParams()
    o = orc.OracleSystem(c1, p)
    c = P.from_system(c1, p)
    c.set_list_skin(skin)
    for period in range(30):
        c.step(p.list_every)
        c.build_pairlist()
        got = c.get_pairlist()
        x = c.get_coordinates()
        ref = o.pairlist(x)
        assert np.array_equal(got, ref), (skin, period, len(got), len(ref))
    rebuilds, searches = c.get_list_stats()
    log(f"skin {skin}: {rebuilds} rebuilds, {searches} cell-grid searches")
    if skin == 0.0:
        assert searches == rebuilds
    if skin >= 4.0:
        assert searches < rebuilds // 2
    c.close()


def test_skin_does_not_change_the_dynamics(P, c1):
    """The same 400 steps with skin 0 and skin 4: the same list at every
    step, each row in ascending partner order, so the trajectories are
    bit-identical."""
    p = RunParams()
    a = P.from_system(c1, p, graph_steps=2)
    a.set_list_skin(0.0)
    b = P.from_system(c1, p, graph_steps=2)
    b.set_list_skin(4.0)
    a.step(400)
    b.step(400)
    xa, xb = a.get_coordinates(), b.get_coordinates()
    d = float(np.linalg.norm(xa - xb, axis=1).max())
    log(f"skin 0 vs 4 after 400 steps: max |dx| {d:.3e} A")
    assert np.array_equal(xa, xb)
    ra, sa = a.get_list_stats()
    rb, sb = b.get_list_stats()
    assert ra == rb == 40
    assert sa == 40 and sb < 20
    a.close()
    b.close()


@pytest.mark.parametrize("skin", [0.0, 4.0])
def test_graph_and_direct_paths_search_alike(P, c1, skin):
    """Graph replays rely on the displacement check of each period's last
    step (or, without a skin, search at every captured rebuild); step-by-step
    launches do the same: bit-identical results."""
    p = RunParams()
    a = P.from_system(c1, p, graph_steps=3)
    b = P.from_system(c1, p, graph_steps=0)
    a.set_list_skin(skin)
    b.set_list_skin(skin)
    for n in (30, 7, 23, 60, 5, 125):
        a.step(n)
        b.step(n)
    assert np.array_equal(a.get_coordinates(), b.get_coordinates())
    assert a.get_list_stats() == b.get_list_stats()
    a.close()
    b.close()


def test_coordinates_force_a_search(P, c1):
    p = RunParams()
    c = P.from_system(c1, p)
    c.step(20)
    r0, s0 = c.get_list_stats()
    c.set_coordinates(c1.x)
    c.step(10)
    r1, s1 = c.get_list_stats()
    assert (r1 - r0, s1 - s0) == (1, 1)
    c.set_step(5)   # off the period: the next rebuild searches again
    c.step(10)
    r2, s2 = c.get_list_stats()
    assert r2 - r1 == 2 and s2 - s1 >= 1
    c.close()
