"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every function include/sop.h declares, and validates arguments and call
order before touching a device."""
import ctypes as C

import numpy as np
import pytest

from synth import RunParams, make_config

P = pytest.importorskip("paper_1003_1148_amd")


@pytest.fixture(scope="module")
def lib():
    try:
        return P.lib()
    except ImportError as e:  # the build step must have run
        pytest.fail(str(e))


def test_exports_every_declared_symbol(lib):
    names = P.declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings(lib):
    for st in [0, -1, -2, -3, -4, -5, -6, -7, -8]:
        assert P.status_string(st)


def test_create_rejects_bad_params(lib):
    for bad in [dict(h=0.0), dict(zeta=-1.0), dict(list_every=0), dict(r_list=-1.0)]:
        with pytest.raises(P.SopError) as e:
            P.Context(RunParams(**bad))
        assert e.value.name == "SOP_E_ARG"


def _ctx(s):
    c = P.Context(RunParams())
    c.load_topology(s.res_offsets, s.bonds, s.bond_r0, s.natives, s.native_r0)
    return c


def test_topology_validation(lib):
    s = make_config("c0")
    c = P.Context(RunParams())
    cases = {
        "out of range": (s.res_offsets, [[0, 56]], [3.8], s.natives, s.native_r0),
        "self pair": (s.res_offsets, [[3, 3]], [3.8], s.natives, s.native_r0),
        "r0 <= 0": (s.res_offsets, [[0, 1]], [0.0], s.natives, s.native_r0),
        "duplicate": (s.res_offsets, [[0, 1], [1, 0]], [3.8, 3.8], s.natives, s.native_r0),
        "bonded and native": (s.res_offsets, [[0, 1]], [3.8], [[0, 1]], [5.0]),
        "across trajectories": ([0, 28, 56], [[27, 28]], [3.8], np.zeros((0, 2)), []),
        "bad offsets": ([0, 30, 20], [[0, 1]], [3.8], np.zeros((0, 2)), []),
    }
    for name, args in cases.items():
        with pytest.raises(P.SopError) as e:
            c.load_topology(*args)
        assert e.value.name == "SOP_E_ARG", name
    c.load_topology(s.res_offsets, s.bonds, s.bond_r0, s.natives, s.native_r0)


def test_call_order_is_enforced(lib):
    s = make_config("c0")
    c = _ctx(s)
    for fn in [lambda: c.set_coordinates(s.x), lambda: c.step(1), lambda: c.build_pairlist(),
               lambda: c.compute_forces(), lambda: c.get_coordinates()]:
        with pytest.raises(P.SopError) as e:
            fn()
        assert e.value.name == "SOP_E_STATE"


def test_workspace_size_and_bind_checks(lib):
    s = make_config("c1")
    c = _ctx(s)
    n1 = c.workspace_size()
    c2 = P.Context(RunParams(list_capacity=256))  # below the default 1024 of the plain schedule
    c2.load_topology(s.res_offsets, s.bonds, s.bond_r0, s.natives, s.native_r0)
    n2 = c2.workspace_size()
    assert n1 > n2 > s.n_res * 64
    with pytest.raises(P.SopError) as e:
        P.Context(RunParams(list_capacity=1040))   # the largest row is 1024 entries
    assert e.value.name == "SOP_E_ARG"
    # null, misaligned or short workspaces are rejected before any device use
    L = P.lib()
    assert L.sop_bind_workspace(c.h, None, n1) == -3
    assert L.sop_bind_workspace(c.h, 0x1000 + 8, n1) == -3
    assert L.sop_bind_workspace(c.h, 0x100000, n1 - 1) == -3


def test_protocol_and_schedule_validation(lib):
    s = make_config("c1")
    c = _ctx(s)
    with pytest.raises(P.SopError):
        c.set_tile(96)
    with pytest.raises(P.SopError):
        c.set_pulling(0, s.n_res, 1.0, np.zeros(3), np.zeros(3))   # residue out of range
    c.set_pulling(0, s.n_res - 1, 1.0, np.zeros(3), np.zeros(3))
    with pytest.raises(P.SopError):
        c.set_pulling(0, s.n_res - 1, 1.0, np.zeros(3), np.zeros(3))  # second on one residue
    with pytest.raises(P.SopError):
        c.set_tip(5.0, 1.0, 0.0, np.zeros(3), np.zeros(3))      # sigma <= 0
    c.set_tip(5.0, 1.0, 1.0, np.zeros(3), np.zeros(3))
    c.set_tip(-1.0, 0.0, 1.0, np.zeros(3), np.zeros(3))          # removes the tip
    for k in [64, 128, 256, 0]:
        c.set_tile(k)
    assert c.get_tile() in (64, 128, 256)


def test_batched_schedule_validation(lib):
    s = make_config("c3", n_traj=8)
    c = _ctx(s)
    longest = int(np.diff(s.res_offsets).max())
    assert longest > 256
    with pytest.raises(P.SopError):
        c.set_batch(256, 50)                      # smaller than the longest trajectory
    with pytest.raises(P.SopError):
        c.set_batch(300, 50)                      # not a supported workgroup size
    with pytest.raises(P.SopError):
        c.set_batch(0, 0)                         # steps per launch >= 1
    with pytest.raises(P.SopError):
        c.set_schedule(7)
    c.set_schedule("batched")
    c.set_batch(1024, 40)
    assert c.get_batch()[:2] == (1024, 40)
    c.set_batch(0, 40)
    assert c.get_batch()[0] == 512                # smallest that holds the longest chain
    n_batched = c.workspace_size()
    assert n_batched > 0
