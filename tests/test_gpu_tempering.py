"""Replica exchange on the batched schedule against the oracle: groups of
replicas of one chain at a ladder of temperatures, Metropolis swaps every 50
steps; the temperature assignments, swap counts and trajectories must match
the oracle's run from the same start and Philox streams."""
import sys

import numpy as np
import pytest

from synth import RunParams, make_config
from synth.structures import System

from parity import TRAJ_TOL

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


def replicas(base, R):
    """Each trajectory of `base` repeated R times in a row (one group each)."""
    xs, offs, bonds, br0, nats, nr0, chain = [], [0], [], [], [], [], []
    for t in range(base.n_traj):
        a, b = int(base.res_offsets[t]), int(base.res_offsets[t + 1])
        kb = (base.bonds[:, 0] >= a) & (base.bonds[:, 0] < b)
        kn = (base.natives[:, 0] >= a) & (base.natives[:, 0] < b)
        for r in range(R):
            o = offs[-1]
            xs.append(base.x[a:b])
            bonds.append(base.bonds[kb] - a + o)
            br0.append(base.bond_r0[kb])
            nats.append(base.natives[kn] - a + o)
            nr0.append(base.native_r0[kn])
            chain.append(np.full(b - a, len(offs) - 1, np.int32))
            offs.append(o + b - a)
    T = len(offs) - 1
    return System("replicas", np.concatenate(xs), np.asarray(offs, np.int64),
                  np.arange(T, dtype=np.uint32), np.concatenate(chain),
                  np.concatenate(bonds).astype(np.int32), np.concatenate(br0),
                  np.concatenate(nats).astype(np.int32), np.concatenate(nr0))


@pytest.mark.parametrize("R", [2, 4])
def test_tempering_matches_the_oracle(P, orc, R):
    base = make_config("c3", n_traj=6)
    s = replicas(base, R)
    p = RunParams()
    kbt = p.kBT * np.array([1.0, 1.15, 1.3, 1.5])[:R]
    c = P.from_system(s, p, schedule="batched", batch=(512, 50))
    c.set_tempering(kbt, 50)
    c.step(300)
    tg, accg, attg = c.get_tempering()
    xg = c.get_coordinates()
    o = orc.OracleSystem(s, p)
    xo, to, acco, atto, st = o.run_tempered(s.x, 300, kbt, 50, np.arange(s.n_traj) % R)
    assert st == 0
    log(f"  R={R}: accepted {list(accg)} of {list(attg)} (oracle {list(acco)} of {list(atto)})")
    assert np.array_equal(attg, atto)
    assert np.array_equal(accg, acco)
    assert np.array_equal(tg, to)
    d = float(np.linalg.norm(xg - xo, axis=1).max())
    log(f"  R={R}: 300-step max |dx| {d:.3e} A")
    assert d <= TRAJ_TOL
    c.close()


def test_tempering_arguments(P):
    base = make_config("c3", n_traj=4)
    s = replicas(base, 2)
    p = RunParams()
    c = P.from_system(s, p, schedule="batched")
    with pytest.raises(P.SopError):
        c.set_tempering(p.kBT * np.ones(3), 10)          # 3 does not divide 8
    with pytest.raises(P.SopError):
        c.set_tempering(p.kBT * np.array([1.0, -1.0]), 10)
    with pytest.raises(P.SopError):
        c.set_tempering(p.kBT * np.ones(2), 10, tidx=np.zeros(8))   # not a permutation
    c.set_tempering(p.kBT * np.ones(2), 10)
    c.step(40)
    tg, acc, att = c.get_tempering()
    assert att[0] == 4 * 2 and acc[0] == att[0]   # equal temperatures: every swap accepted
    c.close()
    d = P.from_system(s, p)   # plain schedule: no tempering
    with pytest.raises(P.SopError):
        d.set_tempering(p.kBT * np.ones(2), 10)
    d.close()
