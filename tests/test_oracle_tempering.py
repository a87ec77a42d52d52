"""Pins of the oracle's replica exchange (parallel tempering over groups of
trajectories): one replica reduces to the plain integrator, equal
temperatures accept every swap, and two temperatures of a harmonic tether
accept swaps at the rate the Boltzmann distributions fix."""
import math

import numpy as np
import pytest

from synth import RunParams, make_config
from synth.structures import Pull, System


def tethers(x, K):
    m = len(x)
    pulls = [Pull(t, t, K, np.zeros(3), np.zeros(3)) for t in range(m)]
    return System("tethers", np.asarray(x, np.float64), np.arange(m + 1, dtype=np.int64),
                  np.arange(m, dtype=np.uint32), np.zeros(m, np.int32),
                  np.zeros((0, 2), np.int32), np.zeros(0), np.zeros((0, 2), np.int32), np.zeros(0),
                  None, pulls)


def test_one_replica_is_the_plain_integrator(orc):
    s = make_config("c3", n_traj=6)
    p = RunParams()
    o = orc.OracleSystem(s, p)
    kbt = np.array([p.kBT])
    x1, tidx, acc, att, st = o.run_tempered(s.x, 60, kbt, 20, np.zeros(6, np.int32))
    x2, _, _, st2 = o.run(s.x, 60)
    assert st == st2 == 0
    assert np.array_equal(x1, x2)
    assert not tidx.any()


def test_equal_temperatures_accept_every_swap(orc):
    s = make_config("c3", n_traj=8)
    p = RunParams()
    o = orc.OracleSystem(s, p)
    kbt = np.full(4, p.kBT)
    tidx0 = np.tile(np.arange(4, dtype=np.int32), 2)
    x, tidx, acc, att, st = o.run_tempered(s.x, 50, kbt, 10, tidx0)
    assert st == 0
    # rounds 0..4 at steps 0, 10, .., 40: pairs (0,1),(2,3) on even rounds, (1,2) on odd
    assert list(att) == [3 * 2, 2 * 2, 3 * 2] and np.array_equal(acc, att)
    # the temperature indices move like the swaps say: five alternating rounds
    perm = list(range(4))  # perm[k] = member holding temperature k
    for r in range(5):
        for k in range(r % 2, 3, 2):
            perm[k], perm[k + 1] = perm[k + 1], perm[k]
    expect = np.empty(4, np.int32)
    for k, member in enumerate(perm):
        expect[member] = k
    assert np.array_equal(tidx, np.tile(expect, 2))


def test_acceptance_rate_of_two_harmonic_replicas(orc):
    """Two replicas of a three-dimensional harmonic tether, E = K |x|^2 / 2,
    at kB T1 < kB T2: in equilibrium E ~ Gamma(3/2, kB T), and the Metropolis
    swap is accepted with probability E[min(1, exp((1/kT1 - 1/kT2)(E1 - E2)))]."""
    K = 1.0
    p = RunParams(r_list=1e-3)
    t1, t2 = p.kBT, 1.6 * p.kBT
    m = 500  # groups
    rng = np.random.default_rng(12)
    x = np.empty((2 * m, 3))
    x[0::2] = rng.normal(scale=math.sqrt(t1 / K), size=(m, 3))
    x[1::2] = rng.normal(scale=math.sqrt(t2 / K), size=(m, 3))
    s = tethers(x, K)
    o = orc.OracleSystem(s, p)
    # exchange every 1,500 steps: 2.4 relaxation times zeta/(K h) = 625 steps
    xe, tidx, acc, att, st = o.run_tempered(s.x, 3001, np.array([t1, t2]), 1500,
                                            np.tile(np.array([0, 1], np.int32), m))
    assert st == 0
    assert att[0] == 2 * m      # rounds 0 and 2 (steps 0 and 3,000)
    rate = acc[0] / att[0]
    g = np.random.default_rng(13)
    e1 = g.gamma(1.5, t1, size=2_000_000)
    e2 = g.gamma(1.5, t2, size=2_000_000)
    expect = np.minimum(1.0, np.exp((1 / t1 - 1 / t2) * (e1 - e2))).mean()
    sd = math.sqrt(expect * (1 - expect) / att[0])
    assert abs(rate - expect) < 5 * sd + 2e-3, (rate, expect)
    # a swap rule of the wrong sign would accept nearly everything
    assert expect < 0.85
