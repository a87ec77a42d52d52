"""Pins of the oracle's underdamped Langevin integrator (BAOAB, Leimkuhler and
Matthews 2013) against properties the mathematics fixes: the exact
Ornstein-Uhlenbeck velocity variance of free particles, the conserved
quadratic form of velocity Verlet (the zero-friction, zero-temperature
limit) for a harmonic oscillator, BAOAB's exact configurational variance
kB T / K for a harmonic oscillator, fixed residues, and resumes."""
import math

import numpy as np
import pytest

from synth import RunParams
from synth.structures import Pull, System


def singles(x, pulls=(), fixed=None):
    """Independent one-residue trajectories at x (no bonds, no natives)."""
    m = len(x)
    return System("singles", np.asarray(x, np.float64), np.arange(m + 1, dtype=np.int64),
                  np.arange(m, dtype=np.uint32), np.zeros(m, np.int32),
                  np.zeros((0, 2), np.int32), np.zeros(0), np.zeros((0, 2), np.int32), np.zeros(0),
                  fixed, list(pulls))


def tethered(m, K, seed=0):
    """m one-residue trajectories, each on a cantilever of spring K anchored
    at the origin (a three-dimensional harmonic oscillator)."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1.0, 1.0, size=(m, 3))
    pulls = [Pull(t, t, K, np.zeros(3), np.zeros(3)) for t in range(m)]
    return singles(x, pulls)


def test_free_particle_velocity_variance(orc):
    p = RunParams(r_list=1e-3, zeta=2.0)
    mass, m, n = 3.0, 6000, 25
    s = singles(np.zeros((m, 3)))
    o = orc.OracleSystem(s, p)
    x, v, st = o.run_underdamped(s.x, np.zeros((m, 3)), n, mass)
    assert st == 0
    c1 = math.exp(-p.zeta / mass * p.h)
    var = p.kBT / mass * (1.0 - c1 ** (2 * n))
    assert v.mean() == pytest.approx(0.0, abs=5 * math.sqrt(var / (3 * m)))
    assert v.var() == pytest.approx(var, rel=5 * math.sqrt(2.0 / (3 * m)))


def test_zero_friction_harmonic_conserves_the_verlet_invariant(orc):
    """kB T = 0 and zeta = 0: BAOAB is velocity Verlet, which keeps
    v^2 + w^2 (1 - h^2 w^2 / 4) x^2 exactly constant on x'' = -w^2 x."""
    K, mass = 2.5, 1.7
    p = RunParams(r_list=1e-3, zeta=0.0, kBT=0.0, h=0.3)
    s = tethered(3, K, seed=4)
    o = orc.OracleSystem(s, p)
    rng = np.random.default_rng(5)
    v0 = rng.normal(size=(3, 3))
    w2 = K / mass

    def Q(x, v):
        return (v * v).sum(1) + w2 * (1 - p.h * p.h * w2 / 4) * (x * x).sum(1)
    q0 = Q(s.x, v0)
    x, v, st = o.run_underdamped(s.x, v0, 5000, mass)
    assert st == 0
    assert np.allclose(Q(x, v), q0, rtol=1e-11)
    # and it does move: the phase has turned by many periods
    assert np.abs(x - s.x).max() > 0.1


def test_harmonic_configurational_variance_is_exact(orc):
    """BAOAB samples x of a harmonic oscillator with variance exactly
    kB T / K whatever the step (Leimkuhler and Matthews)."""
    K, mass, m = 4.0, 1.0, 4000
    p = RunParams(r_list=1e-3, zeta=3.0, h=0.2)
    s = tethered(m, K, seed=7)
    o = orc.OracleSystem(s, p)
    x, v, st = o.run_underdamped(s.x, np.zeros((m, 3)), 400, mass)
    assert st == 0
    var = p.kBT / K
    assert (x * x).mean() == pytest.approx(var, rel=5 * math.sqrt(2.0 / (3 * m)))


def test_fixed_residues_and_resume(orc):
    p = RunParams(r_list=1e-3, zeta=1.0)
    rng = np.random.default_rng(8)
    x0 = rng.uniform(-5, 5, size=(50, 3))
    fixed = np.zeros(50, np.uint8)
    fixed[[3, 17]] = 1
    s = singles(x0, fixed=fixed)
    o = orc.OracleSystem(s, p)
    v0 = rng.normal(size=(50, 3))
    x, v, st = o.run_underdamped(x0, v0, 40, 2.0)
    assert st == 0
    assert np.array_equal(x[[3, 17]], x0[[3, 17]]) and not v[[3, 17]].any()
    xa, va, _ = o.run_underdamped(x0, v0, 20, 2.0)
    xb, vb, _ = o.run_underdamped(xa, va, 20, 2.0, step0=20)
    assert np.array_equal(xb, x) and np.array_equal(vb, v)


def test_rejects_a_nonpositive_mass(orc):
    s = singles(np.zeros((2, 3)))
    o = orc.OracleSystem(s, RunParams(r_list=1e-3))
    _, _, st = o.run_underdamped(s.x, np.zeros((2, 3)), 1, 0.0)
    assert st == orc.E_ARG
