"""Force-spectroscopy observables on the host: the oracle's running average,
peak force and end-to-end distance pinned by closed forms, and the library's
host analysis calls (no device) against the oracle."""
import math

import numpy as np
import pytest

from synth import RunParams, make_config

P = pytest.importorskip("paper_1003_1148_amd")


def test_running_average_closed_forms(orc):
    w = 7
    assert np.allclose(orc.running_average(np.full(50, 3.25), w), 3.25, rtol=0, atol=0)
    k = np.arange(60, dtype=np.float64)
    ramp = 2.0 + 0.5 * k                                  # mean of a linear window: its centre
    assert np.allclose(orc.running_average(ramp, w), 2.0 + 0.5 * (k[:60 - w + 1] + (w - 1) / 2),
                       rtol=1e-15, atol=0)
    y = np.random.default_rng(0).normal(size=300)         # the textbook valid-mode convolution
    assert np.allclose(orc.running_average(y, 25), np.convolve(y, np.ones(25) / 25, "valid"),
                       rtol=0, atol=1e-14)
    assert len(orc.running_average(y, 300)) == 1 and len(orc.running_average(y, 1)) == 300


def test_peak_force_closed_forms(orc):
    t = np.arange(201, dtype=np.float64)
    tri = 100.0 - np.abs(t - 120.0)                        # a triangle peaked at 120
    pk, ix = orc.peak_force(tri, 5)
    assert ix == 118 and pk == pytest.approx(100.0 - 6.0 / 5.0, rel=1e-15)
    pk1, ix1 = orc.peak_force(tri, 1)
    assert (pk1, ix1) == (100.0, 120)
    flat = np.ones(10)
    assert orc.peak_force(flat, 3) == (1.0, 0)             # the first of equal windows


def test_end_to_end_distance(orc):
    from synth.structures import System
    x = np.array([[0, 0, 0], [3, 4, 0], [1, 1, 1], [5, 5, 5], [2, 0, 0]], float)
    s = System("e2e", x, np.array([0, 2, 2, 3, 5]), np.arange(4, dtype=np.uint32),
               np.zeros(5, np.int32), np.zeros((0, 2), np.int32), np.zeros(0),
               np.zeros((0, 2), np.int32), np.zeros(0))
    R = orc.OracleSystem(s, RunParams()).end_to_end(x)
    assert R.tolist() == [5.0, 0.0, 0.0, math.sqrt(9 + 25 + 25)]


@pytest.mark.parametrize("w", [1, 3, 500])
def test_library_running_average_and_peak(orc, w):
    rng = np.random.default_rng(w)
    # a noisy force-extension-like trace: a ramp, a drop (the unfolding), noise
    n = 4000
    t = np.arange(n)
    f = np.where(t < 2600, 0.05 * t, 0.02 * t - 40.0) + 30.0 * rng.normal(size=n) + 1e5
    a = P.running_average(f, w)
    b = orc.running_average(f, w)
    assert np.allclose(a, b, rtol=2e-15 * w, atol=0)
    pa, ia = P.peak_force(f, w)
    pb, ib = orc.peak_force(f, w)
    assert pa == pytest.approx(pb, rel=2e-15 * w) and ia == ib
    with pytest.raises(P.SopError):
        P.running_average(f[:w - 1] if w > 1 else f[:0], w)


def test_library_virial_temperature_on_an_oracle_run(orc):
    """A free 56-residue chain: the virial estimate returns the bath's
    300 K (the equipartition pin of the oracle, read through the library's
    estimator)."""
    s = make_config("c0")
    p = RunParams()
    o = orc.OracleSystem(s, p)
    x, _, _, st = o.run(s.x, 4000)
    x, E, _, st = o.run(x, 40000, step0=4000, energy_every=10)
    assert st == 0
    T = P.virial_temperature(E[:, 0, 4], s.n_res, p.kBT / 300.0)
    assert T == pytest.approx(300.0, rel=0.06)
    assert T == pytest.approx(-E[:, 0, 4].mean() / (3 * (s.n_res - 1) * p.kBT / 300.0), rel=1e-13)
