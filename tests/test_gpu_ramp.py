"""GPU parity of the Section IV.C accuracy model (harmonic Brownian particles
under a force ramp) against the FP64 oracle: per particle with the same
Philox noise, noise-free against the Eq. 4 / Eq. 5 recursions, resumes, and
the ensemble moments."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

# the paper's parameters in pN, nm, ps (Section IV.C): K_sp = 40 pN/nm,
# kB T = 4.14 pN nm, D = kB T/xi = 1.5e-11 cm^2/s = 1.5e-9 nm^2/ps,
# r_f = kappa nu_0 = 10 pN/nm x 1e-9 nm/ps = 1e-8 pN/ps
KSP, KBT = 40.0, 4.14
XI = KBT / 1.5e-9
RF = 1e-8
SEED = 0x5eed1003


@pytest.fixture(scope="module")
def env():
    import torch
    import oracle
    import paper_1003_1148_amd as P
    assert torch.cuda.is_available()
    if not __import__("os").path.exists(oracle._LIB):
        oracle.build()
    return torch, oracle, P


def particles(torch, X0):
    x = torch.zeros((len(X0), 2), dtype=torch.float32, device="cuda")
    x[:, 0] = torch.as_tensor(np.asarray(X0, np.float32))
    return x


def as_f64(x):
    v = x.cpu().numpy().astype(np.float64)
    return v[:, 0] + v[:, 1]


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("h", [1.0, 50.0])
def test_particles_match_the_oracle(env, order, h):
    torch, orc, P = env
    M, n = 777, 3000  # a ragged last block
    x = particles(torch, np.zeros(M))
    rp = P.ramp_params(RF, XI, KSP, KBT, h, order=order, seed=SEED, stream=3)
    P.ramp_run(rp, x, 0, n, moments=False)
    torch.cuda.synchronize()
    got = as_f64(x)
    ref = orc.ramp_run(order, np.zeros(M), 0, n, RF, XI, KSP, KBT, h, SEED, stream=3)
    # per-step Gaussian error about 6e-7 relative (single-precision
    # Box-Muller), accumulated over n steps of a random walk
    sig = math.sqrt(2.0 * KBT * h / XI)
    tol = 1e-5 * sig * math.sqrt(n)
    err = np.abs(got - ref).max()
    print(f"order {order} h {h}: max |dX| {err:.3e} nm, tol {tol:.3e}, spread {ref.std():.3e}")
    assert err <= tol


def test_resume_is_bit_exact(env):
    torch, orc, P = env
    M = 300
    rp = P.ramp_params(RF, XI, KSP, KBT, 25.0, order=2, seed=SEED)
    a = particles(torch, np.zeros(M))
    P.ramp_run(rp, a, 0, 1500, moments=False)
    b = particles(torch, np.zeros(M))
    P.ramp_run(rp, b, 0, 700, moments=False)
    P.ramp_run(rp, b, 700, 800, moments=False)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("order", [1, 2])
def test_noise_free_follows_the_recursion(env, order):
    torch, orc, P = env
    # a short timescale (tau = 5) so that the transient and the ramp both matter
    K, xi, rf, h, n = 2.0, 10.0, 0.3, 0.05, 20000
    for X0 in (0.0, 1.5):
        x = particles(torch, [X0])
        rp = P.ramp_params(rf, xi, K, 0.0, h, order=order)
        P.ramp_run(rp, x, 0, n, moments=False)
        torch.cuda.synchronize()
        got = as_f64(x)[0]
        ref = orc.ramp_mean_recursion(order, X0, rf, xi, K, h, n)
        assert abs(got - ref) <= 2e-6 * abs(ref)


def test_moments(env):
    torch, orc, P = env
    M, n = 100_003, 200
    rp = P.ramp_params(RF, XI, KSP, KBT, 50.0, order=1, seed=SEED)
    x = particles(torch, np.linspace(-0.1, 0.1, M))
    mean, var = P.ramp_run(rp, x, 0, n)
    X = as_f64(x)
    assert mean == pytest.approx(X.mean(), rel=1e-12, abs=1e-15)
    assert var == pytest.approx(X.var(), rel=1e-9)


def test_rejects_bad_arguments(env):
    torch, orc, P = env
    x = particles(torch, [0.0])
    with pytest.raises(P.SopError):
        P.ramp_run(P.ramp_params(RF, XI, KSP, KBT, 1.0, order=3), x, 0, 10)
    with pytest.raises(P.SopError):
        P.ramp_run(P.ramp_params(RF, -1.0, KSP, KBT, 1.0), x, 0, 10)
    with pytest.raises(P.SopError):
        P.ramp_run(P.ramp_params(RF, XI, KSP, KBT, 1.0), x, -1, 10)
