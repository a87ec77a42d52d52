"""Pins of the FP64 oracle against things other than itself.

Each test ties one part of the oracle to what the paper or mathematics fixes:
an independent Philox implementation, closed-form values of the Eq. 1 terms,
finite differences of the energy, Newton's third law, Table I's pair-count
identity, brute force and an independent neighbour search for the list,
and exact statistical properties of the Euler-Maruyama update (free
diffusion, the discrete harmonic stationary variance, the Eq. 4 mean
recursion and Eq. 3).
"""
import math
import os
import subprocess
import tempfile

import numpy as np
import pytest
from scipy import stats
from scipy.spatial import cKDTree

from synth import RunParams, System, make_config
from synth.structures import Pull, Tip

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")


def tiny(x, bonds=(), natives=(), offsets=None, fixed=None, pulls=(), tip=None):
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    b = np.asarray(bonds, dtype=np.int32).reshape(-1, 2)
    nn = np.asarray(natives, dtype=np.int32).reshape(-1, 2)
    br0 = np.linalg.norm(x[b[:, 0]] - x[b[:, 1]], axis=1) if len(b) else np.zeros(0)
    nr0 = np.linalg.norm(x[nn[:, 0]] - x[nn[:, 1]], axis=1) if len(nn) else np.zeros(0)
    offs = np.asarray([0, n] if offsets is None else offsets, dtype=np.int64)
    return System("tiny", x, offs, np.arange(len(offs) - 1, dtype=np.uint32),
                  np.zeros(n, np.int32), b, br0, nn, nr0,
                  None if fixed is None else np.asarray(fixed, np.uint8), list(pulls), tip)


# --------------------------------------------------------------------------
# Philox4x32-10 against rocRAND's open-source implementation
# --------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rocrand_ref():
    src = os.path.join(HERE, "philox_rocrand_ref.cpp")
    if not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers not installed")
    d = tempfile.mkdtemp()
    exe = os.path.join(d, "philox_ref")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-I/opt/rocm/include",
                           "-D__HIP_PLATFORM_AMD__", "-x", "c++", src, "-o", exe])
    return exe


def test_philox_matches_rocrand(orc, rocrand_ref):
    rng = np.random.default_rng(11)
    blocks = rng.integers(0, 2**32, size=(500, 6), dtype=np.uint64)
    blocks[0] = 0
    blocks[1] = 2**32 - 1
    blocks[2, 2:] = 0  # step 0 of counter (i, stream)
    inp = "\n".join(" ".join(str(int(v)) for v in row) for row in blocks) + "\n"
    out = subprocess.run([rocrand_ref], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()],
                   dtype=np.uint64)
    for row, r in zip(blocks, ref):
        got = orc.philox(row[:4].astype(np.uint32), row[4:].astype(np.uint32))
        assert np.array_equal(got.astype(np.uint64), r), (row, got, r)


def test_uniform_is_exact_in_fp32(orc):
    for w in [0, 1, 511, 512, 2**31, 2**32 - 1, 123456789]:
        u = orc.uniform(w)
        assert 0.0 < u < 1.0
        assert float(np.float32(u)) == u
    assert orc.uniform(0) == 2.0 ** -24
    assert orc.uniform(2**32 - 1) == 1.0 - 2.0 ** -24


def test_gaussians_are_standard_normal(orc):
    """Box-Muller output: moments, independence and a KS test per axis."""
    n = 60000
    g = np.array([orc.gauss3(0x1234, i % 3000, 7, i // 3000) for i in range(n)])
    for a in range(3):
        col = g[:, a]
        assert abs(col.mean()) < 5.0 / math.sqrt(n)
        assert abs(col.var() - 1.0) < 5.0 * math.sqrt(2.0 / n)
        assert abs(stats.kurtosis(col, fisher=False) - 3.0) < 5.0 * math.sqrt(24.0 / n)
        assert stats.kstest(col, "norm").pvalue > 1e-4
    c = np.corrcoef(g.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5.0 / math.sqrt(n))


def test_gaussians_depend_on_every_counter_word(orc):
    base = orc.gauss3(9, 5, 3, 1000)
    for args in [(9, 6, 3, 1000), (9, 5, 4, 1000), (9, 5, 3, 1001), (9, 5, 3, 1000 + 2**32),
                 (10, 5, 3, 1000), (9 + 2**32, 5, 3, 1000)]:
        assert not np.allclose(orc.gauss3(*args), base)


# --------------------------------------------------------------------------
# Eq. 1 terms: closed-form values and finite-difference derivatives
# --------------------------------------------------------------------------

def _golden_terms():
    rows = []
    with open(os.path.join(GOLD, "pair_terms.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            t, r, r0, e = line.split()[:4]
            rows.append((t, float(r), float(r0), float(e)))
    return rows


@pytest.mark.parametrize("row", _golden_terms())
def test_pair_term_closed_forms(orc, row):
    t, r, r0, e_ref = row
    if t == "fene":
        e = orc.fene(r, r0, 14.0, 2.0)[0]
    elif t == "native":
        e = orc.native(r, r0, 1.0)[0]
    else:
        e = orc.repulsive(r, 3.8, 1.0)[0]
    assert e == pytest.approx(e_ref, rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("t", ["fene", "native", "repulsive"])
def test_pair_term_derivatives_by_finite_differences(orc, t):
    f = {"fene": lambda r: orc.fene(r, 3.8, 14.0, 2.0),
         "native": lambda r: orc.native(r, 5.5, 1.0),
         "repulsive": lambda r: orc.repulsive(r, 3.8, 1.0)}[t]
    rs = {"fene": np.linspace(2.0, 5.6, 23), "native": np.linspace(3.5, 15.0, 23),
          "repulsive": np.linspace(3.0, 20.0, 23)}[t]
    for r in rs:
        hstep = 1e-6 * r
        num = (f(r + hstep)[0] - f(r - hstep)[0]) / (2 * hstep)
        ana = f(r)[1]
        assert ana == pytest.approx(num, rel=1e-6, abs=1e-8)


def test_fene_breaks_at_R0(orc):
    assert orc.fene(3.8 + 2.0, 3.8, 14.0, 2.0)[2]
    assert orc.fene(3.8 - 2.0, 3.8, 14.0, 2.0)[2]
    assert not orc.fene(3.8 + 1.999, 3.8, 14.0, 2.0)[2]


def test_euler_homogeneity_of_repulsion(orc):
    """(sigma/r)^6 is homogeneous of degree -6: r dE/dr = -6 E."""
    for r in [3.0, 4.1, 9.9, 19.0]:
        e, d = orc.repulsive(r, 3.8, 1.0)
        assert r * d == pytest.approx(-6.0 * e, rel=1e-13)


# --------------------------------------------------------------------------
# whole-system energies and forces
# --------------------------------------------------------------------------

def test_energies_of_a_straight_chain(orc):
    """Four residues on a line 3.8 A apart: bonds at rest, no native pairs,
    repulsive pairs (0,2), (1,3) at 7.6 A and (0,3) at 11.4 A."""
    x = np.array([[0, 0, 0], [3.8, 0, 0], [7.6, 0, 0], [11.4, 0, 0]], float)
    s = tiny(x, bonds=[(0, 1), (1, 2), (2, 3)])
    o = orc.OracleSystem(s, RunParams())
    pairs = o.pairlist(x)
    assert pairs.tolist() == [[0, 2], [0, 3], [1, 3]]
    F, E, _, st = o.forces(x, pairs=pairs)
    e_rep = 2.0 / 64.0 + 1.0 / 729.0
    assert E[0, 0] == pytest.approx(0.0, abs=1e-12)
    assert E[0, 1] == 0.0
    assert E[0, 2] == pytest.approx(e_rep, rel=1e-13)
    assert E[0, 3] == 0.0
    assert E[0, 4] == pytest.approx(6.0 * e_rep, rel=1e-12)   # -sum r dE/dr
    # forces are along x only; end residues are pushed outward
    assert np.allclose(F[:, 1:], 0.0)
    assert F[0, 0] < 0 and F[3, 0] > 0


def test_energies_with_a_native_contact(orc):
    """Square of side 3.8 plus one residue: (0,3) native at its reference distance."""
    x = np.array([[0, 0, 0], [3.8, 0, 0], [3.8, 3.8, 0], [0, 3.8, 0]], float)
    s = tiny(x, bonds=[(0, 1), (1, 2), (2, 3)], natives=[(0, 3)])
    o = orc.OracleSystem(s, RunParams())
    F, E, _, _ = o.forces(x)
    d = 3.8 * math.sqrt(2.0)
    assert E[0, 1] == pytest.approx(-1.0, rel=1e-13)
    assert E[0, 2] == pytest.approx(2.0 * (3.8 / d) ** 6, rel=1e-13)   # (0,2), (1,3)
    assert E[0, 0] == pytest.approx(0.0, abs=1e-12)


def _ext_system():
    s = make_config("c0")
    x = s.x
    s.pulls = [Pull(0, s.n_res - 1, 0.5, x[-1] + np.array([1.0, -0.5, 0.3]),
                    np.array([0.2, 0.1, 0.0]))]
    ztop = x[:, 2].max()
    s.tip = Tip(10.0, 1.0, 1.0, np.array([0.0, 0.0, ztop + 12.0]), np.array([0.0, 0.0, -0.5]))
    return s


@pytest.mark.parametrize("with_ext", [False, True])
def test_forces_are_minus_gradient(orc, with_ext):
    s = _ext_system() if with_ext else make_config("c0")
    rng = np.random.default_rng(5)
    x = s.x + 0.3 * rng.standard_normal(s.x.shape)
    o = orc.OracleSystem(s, RunParams())
    pairs = o.pairlist(x)
    step = 37
    F, E, _, _ = o.forces(x, step=step, pairs=pairs)

    def etot(y):
        return o.forces(y, step=step, pairs=pairs)[1][0, :4].sum()

    h = 1e-5
    G = np.zeros_like(x)
    for i in range(len(x)):
        for a in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, a] += h
            xm[i, a] -= h
            G[i, a] = (etot(xp) - etot(xm)) / (2 * h)
    err = np.linalg.norm(F + G) / np.linalg.norm(F)
    assert err < 1e-7, err


def test_newton_third_law_and_zero_torque(orc):
    s = make_config("c1")
    s.pulls, s.fixed = [], None
    rng = np.random.default_rng(8)
    x = s.x + 0.2 * rng.standard_normal(s.x.shape)
    o = orc.OracleSystem(s, RunParams())
    F, _, _, _ = o.forces(x)
    scale = np.abs(F).sum()
    assert np.abs(F.sum(0)).max() < 1e-12 * scale
    assert np.abs(np.cross(x, F).sum(0)).max() < 1e-12 * scale * np.abs(x).max()


def test_forces_rows_matches_pair_loop(orc):
    s = _ext_system()
    o = orc.OracleSystem(s, RunParams())
    x = s.x.copy()
    F, _, _, _ = o.forces(x, step=3)
    rows = np.arange(s.n_res)
    Fr = o.forces_rows(x, rows, step=3)
    assert np.allclose(Fr, F, rtol=1e-12, atol=1e-12)


def test_external_force_reports(orc):
    """Cantilever alone: E = kappa/2 |A - x|^2 and the report is kappa (A - x).v_hat."""
    x = np.array([[0.0, 0.0, 0.0]])
    p = Pull(0, 0, 2.0, np.array([1.0, 0.0, 0.0]), np.array([0.5, 0.0, 0.0]))
    s = tiny(x, pulls=[p])
    o = orc.OracleSystem(s, RunParams(h=0.1))
    F, E, fe, _ = o.forces(x, step=10)  # t = 1, anchor at 1.5
    assert F[0, 0] == pytest.approx(3.0)
    assert E[0, 3] == pytest.approx(0.5 * 2.0 * 1.5 ** 2)
    assert fe[0] == pytest.approx(3.0)


def test_error_codes(orc):
    x = np.array([[0, 0, 0], [3.8, 0, 0]], float)
    s = tiny(x, bonds=[(0, 1)])
    o = orc.OracleSystem(s, RunParams())
    y = x.copy()
    y[1, 0] = 3.8 + 2.0
    assert o.forces(y, check=False)[3] == orc.E_FENE
    tip = Tip(5.0, 1.0, 1.0, np.array([0.0, 0.0, 4.0]), np.zeros(3))
    s2 = tiny(x, bonds=[(0, 1)], tip=tip)
    assert orc.OracleSystem(s2, RunParams()).forces(x, check=False)[3] == orc.E_TIP


# --------------------------------------------------------------------------
# pair classification and the Verlet list
# --------------------------------------------------------------------------

def test_table1_identity():
    rows = []
    with open(os.path.join(GOLD, "table1.txt")) as f:
        for line in f:
            if not line.startswith("#") and line.strip():
                name, n, b, c, nn, exact = line.split()
                rows.append((name, int(n), int(b), int(c), int(nn), int(exact)))
    for name, n, b, c, nn, exact in rows:
        if exact:
            assert n * (n - 1) // 2 - b - c == nn, name


@pytest.mark.parametrize("cfg", ["c0", "c1"])
def test_all_other_pairs_are_repulsive(orc, cfg):
    """With a cutoff beyond the system size the list holds N(N-1)/2 - b - c pairs."""
    s = make_config(cfg)
    o = orc.OracleSystem(s, RunParams(r_list=1e4))
    pairs = o.pairlist(s.x)
    n = s.n_res
    assert len(pairs) == n * (n - 1) // 2 - len(s.bonds) - len(s.natives)


def test_list_predicate_is_strict_and_single_precision(orc):
    # exactly 20 A apart: d2 == 400 is not < 400
    x = np.array([[0.0, 0, 0], [20.0, 0, 0], [0.0, 19.999, 0]])
    s = tiny(x, offsets=[0, 3])
    o = orc.OracleSystem(s, RunParams())
    assert o.pairlist(x).tolist() == [[0, 2]]
    # true distance just below 20 A that rounds to 20.0f: out of the list
    y = np.array([[0.0, 0, 0], [20.0 - 1e-7, 0, 0]])
    s2 = tiny(y)
    assert float(np.float32(20.0 - 1e-7)) == 20.0
    assert len(orc.OracleSystem(s2, RunParams()).pairlist(y)) == 0


def test_list_only_within_trajectories(orc):
    x = np.array([[0.0, 0, 0], [5.0, 0, 0], [0.0, 5.0, 0], [5.0, 5.0, 0]])
    s = tiny(x, offsets=[0, 2, 4])
    assert orc.OracleSystem(s, RunParams()).pairlist(x).tolist() == [[0, 1], [2, 3]]


@pytest.mark.parametrize("cfg", ["c0", "c1"])
def test_sweep_list_equals_bruteforce(orc, cfg):
    s = make_config(cfg)
    rng = np.random.default_rng(3)
    x = s.x + 0.5 * rng.standard_normal(s.x.shape)
    o = orc.OracleSystem(s, RunParams())
    a = o.pairlist(x)
    b = o.pairlist(x, brute=True)
    assert np.array_equal(a, b)


def test_list_matches_kdtree_away_from_boundary(orc):
    s = make_config("c1")
    x = s.x
    o = orc.OracleSystem(s, RunParams())
    got = {tuple(p) for p in o.pairlist(x).tolist()}
    tree = cKDTree(x)
    near = {tuple(sorted(p)) for p in tree.query_pairs(20.0)}
    excl = {tuple(sorted(p)) for p in np.concatenate([s.bonds, s.natives]).tolist()}
    ref = near - excl
    d = lambda p: np.linalg.norm(x[p[0]] - x[p[1]])
    sym = {p for p in got ^ ref if abs(d(p) - 20.0) > 1e-4}
    assert not sym
    assert len(ref) > 1000


# --------------------------------------------------------------------------
# integrator: exact statistical properties of Euler-Maruyama
# --------------------------------------------------------------------------

def free_particles(m):
    rng = np.random.default_rng(21)
    x = rng.uniform(-1e4, 1e4, size=(m, 3))
    return tiny(x, offsets=np.arange(m + 1))


def test_free_particle_msd(orc):
    """Free diffusion: MSD after n steps is 6 D n h with D = kBT/zeta."""
    m, n = 20000, 10
    p = RunParams(r_list=1e-3)
    s = free_particles(m)
    o = orc.OracleSystem(s, p)
    x1, _, _, st = o.run(s.x, n)
    assert st == 0
    msd = ((x1 - s.x) ** 2).sum(1).mean()
    D = p.kBT / p.zeta
    expect = 6.0 * D * n * p.h
    rel_sd = math.sqrt(2.0 / 3.0) / math.sqrt(m)
    assert abs(msd / expect - 1.0) < 4.5 * rel_sd


def test_harmonic_tether_discrete_variance(orc):
    """Tethered particle, x' = x(1 - hK/zeta) + noise: the exact stationary
    variance per axis is (kBT/K) / (1 - hK/(2 zeta))."""
    m, K = 4000, 14.0
    p = RunParams(r_list=1e-3)
    s = free_particles(m)
    s.pulls = [Pull(t, t, K, s.x[t].copy(), np.zeros(3)) for t in range(m)]
    o = orc.OracleSystem(s, p)
    x, _, _, _ = o.run(s.x, 600)
    samples = []
    step = 600
    for _ in range(15):
        x, _, _, _ = o.run(x, 60, step0=step)
        step += 60
        samples.append(x - s.x)
    var = np.concatenate(samples).var()
    exact = (p.kBT / K) / (1.0 - p.h * K / (2.0 * p.zeta))
    assert abs(var / exact - 1.0) < 0.006
    assert abs(var / (p.kBT / K) - 1.0) > 0.006   # the discrete correction is resolved


def test_cantilever_mean_follows_eq4(orc):
    """Mean position under a moving cantilever follows the first-order recursion
    X_{n+1} = X_n + (r_f t_n / xi - X_n / tau) h with r_f = kappa v, tau = xi/kappa,
    and Eq. 3 up to O(h)."""
    m, kap, v = 6000, 2.0, 0.05
    p = RunParams(r_list=1e-3)
    s = free_particles(m)
    s.pulls = [Pull(t, t, kap, s.x[t].copy(), np.array([v, 0.0, 0.0])) for t in range(m)]
    o = orc.OracleSystem(s, p)
    n = 400
    x, _, _, _ = o.run(s.x, n)
    X = (x - s.x)[:, 0].mean()
    rf, tau, xi, h = kap * v, p.zeta / kap, p.zeta, p.h
    Xr = 0.0
    for k in range(n):
        Xr = Xr + (rf * k * h / xi - Xr / tau) * h
    sd = math.sqrt(p.kBT / kap) / math.sqrt(m)
    assert abs(X - Xr) < 5 * sd
    t = n * h
    X3 = (rf * tau / xi) * (t - tau * (1 - math.exp(-t / tau)))
    assert abs(Xr - X3) < 0.02 * X3


def test_equipartition_from_virial(orc):
    """<-W> = <sum_i r_i . grad_i V> = 3 (N-1) kBT for a free chain, up to O(h)."""
    s = make_config("c0")
    p = RunParams()
    o = orc.OracleSystem(s, p)
    x, _, _, st = o.run(s.x, 4000)
    x, E, _, st = o.run(x, 40000, step0=4000, energy_every=10)
    assert st == 0
    w = -E[:, 0, 4]
    expect = 3 * (s.n_res - 1) * p.kBT
    assert abs(w.mean() / expect - 1.0) < 0.06


def test_resume_is_exact(orc):
    s = make_config("c0")
    o = orc.OracleSystem(s, RunParams())
    a, _, _, _ = o.run(s.x, 60)
    b, _, _, _ = o.run(s.x, 30)
    b, _, _, _ = o.run(b, 30, step0=30)
    assert np.array_equal(a, b)


def test_fixed_residue_does_not_move(orc):
    s = make_config("c1")
    o = orc.OracleSystem(s, RunParams())
    x, _, _, st = o.run(s.x, 20)
    assert st == 0
    assert np.array_equal(x[0], s.x[0])
    assert not np.array_equal(x[1], s.x[1])


def test_compensated_positions_keep_far_coordinates():
    """Why positions are held as hi + lo: at |x| = 1.45e4 A (near the
    fibre's end) the FP32 spacing is 1e-3 A, so adding the per-step displacements
    (sigma = 0.0437 A per axis) in plain FP32 loses about half a spacing per
    step; the TwoSum form used by the update (y = d + lo; hi, lo <- TwoSum(hi, y))
    keeps the sum to FP64 accuracy over 2,000 steps."""
    rng = np.random.default_rng(9)
    n, steps = 4096, 2000
    x64 = 1.45e4 + rng.uniform(-10.0, 10.0, n)
    hi = x64.astype(np.float32)
    lo = (x64 - hi.astype(np.float64)).astype(np.float32)
    x32 = hi.copy()
    for _ in range(steps):
        d = (0.0437 * rng.standard_normal(n)).astype(np.float32)
        x64 = x64 + d.astype(np.float64)
        x32 = (x32 + d).astype(np.float32)
        y = (d + lo).astype(np.float32)
        t = (hi + y).astype(np.float32)
        bp = (t - hi).astype(np.float32)
        e = ((hi - (t - bp)) + (y - bp)).astype(np.float32)
        hi, lo = t, e
    plain = np.abs(x32.astype(np.float64) - x64).max()
    comp = np.abs(hi.astype(np.float64) + lo.astype(np.float64) - x64).max()
    assert plain > 1e-2
    assert comp < 1e-6
