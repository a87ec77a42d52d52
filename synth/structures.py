"""Seeded generators for the five SOP workloads (plain chain, pulled globule,
indented shell assembly, batched ensemble, long fiber).

The paper's systems come from PDB structures (Table I); none is available
here, so seeded self-avoiding C-alpha walks stand in for them.  Bonds join
consecutive residues of a chain; native contacts are the pairs closer than
8 A in the generated reference structure that are either more than two
residues apart within a chain or on different chains (Section IV.A, the
cutoff R_C and the |i-j|>2 rule), and every reference distance r0 is taken
from the generated structure.  Everything here is input preparation: no
energy, force, pair-list or integrator arithmetic is done.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np
from scipy.spatial import cKDTree

BOND = 3.8            # C-alpha virtual bond length, A
MIN_NONBONDED = 4.0   # generator's minimum distance for |i-j| >= 2, A
NATIVE_CUTOFF = 8.0   # native-contact cutoff R_C in the reference structure, A
KB_KCAL = 0.0019872043  # Boltzmann constant, kcal/mol/K

CONFIG_NAMES = ("c0", "c1", "c2", "c3", "c4")


@dataclass
class RunParams:
    """Force-field, thermostat and list parameters (kcal/mol, A, reduced time tau)."""
    k_fene: float = 14.0      # FENE spring, kcal/mol/A^2
    R0: float = 2.0           # FENE tolerance, A
    eps_h: float = 1.0        # native contact depth, kcal/mol
    eps_l: float = 1.0        # repulsion strength, kcal/mol
    sigma: float = 3.8        # repulsion range, A
    r_list: float = 20.0      # Verlet-list cutoff, A
    kBT: float = KB_KCAL * 300.0
    zeta: float = 50.0        # friction, reduced units
    h: float = 0.08           # time step, tau
    list_every: int = 10      # list rebuild period, steps
    seed: int = 0x5eed1003
    list_capacity: int = 0    # list partners per residue on the GPU (0 = library default)


def default_params(**kw) -> RunParams:
    return RunParams(**kw)


@dataclass
class Pull:
    traj: int
    residue: int          # global residue index
    kappa: float          # kcal/mol/A^2
    anchor0: np.ndarray   # (3,) A
    v: np.ndarray         # (3,) A/tau


@dataclass
class Tip:
    radius: float
    eps: float
    sigma: float
    c0: np.ndarray        # (3,) centre at t=0, A
    v: np.ndarray         # (3,) A/tau


@dataclass
class System:
    """A flattened set of independent trajectories ("systems")."""
    name: str
    x: np.ndarray                 # (N,3) float64 reference / start coordinates
    res_offsets: np.ndarray       # (T+1,) int64
    stream_ids: np.ndarray        # (T,) uint32, Philox stream per trajectory
    chain_id: np.ndarray          # (N,) int32, chain label (global)
    bonds: np.ndarray             # (nb,2) int32, i<j global ids
    bond_r0: np.ndarray           # (nb,) float64
    natives: np.ndarray           # (nc,2) int32, i<j global ids
    native_r0: np.ndarray         # (nc,) float64
    fixed: Optional[np.ndarray] = None   # (N,) uint8
    pulls: list = field(default_factory=list)
    tip: Optional[Tip] = None
    steps: int = 0                # step count of the workload recipe
    note: str = ""

    @property
    def n_res(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_traj(self) -> int:
        return int(self.res_offsets.shape[0] - 1)

    def subset(self, trajs) -> "System":
        """A new System holding only the listed trajectories (renumbered)."""
        trajs = list(trajs)
        parts, offs = [], [0]
        gmap = -np.ones(self.n_res, dtype=np.int64)
        for t in trajs:
            a, b = int(self.res_offsets[t]), int(self.res_offsets[t + 1])
            gmap[a:b] = np.arange(offs[-1], offs[-1] + (b - a))
            parts.append(np.arange(a, b))
            offs.append(offs[-1] + (b - a))
        idx = np.concatenate(parts)

        def remap(pairs, r0):
            keep = (gmap[pairs[:, 0]] >= 0) & (gmap[pairs[:, 1]] >= 0)
            return gmap[pairs[keep]].astype(np.int32), r0[keep].copy()

        b, br0 = remap(self.bonds, self.bond_r0)
        nn, nr0 = remap(self.natives, self.native_r0)
        pulls = []
        for p in self.pulls:
            if p.traj in trajs:
                pulls.append(Pull(trajs.index(p.traj), int(gmap[p.residue]), p.kappa,
                                  p.anchor0.copy(), p.v.copy()))
        return System(self.name + "-sub", self.x[idx].copy(), np.asarray(offs, np.int64),
                      self.stream_ids[trajs].copy(), self.chain_id[idx].copy(),
                      b, br0, nn, nr0,
                      None if self.fixed is None else self.fixed[idx].copy(),
                      pulls, self.tip, self.steps, self.note)


# --------------------------------------------------------------------------
# chain growth
# --------------------------------------------------------------------------

def _unit(rng, m):
    v = rng.standard_normal((m, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def saw_batch(lengths, rng, bond=BOND, min_dist=MIN_NONBONDED, max_rounds=400):
    """Grow many unconfined self-avoiding walks at once.

    Bead k of every chain is placed at distance `bond` from bead k-1 in a
    uniformly random direction, re-drawn until it is at least `min_dist` from
    all beads 0..k-2 of the same chain.  A chain that stays trapped for
    `max_rounds` draws is regrown on its own by the backtracking grower.
    Returns a list of (n_t,3) arrays.
    """
    lengths = np.asarray(lengths, dtype=np.int64)
    T, nmax = len(lengths), int(lengths.max())
    X = np.zeros((T, nmax, 3), dtype=np.float64)
    X[:, 1] = bond * _unit(rng, T)
    md2 = min_dist * min_dist
    stuck = np.zeros(T, dtype=bool)
    for k in range(2, nmax):
        pending = np.nonzero((lengths > k) & ~stuck)[0]
        rounds = 0
        while pending.size:
            cand = X[pending, k - 1] + bond * _unit(rng, pending.size)
            ok = np.ones(pending.size, dtype=bool)
            for s in range(0, pending.size, 512):
                sl = slice(s, s + 512)
                d = X[pending[sl], :k - 1] - cand[sl, None, :]
                ok[sl] = ((d * d).sum(-1) >= md2).all(1)
            X[pending[ok], k] = cand[ok]
            pending = pending[~ok]
            rounds += 1
            if rounds > max_rounds:
                stuck[pending] = True
                break
    out = [X[t, :lengths[t]].copy() for t in range(T)]
    for t in np.nonzero(stuck)[0]:
        out[t] = saw_confined(int(lengths[t]), rng, (1e6, 1e6, 1e6), bond, min_dist)
    return out


def saw_confined(n, rng, semi_axes, bond=BOND, min_dist=MIN_NONBONDED, batch=64,
                 max_iter=2_000_000):
    """Grow one self-avoiding walk inside the ellipsoid sum((x/a)^2) <= 1.

    Each bead tries `batch` random directions and takes the first one that is
    inside the ellipsoid and at least `min_dist` from beads 0..k-2; after a
    failure the walk backs off a growing number of beads and regrows.  The
    distance test only looks at beads in the 27 grid cells (edge
    bond + min_dist) around bead k-1, which hold every bead that can be
    closer than min_dist to a candidate, so the walk is the same as with a
    test against all earlier beads.
    """
    a = np.asarray(semi_axes, dtype=np.float64)
    X = np.zeros((n, 3))
    X[0] = 0.3 * a * _unit(rng, 1)[0]
    md2 = min_dist * min_dist
    edge = bond + min_dist
    cells = {}
    cell_of = [None] * n

    def put(j):
        c = tuple(np.floor(X[j] / edge).astype(np.int64))
        if cell_of[j] is not None:
            cells[cell_of[j]].discard(j)
        cells.setdefault(c, set()).add(j)
        cell_of[j] = c

    put(0)
    k, fails, it = 1, 0, 0
    while k < n:
        it += 1
        if it > max_iter:
            raise RuntimeError("confined walk stuck")
        cand = X[k - 1] + bond * _unit(rng, batch)
        ok = ((cand / a) ** 2).sum(1) <= 1.0
        if k > 1 and ok.any():
            cx, cy, cz = cell_of[k - 1]
            near = [j for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
                    for j in cells.get((cx + dx, cy + dy, cz + dz), ()) if j < k - 1]
            if near:
                d = X[None, sorted(near), :] - cand[:, None, :]
                ok &= ((d * d).sum(-1) >= md2).all(1)
        if ok.any():
            X[k] = cand[int(np.argmax(ok))]
            put(k)
            k += 1
            fails = 0
        else:
            fails += 1
            k = max(1, k - min(2 ** min(fails, 6), k - 1))
    return X


def _rotation_to(zaxis):
    """A rotation matrix whose third column is the unit vector `zaxis`."""
    z = zaxis / np.linalg.norm(zaxis)
    t = np.array([1.0, 0.0, 0.0]) if abs(z[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    x = np.cross(t, z)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    return np.stack([x, y, z], axis=1)


def _rot_z(phi):
    c, s = np.cos(phi), np.sin(phi)
    return np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])


def _rot_x(phi):
    c, s = np.cos(phi), np.sin(phi)
    return np.array([[1.0, 0.0, 0.0], [0.0, c, -s], [0.0, s, c]])


# --------------------------------------------------------------------------
# topology
# --------------------------------------------------------------------------

def topology_from_chains(traj_chains, native_cutoff=NATIVE_CUTOFF):
    """Flatten trajectories of chains and derive bonds and native contacts.

    traj_chains: list over trajectories of lists of (n,3) arrays (chains).
    Bonds: consecutive residues of one chain, r0 = their distance.
    Natives: pairs of one trajectory with reference distance < cutoff that are
    on different chains or more than two residues apart on one chain.
    """
    xs, chain_id, res_offsets, local = [], [], [0], []
    cid = 0
    for chains in traj_chains:
        for c in chains:
            xs.append(np.asarray(c, dtype=np.float64))
            chain_id.append(np.full(len(c), cid, dtype=np.int32))
            local.append(np.arange(len(c), dtype=np.int64))
            cid += 1
        res_offsets.append(res_offsets[-1] + sum(len(c) for c in chains))
    x = np.concatenate(xs)
    chain_id = np.concatenate(chain_id)
    seq = np.concatenate(local)
    res_offsets = np.asarray(res_offsets, dtype=np.int64)
    n = x.shape[0]

    same_next = chain_id[1:] == chain_id[:-1]
    bi = np.nonzero(same_next)[0]
    bonds = np.stack([bi, bi + 1], axis=1).astype(np.int32)
    bond_r0 = np.linalg.norm(x[bi + 1] - x[bi], axis=1)

    # spread trajectories far apart for the neighbour query only
    traj_of = np.repeat(np.arange(len(res_offsets) - 1), np.diff(res_offsets))
    span = np.ptp(x, axis=0).max() + 10 * native_cutoff + 1.0
    xq = x.copy()
    xq[:, 0] += traj_of * (span + np.abs(x[:, 0]).max() * 2.0 + 100.0)
    pairs = cKDTree(xq).query_pairs(native_cutoff, output_type="ndarray")
    pairs = np.sort(pairs, axis=1)
    i, j = pairs[:, 0], pairs[:, 1]
    d = np.linalg.norm(x[i] - x[j], axis=1)
    keep = (d < native_cutoff) & (traj_of[i] == traj_of[j]) & (
        (chain_id[i] != chain_id[j]) | (np.abs(seq[i] - seq[j]) > 2))
    nat = pairs[keep]
    order = np.lexsort((nat[:, 1], nat[:, 0]))
    nat = nat[order].astype(np.int32)
    nat_r0 = np.linalg.norm(x[nat[:, 0]] - x[nat[:, 1]], axis=1)
    del n
    return x, res_offsets, chain_id, bonds, bond_r0, nat, nat_r0


def _system(name, traj_chains, **kw):
    x, offs, cid, b, br0, nn, nr0 = topology_from_chains(traj_chains)
    T = len(offs) - 1
    return System(name, x, offs, np.arange(T, dtype=np.uint32), cid, b, br0, nn, nr0, **kw)


# --------------------------------------------------------------------------
# the five workloads
# --------------------------------------------------------------------------

def globule(n, seed, semi_axes=None, vol_per_res=300.0):
    """A compact confined walk centred on its centroid."""
    rng = np.random.default_rng(seed)
    if semi_axes is None:
        r = (3.0 * n * vol_per_res / (4.0 * np.pi)) ** (1.0 / 3.0)
        semi_axes = (r, r, r)
    X = saw_confined(n, rng, semi_axes)
    return X - X.mean(axis=0)


def subunit250(seed=2):
    """250-residue globule in an oblate ellipsoid 31 x 31 x 18 A (z is short)."""
    return globule(250, seed, semi_axes=(31.0, 31.0, 18.0))


def _fibonacci_sphere(m):
    k = np.arange(m) + 0.5
    phi = np.arccos(1.0 - 2.0 * k / m)
    theta = np.pi * (1.0 + 5.0 ** 0.5) * k
    return np.stack([np.cos(theta) * np.sin(phi), np.sin(theta) * np.sin(phi), np.cos(phi)], 1)


def _place_copies(sub, frames, centres, rng, base_rot, min_gap=BOND, tries=64):
    """Place rotated copies, re-drawing the spin angle while a copy comes closer
    than min_gap to an already placed copy (only copies whose bounding spheres
    can touch are checked)."""
    rmax = np.linalg.norm(sub, axis=1).max()
    placed = []
    for F, c in zip(frames, centres):
        near = [placed[k] for k in range(len(placed))
                if np.linalg.norm(centres[k] - c) < 2.0 * rmax + min_gap]
        tree = cKDTree(np.concatenate(near)) if near else None
        for _ in range(tries):
            R = F @ base_rot(rng.uniform(0.0, 2.0 * np.pi))
            y = sub @ R.T + c
            if tree is None or not tree.query_ball_point(y, min_gap, return_length=True).any():
                break
        placed.append(y)
    return placed


def config0():
    rng = np.random.default_rng(0)
    X = saw_batch([56], rng)[0]
    return _system("c0: single 56-residue chain", [[X - X.mean(0)]], steps=10_000)


def config1():
    X = globule(1000, 1)
    kappa = 0.05 * 6.02214076e23 / 4184.0 * 1e-20   # 0.05 N/m in kcal/mol/A^2
    s = _system("c1: 1000-residue pulled globule", [[X]], steps=1_000_000)
    fixed = np.zeros(s.n_res, dtype=np.uint8)
    fixed[0] = 1
    s.fixed = fixed
    e = s.x[-1] - s.x[0]
    e /= np.linalg.norm(e)
    v = 1e4 * 500e-12 * e      # 1 um/s with tau = 500 ps, A/tau
    s.pulls = [Pull(0, s.n_res - 1, kappa, s.x[-1].copy(), v)]
    return s


def config2(n_sub=300, shell_radius=300.0):
    sub = subunit250(2)
    rng = np.random.default_rng(12)
    dirs = _fibonacci_sphere(n_sub)
    frames = [_rotation_to(d) for d in dirs]
    chains = _place_copies(sub, frames, shell_radius * dirs, rng, _rot_z)
    s = _system("c2: 75k-residue shell assembly", [chains], steps=100_000)
    ztop = s.x[:, 2].max()
    s.tip = Tip(50.0, 1.0, 1.0, np.array([0.0, 0.0, ztop + 50.0 + 2.0]),
                np.array([0.0, 0.0, -1e-3]))
    fixed = (s.x[:, 2] < -(shell_radius - 10.0)).astype(np.uint8)
    s.fixed = fixed
    return s


def config3(n_traj=4096, nmin=50, nmax=500, seed=3):
    rng = np.random.default_rng(seed)
    lengths = rng.integers(nmin, nmax + 1, size=n_traj)
    chains = saw_batch(lengths, rng)
    return _system("c3: batched ensemble", [[c - c.mean(0)] for c in chains], steps=100_000)


def _stack_copies(sub, n_sub, spacing, rng, min_gap=BOND, tries=16, nudge=1.0):
    """Copies stacked along x, `spacing` apart, each re-spun about x while it
    comes closer than min_gap to the copies before it; when no spin of the
    `tries` clears them, the copy (and every later one) moves `nudge` further
    along x and the spins are drawn again. The fibre is then centred at the
    origin."""
    placed = []
    x = 0.0
    for _ in range(n_sub):
        near = placed[-2:]
        tree = cKDTree(np.concatenate(near)) if near else None
        while True:
            c = np.array([x, 0.0, 0.0])
            for _ in range(tries):
                y = sub @ _rot_x(rng.uniform(0.0, 2.0 * np.pi)).T + c
                if tree is None or not tree.query_ball_point(y, min_gap, return_length=True).any():
                    break
            else:
                x += nudge
                continue
            break
        placed.append(y)
        x += spacing
    mid = 0.5 * (placed[0][:, 0].mean() + placed[-1][:, 0].mean())
    return [y - np.array([mid, 0.0, 0.0]) for y in placed]


def config4(n_sub=1000):
    sub = subunit250(2)
    # short axis of the disc along the fibre axis x
    base = np.array([[0.0, 0.0, 1.0], [0.0, 1.0, 0.0], [-1.0, 0.0, 0.0]])
    sub = sub @ base.T
    ext = np.ptp(sub[:, 0])
    rng = np.random.default_rng(4)
    chains = _stack_copies(sub, n_sub, ext - 6.0, rng)
    return _system("c4: 250k-residue fibre", [chains], steps=10_000)


def config_dense(n=4800, vol_per_res=116.0, seed=11):
    """A single chain folded to protein density: at 116 A^3 per residue the
    globule holds over 100 repulsive list pairs per residue, the regime of
    the capsid in Table I (HK97, about 140 per residue)."""
    X = globule(n, seed, vol_per_res=vol_per_res)
    return _system(f"dense: {n}-residue globule at {vol_per_res:g} A^3/residue", [[X]],
                   steps=200)


_BUILDERS = {"c0": config0, "c1": config1, "c2": config2, "c3": config3, "c4": config4,
             "dense": config_dense}


def make_config(name, **kw) -> System:
    return _BUILDERS[name](**kw)
