"""The synthetic inputs keep their own recipe: chain geometry and no
clashes between the copies of an assembly."""
import functools

import numpy as np
from scipy.spatial import cKDTree

from synth import make_config as _make_config
from synth.structures import BOND

make_config = functools.lru_cache(maxsize=None)(_make_config)


def _inter_chain_min(s, r):
    pr = cKDTree(s.x).query_pairs(r, output_type="ndarray")
    inter = pr[s.chain_id[pr[:, 0]] != s.chain_id[pr[:, 1]]] if len(pr) else pr
    return len(inter)


def test_assemblies_have_no_clashes():
    """Copies of the subunit in the shell (c2) and in the fibre (c4) keep at
    least a bond length from each other, so no native contact has a
    near-zero r0."""
    for name in ("c2", "c4"):
        s = make_config(name)
        assert _inter_chain_min(s, BOND) == 0, name
        assert s.native_r0.min() > 3.0, name
        d = np.linalg.norm(s.x[s.bonds[:, 0]] - s.x[s.bonds[:, 1]], axis=1)
        assert np.allclose(d, BOND, atol=1e-9), name


def test_fibre_reaches_far_coordinates():
    """The precision workload: 1,000 subunits along x reach |x| > 1.4e4 A,
    where the FP32 spacing of a coordinate exceeds 1e-3 A."""
    s = make_config("c4")
    assert s.n_res == 250_000
    assert np.abs(s.x[:, 0]).max() > 1.4e4
