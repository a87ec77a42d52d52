"""Parity gates shared by the GPU tests (HIP path through the C ABI against
the FP64 oracle).

Forces: the relative L2 error over all components, and element-wise, for
every residue i, |F_gpu,i - F_ref,i| <= 1e-5 S_i + 5e-7 K_i, i.e. 1e-5 of the
scale S_i + 0.05 K_i, where S_i is the oracle's sum of |dE/dr| over the
residue's pairs plus its external force magnitudes, and K_i the sum of
r |d^2E/dr^2| over the same terms: each pair may be off by 1e-5 of its
force and by the change a distance error of 5e-7 r (about eight units in
the last place of single precision) makes.  The second part is what bounds
single-precision rounding where the pair forces vanish: at a bond's or a
native contact's reference length (the minima of the FENE and 12-6 terms of
Eq. 1) dE/dr = 0 while d^2E/dr^2 > 0.  A residue on which nothing acts
(S_i = K_i = 0) must get exactly zero.

Energies, per trajectory and term, against the oracle's magnitude sums Em
(sums of |E| per term; sum of |r dE/dr| for the virial):
  FENE, native, repulsive: |dE| <= 1e-5 Em + 1e-11 N.  The floor covers a
      structure at its reference bond lengths, where the FENE energy is the
      square of single-precision bond-length rounding (about 2e-7 A, i.e.
      1e-12 kcal/mol per bond) and has no relative accuracy at all.
  external: |dE| <= 1e-5 Em (no floor);
  virial:   |dE| <= 1e-5 Em (the virial's terms cancel; their magnitude
      sum is its rounding scale).
"""
import sys

import numpy as np

FORCE_TOL = 1e-5
TRAJ_TOL = 1e-4
STIFF_ETA = 0.05   # 5e-7 / 1e-5: the distance-error allowance in units of FORCE_TOL
E_FLOOR_PER_RES = 1e-11


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def force_gate_scale(o, x, step=0, pairs=None):
    """The per-residue scale of the element-wise gate, S_i + 0.05 K_i."""
    if pairs is None:
        pairs = o.pairlist(x)
    S, _ = o.force_scale(x, step=step, pairs=pairs)
    return S + STIFF_ETA * o.force_stiffness(x, step=step, pairs=pairs)


def oracle_reference(o, x, step=0, pairs=None):
    """Oracle forces, energies, external reports, the element-wise force
    scale S_i + 0.05 K_i and the term magnitudes at x (list built at x
    unless given)."""
    if pairs is None:
        pairs = o.pairlist(x)
    Fo, Eo, feo, st = o.forces(x, step=step, pairs=pairs)
    assert st == 0, f"oracle status {st}"
    S, Em = o.force_scale(x, step=step, pairs=pairs)
    S = S + STIFF_ETA * o.force_stiffness(x, step=step, pairs=pairs)
    return Fo, Eo, feo, S, Em


def force_errors(F, Fo, S):
    d = np.linalg.norm(F - Fo, axis=1)
    nref = np.linalg.norm(Fo)
    l2 = float(np.linalg.norm(F - Fo) / nref) if nref > 0 else float(np.linalg.norm(F - Fo))
    act = S > 0
    ew = float((d[act] / S[act]).max()) if act.any() else 0.0
    worst = int(np.flatnonzero(act)[np.argmax(d[act] / S[act])]) if act.any() else -1
    zero_ok = bool(np.all(d[~act] == 0.0))
    return l2, ew, worst, zero_ok


def assert_forces(F, Fo, S, what=""):
    l2, ew, worst, zero_ok = force_errors(F, Fo, S)
    log(f"  {what} force L2 rel err {l2:.3e}, max per-residue |dF|/(S+0.05K) {ew:.3e} (residue {worst})")
    assert l2 <= FORCE_TOL, (what, l2)
    assert ew <= FORCE_TOL, (what, ew, worst)
    assert zero_ok, (what, "nonzero force on a residue nothing acts on")
    return l2, ew


def assert_energies(E, Eo, Em, res_offsets, what=""):
    n = np.diff(np.asarray(res_offsets))
    worst = 0.0
    for t in range(len(n)):
        for k in range(5):
            tol = 1e-5 * Em[t, k]
            if k < 3:
                tol += E_FLOOR_PER_RES * n[t]
            err = abs(E[t, k] - Eo[t, k])
            if tol > 0:
                worst = max(worst, err / tol)
            assert err <= tol, (what, t, k, E[t, k], Eo[t, k], tol)
    log(f"  {what} energies within {worst:.2f} of their tolerance")
