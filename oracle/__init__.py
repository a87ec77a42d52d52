"""FP64 CPU oracle for SOP overdamped Langevin dynamics -- test infrastructure.

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  The arithmetic lives in ``sop_oracle.c`` (plain C, FP64;
single-threaded, except the residue-parallel OpenMP forms ``forces_par`` and
``run_par``); this module only marshals arrays through ctypes.  It never
imports the HIP library's package, and the HIP library never imports it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sop_oracle.c")
# SOP_ORACLE_LIB names another build of the same source (the sanitizer test
# loads one built with AddressSanitizer and UndefinedBehaviorSanitizer)
_LIB = os.environ.get("SOP_ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

OK, E_ARG, E_FENE, E_OVERFLOW, E_NONFINITE, E_TIP = 0, -1, -5, -6, -7, -8
NTERMS = 5
TERM_NAMES = ("fene", "native", "repulsive", "external", "virial")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, no fast math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-ffp-contract=off", "-fopenmp",
                               "-fno-fast-math", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("k_fene", "R0", "eps_h", "eps_l", "sigma", "r_list", "kBT", "zeta", "h")] + [
        ("list_every", C.c_int32), ("pad", C.c_int32), ("seed", C.c_uint64)]


class SystemC(C.Structure):
    _fields_ = [
        ("n_res", C.c_int64), ("n_traj", C.c_int64),
        ("res_offsets", C.c_void_p), ("stream_ids", C.c_void_p),
        ("n_bonds", C.c_int64), ("bonds", C.c_void_p), ("bond_r0", C.c_void_p),
        ("n_native", C.c_int64), ("natives", C.c_void_p), ("native_r0", C.c_void_p),
        ("fixed", C.c_void_p),
        ("n_pull", C.c_int32), ("has_tip", C.c_int32),
        ("pull_traj", C.c_void_p), ("pull_res", C.c_void_p), ("pull_kappa", C.c_void_p),
        ("pull_anchor0", C.c_void_p), ("pull_v", C.c_void_p),
        ("tip_radius", C.c_double), ("tip_eps", C.c_double), ("tip_sigma", C.c_double),
        ("tip_c0", C.c_double * 3), ("tip_v", C.c_double * 3),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = C.CDLL(_LIB)
        vp, i64, u32, u64 = C.c_void_p, C.c_int64, C.c_uint32, C.c_uint64
        L.orc_philox4x32_10.argtypes = [vp, vp, vp]
        L.orc_uniform.argtypes = [u32]
        L.orc_uniform.restype = C.c_double
        L.orc_gauss3.argtypes = [u64, u32, u32, i64, vp]
        dp = C.POINTER(C.c_double)
        L.orc_fene.argtypes = [C.c_double] * 4 + [dp, C.POINTER(C.c_int)]
        L.orc_fene.restype = C.c_double
        L.orc_native.argtypes = [C.c_double] * 3 + [dp]
        L.orc_native.restype = C.c_double
        L.orc_repulsive.argtypes = [C.c_double] * 3 + [dp]
        L.orc_repulsive.restype = C.c_double
        L.orc_pairlist.argtypes = [vp, vp, vp, vp, i64]
        L.orc_pairlist.restype = i64
        L.orc_pairlist_bruteforce.argtypes = [vp, vp, vp, vp, i64]
        L.orc_pairlist_bruteforce.restype = i64
        L.orc_forces.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp, vp]
        L.orc_forces.restype = C.c_int
        L.orc_forces_rows.argtypes = [vp, vp, vp, vp, i64, vp, i64, vp]
        L.orc_forces_rows.restype = C.c_int
        L.orc_run.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, i64, vp]
        L.orc_run.restype = C.c_int
        L.orc_force_scale.argtypes = [vp, vp, vp, i64, vp, i64, vp, vp]
        L.orc_force_scale.restype = C.c_int
        L.orc_run_tempered.argtypes = [vp, vp, vp, i64, i64, C.c_int32, vp, i64, vp, vp, vp]
        L.orc_run_tempered.restype = C.c_int
        L.orc_run_underdamped.argtypes = [vp, vp, C.c_double, vp, vp, i64, i64]
        L.orc_run_underdamped.restype = C.c_int
        L.orc_force_stiffness.argtypes = [vp, vp, vp, i64, vp, i64, vp]
        L.orc_force_stiffness.restype = C.c_int
        L.orc_force_stiffness_par.argtypes = [vp, vp, vp, i64, vp, C.c_int]
        L.orc_force_stiffness_par.restype = C.c_int
        for nm in ("orc_fene_d2", "orc_native_d2", "orc_repulsive_d2"):
            getattr(L, nm).restype = C.c_double
        L.orc_fene_d2.argtypes = [C.c_double] * 4
        L.orc_native_d2.argtypes = [C.c_double] * 3
        L.orc_repulsive_d2.argtypes = [C.c_double] * 3
        L.orc_forces_par.argtypes = [vp, vp, vp, i64, vp, vp, vp, C.c_int]
        L.orc_forces_par.restype = C.c_int
        L.orc_run_par.argtypes = [vp, vp, vp, i64, i64, i64, vp, vp, i64, vp, C.c_int]
        L.orc_run_par.restype = C.c_int
        L.orc_force_scale_par.argtypes = [vp, vp, vp, i64, vp, C.c_int]
        L.orc_force_scale_par.restype = C.c_int
        L.orc_running_average.argtypes = [vp, i64, C.c_int32, vp]
        L.orc_running_average.restype = C.c_int
        L.orc_peak_force.argtypes = [vp, i64, C.c_int32, vp, vp]
        L.orc_peak_force.restype = C.c_int
        L.orc_end_to_end.argtypes = [vp, vp, vp]
        L.orc_end_to_end.restype = None
        d = C.c_double
        L.orc_ramp_mean_exact.argtypes = [d, d, d, d, d]
        L.orc_ramp_mean_exact.restype = d
        L.orc_ramp_mean_recursion.argtypes = [C.c_int, d, d, d, d, d, i64]
        L.orc_ramp_mean_recursion.restype = d
        L.orc_ramp_run.argtypes = [C.c_int, i64, vp, i64, i64, d, d, d, d, d, u64, u32]
        L.orc_ramp_run.restype = None
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


class OracleSystem:
    """Holds contiguous copies of a synthetic System's arrays for the C side."""

    def __init__(self, sysm, params):
        self.sysm = sysm
        self.p = Params(params.k_fene, params.R0, params.eps_h, params.eps_l, params.sigma,
                        params.r_list, params.kBT, params.zeta, params.h,
                        int(params.list_every), 0, int(params.seed))
        self._keep = []

        def arr(a, dt):
            a = np.ascontiguousarray(a, dtype=dt)
            self._keep.append(a)
            return a

        s = SystemC()
        s.n_res, s.n_traj = sysm.n_res, sysm.n_traj
        s.res_offsets = _ptr(arr(sysm.res_offsets, np.int64))
        s.stream_ids = _ptr(arr(sysm.stream_ids, np.uint32))
        s.n_bonds = len(sysm.bonds)
        s.bonds = _ptr(arr(np.asarray(sysm.bonds).reshape(-1, 2), np.int32))
        s.bond_r0 = _ptr(arr(sysm.bond_r0, np.float64))
        s.n_native = len(sysm.natives)
        s.natives = _ptr(arr(np.asarray(sysm.natives).reshape(-1, 2), np.int32))
        s.native_r0 = _ptr(arr(sysm.native_r0, np.float64))
        s.fixed = None if sysm.fixed is None else _ptr(arr(sysm.fixed, np.uint8))
        pulls = list(sysm.pulls)
        s.n_pull = len(pulls)
        if pulls:
            s.pull_traj = _ptr(arr([p.traj for p in pulls], np.int32))
            s.pull_res = _ptr(arr([p.residue for p in pulls], np.int32))
            s.pull_kappa = _ptr(arr([p.kappa for p in pulls], np.float64))
            s.pull_anchor0 = _ptr(arr(np.stack([p.anchor0 for p in pulls]), np.float64))
            s.pull_v = _ptr(arr(np.stack([p.v for p in pulls]), np.float64))
        if sysm.tip is not None:
            t = sysm.tip
            s.has_tip = 1
            s.tip_radius, s.tip_eps, s.tip_sigma = t.radius, t.eps, t.sigma
            s.tip_c0 = (C.c_double * 3)(*[float(v) for v in t.c0])
            s.tip_v = (C.c_double * 3)(*[float(v) for v in t.v])
        self.s = s

    # -- pieces ---------------------------------------------------------
    def pairlist(self, x, brute=False):
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        fn = L.orc_pairlist_bruteforce if brute else L.orc_pairlist
        m = fn(C.byref(self.s), C.byref(self.p), _ptr(x), None, 0)
        if m < 0:
            raise RuntimeError(f"oracle pairlist failed: {m}")
        ij = np.zeros((max(m, 1), 2), dtype=np.int32)
        m2 = fn(C.byref(self.s), C.byref(self.p), _ptr(x), _ptr(ij), m)
        assert m2 == m
        return ij[:m]

    def forces(self, x, step=0, pairs=None, check=True):
        """Forces, per-trajectory energies (n_traj,5) and external-force reports."""
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        if pairs is None:
            pairs = self.pairlist(x)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32)
        F = np.zeros((self.sysm.n_res, 3))
        E = np.zeros((self.sysm.n_traj, NTERMS))
        fe = np.zeros(self.sysm.n_traj)
        st = L.orc_forces(C.byref(self.s), C.byref(self.p), _ptr(x), int(step), _ptr(pairs),
                          len(pairs), _ptr(F), _ptr(E), _ptr(fe))
        if check and st != OK:
            raise RuntimeError(f"oracle forces status {st}")
        return F, E, fe, st

    def forces_rows(self, x, rows, x_list=None, step=0):
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        xl = x if x_list is None else np.ascontiguousarray(x_list, dtype=np.float64)
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        F = np.zeros((len(rows), 3))
        st = L.orc_forces_rows(C.byref(self.s), C.byref(self.p), _ptr(x), _ptr(xl), int(step),
                               _ptr(rows), len(rows), _ptr(F))
        if st != OK:
            raise RuntimeError(f"oracle forces_rows status {st}")
        return F

    def force_scale(self, x, step=0, pairs=None):
        """Per-residue scale S_i (sum of |dE/dr| over the residue's pairs plus
        its external force magnitudes) and per-trajectory term magnitudes
        (n_traj, 5): sums of |E| per term and of |r dE/dr| for the virial."""
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        if pairs is None:
            pairs = self.pairlist(x)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32)
        S = np.zeros(self.sysm.n_res)
        Em = np.zeros((self.sysm.n_traj, NTERMS))
        st = L.orc_force_scale(C.byref(self.s), C.byref(self.p), _ptr(x), int(step), _ptr(pairs),
                               len(pairs), _ptr(S), _ptr(Em))
        if st != OK:
            raise RuntimeError(f"oracle force_scale status {st}")
        return S, Em

    def force_stiffness(self, x, step=0, pairs=None):
        """Per-residue stiffness scale K_i: the sum of r |d^2E/dr^2| over the
        residue's pairs plus its external terms' change per relative change
        of their distances."""
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        if pairs is None:
            pairs = self.pairlist(x)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32)
        K = np.zeros(self.sysm.n_res)
        st = L.orc_force_stiffness(C.byref(self.s), C.byref(self.p), _ptr(x), int(step), _ptr(pairs),
                                   len(pairs), _ptr(K))
        if st != OK:
            raise RuntimeError(f"oracle force_stiffness status {st}")
        return K

    def force_stiffness_par(self, x, step=0, threads=0):
        """Residue-parallel K (list rebuilt at x)."""
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        K = np.zeros(self.sysm.n_res)
        st = L.orc_force_stiffness_par(C.byref(self.s), C.byref(self.p), _ptr(x), int(step), _ptr(K),
                                       int(threads or default_threads()))
        if st != OK:
            raise RuntimeError(f"oracle force_stiffness_par status {st}")
        return K

    def forces_par(self, x, step=0, threads=0):
        """Residue-parallel forces with the list rebuilt at x; (F, E, f_ext, status)."""
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        F = np.zeros((self.sysm.n_res, 3))
        E = np.zeros((self.sysm.n_traj, NTERMS))
        fe = np.zeros(self.sysm.n_traj)
        st = L.orc_forces_par(C.byref(self.s), C.byref(self.p), _ptr(x), int(step), _ptr(F),
                              _ptr(E), _ptr(fe), int(threads or default_threads()))
        return F, E, fe, st

    def force_scale_par(self, x, step=0, threads=0):
        """Residue-parallel S (list rebuilt at x)."""
        L = lib()
        x = np.ascontiguousarray(x, dtype=np.float64)
        S = np.zeros(self.sysm.n_res)
        st = L.orc_force_scale_par(C.byref(self.s), C.byref(self.p), _ptr(x), int(step), _ptr(S),
                                   int(threads or default_threads()))
        if st != OK:
            raise RuntimeError(f"oracle force_scale_par status {st}")
        return S

    def run_par(self, x, n_steps, step0=0, energy_every=0, threads=0):
        """Residue-parallel run; the same return values as run()."""
        L = lib()
        x = np.array(x, dtype=np.float64, copy=True, order="C")
        nrec_max = 0 if energy_every <= 0 else (n_steps // energy_every + 2)
        E = np.zeros((max(nrec_max, 1), self.sysm.n_traj, NTERMS))
        fe = np.zeros((max(nrec_max, 1), self.sysm.n_traj))
        nrec = C.c_int64(0)
        st = L.orc_run_par(C.byref(self.s), C.byref(self.p), _ptr(x), int(step0), int(n_steps),
                           int(energy_every), _ptr(E), _ptr(fe), nrec_max, C.byref(nrec),
                           int(threads or default_threads()))
        return x, E[:nrec.value], fe[:nrec.value], st

    def run_underdamped(self, x, v, n_steps, mass, step0=0):
        """BAOAB underdamped Langevin steps; returns (x, v, status) at the end."""
        x = np.array(x, dtype=np.float64, copy=True, order="C")
        v = np.array(v, dtype=np.float64, copy=True, order="C")
        st = lib().orc_run_underdamped(C.byref(self.s), C.byref(self.p), float(mass), _ptr(x), _ptr(v),
                                       int(step0), int(n_steps))
        return x, v, st

    def run_tempered(self, x, n_steps, kbt, exchange_every, tidx, step0=0):
        """Replica exchange over groups of len(kbt) consecutive trajectories;
        returns (x, tidx, accepted, attempted, status)."""
        x = np.array(x, dtype=np.float64, copy=True, order="C")
        kbt = np.ascontiguousarray(kbt, dtype=np.float64)
        tidx = np.array(tidx, dtype=np.int32, copy=True, order="C")
        acc = np.zeros(max(len(kbt) - 1, 1), dtype=np.int64)
        att = np.zeros(max(len(kbt) - 1, 1), dtype=np.int64)
        st = lib().orc_run_tempered(C.byref(self.s), C.byref(self.p), _ptr(x), int(step0), int(n_steps),
                                    len(kbt), _ptr(kbt), int(exchange_every), _ptr(tidx), _ptr(acc),
                                    _ptr(att))
        return x, tidx, acc[:len(kbt) - 1], att[:len(kbt) - 1], st

    def end_to_end(self, x):
        """|x_last - x_first| of every trajectory."""
        x = np.ascontiguousarray(x, dtype=np.float64)
        R = np.zeros(self.sysm.n_traj)
        lib().orc_end_to_end(C.byref(self.s), _ptr(x), _ptr(R))
        return R

    def run(self, x, n_steps, step0=0, energy_every=0):
        """Integrate n_steps from step0; returns (x_new, E records, f records, status)."""
        L = lib()
        x = np.array(x, dtype=np.float64, copy=True, order="C")
        nrec_max = 0 if energy_every <= 0 else (n_steps // energy_every + 2)
        E = np.zeros((max(nrec_max, 1), self.sysm.n_traj, NTERMS))
        fe = np.zeros((max(nrec_max, 1), self.sysm.n_traj))
        nrec = C.c_int64(0)
        st = L.orc_run(C.byref(self.s), C.byref(self.p), _ptr(x), int(step0), int(n_steps),
                       int(energy_every), _ptr(E), _ptr(fe), nrec_max, C.byref(nrec))
        return x, E[:nrec.value], fe[:nrec.value], st


def default_threads():
    """Threads for the residue-parallel forms: OMP_NUM_THREADS, else the CPUs
    this process may run on."""
    v = os.environ.get("OMP_NUM_THREADS")
    if v and v.isdigit() and int(v) > 0:
        return int(v)
    return len(os.sched_getaffinity(0))


# -- force-spectroscopy observables (Section IV.B) -------------------------

def running_average(y, w):
    y = np.ascontiguousarray(y, dtype=np.float64)
    out = np.zeros(max(len(y) - int(w) + 1, 1))
    if lib().orc_running_average(_ptr(y), len(y), int(w), _ptr(out)) != OK:
        raise ValueError("bad window")
    return out[:len(y) - int(w) + 1]


def peak_force(f, w):
    f = np.ascontiguousarray(f, dtype=np.float64)
    pk, ix = C.c_double(0.0), C.c_int64(0)
    if lib().orc_peak_force(_ptr(f), len(f), int(w), C.byref(pk), C.byref(ix)) != OK:
        raise ValueError("bad window")
    return pk.value, ix.value


# -- Section IV.C: harmonic Brownian particle under a force ramp ---------

def ramp_mean_exact(X0, rf, xi, Ksp, t):
    """Eq. 3."""
    return lib().orc_ramp_mean_exact(float(X0), float(rf), float(xi), float(Ksp), float(t))


def ramp_mean_recursion(order, X0, rf, xi, Ksp, h, n):
    """Eq. 4 (order 1) or Eq. 5 (order 2) iterated n times from X0."""
    return lib().orc_ramp_mean_recursion(int(order), float(X0), float(rf), float(xi), float(Ksp),
                                         float(h), int(n))


def ramp_run(order, X, step0, n, rf, xi, Ksp, kBT, h, seed, stream=0):
    """Advance particles X (float64 array, copied) by n steps of the given scheme."""
    X = np.array(X, dtype=np.float64, copy=True, order="C")
    lib().orc_ramp_run(int(order), len(X), _ptr(X), int(step0), int(n), float(rf), float(xi),
                       float(Ksp), float(kBT), float(h), int(seed), int(stream))
    return X


# -- scalar helpers ------------------------------------------------------

def philox(ctr, key):
    out = np.zeros(4, dtype=np.uint32)
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    lib().orc_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(w):
    return lib().orc_uniform(int(w) & 0xFFFFFFFF)


def gauss3(seed, local, stream, step):
    g = np.zeros(3)
    lib().orc_gauss3(int(seed), int(local), int(stream), int(step), _ptr(g))
    return g


def fene_d2(r, r0, k, R0):
    return lib().orc_fene_d2(float(r), float(r0), float(k), float(R0))


def native_d2(r, r0, eps):
    return lib().orc_native_d2(float(r), float(r0), float(eps))


def repulsive_d2(r, sigma, eps):
    return lib().orc_repulsive_d2(float(r), float(sigma), float(eps))


def fene(r, r0, k, R0):
    d = C.c_double(0.0)
    b = C.c_int(0)
    e = lib().orc_fene(r, r0, k, R0, C.byref(d), C.byref(b))
    return e, d.value, bool(b.value)


def native(r, r0, eps):
    d = C.c_double(0.0)
    e = lib().orc_native(r, r0, eps, C.byref(d))
    return e, d.value


def repulsive(r, sigma, eps):
    d = C.c_double(0.0)
    e = lib().orc_repulsive(r, sigma, eps, C.byref(d))
    return e, d.value
