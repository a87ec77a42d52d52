"""ctypes binding of libsop.so: argument marshalling only.

Every step of the dynamics runs in the HIP kernels behind the C ABI declared
in include/sop.h.  PyTorch supplies device memory (the workspace) and the
stream; there is no other code path.  Importing fails loudly when the
library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# SOP_LIB names another build of the same sources (the sanitizer test loads
# one whose host code is built with AddressSanitizer)
LIB_PATH = os.environ.get("SOP_LIB") or os.path.join(_PKG, "libsop.so")
HEADER = os.path.join(os.path.dirname(_PKG), "include", "sop.h")

NTERMS = 5
SCHEDULE_PLAIN, SCHEDULE_BATCHED = 0, 1
FORCES_PARTICLE, FORCES_PAIR = 0, 1
INTEGRATOR_OVERDAMPED, INTEGRATOR_UNDERDAMPED = 0, 1
TERM_NAMES = ("fene", "native", "repulsive", "external", "virial")
STATUS = {0: "SOP_OK", -1: "SOP_E_ARG", -2: "SOP_E_STATE", -3: "SOP_E_WORKSPACE",
          -4: "SOP_E_HIP", -5: "SOP_E_FENE", -6: "SOP_E_LIST_OVERFLOW",
          -7: "SOP_E_NONFINITE", -8: "SOP_E_TIP"}


class SopError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status
        self.name = STATUS.get(status, str(status))


class Params(C.Structure):
    _fields_ = [(n, C.c_double) for n in
                ("k_fene", "R0", "eps_h", "eps_l", "sigma", "r_list", "kBT", "zeta", "h")] + [
        ("list_every", C.c_int32), ("list_capacity", C.c_int32), ("seed", C.c_uint64)]


_lib = None


def declared_functions():
    """Names of the functions include/sop.h declares."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(sop_\w+)\s*\(", text, re.M)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                              "python paper_1003_1148_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, dbl, st = C.c_void_p, C.c_int32, C.c_int64, C.c_double, C.c_int
        sigs = {
            "sop_create": [vp, vp, vp],
            "sop_destroy": [vp],
            "sop_load_topology": [vp, i32, vp, vp, i64, vp, vp, i64, vp, vp, vp],
            "sop_set_pulling": [vp, i32, i64, dbl, vp, vp],
            "sop_set_tip": [vp, dbl, dbl, dbl, vp, vp],
            "sop_set_tile": [vp, i32],
            "sop_set_schedule": [vp, i32],
            "sop_set_batch": [vp, i32, i32],
            "sop_get_batch": [vp, vp, vp, vp],
            "sop_autotune": [vp, dbl, C.c_char_p],
            "sop_get_tile": [vp, vp],
            "sop_set_graph_steps": [vp, i32],
            "sop_set_energy_interval": [vp, i64],
            "sop_workspace_size": [vp, vp],
            "sop_bind_workspace": [vp, vp, C.c_size_t],
            "sop_set_coordinates": [vp, vp],
            "sop_get_coordinates": [vp, vp],
            "sop_set_step": [vp, i64],
            "sop_get_step": [vp, vp],
            "sop_step": [vp, i64],
            "sop_build_pairlist": [vp],
            "sop_get_pairlist": [vp, i64, vp, vp],
            "sop_compute_forces": [vp, vp, vp, vp],
            "sop_get_energies": [vp, vp, vp],
            "sop_get_external_force": [vp, vp],
            "sop_synchronize": [vp],
            "sop_sample_noise": [vp, i64, vp, vp],
            "sop_step_timed": [vp, i64, vp],
            "sop_set_list_skin": [vp, dbl],
            "sop_set_force_mode": [vp, i32],
            "sop_set_integrator": [vp, i32, dbl],
            "sop_set_tempering": [vp, i32, vp, i64, vp],
            "sop_get_tempering": [vp, vp, vp, vp],
            "sop_set_velocities": [vp, vp],
            "sop_get_velocities": [vp, vp],
            "sop_get_force_mode": [vp, vp],
            "sop_get_list_stats": [vp, vp, vp],
            "sop_get_list_skin": [vp, vp],
            "sop_running_average": [vp, i64, i32, vp],
            "sop_peak_force": [vp, i64, i32, vp, vp],
            "sop_virial_temperature": [vp, i64, i64, dbl, vp],
            "sop_ramp_workspace_size": [i64, vp],
            "sop_ramp_run": [vp, i64, vp, i64, i64, vp, C.c_size_t, vp, vp],
            "sop_ramp_run_static": [vp, i64, vp, i64, i64, vp, vp],
        }
        for name, args in sigs.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = st
        L.sop_status_string.argtypes = [st]
        L.sop_status_string.restype = C.c_char_p
        L.sop_last_error.argtypes = [vp]
        L.sop_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data


def _stream_handle(stream):
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class Context:
    """One SOP simulation context (one or many trajectories)."""

    def __init__(self, params, stream=None):
        L = lib()
        capacity = int(getattr(params, "list_capacity", 0) or 0)
        self.params = Params(params.k_fene, params.R0, params.eps_h, params.eps_l, params.sigma,
                             params.r_list, params.kBT, params.zeta, params.h,
                             int(params.list_every), capacity, int(params.seed))
        self._stream = stream
        h = C.c_void_p()
        st = L.sop_create(C.byref(self.params), _stream_handle(stream), C.byref(h))
        if st != 0:
            raise SopError(st, "sop_create rejected the parameters")
        self.h = h
        self._ws = None
        self.n_res = 0
        self.n_traj = 0

    # -- helpers ---------------------------------------------------------
    def _check(self, st):
        if st != 0:
            msg = lib().sop_last_error(self.h).decode()
            raise SopError(st, msg)

    def close(self):
        if getattr(self, "h", None):
            lib().sop_destroy(self.h)
            self.h = None
        self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- topology and protocols -----------------------------------------
    def load_topology(self, res_offsets, bonds, bond_r0, natives, native_r0,
                      stream_ids=None, fixed=None):
        ro = np.ascontiguousarray(res_offsets, dtype=np.int64)
        b = np.ascontiguousarray(np.asarray(bonds).reshape(-1, 2), dtype=np.int32)
        br = np.ascontiguousarray(bond_r0, dtype=np.float64)
        nn = np.ascontiguousarray(np.asarray(natives).reshape(-1, 2), dtype=np.int32)
        nr = np.ascontiguousarray(native_r0, dtype=np.float64)
        si = None if stream_ids is None else np.ascontiguousarray(stream_ids, dtype=np.uint32)
        fx = None if fixed is None else np.ascontiguousarray(fixed, dtype=np.uint8)
        self._check(lib().sop_load_topology(self.h, len(ro) - 1, _p(ro), _p(si), len(b), _p(b),
                                            _p(br), len(nn), _p(nn), _p(nr), _p(fx)))
        self.n_traj = len(ro) - 1
        self.n_res = int(ro[-1])

    def set_pulling(self, traj, residue, kappa, anchor0, v):
        a = np.ascontiguousarray(anchor0, dtype=np.float64)
        w = np.ascontiguousarray(v, dtype=np.float64)
        self._check(lib().sop_set_pulling(self.h, int(traj), int(residue), float(kappa), _p(a), _p(w)))

    def set_tip(self, radius, eps, sigma, c0, v):
        a = np.ascontiguousarray(c0, dtype=np.float64)
        w = np.ascontiguousarray(v, dtype=np.float64)
        self._check(lib().sop_set_tip(self.h, float(radius), float(eps), float(sigma), _p(a), _p(w)))

    def set_tile(self, tile):
        self._check(lib().sop_set_tile(self.h, int(tile)))

    def set_schedule(self, schedule):
        if isinstance(schedule, str):
            schedule = {"plain": SCHEDULE_PLAIN, "batched": SCHEDULE_BATCHED}[schedule]
        self._check(lib().sop_set_schedule(self.h, int(schedule)))

    def set_batch(self, wg_residues=0, steps_per_launch=100):
        self._check(lib().sop_set_batch(self.h, int(wg_residues), int(steps_per_launch)))

    def get_batch(self):
        """(residues per workgroup, steps per launch, number of packs)."""
        a, b, c = C.c_int32(0), C.c_int32(0), C.c_int32(0)
        self._check(lib().sop_get_batch(self.h, C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def autotune(self, budget_ms=200.0, cache_path=None):
        cp = None if cache_path is None else os.fsencode(cache_path)
        self._check(lib().sop_autotune(self.h, float(budget_ms), cp))

    def get_tile(self):
        v = C.c_int32(0)
        self._check(lib().sop_get_tile(self.h, C.byref(v)))
        return v.value

    def set_force_mode(self, mode):
        """"particle" (default) or "pair" (SOP_FORCES_*)."""
        m = {"particle": FORCES_PARTICLE, "pair": FORCES_PAIR}.get(mode, mode)
        self._check(lib().sop_set_force_mode(self.h, int(m)))

    def get_force_mode(self):
        v = C.c_int32(0)
        self._check(lib().sop_get_force_mode(self.h, C.byref(v)))
        return "pair" if v.value == FORCES_PAIR else "particle"

    def set_integrator(self, kind, mass=1.0):
        """"overdamped" (default) or "underdamped" (BAOAB, residue mass `mass`)."""
        k = {"overdamped": INTEGRATOR_OVERDAMPED, "underdamped": INTEGRATOR_UNDERDAMPED}.get(kind, kind)
        self._check(lib().sop_set_integrator(self.h, int(k), float(mass)))

    def set_velocities(self, v):
        v = np.ascontiguousarray(v, dtype=np.float64).reshape(-1, 3)
        self._check(lib().sop_set_velocities(self.h, _p(v)))

    def get_velocities(self):
        v = np.zeros((self.n_res, 3))
        self._check(lib().sop_get_velocities(self.h, _p(v)))
        return v

    def set_tempering(self, kbt, exchange_every, tidx=None):
        """Replica exchange over groups of len(kbt) consecutive trajectories."""
        kbt = np.ascontiguousarray(kbt, dtype=np.float64)
        ti = None if tidx is None else np.ascontiguousarray(tidx, dtype=np.int32)
        self._check(lib().sop_set_tempering(self.h, len(kbt), _p(kbt), int(exchange_every), _p(ti)))
        self._n_rep = len(kbt)

    def get_tempering(self):
        """(temperature index per trajectory, accepted, attempted per ladder pair)."""
        R = getattr(self, "_n_rep", 1)
        ti = np.zeros(self.n_traj, dtype=np.int32)
        acc = np.zeros(max(R - 1, 1), dtype=np.int64)
        att = np.zeros(max(R - 1, 1), dtype=np.int64)
        self._check(lib().sop_get_tempering(self.h, _p(ti), _p(acc), _p(att)))
        return ti, acc[:R - 1], att[:R - 1]

    def set_list_skin(self, skin):
        self._check(lib().sop_set_list_skin(self.h, float(skin)))

    def get_list_skin(self):
        v = C.c_double(0.0)
        self._check(lib().sop_get_list_skin(self.h, C.byref(v)))
        return v.value

    def get_list_stats(self):
        """(list rebuilds, skin cell-grid searches) since binding."""
        a, b = C.c_int64(0), C.c_int64(0)
        self._check(lib().sop_get_list_stats(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value

    def set_graph_steps(self, k):
        self._check(lib().sop_set_graph_steps(self.h, int(k)))

    def set_energy_interval(self, k):
        self._check(lib().sop_set_energy_interval(self.h, int(k)))

    # -- workspace ------------------------------------------------------
    def workspace_size(self):
        n = C.c_size_t(0)
        self._check(lib().sop_workspace_size(self.h, C.byref(n)))
        return n.value

    def bind_workspace(self, device_ptr=None, nbytes=None):
        """Bind caller memory, or allocate a torch uint8 CUDA tensor when none is given."""
        if device_ptr is None:
            import torch
            nbytes = self.workspace_size()
            self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device="cuda")
            base = self._ws.data_ptr()
            device_ptr = (base + 255) & ~255
        self._check(lib().sop_bind_workspace(self.h, device_ptr, int(nbytes)))

    # -- state ----------------------------------------------------------
    def set_coordinates(self, x):
        x = np.ascontiguousarray(x, dtype=np.float64)
        assert x.shape == (self.n_res, 3)
        self._check(lib().sop_set_coordinates(self.h, _p(x)))

    def get_coordinates(self):
        x = np.zeros((self.n_res, 3))
        self._check(lib().sop_get_coordinates(self.h, _p(x)))
        return x

    def set_step(self, n):
        self._check(lib().sop_set_step(self.h, int(n)))

    def get_step(self):
        v = C.c_int64(0)
        self._check(lib().sop_get_step(self.h, C.byref(v)))
        return v.value

    def step(self, n):
        self._check(lib().sop_step(self.h, int(n)))

    def step_timed(self, n):
        """Kernel timing. Plain schedule: n back-to-back launches of the step
        kernel, then n of the list rebuild with the skin's cell-grid search,
        then n of the rebuild that only filters the skin rows, each timed as
        one graph; returns (mean step-kernel ms, mean search-and-filter
        rebuild ms, mean filter-only rebuild ms) and leaves the state as it
        was. Batched: advances n steps; (mean persistent-launch ms, 0, steps
        per launch)."""
        ms = np.zeros(3)
        self._check(lib().sop_step_timed(self.h, int(n), _p(ms)))
        return float(ms[0]), float(ms[1]), float(ms[2])

    def synchronize(self):
        self._check(lib().sop_synchronize(self.h))

    # -- list, forces, energies ----------------------------------------
    def build_pairlist(self):
        self._check(lib().sop_build_pairlist(self.h))

    def get_pairlist(self):
        n = C.c_int64(0)
        st = lib().sop_get_pairlist(self.h, 0, None, C.byref(n))
        if st not in (0, -1):
            self._check(st)
        ij = np.zeros((max(n.value, 1), 2), dtype=np.int32)
        self._check(lib().sop_get_pairlist(self.h, n.value, _p(ij), C.byref(n)))
        return ij[:n.value]

    def compute_forces(self):
        F = np.zeros((self.n_res, 3))
        E = np.zeros((self.n_traj, NTERMS))
        fe = np.zeros(self.n_traj)
        self._check(lib().sop_compute_forces(self.h, _p(F), _p(E), _p(fe)))
        return F, E, fe

    def get_energies(self):
        E = np.zeros((self.n_traj, NTERMS))
        s = C.c_int64(0)
        self._check(lib().sop_get_energies(self.h, _p(E), C.byref(s)))
        return E, s.value

    def sample_noise(self, step):
        """(Philox words uint32 (n_res,4), Gaussians (n_res,3)) of one step."""
        w = np.zeros((self.n_res, 4), dtype=np.uint32)
        g = np.zeros((self.n_res, 3))
        self._check(lib().sop_sample_noise(self.h, int(step), _p(w), _p(g)))
        return w, g

    def get_external_force(self):
        fe = np.zeros(self.n_traj)
        self._check(lib().sop_get_external_force(self.h, _p(fe)))
        return fe


def status_string(st):
    return lib().sop_status_string(int(st)).decode()


def _check_host(st, what):
    if st != 0:
        raise SopError(st, what)


def running_average(y, w):
    """w-point running average of a trace (sop_running_average)."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    n = len(y)
    out = np.zeros(max(n - int(w) + 1, 1))
    _check_host(lib().sop_running_average(_p(y), n, int(w), _p(out)), "running average")
    return out[:n - int(w) + 1]


def peak_force(f, w):
    """(largest w-point running average, index of its first window)."""
    f = np.ascontiguousarray(f, dtype=np.float64)
    pk, ix = C.c_double(0.0), C.c_int64(0)
    _check_host(lib().sop_peak_force(_p(f), len(f), int(w), C.byref(pk), C.byref(ix)), "peak force")
    return pk.value, ix.value


def virial_temperature(virial, n_res, kB):
    """Equipartition temperature of a free chain from recorded virials."""
    v = np.ascontiguousarray(virial, dtype=np.float64)
    T = C.c_double(0.0)
    _check_host(lib().sop_virial_temperature(_p(v), len(v), int(n_res), float(kB), C.byref(T)),
                "virial temperature")
    return T.value


class RampParams(C.Structure):
    """sop_ramp_params: the harmonic Brownian particle under a force ramp."""
    _fields_ = [(n, C.c_double) for n in ("rf", "xi", "k_sp", "kBT", "h")] + [
        ("seed", C.c_uint64), ("stream", C.c_uint32), ("order", C.c_int32),
        ("compensated", C.c_int32), ("pad", C.c_int32)]


def ramp_params(rf, xi, k_sp, kBT, h, order=1, seed=0, stream=0, compensated=True):
    return RampParams(float(rf), float(xi), float(k_sp), float(kBT), float(h), int(seed),
                      int(stream), int(order), 1 if compensated else 0, 0)


def ramp_run(rp, x, step0, n_steps, moments=True, stream=None):
    """Advance the particles x (a torch float32 CUDA tensor of shape (M, 2):
    hi, lo) in place by n_steps steps from step0 (sop_ramp_run).  With
    moments, returns (mean, variance) of hi + lo after synchronizing."""
    import torch
    assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[-1] == 2
    M = x.numel() // 2
    nbytes = C.c_size_t(0)
    _check_host(lib().sop_ramp_workspace_size(M, C.byref(nbytes)), "ramp workspace size")
    ws = torch.empty(max(nbytes.value, 8), dtype=torch.uint8, device=x.device) if moments else None
    mom = torch.zeros(2, dtype=torch.float64, device=x.device) if moments else None
    s = _stream_handle(stream if stream is not None else torch.cuda.current_stream())
    _check_host(lib().sop_ramp_run(C.byref(rp), M, x.data_ptr(), int(step0), int(n_steps),
                                   ws.data_ptr() if moments else None, nbytes.value,
                                   mom.data_ptr() if moments else None, s), "sop_ramp_run")
    if not moments:
        return None
    m = mom.cpu().numpy()
    return float(m[0]), float(m[1])


def ramp_run_static(rp, x, step0, n_steps, moments_out=None, stream=None):
    """sop_ramp_run_static: like ramp_run, allocating nothing.  moments_out
    is a caller-owned float64 CUDA tensor of 2 elements (or None); the call
    is asynchronous on the stream."""
    import torch
    assert x.is_cuda and x.dtype == torch.float32 and x.is_contiguous() and x.shape[-1] == 2
    if moments_out is not None:
        assert moments_out.is_cuda and moments_out.dtype == torch.float64 and moments_out.numel() >= 2
    s = _stream_handle(stream if stream is not None else torch.cuda.current_stream())
    _check_host(lib().sop_ramp_run_static(C.byref(rp), x.numel() // 2, x.data_ptr(), int(step0),
                                          int(n_steps),
                                          None if moments_out is None else moments_out.data_ptr(), s),
                "sop_ramp_run_static")


def from_system(system, params, stream=None, tile=0, graph_steps=1, energy_every=0,
                coordinates=None, schedule="plain", batch=None):
    """Load a system description (duck-typed: x, res_offsets, stream_ids, bonds,
    bond_r0, natives, native_r0, fixed, pulls, tip), choose the schedule
    ("plain" or "batched", batch = (residues per workgroup, steps per launch)),
    bind a torch workspace and set the coordinates."""
    ctx = Context(params, stream)
    ctx.load_topology(system.res_offsets, system.bonds, system.bond_r0, system.natives,
                      system.native_r0, stream_ids=system.stream_ids, fixed=system.fixed)
    for p in getattr(system, "pulls", []) or []:
        ctx.set_pulling(p.traj, p.residue, p.kappa, p.anchor0, p.v)
    tip = getattr(system, "tip", None)
    if tip is not None:
        ctx.set_tip(tip.radius, tip.eps, tip.sigma, tip.c0, tip.v)
    ctx.set_schedule(schedule)
    if batch is not None:
        ctx.set_batch(*batch)
    ctx.set_tile(tile)
    ctx.set_graph_steps(graph_steps)
    ctx.set_energy_interval(energy_every)
    ctx.bind_workspace()
    ctx.set_coordinates(system.x if coordinates is None else coordinates)
    return ctx
