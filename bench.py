#!/usr/bin/env python3
"""Throughput of SOP overdamped Langevin dynamics on one MI355X.

Workload: the 75,000-residue shell assembly (300 copies of a 250-residue
globular subunit on a 300 A sphere, inter-subunit native contacts, a 50 A
indentation tip), the configuration the HBM-roofline target is quoted on.
One bench step is one list period: a Verlet-list rebuild plus list_every
(10) fused force/noise/update steps; energies are recorded every 1,000
steps.  The reported value is residue-steps per second over the timed
steps, inputs resident in device memory.

Prints one JSON line on stdout; progress goes to stderr.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("residue-steps/sec on 1 MI355X (plain vs batched/FP32-compensated, "
          "force rel err ≤1e-5)")
HBM_PEAK_GBS = 8000.0


def note(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1003_1148_amd", "csrc", "sop_kernels.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_counters():
    """The committed counter summary of the step kernel (HBM bytes and VALU
    instructions per launch), if it was taken on the current kernel source."""
    path = os.path.join(ROOT, "profiles", "k_tile_step_c2_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return d


def copy_bandwidth(torch, mib=1024, reps=10):
    """Achievable HBM rate of a plain device copy (bytes read + written per
    second), timed with events on the current stream."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2.0 * n * 4 / (ms * 1e-3) / 1e9


def host_cpu(raw=False):
    """CPU model and the number of cores this process may run on (with raw,
    also the count before the cap of 16 worker threads)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    # the box's share of its host: at most 16 worker threads per GPU
    if raw:
        return model, max(1, min(ncpu, 16)), ncpu
    return model, max(1, min(ncpu, 16))


def cpu_baseline(P, np, system, params, n_steps, n_steps_par):
    """The oracle timed on the host over a sample of the workload: its
    residue-parallel form on all the cores this process may use (the
    reported value), and its serial form on one core; plus the GPU path's
    agreement with it on the serial sample: the force error at the start and
    the largest coordinate difference after the sample's steps."""
    import oracle
    model, ncpu, nproc = host_cpu(raw=True)
    o = oracle.OracleSystem(system, params)
    t0 = time.perf_counter()
    xp, _, _, st = o.run_par(system.x, n_steps_par, threads=ncpu)
    dt_par = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError(f"oracle status {st}")
    t0 = time.perf_counter()
    xo, _, _, st = o.run(system.x, n_steps)
    dt = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError(f"oracle status {st}")
    # forces at the start (the native structure: bonded and native terms
    # near zero, so the net forces are small) and at the oracle's end point
    Fo0, _, _, _ = o.forces(system.x, step=0)
    Fo1, _, _, _ = o.forces(xo, step=n_steps)
    S0, _ = o.force_scale(system.x, step=0)
    S0 = S0 + 0.05 * o.force_stiffness(system.x, step=0)
    g = P.from_system(system, params)
    F0, _, _ = g.compute_forces()
    g.step(n_steps)
    xg = g.get_coordinates()
    g.close()
    h = P.from_system(system, params, coordinates=xo)
    h.set_step(n_steps)
    F1, _, _ = h.compute_forces()
    h.close()
    rate_par = system.n_res * n_steps_par / dt_par
    rate_1 = system.n_res * n_steps / dt
    L = params.list_every
    return {"value": rate_par, "unit": "residue-steps/s", "cores": ncpu,
            "kind": "oracle",
            "sample": f"{n_steps_par} steps ({(n_steps_par + L - 1) // L} list rebuilds) of the "
                      f"{system.n_res}-residue workload, FP64, residue-parallel form on {ncpu} threads",
            "seconds": dt_par,
            "cpu_model": model,
            "host_cpus_available": nproc,
            "single_thread": {"value": rate_1, "unit": "residue-steps/s", "cores": 1,
                              "sample": f"{n_steps} steps, serial form", "seconds": dt},
            "agreement": {
                "force_rel_err_start": float(np.linalg.norm(F0 - Fo0) / np.linalg.norm(Fo0)),
                "force_max_scaled_err_start": float(
                    (np.linalg.norm(F0 - Fo0, axis=1) / np.maximum(S0, 1e-300)).max()),
                "force_rel_err_end": float(np.linalg.norm(F1 - Fo1) / np.linalg.norm(Fo1)),
                "max_dx_A": float(np.linalg.norm(xg - xo, axis=1).max()),
                "steps": n_steps,
                "note": "GPU plain schedule against the serial oracle from the same start and "
                        "Philox stream: L2 force error and largest per-residue error over the "
                        "residue's force scale S_i + 0.05 K_i (|dE/dr| and r |d2E/dr2| sums) at "
                        "the start, L2 error at the oracle's end point, largest coordinate "
                        "difference after the steps"}}


def alg_bytes(b, c, p, L):
    """Algorithmic bytes per residue-step: compensated positions read and
    written (64), three row pointers (12), bonded and native entries (8 each),
    list pairs once each (4), and the list rebuild every L steps (position,
    cell and list written: 16 + 12 + 4p)."""
    return 64 + 12 + 8 * b + 8 * c + 4 * p + (28 + 4 * p) / L


def batched_leg(P, make_config, RunParams, np, energy_every, steps, n_seq, seq_steps, n_check):
    """The ensemble of 4,096 trajectories of 50-500 residues in the batched
    schedule, against the same library run one trajectory at a time (plain
    schedule) on a random sample of the ensemble's trajectories; with its
    force error and drift against the oracle on a sample of trajectories."""
    import oracle
    note("generating the 4,096-trajectory ensemble")
    s = make_config("c3")
    p = RunParams()
    ctx = P.from_system(s, p, schedule="batched", energy_every=energy_every)
    ctx.autotune(budget_ms=400.0)
    wg, K, n_packs = ctx.get_batch()
    # accuracy on a sample of trajectories, from the start coordinates
    rng = np.random.default_rng(11)
    chk = sorted(int(t) for t in rng.choice(s.n_traj, size=n_check, replace=False))
    idx = np.concatenate([np.arange(s.res_offsets[t], s.res_offsets[t + 1]) for t in chk])
    sub = s.subset(chk)
    osub = oracle.OracleSystem(sub, p)
    Fg, _, _ = ctx.compute_forces()
    Fo, _, _, st = osub.forces(sub.x)
    So, _ = osub.force_scale(sub.x)
    So = So + 0.05 * osub.force_stiffness(sub.x)
    n_pairs = len(ctx.get_pairlist())
    ctx.step(200)
    xg = ctx.get_coordinates()[idx]
    xo, _, _, st2 = osub.run(sub.x, 200)
    if st != 0 or st2 != 0:
        raise RuntimeError(f"oracle status {st}, {st2}")
    dF = np.linalg.norm(Fg[idx] - Fo, axis=1)
    accuracy = {"trajectories": n_check, "residues": int(len(idx)),
                "force_rel_err": float(np.linalg.norm(Fg[idx] - Fo) / np.linalg.norm(Fo)),
                "force_max_scaled_err": float((dF / np.maximum(So, 1e-300)).max()),
                "max_dx_A_200_steps": float(np.linalg.norm(xg - xo, axis=1).max())}
    note(f"batched accuracy on {n_check} trajectories: {accuracy}")
    ctx.set_coordinates(s.x)
    ctx.set_step(0)
    ctx.step(2 * K)
    ctx.synchronize()
    t0 = time.perf_counter()
    ctx.step(steps)
    ctx.synchronize()
    dt = time.perf_counter() - t0
    rate = s.n_res * steps / dt
    launch_ms, _, _ = ctx.step_timed(3 * K)
    note(f"batched: {s.n_res} residues, {n_packs} packs of <= {wg}, {K} steps/launch: "
         f"{rate:.4e} residue-steps/s ({launch_ms * 1e3:.1f} us per launch)")
    ctx.close()
    N = s.n_res
    b, c, pp = len(s.bonds) / N, len(s.natives) / N, n_pairs / N
    B = alg_bytes(b, c, pp, p.list_every)
    achieved = rate * B / 1e9
    pick = rng.choice(s.n_traj, size=n_seq, replace=False)
    work = tsum = 0.0
    for t in pick:
        sub = s.subset([int(t)])
        c1 = P.from_system(sub, p, energy_every=energy_every)
        c1.step(100)
        c1.synchronize()
        t0 = time.perf_counter()
        c1.step(seq_steps)
        c1.synchronize()
        tsum += time.perf_counter() - t0
        work += sub.n_res * seq_steps
        c1.close()
    seq = work / tsum
    note(f"sequential single-trajectory launches: {seq:.4e} residue-steps/s; "
         f"batched speedup {rate / seq:.1f}x")
    return {
        "workload": f"{s.n_traj} independent trajectories, chain lengths U[50, 500], "
                    f"{s.n_res} residues",
        "value": rate, "unit": "residue-steps/s", "steps": steps,
        "wg_residues": wg, "steps_per_launch": K, "n_packs": n_packs,
        "launch_us": launch_ms * 1e3,
        "roofline": {"bound": "hbm", "kernel": "k_batch (whole ensemble step, rebuilds included)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_residue_step": B,
                     "bonds_per_res": round(b, 4), "natives_per_res": round(c, 4),
                     "list_pairs_per_res": round(pp, 3),
                     "note": "positions stay in LDS between steps, so the kernel's own HBM "
                             "traffic is far below these algorithmic bytes"},
        "accuracy": accuracy,
        "sequential": {"value": seq, "trajectories": int(n_seq), "steps_each": seq_steps,
                       "schedule": "plain, one trajectory per context"},
        "speedup_vs_sequential": rate / seq,
    }


def precision_study(P, np, n_steps, every, out_path):
    """The 250,000-residue fibre (1,000 copies of the 250-residue subunit
    stacked along x, |x| up to 1.8e4 A): the GPU path (single-precision
    forces, compensated single-precision positions) against the FP64 oracle
    from the same start and Philox stream.  Every `every` steps: the force
    error of the GPU forces against the oracle's on the GPU's coordinates
    (L2 relative, and the largest per-residue error over the residue's force
    scale S_i), and the RMS and largest distance between the two
    trajectories.  The oracle runs its residue-parallel form."""
    import oracle
    from synth import RunParams, make_config
    note("generating the 250,000-residue fibre")
    s = make_config("c4")
    p = RunParams()
    _, ncpu = host_cpu()
    o = oracle.OracleSystem(s, p)
    c = P.from_system(s, p, graph_steps=every // p.list_every)
    snaps, rows = [], []
    t0 = time.perf_counter()
    for k in range(1, n_steps // every + 1):
        c.step(every)
        xg = c.get_coordinates()
        F, _, _ = c.compute_forces()
        Fo, _, _, st = o.forces_par(xg, step=k * every, threads=ncpu)
        if st != 0:
            raise RuntimeError(f"oracle status {st}")
        S = (o.force_scale_par(xg, step=k * every, threads=ncpu)
             + 0.05 * o.force_stiffness_par(xg, step=k * every, threads=ncpu))
        dF = np.linalg.norm(F - Fo, axis=1)
        rows.append({"step": k * every,
                     "force_rel_err": float(np.linalg.norm(F - Fo) / np.linalg.norm(Fo)),
                     "force_max_scaled_err": float((dF / np.maximum(S, 1e-300)).max())})
        snaps.append(xg)
        if k % 10 == 0:
            note(f"GPU step {k * every}: force error {rows[-1]['force_rel_err']:.3e} (L2), "
                 f"{rows[-1]['force_max_scaled_err']:.3e} (per residue / S)")
    gpu_s = time.perf_counter() - t0
    rebuilds, searches = c.get_list_stats()
    c.close()
    xo = s.x.copy()
    t1 = time.perf_counter()
    for k in range(1, n_steps // every + 1):
        xo, _, _, st = o.run_par(xo, every, step0=(k - 1) * every, threads=ncpu)
        if st != 0:
            raise RuntimeError(f"oracle status {st}")
        d = np.linalg.norm(snaps[k - 1] - xo, axis=1)
        rows[k - 1]["rms_dx_A"] = float(np.sqrt((d * d).mean()))
        rows[k - 1]["max_dx_A"] = float(d.max())
        r = rows[k - 1]
        note(f"step {r['step']}: force {r['force_rel_err']:.3e} / {r['force_max_scaled_err']:.3e}, "
             f"drift rms {r['rms_dx_A']:.3e} max {r['max_dx_A']:.3e} A "
             f"(oracle {time.perf_counter() - t1:.0f} s)")
    out = {"workload": f"{s.n_res}-residue fibre, |x| up to {np.abs(s.x).max():.0f} A",
           "steps": n_steps, "every": every, "oracle_threads": ncpu,
           "gpu_seconds": gpu_s, "oracle_seconds": time.perf_counter() - t1,
           "list_rebuilds": rebuilds, "skin_searches": searches,
           "max_force_rel_err": max(r["force_rel_err"] for r in rows),
           "max_force_scaled_err": max(r["force_max_scaled_err"] for r in rows),
           "max_dx_A": max(r["max_dx_A"] for r in rows), "rows": rows}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: v for k, v in out.items() if k != "rows"}), flush=True)


def ramp_study(P, np, torch, out_path, n_free, n_noise, m_noise):
    """Section IV.C's accuracy test with the paper's parameters (pN, nm, ps:
    K_sp = 40 pN/nm, kB T = 4.14 pN nm, D = 1.5e-11 cm^2/s, r_f = kappa nu_0 =
    1e-8 pN/ps; X(0) = 0; h = 1, 25, 50 ps): the relative error of the mean
    extension against Eq. 3, for the first- and second-order schemes.
    Noise-free single particles (the schemes' own error, over n_free steps),
    with compensated and with plain single-precision positions, and
    ensembles of m_noise particles with noise over n_noise steps (their mean
    also against the exact mean of the scheme, the Eq. 4 / Eq. 5 recursion,
    with the standard error of the sample mean)."""
    import oracle
    KSP, KBT, RF = 40.0, 4.14, 1e-8
    XI = KBT / 1.5e-9
    rows = []
    for h in (1.0, 25.0, 50.0):
        for order in (1, 2):
            row = {"h_ps": h, "order": order}
            t_free = n_free * h
            exact = oracle.ramp_mean_exact(0.0, RF, XI, KSP, t_free)
            rec = oracle.ramp_mean_recursion(order, 0.0, RF, XI, KSP, h, n_free)
            row["free"] = {"steps": n_free, "t_ps": t_free, "eq3_nm": exact,
                           "recursion_rel_err_vs_eq3": abs(rec - exact) / exact}
            for comp in (True, False):
                x = torch.zeros((1, 2), dtype=torch.float32, device="cuda")
                rp = P.ramp_params(RF, XI, KSP, 0.0, h, order=order, compensated=comp)
                t0 = time.perf_counter()
                P.ramp_run(rp, x, 0, n_free, moments=False)
                torch.cuda.synchronize()
                dt = time.perf_counter() - t0
                v = x.cpu().numpy().astype(np.float64)[0]
                X = v[0] + (v[1] if comp else 0.0)
                key = "compensated" if comp else "plain_fp32"
                row["free"][key] = {"X_nm": X, "rel_err_vs_eq3": abs(X - exact) / exact,
                                    "rel_err_vs_recursion": abs(X - rec) / abs(rec), "seconds": dt}
            t_n = n_noise * h
            exact_n = oracle.ramp_mean_exact(0.0, RF, XI, KSP, t_n)
            rec_n = oracle.ramp_mean_recursion(order, 0.0, RF, XI, KSP, h, n_noise)
            x = torch.zeros((m_noise, 2), dtype=torch.float32, device="cuda")
            rp = P.ramp_params(RF, XI, KSP, KBT, h, order=order, seed=2024, stream=order)
            t0 = time.perf_counter()
            mean, var = P.ramp_run(rp, x, 0, n_noise)
            dt = time.perf_counter() - t0
            se = float(np.sqrt(var / m_noise))
            row["noise"] = {"particles": m_noise, "steps": n_noise, "t_ps": t_n, "eq3_nm": exact_n,
                            "mean_nm": mean, "std_err_nm": se,
                            "rel_err_vs_eq3": abs(mean - exact_n) / exact_n,
                            "rel_err_vs_recursion": abs(mean - rec_n) / abs(rec_n),
                            "rel_std_err": se / exact_n, "seconds": dt,
                            "particle_steps_per_s": m_noise * n_noise / dt}
            note(f"h {h} ps order {order}: free comp {row['free']['compensated']['rel_err_vs_eq3']:.2e} "
                 f"plain {row['free']['plain_fp32']['rel_err_vs_eq3']:.2e}; noise "
                 f"{row['noise']['rel_err_vs_eq3']:.2e} (s.e. {row['noise']['rel_std_err']:.2e})")
            rows.append(row)
    out = {"workload": "harmonic Brownian particle under a force ramp (Section IV.C), paper parameters",
           "rows": rows}
    with open(out_path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed list periods")
    ap.add_argument("--warmup", type=int, default=100, help="untimed list periods")
    ap.add_argument("--tile", type=int, default=0, help="residues per workgroup (64/128/256; 0 = autotune)")
    ap.add_argument("--skin", type=float, default=6.0,
                    help="Verlet skin in A (the library's default is 4); it changes no result, "
                         "only how often the cell-grid search runs (6 A: best of 3-7 A on this "
                         "workload)")
    ap.add_argument("--graph-periods", type=int, default=10)
    ap.add_argument("--energy-every", type=int, default=1000)
    ap.add_argument("--timing-steps", type=int, default=300)
    ap.add_argument("--cpu-steps", type=int, default=60, help="serial oracle sample")
    ap.add_argument("--cpu-steps-par", type=int, default=200, help="residue-parallel oracle sample")
    ap.add_argument("--check-trajectories", type=int, default=12,
                    help="batched trajectories checked against the oracle")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--seq-trajectories", type=int, default=64)
    ap.add_argument("--seq-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (for memory counters)")
    ap.add_argument("--precision-study", metavar="JSON", default=None,
                    help="only run the fibre precision study and write its table to JSON")
    ap.add_argument("--study-steps", type=int, default=10000)
    ap.add_argument("--ramp-study", metavar="JSON", default=None,
                    help="only run the integrator-accuracy study and write it to JSON")
    ap.add_argument("--ramp-free-steps", type=int, default=10**8)
    ap.add_argument("--ramp-noise-steps", type=int, default=10**6)
    ap.add_argument("--ramp-particles", type=int, default=10**5)
    args = ap.parse_args()
    if args.ramp_study:
        import numpy as np
        import torch
        import paper_1003_1148_amd as P
        assert torch.cuda.is_available(), "the accuracy study needs a GPU"
        ramp_study(P, np, torch, args.ramp_study, args.ramp_free_steps, args.ramp_noise_steps,
                   args.ramp_particles)
        return
    if args.precision_study:
        import numpy as np
        import torch
        import paper_1003_1148_amd as P
        assert torch.cuda.is_available(), "the precision study needs a GPU"
        precision_study(P, np, args.study_steps, 100, args.precision_study)
        return
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        note(f"copied {args.calibrate_copy} MiB 5 times")
        return

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(an ensemble shards by trajectory with no communication).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1003_1148_amd as P
    from synth import RunParams, make_config

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    note("generating the 75,000-residue assembly")
    s = make_config("c2")
    p = RunParams()
    L = p.list_every
    ctx = P.from_system(s, p, tile=args.tile, graph_steps=args.graph_periods,
                        energy_every=args.energy_every)
    if args.skin is not None:
        ctx.set_list_skin(args.skin)
    if args.tile == 0:
        ctx.autotune(budget_ms=300.0)
    ctx.build_pairlist()
    n_pairs = len(ctx.get_pairlist())
    N = s.n_res
    b = len(s.bonds) / N
    c = len(s.natives) / N
    pp = n_pairs / N
    note(f"N={N} bonds/res={b:.3f} natives/res={c:.3f} list pairs/res={pp:.2f}")

    note(f"warmup {args.warmup} periods")
    ctx.step(L * args.warmup)
    ctx.synchronize()
    # graph capture and instantiation stay out of the timed region: step on
    # to the next energy record (a multiple of the graph span), then one
    # more whole span, so both graph variants (with and without the energy
    # record) exist before t0
    span = L * max(args.graph_periods, 1)
    st0 = ctx.get_step()
    E = args.energy_every if args.energy_every > 0 else span
    to = ((st0 + E - 1) // E) * E + span - st0
    ctx.step(to)
    ctx.synchronize()
    capture_steps = to

    reb0, srch0 = ctx.get_list_stats()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(L * args.steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    reb1, srch1 = ctx.get_list_stats()
    n_reb, n_srch = reb1 - reb0, srch1 - srch0
    value = N * L * args.steps / dt
    note(f"timed {args.steps} periods in {dt:.3f} s: {value:.4e} residue-steps/s")

    k_ms, search_ms, filter_ms = ctx.step_timed(args.timing_steps)
    B_whole = alg_bytes(b, c, pp, L)
    search_frac = n_srch / max(n_reb, 1)
    rb_ms = filter_ms + search_frac * (search_ms - filter_ms)
    note(f"fused step kernel {k_ms * 1e3:.2f} us; rebuild {filter_ms * 1e3:.2f} us filtering the "
         f"skin, {search_ms * 1e3:.2f} us with the cell-grid search, which {n_srch} of the "
         f"{n_reb} timed rebuilds ran: {rb_ms * 1e3:.2f} us per rebuild on average")
    bytes_step = N * (64 + 12 + 8 * b + 8 * c + 4 * pp)  # one step kernel launch
    achieved = bytes_step / (k_ms * 1e-3) / 1e9
    copy_gbs = copy_bandwidth(torch)
    note(f"device copy {copy_gbs:.0f} GB/s")
    counters = measured_counters()
    traffic = counters.get("hbm_bytes_per_launch") if counters else None
    # share of the chip's vector issue slots the kernel's VALU instructions
    # take: 4 cycles per wave instruction on 1,024 SIMDs at 2.4 GHz
    valu = counters.get("sq_insts_valu_per_dispatch") if counters else None
    valu_frac = valu * 4.0 / (1024 * 2.4e9 * k_ms * 1e-3) if valu else None

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "residue-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "ms_per_md_step": dt * 1e3 / (L * args.steps),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {
            "workload": "75,000-residue shell assembly: 300 x 250-residue subunits on a 300 A "
                        "sphere, indentation tip, list cutoff 20 A rebuilt every 10 steps",
            "n_res": N,
            "md_steps_per_step": L,
            "energy_every": args.energy_every,
            "tile": ctx.get_tile(),
            "skin_A": ctx.get_list_skin(),
            "graph_periods": args.graph_periods,
            "capture_steps_untimed": capture_steps,
            "bonds_per_res": round(b, 4),
            "natives_per_res": round(c, 4),
            "list_pairs_per_res": round(pp, 3),
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "k_tile_step (fused forces + Philox noise + compensated update)",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "copy_GBps": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
            "traffic": traffic,
            "valu_issue_frac": valu_frac,
            "alg_bytes_per_launch": bytes_step,
            "kernel_us": k_ms * 1e3,
            "rebuild_us": rb_ms * 1e3,
            "rebuild_filter_us": filter_ms * 1e3,
            "rebuild_search_us": search_ms * 1e3,
            "rebuild_note": "a rebuild run on its own (explicit list builds): the search kernels' "
                            "early exits and the filter kernel, or the cell-grid search; while "
                            "stepping, the first step of a period filters the skin rows itself",
            "list_upkeep_us_per_period": dt * 1e6 / args.steps - L * k_ms * 1e3,
            "list_upkeep_note": "the timed period less ten plain step launches: the first step's "
                                "filtering, the search kernels (early exits, and the searches "
                                "that fell in the timed periods), the last step's binning, "
                                "energy records and launch gaps",
            "timed_rebuilds": n_reb,
            "timed_skin_searches": n_srch,
            "whole_step": {
                "alg_bytes_per_residue_step": B_whole,
                "achieved": value * B_whole / 1e9,
                "frac": value * B_whole / 1e9 / HBM_PEAK_GBS,
                "note": "the timed rate (list rebuilds, launch gaps and energy records "
                        "included) times the algorithmic bytes of a residue-step with its "
                        "share of the rebuild"},
        },
        "paper_context": {
            "speedup": "about 30x, GPU over CPU",
            "hardware": "GeForce GTX 295 (one GT200 GPU, 240 ALUs at 1.24 GHz, FP32) against one "
                        "core of a Xeon at 2.66 GHz running heavily tuned FP64 code",
            "note": "another machine's figure, for context; the oracle here is a plain FP64 "
                    "reference, not tuned code"},
    }
    if not args.no_batched:
        out["batched"] = batched_leg(P, make_config, RunParams, np, args.energy_every,
                                     args.batched_steps, args.seq_trajectories, args.seq_steps,
                                     args.check_trajectories)
    if not args.no_cpu_baseline:
        note(f"oracle CPU baseline: {args.cpu_steps} steps serial, {args.cpu_steps_par} parallel")
        cb = cpu_baseline(P, np, s, p, args.cpu_steps, args.cpu_steps_par)
        cb["gpu_over_oracle"] = value / cb["value"]
        cb["gpu_over_oracle_single_thread"] = value / cb["single_thread"]["value"]
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
