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


def cpu_baseline(P, np, system, params, n_steps):
    """The oracle timed on one host core over a sample of the workload, and
    the GPU path's agreement with it on that sample: the force error at the
    start and the largest coordinate difference after the sample's steps."""
    import oracle
    o = oracle.OracleSystem(system, params)
    t0 = time.perf_counter()
    xo, _, _, st = o.run(system.x, n_steps)
    dt = time.perf_counter() - t0
    if st != 0:
        raise RuntimeError(f"oracle status {st}")
    # forces at the start (the native structure: bonded and native terms
    # near zero, so the net forces are small) and at the oracle's end point
    Fo0, _, _, _ = o.forces(system.x, step=0)
    Fo1, _, _, _ = o.forces(xo, step=n_steps)
    g = P.from_system(system, params)
    F0, _, _ = g.compute_forces()
    g.step(n_steps)
    xg = g.get_coordinates()
    g.close()
    h = P.from_system(system, params, coordinates=xo)
    h.set_step(n_steps)
    F1, _, _ = h.compute_forces()
    h.close()
    return {"value": system.n_res * n_steps / dt, "unit": "residue-steps/s", "cores": 1,
            "kind": "oracle",
            "sample": f"{n_steps} steps ({(n_steps + params.list_every - 1) // params.list_every} "
                      f"list rebuilds) of the {system.n_res}-residue workload, FP64, one thread",
            "seconds": dt,
            "agreement": {
                "force_rel_err_start": float(np.linalg.norm(F0 - Fo0) / np.linalg.norm(Fo0)),
                "force_rel_err_end": float(np.linalg.norm(F1 - Fo1) / np.linalg.norm(Fo1)),
                "max_dx_A": float(np.linalg.norm(xg - xo, axis=1).max()),
                "steps": n_steps,
                "note": "GPU plain schedule against the oracle from the same start and Philox "
                        "stream: L2 force error at the start and at the oracle's end point, "
                        "largest coordinate difference after the steps"}}


def batched_leg(P, make_config, RunParams, np, energy_every, steps, n_seq, seq_steps):
    """The ensemble of 4,096 trajectories of 50-500 residues in the batched
    schedule, against the same library run one trajectory at a time (plain
    schedule) on a random sample of the ensemble's trajectories."""
    note("generating the 4,096-trajectory ensemble")
    s = make_config("c3")
    p = RunParams()
    ctx = P.from_system(s, p, schedule="batched", energy_every=energy_every)
    ctx.autotune(budget_ms=400.0)
    wg, K, n_packs = ctx.get_batch()
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
    rng = np.random.default_rng(5)
    pick = rng.choice(s.n_traj, size=n_seq, replace=False)
    work = tsum = 0.0
    for t in pick:
        sub = s.subset([int(t)])
        c = P.from_system(sub, p, energy_every=energy_every)
        c.step(100)
        c.synchronize()
        t0 = time.perf_counter()
        c.step(seq_steps)
        c.synchronize()
        tsum += time.perf_counter() - t0
        work += sub.n_res * seq_steps
        c.close()
    seq = work / tsum
    note(f"sequential single-trajectory launches: {seq:.4e} residue-steps/s; "
         f"batched speedup {rate / seq:.1f}x")
    return {
        "workload": f"{s.n_traj} independent trajectories, chain lengths U[50, 500], "
                    f"{s.n_res} residues",
        "value": rate, "unit": "residue-steps/s", "steps": steps,
        "wg_residues": wg, "steps_per_launch": K, "n_packs": n_packs,
        "launch_us": launch_ms * 1e3,
        "sequential": {"value": seq, "trajectories": int(n_seq), "steps_each": seq_steps,
                       "schedule": "plain, one trajectory per context"},
        "speedup_vs_sequential": rate / seq,
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000, help="timed list periods")
    ap.add_argument("--warmup", type=int, default=100, help="untimed list periods")
    ap.add_argument("--tile", type=int, default=0, help="residues per workgroup (64/128/256; 0 = autotune)")
    ap.add_argument("--graph-periods", type=int, default=10)
    ap.add_argument("--energy-every", type=int, default=1000)
    ap.add_argument("--timing-steps", type=int, default=300)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--batched-steps", type=int, default=2000)
    ap.add_argument("--seq-trajectories", type=int, default=64)
    ap.add_argument("--seq-steps", type=int, default=2000)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run device-to-device copies of MIB MiB (for memory counters)")
    args = ap.parse_args()
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
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the ensemble shards with no communication; see the design notes).",
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

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(L * args.steps)
    ctx.synchronize()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    value = N * L * args.steps / dt
    note(f"timed {args.steps} periods in {dt:.3f} s: {value:.4e} residue-steps/s")

    k_ms, rb_ms, _ = ctx.step_timed(args.timing_steps)
    note(f"fused step kernel {k_ms * 1e3:.2f} us, list rebuild {rb_ms * 1e3:.2f} us")
    bytes_step = N * (64 + 12 + 8 * b + 8 * c + 4 * pp)
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
            "graph_periods": args.graph_periods,
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
        },
    }
    if not args.no_batched:
        out["batched"] = batched_leg(P, make_config, RunParams, np, args.energy_every,
                                     args.batched_steps, args.seq_trajectories, args.seq_steps)
    if not args.no_cpu_baseline:
        note(f"oracle CPU baseline: {args.cpu_steps} steps")
        out["cpu_baseline"] = cpu_baseline(P, np, s, p, args.cpu_steps)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
