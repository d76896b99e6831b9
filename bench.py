#!/usr/bin/env python
"""Benchmark of the batched checkerboard Metropolis sweep on one MI355X.

Workload (the batched configuration of the paper's throughput experiments,
Results, Table 3 / Fig. 3, scaled to one MI355X): 1024 Ising replicas of
256x256 with beta on a 64-point grid over [0.30, 0.60] (16 replicas each),
plus 512 q-state Potts lattices with L drawn from {64, 128, 256, 512, 1024}
and q from {3, 4, 6, 8} at beta ~ U[0.9, 1.1] ln(1 + sqrt q), random initial
states, 10^4 sweeps per step.  Inputs are synthetic (seeded), resident in HBM
before timing starts.

Prints ONE JSON line.  ``value`` is spin-update attempts per ns over the
timed steps (all replicas, both colours).  ``roofline`` reports the dominant
kernel (the streamed colour pass) against the 8 TB/s HBM peak with its
algorithmic traffic of 3 bytes per attempt (read own + other colour plane,
write own), timed live with HIP events on the sampler's stream.
``cpu_baseline`` times the oracle (plain C, OpenMP over replicas) on the
host cores for all replicas of the workload over a few sweeps.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_ATTEMPT = 3  # per colour pass: read own plane + other plane, write own plane


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("lattice_kernels.hip", "spinmc_internal.hpp"):
        with open(os.path.join(ROOT, "paper_2304_01772_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read_traffic(sites_per_pass):
    """HBM bytes per launch from the committed rocprofv3 PMC summary, if it
    was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "stream_pass_batched_ising_potts_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    if d.get("sites_per_pass") != sites_per_pass:
        return None
    return d.get("hbm_bytes_per_launch")


def pass_roofline(kms, nl, sites, kernel, what):
    avg_s = kms / nl * 1e-3
    bytes_per_launch = BYTES_PER_ATTEMPT * sites // 2
    achieved = bytes_per_launch / avg_s / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": read_traffic(sites // 2),
            "kernel": kernel, "units": what, "launches": nl, "avg_launch_us": round(avg_s * 1e6, 2),
            "bytes_per_launch": bytes_per_launch,
            "attempts_per_ns": round(sites // 2 / avg_s / 1e9, 1)}


def ising_stream_probe(Sampler, torch, n_rep, sweeps):
    """The batched Ising sweep alone, streamed through HBM (n_rep replicas of
    256x256, the beta grid of the workload), timed per colour-pass launch."""
    import synth
    reps = synth.batched_ising_potts(n_ising=n_rep, n_potts=0)
    smp = Sampler(reps, seed=2, init=True)
    smp.set_schedule(mode="stream")
    smp.sweep(2)
    torch.cuda.synchronize()
    smp.profile(True)
    smp.sweep(sweeps)
    torch.cuda.synchronize()
    kms, nl = smp.profile_read("stream_pass")
    smp.profile(False)
    sites = sum(r["Lx"] * r["Ly"] for r in reps)
    smp.close()
    return pass_roofline(kms, nl, sites, "k_stream_pass",
                         f"{n_rep} Ising 256x256 replicas, {sweeps} sweeps")


def cpu_baseline(reps, seed, sweeps):
    """The oracle on the host cores: every replica of the workload, a few
    sweeps (a bounded sample of the same chain)."""
    import numpy as np
    from oracle import chain as orc
    ising = [r for r in reps if r["model"] == 0]
    potts = [r for r in reps if r["model"] == 1]
    si = [orc.ising_init(r["Lx"], r["Ly"], seed, r["rid"]) for r in ising]
    sp = [orc.potts_init(r["Lx"], r["Ly"], r["q"], seed, r["rid"]) for r in potts]
    t0 = time.perf_counter()
    orc.ising_run_batch(si, [r["Jx"] for r in ising], [r["Jy"] for r in ising],
                        [r["h"] for r in ising], [r["beta"] for r in ising], seed,
                        np.array([r["rid"] for r in ising]), 0, sweeps)
    orc.potts_run_batch(sp, [r["q"] for r in potts], [r["Jx"] for r in potts],
                        [r["h"] for r in potts], [r["beta"] for r in potts], seed,
                        np.array([r["rid"] for r in potts]), 0, sweeps)
    dt = time.perf_counter() - t0
    att = sum(r["Lx"] * r["Ly"] for r in reps) * sweeps
    return dict(value=att / dt / 1e9, unit="attempts/ns", cores=orc.num_threads(), kind="oracle",
                sample=f"all {len(reps)} replicas of the workload, {sweeps} sweeps "
                       f"({att:.3g} attempts, {dt:.1f} s wall)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--sweeps", type=int, default=10000, help="sweeps per step")
    ap.add_argument("--mode", default="tuned",
                    choices=["tuned", "auto", "resident", "stream", "hybrid"],
                    help="schedule; 'tuned' runs the library's autotuner first")
    ap.add_argument("--tune-sweeps", type=int, default=20)
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--threads", type=int, default=0)
    ap.add_argument("--cpu-sweeps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-probes", action="store_true",
                    help="skip the Ising streaming probes (for counter collection runs)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device copy of this many MiB (the reference "
                         "dispatch that scales rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the workload is "
                                   "independent replicas, sharded by replica across GPUs with no "
                                   "communication (see the design notes); --gpus must be 1"}))
        sys.exit(2)

    import torch
    import synth
    from paper_2304_01772_amd.sampler import Sampler

    reps = synth.batched_ising_potts()
    seed = 2
    sites = sum(r["Lx"] * r["Ly"] for r in reps)
    print(f"# workload: {len(reps)} replicas, {sites} sites/sweep, {args.sweeps} sweeps/step",
          file=sys.stderr, flush=True)
    smp = Sampler(reps, seed=seed, init=True)
    tuning = None
    if args.mode == "tuned":
        chosen, rates = smp.autotune(trial_sweeps=args.tune_sweeps)
        tuning = dict(chosen=chosen, candidate_rates=[round(r, 1) for r in rates])
        print(f"# autotune: {tuning}", file=sys.stderr, flush=True)
    else:
        smp.set_schedule(mode=args.mode, tile_rows=args.tile_rows, wg_threads=args.threads)
    for w in range(args.warmup):
        smp.sweep(args.sweeps)
        torch.cuda.synchronize()
        print(f"# warmup step {w + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    smp.profile(True)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(smp.stream)
    for k in range(args.steps):
        smp.sweep(args.sweeps)
    e1.record(smp.stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    print(f"# timed {args.steps} steps: {ms:.1f} ms", file=sys.stderr, flush=True)
    attempts = sites * args.sweeps * args.steps
    value = attempts / (ms * 1e6)

    # dominant kernel: the streamed colour pass (resident kernel if nothing streams)
    streamed, resident = smp.schedule_sites()
    kms, nl = smp.profile_read("stream_pass")
    rms, rl = smp.profile_read("resident")
    smp.profile(False)
    roof = None
    if nl > 0 and streamed > 0:
        roof = pass_roofline(kms, nl, streamed, "k_stream_pass",
                             "batched Ising+Potts, streamed replicas")
    elif rl > 0:
        # LDS-resident multi-sweep kernel: no HBM traffic per sweep; ALU bound
        per_launch_attempts = resident * args.sweeps
        rate = per_launch_attempts / (rms / rl * 1e-3)
        roof = {"bound": "alu", "achieved": round(rate / 1e12, 4), "peak": None,
                "unit": "Tattempts/s", "frac": None, "traffic": None,
                "kernel": "k_resident", "launches": rl}
    sched = smp.get_schedule()
    smp.close()

    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    probes = {}
    for n_rep in (() if args.no_probes else (1024, 8192)):
        probes[f"ising_{n_rep}x256x256_stream"] = ising_stream_probe(Sampler, torch, n_rep, 100)
        print(f"# Ising stream probe {n_rep}: {probes[f'ising_{n_rep}x256x256_stream']}",
              file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("# cpu baseline (oracle on host cores)...", file=sys.stderr, flush=True)
        cpu = cpu_baseline(reps, seed, args.cpu_sweeps)

    out = {
        "metric": "spin-update attempts/ns",
        "value": round(value, 2),
        "unit": "attempts/ns",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms / args.steps, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {
            "workload": "1024 Ising 256x256 (beta grid 0.30-0.60) + 512 Potts L in "
                        "{64..1024}, q in {3,4,6,8}, beta in [0.9,1.1] ln(1+sqrt q); "
                        f"{args.sweeps} checkerboard sweeps per step",
            "replicas": len(reps),
            "sites_per_sweep": sites,
            "sweeps_per_step": args.sweeps,
            "schedule": sched,
            "autotune": tuning,
            "streamed_sites": streamed,
            "resident_sites": resident,
        },
        "roofline": roof,
        "ising_stream_roofline": probes,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
