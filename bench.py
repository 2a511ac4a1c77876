#!/usr/bin/env python3
"""Benchmark of the swarm evaluation of 3DPIFCM on one MI355X.

Workload "ragged6-swarm64": six random-ellipsoid volumes with X, Y uniform in
64..256 and Z in 64..128 (seed 4), 64 particles (lambda, xi) ~ U[0,1)^2
(seed 104) shared by all volumes, C = 4, m = 2, the 3x3x3 neighbourhood,
20 IFCM iterations per (volume, particle) (eps = 0), from each volume's FCM
initial state.  One step = normalise the six raw volumes and evaluate the
whole swarm (iteration invariants, 20 fused iterations per pair, the final
objective) with the batched launch.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Prints one JSON line: throughput in voxel-cluster-iterations per second,
the roofline of the dominant kernel (the fused step) from HIP events on the
stream it runs on, the same workload through one launch per particle, and
the FP64 oracle's rate on a bounded sample of the workload on this host.
"""
import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "voxel-cluster-iters/s + HBM GB/s; batched swarm vs plain per-particle on 1 GPU"
HBM_PEAK_GBPS = 8000.0
KERNEL = "k_ifcm_gather<4, m=2, TY=4, step>"
KERNEL_SOURCES = ("paper_2002_01981_amd/csrc/gather.h", "paper_2002_01981_amd/csrc/common.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_ifcm_gather_ragged6-swarm64_traffic.json")


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def copy_bandwidth(torch, mib=1024, reps=5):
    """GB/s of a plain device-to-device copy (read + write) of mib MiB: the
    bandwidth a streaming kernel reaches on this card, beside the peak."""
    n = mib * (1 << 20) // 4
    a = torch.ones(n, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def cpu_baseline(vol_raw, seconds, threads=None):
    """The FP64 oracle, as it stands, on one (volume, particle) pair of the
    workload: IFCM steps at (lambda, xi) = (0.3, 0.4) on `threads` host
    threads (default: the oracle's own, all cores) until about `seconds` of
    work (whole steps, at least two)."""
    import numpy as np
    import oracle
    before = oracle.get_threads()
    if threads:
        oracle.set_threads(threads)
    try:
        x = oracle.normalize(vol_raw)
        p = oracle.Params(C=4, m=2.0, eps=0.0, max_iter=1)
        c = np.array([0.125, 0.375, 0.625, 0.875])
        U = oracle.init_memberships(x, c, p)
        used = oracle.get_threads()
        t0 = time.perf_counter()
        U, c, _ = oracle.step(x, U, c, p, 0.3, 0.4)
        one = time.perf_counter() - t0
        iters = max(2, int(round(seconds / max(one, 1e-6))))
        for _ in range(iters - 1):
            U, c, _ = oracle.step(x, U, c, p, 0.3, 0.4)
        dt = time.perf_counter() - t0
    finally:
        oracle.set_threads(before)
    return x.size * 4 * iters / dt, dt, iters, used


def adjoint_leg(Context, Params):
    """Forward (K iterations) and backward (ifcm_backward) time on the brain
    phantom of the differentiation workload, and the workspace its own
    context holds."""
    import torch
    import synth
    ctx = Context(0)
    W = synth.WORKLOADS["adjoint-brain-K30"]
    raw, _ = synth.brain_shells(shape=W["shape"], seed=W["seed"], noise_frac=W["noise_frac"])
    x = ctx.pifcm_normalize(torch.from_numpy(raw).cuda())
    c0, U0, _ = ctx.pifcm_fcm_init(x, Params(C=4, m=2.0, eps=0.0, max_iter=10))
    K, s = W["K"], W["ckpt"]
    lam, xi = W["points"][0]
    pk = Params(C=4, m=2.0, eps=0.0, max_iter=K)
    Uo = torch.empty_like(U0)
    for _ in range(2):
        ctx.ifcm_solve(x, pk, lam, xi, c0, U_in=U0, U_out=Uo)
        ctx.ifcm_backward(x, Params(C=4, m=2.0), lam, xi, c0, U0, K, s)
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    reps = 5
    t0 = time.perf_counter()
    for _ in range(reps):
        ctx.ifcm_solve(x, pk, lam, xi, c0, U_in=U0, U_out=Uo)
    t1 = time.perf_counter()
    for _ in range(reps):
        g = ctx.ifcm_backward(x, Params(C=4, m=2.0), lam, xi, c0, U0, K, s)
    t2 = time.perf_counter()
    fwd, bwd = (t1 - t0) * 1e3 / reps, (t2 - t1) * 1e3 / reps
    ws = ctx.workspace_bytes()
    ctx.close()
    return dict(workload="adjoint-brain-K30", volume_zyx=list(W["shape"]), K=K, ckpt_every=s,
                point=[lam, xi], forward_ms=round(fwd, 3), backward_ms=round(bwd, 3),
                backward_over_forward=round(bwd / fwd, 3),
                workspace_bytes=ws, torch_allocated_bytes=int(base),
                J=g["J"], dJ_dlambda=g["dlam"], dJ_dxi=g["dxi"])


def ring_leg(Context, Params, vol_raw, dims):
    """The general neighbourhood of two Chebyshev rings (5x5x5, h = 1; the
    fused two-ring kernel) on the largest volume of the batch: 8 particles x
    5 iterations, batched, timed by the library's HIP events."""
    import numpy as np
    import torch
    import synth
    ctx = Context(0)
    x = ctx.pifcm_normalize(torch.from_numpy(vol_raw).cuda())
    c0, U0, _ = ctx.pifcm_fcm_init(x, Params(C=4, m=2.0, eps=0.0, max_iter=10))
    P, T = 8, 5
    parts = synth.uniform_particles(104, P)
    p = Params(C=4, m=2.0, V=2, h=1.0, eps=0.0, max_iter=T)
    ctx.swarm_evaluate([x], p, parts, c0[None], [U0])
    torch.cuda.synchronize()
    ctx.pifcm_get_timing(reset=True)
    ctx.pifcm_set_timing(True)
    ctx.swarm_evaluate([x], p, parts, c0[None], [U0])
    ctx.pifcm_set_timing(False)
    ms, launches = ctx.pifcm_get_timing(reset=True)
    ctx.close()
    n = int(np.prod(dims))
    per_launch = n * P * (8 * 4 + 4)
    avg = ms / max(launches, 1)
    return dict(kernel="k_ifcm_ring2<4, m=2, step>", neighbourhood="5x5x5, 2 rings, h=1",
                volume_zyx=list(dims), particles=P, iterations=T, avg_launch_us=round(avg * 1e3, 2),
                value=n * 4 * P / (avg * 1e-3), unit="voxel-cluster-iters/s",
                algorithmic_GBps=round(per_launch / (avg * 1e-3) / 1e9, 1))


def pso_leg(Context, Params, name, mode, noise=None):
    """One full particle swarm search (Algorithm 1 steps 2-9: FCM start,
    pifcm_pso with the workload's swarm, stop rule eps, max_iter) on a
    workload of the paper's shapes, after one untimed run of the same
    search.  Rates count the IFCM iterations the evaluations actually ran."""
    import numpy as np
    import torch
    import synth
    from paper_2002_01981_amd import PIFCM_SWARM_BATCHED
    W = synth.WORKLOADS[name]
    if W["kind"] == "nested":
        raw, _ = synth.nested_ellipsoids(shape=W["shape"], seed=W["seed"], sigma=W["sigma"])
    elif W["kind"] == "ellipsoids":
        raw, _ = synth.random_ellipsoids(shape=W["shape"], seed=W["seed"], sigma=W["sigma"])
    else:
        raw, _ = synth.brain_shells(shape=W["shape"], seed=W["seed"], noise_frac=noise)
    ps = W["pso"]
    st = synth.pso_streams(ps["seed"], ps["P"], ps["G"])
    p = Params(C=W["C"], m=W["m"], eps=W["eps"], max_iter=W["max_iter"])
    ctx = Context(0)
    x = ctx.pifcm_normalize(torch.from_numpy(raw).cuda())
    c0, U0, _ = ctx.pifcm_fcm_init(x, p)

    def run():
        return ctx.pifcm_pso([x], p, st, c0[None], [U0], w=ps["w"], c1=ps["c1"], c2=ps["c2"],
                             mode=mode)
    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sw = run()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.close()
    n = int(np.prod(W["shape"]))
    its = int(sw["iters_hist"].sum())
    out = dict(workload=name if noise is None else f"{name} noise {noise:.0%}",
               volume_zyx=list(W["shape"]), swarm=[ps["P"], ps["G"]], eps=W["eps"],
               max_iter=W["max_iter"], mode="batched" if mode == PIFCM_SWARM_BATCHED else "plain",
               seconds=round(dt, 4), evaluations=ps["P"] * ps["G"], iterations=its,
               value=n * W["C"] * its / dt, unit="voxel-cluster-iters/s",
               algorithmic_GBps=round(n * (8 * W["C"] + 4) * its / dt / 1e9, 1),
               best_pos=[round(float(v), 4) for v in sw["best_pos"][0]])
    return out


def cpu_search(name):
    """The FP64 oracle's whole swarm search (FCM start and pifcm_pso's
    schedule) on a small workload: seconds and the iterations it ran."""
    import oracle
    import synth
    W = synth.WORKLOADS[name]
    raw, _ = synth.nested_ellipsoids(shape=W["shape"], seed=W["seed"], sigma=W["sigma"])
    ps = W["pso"]
    st = synth.pso_streams(ps["seed"], ps["P"], ps["G"])
    xo = oracle.normalize(raw)
    po = oracle.Params(C=W["C"], m=W["m"], eps=W["eps"], max_iter=W["max_iter"])
    t0 = time.perf_counter()
    c0, U0, _ = oracle.fcm_init(xo, po)
    oracle.pso(xo, c0, U0, po, st, w=ps["w"], c1=ps["c1"], c2=ps["c2"])
    return dict(workload=name, seconds=round(time.perf_counter() - t0, 4),
                threads=oracle.get_threads())


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", choices=("batched", "plain"), default="batched")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-particle leg")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="length of the oracle's timed sample")
    ap.add_argument("--no-tune", action="store_true", help="keep the default tile shapes")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--no-ring", action="store_true", help="skip the general-neighbourhood leg")
    ap.add_argument("--no-pso", action="store_true",
                    help="skip the full swarm searches on the 32x32x8, 854x854x16 and brain volumes")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a device copy of MIB MiB a few times (counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: libpifcm has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2002_01981_amd import (PIFCM_SWARM_BATCHED, PIFCM_SWARM_PLAIN, Context,
                                      Params)

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} MiB x5")
        return

    W = synth.WORKLOADS["ragged6-swarm64"]
    T, P, C = W["iters"], W["particles"], W["C"]
    dims = synth.ragged_dims(W["seed"], W["count"])
    log(f"workload ragged6-swarm64: volumes {dims}, {P} particles, {T} iterations")
    vols = synth.ragged_batch(seed=W["seed"], count=W["count"], sigma=W["sigma"], dims=dims)
    raws = [torch.from_numpy(r).cuda() for r, _ in vols]
    xs = [torch.empty_like(r) for r in raws]
    ctx = Context(0)
    init_p = Params(C=C, m=W["m"], eps=1e-5, max_iter=50)
    c0s, U0s = [], []
    for r, x in zip(raws, xs):
        ctx.pifcm_normalize(r, out=x)
        c, U0, _ = ctx.pifcm_fcm_init(x, init_p)
        c0s.append(c)
        U0s.append(U0)
    c0s = np.stack(c0s)
    parts = synth.uniform_particles(W["particle_seed"], P)
    particles = np.ascontiguousarray(np.broadcast_to(parts, (len(xs), P, 2)))
    p = Params(C=C, m=W["m"], eps=W["eps"], max_iter=T)
    nvox = [int(np.prod(d)) for d in dims]
    work = sum(nvox) * C * T * P           # voxel-cluster-iterations per step
    mode = PIFCM_SWARM_BATCHED if args.mode == "batched" else PIFCM_SWARM_PLAIN

    def step(m=mode):
        for r, x in zip(raws, xs):
            ctx.pifcm_normalize(r, out=x)
        return ctx.swarm_evaluate(xs, p, particles, c0s, U0s, mode=m)

    tune = None
    if not args.no_tune:
        t0 = time.perf_counter()
        desc = ctx.pifcm_tune(xs, Params(C=C, m=W["m"], eps=0.0, max_iter=4), P)
        tune = dict(choice=desc, seconds=round(time.perf_counter() - t0, 3))
        log(f"tuned: {desc}")

    for i in range(args.warmup):
        out = step()
        log(f"warmup {i + 1}/{args.warmup} done")
    assert np.all(out["iters"] == T) if args.warmup else True
    torch.cuda.synchronize()
    ctx.pifcm_get_timing(reset=True)
    ctx.pifcm_set_timing(True)
    t0 = time.perf_counter()
    for i in range(args.steps):
        out = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.pifcm_set_timing(False)
    kern_ms, launches = ctx.pifcm_get_timing(reset=True)
    log(f"timed {args.steps} steps in {t1 - t0:.3f}s")
    assert np.all(out["iters"] == T) and np.all(np.isfinite(out["fitness"]))
    ms_step = (t1 - t0) * 1e3 / args.steps
    value = work / (ms_step * 1e-3)

    # Roofline of the fused step: algorithmic bytes per launch = per voxel and
    # particle, U^(t) read (4C B) + U^(t+1) written (4C B) + x read (4 B),
    # which a work item of pt particles reads once for all of them.
    pt = 1
    if tune is not None:
        m = re.search(r"particles_per_item=(\d+)", tune["choice"])
        pt = int(m.group(1)) if m else 1
    per_launch_bytes = round(sum(nvox) * P * (8 * C + 4 / pt))
    avg_launch_ms = kern_ms / max(launches, 1)
    achieved = per_launch_bytes / (avg_launch_ms * 1e-3) / 1e9
    traffic = valu = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_hash") == kernel_hash() and tr.get("workload") == "ragged6-swarm64":
            traffic = tr.get("hbm_bytes_per_launch")
            # VALU issue of the same kernel: rocprofv3 SQ_INSTS_VALU per launch
            # against 1024 SIMDs issuing one wave64 instruction per 4 cycles at
            # the engine clock the card holds under this benchmark.
            if tr.get("valu_instructions_per_launch") and tr.get("sclk_mhz_under_bench"):
                n = tr["valu_instructions_per_launch"]
                issue_ms = n / (1024 * tr["sclk_mhz_under_bench"] * 1e6 / 4) * 1e3
                valu = dict(instructions_per_launch=n,
                            per_voxel=round(n * 64 / (sum(nvox) * P), 1),
                            sclk_mhz=tr["sclk_mhz_under_bench"], issue_ms=round(issue_ms, 3),
                            issue_fraction=round(issue_ms / avg_launch_ms, 3))
    copy_gbps = copy_bandwidth(torch)
    log(f"plain device copy: {copy_gbps:.1f} GB/s")
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4), traffic=traffic,
                    kernel=KERNEL, avg_launch_us=round(avg_launch_ms * 1e3, 2),
                    launches=int(launches), algorithmic_bytes_per_launch=per_launch_bytes,
                    algorithmic_bytes_per_voxel_particle=8 * C + 4 / pt, particles_per_item=pt,
                    # measured HBM bytes (counters) over the live launch time,
                    # and what a plain 1 GiB copy reaches in the same run
                    hbm_GBps_measured=(round(traffic / (avg_launch_ms * 1e-3) / 1e9, 1)
                                       if traffic else None),
                    plain_copy_GBps=round(copy_gbps, 1),
                    valu_issue=valu)

    plain = None
    if not args.no_plain and mode == PIFCM_SWARM_BATCHED:
        # The plain mode runs one small launch per (volume, particle): it gets
        # a context of its own with the default decomposition, not the shape
        # tuned for the batched launch, and the batched launch is timed there
        # too, so that the comparison isolates batching.
        ctx_b = ctx
        ctx = Context(0)

        def timed(m):
            step(m)
            torch.cuda.synchronize()
            ctx.pifcm_get_timing(reset=True)
            ctx.pifcm_set_timing(True)
            ta = time.perf_counter()
            o = step(m)
            torch.cuda.synchronize()
            tb = time.perf_counter()
            ctx.pifcm_set_timing(False)
            kms, nl = ctx.pifcm_get_timing(reset=True)
            return o, (tb - ta) * 1e3, kms, nl

        outd, bd_ms, bd_k, bd_n = timed(PIFCM_SWARM_BATCHED)
        outp, pl_ms, pk_ms, pl = timed(PIFCM_SWARM_PLAIN)
        same = float(np.max(np.abs(outp["fitness"] / outd["fitness"] - 1.0)))
        tuned_diff = float(np.max(np.abs(outd["fitness"] / out["fitness"] - 1.0)))
        ctx.close()
        ctx = ctx_b
        plain = dict(decomposition="default (4 waves, each volume's default tile depth, 1 particle per item)",
                     ms_per_step=round(pl_ms, 3), value=work / (pl_ms * 1e-3),
                     launches_per_step=int(pl), avg_launch_us=round(pk_ms / max(pl, 1) * 1e3, 2),
                     batched_ms_per_step=round(bd_ms, 3),
                     batched_avg_launch_us=round(bd_k / max(bd_n, 1) * 1e3, 2),
                     batched_speedup=round(pl_ms / bd_ms, 3),
                     max_rel_fitness_diff_plain_vs_batched=same,
                     tuned_batched_speedup=round(pl_ms / ms_step, 3),
                     max_rel_fitness_diff_default_vs_tuned=tuned_diff)
        log(f"default decomposition: batched {bd_ms:.1f} ms/step, plain {pl_ms:.1f} ms/step, "
            f"max rel diff {same:.2e}")

    ring = None
    if not args.no_ring:
        b = int(np.argmax(nvox))
        ring = ring_leg(Context, Params, vols[b][0], dims[b])
        log(f"ring kernel: {ring['avg_launch_us']} us per launch")

    adjoint = None
    if not args.no_adjoint:
        adjoint = adjoint_leg(Context, Params)
        log(f"adjoint: forward {adjoint['forward_ms']} ms, backward {adjoint['backward_ms']} ms")

    pso = None
    if not args.no_pso:
        pso = [pso_leg(Context, Params, "nested-32x32x8", PIFCM_SWARM_BATCHED),
               pso_leg(Context, Params, "ellipsoids-854x854x16", PIFCM_SWARM_PLAIN)]
        pso += [pso_leg(Context, Params, "brain-181x217x181", PIFCM_SWARM_BATCHED, noise=f)
                for f in (0.03, 0.05, 0.09)]
        for leg in pso:
            log(f"swarm search {leg['workload']}: {leg['seconds']} s, {leg['iterations']} iterations, "
                f"{leg['value']:.3g} vci/s")

    cpu = None
    if not args.no_cpu_baseline:
        b = int(np.argmin(nvox))
        rate, dt, iters, cores = cpu_baseline(vols[b][0], args.cpu_seconds)
        rate1, dt1, iters1, _ = cpu_baseline(vols[b][0], args.cpu_seconds / 3, threads=1)
        cpu = dict(value=rate, unit="voxel-cluster-iters/s", cores=cores, kind="oracle",
                   sample=f"volume {b} of the batch ({dims[b][2]}x{dims[b][1]}x{dims[b][0]}), "
                          f"one particle (0.3, 0.4), {iters} IFCM steps in {dt:.1f} s",
                   host_cpus=os.cpu_count(),
                   one_thread=dict(value=rate1, steps=iters1, seconds=round(dt1, 2)),
                   full_search=cpu_search("nested-32x32x8"))
        log(f"cpu baseline: {rate:.3g} vci/s on {cores} threads in {dt:.1f}s; "
            f"{rate1:.3g} vci/s on 1 thread; {os.cpu_count()} host CPUs")

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "voxel-cluster-iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "ragged6-swarm64",
            "volumes_zyx": dims,
            "particles": P,
            "iterations": T,
            "C": C, "m": W["m"], "neighbourhood": "3x3x3",
            "mode": args.mode,
        },
        "hbm_GBps_algorithmic": round(achieved, 1),
        "roofline": roofline,
        "tune": tune,
        "plain": plain,
        "ring": ring,
        "adjoint": adjoint,
        "swarm_searches": pso,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
