"""Benchmark of the grasp step on one MI355X.

One step = one pass of the whole hot path over every candidate: forward
kinematics, SDF gathers for M = 7 velocity tests and K projection
iterations, the PBD corrections and losses, the hand-written adjoint, and
Adam, in one fused launch. The headline workload is the largest single-GPU
configuration: 65536 candidates of a 5-finger 26-DOF hand with 8192
contacts on a 256^3 SDF of a union of 8 ellipsoids/boxes, K = 16 projection
iterations with pose checkpoints every 4 (the backward recomputes FK and the
samples inside each segment). Inputs are synthetic and resident in HBM.

Prints one JSON line: the headline's contact-evaluations per second (forward
+ backward), its roofline (algorithmic bytes of the accounting below over the
kernel's launch time; the bound chosen from the committed rocprofv3 counters)
and the FP64 oracle timed on the host, with the other workloads beside them:
the differentiable-step workload (4096 candidates, 2048 contacts, 128^3)
fused and in the plain per-job form, 16 uneven jobs in one batched launch per
step, the serving stream (64 Poisson jobs at 20/s and a sub-saturation
stream, each also through the plain per-job form first in first out), the
Gauss-Seidel projection, the post-synthesis metrics and mesh queries.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "contact-evals/s fwd+bwd, fused vs plain, 1 MI355X; p50/p99 grasp-job latency"
HBM_PEAK_GBS = 8000.0
M_SIMS = 7


def algorithmic_bytes(B, Nc, K, n_dof, n, live):
    """Bytes one step must move at least once. Per contact evaluation: the 8
    FP32 corners (32 B) in the backward; in the forward the same 32 B only for
    samples in groups the block bound cannot clear (fraction `live` of the
    groups), plus the 4-byte bound itself, read once per contact when K = 1
    (the seven tests share it) and once per evaluation otherwise. Per
    candidate: each contact's link-local coordinates (forward and backward),
    q/m/v read and written plus dq. The grid and its block table once."""
    evals = B * Nc * M_SIMS * K
    bound = 4 * B * Nc if K == 1 else 4 * evals
    nb = -(-(n - 1) // 4)
    return int(32 * evals * (1.0 + live) + bound + 24 * B * Nc + 28 * B * n_dof + 4 * n ** 3 + 4 * nb ** 3)


def survey_bytes(B, Nc, K, n_dof, n):
    """Algorithmic bytes of one step in the plain accounting: per contact
    evaluation the 8 FP32 corners gathered once in the forward and once in
    the backward (64 B); per (candidate, contact) the link-local coordinates
    (24 B); per (candidate, DOF) q, m, v read and written plus dq (28 B); the
    grid once. No credit for samples the forward skips or for cache hits."""
    return int(64 * B * Nc * M_SIMS * K + 24 * B * Nc + 28 * B * n_dof + 4 * n ** 3)


CLOCK_HZ = 2.4e9      # MI355X peak engine clock
SIMDS = 256 * 4       # 256 CUs x 4 SIMDs; a wave64 FP32 VALU instruction takes 4 cycles on a 16-lane SIMD


def counter_fractions(kernel, workload, launch_s):
    """From the committed rocprofv3 counters of this kernel source: the VALU
    busy fraction (SQ_INSTS_VALU x 4 cycles over the launch's SIMD-cycles at
    2.4 GHz) and the DRAM fraction (copy-scaled FETCH_SIZE + WRITE_SIZE per
    launch over the launch time and 8 TB/s). None when missing or stale."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel, {}).get(workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    traffic = e["fetch_kib"] * 1024 * e["fetch_scale"] + e["write_kib"] * 1024 * e["write_scale"]
    valu = e["sq_insts_valu"] * 4.0 / (launch_s * CLOCK_HZ * SIMDS)
    dram = traffic / launch_s / (HBM_PEAK_GBS * 1e9)
    return {"valu_busy_frac": valu, "dram_frac": dram, "traffic_bytes_per_launch": traffic,
            "sq_insts_valu_per_launch": e["sq_insts_valu"], "profiled_launch_ms": e.get("avg_ms")}


VALU_PEAK_TFLOPS = 2.0 * SIMDS * 16 * CLOCK_HZ / 1e12  # 78.6: one FP32 FMA per lane per cycle (no packed FP32)


def roofline_block(sbytes, launch_s, cf):
    """The roofline of one kernel: bound by whichever of the VALU issue and
    the DRAM traffic the committed counters show busier. HBM: the
    algorithmic bytes (per-unit figures times units) per second against
    8 TB/s. ALU: the issued VALU instruction slots per second, each counted
    as one FMA (2 FLOP), against the 78.6 TFLOP/s of one FP32 FMA per lane
    per cycle; the algorithmic-bytes fraction is kept beside it."""
    hbm_achieved = sbytes / launch_s / 1e9
    out = {"algorithmic_bytes_per_launch": sbytes, "hbm_algorithmic_frac": hbm_achieved / HBM_PEAK_GBS,
           "counters": cf, "traffic": cf["traffic_bytes_per_launch"] if cf else None}
    if cf is not None and cf["valu_busy_frac"] > cf["dram_frac"]:
        ach = cf["sq_insts_valu_per_launch"] * 64 * 2 / launch_s / 1e12
        out.update({"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": ach / VALU_PEAK_TFLOPS,
                    "alu_accounting": "SQ_INSTS_VALU x 64 lanes x 2 FLOP per instruction slot"})
    else:
        out.update({"bound": "hbm", "achieved": hbm_achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": hbm_achieved / HBM_PEAK_GBS})
    return out


def live_fraction(ctx, h, sd, prm, q):
    """Fraction of the sample groups the forward passes of one step gather."""
    live, total = ctx.debug_forward_groups(h, sd, prm, q)
    return live / total if total else 0.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("step_kernels.hip", "device_common.h", "internal.h", "api.cpp"):
        with open(os.path.join(ROOT, "paper_2306_08132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def cpu_baseline(hand, grid, q, prm_kw, budget_s=12.0):
    """The FP64 oracle (forward + dual-number gradient), unmodified, on the
    host's cores over a bounded sample of the same workload's candidates."""
    import numpy as np
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    H, ob = O.Hand(hand.rounded()), O.Obj(grid)
    P = O.Params(**prm_kw)
    chunk = max(threads, 8)
    done, t0 = 0, time.perf_counter()
    while done < q.shape[0] and time.perf_counter() - t0 < budget_s:
        O.step(H, ob, P, q[done:done + chunk].astype(np.float32).astype(np.float64), grad=True,
               threads=threads)
        done += chunk
    dt = time.perf_counter() - t0
    evals = done * hand.n_contacts * M_SIMS * prm_kw.get("K", 1)
    return {"value": evals / dt, "unit": "contact-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of {q.shape[0]} candidates x 1 step ({hand.n_contacts} contacts, 7 tests, "
                      f"K = {prm_kw.get('K', 1)}), forward + dual-number gradient, FP64, {dt:.1f} s",
            "label": "FP64 correctness oracle, not a tuned CPU baseline"}


def cpu_eval_baseline(hand, grid, q, S, budget_s=4.0):
    """The oracle's post-synthesis metrics on the host's cores over a bounded
    sample of the evaluation workload's candidates."""
    import numpy as np
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    evp = S.config_eval_points("diff", hand)
    H, ob, E = O.Hand(hand.rounded()), O.Obj(grid), O.EvalPoints(evp.as_f32())
    chunk = max(threads, 8)
    done, t0 = 0, time.perf_counter()
    while done < q.shape[0] and time.perf_counter() - t0 < budget_s:
        O.evaluate(H, ob, q[done:done + chunk].astype(np.float32).astype(np.float64), E, EVAL_THRESHOLDS,
                   threads=threads)
        done += chunk
    dt = time.perf_counter() - t0
    n = len(evp.surface_link) + len(evp.volume_link)
    return {"value": done * n / dt, "unit": "candidate-samples/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of {q.shape[0]} candidates, FP64, {dt:.1f} s"}


def host_cpu():
    """The host's CPU model and core counts (the machine the oracle runs on)."""
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
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "usable_cores": usable,
            "omp_num_threads": os.environ.get("OMP_NUM_THREADS")}


def cpu_matrix(workloads, budget_s=2.5):
    """The FP64 oracle, unmodified, on every workload's per-candidate shape:
    forward only and forward + dual-number gradient, on all the host threads
    it may use and on one. Each entry runs whole candidates (one optimizer
    step each, at the workload's dilation) until budget_s has passed, at
    least one; candidates are independent, so the rate carries over to any
    count. Label: FP64 correctness oracle, not a tuned CPU baseline."""
    import numpy as np
    import oracle as O
    threads_all = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {}
    for name, (hand, grid, q, prm_kw) in workloads.items():
        H, ob, P = O.Hand(hand.rounded()), O.Obj(grid), O.Params(**prm_kw)
        per_cand = hand.n_contacts * M_SIMS * prm_kw.get("K", 1)
        for threads in (threads_all, 1):
            for grad in (False, True):
                chunk = threads
                done, t0 = 0, time.perf_counter()
                while done < q.shape[0] and (done == 0 or time.perf_counter() - t0 < budget_s):
                    qs = q[done % q.shape[0]:done % q.shape[0] + chunk]
                    O.step(H, ob, P, qs.astype(np.float32).astype(np.float64), grad=grad, threads=threads)
                    done += qs.shape[0]
                dt = time.perf_counter() - t0
                key = f"{name}/{'fwd+grad' if grad else 'fwd'}/{threads}t"
                out[key] = {"contact_evals_per_s": done * per_cand / dt, "candidates": done, "s": round(dt, 2)}
    return out


def c4_jobs(S, n_jobs, rate, steps, device):
    """The serving workload: a Poisson stream (mean `rate` jobs/s, stream seed
    3) of jobs, each with its own random hand (3, 4 or 5 fingers of 3 or 4
    joints, 1024, 2048 or 4096 contacts), its own random union of 3-8
    ellipsoids/boxes on a 64^3..256^3 grid, U[256, 8192] candidates on the
    approach shell, and `steps` optimizer steps."""
    import numpy as np
    stream = S.make_job_stream(n_jobs, rate, seed=3, B_range=(256, 8192), steps=steps)
    jobs = []
    for j in stream:
        hand = S.make_hand(j["fingers"], j["joints"], j["n_contacts"], seed=j["hand_seed"] % (1 << 30))
        prims = S.make_object("mixed", seed=j["obj_seed"] % (1 << 30), n_range=(3, 8))
        grid = S.make_grid(prims, j["res"], device=device)
        q = S.make_candidates(hand, j["B"], seed=j["hand_seed"] % 100003,
                              shell_radius=grid.bound_radius + 0.06).astype(np.float32)
        jobs.append(dict(j, hand=hand, grid=grid, q=q))
    return jobs


def _latency_stats(lat):
    import numpy as np
    lat = np.asarray(lat)
    return {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
            "mean_s": float(lat.mean()), "max_s": float(lat.max())}


def serve_stream(ctx, jobs, res, arrivals):
    """Submits each job at its arrival time (seconds from the start) to the
    serving loop and waits for all: submit-to-result latencies, jobs/s and
    served contact-evaluations/s over the stream's wall time."""
    from paper_2306_08132_amd.api import StepParams
    st0 = ctx.serve_stats()
    t0 = time.perf_counter()
    ids = []
    for j, arr in zip(jobs, arrivals):
        while time.perf_counter() - t0 < arr:
            time.sleep(0.0005)
        h, sd = res[id(j)]
        ids.append((ctx.submit(h, sd, j["q"], T=j["steps"], prm=StepParams()), j))
    lat, ok = [], True
    for jid, j in ids:
        while True:
            r = ctx.poll(jid, j["q"].shape[0], j["hand"].n_dof)
            if r is not None:
                break
            time.sleep(0.001)
        lat.append(r["t_done"] - r["t_submit"])
        ok = ok and r["status"] == 0
    wall = time.perf_counter() - t0
    st1 = ctx.serve_stats()
    evals = st1["contact_evals"] - st0["contact_evals"]
    return dict(_latency_stats(lat), jobs=len(jobs), wall_s=wall, jobs_per_s=len(jobs) / wall,
                contact_evals_per_s=evals / wall, batched_steps=st1["steps"] - st0["steps"], all_ok=bool(ok))


def plain_fifo(ctx, jobs, res, arrivals):
    """The same stream through the plain per-job form, first in first out: one
    job at a time (its T plain steps: unfused stage kernels with HBM
    intermediates, then Adam; the final forward at zero dilation), the next
    job starting when it has both arrived and the previous one has ended.
    Latency = end - arrival."""
    import numpy as np
    import torch
    from paper_2306_08132_amd.api import StepParams
    dev = "cuda:0"
    ws_bytes = 0
    for j in jobs:
        h, sd = res[id(j)]
        ws_bytes = max(ws_bytes, ctx.plain_workspace_bytes(h, sd, StepParams(), j["q"].shape[0]))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    t0 = time.perf_counter()
    lat, evals = [], 0
    for j, arr in zip(jobs, arrivals):
        while time.perf_counter() - t0 < arr:
            time.sleep(0.0005)
        h, sd = res[id(j)]
        q = torch.tensor(j["q"], device=dev)
        m, v = torch.zeros_like(q), torch.zeros_like(q)
        loss = torch.empty(q.shape[0], device=dev)
        T, r0 = j["steps"], 0.01
        for t in range(T):
            r = float(np.float32(np.float64(np.float32(r0)) * (1.0 - min(t, T - 1) / (T - 1))))
            ctx.plain_step(h, sd, StepParams(r_dil=r), q, m, v, t + 1, ws, loss=loss)
        ctx.step_fwd(h, sd, StepParams(r_dil=0.0), q, loss)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - arr)
        evals += q.shape[0] * j["hand"].n_contacts * M_SIMS * T
    wall = time.perf_counter() - t0
    del ws
    return dict(_latency_stats(lat), jobs=len(jobs), wall_s=wall, jobs_per_s=len(jobs) / wall,
                contact_evals_per_s=evals / wall)


def serving_run(ctx, S, args):
    """C4: 64 jobs at Poisson 20 jobs/s (an overload: the offered work is
    several times what one GPU does per second), then the same jobs at 0.7x
    the capacity the first stream measured; each stream also through the
    plain per-job form first in first out. Hands and grids are resident
    before the streams start (loading is not part of a job)."""
    import numpy as np
    print("bench: serving workload (building hands and grids)", file=sys.stderr, flush=True)
    jobs = c4_jobs(S, args.serve_jobs, args.serve_rate, args.serve_steps, "cuda:0")
    res = {}
    for j in jobs:
        res[id(j)] = (ctx.hand(j["hand"]), ctx.sdf(j["grid"]))
    arr = np.array([j["arrival"] for j in jobs])
    arr -= arr[0]
    offered = sum(j["q"].shape[0] * j["hand"].n_contacts * M_SIMS * j["steps"] for j in jobs) / max(arr[-1], 1e-9)
    out = {"jobs": len(jobs), "steps_per_job": args.serve_steps, "candidates": "U[256, 8192]",
           "contacts": sorted({j["hand"].n_contacts for j in jobs}), "grids": sorted({j["grid"].n for j in jobs}),
           "fingers": sorted({j["fingers"] for j in jobs}),
           "contact_evals_per_job_mean": float(np.mean([j["q"].shape[0] * j["hand"].n_contacts * M_SIMS *
                                                         j["steps"] for j in jobs]))}
    print("bench: serving stream at 20 jobs/s", file=sys.stderr, flush=True)
    over = serve_stream(ctx, jobs, res, arr)
    over.update(rate_per_s=args.serve_rate, offered_contact_evals_per_s=offered)
    cap = over["jobs_per_s"]
    rate2 = 0.7 * cap
    arr2 = arr * (args.serve_rate / rate2)
    print(f"bench: serving stream at 0.7 x capacity ({rate2:.2f} jobs/s)", file=sys.stderr, flush=True)
    sub = serve_stream(ctx, jobs, res, arr2)
    sub.update(rate_per_s=rate2)
    out["served"] = {"overload": over, "sub_saturation": sub}
    if not args.no_plain:
        print("bench: the same streams, plain per-job form, first in first out", file=sys.stderr, flush=True)
        p1 = plain_fifo(ctx, jobs, res, arr)
        p1.update(rate_per_s=args.serve_rate)
        p2 = plain_fifo(ctx, jobs, res, arr2)
        p2.update(rate_per_s=rate2)
        out["plain_fifo"] = {"overload": p1, "sub_saturation": p2}
        out["served_over_plain_throughput"] = over["contact_evals_per_s"] / p1["contact_evals_per_s"]
    for h, sd in res.values():
        sd.unload()
    print(f"bench: served p50/p99 {over['p50_s']:.2f}/{over['p99_s']:.2f} s at 20/s, "
          f"{sub['p50_s']:.2f}/{sub['p99_s']:.2f} s at {rate2:.2f}/s", file=sys.stderr, flush=True)
    return out


def batched_run(ctx, S, args):
    """16 uneven jobs (a 5-finger 26-DOF hand with 4096 contacts; unions of
    3-8 ellipsoids/boxes at 64..256^3; 256..4096 candidates each) advanced
    one step per launch, against the same jobs stepped one launch per job."""
    import numpy as np
    import torch
    from paper_2306_08132_amd.api import Batch, BatchJob, StepParams
    print("bench: batched jobs", file=sys.stderr, flush=True)
    rng = np.random.default_rng(2)
    hand = S.make_hand(5, 4, 4096, seed=2)
    h = ctx.hand(hand)
    jobs, evals, abytes = [], 0, 0
    for k in range(16):
        n = int(rng.choice([64, 96, 128, 192, 256]))
        grid = S.make_grid(S.make_object("mixed", seed=400 + k, n_range=(3, 8)), n, device="cuda:0")
        B = int(rng.integers(256, 4097))
        q = S.make_candidates(hand, B, seed=500 + k, shell_radius=grid.bound_radius + 0.06)
        sd = ctx.sdf(grid)
        qt = torch.tensor(q, dtype=torch.float32, device="cuda:0")
        jobs.append((sd, qt))
        evals += B * hand.n_contacts * M_SIMS
        abytes += algorithmic_bytes(B, hand.n_contacts, 1, hand.n_dof, n,
                                    live_fraction(ctx, h, sd, StepParams(r_dil=0.01), qt))
    cap = sum(q.shape[0] for _, q in jobs)
    stream = torch.cuda.Stream()
    bj = [BatchJob(h, sd, StepParams(), q.clone(), T=300) for sd, q in jobs]
    b = Batch(ctx, capacity=cap, max_jobs=16)
    with torch.cuda.stream(stream):
        for _ in range(2):
            b.step(bj, stream=stream)
        stream.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.diff_steps // 5 + 3):
            b.step(bj, stream=stream)
        stream.synchronize()
        tb = (time.perf_counter() - t0) / (args.diff_steps // 5 + 3)
    # the same jobs, one fused launch per job per step
    sj = [(sd, q.clone(), torch.zeros_like(q), torch.zeros_like(q)) for sd, q in jobs]
    for sd, q, m, v in sj:
        ctx.step_fused(h, sd, StepParams(r_dil=0.01), q, m, v, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.diff_steps // 5 + 3):
        for sd, q, m, v in sj:
            ctx.step_fused(h, sd, StepParams(r_dil=0.01), q, m, v, t + 2)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / (args.diff_steps // 5 + 3)
    # the same jobs in the plain per-job form: unfused stages, HBM
    # intermediates, one set of launches per job per step
    ws = ctx.plain_workspace(h, jobs[0][0], StepParams(r_dil=0.01), max(q.shape[0] for _, q in jobs))
    pj = [(sd, q.clone(), torch.zeros_like(q), torch.zeros_like(q), torch.empty(q.shape[0], device=q.device))
          for sd, q in jobs]
    for sd, q, m, v, lp in pj:
        ctx.plain_step(h, sd, StepParams(r_dil=0.01), q, m, v, 1, ws, loss=lp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_plain = max(3, args.diff_steps // 10)
    for t in range(n_plain):
        for sd, q, m, v, lp in pj:
            ctx.plain_step(h, sd, StepParams(r_dil=0.01), q, m, v, t + 2, ws, loss=lp)
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / n_plain
    del ws
    b.close()
    print(f"bench: batched {tb * 1e3:.2f} ms/step, per-job fused {ts * 1e3:.2f}, per-job plain {tp * 1e3:.2f}",
          file=sys.stderr, flush=True)
    return {"jobs": 16, "candidates": cap, "contact_evals_per_step": evals, "ms_per_step": tb * 1e3,
            "contact_evals_per_s": evals / tb, "per_job_launches_ms_per_step": ts * 1e3,
            "batched_over_per_job": ts / tb, "plain_per_job_ms_per_step": tp * 1e3, "batched_over_plain": tp / tb,
            "algorithmic_bytes_per_step": abytes, "roofline_frac": abytes / tb / (HBM_PEAK_GBS * 1e9)}


def large_headline(ctx, S, args):
    """The headline: K = 16 projection iterations on 65536 candidates, 8192
    contacts, 256^3 grid, pose checkpoints every 4 iterations with replay in
    the backward; W untimed steps, then exactly K timed steps, HIP events
    around each step on the launch stream (the candidate order kernel and
    the step kernel); the same with a checkpoint every iteration beside it."""
    import numpy as np
    import torch
    from paper_2306_08132_amd.api import StepParams
    print("bench: building the large workload", file=sys.stderr, flush=True)
    hand, grid, q0 = S.config_workload("large", device="cuda:0")
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    q = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
    m, v = torch.zeros_like(q), torch.zeros_like(q)
    loss = torch.empty(q.shape[0], device="cuda:0")
    stream = torch.cuda.current_stream()
    B, Nc, nd, K = q0.shape[0], hand.n_contacts, hand.n_dof, 16
    T, r0 = 200, 0.01
    tile = (1, 4)  # the step kernel's launch shape for this workload (tuning it costs seconds per shape)
    ctx.set_tile(h, sd, StepParams(K=K, ckpt_every=4), B, *tile)
    ctx.set_tile(h, sd, StepParams(K=K, ckpt_every=1), B, *tile)

    def step(t, ck):
        prm = StepParams(K=K, ckpt_every=ck, r_dil=r0 * (1.0 - min(t, T - 1) / (T - 1)))
        ctx.step_fused(h, sd, prm, q, m, v, t + 1, loss=loss, stream=stream)

    for t in range(args.warmup):
        step(t, 4)
    torch.cuda.synchronize()
    t_live = args.warmup
    live = live_fraction(ctx, h, sd, StepParams(K=K, ckpt_every=1, r_dil=r0 * (1.0 - t_live / (T - 1))), q)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step(args.warmup + i, 4)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    launch_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    # the same steps with a checkpoint every iteration (no replay), for comparison
    ck1 = []
    for i in range(2):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        step(args.warmup + args.steps + i, 1)
        b.record(stream)
        ck1.append((a, b))
    torch.cuda.synchronize()
    ck1_ms = float(np.mean([a.elapsed_time(b) for a, b in ck1]))
    evals = B * Nc * M_SIMS * K
    print(f"bench: large workload {launch_ms:.1f} ms per step (checkpoints every 4), {ck1_ms:.1f} ms (every "
          f"iteration), {evals * args.steps / wall:.3e} contact-evals/s", file=sys.stderr, flush=True)
    res = {"hand": hand, "grid": grid, "q0": q0, "B": B, "Nc": Nc, "n_dof": nd, "K": K, "tile": tile,
           "wall_s": wall, "launch_ms": launch_ms, "ckpt1_launch_ms": ck1_ms, "evals": evals, "live": live,
           "schedule": {"r0_m": r0, "T": T, "timed_steps": [args.warmup, args.warmup + args.steps - 1]}}
    sd_h = (h, sd)
    return res, sd_h


def mesh_run(ctx, S, args):
    """The mesh object of Sec. III-B: Phong signed-distance queries through the
    bounding-volume hierarchy (one lane per point) on ellipsoid meshes of
    5120 and 81920 faces, and a 128^3 grid filled from a mesh on the device."""
    import numpy as np
    import torch
    print("bench: mesh objects", file=sys.stderr, flush=True)
    out = {}
    rng = np.random.default_rng(11)
    for sub in (4, 6):
        m = S.mesh_ellipsoid([0.04, 0.025, 0.035], subdivisions=sub)
        gm = ctx.mesh(m, 0.75)
        R = m.bound_radius()
        r = torch.as_tensor(rng.uniform(-1.5 * R, 1.5 * R, size=(1 << 20, 3)).astype(np.float32), device="cuda:0")
        gm.sample(r)
        torch.cuda.synchronize()
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            gm.sample(r)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        out[f"faces_{m.faces.shape[0]}"] = {"queries_per_s": r.shape[0] / dt, "ms_per_million": dt * 1e3 / (r.shape[0] / 1e6)}
        if sub == 4:
            n = 128
            t0 = time.perf_counter()
            sd = gm.grid(n, (-0.06, -0.06, -0.06), 0.12 / (n - 1))
            torch.cuda.synchronize()
            out["grid_128_from_5120_faces_s"] = time.perf_counter() - t0
            sd.unload()
        gm.unload()
    print(f"bench: mesh queries {out}", file=sys.stderr, flush=True)
    return out


def mesh_step_run(ctx, S, hand, q0, h, sd, args):
    """The grasp step with the object as a mesh queried at every sample
    (Sec. III-B's Phong distance in Sec. III-C's step, forward and adjoint
    through the closest and Phong points), beside the grid step, on the
    differentiable-step hand (2048 contacts) and its 4096 candidates against
    a 5120-face ellipsoid mesh (Phong alpha 0.75), r_dil = 5 mm, K = 1."""
    import numpy as np
    import torch
    from paper_2306_08132_amd.api import StepParams
    print("bench: grasp step on a mesh object", file=sys.stderr, flush=True)
    B, Nc = q0.shape[0], hand.n_contacts
    gm = ctx.mesh(S.mesh_ellipsoid([0.05, 0.035, 0.04], subdivisions=4), 0.75)
    Im = float(np.float32(0.4 * 0.04 ** 2))
    prm = StepParams(K=1, r_dil=0.005)
    stream = torch.cuda.current_stream()
    res = {"candidates": B, "contacts": Nc, "faces": 5120, "phong_alpha": 0.75, "r_dil_m": 0.005, "iterations": 1}
    for name in ("mesh", "grid"):
        q = torch.tensor(q0[:B], dtype=torch.float32, device="cuda:0")
        m, v = torch.zeros_like(q), torch.zeros_like(q)
        loss = torch.empty(B, device="cuda:0")

        def step(t):
            if name == "mesh":
                ctx.step_fused_mesh(h, gm, prm, q, m, v, t + 1, inertia_over_mass=Im, loss=loss, stream=stream)
            else:
                ctx.step_fused(h, sd, prm, q, m, v, t + 1, loss=loss, stream=stream)

        step(0)
        torch.cuda.synchronize()
        n = 3 if name == "mesh" else 20
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
        for i in range(n):
            ev[i][0].record(stream)
            step(1 + i)
            ev[i][1].record(stream)
        torch.cuda.synchronize()
        ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
        res[name] = {"ms_per_step": ms, "contact_evals_per_s": B * Nc * M_SIMS / (ms * 1e-3), "steps": n}
    res["mesh_over_grid_time"] = res["mesh"]["ms_per_step"] / res["grid"]["ms_per_step"]
    gm.unload()
    print(f"bench: mesh step {res['mesh']['ms_per_step']:.2f} ms, grid step {res['grid']['ms_per_step']:.3f} ms "
          f"on {B} candidates", file=sys.stderr, flush=True)
    return res


def gs_run(ctx, S, hand, q0, h, sd, r0, avg_ms, args):
    """The Gauss-Seidel projection (Sec. III-C, constraints swept one after
    another) as a fused step with Adam on the same 4096 candidates, 2048
    contacts and 128^3 grid, with the same dilation schedule."""
    import numpy as np
    import torch
    from paper_2306_08132_amd.api import StepParams
    print("bench: Gauss-Seidel projection", file=sys.stderr, flush=True)
    q = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
    m, v = torch.zeros_like(q), torch.zeros_like(q)
    loss = torch.empty(q.shape[0], device="cuda:0")
    stream = torch.cuda.current_stream()
    T = 500

    def step(t):
        prm = StepParams(K=1, projection=1, r_dil=r0 * (1.0 - min(t, T - 1) / (T - 1)))
        ctx.step_fused(h, sd, prm, q, m, v, t + 1, loss=loss, stream=stream)

    # forward only (loss), at the initial candidates: its share of the step
    fwd_prm = StepParams(K=1, projection=1, r_dil=r0)
    ctx.step_fwd(h, sd, fwd_prm, q, loss, stream=stream)
    fe = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(3)]
    for a, b in fe:
        a.record(stream)
        ctx.step_fwd(h, sd, fwd_prm, q, loss, stream=stream)
        b.record(stream)
    for t in range(2):
        step(t)
    n = max(3, args.diff_steps // 5)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for i, (a, b) in enumerate(evs):
        a.record(stream)
        step(2 + i)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    fwd_ms = float(np.mean([a.elapsed_time(b) for a, b in fe]))
    evals = q.shape[0] * hand.n_contacts * 7
    res = {"kernel": "k_gs_step", "ms_per_step": ms, "forward_only_ms": fwd_ms, "contact_evals_per_s": evals / (ms * 1e-3), "steps": n,
           "averaged_ms_per_step": avg_ms, "gs_over_averaged_time": ms / avg_ms,
           "final_loss_mean": float(loss.mean())}
    print(f"bench: Gauss-Seidel {ms:.3f} ms/step ({ms / avg_ms:.1f}x the averaged step)", file=sys.stderr,
          flush=True)
    return res


def cpu_gs_baseline(hand, grid, q, r0, budget_s=4.0):
    """The oracle's Gauss-Seidel step (forward + dual gradient) over a bounded
    sample of the same candidates."""
    import numpy as np
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    H, ob, P = O.Hand(hand.rounded()), O.Obj(grid), O.Params(K=1, r_dil=r0, projection=1)
    chunk = max(threads, 8)
    done, t0 = 0, time.perf_counter()
    while done < q.shape[0] and time.perf_counter() - t0 < budget_s:
        O.step(H, ob, P, q[done:done + chunk].astype(np.float32).astype(np.float64), grad=True, threads=threads)
        done += chunk
    dt = time.perf_counter() - t0
    return {"value": done * hand.n_contacts * 7 / dt, "unit": "contact-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of {q.shape[0]} candidates, 1 Gauss-Seidel step, forward + gradient, FP64, {dt:.1f} s"}


def cpu_mesh_step_baseline(hand, q, S, budget_s=10.0):
    """The oracle's grasp step on the mesh object of the mesh-step leg
    (forward + dual gradient, every face tested per sample in FP64) over a
    bounded sample of the same candidates, one candidate per thread."""
    import numpy as np
    import oracle as O
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    m = S.mesh_ellipsoid([0.05, 0.035, 0.04], subdivisions=4)
    f32 = lambda a: np.asarray(a, np.float64).astype(np.float32).astype(np.float64)
    M = O.Mesh(f32(m.vertices), m.faces, f32(m.normals), float(np.float32(0.75)))
    ob = O.Obj(mesh=M, inertia_over_mass=float(np.float32(0.4 * 0.04 ** 2)))
    H, P = O.Hand(hand.rounded()), O.Params(K=1, r_dil=float(np.float32(0.005)))
    done, t0 = 0, time.perf_counter()
    while done < q.shape[0] and time.perf_counter() - t0 < budget_s:
        O.step(H, ob, P, f32(q[done:done + threads]), grad=True, threads=threads)
        done += threads
    dt = time.perf_counter() - t0
    return {"value": done * hand.n_contacts * 7 / dt, "unit": "contact-evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{done} of {q.shape[0]} candidates, 1 step on the 5120-face mesh, forward + gradient, FP64, "
                      f"{dt:.1f} s"}


EVAL_THRESHOLDS = (0.002, 0.005, 0.009)  # contact thresholds of the paper's metric figures (m)


def eval_run(ctx, S, hand, grid, q0, h, sd, key, args):
    """Post-synthesis evaluation (Sec. V-A metrics) of the 4096 candidates of
    the differentiable-step workload at their synthetic poses: contact area at
    2/5/9 mm and intersection volume from 4096 surface + 4096 volume samples
    per hand, then the top-10 by a key (the final loss) and their means."""
    import numpy as np
    import torch
    print("bench: post-synthesis evaluation", file=sys.stderr, flush=True)
    evp = S.config_eval_points("diff", hand)
    gev = ctx.eval_points(h, evp)
    q = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
    stream = torch.cuda.current_stream()
    out = torch.empty((q.shape[0], len(EVAL_THRESHOLDS) + 1), device="cuda:0")
    for _ in range(3):
        ctx.evaluate(gev, sd, q, EVAL_THRESHOLDS, out=out, stream=stream)
    reps = 20
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for a, b in evs:
        a.record(stream)
        ctx.evaluate(gev, sd, q, EVAL_THRESHOLDS, out=out, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    sel = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        top, mean = ctx.select_top(key, 10, False, out, stream=stream)
        b.record(stream)
        sel.append((a, b))
    torch.cuda.synchronize()
    top_ms = float(np.mean([a.elapsed_time(b) for a, b in sel]))
    n = len(evp.surface_link) + len(evp.volume_link)
    # the same samples against a mesh object (5120-face ellipsoid, Phong alpha 0.75) instead of the grid
    gm = ctx.mesh(S.mesh_ellipsoid([0.05, 0.035, 0.04], subdivisions=4), 0.75)
    mout = ctx.evaluate_mesh(gev, gm, q, EVAL_THRESHOLDS)
    me = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(5)]
    for a, b in me:
        a.record(stream)
        ctx.evaluate_mesh(gev, gm, q, EVAL_THRESHOLDS, out=mout, stream=stream)
        b.record(stream)
    torch.cuda.synchronize()
    mesh_ms = float(np.mean([a.elapsed_time(b) for a, b in me]))
    gm.unload()
    res = {"candidates": q.shape[0], "surface_samples": len(evp.surface_link), "volume_samples": len(evp.volume_link),
           "mesh_5120_faces_ms_per_launch": mesh_ms,
           "thresholds_m": list(EVAL_THRESHOLDS), "kernel": "k_evaluate", "avg_launch_ms": ms,
           "candidate_samples_per_s": q.shape[0] * n / (ms * 1e-3), "top10_ms": top_ms,
           "top10_mean_ca_cm2": [float(x) * 1e4 for x in mean[:3].cpu()], "top10_mean_iv_cm3": float(mean[3]) * 1e6,
           "all_mean_ca5_cm2": float(out[:, 1].mean()) * 1e4, "all_mean_iv_cm3": float(out[:, 3].mean()) * 1e6}
    gev.unload()
    print(f"bench: evaluation {ms:.3f} ms/launch ({res['candidate_samples_per_s']:.3e} candidate-samples/s), "
          f"top-10 {top_ms:.3f} ms, against a 5120-face mesh {mesh_ms:.2f} ms", file=sys.stderr, flush=True)
    return res


def diff_run(ctx, S, args):
    """The differentiable-step workload (4-finger 22-DOF hand, 2048 contacts,
    128^3 union of ellipsoids, 4096 candidates, K = 1): fused steps along the
    dilation schedule from r0 = 1 cm over T = 500 steps, 10 untimed then 50
    timed, and the plain per-job form on the same candidates."""
    import numpy as np
    import torch
    from paper_2306_08132_amd.api import StepParams
    print("bench: building the differentiable-step workload", file=sys.stderr, flush=True)
    hand, grid, q0 = S.config_workload("diff", device="cuda:0")
    B, Nc, nd, K = q0.shape[0], hand.n_contacts, hand.n_dof, 1
    T_sched, r0 = 500, 0.01
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    stream = torch.cuda.current_stream()
    q = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
    m, v = torch.zeros_like(q), torch.zeros_like(q)
    loss = torch.empty(B, device="cuda:0")

    def step(t):
        prm = StepParams(K=K, r_dil=r0 * (1.0 - min(t, T_sched - 1) / (T_sched - 1)))
        ctx.step_fused(h, sd, prm, q, m, v, t + 1, loss=loss, stream=stream)

    if args.tile:
        tile = tuple(int(x) for x in args.tile.split(","))
        ctx.set_tile(h, sd, StepParams(K=K, r_dil=r0), B, tile[0], tile[1])
    else:
        tile, _ = ctx.tune(h, sd, StepParams(K=K, r_dil=r0), q, reps=3)
    warm, steps = args.diff_warmup, args.diff_steps
    for t in range(warm):
        step(t)
    torch.cuda.synchronize()
    live = live_fraction(ctx, h, sd, StepParams(K=K, r_dil=r0 * (1.0 - warm / (T_sched - 1))), q)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        step(warm + i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    avg_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    evals = B * Nc * M_SIMS * K
    value = evals * steps / wall
    sbytes = survey_bytes(B, Nc, K, nd, grid.n)
    cbytes = algorithmic_bytes(B, Nc, K, nd, grid.n, live)
    cf = counter_fractions("k_step", "diff-step", avg_ms * 1e-3)
    out = {"workload": "diff-step", "hand": "4 fingers x 4 joints, 22 DOF", "contacts": Nc, "candidates": B,
           "sdf": f"union of {len(grid.prims)} ellipsoids, {grid.n}^3 FP32", "iterations": K,
           "schedule": {"r0_m": r0, "T": T_sched, "timed_steps": [warm, warm + steps - 1]},
           "steps": steps, "warmup": warm, "ms_per_step": wall * 1e3 / steps, "avg_launch_ms": avg_ms,
           "contact_evals_per_s": value, "tile": list(tile),
           "roofline": roofline_block(sbytes, avg_ms * 1e-3, cf)}
    out["roofline"].update({"culled_accounting_bytes_per_launch": cbytes,
                            "culled_accounting_frac": cbytes / (avg_ms * 1e-3) / (HBM_PEAK_GBS * 1e9),
                            "forward_live_fraction": live})
    print(f"bench: diff-step fused {avg_ms:.3f} ms/launch, {value:.3e} contact-evals/s", file=sys.stderr,
          flush=True)
    if not args.no_plain:
        # the plain per-job form on the same candidates: unfused stages, HBM
        # intermediates, one launch per stage per step, no graph
        qp = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
        mp, vp = torch.zeros_like(qp), torch.zeros_like(qp)
        prm0 = StepParams(K=K, r_dil=r0)
        ws = ctx.plain_workspace(h, sd, prm0, B)
        n_plain = max(3, steps // 5)
        for t in range(2):
            ctx.plain_step(h, sd, prm0, qp, mp, vp, t + 1, ws, loss=loss, stream=stream)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for t in range(n_plain):
            prm = StepParams(K=K, r_dil=r0 * (1.0 - min(t + 2, T_sched - 1) / (T_sched - 1)))
            ctx.plain_step(h, sd, prm, qp, mp, vp, t + 3, ws, loss=loss, stream=stream)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - tp0) / n_plain
        out["plain"] = {"contact_evals_per_s": evals / tp, "ms_per_step": tp * 1e3, "steps": n_plain,
                        "workspace_bytes": ws.numel()}
        out["fused_over_plain"] = value / (evals / tp)
        del ws
        print(f"bench: plain {tp * 1e3:.3f} ms/step, fused/plain {out['fused_over_plain']:.2f}x", file=sys.stderr,
              flush=True)
    return out, (hand, grid, q0, h, sd, loss, avg_ms)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5, help="timed steps of the headline (large) workload")
    ap.add_argument("--warmup", type=int, default=2, help="untimed steps of the headline workload")
    ap.add_argument("--diff-steps", type=int, default=50, help="timed steps of the differentiable-step workload")
    ap.add_argument("--diff-warmup", type=int, default=10)
    ap.add_argument("--headline-only", action="store_true", help="only the headline workload (profiling runs)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baselines")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-job forms")
    ap.add_argument("--no-diff", action="store_true", help="skip the differentiable-step workload")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving streams")
    ap.add_argument("--serve-jobs", type=int, default=64)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-steps", type=int, default=300, help="optimizer steps per served job")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16 uneven jobs in one launch per step")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh-object queries")
    ap.add_argument("--no-eval", action="store_true", help="skip the post-synthesis evaluation")
    ap.add_argument("--no-gs", action="store_true", help="skip the Gauss-Seidel projection")
    ap.add_argument("--tile", type=str, default=None,
                    help="launch tile 'waves_per_block,min_waves_per_simd' of the differentiable-step workload "
                         "instead of tuning")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reads 1 GiB, writes 1 GiB) three times, "
                         "the reference that scales HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the grasp step shards by "
              "candidates with no exchange inside a step, so one GPU's share is what it measures.",
              file=sys.stderr)
        sys.exit(2)
    if args.headline_only:
        args.no_cpu = args.no_plain = args.no_diff = args.no_serving = args.no_batched = True
        args.no_mesh = args.no_eval = args.no_gs = True

    import torch
    from paper_2306_08132_amd import _lib
    from paper_2306_08132_amd import synth as S
    from paper_2306_08132_amd.api import Context

    if not os.path.exists(_lib.LIB_PATH):
        from __graft_entry__ import build
        build()
    if args.calibrate_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    ctx = Context(0, arena_bytes=24 << 30)

    # ---- the headline: the large workload ----
    L, (hL, sdL) = large_headline(ctx, S, args)
    value = L["evals"] * args.steps / L["wall_s"]
    launch_s = L["launch_ms"] * 1e-3
    sbytes = survey_bytes(L["B"], L["Nc"], L["K"], L["n_dof"], L["grid"].n)
    cbytes = algorithmic_bytes(L["B"], L["Nc"], L["K"], L["n_dof"], L["grid"].n, L["live"])
    cf = counter_fractions("k_step", "large-k16", launch_s)
    roofline = roofline_block(sbytes, launch_s, cf)
    roofline.update({
        "kernel": "k_step<K=16> (fused, pose checkpoints every 4)", "avg_launch_ms": L["launch_ms"],
        "accounting": "64 B per contact evaluation (8 FP32 corners in the forward and in the backward) "
                      "+ 24 B per (candidate, contact) + 28 B per (candidate, DOF) + the grid once",
        "culled_accounting_bytes_per_launch": cbytes,
        "culled_accounting_frac": cbytes / launch_s / (HBM_PEAK_GBS * 1e9),
        "forward_live_fraction": L["live"],
        "tile": {"waves_per_block": L["tile"][0], "min_waves_per_simd": L["tile"][1]},
        "checkpoint_every_iteration_ms": L["ckpt1_launch_ms"]})
    cpu = None
    if not args.no_cpu:
        print("bench: oracle CPU baseline (large workload)", file=sys.stderr, flush=True)
        cpu = cpu_baseline(L["hand"], L["grid"], L["q0"], {"K": 16, "r_dil": 0.01})
        cpu["host"] = host_cpu()

    # ---- the other workloads ----
    diff = None
    if not args.no_diff:
        diff, (hand2, grid2, q2, h2, sd2, loss2, avg2) = diff_run(ctx, S, args)
    batched = None if args.no_batched else batched_run(ctx, S, args)
    serving = None if args.no_serving else serving_run(ctx, S, args)
    mesh = None if args.no_mesh else mesh_run(ctx, S, args)
    evaluation = gauss_seidel = None
    if diff is not None:
        evaluation = None if args.no_eval else eval_run(ctx, S, hand2, grid2, q2, h2, sd2, loss2, args)
        gauss_seidel = None if args.no_gs else gs_run(ctx, S, hand2, q2, h2, sd2, 0.01, avg2, args)
        if mesh is not None:
            mesh["step"] = mesh_step_run(ctx, S, hand2, q2, h2, sd2, args)
    if cpu is not None:
        print("bench: oracle CPU matrix", file=sys.stderr, flush=True)
        work = {"large": (L["hand"], L["grid"], L["q0"], {"K": 16, "r_dil": 0.01})}
        h1, g1, q1 = S.config_workload("tiny")
        work["tiny"] = (h1, g1, q1, {"K": 1, "r_dil": 0.01})
        if diff is not None:
            work["diff-step"] = (hand2, grid2, q2, {"K": 1, "r_dil": 0.01})
            hb = S.make_hand(5, 4, 4096, seed=2)
            gb = S.make_grid(S.make_object("mixed", seed=400, n_range=(3, 8)), 128, device="cuda:0")
            qb = S.make_candidates(hb, 64, seed=500, shell_radius=gb.bound_radius + 0.06)
            work["batched-job"] = (hb, gb, qb, {"K": 1, "r_dil": 0.01})
        cpu["matrix"] = cpu_matrix(work)
        if diff is not None:
            cpu["evaluation"] = cpu_eval_baseline(hand2, grid2, q2, S)
            cpu["gauss_seidel"] = cpu_gs_baseline(hand2, grid2, q2, 0.01)
            if mesh is not None:
                cpu["mesh_step"] = cpu_mesh_step_baseline(hand2, q2, S)

    hand = L["hand"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "contact-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": L["wall_s"] * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "large", "hand": "5 fingers x 4 joints, 26 DOF", "contacts": L["Nc"],
                   "sdf": f"union of {len(L['grid'].prims)} ellipsoids/boxes, {L['grid'].n}^3 FP32",
                   "candidates": L["B"], "tests_per_candidate": M_SIMS, "iterations": L["K"],
                   "checkpoint_every": 4, "contact_evals_per_step": L["evals"],
                   "schedule": L["schedule"],
                   "step": "fused forward + adjoint (segments recomputed) + Adam, one launch"},
        "roofline": roofline,
        "diff_step": diff,
        "batched": batched,
        "serving": serving,
        "mesh": mesh,
        "evaluation": evaluation,
        "gauss_seidel": gauss_seidel,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
