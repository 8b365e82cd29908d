"""Benchmark of the fused grasp step on one MI355X.

One step = one pass of the whole hot path over every candidate: forward
kinematics, SDF gathers for M = 7 velocity tests, the PBD corrections and
losses, the hand-written adjoint, and Adam (a single fused launch). The
workload is the differentiable-step configuration: a 4-finger 22-DOF hand
with 2048 contacts, a 128^3 SDF of a union of ellipsoids, 4096 candidates,
synthetic inputs already resident in HBM.

Prints one JSON line: contact-evaluations per second (forward + backward),
the roofline of the step kernel and the FP64 oracle timed on the host, with
the other workloads beside them: the plain per-job form on the same
candidates, a Poisson stream of jobs through the serving loop, 16 uneven
jobs in one batched launch per step, K = 16 projection iterations on 65536
candidates (256^3 grid), and Phong signed-distance queries on mesh objects.
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


def live_fraction(ctx, h, sd, prm, q):
    """Fraction of the sample groups the forward passes of one step gather."""
    live, total = ctx.debug_forward_groups(h, sd, prm, q)
    return live / total if total else 0.0


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("step_kernels.hip", "device_common.h", "internal.h"):
        with open(os.path.join(ROOT, "paper_2306_08132_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when it is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    e = d.get(kernel, {}).get(workload)
    if not e or e.get("source_hash") != kernel_source_hash():
        return None
    return e.get("bytes_per_launch")


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
            "sample": f"{done} of {q.shape[0]} candidates, 1 step, forward + gradient, FP64, {dt:.1f} s"}


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


def serving_pool(S, device):
    """A few hands and objects for the served jobs (geometry is built once
    and stays resident; jobs draw from it)."""
    import numpy as np
    hands = {F: S.make_hand(F, 4 if F > 3 else 3, 2048, seed=200 + F) for F in (3, 4, 5)}
    objs = []
    for k, n in enumerate((64, 96, 128)):
        prims = S.make_object("mixed", seed=300 + k, n_range=(3, 6))
        objs.append(S.make_grid(prims, n, device=device))
    return hands, objs


def serving_run(ctx, S, n_jobs, rate, steps):
    """Poisson stream of grasp jobs through the serving loop: p50/p99 of
    submit-to-result latency and served contact-evaluations per second."""
    import numpy as np
    from paper_2306_08132_amd.api import StepParams
    hands, objs = serving_pool(S, "cuda:0")
    rh = {F: ctx.hand(h) for F, h in hands.items()}
    ro = [ctx.sdf(g) for g in objs]
    stream = S.make_job_stream(n_jobs, rate, seed=3, B_range=(256, 2048), steps=steps)
    rng = np.random.default_rng(3)
    jobs = []
    for j in stream:
        F = int(rng.integers(3, 6))
        g = int(rng.integers(0, len(objs)))
        q = S.make_candidates(hands[F], j["B"], seed=j["hand_seed"] % 100000,
                              shell_radius=objs[g].bound_radius + 0.06).astype(np.float32)
        jobs.append((j["arrival"], F, g, q))
    st0 = ctx.serve_stats()
    t0 = time.perf_counter()
    ids = []
    for arr, F, g, q in jobs:
        while time.perf_counter() - t0 < arr:
            time.sleep(0.0005)
        ids.append((ctx.submit(rh[F], ro[g], q, T=steps, prm=StepParams()), F, q.shape[0]))
    lat, status = [], []
    for jid, F, B in ids:
        while True:
            r = ctx.poll(jid, B, hands[F].n_dof)
            if r is not None:
                break
            time.sleep(0.001)
        lat.append(r["t_done"] - r["t_submit"])
        status.append(r["status"])
    wall = time.perf_counter() - t0
    st1 = ctx.serve_stats()
    lat = np.array(lat)
    evals = st1["contact_evals"] - st0["contact_evals"]
    return {"jobs": n_jobs, "rate_per_s": rate, "steps_per_job": steps, "candidates": "U[256, 2048]",
            "contacts": 2048, "grids": [g.n for g in objs], "p50_s": float(np.percentile(lat, 50)),
            "p99_s": float(np.percentile(lat, 99)), "jobs_per_s": n_jobs / wall,
            "contact_evals_per_s": evals / wall, "batched_steps": st1["steps"] - st0["steps"],
            "all_ok": bool(all(s_ == 0 for s_ in status))}


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
        for _ in range(args.steps // 5 + 3):
            b.step(bj, stream=stream)
        stream.synchronize()
        tb = (time.perf_counter() - t0) / (args.steps // 5 + 3)
    # the same jobs, one fused launch per job per step
    sj = [(sd, q.clone(), torch.zeros_like(q), torch.zeros_like(q)) for sd, q in jobs]
    for sd, q, m, v in sj:
        ctx.step_fused(h, sd, StepParams(r_dil=0.01), q, m, v, 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t in range(args.steps // 5 + 3):
        for sd, q, m, v in sj:
            ctx.step_fused(h, sd, StepParams(r_dil=0.01), q, m, v, t + 2)
    torch.cuda.synchronize()
    ts = (time.perf_counter() - t0) / (args.steps // 5 + 3)
    # the same jobs in the plain per-job form: unfused stages, HBM
    # intermediates, one set of launches per job per step
    ws = ctx.plain_workspace(h, jobs[0][0], StepParams(r_dil=0.01), max(q.shape[0] for _, q in jobs))
    pj = [(sd, q.clone(), torch.zeros_like(q), torch.zeros_like(q), torch.empty(q.shape[0], device=q.device))
          for sd, q in jobs]
    for sd, q, m, v, lp in pj:
        ctx.plain_step(h, sd, StepParams(r_dil=0.01), q, m, v, 1, ws, loss=lp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_plain = max(3, args.steps // 10)
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


def large_run(ctx, S, args):
    """K = 16 projection iterations, 65536 candidates, 8192 contacts, 256^3
    grid; pose checkpoints every 4 iterations with replay in the backward."""
    import torch
    from paper_2306_08132_amd.api import StepParams
    print("bench: K = 16 workload", file=sys.stderr, flush=True)
    hand, grid, q0 = S.config_workload("large", device="cuda:0")
    h, sd = ctx.hand(hand), ctx.sdf(grid)
    q = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
    m, v = torch.zeros_like(q), torch.zeros_like(q)
    live = live_fraction(ctx, h, sd, StepParams(K=16, ckpt_every=1, r_dil=0.01), q)
    abytes = algorithmic_bytes(q0.shape[0], hand.n_contacts, 16, hand.n_dof, grid.n, live)
    out = {"forward_live_fraction": live}
    for ck in (4, 1):
        prm = StepParams(K=16, ckpt_every=ck, r_dil=0.01)
        ctx.step_fused(h, sd, prm, q, m, v, 1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for t in range(2):
            ctx.step_fused(h, sd, prm, q, m, v, t + 2)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / 2
        evals = q.shape[0] * hand.n_contacts * M_SIMS * 16
        out[f"ckpt{ck}"] = {"s_per_iteration": dt, "contact_evals_per_s": evals / dt,
                            "roofline_frac": abytes / dt / (HBM_PEAK_GBS * 1e9)}
        print(f"bench: K = 16, checkpoints every {ck}: {dt:.3f} s per step", file=sys.stderr, flush=True)
    out["contact_evals_per_iteration"] = q.shape[0] * hand.n_contacts * M_SIMS * 16
    out["algorithmic_bytes_per_iteration"] = abytes
    return out


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
    n = max(3, args.steps // 5)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the plain per-job form")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream")
    ap.add_argument("--serve-jobs", type=int, default=24)
    ap.add_argument("--serve-rate", type=float, default=20.0, help="Poisson arrivals per second")
    ap.add_argument("--serve-steps", type=int, default=60, help="optimizer steps per served job")
    ap.add_argument("--no-batched", action="store_true", help="skip the 16 uneven jobs in one launch per step")
    ap.add_argument("--no-large", action="store_true", help="skip the K = 16 workload (65536 candidates)")
    ap.add_argument("--no-mesh", action="store_true", help="skip the mesh-object queries")
    ap.add_argument("--no-eval", action="store_true", help="skip the post-synthesis evaluation")
    ap.add_argument("--no-gs", action="store_true", help="skip the Gauss-Seidel projection")
    ap.add_argument("--tile", type=str, default=None,
                    help="launch tile 'waves_per_block,min_waves_per_simd' instead of tuning (profiled runs: "
                         "every step dispatch is then a timed shape)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (reads 1 GiB, writes 1 GiB) three times, "
                         "the reference that scales HBM counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the grasp step shards by "
              "candidates with no exchange inside a step, so one GPU's share is what it measures.",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2306_08132_amd import _lib
    from paper_2306_08132_amd import synth as S
    from paper_2306_08132_amd.api import Context, StepParams

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
    print("bench: building the workload", file=sys.stderr, flush=True)
    hand, grid, q0 = S.config_workload("diff", device="cuda:0")
    B, Nc, nd, K = q0.shape[0], hand.n_contacts, hand.n_dof, 1
    T_sched, r0 = 500, 0.01
    ctx = Context(0, arena_bytes=8 << 30)
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
        print(f"bench: tile {tile} (given)", file=sys.stderr, flush=True)
    else:
        print("bench: tuning the launch tile", file=sys.stderr, flush=True)
        tile, tile_ms = ctx.tune(h, sd, StepParams(K=K, r_dil=r0), q, reps=3)
        print(f"bench: tile {tile} at {tile_ms:.3f} ms", file=sys.stderr, flush=True)
    print("bench: warmup", file=sys.stderr, flush=True)
    for t in range(args.warmup):
        step(t)
    torch.cuda.synchronize()
    live = live_fraction(ctx, h, sd, StepParams(K=K, r_dil=r0 * (1.0 - args.warmup / (T_sched - 1))), q)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        ev[i][0].record(stream)
        step(args.warmup + i)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]
    avg_ms = float(np.mean(kern_ms))
    evals = B * Nc * M_SIMS * K
    value = evals * args.steps / wall
    abytes = algorithmic_bytes(B, Nc, K, nd, grid.n, live)
    achieved = abytes / (avg_ms * 1e-3) / 1e9
    workload = "diff-step"
    traffic = measured_traffic("k_step", workload)
    print(f"bench: fused step {avg_ms:.3f} ms/launch, {value:.3e} contact-evals/s", file=sys.stderr, flush=True)

    plain = None
    if not args.no_plain:
        # the plain per-job form on the same candidates: unfused stages, HBM
        # intermediates, one launch per stage per step, no graph
        print("bench: plain per-job form", file=sys.stderr, flush=True)
        qp = torch.tensor(q0, dtype=torch.float32, device="cuda:0")
        mp, vp = torch.zeros_like(qp), torch.zeros_like(qp)
        prm0 = StepParams(K=K, r_dil=r0)
        ws = ctx.plain_workspace(h, sd, prm0, B)
        n_plain = max(3, args.steps // 5)
        for t in range(2):
            ctx.plain_step(h, sd, prm0, qp, mp, vp, t + 1, ws, loss=loss, stream=stream)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        for t in range(n_plain):
            prm = StepParams(K=K, r_dil=r0 * (1.0 - min(t, T_sched - 1) / (T_sched - 1)))
            ctx.plain_step(h, sd, prm, qp, mp, vp, t + 3, ws, loss=loss, stream=stream)
        torch.cuda.synchronize()
        tp = (time.perf_counter() - tp0) / n_plain
        plain = {"value": evals / tp, "unit": "contact-evals/s", "ms_per_step": tp * 1e3, "steps": n_plain,
                 "workspace_bytes": ws.numel(), "fused_over_plain": value / (evals / tp)}
        del ws
        print(f"bench: plain {tp * 1e3:.3f} ms/step, fused/plain {value / (evals / tp):.2f}x", file=sys.stderr,
              flush=True)

    serving = None
    if not args.no_serving:
        print("bench: serving stream", file=sys.stderr, flush=True)
        serving = serving_run(ctx, S, n_jobs=args.serve_jobs, rate=args.serve_rate, steps=args.serve_steps)
    batched = None if args.no_batched else batched_run(ctx, S, args)
    large = None if args.no_large else large_run(ctx, S, args)
    mesh = None if args.no_mesh else mesh_run(ctx, S, args)
    evaluation = None if args.no_eval else eval_run(ctx, S, hand, grid, q0, h, sd, loss, args)
    gauss_seidel = None if args.no_gs else gs_run(ctx, S, hand, q0, h, sd, r0, avg_ms, args)

    cpu = None
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        cpu = cpu_baseline(hand, grid, q0, {"K": K, "r_dil": r0})
        cpu["evaluation"] = cpu_eval_baseline(hand, grid, q0, S)
        cpu["gauss_seidel"] = cpu_gs_baseline(hand, grid, q0, r0)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "contact-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload, "hand": "4 fingers x 4 joints, 22 DOF", "contacts": Nc,
                   "sdf": f"union of {len(grid.prims)} ellipsoids, {grid.n}^3 FP32", "candidates": B,
                   "tests_per_candidate": M_SIMS, "iterations": K, "contact_evals_per_step": evals,
                   "step": "fused forward + adjoint + Adam, one launch"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_step<K=1> (fused)", "avg_launch_ms": avg_ms,
                     "tile": {"waves_per_block": tile[0], "min_waves_per_simd": tile[1]},
                     "algorithmic_bytes_per_launch": abytes, "forward_live_fraction": live},
        "plain": plain,
        "serving": serving,
        "batched": batched,
        "large": large,
        "mesh": mesh,
        "evaluation": evaluation,
        "gauss_seidel": gauss_seidel,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
