"""Throughput of the autotuned leapfrog star-stencil step on one MI355X.

Workload: 512^3 layered velocity model (20 layers, 1500-4500 m/s, 2% noise,
seed 13108232), h = 10 m, Courant 0.4, 8th order (R = 4), FP32, centred 15 Hz
Ricker source, the time loop's steps W..W+K-1 timed after W warm-up steps.
A "step" is one leapfrog update of all 512^3 points (one sweep launch with the
source fused). Before the timed region the blocksize search picks the tile
(its cost is reported, not timed); the plain-tiling kernel and the built-in
default tile are timed on the same buffers for comparison.

Prints one JSON line (rank 0). The roofline entry uses 16 algorithmic bytes
per point update (read u^n, u^{n-1}, kappa; write u^{n+1}) divided by the
sweep's average duration from HIP events on the launch stream.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 16
METRIC = "Gpoint-updates/s + % of HBM roofline, 512^3 8th-order FP32 vs plain tiling"


def sweep_source_hash() -> str:
    """Hash of the sources that define the sweep kernels (one- and two-step)
    and their instantiations: counter summaries taken on other code do not
    apply."""
    h = hashlib.sha256()
    for f in ("internal.h", "sweep.hpp", "sweep2.hpp", "kernels_radius.hip"):
        with open(os.path.join(ROOT, "paper_1310_8232_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def load_traffic(tile: dict, n_points: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source and the chosen tile."""
    path = os.path.join(ROOT, "profiles", "sweep_512_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != sweep_source_hash():
        return None
    key = "{kind}-{bx}-{by}-{ry}-{dz}-{vw}-{xcd}-{pf}".format(**tile)
    entry = rec.get("tiles", {}).get(key)
    if not entry:
        return None
    return entry.get("hbm_bytes_per_launch")


def time_steps(prop, a, b, nsteps, it0, src, stream, temporal=1, spare=None, nseg=1):
    """Time nsteps steps with HIP events on `stream`; with nseg > 1 the steps
    run in nseg equal segments with an event between segments (no host
    synchronisation inside the timed region). Returns (total ms, a, b) or,
    with nseg > 1, (total ms, a, b, per-segment ms)."""
    import torch
    if nseg < 1 or nsteps % (nseg * temporal):
        nseg = 1
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(nseg + 1)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    per = nsteps // nseg
    for k in range(nseg):
        a, b = prop.run(a, b, per, src, it0=it0 + k * per, stream=stream, temporal=temporal, spare=spare)
        ev[k + 1].record(stream)
    torch.cuda.synchronize()
    total = ev[0].elapsed_time(ev[nseg])
    if nseg == 1:
        return total, a, b
    return total, a, b, [ev[k].elapsed_time(ev[k + 1]) for k in range(nseg)]


def cpu_model() -> str:
    """The host CPU's model name (Linux /proc/cpuinfo), or "unknown"."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, budget_s: float):
    import numpy as np

    import oracle
    kap = oracle.kappa(cfg["v"], cfg["dt"], cfg["h"])
    z = np.zeros(kap.shape)
    amp = cfg["amp"].astype(np.float64)
    t0 = time.perf_counter()
    uc, up = oracle.leapfrog(kap, z, z, cfg["radius"], 1, src_idx=cfg["src_idx"], amp=amp)
    t1 = time.perf_counter() - t0
    more = max(0, min(int(budget_s / max(t1, 1e-3)) - 1, cfg["nt"] - 1))
    t0 = time.perf_counter()
    if more:
        oracle.leapfrog(kap, uc, up, cfg["radius"], more, it0=1, src_idx=cfg["src_idx"], amp=amp)
    t2 = time.perf_counter() - t0
    steps = 1 + more
    npts = kap.size
    cores = oracle.num_threads()
    # The same oracle on one thread, one step (the next step of the run).
    oracle.set_num_threads(1)
    t0 = time.perf_counter()
    oracle.leapfrog(kap, uc, up, cfg["radius"], 1, it0=1, src_idx=cfg["src_idx"], amp=amp)
    t3 = time.perf_counter() - t0
    oracle.set_num_threads(cores)
    return {"value": npts * steps / (t1 + t2) / 1e9, "unit": "Gpt/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": f"FP64 oracle, {steps} leapfrog steps of the same {cfg['nx']}x{cfg['ny']}x{cfg['nz']} "
                      f"layered workload from rest (source on), {t1 + t2:.1f} s",
            "single_thread": {"value": npts / t3 / 1e9, "unit": "Gpt/s", "sample": f"1 step, {t3:.1f} s"}}


def stream_rate(mib: int, n_in: int, steps: int, warmup: int):
    """(ms per launch, GB/s) of the library's streaming reference: n_in inputs
    of mib MiB read and one of mib MiB written per launch."""
    import torch

    import paper_1310_8232_amd as p
    nbytes = mib << 20
    ins = [torch.ones(nbytes // 4, device="cuda:0") for _ in range(n_in)] + [None] * (3 - n_in)
    out = torch.empty(nbytes // 4, device="cuda:0")
    for _ in range(warmup):
        p.stencil_stream_probe(*ins, out, nbytes)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        p.stencil_stream_probe(*ins, out, nbytes)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return ms, (n_in + 1) * nbytes / (ms * 1e-3) / 1e9


def stream_march_rate(n: int, steps: int, warmup: int):
    """(ms per launch, GB/s) of the streaming reference in the sweep's access
    order (three n^3 FP32 inputs, one output)."""
    import torch

    import paper_1310_8232_amd as p
    f = [torch.ones((n, n, n), device="cuda:0") for _ in range(3)]
    out = torch.empty((n, n, n), device="cuda:0")
    for _ in range(warmup):
        p.stencil_stream_probe_march(*f, out, (n, n, n))
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        p.stencil_stream_probe_march(*f, out, (n, n, n))
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    return ms, 16 * n ** 3 / (ms * 1e-3) / 1e9


def stream_probe(mib: int, n_in: int, steps: int, warmup: int) -> int:
    """Print the streaming reference's rate (n_in = 3 is the sweep's traffic mix)."""
    nbytes = mib << 20
    ms, gbs = stream_rate(mib, n_in, steps, warmup)
    print(json.dumps({"stream_probe": {"inputs": n_in, "bytes_read": n_in * nbytes, "bytes_written": nbytes,
                                       "launches": steps, "ms_per_launch": round(ms, 5),
                                       "gbs": round(gbs, 1)}}), flush=True)
    return 0


def gradient_bench(args) -> int:
    """One misfit + gradient evaluation (forward with checkpoints, residuals,
    segment recompute, adjoint steps, FP64 gradient accumulation) on the
    256^3 layered workload with a -5% velocity blob, 500 steps."""
    import numpy as np
    import torch

    import paper_1310_8232_amd as p
    from paper_1310_8232_amd import adjoint
    import workloads

    n = args.n if args.n != 512 else 256
    nt = args.nt or 500
    c = workloads.config_gradient(n, n, n, nt=nt)
    dev = torch.device("cuda:0")
    cu = lambda a, dt=torch.float32: torch.from_numpy(np.ascontiguousarray(a)).to(dev, dt)
    survey = adjoint.Survey(cu(c["src_idx"], torch.int64), cu(c["amp"].reshape(-1, 1)), cu(c["rec_idx"], torch.int64))
    # Observed data: the true model's traces (same kernels).
    pt = p.Propagator(cu(c["m_true"]), c["h"], c["dt"], 4, slowness2=True)
    obs, _, _ = adjoint.forward(pt, survey)
    del pt
    prop = p.Propagator(cu(c["m_cur"]), c["h"], c["dt"], 4, slowness2=True)
    sa, sb = torch.zeros_like(prop.kappa), torch.zeros_like(prop.kappa)
    rep, _, _ = prop.tune(sa, sb)
    del sa, sb
    adjoint.misfit_gradient(prop, survey, obs, checkpoint_every=args.checkpoint_every)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e2 = torch.cuda.Event(enable_timing=True)
    e0.record()
    traces, ckpts, _ = adjoint.forward(prop, survey, args.checkpoint_every)
    J, resid = adjoint.misfit(traces, obs)
    e1.record()
    g = adjoint.backward(prop, survey, resid, ckpts, args.checkpoint_every)
    e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    fwd_ms = e0.elapsed_time(e1)
    bwd_ms = e1.elapsed_time(e2)
    tot = fwd_ms + bwd_ms
    npts = n ** 3
    gnorm = float(torch.linalg.vector_norm(g).item())
    del traces, ckpts, g
    # The same evaluation keeping every time level in HBM (no recompute),
    # when (nt + 2) wavefields fit in half the free device memory.
    keep = None
    free, _ = torch.cuda.mem_get_info()
    if (nt + 2) * npts * 4 < free // 2:
        adjoint.misfit_gradient(prop, survey, obs, checkpoint_every=0)  # warm-up
        torch.cuda.synchronize()
        e0.record()
        Jk, gk, _ = adjoint.misfit_gradient(prop, survey, obs, checkpoint_every=0)
        e1.record()
        torch.cuda.synchronize()
        kms = e0.elapsed_time(e1)
        keep = {"ms": round(kms, 3), "gradients_per_s": round(1000.0 / kms, 4),
                "level_bytes": (nt + 2) * npts * 4, "same_misfit": bool(float(Jk.item()) == float(J.item()))}
        del gk
    out = {"metric": "misfit gradient evaluations per second (forward + checkpointed adjoint), 256^3 FP32",
           "value": round(1000.0 / tot, 4), "unit": "gradients/s", "n_gpus": 1, "steps": nt, "warmup": 1,
           "ms_per_step": round(tot / nt, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32 (FP64 misfit and gradient accumulation)", "data": "synthetic",
           "config": {"workload": f"{c['name']} layered + -5% blob, {nt} steps, receivers {len(c['rec_idx'])}, "
                                  f"checkpoint every {args.checkpoint_every}",
                      "tile": rep["tile"], "forward_ms": round(fwd_ms, 3), "backward_ms": round(bwd_ms, 3),
                      "wall_s": round(wall, 3), "misfit": float(J.item()),
                      "point_updates_per_s_G": round(npts * nt * 3 / (tot * 1e-3) / 1e9, 2),
                      "grad_norm": gnorm, "every_level_kept": keep}}
    print(json.dumps(out), flush=True)
    return 0


def batch_bench(args) -> int:
    """16 uneven shots (96^3 .. 256^3 and non-cubic), per-shape tuned tiles,
    500 steps each: sequential per-shot launches vs the batched launch, eager
    and captured in one HIP graph."""
    import numpy as np
    import torch

    import paper_1310_8232_amd as p
    import workloads

    nt = args.nt or 500
    cfgs = workloads.config_batch(nt=nt)
    dev = torch.device("cuda:0")
    shots = []
    t_tune = time.perf_counter()
    for c in cfgs:
        pr = p.Propagator(torch.from_numpy(c["v"]).to(dev), c["h"], c["dt"], 4, vmax=c["vmax"])
        pr.tune(parts=args.tune_parts, n_iter=args.tune_iter, n_rep=args.tune_rep)
        idx = torch.tensor(c["src_idx"], dtype=torch.int64, device=dev)
        amp = torch.from_numpy(c["amp"].reshape(-1, 1)).to(dev)
        shots.append((pr, p.make_src(idx, amp), (idx, amp)))
    t_tune = time.perf_counter() - t_tune
    total_pts = sum(int(np.prod(pr.shape)) for pr, _, _ in shots)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)

    # (a) one launch per shot per step, shots in turn.
    bufs = [(torch.zeros(pr.shape, device=dev), torch.zeros(pr.shape, device=dev)) for pr, _, _ in shots]
    def seq(k):
        st = [list(b) for b in bufs]
        for it in range(k):
            for (pr, src, _), s in zip(shots, st):
                p.stencil_step(pr.ctx, pr.kappa, s[0], s[1], it, src)
                s[0], s[1] = s[1], s[0]
    seq(5)
    torch.cuda.synchronize()
    e0.record()
    seq(nt)
    e1.record()
    torch.cuda.synchronize()
    seq_ms = e0.elapsed_time(e1)
    del bufs

    # (b) batched with the per-shot tiles, eager (the tiles each shot's own
    # search picked on an otherwise idle GPU).
    own = p.Batch([(pr, src) for pr, src, _ in shots])
    own.run(5)
    torch.cuda.synchronize()
    e0.record()
    own.run(nt)
    e1.record()
    torch.cuda.synchronize()
    own_ms = e0.elapsed_time(e1)
    own_launches = own.launches_per_step
    del own

    # (c) one tile for the whole batch, searched on the batch step itself;
    # eager, then the whole run captured in one graph.
    t_bt = time.perf_counter()
    batch = p.Batch([(pr, src) for pr, src, _ in shots],
                    tune=dict(n_iter=args.tune_iter, n_rep=args.tune_rep, parts=args.tune_parts))
    t_bt = time.perf_counter() - t_bt
    batch.run(5)
    torch.cuda.synchronize()
    e0.record()
    batch.run(nt)
    e1.record()
    torch.cuda.synchronize()
    batch_ms = e0.elapsed_time(e1)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            batch.run(nt)
    torch.cuda.current_stream().wait_stream(s)
    g.replay()
    torch.cuda.synchronize()
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1)
    gpts = lambda ms: round(total_pts * nt / (ms * 1e-3) / 1e9, 2)
    out = {"metric": "aggregate Gpoint-updates/s, 16 uneven shots, 8th-order FP32, graph-captured batched launch",
           "value": gpts(graph_ms), "unit": "Gpt/s", "n_gpus": 1, "steps": nt, "warmup": 5,
           "ms_per_step": round(graph_ms / nt, 5), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": f"16 uneven shots ({total_pts / 1e6:.1f} M points), layered models, centred "
                                  f"Ricker, {nt} steps", "shapes": [list(pr.shape[::-1]) for pr, _, _ in shots],
                      "per_shot_tune_seconds": round(t_tune, 2), "batch_tune_seconds": round(t_bt, 2),
                      "batch_tile": batch.tune_report["tile"], "batch_tune_gap": batch.tune_report["gap"],
                      "launches_per_step": batch.launches_per_step,
                      "sequential_per_shot_tiles_gpts": gpts(seq_ms),
                      "batched_per_shot_tiles_gpts": gpts(own_ms), "batched_per_shot_tiles_launches": own_launches,
                      "batched_eager_gpts": gpts(batch_ms), "graph_gpts": gpts(graph_ms)}}
    print(json.dumps(out), flush=True)
    return 0


def precision_bench(args) -> int:
    """The same sweep with the wavefield stored as FP32, FP16 and BF16 (scaled),
    FP32 arithmetic, on the 1024x1024x512 layered model: throughput per
    storage type (each with its own tuned tile)."""
    import torch

    import paper_1310_8232_amd as p
    import workloads

    nx, ny, nz = 1024, 1024, 512
    nt = args.steps
    c = workloads.config_layered(nx, ny, nz, nt=nt + args.warmup, seed=workloads.SEED + 3)
    dev = torch.device("cuda:0")
    v = torch.from_numpy(c["v"]).to(dev)
    idx = torch.tensor(c["src_idx"], dtype=torch.int64, device=dev)
    amp = torch.from_numpy(c["amp"].reshape(-1, 1)).to(dev)
    npts = nx * ny * nz
    res = {}
    for storage, nbytes in (("f32", 16), ("f16", 10), ("bf16", 10)):
        prop = p.Propagator(v, c["h"], c["dt"], 4, vmax=c["vmax"], storage=storage,
                            storage_scale=1.0 if storage == "f32" else 2.0 ** 12)
        rep, _, _ = prop.tune(n_iter=args.tune_iter, n_rep=args.tune_rep, parts=args.tune_parts)
        src = p.make_src(idx, amp)
        a, b = prop.zeros(), prop.zeros()
        a, b = prop.run(a, b, args.warmup, src)
        ms, a, b = time_steps(prop, a, b, nt, args.warmup, src, torch.cuda.current_stream())
        step = ms / nt
        res[storage] = {"gpts": round(npts / (step * 1e-3) / 1e9, 2), "ms_per_step": round(step, 5),
                        "bytes_per_update": nbytes,
                        "hbm_gbs_algorithmic": round(nbytes * npts / (step * 1e-3) / 1e9, 1),
                        "tile": prop.tile.as_dict(), "tune_s": round(rep["seconds"], 2)}
        del prop, a, b
        torch.cuda.empty_cache()
    out = {"metric": "Gpoint-updates/s by wavefield storage type, 1024x1024x512 8th-order, FP32 arithmetic",
           "value": res["f16"]["gpts"], "unit": "Gpt/s", "n_gpus": 1, "steps": nt, "warmup": args.warmup,
           "ms_per_step": res["f16"]["ms_per_step"], "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f16 storage, f32 compute", "data": "synthetic",
           "config": {"workload": f"layered 1024x1024x512, R=4, {nt} steps, storage scale 2^12 for 16-bit",
                      "by_storage": res,
                      "speedup_f16_vs_f32": round(res["f16"]["gpts"] / res["f32"]["gpts"], 3),
                      "speedup_bf16_vs_f32": round(res["bf16"]["gpts"] / res["f32"]["gpts"], 3)}}
    print(json.dumps(out), flush=True)
    return 0


def paper_bench(args) -> int:
    """The paper's blocksize-search experiments on the GPU tile space, at its
    per-process shapes and order (R = 5): exhaustive sweep (Section 3.5),
    repeated searches per policy with MinTime / ActualTime / gap and the time
    of a 448-step run with the chosen tile (Tables 4-5), and the P-part budget
    sweep against the exhaustive best (Section 3.7, Table 6)."""
    import statistics

    import torch

    import paper_1310_8232_amd as p
    import workloads

    iters = 448  # the paper's iteration count
    dev = torch.device("cuda:0")
    shapes = [(200, 200, 800), (300, 300, 800), (250, 250, 1500)]
    if args.paper_shapes:
        shapes = [tuple(int(v) for v in sh.split("x")) for sh in args.paper_shapes.split(",")]
    out = {}
    for (nx, ny, nz) in shapes:
        c = workloads.config_layered(nx, ny, nz, nt=iters, radius=5)
        prop = p.Propagator(torch.from_numpy(c["v"]).to(dev), c["h"], c["dt"], 5, vmax=c["vmax"])
        idx = torch.tensor(c["src_idx"], dtype=torch.int64, device=dev)
        amp = torch.from_numpy(c["amp"].reshape(-1, 1)).to(dev)
        src = p.make_src(idx, amp)

        def total_ms():
            a, b = prop.zeros(), prop.zeros()
            ms, _, _ = time_steps(prop, a, b, iters, 0, src, torch.cuda.current_stream())
            return ms

        key = f"{nx}x{ny}x{nz}"
        rec = {}
        rep, tab, cands = prop.tune(n_iter=args.tune_iter, n_rep=1, parts=0, include_plain=True, table_cap=2048)
        best = total_ms()
        # The whole exhaustive table (the GPU form of the paper's blocksize
        # landscapes, Figs. 3-4): Gpt/s of every candidate over n_iter steps.
        npts = nx * ny * nz
        landscape = [{"tile": t, "gpts": round(npts * args.tune_iter / (ms * 1e-3) / 1e9, 2)}
                     for t, ms in zip(cands or [], (tab or [[]])[0])]
        rec["exhaustive"] = {"n_candidates": rep["n_candidates"], "tile": rep["tile"], "seconds": rep["seconds"],
                             "total_ms_448": round(best, 3), "landscape": landscape}
        pol = {}
        for policy in ("ob", "min", "worst", "avg"):
            runs = []
            for _ in range(args.paper_repeats):
                rep, _, _ = prop.tune(policy=policy, n_iter=args.tune_iter, n_rep=3, parts=5)
                runs.append({"tile": rep["tile"], "min_time_ms": round(rep["min_time_ms"], 4),
                             "actual_time_ms": round(rep["actual_time_ms"], 4), "gap": round(rep["gap"], 5),
                             "n_candidates": rep["n_candidates"], "total_ms_448": round(total_ms(), 3)})
            tot = [r["total_ms_448"] for r in runs]
            pol[policy] = {"runs": runs, "best": min(tot), "avg": round(statistics.mean(tot), 3), "worst": max(tot),
                           "std": round(statistics.pstdev(tot), 4),
                           "mean_abs_gap": round(statistics.mean(abs(r["gap"]) for r in runs), 5)}
        rec["policies"] = pol
        sweep = []
        for P in (2, 3, 4, 5, 6):
            rep, _, _ = prop.tune(policy="worst", n_iter=args.tune_iter, n_rep=3, parts=P)
            t = total_ms()
            sweep.append({"P": P, "n_candidates": rep["n_candidates"], "search_s": round(rep["seconds"], 3),
                          "tile": rep["tile"], "total_ms_448": round(t, 3),
                          "vs_exhaustive": round(t / best - 1.0, 4)})
        rec["budget_sweep"] = sweep
        out[key] = rec
        print(f"bench: paper experiments {key} done", file=sys.stderr, flush=True)
        del prop
        torch.cuda.empty_cache()
    print(json.dumps({"paper_experiments": out, "radius": 5, "iterations": iters,
                      "repeats_per_policy": args.paper_repeats}), flush=True)
    return 0


def pitch_bench(args) -> int:
    """Rows padded to 128 bytes at the paper's per-process shapes (R = 5):
    Gpt/s of a 448-step run with the searched tile for the grid as given,
    the same grid with padded rows, and a grid of the padded width and the
    same volume (the aligned reference)."""
    import torch

    import paper_1310_8232_amd as p
    import workloads

    iters = 448
    dev = torch.device("cuda:0")
    shapes = [(200, 200, 800), (300, 300, 800), (250, 250, 1500)]
    if args.paper_shapes:
        shapes = [tuple(int(v) for v in sh.split("x")) for sh in args.paper_shapes.split(",")]
    out = {}

    def run(nx, ny, nz, pitch):
        c = workloads.config_layered(nx, ny, nz, nt=iters, radius=5)
        prop = p.Propagator(torch.from_numpy(c["v"]).to(dev), c["h"], c["dt"], 5, vmax=c["vmax"], pitch=pitch)
        idx = torch.tensor([prop.index(nz // 2, ny // 2, nx // 2)], dtype=torch.int64, device=dev)
        amp = torch.from_numpy(c["amp"].reshape(-1, 1)).to(dev)
        src = p.make_src(idx, amp)
        rep, _, _ = prop.tune(n_iter=args.tune_iter, n_rep=3)
        a, b = prop.zeros(), prop.zeros()
        ms, _, _ = time_steps(prop, a, b, iters, 0, src, torch.cuda.current_stream())
        r = {"grid": [nx, ny, nz], "pitch": prop.pitch, "tile": rep["tile"], "ms_448": round(ms, 3),
             "gpts": round(nx * ny * nz * iters / (ms * 1e-3) / 1e9, 2)}
        del prop, a, b
        torch.cuda.empty_cache()
        return r

    for (nx, ny, nz) in shapes:
        plain = run(nx, ny, nz, None)
        padded = run(nx, ny, nz, "align")
        P = padded["pitch"]
        nz_ref = max(1, round(nx * nz / P))
        ref = run(P, ny, nz_ref, None)
        out[f"{nx}x{ny}x{nz}"] = {"as_given": plain, "padded": padded, "aligned_same_volume": ref,
                                  "padded_vs_given": round(padded["gpts"] / plain["gpts"], 4),
                                  "padded_vs_aligned": round(padded["gpts"] / ref["gpts"], 4)}
        print(f"bench: pitch {nx}x{ny}x{nz}: {plain['gpts']} -> {padded['gpts']} Gpt/s padded to {P} "
              f"(aligned {P}x{ny}x{nz_ref}: {ref['gpts']})", file=sys.stderr, flush=True)
    print(json.dumps({"padded_rows": out, "radius": 5, "iterations": iters}), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=512, help="grid points per axis")
    ap.add_argument("--radius", type=int, default=4)
    ap.add_argument("--tune-parts", type=int, default=0, help="0 = every tile, P >= 2 = P-part grid")
    ap.add_argument("--tune-iter", type=int, default=10)
    ap.add_argument("--tune-rep", type=int, default=3)
    ap.add_argument("--tile", type=str, default="", help="fixed tile bx,by,ry,dz,vw,xcd,pf (skips the search)")
    ap.add_argument("--tile2", type=str, default="",
                    help="fixed two-step tile bx,by,dz,vw,xcd,pf: runs two-step launches (skips the search)")
    ap.add_argument("--compare-steps", type=int, default=200, help="steps timed for plain and default tiles")
    ap.add_argument("--cpu-budget", type=float, default=16.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true")
    ap.add_argument("--no-two-step", action="store_true", help="search one-step tiles only")
    ap.add_argument("--paper-repeats", type=int, default=10, help="searches per policy (paper workload; the paper reports 10 executions)")
    ap.add_argument("--paper-shapes", type=str, default="", help="e.g. 200x200x800,300x300x800")
    ap.add_argument("--workload", choices=("sweep", "gradient", "batch", "precision", "paper", "pitch"),
                    default="sweep",
                    help="sweep: the autotuned step (default); gradient: misfit + adjoint gradient; "
                         "batch: 16 uneven shots; precision: 16-bit storage; paper: the search experiments; "
                         "pitch: rows padded to 128 bytes at the paper's shapes")
    ap.add_argument("--nt", type=int, default=0, help="time steps of the gradient workload (default 500)")
    ap.add_argument("--checkpoint-every", type=int, default=50)
    ap.add_argument("--stream-probe", type=int, default=0, metavar="MIB",
                    help="only time the library's streaming reference over MIB MiB arrays")
    ap.add_argument("--stream-inputs", type=int, default=3, choices=(1, 2, 3),
                    help="inputs of the streaming reference (1 = copy, 3 = the sweep's read/write mix)")
    args = ap.parse_args(argv)

    if args.gpus != 1:
        print(f"bench.py: the sweep runs on one GPU; --gpus {args.gpus} is not supported "
              "(sharding across GPUs is a design note only).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1310_8232_amd as p
    import workloads

    dev = torch.device("cuda:0")
    if args.stream_probe:
        return stream_probe(args.stream_probe, args.stream_inputs, args.steps, args.warmup)
    if args.workload == "gradient":
        return gradient_bench(args)
    if args.workload == "batch":
        return batch_bench(args)
    if args.workload == "precision":
        return precision_bench(args)
    if args.workload == "paper":
        return paper_bench(args)
    if args.workload == "pitch":
        return pitch_bench(args)
    n = args.n
    nt = args.warmup + args.steps
    t0 = time.perf_counter()
    cfg = workloads.config_layered(n, n, n, nt=max(nt, 1), radius=args.radius)
    print(f"bench: inputs {cfg['name']} dt={cfg['dt']:.6e} vmax={cfg['vmax']:.1f} "
          f"({time.perf_counter() - t0:.1f}s)", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    prop = p.Propagator(torch.from_numpy(cfg["v"]).to(dev), cfg["h"], cfg["dt"], args.radius, vmax=cfg["vmax"])
    idx = torch.tensor(cfg["src_idx"], dtype=torch.int64, device=dev)
    amp = torch.from_numpy(cfg["amp"].reshape(-1, 1)).to(dev)
    src = p.make_src(idx, amp)
    npts = n * n * n

    tune = None
    temporal = 1
    if args.tile2:
        bx, by, dz, vw, xcd, pf = [int(x) for x in args.tile2.split(",")]
        prop.tile = p.make_tile(p.TILE_ZMARCH2, bx, by, 1, dz, vw, xcd, pf)
        temporal = 2
    elif args.tile:
        f = [int(x) for x in args.tile.split(",")]
        prop.tile = p.make_tile(p.TILE_ZMARCH, *f)
    else:
        # The search covers one-step tiles and two-step (time-blocked) tiles;
        # the mode with the smaller selected time per step runs.
        sa = torch.zeros_like(prop.kappa)
        sb = torch.zeros_like(prop.kappa)
        rep, _, _ = prop.tune(sa, sb, n_iter=args.tune_iter, n_rep=args.tune_rep, parts=args.tune_parts)
        rep2 = None
        if args.radius in (3, 4, 5) and not args.no_two_step:
            rep2, _, _ = prop.tune(sa, sb, n_iter=args.tune_iter, n_rep=args.tune_rep, parts=args.tune_parts,
                                   temporal=2)
            if rep2["actual_time_ms"] < rep["actual_time_ms"]:
                temporal = 2
        del sa, sb
        tune = {"policy": "MWMB", "n_candidates": rep["n_candidates"], "n_iter": args.tune_iter,
                "n_rep": args.tune_rep, "min_time_ms": rep["min_time_ms"], "actual_time_ms": rep["actual_time_ms"],
                "gap": rep["gap"], "seconds": rep["seconds"], "default_tile_ms": rep["default_time_ms"],
                "two_step": None if rep2 is None else
                {"tile": rep2["tile"], "n_candidates": rep2["n_candidates"], "min_time_ms": rep2["min_time_ms"],
                 "actual_time_ms": rep2["actual_time_ms"], "gap": rep2["gap"], "seconds": rep2["seconds"]},
                "mode": "two-step" if temporal == 2 else "one-step"}
        print(f"bench: tuned {rep['tile']} nC={rep['n_candidates']} in {rep['seconds']:.1f}s "
              f"gap={rep['gap']:+.4f}; two-step {None if rep2 is None else rep2['tile']} "
              f"({None if rep2 is None else round(rep2['actual_time_ms'], 3)} vs {rep['actual_time_ms']:.3f} ms)",
              file=sys.stderr, flush=True)
    tile = (prop.tile2 if temporal == 2 else prop.tile).as_dict()

    a = torch.zeros_like(prop.kappa)
    b = torch.zeros_like(prop.kappa)
    compare = {}
    if not args.no_compare:
        chosen = prop.tile
        for name, t in (("plain_tiling", p.make_tile(p.TILE_PLAIN, bx=64, by=4, dz=1)),
                        ("default_tile", p.StencilTile())):
            prop.tile = t
            k = min(args.compare_steps, args.steps)
            ms, _, _ = time_steps(prop, a, b, k, 0, src, stream)
            compare[name] = {"tile": prop.tile.as_dict(), "gpts": npts * k / (ms * 1e-3) / 1e9,
                             "ms_per_step": ms / k}
        prop.tile = chosen
        a.zero_()
        b.zero_()

    # Warm-up, then exactly `steps` timed steps of the time loop.
    spare = [torch.zeros_like(prop.kappa), torch.zeros_like(prop.kappa)] if temporal == 2 else None
    a, b = prop.run(a, b, args.warmup, src, it0=0, stream=stream, temporal=temporal, spare=spare)
    torch.cuda.synchronize()
    res = time_steps(prop, a, b, args.steps, args.warmup, src, stream, temporal=temporal, spare=spare, nseg=5)
    ms, a, b = res[:3]
    seg = None
    if len(res) == 4:
        g = sorted(npts * (args.steps // 5) / (t * 1e-3) / 1e9 for t in res[3])
        seg = {"segments": 5, "gpts_min": round(g[0], 3), "gpts_median": round(g[2], 3), "gpts_max": round(g[-1], 3)}
    if not bool(torch.isfinite(a).all()):
        print("bench: non-finite wavefield", file=sys.stderr)
        return 1
    step_ms = ms / args.steps
    gpts = npts / (step_ms * 1e-3) / 1e9
    # Algorithmic bytes per launch: 16 B per point for a one-step sweep,
    # 20 B per point for a two-step one (reads u^n, u^{n-1}, kappa; writes
    # u^{n+1}, u^{n+2}); launch duration = 1 or 2 steps.
    launch_ms = step_ms * temporal
    launch_bytes = (BYTES_PER_UPDATE if temporal == 1 else 20) * npts
    achieved = launch_bytes / (launch_ms * 1e-3) / 1e9
    traffic = load_traffic(tile, npts)
    # Streaming references with the one-step sweep's traffic mix (three
    # inputs, one output), timed after the sweep: contiguous chunks per
    # workgroup, and the sweep's own access order without the stencil (the
    # practical HBM ceiling of that pattern).
    del a, b, spare
    s_ms, s_gbs = stream_rate(512, 3, 20, 3)
    m_ms, m_gbs = stream_march_rate(n, 20, 3) if n % 4 == 0 else (None, None)
    sweep_gbs = achieved  # algorithmic bytes of the launches that ran (16 B/update, or 20 B per two)
    ceiling = {"stream_3in_1out_gbs": round(s_gbs, 1),
               "stream_sweep_order_gbs": None if m_gbs is None else round(m_gbs, 1),
               "sweep_frac_of_stream": round(sweep_gbs / max(s_gbs, m_gbs or 0.0), 4)}
    out = {
        "metric": METRIC, "value": round(gpts, 3), "unit": "Gpt/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(step_ms, 5), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{cfg['name']} model, order {2 * args.radius} (R={args.radius}) {6 * args.radius + 1}-point star, "
                               f"FP32, Ricker source, {args.steps} timed steps",
                   "grid": [n, n, n], "radius": args.radius, "tile": tile, "tune": tune,
                   "plain_tiling": compare.get("plain_tiling"), "default_tile": compare.get("default_tile"),
                   "speedup_vs_plain": (round(gpts / compare["plain_tiling"]["gpts"], 3)
                                        if "plain_tiling" in compare else None),
                   "timed_segments": seg, "stream_ceiling": ceiling},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     # what the figures above are per: one launch of the dominant kernel
                     "kernel": "two-step sweep (zmarch2)" if temporal == 2 else "one-step sweep (zmarch)",
                     "updates_per_launch": temporal, "algorithmic_bytes_per_launch": launch_bytes,
                     "launch_ms": round(launch_ms, 5),
                     # measured bytes per launch over the launch time: the rate the kernel moves
                     "traffic_gbs": None if traffic is None else round(traffic / (launch_ms * 1e-3) / 1e9, 1),
                     # the one-step sweep's 16 B per update at this update rate
                     "one_step_equivalent_gbs": round(gpts * BYTES_PER_UPDATE, 1)},
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
