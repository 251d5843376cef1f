#!/usr/bin/env python3
"""Throughput of the acoustic FWI hot path on one MI355X.

A step is one shot gradient: forward solve with source injection and receiver
sampling, forward states kept within the HBM budget (every state when it fits;
otherwise the library's choice of segmented history or binomial
checkpointing), residual and misfit, adjoint solve with the imaging condition,
and the gradient finalise: the whole hot path once over one shot of the
workload.  The default workload is the 3D head (256^3 at 0.5 mm + 30-cell
sponge = 316^3 padded, 10th order, 3000 steps, 1024 receivers, 256 GiB
budget): the largest single-GPU configuration, whose fields exceed the
Infinity Cache, so that the HBM fraction measures HBM.

value = grid-point updates per second of forward + adjoint propagation,
2 * N_padded * (nt - 1) per step (recomputation is not counted as work; its
factor is reported).

roofline: the dominant kernel is the adjoint step of the path the gradient
takes.  Imaging from the stored v (full or segmented history) it alternates an
adjoint step without imaging (reads w^{m+1}, w^{m+2}, k; writes w^m: 16 bytes)
and one adding two imaging terms (also reads v^m, v^{m+1}, G and writes G: 32
bytes), 24 bytes per grid-point update on average; the fused adjoint of
binomial checkpointing reads u^m, w^{m+1}, w^{m+2}, k, G and writes w^m, G (28
bytes).  The line gives both fractions.  Beside it, the forward step at 16
bytes (reads u^n, u^{n-1}, k; writes u^{n+1}).  Kernel times come from HIP
events the library records on the solve stream around its time loops during
the timed steps, with the step and launch counts.  The "binomial" key times
the same gradient with binomial checkpointing forced in the same workspace.

Extra keys: the config-2 2D shot gradient and forward (same steps), and a
bounded serving run over the full six-class request mix (2D 256^2, 512^2,
1024^2 and 3D 128^3, 192^3, 256^3, nt 500-3000; --leg-requests requests,
arriving at --load times the one-at-a-time rate): served shot solves/s and
p50/p99 against one request at a time.
--fourth-order, --sinc, --medium and --pml add those solver variants.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of the dominant kernel, from two rocprofv3 --pmc runs
# (FETCH_SIZE, then WRITE_SIZE, KiB per dispatch, averaged over the kernel's
# dispatches) scaled by what the same counters read for a 1 GiB device copy.
# Valid only for the kernel source they were taken with: the sha256 of the
# kernel file and its header; any change makes `traffic` null until the
# counters are taken again.
MEASURED_TRAFFIC = {
    # keyed by workload and the adjoint kernel: "pair" = the adjoint imaging
    # from the stored v (mode 6, no imaging, and mode 5, two imaging terms, in
    # turn; per-dispatch figures averaged over the pair), "fused" = the adjoint
    # with its own stencil of u^m (mode 0, binomial checkpointing), "forward" =
    # the plain forward step of a forward solve
    "config2/pair": {"sha256": "a3a270b9d6f6091d300dcb38d0a3b444e81e7962e9e1de5ce89ad9c84cea5057",
                     "fetch_kib": 10940.59, "write_kib": 7153.05,
                     "copy_fetch_kib": 524308.00, "copy_write_kib": 1048576.0},
    "config4/pair": {"sha256": "a3a270b9d6f6091d300dcb38d0a3b444e81e7962e9e1de5ce89ad9c84cea5057",
                     "fetch_kib": 338138.13, "write_kib": 187230.00,
                     "copy_fetch_kib": 524315.50, "copy_write_kib": 1048576.0},
    "config4/fused": {"sha256": "a3a270b9d6f6091d300dcb38d0a3b444e81e7962e9e1de5ce89ad9c84cea5057",
                      "fetch_kib": 477481.36, "write_kib": 249640.00,
                      "copy_fetch_kib": 524308.00, "copy_write_kib": 1048576.0},
    "config4/forward": {"sha256": "a3a270b9d6f6091d300dcb38d0a3b444e81e7962e9e1de5ce89ad9c84cea5057",
                        "fetch_kib": 240994.32, "write_kib": 124852.00,
                        "copy_fetch_kib": 524315.50, "copy_write_kib": 1048576.0},
}


def kernel_source_sha():
    import hashlib
    h = hashlib.sha256()
    for f in ("csrc/step_kernels.h", "csrc/common.h"):
        with open(os.path.join(ROOT, "paper_2110_03345_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(key):
    """HBM bytes per launch of a kernel ("workload/kernel"), or None if not
    measured for the current kernel source."""
    m = MEASURED_TRAFFIC.get(key)
    if not m or m["sha256"] != kernel_source_sha():
        return None
    gib_kib = float(1 << 20)
    reads = m["fetch_kib"] * 1024 * gib_kib / m["copy_fetch_kib"]
    writes = m["write_kib"] * 1024 * gib_kib / m["copy_write_kib"]
    return reads + writes
FWD_BYTES = 16   # read u^n, u^{n-1}, k; write u^{n+1}
FWD4_BYTES = 32  # fourth order: read u^n, k, write p; read p, u^n, u^{n-1}, k, write u^{n+1}
ADJ_BYTES = 28   # read u^m, w^{m+1}, w^{m+2}, k, G; write w^m, G
# full history: the adjoint reads v^m instead of u^m and G is read and written
# every other step (two imaging terms per even step): 16 B and 32 B in turn
ADJ_BYTES_PAIRED = 24
# fourth-order adjoint step: read u^m, k, write p; read w^{m+1}, k, write q;
# read q, p, w^{m+1}, w^{m+2}, k, H, write w^m, H
ADJ4_BYTES = 56
# with p^n kept (every state, or segment by segment) the adjoint drops its first
# launch: read w^{m+1}, k, write q; read q, p, w^{m+1}, w^{m+2}, k, H, write w^m, H
ADJ4_BYTES_FULL = 44
# medium forward step: read u^n, u^{n-1}, k, ndim density gradients, attenuation; write u^{n+1}


def medium_bytes(ndim):
    return 4 * (5 + ndim)

WORKLOADS = {
    "config2": "2D breast-like phantom, 1024^2 at 0.2 mm + 40-cell sponge (1104^2 padded), "
               "8th order, 2500 steps, 1 shot, 256 ring receivers; gradient at the 1500 m/s "
               "starting model against data from the phantom",
    "config4": "3D head-like phantom, 256^3 at 0.5 mm + 30-cell sponge (316^3 padded), 10th order, "
               "3000 steps, 1 shot, 1024 hemisphere receivers; gradient at the skull-only starting "
               "model, forward states kept within a 256 GiB HBM budget (segmented history)",
    "config3": "2D breast-like phantom, 512^2 at 0.2 mm + 40-cell sponge (592^2 padded), 8th order, "
               "1500 steps, shot 0 of the 64-shot ring survey; gradient at 1500 m/s",
    "fwi": "frequency-block inversion of the 2D breast-like phantom of config 3 (512^2 at 0.2 mm, "
           "1500 steps, 64 shots on a 256-element ring): bands 300/400/500/600 kHz, 4 iterations of 16 "
           "random shots per band (each shot once per band), masked normalised gradient descent of "
           "10 m/s from 1500 m/s",
    "serving": "seeded Poisson stream of forward (70%) and gradient (30%) requests of 1-16 shots, each "
               "with its own phantom and ring/hemisphere geometry; served with continuous batching vs "
               "one request at a time through the plain entry points",
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="config4", choices=sorted(WORKLOADS))
    ap.add_argument("--budget-gb", type=float, default=256.0,
                    help="HBM budget of the gradient workspace in GiB (checkpointing beyond it)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-forward", action="store_true")
    ap.add_argument("--binomial", action="store_true",
                    help="headline gradient with binomial checkpointing (checkpointing = 1)")
    ap.add_argument("--no-binomial", action="store_true",
                    help="skip the binomial-checkpointing leg beside a checkpointed headline")
    ap.add_argument("--no-config2", action="store_true",
                    help="skip the extra config-2 (2D breast) shot gradient and forward")
    ap.add_argument("--no-serving", action="store_true", help="skip the bounded serving leg")
    ap.add_argument("--fourth-order", action="store_true",
                    help="also time the forward and gradient solves with fourth-order time")
    ap.add_argument("--sinc", action="store_true",
                    help="also time the shot gradient with windowed-sinc sources and receivers")
    ap.add_argument("--medium", action="store_true",
                    help="also time forward solves in a heterogeneous medium (density, attenuation) "
                         "and the medium shot gradient on the 2D breast grid")
    ap.add_argument("--pml", action="store_true",
                    help="also time the forward solve with the perfectly matched layer")
    ap.add_argument("--nt", type=int, default=0,
                    help="override the number of time steps (profiling runs only)")
    ap.add_argument("--requests", type=int, default=60, help="serving: number of requests")
    ap.add_argument("--leg-requests", type=int, default=40,
                    help="serving leg of the default run: number of requests of the full six-class "
                         "mix")
    ap.add_argument("--full-mix", action="store_true",
                    help="serving: all six grid classes and nt 500-3000 (default: 2D classes and "
                         "128^3, nt 500-1500)")
    ap.add_argument("--classes-2d", default=None,
                    help="serving: comma-separated 2D grid classes (overrides the mix; '' for none)")
    ap.add_argument("--classes-3d", default=None,
                    help="serving: comma-separated 3D grid classes (overrides the mix; '' for none)")
    ap.add_argument("--frac-gradient", type=float, default=0.3,
                    help="serving: fraction of gradient requests (the rest are forward solves)")
    ap.add_argument("--no-graphs", action="store_true", help="serving: direct launches, no hipGraphs")
    ap.add_argument("--max-slots", type=int, default=32, help="serving: shots per engine")
    ap.add_argument("--max-chunk", type=int, default=64, help="serving: ticks per graph chunk")
    ap.add_argument("--no-baseline", action="store_true", help="serving: skip the one-at-a-time run")
    ap.add_argument("--load", type=float, default=3.0,
                    help="serving: arrival rate in units of the one-at-a-time service rate of the "
                         "stream's first requests (3 keeps both systems busy through the stream, "
                         "so solves/s measures capacity; near 1.5 the server waits for arrivals)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 1 GiB device-to-device copy first (scale for HBM byte counters)")
    return ap.parse_args()


def build_workload(name, nt=0):
    import numpy as np
    import workloads as W
    kw = {"nt": nt} if nt else {}
    if name == "config2":
        w = W.config2(**kw)
        vp_model = np.full(w.shape, 1500.0, dtype=np.float32)
        return w, w.vp, vp_model
    if name == "config3":
        w = W.config3(**kw)
        return w, w.vp_true, w.vp_start
    if name == "config4":
        w = W.config4(**kw)
        return w, w.vp_true, w.vp_start
    raise ValueError(name)


def cpu_baseline(w, vp_model, obs_np, seconds):
    """The FP64 oracle's shot gradient on the same grid, for a bounded number
    of time steps chosen to take about `seconds` on the host cores."""
    import numpy as np
    import oracle
    npad = w.padded_points

    def run(nt):
        g = oracle.Grid(**{**w.grid_kwargs(), "nt": nt})
        t0 = time.perf_counter()
        oracle.gradient(g, vp_model, w.src_xyz, w.wavelet[:, :nt], w.rec_xyz, obs_np[:, :nt])
        return time.perf_counter() - t0

    # cost per step from two short runs (their difference drops the set-up)
    per_step = max(run(12) - run(4), 1e-9) / 8
    nt_s = int(max(8, min(w.nt, seconds / per_step)))
    el = run(nt_s)
    cores = oracle.num_threads()
    # one thread: the per-step cost from 3 and 1 steps (about the same set-up)
    oracle.set_num_threads(1)
    try:
        per_step_1 = max(run(3) - run(1), 1e-9) / 2
    finally:
        oracle.set_num_threads(cores)
    return {
        "value": 2.0 * npad * (nt_s - 1) / el,
        "unit": "grid-point updates/s (fwd+adj)",
        "cores": cores,
        "kind": "oracle",
        "sample": f"{w.name} grid ({'x'.join(map(str, w.padded_shape))} padded), first {nt_s} of "
                  f"{w.nt} steps, one shot gradient (FP64 C, OpenMP), {el:.1f} s",
        "cpu_model": cpu_model(),
        "one_thread_value": 2.0 * npad / per_step_1,
    }


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def fwi_bench(args):
    """Shot gradients per second inside the frequency-block inversion loop and
    the reconstruction it reaches (mean |vp - vp_true| inside the ring)."""
    import numpy as np
    import torch

    import paper_2110_03345_amd as S
    import workloads as W
    from paper_2110_03345_amd import fwi

    dev = torch.device("cuda:0")
    w = W.config3()
    shots = w.shot_src_xyz
    wav = torch.from_numpy(w.wavelet[0]).to(dev)
    vp_t = torch.from_numpy(w.vp_true).to(dev)
    obs = torch.empty((shots.shape[0], w.rec_xyz.shape[0], w.nt), dtype=torch.float32, device=dev)
    fws = None
    for i in range(shots.shape[0]):          # observed data: forward solves on the phantom
        plan = S.Plan.from_workload(w, src_xyz=shots[i:i + 1])
        if fws is None:
            fws = plan.workspace(S.STRIDE_MODE_FORWARD, device=dev)
        plan.forward(vp_t, wav.reshape(1, -1), traces=obs[i], ws=fws)
    torch.cuda.synchronize()
    del fws
    X = np.meshgrid(*[np.arange(n) * w.spacing for n in w.shape], indexing="ij")
    cen = (w.shape[0] - 1) * w.spacing / 2
    roi = (X[0] - cen) ** 2 + (X[1] - cen) ** 2 < (45e-3 - 4e-3) ** 2
    survey = fwi.Survey(w.shape, w.spacing, w.space_order, w.nb, w.vref, w.dt, w.nt, shots,
                        w.rec_xyz, wav, obs)
    opt = fwi.GradientDescent(10.0, bounds=(1400.0, 1650.0),
                              mask=torch.from_numpy(roi.astype(np.float32)).to(dev))
    vp0 = torch.from_numpy(w.vp_start).to(dev)
    freqs = (3e5, 4e5, 5e5, 6e5)
    vp, hist = fwi.invert(survey, vp0, freqs, 4, 16, opt, seed=0,
                          log=lambda m: print("[bench] " + m, file=sys.stderr, flush=True))
    err0 = float(np.abs(w.vp_start - w.vp_true)[roi].mean())
    err = float(np.abs(vp.cpu().numpy() - w.vp_true)[roi].mean())
    line = {
        "metric": "shot gradients/s inside the frequency-block inversion loop",
        "value": hist.shot_gradients / hist.seconds,
        "unit": "shot gradients/s",
        "n_gpus": 1,
        "steps": len(hist.misfit),
        "warmup": 0,
        "ms_per_step": 1e3 * hist.seconds / len(hist.misfit),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded breast-like phantom; observed data from forward solves on it)",
        "config": {"workload": f"fwi: {WORKLOADS['fwi']}", "padded_points": w.padded_points,
                   "nt": w.nt, "shots": int(shots.shape[0]), "shot_gradients": hist.shot_gradients},
        "seconds": hist.seconds,
        "misfit_per_iteration": hist.misfit,
        "roi_model_error_m_s": {"start": err0, "final": err},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def serving_run(args, nreq, full_mix=None):
    """Served shot solves per second and p50/p99 latency against one request at
    a time, on the same seeded request stream of nreq requests; every served
    result is compared bit for bit with its one-at-a-time result.  full_mix:
    all six grid classes with nt 500-3000 (default: args.full_mix)."""
    import torch

    from paper_2110_03345_amd.serving import Server, serve_one_at_a_time
    from workloads.serving_mix import materialise, request_stream

    if args.full_mix if full_mix is None else full_mix:
        kw = dict(nt_range=(500, 3000), classes_2d=(256, 512, 1024), classes_3d=(128, 192, 256))
    else:
        kw = dict(nt_range=(500, 1500), classes_2d=(256, 512, 1024), classes_3d=(128,))
    for dim in ("2d", "3d"):
        sel = getattr(args, "classes_" + dim)
        if sel is not None:
            kw["classes_" + dim] = tuple(int(c) for c in sel.split(",") if c)
    kw["frac_gradient"] = args.frac_gradient
    # calibration: the one-at-a-time service time of the stream's first requests
    # sets the arrival rate (a request's content does not depend on the rate:
    # the generator draws the same numbers for it at any rate, only the
    # arrival times scale)
    seed = 2024
    probe = [materialise(r) for r in request_stream(min(24, nreq), seed, 1.0, **kw)]
    serve_one_at_a_time(probe[:1], realtime=False)
    cal = serve_one_at_a_time(probe, realtime=False)
    mean_service = cal["makespan_s"] / len(probe)
    rate = args.load / mean_service
    specs = [materialise(r) for r in request_stream(nreq, seed, rate, **kw)]
    print(f"[bench] serving: {len(specs)} requests, {sum(r.nshots for r in specs)} shots, "
          f"mean one-at-a-time service {mean_service * 1e3:.1f} ms, rate {rate:.2f}/s",
          file=sys.stderr, flush=True)
    torch.cuda.synchronize()

    def progress(tag):
        return lambda n, total: print(f"[bench] {tag}: {n}/{total} requests done", file=sys.stderr,
                                      flush=True)

    torch.cuda.empty_cache()   # the calibration's cached blocks would shrink the server's budget
    srv = Server(use_graphs=not args.no_graphs, max_slots=args.max_slots, max_chunk=args.max_chunk)
    try:
        served = srv.run(specs, realtime=True, progress=progress("served"))
    finally:
        srv.close()
    print(f"[bench] served: {served['solves_per_s']:.1f} shot solves/s, p50 {served['p50_s']:.3f} s, "
          f"p99 {served['p99_s']:.3f} s", file=sys.stderr, flush=True)
    out = {
        "requests": len(specs),
        "shots": served["shot_solves"],
        "grid_classes": {"2d": list(kw["classes_2d"]), "3d": list(kw["classes_3d"])},
        "frac_gradient": kw["frac_gradient"],
        "nt_range": list(kw["nt_range"]),
        "arrival_rate_per_s": rate,
        "load": args.load,
        "max_slots": args.max_slots,
        "max_chunk": args.max_chunk,
        "solves_per_s": served["solves_per_s"],
        "requests_per_s": served["requests_per_s"],
        "p50_s": served["p50_s"],
        "p99_s": served["p99_s"],
        "makespan_s": served["makespan_s"],
        "peak_hbm_gb": served["peak_hbm_gb"],
    }
    if args.no_baseline:
        return out
    base = serve_one_at_a_time(specs, realtime=True, progress=progress("one at a time"))
    print(f"[bench] one at a time: {base['solves_per_s']:.1f} shot solves/s, p50 {base['p50_s']:.3f} s, "
          f"p99 {base['p99_s']:.3f} s", file=sys.stderr, flush=True)
    # equal accuracy: every served request equals its one-at-a-time result
    same = 0
    for r, b in zip(sorted(served["requests"], key=lambda q: q.spec.arrival), base["results"]):
        ok = all(torch.equal(x, y) for x, y in zip(r.result["traces"], b["traces"]))
        if r.spec.kind == "gradient":
            ok = ok and torch.equal(r.result["dvp"], b["dvp"])
        same += int(ok)
    out["one_at_a_time"] = {k: base[k] for k in ("solves_per_s", "requests_per_s", "p50_s", "p99_s",
                                                 "makespan_s")}
    out["speedup_solves_per_s"] = served["solves_per_s"] / base["solves_per_s"]
    # the load as measured: arrivals per second over the requests per second one
    # at a time completes on this stream (above 1: the baseline is saturated)
    out["arrival_over_one_at_a_time_rate"] = rate / base["requests_per_s"]
    out["identical_results"] = f"{same}/{len(specs)}"
    return out


def serving_bench(args):
    res = serving_run(args, args.requests)
    line = {
        "metric": "grid-point updates/s (fwd, fwd+adj), % HBM peak; served solves/s + p50/p99",
        "value": res["solves_per_s"],
        "unit": "shot solves/s (served)",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 0,
        "ms_per_step": res["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded request stream, phantoms and geometries)",
        "config": {"workload": f"serving: {WORKLOADS['serving']}",
                   **{k: res[k] for k in ("requests", "shots", "grid_classes", "nt_range",
                                          "arrival_rate_per_s", "load", "max_slots", "max_chunk",
                                          "frac_gradient")}},
        **{k: v for k, v in res.items() if k in ("p50_s", "p99_s", "requests_per_s", "peak_hbm_gb",
                                                  "one_at_a_time", "speedup_solves_per_s",
                                                  "identical_results",
                                                  "arrival_over_one_at_a_time_rate")},
        "roofline": None,
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)


def _timed(fn, steps, label=None):
    """Runs fn(i) for i < steps between two device synchronisations with the
    library's HIP-event timing on; returns (seconds, timing counters)."""
    import torch

    import paper_2110_03345_amd as S
    torch.cuda.synchronize()
    S.stride_timing_read()
    S.stride_timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        fn(i)
        if label:
            print(f"[bench] {label} {i + 1}/{steps} enqueued", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    S.stride_timing_enable(False)
    return t1 - t0, S.stride_timing_read()


def gradient_budget(args):
    """The gradient workspace budget: --budget-gb, but never more than 90 % of
    the device memory free when the bench starts (so a box with less free
    memory still runs; the line reports the workspace actually used)."""
    import torch
    global _FREE_AT_START
    if _FREE_AT_START is None:
        _FREE_AT_START = torch.cuda.mem_get_info()[0]
    return min(int(args.budget_gb * 2**30), int(0.9 * _FREE_AT_START))


_FREE_AT_START = None


def measure(name, args, dev, headline, built=None, checkpointing=0, forward=True):
    """Shot gradient and forward solve of one workload: timing of the whole
    step, and per-kernel figures from the library's HIP events.  built: the
    (workload, vp_true, vp_model) of an earlier call; checkpointing 1 forces
    binomial checkpointing."""
    import torch

    import paper_2110_03345_amd as S

    w, vp_true, vp_model = built or build_workload(name, args.nt)
    npad = w.padded_points
    print(f"[bench] {name}: padded {w.padded_shape} = {npad} points, nt={w.nt}",
          file=sys.stderr, flush=True)
    plan = S.Plan.from_workload(w, checkpointing=checkpointing)
    vp_t = torch.from_numpy(vp_true).to(dev)
    vp_m = torch.from_numpy(vp_model).to(dev)
    wav = torch.from_numpy(w.wavelet).to(dev)
    obs = plan.forward(vp_t, wav)        # observed data: forward on the phantom
    torch.cuda.synchronize()

    budget = gradient_budget(args)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    ws_bytes = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT, min(full, budget))
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    traces = torch.empty((plan.nrec, plan.nt), dtype=torch.float32, device=dev)
    misfit = torch.zeros(1, dtype=torch.float64, device=dev)
    dvp = torch.empty_like(vp_m)

    def grad_step(_):
        S.stride_plan_gradient(plan.handle, vp_m, wav, obs, traces, misfit, dvp, ws)

    steps = args.steps if headline else max(1, min(args.steps, 10))
    warm = args.warmup if headline else 1
    for _ in range(warm):
        grad_step(0)
    elapsed, (f_ms, f_n, f_l, a_ms, a_n, a_l) = _timed(
        grad_step, steps, f"{name} gradient step" if headline else None)
    ms_per_step = 1e3 * elapsed / steps
    value = 2.0 * npad * (w.nt - 1) * steps / elapsed
    adj_step_s = a_ms * 1e-3 / max(a_n, 1)
    adj_launch_s = a_ms * 1e-3 / max(a_l, 1)
    adj_spl = a_n / max(a_l, 1)
    fwd_step_s = f_ms * 1e-3 / max(f_n, 1)
    # with every state kept (full history) or segment by segment (segmented
    # history) the forward also stores v = L u + S (4 B more) and the adjoint
    # images from it two terms at a time (modes 6 and 5 in turn: 24 B per step
    # on average); with binomial checkpointing the fused adjoint (mode 0, 28 B)
    path, path_fsteps, nseg = plan.gradient_path(ws_bytes)
    full_history = path == S.STRIDE_PATH_FULL_HISTORY
    from_v = path != S.STRIDE_PATH_BINOMIAL
    adj_bytes = ADJ_BYTES_PAIRED if from_v else ADJ_BYTES
    adj_gbs = adj_bytes * npad / adj_step_s / 1e9
    # segmented: the steps before the last segment run once without v (first
    # sweep) and once with it (recomputation); every other step keeps v
    v_steps = w.nt - 1 if from_v else 0
    fwd_in_grad_bytes = (FWD_BYTES * path_fsteps + 4 * v_steps) / path_fsteps
    path_name = {S.STRIDE_PATH_FULL_HISTORY: "full history",
                 S.STRIDE_PATH_SEGMENTED: "segmented history, %d segments" % nseg,
                 S.STRIDE_PATH_BINOMIAL: "binomial checkpointing"}[path]
    print(f"[bench] {name} gradient: {ms_per_step:.2f} ms/step, adjoint {adj_step_s * 1e6:.2f} us/step "
          f"({adj_gbs:.0f} GB/s), forward {fwd_step_s * 1e6:.2f} us/step, forward steps per "
          f"gradient {f_n / steps:.0f} ({path_name})", file=sys.stderr, flush=True)
    out = {
        "w": w, "plan": plan, "vp_true": vp_true, "vp_model": vp_model, "obs": obs,
        "npad": npad, "value": value, "ms_per_step": ms_per_step, "steps": steps,
        "ws_bytes": ws_bytes, "forward_steps_per_gradient": f_n / steps,
        "recompute_factor": f_n / max(1, steps * (w.nt - 1)), "full_history": full_history,
        "gradient_path": path_name,
        "traffic_key": f"{name}/{'pair' if from_v else 'fused'}",
        "adjoint": {
            "kernel": ("adjoint leapfrog steps, imaging from the stored v two terms per even step "
                       "(step%dd_kernel<R, true, ., ., 6> and <..., 5> in turn; per-launch figures "
                       "average the pair)" % w.ndim) if from_v else
                      "adjoint leapfrog step + imaging (step%dd_kernel<R, true, ., ., 0>)" % w.ndim,
            "bytes_per_point": adj_bytes,
            "achieved": adj_gbs,
            "frac": adj_gbs / HBM_PEAK_GBS,
            "frac_at_28B": ADJ_BYTES * npad / adj_step_s / 1e9 / HBM_PEAK_GBS,
            "us_per_launch": adj_launch_s * 1e6,
            "us_per_step": adj_step_s * 1e6,
            "steps_per_launch": adj_spl,
        },
        "forward_in_gradient": {
            "bytes_per_point": fwd_in_grad_bytes,
            "us_per_step": fwd_step_s * 1e6,
            "achieved": fwd_in_grad_bytes * npad / fwd_step_s / 1e9,
        },
    }
    if forward and not args.no_forward:
        del ws
        fws = plan.workspace(S.STRIDE_MODE_FORWARD, device=dev)
        plan.forward(vp_m, wav, traces=traces, ws=fws)
        el_f, (ff_ms, ff_n, ff_l, _, _, _) = _timed(
            lambda _: plan.forward(vp_m, wav, traces=traces, ws=fws), steps)
        f_step = ff_ms * 1e-3 / max(ff_n, 1)
        out["forward"] = {
            "kernel": "forward leapfrog step (step%dd_kernel<R, false, ., ., 0>)" % w.ndim,
            "updates_per_s": npad * (w.nt - 1) * steps / el_f,
            "ms_per_solve": 1e3 * el_f / steps,
            "bytes_per_point": FWD_BYTES,
            "achieved": FWD_BYTES * npad / f_step / 1e9,
            "frac": FWD_BYTES * npad / f_step / 1e9 / HBM_PEAK_GBS,
            "us_per_launch": ff_ms * 1e3 / max(ff_l, 1),
            "us_per_step": f_step * 1e6,
        }
        del fws
        print(f"[bench] {name} forward: {out['forward']['ms_per_solve']:.2f} ms/solve, "
              f"{out['forward']['us_per_step']:.2f} us/step ({out['forward']['achieved']:.0f} GB/s)",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    return out


def variants(m, args, dev):
    """The headline workload's solves with fourth-order time, windowed-sinc
    points or a heterogeneous medium (each behind its flag)."""
    import torch

    import paper_2110_03345_amd as S
    w, plan, obs, npad = m["w"], m["plan"], m["obs"], m["npad"]
    vp_m = torch.from_numpy(m["vp_model"]).to(dev)
    vp_t = torch.from_numpy(m["vp_true"]).to(dev)
    wav = torch.from_numpy(w.wavelet).to(dev)
    traces = torch.empty((plan.nrec, plan.nt), dtype=torch.float32, device=dev)
    misfit = torch.zeros(1, dtype=torch.float64, device=dev)
    dvp = torch.empty_like(vp_m)
    budget = gradient_budget(args)
    steps = args.steps
    out = {}

    def grad_ws(p):
        full_b = p.workspace_bytes(S.STRIDE_MODE_GRADIENT)
        return torch.empty(p.workspace_bytes(S.STRIDE_MODE_GRADIENT, min(full_b, budget)),
                           dtype=torch.uint8, device=dev)

    if args.fourth_order:
        plan4 = S.Plan.from_workload(w, time_order=4)
        fws4 = plan4.workspace(S.STRIDE_MODE_FORWARD, device=dev)
        plan4.forward(vp_m, wav, traces=traces, ws=fws4)
        el, (f4_ms, f4_n, f4_l, _, _, _) = _timed(
            lambda _: plan4.forward(vp_m, wav, traces=traces, ws=fws4), steps)
        f4_step = f4_ms * 1e-3 / max(f4_n, 1)
        del fws4
        four = {
            "scheme": "leapfrog + modified-equation correction (fourth order in time); forward: two "
                      "launches per step, adjoint: three (two when p is kept: full or segmented "
                      "history)",
            "forward": {"updates_per_s": npad * (w.nt - 1) * steps / el,
                        "ms_per_solve": 1e3 * el / steps, "us_per_step": f4_step * 1e6,
                        "launches_per_step": f4_l / max(f4_n, 1), "bytes_per_point": FWD4_BYTES,
                        "gbs": FWD4_BYTES * npad / f4_step / 1e9},
        }
        ws4 = grad_ws(plan4)
        S.stride_plan_gradient(plan4.handle, vp_m, wav, obs, traces, misfit, dvp, ws4)
        el, g4 = _timed(lambda _: S.stride_plan_gradient(plan4.handle, vp_m, wav, obs, traces,
                                                         misfit, dvp, ws4), steps)
        a4_step = g4[3] * 1e-3 / max(g4[4], 1)
        # p^m kept (full or segmented history): two adjoint launches, 44 B
        kept = plan4.gradient_path(ws4.numel())[0] != S.STRIDE_PATH_BINOMIAL
        a4_bytes = ADJ4_BYTES_FULL if kept else ADJ4_BYTES
        four["gradient"] = {"updates_per_s": 2.0 * npad * (w.nt - 1) * steps / el,
                            "ms_per_solve": 1e3 * el / steps,
                            "forward_steps_per_gradient": g4[1] / steps,
                            "adjoint_us_per_step": a4_step * 1e6,
                            "adjoint_launches_per_step": g4[5] / max(g4[4], 1),
                            "adjoint_bytes_per_point": a4_bytes,
                            "adjoint_gbs": a4_bytes * npad / a4_step / 1e9}
        del ws4, plan4
        out["fourth_order"] = four
        print(f"[bench] fourth order: forward {four['forward']['ms_per_solve']:.2f} ms/solve, gradient "
              f"{four['gradient']['ms_per_solve']:.2f} ms/solve", file=sys.stderr, flush=True)

    if args.sinc:
        plan_s = S.Plan.from_workload(w, interp=1)
        ws_s = grad_ws(plan_s)
        S.stride_plan_gradient(plan_s.handle, vp_m, wav, obs, traces, misfit, dvp, ws_s)
        el, gs = _timed(lambda _: S.stride_plan_gradient(plan_s.handle, vp_m, wav, obs, traces,
                                                         misfit, dvp, ws_s), steps)
        out["sinc_taps"] = {"taps_per_point": 8 ** w.ndim,
                            "gradient_ms_per_solve": 1e3 * el / steps,
                            "updates_per_s": 2.0 * npad * (w.nt - 1) * steps / el,
                            "forward_us_per_step": gs[0] * 1e3 / max(gs[1], 1),
                            "adjoint_us_per_step": gs[3] * 1e3 / max(gs[4], 1)}
        del ws_s, plan_s
        print(f"[bench] windowed-sinc taps: gradient {out['sinc_taps']['gradient_ms_per_solve']:.2f} "
              f"ms/solve", file=sys.stderr, flush=True)

    if args.medium:
        import workloads as W
        mws = plan.workspace(S.STRIDE_MODE_FORWARD_MEDIUM, device=dev)
        med = {"bytes_per_point": medium_bytes(w.ndim)}
        for y in (0, 2):
            # y = 2 at 500 kHz: bone at 10 Np/m keeps the explicit viscous term
            # within the stability limit at the workload's dt (40 Np/m would not)
            rho, alpha0 = W.medium(m["vp_true"], w.spacing, 11, att_power=y,
                                   alpha_bone=40.0 if y == 0 else 10.0)
            rho_t, al_t = torch.from_numpy(rho).to(dev), torch.from_numpy(alpha0).to(dev)

            def run(_):
                plan.forward_medium(vp_t, wav, rho=rho_t, alpha0=al_t, att_power=y, traces=traces,
                                    ws=mws)
            run(0)
            el, (m_ms, m_n, _, _, _, _) = _timed(run, steps)
            m_step = m_ms * 1e-3 / max(m_n, 1)
            med[f"y{y}"] = {"updates_per_s": npad * (w.nt - 1) * steps / el,
                            "ms_per_solve": 1e3 * el / steps, "us_per_step": m_step * 1e6,
                            "gbs": medium_bytes(w.ndim) * npad / m_step / 1e9}
            print(f"[bench] medium y={y}: {med[f'y{y}']['ms_per_solve']:.2f} ms/solve",
                  file=sys.stderr, flush=True)
            if y == 0:
                # data for the 3D medium gradient below: the phantom in its medium
                obs_m = plan.forward_medium(vp_t, wav, rho=rho_t, alpha0=al_t, att_power=0, ws=mws)
                rho4, al4 = rho_t, al_t
            else:
                del rho_t, al_t
        del mws
        # the 3D medium shot gradient within the budget (every imaging factor
        # would take about 3000 fields): segmented history, one warm-up and one
        # timed gradient at the skull-only starting model
        torch.cuda.empty_cache()
        full_m = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT_MEDIUM)
        gws4 = plan.workspace(S.STRIDE_MODE_GRADIENT_MEDIUM, min(full_m, budget), device=dev)

        def grad4(_):
            plan.gradient_medium(vp_m, wav, obs_m, rho=rho4, alpha0=al4, att_power=0, ws=gws4)
        grad4(0)
        el, _ = _timed(grad4, 1)
        med["gradient_config4_y0"] = {"ms_per_gradient": 1e3 * el,
                                      "updates_per_s": 2.0 * npad * (w.nt - 1) / el,
                                      "workspace_gb": gws4.numel() / 2**30}
        print(f"[bench] medium gradient (config4, y=0): {1e3 * el:.2f} ms/gradient",
              file=sys.stderr, flush=True)
        del gws4, obs_m, rho4, al4
        torch.cuda.empty_cache()
        # the medium shot gradient keeps every step's imaging factor, so it is
        # timed on the 2D breast grid (1104^2, 2500 steps: 12.5 GB), at the
        # 1500 m/s model against data from the phantom in its medium, y = 0
        w2 = W.config2()
        vt2 = torch.from_numpy(w2.vp).to(dev)
        v02 = torch.full_like(vt2, 1500.0)
        wav2 = torch.from_numpy(w2.wavelet).to(dev)
        rho, alpha0 = W.medium(w2.vp, w2.spacing, 11, att_power=0)
        rho_t, al_t = torch.from_numpy(rho).to(dev), torch.from_numpy(alpha0).to(dev)
        plan2 = S.Plan.from_workload(w2)
        mws2 = plan2.workspace(S.STRIDE_MODE_FORWARD_MEDIUM, device=dev)
        obs2 = plan2.forward_medium(vt2, wav2, rho=rho_t, alpha0=al_t, att_power=0, ws=mws2)
        del mws2
        gws2 = plan2.workspace(S.STRIDE_MODE_GRADIENT_MEDIUM, device=dev)

        def grad(_):
            plan2.gradient_medium(v02, wav2, obs2, rho=rho_t, alpha0=al_t, att_power=0, ws=gws2)
        grad(0)
        el, _ = _timed(grad, steps)
        npad2 = w2.padded_points
        med["gradient_config2_y0"] = {"ms_per_gradient": 1e3 * el / steps,
                                      "updates_per_s": 2.0 * npad2 * (w2.nt - 1) * steps / el,
                                      "workspace_gb": gws2.numel() / 1e9}
        print(f"[bench] medium gradient (config2, y=0): {1e3 * el / steps:.2f} ms/gradient",
              file=sys.stderr, flush=True)
        del gws2, plan2, rho_t, al_t
        out["medium"] = med

    if args.pml:
        # forward solves with the perfectly matched layer in the padded cells
        plan_p = S.Plan.from_workload(w, boundary=1)
        fws_p = plan_p.workspace(S.STRIDE_MODE_FORWARD, device=dev)
        plan_p.forward(vp_m, wav, traces=traces, ws=fws_p)
        el, (p_ms, p_n, p_l, _, _, _) = _timed(
            lambda _: plan_p.forward(vp_m, wav, traces=traces, ws=fws_p), steps)
        p_step = p_ms * 1e-3 / max(p_n, 1)
        out["pml"] = {"boundary": "perfectly matched layer (leapfrog launch + layer correction)",
                      "updates_per_s": npad * (w.nt - 1) * steps / el,
                      "ms_per_solve": 1e3 * el / steps, "us_per_step": p_step * 1e6,
                      "launches_per_step": p_l / max(p_n, 1)}
        print(f"[bench] pml forward: {out['pml']['ms_per_solve']:.2f} ms/solve, "
              f"{out['pml']['us_per_step']:.2f} us/step", file=sys.stderr, flush=True)
        del fws_p, plan_p
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the shot-parallel multi-GPU design is described, not built)", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.workload == "serving":
        torch.cuda.set_device(0)
        return serving_bench(args)
    if args.workload == "fwi":
        torch.cuda.set_device(0)
        return fwi_bench(args)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        a = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    m = measure(args.workload, args, dev, headline=True, checkpointing=1 if args.binomial else 0)
    w, npad = m["w"], m["npad"]
    binomial = None
    if not args.binomial and not args.no_binomial and m["gradient_path"] != "full history":
        # the same gradient with binomial checkpointing in the same budget
        torch.cuda.empty_cache()
        b = measure(args.workload, args, dev, headline=False,
                    built=(w, m["vp_true"], m["vp_model"]), checkpointing=1, forward=False)
        btraffic = measured_traffic(b["traffic_key"])
        binomial = {
            "gradient_path": b["gradient_path"], "ms_per_step": b["ms_per_step"],
            "updates_per_s": b["value"], "steps": b["steps"],
            "forward_steps_per_gradient": b["forward_steps_per_gradient"],
            "recompute_factor": b["recompute_factor"], "adjoint": b["adjoint"],
            "forward_in_gradient": b["forward_in_gradient"], "traffic": btraffic,
            "traffic_over_algorithmic": (btraffic / (b["adjoint"]["bytes_per_point"] * npad))
                                        if btraffic else None,
        }
        del b
        torch.cuda.empty_cache()
    extra = variants(m, args, dev)
    obs_np = m["obs"].cpu().numpy()
    for k in ("plan", "obs"):
        m.pop(k, None)
    torch.cuda.empty_cache()

    adj = m["adjoint"]
    traffic = measured_traffic(m["traffic_key"])
    roofline = {
        "bound": "hbm",
        "kernel": adj["kernel"],
        "achieved": adj["achieved"],
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": adj["frac"],
        "traffic": traffic,
        "traffic_unit": "HBM bytes per launch",
        "traffic_over_algorithmic": (traffic / (adj["bytes_per_point"] * npad * adj["steps_per_launch"]))
                                    if traffic else None,
        "bytes_per_point": adj["bytes_per_point"],
        "algorithmic_bytes_per_launch": adj["bytes_per_point"] * npad * adj["steps_per_launch"],
        "steps_per_launch": adj["steps_per_launch"],
        "us_per_launch": adj["us_per_launch"],
        "us_per_step": adj["us_per_step"],
        "frac_at_28B": adj["frac_at_28B"],
        "forward_in_gradient": m["forward_in_gradient"],
    }
    if "forward" in m:
        ftraffic = measured_traffic(args.workload + "/forward")
        roofline["forward"] = {
            **m["forward"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "traffic": ftraffic,
            "traffic_over_algorithmic": (ftraffic / (FWD_BYTES * npad)) if ftraffic else None,
        }

    legs = {}
    if not args.no_config2 and args.workload != "config2":
        c2 = measure("config2", args, dev, headline=False)
        legs["config2"] = {
            "workload": f"config2: {WORKLOADS['config2']}",
            "updates_per_s": c2["value"], "ms_per_step": c2["ms_per_step"], "steps": c2["steps"],
            "full_history": c2["full_history"], "adjoint": c2["adjoint"],
            "forward_in_gradient": c2["forward_in_gradient"], "forward": c2.get("forward"),
        }
        del c2
        torch.cuda.empty_cache()
    if not args.no_serving:
        legs["serving"] = serving_run(args, args.leg_requests, full_mix=True)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, m["vp_model"], obs_np, args.cpu_seconds)
        print(f"[bench] cpu baseline: {cpu['value']:.3e} updates/s on {cpu['cores']} threads",
              file=sys.stderr, flush=True)

    line = {
        "metric": "grid-point updates/s (fwd, fwd+adj), % HBM peak; served solves/s + p50/p99",
        "value": m["value"],
        "unit": "grid-point updates/s (fwd+adj)",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": m["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded phantom and transducer geometry; observed data from a forward "
                "solve on the phantom)",
        "config": {
            "workload": f"{args.workload}: {WORKLOADS[args.workload]}",
            "padded_shape": list(w.padded_shape),
            "padded_points": npad,
            "nt": w.nt,
            "nrec": int(w.rec_xyz.shape[0]),
            "step": "one shot gradient (forward + residual/misfit + adjoint/imaging + finalise)",
            "workspace_gb": m["ws_bytes"] / 2**30,
            "forward_steps_per_gradient": m["forward_steps_per_gradient"],
            "recompute_factor": m["recompute_factor"],
        },
        "roofline": roofline,
        "fwd_updates_per_s": m["forward"]["updates_per_s"] if "forward" in m else None,
        "binomial": binomial,
        **legs,
        **extra,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
