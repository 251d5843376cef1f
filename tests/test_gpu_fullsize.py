"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (default tile shapes and chunk lengths).

- 2D breast-like shot gradient (1104^2 padded, 2500 steps, every forward
  state kept: the forward stores v = L u + S and the adjoint images from it)
  against the FP64 oracle run here, with observed data from the oracle's
  forward on the phantom (rounded to FP32): misfit, dvp over the whole grid,
  its interior and its edge strip, and every receiver's trace.
- 3D head-like forward (316^3 padded, all 3000 steps) against the oracle's
  traces stored in tests/golden/config4_forward.npz by
  tests/golden/make_config4_golden.py: 64 sampled receivers sample by sample,
  and the norm and peak of every one of the 1024 traces.
- 3D shot gradient (316^3, first 1000 steps, observed data zero), checkpointed
  with the ratio of stored wavefields to steps of a 200 GiB budget (1676 for
  3000; the library takes the segmented history there, and binomial
  checkpointing forced in the same workspace gives the same bits),
  against tests/golden/config4_gradient.npz: misfit, dvp on the plane of
  largest norm of each axis (through the source) and on the physical face of
  axis 0 nearest the source (where the padding transpose adds the layer), and
  its norms over every plane, the interior and the edge strip.

Tolerances (relative L2): 1e-4 up to 1000 steps, 1e-3 up to 3000.
"""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_field, check_traces, rel

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2110_03345_amd as S

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_config2_full_history_gradient_matches_oracle():
    w = W.config2()
    vp0 = np.full(w.shape, 1500.0, dtype=np.float32)
    print(f"config2 gradient {w.padded_shape} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs())
    obs = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz).astype(np.float32)
    tr_ref, J, dvp_ref = oracle.gradient(g, vp0, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    plan = S.Plan.from_workload(w)
    traces = torch.empty((plan.nrec, plan.nt), dtype=torch.float32, device="cuda")
    misfit, dvp = plan.gradient(dev(vp0), dev(w.wavelet), dev(obs), traces=traces)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    assert S.stride_schedule_info(w.nt, 10**6)[1] == w.nt - 1 and full > 0
    e_J = abs(misfit.item() - J) / J
    st = check_traces(traces.cpu().numpy(), tr_ref, 1e-3)
    sf = check_field(dvp.cpu().numpy(), dvp_ref, 1e-3)
    print(f"config2 misfit rel {e_J:.2e}; traces {st}; dvp {sf}", flush=True)
    assert e_J < 1e-3


def test_config4_full_forward_matches_golden():
    ref = np.load(os.path.join(GOLDEN, "config4_forward.npz"))
    w = W.config4()
    print(f"config4 forward {w.padded_shape} nt={w.nt}", flush=True)
    tr = S.Plan.from_workload(w).forward(dev(w.vp_true), dev(w.wavelet)).cpu().numpy()
    tr = tr.astype(np.float64)
    rec = ref["receivers"]
    st = check_traces(tr[rec], ref["traces"], 1e-3)
    norms = np.linalg.norm(tr, axis=1)
    strong = ref["norms"] >= 1e-3 * ref["norms"].max()
    e_norm = np.abs(norms - ref["norms"])[strong] / ref["norms"][strong]
    e_peak = np.abs(np.abs(tr).max(axis=1) - ref["peak"])[strong] / ref["peak"][strong]
    print(f"config4 sampled traces {st}; norms worst {e_norm.max():.2e}, peaks worst "
          f"{e_peak.max():.2e} over {int(strong.sum())} receivers", flush=True)
    assert e_norm.max() < 1e-2 and e_peak.max() < 1e-2


def test_config4_checkpointed_gradient_matches_golden():
    ref = np.load(os.path.join(GOLDEN, "config4_gradient.npz"))
    w = W.config4(nt=1000)
    plan = S.Plan.from_workload(w)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    ws = plan.workspace(S.STRIDE_MODE_GRADIENT, int(full * 1676 / 3000))
    print(f"config4 gradient {w.padded_shape} nt={w.nt}, workspace {ws.numel() / 2**30:.1f} GiB "
          f"of {full / 2**30:.1f}", flush=True)
    obs = torch.zeros((plan.nrec, plan.nt), dtype=torch.float32, device="cuda")
    S.stride_timing_read()
    S.stride_timing_enable(True)
    misfit, dvp = plan.gradient(dev(w.vp_start), dev(w.wavelet), obs, ws=ws)
    torch.cuda.synchronize()
    S.stride_timing_enable(False)
    fwd_steps = S.stride_timing_read()[1]
    assert fwd_steps > w.nt - 1, "the gradient did not checkpoint"
    # the same workspace with binomial checkpointing forced: the same bits
    path = plan.gradient_path(ws.numel())
    plan_b = S.Plan.from_workload(w, checkpointing=1)
    misfit_b, dvp_b = plan_b.gradient(dev(w.vp_start), dev(w.wavelet), obs, ws=ws)
    assert torch.equal(misfit, misfit_b) and torch.equal(dvp, dvp_b), path
    d = dvp.cpu().numpy().astype(np.float64)
    tol = 1e-4
    e_J = abs(misfit.item() - float(ref["misfit"])) / float(ref["misfit"])
    total = float(ref["norm_all"])
    errs = {}
    for i, (a, k) in enumerate(zip(ref["slice_axes"], ref["slice_index"])):
        want = ref[f"slice_{i}"].astype(np.float64)
        diff = np.linalg.norm(np.take(d, int(k), axis=int(a)) - want)
        # a plane holding at least 1 % of the gradient's norm is bounded relative to
        # its own norm, a weaker one relative to one hundredth of the whole
        scale = max(np.linalg.norm(want), 1e-2 * total)
        errs[f"axis {a} plane {k}"] = diff / scale
    print(f"config4 gradient: {fwd_steps} forward steps, misfit rel {e_J:.2e}, planes {errs}", flush=True)
    assert e_J < tol
    for k, e in errs.items():
        assert e < 3 * tol, (k, e)
    from parity import regions
    inner, edge = regions(w.shape)
    for name, got in (("norm_all", np.linalg.norm(d)), ("norm_interior", np.linalg.norm(d[inner])),
                      ("norm_edge", np.linalg.norm(d[edge]))):
        assert abs(got - float(ref[name])) < tol * float(ref[name]), name
    for a in range(3):
        axes = tuple(x for x in range(3) if x != a)
        got = np.linalg.norm(d, axis=axes)
        want = ref[f"norms_a{a}"]
        strong = want >= 1e-3 * want.max()
        assert (np.abs(got - want)[strong] / want[strong]).max() < 3 * tol, a
