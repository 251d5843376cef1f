"""Batching engine and solve server: a shot computes the same bits alone and in
any batch; every request served in a mix equals its one-at-a-time solve."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from workloads.serving_mix import materialise, request_stream

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2110_03345_amd as S
    from paper_2110_03345_amd import _abi
    from paper_2110_03345_amd.serving import Server, serve_one_at_a_time, solve_one


def _shots(maker, n, seed=0, **kw):
    base = maker(seed=seed, **kw)
    kw.pop("nt", None)
    out = []
    rng = np.random.default_rng(seed + 77)
    for i in range(n):
        nt = int(rng.integers(int(0.6 * base.nt), base.nt + 1))
        cfl = float(rng.uniform(0.25, 0.4))
        w = maker(seed=seed, nt=nt, cfl=cfl, **kw)
        ext = [(s - 1) * w.spacing for s in w.shape]
        w.src_xyz = np.stack([rng.uniform(0.2, 0.8) * e for e in ext])[None, :]
        w.wavelet = w.wavelet[:1].copy()
        out.append(w)
    return out


def _run_engine(shots, kinds, use_graphs, budget_frac=None, max_chunk=16, orders=None, fracs=None):
    """Runs the shots through one engine of 4 slots; orders / fracs: time
    order and gradient workspace fraction per shot (default 2 and full)."""
    dev = torch.device("cuda")
    w0 = shots[0]
    grid = S.make_grid(**w0.grid_kwargs())
    eng = _abi.stride_engine_create(grid, 4, 64, max_chunk, use_graphs)
    stream = torch.cuda.Stream()
    outs, keep = [], []
    pending = list(range(len(shots)))
    attached = {}
    try:
        while pending or attached:
            while pending and len(attached) < 4:
                i = pending.pop(0)
                w, kind = shots[i], kinds[i]
                plan = S.Plan.from_workload(w, time_order=orders[i] if orders else 2)
                vp = torch.from_numpy(w.vp).to(dev)
                wav = torch.from_numpy(w.wavelet).to(dev)
                tr = torch.empty((plan.nrec, w.nt), dtype=torch.float32, device=dev)
                res = {"plan": plan, "vp": vp, "wav": wav, "traces": tr}
                if kind == "forward":
                    ws = plan.workspace(S.STRIDE_MODE_FORWARD)
                    obs = mis = dvp = None
                else:
                    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
                    frac = fracs[i] if fracs else budget_frac
                    budget = int(full * frac) if frac else 0
                    ws = plan.workspace(S.STRIDE_MODE_GRADIENT, budget)
                    rng = np.random.default_rng(i)
                    obs = torch.from_numpy(
                        (1e-3 * rng.standard_normal((plan.nrec, w.nt))).astype(np.float32)).to(dev)
                    mis = torch.zeros(1, dtype=torch.float64, device=dev)
                    dvp = torch.empty_like(vp)
                torch.cuda.synchronize()
                mode = S.STRIDE_MODE_FORWARD if kind == "forward" else S.STRIDE_MODE_GRADIENT
                slot = _abi.stride_engine_attach(eng, plan.handle, mode, vp, float(w.vp.max()), wav,
                                                 obs, tr, mis, dvp, ws, stream)
                res.update(ws=ws, obs=obs, misfit=mis, dvp=dvp, i=i, kind=kind)
                attached[slot] = res
                keep.append(res)
            n, fin = _abi.stride_engine_run(eng, max_chunk, 4, stream)
            for j in fin:
                _abi.stride_engine_detach(eng, j)
                outs.append(attached.pop(j))
        stream.synchronize()
    finally:
        _abi.stride_engine_destroy(eng)
    return sorted(outs, key=lambda r: r["i"])


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
@pytest.mark.parametrize("use_graphs", [True, False])
def test_engine_slots_equal_single_shot_solves(maker, use_graphs):
    shots = _shots(maker, 6, nt=70)
    kinds = ["forward", "gradient", "forward", "gradient", "gradient", "forward"]
    outs = _run_engine(shots, kinds, use_graphs)
    for r in outs:
        plan, vp, wav = r["plan"], r["vp"], r["wav"]
        print(f"shot {r['i']} {r['kind']} nt={shots[r['i']].nt}", flush=True)
        if r["kind"] == "forward":
            ref = plan.forward(vp, wav)
            assert torch.equal(ref, r["traces"])
        else:
            tr = torch.empty_like(r["traces"])
            m, d = plan.gradient(vp, wav, r["obs"], traces=tr)
            assert torch.equal(tr, r["traces"])
            assert torch.equal(m, r["misfit"])
            assert torch.equal(d, r["dvp"])


def test_engine_checkpointed_gradients_equal_single_shot():
    shots = _shots(W.tiny_2d, 4, nt=90, seed=3)
    outs = _run_engine(shots, ["gradient"] * 4, True, budget_frac=0.12, max_chunk=8)
    for r in outs:
        m, d = r["plan"].gradient(r["vp"], r["wav"], r["obs"])
        assert torch.equal(d, r["dvp"]) and torch.equal(m, r["misfit"])


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
@pytest.mark.parametrize("use_graphs", [True, False])
def test_engine_gradient_paths_equal_single_shot(maker, use_graphs):
    """Gradient slots on every path in one engine, full history, segmented
    history (2 to 4 segments) and binomial checkpointing, chosen by their
    workspaces as the single-shot solve chooses: each equals its single-shot
    solve bit for bit (traces, misfit, dvp)."""
    shots = _shots(maker, 6, nt=80, seed=9)
    fracs = [None, 0.7, 0.45, 0.25, 0.6, 0.35]
    outs = _run_engine(shots, ["gradient"] * 6, use_graphs, max_chunk=8, fracs=fracs)
    paths = set()
    for r in outs:
        plan, vp, wav = r["plan"], r["vp"], r["wav"]
        path = plan.gradient_path(r["ws"].numel())
        paths.add(path[0])
        print(f"shot {r['i']} nt={shots[r['i']].nt} frac={fracs[r['i']]} path {path}", flush=True)
        tr = torch.empty_like(r["traces"])
        m, d = plan.gradient(vp, wav, r["obs"], traces=tr, ws=r["ws"])
        assert torch.equal(tr, r["traces"])
        assert torch.equal(m, r["misfit"])
        assert torch.equal(d, r["dvp"])
    assert {S.STRIDE_PATH_FULL_HISTORY, S.STRIDE_PATH_SEGMENTED, S.STRIDE_PATH_BINOMIAL} <= paths


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
def test_engine_fourth_order_and_mixed_slots_equal_single_shot(maker):
    """Fourth-order forward and gradient slots (full history and
    checkpointed) next to second-order ones in one engine: each equals its
    single-shot solve bit for bit."""
    shots = _shots(maker, 7, nt=64, seed=5)
    kinds = ["forward", "gradient", "gradient", "forward", "gradient", "gradient", "forward"]
    orders = [4, 4, 4, 2, 2, 4, 4]
    fracs = [None, None, 0.35, None, 0.3, 0.5, None]
    outs = _run_engine(shots, kinds, True, max_chunk=8, orders=orders, fracs=fracs)
    for r in outs:
        plan, vp, wav = r["plan"], r["vp"], r["wav"]
        print(f"shot {r['i']} {r['kind']} order {orders[r['i']]} nt={shots[r['i']].nt}", flush=True)
        if r["kind"] == "forward":
            assert torch.equal(plan.forward(vp, wav), r["traces"])
        else:
            tr = torch.empty_like(r["traces"])
            m, d = plan.gradient(vp, wav, r["obs"], traces=tr)
            assert torch.equal(tr, r["traces"])
            assert torch.equal(m, r["misfit"])
            assert torch.equal(d, r["dvp"])


def test_engine_rejects_mismatched_grid_and_full_slots():
    w = W.tiny_2d()
    grid = S.make_grid(**w.grid_kwargs())
    eng = _abi.stride_engine_create(grid, 1, 64, 8, False)
    try:
        other = W.tiny_2d(n=(40, 56))
        plan = S.Plan.from_workload(other)
        vp = torch.from_numpy(other.vp).cuda()
        wav = torch.from_numpy(other.wavelet).cuda()
        tr = torch.empty((plan.nrec, other.nt), device="cuda")
        ws = plan.workspace(S.STRIDE_MODE_FORWARD)
        with pytest.raises(S.StrideError):
            _abi.stride_engine_attach(eng, plan.handle, S.STRIDE_MODE_FORWARD, vp, 2000.0, wav,
                                      None, tr, None, None, ws)
        plan = S.Plan.from_workload(w)
        vp = torch.from_numpy(w.vp).cuda()
        wav = torch.from_numpy(w.wavelet).cuda()
        tr = torch.empty((plan.nrec, w.nt), device="cuda")
        ws = plan.workspace(S.STRIDE_MODE_FORWARD)
        _abi.stride_engine_attach(eng, plan.handle, S.STRIDE_MODE_FORWARD, vp, float(w.vp.max()),
                                  wav, None, tr, None, None, ws)
        with pytest.raises(S.StrideError):
            _abi.stride_engine_attach(eng, plan.handle, S.STRIDE_MODE_FORWARD, vp,
                                      float(w.vp.max()), wav, None, tr, None, None, ws)
        with pytest.raises(S.StrideError) as e:   # CFL checked against the given maximum
            _abi.stride_engine_detach(eng, 0)
            _abi.stride_engine_attach(eng, plan.handle, S.STRIDE_MODE_FORWARD, vp, 1e5, wav,
                                      None, tr, None, None, ws)
        assert e.value.code == -2
        torch.cuda.synchronize()
    finally:
        _abi.stride_engine_destroy(eng)


def _small_mix(n, seed):
    specs = request_stream(n, seed, rate_hz=200.0, nt_range=(60, 160), shots_range=(1, 5),
                           classes_2d=(48, 64), classes_3d=(24,))
    return [materialise(s, nrec_2d=24, nrec_3d=32) for s in specs]


@pytest.mark.parametrize("realtime", [False, True])
def test_server_results_equal_solo_solves(realtime):
    specs = _small_mix(14, seed=5)
    srv = Server(max_slots=6, max_chunk=16, use_graphs=True)
    try:
        out = srv.run(specs, realtime=realtime)
    finally:
        srv.close()
    assert len(out["requests"]) == len(specs)
    for r in out["requests"]:
        solo = solve_one(r.spec)
        res = r.result
        print(f"request {r.spec.rid} {r.spec.kind} n={r.spec.n} shots={r.spec.nshots}", flush=True)
        for a, b in zip(res["traces"], solo["traces"]):
            assert torch.equal(a, b)
        if r.spec.kind == "gradient":
            assert torch.equal(res["dvp"], solo["dvp"])
            assert res["misfit"] == solo["misfit"]
    assert out["p99_s"] >= out["p50_s"] > 0


def test_server_checkpointed_gradients_equal_solo_solves():
    """Gradient requests under a 3 MiB per-shot cap, so that no shot keeps
    every state: the 2D shots take the segmented history and the 3D ones
    (whose minimum is above the cap) binomial checkpointing, in the server's
    engine as in the one-at-a-time solves; every result is the same bits."""
    from paper_2110_03345_amd.serving import _ws_bytes
    specs = request_stream(8, 11, 200.0, nt_range=(80, 160), shots_range=(1, 3),
                           classes_2d=(48, 64), classes_3d=(24,), frac_gradient=1.0)
    specs = [materialise(s, nrec_2d=24, nrec_3d=32) for s in specs]
    cap = 3 << 20
    srv = Server(max_slots=6, max_chunk=16, use_graphs=True, grad_cap=cap)
    try:
        out = srv.run(specs, realtime=False)
    finally:
        srv.close()
    paths = set()
    for r in out["requests"]:
        g = S.make_grid(r.spec.shape, r.spec.spacing, r.spec.space_order, r.spec.nb, r.spec.vref,
                        r.spec.dt, r.spec.nt)
        nrec = r.spec.rec_xyz.shape[0]
        path = S.stride_gradient_path(g, nrec, _ws_bytes(g, nrec, "gradient", cap))
        paths.add(path[0])
        print(f"request {r.spec.rid} shape {r.spec.shape} nt={r.spec.nt} shots={r.spec.nshots} "
              f"path {path}", flush=True)
        solo = solve_one(r.spec, grad_cap=cap)
        for a, b in zip(r.result["traces"], solo["traces"]):
            assert torch.equal(a, b)
        assert torch.equal(r.result["dvp"], solo["dvp"])
        assert r.result["misfit"] == solo["misfit"]
    assert {S.STRIDE_PATH_SEGMENTED, S.STRIDE_PATH_BINOMIAL} <= paths


def test_server_io_limit_overrun_path():
    """An I/O limit too small for any shot: a shot is admitted only when no
    shot runs anywhere (one beyond the limit at a time), every request still
    completes, and each result equals its one-at-a-time solve."""
    specs = _small_mix(8, seed=21)
    srv = Server(max_slots=6, max_chunk=16, use_graphs=True, io_limit=1)
    try:
        out = srv.run(specs, realtime=False)
    finally:
        srv.close()
    assert len(out["requests"]) == len(specs)
    assert out["max_attached_shots"] == 1     # one shot beyond the limit at a time

    def shot_io(sp):
        grad = sp.kind == "gradient"
        return sp.rec_xyz.shape[0] * sp.nt * 4 * (2 if grad else 1) + (sp.vp.nbytes if grad else 0)

    # the overrun: staged inputs, plus the outputs of the request being admitted
    # and of the one before it, whose shots stay counted until it completes
    staged = sum(r.spec.vp.nbytes + r.spec.wavelet.nbytes for r in out["requests"])
    per_req = sorted((shot_io(r.spec) * r.spec.nshots for r in out["requests"]), reverse=True)
    assert 1 < out["io_peak_bytes"] <= 1 + staged + per_req[0] + per_req[1]
    for r in out["requests"]:
        solo = solve_one(r.spec)
        for a, b in zip(r.result["traces"], solo["traces"]):
            assert torch.equal(a, b)
        if r.spec.kind == "gradient":
            assert torch.equal(r.result["dvp"], solo["dvp"])


def test_served_requests_match_the_oracle():
    """Sampled requests of a served mix (one forward, one gradient, each of
    several shots) against the FP64 oracle."""
    import oracle
    specs = _small_mix(10, seed=11)
    srv = Server(max_slots=6, max_chunk=16, use_graphs=True)
    try:
        out = srv.run(specs, realtime=False)
    finally:
        srv.close()
    checked = set()
    for r in sorted(out["requests"], key=lambda q: q.spec.rid):
        sp = r.spec
        if sp.kind in checked:
            continue
        checked.add(sp.kind)
        print(f"oracle check: request {sp.rid} {sp.kind} n={sp.n} shots={sp.nshots}", flush=True)
        g = oracle.Grid(**sp.grid_kwargs())
        J, dvp = 0.0, np.zeros(sp.shape)
        for i in range(sp.nshots):
            src = sp.src_xyz[i:i + 1]
            if sp.kind == "forward":
                ref = oracle.forward(g, sp.vp, src, sp.wavelet, sp.rec_xyz)
                got = r.result["traces"][i].cpu().numpy()
                assert np.linalg.norm(got - ref) <= 1e-4 * np.linalg.norm(ref)
            else:
                _, j, d = oracle.gradient(g, sp.vp, src, sp.wavelet, sp.rec_xyz, sp.observed[i])
                J += j
                dvp += d
        if sp.kind == "gradient":
            got = r.result["dvp"].cpu().numpy()
            assert np.linalg.norm(got - dvp) <= 1e-4 * np.linalg.norm(dvp)
            assert abs(r.result["misfit"] - J) <= 1e-4 * J
    assert checked == {"forward", "gradient"}


def test_server_respects_the_hbm_budget():
    specs = _small_mix(8, seed=9)
    srv = Server(hbm_budget=64 << 20, max_slots=8, max_chunk=16)
    try:
        out = srv.run(specs, realtime=False)
    finally:
        srv.close()
    assert out["workspace_peak_bytes"] <= out["workspace_budget_bytes"] <= 64 << 20
    base = serve_one_at_a_time(specs, realtime=False)
    for r, b in zip(sorted(out["requests"], key=lambda q: q.spec.arrival), base["results"]):
        for x, y in zip(r.result["traces"], b["traces"]):
            assert torch.equal(x, y)
