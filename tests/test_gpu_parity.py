"""HIP path vs the FP64 oracle, through the C ABI.

Tolerances (relative L2 over the whole output): 1e-4 for solves of at most
1000 steps and 1e-3 for at most 3000 steps; the FP32 kernel and the FP64
oracle differ only by rounding, which grows with the number of steps.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_field, check_traces

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2110_03345_amd as S


def tol_for(nt):
    return 1e-4 if nt <= 1000 else 1e-3


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _case(maker, order, **kw):
    w = maker(space_order=order, **kw)
    return w, oracle.Grid(**w.grid_kwargs()), S.Plan.from_workload(w)


CASES = [
    ("2d_o8", W.tiny_2d, 8, {}),
    ("2d_o10", W.tiny_2d, 10, {}),
    ("2d_o8_ragged", W.tiny_2d, 8, dict(n=(83, 141), nb=7, nt=150)),
    ("3d_o10", W.tiny_3d, 10, {}),
    ("3d_o8", W.tiny_3d, 8, {}),
    ("3d_o10_ragged", W.tiny_3d, 10, dict(n=(37, 21, 70), nb=4, nt=70)),
]


@pytest.mark.parametrize("name,maker,order,kw", CASES, ids=[c[0] for c in CASES])
def test_forward_matches_oracle(name, maker, order, kw):
    w, g, plan = _case(maker, order, **kw)
    print(f"case {name} shape={w.shape} nt={w.nt}", flush=True)
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = plan.forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    assert np.all(tr[:, 0] == 0.0)
    print(check_traces(tr, ref, tol_for(w.nt)), flush=True)


@pytest.mark.parametrize("name,maker,order,kw", CASES, ids=[c[0] for c in CASES])
def test_gradient_matches_oracle(name, maker, order, kw):
    w, g, plan = _case(maker, order, **kw)
    print(f"case {name} shape={w.shape} nt={w.nt}", flush=True)
    rng = np.random.default_rng(7)
    obs = oracle.forward(g, w.vp * (1 + 0.02 * rng.standard_normal(w.shape).clip(-2, 2)),
                         w.src_xyz, w.wavelet, w.rec_xyz).astype(np.float32)
    _, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    misfit, dvp = plan.gradient(dev(w.vp), dev(w.wavelet), dev(obs))
    assert abs(misfit.item() - J) <= tol_for(w.nt) * abs(J)
    print(check_field(dvp.cpu().numpy(), dvp_ref, tol_for(w.nt)), flush=True)


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
def test_backward_vjp_matches_oracle(maker):
    w = maker()
    g = oracle.Grid(**w.grid_kwargs())
    plan = S.Plan.from_workload(w)
    rng = np.random.default_rng(3)
    gt = rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32)
    dvp_ref, dwav_ref = oracle.adjoint(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, gt)
    ws = plan.workspace(S.STRIDE_MODE_GRADIENT)
    vp, wav = dev(w.vp), dev(w.wavelet)
    plan.forward_save(vp, wav, ws)
    dvp, dwav = plan.backward(vp, wav, dev(gt), ws, want_dwavelet=True)
    assert rel(dvp.cpu().numpy(), dvp_ref) < 1e-4
    assert rel(dwav.cpu().numpy(), dwav_ref) < 1e-4


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
def test_dot_product_fp32(maker):
    """<F s, d> = <s, F^T d> for the wavelet -> traces map on the GPU."""
    w = maker()
    plan = S.Plan.from_workload(w)
    rng = np.random.default_rng(12)
    s = rng.standard_normal(w.wavelet.shape).astype(np.float32)
    d = rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32)
    vp, sd = dev(w.vp), dev(s)
    ws = plan.workspace(S.STRIDE_MODE_GRADIENT)
    Fs = plan.forward_save(vp, sd, ws).cpu().numpy().astype(np.float64)
    _, FTd = plan.backward(vp, sd, dev(d), ws, want_dwavelet=True)
    lhs = np.sum(Fs * d)
    rhs = np.sum(s.astype(np.float64) * FTd.cpu().numpy())
    assert abs(lhs - rhs) <= 1e-5 * max(abs(lhs), abs(rhs)), (lhs, rhs)


@pytest.mark.parametrize("maker,kw", [(W.tiny_2d, dict(nt=90)), (W.tiny_3d, dict(nt=50))])
def test_checkpointing_is_bitwise_invisible(maker, kw):
    """The gradient is the same bits with every state kept and with binomial
    checkpointing at several budgets; repeated runs are bitwise identical."""
    w = maker(**kw)
    plan = S.Plan.from_workload(w)
    rng = np.random.default_rng(5)
    obs = dev(rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32) * 1e-3)
    vp, wav = dev(w.vp), dev(w.wavelet)
    m0, g0 = plan.gradient(vp, wav, obs)
    m1, g1 = plan.gradient(vp, wav, obs)
    assert torch.equal(g0, g1) and torch.equal(m0, m1)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    fixed = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT, 1 << 62) - 0  # == full
    assert fixed == full
    field_est = (full - plan.workspace_bytes(S.STRIDE_MODE_GRADIENT, full // 2)) > 0
    assert field_est
    for frac in (0.5, 0.2, 0.08):
        budget = int(full * frac)
        try:
            ws = plan.workspace(S.STRIDE_MODE_GRADIENT, budget)
        except S.StrideError:
            continue
        m2, g2 = plan.gradient(vp, wav, obs, ws=ws)
        assert torch.equal(g0, g2), frac
        assert torch.equal(m0, m2)


@pytest.mark.parametrize("maker,kw,order", [
    (W.tiny_2d, dict(nt=90), 2), (W.tiny_2d, dict(nt=91), 2),
    (W.tiny_3d, dict(nt=50), 2), (W.tiny_3d, dict(nt=51), 2),
    (W.tiny_2d, dict(nt=91), 4), (W.tiny_3d, dict(nt=50), 4)])
def test_gradient_paths_give_the_same_bits(maker, kw, order):
    """Full history, segmented history and binomial checkpointing (the same
    workspace, checkpointing = 1 forcing the last) give the same bits: the
    gradient with its misfit, and the split forward / backward with the
    wavelet cotangent; both parities of nt, several segment counts, second-
    and fourth-order time."""
    w = maker(**kw)
    plan = S.Plan.from_workload(w, time_order=order)
    plan_b = S.Plan.from_workload(w, time_order=order, checkpointing=1)
    rng = np.random.default_rng(7)
    obs = dev(rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32) * 1e-3)
    gtr = dev(rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32))
    vp, wav = dev(w.vp), dev(w.wavelet)

    def vjp(p, ws):
        tr = torch.empty((p.nrec, p.nt), dtype=torch.float32, device="cuda")
        S.stride_forward_save(p.handle, vp, wav, tr, ws)
        dvp, dw = torch.empty_like(vp), torch.zeros_like(wav)
        S.stride_backward(p.handle, vp, wav, gtr, dvp, dw, ws)
        return tr, dvp, dw

    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    ws_full = plan.workspace(S.STRIDE_MODE_GRADIENT)
    m0, g0 = plan.gradient(vp, wav, obs, ws=ws_full)
    v0 = vjp(plan, ws_full)
    seen = set()
    for frac in (0.7, 0.45, 0.25):
        ws = plan.workspace(S.STRIDE_MODE_GRADIENT, int(full * frac))
        path = plan.gradient_path(ws.numel())
        seen.add(path[0])
        print(f"{w.shape} nt={w.nt} frac={frac}: path {path}", flush=True)
        for p in (plan, plan_b):
            m1, g1 = p.gradient(vp, wav, obs, ws=ws)
            assert torch.equal(m0, m1) and torch.equal(g0, g1), (frac, p.grid.checkpointing)
            v1 = vjp(p, ws)
            assert all(torch.equal(a, b) for a, b in zip(v0, v1)), (frac, p.grid.checkpointing)
        del ws
    assert S.STRIDE_PATH_SEGMENTED in seen


def _dense_geometry(w, nsrc, nrec, seed):
    """Sources and receivers packed into a few cells around one point: one
    step-kernel block gets more injection entries than it has threads, some
    points get several entries (duplicated positions) and some taps have
    zero weight (positions on grid nodes)."""
    rng = np.random.default_rng(seed)
    nd = len(w.shape)
    c = np.array([(s // 2) * w.spacing for s in w.shape])
    def cluster(n, cells):
        p = c + rng.uniform(-cells, cells, size=(n, nd)) * w.spacing
        k = n // 6
        p[k:2 * k] = p[:k]                                         # duplicates
        p[2 * k:3 * k] = np.round(p[2 * k:3 * k] / w.spacing) * w.spacing   # on nodes
        return p
    w.src_xyz = cluster(nsrc, 3.0)
    w.rec_xyz = cluster(nrec, 4.0)
    wav = np.repeat(w.wavelet[:1], nsrc, axis=0)
    w.wavelet = (wav * rng.uniform(0.5, 1.5, size=(nsrc, 1))).astype(np.float32)
    return w


@pytest.mark.parametrize("maker,nsrc,nrec", [(W.tiny_2d, 150, 300), (W.tiny_3d, 40, 120)])
def test_dense_geometry_matches_oracle(maker, nsrc, nrec):
    w = _dense_geometry(maker(nsrc=1), nsrc, nrec, seed=21)
    g = oracle.Grid(**w.grid_kwargs())
    plan = S.Plan.from_workload(w)
    print(f"dense geometry {w.shape}: {nsrc} sources, {nrec} receivers", flush=True)
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = plan.forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    assert rel(tr, ref) < 1e-4, rel(tr, ref)
    # residual of the size of the traces: with observed data within a few per
    # cent of the traces, FP32 traces - observed would lose the digits this
    # test is about (the cancellation, not the injection, would be measured)
    rng = np.random.default_rng(8)
    obs = (0.5 * ref + np.std(ref) * rng.standard_normal(ref.shape)).astype(np.float32)
    _, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    misfit, dvp = plan.gradient(dev(w.vp), dev(w.wavelet), dev(obs))
    assert abs(misfit.item() - J) <= 1e-4 * abs(J)
    assert rel(dvp.cpu().numpy(), dvp_ref) < 1e-4, rel(dvp.cpu().numpy(), dvp_ref)


def _aniso(w, factors):
    w.spacing = tuple(w.spacing * f for f in factors)   # larger spacing: still inside, still stable
    return w


EDGE_CASES = [
    ("one_step", lambda: W.tiny_2d(nt=2)),
    ("grid_smaller_than_stencil_2d", lambda: W.tiny_2d(n=(5, 3), nb=0, nt=40)),
    ("grid_smaller_than_stencil_3d", lambda: W.tiny_3d(n=(3, 4, 5), nb=0, nt=30)),
    ("anisotropic_2d", lambda: _aniso(W.tiny_2d(), (1.0, 1.3))),
    ("anisotropic_3d", lambda: _aniso(W.tiny_3d(), (1.0, 1.2, 1.4))),
]


@pytest.mark.parametrize("name,make", EDGE_CASES, ids=[c[0] for c in EDGE_CASES])
def test_edge_cases_match_oracle(name, make):
    w = make()
    print(f"edge case {name}: shape={w.shape} spacing={w.spacing} nb={w.nb} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs())
    plan = S.Plan.from_workload(w)
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = plan.forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    if np.linalg.norm(ref) == 0:
        assert np.all(tr == 0)
    else:
        assert rel(tr, ref) < 1e-4, rel(tr, ref)
    rng = np.random.default_rng(6)
    obs = (0.5 * ref + 1e-3 * rng.standard_normal(ref.shape)).astype(np.float32)
    _, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    misfit, dvp = plan.gradient(dev(w.vp), dev(w.wavelet), dev(obs))
    assert abs(misfit.item() - J) <= 1e-4 * abs(J)
    if np.linalg.norm(dvp_ref) == 0:
        assert np.all(dvp.cpu().numpy() == 0)
    else:
        assert rel(dvp.cpu().numpy(), dvp_ref) < 1e-4, rel(dvp.cpu().numpy(), dvp_ref)


@pytest.mark.parametrize("empty", ["receivers", "sources"])
def test_empty_geometry(empty):
    """No receivers: empty traces, zero misfit and gradient.  No sources: the
    field stays zero, so traces and gradient are zero."""
    w = W.tiny_2d()
    if empty == "receivers":
        w.rec_xyz = np.zeros((0, 2))
    else:
        w.src_xyz = np.zeros((0, 2))
        w.wavelet = np.zeros((0, w.nt), dtype=np.float32)
    plan = S.Plan.from_workload(w)
    vp, wav = dev(w.vp), dev(w.wavelet)
    tr = plan.forward(vp, wav)
    assert tuple(tr.shape) == (w.rec_xyz.shape[0], w.nt)
    assert torch.count_nonzero(tr).item() == 0
    obs = torch.zeros_like(tr)
    misfit, dvp = plan.gradient(vp, wav, obs)
    assert misfit.item() == 0.0
    assert torch.count_nonzero(dvp).item() == 0


def test_config1_forward_matches_oracle():
    w = W.config1()
    g = oracle.Grid(**w.grid_kwargs())
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = S.Plan.from_workload(w).forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    assert rel(tr, ref) < tol_for(w.nt), rel(tr, ref)


def test_errors_are_reported_before_launch():
    w = W.tiny_2d()
    plan = S.Plan.from_workload(w)
    vp = dev(w.vp * 3.0)       # violates the CFL limit at this dt
    with pytest.raises(S.StrideError) as e:
        plan.forward(vp, dev(w.wavelet))
    assert e.value.code == -2
    bad = w.vp.copy()
    bad[3, 4] = np.nan
    with pytest.raises(S.StrideError) as e:
        plan.forward(dev(bad), dev(w.wavelet))
    assert e.value.code == -1
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(S.StrideError) as e:
        plan.forward(dev(w.vp), dev(w.wavelet), ws=small)
    assert e.value.code == -4


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
@pytest.mark.parametrize("nt", [41, 42])
def test_full_history_path_both_step_parities(maker, nt):
    """The full-history gradient (v stored, imaging terms added in pairs) gives
    the checkpointed path's bits whether the first adjoint step images (nt - 1
    even) or not (nt - 1 odd), and both match the oracle."""
    w = maker(nt=nt)
    g = oracle.Grid(**w.grid_kwargs())
    plan = S.Plan.from_workload(w)
    rng = np.random.default_rng(nt)
    obs = (1e-3 * rng.standard_normal((w.rec_xyz.shape[0], w.nt))).astype(np.float32)
    vp, wav, ob = dev(w.vp), dev(w.wavelet), dev(obs)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    m0, g0 = plan.gradient(vp, wav, ob)
    small = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT, full // 3)
    assert small < full
    m1, g1 = plan.gradient(vp, wav, ob, budget_bytes=small)
    assert torch.equal(g0, g1) and torch.equal(m0, m1)
    _, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    assert abs(m0.item() - J) <= 1e-4 * abs(J)
    assert rel(g0.cpu().numpy(), dvp_ref) < 1e-4


def test_nonfinite_outputs_are_reported():
    """A NaN in the wavelet or an infinity in the observed data makes the
    outputs non-finite: the solve returns STRIDE_E_NONFINITE naming them
    (with the check switched off it returns normally)."""
    w = W.tiny_2d(nt=60)
    plan = S.Plan.from_workload(w)
    vp = dev(w.vp)
    bad_wav = w.wavelet.copy()
    bad_wav[0, 5] = np.nan
    with pytest.raises(S.StrideError) as e:
        plan.forward(vp, dev(bad_wav))
    assert e.value.code == -6 and "traces" in str(e.value)
    obs = np.zeros((w.rec_xyz.shape[0], w.nt), dtype=np.float32)
    obs[1, 7] = np.inf
    with pytest.raises(S.StrideError) as e:
        plan.gradient(vp, dev(w.wavelet), dev(obs))
    assert e.value.code == -6 and "misfit" in str(e.value) and "dvp" in str(e.value)
    assert "traces" not in str(e.value)
    S.stride_check_finite(False)
    try:
        tr = plan.forward(vp, dev(bad_wav))
        torch.cuda.synchronize()
        assert torch.isnan(tr).any()
    finally:
        S.stride_check_finite(True)
    ok = plan.forward(vp, dev(w.wavelet))
    assert torch.isfinite(ok).all()
