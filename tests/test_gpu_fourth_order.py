"""Fourth-order time (leapfrog with the modified-equation correction and the
time-filtered source): HIP forward traces and gradients against the FP64
oracle's, at the workloads' CFL and near the larger stability limit of the
corrected scheme; the CFL check of each order; checkpointing invisible in the
gradient; the wavelet gradient and the FP32 dot product; the autograd operator."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2110_03345_amd as S


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _at_cfl(w, cfl):
    """The workload with dt set to cfl * dx / vmax (wavelet resampled)."""
    w.dt = cfl * min(np.atleast_1d(w.spacing)) / float(w.vp.max())
    w.wavelet = (W.tone_burst(w.nt, w.dt, f0=1.0e6, nsrc=w.wavelet.shape[0])).astype(np.float32)
    return w


CASES = [
    ("2d_o8", lambda: W.tiny_2d()),
    ("2d_o10_ragged", lambda: W.tiny_2d(space_order=10, n=(83, 141), nb=7, nt=150)),
    ("2d_o8_cfl085", lambda: _at_cfl(W.tiny_2d(nt=200), 0.85)),
    ("3d_o10", lambda: W.tiny_3d()),
    ("3d_o8_ragged", lambda: W.tiny_3d(space_order=8, n=(37, 21, 70), nb=4, nt=70)),
    ("3d_o10_cfl07", lambda: _at_cfl(W.tiny_3d(nt=90), 0.7)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_fourth_order_forward_matches_oracle(name, make):
    w = make()
    print(f"fourth order {name}: shape={w.shape} nt={w.nt} dt={w.dt:.3e}", flush=True)
    g = oracle.Grid(**w.grid_kwargs(), time_order=4)
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    plan = S.Plan.from_workload(w, time_order=4)
    tr = plan.forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    assert rel(tr, ref) < 1e-4, rel(tr, ref)


def test_config1_fourth_order_matches_oracle():
    w = W.config1()
    g = oracle.Grid(**w.grid_kwargs(), time_order=4)
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = S.Plan.from_workload(w, time_order=4).forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    assert rel(tr, ref) < 1e-4, rel(tr, ref)


def test_stability_limit_per_order():
    """dt at 0.85 dx/v (2D, order 8): past the leapfrog limit (0.555), within
    the corrected scheme's (0.961)."""
    w = _at_cfl(W.tiny_2d(nt=50), 0.85)
    vp, wav = dev(w.vp), dev(w.wavelet)
    S.Plan.from_workload(w, time_order=4).forward(vp, wav)
    with pytest.raises(S.StrideError) as e:
        S.Plan.from_workload(w, time_order=2).forward(vp, wav)
    assert e.value.code == -2


GRAD_CASES = [
    ("2d_o8", lambda: W.tiny_2d()),
    ("2d_o10_ragged", lambda: W.tiny_2d(space_order=10, n=(83, 141), nb=7, nt=150)),
    ("2d_o8_cfl085", lambda: _at_cfl(W.tiny_2d(nt=160), 0.85)),
    ("3d_o10", lambda: W.tiny_3d()),
    ("3d_o8_ragged", lambda: W.tiny_3d(space_order=8, n=(37, 21, 70), nb=4, nt=70)),
]


@pytest.mark.parametrize("name,make", GRAD_CASES, ids=[c[0] for c in GRAD_CASES])
def test_fourth_order_gradient_matches_oracle(name, make):
    w = make()
    print(f"fourth-order gradient {name}: shape={w.shape} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs(), time_order=4)
    rng = np.random.default_rng(7)
    obs = oracle.forward(g, w.vp * (1 + 0.02 * rng.standard_normal(w.shape).clip(-2, 2)),
                         w.src_xyz, w.wavelet, w.rec_xyz).astype(np.float32)
    tr_ref, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    plan = S.Plan.from_workload(w, time_order=4)
    tr = torch.empty((plan.nrec, w.nt), dtype=torch.float32, device="cuda")
    misfit, dvp = plan.gradient(dev(w.vp), dev(w.wavelet), dev(obs), traces=tr)
    assert rel(tr.cpu().numpy(), tr_ref) < 1e-4
    assert abs(misfit.item() - J) <= 1e-4 * abs(J)
    assert rel(dvp.cpu().numpy(), dvp_ref) < 1e-4, rel(dvp.cpu().numpy(), dvp_ref)


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
def test_fourth_order_backward_vjp_matches_oracle(maker):
    w = maker()
    g = oracle.Grid(**w.grid_kwargs(), time_order=4)
    plan = S.Plan.from_workload(w, time_order=4)
    rng = np.random.default_rng(3)
    gt = rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32)
    dvp_ref, dwav_ref = oracle.adjoint(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, gt)
    ws = plan.workspace(S.STRIDE_MODE_GRADIENT)
    vp, wav = dev(w.vp), dev(w.wavelet)
    plan.forward_save(vp, wav, ws)
    dvp, _ = plan.backward(vp, wav, dev(gt), ws)
    assert rel(dvp.cpu().numpy(), dvp_ref) < 1e-4, rel(dvp.cpu().numpy(), dvp_ref)
    plan.forward_save(vp, wav, ws)
    dvp2, dwav = plan.backward(vp, wav, dev(gt), ws, want_dwavelet=True)
    assert torch.equal(dvp, dvp2)
    assert rel(dwav.cpu().numpy(), dwav_ref) < 1e-4, rel(dwav.cpu().numpy(), dwav_ref)


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
def test_fourth_order_dot_product_fp32(maker):
    """<F s, d> = <s, F^T d> for the fourth-order wavelet -> traces map on the GPU."""
    w = maker()
    plan = S.Plan.from_workload(w, time_order=4)
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
def test_fourth_order_checkpointing_is_bitwise_invisible(maker, kw):
    w = maker(**kw)
    plan = S.Plan.from_workload(w, time_order=4)
    rng = np.random.default_rng(5)
    obs = dev(rng.standard_normal((w.rec_xyz.shape[0], w.nt)).astype(np.float32) * 1e-3)
    vp, wav = dev(w.vp), dev(w.wavelet)
    m0, g0 = plan.gradient(vp, wav, obs)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    for frac in (0.5, 0.25):
        budget = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT, int(full * frac))
        assert budget < full
        print(f"budget {budget} of {full}", flush=True)
        m1, g1 = plan.gradient(vp, wav, obs, budget_bytes=budget)
        assert torch.equal(g0, g1) and torch.equal(m0, m1)


def test_fourth_order_autograd_matches_oracle():
    from paper_2110_03345_amd.autograd import wave_traces
    w = W.tiny_2d(nt=120)
    g = oracle.Grid(**w.grid_kwargs(), time_order=4)
    plan = S.Plan.from_workload(w, time_order=4)
    rng = np.random.default_rng(9)
    obs = (0.5 * oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
           + 1e-3 * rng.standard_normal((w.rec_xyz.shape[0], w.nt))).astype(np.float32)
    _, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    vp = dev(w.vp).requires_grad_(True)
    tr = wave_traces(vp, dev(w.wavelet), plan, plan.workspace_bytes(S.STRIDE_MODE_GRADIENT) // 2)
    loss = 0.5 * ((tr.double() - dev(obs).double()) ** 2).sum()
    loss.backward()
    assert abs(loss.item() - J) <= 1e-4 * abs(J)
    assert rel(vp.grad.cpu().numpy(), dvp_ref) < 1e-4
    # the wavelet gradient through the operator against the oracle's VJP of its
    # own residual
    wav = dev(w.wavelet).requires_grad_(True)
    tr = wave_traces(dev(w.vp), wav, plan)
    (0.5 * ((tr.double() - dev(obs).double()) ** 2).sum()).backward()
    res_ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz) - obs
    _, dwav_ref = oracle.adjoint(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, res_ref)
    assert rel(wav.grad.cpu().numpy(), dwav_ref) < 1e-4
