"""The autograd form: torch losses on HIP traces, gradients from the adjoint
kernel, checked against the oracle, the fused gradient entry point and finite
differences of the misfit."""
import numpy as np
import pytest

import oracle
import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2110_03345_amd as S
    from paper_2110_03345_amd.autograd import StrideWave, WavePropagator, wave_traces


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def _setup(maker=None, **kw):
    w = (maker or W.tiny_2d)(**kw)
    g = oracle.Grid(**w.grid_kwargs())
    rng = np.random.default_rng(21)
    from scipy.ndimage import gaussian_filter
    bump = gaussian_filter(rng.standard_normal(w.shape), 3)
    vp_true = (w.vp * (1 + 0.03 * bump / np.abs(bump).max())).astype(np.float32)
    obs = oracle.forward(g, vp_true, w.src_xyz, w.wavelet, w.rec_xyz).astype(np.float32)
    return w, g, obs


@pytest.mark.parametrize("maker", [W.tiny_2d, W.tiny_3d])
def test_autograd_matches_oracle_and_fused_gradient(maker):
    w, g, obs = _setup(maker)
    plan = S.Plan.from_workload(w)
    vp = torch.from_numpy(w.vp).cuda().requires_grad_(True)
    wav = torch.from_numpy(w.wavelet).cuda()
    obs_t = torch.from_numpy(obs).cuda()
    traces = wave_traces(vp, wav, plan)
    loss = 0.5 * ((traces - obs_t) ** 2).sum()
    loss.backward()
    _, J, dvp_ref = oracle.gradient(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, obs)
    assert abs(loss.item() - J) <= 1e-4 * J
    assert rel(vp.grad.cpu().numpy(), dvp_ref) < 1e-4
    # the same arithmetic as the fused entry point: identical bits
    _, dvp_fused = plan.gradient(vp.detach(), wav, obs_t)
    assert torch.equal(vp.grad, dvp_fused)


def test_autograd_wavelet_gradient_and_module():
    w, g, obs = _setup()
    plan = S.Plan.from_workload(w)
    vp = torch.from_numpy(w.vp).cuda().requires_grad_(True)
    wav = torch.from_numpy(w.wavelet).cuda().requires_grad_(True)
    prop = WavePropagator(plan)
    traces = prop(vp, wav)
    loss = 0.5 * ((traces - torch.from_numpy(obs).cuda()) ** 2).sum()
    loss.backward()
    res = traces.detach().cpu().numpy().astype(np.float64) - obs
    dvp_ref, dwav_ref = oracle.adjoint(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz, res)
    assert rel(wav.grad.cpu().numpy(), dwav_ref) < 1e-4
    assert rel(vp.grad.cpu().numpy(), dvp_ref) < 1e-4


def test_autograd_checkpointed_equals_full_history():
    w, _, obs = _setup(nt=110)
    plan = S.Plan.from_workload(w)
    wav = torch.from_numpy(w.wavelet).cuda()
    obs_t = torch.from_numpy(obs).cuda()
    grads = []
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    for budget in (0, int(full * 0.15)):
        vp = torch.from_numpy(w.vp).cuda().requires_grad_(True)
        loss = 0.5 * ((StrideWave.apply(vp, wav, plan, budget) - obs_t) ** 2).sum()
        loss.backward()
        grads.append(vp.grad.clone())
    assert torch.equal(grads[0], grads[1])


def test_autograd_matches_finite_differences_fp32():
    """Central differences of the FP32 misfit along a smooth direction."""
    w, _, obs = _setup(nt=140)
    plan = S.Plan.from_workload(w)
    wav = torch.from_numpy(w.wavelet).cuda()
    obs_t = torch.from_numpy(obs).cuda()
    rng = np.random.default_rng(8)
    from scipy.ndimage import gaussian_filter
    dm = gaussian_filter(rng.standard_normal(w.shape), 4)
    dm = torch.from_numpy((dm / np.abs(dm).max()).astype(np.float32)).cuda()
    vp = torch.from_numpy(w.vp).cuda().requires_grad_(True)
    loss = 0.5 * ((wave_traces(vp, wav, plan) - obs_t).double() ** 2).sum()
    loss.backward()
    gd = float((vp.grad.double() * dm.double()).sum())

    def J(v):
        tr = plan.forward(v.contiguous(), wav)
        return float(0.5 * ((tr - obs_t).double() ** 2).sum())

    h = 2.0
    fd = (J(vp.detach() + h * dm) - J(vp.detach() - h * dm)) / (2 * h)
    assert abs(fd - gd) <= 1e-2 * abs(gd), (fd, gd)


def test_backward_twice_is_refused():
    w, _, obs = _setup()
    plan = S.Plan.from_workload(w)
    vp = torch.from_numpy(w.vp).cuda().requires_grad_(True)
    wav = torch.from_numpy(w.wavelet).cuda()
    loss = (wave_traces(vp, wav, plan) ** 2).sum()
    loss.backward(retain_graph=True)
    with pytest.raises(RuntimeError):
        loss.backward()
