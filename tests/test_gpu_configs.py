"""Parity at the sizes of the benchmark configurations, in the launch
configuration bench.py times (default tile shapes and chunk lengths).

- 2D breast-like forward, 1104^2 padded, 2500 steps: every trace sample
  against the FP64 oracle (1e-3 relative L2 for up to 3000 steps).
- 2D FWI gradient through the autograd function, 592^2 padded, 1500 steps,
  two of the 64 ring shots with checkpointed forward wavefields: the summed
  gradient and misfit against the oracle's.
- 3D head-like grid, 316^3 padded, 10th order: traces of a 150-step forward
  against the oracle, and the gradient bitwise unchanged by the checkpointing
  budget at this size.
(The full 3000-step 3D forward and a checkpointed 3D gradient at this size are
compared in test_gpu_fullsize.py.)  Besides the relative L2 over each output,
every trace and the interior and edge strip of each gradient are bounded on
their own (tests/parity.py).
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
    from paper_2110_03345_amd.autograd import wave_traces


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_config2_forward_full_size_matches_oracle():
    w = W.config2()
    print(f"config2 {w.padded_shape} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs())
    tr = S.Plan.from_workload(w).forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    ref = oracle.forward(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    print(f"config2 traces {check_traces(tr, ref, 1e-3)}", flush=True)


def test_config3_autograd_gradient_matches_oracle():
    w = W.config3()
    g = oracle.Grid(**w.grid_kwargs())
    shots = [0, 32]
    print(f"config3 {w.padded_shape} nt={w.nt} shots {shots}", flush=True)
    vp = dev(w.vp_start).requires_grad_(True)
    wav = dev(w.wavelet)
    loss = 0.0
    J_ref, dvp_ref = 0.0, np.zeros(w.shape)
    for i in shots:
        src = w.shot_src_xyz[i:i + 1]
        obs = oracle.forward(g, w.vp_true, src, w.wavelet, w.rec_xyz).astype(np.float32)
        plan = S.Plan(w.shape, w.spacing, w.space_order, w.nb, w.vref, w.dt, w.nt, src, w.rec_xyz)
        # checkpointed forward wavefields: a budget of a quarter of the full history
        budget = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT) // 4
        traces = wave_traces(vp, wav, plan, budget)
        loss = loss + 0.5 * ((traces - dev(obs)) ** 2).sum()
        _, J, d = oracle.gradient(g, w.vp_start, src, w.wavelet, w.rec_xyz, obs)
        J_ref += J
        dvp_ref += d
    loss.backward()
    st = check_field(vp.grad.cpu().numpy(), dvp_ref, 1e-3)
    print(f"config3 misfit {loss.item():.6e} vs {J_ref:.6e}, dvp {st}", flush=True)
    assert abs(loss.item() - J_ref) <= 1e-3 * J_ref


def test_config4_full_grid_forward_and_checkpointing():
    w = W.config4(nt=150)
    print(f"config4 {w.padded_shape} nt={w.nt}", flush=True)
    plan = S.Plan.from_workload(w)
    vp, wav = dev(w.vp_start), dev(w.wavelet)
    tr = plan.forward(vp, wav).cpu().numpy()
    g = oracle.Grid(**w.grid_kwargs())
    ref = oracle.forward(g, w.vp_start, w.src_xyz, w.wavelet, w.rec_xyz)
    print(f"config4 traces {check_traces(tr, ref, 1e-4)}", flush=True)
    obs = plan.forward(dev(w.vp_true), wav)      # data for the misfit (any values will do)
    m0, g0 = plan.gradient(vp, wav, obs)
    full = plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    for frac in (0.3, 0.12):
        ws = plan.workspace(S.STRIDE_MODE_GRADIENT, int(full * frac))
        m1, g1 = plan.gradient(vp, wav, obs, ws=ws)
        del ws
        assert torch.equal(m0, m1) and torch.equal(g0, g1), frac
