"""Fourth-order time (leapfrog with the modified-equation correction and the
time-filtered source): HIP forward traces against the FP64 oracle's, at the
workloads' CFL and near the larger stability limit of the corrected scheme;
the CFL check of each order; gradients refused for the fourth-order scheme."""
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


def test_gradients_refuse_the_fourth_order_scheme():
    w = W.tiny_2d()
    plan = S.Plan.from_workload(w, time_order=4)
    with pytest.raises(S.StrideError) as e:
        plan.workspace_bytes(S.STRIDE_MODE_GRADIENT)
    assert e.value.code == -1
