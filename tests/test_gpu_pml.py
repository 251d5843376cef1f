"""Perfectly matched layer on the GPU (boundary = 1): forward traces against
the oracle's PML forward, 2D and 3D, orders 8 and 10, ragged shapes that span
several tiles, the 2D benchmark grid (1104^2 padded, 2500 steps) and the 3D
head grid (316^3, 200 steps: the wave enters the layer); the allocation-free
forward equal to the workspace one; refusal of every other solve."""
import numpy as np
import pytest

import oracle
import workloads as W
from parity import check_traces

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if torch.cuda.is_available():
    import paper_2110_03345_amd as S
    from paper_2110_03345_amd import _abi


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def tol_for(nt):
    return 1e-4 if nt <= 1000 else 1e-3


def _near_edge(w, frac=0.08):
    """Receivers close to the physical edges, where the layer acts first."""
    ext = np.array([(s - 1) * w.spacing for s in w.shape])
    rng = np.random.default_rng(5)
    pts = rng.uniform(0.1, 0.9, (12, len(w.shape))) * ext
    for i in range(len(pts)):
        a = i % len(w.shape)
        pts[i, a] = frac * ext[a] if i % 2 else (1 - frac) * ext[a]
    return pts


CASES = [
    ("2d_o8", lambda: W.tiny_2d(nt=260)),
    ("2d_o10_ragged", lambda: W.tiny_2d(n=(83, 141), nb=9, nt=300, space_order=10)),
    ("3d_o10", lambda: W.tiny_3d(nt=120)),
    ("3d_o8_ragged", lambda: W.tiny_3d(n=(37, 21, 70), nb=6, nt=110, space_order=8)),
]


@pytest.mark.parametrize("name,maker", CASES, ids=[c[0] for c in CASES])
def test_pml_forward_matches_oracle(name, maker):
    w = maker()
    rec = np.concatenate([w.rec_xyz, _near_edge(w)])
    print(f"pml {name} shape={w.shape} nb={w.nb} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs())
    ref = oracle.forward_pml(g, w.vp, w.src_xyz, w.wavelet, rec)
    plan = S.Plan.from_workload(w, rec_xyz=rec, boundary=1)
    tr = plan.forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    print(check_traces(tr, ref, tol_for(w.nt)), flush=True)
    # the layer matters here: the sponge gives other traces
    sp = S.Plan.from_workload(w, rec_xyz=rec).forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    assert np.linalg.norm(sp - ref) > 1e-3 * np.linalg.norm(ref)


def test_pml_benchmark_grids_match_oracle():
    w = W.config2()
    print(f"pml config2 {w.padded_shape} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs())
    ref = oracle.forward_pml(g, w.vp, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = S.Plan.from_workload(w, boundary=1).forward(dev(w.vp), dev(w.wavelet)).cpu().numpy()
    print(check_traces(tr, ref, 1e-3), flush=True)
    w = W.config4(nt=200)
    print(f"pml config4 {w.padded_shape} nt={w.nt}", flush=True)
    g = oracle.Grid(**w.grid_kwargs())
    ref = oracle.forward_pml(g, w.vp_true, w.src_xyz, w.wavelet, w.rec_xyz)
    tr = S.Plan.from_workload(w, boundary=1).forward(dev(w.vp_true), dev(w.wavelet)).cpu().numpy()
    print(check_traces(tr, ref, 1e-4), flush=True)


def test_pml_static_forward_and_refusals():
    w = W.tiny_2d(nt=120)
    plan = S.Plan.from_workload(w, boundary=1)
    vp, wav = dev(w.vp), dev(w.wavelet)
    ref = plan.forward(vp, wav)
    out = torch.full_like(ref, float("nan"))
    _abi.stride_plan_forward_static(plan.handle, vp, wav, out)
    torch.cuda.synchronize()
    assert torch.equal(ref, out)
    obs = torch.zeros_like(ref)
    with pytest.raises(S.StrideError) as e:
        plan.gradient(vp, wav, obs, ws=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
    assert e.value.code == -1 and "PML" in str(e.value)
    with pytest.raises(S.StrideError):
        plan.forward_medium(vp, wav, ws=torch.empty(1 << 20, dtype=torch.uint8, device="cuda"))
