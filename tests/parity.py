"""Comparison of HIP results with the FP64 oracle.

Besides the relative L2 over a whole output, the checks bound the error of
every receiver trace and of each region of a gradient separately, so that a
wrong weak receiver, or a wrong band of cells, cannot hide under a norm that
the strongest signals dominate:

- traces: every trace carrying at least `floor` of the largest trace norm is
  within `per` x tol of its own norm; the weaker ones (signal that has barely
  arrived) are within `per` x tol x floor of the largest norm;
- fields on the physical grid (dvp): the interior (cells at least `inner` from
  every face) and the edge strip (cells within `edge` of a face, where the
  padding transpose adds the absorbing layer into the edge cells) are each
  within `per` x tol of their own norm, or of `floor` x the whole field's norm
  when the region holds less (a strip the wave has barely reached).

The FP32 kernels and the FP64 oracle differ by rounding only, and rounding
errors are relative to the local signal, so per-trace and per-region errors
stay within a small factor of the global one; a wrong tap, term, sign or
strip gives an error of order one in the part it touches.
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def check_traces(tr, ref, tol, per=10.0, floor=1e-3, what="traces"):
    tr = np.asarray(tr, dtype=np.float64).reshape(len(ref), -1)
    ref = np.asarray(ref, dtype=np.float64)
    glob = rel(tr, ref)
    assert glob < tol, f"{what}: relative L2 {glob:.3e} >= {tol:.1e}"
    norms = np.linalg.norm(ref, axis=1)
    errs = np.linalg.norm(tr - ref, axis=1)
    big = norms >= floor * norms.max()
    worst_rel = float((errs[big] / norms[big]).max()) if big.any() else 0.0
    worst_abs = float(errs[~big].max() / norms.max()) if (~big).any() else 0.0
    assert worst_rel < per * tol, (
        f"{what}: receiver {int(np.flatnonzero(big)[np.argmax(errs[big] / norms[big])])} "
        f"relative error {worst_rel:.3e} >= {per * tol:.1e}")
    assert worst_abs < per * tol * floor, f"{what}: weak-trace error {worst_abs:.3e}"
    return {"global": glob, "worst_trace": worst_rel, "weak_abs": worst_abs,
            "strong_traces": int(big.sum())}


def regions(shape, inner=4, edge=2):
    """(interior mask, edge-strip mask) of a physical grid."""
    idx = np.indices(shape)
    dist = np.min([np.minimum(i, n - 1 - i) for i, n in zip(idx, shape)], axis=0)
    return dist >= inner, dist < edge


def check_field(d, ref, tol, per=3.0, inner=4, edge=2, floor=1e-2, what="dvp"):
    d = np.asarray(d, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    glob = rel(d, ref)
    assert glob < tol, f"{what}: relative L2 {glob:.3e} >= {tol:.1e}"
    ins, strip = regions(ref.shape, inner, edge)
    total = np.linalg.norm(ref)

    def region(m):
        return float(np.linalg.norm(d[m] - ref[m]) / max(np.linalg.norm(ref[m]), floor * total))

    e_in = region(ins)
    e_edge = region(strip)
    assert e_in < per * tol, f"{what}: interior relative L2 {e_in:.3e} >= {per * tol:.1e}"
    assert e_edge < per * tol, f"{what}: edge strip relative L2 {e_edge:.3e} >= {per * tol:.1e}"
    return {"global": glob, "interior": e_in, "edge": e_edge}
