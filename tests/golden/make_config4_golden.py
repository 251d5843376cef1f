#!/usr/bin/env python3
"""Writes the FP64 oracle's reference values for the 3D head-like workload
(256^3 at 0.5 mm + 30-cell sponge = 316^3 padded, 10th order, source at
element 0 of the 1024-element hemisphere) into tests/golden/:

  config4_forward.npz   forward on the head phantom, all 3000 steps:
      receivers   indices of the sampled receivers (every 16th)
      traces      their traces, float32 [64][3000]
      norms, peak L2 norm and max |trace| of every receiver's trace [1024]
  config4_gradient.npz  shot gradient at the skull-only starting model, first
                        1000 steps, observed data zero (J = 1/2 sum traces^2):
      misfit      J
      slice_axes, slice_index        the planes stored: per axis the plane of
                                     largest norm (through the source), and the
                                     physical face of axis 0 of larger norm (the
                                     padding transpose sums the layer into it)
      slice_0 .. slice_3             dvp on those planes, float32
      norms_a0, norms_a1, norms_a2   L2 norm of dvp over each plane of each axis
      norm_all, norm_interior, norm_edge   L2 norms over all cells, cells at least
                                     4 from every face, cells within 2 of a face

Only oracle/ and the seeded workload generators are used.  It runs for tens
of minutes on a few host cores:  python tests/golden/make_config4_golden.py
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads as W  # noqa: E402

GRAD_NT = 1000
EVERY = 16


def edge_masks(shape, inner=4, edge=2):
    idx = np.indices(shape)
    dist = np.min([np.minimum(i, n - 1 - i) for i, n in zip(idx, shape)], axis=0)
    return dist >= inner, dist < edge


def main(which):
    if "forward" in which:
        w = W.config4()
        g = oracle.Grid(**w.grid_kwargs())
        t0 = time.time()
        tr = oracle.forward(g, w.vp_true, w.src_xyz, w.wavelet, w.rec_xyz)
        print(f"forward {w.padded_shape} nt={w.nt}: {time.time() - t0:.0f} s", flush=True)
        rec = np.arange(0, w.rec_xyz.shape[0], EVERY)
        np.savez_compressed(os.path.join(HERE, "config4_forward.npz"), receivers=rec,
                            traces=tr[rec].astype(np.float32), norms=np.linalg.norm(tr, axis=1),
                            peak=np.abs(tr).max(axis=1))
    if "gradient" in which:
        w = W.config4(nt=GRAD_NT)
        g = oracle.Grid(**w.grid_kwargs())
        obs = np.zeros((w.rec_xyz.shape[0], w.nt))
        t0 = time.time()
        _, J, dvp = oracle.gradient(g, w.vp_start, w.src_xyz, w.wavelet, w.rec_xyz, obs)
        print(f"gradient {w.padded_shape} nt={w.nt}: {time.time() - t0:.0f} s, J = {J:.6e}", flush=True)
        inner, edge = edge_masks(w.shape)
        norms = [np.linalg.norm(dvp, axis=tuple(b for b in range(3) if b != a)) for a in range(3)]
        axes = [0, 1, 2, 0]
        index = [int(np.argmax(n)) for n in norms]
        index.append(0 if norms[0][0] > norms[0][-1] else w.shape[0] - 1)
        slices = {f"slice_{i}": np.take(dvp, k, axis=a).astype(np.float32)
                  for i, (a, k) in enumerate(zip(axes, index))}
        np.savez_compressed(
            os.path.join(HERE, "config4_gradient.npz"), misfit=J, slice_axes=np.array(axes),
            slice_index=np.array(index), **slices, norms_a0=norms[0], norms_a1=norms[1],
            norms_a2=norms[2], norm_all=np.linalg.norm(dvp),
            norm_interior=np.linalg.norm(dvp[inner]), norm_edge=np.linalg.norm(dvp[edge]))


if __name__ == "__main__":
    main(sys.argv[1:] or ["forward", "gradient"])
