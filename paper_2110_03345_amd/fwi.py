"""Outer full-waveform-inversion loop on one GPU.

The paper poses FWI as an optimisation loop of blocks and iterations (Sec. 2.2:
an OptimisationLoop whose blocks group iterations, a local optimiser that
steps the model along the gradient); for imaging (Sec. 3.2) every block is a
frequency band, wavelets and traces are band-limited to the block's upper
frequency, and each iteration draws a random mini-batch of shots without
replacement (each shot once per band), sums their gradients and takes a
gradient-descent step.

Here the shot gradients of a mini-batch run together through the batching
engine of libstride_hip (one launch per time step advances every shot of the
batch), the band-limiting is the library's zero-phase low-pass, and the
per-shot gradients are summed on the device in shot order.  Nothing in the
loop runs on the host but bookkeeping.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi
from ._abi import STRIDE_MODE_GRADIENT, Plan


class GradientDescent:
    """vp <- clamp(vp - step_size * m g / max|m g|, bounds) (libstride_hip's
    stride_descent_step).

    The paper's optimiser takes a step size and the gradient; the scale of a
    raw dJ/dvp depends on the data, so the direction is normalised to unit
    maximum and step_size is the largest model change per step (m/s).  The
    optional mask m confines the update to a region of interest (the paper's
    reconstructions lie inside the transducer ring; next to the transducers
    the source and receiver footprints dominate the gradient)."""

    def __init__(self, step_size: float, bounds: Sequence[float] = (0.0, float("inf")),
                 mask: Optional[torch.Tensor] = None):
        self.step_size = float(step_size)
        self.bounds = (float(bounds[0]), float(bounds[1]))
        self.mask = mask.contiguous() if mask is not None else None
        self._work = None

    def step(self, vp: torch.Tensor, grad: torch.Tensor, stream=None) -> None:
        if self._work is None:
            self._work = torch.zeros(1, dtype=torch.int32, device=vp.device)
        _abi.stride_descent_step(vp, grad.contiguous(), self.step_size, self.bounds[0],
                                 self.bounds[1], self._work, mask=self.mask, stream=stream)


def shot_batches(nshots: int, per_iter: int, iters: int, rng: np.random.Generator) -> List[List[int]]:
    """Mini-batches for one block: shots drawn without replacement from a
    fresh permutation; when a block needs more shots than there are, the
    permutation is redrawn (each shot is used once before any is reused)."""
    out, pool = [], []
    for _ in range(iters):
        batch = []
        while len(batch) < per_iter:
            if not pool:
                pool = list(rng.permutation(nshots))
            batch.append(int(pool.pop()))
        out.append(sorted(batch))
    return out


@dataclass
class Survey:
    """Shots of one grid: a source position per shot, common receivers, one
    wavelet [nt] for all shots and observed traces [nshots][nrec][nt] (CUDA)."""
    shape: Sequence[int]
    spacing: float
    space_order: int
    nb: int
    vref: float
    dt: float
    nt: int
    src_xyz: np.ndarray          # [nshots][ndim]
    rec_xyz: np.ndarray          # [nrec][ndim]
    wavelet: torch.Tensor        # [nt]
    observed: torch.Tensor       # [nshots][nrec][nt]
    interp: int = 0

    @property
    def nshots(self) -> int:
        return int(self.src_xyz.shape[0])


@dataclass
class History:
    f_max: List[float] = field(default_factory=list)
    misfit: List[float] = field(default_factory=list)      # per iteration, summed over its shots
    shots: List[List[int]] = field(default_factory=list)
    seconds: float = 0.0
    shot_gradients: int = 0


class BatchGradient:
    """Shot gradients of a mini-batch through one engine: every shot of the
    batch occupies a slot, all advance together; dvp is the sum over the batch
    in shot order and the misfit the sum of the shots' FP64 misfits."""

    def __init__(self, survey: Survey, max_slots: int, max_chunk: int = 64, use_graphs: bool = True,
                 budget_bytes: int = 0, device=None):
        self.s = survey
        self.dev = device or torch.device("cuda")
        nd = len(survey.shape)
        self.plans = [Plan(survey.shape, survey.spacing, survey.space_order, survey.nb, survey.vref,
                           survey.dt, survey.nt, survey.src_xyz[i:i + 1].reshape(1, nd),
                           survey.rec_xyz, interp=survey.interp)
                      for i in range(survey.nshots)]
        self.grid = _abi.make_grid(survey.shape, survey.spacing, survey.space_order, survey.nb,
                                   survey.vref, survey.dt, survey.nt, interp=survey.interp)
        nrec = survey.rec_xyz.shape[0]
        self.max_slots = max_slots
        self.max_chunk = max_chunk
        self.engine = _abi.stride_engine_create(self.grid, max_slots, max(nrec, 1), max_chunk,
                                                use_graphs)
        ws_bytes = self.plans[0].workspace_bytes(STRIDE_MODE_GRADIENT, budget_bytes)
        self.ws = [torch.empty(ws_bytes, dtype=torch.uint8, device=self.dev) for _ in range(max_slots)]
        self.traces = [torch.empty((nrec, survey.nt), dtype=torch.float32, device=self.dev)
                       for _ in range(max_slots)]
        self.dvp = [None] * max_slots
        self.misfit = torch.zeros((max_slots, 1), dtype=torch.float64, device=self.dev)
        self.stream = torch.cuda.Stream(device=self.dev)

    def close(self):
        if self.engine is not None:
            _abi.stride_engine_destroy(self.engine)
            self.engine = None

    def __call__(self, vp: torch.Tensor, wavelet: torch.Tensor, observed: torch.Tensor,
                 shots: Sequence[int]):
        """(sum of misfits, summed dvp) over `shots`; wavelet [nt] and
        observed [nshots][nrec][nt] already band-limited."""
        wav = wavelet.reshape(1, -1).contiguous()
        vmax = float(vp.max())
        total = torch.zeros_like(vp)
        results = {}
        pending = list(shots)
        slot_of, free = {}, list(range(self.max_slots))[::-1]
        torch.cuda.current_stream().synchronize()
        s = self.stream
        while pending or slot_of:
            while pending and free:
                i = pending.pop(0)
                k = free.pop()
                if self.dvp[k] is None:
                    self.dvp[k] = torch.empty_like(vp)
                slot = _abi.stride_engine_attach(self.engine, self.plans[i].handle, STRIDE_MODE_GRADIENT,
                                                 vp, vmax, wav, observed[i], self.traces[k],
                                                 self.misfit[k], self.dvp[k], self.ws[k], s)
                slot_of[slot] = (i, k)
            _, fin = _abi.stride_engine_run(self.engine, self.max_chunk, self.max_slots, s)
            for slot in fin:
                i, k = slot_of.pop(slot)
                _abi.stride_engine_detach(self.engine, slot)
                # keep the shot's result until the batch is summed in shot order
                # (copied on the engine's stream, behind the shot's last kernels)
                with torch.cuda.stream(s):
                    results[i] = (self.dvp[k].clone(), self.misfit[k].clone())
                free.append(k)
        s.synchronize()
        J = 0.0
        with torch.cuda.stream(s):
            for i in sorted(results):
                _abi.stride_accumulate(total, results[i][0], stream=s)
                J += float(results[i][1])
        s.synchronize()
        return J, total


def invert(survey: Survey, vp0: torch.Tensor, freqs: Sequence[float], iters_per_block: int,
           shots_per_iter: int, optimiser: GradientDescent, seed: int = 0, max_slots: int = 16,
           budget_bytes: int = 0, log=None):
    """Frequency-block FWI from vp0: for each f_max, band-limit the wavelet and
    the observed traces, then run iters_per_block gradient-descent steps on
    random mini-batches of shots_per_iter shots.  Returns (vp, History)."""
    import time
    rng = np.random.default_rng(seed)
    vp = vp0.clone().contiguous()
    hist = History()
    grad = BatchGradient(survey, min(max_slots, shots_per_iter), budget_bytes=budget_bytes,
                         device=vp.device)
    t0 = time.perf_counter()
    try:
        for f_max in freqs:
            wav = _abi.stride_lowpass(survey.wavelet.reshape(1, -1).contiguous(), survey.dt, f_max)
            obs = _abi.stride_lowpass(survey.observed.contiguous(), survey.dt, f_max)
            for batch in shot_batches(survey.nshots, shots_per_iter, iters_per_block, rng):
                J, g = grad(vp, wav, obs, batch)
                optimiser.step(vp, g)
                hist.f_max.append(float(f_max))
                hist.misfit.append(J)
                hist.shots.append(batch)
                hist.shot_gradients += len(batch)
                if log:
                    log(f"f_max {f_max / 1e3:.0f} kHz  shots {batch}  misfit {J:.4e}")
        torch.cuda.synchronize()
    finally:
        grad.close()
    hist.seconds = time.perf_counter() - t0
    return vp, hist


__all__ = ["GradientDescent", "Survey", "History", "BatchGradient", "shot_batches", "invert"]
