"""Learned start solution for MALI: training and use.

The start populations decide how many iterations a column needs (Sec. 2.3).
A network trained on populations that MALI itself converged predicts the
log departure coefficients of every depth point; those give the start
populations of a new batch of columns, and MALI iterates from there to the
same convergence test.  Columns that fail from the learned start are solved
again from LTE, so the network can cost iterations but never the answer.

Every numerical step runs in the library's kernels (rh15d_mlp_*,
rh15d_departures, rh15d_pops_from_departures, rh15d_solve_columns); this
module only sequences the calls and moves tensors.
"""
from __future__ import annotations

import dataclasses
import math
import time

import numpy as np

from . import rh15d as rh

# Predicted |ln b| below this is replaced by LTE (0): about the network's
# mean error on held-out columns of the synthetic cubes.
SHRINK = 0.01


@dataclasses.dataclass
class TrainReport:
    points: int
    steps: int
    batch: int
    seconds: float
    loss_first: float
    loss_last: float
    losses: list


def train(atom: rh.Atom, dc: rh.DeviceColumns, pops, n_hidden=256, n_layers=3, steps=2000, batch=4096,
          lr=1e-3, seed=0, log_every=0, stream=None) -> tuple[rh.MLP, TrainReport]:
    """Fit a network to the log departure coefficients of converged
    populations `pops` (CUDA float64 [total_depth][L]) of the columns `dc`.

    Adam with a cosine learning-rate decay from lr to 0; mini-batches are
    consecutive slices of a seeded permutation of the depth points,
    reshuffled every epoch.  The steps of an epoch run as replays of one
    captured training step (MLP.train_batches)."""
    import torch
    dev = dc.z.device
    P = dc.total_depth
    net = rh.MLP(n_hidden, n_layers, atom.n_levels, seed)
    target_all = rh.departures(atom, dc, pops, stream=stream)
    rng = np.random.default_rng(seed)
    feats = torch.empty((P, rh.N_FEATURES), dtype=torch.float32, device=dev)
    target = torch.empty_like(target_all)

    def shuffle():
        perm = torch.as_tensor(rng.permutation(P), dtype=torch.int64, device=dev)
        rh.MLP.features(dc, perm, out=feats, stream=stream)
        torch.index_select(target_all, 0, perm, out=target)

    shuffle()
    net.fit_normalization(feats, stream=stream)
    batch = min(batch, P)
    per_epoch = max(1, P // batch)
    losses = []
    loss_buf = torch.empty(per_epoch, dtype=torch.float32, device=dev)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    s = 0
    while s < steps:
        e, b = divmod(s, per_epoch)
        if b == 0 and e > 0:
            shuffle()
        n = min(per_epoch - b, steps - s)
        lrs = [lr * 0.5 * (1.0 + math.cos(math.pi * (s + i) / steps)) for i in range(n)]
        net.train_batches(feats[b * batch:], target[b * batch:], batch, lrs, losses=loss_buf, stream=stream)
        want = [i for i in range(n) if s + i == 0 or s + i == steps - 1 or (log_every and (s + i) % log_every == 0)]
        if want:
            lv = loss_buf[:n].cpu().numpy()
            losses += [(s + i, float(lv[i])) for i in want]
        s += n
    torch.cuda.synchronize(dev)
    rep = TrainReport(points=P, steps=steps, batch=batch, seconds=time.perf_counter() - t0,
                      loss_first=losses[0][1], loss_last=losses[-1][1], losses=losses)
    return net, rep


class WarmStartSolver:
    """rh15d.Solver with the start populations predicted by `net`.

    run() = stencil features -> network -> start populations -> MALI from
    that start; the buffers are allocated once, so repeated runs allocate
    nothing on the device.  refine_failed() solves the columns that did not
    converge again from LTE (a host synchronisation)."""

    def __init__(self, atom: rh.Atom, dc: rh.DeviceColumns, net: rh.MLP, opts: rh.Options, shrink=SHRINK,
                 want_spectrum=True, want_psi=False, want_history=True, workspace=None):
        import torch
        if net.n_out != atom.n_levels:
            raise ValueError(f"network has {net.n_out} outputs, atom {atom.n_levels} levels")
        dev = dc.z.device
        P = dc.total_depth
        self.atom, self.net, self.dc, self.shrink = atom, net, dc, shrink
        self.feats = torch.empty((P, rh.N_FEATURES), dtype=torch.float32, device=dev)
        self.log_b = torch.empty((P, atom.n_levels), dtype=torch.float32, device=dev)
        self.init = torch.empty((P, atom.n_levels), dtype=torch.float64, device=dev)
        o = rh.Options.from_buffer_copy(opts)
        o.start = rh.START_PROVIDED
        self.opts = o
        self.dc_warm = dataclasses.replace(dc, init_pops=self.init)
        self.solver = rh.Solver(atom, self.dc_warm, o, want_spectrum=want_spectrum, want_psi=want_psi,
                                want_history=want_history, workspace=workspace)
        self.refined = 0

    def predict(self, stream=None):
        rh.MLP.features(self.dc, out=self.feats, stream=stream)
        self.net.forward(self.feats, out=self.log_b, stream=stream)
        rh.pops_from_departures(self.atom, self.dc, self.log_b, shrink=self.shrink, out=self.init, stream=stream)
        return self.init

    def run(self, stream=None):
        self.predict(stream)
        self.solver.run(stream)
        return self

    def refine_failed(self, stream=None) -> int:
        """Re-solve every column whose status is not converged from LTE and
        write its results into this solver's outputs; n_iter then counts the
        iterations of both attempts.  Returns the number of columns redone."""
        o = rh.Options.from_buffer_copy(self.opts)
        o.start = rh.START_LTE
        self.refined = rh.resolve_failed(self.atom, self.dc, self.solver.result(), o, stream=stream)
        return self.refined

    def result(self) -> dict:
        return self.solver.result()
