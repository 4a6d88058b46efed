"""Domain-decomposed training loop on one GPU (Algorithm 1).

At every iteration i (1-based) with i mod I_comm = 0, as in Algorithm 1, the
neighbour targets of every ghost point are refreshed on the device
(pinn_exchange: value forward of the owning neighbour, with the
reference-anchor subtraction p - p(x_anc, t) when that neighbour is a master,
section 2.2); then all subdomains take one fused training step together (one
grouped launch).  The targets are written into the subdomains' own gh_up
tensors, which the step reads; between exchanges they stay fixed.  One
addition to Algorithm 1: by default the targets are also exchanged before the
first iteration when 1 mod I_comm != 0, so that no step trains against targets
that no neighbour produced (with I_comm = 1, the paper's setting, the two
schedules are the same).
The optional step decay of the learning rate (appendix B: factor and
interval) is computed by pinn_step from the step number t.
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import torch

from .context import Context


class DDTrainer:
    def __init__(self, ctx: Context, faces: Sequence[Tuple[int, int, int, int]], x_anc,
                 i_comm: int = 1, initial_exchange: bool = True):
        if int(i_comm) < 1:
            raise ValueError("i_comm must be >= 1")
        self.ctx = ctx
        self.faces = list(faces)
        self.x_anc = list(x_anc)
        self.i_comm = int(i_comm)
        self.initial_exchange = bool(initial_exchange)
        self.t = 0
        self.targets: List[torch.Tensor] = [s.gh_up if s.gh_up.numel() else None for s in ctx.subs]

    def exchange(self, stream=None):
        if self.faces:
            self.ctx.exchange(self.faces, self.x_anc, self.targets, stream=stream)

    def exchange_due(self, t: int) -> bool:
        """Exchange before iteration t: t mod I_comm = 0 (Algorithm 1), and at
        t = 1 when the initial exchange is on."""
        return t % self.i_comm == 0 or (t == 1 and self.initial_exchange)

    def step(self, stream=None):
        """One iteration: exchange when due, then one step of every subdomain.
        Returns the device loss tensor [n_sub, 7]."""
        self.t += 1
        if self.exchange_due(self.t):
            self.exchange(stream)
        loss, _ = self.ctx.step(self.t, stream=stream)
        return loss


def faces_of(problem) -> List[Tuple[int, int, int, int]]:
    """(receiver, owner, first ghost index, count) for every ghost face of a
    host problem description whose subdomains list their faces."""
    out = []
    for a, s in enumerate(problem.subs):
        for (b, _kind, first, count) in getattr(s, "faces", []):
            out.append((a, b, first, count))
    return out
