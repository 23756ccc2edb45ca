"""Receding-horizon PI^2 controller on one GPU (Sec. 3.1, last paragraph).

Each control step runs `iterations` path-integral iterations (rollouts through
the LWPR model, then the update of the nominal controls), executes the first
control on the plant (a draw from the learned model) and warm-starts the next
step with the shifted plan.  The controller state is (x0, u_nom, iter) on the
device, so a whole control step can be captured once into a HIP graph and
replayed: replays read and advance the device-resident state and need no
host-side parameter updates.
"""
from __future__ import annotations

from typing import Optional

import torch

from . import (DeviceModel, DeviceProblem, PI_OP_ROLLOUT, PI_OP_RH_SHIFT, PI_OP_UPDATE,
               rh_shift, rollout_cost, update, workspace, workspace_bytes)


class RHController:
    """The model is folded once here (DeviceModel.fold) unless fold_model is
    False: it stays fixed over the loop; call model.fold() again after changing
    its tensors."""

    def __init__(self, prob: DeviceProblem, model: DeviceModel, iterations: int = 1,
                 graph: bool = True, fold_model: bool = True):
        self.prob, self.model = prob, model
        if fold_model:
            model.fold()
        self.iterations = int(iterations)
        self.cost = torch.empty((prob.K, prob.T), dtype=prob.dtype, device=prob.device)
        need = max(workspace_bytes(PI_OP_ROLLOUT, prob, model),
                   workspace_bytes(PI_OP_UPDATE, prob, None),
                   workspace_bytes(PI_OP_RH_SHIFT, prob, model))
        workspace(need, prob.device)           # reserve before any capture
        self.use_graph = graph
        self.graph: Optional[torch.cuda.CUDAGraph] = None

    # one control step on the current stream
    def _step_eager(self):
        for _ in range(self.iterations):
            rollout_cost(self.prob, self.model, out=self.cost)
            update(self.prob, self.cost)
        rh_shift(self.prob, self.model)

    def capture(self):
        """Records one control step into a HIP graph (state is not advanced)."""
        saved = self.state()
        # a first eager step initialises the library's per-device checks
        self._step_eager()
        torch.cuda.synchronize()
        self.load_state(saved)
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        g = torch.cuda.CUDAGraph()
        with torch.cuda.stream(s):
            with torch.cuda.graph(g, stream=s):
                self._step_eager()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        # capture does not execute: restore the state anyway for clarity
        self.load_state(saved)
        self.graph = g
        return g

    def step(self):
        if self.use_graph:
            if self.graph is None:
                self.capture()
            self.graph.replay()
        else:
            self._step_eager()

    # ------------------------------------------------------ checkpoint/resume
    def state(self) -> dict:
        """Everything needed to resume bit-for-bit: the random stream is
        counter-based, so (x0, u_nom, iter) and the seed fix all future draws."""
        p = self.prob
        return {"x0": p.x0.detach().clone(), "u_nom": p.u_nom.detach().clone(),
                "iter": p.iter.detach().clone(), "seed": int(p.prob.seed)}

    def load_state(self, st: dict):
        p = self.prob
        if int(st.get("seed", p.prob.seed)) != int(p.prob.seed):
            raise ValueError("state belongs to a different random stream")
        p.x0.copy_(st["x0"])
        p.u_nom.copy_(st["u_nom"])
        p.iter.copy_(st["iter"])
