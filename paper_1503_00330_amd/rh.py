"""Receding-horizon PI^2 controller on one GPU (Sec. 3.1, last paragraph).

Each control step runs `iterations` path-integral iterations (rollouts through
the LWPR model, then the update of the nominal controls), executes the first
control on the plant (a draw from the learned model) and warm-starts the next
step with the shifted plan.  The controller state is (x0, u_nom, iter) on the
device, so a whole control step can be captured once into a HIP graph and
replayed: replays read and advance the device-resident state and need no
host-side parameter updates.

With a list of goals the controller also keeps the task layer of the flight
experiments (Sec. 5): the state cost pulls toward the current goal, and once
the plant's position has come within the switch radius of it (0.25 m in the
paper) the goal moves on to the next point of the cycle.  The check reads the
position after each control step; the goal is a launch argument, so a switch
captures the control step again.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import (DeviceModel, DeviceProblem, PI_DYN_POINTMASS2D, PI_OP_ROLLOUT, PI_OP_RH_SHIFT,
               PI_OP_UPDATE, rh_shift, rollout_cost, update, workspace, workspace_bytes)


class RHController:
    """The model is folded once here (DeviceModel.fold) unless fold_model is
    False: it stays fixed over the loop; call model.fold() again after changing
    its tensors.  With tune=True the rollout launch shape comes from the
    autotuner (tune.ensure).  With `goals` (points of the cycle, rows of 3 coordinates)
    the controller sets the problem's goal itself (it writes prob.prob.goal)
    and switches to the next point within `switch_radius` of the current one."""

    def __init__(self, prob: DeviceProblem, model: DeviceModel, iterations: int = 1,
                 graph: bool = True, fold_model: bool = True, goals=None,
                 switch_radius: float = 0.25, tune: bool = False):
        self.prob, self.model = prob, model
        if tune:
            # the rollout launch from the autotuner's cache, tuned now if absent
            from . import tune as _tune
            _tune.ensure(prob, model)
        self.goals = None
        self.goal_index = 0
        self.switch_radius = float(switch_radius)
        if goals is not None:
            self.goals = np.array(goals, dtype=np.float64).reshape(-1, 3)
            if len(self.goals) == 0:
                raise ValueError("goals: at least one point")
            if not self.switch_radius >= 0.0:
                raise ValueError("switch_radius must be >= 0")
            self._set_goal(0)
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
        if self.goals is not None:
            self._switch_goal()

    def _set_goal(self, g: int):
        self.goal_index = int(g)
        self.prob.prob.goal = self.goals[self.goal_index].copy()
        self.graph = None   # the goal is a launch argument of the captured step

    def _switch_goal(self):
        # the plant's position after this control step (the read waits for it)
        npos = 2 if self.prob.dyn == PI_DYN_POINTMASS2D else 3
        pos = self.prob.x0[:npos].to(torch.float64).cpu().numpy()
        if np.sqrt(np.sum((pos - self.goals[self.goal_index, :npos]) ** 2)) < self.switch_radius:
            self._set_goal((self.goal_index + 1) % len(self.goals))

    # ------------------------------------------------------ checkpoint/resume
    def state(self) -> dict:
        """Everything needed to resume bit-for-bit: the random stream is
        counter-based, so (x0, u_nom, iter) and the seed fix all future draws."""
        p = self.prob
        return {"x0": p.x0.detach().clone(), "u_nom": p.u_nom.detach().clone(),
                "iter": p.iter.detach().clone(), "seed": int(p.prob.seed),
                "goal_index": self.goal_index}

    def load_state(self, st: dict):
        p = self.prob
        if int(st.get("seed", p.prob.seed)) != int(p.prob.seed):
            raise ValueError("state belongs to a different random stream")
        p.x0.copy_(st["x0"])
        p.u_nom.copy_(st["u_nom"])
        p.iter.copy_(st["iter"])
        if self.goals is not None and int(st.get("goal_index", 0)) != self.goal_index:
            self._set_goal(int(st.get("goal_index", 0)) % len(self.goals))
