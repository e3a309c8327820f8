"""torch.autograd.Function around the engine's checkpointed forward run and
hand-written adjoint.

    J = LBMObjective.apply(q, wall_u, g, s, problem)

q (L,), wall_u (L, D), g (D,) and s (Q,) are float64 tensors (any device;
they are copied to the host for the ABI, which is argument marshalling).
`problem` is a Problem holding the solver, how to initialise it, the number
of steps, the checkpoint interval and the objective.  forward() runs the
steps with a snapshot every `every` steps (sqrt(n) checkpointing when
every ~ sqrt(n)); backward() replays each segment and runs the adjoint
kernel backwards through it, returning dJ/dq, dJ/dwall_u, dJ/dg, dJ/ds.
When s does not require a gradient, forward() turns the solver's rate
gradients off (lbm_set_rate_gradient), so that the reverse sweep reads the
forward step records instead of the states (every = 1 then keeps no
snapshot at all); the returned gradient of s is then None.
"""

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np
import torch


@dataclass
class Problem:
    solver: object                      # binding.Solver with its geometry set
    steps: int
    every: int
    objective: str = "force_x"          # "force_x", "mean_ux" or "pressure_drop"
    tag: int = 0
    window: tuple = (0, 1)              # [t_begin, t_end)
    planes: Optional[tuple] = None      # (x_in, x_out) of "pressure_drop"
    init: Optional[Callable] = None     # init(solver); default: rest state
    last_J: float = field(default=float("nan"))


def _np(t):
    return t.detach().to("cpu", torch.float64).numpy()


class LBMObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, q, wall_u, g, s, problem):
        sv = problem.solver
        sv.update_links(_np(q), _np(wall_u))
        sv.set_parameters(_np(s), _np(g))
        if problem.init is None:
            sv.init()
        else:
            problem.init(sv)
        sv.set_objective(problem.objective, problem.tag, *problem.window, planes=problem.planes)
        sv.set_rate_gradient(bool(ctx.needs_input_grad[3]))
        sv.run_checkpointed(problem.steps, problem.every)
        J = sv.objective()
        problem.last_J = J
        ctx.problem = problem
        ctx.meta = [(t.device, t.dtype, t.shape) for t in (q, wall_u, g, s)]
        return torch.tensor(J, dtype=torch.float64, device=q.device)

    @staticmethod
    def backward(ctx, grad_out):
        sv = ctx.problem.solver
        sv.adjoint()
        (dev_q, _, _), (dev_u, _, _) = ctx.meta[0], ctx.meta[1]
        if dev_q.type == "cuda" and dev_u.type == "cuda":
            # per-link gradients stay on the device (no host round trip)
            nf, nl = sv.counts()
            dq = torch.empty(nl, dtype=torch.float64, device=dev_q)
            du = torch.empty((nl, sv.D), dtype=torch.float64, device=dev_u)
            small = sv.grad_device(dq, du)
            gr = dict(q=dq, wall_u=du, g=torch.as_tensor(small["g"]), s=torch.as_tensor(small["s"]))
        else:
            gr = {k: torch.as_tensor(v) for k, v in sv.grad().items()}
        scale = float(grad_out)
        outs = []
        for key, (dev, dt, shape) in zip(("q", "wall_u", "g", "s"), ctx.meta):
            outs.append((gr[key] * scale).to(dtype=dt).reshape(shape).to(dev))
        if not ctx.needs_input_grad[3]:
            outs[3] = None
        return outs[0], outs[1], outs[2], outs[3], None


def objective(q, wall_u, g, s, problem):
    return LBMObjective.apply(q, wall_u, g, s, problem)


def sqrt_checkpoint_interval(n_steps):
    """Interval giving about sqrt(n) snapshots and a sqrt(n)-long replay."""
    return max(1, int(round(np.sqrt(n_steps))))
