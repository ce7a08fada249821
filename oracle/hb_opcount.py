"""Floating-point operation count of the FP64 oracle's evaluation (the op
counter of the oracle, measurement infrastructure).

TEST AND MEASUREMENT INFRASTRUCTURE ONLY: the tests and the CPU-baseline
leg of the benchmark use it; the HIP library never does.

The count is taken by running the oracle's own code under a PyTorch
dispatch mode that tallies, per elementwise arithmetic operator, the
number of result elements (one operation each: add, subtract, multiply,
divide, square root, absolute value, comparison, selection, minimum and
maximum), reductions as one addition per reduced element, and contractions
(matrix and einsum products) as two operations per multiply-add.  Moving
data (indexing, stacking, copies) costs nothing.  Divided by the units of
work the evaluation performed, it gives the method's operations per unit
as the oracle writes them out; a kernel that shares subexpressions
between faces does fewer, one that recomputes more does more."""
from __future__ import annotations

import math
from typing import Callable, Dict, Tuple

import torch
from torch.utils._python_dispatch import TorchDispatchMode

# elementwise operators counted as one operation per output element
_ELEMENTWISE = {
    "add", "sub", "mul", "div", "neg", "sqrt", "abs", "maximum", "minimum", "where",
    "lt", "le", "gt", "ge", "eq", "ne", "rsub", "reciprocal", "pow", "sin", "cos",
    "clamp", "sign", "atan2",
}
_REDUCE = {"sum", "mean"}
_CONTRACT = {"mm", "bmm", "matmul", "addmm", "einsum", "dot"}


def _base(name: str) -> str:
    # "aten.mul.Tensor" -> "mul"; in-place "aten.add_.Tensor" -> "add"
    parts = name.split(".")
    op = parts[1] if len(parts) > 1 else parts[0]
    return op[:-1] if op.endswith("_") else op


class OpCounter(TorchDispatchMode):
    """Tallies floating-point operations of the torch code run under it."""

    def __init__(self):
        super().__init__()
        self.by_op: Dict[str, float] = {}

    @property
    def total(self) -> float:
        return float(sum(self.by_op.values()))

    def _add(self, op: str, n: float):
        if n:
            self.by_op[op] = self.by_op.get(op, 0.0) + float(n)

    def __torch_dispatch__(self, func, types, args=(), kwargs=None):
        kwargs = kwargs or {}
        out = func(*args, **kwargs)
        op = _base(str(func))
        floating = any(isinstance(a, torch.Tensor) and a.is_floating_point() for a in args)
        if not floating:
            return out
        if op in _ELEMENTWISE and isinstance(out, torch.Tensor):
            self._add(op, out.numel())
        elif op in _REDUCE and isinstance(out, torch.Tensor):
            self._add(op, max(0, args[0].numel() - out.numel()))
        elif op in ("mm", "bmm", "addmm", "dot", "matmul"):
            a, b = [x for x in args if isinstance(x, torch.Tensor)][-2:]
            k = a.shape[-1]
            self._add(op, 2 * out.numel() * k)
        return out


def count(fn: Callable, *args, **kwargs) -> Tuple[object, OpCounter]:
    """Run fn(*args, **kwargs) under the counter; returns (result, counter)."""
    with OpCounter() as c:
        res = fn(*args, **kwargs)
    return res, c


def ops_per_unit(blocks, q, flow, solver) -> Dict[str, float]:
    """Operations of one pseudo-time iteration of the oracle (four residual
    evaluations, the local step, the stage updates and the norm) per unit of
    work (one cell-snapshot Runge-Kutta-stage update), and of one residual
    evaluation per cell-snapshot."""
    from oracle import hb_oracle as O
    cs = sum(b.ns * b.ni * b.nj for b in blocks)
    stages = len(solver.rk_alpha)
    _, ci = count(O.rk_iterate, blocks, q, flow, solver, 1)
    _, cr = count(O.residual_all, blocks, q, flow, solver)
    return {"per_unit": ci.total / (cs * stages), "residual_per_cell_snapshot": cr.total / cs,
            "cell_snapshots": float(cs)}
