"""Python binding of libhb (ctypes).  Argument marshalling only: every step
of the residual, the iteration and the forces runs in the HIP library.
PyTorch provides device memory (tensors) and the current stream.

The binding fails loudly when libhb.so is missing or a tensor is not a
contiguous FP64 device tensor of the right size; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhb.so")

HB_OK, HB_ERR_ARG, HB_ERR_DEVICE, HB_ERR_OOM, HB_ERR_NONFINITE, HB_ERR_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5
HB_FP64, HB_FP32_BULK = 0, 1
HB_PREPARE_ADJOINT, HB_PREPARE_ADJOINT_ITERATE, HB_PREPARE_TD = 1, 2, 4
EXPORTS = ["hb_grid_create", "hb_grid_destroy", "hb_state_size", "hb_forces_size",
           "hb_xy_size", "hb_residual", "hb_rk_iterate", "hb_forces", "hb_residual_adjoint",
           "hb_forces_adjoint", "hb_adjoint_iterate", "hb_td_march", "hb_td_march_noalloc",
           "hb_prepare", "hb_save_state", "hb_load_state", "hb_save_solution", "hb_autotune",
           "hb_set_tuning",
           "hb_get_tuning", "hb_set_xy", "hb_set_alpha0", "hb_set_motion", "hb_get_status",
           "hb_profile_stages", "hb_stage_stats", "hb_last_error"]


class HBError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("libhb error %d: %s" % (code, msg))
        self.code = code


class c_block(ctypes.Structure):
    _fields_ = [("ni", ctypes.c_int32), ("nj", ctypes.c_int32), ("n_harm", ctypes.c_int32),
                ("xy", ctypes.POINTER(ctypes.c_double)), ("bc", ctypes.c_int32 * 4),
                ("wake_ncells", ctypes.c_int32), ("body_id", ctypes.c_int32)]


class c_cut(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in
                ("blk_a", "side_a", "start_a", "blk_b", "side_b", "start_b", "len", "reversed")]


class c_tuning(ctypes.Structure):
    _fields_ = [("tile_i", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("xcd_order", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("stage_ms", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class c_flow(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("mach", "reynolds", "prandtl", "gamma", "alpha0", "alpha_amp", "k_red", "l_ref",
                 "x_mom", "y_mom")]


class c_motion(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in
                ("pitch_amp", "pitch_phase", "heave_amp", "x_pivot", "y_pivot")]


class c_solver(ctypes.Structure):
    _fields_ = [("cfl", ctypes.c_double), ("n_stages", ctypes.c_int32),
                ("rk_alpha", ctypes.c_double * 8), ("precision", ctypes.c_int32),
                ("entropy_delta", ctypes.c_double), ("limiter_eps", ctypes.c_double),
                ("batched", ctypes.c_int32), ("graph_iters", ctypes.c_int32)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libhb.so (built in-tree by paper_1304_7654_amd.build)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhb.so is not built (run: python -m paper_1304_7654_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    L.hb_grid_create.argtypes = [ctypes.POINTER(c_block), i32, ctypes.POINTER(c_cut), i32,
                                 ctypes.POINTER(c_flow), ctypes.POINTER(c_solver),
                                 ctypes.POINTER(vp)]
    L.hb_grid_destroy.argtypes = [vp]
    for f in ("hb_state_size", "hb_forces_size", "hb_xy_size"):
        getattr(L, f).argtypes = [vp]
        getattr(L, f).restype = i64
    L.hb_residual.argtypes = [vp, vp, vp, vp]
    L.hb_rk_iterate.argtypes = [vp, vp, i32, vp, vp, vp]
    L.hb_forces.argtypes = [vp, vp, vp, vp]
    L.hb_residual_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.hb_forces_adjoint.argtypes = [vp, vp, vp, vp, vp, vp, vp]
    L.hb_adjoint_iterate.argtypes = [vp, vp, vp, vp, i32, vp, vp]
    L.hb_td_march.argtypes = [vp, vp, dp, dp, i32, vp]
    L.hb_td_march_noalloc.argtypes = [vp, vp, dp, dp, i32, vp]
    L.hb_save_state.argtypes = [vp, vp, i64, ctypes.c_char_p, vp]
    L.hb_load_state.argtypes = [vp, vp, ctypes.POINTER(i64), ctypes.c_char_p, vp]
    L.hb_save_solution.argtypes = [vp, vp, ctypes.c_char_p, vp]
    L.hb_autotune.argtypes = [vp, vp, ctypes.c_char_p, i32, ctypes.POINTER(c_tuning), vp]
    L.hb_set_tuning.argtypes = [vp, ctypes.POINTER(c_tuning)]
    L.hb_get_tuning.argtypes = [vp, ctypes.POINTER(c_tuning)]
    L.hb_set_xy.argtypes = [vp, vp, vp]
    L.hb_set_alpha0.argtypes = [vp, dp]
    L.hb_set_motion.argtypes = [vp, ctypes.POINTER(c_motion)]
    L.hb_get_status.argtypes = [vp]
    L.hb_profile_stages.argtypes = [vp, i32]
    L.hb_stage_stats.argtypes = [vp, ctypes.POINTER(dp), ctypes.POINTER(i64)]
    L.hb_last_error.restype = ctypes.c_char_p
    for f in EXPORTS:
        if f not in ("hb_state_size", "hb_forces_size", "hb_xy_size", "hb_last_error"):
            getattr(L, f).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc != HB_OK:
        raise HBError(rc, lib().hb_last_error().decode())


def _ptr(t: Optional[torch.Tensor], n: Optional[int], name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda \
            or not t.is_contiguous():
        raise TypeError("%s must be a contiguous float64 device tensor" % name)
    if n is not None and t.numel() != n:
        raise ValueError("%s has %d elements, expected %d" % (name, t.numel(), n))
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Grid:
    """A libhb grid built from blocks/flow/solver descriptions (any objects
    with the attributes of paper_1304_7654_amd.synth.Block/Flow/Solver)."""

    def __init__(self, blocks: Sequence, flow, solver, cuts: Sequence = (),
                 precision: Optional[int] = None, batched: Optional[int] = None):
        L = lib()
        self._keep = [np.ascontiguousarray(b.xy, dtype=np.float64) for b in blocks]
        cb = (c_block * len(blocks))()
        for k, b in enumerate(blocks):
            cb[k].ni, cb[k].nj, cb[k].n_harm = b.ni, b.nj, b.n_harm
            cb[k].xy = self._keep[k].ctypes.data_as(ctypes.POINTER(ctypes.c_double))
            for s in range(4):
                cb[k].bc[s] = int(b.bc[s])
            cb[k].wake_ncells = int(b.wake_ncells)
            cb[k].body_id = int(b.body_id)
        cc = (c_cut * max(1, len(cuts)))()
        for k, c in enumerate(cuts):
            if len(c) == 8:      # (blk_a, side_a, start_a, blk_b, side_b, start_b, len, reversed)
                vals = [int(x) for x in c]
            else:                # (blk_a, side_a, blk_b, side_b[, reversed]): whole sides
                a, sa, b, sb = (int(x) for x in c[:4])
                side = blocks[a].nj if sa < 2 else blocks[a].ni
                vals = [a, sa, 0, b, sb, 0, side, int(c[4]) if len(c) > 4 else 0]
            for name, v in zip(("blk_a", "side_a", "start_a", "blk_b", "side_b", "start_b",
                                "len", "reversed"), vals):
                setattr(cc[k], name, v)
        cf = c_flow(flow.mach, flow.reynolds, flow.prandtl, flow.gamma, flow.alpha0,
                    flow.alpha_amp, flow.k_red, flow.l_ref, flow.x_mom, flow.y_mom)
        cs = c_solver()
        cs.cfl = solver.cfl
        cs.n_stages = len(solver.rk_alpha)
        for k, a in enumerate(solver.rk_alpha):
            cs.rk_alpha[k] = a
        cs.precision = solver.precision if precision is None else precision
        cs.entropy_delta = solver.entropy_delta
        cs.limiter_eps = solver.limiter_eps
        cs.batched = solver.batched if batched is None else batched
        cs.graph_iters = solver.graph_iters
        h = ctypes.c_void_p()
        _check(L.hb_grid_create(cb, len(blocks), cc, len(cuts), ctypes.byref(cf),
                                ctypes.byref(cs), ctypes.byref(h)))
        self.h = h
        self.n_state = L.hb_state_size(h)
        self.n_forces = L.hb_forces_size(h)
        self.n_xy = L.hb_xy_size(h)
        self.precision = cs.precision
        self.batched = cs.batched

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            lib().hb_grid_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- entry points -----------------------------------------------------
    def residual(self, q: torch.Tensor, r: Optional[torch.Tensor] = None) -> torch.Tensor:
        if r is None:
            r = torch.empty_like(q)
        _check(lib().hb_residual(self.h, _ptr(q, self.n_state, "q"),
                                 _ptr(r, self.n_state, "r"), _stream()))
        return r

    def rk_iterate(self, q: torch.Tensor, n_iter: int, resnorm: Optional[torch.Tensor] = None,
                   forces: Optional[torch.Tensor] = None):
        _check(lib().hb_rk_iterate(self.h, _ptr(q, self.n_state, "q"), int(n_iter),
                                   _ptr(resnorm, n_iter, "resnorm"),
                                   _ptr(forces, self.n_forces, "forces"), _stream()))
        return q

    def forces(self, q: torch.Tensor, cf: Optional[torch.Tensor] = None) -> torch.Tensor:
        if cf is None:
            cf = torch.empty(self.n_forces, dtype=torch.float64, device=q.device)
        _check(lib().hb_forces(self.h, _ptr(q, self.n_state, "q"),
                               _ptr(cf, self.n_forces, "cf"), _stream()))
        return cf

    def residual_adjoint(self, q, rbar, qbar=None, xybar=None, flowbar=None):
        if qbar is None:
            qbar = torch.empty_like(q)
        _check(lib().hb_residual_adjoint(self.h, _ptr(q, self.n_state, "q"),
                                         _ptr(rbar, self.n_state, "rbar"),
                                         _ptr(qbar, self.n_state, "qbar"),
                                         _ptr(xybar, self.n_xy, "xybar"),
                                         _ptr(flowbar, 1, "flowbar"), _stream()))
        return qbar

    def forces_adjoint(self, q, cfbar, qbar=None, xybar=None, flowbar=None):
        if qbar is None:
            qbar = torch.empty_like(q)
        _check(lib().hb_forces_adjoint(self.h, _ptr(q, self.n_state, "q"),
                                       _ptr(cfbar, self.n_forces, "cfbar"),
                                       _ptr(qbar, self.n_state, "qbar"),
                                       _ptr(xybar, self.n_xy, "xybar"),
                                       _ptr(flowbar, 1, "flowbar"), _stream()))
        return qbar

    def adjoint_iterate(self, q, lam, gq, n_iter: int, resnorm=None):
        """n_iter adjoint pseudo-time iterations in place on lam towards
        J_Q^T lam = -gq at the state q."""
        _check(lib().hb_adjoint_iterate(self.h, _ptr(q, self.n_state, "q"),
                                        _ptr(lam, self.n_state, "lam"),
                                        _ptr(gq, self.n_state, "gq"), int(n_iter),
                                        _ptr(resnorm, n_iter, "resnorm"), _stream()))
        return lam

    def save_state(self, q: torch.Tensor, path: str, iteration: int = 0):
        _check(lib().hb_save_state(self.h, _ptr(q, self.n_state, "q"), int(iteration),
                                   str(path).encode(), _stream()))

    def load_state(self, q: torch.Tensor, path: str) -> int:
        """Read a restart file into q; returns the stored iteration counter."""
        it = ctypes.c_int64()
        _check(lib().hb_load_state(self.h, _ptr(q, self.n_state, "q"), ctypes.byref(it),
                                   str(path).encode(), _stream()))
        return it.value

    def save_solution(self, q: torch.Tensor, prefix: str):
        """Per-snapshot solution files <prefix>.snap<k> (nodes and primitives
        of every block with more than k snapshots, one write per file)."""
        _check(lib().hb_save_solution(self.h, _ptr(q, self.n_state, "q"), str(prefix).encode(),
                                      _stream()))

    def td_march(self, q: torch.Tensor, t0: float, dt: float, n_steps: int):
        """n_steps fourth-order Runge-Kutta steps in physical time from t0,
        in place on q (grids with n_harm = 0)."""
        _check(lib().hb_td_march(self.h, _ptr(q, self.n_state, "q"), float(t0), float(dt),
                                 int(n_steps), _stream()))
        return q

    def prepare(self, what: int):
        """Allocate now the scratch of the calls named by `what` (a bitwise
        OR of HB_PREPARE_ADJOINT, HB_PREPARE_ADJOINT_ITERATE, HB_PREPARE_TD)."""
        _check(lib().hb_prepare(self.h, int(what)))

    def td_march_noalloc(self, q: torch.Tensor, t0: float, dt: float, n_steps: int):
        """td_march without any device allocation (static per-device scratch
        of at most 2^21 doubles per state copy)."""
        _check(lib().hb_td_march_noalloc(self.h, _ptr(q, self.n_state, "q"), float(t0),
                                         float(dt), int(n_steps), _stream()))
        return q

    def autotune(self, q: torch.Tensor, cache_path: Optional[str] = None, force: bool = False):
        """Time the launch configurations of the batched kernel on a scratch
        copy of q, apply the fastest (or the cached choice); returns it."""
        t = c_tuning()
        _check(lib().hb_autotune(self.h, _ptr(q, self.n_state, "q"),
                                 None if cache_path is None else cache_path.encode(),
                                 1 if force else 0, ctypes.byref(t), _stream()))
        return t.as_dict()

    def set_tuning(self, tile_i: int = 16, wg_per_cu: int = 0, xcd_order: int = 1,
                   tile_order: int = 0):
        t = c_tuning(tile_i, wg_per_cu, xcd_order, tile_order, 0.0)
        _check(lib().hb_set_tuning(self.h, ctypes.byref(t)))

    def get_tuning(self) -> dict:
        t = c_tuning()
        _check(lib().hb_get_tuning(self.h, ctypes.byref(t)))
        return t.as_dict()

    def set_xy(self, xy: torch.Tensor):
        _check(lib().hb_set_xy(self.h, _ptr(xy, self.n_xy, "xy"), _stream()))

    def set_alpha0(self, a: float):
        _check(lib().hb_set_alpha0(self.h, float(a)))

    def set_motion(self, pitch_amp: float = 0.0, pitch_phase: float = 0.0, heave_amp: float = 0.0,
                   x_pivot: float = 0.0, y_pivot: float = 0.0):
        """Rigid heave and pitch of the whole grid (hb_set_motion); all zero
        amplitudes clear it."""
        m = c_motion(float(pitch_amp), float(pitch_phase), float(heave_amp), float(x_pivot),
                     float(y_pivot))
        _check(lib().hb_set_motion(self.h, ctypes.byref(m)))

    def status(self) -> int:
        return lib().hb_get_status(self.h)

    def profile_stages(self, enable: bool):
        _check(lib().hb_profile_stages(self.h, 1 if enable else 0))

    def stage_stats(self):
        """(summed milliseconds, number of stages) since the last call."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        _check(lib().hb_stage_stats(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value
