"""ctypes wrapper of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE: imported only by the test suite, the smoke check and
the benchmark's CPU-baseline leg.  It shares no code with the GPU library
and never imports it.  Instances come in as plain numpy arrays (the
``paper_2603_04621_amd.instances.Instance`` fields), in original units.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")
SRC_PATH = os.path.join(HERE, "oracle.c")

SIMPLEX = 0
BOX = 1
CAPPED = 2
TRACE_W = 6


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C99, no FMA contraction)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
                               "-Wall", "-shared", "-fPIC", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


class _LP(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64),
                ("colptr", ctypes.c_void_p), ("rowidx", ctypes.c_void_p),
                ("val", ctypes.c_void_p), ("c", ctypes.c_void_p), ("b", ctypes.c_void_p),
                ("nblocks", ctypes.c_int64), ("block_off", ctypes.c_void_p),
                ("block_proj", ctypes.c_void_p), ("upper", ctypes.c_void_p),
                ("v", ctypes.c_void_p)]


class _Eval(ctypes.Structure):
    _fields_ = [(k, ctypes.c_double) for k in ("g", "cx", "reg", "P", "rel_gap", "max_infeas")]


class _Opts(ctypes.Structure):
    _fields_ = [("gamma0", ctypes.c_double), ("gamma_final", ctypes.c_double),
                ("n_stages", ctypes.c_int32), ("row_normalize", ctypes.c_int32),
                ("stage_iters", ctypes.c_int64), ("stage_tol", ctypes.c_double),
                ("tol_rel_gap", ctypes.c_double), ("max_iters", ctypes.c_int64),
                ("check_every", ctypes.c_int64), ("max_step", ctypes.c_double),
                ("init_step", ctypes.c_double), ("momentum", ctypes.c_int32),
                ("adaptive", ctypes.c_int32)]


class _Res(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int64), ("converged", ctypes.c_int32),
                ("stage", ctypes.c_int32), ("gamma", ctypes.c_double), ("g", ctypes.c_double),
                ("P", ctypes.c_double), ("rel_gap", ctypes.c_double),
                ("max_infeas", ctypes.c_double)]


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        L.orc_project_block.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p]
        L.orc_dual_eval.argtypes = [ctypes.POINTER(_LP), ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(_Eval)]
        L.orc_row_scale.argtypes = [ctypes.POINTER(_LP), ctypes.c_void_p]
        L.orc_colnorm_scale.argtypes = [ctypes.POINTER(_LP), ctypes.c_void_p]
        L.orc_solve.argtypes = [ctypes.POINTER(_LP), ctypes.POINTER(_Opts), ctypes.c_void_p,
                                ctypes.POINTER(_Res), ctypes.c_void_p]
        _LIB = L
    return _LIB


def _p(a):
    return None if a is None else a.ctypes.data


class LP:
    """Holds contiguous float64/int arrays of one LP and its ctypes view."""

    def __init__(self, m, n, rowidx, val, c, b, block_off, block_proj, upper=None,
                 v=None, colptr=None):
        self.m, self.n = int(m), int(n)
        self.colptr = None if colptr is None else np.ascontiguousarray(colptr, dtype=np.int64)
        self.rowidx = np.ascontiguousarray(rowidx, dtype=np.int32)
        self.val = np.ascontiguousarray(val, dtype=np.float64)
        self.c = np.ascontiguousarray(c, dtype=np.float64)
        self.b = np.ascontiguousarray(b, dtype=np.float64)
        self.block_off = np.ascontiguousarray(block_off, dtype=np.int64)
        self.block_proj = np.ascontiguousarray(block_proj, dtype=np.uint8)
        self.upper = None if upper is None else np.ascontiguousarray(upper, dtype=np.float64)
        self.v = None if v is None else np.ascontiguousarray(v, dtype=np.float64)
        self.s = _LP(self.m, self.n, _p(self.colptr), _p(self.rowidx), _p(self.val),
                     _p(self.c), _p(self.b), self.block_off.shape[0] - 1, _p(self.block_off),
                     _p(self.block_proj), _p(self.upper), _p(self.v))

    @classmethod
    def from_instance(cls, inst, v=None) -> "LP":
        if hasattr(inst, "colptr"):        # several entries per column (CSC)
            return cls(inst.m, inst.n, inst.rowidx, inst.val, inst.c, inst.b, inst.block_off,
                       inst.block_proj, inst.upper, v, colptr=inst.colptr)
        return cls(inst.m, inst.n, inst.dst, inst.a, inst.c, inst.b, inst.block_off,
                   inst.block_proj, inst.upper, v)


@dataclass
class Eval:
    x: np.ndarray
    grad: np.ndarray
    g: float
    cx: float
    reg: float
    P: float
    rel_gap: float
    max_infeas: float


def project_block(proj: int, t, w, u=None):
    """(x, tau) of one block, t and w float64 arrays."""
    t = np.ascontiguousarray(t, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = None if u is None else np.ascontiguousarray(u, dtype=np.float64)
    x = np.empty_like(t)
    tau = ctypes.c_double(0.0)
    rc = lib().orc_project_block(int(proj), t.shape[0], _p(t), _p(w), _p(u), _p(x),
                                 ctypes.addressof(tau))
    if rc:
        raise RuntimeError(f"orc_project_block rc={rc}")
    return x, tau.value


def dual_eval(lp, lam, gamma: float, v=None) -> Eval:
    """x*(lam), grad g(lam) and scalars at lam (original units)."""
    if not isinstance(lp, LP):
        lp = LP.from_instance(lp, v)
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    x = np.empty(lp.n)
    grad = np.empty(lp.m)
    ev = _Eval()
    rc = lib().orc_dual_eval(ctypes.byref(lp.s), _p(lam), float(gamma), _p(x), _p(grad),
                             ctypes.byref(ev))
    if rc:
        raise RuntimeError(f"orc_dual_eval rc={rc}")
    return Eval(x, grad, ev.g, ev.cx, ev.reg, ev.P, ev.rel_gap, ev.max_infeas)


def row_scale(lp, v=None) -> np.ndarray:
    if not isinstance(lp, LP):
        lp = LP.from_instance(lp, v)
    D = np.empty(lp.m)
    lib().orc_row_scale(ctypes.byref(lp.s), _p(D))
    return D


def colnorm_scale(lp) -> np.ndarray:
    if not isinstance(lp, LP):
        lp = LP.from_instance(lp)
    v = np.empty(lp.n)
    lib().orc_colnorm_scale(ctypes.byref(lp.s), _p(v))
    return v


@dataclass
class SolveOpts:
    gamma0: float = 1e-2
    gamma_final: float = 1e-2
    n_stages: int = 1
    row_normalize: int = 1
    stage_iters: int = 0
    stage_tol: float = 0.0
    tol_rel_gap: float = 1e-4
    max_iters: int = 1000
    check_every: int = 10
    max_step: float = 1e-3
    init_step: float = 1e-5
    momentum: int = 1
    adaptive: int = 1


@dataclass
class SolveResult:
    lam: np.ndarray
    iters: int
    converged: bool
    stage: int
    gamma: float
    g: float
    P: float
    rel_gap: float
    max_infeas: float
    trace: Optional[np.ndarray]


def solve(lp, opts: SolveOpts, lam0=None, v=None, trace: bool = True) -> SolveResult:
    if not isinstance(lp, LP):
        lp = LP.from_instance(lp, v)
    lam = np.zeros(lp.m) if lam0 is None else np.array(lam0, dtype=np.float64)
    o = _Opts(opts.gamma0, opts.gamma_final, opts.n_stages, opts.row_normalize,
              opts.stage_iters, opts.stage_tol, opts.tol_rel_gap, opts.max_iters,
              opts.check_every, opts.max_step, opts.init_step, opts.momentum, opts.adaptive)
    tr = np.full((max(opts.max_iters, 1), TRACE_W), np.nan) if trace else None
    r = _Res()
    rc = lib().orc_solve(ctypes.byref(lp.s), ctypes.byref(o), _p(lam), ctypes.byref(r), _p(tr))
    if rc:
        raise RuntimeError(f"orc_solve rc={rc}")
    if tr is not None:
        tr = tr[: r.iters]
    return SolveResult(lam, r.iters, bool(r.converged), r.stage, r.gamma, r.g, r.P,
                       r.rel_gap, r.max_infeas, tr)
