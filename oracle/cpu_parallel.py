"""ctypes wrapper of the multi-core CPU baseline (cpu_parallel.c).

BENCHMARK CONTEXT, NOT THE ORACLE: the benchmark's CPU-baseline leg times it
on all host cores beside the single-threaded oracle; the tests check it
against the oracle.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpuparallel.so")
SRC_PATH = os.path.join(HERE, "cpu_parallel.c")
_lib = None


def build(force: bool = True) -> str:
    """Compile cpu_parallel.c with gcc -O3 and OpenMP (AVX2-level x86-64)."""
    if force or not os.path.exists(LIB_PATH):
        tmp = LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-march=x86-64-v3", "-std=c99", "-fopenmp", "-Wall",
                               "-shared", "-fPIC", "-o", tmp, SRC_PATH, "-lm"])
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        v = ctypes.c_void_p
        L.cpb_dual_grad.argtypes = [ctypes.c_int64, ctypes.c_int64, v, v, v, v, v, v, v, v,
                                    ctypes.c_double, v, v, v]
        L.cpb_dual_grad.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


class Arrays:
    """The instance's arrays as the C function takes them (float64 values)."""

    def __init__(self, inst):
        self.m = int(inst.m)
        self.block_off = np.ascontiguousarray(inst.block_off, dtype=np.int64)
        self.block_proj = np.ascontiguousarray(inst.block_proj, dtype=np.uint8)
        self.dst = np.ascontiguousarray(inst.dst, dtype=np.int32)
        self.a = np.ascontiguousarray(inst.a, dtype=np.float64)
        self.c = np.ascontiguousarray(inst.c, dtype=np.float64)
        self.upper = None if inst.upper is None else np.ascontiguousarray(inst.upper, dtype=np.float64)
        self.b = np.ascontiguousarray(inst.b, dtype=np.float64)


def dual_grad(arr: Arrays, lam, gamma: float):
    """(g, grad, threads used) at lam."""
    lam = np.ascontiguousarray(lam, dtype=np.float64)
    grad = np.empty(arr.m)
    g = ctypes.c_double(0.0)
    nt = ctypes.c_int(0)
    rc = lib().cpb_dual_grad(arr.m, arr.block_off.shape[0] - 1, _p(arr.block_off), _p(arr.block_proj),
                             _p(arr.dst), _p(arr.a), _p(arr.c), _p(arr.upper), _p(arr.b), _p(lam),
                             float(gamma), _p(grad), ctypes.addressof(g), ctypes.addressof(nt))
    if rc:
        raise RuntimeError(f"cpb_dual_grad rc={rc}")
    return g.value, grad, nt.value
