"""Python face of libdualip: marshals numpy/torch arrays into the C ABI.

Every computation runs in the HIP library; this module only builds the
descriptors, hands over device pointers (torch tensors on the current ROCm
device) and the current HIP stream, and checks status codes.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _lib as L


def _np_ptr(a):
    return None if a is None else a.ctypes.data


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class _HostDesc:
    """Keeps the contiguous host arrays alive while the descriptor is in use."""

    def __init__(self, inst, layout: str = "csc"):
        self.m, self.n = int(inst.m), int(inst.n)
        multi = hasattr(inst, "colptr")      # several entries per column
        if layout == "csc" and multi:
            self.ptr = np.ascontiguousarray(inst.colptr, dtype=np.int64)
            self.idx = np.ascontiguousarray(inst.rowidx, dtype=np.int32)
            self.val = np.ascontiguousarray(inst.val, dtype=np.float64)
            lay = L.DL_CSC
        elif layout == "csc":
            self.ptr = None
            self.idx = np.ascontiguousarray(inst.dst, dtype=np.int32)
            self.val = np.ascontiguousarray(inst.a, dtype=np.float64)
            lay = L.DL_CSC
        elif layout == "csr":
            rp, ci, v = inst.csr()
            self.ptr = np.ascontiguousarray(rp, dtype=np.int64)
            self.idx = np.ascontiguousarray(ci, dtype=np.int32)
            self.val = np.ascontiguousarray(v, dtype=np.float64)
            lay = L.DL_CSR
        else:
            raise ValueError(layout)
        self.c = np.ascontiguousarray(inst.c, dtype=np.float64)
        self.b = np.ascontiguousarray(inst.b, dtype=np.float64)
        self.block_off = np.ascontiguousarray(inst.block_off, dtype=np.int64)
        self.block_proj = np.ascontiguousarray(inst.block_proj, dtype=np.uint8)
        self.upper = None if inst.upper is None else np.ascontiguousarray(inst.upper, np.float64)
        self.desc = L.ProblemDesc(self.m, self.n, self.idx.shape[0], lay, _np_ptr(self.ptr),
                                  _np_ptr(self.idx), _np_ptr(self.val), _np_ptr(self.c),
                                  _np_ptr(self.b), self.block_off.shape[0] - 1,
                                  _np_ptr(self.block_off), _np_ptr(self.block_proj),
                                  _np_ptr(self.upper))


LAYOUT_KEYS = ("lane_cap", "seg_rmax", "wg_min", "chunks_per_cu")


def make_opts(storage: str = "f32", row_normalize: bool = True, primal_scale: int = 0, v=None,
              autotune: bool = False, deterministic: bool = False, work_layout=None):
    """dl_problem_opts; work_layout: dict with any of LAYOUT_KEYS (0 = default)."""
    o = L.ProblemOpts()
    L.lib().dl_problem_opts_init(ctypes.byref(o))
    o.storage = L.STORAGE[storage]
    o.row_normalize = 1 if row_normalize else 0
    o.primal_scale = int(primal_scale)
    o.autotune = 1 if autotune else 0
    o.deterministic = 1 if deterministic else 0
    for k, val in (work_layout or {}).items():
        if k not in LAYOUT_KEYS:
            raise KeyError(k)
        setattr(o, k, int(val))
    keep = None
    if v is not None:
        keep = np.ascontiguousarray(v, dtype=np.float64)
        o.v = keep.ctypes.data
    return o, keep


def apply_preset(settings: "SolveSettings", anorm2: float = 1.0) -> "SolveSettings":
    """The settings with max_step and init_step resolved by the C library's
    dl_solve_opts_apply_preset for an iteration matrix of squared norm
    anorm2 (host only)."""
    o = settings.to_c(None)
    L.check(L.lib().dl_solve_opts_apply_preset(ctypes.byref(o), float(anorm2)),
            "dl_solve_opts_apply_preset")
    return SolveSettings(**{**settings.__dict__, "max_step": o.max_step,
                            "init_step": o.init_step})


def validate(inst, layout: str = "csc", **opts) -> int:
    """dl_problem_validate (host only).  Returns the status code."""
    hd = _HostDesc(inst, layout)
    o, _keep = make_opts(**opts)
    return L.lib().dl_problem_validate(ctypes.byref(hd.desc), ctypes.byref(o))


@dataclass
class SolveSettings:
    """Mirrors dl_solve_opts (include/dualip.h)."""
    gamma0: float = 0.01
    gamma_final: float = 0.01
    n_stages: int = 1
    momentum: int = 1
    stage_iters: int = 0
    stage_tol: float = 0.0
    tol_rel_gap: float = 1e-4
    max_iters: int = 10000
    check_every: int = 10
    max_step: float = 0.01
    init_step: float = 1e-4
    adaptive: int = 1
    warm_start: int = 0
    graph_iters: int = 0
    time_kernels: int = 0
    trace: bool = False
    preset: str = "custom"          # "custom" | "paper" | "natural" (dl_preset)

    def to_c(self, trace_buf=None) -> L.SolveOpts:
        o = L.SolveOpts()
        L.lib().dl_solve_opts_init(ctypes.byref(o))
        for k in ("gamma0", "gamma_final", "n_stages", "momentum", "stage_iters", "stage_tol",
                  "tol_rel_gap", "max_iters", "check_every", "max_step", "init_step",
                  "adaptive", "warm_start", "graph_iters", "time_kernels"):
            setattr(o, k, getattr(self, k))
        o.preset = L.PRESET[self.preset]
        o.trace_host = None if trace_buf is None else trace_buf.ctypes.data
        return o


@dataclass
class SolveOutcome:
    status: int
    converged: bool
    stage: int
    iters: int
    gamma: float
    g: float
    P: float
    rel_gap: float
    max_infeas: float
    seconds: float
    grad_kernel_ms: float
    grad_launches: int
    check_kernel_ms: float = 0.0
    check_launches: int = 0
    trace: Optional[np.ndarray] = field(default=None, repr=False)


def outcome(r: L.SolveResult, trace=None) -> SolveOutcome:
    return SolveOutcome(r.status, bool(r.converged), r.stage, r.iters, r.gamma, r.g, r.P,
                        r.rel_gap, r.max_infeas, r.seconds, r.grad_kernel_ms, r.grad_launches,
                        r.check_kernel_ms, r.check_launches,
                        None if trace is None else trace[: r.iters])


class Problem:
    """A matching LP created on the current HIP device (dl_problem_create)."""

    def __init__(self, inst, storage: str = "f32", row_normalize: bool = True,
                 primal_scale: int = 0, v=None, layout: str = "csc", stream=None,
                 autotune: bool = False, deterministic: bool = False, work_layout=None):
        import torch
        self.m, self.n = int(inst.m), int(inst.n)
        self.device = torch.device("cuda", torch.cuda.current_device())
        hd = _HostDesc(inst, layout)
        o, _keep = make_opts(storage, row_normalize, primal_scale, v, autotune, deterministic,
                             work_layout)
        h = ctypes.c_void_p()
        L.check(L.lib().dl_problem_create(ctypes.byref(hd.desc), ctypes.byref(o),
                                          _stream(stream), ctypes.byref(h)), "dl_problem_create")
        self._h = h

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        i = L.ProblemInfo()
        L.check(L.lib().dl_problem_get_info(self._h, ctypes.byref(i)), "dl_problem_get_info")
        return {k: getattr(i, k) for k, _ in L.ProblemInfo._fields_}

    def dual_grad(self, lam, gamma: float, want_x: bool = False, want_eval: bool = False,
                  stream=None, noalloc: bool = False, out=None):
        """(grad [m] fp64 tensor, x [n] or None, dict of scalars or None).

        noalloc=True calls dl_dual_grad_noalloc (static library scratch); out
        may pass preallocated (grad, x) tensors so that the call itself
        allocates nothing on the device either."""
        import torch
        lam = lam.to(device=self.device, dtype=torch.float64).contiguous()
        if out is not None:
            grad, x = out
        else:
            grad = torch.empty(self.m, dtype=torch.float64, device=self.device)
            x = torch.empty(self.n, dtype=torch.float64, device=self.device) if want_x else None
        ev = L.Eval() if want_eval else None
        fn = L.lib().dl_dual_grad_noalloc if noalloc else L.lib().dl_dual_grad
        L.check(fn(self._h, lam.data_ptr(), float(gamma), grad.data_ptr(),
                   None if x is None else x.data_ptr(),
                   ctypes.byref(ev) if ev is not None else None,
                   _stream(stream)), "dl_dual_grad_noalloc" if noalloc else "dl_dual_grad")
        evd = None if ev is None else {k: getattr(ev, k) for k, _ in L.Eval._fields_}
        return grad, x, evd

    def time_grad_kernel(self, lam, gamma: float, iters: int = 10, check: bool = False,
                         stream=None) -> float:
        import torch
        lam = lam.to(device=self.device, dtype=torch.float64).contiguous()
        ms = ctypes.c_double()
        L.check(L.lib().dl_time_grad_kernel(self._h, lam.data_ptr(), float(gamma), int(iters),
                                            1 if check else 0, ctypes.byref(ms), _stream(stream)),
                "dl_time_grad_kernel")
        return ms.value

    def solve(self, settings: SolveSettings, lam0=None, stream=None):
        """(lam tensor [m], SolveOutcome); lam0 warm-starts when given."""
        import torch
        lam = torch.zeros(self.m, dtype=torch.float64, device=self.device)
        st = SolveSettings(**{**settings.__dict__})
        if lam0 is not None:
            lam.copy_(lam0.to(device=self.device, dtype=torch.float64))
            st.warm_start = 1
        tr = np.full((max(st.max_iters, 1), L.DL_TRACE_W), np.nan) if st.trace else None
        o = st.to_c(tr)
        r = L.SolveResult()
        L.check(L.lib().dl_solve(self._h, ctypes.byref(o), lam.data_ptr(), ctypes.byref(r),
                                 _stream(stream)),
                "dl_solve", ok=(L.DL_OK, L.DL_ERR_NOT_CONVERGED))
        return lam, outcome(r, tr)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().dl_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def batch_solve(problems, settings: SolveSettings, lam0s=None, stream=None):
    """dl_batch_solve over several Problems: (list of lam tensors, list of SolveOutcome)."""
    import torch
    n = len(problems)
    lams = []
    st = SolveSettings(**{**settings.__dict__})
    st.trace = False
    for k, p in enumerate(problems):
        lam = torch.zeros(p.m, dtype=torch.float64, device=p.device)
        if lam0s is not None and lam0s[k] is not None:
            lam.copy_(lam0s[k].to(device=p.device, dtype=torch.float64))
            st.warm_start = 1
        lams.append(lam)
    hs = (ctypes.c_void_p * n)(*[p.handle.value for p in problems])
    ls = (ctypes.c_void_p * n)(*[l.data_ptr() for l in lams])
    res = (L.SolveResult * n)()
    o = st.to_c(None)
    L.check(L.lib().dl_batch_solve(hs, n, ctypes.byref(o), ls, res, _stream(stream)),
            "dl_batch_solve", ok=(L.DL_OK, L.DL_ERR_NOT_CONVERGED))
    return lams, [outcome(r) for r in res]


class Server:
    """dl_server: continuous batching of solve requests on the current device."""

    def __init__(self, hbm_budget_bytes: float = 200e9, max_slots: int = 64):
        h = ctypes.c_void_p()
        L.check(L.lib().dl_server_create(int(hbm_budget_bytes), int(max_slots), ctypes.byref(h)),
                "dl_server_create")
        self._h = h
        self._m = {}

    def submit(self, inst, settings: SolveSettings, storage: str = "f32", **popts) -> int:
        hd = _HostDesc(inst)
        o, _keep = make_opts(storage, **popts)
        t = ctypes.c_uint64()
        L.check(L.lib().dl_server_submit(self._h, ctypes.byref(hd.desc), ctypes.byref(o),
                                         ctypes.byref(settings.to_c(None)), ctypes.byref(t)),
                "dl_server_submit")
        self._m[t.value] = inst.m
        return t.value

    def times(self, ticket: int):
        ts, tb, td = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        L.check(L.lib().dl_server_times(self._h, ticket, ctypes.byref(ts), ctypes.byref(tb),
                                        ctypes.byref(td)), "dl_server_times")
        return ts.value, tb.value, td.value

    def poll(self, ticket: int):
        """None while running; else (SolveOutcome, lam ndarray, (t_submit, t_start, t_done))."""
        ts, tb, td = self.times(ticket)
        if td <= 0.0:
            return None
        done = ctypes.c_int32()
        r = L.SolveResult()
        lam = np.empty(self._m[ticket])
        L.check(L.lib().dl_server_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(r),
                                       lam.ctypes.data), "dl_server_poll")
        if not done.value:
            return None
        del self._m[ticket]
        return outcome(r), lam, (ts, tb, td)

    def close(self):
        if getattr(self, "_h", None):
            L.lib().dl_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
