"""Host-only checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects malformed problems before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2603_04621_amd import _lib as L
from paper_2603_04621_amd import api
from paper_2603_04621_amd import instances as I

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    txt = open(os.path.join(ROOT, "include", "dualip.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    names = re.findall(r"\b(dl_[a-z0-9_]+)\s*\(", txt)
    return sorted(set(n for n in names if not n.endswith("_t")))


def test_header_symbols_are_exported():
    names = header_functions()
    assert len(names) >= 15
    assert sorted(L.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    lib = L.lib()
    for n in names:
        assert hasattr(lib, n)


def test_status_strings():
    assert L.status_str(L.DL_OK) == "ok"
    assert L.status_str(L.DL_ERR_UNSUPPORTED) == "unsupported"
    assert L.status_str(99) == "unknown status"


def small():
    return I.random_small(5, I=30, J=6, dmax=5, box_frac=0.3)


def test_validate_accepts_good_problem_both_layouts():
    inst = small()
    assert api.validate(inst, "csc") == L.DL_OK
    assert api.validate(inst, "csr") == L.DL_OK
    assert api.validate(inst, "csc", storage="bf16", primal_scale=1) == L.DL_OK


def run_desc(mutate, opts_kw=None):
    inst = small()
    hd = api._HostDesc(inst, "csc")
    mutate(hd, inst)
    o, keep = api.make_opts(**(opts_kw or {}))
    st = L.lib().dl_problem_validate(ctypes.byref(hd.desc), ctypes.byref(o))
    return st, L.last_error()


def test_validate_rejects_malformed_input():
    def bad_row(hd, inst):
        hd.idx[3] = inst.m
    assert run_desc(bad_row)[0] == L.DL_ERR_INVALID_ARG

    def nan_c(hd, inst):
        hd.c[0] = np.nan
    st, msg = run_desc(nan_c)
    assert st == L.DL_ERR_INVALID_ARG and "c" in msg

    def bad_blocks(hd, inst):
        hd.block_off[2] = hd.block_off[1] - 1
    assert run_desc(bad_blocks)[0] == L.DL_ERR_INVALID_ARG

    def bad_end(hd, inst):
        hd.block_off[-1] = inst.n - 1
    assert run_desc(bad_end)[0] == L.DL_ERR_INVALID_ARG

    def bad_proj(hd, inst):
        hd.block_proj[0] = 7
    assert run_desc(bad_proj)[0] == L.DL_ERR_INVALID_ARG

    def neg_upper(hd, inst):
        hd.upper = np.ones(inst.n)
        hd.upper[1] = -1.0
        hd.desc.upper = hd.upper.ctypes.data
    assert run_desc(neg_upper)[0] == L.DL_ERR_INVALID_ARG

    def m_zero(hd, inst):
        hd.desc.m = 0
    assert run_desc(m_zero)[0] == L.DL_ERR_INVALID_ARG

    assert run_desc(lambda hd, inst: None, {"storage": "f32", "primal_scale": 2})[0] == \
        L.DL_ERR_INVALID_ARG
    st = L.lib().dl_problem_validate(None, None)
    assert st == L.DL_ERR_INVALID_ARG


def test_columns_with_several_entries():
    """Several matching families (Definition 1) and the count row: up to four
    entries per column are accepted in both layouts; a fifth is unsupported,
    as is deterministic mode with several entries per column."""
    multi = I.multi_family(I=20, J=4, families=3, count_row=True, seed=3, dmax=4)
    assert np.all(np.diff(multi.colptr) == 4)
    assert api.validate(multi, "csc") == L.DL_OK
    assert api.validate(multi, "csr") == L.DL_OK
    assert api.validate(multi, "csc", deterministic=True) == L.DL_ERR_UNSUPPORTED
    assert "one entry per column" in L.last_error()
    five = I.multi_family(I=20, J=4, families=4, count_row=True, seed=3, dmax=4)
    assert api.validate(five, "csc") == L.DL_ERR_UNSUPPORTED
    assert "at most 4" in L.last_error()
    assert api.validate(five, "csr") == L.DL_ERR_UNSUPPORTED


def test_csc_columns_may_repeat_a_row():
    """A column listing one row twice is two entries whose coefficients add."""
    inst = small()
    hd = api._HostDesc(inst, "csc")
    ptr = np.arange(inst.n + 1, dtype=np.int64)
    ptr[1:] += 1
    idx = np.concatenate([[hd.idx[0]], hd.idx]).astype(np.int32)
    val = np.concatenate([[1.0], hd.val])
    hd.desc.ptr = ptr.ctypes.data
    hd.desc.idx = idx.ctypes.data
    hd.desc.val = val.ctypes.data
    hd.desc.nnz = inst.n + 1
    o, _ = api.make_opts()
    assert L.lib().dl_problem_validate(ctypes.byref(hd.desc), ctypes.byref(o)) == L.DL_OK


def test_solve_opts_defaults():
    o = L.SolveOpts()
    L.lib().dl_solve_opts_init(ctypes.byref(o))
    assert o.gamma0 == 0.01 and o.max_step == o.gamma0
    assert o.init_step == pytest.approx(1e-2 * o.gamma0)
    assert o.check_every == 10 and o.momentum == 1 and o.adaptive == 1


def test_problem_opts_defaults_and_autotune_flag():
    """Defaults leave autotune off; a value other than 0 or 1 is rejected
    before any device work (so this runs without a GPU)."""
    o, _ = api.make_opts()
    assert o.storage == L.STORAGE["f32"] and o.row_normalize == 1 and o.primal_scale == 0
    assert o.autotune == 0 and o.deterministic == 0
    assert (o.lane_cap, o.seg_rmax, o.wg_min, o.chunks_per_cu) == (0, 0, 0, 0)
    inst = I.tiny()
    hd = api._HostDesc(inst, "csc")
    o.autotune = 2
    h = ctypes.c_void_p()
    st = L.lib().dl_problem_create(ctypes.byref(hd.desc), ctypes.byref(o), None, ctypes.byref(h))
    assert st == L.DL_ERR_INVALID_ARG and not h.value
    assert "autotune" in L.lib().dl_last_error().decode()


def test_solve_presets_host_side():
    """dl_solve_opts_apply_preset: PAPER reproduces Appendix B's fixed step
    sizes (max-step 1e-3, initial-step 1e-5 at gamma = 0.01, with |A'| = 1
    after row normalization of one family); NATURAL gives the classical
    1/L = gamma/|A'|^2 (Lemma 2's L); both scale with 1/|A'|^2; CUSTOM keeps
    the caller's values; unknown presets and non-positive norms are
    rejected."""
    import json
    with open(os.path.join(ROOT, "tests", "golden", "paper_hyperparameters.json")) as f:
        hp = json.load(f)
    s = api.SolveSettings(gamma0=hp["gamma"], max_step=7.0, init_step=3.0, preset="paper")
    r = api.apply_preset(s, 1.0)
    assert r.max_step == pytest.approx(hp["max_step_size"], rel=1e-15)
    assert r.init_step == pytest.approx(hp["initial_step_size"], rel=1e-15)
    r4 = api.apply_preset(s, 4.0)
    assert r4.max_step == pytest.approx(hp["max_step_size"] / 4, rel=1e-15)
    n = api.apply_preset(api.SolveSettings(gamma0=0.05, preset="natural"), 2.0)
    assert n.max_step == pytest.approx(0.05 / 2.0, rel=1e-15)
    assert n.init_step == pytest.approx(1e-2 * 0.05 / 2.0, rel=1e-15)
    c = api.apply_preset(api.SolveSettings(gamma0=0.05, max_step=7.0, init_step=3.0), 9.0)
    assert (c.max_step, c.init_step) == (7.0, 3.0)
    o = s.to_c(None)
    o.preset = 9
    assert L.lib().dl_solve_opts_apply_preset(ctypes.byref(o), 1.0) == L.DL_ERR_INVALID_ARG
    o.preset = L.DL_PRESET_PAPER
    assert L.lib().dl_solve_opts_apply_preset(ctypes.byref(o), 0.0) == L.DL_ERR_INVALID_ARG
    assert L.lib().dl_solve_opts_apply_preset(ctypes.byref(o), float("nan")) == L.DL_ERR_INVALID_ARG


def test_work_layout_fields_are_validated():
    """Layout fields by hand: 0 and positive values pass, negative ones and
    more than 8 workgroups per compute unit are rejected on the host."""
    inst = small()
    assert api.validate(inst, work_layout={"lane_cap": 8, "seg_rmax": 2, "wg_min": 100,
                                            "chunks_per_cu": 8}) == L.DL_OK
    for bad in ({"lane_cap": -1}, {"seg_rmax": -2}, {"wg_min": -5}, {"chunks_per_cu": 9}):
        assert api.validate(inst, work_layout=bad) == L.DL_ERR_INVALID_ARG
        assert "layout" in L.last_error()
    with pytest.raises(KeyError):
        api.make_opts(work_layout={"lanes": 3})
