"""dl_dual_grad_noalloc (static library scratch, no allocation) against
dl_dual_grad on the same problems, through the C ABI.

Two calls in a row on different problems, the second smaller than the
first, so the second runs on scratch that still holds the first call's
contents.  The first problem has rows beyond LDS (FP64 accumulators in the
scratch) and box blocks; both calls request x and the scalars.

Bar (as for the oracle parity tests): gradient per destination within
1e-5 (sum_{e->j} |a_e x_e| + |b_j|), g and P within 1e-6; x is computed in
registers from the same stored values by the same kernel, so it must be
bitwise equal.
"""
import ctypes

import numpy as np
import pytest

from paper_2603_04621_amd import instances as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def _lam(inst, seed):
    rng = np.random.default_rng(seed)
    return rng.exponential(2.0, size=inst.m) * (rng.random(inst.m) < 0.8)


def _check_pair(inst, storage, lam, gamma):
    from paper_2603_04621_amd.api import Problem
    with Problem(inst, storage=storage) as p:
        info = p.info()
        lt = torch.from_numpy(lam)
        g_ref, x_ref, e_ref = p.dual_grad(lt, gamma, want_x=True, want_eval=True)
        out = (torch.empty(inst.m, dtype=torch.float64, device="cuda"),
               torch.full((inst.n,), -1.0, dtype=torch.float64, device="cuda"))
        g_na, x_na, e_na = p.dual_grad(lt, gamma, want_x=True, want_eval=True, noalloc=True,
                                       out=out)
        torch.cuda.synchronize()
    g_ref, x_ref = g_ref.cpu().numpy(), x_ref.cpu().numpy()
    g_na, x_na = g_na.cpu().numpy(), x_na.cpu().numpy()
    a = inst.rounded(storage).a
    scale = np.bincount(inst.dst, weights=np.abs(a * x_ref), minlength=inst.m) + np.abs(inst.b)
    gerr = np.abs(g_na - g_ref) / np.maximum(scale, 1e-300)
    gerr[(scale == 0) & (g_na == g_ref)] = 0.0
    assert float(gerr.max()) <= 1e-5, float(gerr.max())
    assert np.array_equal(x_na, x_ref)
    assert abs(e_na["g"] - e_ref["g"]) <= 1e-6 * max(1.0, abs(e_ref["g"]))
    pmag = abs(e_ref["cx"]) + abs(e_ref["reg"])
    assert abs(e_na["P"] - e_ref["P"]) <= 1e-6 * max(1.0, pmag)
    assert abs(e_na["max_infeas"] - e_ref["max_infeas"]) <= 1e-6 * max(1.0, abs(e_ref["max_infeas"]))
    return info


def test_noalloc_matches_dual_grad_two_calls(dev):
    big = I.heavy(I=12_000, J=20_000, dmax=4096, capacity="greedy")
    info = _check_pair(big, "f32", _lam(big, 1), 1e-2)
    assert info["lds_rows"] < big.m          # rows beyond LDS used the scratch accumulators
    small = I.tiny(capacity="greedy")
    assert small.m < big.m and small.n < big.n
    _check_pair(small, "f64", _lam(small, 2), 1e-3)


def test_noalloc_rejects_problem_beyond_scratch(dev):
    from paper_2603_04621_amd import _lib as L
    from paper_2603_04621_amd.api import Problem
    # 32 B of row scratch per destination: 2.5M destinations need more than
    # the 64 MiB array holds
    inst = I.random_small(3, I=200, J=2_500_000, dmax=8)
    with Problem(inst, storage="f32") as p:
        lam = torch.zeros(inst.m, dtype=torch.float64, device="cuda")
        grad = torch.zeros(inst.m, dtype=torch.float64, device="cuda")
        st = L.lib().dl_dual_grad_noalloc(p.handle, lam.data_ptr(), 1e-2, grad.data_ptr(), None,
                                          None, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        assert st == L.DL_ERR_UNSUPPORTED
        assert "scratch" in L.last_error()
        # the problem still evaluates through the allocating entry point
        p.dual_grad(lam, 1e-2)


def test_noalloc_columns_with_several_entries(dev):
    """Two families and the count row: the allocation-free call (its
    restoration pass takes the row ratios and partials from the static
    scratch too) equals dl_dual_grad."""
    from paper_2603_04621_amd.api import Problem
    inst = I.multi_family(I=5_000, J=300, families=2, count_row=True, seed=31, box_frac=0.3)
    lam = torch.from_numpy(np.random.default_rng(7).exponential(0.5, size=inst.m))
    with Problem(inst, storage="f32") as p:
        g_ref, x_ref, e_ref = p.dual_grad(lam, 1e-2, want_x=True, want_eval=True)
        g_na, x_na, e_na = p.dual_grad(lam, 1e-2, want_x=True, want_eval=True, noalloc=True)
    g_ref, g_na = g_ref.cpu().numpy(), g_na.cpu().numpy()
    x_ref = x_ref.cpu().numpy()
    cols = np.repeat(np.arange(inst.n), np.diff(inst.colptr))
    val = inst.rounded("f32").val
    scale = np.bincount(inst.rowidx, weights=np.abs(val * x_ref[cols]), minlength=inst.m) + \
        np.abs(inst.b)
    assert float(np.max(np.abs(g_na - g_ref) / np.maximum(scale, 1e-300))) <= 1e-5
    assert np.array_equal(x_na.cpu().numpy(), x_ref)
    assert abs(e_na["g"] - e_ref["g"]) <= 1e-6 * max(1.0, abs(e_ref["g"]))
    assert abs(e_na["P"] - e_ref["P"]) <= 1e-6 * max(1.0, abs(e_ref["cx"]) + abs(e_ref["reg"]))
