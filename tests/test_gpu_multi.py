"""GPU parity for columns with several entries: several matching families
(Definition 1) and the global count row (Section 4), against the FP64 oracle.

Tolerances as in test_gpu_parity.py: gradient per row within 1e-5 of
sum_{e} |A_re x_e| + |b_r|, g within 1e-6 relative (FP64 storage: 1e-12),
the restored primal value P within 1e-6 of |c'x| + gamma/2 |x|^2 (P is
built from per-edge restoration ratios, whose inputs are f32 row partials),
per-edge x within the rounding bound of t and tau.
"""
import numpy as np
import pytest

from paper_2603_04621_amd import instances as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def O():
    from oracle import oracle
    oracle.lib()
    return oracle


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def problem(inst, storage="f32", **kw):
    from paper_2603_04621_amd.api import Problem
    return Problem(inst, storage=storage, **kw)


def lam_for(inst, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return rng.exponential(scale, size=inst.m) * (rng.random(inst.m) < 0.8)


def compare_multi(O, inst, storage, lam, gamma, g_tol=1e-6, layout="csc"):
    ref = inst.rounded(storage)
    ev = O.dual_eval(ref, lam, gamma)
    with problem(inst, storage, layout=layout) as p:
        info = p.info()
        grad, x, e = p.dual_grad(torch.from_numpy(lam), gamma, want_x=True, want_eval=True)
        grad, x = grad.cpu().numpy(), x.cpu().numpy()
    cols = np.repeat(np.arange(inst.n), np.diff(inst.colptr))
    scale = np.bincount(inst.rowidx, weights=np.abs(ref.val * ev.x[cols]), minlength=inst.m) + \
        np.abs(inst.b)
    gerr = np.abs(grad - ev.grad) / np.maximum(scale, 1e-300)
    gerr[(scale == 0) & (grad == ev.grad)] = 0.0
    assert gerr.max() <= 1e-5, float(gerr.max())
    assert abs(e["g"] - ev.g) <= g_tol * max(1.0, abs(ev.g)), (e["g"], ev.g)
    pmag = float(np.sum(np.abs(ref.c * ev.x)) + 0.5 * gamma * np.sum(ev.x ** 2))
    assert abs(e["P"] - ev.P) <= 1e-6 * max(1.0, pmag), (e["P"], ev.P)
    # per edge: both sides compute clamp(w (t - tau), 0, u) in FP64 from the
    # same stored values; t carries a few ulps of |c| + sum |a lam|
    mag = np.abs(ref.c) + np.bincount(cols, weights=np.abs(ref.val * lam[inst.rowidx]), minlength=inst.n)
    deg = np.diff(inst.block_off)
    bid = np.repeat(np.arange(deg.size), deg)
    bmax = np.zeros(deg.size)
    np.maximum.at(bmax, bid, mag)
    tol = 64 * np.finfo(np.float64).eps / gamma * bmax[bid] * np.maximum(deg[bid], 1) + 1e-15
    bad = np.nonzero(np.abs(x - ev.x) > tol)[0]
    assert bad.size == 0, (bad[:5], np.abs(x - ev.x)[bad[:5]], tol[bad[:5]])
    return info


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_two_families_and_count_row_all_paths(O, dev, storage):
    """Two families plus the count row (three entries per column); degrees
    1..1500 so blocks run on one lane, on 4/16/64-lane segments and on whole
    workgroups; simplex, box and capped blocks; several prices and gammas."""
    inst = I.multi_family(I=6_000, J=2_000, families=2, count_row=True, seed=21, box_frac=0.25,
                          capped_frac=0.25, dmax=1500)
    deg = np.diff(inst.block_off)
    assert deg.max() > 512 and np.sum(deg <= 8) > 0
    for seed, gamma in ((1, 1e-1), (2, 1e-2), (3, 1e-3)):
        info = compare_multi(O, inst, storage, lam_for(inst, seed, 0.5), gamma,
                             g_tol=1e-12 if storage == "f64" else 1e-6)
    assert info["col_entries"] == 3
    assert info["lane_groups"] > 0 and info["seg_groups"] > 0 and info["wg_blocks"] > 0


def test_three_families_rows_beyond_lds_and_csr(O, dev):
    """Three families without the count row over 3 x 8,000 rows, more than
    LDS holds (the rows beyond take global accumulators); the CSR layout of
    the same matrix gives the same result."""
    inst = I.multi_family(I=40_000, J=8_000, families=3, count_row=False, seed=22, box_frac=0.3)
    info = compare_multi(O, inst, "f32", lam_for(inst, 4, 0.5), 1e-2)
    assert info["lds_rows"] < inst.m
    compare_multi(O, inst, "f64", lam_for(inst, 5, 0.5), 1e-2, g_tol=1e-12, layout="csr")


def test_full_size_two_families_and_count_row(O, dev):
    """The timed multi-entry workload at full size: 2M sources, two families
    of 10k destinations and the count row (20,001 rows, 60,015,519 entries),
    FP32, 80% simplex / 20% box blocks.  The ordinary pass (no x, no
    scalars) and the gap check with its restoration pass against the
    oracle's evaluation of every row and edge."""
    inst = I.multi_family(I=2_000_000, J=10_000, families=2, count_row=True, box_frac=0.2)
    lam = lam_for(inst, 6, 0.5)
    gamma = 1e-3
    ref = inst.rounded("f32")
    ev = O.dual_eval(ref, lam, gamma)
    with problem(inst) as p:
        grad, _, _ = p.dual_grad(torch.from_numpy(lam), gamma)
        grad = grad.cpu().numpy()
    cols = np.repeat(np.arange(inst.n), np.diff(inst.colptr))
    scale = np.bincount(inst.rowidx, weights=np.abs(ref.val * ev.x[cols]), minlength=inst.m) + \
        np.abs(inst.b)
    gerr = np.abs(grad - ev.grad) / np.maximum(scale, 1e-300)
    gerr[(scale == 0) & (grad == ev.grad)] = 0.0
    assert gerr.max() <= 1e-5, float(gerr.max())
    del ev, grad, gerr, scale, cols
    info = compare_multi(O, inst, "f32", lam, gamma)
    assert info["col_entries"] == 3 and info["lds_rows"] < inst.m


def test_iteration_norm_by_power_iteration(dev):
    """|A'|^2 of the iteration matrix (rows normalised) from the host's power
    iteration equals the largest eigenvalue of A'A'^T (within its 1e-3
    margin, from above)."""
    inst = I.multi_family(I=300, J=20, families=2, count_row=True, seed=23, dmax=8)
    A = inst.dense()
    rn = np.sqrt((A ** 2).sum(axis=1))
    D = np.where(rn > 0, 1.0 / np.where(rn > 0, rn, 1.0), 1.0)
    lmax = np.linalg.eigvalsh((D[:, None] * A) @ (D[:, None] * A).T).max()
    with problem(inst) as p:
        a2 = p.info()["anorm2"]
    assert lmax <= a2 <= lmax * (1 + 1.2e-3), (a2, lmax)
    assert lmax > 1.5          # not diagonal any more (one family would give 1)


def test_solve_trajectory_fp64(O, dev):
    """300 accelerated iterations with a gap check every 10 (each with the
    restoration pass) follow the oracle's g, gap and prices."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.multi_family(I=3_000, J=100, families=2, count_row=True, seed=24, box_frac=0.3,
                          dmax=30)
    s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=300, check_every=10,
                      tol_rel_gap=-1.0, max_step=2e-3, init_step=1e-5, trace=True)
    r_or = O.solve(inst, O.SolveOpts(gamma0=s.gamma0, gamma_final=s.gamma_final, max_iters=300,
                                     check_every=10, tol_rel_gap=-1.0, max_step=s.max_step,
                                     init_step=s.init_step))
    with problem(inst, "f64") as p:
        lam, r = p.solve(s)
    assert r.iters == 300 == r_or.iters
    rel = np.abs(r.trace[:, 0] - r_or.trace[:, 0]) / np.maximum(1.0, np.abs(r_or.trace[:, 0]))
    assert rel.max() <= 1e-6, (rel.max(), int(rel.argmax()))
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6
    lo = lam.cpu().numpy()
    assert np.max(np.abs(lo - r_or.lam)) <= 1e-5 * max(1.0, np.max(np.abs(r_or.lam)))


def test_continuation_solve_gap_certified(O, dev):
    """Continuation with the natural preset (steps from the power-iteration
    |A'|^2): at the GPU's final prices the oracle reproduces g and the
    reported gap, and the gap went down to 1e-4."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.multi_family(I=50_000, J=500, families=2, count_row=True, seed=25, box_frac=0.2)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-2, n_stages=3, stage_iters=3000,
                      stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=12000, check_every=10,
                      preset="natural")
    with problem(inst, "f32") as p:
        lam, r = p.solve(s)
    assert r.converged, r
    ev = O.dual_eval(inst.rounded("f32"), lam.cpu().numpy(), r.gamma)
    assert abs(ev.g - r.g) <= 1e-6 * max(1.0, abs(ev.g))
    assert abs(ev.rel_gap - r.rel_gap) <= 1e-6
    assert ev.rel_gap <= 1.01e-4


def test_batched_and_served_reject_several_entries(dev):
    from paper_2603_04621_amd import _lib as L
    from paper_2603_04621_amd.api import Server, SolveSettings, batch_solve
    inst = I.multi_family(I=200, J=10, families=2, count_row=False, seed=26, dmax=5)
    with problem(inst) as p:
        with pytest.raises(L.DualipError) as ei:
            batch_solve([p], SolveSettings(max_iters=10))
        assert ei.value.status == L.DL_ERR_UNSUPPORTED
    srv = Server(hbm_budget_bytes=1e9, max_slots=2)
    try:
        with pytest.raises(L.DualipError) as ei:
            srv.submit(inst, SolveSettings(max_iters=10))
        assert ei.value.status == L.DL_ERR_UNSUPPORTED
    finally:
        srv.close()
