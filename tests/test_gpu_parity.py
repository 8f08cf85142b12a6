"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle.

Tolerances (per destination j, per edge e, at identical lam and identical
stored inputs -- the oracle reads the values the device store holds):
  gradient   |G_gpu - G_orc|_j <= 1e-5 (sum_{e->j} |a_e x_e| + |b_j|)
  objective  |g_gpu - g_orc| <= 1e-6 max(1, |g_orc|)
  active set every edge whose oracle x is more than 2e-5 away from a class
             boundary (0, the box bound) is classified alike; every simplex
             block whose oracle sum is more than 2e-5 from 1 likewise.
The per-destination sums are f32 partials in LDS whatever the storage type
(combined in FP64 across workgroups), so FP64 storage meets the same gradient
bound (observed ~1e-7); its dual objective, which does not go through those
sums (g = -t'x + gamma/2 |D_v x|^2 - lam'b), matches to 1e-12.
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


def gpu_problem(inst, storage="f32", **kw):
    from paper_2603_04621_amd.api import Problem
    return Problem(inst, storage=storage, **kw)


def compare(O, inst, storage, lam, gamma, grad_tol=1e-5, g_tol=1e-6, layout="csc", v=None,
            primal_scale=0, autotune=False, deterministic=False, work_layout=None):
    """Runs one evaluation on both sides; returns the measured errors."""
    ref_inst = inst.rounded(storage)
    vv = None
    if primal_scale == 1:
        vv = np.abs(inst.a)
        vv[vv == 0] = 1.0
    elif primal_scale == 2:
        vv = v
    v_dev = None
    if vv is not None:
        # the device keeps 1/v^2 in float32
        v_dev = 1.0 / np.sqrt((1.0 / vv ** 2).astype(np.float32).astype(np.float64))
    ev = O.dual_eval(ref_inst, lam, gamma, v=v_dev)
    with gpu_problem(inst, storage, layout=layout, primal_scale=primal_scale, v=v,
                     autotune=autotune, deterministic=deterministic, work_layout=work_layout) as p:
        grad, x, e = p.dual_grad(torch.from_numpy(lam), gamma, want_x=True, want_eval=True)
        grad = grad.cpu().numpy()
        x = x.cpu().numpy()
        # the same evaluation without x (the solve's form: some paths, such
        # as wave-streamed blocks with one active edge, skip work when x is
        # not written)
        grad_nx, _, e_nx = p.dual_grad(torch.from_numpy(lam), gamma, want_x=False, want_eval=True)
        grad_nx = grad_nx.cpu().numpy()
    scale = np.bincount(inst.dst, weights=np.abs(ref_inst.a * ev.x), minlength=inst.m) + np.abs(inst.b)
    gerr = np.abs(grad - ev.grad) / np.maximum(scale, 1e-300)
    gerr[(scale == 0) & (grad == ev.grad)] = 0.0
    gerr_nx = np.abs(grad_nx - ev.grad) / np.maximum(scale, 1e-300)
    gerr_nx[(scale == 0) & (grad_nx == ev.grad)] = 0.0
    assert (gerr_nx.max() if gerr_nx.size else 0.0) <= grad_tol, float(gerr_nx.max())
    assert abs(e_nx["g"] - ev.g) / max(1.0, abs(ev.g)) <= g_tol, (e_nx["g"], ev.g)
    v2 = vv ** 2 if vv is not None else 1.0
    pmag = float(np.sum(np.abs(ref_inst.c * ev.x)) + 0.5 * gamma * np.sum(v2 * ev.x ** 2))
    out = {"grad": float(gerr.max()) if gerr.size else 0.0,
           "g": abs(e["g"] - ev.g) / max(1.0, abs(ev.g)),
           # P is built from f32 per-destination partial sums of c x and
           # v^2 x^2, whose error is relative to the summed magnitudes; the
           # two parts of P cancel, so it is measured against those
           "P": abs(e["P"] - ev.P) / max(1.0, pmag),
           "cx": abs(e["cx"] - ev.cx) / max(1.0, abs(ev.cx)),
           "infeas": abs(e["max_infeas"] - ev.max_infeas) / max(1.0, abs(ev.max_infeas)),
           "x_abs": float(np.max(np.abs(x - ev.x))) if x.size else 0.0}
    assert out["grad"] <= grad_tol, out
    assert out["g"] <= g_tol, out
    assert out["P"] <= 1e-6, out
    assert abs(e_nx["P"] - ev.P) / max(1.0, pmag) <= 1e-6, (e_nx["P"], ev.P)
    assert_x_close(ref_inst, lam, gamma, vv if v_dev is None else v_dev, ev.x, x)
    check_active_sets(ref_inst, ev.x, x)
    return out


def assert_x_close(inst, lam, gamma, v, xo, xg):
    """Per-edge x.  Both sides compute x = clamp(w (t - tau), 0, u) in FP64
    from the same stored values, so they differ by rounding only: t = -(c +
    a lam) carries a few ulps of |c| + |a lam|, tau (a sort-based threshold
    on one side, a fixed point on the other) a few ulps of the block's
    largest such magnitude times its degree, and w = 1/(gamma v^2) scales
    both.  The bound allows 64 ulps of that magnitude per block edge, which
    a wrong threshold or a wrong edge order exceeds by orders."""
    deg = np.diff(inst.block_off)
    bid = np.repeat(np.arange(deg.size), deg)
    mag = np.abs(inst.c) + np.abs(inst.a * lam[inst.dst])
    bmax = np.zeros(deg.size)
    np.maximum.at(bmax, bid, mag)
    w = 1.0 / (gamma * (np.ones(inst.n) if v is None else v ** 2))
    tol = 64 * np.finfo(np.float64).eps * w * bmax[bid] * np.maximum(deg[bid], 1) + 1e-15
    err = np.abs(xg - xo)
    bad = np.nonzero(err > tol)[0]
    assert bad.size == 0, (f"{bad.size} edges with |x_gpu - x_orc| above the rounding bound, "
                           f"e.g. {bad[:5]}: {err[bad[:5]]} vs {tol[bad[:5]]}")


def check_active_sets(inst, xo, xg, thr=1e-5, band=2e-5):
    u = inst.upper if inst.upper is not None else np.ones(inst.n)
    # edges with a bound u (box and capped blocks) have a third class at u
    box = np.repeat(inst.block_proj != I.PROJ_SIMPLEX, np.diff(inst.block_off))
    cls_o = np.where(xo <= thr, 0, np.where(box & (u - xo <= thr), 2, 1))
    cls_g = np.where(xg <= thr, 0, np.where(box & (u - xg <= thr), 2, 1))
    far = (np.abs(xo - thr) > band) & (~box | (np.abs((u - xo) - thr) > band))
    bad = np.nonzero(far & (cls_o != cls_g))[0]
    assert bad.size == 0, f"{bad.size} edges change class, e.g. {bad[:5]}"
    sums_o = np.add.reduceat(xo, inst.block_off[:-1]) if inst.n else np.zeros(0)
    sums_g = np.add.reduceat(xg, inst.block_off[:-1]) if inst.n else np.zeros(0)
    nonempty = np.diff(inst.block_off) > 0
    simp = (inst.block_proj != I.PROJ_BOX) & nonempty      # blocks with sum x <= 1
    bind_o = sums_o >= 1 - thr
    bind_g = sums_g >= 1 - thr
    farb = np.abs(sums_o - (1 - thr)) > band
    assert not np.any(simp & farb & (bind_o != bind_g))


def lam_close(a, b, tol=1e-5):
    """Dual iterates agree to tol relative to the largest price."""
    return float(np.max(np.abs(a - b), initial=0.0)) <= tol * max(1.0, float(np.max(np.abs(b), initial=0.0)))


def lam_for(inst, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    # typical dual values: a fraction of the per-edge cost scale, some rows at 0
    lam = rng.exponential(scale, size=inst.m) * (rng.random(inst.m) < 0.8)
    return lam


# --------------------------------------------------------------------------
# dual gradient at identical lam
# --------------------------------------------------------------------------

@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("gamma", [1e-1, 1e-3])
def test_grad_tiny_uniform(O, dev, storage, gamma):
    inst = I.tiny(capacity="greedy")
    for seed in range(3):
        lam = lam_for(inst, seed, 0.5) if seed else np.zeros(inst.m)
        compare(O, inst, storage, lam, gamma, g_tol=1e-12 if storage == "f64" else 1e-6)


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_grad_mixed_degrees_all_paths(O, dev, storage):
    """Degrees 1..1500: one-lane blocks, blocks on 4, 16 and 64 lanes (every
    row class, full and compacted last rows) and workgroup blocks, simplex
    and box, several groups per class and ragged last groups."""
    rng = np.random.default_rng(11)
    deg = np.concatenate([rng.integers(1, 33, size=3000), rng.integers(33, 65, size=150),
                          rng.integers(65, 257, size=60), rng.integers(257, 1025, size=16),
                          rng.integers(1025, 1500, size=4)])
    rng.shuffle(deg)
    inst = I._finish("mixed", 11, deg.size, 2000, deg, rng, I.zipf_cdf(2000, 1.1),
                     I._neg_lognormal, I._lognormal_a, 0.3, box_frac=0.3, capacity="greedy",
                     seed_key=[11, 1])
    with gpu_problem(inst, storage) as p:
        info = p.info()
    assert info["lane_groups"] > 0 and info["seg_groups"] > 0 and info["wg_blocks"] > 0
    for seed, gamma in ((1, 1e-2), (2, 1e-3)):
        compare(O, inst, storage, lam_for(inst, seed, 1.0), gamma)


def test_grad_zipf_large_degree_config_shape(O, dev):
    inst = I.large(I=200_000, J=2_000, capacity="greedy")
    compare(O, inst, "f32", lam_for(inst, 3, 2.0), 1e-3)


@pytest.mark.parametrize("workload,storage", [("large", "f32"), ("heavy", "f32"), ("large", "bf16")])
def test_grad_full_size_workloads(O, dev, workload, storage):
    """The two timed workloads at full size, default layout: 10M sources x
    10k destinations (100,007,779 nonzeros, every row in LDS; FP32 and BF16
    storage) and the heavy-tailed 2M x 50k (60,145,687 nonzeros, rows beyond
    LDS; FP32).  The ordinary pass the solve runs (no x, no scalars) and the
    gap-check pass (x and scalars) against the oracle's evaluation of every
    row and edge on the same stored values, at the tolerances of the smaller
    cases."""
    inst = (I.large if workload == "large" else I.heavy)(capacity="greedy")
    lam = lam_for(inst, 17, 2.0)
    gamma = 1e-3
    ref = inst.rounded(storage)
    ev = O.dual_eval(ref, lam, gamma)
    with gpu_problem(inst, storage) as p:
        info = p.info()
        grad, _, _ = p.dual_grad(torch.from_numpy(lam), gamma)
        grad = grad.cpu().numpy()
    assert (info["lds_rows"] == inst.m) == (workload == "large")
    scale = np.bincount(inst.dst, weights=np.abs(ref.a * ev.x), minlength=inst.m) + np.abs(inst.b)
    gerr = np.abs(grad - ev.grad) / np.maximum(scale, 1e-300)
    gerr[(scale == 0) & (grad == ev.grad)] = 0.0
    assert gerr.max() <= 1e-5, float(gerr.max())
    del ev, grad, gerr, scale
    compare(O, inst, storage, lam, gamma)


def test_grad_check_sums_partly_in_lds(O, dev):
    """J = 10k destinations, all in LDS: the gap-check pass keeps lam and the
    a x sums of every row in LDS but the c x and v^2 x^2 sums of only the
    first rows (the rest through global accumulators)."""
    inst = I.large(I=150_000, J=10_000, capacity="greedy")
    with gpu_problem(inst) as p:
        assert p.info()["lds_rows"] == inst.m
    compare(O, inst, "f32", lam_for(inst, 15, 2.0), 1e-3)
    compare(O, inst, "f64", lam_for(inst, 16, 2.0), 1e-2, grad_tol=1e-5)


def test_grad_heavy_tailed_mixed(O, dev):
    inst = I.heavy(I=20_000, J=4_000, dmax=4096, capacity="greedy")
    compare(O, inst, "f32", lam_for(inst, 4, 2.0), 1e-2)
    compare(O, inst, "bf16", lam_for(inst, 5, 2.0), 1e-2)


def test_grad_heavy_tailed_rows_beyond_lds(O, dev):
    """Heavy-tailed blocks on every lane width with more destinations than
    LDS holds (the tail-row variant of each path)."""
    inst = I.heavy(I=12_000, J=20_000, dmax=4096, capacity="greedy")
    with gpu_problem(inst) as p:
        info = p.info()
    assert info["lds_rows"] < inst.m and info["seg_groups"] > 0 and info["wg_blocks"] > 0
    compare(O, inst, "f32", lam_for(inst, 12, 2.0), 1e-2)
    compare(O, inst, "f64", lam_for(inst, 13, 2.0), 1e-2, grad_tol=1e-5)


def test_grad_rows_beyond_lds(O, dev):
    """More destinations than fit in LDS: the tail rows take the global path."""
    inst = I.large(I=60_000, J=20_000, capacity="greedy")
    with gpu_problem(inst) as p:
        info = p.info()
    assert info["lds_rows"] < inst.m
    compare(O, inst, "f32", lam_for(inst, 6, 2.0), 1e-3)
    compare(O, inst, "f64", lam_for(inst, 7, 2.0), 1e-2, grad_tol=1e-5)


def test_autotuned_layout_matches_oracle(O, dev):
    """A problem built with autotune (layouts timed on a sample of its blocks
    at the prices of a short solve) reports the chosen layout and gives the
    oracle's gradient."""
    inst = I.heavy(I=12_000, J=3_000, dmax=2048, capacity="greedy")
    with gpu_problem(inst, "f32", autotune=True) as p:
        info = p.info()
    assert info["tuned"] == 1 and info["chunks_per_cu"] in (1, 2)
    assert info["lane_cap"] in (8, 16, 24, 32) and info["seg_rmax"] in (4, 8, 12, 16)
    assert info["wg_min"] in (0, 256, 512, 1024)
    compare(O, inst, "f32", lam_for(inst, 14, 2.0), 1e-2, autotune=True)


@pytest.mark.parametrize("wl", [
    {"lane_cap": 8, "seg_rmax": 4, "wg_min": 256, "chunks_per_cu": 2},
    {"wg_min": 33},
    {"lane_cap": 1, "seg_rmax": 1, "chunks_per_cu": 3},
    {"lane_cap": 24, "seg_rmax": 12, "wg_min": 512},
])
def test_work_layouts_by_hand(O, dev, wl):
    """Layouts set by hand (the tuner's search space and its corners: every
    block of more than one edge on segments, blocks from 33 edges on whole
    workgroups) give the oracle's gradient on simplex, box and capped blocks
    of degrees 1..2048, in both storages; the info reports the layout."""
    inst = I.heavy(I=6_000, J=2_000, dmax=2048, capacity="greedy", box_frac=0.3, capped_frac=0.2,
                   seed=31)
    with gpu_problem(inst, "f32", work_layout=wl) as p:
        info = p.info()
    for k, val in wl.items():
        if k == "wg_min":
            assert info[k] == max(val, info["lane_cap"] + 1)
        else:
            assert info[k] == val, (k, info[k])
    assert info["wg_blocks"] > 0 and info["tuned"] == 0
    compare(O, inst, "f32", lam_for(inst, 15, 1.0), 1e-2, work_layout=wl)
    compare(O, inst, "f64", lam_for(inst, 16, 1.0), 1e-3, grad_tol=1e-5, work_layout=wl)


@pytest.mark.parametrize("J", [10_224, 10_225, 13_632, 13_633])
def test_lds_capacity_edges(O, dev, J):
    """Destinations at the edges of the LDS capacities of gfx950's 160 KB:
    up to 10,224 rows all stay in LDS with FP64 sums in ordinary passes; one
    more row puts the coldest beyond LDS (10,224 kept); from 13,633 rows on,
    13,632 rows stay with f32 sums.  Ordinary and gap-check passes match the
    oracle on each side."""
    inst = I.large(I=40_000, J=J, capacity="greedy")
    with gpu_problem(inst) as p:
        rows = p.info()["lds_rows"]
    expect = {10_224: 10_224, 10_225: 10_224, 13_632: 10_224, 13_633: 13_632}[J]
    assert rows == expect, (J, rows)
    compare(O, inst, "f32", lam_for(inst, 17, 2.0), 1e-3)
    compare(O, inst, "f64", lam_for(inst, 18, 2.0), 1e-2, grad_tol=1e-5)


def test_grad_csr_equals_csc(O, dev):
    inst = I.random_small(21, I=500, J=40, dmax=30, box_frac=0.3)
    lam = lam_for(inst, 8)
    a = compare(O, inst, "f64", lam, 1e-2, layout="csr", g_tol=1e-12)
    b = compare(O, inst, "f64", lam, 1e-2, layout="csc", g_tol=1e-12)
    assert a["g"] <= 1e-12 and b["g"] <= 1e-12


@pytest.mark.parametrize("ps", [1, 2])
def test_grad_primal_scaling(O, dev, ps):
    inst = I.random_small(22, I=800, J=50, dmax=40, box_frac=0.3)
    v = np.random.default_rng(3).uniform(0.5, 2.0, size=inst.n) if ps == 2 else None
    compare(O, inst, "f64", lam_for(inst, 9), 1e-2, primal_scale=ps, v=v)


def test_edge_cases(O, dev):
    rng = np.random.default_rng(5)
    # empty blocks, degree-1 blocks, one block per item kind, zero box bounds
    deg = np.array([0, 1, 3, 0, 17, 1, 0, 600, 2])
    inst = I._finish("edge", 5, deg.size, 700, deg, rng, I.uniform_cdf(700), I._neg_lognormal,
                     I._lognormal_a, 0.3, box_frac=0.5, capacity="greedy", seed_key=[5, 1])
    assert list(np.diff(inst.block_off)) == list(deg)
    if inst.upper is not None:
        inst.upper[:3] = 0.0
    for lam in (np.zeros(inst.m), np.full(inst.m, 1e6), lam_for(inst, 1, 0.7)):
        compare(O, inst, "f64", lam, 1e-2, grad_tol=1e-5)
    # a single destination
    deg = np.ones(50, dtype=np.int64)
    one = I._finish("one", 6, 50, 1, deg, rng, I.uniform_cdf(1), I._neg_lognormal,
                    I._lognormal_a, 0.3, box_frac=0.5, capacity="greedy", seed_key=[6, 1])
    for lam in (np.zeros(1), np.array([1e6]), np.array([0.7])):
        compare(O, one, "f64", lam, 1e-2, grad_tol=1e-5)
    # all x = 0 (huge prices)
    inst = I.random_small(23, I=100, J=10, dmax=20)
    compare(O, inst, "f32", np.full(inst.m, 1e8), 1e-3)
    # a block longer than a workgroup holds in registers (multi-pass path)
    deg = np.array([5000, 3, 40, 1, 700])
    big = I._finish("big", 7, deg.size, 6000, deg, rng, I.uniform_cdf(6000), I._neg_lognormal,
                    I._lognormal_a, 0.3, box_frac=0.0, capacity="greedy", seed_key=[7, 1])
    for lam in (np.zeros(big.m), lam_for(big, 2, 0.7)):
        compare(O, big, "f32", lam, 1e-2)
        compare(O, big, "f64", lam, 1e-2, grad_tol=1e-5)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_grad_capped_all_paths(O, dev, storage):
    """Capped-simplex blocks {0 <= x <= u, sum x <= 1} beside simplex and box
    blocks on every work path: one-lane blocks, blocks on 4, 16 and 64 lanes,
    workgroup blocks in registers and beyond them (multi-pass), at gammas
    where the caps bind, the sum binds, or neither."""
    rng = np.random.default_rng(31)
    deg = np.concatenate([rng.integers(1, 33, size=2000), rng.integers(33, 65, size=120),
                          rng.integers(65, 257, size=50), rng.integers(257, 1025, size=16),
                          rng.integers(1025, 4096, size=6), np.array([4500, 5200, 6000])])
    rng.shuffle(deg)
    inst = I._finish("capped", 31, deg.size, 7000, deg, rng, I.zipf_cdf(7000, 1.1),
                     I._neg_lognormal, I._lognormal_a, 0.3, box_frac=0.2, capped_frac=0.5,
                     capacity="greedy", seed_key=[31, 1])
    capped = inst.block_proj == I.PROJ_CAPPED
    assert capped.sum() > 100 and np.max(np.diff(inst.block_off)[capped]) > 4096
    with gpu_problem(inst, storage) as p:
        info = p.info()
    assert info["lane_groups"] > 0 and info["seg_groups"] > 0 and info["wg_blocks"] > 0
    for seed, gamma in ((1, 1e-1), (2, 1e-2), (3, 1e-3)):
        compare(O, inst, storage, lam_for(inst, seed, 1.0), gamma,
                g_tol=1e-12 if storage == "f64" else 1e-6)
    # huge prices: every x = 0; zero prices: every block's positive part
    compare(O, inst, storage, np.zeros(inst.m), 1e-2)
    compare(O, inst, storage, np.full(inst.m, 1e6), 1e-2)


def test_grad_capped_rows_beyond_lds_and_primal_scale(O, dev):
    """Capped blocks with destinations beyond LDS (tail variant) and with
    per-edge weights w = 1/(gamma v^2) (primal scaling)."""
    inst = I.heavy(I=12_000, J=20_000, dmax=4096, capacity="greedy", capped_frac=0.4)
    with gpu_problem(inst) as p:
        assert p.info()["lds_rows"] < inst.m
    compare(O, inst, "f32", lam_for(inst, 41, 2.0), 1e-2)
    small = I.random_small(42, I=800, J=50, dmax=300, box_frac=0.2, capped_frac=0.5)
    v = np.random.default_rng(4).uniform(0.5, 2.0, size=small.n)
    compare(O, small, "f64", lam_for(small, 43), 1e-2, primal_scale=2, v=v)
    compare(O, small, "f64", lam_for(small, 44), 1e-2, primal_scale=1)


def test_grad_appendix_b_workload(O, dev):
    """The paper's own synthetic construction (Appendix B): row norms that
    differ by orders of magnitude, Poisson resource degrees; prices scaled
    per row (lam_j ~ Exp(1) / s_j) so that every row has active edges."""
    inst = I.appendix_b(I=60_000, J=400, seed=4621)
    rng = np.random.default_rng(52)
    lam = rng.exponential(1.0, size=inst.m) / inst.meta["s"]
    for storage, gamma in (("f64", 1e-2), ("f32", 1e-2), ("f32", 1e-3), ("bf16", 1e-2)):
        compare(O, inst, storage, lam, gamma, g_tol=1e-12 if storage == "f64" else 1e-6)


def test_solve_appendix_b_gap_certified(O, dev):
    """Continuation to gap 1e-4 on the Appendix B workload (Jacobi rows):
    the oracle at the GPU's final prices reproduces g and certifies the gap."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.appendix_b(I=60_000, J=400, seed=4622)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-2, n_stages=4, stage_iters=2000,
                      stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=8000, check_every=10,
                      preset="natural")
    with gpu_problem(inst, "f32") as p:
        lam, r = p.solve(s)
    assert r.converged, r
    ev = O.dual_eval(inst.rounded("f32"), lam.cpu().numpy(), r.gamma)
    assert abs(ev.g - r.g) <= 1e-6 * max(1.0, abs(ev.g))
    assert ev.rel_gap <= 1.01e-4


def _bitwise_twice(p, lam, gamma):
    """Two evaluations with x and scalars, and two without: identical bits."""
    lt = torch.from_numpy(lam)
    g1, x1, e1 = p.dual_grad(lt, gamma, want_x=True, want_eval=True)
    g2, x2, e2 = p.dual_grad(lt, gamma, want_x=True, want_eval=True)
    assert torch.equal(g1, g2) and torch.equal(x1, x2)
    assert e1 == e2, (e1, e2)
    g3, _, _ = p.dual_grad(lt, gamma)
    g4, _, _ = p.dual_grad(lt, gamma)
    assert torch.equal(g3, g4) and torch.equal(g1, g3)


def test_deterministic_mode_bitwise_and_oracle_parity(O, dev):
    """deterministic = 1: fixed-point integer sums (LDS and global) make
    repeated evaluations and solves bit-identical, on a problem with rows
    beyond LDS and box blocks and on one whose gap-check sums are partly in
    LDS; both still match the oracle to the usual tolerances."""
    from paper_2603_04621_amd.api import SolveSettings
    heavy = I.heavy(I=12_000, J=20_000, dmax=4096, capacity="greedy", capped_frac=0.2)
    large = I.large(I=150_000, J=10_000, capacity="greedy")
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-2, n_stages=3, stage_iters=50,
                      tol_rel_gap=-1.0, max_iters=200, check_every=10, preset="natural")
    for inst, seed in ((heavy, 61), (large, 62)):
        lam = lam_for(inst, seed, 2.0)
        compare(O, inst, "f32", lam, 1e-2, deterministic=True)
        with gpu_problem(inst, "f32", deterministic=True) as p:
            info = p.info()
            assert info["deterministic"] == 1
            _bitwise_twice(p, lam, 1e-2)
            la, ra = p.solve(s)
            lb, rb = p.solve(s)
            assert torch.equal(la, lb) and ra.g == rb.g and ra.rel_gap == rb.rel_gap
        if inst is heavy:
            assert info["lds_rows"] < inst.m
    # the same solve without the flag differs from the deterministic one by
    # rounding only
    with gpu_problem(large, "f32") as p:
        lc, rc = p.solve(s)
    assert abs(rc.g - ra.g) <= 1e-6 * max(1.0, abs(ra.g))
    assert lam_close(lc.cpu().numpy(), la.cpu().numpy(), tol=1e-4)


def tie_instance(gamma, seed=11):
    """Blocks of every item kind (lam = 0, a = 1, so t = -c) with the largest
    t = 3/4 and the second 3/4 (a tie), 3/4 - gamma/2 or 3/4 - 3 gamma/2; the
    other t lie in [1/4, 1/2].  With gamma = 1/64 every value sits on a grid
    that bf16, f32 and f64 store exactly."""
    rng = np.random.default_rng(seed)
    J = 2500
    degs, cs = [], []
    for d in (2, 3, 10, 30, 40, 100, 500, 2000):
        for case in ("tie", "near", "gap", "gap") * 3:
            c = -np.round(rng.uniform(0.25, 0.5, size=d) * 64) / 64
            top, second = rng.choice(d, size=2, replace=False)
            c[top] = -0.75
            c[second] = -0.75 + {"tie": 0.0, "near": 0.5 * gamma, "gap": 1.5 * gamma}[case]
            degs.append(d)
            cs.append(c)
    deg = np.array(degs, dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    n = int(off[-1])
    dst = np.concatenate([rng.choice(J, size=d, replace=False) for d in deg]).astype(np.int32)
    a = np.ones(n)
    c = np.concatenate(cs)
    b = 0.3 * np.bincount(dst, weights=a, minlength=J)
    return I.Instance(J, n, dst, a, c, b, off, np.zeros(deg.size, dtype=np.uint8), None,
                      "ties", seed)


@pytest.mark.parametrize("storage", ["f64", "f32", "bf16"])
def test_grad_ties_and_near_ties(O, dev, storage):
    # the simplex threshold skips its fixed-point passes only when the second
    # largest t is at most max t - gamma; exact ties and near ties must take
    # the full passes and still match the oracle (gamma on the value grid)
    gamma = 1.0 / 64
    inst = tie_instance(gamma)
    compare(O, inst, storage, np.zeros(inst.m), gamma)
    with gpu_problem(inst, storage) as p:
        _, x, _ = p.dual_grad(torch.zeros(inst.m, dtype=torch.float64), gamma, want_x=True)
        x = x.cpu().numpy()
    for i in range(inst.block_off.shape[0] - 1):
        xb = x[inst.block_off[i]:inst.block_off[i + 1]]
        k = i % 4
        pos = int(np.sum(xb > 0))
        # tie: two edges at 1/2 each; near: two edges (3/4, 1/4); gap: one edge at 1
        assert pos == (1 if k == 2 or k == 3 else 2), (i, pos)
        assert abs(xb.sum() - 1.0) < 1e-9
    compare(O, inst, storage, lam_for(inst, 3, 0.01), gamma)


def test_grad_repeatable(dev):
    """Repeated evaluations differ only by the order of the f32 LDS atomic
    adds: far inside the gradient tolerance; g (which does not use those sums)
    is reproduced exactly up to FP64 summation order of fixed partials."""
    inst = I.large(I=100_000, J=1_000)
    lam = torch.from_numpy(lam_for(inst, 10))
    with gpu_problem(inst) as p:
        g1, x1, e1 = p.dual_grad(lam, 1e-3, want_x=True, want_eval=True)
        g2, x2, e2 = p.dual_grad(lam, 1e-3, want_x=True, want_eval=True)
    assert torch.equal(x1, x2)
    scale = np.bincount(inst.dst, weights=np.abs(inst.a * x1.cpu().numpy()), minlength=inst.m) + inst.b
    assert np.max(np.abs((g1 - g2).cpu().numpy()) / scale) <= 1e-6
    assert e1["g"] == e2["g"]


# --------------------------------------------------------------------------
# solve: trajectory against the oracle
# --------------------------------------------------------------------------

def oracle_opts(O, s):
    return O.SolveOpts(gamma0=s.gamma0, gamma_final=s.gamma_final, n_stages=s.n_stages,
                       row_normalize=1, stage_iters=s.stage_iters, stage_tol=s.stage_tol,
                       tol_rel_gap=s.tol_rel_gap, max_iters=s.max_iters,
                       check_every=s.check_every, max_step=s.max_step, init_step=s.init_step,
                       momentum=s.momentum, adaptive=s.adaptive)


@pytest.mark.parametrize("graph", [0, 1])
def test_solve_tiny_trajectory_fp64(O, dev, graph):
    """1,000 accelerated iterations at gamma = 1e-3 with the paper's step
    sizes, FP64 storage: g along the run and at the end within 1e-6."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.tiny(capacity="greedy")
    s = SolveSettings(gamma0=1e-3, gamma_final=1e-3, max_iters=1000, check_every=0,
                      tol_rel_gap=0.0, max_step=1e-3, init_step=1e-5, trace=True,
                      time_kernels=0 if graph else 1, graph_iters=16 if graph else 0)
    r_or = O.solve(inst, oracle_opts(O, s))
    with gpu_problem(inst, "f64") as p:
        lam, r = p.solve(s)
    assert r.iters == 1000 == r_or.iters
    tr_g, tr_o = r.trace[:, 0], r_or.trace[:, 0]
    rel = np.abs(tr_g - tr_o) / np.maximum(1.0, np.abs(tr_o))
    assert rel.max() <= 1e-6, (rel.max(), int(rel.argmax()))
    assert abs(r.g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g))
    assert lam_close(lam.cpu().numpy(), r_or.lam)


@pytest.mark.parametrize("graph", [0, 1])
def test_solve_trajectory_many_rows(O, dev, graph):
    """J = 20,000 destinations: more rows than one workgroup steps by itself
    (the scalar-step and row-step kernels run) and than LDS holds (tail
    rows); 300 iterations with a gap check every 10 follow the oracle's g
    within 1e-6."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.random_small(41, I=40_000, J=20_000, dmax=8, box_frac=0.2, capacity="greedy")
    s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=300, check_every=10,
                      tol_rel_gap=-1.0, max_step=1e-2, init_step=1e-4, trace=True,
                      time_kernels=0 if graph else 1, graph_iters=20 if graph else 0)
    r_or = O.solve(inst, oracle_opts(O, s))
    with gpu_problem(inst, "f64") as p:
        assert p.info()["lds_rows"] < inst.m
        lam, r = p.solve(s)
    assert r.iters == 300 == r_or.iters
    tr_g, tr_o = r.trace[:, 0], r_or.trace[:, 0]
    rel = np.abs(tr_g - tr_o) / np.maximum(1.0, np.abs(tr_o))
    assert rel.max() <= 1e-6, (rel.max(), int(rel.argmax()))
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6
    assert lam_close(lam.cpu().numpy(), r_or.lam)


@pytest.mark.parametrize("stop", ["iteration_cap", "converged"])
def test_solve_many_rows_stops_inside_graph(O, dev, stop):
    """J = 20,000 destinations (the scalar-step and row-step kernels): a
    solve that ends inside a 40-iteration graph, at the iteration cap (290)
    or at a gap tolerance first met at a later check, leaves the rest of the
    graph without effect: iterations, g, gap and prices as the oracle's."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.random_small(41, I=40_000, J=20_000, dmax=8, box_frac=0.2, capacity="greedy")
    s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=290, check_every=10,
                      tol_rel_gap=-1.0, max_step=1e-2, init_step=1e-4, trace=True, graph_iters=40)
    if stop == "converged":
        # a tolerance halfway between a check's gap and the smallest before
        # it (a margin far above the 1e-6 the two sides' gaps agree to)
        tr = O.solve(inst, oracle_opts(O, s)).trace[:, 1]
        rel = tr[~np.isnan(tr)]
        s.max_iters = 1000
        for i in range(6, rel.size):
            if not rel[i] < 0.99 * rel[:i].min():
                continue
            s.tol_rel_gap = 0.5 * (rel[i] + rel[:i].min())
            r_or = O.solve(inst, oracle_opts(O, s))
            if r_or.converged and r_or.iters >= 60 and r_or.iters % 40 != 0:
                break
        else:
            pytest.fail("no gap tolerance met inside a graph")
    else:
        r_or = O.solve(inst, oracle_opts(O, s))
    with gpu_problem(inst, "f64") as p:
        lam, r = p.solve(s)
    assert r.iters == r_or.iters and r.converged == r_or.converged == (stop == "converged")
    assert r.iters % 40 != 0
    assert abs(r.g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g))
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6
    assert lam_close(lam.cpu().numpy(), r_or.lam)


def test_solve_continuation_to_gap(O, dev):
    """gamma continuation with stage changes on the gap and on the iteration
    budget, stopping at rel_gap 1e-4; FP64 storage follows the oracle."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.random_small(31, I=3000, J=60, dmax=20, box_frac=0.3)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=5, stage_iters=300,
                      stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=3000, check_every=10,
                      max_step=1e-1, init_step=1e-3, trace=True)
    r_or = O.solve(inst, oracle_opts(O, s))
    with gpu_problem(inst, "f64") as p:
        lam, r = p.solve(s)
    assert r.converged == r_or.converged
    assert r.iters == r_or.iters
    assert r.stage == r_or.stage
    assert abs(r.g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g))
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6
    np.testing.assert_allclose(r.trace[:, 3], r_or.trace[:, 3], rtol=1e-12)   # gamma schedule


def test_solve_fp32_converges_and_matches_evaluation(O, dev):
    """FP32 storage run to gap 1e-4: the oracle, evaluated at the GPU's final
    lam on the stored (rounded) data, reproduces its g within 1e-6 and
    certifies the gap."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.large(I=100_000, J=1_000, capacity="greedy")
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=5, stage_iters=2000,
                      stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=6000, check_every=10,
                      max_step=1e-1, init_step=1e-3)
    with gpu_problem(inst, "f32") as p:
        lam, r = p.solve(s)
    assert r.converged, r
    ev = O.dual_eval(inst.rounded("f32"), lam.cpu().numpy(), r.gamma)
    assert abs(ev.g - r.g) <= 1e-6 * max(1.0, abs(ev.g))
    assert ev.rel_gap <= 1.01e-4


def test_solve_capped_blocks_gap_certified(O, dev):
    """A continuation solve over simplex, box and capped-simplex blocks (FP32
    storage): at the GPU's final lam the oracle, on the stored data,
    reproduces g and the reported gap (the capped set is down-closed, so the
    restored point is feasible and the gap is a certificate)."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.heavy(I=40_000, J=2_000, dmax=512, capacity="greedy", capped_frac=0.4)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=5, stage_iters=2000,
                      stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=3000, check_every=10,
                      preset="natural")
    with gpu_problem(inst, "f32") as p:
        lam, r = p.solve(s)
    assert r.rel_gap < 1e-3, r
    ev = O.dual_eval(inst.rounded("f32"), lam.cpu().numpy(), r.gamma)
    assert abs(ev.g - r.g) <= 1e-6 * max(1.0, abs(ev.g))
    assert abs(ev.rel_gap - r.rel_gap) <= 1e-6


def test_solve_capped_trajectory_fp64(O, dev):
    """300 accelerated iterations over capped-simplex, box and simplex blocks
    with FP64 storage follow the oracle's g (every iteration), gap and lam."""
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.random_small(45, I=3_000, J=80, dmax=40, box_frac=0.2, capped_frac=0.5)
    s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=300, check_every=10,
                      tol_rel_gap=-1.0, max_step=1e-2, init_step=1e-4, trace=True)
    r_or = O.solve(inst, oracle_opts(O, s))
    with gpu_problem(inst, "f64") as p:
        lam, r = p.solve(s)
    assert r.iters == 300 == r_or.iters
    rel = np.abs(r.trace[:, 0] - r_or.trace[:, 0]) / np.maximum(1.0, np.abs(r_or.trace[:, 0]))
    assert rel.max() <= 1e-6, (rel.max(), int(rel.argmax()))
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6
    assert lam_close(lam.cpu().numpy(), r_or.lam)


def test_solve_warm_start_and_max_iters(O, dev):
    from paper_2603_04621_amd.api import SolveSettings
    inst = I.random_small(32, I=500, J=30, dmax=12)
    s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=37, check_every=10,
                      tol_rel_gap=0.0, max_step=1e-2, init_step=1e-4, trace=True)
    lam0 = lam_for(inst, 12, 0.3)
    r_or = O.solve(inst, oracle_opts(O, s), lam0=lam0)
    with gpu_problem(inst, "f64") as p:
        lam, r = p.solve(s, lam0=torch.from_numpy(lam0))
    assert r.status == 6 and not r.converged and r.iters == 37
    # lam carries the f32 rounding of the per-destination sums along the run
    assert lam_close(lam.cpu().numpy(), r_or.lam)
    assert abs(r.g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g))
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6


def test_solve_presets_follow_the_iteration_norm(O, dev):
    """|A'|^2 reported by the problem is 1 with row normalization (one family)
    and the largest squared row norm without it; a solve with the PAPER or
    NATURAL preset runs exactly the trajectory of a CUSTOM solve given the
    resolved steps (and the oracle's, FP64 storage)."""
    from paper_2603_04621_amd.api import SolveSettings, apply_preset
    inst = I.random_small(33, I=600, J=25, dmax=12, box_frac=0.2, capacity="greedy")
    r2max = float(np.bincount(inst.dst, weights=inst.a ** 2, minlength=inst.m).max())
    for rn, expect in ((True, 1.0), (False, r2max)):
        with gpu_problem(inst, "f64", row_normalize=rn) as p:
            assert p.info()["anorm2"] == pytest.approx(expect, rel=1e-12)
    for preset in ("paper", "natural"):
        s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=120, check_every=10,
                          tol_rel_gap=-1.0, preset=preset, trace=True)
        resolved = apply_preset(s, 1.0)
        custom = SolveSettings(**{**resolved.__dict__, "preset": "custom"})
        with gpu_problem(inst, "f64") as p:
            _, r1 = p.solve(s)
            _, r2 = p.solve(custom)
        # the f32 per-destination sums are added in timing order, so two runs
        # agree to rounding: the first step exactly, the rest within 1e-6
        assert r1.trace[0, 2] == r2.trace[0, 2] == resolved.init_step
        assert np.all(r1.trace[:, 2] <= resolved.max_step * (1 + 1e-15))
        np.testing.assert_allclose(r1.trace[:, 0], r2.trace[:, 0], rtol=1e-6)
        r_or = O.solve(inst, oracle_opts(O, custom))
        assert abs(r1.g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g))
