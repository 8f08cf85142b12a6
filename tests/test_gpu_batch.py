"""Batched solves: every LP of a batch reproduces its solo dl_solve run.

Each problem keeps its own chunking, reduction order and FP64 state inside the
fused batched launches; the only difference between two runs is the order in
which the waves of a workgroup add into the f32 LDS partial sums (atomics), so
results agree to rounding, not bit for bit."""
import numpy as np
import pytest

from paper_2603_04621_amd import instances as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    return torch.device("cuda", 0)


def same_solve(k, lam1, r1, lam2, r2, s):
    """Two runs of one solve agree to rounding: the same stopping iteration
    (or one check period apart when a gap test sits at the tolerance), the
    same status, and g and lam equal to rounding.

    When the two runs stop one check apart, both certified rel_gap <= tol at
    the same final gamma.  Weak duality puts each g in [P* - tol max(1,|g|),
    P*] (P* the optimum of the regularized primal), so the two g differ by
    at most tol max(1, |g|).  lam is not compared then: the dual maximiser
    need not be unique (active bounds), and a check period of further
    ascent moves lam by more than rounding."""
    assert r2.converged == r1.converged, (k, r1, r2)
    if r2.iters == r1.iters:
        assert abs(r2.g - r1.g) <= 1e-9 * max(1.0, abs(r1.g)), (k, r1.g, r2.g)
        assert np.max(np.abs(lam2 - lam1), initial=0.0) <= 1e-5 * max(1.0, np.abs(lam1).max(initial=0.0))
    else:
        assert abs(r2.iters - r1.iters) <= s.check_every, (k, r1.iters, r2.iters)
        assert r1.converged, (k, r1, r2)    # unconverged runs both stop at max_iters
        assert r1.rel_gap <= s.tol_rel_gap and r2.rel_gap <= s.tol_rel_gap
        assert r1.gamma == r2.gamma and r1.stage == r2.stage, (k, r1, r2)
        assert abs(r2.g - r1.g) <= 1.01 * s.tol_rel_gap * max(1.0, abs(r1.g)), (k, r1.g, r2.g)


def make_batch(count=10, seed=4621100):
    sizes = I.batch_sizes(count, lo=1e3, hi=2e5, seed=seed)
    insts = [I.batch_member(int(s), k, seed=seed, capacity="greedy") for k, s in enumerate(sizes)]
    # one mixed-projection member with a heavier tail
    insts.append(I.heavy(I=3000, J=400, dmax=700, capacity="greedy"))
    return insts


@pytest.mark.parametrize("storage", ["f32", "f64"])
def test_batch_equals_solo(dev, storage):
    from paper_2603_04621_amd.api import Problem, SolveSettings, batch_solve
    insts = make_batch()
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=3, stage_iters=400, stage_tol=1e-3,
                      tol_rel_gap=1e-4, max_iters=1500, check_every=10, max_step=1e-1,
                      init_step=1e-3)
    probs = [Problem(x, storage=storage) for x in insts]
    solo = [p.solve(s) for p in probs]
    lams, outs = batch_solve(probs, s)
    for k, ((l1, r1), l2, r2) in enumerate(zip(solo, lams, outs)):
        same_solve(k, l1.cpu().numpy(), r1, l2.cpu().numpy(), r2, s)
    assert sum(r.converged for r in outs) >= len(outs) - 1
    for p in probs:
        p.close()


def test_batch_mixed_kernel_groups(dev):
    """One batch whose members need different gradient kernels (FP32, BF16,
    per-edge primal scales, rows beyond LDS, box blocks): each member's
    batched solve equals its solo solve."""
    from paper_2603_04621_amd.api import Problem, SolveSettings, batch_solve
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=3, stage_iters=300, stage_tol=1e-3,
                      tol_rel_gap=1e-4, max_iters=1200, check_every=10, max_step=1e-1,
                      init_step=1e-3)
    small = make_batch(count=3, seed=4621300)
    rows_beyond_lds = I.heavy(I=30_000, J=16_000, dmax=300, capacity="greedy")
    members = [(small[0], "f32", 0), (small[1], "bf16", 0), (small[2], "f32", 1),
               (small[3], "bf16", 0), (rows_beyond_lds, "f32", 0)]
    probs = [Problem(x, storage=st, primal_scale=ps) for x, st, ps in members]
    assert probs[-1].info()["lds_rows"] < rows_beyond_lds.m
    solo = [p.solve(s) for p in probs]
    lams, outs = batch_solve(probs, s)
    for k, ((l1, r1), l2, r2) in enumerate(zip(solo, lams, outs)):
        same_solve(k, l1.cpu().numpy(), r1, l2.cpu().numpy(), r2, s)
    for p in probs:
        p.close()


def test_batch_matches_oracle_member(dev):
    """One batched member against the CPU oracle directly (FP64 storage)."""
    from oracle import oracle as O
    from paper_2603_04621_amd.api import Problem, SolveSettings, batch_solve
    insts = make_batch(count=4, seed=4621200)
    s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, tol_rel_gap=0.0, max_iters=200,
                      check_every=10, max_step=1e-2, init_step=1e-4)
    probs = [Problem(x, storage="f64") for x in insts]
    lams, outs = batch_solve(probs, s)
    k = 2
    r_or = O.solve(insts[k], O.SolveOpts(gamma0=1e-2, gamma_final=1e-2, tol_rel_gap=0.0,
                                         max_iters=200, check_every=10, max_step=1e-2,
                                         init_step=1e-4))
    assert abs(outs[k].g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g))
    la = lams[k].cpu().numpy()
    assert np.max(np.abs(la - r_or.lam)) <= 1e-5 * max(1.0, np.max(np.abs(r_or.lam)))
    for p in probs:
        p.close()


def oracle_settings(O, s):
    return O.SolveOpts(gamma0=s.gamma0, gamma_final=s.gamma_final, n_stages=s.n_stages,
                       row_normalize=1, stage_iters=s.stage_iters, stage_tol=s.stage_tol,
                       tol_rel_gap=s.tol_rel_gap, max_iters=s.max_iters,
                       check_every=s.check_every, max_step=s.max_step, init_step=s.init_step,
                       momentum=s.momentum, adaptive=s.adaptive)


def assert_matches_oracle(r, lam, r_or, gamma_trace=None):
    """A GPU solve (FP64 storage) against the oracle's solve under the same
    settings: same stopping iteration, stage and gamma, g and rel_gap within
    1e-6, lam within 1e-5 of the largest price."""
    assert r.converged == r_or.converged, (r, r_or)
    assert r.iters == r_or.iters, (r.iters, r_or.iters)
    assert r.stage == r_or.stage and r.gamma == pytest.approx(r_or.gamma, rel=1e-12)
    assert abs(r.g - r_or.g) <= 1e-6 * max(1.0, abs(r_or.g)), (r.g, r_or.g)
    assert abs(r.rel_gap - r_or.rel_gap) <= 1e-6, (r.rel_gap, r_or.rel_gap)
    assert np.max(np.abs(lam - r_or.lam), initial=0.0) <= 1e-5 * max(1.0, np.max(np.abs(r_or.lam)))


def test_batch_member_under_continuation_matches_oracle(dev):
    """Members of one batch, each solved with gamma continuation (stage
    changes on the gap and on the stage budget) to rel_gap 1e-4, against the
    CPU oracle's solve of the same LP under the same settings (FP64
    storage)."""
    from oracle import oracle as O
    from paper_2603_04621_amd.api import Problem, SolveSettings, batch_solve
    insts = make_batch(count=5, seed=4621400)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=3, stage_iters=300,
                      stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=1500, check_every=10,
                      max_step=1e-1, init_step=1e-3)
    probs = [Problem(x, storage="f64") for x in insts]
    lams, outs = batch_solve(probs, s)
    for k in (0, 3, len(insts) - 1):
        r_or = O.solve(insts[k], oracle_settings(O, s))
        assert_matches_oracle(outs[k], lams[k].cpu().numpy(), r_or)
    for p in probs:
        p.close()


def test_early_stop_does_not_run_out_the_iteration_cap(dev):
    """A solve that reaches its gap long before max_iters returns promptly:
    once the device has stopped, no further iterations are enqueued (solo
    and batched).  Regression test: the remainder used to be launched
    eagerly, one no-op iteration at a time."""
    import time
    import torch
    from paper_2603_04621_amd.api import Problem, SolveSettings, batch_solve
    inst = I.large(I=20_000, J=100, capacity="greedy")

    def settings(cap):
        return SolveSettings(gamma0=1e-2, gamma_final=1e-2, tol_rel_gap=1e-4, max_iters=cap,
                             check_every=10, max_step=1e-2, init_step=1e-4)

    with Problem(inst) as p:
        times = {}
        for cap in (5_000, 300_000):
            p.solve(settings(cap))
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, r = p.solve(settings(cap))
            times[cap] = time.perf_counter() - t0
            assert r.converged and r.iters < 5_000
        assert times[300_000] < times[5_000] + 0.25, times
        btimes = {}
        for cap in (5_000, 300_000):
            batch_solve([p], settings(cap))
            t0 = time.perf_counter()
            _, rs = batch_solve([p], settings(cap))
            btimes[cap] = time.perf_counter() - t0
            assert rs[0].converged
        assert btimes[300_000] < btimes[5_000] + 0.25, btimes
