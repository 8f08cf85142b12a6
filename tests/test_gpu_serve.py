"""Serving: requests submitted while others run are admitted as slots free
up, run in shared fused ticks, and each result equals the request's solo
dl_solve result (to rounding: see test_gpu_batch)."""
import time

import numpy as np
import pytest

from paper_2603_04621_amd import instances as I

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_served_results_equal_solo():
    from paper_2603_04621_amd.api import Problem, Server, SolveSettings
    torch.cuda.set_device(0)
    rng = np.random.default_rng(3)
    sizes = np.rint(np.exp(rng.uniform(np.log(2e3), np.log(6e4), size=12))).astype(int)
    insts = [I.serve_member(int(s), k, capacity="greedy") for k, s in enumerate(sizes)]
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=3, stage_iters=300, stage_tol=1e-3,
                      tol_rel_gap=1e-4, max_iters=2000, check_every=10, max_step=1e-1,
                      init_step=1e-3)
    solo = []
    for x in insts:
        with Problem(x) as p:
            lam, r = p.solve(s)
            solo.append((lam.cpu().numpy(), r))
    srv = Server(hbm_budget_bytes=8e9, max_slots=4)      # fewer slots than requests
    tickets = []
    for k, x in enumerate(insts):
        tickets.append(srv.submit(x, s))
        time.sleep(0.002 * (k % 3))                      # arrivals while others run
    res = {}
    t_end = time.time() + 120
    while len(res) < len(tickets) and time.time() < t_end:
        for t in tickets:
            if t not in res:
                out = srv.poll(t)
                if out is not None:
                    res[t] = out
        time.sleep(0.001)
    srv.close()
    assert len(res) == len(tickets)
    starts = sorted(v[2][1] for v in res.values())
    dones = sorted(v[2][2] for v in res.values())
    assert starts[-1] > dones[0], "later requests should be admitted after earlier ones finish"
    from test_gpu_batch import same_solve
    for k, t in enumerate(tickets):
        r_srv, lam_srv, _ = res[t]
        lam_solo, r_solo = solo[k]
        same_solve(k, lam_solo, r_solo, lam_srv, r_srv, s)


def test_served_mixed_kernel_groups_equal_solo():
    """Requests that need different gradient kernels (FP32 and BF16 storage,
    per-edge primal scales, rows beyond LDS) share the server's ticks; each
    result equals the request's solo solve, and the memory of every retired
    request returns to the budget (the budget holds the largest request and
    one more, so the later ones are admitted only as earlier ones retire)."""
    from paper_2603_04621_amd.api import Problem, Server, SolveSettings
    torch.cuda.set_device(0)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=3, stage_iters=300, stage_tol=1e-3,
                      tol_rel_gap=1e-4, max_iters=1500, check_every=10, max_step=1e-1,
                      init_step=1e-3)
    reqs = [(I.serve_member(20_000, 0, capacity="greedy"), "f32", {}),
            (I.serve_member(30_000, 1, capacity="greedy"), "bf16", {}),
            (I.serve_member(25_000, 2, capacity="greedy"), "f32", {"primal_scale": 1}),
            (I.heavy(I=30_000, J=16_000, dmax=300, capacity="greedy"), "f32", {}),
            (I.serve_member(15_000, 3, capacity="greedy"), "bf16", {})]
    solo = []
    for x, st, po in reqs:
        with Problem(x, storage=st, **po) as p:
            lam, r = p.solve(s)
            solo.append((lam.cpu().numpy(), r))
    srv = Server(hbm_budget_bytes=35e6, max_slots=3)   # the largest request plus one more
    tickets = [srv.submit(x, s, storage=st, **po) for x, st, po in reqs]
    res = {}
    t_end = time.time() + 120
    while len(res) < len(tickets) and time.time() < t_end:
        for t in tickets:
            if t not in res:
                out = srv.poll(t)
                if out is not None:
                    res[t] = out
        time.sleep(0.001)
    srv.close()
    assert len(res) == len(tickets)
    from test_gpu_batch import same_solve
    for k, t in enumerate(tickets):
        r_srv, lam_srv, _ = res[t]
        lam_solo, r_solo = solo[k]
        same_solve(k, lam_solo, r_solo, lam_srv, r_srv, s)


def test_served_request_in_a_mix_matches_oracle():
    """An FP64 request served together with FP32 and BF16 requests (shared
    ticks, admissions while it runs) against the CPU oracle's solve of the
    same LP under the same settings: same stopping iteration, stage and
    gamma; g, rel_gap and lam within the parity tolerances."""
    from oracle import oracle as O
    from paper_2603_04621_amd.api import Server, SolveSettings
    from test_gpu_batch import assert_matches_oracle, oracle_settings
    torch.cuda.set_device(0)
    s = SolveSettings(gamma0=1e-1, gamma_final=1e-3, n_stages=3, stage_iters=300, stage_tol=1e-3,
                      tol_rel_gap=1e-4, max_iters=2000, check_every=10, max_step=1e-1,
                      init_step=1e-3)
    target = I.serve_member(6_000, 7, capacity="greedy")
    others = [(I.serve_member(20_000, 8, capacity="greedy"), "f32"),
              (I.serve_member(9_000, 9, capacity="greedy"), "bf16"),
              (I.serve_member(30_000, 10, capacity="greedy"), "f32")]
    srv = Server(hbm_budget_bytes=8e9, max_slots=3)
    tickets = [srv.submit(others[0][0], s, storage=others[0][1]),
               srv.submit(target, s, storage="f64")]
    time.sleep(0.002)
    tickets += [srv.submit(x, s, storage=st) for x, st in others[1:]]
    res = {}
    t_end = time.time() + 120
    while len(res) < len(tickets) and time.time() < t_end:
        for t in tickets:
            if t not in res:
                out = srv.poll(t)
                if out is not None:
                    res[t] = out
        time.sleep(0.001)
    srv.close()
    assert len(res) == len(tickets)
    r_srv, lam_srv, _ = res[tickets[1]]
    r_or = O.solve(target, oracle_settings(O, s))
    assert r_or.converged
    assert_matches_oracle(r_srv, lam_srv, r_or)


def test_server_rejects_oversized_request():
    from paper_2603_04621_amd import _lib as L
    from paper_2603_04621_amd.api import Server, SolveSettings
    torch.cuda.set_device(0)
    srv = Server(hbm_budget_bytes=1 << 20, max_slots=2)
    with pytest.raises(L.DualipError) as e:
        srv.submit(I.large(I=200_000, J=1000), SolveSettings())
    assert e.value.status == L.DL_ERR_UNSUPPORTED
    srv.close()
