"""Pins of the FP64 oracle against facts that do not come from its own code.

Each test checks the oracle (oracle/oracle.c) against brute force, an
independent library solver, dense linear algebra, finite differences, a
closed form or an invariant stated in the paper, or the hyper-parameters
the paper prints.  A plausible slip in the oracle (a dropped term, a sign,
a transposed product, a wrong threshold index) fails at least one of them.
"""
import itertools
import json
import os

import numpy as np
import pytest
import scipy.optimize as so

from paper_2603_04621_amd import instances as I

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# projection (Eq.(4),(5) simplex; box)
# ---------------------------------------------------------------------------

def brute_simplex(t, w):
    """min sum (1/(2w)) x^2 - t x over {x >= 0, sum x <= 1}, by enumerating
    every face: for each support S, the face minimiser with the sum
    constraint free (x_S = w t) and with it tight (Lagrange on sum_S x = 1);
    keep the feasible candidates, return the one of least objective."""
    d = len(t)
    f = lambda x: np.sum(x * x / (2 * w) - t * x)
    best, bx = np.inf, None
    for r in range(0, d + 1):
        for S in itertools.combinations(range(d), r):
            S = list(S)
            for tight in (False, True):
                x = np.zeros(d)
                if tight:
                    if not S:
                        continue
                    tau = (np.sum(w[S] * t[S]) - 1.0) / np.sum(w[S])
                    x[S] = w[S] * (t[S] - tau)
                else:
                    x[S] = w[S] * t[S]
                if np.all(x >= -1e-13) and x.sum() <= 1 + 1e-12:
                    v = f(x)
                    if v < best:
                        best, bx = v, x
    return bx


def brute_box(t, w, u):
    """Per coordinate, the least of the objective at 0, u and the interior stationary point."""
    x = np.empty_like(t)
    for e in range(len(t)):
        cands = [0.0, u[e]]
        z = w[e] * t[e]
        if 0.0 < z < u[e]:
            cands.append(z)
        vals = [c * c / (2 * w[e]) - t[e] * c for c in cands]
        x[e] = cands[int(np.argmin(vals))]
    return x


@pytest.mark.parametrize("seed", range(40))
def test_simplex_projection_matches_face_enumeration(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(seed)
    d = int(rng.integers(1, 9))
    scale = 10.0 ** rng.uniform(-3, 1)
    t = rng.normal(size=d) * scale + rng.uniform(-0.5, 1.0) * scale
    w = rng.uniform(0.5, 2.0, size=d) / scale if seed % 2 else np.full(d, 1.0 / scale)
    x, tau = O.project_block(O.SIMPLEX, t, w)
    xb = brute_simplex(t, w)
    np.testing.assert_allclose(x, xb, rtol=1e-9, atol=1e-12)
    assert tau >= 0.0


@pytest.mark.parametrize("seed", range(10))
def test_box_projection_matches_candidates(oracle_lib, seed):
    O = oracle_lib
    rng = np.random.default_rng(100 + seed)
    d = 12
    t = rng.normal(size=d)
    w = rng.uniform(0.1, 10.0, size=d)
    u = rng.uniform(0.2, 1.0, size=d)
    x, _ = O.project_block(O.BOX, t, w, u)
    np.testing.assert_allclose(x, brute_box(t, w, u), rtol=1e-14, atol=0)


def test_projection_special_cases(oracle_lib):
    O = oracle_lib
    # d = 1 simplex is the box [0, 1]
    for t in (-2.0, 0.3, 5.0):
        xs, _ = O.project_block(O.SIMPLEX, [t], [1.0])
        xb, _ = O.project_block(O.BOX, [t], [1.0], [1.0])
        assert xs[0] == xb[0]
    # all t <= 0: x = 0
    x, tau = O.project_block(O.SIMPLEX, [-1.0, -0.5, 0.0], [3.0, 3.0, 3.0])
    assert np.all(x == 0) and tau == 0
    # sum of positive parts <= 1: plain ReLU, tau = 0
    x, tau = O.project_block(O.SIMPLEX, [0.1, -0.3, 0.2], [2.0, 2.0, 2.0])
    np.testing.assert_allclose(x, [0.2, 0.0, 0.4])
    assert tau == 0
    # equal t large: uniform 1/d
    x, _ = O.project_block(O.SIMPLEX, [7.0] * 5, [1.0] * 5)
    np.testing.assert_allclose(x, [0.2] * 5, rtol=1e-15)
    # large gamma-scaled gaps: only the top element survives, at 1
    x, _ = O.project_block(O.SIMPLEX, [3.0, 1.0, 0.5], [1e3, 1e3, 1e3])
    np.testing.assert_allclose(x, [1.0, 0.0, 0.0])


def brute_capped(t, w, u):
    """min sum (1/(2w)) x^2 - t x over {0 <= x <= u, sum x <= 1}, by
    enumerating every face: each coordinate at 0, at u or free, with the sum
    constraint free (free x = w t) or tight (free x = w (t - tau), tau from
    sum x = 1); keep the feasible candidates, return the least objective."""
    d = len(t)
    f = lambda x: np.sum(x * x / (2 * w) - t * x)
    best, bx = np.inf, None
    for lab in itertools.product((0, 1, 2), repeat=d):     # 0: at 0, 1: at u, 2: free
        lab = np.array(lab)
        F, U = lab == 2, lab == 1
        for tight in (False, True):
            x = np.where(U, u, 0.0)
            if tight:
                if not F.any():
                    if abs(x.sum() - 1.0) > 1e-12:
                        continue
                else:
                    tau = (np.sum(w[F] * t[F]) + np.sum(u[U]) - 1.0) / np.sum(w[F])
                    x[F] = w[F] * (t[F] - tau)
            else:
                x[F] = w[F] * t[F]
            if np.all(x >= -1e-13) and np.all(x <= u + 1e-13) and x.sum() <= 1 + 1e-12:
                v = f(x)
                if v < best:
                    best, bx = v, x
    return bx


@pytest.mark.parametrize("seed", range(40))
def test_capped_projection_matches_face_enumeration(oracle_lib, seed):
    """The capped simplex (the box-cut reading): breakpoint search against
    enumeration of all 3^d bound patterns, sum tight or slack.  Draws cover
    bounds below and above 1, the sum binding or not, ties among t."""
    O = oracle_lib
    rng = np.random.default_rng(500 + seed)
    d = int(rng.integers(1, 7))
    scale = 10.0 ** rng.uniform(-3, 1)
    t = rng.normal(size=d) * scale + rng.uniform(-0.5, 1.0) * scale
    if seed % 5 == 0 and d > 1:
        t[1] = t[0]
    w = rng.uniform(0.5, 2.0, size=d) / scale if seed % 2 else np.full(d, 1.0 / scale)
    u = rng.uniform(0.05, 1.2, size=d)
    if seed % 7 == 3:
        u[0] = 0.0
    x, tau = O.project_block(O.CAPPED, t, w, u)
    xb = brute_capped(t, w, u)
    np.testing.assert_allclose(x, xb, rtol=1e-9, atol=1e-12)
    assert tau >= 0.0


def test_capped_projection_reductions(oracle_lib):
    """Bounds u >= 1 never bind under sum x <= 1: the simplex projection;
    a box solution summing to at most 1: the box projection; one edge:
    the clamp to [0, min(u, 1)]."""
    O = oracle_lib
    rng = np.random.default_rng(77)
    for _ in range(20):
        d = int(rng.integers(1, 30))
        t = rng.normal(size=d) * 3
        w = rng.uniform(0.5, 2.0, size=d)
        xc, tc = O.project_block(O.CAPPED, t, w, 1.0 + rng.uniform(0, 2, size=d))
        xs, ts = O.project_block(O.SIMPLEX, t, w)
        np.testing.assert_allclose(xc, xs, rtol=1e-12, atol=1e-14)
        u = rng.uniform(0.0, 1.0 / d, size=d)
        xc, tc = O.project_block(O.CAPPED, t, w, u)
        xb, _ = O.project_block(O.BOX, t, w, u)
        assert tc == 0.0 and np.array_equal(xc, xb)
    for t0, u0 in ((-1.0, 0.5), (0.3, 0.5), (3.0, 0.5), (3.0, 2.0), (0.7, 2.0)):
        x, _ = O.project_block(O.CAPPED, [t0], [1.0], [u0])
        assert x[0] == pytest.approx(min(max(t0, 0.0), u0, 1.0), rel=1e-15)


def capped_kkt_residual(t, w, u, x):
    """KKT of the capped simplex: x = clamp(w (t - tau), 0, u) for one
    tau >= 0 with tau (1 - sum x) = 0 and sum x <= 1."""
    r = max(0.0, float(x.sum()) - 1.0, float(np.max(x - u, initial=0.0)), float(-x.min()))
    free = (x > 1e-12) & (x < u - 1e-12)
    if free.any():
        taus = t[free] - x[free] / w[free]
        tau = float(np.mean(taus))
        r = max(r, float(np.max(np.abs(taus - tau))) / max(1.0, abs(tau)))
    else:
        # no interior edge: tau is only bracketed (at least t_e of the edges
        # at 0, and 0 unless the sum is tight); the smallest admissible value
        # must reproduce x
        tau = max(0.0, float(np.max(t[x <= 1e-12], initial=0.0))) if x.sum() >= 1 - 1e-12 else 0.0
    z = np.clip(w * (t - tau), 0.0, u)
    r = max(r, float(np.max(np.abs(z - x))))
    r = max(r, -tau / max(1.0, abs(tau)), abs(tau * (1.0 - x.sum())) / max(1.0, abs(tau)))
    return r


def kkt_residual(proj, t, w, u, x):
    """Largest violation of the block's KKT conditions."""
    r = 0.0
    if proj == 1:
        z = np.clip(w * t, 0.0, u)
        return float(np.max(np.abs(z - x)))
    r = max(r, -x.min(), x.sum() - 1.0)
    act = x > 0
    if act.any():
        taus = t[act] - x[act] / w[act]
        tau = float(np.mean(taus))
        r = max(r, float(np.max(np.abs(taus - tau))) / max(1.0, abs(tau)))
        r = max(r, -tau / max(1.0, abs(tau)))
        r = max(r, float(np.max(t[~act] - tau, initial=-np.inf)) / max(1.0, abs(tau)))
        r = max(r, abs(tau * (1.0 - x.sum())))
    else:
        r = max(r, float(np.max(t)))
    return r


@pytest.mark.parametrize("seed", range(3))
def test_kkt_on_every_block(oracle_lib, seed):
    O = oracle_lib
    inst = I.random_small(seed, I=300, J=40, dmax=40, box_frac=0.4)
    rng = np.random.default_rng(seed)
    gamma = 10.0 ** rng.uniform(-3, -1)
    lam = rng.uniform(0, 2, size=inst.m)
    ev = O.dual_eval(inst, lam, gamma)
    t = -(inst.c + inst.a * lam[inst.dst])
    w = np.full(inst.n, 1.0 / gamma)
    u = inst.upper if inst.upper is not None else np.ones(inst.n)
    worst = 0.0
    for i in range(inst.num_blocks):
        lo, hi = inst.block_off[i], inst.block_off[i + 1]
        worst = max(worst, kkt_residual(int(inst.block_proj[i]), t[lo:hi], w[lo:hi],
                                        u[lo:hi], ev.x[lo:hi]))
    assert worst < 1e-9


@pytest.mark.parametrize("seed", range(3))
def test_kkt_on_every_capped_block(oracle_lib, seed):
    O = oracle_lib
    inst = I.random_small(seed, I=300, J=40, dmax=40, box_frac=0.2, capped_frac=0.5)
    assert np.any(inst.block_proj == I.PROJ_CAPPED)
    rng = np.random.default_rng(seed)
    gamma = 10.0 ** rng.uniform(-3, -1)
    lam = rng.uniform(0, 2, size=inst.m)
    ev = O.dual_eval(inst, lam, gamma)
    t = -(inst.c + inst.a * lam[inst.dst])
    w = np.full(inst.n, 1.0 / gamma)
    worst = 0.0
    for i in np.nonzero(inst.block_proj == I.PROJ_CAPPED)[0]:
        lo, hi = inst.block_off[i], inst.block_off[i + 1]
        worst = max(worst, capped_kkt_residual(t[lo:hi], w[lo:hi], inst.upper[lo:hi],
                                               ev.x[lo:hi]))
    assert worst < 1e-9


# ---------------------------------------------------------------------------
# dual gradient: A'lam, projection, A x (Danskin), dual objective Eq.(2)
# ---------------------------------------------------------------------------

def test_products_match_dense_algebra(oracle_lib):
    O = oracle_lib
    inst = I.random_small(3, I=25, J=6, dmax=6, box_frac=0.3, capped_frac=0.4)
    assert np.any(inst.block_proj == I.PROJ_CAPPED)
    A = inst.dense()
    rng = np.random.default_rng(0)
    lam = rng.uniform(0, 1, size=inst.m)
    gamma = 0.05
    ev = O.dual_eval(inst, lam, gamma)
    t = -(A.T @ lam + inst.c)
    # projection blockwise by brute force
    x = np.empty(inst.n)
    u = inst.upper if inst.upper is not None else np.ones(inst.n)
    for i in range(inst.num_blocks):
        lo, hi = inst.block_off[i], inst.block_off[i + 1]
        w = np.full(hi - lo, 1.0 / gamma)
        if inst.block_proj[i] == I.PROJ_SIMPLEX:
            x[lo:hi] = brute_simplex(t[lo:hi], w)
        elif inst.block_proj[i] == I.PROJ_CAPPED:
            x[lo:hi] = brute_capped(t[lo:hi], w, u[lo:hi])
        else:
            x[lo:hi] = brute_box(t[lo:hi], w, u[lo:hi])
    np.testing.assert_allclose(ev.x, x, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ev.grad, A @ x - inst.b, rtol=1e-12, atol=1e-12)
    g = inst.c @ x + 0.5 * gamma * x @ x + lam @ (A @ x - inst.b)
    assert ev.g == pytest.approx(g, rel=1e-12)


def test_general_csc_two_families(oracle_lib):
    """Columns with two entries (two matching families, Definition 1): the
    oracle's CSC loops must agree with dense A'lam and A x."""
    O = oracle_lib
    rng = np.random.default_rng(7)
    J, Ib, d = 5, 12, 4
    n = Ib * d
    m = 2 * J
    A = np.zeros((m, n))
    for e in range(n):
        j = rng.integers(0, J)
        A[j, e] = rng.uniform(0.5, 1.5)          # family 1, row j
        A[J + j, e] = rng.uniform(0.1, 1.0)      # family 2, same destination
    colptr = np.zeros(n + 1, dtype=np.int64)
    rows, vals = [], []
    for e in range(n):
        nz = np.nonzero(A[:, e])[0]
        rows += list(nz)
        vals += list(A[nz, e])
        colptr[e + 1] = colptr[e] + len(nz)
    c = -rng.uniform(0, 1, size=n)
    b = 0.3 * A.sum(axis=1)
    off = np.arange(0, n + 1, d, dtype=np.int64)
    lp = O.LP(m, n, np.array(rows), np.array(vals), c, b, off,
              np.zeros(Ib, dtype=np.uint8), colptr=colptr)
    lam = rng.uniform(0, 0.5, size=m)
    gamma = 0.1
    ev = O.dual_eval(lp, lam, gamma)
    t = -(A.T @ lam + c)
    x = np.concatenate([brute_simplex(t[k:k + d], np.full(d, 1 / gamma)) for k in range(0, n, d)])
    np.testing.assert_allclose(ev.x, x, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ev.grad, A @ x - b, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("seed", range(3))
def test_gradient_is_finite_difference_of_g(oracle_lib, seed):
    O = oracle_lib
    inst = I.random_small(10 + seed, I=150, J=12, dmax=10, box_frac=0.3)
    rng = np.random.default_rng(seed)
    gamma = 0.02
    lam = rng.uniform(0.2, 1.5, size=inst.m)
    ev = O.dual_eval(inst, lam, gamma)
    for h in (1e-5, 1e-6):
        fd = np.empty(inst.m)
        for j in range(inst.m):
            e = np.zeros(inst.m)
            e[j] = h
            fd[j] = (O.dual_eval(inst, lam + e, gamma).g - O.dual_eval(inst, lam - e, gamma).g) / (2 * h)
        scale = np.abs(inst.b) + 1.0
        assert np.max(np.abs(fd - ev.grad) / scale) < 1e-4


def test_inactive_regime_closed_form(oracle_lib):
    """With every projection inactive (box with huge bound, t > 0), the
    gradient is -(A A' lam + A c)/gamma - b and g is the quadratic it
    integrates (Section 5, Jacobi preconditioning paragraph)."""
    O = oracle_lib
    inst = I.random_small(21, I=40, J=7, dmax=5, box_frac=1.0)
    inst.upper = np.full(inst.n, 1e12)
    inst.c = inst.c - 10.0                      # t = -(c + a lam) > 0 for small lam
    A = inst.dense()
    gamma = 0.3
    lam = np.random.default_rng(1).uniform(0, 0.5, size=inst.m)
    ev = O.dual_eval(inst, lam, gamma)
    closed = -(A @ A.T @ lam + A @ inst.c) / gamma - inst.b
    np.testing.assert_allclose(ev.grad, closed, rtol=1e-11, atol=1e-9)
    # Hessian -A A'/gamma: a second evaluation moves the gradient by exactly that
    dl = np.random.default_rng(2).uniform(0, 0.1, size=inst.m)
    ev2 = O.dual_eval(inst, lam + dl, gamma)
    np.testing.assert_allclose(ev2.grad - ev.grad, -(A @ A.T @ dl) / gamma, rtol=1e-8, atol=1e-8)


@pytest.mark.parametrize("seed", range(3))
def test_concavity_and_first_order_bound(oracle_lib, seed):
    O = oracle_lib
    inst = I.random_small(30 + seed, I=120, J=15, dmax=12, box_frac=0.3)
    rng = np.random.default_rng(seed)
    gamma = 0.01
    for _ in range(5):
        l1 = rng.uniform(0, 2, size=inst.m)
        l2 = rng.uniform(0, 2, size=inst.m)
        e1 = O.dual_eval(inst, l1, gamma)
        e2 = O.dual_eval(inst, l2, gamma)
        th = rng.uniform()
        em = O.dual_eval(inst, th * l1 + (1 - th) * l2, gamma)
        tol = 1e-12 * (abs(e1.g) + abs(e2.g))
        assert em.g >= th * e1.g + (1 - th) * e2.g - tol
        assert e2.g <= e1.g + e1.grad @ (l2 - l1) + tol


# ---------------------------------------------------------------------------
# Jacobi row normalization (Section 5) and primal scaling
# ---------------------------------------------------------------------------

def test_row_normalization_invariants(oracle_lib):
    O = oracle_lib
    inst = I.random_small(41, I=200, J=30, dmax=8, box_frac=0.3, zipf=True)
    inst.a = inst.a * np.random.default_rng(0).lognormal(0, 2, size=inst.m)[inst.dst]
    D = O.row_scale(inst)
    ssq = np.bincount(inst.dst, weights=(D[inst.dst] * inst.a) ** 2, minlength=inst.m)
    nonempty = np.bincount(inst.dst, minlength=inst.m) > 0
    np.testing.assert_allclose(ssq[nonempty], 1.0, rtol=1e-13)
    assert np.all(D[~nonempty] == 1.0)
    # A' A'^T = I for one family (Lemma 1 with m = 1)
    A2 = D[:, None] * inst.dense()
    G = A2 @ A2.T
    np.testing.assert_allclose(G[np.ix_(nonempty, nonempty)], np.eye(nonempty.sum()), atol=1e-13)
    # g'(lam') = g(D lam'), grad' = D grad
    scaled = I.Instance(inst.m, inst.n, inst.dst, D[inst.dst] * inst.a, inst.c, D * inst.b,
                        inst.block_off, inst.block_proj, inst.upper)
    lamp = np.random.default_rng(1).uniform(0, 3, size=inst.m)
    e1 = O.dual_eval(scaled, lamp, 0.01)
    e0 = O.dual_eval(inst, D * lamp, 0.01)
    assert e1.g == pytest.approx(e0.g, rel=1e-12)
    np.testing.assert_allclose(e1.grad, D * e0.grad, rtol=1e-10, atol=1e-12)


def test_colnorm_primal_scale(oracle_lib):
    O = oracle_lib
    inst = I.random_small(42, I=30, J=6, dmax=5)
    v = O.colnorm_scale(inst)
    np.testing.assert_allclose(v, np.abs(inst.a), rtol=1e-15)
    # primal scaling view (i): regularizer gamma/2 sum v^2 x^2 equals, after
    # z = v x, the plain ridge on z with c/v and A/v (view (ii)) for box blocks
    inst.block_proj[:] = I.PROJ_BOX
    inst.upper = np.full(inst.n, 1e9)
    lam = np.random.default_rng(3).uniform(0, 1, size=inst.m)
    e_i = O.dual_eval(inst, lam, 0.1, v=v)
    view2 = I.Instance(inst.m, inst.n, inst.dst, inst.a / v, inst.c / v, inst.b,
                       inst.block_off, inst.block_proj, inst.upper * v)
    e_ii = O.dual_eval(view2, lam, 0.1)
    assert e_i.g == pytest.approx(e_ii.g, rel=1e-12)
    np.testing.assert_allclose(e_i.x * v, e_ii.x, rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------
# duality gap, optimum against independent solvers
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(4))
def test_weak_duality(oracle_lib, seed):
    O = oracle_lib
    inst = I.random_small(50 + seed, I=200, J=20, dmax=10, box_frac=0.3)
    rng = np.random.default_rng(seed)
    for _ in range(5):
        lam = rng.exponential(2.0, size=inst.m) * (rng.random(inst.m) < 0.7)
        ev = O.dual_eval(inst, lam, 10.0 ** rng.uniform(-3, -1))
        assert ev.rel_gap >= -1e-12
        assert ev.P >= ev.g - 1e-9 * max(1, abs(ev.g))


def qp_optimum(inst, gamma):
    """P*_gamma = min c'x + gamma/2 |x|^2 over Ax <= b, x in C, by SLSQP."""
    A = inst.dense()
    n = inst.n
    u = inst.upper if inst.upper is not None else np.ones(n)
    bounds = [(0.0, u[e] if inst.block_proj[np.searchsorted(inst.block_off, e, 'right') - 1] != 0
               else None) for e in range(n)]
    cons = [{"type": "ineq", "fun": lambda x: inst.b - A @ x, "jac": lambda x: -A}]
    for i in range(inst.num_blocks):
        if inst.block_proj[i] != I.PROJ_BOX:
            lo, hi = int(inst.block_off[i]), int(inst.block_off[i + 1])
            row = np.zeros(n)
            row[lo:hi] = 1.0
            cons.append({"type": "ineq", "fun": lambda x, r=row: 1.0 - r @ x,
                         "jac": lambda x, r=row: -r})
    f = lambda x: inst.c @ x + 0.5 * gamma * x @ x
    jac = lambda x: inst.c + gamma * x
    r = so.minimize(f, np.zeros(n), jac=jac, bounds=bounds, constraints=cons, method="SLSQP",
                    options={"ftol": 1e-14, "maxiter": 2000})
    # status 8 (no descent direction left at this ftol) is SLSQP's own "cannot
    # improve": accept it once the point is checked feasible
    assert r.success or r.status == 8, r.message
    x = r.x
    viol = max(float(np.max(A @ x - inst.b)), float(-x.min()))
    for con in cons[1:]:
        viol = max(viol, -float(con["fun"](x)))
    assert viol < 1e-9
    return r.fun, x


def lp_optimum(inst):
    A = inst.dense()
    n = inst.n
    rows = [A]
    rhs = [inst.b]
    for i in range(inst.num_blocks):
        if inst.block_proj[i] != I.PROJ_BOX:
            row = np.zeros((1, n))
            row[0, inst.block_off[i]:inst.block_off[i + 1]] = 1.0
            rows.append(row)
            rhs.append([1.0])
    u = inst.upper if inst.upper is not None else np.ones(n)
    bounds = []
    for e in range(n):
        i = np.searchsorted(inst.block_off, e, "right") - 1
        bounds.append((0.0, u[e] if inst.block_proj[i] != 0 else None))
    r = so.linprog(inst.c, A_ub=np.vstack(rows), b_ub=np.concatenate(rhs), bounds=bounds,
                   method="highs")
    assert r.status == 0
    return r.fun, r.x


def tiny_binding(seed):
    return I.random_small(seed, I=12, J=4, dmax=5, box_frac=0.34, capacity="greedy")


@pytest.mark.parametrize("seed", [60, 61, 62])
def test_converged_dual_equals_qp_optimum(oracle_lib, seed):
    O = oracle_lib
    inst = tiny_binding(seed)
    gamma = 0.05
    Pstar, _ = qp_optimum(inst, gamma)
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=20000,
                                  check_every=10, tol_rel_gap=1e-11, max_step=gamma,
                                  init_step=1e-2 * gamma))
    assert r.converged
    scale = max(1.0, abs(Pstar))
    assert abs(r.g - Pstar) / scale < 1e-7
    assert r.g <= Pstar + 1e-8 * scale          # weak duality against the QP optimum
    assert r.P >= Pstar - 1e-8 * scale          # restored point is feasible


@pytest.mark.parametrize("seed", [70, 71])
def test_small_gamma_approaches_lp_optimum(oracle_lib, seed):
    """0 <= P*_gamma - P*_0 <= gamma/2 |x_LP|^2 (the ridge perturbs the LP by at most that)."""
    O = oracle_lib
    inst = tiny_binding(seed)
    P0, xlp = lp_optimum(inst)
    for gamma in (1e-2, 1e-3):
        r = O.solve(inst, O.SolveOpts(gamma0=0.1, gamma_final=gamma, n_stages=4,
                                      stage_iters=3000, stage_tol=1e-6, max_iters=60000,
                                      check_every=10, tol_rel_gap=1e-10, max_step=0.1,
                                      init_step=1e-3))
        assert r.converged
        slack = 1e-8 * max(1.0, abs(P0))
        assert r.g >= P0 - slack - 0.0
        assert r.g <= P0 + 0.5 * gamma * xlp @ xlp + slack


# ---------------------------------------------------------------------------
# ascent and the primal-infeasibility bound (Lemma 2, Eq.(7), Eq.(8))
# ---------------------------------------------------------------------------

def test_projected_gradient_ascent_lemma(oracle_lib):
    """Plain step lam+ = Pi_{>=0}(lam + grad/L), L = |A'|^2/gamma = 1/gamma after
    row normalization: every step gains at least |(grad)_+|^2/(2L), and
    Lemma 2 bounds the infeasibility by sqrt(2L(g* - g))."""
    O = oracle_lib
    inst = tiny_binding(80)
    gamma = 0.05
    Pstar, _ = qp_optimum(inst, gamma)
    D = O.row_scale(inst)
    scaled = I.Instance(inst.m, inst.n, inst.dst, D[inst.dst] * inst.a, inst.c, D * inst.b,
                        inst.block_off, inst.block_proj, inst.upper)
    L = 1.0 / gamma
    lam = np.zeros(inst.m)
    prev = O.dual_eval(scaled, lam, gamma)
    gs = [prev.g]
    for _ in range(200):
        lam = np.maximum(0.0, lam + prev.grad / L)
        ev = O.dual_eval(scaled, lam, gamma)
        gain = ev.g - prev.g
        need = np.sum(np.maximum(prev.grad, 0) ** 2) / (2 * L)
        assert gain >= need - 1e-10 * max(1, abs(ev.g))
        infeas = np.linalg.norm(np.maximum(ev.grad, 0))
        assert infeas <= np.sqrt(2 * L * max(Pstar - ev.g, 0.0)) + 1e-7
        prev = ev
        gs.append(ev.g)
    # the oracle's solve loop with momentum and the secant estimate off is that
    # same iteration
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=201,
                                  check_every=0, max_step=gamma, init_step=gamma,
                                  momentum=0, adaptive=0))
    np.testing.assert_allclose(r.trace[:, 0], gs, rtol=1e-12)


def test_accelerated_run_is_valid(oracle_lib):
    """The accelerated loop keeps lam >= 0, never steps beyond the cap, and
    its Lipschitz estimates never exceed L = 1/gamma (normalized A)."""
    O = oracle_lib
    inst = I.random_small(81, I=300, J=25, dmax=10, box_frac=0.3, capacity="greedy")
    gamma = 0.01
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=400,
                                  check_every=10, tol_rel_gap=0.0, max_step=10 * gamma,
                                  init_step=1e-2 * gamma))
    assert np.all(r.lam >= 0)
    eta = r.trace[:, 2]
    assert np.all(eta <= 10 * gamma * (1 + 1e-15))
    assert np.all(eta[1:] >= gamma * (1 - 1e-9))   # 1/L^ >= 1/L
    gaps = r.trace[:, 1]
    gaps = gaps[~np.isnan(gaps)]
    assert np.all(gaps >= -1e-12)
    assert gaps[-1] < gaps[0]


# ---------------------------------------------------------------------------
# printed hyper-parameters and the gamma schedule
# ---------------------------------------------------------------------------

def test_paper_gamma_schedule_and_step_cap(oracle_lib):
    O = oracle_lib
    with open(os.path.join(HERE, "golden", "paper_hyperparameters.json")) as f:
        hp = json.load(f)
    cont = hp["continuation"]
    inst = tiny_binding(90)
    n_st = len(cont["expected_gammas"])
    every = cont["halve_every_iters"]
    r = O.solve(inst, O.SolveOpts(gamma0=cont["gamma_start"], gamma_final=cont["gamma_end"],
                                  n_stages=n_st, stage_iters=every, max_iters=every * n_st + 7,
                                  check_every=0, max_step=hp["max_step_size"],
                                  init_step=hp["initial_step_size"], adaptive=0))
    gam = r.trace[:, 3]
    for s, gexp in enumerate(cont["expected_gammas"]):
        seg = gam[s * every:(s + 1) * every]
        np.testing.assert_allclose(seg, gexp, rtol=1e-12)
    # step cap scales with gamma (Section 5, regularization decay)
    eta = r.trace[:, 2]
    np.testing.assert_allclose(eta, hp["max_step_size"] * gam / cont["gamma_start"], rtol=1e-12)
    # first step of the adaptive run is the printed initial step size
    r2 = O.solve(inst, O.SolveOpts(gamma0=hp["gamma"], gamma_final=hp["gamma"], max_iters=3,
                                   check_every=0, max_step=hp["max_step_size"],
                                   init_step=hp["initial_step_size"]))
    assert r2.trace[0, 2] == hp["initial_step_size"]
    assert r2.trace[1, 2] <= hp["max_step_size"]


def test_row_scale_uses_primal_scale(oracle_lib):
    """Row norms are taken of A D_v^{-1}: sum_{e->j} (D_j a_e / v_e)^2 = 1."""
    O = oracle_lib
    inst = I.random_small(43, I=100, J=12, dmax=6)
    v = np.random.default_rng(5).uniform(0.2, 3.0, size=inst.n)
    D = O.row_scale(inst, v=v)
    ssq = np.bincount(inst.dst, weights=(D[inst.dst] * inst.a / v) ** 2, minlength=inst.m)
    nonempty = np.bincount(inst.dst, minlength=inst.m) > 0
    np.testing.assert_allclose(ssq[nonempty], 1.0, rtol=1e-13)


def quadratic_regime_instance(seed):
    """Box blocks with unreachable bounds and c far below zero, A already row
    normalized: every projection stays inactive, so g is the concave quadratic
    of the Section 5 closed form with Hessian -A A'/gamma = -I/gamma, and
    lam* is chosen positive by setting b = (-A c - lam*)/gamma."""
    inst = I.random_small(seed, I=80, J=9, dmax=6, box_frac=1.0)
    rng = np.random.default_rng(seed)
    ssq = np.bincount(inst.dst, weights=inst.a ** 2, minlength=inst.m)
    assert np.all(ssq > 0)
    inst.a = inst.a / np.sqrt(ssq[inst.dst])
    inst.c = -10.0 - rng.uniform(0, 1, size=inst.n)
    inst.upper = np.full(inst.n, 1e12)
    gamma = 0.05
    lam_star = rng.uniform(0.1, 0.5, size=inst.m)
    A = inst.dense()
    inst.b = (-(A @ inst.c) - lam_star) / gamma
    return inst, A, gamma, lam_star


def quad_g(inst, A, gamma, lam):
    x = -(inst.c + A.T @ lam) / gamma
    return inst.c @ x + 0.5 * gamma * x @ x + lam @ (A @ x - inst.b)


def test_momentum_on_exact_quadratic(oracle_lib):
    """Step 1/L = gamma reaches lam* in one step; FISTA's first momentum
    coefficient (t_0 - 1)/t_1 is zero, so every later evaluation sits at
    lam* and g stays at the closed-form optimum."""
    O = oracle_lib
    inst, A, gamma, lam_star = quadratic_regime_instance(91)
    gstar = quad_g(inst, A, gamma, lam_star)
    assert quad_g(inst, A, gamma, lam_star * 1.01) < gstar
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=6, check_every=0,
                                  max_step=gamma, init_step=gamma, adaptive=0))
    g0 = quad_g(inst, A, gamma, np.zeros(inst.m))
    assert r.trace[0, 0] == pytest.approx(g0, rel=1e-12)
    np.testing.assert_allclose(r.trace[1:, 0], gstar, rtol=1e-12)
    np.testing.assert_allclose(r.lam, lam_star, rtol=1e-9)


def test_secant_lipschitz_estimate_on_exact_quadratic(oracle_lib):
    """On the quadratic with Hessian -I/gamma the secant estimate
    |G - G_prev|/|y - y_prev| is exactly 1/gamma, so every step after the
    initial one is gamma when the cap is larger."""
    O = oracle_lib
    inst, A, gamma, lam_star = quadratic_regime_instance(92)
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=8, check_every=0,
                                  max_step=5 * gamma, init_step=0.1 * gamma))
    assert r.trace[0, 2] == 0.1 * gamma
    # while the iterates still move (|G| well above rounding) the estimate is exact
    moving = np.nonzero(r.trace[:, 5] > 1e-6)[0]
    k_last = int(moving[-1]) + 1          # uses the last moving pair
    assert k_last >= 3
    np.testing.assert_allclose(r.trace[1:k_last + 1, 2], gamma, rtol=1e-9)


def test_fista_golden_sequence_is_self_consistent():
    """The stored FISTA sequence obeys its defining identities (Beck and
    Teboulle 2009): t_0 = 1, t_1 is the golden ratio, t_{k+1}^2 - t_{k+1} =
    t_k^2, t_k >= (k+2)/2 (their Lemma 4.3, shifted to a 0-based count) and
    beta_k = (t_k - 1)/t_{k+1}."""
    with open(os.path.join(HERE, "golden", "fista_sequence.json")) as f:
        fs = json.load(f)
    t = np.array(fs["t"])
    beta = np.array(fs["beta"])
    assert t[0] == 1.0
    assert t[1] == pytest.approx((1 + 5 ** 0.5) / 2, rel=1e-15)
    np.testing.assert_allclose(t[1:] ** 2 - t[1:], t[:-1] ** 2, rtol=1e-14)
    assert np.all(t >= (np.arange(len(t)) + 2) / 2)
    np.testing.assert_allclose(beta, (t[:-1] - 1) / t[1:], rtol=1e-14, atol=1e-16)


def two_curvature_quadratic(seed):
    """Quadratic regime (every projection inactive, as in
    quadratic_regime_instance) without row normalization: rows of even index
    have norm 1, odd rows norm 1/2, so A A' = diag(n_j^2) and the dual is the
    separable quadratic g(lam) = g* - 1/2 sum_j h_j (lam_j - lam*_j)^2 with
    two curvatures h_j = n_j^2/gamma.  b = (-A c - diag(n^2) lam*)/gamma puts
    the maximiser at lam* > 0."""
    inst = I.random_small(seed, I=60, J=8, dmax=5, box_frac=1.0)
    rng = np.random.default_rng(seed)
    ssq = np.bincount(inst.dst, weights=inst.a ** 2, minlength=inst.m)
    assert np.all(ssq > 0)
    nrm = np.where(np.arange(inst.m) % 2 == 0, 1.0, 0.5)
    inst.a = inst.a * nrm[inst.dst] / np.sqrt(ssq[inst.dst])
    inst.c = -10.0 - rng.uniform(0, 1, size=inst.n)
    inst.upper = np.full(inst.n, 1e12)
    gamma = 0.05
    lam_star = rng.uniform(0.2, 0.6, size=inst.m)
    A = inst.dense()
    inst.b = (-(A @ inst.c) - nrm ** 2 * lam_star) / gamma
    return inst, A, gamma, lam_star, nrm ** 2 / gamma


def test_fista_momentum_trajectory_on_separable_quadratic(oracle_lib):
    """Pins the momentum of the accelerated loop (coefficient and t-update).

    With a fixed step eta below 1/L and every projection inactive, each
    coordinate's error e = lam - lam* follows a scalar linear recursion:
    the step multiplies it by (1 - eta h_j), and the momentum point is
    y = lam_+ + beta_k (lam_+ - lam) with the stored FISTA coefficients.
    The expected g(y_k) = g* - 1/2 sum_j h_j e_j(y_k)^2 follows from that
    recursion alone; the oracle evaluates gradients of the full LP instead.
    A wrong coefficient ((t-1)/(t+1), or t_+ = (1 + sqrt(1 + t^2))/2) moves
    g(y_2) and every later value by far more than the tolerance."""
    O = oracle_lib
    with open(os.path.join(HERE, "golden", "fista_sequence.json")) as f:
        beta = np.array(json.load(f)["beta"])
    inst, A, gamma, lam_star, h = two_curvature_quadratic(93)
    gstar = quad_g(inst, A, gamma, lam_star)
    eta = gamma / 3.0                       # below 1/L = gamma / max n_j^2
    K = len(beta)                           # evaluations y_0 .. y_{K-1}
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=K,
                                  check_every=0, max_step=eta, init_step=eta, adaptive=0,
                                  row_normalize=0))
    # scalar recursion per coordinate, errors relative to lam*
    e_lam = -lam_star.copy()                # lam_0 = 0
    e_y = -lam_star.copy()                  # y_0 = 0
    expect = []
    for k in range(K):
        expect.append(-0.5 * np.sum(h * e_y ** 2))
        e_new = (1.0 - eta * h) * e_y
        e_y = e_new + beta[k] * (e_new - e_lam)
        e_lam = e_new
        assert np.all(lam_star + e_y > 0)   # projections onto lam >= 0 stay inactive
    expect = np.array(expect)
    got = r.trace[:, 0] - gstar
    assert got[-1] < -1e-3                  # still far from lam*: momentum matters
    np.testing.assert_allclose(got, expect, rtol=1e-7)
    # the returned point is the last evaluated one, y_{K-1}
    e_last = -lam_star.copy()
    e_l = -lam_star.copy()
    for k in range(K - 1):
        e_new = (1.0 - eta * h) * e_last
        e_last, e_l = e_new + beta[k] * (e_new - e_l), e_new
    np.testing.assert_allclose(r.lam, lam_star + e_last, rtol=1e-9)


def test_momentum_restarts_at_gamma_stage(oracle_lib):
    """At a stage change the momentum restarts (t = 1, y = lam_+): the first
    step of the new stage carries no momentum.  On the separable quadratic a
    two-stage run with stage_iters = 3 gives, in stage 1, the same error
    recursion as a fresh run started from the stage-0 iterate."""
    O = oracle_lib
    with open(os.path.join(HERE, "golden", "fista_sequence.json")) as f:
        beta = np.array(json.load(f)["beta"])
    inst, A, gamma, lam_star, h = two_curvature_quadratic(94)
    # both stages at the same gamma, so the quadratic does not change
    eta = gamma / 3.0
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, n_stages=2, stage_iters=3,
                                  max_iters=7, check_every=0, max_step=eta, init_step=eta,
                                  adaptive=0, row_normalize=0))
    gstar = quad_g(inst, A, gamma, lam_star)
    e_lam = -lam_star.copy()
    e_y = -lam_star.copy()
    expect, kb = [], 0
    for k in range(7):
        expect.append(-0.5 * np.sum(h * e_y ** 2))
        e_new = (1.0 - eta * h) * e_y
        if k == 2:                          # stage advance after 3 iterations
            e_y, e_lam, kb = e_new.copy(), e_new, 0
            continue
        e_y = e_new + beta[kb] * (e_new - e_lam)
        e_lam = e_new
        kb += 1
    np.testing.assert_allclose(r.trace[:, 0] - gstar, expect, rtol=1e-7)
    np.testing.assert_array_equal(r.trace[:, 4], [0, 0, 0, 1, 1, 1, 1])


def test_momentum_point_is_projected_to_nonnegative(oracle_lib):
    """The momentum point y is projected onto lam >= 0, so every evaluated
    g(y) is a valid dual bound.  On the separable quadratic with the
    unconstrained maximiser negative in half the coordinates and a warm
    start at lam = 1, the step drives those coordinates to 0 and the momentum
    would push y below 0; the expected values clip y at 0, and g(y) is the
    closed-form quadratic at the clipped point."""
    O = oracle_lib
    with open(os.path.join(HERE, "golden", "fista_sequence.json")) as f:
        beta = np.array(json.load(f)["beta"])
    inst, A, gamma, lam_pos, h = two_curvature_quadratic(95)
    lam_star = lam_pos * np.where(np.arange(inst.m) % 4 < 2, 1.0, -1.0)
    nrm2 = h * gamma
    inst.b = (-(A @ inst.c) - nrm2 * lam_star) / gamma
    gstar = quad_g(inst, A, gamma, lam_star)
    eta = gamma / 1.5
    K = len(beta)
    lam0 = np.ones(inst.m)
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=K,
                                  check_every=0, max_step=eta, init_step=eta, adaptive=0,
                                  row_normalize=0), lam0=lam0)
    lam, y = lam0.copy(), lam0.copy()
    expect, clipped = [], False
    for k in range(K):
        expect.append(-0.5 * np.sum(h * (y - lam_star) ** 2))
        ln = np.maximum(0.0, y + eta * h * (lam_star - y))
        z = ln + beta[k] * (ln - lam)
        clipped |= bool(np.any(z < 0))
        y, lam = np.maximum(0.0, z), ln
    assert clipped                          # the projection of y is exercised
    np.testing.assert_allclose(r.trace[:, 0] - gstar, expect, rtol=1e-7)


# ---------------------------------------------------------------------------
# several matching families (Definition 1) and the global count row (Section 4)
# ---------------------------------------------------------------------------

def brute_block(proj, t, w, u):
    if proj == I.PROJ_SIMPLEX:
        return brute_simplex(t, w)
    if proj == I.PROJ_CAPPED:
        return brute_capped(t, w, u)
    return brute_box(t, w, u)


@pytest.mark.parametrize("count", [False, True])
def test_multi_family_products_projection_and_row_scale(oracle_lib, count):
    """Columns with one entry per family (and one in the count row): x is the
    blockwise projection of -(A'lam + c)/gamma by brute force on dense A, the
    gradient is A x - b, g follows Eq.(2); every nonempty row of D A has unit
    norm (A'A'^T has a unit diagonal, Section 5) and g'(lam') = g(D lam')."""
    O = oracle_lib
    inst = I.multi_family(I=30, J=5, families=3 if not count else 2, count_row=count, seed=9,
                          box_frac=0.3, capped_frac=0.3, dmax=5)
    A = inst.dense()
    rng = np.random.default_rng(4)
    lam = rng.uniform(0, 0.6, size=inst.m)
    gamma = 0.05
    ev = O.dual_eval(inst, lam, gamma)
    t = -(A.T @ lam + inst.c)
    u = inst.upper if inst.upper is not None else np.ones(inst.n)
    x = np.concatenate([brute_block(int(inst.block_proj[i]), t[lo:hi], np.full(hi - lo, 1 / gamma),
                                    u[lo:hi])
                        for i, (lo, hi) in enumerate(zip(inst.block_off[:-1], inst.block_off[1:]))])
    np.testing.assert_allclose(ev.x, x, rtol=1e-9, atol=1e-12)
    np.testing.assert_allclose(ev.grad, A @ x - inst.b, rtol=1e-12, atol=1e-12)
    g = inst.c @ x + 0.5 * gamma * x @ x + lam @ (A @ x - inst.b)
    assert ev.g == pytest.approx(g, rel=1e-12)
    D = O.row_scale(inst)
    A2 = D[:, None] * A
    nonempty = np.abs(A).sum(axis=1) > 0
    np.testing.assert_allclose(np.diag(A2 @ A2.T)[nonempty], 1.0, rtol=1e-13)
    scaled = I.MultiInstance(inst.m, inst.n, inst.colptr, inst.rowidx,
                             D[inst.rowidx] * inst.val, inst.c, D * inst.b, inst.block_off,
                             inst.block_proj, inst.upper, inst.J, inst.families, inst.count_row)
    e1 = O.dual_eval(scaled, lam, gamma)
    e0 = O.dual_eval(inst, D * lam, gamma)
    assert e1.g == pytest.approx(e0.g, rel=1e-12)
    np.testing.assert_allclose(e1.grad, D * e0.grad, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("seed", [80, 81])
def test_multi_family_gap_brackets_qp_optimum(oracle_lib, seed):
    """With columns in several rows the restored point scales each edge by
    the worst ratio of its rows: it must be feasible, so at any lam >= 0
    g <= P*_gamma <= P (P* from SLSQP on the dense primal QP), and a converged
    solve reaches P* (1e-7)."""
    O = oracle_lib
    inst = I.multi_family(I=10, J=3, families=2, count_row=True, seed=seed, box_frac=0.3,
                          dmax=3, count_frac=0.4)
    gamma = 0.05
    Pstar, _ = qp_optimum(inst, gamma)
    scale = max(1.0, abs(Pstar))
    rng = np.random.default_rng(seed)
    for _ in range(6):
        lam = rng.exponential(1.0, size=inst.m) * (rng.random(inst.m) < 0.7)
        ev = O.dual_eval(inst, lam, gamma)
        assert ev.g <= Pstar + 1e-9 * scale
        assert ev.P >= Pstar - 1e-9 * scale
    r = O.solve(inst, O.SolveOpts(gamma0=gamma, gamma_final=gamma, max_iters=40000,
                                  check_every=10, tol_rel_gap=1e-11, max_step=0.2 * gamma,
                                  init_step=1e-3 * gamma))
    assert r.converged
    assert abs(r.g - Pstar) / scale < 1e-7


def test_multi_family_gradient_is_finite_difference_of_g(oracle_lib):
    O = oracle_lib
    inst = I.multi_family(I=40, J=6, families=2, count_row=True, seed=12, box_frac=0.3, dmax=6)
    rng = np.random.default_rng(5)
    lam = rng.uniform(0.1, 0.8, size=inst.m)
    gamma = 0.1
    ev = O.dual_eval(inst, lam, gamma)
    for h in (1e-6, 1e-7):
        fd = np.empty(inst.m)
        for r in range(inst.m):
            e = np.zeros(inst.m)
            e[r] = h
            fd[r] = (O.dual_eval(inst, lam + e, gamma).g - O.dual_eval(inst, lam - e, gamma).g) / (2 * h)
        np.testing.assert_allclose(fd, ev.grad, rtol=1e-5, atol=1e-6)


def test_multi_row_restoration_worked_example(oracle_lib):
    """A column in two violated rows is scaled by the smaller ratio: the
    hand-derived example in tests/golden/multi_row_restoration.json."""
    O = oracle_lib
    with open(os.path.join(HERE, "golden", "multi_row_restoration.json")) as f:
        ex = json.load(f)
    inst = ex["instance"]
    colptr = [0]
    rows, vals = [], []
    for col in inst["columns"]:
        for r, v in col["entries"]:
            rows.append(r)
            vals.append(v)
        colptr.append(len(rows))
    lp = O.LP(inst["rows"], 2, np.array(rows, dtype=np.int32), np.array(vals),
              np.array(inst["c"]), np.array(inst["b"]), np.array([0, 2], dtype=np.int64),
              np.array([I.PROJ_BOX], dtype=np.uint8), upper=np.ones(2),
              colptr=np.array(colptr, dtype=np.int64))
    ev = O.dual_eval(lp, np.array(inst["lambda"]), inst["gamma"])
    np.testing.assert_allclose(ev.x, ex["x"], rtol=1e-15)
    assert ev.g == pytest.approx(ex["g"], rel=1e-15)
    assert ev.P == pytest.approx(ex["P"], rel=1e-15)
