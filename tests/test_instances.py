"""Host checks of the seeded instance recipes (no solver arithmetic).

The Appendix B construction is checked against its description: Poisson
resource degrees truncated at I, distinct requests per resource, values
capped at c_max with the cost their negative, coefficients a_ij = s_j c_ij
with one scale per resource, capacities b_j = rho_j (l_j + eps) with rho_j in
[0.5, 1] from the greedy load l_j recomputed here edge by edge.
"""
import numpy as np

from paper_2603_04621_amd import instances as I


def test_counting_order_is_a_stable_argsort():
    rng = np.random.default_rng(3)
    for nkeys in (1, 7, 1000):
        k = rng.integers(0, nkeys, size=5000)
        assert np.array_equal(I.counting_order(k, nkeys), np.argsort(k, kind="stable"))


def test_appendix_b_construction():
    Ireq, J = 20_000, 300
    x = I.appendix_b(I=Ireq, J=J, nu=10.0, seed=99)
    K = x.meta["K"]
    assert np.all(K <= Ireq)
    # edges per resource are exactly the Poisson draws; total near I * nu
    assert np.array_equal(np.bincount(x.dst, minlength=J), K)
    assert abs(x.n / Ireq - 10.0) < 0.5
    # source-major blocks: one per request, destinations distinct within it
    deg = np.diff(x.block_off)
    assert deg.shape[0] == Ireq and deg.sum() == x.n
    for i in range(0, Ireq, 97):
        d = x.dst[x.block_off[i]:x.block_off[i + 1]]
        assert np.unique(d).size == d.size
    # values in (0, c_max], costs their negatives, a_ij = s_j * value
    val = -x.c
    assert np.all(val > 0) and np.all(val <= I.APPB_CMAX) and np.any(val == I.APPB_CMAX)
    s = x.meta["s"]
    np.testing.assert_allclose(x.a, s[x.dst] * val, rtol=1e-15)
    # rows differ in magnitude by orders (the point of the construction)
    rn = np.sqrt(np.bincount(x.dst, weights=x.a ** 2, minlength=J))
    assert rn[rn > 0].max() / rn[rn > 0].min() > 100
    # greedy load: each request's largest a_ij sent to its resource
    load = np.zeros(J)
    for i in range(Ireq):
        lo, hi = x.block_off[i], x.block_off[i + 1]
        if hi > lo:
            e = lo + int(np.argmax(x.a[lo:hi]))
            load[x.dst[e]] += x.a[e]
    rho = x.b / (load + I.APPB_EPS)
    assert np.all(rho >= 0.5 - 1e-12) and np.all(rho <= 1.0 + 1e-12)
    assert np.all(x.block_proj == I.PROJ_SIMPLEX)


def test_appendix_b_is_seeded():
    a = I.appendix_b(I=3000, J=50, seed=5)
    b = I.appendix_b(I=3000, J=50, seed=5)
    c = I.appendix_b(I=3000, J=50, seed=6)
    assert np.array_equal(a.dst, b.dst) and np.array_equal(a.a, b.a) and np.array_equal(a.b, b.b)
    assert not (a.n == c.n and np.array_equal(a.a, c.a))
