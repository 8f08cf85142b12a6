"""Seeded synthetic matching-LP instances.

This module holds only random draws and the definitions of the synthetic
workloads (sizes, distributions, capacities).  It contains none of the
solver's arithmetic, so both the CPU oracle's tests and the GPU path can read
the same arrays from it.

Problem shape (single matching family, Section 3.2 of the paper): sources
i = 0..I-1 own contiguous blocks of primal variables, one variable per
eligible (source, destination) edge; each variable has exactly one nonzero
a_e in row j(e) of A (destination capacity, Eq.(3)); every block carries one
simple constraint: the per-source simplex sum_e x_e <= 1, x >= 0
(Eq.(4),(5)), a box 0 <= x_e <= u_e, or the capped simplex (both).

A is handed over in CSC form with one entry per column, so the column
pointer is the identity and is not materialised (``Instance.csc`` returns
it on demand); ``Instance.csr`` builds the row-major form of the same matrix.

Workload recipes (all draws in float64 from numpy's PCG64, seed
4621000 + k unless stated):

* ``tiny``   I=1000, J=50, 10 distinct uniform destinations per source,
             c=-U(0,1), a=U(0.5,1.5), simplex blocks, b_j=0.4*sum_{e->j} a_e.
* ``large``  I=10M, J=10k, degree 1+Poisson(9), destinations Zipf(1.1)
             (ranks mapped to ids by a seeded permutation, duplicates within
             a source discarded and redrawn), c=-LogNormal(0,1),
             a=LogNormal(0,0.5), simplex blocks, b_j=0.3*sum_{e->j} a_e.
* ``heavy``  I=2M, J=50k, degree clip(round(6.5*U^(-1/1.2)),1,4096)
             (Pareto alpha=1.2, scale 6.5), Zipf(1.1) destinations, 30% of
             sources box-constrained with u_e=U(0.2,1), others simplex.
* ``batch``  256 LPs, I log-uniform in [1e3,1e6], J=max(1,I//200), degree
             min(J, 1+Poisson(9)), as ``large`` otherwise.
* ``serve``  request stream, Poisson arrivals, I log-uniform, J=I//500,
             70/30 simplex/box blocks, as ``heavy`` otherwise.
* ``appendix_b`` the paper's own synthetic construction (Appendix B):
             lognormal resource breadths, Poisson resource degrees, values
             min(v_j u_i eps_ij, c_max), a_ij = s_j c_ij with lognormal s_j,
             greedy-load capacities; constants in APPB_* below.

Every generator takes explicit sizes so the same recipe can be drawn at a
scale the oracle finishes in seconds.

Capacities.  ``capacity="sum"`` is the rule of the recipes above
(b_j = frac * sum_{e->j} a_e).  Since a source can put at most a unit of mass
on its ~10 edges, that rule never binds (the load at lam = 0 stays below b), so
lam* = 0.  ``capacity="greedy"`` is the paper's own construction (Appendix B:
b_j = rho_j (l_j + eps) from the greedy load l_j, rho_j ~ U[0.5, 1],
eps = 0.01), under which some constraints bind; convergence checks use it.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Iterator, Optional

import numpy as np

PROJ_SIMPLEX = 0
PROJ_BOX = 1
PROJ_CAPPED = 2

SEED_BASE = 4621000


@dataclass
class Instance:
    """One matching LP: min c'x s.t. A x <= b, x in C (Eq.(1))."""

    m: int                       # rows of A = destinations J
    n: int                       # columns of A = edges / primal variables
    dst: np.ndarray              # int32 [n]   row of column e's single entry
    a: np.ndarray                # float64 [n] value of that entry
    c: np.ndarray                # float64 [n]
    b: np.ndarray                # float64 [m]
    block_off: np.ndarray        # int64 [I+1] contiguous cover of [0, n)
    block_proj: np.ndarray       # uint8 [I]   PROJ_SIMPLEX / PROJ_BOX
    upper: Optional[np.ndarray]  # float64 [n] box bounds, None = all 1.0
    name: str = ""
    seed: int = 0
    meta: dict = field(default_factory=dict)

    @property
    def num_blocks(self) -> int:
        return int(self.block_off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.n)

    def degrees(self) -> np.ndarray:
        return np.diff(self.block_off)

    def csc(self):
        """(colptr int64 [n+1], rowidx int32 [n], val float64 [n])."""
        return np.arange(self.n + 1, dtype=np.int64), self.dst, self.a

    def csr(self):
        """(rowptr int64 [m+1], colidx int32 [n], val float64 [n]) of the same A."""
        order = np.argsort(self.dst, kind="stable")
        counts = np.bincount(self.dst, minlength=self.m)
        rowptr = np.zeros(self.m + 1, dtype=np.int64)
        np.cumsum(counts, out=rowptr[1:])
        return rowptr, order.astype(np.int32), self.a[order]

    def dense(self) -> np.ndarray:
        """Dense A (tiny instances only)."""
        A = np.zeros((self.m, self.n))
        A[self.dst, np.arange(self.n)] = self.a
        return A

    def rounded(self, storage: str) -> "Instance":
        """Same instance with the values a device store of type ``storage``
        ("f64", "f32", "bf16") holds: a and c rounded to that type, box bounds
        to float32 (they are always stored as float32), widened back to float64.
        Used so a CPU check at float64 sees exactly the stored values.
        """
        def rnd(v):
            if storage == "bf16":
                return _round_bf16(v)
            if storage == "f32":
                return v.astype(np.float32).astype(np.float64)
            return v.copy()
        up = None if self.upper is None else self.upper.astype(np.float32).astype(np.float64)
        return Instance(self.m, self.n, self.dst, rnd(self.a), rnd(self.c), self.b,
                        self.block_off, self.block_proj, up,
                        self.name + f"[{storage}]", self.seed, dict(self.meta))


def _round_bf16(v: np.ndarray) -> np.ndarray:
    """Round float64 -> bfloat16 (nearest-even via float32) -> float64."""
    f = v.astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ----------------------------------------------------------------------------
# samplers
# ----------------------------------------------------------------------------

def zipf_cdf(J: int, s: float) -> np.ndarray:
    """CDF of ranks 0..J-1 with P(rank k) proportional to (k+1)^-s (truncated Zipf)."""
    k = np.arange(1, J + 1, dtype=np.float64)
    p = k ** (-s)
    p /= p.sum()
    cdf = np.cumsum(p)
    cdf[-1] = 1.0
    return cdf


def uniform_cdf(J: int) -> np.ndarray:
    cdf = np.arange(1, J + 1, dtype=np.float64) / J
    cdf[-1] = 1.0
    return cdf


_SAMPLER_LIB = None


def _sampler_lib():
    """ctypes handle of the compiled distinct-rank helper (built by build())."""
    global _SAMPLER_LIB
    if _SAMPLER_LIB is None:
        import ctypes
        import os
        path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdlsample.so")
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: run __graft_entry__.build() first")
        lib = ctypes.CDLL(path)
        f = lib.dl_gen_distinct
        f.restype = ctypes.c_int64
        f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                      ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                      ctypes.c_void_p]
        _SAMPLER_LIB = lib
    return _SAMPLER_LIB


SOURCES_PER_CHUNK = 1 << 19


def distinct_destinations(seed_key, deg: np.ndarray, J: int, cdf: np.ndarray) -> np.ndarray:
    """For each source draw deg[i] distinct ranks in 0..J-1: successive
    inverse-CDF draws, a rank already held by the source being discarded
    (the without-replacement law of ``cdf``).  Sources are taken in chunks of
    SOURCES_PER_CHUNK; chunk q reads uniforms from its own PCG64 stream keyed
    by ``seed_key + [q]``, so chunks can be drawn on several threads and the
    result does not depend on the thread count.  Ranks keep their draw order.
    """
    import os
    from concurrent.futures import ThreadPoolExecutor
    lib = _sampler_lib()
    deg = np.ascontiguousarray(deg, dtype=np.int64)
    I = deg.shape[0]
    off = np.zeros(I + 1, dtype=np.int64)
    np.cumsum(deg, out=off[1:])
    out = np.empty(int(off[-1]), dtype=np.int32)
    cdf = np.ascontiguousarray(cdf, dtype=np.float64)
    key = list(seed_key) if isinstance(seed_key, (list, tuple)) else [seed_key]

    def run(q):
        s0 = q * SOURCES_PER_CHUNK
        s1 = min(I, s0 + SOURCES_PER_CHUNK)
        d = deg[s0:s1]
        n = int(off[s1] - off[s0])
        mark = np.empty(5 * J, dtype=np.int32)
        nfb = np.zeros(1, dtype=np.int64)
        view = out[off[s0]:off[s1]]
        size = n + n // 2 + 4096
        while True:
            u = np.random.default_rng(key + [q]).random(size)
            used = lib.dl_gen_distinct(s1 - s0, d.ctypes.data, J, cdf.ctypes.data,
                                       u.ctypes.data, size, view.ctypes.data,
                                       mark.ctypes.data, nfb.ctypes.data)
            if used >= 0:
                return
            if used == -2:
                raise ValueError("bad arguments to the distinct-rank sampler")
            size *= 2

    nq = (I + SOURCES_PER_CHUNK - 1) // SOURCES_PER_CHUNK
    workers = max(1, min(nq, 16, os.cpu_count() or 1))
    if workers == 1:
        for q in range(nq):
            run(q)
    else:
        with ThreadPoolExecutor(workers) as ex:
            list(ex.map(run, range(nq)))
    return out


def counting_order(key: np.ndarray, nkeys: int) -> np.ndarray:
    """Stable order of the positions of `key` (int64 in [0, nkeys)) by key:
    what np.argsort(key, kind="stable") returns, in O(n)."""
    import ctypes
    lib = _sampler_lib()
    f = lib.dl_counting_order
    f.restype = ctypes.c_int64
    f.argtypes = [ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                  ctypes.c_void_p]
    key = np.ascontiguousarray(key, dtype=np.int64)
    out = np.empty(key.shape[0], dtype=np.int64)
    cnt = np.empty(int(nkeys) + 1, dtype=np.int64)
    if f(key.shape[0], key.ctypes.data, int(nkeys), cnt.ctypes.data, out.ctypes.data) != 0:
        raise ValueError("key out of range")
    return out


def greedy_capacity(dst, a, block_off, J, seed_key, eps: float = 1e-2) -> np.ndarray:
    """Capacities of the paper's synthetic construction (Appendix B): every
    source sends its largest a_e to that edge's destination, giving the greedy
    load l_j; then b_j = rho_j (l_j + eps) with rho_j ~ U[0.5, 1] drawn from
    their own stream.  Some constraints bind at the optimum, others stay slack.
    """
    deg = np.diff(block_off)
    nz = deg > 0
    starts = block_off[:-1][nz]
    # index of the largest a in each block (first one on ties): the first
    # position at or after the block start that holds the block maximum
    mx = np.maximum.reduceat(a, starts)
    hits = np.flatnonzero(a == np.repeat(mx, deg[nz]))
    best = hits[np.searchsorted(hits, starts)]
    load = np.bincount(dst[best], weights=a[best], minlength=J)
    rho = np.random.default_rng(seed_key).uniform(0.5, 1.0, size=J)
    return rho * (load + eps)


def _finish(name, seed, I, J, deg, rng, cdf, c_law, a_law, b_frac,
            box_frac=0.0, perm_ids=True, meta=None, seed_key=None,
            capacity: str = "sum", capped_frac: float = 0.0) -> Instance:
    deg = np.minimum(deg.astype(np.int64), J)
    if seed_key is None:
        seed_key = [seed, 1]
    ranks = distinct_destinations(seed_key, deg, J, cdf)
    if perm_ids:
        perm = rng.permutation(J)
        dst = perm[ranks].astype(np.int32)
    else:
        dst = ranks.astype(np.int32)
    n = int(deg.sum())
    c = c_law(rng, n)
    a = a_law(rng, n)
    block_off = np.zeros(I + 1, dtype=np.int64)
    np.cumsum(deg, out=block_off[1:])
    if capacity == "sum":
        b = b_frac * np.bincount(dst, weights=a, minlength=J)
    elif capacity == "greedy":
        b = greedy_capacity(dst, a, block_off, J, list(seed_key) + [2])
    else:
        raise ValueError(f"unknown capacity rule {capacity!r}")
    if box_frac > 0.0 or capped_frac > 0.0:
        # one uniform per source: box below box_frac, capped simplex in the
        # next capped_frac, simplex above; bounds u = U(0.2, 1) on box and
        # capped blocks
        r = rng.random(I)
        block_proj = (r < box_frac).astype(np.uint8)
        block_proj[(r >= box_frac) & (r < box_frac + capped_frac)] = PROJ_CAPPED
        upper = np.ones(n)
        is_box = np.repeat(block_proj != PROJ_SIMPLEX, deg)
        upper[is_box] = rng.uniform(0.2, 1.0, size=int(is_box.sum()))
    else:
        block_proj = np.zeros(I, dtype=np.uint8)
        upper = None
    meta = dict(meta or {})
    meta["capacity"] = capacity
    return Instance(J, n, dst, a, c, b, block_off, block_proj, upper, name, seed, meta)


def _neg_uniform(rng, n):
    return -rng.random(n)


def _uniform_a(rng, n):
    return rng.uniform(0.5, 1.5, size=n)


def _neg_lognormal(rng, n):
    return -rng.lognormal(0.0, 1.0, size=n)


def _lognormal_a(rng, n):
    return rng.lognormal(0.0, 0.5, size=n)


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------

def tiny(I: int = 1000, J: int = 50, d: int = 10, seed: int = SEED_BASE + 1,
         capacity: str = "sum") -> Instance:
    """Tiny uniform matching LP (the 1,000-source, 50-destination recipe)."""
    rng = np.random.default_rng(seed)
    deg = np.full(I, d, dtype=np.int64)
    return _finish("tiny", seed, I, J, deg, rng, uniform_cdf(J),
                   _neg_uniform, _uniform_a, 0.4, perm_ids=False,
                   meta={"I": I, "J": J, "d": d}, capacity=capacity)


def large(I: int = 10_000_000, J: int = 10_000, seed: int = SEED_BASE + 2,
          capacity: str = "sum") -> Instance:
    """Zipf-destination matching LP (10M sources, 10k destinations at full size)."""
    rng = np.random.default_rng(seed)
    deg = 1 + rng.poisson(9.0, size=I)
    return _finish("large", seed, I, J, deg, rng, zipf_cdf(J, 1.1),
                   _neg_lognormal, _lognormal_a, 0.3, meta={"I": I, "J": J},
                   capacity=capacity)


def pareto_degrees(rng, I: int, alpha: float = 1.2, scale: float = 6.5,
                   dmax: int = 4096) -> np.ndarray:
    u = 1.0 - rng.random(I)          # (0, 1]
    d = np.rint(scale * u ** (-1.0 / alpha))
    return np.clip(d, 1, dmax).astype(np.int64)


def heavy(I: int = 2_000_000, J: int = 50_000, seed: int = SEED_BASE + 3,
          dmax: int = 4096, box_frac: float = 0.3, capacity: str = "sum",
          capped_frac: float = 0.0) -> Instance:
    """Heavy-tailed blocks with mixed simplex/box projections (2M x 50k full size);
    capped_frac > 0 turns that share of the simplex blocks into capped simplices."""
    rng = np.random.default_rng(seed)
    deg = pareto_degrees(rng, I, dmax=dmax)
    return _finish("heavy", seed, I, J, deg, rng, zipf_cdf(J, 1.1),
                   _neg_lognormal, _lognormal_a, 0.3, box_frac=box_frac,
                   meta={"I": I, "J": J}, capacity=capacity, capped_frac=capped_frac)


def batch_sizes(count: int = 256, lo: float = 1e3, hi: float = 1e6,
                seed: int = SEED_BASE + 4) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)


def batch_member(I: int, k: int, seed: int = SEED_BASE + 4, j_div: int = 200,
                 capacity: str = "sum") -> Instance:
    """k-th LP of the batched workload (J = I/200, Poisson degrees, Zipf)."""
    rng = np.random.default_rng([seed, k])
    J = max(1, int(I) // j_div)
    deg = np.minimum(J, 1 + rng.poisson(9.0, size=int(I)))
    return _finish(f"batch[{k}]", seed, int(I), J, deg, rng, zipf_cdf(J, 1.1),
                   _neg_lognormal, _lognormal_a, 0.3, meta={"I": int(I), "J": J, "k": k},
                   seed_key=[seed, k, 1], capacity=capacity)


def batch(count: int = 256, lo: float = 1e3, hi: float = 1e6,
          seed: int = SEED_BASE + 4, capacity: str = "sum") -> list[Instance]:
    sizes = batch_sizes(count, lo, hi, seed)
    return [batch_member(int(I), k, seed, capacity=capacity) for k, I in enumerate(sizes)]


def serve_member(I: int, k: int, seed: int = SEED_BASE + 5, j_div: int = 500,
                 box_frac: float = 0.3, capacity: str = "sum") -> Instance:
    rng = np.random.default_rng([seed, k])
    J = max(1, int(I) // j_div)
    deg = np.minimum(J, 1 + rng.poisson(9.0, size=int(I)))
    return _finish(f"serve[{k}]", seed, int(I), J, deg, rng, zipf_cdf(J, 1.1),
                   _neg_lognormal, _lognormal_a, 0.3, box_frac=box_frac,
                   meta={"I": int(I), "J": J, "k": k}, seed_key=[seed, k, 1],
                   capacity=capacity)


def serve_stream(count: int, rate: float = 200.0, lo: float = 1e4, hi: float = 5e6,
                 seed: int = SEED_BASE + 5) -> list[tuple[float, int]]:
    """(arrival time in seconds, source count I) for a Poisson request stream."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    sizes = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=count))).astype(np.int64)
    t = np.cumsum(gaps) - gaps[0]
    return [(float(t[k]), int(sizes[k])) for k in range(count)]


def random_small(seed: int, I: int, J: int, dmax: int, box_frac: float = 0.5,
                 zipf: bool = False, b_frac: float = 0.3, capacity: str = "greedy",
                 capped_frac: float = 0.0) -> Instance:
    """Small mixed instance for property tests (degrees uniform in 1..dmax)."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(1, dmax + 1, size=I)
    cdf = zipf_cdf(J, 1.1) if zipf else uniform_cdf(J)
    return _finish("random_small", seed, I, J, deg, rng, cdf, _neg_lognormal,
                   _lognormal_a, b_frac, box_frac=box_frac, capacity=capacity,
                   capped_frac=capped_frac)


# Constants of the Appendix B construction that the paper leaves unstated
# (chosen here; all lognormals have location 0): spread of the resource
# breadths, of the resource value scales v_j, of the request factors u_i, of
# the edge noise eps_ij and of the per-resource coefficient scales s_j, the
# value cap c_max, and the small constant added to the greedy load.
APPB_SIGMA_BREADTH = 1.0
APPB_SIGMA_V = 0.5
APPB_SIGMA_U = 0.5
APPB_SIGMA_EPS = 0.25
APPB_SIGMA_S = 1.5
APPB_CMAX = 10.0
APPB_EPS = 1e-2


def appendix_b(I: int = 1_000_000, J: int = 2_000, nu: float = 10.0,
               seed: int = SEED_BASE + 6) -> Instance:
    """The synthetic construction of Appendix B ("Synthetic LP construction",
    "Source capacities and right-hand side"):

    * resource j gets a lognormal breadth; normalised, they give p_j;
    * K_j ~ Poisson(p_j I nu), truncated at I, distinct requests drawn
      uniformly for resource j (nu = nonzeros per request on average);
    * on edge (i, j): value min(v_j u_i eps_ij, c_max) with lognormal v_j,
      u_i, eps_ij; the LP cost is its negative (a maximisation of value);
    * a_ij = s_j * value with a lognormal per-resource s_j, so rows differ in
      support and in magnitude by orders;
    * b_j = rho_j (l_j + eps), rho_j ~ U[0.5, 1], from the greedy load l_j
      (each request's largest a_ij sent to its resource);
    * one simplex block per request (requests without edges have empty blocks).
    """
    rng = np.random.default_rng(seed)
    breadth = rng.lognormal(0.0, APPB_SIGMA_BREADTH, size=J)
    p = breadth / breadth.sum()
    K = np.minimum(rng.poisson(p * I * nu), I).astype(np.int64)
    # distinct requests per resource (resource-major), then source-major order
    req = np.empty(int(K.sum()), dtype=np.int64)
    off = np.concatenate([[0], np.cumsum(K)])
    for j in range(J):
        if K[j]:
            req[off[j]:off[j + 1]] = rng.choice(I, size=int(K[j]), replace=False)
    res = np.repeat(np.arange(J, dtype=np.int64), K)
    order = counting_order(req, I)       # by request, resources ascending within
    req, res = req[order], res[order]
    n = int(req.shape[0])
    v = rng.lognormal(0.0, APPB_SIGMA_V, size=J)
    u = rng.lognormal(0.0, APPB_SIGMA_U, size=I)
    eps = rng.lognormal(0.0, APPB_SIGMA_EPS, size=n)
    val = np.minimum(v[res] * u[req] * eps, APPB_CMAX)
    sj = rng.lognormal(0.0, APPB_SIGMA_S, size=J)
    a = sj[res] * val
    c = -val
    deg = np.bincount(req, minlength=I).astype(np.int64)
    block_off = np.zeros(I + 1, dtype=np.int64)
    np.cumsum(deg, out=block_off[1:])
    dst = res.astype(np.int32)
    b = greedy_capacity(dst, a, block_off, J, [seed, 2], eps=APPB_EPS)
    return Instance(J, n, dst, a, c, b, block_off, np.zeros(I, dtype=np.uint8), None,
                    "appendix_b", seed, {"I": I, "J": J, "nu": nu, "capacity": "greedy",
                                         "K": K, "s": sj})


@dataclass
class MultiInstance:
    """A matching LP with several constraint families (Definition 1) and
    optionally the global count row of Section 4 (sum_e x_e <= cap): column e
    (one per edge (i, j)) has an entry in row k J + j of every family k and,
    with the count row, in row m J.  A is held in CSC form."""

    m: int                       # rows: families * J (+ 1 with the count row)
    n: int                       # columns = edges
    colptr: np.ndarray           # int64 [n+1]
    rowidx: np.ndarray           # int32 [nnz]
    val: np.ndarray              # float64 [nnz]
    c: np.ndarray                # float64 [n]
    b: np.ndarray                # float64 [m]
    block_off: np.ndarray        # int64 [I+1]
    block_proj: np.ndarray       # uint8 [I]
    upper: Optional[np.ndarray]  # float64 [n] or None
    J: int = 0
    families: int = 1
    count_row: bool = False
    name: str = ""
    seed: int = 0

    @property
    def num_blocks(self) -> int:
        return int(self.block_off.shape[0] - 1)

    @property
    def nnz(self) -> int:
        return int(self.rowidx.shape[0])

    def dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        cols = np.repeat(np.arange(self.n), np.diff(self.colptr))
        A[self.rowidx, cols] = self.val
        return A

    def csr(self):
        """(rowptr int64 [m+1], colidx int32 [nnz], val float64 [nnz])."""
        cols = np.repeat(np.arange(self.n, dtype=np.int64), np.diff(self.colptr))
        order = np.argsort(self.rowidx, kind="stable")
        rowptr = np.zeros(self.m + 1, dtype=np.int64)
        np.cumsum(np.bincount(self.rowidx, minlength=self.m), out=rowptr[1:])
        return rowptr, cols[order].astype(np.int32), self.val[order]

    def rounded(self, storage: str) -> "MultiInstance":
        """The values a device store of type ``storage`` holds (see Instance.rounded)."""
        def rnd(v):
            if storage == "bf16":
                return _round_bf16(v)
            if storage == "f32":
                return v.astype(np.float32).astype(np.float64)
            return v.copy()
        up = None if self.upper is None else self.upper.astype(np.float32).astype(np.float64)
        return MultiInstance(self.m, self.n, self.colptr, self.rowidx, rnd(self.val), rnd(self.c),
                             self.b, self.block_off, self.block_proj, up, self.J, self.families,
                             self.count_row, self.name + f"[{storage}]", self.seed)


def multi_family(I: int = 100_000, J: int = 1_000, families: int = 2, count_row: bool = True,
                 seed: int = SEED_BASE + 7, box_frac: float = 0.0, capped_frac: float = 0.0,
                 count_frac: float = 0.5, zipf: bool = True, dmax: Optional[int] = None
                 ) -> MultiInstance:
    """Several matching families on one edge set (Definition 1): sources with
    1+Poisson(9) distinct destinations (Zipf(1.1) through a seeded permutation,
    or uniform; dmax > 0 draws degrees uniform in 1..dmax instead), costs
    c = -LogNormal(0,1), one coefficient per family a^k = LogNormal(0,0.5)
    drawn independently, greedy-load capacities per family (Appendix B rule
    applied to that family's coefficients), and with count_row the global
    count constraint sum_e x_e <= count_frac * (number of sources with edges)."""
    rng = np.random.default_rng(seed)
    deg = (1 + rng.poisson(9.0, size=I)) if dmax is None else rng.integers(1, dmax + 1, size=I)
    deg = np.minimum(deg.astype(np.int64), J)
    cdf = zipf_cdf(J, 1.1) if zipf else uniform_cdf(J)
    base = _finish("multi", seed, I, J, deg, rng, cdf, _neg_lognormal, _lognormal_a, 0.3,
                   box_frac=box_frac, capacity="greedy", seed_key=[seed, 1],
                   capped_frac=capped_frac)
    n = base.n
    coefs = [base.a] + [rng.lognormal(0.0, 0.5, size=n) for _ in range(families - 1)]
    b = [base.b] + [greedy_capacity(base.dst, coefs[k], base.block_off, J, [seed, 2, k])
                    for k in range(1, families)]
    per = families + (1 if count_row else 0)
    m = families * J + (1 if count_row else 0)
    rowidx = np.empty((n, per), dtype=np.int32)
    val = np.empty((n, per))
    for k in range(families):
        rowidx[:, k] = k * J + base.dst
        val[:, k] = coefs[k]
    bb = np.concatenate(b)
    if count_row:
        rowidx[:, families] = families * J
        val[:, families] = 1.0
        active = int(np.sum(np.diff(base.block_off) > 0))
        bb = np.concatenate([bb, [count_frac * active]])
    colptr = np.arange(0, n * per + 1, per, dtype=np.int64)
    return MultiInstance(m, n, colptr, rowidx.ravel(), val.ravel(), base.c, bb, base.block_off,
                         base.block_proj, base.upper, J, families, count_row,
                         f"multi{families}{'+count' if count_row else ''}", seed)


CONFIGS: dict[str, Callable[..., Instance]] = {
    "tiny": tiny,
    "large": large,
    "heavy": heavy,
    "appendix_b": appendix_b,
    "multi_family": multi_family,
}


def iter_batch(sizes) -> Iterator[Instance]:
    for k, I in enumerate(sizes):
        yield batch_member(int(I), k)
