"""The multi-core CPU baseline of the benchmark agrees with the FP64 oracle
(dual objective and gradient, Section 3.1 / Eq.(2)) on seeded instances with
simplex and box blocks, at several gamma and thread counts."""
import numpy as np
import pytest

from paper_2603_04621_amd import instances as I
from oracle import oracle as O
from oracle import cpu_parallel as CP


@pytest.mark.parametrize("gamma", [1e-1, 1e-3])
@pytest.mark.parametrize("which", ["tiny", "heavy"])
def test_cpu_baseline_matches_oracle(which, gamma):
    inst = I.tiny() if which == "tiny" else I.heavy(I=3000, J=200, dmax=600)
    lam = np.random.default_rng(7).exponential(0.3, size=inst.m)
    ev = O.dual_eval(O.LP.from_instance(inst), lam, gamma)
    g, grad, nt = CP.dual_grad(CP.Arrays(inst), lam, gamma)
    assert nt >= 1
    scale = np.bincount(inst.dst, weights=np.abs(inst.a * ev.x), minlength=inst.m) + np.abs(inst.b)
    assert np.max(np.abs(grad - ev.grad) / np.maximum(scale, 1e-300)) < 1e-12
    assert abs(g - ev.g) <= 1e-12 * max(1.0, abs(ev.g))


def test_cpu_baseline_empty_blocks_and_zero_lambda():
    base = I.heavy(I=500, J=40, dmax=100)
    # an empty block after every third block
    nb = base.block_off.shape[0] - 1
    extra = np.arange(0, nb, 3)
    off = np.insert(base.block_off, extra + 1, base.block_off[extra + 1])
    proj = np.insert(base.block_proj, extra + 1, 0)
    inst = I.Instance(base.m, base.n, base.dst, base.a, base.c, base.b, off, proj, base.upper,
                      "heavy-with-empty-blocks", base.seed)
    lam = np.zeros(inst.m)
    ev = O.dual_eval(O.LP.from_instance(inst), lam, 1e-2)
    g, grad, _ = CP.dual_grad(CP.Arrays(inst), lam, 1e-2)
    assert np.allclose(grad, ev.grad, rtol=1e-12, atol=1e-12)
    assert abs(g - ev.g) <= 1e-12 * max(1.0, abs(ev.g))
