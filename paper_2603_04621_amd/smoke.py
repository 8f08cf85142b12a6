"""One small dual-gradient evaluation and a short solve on cuda:0, checked
against the CPU oracle (the checker is test infrastructure; the computation
runs in the HIP library)."""
import numpy as np


def run() -> None:
    import torch

    from oracle import oracle as O

    from . import instances as I
    from .api import Problem, SolveSettings

    assert torch.cuda.is_available(), "smoke needs a ROCm device"
    torch.cuda.set_device(0)
    inst = I.random_small(7, I=2000, J=80, dmax=40, box_frac=0.3)
    lam = np.random.default_rng(0).exponential(1.0, size=inst.m)
    ref = O.dual_eval(inst.rounded("f32"), lam, 1e-2)
    with Problem(inst, storage="f32") as p:
        grad, _, ev = p.dual_grad(torch.from_numpy(lam), 1e-2, want_eval=True)
        scale = np.bincount(inst.dst, weights=np.abs(inst.rounded("f32").a * ref.x),
                            minlength=inst.m) + np.abs(inst.b)
        err = np.max(np.abs(grad.cpu().numpy() - ref.grad) / np.maximum(scale, 1e-300))
        assert err <= 1e-5, f"gradient error {err}"
        assert abs(ev["g"] - ref.g) <= 1e-6 * max(1.0, abs(ref.g)), (ev["g"], ref.g)
        s = SolveSettings(gamma0=1e-2, gamma_final=1e-2, max_iters=50, check_every=10,
                          tol_rel_gap=0.0, max_step=1e-2, init_step=1e-4)
        lam_out, r = p.solve(s)
        ro = O.solve(inst.rounded("f32"), O.SolveOpts(gamma0=1e-2, gamma_final=1e-2,
                                                      max_iters=50, check_every=10,
                                                      tol_rel_gap=0.0, max_step=1e-2,
                                                      init_step=1e-4))
        assert r.iters == 50
        assert abs(r.g - ro.g) <= 1e-6 * max(1.0, abs(ro.g)), (r.g, ro.g)
    print(f"smoke ok: grad err {err:.2e}, g {ev['g']:.6f}, solve g {r.g:.6f} (oracle {ro.g:.6f})")
