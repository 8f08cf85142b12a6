#!/usr/bin/env python3
"""Benchmark of the dual-ascent hot path on one MI355X.

Headline (`value`): accelerated dual-ascent iterations per second on the
100M-nnz matching LP (I = 10M sources, J = 10k destinations, degree
1+Poisson(9), Zipf(1.1) destinations, FP32-stored a and c, FP64 arithmetic
and scalars) with the paper's greedy-load capacities (Appendix B), under which
constraints bind and the prices move.  One step = one full iteration of the
hot path on the hipGraph path dl_solve uses: the fused gradient pass (gather,
projection, per-destination sums), the FP64 reduction and the ascent step,
with the gap test every 10 iterations.  Inputs are resident in HBM before the
timed region; exactly `steps` iterations are timed, after `warmup` untimed
ones (at least two graph lengths, so the timed solve replays the graph the
warm-up captured).

The same JSON line carries:
  roofline        the fused gradient kernel's algorithmic bytes per launch over
                  its mean launch time, from a separate pass with HIP events
                  around every launch on the solve's stream
  continuation    the 5-stage gamma continuation (1e-1 -> 1e-3) run to
                  rel_gap 1e-4: iterations, seconds, and the iteration rate of
                  each stage at the prices that stage sees
  batched         256 LPs (I log-uniform [1e3, 1e6]) solved to gap 1e-4 in one
                  batched solve against 256 one-at-a-time solves
  served          a Poisson stream at 200 req/s (I log-uniform [1e4, 5e6]) to
                  gap 1e-4 through the server against one-at-a-time solves,
                  p50/p99 latency
  heavy           the heavy-tailed mixed-projection workload (2M sources, 50k
                  destinations, ~60M nnz): kernel rate and roofline, FP32/BF16
  multi_family    two matching families plus the count row (2M sources):
                  kernel rate and roofline, continuation solve to gap 1e-4
  precision       errors against the FP64 oracle of every storage type on the
                  headline and the heavy-tailed workloads
  cpu_baseline    the oracle on one host core (bounded sample)
  cpu_parallel_baseline  a multi-core OpenMP implementation on all host cores

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-systems] [--no-heavy]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, 8 TB/s
METRIC = "dual-ascent iter/s + achieved HBM GB/s at 100M nnz; batched solves/s, p99 lat"
GAMMA = 1e-3                   # final gamma of every solve here
GEN_THREADS = 8


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("grad_impl.hpp", "lanes.hpp", "common.hpp", "kernels.hpp"):
        with open(os.path.join(ROOT, "paper_2603_04621_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload_key: str):
    """HBM bytes per gradient launch from the committed counter summary, if it
    was taken on the current kernel source and workload; else None."""
    path = os.path.join(ROOT, "profiles", "grad_kernel_large_counters.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_source_hash() or d.get("workload") != workload_key:
        return None
    return d.get("bytes_per_launch")


def sync():
    import torch
    torch.cuda.synchronize()


def continuation_settings(**kw):
    """gamma 1e-1 -> 1e-3 geometric in 5 stages (a stage ends after 2000
    iterations or at rel_gap 1e-3), the last stage to rel_gap 1e-4; the step
    cap is 1/L at each stage (natural preset)."""
    from paper_2603_04621_amd.api import SolveSettings
    d = dict(gamma0=1e-1, gamma_final=GAMMA, n_stages=5, stage_iters=2000, stage_tol=1e-3,
             tol_rel_gap=1e-4, max_iters=20000, check_every=10, preset="natural")
    d.update(kw)
    return SolveSettings(**d)


def fixed_settings(gamma, iters, check_every=10, **kw):
    """One stage at gamma, natural steps, the gap never stops it."""
    from paper_2603_04621_amd.api import SolveSettings
    return SolveSettings(gamma0=gamma, gamma_final=gamma, max_iters=iters,
                         check_every=check_every, tol_rel_gap=-1.0, preset="natural", **kw)


def graph_rate(p, gamma, steps, warmup, check_every=10, lam0=None):
    """(lam, outcome, seconds) of exactly `steps` graph-path iterations at
    gamma, after untimed warm-up solves: one of at least `warmup` iterations
    that captures the graph, then two of the timed length (the first solves
    after a capture run slower by about 0.3 ms, which at 20 steps would be
    8% of the timed region; a solve to a gap runs hundreds of iterations)."""
    p.solve(fixed_settings(gamma, max(warmup, 2 * check_every), check_every), lam0=lam0)
    for _ in range(2):
        p.solve(fixed_settings(gamma, steps, check_every), lam0=lam0)
    sync()
    t0 = time.perf_counter()
    lam, r = p.solve(fixed_settings(gamma, steps, check_every), lam0=lam0)
    sync()
    el = time.perf_counter() - t0
    assert r.iters == steps, r
    return lam, r, el


def kernel_times(p, gamma, iters, check_every=10, lam0=None):
    """Mean fused-gradient launch times (ordinary, gap-check) in ms from the
    eager pass with HIP events around every launch on the solve's stream."""
    _, r = p.solve(fixed_settings(gamma, iters, check_every, time_kernels=1), lam0=lam0)
    return r.grad_kernel_ms, r.check_kernel_ms


def stage_rate(p, gamma, lam0, iters):
    """Graph-path iterations/s at gamma from lam0: the difference of two
    timed solves of 10 and 10 + iters iterations (fixed costs cancel)."""
    p.solve(fixed_settings(gamma, 20), lam0=lam0)   # captures the graph
    ts = []
    for k in (10, 10 + iters):
        sync()
        t0 = time.perf_counter()
        p.solve(fixed_settings(gamma, k), lam0=lam0)
        sync()
        ts.append(time.perf_counter() - t0)
    return iters / max(ts[1] - ts[0], 1e-9)


# ----------------------------------------------------------------------------
# CPU baselines and error statements
# ----------------------------------------------------------------------------

def grad_errors(inst, ref_inst, ev, g, grad):
    """(relative error of g, max componentwise gradient error) of a GPU
    evaluation against an oracle evaluation `ev` on ref_inst's values."""
    scale = np.bincount(inst.dst, weights=np.abs(ref_inst.a * ev.x), minlength=inst.m) + \
        np.abs(inst.b)
    ge = np.abs(grad - ev.grad) / np.maximum(scale, 1e-300)
    return abs(g - ev.g) / max(1.0, abs(ev.g)), float(ge.max())


def precision_statement(inst, lam_np, gamma, gpu_evals, what):
    """Errors of each storage's GPU evaluation at lam against the oracle on
    the identically rounded data (kernel error) and on the FP64 data (storage
    error included)."""
    from oracle import oracle as O
    ev64 = O.dual_eval(O.LP.from_instance(inst), lam_np, gamma)
    out = {"lambda": what, "gamma": gamma,
           "tolerance": {"grad_componentwise": 1e-5, "g": 1e-6},
           "oracle_g_fp64_data": ev64.g}
    for st, (g, grad) in gpu_evals.items():
        d = {}
        if st != "f64":
            ref = inst.rounded(st)
            evr = O.dual_eval(O.LP.from_instance(ref), lam_np, gamma)
            d["g_rel_err_same_data"], d["grad_max_rel_err_same_data"] = \
                grad_errors(inst, ref, evr, g, grad)
        d["g_rel_err_fp64_data"], d["grad_max_rel_err_fp64_data"] = \
            grad_errors(inst, inst, ev64, g, grad)
        out[st] = d
    return out


def cpu_baseline(inst, lam_np, gamma, budget_s: float = 20.0):
    """The FP64 oracle's dual evaluation on one host core, on a bounded
    sample: whole-instance evaluations while the budget lasts (1 to 3)."""
    from oracle import oracle as O
    lp = O.LP.from_instance(inst.rounded("f32"))
    t0 = time.perf_counter()
    n = 0
    while True:
        O.dual_eval(lp, lam_np, gamma)
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 3 or el * (n + 1) / n > budget_s * 1.5:
            break
    per = el / n
    return {"value": 1.0 / per, "unit": "iter/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} full FP64 dual-gradient evaluation(s) of the same {inst.n}-nnz "
                      f"instance on one host core ({per:.2f} s each); the O(m) ascent step is "
                      f"not included"}


def cpu_parallel_baseline(inst, lam_np, gamma, evals: int = 3):
    """The same dual-gradient evaluation on all host cores (OpenMP C, FP64 on
    the FP32-rounded data; not the oracle): mean of `evals` whole-instance
    evaluations after one warm-up."""
    from oracle import cpu_parallel as CP
    arr = CP.Arrays(inst.rounded("f32"))
    CP.dual_grad(arr, lam_np, gamma)
    t0 = time.perf_counter()
    for _ in range(evals):
        _, _, nt = CP.dual_grad(arr, lam_np, gamma)
    per = (time.perf_counter() - t0) / evals
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": 1.0 / per, "unit": "iter/s", "cores": nt, "kind": "openmp",
            "nproc": os.cpu_count(), "cpu_model": model,
            "sample": f"{evals} full FP64 dual-gradient evaluations of the same {inst.n}-nnz "
                      f"instance on {nt} threads ({per * 1e3:.1f} ms each); the O(m) ascent "
                      f"step is not included"}


# ----------------------------------------------------------------------------
# instances
# ----------------------------------------------------------------------------

def make_instance(I, config, sources, dests, cache=None):
    """The headline (large) or heavy-tailed instance with greedy-load
    capacities (Appendix B), optionally cached as npy files."""
    fields = ("dst", "a", "c", "b", "block_off", "block_proj", "upper")
    tag = f"{config}_{sources}_{dests}_greedy"
    seed = I.SEED_BASE + (2 if config == "large" else 3)
    if cache:
        d = os.path.join(cache, tag)
        if all(os.path.exists(os.path.join(d, f + ".npy")) for f in fields[:-1]):
            arr = {f: np.load(os.path.join(d, f + ".npy")) for f in fields
                   if os.path.exists(os.path.join(d, f + ".npy"))}
            return I.Instance(dests, int(arr["dst"].shape[0]), arr["dst"], arr["a"], arr["c"],
                              arr["b"], arr["block_off"], arr["block_proj"], arr.get("upper"),
                              config + "-greedy", seed, {"capacity": "greedy"})
    if config == "large":
        inst = I.large(I=sources, J=dests, capacity="greedy")
    else:
        inst = I.heavy(I=sources, J=dests, capacity="greedy")
    if cache:
        d = os.path.join(cache, tag)
        os.makedirs(d, exist_ok=True)
        for f in fields:
            if getattr(inst, f) is not None:
                np.save(os.path.join(d, f + ".npy"), getattr(inst, f))
    return inst


def generate(fn, items):
    with ThreadPoolExecutor(GEN_THREADS) as ex:
        return list(ex.map(fn, items))


# ----------------------------------------------------------------------------
# legs
# ----------------------------------------------------------------------------

def headline(args, I, Problem):
    t0 = time.perf_counter()
    inst = make_instance(I, "large", args.sources, args.dests, args.cache)
    log(f"large instance with {inst.n} nnz ready in {time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    prob = Problem(inst, storage=args.storage, autotune=args.autotune)
    info = prob.info()
    create_s = time.perf_counter() - t0
    log(f"created in {create_s:.1f}s: {info}")

    lam, r, el = graph_rate(prob, GAMMA, args.steps, args.warmup)
    ips = args.steps / el
    kms, cms = kernel_times(prob, GAMMA, max(args.steps, 100))
    bytes_per = info["stream_bytes"]
    log(f"headline: {ips:.1f} iter/s, gradient {kms:.4f} ms, check {cms:.4f} ms")

    continuation = None
    lam_c = lam
    if not args.no_continuation:
        continuation, lam_c = continuation_leg(args, prob)
    out = {
        "value": ips, "ms_per_step": el * 1e3 / args.steps,
        "config": {"workload": (
            "matching LP: I=%d sources, J=%d destinations, degree 1+Poisson(9), Zipf(1.1) "
            "destinations, c=-LogNormal(0,1), a=LogNormal(0,0.5), simplex blocks, greedy-load "
            "capacities (Appendix B), gamma=1e-3, gap test every 10 iterations"
            % (args.sources, args.dests)),
            "nnz": inst.n, "storage": args.storage, "seed": inst.seed},
        "nnz_per_s": inst.n * ips,
        "achieved_hbm_gbs": bytes_per / (kms * 1e-3) / 1e9,
        "stream_gbs": bytes_per * ips / 1e9,
        "grad_kernel_ms": kms, "check_kernel_ms": cms,
        "roofline": {"bound": "hbm", "achieved": bytes_per / (kms * 1e-3) / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": bytes_per / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"large-greedy I={args.sources} J={args.dests} "
                                                 f"{args.storage}"),
                     "bytes_per_launch": bytes_per,
                     "kernel": "grad_kernel, ordinary iterations (fused gather + projection + "
                               "per-destination sums)"},
        "final_g": r.g, "final_rel_gap": r.rel_gap,
        "layout": {k: info[k] for k in ("lane_groups", "seg_groups", "wg_blocks", "chunks",
                                        "lds_rows", "lane_cap", "seg_rmax", "chunks_per_cu",
                                        "tuned")},
        "create_seconds": create_s,
    }
    if continuation is not None:
        out["continuation"] = continuation
    return headline_rest(args, Problem, inst, prob, out, lam_c, bytes_per)


def continuation_leg(args, prob):
    """The library's 5-stage continuation solve to gap 1e-4 (second of two
    runs: the first captures the graphs), and the iteration rate of each
    stage at the prices that stage starts from."""
    cont = continuation_settings()
    prob.solve(cont)
    sync()
    t0 = time.perf_counter()
    lam_c, rc = prob.solve(cont)
    sync()
    t_gap = time.perf_counter() - t0
    _, rtr = prob.solve(continuation_settings(trace=True))
    stage_of = rtr.trace[:, 4].astype(int) if rtr.trace is not None else np.zeros(0, int)
    gammas = [1e-1 * (GAMMA / 1e-1) ** (s / 4) for s in range(5)]
    stages = []
    lam_s = None
    for s, gs in enumerate(gammas):
        n_s = int(np.sum(stage_of == s))
        rate = stage_rate(prob, gs, lam_s, max(args.steps, 100))
        stages.append({"stage": s, "gamma": gs, "iterations": n_s, "iter_per_s": rate})
        # the prices at the end of this stage start the next one
        last = s == 4
        ss = fixed_settings(gs, 2000 if not last else 20000)
        ss.tol_rel_gap = 1e-3 if not last else 1e-4
        lam_s, _ = prob.solve(ss, lam0=lam_s)
    sync()
    continuation = {
        "schedule": "gamma 1e-1 -> 1e-3 geometric, 5 stages; a stage ends at rel_gap 1e-3 or "
                    "2000 iterations; the last runs to rel_gap 1e-4; step cap 1/L per stage",
        "converged": bool(rc.converged), "iterations": int(rc.iters), "seconds": t_gap,
        "final_rel_gap": rc.rel_gap, "final_g": rc.g, "final_gamma": rc.gamma,
        "stages": stages}
    log(f"continuation: {continuation}")
    return continuation, lam_c


def headline_rest(args, Problem, inst, prob, out, lam_eval, bytes_per):
    """Every storage type evaluated at the converged prices (for the error
    statement) with its own kernel rate, and the deterministic mode's cost."""
    gpu_evals = {}
    if not args.no_precision:
        gg, _, ee = prob.dual_grad(lam_eval, GAMMA, want_eval=True)
        gpu_evals[args.storage] = (ee["g"], gg.cpu().numpy())
    prob.close()
    if not args.no_autotune_report and not args.autotune and args.storage == "f32":
        out["autotune"] = tune_report(args, Problem, inst, None, out["grad_kernel_ms"],
                                      out["check_kernel_ms"], out["create_seconds"])
    storages = {}
    if not args.no_precision:
        for st in ("bf16", "f64"):
            if st == args.storage:
                continue
            with Problem(inst, storage=st) as ps:
                _, _, els = graph_rate(ps, GAMMA, args.steps, args.warmup)
                kms_s, _ = kernel_times(ps, GAMMA, max(args.steps, 100))
                gs, _, es = ps.dual_grad(lam_eval, GAMMA, want_eval=True)
                gpu_evals[st] = (es["g"], gs.cpu().numpy())
                sb = ps.info()["stream_bytes"]
                storages[st] = {"iter_per_s": args.steps / els, "grad_kernel_ms": kms_s,
                                "achieved_gbs": sb / (kms_s * 1e-3) / 1e9,
                                "bytes_per_launch": sb}
        # deterministic mode (integer per-destination sums): its cost
        with Problem(inst, storage=args.storage, deterministic=True) as pd:
            kms_d, cms_d = kernel_times(pd, GAMMA, max(args.steps, 100))
            storages[args.storage + "_deterministic"] = {
                "grad_kernel_ms": kms_d, "check_kernel_ms": cms_d,
                "achieved_gbs": bytes_per / (kms_d * 1e-3) / 1e9, "bytes_per_launch": bytes_per}
        out["storage_variants"] = storages
    return out, inst, lam_eval.cpu().numpy(), gpu_evals


def tune_report(args, Problem, inst, lam, ref_kms, ref_cms, ref_create_s):
    """The layout autotune on this workload: its pick, the kernel times of
    the tuned layout at the same prices and their gain over the default,
    and what the tuning adds to create."""
    from paper_2603_04621_amd.api import LAYOUT_KEYS
    t0 = time.perf_counter()
    with Problem(inst, storage="f32", autotune=True) as p:
        create_s = time.perf_counter() - t0
        info = p.info()
        kms, cms = kernel_times(p, GAMMA, max(args.steps, 100), lam0=lam)
    out = {"pick": {k: info[k] for k in LAYOUT_KEYS},
           "layout": {k: info[k] for k in ("lane_groups", "seg_groups", "wg_blocks")},
           "grad_kernel_ms": kms, "check_kernel_ms": cms,
           "default_grad_kernel_ms": ref_kms, "default_check_kernel_ms": ref_cms,
           "gain": ref_kms / kms, "check_gain": ref_cms / cms,
           "create_seconds": create_s, "default_create_seconds": ref_create_s}
    log(f"autotune: {out}")
    return out


def heavy_leg(args, I, Problem):
    """The heavy-tailed workload at full size: kernel rate and roofline for
    FP32 and BF16 storage, and the error statement of every storage type."""
    t0 = time.perf_counter()
    inst = make_instance(I, "heavy", args.heavy_sources, args.heavy_dests, args.cache)
    log(f"heavy instance with {inst.n} nnz ready in {time.perf_counter() - t0:.1f}s")
    nbox = int(np.sum(np.repeat(inst.block_proj == I.PROJ_BOX, np.diff(inst.block_off))))
    out = {"workload": (
        "matching LP: I=%d sources, J=%d destinations, degree Pareto(1.2, scale 6.5) clipped "
        "to [1, 4096], Zipf(1.1) destinations, 70%% simplex / 30%% box blocks (u=U(0.2,1)), "
        "greedy-load capacities, gamma=1e-3" % (args.heavy_sources, args.heavy_dests)),
        "nnz": inst.n, "nnz_box": nbox}
    lam = None
    gpu_evals = {}
    for st in ("f32", "bf16", "f64"):
        t0 = time.perf_counter()
        with Problem(inst, storage=st) as p:
            info = p.info()
            create_s = time.perf_counter() - t0
            if lam is None:
                # prices of a short solve at the final gamma
                lam, _ = p.solve(fixed_settings(GAMMA, 200))
            _, r, el = graph_rate(p, GAMMA, args.steps, args.warmup, lam0=lam)
            kms, cms = kernel_times(p, GAMMA, max(args.steps, 100), lam0=lam)
            g, _, e = p.dual_grad(lam, GAMMA, want_eval=True)
            gpu_evals[st] = (e["g"], g.cpu().numpy())
            sb = info["stream_bytes"]
            out[st] = {"iter_per_s": args.steps / el, "grad_kernel_ms": kms,
                       "check_kernel_ms": cms, "bytes_per_launch": sb,
                       "achieved_gbs": sb / (kms * 1e-3) / 1e9,
                       "frac": sb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                       "create_seconds": create_s,
                       "layout": {k: info[k] for k in ("lane_groups", "seg_groups", "wg_blocks",
                                                       "chunks", "lds_rows")}}
            log(f"heavy {st}: {out[st]}")
    if not args.no_autotune_report:
        out["autotune"] = tune_report(args, Problem, inst, lam, out["f32"]["grad_kernel_ms"],
                                      out["f32"]["check_kernel_ms"], out["f32"]["create_seconds"])
    if not args.no_precision:
        out["precision"] = precision_statement(inst, lam.cpu().numpy(), GAMMA, gpu_evals,
                                               "prices after 200 iterations at gamma = 1e-3")
    return out


def multi_leg(args, I, Problem):
    """Several matching families (Definition 1) with the global count row:
    kernel rate and roofline of the multi-entry gradient kernel, and a
    continuation solve to gap 1e-4 (natural steps from the power-iteration
    |A'|^2)."""
    t0 = time.perf_counter()
    inst = I.multi_family(I=args.multi_sources, J=args.multi_dests, families=2, count_row=True,
                          box_frac=0.2)
    log(f"multi-family instance: {inst.n} columns, {inst.nnz} entries in "
        f"{time.perf_counter() - t0:.1f}s")
    t0 = time.perf_counter()
    out = {"workload": (
        "matching LP with 2 families and the count row: I=%d sources, J=%d destinations per "
        "family (%d rows), degree 1+Poisson(9), Zipf(1.1), a^k = LogNormal(0,0.5) per family, "
        "greedy-load capacities per family, count cap 0.5 I, 80%% simplex / 20%% box blocks, "
        "FP32, gamma=1e-3" % (args.multi_sources, args.multi_dests, inst.m)),
        "columns": inst.n, "entries": inst.nnz}
    with Problem(inst, storage="f32") as p:
        info = p.info()
        out["create_seconds"] = time.perf_counter() - t0
        out["anorm2"] = info["anorm2"]
        cont = continuation_settings(gamma_final=GAMMA, max_iters=20000)
        sync()
        t1 = time.perf_counter()
        lam, r = p.solve(cont)
        sync()
        out["continuation"] = {"converged": bool(r.converged), "iterations": int(r.iters),
                               "seconds": time.perf_counter() - t1, "rel_gap": r.rel_gap}
        _, _, el = graph_rate(p, GAMMA, args.steps, args.warmup, lam0=lam)
        kms, cms = kernel_times(p, GAMMA, max(args.steps, 100), lam0=lam)
        sb = info["stream_bytes"]
        out.update({"iter_per_s": args.steps / el, "grad_kernel_ms": kms, "check_kernel_ms": cms,
                    "bytes_per_launch": sb, "achieved_gbs": sb / (kms * 1e-3) / 1e9,
                    "frac": sb / (kms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                    "layout": {k: info[k] for k in ("lane_groups", "seg_groups", "wg_blocks",
                                                    "chunks", "lds_rows", "col_entries")}})
    log(f"multi-family: {out}")
    return out


def fcfs_latencies(arrivals, service):
    """Latencies of one-at-a-time service in arrival order."""
    done_prev, out = 0.0, []
    for ta, sv in zip(arrivals, service):
        begin = max(ta, done_prev)
        done_prev = begin + sv
        out.append(done_prev - ta)
    return np.array(out), done_prev


def serve_stream_run(reqs, arrivals, st, slots):
    """Submits reqs[k] at arrivals[k] seconds to a fresh server; returns the
    wall time from the first arrival to the last completion, per-request
    latencies (completion - arrival) and the poll results."""
    import threading
    from paper_2603_04621_amd.api import Server
    srv = Server(hbm_budget_bytes=200e9, max_slots=slots)
    tickets = [None] * len(reqs)
    t_arr = [None] * len(reqs)
    start = time.perf_counter()

    def feeder():
        for k, ta in enumerate(arrivals):
            dt = start + ta - time.perf_counter()
            if dt > 0:
                time.sleep(dt)
            t_arr[k] = time.perf_counter()
            tickets[k] = srv.submit(reqs[k], st)

    th = threading.Thread(target=feeder)
    th.start()
    lat, res = [None] * len(reqs), [None] * len(reqs)
    left = set(range(len(reqs)))
    while left:
        for k in list(left):
            if tickets[k] is None:
                continue
            o = srv.poll(tickets[k])
            if o is not None:
                res[k] = o
                lat[k] = time.perf_counter() - t_arr[k]
                left.discard(k)
        time.sleep(0.0005)
    th.join()
    t_srv = time.perf_counter() - start
    srv.close()
    return t_srv, np.array(lat), res


def batched_leg(args, I, Problem, batch_solve):
    st = continuation_settings()
    sizes = I.batch_sizes(args.batch_count, 1e3, args.batch_hi)
    t0 = time.perf_counter()
    insts = generate(lambda kn: I.batch_member(int(kn[1]), kn[0], capacity="greedy"),
                     list(enumerate(sizes)))
    nnz = int(sum(x.n for x in insts))
    log(f"batch: {len(insts)} LPs, {nnz} nnz generated in {time.perf_counter() - t0:.1f}s")
    probs = [Problem(x) for x in insts]
    sync()
    t0 = time.perf_counter()
    seq = [p.solve(st)[1] for p in probs]
    sync()
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, bat = batch_solve(probs, st)
    sync()
    t_bat = time.perf_counter() - t0
    for p in probs:
        p.close()
    out = {
        "workload": f"{len(insts)} matching LPs, I log-uniform [1e3, {args.batch_hi:.0e}], "
                    f"J = I/200, degree 1+Poisson(9), Zipf(1.1), greedy-load capacities, "
                    f"gamma 1e-1 -> 1e-3 in 5 stages, to rel_gap 1e-4",
        "nnz_total": nnz,
        "solves_per_s": len(insts) / t_bat, "seconds": t_bat,
        "sequential_solves_per_s": len(insts) / t_seq, "sequential_seconds": t_seq,
        "speedup": t_seq / t_bat,
        "converged": int(sum(r.converged for r in bat)),
        "sequential_converged": int(sum(r.converged for r in seq)),
        "max_rel_gap": float(max(r.rel_gap for r in bat)),
        "sequential_max_rel_gap": float(max(r.rel_gap for r in seq)),
        "iters_max": int(max(r.iters for r in bat)),
    }
    log(f"batched: {out}")
    return out


def served_leg(args, I, Problem):
    st = continuation_settings()
    arr = I.serve_stream(args.serve_count, rate=args.serve_rate, lo=1e4, hi=args.serve_hi)
    t0 = time.perf_counter()
    reqs = generate(lambda kv: I.serve_member(kv[1][1], kv[0], capacity="greedy"),
                    list(enumerate(arr)))
    nnz = int(sum(x.n for x in reqs))
    log(f"serve: {len(reqs)} requests, {nnz} nnz generated in {time.perf_counter() - t0:.1f}s")
    t_srv, lat, res = serve_stream_run(reqs, [ta for ta, _ in arr], st, args.serve_slots)
    # one-at-a-time baseline: measured create + solve per request, first come
    # first served on the same arrival times
    svc = []
    for x in reqs:
        sync()
        t1 = time.perf_counter()
        with Problem(x) as p:
            p.solve(st)
        sync()
        svc.append(time.perf_counter() - t1)
    seq_lat, done_prev = fcfs_latencies([ta for ta, _ in arr], svc)
    out = {
        "workload": f"{len(reqs)} requests, Poisson arrivals at {args.serve_rate:g}/s, "
                    f"I log-uniform [1e4, {args.serve_hi:.0e}], J = I/500, degree 1+Poisson(9), "
                    f"70/30 simplex/box, greedy-load capacities, to rel_gap 1e-4; "
                    f"{args.serve_slots} slots, 200 GB budget; requests generated on the host "
                    f"before the stream starts",
        "nnz_total": nnz,
        "solves_per_s": len(reqs) / t_srv,
        "p50_latency_s": float(np.percentile(lat, 50)),
        "p99_latency_s": float(np.percentile(lat, 99)),
        "p50_admission_s": float(np.percentile([r[2][1] - r[2][0] for r in res], 50)),
        "p50_on_device_s": float(np.percentile([r[2][2] - r[2][1] for r in res], 50)),
        "sequential_solves_per_s": len(reqs) / done_prev,
        "sequential_p50_latency_s": float(np.percentile(seq_lat, 50)),
        "sequential_p99_latency_s": float(np.percentile(seq_lat, 99)),
        "converged": int(sum(r[0].converged for r in res)),
        "max_rel_gap": float(max(r[0].rel_gap for r in res)),
    }
    log(f"served: {out}")
    sweep = []
    for rate in [float(x) for x in args.serve_sweep.split(",") if x]:
        arr_r = [ta * args.serve_rate / rate for ta, _ in arr]
        t_r, lat_r, res_r = serve_stream_run(reqs, arr_r, st, args.serve_slots)
        sl, sd = fcfs_latencies(arr_r, svc)
        sweep.append({"rate": rate, "solves_per_s": len(reqs) / t_r,
                      "p50_latency_s": float(np.percentile(lat_r, 50)),
                      "p99_latency_s": float(np.percentile(lat_r, 99)),
                      "sequential_solves_per_s": len(reqs) / sd,
                      "sequential_p50_latency_s": float(np.percentile(sl, 50)),
                      "sequential_p99_latency_s": float(np.percentile(sl, 99)),
                      "converged": int(sum(r[0].converged for r in res_r))})
        log(f"served at {rate:g}/s: {sweep[-1]}")
    if sweep:
        out["rate_sweep"] = sweep
    return out


def ablations(args, I, Problem):
    """Section 7's two ablations on the paper's own construction (Appendix B,
    rows whose norms differ by orders): diagonal (Jacobi) preconditioning and
    gamma continuation, with the paper's hyper-parameters (max step 1e-3,
    initial step 1e-5, gamma = 0.01, a fixed iteration count).  Reported the
    way the paper plots them: log10 |L - L^| / |L^| along the iterations, L
    the dual objective at gamma = 0.01 and L^ its converged value (a long
    continuation solve of the same problem to rel_gap 1e-7), and the
    iterations to 1e-2, 1e-3 and 1e-4.  The continuation run decays gamma from
    0.16 to 0.01, halved every 25 iterations (only its iterations at 0.01
    count).  Also: iterations to rel_gap 1e-4 with the safe 1/L step cap,
    with and without preconditioning."""
    from paper_2603_04621_amd.api import SolveSettings
    t0 = time.perf_counter()
    inst = I.appendix_b(I=args.ablation_sources, J=args.ablation_dests)
    log(f"appendix-B instance: {inst.n} nnz in {time.perf_counter() - t0:.1f}s")
    rn = np.sqrt(np.bincount(inst.dst, weights=inst.a ** 2, minlength=inst.m))
    N = args.ablation_iters
    g_final = 0.01

    def run(rnorm, settings):
        with Problem(inst, storage="f32", row_normalize=rnorm) as p:
            sync()
            t1 = time.perf_counter()
            _, r = p.solve(settings)
            sync()
            return r, time.perf_counter() - t1

    ref, _ = run(True, SolveSettings(gamma0=0.16, gamma_final=g_final, n_stages=5, stage_iters=0,
                                     stage_tol=1e-4, tol_rel_gap=1e-7, max_iters=200000,
                                     check_every=10, preset="natural"))
    Lh = ref.g
    log(f"reference: {ref}")
    marks = [k for k in (1, 10, 25, 50, 100, 150, 200, 300, 500, 1000, 2000, 5000, 10000) if k <= N]
    cases = [
        ("jacobi, paper steps, fixed gamma", True,
         dict(gamma0=g_final, gamma_final=g_final, n_stages=1, max_step=1e-3, init_step=1e-5)),
        ("no preconditioning, paper steps, fixed gamma", False,
         dict(gamma0=g_final, gamma_final=g_final, n_stages=1, max_step=1e-3, init_step=1e-5)),
        ("jacobi, paper steps, gamma 0.16 -> 0.01 halved every 25 iterations", True,
         dict(gamma0=0.16, gamma_final=g_final, n_stages=5, stage_iters=25,
              max_step=1e-3 * 16, init_step=1e-5 * 16)),
        ("no preconditioning, paper steps, gamma 0.16 -> 0.01 halved every 25 iterations", False,
         dict(gamma0=0.16, gamma_final=g_final, n_stages=5, stage_iters=25,
              max_step=1e-3 * 16, init_step=1e-5 * 16)),
    ]
    from paper_2603_04621_amd._lib import DualipError
    curves = []
    for name, rnorm, kw in cases:
        st = SolveSettings(tol_rel_gap=-1.0, max_iters=N, check_every=10, trace=True, **kw)
        try:
            r, el = run(rnorm, st)
        except DualipError as e:      # a diverging run (non-finite objective)
            curves.append({"case": name, "failed": str(e)})
            log(f"ablation {curves[-1]}")
            continue
        tr = r.trace
        final = np.abs(tr[:, 3] - g_final) <= 1e-12 * g_final
        sub = np.abs(tr[:, 0] - Lh) / abs(Lh)
        sub[~final] = np.nan
        first = {}
        for lvl in (1e-2, 1e-3, 1e-4):
            hit = np.nonzero(sub <= lvl)[0]
            first[f"{lvl:g}"] = int(hit[0]) + 1 if hit.size else None
        curves.append({"case": name, "seconds": el,
                       "log10_rel_subopt": {str(k): (None if np.isnan(sub[k - 1]) else
                                                     float(np.log10(max(sub[k - 1], 1e-16))))
                                            for k in marks},
                       "iterations_to_rel_subopt": first})
        log(f"ablation {curves[-1]}")
    to_gap = []
    for rnorm in (True, False):
        st = SolveSettings(gamma0=0.16, gamma_final=g_final, n_stages=5, stage_iters=2000,
                           stage_tol=1e-3, tol_rel_gap=1e-4, max_iters=args.ablation_gap_iters,
                           check_every=10, preset="natural")
        try:
            r, el = run(rnorm, st)
        except DualipError as e:
            to_gap.append({"preconditioning": "jacobi" if rnorm else "none", "failed": str(e)})
            continue
        to_gap.append({"preconditioning": "jacobi" if rnorm else "none",
                       "converged": bool(r.converged), "iterations": int(r.iters),
                       "seconds": el, "rel_gap": r.rel_gap})
        log(f"to gap {to_gap[-1]}")
    return {"workload": "Appendix B construction: I=%d requests, J=%d resources, nu=10 "
                        "(%d nnz), row norms %.3g..%.3g, greedy-load capacities, FP32"
                        % (args.ablation_sources, args.ablation_dests, inst.n,
                           float(rn[rn > 0].min()), float(rn.max())),
            "reference_L": Lh, "reference_rel_gap": ref.rel_gap, "curves": curves,
            "to_gap_1e-4_natural_steps": to_gap}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--sources", type=int, default=10_000_000)
    ap.add_argument("--dests", type=int, default=10_000)
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "f64"])
    ap.add_argument("--heavy-sources", type=int, default=2_000_000)
    ap.add_argument("--heavy-dests", type=int, default=50_000)
    ap.add_argument("--no-heavy", action="store_true", help="skip the heavy-tailed leg")
    ap.add_argument("--no-multi", action="store_true", help="skip the multi-family leg")
    ap.add_argument("--no-continuation", action="store_true",
                    help="skip the continuation solve and the per-stage rates")
    ap.add_argument("--multi-sources", type=int, default=2_000_000)
    ap.add_argument("--multi-dests", type=int, default=10_000)
    ap.add_argument("--no-systems", action="store_true",
                    help="skip the batched and served legs")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the BF16 / FP64 storage runs and the error statements")
    ap.add_argument("--batch-count", type=int, default=256)
    ap.add_argument("--batch-hi", type=float, default=1e6)
    ap.add_argument("--serve-count", type=int, default=200)
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-hi", type=float, default=5e6)
    ap.add_argument("--serve-slots", type=int, default=32)
    ap.add_argument("--serve-sweep", default="",
                    help="lower arrival rates (req/s) re-run with the same requests")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--ablations", action="store_true",
                    help="also run the preconditioning / continuation ablations")
    ap.add_argument("--ablation-sources", type=int, default=25_000_000)
    ap.add_argument("--ablation-dests", type=int, default=10_000)
    ap.add_argument("--ablation-iters", type=int, default=2000)
    ap.add_argument("--ablation-gap-iters", type=int, default=20000)
    ap.add_argument("--no-autotune-report", action="store_true",
                    help="skip the autotuned layouts of the headline and heavy-tailed workloads")
    ap.add_argument("--autotune", action="store_true",
                    help="pick the work layout by timing candidates on a sample at create")
    ap.add_argument("--cache", default=None,
                    help="directory to save/load the generated instances (npy files)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run plain 1 GiB device copies (counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        torch.cuda.set_device(0)
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")   # 1 GiB
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": a.numel() * 4,
                          "launches": 5}))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(--gpus must be 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2603_04621_amd import instances as I
    from paper_2603_04621_amd.api import Problem, batch_solve

    torch.cuda.set_device(0)
    head, inst, lam_np, gpu_evals = headline(args, I, Problem)
    out = {"metric": METRIC, "value": head.pop("value"), "unit": "iter/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": head.pop("ms_per_step"), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic"}
    out.update(head)
    if not args.no_systems:
        out["batched"] = batched_leg(args, I, Problem, batch_solve)
        out["batched_solves_per_s"] = out["batched"]["solves_per_s"]
        out["served"] = served_leg(args, I, Problem)
        out["served_solves_per_s"] = out["served"]["solves_per_s"]
        out["served_p99_latency_s"] = out["served"]["p99_latency_s"]
    if not args.no_heavy:
        out["heavy"] = heavy_leg(args, I, Problem)
    if not args.no_multi:
        out["multi_family"] = multi_leg(args, I, Problem)
    if args.ablations:
        out["ablations"] = ablations(args, I, Problem)
    if not args.no_precision and gpu_evals:
        log("error statement against the oracle")
        out["precision"] = precision_statement(inst, lam_np, GAMMA, gpu_evals,
                                               "final prices of the continuation solve")
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(inst, lam_np, GAMMA, args.cpu_budget)
        log("timing the multi-core CPU baseline")
        out["cpu_parallel_baseline"] = cpu_parallel_baseline(inst, lam_np, GAMMA)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
