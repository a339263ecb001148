#!/usr/bin/env python3
"""Throughput of the per-step TK-WFP update on one MI355X (source x time-steps per second).

A "step" is one pass of the whole hot path over one time sample: ingest of
sigma(t_n), packed type-1 NUFFT, near- and far-history recurrences of every
Fourier mode, type-2 NUFFT and the local singular quadrature at every target
(``wfp2d_step`` + ``wfp2d_evaluate``).  Inputs are seeded synthetic closed-form
signatures; the samples of the timed steps are generated into HBM before the
timed region starts.

Default workload: M = 10^6 random sources = targets in a 300 x 300-wavelength
square, eps = 1e-7, W = 16, p = 20, dt = 8/7150, timed over steps 5801..6000
(after the far history has become active at step LA = 4300).

Prints one JSON line (rank 0, one GPU).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, vendor figure
PEAK_FP64_TFLOPS = 78.6        # vector FP64
PEAK_FP32_TFLOPS = 157.3       # vector FP32


def kernels_digest() -> str:
    """sha256 prefix of the kernels source with comments and blank lines removed (so that
    only a change of code, not of its comments, invalidates the committed byte counters)."""
    import hashlib
    import re
    src = open(os.path.join(ROOT, "paper_2604_07170_amd", "csrc", "wfp2d_kernels.hip")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    code = [re.sub(r"//.*$", "", l).rstrip() for l in src.splitlines()]
    return hashlib.sha256("\n".join(l for l in code if l.strip()).encode()).hexdigest()[:16]


def traffic_summary_path(precision: str) -> str:
    return os.path.join(ROOT, "profiles", f"hbm_counters_cfg4_M1e6_{precision}.md")


def kernel_row_matches(name: str, base: str, targs) -> bool:
    """True when the rocprofv3 kernel name `name` (e.g. ``wfp2d::k_near<float>``) is kernel
    `base` whose leading template arguments are `targs` (strings; () = any)."""
    m = re.fullmatch(r"(?:wfp2d::)?(\w+)(?:<(.*)>)?", name.strip())
    if not m or m.group(1) != base:
        return False
    args = [a.strip() for a in (m.group(2) or "").split(",")] if m.group(2) else []
    return list(args[:len(targs)]) == [str(t) for t in targs]


def measured_traffic(base: str, targs=(), precision: str = "mixed"):
    """HBM bytes per launch (read + written) of kernel `base`<targs...> from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE summary of that precision, scaled by its copy-kernel
    calibration; None when the summary is missing, lists no such instantiation (exactly one
    must match), or was taken on other kernel code."""
    try:
        text = open(traffic_summary_path(precision)).read()
        digest = kernels_digest()
    except OSError:
        return None
    m = re.search(r"code sha256 prefix: ([0-9a-f]{16})", text)
    if not m or m.group(1) != digest:
        return None
    hits = []
    for line in text.splitlines():
        cells = [c.strip().strip("`") for c in line.strip().strip("|").split("|")]
        if len(cells) == 4 and kernel_row_matches(cells[0], base, targs):
            try:
                hits.append(int(round((float(cells[2]) + float(cells[3])) * 1e6)))
            except ValueError:
                return None
    return hits[0] if len(hits) == 1 else None


def copy_bandwidth(dev, gib: float = 1.0, reps: int = 5) -> float:
    """Bytes read + written per second by a plain device-to-device copy of `gib` GiB
    (torch's copy kernel), the practical HBM ceiling the stage fractions are read against."""
    import torch
    n = int(gib * 2**30) // 8
    a = torch.ones(n, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    bw = 2.0 * n * 8 * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return bw


def n_max(info: dict) -> int:
    """Sigma levels per pair in the paper's local sum (Sec. 6): W + 1 + ceil(p/2)."""
    return info["W"] + 1 + (info["p"] + 1) // 2


def local_impl_flops(info: dict) -> int:
    """FP64 flops of the local kernel as executed: per source, the polynomial profile on every
    regular sub-panel (each coefficient a dot product over the sigma levels); with stored pair
    lists, per list entry (pairs and run padding) one Horner evaluation (2 flops per term) plus
    the decoded coordinate (2 flops); with the per-step pair search, per pair one Clenshaw
    evaluation plus distance and sub-panel coordinate (~12 flops)."""
    prof = 2 * info["M"] * info["n_regular_subpanels"] * info["cheb_degree"] * info["n_levels"]
    if info.get("local_pair_words", 0) > 0:
        return prof + info["local_pair_words"] * (2 * info["cheb_degree"] + 2)
    return prof + info["n_local_pairs"] * (2 * info["cheb_degree"] + 12)


def stage_kernel(stage: str, info: dict):
    """(kernel base name, leading template arguments) of the kernel a stage launches."""
    r = "float" if info["precision"] == 1 else "double"
    table = {"ingest": ("k_ingest", ()), "spread": ("k_spread", (r,)), "fft_rows1": ("k_fft_t1", (r, 0)),
             "fft_cols1": ("k_fft_t1", (r, 1)), "split": ("k_split", (r,)), "near": ("k_near", (r,)),
             "far": ("k_far", (r,)), "fft_cols2": ("k_fft_t2", (r, 0)), "fft_rows2": ("k_fft_t2", (r, 1)),
             "interp": ("k_interp", (r,)), "combine": ("k_combine", ())}
    if stage == "local":
        path = info["local_path"]
        if path == 2:
            return "k_local_pc", (info["n_levels"], info["cheb_degree"])
        return ("k_local_fast", (info["n_levels"],)) if path == 1 else ("k_local", ())
    return table[stage]


def golden_samples(name: str):
    """{(target, step): u} of the stored oracle samples of a workload, or {} when none are
    committed (tests/golden/<workload>_oracle_samples.txt, written by the script beside it)."""
    path = os.path.join(ROOT, "tests", "golden", name.split("_")[0] + "_oracle_samples.txt")
    out = {}
    if not os.path.exists(path):
        return out
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        i, n, v = line.split()
        out[(int(i), int(n))] = float(v)
    return out


def init_phases(info: dict) -> dict:
    """The plan's set-up time by phase (wfp2d_info.init_ms), in ms."""
    names = ("modes_geometry", "nufft_point_data", "history_tables", "local_tables", "device_memory",
             "pair_lists", "total")
    return {n: round(v, 1) for n, v in zip(names, info.get("init_ms", [0.0] * 7))}


def timed_window(nt: int, LA: int, W: int, K: int):
    """First and last reported step of the timed window: the window ends at the workload's
    last step nt (extended past it when K steps would reach back before the far history
    starts), so every timed step has the far history active."""
    last = max(nt, LA + W + 1 + K)
    return last - K + 1, last


def stage_costs(info: dict) -> dict:
    """Algorithmic work of one launch of each stage: (bound, amount, unit).

    HBM-bound stages count the bytes a launch must move at least once
    (reads + writes of its inputs, state and outputs); the local part counts
    the method's FP64 flops (2 per source-target pair and sigma level).
    """
    c = 4 if info["precision"] == 1 else 8          # bytes per real in the grid/FFT/ring precision
    H, W = info["n_modes"], info["W"]
    Lp, N, R = info["band"], 2 * info["R"] + 1, info["R"]
    M, Nx, w = info["M"], info["Nx"], info["nufft_w"]
    nfar, nlev = info["n_far"], info["n_levels"]
    cost = {
        "ingest": ("hbm", M * (8 + 4 + 8)),
        "spread": ("hbm", M * (2 * 8 + 8 + 2 * w * c) + Lp * Lp * 2 * c),
        "fft_rows1": ("hbm", Lp * Lp * 2 * c + Lp * N * 2 * c),
        "fft_cols1": ("hbm", Lp * N * 2 * c + 2 * H * 2 * c),
        "split": ("hbm", 2 * H * 2 * c + 2 * H * 2 * c),
        # state D, C read+write (FP64 complex), 2W-1 ring taps, combined coefficient out
        "near": ("hbm", H * (4 * 16 + (2 * W - 1) * 2 * c + 2 * c)),
        "far": ("hbm", nfar * (640 * (16 + 16 + 8) + W * 2 * c + 2 * 2 * c)),
        "fft_cols2": ("hbm", H * 2 * c + (R + 1) * Lp * 2 * c),
        "fft_rows2": ("hbm", (R + 1) * Lp * 2 * c + Lp * Lp * c),
        "interp": ("hbm", Lp * Lp * c + Nx * (8 + 2 * w * c + 8)),
        # the method's FP64 work (Sec. 6, eq. local2 after eq. sigInterp): one multiply-add per
        # source-target pair and sigma level, n_max = W + 1 + ceil(p/2) levels per pair
        "local": ("alu", 2 * info["n_local_pairs"] * n_max(info)),
        "combine": ("hbm", Nx * (8 + 8 + 4 + 8)),
    }
    return cost


def adjoint_check(args, log):
    """Backward throughput and a finite-difference check of the strength gradient.

    The workload's sources, targets, time step and signature families, with the
    signature onsets moved into the first steps so that a short window carries
    signal: loss = 1/2 sum of u^2 over reported steps m0..nt."""
    import dataclasses
    import torch
    import paper_2604_07170_amd as pa
    from paper_2604_07170_amd.adjoint import StrengthRun, strength_field
    from wfp_workloads import config

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = config(args.config)
    w = dataclasses.replace(w, t0=np.random.default_rng(21).uniform(0.0, 0.02, size=w.M))
    nt, m0 = 40, 21
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=args.precision, interp_order=w.p)
    la = plan.info()["lookahead"]
    wu = dataclasses.replace(w, amp=np.ones(w.M))
    params = wu.torch_params(dev)
    S = torch.stack([wu.sigma_torch(l * w.dt, dev, params) for l in range(1, nt + la + 1)])
    run = StrengthRun(plan, lambda l: S[l - 1], nt=nt, m0=m0)
    A0 = torch.as_tensor(w.amp, dtype=torch.float64, device=dev)
    A = A0.clone().requires_grad_(True)
    t0 = time.time()
    u = strength_field(A, run)
    L = 0.5 * (u * u).sum()
    torch.cuda.synchronize()
    fwd_s = time.time() - t0
    # backward steps timed with events on the plans' stream (torch's current stream)
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    _ = run.adj                                        # build the transposed plan outside the timed region
    torch.cuda.synchronize()
    ev0.record(stream)
    L.backward()
    ev1.record(stream)
    torch.cuda.synchronize()
    bwd_ms = ev0.elapsed_time(ev1)
    n_adj = nt + 2 * la
    grad = A.grad.detach().cpu().numpy()
    log(f"[adjoint] forward {nt + la} steps in {fwd_s:.2f}s; backward {n_adj} steps {bwd_ms:.1f} ms")
    rng = np.random.default_rng(32)
    idx = np.sort(rng.choice(w.M, size=args.fd_strengths, replace=False))
    h = 1.0 if args.precision == "fp64" else float(np.sqrt(w.M))
    fd = np.zeros(len(idx))
    t0 = time.time()
    for k, j in enumerate(idx):
        e = torch.zeros_like(A0)
        e[j] = h
        up = run.forward_field(A0 + e)
        um = run.forward_field(A0 - e)
        fd[k] = float(0.5 * ((up * up).sum() - (um * um).sum())) / (2 * h)
        if k % 8 == 7:
            log(f"[adjoint] FD {k + 1}/{len(idx)} ({time.time() - t0:.1f}s)")
    err = float(np.linalg.norm(grad[idx] - fd) / np.linalg.norm(fd))
    out = {"metric": "adjoint source*steps/s and FD check of d(loss)/d(strengths)",
           "value": w.M * n_adj / (bwd_ms / 1e3), "unit": "source*steps/s", "n_gpus": 1,
           "backward_steps": n_adj, "backward_ms_per_step": bwd_ms / n_adj,
           "precision": args.precision, "workload": w.name + "_onsets_shifted",
           "loss": "1/2 sum u^2 over reported steps %d..%d" % (m0, nt),
           "fd": {"strengths": len(idx), "h": h, "rel_l2_adjoint_vs_fd": err,
                  "grad_norm_fd": float(np.linalg.norm(fd))}}
    print(json.dumps(out), flush=True)
    run.close()
    plan.close()


def batch_bench(args, log):
    """Batched workload: n independent scatterers of uneven size (star curves, 500 to
    20000 sources, 10 to 50 wavelengths, each with its own time step) advanced
    together by one graph launch per step, every plan's step and evaluation inside
    it, spreading tiles chosen by the autotuner.  Timed after every instance's far
    history has started.  The samples of the timed steps are synthesised into HBM
    before timing; each timed step copies its samples into the graph's fixed input
    buffer (one device copy) and launches the graph.  A seeded oracle sample of
    every eighth instance (by size) checks the fields at the last timed step."""
    import torch
    import paper_2604_07170_amd as pa
    from wfp_workloads import batch_instances
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    ws = batch_instances(args.batch)
    s = torch.cuda.Stream(dev)                 # graphs are captured on a created stream
    with torch.cuda.stream(s):
        t0 = time.time()
        plans = [pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=args.precision, interp_order=w.p, stream=s)
                 for w in ws]
        infos = [p.info() for p in plans]
        init_s = time.time() - t0
        Ms = np.array([w.M for w in ws], np.int64)
        Ns = np.array([w.Nx for w in ws], np.int64)
        mo = [0] + np.cumsum(Ms).tolist()          # offsets of each instance's samples and targets
        no = [0] + np.cumsum(Ns).tolist()
        sig_all = torch.zeros(mo[-1], dtype=torch.float64, device=dev)
        u_all = torch.zeros(no[-1], dtype=torch.float64, device=dev)
        sig = [sig_all[mo[i]:mo[i + 1]] for i in range(len(ws))]
        u = [u_all[no[i]:no[i + 1]] for i in range(len(ws))]
        params = [w.torch_params(dev) for w in ws]
        batch = pa.Batch(plans, sig, u, n_streams=4, stream=s, autotune=not args.no_autotune)
        log(f"[bench] batch of {len(ws)}: {mo[-1]} sources in all, plans ready in {init_s:.1f}s")

        nw = max(i["LA"] + i["W"] + i["lookahead"] for i in infos) + 1
        t0 = time.time()
        for n in range(1, nw + 1):
            for i, w in enumerate(ws):
                sig[i].copy_(w.sigma_torch(n * w.dt, dev, params[i]))
            batch.launch()
            if n % 200 == 0:
                s.synchronize()
                log(f"[bench] warm-up step {n}/{nw} ({time.time() - t0:.1f}s)")
        K = args.steps
        pre = torch.empty((K, mo[-1]), dtype=torch.float64, device=dev)
        for k in range(K):
            for i, w in enumerate(ws):
                pre[k, mo[i]:mo[i + 1]] = w.sigma_torch((nw + 1 + k) * w.dt, dev, params[i])
        s.synchronize()

        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(s)
        for k in range(K):
            sig_all.copy_(pre[k])
            batch.launch()
        ev1.record(s)
        s.synchronize()
    elapsed_ms = ev0.elapsed_time(ev1)
    value = mo[-1] * K / (elapsed_ms / 1e3)
    log(f"[bench] timed {K} batched steps: {elapsed_ms:.1f} ms, {elapsed_ms / K:.3f} ms/step")

    errs = {}
    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(78)
        for i in np.argsort(Ms)[::8].tolist():
            w, info = ws[i], plans[i].info()
            ti = rng.choice(w.Nx, size=2, replace=False)
            t_rep = info["step_reported"] * w.dt
            ref = oracle.u_workload(w, ti, [t_rep], self_mode=1, delta=info["delta"], b=info["b"])[:, 0]
            got = u[i].cpu().numpy()[ti]
            errs[w.name] = float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))
        log(f"[bench] oracle samples: worst rel err {max(errs.values()):.2e}")
    tiles = {}
    for t in batch.tuning:
        key = "x".join(str(v) for v in t["tile"])
        tiles[key] = tiles.get(key, 0) + 1
    out = {
        "metric": "batched source*timesteps/sec (independent scatterers of uneven size, one graph launch per step)",
        "value": value,
        "unit": "source*steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": int(nw),
        "ms_per_step": elapsed_ms / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic (seeded star curves and closed-form signatures)",
        "config": {"workload": f"batch{len(ws)}_star_E", "instances": len(ws), "M_total": mo[-1],
                   "M_range": [int(Ms.min()), int(Ms.max())], "precision": args.precision,
                   "timed_steps": f"{nw + 1}..{nw + K} (each instance's far history active)",
                   "spread_tiles": tiles},
        "plan_init_s": round(init_s, 2),
        "sample_rel_err_vs_oracle": errs or None,
    }
    print(json.dumps(out), flush=True)
    batch.close()
    for p in plans:
        p.close()


def run_form(args, w, precision: str, dev, log, golden: dict) -> dict:
    """Time K whole steps of one plan over the workload's fixed window and check them.

    The plan is pre-rolled (steps only: evaluation keeps no state) up to the window, then
    runs `warmup` untimed step+evaluate pairs, then K timed ones.  Reported steps are
    first..last (ingested steps first + lookahead .. last + lookahead)."""
    import torch
    import paper_2604_07170_amd as pa

    K, Wu = args.steps, args.warmup
    t0 = time.time()
    plan = pa.Wfp2d(w.src, w.tgt, w.dt, w.W, w.tol, precision=precision, interp_order=w.p,
                    lookahead=args.lookahead, max_steps=max(w.nt, 1) + K + 64)
    info = plan.info()
    init_s = time.time() - t0
    L = info["lookahead"]
    first, last = timed_window(w.nt, info["LA"], info["W"], K)
    n_first = first + L                                   # first timed ingested step
    Wu = min(Wu, n_first - 1)
    log(f"[bench] {w.name} {precision}: plan ready in {init_s:.1f}s  modes={info['n_modes']} nf={info['nf']} "
        f"band={info['band']} pairs={info['n_local_pairs']} pair_words={info['local_pair_words']} lookahead={L} HBM={info['bytes_device'] / 2**30:.1f}GiB; "
        f"timed steps report u(t_{first}..t_{last})")
    params = w.torch_params(dev)
    tuning = None
    if not args.no_autotune:
        from paper_2604_07170_amd.autotune import tune_spread
        tuning = tune_spread(plan)
        log(f"[bench] spreading tile {tuning['tile']} ({tuning['class']}): {tuning['ms']}")
    u_last = torch.empty(w.Nx, dtype=torch.float64, device=dev)

    # ---- pre-roll to the window, then the untimed warm-up steps ----
    t0 = time.time()
    for n in range(1, n_first):
        plan.step(w.sigma_torch(n * w.dt, dev, params))
        if n >= n_first - Wu:
            plan.evaluate(u_last)
        if n % 1000 == 0:
            torch.cuda.synchronize()
            log(f"[bench] pre-roll step {n}/{n_first - 1} ({time.time() - t0:.1f}s)")
    torch.cuda.synchronize()

    # ---- inputs of the timed steps, resident in HBM before timing; one output row per step ----
    sig = torch.empty((K, w.M), dtype=torch.float64, device=dev)
    for k in range(K):
        sig[k] = w.sigma_torch((n_first + k) * w.dt, dev, params)
    nonzero = int((sig.abs().amax(dim=1) > 0).sum())
    if nonzero < K:
        raise SystemExit(f"bench: {K - nonzero} of the {K} timed steps have sigma == 0 everywhere")
    u_out = torch.empty((K, w.Nx), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()

    # ---- timed region: K whole steps, HIP events on the plan's stream ----
    stream = torch.cuda.current_stream(dev)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    plan.set_timing(True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    ev0.record(stream)
    for k in range(K):
        plan.step(sig[k])
        plan.evaluate(u_out[k])
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    elapsed_ms = ev0.elapsed_time(ev1)
    stages = plan.get_timing()
    plan.set_timing(False)
    assert plan.info()["step_reported"] == last
    ms_per_step = elapsed_ms / K
    log(f"[bench] {precision}: timed {K} steps: {elapsed_ms:.1f} ms (wall {wall * 1e3:.1f} ms), "
        f"{ms_per_step:.3f} ms/step")

    # ---- per-stage roofline ----
    costs = stage_costs(info)
    per_stage = {}
    for s, (ms, n) in stages.items():
        if n == 0:
            continue
        bound, amt = costs[s]
        avg_ms = ms / n
        if bound == "hbm":
            ach = amt / (avg_ms * 1e-3) / 1e9
            per_stage[s] = dict(avg_ms=round(avg_ms, 5), bound="hbm", achieved_GBs=round(ach, 1),
                                frac=round(ach / PEAK_HBM_GBS, 4), bytes=int(amt))
        else:
            ach = amt / (avg_ms * 1e-3) / 1e12
            impl = local_impl_flops(info)
            per_stage[s] = dict(avg_ms=round(avg_ms, 5), bound="alu", achieved_TFLOPs=round(ach, 3),
                                frac=round(ach / PEAK_FP64_TFLOPS, 4), flops=int(amt), impl_flops=int(impl),
                                impl_TFLOPs=round(impl / (avg_ms * 1e-3) / 1e12, 3))
    hbm_bytes = sum(costs[s][1] for s in per_stage if costs[s][0] == "hbm")

    # ---- parity inside the window: stored oracle samples at the timed steps ----
    checks = sorted({n for (_, n) in golden if first <= n <= last})
    got, ref = [], []
    for n in checks:
        idx = sorted(i for (i, m) in golden if m == n)
        row = u_out[n - first].index_select(0, torch.as_tensor(idx, device=dev)).cpu().numpy()
        got.extend(row.tolist())
        ref.extend(golden[(i, n)] for i in idx)
    stored = None
    if ref:
        got, ref = np.array(got), np.array(ref)
        if not np.linalg.norm(ref) > 0:
            raise SystemExit("bench: the stored oracle samples of the window are all zero")
        stored = {"rel_l2": float(np.linalg.norm(got - ref) / np.linalg.norm(ref)), "samples": int(ref.size),
                  "steps": checks}
        log(f"[bench] {precision}: {ref.size} stored oracle samples at steps {checks}: rel L2 {stored['rel_l2']:.2e}")
    res = dict(plan=plan, info=info, init_s=init_s, first=first, last=last, K=K, warmup=Wu,
               elapsed_ms=elapsed_ms, ms_per_step=ms_per_step, per_stage=per_stage, hbm_bytes=hbm_bytes,
               stored=stored, u_last=u_out[K - 1].clone(), tuning=tuning)
    del u_out, sig
    return res


def cpu_oracle_sample(args, w, info, step: int, u_gpu, log):
    """Time the CPU oracle at `step` on a seeded sample of targets (all M sources each) and
    compare the GPU field there; the rate extrapolates the sample to all Nx targets."""
    import oracle
    rng = np.random.default_rng(77)
    ti = np.sort(rng.choice(w.Nx, size=args.cpu_sample_targets, replace=False))
    nth = oracle.threads()
    c0 = time.perf_counter()
    u_ref = oracle.u_workload(w, ti, [step * w.dt], self_mode=1, delta=info["delta"], b=info["b"])[:, 0]
    t_cpu = time.perf_counter() - c0
    if not np.linalg.norm(u_ref) > 0:
        raise SystemExit(f"bench: the oracle field at step {step} is zero at the sampled targets")
    rate = w.M * len(ti) / (t_cpu * w.Nx)
    cpu = {"value": rate, "unit": "source*steps/s", "cores": nth, "kind": "oracle",
           "sample": f"{len(ti)} seeded target(s) x 1 step (t_{step}, far history active) x all {w.M} "
                     f"sources, {t_cpu:.1f} s on {nth} threads; rate = M * samples / (t_sample * Nx)"}
    err = float(np.linalg.norm(u_gpu[ti] - u_ref) / np.linalg.norm(u_ref))
    log(f"[bench] oracle sample at step {step}: {t_cpu:.1f}s on {nth} threads; GPU vs oracle rel err {err:.2e}")
    return cpu, err, ti, u_ref


def roofline_of(res, precision):
    per_stage, info = res["per_stage"], res["info"]
    dom = max(per_stage, key=lambda s: per_stage[s]["avg_ms"])
    d = per_stage[dom]
    base, targs = stage_kernel(dom, info)
    kname = base + ("<" + ", ".join(str(t) for t in targs) + ">" if targs else "")
    if d["bound"] == "hbm":
        roof = {"bound": "hbm", "kernel": kname, "achieved": d["achieved_GBs"], "peak": PEAK_HBM_GBS,
                "unit": "GB/s", "frac": d["frac"]}
    else:
        roof = {"bound": "alu", "kernel": kname, "achieved": d["achieved_TFLOPs"], "peak": PEAK_FP64_TFLOPS,
                "unit": "TFLOP/s", "frac": d["frac"], "work": "2 FP64 flops per source-target pair and sigma "
                "level, n_max = W + 1 + ceil(p/2) levels (the method's count)",
                "impl_TFLOPs": d["impl_TFLOPs"]}
    roof["traffic"] = measured_traffic(base, targs, precision)
    roof["avg_ms"] = d["avg_ms"]
    return roof


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed step+evaluate iterations just before the timed window (the plan is "
                         "pre-rolled to the window regardless)")
    ap.add_argument("--config", type=int, default=4)
    ap.add_argument("--forms", default="mixed,fp64",
                    help="comma list of precisions to time; the first gives the headline value")
    ap.add_argument("--precision", choices=["mixed", "fp64"], default=None,
                    help="shorthand for --forms with one precision (also the adjoint / batch precision)")
    ap.add_argument("--lookahead", type=int, default=-1, help="reporting delay of the plan (-1 = its default)")
    ap.add_argument("--cpu-sample-targets", type=int, default=1,
                    help="targets of the timed CPU oracle sample (at the last timed step)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default spreading tile shape")
    ap.add_argument("--adjoint", action="store_true",
                    help="instead: time the adjoint (backward) steps and check d(loss)/d(strengths) by central "
                         "finite differences on 32 strengths, on the workload's geometry over a short window")
    ap.add_argument("--fd-strengths", type=int, default=32)
    ap.add_argument("--batch", type=int, default=0,
                    help="instead: time this many independent scatterers of uneven size (64 = the batched "
                         "workload) advanced by one graph launch per step")
    ap.add_argument("--quiet", action="store_true")
    ap.add_argument("--copy-probe-gib", type=float, default=0.0,
                    help="only run a device-to-device copy of this many GiB (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.precision is not None:
        args.forms = args.precision
    forms = [f.strip() for f in args.forms.split(",") if f.strip()]
    if not forms or any(f not in ("mixed", "fp64") for f in forms):
        raise SystemExit("--forms takes mixed and/or fp64")
    args.precision = forms[0]

    if args.copy_probe_gib > 0:
        import torch
        n = int(args.copy_probe_gib * 2**30) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_each_way": n * 8, "launches": 3}))
        return

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only: the sharding of the method over "
                                   "several GPUs is not built", "n_gpus": args.gpus}))
        sys.exit(2)
    if args.steps < 1 or args.warmup < 0:
        raise SystemExit("--steps must be >= 1 and --warmup >= 0")

    import torch
    from wfp_workloads import config

    log = (lambda *a: None) if args.quiet else (lambda *a: print(*a, file=sys.stderr, flush=True))
    if args.adjoint:
        adjoint_check(args, log)
        return
    if args.batch > 0:
        batch_bench(args, log)
        return
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = config(args.config)
    golden = golden_samples(w.name)
    copy_gbs = copy_bandwidth(dev)            # before the plans take their memory
    log(f"[bench] device copy: {copy_gbs:.0f} GB/s (read + write)")

    results = {}
    cpu, live_err = None, {}
    for f in forms:
        res = run_form(args, w, f, dev, log, golden)
        if f == forms[0] and not args.no_cpu_baseline:
            u_gpu = res["u_last"].cpu().numpy()
            cpu, live_err[f], live_idx, live_ref = cpu_oracle_sample(args, w, res["info"], res["last"], u_gpu, log)
            live_step = res["last"]
        elif cpu is not None and res["last"] == live_step:
            # every form reports the same steps: compare with the oracle values already computed
            u_gpu = res["u_last"].cpu().numpy()[live_idx]
            live_err[f] = float(np.linalg.norm(u_gpu - live_ref) / np.linalg.norm(live_ref))
        res["plan"].close()
        del res["plan"], res["u_last"]
        torch.cuda.empty_cache()
        results[f] = res

    def summary(f):
        r = results[f]
        return {"value": w.M * r["K"] / (r["elapsed_ms"] / 1e3), "ms_per_step": r["ms_per_step"],
                "roofline": roofline_of(r, f),
                "hbm_roofline_step_frac": round(r["hbm_bytes"] / (r["ms_per_step"] * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                "sample_rel_err_vs_oracle": r["stored"]["rel_l2"] if r["stored"] else live_err.get(f),
                "stored_oracle_check": r["stored"], "live_oracle_rel_err": live_err.get(f),
                "plan_init_s": round(r["init_s"], 2), "plan_init_ms": init_phases(r["info"]),
                "stages": r["per_stage"]}

    head_f = forms[0]
    h = results[head_f]
    hs = summary(head_f)
    info = h["info"]
    out = {
        "metric": "source\u00b7timesteps/sec at 1e-6 rel L2 error; % of HBM roofline (mixed vs FP64)",
        "value": hs["value"],
        "unit": "source*steps/s",
        "n_gpus": 1,
        "steps": h["K"],
        "warmup": h["warmup"],
        "ms_per_step": hs["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_f == "mixed" else "f64",
        "data": "synthetic (seeded closed-form signatures, random sources)",
        "config": {"workload": w.name, "M": w.M, "Nx": w.Nx, "dt": w.dt, "W": w.W, "p": w.p, "eps": w.tol,
                   "timed_steps": f"{h['first'] + info['lookahead']}..{h['last'] + info['lookahead']} ingested, "
                                  f"reporting u(t_{h['first']})..u(t_{h['last']}) (far history active from step "
                                  f"{info['LA'] + info['W']}); pre-rolled to the window, then {h['warmup']} "
                                  f"untimed warm-up steps",
                   "precision": head_f, "lookahead": info["lookahead"],
                   "n_modes": info["n_modes"], "nf": info["nf"], "local_pairs": info["n_local_pairs"],
                   "spread_tile": list(h["tuning"]["tile"]) if h["tuning"] else None,
                   "local_path": ["generic", "pair search", "pair lists"][info["local_path"]],
                   "cheb_terms": info["cheb_degree"]},
        "roofline": hs["roofline"],
        "hbm_roofline_step_frac": hs["hbm_roofline_step_frac"],
        "hbm_copy_GBs": round(copy_gbs, 1),
        "plan_init_s": hs["plan_init_s"],
        "plan_init_ms": hs["plan_init_ms"],
        "stages": hs["stages"],
        "cpu_baseline": cpu,
        "sample_rel_err_vs_oracle": hs["sample_rel_err_vs_oracle"],
        "stored_oracle_check": hs["stored_oracle_check"],
        "live_oracle_rel_err": hs["live_oracle_rel_err"],
    }
    for f in forms[1:]:
        s = summary(f)
        out[f] = {k: s[k] for k in ("value", "ms_per_step", "roofline", "hbm_roofline_step_frac",
                                    "sample_rel_err_vs_oracle", "stored_oracle_check", "live_oracle_rel_err",
                                    "plan_init_s", "plan_init_ms", "stages")}
        out[f"{head_f}_over_{f}"] = round(hs["value"] / s["value"], 3)
    errs = [e for e in [hs["sample_rel_err_vs_oracle"]] + [out[f]["sample_rel_err_vs_oracle"] for f in forms[1:]]
            if e is not None]
    print(json.dumps(out), flush=True)
    if errs and max(errs) > 1e-6:
        log(f"[bench] WARNING: oracle check above 1e-6 ({max(errs):.2e})")
        sys.exit(3)


if __name__ == "__main__":
    main()
