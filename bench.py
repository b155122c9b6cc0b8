#!/usr/bin/env python3
"""Benchmark: B3/S23 life step on an r = 16 embedded Sierpinski gasket
(n = 65,536, 3^16 = 43,046,721 cells, uint8 state), lambda(omega) block map
against the bounding-box map, on one MI355X.

    python bench.py [--gpus 1] [--steps 100] [--warmup 10]

Prints ONE JSON line.  `value` is gasket cells updated per second by the
lambda-mapped step at its best block side rho; the bounding-box map at every
rho, the paper's write pass (lambda vs bounding box) and the roofline of the
dominant kernel are reported beside it.  Inputs are seeded synthetic states
(Bernoulli(0.5) on the gasket cells, seed 1706) resident in HBM before the
timed region; the oracle's CPU time on a bounded sample is reported as
`cpu_baseline`.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

PEAK_HBM_GBS = 8000.0          # MI355X HBM3E, published
# 32-bit VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
PEAK_ALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# algorithmic work of a life generation, bit-sliced (one 32-bit lane op acts on
# 32 cells): a row's horizontal 3-cell sums (two funnel shifts, a three-input
# XOR, a three-input majority), the 3 x 3 sum and the rule (eight three-input
# functions), the gasket mask (one AND): 13 lane ops per 32 cells
LIFE_OPS_PER_CELL = 13 / 32
CA_BYTES_PER_CELL = 2          # read own state once, write it once
# FP32 work of a diffusion step per gasket cell: (W + E) + (N + S) (three
# adds), - deg * u + that (one fma), u + alpha * t (one fma): 7 flops
DIFF_FLOPS_PER_CELL = 7
PEAK_FP32_TFLOPS = 157.3        # MI355X vector FP32, published
WRITE_BYTES_PER_CELL = 1       # store the constant once
RHOS = (4, 8, 16, 32, 64, 128, 256)
TB_RHOS = (32, 64, 128, 256)
TB_SMALL_RHOS = (16,)           # byte-plane tile pass, up to 16 generations per pass
COMPACT_RHOS = (64, 128, 256)   # tile sides of block-compacted storage
R = 16
SEED = 1706
PAPER_BEST_VS_BEST = "about 10x (best lambda, rho=16, vs best bounding box, rho=32; Titan-X Pascal GP102; write pass at n=2^16)"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_region(torch, fn, steps, warmup):
    """Average ms per call of `fn` over `steps` calls, HIP events on the stream
    the kernels are launched on (torch's current stream)."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def time_samples(torch, fn, samples, warmup, calls=1):
    """`samples` timings (ms per call) of `calls` back-to-back calls of `fn`
    each, after `warmup` untimed calls; HIP events on torch's current stream
    (the stream the library launches on), the device synchronised before and
    after every sample."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(samples):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(calls):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out.append(e0.elapsed_time(e1) / calls)
    return out


def stats(ms):
    """Median, standard error of the mean, extremes and count of timings."""
    a = np.asarray(ms, dtype=np.float64)
    se = float(a.std(ddof=1) / np.sqrt(len(a))) if len(a) > 1 else 0.0
    return {"median_ms": float(np.median(a)), "mean_ms": float(a.mean()), "se_ms": se,
            "min_ms": float(a.min()), "max_ms": float(a.max()), "n": int(len(a))}


def ms_stats(ms):
    """stats() in milliseconds, rounded for the report."""
    st = stats(ms)
    return {"median_ms": round(st["median_ms"], 4), "se_ms": round(st["se_ms"], 4),
            "min_ms": round(st["min_ms"], 4), "max_ms": round(st["max_ms"], 4), "n": st["n"]}


def us_stats(ms, per=1):
    """stats() in microseconds per `per` units, rounded for the report."""
    st = stats(np.asarray(ms) / per)
    return {"median_us": round(st["median_ms"] * 1e3, 3), "se_us": round(st["se_ms"] * 1e3, 3),
            "min_us": round(st["min_ms"] * 1e3, 3), "max_us": round(st["max_ms"] * 1e3, 3),
            "n": st["n"]}


def kernel_profile(tag):
    """The committed rocprofv3 figures of one kernel shape (HBM bytes per
    launch from FETCH_SIZE / WRITE_SIZE, VALU counters), if they were taken
    on the current sources of that kernel."""
    path = os.path.join(HERE, "profiles", f"{tag}.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path))
    except ValueError:
        return None
    from paper_1706_04552_amd.build import source_digest
    if rec.get("source_digest") != source_digest(rec.get("sources")):
        return None
    return rec


def _oracle_rate(step, a0_host, cells, min_seconds, max_gens):
    """Generations of `step` from a0_host until about `min_seconds` have
    passed: (cells per second, generations, seconds)."""
    cur = a0_host
    gens = 0
    t0 = time.perf_counter()
    while True:
        cur = step(cur)
        gens += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or gens >= max_gens:
            break
    return gens * cells / dt, gens, dt


def cpu_baseline(r, a0_host, seconds=8.0):
    """The oracle, as it stands, on bounded samples of the same r = 16 life
    run: its gasket-only step (rows y, columns x over the submasks of ~y) on
    all host cores and on one core, and its whole-array step on all cores."""
    import oracle as O
    threads = O.threads()
    cells = 3 ** r
    log(f"cpu baseline: gasket-only oracle step, {threads} threads")
    v_all, g_all, dt_all = _oracle_rate(lambda a: O.life_step_sparse(r, a), a0_host, cells,
                                        seconds, 100)
    log(f"cpu baseline: gasket-only oracle step, 1 thread")
    O.set_threads(1)
    try:
        v_one, g_one, dt_one = _oracle_rate(lambda a: O.life_step_sparse(r, a), a0_host, cells,
                                            seconds, 100)
    finally:
        O.set_threads(threads)
    log(f"cpu baseline: whole-array oracle step, {threads} threads")
    v_dense, g_dense, dt_dense = _oracle_rate(lambda a: O.life_step(r, a), a0_host, cells,
                                              seconds / 2, 100)
    return {"value": v_all, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{g_all} generations of the r={r} gasket ({cells} cells each) from the "
                      f"benchmark's initial state, the oracle's gasket-only C step on {threads} "
                      f"threads, {dt_all:.1f} s wall",
            "single_core": {"value": v_one, "unit": "cells/s", "cores": 1,
                            "sample": f"{g_one} generations, gasket-only step, 1 thread, "
                                      f"{dt_one:.1f} s wall"},
            "whole_array_all_cores": {"value": v_dense, "unit": "cells/s", "cores": threads,
                                      "sample": f"{g_dense} generations, whole-array step "
                                                f"(4^{r} cells visited), {dt_dense:.1f} s wall"}}


def diffusion_error_vs_fp64(torch, sg, inputs, shapes, steps=500):
    """The diffusion workload's accuracy report (r = 14, 500 steps): the
    oracle's FP64 run (gasket-graph step, timed as the CPU baseline of this
    workload) against the FP32 device runs of `shapes` [(map, rho,
    steps_per_pass)], as max-abs error, its scale max|u| and relative L2
    error over every gasket cell."""
    import oracle as O
    r = 14
    u0 = inputs.uniform_field(r, SEED)
    t0 = time.perf_counter()
    pos, ref = O.diffuse_steps_graph(r, u0, steps, 0.2)
    dt = time.perf_counter() - t0
    out = {"r": r, "steps": steps,
           "cpu_oracle_fp64": {"value": 3 ** r * steps / dt, "unit": "cell-steps/s",
                               "cores": O.threads(), "seconds": round(dt, 2)},
           "runs": {}}
    U = torch.from_numpy(u0).cuda()
    dpos = torch.from_numpy(pos).cuda()
    dref = torch.from_numpy(ref).cuda()
    scale = float(dref.abs().max())
    for map_kind, rho, T in shapes:
        o, w = torch.zeros_like(U), torch.zeros_like(U)
        sg.sg_diffuse_steps(map_kind, r, rho, steps, U, o, w, 0.2, steps_per_pass=T)
        torch.cuda.synchronize()
        d = o.reshape(-1)[dpos].double() - dref
        max_abs = float(d.abs().max())
        rel_l2 = float(d.norm() / dref.norm())
        out["runs"][f"{map_kind}_rho{rho}_T{T}"] = {
            "max_abs": max_abs, "scale": scale, "rel_l2": rel_l2,
            "within_1e-5": bool(max_abs <= 1e-5 * scale and rel_l2 <= 1e-5)}
        log(f"diffuse r=14 {steps} steps {map_kind} rho={rho} {T}/pass: max_abs {max_abs:.2e} "
            f"(scale {scale:.3f}) rel_l2 {rel_l2:.2e}")
        del o, w
    del U, dpos, dref
    torch.cuda.empty_cache()
    return out


def graph_time(torch, launch, steps, reps=10):
    """ms per step of `steps` launches captured in one hipGraph (the graph's
    replay time; no host launch overhead), for each of `reps` replays."""
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture
        for _ in range(2):
            launch()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        for _ in range(steps):
            launch()
    g.replay()
    torch.cuda.synchronize()
    out = time_samples(torch, g.replay, reps, 0)
    del g
    return [ms / steps for ms in out]


def bench_sweep(torch, sg, inputs, rs, rhos, steps):
    """Life steps (one launch per generation) at smaller sizes: lambda against
    the bounding box at every rho, both timed as hipGraph replays."""
    out = {}
    for r in rs:
        a0 = inputs.bernoulli_state(r, 0.5, SEED)
        A = torch.from_numpy(a0).cuda()
        Bf = torch.zeros_like(A)
        row = {}
        for rho in rhos:
            t = {}
            for map_kind in ("lambda", "bbox"):
                bufs = [A.clone(), Bf.clone()]
                st = {"i": 0}

                def launch():
                    i = st["i"]
                    sg.sg_ca_step(map_kind, r, rho, bufs[i], bufs[1 - i])
                    st["i"] = 1 - i
                t[map_kind] = graph_time(torch, launch, steps)
            lam, box = stats(t["lambda"]), stats(t["bbox"])
            row[str(rho)] = {"lambda_us": us_stats(t["lambda"]), "bbox_us": us_stats(t["bbox"]),
                             "speedup": round(box["median_ms"] / lam["median_ms"], 3)}
            log(f"sweep r={r} rho={rho:3d}: lambda {lam['median_ms'] * 1e3:8.2f} us  bbox "
                f"{box['median_ms'] * 1e3:8.2f} us  x{box['median_ms'] / lam['median_ms']:.2f}")
        out[str(r)] = row
        del A, Bf
    return out


DIFF_TB_SHAPES = [(rho, T) for rho in (16, 32, 64) for T in (4, 8, 12, 16)]


def _shape(text):
    rho, T = text.lower().split("x")
    return int(rho), int(T)


def bench_diffusion(torch, sg, inputs, rhos, steps, warmup, reps, shapes=DIFF_TB_SHAPES):
    """FP32 diffusion at r = 14 (the diffusion workload's size), lambda and
    bounding box: one launch per step at each rho (`reps` samples of a tenth
    of `steps` launches), and the temporally blocked passes at rho = 16, 32
    and 64 with 4, 8, 12 or 16 steps per pass (`shapes`; `reps` calls of 48
    steps, so every pass length divides them); 8 algorithmic bytes per cell
    and step."""
    r = 14
    cells = 3 ** r
    u0 = inputs.uniform_field(r, SEED)
    U = torch.from_numpy(u0).cuda()
    V = torch.zeros_like(U)
    calls = max(1, steps // 10)
    res = {"lambda": {}, "bbox": {}}
    for map_kind in ("lambda", "bbox"):
        for rho in rhos:
            bufs = [U.clone(), V]
            st = {"i": 0}

            def step():
                i = st["i"]
                sg.sg_diffuse_step(map_kind, r, rho, bufs[i], bufs[1 - i], 0.2)
                st["i"] = 1 - i
            res[map_kind][rho] = time_samples(torch, step, reps, warmup, calls)
            log(f"diffuse r=14 {map_kind:6s} rho={rho:3d}: "
                f"{stats(res[map_kind][rho])['median_ms'] * 1e3:8.2f} us/step")
            del bufs
    tb = {"lambda": {}, "bbox": {}}
    Out, Work = torch.zeros_like(U), torch.zeros_like(U)
    tb_steps = 48
    for map_kind in ("lambda", "bbox"):
        for rho, T in shapes:
            def run():
                sg.sg_diffuse_steps(map_kind, r, rho, tb_steps, U, Out, Work, 0.2,
                                    steps_per_pass=T)
            try:
                run()
            except RuntimeError as e:  # a pass the device's LDS cannot hold
                log(f"diffuse r=14 {map_kind:6s} rho={rho:3d} {T}/pass: not run ({e})")
                continue
            tb[map_kind][(rho, T)] = [ms / tb_steps for ms in time_samples(torch, run, reps, 1)]
            log(f"diffuse r=14 {map_kind:6s} rho={rho:3d} {T:2d}/pass: "
                f"{stats(tb[map_kind][(rho, T)])['median_ms'] * 1e3:8.2f} us/step")
    med = lambda v: stats(v)["median_ms"]  # noqa: E731
    cands = [((rho, 1), med(v)) for rho, v in res["lambda"].items()]
    cands += [(k, med(v)) for k, v in tb["lambda"].items()]
    (best, best_T), ms = min(cands, key=lambda kv: kv[1])
    bb_cands = [((rho, 1), med(v)) for rho, v in res["bbox"].items()]
    bb_cands += [(k, med(v)) for k, v in tb["bbox"].items()]
    (bb_best, bb_T), bb_ms = min(bb_cands, key=lambda kv: kv[1])
    return {"r": r, "cells": cells,
            "one_launch_per_step_us": {m: {str(k): us_stats(v) for k, v in res[m].items()}
                                       for m in res},
            "temporally_blocked_us": {m: {f"rho{k[0]}_T{k[1]}": us_stats(v)
                                          for k, v in tb[m].items()} for m in tb},
            "best": {"rho": best, "steps_per_launch": best_T, "us_per_step": round(ms * 1e3, 3)},
            "best_bbox": {"rho": bb_best, "steps_per_launch": bb_T,
                          "us_per_step": round(bb_ms * 1e3, 3)},
            "cells_per_s": cells / (ms * 1e-3),
            "best_vs_best_bbox": round(bb_ms / ms, 3),
            "effective_hbm_frac": round(8 * cells / (ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
            "roofline": diffusion_roofline(cells, best, best_T, ms)}


def diffusion_roofline(cells, rho, T, ms_per_step):
    """The best diffusion shape against the vector FP32 peak: the temporally
    blocked passes are bound by VALU issue on chip (their committed profile's
    busy share), so algorithmic flops per second is the achieved figure; the
    profile's counter bytes give the measured HBM traffic per launch."""
    flops = DIFF_FLOPS_PER_CELL * cells / (ms_per_step * 1e-3) / 1e12
    out = {"kernel": f"k_diffuse_tb<{rho}, lambda>" if T > 1 else f"one launch per step, rho={rho}",
           "bound": "alu" if T > 1 else "hbm",
           "achieved": round(flops, 3), "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
           "frac": round(flops / PEAK_FP32_TFLOPS, 4),
           "flops_per_cell_step": DIFF_FLOPS_PER_CELL, "traffic": None}
    prof = kernel_profile(f"diffuse_tb_rho{rho}_T{T}_r14") if T > 1 else None
    if prof:
        out["traffic"] = prof.get("bytes_per_launch")
        out["profile"] = f"profiles/diffuse_tb_rho{rho}_T{T}_r14.json"
        for key in ("valu_busy", "lds_bank_conflict_share", "avg_duration_us",
                    "issued_lane_ops_per_cell_generation"):
            if key in prof:
                out[f"profile_{key}"] = prof[key]
    return out


def bench_batched(torch, sg, inputs, count, steps, runs):
    """Many gaskets of uneven level (r ~ U{6..13}, Bernoulli(p), p ~ U[0.2, 0.8])
    advanced `steps` generations: autotuned persistent batched passes in one
    hipGraph, against the same launches without the graph and against one
    gasket at a time."""
    from paper_1706_04552_amd import batch
    specs = inputs.batch_specs(count)
    gs = []
    for spec in specs:
        inp = torch.from_numpy(spec.state()).cuda()
        gs.append(batch.Gasket(spec.r, steps, inp, torch.zeros_like(inp), torch.zeros_like(inp)))
    cell_steps = sum(3 ** g.r * steps for g in gs)
    tune, tune_ms = batch.autotune(gs)
    log(f"batched: autotuned {tune.as_dict()} ({tune_ms:.2f} ms)")
    out = {"gaskets": count, "steps": steps, "cell_steps": cell_steps, "tune": tune.as_dict()}
    with batch.Batch(gs, tune) as bt:
        for name, graph in (("graph", True), ("eager", False)):
            t = time_samples(torch, lambda: bt.run(graph=graph), runs, 1)
            ms = stats(t)["median_ms"]
            out[f"{name}_ms"] = ms_stats(t)
            out[f"{name}_cells_per_s"] = cell_steps / (ms * 1e-3)
            log(f"batched {name}: {ms:.3f} ms per run, {cell_steps / (ms * 1e-3) / 1e9:.1f} Gcells/s")
        got = [g.out.clone() for g in gs[:8]]

    def one_at_a_time():
        for g in gs:
            sg.sg_ca_steps("lambda", g.r, min(256, 1 << g.r), steps, g.inp, g.out, g.work,
                           steps_per_pass=0)
    t = time_samples(torch, one_at_a_time, runs, 1)
    ms = stats(t)["median_ms"]
    out["one_at_a_time_ms"] = ms_stats(t)
    out["one_at_a_time_cells_per_s"] = cell_steps / (ms * 1e-3)
    log(f"batched one-at-a-time: {ms:.3f} ms")
    out["same_as_alone"] = all(torch.equal(a, g.out) for a, g in zip(got, gs[:8]))
    return out


def bench_fractals(torch, sg, r, steps):
    """Other embedded fractals at r = 10 (n = 59049, a 3.5 GB uint8 embedding):
    the write pass and the life step, generalised block map against the
    bounding box, at every block side 3^q.  The life state is Bernoulli(0.5)
    on the fractal's cells, drawn on the device (torch generator, seed 1706)."""
    motifs = {"carpet": (3, [(x, y) for y in range(3) for x in range(3) if (x, y) != (1, 1)]),
              "vicsek": (3, [(1, 0), (0, 1), (1, 1), (2, 1), (1, 2)])}
    out = {}
    for name, (m, offs) in motifs.items():
        f = sg.fractal(m, offs)
        n = m ** r
        cells = len(offs) ** r
        A = torch.zeros((n, n), dtype=torch.uint8, device="cuda")
        sg.sg_frac_write(f, "lambda", r, 1, A, 1)  # the fractal's mask
        g = torch.Generator(device="cuda")
        g.manual_seed(SEED)
        step_rows = max(1, (1 << 28) // n)
        for y0 in range(0, n, step_rows):
            rows = A[y0:y0 + step_rows]
            rows &= (torch.rand(rows.shape, generator=g, device="cuda") < 0.5).to(torch.uint8)
        B = torch.zeros_like(A)
        W = torch.zeros_like(A)
        res = {"n": n, "cells": cells, "write_us": {}, "life_us": {}}
        rho = 3
        while rho <= 243:
            for map_kind in ("lambda", "bbox"):
                wt = time_samples(torch, lambda: sg.sg_frac_write(f, map_kind, r, rho, W, 1),
                                  steps, 2)
                bufs, st = [A.clone(), B], {"i": 0}

                def life():
                    i = st["i"]
                    sg.sg_frac_life_step(f, map_kind, r, rho, bufs[i], bufs[1 - i])
                    st["i"] = 1 - i
                lt = time_samples(torch, life, steps, 2)
                res["write_us"].setdefault(map_kind, {})[str(rho)] = round(stats(wt)["median_ms"] * 1e3, 2)
                res["life_us"].setdefault(map_kind, {})[str(rho)] = round(stats(lt)["median_ms"] * 1e3, 2)
                res.setdefault("se_us", {}).setdefault(map_kind, {})[str(rho)] = {
                    "write": round(stats(wt)["se_ms"] * 1e3, 2), "life": round(stats(lt)["se_ms"] * 1e3, 2)}
                del bufs
            log(f"{name} r={r} rho={rho:3d}: write lambda {res['write_us']['lambda'][str(rho)]:9.1f} us "
                f"bbox {res['write_us']['bbox'][str(rho)]:9.1f} us; life lambda "
                f"{res['life_us']['lambda'][str(rho)]:9.1f} us bbox {res['life_us']['bbox'][str(rho)]:9.1f} us")
            rho *= 3
        for kind in ("write_us", "life_us"):
            lam = min(res[kind]["lambda"].values())
            box = min(res[kind]["bbox"].values())
            res[kind.replace("_us", "_best_vs_best")] = round(box / lam, 3)
        res["life_cells_per_s"] = cells / (min(res["life_us"]["lambda"].values()) * 1e-6)
        out[name] = res
        del A, B, W
        torch.cuda.empty_cache()
    return out


def bench_serving(torch, sg, inputs, qps_list, count, cap_gb, horizon_cells=None,
                  budget_cells=None):
    """Poisson arrivals of life solves (r ~ U{8..15}, steps ~ U{10..200})
    served by the native continuous-batching server (sg_server_replay: the
    arrivals, admission by HBM footprint under the cap, the rounds of batched
    passes and the latency clock are all in native code), against the same
    loop admitting one request at a time (max_active = 1) on the same
    arrivals.  In host mode the server starts a request's upload only while
    no other host transfer is in flight (its default transfer window of 1);
    the same run without that window is reported too.  Two input modes:
      host: each request's initial state is uploaded from pinned host memory
        when it is admitted and its result read back into pinned host memory
        when it finishes (copy streams beside the passes); a request's
        latency ends when its read-back has completed;
      resident: initial states already on the device, results left there.
    Requests of one level share an initial state (Bernoulli(0.5), seed
    1706 + r) and, in host mode, one pinned result buffer: the passes' and
    transfers' costs do not depend on the contents."""
    from paper_1706_04552_amd import batch, serving
    levels = range(8, 16)
    dev_t = {r: torch.from_numpy(inputs.bernoulli_state(r, 0.5, SEED + r)).cuda() for r in levels}
    host_t = {r: dev_t[r].cpu().pin_memory() for r in levels}
    host_o = {r: torch.empty_like(host_t[r]).pin_memory() for r in levels}
    # launch shape: autotuned once on a sample of the request mix
    sample = inputs.poisson_requests(1.0, 48, seed=SEED + 7)
    gs = [batch.Gasket(q.r, q.steps, dev_t[q.r], torch.zeros_like(dev_t[q.r]),
                       torch.zeros_like(dev_t[q.r])) for q in sample]
    tune, _ = batch.autotune(gs)
    del gs
    torch.cuda.empty_cache()
    cap = int(cap_gb * 1e9)
    server = serving.NativeServer(tune, cap, count, int(horizon_cells or 0), int(budget_cells or 0))
    first = inputs.poisson_requests(qps_list[0], count)
    server.reserve([q.r for q in first])  # the server's pool, sized at start
    results = []
    for qps in qps_list:
        reqs = inputs.poisson_requests(qps, count)
        rq = [serving.Request(q.rid, q.arrival, q.r, q.steps) for q in reqs]
        cells = float(sum(3 ** q.r * q.steps for q in rq))
        row = {"qps": qps, "cap_gb": cap_gb, "requests": len(rq)}
        for io in ("host", "resident"):
            inits = {q.rid: (host_t if io == "host" else dev_t)[q.r] for q in rq}
            outs = {q.rid: host_o[q.r] for q in rq} if io == "host" else None
            modes = [("continuous", 0, 1), ("one_at_a_time", 1, 1)]
            if io == "host":  # uploads not held back: interleaved with read-backs
                modes.insert(1, ("continuous_no_transfer_window", 0, 0))
            for mode, k, window in modes:
                server.set_max_active(k)
                server.set_transfer_window(window)
                server.replay(rq[:16], inits, outs)  # warm-up (first-call costs)
                st = server.replay(rq, inits, outs)
                summ = st.summary()
                summ["cells_per_s"] = cells / max(st.makespan, 1e-12)
                row[f"{io}_{mode}"] = summ
                log(f"serving qps={qps:.0f} {io:8s} {mode:29s}: p50 {summ['p50_ms']:8.2f} ms "
                    f"p99 {summ['p99_ms']:8.2f} ms  {summ['cells_per_s'] / 1e9:8.1f} Gcells/s "
                    f"makespan {st.makespan * 1e3:8.1f} ms")
        server.set_max_active(0)
        server.set_transfer_window(1)
        results.append(row)
    stats = server.stats()
    server.close()
    del dev_t, host_t, host_o
    torch.cuda.empty_cache()
    return {"tune": tune.as_dict(), "requests": count, "horizon_cells": horizon_cells,
            "budget_cells": budget_cells, "server": {k: int(v) for k, v in stats.items()},
            "by_qps": results}


def bench_compact_large(torch, sg, r, rho, steps, reps):
    """Life on a gasket whose embedding cannot exist (2^(2r) bytes): the
    block-compacted state (3^(r-k) tiles of rho^2 bytes) written on the device
    from the counter-based Bernoulli(0.5) generator, then `steps` generations
    at up to 32 per pass; `reps` timed calls after one warm-up call."""
    size = sg.sg_compact_bytes(r, rho)
    a = torch.empty(size, dtype=torch.uint8, device="cuda")
    out, work = torch.empty_like(a), torch.empty_like(a)
    init_ms = time_region(torch, lambda: sg.sg_compact_init_bernoulli(r, rho, SEED, 0.5, a), 1, 1)
    t = time_samples(torch, lambda: sg.sg_ca_steps_compact(r, rho, steps, a, out, work), reps, 1)
    ms = stats(t)["median_ms"]
    cells = 3 ** r
    us = ms * 1e3 / steps
    frac = CA_BYTES_PER_CELL * cells / (us * 1e-6) / (PEAK_HBM_GBS * 1e9)
    log(f"compact r={r} rho={rho}: {3 * size / 1e9:.1f} GB of states, init {init_ms:.2f} ms, "
        f"{us:.1f} us/gen, {cells / (us * 1e-6) / 1e12:.2f} Tcells/s ({frac:.2f} of the HBM "
        f"peak in fractal bytes, temporally blocked)")
    del a, out, work
    torch.cuda.empty_cache()
    return {"r": r, "rho": rho, "cells": cells, "state_gb": round(size / 1e9, 2),
            "embedding_bytes": 1 << (2 * r), "init_ms": round(init_ms, 3), "steps": steps,
            "us_per_step": round(us, 2), "se_us_per_step": round(stats(t)["se_ms"] * 1e3 / steps, 3),
            "repeats": len(t), "cells_per_s": cells / (us * 1e-6),
            "effective_hbm_frac": round(frac, 4)}


EXTRA_LEGS = ("sweep", "diffusion", "batched", "fractals", "serving", "compact_r20")


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100,
                    help="generations in each timed region")
    ap.add_argument("--warmup", type=int, default=10,
                    help="untimed generations before the timed regions")
    ap.add_argument("--repeats", type=int, default=10,
                    help="timed regions per configuration (median and standard error)")
    ap.add_argument("--rho", type=int, nargs="*", default=list(RHOS))
    ap.add_argument("--per-pass", type=int, nargs="*", default=[8, 16, 32],
                    help="generations per pass for the temporally blocked step")
    ap.add_argument("--skip-single", action="store_true",
                    help="skip the one-launch-per-generation sweep")
    ap.add_argument("--skip-write", action="store_true",
                    help="skip the write-pass legs")
    ap.add_argument("--skip-write-variants", action="store_true",
                    help="time only the write pass itself (no intra-block, rectangular or "
                         "paper-protocol legs)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the sweep, diffusion, batched, fractal and serving legs")
    ap.add_argument("--extras", nargs="*", choices=EXTRA_LEGS, default=list(EXTRA_LEGS),
                    help="which of the extra legs to run (default: all)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--serve-qps", type=float, nargs="*", default=[1000.0, 4000.0, 16000.0])
    ap.add_argument("--serve-requests", type=int, default=400)
    ap.add_argument("--serve-horizon", type=float, default=4e9,
                    help="cell updates queued per scheduling round (0: one pass per round)")
    ap.add_argument("--serve-budget", type=float, default=2e9,
                    help="cell updates per batched pass, oldest requests first (0: no budget)")
    ap.add_argument("--diffusion-shapes", nargs="*", type=_shape, default=DIFF_TB_SHAPES,
                    help="temporally blocked diffusion passes to time, as RHOxT (default: "
                         "rho 16, 32, 64 x 4, 8, 12, 16 steps per pass)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: --gpus {args.gpus} is not supported "
              f"(the gasket path is measured on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    K, W, REPS = args.steps, args.warmup, max(1, args.repeats)
    if K < 1:
        print("--steps must be at least 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1706_04552_amd import inputs, sg
    sg.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = 1 << R
    cells = 3 ** R

    log(f"generating r={R} state (n={n}, {cells} gasket cells)")
    a0 = inputs.bernoulli_state(R, 0.5, SEED)
    A = torch.from_numpy(a0).to(dev)
    B = torch.zeros_like(A)
    torch.cuda.synchronize()

    if args.copy_calibration:
        # a plain streaming kernel of known traffic: reads 1 GiB, writes 1 GiB
        src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        ms = time_region(torch, lambda: torch.bitwise_not(src, out=dst), 5, 1)
        log(f"copy calibration: 1 GiB in {ms * 1e3:.1f} us = {2 * (1 << 30) / (ms * 1e-3) / 1e9:.0f} GB/s")
        del src, dst

    # every timed region below is K generations, bracketed by device
    # synchronisations; REPS regions per configuration; ms per generation
    results = {"lambda": {}, "bbox": {}}
    if not args.skip_single:
        for map_kind in ("lambda", "bbox"):
            for rho in args.rho:
                bufs = [A.clone(), B]
                state = {"i": 0}

                def step():
                    i = state["i"]
                    sg.sg_ca_step(map_kind, R, rho, bufs[i], bufs[1 - i])
                    state["i"] = 1 - i

                results[map_kind][rho] = time_samples(torch, step, REPS, W, K)
                ms = stats(results[map_kind][rho])["median_ms"]
                log(f"ca 1/launch {map_kind:6s} rho={rho:3d}: {ms * 1e3:9.2f} us/step  "
                    f"{cells / (ms * 1e-3) / 1e9:8.2f} Gcells/s")
                del bufs
                B.zero_()

    # temporally blocked: K generations per call, up to T per pass
    warm_calls = -(-W // K) if W > 0 else 0
    multi = {"lambda": {}, "bbox": {}}
    Out = torch.zeros_like(A)
    Work = torch.zeros_like(A)
    for map_kind in ("lambda", "bbox"):
        shapes = [(rho, T) for rho in args.rho if rho in TB_RHOS for T in args.per_pass if T > 1]
        shapes += [(rho, T) for rho in args.rho if rho in TB_SMALL_RHOS
                   for T in args.per_pass if 1 < T <= 16]
        for rho, T in shapes:
            def run():
                sg.sg_ca_steps(map_kind, R, rho, K, A, Out, Work, steps_per_pass=T)
            multi[map_kind][(rho, T)] = [ms / K for ms in time_samples(torch, run, REPS, warm_calls)]
            ms = stats(multi[map_kind][(rho, T)])["median_ms"]
            log(f"ca {T:2d}/pass   {map_kind:6s} rho={rho:3d}: {ms * 1e3:9.2f} us/step  "
                f"{cells / (ms * 1e-3) / 1e9:8.2f} Gcells/s")
    del Out, Work

    # block-compacted storage: only the fractal tiles, (4/3)^k * 3^r bytes
    compact = {}
    for rho in [x for x in args.rho if x in COMPACT_RHOS]:
        size = sg.sg_compact_bytes(R, rho)
        Cin = torch.empty(size, dtype=torch.uint8, device=dev)
        sg.sg_compact_pack(R, rho, A, Cin)
        Cout, Cwork = torch.empty_like(Cin), torch.empty_like(Cin)
        for T in [t for t in args.per_pass if t > 1]:
            def run():
                sg.sg_ca_steps_compact(R, rho, K, Cin, Cout, Cwork, steps_per_pass=T)
            t = [ms / K for ms in time_samples(torch, run, REPS, warm_calls)]
            compact[f"rho{rho}_T{T}"] = us_stats(t)
            ms = stats(t)["median_ms"]
            log(f"ca {T:2d}/pass   compact rho={rho:3d}: {ms * 1e3:9.2f} us/step  "
                f"{cells / (ms * 1e-3) / 1e9:8.2f} Gcells/s  ({size / 2 ** 30:.2f} GiB state)")
        compact[f"rho{rho}_state_gib"] = round(size / 2 ** 30, 3)
        del Cin, Cout, Cwork

    med = lambda v: stats(v)["median_ms"]  # noqa: E731
    cands = [((rho, 1), v) for rho, v in results["lambda"].items()]
    cands += list(multi["lambda"].items())
    (best_rho, best_T), best_samples = min(cands, key=lambda kv: med(kv[1]))
    best = stats(best_samples)
    best_ms = best["median_ms"]
    bb_cands = [((rho, 1), v) for rho, v in results["bbox"].items()] + list(multi["bbox"].items())
    (bb_rho, bb_T), bb_samples = min(bb_cands, key=lambda kv: med(kv[1]))
    bb_ms = med(bb_samples)

    # the paper's experiment: write a constant on every gasket cell
    wp = {"lambda": {}, "bbox": {}}
    intra, rect = {}, {}
    paper = {"lambda": {}, "bbox": {}}
    write_calls = max(1, K // 10)
    if not args.skip_write:
        Wt = torch.zeros_like(A)
        for map_kind in ("lambda", "bbox"):
            for rho in args.rho:
                wp[map_kind][rho] = time_samples(
                    torch, lambda: sg.sg_write_pass(map_kind, R, rho, Wt, 1), REPS, W, write_calls)
                log(f"write {map_kind:6s} rho={rho:3d}: {med(wp[map_kind][rho]) * 1e3:9.2f} us")
        # the paper's other intra-block mappings (one thread per gasket cell)
        for variant in (() if args.skip_write_variants else ("unroll", "lut")):
            for map_kind in ("lambda", "bbox"):
                for rho in [x for x in args.rho if x <= 32]:
                    t = time_samples(torch, lambda: sg.sg_write_pass_intra(map_kind, variant, R, rho, Wt, 1),
                                     REPS, W, write_calls)
                    intra.setdefault(variant, {}).setdefault(map_kind, {})[str(rho)] = us_stats(t)
                    log(f"write {variant:6s} {map_kind:6s} rho={rho:3d}: {med(t) * 1e3:9.2f} us")
        # rectangular blocks: whole 64-byte rows with fewer cells per block
        for (rx, ry) in (() if args.skip_write_variants else
                         ((64, 4), (64, 16), (128, 8), (256, 4), (256, 16), (256, 64))):
            for map_kind in ("lambda", "bbox"):
                t = time_samples(torch, lambda: sg.sg_write_pass_rect(map_kind, R, rx, ry, Wt, 1),
                                 REPS, W, write_calls)
                rect.setdefault(map_kind, {})[f"{rx}x{ry}"] = us_stats(t)
            log(f"write rect {rx:3d}x{ry:<3d}: lambda {rect['lambda'][f'{rx}x{ry}']['median_us']:9.2f} us  "
                f"bbox {rect['bbox'][f'{rx}x{ry}']['median_us']:9.2f} us")
        # the paper's timing protocol (Section IV): the mean of 100 sub-averages,
        # each the mean time of 10 consecutive calls, every call followed by a
        # device synchronisation; host clock, so launch and synchronisation
        # overhead are included.  Over the paper's block sides rho = 1..32.
        for map_kind in (() if args.skip_write_variants else ("lambda", "bbox")):
            for rho in (1, 2, 4, 8, 16, 32):
                sg.sg_write_pass(map_kind, R, rho, Wt, 1)
                torch.cuda.synchronize()
                subs = []
                for _ in range(100):
                    t0 = time.perf_counter()
                    for _ in range(10):
                        sg.sg_write_pass(map_kind, R, rho, Wt, 1)
                        torch.cuda.synchronize()
                    subs.append((time.perf_counter() - t0) / 10)
                mean = float(np.mean(subs))
                se = float(np.std(subs, ddof=1)) / 10.0
                paper[map_kind][str(rho)] = {"us": round(mean * 1e6, 2),
                                             "se_pct": round(100.0 * se / mean, 3)}
            log(f"write (paper protocol) {map_kind:6s}: " + "  ".join(
                f"rho={k}: {v['us']:.1f} us" for k, v in paper[map_kind].items()))
        del Wt

    # roofline of the dominant kernel, per launch: a timed region of K
    # generations runs `launches` launches of it, which split the K
    # generations evenly (floor or ceil of K / launches each)
    launches = -(-K // best_T)
    gens_per_launch = K / launches
    launch_us = best_ms * K / launches * 1e3
    if best_T > 1:
        if best_rho < 32:
            kname = f"k_life_tbs<{best_rho}, lambda>"
        elif launches == 1:
            kname = f"k_life_tb<{best_rho}, lambda>"
        else:
            # the state between launches is bit-packed tiles
            kname = (f"k_life_tb_bits<{best_rho}, lambda> (bytes to bits, "
                     f"{launches - 2} x bits to bits, bits to bytes)")
        tag = (f"life_tb_rho{best_rho}_T{K // launches}_r{R}" if K % launches == 0 else None)
    else:
        kname = f"k_life_strip<{best_rho}, lambda>" if best_rho >= 32 else f"k_life<{best_rho}, lambda>"
        tag = f"life_step_rho{best_rho}_r{R}"
    prof = kernel_profile(tag) if tag else None
    traffic = prof.get("bytes_per_launch") if prof else None
    frac_bytes = CA_BYTES_PER_CELL * cells / (best_ms * 1e-3) / 1e9 / PEAK_HBM_GBS
    if best_T > 1:
        # on-chip generations: VALU issue binds (the profile's busy share);
        # algorithmic work is the bit-sliced rule on the gasket's cells
        ops = LIFE_OPS_PER_CELL * cells * gens_per_launch
        achieved = ops / (launch_us * 1e-6) / 1e12
        roofline = {"bound": "alu", "achieved": round(achieved, 4), "peak": PEAK_ALU_TOPS,
                    "unit": "TOP/s", "frac": round(achieved / PEAK_ALU_TOPS, 4), "traffic": traffic,
                    "ops_per_cell_generation": LIFE_OPS_PER_CELL,
                    "algorithmic_ops_per_launch": round(ops)}
    else:
        launch_bytes = CA_BYTES_PER_CELL * cells
        achieved = launch_bytes / (launch_us * 1e-6) / 1e9
        roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                    "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": traffic,
                    "algorithmic_bytes_per_launch": launch_bytes}
    roofline.update({
        "kernel": kname, "launch_duration_us": round(launch_us, 2), "launches": launches,
        "generations_per_launch": round(gens_per_launch, 3),
        "effective_hbm_frac": round(frac_bytes, 4),
        "measured_hbm_frac": (round(traffic / (launch_us * 1e-6) / (PEAK_HBM_GBS * 1e9), 4)
                              if traffic else None),
        # measured HBM bytes of a launch over the fractal bytes it must move
        # (every gasket cell read once and written once)
        "traffic_over_fractal_bytes": (round(traffic / (CA_BYTES_PER_CELL * cells), 3)
                                       if traffic else None),
        "profile": (f"profiles/{tag}.json" if prof else None)})
    if prof:
        for key in ("valu_busy", "lds_bank_conflict_share", "avg_duration_us"):
            if key in prof:
                roofline[f"profile_{key}"] = prof[key]
        if "sq_insts_valu" in prof and best_T > 1:
            roofline["issued_lane_ops_per_cell_generation"] = round(
                prof["sq_insts_valu"] * 64 / (cells * gens_per_launch), 3)

    extras = {}
    legs = [] if args.no_extras else args.extras
    if legs:
        del A, B
        torch.cuda.empty_cache()
    if "sweep" in legs:
        extras["sweep_one_launch_per_step"] = bench_sweep(torch, sg, inputs, (10, 12, 14),
                                                          (4, 8, 16, 32, 64, 128, 256), 100)
    if "diffusion" in legs:
        extras["diffusion"] = bench_diffusion(torch, sg, inputs, (16, 64, 128, 256), K, W, REPS,
                                              args.diffusion_shapes)
    if "batched" in legs:
        extras["batched"] = bench_batched(torch, sg, inputs, args.batch_count, 50, REPS)
    if "fractals" in legs:
        extras["other_fractals"] = bench_fractals(torch, sg, 10, max(REPS, 20))
        torch.cuda.empty_cache()
    if "compact_r20" in legs:
        extras["compact_r20"] = bench_compact_large(torch, sg, 20, 256, 64, REPS)
    if "serving" in legs:
        extras["serving"] = bench_serving(torch, sg, inputs, args.serve_qps, args.serve_requests,
                                          200.0, int(args.serve_horizon) or None,
                                          int(args.serve_budget) or None)
        torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle (r=16 generations, bounded samples)")
        cpu = cpu_baseline(R, a0)
        if "diffusion" in legs:
            # the diffusion workload's error against the oracle's FP64 run,
            # which is also that workload's CPU baseline
            extras["diffusion"]["error_vs_fp64"] = diffusion_error_vs_fp64(
                torch, sg, inputs, [("lambda", 16, 1), ("lambda", 16, 8), ("lambda", 16, 16),
                                    ("lambda", 32, 8), ("bbox", 16, 8)])

    prop = torch.cuda.get_device_properties(0)
    wl = min(wp["lambda"], key=lambda k: med(wp["lambda"][k])) if wp["lambda"] else None
    wb = min(wp["bbox"], key=lambda k: med(wp["bbox"][k])) if wp["bbox"] else None
    pl = min(paper["lambda"], key=lambda k: paper["lambda"][k]["us"]) if paper["lambda"] else None
    pb = min(paper["bbox"], key=lambda k: paper["bbox"][k]["us"]) if paper["bbox"] else None
    out = {
        "metric": "fractal cells updated/s + % HBM peak, lambda vs bbox map, n=2^16 CA step",
        "value": cells / (best_ms * 1e-3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": best_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic: Bernoulli(0.5) uint8 on the gasket cells, seed 1706",
        "config": {"workload": "B3/S23 life step on the r=16 embedded Sierpinski gasket "
                               "(n=65536, 43,046,721 cells), uint8, lambda map",
                   "r": R, "rho": best_rho, "map": "lambda",
                   "steps_per_pass_limit": best_T, "launches_per_timed_region": launches,
                   "generations_per_launch": round(gens_per_launch, 3),
                   "temporal_blocking": best_T > 1},
        "timing": {"timed_regions": best["n"], "generations_per_region": K,
                   "median_ms_per_step": best_ms, "se_ms_per_step": best["se_ms"],
                   "min_ms_per_step": best["min_ms"], "max_ms_per_step": best["max_ms"],
                   "value_is": "median over the timed regions"},
        "roofline": roofline,
        "device": {"name": prop.name, "arch": getattr(prop, "gcnArchName", ""),
                   "cus": prop.multi_processor_count,
                   "hbm_gib": round(prop.total_memory / 2 ** 30, 1)},
        "cpu_baseline": cpu,
        "effective_hbm_frac_fractal_bytes": round(frac_bytes, 4),
        "lambda_vs_bbox": {
            "one_launch_per_step_us": {m: {str(k): us_stats(v) for k, v in results[m].items()}
                                       for m in results},
            "speedup_per_rho": {str(k): round(med(results["bbox"][k]) / med(results["lambda"][k]), 3)
                                for k in results["lambda"] if k in results["bbox"]},
            "temporally_blocked_us": {m: {f"rho{k[0]}_T{k[1]}": us_stats(v)
                                          for k, v in multi[m].items()} for m in multi},
            "best_vs_best": round(bb_ms / best_ms, 3),
            "best": {"lambda": {"rho": best_rho, "steps_per_pass_limit": best_T},
                     "bbox": {"rho": bb_rho, "steps_per_pass_limit": bb_T,
                              "us_per_step": round(bb_ms * 1e3, 3)}},
            "compact_storage_us": compact,
            "embedding_state_gib": round(n * n / 2 ** 30, 3),
        },
    }
    if wl is not None:
        out["write_pass"] = {
            "us": {m: {str(k): us_stats(v) for k, v in wp[m].items()} for m in wp},
            "best_vs_best": round(med(wp["bbox"][wb]) / med(wp["lambda"][wl]), 3),
            "best_rho": {"lambda": wl, "bbox": wb},
            "intra_block_variants_us": intra,
            "rectangular_blocks_us": rect,
            "paper_protocol": None if pl is None else {
                "what": "mean of 100 sub-averages of 10 consecutive calls, each followed by a "
                        "device synchronisation (host clock: launch and sync overhead included)",
                "us": paper, "best_rho": {"lambda": int(pl), "bbox": int(pb)},
                "best_vs_best": round(paper["bbox"][pb]["us"] / paper["lambda"][pl]["us"], 3)},
            "lambda_cells_per_s": cells / (med(wp["lambda"][wl]) * 1e-3),
            "paper_context": PAPER_BEST_VS_BEST,
        }
    out.update(extras)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
