#!/usr/bin/env python
"""sDTW throughput on one MI355X.

Workload (the shape of the paper's Section 6 experiment): 512 queries of
2,000 samples against one 100,000-sample reference, FP32, squared-difference
cost; seeded synthetic z-normalised random walks (half of the queries are
time-warped noisy excerpts of the reference).  One step = one sdtw_forward
call over the whole batch (DP fill, last-row minimum and end position), with
every input already resident in device memory.

Prints ONE JSON line.  Beside the headline value it reports:
  roofline      the dominant kernel against the chip's FP32 vector peak,
                157.3 TFLOP/s (256 CUs x 2.4 GHz; an FMA counted as two
                flops), with a DP cell counted as 5 flops (subtraction,
                product, two comparisons of the three-way minimum, sum); and
                against the issue ceiling of its own instructions: 4 VALU
                instructions per cell, two per SIMD per quad-cycle at most
                (78.6 T lane-instructions/s), both also at the shader clock
                measured during a sustained run;
  cpu_baseline  the CPU oracle timed on the same workload (all 512 queries)
                on the host's cores, checked bit for bit against the GPU;
  batched       the persistent uneven-length form (4,096 queries of
                250..4,000 samples vs 200,000) and the same batch run as a
                loop of plain launches over 16 length buckets;
  fwd_bwd       forward with checkpoints plus the walk-back gradient
                (256 x 1,000 vs 50,000), and the alignment-path output
                (sdtw_align) on the same forward;
  long_ref      512 x 2,000 vs a 2,000,000-sample reference, squared and
                absolute cost (3 VALU instructions per cell: |t| is a source
                modifier), each against its own roofline;
  f16           the same workload in binary16 arithmetic (two queries per
                packed value), against the packed-FP16 issue rate: gfx950
                never dual-issues packed (VOP3P) instructions, so its roofline
                is 256 CUs x 64 lanes x 2.4 GHz / 2.5 instructions per cell;
  pruned        the same workload with Section 8's early pruning (+inf cost
                for |q - r| > tau), 7 VALU instructions per cell, and how many
                queries keep their exact result at several tau;
  u8            the same workload on uint8 codes (Section 8's codebook
                quantisation): codebook, codes and the binary32 DP of the
                codes, 3 VALU instructions per cell (the code difference
                squared is exact, so the product and sum fuse), with the
                error of the scaled cost against the exact one;
  znorm         the batch z-normaliser that prepares the inputs, against
                the 8 TB/s HBM roofline (8 algorithmic bytes per sample:
                one read, one write).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PAPER_MS = 11036.5               # paper Table 1: sDTW kernel time, same shape
PAPER_CELLS = 512 * 2000 * 100000
PAPER_GCUPS = PAPER_CELLS / (PAPER_MS * 1e6)
PEAK_CUS = 256
PEAK_GHZ = 2.4
LANES_PER_CU_CLK = 128      # 4 SIMDs x 16 lanes x 2 (VALU dual issue)
PEAK_FP32_TFLOPS = 157.3    # MI355X FP32 vector peak (FMA = 2 flops)
# flops of one DP cell: subtraction, product (squared cost only), the two
# comparisons of the three-way minimum, sum
FLOPS_PER_CELL = {"squared": 5, "absolute": 4}


def valu_peak_gcups(ops_per_cell, cus=PEAK_CUS, ghz=PEAK_GHZ, lanes=LANES_PER_CU_CLK):
    return cus * lanes * ghz / ops_per_cell   # G lane-instr/s / instr per cell


# Sources that define the forward kernel's code (its arithmetic, memory
# traffic and compile flags); counter summaries are tied to their digest.
FWD_SOURCES = ("sdtw_common.hpp", "sdtw_argmin.hpp", "sdtw_value.hpp", "sdtw_fwd.hpp",
               "sdtw_variant.hpp", "sdtw_variant_tu.hip", "build.py")


def source_digest():
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2403_06931_amd", "csrc")
    for name in FWD_SOURCES:
        with open(os.path.join(d, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_tag):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", f"{kernel_tag}_counters.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_digest") != source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def progress(msg):
    """One line per finished step of the benchmark, on stderr (the JSON result
    goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def sample_sclk(run, launches, torch):
    """Median graphics clock (GHz) reported by amd-smi while `launches` calls of
    `run` keep the GPU busy; None where the clock cannot be read."""
    import threading
    try:
        import amdsmi
    except ImportError:
        return None
    samples, stop, state = [], threading.Event(), {}

    def poll():
        try:
            amdsmi.amdsmi_init()
            handles = amdsmi.amdsmi_get_processor_handles()
            bus = getattr(torch.cuda.get_device_properties(0), "pci_bus_id", None)
            pick = handles[0] if len(handles) == 1 else None
            for h in handles:
                if bus is not None and pick is None:
                    bdf = amdsmi.amdsmi_get_gpu_device_bdf(h)
                    if int(bdf.split(":")[1], 16) == int(bus):
                        pick = h
            if pick is None:
                return
            state["ok"] = True
            while not stop.is_set():
                samples.append(amdsmi.amdsmi_get_clock_info(
                    pick, amdsmi.AmdSmiClkType.GFX)["clk"])
                time.sleep(0.005)
        except Exception as exc:                  # noqa: BLE001 - reported as unavailable
            state["error"] = repr(exc)
        finally:
            try:
                amdsmi.amdsmi_shut_down()
            except Exception:                     # noqa: BLE001
                pass

    t = threading.Thread(target=poll, daemon=True)
    for _ in range(launches):
        run()
    t.start()
    torch.cuda.synchronize()
    stop.set()
    t.join(5)
    vals = sorted(v for v in samples if isinstance(v, (int, float)) and v > 0)
    if not vals:
        return None
    # samples taken while the GPU was busy: a profiler that serialises the
    # launches leaves the GPU idle (at its idle clock) between them
    busy = [v for v in vals if v >= 0.5 * vals[-1]]
    if busy[-1] < 1000:
        # every sample at an idle-level clock (below 1 GHz): the launches did
        # not keep the GPU busy while sampling (a profiler serialises them),
        # so there is no loaded clock to report
        return None
    return {"ghz": busy[len(busy) // 2] / 1000.0, "samples": len(vals), "busy_samples": len(busy),
            "min_ghz": vals[0] / 1000.0, "max_ghz": vals[-1] / 1000.0}


def oracle_subset(w, idx, kind, gpu_cost, gpu_end, cores):
    """The oracle on queries idx of workload w: GCUPS on the host cores, the
    full workload's time extrapolated from it, and bit-exact agreement with
    the GPU's results for those queries."""
    import numpy as np

    import oracle
    sub = w.subset(idx)
    t0 = time.perf_counter()
    c, e = oracle.sdtw_f32(sub.queries, sub.lens, sub.reference, kind, nthreads=cores)
    dt = time.perf_counter() - t0
    gcups = sub.cells / dt / 1e9
    return {"gcups": gcups, "cores": int(cores), "queries": int(len(idx)),
            "wall_s": dt, "extrapolated_full_s": w.cells / (gcups * 1e9),
            "bit_exact_vs_gpu": bool(np.array_equal(c.view(np.uint32),
                                                    gpu_cost[idx].view(np.uint32))
                                     and np.array_equal(e, gpu_end[idx]))}


def host_cores():
    import oracle
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return max(1, min(cores, oracle.max_threads()))


def time_steps(fn, steps, warmup, torch):
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return wall / steps * 1e3, ev0.elapsed_time(ev1) / steps


def cpu_baseline(w, gpu_cost, gpu_end):
    """The FP32 oracle on every query of the headline workload, OpenMP over
    queries on the host's cores."""
    import numpy as np
    cores = host_cores()
    rec = oracle_subset(w, np.arange(w.batch), 0, gpu_cost, gpu_end, cores)
    return {"value": rec["gcups"], "unit": "GCUPS", "cores": rec["cores"], "kind": "oracle",
            "sample": f"all {w.batch} queries (2,000 x 100,000 cells each), "
                      f"{rec['wall_s']:.1f} s wall", "cpu_model": cpu_model(),
            "bit_exact_vs_gpu": rec["bit_exact_vs_gpu"]}


def batched_leg(P, torch, steps, warmup, oracle_legs=True):
    import numpy as np

    import workloads
    w = workloads.make_config(3)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    rec, rec_grid = {}, {}
    # persistent candidates: at most four wavefronts per query (wider teams
    # waste most of their lanes on the short queries of this batch), timed
    # with the default grid; then the four fastest with grids of 2, 3 and 4
    # resident wavefronts per SIMD
    cands = [v for v in range(P.sdtw_variant_count()) if P.sdtw_variant_info(v)[2] <= 4]
    P.autotune.tune(q, w.lens, l, r, 0, P.SDTW_F_PERSISTENT, candidates=cands, reps=1,
                    record=rec)
    top = sorted(rec["times_ms"], key=rec["times_ms"].get)[:4]
    variant, flags = P.autotune.tune_persistent(q, w.lens, l, r, 0, candidates=top,
                                                waves_per_simd=(2, 3, 4), reps=1,
                                                record=rec_grid)
    # the timed step is the captured launch sequence (order + work-counter
    # reset, persistent kernel), replayed
    g = P.ForwardGraph(q, w.lens, l, r, 0, flags=flags, variant=variant)
    wall_ms, ev_ms = time_steps(g.replay, steps, warmup, torch)
    pc = g.cost.cpu().numpy().copy()
    pe = g.end_pos.cpu().numpy().copy()

    # baseline: plain launches over 16 equal-width length buckets
    edges = np.linspace(w.lens.min(), w.lens.max() + 1, 17)
    buckets = []
    for k in range(16):
        idx = np.nonzero((w.lens >= edges[k]) & (w.lens < edges[k + 1]))[0]
        if idx.size == 0:
            continue
        sub = w.subset(idx)
        qb = torch.from_numpy(sub.queries).to(dev)
        lb = torch.from_numpy(sub.lens).to(dev)
        wsb = P.workspace(P.sdtw_forward_workspace_bytes(sub.lens, w.ref_len, 0), dev)
        cb = torch.empty(sub.batch, dtype=torch.float32, device=dev)
        eb = torch.empty(sub.batch, dtype=torch.int64, device=dev)
        buckets.append((idx, sub.lens, qb, lb, wsb, cb, eb))

    def bucketed():
        for idx, hl, qb, lb, wsb, cb, eb in buckets:
            P.sdtw_forward(qb, hl, lb, r, 0, cost=cb, end_pos=eb, workspace_buf=wsb)
    bwall, bev = time_steps(bucketed, steps, warmup, torch)
    same = all(np.array_equal(cb.cpu().numpy().view(np.uint32), pc[idx].view(np.uint32))
               for idx, _, _, _, _, cb, _ in buckets)
    del g, buckets
    out = {"workload": w.name, "digest": workloads.digest(w), "cells": w.cells,
           "variant": P.sdtw_variant_info(variant), "waves_per_simd": (flags >> 8) & 0xf,
           "tuned_over": len(rec.get("times_ms", {})) + len(rec_grid.get("times_ms", {})),
           "grid_times_ms": rec_grid.get("times_ms"),
           "timed": "ForwardGraph.replay() (hipGraph of the persistent launch)",
           "gcups": w.cells / (ev_ms * 1e6), "ms_per_step": ev_ms,
           "gsps": float(w.lens.sum()) / (ev_ms * 1e6),
           "bucketed_loop_gcups": w.cells / (bev * 1e6), "bucketed_loop_ms": bev,
           "bit_identical_to_bucketed": bool(same)}
    if oracle_legs:
        # 64 seeded queries, two of them the shortest and the longest
        extremes = {int(np.argmin(w.lens)), int(np.argmax(w.lens))}
        rest = [int(b) for b in workloads.subset_indices(w, 70, seed=31) if b not in extremes]
        idx = np.array(sorted(extremes | set(rest[:64 - len(extremes)])), np.int64)
        out["oracle"] = oracle_subset(w, idx, 0, pc, pe, host_cores())
    return out


def fwd_bwd_leg(P, torch, steps, warmup, oracle_legs=True):
    import numpy as np

    import workloads
    w = workloads.make_config(4)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    K = 1024
    flags = P.SDTW_F_CHECKPOINT
    wsb = P.workspace(P.sdtw_backward_workspace_bytes(w.lens, w.ref_len, K), dev)
    ckpt = torch.empty(P.sdtw_checkpoint_floats(w.lens, w.ref_len, K), dtype=torch.float32,
                       device=dev)
    cost = torch.empty(w.batch, dtype=torch.float32, device=dev)
    end = torch.empty(w.batch, dtype=torch.int64, device=dev)
    g = torch.ones(w.batch, dtype=torch.float32, device=dev)
    gq = torch.empty_like(q)
    gr = torch.empty_like(r)

    # forward tile for this shape, timed with checkpoints
    from paper_2403_06931_amd import autotune as A
    rec = {}
    var = A.tune(q, w.lens, l, r, 0, flags, reps=2, record=rec, ckpt=ckpt, ckpt_every=K)
    ws = P.workspace(P.sdtw_forward_workspace_bytes(w.lens, w.ref_len, flags, var), dev)

    def fwd():
        P.sdtw_forward(q, w.lens, l, r, 0, cost=cost, end_pos=end, ckpt=ckpt, ckpt_every=K,
                       variant=var, flags=flags, workspace_buf=ws)

    def bwd():
        P.sdtw_backward(q, w.lens, l, r, 0, g, cost, end, ckpt, K, grad_queries=gq,
                        grad_reference=gr, workspace_buf=wsb)

    def both():
        fwd()
        bwd()
    _, f_ms = time_steps(fwd, steps, warmup, torch)
    _, b_ms = time_steps(bwd, steps, warmup, torch)
    _, fb_ms = time_steps(both, steps, warmup, torch)

    def plain():
        P.sdtw_forward(q, w.lens, l, r, 0, cost=cost, end_pos=end, variant=var,
                       workspace_buf=ws)
    _, p_ms = time_steps(plain, steps, warmup, torch)

    # alignment path output (start position and per-row ranges) from the
    # same checkpointed forward
    fwd()
    wsa = P.workspace(P.sdtw_align_workspace_bytes(w.lens, w.ref_len, K), dev)

    def align():
        P.sdtw_align(q, w.lens, l, r, 0, cost, end, ckpt, K, workspace_buf=wsa)
    _, a_ms = time_steps(align, steps, warmup, torch)
    out = {"workload": w.name, "digest": workloads.digest(w), "cells": w.cells,
           "ckpt_every": K, "gcups": w.cells / (fb_ms * 1e6), "ms_per_step": fb_ms,
           "fwd_ckpt_ms": f_ms, "bwd_ms": b_ms, "plain_fwd_ms": p_ms,
           "plain_fwd_gcups": w.cells / (p_ms * 1e6), "align_ms": a_ms,
           "variant": P.sdtw_variant_info(var), "tuned_over": len(rec.get("times_ms", {}))}
    if oracle_legs:
        import oracle
        both()
        torch.cuda.synchronize()
        cores = host_cores()
        t0 = time.perf_counter()
        oc, oe, _, ogq, ogr = oracle.sdtw_grad_f32(w.queries, w.lens, w.reference,
                                                   np.ones(w.batch, np.float32), 0,
                                                   nthreads=cores)
        dt = time.perf_counter() - t0
        same = (np.array_equal(oc.view(np.uint32), cost.cpu().numpy().view(np.uint32))
                and np.array_equal(oe, end.cpu().numpy())
                and np.array_equal(ogq.view(np.uint32), gq.cpu().numpy().view(np.uint32))
                and np.array_equal(ogr.view(np.uint32), gr.cpu().numpy().view(np.uint32)))
        out["oracle"] = {"what": "full-matrix forward and walk-back gradient, all 256 queries",
                         "gcups": w.cells / dt / 1e9, "cores": int(cores), "wall_s": dt,
                         "bit_exact_vs_gpu": bool(same)}
    return out


HBM_PEAK_GBS = 8000.0


def long_ref_leg(P, torch, variant, steps, warmup, oracle_legs=True):
    """512 x 2,000 vs 2,000,000, both cost kinds, in the headline's tile."""
    import numpy as np

    import workloads
    w = workloads.make_config(2)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    ws = P.workspace(P.sdtw_forward_workspace_bytes(w.lens, w.ref_len, 0, variant), dev)
    cost = torch.empty(w.batch, dtype=torch.float32, device=dev)
    end = torch.empty(w.batch, dtype=torch.int64, device=dev)
    out = {"workload": w.name, "digest": workloads.digest(w), "cells": w.cells,
           "variant": P.sdtw_variant_info(variant),
           "workspace_bytes": int(ws.numel())}
    for kind, name, ops in ((0, "squared", 4), (1, "absolute", 3)):
        def step(kind=kind):
            P.sdtw_forward(q, w.lens, l, r, kind, cost=cost, end_pos=end, variant=variant,
                           workspace_buf=ws)
        wall_ms, ev_ms = time_steps(step, steps, warmup, torch)
        peak = valu_peak_gcups(ops)
        gcups = w.cells / (ev_ms * 1e6)
        out[name] = {"ms_per_step": wall_ms, "gcups": w.cells / (wall_ms * 1e6),
                     "issue_frac": gcups / peak, "peak_gcups": peak,
                     "flop_frac": gcups * FLOPS_PER_CELL[name] / 1e3 / PEAK_FP32_TFLOPS}
        if oracle_legs:
            idx = np.sort(np.random.default_rng(workloads.BASE_SEED + 2 + kind)
                          .choice(w.batch, 16, replace=False))
            out[name]["oracle"] = oracle_subset(w, idx, kind, cost.cpu().numpy(),
                                                end.cpu().numpy(), host_cores())
    return out


def f16_leg(P, torch, steps, warmup):
    """sdtw_forward_f16 on the headline workload; the tile variant is picked
    by timing every compiled variant once (two calls each)."""
    import workloads
    w = workloads.make_config(1)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    ws = P.workspace(P.sdtw_forward_f16_workspace_bytes(w.lens, w.ref_len), dev)
    cost = torch.empty(w.batch, dtype=torch.float32, device=dev)
    end = torch.empty(w.batch, dtype=torch.int64, device=dev)
    times = {}
    for v in range(P.sdtw_variant_count()):
        def run(v=v):
            P.sdtw_forward_f16(q, w.lens, l, r, 0, cost=cost, end_pos=end, variant=v,
                               workspace_buf=ws)
        times[v] = time_steps(run, 1, 1, torch)[1]
    best = min(times, key=times.get)

    def step():
        P.sdtw_forward_f16(q, w.lens, l, r, 0, cost=cost, end_pos=end, variant=best,
                           workspace_buf=ws)
    wall_ms, ev_ms = time_steps(step, steps, warmup, torch)
    peak = valu_peak_gcups(2.5, lanes=64)
    return {"workload": w.name, "dtype": "f16", "cells": w.cells, "ms_per_step": wall_ms,
            "gcups": w.cells / (wall_ms * 1e6), "kernel_ms": ev_ms,
            "variant": P.sdtw_variant_info(best),
            "roofline": {"bound": "alu", "achieved": w.cells / (ev_ms * 1e6), "peak": peak,
                         "unit": "GCUPS", "frac": w.cells / (ev_ms * 1e6) / peak,
                         "peak_basis": "256 CU x 64 lanes/clk (packed FP16 is never "
                                       "dual-issued) x 2.4 GHz / 2.5 VALU ops per cell"}}


def pruned_leg(P, torch, exact_cost, exact_end, steps, warmup):
    """sdtw_forward_pruned (Section 8's early pruning) on the headline
    workload: speed at tau = 2 in the fastest variant (each timed once), and,
    for several tau, how many queries keep their exact cost and end position
    (exact_cost / exact_end: the squared-cost forward's outputs)."""
    import numpy as np

    import workloads
    w = workloads.make_config(1)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    ws = P.workspace(max(P.sdtw_forward_workspace_bytes(w.lens, w.ref_len, 0, v)
                         for v in range(P.sdtw_variant_count())), dev)
    cost = torch.empty(w.batch, dtype=torch.float32, device=dev)
    end = torch.empty(w.batch, dtype=torch.int64, device=dev)
    tau0 = 2.0
    times = {}
    for v in range(P.sdtw_variant_count()):
        def run(v=v):
            P.sdtw_forward_pruned(q, w.lens, l, r, tau0, cost=cost, end_pos=end, variant=v,
                                  workspace_buf=ws)
        times[v] = time_steps(run, 1, 1, torch)[1]
    best = min(times, key=times.get)

    def step():
        P.sdtw_forward_pruned(q, w.lens, l, r, tau0, cost=cost, end_pos=end, variant=best,
                              workspace_buf=ws)
    wall_ms, ev_ms = time_steps(step, steps, warmup, torch)
    peak = valu_peak_gcups(7)
    accuracy = {}
    for tau in (0.5, 1.0, 2.0, 3.0, 4.0):
        P.sdtw_forward_pruned(q, w.lens, l, r, tau, cost=cost, end_pos=end, variant=best,
                              workspace_buf=ws)
        c = cost.cpu().numpy()
        e = end.cpu().numpy()
        same = (c.view(np.uint32) == exact_cost.view(np.uint32)) & (e == exact_end)
        fin = np.isfinite(c)
        pos = fin & (exact_cost > 0)
        accuracy[str(tau)] = {"exact_queries": int(same.sum()), "pruned_to_inf": int((~fin).sum()),
                              "median_cost_ratio": float(np.median(c[pos] / exact_cost[pos]))
                              if pos.any() else None}
    return {"workload": w.name, "tau": tau0, "cells": w.cells, "ms_per_step": wall_ms,
            "gcups": w.cells / (wall_ms * 1e6), "kernel_ms": ev_ms,
            "variant": P.sdtw_variant_info(best),
            "speed_vs_exact_kernel": None,
            "roofline": {"bound": "alu", "achieved": w.cells / (ev_ms * 1e6), "peak": peak,
                         "unit": "GCUPS", "frac": w.cells / (ev_ms * 1e6) / peak,
                         "peak_basis": "256 CU x 128 lanes/clk (VALU dual issue) x 2.4 GHz / "
                                       "7 VALU ops per cell"},
            "accuracy_of_512_queries": accuracy}


def u8_leg(P, torch, exact_cost, exact_end, steps, warmup):
    """sdtw_forward_u8 (Section 8's uint8 codebook quantisation) on the
    headline workload: one call builds the codebook, codes queries and
    reference and runs the integer DP; the fastest variant (each timed once)
    is timed, and its results are compared with the exact FP32 ones
    (exact_cost / exact_end)."""
    import numpy as np

    import workloads
    w = workloads.make_config(1)
    dev = torch.device("cuda:0")
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    ws = P.workspace(P.sdtw_forward_u8_workspace_bytes(w.lens, w.ref_len), dev)
    cost = torch.empty(w.batch, dtype=torch.float32, device=dev)
    end = torch.empty(w.batch, dtype=torch.int64, device=dev)
    book = torch.empty(2, dtype=torch.float32, device=dev)
    times = {}
    for v in range(P.sdtw_variant_count()):
        def run(v=v):
            P.sdtw_forward_u8(q, w.lens, l, r, cost=cost, end_pos=end, codebook=book,
                              variant=v, workspace_buf=ws)
        times[v] = time_steps(run, 1, 1, torch)[1]
    best = min(times, key=times.get)

    def step():
        P.sdtw_forward_u8(q, w.lens, l, r, cost=cost, end_pos=end, codebook=book,
                          variant=best, workspace_buf=ws)
    wall_ms, ev_ms = time_steps(step, steps, warmup, torch)
    lo, hi = (float(x) for x in book.cpu().numpy())
    s2 = ((hi - lo) / 255.0) ** 2
    c = cost.cpu().numpy().astype(np.float64) * s2
    e = end.cpu().numpy()
    if exact_cost is None:
        exact_cost, exact_end = c, e               # timing only: no comparison
    pos = exact_cost > 0
    rel = np.abs(c[pos] - exact_cost[pos]) / exact_cost[pos]
    peak = valu_peak_gcups(3)
    return {"workload": w.name, "cells": w.cells, "ms_per_step": wall_ms,
            "gcups": w.cells / (wall_ms * 1e6), "call_ms": ev_ms,
            "variant": P.sdtw_variant_info(best), "codebook": [lo, hi],
            "speed_vs_exact_kernel": None,
            "roofline": {"bound": "alu", "achieved": w.cells / (ev_ms * 1e6), "peak": peak,
                         "unit": "GCUPS", "frac": w.cells / (ev_ms * 1e6) / peak,
                         "peak_basis": "256 CU x 128 lanes/clk (VALU dual issue) x 2.4 GHz / "
                                       "3 VALU ops per cell (sub, min3, fma); achieved "
                                       "over the whole call (codebook, codes, DP)"},
            "accuracy_of_512_queries": {
                "same_end_pos": int((e == exact_end).sum()),
                "median_rel_cost_error": float(np.median(rel)) if rel.size else None,
                "max_rel_cost_error": float(rel.max()) if rel.size else None}}


def znorm_leg(P, torch, steps, warmup):
    """sdtw_znorm on raw (unnormalised) series of the evaluation's shapes.
    A call takes microseconds, less than the host needs to enqueue it, so
    back-to-back eager calls measure the host; the GPU time per call is taken
    from one HIP graph holding `steps` calls, replayed between events (the
    eager time per call is reported beside it)."""
    import numpy as np

    import workloads
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(240306931)
    sets = {
        "512x2000+100k": [2000] * 512 + [100_000],
        "4096xU[250,4000]": list(rng.integers(250, 4001, 4096)),
        "2M": [2_000_000],
    }
    out = {}
    for name, lens in sets.items():
        x = torch.from_numpy(workloads.raw_series(lens, seed=len(lens))).to(dev)
        h = np.asarray(lens, np.int32)
        lt = torch.from_numpy(h).to(dev)
        z = torch.empty_like(x)
        wsb = P.workspace(P.sdtw_znorm_workspace_bytes(h), dev)

        def run():
            P.sdtw_znorm(x, h, lt, out=z, workspace_buf=wsb)
        wall_ms, ev_ms = time_steps(run, steps, warmup, torch)
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            for _ in range(steps):
                run()
        graph.replay()
        torch.cuda.synchronize()
        reps = 5
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            graph.replay()
        e1.record()
        torch.cuda.synchronize()
        g_ms = e0.elapsed_time(e1) / (reps * steps)
        del graph
        gbs = 8.0 * x.numel() / (g_ms * 1e6)
        out[name] = {"samples": int(x.numel()), "ms": g_ms, "timed": "HIP graph of back-to-back calls",
                     "eager_ms": ev_ms, "eager_wall_ms": wall_ms,
                     "GB/s": gbs, "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    return {"bound": "hbm", "peak_GB/s": HBM_PEAK_GBS,
            "bytes_per_sample": 8, "sets": out}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", type=int, default=-1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the batched and fwd+bwd legs")
    ap.add_argument("--u8-only", action="store_true",
                    help="only time the uint8-code forward (sdtw_forward_u8) and exit")
    ap.add_argument("--znorm-only", action="store_true",
                    help="only time the batch z-normaliser (sdtw_znorm) and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="use the library's built-in variant choice instead of timing all variants")
    ap.add_argument("--leg-only", choices=("batched", "fwd_bwd", "long_ref", "f16"),
                    help="time only this leg (no headline, no oracle) and print its record")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build measures one GPU only; the sDTW batch shards "
                                   "over queries without communication, so run --gpus 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2403_06931_amd as P
    import workloads

    if args.znorm_only:
        print(json.dumps({"znorm": znorm_leg(P, torch, steps=args.steps, warmup=args.warmup)}),
              flush=True)
        return
    if args.u8_only:
        print(json.dumps({"u8": u8_leg(P, torch, None, None, steps=args.steps,
                                       warmup=args.warmup)}), flush=True)
        return
    if args.leg_only:
        if args.leg_only == "long_ref":
            w1 = workloads.make_config(1)
            v = args.variant if args.variant >= 0 else P.sdtw_default_variant(w1.lens, w1.ref_len)
            rec = long_ref_leg(P, torch, v, steps=args.steps, warmup=args.warmup,
                               oracle_legs=False)
        elif args.leg_only == "f16":
            rec = f16_leg(P, torch, steps=args.steps, warmup=args.warmup)
        else:
            fn = batched_leg if args.leg_only == "batched" else fwd_bwd_leg
            rec = fn(P, torch, steps=args.steps, warmup=args.warmup, oracle_legs=False)
        print(json.dumps({args.leg_only: rec}), flush=True)
        return

    dev = torch.device("cuda:0")
    props = torch.cuda.get_device_properties(dev)
    w = workloads.make_config(1)
    q = torch.from_numpy(w.queries).to(dev)
    l = torch.from_numpy(w.lens).to(dev)
    r = torch.from_numpy(w.reference).to(dev)
    cost = torch.empty(w.batch, dtype=torch.float32, device=dev)
    end = torch.empty(w.batch, dtype=torch.int64, device=dev)
    if args.variant >= 0:
        variant = args.variant
    elif args.no_tune:
        variant = P.sdtw_default_variant(w.lens, w.ref_len, 0)
    else:
        variant = P.autotune.tune(q, w.lens, l, r, 0, 0, reps=3)
    ws = P.workspace(P.sdtw_forward_workspace_bytes(w.lens, w.ref_len, 0, variant), dev)

    def step():
        P.sdtw_forward(q, w.lens, l, r, P.SDTW_COST_SQUARED, cost=cost, end_pos=end,
                       variant=variant, workspace_buf=ws)

    progress(f"headline variant {P.sdtw_variant_info(variant)} chosen")
    wall_ms, ev_ms = time_steps(step, args.steps, args.warmup, torch)
    progress(f"headline timed: {ev_ms:.3f} ms per step")
    cells = w.cells
    value = cells / (wall_ms * 1e6)
    achieved = cells / (ev_ms * 1e6)          # GCUPS of the one kernel launch per step
    tflops = achieved * FLOPS_PER_CELL["squared"] / 1e3
    issue_peak = valu_peak_gcups(4)           # GCUPS at 2 VALU instr / SIMD / quad-cycle
    R, T, W, KS, XL = P.sdtw_variant_info(variant)
    gc = cost.cpu().numpy()
    ge = end.cpu().numpy()
    # shader clock while the same launch keeps the GPU busy (outside the timed
    # steps); the roofline at the clock actually run is peak x clock / 2.4 GHz
    sclk = sample_sclk(step, 80, torch)
    at_clk = (PEAK_GHZ / sclk["ghz"]) if sclk else None
    kernel_tag = "sdtw_fwd_512x2000_vs_100k"
    out = {
        "metric": "sDTW GCUPS, 512x2000 queries vs 1e5 reference (FP32, squared cost)",
        "value": value,
        "unit": "GCUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": value / PAPER_GCUPS,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name, "queries": w.batch, "query_len": 2000,
                   "ref_len": w.ref_len, "cost": "squared", "cells": cells,
                   "digest": workloads.digest(w),
                   "variant": {"rows_per_lane": R, "tile_cols": T, "waves": W,
                               "steps_per_barrier": KS,
                               "lane_exchange": "lds" if XL else "dpp"},
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "achieved": tflops, "peak": PEAK_FP32_TFLOPS,
                     "unit": "TFLOP/s", "frac": tflops / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(kernel_tag),
                     "flops_per_cell": FLOPS_PER_CELL["squared"],
                     "peak_basis": "MI355X FP32 vector peak: 256 CUs x 2.4 GHz, an FMA "
                                   "counted as two flops; a cell is 5 flops (sub, mul, "
                                   "two compares, add) in 4 VALU instructions, so this "
                                   "kernel's ceiling on this basis is 5/8 = 0.625",
                     "kernel": f"sdtw_fwd_kernel<{R},{T},{W},{KS},{XL},squared>",
                     "kernel_ms": ev_ms, "gcups": achieved,
                     "issue": {"achieved_gcups": achieved, "peak_gcups": issue_peak,
                               "frac": achieved / issue_peak,
                               "basis": "4 VALU instructions per cell; 256 CUs x 4 SIMDs x "
                                        "16 lanes x 2 instructions per quad-cycle x 2.4 GHz "
                                        "= 78.6 T lane-instructions/s",
                               "single_issue_peak_gcups": valu_peak_gcups(4, lanes=64)},
                     "sclk_measured": sclk,
                     "frac_at_measured_sclk": (tflops / PEAK_FP32_TFLOPS * at_clk)
                     if at_clk else None,
                     "issue_frac_at_measured_sclk": (achieved / issue_peak * at_clk)
                     if at_clk else None,
                     "device_cus": props.multi_processor_count},
        "gsps": float(w.lens.sum()) / (wall_ms * 1e6),
        "gsps_note": "the paper's throughput unit (Eq. (3)): query samples processed "
                     "per second, in 1e9",
    }
    progress(f"clock sampled: {sclk}")
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, gc, ge)
        progress("cpu baseline done")
    if not args.no_extra:
        del ws
        torch.cuda.empty_cache()
        ol = not args.no_cpu_baseline
        out["batched"] = batched_leg(P, torch, steps=3, warmup=1, oracle_legs=ol)
        progress("batched leg done")
        out["fwd_bwd"] = fwd_bwd_leg(P, torch, steps=5, warmup=1, oracle_legs=ol)
        progress("fwd+bwd leg done")
        out["long_ref"] = long_ref_leg(P, torch, variant, steps=2, warmup=1, oracle_legs=ol)
        progress("long-reference leg done")
        out["f16"] = f16_leg(P, torch, steps=5, warmup=1)
        progress("binary16 leg done")
        out["pruned"] = pruned_leg(P, torch, gc, ge, steps=5, warmup=1)
        out["pruned"]["speed_vs_exact_kernel"] = ev_ms / out["pruned"]["kernel_ms"]
        progress("pruned leg done")
        out["u8"] = u8_leg(P, torch, gc, ge, steps=5, warmup=1)
        out["u8"]["speed_vs_exact_kernel"] = ev_ms / out["u8"]["call_ms"]
        progress("uint8 leg done")
        out["znorm"] = znorm_leg(P, torch, steps=20, warmup=3)
        progress("normaliser leg done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
