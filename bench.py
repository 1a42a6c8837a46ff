"""Benchmark: grid points/s per Poisson solve on one MI355X.

Workload (the uniform benchmark configuration): 8x8x8 blocks of 16^3 cells (2,097,152 unknowns),
source = 16 seeded Gaussians (centres uniform in the inner half, widths U[1.5, 4] cells,
amplitudes N(0, 1)), Lagrange order 8.  One step = one complete solve (all FMM levels, both
FFT directions, the spectral MAC, anterpolation/interpolation and, for the FP32 form, the FP64
residual + FP32 re-solve + FP64 update of defect correction) with f and u resident in HBM.

Two forms are timed on the same plan shape: FP64 plain and FP32 + one FP64 defect-correction
iteration.  The headline value is the faster of the two among those within 1e-6 relative L-inf
of the FP64 oracle; both carry the roofline of their dominant kernel.  Extra fields of the same
JSON line: the forward operators, the multi-resolution torus layout (15 M stored unknowns) with
its GPU re-layout and re-plan time, 64 independent layouts in one batched solve, a
Poisson-arrival request stream through the server (p50/p99 latency, HBM budget that binds,
layout-keyed plan cache, a sample of served results checked against the oracle), and the CPU
oracle on the host's cores.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp32_vector_tflops": 157.3, "fp64_vector_tflops": 78.6, "hbm_gbs": 8000.0}
METRIC = "grid points/s per Poisson solve, FP32+refine vs FP64 plain; p50/p99 latency"
HOST_CORES_MAX = 16          # host cores available to one GPU's process


def measured_traffic(name, source):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE summary, or None
    when the kernel source changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_uniform8_nb16.md")
    if not os.path.exists(path):
        return None
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1911_10228_amd", "csrc", source), "rb").read()).hexdigest()
    for line in open(path):
        parts = line.split()
        if len(parts) == 6 and parts[0] == "traffic" and parts[1] == name and parts[5] == sha:
            return float(parts[2])
    return None


def spectrum_size(n_b):
    P = 2 * n_b
    return P * P * (n_b + 1)


def algorithmic(entry, n_b, info, passes):
    """Algorithmic work of one profiled entry (summed over its launches, `passes` solve passes):
    (flops, flop peak in TFLOP/s, compulsory HBM bytes), None where not defined.  MACs: 8 flops
    per complex multiply-add, S per (target, source) pair (work = pairs); a MAC reads each source
    spectrum and each kernel spectrum of its level once and writes each target spectrum once
    (near MAC: the super-block spectra and 14 of the 27 super-block kernels, the others being
    their conjugates; coarse MAC: the block spectra of the coarse levels and 172 of the 316
    kernels per level, likewise).  The fused near step (modes 42, 44) reads the line-major
    planes of every source super-block (half a spectrum: B2 values of z per line) and the 14
    kernel columns (a full spectrum each) and writes the planes of every target super-block;
    its flops are counted as those of the MAC alone.  FP32 tiles compute in FP32; FP64 spectra
    in FP64.  Transforms: per item (work = items) the block or the 8 child blocks of a
    super-block, and the half spectrum (2 S reals), or for the line-major super-block passes
    (mode 1) the planes (S2 reals)."""
    es = 4 if entry["precision"] == "fp32" else 8
    esc = 4 if entry["precision"] in ("fp32", "fp32/fp64") else 8     # child blocks
    S, S2 = spectrum_size(n_b), spectrum_size(2 * n_b)
    N3 = n_b ** 3
    k, mode = entry["kernel"], entry.get("mode", 0)
    peak = PEAK["fp32_vector_tflops"] if entry["precision"] == "fp32" else PEAK["fp64_vector_tflops"]
    if k == "mac":
        levels = (info["spectra"] - (27 if info["super_forward"] else 343)) // 316
        per_pass = (info["fft_forward"] + info["fft_inverse"] + 172 * levels) * 2 * S * es
        return 8.0 * S * entry["work"], peak, per_pass * passes
    if k == "near_mac" and mode in (42, 44):
        per_launch = (info["super_forward"] + info["super_inverse"]) * S2 * es + 14 * 2 * S2 * es
        return 8.0 * S2 * entry["work"], peak, per_launch * entry["launches"]
    if k == "near_mac":
        per_launch = (info["super_forward"] + info["super_inverse"] + 14) * 2 * S2 * es
        return 8.0 * S2 * entry["work"], peak, per_launch * entry["launches"]
    if k in ("fft_fwd", "fft_inv"):
        return None, None, float(entry["work"]) * (N3 * es + 2 * S * es)
    if k in ("super_fwd", "super_inv"):
        planes = S2 * es if mode == 1 else 2 * S2 * es
        return None, None, float(entry["work"]) * (8 * N3 * esc + planes)
    return None, None, None


def time_solves(plan, f, u, steps, warmup, torch, stream):
    """Seconds per solve on a non-default stream (repeat solves replay a captured graph)."""
    for _ in range(warmup):
        plan.solve(f, u, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        plan.solve(f, u, stream=stream)
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps


def profiled(lgf, plan, f, u, steps, torch, stream):
    """Per-kernel HIP-event times over `steps` solves (direct launches on the given stream,
    events recorded on that stream around each kernel, which runs alone)."""
    lgf.profile_read()
    lgf.profile(True)
    for _ in range(steps):
        plan.solve(f, u, stream=stream)
    torch.cuda.synchronize()
    lgf.profile(False)
    return lgf.profile_read()


def roofline_of(prof, n_b, info, passes):
    """Per-kernel table and the roofline block of the dominant kernel (largest total time):
    the larger of the HBM time of its compulsory bytes and the ALU time of its flops, over the
    measured time."""
    kern = []
    for e in prof:
        flops, fpeak, nbytes = algorithmic(e, n_b, info, passes)
        e = dict(e, avg_us=1e3 * e["ms"] / max(e["launches"], 1))
        t = e["ms"] * 1e-3
        if flops is not None:
            e.update(flops_per_launch=flops / e["launches"], tflops=flops / t / 1e12, flop_peak=fpeak)
        if nbytes is not None:
            e.update(bytes_per_launch=nbytes / e["launches"], gbs=nbytes / t / 1e9)
        kern.append(e)
    kern.sort(key=lambda e: -e["ms"])
    dom = kern[0]
    tag = f"{dom['kernel']}_{dom['precision']}_nb{dom['n_b']}_mode{dom.get('mode', 0)}"
    src = {"mac": "mac.hip", "near_mac": "mac.hip", "fft_fwd": "fft_blocks.hip", "fft_inv": "fft_blocks.hip",
           "super_fwd": "fft_super.hip", "super_inv": "fft_super.hip"}.get(dom["kernel"])
    traffic = measured_traffic(tag, src) if src else None
    t_hbm = dom["bytes_per_launch"] / (PEAK["hbm_gbs"] * 1e9) if "bytes_per_launch" in dom else 0.0
    t_alu = dom["flops_per_launch"] / (dom["flop_peak"] * 1e12) if "flops_per_launch" in dom else 0.0
    name = f"{dom['kernel']} ({dom['precision']} storage, n_b={dom['n_b']}, launch shape {dom.get('mode', 0)})"
    if t_hbm == 0.0 and t_alu == 0.0:
        roof = {"bound": "hbm", "achieved": None, "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": None,
                "traffic": traffic, "kernel": name}
    elif t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": round(dom["gbs"] / PEAK["hbm_gbs"], 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(dom["avg_us"], 2), "bytes_per_launch": dom["bytes_per_launch"],
                "alu": {"achieved_tflops": round(dom.get("tflops", 0.0), 3), "peak": dom.get("flop_peak")}}
    else:
        roof = {"bound": "alu", "achieved": round(dom["tflops"], 3), "peak": dom["flop_peak"], "unit": "TFLOP/s",
                "frac": round(dom["tflops"] / dom["flop_peak"], 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(dom["avg_us"], 2)}
    table = [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in e.items()} for e in kern]
    return roof, table


def bench_fwd_ops(lgf, plan, m, torch, stream, reps=20):
    """lgf_apply (Laplacian, gradient, curl) on the bench layout: microseconds per launch from HIP
    events on the launch stream around `reps` back-to-back launches, and the algorithmic HBM bytes
    (every input component read once, every output component written once, 8 bytes a value) over
    that time."""
    res = {}
    for op, name, nin, nout in ((lgf.LAPLACIAN, "laplacian", 1, 1), (lgf.GRADIENT, "gradient", 1, 3),
                                (lgf.CURL, "curl", 3, 3)):
        x = torch.randn(nin * m, dtype=torch.float64, device="cuda")
        y = torch.empty(nout * m, dtype=torch.float64, device="cuda")
        for _ in range(3):
            plan.apply(op, x, y, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            plan.apply(op, x, y, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        us = e0.elapsed_time(e1) * 1e3 / reps
        gbs = 8.0 * (nin + nout) * m / us / 1e3
        res[name] = {"us": round(us, 2), "GB/s": round(gbs, 1), "frac_hbm_peak": round(gbs / 8000.0, 3)}
    return res


def bench_torus(lgf, workloads, torch, stream, steps, warmup, dc):
    """Multi-resolution solve of the torus layout (8^3 base blocks of 16^3, two refinement
    levels): grid points (all stored unknowns) per second, FP32 + DC and FP64 plain.  Also the
    adaptation of the layout on the GPU (two steps of the refinement criterion from the base
    blocks, the field evaluated on each new layout on the host and uploaded, not timed) and the
    plan of the new layout (the kernel spectra and tuned launch shapes are resident)."""
    L = workloads.torus()
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    out = {"layout": f"{L.name}, {len(L.blocks)} blocks", "unknowns": L.unknowns}
    res = {}
    for name, prec, k in (("fp32_dc", lgf.LGF_FP32_REFINE, dc), ("fp64_plain", lgf.LGF_FP64_PLAIN, 0)):
        p = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, prec, k, autotune=1)
        u = torch.zeros_like(f)
        dt = time_solves(p, f, u, steps, warmup, torch, stream)
        res[name] = u.cpu().numpy()
        out[name] = {"value": L.unknowns / dt, "ms_per_step": dt * 1e3}
        p.close()
    out["fp32_dc"]["diff_vs_fp64_plain"] = float(np.abs(res["fp32_dc"] - res["fp64_plain"]).max()
                                                 / np.abs(res["fp64_plain"]).max())
    # re-layout and re-plan
    m = L.meta
    src = lambda b, lv: workloads.torus_source(workloads.cell_centres(b, lv, L.n_b), m["centre"], m["axis"],
                                               m["R"], m["sigma"])[0]
    blocks = workloads.box_blocks(8, 8, 8).astype(np.int32)
    levels = np.zeros(len(blocks), np.int32)
    adapt_ms = []
    for _ in range(2):
        field = torch.from_numpy(np.ascontiguousarray(src(blocks, levels))).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        blocks, levels = lgf.adapt_layout(blocks, levels, L.n_b, field, 3)
        adapt_ms.append((time.perf_counter() - t0) * 1e3)
    t0 = time.perf_counter()
    p = lgf.Plan(blocks, levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, dc, autotune=1)
    plan_ms = (time.perf_counter() - t0) * 1e3
    p.close()
    out["replan"] = {"adapt_ms_per_step": [round(x, 2) for x in adapt_ms], "plan_ms": round(plan_ms, 1),
                     "same_layout_as_generator": bool(np.array_equal(blocks, L.blocks)
                                                      and np.array_equal(levels, L.levels))}
    return out


def bench_batch(lgf, workloads, torch, stream, steps, warmup, dc):
    """64 independent layouts in one batched solve (shared launches, captured graph replays),
    FP32 + DC with autotuned MAC launch shapes: aggregate grid points per second."""
    Ls = workloads.batch()
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, dc, autotune=1)
             for L in Ls]
    fs = [torch.from_numpy(np.ascontiguousarray(L.f)).cuda() for L in Ls]
    us = [torch.zeros_like(f) for f in fs]
    for _ in range(warmup):
        lgf.solve_batch(plans, fs, us, stream=stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        lgf.solve_batch(plans, fs, us, stream=stream)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    total = sum(L.unknowns for L in Ls)
    for p in plans:
        p.close()
    return {"solves": len(Ls), "unknowns": total, "value": total / dt, "ms_per_batch": dt * 1e3}


def bench_serving(lgf, workloads, torch, capacity_pts, dc, count=1000, pool_size=48, check=True):
    """Poisson-arrival request stream through the continuous-batching server.  Requests name one
    of `pool_size` layouts (4096 .. 16.7M unknowns, log-uniform; popular layouts more often,
    weight 1 / (rank + 1)) and bring a source; the server resolves the layout through its plan
    cache (planned on first sight) and admits requests as workspace slots fit a budget of a
    quarter of the pool's workspaces.  The rate offers 0.7 of the measured batched capacity.  A
    warm-up pass plans every layout once (plan-build times reported); latency = completion -
    arrival over the timed stream, on the same server (plans cached, memory reserved).  A seeded sample of served results is checked against the
    FP64 oracle's defect correction (FP64 inner solves, the same iteration count)."""
    pool = workloads.request_pool(count=pool_size)
    ws = [lgf.plan_check(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, dc)["workspace_bytes"]
          for L in pool]
    budget = max(sum(ws) // 4, max(ws) + (1 << 20))
    fs = [torch.from_numpy(np.ascontiguousarray(L.f)).cuda() for L in pool]
    us = [torch.zeros_like(f) for f in fs]
    srv = lgf.Server(hbm_budget=budget, stream=torch.cuda.Stream())
    for L, f, u in zip(pool, fs, us):                       # warm-up: every layout planned once
        srv.submit_layout(L.blocks, L.levels, L.n_b, L.interp_order, f, u, lgf.LGF_FP32_REFINE, dc)
    srv.wait_all()
    warm = srv.info()
    rng = np.random.default_rng(5)
    order = rng.permutation(len(pool))
    weight = 1.0 / (np.arange(len(pool)) + 1.0)
    which = order[rng.choice(len(pool), size=count, p=weight / weight.sum())]
    mean_pts = float(np.mean([pool[k].unknowns for k in which]))
    rate = 0.7 * capacity_pts / mean_pts
    times, _ = workloads.arrivals(seed=5, count=count, rate_hz=rate)
    # the sample to check: the first three requests of layouts up to 300k unknowns, each with an
    # output of its own (other requests of one layout share one output buffer)
    small = [i for i, k in enumerate(which) if pool[k].unknowns <= 300_000][:3]
    own = {i: torch.zeros_like(fs[which[i]]) for i in small}
    srv.reset_stats()
    t0 = time.perf_counter()
    for i, (t, k) in enumerate(zip(times, which)):
        while time.perf_counter() - t0 < t:
            pass
        L = pool[k]
        srv.submit_layout(L.blocks, L.levels, L.n_b, L.interp_order, fs[k], own.get(i, us[k]),
                          lgf.LGF_FP32_REFINE, dc)
    srv.wait_all()
    st, info = srv.stats(), srv.info()
    srv.close()
    out = {"requests": count, "rate_hz": rate, "layouts": len(pool), "hbm_budget_bytes": int(budget),
           "pool_workspace_bytes": int(sum(ws)), "p50_ms": st["p50_us"] / 1e3, "p99_ms": st["p99_us"] / 1e3,
           "value": st["points_per_s"], "unit": "grid points/s",
           "peak_slots": info["peak_slots"], "peak_in_use_bytes": info["peak_in_use_bytes"],
           "reserved_bytes": info["reserved_bytes"], "slot_binds": info["binds"],
           "plan_cache": {"hits": info["plan_hits"], "misses": info["plan_misses"],
                          "planned_in_warmup": warm["plan_misses"]},
           "plan_build_ms": {"mean": warm["plan_ms_total"] / max(warm["plan_misses"], 1),
                             "max": warm["plan_ms_max"], "layouts": warm["plan_misses"]},
           "pool": f"{len(pool)} layouts, 4096..16.7M unknowns log-uniform, n_b 8/16, 1..3 levels"}
    if check and small:
        from oracle import dc as dc_oracle
        errs = []
        for i in small:
            L = pool[which[i]]
            ref = dc_oracle.solve_dc(L.blocks, L.levels, L.f, L.n_b, L.interp_order, iters=dc,
                                     dtype=np.float64)[dc]
            got = own[i].cpu().numpy()
            errs.append(float(np.abs(got - ref).max() / np.abs(ref).max()))
        out["checked"] = {"requests": small, "unknowns": [pool[which[i]].unknowns for i in small],
                          "err_vs_oracle_dc": errs}
    return out


def _oracle_worker(args):
    """One FP64 oracle solve of the bench workload in a process of its own: (start, end) times."""
    n_b, nblk, order = args
    from oracle import fmm
    from paper_1911_10228_amd import workloads
    L = workloads.uniform_mixture(nblk=nblk, n_b=n_b, n_gauss=16, seed=2, interp_order=order)
    t0 = time.time()
    fmm.flgf(L.blocks, L.f, L.n_b, order)
    return t0, time.time(), L.unknowns


def cpu_baseline(n_b=16, nblk=8, order=8):
    """The FP64 oracle as it stands on the host's cores: one solve of the bench workload per
    process, as many processes as cores in parallel (len(os.sched_getaffinity(0)), at most the
    box's CPU share); value = unknowns solved / wall time.  Also returns the oracle's solution
    and, untimed, its one-step defect correction with an FP64 inner solve (the FP32 + DC form's
    reference)."""
    import concurrent.futures as cf
    import multiprocessing as mp
    from oracle import fmm, multires
    from paper_1911_10228_amd import workloads
    cores = max(1, min(len(os.sched_getaffinity(0)), HOST_CORES_MAX))
    with cf.ProcessPoolExecutor(max_workers=cores, mp_context=mp.get_context("spawn")) as ex:
        runs = list(ex.map(_oracle_worker, [(n_b, nblk, order)] * cores))
    wall = max(r[1] for r in runs) - min(r[0] for r in runs)
    solved = sum(r[2] for r in runs)
    L = workloads.uniform_mixture(nblk=nblk, n_b=n_b, n_gauss=16, seed=2, interp_order=order)
    u = fmm.flgf(L.blocks, L.f, L.n_b, order)
    mask = multires.residual_mask(L.blocks, L.levels, L.n_b)
    r = np.where(mask, L.f - multires.apply_laplace(L.blocks, L.levels, u, L.n_b), 0.0)
    u1 = u + fmm.flgf(L.blocks, r, L.n_b, order)
    res = {"value": solved / wall, "unit": "grid points/s", "cores": cores, "kind": "oracle",
           "sample": f"{cores} FP64 oracle solves of {nblk}^3 blocks of {n_b}^3 ({L.unknowns} unknowns each, "
                     f"same recipe, order {order}), one per process, in {wall:.1f} s wall"}
    return res, u, u1


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--dc", type=int, default=1, help="defect-correction iterations of the FP32 form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the torus, 64-layout batch and serving measurements")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch every kernel directly (no captured-graph replays), for profilers")
    ap.add_argument("--serial", action="store_true",
                    help="one stream per solve (no base-level/far-field overlap), so that a "
                         "profiler's kernel durations are those of kernels running alone")
    ap.add_argument("--profiler-exit", action="store_true",
                    help="end through the interpreter's normal exit (a profiler such as rocprofv3 "
                         "writes its results there) instead of exiting at once")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device-to-device copy 3 times (counter calibration)")
    ap.add_argument("--torus-only", action="store_true",
                    help="only plan the multi-resolution torus layout (FP64 plain, then FP32 + DC; "
                         "autotuned) and solve it --steps times with each plan, then exit: a "
                         "kernel profile of the refined levels")
    ap.add_argument("--timeline", action="store_true",
                    help="only plan, then replay 8 FP64 plain and 8 FP32 + DC solves as the timed "
                         "region does (captured graphs, two streams) and exit: a kernel trace of "
                         "the overlapped solve for a profiler")
    args = ap.parse_args()
    if args.no_graph:
        os.environ["LGF_NO_GRAPH"] = "1"
    if args.serial:
        os.environ["LGF_NO_FORK"] = "1"
    if args.copy_calibration:
        import torch
        a = torch.empty(64 << 20, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_each_way": a.numel() * 8, "copies": 3}))
        return args
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library solves on a "
              "single GPU and has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_10228_amd import lgf, workloads

    torch.cuda.set_device(0)
    if args.torus_only:
        T = workloads.torus()
        ft = torch.from_numpy(np.ascontiguousarray(T.f)).cuda()
        ut = torch.zeros_like(ft)
        st = torch.cuda.Stream()
        for precision, dc in ((lgf.LGF_FP64_PLAIN, 0), (lgf.LGF_FP32_REFINE, args.dc)):
            p = lgf.Plan(T.blocks, T.levels, T.n_b, T.interp_order, precision, dc, autotune=1)
            print(f"# torus plan (precision {precision}, dc {dc}): {p.info()}", file=sys.stderr, flush=True)
            for _ in range(args.steps):
                p.solve(ft, ut, stream=st)
            torch.cuda.synchronize()
            p.close()
        return args
    L = workloads.uniform_mixture(nblk=8, n_b=16, n_gauss=16, seed=2, interp_order=8)
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    u32, u64, u0 = torch.zeros_like(f), torch.zeros_like(f), torch.zeros_like(f)
    # launch shapes chosen by the plan-time autotuner
    p32 = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, args.dc, autotune=1)
    p64 = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP64_PLAIN, 0, autotune=1)
    p0 = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, 0, autotune=1)
    info32, info64 = p32.info(), p64.info()
    print(f"# plan: {info32}", file=sys.stderr, flush=True)

    stream = torch.cuda.Stream()
    if args.timeline:
        for p, u in ((p64, u64), (p32, u32)):
            for _ in range(8):
                p.solve(f, u, stream=stream)
        torch.cuda.synchronize()
        for p in (p32, p64, p0):
            p.close()
        return args
    dt32 = time_solves(p32, f, u32, args.steps, args.warmup, torch, stream)
    print(f"# fp32+dc{args.dc}: {dt32 * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    dt64 = time_solves(p64, f, u64, args.steps, args.warmup, torch, stream)
    print(f"# fp64 plain: {dt64 * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    dt0 = time_solves(p0, f, u0, args.steps, args.warmup, torch, stream)
    print(f"# fp32 no dc: {dt0 * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    # per-kernel event times of both forms (kernels running alone)
    prof32 = profiled(lgf, p32, f, u32, args.steps, torch, stream)
    prof64 = profiled(lgf, p64, f, u64, args.steps, torch, stream)
    # the same FP32 + DC solve with the per-block base level (the paper's block convolutions)
    pb = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, args.dc,
                  base_level=lgf.LGF_BASE_BLOCK)
    ub = torch.zeros_like(f)
    dtb = time_solves(pb, f, ub, args.steps, args.warmup, torch, stream)
    print(f"# fp32+dc{args.dc}, per-block base level: {dtb * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    pb.close()

    a32, a64, a0 = u32.cpu().numpy(), u64.cpu().numpy(), u0.cpu().numpy()

    def rel(a, b):
        return float(np.abs(a - b).max() / np.abs(b).max())

    roof32, kern32 = roofline_of(prof32, L.n_b, info32, args.steps * (1 + args.dc))
    roof64, kern64 = roofline_of(prof64, L.n_b, info64, args.steps)
    forms = {
        "fp64_plain": {"value": L.unknowns / dt64, "ms_per_step": dt64 * 1e3, "dtype": "f64",
                       "precision": "FP64 FFTs, MAC and operators", "roofline": roof64, "kernels": kern64},
        "fp32_dc": {"value": L.unknowns / dt32, "ms_per_step": dt32 * 1e3, "dtype": "f32",
                    "precision": f"FP32 base-level FFT/MAC, FP64 far field, {args.dc} FP64 DC iteration(s)",
                    "err_vs_fp64": rel(a32, a64), "roofline": roof32, "kernels": kern32},
    }
    extra = {"fp32_no_dc": {"value": L.unknowns / dt0, "ms_per_step": dt0 * 1e3, "err_vs_fp64": rel(a0, a64)},
             "fp32_block_base": {"value": L.unknowns / dtb, "ms_per_step": dtb * 1e3,
                                 "err_vs_fp64": rel(ub.cpu().numpy(), a64)}}

    out_extra = {}
    if not args.no_extra:
        out_extra["forward_ops"] = bench_fwd_ops(lgf, p64, u64.numel(), torch, stream)
        print(f"# forward ops (FP64, bench layout): {out_extra['forward_ops']}", file=sys.stderr, flush=True)
        out_extra["multires_torus"] = bench_torus(lgf, workloads, torch, stream, max(args.steps // 4, 3), 1,
                                                  args.dc)
        print(f"# torus: {out_extra['multires_torus']}", file=sys.stderr, flush=True)
        out_extra["batch64"] = bench_batch(lgf, workloads, torch, stream, max(args.steps // 4, 3), 1, args.dc)
        print(f"# batch64: {out_extra['batch64']}", file=sys.stderr, flush=True)
        out_extra["serving"] = bench_serving(lgf, workloads, torch, out_extra["batch64"]["value"], args.dc,
                                             check=not args.no_cpu)
        print(f"# serving: {out_extra['serving']}", file=sys.stderr, flush=True)
    for p in (p32, p64, p0):
        p.close()

    errs = None
    if not args.no_cpu:
        out_extra["cpu_baseline"], uo, uo1 = cpu_baseline()
        # every form against the oracle on the bench workload (FP32 + DC against the oracle's
        # own defect-correction step)
        errs = {"fp64_plain": rel(a64.reshape(uo.shape), uo), "fp32_no_dc": rel(a0.reshape(uo.shape), uo),
                "fp32_dc": rel(a32.reshape(uo.shape), uo1)}
        out_extra["err_vs_oracle"] = errs
        print(f"# err vs oracle: {errs}", file=sys.stderr, flush=True)
    # headline: the faster of the two forms among those within 1e-6 of the oracle (without the
    # oracle: of the FP64 GPU solve, for the FP32 form)
    ok = {k: (errs[k] if errs else (0.0 if k == "fp64_plain" else forms[k]["err_vs_fp64"])) <= 1e-6 for k in forms}
    head = min((k for k in forms if ok[k]), key=lambda k: forms[k]["ms_per_step"])
    other = "fp32_dc" if head == "fp64_plain" else "fp64_plain"
    H = forms[head]
    out = {
        "metric": METRIC,
        "value": H["value"],
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": H["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": H["dtype"],
        "data": "synthetic",
        "config": {"workload": "uniform 8x8x8 blocks of 16^3 (2,097,152 unknowns), 16 seeded "
                               "Gaussians, Lagrange order 8",
                   "form": head, "precision": H["precision"],
                   "base_level": "parent super-blocks (2 N_b cells, FFT size 4 N_b)"},
        "roofline": H["roofline"],
        "headline_rule": "the faster of fp64_plain and fp32_dc among those within 1e-6 relative L-inf of the oracle",
        head: {k: v for k, v in H.items() if k not in ("roofline", "kernels")},
        other: {k: v for k, v in forms[other].items() if k != "kernels"},
        "kernels": {head: H["kernels"], other: forms[other]["kernels"]},
    }
    out.update(extra)
    out.update(out_extra)
    print(json.dumps(out), flush=True)
    return args


if __name__ == "__main__":
    a = main()
    sys.stdout.flush()
    sys.stderr.flush()
    # end at once: no library or runtime teardown left running after the result is printed
    if a is None or not a.profiler_exit:
        os._exit(0)
