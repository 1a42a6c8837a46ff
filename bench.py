"""Benchmark: grid points/s per Poisson solve on one MI355X.

Workload (the uniform benchmark configuration): 8x8x8 blocks of 16^3 cells (2,097,152 unknowns),
source = 16 seeded Gaussians (centres uniform in the inner half, widths U[1.5, 4] cells,
amplitudes N(0, 1)), Lagrange order 8.  One step = one complete solve (all FMM levels, both
FFT directions, the spectral MAC, anterpolation/interpolation and, for the FP32 form, the FP64
residual + FP32 re-solve + FP64 update of defect correction) with f and u resident in HBM.

Headline value: FP32 FFT/MAC on the base octree level (FP64 on the coarse far-field levels)
with one FP64 defect-correction iteration.  The FP64 plain solve of the same plan shape is timed
beside it, and so are, as extra fields of the same JSON line: the multi-resolution torus layout
(15.5M stored unknowns), 64 independent layouts in one batched solve, and a Poisson-arrival
request stream through the server (p50/p99 latency).  Prints one JSON line.
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
    kernels per level, likewise).  FP32 tiles compute in FP32;
    FP64 spectra in FP64.  Transforms: per item (work = items) the block or the 8 child blocks
    of a super-block, and the half spectrum (2 S reals)."""
    es = 4 if entry["precision"] == "fp32" else 8
    S, S2 = spectrum_size(n_b), spectrum_size(2 * n_b)
    N3 = n_b ** 3
    k = entry["kernel"]
    peak = PEAK["fp32_vector_tflops"] if entry["precision"] == "fp32" else PEAK["fp64_vector_tflops"]
    if k == "mac":
        # 172 of each coarse level's 316 kernel spectra (d >= 0; the others are conjugates)
        levels = (info["spectra"] - (27 if info["super_forward"] else 343)) // 316
        per_pass = (info["fft_forward"] + info["fft_inverse"] + 172 * levels) * 2 * S * es
        return 8.0 * S * entry["work"], peak, per_pass * passes
    if k == "near_mac":
        per_launch = (info["super_forward"] + info["super_inverse"] + 14) * 2 * S2 * es
        return 8.0 * S2 * entry["work"], peak, per_launch * entry["launches"]
    if k in ("fft_fwd", "fft_inv"):
        return None, None, float(entry["work"]) * (N3 * es + 2 * S * es)
    if k in ("super_fwd", "super_inv"):
        return None, None, float(entry["work"]) * (8 * N3 * es + 2 * S2 * es)
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


def profiled(lgf, plan, f, u, steps, torch, stream):
    """Per-kernel HIP-event times over `steps` solves (direct launches on one stream: events
    bracket each kernel running alone)."""
    lgf.profile_read()
    lgf.profile(True)
    for _ in range(steps):
        plan.solve(f, u, stream=stream)
    torch.cuda.synchronize()
    lgf.profile(False)
    return lgf.profile_read()


def bench_torus(lgf, workloads, torch, stream, steps, warmup, dc):
    """Multi-resolution solve of the torus layout (8^3 base blocks of 16^3, two refinement
    levels): grid points (all stored unknowns) per second, FP32 + DC and FP64 plain."""
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


def bench_serving(lgf, workloads, torch, capacity_pts, dc, count=1000):
    """Poisson-arrival request stream through the continuous-batching server: requests draw a
    layout from a pool of 24 (4096 .. 16.7M unknowns, log-uniform) and bring a source; the rate
    offers 0.7 of the measured batched capacity; latency = completion - arrival."""
    pool = workloads.request_pool(count=24)
    plans = [lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, dc) for L in pool]
    fs = [torch.from_numpy(np.ascontiguousarray(L.f)).cuda() for L in pool]
    mean_pts = float(np.mean([L.unknowns for L in pool]))
    rate = 0.7 * capacity_pts / mean_pts
    times, _ = workloads.arrivals(seed=5, count=count, rate_hz=rate)
    which = np.random.default_rng(5).integers(0, len(pool), size=count)
    us = [torch.zeros_like(f) for f in fs]
    budget = 200 << 30
    srv = lgf.Server(hbm_budget=budget, stream=torch.cuda.Stream())
    t0 = time.perf_counter()
    for t, k in zip(times, which):
        while time.perf_counter() - t0 < t:
            pass
        srv.submit(plans[k], fs[k], us[k])
    srv.wait_all()
    st = srv.stats()
    srv.close()
    for p in plans:
        p.close()
    return {"requests": count, "rate_hz": rate, "hbm_budget_bytes": budget, "p50_ms": st["p50_us"] / 1e3,
            "p99_ms": st["p99_us"] / 1e3, "value": st["points_per_s"], "unit": "grid points/s",
            "pool": "24 layouts, 4096..16.7M unknowns log-uniform, n_b 8/16, 1..3 levels"}


def cpu_baseline(n_b=16, nblk=8, order=8):
    """The FP64 oracle, single-threaded, on a bounded sample of the same workload recipe (here
    the whole bench workload: one solve).  Also returns the oracle's solution and, untimed, its
    one-step defect correction with an FP64 inner solve (the FP32 + DC form's reference)."""
    from threadpoolctl import threadpool_limits
    from oracle import fmm, multires
    from paper_1911_10228_amd import workloads
    L = workloads.uniform_mixture(nblk=nblk, n_b=n_b, n_gauss=16, seed=2, interp_order=order)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        u = fmm.flgf(L.blocks, L.f, L.n_b, order)
        dt = time.perf_counter() - t0
        mask = multires.residual_mask(L.blocks, L.levels, L.n_b)
        r = np.where(mask, L.f - multires.apply_laplace(L.blocks, L.levels, u, L.n_b), 0.0)
        u1 = u + fmm.flgf(L.blocks, r, L.n_b, order)
    res = {"value": L.unknowns / dt, "unit": "grid points/s", "cores": 1, "kind": "oracle",
           "sample": f"one FP64 oracle solve of {nblk}^3 blocks of {n_b}^3 ({L.unknowns} unknowns, "
                     f"same recipe, order {order}) in {dt:.1f} s"}
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
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 512 MiB device-to-device copy 3 times (counter calibration)")
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
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library solves on a "
              "single GPU and has no multi-GPU sharding", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1911_10228_amd import lgf, workloads

    torch.cuda.set_device(0)
    L = workloads.uniform_mixture(nblk=8, n_b=16, n_gauss=16, seed=2, interp_order=8)
    f = torch.from_numpy(np.ascontiguousarray(L.f)).cuda()
    u32 = torch.zeros_like(f)
    u64 = torch.zeros_like(f)
    u0 = torch.zeros_like(f)
    # launch shapes chosen by the plan-time autotuner
    p32 = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, args.dc, autotune=1)
    p64 = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP64_PLAIN, 0, autotune=1)
    p0 = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, 0, autotune=1)
    info = p32.info()
    print(f"# plan: {info}", file=sys.stderr, flush=True)

    stream = torch.cuda.Stream()
    # headline: FP32 + DC; then the same number of solves with every kernel bracketed by events
    dt32 = time_solves(p32, f, u32, args.steps, args.warmup, torch, stream)
    print(f"# fp32+dc{args.dc}: {dt32 * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    prof = profiled(lgf, p32, f, u32, args.steps, torch, stream)
    dt64 = time_solves(p64, f, u64, args.steps, args.warmup, torch, stream)
    print(f"# fp64 plain: {dt64 * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    dt0 = time_solves(p0, f, u0, args.steps, args.warmup, torch, stream)
    print(f"# fp32 no dc: {dt0 * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)
    # the same FP32 + DC solve with the per-block base level (the paper's block convolutions)
    pb = lgf.Plan(L.blocks, L.levels, L.n_b, L.interp_order, lgf.LGF_FP32_REFINE, args.dc,
                  base_level=lgf.LGF_BASE_BLOCK)
    ub = torch.zeros_like(f)
    dtb = time_solves(pb, f, ub, args.steps, args.warmup, torch, stream)
    print(f"# fp32+dc{args.dc}, per-block base level: {dtb * 1e3:.3f} ms/solve", file=sys.stderr, flush=True)

    a32, a64, a0 = u32.cpu().numpy(), u64.cpu().numpy(), u0.cpu().numpy()
    err32 = float(np.abs(a32 - a64).max() / np.abs(a64).max())
    err0 = float(np.abs(a0 - a64).max() / np.abs(a64).max())
    errb = float(np.abs(ub.cpu().numpy() - a64).max() / np.abs(a64).max())

    # dominant kernel of the headline form (per-launch event times of kernels running alone);
    # its roofline is the larger of the HBM time of its compulsory bytes and the ALU time of its
    # flops, over the measured time
    kern = []
    for e in prof:
        flops, fpeak, nbytes = algorithmic(e, L.n_b, info, args.steps * (1 + args.dc))
        e = dict(e, avg_us=1e3 * e["ms"] / max(e["launches"], 1))
        t = e["ms"] * 1e-3
        if flops is not None:
            e.update(flops_per_launch=flops / e["launches"], tflops=flops / t / 1e12, flop_peak=fpeak)
        if nbytes is not None:
            e.update(bytes_per_launch=nbytes / e["launches"], gbs=nbytes / t / 1e9)
        kern.append(e)
    kern.sort(key=lambda e: -e["ms"])
    dom = kern[0]
    tag = f"{dom['kernel']}_{dom['precision']}_nb{dom['n_b']}"
    src = {"mac": "mac.hip", "near_mac": "mac.hip", "fft_fwd": "fft_blocks.hip", "fft_inv": "fft_blocks.hip",
           "super_fwd": "fft_super.hip", "super_inv": "fft_super.hip"}.get(dom["kernel"])
    traffic = measured_traffic(tag, src) if src else None
    t_hbm = dom["bytes_per_launch"] / (PEAK["hbm_gbs"] * 1e9) if "bytes_per_launch" in dom else 0.0
    t_alu = dom["flops_per_launch"] / (dom["flop_peak"] * 1e12) if "flops_per_launch" in dom else 0.0
    name = f"{dom['kernel']} ({dom['precision']} storage, n_b={dom['n_b']})"
    if t_hbm == 0.0 and t_alu == 0.0:
        roof = {"bound": "hbm", "achieved": None, "peak": PEAK["hbm_gbs"], "unit": "GB/s", "frac": None,
                "traffic": traffic, "kernel": name}
    elif t_hbm >= t_alu:
        roof = {"bound": "hbm", "achieved": round(dom["gbs"], 1), "peak": PEAK["hbm_gbs"], "unit": "GB/s",
                "frac": round(dom["gbs"] / PEAK["hbm_gbs"], 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(dom["avg_us"], 2),
                "alu": {"achieved_tflops": round(dom.get("tflops", 0.0), 3), "peak": dom.get("flop_peak")}}
    else:
        roof = {"bound": "alu", "achieved": round(dom["tflops"], 3), "peak": dom["flop_peak"], "unit": "TFLOP/s",
                "frac": round(dom["tflops"] / dom["flop_peak"], 4), "traffic": traffic, "kernel": name,
                "avg_launch_us": round(dom["avg_us"], 2)}

    out = {
        "metric": "grid points/s per Poisson solve (FP32+refine; FP64 plain beside it)",
        "value": L.unknowns / dt32,
        "unit": "grid points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "uniform 8x8x8 blocks of 16^3 (2,097,152 unknowns), 16 seeded "
                               "Gaussians, Lagrange order 8",
                   "precision": f"FP32 base-level FFT/MAC, FP64 far field, {args.dc} FP64 DC iteration(s)",
                   "base_level": "parent super-blocks (2 N_b cells, FFT size 4 N_b)"},
        "roofline": roof,
        "fp64_plain": {"value": L.unknowns / dt64, "ms_per_step": dt64 * 1e3},
        "fp32_no_dc": {"value": L.unknowns / dt0, "ms_per_step": dt0 * 1e3, "err_vs_fp64": err0},
        "fp32_block_base": {"value": L.unknowns / dtb, "ms_per_step": dtb * 1e3, "err_vs_fp64": errb},
        "err_vs_fp64": err32,
        "kernels": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in e.items()} for e in kern],
    }
    if not args.no_extra:
        out["forward_ops"] = bench_fwd_ops(lgf, p64, u64.numel(), torch, stream)
        print(f"# forward ops (FP64, bench layout): {out['forward_ops']}", file=sys.stderr, flush=True)
        out["multires_torus"] = bench_torus(lgf, workloads, torch, stream, max(args.steps // 4, 3), 1, args.dc)
        print(f"# torus: {out['multires_torus']}", file=sys.stderr, flush=True)
        out["batch64"] = bench_batch(lgf, workloads, torch, stream, max(args.steps // 4, 3), 1, args.dc)
        print(f"# batch64: {out['batch64']}", file=sys.stderr, flush=True)
        out["serving"] = bench_serving(lgf, workloads, torch, out["batch64"]["value"], args.dc)
        print(f"# serving: {out['serving']}", file=sys.stderr, flush=True)
    if not args.no_cpu:
        out["cpu_baseline"], uo, uo1 = cpu_baseline()

        def rel(a, b):
            return float(np.abs(a - b).max() / np.abs(b).max())
        # every form against the oracle on the bench workload (FP32 + DC against the oracle's
        # own defect-correction step)
        out["err_vs_oracle"] = {"fp64_plain": rel(a64.reshape(uo.shape), uo),
                                "fp32_no_dc": rel(a0.reshape(uo.shape), uo),
                                "fp32_dc": rel(a32.reshape(uo.shape), uo1)}
        print(f"# err vs oracle: {out['err_vs_oracle']}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
