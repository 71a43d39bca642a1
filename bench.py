"""Benchmark of the SW2 rigid-alignment hot path on one MI355X.

Workload (default): 1 clean 8-blob reference against 10,000 noisy rotated,
shifted and jittered copies at L = 128 with n = Q = 128 (SNR 1, +-8 px,
jitter 2 px).  One step is the whole path, images already resident in HBM:
reference and image stacks to quantile tables (projection, CDF, quantiles),
then angle FFTs, spectral correlation, inverse transform over the lags,
translation correction, argmin and FP32 rescore for every pair.

Prints ONE JSON line.  Timing: W untimed warm-up steps, then K steps
bracketed by device synchronisation, with HIP events recorded on the launch
stream around every stage for per-kernel durations.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

METRIC = "alignments/s at L=128, plain FP32 vs served BF16 form; p50/p99 latency"
LEGS = ("ramp", "msw", "fourier", "all_pairs", "uneven", "single", "table4", "serving",
        "serving_mixed")
PEAK_HBM_GBS = 8000.0
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_TFLOPS = 2500.0

# Per-kernel figures from committed rocprofv3 summaries (profiles/): HBM
# traffic from two counter passes (FETCH_SIZE, WRITE_SIZE) scaled by a plain
# copy kernel, MFMA counters, kernel durations.  A kernel's figures are used
# only while its sources hash to what the summary records.
PROFILES = os.path.join(ROOT, "profiles")
HBM_FILE = os.path.join(PROFILES, "hbm_traffic_L128_10k_and_all_pairs.txt")
MFMA_FILE = os.path.join(PROFILES, "mfma_k_corr_mfma_all_pairs_2000.txt")
STATS_FILE = os.path.join(PROFILES, "kernels_all_legs_stats.txt")
KERNEL_SOURCES = {
    "k_tables2": ["k_tables.hip", "proj2_dev.h", "proj_dev.h", "quant_dev.h", "sw_internal.h"],
    "k_project2": ["k_project.hip", "proj2_dev.h", "proj_dev.h", "sw_internal.h"],
    "k_quantile": ["k_quantile.hip", "quant_dev.h", "sw_internal.h"],
    "k_align128w": ["k_align128.hip", "align128_dev.h", "align_dev.h", "fft_dev.h",
                    "sw_internal.h"],
    "k_spectrum": ["k_align.hip", "align_dev.h", "fft_dev.h", "sw_internal.h"],
    "k_corr_mfma": ["k_mfma.hip", "sw_internal.h"],
    "k_rescore_tiles": ["k_mfma.hip", "sw_internal.h"],
}


def sources_sha256(kernel):
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2503_13756_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def read_sections(path):
    """{section: {key: value}} of a summary file ("[name]" headers, "key:
    value" lines, "#" comments)."""
    out, cur = {}, None
    if not os.path.exists(path):
        return out
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("[") and line.endswith("]"):
                cur = out.setdefault(line[1:-1], {})
            elif ":" in line and cur is not None:
                k, v = line.split(":", 1)
                cur[k.strip()] = v.strip()
    return out


def profile_figures(path, kernel):
    """(figures, source note) of a kernel from a summary file, or (None, why)."""
    sec = read_sections(path).get(kernel)
    if sec is None:
        return None, f"no summary for {kernel}"
    if sec.get("sources_sha256") != sources_sha256(kernel):
        return None, "kernel changed since the counters were taken"
    return sec, os.path.relpath(path, ROOT)


def log(msg):
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def disk_pixels(L):
    j = np.arange(L)
    a = (2 * j - L + 1)[None, :] ** 2 + (2 * j - L + 1)[:, None] ** 2
    return int((a <= (L - 2) ** 2).sum())


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--images", type=int, default=10000)
    p.add_argument("--cpu-sample", type=int, default=10000,
                   help="images of the workload the oracle aligns for the CPU baseline")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-probe", action="store_true",
                   help="also run a plain 512 MiB device copy (HBM counter calibration)")
    p.add_argument("--out", default=None, help="also write the JSON line to this file")
    p.add_argument("--skip-extra", action="store_true",
                   help="only the 1-vs-10,000 workload (for profiling runs)")
    p.add_argument("--leg", action="append", choices=LEGS, default=None,
                   help="run only these further workloads (repeatable); default: all of them")
    p.add_argument("--no-h2d", action="store_true",
                   help="skip the host-resident (PCIe-inclusive) run of the headline workload")
    p.add_argument("--requests", type=int, default=2000, help="serving trace length (L = 128)")
    p.add_argument("--requests-mixed", type=int, default=2000,
                   help="serving trace length (L in {64, 128, 256})")
    return p.parse_args()


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "summarize":
        summarize(sys.argv[2:])
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported (the path "
              "is data-parallel over images and would shard by image stacks, which is not "
              "implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2503_13756_amd import api

    L = n = Q = 128
    N = args.images
    t_gen = time.time()
    w = synth.workload(1, N=N)
    t_gen = time.time() - t_gen
    ctx = api.Context(0)
    dev = torch.device("cuda", 0)
    ref = torch.from_numpy(w["ref"][None].copy()).to(dev)
    imgs = torch.from_numpy(w["imgs"]).to(dev)
    rq = torch.empty((1, Q, n), dtype=torch.float32, device=dev)
    ra = torch.empty((1, 4), dtype=torch.float64, device=dev)
    iq = torch.empty((N, Q, n), dtype=torch.float32, device=dev)
    ia = torch.empty((N, 4), dtype=torch.float64, device=dev)
    res = torch.empty((N, 6), dtype=torch.int32, device=dev)
    pmf = torch.empty((N, n, L), dtype=torch.float32, device=dev)
    torch.cuda.synchronize()

    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    # The reference's tables do not depend on the images: they run on a side
    # stream (default priority) next to the image tables, after the previous
    # step's alignment has read them, and the alignment waits for both.
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream(device=dev)

    def step(prec, ev=None):
        start, ref_done = (ev[0], ev[1]) if ev else (E(), E())
        start.record(main)
        side.wait_event(start)
        with torch.cuda.stream(side):
            api.tables(ctx, ref, n, Q, out=rq, aux=ra)
            ref_done.record(side)
        api.tables(ctx, imgs, n, Q, out=iq, aux=ia)
        if ev:
            ev[2].record(main)
        main.wait_event(ref_done)
        api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec, out=res)
        if ev:
            ev[3].record(main)

    def staged_step(ev=None):
        if ev:
            ev[0].record()
        api.project(ctx, imgs, n, out=pmf)
        if ev:
            ev[1].record()
        api.quantiles(ctx, pmf, Q, out=iq, aux=ia)
        if ev:
            ev[2].record()

    def run(fn, K, W, nev):
        for _ in range(W):
            fn(None)
        torch.cuda.synchronize()
        evs = [[E() for _ in range(nev)] for _ in range(K)]
        t0 = time.perf_counter()
        for k in range(K):
            fn(evs[k])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / K
        seg = np.array([[evs[k][i].elapsed_time(evs[k][i + 1]) for i in range(nev - 1)]
                        for k in range(K)])
        return wall * 1e3, seg.mean(axis=0), seg

    K, W = args.steps, args.warmup
    # untimed steps for at least 0.3 s before the warm-up proper, so that the
    # device has left its idle clocks when the first timed leg starts (the
    # FP32 leg, timed first, otherwise ran ~3 % slower than the same kernels
    # in the BF16 leg after it)
    t_pre = time.perf_counter()
    n_pre = 0
    while time.perf_counter() - t_pre < 0.3:
        step(0, None)
        torch.cuda.synchronize()
        n_pre += 1
    log(f"inputs ready ({t_gen:.1f} s); {n_pre} untimed steps; timing {K} FP32 steps after "
        f"{W} warm-up")
    ms32, seg32, _ = run(lambda ev: step(0, ev), K, W, 4)
    res32 = api.unpack_results(res)
    log(f"FP32 {ms32:.3f} ms/step; timing BF16-split steps")
    ms16, seg16, _ = run(lambda ev: step(1, ev), K, W, 4)
    res16 = api.unpack_results(res)
    log(f"BF16 {ms16:.3f} ms/step; timing staged tables")
    mss, segs, _ = run(staged_step, max(3, K // 4), 1, 3)

    value = N / (ms32 * 1e-3)
    # events: start (main), reference done (side), images done, alignment done
    # (main); the image tables run from the start event on the main stream
    seg32 = np.array([seg32[0], seg32[0] + seg32[1], seg32[2]])
    seg16 = np.array([seg16[0], seg16[0] + seg16[1], seg16[2]])
    # dominant kernel: per-launch durations from the events
    t_tables = seg32[1] * 1e-3  # s, one k_tables launch over N images
    t_align = seg32[2] * 1e-3   # s, k_spectrum (1 reference) + k_align128w
    M = disk_pixels(L)
    flops_tables = 4.0 * (n // 2) * M * N          # two FMAs per masked pixel and computed angle
    bytes_tables = 4.0 * L * L * N + 4.0 * Q * n * N + 32.0 * N
    bytes_align = 4.0 * Q * n * N + 24.0 * N       # image tables in, results out
    stages = {
        "tables_ref_ms": seg32[0], "tables_imgs_ms": seg32[1], "align_ms": seg32[2],
        "tables_imgs_tflops": flops_tables / t_tables * 1e-12,
        "tables_imgs_hbm_gbs": bytes_tables / t_tables * 1e-9,
        "align_hbm_gbs": bytes_align / t_align * 1e-9,
        "staged_project_ms": segs[0], "staged_quantiles_ms": segs[1],
        "bf16_tables_imgs_ms": seg16[1], "bf16_align_ms": seg16[2],
    }
    if t_tables >= t_align:
        roof = {"kernel": "k_tables", "bound": "alu", "achieved": flops_tables / t_tables * 1e-12,
                "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s"}
    else:
        roof = {"kernel": "k_align_pairs", "bound": "hbm", "achieved": bytes_align / t_align * 1e-9,
                "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = None
    if roof["kernel"] == "k_tables":
        roof["kernel"] = "k_tables2"  # two images per block
        roof["algorithmic_bytes"] = bytes_tables
        fig, note = profile_figures(HBM_FILE, "k_tables2")
        roof["traffic"] = float(fig["traffic_bytes"]) if fig else None
        roof["traffic_source"] = note

    if args.copy_probe:
        # a plain elementwise kernel over 512 MiB (reads 512 MiB, writes
        # 512 MiB): the reference for scaling the HBM byte counters
        a = torch.ones(128 << 20, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        for _ in range(3):
            torch.neg(a, out=b)
        torch.cuda.synchronize()
        del a, b

    line = {
        "metric": METRIC, "value": value, "unit": "alignments/s", "n_gpus": 1, "steps": K,
        "warmup": W, "ms_per_step": ms32, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"1 reference vs {N} images, L=128, n=Q=128, 8 blobs, +-8 px "
                               "shift, 2 px jitter, SNR 1 (plain FP32 path, images to results)",
                   "images": N, "L": L, "n_angles": n, "n_quantiles": Q},
        "roofline": roof,
        "bf16_split": {"value": N / (ms16 * 1e-3), "ms_per_step": ms16, "top_k": 4},
        "stages_ms": {k: float(v) for k, v in stages.items()},
        "paper_context": {"value": 103.0, "unit": "alignments/s",
                          "what": "SW2 over 128 rotations, one 128x128 pair, CPU (Table 3)"},
        "input_generation_s": t_gen,
    }

    if not args.no_h2d:
        log("host-resident images: chunked copies overlapped with the path")
        line["value_h2d"] = bench_h2d(api, ctx, torch, w, res32, L, n, Q)

    legs = set(args.leg) if args.leg else (set() if args.skip_extra else set(LEGS))
    extra_res = {}
    if "ramp" in legs:
        log("ramp-filtered SW2")
        line["ramp_filtered"], extra_res["ramp"] = bench_ramp(api, ctx, torch, ref, imgs, L, n, Q,
                                                              ms32)
    if "msw" in legs:
        log("max-sliced SW2")
        line["max_sliced"], extra_res["msw"] = bench_msw(api, ctx, torch, rq, ra, iq, ia, L,
                                                         seg32[0] + seg32[1])
    if "fourier" in legs:
        log("Fourier-slice projector")
        line["fourier_slice"], extra_res["fourier"] = bench_fourier(api, ctx, torch, ref, imgs, pmf,
                                                                    L, n, Q, seg32[0] + seg32[1])
    del pmf, iq, ia, res
    torch.cuda.empty_cache()
    if "all_pairs" in legs:
        log("all pairs")
        line["all_pairs"], extra_res["all_pairs"] = bench_all_pairs(api, ctx, torch)
        torch.cuda.empty_cache()
    if "uneven" in legs:
        log("uneven stacks")
        line["uneven_stacks"], extra_res["uneven"] = bench_uneven(api, ctx, torch)
        torch.cuda.empty_cache()
    if "single" in legs:
        log("single pair")
        line["single_pair"] = single_pair(api, ctx, torch)
    if "table4" in legs:
        log("1 vs 1,031 at L=39")
        line["table4_context"], extra_res["table4"] = table4_context(api, ctx, torch)
    if "serving" in legs:
        log("serving trace")
        line["serving"] = bench_serving(api, torch, args.requests, budget=1 << 30)
        torch.cuda.empty_cache()
    if "serving_mixed" in legs:
        log("serving trace, mixed L")
        line["serving_mixed_L"] = bench_serving(api, torch, args.requests_mixed, Ls=(64, 128, 256),
                                                distinct=1000, budget=4 << 30)
    line["stage_rooflines"] = stage_rooflines(line, N, L, n, Q)
    if not args.no_cpu_baseline:
        log("CPU baseline (oracle)")
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample, res32, res16, L, n, Q)
        if "all_pairs" in extra_res:
            line["cpu_baseline"]["all_pairs_error"] = all_pairs_error(*extra_res["all_pairs"])
        if "uneven" in extra_res:
            log("uneven stacks parity (oracle)")
            line["cpu_baseline"]["uneven_parity"] = uneven_parity(*extra_res["uneven"])
        if "ramp" in extra_res:
            log("ramp-filtered parity (oracle)")
            line["cpu_baseline"]["ramp_parity"] = ramp_parity(w, *extra_res["ramp"], L, n, Q)
        if "fourier" in extra_res:
            log("Fourier-slice parity (oracle)")
            line["cpu_baseline"]["fourier_parity"] = fourier_parity(w, extra_res["fourier"], L, n, Q)
        if "table4" in extra_res:
            log("L=39 parity (oracle)")
            line["cpu_baseline"]["table4_parity"] = table4_parity(*extra_res["table4"])
        if "msw" in extra_res:
            log("max-sliced parity (oracle)")
            line["cpu_baseline"]["max_sliced_parity"] = msw_parity(w, extra_res["msw"], L, n, Q)

    s = json.dumps(line)
    print(s, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(s + "\n")
    ctx.close()


def stage_rooflines(line, N, L, n, Q):
    """Every stage of the headline path (and of the all-pairs path when that
    leg ran) against the roofline that bounds it: achieved = algorithmic
    bytes or flops per launch / the launch's duration, next to the measured
    HBM traffic and MFMA counters of the committed rocprofv3 summaries.
    Durations: HIP events of this run where a stage is one library call, else
    the kernel-trace summary (named in `duration`)."""
    st = line["stages_ms"]
    M = disk_pixels(L)
    out = []

    def add(kernel, bound, work, ms, note, extra=None):
        unit = {"hbm": "GB/s", "alu": "TFLOP/s", "mfma": "TFLOP/s"}[bound]
        peak = {"hbm": PEAK_HBM_GBS, "alu": PEAK_FP32_TFLOPS, "mfma": PEAK_BF16_TFLOPS}[bound]
        scale = 1e-9 if bound == "hbm" else 1e-12
        ach = work / (ms * 1e-3) * scale
        e = {"kernel": kernel, "bound": bound, "achieved": ach, "peak": peak, "unit": unit,
             "frac": ach / peak, "ms": ms, "duration": note,
             ("algorithmic_bytes" if bound == "hbm" else "algorithmic_flops"): work}
        fig, src = profile_figures(HBM_FILE, kernel)
        e["traffic"] = float(fig["traffic_bytes"]) if fig else None
        e["traffic_source"] = src
        if e["traffic"]:
            e["traffic_gbs"] = e["traffic"] / (ms * 1e-3) * 1e-9
            e["traffic_frac_of_hbm"] = e["traffic_gbs"] / PEAK_HBM_GBS
        if extra:
            e.update(extra)
        out.append(e)

    flops_proj = 4.0 * (n // 2) * M * N
    add("k_tables2", "alu", flops_proj, st["tables_imgs_ms"], "HIP events (images -> tables)")
    add("k_project2", "alu", flops_proj, st["staged_project_ms"], "HIP events (staged projection)")
    add("k_quantile", "hbm", (4.0 * n * L + 4.0 * Q * n + 32.0) * N, st["staged_quantiles_ms"],
        "HIP events (staged quantiles)")
    add("k_align128w", "hbm", (4.0 * Q * n + 24.0) * N, st["align_ms"],
        "HIP events (reference spectrum, coefficients and k_align128w)")
    ap = line.get("all_pairs")
    if ap:
        NA, LA = 2000, 64
        P = NA * NA
        stats = read_sections(STATS_FILE)
        for kernel, bound, work in (
                ("k_spectrum", "hbm", (4.0 * LA * LA + 4.0 * (LA // 2 + 1) * LA) * NA),
                ("k_corr_mfma", "mfma", ap["mfma_flops_per_step"]),
                ("k_rescore_tiles", "alu", 4 * 3.0 * LA * LA * P)):
            fig, src = profile_figures(STATS_FILE, kernel)
            if not fig:
                out.append({"kernel": kernel, "bound": bound, "achieved": None, "note": src})
                continue
            extra = None
            if kernel == "k_corr_mfma":
                mf, msrc = profile_figures(MFMA_FILE, kernel)
                extra = {"mfma_util_pct": float(mf["mfma_util_pct"]) if mf else None,
                         "mfma_bf16_flops_counted": float(mf["mfma_bf16_flops"]) if mf else None,
                         "mfma_source": msrc}
            add(kernel, bound, work, float(fig["avg_us"]) * 1e-3, f"kernel trace ({src})", extra)
        del stats
    return out


def summarize(argv):
    """Summaries of rocprofv3 CSV output for profiles/ (text on stdout):
      summarize hbm FETCH_DIR WRITE_DIR "command"  HBM bytes per dispatch of the
          path's kernels, each counter scaled by what it reads for the plain
          512 MiB elementwise kernel of --copy-probe (512 MiB read + written)
      summarize rdreq PMC_DIR "command"            bytes read from memory per dispatch
          from the L2's read-request counts by size (128/64/32 B): a check of
          the FETCH_SIZE calibration (gfx950's FETCH_SIZE counts a 128-byte
          request as 64 bytes when TCC_BUBBLE stays zero)
      summarize mfma PMC_DIR "command"             MFMA counters of k_corr_mfma
      summarize sq PMC_DIR[,PMC_DIR2] "command"    SQ counters of k_tables2
      summarize stats TRACE_DIR "command"          kernel durations
    Per kernel the dispatches with the largest grid are taken (the full
    workloads), averaged; every section records the kernel's source hash."""
    import csv
    import glob

    kind, rest = argv[0], argv[1:]

    def counters(d):
        rows = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += list(csv.DictReader(open(path)))
        agg = {}
        for r in rows:
            key = (r["Kernel_Name"], int(r["Grid_Size"]))
            a = agg.setdefault(key, {"dispatches": set()})
            a["dispatches"].add(r["Dispatch_Id"])
            a[r["Counter_Name"]] = a.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        return agg

    def pick(agg, pattern):
        best = None
        for (name, grid), a in agg.items():
            if pattern in name and (best is None or grid > best[1]):
                best = (name, grid, a)
        return best

    def per_dispatch(a, c):
        return a[c] / len(a["dispatches"])

    print(f"# rocprofv3 summary ({kind}); command(s): {rest[-1]}")
    print("# values per dispatch (summed over the device by rocprofv3), averaged over the "
          "dispatches of the largest grid of each kernel")
    if kind == "hbm":
        fa, wa = counters(rest[0]), counters(rest[1])
        cf = pick(fa, "neg_kernel")
        cw = pick(wa, "neg_kernel")
        ff = (512 << 10) / per_dispatch(cf[2], "FETCH_SIZE")   # KiB read by the copy
        wf = (512 << 10) / per_dispatch(cw[2], "WRITE_SIZE")   # KiB written
        print(f"[calibration]\ncopy_kernel: {cf[0][:80]}\nfetch_factor: {ff:.4f}\n"
              f"write_factor: {wf:.4f}")
        for k in KERNEL_SOURCES:
            f, w = pick(fa, f"sw::{k}<"), pick(wa, f"sw::{k}<")
            if not f or not w:
                continue
            fk, wk = per_dispatch(f[2], "FETCH_SIZE"), per_dispatch(w[2], "WRITE_SIZE")
            print(f"[{k}]\nkernel: {f[0][:100]}\ngrid: {f[1]}\ndispatches: {len(f[2]['dispatches'])}\n"
                  f"fetch_kib: {fk:.1f}\nwrite_kib: {wk:.1f}\n"
                  f"traffic_bytes: {1024 * (fk * ff + wk * wf):.0f}\n"
                  f"sources_sha256: {sources_sha256(k)}")
    elif kind == "rdreq":
        agg = counters(rest[0])
        sizes = (("TCC_EA0_RDREQ_128B_sum", 128), ("TCC_EA0_RDREQ_64B_sum", 64),
                 ("TCC_EA0_RDREQ_32B_sum", 32))

        def read_bytes(a):
            return sum(w * per_dispatch(a, c) for c, w in sizes)

        cp = pick(agg, "neg_kernel")
        print(f"[copy]\nkernel: {cp[0][:80]}\nbytes_read: {read_bytes(cp[2]):.0f}\n"
              f"bytes_known: {512 << 20}\nTCC_BUBBLE_sum: {per_dispatch(cp[2], 'TCC_BUBBLE_sum'):.0f}")
        for k in KERNEL_SOURCES:
            b = pick(agg, f"sw::{k}<")
            if not b:
                continue
            print(f"[{k}]\nkernel: {b[0][:100]}\ngrid: {b[1]}\ndispatches: {len(b[2]['dispatches'])}")
            for c, _ in sizes:
                print(f"{c}: {per_dispatch(b[2], c):.0f}")
            print(f"bytes_read: {read_bytes(b[2]):.0f}\nsources_sha256: {sources_sha256(k)}")
    elif kind in ("mfma", "sq"):
        aggs = [counters(d) for d in rest[0].split(",")]
        k = "k_corr_mfma" if kind == "mfma" else "k_tables2"
        print(f"[{k}]")
        for agg in aggs:
            b = pick(agg, f"sw::{k}<")
            print(f"kernel: {b[0][:100]}\ngrid: {b[1]}\ndispatches: {len(b[2]['dispatches'])}")
            for c in sorted(x for x in b[2] if x != "dispatches"):
                print(f"{c}: {per_dispatch(b[2], c):.1f}")
            if kind == "mfma" and "SQ_INSTS_VALU_MFMA_MOPS_BF16" in b[2]:
                print(f"mfma_bf16_flops: {512 * per_dispatch(b[2], 'SQ_INSTS_VALU_MFMA_MOPS_BF16'):.0f}")
                print(f"mfma_f32_flops: {512 * per_dispatch(b[2], 'SQ_INSTS_VALU_MFMA_MOPS_F32'):.0f}")
                # busy cycles of all 1024 SIMDs over the active cycles of one XCD
                # (GRBM_GUI_ACTIVE comes summed over the 8 XCDs)
                busy = per_dispatch(b[2], "SQ_VALU_MFMA_BUSY_CYCLES")
                active = per_dispatch(b[2], "GRBM_GUI_ACTIVE") / 8
                print(f"mfma_util_pct: {100 * busy / (active * 1024):.1f}")
            if kind == "sq" and "SQ_INSTS_VALU" in b[2]:
                imgs = b[1] // 512 * 2  # two images per 512-thread block
                print(f"valu_wave_instructions_per_image: {per_dispatch(b[2], 'SQ_INSTS_VALU') / imgs:.0f}")
            if "SQ_LDS_BANK_CONFLICT" in b[2]:
                print("lds_bank_conflict_share_of_lds_active: "
                      f"{b[2]['SQ_LDS_BANK_CONFLICT'] / b[2]['SQ_LDS_IDX_ACTIVE']:.3f}")
        print(f"sources_sha256: {sources_sha256(k)}")
    elif kind == "stats":
        rows = []
        for path in glob.glob(os.path.join(rest[0], "**", "*kernel_trace.csv"), recursive=True):
            rows += list(csv.DictReader(open(path)))
        by = {}
        for r in rows:
            d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            by.setdefault(r["Kernel_Name"], []).append((grid, d))
        tot = sum(d for v in by.values() for _, d in v)
        print(f"{'kernel':88s} {'calls':>6s} {'avg_us':>10s} {'min_us':>10s} {'max_us':>10s} {'pct':>6s}")
        for name, v in sorted(by.items(), key=lambda kv: -sum(d for _, d in kv[1]))[:40]:
            ds = [d for _, d in v]
            print(f"{name[:88]:88s} {len(ds):6d} {sum(ds) / len(ds):10.2f} {min(ds):10.2f} "
                  f"{max(ds):10.2f} {100 * sum(ds) / tot:6.2f}")
        for k in KERNEL_SOURCES:
            cand = [(n_, v) for n_, v in by.items() if f"sw::{k}<" in n_]
            if not cand:
                continue
            gmax = max(g for _, v in cand for g, _ in v)
            ds = [d for _, v in cand for g, d in v if g == gmax]
            print(f"[{k}]\ngrid: {gmax}\ncalls: {len(ds)}\navg_us: {sum(ds) / len(ds):.2f}\n"
                  f"sources_sha256: {sources_sha256(k)}")


def timed(torch, fn, K, W=1):
    for _ in range(W):
        fn()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(K):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / K


def bench_h2d(api, ctx, torch, w, res_resident, L, n, Q, chunk=1000, K=3):
    """The headline workload with the images in pinned host memory and the
    results returned to pinned host memory: the reference and chunks of
    `chunk` images are copied on a copy stream while the previous chunk's
    tables and alignment run on the compute stream (two device buffers);
    the clock runs from the first host-to-device copy to the last result
    back on the host.  The results must equal the HBM-resident run's
    bitwise (same kernels; a pair's result does not depend on its batch)."""
    dev = torch.device("cuda", 0)
    N = len(w["imgs"])
    h_ref = torch.from_numpy(w["ref"][None].copy()).pin_memory()
    h_imgs = torch.from_numpy(w["imgs"]).pin_memory()
    h_res = torch.empty((N, 6), dtype=torch.int32).pin_memory()
    d_ref = torch.empty((1, L, L), dtype=torch.float32, device=dev)
    rq = torch.empty((1, Q, n), dtype=torch.float32, device=dev)
    ra = torch.empty((1, 4), dtype=torch.float64, device=dev)
    bufs = [torch.empty((chunk, L, L), dtype=torch.float32, device=dev) for _ in range(2)]
    qts = [torch.empty((chunk, Q, n), dtype=torch.float32, device=dev) for _ in range(2)]
    auxs = [torch.empty((chunk, 4), dtype=torch.float64, device=dev) for _ in range(2)]
    ress = [torch.empty((chunk, 6), dtype=torch.int32, device=dev) for _ in range(2)]
    comp = torch.cuda.current_stream()
    copy_s = torch.cuda.Stream(device=dev)
    E = lambda: torch.cuda.Event()  # noqa: E731
    nch = (N + chunk - 1) // chunk

    def one():
        copied = [E() for _ in range(nch)]
        freed = [E() for _ in range(nch)]
        ref_in = E()
        with torch.cuda.stream(copy_s):
            d_ref.copy_(h_ref, non_blocking=True)
            ref_in.record(copy_s)

        def issue_copy(c):
            b, c0, c1 = c % 2, c * chunk, min(N, (c + 1) * chunk)
            with torch.cuda.stream(copy_s):
                if c >= 2:
                    copy_s.wait_event(freed[c - 2])  # chunk c - 2's tables read this buffer
                bufs[b][:c1 - c0].copy_(h_imgs[c0:c1], non_blocking=True)
                copied[c].record(copy_s)

        issue_copy(0)
        comp.wait_event(ref_in)
        api.tables(ctx, d_ref, n, Q, out=rq, aux=ra)
        for c in range(nch):
            if c + 1 < nch:
                issue_copy(c + 1)
            b, c0, c1 = c % 2, c * chunk, min(N, (c + 1) * chunk)
            m = c1 - c0
            comp.wait_event(copied[c])
            api.tables(ctx, bufs[b][:m], n, Q, out=qts[b][:m], aux=auxs[b][:m])
            freed[c].record(comp)
            api.align_batch(ctx, rq, ra, qts[b][:m], auxs[b][:m], L, out=ress[b][:m])
            h_res[c0:c1].copy_(ress[b][:m], non_blocking=True)
        comp.synchronize()

    one()  # warm-up
    torch.cuda.synchronize()
    times = []
    for _ in range(K):
        t0 = time.perf_counter()
        one()
        times.append(time.perf_counter() - t0)
    # the copies alone, for the PCIe rate
    torch.cuda.synchronize()
    big = torch.empty((N, L, L), dtype=torch.float32, device=dev)
    t0 = time.perf_counter()
    big.copy_(h_imgs, non_blocking=True)
    torch.cuda.synchronize()
    t_copy = time.perf_counter() - t0
    del big
    same = bool(np.array_equal(h_res.numpy(), res_resident_records(res_resident)))
    t = float(np.median(times))
    return {"workload": f"the headline workload from pinned host memory: reference and {N} "
                        f"images copied in chunks of {chunk} on a copy stream, overlapped with "
                        "the tables and alignment of the previous chunk; results copied back",
            "value": N / t, "unit": "alignments/s", "ms": t * 1e3,
            "h2d_copy_ms": t_copy * 1e3, "h2d_gbs": h_imgs.numel() * 4 / t_copy * 1e-9,
            "results_equal_resident_run": same}


def res_resident_records(r):
    """Result dict (unpack_results) back to [N, 6] int32 records."""
    rec = np.zeros((len(r["rot_index"]), 6), np.int32)
    rec[:, 0] = r["rot_index"]
    rec[:, 1] = np.asarray(r["theta_rad"], np.float32).view(np.int32)
    rec[:, 2:4] = np.asarray(r["shift_px"], np.float32).view(np.int32)
    rec[:, 4] = np.asarray(r["sw2sq"], np.float32).view(np.int32)
    rec[:, 5] = r["status"]
    return rec


def bench_ramp(api, ctx, torch, ref, imgs, L, n, Q, ms_sw2, K=5):
    """Ramp-filtered SW2 on the 1-vs-many workload: stacked signed-part tables
    of the reference and of every image (projection, ramp filter, two
    inversions), then the alignment of the 2Q-row tables, FP32 and BF16."""
    N = imgs.shape[0]
    dev = imgs.device
    rq = torch.empty((1, 2 * Q, n), dtype=torch.float32, device=dev)
    ra = torch.empty((1, 4), dtype=torch.float64, device=dev)
    iq = torch.empty((N, 2 * Q, n), dtype=torch.float32, device=dev)
    ia = torch.empty((N, 4), dtype=torch.float64, device=dev)
    res = torch.empty((N, 6), dtype=torch.int32, device=dev)
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    def step(prec, ev):
        ev[0].record()
        api.tables(ctx, ref, n, Q, out=rq, aux=ra, ramp=True)
        api.tables(ctx, imgs, n, Q, out=iq, aux=ia, ramp=True)
        ev[1].record()
        api.align_batch(ctx, rq, ra, iq, ia, L, prec=prec, out=res, ramp=True)
        ev[2].record()

    out = {"workload": f"1 reference vs {N} images, L=128, n=Q=128 (images as in the main line), "
                       "ramp-filtered SW2: stacked 2Q-row tables, images to results"}
    results = {}
    for prec, name in ((0, "fp32"), (1, "bf16_split")):
        step(prec, [E(), E(), E()])
        torch.cuda.synchronize()
        evs = [[E(), E(), E()] for _ in range(K)]
        t0 = time.perf_counter()
        for k in range(K):
            step(prec, evs[k])
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / K * 1e3
        tab = float(np.mean([e[0].elapsed_time(e[1]) for e in evs]))
        ali = float(np.mean([e[1].elapsed_time(e[2]) for e in evs]))
        out[name] = {"value": N / (wall * 1e-3), "ms_per_step": wall, "tables_ms": tab,
                     "align_ms": ali}
        results[name] = api.unpack_results(res)
    out["unit"] = "alignments/s"
    out["cost_vs_sw2_fp32"] = out["fp32"]["ms_per_step"] / ms_sw2
    out["paper_context"] = "RFSW2 costs 1.3-1.4x SW2 on CPU (Table 4: 0.831 s vs 0.586 s)"
    return out, (results["fp32"], results["bf16_split"])


def ramp_parity(w, r32, r16, L, n, Q, S=1000):
    """Oracle ramp-filtered alignment of the first S images against the GPU's
    FP32 and BF16 results of the timed run."""
    from oracle import oracle as O
    from tests import parity

    S = min(S, len(w["imgs"]))
    o = O.align_images(w["ref"], w["imgs"][:S], n, Q, want_curve=True, ramp=True)
    out = {"pairs": S}
    for name, r in (("fp32", r32), ("bf16_split", r16)):
        sub = {k: v[:S] for k, v in r.items()}
        try:
            rep = parity.check(sub, o, L, parity.TAU_RF, o["curve"])
            out[name] = f"{rep['pairs']} pairs ok, exact rotation {rep['exact_rot']}"
        except AssertionError as e:
            out[name] = "FAILED: " + str(e)[:300]
    truth = w["truth_theta"][:S]
    d = (r32["theta_rad"][:S] - truth + math.pi) % (2 * math.pi) - math.pi
    out["gpu_within_15deg_of_truth"] = float(np.mean(np.abs(d) <= math.radians(15)))
    return out


def bench_msw(api, ctx, torch, rq, ra, iq, ia, L, tables_ms, K=5):
    """Max-sliced alignment (rotation only) of the reference against the image
    tables of the main line, already in HBM: the alignment alone is timed,
    and the whole-path rate adds the tables time of the main line."""
    N = iq.shape[0]
    res = torch.empty((N, 6), dtype=torch.int32, device=iq.device)
    E = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    api.align_batch(ctx, rq, ra, iq, ia, L, mode=2, out=res)
    torch.cuda.synchronize()
    e0, e1 = E(), E()
    e0.record()
    for _ in range(K):
        api.align_batch(ctx, rq, ra, iq, ia, L, mode=2, out=res)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / K
    out = {"workload": f"1 reference vs {N} image tables, L=128, n=Q=128 (tables of the main line), "
                       "max-sliced SW2 over rotations (rotation only), top-1 rescore",
           "align_ms": ms, "align_value": N / (ms * 1e-3), "unit": "alignments/s",
           "value_with_tables": N / ((ms + tables_ms) * 1e-3),
           "paper_context": "max-sliced costs 3.7x SW2 on CPU (Table 4 of the extended results: "
                            "2.181 s vs 0.586 s)"}
    return out, api.unpack_results(res)


def msw_parity(w, r, L, n, Q, S=500):
    """Oracle max-sliced alignment of the first S images against the GPU's."""
    from oracle import oracle as O
    from tests import parity

    S = min(S, len(w["imgs"]))
    o = O.align_images(w["ref"], w["imgs"][:S], n, Q, mode=O.MODE_MAX_SLICED, want_curve=True)
    sub = {k: v[:S] for k, v in r.items()}
    try:
        rep = parity.check(sub, o, L, parity.TAU_FP32, o["curve"])
        return f"{rep['pairs']} pairs ok, exact rotation {rep['exact_rot']}"
    except AssertionError as e:
        return "FAILED: " + str(e)[:300]


def fourier_flops(L, n):
    """Algorithmic FP32 flops of the Fourier-slice projector per image:
    5 N log2 N per complex FFT (L/2 row transforms and L+1 column transforms
    of length 2L, n/4 slice transforms of length L) and 4 per kernel tap
    (W^2 = 49 taps per slice point, n/2 (L/2 + 1) points)."""
    Nf = 2 * L
    fft = 5 * Nf * math.log2(Nf) * (L // 2 + L + 1) + 5 * L * math.log2(L) * (n // 4)
    return fft + 4 * 49 * (n // 2) * (L // 2 + 1)


def bench_fourier(api, ctx, torch, ref, imgs, pmf, L, n, Q, line_tables_ms, K=5):
    """Fourier-slice projector (NUFFT) on the images of the main line: the
    projector alone next to the line-sum projector, and the whole path
    (images -> Fourier tables -> alignment against the reference's Fourier
    tables); then the projector alone at L = 256 on 3000 blob images."""
    N = imgs.shape[0]
    dev = imgs.device
    t_f = timed(torch, lambda: api.project_fourier(ctx, imgs, n, out=pmf), K)
    t_l = timed(torch, lambda: api.project(ctx, imgs, n, out=pmf), K)
    rq, ra = api.tables_fourier(ctx, ref, n, Q)
    iq = torch.empty((N, Q, n), dtype=torch.float32, device=dev)
    ia = torch.empty((N, 4), dtype=torch.float64, device=dev)
    res = torch.empty((N, 6), dtype=torch.int32, device=dev)
    t_t = timed(torch, lambda: api.tables_fourier(ctx, imgs, n, Q, out=iq, aux=ia), K)
    t_a = timed(torch, lambda: api.align_batch(ctx, rq, ra, iq, ia, L, out=res), K)
    fl = fourier_flops(L, n)
    out = {"workload": f"1 reference vs {N} images, L={L}, n=Q={L} (images of the main line), "
                       "Fourier-slice projections (type-2 NUFFT, width-7 kernel, grid x2), "
                       "negative lobes clipped, images to results",
           "projector_ms": t_f, "line_sum_projector_ms": t_l, "tables_ms": t_t, "align_ms": t_a,
           "value": N / ((t_t + t_a) * 1e-3), "unit": "alignments/s",
           "line_sum_tables_ms": line_tables_ms,
           "projector_tflops": fl * N / (t_f * 1e-3) / 1e12,
           "paper_context": "the paper projects with a NUFFT in O(L^2 log L) per image (Sec. 2.3)"}
    del iq, ia
    L2, N2 = 256, 3000
    _, big = _pool(L2, N2, 1210, distinct=64)
    big = big.to(dev)
    p2 = torch.empty((N2, L2, L2), dtype=torch.float32, device=dev)
    t_f2 = timed(torch, lambda: api.project_fourier(ctx, big, L2, out=p2), K)
    t_l2 = timed(torch, lambda: api.project(ctx, big, L2, out=p2), K)
    out["L256"] = {"images": N2, "projector_ms": t_f2, "line_sum_projector_ms": t_l2,
                   "projector_tflops": fourier_flops(L2, L2) * N2 / (t_f2 * 1e-3) / 1e12}
    del big, p2
    fourier_res = (rq, ra, api.unpack_results(res))
    # Monte-Carlo SW2 (extended alignment results): the same images, slices at
    # n sorted random directions (seeded), rotation-only scan
    theta = synth.mc_angles(n, 2024)
    iq = torch.empty((N, Q, n), dtype=torch.float32, device=dev)
    ia = torch.empty((N, 4), dtype=torch.float64, device=dev)
    mq, ma = api.tables_fourier(ctx, ref, n, Q, theta=theta)
    t_mt = timed(torch, lambda: api.tables_fourier(ctx, imgs, n, Q, out=iq, aux=ia, theta=theta), K)
    t_ma = timed(torch, lambda: api.align_batch(ctx, mq, ma, iq, ia, L, mode=1, out=res), K)
    out["monte_carlo"] = {
        "workload": f"1 reference vs {N} images, L={L}, n=Q={L}: slices at {n} sorted uniform "
                    "random directions (seed 2024), rotation-only scan",
        "tables_ms": t_mt, "align_ms": t_ma, "value": N / ((t_mt + t_ma) * 1e-3),
        "unit": "alignments/s",
        "paper_context": "Monte-Carlo SW2 costs 0.97x SW2 on CPU (Table 4 of the extended results: "
                         "0.568 s vs 0.586 s)"}
    del iq, ia
    return out, (fourier_res, (theta, api.unpack_results(res)))


def fourier_parity(w, r, L, n, Q, S=16):
    """Oracle Fourier-slice tables and alignment of the first S images against
    the GPU's, for the grid directions and for the Monte-Carlo ones."""
    from oracle import oracle as O
    from tests import parity

    (rq, ra, g), (theta, gm) = r
    S = min(S, len(w["imgs"]))
    out = {}
    oq, oa = O.fourier_tables(w["ref"][None], n, Q)
    iq0, ia0 = O.fourier_tables(w["imgs"][:S], n, Q)
    cases = (("fourier", g, lambda: O.align(oq, oa, iq0, ia0, L, want_curve=True)),
             ("monte_carlo", gm, lambda: O.mc_align_images(w["ref"][None], w["imgs"][:S], n, Q,
                                                           theta, want_curve=True)))
    for name, gg, orc in cases:
        o = orc()
        sub = {k: v[:S] for k, v in gg.items()}
        try:
            rep = parity.check(sub, o, L, parity.TAU_FP32, o["curve"])
            out[name] = f"{rep['pairs']} pairs ok, exact rotation {rep['exact_rot']}"
        except AssertionError as e:
            out[name] = "FAILED: " + str(e)[:300]
    return out


def bench_all_pairs(api, ctx, torch, N=2000, L=64):
    """All ordered pairs of 2,000 images at L = 64 (4,000,000 alignments):
    tables, then bf16 angle spectra and the MFMA correlation with top-4 FP32
    rescoring."""
    w = synth.workload(2, N=N)
    imgs = torch.from_numpy(w["imgs"]).cuda()
    q = torch.empty((N, L, L), dtype=torch.float32, device="cuda")
    a = torch.empty((N, 4), dtype=torch.float64, device="cuda")
    res = torch.empty((N * N, 6), dtype=torch.int32, device="cuda")
    t_tab = timed(torch, lambda: api.tables(ctx, imgs, L, L, out=q, aux=a), 5)
    t_al = timed(torch, lambda: api.align_batch(ctx, q, a, q, a, L, prec=1, top_k=4, out=res), 5)
    ms = t_tab + t_al
    # algorithmic MFMA work: two real GEMMs of K = 2Q per frequency and pair
    flops = 2.0 * 2.0 * (L // 2 + 1) * (2 * L) * N * N
    out = {"workload": f"all ordered pairs of {N} images, L={L}, n=Q={L}, bf16 MFMA correlation, "
                       "top-4 FP32 rescore", "alignments": N * N, "ms_per_step": ms,
           "value": N * N / (ms * 1e-3), "unit": "alignments/s", "tables_ms": t_tab,
           "align_ms": t_al, "mfma_flops_per_step": flops}
    return out, (w, api.unpack_results(res), L)


def all_pairs_error(w, g, L, S=1000):
    """GPU all-pairs results against the FP64 oracle on a seeded sample."""
    from oracle import oracle as O
    from tests import parity

    N = len(w["imgs"])
    rng = np.random.Generator(np.random.PCG64(1002))
    pairs = np.stack([rng.integers(0, N, S), rng.integers(0, N, S)], axis=1)
    pairs[:10, 1] = pairs[:10, 0]  # ten diagonal pairs
    ids = np.unique(pairs)
    q, a = O.tables(w["imgs"][ids], L, L)
    remap = {v: i for i, v in enumerate(ids)}
    lp = np.array([[remap[x] for x in p] for p in pairs])
    o = O.align(q, a, q, a, L, pairs=lp, want_curve=True)
    sub = {k: v[pairs[:, 0] * N + pairs[:, 1]] for k, v in g.items()}
    rel = np.abs(sub["sw2sq"] - o["sw2sq"]) / np.maximum(o["sw2sq"], 1e-12)
    out = {"pairs": S, "max_rel_err_sw2sq": float(np.max(rel[10:])),
           "median_rel_err_sw2sq": float(np.median(rel[10:])),
           "rot_exact_rate": float(np.mean(sub["rot_index"] == o["rot_index"])),
           "diagonal_zero": bool(np.all(sub["sw2sq"][:10] == 0.0))}
    try:
        rep = parity.check(sub, o, L, parity.TAU_BF16, o["curve"])
        out["parity"] = f"{rep['pairs']} pairs ok (bf16 tolerance)"
    except AssertionError as e:
        out["parity"] = "FAILED: " + str(e)[:300]
    return out


def bench_uneven(api, ctx, torch, total=50000, distinct=200):
    """Stacks of L in {64, 96, 128, 192, 256} with sizes drawn uniformly in
    [100, 5000] until 50,000 images, each with its own reference, through the
    mixed persistent launches.  Each stack holds `distinct` rendered copies of
    its reference, tiled to the drawn size."""
    stacks = synth.uneven_stacks(total=total, cap_per_stack=distinct)
    dev = []
    for L, ref, imgs, size in stacks:
        x = torch.from_numpy(imgs).cuda()
        reps = (size + len(imgs) - 1) // len(imgs)
        dev.append((torch.from_numpy(ref).cuda(), x.repeat(reps, 1, 1)[:size].contiguous()))
    # launch tiles per L (strip rows, tasks per wave, alignment blocks per CU),
    # measured once on this device (a plan step, untimed)
    import tempfile

    t0 = time.perf_counter()
    tiles_path = os.path.join(tempfile.mkdtemp(), "tiles.json")
    api.autotune(ctx, sorted({s[0] for s in stacks}), out_json=tiles_path)
    t_tune = time.perf_counter() - t0
    ms = timed(torch, lambda: api.align_stacks(ctx, dev, prec=1), 3)
    outs = api.align_stacks(ctx, dev, prec=1)
    torch.cuda.synchronize()
    res = [api.unpack_results(o["res"]) for o in outs]
    per_L = {}
    for L in sorted({s[0] for s in stacks}):
        sub = [d for d, s in zip(dev, stacks) if s[0] == L]
        nimg = sum(int(d[1].shape[0]) for d in sub)
        t = timed(torch, lambda: api.align_stacks(ctx, sub, prec=1), 3)
        per_L[str(L)] = {"images": nimg, "ms": t, "alignments_per_s": nimg / (t * 1e-3)}
    n = sum(int(d[1].shape[0]) for d in dev)
    return ({"workload": f"{len(stacks)} stacks, {n} images, L in {{64,96,128,192,256}}, sizes "
                         "U[100,5000], own reference each, FP32 tables, bf16 correlation, top-4 "
                         "FP32 rescore, strip tiles autotuned per L", "images": n, "ms_per_step": ms,
             "autotune_s": t_tune, "tiles": json.load(open(tiles_path))["tiles"],
             "value": n / (ms * 1e-3), "unit": "alignments/s", "per_L": per_L},
            (stacks, res))


def uneven_parity(stacks, res, S=200):
    """GPU results of the uneven stacks against the FP64 oracle on the first
    S images of every stack (the distinct rendered copies)."""
    from oracle import oracle as O
    from tests import parity

    ok, total, worst = 0, 0, 0.0
    fails = []
    for (L, ref, imgs, size), r in zip(stacks, res):
        m = min(S, len(imgs), size)
        o = O.align_images(ref, imgs[:m], L, L, want_curve=True)
        sub = {k: v[:m] for k, v in r.items()}
        try:
            parity.check(sub, o, L, parity.TAU_BF16, o["curve"])
            ok += m
        except AssertionError as e:
            fails.append(f"L={L}: " + str(e)[:120])
        rel = np.abs(sub["sw2sq"] - o["sw2sq"]) / np.maximum(o["sw2sq"], 1e-12)
        worst = max(worst, float(rel.max()))
        total += m
    return {"pairs": total, "parity_ok_pairs": ok, "max_rel_err_sw2sq": worst,
            "failures": fails[:3]}


def single_pair(api, ctx, torch, reps=50):
    """The single-pair workload (L = 64, n = Q = 64): images to result, one
    call sequence per pair, synchronised; mean latency."""
    w = synth.workload(0)
    L = 64
    r = torch.from_numpy(w["ref"][None].copy()).cuda()
    x = torch.from_numpy(np.ascontiguousarray(w["imgs"])).cuda()

    def one():
        rq, ra = api.tables(ctx, r, L, L)
        iq, ia = api.tables(ctx, x, L, L)
        res, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
        return res

    for _ in range(5):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        one()
        torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    g = api.unpack_results(one())
    return {"workload": "1 pair, L=64, n=Q=64 (images to result, synchronised per pair)",
            "latency_ms": dt * 1e3, "rot_index": int(g["rot_index"][0]),
            "shift_px": [float(v) for v in g["shift_px"][0]], "sw2sq": float(g["sw2sq"][0]),
            "paper_context": "0.0027 s per pair at L=64 on CPU (Table 3)"}


def table4_context(api, ctx, torch, reps=20):
    """1 reference + 1,031 images at L = 39 (the digits' size and count in the
    paper's Table 4), n = Q = 48: host images (pinned) to results back on the
    host, synchronised per job; the oracle's parity on every pair."""
    L, n, Q, N = 39, 48, 48, 1031
    ref, imgs, _, _ = synth.make_stack(1005, L, N, K=8, shift_px=6.0, jitter_px=1.0, snr=1.0)
    r_h = torch.from_numpy(ref[None].copy()).pin_memory()
    x_h = torch.from_numpy(np.ascontiguousarray(imgs)).pin_memory()

    def one():
        r = r_h.cuda(non_blocking=True)
        x = x_h.cuda(non_blocking=True)
        rq, ra = api.tables(ctx, r, n, Q)
        iq, ia = api.tables(ctx, x, n, Q)
        res, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
        return res.cpu()

    for _ in range(3):
        one()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        res = one()
    dt = (time.perf_counter() - t0) / reps
    return ({"workload": "1 reference + 1031 images, L=39, n=Q=48, 8 blobs, +-6 px, SNR 1; "
                         "pinned host images to host results, synchronised per job",
             "ms": dt * 1e3, "alignments_per_s": N / dt,
             "paper_context": "0.586 s for SW2, 1 vs 1031 digits at L=39 on CPU (Table 4)"},
            (ref, imgs, api.unpack_results(res), n, Q, L))


def table4_parity(ref, imgs, g, n, Q, L):
    """The oracle on every pair of the L = 39 job."""
    from oracle import oracle as O
    from tests import parity

    o = O.align_images(ref, imgs, n, Q, want_curve=True)
    try:
        rep = parity.check(g, o, L, parity.TAU_FP32, o["curve"])
        return f"{rep['pairs']} pairs ok, exact rotation {rep['exact_rot']}"
    except AssertionError as e:
        return "FAILED: " + str(e)[:300]


def _pool(L, N, seed, distinct=None):
    """Rendered copies for the serving trace, in pinned (page-locked) host
    memory as a serving front end would hold request buffers, so host to
    device copies run at DMA speed for both forms.  With `distinct`, that
    many copies are rendered and tiled to N."""
    import torch

    m = N if distinct is None else min(N, distinct)
    ref, imgs, _, _ = synth.make_stack(seed, L, m)
    if m < N:
        imgs = np.ascontiguousarray(np.tile(imgs, ((N + m - 1) // m, 1, 1))[:N])
    ref_p = torch.from_numpy(ref).pin_memory()
    imgs_p = torch.from_numpy(imgs).pin_memory()
    return ref_p, imgs_p


def bench_serving(api, torch, n_req, Ls=(128,), pool_n=5000, seed=1004, distinct=None,
                  max_slots=32, budget=1 << 30, max_per_step=8):
    """Poisson trace of requests (1 reference + N images, N log-uniform in
    [1, 5000]); served bf16 form (continuous batching) against the plain FP32
    path serving one request at a time, and the served FP32 form (the same
    batching without the precision split).  Images come from a pool of
    rendered copies per L in pinned host memory (requests take slices), so
    host rendering stays out of the clocks; every form includes the host to
    device copies.  Reported: saturated alignments/s (all requests arrive at
    once) and latency percentiles at a fixed arrival rate of 0.8x the plain
    form's measured capacity.  The server keeps up to max_slots requests in
    flight and launches at most max_per_step of them per step, so the next
    step's host to device copies run beside the current step's kernels (32
    and 8: the best saturated rates of the pairs tried, 8 to 32 and 4 to 16,
    on both traces), within an HBM budget small enough that admission waits
    for memory; the counts of requests that waited for memory and for a slot
    are reported."""
    import threading

    rng = np.random.Generator(np.random.PCG64(seed))
    pools = {L: _pool(L, pool_n, 3000 + L, distinct) for L in Ls}
    reqs = []
    for _ in range(n_req):
        L = int(rng.choice(Ls))
        N = int(max(1, min(5000, round(math.exp(rng.uniform(0, math.log(5000)))))))
        off = int(rng.integers(0, pool_n - N + 1))
        reqs.append((L, N, off))
    total = sum(r[1] for r in reqs)

    def plain(arrivals):
        ctx = api.Context(0)
        done = []
        t0 = time.perf_counter()
        for (L, N, off), ta in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if now < ta:
                time.sleep(ta - now)
            ref, imgs = pools[L]
            x = imgs[off:off + N].cuda()
            r = ref[None].cuda()
            rq, ra = api.tables(ctx, r, L, L)
            iq, ia = api.tables(ctx, x, L, L)
            res, _ = api.align_batch(ctx, rq, ra, iq, ia, L)
            res.cpu()
            done.append(time.perf_counter() - t0)
        ctx.close()
        return np.array(done)

    def served(arrivals, prec=1):
        ctx = api.Context(0)
        srv = api.Server(ctx, hbm_budget_bytes=budget, prec=prec, max_slots=max_slots,
                         max_per_step=max_per_step)
        tickets = [None] * len(reqs)
        done = np.zeros(len(reqs))
        t0 = time.perf_counter()

        def submitter():
            for i, ((L, N, off), ta) in enumerate(zip(reqs, arrivals)):
                now = time.perf_counter() - t0
                if now < ta:
                    time.sleep(ta - now)
                ref, imgs = pools[L]
                while True:
                    try:
                        tickets[i] = srv.submit(ref.numpy(), imgs[off:off + N].numpy())
                        break
                    except Exception as e:
                        if "BUSY" not in str(e):
                            raise
                        time.sleep(0.0005)

        th = threading.Thread(target=submitter)
        th.start()
        left = set(range(len(reqs)))
        while left:
            for i in list(left):
                if tickets[i] is not None and srv.poll(tickets[i]) is not None:
                    done[i] = time.perf_counter() - t0
                    left.discard(i)
            time.sleep(0.0002)
        th.join()
        st = srv.stats()
        srv.stop()
        ctx.close()
        return done, st

    zero = np.zeros(len(reqs))
    plain(zero[:8])  # warm-up
    d_plain = plain(zero)
    cap_req_s = len(reqs) / d_plain[-1]
    log(f"serving: plain saturated {d_plain[-1]:.2f} s")
    d_srv, st_sat = served(zero)
    log(f"serving: served saturated {d_srv.max():.2f} s")
    d_f32, st_f32 = served(zero, prec=0)
    log(f"serving: served FP32 saturated {d_f32.max():.2f} s")
    lam = 0.8 * cap_req_s
    arr = np.cumsum(rng.exponential(1.0 / lam, len(reqs)))
    arr -= arr[0]
    d_plain_l = plain(arr)
    log("serving: plain at fixed rate done")
    d_srv_l, st_l = served(arr)
    d_f32_l, st_f32_l = served(arr, prec=0)

    def lat(d):
        x = (d - arr) * 1e3
        return {"p50_ms": float(np.percentile(x, 50)), "p99_ms": float(np.percentile(x, 99)),
                "alignments_per_s": float(total / (d.max() - arr[0]))}

    def admission(st_a, st_b):
        return {"saturated": {"waited_memory": int(st_a["waited_memory"]),
                              "waited_slot": int(st_a["waited_slot"])},
                "at_rate": {"waited_memory": int(st_b["waited_memory"]),
                            "waited_slot": int(st_b["waited_slot"])}}

    def served_line(d_sat, st_a, d_rate, st_b):
        return {"saturated_alignments_per_s": float(total / d_sat.max()), **lat(d_rate),
                "steps": int(st_a["steps"]), "graph_launches": int(st_a["graph_launches"]),
                "arena_peak_bytes": int(st_a["arena_peak"]),
                "admission_waits": admission(st_a, st_b)}

    return {
        "workload": f"{len(reqs)} requests (seed {seed}), L in {list(Ls)}, N log-uniform "
                    f"[1, 5000] ({total} images), Poisson arrivals at {lam:.1f} req/s = 0.8 x "
                    f"plain capacity; HBM budget {budget / 2**30:.0f} GiB, {max_slots} slots, "
                    f"{max_per_step} requests per step",
        "served_bf16": served_line(d_srv, st_sat, d_srv_l, st_l),
        "served_fp32": served_line(d_f32, st_f32, d_f32_l, st_f32_l),
        "plain_fp32_one_at_a_time": {"saturated_alignments_per_s": float(total / d_plain.max()),
                                     **lat(d_plain_l)},
        "arrival_rate_req_per_s": lam,
        "latency_samples": len(reqs),
    }


def cpu_baseline(w, S, res32, res16, L, n, Q):
    """The FP64 oracle, untuned, on the first S images of the same workload;
    also reports GPU-vs-oracle parity on that sample."""
    from oracle import oracle as O
    from tests import parity

    S = min(S, len(w["imgs"]))
    t0 = time.perf_counter()
    o = O.align_images(w["ref"], w["imgs"][:S], n, Q, want_curve=True)
    dt = time.perf_counter() - t0
    out = {"value": S / dt, "unit": "alignments/s", "cores": O.num_threads(), "kind": "oracle",
           "sample": (f"all {S} images against the reference" if S == len(w["imgs"]) else
                      f"first {S} of the images against the reference") +
                     ", whole path (projection, quantiles, all lags, translation; FP64)",
           "seconds": dt}
    for name, r, tau in (("fp32", res32, parity.TAU_FP32), ("bf16_split", res16, parity.TAU_BF16)):
        sub = {k: v[:S] for k, v in r.items()}
        try:
            rep = parity.check(sub, o, L, tau, o["curve"])
            out[f"parity_{name}"] = f"{rep['pairs']} pairs ok, exact rotation {rep['exact_rot']}"
        except AssertionError as e:
            out[f"parity_{name}"] = "FAILED: " + str(e)[:300]
    truth = w["truth_theta"][:S]
    d = (res32["theta_rad"][:S] - truth + math.pi) % (2 * math.pi) - math.pi
    out["gpu_within_15deg_of_truth"] = float(np.mean(np.abs(d) <= math.radians(15)))
    return out


if __name__ == "__main__":
    main()
