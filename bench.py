#!/usr/bin/env python3
"""Benchmark of the NNCP hot path on one MI355X.

Workload: a 512 x 512 x 512 nonnegative tensor (rank-32 uniform factors plus
5% |Gaussian| noise), rank R = 32, HALS updates.  One step = one sweep of
Algorithm 1 over all three modes (MTTKRP through the dimension tree, Gram /
Hadamard, HALS update, normalisation, relative error).  The timed region runs
`--steps` sweeps (50 by default, the workload's sweep count) from the start
factors, for two forms of the same problem on the same GPU:
  fp32  FP32 tensor, FP32 matrix-core partial MTTKRP
  bf16  the tensor rounded once to BF16, BF16 matrix-core partial MTTKRP with
        FP32 accumulation (the reported `value`)
Inputs are resident in HBM before timing starts.  The reported rate is the
median of `--reps` timed replays (each from the start factors) of the sweeps
captured as one HIP graph; per-kernel times (for the roofline) come from HIP
events around every launch in a further pass of the same sweeps with plain
launches.  Beside them: the device's streaming-read ceiling
(nncp_read_probe), the BF16 partial MTTKRPs with the last-level cache evicted
first, and the same kernels on the 8 GiB 256^4 workload (DRAM-only rates);
and the oracle on the host's CPU share.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
METRIC = "MTTKRP HBM GB/s and NNCP sweeps/s, BF16-MFMA vs FP32 at stated rel error"
WORKLOAD = "512x512x512 rank-32 uniform + 5% |gaussian| noise, R=32, HALS, {n} sweeps"
ANCHOR = "256x256x256x256 bf16 rank-64 exponential + 2% |gaussian| noise, R=64, HALS"
KERNEL_SRC = os.path.join(ROOT, "paper_1909_01149_amd", "csrc", "partial_mttkrp.hip")
CAT_NAMES = ["gemm_left", "gemm_right", "krp", "mttv", "update"]


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def source_sha() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def read_traffic(kernel: str):
    """HBM bytes per launch from the committed counter summary, or None if it
    is missing or was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha") != source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_form(nn, torch, X, H0, steps, warmup, algo, reps):
    """Warm up; time `reps` replays of `steps` sweeps from the start factors
    (one HIP graph; the factors are reset before each replay, outside the
    timed region) and take the median; then time the same sweeps again with
    plain launches and per-launch HIP events (the per-kernel times)."""
    dev = X.device
    H = [h.clone() for h in H0]
    lam = torch.ones(H0[0].shape[1], dtype=torch.float64, device=dev)
    ctx = nn.Context(X, H, lam)
    if warmup > 0:
        ctx.sweep(algo, warmup)
    torch.cuda.synchronize()

    def reset():
        for f, h0 in zip(ctx.factors, H0):
            f.copy_(h0)
        ctx.lam.fill_(1.0)
        ctx.refresh_grams()
        torch.cuda.synchronize()

    n = max(1, steps)
    rel = torch.empty(n, dtype=torch.float64, device=dev)
    reset()
    ctx.capture(algo, n, rel)
    torch.cuda.synchronize()
    times, walls, rels = [], [], []
    for _ in range(max(1, reps)):
        reset()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record()
        ctx.sweep(algo, n, rel)
        e1.record()
        torch.cuda.synchronize()
        walls.append(time.perf_counter() - t0)
        times.append(e0.elapsed_time(e1))
        rels.append(rel.clone())
    ms = statistics.median(times)
    reps_equal = all(torch.equal(rels[0], r) for r in rels[1:])
    # same sweeps, plain launches with per-launch events
    rel2 = torch.empty(n, dtype=torch.float64, device=dev)
    reset()
    ctx.timers_enable(True)
    f0, f1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    f0.record()
    ctx.sweep(algo, n, rel2)
    f1.record()
    torch.cuda.synchronize()
    ms_eager = f0.elapsed_time(f1)
    cat_ms, cat_n = ctx.timers_read()
    ctx.timers_enable(False)
    # the factors are left at the result of `steps` sweeps from the start
    same = bool(torch.equal(rel, rel2)) and reps_equal
    return ctx, dict(ms=ms, ms_reps=times, wall_s=statistics.median(walls),
                     ms_eager_timed=ms_eager, relerr=rel.cpu().tolist()[:steps],
                     graph_equals_eager=same, cat_ms=cat_ms, cat_n=cat_n)


def gemm_bytes(dims, R, xbytes, side):
    """Algorithmic bytes of one partial MTTKRP: the tensor once plus the
    output temporary (the Khatri-Rao operand is formed on chip)."""
    import math
    I = math.prod(dims)
    m = dims[0] * dims[1]
    k = dims[2]
    out_rows = m if side == 0 else k
    return I * xbytes + out_rows * R * 4


def cpu_baseline(X32, H0, algo_oracle, nthreads, min_seconds=10.0, max_sweeps=30):
    """The oracle on the host: HALS sweeps of the same 512^3 tensor in FP64,
    run one after another from the same start until min_seconds have passed
    (at most max_sweeps), reported as sweeps/s."""
    import numpy as np
    import oracle
    Xh = X32.double().cpu().numpy().reshape(-1)
    Hh = [h.double().cpu().numpy() for h in H0]
    R = Hh[0].shape[1]
    lam = np.ones(R)
    n = 0
    t0 = time.perf_counter()
    while True:
        Hh, lam, _, _ = oracle.sweeps(Xh, Hh, lam, algo_oracle, 1, nthreads=nthreads)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or n >= max_sweeps:
            break
    return dict(value=n / dt, unit="sweeps/s", cores=nthreads, kind="oracle",
                sample=f"{n} HALS sweeps (3 MTTKRPs by definition + updates each) of the same "
                       f"512^3 tensor in FP64, {dt:.1f} s on {nthreads} host threads")


# ---------------------------------------------------------------------------
# the other workloads (parity cases of the test suite), timed on request:
# `python bench.py --configs c1,c3,c4,c5` writes one JSON object per line to
# stdout; the default run is unaffected
# ---------------------------------------------------------------------------

def _side_bytes(dims, R, xbytes, S, side):
    import math
    I = math.prod(dims)
    rows = math.prod(dims[:S]) if side == 0 else math.prod(dims[S:])
    return I * xbytes + rows * R * 4


def _timed_sweeps(nn, torch, ctx, algo, n):
    """n sweeps as one graph replay (rate), then the same count eagerly with
    per-launch events (per-kernel means); returns rate, relerr, category times."""
    dev = ctx.X.device
    ctx.sweep(algo, 1)
    rel = torch.empty(n, dtype=torch.float64, device=dev)
    ctx.capture(algo, n, rel)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    ctx.sweep(algo, n, rel)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    rel_list = rel.cpu().tolist()
    ctx.timers_enable(True)
    ctx.sweep(algo, n)
    torch.cuda.synchronize()
    cat_ms, cat_n = ctx.timers_read()
    ctx.timers_enable(False)
    return ms / n, rel_list, cat_ms, cat_n


def _gemm_rates(dims, R, xbytes, S, cat_ms, cat_n):
    out = {}
    for side, name in ((0, "gemm_left"), (1, "gemm_right")):
        if cat_n[side]:
            avg = cat_ms[side] / cat_n[side]
            out[name] = {"avg_ms": avg, "GBps": _side_bytes(dims, R, xbytes, S, side) / (avg / 1e3) / 1e9}
    return out


def run_configs(names):
    import torch
    import nncp_inputs as gen
    import paper_1909_01149_amd as nn
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    for name in names:
        log(f"config {name}")
        if name == "c1":
            w = gen.workload1()
            X = torch.from_numpy(w["X"]).to(dev)
            H = [torch.from_numpy(h).to(dev) for h in w["H0"]]
            ctx = nn.Context(X, H)
            mps, rel, cm, cn = _timed_sweeps(nn, torch, ctx, nn.NNCP_MU, 20)
            res = dict(config="c1", workload=w["name"], sweeps=20, ms_per_sweep=mps,
                       sweeps_per_s=1e3 / mps, final_relerr=rel[-1],
                       **_gemm_rates(w["dims"], w["R"], 8, ctx.split(), cm, cn))
            ctx.close()
        elif name == "c2bpp":
            # the 512^3 BF16 workload, 50 sweeps with HALS and with BPP from
            # the same start; BPP's time to reach HALS's final error
            w = gen.workload2(keep_fp32=False)
            H0 = [torch.from_numpy(h).float().to(dev) for h in w["H0"]]
            res = dict(config="c2bpp", workload=w["name"], sweeps=50)
            algos = ((nn.NNCP_HALS, "hals"), (nn.NNCP_BPP, "bpp"), (nn.NNCP_ADMM, "admm"),
                     (nn.NNCP_NES, "nes"), (nn.NNCP_NES_OUTER, "nes_outer"))
            for algo, an in algos:
                ctx = nn.Context(w["Xbf16"], [h.clone() for h in H0])
                mps, rel, cm, cn = _timed_sweeps(nn, torch, ctx, algo, 50)
                res[an] = dict(ms_per_sweep=mps, sweeps_per_s=1e3 / mps, final_relerr=rel[-1],
                               relerr_every_10=rel[9::10], update_ms_per_sweep=cm[4] / 50)
                ctx.close()
            # error trajectories from the start factors (the timed replays
            # above began after one warm-up sweep)
            traj = {}
            for algo, an in algos:
                ctx = nn.Context(w["Xbf16"], [h.clone() for h in H0])
                traj[an] = ctx.sweep(algo, 50).cpu().tolist()
                ctx.close()
            target = traj["hals"][-1]
            res["hals_relerr_after_50"] = target
            res["hals_ms_for_50_sweeps"] = 50 * res["hals"]["ms_per_sweep"]
            for an in ("bpp", "admm", "nes", "nes_outer"):
                rl = traj[an]
                res[f"{an}_relerr_after_50"] = rl[-1]
                k = next((i + 1 for i, r in enumerate(rl) if r <= target), None)
                res[f"{an}_sweeps_to_hals_final_relerr"] = k
                res[f"{an}_ms_to_hals_final_relerr"] = None if k is None else k * res[an]["ms_per_sweep"]
            del w
        elif name == "c3":
            w = gen.workload3()
            H = [torch.from_numpy(h).float().to(dev) for h in w["H0"]]
            ctx = nn.Context(w["X"], H)
            n = 5
            mps, rel, cm, cn = _timed_sweeps(nn, torch, ctx, nn.NNCP_HALS, n)
            res = dict(config="c3", workload=w["name"], sweeps=n, ms_per_sweep=mps,
                       sweeps_per_s=1e3 / mps, relerr=rel,
                       **_gemm_rates(w["dims"], w["R"], 2, ctx.split(), cm, cn))
            ctx.close()
            del w
        elif name == "c4":
            w = gen.workload4()
            H0 = [torch.from_numpy(h).float().to(dev) for h in w["H0"]]
            res = dict(config="c4", workload=w["name"], sweeps=30)
            for algo, an in ((nn.NNCP_MU, "mu"), (nn.NNCP_HALS, "hals")):
                ctx = nn.Context(w["X"], [h.clone() for h in H0])
                mps, rel, cm, cn = _timed_sweeps(nn, torch, ctx, algo, 30)
                res[an] = dict(ms_per_sweep=mps, sweeps_per_s=1e3 / mps, final_relerr=rel[-1],
                               **_gemm_rates(w["dims"], w["R"], 2, ctx.split(), cm, cn))
                ctx.close()
            del w
        elif name == "c5":
            w = gen.workload5(keep_bf16=True)
            H0 = [torch.from_numpy(h).float().to(dev) for h in w["H0"]]
            res = dict(config="c5", workload=w["name"])
            for form in ("X32", "Xbf16"):
                ctx = nn.Context(w[form], [h.clone() for h in H0])
                grads, loss = ctx.grad()
                torch.cuda.synchronize()
                reps = 10
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(reps):
                    ctx.grad(grads, loss)
                e1.record()
                torch.cuda.synchronize()
                gms = e0.elapsed_time(e1) / reps
                L0 = float(loss.item())
                t0 = time.perf_counter()
                lh, eh = ctx.pgd(100)
                torch.cuda.synchronize()
                pgd_s = time.perf_counter() - t0
                res[form] = dict(ms_per_gradient=gms, gradients_per_s=1e3 / gms,
                                 bytes_per_gradient_GBps=(w[form].numel() * w[form].element_size()
                                                          * 2 / (gms / 1e3) / 1e9),
                                 loss0=L0, loss_after_100_pgd=float(lh[-1]),
                                 pgd_100_steps_s=pgd_s,
                                 accepted_steps=int(sum(1 for e in eh if e > 0)))
                ctx.close()
            del w
        else:
            raise SystemExit(f"unknown config {name}")
        print(json.dumps(res), flush=True)
        torch.cuda.empty_cache()


# ---------------------------------------------------------------------------
# counter summaries for profiles/ (run on the CSVs that rocprofv3 wrote)
# ---------------------------------------------------------------------------

COPY_PROBE_BYTES = 1 << 28
KERNEL_PATTERNS = {
    # (kernel file name, substring tests on the demangled / mangled name)
    "bf16_gemm_right": lambda n: "k_gemm_right_mfma" in n and not any(
        t in n for t in ("<float", "<double", "_Float16", "DF16_")),
    "bf16_gemm_left": lambda n: "k_gemm_left_mfma" in n and ("DF16b" in n or "__bf16" in n),
    "fp32_gemm_right": lambda n: "k_gemm_right_mfma<float" in n,
    "fp32_gemm_left": lambda n: "k_gemm_left_mfma<float" in n,
}


def _read_counter_csv(path, counter):
    import csv
    rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
    return {int(r["Dispatch_Id"]): (r["Kernel_Name"], float(r["Counter_Value"])) for r in rows}


def summarize_counters(fetch_csv, write_csv, cmd_fetch, cmd_write, prefix="",
                       workload="512x512x512, R=32, HALS (bench.py default workload)"):
    """Write profiles/traffic_<kernel>.txt: HBM bytes per launch from FETCH_SIZE
    and WRITE_SIZE (KiB per dispatch), each scaled by what the counter reads for
    the --copy-probe device copy of COPY_PROBE_BYTES (found as the copy dispatch
    that writes exactly that many bytes; the two runs dispatch the same kernels
    in the same order, so dispatch ids match)."""
    import statistics
    fe = _read_counter_csv(fetch_csv, "FETCH_SIZE")
    wr = _read_counter_csv(write_csv, "WRITE_SIZE")
    # the probe is the first copy of exactly COPY_PROBE_BYTES (it runs before
    # anything else; the 256^4 workload is generated in copies of that size)
    probe = [d for d, (n, v) in wr.items() if "copyBuffer" in n and abs(v * 1024 - COPY_PROBE_BYTES) < 1]
    if not probe:
        raise SystemExit("copy probe dispatch not found")
    d0 = min(probe)
    f_read = COPY_PROBE_BYTES / (fe[d0][1] * 1024)
    f_write = COPY_PROBE_BYTES / (wr[d0][1] * 1024)
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    for kname, test in KERNEL_PATTERNS.items():
        ids = [d for d, (n, _) in fe.items() if test(n) and d in wr]
        if not ids:
            continue
        fkib = statistics.mean(fe[d][1] for d in ids)
        wkib = statistics.mean(wr[d][1] for d in ids)
        hbm = (fkib * f_read + wkib * f_write) * 1024
        with open(os.path.join(ROOT, "profiles", f"traffic_{prefix}{kname}.txt"), "w") as fh:
            fh.write(f"# HBM traffic per launch of the {kname.replace('_', ' ')} partial MTTKRP kernel\n")
            fh.write(f"# workload: {workload}\n")
            fh.write(f"# fetch run: {cmd_fetch}\n# write run: {cmd_write}\n")
            fh.write(f"# summarised with: python bench.py --summarize-counters <fetch csv> <write csv>\n")
            fh.write(f"# calibration: the --copy-probe device copy of {COPY_PROBE_BYTES} bytes reads "
                     f"{fe[d0][1]:.1f} KiB FETCH_SIZE and {wr[d0][1]:.1f} KiB WRITE_SIZE\n")
            fh.write(f"dispatches = {len(ids)}\n")
            fh.write(f"fetch_kib_per_dispatch = {fkib:.1f}\nwrite_kib_per_dispatch = {wkib:.1f}\n")
            fh.write(f"read_scale = {f_read:.5f}\nwrite_scale = {f_write:.5f}\n")
            fh.write(f"hbm_bytes_per_launch = {hbm:.0f}\n")
            fh.write(f"kernel_source_sha = {source_sha()}\n")
        print(f"{prefix}{kname}: {len(ids)} dispatches, {hbm / 2**20:.1f} MiB per launch")


def summarize_mfma(csv_path, cmd):
    """MFMA utilisation per partial-MTTKRP kernel from a rocprofv3 --pmc run of
    SQ_VALU_MFMA_BUSY_CYCLES (summed over every SIMD) and GRBM_GUI_ACTIVE
    (summed over the 8 XCDs): busy / (GUI cycles per XCD x 1024 SIMDs)."""
    import collections
    import csv
    by = collections.defaultdict(dict)
    for r in csv.DictReader(open(csv_path)):
        d = by[int(r["Dispatch_Id"])]
        d[r["Counter_Name"]] = float(r["Counter_Value"])
        d["name"] = r["Kernel_Name"]
    lines = [f"# MFMA utilisation of the partial MTTKRP kernels, 512x512x512 R=32 HALS workload",
             f"# command: {cmd}",
             f"# summarised with: python bench.py --summarize-mfma <counter_collection.csv>",
             f"# kernel_source_sha = {source_sha()}",
             f"# util = SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 * 1024 SIMDs)",
             " dispatches  mfma_busy_cycles  gui_active_per_xcd   util  kernel"]
    for key, test in KERNEL_PATTERNS.items():
        rows = [v for v in by.values() if test(v["name"])]
        if not rows:
            continue
        mb = sum(v.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) for v in rows) / len(rows)
        ga = sum(v.get("GRBM_GUI_ACTIVE", 0.0) for v in rows) / len(rows) / 8.0
        lines.append(f" {len(rows):10d}  {mb:16.0f}  {ga:18.0f}  {mb / (ga * 1024):5.3f}  {key}")
    with open(os.path.join(ROOT, "profiles", "mfma_util_512cube.txt"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def summarize_trace(stats_csv, cmd, out_name="kernels_512cube_hals.txt",
                    title="512x512x512 R=32 HALS workload (FP32 and BF16 forms)"):
    """Write profiles/<out_name>: the library's kernels from a rocprofv3
    --kernel-trace --stats run (calls, average and total duration)."""
    import csv
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# rocprofv3 kernel statistics, {title}",
             f"# command: {cmd}",
             f"# summarised with: python bench.py --summarize-trace <kernel_stats.csv>",
             f"# kernel_source_sha = {source_sha()}",
             f"{'calls':>6} {'avg_us':>9} {'total_us':>10}  kernel"]
    for r in rows:
        name = r["Name"]
        if "nncp" not in name:
            continue
        short = name.replace("nncp::", "").split("(")[0]
        lines.append(f"{int(r['Calls']):6d} {float(r['AverageNs']) / 1e3:9.2f} "
                     f"{float(r['TotalDurationNs']) / 1e3:10.1f}  {short}")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _prof_args(csv_path):
    """`-d <dir> -o <prefix>` of the rocprofv3 run that wrote csv_path (the
    directory holding it and the file-name prefix before the first '_')."""
    d = os.path.relpath(os.path.dirname(os.path.abspath(csv_path)), ROOT)
    prefix = os.path.basename(csv_path).split("_")[0]
    return f"-d {d} -o {prefix}"


def main():
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-trace":
        pa = _prof_args(sys.argv[2])
        if len(sys.argv) > 3 and sys.argv[3] == "nls":
            # the c2bpp configuration: HALS, BPP, ADMM and NES on the BF16 512^3 tensor
            summarize_trace(sys.argv[2], "rocprofv3 --kernel-trace --stats --output-format csv "
                            f"{pa} -- python3 bench.py --configs c2bpp",
                            "kernels_512cube_nls.txt",
                            "512x512x512 R=32 BF16 tensor, 50 sweeps each of HALS, BPP, ADMM, NES "
                            "and NES with the outer step "
                            "(timed and untimed passes)")
            return
        if len(sys.argv) > 3 and sys.argv[3] == "grad":
            summarize_trace(sys.argv[2], "rocprofv3 --kernel-trace --stats --output-format csv "
                            f"{pa} -- python3 bench.py --configs c5", "kernels_64x5_grad.txt",
                            "64x64x64x64x64 R=32 gradient workload (FP32 and BF16 tensors: "
                            "timed gradients and 100 PGD steps each)")
            return
        if len(sys.argv) > 3 and sys.argv[3] == "anchor":
            summarize_trace(sys.argv[2], "rocprofv3 --kernel-trace --stats --output-format csv "
                            f"{pa} -- python3 bench.py --anchor-only", "kernels_256x4_hals.txt",
                            ANCHOR + " (10 graph-replayed and 10 event-timed sweeps)")
            return
        summarize_trace(sys.argv[2], "rocprofv3 --kernel-trace --stats --output-format csv "
                        f"{pa} -- python3 bench.py --steps 10 --warmup 2 --reps 5 "
                        "--no-cpu-baseline --no-dram")
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-counters":
        fetch_csv, write_csv = sys.argv[2], sys.argv[3]
        anchor = len(sys.argv) > 4 and sys.argv[4] == "anchor"
        run = ("-- python3 bench.py --anchor-only --copy-probe" if anchor else
               "-- python3 bench.py --steps 3 --warmup 1 --reps 1 --no-cpu-baseline --no-dram "
               "--copy-probe")
        cmd_f = f"rocprofv3 --pmc FETCH_SIZE --output-format csv {_prof_args(fetch_csv)} {run}"
        cmd_w = f"rocprofv3 --pmc WRITE_SIZE --output-format csv {_prof_args(write_csv)} {run}"
        if anchor:
            summarize_counters(fetch_csv, write_csv, cmd_f, cmd_w, "anchor_", ANCHOR)
        else:
            summarize_counters(fetch_csv, write_csv, cmd_f, cmd_w)
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--summarize-mfma":
        summarize_mfma(sys.argv[2], "rocprofv3 --pmc SQ_VALU_MFMA_BUSY_CYCLES GRBM_GUI_ACTIVE "
                       f"--output-format csv {_prof_args(sys.argv[2])} -- python3 bench.py "
                       "--steps 3 --warmup 1 --reps 1 --no-cpu-baseline --no-dram")
        return
    if len(sys.argv) > 1 and sys.argv[1] == "--configs":
        run_configs(sys.argv[2].split(","))
        return
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--reps", type=int, default=5, help="timed replays (median reported)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dram", action="store_true",
                    help="skip the measurements beside the 512^3 sweep (LLC-cold 512^3 products, "
                         "256^4 workload, 64^5 gradient)")
    ap.add_argument("--anchor-only", action="store_true",
                    help="only the 256^4 measurement (for its counter runs)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 256 MiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: this benchmark measures a single MI355X; --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    # the 256^4 and 64^5 measurements run first, each in a process of its own
    # started before this one touches the GPU: in one process, the 8 GiB
    # workload measured after other device memory had been allocated and
    # freed ran about 6% slower in both partial MTTKRPs (GEMM-L 5,671
    # against 6,066 GB/s), which depends on the process's allocation
    # history, not on the kernels
    anchor_child = grad_child = None
    if not args.no_dram and not args.anchor_only:
        anchor_child = anchor_subprocess()
        grad_child = gradient_subprocess()

    import torch
    import nncp_inputs as gen
    import paper_1909_01149_amd as nn

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_probe:
        src = torch.empty(COPY_PROBE_BYTES, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    if args.anchor_only:
        print(json.dumps({"dram_anchor": dram_anchor(nn, torch, gen, dev)}), flush=True)
        return

    log("generating 512^3 workload on the GPU")
    w = gen.workload2(device="cuda:0", keep_fp32=False)
    dims, R = w["dims"], w["R"]
    H0 = [torch.from_numpy(h).float().to(dev) for h in w["H0"]]
    torch.cuda.synchronize()

    res = {}
    ctxs = {}
    for form, X in (("fp32", w["X32"]), ("bf16", w["Xbf16"])):
        log(f"timing {form}: {args.warmup} warmup + {args.reps} x {args.steps} sweeps")
        ctx, r = run_form(nn, torch, X, H0, args.steps, args.warmup, nn.NNCP_HALS, args.reps)
        r["paths"] = [ctx.gemm_path(0), ctx.gemm_path(1)]
        res[form] = r
        ctxs[form] = ctx
        log(form, f"{r['ms'] / max(1, args.steps):.4f} ms/sweep (median of {len(r['ms_reps'])})",
            "cat_ms", [round(x, 3) for x in r["cat_ms"]],
            "launches", r["cat_n"], "final relerr", r["relerr"][-1] if r["relerr"] else None)

    # BF16 run's final error measured against the unrounded FP32 tensor
    rel_bf16_vs_fp32 = None
    if args.steps > 0:
        c32 = ctxs["fp32"]
        cb = ctxs["bf16"]
        c32.set_factors(cb.factors, cb.lam)
        rel_bf16_vs_fp32 = float(c32.cp_loss()[1].item())

    steps = max(1, args.steps)
    b = res["bf16"]
    f = res["fp32"]
    sweeps_bf16 = steps / (b["ms"] / 1e3)
    sweeps_fp32 = steps / (f["ms"] / 1e3)

    def gbps(form, side):
        r = res[form]
        n = r["cat_n"][side]
        if n == 0:
            return None, None
        avg_ms = r["cat_ms"][side] / n
        xb = 2 if form == "bf16" else 4
        return gemm_bytes(dims, R, xb, side) / (avg_ms / 1e3) / 1e9, avg_ms

    mt = {}
    for form in ("fp32", "bf16"):
        for side, name in ((0, "gemm_left"), (1, "gemm_right")):
            g, a = gbps(form, side)
            mt[f"{form}_{name}"] = {"GBps": g, "avg_ms": a}

    log("streaming-read ceiling")
    ceiling = stream_ceiling(nn, torch, dev)
    cold = None
    if not args.no_dram:
        log("LLC-cold partial MTTKRPs")
        cold = llc_cold_gemms(nn, torch, ctxs["bf16"], dims, R)
    for c in ctxs.values():
        c.close()
    del ctxs

    # dominant kernel of the reported (bf16) form
    dom_side = 0 if b["cat_ms"][0] >= b["cat_ms"][1] else 1
    dom_name = CAT_NAMES[dom_side]
    ach, avg_ms = gbps("bf16", dom_side)
    traffic = read_traffic(f"bf16_{dom_name}")
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": (ach / HBM_PEAK_GBPS) if ach else None, "traffic": traffic,
            "kernel": f"bf16 {dom_name} partial MTTKRP", "avg_launch_ms": avg_ms,
            "algorithmic_bytes_per_launch": gemm_bytes(dims, R, 2, dom_side),
            "frac_of_stream_read_ceiling": ach / ceiling["ceiling_GBps"],
            "note": "the 256 MiB BF16 tensor fits the 256 MB last-level cache, so this rate is "
                    "partly cache bandwidth; llc_cold and dram_anchor give the DRAM-only rates"}

    anchor = None
    if not args.no_dram:
        anchor = anchor_child

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        info = host_info()
        log(f"timing the oracle on {info['threads']} host threads "
            f"({info['cpu_model']}, {info['logical_cpus']} logical CPUs)")
        cpu = cpu_baseline(w["X32"], H0, oracle.HALS, info["threads"])
        cpu["cpu_model"] = info["cpu_model"]
        cpu["host_logical_cpus"] = info["logical_cpus"]
        cpu["threads_from"] = info["threads_from"]

    out = {
        "metric": METRIC,
        "value": sweeps_bf16,
        "unit": "sweeps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": b["ms"] / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded; rank-32 uniform factors + 5% |gaussian| noise)",
        "config": {"workload": WORKLOAD.format(n=args.steps), "dims": dims, "R": R, "algo": "hals",
                   "tensor_dtype": "bf16", "accumulate": "fp32", "factors": "fp32",
                   "krp_operand": "bf16 hi+lo", "parallelism": "single GPU",
                   "timed_replays": args.reps, "statistic": "median"},
        "fp32_form": {"sweeps_per_s": sweeps_fp32, "ms_per_step": f["ms"] / steps,
                      "ms_per_step_reps": [t / steps for t in f["ms_reps"]],
                      "final_relerr": f["relerr"][-1] if f["relerr"] else None,
                      "ms_per_step_eager_timed": f["ms_eager_timed"] / steps},
        "bf16_form": {"sweeps_per_s": sweeps_bf16,
                      "ms_per_step_reps": [t / steps for t in b["ms_reps"]],
                      "final_relerr": b["relerr"][-1] if b["relerr"] else None,
                      "final_relerr_vs_fp32_tensor": rel_bf16_vs_fp32,
                      "ms_per_step_eager_timed": b["ms_eager_timed"] / steps},
        "graph_replay_equals_eager": bool(b["graph_equals_eager"] and f["graph_equals_eager"]),
        "bf16_speedup_over_fp32": sweeps_bf16 / sweeps_fp32,
        "mttkrp": mt,
        "category_ms_per_sweep": {form: {CAT_NAMES[k]: res[form]["cat_ms"][k] / steps for k in range(5)}
                                  for form in res},
        "wall_s": {form: res[form]["wall_s"] for form in res},
        "stream_read": ceiling,
        "llc_cold": cold,
        "dram_anchor": anchor,
        "gradient": grad_child,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def host_info():
    """CPU model, logical CPUs, and the oracle's thread count: OMP_NUM_THREADS
    when set (the host's CPU share for this GPU), else the CPUs this process
    may run on."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        threads, src = min(int(env), avail), "OMP_NUM_THREADS"
    else:
        threads, src = avail, "sched_getaffinity"
    return dict(cpu_model=model, logical_cpus=os.cpu_count(), threads=threads, threads_from=src)


def stream_ceiling(nn, torch, dev, sizes=(1 << 28, 1 << 32), iters=10, wgs=(4096, 8192, 16384)):
    """Streaming-read rate (nncp_read_probe, best of a few grid sizes) of a
    256 MiB buffer (about the last-level cache) and of a 4 GiB one (DRAM);
    the 4 GiB rate is the attainable ceiling reported beside the 8 TB/s
    datasheet figure."""
    out = {}
    for nbytes in sizes:
        buf = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        best = 0.0
        for wg in wgs:
            for _ in range(3):
                nn.nncp_read_probe(buf, wg)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(iters):
                nn.nncp_read_probe(buf, wg)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / iters
            best = max(best, nbytes / (ms / 1e3) / 1e9)
        out[f"{nbytes >> 20}MiB_GBps"] = best
        del buf
    out["ceiling_GBps"] = out[f"{sizes[-1] >> 20}MiB_GBps"]
    out["ceiling_frac_of_8TBps"] = out["ceiling_GBps"] / HBM_PEAK_GBPS
    out["probe"] = "nncp_read_probe: 16-byte non-temporal loads, 8 in flight per lane, best of %s workgroups" % (list(wgs),)
    torch.cuda.empty_cache()
    return out


def llc_cold_gemms(nn, torch, ctx, dims, R, reps=5):
    """The BF16 512^3 partial MTTKRPs with the last-level cache evicted first
    (a streaming read of another 1 GiB before each product: clean lines, so
    the product pays no write-back), timed by the library's events: the
    DRAM-only rate of the headline kernels."""
    flush = torch.ones(1 << 28, dtype=torch.float32, device=ctx.X.device)
    ctx.timers_enable(True)
    for k in range(reps):
        for mode in (0, 2):
            nn.nncp_read_probe(flush)
            ctx.mttkrp(mode)
    ms, n = ctx.timers_read()
    ctx.timers_enable(False)
    del flush
    out = {}
    for side, name in ((0, "gemm_left"), (1, "gemm_right")):
        avg = ms[side] / n[side]
        gb = gemm_bytes(dims, R, 2, side) / (avg / 1e3) / 1e9
        out[name] = {"avg_ms": avg, "GBps": gb, "frac": gb / HBM_PEAK_GBPS, "launches": n[side]}
    return out


def child_json(argv, what):
    """Run `bench.py <argv>` as a child process and return the last JSON
    line it prints (its log lines pass through to stderr)."""
    import subprocess
    log(f"{what} in a child process")
    p = subprocess.run([sys.executable, os.path.abspath(__file__)] + argv,
                       stdout=subprocess.PIPE, stderr=None, text=True, timeout=900)
    if p.returncode != 0:
        raise RuntimeError(f"the {what} measurement failed (exit {p.returncode})")
    lines = [ln for ln in p.stdout.splitlines() if ln.startswith("{")]
    if not lines:
        raise RuntimeError(f"the {what} measurement printed no result")
    return json.loads(lines[-1])


def anchor_subprocess():
    """The dram_anchor record of `bench.py --anchor-only`, run as a child."""
    return child_json(["--anchor-only"], "256^4 workload")["dram_anchor"]


def gradient_subprocess():
    """The 64^5 R = 32 gradient (`bench.py --configs c5`, run as a child):
    gradients/s of the BF16 tensor (one fused pass over X) and the FP32
    tensor (two passes), each the mean of 10 back-to-back gradients."""
    r = child_json(["--configs", "c5"], "64^5 gradient")
    out = {"workload": r["workload"], "R": 32}
    for key, form in (("Xbf16", "bf16"), ("X32", "fp32")):
        out[form] = {k: r[key][k] for k in ("ms_per_gradient", "gradients_per_s",
                                             "loss0", "loss_after_100_pgd", "pgd_100_steps_s")}
    return out


def dram_anchor(nn, torch, gen, dev, nsweeps=10):
    """The 256^4 BF16 R = 64 HALS workload (8 GiB, far beyond the last-level
    cache): sweeps/s by graph replay, and the partial MTTKRPs' event-timed
    rates (algorithmic bytes: the tensor once plus the output temporary)."""
    log("generating the 256^4 workload on the GPU")
    w = gen.workload3(device=str(dev))
    H = [torch.from_numpy(h).float().to(dev) for h in w["H0"]]
    ctx = nn.Context(w["X"], H)
    mps, rel, cm, cn = _timed_sweeps(nn, torch, ctx, nn.NNCP_HALS, nsweeps)
    rates = _gemm_rates(w["dims"], w["R"], 2, ctx.split(), cm, cn)
    for name in rates:
        rates[name]["frac"] = rates[name]["GBps"] / HBM_PEAK_GBPS
        rates[name]["bytes"] = _side_bytes(w["dims"], w["R"], 2, ctx.split(),
                                           0 if name == "gemm_left" else 1)
        rates[name]["traffic"] = read_traffic(f"anchor_bf16_{name}")
    ctx.close()
    del w, H
    torch.cuda.empty_cache()
    log(f"256^4: {mps:.3f} ms/sweep, " + ", ".join(
        f"{k} {v['GBps']:.0f} GB/s" for k, v in rates.items()))
    return {"workload": ANCHOR, "sweeps": nsweeps, "ms_per_sweep": mps, "sweeps_per_s": 1e3 / mps,
            "relerr": rel, **rates}


if __name__ == "__main__":
    main()
