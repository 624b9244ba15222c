"""Benchmark: one q-point of chi0(q, i omega) (all frequencies) plus the FP64
dielectric inverse, on one MI355X.

A step = chi0_accumulate (every frequency of the q-point) + dielectric_invert,
on synthetic inputs already resident in HBM.  Prints one JSON line.  The
step's inverse is the Hermitian positive definite sweep by default (eps =
1 - v^1/2 chi0 v^1/2 with chi0 negative semidefinite), redone with the
pivoted Gauss-Jordan inverse if a pivot is not positive; --inverse gj times
the pivoted inverse alone.

Default workload: npb = 2048, nk = 16, nocc = 200, nunocc = 1200, 12
Gauss-Legendre imaginary frequencies, complex64 Z (62.9 GB), BF16x3 split
path; the FP64 path is timed once on the same workload (complex128 Z) for the
FP64-vs-split comparison.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
# sources of each rank-K kernel (the traffic counters are valid while these are unchanged)
_LOWP = ("paper_2506_03477_amd/csrc/herk_lowp.hip", "paper_2506_03477_amd/csrc/herk_wgroup.hip",
         "paper_2506_03477_amd/csrc/herk_direct.hip", "paper_2506_03477_amd/csrc/bf16_tall.h",
         "paper_2506_03477_amd/csrc/herk_common.h", "paper_2506_03477_amd/csrc/common.h")
KERNEL_SOURCE = {"fp64": ("paper_2506_03477_amd/csrc/herk_fp64.hip", "paper_2506_03477_amd/csrc/herk_common.h"),
                 "fp32": _LOWP, "bf16x3": _LOWP}
STEP_INVERSE = {"hpd_fallback_gj": "HPD sweeps, pivoted Gauss-Jordan if a pivot is not positive",
                "gj": "pivoted Gauss-Jordan", "hpd": "HPD sweeps"}
KERNEL_NAME = {"fp64": "herk_fp64", "fp32": "herk_fp32", "bf16x3": "herk_bf16x3"}
CALIB_BYTES = 1 << 30   # plain device copy used to calibrate the byte counters
MFMA_DTYPE = {"fp64": "f64", "fp32": "f32", "bf16x3": "bf16"}
SPLIT_FACTOR = {"fp64": 1, "fp32": 1, "bf16x3": 3}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def zherk_flops(npb, npairs, nomega):
    """Algorithmic flops of chi0 for one q-point: a Hermitian rank-K update
    per frequency, 8 real flops per complex multiply-add on the lower
    triangle including the diagonal."""
    return 4.0 * npairs * npb * (npb + 1) * nomega


def inverse_flops(npb, nomega):
    """Complex LU + inverse (Gauss-Jordan) flops: 8 n^3 real per matrix."""
    return 8.0 * npb ** 3 * nomega


def lower_tile_count(npb, tp, tq):
    """Tiles of a tp x tq tiling holding an entry on or below the diagonal."""
    n = 0
    for r in range(-(-npb // tp)):
        last_row = min((r + 1) * tp, npb) - 1
        n += last_row // tq + 1
    return n


def executed_mfma_flops(npb, npairs, nomega, tile_p, tile_q, prec, diag_skip=False):
    """Matrix-core flops actually issued: whole tp x tq tiles holding
    lower-triangle entries (tiles on the diagonal are computed whole, or,
    with diag_skip, only their 32 x 32 blocks holding such entries), 8 real
    flops per complex MAC, times the number of split products."""
    if diag_skip:
        blocks = 0
        for r in range(-(-npb // tile_p)):
            last_row = min((r + 1) * tile_p, npb) - 1
            for c in range(last_row // tile_q + 1):
                for i in range(tile_p // 32):
                    for j in range(tile_q // 32):
                        blocks += (r * tile_p + 32 * i) // 32 >= (c * tile_q + 32 * j) // 32
        area = blocks * 32 * 32
    else:
        area = lower_tile_count(npb, tile_p, tile_q) * tile_p * tile_q
    return 8.0 * npairs * area * nomega * SPLIT_FACTOR[prec]


def size_sample(run, nmax, target_s):
    """Size an oracle sample to about target_s seconds: one warm-up call
    (thread pools, caches), a one-state probe, the sized run, and one resize
    (from the line through the probe and that run, so a fixed cost per call
    counts) if that run took under two thirds of the target, then a second,
    proportional resize if the first still fell that short.  run(n) returns
    the seconds (or a tuple whose first item is).  Returns (n, the last run's
    result)."""
    def secs(r):
        return r[0] if isinstance(r, tuple) else r

    run(1)
    r = run(1)
    t1 = secs(r)
    n = int(min(nmax, max(1, round(target_s / max(t1, 1e-4)))))
    if n > 1:
        r = run(n)
    t = secs(r)
    if t < (2.0 / 3.0) * target_s and n < nmax:
        if n > 1 and t > t1:           # seconds = a + b n through the probe and the sized run
            b = (t - t1) / (n - 1)
            a = max(0.0, t1 - b)
            n2 = round((target_s - a) / b)
        else:
            n2 = round(n * target_s / max(t, 1e-4))
        n = int(min(nmax, max(n + 1, n2)))
        r = run(n)
        t = secs(r)
        # a probe slowed by noise (a page-in, a busy core) undersizes the
        # line's slope: one more resize, in proportion, from the run itself
        if t < (2.0 / 3.0) * target_s and n < nmax:
            n = int(min(nmax, max(n + 1, round(n * target_s / max(t, 1e-4)))))
            r = run(n)
    return n, r


def cpu_baseline(wl, target_s=15.0):
    """Time the oracle on a bounded sample of the workload (first occupied
    states of the first block, all product-basis functions, all frequencies)
    and return its throughput in the metric's unit."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle

    blk = wl.blocks(0)[0]
    eo, eu = wl.energies(blk)

    def run(nocc_s):
        sub = blk.__class__(q=blk.q, spin=blk.spin, k=blk.k, nocc=nocc_s, nunocc=blk.nunocc,
                            wk=blk.wk, bid=blk.bid)
        z = wl.z_block(sub)            # the first nocc_s occupied rows of the block
        t0 = time.perf_counter()
        oracle.chi0_ref([(z, eo[:nocc_s], eu, blk.wk)], wl.npb, wl.omega, wl.delta_min)
        return time.perf_counter() - t0

    nocc_s, t_meas = size_sample(run, blk.nocc, target_s)
    flops = zherk_flops(wl.npb, nocc_s * blk.nunocc, wl.nomega)
    threads = 0
    for info in threadpool_info():
        if info.get("user_api") == "blas":
            threads = max(threads, int(info.get("num_threads", 0)))
    return {"value": flops / t_meas / 1e12, "unit": "TFLOP/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"{nocc_s} occupied x {blk.nunocc} unoccupied states of one k-block, "
                      f"npb={wl.npb}, all {wl.nomega} frequencies (FP64 chi0 only, "
                      f"{t_meas:.1f} s)",
            "seconds": t_meas}


def source_sha(prec):
    """Hash of the kernel's sources with comments and blank space removed, so
    the stored counters stay valid across comment-only edits."""
    import hashlib
    import re
    h = hashlib.sha256()
    for path in KERNEL_SOURCE[prec]:
        with open(os.path.join(ROOT, path), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def traffic_file(prec, workload_name):
    return os.path.join(ROOT, "profiles", f"traffic_{KERNEL_NAME[prec]}_{workload_name}.json")


def stored_traffic(prec, workload_name):
    """HBM bytes per launch from the stored counter runs, or None when there
    are none or the kernel's code has changed since they were taken."""
    tf = traffic_file(prec, workload_name)
    if not os.path.exists(tf):
        return None
    with open(tf) as f:
        t = json.load(f)
    if t.get("kernel_source_sha") != source_sha(prec):
        return None
    return round(t["traffic_bytes_per_launch"])


def _dispatch_counters(db, counter):
    """{kernel_name: [value per dispatch]} for one counter of a rocprofv3 --pmc run."""
    import sqlite3
    con = sqlite3.connect(db)
    out = {}
    for name, val in con.execute("select kernel_name, value from counters_collection "
                                 "where counter_name = ?", (counter,)):
        out.setdefault(name, []).append(float(val))
    return out


def summarize_pmc(fetch_db, write_db, prec, workload_name, command):
    """HBM bytes per launch of the rank-K kernel from FETCH_SIZE / WRITE_SIZE
    runs (KiB per dispatch), each scaled by what the same counter reads for a
    plain device copy of CALIB_BYTES (run by --copy-calibration)."""
    res = {"kernel": KERNEL_NAME[prec], "workload": workload_name, "command": command,
           "kernel_source_sha": source_sha(prec)}
    for counter, db in (("FETCH_SIZE", fetch_db), ("WRITE_SIZE", write_db)):
        per = _dispatch_counters(db, counter)
        herk = [v for k, v in per.items() if KERNEL_NAME[prec] in k]
        copy = [v for k, v in per.items() if "copy" in k.lower()]
        herk_vals = [x for vs in herk for x in vs]
        copy_vals = [x for vs in copy for x in vs]
        if not herk_vals or not copy_vals:
            raise SystemExit(f"{counter}: kernel or copy dispatches missing in {db}")
        kib_copy = max(copy_vals)                 # the 1 GiB calibration copy
        factor = (CALIB_BYTES / 1024.0) / kib_copy
        kib = sum(herk_vals) / len(herk_vals)
        res[counter] = {"kib_per_dispatch": kib, "copy_kib": kib_copy,
                        "scale": factor, "bytes_per_launch": kib * 1024.0 * factor}
    res["traffic_bytes_per_launch"] = (res["FETCH_SIZE"]["bytes_per_launch"] +
                                       res["WRITE_SIZE"]["bytes_per_launch"])
    path = traffic_file(prec, workload_name)
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print(f"wrote {path}")


def summarize_trace(db, out_path, command):
    """Short text summary (per-kernel calls, total and mean duration) of a
    rocprofv3 --kernel-trace run."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = list(con.execute("select name, total_calls, total_duration, average, percentage "
                            "from top_kernels"))
    with open(out_path, "w") as f:
        f.write(f"# rocprofv3 kernel-trace summary\n\ncommand: `{command}`\n\n")
        f.write("| kernel | calls | total ms | mean ms | % |\n|---|---|---|---|---|\n")
        for name, calls, tot, avg, pct in rows:   # top_kernels durations are in microseconds
            short = name.replace("(anonymous namespace)::", "").replace("void ", "")
            short = short.split("(")[0][:90]
            f.write(f"| {short} | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.4f} | {pct:.2f} |\n")
    print(f"wrote {out_path}")


def summarize_counters(db, out_path, command):
    """Per-kernel mean of every counter of a rocprofv3 --pmc run (text)."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = {}
    for name, counter, val in con.execute("select kernel_name, counter_name, value "
                                          "from counters_collection"):
        short = name.replace("(anonymous namespace)::", "").replace("void ", "").split("(")[0]
        rows.setdefault(short[:80], {}).setdefault(counter, []).append(float(val))
    counters = sorted({c for r in rows.values() for c in r})
    with open(out_path, "w") as f:
        f.write(f"# rocprofv3 counters (mean per dispatch)\n\ncommand: `{command}`\n\n")
        f.write("| kernel | dispatches | " + " | ".join(counters) + " |\n")
        f.write("|---|---|" + "---|" * len(counters) + "\n")
        for k, r in sorted(rows.items()):
            n = max(len(v) for v in r.values())
            vals = [f"{sum(r[c]) / len(r[c]):.4g}" if c in r else "" for c in counters]
            f.write(f"| {k} | {n} | " + " | ".join(vals) + " |\n")
    print(f"wrote {out_path}")


def sigx_cpu_baseline(wl, target_s=10.0):
    """The exchange oracle on a bounded sample: the first n' rows of one k-point."""
    from threadpoolctl import threadpool_info

    from oracle.sigx_oracle import sigx_ref

    blk = wl.blocks(0)[0]
    v = wl.coulomb(blk)

    def run(nocc_s):
        sub = blk.__class__(q=blk.q, spin=blk.spin, k=blk.k, nocc=nocc_s, nunocc=blk.nunocc,
                            wk=blk.wk, bid=blk.bid)
        z = wl.z_block(sub)
        t0 = time.perf_counter()
        sigx_ref([(z, v, blk.wk)], wl.npb)
        return time.perf_counter() - t0

    nocc_s, t_meas = size_sample(run, blk.nocc, target_s)
    flops = zherk_flops(wl.npb, nocc_s * blk.nunocc, 1)
    threads = 0
    for info in threadpool_info():
        if info.get("user_api") == "blas":
            threads = max(threads, int(info.get("num_threads", 0)))
    return {"value": flops / t_meas / 1e12, "unit": "TFLOP/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"{nocc_s} occupied x {blk.nunocc} product-basis rows of one k-point, "
                      f"nqp={wl.npb} ({t_meas:.1f} s)"}


def bench_sigx(args):
    """Exchange self-energy (Eq.(sigx)) of one q-point: one JSON line."""
    import torch

    from paper_2506_03477_amd import Context, SigxBlock, SigxProblem
    from synth import workload
    from synth.gpu import z_block_device

    wl = workload(5)
    prec = args.precision or "fp64"
    ztype = "c128" if prec == "fp64" else "c64"
    torch.cuda.set_device(0)
    ctx = Context(0)
    if args.tile >= 0:
        ctx.set_tile(prec, args.tile)
    log(f"generating {wl.name} inputs ({ztype}) on the GPU")
    blocks = []
    for blk in wl.blocks(0):
        z = z_block_device(wl, blk, "cuda", ztype=ztype)
        blocks.append(SigxBlock(z, torch.from_numpy(wl.coulomb(blk)).cuda(), blk.wk))
    out = torch.empty((wl.npb, wl.npb), dtype=torch.complex128, device="cuda")
    prob = SigxProblem(blocks, out)
    rows = sum(b.npairs for b in wl.blocks(0))
    for _ in range(args.warmup):
        ctx.sigx_accumulate([prob], precision=prec)
    ctx.sync()
    ctx.profile_enable(True)
    ctx.profile_read()
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(args.steps):
        ctx.sigx_accumulate([prob], precision=prec)
    b.record(stream)
    b.synchronize()
    ctx.sync()
    ms = a.elapsed_time(b) / args.steps
    kern_ms, n = ctx.profile_read()
    kern_avg = kern_ms / n if n else None
    flops = zherk_flops(wl.npb, rows, 1)
    tinfo = ctx.tile_info(prec, ctx.last_tile(prec))
    roof = None
    if kern_avg:
        ach = flops / (kern_avg * 1e-3) / 1e12
        exe = executed_mfma_flops(wl.npb, rows, 1, tinfo["tile_p"], tinfo["tile_q"], prec) / \
            (kern_avg * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[prec], 4), "traffic": None,
                "kernel": f"herk_{prec}", "kernel_ms": round(kern_avg, 3),
                "executed_mfma_tflops": round(exe, 3),
                "executed_mfma_frac": round(exe / PEAK_TFLOPS[prec], 4)}
    cpu = None if args.no_cpu_baseline else sigx_cpu_baseline(wl)
    print(json.dumps({
        "metric": "Sigma^x TFLOP/s per q-point (exchange self-energy, Eq. sigx)",
        "value": round(flops / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": MFMA_DTYPE[prec] if prec != "bf16x3" else "bf16x3", "data": "synthetic",
        "config": {"workload": wl.name, "nqp": wl.npb, "nk": wl.nk, "nocc": wl.nocc,
                   "nmu": wl.nunocc, "ztype": ztype, "path": prec,
                   "tile": [tinfo["tile_p"], tinfo["tile_q"]]},
        "roofline": roof, "cpu_baseline": cpu}), flush=True)
    ctx.close()


def sigc_flops(nqp, nall, nmu, nomega):
    """Algorithmic flops of one block of the imaginary-axis correlation
    self-energy: the first contraction (rows (n', n), columns nu, contraction
    (i, mu)) and the second (nqp x nqp, contraction (n', nu)), 8 flops per
    complex multiply-add."""
    first = 8.0 * nall * nqp * nmu * nomega * nmu
    second = 8.0 * nqp * nqp * nall * nmu
    return first, second


def sigc_cpu_baseline(wl, target_s=15.0):
    """The correlation oracle on a bounded sample: the first n' states of one
    k-point at full nqp, product-basis size and mesh."""
    from threadpoolctl import threadpool_info

    from oracle.sigc_oracle import sigc_ref

    blk = wl.blocks(0)[0]
    wc = wl.wc_block(blk)
    eps_mid = wl.eps_mid(blk)
    eps_qp = wl.eps_qp()

    def run(nall_s):
        sub = blk.__class__(q=blk.q, spin=blk.spin, k=blk.k, nocc=nall_s, nunocc=blk.nunocc,
                            wk=blk.wk, bid=blk.bid)
        z = wl.z_block(sub)
        t0 = time.perf_counter()
        sigc_ref([(z, wc, eps_mid[:nall_s], blk.wk)], eps_qp, wl.omega)
        return time.perf_counter() - t0

    nall_s, t_meas = size_sample(run, blk.nocc, target_s)
    flops = sum(sigc_flops(wl.npb, nall_s, blk.nunocc, wl.nomega))
    threads = 0
    for info in threadpool_info():
        if info.get("user_api") == "blas":
            threads = max(threads, int(info.get("num_threads", 0)))
    return {"value": flops / t_meas / 1e12, "unit": "TFLOP/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"{nall_s} of {blk.nocc} intermediate states of one k-point, nqp={wl.npb}, "
                      f"{blk.nunocc} product-basis functions, {wl.nomega} frequencies "
                      f"({t_meas:.1f} s)"}


def bench_sigc(args):
    """Imaginary-axis correlation self-energy (Eq.(sigci)) of one q-point,
    FP64 path: one JSON line."""
    import torch

    from paper_2506_03477_amd import Context, SigcBlock, SigcProblem
    from synth import workload
    from synth.gpu import device_sigc_workload

    wl = workload(6)
    prec = args.precision or "fp64"
    if prec not in ("fp64", "bf16x3"):
        raise SystemExit("the correlation self-energy runs on the FP64 and BF16x3 paths")
    torch.cuda.set_device(0)
    ctx = Context(0)
    if args.tile >= 0:
        ctx.sigc_set_variant(args.tile)
    log(f"generating {wl.name} inputs on the GPU")
    blks, eps_qp = device_sigc_workload(wl)
    out = torch.empty((wl.npb, wl.npb), dtype=torch.complex128, device="cuda")
    prob = SigcProblem([SigcBlock(z, wc, em, wk) for z, wc, em, wk, _ in blks], eps_qp,
                       wl.omega_array(), out)
    first = second = 0.0
    exe_first = 0.0
    tp, kq = (256, 16) if prec == "bf16x3" else (128, 8)
    split = 3.0 if prec == "bf16x3" else 1.0
    for b in wl.blocks(0):
        f1, f2 = sigc_flops(wl.npb, b.nocc, b.nunocc, wl.nomega)
        first += f1
        second += f2
        rows = -(-b.nocc * wl.npb // 128) * 128
        cols = -(-b.nunocc // tp) * tp
        exe_first += split * 8.0 * rows * cols * wl.nomega * (-(-b.nunocc // kq) * kq)
    for _ in range(args.warmup):
        ctx.sigc_accumulate([prob], precision=prec)
    ctx.sync()
    ctx.profile_enable(True)
    ctx.profile_read()
    stream = torch.cuda.current_stream()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for s in range(args.steps):
        ctx.sigc_accumulate([prob], precision=prec)
    b.record(stream)
    b.synchronize()
    ctx.sync()
    ms = a.elapsed_time(b) / args.steps
    kern_ms, n = ctx.profile_read()
    roof = None
    if n:
        launches_per_step = n / args.steps
        kern_avg = kern_ms / n
        per_launch = first / launches_per_step
        ach = per_launch / (kern_avg * 1e-3) / 1e12
        exe = exe_first / launches_per_step / (kern_avg * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[prec], 4), "traffic": None,
                "kernel": ("sigc_bf16x3_kernel" if prec == "bf16x3" else "sigc_gemm_kernel")
                          + " (first contraction)", "kernel_ms": round(kern_avg, 3),
                "launches_per_step": launches_per_step,
                "executed_mfma_tflops": round(exe, 3),
                "executed_mfma_frac": round(exe / PEAK_TFLOPS[prec], 4)}
    extra = {}
    if prec != "fp64" and not args.no_fp64_compare:
        # The FP64 path on the same inputs (it is checked against the oracle
        # by the GPU tests): its time (median of 3 after one untimed call)
        # and the relative Frobenius error of the timed output against it.
        ctx.profile_enable(False)
        out64 = torch.empty_like(out)
        prob64 = SigcProblem(prob.blocks, eps_qp, wl.omega_array(), out64)
        ctx.sigc_accumulate([prob64], precision="fp64")
        ctx.sync()
        runs = []
        for r in range(3):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.sigc_accumulate([prob64], precision="fp64")
            b.record(stream)
            b.synchronize()
            runs.append(a.elapsed_time(b))
        fp64_ms = sorted(runs)[1]
        err = float((torch.linalg.norm(out - out64) / torch.linalg.norm(out64)).item())
        extra = {"fp64_ms_per_q": round(fp64_ms, 3), "fp64_ms_runs": [round(x, 3) for x in runs],
                 "split_speedup_vs_fp64": round(fp64_ms / ms, 3),
                 "max_rel_err": {"sigma_c": float(f"{err:.3e}"),
                                 "vs": "FP64 path on the same inputs (relative Frobenius "
                                       "error, whole matrix)"}}
        log(f"rel err vs FP64: {err:.3e}; FP64 {fp64_ms:.1f} ms")
    cpu = None if args.no_cpu_baseline else sigc_cpu_baseline(wl)
    print(json.dumps({
        "metric": "I^c TFLOP/s per q-point (imaginary-axis correlation self-energy, Eq. sigci)",
        "value": round((first + second) / (ms * 1e-3) / 1e12, 3), "unit": "TFLOP/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == "fp64" else "bf16x3", "data": "synthetic",
        "config": {"workload": wl.name, "nqp": wl.npb, "nk": wl.nk, "nall": wl.nocc,
                   "nmu": wl.nunocc, "nomega": wl.nomega, "path": prec,
                   "variant": args.tile if args.tile >= 0 else 1},
        "flops_first": first, "flops_second": second,
        "roofline": roof, "cpu_baseline": cpu, **extra}), flush=True)
    ctx.close()


HIST_SIGMA = 0.015


def hist_cpu_baseline(wl, edges, target_s=10.0):
    """The histogram oracle on a bounded sample: the first occupied states of
    one k-block at full npb, into a window of 32 bins around the median
    transition energy (the oracle holds every bin as a dense npb x npb
    matrix, so all bins of the mesh at npb = 2048 would not fit in host
    memory)."""
    import numpy as np
    from threadpoolctl import threadpool_info

    import oracle.hist_oracle as H

    blk = wl.blocks(0)[0]
    eo, eu = wl.energies(blk)
    med = float(np.median(eu[None, :] - eo[:, None]))
    j0 = max(0, int(np.searchsorted(edges, med)) - 16)
    win = edges[j0:j0 + 33]

    def run(nocc_s):
        sub = blk.__class__(q=blk.q, spin=blk.spin, k=blk.k, nocc=nocc_s, nunocc=blk.nunocc,
                            wk=blk.wk, bid=blk.bid)
        z = wl.z_block(sub).astype(np.complex128)
        t0 = time.perf_counter()
        H.hist_ref([(z, eo[:nocc_s], eu, blk.wk)], wl.npb, win, HIST_SIGMA)
        dt = time.perf_counter() - t0
        bins, _ = H.pair_bins(eo[:nocc_s], eu, win, HIST_SIGMA, 0.0, blk.wk)
        return dt, int((bins >= 0).sum())

    nocc_s, (t_meas, nrec) = size_sample(run, blk.nocc, target_s)
    flops = zherk_flops(wl.npb, nrec, 1)
    threads = 0
    for info in threadpool_info():
        if info.get("user_api") == "blas":
            threads = max(threads, int(info.get("num_threads", 0)))
    return {"value": flops / t_meas / 1e12, "unit": "TFLOP/s", "cores": threads or os.cpu_count(),
            "kind": "oracle",
            "sample": f"{nocc_s} occupied x {blk.nunocc} unoccupied states of one k-block, "
                      f"32 bins around the median transition ({nrec} records), npb={wl.npb} "
                      f"({t_meas:.1f} s)"}


def bench_hist(args):
    """chi0 at every imaginary frequency through the histogram route
    (binning, per-bin rank-K updates, Hilbert transform): one JSON line."""
    import torch

    from paper_2506_03477_amd import Block, Context, HistSpec, Problem
    from synth import hist_edges, workload
    from synth.gpu import device_workload

    wl = workload(args.workload)
    prec = args.precision or wl.paths[0]
    ztype = "c128" if prec == "fp64" else "c64"
    emax = max(wl.unocc_range[1] - wl.occ_range[0], 1e-3) * 1.05
    edges = hist_edges(emax)
    torch.cuda.set_device(0)
    ctx = Context(0)
    log(f"generating {wl.name} inputs ({ztype}) on the GPU")
    blks, omega, _ = device_workload(wl, 0, ztype=ztype)
    out = torch.empty((wl.nomega, wl.npb, wl.npb), dtype=torch.complex128, device="cuda")
    prob = Problem([Block(z, eo, eu, wk) for z, eo, eu, wk, _ in blks], omega, out)
    spec = HistSpec(edges, HIST_SIGMA)
    if args.tile >= 0:
        ctx.set_tile(prec, args.tile)
    for _ in range(args.warmup):
        ctx.chi0_hist_accumulate([prob], [spec], precision=prec, delta_min=wl.delta_min)
    ctx.sync()
    ctx.profile_enable(True)
    ctx.profile_read()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ctx.chi0_hist_accumulate([prob], [spec], precision=prec, delta_min=wl.delta_min)
    ctx.sync()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    kern_ms, n = ctx.profile_read()
    records, bins_used = ctx.hist_stats()
    flops = zherk_flops(wl.npb, records, 1)
    direct = zherk_flops(wl.npb, wl.npairs(0), wl.nomega)
    roof = None
    if n:
        kern_avg = kern_ms / n
        ach = flops / (kern_avg * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[prec], 4), "traffic": None,
                "kernel": f"herk_{prec} (gathered rows)", "kernel_ms": round(kern_avg, 3)}
    extra = {}
    if prec != "fp64" and not args.no_fp64_compare:
        # The same values in FP64 (Z upcast exactly): the histogram route's
        # precision error (this path against the FP64 histogram route) and
        # its method error (the FP64 histogram route against the direct FP64
        # sum over pairs), relative Frobenius per frequency.
        # Memory: the BF16x3 route's pre-split rows are released with its
        # context, and each complex64 block is dropped once upcast.
        import numpy as np
        ctx.close()
        ctx = Context(0)
        src = list(prob.blocks)
        del prob, blks
        blocks64 = []
        while src:
            b = src.pop(0)
            blocks64.append(Block(b.z.to(torch.complex128), b.eps_occ, b.eps_unocc, b.wk))
            del b
            torch.cuda.empty_cache()
        h64 = torch.empty_like(out)
        ctx.chi0_hist_accumulate([Problem(blocks64, omega, h64)], [spec], precision="fp64",
                                 delta_min=wl.delta_min)
        d64 = torch.empty_like(out)
        ctx.chi0_accumulate([Problem(blocks64, omega, d64)], precision="fp64",
                            delta_min=wl.delta_min)
        ctx.sync()

        def rel(x, y):
            d = torch.linalg.norm((x - y).reshape(wl.nomega, -1), dim=1)
            return (d / torch.linalg.norm(y.reshape(wl.nomega, -1), dim=1)).cpu().numpy()

        e_prec, e_meth = rel(out, h64), rel(h64, d64)
        extra["max_rel_err"] = {
            "chi0_vs_fp64_hist": float(f"{np.max(e_prec):.3e}"),
            "fp64_hist_vs_direct": float(f"{np.max(e_meth):.3e}"),
            "vs": "the FP64 histogram route and the direct FP64 sum on the same values "
                  "(complex64 Z upcast to complex128; relative Frobenius per frequency)"}
        log(f"rel err vs FP64 histogram route {np.max(e_prec):.3e}; FP64 histogram route vs "
            f"direct sum {np.max(e_meth):.3e}")
        del blocks64, h64, d64
    cpu = None if args.no_cpu_baseline else hist_cpu_baseline(wl, edges)
    print(json.dumps({
        "metric": "chi0 ms per q-point (all omega) through the histogram route (Eq. impolf + Eq. hilbert)",
        "value": round(ms, 3), "unit": "ms", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": False, "scaling": "weak",
        "vs_baseline": None, "dtype": MFMA_DTYPE[prec] if prec != "bf16x3" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": wl.name, "npb": wl.npb, "nomega": wl.nomega, "path": prec,
                   "bins": len(edges) - 1, "bins_used": bins_used, "sigma": HIST_SIGMA,
                   "mesh": "5e-6 Ha * 1.03^j"},
        "records": records, "records_per_pair": round(records / wl.npairs(0), 4),
        "rank_k_tflops": round(flops / (ms * 1e-3) / 1e12, 3),
        "direct_equivalent_tflops": round(direct / (ms * 1e-3) / 1e12, 3),
        "roofline": roof, "cpu_baseline": cpu, **extra}), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, help="synthetic workload index (0-4)")
    ap.add_argument("--precision", default=None, help="fp64 | fp32 | bf16x3 (default: the "
                    "workload's split path)")
    ap.add_argument("--no-fp64-compare", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--graph", action="store_true", help="replay chi0 from a hipGraph")
    ap.add_argument("--inverse", default="hpd_fallback_gj", choices=("hpd_fallback_gj", "gj", "hpd"),
                    help="the step's FP64 inverse of eps")
    ap.add_argument("--tile", type=int, default=-1,
                    help="tile configuration index (default: the library's default)")
    ap.add_argument("--flush", type=int, default=0,
                    help="FP32 run length in pairs between flushes to the FP64 partials (0: the "
                         "library's per-problem length, min(4096, 4 sqrt K))")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (byte-counter calibration)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DB", "WRITE_DB"),
                    help="write profiles/traffic_*.json from two rocprofv3 --pmc databases")
    ap.add_argument("--summarize-trace", nargs=2, metavar=("TRACE_DB", "OUT"),
                    help="write a text summary of a rocprofv3 --kernel-trace database")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("PMC_DB", "OUT"),
                    help="write a text table of every counter of a rocprofv3 --pmc database")
    ap.add_argument("--command", default="", help="profiled command (for the summaries)")
    ap.add_argument("--sigx", action="store_true",
                    help="time the exchange self-energy (Eq. sigx) instead of chi0")
    ap.add_argument("--sigc", action="store_true",
                    help="time the imaginary-axis correlation self-energy (Eq. sigci)")
    ap.add_argument("--hist", action="store_true",
                    help="time chi0 through the histogram route (Eq. impolf + Eq. hilbert)")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(args.summarize_counters[0], args.summarize_counters[1], args.command)
        return
    if args.summarize_pmc or args.summarize_trace:
        from synth import workload as _wl
        name = _wl(args.workload).name
        if args.summarize_pmc:
            summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1],
                          args.precision or _wl(args.workload).paths[0], name, args.command)
        if args.summarize_trace:
            summarize_trace(args.summarize_trace[0], args.summarize_trace[1], args.command)
        return

    if args.sigx and args.gpus == 1:
        bench_sigx(args)
        return
    if args.sigc and args.gpus == 1:
        bench_sigc(args)
        return
    if args.hist and args.gpus == 1:
        bench_hist(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU; --gpus must be 1 (sharding "
                                   "q-points and k-blocks over GPUs is designed, not built)"}))
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2506_03477_amd import Block, Context, Problem
    from synth import workload
    from synth.gpu import device_workload

    wl = workload(args.workload)
    prec = args.precision or wl.paths[0]
    dev = "cuda:0"
    torch.cuda.set_device(0)
    ctx = Context(0)
    if ctx.tile_count(prec) <= 0:
        raise SystemExit(f"precision {prec} has no kernel in this library")
    if args.tile >= 0:
        ctx.set_tile(prec, args.tile)
    if args.flush:
        ctx.set_flush(args.flush)
    ztype = "c128" if prec == "fp64" else "c64"

    if args.copy_calibration:
        src = torch.ones(CALIB_BYTES // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy done")
    log(f"generating {wl.name} inputs ({ztype}, {wl.nq} q-point(s)) on the GPU")
    t0 = time.time()
    probs, chis, invs = [], [], []
    npairs = 0
    for q in range(wl.nq):
        blks, omega, vsqrt = device_workload(wl, q, dev, ztype=ztype)
        npairs += sum(b[4].npairs for b in blks)
        chi = torch.empty((wl.nomega, wl.npb, wl.npb), dtype=torch.complex128, device=dev)
        chis.append(chi)
        invs.append(torch.empty_like(chi))
        probs.append(Problem([Block(z, eo, eu, wk) for z, eo, eu, wk, _ in blks], omega, chi))
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s")

    def invert_all():
        for chi, inv in zip(chis, invs):
            ctx.dielectric_invert(vsqrt, chi, inv, method=args.inverse)

    def step():
        ctx.chi0_accumulate(probs, precision=prec, delta_min=wl.delta_min, graph=args.graph)
        invert_all()

    for i in range(args.warmup):
        step()
        ctx.sync()
        log(f"warmup {i + 1}/{args.warmup} done")

    stream = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ctx.profile_enable(not args.graph)
    ctx.profile_read()
    torch.cuda.synchronize()
    ev[0].record(stream)
    chi_ms = 0.0
    for i in range(args.steps):
        e_a = torch.cuda.Event(enable_timing=True)
        e_b = torch.cuda.Event(enable_timing=True)
        e_a.record(stream)
        ctx.chi0_accumulate(probs, precision=prec, delta_min=wl.delta_min, graph=args.graph)
        e_b.record(stream)
        invert_all()
        e_b.synchronize()
        chi_ms += e_a.elapsed_time(e_b)
        log(f"step {i + 1}/{args.steps}")
    ev[1].record(stream)
    torch.cuda.synchronize()
    ctx.sync()
    total_ms = ev[0].elapsed_time(ev[1])
    kern_ms, nlaunch = ctx.profile_read()
    ms_per_step = total_ms / args.steps
    tinfo = ctx.tile_info(prec, ctx.last_tile(prec))
    tile = tinfo["tile_p"]

    flops = zherk_flops(wl.npb, npairs, wl.nomega)
    value = flops / (ms_per_step * 1e-3) / 1e12
    kern_avg_ms = kern_ms / nlaunch if nlaunch else None
    roof = None
    if kern_avg_ms:
        ach = flops / (kern_avg_ms * 1e-3) / 1e12
        exe = executed_mfma_flops(wl.npb, npairs, wl.nomega, tinfo["tile_p"], tinfo["tile_q"],
                                  prec, ctx.tile_diag_skip(prec, ctx.last_tile(prec))) / \
            (kern_avg_ms * 1e-3) / 1e12
        traffic = stored_traffic(prec, wl.name)
        roof = {"bound": "mfma", "achieved": round(ach, 3), "peak": PEAK_TFLOPS[prec],
                "unit": "TFLOP/s", "frac": round(ach / PEAK_TFLOPS[prec], 4), "traffic": traffic,
                "algorithmic_bytes": int(npairs * wl.npb * (16 if prec == "fp64" else 8)
                                         + wl.nomega * wl.npb * (wl.npb + 1) // 2 * 16),
                "kernel": f"herk_{prec}", "kernel_ms": round(kern_avg_ms, 3),
                "hbm_gbs": round(traffic / (kern_avg_ms * 1e-3) / 1e9, 1) if traffic else None,
                "executed_mfma_tflops": round(exe, 3),
                "executed_mfma_frac": round(exe / PEAK_TFLOPS[prec], 4)}

    inv_ms = {}
    # the step's own inverse last, so that invs holds the timed step's kind of output
    for method in [m for m in ("gj", "hpd", "hpd_fallback_gj") if m != args.inverse] + [args.inverse]:
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for chi, inv in zip(chis, invs):
            ctx.dielectric_invert(vsqrt, chi, inv, method=method)
        b.record(stream)
        b.synchronize()
        ctx.sync()
        inv_ms[method] = round(a.elapsed_time(b) / wl.nq, 3)
    log(f"inverse ms per q: {inv_ms}")

    extra = {"ms_per_q_chi0": round(chi_ms / args.steps / wl.nq, 3),
             "ms_per_q_inverse_gj": inv_ms["gj"], "ms_per_q_inverse_hpd": inv_ms["hpd"],
             "ms_per_q_inverse_hpd_fallback_gj": inv_ms["hpd_fallback_gj"],
             "ms_per_q_chi0_plus_inverse": round(ms_per_step / wl.nq, 3),
             "nq_per_step": wl.nq, "tile": [tinfo["tile_p"], tinfo["tile_q"]],
             "tile_index": ctx.last_tile(prec), "npairs": npairs}
    if args.flush:
        extra["flush_pairs"] = args.flush
    if wl.paths and "fp64" in wl.paths and prec != "fp64" and not args.no_fp64_compare:
        # The FP64 path on the same values (the complex64 Z upcast exactly to
        # complex128): its time for the speed ratio (median of 3 after one
        # untimed call) and, per frequency, the error of the timed output
        # (chi0 of the last step and its inverse) against it.  The FP64 path
        # itself is checked against the oracle on whole matrices by the
        # full-size tests.
        log("FP64 comparison: upcasting the complex64 inputs to complex128")
        probs64 = []
        for q in range(wl.nq):
            probs64.append(Problem([Block(b.z.to(torch.complex128), b.eps_occ, b.eps_unocc, b.wk)
                                    for b in probs[q].blocks], probs[q].omega,
                                   torch.empty_like(chis[q])))
        ctx.profile_enable(False)
        ctx.set_flush(0)
        ctx.chi0_accumulate(probs64, precision="fp64", delta_min=wl.delta_min)
        ctx.sync()
        fp64_runs = []
        for r in range(3):
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record(stream)
            ctx.chi0_accumulate(probs64, precision="fp64", delta_min=wl.delta_min)
            b.record(stream)
            b.synchronize()
            fp64_runs.append(a.elapsed_time(b))
            log(f"FP64 comparison: run {r + 1}/3 {fp64_runs[-1]:.0f} ms")
        fp64_ms = float(np.median(fp64_runs))
        extra["fp64_ms_per_q_chi0"] = round(fp64_ms / wl.nq, 3)
        extra["fp64_ms_runs"] = [round(x / wl.nq, 3) for x in fp64_runs]
        extra["fp64_tflops"] = round(flops / (fp64_ms * 1e-3) / 1e12, 3)
        extra["split_speedup_vs_fp64"] = round(fp64_ms / (chi_ms / args.steps), 3)
        for p64 in probs64:
            p64.blocks = []
        torch.cuda.empty_cache()
        e_chi, e_inv = [], []
        for q in range(wl.nq):
            inv64 = torch.empty_like(chis[q])
            ctx.dielectric_invert(vsqrt, probs64[q].chi0, inv64, method=args.inverse)
            ctx.sync()
            for x, y, acc in ((chis[q], probs64[q].chi0, e_chi), (invs[q], inv64, e_inv)):
                d = torch.linalg.norm((x - y).reshape(wl.nomega, -1), dim=1)
                n = torch.linalg.norm(y.reshape(wl.nomega, -1), dim=1)
                acc.append((d / n).cpu().numpy())
            del inv64
        e_chi = np.max(np.stack(e_chi), axis=0)
        e_inv = np.max(np.stack(e_inv), axis=0)
        extra["max_rel_err"] = {
            "chi0": float(f"{e_chi.max():.3e}"), "eps_inv": float(f"{e_inv.max():.3e}"),
            "vs": "FP64 path on the same complex64 inputs upcast to complex128 "
                  "(relative Frobenius error per frequency, whole matrices)",
            "per_omega_chi0": [float(f"{x:.3e}") for x in e_chi],
            "per_omega_eps_inv": [float(f"{x:.3e}") for x in e_inv]}
        log(f"max rel err vs FP64: chi0 {e_chi.max():.3e}, eps^-1 {e_inv.max():.3e}")
        del probs64

    cpu = None
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        cpu = cpu_baseline(wl)
        log(f"oracle sample took {cpu.pop('seconds'):.1f} s")

    out = {
        "metric": "chi0 TFLOP/s and ms per q-point (all omega), FP64 vs split-precision at "
                  "<=1e-6 rel err",
        "value": round(value, 3),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": MFMA_DTYPE[prec] if prec != "bf16x3" else "bf16x3",
        "data": "synthetic",
        "config": {"workload": wl.name, "npb": wl.npb, "nq": wl.nq, "nk": wl.nk, "nspin": wl.nspin,
                   "nocc": wl.nocc, "nunocc": wl.nunocc, "nomega": wl.nomega,
                   "ztype": ztype, "path": prec,
                   "step": "chi0 (all omega) + FP64 inverse of eps",
                   "inverse": STEP_INVERSE[args.inverse]},
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
