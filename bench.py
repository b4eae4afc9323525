"""Benchmark: Richardson-Lucy deconvolution throughput on one MI355X.

A step is one complete deconvolution of one synthetic volume: reset the
estimate to u0 = mean(d) and run the configured number of RL iterations
(rl_iterate through the C ABI).  The headline workload is the 256x512x512
organoid-scale volume with 50 iterations, whose working set (about 1.1 GB) is
larger than the chip's 256 MB last-level cache, so its passes stream from HBM.
The 128x256x256 widefield-like volume (100 iterations) fits that cache; it is
reported beside the headline as `mall_resident`, not as an HBM figure.

Printed: one JSON line with value = voxel-iterations per second (whole job,
inputs resident in HBM), a roofline object for the dominant kernel, and the FP64
oracle timed on the host cores on a bounded sample of the headline workload.
The roofline's kernel duration is the average of that kernel's back-to-back
launches in a committed rocprofv3 kernel trace of this benchmark (used only
while the trace was taken on the current kernel source); the duration measured
live here with HIP events around every launch is reported beside it.

`python bench.py --rocprof-summary TRACE_DIR [FETCH_DIR WRITE_DIR] --out FILE`
turns the CSV output of rocprofv3 runs of this benchmark (a kernel trace, and
optionally FETCH_SIZE and WRITE_SIZE counter runs) into the summary table that
the roofline reads.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0  # MI355X HBM3E, datasheet
KERNEL_SOURCE = os.path.join(ROOT, "paper_2510_14143_amd", "csrc", "rl_kernels.hip")
PROFILES = os.path.join(ROOT, "profiles")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def optional_leg(name, fn):
    """Runs one of the secondary workloads.  A failure is logged with its traceback
    and recorded in the workload's place, so that the headline line is still printed."""
    try:
        return fn()
    except Exception as e:  # any failure of a secondary workload
        import traceback
        traceback.print_exc()
        log(f"{name} failed: {e!r}")
        return {"error": f"{type(e).__name__}: {e}"}


def kernel_bytes(shape) -> dict:
    """Algorithmic HBM bytes per launch of each kernel kind (compulsory reads + writes)."""
    nz, ny, nx = shape
    nvox = nz * ny * nx
    spec = nz * ny * (nx // 2 + 1) * 8  # valid half-spectrum bytes
    real = nvox * 4
    return {
        "x_r2c": real + spec,
        "x_c2r": spec + real,
        "x_ratio": spec + real + spec,
        # update: spectrum in, u in, u out, spectrum out (absent on the last iteration)
        "x_update": spec + real + real + spec,
        "x_update_last": spec + real + real,
        "y": 2 * spec,
        "z_otf": 3 * spec,
    }


def source_hash() -> str:
    with open(KERNEL_SOURCE, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


# ---------------------------------------------------------------------------
# rocprofv3 summaries
# ---------------------------------------------------------------------------
B2B_GAP_NS = 1000  # a launch starting less than this after the previous kernel ended
COPY_BYTES = 1 << 30  # the copy probe moves this many bytes each way per launch
_ROW = re.compile(r"^\| `(?P<name>[^`]+)` \| (?P<threads>\d+) \| (?P<n>\d+) \| "
                  r"(?P<avg>[0-9.]+) \| (?P<nb>\d+) \| (?P<bavg>[0-9.]+|nan) \| "
                  r"(?P<rd>[0-9.eE+]+|nan) \| (?P<wr>[0-9.eE+]+|nan) \|$")


def kernel_short_name(name: str) -> str:
    """'void rlmi::k_pencil<8, 0, 1024, 0>(HIP_vector_type<float, 2u>*, ...)' ->
    'k_pencil<8, 0, 1024, 0>' (namespaces, return type and parameter list dropped)."""
    n = name.strip().strip('"')
    if n.startswith("void "):
        n = n[5:]
    depth = 0
    for i, ch in enumerate(n):  # cut at the parameter list (outside template brackets)
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            n = n[:i]
            break
    head, sep, tail = n.partition("<")
    return head.split("::")[-1] + sep + tail


def _csv_rows(directory: str, suffix: str) -> list:
    import csv
    rows = []
    for root, _, files in os.walk(directory):
        for f in sorted(files):
            if f.endswith(suffix):
                with open(os.path.join(root, f), newline="") as fh:
                    rows.extend(csv.DictReader(fh))
    return rows


def _threads(row: dict) -> int:
    if row.get("Grid_Size") not in (None, ""):
        return int(row["Grid_Size"])
    return (int(row.get("Grid_Size_X") or 1) * int(row.get("Grid_Size_Y") or 1)
            * int(row.get("Grid_Size_Z") or 1))


def trace_table(trace_dir: str) -> dict:
    """Per (kernel, threads): launch count, average duration, and the same over the
    back-to-back launches (started < B2B_GAP_NS after the previous kernel on the queue
    ended), from a rocprofv3 kernel-trace CSV."""
    rows = _csv_rows(trace_dir, "kernel_trace.csv")
    if not rows:
        raise FileNotFoundError(f"no *kernel_trace.csv under {trace_dir}")
    by_queue = {}
    for r in rows:
        q = r.get("Queue_Id") or r.get("Stream_Id") or "0"
        by_queue.setdefault(q, []).append(
            (int(r["Start_Timestamp"]), int(r["End_Timestamp"]),
             kernel_short_name(r["Kernel_Name"]), _threads(r)))
    out = {}
    for launches in by_queue.values():
        launches.sort()
        prev_end = None
        for start, end, name, threads in launches:
            e = out.setdefault((name, threads), {"n": 0, "ns": 0, "nb": 0, "bns": 0})
            e["n"] += 1
            e["ns"] += end - start
            if prev_end is not None and start - prev_end < B2B_GAP_NS:
                e["nb"] += 1
                e["bns"] += end - start
            prev_end = end if prev_end is None else max(prev_end, end)
    return out


def counter_table(pmc_dir: str, counter: str) -> dict:
    """Per (kernel, threads): mean value of one rocprofv3 counter per dispatch."""
    acc = {}
    for r in _csv_rows(pmc_dir, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = (kernel_short_name(r["Kernel_Name"]), _threads(r))
        s, n = acc.get(k, (0.0, 0))
        acc[k] = (s + float(r["Counter_Value"]), n + 1)
    return {k: s / n for k, (s, n) in acc.items()}


def rocprof_summary(trace_dir: str, fetch_dir=None, write_dir=None, title: str = "",
                    commands=(), src_hash=None) -> str:
    """Markdown summary of one profiled benchmark command: per kernel and thread
    count, launches and durations from the kernel trace, and HBM read / write bytes
    per launch from FETCH_SIZE / WRITE_SIZE (KiB per dispatch), each scaled so that
    the library's copy kernel reads and writes exactly its known 1 GiB."""
    tt = trace_table(trace_dir)
    fetch = counter_table(fetch_dir, "FETCH_SIZE") if fetch_dir else {}
    write = counter_table(write_dir, "WRITE_SIZE") if write_dir else {}

    def calib(tab):
        copy = [v for (n, _), v in tab.items() if n == "k_copy"]
        return COPY_BYTES / (copy[0] * 1024.0) if copy and copy[0] > 0 else float("nan")

    fcal, wcal = calib(fetch), calib(write)
    lines = [f"# rocprofv3 kernel trace: {title}", "",
             "Commands (run from the repository root on one MI355X, ROCm 7.2, after "
             "`cd /tmp && export TMPDIR=/tmp`):", ""]
    lines += [f"    {c}" for c in commands]
    lines += ["", f"Kernel source sha256[:16]: `{src_hash or source_hash()}`.", "",
              "Durations from the kernel trace.  Back-to-back launches started less than "
              f"{B2B_GAP_NS / 1000:g} µs after the previous kernel on their queue ended (the "
              "iteration sequence of the timed steps); the others follow an idle gap (launches "
              "bracketed by timing events, bursts, plan creation).  HBM bytes per launch = "
              "counter (KiB x 1024) x calibration from the library's copy kernel moving 1 GiB "
              f"each way in the same command (FETCH_SIZE x{fcal:.3f}, WRITE_SIZE x{wcal:.3f}); "
              "nan where the counter run has no dispatch of that kernel.", "",
              "| kernel | threads | launches | avg µs | back-to-back launches | back-to-back avg µs "
              "| HBM read B/launch | HBM write B/launch |",
              "|---|---|---|---|---|---|---|---|"]
    for (name, threads), e in sorted(tt.items(), key=lambda kv: -kv[1]["ns"]):
        rd = fetch.get((name, threads))
        wr = write.get((name, threads))
        lines.append(
            f"| `{name}` | {threads} | {e['n']} | {e['ns'] / e['n'] / 1e3:.3f} | {e['nb']} | "
            + (f"{e['bns'] / e['nb'] / 1e3:.3f}" if e["nb"] else "nan") + " | "
            + (f"{rd * 1024 * fcal:.0f}" if rd is not None else "nan") + " | "
            + (f"{wr * 1024 * wcal:.0f}" if wr is not None else "nan") + " |")
    return "\n".join(lines) + "\n"


def read_summary(path: str):
    """Rows of a committed summary {(kernel, threads): dict}, or None if the file is
    absent or was taken on another kernel source."""
    if not os.path.exists(path):
        return None
    text = open(path).read()
    h = re.search(r"Kernel source sha256\[:16\]:\s*`([0-9a-f]{16})`", text)
    if not h or h.group(1) != source_hash():
        return None
    rows = {}
    for line in text.splitlines():
        m = _ROW.match(line.strip())
        if m:
            rows[(m["name"], int(m["threads"]))] = dict(
                n=int(m["n"]), avg_us=float(m["avg"]), nb=int(m["nb"]),
                b2b_us=float(m["bavg"]), read=float(m["rd"]), write=float(m["wr"]))
    return rows


def trace_figures(path: str, names, threads: int):
    """Launch-weighted back-to-back duration and HBM bytes of the named kernels (at
    `threads` threads per launch) from a committed summary; None when unavailable."""
    rows = read_summary(path)
    if not rows:
        return None
    sel = [rows[(n, threads)] for n in names if (n, threads) in rows]
    if not sel or sum(r["nb"] for r in sel) == 0:
        return None
    nb = sum(r["nb"] for r in sel)
    n = sum(r["n"] for r in sel)
    out = {"b2b_us": sum(r["b2b_us"] * r["nb"] for r in sel if r["nb"]) / nb,
           "avg_us": sum(r["avg_us"] * r["n"] for r in sel) / n, "launches": n,
           "b2b_launches": nb}
    if all(np.isfinite(r["read"]) and np.isfinite(r["write"]) for r in sel):
        out["traffic"] = sum((r["read"] + r["write"]) * r["n"] for r in sel) / n
    return out


def summary_path(workload: str) -> str:
    return os.path.join(PROFILES, f"kernel_trace_{workload}.md")


def run_workload(torch, rl, synth, cfg: int, steps: int, warmup: int, workload: str):
    c = synth.make_config(cfg)
    shape, n_iter = c["shape"], c["n_iter"]
    dev = torch.device("cuda:0")
    psf = torch.from_numpy(c["psf"]).to(dev)
    d = torch.from_numpy(c["d"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    u = u0.clone()
    plan = rl.Plan(psf, autotune=True)  # tuned at creation, outside the timed region
    launch_cfg = plan.launch()
    nvox = int(np.prod(shape))

    def step():
        u.copy_(u0)
        plan.iterate(d, u, n_iter)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)

    def timed(events: bool):
        plan.set_timing(events)
        start.record()
        for _ in range(steps):
            step()
        stop.record()
        torch.cuda.synchronize()
        live = plan.timing() if events else None
        plan.set_timing(False)
        return start.elapsed_time(stop) / steps, live

    # The timed region gives the throughput.  The same steps are then repeated with
    # every launch of the plan bracketed by a pair of HIP events on the plan's
    # stream, stamped by the launch itself: each pass's duration comes from the
    # real iteration sequence.  The events leave idle gaps between launches (not
    # inside them), so the throughput is taken without them.
    ms, _ = timed(False)
    u_final = u.clone()  # the estimate after n_iter iterations (last timed step)
    ms_events, live = timed(True)
    value = nvox * n_iter / (ms * 1e-3) / 1e9

    flux = plan.flux()
    total = float(c["d"].sum(dtype=np.float64))
    drift = float(np.max(np.abs(flux - total)) / total)

    kb = kernel_bytes(shape)
    # per-pass durations from the timed region; beside them, a burst of 20
    # back-to-back launches of the same pass (each launch follows one of its own
    # kind, not the pass before it in the iteration)
    scratch = u0.clone()
    per_kind = {}
    for kind in ("x_ratio", "x_update", "y", "z_otf"):
        cnt, kms = live[kind]
        avg_us = kms / cnt * 1e3
        byts = kb[kind]
        burst_us = plan.time_pass(kind, d, scratch, reps=20) * 1e3
        names, threads = plan.pass_kernel(kind)
        per_kind[kind] = dict(launches_per_step=cnt / steps, avg_us=round(avg_us, 3),
                              total_ms=round(kms / steps, 4), bytes_per_launch=byts,
                              gbs=round(byts / (avg_us * 1e-6) / 1e9, 1),
                              burst_us=round(burst_us, 3), kernels=names, threads=threads)
    dom = max(per_kind, key=lambda k: per_kind[k]["total_ms"])
    dk = per_kind[dom]
    events_gbs = dk["bytes_per_launch"] / (dk["avg_us"] * 1e-6) / 1e9
    tr = trace_figures(summary_path(workload), dk["kernels"], dk["threads"])
    if tr is not None:
        dur_us = tr["b2b_us"]
        source = (f"rocprofv3 kernel trace of this benchmark ({os.path.basename(summary_path(workload))}): "
                  f"average of the kernel's {tr['b2b_launches']} back-to-back launches")
    else:
        dur_us = dk["avg_us"]
        source = "HIP events around every launch over a repeat of the timed steps (no current trace)"
    achieved = dk["bytes_per_launch"] / (dur_us * 1e-6) / 1e9
    roof = {"bound": "hbm", "kernel": dom, "kernels": dk["kernels"], "threads": dk["threads"],
            "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
            "frac": round(achieved / PEAK_HBM_GBS, 4),
            "traffic": round(tr["traffic"]) if tr and "traffic" in tr else None,
            "bytes_per_launch": dk["bytes_per_launch"], "avg_launch_us": round(dur_us, 3),
            "duration_source": source,
            "events_avg_launch_us": dk["avg_us"], "events_achieved": round(events_gbs, 1),
            "events_frac": round(events_gbs / PEAK_HBM_GBS, 4)}
    # whole-iteration effective bandwidth over all passes (the prologue's X r2c, and
    # the last update, which skips the forward transform, included); kernel time is
    # every timed launch of the plan, flux reductions included
    model_bytes = (sum(v["bytes_per_launch"] * v["launches_per_step"] for v in per_kind.values())
                   + kb["x_r2c"] * live["x_r2c"][0] / steps
                   - (kb["x_update"] - kb["x_update_last"]))
    kernel_ms = sum(kms for _, kms in live.values()) / steps
    plan.close()
    return dict(shape=shape, n_iter=n_iter, nvox=nvox, ms=ms, value=value, roofline=roof,
                ms_events=ms_events, per_kind=per_kind, flux_drift=drift,
                launch=launch_cfg, u=u_final,
                launches_per_step={k: cnt / steps for k, (cnt, _) in live.items() if cnt},
                all_kernels_gbs=round(model_bytes / (kernel_ms * 1e-3) / 1e9, 1),
                bytes_per_vi=round(model_bytes / (nvox * n_iter), 2),
                model_effective_gbs=round(model_bytes / (nvox * n_iter) * value, 1))


def run_batched(torch, rl, synth, steps: int, warmup: int, count: int = 96, n_iter: int = 50,
                autotune: bool = True):
    """Batched form: `count` uneven volumes with their own PSFs, one graph launch per
    shape class and iteration (the class's per-pass kernels), against the same volumes
    run one plain plan at a time.  With
    `autotune`, the batch plan tunes each shape class once and the plain plans reuse
    those choices through a temporary tuning cache (both sides tuned alike; plan
    creation is outside the timed region)."""
    import tempfile
    vols = synth.make_batch(count)
    dev = torch.device("cuda:0")
    psfs = [torch.from_numpy(v["psf"]).to(dev) for v in vols]
    d = [torch.from_numpy(v["d"]).to(dev) for v in vols]
    u0 = [torch.from_numpy(v["u0"]).to(dev) for v in vols]
    u = [t.clone() for t in u0]
    nvox = sum(int(np.prod(v["shape"])) for v in vols)
    # a caller's tuning cache (RLMI_TUNE_CACHE) serves both sides; else a temporary one
    saved = os.environ.get("RLMI_TUNE_CACHE")
    cache = tempfile.mkdtemp() if saved is None else None
    if autotune and cache is not None:
        os.environ["RLMI_TUNE_CACHE"] = os.path.join(cache, "tune.txt")
    try:
        bp = rl.BatchPlan(psfs, autotune=autotune)
        plans = [rl.Plan(h, autotune=autotune) for h in psfs]
    finally:
        if cache is not None:
            os.environ.pop("RLMI_TUNE_CACHE", None)
            if os.path.exists(os.path.join(cache, "tune.txt")):
                os.remove(os.path.join(cache, "tune.txt"))
            os.rmdir(cache)
    launch = bp.launch()
    mode = bp.mode()

    def step_batched():
        for a, b in zip(u, u0):
            a.copy_(b)
        bp.iterate(d, u, n_iter)

    def step_plain():
        for a, b in zip(u, u0):
            a.copy_(b)
        for p, dd, uu in zip(plans, d, u):
            p.iterate(dd, uu, n_iter)

    out = {}
    for name, fn in (("batched", step_batched), ("plain", step_plain)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            fn()
        b.record()
        torch.cuda.synchronize()
        out[name] = a.elapsed_time(b) / steps
    flux = bp.flux()
    totals = np.array([float(v["d"].sum(dtype=np.float64)) for v in vols])
    drift = float(np.max(np.abs(flux - totals[:, None]) / totals[:, None]))
    for p in plans:
        p.close()
    bp.close()
    classes = {}
    for v in vols:
        classes[str(v["shape"])] = classes.get(str(v["shape"]), 0) + 1
    # algorithmic bytes of one iteration of every volume (the pass model of the
    # single-volume plans), over the whole step
    it_bytes = 0
    for v in vols:
        kb = kernel_bytes(v["shape"])
        it_bytes += kb["x_ratio"] + kb["x_update"] + 4 * kb["y"] + 2 * kb["z_otf"]
    value = nvox * n_iter / (out["batched"] * 1e-3) / 1e9
    bpvi = it_bytes / nvox
    return {"workload": f"rl_fp32_batch{count}_uneven_{n_iter}it", "volumes": count,
            "voxels": nvox, "shape_classes": classes,
            "value": round(value, 3),
            "bytes_per_vi": round(bpvi, 2),
            "model_effective_gbs": round(bpvi * value, 1),
            "model_frac": round(bpvi * value / PEAK_HBM_GBS, 4),
            "unit": "Gvoxel-iter/s", "ms_per_step": round(out["batched"], 3), "mode": mode,
            "plain_one_plan_per_volume_ms": round(out["plain"], 3),
            "speedup_vs_plain": round(out["plain"] / out["batched"], 3), "flux_drift": drift,
            "autotuned": autotune, "launch": launch}


GOLDEN_512 = os.path.join(ROOT, "tests", "golden", "rl_512x512x256_samples.txt")


def oracle_samples():
    """The FP64 oracle's estimate of the 512x512x256 workload after 10 and 50
    iterations at stored sample voxels (written once by the script beside the
    file, which calls only the oracle); None if the file is absent."""
    if not os.path.exists(GOLDEN_512):
        return None
    a = np.loadtxt(GOLDEN_512, comments="#")
    return a[:, :3].astype(np.int64), {10: a[:, 3], 50: a[:, 4]}


def run_split(torch, rl, synth, steps: int, cfg: int = 2):
    """Split-precision forms on the organoid-scale volume: time per step against the
    plain FP32 form, relative L2 to the FP32 result after 10 and 50 iterations, and
    relative L2 to the FP64 oracle over its stored sample voxels."""
    c = synth.make_config(cfg)
    n_iter = c["n_iter"]
    dev = torch.device("cuda:0")
    psf = torch.from_numpy(c["psf"]).to(dev)
    d = torch.from_numpy(c["d"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    nvox = int(np.prod(c["shape"]))
    res, ref = {}, {}
    samples = oracle_samples()
    for prec in ("fp32", "split_bf16", "split_fp16"):
        plan = rl.Plan(psf, precision=prec, autotune=True)  # each form tuned alike
        u = u0.clone()
        plan.iterate(d, u, 10)
        u10 = u.clone()
        plan.iterate(d, u, n_iter - 10)
        u50 = u.clone()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            u.copy_(u0)
            plan.iterate(d, u, n_iter)
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        plan.close()
        if prec == "fp32":
            ref = {10: u10.double(), 50: u50.double()}
        value = nvox * n_iter / (ms * 1e-3) / 1e9
        kb = kernel_bytes(c["shape"])
        bpvi = (kb["x_ratio"] + kb["x_update"] + 4 * kb["y"] + 2 * kb["z_otf"]) / nvox
        # the split forms keep every array in FP32 in HBM: the same bytes per iteration
        entry = {"ms_per_step": round(ms, 3), "value": round(value, 3),
                 "model_effective_gbs": round(bpvi * value, 1),
                 "model_frac": round(bpvi * value / PEAK_HBM_GBS, 4)}
        if prec != "fp32":
            for k, uu in ((10, u10), (50, u50)):
                entry[f"rel_l2_vs_fp32_at_{k}"] = float(
                    (torch.linalg.vector_norm(uu.double() - ref[k]) /
                     torch.linalg.vector_norm(ref[k])).item())
        if samples is not None:
            pts, vals = samples
            idx = torch.from_numpy(pts).to(dev)
            for k, uu in ((10, u10), (50, u50)):
                g = uu[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
                entry[f"rel_l2_vs_oracle_at_{k}"] = float(
                    np.linalg.norm(g - vals[k]) / np.linalg.norm(vals[k]))
            entry["oracle_samples"] = int(len(pts))
        res[prec] = entry
    for prec in ("split_bf16", "split_fp16"):
        res[prec]["speedup_vs_fp32"] = round(res["fp32"]["ms_per_step"] /
                                             res[prec]["ms_per_step"], 3)
    return {"workload": "rl_split_256x512x512_50it", "unit": "Gvoxel-iter/s", **res}


def run_accel(torch, rl, synth, steps: int, cfg: int = 1):
    """Biggs-Andrews extrapolated form on the 128x256x256 volume: throughput per
    iteration at the plain form's iteration count, and the time to reach the
    Poisson log-likelihood that the plain form reaches after that many iterations.
    The likelihood sum(d log Hu - Hu) is evaluated with the plan's own convolution
    and a float64 reduction (evaluation only)."""
    c = synth.make_config(cfg)
    n_plain = c["n_iter"]
    dev = torch.device("cuda:0")
    psf = torch.from_numpy(c["psf"]).to(dev)
    d = torch.from_numpy(c["d"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    nvox = int(np.prod(c["shape"]))
    d64 = d.double()

    def loglik(plan, u):
        q = plan.conv(u).double()
        ok = q > 1e-12
        return float(torch.where(ok, d64 * torch.log(torch.where(ok, q, 1.0)) - q, 0.0).sum())

    def timed(plan, n):
        u = u0.clone()
        plan.iterate(d, u, n)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            u.copy_(u0)
            plan.iterate(d, u, n)
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    plain = rl.Plan(psf, autotune=True)
    acc = rl.Plan(psf, autotune=True, accel="biggs_andrews")
    u = u0.clone()
    plain.iterate(d, u, n_plain)
    target = loglik(plain, u)
    n_equiv = None
    for n in list(range(5, n_plain, 5)) + [n_plain]:
        u = u0.clone()
        acc.iterate(d, u, n)
        if loglik(acc, u) >= target:
            n_equiv = n
            break
    ms_plain = timed(plain, n_plain)
    ms_acc = timed(acc, n_plain)
    ms_equiv = timed(acc, n_equiv) if n_equiv else None
    alpha = acc.alpha()
    plain.close()
    acc.close()
    return {"workload": "rl_biggs_andrews_128x256x256", "unit": "Gvoxel-iter/s",
            "plain_iterations": n_plain, "plain_ms": round(ms_plain, 3),
            "accel_ms_at_plain_iterations": round(ms_acc, 3),
            "accel_value": round(nvox * n_plain / (ms_acc * 1e-3) / 1e9, 3),
            "accel_iterations_to_plain_loglik": n_equiv,
            "accel_ms_to_plain_loglik": round(ms_equiv, 3) if ms_equiv else None,
            "time_to_quality_speedup": round(ms_plain / ms_equiv, 3) if ms_equiv else None,
            "plain_loglik": target, "mean_alpha": round(float(np.mean(alpha[2:])), 4)}


def run_zero_boundary(torch, rl, synth, steps: int, cfg: int = 1):
    """Zero (linear) boundary on the 128x256x256 volume with its Gaussian PSF cut
    to a +-4 sigma box (entries outside it are exactly zero): throughput over the
    caller's voxels, the padded transform grid, and the periodic form beside it."""
    c = synth.make_config(cfg)
    n_iter = c["n_iter"]
    shape = c["shape"]
    sx, sy, sz = c["sigma"]
    pshape = tuple(2 * int(np.ceil(4 * s)) + 1 for s in (sz, sy, sx))
    dev = torch.device("cuda:0")
    psf = torch.from_numpy(synth.gaussian_psf(pshape, (sx, sy, sz))).to(dev)
    d = torch.from_numpy(c["d"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    nvox = int(np.prod(shape))
    plan = rl.Plan(psf, shape=shape, boundary="zero", autotune=True)
    u = u0.clone()
    plan.iterate(d, u, n_iter)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        u.copy_(u0)
        plan.iterate(d, u, n_iter)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    flux = plan.flux()
    total = float(c["d"].sum(dtype=np.float64))
    grid = plan.grid()
    plan.close()
    return {"workload": "rl_zero_boundary_128x256x256_100it", "unit": "Gvoxel-iter/s",
            "psf_shape_zyx": list(pshape), "grid_zyx": list(grid),
            "grid_voxels_per_voxel": round(float(np.prod(grid)) / nvox, 3),
            "ms_per_step": round(ms, 3), "value": round(nvox * n_iter / (ms * 1e-3) / 1e9, 3),
            "flux_drift": float(np.max(np.abs(flux - total)) / total)}


def run_paper_shape(torch, rl, synth, steps: int, n_iter: int = 20):
    """The paper's own stack shape, 30x2160x2560 (periodic, PSF of the volume's
    shape): throughput of n_iter iterations per step (the paper states no iteration
    count) and the plan's launch configuration."""
    c = synth.make_paper_shape()
    dev = torch.device("cuda:0")
    psf = torch.from_numpy(c["psf"]).to(dev)
    d = torch.from_numpy(c["d"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    nvox = int(np.prod(c["shape"]))
    plan = rl.Plan(psf, autotune=True)
    u = u0.clone()
    plan.iterate(d, u, n_iter)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(steps):
        u.copy_(u0)
        plan.iterate(d, u, n_iter)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / steps
    flux = plan.flux()
    total = float(c["d"].sum(dtype=np.float64))
    launch = plan.launch()
    # per-pass durations: one more step with every launch bracketed by events
    plan.set_timing(True)
    u.copy_(u0)
    plan.iterate(d, u, n_iter)
    torch.cuda.synchronize()
    live = plan.timing()
    plan.set_timing(False)
    kb = kernel_bytes(c["shape"])
    per_kind = {}
    for kind in ("x_ratio", "x_update", "y", "z_otf"):
        cnt, kms = live[kind]
        avg_us = kms / cnt * 1e3
        per_kind[kind] = dict(launches_per_step=cnt, avg_us=round(avg_us, 3),
                              bytes_per_launch=kb[kind],
                              gbs=round(kb[kind] / (avg_us * 1e-6) / 1e9, 1),
                              kernels=plan.pass_kernel(kind)[0])
    plan.close()
    return {"workload": f"rl_fp32_2560x2160x30_{n_iter}it", "shape_zyx": list(c["shape"]),
            "unit": "Gvoxel-iter/s", "ms_per_step": round(ms, 3),
            "value": round(nvox * n_iter / (ms * 1e-3) / 1e9, 3), "launch": launch,
            "per_kind": per_kind, "flux_drift": float(np.max(np.abs(flux - total)) / total)}


def run_stop(torch, rl, synth, steps: int, cfg: int = 1):
    """Metric-guided stopping on the 128x256x256 volume: iterations chosen by each
    rule (at most the configuration's 100) and the wall-clock time of the call,
    against 100 fixed iterations; the per-iteration cost of carrying the metric."""
    c = synth.make_config(cfg)
    n_max = c["n_iter"]
    dev = torch.device("cuda:0")
    psf = torch.from_numpy(c["psf"]).to(dev)
    d = torch.from_numpy(c["d"]).to(dev)
    u0 = torch.from_numpy(c["u0"]).to(dev)
    truth = torch.from_numpy(c["truth"]).to(dev)
    nvox = int(np.prod(c["shape"]))
    plan = rl.Plan(psf, autotune=True)
    u = u0.clone()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            u.copy_(u0)
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / steps

    out = {"workload": "rl_stop_128x256x256", "max_iter": n_max,
           "fixed_ms": round(timed(lambda: plan.iterate(d, u, n_max)), 3)}
    # the log-likelihood threshold lies between two consecutive relative improvements
    # of the FP64 oracle on this volume (1.50e-4 and 1.00e-4), clear of both
    # fsc: stop once the single-image FSC resolution no longer improves (threshold 0)
    rules = {"loglik": (1.2e-4, None), "change": (2e-3, None), "psnr": (0.01, truth),
             "ssim": (1e-3, truth), "fsc": (0.0, None)}
    for name, (tau, ref) in rules.items():
        ms = timed(lambda: plan.iterate_until(d, u, n_max, name, tau, reference=ref))
        n, hist = plan.stop()
        # per-iteration cost of the metric: the full 100 iterations with a rule that never fires
        ms_all = timed(lambda: plan.iterate_until(d, u, n_max, name, -1e300, reference=ref))
        out[name] = {"threshold": tau, "iterations": n, "ms": round(ms, 3),
                     "last_metric": float(hist[-1]) if len(hist) else None,
                     "metric_overhead_per_iter_pct": round(100 * (ms_all / out["fixed_ms"] - 1), 2),
                     "value": round(nvox * n / (ms * 1e-3) / 1e9, 3) if n else None}
    # single-image FSC of the 100-iteration estimate: split + two transforms + shell
    # sums on the device, against numpy's FFT on the host (context)
    u.copy_(u0)
    plan.iterate(d, u, n_max)
    half = tuple(n // 2 for n in c["shape"])
    delta = torch.zeros(half, dtype=torch.float32, device=dev)
    delta[tuple(n // 2 for n in half)] = 1.0
    with rl.Plan(delta) as q:
        a, b = rl.split_diagonal(u)
        q.fsc(a, b, 64)
        torch.cuda.synchronize()
        t = time.perf_counter()
        reps = 10
        for _ in range(reps):
            a, b = rl.split_diagonal(u)
            _, res = q.fsc(a, b, 64)
        fsc_ms = (time.perf_counter() - t) * 1e3 / reps
    un = u.cpu().numpy().astype(np.float64)
    t = time.perf_counter()
    fa = np.fft.rfftn(un[0::2, 0::2, 0::2])
    fb = np.fft.rfftn(un[1::2, 1::2, 1::2])
    _ = np.real(fa * np.conj(fb)).sum(), (np.abs(fa) ** 2).sum(), (np.abs(fb) ** 2).sum()
    host_ms = (time.perf_counter() - t) * 1e3
    out["fsc"].update({"single_image_fsc_ms": round(fsc_ms, 3),
                       "resolution_cycles_per_voxel": res,
                       "numpy_fft_only_ms_context": round(host_ms, 1)})
    plan.close()
    return out


def copy_probe(torch, rl, nbytes: int = 1 << 30, reps: int = 20) -> float:
    """Plain streaming copy kernel of the library: read + write bytes per second (GB/s)."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    stream = int(torch.cuda.current_stream().cuda_stream)
    for _ in range(5):
        rl.rl_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        rl.rl_probe_copy(src.data_ptr(), dst.data_ptr(), nbytes, stream)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_baseline(c: dict, n_iter_sample: int = 2):
    """The FP64 oracle on the host cores, on a bounded sample of the headline
    workload (its first iteration(s)).  Returns the record and the oracle's estimate
    after the sample's iterations."""
    import oracle
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()
                       if i.get("internal_api") in ("openblas", "mkl", "blis")] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    nvox = int(np.prod(c["shape"]))
    t = time.perf_counter()
    u, _, _ = oracle.rl(c["d"], c["psf"], c["u0"], n_iter_sample)
    dt = time.perf_counter() - t
    shp = "x".join(str(n) for n in reversed(c["shape"]))
    return ({"value": round(nvox * n_iter_sample / dt / 1e9, 6), "unit": "Gvoxel-iter/s",
             "cores": threads, "kind": "oracle",
             "sample": f"{n_iter_sample} FP64 RL iteration(s) of the {shp} volume, transfer "
                       f"function included (naive per-axis DFT by BLAS matrix products), "
                       f"{dt:.1f} s"}, u)


def cpu_fft_context(synth, n_iter: int = 4) -> dict:
    """Context only (not the oracle, not a baseline): a conventional host RL with
    scipy's multithreaded FFT in FP32 on the same 128x256x256 volume."""
    import scipy.fft as sfft
    c = synth.make_config(1)
    d, h = c["d"].astype(np.float32), c["psf"].astype(np.float64)
    k = np.roll(h / h.sum(), [-(n // 2) for n in h.shape], axis=(0, 1, 2)).astype(np.float32)
    workers = os.cpu_count() or 1
    K = sfft.rfftn(k, workers=workers)
    u = c["u0"].astype(np.float32).copy()
    t = time.perf_counter()
    for _ in range(n_iter):
        q = sfft.irfftn(K * sfft.rfftn(u, workers=workers), s=u.shape, workers=workers)
        r = np.where(q > 1e-12, d / np.where(q > 1e-12, q, 1), 0).astype(np.float32)
        cc = sfft.irfftn(np.conj(K) * sfft.rfftn(r, workers=workers), s=u.shape, workers=workers)
        u *= np.maximum(cc, 0)
    dt = time.perf_counter() - t
    nvox = int(np.prod(c["shape"]))
    return {"value": round(nvox * n_iter / dt / 1e9, 5), "unit": "Gvoxel-iter/s",
            "workers": workers, "kind": "scipy.fft FP32 RL (context)",
            "sample": f"{n_iter} iterations of the 128x256x256 volume, {dt:.1f} s"}


def gpu_estimate_after(torch, rl, c: dict, n_iter: int) -> np.ndarray:
    with rl.Plan(torch.from_numpy(c["psf"]).to("cuda:0"), autotune=True) as p:
        u = torch.from_numpy(c["u0"]).to("cuda:0")
        p.iterate(torch.from_numpy(c["d"]).to("cuda:0"), u, n_iter)
        return u.cpu().numpy()


def sample_rel_l2(u, samples, n_iter: int):
    """Relative L2 distance of the estimate u (device tensor) to the oracle's stored
    values at its sample voxels after n_iter iterations; None if not stored."""
    if samples is None or n_iter not in samples[1]:
        return None
    pts, vals = samples
    g = u[tuple(pts.T)].double().cpu().numpy() if hasattr(u, "cpu") else u[tuple(pts.T)]
    return float(np.linalg.norm(g - vals[n_iter]) / np.linalg.norm(vals[n_iter]))


def summarize_main(argv):
    ap = argparse.ArgumentParser(prog="bench.py --rocprof-summary")
    ap.add_argument("--rocprof-summary", nargs="+", metavar="DIR", required=True,
                    help="kernel-trace directory, then optionally FETCH_SIZE and WRITE_SIZE "
                         "counter directories")
    ap.add_argument("--out", required=True)
    ap.add_argument("--title", default="")
    ap.add_argument("--cmd", action="append", default=[],
                    help="the profiled command(s), recorded in the summary")
    ap.add_argument("--bench-log", required=True,
                    help="stderr of the profiled benchmark run: the kernel source hash it "
                         "ran on is taken from there")
    a = ap.parse_args(argv)
    m = re.search(r"kernel source sha256\[:16\]: ([0-9a-f]{16})", open(a.bench_log).read())
    if not m:
        sys.exit(f"{a.bench_log}: no kernel source hash")
    dirs = a.rocprof_summary + [None] * (3 - len(a.rocprof_summary))
    text = rocprof_summary(dirs[0], dirs[1], dirs[2], a.title, a.cmd, src_hash=m.group(1))
    with open(a.out, "w") as f:
        f.write(text)
    print(f"wrote {a.out}")


class _CachedInputs:
    """The seeded generator with each configuration drawn once per process."""

    def __init__(self, synth):
        self._synth = synth
        self._cache = {}

    def make_config(self, cfg: int) -> dict:
        if cfg not in self._cache:
            self._cache[cfg] = self._synth.make_config(cfg)
        return self._cache[cfg]

    def __getattr__(self, name):
        return getattr(self._synth, name)


GOLDEN_256 = os.path.join(ROOT, "tests", "golden", "rl_256x256x128_samples.txt")


def oracle_samples_cfg1():
    """The FP64 oracle's estimate of the 256x256x128 workload after 50 and 100
    iterations at stored sample voxels (written by the script beside the file)."""
    if not os.path.exists(GOLDEN_256):
        return None
    a = np.loadtxt(GOLDEN_256, comments="#")
    return a[:, :3].astype(np.int64), {50: a[:, 3], 100: a[:, 4]}


def record(run: dict, workload: str, sigma) -> dict:
    return {"workload": workload, "shape_zyx": list(run["shape"]), "n_iter": run["n_iter"],
            "psf_sigma_xyz": list(sigma), "value": round(run["value"], 3),
            "unit": "Gvoxel-iter/s", "ms_per_step": round(run["ms"], 4),
            "ms_per_step_with_launch_events": round(run["ms_events"], 4),
            "roofline": run["roofline"], "all_kernels_gbs": run["all_kernels_gbs"],
            "bytes_per_vi": run["bytes_per_vi"], "model_effective_gbs": run["model_effective_gbs"],
            "per_kind": run["per_kind"], "launch": run["launch"], "flux_drift": run["flux_drift"]}


def main():
    if "--rocprof-summary" in sys.argv:
        return summarize_main(sys.argv[1:])
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mall", action="store_true",
                    help="skip the 256x256x128 (last-level-cache resident) workload")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 96-volume workload")
    ap.add_argument("--no-split", action="store_true", help="skip the split-precision forms")
    ap.add_argument("--no-accel", action="store_true", help="skip the extrapolated form")
    ap.add_argument("--no-zero", action="store_true", help="skip the zero-boundary form")
    ap.add_argument("--no-stop", action="store_true", help="skip metric-guided stopping")
    ap.add_argument("--no-paper", action="store_true",
                    help="skip the paper's 30x2160x2560 stack shape")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only (the batched and single-volume paths "
              "are single-GPU); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    rank = int(os.environ.get("RANK", "0"))

    import torch
    from paper_2510_14143_amd import rl, synth as synth_mod
    synth = _CachedInputs(synth_mod)

    log(f"kernel source sha256[:16]: {source_hash()}")
    copy_gbs = copy_probe(torch, rl)
    log(f"copy probe: {copy_gbs:.1f} GB/s (read + write)")
    log("workload: 256x512x512 volume, 50 iterations (headline)")
    head_w = "rl_fp32_256x512x512_50it"
    main_run = run_workload(torch, rl, synth, 2, args.steps, args.warmup, head_w)
    head_rel50 = sample_rel_l2(main_run.pop("u"), oracle_samples(), 50)
    log(json.dumps({"headline_per_kind": main_run["per_kind"]}))
    mall = None
    if not args.no_mall:
        log("workload: 128x256x256 volume, 100 iterations (fits the last-level cache)")
        w1 = "rl_fp32_128x256x256_100it"
        r1 = run_workload(torch, rl, synth, 1, args.steps, args.warmup, w1)
        mall = record(r1, w1, synth.CONFIGS[1]["sigma"])
        mall["note"] = ("working set about 135 MB, inside the 256 MB last-level cache: its "
                        "bandwidth figures include cache hits and are not HBM figures")
        mall["rel_l2_vs_oracle_samples_at_100"] = sample_rel_l2(r1["u"], oracle_samples_cfg1(), 100)
        log(json.dumps({"mall_resident": mall}))
    batched = None
    if not args.no_batch:
        log("workload: batched, 96 uneven volumes, 50 it")
        batched = optional_leg("batched",
                               lambda: run_batched(torch, rl, synth, max(1, args.steps // 5), 1))
        log(json.dumps({"batched": batched}))
    accel = None
    if not args.no_accel:
        log("workload: Biggs-Andrews extrapolation (128x256x256)")
        accel = optional_leg("accel", lambda: run_accel(torch, rl, synth, max(1, args.steps // 2)))
        log(json.dumps({"accel": accel}))
    zero = None
    if not args.no_zero:
        log("workload: zero boundary (128x256x256, truncated PSF)")
        zero = optional_leg("zero_boundary",
                            lambda: run_zero_boundary(torch, rl, synth, max(1, args.steps // 2)))
        log(json.dumps({"zero_boundary": zero}))
    stop = None
    if not args.no_stop:
        log("workload: metric-guided stopping (128x256x256)")
        stop = optional_leg("stop", lambda: run_stop(torch, rl, synth, max(1, args.steps // 2)))
        log(json.dumps({"stop": stop}))
    split = None
    if not args.no_split:
        log("workload: split-precision forms, 256x512x512, 50 it")
        split = optional_leg("split", lambda: run_split(torch, rl, synth, max(1, args.steps // 5)))
        log(json.dumps({"split": split}))
    paper = None
    if not args.no_paper:
        log("workload: the paper's stack shape 30x2160x2560, 20 it")
        paper = optional_leg("paper_shape",
                             lambda: run_paper_shape(torch, rl, synth, max(1, args.steps // 5)))
        log(json.dumps({"paper_shape": paper}))
    cpu = cpu_ctx = None
    if rank == 0 and not args.no_cpu:
        log("cpu baseline (oracle, first iterations of the headline volume)")
        c2 = synth.make_config(2)
        n_s = 2
        cpu, u_ref = cpu_baseline(c2, n_s)
        import oracle
        rel = optional_leg("gpu estimate beside the cpu baseline",
                           lambda: float(oracle.rel_l2(gpu_estimate_after(torch, rl, c2, n_s),
                                                       u_ref)))
        cpu["gpu_rel_l2_vs_oracle"] = rel if isinstance(rel, float) else None
        cpu["gpu_rel_l2_iterations"] = n_s
        del u_ref
        log("cpu FFT context (scipy)")
        cpu_ctx = cpu_fft_context(synth)

    out = {
        "metric": "RL Gvoxel-iter/s (plain FP32, one volume)",
        "value": round(main_run["value"], 3),
        "unit": "Gvoxel-iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_run["ms"], 4),
        "ms_per_step_with_launch_events": round(main_run["ms_events"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": head_w, "shape_zyx": list(main_run["shape"]),
                   "n_iter": main_run["n_iter"], "psf_sigma_xyz": list(synth.CONFIGS[2]["sigma"]),
                   "boundary": "periodic", "parallelism": "single_gpu",
                   "launch": main_run["launch"]},
        "roofline": main_run["roofline"],
        "cpu_baseline": cpu,
        "cpu_fft_context": cpu_ctx,
        "rel_l2_vs_oracle_samples_at_50": head_rel50,
        "all_kernels_gbs": main_run["all_kernels_gbs"],
        "bytes_per_vi": main_run["bytes_per_vi"],
        "model_effective_gbs": main_run["model_effective_gbs"],
        "flux_drift": main_run["flux_drift"],
        "per_kind": main_run["per_kind"],
        "mall_resident": mall,
        "batched": batched,
        "split": split,
        "accel": accel,
        "zero_boundary": zero,
        "stop": stop,
        "paper_shape": paper,
        "copy_probe_gbs": round(copy_gbs, 1),
    }
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
