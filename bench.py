#!/usr/bin/env python3
"""Benchmark of the control-scheduled gate kernels on one MI355X.

Workload (one step): the n=28 complex128 controlled-gate sweep.  A 4 GiB
state with i.i.d. N(0,1) real and imaginary parts, normalised (seed 1); one
Haar-random 2x2 unitary (seed 2); for every target t in {0, 13, 27} and every
control count c = 0..8 (random distinct control qubits, seed 3, value 1) the
gate is applied once with the scheduled kernels (27 launches per step).  The
same sweep with the masked baseline kernel (all 2^(n-1) pairs, control test
per pair) is timed separately for comparison.

Prints one JSON line: gate updates/s of the scheduled sweep, the roofline
of its dominant kernel (algorithmic bytes / HIP-event launch duration against
the 8 TB/s HBM peak), per-(t, c) rows, and the CPU oracle timed on a bounded
sample of the same sweep.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
N_QUBITS = 28
AMP_BYTES = 16


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha1()
    for f in ("gate_kernels.hip", "gate_math.hpp", "sv_internal.hpp", "tile.hpp"):
        with open(os.path.join(ROOT, "paper_2411_18354_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def load_traffic(kernel, src_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary, or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_k_pair_config1_n28.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = {k: v for k, v in re.findall(r"^- (\w+): (\S+)$", txt, flags=re.M)}
    if m.get("kernel_source_hash") != src_hash or m.get("kernel") is None:
        return None
    if m["kernel"].replace("_", " ") not in kernel.replace("_", " "):
        return None
    try:
        return float(m["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


COPY_KERNEL = "sv::k_copy"
COPY_BYTES = 1 << 30  # read and written per calibration launch


def _read_csv_rows(d, suffix):
    import csv
    import glob
    rows = []
    for f in glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True):
        with open(f) as fh:
            rows += list(csv.DictReader(fh))
    return rows


def _counter_per_kernel(d, counter):
    """{kernel name: [counter value per dispatch]} from counter_collection.csv."""
    out = {}
    for r in _read_csv_rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        out.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]))
    return out


def summarize_profile(trace_dir, fetch_dir, write_dir):
    """Write the kernel-trace summary and the HBM-traffic record of the
    dominant kernel under profiles/ from rocprofv3 CSV output."""
    import subprocess
    import workloads as W
    import paper_2411_18354_amd as sv
    n = N_QUBITS
    cases = W.config1_cases(n, seed=3)
    plan = {}
    for t, ctrls in cases:
        cm = sum(1 << q for q in ctrls)
        name, pairs = sv.sv_gate_plan(n, sv.SV_C128, t, cm, cm, "auto")
        plan.setdefault(name, []).append(2 * (1 << (n - 1 - len(ctrls))) * 2 * AMP_BYTES)
    stats = _read_csv_rows(trace_dir, "kernel_stats.csv")
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    dom = None
    for r in stats:
        for k in plan:
            if r["Name"].startswith("void " + k) or r["Name"].startswith(k):
                dom = (k, r)
                break
        if dom:
            break
    assert dom, "dominant kernel not found in the trace"
    kname, krow = dom
    alg = sum(plan[kname]) / len(plan[kname])
    src_hash = kernel_source_hash()
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    lines = ["# Kernel trace: controlled-gate sweep, n=28 complex128", "",
             "Command (from the repository root; rocprofv3 1.x, ROCm 7.2):", "",
             "    rocprofv3 --kernel-trace --stats -f csv -d <dir> -o bench -- "
             "python3 bench.py --steps 5 --warmup 1 --cpu-seconds 0 --no-masked --pmc-copy", "",
             "kernel_source_hash: %s" % src_hash, "",
             "| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in stats[:12]:
        nm = r["Name"].split("(")[0].replace("void ", "")
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.1f%% |" % (
            nm, r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3,
            float(r["Percentage"])))
    lines += ["", "Dominant scheduled kernel: `%s`, average %.2f us over %s launches; "
              "average algorithmic bytes per launch %.4g (read + write of every touched "
              "amplitude), i.e. %.1f GB/s." % (kname, float(krow["AverageNs"]) / 1e3, krow["Calls"], alg,
                                                alg / float(krow["AverageNs"]))]
    with open(os.path.join(ROOT, "profiles", "kernel_trace_config1_n28.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # traffic: FETCH_SIZE and WRITE_SIZE (KiB per dispatch), scaled by the copy kernel
    fetch = _counter_per_kernel(fetch_dir, "FETCH_SIZE")
    write = _counter_per_kernel(write_dir, "WRITE_SIZE")

    def pick(dct, key):
        for k, v in dct.items():
            if k.replace("void ", "").startswith(key):
                return v
        return None
    fk, wk = pick(fetch, kname), pick(write, kname)
    fc, wc = pick(fetch, COPY_KERNEL), pick(write, COPY_KERNEL)
    assert fk and wk and fc and wc, "counters missing for the kernel or the copy calibration"
    f_scale = COPY_BYTES / (sum(fc) / len(fc) * 1024.0)
    w_scale = COPY_BYTES / (sum(wc) / len(wc) * 1024.0)
    f_b = sum(fk) / len(fk) * 1024.0 * f_scale
    w_b = sum(wk) / len(wk) * 1024.0 * w_scale
    tl = ["# HBM traffic of the dominant kernel: controlled-gate sweep, n=28 complex128", "",
          "Commands (each its own run, from the repository root):", "",
          "    rocprofv3 --pmc FETCH_SIZE -f csv -d <fetch_dir> -o bench -- python3 bench.py --steps 2 "
          "--warmup 0 --cpu-seconds 0 --no-masked --pmc-copy",
          "    rocprofv3 --pmc WRITE_SIZE -f csv -d <write_dir> -o bench -- python3 bench.py --steps 2 "
          "--warmup 0 --cpu-seconds 0 --no-masked --pmc-copy", "",
          "Counters are KiB per dispatch.  Each is scaled by what it reads for the library's plain copy "
          "kernel `sv::k_copy` moving a known 1 GiB (read 1 GiB, write 1 GiB): FETCH scale %.4f, "
          "WRITE scale %.4f." % (f_scale, w_scale), "",
          "- kernel: %s" % kname.replace(" ", "_"),
          "- kernel_source_hash: %s" % src_hash,
          "- dispatches: %d" % len(fk),
          "- fetch_bytes_per_launch: %.6g" % f_b,
          "- write_bytes_per_launch: %.6g" % w_b,
          "- hbm_bytes_per_launch: %.6g" % (f_b + w_b),
          "- alg_bytes_per_launch: %.6g" % alg,
          "- traffic_over_alg: %.4f" % ((f_b + w_b) / alg), ""]
    with open(os.path.join(ROOT, "profiles", "traffic_k_pair_config1_n28.md"), "w") as fh:
        fh.write("\n".join(tl) + "\n")
    print("\n".join(lines + [""] + tl))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="time budget of the CPU-oracle baseline sample (0 disables it)")
    ap.add_argument("--no-masked", action="store_true", help="skip the masked-baseline sweep")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="first copy a 1 GiB state three times with the library's plain copy kernel "
                         "(calibration of the rocprofv3 byte counters)")
    ap.add_argument("--summarize-profile", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ summaries from rocprofv3 CSV output of this script and exit")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(*args.summarize_profile)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: this build has no multi-GPU path "
              "(the sharding design is described in DESIGN.md); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    import paper_2411_18354_amd as sv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    n = N_QUBITS
    log("generating n=%d input state" % n)
    psi_host = W.random_state(n, seed=1)
    U = np.asarray(W.config1_gate(seed=2), dtype=np.float64)
    cases = W.config1_cases(n, seed=3)
    # interleave targets and control counts so consecutive gates touch
    # unrelated amplitudes
    order = sorted(range(len(cases)), key=lambda i: (len(cases[i][1]), cases[i][0]))
    cases = [cases[i] for i in order]
    d = torch.from_numpy(psi_host).to(dev)
    stream = torch.cuda.Stream(device=dev)  # default priority
    if args.pmc_copy:
        a = torch.zeros(1 << 26, dtype=torch.complex128, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            sv.sv_copy_state(b, a, stream=stream)
        torch.cuda.synchronize()
        del a, b

    plans = {}
    for mode in ("auto", "masked"):
        for t, ctrls in cases:
            cm = sum(1 << q for q in ctrls)
            plans[(mode, t, ctrls)] = sv.sv_gate_plan(n, sv.SV_C128, t, cm, cm, mode)

    def sweep(mode, steps, warmup):
        per = {(t, ctrls): [] for t, ctrls in cases}
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                for t, ctrls in cases:
                    sv.sv_apply_gate(d, t, ctrls, None, U, mode=mode, stream=stream)
            torch.cuda.synchronize()
            evs = []
            t_start = torch.cuda.Event(enable_timing=True)
            t_end = torch.cuda.Event(enable_timing=True)
            t_start.record(stream)
            for _ in range(steps):
                for t, ctrls in cases:
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    sv.sv_apply_gate(d, t, ctrls, None, U, mode=mode, stream=stream)
                    e1.record(stream)
                    evs.append(((t, ctrls), e0, e1))
            t_end.record(stream)
        torch.cuda.synchronize()
        total_ms = t_start.elapsed_time(t_end)
        for key, e0, e1 in evs:
            per[key].append(e0.elapsed_time(e1))
        return total_ms, per

    torch.cuda.synchronize()
    log("scheduled sweep: %d warmup + %d timed steps of %d gates" % (args.warmup, args.steps, len(cases)))
    total_ms, per = sweep("auto", args.steps, args.warmup)
    masked_total, per_m = (None, None)
    if not args.no_masked:
        log("masked sweep")
        masked_total, per_m = sweep("masked", args.steps, args.warmup)

    ngates = args.steps * len(cases)
    value = ngates / (total_ms / 1e3)
    rows = []
    kstats = {}
    alg_total = 0.0
    for t, ctrls in cases:
        c = len(ctrls)
        pairs = 1 << (n - 1 - c)
        alg = 2 * pairs * 2 * AMP_BYTES  # read + write of both pair elements
        ts = per[(t, ctrls)]
        med = float(np.median(ts))
        kname = plans[("auto", t, ctrls)][0]
        ks = kstats.setdefault(kname, {"ms": 0.0, "bytes": 0.0, "launches": 0})
        ks["ms"] += float(np.sum(ts))
        ks["bytes"] += alg * len(ts)
        ks["launches"] += len(ts)
        alg_total += alg * len(ts)
        row = {"t": t, "c": c, "controls": list(ctrls), "sched_us": round(med * 1e3, 2),
               "sched_GBps": round(alg / med / 1e6, 1), "sched_frac": round(alg / med / 1e6 / HBM_PEAK_GBPS, 3),
               "pair_updates_per_s": pairs / (med / 1e3), "kernel": kname}
        if per_m is not None:
            mm = float(np.median(per_m[(t, ctrls)]))
            row["masked_us"] = round(mm * 1e3, 2)
            row["masked_over_sched"] = round(mm / med, 2)
        rows.append(row)

    dom = max(kstats, key=lambda k: kstats[k]["ms"])
    ks = kstats[dom]
    avg_ms = ks["ms"] / ks["launches"]
    avg_bytes = ks["bytes"] / ks["launches"]
    achieved = avg_bytes / avg_ms / 1e6
    src_hash = kernel_source_hash()
    traffic = load_traffic(dom, src_hash)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": traffic,
                "kernel": dom, "avg_launch_us": round(avg_ms * 1e3, 2),
                "alg_bytes_per_launch": avg_bytes, "launches": ks["launches"],
                "kernel_source_hash": src_hash}

    cpu = None
    if args.cpu_seconds > 0:
        import oracle
        log("CPU oracle baseline (budget %.0f s)" % args.cpu_seconds)
        Uc = oracle.gate_matrix("U", matrix=tuple(U))
        host = psi_host.copy()
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            t, ctrls = cases[done % len(cases)]
            oracle.apply_gate(host, n, t, ctrls, (), Uc)
            done += 1
        el = time.perf_counter() - t0
        cpu = {"value": round(done / el, 4), "unit": "gate updates/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": "%d gates (the %d-gate sweep in order, repeated) on the same n=28 complex128 state "
                         "(plain loop over all 2^28 indices per gate, OpenMP), %.1f s" % (done, len(cases), el)}
        del host

    out = {
        "metric": "gate updates/s (n=28 complex128 controlled-gate sweep, c=0..8)",
        "value": round(value, 2),
        "unit": "gate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "controlled-gate sweep: n=28 complex128 state (4 GiB), Haar 2x2, "
                               "t in {0,13,27} x c=0..8 random controls, scheduled kernels",
                   "n": n, "gates_per_step": len(cases), "seeds": {"state": 1, "gate": 2, "controls": 3}},
        "hbm_GBps_alg": round(alg_total / total_ms / 1e6, 1),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "masked_value": None if masked_total is None else round(ngates / (masked_total / 1e3), 2),
        "sweep": rows,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
