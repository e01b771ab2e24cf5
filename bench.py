#!/usr/bin/env python3
"""Benchmark of the control-scheduled gate kernels on one MI355X.

Workload (one step): the n=28 complex128 controlled-gate sweep.  A 4 GiB
state with i.i.d. N(0,1) real and imaginary parts, normalised (seed 1); one
Haar-random 2x2 unitary (seed 2); for every target t in {0, 13, 27} and every
control count c = 0..8 (random distinct control qubits, seed 3, value 1) the
gate is applied once with the scheduled kernels (27 launches per step).  The
same sweep with the masked baseline kernel (all 2^(n-1) pairs, control test
per pair) is timed separately for comparison.

The last stdout line is one short JSON object: gate updates/s of the
scheduled sweep, the roofline of its dominant kernel (algorithmic bytes /
HIP-event launch duration against the 8 TB/s HBM peak), the CPU oracle timed
on a bounded sample of the same sweep, and a per-control-count summary.  The
per-(t, c) rows and the extra measurements go to a JSON file (--detail-out)
and to stderr.
"""
import argparse
import gc
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
    for f in ("gate_kernels.hip", "gate_math.hpp", "sv_internal.hpp"):  # the sources of k_pair and k_wave
        with open(os.path.join(ROOT, "paper_2411_18354_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:12]


def load_traffic(kernel, src_hash):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary, or None when absent or taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_k_pair_gate_sweep_n28.md")
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


COPY_KERNEL = "sv::k_hbm_probe<double, 0>"  # counter calibration: in-place read-modify-write
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
    cases = W.gate_sweep_cases(n, seed=3)
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
             "python3 bench.py --steps 5 --warmup 1 --cpu-seconds 0 --no-masked --no-extras --pmc-copy", "",
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
    with open(os.path.join(ROOT, "profiles", "kernel_trace_gate_sweep_n28.md"), "w") as fh:
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
          "--warmup 0 --cpu-seconds 0 --no-masked --no-extras --pmc-copy",
          "    rocprofv3 --pmc WRITE_SIZE -f csv -d <write_dir> -o bench -- python3 bench.py --steps 2 "
          "--warmup 0 --cpu-seconds 0 --no-masked --no-extras --pmc-copy", "",
          "Counters are KiB per dispatch.  Each is scaled by what it reads for the library's HBM probe "
          "`sv::k_hbm_probe<double, 0>` streaming a known 1 GiB in place (read 1 GiB, write 1 GiB): FETCH scale %.4f, "
          "WRITE scale %.4f." % (f_scale, w_scale), "",
          "- kernel: %s" % kname.replace(" ", "_"),
          "- kernel_source_hash: %s" % src_hash,
          "- dispatches: %d" % len(fk),
          "- fetch_bytes_per_launch: %.6g" % f_b,
          "- write_bytes_per_launch: %.6g" % w_b,
          "- hbm_bytes_per_launch: %.6g" % (f_b + w_b),
          "- alg_bytes_per_launch: %.6g" % alg,
          "- traffic_over_alg: %.4f" % ((f_b + w_b) / alg), ""]
    with open(os.path.join(ROOT, "profiles", "traffic_k_pair_gate_sweep_n28.md"), "w") as fh:
        fh.write("\n".join(tl) + "\n")
    print("\n".join(lines + [""] + tl))


def _position_cases(n, t=13):
    """(placement, c, controls) of the control-position sweep, in launch order."""
    out = []
    for place in ("lowest", "highest"):
        free = [q for q in range(n) if q != t]
        if place == "highest":
            free = free[::-1]
        for c in range(1, 9):
            out.append((place, c, tuple(sorted(free[:c]))))
    return out


def _counter_by_dispatch(d, counter):
    """[(dispatch id, kernel name, value)] in dispatch order (values of one
    dispatch summed over the rows rocprofv3 writes for it)."""
    acc = {}
    for r in _read_csv_rows(d, "counter_collection.csv"):
        if r.get("Counter_Name") != counter:
            continue
        k = int(r["Dispatch_Id"])
        name, v = acc.get(k, (r["Kernel_Name"], 0.0))
        acc[k] = (name, v + float(r["Counter_Value"]))
    return [(k, acc[k][0], acc[k][1]) for k in sorted(acc)]


def summarize_positions(fetch_dir, write_dir):
    """HBM bytes of every control-position gate (bench.py --positions-only
    under rocprofv3 --pmc) against its algorithmic bytes: exposes the
    cache-line granularity of skipped pairs."""
    n, t = N_QUBITS, 13
    fetch = _counter_by_dispatch(fetch_dir, "FETCH_SIZE")
    write = _counter_by_dispatch(write_dir, "WRITE_SIZE")

    def copy_scale(rows):
        v = [x for _, nm, x in rows if COPY_KERNEL in nm]
        assert v, "copy calibration missing"
        return COPY_BYTES / (sum(v) / len(v) * 1024.0)

    def gates(rows):
        return [x for _, nm, x in rows if "sv::k_pair" in nm or "sv::k_wave" in nm]
    fs, ws = copy_scale(fetch), copy_scale(write)
    gf, gw = gates(fetch), gates(write)
    cases = _position_cases(n, t)
    want = len(cases) * 2 * 2  # two modes, warm-up + one timed launch each
    assert len(gf) == want and len(gw) == want, (len(gf), len(gw), want)
    lines = ["# HBM traffic against control position: n=28 complex128, target 13", "",
             "Commands (each its own run, from the repository root):", "",
             "    rocprofv3 --pmc FETCH_SIZE -f csv -d <fetch_dir> -o pos -- python3 bench.py --positions-only "
             "--pmc-copy",
             "    rocprofv3 --pmc WRITE_SIZE -f csv -d <write_dir> -o pos -- python3 bench.py --positions-only "
             "--pmc-copy", "",
             "Counters (KiB per dispatch) are scaled by what they read for the HBM probe streaming a "
             "known 1 GiB: FETCH scale %.4f, WRITE scale %.4f.  Algorithmic bytes are the read and write of "
             "every amplitude of a satisfying pair, 2 * 2^(n-c) * 16.  Controls placed on the lowest free "
             "qubits sit below the 128-byte granule (qubits 0-2 of a complex128 index) until c >= 4; "
             "there a scheduled skip saves no DRAM traffic." % (fs, ws), "",
             "| placement | c | controls | mode | alg GB | HBM GB | HBM / alg |", "|---|---|---|---|---|---|---|"]
    i = 0
    for place, c, ctrls in cases:
        for mode in ("scheduled", "masked"):
            f_b = gf[i + 1] * 1024.0 * fs  # the launch after the warm-up
            w_b = gw[i + 1] * 1024.0 * ws
            i += 2
            alg = 2 * (1 << (n - c)) * AMP_BYTES
            lines.append("| %s | %d | %s | %s | %.3f | %.3f | %.2f |" % (
                place, c, ",".join(map(str, ctrls)), mode, alg / 1e9, (f_b + w_b) / 1e9, (f_b + w_b) / alg))
    path = os.path.join(ROOT, "profiles", "traffic_control_positions_n28.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


EXTRAS_TRACE_CMD = ("rocprofv3 --kernel-trace --stats -f csv -d <dir> -o extras -- python3 bench.py --steps 1 "
                    "--warmup 0 --cpu-seconds 0 --no-masked --no-protocol")


def summarize_trace(trace_dir):
    """Every kernel of a full bench run (the sweep plus the extras: fused
    circuits, adjoint, batches, dense blocks, expectation values, qubit
    exchange, fixed-point states) from rocprofv3 --kernel-trace --stats."""
    stats = _read_csv_rows(trace_dir, "kernel_stats.csv")
    assert stats, "no kernel_stats.csv under %s" % trace_dir
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["# Kernel trace: bench.py with every extra measurement", "",
             "Command (from the repository root):", "", "    " + EXTRAS_TRACE_CMD, "",
             "One sweep step, the control-position sweep, then the extras in bench order: the adjoint, "
             "the batches, dense blocks, the paper's 29-qubit circuits (masked, scheduled, fused; energy "
             "runs included), the remapped low-control circuit, and the fixed-point sweeps and circuits.  "
             "Library kernels are in the `sv::` namespace.", "",
             "| kernel | calls | total ms | avg us | min us | max us | share |", "|---|---|---|---|---|---|---|"]
    for r in stats[:40]:
        nm = r["Name"].split("(")[0].replace("void ", "")
        if len(nm) > 110:
            nm = nm[:107] + "..."
        lines.append("| `%s` | %s | %.2f | %.2f | %.2f | %.2f | %.2f%% |" % (
            nm, r["Calls"], float(r["TotalDurationNs"]) / 1e6, float(r["AverageNs"]) / 1e3,
            float(r["MinNs"]) / 1e3, float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
    path = os.path.join(ROOT, "profiles", "kernel_trace_bench_extras.md")
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


FUSED_ONLY_CMD = "python3 bench.py --fused-only"


def run_fused_only(sv, W, torch, np, stream):
    """One run each of the fused workloads whose kernels the counter
    profiles cover: the layered circuit at n=28 (5 layers, complex128), QFT29
    fused (complex128), and the n=24 ansatz forward and adjoint backward."""
    dev = torch.device("cuda:0")
    c2 = W.layered_circuit_n32(n=28, layers=5)
    st = torch.empty(1 << 28, dtype=torch.complex128, device=dev)
    p = sv.Circuit(28, c2, flags=sv.SV_FUSE)
    sv.sv_init(st, 0, stream=stream)
    p.run(st, stream=stream)
    p.close()
    del st
    st = torch.empty(1 << 29, dtype=torch.complex128, device=dev)
    p = sv.Circuit(29, W.qft(29), flags=sv.SV_FUSE)
    sv.sv_init(st, 1, stream=stream)
    p.run(st, stream=stream)
    p.close()
    del st
    c3, H = W.hea_problem_n24()
    params = torch.from_numpy(c3.params).to(dev)
    psi = torch.empty(1 << c3.n, dtype=torch.complex128, device=dev)
    lam = torch.empty_like(psi)
    plan = sv.Circuit(c3.n, c3, nparams=c3.nparams, flags=sv.SV_FUSE)
    sv.sv_init(psi, 0, stream=stream)
    plan.run(psi, params, stream=stream)
    sv.sv_adjoint_grad(psi, lam, sv.circuit_gates(c3), params, sv.pauli_terms(H), stream=stream)
    plan.close()
    torch.cuda.synchronize()
    print(json.dumps({"fused_only": "done"}), flush=True)


def run_expect_only(sv, W, torch, np, stream):
    """One expectation call each on an n=24 complex128 and 16-bit fixed-point
    state (the 47-term chain ZZ + X Hamiltonian: 3 tile passes), for
    counters."""
    dev = torch.device("cuda:0")
    h_arr = sv.pauli_terms(W.zz_x_hamiltonian(24, 5))
    ps = torch.randn(1 << 24, dtype=torch.complex128, device=dev)
    ps /= torch.linalg.vector_norm(ps)
    q = sv.FixedState(24, sv.SV_CQ16)
    sv.sv_convert(q, ps)
    eo = torch.empty(1, dtype=torch.float64, device=dev)
    for st_ in (ps, q):
        sv.sv_expect_noalloc(st_, h_arr, eo, stream=stream)
    torch.cuda.synchronize()
    print(json.dumps({"expect_only": "done", "value": eo.item()}), flush=True)


def summarize_counters(name, cmd, dirs):
    """Per-kernel averages of rocprofv3 --pmc counters (one directory per
    pass) into profiles/counters_<name>.md."""
    table = {}
    for d in dirs:
        acc = {}
        for r in _read_csv_rows(d, "counter_collection.csv"):
            k = (r["Kernel_Name"].split("(")[0].replace("void ", ""), r["Counter_Name"])
            key = (k, int(r["Dispatch_Id"]))
            acc[key] = acc.get(key, 0.0) + float(r["Counter_Value"])
        for ((kern, ctr), _), v in acc.items():
            table.setdefault(kern, {}).setdefault(ctr, []).append(v)
    ctrs = sorted({c for k in table.values() for c in k})
    lines = ["# Counters: %s" % name, "", "Commands (one pass each, from the repository root):", ""]
    lines += ["    " + c for c in cmd]
    lines += ["", "Average per dispatch over the dispatches of each kernel (sums over the rows rocprofv3 writes "
              "for one dispatch).", "", "| kernel | dispatches | " + " | ".join(ctrs) + " |",
              "|---|---|" + "---|" * len(ctrs)]
    for kern in sorted(table, key=lambda k: -max(len(v) for v in table[k].values())):
        vals = table[kern]
        nd = max(len(v) for v in vals.values())
        nm = kern if len(kern) <= 90 else kern[:87] + "..."
        lines.append("| `%s` | %d | " % (nm, nd) + " | ".join(
            ("%.4g" % (sum(vals[c]) / len(vals[c]))) if c in vals else "-" for c in ctrs) + " |")
    path = os.path.join(ROOT, "profiles", "counters_%s.md" % name)
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _time_ms(torch, stream, fn, reps):
    """Median of reps HIP-event timings of fn() on stream (after one warmup)."""
    with torch.cuda.stream(stream):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            fn()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def control_position_sweep(sv, torch, np, d, U, stream, n, t=13, reps=5):
    """Target 13 with c = 1..8 controls placed on the lowest free qubits and
    on the highest ones: exposes the cache-line granularity of skipped pairs
    (controls below bit 3 of a complex128 index share 128-byte lines with
    updated pairs).  Median HIP-event time per gate, scheduled and masked."""
    out = []
    for place, c, ctrls in _position_cases(n, t):
        row = {"placement": place, "t": t, "c": c, "controls": list(ctrls)}
        alg = 2 * (1 << (n - c)) * AMP_BYTES
        for mode in ("auto", "masked"):
            ts = []
            with torch.cuda.stream(stream):
                sv.sv_apply_gate(d, t, ctrls, None, U, mode=mode, stream=stream)
                for _ in range(reps):
                    e0 = torch.cuda.Event(enable_timing=True)
                    e1 = torch.cuda.Event(enable_timing=True)
                    e0.record(stream)
                    sv.sv_apply_gate(d, t, ctrls, None, U, mode=mode, stream=stream)
                    e1.record(stream)
                    ts.append((e0, e1))
            torch.cuda.synchronize()
            med = float(np.median([a.elapsed_time(b) for a, b in ts]))
            key = "sched" if mode == "auto" else "masked"
            row[key + "_us"] = round(med * 1e3, 2)
            row[key + "_GBps"] = round(alg / med / 1e6, 1)
        row["masked_over_sched"] = round(row["masked_us"] / row["sched_us"], 2)
        out.append(row)
    return out


def _deposit(v, mask):
    """Spread the low bits of v over the set bits of mask, in ascending order."""
    out, b = 0, 0
    for q in range(64):
        if (mask >> q) & 1:
            if (v >> b) & 1:
                out |= 1 << q
            b += 1
    return out


MALL_ROTATE_BYTES = 512 << 20  # twice the 256 MB Infinity Cache


def graph_protocol(sv, torch, np, st, n, cases, U, stream, amp_bytes=AMP_BYTES, target_ms=50.0, trials=7,
                   modes=("auto", "masked", "probe")):
    """Per (target, controls) and kernel form: R back-to-back launches of the
    gate captured once as a HIP graph and replayed, median of `trials`
    replays after one warm-up, R chosen so that a replay lasts about
    target_ms.  Consecutive launches rotate over K distinct control-value
    combinations (K * touched bytes >= 512 MiB, at most 2^c), so each launch
    touches amplitudes disjoint from the previous K - 1 and the 256 MB
    Infinity Cache cannot serve them; the kernels do the same work for any
    control values (the values are only the fixed bits of the index
    expansion).  Both forms use the same launch machinery.  Mode "probe"
    streams the HBM probe over the same address set (the scheduled controls
    fixed, the rest of each cache line included) with the same rotation: the
    bandwidth that set can reach with no gate arithmetic."""
    rows = []
    for t, ctrls in cases:
        c = len(ctrls)
        cm = sum(1 << q for q in ctrls)
        touched = (1 << (n - c)) * amp_bytes
        K = min(1 << c, max(1, -(-MALL_ROTATE_BYTES // touched)))
        vals = [_deposit((1 << c) - 1 - r, cm) for r in range(K)]
        alg = 2 * touched
        row = {"t": t, "c": c, "K_vals": K}
        gb = sv.sv_tune_get("granule_bits_c128" if amp_bytes == 16 else "granule_bits_c64")
        pm = cm & ~((1 << gb) - 1)  # the controls the kernel schedules; lower ones are rewritten

        def launch(mode, r):
            if mode == "probe":
                sv.sv_hbm_probe(st, pm, vals[r] & pm, "rmw", stream=stream)
            else:
                sv.sv_apply_gate_masks(st, t, cm, vals[r], U, mode=mode, stream=stream)
        for mode in modes:
            with torch.cuda.stream(stream):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                launch(mode, 0)
                e0.record(stream)
                for r in range(K):
                    launch(mode, r)
                e1.record(stream)
            torch.cuda.synchronize()
            est = max(e0.elapsed_time(e1) / K, 1e-3)
            R = int(min(8192, max(K, np.ceil(target_ms / est))))
            R = -(-R // K) * K
            g = torch.cuda.CUDAGraph()
            with torch.cuda.graph(g, stream=stream):
                for r in range(R):
                    launch(mode, r % K)
            ts = []
            with torch.cuda.stream(stream):
                g.replay()
                torch.cuda.synchronize()
                for _ in range(trials):
                    a = torch.cuda.Event(enable_timing=True)
                    b = torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    g.replay()
                    b.record(stream)
                    torch.cuda.synchronize()
                    ts.append(a.elapsed_time(b) / R)
            del g
            med = float(np.median(ts))
            key = {"auto": "sched", "masked": "masked", "probe": "probe"}[mode]
            byts = 2 * (1 << (n - bin(pm).count("1"))) * amp_bytes if mode == "probe" else alg
            row[key + "_R"] = R
            row[key + "_us"] = round(med * 1e3, 2)
            row[key + "_GBps"] = round(byts / med / 1e6, 1)
            row[key + "_frac"] = round(byts / med / 1e6 / HBM_PEAK_GBPS, 3)
        if "sched_us" in row and "masked_us" in row:
            row["masked_over_sched"] = round(row["masked_us"] / row["sched_us"], 2)
        if "sched_us" in row and "probe_us" in row:
            row["sched_over_probe"] = round(row["sched_us"] / row["probe_us"], 3)
        rows.append(row)
    return rows


def protocol_summary(rows):
    """Mean over targets, per control count, of the protocol rows."""
    by = {}
    for r in rows:
        by.setdefault(r["c"], []).append(r)
    out = {"c": sorted(by)}
    for k in ("sched_frac", "masked_frac", "masked_over_sched", "sched_us", "probe_frac", "sched_over_probe"):
        if all(k in r for r in rows):
            out[k] = [round(float(sum(r[k] for r in by[c]) / len(by[c])), 3) for c in out["c"]]
    return out


def hbm_ceiling(sv, torch, np, st, stream, reps=10, trials=5):
    """HBM probe over the whole state: in-place read-modify-write and
    read-only passes, reps back-to-back launches per HIP-event pair, median
    of trials (after one warm-up)."""
    nbytes = st.numel() * st.element_size()
    out = {}
    for op, mult in (("rmw", 2), ("read", 1)):
        ts = []
        with torch.cuda.stream(stream):
            sv.sv_hbm_probe(st, 0, 0, op, stream=stream)
            torch.cuda.synchronize()
            for _ in range(trials):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for _ in range(reps):
                    sv.sv_hbm_probe(st, 0, 0, op, stream=stream)
                b.record(stream)
                torch.cuda.synchronize()
                ts.append(a.elapsed_time(b) / reps)
        out[op + "_GBps"] = round(mult * nbytes / float(np.median(ts)) / 1e6, 1)
    return out


def protocol_n32(sv, W, torch, np, stream, U):
    """The controlled-gate sweep at the metric's n=32 end: a 64 GiB
    complex128 state of i.i.d. N(0,1) components (torch generator seed 11),
    targets {0, 16, 31}, c = 0..8 random controls (seed 3), scheduled and
    masked, timed by graph_protocol."""
    n = 32
    log("graph-launched sweep, n=32 complex128 (64 GiB)")
    cases = W.gate_sweep_cases(n, seed=3, targets=(0, 16, 31))
    st = torch.empty(1 << n, dtype=torch.complex128, device="cuda:0")
    gen = torch.Generator(device="cuda:0")
    gen.manual_seed(11)
    st.view(torch.float64).normal_(generator=gen)
    rows = graph_protocol(sv, torch, np, st, n, cases, U, stream)
    del st
    torch.cuda.empty_cache()
    return rows


RATED_POWER_W = 1400.0  # MI355X total board power


def _energy_reader():
    """The board energy counter of the (single) GPU through amdsmi, as
    (joules, counter timestamp in seconds), or None where it cannot be read."""
    try:
        import amdsmi
        amdsmi.amdsmi_init()
        h = amdsmi.amdsmi_get_processor_handles()[0]

        def read():
            e = amdsmi.amdsmi_get_energy_count(h)
            joules = float(e["energy_accumulator"]) * float(e["counter_resolution"]) * 1e-6  # uJ -> J
            return joules, float(e["timestamp"]) * 1e-9
        read()
        return read
    except Exception:
        return None


def _energy_per_run(torch, stream, fn, read, min_s=1.0):
    """Joules per call of fn and the board's average watts, over at least
    min_s seconds of back-to-back calls.  The counter advances in steps, so
    the power is taken between its own timestamps and multiplied by the
    measured time per call."""
    with torch.cuda.stream(stream):
        fn()
        torch.cuda.synchronize()
        (e0, s0), t0, reps = read(), time.perf_counter(), 0
        while True:
            fn()
            reps += 1
            torch.cuda.synchronize()
            if time.perf_counter() - t0 >= min_s:
                break
        (e1, s1), t1 = read(), time.perf_counter()
    if s1 <= s0:
        return None, None
    watts = (e1 - e0) / (s1 - s0)
    return watts * (t1 - t0) / reps, watts


def _case_sweep(sv, torch, np, st, cases, U, stream, mode, reps=3):
    """Median HIP-event time (ms) of every (target, controls) gate of the sweep
    on state st, and the total time of reps back-to-back passes."""
    with torch.cuda.stream(stream):
        for t, ctrls in cases:
            sv.sv_apply_gate(st, t, ctrls, None, U, mode=mode, stream=stream)
        torch.cuda.synchronize()
        evs = []
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(stream)
        for _ in range(reps):
            for t, ctrls in cases:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                sv.sv_apply_gate(st, t, ctrls, None, U, mode=mode, stream=stream)
                e1.record(stream)
                evs.append(((t, ctrls), e0, e1))
        b.record(stream)
    torch.cuda.synchronize()
    per = {}
    for key, e0, e1 in evs:
        per.setdefault(key, []).append(e0.elapsed_time(e1))
    return a.elapsed_time(b), {k: float(np.median(v)) for k, v in per.items()}


def measure_fixed_point(sv, W, torch, np, stream, psi_host, cases, U, energy):
    """Block-scaled fixed-point states, 16-bit codes (4 bytes per amplitude)
    and 32-bit codes (8), beside complex64 (8) on the same controlled-gate
    sweep, the paper's 29-qubit circuits in fixed point, and the QFT's error
    against its closed form."""
    dev = torch.device("cuda:0")
    n = 28
    out = {}
    src = torch.from_numpy(psi_host).to(dev)
    q = sv.FixedState(n, sv.SV_CQ16)
    sv.sv_convert(q, src, stream=stream)
    q32 = sv.FixedState(n, sv.SV_CQ32)
    sv.sv_convert(q32, src, stream=stream)
    c64 = torch.empty(1 << n, dtype=torch.complex64, device=dev)
    sv.sv_convert(c64, src, stream=stream)
    torch.cuda.synchronize()
    del src
    torch.cuda.empty_cache()
    log("fixed-point sweeps n=28 (16-bit scheduled and masked, 32-bit) and complex64 sweep")
    tq, pq = _case_sweep(sv, torch, np, q, cases, U, stream, "auto")
    tm, pm = _case_sweep(sv, torch, np, q, cases, U, stream, "masked")
    t32, p32 = _case_sweep(sv, torch, np, q32, cases, U, stream, "auto")
    t64, p64 = _case_sweep(sv, torch, np, c64, cases, U, stream, "auto")
    reps = 3
    rows = []
    for t, ctrls in cases:
        c = len(ctrls)
        ch = sum(1 for x in ctrls if x >= 6)  # controls scheduled over the block index
        scl = 2 * (1 << (n - 6 - ch))  # the touched blocks' scales
        alg_q = 2 * (1 << (n - c)) * 4 + scl  # satisfying amplitudes + their scales
        alg_32 = 2 * (1 << (n - c)) * 8 + scl
        alg_64 = 2 * (1 << (n - c)) * 8
        key = (t, ctrls)
        rows.append({"t": t, "c": c, "c_in_block": c - ch,
                     "q16_us": round(pq[key] * 1e3, 2), "q16_GBps": round(alg_q / pq[key] / 1e6, 1),
                     "q16_masked_us": round(pm[key] * 1e3, 2),
                     "q32_us": round(p32[key] * 1e3, 2), "q32_GBps": round(alg_32 / p32[key] / 1e6, 1),
                     "c64_us": round(p64[key] * 1e3, 2), "c64_GBps": round(alg_64 / p64[key] / 1e6, 1)})
    ng = reps * len(cases)
    out["sweep_n28"] = {"q16_gates_per_s": round(ng / (tq / 1e3), 1),
                        "q16_masked_gates_per_s": round(ng / (tm / 1e3), 1),
                        "q32_gates_per_s": round(ng / (t32 / 1e3), 1),
                        "c64_gates_per_s": round(ng / (t64 / 1e3), 1), "rows": rows}
    del q, q32, c64
    torch.cuda.empty_cache()
    for bits, dtype in ((16, sv.SV_CQ16), (32, sv.SV_CQ32)):
        for name, circ in (("qft29", W.qft(29)), ("stream29", W.stream(29))):
            log("paper circuit", name, "%d-bit fixed point" % bits)
            st = sv.FixedState(29, dtype)
            row = {"gates": len(circ.gates)}
            for label, fl in (("masked", sv.SV_MASKED), ("scheduled", 0), ("scheduled_fused", sv.SV_FUSE)):
                p = sv.Circuit(29, circ, dtype=dtype, flags=fl)
                row[label + "_passes"] = p.info()["passes"]

                def run():
                    sv.sv_init(st, 1, stream=stream)
                    p.run(st, stream=stream)
                row[label + "_ms"] = round(_time_ms(torch, stream, run, 3), 3)
                row[label + "_J_rated"] = round(row[label + "_ms"] * 1e-3 * RATED_POWER_W, 2)
                if energy is not None:
                    j, w = _energy_per_run(torch, stream, run, energy)
                    if j is not None:
                        row[label + "_J_measured"] = round(j, 3)
                        row[label + "_W_avg"] = round(w, 1)
                p.close()
            row["masked_over_scheduled"] = round(row["masked_ms"] / row["scheduled_ms"], 2)
            out["%s_q%d" % (name, bits)] = row
            del st
            torch.cuda.empty_cache()
    # accuracy: QFT (as drawn, no swaps) of a random state against the
    # closed form ifft(psi[bit-reversed]) * sqrt(N)
    ne = 20
    log("QFT n=%d error against its closed form" % ne)
    psi0 = W.random_state(ne, 34)
    N = 1 << ne
    rev = np.zeros(N, dtype=np.int64)
    for b in range(ne):
        rev |= ((np.arange(N) >> b) & 1) << (ne - 1 - b)
    want = np.fft.ifft(psi0[rev]) * np.sqrt(N)
    circ = W.qft(ne)
    errs = {}
    for label, td, fl in (("c128", torch.complex128, 0), ("c64", torch.complex64, 0), ("q32", sv.SV_CQ32, 0),
                          ("q16", sv.SV_CQ16, 0), ("q32_fused", sv.SV_CQ32, sv.SV_FUSE),
                          ("q16_fused", sv.SV_CQ16, sv.SV_FUSE)):
        src = torch.from_numpy(psi0).to(dev)
        if isinstance(td, int):
            st = sv.FixedState(ne, td)
        else:
            st = torch.empty(N, dtype=td, device=dev)
        sv.sv_convert(st, src, stream=stream)
        sv.sv_apply_circuit(st, circ, flags=fl, stream=stream)
        res = torch.empty(N, dtype=torch.complex128, device=dev)
        sv.sv_convert(res, st, stream=stream)
        torch.cuda.synchronize()
        got = res.cpu().numpy()
        errs[label] = {"l2": float("%.3e" % np.linalg.norm(got - want)),
                       "max_over_maxabs": float("%.3e" % (np.abs(got - want).max() / np.abs(want).max()))}
    out["qft20_error_vs_closed_form"] = errs
    return out


def batch_occupancy(np, st, ns_tick, ns, workgroups, items=None):
    """From per-work-item [start, end] clock stamps of one persistent batched
    run (items[i] = the item's circuit; None: one item per circuit, i = c):
    the run's span, the mean number of workgroups busy with an item over the
    span against the workgroups launched, the longest circuit (first start to
    last end of its items), and per width n the count and mean/max time per
    circuit."""
    if items is None:
        items = list(range(len(ns)))
    items = np.asarray(items)
    st = st[:2 * len(items)]
    t0, t1 = st[0::2].astype(np.float64), st[1::2].astype(np.float64)
    span = (t1.max() - t0.min()) * ns_tick * 1e-6
    busy = (t1 - t0) * ns_tick * 1e-6
    c0 = np.full(len(ns), np.inf)
    c1 = np.full(len(ns), -np.inf)
    np.minimum.at(c0, items, t0)
    np.maximum.at(c1, items, t1)
    ctime = (c1 - c0) * ns_tick * 1e-6
    per = {}
    for n in sorted(set(ns)):
        sel = np.array(ns) == n
        per[str(n)] = [int(sel.sum()), round(float(ctime[sel].mean()), 4), round(float(ctime[sel].max()), 4)]
    last_start = (t0.max() - t0.min()) * ns_tick * 1e-6
    counts = np.bincount(items, minlength=len(ns))
    return {"span_ms": round(span, 3), "workgroups": workgroups, "items": int(len(items)),
            "split_circuits": int((counts > 1).sum()),
            "mean_busy_workgroups": round(float(busy.sum() / span), 1),
            "utilisation": round(float(busy.sum() / span / workgroups), 3),
            "longest_circuit_ms": round(float(ctime.max()), 3), "last_start_ms": round(last_start, 3),
            "per_n_count_mean_max_ms": per}


def measure_extras(sv, W, torch, np, stream, with_layered, psi_host=None, cases=None, U=None):
    """Adjoint gradients (n=24 ansatz), batched circuits (4096 uneven circuits), the paper's
    QFT and streaming circuits at 29 qubits, fixed-point states, and optionally the
    layered n=32 circuit."""
    out = {}
    dev = torch.device("cuda:0")
    # ---- adjoint gradients: n=24 HEA, 768 parameters
    log("adjoint: n=24 ansatz")
    c3, H = W.hea_problem_n24()
    params = torch.from_numpy(c3.params).to(dev)
    psi = torch.empty(1 << c3.n, dtype=torch.complex128, device=dev)
    work = torch.empty_like(psi)
    lam = torch.empty_like(psi)
    plan = sv.Circuit(c3.n, c3, nparams=c3.nparams, flags=sv.SV_FUSE)
    gates = sv.circuit_gates(c3)
    terms = sv.pauli_terms(H)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    grad = torch.empty(c3.nparams, dtype=torch.float64, device=dev)

    def fwd():
        sv.sv_init(psi, 0, stream=stream)
        plan.run(psi, params, stream=stream)
        sv.sv_expect(psi, terms, out=loss, stream=stream)

    aplan = sv.AdjointPlan(c3.n, gates, terms, c3.nparams)

    def bwd():
        sv.sv_copy_state(work, psi, stream=stream)
        aplan.run(work, lam, params, grad=grad, stream=stream)

    def bwd_once():
        sv.sv_copy_state(work, psi, stream=stream)
        sv.sv_adjoint_grad(work, lam, gates, params, terms, grad=grad, stream=stream)

    t_f = _time_ms(torch, stream, fwd, 5)
    t_b = _time_ms(torch, stream, bwd, 5)
    t_b1 = _time_ms(torch, stream, bwd_once, 5)
    out["adjoint_hea_n24"] = {
        "n": c3.n, "params": c3.nparams, "gates": len(c3.gates), "forward_ms": round(t_f, 3),
        "backward_ms": round(t_b, 3), "backward_over_forward": round(t_b / t_f, 2),
        "backward_one_shot_ms": round(t_b1, 3),
        "gradients_per_s": round(1e3 / t_b, 3), "param_derivatives_per_s": round(c3.nparams * 1e3 / t_b, 1),
        "forward_passes": plan.info()["passes"]}
    plan.close()
    aplan.close()
    del psi, work, lam
    torch.cuda.empty_cache()
    # ---- expectation values: the chain ZZ + X Hamiltonian (47 / 55 terms), every dtype
    for n_e in (24, 28):
        log("expectation: n=%d chain Hamiltonian, four dtypes" % n_e)
        h_arr = sv.pauli_terms(W.zz_x_hamiltonian(n_e, 5))
        ps = torch.randn(1 << n_e, dtype=torch.complex128, device=dev)
        ps /= torch.linalg.vector_norm(ps)
        states = {"c128": ps, "c64": ps.to(torch.complex64)}
        for name, code in (("q16", sv.SV_CQ16), ("q32", sv.SV_CQ32)):
            q = sv.FixedState(n_e, code)
            sv.sv_convert(q, ps)
            states[name] = q
        eo = torch.empty(1, dtype=torch.float64, device=dev)
        row = {"terms": len(h_arr)}
        for name, st_ in states.items():
            ms = _time_ms(torch, stream, lambda: sv.sv_expect_noalloc(st_, h_arr, eo, stream=stream), 5)
            nbytes = sv.sv_state_bytes(n_e, {"c128": sv.SV_C128, "c64": sv.SV_C64, "q16": sv.SV_CQ16,
                                             "q32": sv.SV_CQ32}[name])
            row[name] = {"ms": round(ms, 3), "one_read_GBps": round(nbytes / ms / 1e6, 1)}
        out["expect_chain_n%d" % n_e] = row
        del states, ps
        torch.cuda.empty_cache()
    # ---- batched: 4096 uneven circuits forward (complex128 and complex64) and batched adjoint
    for dt, td in (("c128", torch.complex128), ("c64", torch.complex64)):
        log("batched: 4096 uneven circuits", dt)
        circs = W.uneven_batch()
        ns = [c.n for c in circs]
        offs = np.concatenate([[0], np.cumsum([1 << n for n in ns])])
        buf = torch.zeros(int(offs[-1]), dtype=td, device=dev)
        views = [buf[int(offs[i]):int(offs[i + 1])] for i in range(len(circs))]
        t0 = time.perf_counter()
        batch = sv.Batch(views, circs)
        t_create = (time.perf_counter() - t0) * 1e3
        t_b4 = _time_ms(torch, stream, lambda: batch.run(stream=stream), 3)
        t0 = time.perf_counter()
        sv.sv_apply_circuits_batched(views, circs, stream=stream)
        torch.cuda.synchronize()
        t_once = (time.perf_counter() - t0) * 1e3
        # per-circuit device clock stamps of one more run: time per circuit
        # width, and how busy the persistent workgroups are over the run
        items = batch.items()
        stamps = torch.zeros(2 * max(len(circs), len(items)), dtype=torch.int64, device=dev)
        ns_tick = batch.set_timing(stamps)
        batch.run(stream=stream)
        torch.cuda.synchronize()
        batch.set_timing(None)
        occ = batch_occupancy(np, stamps.cpu().numpy(), ns_tick, ns,
                              min(len(items), 2 * torch.cuda.get_device_properties(0).multi_processor_count),
                              items)
        ngates = sum(len(c.gates) for c in circs)
        alg = sum(len(c.gates) * (1 << c.n) * 2 * (16 if dt == "c128" else 8) for c in circs)
        out["batched_uneven4096_" + dt] = {"circuits": len(circs), "gates": ngates, "ms": round(t_b4, 2),
                                        "circuits_per_s": round(len(circs) * 1e3 / t_b4, 1),
                                        "gate_updates_per_s": round(ngates * 1e3 / t_b4, 1),
                                        "unfused_equivalent_GBps": round(alg / t_b4 / 1e6, 1),
                                        "plan_ms": round(t_create, 1), "one_shot_ms": round(t_once, 1),
                                        "occupancy": occ}
        batch.close()
        del buf, views
        torch.cuda.empty_cache()
    log("batched adjoint: 256 x n=16")
    pairs = W.hea_batch_n16()
    circs = [c for c, _ in pairs]
    hams = [h for _, h in pairs]
    buf = torch.zeros(len(circs) << 16, dtype=torch.complex128, device=dev)
    lbuf = torch.empty_like(buf)
    views = [buf[i << 16:(i + 1) << 16] for i in range(len(circs))]
    lviews = [lbuf[i << 16:(i + 1) << 16] for i in range(len(circs))]
    bparams = torch.from_numpy(np.concatenate([c.params for c in circs])).to(dev)
    bgrad = torch.empty(bparams.numel(), dtype=torch.float64, device=dev)
    bloss = torch.empty(len(circs), dtype=torch.float64, device=dev)

    hbatch = sv.Batch(views, circs, lam_states=lviews, hamiltonians=hams)

    def bfwd():
        buf.zero_()
        buf[::1 << 16] = 1
        hbatch.run(bparams, stream=stream)

    def bboth():
        bfwd()
        hbatch.adjoint(bparams, grad=bgrad, loss=bloss, stream=stream)

    t_bf = _time_ms(torch, stream, bfwd, 3)
    t_bb = _time_ms(torch, stream, bboth, 3) - t_bf
    stamps = torch.zeros(2 * len(circs), dtype=torch.int64, device=dev)
    with torch.cuda.stream(stream):
        bfwd()
        ns_tick = hbatch.set_timing(stamps)  # stamps of the adjoint run only
        hbatch.adjoint(bparams, grad=bgrad, loss=bloss, stream=stream)
    torch.cuda.synchronize()
    hbatch.set_timing(None)
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    # the batched adjoint runs one 1024-lane workgroup per circuit when there
    # are at most as many circuits as CUs, else two 512-lane ones per CU
    occ = batch_occupancy(np, stamps.cpu().numpy(), ns_tick, [16] * len(circs),
                          len(circs) if len(circs) <= cus else 2 * cus)
    out["batched_adjoint_hea256_n16"] = {"circuits": len(circs), "n": 16, "params_each": circs[0].nparams,
                                      "forward_ms": round(t_bf, 2), "backward_ms": round(t_bb, 2),
                                      "gradients_per_s": round(len(circs) * 1e3 / t_bb, 1), "occupancy": occ}
    hbatch.close()
    del buf, lbuf, views, lviews
    torch.cuda.empty_cache()
    # ---- dense k-qubit block on matrix cores (4 GiB states)
    for dt, td, n_d, k in (("c128", torch.complex128, 28, 4), ("c64", torch.complex64, 29, 5)):
        log("dense block", dt, "k=%d n=%d" % (k, n_d))
        st = torch.zeros(1 << n_d, dtype=td, device=dev)
        rng = np.random.default_rng(k)
        z = rng.standard_normal((1 << k, 1 << k)) + 1j * rng.standard_normal((1 << k, 1 << k))
        M, _ = np.linalg.qr(z)
        ms = _time_ms(torch, stream, lambda: sv.sv_apply_dense_low(st, k, M, stream=stream), 5)
        amps = 1 << n_d
        byts = 2 * amps * (16 if dt == "c128" else 8)
        flops = amps * (8 << k)  # 2^(k+1) reals per row times 2^(k+1) multiply-adds
        out["dense_k%d_n%d_%s" % (k, n_d, dt)] = {"ms": round(ms, 3), "GBps": round(byts / ms / 1e6, 1),
                                                  "TFLOPs": round(flops / ms / 1e9, 2),
                                                  "hbm_frac": round(byts / ms / 1e6 / HBM_PEAK_GBPS, 3)}
        del st
        torch.cuda.empty_cache()
    # ---- the paper's 29-qubit circuits, masked vs scheduled (vs fused), with
    # energy per circuit from the board's energy counter where readable
    energy = _energy_reader()
    for name, circ in (("qft29", W.qft(29)), ("stream29", W.stream(29))):
        for dt, td in (("c64", torch.complex64), ("c128", torch.complex128)):
            log("paper circuit", name, dt)
            st = torch.empty(1 << 29, dtype=td, device=dev)
            row = {"gates": len(circ.gates)}
            for label, fl in (("masked", sv.SV_MASKED), ("scheduled", 0), ("scheduled_fused", sv.SV_FUSE)):
                p = sv.Circuit(29, circ, dtype=sv.SV_C128 if dt == "c128" else sv.SV_C64, flags=fl)

                def run():
                    sv.sv_init(st, 1, stream=stream)
                    p.run(st, stream=stream)
                row[label + "_ms"] = round(_time_ms(torch, stream, run, 3), 3)
                # the paper's method: time x rated board power
                row[label + "_J_rated"] = round(row[label + "_ms"] * 1e-3 * RATED_POWER_W, 2)
                if energy is not None:
                    j, w = _energy_per_run(torch, stream, run, energy)
                    if j is not None:
                        row[label + "_J_measured"] = round(j, 3)
                        row[label + "_W_avg"] = round(w, 1)
                p.close()
            row["masked_over_scheduled"] = round(row["masked_ms"] / row["scheduled_ms"], 2)
            out["%s_%s" % (name, dt)] = row
            del st
            torch.cuda.empty_cache()
    # ---- qubit remapping: controls on the lowest qubits moved to high bits
    log("low-control circuit n=28 c128, with and without SV_REMAP")
    lc = W.low_control_circuit(n=28, ngates=24)
    st = torch.empty(1 << 28, dtype=torch.complex128, device=dev)
    row = {"gates": len(lc.gates)}
    for label, fl in (("scheduled", 0), ("scheduled_remap", sv.SV_REMAP)):
        p = sv.Circuit(28, lc, flags=fl)
        row[label + "_passes"] = p.info()["passes"]

        def run():
            sv.sv_init(st, 0, stream=stream)
            p.run(st, stream=stream)
        row[label + "_ms"] = round(_time_ms(torch, stream, run, 3), 3)
        p.close()
    out["low_control_n28"] = row
    del st
    torch.cuda.empty_cache()
    if psi_host is not None:
        out["fixed_point"] = measure_fixed_point(sv, W, torch, np, stream, psi_host, cases, U, energy)
    if with_layered:
        log("layered circuit: n=32 complex128")
        c2 = W.layered_circuit_n32()
        st = torch.empty(1 << 32, dtype=torch.complex128, device=dev)
        row = {"gates": len(c2.gates)}
        for label, fl in (("unfused", 0), ("fused", sv.SV_FUSE)):
            p = sv.Circuit(32, c2, flags=fl)
            row[label + "_passes"] = p.info()["passes"]

            def run():
                sv.sv_init(st, 0, stream=stream)
                p.run(st, stream=stream)
            row[label + "_ms"] = round(_time_ms(torch, stream, run, 1), 1)
            p.close()
        out["layered_n32"] = row
        del st
        torch.cuda.empty_cache()
    return out


METRIC = "gate updates/s & HBM GB/s vs #controls (n=28-32); adjoint grads/s"


def cpu_model():
    """CPU model name and physical core count of this host (from /proc/cpuinfo)."""
    model, cores = None, set()
    phys = core = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                k, _, v = line.partition(":")
                k, v = k.strip(), v.strip()
                if k == "model name" and model is None:
                    model = v
                elif k == "physical id":
                    phys = v
                elif k == "core id":
                    core = v
                elif not k and phys is not None:
                    cores.add((phys, core))
                    phys = core = None
        if phys is not None:
            cores.add((phys, core))
    except OSError:
        pass
    return model, (len(cores) or None)


def write_detail(detail, path):
    """Write the per-row tables and extra measurements as JSON (also echoed on
    stderr); returns the path written, or None."""
    log("detail " + json.dumps(detail, separators=(",", ":")))
    if not path:
        return None
    try:
        d = os.path.dirname(os.path.abspath(path))
        os.makedirs(d, exist_ok=True)
        with open(path, "w") as fh:
            json.dump(detail, fh, indent=1)
        return os.path.relpath(path, ROOT) if os.path.abspath(path).startswith(ROOT) else path
    except OSError as e:
        log("could not write %s: %s" % (path, e))
        return None


def compact_adjoint(extras):
    a = extras.get("adjoint_hea_n24")
    if not a:
        return None
    return {"workload": "n=24 ansatz, 768 params", "grads_per_s": a["gradients_per_s"],
            "param_derivs_per_s": a["param_derivatives_per_s"], "bwd_over_fwd": a["backward_over_forward"]}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="time budget of the CPU-oracle baseline sample (0 disables it)")
    ap.add_argument("--no-masked", action="store_true", help="skip the masked-baseline sweep")
    ap.add_argument("--pmc-copy", action="store_true",
                    help="first stream the HBM probe three times over a 1 GiB state, read and written in "
                         "place (calibration of the rocprofv3 byte counters)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint, batched and paper-circuit measurements")
    ap.add_argument("--no-protocol", action="store_true",
                    help="skip the graph-launched per-gate sweeps (n=28 and n=32)")
    ap.add_argument("--no-n32", action="store_true", help="skip the n=32 graph-launched sweep (64 GiB state)")
    ap.add_argument("--layered-n32", action="store_true",
                    help="also time the layered n=32 circuit (64 GiB) with and without LDS fusion (about a minute)")
    ap.add_argument("--summarize-profile", nargs=3, metavar=("TRACE_DIR", "FETCH_DIR", "WRITE_DIR"),
                    help="write profiles/ summaries from rocprofv3 CSV output of this script and exit")
    ap.add_argument("--positions-only", action="store_true",
                    help="run only the control-position sweep (one timed launch per point), for rocprofv3 "
                         "byte counters")
    ap.add_argument("--summarize-positions", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the control-position traffic summary from rocprofv3 --pmc output of "
                         "--positions-only and exit")
    ap.add_argument("--detail-out", default=os.path.join(ROOT, "gpurun_out", "bench_detail.json"),
                    help="file receiving the per-row tables and extra measurements as JSON ('' disables)")
    ap.add_argument("--fused-only", action="store_true",
                    help="run once each the fused layered circuit (n=28), QFT29 and the n=24 adjoint, for counters")
    ap.add_argument("--expect-only", action="store_true",
                    help="run one expectation call each on n=24 complex128 and 16-bit states, for counters")
    ap.add_argument("--summarize-counters", nargs="+", metavar="ARG",
                    help="NAME CMDFILE DIR...: per-kernel averages of rocprofv3 --pmc passes into "
                         "profiles/counters_NAME.md (CMDFILE: the commands, one per line)")
    ap.add_argument("--summarize-trace", metavar="TRACE_DIR",
                    help="write the all-kernel summary of a full run from rocprofv3 --kernel-trace output and exit")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    if args.summarize_counters:
        name, cmdfile, *dirs = args.summarize_counters
        with open(cmdfile) as fh:
            cmds = [l.strip() for l in fh if l.strip()]
        summarize_counters(name, cmds, dirs)
        return
    if args.summarize_profile:
        summarize_profile(*args.summarize_profile)
        return
    if args.summarize_positions:
        summarize_positions(*args.summarize_positions)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(only its sharding design exists); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    import paper_2411_18354_amd as sv

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.fused_only:
        run_fused_only(sv, W, torch, np, torch.cuda.Stream(device=dev))
        return
    if args.expect_only:
        run_expect_only(sv, W, torch, np, torch.cuda.Stream(device=dev))
        return
    n = N_QUBITS
    log("generating n=%d input state" % n)
    psi_host = W.random_state(n, seed=1)
    U = np.asarray(W.sweep_unitary(seed=2), dtype=np.float64)
    cases = W.gate_sweep_cases(n, seed=3)
    # interleave targets and control counts so consecutive gates touch
    # unrelated amplitudes
    order = sorted(range(len(cases)), key=lambda i: (len(cases[i][1]), cases[i][0]))
    cases = [cases[i] for i in order]
    d = torch.from_numpy(psi_host).to(dev)
    stream = torch.cuda.Stream(device=dev)  # default priority
    if args.pmc_copy:
        a = torch.zeros(1 << 26, dtype=torch.complex128, device=dev)  # 1 GiB
        for _ in range(3):
            sv.sv_hbm_probe(a, 0, 0, "rmw", stream=stream)
        torch.cuda.synchronize()
        del a

    if args.positions_only:
        rows = control_position_sweep(sv, torch, np, d, U, stream, n, reps=1)
        print(json.dumps({"control_positions": rows}), flush=True)
        return

    plans = {}
    for mode in ("auto", "masked"):
        for t, ctrls in cases:
            cm = sum(1 << q for q in ctrls)
            plans[(mode, t, ctrls)] = sv.sv_gate_plan(n, sv.SV_C128, t, cm, cm, mode)

    def sweep(mode, steps, warmup):
        """Warm-up steps, then `steps` timed steps of the sweep: HIP events
        around the whole region, around every step and around every gate
        (all created before the region; Python's collector paused inside)."""
        per = {(t, ctrls): [] for t, ctrls in cases}
        ng = len(cases)
        gev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps * ng)]
        sev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        with torch.cuda.stream(stream):
            for _ in range(warmup):
                for t, ctrls in cases:
                    sv.sv_apply_gate(d, t, ctrls, None, U, mode=mode, stream=stream)
            torch.cuda.synchronize()
            gc.disable()
            try:
                sev[0].record(stream)
                for k in range(steps):
                    for j, (t, ctrls) in enumerate(cases):
                        e0, e1 = gev[k * ng + j]
                        e0.record(stream)
                        sv.sv_apply_gate(d, t, ctrls, None, U, mode=mode, stream=stream)
                        e1.record(stream)
                    sev[k + 1].record(stream)
            finally:
                gc.enable()
        torch.cuda.synchronize()
        total_ms = sev[0].elapsed_time(sev[-1])
        step_ms = [sev[k].elapsed_time(sev[k + 1]) for k in range(steps)]
        for k in range(steps):
            for j, key in enumerate(cases):
                e0, e1 = gev[k * ng + j]
                per[key].append(e0.elapsed_time(e1))
        return total_ms, per, step_ms

    torch.cuda.synchronize()
    ceiling = {"rmw_GBps": None, "read_GBps": None}
    if not args.pmc_copy:  # under the byte counters the probe is the calibration only
        log("HBM probe over the 4 GiB state")
        ceiling = hbm_ceiling(sv, torch, np, d, stream)
    log("scheduled sweep: %d warmup + %d timed steps of %d gates" % (args.warmup, args.steps, len(cases)))
    total_ms, per, step_ms = sweep("auto", args.steps, args.warmup)
    masked_total, per_m = (None, None)
    if not args.no_masked:
        log("masked sweep")
        masked_total, per_m, _ = sweep("masked", args.steps, args.warmup)

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
                "probe_rmw_GBps": ceiling["rmw_GBps"], "probe_read_GBps": ceiling["read_GBps"],
                "frac_of_probe": round(achieved / ceiling["rmw_GBps"], 3) if ceiling["rmw_GBps"] else None,
                "kernel": dom, "avg_launch_us": round(avg_ms * 1e3, 2),
                "alg_bytes_per_launch": avg_bytes, "launches": ks["launches"],
                "kernel_source_hash": src_hash}

    positions = None
    if not args.no_extras:
        positions = control_position_sweep(sv, torch, np, d, U, stream, n)

    protocol = None
    if not args.no_extras and not args.no_protocol:
        log("graph-launched sweep, n=28 (control values rotated against the Infinity Cache)")
        protocol = graph_protocol(sv, torch, np, d, n, cases, U, stream)

    extras = None
    if not args.no_extras:
        del d
        torch.cuda.empty_cache()
        extras = measure_extras(sv, W, torch, np, stream, args.layered_n32, psi_host, cases, U)

    protocol32 = None
    if not args.no_extras and not args.no_protocol and not args.no_n32:
        protocol32 = protocol_n32(sv, W, torch, np, stream, U)

    cpu = None
    cpu_detail = None
    if args.cpu_seconds > 0:
        import oracle
        log("CPU oracle baseline (budget %.0f s)" % args.cpu_seconds)
        Uc = oracle.gate_matrix("U", matrix=tuple(U))
        host = psi_host.copy()
        threads = oracle.num_threads()
        per_case = [[] for _ in cases]
        done, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < args.cpu_seconds:
            t, ctrls = cases[done % len(cases)]
            g0 = time.perf_counter()
            oracle.apply_gate(host, n, t, ctrls, (), Uc)
            per_case[done % len(cases)].append(time.perf_counter() - g0)
            done += 1
        el = time.perf_counter() - t0
        # the same loop on one thread, over a shorter budget
        oracle.set_num_threads(1)
        done1, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < args.cpu_seconds / 3:
            t, ctrls = cases[done1 % len(cases)]
            oracle.apply_gate(host, n, t, ctrls, (), Uc)
            done1 += 1
        el1 = time.perf_counter() - t1
        oracle.set_num_threads(threads)
        # the 200-gate n=12 random circuit, once, all threads
        c0 = W.random_gates_n12()
        g0 = time.perf_counter()
        oracle.run_circuit(c0)
        cfg0_ms = (time.perf_counter() - g0) * 1e3
        model, phys = cpu_model()
        cpu = {"value": round(done / el, 4), "unit": "gate updates/s", "cores": threads,
               "kind": "oracle", "cpu_model": model, "physical_cores": phys,
               "single_thread_value": round(done1 / el1, 4),
               "sample": "%d gates of the %d-gate sweep in order on the same n=28 state, plain loop over "
                         "all 2^28 indices per gate, OpenMP, %.1f s (single thread: %d gates, %.1f s)"
                         % (done, len(cases), el, done1, el1)}
        cpu_detail = {"per_case_ms_mean": [{"t": t, "c": len(ctrls), "controls": list(ctrls), "calls": len(v),
                                            "ms": round(1e3 * float(np.mean(v)), 2) if v else None}
                                           for (t, ctrls), v in zip(cases, per_case)],
                      "random_gates_n12_200_gates_ms": round(cfg0_ms, 2), "threads": threads}
        del host

    by_c = {}
    for r in rows:
        by_c.setdefault(r["c"], []).append(r)
    cs = sorted(by_c)
    summary_by_c = {"c": cs, "eager_frac": [round(float(np.mean([r["sched_frac"] for r in by_c[c]])), 3)
                                            for c in cs]}
    if protocol:
        ps = protocol_summary(protocol)
        summary_by_c["graph_frac"] = ps.get("sched_frac")
        summary_by_c["graph_masked_frac"] = ps.get("masked_frac")
        summary_by_c["graph_masked_over_sched"] = ps.get("masked_over_sched")
        summary_by_c["graph_probe_frac"] = ps.get("probe_frac")
    if protocol32:
        ps = protocol_summary(protocol32)
        summary_by_c["n32_graph_frac"] = ps.get("sched_frac")
        summary_by_c["n32_graph_masked_over_sched"] = ps.get("masked_over_sched")
    detail = {
        "step_ms": [round(x, 4) for x in step_ms],
        "sweep": rows,
        "graph_protocol_n28": protocol,
        "graph_protocol_n32": protocol32,
        "control_positions": positions,
        "extras": extras,
        "cpu_oracle": cpu_detail,
    }
    detail_path = write_detail(detail, args.detail_out)
    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "gate updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(total_ms / args.steps, 4),
        "step_ms_median_max": [round(float(np.median(step_ms)), 3), round(max(step_ms), 3)],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "n=28 complex128 controlled-gate sweep: Haar 2x2, t in {0,13,27} x c=0..8 "
                               "random controls (value 1), scheduled kernels, 27 gates per step",
                   "n": n, "gates_per_step": len(cases), "seeds": [1, 2, 3]},
        "hbm_GBps_alg": round(alg_total / total_ms / 1e6, 1),
        "roofline": {k: roofline[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic", "kernel",
                                              "avg_launch_us", "probe_rmw_GBps", "frac_of_probe")},
        "cpu_baseline": cpu,
        "masked_value": None if masked_total is None else round(ngates / (masked_total / 1e3), 2),
        "by_c": summary_by_c,
        "adjoint": None if not extras else compact_adjoint(extras),
        "detail": detail_path,
    }
    line = json.dumps(out, separators=(",", ":"))
    for k in ("graph_masked_frac", "graph_probe_frac", "n32_graph_masked_over_sched", "eager_frac",
              "graph_masked_over_sched"):
        if len(line) <= 2000:  # keep the last line short enough for any log tail
            break
        out["by_c"].pop(k, None)
        line = json.dumps(out, separators=(",", ":"))
    print(line, flush=True)


if __name__ == "__main__":
    main()
