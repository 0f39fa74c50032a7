"""Benchmark of the FSMP hot path on one MI355X.

One step = one pass of the whole path over one batch: fsmp_sample (prologue + chain
kernels: every chain's Gibbs / RJMCMC sweeps) and fsmp_posterior (with P(N = k)), with the
waveforms already resident in device memory when the timed region starts.  The default
workload is the largest single-GPU one, the uneven batch: 250,000 windows of 128 / 256 /
512 / 1,024 / 2,048 samples, lambda ~ logU[0.05, 100] (PE capacities 16-160), rise 2 /
decay 25 ns light curve, one chain per waveform, FP64, with the kernel design per PE
capacity (fsmp_autotune) and the sweeps per waveform (fsmp_autotune_steps: 500-4,000 from
a 200-sweep pilot's batch-means MCSE of N) tuned before the timed region.

Prints one JSON line: waveforms/s (whole job) and MCMC steps/s; the roofline of the chain
launch with the longest time in the step (HIP events on its own stream inside the timed
region); the oracle timed on the host cores over a bounded sample; and as extra keys the
FP32+refresh form at refresh_M = 16, 64, 256, the batched workload (100,000 x 1,024
samples, 4 chains x 1,000 sweeps), the serving loop over trigger rates, the Lucy-Richardson
initialisation stage and the MCP-PMT mixture law.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload uneven|batched|plain|pileup]

Roofline: algorithmic bytes = the words of a packed Cholesky factor that the proposals must
read and the accepted moves must edit (birth K(K+1)/2 + 2K + 3 and K + 3; death
(K-j)(K-j+1)/2 + 1 and (K-1-j)(K-j) + K(K+1)/2; update both, with the birth on K - 1 PEs;
K the PE count, j the removed PE's index), 8 bytes a word, counted on the device for every
chain (fsmp_samples.work), summed over the chains of the launch, over the launch's mean
duration; against the 8 TB/s HBM peak, and against the LDS stream bandwidth that
liblds_probe.so measures on the device (the LDS fraction).  `traffic` is the HBM bytes per
launch that rocprofv3 counters recorded for that kernel (FETCH_SIZE + WRITE_SIZE, scaled by
the factor a plain copy of known size gives), read from profiles/traffic_<workload>.json
while the kernel source is unchanged:

    rocprofv3 --pmc FETCH_SIZE -d DIR_F -o pmc -- python bench.py --pmc-run
    rocprofv3 --pmc WRITE_SIZE -d DIR_W -o pmc -- python bench.py --pmc-run
    python bench.py --pmc-summary DIR_F DIR_W

The chain kernels are limited by instruction issue, not by bytes: two more counter runs give
each kernel's VALU busy fraction (4 x SQ_ACTIVE_INST_VALU SIMD cycles over 1,024 SIMDs x
2.4 GHz x its duration; a wave64 VALU instruction occupies its SIMD 4 cycles, so the issue
ceiling is 614.4e9 wave-instructions/s, the FP64 vector peak over 128 flops):

    rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES
              SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU -d DIR_A -o pmc -- python bench.py --pmc-run
    rocprofv3 --pmc SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SMEM SQ_INSTS_FLAT SQ_WAIT_ANY
              SQ_INSTS_BRANCH GRBM_GUI_ACTIVE -d DIR_B -o pmc -- python bench.py --pmc-run
    python bench.py --issue-summary DIR_A DIR_B
"""
import hashlib
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12  # MI355X dense FP64 vector, FLOP/s
PEAK_HBM = 8.0e12    # MI355X HBM3E, bytes/s
N_SIMD, CLOCK_HZ = 1024, 2.4e9  # MI355X: 256 CUs x 4 SIMDs, peak engine clock
KSRC = os.path.join(ROOT, "paper_2403_03156_amd", "csrc", "fsmp_kernels.hip")
COPY_PROBE_MIB = 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="uneven")
    ap.add_argument("--n-wave", type=int, default=0, help="override the workload's waveform count")
    ap.add_argument("--chain-steps", type=int, default=0, help="fixed sweeps per chain (no step autotuning)")
    ap.add_argument("--refresh", type=int, default=-1,
                    help="FP64 form: rebuild G^-1 from scratch every this many sweeps (-1: the sampler's default)")
    ap.add_argument("--trial-steps", type=int, default=100,
                    help="mean sweeps per chain of the design autotuner's trial (proportional to the tuned counts)")
    ap.add_argument("--target-mcse", type=float, default=0.02,
                    help="relative batch-means MCSE of N the step autotuner aims at")
    ap.add_argument("--cpu-wave", type=int, default=6000, help="waveforms in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve", action="store_true", help="only the serving study (rates x precisions)")
    ap.add_argument("--serve-events", type=int, default=160,
                    help="events per serving run (enough that one event's drain after the last arrival is a "
                         "few percent of the arrival window at the sustainable rates)")
    ap.add_argument("--serve-rates", default="50,100,150,200,250,300,350,400,2000,5000,10000,20000",
                    help="comma-separated event rates (Hz)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--hw-queues", type=int, default=8,
                    help="hardware queues the process asks HIP for (GPU_MAX_HW_QUEUES, read once when the "
                         "runtime starts; HIP's default is 4): with 8 every capacity bucket of a step runs on a "
                         "lane of its own; 0 leaves the environment as it is")
    ap.add_argument("--legs", default="fp32,batched,lucy,mcp",
                    help="comma-separated extra legs to run (fp32, batched, lucy, mcp; empty: none)")
    ap.add_argument("--lucy-iter", type=int, default=2000, help="Lucy-Richardson iterations of the init stage (0: skip)")
    ap.add_argument("--no-mcp", action="store_true", help="skip the MCP-PMT mixture-law leg")
    ap.add_argument("--pmc-run", action="store_true",
                    help="one untimed step after a plain device copy of known size (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs into profiles/")
    ap.add_argument("--issue-summary", nargs=2, metavar=("SQ_DIR_A", "SQ_DIR_B"),
                    help="summarise two rocprofv3 --pmc runs of SQ counters into profiles/")
    ap.add_argument("--step-ms", type=float, default=0.0, help="concurrent step time for --issue-summary")
    ap.add_argument("--precision-study", type=int, default=0, metavar="N_WAVE",
                    help="only the precision study: FP64 and FP32+refresh against the oracle on N_WAVE high pile-up "
                         "waveforms per noise level")
    ap.add_argument("--trace-summary", nargs=2, metavar=("TRACE_DIR", "LAST"),
                    help="per-kernel durations of the last LAST dispatches of a rocprofv3 --kernel-trace run")
    return ap.parse_args()


def kernel_label(name):
    """bench name of a chain / prologue kernel from its demangled rocprofv3 name"""
    import re
    # chain_kernel<KCAP, lanes per chain, wavefronts per workgroup, G^-1 in device memory,
    # replay, FP32 storage, mixture charge law>
    m = re.search(r"chain_kernel<(\d+), (\d+), (\d+), (true|false)(?:, (true|false))?(?:, (true|false))?"
                  r"(?:, (true|false))?>", name)
    if m:
        if m.group(5) == "true":
            return "chain_replay_k" + m.group(1)
        base = "chain_group_dm" if m.group(4) == "true" else "chain_group"
        return (base + ("_fp32" if m.group(6) == "true" else "") + ("_mcp" if m.group(7) == "true" else "")
                + "_k" + m.group(1))
    m = re.search(r"chain_lane_kernel<(\d+)>", name)
    if m:
        return "chain_lane_k" + m.group(1)
    for k in ("prologue_kernel", "posterior_kernel"):
        if k in name:
            return k.replace("_kernel", "")
    return None


def source_hash():
    """SHA-256 of the kernel source with its comments and blank space removed: what the
    compiled kernels depend on, so that a comment edit keeps recorded counters valid"""
    import re
    text = open(KSRC).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    text = re.sub(r"//[^\n]*", " ", text)
    text = " ".join(text.split())
    return hashlib.sha256(text.encode()).hexdigest()


def pmc_summary(fdir, wdir, workload):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of two rocprofv3 --pmc runs -> HBM bytes per
    launch of each kernel, scaled by what the counters read for the plain copy of known size."""
    import csv
    import glob

    def read(d, counter):
        rows = {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                if r.get("Counter_Name") != counter:
                    continue
                key = (r.get("Dispatch_Id"), r.get("Kernel_Name"))
                rows[key] = rows.get(key, 0.0) + float(r["Counter_Value"])
        return rows

    fetch, write = read(fdir, "FETCH_SIZE"), read(wdir, "WRITE_SIZE")
    copy_bytes = COPY_PROBE_MIB * 2 ** 20

    def by_kernel(rows):
        # the last dispatch of each kernel: the counter run's step comes after the set-up
        # (autotuner trials and pilot) and after the copy probe
        last = {}
        for (did, name), kib in rows.items():
            lab = kernel_label(name)
            if lab is None and ("copy" in name.lower() or "elementwise" in name.lower()):
                lab = "copy"
            if lab and (lab not in last or int(did) > last[lab][0]):
                last[lab] = (int(did), kib * 1024.0)
        return {lab: [v] for lab, (_, v) in last.items()}

    def copies(rows):
        return [kib * 1024.0 for (_, name), kib in rows.items()
                if kernel_label(name) is None and ("copy" in name.lower() or "elementwise" in name.lower())]

    fk, wk = by_kernel(fetch), by_kernel(write)
    # the copy probe is the largest copy-like dispatch: it reads and writes copy_bytes
    f_scale = copy_bytes / max(copies(fetch) or [copy_bytes])
    w_scale = copy_bytes / max(copies(write) or [copy_bytes])
    kern = {}
    for lab in sorted(set(fk) | set(wk)):
        if lab == "copy":
            continue
        f = float(np.mean(fk.get(lab, [0.0]))) * f_scale
        w = float(np.mean(wk.get(lab, [0.0]))) * w_scale
        kern[lab] = {"fetch_bytes": f, "write_bytes": w, "hbm_bytes": f + w}
    res = {"workload": workload, "source_sha256": source_hash(), "fetch_scale": f_scale, "write_scale": w_scale,
           "copy_probe_bytes": copy_bytes, "kernels": kern}
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    json.dump(res, open(path, "w"), indent=1)
    print(json.dumps(res, indent=1))


def issue_summary(adir, bdir, workload, step_ms):
    """Per-kernel instruction mix and VALU busy fraction from two rocprofv3 --pmc runs of SQ
    counters (--pmc-run: the kernels run one at a time, so each duration is the kernel alone)."""
    import csv
    import glob

    def read(d):
        # the last dispatch of each kernel (the counter run's step, after the set-up)
        rows = []
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            rows += [r for r in csv.DictReader(open(f)) if kernel_label(r["Kernel_Name"]) is not None]
        last = {}
        for r in rows:
            lab = kernel_label(r["Kernel_Name"])
            last[lab] = max(last.get(lab, -1), int(r["Dispatch_Id"]))
        agg, t = {}, {}
        for r in rows:
            lab = kernel_label(r["Kernel_Name"])
            if int(r["Dispatch_Id"]) != last[lab]:
                continue
            agg.setdefault(lab, {})
            agg[lab][r["Counter_Name"]] = agg[lab].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            t[lab] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        return agg, t

    a, ta = read(adir)
    b, _ = read(bdir)
    lines = [f"# Instruction issue of the {workload} step, per kernel", "",
             "Commands (each counter pass a run of its own, the kernels of one step run one at a time):", "",
             "    rocprofv3 --pmc SQ_WAVES SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
             "SQ_WAIT_INST_ANY SQ_ACTIVE_INST_VALU --output-format csv -d " + adir + " -o pmc -- python bench.py "
             "--pmc-run",
             "    rocprofv3 --pmc SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR SQ_INSTS_SMEM SQ_INSTS_FLAT SQ_WAIT_ANY "
             "SQ_INSTS_BRANCH GRBM_GUI_ACTIVE --output-format csv -d " + bdir + " -o pmc -- python bench.py --pmc-run",
             f"    python bench.py --issue-summary {adir} {bdir}", "",
             f"Source sha256 of the kernels: `{source_hash()}`.", "",
             "VALU busy = 4 x SQ_ACTIVE_INST_VALU (quad-cycles; it reads 1.00-1.05 x SQ_INSTS_VALU here) over "
             f"{N_SIMD} SIMDs x {CLOCK_HZ / 1e9:.1f} GHz x the kernel's duration.  The issue ceiling, one wave64 VALU "
             f"instruction per SIMD every 4 cycles, is {N_SIMD * CLOCK_HZ / 4 / 1e9:.1f}e9 wave-instructions/s "
             "(the 78.6 TFLOP/s FP64 vector peak over 64 lanes x 2 flops).", "",
             "| kernel | ms alone | waves | VALU instr | VALU instr/s | VALU busy | SALU/VALU | LDS/VALU | "
             "branch/VALU | VMEM rd+wr/VALU |",
             "|---|---|---|---|---|---|---|---|---|---|"]
    busy_total = 0.0
    for lab in sorted(a, key=lambda k: -a[k].get("SQ_INSTS_VALU", 0.0)):
        v, w, t = a[lab], b.get(lab, {}), ta[lab]
        valu = v.get("SQ_INSTS_VALU", 0.0)
        busy = 4.0 * v.get("SQ_ACTIVE_INST_VALU", 0.0)
        busy_total += busy
        if valu <= 0:
            continue
        vm = w.get("SQ_INSTS_VMEM_RD", 0.0) + w.get("SQ_INSTS_VMEM_WR", 0.0)
        lines.append(f"| {lab} | {t * 1e3:.1f} | {v.get('SQ_WAVES', 0):.0f} | {valu:.3g} | {valu / t / 1e9:.0f}e9 | "
                     f"{busy / (N_SIMD * CLOCK_HZ * t):.1%} | {v.get('SQ_INSTS_SALU', 0) / valu:.2f} | "
                     f"{v.get('SQ_INSTS_LDS', 0) / valu:.3f} | {w.get('SQ_INSTS_BRANCH', 0) / valu:.3f} | "
                     f"{vm / valu:.3f} |")
    lines += ["", f"Whole step: {busy_total / 4:.3g} VALU quad-cycles; over the concurrent step of {step_ms:.1f} ms "
              f"that is {busy_total / (N_SIMD * CLOCK_HZ * step_ms * 1e-3):.1%} VALU busy on every SIMD.", ""]
    path = os.path.join(ROOT, "profiles", f"chain_kernels_{workload}_valu_issue.md")
    open(path, "w").write("\n".join(lines))
    print("\n".join(lines))


def trace_summary(tdir, last, workload):
    """mean / min / max duration of the last `last` dispatches of every chain, prologue and
    posterior kernel in a rocprofv3 --kernel-trace run (csv), as markdown"""
    import csv
    import glob
    rows = {}
    for f in glob.glob(os.path.join(tdir, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            lab = kernel_label(r["Kernel_Name"])
            if lab is None:
                continue
            ms = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
            rows.setdefault(lab, []).append((int(r["Dispatch_Id"]), ms, r["Kernel_Name"]))
    lines = [f"| kernel | label | dispatches averaged | average ms | min ms | max ms |", "|---|---|---|---|---|---|"]
    res = {}
    for lab in sorted(rows, key=lambda k: -np.mean([m for _, m, _ in sorted(rows[k])[-last:]])):
        sel = sorted(rows[lab])[-last:]
        ms = [m for _, m, _ in sel]
        res[lab] = float(np.mean(ms))
        lines.append(f"| `{sel[-1][2][:110]}` | {lab} | {len(ms)} | {np.mean(ms):.2f} | {min(ms):.2f} | {max(ms):.2f} |")
    print("\n".join(lines))
    return res


def recorded_traffic(workload, kernel):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_sha256") != source_hash() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["hbm_bytes"]


def step_traffic(workload, kernels, ms_per_step):
    """HBM bytes of a step from the recorded counters (every kernel of the step, the posterior
    included), and their rate over the step against the HBM peak; None if any is missing"""
    per = [recorded_traffic(workload, k) for k in list(kernels) + ["posterior"]]
    if any(v is None for v in per):
        return None
    tot = float(sum(per))
    return {"hbm_bytes": tot, "GBps": tot / (ms_per_step / 1e3) / 1e9, "frac": tot / (ms_per_step / 1e3) / PEAK_HBM}


def serving_run(fsmp, synth, pool, rate, n_events, precision, seed=0, n_streams=4, max_batch_wave=20000):
    """Poisson arrivals of trigger events (500-2000 channels drawn from a pool of synthetic
    channels, 1,024 samples each) submitted to the serving loop as they arrive; latency
    percentiles, throughput, and whether the run kept pace: it ends within 5% of the last
    arrival plus the median latency (a server that keeps pace drains one event after the last
    arrival), and the queue does not grow (the last third of the events waits at most 1.25x
    as long as the first third, plus 20 ms for the jitter of short waits).  The arrival
    window is about 1.5 s (n_events to 3 n_events events), so an overload of a few percent
    shows as a growing latency."""
    wl = synth.PRESETS["serving"]
    n_events = int(np.clip(round(rate * 1.5), n_events, 3 * n_events))
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, n_events)
    arrive = np.cumsum(gaps) - gaps[0]
    events = []
    L = 1024
    for e in range(n_events):
        n = int(rng.integers(500, 2001))
        idx = rng.integers(0, pool["n"], n)
        wave = pool["wave"].reshape(pool["n"], L)[idx].reshape(-1)
        events.append((e + 1, wave, np.arange(n + 1, dtype=np.int64) * L, pool["lam"][idx], pool["kmax"][idx]))
    kw = dict(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay, t0_min=wl.t0_min,
              t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q, n_steps=wl.n_steps,
              n_chains=1, seed=seed, precision=precision, refresh_M=64)
    srv = fsmp.Server(kw, n_streams=n_streams, max_batch_wave=max_batch_wave, memory_budget=32 << 30)
    # warm the server's buffers with one event (allocations happen once)
    srv.submit(1 << 40, events[0][1], events[0][2], events[0][3], events[0][4])
    while srv.result(1 << 40) is None:
        srv.progress(wait=True)
    lat, done, i = {}, 0, 0
    t0 = time.perf_counter()
    while done < n_events:
        now = time.perf_counter() - t0
        while i < n_events and arrive[i] <= now:
            eid, w, off, lam, km = events[i]
            srv.submit(eid, w, off, lam, km)
            i += 1
        srv.progress(wait=(i == n_events))
        for eid, *_ in events[:i]:
            if eid not in lat:
                r = srv.result(eid)
                if r is not None:
                    lat[eid] = r["latency"]
                    done += 1
        if i < n_events and done < i:
            time.sleep(0)
    t_end = time.perf_counter() - t0
    srv.close()
    waves = sum(len(e[3]) for e in events)
    l = np.array([lat[e[0]] for e in events])
    third = max(1, n_events // 3)
    served = waves / t_end
    offered = waves / max(arrive[-1], 1e-9)
    keeps_pace = bool(t_end <= 1.05 * (arrive[-1] + np.percentile(l, 50))
                      and l[-third:].mean() <= 1.25 * l[:third].mean() + 0.020)
    return {"rate_hz": rate, "events": n_events, "waveforms": waves, "precision": "fp32+refresh" if precision else "fp64",
            "p50_ms": float(np.percentile(l, 50) * 1e3), "p99_ms": float(np.percentile(l, 99) * 1e3),
            "arrival_window_ms": float(arrive[-1] * 1e3), "drain_ms": float((t_end - arrive[-1]) * 1e3),
            "mean_ms_first_third": float(l[:third].mean() * 1e3), "mean_ms_last_third": float(l[-third:].mean() * 1e3),
            "waveforms_per_s": served, "offered_waveforms_per_s": offered, "keeps_pace": keeps_pace}


def serving_pool(synth, n=20000, seed=5):
    wl = synth.PRESETS["serving"]
    b = synth.generate(wl, n_wave=n, seed=seed)
    return {"n": n, "wave": b["wave"], "lam": b["lam"], "kmax": synth.kmax_for(b["lam"])}


def serving_study(fsmp, synth, rates, n_events):
    """both precision forms over the rates; per form the saturation throughput (the most
    waveforms/s any of its runs served), and the largest sustained rate with the p50 / p99
    latency there.  A rate is sustained if its run kept pace (serving_run) and it offers at
    most 95% of the saturation throughput: a queue fed faster than it is served grows without
    bound, however slowly that shows within one run."""
    pool = serving_pool(synth)
    runs, best, sat = [], {}, {}
    for prec in (fsmp.FSMP_FP64, fsmp.FSMP_FP32_REFRESH):
        mine = []
        for rate in rates:
            r = serving_run(fsmp, synth, pool, rate, n_events, prec)
            print(f"[bench] serving {json.dumps(r)}", file=sys.stderr, flush=True)
            mine.append(r)
        top = max(r["waveforms_per_s"] for r in mine)
        for r in mine:
            r["sustained"] = bool(r["keeps_pace"] and r["offered_waveforms_per_s"] <= 0.95 * top)
            if r["sustained"] and r["rate_hz"] > best.get(r["precision"], {}).get("rate_hz", -1):
                best[r["precision"]] = {k: r[k] for k in ("rate_hz", "p50_ms", "p99_ms", "waveforms_per_s")}
        sat[mine[0]["precision"]] = top
        runs += mine
    return {"runs": runs, "saturation_waveforms_per_s": sat, "largest_sustained": best}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def lds_peak():
    """LDS stream bandwidth of device 0 in bytes/s (reads, writes) from liblds_probe.so"""
    import ctypes
    path = os.path.join(ROOT, "paper_2403_03156_amd", "liblds_probe.so")
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built (python -m paper_2403_03156_amd.build)")
    L = ctypes.CDLL(path)
    L.lds_probe.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    L.lds_probe.restype = ctypes.c_int
    r, w = ctypes.c_double(0.0), ctypes.c_double(0.0)
    rc = L.lds_probe(0, 400, ctypes.byref(r), ctypes.byref(w))
    if rc != 0:
        raise RuntimeError(f"lds_probe failed (HIP error {rc})")
    return r.value, w.value


def algorithmic_bytes(work):
    """bytes of a packed FP64 Cholesky factor the proposals must read and the accepted moves
    must edit (work counters 0 and 1, 8-byte words)"""
    return 8.0 * (work[:, 0].sum() + work[:, 1].sum())


def timed_steps(smp, one_step, n, warm):
    """warm untimed steps, then n timed ones (synchronised around); ms per step and the mean
    HIP-event time of every kernel launch"""
    import torch
    for _ in range(warm):
        one_step()
    torch.cuda.synchronize()
    smp.set_timing(True)
    kernel_ms = {}
    t0 = time.perf_counter()
    for _ in range(n):
        one_step()
        for t in smp.last_timings():  # waits for this step's kernels (events on their streams)
            kernel_ms.setdefault(t["name"], []).append(t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    smp.set_timing(False)
    return (t1 - t0) * 1e3 / n, kernel_ms


def serial_kernel_ms(smp, one_step):
    """one untimed step with the capacity buckets one after another on the caller's stream
    (the library takes its lane count from GPU_MAX_HW_QUEUES on each call; the HIP runtime
    read it once at start-up and keeps its queues): the HIP-event time of every launch alone"""
    import torch
    prev = os.environ.get("GPU_MAX_HW_QUEUES")
    os.environ["GPU_MAX_HW_QUEUES"] = "1"
    try:
        torch.cuda.synchronize()
        smp.set_timing(True)
        one_step()
        res = {t["name"]: float(t["ms"]) for t in smp.last_timings()}
        torch.cuda.synchronize()
    finally:
        smp.set_timing(False)
        if prev is None:
            del os.environ["GPU_MAX_HW_QUEUES"]
        else:
            os.environ["GPU_MAX_HW_QUEUES"] = prev
    return res


def precision_study(fsmp, synth, oracle, n_wave, n_steps=1000, refresh_M=64):
    """The high pile-up precision study (lambda ~ U[20, 100], charges N(1, 0.35), 1,024 samples)
    at sigma_eps = 0.05, 0.1, 0.2: per form (FP64, FP32+refresh) the relative error of every
    proposal's delta-nu against the oracle's extended-precision replay of that chain's log,
    and the relative errors |m - m_oracle| / max(|m_oracle|, 1) of the posterior means of N,
    total charge and t0 against the oracle's chains (same seeds), with the share of chains
    identical to the oracle's and the FP64 re-evaluations per proposal."""
    import concurrent.futures
    import torch
    base = synth.PRESETS["pileup"]
    rows = []
    for sig in (0.05, 0.1, 0.2):
        wl = synth.Workload("pileup", n_wave, base.lengths, "uniform", 20.0, 100.0, phi_kind=base.phi_kind,
                            tau_rise=base.tau_rise, tau_decay=base.tau_decay, sigma_q=0.35, sigma_eps=sig)
        b = synth.generate(wl, n_wave=n_wave, seed=41)
        km = synth.kmax_for(b["lam"])
        kz = int(km.max())
        burn = n_steps // 2
        p = oracle.make_params(ser=wl.ser, sigma_eps=sig, mu_q=wl.mu_q, sigma_q=wl.sigma_q, phi_kind=wl.phi_kind,
                               tau_rise=wl.tau_rise, tau_decay=wl.tau_decay, t0_min=wl.t0_min, t0_max=wl.t0_max)
        t = time.perf_counter()
        o = oracle.run(p, b["wave"], b["offsets"], b["lam"], 1, n_steps, burn, 7, kz, kmax=km,
                       n_threads=int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count())
        so = oracle.summarize(o.acc, n_steps, burn, 1)
        print(f"[precision] sigma_eps={sig}: oracle {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
        wave = torch.from_numpy(b["wave"]).cuda()
        for prec in (fsmp.FSMP_FP64, fsmp.FSMP_FP32_REFRESH):
            smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                               t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=sig, mu_q=wl.mu_q, sigma_q=wl.sigma_q,
                               n_steps=n_steps, n_chains=1, burn_in=burn, seed=7, device=0, precision=prec,
                               refresh_M=refresh_M, record_flags=fsmp.FSMP_REC_LOG)
            out = smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, work=True)
            post = smp.posterior(n_wave, out)
            torch.cuda.synchronize()
            logs = fsmp.log_records(out["log"])
            mean = post["mean"].cpu().numpy()
            work = out["work"].cpu().numpy()

            def one(c):
                w = b["wave"][b["offsets"][c]:b["offsets"][c + 1]]
                d, _, bad = oracle.replay(p, w, b["lam"][c], int(km[c]), 0, 4 * len(w) - 1, c, 7, logs[c],
                                          tie_eps=1e-9, ext=True)
                # the oracle's own FP64 (two nu's from scratch) along the same path
                d64, _, _ = oracle.replay(p, w, b["lam"][c], int(km[c]), 0, 4 * len(w) - 1, c, 7, logs[c],
                                          tie_eps=1e-9, ext=False)
                v = (logs[c]["flags"] & 1) != 0
                den = np.maximum(np.abs(d[v]), 1.0)
                return np.abs(logs[c]["dnu"][v] - d[v]) / den, bad, np.abs(d64[v] - d[v]) / den
            with concurrent.futures.ThreadPoolExecutor(max_workers=16) as ex:
                rep = list(ex.map(one, range(n_wave)))
            e = np.concatenate([r[0] for r in rep])
            caps = np.asarray(synth.KCAPS)[np.searchsorted(synth.KCAPS, km)]
            by_cap = {int(k): float(np.concatenate([rep[c][0] for c in range(n_wave) if caps[c] == k] +
                                                   [np.zeros(1)]).max()) for k in sorted(set(caps.tolist()))}
            row = {"sigma_eps": sig, "form": "fp64" if prec == fsmp.FSMP_FP64 else f"fp32+refresh M={refresh_M}",
                   "proposals": int(e.size), "dnu_rel_err_max": float(e.max()), "dnu_rel_err_p99": float(np.quantile(e, 0.99)),
                   "dnu_rel_err_median": float(np.median(e)), "dnu_rel_err_max_by_capacity": by_cap,
                   "oracle_fp64_dnu_rel_err_max": float(np.concatenate([r[2] for r in rep]).max()),
                   "oracle_fp64_dnu_rel_err_p99": float(np.quantile(np.concatenate([r[2] for r in rep]), 0.99)),
                   "decision_flips": int(sum(r[1] for r in rep)),
                   "chains_identical": float((out["z"].cpu().numpy() == o.z).all(1).mean()),
                   "fp64_reevaluations_per_proposal": float(work[:, 4].sum() / max(e.size, 1))}
            for a, name in enumerate(("N", "Q", "t0")):
                ref = so[name][0]
                r = np.abs(mean[:, a] - ref) / np.maximum(np.abs(ref), 1.0)
                row[f"mean_{name}_rel_err_max"] = float(r.max())
                row[f"mean_{name}_rel_err_median"] = float(np.median(r))
            rows.append(row)
            print(f"[precision] {json.dumps(row)}", file=sys.stderr, flush=True)
            smp.close()
    return rows


def main():
    args = parse()
    if args.hw_queues > 0:
        # before anything starts the HIP runtime; the library sizes its lanes from the same variable
        os.environ["GPU_MAX_HW_QUEUES"] = str(args.hw_queues)
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the sampler has no cross-GPU path: waveforms are independent)", file=sys.stderr)
        sys.exit(2)
    import torch

    import oracle
    from paper_2403_03156_amd import fsmp, synth

    if args.pmc_summary:
        pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.workload)
        return
    if args.issue_summary:
        issue_summary(args.issue_summary[0], args.issue_summary[1], args.workload, args.step_ms)
        return
    if args.trace_summary:
        trace_summary(args.trace_summary[0], int(args.trace_summary[1]), args.workload)
        return
    if args.serve:
        res = serving_study(fsmp, synth, [float(r) for r in args.serve_rates.split(",")], args.serve_events)
        print(json.dumps({"serving": res}), flush=True)
        return
    if args.precision_study:
        print(json.dumps({"precision_study": precision_study(fsmp, synth, oracle, args.precision_study)}), flush=True)
        return

    wl = synth.PRESETS[args.workload]
    n_wave = args.n_wave or wl.n_wave
    tuned = wl.name == "uneven" and not args.chain_steps
    n_steps = 4000 if tuned else (args.chain_steps or wl.n_steps)
    burn = n_steps // 2
    t_gen = time.time()
    b = synth.generate(wl, n_wave=n_wave, seed=wl.seed)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[bench] generated {n_wave} waveforms in {time.time() - t_gen:.1f}s; kmax buckets "
          f"{dict(zip(*np.unique(km, return_counts=True)))}", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    wave = torch.from_numpy(b["wave"]).to(dev)
    stream = torch.cuda.current_stream(dev)

    def sampler(precision=fsmp.FSMP_FP64, refresh_M=None, chains=wl.n_chains):
        if refresh_M is None:
            refresh_M = args.refresh if args.refresh >= 0 else fsmp.Sampler.default_refresh(precision)
        return fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                            t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                            sigma_q=wl.sigma_q, n_steps=n_steps, n_chains=chains, burn_in=burn, seed=wl.seed,
                            device=0, precision=precision, refresh_M=refresh_M)

    smp = sampler()
    steps, designs = None, None
    if tuned:
        # set-up, outside the timed region: the sweeps per waveform from a pilot run, then the
        # kernel design per PE capacity for those sweeps
        t_tune = time.time()
        steps = smp.autotune_steps(wave, b["offsets"], b["lam"], kmax=km, pilot_steps=200,
                                   target_rel_mcse=args.target_mcse, min_steps=500, max_steps=4000)
        designs = smp.autotune(wave, b["offsets"], b["lam"], kmax=km, trial_steps=args.trial_steps, n_steps=steps)
        torch.cuda.synchronize()
        print(f"[bench] autotuned in {time.time() - t_tune:.1f}s: designs {designs}; sweeps min {steps.min()} "
              f"median {int(np.median(steps))} mean {steps.mean():.0f} max {steps.max()}", file=sys.stderr, flush=True)
    chain_sweeps = float(steps.sum()) * wl.n_chains if tuned else float(n_wave) * wl.n_chains * n_steps
    out = smp.alloc_samples(n_wave, kz, work=True)

    def one_step(s=smp, o=out):
        s.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, out=o, stream=stream, n_steps=steps)
        return s.posterior(n_wave, o, with_pn=True, stream=stream)

    if args.pmc_run:
        # counter run: a plain copy of known size (the scale for FETCH_SIZE / WRITE_SIZE), then
        # one step; nothing is timed
        x = torch.empty(COPY_PROBE_MIB * 2 ** 20 // 4, dtype=torch.float32, device=dev).fill_(1.0)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y
        one_step()
        torch.cuda.synchronize()
        print("[bench] counter run done", file=sys.stderr, flush=True)
        return

    alone = serial_kernel_ms(smp, one_step)
    ms_per_step, kernel_ms = timed_steps(smp, one_step, args.steps, args.warmup)
    print("[bench] timed steps done", file=sys.stderr, flush=True)
    wps = n_wave / (ms_per_step / 1e3)
    sps = chain_sweeps / (ms_per_step / 1e3)

    # ---- roofline of the chain launch with the longest time in the step
    work = out["work"].cpu().numpy()
    caps = np.asarray(synth.KCAPS)
    chain_kcap = np.repeat(caps[np.searchsorted(caps, km)], wl.n_chains)
    avg = {name: float(np.mean([t["ms"] for t in ts])) for name, ts in kernel_ms.items()}
    chains_of = {name: ts[0]["kcap"] for name, ts in kernel_ms.items() if ts[0]["kcap"] > 0}
    dom = max(chains_of, key=lambda k: avg[k])
    wsel = work[chain_kcap == chains_of[dom]]
    nbytes = algorithmic_bytes(wsel)
    achieved = nbytes / (avg[dom] / 1e3)
    lds_r, lds_w = lds_peak()
    roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                "frac": achieved / PEAK_HBM, "traffic": recorded_traffic(args.workload, dom), "kernel": dom,
                "kernel_ms": avg[dom], "bytes_per_launch": nbytes,
                "lds": {"peak_read_measured_GBps": lds_r / 1e9, "peak_write_measured_GBps": lds_w / 1e9,
                        "frac_of_read_peak": achieved / lds_r,
                        "peak_nominal_GBps": 256 * 128 * CLOCK_HZ / 1e9},
                "impl_bytes_per_launch": 8.0 * (wsel[:, 2].sum() + wsel[:, 3].sum()),
                # the counters' HBM bytes of every kernel of the step (while the kernel source is the
                # one they were taken with) over the step's time: the whole step against HBM
                "step_traffic": step_traffic(args.workload, list(avg), ms_per_step),
                # every chain launch: its time in the step, the algorithmic bytes (packed factor) and
                # the G^-1 / G elements the implementation reads and writes, per launch
                "by_kernel": {name: {"ms": avg[name],
                                     "alg_bytes": algorithmic_bytes(work[chain_kcap == chains_of[name]]),
                                     "impl_bytes": 8.0 * float(work[chain_kcap == chains_of[name]][:, 2:4].sum())}
                              for name in sorted(chains_of, key=lambda k: -avg[k])}}
    # the same kernel with the chip to itself (the step's launches one after another, one
    # untimed step before the timed ones): over the concurrent duration above, a launch's
    # fraction falls as more launches share the chip
    if dom in alone:
        roofline["alone"] = {"kernel_ms": alone[dom], "achieved": nbytes / (alone[dom] / 1e3) / 1e9,
                             "frac": nbytes / (alone[dom] / 1e3) / PEAK_HBM,
                             "by_kernel_ms": {k: alone[k] for k in sorted(chains_of, key=lambda k: -avg[k]) if k in alone}}
    print(f"[bench] kernels (mean ms): {json.dumps(avg)}; alone: {json.dumps(alone)}", file=sys.stderr, flush=True)
    res = {
        "metric": "waveforms/s and MCMC steps/s at matched posterior accuracy; p99 event latency",
        "value": wps,
        "unit": "waveforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": (f"{wl.name}: {n_wave} waveforms x {wl.lengths} samples, lambda {wl.lam_dist}"
                                f"[{wl.lam_lo}, {wl.lam_hi}], {wl.n_chains} chain(s) x "
                                + (f"autotuned {int(steps.min())}-{int(steps.max())} sweeps (mean {steps.mean():.0f})"
                                   if tuned else f"{n_steps} sweeps") + ", FP64"),
                   "n_wave": n_wave, "chains": wl.n_chains,
                   "sweeps_mean": chain_sweeps / (n_wave * wl.n_chains), "parallelism": "single GPU"},
        "mcmc_steps_per_s": sps,
        "kernel_ms": avg,
        "roofline": roofline,
    }

    # ---- the FP32+refresh form on the same batch and sweeps: one timed step per refresh_M
    legs = set(x for x in args.legs.split(",") if x)
    if "fp32" in legs:
        fp32 = []
        for M in (16, 64, 256):
            s32 = sampler(fsmp.FSMP_FP32_REFRESH, M)
            o32 = s32.alloc_samples(n_wave, kz, work=True)
            ms32, _ = timed_steps(s32, lambda: one_step(s32, o32), 1, 1)
            w32 = o32["work"].cpu().numpy()
            fp32.append({"refresh_M": M, "ms_per_step": ms32, "waveforms_per_s": n_wave / (ms32 / 1e3),
                         "fp64_reevaluations_per_sweep": float(w32[:, 4].sum() / chain_sweeps)})
            s32.close()
            print(f"[bench] fp32 refresh_M={M}: {ms32:.1f} ms", file=sys.stderr, flush=True)
        res["fp32_refresh"] = fp32

    # ---- the batched workload (100,000 x 1,024 samples, 4 chains x 1,000 sweeps): one timed step
    if "batched" in legs and wl.name != "batched":
        bw = synth.PRESETS["batched"]
        bb = synth.generate(bw, seed=bw.seed)
        bkm = synth.kmax_for(bb["lam"])
        bwave = torch.from_numpy(bb["wave"]).to(dev)
        bs = fsmp.Sampler(ser=bw.ser, phi_kind=bw.phi_kind, tau_rise=bw.tau_rise, tau_decay=bw.tau_decay,
                          t0_min=bw.t0_min, t0_max=bw.t0_max, sigma_eps=bw.sigma_eps, mu_q=bw.mu_q,
                          sigma_q=bw.sigma_q, n_steps=bw.n_steps, n_chains=bw.n_chains, burn_in=bw.n_steps // 2,
                          seed=bw.seed, device=0)
        bo = bs.alloc_samples(bw.n_wave, int(bkm.max()))

        def bstep():
            bs.sample(bwave, bb["offsets"], bb["lam"], kmax=bkm, kz=int(bkm.max()), out=bo, stream=stream)
            return bs.posterior(bw.n_wave, bo, with_pn=True, stream=stream)
        bms, _ = timed_steps(bs, bstep, 2, 1)
        res["batched"] = {"workload": "batched: 100000 waveforms x 1024 samples, lambda loguniform[0.1, 30], "
                                      "4 chains x 1000 sweeps, FP64",
                          "ms_per_step": bms, "waveforms_per_s": bw.n_wave / (bms / 1e3),
                          "mcmc_steps_per_s": bw.n_wave * bw.n_chains * bw.n_steps / (bms / 1e3)}
        bs.close()
        del bwave
        print(f"[bench] batched: {bms:.1f} ms per step", file=sys.stderr, flush=True)

    # ---- the initialisation stage: Lucy-Richardson deconvolution of every waveform (fsmp_lucy),
    # timed with events on the stream it runs on; algorithmic flops = the two sums of each
    # iteration, 2 (L_w L_V + (L_w + L_V - 1) L_V) per waveform
    if "lucy" in legs and args.lucy_iter > 0:
        LV = smp.support_samples()
        smp.lucy(wave, b["offsets"], kmax=km, kz=kz, n_iter=args.lucy_iter, stream=stream)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lres = smp.lucy(wave, b["offsets"], kmax=km, kz=kz, n_iter=args.lucy_iter, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        lms = e0.elapsed_time(e1)
        L = np.diff(b["offsets"]).astype(np.float64)
        lflops = 2.0 * args.lucy_iter * float((L * LV + (L + LV - 1) * LV).sum())
        lach = lflops / (lms / 1e3)
        res["init_stage"] = {"iterations": args.lucy_iter, "ms": lms, "waveforms_per_s": n_wave / (lms / 1e3),
                             "initial_pes": int(lres["n_pe"].sum()),
                             "roofline": {"bound": "alu", "achieved": lach / 1e12, "peak": PEAK_FP64 / 1e12,
                                          "unit": "TFLOP/s", "frac": lach / PEAK_FP64, "traffic": None,
                                          "kernel": "lucy_kernel", "flops_per_launch": lflops}}
        print(f"[bench] lucy {args.lucy_iter} iterations: {lms:.1f} ms", file=sys.stderr, flush=True)

    # ---- the MCP-PMT charge law (the paper's five-Gaussian table) on the same batch and sweeps
    if "mcp" in legs and not args.no_mcp:
        mix = ([0.041, 0.516, 0.187, 0.195, 0.061], [0.92, 1.98, 3.01, 4.70, 6.79], [0.22, 0.48, 0.80, 1.30, 2.04])
        msmp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                            t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                            sigma_q=wl.sigma_q, n_steps=n_steps, n_chains=wl.n_chains, burn_in=burn, seed=wl.seed,
                            device=0, mix=mix)
        mout = msmp.alloc_samples(n_wave, kz)
        mms, _ = timed_steps(msmp, lambda: one_step(msmp, mout), 1, 1)
        res["mcp_charge_law"] = {"components": len(mix[0]), "ms_per_step": mms, "waveforms_per_s": n_wave / (mms / 1e3),
                                 "mcmc_steps_per_s": chain_sweeps / (mms / 1e3)}
        msmp.close()
        print(f"[bench] mcp mixture law: {mms:.1f} ms per step", file=sys.stderr, flush=True)

    # ---- oracle on a bounded sample of the same workload (first cpu_wave waveforms, same chains
    # and sweeps)
    if not args.no_cpu:
        m = min(args.cpu_wave, n_wave)
        off = b["offsets"][: m + 1]
        p = oracle.make_params(ser=wl.ser, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q,
                               phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                               t0_min=wl.t0_min, t0_max=wl.t0_max)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        tc = time.perf_counter()
        o = oracle.run(p, b["wave"][: off[-1]], off, b["lam"][:m], wl.n_chains, n_steps, burn, wl.seed, kz,
                       kmax=km[:m], n_threads=threads, wsteps=None if steps is None else steps[:m])
        dt = time.perf_counter() - tc
        # the sampled chains are the chains the GPU ran: they must agree exactly
        same = (out["z"][: m * wl.n_chains].cpu().numpy() == o.z).all(1).mean()
        sweeps = float(steps[:m].sum()) * wl.n_chains if tuned else float(m) * wl.n_chains * n_steps
        res["cpu_baseline"] = {"value": m / dt, "unit": "waveforms/s", "cores": threads, "kind": "oracle",
                               "cpu": cpu_model(),
                               "sample": f"first {m} of the {n_wave} waveforms, {wl.n_chains} chain(s), the same "
                                         f"sweeps ({sweeps / (m * wl.n_chains):.0f} mean), {dt:.1f}s; "
                                         f"{same * 100:.2f}% of its chains identical to the GPU's",
                               "steps_per_s": sweeps / dt}
        print(f"[bench] oracle {m} waveforms in {dt:.1f}s on {threads} threads", file=sys.stderr, flush=True)
    else:
        res["cpu_baseline"] = None

    # ---- serving: continuous batching over trigger rates, FP64 and FP32+refresh forms
    if not args.no_serve:
        res["serving"] = serving_study(fsmp, synth, [float(r) for r in args.serve_rates.split(",")],
                                       args.serve_events)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
