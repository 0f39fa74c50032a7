"""Benchmark of the FSMP hot path on one MI355X.

One step = one pass of the whole path over one batch: fsmp_sample (prologue +
chain kernels: every chain's Gibbs / RJMCMC sweeps) and fsmp_posterior, over the
batched workload (100,000 waveforms x 1,024 samples, lambda ~ logU[0.1, 30],
rise 2 / decay 25 ns light curve, 4 chains x 1,000 sweeps, FP64), with the
waveforms already resident in device memory when the timed region starts.

Prints one JSON line: waveforms/s (whole job) plus MCMC steps/s, the roofline
of the dominant kernel (measured with HIP events on its stream inside the timed
region) and the oracle timed on the host cores over a bounded sample.

    python bench.py [--gpus 1] [--steps 3] [--warmup 1] [--workload batched]

Roofline of a chain kernel whose state lives in device memory (one lane per chain, or
lane groups with G^-1 in device memory): algorithmic bytes = the G^-1 elements the
sweeps must touch, 8 bytes (4 in the FP32 form) per element read by a K x K mat-vec and
per element read and written by a rank-one or rank-two edit, summed from the device work
counters of the launch's chains, over the launch's mean duration, against 8 TB/s.  The
dominant kernel is the chain launch with the most such bytes.  Lane-group kernels with
G^-1 in LDS are reported against the FP64 vector peak with the same work counted as
flops.  `traffic` is the HBM bytes per launch that rocprofv3 counters recorded for that
kernel (FETCH_SIZE + WRITE_SIZE, scaled by the factor a plain copy of known size gives),
read from profiles/traffic_<workload>.json while the kernel source is unchanged:

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
    ap.add_argument("--workload", default="batched")
    ap.add_argument("--n-wave", type=int, default=0, help="override the workload's waveform count")
    ap.add_argument("--chain-steps", type=int, default=0, help="override the sweeps per chain")
    ap.add_argument("--cpu-wave", type=int, default=15000, help="waveforms in the oracle's timed sample")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--serve", action="store_true", help="only the serving study (rates x precisions)")
    ap.add_argument("--serve-events", type=int, default=40, help="events per serving run")
    ap.add_argument("--serve-rates", default="2000", help="comma-separated event rates (Hz)")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--lucy-iter", type=int, default=2000, help="Lucy-Richardson iterations of the init stage (0: skip)")
    ap.add_argument("--no-mcp", action="store_true", help="skip the MCP-PMT mixture-law leg")
    ap.add_argument("--pmc-run", action="store_true",
                    help="one untimed step after a plain device copy of known size (for rocprofv3 --pmc)")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="summarise two rocprofv3 --pmc runs into profiles/")
    ap.add_argument("--issue-summary", nargs=2, metavar=("SQ_DIR_A", "SQ_DIR_B"),
                    help="summarise two rocprofv3 --pmc runs of SQ counters into profiles/")
    ap.add_argument("--step-ms", type=float, default=0.0, help="concurrent step time for --issue-summary")
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
    m = re.search(r"chain_lane_kernel<(\d+), (double|float)>", name)
    if m:
        return ("chain_lane_k" if m.group(2) == "double" else "chain_lane_fp32_k") + m.group(1)
    for k in ("prologue_kernel", "posterior_kernel"):
        if k in name:
            return k.replace("_kernel", "")
    return None


def source_hash():
    return hashlib.sha256(open(KSRC, "rb").read()).hexdigest()


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
        out = {}
        for (_, name), kib in rows.items():
            lab = kernel_label(name)
            if lab is None and ("copy" in name.lower() or "elementwise" in name.lower()):
                lab = "copy"
            if lab:
                out.setdefault(lab, []).append(kib * 1024.0)
        return out

    fk, wk = by_kernel(fetch), by_kernel(write)
    # the copy probe is the largest copy-like dispatch: it reads and writes copy_bytes
    f_scale = copy_bytes / max(fk.get("copy", [copy_bytes]))
    w_scale = copy_bytes / max(wk.get("copy", [copy_bytes]))
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
        agg, dur = {}, {}
        for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            for r in csv.DictReader(open(f)):
                lab = kernel_label(r["Kernel_Name"])
                if lab is None:
                    continue
                agg.setdefault(lab, {})
                agg[lab][r["Counter_Name"]] = agg[lab].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
                dur[(lab, r["Dispatch_Id"])] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-9
        t = {}
        for (lab, _), v in dur.items():
            t[lab] = t.get(lab, 0.0) + v
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


def recorded_traffic(workload, kernel):
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    t = json.load(open(path))
    if t.get("source_sha256") != source_hash() or kernel not in t.get("kernels", {}):
        return None
    return t["kernels"][kernel]["hbm_bytes"]


def serving_run(fsmp, synth, pool, rate, n_events, precision, seed=0, n_streams=4, max_batch_wave=20000):
    """Poisson arrivals of trigger events (500-2000 channels drawn from a pool of synthetic
    channels, 1,024 samples each); returns latency percentiles and throughput."""
    wl = synth.PRESETS["serving"]
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
    l = np.array(list(lat.values()))
    return {"rate_hz": rate, "events": n_events, "waveforms": waves, "precision": "fp32+refresh" if precision else "fp64",
            "p50_ms": float(np.percentile(l, 50) * 1e3), "p99_ms": float(np.percentile(l, 99) * 1e3),
            "mean_ms": float(l.mean() * 1e3), "waveforms_per_s": waves / t_end,
            "offered_waveforms_per_s": waves / max(arrive[-1], 1e-9)}


def serving_pool(synth, n=20000, seed=5):
    wl = synth.PRESETS["serving"]
    b = synth.generate(wl, n_wave=n, seed=seed)
    return {"n": n, "wave": b["wave"], "lam": b["lam"], "kmax": synth.kmax_for(b["lam"])}


def algorithmic_flops(work):
    """FP64 flops of the PE-space linear algebra: 2K^2 per K x K mat-vec, 2K^2 per rank-one
    edit of the symmetric inverse Gram matrix, 4K^2 per rank-two edit."""
    return 2.0 * work[:, 0].sum() + 2.0 * work[:, 1].sum() + 4.0 * work[:, 2].sum()


def algorithmic_bytes(work, word):
    """device-memory bytes of G^-1 the sweeps must move: K^2 elements read per mat-vec,
    K^2 read and K^2 written per rank-one or rank-two edit"""
    return word * (work[:, 0].sum() + 2.0 * work[:, 1].sum() + 2.0 * work[:, 2].sum())


def main():
    args = parse()
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

    if args.serve:
        pool = serving_pool(synth)
        for prec in (fsmp.FSMP_FP64, fsmp.FSMP_FP32_REFRESH):
            for rate in [float(r) for r in args.serve_rates.split(",")]:
                r = serving_run(fsmp, synth, pool, rate, args.serve_events, prec)
                print(json.dumps({"serving": r}), flush=True)
        return

    wl = synth.PRESETS[args.workload]
    n_wave = args.n_wave or wl.n_wave
    n_steps = args.chain_steps or wl.n_steps
    burn = n_steps // 2
    t_gen = time.time()
    b = synth.generate(wl, n_wave=n_wave, seed=wl.seed)
    km = synth.kmax_for(b["lam"])
    kz = int(km.max())
    print(f"[bench] generated {n_wave} waveforms in {time.time() - t_gen:.1f}s; kmax buckets "
          f"{dict(zip(*np.unique(km, return_counts=True)))}", file=sys.stderr, flush=True)

    dev = torch.device("cuda", 0)
    wave = torch.from_numpy(b["wave"]).to(dev)
    smp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                       t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q,
                       n_steps=n_steps, n_chains=wl.n_chains, burn_in=burn, seed=wl.seed, device=0)
    out = smp.alloc_samples(n_wave, kz, work=True)
    stream = torch.cuda.current_stream(dev)

    def one_step():
        smp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, out=out, stream=stream)
        return smp.posterior(n_wave, out, with_pn=False, stream=stream)

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

    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    print("[bench] warmup done", file=sys.stderr, flush=True)

    smp.set_timing(True)
    kernel_ms = {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        post = one_step()
        for t in smp.last_timings():  # waits for this step's kernels (events on the same stream)
            kernel_ms.setdefault(t["name"], []).append(t)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    smp.set_timing(False)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    chain_steps = n_wave * wl.n_chains * n_steps
    wps = n_wave / (ms_per_step / 1e3)
    sps = chain_steps / (ms_per_step / 1e3)

    # ---- dominant kernel roofline: the chain launch with the most algorithmic bytes
    work = out["work"].cpu().numpy()
    caps = np.asarray(synth.KCAPS)
    chain_kcap = np.repeat(caps[np.searchsorted(caps, km)], wl.n_chains)
    avg = {name: float(np.mean([t["ms"] for t in ts])) for name, ts in kernel_ms.items()}
    per = {}
    for name, ts in kernel_ms.items():
        if ts[0]["kcap"] > 0:
            wsel = work[chain_kcap == ts[0]["kcap"]]
            per[name] = (algorithmic_bytes(wsel, 4.0 if "fp32" in name else 8.0), algorithmic_flops(wsel))
    dom = max(per, key=lambda k: per[k][0])
    nbytes, flops = per[dom]
    if dom.startswith("chain_group_k"):  # G^-1 in LDS: no device-memory state traffic
        achieved = flops / (avg[dom] / 1e3)
        roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                    "frac": achieved / PEAK_FP64, "traffic": recorded_traffic(args.workload, dom), "kernel": dom,
                    "kernel_ms": avg[dom], "flops_per_launch": flops}
    else:
        achieved = nbytes / (avg[dom] / 1e3)
        roofline = {"bound": "hbm", "achieved": achieved / 1e9, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
                    "frac": achieved / PEAK_HBM, "traffic": recorded_traffic(args.workload, dom), "kernel": dom,
                    "kernel_ms": avg[dom], "bytes_per_launch": nbytes}
    print(f"[bench] kernels (mean ms): {json.dumps(avg)}", file=sys.stderr, flush=True)

    # ---- the initialisation stage: Lucy-Richardson deconvolution of every waveform (fsmp_lucy),
    # timed with events on the stream it runs on; algorithmic flops = the two sums of each
    # iteration, 2 (L_w L_V + (L_w + L_V - 1) L_V) per waveform
    lucy = None
    if args.lucy_iter > 0:
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
        lucy = {"iterations": args.lucy_iter, "ms": lms, "waveforms_per_s": n_wave / (lms / 1e3),
                "initial_pes": int(lres["n_pe"].sum()),
                "roofline": {"bound": "alu", "achieved": lach / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                             "frac": lach / PEAK_FP64, "traffic": None, "kernel": "lucy_kernel",
                             "flops_per_launch": lflops}}
        print(f"[bench] lucy {args.lucy_iter} iterations: {lms:.1f} ms", file=sys.stderr, flush=True)

    # ---- the MCP-PMT charge law (the paper's five-Gaussian table) on the same batch: one
    # timed step of sample + posterior after a warm-up, HIP events around the step on the stream
    mcp = None
    if not args.no_mcp:
        mix = ([0.041, 0.516, 0.187, 0.195, 0.061], [0.92, 1.98, 3.01, 4.70, 6.79], [0.22, 0.48, 0.80, 1.30, 2.04])
        msmp = fsmp.Sampler(ser=wl.ser, phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                            t0_min=wl.t0_min, t0_max=wl.t0_max, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q,
                            sigma_q=wl.sigma_q, n_steps=n_steps, n_chains=wl.n_chains, burn_in=burn, seed=wl.seed,
                            device=0, mix=mix)
        mout = msmp.alloc_samples(n_wave, kz)
        msmp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, out=mout, stream=stream)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        msmp.sample(wave, b["offsets"], b["lam"], kmax=km, kz=kz, out=mout, stream=stream)
        msmp.posterior(n_wave, mout, with_pn=False, stream=stream)
        e1.record(stream)
        torch.cuda.synchronize()
        mms = e0.elapsed_time(e1)
        mcp = {"components": len(mix[0]), "ms_per_step": mms, "waveforms_per_s": n_wave / (mms / 1e3),
               "mcmc_steps_per_s": chain_steps / (mms / 1e3)}
        msmp.close()
        print(f"[bench] mcp mixture law: {mms:.1f} ms per step", file=sys.stderr, flush=True)

    # ---- oracle on a bounded sample of the same workload (first cpu_wave waveforms, same chains)
    cpu = None
    if not args.no_cpu:
        m = min(args.cpu_wave, n_wave)
        off = b["offsets"][: m + 1]
        p = oracle.make_params(ser=wl.ser, sigma_eps=wl.sigma_eps, mu_q=wl.mu_q, sigma_q=wl.sigma_q,
                               phi_kind=wl.phi_kind, tau_rise=wl.tau_rise, tau_decay=wl.tau_decay,
                               t0_min=wl.t0_min, t0_max=wl.t0_max)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
        tc = time.perf_counter()
        o = oracle.run(p, b["wave"][: off[-1]], off, b["lam"][:m], wl.n_chains, n_steps, burn, wl.seed, kz,
                       kmax=km[:m], n_threads=threads)
        dt = time.perf_counter() - tc
        # the sampled chains are the same chains the GPU ran: they must agree exactly
        same = (out["z"][: m * wl.n_chains].cpu().numpy() == o.z).all(1).mean()
        cpu = {"value": m / dt, "unit": "waveforms/s", "cores": threads, "kind": "oracle",
               "sample": f"first {m} of the {n_wave} waveforms, {wl.n_chains} chains x {n_steps} sweeps, "
                         f"{dt:.1f}s; {same * 100:.2f}% of its chains identical to the GPU's",
               "steps_per_s": m * wl.n_chains * n_steps / dt}
        print(f"[bench] oracle {m} waveforms in {dt:.1f}s on {threads} threads", file=sys.stderr, flush=True)

    # ---- serving: continuous batching at 2 kHz trigger rate, FP64 and FP32+refresh forms
    serving = None
    if not args.no_serve:
        pool = serving_pool(synth)
        serving = [serving_run(fsmp, synth, pool, float(r), args.serve_events, prec)
                   for prec in (fsmp.FSMP_FP64, fsmp.FSMP_FP32_REFRESH) for r in args.serve_rates.split(",")]
        print(f"[bench] serving {json.dumps(serving)}", file=sys.stderr, flush=True)

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
        "config": {"workload": f"{wl.name}: {n_wave} waveforms x {wl.lengths} samples, lambda {wl.lam_dist}"
                               f"[{wl.lam_lo}, {wl.lam_hi}], {wl.n_chains} chains x {n_steps} sweeps, FP64",
                   "n_wave": n_wave, "chains": wl.n_chains, "sweeps": n_steps, "parallelism": "single GPU"},
        "mcmc_steps_per_s": sps,
        "kernel_ms": avg,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "serving": serving,
        "init_stage": lucy,
        "mcp_charge_law": mcp,
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
