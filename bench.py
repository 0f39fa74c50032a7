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
"""
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
    return ap.parse_args()


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              f"(the sampler has no cross-GPU path: waveforms are independent)", file=sys.stderr)
        sys.exit(2)
    import torch

    import oracle
    from paper_2403_03156_amd import fsmp, synth

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

    # ---- dominant kernel roofline (algorithmic FP64 flops of its chains / its mean duration)
    work = out["work"].cpu().numpy()
    caps = np.asarray(synth.KCAPS)
    chain_kcap = np.repeat(caps[np.searchsorted(caps, km)], wl.n_chains)
    avg = {name: float(np.mean([t["ms"] for t in ts])) for name, ts in kernel_ms.items()}
    dom = max(avg, key=avg.get)
    dom_t = kernel_ms[dom][0]
    if dom_t["kcap"] > 0:
        flops = algorithmic_flops(work[chain_kcap == dom_t["kcap"]])
    else:
        flops = 0.0
    achieved = flops / (avg[dom] / 1e3)
    roofline = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64 / 1e12, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP64, "traffic": None, "kernel": dom, "kernel_ms": avg[dom],
                "flops_per_launch": flops}
    print(f"[bench] kernels (mean ms): {json.dumps(avg)}", file=sys.stderr, flush=True)

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
    }
    print(json.dumps(res))


if __name__ == "__main__":
    main()
