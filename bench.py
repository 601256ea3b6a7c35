#!/usr/bin/env python3
"""Throughput of the sFFT4.0 hot path on one MI355X.

Workload (default): a batch of 512 synthetic signals of length N = 2^22,
each exactly K = 1000 sparse (support uniform without replacement, magnitude
1, uniform phase; Sec. 4.1 setup), complex64 in HBM.  One plan for the batch:
B = 2048 buckets, w = 45057 taps, 12 iterations, (l, q) = (16, 1),
delta = 1e-6, plan seed 602; signal i uses seed 601 + i.

Layout (default): position-major, sample c of signal s at X[c, s], so that
every tap of the gather reads one contiguous row segment of the batch;
--layout per-signal keeps one buffer per signal (the layout of uneven
batches), and the other layout is timed beside the main one for context.

A step is one pass of the whole hot path over the batch: the fold stage
(permuted gather + window + fold for every round of every iteration), the
bucket DFTs, and the recovery stage (subtraction, detection, location,
estimation, accumulation, top-K).  The timed steps launch the three stages
one by one with HIP events between them (the per-stage times come from
those events); the graph replay that sfft_execute_batch uses is timed
separately as graph_ms_per_step.

Prints one JSON line on stdout; progress goes to stderr.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "signals/s and HBM GB/s (gather-fold), N=2^22 K=1000, vs dense FFT, rel-L2≤1e-4"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def make_batch(torch, n, N, K, snr, dtype, dev, seed0):
    """Planted K-sparse spectra from the seeded generator; time signals by an
    inverse DFT on the device (input synthesis only), stored in `dtype`."""
    from paper_2011_05698_amd.signals import planted_spectrum

    if dtype == "f16x2":
        X = torch.empty((n, N, 2), dtype=torch.float16, device=dev)
    else:
        X = torch.empty((n, N), dtype=torch.complex64 if dtype == "c64" else torch.complex128, device=dev)
    scales = []
    gen = torch.Generator(device=dev)
    for i in range(n):
        sup, vals = planted_spectrum(N, K, seed0 + i)
        xh = torch.zeros(N, dtype=torch.complex128, device=dev)
        xh[torch.from_numpy(sup).to(dev)] = torch.from_numpy(vals).to(dev)
        x = torch.fft.ifft(xh) * N
        if snr is not None:
            gen.manual_seed(seed0 + i + 0x5EED)
            s2 = float((x.abs() ** 2).sum()) / N * 10.0 ** (-snr / 10.0)
            noise = torch.randn(N, dtype=torch.complex128, device=dev, generator=gen)  # unit variance
            x = x + noise * math.sqrt(s2)
        if dtype == "f16x2":
            s = float(torch.maximum(x.real.abs().max(), x.imag.abs().max()))
            X[i, :, 0] = (x.real / s).to(torch.float16)
            X[i, :, 1] = (x.imag / s).to(torch.float16)
            scales.append(s)
        else:
            X[i] = x.to(X.dtype)
            scales.append(1.0)
    return X, scales


FOLD_SOURCES = ("fold.hip", "fold_body.h", "device_common.h", "internal.h", "plan.cpp")


def measured_traffic(workload_tag):
    """HBM bytes per fold launch from the committed rocprofv3 summary of this
    workload and layout, if the fold kernel and its launch order are the ones
    the counters were taken with (else None)."""
    import hashlib

    path = os.path.join(ROOT, "profiles", f"fold_kernel_hbm_bytes_{workload_tag}.txt")
    if not os.path.exists(path):
        return None, None
    vals = {}
    for line in open(path):
        if line.startswith("#") or " " not in line:
            continue
        k, v = line.split(None, 1)
        vals[k] = v.strip()
    # the kernel (fold.hip, fold_body.h and the helpers and layout they use)
    # and the order its tiles are launched in (plan.cpp)
    csrc = os.path.join(ROOT, "paper_2011_05698_amd", "csrc")
    src = b"".join(open(os.path.join(csrc, f), "rb").read() for f in FOLD_SOURCES)
    if vals.get("fold_sources_sha256_16") != hashlib.sha256(src).hexdigest()[:16]:
        return None, "fold kernel or its launch order changed since the counters were taken"
    # the launch shape moves no bytes (every shape gathers the same samples), so
    # counters taken at another unroll or cap still price this launch
    # position-major: one fold launch per step; per-signal: the union-tile and
    # one-round launches of one step together
    nbytes = vals.get("fold_hbm_bytes_per_launch", vals.get("fold_hbm_bytes_per_step"))
    if nbytes is None:
        return None, f"{os.path.relpath(path, ROOT)} holds no fold byte count"
    return int(float(nbytes)), os.path.relpath(path, ROOT)


def experiments(torch, sfft, dev):
    """The parameter experiments of Sec. 4.2 on the GPU path (none of the
    comparison systems).  Signals as in Sec. 4.1: K = 50 unit tones, complex
    white noise at the given SNR.

    fig5: phase error of the two-round phase difference (Eq. 15-17) in
      buckets that hold one tone, at the four (N, L) of Fig. 5 and SNR from
      -20 to 120 dB.  The error is the circular distance between
      arg(yhat_0 conj yhat_1) of the GPU bucket values and the tone's own
      phase 2 pi (tau_1 u mod N) / N.  Quantiles of log10 of the error.
    fig6: time per signal vs N (2^14..2^22) for l in {4, 8, 16, 32} at q = 1,
      and q in {1/4, 1/2, 1, 2, 4} at l = 16, at 20 dB (the general sparse
      case).  Signals run in position-major batches of 256; plus the fraction
      of the signal sampled (the method's own curve of Fig. 9).
    fig7: L1 error vs SNR at N = 2^16 for the same (l, q): the mean over 64
      signals of (1/K) sum |xhat_f - xhat'_f| over the planted and recovered
      frequencies (noise not counted).
    Plans: B = 2^ceil(log2 2K) = 128, w = B log2 N, loops = ceil(log2 K) + 2.
    l = 2 with q = 1 is not run: the region would not shrink."""
    import numpy as np
    from paper_2011_05698_amd.signals import planted_spectrum

    K = 50
    out = {"fig5": [], "fig6": [], "fig7": []}
    for N, L in ((8192, 32), (131072, 2048), (1048576, 2048), (4194304, 8192)):
        B = N // L
        plan = sfft.Plan(N, K, B, (B * int(math.log2(N))) | 1, 1, 16, 1.0, delta=1e-6, seed=51)
        it = plan.iteration(0)
        D, tau1, sig = it["L"] // 2 + it["e"], it["tau"][1], it["sigma"]
        for snr in (-20, -10, 0, 20, 40, 60, 120):
            nsig = 24
            X, _ = make_batch(torch, nsig, N, K, snr, "c64", dev, 5000 + N % 997 + 31 * snr)
            errs = []
            for s_ in range(nsig):
                y = plan.hash_to_bins(X[s_]).cpu().numpy().astype(np.complex128)
                sup, _ = planted_spectrum(N, K, 5000 + N % 997 + 31 * snr + s_)
                us = (sig * sup) % N
                for u in us.tolist():
                    i = int(round(u / L)) % B
                    d = np.abs(((us - i * L) + N // 2) % N - N // 2)
                    if np.count_nonzero(d <= D) != 1:
                        continue  # another tone reaches this bucket
                    th = np.angle(y[i] * np.conj(y[B + i]))
                    ref = 2 * math.pi * ((tau1 * u) % N) / N
                    errs.append(abs((th - ref + math.pi) % (2 * math.pi) - math.pi))
            e = np.log10(np.maximum(np.array(errs), 1e-300))
            out["fig5"].append({"N": N, "L": L, "snr_db": snr, "buckets": len(errs),
                                "log10_err_p01": round(float(np.quantile(e, 0.01)), 3),
                                "log10_err_p50": round(float(np.quantile(e, 0.5)), 3),
                                "log10_err_p99": round(float(np.quantile(e, 0.99)), 3)})
            log(f"[fig5] N={N} L={L} snr={snr}: {out['fig5'][-1]}")
    grid = [(l, 1.0) for l in (4, 8, 16, 32)] + [(16, q) for q in (0.25, 0.5, 2.0, 4.0)]
    B, loops = 128, int(math.ceil(math.log2(K))) + 2

    def l1_error(idx, val, cnt, seeds, N):
        errs = []
        for s_, sd in enumerate(seeds):
            sup, vals = planted_spectrum(N, K, sd)
            c = int(cnt[s_].item())
            got = dict(zip(idx[s_, :c].cpu().numpy().tolist(), val[s_, :c].cpu().numpy().astype(np.complex128)))
            want = dict(zip(sup.tolist(), vals))
            errs.append(sum(abs(got.get(f, 0) - want.get(f, 0)) for f in set(got) | set(want)) / K)
        return float(np.mean(errs))

    for logN in (14, 16, 18, 20, 22):
        N, nsig = 1 << logN, 256
        X, _ = make_batch(torch, nsig, N, K, 20.0, "c64", dev, 7000 + logN)
        XT = X.transpose(0, 1).contiguous()
        del X
        for l, q in grid:
            plan = sfft.Plan(N, K, B, (B * logN) | 1, loops, l, q, delta=1e-6, seed=61)
            b = sfft.InterleavedBatch(plan, nsig)
            o = b.outputs(dev)
            for _ in range(2):
                b.execute(XT, outs=o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(5):
                b.execute(XT, outs=o)
            torch.cuda.synchronize()
            us = (time.perf_counter() - t0) / (5 * nsig) * 1e6
            out["fig6"].append({"N": N, "l": l, "q": q, "us_per_signal": round(us, 3),
                                "sampled_fraction": round(plan.samples / N, 5),
                                "l1_error_20db": round(l1_error(*o, range(7000 + logN, 7000 + logN + nsig), N), 6)})
            b.close()
            log(f"[fig6] {out['fig6'][-1]}")
        del XT
    N = 1 << 16
    for snr in (-10, 0, 10, 20, 30, 40, 60):
        X, _ = make_batch(torch, 64, N, K, float(snr), "c64", dev, 9000 + snr)
        XT = X.transpose(0, 1).contiguous()
        for l, q in grid:
            plan = sfft.Plan(N, K, B, (B * 16) | 1, loops, l, q, delta=1e-6, seed=71)
            b = sfft.InterleavedBatch(plan, 64)
            o = b.execute(XT)
            torch.cuda.synchronize()
            out["fig7"].append({"snr_db": snr, "l": l, "q": q,
                                "l1_error": round(l1_error(*o, range(9000 + snr, 9064 + snr), N), 6)})
            b.close()
        log(f"[fig7] snr={snr}: " + ", ".join(f"({r['l']},{r['q']}) {r['l1_error']}" for r in out["fig7"][-len(grid):]))
    return out


def host_cpu():
    """CPU model and logical CPU count of this host (lscpu fields)."""
    info = {"logical_cpus": os.cpu_count()}
    try:
        import subprocess

        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            k, _, v = ln.partition(":")
            if k.strip() in ("Model name", "CPU(s)", "Thread(s) per core", "Core(s) per socket", "Socket(s)"):
                info[k.strip()] = v.strip()
    except Exception as exc:  # lscpu missing: keep the count alone
        info["lscpu"] = f"unavailable ({exc.__class__.__name__})"
    return info


class one_thread:
    """Limits the BLAS and OpenMP thread pools of this process to one thread
    while the oracle is timed; yields the pools seen (library, threads)."""

    def __enter__(self):
        try:
            from threadpoolctl import threadpool_info, threadpool_limits
        except ImportError:
            self.ctl = None
            return [{"threadpoolctl": "unavailable"}]
        self.ctl = threadpool_limits(limits=1)
        return [{"library": p.get("internal_api"), "threads": p.get("num_threads")} for p in threadpool_info()]

    def __exit__(self, *exc):
        if self.ctl is not None:
            self.ctl.restore_original_limits()
        return False


def host_copy(torch, X, i, dtype, scale):
    import numpy as np

    if dtype == "f16x2":
        h = X[i].float().cpu().numpy().astype(np.float64)
        return (h[:, 0] + 1j * h[:, 1]) * scale
    return X[i].cpu().numpy().astype(np.complex128)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--N", type=int, default=2 ** 22)
    ap.add_argument("--K", type=int, default=1000)
    ap.add_argument("--B", type=int, default=2048)
    ap.add_argument("--loops", type=int, default=12)
    ap.add_argument("--snr", type=float, default=None, help="SNR in dB (default: noiseless)")
    ap.add_argument("--dtype", default="c64", choices=["c64", "f16x2", "c128"])
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default fold launch shape")
    ap.add_argument("--layout", default="position-major", choices=["position-major", "per-signal"],
                    help="batch storage: sample c of signal s at X[c, s] (one plan), or one buffer per signal")
    ap.add_argument("--no-context", action="store_true", help="skip timing the other layout")
    ap.add_argument("--no-forms", action="store_true", help="skip the FP16 and uneven-batch context lines")
    ap.add_argument("--large-oracle", type=int, default=0, metavar="SIGNALS",
                    help="with --large-form: run the FP64 oracle on this many of its signals (about a minute each)")
    ap.add_argument("--large-form", type=int, default=0, metavar="SIGNALS",
                    help="also time the N=2^27, K=8192, B=16384 FP16 workload on this many signals")
    ap.add_argument("--fold-config", default=None, metavar="U,CAP",
                    help="fold launch shape (taps per thread, workgroups per CU cap) instead of tuning")
    ap.add_argument("--experiments", action="store_true",
                    help="run the parameter experiments of Sec. 4.2 (Fig. 5-7) instead; prints their JSON")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB a few times (scales HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the sparse FFT hot path is built and measured on a single "
              "MI355X (signals of a batch are independent: several GPUs would each take a slice of the batch).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = args.copy_calibration * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": args.copy_calibration, "launches": 5,
                          "expected_fetch_kib": n * 4 / 1024, "expected_write_kib": n * 4 / 1024}))
        return

    from paper_2011_05698_amd import sfft

    dev = torch.device("cuda:0")
    if args.experiments:
        print(json.dumps(experiments(torch, sfft, dev)))
        return
    N, K, B, M, n = args.N, args.K, args.B, args.loops, args.batch
    logN = int(math.log2(N))
    w = (B * logN) | 1
    l, q, delta, plan_seed, sig_seed = 16, 1.0, 1e-6, 602, 601
    dt = args.dtype

    log(f"generating {n} signals N=2^{logN} K={K} dtype={dt} snr={args.snr}")
    t0 = time.perf_counter()
    X, scales = make_batch(torch, n, N, K, args.snr, dt, dev, sig_seed)
    torch.cuda.synchronize()
    log(f"signals ready in {time.perf_counter() - t0:.1f}s")

    t0 = time.perf_counter()
    plan = sfft.Plan(N, K, B, w, M, l, q, delta=delta, seed=plan_seed, dtype=dt)
    log(f"plan built in {time.perf_counter() - t0:.1f}s (samples/signal {plan.samples})")
    stream = torch.cuda.current_stream()
    XT = None
    if args.layout == "position-major" or not args.no_context:
        # sample c of signal s at XT[c, s]: one transpose of the batch (synthesis, untimed)
        XT = X.transpose(0, 1).contiguous()
        torch.cuda.synchronize()

    def time_batch(batch, run, steps, tag, position_major):
        """Bind, tune, warm up and time `steps` passes of a bound batch."""
        run()  # binds buffers, builds the graph
        torch.cuda.synchronize()
        fold_cfg = None
        if args.fold_config:
            u, cap = (int(v) for v in args.fold_config.split(","))
            cap = 0 if position_major else cap
            batch.set_fold_config(u, cap)
            fold_cfg = {"unroll": u, "wg_per_cu": cap, "fold_ms": None}
        elif not args.no_autotune:
            t1 = time.perf_counter()
            fold_cfg = batch.autotune()
            log(f"[{tag}] fold autotune: {fold_cfg} in {time.perf_counter() - t1:.1f}s")
        run()  # captures with the chosen launch shape
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        tuning = batch.tuning()
        fused = tuning["mode"] == "fused"
        # timed region: the chosen configuration, launch by launch with events
        # between the stages (the fused mode is one launch per step)
        ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            if fused:
                batch.launch_stage(3)
                for i in (1, 2, 3):
                    ev[k][i].record(stream)
                continue
            batch.launch_stage(0)
            ev[k][1].record(stream)
            batch.launch_stage(1)
            ev[k][2].record(stream)
            batch.launch_stage(2)
            ev[k][3].record(stream)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t1
        stage_ms = [float(np.mean([ev[k][i].elapsed_time(ev[k][i + 1]) for k in range(steps)])) for i in range(3)]
        # graph replay of the same work (the execute path)
        torch.cuda.synchronize()
        tg = time.perf_counter()
        for _ in range(steps):
            run()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - tg) * 1e3 / steps
        # spread of single graph replays (events on the launch stream), at
        # least 20 of them
        reps = max(20, steps)
        evg = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for e0, e1 in evg:
            e0.record(stream)
            run()
            e1.record(stream)
        torch.cuda.synchronize()
        gms = np.array([e0.elapsed_time(e1) for e0, e1 in evg])
        graph_spread = {"replays": reps, "median_ms": round(float(np.median(gms)), 4),
                        "p10_ms": round(float(np.quantile(gms, 0.1)), 4), "p90_ms": round(float(np.quantile(gms, 0.9)), 4)}
        nsig = len(batch.plans)
        res = {"value": nsig * steps / elapsed, "ms_per_step": elapsed * 1e3 / steps,
               "stage_ms": stage_ms, "graph_ms_per_step": graph_ms, "graph_replay_spread": graph_spread,
               "fold_cfg": fold_cfg, "tuning": tuning}
        if tuning["fused_available"]:  # the other mode, for context
            other = "stages" if fused else "fused"
            batch.set_tuning(mode=other)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            fn = (lambda: [batch.launch_stage(i) for i in (0, 1, 2)]) if other == "stages" else (lambda: batch.launch_stage(3))
            fn()
            e0.record(stream)
            for _ in range(3):
                fn()
            e1.record(stream)
            torch.cuda.synchronize()
            res["other_mode"] = {"mode": other, "ms_per_step": round(e0.elapsed_time(e1) / 3, 4),
                                 "fused_chunk": batch.tuning()["fused_chunk"]}
            batch.set_tuning(mode=tuning["mode"])
        log(f"[{tag}] timed {steps} steps: {res['ms_per_step']:.3f} ms/step, {res['value']:.1f} signals/s; "
            f"stages ms {[round(v, 4) for v in stage_ms]}; graph {graph_ms:.3f} ms/step")
        return res

    def run_layout(layout, steps):
        """The metric batch in one layout: bind, tune, warm up, time."""
        if layout == "position-major":
            batch = sfft.InterleavedBatch(plan, n)
            outs = batch.outputs(dev)
            run = lambda: batch.execute(XT, scales=scales, outs=outs)  # noqa: E731
        else:
            batch = sfft.Batch([plan] * n)
            outs = batch.outputs(dev)
            xs = [X[i] for i in range(n)]
            run = lambda: batch.execute(xs, scales=scales, outs=outs)  # noqa: E731
        res = time_batch(batch, run, steps, layout, layout == "position-major")
        res["layout"] = layout
        res["outs"] = outs
        batch.close()
        return res

    def precision_form(steps):
        """The same signals stored as FP16 (re, im) pairs with a per-signal FP32
        scale (max |re|, |im|), position-major; window and sums in FP32."""
        X16 = torch.empty((N, n, 2), dtype=torch.float16, device=dev)
        sc16 = []
        for c0 in range(0, n, 64):
            xc = X[c0:c0 + 64]
            sc = torch.maximum(xc.real.abs().amax(1), xc.imag.abs().amax(1))
            h = torch.stack([xc.real / sc[:, None], xc.imag / sc[:, None]], -1).to(torch.float16)
            X16[:, c0:c0 + 64] = h.transpose(0, 1)
            sc16 += [float(v) for v in sc.cpu()]
            del xc, h
        torch.cuda.synchronize()
        plan16 = sfft.Plan(N, K, B, w, M, l, q, delta=delta, seed=plan_seed, dtype="f16x2")
        b16 = sfft.InterleavedBatch(plan16, n)
        outs16 = b16.outputs(dev)
        r = time_batch(b16, lambda: b16.execute(X16, scales=sc16, outs=outs16), steps, "precision f16x2", True)
        b16.close()
        alg = n * (plan16.samples * 4 + plan16.yhat_elems * 8)
        line = {"storage": "f16 pairs + per-signal f32 scale", "layout": "position-major",
                "signals_per_s": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                             "recover": round(r["stage_ms"][2], 4)},
                "fold_alg_gbs": round(alg / (r["stage_ms"][0] * 1e-3) / 1e9, 1),
                "fold_alg_frac": round(alg / (r["stage_ms"][0] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "fold_launch": r["fold_cfg"]}
        return line, (X16, sc16, outs16)

    def batching_form(steps):
        """512 signals of uneven N, K and SNR, one plan each, one buffer each:
        N = 2^U{16..22}, K log-uniform on [10, 2000], SNR uniform on [10, 40] dB;
        B = 2^ceil(log2 2K) capped at N/32 (so that w = B log2 N | 1 < N),
        K capped at B/2, loops = ceil(log2 K) + 2, (l, q) = (16, 1);
        seeds 401 + i (signal draws) and 402 + i (plan)."""
        from paper_2011_05698_amd.signals import planted_spectrum

        from concurrent.futures import ThreadPoolExecutor

        nb = n
        xs_b, spec = [], []
        for i in range(nb):
            g = np.random.default_rng(401 + i)
            ln = int(g.integers(16, 23))
            Ni = 1 << ln
            Ki = int(round(math.exp(g.uniform(math.log(10), math.log(2000)))))
            snr = float(g.uniform(10, 40))
            Bi = min(1 << math.ceil(math.log2(2 * Ki)), Ni // 32)
            Ki = min(Ki, Bi // 2)
            Mi = math.ceil(math.log2(Ki)) + 2
            spec.append((Ni, Ki, Bi, (Bi * ln) | 1, Mi, snr))
        t1 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=16) as ex:  # plan synthesis is host work; the C calls drop the GIL
            plans_b = list(ex.map(lambda i: sfft.Plan(*spec[i][:5], l, q, delta=delta, seed=402 + i), range(nb)))
        log(f"[batching uneven] {nb} plans built in {time.perf_counter() - t1:.1f}s")
        gen = torch.Generator(device=dev)
        for i in range(nb):
            Ni, Ki, Bi, wi, Mi, snr = spec[i]
            sup, vals = planted_spectrum(Ni, Ki, 401 + i)
            xh = torch.zeros(Ni, dtype=torch.complex128, device=dev)
            xh[torch.from_numpy(sup).to(dev)] = torch.from_numpy(vals).to(dev)
            x = torch.fft.ifft(xh) * Ni
            gen.manual_seed(401 + i + 0x5EED)
            s2 = float((x.abs() ** 2).sum()) / Ni * 10.0 ** (-snr / 10.0)
            x = x + torch.randn(Ni, dtype=torch.complex128, device=dev, generator=gen) * math.sqrt(s2)
            xs_b.append(x.to(torch.complex64))
        torch.cuda.synchronize()
        bb = sfft.Batch(plans_b)
        outs_b = bb.outputs(dev)
        r = time_batch(bb, lambda: bb.execute(xs_b, outs=outs_b), steps, "batching uneven", False)
        bb.close()
        samples = sum(p.samples for p in plans_b)
        alg = samples * 8 + sum(p.yhat_elems for p in plans_b) * 8
        line = {"signals": nb, "N": "2^16..2^22", "K": "10..2000", "snr_db": "10..40", "layout": "per-signal",
                "signals_per_s": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                             "recover": round(r["stage_ms"][2], 4)},
                "graph_ms_per_step": round(r["graph_ms_per_step"], 4),
                "fold_alg_gbs": round(alg / (r["stage_ms"][0] * 1e-3) / 1e9, 1),
                "fold_launch": r["fold_cfg"], "tuning": r["tuning"], "other_mode": r.get("other_mode")}
        return line, (xs_b, spec, outs_b)

    def large_form(nl, steps):
        """The large reduced-precision workload: N = 2^27, K = 8192, magnitudes
        log-uniform on [1e-2, 1], 40 dB, B = 16384, w = 16384 * 27 + 1, 15
        iterations, FP16 pairs with a per-signal scale (position-major, one
        plan); compared with the planted support and with the FP32 path on the
        same signals (seeds 501 + i / plan 502)."""
        from paper_2011_05698_amd.signals import planted_spectrum

        NL, KL, BL, ML = 2 ** 27, 8192, 16384, 15
        wl = (BL * 27) | 1
        X32 = torch.empty((NL, nl), dtype=torch.complex64, device=dev)
        X16 = torch.empty((NL, nl, 2), dtype=torch.float16, device=dev)
        sc, sups = [], []
        gen = torch.Generator(device=dev)
        for i in range(nl):
            sup, vals = planted_spectrum(NL, KL, 501 + i, mags="loguniform")
            xh = torch.zeros(NL, dtype=torch.complex128, device=dev)
            xh[torch.from_numpy(sup).to(dev)] = torch.from_numpy(vals).to(dev)
            x = torch.fft.ifft(xh) * NL
            del xh
            gen.manual_seed(501 + i + 0x5EED)
            s2 = float((x.abs() ** 2).sum()) / NL * 10.0 ** (-40 / 10.0)
            x = x + torch.randn(NL, dtype=torch.complex128, device=dev, generator=gen) * math.sqrt(s2)
            X32[:, i] = x.to(torch.complex64)
            m = float(torch.maximum(x.real.abs().max(), x.imag.abs().max()))
            X16[:, i, 0] = (x.real / m).to(torch.float16)
            X16[:, i, 1] = (x.imag / m).to(torch.float16)
            sc.append(m)
            sups.append(sup)
            del x
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        p16 = sfft.Plan(NL, KL, BL, wl, ML, l, q, delta=delta, seed=502, dtype="f16x2")
        p32 = sfft.Plan(NL, KL, BL, wl, ML, l, q, delta=delta, seed=502)
        log(f"[large f16x2] plans built in {time.perf_counter() - t1:.1f}s")
        b16 = sfft.InterleavedBatch(p16, nl)
        o16 = b16.outputs(dev)
        r = time_batch(b16, lambda: b16.execute(X16, scales=sc, outs=o16), steps, "large f16x2", True)
        b16.close()
        b32 = sfft.InterleavedBatch(p32, nl)
        o32 = b32.execute(X32)
        torch.cuda.synchronize()
        b32.close()
        recall16, recall32, agree, worst = [], [], [], 0.0
        for i in range(nl):
            c16, c32 = int(o16[2][i].item()), int(o32[2][i].item())
            g16, g32 = o16[0][i, :c16].cpu().numpy(), o32[0][i, :c32].cpu().numpy()
            v16 = o16[1][i, :c16].cpu().numpy().astype(np.complex128)
            v32 = o32[1][i, :c32].cpu().numpy().astype(np.complex128)
            recall16.append(len(np.intersect1d(g16, sups[i])) / KL)
            recall32.append(len(np.intersect1d(g32, sups[i])) / KL)
            common, a16, a32 = np.intersect1d(g16, g32, return_indices=True)
            agree.append(len(common) / max(len(g32), 1))
            worst = max(worst, float(np.linalg.norm(v16[a16] - v32[a32]) / max(np.linalg.norm(v32[a32]), 1e-300)))
        # recall by magnitude decade: what the method finds of the planted
        # coefficients of each size (log-uniform on [1e-2, 1])
        by_mag = {}
        for lo, hi in ((1e-2, 1e-1), (1e-1, 1.0)):
            hit = tot = 0
            for i in range(nl):
                sup, vals = planted_spectrum(NL, KL, 501 + i, mags="loguniform")
                sel = sup[(np.abs(vals) >= lo) & (np.abs(vals) < hi)]
                c16 = int(o16[2][i].item())
                hit += len(np.intersect1d(o16[0][i, :c16].cpu().numpy(), sel))
                tot += len(sel)
            by_mag[f"[{lo:g}, {hi:g})"] = round(hit / max(tot, 1), 4)
        oracle_cmp = None
        if args.large_oracle:
            from fractions import Fraction

            from oracle import sfft_oracle as O

            PL = O.make_plan(NL, KL, BL, wl, ML, l, Fraction(q), delta, seed=502)
            oracle_cmp = []
            for i in range(min(args.large_oracle, nl)):
                row = {"signal": i}
                h = X16[:, i].float().cpu().numpy().astype(np.float64)
                for tag, xin, outs_ in (("f16", (h[:, 0] + 1j * h[:, 1]) * sc[i], o16),
                                        ("f32", X32[:, i].cpu().numpy().astype(np.complex128), o32)):
                    t1 = time.perf_counter()
                    oi, ov, _ = O.sfft(xin, PL)
                    c = int(outs_[2][i].item())
                    gi = outs_[0][i, :c].cpu().numpy()
                    gv = outs_[1][i, :c].cpu().numpy().astype(np.complex128)
                    common, ga, oa = np.intersect1d(gi, oi, return_indices=True)
                    pc = np.abs(gv[ga] - ov[oa]) / np.maximum(np.abs(ov[oa]), 1e-300)
                    row[tag] = {"oracle_s": round(time.perf_counter() - t1, 1), "gpu_count": c, "oracle_count": len(oi),
                                "support_identical": bool(np.array_equal(gi, oi)),
                                "support_agreement": round(len(common) / max(len(oi), len(gi), 1), 5),
                                "rel_l2_common": float(np.linalg.norm(gv[ga] - ov[oa]) /
                                                       max(np.linalg.norm(ov[oa]), 1e-300)),
                                "per_coefficient_rel_err": {"max": float(pc.max()) if len(pc) else 0.0,
                                                            "p99": float(np.quantile(pc, 0.99)) if len(pc) else 0.0,
                                                            "median": float(np.median(pc)) if len(pc) else 0.0}}
                    log(f"[large {tag}] oracle on signal {i}: {row[tag]}")
                oracle_cmp.append(row)
                del h
        alg = nl * (p16.samples * 4 + p16.yhat_elems * 8)
        return {"N": NL, "K": KL, "B": BL, "w": wl, "loops": ML, "signals": nl, "snr_db": 40,
                "recall_f16_by_magnitude": by_mag, "oracle": oracle_cmp,
                "mags": "log-uniform [1e-2, 1]", "storage": "f16 pairs + per-signal f32 scale",
                "signals_per_s": round(r["value"], 2), "ms_per_step": round(r["ms_per_step"], 3),
                "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                             "recover": round(r["stage_ms"][2], 4)},
                "fold_alg_gbs": round(alg / (r["stage_ms"][0] * 1e-3) / 1e9, 1),
                "recall_f16": round(float(np.mean(recall16)), 4), "recall_f32": round(float(np.mean(recall32)), 4),
                "support_agreement_f16_vs_f32": round(float(np.min(agree)), 4),
                "max_rel_l2_f16_vs_f32_common": worst}

    def direct_form(steps):
        """The same batch and plan parameters with the two-round direct location
        (sFFT3.0 reading: one step with tau = 1 instead of the multiscale
        schedule), position-major; recall against the planted supports."""
        from paper_2011_05698_amd.signals import planted_spectrum

        pdir = sfft.Plan(N, K, B, w, M, l, q, delta=delta, seed=plan_seed, location="direct")
        bd = sfft.InterleavedBatch(pdir, n)
        od = bd.outputs(dev)
        r = time_batch(bd, lambda: bd.execute(XT, scales=scales, outs=od), steps, "direct location", True)
        bd.close()
        rec = []
        for s_ in range(8):
            sup, _ = planted_spectrum(N, K, sig_seed + s_)
            c = int(od[2][s_].item())
            rec.append(len(np.intersect1d(od[0][s_, :c].cpu().numpy(), sup)) / K)
        return {"location": "two rounds, u = round(theta N / 2 pi)", "layout": "position-major",
                "samples_per_signal": pdir.samples, "signals_per_s": round(r["value"], 1),
                "ms_per_step": round(r["ms_per_step"], 4),
                "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                             "recover": round(r["stage_ms"][2], 4)},
                "recall_first_8": round(float(np.mean(rec)), 4),
                "note": "K/B = 0.49 here: two rounds cannot screen collisions as the multiscale rounds do"}

    def vote_form(steps):
        """The same batch and plan parameters with the vote over loops (every
        loop keeps B and w, nothing subtracted, kept when at least half of the
        loops located it, median over loops), position-major; recall against
        the planted supports."""
        from paper_2011_05698_amd.signals import planted_spectrum

        pv = sfft.Plan(N, K, B, w, M, l, q, delta=delta, seed=plan_seed, combine="vote")
        bv = sfft.InterleavedBatch(pv, n)
        ov = bv.outputs(dev)
        r = time_batch(bv, lambda: bv.execute(XT, scales=scales, outs=ov), steps, "vote over loops", True)
        bv.close()
        rec = []
        for s_ in range(8):
            sup, _ = planted_spectrum(N, K, sig_seed + s_)
            c = int(ov[2][s_].item())
            rec.append(len(np.intersect1d(ov[0][s_, :c].cpu().numpy(), sup)) / K)
        return ({"combine": "vote over loops: B and w in every loop, no subtraction, kept by >= half, median",
                 "layout": "position-major", "samples_per_signal": pv.samples,
                 "signals_per_s": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                 "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                              "recover": round(r["stage_ms"][2], 4)},
                 "recall_first_8": round(float(np.mean(rec)), 4),
                 "note": "a coefficient that collides in more than half of the loops is dropped"}, ov)

    def metric_variants(steps):
        """The metric workload at the other plan sizes the workload list names
        (B = 4096, and B = 16384 by the square-root rule; w = B log2 N | 1),
        with 20 dB of noise at B = 2048, and with the compensated (Kahan) fold,
        position-major, one plan each."""
        res, keep = {}, {}
        for tag, Bv, snr, kahan in (("B4096", 4096, None, False), ("B16384", 16384, None, False),
                                    ("snr20", B, 20.0, False), ("kahan", B, None, True)):
            wv = (Bv * logN) | 1
            if snr is None:
                Xv, XTv, scv = X, XT, scales
            else:
                Xn, scv = make_batch(torch, n, N, K, snr, dt, dev, sig_seed)
                XTv = Xn.transpose(0, 1).contiguous()
                Xv = None
                keep_x0 = [host_copy(torch, Xn, s_, dt, scv[s_]) for s_ in (0, 1)]
                del Xn
            pv = sfft.Plan(N, K, Bv, wv, M, l, q, delta=delta, seed=plan_seed, dtype=dt, kahan=kahan)
            bv = sfft.InterleavedBatch(pv, n)
            ov = bv.outputs(dev)
            r = time_batch(bv, lambda: bv.execute(XTv, scales=scv, outs=ov), steps, f"metric {tag}", True)
            bv.close()
            res[tag] = {"B": Bv, "w": wv, "snr_db": snr, "kahan": kahan, "layout": "position-major",
                        "samples_per_signal": pv.samples, "signals_per_s": round(r["value"], 1),
                        "ms_per_step": round(r["ms_per_step"], 4),
                        "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                                     "recover": round(r["stage_ms"][2], 4)},
                        "tuning_mode": r["tuning"]["mode"]}
            keep[tag] = (Bv, wv, snr, ov, keep_x0 if snr is not None else None)
            if snr is not None:
                del XTv
                torch.cuda.empty_cache()
        return res, keep

    def plain_form(reps):
        """One signal of the metric workload (signal 0, the same plan), as a
        caller with a single signal runs it: sfft_execute (fold, bucket DFT and
        recovery launched on the stream), and the same three stages replayed
        from a graph (a batch of one)."""
        x0 = X[0].contiguous() if dt != "f16x2" else X[0].contiguous().view(torch.float16)
        sc0 = scales[0]
        outs = plan.execute(x0, sc0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(3):
            plan.execute(x0, sc0)
        e0.record(stream)
        for _ in range(reps):
            sfft.sfft_execute(plan.handle, x0, sc0, outs[0], outs[1], outs[2])
        e1.record(stream)
        torch.cuda.synchronize()
        ms_exec = e0.elapsed_time(e1) / reps
        b1 = sfft.Batch([plan])
        o1 = b1.outputs(dev)
        for _ in range(3):
            b1.execute([x0], scales=[sc0], outs=o1)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(reps):
            b1.execute([x0], scales=[sc0], outs=o1)
        e1.record(stream)
        torch.cuda.synchronize()
        ms_graph = e0.elapsed_time(e1) / reps
        b1.close()
        log(f"[plain single signal] execute {ms_exec:.4f} ms, graph {ms_graph:.4f} ms")
        return {"signals": 1, "layout": "one buffer", "reps": reps,
                "execute_ms": round(ms_exec, 4), "execute_signals_per_s": round(1e3 / ms_exec, 1),
                "graph_ms": round(ms_graph, 4), "graph_signals_per_s": round(1e3 / ms_graph, 1),
                "note": "one signal keeps one workgroup busy through the twelve dependent iterations of "
                        "the recovery; the rest of the GPU idles"}

    def independent_plans_form(steps):
        """The metric batch with one plan per signal (plan seeds 602 + i, so
        every signal has its own draws of sigma and tau), one buffer per
        signal: the layout a batch of independently planned signals needs."""
        from concurrent.futures import ThreadPoolExecutor

        t1 = time.perf_counter()
        with ThreadPoolExecutor(max_workers=16) as ex:
            plans_i = list(ex.map(lambda i: sfft.Plan(N, K, B, w, M, l, q, delta=delta, seed=plan_seed + i,
                                                      dtype=dt), range(n)))
        log(f"[independent plans] {n} plans built in {time.perf_counter() - t1:.1f}s")
        bi = sfft.Batch(plans_i)
        oi_ = bi.outputs(dev)
        xs = [X[i] for i in range(n)]
        r = time_batch(bi, lambda: bi.execute(xs, scales=scales, outs=oi_), steps, "independent plans", False)
        bi.close()
        return {"plans": f"one per signal, seeds {plan_seed}..{plan_seed + n - 1}", "layout": "per-signal",
                "signals_per_s": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                             "recover": round(r["stage_ms"][2], 4)},
                "graph_ms_per_step": round(r["graph_ms_per_step"], 4), "fold_launch": r["fold_cfg"]}, (plans_i, oi_)

    main_res = run_layout(args.layout, args.steps)
    context = None
    if not args.no_context:
        other = "per-signal" if args.layout == "position-major" else "position-major"
        r = run_layout(other, max(2, args.steps // 2))
        context = {"layout": other, "signals_per_s": round(r["value"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                   "stage_ms": {"fold": round(r["stage_ms"][0], 4), "bucket_fft": round(r["stage_ms"][1], 4),
                                "recover": round(r["stage_ms"][2], 4)},
                   "fold_launch": r["fold_cfg"]}
    # ---- the two other forms of the method (context lines) ----
    forms, form_outs = {}, {}
    if not args.no_forms and dt == "c64":
        forms["precision"], form_outs["precision"] = precision_form(max(2, args.steps // 2))
        forms["batching"], form_outs["batching"] = batching_form(max(2, args.steps // 2))
    if not args.no_forms and dt == "c64":
        forms["direct_location"] = direct_form(max(2, args.steps // 2))
        forms["vote"], form_outs["vote"] = vote_form(max(2, args.steps // 2))
    if not args.no_forms and dt == "c64" and args.layout == "position-major":
        forms["metric_variants"], form_outs["metric_variants"] = metric_variants(max(2, args.steps // 2))
    if not args.no_forms:
        forms["plain"] = plain_form(20)
        forms["independent_plans"], form_outs["independent_plans"] = independent_plans_form(max(2, args.steps // 2))
    if args.large_form:
        forms["large_precision"] = large_form(args.large_form, max(2, args.steps // 2))

    K_steps = args.steps
    stage_ms, ms_per_step, value = main_res["stage_ms"], main_res["ms_per_step"], main_res["value"]
    graph_ms, fold_cfg, outs = main_res["graph_ms_per_step"], main_res["fold_cfg"], main_res["outs"]
    if XT is not None and args.layout != "position-major":
        del XT

    # ---- roofline of the gather-fold, the kernel whose HBM rate the metric
    # names; the longest stage is the recovery, bound by dependent latency
    # rather than by HBM or arithmetic (stage_roofline below) ----
    bytes_per_sample = {"c64": 8, "f16x2": 4, "c128": 16}[dt]
    out_bytes = 16 if dt == "c128" else 8
    alg_bytes = n * (plan.samples * bytes_per_sample + plan.yhat_elems * out_bytes)
    achieved = alg_bytes / (stage_ms[0] * 1e-3) / 1e9
    lay = "posmajor" if args.layout == "position-major" else "persignal"
    tag = f"metric_batch{n}_{dt}_{lay}" if (N, K, B, M, args.snr) == (2 ** 22, 1000, 2048, 12, None) else None
    traffic, source = measured_traffic(tag) if tag else (None, None)
    fold_kernel = ("fold_interleaved_kernel" if args.layout == "position-major"
                   else "fold_union_kernel + fold_kernel (the fold stage's two launches)")
    if main_res["tuning"]["mode"] == "fused":  # one kernel per step: price the whole step's gathers on it
        fold_kernel, traffic, source = "fused_kernel", None, "the fused launch: counters not taken"
    roofline = {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": traffic,
                "kernel": fold_kernel,
                "why_this_kernel": "the gather-fold, whose HBM rate the metric names; the longest stage "
                                   "(the recovery) is latency-bound, see stage_roofline",
                "alg_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(stage_ms[0], 5)}
    if traffic:
        roofline["traffic_gbs"] = round(traffic / (stage_ms[0] * 1e-3) / 1e9, 1)
        roofline["traffic_source"] = source
    elif source:
        roofline["traffic_note"] = source

    # ---- dense FFT of the same N on the same device (context) ----
    dense = None
    if not args.no_dense:
        chunk = min(n, 64)
        Xd = X[:chunk] if dt != "f16x2" else torch.view_as_complex(X[:chunk].float())
        Xd = Xd.to(torch.complex64)
        for _ in range(2):
            torch.fft.fft(Xd, dim=-1)
        torch.cuda.synchronize()
        td = time.perf_counter()
        reps = 5
        for _ in range(reps):
            torch.fft.fft(Xd, dim=-1)
        torch.cuda.synchronize()
        dense_s = (time.perf_counter() - td) / (reps * chunk)
        dense = {"impl": "torch.fft.fft (rocFFT), complex64", "signals_per_s": round(1.0 / dense_s, 1),
                 "speedup_of_sfft": round(value * dense_s, 3)}
        del Xd
        log(f"dense FFT: {1.0 / dense_s:.1f} signals/s")
        # the paper compares with a CPU FFT library: a dense FP64 FFT of the
        # same N on the host, on every core and on one
        try:
            import scipy.fft as sfft_cpu

            xc = host_copy(torch, X, 0, dt, scales[0])
            cpu_fft = {"impl": "scipy.fft.fft, complex128", "host_cpu": host_cpu(),
                       "note": "its workers split a batch of transforms; one transform of one signal runs on one core"}
            for label, workers in (("all_cores", os.cpu_count() or 1), ("one_core", 1)):
                sfft_cpu.fft(xc, workers=workers)
                t1 = time.perf_counter()
                for _ in range(3):
                    sfft_cpu.fft(xc, workers=workers)
                cpu_fft[label] = {"workers": workers, "signals_per_s": round(3 / (time.perf_counter() - t1), 2)}
            dense["cpu_fft"] = cpu_fft
            log(f"dense CPU FFT: {cpu_fft['all_cores']['signals_per_s']} signals/s on "
                f"{cpu_fft['all_cores']['workers']} workers, {cpu_fft['one_core']['signals_per_s']} on one")
        except ImportError:
            pass

    # ---- oracle on a bounded sample; parity of that sample ----
    cpu = None
    parity = None
    if not args.no_cpu_baseline:
        from fractions import Fraction

        from oracle import sfft_oracle as O

        P = O.make_plan(N, K, B, w, M, l, Fraction(q), delta, seed=plan_seed)
        idxs, vals, counts = outs
        cnt = counts.cpu().numpy()
        spent, done, same, worst, worst_pc, pcs = 0.0, 0, 0, 0.0, 0.0, []
        host = host_cpu()
        while done < n and (spent < args.cpu_seconds or done == 0):
            xh = host_copy(torch, X, done, dt, scales[done])
            with one_thread() as pools:
                t1 = time.perf_counter()
                oi, ov, _ = O.sfft(xh, P)
                spent += time.perf_counter() - t1
            c = int(cnt[done])
            gi = idxs[done][:c].cpu().numpy()
            gv = vals[done][:c].cpu().numpy().astype(np.complex128)
            if np.array_equal(gi, oi):
                same += 1
                worst = max(worst, float(np.linalg.norm(gv - ov) / max(np.linalg.norm(ov), 1e-300)))
                pc = np.abs(gv - ov) / np.maximum(np.abs(ov), 1e-300)
                worst_pc = max(worst_pc, float(pc.max()) if len(pc) else 0.0)
                pcs.append(pc)
            done += 1
        cpu = {"value": round(done / spent, 4), "unit": "signals/s", "cores": 1, "kind": "oracle",
               "sample": f"first {done} signals of the batch (same inputs), FP64 NumPy oracle, plan untimed",
               "threads": "one: BLAS/OpenMP pools limited to 1 thread while timed (threadpoolctl); "
                          "NumPy's FFT, sort and bincount are single-threaded",
               "thread_pools_during_timing": pools, "host_cpu": host}
        allpc = np.concatenate(pcs) if pcs else np.zeros(1)
        parity = {"signals_checked": done, "support_identical": same, "max_rel_l2_identical": worst,
                  "per_coefficient_rel_err": {"max": worst_pc, "p99": float(np.quantile(allpc, 0.99)),
                                              "median": float(np.median(allpc)), "coefficients": int(allpc.size)}}
        log(f"oracle: {done} signals in {spent:.1f}s; parity {same}/{done}, max rel-L2 {worst:.2e}")
        # the other forms, a few signals each (not timed)
        if "precision" in form_outs:
            X16, sc16, (i16, v16, c16) = form_outs["precision"]
            P16 = O.make_plan(N, K, B, w, M, l, Fraction(q), delta, seed=plan_seed)
            chk, same16, worst16 = 0, 0, 0.0
            for s_ in range(2):
                h = X16[:, s_].float().cpu().numpy().astype(np.float64)
                oi, ov, _ = O.sfft((h[:, 0] + 1j * h[:, 1]) * sc16[s_], P16)
                c = int(c16[s_].item())
                gi, gv = i16[s_, :c].cpu().numpy(), v16[s_, :c].cpu().numpy().astype(np.complex128)
                chk += 1
                if np.array_equal(gi, oi):
                    same16 += 1
                    worst16 = max(worst16, float(np.linalg.norm(gv - ov) / max(np.linalg.norm(ov), 1e-300)))
            forms["precision"]["parity"] = {"signals_checked": chk, "support_identical": same16,
                                            "max_rel_l2_identical": worst16,
                                            "oracle_input": "the dequantized FP16 samples"}
        if "batching" in form_outs:
            xs_b, spec, (ib, vb, cb) = form_outs["batching"]
            agree, worst_b = [], 0.0
            for s_ in range(4):
                Ni, Ki, Bi, wi, Mi, snr = spec[s_]
                Pb = O.make_plan(Ni, Ki, Bi, wi, Mi, l, Fraction(q), delta, seed=402 + s_)
                oi, ov, _ = O.sfft(xs_b[s_].cpu().numpy().astype(np.complex128), Pb)
                c = int(cb[s_].item())
                gi, gv = ib[s_][:c].cpu().numpy(), vb[s_][:c].cpu().numpy().astype(np.complex128)
                common, ga, oa = np.intersect1d(gi, oi, return_indices=True)
                agree.append(len(common) / max(len(oi), len(gi), 1))
                if len(common):
                    worst_b = max(worst_b, float(np.linalg.norm(gv[ga] - ov[oa]) / max(np.linalg.norm(ov[oa]), 1e-300)))
            forms["batching"]["parity"] = {"signals_checked": len(agree), "min_support_agreement": round(min(agree), 4),
                                           "max_rel_l2_common": worst_b,
                                           "note": "noisy inputs: decisions near the threshold may flip"}

        if "independent_plans" in form_outs:
            plans_i, (ii, vi, ci) = form_outs["independent_plans"]
            chk, samei, worsti, worsti_pc = 0, 0, 0.0, 0.0
            for s_ in (0, n - 1):
                Pi = O.make_plan(N, K, B, w, M, l, Fraction(q), delta, seed=plan_seed + s_)
                oi, ov_, _ = O.sfft(host_copy(torch, X, s_, dt, scales[s_]), Pi)
                c = int(ci[s_].item())
                gi, gv = ii[s_][:c].cpu().numpy(), vi[s_][:c].cpu().numpy().astype(np.complex128)
                chk += 1
                if np.array_equal(gi, oi):
                    samei += 1
                    worsti = max(worsti, float(np.linalg.norm(gv - ov_) / max(np.linalg.norm(ov_), 1e-300)))
                    worsti_pc = max(worsti_pc, float(np.max(np.abs(gv - ov_) / np.maximum(np.abs(ov_), 1e-300))))
            forms["independent_plans"]["parity"] = {"signals_checked": chk, "support_identical": samei,
                                                    "max_rel_l2_identical": worsti,
                                                    "max_per_coefficient_rel_err": worsti_pc}

        if "metric_variants" in form_outs:
            for tag, (Bv, wv, snr, (iv_, vv_, cv_), xs0) in form_outs["metric_variants"].items():
                Pm = O.make_plan(N, K, Bv, wv, M, l, Fraction(q), delta, seed=plan_seed)
                agree, worst_m, worst_pc = [], 0.0, 0.0
                for s_ in (0, 1):
                    xh = host_copy(torch, X, s_, dt, scales[s_]) if xs0 is None else xs0[s_]
                    oi, ov_, _ = O.sfft(xh, Pm)
                    c = int(cv_[s_].item())
                    gi, gv = iv_[s_, :c].cpu().numpy(), vv_[s_, :c].cpu().numpy().astype(np.complex128)
                    common, ga, oa = np.intersect1d(gi, oi, return_indices=True)
                    agree.append(len(common) / max(len(oi), len(gi), 1))
                    if len(common):
                        worst_m = max(worst_m, float(np.linalg.norm(gv[ga] - ov_[oa]) /
                                                     max(np.linalg.norm(ov_[oa]), 1e-300)))
                        worst_pc = max(worst_pc, float(np.max(np.abs(gv[ga] - ov_[oa]) /
                                                              np.maximum(np.abs(ov_[oa]), 1e-300))))
                forms["metric_variants"][tag]["parity"] = {
                    "signals_checked": len(agree), "min_support_agreement": round(min(agree), 4),
                    "max_rel_l2_common": worst_m, "max_per_coefficient_rel_err_common": worst_pc}

        if "vote" in form_outs:
            iv, vv, cv = form_outs["vote"]
            Pv = O.make_plan(N, K, B, w, M, l, Fraction(q), delta, seed=plan_seed, combine="vote")
            chk, samev, worstv = 0, 0, 0.0
            for s_ in range(2):
                oi, ov_, _ = O.sfft(XT[:, s_].cpu().numpy().astype(np.complex128), Pv)
                c = int(cv[s_].item())
                gi, gv = iv[s_, :c].cpu().numpy(), vv[s_, :c].cpu().numpy().astype(np.complex128)
                chk += 1
                if np.array_equal(gi, oi):
                    samev += 1
                    worstv = max(worstv, float(np.linalg.norm(gv - ov_) / max(np.linalg.norm(ov_), 1e-300)))
            forms["vote"]["parity"] = {"signals_checked": chk, "support_identical": samev,
                                       "max_rel_l2_identical": worstv}

    line = {
        "metric": METRIC, "value": round(value, 2), "unit": "signals/s", "n_gpus": 1, "steps": K_steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": {"c64": "f32", "f16x2": "f32", "c128": "f64"}[dt], "data": "synthetic",
        "config": {"workload": f"sFFT4.0 batch of {n} signals, N=2^{logN}, K={K}, B={B}, w={w}, loops={M}, "
                               f"l={l}, q={q}, delta={delta}, storage {dt}, "
                               f"{'noiseless' if args.snr is None else f'SNR {args.snr} dB'}",
                   "batch": n, "N": N, "K": K, "B": B, "w": w, "loops": M, "multiscale": l, "extension": q,
                   "storage": dt, "snr_db": args.snr, "samples_per_signal": plan.samples,
                   "layout": args.layout, "plan": "one plan (one sigma/tau draw) for the whole batch"},
        "roofline": roofline, "cpu_baseline": cpu, "parity": parity, "dense_fft": dense,
        "stage_ms": {"fold": round(stage_ms[0], 4), "bucket_fft": round(stage_ms[1], 4),
                     "recover": round(stage_ms[2], 4)},
        "graph_ms_per_step": round(graph_ms, 4),
        "graph_replay_spread": main_res["graph_replay_spread"],
        # the two other stages against HBM: bucket values read and written once
        # by the bucket DFT, read once by the recovery (its store and outputs
        # are smaller).  Neither reaches the HBM peak: the DFT is bound by the
        # load latency of its waves (load, in-register DFTs, store in sequence
        # at two waves per SIMD), the recovery by dependent latency (one
        # workgroup per signal, iterations in order).
        "stage_roofline": {
            st: {"bound": bound, "alg_bytes_per_launch": nb,
                 "achieved_gbs": round(nb / (ms * 1e-3) / 1e9, 1),
                 "frac_of_hbm_peak": round(nb / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            for st, bound, nb, ms in (
                ("bucket_fft", "latency", n * plan.yhat_elems * (16 if dt == "c128" else 8) * 2, stage_ms[1]),
                ("recover", "latency", n * plan.yhat_elems * (16 if dt == "c128" else 8), stage_ms[2]))},
        "fold_launch": fold_cfg,
        "tuning": main_res["tuning"], "other_mode": main_res.get("other_mode"),
        "other_layout": context,
        "forms": forms or None,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
