#!/usr/bin/env python3
"""Throughput of the ATSFFT hot path on one MI355X.

Workload: 1D complex64 signals of n = 2^22 with k = 64 planted frequencies
(magnitudes uniform in [0.5, 1], uniform phases) plus complex Gaussian noise
at 40 dB SNR; k is unknown to the transform and probed by the adaptive loop.
One step is one execute of the whole path (probe, location loops, vote,
estimation) over a batch of distinct signals already resident in HBM.

Printed as one JSON line: transforms/s, the same-GPU dense FFT (torch.fft,
rocFFT) on the same batch, the plain per-signal form, the L1 error of the
paper's error display against the full FFT and against the planted spectrum,
the roofline of the dominant kernel, and the FP64 CPU oracle timed on a
bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sparse transforms/sec and speedup vs same-GPU dense FFT at n=2^22,k=64; L1 error"
WORKLOAD = "c2_1d_c64_n4m_k64_snr40"
HBM_PEAK_GBS = 8000.0
PLAN_SEED = 2019


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def timed(fn, steps, stream):
    import torch

    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def oracle_params(desc, signal):
    import oracle

    return oracle.Params(
        ndim=desc.ndim, n=desc.n, B0=desc.B0, B_max=desc.B_max, alpha_probe=desc.alpha_probe,
        alpha=desc.alpha, L_loc=desc.L_loc, L_est=desc.L_est, T_vote=desc.T_vote, P_max=desc.P_max,
        d=desc.d, gamma=desc.gamma, delta=desc.delta, q=desc.q, noise_rate=desc.noise_rate, rho=desc.rho,
        seed=desc.seed, signal=signal, max_out=desc.max_out)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hash_main_c2_n4m_k64_b32_hbm_traffic.txt")
KERNEL_SRC = os.path.join(ROOT, "paper_1908_02461_amd", "csrc", "atsfft_kernels.hip")


def section_sha256(first, last):
    """SHA-256 of the kernel source from the divider titled `first` up to the
    one titled `last`."""
    import hashlib

    src = open(KERNEL_SRC).read()
    lines = src.splitlines(keepends=True)
    pos, a, b = 0, None, None
    for ln in lines:
        if ln.startswith("// ---") and ln.rstrip().endswith(" ----"):
            title = ln.rstrip()[:-5].lstrip("/ -")
            if title == first and a is None:
                a = pos
            elif title == last and a is not None:
                b = pos
                break
        pos += len(ln)
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def hash_kernel_sha256():
    """SHA-256 of the k_hash section of the kernel source."""
    return section_sha256("k_hash", "LDS FFT")


def hash_launch_sha256():
    """SHA-256 of the kernel-source lines that size the main-loop hash grid
    (its tile slots per address slab), which the traffic also depends on."""
    import hashlib

    src = open(KERNEL_SRC).read().splitlines(keepends=True)
    return hashlib.sha256("".join(ln for ln in src if "main_slots" in ln or "hash_blocks =" in ln).encode()).hexdigest()


def measured_traffic(batch, path=None, sha=None, key="k_hash_source_sha256"):
    """HBM bytes per launch from a committed counter summary (default: the 1D
    main-loop k_hash), if it was taken on the current source section and
    batch; otherwise None."""
    try:
        kv = {}
        with open(path or TRAFFIC_FILE) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get(key) != (sha or hash_kernel_sha256()) or int(kv.get("batch", -1)) != batch:
            return None
        if path is None and kv.get("k_hash_launch_sha256") != hash_launch_sha256():
            return None
        return float(kv["hbm_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        return None


MASK64 = (1 << 64) - 1


def _splitmix64_at(seed, index):
    """SplitMix64 output at a counter index (the library's draw generator)."""
    z = (seed + (index + 1) * 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _loop_lines(seed, sig, phase, it, n, w):
    """128-byte lines of c64 samples one 1D loop reads: x[(sigma t + tau) mod n],
    t in [-w/2, w/2), with (sigma, tau) drawn as the library documents."""
    r = _splitmix64_at(seed, ((sig * 4 + phase) * 256 + it) * 2)
    sigma, tau = (r % n) | 1, (r >> 32) % n
    t = np.arange(w, dtype=np.int64) - w // 2
    return ((sigma * t + tau) % n) >> 4


def touched_bytes(desc, trs):
    """Distinct 128-byte lines of the input (times 128) plus the bucket values
    written, per batch: for the main-loop hash launch, and for the whole step
    (probe levels the trace shows, plus the main loops)."""
    from paper_1908_02461_amd import atsfft as A

    n, L = desc.n, desc.L_loc + desc.L_est
    main = step = 0
    for s, t in enumerate(trs):
        if t["status"] & A.SIG_EMPTY:  # no main loops
            continue
        B = t["B_star"]
        w = min(desc.alpha * B, n)
        lines = [_loop_lines(desc.seed, s, 1 if l < desc.L_loc else 2,
                             l if l < desc.L_loc else l - desc.L_loc, n, w) for l in range(L)]
        u = np.unique(np.concatenate(lines))
        main += 128 * u.size + L * B * 8
        probe = [_loop_lines(desc.seed, s, 0, i, n, min(desc.alpha_probe * Bp, n))
                 for i, Bp in enumerate(t["probe_B"])]
        up = np.unique(np.concatenate([u] + probe))
        step += 128 * up.size + L * B * 8 + sum(Bp * 8 for Bp in t["probe_B"])
    return main, step


def cpu_model():
    """The host CPU's model name (from /proc/cpuinfo), or the platform's."""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform

    return platform.processor() or platform.machine()


def cpu_baseline(desc, xs, budget_s, min_signals=8):
    """The FP64 oracle, single-threaded, on the first signals of the batch
    (at least min_signals, then until the time budget is spent).  Returns the
    baseline record and the oracle's results, signal by signal."""
    import oracle

    done, t0, results = 0, time.perf_counter(), []
    while done < len(xs):
        results.append(oracle.atsfft(xs[done].astype(np.complex128), oracle_params(desc, done), trace=False))
        done += 1
        log(f"cpu baseline: {done} transform(s), {time.perf_counter() - t0:.1f} s")
        if done >= min_signals and time.perf_counter() - t0 >= budget_s:
            break
    el = time.perf_counter() - t0
    rec = {"value": done / el, "unit": "transforms/s", "cores": 1, "kind": "oracle",
           "sample": f"{done} full-size transforms (n=2^22, c64 input upcast to FP64), one thread, {el:.1f} s",
           "cpu_model": cpu_model(), "nproc": os.cpu_count()}
    return rec, results


def oracle_agreement(res, refs, floor=1e-2):
    """GPU results against the oracle's on the same signals: the located sets'
    symmetric difference (summed and per signal) and the largest relative value
    error, with the denominator max(|X_oracle(f)|, floor max_g |X_oracle(g)|) on
    the frequencies both located (floor 1e-2 for FP32 results: below it a
    value's absolute error, about one unit roundoff of the largest bucket value
    per FFT stage, is no longer a small fraction of the value)."""
    diffs, errs = [], []
    for r, o in zip(res, refs):
        diffs.append(int(np.setxor1d(r["locs"], o["locs"]).size))
        common, ig, io = np.intersect1d(r["locs"], o["locs"], return_indices=True)
        if common.size:
            ref = o["vals"][io]
            den = np.maximum(np.abs(ref), floor * np.max(np.abs(o["vals"])))
            errs.append(float(np.max(np.abs(r["vals"][ig] - ref) / den)))
        else:
            errs.append(0.0)
    return {"oracle_signals": len(refs), "oracle_set_diff": int(sum(diffs)),
            "oracle_set_diff_per_signal": diffs, "oracle_max_rel_err": max(errs) if errs else None,
            "oracle_mean_rel_err": float(np.mean(errs)) if errs else None}


def _oracle_uneven_one(job):
    """One signal of the uneven workload through the oracle (a pool worker)."""
    import oracle

    i, m, k, snr, seed = job
    from paper_1908_02461_amd import synth

    x = synth.planted_1d(m, k, seed, mag=("uniform", 0.5, 1.0), snr_db=snr)[0]
    p = oracle.Params.defaults(1, m, seed=11, signal=i, delta=1e-6)
    t0 = time.perf_counter()
    oracle.atsfft(x, p, trace=False)
    return time.perf_counter() - t0


def cpu_baseline_uneven(budget_s, workers=None):
    """The FP64 oracle over the uneven workload's signals, one process per
    host core (at most 16), each signal generated on the host with the same
    recipe (the lengths, sparsities and SNRs of the batch's first signals);
    signals per second of wall clock over the pool.  Runs before the process
    touches the GPU (the pool forks it)."""
    import multiprocessing as mp

    rng = np.random.Generator(np.random.PCG64(4242))  # the uneven workload's draws
    batch = 512
    ns = (1 << rng.integers(16, 23, size=batch)).astype(np.int64)
    ks = np.rint(np.exp(rng.uniform(np.log(4), np.log(1024), size=batch))).astype(np.int64)
    snrs = rng.uniform(20.0, 60.0, size=batch)
    workers = workers or min(16, os.cpu_count() or 1)
    jobs = [(i, int(ns[i]), int(ks[i]), float(snrs[i]), 3000 + i) for i in range(batch)]
    done, t0 = 0, time.perf_counter()
    with mp.get_context("fork").Pool(workers) as pool:
        for _ in pool.imap_unordered(_oracle_uneven_one, jobs[: 4 * workers * 8], chunksize=1):
            done += 1
            if time.perf_counter() - t0 >= budget_s:
                pool.terminate()
                break
    el = time.perf_counter() - t0
    log(f"cpu baseline: {done} signals in {el:.1f} s on {workers} processes")
    return {"value": done / el, "unit": "transforms/s", "cores": workers, "kind": "oracle",
            "sample": f"the first {done} signals of the uneven workload's recipe (host-generated), FP64 oracle, "
                      f"{workers} processes, {el:.1f} s wall"}


def copy_bandwidth_gbs(reps: int = 10) -> float:
    """Attainable HBM bandwidth: a plain 1 GiB device-to-device copy (1 GiB
    read + 1 GiB written), timed with HIP events."""
    import torch

    src = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * (1 << 30) / (ms * 1e-3) / 1e9


def copy_calibration():
    """One plain 1 GiB device copy: the reference for the HBM byte counters."""
    import torch

    src = torch.empty(1 << 27, dtype=torch.complex64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=32)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--error-signals", type=int, default=4)
    ap.add_argument("--no-per-signal", action="store_true", help="skip the plain per-signal form")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="end with one plain 1 GiB device copy (reference for HBM byte counters)")
    ap.add_argument("--workload", default="c2", choices=("c2", "c3", "c4", "c5", "known_k", "ksweep"),
                    help="c2: 1D n=2^22 k=64 (default); c3: 2D 4096^2 k=256; c4: uneven batch of 512; "
                         "c5: forward + adjoint, batch 64 of n=2^20 k=128; "
                         "known_k: ATSFFT against the known-k form of Algorithm 1; "
                         "ksweep: n=2^22 for k = 16..256 against the dense FFT")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the transform of one signal does not span GPUs "
              "and the library has no multi-GPU path; run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    if args.workload != "c2":
        import bench_workloads

        cpu = None
        if args.workload == "c4" and not args.no_cpu_baseline:
            # before anything touches the GPU: the pool forks this process
            log("cpu baseline (oracle, process pool)")
            cpu = cpu_baseline_uneven(args.cpu_seconds)
        line = bench_workloads.run(args)
        if cpu is not None:
            line["cpu_baseline"] = cpu
        if args.copy_calibration:
            copy_calibration()
        print(json.dumps(line), flush=True)
        return

    import torch

    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import synth

    w = synth.WORKLOADS[WORKLOAD]
    n, k, batch = w["n"], w["k"], args.batch
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)

    log(f"generating {batch} signals n={n} k={k}")
    sigs = []
    for i in range(batch):
        sigs.append(synth.make(WORKLOAD, 1000 + i))
        if (i + 1) % 8 == 0:
            log(f"  {i + 1}/{batch}")
    xh = np.stack([s[0] for s in sigs])
    x = torch.from_numpy(xh).to(dev)

    plan = A.Plan(1, n, "c64", seed=PLAN_SEED, max_batch=batch)
    out = plan.outputs(batch, dev)
    ws = plan.workspace(batch, dev)
    step = lambda: plan.execute_batched(x, out=out, ws=ws)
    log("warmup")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")
    ms_step = timed(step, args.steps, stream)
    value = batch / (ms_step / 1e3)

    # results of the last step
    res = [plan.results(out, i) for i in range(batch)]
    trs = [plan.trace(ws, i, full=False) for i in range(batch)]

    # stage timing with HIP events on the library's stream (separate plan,
    # same knobs and draws)
    pplan = A.Plan(1, n, "c64", seed=PLAN_SEED, max_batch=batch, profile=True)
    pout = pplan.outputs(batch, dev)
    pws = pplan.workspace(batch, dev)
    pstep = lambda: pplan.execute_batched(x, out=pout, ws=pws)
    pstep()
    pplan.profile_read()
    log("profiled steps")
    ms_prof = timed(pstep, args.steps, stream)
    prof = pplan.profile_read()
    stage_ms = {s: prof[s] / prof["executes"] for s in A.STAGES}

    # roofline of the dominant kernel (the main-loop permute/window/fold):
    # algorithmic bytes = the samples it reads (8 B each) plus the bucket
    # values it writes, summed over the batch's loops
    d = plan.desc
    L = d.L_loc + d.L_est
    alg_bytes = 0
    for t in trs:
        if t["status"] & A.SIG_EMPTY:
            continue
        B = t["B_star"]
        wlen = min(d.alpha * B, n)
        alg_bytes += L * (wlen * 8 + B * 8)
    hash_s = stage_ms["hash_main"] / 1e3
    achieved = alg_bytes / hash_s / 1e9
    log("touched lines")
    touched_main, touched_step = touched_bytes(d, trs)
    copy_gbs = copy_bandwidth_gbs()

    # plain per-signal form
    plan1 = A.Plan(1, n, "c64", seed=PLAN_SEED, max_batch=1)
    out1 = plan1.outputs(1, dev)
    ws1 = plan1.workspace(1, dev)
    xs1 = [x[i:i + 1] for i in range(batch)]

    def per_signal():
        for xi in xs1:
            plan1.execute_batched(xi, out=out1, ws=ws1)

    # the same per-signal form replayed from HIP graphs (ATSFFT_FLAG_GRAPH)
    plan1g = A.Plan(1, n, "c64", seed=PLAN_SEED, max_batch=1, graph=True)
    out1g = plan1g.outputs(1, dev)
    ws1g = plan1g.workspace(1, dev)

    def per_signal_graph():
        for xi in xs1:
            plan1g.execute_batched(xi, out=out1g, ws=ws1g)

    ms_single = ms_single_graph = None
    if not args.no_per_signal:
        per_signal()
        log("per-signal form")
        ms_single = timed(per_signal, max(1, args.steps // 5), stream) / batch
        per_signal_graph()
        ms_single_graph = timed(per_signal_graph, max(1, args.steps // 5), stream) / batch

    # same-GPU dense FFT (rocFFT through torch.fft) on the same batch
    y = torch.empty_like(x)
    dense = lambda: torch.fft.fft(x, dim=-1, out=y)
    for _ in range(args.warmup):
        dense()
    log("dense FFT")
    ms_dense = timed(dense, args.steps, stream)

    # L1 error (the paper's error display) on the first signals: against the
    # FFT of x (FP64) and against the planted noise-free spectrum
    errs, errs_truth, recovered = [], [], []
    for i in range(min(args.error_signals, batch)):
        r = res[i]
        X = torch.fft.fft(x[i].to(torch.complex128))
        locs = torch.from_numpy(r["locs"]).to(dev)
        vals = torch.from_numpy(r["vals"]).to(dev)
        tot = torch.sum(torch.abs(X)) - torch.sum(torch.abs(X[locs])) + torch.sum(torch.abs(vals - X[locs]))
        errs.append(float(tot) / k)
        _, plocs, pamps = sigs[i]
        idx = np.searchsorted(r["locs"], plocs)
        idx = np.clip(idx, 0, max(len(r["locs"]) - 1, 0))
        hit = (len(r["locs"]) > 0) & (r["locs"][idx] == plocs) if len(r["locs"]) else np.zeros(k, bool)
        e = np.sum(np.abs(np.where(hit, r["vals"][idx] if len(r["locs"]) else 0, 0) - pamps))
        extra = np.setdiff1d(np.arange(len(r["locs"])), idx[hit])
        e += np.sum(np.abs(r["vals"][extra]))
        errs_truth.append(e / k)
        recovered.append(float(np.mean(hit)))

    if args.copy_calibration:
        copy_calibration()

    cpu, agree = None, {}
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu, refs = cpu_baseline(d, xh, args.cpu_seconds)
        agree = oracle_agreement(res[:len(refs)], refs)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "transforms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n": n, "k": k, "snr_db": 40.0, "batch": batch,
                   "magnitudes": "uniform[0.5,1]", "input": "c64", "parallelism": "none (1 GPU)"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(batch),
                     "kernel": "k_hash (main loops)", "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_ms": stage_ms["hash_main"],
                     "touched_bytes_per_launch": touched_main,
                     "touched_frac": touched_main / hash_s / 1e9 / HBM_PEAK_GBS,
                     "attainable_copy_gbs": copy_gbs},
        "touched_bytes_per_step": touched_step,
        "touched_frac_of_step": touched_step / (ms_step / 1e3) / 1e9 / HBM_PEAK_GBS,
        "cpu_baseline": cpu,
        **agree,
        "dense_fft_ms_per_transform": ms_dense / batch,
        "atsfft_ms_per_transform": ms_step / batch,
        "speedup_vs_dense_fft": ms_dense / ms_step,
        "per_signal_ms_per_transform": ms_single,
        "per_signal_graph_ms_per_transform": ms_single_graph,
        "k_hash_source_sha256": hash_kernel_sha256(),
        "stage_ms_per_step": stage_ms,
        "profiled_ms_per_step": ms_prof,
        "l1_error": float(np.mean(errs)) if errs else None,
        "l1_error_vs_planted": float(np.mean(errs_truth)) if errs_truth else None,
        "recovered_fraction": float(np.mean(recovered)) if recovered else None,
        "B_star": sorted({t["B_star"] for t in trs}),
        "khat_range": [min(r["khat"] for r in res), max(r["khat"] for r in res)],
        "located_range": [min(r["count"] for r in res), max(r["count"] for r in res)],
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
