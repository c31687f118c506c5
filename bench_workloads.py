"""Benchmarks of the workloads beyond the headline one (bench.py --workload):
the 2D image workload, the uneven batch, forward + adjoint, and the known-k
comparator.  Each returns one JSON-serialisable record; bench.py adds the
CPU baseline where it has one."""
from __future__ import annotations

import os
import sys

import numpy as np


def _log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def _timed(fn, steps):
    import torch

    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _base(metric, value, unit, args, ms, config, dtype="f32"):
    return {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": dtype, "data": "synthetic", "config": config}


def run_c3(args):
    """2D: 4096 x 4096 c64 images, k = 256 log-uniform [0.1, 1], 30 dB."""
    import torch

    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import synth

    N, k, batch = 4096, 256, 8
    _log(f"generating {batch} images")
    imgs = [synth.make("c3_2d_c64_n4096_k256_snr30", 2000 + i) for i in range(batch)]
    x = torch.from_numpy(np.stack([t[0] for t in imgs])).cuda()
    plan = A.Plan(2, N, "c64", seed=7, max_batch=batch)
    out = plan.outputs(batch, x.device)
    ws = plan.workspace(batch, x.device)
    step = lambda: plan.execute_batched(x, out=out, ws=ws)
    for _ in range(args.warmup):
        step()
    ms = _timed(step, args.steps)
    y = torch.empty_like(x)
    dense = lambda: torch.fft.fft2(x, out=y)
    for _ in range(args.warmup):
        dense()
    ms_dense = _timed(dense, args.steps)
    rec = []
    for i in range(batch):
        r = plan.results(out, i)
        rec.append(float(np.mean(np.isin(imgs[i][1], r["locs"]))))
    line = _base("sparse 2D transforms/sec and speedup vs same-GPU dense FFT2 at 4096^2, k=256",
                 batch / (ms / 1e3), "transforms/s", args, ms,
                 {"workload": "c3_2d_c64_n4096_k256_snr30", "N": N, "k": k, "batch": batch})
    line.update({"dense_fft2_ms_per_transform": ms_dense / batch, "speedup_vs_dense_fft2": ms_dense / ms,
                 "recovered_fraction": float(np.mean(rec)),
                 "B_star": sorted({plan.trace(ws, i, full=False)["B_star"] for i in range(batch)})})
    # roofline of the dominant kernel, the 2D main-loop hash (streamed rows),
    # timed with HIP events at the plan's stage marks on the library stream
    prof = A.Plan(2, N, "c64", seed=7, max_batch=batch, profile=True)
    pws = prof.workspace(batch, x.device)
    pout = prof.outputs(batch, x.device)
    for _ in range(max(1, args.warmup)):
        prof.execute_batched(x, out=pout, ws=pws)
    torch.cuda.synchronize()
    prof.profile_read()
    for _ in range(args.steps):
        prof.execute_batched(x, out=pout, ws=pws)
    pr = prof.profile_read()
    stages = {kk: v / pr["executes"] for kk, v in pr.items() if kk != "executes"}
    alg = hash2d_stream_bytes(prof.desc, [prof.trace(pws, i, full=False) for i in range(batch)])
    hms = stages["hash_main"]
    from bench import ROOT, copy_bandwidth_gbs, measured_traffic, section_sha256

    traffic = measured_traffic(batch, os.path.join(ROOT, "profiles", "hash2d_stream_c3_n4096_k256_b8_hbm_traffic.txt"),
                               section_sha256("2D row hash", "probe control"), key="section_sha256")
    line["roofline"] = {"bound": "hbm", "achieved": alg / (hms * 1e-3) / 1e9, "peak": 8000.0, "unit": "GB/s",
                        "frac": alg / (hms * 1e-3) / 8e12, "traffic": traffic,
                        "kernel": "k_hash2d_stream (main loops)", "alg_bytes_per_launch": alg,
                        "avg_launch_ms": hms, "attainable_copy_gbs": copy_bandwidth_gbs()}
    line["stage_ms_per_step"] = stages
    prof.close()
    return line


def hash2d_stream_bytes(desc, trs):
    """Bytes the streamed 2D main-loop hash must move per batch: every row
    some loop uses, read once (N c64 samples), plus one B x B partial per row
    wrap and loop written.  Loop l uses rows sigma1 (i1 - w/2) + tau1 mod N,
    i1 < w, with (sigma1, tau1) drawn as the library documents."""
    from bench import _splitmix64_at

    from paper_1908_02461_amd import atsfft as A

    N, L = desc.n, desc.L_loc + desc.L_est
    total = 0
    for s, t in enumerate(trs):
        if t["status"] & A.SIG_EMPTY:
            continue
        B = t["B_star"]
        w = min(desc.alpha * B, N)
        rows = []
        for l in range(L):
            phase, it = (1, l) if l < desc.L_loc else (2, l - desc.L_loc)
            r = _splitmix64_at(desc.seed, ((s * 4 + phase) * 256 + it) * 2)
            sigma, tau = (r % N) | 1, (r >> 32) % N
            rows.append((sigma * (np.arange(w, dtype=np.int64) - w // 2) + tau) % N)
        total += np.unique(np.concatenate(rows)).size * N * 8 + L * (w // B) * B * B * 8
    return int(total)


def run_c4(args):
    """512 c64 signals, n uniform over 2^16..2^22, k log-uniform [4, 1024],
    SNR uniform [20, 60] dB, magnitudes uniform [0.5, 1]; one uneven call."""
    import torch

    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import synth

    batch = 512
    rng = np.random.Generator(np.random.PCG64(4242))
    ns = (1 << rng.integers(16, 23, size=batch)).astype(np.int64)
    ks = np.rint(np.exp(rng.uniform(np.log(4), np.log(1024), size=batch))).astype(np.int64)
    snrs = rng.uniform(20.0, 60.0, size=batch)
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    total = int(ns.sum())
    _log(f"generating {batch} signals, {total * 8 / 2**30:.2f} GiB")
    x = torch.empty(total, dtype=torch.complex64, device="cuda")
    planted, truth = [], []
    for i in range(batch):
        xi, locs, amps = synth.planted_1d_device(int(ns[i]), int(ks[i]), 3000 + i, mag=("uniform", 0.5, 1.0),
                                                 snr_db=float(snrs[i]))
        x[offs[i]:offs[i] + ns[i]] = xi
        planted.append(locs)
        truth.append((locs, amps))
        if (i + 1) % 128 == 0:
            _log(f"  {i + 1}/{batch}")
    # the knobs: the autotuner on this batch (filter factor and loop counts
    # against recovery of the planted spectra), the library defaults as its
    # baseline
    from paper_1908_02461_amd import autotune

    _log("autotuning")
    tuned = autotune.tune_uneven(x, offs, ns, truth, n_max=1 << 22, n_min=1 << 16, seed=11)
    knobs = tuned.knobs
    _log(f"tuned knobs {knobs}")
    plan = A.Plan(1, 1 << 22, "c64", seed=11, n_min=1 << 16, max_batch=batch, **knobs)
    out = plan.outputs(batch, x.device)
    step = lambda: plan.execute_uneven(x, offs, ns, out=out)
    o = step()
    ws = o["ws"]
    step = lambda: plan.execute_uneven(x, offs, ns, out=out, ws=ws)
    for _ in range(args.warmup):
        step()
    ms_grouped = _timed(step, args.steps)
    # the same call with the lengths and offsets on the device: one launch
    # sequence for all lengths, eager and replayed from a HIP graph
    offs_d = torch.from_numpy(offs).cuda()
    ns_d = torch.from_numpy(ns.astype(np.int64)).cuda()
    outd = plan.outputs(batch, x.device)
    wsd = torch.empty(plan.workspace_size_uneven_dev(batch), dtype=torch.uint8, device="cuda")
    stepd = lambda: plan.execute_uneven_dev(x, offs_d, ns_d, out=outd, ws=wsd)
    for _ in range(args.warmup):
        stepd()
    ms_dev = _timed(stepd, args.steps)
    plang = A.Plan(1, 1 << 22, "c64", seed=11, n_min=1 << 16, max_batch=batch, graph=True, **knobs)
    outg = plang.outputs(batch, x.device)
    stepg = lambda: plang.execute_uneven_dev(x, offs_d, ns_d, out=outg, ws=wsd)
    for _ in range(args.warmup):
        stepg()
    ms = _timed(stepg, args.steps)
    torch.cuda.synchronize()
    same = all(torch.equal(outg[k], out[k]) for k in ("count", "khat", "status"))
    # dense FFT of every signal, grouped by length
    groups = {}
    for i, m in enumerate(ns):
        groups.setdefault(int(m), []).append(i)
    views = {m: torch.stack([x[offs[i]:offs[i] + m] for i in idx]) for m, idx in groups.items()}
    outs = {m: torch.empty_like(v) for m, v in views.items()}

    def dense():
        for m, v in views.items():
            torch.fft.fft(v, dim=-1, out=outs[m])

    for _ in range(args.warmup):
        dense()
    ms_dense = _timed(dense, args.steps)
    rec, sat = [], 0
    for i in range(batch):
        r = plan.results(out, i)
        rec.append(float(np.mean(np.isin(planted[i], r["locs"]))))
        sat += bool(r["status"] & A.SIG_PROBE_SATURATED)
    # the plain per-signal form: every signal through a plan of its length,
    # one execute each; its traces give each signal's bucket count
    plans = {m: A.Plan(1, m, "c64", seed=11, max_batch=1, **knobs) for m in groups}
    pout = {m: p1.outputs(1, x.device) for m, p1 in plans.items()}
    pws = {m: p1.workspace(1, x.device) for m, p1 in plans.items()}
    views1 = [x[offs[i]:offs[i] + ns[i]].view(1, int(ns[i])) for i in range(batch)]

    def per_signal():
        for i in range(batch):
            m = int(ns[i])
            plans[m].execute_batched(views1[i], out=pout[m], ws=pws[m])

    per_signal()
    ms_single = _timed(per_signal, max(1, args.steps // 5))
    Bs = []
    for i in range(batch):
        m = int(ns[i])
        plans[m].execute_batched(views1[i], out=pout[m], ws=pws[m])
        Bs.append(plans[m].trace(pws[m], 0, full=False)["B_star"])
    # touched bytes of the main loops (distinct 128-byte input lines plus the
    # bucket values written), each signal at the B of
    # its per-signal run and with the draws of its index in the uneven call
    import bench

    d0 = plan.desc
    tb = 0
    for i in range(batch):
        m, B = int(ns[i]), Bs[i]
        w = min(d0.alpha * B, m)
        L = d0.L_loc + d0.L_est
        lines = [bench._loop_lines(d0.seed, i, 1 if l < d0.L_loc else 2, l if l < d0.L_loc else l - d0.L_loc, m, w)
                 for l in range(L)]
        tb += 128 * np.unique(np.concatenate(lines)).size + L * B * 8
    line = _base("sparse transforms/sec, uneven batch of 512 (n 2^16..2^22, k 4..1024)", batch / (ms / 1e3),
                 "transforms/s", args, ms,
                 {"workload": "c4_1d_c64_uneven_b512", "batch": batch, "n_range": [1 << 16, 1 << 22],
                  "k_range": [4, 1024], "snr_db_range": [20, 60], "total_gib": total * 8 / 2**30,
                  "form": "device-side lengths, one launch sequence replayed from a HIP graph"})
    line.update({"grouped_ms_per_batch": ms_grouped, "device_lengths_eager_ms_per_batch": ms_dev,
                 "graph_matches_grouped": bool(same),
                 "dense_fft_ms_per_batch": ms_dense, "speedup_vs_dense_fft": ms_dense / ms,
                 "recovered_fraction": float(np.mean(rec)), "probe_saturated": sat,
                 "per_signal_ms_per_batch": ms_single, "batched_over_per_signal": ms_single / ms,
                 "touched_bytes_per_batch": tb, "touched_gbs_per_batch_time": tb / (ms / 1e3) / 1e9,
                 "touched_frac_of_peak": tb / (ms / 1e3) / 1e9 / 8000.0,
                 "tuned_knobs": knobs, "default_knobs_ms_per_batch": tuned.baseline_ms_per_transform * batch,
                 "tuning_candidates": [{"knobs": t["knobs"], "ms_per_batch": t["ms_per_transform"] * batch,
                                        "recovery": t["recovery"], "l1_vs_planted": t["l1_vs_planted"]}
                                       for t in tuned.tried if t["valid"]]})
    return line


def run_c5(args):
    """Forward + adjoint: batch 64 of c64 n = 2^20, k = 128, 40 dB; loss =
    sum |X_hat(located) - target|^2 with random complex targets."""
    import torch

    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import synth

    n, k, batch = 1 << 20, 128, 64
    _log(f"generating {batch} signals n={n}")
    x = torch.stack([synth.planted_1d_device(n, k, 5000 + i, mag=("uniform", 0.5, 1.0), snr_db=40.0)[0]
                     for i in range(batch)]).contiguous()
    plan = A.Plan(1, n, "c64", seed=13, max_batch=batch)
    g = torch.Generator(device="cuda")
    g.manual_seed(77)
    targets = torch.randn((batch, plan.max_out), generator=g, device="cuda", dtype=torch.complex64)
    xr = x.clone().requires_grad_(True)

    def step():
        xr.grad = None
        vals, locs, count, khat, status = A.sparse_fft(xr, plan)
        mask = torch.arange(plan.max_out, device="cuda")[None, :] < count[:, None]
        loss = torch.sum(torch.abs(vals - targets) ** 2 * mask)
        loss.backward()

    for _ in range(args.warmup):
        step()
    ms = _timed(step, args.steps)
    fwd = lambda: plan.execute_batched(x)
    for _ in range(args.warmup):
        fwd()
    ms_fwd = _timed(fwd, args.steps)
    line = _base("forward+adjoint transforms/sec at n=2^20, k=128 (loss over located values)",
                 batch / (ms / 1e3), "transforms/s", args, ms,
                 {"workload": "c5_1d_c64_n1m_k128_snr40_grad", "n": n, "k": k, "batch": batch})
    line.update({"forward_only_ms_per_step": ms_fwd, "adjoint_share": 1.0 - ms_fwd / ms})
    return line


def _planted_error(r, plocs, pamps):
    """Recovered fraction and L1 error per planted coefficient against the
    planted noise-free spectrum (false positives count with their magnitude)."""
    locs, vals = r["locs"], r["vals"]
    k = len(plocs)
    if len(locs) == 0:
        return 0.0, float(np.sum(np.abs(pamps))) / k
    idx = np.clip(np.searchsorted(locs, plocs), 0, len(locs) - 1)
    hit = locs[idx] == plocs
    e = np.sum(np.abs(np.where(hit, vals[idx], 0) - pamps))
    extra = np.setdiff1d(np.arange(len(locs)), idx[hit])
    e += np.sum(np.abs(vals[extra]))
    return float(np.mean(hit)), float(e) / k


def _compare_known_k(A, ndim, n, k, x, truth, args, seed, wide=None):
    """Time ATSFFT and the known-k form on one batch; B_kk = sqrt(n k) per axis
    rounded to a power of two and clipped to the largest bucket count a plan
    takes (1D: the plan's cap; 2D: 1024 per axis, the arrays then held in
    device memory).  `wide`: knobs of a further ATSFFT plan (a B_max beyond
    the default cap), timed as "atsfft_wide"."""
    import torch

    batch = x.shape[0]
    ada = A.Plan(ndim, n, "c64", seed=seed, max_batch=batch)
    cap = ada.desc.B_max if ndim == 1 else min(1024, n // 2)
    b_paper = int(round(np.log2(np.sqrt(float(n) * k))))
    B_kk = min(1 << b_paper, cap)
    kk = A.Plan(ndim, n, "c64", seed=seed, max_batch=batch, fixed_B=B_kk, fixed_k=k)
    rows = {}
    plans = [("atsfft", ada), ("known_k", kk)]
    if wide:
        plans.append(("atsfft_wide", A.Plan(ndim, n, "c64", seed=seed, max_batch=batch, **wide)))
    for name, plan in plans:
        out = plan.outputs(batch, x.device)
        ws = plan.workspace(batch, x.device)
        step = lambda: plan.execute_batched(x, out=out, ws=ws)
        for _ in range(args.warmup):
            step()
        ms = _timed(step, args.steps)
        rec, err = zip(*[_planted_error(plan.results(out, i), *truth[i]) for i in range(batch)])
        rows[name] = {"ms_per_transform": ms / batch, "recovered_fraction": float(np.mean(rec)),
                      "l1_error_vs_planted": float(np.mean(err)),
                      "B": sorted({plan.trace(ws, i, full=False)["B_star"] for i in range(batch)})}
        del out, ws
        torch.cuda.synchronize()
    rows["known_k"]["B_formula"] = 1 << b_paper
    rows["known_k"]["B_clipped"] = B_kk != (1 << b_paper)
    return rows


def run_known_k(args):
    """The paper's comparison in kind: ATSFFT (k probed) against the known-k
    sparse FFT of Algorithm 1 (B = sqrt(n k), num = d k, no probe), same GPU,
    same inputs: 16 signals of n = 2^22, k = 64, 40 dB, and 8 images of
    4096^2, k = 256, 30 dB."""
    import torch

    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import synth

    _log("generating 16 signals n=2^22")
    sig = [synth.make("c2_1d_c64_n4m_k64_snr40", 1000 + i) for i in range(16)]
    x = torch.from_numpy(np.stack([t[0] for t in sig])).cuda()
    one = _compare_known_k(A, 1, 1 << 22, 64, x, [(t[1], t[2]) for t in sig], args, 7)
    del x
    _log("generating 8 images 4096^2")
    img = [synth.make("c3_2d_c64_n4096_k256_snr30", 2000 + i) for i in range(8)]
    x = torch.from_numpy(np.stack([t[0] for t in img])).cuda()
    two = _compare_known_k(A, 2, 4096, 256, x, [(t[1], t[2]) for t in img], args, 7)
    del x
    # the paper's fixed-size sweep in kind (its Table 2): 2048^2 images, k
    # planted frequencies of magnitude 1 and no noise, k = 50 .. 1000
    sweep = []
    for k in (50, 100, 200, 400, 800, 1000):
        _log(f"2048^2 sweep: k = {k}")
        img = [synth.planted_2d(2048, k, 9000 + 10 * k + i, dtype=np.complex64) for i in range(4)]
        x = torch.from_numpy(np.stack([t[0] for t in img])).cuda()
        r = _compare_known_k(A, 2, 2048, k, x, [(t[1], t[2]) for t in img], args, 7, wide={"B_max": 1024})
        r["k"] = k
        r["speedup"] = r["known_k"]["ms_per_transform"] / r["atsfft"]["ms_per_transform"]
        r["speedup_wide"] = r["known_k"]["ms_per_transform"] / r["atsfft_wide"]["ms_per_transform"]
        sweep.append(r)
        del x
    speed = one["known_k"]["ms_per_transform"] / one["atsfft"]["ms_per_transform"]
    line = _base("speedup of ATSFFT (k probed) over the known-k sparse FFT (B = sqrt(nk)), n=2^22 k=64",
                 speed, "x", args, one["atsfft"]["ms_per_transform"] * 16,
                 {"workload": "known_k_vs_atsfft", "1d": "16 x n=2^22 c64 k=64 40dB",
                  "2d": "8 x 4096^2 c64 k=256 30dB", "2d_sweep": "4 x 2048^2 c64 |a|=1 no noise, k=50..1000, "
                               "ATSFFT at its default B_max (128) and at B_max = 1024"})
    line.update({"1d": one, "2d": two,
                 "speedup_2d": two["known_k"]["ms_per_transform"] / two["atsfft"]["ms_per_transform"],
                 "2d_sweep": sweep})
    return line


def run_ksweep(args):
    """The headline length (n = 2^22 c64, 40 dB, magnitudes uniform [0.5, 1])
    across sparsities k = 16, 64, 128, 256: batched ATSFFT (library defaults,
    16 signals per k) against the same GPU's dense FFT of the same batch."""
    import torch

    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import synth

    n, batch = 1 << 22, 16
    rows = []
    for k in (16, 64, 128, 256):
        _log(f"k = {k}")
        sig = [synth.planted_1d_device(n, k, 7000 + 100 * k + i, mag=("uniform", 0.5, 1.0), snr_db=40.0)
               for i in range(batch)]
        x = torch.stack([t[0] for t in sig]).contiguous()
        plan = A.Plan(1, n, "c64", seed=5, max_batch=batch)
        out = plan.outputs(batch, x.device)
        ws = plan.workspace(batch, x.device)
        step = lambda: plan.execute_batched(x, out=out, ws=ws)
        for _ in range(args.warmup):
            step()
        ms = _timed(step, args.steps)
        y = torch.empty_like(x)
        dense = lambda: torch.fft.fft(x, dim=-1, out=y)
        for _ in range(args.warmup):
            dense()
        ms_dense = _timed(dense, args.steps)
        rec, err = [], []
        for i in range(batch):
            r = plan.results(out, i)
            locs, amps = sig[i][1], sig[i][2]
            hit = np.isin(locs, r["locs"])
            rec.append(float(np.mean(hit)))
            idx = np.searchsorted(r["locs"], locs[hit])
            err.append(float(np.mean(np.abs(r["vals"][idx] - amps[hit]))) if hit.any() else float("nan"))
        rows.append({"k": k, "ms_per_transform": ms / batch, "dense_fft_ms_per_transform": ms_dense / batch,
                     "speedup_vs_dense_fft": ms_dense / ms, "recovered_fraction": float(np.mean(rec)),
                     "mean_abs_err_recovered": float(np.nanmean(err)),
                     "B_star": sorted({plan.trace(ws, i, full=False)["B_star"] for i in range(batch)})})
        plan.close()
        del x, y
    worst = min(r["speedup_vs_dense_fft"] for r in rows)
    line = _base("smallest speedup of batched ATSFFT over the same GPU's dense FFT, n=2^22, k in {16,64,128,256}",
                 worst, "x", args, sum(r["ms_per_transform"] for r in rows) * batch,
                 {"workload": "ksweep_1d_c64_n4m_snr40", "n": n, "k": [16, 64, 128, 256], "batch": batch})
    line["per_k"] = rows
    return line


def run(args):
    return {"c3": run_c3, "c4": run_c4, "c5": run_c5, "known_k": run_known_k,
            "ksweep": run_ksweep}[args.workload](args)
