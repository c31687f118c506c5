"""GPU parity: libatsfft.so on an MI355X against the FP64 oracle, same draws.

Each case runs the library through its C ABI and the oracle on identical
inputs and knobs, then checks every discrete decision (probe bucket counts
and local-maximum counts, cutoffs, located set, status) for identity and the
bucket DFTs and values against the tolerance of the precision.
"""
import numpy as np
import pytest

import oracle
from paper_1908_02461_amd import synth

from parity_util import compare, oracle_params, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _check_batch(A, plan, xs, label, trace=True):
    out = run_gpu(plan, np.stack(xs))
    infos = []
    for i, x in enumerate(xs):
        res = plan.results(out, i)
        tr = plan.trace(out["ws"], i)
        ref = oracle.atsfft(x, oracle_params(plan, i), trace=True)
        infos.append(compare(plan, res, tr, ref, f"{label}[{i}]"))
    print(label, infos, flush=True)
    return out, infos


def test_small_1d_c128_noiseless(A):
    """n = 2^14, k = 8, |a| = 1, no noise (the small 1D workload)."""
    n, k = 1 << 14, 8
    for seed in range(4):
        plan = A.Plan(1, n, "c128", seed=seed, max_batch=2)
        xs = [synth.planted_1d(n, k, 100 * seed + i)[0] for i in range(2)]
        _check_batch(A, plan, xs, f"c1 seed={seed}")
        out = run_gpu(plan, np.stack(xs))
        for i in range(2):
            x, locs, amps = synth.planted_1d(n, k, 100 * seed + i)
            res = plan.results(out, i)
            idx = np.searchsorted(res["locs"], locs)
            assert np.array_equal(res["locs"][idx], locs)
            assert np.max(np.abs(res["vals"][idx] - amps)) < 1e-9


def test_1d_c64_noisy(A):
    n, k = 1 << 16, 16
    plan = A.Plan(1, n, "c64", seed=11, max_batch=3)
    xs = [synth.planted_1d(n, k, s, mag=("uniform", 0.5, 1.0), snr_db=30.0, dtype=np.complex64)[0]
          for s in range(3)]
    _check_batch(A, plan, xs, "1d c64 snr30")


def test_full_size_1d_c64(A):
    """n = 2^22, k = 64, |a| in [0.5, 1], SNR 40 dB: the benchmark workload."""
    n = 1 << 22
    plan = A.Plan(1, n, "c64", seed=2019, max_batch=2)
    xs = [synth.make("c2_1d_c64_n4m_k64_snr40", s)[0] for s in (1, 2)]
    _check_batch(A, plan, xs, "c2 full")


def test_small_2d(A):
    N, k = 256, 4
    for dt in ("c128", "c64"):
        plan = A.Plan(2, N, dt, seed=5, max_batch=2, B_max=32)
        npdt = np.complex128 if dt == "c128" else np.complex64
        snr = None if dt == "c128" else 40.0
        mag = None if dt == "c128" else ("uniform", 0.5, 1.0)
        xs = [synth.planted_2d(N, k, s, mag=mag, snr_db=snr, dtype=npdt)[0] for s in range(2)]
        _check_batch(A, plan, xs, f"2d {dt}")


def test_full_size_2d_c64(A):
    """4096 x 4096, k = 256, |a| log-uniform in [0.1, 1], SNR 30 dB."""
    plan = A.Plan(2, 4096, "c64", seed=77, max_batch=1)
    x = synth.make("c3_2d_c64_n4096_k256_snr30", 3)[0]
    _check_batch(A, plan, [x], "c3 full")


def test_fixed_bucket_count(A):
    """Algorithm 1 form: the probe is skipped, B and k are given."""
    n, k = 1 << 14, 8
    plan = A.Plan(1, n, "c128", seed=3, fixed_B=256, fixed_k=8)
    x = synth.planted_1d(n, k, 4)[0]
    _check_batch(A, plan, [x], "fixed B")


@pytest.mark.parametrize("ndim,n,k,dt,snr", [(1, 1 << 16, 16, "c128", None), (1, 1 << 16, 16, "c64", 30.0),
                                              (2, 256, 4, "c128", None)])
def test_known_k_form_at_sqrt_nk(A, ndim, n, k, dt, snr):
    """The known-k sparse FFT the paper compares against (Algorithm 1, the
    bucket count B = sqrt(n k) per axis, num = d k): 1D n = 2^16, k = 16 gives
    B = 1024; 2D N = 256, k = 4 gives 32 per axis."""
    B = int(round(np.sqrt(n * k)))
    assert B & (B - 1) == 0
    plan = A.Plan(ndim, n, dt, seed=5, max_batch=2, fixed_B=B, fixed_k=k)
    npdt = np.complex64 if dt == "c64" else np.complex128
    make = synth.planted_1d if ndim == 1 else synth.planted_2d
    xs = [make(n, k, 60 + i, mag=("uniform", 0.5, 1.0), snr_db=snr, dtype=npdt)[0] for i in range(2)]
    out, _ = _check_batch(A, plan, xs, f"known-k {ndim}D {dt}")
    for i in range(2):
        assert plan.results(out, i)["khat"] == k


def test_zero_signal_is_empty(A):
    n = 1 << 12
    plan = A.Plan(1, n, "c64", seed=1, max_batch=2, B_max=64)
    xs = [np.zeros(n, np.complex64), synth.planted_1d(n, 2, 9, dtype=np.complex64)[0]]
    out, _ = _check_batch(A, plan, xs, "zero + planted")
    res = plan.results(out, 0)
    assert res["status"] & A.SIG_EMPTY and res["count"] == 0 and res["khat"] == 0


def test_truncated_when_capacity_is_small(A):
    n, k = 1 << 14, 8
    plan = A.Plan(1, n, "c128", seed=8, max_out=3)
    x = synth.planted_1d(n, k, 12)[0]
    out, _ = _check_batch(A, plan, [x], "truncated")
    res = plan.results(out, 0)
    assert res["status"] & A.SIG_TRUNCATED and res["count"] >= k


def test_small_bucket_counts_ragged_tiles(A):
    """B below the 64-bucket hash tile and odd loop counts."""
    n = 1 << 10
    plan = A.Plan(1, n, "c128", seed=21, B0=4, B_max=16, alpha=8, alpha_probe=4, gamma=4,
                  L_loc=5, L_est=3, T_vote=3, max_batch=2)
    xs = [synth.planted_1d(n, 1, s)[0] for s in range(2)]
    _check_batch(A, plan, xs, "ragged")


@pytest.mark.parametrize("L_est,L_loc,T_vote", [(1, 3, 3), (15, 7, 2), (31, 11, 6)])
def test_loop_count_variants(A, L_est, L_loc, T_vote):
    n, k = 1 << 14, 6
    plan = A.Plan(1, n, "c128", seed=L_est, L_est=L_est, L_loc=L_loc, T_vote=T_vote)
    x = synth.planted_1d(n, k, 40 + L_est)[0]
    _check_batch(A, plan, [x], f"loops {L_est}/{L_loc}/{T_vote}")


def test_repeat_runs_are_bitwise_identical(A):
    n = 1 << 16
    plan = A.Plan(1, n, "c64", seed=99, max_batch=2)
    xs = np.stack([synth.planted_1d(n, 12, s, mag=("uniform", 0.5, 1.0), snr_db=35.0,
                                    dtype=np.complex64)[0] for s in range(2)])
    a = run_gpu(plan, xs)
    ra = [plan.results(a, i) for i in range(2)]
    b = run_gpu(plan, xs)
    rb = [plan.results(b, i) for i in range(2)]
    for u, v in zip(ra, rb):
        assert np.array_equal(u["locs"], v["locs"])
        assert np.array_equal(u["vals"], v["vals"])


@pytest.mark.parametrize("n,k,knobs", [(1 << 22, 64, {}), (1 << 16, 16, dict(alpha=256, B_max=128))])
def test_compensated_fold(A, n, k, knobs):
    """ATSFFT_FLAG_COMPENSATED (Neumaier FP32 fold sums, FP64 slab partials):
    parity with the oracle, and bucket DFTs on average no farther from it than
    the plain FP32 fold's (measured: 6 to 12 % closer; the FP32 taps and DFT
    bound the rest)."""
    x = synth.planted_1d(n, k, 5, mag=("uniform", 0.5, 1.0), snr_db=30.0, dtype=np.complex64)[0]
    means = {}
    for comp in (False, True):
        plan = A.Plan(1, n, "c64", seed=3, compensated=comp, **knobs)
        out, infos = _check_batch(A, plan, [x], f"compensated={comp}")
        ref = oracle.atsfft(x.astype(np.complex128), oracle_params(plan, 0), trace=True)
        yr, yg = ref["yhat"], plan.trace(out["ws"], 0)["yhat"]
        means[comp] = float(np.mean(np.abs(yg - yr) / np.max(np.abs(yr), axis=1, keepdims=True)))
    print("mean bucket error plain / compensated", means, flush=True)
    assert means[True] <= means[False]


def test_batch_of_seven(A):
    """A batch of seven signals of different sparsity, each against the oracle
    with its index in the call as draw key."""
    n = 1 << 14
    plan = A.Plan(1, n, "c128", seed=41, max_batch=7)
    xs = [synth.planted_1d(n, 3 + i, 500 + i, mag=("uniform", 0.5, 1.0), snr_db=35.0)[0] for i in range(7)]
    _check_batch(A, plan, xs, "batch of seven")


@pytest.mark.parametrize("form", [0, 1, 2])
@pytest.mark.parametrize("N,dt,knobs", [
    (512, "c64", dict(B_max=32)),                 # w = 8B < N: eight row wraps
    (256, "c128", dict(fixed_B=64, fixed_k=6)),   # w = N: four row wraps
    (512, "c64", dict(alpha=12, B_max=32)),       # alpha above 8: no streamed form
    (4096, "c128", dict(B_max=16)),               # 64 KiB rows, the largest staged
])
def test_2d_main_hash_forms(A, monkeypatch, form, N, dt, knobs):
    """The 2D main-loop hash in each of its forms (ATSFFT_ROWS2D: 0 the
    slab gather, 1 one workgroup per bucket row, 2 rows streamed once; a plan
    falls back to the lower form where the higher does not apply) against the
    oracle, and bitwise repeatable."""
    monkeypatch.setenv("ATSFFT_ROWS2D", str(form))
    plan = A.Plan(2, N, dt, seed=13, max_batch=2, **knobs)
    npdt = np.complex128 if dt == "c128" else np.complex64
    xs = [synth.planted_2d(N, 6, 70 + s, mag=("uniform", 0.5, 1.0), snr_db=40.0, dtype=npdt)[0]
          for s in range(2)]
    out, _ = _check_batch(A, plan, xs, f"2d form {form} {N} {dt} {knobs}")
    again = run_gpu(plan, np.stack(xs))
    for i in range(2):
        u, v = plan.results(out, i), plan.results(again, i)
        assert np.array_equal(u["locs"], v["locs"]) and np.array_equal(u["vals"], v["vals"])


@pytest.mark.parametrize("k", [900, 1100])
def test_large_located_sets(A, k):
    """Located sets on either side of the estimator's 1024-entry rank sort
    (above it the bitonic sort runs): Algorithm 1 form at B = 16384, n = 2^16,
    alpha = 4, noiseless planted spectrum."""
    n = 1 << 16
    plan = A.Plan(1, n, "c64", seed=21, alpha=4, fixed_B=16384, fixed_k=k, max_batch=1)
    x = synth.planted_1d(n, k, 400 + k, mag=("uniform", 0.5, 1.0), dtype=np.complex64)[0]
    out, _ = _check_batch(A, plan, [x], f"large S k={k}")
    res = plan.results(out, 0)
    assert (res["count"] > 1024) == (k > 1024), res["count"]
    assert np.all(np.diff(res["locs"]) > 0)


@pytest.mark.parametrize("N,B,alpha,k", [
    (64, 32, 2, 3),       # W = 2 preimages per axis: one candidate per thread
    (128, 32, 4, 4),      # W = 4: one 4 x 4 block per bucket, word-aligned rows
    (256, 16, 4, 5),      # rows of 16 bits: two rows per bitmap word
    (1024, 8, 8, 4),      # W = 128: a bucket's blocks span four workgroup rounds
    (128, 16, 8, 40),     # dense cutoffs: most candidates reach the queue
])
def test_2d_vote_blocks(A, N, B, alpha, k):
    """The 2D vote's row x column blocks of preimages (and the per-candidate
    form below four preimages per axis) give the oracle's located set, at
    fixed B = B per axis with k given."""
    plan = A.Plan(2, N, "c128", seed=31, max_batch=2, alpha=alpha, fixed_B=B, fixed_k=k)
    xs = [synth.planted_2d(N, k, 90 + s, mag=("uniform", 0.5, 1.0))[0] for s in range(2)]
    out, _ = _check_batch(A, plan, xs, f"2d vote N={N} B={B} alpha={alpha} k={k}")
    for i in range(2):
        assert plan.results(out, i)["count"] > 0


@pytest.mark.parametrize("ndim,n,k,dt,snr", [(1, 1 << 14, 8, "c128", None), (1, 1 << 16, 16, "c64", 30.0),
                                              (2, 256, 4, "c128", None)])
def test_probe_without_occupancy_guard(A, ndim, n, k, dt, snr):
    """gamma = 0: the B-update display of Sec. III-A acted on at every level
    (no occupancy guard); on these inputs it stops at a smaller B than the
    guarded probe for most seeds (B* 32-64 at n = 2^14, 8 x 8 at 256^2) and
    locates sets of 30-1200 frequencies, which must match the oracle's."""
    npdt = np.complex64 if dt == "c64" else np.complex128
    kw = dict(B_max=32) if ndim == 2 else {}
    plan = A.Plan(ndim, n, dt, seed=0, max_batch=3, gamma=0, **kw)
    make = synth.planted_1d if ndim == 1 else synth.planted_2d
    mag = None if snr is None else ("uniform", 0.5, 1.0)
    xs = [make(n, k, s, mag=mag, snr_db=snr, dtype=npdt)[0] for s in range(3)]
    _check_batch(A, plan, xs, f"gamma=0 {ndim}D {dt}")


@pytest.mark.parametrize("ndim,n,k,dt,snr,batch", [(1, 1 << 16, 16, "c64", 30.0, 2), (2, 1024, 40, "c64", 30.0, 2),
                                                   (1, 1 << 14, 8, "c128", None, 1)])
def test_cutoff_tie_path(A, monkeypatch, ndim, n, k, dt, snr, batch):
    """The top-num cutoff has two paths: the plain one (J = {m > T}, or
    {m >= v} when exactly num buckets reach the cut value v, the usual case)
    and the tie-aware one (of the buckets equal to v, the first `need` in
    index order), which inputs rarely reach since it needs bitwise-equal
    bucket magnitudes at the cut.  A test hook forces the tie-aware path:
    both give the same bits (cutoff bitmaps and lists, located set, values),
    and both match the oracle."""
    npdt = np.complex64 if dt == "c64" else np.complex128
    mag = ("uniform", 0.5, 1.0) if snr is not None else None
    gen = synth.planted_1d if ndim == 1 else synth.planted_2d
    xs = [gen(n, k, 600 + i, mag=mag, snr_db=snr, dtype=npdt)[0] for i in range(batch)]
    plain = A.Plan(ndim, n, dt, seed=17, max_batch=batch)
    monkeypatch.setenv("ATSFFT_CUTOFF_TIES", "1")
    ties = A.Plan(ndim, n, dt, seed=17, max_batch=batch)
    monkeypatch.delenv("ATSFFT_CUTOFF_TIES")
    print(f"cutoff paths: ndim={ndim} n={n} k={k} {dt}", flush=True)
    a, _ = _check_batch(A, plain, xs, "plain cutoff")
    b, _ = _check_batch(A, ties, xs, "tie-aware cutoff")
    for i in range(batch):
        u, w = plain.results(a, i), ties.results(b, i)
        assert np.array_equal(u["locs"], w["locs"]) and np.array_equal(u["vals"], w["vals"]), i
        tu, tw = plain.trace(a["ws"], i), ties.trace(b["ws"], i)
        assert np.array_equal(tu["J"], tw["J"]), i


def test_main_grid_beyond_the_chip(A):
    """A main pass with more bucket arrays than CUs (16 signals x 18 loops)
    runs the arrays of at most 4096 buckets in 256-thread workgroups and the
    larger ones in a 1024-thread launch of their own; sparsities from 8 to 300
    at n = 2^18 give B* on both sides of 4096.  Every signal against the
    oracle."""
    import torch

    n = 1 << 18
    ks = [8, 16, 32, 64, 128, 200, 256, 300] * 2
    plan = A.Plan(1, n, "c64", seed=23, max_batch=len(ks))
    loops = plan.desc.L_loc + plan.desc.L_est
    assert loops * len(ks) > torch.cuda.get_device_properties(0).multi_processor_count
    xs = [synth.planted_1d(n, k, 700 + i, mag=("uniform", 0.5, 1.0), snr_db=30.0, dtype=np.complex64)[0]
          for i, k in enumerate(ks)]
    out, _ = _check_batch(A, plan, xs, "grid beyond the chip")
    bstar = [plan.trace(out["ws"], i, full=False)["B_star"] for i in range(len(ks))]
    print("B*", bstar, flush=True)
    assert min(bstar) <= 4096 < max(bstar), bstar


@pytest.mark.parametrize("slots", [1, 7, 32])
def test_main_hash_slots_leave_results_bitwise(A, monkeypatch, slots):
    """The main-loop hash's tile slots per address slab (ATSFFT_MAIN_SLOTS)
    only spread the 64-bucket tiles over workgroups: every bucket's partial is
    summed by one thread in the same wrap order, so the bucket DFTs, located
    set and values are bitwise those of the default (64 slots at this batch),
    for a signal with fewer tiles than slots and one with more (B* = 8192)."""
    n = 1 << 18
    ks = [40, 300]
    xs = np.stack([synth.planted_1d(n, k, 900 + i, mag=("uniform", 0.5, 1.0), snr_db=30.0,
                                    dtype=np.complex64)[0] for i, k in enumerate(ks)])
    ref_plan = A.Plan(1, n, "c64", seed=31, max_batch=2)
    ref = run_gpu(ref_plan, xs)
    monkeypatch.setenv("ATSFFT_MAIN_SLOTS", str(slots))
    plan = A.Plan(1, n, "c64", seed=31, max_batch=2)
    out = run_gpu(plan, xs)
    print("main slots", slots, [ref_plan.trace(ref["ws"], i, full=False)["B_star"] for i in range(2)], flush=True)
    for i in range(2):
        u, v = ref_plan.results(ref, i), plan.results(out, i)
        assert (u["count"], u["khat"], u["status"]) == (v["count"], v["khat"], v["status"])
        assert np.array_equal(u["locs"], v["locs"]) and np.array_equal(u["vals"], v["vals"])
        tu, tv = ref_plan.trace(ref["ws"], i), plan.trace(out["ws"], i)
        assert np.array_equal(tu["yhat"], tv["yhat"])


@pytest.mark.parametrize("one_slab", ["default", "0"])
def test_filter_factor_8_slab_forms(A, monkeypatch, one_slab):
    """At alpha = 8 the 1D main-loop hash of lengths up to 2^21 runs as one
    address slab (one partial per bucket); with ATSFFT_ONE_SLAB_MAX_N=0 as
    eight.  Both against the oracle, with a signal at 2^16 and one at 2^18."""
    if one_slab != "default":
        monkeypatch.setenv("ATSFFT_ONE_SLAB_MAX_N", one_slab)
    for n, k in ((1 << 16, 20), (1 << 18, 90)):
        plan = A.Plan(1, n, "c64", seed=41, max_batch=2, alpha=8, L_loc=7, L_est=7, T_vote=4, alpha_probe=8)
        xs = [synth.planted_1d(n, k, 960 + i, mag=("uniform", 0.5, 1.0), snr_db=35.0, dtype=np.complex64)[0]
              for i in range(2)]
        _check_batch(A, plan, xs, f"alpha 8 n={n} one_slab={one_slab}")


def test_probe_rounds_beyond_the_chip(A):
    """80 signals of 2^16: the first probe round (seven levels, 32 to 2048
    buckets) is a grid of 560 workgroups, more than two per CU, so it runs
    in 256-thread workgroups; every probe count, decision and the rest
    against the oracle."""
    import torch

    n = 1 << 16
    ks = [4, 9, 17, 33, 60, 120, 200, 333] * 10
    plan = A.Plan(1, n, "c64", seed=43, max_batch=len(ks))
    assert 7 * len(ks) > 2 * torch.cuda.get_device_properties(0).multi_processor_count
    xs = [synth.planted_1d(n, k, 1200 + i, mag=("uniform", 0.5, 1.0), snr_db=30.0, dtype=np.complex64)[0]
          for i, k in enumerate(ks)]
    _check_batch(A, plan, xs, "probe rounds beyond the chip")
