"""GPU parity of 2D bucket arrays above the LDS-resident size: the known-k
form (Algorithm 1: B and k given, no probe) at the sparse FFT's bucket count
B = sqrt(N k) per axis (Sec. III-A), where B x B runs from 65536 to 2^20
buckets and the bucket DFTs, thresholds and cutoffs run in device memory, and
the adaptive form (Algorithm 2) with B_max above the LDS size, whose large
probe levels (local maxima and the B-update rule) and main loops take the
same device-memory path while the small ones stay in LDS.  Every decision
(probe counts and decisions, cutoff bits, located set) and the bucket DFTs
and values are compared with the oracle on identical draws, as in
test_gpu_parity."""
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


@pytest.mark.parametrize("N,k,dt,snr,batch", [(1024, 64, "c64", 30.0, 2), (1024, 64, "c128", None, 1),
                                              (2048, 128, "c64", 30.0, 1)])
def test_large_bucket_arrays_match_oracle(A, N, k, dt, snr, batch):
    B = int(round(np.sqrt(N * k)))
    assert B & (B - 1) == 0 and B * B > 16384
    npdt = np.complex64 if dt == "c64" else np.complex128
    mag = ("loguniform", 0.1, 1.0) if snr is not None else None
    plan = A.Plan(2, N, dt, seed=21, max_batch=batch, fixed_B=B, fixed_k=k)
    xs = [synth.planted_2d(N, k, 400 + i, mag=mag, snr_db=snr, dtype=npdt)[0] for i in range(batch)]
    print(f"large 2D bucket arrays: N={N} k={k} B={B} {dt} batch {batch}", flush=True)
    out = run_gpu(plan, np.stack(xs))
    for i, x in enumerate(xs):
        res = plan.results(out, i)
        tr = plan.trace(out["ws"], i)
        ref = oracle.atsfft(x.astype(np.complex128), oracle_params(plan, i), trace=True)
        info = compare(plan, res, tr, ref, f"big2d N={N} B={B} [{i}]")
        print("  ", info, "|S|", res["count"], flush=True)
        if snr is None:
            # noiseless planted spectrum: every planted frequency located
            locs = synth.planted_2d(N, k, 400 + i)[1]
            assert np.all(np.isin(locs, res["locs"])), i


# (N, k per signal, dtype, SNR, B_max): at gamma = 32 the probe acts on a
# count only once B^2 >= 32 k, so k = 800 at N = 2048 and k = 200 at N = 1024
# reach levels above the LDS size (c64 holds up to 128 x 128 there, c128 up
# to 64 x 64); the k = 12 signal of the first batch stops in LDS, so one
# batch runs both kinds of main loop
@pytest.mark.parametrize("N,ks,dt,snr,Bmax", [(2048, (800, 12), "c64", 30.0, 512),
                                              (1024, (200,), "c128", None, 256)])
def test_probe_beyond_lds_matches_oracle(A, N, ks, dt, snr, Bmax):
    npdt = np.complex64 if dt == "c64" else np.complex128
    mag = ("loguniform", 0.1, 1.0) if snr is not None else None
    plan = A.Plan(2, N, dt, seed=33, max_batch=len(ks), B_max=Bmax)
    xs = [synth.planted_2d(N, k, 500 + i, mag=mag, snr_db=snr, dtype=npdt)[0] for i, k in enumerate(ks)]
    print(f"probed 2D plan beyond the LDS size: N={N} k={ks} B_max={Bmax} {dt}", flush=True)
    out = run_gpu(plan, np.stack(xs))
    lds_side = 128 if dt == "c64" else 64
    for i, (x, k) in enumerate(zip(xs, ks)):
        res = plan.results(out, i)
        tr = plan.trace(out["ws"], i)
        ref = oracle.atsfft(x.astype(np.complex128), oracle_params(plan, i), trace=True)
        info = compare(plan, res, tr, ref, f"probe2d N={N} k={k} [{i}]")
        print("  ", info, "B*", tr["B_star"], "probe", tr["probe_B"], tr["probe_k"], "|S|", res["count"], flush=True)
        assert (tr["B_star"] > lds_side) == (k >= 200), (k, tr["B_star"])
        if snr is None:
            locs = synth.planted_2d(N, k, 500 + i)[1]
            assert np.all(np.isin(locs, res["locs"])), i


def test_large_bucket_plan_limits(A):
    import torch

    d = dict(fixed_B=256, fixed_k=16)
    for bad in (dict(res_tol=0.1, B_max=128), dict(compensated=True), dict(alpha=16)):
        with pytest.raises(A.AtsfftError) as e:
            A.Plan(2, 1024, "c64", **d, **bad)
        assert e.value.status == A.EINVAL, bad
    for big in (dict(fixed_B=2048, fixed_k=16), dict(B_max=2048)):  # above 1024 per axis
        with pytest.raises(A.AtsfftError) as e:
            A.Plan(2, 4096, "c64", **big)
        assert e.value.status == A.EINVAL
    plan = A.Plan(2, 1024, "c64", seed=2, **d)
    x = torch.from_numpy(synth.planted_2d(1024, 16, 9, dtype=np.complex64)[0][None].copy()).cuda()
    out = plan.execute_batched(x)
    g = torch.zeros((1, plan.max_out), dtype=torch.complex64, device="cuda")
    gx = torch.empty_like(x)
    with pytest.raises(A.AtsfftError) as e:
        plan.backward(g, out["ws"], gx)
    assert e.value.status == A.ENOTSUPPORTED
