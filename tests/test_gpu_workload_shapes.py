"""GPU parity at the shapes of the uneven-batch and forward + adjoint
workloads.

Uneven batch: signals of the batched workload's recipe (n = 2^e, e in
16..22, k log-uniform in [4, 1024], SNR uniform in [20, 60] dB, magnitudes
uniform in [0.5, 1]) under the knobs the benchmark tunes on it (alpha = 8,
7 location and 7 estimation loops, vote threshold 4, probe filter factor 8),
each against the oracle at its own length; saturated, truncated and
failed-probe signals included.

Forward + adjoint: a batch of n = 2^20, k = 128, 40 dB signals; the
gradient of sum |X_hat(located) - target|^2 against FP64 central differences
of the oracle's loss on two of them, and the adjoint gather's grid stride
(workgroups capped at a few per signal) against the default launch.
"""
import numpy as np
import pytest

import oracle
from paper_1908_02461_amd import synth

from parity_util import VAL_TOL, oracle_params, sub_params, value_rel_err

pytestmark = pytest.mark.gpu

# signals of the batched workload's draws (generator PCG64(4242), 512 signals):
# for each length the largest and the smallest k
C4_PICK = (377, 102, 115, 142, 353, 253, 133, 0, 3, 67, 36, 147, 98, 96)
C4_KNOBS = dict(alpha=8, L_loc=7, L_est=7, T_vote=4, alpha_probe=8, B0=32)


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _c4_recipe():
    rng = np.random.Generator(np.random.PCG64(4242))
    ns = (1 << rng.integers(16, 23, size=512)).astype(np.int64)
    ks = np.rint(np.exp(rng.uniform(np.log(4), np.log(1024), size=512))).astype(np.int64)
    snrs = rng.uniform(20.0, 60.0, size=512)
    return ns, ks, snrs


def test_uneven_batch_at_tuned_knobs(A):
    import torch

    ns_all, ks_all, snr_all = _c4_recipe()
    ns = [int(ns_all[i]) for i in C4_PICK]
    xs = [synth.planted_1d(int(ns_all[i]), int(ks_all[i]), 3000 + i, mag=("uniform", 0.5, 1.0),
                           snr_db=float(snr_all[i]), dtype=np.complex64)[0] for i in C4_PICK]
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    packed = np.concatenate(xs)
    plan = A.Plan(1, 1 << 22, "c64", seed=11, n_min=1 << 16, max_batch=len(ns), max_out=16384, **C4_KNOBS)
    print(f"uneven tuned knobs: {len(ns)} signals, n 2^16..2^22", flush=True)
    out = plan.execute_uneven(torch.from_numpy(packed).cuda(), offs, ns)
    torch.cuda.synchronize()
    sat = trunc = 0
    for i, (x, m) in enumerate(zip(xs, ns)):
        res = plan.results(out, i)
        ref = oracle.atsfft(x.astype(np.complex128), sub_params(plan.desc, m, i), trace=False)
        label = (i, C4_PICK[i], m, res["status"], ref["status"])
        assert res["status"] == ref["status"] and res["khat"] == ref["khat"], label
        assert res["count"] == ref["count"], (label, res["count"], ref["count"])
        assert np.array_equal(res["locs"], ref["locs"]), label
        err = value_rel_err(res["vals"], ref["vals"], "c64")
        assert err < VAL_TOL["c64"], (label, err)
        sat += bool(res["status"] & A.SIG_PROBE_SATURATED)
        trunc += bool(res["status"] & A.SIG_TRUNCATED)
        print(f"  signal {C4_PICK[i]} n=2^{m.bit_length() - 1} |S|={res['count']} status={res['status']} "
              f"rel err {err:.2e}", flush=True)
    assert sat >= 2 and trunc >= 1


def _medians(est):
    out = []
    for row in est:
        mr, mi = np.median(row.real), np.median(row.imag)
        out.append((int(np.flatnonzero(row.real == mr)[0]), int(np.flatnonzero(row.imag == mi)[0])))
    return out


def _forward_backward(A, plan, x, targets):
    import torch

    xd = torch.from_numpy(x.copy()).cuda().requires_grad_(True)
    vals, locs, count, khat, status = A.sparse_fft(xd, plan)
    mask = torch.arange(plan.max_out, device="cuda")[None, :] < count[:, None]
    loss = torch.sum(torch.abs(vals - targets) ** 2 * mask)
    loss.backward()
    torch.cuda.synchronize()
    return xd.grad.cpu().numpy().astype(np.complex128), locs.cpu().numpy(), count.cpu().numpy()


def test_adjoint_at_forward_adjoint_shape(A, monkeypatch):
    import torch

    n, k, batch = 1 << 20, 128, 4
    x = np.stack([synth.planted_1d(n, k, 5000 + i, mag=("uniform", 0.5, 1.0), snr_db=40.0,
                                   dtype=np.complex64)[0] for i in range(batch)])
    plan = A.Plan(1, n, "c64", seed=13, max_batch=batch)
    rng = np.random.default_rng(77)
    tg = (rng.standard_normal((batch, plan.max_out)) + 1j * rng.standard_normal((batch, plan.max_out)))
    targets = torch.from_numpy(tg.astype(np.complex64)).cuda()
    print(f"forward + adjoint: batch {batch} n=2^20 k={k}", flush=True)
    grad, locs, count = _forward_backward(A, plan, x, targets)

    # the gather's grid stride: at most 3 workgroups per signal instead of 64
    monkeypatch.setenv("ATSFFT_GATHER_BLOCKS", "3")
    plan3 = A.Plan(1, n, "c64", seed=13, max_batch=batch)
    monkeypatch.delenv("ATSFFT_GATHER_BLOCKS")
    grad3, locs3, count3 = _forward_backward(A, plan3, x, targets)
    assert np.array_equal(count3, count) and np.array_equal(locs3, locs)
    scale = np.max(np.abs(grad))
    # only the bucket cotangents of colliding frequencies add in varying order
    assert np.max(np.abs(grad3 - grad)) <= 1e-5 * scale

    # FP64 central differences of the oracle's loss on two signals
    for s in (0, 2):
        cnt = int(count[s])
        assert cnt > 0
        p = oracle_params(plan, s)
        x64 = x[s].astype(np.complex128)
        r0 = oracle.atsfft(x64, p, trace=True)
        assert np.array_equal(r0["locs"], locs[s, :cnt])
        med = _medians(r0["est"])
        t = tg[s, :cnt].astype(np.complex64).astype(np.complex128)
        rms = float(np.sqrt(np.mean(np.abs(x64) ** 2)))
        for trial in range(2):
            v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
            # the loss is quadratic only while the located set and the median
            # choices stay put: estimates of two loops can lie within 1e-6 of
            # each other here, so the step shrinks until no decision moves
            # (central differences of this loss agree to 3e-5 or better down
            # to 1e-10 rms in FP64)
            for rel in (1e-8, 1e-9, 1e-10):
                eps = rel * rms
                lo, same = [], True
                for sign in (1, -1):
                    r = oracle.atsfft(x64 + sign * eps * v, p, trace=True)
                    same = same and np.array_equal(r["locs"], r0["locs"]) and _medians(r["est"]) == med
                    lo.append(float(np.sum(np.abs(r["vals"] - t) ** 2)))
                if same:
                    break
            assert same, (s, trial, "a decision moved at every step size")
            fd = (lo[0] - lo[1]) / (2 * eps)
            an = float(np.sum(grad[s].real * v.real + grad[s].imag * v.imag))
            scale_s = float(np.sum(np.abs(grad[s]) * np.abs(v)))
            print(f"  signal {s} trial {trial}: adjoint {an:.6e} central difference {fd:.6e}", flush=True)
            assert abs(an - fd) <= 2e-3 * max(abs(fd), 1e-3 * scale_s), (s, trial, an, fd)
