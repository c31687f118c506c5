"""Pins of the oracle's residual test, an addition to the method (the paper
has no such check): the model of a loop's bucket DFT from the located values,
by Lemma 1 and the fold, against bucket DFTs computed by actually hashing the
signal those values define; a known perturbation; and the retry it drives.

Everything here runs on the CPU.
"""
import numpy as np
import pytest

from paper_1908_02461_amd import synth


def _sparse_signal(rng, ndim, n, k):
    total = n if ndim == 1 else n * n
    locs = np.sort(rng.choice(total, size=k, replace=False)).astype(np.int64)
    vals = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    X = np.zeros(total, np.complex128)
    X[locs] = vals
    x = np.fft.ifft(X) if ndim == 1 else np.fft.ifft2(X.reshape(n, n))
    return x, locs, vals


def _hashed_loops(orc, x, ndim, n, B, w, G, L, seed):
    ys, sig, tau = [], [], []
    for l in range(L):
        if ndim == 1:
            s, t, _ = orc.draw(seed, 0, orc.PHASE_EST, l, 0, n)
            ys.append(orc.hash_1d(x, s, t, B, w, G))
            sig.append(s)
            tau.append(t)
        else:
            d = [orc.draw(seed, 0, orc.PHASE_EST, l, a, n) for a in range(2)]
            s, t = [d[0][0], d[1][0]], [d[0][1], d[1][1]]
            ys.append(orc.hash_2d(x, s, t, B, w, G).ravel())
            sig.append(s)
            tau.append(t)
    return np.array(ys), np.array(sig), np.array(tau)


@pytest.mark.parametrize("ndim,n,B,k,alpha", [(1, 1 << 12, 64, 20, 32), (1, 1 << 14, 256, 40, 32),
                                               (1, 1 << 12, 64, 20, 16), (2, 128, 16, 12, 8), (2, 256, 16, 20, 8)])
def test_model_reproduces_hashed_buckets(orc, ndim, n, B, k, alpha):
    """For the exact values of a k-sparse spectrum the model leaves only the
    window's response beyond its reach: E_res / E_tot below 1e-10 at
    delta = 1e-8, against bucket DFTs computed by hashing the signal."""
    rng = np.random.default_rng(ndim * 100 + k + alpha)
    x, locs, vals = _sparse_signal(rng, ndim, n, k)
    delta = 1e-8
    w = orc.window_len(n, B, alpha)
    G = orc.window_taps(n, B, w, delta)
    R = orc.residual_reach(alpha, delta)
    ys, sig, tau = _hashed_loops(orc, x, ndim, n, B, w, G, 5, seed=3)
    er, et = orc.residual(ndim, n, B, w, G, sig, tau, ys, locs, vals, R)
    assert et > 0
    assert er / et < 1e-10, er / et
    # a reach one bucket short leaves part of the transition band out
    er1, _ = orc.residual(ndim, n, B, w, G, sig, tau, ys, locs, vals, R - 1)
    assert er1 > 100 * er and er1 / et > 1e-12, (er1 / et, er / et)


def test_reach_covers_the_transition_band(orc):
    """R = ceil(2 ln(1/delta) / (pi alpha)): 1 for alpha = 32 and 16, 2 for 8
    at delta = 1e-8; the window's response at (R + 1/2) n/B is near delta and
    at (R - 1/2) n/B, where bucket R begins, it is not."""
    assert [orc.residual_reach(a, 1e-8) for a in (32, 16, 8)] == [1, 1, 2]
    assert orc.residual_reach(32, 1e-6) == 1
    for n, B, alpha in ((1 << 12, 64, 32), (1 << 12, 64, 16), (1024, 32, 8)):
        w = orc.window_len(n, B, alpha)
        G = orc.window_taps(n, B, w, 1e-8)
        R = orc.residual_reach(alpha, 1e-8)
        nb = n // B
        assert abs(orc.window_hat(n, w, G, (2 * R + 1) * nb // 2)) < 1e-6
        assert abs(orc.window_hat(n, w, G, (2 * R - 1) * nb // 2)) > 1e-6


def test_known_perturbation(orc):
    """Changing one modelled value by D adds |D|^2 sum_l sum_b G'(q_b)^2 over
    the buckets the model gives that frequency (own bucket +- R)."""
    n, B, k = 1 << 12, 64, 10
    rng = np.random.default_rng(7)
    x, locs, vals = _sparse_signal(rng, 1, n, k)
    w = orc.window_len(n, B, 32)
    G = orc.window_taps(n, B, w, 1e-8)
    ys, sig, tau = _hashed_loops(orc, x, 1, n, B, w, G, 3, seed=11)
    D = 0.3 - 0.2j
    v2 = vals.copy()
    v2[4] += D
    R = orc.residual_reach(32, 1e-8)
    er0, _ = orc.residual(1, n, B, w, G, sig, tau, ys, locs, vals, R)
    er1, _ = orc.residual(1, n, B, w, G, sig, tau, ys, locs, v2, R)
    f = int(locs[4])
    expect = 0.0
    for l in range(3):
        o = orc.hash_offset(n, B, int(sig[l]), f)
        expect += sum(orc.window_hat(n, w, G, o + j * (n // B)) ** 2 for j in range(-R, R + 1))
    expect *= abs(D) ** 2
    assert er1 - er0 == pytest.approx(expect, rel=1e-6, abs=1e-12)


def test_ratio_matches_trace_and_off_by_default(orc):
    """The driver's reported ratio is or_residual on its own estimation loops;
    with the test off (the default) the ratio is 0 and nothing re-runs."""
    n, k = 1 << 12, 6
    x = synth.planted_1d(n, k, 5, mag=("uniform", 0.5, 1.0), snr_db=30.0)[0]
    p = orc.Params.defaults(1, n, seed=9, B_max=128)
    assert p.res_tol == 0.0
    r0 = orc.atsfft(x, p)
    assert r0["res_ratio"] == 0.0 and r0["retries"] == 0 and not r0["status"] & orc.RETRIED
    p.res_tol = 0.5  # on, but far above the noise: no re-run
    r1 = orc.atsfft(x, p)
    assert r1["retries"] == 0 and np.array_equal(r1["locs"], r0["locs"])
    assert 0 < r1["res_ratio"] < 0.5
    B = r1["B_star"]
    w = orc.window_len(n, B, p.alpha)
    G = orc.window_taps(n, B, w, p.delta)
    sig = [orc.draw(p.seed, 0, orc.PHASE_EST, l, 0, n)[0] for l in range(p.L_est)]
    tau = [orc.draw(p.seed, 0, orc.PHASE_EST, l, 0, n)[1] for l in range(p.L_est)]
    er, et = orc.residual(1, n, B, w, G, sig, tau, r1["yhat"][p.L_loc:], r1["locs"], r1["vals"],
                          orc.residual_reach(p.alpha, p.delta))
    assert er / et == pytest.approx(r1["res_ratio"], rel=1e-12)


def test_retry_recovers_what_a_small_bucket_count_missed(orc):
    """Algorithm 1 form at a bucket count too small for k (collisions lose
    frequencies): the residual flags it, location and estimation re-run at
    2B with fresh draws, and the planted set is recovered."""
    n, k = 1 << 14, 24
    x, plocs, _ = synth.planted_1d(n, k, 21, mag=("uniform", 0.5, 1.0))
    base = dict(seed=4, fixed_B=32, fixed_k=k, B_max=256)
    r0 = orc.atsfft(x, orc.Params.defaults(1, n, **base))
    assert r0["status"] & orc.TRUNCATED and not r0["status"] & orc.RETRIED
    r1 = orc.atsfft(x, orc.Params.defaults(1, n, res_tol=1e-3, res_retries=3, **base))
    assert r1["status"] & orc.RETRIED and r1["retries"] >= 1
    assert r1["B_star"] == 32 << r1["retries"]
    assert np.isin(plocs, r1["locs"]).all()
    assert r1["res_ratio"] <= 1e-3
    # one re-run allowed: B doubles once; that pass is still truncated, which
    # counts as an infinite ratio
    r2 = orc.atsfft(x, orc.Params.defaults(1, n, res_tol=1e-3, res_retries=1, **base))
    assert r2["retries"] == 1 and r2["B_star"] == 64
    assert r2["status"] & orc.TRUNCATED and r2["res_ratio"] == float("inf")


def test_retry_stops_at_the_bucket_cap(orc):
    n, k = 1 << 12, 24
    x = synth.planted_1d(n, k, 3)[0]
    r = orc.atsfft(x, orc.Params.defaults(1, n, seed=1, fixed_B=32, fixed_k=k, B_max=64, res_tol=1e-9,
                                          res_retries=5))
    assert r["B_star"] <= 64 and r["retries"] <= 1


def test_residual_parameters_validated(orc):
    n = 1 << 10
    x = np.zeros(n, np.complex128)
    for bad in (dict(res_tol=-1.0), dict(res_retries=8), dict(res_retries=-1)):
        with pytest.raises(ValueError):
            orc.atsfft(x, orc.Params.defaults(1, n, **bad))
