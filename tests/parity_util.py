"""Helpers shared by the GPU parity tests: run the library and the oracle on
the same input with the same knobs and compare them to the stated bar."""
from __future__ import annotations

import numpy as np

import oracle
from paper_1908_02461_amd import atsfft as A

# value tolerance of the parity bar: relative, with the denominator
# max(|X_oracle(f)|, floor * max_g |X_oracle(g)|).  The floor is where the
# relative bar becomes attainable in the plan's arithmetic: an estimate comes
# out of a B-point FFT of the folded buckets, whose error per entry is
# sqrt(log2 B) to log2 B unit roundoffs of the largest bucket value (about
# max |X| over G'), so in FP32 (unit roundoff 6e-8, B <= 2^14) values below
# about 1e-2 max |X| carry absolute errors of 1e-7 to 1e-6 max |X|, which
# 1e-4 of them cannot cover; in FP64 the same argument leaves 1e-3 ample.
VAL_TOL = {"c64": 1e-4, "c128": 1e-10}
VAL_FLOOR = {"c64": 1e-2, "c128": 1e-3}
# bound on the error of a bucket DFT value, relative to the largest |y_hat|
# of its loop: FP32 fold of up to 2^10 products plus a 2^14-point DFT, and the
# FP64 path
YHAT_TOL = {"c64": 2e-5, "c128": 1e-12}


def oracle_params(plan: A.Plan, signal: int = 0) -> oracle.Params:
    d = plan.desc
    fixed = bool(d.flags & A.FLAG_FIXED_B)
    return oracle.Params(
        ndim=d.ndim, n=d.n, B0=d.B0, B_max=d.B_max, alpha_probe=d.alpha_probe, alpha=d.alpha,
        L_loc=d.L_loc, L_est=d.L_est, T_vote=d.T_vote, P_max=d.P_max, d=d.d, gamma=d.gamma,
        delta=d.delta, q=d.q, noise_rate=d.noise_rate, rho=d.rho, seed=d.seed, signal=signal,
        fixed_B=d.fixed_B if fixed else 0, fixed_k=d.fixed_k if fixed else 0, max_out=d.max_out,
        res_tol=d.res_tol, res_retries=d.res_retries,
    )


def sub_params(d, m: int, signal: int) -> oracle.Params:
    """The oracle knobs of an uneven plan's table for length m (B0 and B_max
    clipped to m as the library documents) and the signal's index in the call."""
    B_max = min(d.B_max, max(m // d.alpha, 1))
    B_max = max(B_max, 2 if d.ndim == 1 else 4)
    B0 = min(d.B0, B_max)
    return oracle.Params(
        ndim=d.ndim, n=m, B0=B0, B_max=B_max, alpha_probe=d.alpha_probe, alpha=d.alpha, L_loc=d.L_loc,
        L_est=d.L_est, T_vote=d.T_vote, P_max=d.P_max, d=d.d, gamma=d.gamma, delta=d.delta, q=d.q,
        noise_rate=d.noise_rate, rho=d.rho, seed=d.seed, signal=signal, max_out=d.max_out)


def value_rel_err(got: np.ndarray, ref: np.ndarray, dtype: str) -> float:
    if ref.size == 0:
        return 0.0
    den = np.maximum(np.abs(ref), VAL_FLOOR[dtype] * np.max(np.abs(ref)))
    return float(np.max(np.abs(got - ref) / den))


def compare(plan: A.Plan, res: dict, tr: dict, ref: dict, label: str = "") -> dict:
    """Assert GPU == oracle for one signal; return the measured errors."""
    dt = plan.dtype
    info = {}
    # probe: every discrete decision identical
    assert tr["probe_B"] == ref["probe_B"], (label, tr["probe_B"], ref["probe_B"])
    assert tr["probe_k"] == ref["probe_k"], (label, tr["probe_k"], ref["probe_k"])
    assert tr["probe_decision"] == ref["probe_decision"], label
    assert tr["B_star"] == ref["B_star"] and tr["khat"] == ref["khat"], (label, tr["B_star"], ref["B_star"])
    assert res["status"] == ref["status"], (label, res["status"], ref["status"])
    assert res["khat"] == ref["khat"]
    assert res["count"] == ref["count"], (label, res["count"], ref["count"])
    if ref["status"] & oracle.EMPTY:
        return info
    # bucket DFTs of every location and estimation loop
    yr = ref["yhat"]
    yg = tr["yhat"]
    assert yg.shape == yr.shape
    scale = np.max(np.abs(yr), axis=1, keepdims=True)
    yerr = float(np.max(np.abs(yg - yr) / scale))
    info["yhat_rel"] = yerr
    assert yerr < YHAT_TOL[dt], (label, yerr)
    # cutoffs: identical except where the oracle's value sits within the
    # bucket-value error of the decision boundary
    L_loc = plan.desc.L_loc
    num = min(plan.desc.d * ref["khat"], yr.shape[1])
    flips = 0
    for l in range(L_loc):
        m = np.abs(yr[l]) ** 2
        diff = tr["J"][l] != ref["J"][l]
        if not diff.any():
            continue
        T = ref["T_loc"][l]
        above = np.sort(m[m > T])[::-1]
        cut = above[num - 1] if above.size > num else T
        eps = YHAT_TOL[dt] * scale[l, 0]
        margin = 2 * np.sqrt(m) * eps + eps * eps
        ok = (np.abs(m - T) <= margin + 1e-6 * T) | (np.abs(m - cut) <= margin + 1e-6 * cut)
        assert np.all(ok[diff]), (label, l, np.flatnonzero(diff & ~ok)[:5])
        flips += int(diff.sum())
    info["J_margin_flips"] = flips
    # located set: identical
    assert np.array_equal(res["locs"], ref["locs"]), (label, np.setxor1d(res["locs"], ref["locs"])[:10])
    rel = value_rel_err(res["vals"], ref["vals"], dt)
    info["vals_rel"] = rel
    assert rel < VAL_TOL[dt], (label, rel)
    return info


def run_gpu(plan: A.Plan, x_batch: np.ndarray):
    import torch

    xd = torch.from_numpy(np.ascontiguousarray(x_batch)).to("cuda")
    out = plan.execute_batched(xd)
    torch.cuda.synchronize()
    return out
