"""The autotuner on the GPU: a small class, a three-candidate space, the
JSON cache, and a plan built from the winner."""
import numpy as np
import pytest

from paper_1908_02461_amd import synth

pytestmark = pytest.mark.gpu


def test_tune_small_class(tmp_path):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import autotune as T

    path = str(tmp_path / "tune.json")
    space = [dict(B0=32, alpha=16, L_loc=7, L_est=7, T_vote=4), dict(B0=16, alpha=24, L_loc=9, L_est=9, T_vote=5),
             dict(B0=64, alpha=32, L_loc=11, L_est=11, T_vote=6)]
    r = T.tune(1, 1 << 14, "c64", (4, 16), 40.0, batch=4, steps=2, cache=path, space=space)
    assert len(r.tried) == 4 and r.recovery >= 0.99 * min(t["recovery"] for t in r.tried[:1])
    assert r.knobs in space or r.knobs == {k: r.tried[0]["knobs"][k] for k in T.KNOBS}
    assert all(np.isfinite(t["ms_per_transform"]) for t in r.tried)
    print("tuned", r.key, r.knobs, r.ms_per_transform, "baseline", r.baseline_ms_per_transform, flush=True)
    again = T.tune(1, 1 << 14, "c64", (4, 16), 40.0, cache=path, space=[])
    assert again.knobs == r.knobs
    # the winner runs and recovers a fresh planted signal of the class
    plan = A.Plan(1, 1 << 14, "c64", seed=5, **r.knobs)
    x, locs, _ = synth.planted_1d(1 << 14, 10, 77, mag=("uniform", 0.5, 1.0), snr_db=40.0, dtype=np.complex64)
    out = plan.execute_batched(torch.from_numpy(x[None].copy()).cuda())
    res = plan.results(out, 0)
    assert np.isin(locs, res["locs"]).all()


def test_tune_uneven_batch():
    """tune_uneven on a small uneven batch: every candidate is measured on the
    call, the winner meets the selection rule against the defaults, and a plan
    built from it recovers the planted sets."""
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft as A
    from paper_1908_02461_amd import autotune as T

    ns = np.array([1 << 14, 1 << 16, 1 << 14, 1 << 15, 1 << 16, 1 << 14], np.int64)
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    x = torch.empty(int(ns.sum()), dtype=torch.complex64, device="cuda")
    truth = []
    for i, m in enumerate(ns):
        xi, locs, amps = synth.planted_1d_device(int(m), 6 + 2 * i, 900 + i, mag=("uniform", 0.5, 1.0), snr_db=40.0)
        x[offs[i]:offs[i] + m] = xi
        truth.append((locs, amps))
    space = [dict(B0=32, alpha=16, L_loc=7, L_est=7, T_vote=4), dict(B0=32, alpha=16, L_loc=9, L_est=9, T_vote=5)]
    r = T.tune_uneven(x, offs, ns, truth, n_max=1 << 16, n_min=1 << 14, seed=3, space=space, steps=2)
    assert len(r.tried) == 3 and all(t["valid"] for t in r.tried)
    base = r.tried[0]
    assert r.recovery >= min(0.99, base["recovery"]) and r.l1_vs_planted <= max(1.5 * base["l1_vs_planted"], 1e-6)
    print("tuned", r.key, r.knobs, r.ms_per_transform, "baseline", r.baseline_ms_per_transform, flush=True)
    plan = A.Plan(1, 1 << 16, "c64", seed=3, n_min=1 << 14, max_batch=len(ns), **r.knobs)
    out = plan.execute_uneven(x, offs, ns)
    for i in range(len(ns)):
        assert np.isin(truth[i][0], plan.results(out, i)["locs"]).all()
