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
