"""Host logic of the autotuner (no GPU): the search space is valid for the
library's validation, the touched-bytes prediction behaves, the selection
rule, and the JSON cache."""
import ctypes as C
import json
import math

import pytest

from paper_1908_02461_amd import atsfft as A
from paper_1908_02461_amd import autotune as T


@pytest.mark.parametrize("ndim,n", [(1, 1 << 14), (1, 1 << 22), (2, 4096)])
def test_every_candidate_passes_validation(ndim, n):
    lib = A.load()
    for kn in T.candidates(ndim):
        d = A.default_desc(ndim, n, "c64", **kn)
        h = C.c_void_p()
        st = lib.atsfft_plan(C.byref(h), C.byref(d))
        assert st != A.EINVAL, (kn, lib.atsfft_last_error())
        if h.value:
            lib.atsfft_destroy(h)


def test_touched_bytes_prediction():
    kn = dict(B0=32, alpha=32, L_loc=9, L_est=9, T_vote=5)
    n = 1 << 22
    full = 8.0 * n
    t = T.predicted_touched_bytes(1, n, "c64", 64, kn, B_max=16384)
    # B* = 2048, 18 loops of 65536 samples over 262144 lines: 1 - e^{-4.5}
    assert t == pytest.approx(full * (1 - math.exp(-4.5)), rel=1e-12)
    assert t < full
    small = T.predicted_touched_bytes(1, n, "c64", 64, dict(kn, alpha=16), B_max=16384)
    fewer = T.predicted_touched_bytes(1, n, "c64", 64, dict(kn, L_loc=7, L_est=7), B_max=16384)
    assert small < t and fewer < t
    # a tiny window over a long signal: one line per sample
    tiny = T.predicted_touched_bytes(1, 1 << 30, "c64", 4, dict(kn, alpha=2, L_loc=1, L_est=1), B_max=16384)
    assert tiny == pytest.approx(128 * 2 * 2 * 128, rel=1e-3)


def _m(ms, rec, err, tb=0.0, **kn):
    return T.Measured(dict(kn), ms, rec, err, tb)


def test_selection_rule():
    base = _m(1.0, 1.0, 1e-3, 100, alpha=32)
    fast_bad_rec = _m(0.5, 0.9, 1e-3, 50, alpha=16)
    fast_bad_err = _m(0.6, 1.0, 5e-3, 50, alpha=18)
    good = _m(0.7, 1.0, 1.2e-3, 80, alpha=24)
    near_leaner = _m(0.71, 1.0, 1.0e-3, 60, alpha=22)
    got = T.select([base, fast_bad_rec, fast_bad_err, good, near_leaner], base)
    assert got is near_leaner  # within 3 % of the fastest admissible, fewer bytes
    assert T.select([base, fast_bad_rec, fast_bad_err], base) is base
    # the recovery bar never exceeds what the defaults reach
    weak_base = _m(1.0, 0.95, 1e-3, alpha=32)
    assert T.select([weak_base, _m(0.5, 0.95, 1e-3, alpha=16)], weak_base).ms_per_transform == 0.5
    invalid = T.Measured(dict(alpha=3), 0.1, 1.0, 0.0, valid=False)
    assert T.select([base, invalid], base) is base


def test_cached_class_is_returned_without_measuring(tmp_path):
    path = str(tmp_path / "tune.json")
    key = T.class_key(1, 1 << 14, "c64", (4, 16), 40.0)
    assert key == "1d/n16384/c64/k4-16/snr40"
    entry = dict(key=key, knobs=dict(B0=16, alpha=24, L_loc=9, L_est=9, T_vote=5), ms_per_transform=0.01,
                 recovery=1.0, l1_vs_planted=1e-3, baseline_ms_per_transform=0.012, touched_bytes=1.0, tried=[])
    T.save_cache(path, {key: entry})
    r = T.tune(1, 1 << 14, "c64", (4, 16), 40.0, cache=path, device="cpu")
    assert r.knobs == entry["knobs"] and r.ms_per_transform == 0.01
    assert json.load(open(path))[key]["knobs"]["alpha"] == 24
    assert T.load_cache(str(tmp_path / "missing.json")) == {}
