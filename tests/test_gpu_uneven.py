"""GPU parity of uneven batches (atsfft_execute_uneven): signals of different
lengths packed in one buffer, each compared with the oracle at its own length,
with its index in the call as its draw key."""
import numpy as np
import pytest

import oracle
from paper_1908_02461_amd import synth

from parity_util import VAL_TOL, sub_params, value_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


@pytest.mark.parametrize("dt", ["c128", "c64"])
def test_uneven_lengths_match_oracle(A, dt):
    import torch

    ns = [1 << 12, 1 << 14, 1 << 13, 1 << 12, 1 << 14, 1 << 15, 1 << 13]
    ks = [2, 8, 4, 3, 6, 10, 1]
    npdt = np.complex64 if dt == "c64" else np.complex128
    mag = ("uniform", 0.5, 1.0) if dt == "c64" else None
    snr = 35.0 if dt == "c64" else None
    xs = [synth.planted_1d(m, k, 50 + i, mag=mag, snr_db=snr, dtype=npdt)[0] for i, (m, k) in enumerate(zip(ns, ks))]
    gap = 5  # signals need not be adjacent
    offs, pos = [], 0
    for x in xs:
        offs.append(pos)
        pos += x.size + gap
    packed = np.zeros(pos, dtype=npdt)
    for o, x in zip(offs, xs):
        packed[o:o + x.size] = x
    plan = A.Plan(1, 1 << 15, dt, seed=31, n_min=1 << 12, max_batch=len(ns))
    out = plan.execute_uneven(torch.from_numpy(packed).cuda(), offs, ns)
    torch.cuda.synchronize()
    for i, (x, m) in enumerate(zip(xs, ns)):
        res = plan.results(out, i)
        ref = oracle.atsfft(x.astype(np.complex128), sub_params(plan.desc, m, i), trace=False)
        assert res["status"] == ref["status"] and res["khat"] == ref["khat"], (i, res["status"], ref["status"])
        assert res["count"] == ref["count"], (i, res["count"], ref["count"])
        assert np.array_equal(res["locs"], ref["locs"]), i
        assert value_rel_err(res["vals"], ref["vals"], dt) < VAL_TOL[dt], i


def test_uneven_rejects_uncovered_length(A):
    import torch

    plan = A.Plan(1, 1 << 14, "c64", seed=1, n_min=1 << 12, max_batch=2)
    x = torch.zeros(1 << 16, dtype=torch.complex64, device="cuda")
    with pytest.raises(A.AtsfftError):
        plan.execute_uneven(x, [0, 4096], [1 << 11, 1 << 12])
    with pytest.raises(A.AtsfftError):
        plan.execute_uneven(x, [0, 4096], [1 << 15, 1 << 12])
