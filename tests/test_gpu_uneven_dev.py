"""GPU checks of atsfft_execute_uneven_dev: an uneven 1D batch whose lengths
and offsets are device arrays runs as one fixed launch sequence (every signal
with the parameters of its own length), gives what the host-grouped uneven
execute gives, matches the oracle signal by signal, flags lengths the plan
does not cover, and replays from HIP graphs (the library's and a caller's)."""
import numpy as np
import pytest

import oracle
from paper_1908_02461_amd import synth

from parity_util import VAL_TOL, sub_params, value_rel_err
from test_gpu_workload_shapes import C4_KNOBS, C4_PICK, _c4_recipe

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _c4_batch():
    ns_all, ks_all, snr_all = _c4_recipe()
    ns = np.array([int(ns_all[i]) for i in C4_PICK], dtype=np.int64)
    xs = [synth.planted_1d(int(ns_all[i]), int(ks_all[i]), 3000 + i, mag=("uniform", 0.5, 1.0),
                           snr_db=float(snr_all[i]), dtype=np.complex64)[0] for i in C4_PICK]
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    return xs, ns, offs


def _same_outputs(a, b, batch, label):
    for key in ("count", "khat", "status"):
        assert np.array_equal(a[key].cpu().numpy()[:batch], b[key].cpu().numpy()[:batch]), (label, key)
    for i in range(batch):
        c = int(a["count"][i])
        if c > a["locs"].shape[1] or int(a["status"][i]) & 1:
            continue
        assert np.array_equal(a["locs"][i, :c].cpu().numpy(), b["locs"][i, :c].cpu().numpy()), (label, i)
        assert np.array_equal(a["vals"][i, :c].cpu().numpy(), b["vals"][i, :c].cpu().numpy()), (label, i)


def test_device_lengths_match_grouped_execute_and_oracle(A):
    import torch

    xs, ns, offs = _c4_batch()
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    plan = A.Plan(1, 1 << 22, "c64", seed=11, n_min=1 << 16, max_batch=len(ns), max_out=16384, **C4_KNOBS)
    print(f"device-length uneven call: {len(ns)} signals", flush=True)
    dev = plan.execute_uneven_dev(x, torch.from_numpy(offs).cuda(), torch.from_numpy(ns).cuda())
    grp = plan.execute_uneven(x, offs, ns)
    torch.cuda.synchronize()
    _same_outputs(dev, grp, len(ns), "device vs grouped")
    for i, (xi, m) in enumerate(zip(xs, ns)):
        res = plan.results(dev, i)
        ref = oracle.atsfft(xi.astype(np.complex128), sub_params(plan.desc, int(m), i), trace=False)
        assert (res["status"], res["khat"], res["count"]) == (ref["status"], ref["khat"], ref["count"]), i
        assert np.array_equal(res["locs"], ref["locs"]), i
        assert value_rel_err(res["vals"], ref["vals"], "c64") < VAL_TOL["c64"], i


def test_uncovered_lengths_are_flagged(A):
    import torch

    n_max = 1 << 16
    plan = A.Plan(1, n_max, "c64", seed=3, n_min=1 << 12, max_batch=6)
    good = [(1 << 14, 6), (1 << 12, 3), (1 << 16, 10)]
    xs = [synth.planted_1d(m, k, 90 + i, mag=("uniform", 0.5, 1.0), snr_db=40.0, dtype=np.complex64)[0]
          for i, (m, k) in enumerate(good)]
    # signals 1, 3 and 5 have lengths the plan does not cover (not a power of
    # two, below n_min, above n); their offsets point inside x all the same
    ns = np.array([1 << 14, 3000, 1 << 12, 1 << 11, 1 << 16, 1 << 17], dtype=np.int64)
    offs = np.array([0, 0, 1 << 14, 0, (1 << 14) + (1 << 12), 0], dtype=np.int64)
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    print("device-length uneven call with uncovered lengths", flush=True)
    out = plan.execute_uneven_dev(x, torch.from_numpy(offs).cuda(), torch.from_numpy(ns).cuda())
    torch.cuda.synchronize()
    for i in (1, 3, 5):
        r = plan.results(out, i)
        assert r["status"] == A.SIG_BAD_LENGTH | A.SIG_EMPTY and r["count"] == 0 and r["khat"] == 0, (i, r)
    ref = plan.execute_uneven(x, offs[[0, 2, 4]], ns[[0, 2, 4]])
    torch.cuda.synchronize()
    for j, i in enumerate((0, 2, 4)):
        a, b = plan.results(out, i), plan.results(ref, j)
        # signal keys are call indices: signal i here is signal j there, so
        # compare each with the oracle under its own key instead
        p = sub_params(plan.desc, int(ns[i]), i)
        o = oracle.atsfft(xs[j].astype(np.complex128), p, trace=False)
        assert np.array_equal(a["locs"], o["locs"]) and a["status"] == o["status"], i
        assert value_rel_err(a["vals"], o["vals"], "c64") < VAL_TOL["c64"], i
        assert b["status"] == 0


def _rewrite(x, xs, scale):
    import torch

    x.copy_(torch.from_numpy(np.concatenate(xs) * np.complex64(scale)).cuda())


@pytest.mark.parametrize("how", ["library", "caller"])
def test_graph_replays_match_eager(A, how):
    import torch

    n_max = 1 << 16
    ks = [(1 << 16, 12), (1 << 13, 4), (1 << 15, 30), (1 << 14, 8), (1 << 16, 5)]
    xs = [synth.planted_1d(m, k, 120 + i, mag=("uniform", 0.5, 1.0), snr_db=35.0, dtype=np.complex64)[0]
          for i, (m, k) in enumerate(ks)]
    ns = torch.tensor([m for m, _ in ks], dtype=torch.int64, device="cuda")
    offs = torch.tensor(np.concatenate([[0], np.cumsum([m for m, _ in ks])[:-1]]), dtype=torch.int64, device="cuda")
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    eager = A.Plan(1, n_max, "c64", seed=8, n_min=1 << 13, max_batch=len(ks))
    plan = A.Plan(1, n_max, "c64", seed=8, n_min=1 << 13, max_batch=len(ks), graph=(how == "library"))
    out = plan.outputs(len(ks), x.device)
    ws = torch.empty(plan.workspace_size_uneven_dev(len(ks)), dtype=torch.uint8, device="cuda")
    print(f"graph replay ({how})", flush=True)
    if how == "caller":
        plan.execute_uneven_dev(x, offs, ns, out=out, ws=ws)  # warm up outside the capture
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            plan.execute_uneven_dev(x, offs, ns, out=out, ws=ws)
        run = g.replay
    else:
        run = lambda: plan.execute_uneven_dev(x, offs, ns, out=out, ws=ws)
    for rep, scale in enumerate((1.0, 0.5, 2.0, 1.0)):
        _rewrite(x, xs, scale)
        run()
        torch.cuda.synchronize()
        ref = eager.execute_uneven_dev(x, offs, ns)
        torch.cuda.synchronize()
        _same_outputs(out, ref, len(ks), f"{how} replay {rep}")
        out["count"].fill_(-1)  # eager work between replays
        torch.cuda.synchronize()


def test_device_lengths_grid_beyond_the_chip(A):
    """24 signals x 18 loops: the device-length main pass runs its arrays
    (all of at most 4096 buckets here) in 256-thread workgroups; the same as
    the grouped execute, and each signal the oracle's."""
    import torch

    n_max = 1 << 16
    ms = [1 << (12 + (i % 5)) for i in range(24)]
    ks = [3 + (i * 7) % 20 for i in range(24)]
    xs = [synth.planted_1d(m, k, 800 + i, mag=("uniform", 0.5, 1.0), snr_db=35.0, dtype=np.complex64)[0]
          for i, (m, k) in enumerate(zip(ms, ks))]
    ns = np.array(ms, dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(ns)[:-1]]).astype(np.int64)
    x = torch.from_numpy(np.concatenate(xs)).cuda()
    plan = A.Plan(1, n_max, "c64", seed=19, n_min=1 << 12, max_batch=len(ms))
    loops = plan.desc.L_loc + plan.desc.L_est
    assert loops * len(ms) > torch.cuda.get_device_properties(0).multi_processor_count
    print(f"device-length call beyond the chip: {len(ms)} signals", flush=True)
    dev = plan.execute_uneven_dev(x, torch.from_numpy(offs).cuda(), torch.from_numpy(ns).cuda())
    grp = plan.execute_uneven(x, offs, ns)
    torch.cuda.synchronize()
    _same_outputs(dev, grp, len(ms), "device vs grouped")
    for i, (xi, m) in enumerate(zip(xs, ms)):
        res = plan.results(dev, i)
        ref = oracle.atsfft(xi.astype(np.complex128), sub_params(plan.desc, int(m), i), trace=False)
        assert (res["status"], res["khat"], res["count"]) == (ref["status"], ref["khat"], ref["count"]), i
        assert np.array_equal(res["locs"], ref["locs"]), i
        assert value_rel_err(res["vals"], ref["vals"], "c64") < VAL_TOL["c64"], i
