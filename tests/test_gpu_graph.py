"""HIP graph replay of the execute (ATSFFT_FLAG_GRAPH) and capture of a plain
plan's execute by the caller (torch.cuda.graph): every replay, with the input
rewritten in place and eager work in between, gives bitwise the results of an
eager execute of the same input (the forward path is deterministic)."""
import numpy as np
import pytest

from paper_1908_02461_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("locs", "vals", "count", "khat", "status")


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _inputs(n, batch, seed0):
    return [np.stack([synth.planted_1d(n, 6 + (i + s) % 5, seed0 + 10 * s + i, mag=("uniform", 0.5, 1.0),
                                       snr_db=35.0, dtype=np.complex64)[0] for i in range(batch)])
            for s in range(3)]


def _eager(A, n, xs, **knobs):
    import torch

    plan = A.Plan(1, n, "c64", seed=9, max_batch=xs.shape[0], **knobs)
    out = plan.execute_batched(torch.from_numpy(xs).cuda())
    torch.cuda.synchronize()
    return {k: out[k].cpu().clone() for k in KEYS}


def _same(a, b):
    """Identical counts, k-hat and statuses, and identical locations and values
    in the first count entries of each signal (the rest is undefined)."""
    import torch

    for k in ("count", "khat", "status"):
        assert torch.equal(a[k], b[k]), k
    for i, c in enumerate(a["count"].tolist()):
        if a["status"][i].item() & 1:  # truncated: nothing written
            continue
        for k in ("locs", "vals"):
            assert torch.equal(a[k][i, :c], b[k][i, :c]), (k, i)


@pytest.mark.parametrize("knobs", [{}, dict(res_tol=1e-6, res_retries=2, B_max=1024, P_max=3)])
def test_graph_flag_replays_match_eager(A, knobs):
    import torch

    n, batch = 1 << 14, 5
    xs = _inputs(n, batch, 100)
    plan = A.Plan(1, n, "c64", seed=9, max_batch=batch, graph=True, **knobs)
    x = torch.empty((batch, n), dtype=torch.complex64, device="cuda")
    out = plan.outputs(batch, x.device)
    ws = plan.workspace(batch, x.device)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(2):
        for s, xh in enumerate(xs):
            x.copy_(torch.from_numpy(xh))
            plan.execute_batched(x, out=out, ws=ws)
            junk.mul_(1.0001).add_(0.5)  # eager work between replays
            torch.cuda.synchronize()
            _same({k: out[k].cpu() for k in KEYS}, _eager(A, n, xh, **knobs))
    if knobs:
        st = out["status"].cpu().numpy()
        assert (st & A.SIG_RETRIED).any(), st


def test_graph_shapes_beyond_the_cache(A):
    """More call shapes than the plan keeps: the oldest are dropped and
    captured again when they return."""
    import torch

    n = 1 << 12
    xh = _inputs(n, 2, 300)[0]
    plan = A.Plan(1, n, "c64", seed=9, max_batch=2, graph=True)
    x = torch.from_numpy(xh).cuda()
    ref = _eager(A, n, xh)
    outs = [plan.outputs(2, x.device) for _ in range(70)]
    ws = plan.workspace(2, x.device)
    for rep in range(2):
        for o in outs:
            plan.execute_batched(x, out=o, ws=ws)
    torch.cuda.synchronize()
    for o in outs:
        _same({k: o[k].cpu() for k in KEYS}, ref)


def test_caller_capture_of_a_plain_plan(A):
    import torch

    n, batch = 1 << 14, 2
    xs = _inputs(n, batch, 200)
    plan = A.Plan(1, n, "c64", seed=9, max_batch=batch)
    x = torch.from_numpy(xs[0]).cuda()
    out = plan.outputs(batch, x.device)
    ws = plan.workspace(batch, x.device)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        plan.execute_batched(x, out=out, ws=ws)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.execute_batched(x, out=out, ws=ws)
    junk = torch.randn(1 << 20, device="cuda")
    for rep in range(2):
        for xh in xs:
            x.copy_(torch.from_numpy(xh))
            g.replay()
            junk.mul_(1.0001).add_(0.5)
            torch.cuda.synchronize()
            _same({k: out[k].cpu() for k in KEYS}, _eager(A, n, xh))
