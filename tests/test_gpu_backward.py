"""GPU checks of the adjoint (atsfft_backward) through value estimation.

The values are real-linear in x once the located set and the median choices
are fixed, so a quadratic loss has exact central differences: the library's
gradient is checked against FP64 central differences of the oracle's loss
(same draws, decisions verified unchanged), against the restricted dense-DFT
identity DFT(grad_x)_f = 2 n r_f at located f that no other located
frequency's median loops put in or next to its bucket, and with
torch.autograd.gradcheck.
"""
import numpy as np
import pytest

import oracle
from paper_1908_02461_amd import synth

from parity_util import oracle_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _medians(est):
    """Index of the first loop whose estimate equals the median, Re and Im."""
    out = []
    for row in est:
        mr, mi = np.median(row.real), np.median(row.imag)
        out.append((int(np.flatnonzero(row.real == mr)[0]), int(np.flatnonzero(row.imag == mi)[0])))
    return out


def _oracle_loss(x, p, targets, locs_ref, med_ref):
    r = oracle.atsfft(x, p, trace=True)
    assert np.array_equal(r["locs"], locs_ref), "located set moved under the perturbation"
    assert _medians(r["est"]) == med_ref, "a median choice moved under the perturbation"
    return float(np.sum(np.abs(r["vals"] - targets) ** 2))


@pytest.mark.parametrize("ndim,dt", [(1, "c128"), (1, "c64"), (2, "c128")])
def test_gradient_matches_oracle_central_differences(A, ndim, dt):
    import torch

    if ndim == 1:
        n, k = 1 << 12, 6
        x, _, _ = synth.planted_1d(n, k, 3, mag=("uniform", 0.5, 1.0), snr_db=30.0)
        plan = A.Plan(1, n, dt, seed=17, B_max=128)
    else:
        n, k = 128, 4
        x, _, _ = synth.planted_2d(n, k, 3, mag=("uniform", 0.5, 1.0), snr_db=30.0)
        plan = A.Plan(2, n, dt, seed=17, B_max=16)
    npdt = np.complex64 if dt == "c64" else np.complex128
    x = x.astype(npdt)
    xd = torch.from_numpy(x[None].copy()).cuda().requires_grad_(True)
    vals, locs, count, khat, status = A.sparse_fft(xd, plan)
    cnt = int(count[0])
    assert cnt > 0 and not int(status[0]) & (A.SIG_TRUNCATED | A.SIG_EMPTY)
    rng = np.random.default_rng(5)
    targets = rng.standard_normal(cnt) + 1j * rng.standard_normal(cnt)
    tt = torch.from_numpy(targets.astype(npdt)).cuda()
    loss = torch.sum(torch.abs(vals[0, :cnt] - tt) ** 2)
    loss.backward()
    grad = xd.grad[0].cpu().numpy().astype(np.complex128)

    p = oracle_params(plan, 0)
    x64 = x.astype(np.complex128)
    r0 = oracle.atsfft(x64, p, trace=True)
    assert np.array_equal(r0["locs"], locs[0, :cnt].cpu().numpy())
    med = _medians(r0["est"])
    eps = 1e-6 * float(np.sqrt(np.mean(np.abs(x64) ** 2)))
    for trial in range(3):
        v = rng.standard_normal(x.shape) + 1j * rng.standard_normal(x.shape)
        lp = _oracle_loss(x64 + eps * v, p, targets, r0["locs"], med)
        lm = _oracle_loss(x64 - eps * v, p, targets, r0["locs"], med)
        fd = (lp - lm) / (2 * eps)
        an = float(np.sum(grad.real * v.real + grad.imag * v.imag))
        tol = 1e-7 if dt == "c128" else 2e-3
        assert abs(an - fd) <= tol * max(abs(fd), 1e-3 * float(np.sum(np.abs(grad) * np.abs(v)))), (trial, an, fd)


def test_restricted_dense_dft_gradient(A):
    """DFT(grad_x)_f = 2 n r_f for located f whose median loops hold no other
    located frequency in the same bucket (leakage of the window aside)."""
    import torch

    n, k = 1 << 16, 12
    x, _, _ = synth.planted_1d(n, k, 8, mag=("uniform", 0.5, 1.0), snr_db=40.0, dtype=np.complex64)
    plan = A.Plan(1, n, "c64", seed=23)
    xd = torch.from_numpy(x[None].copy()).cuda().requires_grad_(True)
    vals, locs, count, khat, status = A.sparse_fft(xd, plan)
    cnt = int(count[0])
    rng = np.random.default_rng(9)
    targets = torch.from_numpy((rng.standard_normal(cnt) + 1j * rng.standard_normal(cnt)).astype(np.complex64)).cuda()
    r = vals[0, :cnt] - targets
    torch.sum(torch.abs(r) ** 2).backward()
    G = torch.fft.fft(xd.grad[0].to(torch.complex128)).cpu().numpy()
    S = locs[0, :cnt].cpu().numpy()
    rr = r.detach().cpu().numpy().astype(np.complex128)
    # median loops of every located f, from the oracle on the same draws
    ro = oracle.atsfft(x.astype(np.complex128), oracle_params(plan, 0), trace=True)
    assert np.array_equal(ro["locs"], S)
    med = _medians(ro["est"])
    B = ro["B_star"]
    draws = [oracle.draw(plan.desc.seed, 0, oracle.PHASE_EST, l, 0, n) for l in range(plan.desc.L_est)]
    buckets = np.array([[oracle.hash_bucket(n, B, draws[l][0], int(f)) for l in range(plan.desc.L_est)] for f in S])
    L_est = plan.desc.L_est

    def near(l, i, j):
        d = abs(int(buckets[i, l]) - int(buckets[j, l]))
        return min(d, B - d) <= 1

    checked = 0
    for i, f in enumerate(S):
        # G[f] also collects n conj(est_f'(tone f)) g_f' of every other located
        # f' whose median loops put f in or next to f''s bucket
        alone = all(not near(l, i, j) for j in range(len(S)) if j != i for l in set(med[j]))
        if not alone:
            continue
        checked += 1
        assert abs(G[f] - 2 * n * rr[i]) <= 1e-3 * abs(2 * n * rr[i]), (f, G[f], 2 * n * rr[i])
    assert checked >= max(1, len(S) // 2)


def test_torch_gradcheck_small(A):
    import torch

    n = 256
    x, _, _ = synth.planted_1d(n, 2, 1, mag=("uniform", 0.5, 1.0), snr_db=40.0)
    plan = A.Plan(1, n, "c128", seed=4, B0=4, B_max=16, alpha=8, alpha_probe=4, gamma=4)
    xd = torch.from_numpy(x[None].copy()).cuda().requires_grad_(True)
    with torch.no_grad():
        cnt = int(A.sparse_fft(xd, plan)[2][0])
    assert cnt > 0
    w = torch.randn(cnt, dtype=torch.complex128, device="cuda")

    def f(inp):
        return (A.sparse_fft(inp, plan)[0][0, :cnt] * w).sum()

    # atomics add the loops in any order: allow last-bit differences between calls
    assert torch.autograd.gradcheck(f, (xd,), eps=1e-7, atol=1e-6, rtol=1e-5, fast_mode=True, nondet_tol=1e-12)


def test_backward_of_empty_signal_is_zero(A):
    import torch

    n = 1 << 12
    plan = A.Plan(1, n, "c64", seed=1, B_max=64)
    xd = torch.zeros((1, n), dtype=torch.complex64, device="cuda", requires_grad=True)
    vals, locs, count, khat, status = A.sparse_fft(xd, plan)
    assert int(status[0]) & A.SIG_EMPTY
    (vals.abs() ** 2).sum().backward()
    assert torch.count_nonzero(xd.grad) == 0


@pytest.mark.parametrize("ndim,n,k", [(1, 1 << 16, 12), (2, 256, 6)])
def test_gather_staged_equals_unstaged(A, monkeypatch, ndim, n, k):
    """The adjoint gather with each loop's bucket adjoint staged in LDS gives
    the gradient it gives with every read from device memory
    (ATSFFT_GATHER_LDS=0): the loops are added in the same order either way,
    and only the bucket cotangent's atomic adds of located frequencies that
    share a bucket may reorder between calls."""
    import torch

    make = synth.planted_1d if ndim == 1 else synth.planted_2d
    x = make(n, k, 12, mag=("uniform", 0.5, 1.0), snr_db=40.0, dtype=np.complex64)[0]
    grads = []
    for env in (None, "0"):
        if env is None:
            monkeypatch.delenv("ATSFFT_GATHER_LDS", raising=False)
        else:
            monkeypatch.setenv("ATSFFT_GATHER_LDS", env)
        plan = A.Plan(ndim, n, "c64", seed=29)
        xd = torch.from_numpy(x[None].copy()).cuda().requires_grad_(True)
        vals, locs, count, khat, status = A.sparse_fft(xd, plan)
        cnt = int(count[0])
        assert cnt > 0
        w = torch.linspace(0.5, 1.5, cnt, device="cuda").to(torch.complex64)
        (torch.abs(vals[0, :cnt] * w) ** 2).sum().backward()
        grads.append(xd.grad.detach().cpu().numpy())
    assert np.count_nonzero(grads[0]) > 0
    assert np.max(np.abs(grads[0] - grads[1])) <= 1e-6 * np.max(np.abs(grads[0]))
