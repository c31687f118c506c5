"""Python binding of the ATSFFT C ABI (include/atsfft.h).

Argument marshalling only: every step of the transform runs in libatsfft.so
on the GPU.  PyTorch supplies device memory and the current HIP stream.
Importing this module does not need a GPU; creating a Plan does, and raises
if the library is missing or the device is not a gfx950.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libatsfft.so")

SUCCESS, EINVAL, ENODEVICE, ENOMEM, ELAUNCH, ENOTSUPPORTED = range(6)
C64, C128 = 0, 1
SIG_OK, SIG_TRUNCATED, SIG_PROBE_NOT_CONVERGED, SIG_PROBE_SATURATED, SIG_EMPTY, SIG_RETRIED = 0, 1, 2, 4, 8, 16
SIG_PROBE_TIMEOUT = 32
SIG_BAD_LENGTH = 64
FLAG_FIXED_B = 1
FLAG_PROFILE = 2
FLAG_COMPENSATED = 4
FLAG_GRAPH = 8
STAGES = ("probe", "hash_main", "bucket_main", "vote", "estimate")


class Desc(C.Structure):
    _fields_ = [
        ("ndim", C.c_int32),
        ("dtype", C.c_int32),
        ("n", C.c_int64),
        ("max_out", C.c_int64),
        ("seed", C.c_uint64),
        ("flags", C.c_uint32),
        ("max_batch", C.c_int32),
        ("B0", C.c_int64),
        ("B_max", C.c_int64),
        ("alpha_probe", C.c_int32),
        ("alpha", C.c_int32),
        ("L_loc", C.c_int32),
        ("L_est", C.c_int32),
        ("T_vote", C.c_int32),
        ("P_max", C.c_int32),
        ("d", C.c_int32),
        ("gamma", C.c_int32),
        ("delta", C.c_double),
        ("q", C.c_double),
        ("noise_rate", C.c_double),
        ("rho", C.c_double),
        ("fixed_B", C.c_int64),
        ("fixed_k", C.c_int64),
        ("n_min", C.c_int64),
        ("res_tol", C.c_double),
        ("res_retries", C.c_int32),
        ("pad0", C.c_int32),
    ]


class Trace(C.Structure):
    _fields_ = [
        ("B_star", C.c_int32),
        ("khat", C.c_int32),
        ("n_probe", C.c_int32),
        ("count", C.c_int32),
        ("status", C.c_uint32),
        ("probe_B", C.POINTER(C.c_int32)),
        ("probe_k", C.POINTER(C.c_int32)),
        ("probe_dec", C.POINTER(C.c_int32)),
        ("probe_T", C.POINTER(C.c_double)),
        ("T_loc", C.POINTER(C.c_double)),
        ("J_count", C.POINTER(C.c_int32)),
        ("yhat", C.c_void_p),
        ("J_bits", C.POINTER(C.c_uint32)),
        ("res_ratio", C.c_double),
        ("retries", C.c_int32),
        ("pad0", C.c_int32),
    ]


# every symbol include/atsfft.h declares
EXPORTS = (
    "atsfft_default_desc", "atsfft_plan", "atsfft_workspace_size", "atsfft_execute_batched",
    "atsfft_execute", "atsfft_backward", "atsfft_trace_read", "atsfft_destroy",
    "atsfft_status_string", "atsfft_version", "atsfft_last_error", "atsfft_profile_read",
    "atsfft_execute_uneven", "atsfft_workspace_size_uneven", "atsfft_execute_batched_noalloc",
    "atsfft_execute_uneven_dev", "atsfft_workspace_size_uneven_dev",
)
NOALLOC_WORKSPACE_BYTES = 64 << 20  # ATSFFT_NOALLOC_WORKSPACE_BYTES

_lib = None


class AtsfftError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = load()
        msg = lib.atsfft_status_string(status).decode()
        detail = lib.atsfft_last_error().decode()
        super().__init__(f"{where}: {msg}" + (f" ({detail})" if detail else ""))
        self.status = status


def load():
    """Load libatsfft.so; raise if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with python -m paper_1908_02461_amd.build")
    L = C.CDLL(LIB_PATH)
    vp, sz = C.c_void_p, C.c_size_t
    L.atsfft_default_desc.argtypes = [C.POINTER(Desc), C.c_int32, C.c_int64, C.c_int32]
    L.atsfft_plan.argtypes = [C.POINTER(vp), C.POINTER(Desc)]
    L.atsfft_workspace_size.argtypes = [vp, C.c_int32, C.POINTER(sz)]
    L.atsfft_execute_batched.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.atsfft_execute.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.atsfft_execute_batched_noalloc.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp]
    L.atsfft_backward.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    L.atsfft_trace_read.argtypes = [vp, vp, C.c_int32, C.POINTER(Trace), vp]
    L.atsfft_destroy.argtypes = [vp]
    L.atsfft_profile_read.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(C.c_int32)]
    I64P = C.POINTER(C.c_int64)
    L.atsfft_execute_uneven.argtypes = [vp, C.c_int32, vp, I64P, I64P, vp, vp, vp, vp, vp, vp, sz, vp]
    L.atsfft_workspace_size_uneven.argtypes = [vp, C.c_int32, I64P, C.POINTER(sz)]
    L.atsfft_execute_uneven_dev.argtypes = [vp, C.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
    L.atsfft_workspace_size_uneven_dev.argtypes = [vp, C.c_int32, C.POINTER(sz)]
    L.atsfft_status_string.argtypes = [C.c_int]
    L.atsfft_status_string.restype = C.c_char_p
    L.atsfft_version.restype = C.c_char_p
    L.atsfft_last_error.restype = C.c_char_p
    for name in ("atsfft_default_desc", "atsfft_plan", "atsfft_workspace_size", "atsfft_execute_batched",
                 "atsfft_execute", "atsfft_backward", "atsfft_trace_read", "atsfft_destroy",
                 "atsfft_profile_read", "atsfft_execute_uneven", "atsfft_workspace_size_uneven",
                 "atsfft_execute_batched_noalloc", "atsfft_execute_uneven_dev",
                 "atsfft_workspace_size_uneven_dev"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


def _check(status: int, where: str):
    if status != SUCCESS:
        raise AtsfftError(status, where)


def default_desc(ndim: int, n: int, dtype: str = "c64", **knobs) -> Desc:
    d = Desc()
    _check(load().atsfft_default_desc(C.byref(d), ndim, n, C64 if dtype == "c64" else C128),
           "atsfft_default_desc")
    profile = bool(knobs.pop("profile", False))
    compensated = bool(knobs.pop("compensated", False))
    graph = bool(knobs.pop("graph", False))
    for k, v in knobs.items():
        if not hasattr(d, k):
            raise TypeError(f"unknown knob {k!r}")
        setattr(d, k, v)
    if knobs.get("fixed_B", 0):
        d.flags |= FLAG_FIXED_B
    if profile:
        d.flags |= FLAG_PROFILE
    if compensated:
        d.flags |= FLAG_COMPENSATED
    if graph:
        d.flags |= FLAG_GRAPH
    return d


def desc_dict(d: Desc) -> dict:
    return {name: getattr(d, name) for name, _ in Desc._fields_}


class Plan:
    """A plan for signals of one size and precision (atsfft_plan)."""

    def __init__(self, ndim: int, n: int, dtype: str = "c64", **knobs):
        import torch

        if dtype not in ("c64", "c128"):
            raise ValueError("dtype must be 'c64' or 'c128'")
        self.ndim, self.n, self.dtype = ndim, n, dtype
        self.torch_dtype = torch.complex64 if dtype == "c64" else torch.complex128
        self.desc = default_desc(ndim, n, dtype, **knobs)
        self._h = C.c_void_p()
        _check(load().atsfft_plan(C.byref(self._h), C.byref(self.desc)), "atsfft_plan")
        self._ws = None

    # -- sizes --
    @property
    def max_out(self) -> int:
        return int(self.desc.max_out)

    @property
    def main_bmax(self) -> int:
        """Largest bucket count per axis of the location and estimation loops
        (B_max; fixed_B in the Algorithm 1 form, up to B_max with the residual
        test on)."""
        d = self.desc
        if not d.flags & FLAG_FIXED_B:
            return int(d.B_max)
        return int(max(d.fixed_B, d.B_max) if d.res_tol > 0 else d.fixed_B)

    def workspace_size(self, batch: int) -> int:
        b = C.c_size_t()
        _check(load().atsfft_workspace_size(self._h, batch, C.byref(b)), "atsfft_workspace_size")
        return int(b.value)

    def workspace(self, batch: int, device=None):
        import torch

        need = self.workspace_size(batch)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=device or "cuda")
        return self._ws

    # -- execution --
    def outputs(self, batch: int, device):
        import torch

        return dict(
            locs=torch.zeros((batch, self.max_out), dtype=torch.int64, device=device),
            vals=torch.zeros((batch, self.max_out), dtype=self.torch_dtype, device=device),
            count=torch.empty(batch, dtype=torch.int32, device=device),
            khat=torch.empty(batch, dtype=torch.int32, device=device),
            status=torch.empty(batch, dtype=torch.int32, device=device),
        )

    def execute_batched(self, x, out: Optional[dict] = None, ws=None, stream=None) -> dict:
        """x: [batch, n] or [batch, N, N] contiguous device tensor of the plan's dtype."""
        import torch

        if not x.is_cuda or x.dtype != self.torch_dtype or not x.is_contiguous():
            raise ValueError("x must be a contiguous device tensor of the plan's complex dtype")
        shape = (self.n,) if self.ndim == 1 else (self.n, self.n)
        if tuple(x.shape[1:]) != shape:
            raise ValueError(f"x must have shape [batch, {', '.join(map(str, shape))}]")
        batch = x.shape[0]
        out = out or self.outputs(batch, x.device)
        ws = ws if ws is not None else self.workspace(batch, x.device)
        s = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
        _check(load().atsfft_execute_batched(
            self._h, batch, x.data_ptr(), out["locs"].data_ptr(), out["vals"].data_ptr(),
            out["count"].data_ptr(), out["khat"].data_ptr(), out["status"].data_ptr(), ws.data_ptr(),
            ws.numel(), s), "atsfft_execute_batched")
        out["ws"] = ws
        return out

    def execute_noalloc(self, x, out: dict, stream=None) -> dict:
        """atsfft_execute_batched_noalloc: the batched execute with the
        library's fixed device workspace; out (from outputs()) is required so
        that the call itself allocates nothing."""
        import torch

        if not x.is_cuda or x.dtype != self.torch_dtype or not x.is_contiguous():
            raise ValueError("x must be a contiguous device tensor of the plan's complex dtype")
        shape = (self.n,) if self.ndim == 1 else (self.n, self.n)
        if tuple(x.shape[1:]) != shape:
            raise ValueError(f"x must have shape [batch, {', '.join(map(str, shape))}]")
        batch = x.shape[0]
        s = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
        _check(load().atsfft_execute_batched_noalloc(
            self._h, batch, x.data_ptr(), out["locs"].data_ptr(), out["vals"].data_ptr(),
            out["count"].data_ptr(), out["khat"].data_ptr(), out["status"].data_ptr(), s),
            "atsfft_execute_batched_noalloc")
        return out

    def execute_uneven(self, x, offsets, ns, out: Optional[dict] = None, ws=None, stream=None) -> dict:
        """Signals of different lengths packed in the 1D device tensor x;
        offsets and ns are sequences (host) of element offsets and lengths."""
        import torch

        if not x.is_cuda or x.dtype != self.torch_dtype or not x.is_contiguous():
            raise ValueError("x must be a contiguous device tensor of the plan's complex dtype")
        offs = np.ascontiguousarray(offsets, dtype=np.int64)
        nsa = np.ascontiguousarray(ns, dtype=np.int64)
        batch = int(nsa.size)
        if offs.size != batch:
            raise ValueError("offsets and ns must have the same length")
        per = nsa if self.ndim == 1 else nsa * nsa
        if np.any(offs + per > x.numel()):
            raise ValueError("a signal runs past the end of x")
        I64P = C.POINTER(C.c_int64)
        b = C.c_size_t()
        _check(load().atsfft_workspace_size_uneven(self._h, batch, nsa.ctypes.data_as(I64P), C.byref(b)),
               "atsfft_workspace_size_uneven")
        if ws is None or ws.numel() < b.value:
            ws = torch.empty(b.value, dtype=torch.uint8, device=x.device)
        out = out or self.outputs(batch, x.device)
        s = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
        _check(load().atsfft_execute_uneven(
            self._h, batch, x.data_ptr(), offs.ctypes.data_as(I64P), nsa.ctypes.data_as(I64P),
            out["locs"].data_ptr(), out["vals"].data_ptr(), out["count"].data_ptr(), out["khat"].data_ptr(),
            out["status"].data_ptr(), ws.data_ptr(), ws.numel(), s), "atsfft_execute_uneven")
        out["ws"] = ws
        return out

    def workspace_size_uneven_dev(self, batch: int) -> int:
        b = C.c_size_t()
        _check(load().atsfft_workspace_size_uneven_dev(self._h, batch, C.byref(b)),
               "atsfft_workspace_size_uneven_dev")
        return int(b.value)

    def execute_uneven_dev(self, x, offsets, ns, out: Optional[dict] = None, ws=None, stream=None) -> dict:
        """Signals of different lengths packed in the 1D device tensor x, with
        offsets and lengths given as int64 device tensors (the host reads
        neither: the call can be captured into a graph)."""
        import torch

        if not x.is_cuda or x.dtype != self.torch_dtype or not x.is_contiguous():
            raise ValueError("x must be a contiguous device tensor of the plan's complex dtype")
        for t in (offsets, ns):
            if not (t.is_cuda and t.dtype == torch.int64 and t.is_contiguous() and t.dim() == 1):
                raise ValueError("offsets and ns must be contiguous 1D int64 device tensors")
        batch = int(ns.numel())
        if offsets.numel() != batch:
            raise ValueError("offsets and ns must have the same length")
        need = self.workspace_size_uneven_dev(batch)
        if ws is None or ws.numel() < need:
            ws = torch.empty(need, dtype=torch.uint8, device=x.device)
        out = out or self.outputs(batch, x.device)
        s = stream if stream is not None else torch.cuda.current_stream(x.device).cuda_stream
        _check(load().atsfft_execute_uneven_dev(
            self._h, batch, x.data_ptr(), offsets.data_ptr(), ns.data_ptr(), out["locs"].data_ptr(),
            out["vals"].data_ptr(), out["count"].data_ptr(), out["khat"].data_ptr(), out["status"].data_ptr(),
            ws.data_ptr(), ws.numel(), s), "atsfft_execute_uneven_dev")
        out["ws"] = ws
        return out

    def execute(self, x, **kw) -> dict:
        return self.execute_batched(x.unsqueeze(0), **kw)

    def results(self, out: dict, signal: int = 0) -> dict:
        """Host copy of one signal's located set and values."""
        cnt = int(out["count"][signal])
        st = int(out["status"][signal])
        kept = 0 if st & (SIG_TRUNCATED | SIG_EMPTY) else cnt
        return dict(
            count=cnt, status=st, khat=int(out["khat"][signal]),
            locs=out["locs"][signal, :kept].cpu().numpy(),
            vals=out["vals"][signal, :kept].cpu().numpy().astype(np.complex128),
        )

    def trace(self, ws, signal: int = 0, full: bool = True) -> dict:
        """atsfft_trace_read: probe history, thresholds, bucket DFTs and cutoffs
        (the last two only when ``full``)."""
        import torch

        d = self.desc
        Bbig = self.main_bmax
        bc = Bbig if self.ndim == 1 else Bbig * Bbig
        L = d.L_loc + d.L_est
        pB = np.zeros(32, np.int32)
        pk = np.zeros(32, np.int32)
        pd = np.zeros(32, np.int32)
        pT = np.zeros(32, np.float64)
        tl = np.zeros(32, np.float64)
        jc = np.zeros(32, np.int32)
        yh = np.zeros((L, bc), dtype=np.complex64 if self.dtype == "c64" else np.complex128)
        words = (bc + 31) // 32
        jb = np.zeros((d.L_loc, words), np.uint32)
        t = Trace()
        t.probe_B = pB.ctypes.data_as(C.POINTER(C.c_int32))
        t.probe_k = pk.ctypes.data_as(C.POINTER(C.c_int32))
        t.probe_dec = pd.ctypes.data_as(C.POINTER(C.c_int32))
        t.probe_T = pT.ctypes.data_as(C.POINTER(C.c_double))
        t.T_loc = tl.ctypes.data_as(C.POINTER(C.c_double))
        t.J_count = jc.ctypes.data_as(C.POINTER(C.c_int32))
        if full:
            t.yhat = yh.ctypes.data
            t.J_bits = jb.ctypes.data_as(C.POINTER(C.c_uint32))
        s = torch.cuda.current_stream(ws.device).cuda_stream
        _check(load().atsfft_trace_read(self._h, ws.data_ptr(), signal, C.byref(t), s), "atsfft_trace_read")
        npb = int(t.n_probe)
        B = int(t.B_star)
        c = B if self.ndim == 1 else B * B
        bits = np.unpackbits(jb.view(np.uint8), bitorder="little").reshape(d.L_loc, words * 32)
        if not full:
            yh, bits = yh[:, :0], bits[:, :0]
            c = 0
        return dict(
            B_star=B, khat=int(t.khat), n_probe=npb, count=int(t.count), status=int(t.status),
            probe_B=pB[:npb].tolist(), probe_k=pk[:npb].tolist(), probe_decision=pd[:npb].tolist(),
            probe_T=pT[:npb].tolist(), T_loc=tl[: d.L_loc].tolist(), J_count=jc[: d.L_loc].tolist(),
            yhat=yh[:, :c].astype(np.complex128), J=bits[:, :c].astype(bool),
            res_ratio=float(t.res_ratio), retries=int(t.retries),
        )

    def profile_read(self) -> dict:
        """Summed stage times (ms) and execute count since the last read."""
        ms = (C.c_double * len(STAGES))()
        cnt = C.c_int32()
        _check(load().atsfft_profile_read(self._h, ms, C.byref(cnt)), "atsfft_profile_read")
        return {"executes": int(cnt.value), **{s: float(ms[i]) for i, s in enumerate(STAGES)}}

    def backward(self, grad_vals, ws, grad_x, stream=None):
        """atsfft_backward: grad_x (written in full) from grad_vals [batch, max_out]."""
        import torch

        if grad_vals.dtype != self.torch_dtype or grad_x.dtype != self.torch_dtype:
            raise ValueError("grad_vals and grad_x must have the plan's complex dtype")
        if not (grad_vals.is_contiguous() and grad_x.is_contiguous()):
            raise ValueError("grad_vals and grad_x must be contiguous")
        s = stream if stream is not None else torch.cuda.current_stream(grad_x.device).cuda_stream
        _check(load().atsfft_backward(self._h, grad_vals.shape[0], grad_vals.data_ptr(), ws.data_ptr(),
                                      grad_x.data_ptr(), s), "atsfft_backward")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            load().atsfft_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sparse_fft(x, plan: Plan):
    """Differentiable transform of a batch x [batch, n] (or [batch, N, N]).

    Returns (vals, locs, count, khat, status); vals [batch, max_out] carries
    autograd through the value estimates at fixed located frequencies and
    median choices (atsfft_backward); entries at or past count are zero.
    """
    return _SparseFFT.apply(x, plan)


def _make_function():
    import torch

    class _SparseFFTFn(torch.autograd.Function):
        @staticmethod
        def forward(ctx, x, plan):
            x = x.contiguous()
            ws = torch.empty(plan.workspace_size(x.shape[0]), dtype=torch.uint8, device=x.device)
            out = plan.execute_batched(x, ws=ws)
            ctx.plan, ctx.ws = plan, ws
            ctx.xshape, ctx.xdtype = x.shape, x.dtype
            ctx.mark_non_differentiable(out["locs"], out["count"], out["khat"], out["status"])
            return out["vals"], out["locs"], out["count"], out["khat"], out["status"]

        @staticmethod
        def backward(ctx, gvals, *unused):
            gx = torch.empty(ctx.xshape, dtype=ctx.xdtype, device=ctx.ws.device)
            if gvals is None:
                gx.zero_()
            else:
                ctx.plan.backward(gvals.contiguous(), ctx.ws, gx)
            return gx, None

    return _SparseFFTFn


class _Lazy:
    _fn = None

    def apply(self, *a):
        if _Lazy._fn is None:
            _Lazy._fn = _make_function()
        return _Lazy._fn.apply(*a)


_SparseFFT = _Lazy()
