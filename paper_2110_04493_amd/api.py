"""PyTorch-facing API: device tensors in, device tensors out.

Torch provides device memory (outputs are allocated through torch's caching
allocator via the library's allocator callback) and the stream (the current
torch stream); the computation itself runs in the gfx950 library.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import capi


class _TorchAllocator:
    """Allocator callback handing torch uint8 buffers to the library.

    Buffers are allocated on the plan's stream, the stream the library writes
    them on, so that torch's caching allocator orders their reuse after the
    library's work."""

    def __init__(self, device, stream):
        self.device = device
        self.stream = stream
        self.live: dict[int, torch.Tensor] = {}
        self._alloc = capi.ALLOC_FN(self._do_alloc)
        self._free = capi.FREE_FN(self._do_free)
        self.struct = capi.expm_allocator(self._alloc, self._free, None)

    def _do_alloc(self, nbytes, stream, ctx):
        try:
            with torch.cuda.stream(self.stream):
                t = torch.empty(int(nbytes), dtype=torch.uint8, device=self.device)
        except RuntimeError:
            return None
        self.live[t.data_ptr()] = t
        return t.data_ptr()

    def _do_free(self, ptr, stream, ctx):
        self.live.pop(ptr, None)

    def take(self, ptr: int, count: int, dtype: torch.dtype) -> torch.Tensor:
        """Moves ownership of one output buffer to the caller as a typed view.
        The caller's current stream is made to wait for the plan's stream
        (see Plan._handover); the buffer is marked as used on the current
        stream so that torch does not reuse it before that stream's work on
        it is done."""
        if count == 0:
            self.live.pop(ptr, None)
            return torch.empty(0, dtype=dtype, device=self.device)
        t = self.live.pop(ptr)
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            t.record_stream(cur)
        nbytes = count * torch.empty(0, dtype=dtype).element_size()
        return t[:nbytes].view(dtype)


def _view(crow: torch.Tensor, col: torch.Tensor, val: torch.Tensor) -> capi.expm_csr_cview:
    n = crow.numel() - 1
    return capi.expm_csr_cview(n, val.numel(), crow.data_ptr(), col.data_ptr(), val.data_ptr())


def _check_inputs(crow, col, val, vdtype=torch.float64):
    dev = val.device
    if dev.type != "cuda":
        raise ValueError("the gfx950 library takes device tensors (no CPU path)")
    if crow.dtype != torch.int64 or col.dtype != torch.int32 or val.dtype != vdtype:
        raise TypeError(f"expects int64 row pointers, int32 columns and {vdtype} values")
    for t in (crow, col, val):
        if not t.is_contiguous() or t.device != dev:
            raise ValueError("inputs must be contiguous tensors on one device")


@dataclass
class Options:
    normal: int = capi.EXPM_NORMAL_AUTO
    filter_mode: int = capi.EXPM_FILTER_PAPER
    e_r: float = 0.1
    max_filter_iter: int = 64
    keep_checkpoints: bool = False
    checkpoint_interval: int = 0   # 0: auto (all iterates while they fit), -1: last ceil(sqrt(N))
    profile: int = 0           # 1: phase timers and work counts, 2: tile kernel timers only
    reorder: int = -1
    tile_min_fill: float = -1.0
    norm: int = capi.EXPM_NORM_FRO
    exact_ri: bool = False
    diagnostics: bool = False
    literal_a: bool = False    # non-normal H: a = 1/||H|| (Algorithm 4.2 step 2) instead of the min
    batch_solo_n: int = 4096   # expm_batched: instances with n >= this run on their own (0: none)
    use_symmetry: bool = True  # symmetric H: tile products form the upper triangle only


class Plan:
    """Owns one ``expm_plan_t`` (workspace pool, stream binding)."""

    def __init__(self, device=None, options: Options | None = None, stream=None):
        self.device = torch.device(device if device is not None else "cuda", )
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.options = options or Options()
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.alloc = _TorchAllocator(self.device, self.stream)
        o = capi.expm_opts_default()
        o.normal = self.options.normal
        o.filter_mode = self.options.filter_mode
        o.e_r = self.options.e_r
        o.max_filter_iter = self.options.max_filter_iter
        o.keep_checkpoints = int(self.options.keep_checkpoints)
        o.checkpoint_interval = self.options.checkpoint_interval
        o.stream = self.stream.cuda_stream
        o.allocator = C.pointer(self.alloc.struct)
        o.profile = int(self.options.profile)
        o.reorder = int(self.options.reorder)
        o.tile_min_fill = float(self.options.tile_min_fill)
        o.norm = int(self.options.norm)
        o.exact_ri = int(self.options.exact_ri)
        o.diagnostics = int(self.options.diagnostics)
        o.literal_a = int(self.options.literal_a)
        o.batch_solo_n = int(self.options.batch_solo_n)
        o.use_symmetry = int(self.options.use_symmetry)
        self._opts = o
        with torch.cuda.device(self.device):
            self.handle = capi.expm_plan(o)

    def _inputs_ready(self):
        """The library reads its inputs on the plan's stream: order that
        after the caller's current stream, which produced them."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            self.stream.wait_stream(cur)

    def _handover(self):
        """Outputs are written on the plan's stream (expm_sparse returns
        without waiting for the device): order the caller's current stream
        after it before the caller sees them."""
        cur = torch.cuda.current_stream(self.device)
        if cur != self.stream:
            cur.wait_stream(self.stream)

    def _take(self, E: capi.expm_csr, vdtype=torch.float64):
        self._handover()
        n = E.n
        rp = self.alloc.take(E.rowptr, n + 1, torch.int64)
        ci = self.alloc.take(E.col, E.nnz, torch.int32) if E.col else \
            torch.empty(0, dtype=torch.int32, device=self.device)
        v = self.alloc.take(E.val, E.nnz, vdtype) if E.val else \
            torch.empty(0, dtype=vdtype, device=self.device)
        capi.expm_csr_release(self.handle, E)
        return rp, ci, v

    def expm(self, crow, col, val, eps: float):
        """E = e^H as (rowptr int64, col int32, val float64) device tensors."""
        _check_inputs(crow, col, val)
        with torch.cuda.device(self.device):
            self._inputs_ready()
            E = capi.expm_sparse(self.handle, _view(crow, col, val), eps)
            return self._take(E)

    def expm_z(self, crow, col, val, eps: float):
        """E = e^H for complex H (complex128 values), as (rowptr int64, col
        int32, val complex128) device tensors."""
        _check_inputs(crow, col, val, torch.complex128)
        with torch.cuda.device(self.device):
            self._inputs_ready()
            E = capi.expm_sparse_z(self.handle, _view(crow, col, val), eps)
            return self._take(E, torch.complex128)

    def backward(self, dE: torch.Tensor, nnz_h: int) -> torch.Tensor:
        dE = dE.contiguous().to(torch.float64)
        with torch.cuda.device(self.device):
            with torch.cuda.stream(self.stream):
                dH = torch.empty(nnz_h, dtype=torch.float64, device=self.device)
            self._inputs_ready()
            capi.expm_sparse_backward(self.handle, dE.data_ptr(), dH.data_ptr())
            self._handover()
            cur = torch.cuda.current_stream(self.device)
            if cur != self.stream:
                dE.record_stream(self.stream)
                dH.record_stream(cur)
        return dH

    def expm_batched(self, mats, eps):
        views = []
        for crow, col, val in mats:
            _check_inputs(crow, col, val)
            views.append(_view(crow, col, val))
        with torch.cuda.device(self.device):
            self._inputs_ready()
            outs = capi.expm_sparse_batched(self.handle, views, list(eps))
            return [self._take(E) for E in outs]

    def stats(self) -> dict:
        return capi.expm_get_stats(self.handle)

    def analyze(self, crow, col, val, eps: float) -> dict:
        """Algorithm 4.2 steps 1-3 for H (norms, (M, N), normality, a, r0,
        the Taylor budget) without running the method."""
        _check_inputs(crow, col, val)
        with torch.cuda.device(self.device):
            self._inputs_ready()
            return capi.expm_analyze(self.handle, _view(crow, col, val), eps)

    def spmm(self, crow, col, val, X: torch.Tensor) -> torch.Tensor:
        """Y = A X for a CSR matrix A (typically E) and a dense block X."""
        _check_inputs(crow, col, val)
        X = X.contiguous()
        if X.dtype != torch.float64 or X.device != val.device or X.dim() != 2:
            raise TypeError("X must be a 2-D float64 tensor on the matrix's device")
        with torch.cuda.device(self.device):
            with torch.cuda.stream(self.stream):
                Y = torch.empty_like(X)
            self._inputs_ready()
            capi.expm_spmm(self.handle, _view(crow, col, val), X.shape[1], X.data_ptr(),
                           X.shape[1], Y.data_ptr(), Y.shape[1])
            self._handover()
        return Y

    def propagate(self, crow, col, val, U0: torch.Tensor, steps: int) -> torch.Tensor:
        """U_steps of Eq. (2.2)'s time stepping U_{k+1} = E U_k."""
        _check_inputs(crow, col, val)
        U0 = U0.contiguous()
        with torch.cuda.device(self.device):
            with torch.cuda.stream(self.stream):
                U = torch.empty_like(U0)
            self._inputs_ready()
            capi.expm_propagate(self.handle, _view(crow, col, val), U0.shape[1], U0.data_ptr(),
                                int(steps), U.data_ptr())
            self._handover()
        return U

    def power_norms(self, crow, col, val, K: int) -> list:
        """||H^k||_F for k = 1..K (the norms behind h_{M,N} of Eq. (4.9))."""
        _check_inputs(crow, col, val)
        with torch.cuda.device(self.device):
            self._inputs_ready()
            return capi.expm_power_norms(self.handle, _view(crow, col, val), K)

    def close(self):
        if getattr(self, "handle", None):
            self.stream.synchronize()
            capi.expm_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def csr_parts(H: torch.Tensor):
    """(crow int64, col int32, val float64) of a torch sparse CSR tensor."""
    return (H.crow_indices().to(torch.int64).contiguous(),
            H.col_indices().to(torch.int32).contiguous(),
            H.values().to(torch.float64).contiguous())


def expm(H: torch.Tensor, eps: float, **options) -> torch.Tensor:
    """e^H for a float64 sparse CSR tensor on the GPU (Algorithm 4.2)."""
    crow, col, val = csr_parts(H)
    plan = Plan(val.device, Options(**options))
    try:
        rp, ci, v = plan.expm(crow, col, val, eps)
    finally:
        plan.close()
    n = rp.numel() - 1
    return torch.sparse_csr_tensor(rp, ci.to(torch.int64), v, size=(n, n))


class ExpmFn(torch.autograd.Function):
    """Values of E = e^H as a differentiable function of the values of H.

    forward(crow, col, vals, eps) returns (E_vals, E_crow, E_col); only
    E_vals carries a gradient.  backward returns dL/d(vals of H), the exact
    derivative of the computed map with the filter masks held fixed."""

    @staticmethod
    def forward(ctx, crow, col, vals, eps, checkpoint_interval=0):
        plan = Plan(vals.device, Options(keep_checkpoints=True,
                                         checkpoint_interval=checkpoint_interval))
        rp, ci, v = plan.expm(crow, col, vals.detach(), eps)
        ctx.plan = plan
        ctx.nnz_h = vals.numel()
        ctx.mark_non_differentiable(rp, ci)
        return v, rp, ci

    @staticmethod
    def backward(ctx, gE, _grp, _gci):
        dH = ctx.plan.backward(gE, ctx.nnz_h)
        ctx.plan.close()
        return None, None, dH, None, None


def expm_batched(mats, eps, tune: bool = False, **options):
    """Exponentials of several CSR matrices (list of (crow, col, vals)) in one
    batched call; returns a list of (rowptr, col, val).  With tune, the tile
    threshold comes from the autotuner's cache for the batch's architecture
    and shape bucket (tuned on this batch when the bucket is new)."""
    if not mats:
        return []
    opts = Options(**options)
    if tune:
        from . import autotune
        opts, _ = autotune.tuned_batched_options(mats, eps, base=opts)
    plan = Plan(mats[0][2].device, opts)
    try:
        return plan.expm_batched(mats, eps)
    finally:
        plan.close()
