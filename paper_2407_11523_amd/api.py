"""Python binding of the bp4 C ABI: argument marshalling over torch device tensors.

Every computation runs in the HIP kernels of libbp4.so; this module only
allocates torch tensors, passes their pointers and the current stream, and
turns error codes into exceptions.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from ._lib import BP4Error, CodeBatch as _CCodeBatch, Params as _CParams, Tuning as _CTuning, check, load

VARIANTS = {"bp": 0, "momentum": 1, "adagrad": 2, "ewainit": 3, "aewa": 4}
ALLOW_ANTICOMMUTING = 1


def _stream(device=None) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _ptr(t: Optional[torch.Tensor]) -> ctypes.c_void_p:
    return ctypes.c_void_p(0 if t is None else t.data_ptr())


def _u8(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.uint8)


@dataclass
class Params:
    """Decoder hyperparameters (section III of the paper)."""
    variant: str = "bp"
    max_iter: int = 100
    stop_on_syndrome: bool = True
    adagrad_g_from_t1: bool = False
    alpha: float = 1.0
    gamma: float = 0.0
    eps: float = 1e-8
    llr_clamp: float = 30.0
    alpha_last: float = 0.0   # AEWA: discount of the last attempt (alpha is the first)
    alpha_steps: int = 11     # AEWA: number of attempts
    serial: bool = False      # serial schedule (Algorithm 1) instead of flooding (Algorithm 2)

    def c(self) -> _CParams:
        return _CParams(VARIANTS[self.variant], int(self.max_iter), int(bool(self.stop_on_syndrome)),
                        int(bool(self.adagrad_g_from_t1)), float(self.alpha), float(self.gamma),
                        float(self.eps), float(self.llr_clamp), float(self.alpha_last), int(self.alpha_steps),
                        int(bool(self.serial)))


class Graph:
    """A code's Tanner graph: host object plus its uploaded device image."""

    def __init__(self, hx, hz, lx=None, lz=None, *, allow_anticommuting: bool = False,
                 device: Optional[torch.device] = None, upload: bool = True, coords=None):
        lib = load()
        hx, hz = _u8(hx), _u8(hz)
        if hx.ndim != 2 or hx.shape != hz.shape:
            raise BP4Error(-1, "hx and hz must be 2-D arrays of one shape")
        m, n = hx.shape
        h = ctypes.c_void_p()
        check(lib.bp4_graph_create(hx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   hz.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)), m, n,
                                   ALLOW_ANTICOMMUTING if allow_anticommuting else 0, ctypes.byref(h)))
        self._h = h
        self._lib = lib
        vals = [ctypes.c_int32() for _ in range(5)]
        check(lib.bp4_graph_info(h, *[ctypes.byref(v) for v in vals]))
        self.n, self.m, self.nnz, self.max_cdeg, self.max_vdeg = (int(v.value) for v in vals)
        self.nlog = 0
        if lx is not None:
            self.set_logicals(lx, lz)
        self.dev = None
        if coords is not None:
            self.set_coords(coords)
        if upload:
            self.upload(device)

    def set_logicals(self, lx, lz) -> None:
        lx, lz = _u8(lx), _u8(lz)
        check(self._lib.bp4_graph_set_logicals(self._h, lx.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                               lz.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                               int(lx.shape[0])))
        self.nlog = int(lx.shape[0])
        if getattr(self, "dev", None) is not None:
            self.upload(self.dev.device)

    def set_coords(self, coords) -> None:
        """Qubit positions [n][2] on a 2-D layout: a locality hint for the single-pass
        HBM kernel's walk order (results do not depend on it)."""
        xy = np.ascontiguousarray(np.asarray(coords), dtype=np.int32)
        if xy.shape != (self.n, 2):
            raise BP4Error(-1, f"coords must have shape ({self.n}, 2), got {xy.shape}")
        check(self._lib.bp4_graph_set_coords(self._h, xy.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        if getattr(self, "dev", None) is not None:
            self.upload(self.dev.device)

    def device_bytes(self) -> int:
        b = ctypes.c_size_t()
        check(self._lib.bp4_graph_device_bytes(self._h, ctypes.byref(b)))
        return int(b.value)

    def upload(self, device=None) -> None:
        device = torch.device(device if device is not None else "cuda")
        buf = torch.empty(self.device_bytes(), dtype=torch.uint8, device=device)
        check(self._lib.bp4_graph_upload(self._h, _ptr(buf), buf.numel(), _stream(device)))
        self.dev = buf

    def edges(self):
        """(check, qubit) of every edge in canonical (row-major) order."""
        c = np.zeros(self.nnz, np.int32)
        q = np.zeros(self.nnz, np.int32)
        check(self._lib.bp4_graph_edges(self._h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                        q.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))))
        return c, q

    def workspace_bytes(self, params: Params, shots: int) -> int:
        b = ctypes.c_size_t()
        cp = params.c()
        check(self._lib.bp4_workspace_bytes(self._h, ctypes.byref(cp), int(shots), ctypes.byref(b)))
        return int(b.value)

    def soa_workspace_bytes(self, params: Params, shots: int, soa_lanes: int = 0) -> int:
        b = ctypes.c_size_t()
        cp = params.c()
        check(self._lib.bp4_soa_workspace_bytes(self._h, ctypes.byref(cp), int(shots), int(soa_lanes),
                                                ctypes.byref(b)))
        return int(b.value)

    def gather_workspace_bytes(self, params: Params, shots: int, gather_waves: int = 0) -> int:
        b = ctypes.c_size_t()
        cp = params.c()
        check(self._lib.bp4_gather_workspace_bytes(self._h, ctypes.byref(cp), int(shots), int(gather_waves),
                                                   ctypes.byref(b)))
        return int(b.value)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            self._lib.bp4_graph_destroy(h)
            self._h = None


def prior_llr(probs, device=None) -> torch.Tensor:
    """Pi_{v,W} = ln(p^I / p^W) (section II-B1) as a float32 [n][3] device tensor,
    computed by the library's kernel (bp4_prior_llr) from probabilities (p_X, p_Y, p_Z)."""
    probs = np.ascontiguousarray(probs, dtype=np.float64)
    if probs.ndim != 2 or probs.shape[1] != 3 or probs.shape[0] < 1:
        raise BP4Error(-1, "probs must be an [n][3] array of (p_X, p_Y, p_Z)")
    if not np.all(np.isfinite(probs)) or np.any(probs <= 0.0) or np.any(probs.sum(axis=1) >= 1.0):
        raise BP4Error(-1, "probs must be finite, positive, and sum to less than 1 per qubit")
    dev = torch.device(device if device is not None else "cuda")
    p_dev = torch.as_tensor(probs, device=dev)
    out = torch.empty((probs.shape[0], 3), dtype=torch.float32, device=dev)
    # p_dev is released after the launch, on the stream the kernel runs on: torch's
    # caching allocator hands the block out again only in that stream's order
    check(load().bp4_prior_llr(int(probs.shape[0]), _ptr(p_dev), _ptr(out), _stream(dev)))
    return out


def sample(g: Graph, shots: int, thr, seed: int, stream_id: int = 0, shot0: int = 0,
           err: Optional[torch.Tensor] = None, synd: Optional[torch.Tensor] = None):
    """Errors [shots][n] and syndromes [shots][m] (uint8 device tensors)."""
    dev = g.dev.device
    if err is None:
        err = torch.empty((shots, g.n), dtype=torch.uint8, device=dev)
    if synd is None:
        synd = torch.empty((shots, g.m), dtype=torch.uint8, device=dev)
    t = (ctypes.c_uint32 * 3)(*[int(x) for x in thr])
    check(g._lib.bp4_sample(g.handle, _ptr(g.dev), int(shots), int(shot0), t,
                            ctypes.c_uint64(seed & (2 ** 64 - 1)), ctypes.c_uint64(stream_id & (2 ** 64 - 1)),
                            _ptr(err), _ptr(synd), _stream(dev)))
    return err, synd


KERNELS = {"auto": 0, "lds": 1, "soa": 2, "gather": 3}


def decode(g: Graph, params: Params, prior: torch.Tensor, synd: torch.Tensor, *, trace: bool = False,
           group_lanes: int = 0, block_shots: int = 0, lds_bytes: int = 0, kernel: str = "auto",
           soa_lanes: int = 0, soa_iter_block: int = 0, gather_waves: int = 0, out: Optional[dict] = None,
           ws: Optional[torch.Tensor] = None):
    """Decode syndromes [shots][m]; returns dict(est, conv, iters[, q, mvc, mcv]).

    group_lanes (4..64: lanes of one wavefront per shot) or block_shots (shots
    sharing a 512-lane workgroup) force the LDS kernel's lane mapping (0 and 0:
    automatic); lds_bytes reserves at least that much LDS per workgroup; kernel picks the
    LDS ("lds"), the two-phase structure-of-arrays ("soa") or the single-pass
    HBM ("gather") kernel ("auto": by code size; large codes take "gather"
    unless trace or serial asks for "soa"); soa_lanes sets the shots the
    SOA kernel keeps in flight and soa_iter_block its iterations per launch,
    gather_waves the wavefronts per workgroup of the single-pass kernel (0:
    defaults)."""
    dev = g.dev.device
    if synd.dtype != torch.uint8 or synd.dim() != 2 or synd.shape[1] != g.m or not synd.is_contiguous():
        raise BP4Error(-1, "synd must be a contiguous uint8 [shots][m] tensor")
    if prior.dtype != torch.float32 or tuple(prior.shape) != (g.n, 3) or not prior.is_contiguous():
        raise BP4Error(-1, "prior must be a contiguous float32 [n][3] tensor")
    shots = synd.shape[0]
    o = out if out is not None else {}
    est = o.get("est")
    if est is None:
        est = torch.empty((shots, g.n), dtype=torch.uint8, device=dev)
    conv = o.get("conv")
    if conv is None:
        conv = torch.empty(shots, dtype=torch.uint8, device=dev)
    iters = o.get("iters")
    if iters is None:
        iters = torch.empty(shots, dtype=torch.int32, device=dev)
    cp = params.c()
    if ws is None:
        if kernel == "soa" or soa_lanes or soa_iter_block:
            nbytes = g.soa_workspace_bytes(params, shots, soa_lanes)
        elif kernel == "gather" or gather_waves:
            nbytes = g.gather_workspace_bytes(params, shots, gather_waves)
        else:
            nbytes = g.workspace_bytes(params, shots)
            if trace and kernel == "auto":   # a large code then runs the SOA kernel
                nbytes = max(nbytes, g.soa_workspace_bytes(params, shots, 0))
        ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    res = {"est": est, "conv": conv, "iters": iters}
    if (trace or group_lanes or block_shots or lds_bytes or soa_lanes or soa_iter_block or gather_waves
            or kernel != "auto"):
        q = mvc = mcv = None
        if trace:
            q = torch.empty((shots, g.n, 3), dtype=torch.float32, device=dev)
            mvc = torch.empty((shots, g.nnz), dtype=torch.float32, device=dev)
            mcv = torch.empty((shots, g.nnz), dtype=torch.float32, device=dev)
            res.update(q=q, mvc=mvc, mcv=mcv)
        tune = _CTuning(int(group_lanes), int(lds_bytes), KERNELS[kernel], int(soa_lanes), int(soa_iter_block),
                        int(block_shots), int(gather_waves))
        check(g._lib.bp4_decode_ex(g.handle, _ptr(g.dev), ctypes.byref(cp), ctypes.byref(tune), shots,
                                   _ptr(prior), _ptr(synd), _ptr(est), _ptr(conv), _ptr(iters), _ptr(q),
                                   _ptr(mvc), _ptr(mcv), _ptr(ws), ws.numel(), _stream(dev)))
    else:
        check(g._lib.bp4_decode(g.handle, _ptr(g.dev), ctypes.byref(cp), shots, _ptr(prior), _ptr(synd),
                                _ptr(est), _ptr(conv), _ptr(iters), _ptr(ws), ws.numel(), _stream(dev)))
    return res


def bookkeep(g: Graph, err: torch.Tensor, est: torch.Tensor, counts: Optional[torch.Tensor] = None):
    """Per-shot class (0 ok, 1 detected, 2 undetected) and int64[3] class counts."""
    dev = g.dev.device
    shots = err.shape[0]
    fail = torch.empty(shots, dtype=torch.uint8, device=dev)
    if counts is None:
        counts = torch.zeros(3, dtype=torch.int64, device=dev)
    check(g._lib.bp4_bookkeep(g.handle, _ptr(g.dev), shots, _ptr(err), _ptr(est), _ptr(fail), _ptr(counts),
                              _stream(dev)))
    return fail, counts


def _outputs(g: Graph, shots: int, out: Optional[dict]):
    dev = g.dev.device
    o = out if out is not None else {}
    est = o.get("est")
    if est is None:
        est = torch.empty((shots, g.n), dtype=torch.uint8, device=dev)
    conv = o.get("conv")
    if conv is None:
        conv = torch.empty(shots, dtype=torch.uint8, device=dev)
    iters = o.get("iters")
    if iters is None:
        iters = torch.empty(shots, dtype=torch.int32, device=dev)
    return {"est": est, "conv": conv, "iters": iters}


def _check_inputs(g: Graph, prior: torch.Tensor, synd: torch.Tensor):
    if synd.dtype != torch.uint8 or synd.dim() != 2 or synd.shape[1] != g.m or not synd.is_contiguous():
        raise BP4Error(-1, "synd must be a contiguous uint8 [shots][m] tensor")
    if prior.dtype != torch.float32 or tuple(prior.shape) != (g.n, 3) or not prior.is_contiguous():
        raise BP4Error(-1, "prior must be a contiguous float32 [n][3] tensor")


class MixedBatch:
    """Codes decoded together by one persistent launch (bp4_decode_mixed).

    Each entry is (graph, params, prior [n][3], synd [shots][m], lanes), lanes =
    group_lanes or (group_lanes, block_shots) as in decode(); the outputs are
    allocated once and reused by every call of run()."""

    def __init__(self, entries, outs=None):
        self.entries = list(entries)
        if not 1 <= len(self.entries) <= 16:
            raise BP4Error(-1, "a mixed batch holds 1 to 16 codes")
        self.outs = []
        arr = (_CCodeBatch * len(self.entries))()
        for i, (g, params, prior, synd, lanes) in enumerate(self.entries):
            _check_inputs(g, prior, synd)
            o = _outputs(g, synd.shape[0], outs[i] if outs else None)
            self.outs.append(o)
            G, S = (lanes if isinstance(lanes, (tuple, list)) else (lanes, 0))
            arr[i] = _CCodeBatch(g.handle.value, g.dev.data_ptr(), params.c(), synd.shape[0], prior.data_ptr(),
                                 synd.data_ptr(), o["est"].data_ptr(), o["conv"].data_ptr(),
                                 o["iters"].data_ptr(), int(G), int(S))
        self._arr = arr
        lib = load()
        b = ctypes.c_size_t()
        check(lib.bp4_mixed_workspace_bytes(len(self.entries), ctypes.byref(b)))
        self.ws = torch.empty(int(b.value), dtype=torch.uint8, device=self.entries[0][0].dev.device)

    def run(self):
        lib = load()
        check(lib.bp4_decode_mixed(len(self.entries), self._arr, _ptr(self.ws), self.ws.numel(),
                                   _stream(self.ws.device)))
        return self.outs


def decode_mixed(entries):
    """Decode several codes in one persistent launch; returns one output dict per code."""
    return MixedBatch(entries).run()


def decode_plain(g: Graph, params: Params, prior: torch.Tensor, synd: torch.Tensor, *,
                 out: Optional[dict] = None, ws: Optional[torch.Tensor] = None):
    """The textbook per-phase GPU decoder (bp4_decode_plain); blocks until done."""
    _check_inputs(g, prior, synd)
    dev = g.dev.device
    shots = synd.shape[0]
    res = _outputs(g, shots, out)
    cp = params.c()
    if ws is None:
        b = ctypes.c_size_t()
        check(g._lib.bp4_plain_workspace_bytes(g.handle, ctypes.byref(cp), shots, ctypes.byref(b)))
        ws = torch.empty(int(b.value), dtype=torch.uint8, device=dev)
    it = ctypes.c_int32()
    check(g._lib.bp4_decode_plain(g.handle, _ptr(g.dev), ctypes.byref(cp), shots, _ptr(prior), _ptr(synd),
                                  _ptr(res["est"]), _ptr(res["conv"]), _ptr(res["iters"]), _ptr(ws), ws.numel(),
                                  _stream(dev), ctypes.byref(it)))
    res["iterations_run"] = int(it.value)
    return res


class Captured:
    """Library calls recorded once as a HIP graph (torch.cuda.CUDAGraph) and replayed.

    fn issues library calls on the current stream with buffers that outlive the
    graph; inputs written into those buffers between replays are what the next
    replay reads.  decode (both kernels, and the SOA kernel's iteration blocks with
    their packing steps), decode_mixed, sample, bookkeep and the unrolled forward and
    backward launch kernels only (queue heads and counters are cleared by a fill
    kernel, never by a memset), so they can be captured; decode_plain cannot (its host
    loop reads a device counter every iteration)."""

    def __init__(self, fn, warmup: int = 1):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.result = fn()

    def replay(self):
        self.graph.replay()
        return self.result


# ---------------------------------------------------------------------------
# Differentiable unrolled EWAInit-BP and Momentum-BP
# ---------------------------------------------------------------------------

# per-iteration parameters of each unrolled variant: EWAInit alpha_t [T]; Momentum
# (alpha_t, gamma_t) [T, 2]
UNROLLED_PARAMS = {"ewainit": 1, "momentum": 2}


def unrolled_sizes(g: Graph, T: int, ckpt_every: int, shots: int, variant: str = "ewainit"):
    """(checkpoint bytes, workspace bytes) of the unrolled forward/backward."""
    a, b = ctypes.c_size_t(), ctypes.c_size_t()
    check(g._lib.bp4_unrolled_sizes(g.handle, VARIANTS[variant], int(T), int(ckpt_every), int(shots),
                                    ctypes.byref(a), ctypes.byref(b)))
    return int(a.value), int(b.value)


def _unrolled_inputs(g: Graph, params, prior, synd, err, T: int, variant: str):
    """Validated, contiguous device inputs of the unrolled kernels: params float32 [T]
    (EWAInit) or [T, 2] (Momentum), prior float32 [n, 3], synd uint8 [shots, m], err uint8
    [shots, n] on the graph's device."""
    dev = g.dev.device
    if variant not in UNROLLED_PARAMS:
        raise BP4Error(-6, f"the unrolled path is built for {sorted(UNROLLED_PARAMS)}, not {variant}")
    for name, t in (("params", params), ("prior", prior), ("synd", synd), ("err", err)):
        if not isinstance(t, torch.Tensor) or t.device != dev:
            raise BP4Error(-1, f"{name} must be a tensor on {dev}")
    if synd.dtype != torch.uint8 or err.dtype != torch.uint8:
        raise BP4Error(-1, "synd and err must be uint8 tensors")
    if synd.dim() != 2 or synd.shape[1] != g.m or synd.shape[0] < 1:
        raise BP4Error(-1, "synd must be [shots, m] with shots >= 1")
    if tuple(err.shape) != (synd.shape[0], g.n):
        raise BP4Error(-1, "err must be [shots, n]")
    k = UNROLLED_PARAMS[variant]
    want = (int(T),) if k == 1 else (int(T), k)
    if tuple(params.shape) != want or tuple(prior.shape) != (g.n, 3):
        raise BP4Error(-1, f"{variant} parameters must be {list(want)} and prior [n, 3]")
    if not (params.is_floating_point() and prior.is_floating_point()):
        raise BP4Error(-1, "parameters and prior must be floating point")
    return (params.detach().to(torch.float32).contiguous(), prior.detach().to(torch.float32).contiguous(),
            synd.contiguous(), err.contiguous())


class UnrolledBP(torch.autograd.Function):
    """Soft loss of T unrolled EWAInit-BP or Momentum-BP iterations (HIP forward and
    hand-written adjoint).

    forward(params, prior [n, 3], graph, synd, err, T, ckpt_every, clamp, variant):
    params is EWAInit's discounts alpha_t [T] or Momentum's steps and decays
    (alpha_t, gamma_t) [T, 2]; returns the mean over shots and qubits of
    ln(1 + sum_W e^{-Q_W}) + Q_{e_v} at t = T as a float64 scalar; backward gives the
    gradients of params and prior."""

    @staticmethod
    def forward(ctx, params, prior, g, synd, err, T, ckpt_every, clamp, variant):
        dev = synd.device
        p32, pr32, syn, er = _unrolled_inputs(g, params, prior, synd, err, T, variant)
        shots = syn.shape[0]
        sb, wb = unrolled_sizes(g, T, ckpt_every, shots, variant)
        saved = torch.empty(sb, dtype=torch.uint8, device=dev)
        ws = torch.empty(wb, dtype=torch.uint8, device=dev)
        loss = torch.empty(1, dtype=torch.float64, device=dev)
        check(g._lib.bp4_unrolled_forward(g.handle, _ptr(g.dev), VARIANTS[variant], int(T), int(ckpt_every),
                                          float(clamp), shots, _ptr(p32), _ptr(pr32), _ptr(syn), _ptr(er),
                                          _ptr(loss), ctypes.c_void_p(0), _ptr(saved), sb, _ptr(ws), wb,
                                          _stream(dev)))
        ctx.g, ctx.T, ctx.K, ctx.clamp, ctx.variant = g, int(T), int(ckpt_every), float(clamp), variant
        ctx.bufs = (p32, pr32, syn, er, saved, ws)
        ctx.dtypes = (params.dtype, prior.dtype)
        return loss[0]

    @staticmethod
    def backward(ctx, dloss):
        params, prior, synd, err, saved, ws = ctx.bufs
        g = ctx.g
        dev = synd.device
        dl = dloss.detach().to(device=dev, dtype=torch.float32).reshape(1).contiguous()
        dparams = torch.empty(params.shape, dtype=torch.float64, device=dev)
        dprior = torch.empty(g.n, 3, dtype=torch.float64, device=dev)
        check(g._lib.bp4_unrolled_backward(g.handle, _ptr(g.dev), VARIANTS[ctx.variant], ctx.T, ctx.K, ctx.clamp,
                                           synd.shape[0], _ptr(params), _ptr(prior), _ptr(synd), _ptr(err), _ptr(dl),
                                           _ptr(saved), saved.numel(), _ptr(dparams), _ptr(dprior), _ptr(ws),
                                           ws.numel(), _stream(dev)))
        ctx.bufs = None
        return dparams.to(ctx.dtypes[0]), dprior.to(ctx.dtypes[1]), None, None, None, None, None, None, None


class UnrolledEWAInit(torch.autograd.Function):
    """UnrolledBP for EWAInit: forward(alpha [T], prior [n, 3], graph, synd, err, T,
    ckpt_every, clamp)."""

    @staticmethod
    def forward(ctx, alpha, prior, g, synd, err, T, ckpt_every, clamp):
        return UnrolledBP.forward(ctx, alpha, prior, g, synd, err, T, ckpt_every, clamp, "ewainit")

    @staticmethod
    def backward(ctx, dloss):
        return UnrolledBP.backward(ctx, dloss)[:8]


def unrolled_loss(g: Graph, params: torch.Tensor, prior: torch.Tensor, synd: torch.Tensor, err: torch.Tensor,
                  T: int, ckpt_every: int = 8, clamp: float = 30.0, variant: str = "ewainit") -> torch.Tensor:
    """Differentiable soft loss of T unrolled iterations of `variant` (see UnrolledBP)."""
    return UnrolledBP.apply(params, prior, g, synd, err, T, ckpt_every, clamp, variant)


def unrolled_forward(g: Graph, params: torch.Tensor, prior: torch.Tensor, synd: torch.Tensor, err: torch.Tensor,
                     T: int, ckpt_every: int = 8, clamp: float = 30.0, want_q: bool = False,
                     variant: str = "ewainit"):
    """Forward only: (loss float64 [1], Q^{(T)} [shots, n, 3] or None)."""
    dev = synd.device
    p32, pr32, syn, er = _unrolled_inputs(g, params, prior, synd, err, T, variant)
    shots = syn.shape[0]
    sb, wb = unrolled_sizes(g, T, ckpt_every, shots, variant)
    saved = torch.empty(sb, dtype=torch.uint8, device=dev)
    ws = torch.empty(wb, dtype=torch.uint8, device=dev)
    loss = torch.empty(1, dtype=torch.float64, device=dev)
    q = torch.empty(shots, g.n, 3, dtype=torch.float32, device=dev) if want_q else None
    check(g._lib.bp4_unrolled_forward(g.handle, _ptr(g.dev), VARIANTS[variant], int(T), int(ckpt_every),
                                      float(clamp), shots, _ptr(p32), _ptr(pr32), _ptr(syn), _ptr(er), _ptr(loss),
                                      _ptr(q), _ptr(saved), sb, _ptr(ws), wb, _stream(dev)))
    # the contiguous copies are named, so none is freed (and reused) before the launch
    return loss, q
