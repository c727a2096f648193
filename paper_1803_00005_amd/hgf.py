"""Python binding of libhgf.so (ctypes; argument marshalling only).

Every step of the filter runs in the library's HIP kernels.  PyTorch supplies
device memory (``torch.empty(..., device="cuda")``) and the current stream.
There is no fallback: if the library is not built, or no GPU is present,
the calls raise.

Names follow include/hgf.h.  Layouts: guide float32 [m][H][W]; cost float32,
bfloat16 or float16 [H][W][L] (labels contiguous); filtered costs float32
[H][W][L]; labels int32 [H][W].
"""
from __future__ import annotations

import ctypes
import os
import re
from typing import Optional, Sequence

import torch  # imported before the library so both share one HIP runtime

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libhgf.so")
HEADER_PATH = os.path.join(os.path.dirname(_PKG), "include", "hgf.h")

HGF_OK, HGF_E_INVALID, HGF_E_NOMEM, HGF_E_DEVICE, HGF_E_UNSUPPORTED, HGF_E_BUSY = 0, -1, -2, -3, -4, -5
HGF_F32, HGF_BF16, HGF_F16, HGF_F64 = 0, 1, 2, 3
COST_DTYPES = {"f32": HGF_F32, "bf16": HGF_BF16, "f16": HGF_F16}
STATS_DTYPES = {"f32": HGF_F32, "f64": HGF_F64}
BASIS = {"monomial": 0, "power": 1}
REG = {"covariance": 0, "ridge": 1}
STAGES = ["guide_mean", "guide_synth", "guide_moments", "guide_invert", "coef", "out_wta", "wta_keys"]


class HGFError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Completion(ctypes.Structure):
    _fields_ = [("id", ctypes.c_int64), ("status", ctypes.c_int32), ("slot", ctypes.c_int32),
                ("start_ms", ctypes.c_double), ("end_ms", ctypes.c_double)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("pending", ctypes.c_int32), ("running", ctypes.c_int32),
                ("completed", ctypes.c_int64), ("arena_bytes", ctypes.c_size_t),
                ("arena_in_use", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t)]


class Params(ctypes.Structure):
    _fields_ = [
        ("height", ctypes.c_int32), ("width", ctypes.c_int32),
        ("guide_channels", ctypes.c_int32), ("degree", ctypes.c_int32),
        ("basis", ctypes.c_int32), ("reg", ctypes.c_int32),
        ("radius", ctypes.c_int32), ("num_labels", ctypes.c_int32),
        ("eps", ctypes.c_double),
        ("cost_dtype", ctypes.c_int32), ("cost_ld", ctypes.c_int32),
        ("out_ld", ctypes.c_int32), ("stats_dtype", ctypes.c_int32),
    ]


def make_params(height: int, width: int, labels: int, *, radius: int, eps: float, degree: int,
                guide_channels: int = 3, basis: str = "monomial", reg: str = "covariance",
                cost_dtype: str = "f32", cost_ld: int = 0, out_ld: int = 0,
                stats_dtype: str = "f32") -> Params:
    return Params(height, width, guide_channels, degree, BASIS[basis], REG[reg], radius, labels,
                  float(eps), COST_DTYPES[cost_dtype], cost_ld, out_ld, STATS_DTYPES[stats_dtype])


_TORCH_COST = {torch.float32: "f32", torch.bfloat16: "bf16", torch.float16: "f16"}
_COST_TYPES = tuple(_TORCH_COST)


def cost_dtype_of(t: torch.Tensor) -> str:
    return _TORCH_COST[t.dtype]


_lib = None
_vp = ctypes.c_void_p


def _declare(lib):
    P = ctypes.POINTER(Params)
    sig = {
        "hgf_num_channels": (ctypes.c_int32, [ctypes.c_int32] * 3),
        "hgf_is_supported": (ctypes.c_int32, [ctypes.c_int32] * 3),
        "hgf_create": (ctypes.c_int, [ctypes.c_int32, ctypes.c_size_t, ctypes.POINTER(_vp)]),
        "hgf_destroy": (None, [_vp]),
        "hgf_workspace_size": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "hgf_set_group_bytes": (ctypes.c_int, [_vp, ctypes.c_size_t]),
        "hgf_filter": (ctypes.c_int, [_vp, P, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "hgf_guide_create": (ctypes.c_int, [_vp, P, _vp, _vp, ctypes.POINTER(_vp)]),
        "hgf_guide_filter": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, _vp, _vp, _vp, _vp]),
        "hgf_guide_bytes": (ctypes.c_size_t, [_vp]),
        "hgf_guide_destroy": (None, [_vp]),
        "hgf_guide_export": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp]),
        "hgf_filter_batch": (ctypes.c_int, [_vp, ctypes.c_int32, P, _vp, _vp, _vp, _vp, _vp]),
        "hgf_autotune": (ctypes.c_int, [_vp, P, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp]),
        "hgf_tune_entries": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
        "hgf_tune_set": (ctypes.c_int, [_vp, _vp]),
        "hgf_tune_save": (ctypes.c_int, [_vp, ctypes.c_char_p]),
        "hgf_tune_load": (ctypes.c_int, [_vp, ctypes.c_char_p]),
        "hgf_server_create": (ctypes.c_int, [_vp, ctypes.c_int32, ctypes.c_size_t, ctypes.c_int32,
                                             ctypes.POINTER(_vp)]),
        "hgf_server_destroy": (None, [_vp]),
        "hgf_server_submit": (ctypes.c_int, [_vp, P, _vp, _vp, _vp, _vp, _vp,
                                             ctypes.POINTER(ctypes.c_int64)]),
        "hgf_server_poll": (ctypes.c_int, [_vp, ctypes.POINTER(Completion), ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_int32)]),
        "hgf_server_drain": (ctypes.c_int, [_vp]),
        "hgf_server_stats": (ctypes.c_int, [_vp, ctypes.POINTER(ServerInfo)]),
        "hgf_server_now": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_double)]),
        "hgf_filter_static": (ctypes.c_int, [_vp, P, _vp, _vp, _vp, _vp, _vp]),
        "hgf_static_scratch_bytes": (ctypes.c_size_t, []),
        "hgf_box_sum": (ctypes.c_int, [_vp, _vp] + [ctypes.c_int32] * 4 + [_vp]),
        "hgf_spd_inverse": (ctypes.c_int, [_vp, _vp, ctypes.c_int32, ctypes.c_int32, _vp]),
        "hgf_set_stage_timing": (ctypes.c_int, [_vp, ctypes.c_int32]),
        "hgf_stage_times": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32]),
        "hgf_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "hgf_last_error": (ctypes.c_char_p, [_vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() "
                              "(or python -m paper_1803_00005_amd.build_lib) first")
        _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def header_functions() -> list[str]:
    """Names of the functions include/hgf.h declares."""
    text = open(HEADER_PATH).read()
    return sorted(set(re.findall(r"\b(hgf_[a-z_0-9]+)\s*\(", text)))


def _check(status: int, where: str, ctx=None):
    """Raise on a failed call; ``ctx`` is the context handle the call took (its
    detail string), or None for calls without one."""
    if status != HGF_OK:
        detail = lib().hgf_last_error(ctx).decode(errors="replace")
        raise HGFError(status, where, detail)


def num_channels(m: int, d: int, basis: str = "monomial") -> int:
    return int(lib().hgf_num_channels(m, d, BASIS[basis]))


def is_supported(n: int, radius: int, reg: str = "covariance") -> bool:
    return bool(lib().hgf_is_supported(n, radius, REG[reg]))


def workspace_size(params: Params) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().hgf_workspace_size(ctypes.byref(params), ctypes.byref(out)), "hgf_workspace_size")
    return int(out.value)


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _need_cuda(t: torch.Tensor, name: str, dtypes):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Context:
    """A library context on one device (owns scratch memory and resident guides)."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        h = ctypes.c_void_p()
        _check(lib().hgf_create(device, hbm_budget_bytes, ctypes.byref(h)), "hgf_create")
        self.handle = h
        self.device = device

    def close(self):
        if getattr(self, "handle", None):
            lib().hgf_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_group_bytes(self, nbytes: int):
        """Upper bound of one launch group's coefficient workspace (0 = default 12 GiB)."""
        _check(lib().hgf_set_group_bytes(self.handle, nbytes), "hgf_set_group_bytes", self.handle)

    # -- per-stage event timing ---------------------------------------------
    def set_stage_timing(self, enable: bool):
        _check(lib().hgf_set_stage_timing(self.handle, 1 if enable else 0), "hgf_set_stage_timing", self.handle)

    def stage_times(self):
        """{stage name: (milliseconds summed, launches)} since the last call; waits for the events."""
        n = len(STAGES)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int32 * n)()
        _check(lib().hgf_stage_times(self.handle, ms, cnt, n), "hgf_stage_times", self.handle)
        return {STAGES[i]: (float(ms[i]), int(cnt[i])) for i in range(n)}

    # -- plain path ---------------------------------------------------------
    def filter(self, guide: torch.Tensor, cost: torch.Tensor, *, radius: int, eps: float,
               degree: int, basis: str = "monomial", reg: str = "covariance",
               stats_dtype: str = "f32", want_out: bool = True, want_labels: bool = True, out: Optional[torch.Tensor] = None,
               labels: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
               stream=None):
        """Filter every label slice of ``cost`` under ``guide``; returns (Z, labels)."""
        _need_cuda(guide, "guide", (torch.float32,))
        _need_cuda(cost, "cost", _COST_TYPES)
        m, H, W = guide.shape
        if cost.dim() != 3 or cost.shape[0] != H or cost.shape[1] != W:
            raise ValueError("cost must be [H][W][L] with the guide's H and W")
        L = cost.shape[2]
        p = make_params(H, W, L, radius=radius, eps=eps, degree=degree, guide_channels=m,
                        basis=basis, reg=reg,
                        cost_dtype=cost_dtype_of(cost), stats_dtype=stats_dtype)
        if want_out and out is None:
            out = torch.empty((H, W, L), dtype=torch.float32, device=guide.device)
        if want_labels and labels is None:
            labels = torch.empty((H, W), dtype=torch.int32, device=guide.device)
        if workspace is None:
            workspace = torch.empty(workspace_size(p), dtype=torch.uint8, device=guide.device)
        _check(lib().hgf_filter(self.handle, ctypes.byref(p), _ptr(guide), _ptr(cost),
                                _ptr(out if want_out else None),
                                _ptr(labels if want_labels else None), _ptr(workspace),
                                workspace.numel(), _stream(stream)), "hgf_filter", self.handle)
        return (out if want_out else None), (labels if want_labels else None)

    def filter_static(self, guide: torch.Tensor, cost: torch.Tensor, out: torch.Tensor,
                      labels: Optional[torch.Tensor], *, radius: int, eps: float, degree: int,
                      basis: str = "monomial", reg: str = "covariance", stats_dtype: str = "f32",
                      stream=None):
        """hgf_filter_static: the plain filter with the library's static device
        workspace (allocates nothing; the caller gives the outputs)."""
        _need_cuda(guide, "guide", (torch.float32,))
        _need_cuda(cost, "cost", _COST_TYPES)
        m, H, W = guide.shape
        p = make_params(H, W, cost.shape[2], radius=radius, eps=eps, degree=degree,
                        guide_channels=m, basis=basis, reg=reg, cost_dtype=cost_dtype_of(cost),
                        stats_dtype=stats_dtype)
        _check(lib().hgf_filter_static(self.handle, ctypes.byref(p), _ptr(guide), _ptr(cost),
                                       _ptr(out), _ptr(labels), _stream(stream)),
               "hgf_filter_static", self.handle)
        return out, labels

    # -- tuning table ------------------------------------------------------
    def autotune(self, guide: torch.Tensor, cost: torch.Tensor, *, radius: int, eps: float,
                 degree: int, basis: str = "monomial", reg: str = "covariance",
                 stats_dtype: str = "f32",
                 out: Optional[torch.Tensor] = None, stream=None):
        """Time the strip-decomposition candidates on these inputs and keep the fastest."""
        _need_cuda(guide, "guide", (torch.float32,))
        _need_cuda(cost, "cost", _COST_TYPES)
        m, H, W = guide.shape
        L = cost.shape[2]
        p = make_params(H, W, L, radius=radius, eps=eps, degree=degree, guide_channels=m,
                        basis=basis, reg=reg,
                        cost_dtype=cost_dtype_of(cost), stats_dtype=stats_dtype)
        ws = torch.empty(workspace_size(p), dtype=torch.uint8, device=guide.device)
        _check(lib().hgf_autotune(self.handle, ctypes.byref(p), _ptr(guide), _ptr(cost), _ptr(out),
                                  _ptr(ws), ws.numel(), _stream(stream)), "hgf_autotune", self.handle)

    def tune_entries(self) -> list[tuple[int, ...]]:
        """Rows (kernel, n, radius, reg, bf16, size_class, target_blocks) of the tuning table."""
        cnt = ctypes.c_int32(0)
        _check(lib().hgf_tune_entries(self.handle, None, 0, ctypes.byref(cnt)), "hgf_tune_entries", self.handle)
        rows = (ctypes.c_int32 * (7 * max(1, cnt.value)))()
        _check(lib().hgf_tune_entries(self.handle, rows, cnt.value, ctypes.byref(cnt)), "hgf_tune_entries", self.handle)
        return [tuple(int(rows[7 * i + k]) for k in range(7)) for i in range(cnt.value)]

    def tune_set(self, row: Sequence[int]):
        arr = (ctypes.c_int32 * 7)(*row)
        _check(lib().hgf_tune_set(self.handle, arr), "hgf_tune_set", self.handle)

    def tune_save(self, path: str):
        _check(lib().hgf_tune_save(self.handle, os.fsencode(path)), "hgf_tune_save", self.handle)

    def tune_load(self, path: str):
        _check(lib().hgf_tune_load(self.handle, os.fsencode(path)), "hgf_tune_load", self.handle)

    # -- batched path -------------------------------------------------------
    def filter_batch(self, items: Sequence[dict], stream=None, outputs=None):
        """items: dicts with guide, cost, radius, eps, degree[, basis, reg]; returns [(Z, labels)].

        ``outputs`` optionally gives the (Z, labels) tensors to write; a call
        with the same inputs, outputs and parameters as the previous one
        replays the cached graph."""
        n = len(items)
        arr = (Params * n)()
        guides = (ctypes.c_void_p * n)()
        costs = (ctypes.c_void_p * n)()
        outs = (ctypes.c_void_p * n)()
        labs = (ctypes.c_void_p * n)()
        results = []
        for i, it in enumerate(items):
            g, c = it["guide"], it["cost"]
            _need_cuda(g, "guide", (torch.float32,))
            _need_cuda(c, "cost", _COST_TYPES)
            m, H, W = g.shape
            L = c.shape[2]
            arr[i] = make_params(H, W, L, radius=it["radius"], eps=it["eps"], degree=it["degree"],
                                 guide_channels=m, basis=it.get("basis", "monomial"),
                                 reg=it.get("reg", "covariance"),
                                 cost_dtype=cost_dtype_of(c),
                                 stats_dtype=it.get("stats_dtype", "f32"))
            if outputs is not None:
                z, lb = outputs[i]
                _need_cuda(z, "out", (torch.float32,))
                _need_cuda(lb, "labels", (torch.int32,))
                if tuple(z.shape) != (H, W, L) or tuple(lb.shape) != (H, W):
                    raise ValueError(f"outputs[{i}] has the wrong shape")
            else:
                z = torch.empty((H, W, L), dtype=torch.float32, device=g.device)
                lb = torch.empty((H, W), dtype=torch.int32, device=g.device)
            guides[i], costs[i], outs[i], labs[i] = g.data_ptr(), c.data_ptr(), z.data_ptr(), lb.data_ptr()
            results.append((z, lb))
        _check(lib().hgf_filter_batch(self.handle, n, arr, guides, costs, outs, labs,
                                      _stream(stream)), "hgf_filter_batch", self.handle)
        return results


class Server:
    """Serving form: requests filtered as soon as the arena has room (continuous batching)."""

    def __init__(self, ctx: Context, *, slots: int = 4, arena_bytes: int = 8 << 30,
                 max_queue: int = 1024):
        h = ctypes.c_void_p()
        _check(lib().hgf_server_create(ctx.handle, slots, arena_bytes, max_queue, ctypes.byref(h)), "hgf_server_create", ctx.handle)
        self.handle = h
        self.ctx = ctx

    def submit(self, guide: torch.Tensor, cost: torch.Tensor, out: Optional[torch.Tensor],
               labels: Optional[torch.Tensor], *, radius: int, eps: float, degree: int,
               basis: str = "monomial", reg: str = "covariance", stats_dtype: str = "f32",
               stream=None) -> int:
        """Queue one request; the caller keeps every tensor alive until it completes."""
        _need_cuda(guide, "guide", (torch.float32,))
        _need_cuda(cost, "cost", _COST_TYPES)
        m, H, W = guide.shape
        L = cost.shape[2]
        p = make_params(H, W, L, radius=radius, eps=eps, degree=degree, guide_channels=m,
                        basis=basis, reg=reg,
                        cost_dtype=cost_dtype_of(cost), stats_dtype=stats_dtype)
        rid = ctypes.c_int64(-1)
        _check(lib().hgf_server_submit(self.handle, ctypes.byref(p), _ptr(guide), _ptr(cost),
                                       _ptr(out), _ptr(labels), _stream(stream),
                                       ctypes.byref(rid)), "hgf_server_submit", self.ctx.handle)
        return int(rid.value)

    def poll(self, max_done: int = 256) -> list[Completion]:
        buf = (Completion * max_done)()
        cnt = ctypes.c_int32(0)
        _check(lib().hgf_server_poll(self.handle, buf, max_done, ctypes.byref(cnt)), "hgf_server_poll", self.ctx.handle)
        return [buf[i] for i in range(cnt.value)]

    def drain(self):
        _check(lib().hgf_server_drain(self.handle), "hgf_server_drain", self.ctx.handle)

    def now_ms(self) -> float:
        """Device clock in ms since the server was created."""
        t = ctypes.c_double(0.0)
        _check(lib().hgf_server_now(self.handle, ctypes.byref(t)), "hgf_server_now", self.ctx.handle)
        return float(t.value)

    def stats(self) -> dict:
        info = ServerInfo()
        _check(lib().hgf_server_stats(self.handle, ctypes.byref(info)), "hgf_server_stats", self.ctx.handle)
        return {k: int(getattr(info, k)) for k, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "handle", None):
            lib().hgf_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Guide:
    """Guidance statistics resident on the device, reused across label chunks."""

    def __init__(self, ctx: Context, guide: torch.Tensor, *, labels: int, radius: int, eps: float,
                 degree: int, basis: str = "monomial", reg: str = "covariance",
                 cost_dtype: str = "f32", stats_dtype: str = "f32", stream=None):
        _need_cuda(guide, "guide", (torch.float32,))
        m, H, W = guide.shape
        self.ctx = ctx
        self.shape = (H, W)
        self.labels = labels
        self.cost_dtype = cost_dtype
        self.params = make_params(H, W, labels, radius=radius, eps=eps, degree=degree,
                                  guide_channels=m, basis=basis, reg=reg, cost_dtype=cost_dtype,
                                  stats_dtype=stats_dtype)
        h = ctypes.c_void_p()
        _check(lib().hgf_guide_create(ctx.handle, ctypes.byref(self.params), _ptr(guide),
                                      _stream(stream), ctypes.byref(h)), "hgf_guide_create", ctx.handle)
        self.handle = h
        self.n = num_channels(m, degree, basis)
        self.dim = self.n + 1 if reg == "ridge" else self.n

    @property
    def nbytes(self) -> int:
        return int(lib().hgf_guide_bytes(self.handle))

    def filter(self, cost_chunk: torch.Tensor, label_begin: int, *, out: Optional[torch.Tensor] = None,
               best: Optional[torch.Tensor] = None, labels: Optional[torch.Tensor] = None,
               stream=None):
        _need_cuda(cost_chunk, "cost_chunk", _COST_TYPES)
        count = cost_chunk.shape[2]
        _check(lib().hgf_guide_filter(self.ctx.handle, self.handle, _ptr(cost_chunk), label_begin,
                                      count, cost_chunk.shape[2], _ptr(out), _ptr(best),
                                      _ptr(labels), _stream(stream)), "hgf_guide_filter", self.ctx.handle)
        return out, best, labels

    def export(self, stream=None):
        """(mu [H][W][n] float64, packed inverse [H][W][D(D+1)/2] (float32 in the
        covariance form with float32 statistics, float64 otherwise), shift [n]
        float64) as device tensors."""
        H, W = self.shape
        dev = torch.device("cuda", self.ctx.device)
        mu = torch.empty((H, W, self.n), dtype=torch.float64, device=dev)
        mdt = (torch.float32 if self.params.reg == REG["covariance"]
               and self.params.stats_dtype == HGF_F32 else torch.float64)
        minv = torch.empty((H, W, self.dim * (self.dim + 1) // 2), dtype=mdt, device=dev)
        shift = torch.empty((self.n,), dtype=torch.float64, device=dev)
        _check(lib().hgf_guide_export(self.handle, _ptr(mu), _ptr(minv), _ptr(shift),
                                      _stream(stream)), "hgf_guide_export", self.ctx.handle)
        return mu, minv, shift

    def close(self):
        if getattr(self, "handle", None):
            lib().hgf_guide_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def box_sum(x: torch.Tensor, radius: int, stream=None) -> torch.Tensor:
    """Clipped box sum of a float32 [C][H][W] stack."""
    _need_cuda(x, "x", (torch.float32,))
    C, H, W = x.shape
    out = torch.empty_like(x)
    _check(lib().hgf_box_sum(_ptr(x), _ptr(out), C, H, W, radius, _stream(stream)), "hgf_box_sum")
    return out


def spd_inverse(a: torch.Tensor, stream=None) -> torch.Tensor:
    """Inverse of a float64 [count][D][D] stack of SPD matrices by the recursion of Prop. 1."""
    _need_cuda(a, "a", (torch.float64,))
    count, D, D2 = a.shape
    if D != D2:
        raise ValueError("matrices must be square")
    out = torch.empty_like(a)
    _check(lib().hgf_spd_inverse(_ptr(a), _ptr(out), D, count, _stream(stream)), "hgf_spd_inverse")
    return out
