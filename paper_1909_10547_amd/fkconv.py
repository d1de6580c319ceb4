"""Python binding of the fkconv C ABI (``include/fkconv.h``).

Argument marshalling only: numpy arrays become host pointers, torch CUDA
tensors become device pointers, the current torch stream becomes the HIP
stream.  Every computation runs in ``lib/libfkconv.so``; when that library
is missing this module raises instead of falling back to anything else.
The functions keep the C names.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lib", "libfkconv.so")
_lib = None

FK_OK = 0
FK_E_ARG, FK_E_SHAPE, FK_E_GRID, FK_E_HANDLE, FK_E_BUDGET = -1, -2, -3, -4, -5
FK_E_TOO_LARGE, FK_E_HIP, FK_E_NOTPD, FK_E_STATE, FK_E_QUEUE_FULL = -6, -7, -8, -9, -10
FK_DIS, FK_HAD = 1, 2
FK_F32, FK_BF16, FK_FP8E4M3 = 0, 1, 2
FK_QUEUED, FK_RUNNING, FK_DONE, FK_FAILED = 0, 1, 2, 3

DTYPES = {"f32": FK_F32, "bf16": FK_BF16, "e4m3": FK_FP8E4M3}

# name -> (restype, argtypes)
_P, _I32, _I64, _U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
_PI64 = ctypes.POINTER(ctypes.c_int64)
_PI32 = ctypes.POINTER(ctypes.c_int32)
_PU64 = ctypes.POINTER(ctypes.c_uint64)


FK_OPT_KERNELS = 1
FK_KERNELS_STREAM, FK_KERNELS_ITEM = 0, 1


class fk_request(ctypes.Structure):
    _fields_ = [("table", ctypes.c_int64), ("nrep", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("pdf", ctypes.c_void_p),
                ("out", ctypes.c_void_p), ("tag", ctypes.c_uint64),
                ("ready", ctypes.c_void_p)]


SIGNATURES = {
    "fk_create": (_I32, [ctypes.POINTER(_P), _I32, _U64]),
    "fk_destroy": (_I32, [_P]),
    "fk_last_error": (ctypes.c_char_p, [_P]),
    "fk_memory": (_I32, [_P, _PU64, _PU64]),
    "fk_set_option": (_I32, [_P, _I32, _I64]),
    "fk_load_table": (_I32, [_P, _I32, _I32, _I32, _I32, _P, _P, _P, _I32, _PI64]),
    "fk_unload_table": (_I32, [_P, _I64]),
    "fk_group_create": (_I32, [_P, _I32, _P, _PI64]),
    "fk_table_info": (_I32, [_P, _I64, _PI32, _PI32, _PI32, _PI32, _PI32, _PU64]),
    "fk_conv_dis": (_I32, [_P, _I64, _P, _P, _I32, _P, _P]),
    "fk_conv_had": (_I32, [_P, _I64, _P, _P, _I32, _P, _P]),
    "fk_conv_dis_static": (_I32, [_P, _I64, _P, _P, _I32, _P, _P]),
    "fk_conv_backward": (_I32, [_P, _I64, _P, _P, _I32, _P, _I32, _P]),
    "fk_luminosity": (_I32, [_P, _I32, _I32, _P, _P, _I32, _P, _P]),
    "fk_flat_conv_workspace": (_I32, [_P, _I64, _I64, _I64, _PU64]),
    "fk_flat_conv": (_I32, [_P, _I64, _I64, _I64, _P, _P, _P, _P, _U64, _P]),
    "fk_mlp_create": (_I32, [_P, _I32, _I32, _P, _I32, _I32, _P, _P, _PI64, _PI32]),
    "fk_mlp_destroy": (_I32, [_P, _I64]),
    "fk_mlp_forward": (_I32, [_P, _I64, _P, _I32, _P, _P]),
    "fk_mlp_backward": (_I32, [_P, _I64, _P, _P, _I32, _P, _P]),
    "fk_sgd_update": (_I32, [_P, _P, _P, _I64, ctypes.c_float, _P]),
    "fk_load_covariance": (_I32, [_P, _I32, _P, _P, _PI64]),
    "fk_unload_covariance": (_I32, [_P, _I64]),
    "fk_chi2": (_I32, [_P, _I64, _P, _P, _I32, _P, _P, _P]),
    "fk_timing_enable": (_I32, [_P, _I32]),
    "fk_timing_read": (_I32, [_P, _P, _P]),
    "fk_measure_mfma_peak": (_I32, [_P, _I32, ctypes.POINTER(ctypes.c_double)]),
    "fk_serve_start": (_I32, [_P, _I32, _I32, _U64]),
    "fk_serve_stop": (_I32, [_P]),
    "fk_table_set_fallback": (_I32, [_P, _I64, _I64]),
    "fk_table_probe": (_I32, [_P, _I64, _P, _I32, ctypes.c_double, ctypes.POINTER(ctypes.c_double), _P]),
    "fk_submit": (_I32, [_P, ctypes.POINTER(fk_request), _PI64]),
    "fk_poll": (_I32, [_P, _I64, _PI32]),
    "fk_ticket_times": (_I32, [_P, _I64, _PU64, _PU64, _PU64]),
}


class FKError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"fkconv error {code}: {msg}")
        self.code = code


def library_path() -> str:
    return _LIB_PATH


def lib():
    """Load libfkconv.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(f"{_LIB_PATH} is not built; run __graft_entry__.build() "
                               "or python -m paper_1909_10547_amd.build")
        l = ctypes.CDLL(_LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(l, name)
            f.restype = res
            f.argtypes = args
        _lib = l
    return _lib


def _check(ctx, st: int):
    if st != FK_OK:
        msg = lib().fk_last_error(ctx)
        raise FKError(st, msg.decode() if msg else "")


def _stream(stream):
    import torch
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype_name: str, what: str):
    import torch
    want = {"f32": torch.float32, "f64": torch.float64}[dtype_name]
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype != want or not t.is_contiguous():
        raise TypeError(f"{what} must be a contiguous {want} tensor")
    return ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# context
# ---------------------------------------------------------------------------

def fk_create(device: int = 0, hbm_budget_bytes: int = 0):
    ctx = ctypes.c_void_p()
    st = lib().fk_create(ctypes.byref(ctx), device, hbm_budget_bytes)
    if st != FK_OK:
        raise FKError(st, lib().fk_last_error(None).decode())
    return ctx


def fk_destroy(ctx):
    _check(ctx, lib().fk_destroy(ctx))


def fk_last_error(ctx) -> str:
    m = lib().fk_last_error(ctx)
    return m.decode() if m else ""


def fk_memory(ctx):
    u, b = ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, lib().fk_memory(ctx, ctypes.byref(u), ctypes.byref(b)))
    return u.value, b.value


def fk_set_option(ctx, option: int, value: int):
    _check(ctx, lib().fk_set_option(ctx, option, value))


# ---------------------------------------------------------------------------
# tables
# ---------------------------------------------------------------------------

def fk_load_table(ctx, kind: int, xgrid, mask, fk, store_dtype) -> int:
    """fk: DIS [N][nact][X] or hadronic [N][npairs][X][X] float64 (active blocks)."""
    if isinstance(store_dtype, str):
        store_dtype = DTYPES[store_dtype]
    xg = np.ascontiguousarray(xgrid, dtype=np.float64)
    mk = np.ascontiguousarray(mask, dtype=np.uint8)
    fkv = np.ascontiguousarray(fk, dtype=np.float64)
    nflav = mk.shape[0]
    h = ctypes.c_int64()
    _check(ctx, lib().fk_load_table(ctx, kind, fkv.shape[0], nflav, xg.shape[0], _hptr(xg),
                                    _hptr(mk), _hptr(fkv), store_dtype, ctypes.byref(h)))
    return h.value


def fk_unload_table(ctx, table: int):
    _check(ctx, lib().fk_unload_table(ctx, table))


def fk_group_create(ctx, tables: Sequence[int]) -> int:
    arr = np.ascontiguousarray(tables, dtype=np.int64)
    h = ctypes.c_int64()
    _check(ctx, lib().fk_group_create(ctx, len(arr), _hptr(arr), ctypes.byref(h)))
    return h.value


def fk_table_info(ctx, table: int) -> dict:
    v = [ctypes.c_int32() for _ in range(5)]
    b = ctypes.c_uint64()
    _check(ctx, lib().fk_table_info(ctx, table, *[ctypes.byref(x) for x in v], ctypes.byref(b)))
    return dict(kind=v[0].value, ndata=v[1].value, nflav=v[2].value, nx=v[3].value,
                store_dtype=v[4].value, device_bytes=b.value)


# ---------------------------------------------------------------------------
# convolutions
# ---------------------------------------------------------------------------

def _conv(fn, ctx, table, pdf, out, pdf_xgrid, stream):
    import torch
    info = fk_table_info(ctx, table)
    if pdf.dim() != 3 or pdf.shape[0] != info["nflav"] or pdf.shape[1] != info["nx"]:
        raise ValueError(f"pdf must be [{info['nflav']}][{info['nx']}][R], got {tuple(pdf.shape)}")
    R = pdf.shape[2]
    if out is None:
        out = torch.empty((info["ndata"], R), dtype=torch.float32, device=pdf.device)
    if tuple(out.shape) != (info["ndata"], R):
        raise ValueError(f"out must be [{info['ndata']}][{R}]")
    xg = None
    if pdf_xgrid is not None:
        xg = np.ascontiguousarray(pdf_xgrid, dtype=np.float64)
        if xg.shape != (info["nx"],):
            raise ValueError("pdf_xgrid has the wrong length")
    _check(ctx, fn(ctx, table, _hptr(xg) if xg is not None else None,
                   _dptr(pdf, "f32", "pdf"), R, _dptr(out, "f32", "out"), _stream(stream)))
    return out


def fk_conv_dis(ctx, table: int, pdf, out=None, pdf_xgrid=None, stream=None):
    return _conv(lib().fk_conv_dis, ctx, table, pdf, out, pdf_xgrid, stream)


def fk_conv_dis_static(ctx, table: int, pdf, out=None, pdf_xgrid=None, stream=None):
    """fk_conv_dis with the staged operand in the library's static scratch
    (allocates no device memory in the library; calls on one GPU must not
    overlap)."""
    return _conv(lib().fk_conv_dis_static, ctx, table, pdf, out, pdf_xgrid, stream)


def fk_conv_had(ctx, table: int, pdf, out=None, pdf_xgrid=None, stream=None):
    return _conv(lib().fk_conv_had, ctx, table, pdf, out, pdf_xgrid, stream)


def fk_conv_backward(ctx, table: int, pdf, grad_out, grad_pdf=None, accumulate=False,
                     stream=None):
    import torch
    info = fk_table_info(ctx, table)
    R = grad_out.shape[1]
    if tuple(grad_out.shape) != (info["ndata"], R):
        raise ValueError(f"grad_out must be [{info['ndata']}][R]")
    if grad_pdf is None:
        grad_pdf = torch.empty((info["nflav"], info["nx"], R), dtype=torch.float32,
                               device=grad_out.device)
    if tuple(grad_pdf.shape) != (info["nflav"], info["nx"], R):
        raise ValueError("grad_pdf has the wrong shape")
    pp = None
    if pdf is not None:
        if tuple(pdf.shape) != (info["nflav"], info["nx"], R):
            raise ValueError("pdf has the wrong shape")
        pp = _dptr(pdf, "f32", "pdf")
    _check(ctx, lib().fk_conv_backward(ctx, table, pp, _dptr(grad_out, "f32", "grad_out"), R,
                                       _dptr(grad_pdf, "f32", "grad_pdf"), 1 if accumulate else 0,
                                       _stream(stream)))
    return grad_pdf


# ---------------------------------------------------------------------------
# flattened form of Table 3
# ---------------------------------------------------------------------------

def fk_luminosity(ctx, mask, pdf, lum=None, stream=None):
    """L[(c, alpha, beta)][r] = f[a_c][alpha][r] f[b_c][beta][r] over the
    active pairs of ``mask`` (host [nflav][nflav]); pdf [nflav][nx][R]."""
    import torch
    mk = np.ascontiguousarray(mask, dtype=np.uint8)
    F, X, R = pdf.shape
    if mk.shape != (F, F):
        raise ValueError(f"mask must be [{F}][{F}]")
    K = int(mk.astype(bool).sum()) * X * X
    if lum is None:
        lum = torch.empty((K, R), dtype=torch.float32, device=pdf.device)
    if tuple(lum.shape) != (K, R):
        raise ValueError(f"lum must be [{K}][{R}]")
    _check(ctx, lib().fk_luminosity(ctx, F, X, _hptr(mk), _dptr(pdf, "f32", "pdf"), R,
                                    _dptr(lum, "f32", "lum"), _stream(stream)))
    return lum


def fk_flat_conv_workspace(ctx, n: int, k: int, r: int) -> int:
    b = ctypes.c_uint64()
    _check(ctx, lib().fk_flat_conv_workspace(ctx, n, k, r, ctypes.byref(b)))
    return b.value


def fk_flat_conv(ctx, fk, lum, out=None, work=None, stream=None):
    """out[N][R] = fk[N][K] lum[K][R] (FP32); allocates the workspace when
    none is given."""
    import torch
    N, K = fk.shape
    K2, R = lum.shape
    if K2 != K:
        raise ValueError("fk and lum disagree on K")
    if out is None:
        out = torch.empty((N, R), dtype=torch.float32, device=fk.device)
    need = fk_flat_conv_workspace(ctx, N, K, R)
    if work is None and need:
        work = torch.empty(need // 4, dtype=torch.float32, device=fk.device)
    wp = _dptr(work, "f32", "work") if work is not None else None
    wb = work.numel() * 4 if work is not None else 0
    _check(ctx, lib().fk_flat_conv(ctx, N, K, R, _dptr(fk, "f32", "fk"), _dptr(lum, "f32", "lum"),
                                   _dptr(out, "f32", "out"), wp, wb, _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# network PDF and gradient descent
# ---------------------------------------------------------------------------

def fk_mlp_create(ctx, xgrid, h1: int, h2: int, pre_alpha, pre_beta):
    """(handle, nparams) of a network PDF on ``xgrid``; nflav = len(pre_alpha)."""
    xg = np.ascontiguousarray(xgrid, dtype=np.float64)
    pa = np.ascontiguousarray(pre_alpha, dtype=np.float64)
    pb = np.ascontiguousarray(pre_beta, dtype=np.float64)
    if pa.shape != pb.shape or pa.ndim != 1:
        raise ValueError("pre_alpha and pre_beta must be [nflav]")
    h, n = ctypes.c_int64(), ctypes.c_int32()
    _check(ctx, lib().fk_mlp_create(ctx, len(pa), len(xg), _hptr(xg), h1, h2, _hptr(pa), _hptr(pb),
                                    ctypes.byref(h), ctypes.byref(n)))
    return h.value, n.value


def fk_mlp_destroy(ctx, mlp: int):
    _check(ctx, lib().fk_mlp_destroy(ctx, mlp))


def fk_mlp_forward(ctx, mlp: int, params, nflav: int, nx: int, pdf=None, stream=None):
    import torch
    R = params.shape[0]
    if pdf is None:
        pdf = torch.empty((nflav, nx, R), dtype=torch.float32, device=params.device)
    _check(ctx, lib().fk_mlp_forward(ctx, mlp, _dptr(params, "f32", "params"), R,
                                     _dptr(pdf, "f32", "pdf"), _stream(stream)))
    return pdf


def fk_mlp_backward(ctx, mlp: int, params, grad_pdf, grad_params=None, stream=None):
    import torch
    R = params.shape[0]
    if grad_pdf.shape[2] != R:
        raise ValueError("grad_pdf must be [nflav][nx][R] with the params' R")
    if grad_params is None:
        grad_params = torch.empty_like(params)
    _check(ctx, lib().fk_mlp_backward(ctx, mlp, _dptr(params, "f32", "params"),
                                      _dptr(grad_pdf, "f32", "grad_pdf"), R,
                                      _dptr(grad_params, "f32", "grad_params"), _stream(stream)))
    return grad_params


def fk_sgd_update(ctx, params, grad, lr: float, stream=None):
    if params.shape != grad.shape:
        raise ValueError("params and grad differ in shape")
    _check(ctx, lib().fk_sgd_update(ctx, _dptr(params, "f32", "params"), _dptr(grad, "f32", "grad"),
                                    params.numel(), lr, _stream(stream)))


# ---------------------------------------------------------------------------
# chi2
# ---------------------------------------------------------------------------

def fk_load_covariance(ctx, blocks: Sequence[np.ndarray]) -> int:
    n = np.asarray([b.shape[0] for b in blocks], dtype=np.int32)
    flat = np.ascontiguousarray(np.concatenate([np.ascontiguousarray(b, dtype=np.float64).ravel()
                                                for b in blocks]))
    h = ctypes.c_int64()
    _check(ctx, lib().fk_load_covariance(ctx, len(n), _hptr(n), _hptr(flat), ctypes.byref(h)))
    return h.value


def fk_unload_covariance(ctx, cov: int):
    _check(ctx, lib().fk_unload_covariance(ctx, cov))


def fk_chi2(ctx, cov: int, sigma, data, chi2=None, dchi2_dsigma=None, want_grad=True,
            stream=None):
    import torch
    R = sigma.shape[1]
    if chi2 is None:
        chi2 = torch.empty(R, dtype=torch.float64, device=sigma.device)
    if want_grad and dchi2_dsigma is None:
        dchi2_dsigma = torch.empty_like(sigma)
    _check(ctx, lib().fk_chi2(ctx, cov, _dptr(sigma, "f32", "sigma"), _dptr(data, "f64", "data"), R,
                              _dptr(chi2, "f64", "chi2"),
                              _dptr(dchi2_dsigma, "f32", "dchi2_dsigma") if want_grad else None,
                              _stream(stream)))
    return chi2, (dchi2_dsigma if want_grad else None)


# ---------------------------------------------------------------------------
# kernel timing
# ---------------------------------------------------------------------------
KERNEL_KINDS = ["stage", "had_fwd", "dis_fwd", "fwd_reduce", "had_adj", "dis_adj",
                "adj_reduce", "chi2", "had_stream", "dis_stream", "had_adj_stream"]


def fk_timing_enable(ctx, enable: bool = True):
    _check(ctx, lib().fk_timing_enable(ctx, 1 if enable else 0))


def fk_timing_read(ctx) -> dict:
    """{kind: (total_ms, launches)} since the previous read."""
    ms = np.zeros(len(KERNEL_KINDS), dtype=np.float64)
    n = np.zeros(len(KERNEL_KINDS), dtype=np.int64)
    _check(ctx, lib().fk_timing_read(ctx, _hptr(ms), _hptr(n)))
    return {k: (float(ms[i]), int(n[i])) for i, k in enumerate(KERNEL_KINDS)}


def fk_measure_mfma_peak(ctx, iters: int = 20000) -> float:
    """Dense BF16 TFLOP/s of a register-only MFMA loop on this device."""
    v = ctypes.c_double()
    _check(ctx, lib().fk_measure_mfma_peak(ctx, iters, ctypes.byref(v)))
    return v.value


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------

def fk_serve_start(ctx, nslots: int = 64, nstreams: int = 4, request_budget_bytes: int = 256 << 20):
    _check(ctx, lib().fk_serve_start(ctx, nslots, nstreams, request_budget_bytes))


def fk_serve_stop(ctx):
    _check(ctx, lib().fk_serve_stop(ctx))
    for k in [k for k in _ready_events if k[0] == ctx.value]:
        del _ready_events[k]


def fk_table_set_fallback(ctx, table: int, fallback: int):
    _check(ctx, lib().fk_table_set_fallback(ctx, table, fallback))


def fk_table_probe(ctx, table: int, pdf, tol: float = 5e-3, stream=None) -> float:
    """Error of ``table`` against its linked FP32 fallback on ``pdf``; served
    requests for the table's own format go to the fallback when it exceeds
    ``tol``."""
    err = ctypes.c_double()
    _check(ctx, lib().fk_table_probe(ctx, table, _dptr(pdf, "f32", "pdf"), pdf.shape[2], tol,
                                     ctypes.byref(err), _stream(stream)))
    return err.value


# events of submitted requests, kept alive until their ticket is finished
_ready_events = {}


def fk_submit(ctx, table: int, pdf, out, precision: int = FK_BF16, tag: int = 0,
              stream=None) -> int:
    """Queue a request.  An event recorded on ``stream`` (default: the current
    torch stream) orders the pass after the work that produced ``pdf``."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    ev = torch.cuda.Event()
    ev.record(s)
    req = fk_request(table=table, nrep=pdf.shape[2], precision=precision,
                     pdf=_dptr(pdf, "f32", "pdf").value, out=_dptr(out, "f32", "out").value,
                     tag=tag, ready=ctypes.c_void_p(ev.cuda_event))
    t = ctypes.c_int64()
    _check(ctx, lib().fk_submit(ctx, ctypes.byref(req), ctypes.byref(t)))
    _ready_events[(ctx.value, t.value)] = ev
    return t.value


def fk_poll(ctx, ticket: int) -> int:
    s = ctypes.c_int32()
    _check(ctx, lib().fk_poll(ctx, ticket, ctypes.byref(s)))
    if s.value in (FK_DONE, FK_FAILED):
        _ready_events.pop((ctx.value, ticket), None)
    return s.value


def fk_ticket_times(ctx, ticket: int):
    a, b, c = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
    _check(ctx, lib().fk_ticket_times(ctx, ticket, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return a.value, b.value, c.value


# ---------------------------------------------------------------------------
# convenience wrapper
# ---------------------------------------------------------------------------

class Context:
    """Owns an fk_ctx; ``with Context() as c: ...`` destroys it on exit."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 0):
        self.ctx = fk_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx is not None:
            fk_destroy(self.ctx)
            self.ctx = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def load(self, table, store_dtype="bf16") -> int:
        """Load a synth.DisTable / synth.HadTable."""
        kind = FK_HAD if table.mask.ndim == 2 else FK_DIS
        return fk_load_table(self.ctx, kind, table.xgrid, table.mask, table.fk, store_dtype)
