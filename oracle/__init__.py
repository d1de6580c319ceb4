"""FP64 CPU oracle for the FK-table convolution -- TEST INFRASTRUCTURE ONLY.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The library product never calls it and
shares no code with it: the loops live in ``fkoracle.c`` (plain C, gcc,
optional OpenMP over output elements), the quantisers below are numpy.

What each function follows:

* ``dis``            DIS observable, the linear one-PDF convolution of
                     Section 3 (Table 1, "DIS" rows).
* ``had``            hadronic observable, Eq. (1) of Section 3.
* ``had_bilinear``   Eq. (1) with separate left and right PDFs (used by the
                     stored-operand mode below).
* ``dis_grad``, ``had_grad``  gradient of sum_{i,r} gbar[i,r] obs[i,r] with
                     respect to the PDF (Table 1, "Gradient" rows).
* ``cholesky``, ``chi2``  FP64 chi2 = (sigma - D)^T C^{-1} (sigma - D) with a
                     block-diagonal covariance and its gradient 2 C^{-1} e.
                     The paper never writes its loss; this is the standard
                     correlated chi2 the fit minimises.
* ``quantize``       round-to-nearest-even to bfloat16 or OCP e4m3fn
                     (saturating at +-448), emulated in FP64 from the format
                     definitions.
* ``dis_stored``, ``had_stored``, ``*_quantized``  the "quantized-input
                     mode": the definitions above evaluated in FP64 on
                     operands rounded to a storage format.  It separates
                     kernel arithmetic errors from input-rounding errors.
                     The hadronic variant stores the symmetric part
                     S = FK + FK^T (sigma = 1/2 f^T S f), rounds the right
                     PDF factor to the storage format and keeps the left one
                     in FP32, which is the operand set a half-precision
                     kernel of the bilinear form consumes.
* ``luminosity``, ``flat_conv``  the flattened form Table 3 times: the
                     luminosity L[(a,b,alpha,beta), r] = f_a(x_alpha) f_b(x_beta)
                     over the active pairs, and the plain product FK[N][K] L[K][R]
                     (a library matmul in FP64).
* ``mlp_pdf``, ``mlp_pdf_grad``  the PDF as the output of a neural network
                     sampled on the x-grid (Section 2: the fit parametrises
                     the PDF with a network trained by gradient descent;
                     Section 3: the network generates the PDF on the grid
                     that the convolution consumes), and the gradient of a
                     linear functional of that PDF with respect to the
                     network parameters (reverse-mode chain rule, layer by
                     layer).  The paper gives no architecture; the one here
                     (inputs x and ln x, two tanh layers, a linear output per
                     flavour times x^alpha (1-x)^beta) is a reading.
* ``normwise_rel``, ``error_report``  the error measures every parity test
                     gates on or reports.

Pins (``tests/test_oracle_*.py``): invariants, closed forms, exact integer
brute force, library routines for special cases and finite differences for
the convolutions, gradients and chi2; hand-computed values for the error
measures; torch's own casts for the quantisers; FP64-mode identities and
exact integer cases for the stored-operand functions.  Planted slips in the
C loops and in this file must each fail one of them
(``tests/test_oracle_mutants.py``).  One modelling choice is not pinned by
the mathematics: which factor of the bilinear form the stored-operand mode
rounds (the right one, as the kernels do); the pins only fix that the mode
reduces to the definition when rounding is exact.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fkoracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the mutation tests point this at a deliberately broken build of fkoracle.c
_LIB_OVERRIDE = os.environ.get("FK_ORACLE_LIB")
_lib = None


def build(force: bool = True) -> str:
    """Compile fkoracle.c with gcc (OpenMP) into liboracle.so."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            lib = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        lib.oracle_dis.argtypes = [I, I, I, P, P, I, P, P]
        lib.oracle_had.argtypes = [I, I, I, P, P, I, P, P]
        lib.oracle_had_bilinear.argtypes = [I, I, I, P, P, I, P, P, P]
        lib.oracle_dis_grad.argtypes = [I, I, I, P, P, I, P, P]
        lib.oracle_had_grad.argtypes = [I, I, I, P, P, I, P, P, P]
        lib.oracle_cholesky.argtypes = [I, P, P]
        lib.oracle_cholesky.restype = I
        lib.oracle_chi2.argtypes = [I, P, P, I, P, P, P, P]
        lib.oracle_num_threads.restype = I
        lib.oracle_set_num_threads.argtypes = [I]
        lib.oracle_set_num_threads.restype = None
        _lib = lib
    return _lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _u8(a):
    return np.ascontiguousarray(a, dtype=np.uint8)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads of the oracle's parallel loops (one thread per output, so the
    results do not depend on it)."""
    _load().oracle_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# convolutions
# ---------------------------------------------------------------------------

def dis(mask, fk, pdf) -> np.ndarray:
    """T[i,r] = sum_{a active, alpha} FK[i,a,alpha] f[a,alpha,r]."""
    mask, fk, pdf = _u8(mask), _f64(fk), _f64(pdf)
    F, X, R = pdf.shape
    N = fk.shape[0]
    assert mask.shape == (F,) and fk.shape == (N, int(mask.sum()), X)
    out = np.empty((N, R))
    _load().oracle_dis(N, F, X, _p(mask), _p(fk), R, _p(pdf), _p(out))
    return out


def had_bilinear(mask, fk, pdf_left, pdf_right) -> np.ndarray:
    """s[i,r] = sum_{(a,b) active} sum FK[i,ab,alpha,beta] fl[a,alpha,r] fr[b,beta,r]."""
    mask, fk = _u8(mask), _f64(fk)
    pl, pr = _f64(pdf_left), _f64(pdf_right)
    F, X, R = pl.shape
    N = fk.shape[0]
    assert pr.shape == pl.shape and mask.shape == (F, F)
    assert fk.shape == (N, int(mask.sum()), X, X)
    out = np.empty((N, R))
    _load().oracle_had_bilinear(N, F, X, _p(mask), _p(fk), R, _p(pl), _p(pr), _p(out))
    return out


def had(mask, fk, pdf) -> np.ndarray:
    """Eq. (1): sigma[i,r] = sum FK[i,a,b,alpha,beta] f[a,alpha,r] f[b,beta,r]."""
    mask, fk, pdf = _u8(mask), _f64(fk), _f64(pdf)
    F, X, R = pdf.shape
    N = fk.shape[0]
    assert mask.shape == (F, F) and fk.shape == (N, int(mask.sum()), X, X)
    out = np.empty((N, R))
    _load().oracle_had(N, F, X, _p(mask), _p(fk), R, _p(pdf), _p(out))
    return out


def dis_grad(mask, fk, gbar, nflav=None, nx=None) -> np.ndarray:
    """g[a,alpha,r] = sum_i gbar[i,r] FK[i,a,alpha] (0 for inactive a)."""
    mask, fk, gbar = _u8(mask), _f64(fk), _f64(gbar)
    N, nact, X = fk.shape
    F = mask.shape[0]
    R = gbar.shape[1]
    g = np.empty((F, X, R))
    _load().oracle_dis_grad(N, F, X, _p(mask), _p(fk), R, _p(gbar), _p(g))
    return g


def had_grad(mask, fk, pdf, gbar) -> np.ndarray:
    """g[p,r] = sum_i gbar[i,r] (sum_q FK[i,p,q] f[q,r] + sum_q FK[i,q,p] f[q,r])."""
    mask, fk, pdf, gbar = _u8(mask), _f64(fk), _f64(pdf), _f64(gbar)
    F, X, R = pdf.shape
    N = fk.shape[0]
    g = np.empty((F, X, R))
    _load().oracle_had_grad(N, F, X, _p(mask), _p(fk), R, _p(pdf), _p(gbar), _p(g))
    return g


# ---------------------------------------------------------------------------
# flattened form (Table 3: FK table N x K against a "PDF" K x R)
# ---------------------------------------------------------------------------

def luminosity(mask, pdf) -> np.ndarray:
    """L[(c, alpha, beta), r] = f[a_c, alpha, r] f[b_c, beta, r] for the
    active pairs c = (a_c, b_c) in row-major (a, b) order: [np*X*X][R]."""
    mask, pdf = _u8(mask), _f64(pdf)
    F, X, R = pdf.shape
    a, b = np.nonzero(mask)
    L = np.empty((len(a), X, X, R))
    for c in range(len(a)):
        L[c] = pdf[a[c]][:, None, :] * pdf[b[c]][None, :, :]
    return L.reshape(len(a) * X * X, R)


def flat_conv(fk_flat, lum) -> np.ndarray:
    """out[N][R] = FK[N][K] L[K][R] in FP64."""
    return np.matmul(_f64(fk_flat), _f64(lum))


# ---------------------------------------------------------------------------
# chi2
# ---------------------------------------------------------------------------

def cholesky(C) -> np.ndarray:
    C = _f64(C)
    n = C.shape[0]
    L = np.empty_like(C)
    rc = _load().oracle_cholesky(n, _p(C), _p(L))
    if rc != 0:
        raise np.linalg.LinAlgError(f"not positive definite at row {-rc - 1}")
    return L


def chi2(Ls: Sequence[np.ndarray], sigma, data, want_grad=True):
    """chi2_r over block-diagonal covariance given the Cholesky factors of
    the blocks (in order).  Returns (chi2 [R], dchi2/dsigma [Ntot][R] or None)."""
    sigma, data = _f64(sigma), _f64(data)
    Ntot, R = sigma.shape
    bn = np.asarray([L.shape[0] for L in Ls], dtype=np.int32)
    assert int(bn.sum()) == Ntot and data.shape == (Ntot,)
    Lp = _f64(np.concatenate([_f64(L).ravel() for L in Ls])) if len(Ls) else np.zeros(1)
    out = np.empty(R)
    d = np.empty((Ntot, R)) if want_grad else None
    _load().oracle_chi2(len(Ls), _p(bn), _p(Lp), R, _p(sigma), _p(data), _p(out),
                        _p(d) if d is not None else None)
    return out, d


# ---------------------------------------------------------------------------
# rounding to storage formats (round to nearest, ties to even)
# ---------------------------------------------------------------------------

_FMT = {
    # name: (mantissa bits kept, min exponent of a normal, max finite, saturate)
    "bf16": (7, -126, float(np.ldexp(255.0, 120)), False),   # (2-2^-7)*2^127
    "e4m3": (3, -6, 448.0, True),
}


def quantize(x, fmt: str) -> np.ndarray:
    """Round float64 values to ``fmt`` ("f32", "bf16", "e4m3"), returned as
    float64.  bf16: 8 significant bits, exponent range of binary32, overflow
    to inf.  e4m3 (OCP e4m3fn): 4 significant bits, min normal 2^-6,
    subnormal quantum 2^-9, saturating to +-448."""
    x = np.asarray(x, dtype=np.float64)
    if fmt == "f32":
        return x.astype(np.float32).astype(np.float64)
    if fmt == "f64":
        return x.copy()
    mbits, emin, maxf, sat = _FMT[fmt]
    _, E = np.frexp(x)                      # |x| in [2^(E-1), 2^E)
    qe = np.maximum(E - 1 - mbits, emin - mbits)
    y = np.ldexp(np.rint(np.ldexp(x, -qe)), qe)
    y = np.where(x == 0, x, y)
    big = np.abs(y) > maxf
    if sat:
        y = np.where(big, np.copysign(maxf, x), y)
    else:
        y = np.where(big, np.copysign(np.inf, x), y)
    return y


_QMAX = {"f64": 1.0, "f32": 1.0, "bf16": 1.0, "e4m3": 448.0}


def datapoint_scale(absmax, fmt: str) -> np.ndarray:
    """s_i = 2^e_i with e_i the smallest integer such that
    max|row_i| / 2^e_i <= qmax (qmax = 1, or 448 for e4m3); 1 for a zero row."""
    absmax = np.asarray(absmax, dtype=np.float64)
    qmax = _QMAX[fmt]
    pos = absmax > 0
    with np.errstate(divide="ignore"):
        e = np.where(pos, np.ceil(np.log2(np.where(pos, absmax, 1.0) / qmax)), 0.0)
    e = e.astype(np.int64)
    # log2 in floating point may be one off near powers of two: fix exactly
    e = np.where(pos & (absmax > qmax * np.ldexp(1.0, e)), e + 1, e)
    e = np.where(pos & (absmax <= qmax * np.ldexp(1.0, e - 1)), e - 1, e)
    return np.ldexp(1.0, e)


def dis_stored(fk, fmt: str):
    """(s [N], FKhat [N][nact][X]) with FKhat = Q(FK_i / s_i)."""
    fk = _f64(fk)
    s = datapoint_scale(np.abs(fk).reshape(fk.shape[0], -1).max(axis=1, initial=0.0), fmt)
    return s, quantize(fk / s[:, None, None], fmt)


def symmetric_part(mask, fk) -> Tuple[np.ndarray, np.ndarray]:
    """Pattern Ps = P | P^T and S[i,(a,b)] = FK[i,(a,b)] + FK[i,(b,a)]^T over
    it (a missing block counts as zero)."""
    mask, fk = _u8(mask), _f64(fk)
    F = mask.shape[0]
    N, npairs, X, _ = fk.shape
    idx = -np.ones((F, F), dtype=np.int64)
    a, b = np.nonzero(mask)
    idx[a, b] = np.arange(len(a))
    ms = (mask | mask.T).astype(np.uint8)
    sa, sb = np.nonzero(ms)
    S = np.zeros((N, len(sa), X, X))
    for c, (pa, pb) in enumerate(zip(sa, sb)):
        if idx[pa, pb] >= 0:
            S[:, c] += fk[:, idx[pa, pb]]
        if idx[pb, pa] >= 0:
            S[:, c] += np.transpose(fk[:, idx[pb, pa]], (0, 2, 1))
    return ms, S


def had_stored(mask, fk, fmt: str):
    """(Ps, s [N], Shat) with Shat = Q(S_i / s_i), S the symmetric part."""
    ms, S = symmetric_part(mask, fk)
    s = datapoint_scale(np.abs(S).reshape(S.shape[0], -1).max(axis=1, initial=0.0), fmt)
    return ms, s, quantize(S / s[:, None, None, None], fmt)


def dis_quantized(mask, fk, pdf, fmt: str) -> np.ndarray:
    """T computed in FP64 from Q(FK/s) and Q(f), rescaled by s."""
    s, fq = dis_stored(fk, fmt)
    return s[:, None] * dis(mask, fq, quantize(pdf, fmt))


def had_stored_upper(mask, fk, fmt: str):
    """The symmetric part over unordered flavour pairs: (U, s [N], Uhat) with
    U the blocks (a, b) of Ps with a <= b, Uhat = Q(S'_i / s_i), S'_ab = S_ab
    for a < b and S'_aa = S_aa / 2, and s_i the scale of the full S_i.
    Eq. (1) equals sum over a <= b of f_a S'_ab f_b."""
    ms, S = symmetric_part(mask, fk)
    s = datapoint_scale(np.abs(S).reshape(S.shape[0], -1).max(axis=1, initial=0.0), fmt)
    sa, sb = np.nonzero(ms)
    keep = sa <= sb
    U = S[:, keep] / s[:, None, None, None]
    U[:, (sa == sb)[keep]] *= 0.5
    mu = np.zeros_like(ms)
    mu[sa[keep], sb[keep]] = 1
    return mu, s, quantize(U, fmt)


def had_quantized(mask, fk, pdf, fmt: str) -> np.ndarray:
    """sigma = s sum_{a<=b} f_a Uhat[a,b] Q(f_b) in FP64, f_a in FP32 (the
    forward's stored form, had_stored_upper)."""
    mu, s, Uq = had_stored_upper(mask, fk, fmt)
    return s[:, None] * had_bilinear(mu, Uq, quantize(pdf, "f32"), quantize(pdf, fmt))


def dis_grad_quantized(mask, fk, gbar, fmt: str) -> np.ndarray:
    """g = sum_i Q(FK_i/s_i) Q(gbar_i s_i)."""
    s, fq = dis_stored(fk, fmt)
    return dis_grad(mask, fq, quantize(_f64(gbar) * s[:, None], fmt))


def had_grad_quantized(mask, fk, pdf, gbar, fmt: str) -> np.ndarray:
    """g[p,r] = sum_i gbar[i,r] s_i sum_q Shat_i[p,q] Q(f)[q,r]."""
    ms, s, Sq = had_stored(mask, fk, fmt)
    w = quantize(_f64(gbar) * s[:, None], "f32")
    return 0.5 * had_grad(ms, Sq, quantize(pdf, fmt), w)


# ---------------------------------------------------------------------------
# error measures
# ---------------------------------------------------------------------------

# ---------------------------------------------------------------------------
# PDF from a neural network on the x-grid (Sections 2 and 3)
# ---------------------------------------------------------------------------

def mlp_nparams(nflav: int, h1: int, h2: int) -> int:
    """Parameters of one replica's network, in the order W1 [h1][2], b1 [h1],
    W2 [h2][h1], b2 [h2], W3 [nflav][h2], b3 [nflav]."""
    return h1 * 2 + h1 + h2 * h1 + h2 + nflav * h2 + nflav


def mlp_unpack(p, nflav: int, h1: int, h2: int):
    p = _f64(p)
    o = 0
    out = []
    for shape in ((h1, 2), (h1,), (h2, h1), (h2,), (nflav, h2), (nflav,)):
        n = int(np.prod(shape))
        out.append(p[o:o + n].reshape(shape))
        o += n
    return out


def mlp_preprocessing(xgrid, pre_alpha, pre_beta) -> np.ndarray:
    """x^alpha_a (1 - x)^beta_a on the grid, [nflav][X]."""
    x = _f64(xgrid)
    return x[None, :] ** _f64(pre_alpha)[:, None] * (1.0 - x[None, :]) ** _f64(pre_beta)[:, None]


def mlp_pdf(params, xgrid, pre_alpha, pre_beta, h1: int, h2: int) -> np.ndarray:
    """f[a, alpha, r] = x_alpha^alpha_a (1 - x_alpha)^beta_a NN_r(x_alpha)_a
    for the network of replica r (params [R][P]): inputs (x, ln x), a tanh
    layer of h1 units, a tanh layer of h2 units, a linear output per flavour.
    Returns [nflav][X][R]."""
    params, x = _f64(params), _f64(xgrid)
    F = len(pre_alpha)
    R, X = params.shape[0], len(x)
    inp = np.stack([x, np.log(x)], axis=1)  # [X][2]
    pre = mlp_preprocessing(x, pre_alpha, pre_beta)
    f = np.empty((F, X, R))
    for r in range(R):
        W1, b1, W2, b2, W3, b3 = mlp_unpack(params[r], F, h1, h2)
        a1 = np.tanh(inp @ W1.T + b1)  # [X][h1]
        a2 = np.tanh(a1 @ W2.T + b2)   # [X][h2]
        out = a2 @ W3.T + b3           # [X][F]
        f[:, :, r] = pre * out.T
    return f


def mlp_pdf_grad(params, xgrid, pre_alpha, pre_beta, h1: int, h2: int, gpdf) -> np.ndarray:
    """Gradient with respect to params [R][P] of sum_{a,alpha,r} gpdf[a,alpha,r]
    f[a,alpha,r] (gpdf: [nflav][X][R], e.g. d chi2 / d f from the adjoint of
    the convolution).  Reverse mode: output layer, then each tanh layer with
    the factor 1 - tanh^2."""
    params, x, gpdf = _f64(params), _f64(xgrid), _f64(gpdf)
    F = len(pre_alpha)
    R = params.shape[0]
    inp = np.stack([x, np.log(x)], axis=1)
    pre = mlp_preprocessing(x, pre_alpha, pre_beta)
    g = np.empty_like(params)
    for r in range(R):
        W1, b1, W2, b2, W3, b3 = mlp_unpack(params[r], F, h1, h2)
        a1 = np.tanh(inp @ W1.T + b1)
        a2 = np.tanh(a1 @ W2.T + b2)
        dout = (gpdf[:, :, r] * pre).T        # d/d out, [X][F]
        d2 = (dout @ W3) * (1.0 - a2 ** 2)    # d/d (W2 a1 + b2), [X][h2]
        d1 = (d2 @ W2) * (1.0 - a1 ** 2)      # d/d (W1 inp + b1), [X][h1]
        g[r] = np.concatenate([(d1.T @ inp).ravel(), d1.sum(axis=0), (d2.T @ a1).ravel(),
                               d2.sum(axis=0), (dout.T @ a2).ravel(), dout.sum(axis=0)])
    return g


def normwise_rel(y, yref) -> float:
    """max over replica columns (the last axis) of ||y - y*||_2 / ||y*||_2;
    a zero reference column counts as 0 if y matches it exactly, else inf."""
    y = np.asarray(y, dtype=np.float64)
    yref = np.asarray(yref, dtype=np.float64)
    if y.size == 0:
        return 0.0
    y2 = y.reshape(-1, y.shape[-1]) if y.ndim >= 2 else y[:, None]
    r2 = yref.reshape(-1, yref.shape[-1]) if yref.ndim >= 2 else yref[:, None]
    num = np.sqrt(np.sum((y2 - r2) ** 2, axis=0))
    den = np.sqrt(np.sum(r2 ** 2, axis=0))
    rel = np.where(den > 0, num / np.where(den > 0, den, 1.0),
                   np.where(num > 0, np.inf, 0.0))
    return float(np.max(rel))


def error_report(y, yref) -> dict:
    """Normwise (gate) plus elementwise statistics over |y*| >= 1e-3 ||y*||_inf."""
    y = np.asarray(y, dtype=np.float64)
    yref = np.asarray(yref, dtype=np.float64)
    out = {"normwise": normwise_rel(y, yref)}
    if yref.size:
        thr = 1e-3 * float(np.max(np.abs(yref)))
        sel = np.abs(yref) >= thr
        if np.any(sel):
            e = np.abs(y[sel] - yref[sel]) / np.abs(yref[sel])
            out.update(elem_p50=float(np.percentile(e, 50)),
                       elem_p99=float(np.percentile(e, 99)),
                       elem_max=float(np.max(e)))
    return out
