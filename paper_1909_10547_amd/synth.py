"""Seeded synthetic inputs shaped like the FK-table workloads of the paper.

This module draws inputs only: x-grids, PDF replicas sampled on the grid,
flavour masks, FK tables and experimental covariances.  It contains none of
the convolution arithmetic (no contraction, no quantisation, no solve), so
both the CPU oracle and the HIP path can consume what it produces.

Conventions (shared by every consumer):

* ``xgrid``          float64 [X], increasing.
* PDF                float64 [F][X][R]  (R, the replica index, fastest).
* DIS table          ``mask`` uint8 [F]; ``fk`` float64 [N][nact][X] with
                     the active flavours in increasing flavour order.
* hadronic table     ``mask`` uint8 [F][F]; ``fk`` float64
                     [N][npairs][X][X] with the active (a, b) pairs in
                     row-major (a, b) order; element [i, c, alpha, beta]
                     multiplies f_a(x_alpha) f_b(x_beta).

Only the active flavour (pair) blocks are stored, as in the paper's base FK
table, which holds 49 flavour combinations on a 27-point grid (Section 3,
Table 3 caption).  Index names follow the convolution of Section 3, Eq. (1),
with datapoint i, flavours a, b and grid points alpha, beta.

Seeds: every draw uses ``numpy.random.default_rng([cfg_seed, stream])`` with a
fixed stream number per purpose, so a dataset can be regenerated on its own.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Iterator, List, Optional, Sequence

import numpy as np

NFLAV = 14

# stream numbers for default_rng([seed, stream])
_S_SIZES = 0
_S_PDF = 1
_S_COV = 2
_S_DATASET0 = 100


def rng_for(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


# ---------------------------------------------------------------------------
# grids and PDFs
# ---------------------------------------------------------------------------

def xgrid_geom(xmin: float, xmax: float, nx: int) -> np.ndarray:
    """Log-spaced grid including both endpoints."""
    return np.geomspace(xmin, xmax, nx)


@dataclass
class PdfParams:
    A: np.ndarray  # [F]
    p: np.ndarray  # [F]   small-x exponent
    q: np.ndarray  # [F]   large-x exponent


def draw_pdf_params(rng: np.random.Generator, nflav: int = NFLAV) -> PdfParams:
    """f_a(x) = A_a x^p_a (1-x)^q_a with p~U(-0.3,0.8), q~U(1,5), A~U(0.5,2)."""
    p = rng.uniform(-0.3, 0.8, size=nflav)
    q = rng.uniform(1.0, 5.0, size=nflav)
    A = rng.uniform(0.5, 2.0, size=nflav)
    return PdfParams(A=A, p=p, q=q)


def sample_pdf(params: PdfParams, xgrid: np.ndarray, nrep: int,
               jitter: float = 0.0,
               rng: Optional[np.random.Generator] = None) -> np.ndarray:
    """PDF replicas on the grid, float64 [F][X][R].

    Replica r uses exponents p_a + dp_{r,a}, q_a + dq_{r,a} with
    dp, dq ~ N(0, jitter) drawn independently (A_a is not jittered).
    With jitter == 0 every replica equals the central PDF.
    """
    F = params.A.shape[0]
    if jitter > 0.0:
        assert rng is not None
        dp = rng.normal(0.0, jitter, size=(nrep, F))
        dq = rng.normal(0.0, jitter, size=(nrep, F))
    else:
        dp = np.zeros((nrep, F))
        dq = np.zeros((nrep, F))
    p = params.p[None, :] + dp          # [R][F]
    q = params.q[None, :] + dq
    x = xgrid[None, None, :]            # [1][1][X]
    with np.errstate(divide="ignore", invalid="ignore"):
        val = (params.A[None, :, None] * x ** p[:, :, None]
               * (1.0 - x) ** q[:, :, None])          # [R][F][X]
    val = np.where(np.isfinite(val), val, 0.0)
    return np.ascontiguousarray(np.transpose(val, (1, 2, 0)))


# ---------------------------------------------------------------------------
# FK tables
# ---------------------------------------------------------------------------

@dataclass
class DisTable:
    mask: np.ndarray     # uint8 [F]
    fk: np.ndarray       # float64 [N][nact][X]
    xgrid: np.ndarray

    @property
    def ndata(self) -> int:
        return self.fk.shape[0]


@dataclass
class HadTable:
    mask: np.ndarray     # uint8 [F][F]
    fk: np.ndarray       # float64 [N][npairs][X][X]
    xgrid: np.ndarray

    @property
    def ndata(self) -> int:
        return self.fk.shape[0]


def _log_uniform_points(rng, xgrid, n):
    lo, hi = np.log(xgrid[0]), np.log(xgrid[-1])
    return rng.uniform(lo, hi, size=n)   # ln x_i


def draw_dis_table(rng: np.random.Generator, xgrid: np.ndarray, ndata: int,
                   nactive: int = 9, nflav: int = NFLAV) -> DisTable:
    """FK[i,a,alpha] = N(0,1) * exp(-|ln x_alpha - ln x_i|) on ``nactive``
    flavours chosen without replacement; ln x_i uniform over the grid range.

    Draw order: active flavours, ln x_i, the normal deviates [N][nact][X].
    """
    act = np.sort(rng.choice(nflav, size=nactive, replace=False))
    mask = np.zeros(nflav, dtype=np.uint8)
    mask[act] = 1
    lnxi = _log_uniform_points(rng, xgrid, ndata)
    z = rng.standard_normal(size=(ndata, nactive, xgrid.shape[0]))
    w = np.exp(-np.abs(np.log(xgrid)[None, :] - lnxi[:, None]))   # [N][X]
    fk = z * w[:, None, :]
    return DisTable(mask=mask, fk=np.ascontiguousarray(fk), xgrid=xgrid)


def pair_list(mask: np.ndarray) -> np.ndarray:
    """Active (a, b) pairs of a [F][F] mask in row-major order, int [np][2]."""
    a, b = np.nonzero(mask)
    return np.stack([a, b], axis=1)


def draw_symmetric_mask(rng: np.random.Generator, ndiag: int, noff: int,
                        nflav: int = NFLAV) -> np.ndarray:
    """Symmetric [F][F] mask with ``ndiag`` diagonal pairs and ``noff``
    unordered off-diagonal pairs (each stored in both orders), so
    ndiag + 2*noff ordered pairs are active."""
    mask = np.zeros((nflav, nflav), dtype=np.uint8)
    diag = rng.choice(nflav, size=ndiag, replace=False)
    mask[diag, diag] = 1
    iu = np.array([(a, b) for a in range(nflav) for b in range(a + 1, nflav)])
    sel = iu[rng.choice(len(iu), size=noff, replace=False)]
    mask[sel[:, 0], sel[:, 1]] = 1
    mask[sel[:, 1], sel[:, 0]] = 1
    return mask


def draw_had_table(rng: np.random.Generator, xgrid: np.ndarray, ndata: int,
                   ndiag: int = 4, noff: int = 28,
                   nflav: int = NFLAV) -> HadTable:
    """Symmetric hadronic FK: FK[i,a,b,alpha,beta] = FK[i,b,a,beta,alpha],
    values N(0,1) * exp(-d^2/2) with d = ln x_alpha + ln x_beta - 2 ln x_i.

    Draw order: mask (diagonal flavours, then off-diagonal pairs), ln x_i,
    then for each unordered active pair in row-major (a <= b) order the
    normal deviates [N][X][X]; for a == b only the upper triangle (including
    the diagonal) of each deviate matrix is used and mirrored.
    """
    X = xgrid.shape[0]
    mask = draw_symmetric_mask(rng, ndiag, noff, nflav)
    pairs = pair_list(mask)
    index = {(int(a), int(b)): c for c, (a, b) in enumerate(pairs)}
    lnxi = _log_uniform_points(rng, xgrid, ndata)
    lx = np.log(xgrid)
    d = lx[None, :, None] + lx[None, None, :] - 2.0 * lnxi[:, None, None]
    g = np.exp(-0.5 * d * d)                              # [N][X][X]
    fk = np.zeros((ndata, len(pairs), X, X))
    iu = np.triu_indices(X)
    for (a, b) in [(int(a), int(b)) for a, b in pairs if a <= b]:
        z = rng.standard_normal(size=(ndata, X, X))
        if a == b:
            s = np.zeros_like(z)
            s[:, iu[0], iu[1]] = z[:, iu[0], iu[1]]
            s = s + np.transpose(s, (0, 2, 1))
            s[:, np.arange(X), np.arange(X)] *= 0.5
            fk[:, index[(a, a)]] = s * g
        else:
            blk = z * g
            fk[:, index[(a, b)]] = blk
            fk[:, index[(b, a)]] = np.transpose(blk, (0, 2, 1))
    return HadTable(mask=mask, fk=fk, xgrid=xgrid)


def draw_general_had_table(rng: np.random.Generator, xgrid: np.ndarray,
                           ndata: int, npairs: int,
                           nflav: int = NFLAV) -> HadTable:
    """A non-symmetric hadronic table with a non-symmetric mask: ``npairs``
    ordered pairs chosen at random and N(0,1) entries.  Used to check that
    the path accepts general FK."""
    X = xgrid.shape[0]
    flat = np.sort(rng.choice(nflav * nflav, size=npairs, replace=False))
    mask = np.zeros(nflav * nflav, dtype=np.uint8)
    mask[flat] = 1
    mask = mask.reshape(nflav, nflav)
    fk = rng.standard_normal(size=(ndata, npairs, X, X))
    return HadTable(mask=mask, fk=fk, xgrid=xgrid)


# ---------------------------------------------------------------------------
# covariance (input generation only: C is built from its definition and the
# pseudo-data noise is drawn from the same factor structure, no factorisation)
# ---------------------------------------------------------------------------

def covariance_block(central: np.ndarray, rng: np.random.Generator,
                     unc: float = 0.05, sys: float = 0.03):
    """Covariance and pseudo-data for one dataset.

    m_i = max(|c_i|, 0.1 * rms(c)); uncorrelated sd unc*m_i; three
    systematics beta_k = sys*m_i*v_k with v_1 = 1, v_2 a linear ramp over
    [-1, 1], v_3 ~ N(0, 1).  C = diag((unc*m)^2) + sum_k beta_k beta_k^T.
    Pseudo-data D = c + unc*m*z0 + sum_k beta_k z_k, which has covariance C.
    Returns (C [n][n] float64, D [n] float64).
    """
    n = central.shape[0]
    rms = float(np.sqrt(np.mean(central ** 2))) if n else 0.0
    m = np.maximum(np.abs(central), 0.1 * rms)
    m = np.where(m > 0, m, 1.0)
    v1 = np.ones(n)
    v2 = np.linspace(-1.0, 1.0, n) if n > 1 else np.zeros(n)
    v3 = rng.standard_normal(n)
    B = sys * m[:, None] * np.stack([v1, v2, v3], axis=1)      # [n][3]
    sd = unc * m
    C = np.diag(sd * sd) + B @ B.T
    z0 = rng.standard_normal(n)
    zs = rng.standard_normal(3)
    D = central + sd * z0 + B @ zs
    return C, D


# ---------------------------------------------------------------------------
# the five workload configurations
# ---------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    seed: int
    xgrid: np.ndarray
    kind: str                       # "dis", "had" or "mixed"
    ndata: List[int]
    nrep: int
    nflav: int = NFLAV
    jitter: float = 0.05
    notes: str = ""
    kinds: List[str] = field(default_factory=list)   # per dataset

    def pdf(self, nrep: Optional[int] = None) -> np.ndarray:
        R = self.nrep if nrep is None else nrep
        prm = draw_pdf_params(rng_for(self.seed, _S_PDF), self.nflav)
        jit = self.jitter if R > 1 else 0.0
        return sample_pdf(prm, self.xgrid, R, jit, rng_for(self.seed, _S_PDF + 10))

    def central_pdf(self) -> np.ndarray:
        prm = draw_pdf_params(rng_for(self.seed, _S_PDF), self.nflav)
        return sample_pdf(prm, self.xgrid, 1, 0.0)

    def table(self, d: int):
        rng = rng_for(self.seed, _S_DATASET0 + d)
        kind = self.kinds[d]
        if kind == "dis":
            return draw_dis_table(rng, self.xgrid, self.ndata[d], 9, self.nflav)
        return draw_had_table(rng, self.xgrid, self.ndata[d], 4, 28, self.nflav)

    def tables(self) -> Iterator:
        for d in range(len(self.ndata)):
            yield self.table(d)


def dis_single_workload() -> Workload:
    """One DIS dataset, N=100, 14 flavours (9 active), 30 log-spaced points
    in [1e-5, 0.9], one replica, seed 0."""
    return Workload(name="dis_cpu_n100_x30_r1", seed=0,
                    xgrid=xgrid_geom(1e-5, 0.9, 30), kind="dis",
                    ndata=[100], nrep=1, jitter=0.0, kinds=["dis"])


def dis_fit_workload(scale: float = 1.0) -> Workload:
    """20 DIS datasets, N ~ U{50..600}, X=50 in [1e-7, 1], 9 active
    flavours each, R=100 jittered replicas, seed 1.  ``scale`` shrinks N
    for CPU-sized tests."""
    rng = rng_for(1, _S_SIZES)
    n = rng.integers(50, 601, size=20)
    n = [max(1, int(round(v * scale))) for v in n]
    return Workload(name="dis_global_20ds_x50_r100", seed=1,
                    xgrid=xgrid_geom(1e-7, 1.0, 50), kind="dis",
                    ndata=n, nrep=100, kinds=["dis"] * 20)


def had_fit_workload(scale: float = 1.0) -> Workload:
    """10 hadronic datasets, N ~ U{20..1000}, 60 active ordered flavour
    pairs from a random symmetric mask, X=50 in [1e-7, 1], symmetric FK,
    R=100 jittered replicas, seed 2."""
    rng = rng_for(2, _S_SIZES)
    n = rng.integers(20, 1001, size=10)
    n = [max(1, int(round(v * scale))) for v in n]
    return Workload(name="had_10ds_60pairs_x50_r100", seed=2,
                    xgrid=xgrid_geom(1e-7, 1.0, 50), kind="had",
                    ndata=n, nrep=100, kinds=["had"] * 10)


@dataclass
class FitWorkload:
    """Datasets of the DIS and hadronic fit workloads with a covariance per dataset (seed 3)."""
    dis: Workload
    had: Workload
    seed: int = 3
    nrep: int = 100

    def pdf(self) -> np.ndarray:
        prm = draw_pdf_params(rng_for(self.seed, _S_PDF))
        return sample_pdf(prm, self.dis.xgrid, self.nrep, 0.05,
                          rng_for(self.seed, _S_PDF + 10))

    def central_pdf(self) -> np.ndarray:
        prm = draw_pdf_params(rng_for(self.seed, _S_PDF))
        return sample_pdf(prm, self.dis.xgrid, 1, 0.0)

    def tables(self):
        yield from self.dis.tables()
        yield from self.had.tables()

    @property
    def ndata(self) -> List[int]:
        return list(self.dis.ndata) + list(self.had.ndata)

    def covariances(self, centrals: Sequence[np.ndarray]):
        """``centrals[d]`` is the central prediction of dataset d; returns
        lists of (C_d, D_d)."""
        rng = rng_for(self.seed, _S_COV)
        out = [covariance_block(np.asarray(c, dtype=np.float64), rng)
               for c in centrals]
        return [c for c, _ in out], [d for _, d in out]


def global_fit_workload(scale: float = 1.0) -> FitWorkload:
    return FitWorkload(dis=dis_fit_workload(scale), had=had_fit_workload(scale))


@dataclass
class ServingWorkload:
    """Table catalogue and request stream of the serving workload (seed 4)."""
    dis: Workload
    had: Workload
    big_n: int = 2000
    seed: int = 4
    rep_choices: tuple = (1, 4, 16, 100)

    def catalogue(self):
        """Yields ("dis"|"had", table).  dis_fit's 20 DIS, had_fit's 10 hadronic,
        then 2 DIS and 2 hadronic tables with N = big_n."""
        for t in self.dis.tables():
            yield "dis", t
        for t in self.had.tables():
            yield "had", t
        for k in range(2):
            rng = rng_for(self.seed, _S_DATASET0 + k)
            yield "dis", draw_dis_table(rng, self.dis.xgrid, self.big_n)
        for k in range(2):
            rng = rng_for(self.seed, _S_DATASET0 + 10 + k)
            yield "had", draw_had_table(rng, self.had.xgrid, self.big_n)

    def requests(self, n: int, rate: float, ntables: int):
        """Poisson arrivals (seconds), table ids uniform, R uniform over
        ``rep_choices``, and a per-request PDF seed."""
        rng = rng_for(self.seed, 1000 + int(round(rate * 1000)))
        gaps = rng.exponential(1.0 / rate, size=n)
        t = np.cumsum(gaps)
        tab = rng.integers(0, ntables, size=n)
        R = np.asarray(self.rep_choices)[rng.integers(0, len(self.rep_choices), size=n)]
        pseed = rng.integers(0, 2**31 - 1, size=n)
        return t, tab, R, pseed

    def request_pdf(self, nrep: int, pseed: int) -> np.ndarray:
        prm = draw_pdf_params(rng_for(self.seed, _S_PDF))
        rng = np.random.default_rng([self.seed, 7, int(pseed)])
        return sample_pdf(prm, self.dis.xgrid, nrep, 0.05 if nrep > 1 else 0.0, rng)


def serving_workload(scale: float = 1.0, big_n: int = 2000) -> ServingWorkload:
    return ServingWorkload(dis=dis_fit_workload(scale), had=had_fit_workload(scale), big_n=big_n)


# ---------------------------------------------------------------------------
# network PDF parametrisation: initial parameters and preprocessing
# ---------------------------------------------------------------------------

MLP_H1, MLP_H2 = 25, 20   # hidden layer widths of the fit-step network
_S_MLP = 600


def mlp_preprocessing_exponents(nflav: int = NFLAV, seed: int = 3):
    """(alpha [F], beta [F]) of x^alpha (1-x)^beta, drawn like the PDF
    exponents of the workloads (alpha ~ U(-0.3, 0.8), beta ~ U(1, 5))."""
    rng = rng_for(seed, _S_MLP)
    return rng.uniform(-0.3, 0.8, size=nflav), rng.uniform(1.0, 5.0, size=nflav)


def mlp_init(nrep: int, nflav: int = NFLAV, h1: int = MLP_H1, h2: int = MLP_H2,
             seed: int = 3) -> np.ndarray:
    """Initial parameters of ``nrep`` independent networks, float32
    [nrep][P] in the layout W1 [h1][2], b1, W2 [h2][h1], b2, W3 [F][h2], b3:
    weights N(0, 1/fan_in), biases N(0, 0.1); the output bias is centred on 1
    so that the initial PDF is close to its preprocessing factor."""
    rng = rng_for(seed, _S_MLP + 1)
    parts = []
    for r in range(nrep):
        parts.append(np.concatenate([
            rng.normal(scale=1.0 / np.sqrt(2.0), size=h1 * 2), rng.normal(scale=0.1, size=h1),
            rng.normal(scale=1.0 / np.sqrt(h1), size=h2 * h1), rng.normal(scale=0.1, size=h2),
            rng.normal(scale=1.0 / np.sqrt(h2), size=nflav * h2), 1.0 + rng.normal(scale=0.1, size=nflav)]))
    return np.asarray(parts, dtype=np.float32)


# ---------------------------------------------------------------------------
# the shapes of Table 3 (flattened form: FK N x K against a PDF matrix K x R)
# ---------------------------------------------------------------------------

TABLE3_NX = 27       # grid of the base table
TABLE3_NFLAV7 = 7    # 7 x 7 = 49 flavour combinations, K = 49 * 27^2 = 35721
_S_TABLE3 = 500


def table3_mask(seed: int = 5) -> np.ndarray:
    """[14][14] mask with the 49 pairs of 7 seeded flavours (a, b both in the
    set): the base table's 49 flavour combinations."""
    fl = np.sort(rng_for(seed, _S_TABLE3).choice(NFLAV, size=TABLE3_NFLAV7, replace=False))
    mask = np.zeros((NFLAV, NFLAV), dtype=np.uint8)
    mask[np.ix_(fl, fl)] = 1
    return mask


def table3_pdf(nrep: int, seed: int = 5) -> np.ndarray:
    """PDF replicas on the 27-point grid geomspace(1e-7, 1), float64 [14][27][R]."""
    prm = draw_pdf_params(rng_for(seed, _S_TABLE3 + 1))
    return sample_pdf(prm, xgrid_geom(1e-7, 1.0, TABLE3_NX), nrep, 0.05 if nrep > 1 else 0.0,
                      rng_for(seed, _S_TABLE3 + 2))


def table3_fk(n: int, k: int, seed: int = 5) -> np.ndarray:
    """A flattened FK table [n][k] of N(0,1) entries, float32 (the toy tables
    of Table 3 carry no structure beyond their size)."""
    return rng_for(seed, _S_TABLE3 + 3 + n).standard_normal((n, k), dtype=np.float32)


def table3_matrix(k: int, r: int, seed: int = 5) -> np.ndarray:
    """A toy PDF matrix [k][r] for the rows of Table 3 whose K is not a
    luminosity (K = 1e6 .. 1e8): positive, like PDF products, float32."""
    return rng_for(seed, _S_TABLE3 + 4 + r).uniform(0.0, 2.0, size=(k, r)).astype(np.float32)


# ---------------------------------------------------------------------------
# small helpers for tests
# ---------------------------------------------------------------------------

def integer_dis_table(rng, nflav, nx, ndata, nactive, lim=16):
    """Integer-valued DIS table, entries in [-lim, lim]."""
    act = np.sort(rng.choice(nflav, size=nactive, replace=False))
    mask = np.zeros(nflav, dtype=np.uint8)
    mask[act] = 1
    fk = rng.integers(-lim, lim + 1, size=(ndata, nactive, nx)).astype(np.float64)
    return DisTable(mask=mask, fk=fk, xgrid=xgrid_geom(1e-3, 0.9, nx))


def integer_had_table(rng, nflav, nx, ndata, npairs, lim=16):
    """Integer-valued general hadronic table with a random (not necessarily
    symmetric) mask, entries in [-lim, lim]."""
    flat = np.sort(rng.choice(nflav * nflav, size=npairs, replace=False))
    mask = np.zeros(nflav * nflav, dtype=np.uint8)
    mask[flat] = 1
    fk = rng.integers(-lim, lim + 1, size=(ndata, npairs, nx, nx)).astype(np.float64)
    return HadTable(mask=mask.reshape(nflav, nflav), fk=fk,
                    xgrid=xgrid_geom(1e-3, 0.9, nx))


def integer_pdf(rng, nflav, nx, nrep, lim=16):
    return rng.integers(-lim, lim + 1, size=(nflav, nx, nrep)).astype(np.float64)
