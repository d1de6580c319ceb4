"""GPU FP64 chi2 against the oracle (Cholesky of its own, substitutions in
FP64) and the differentiable fit step: chi2 -> d chi2/d sigma -> adjoint ->
d chi2/d f, checked against the oracle's analytic gradient and against the
oracle's own FP64 central differences with h = 1e-4."""
import sys

import numpy as np
import pytest

import oracle
from paper_1909_10547_amd import autograd, fkconv, synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = fkconv.Context(0)
    yield c
    c.close()


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def test_chi2_matches_oracle(ctx):
    rng = np.random.default_rng(1)
    sizes = [1, 2, 31, 32, 33, 70, 150]
    Cs = []
    for n in sizes:
        A = rng.normal(size=(n, n))
        Cs.append(A @ A.T + n * np.eye(n))
    Ntot = sum(sizes)
    for R in (1, 100, 130):
        sig = f32(rng.normal(size=(Ntot, R)) * 3)
        D = rng.normal(size=Ntot)
        cv = fkconv.fk_load_covariance(ctx.ctx, Cs)
        chi, d = fkconv.fk_chi2(ctx.ctx, cv, torch.from_numpy(sig.astype(np.float32)).cuda(),
                                torch.from_numpy(D).cuda())
        torch.cuda.synchronize()
        ref, dref = oracle.chi2([oracle.cholesky(C) for C in Cs], sig, D)
        e = float(np.max(np.abs(chi.cpu().numpy() - ref) / np.abs(ref)))
        eg = oracle.normwise_rel(d.cpu().double().numpy(), dref)
        say(f"chi2 R={R}: rel err {e:.2e}, gradient (FP32 output) {eg:.2e}")
        assert e < 1e-11
        assert eg < 1e-6
        fkconv.fk_unload_covariance(ctx.ctx, cv)


def test_chi2_large_block(ctx):
    """A block of 1100 points (35 row tiles: the split products take five
    tiles per entry there) beside a small one."""
    rng = np.random.default_rng(7)
    Cs = []
    for n in (1100, 40):
        A = rng.normal(size=(n, n))
        Cs.append(A @ A.T + n * np.eye(n))
    Ntot = 1140
    R = 16
    sig = f32(rng.normal(size=(Ntot, R)) * 3)
    D = rng.normal(size=Ntot)
    cv = fkconv.fk_load_covariance(ctx.ctx, Cs)
    chi, d = fkconv.fk_chi2(ctx.ctx, cv, torch.from_numpy(sig.astype(np.float32)).cuda(),
                            torch.from_numpy(D).cuda())
    torch.cuda.synchronize()
    ref, dref = oracle.chi2([oracle.cholesky(C) for C in Cs], sig, D)
    e = float(np.max(np.abs(chi.cpu().numpy() - ref) / np.abs(ref)))
    eg = oracle.normwise_rel(d.cpu().double().numpy(), dref)
    say(f"chi2 large block: rel err {e:.2e}, gradient (FP32 output) {eg:.2e}")
    assert e < 1e-10
    assert eg < 1e-6
    fkconv.fk_unload_covariance(ctx.ctx, cv)


def test_not_positive_definite(ctx):
    C = np.eye(5)
    C[3, 3] = -1.0
    with pytest.raises(fkconv.FKError) as e:
        fkconv.fk_load_covariance(ctx.ctx, [np.eye(3), C])
    assert e.value.code == fkconv.FK_E_NOTPD


def test_fit_gradient_against_oracle(ctx):
    # datasets of the DIS and hadronic fit workloads (reduced sizes), covariance per dataset
    w = synth.global_fit_workload(scale=0.04)
    dis_t = [w.dis.table(d) for d in range(4)]
    had_t = [w.had.table(d) for d in range(3)]
    R = 6
    pdf = f32(w.pdf()[:, :, :R])
    cen = w.central_pdf()
    centrals = [oracle.dis(t.mask, t.fk, cen)[:, 0] for t in dis_t] + \
               [oracle.had(t.mask, t.fk, cen)[:, 0] for t in had_t]
    Cs, Ds = w.covariances(centrals)
    D = np.concatenate(Ds)
    hd = [ctx.load(t, "f32") for t in dis_t]
    hh = [ctx.load(t, "f32") for t in had_t]
    gd = fkconv.fk_group_create(ctx.ctx, hd)
    gh = fkconv.fk_group_create(ctx.ctx, hh)
    cv = fkconv.fk_load_covariance(ctx.ctx, Cs)
    x = torch.from_numpy(pdf.astype(np.float32)).cuda().requires_grad_(True)
    sigma = torch.cat([autograd.fk_conv(ctx.ctx, gd, x), autograd.fk_conv(ctx.ctx, gh, x)])
    chi = autograd.fk_chi2(ctx.ctx, cv, sigma, torch.from_numpy(D).cuda())
    chi.sum().backward()
    g = x.grad.double().cpu().numpy()

    def oracle_chi2(f):
        s = np.concatenate([oracle.dis(t.mask, t.fk, f) for t in dis_t] +
                           [oracle.had(t.mask, t.fk, f) for t in had_t])
        return s

    Ls = [oracle.cholesky(C) for C in Cs]
    s = oracle_chi2(pdf)
    c_ref, dchi = oracle.chi2(Ls, s, D)
    gref = np.zeros_like(pdf)
    off = 0
    for t in dis_t:
        gref += oracle.dis_grad(t.mask, t.fk, dchi[off:off + t.ndata])
        off += t.ndata
    for t in had_t:
        gref += oracle.had_grad(t.mask, t.fk, pdf, dchi[off:off + t.ndata])
        off += t.ndata
    e = oracle.normwise_rel(g, gref)
    ec = float(np.max(np.abs(chi.detach().cpu().numpy() - c_ref) / c_ref))
    say(f"fit step: chi2 rel err {ec:.2e}, d chi2/d f normwise vs oracle {e:.2e}")
    # sigma enters as FP32 (~1e-7 of |sigma|) and chi2 depends on the
    # residual sigma - D only, so allow that error amplified by |sigma|/|e|
    assert ec < 1e-4 and e < 1e-4
    # oracle FP64 central differences, h = 1e-4 (relative to |f|)
    rng = np.random.default_rng(2)
    nz = np.argwhere(np.abs(gref[:, :, 0]) > 1e-3 * np.max(np.abs(gref[:, :, 0])))
    for k in rng.choice(len(nz), size=min(12, len(nz)), replace=False):
        a, al = nz[k]
        hstep = 1e-4 * max(1.0, abs(pdf[a, al, 0]))
        fp = pdf.copy(); fp[a, al, 0] += hstep
        fm = pdf.copy(); fm[a, al, 0] -= hstep
        cp, _ = oracle.chi2(Ls, oracle_chi2(fp), D, want_grad=False)
        cm, _ = oracle.chi2(Ls, oracle_chi2(fm), D, want_grad=False)
        fd = (cp[0] - cm[0]) / (2 * hstep)
        say(f"  f[{a},{al},0]: FD {fd:.6e} GPU {g[a, al, 0]:.6e}")
        assert abs(fd - g[a, al, 0]) <= 1e-3 * abs(fd) + 1e-6 * np.max(np.abs(gref[:, :, 0]))
    for hdl in (gd, gh, *hd, *hh):
        fkconv.fk_unload_table(ctx.ctx, hdl)
    fkconv.fk_unload_covariance(ctx.ctx, cv)


@pytest.mark.parametrize("cond", [1e4, 1e8, 1e12])
def test_chi2_ill_conditioned_covariance(ctx, cond):
    """The per-call products use the triangular inverse of L computed at load
    time; on covariances with condition numbers up to 1e12 (eigenvalues
    spread log-uniformly, random eigenvectors) chi2 and its gradient still
    match the oracle's substitutions to the accuracy FP64 allows for that
    condition number (relative error <= 1e-15 * cond, at least 1e-11)."""
    rng = np.random.default_rng(int(np.log10(cond)))
    sizes = [40, 97]
    Cs = []
    for n in sizes:
        Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
        ev = np.geomspace(1.0, 1.0 / cond, n)
        C = (Q * ev) @ Q.T
        Cs.append(0.5 * (C + C.T))
    Ntot, R = sum(sizes), 16
    sig = f32(rng.normal(size=(Ntot, R)))
    D = rng.normal(size=Ntot)
    cv = fkconv.fk_load_covariance(ctx.ctx, Cs)
    chi, d = fkconv.fk_chi2(ctx.ctx, cv, torch.from_numpy(sig.astype(np.float32)).cuda(),
                            torch.from_numpy(D).cuda())
    torch.cuda.synchronize()
    ref, dref = oracle.chi2([oracle.cholesky(C) for C in Cs], sig, D)
    e = float(np.max(np.abs(chi.cpu().numpy() - ref) / np.abs(ref)))
    dgot = d.cpu().double().numpy()
    # the gradient is returned in FP32: compare to the FP32-rounded reference scale
    eg = oracle.normwise_rel(dgot, dref)
    say(f"chi2 cond={cond:.0e}: rel err {e:.2e}, gradient {eg:.2e}")
    fkconv.fk_unload_covariance(ctx.ctx, cv)
    assert e <= max(1e-11, 1e-15 * cond)
    assert eg <= max(1e-6, 1e-15 * cond)
