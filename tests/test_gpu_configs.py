"""GPU parity at the real sizes of the benchmark configurations, through the C ABI.

Full-size results are checked with the CPU oracle where it can afford it: one FP64 oracle
operator application per checked mass gives the true residual |b - M x|/|b| (1e-8 for mixed
precision), and the FP64 operator itself is compared element by element.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1103_5103_amd as wd

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _n(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def big():
    """32^3x64, near-Haar links and the Gaussian source of the benchmark (same seeds)."""
    dims = (32, 32, 32, 64)
    _say("generating 32^3x64 inputs")
    U = li.random_links(dims, 1.0, 1002)
    b = li.gaussian_field(dims, 2002)
    g = wd.wd_gauge_create(_t(U), hint=wd.params())
    yield dims, U, b, g
    g.close()


def test_apply_full_size(big):
    dims, U, b, g = big
    out = _n(wd.wd_apply(g, 0.134, _t(b)))
    ref = oracle.apply(U, 0.134, b)
    assert np.linalg.norm(out - ref) / np.linalg.norm(ref) < 1e-14


@pytest.mark.parametrize("fmt", ["f32/f16", "f32/bf16", "f16/f16"])
def test_lowprec_operator_full_size(big, fmt):
    """The solvers' low-precision even-odd operator at 32^3x64, in the launch configuration the
    benchmark times (tuned block order, non-temporal loads), against the oracle's M_prec and
    hopping term site by site (tolerances as in test_gpu_lowprec: 1e-2 FP16, 2e-2 BF16, relative
    to the RMS site norm)."""
    dims, U, b, g = big
    spinor, links = fmt.split("/")
    tol = 2e-2 if "bf16" in fmt else 1e-2
    kappa = 0.134
    odd = oracle.parity_mask(dims)
    pe = b.copy()
    pe[odd] = 0
    ref = oracle.mprec(U, kappa, pe)
    ref[odd] = oracle.hopping(U, pe)[odd]
    for red in ("none", "zdot", "outx"):
        out, dots = wd.wd_apply_prec(g, kappa, _t(b), p=wd.params(spinor=spinor, links=links),
                                     v=wd.op_variant(red=red))
        out = _n(out)
        for name, m in (("even", ~odd), ("odd", odd)):
            d = np.linalg.norm((out[m] - ref[m]).reshape(-1, 12), axis=1)
            scale = np.sqrt(np.mean(np.linalg.norm(ref[m].reshape(-1, 12), axis=1) ** 2))
            _say("32^3x64 operator", fmt, red, name, "max", d.max() / scale, "rms", np.sqrt(np.mean(d ** 2)) / scale)
            assert d.max() / scale < tol
        if red == "outx":
            o = out[~odd].reshape(-1)
            assert abs(dots[0, 2] - np.vdot(o, o).real) < tol * np.vdot(o, o).real
        del out


@pytest.mark.parametrize("fmt,rhs", [("f32/f16", -1), ("f32/f16", 0), ("f16/f16", 2)])
def test_lowprec_operator_full_size_nonchiral(big, fmt, rhs):
    """The benchmark's handle (non-chiral spin basis) at 32^3x64: the low-precision operator per
    site against the oracle's chiral M_prec and hopping term (the basis is internal), for one
    system in the tuned launch configuration (rhs -1) and for two systems in one launch, as
    interleaved block pairs (rhs 0) or in the multi-RHS hop (rhs 2, the batched FP16 solves'
    choice at this size); each copy also against the same system alone. Tolerances as in
    test_gpu_lowprec (1e-2 with FP16 storage)."""
    dims, U, b, _ = big
    spinor, links = fmt.split("/")
    kappa = 0.134
    odd = oracle.parity_mask(dims)
    srcs = [b, li.gaussian_field(dims, 2003)]
    refs = []
    for s in srcs:
        pe = s.copy()
        pe[odd] = 0
        ref = oracle.mprec(U, kappa, pe)
        ref[odd] = oracle.hopping(U, pe)[odd]
        refs.append(ref)
    g = wd.wd_gauge_create(_t(U), hint=wd.params(nonchiral=True))
    try:
        p = wd.params(spinor=spinor, links=links)
        for red in ("none", "zdot", "outx"):
            if rhs < 0:
                out, dots = wd.wd_apply_prec(g, kappa, _t(b), p=p, v=wd.op_variant(red=red))
                outs = [_n(out)]
            else:
                out, dots = wd.wd_apply_prec(g, kappa, _t(np.stack(srcs)), p=p,
                                             v=wd.op_variant(red=red, copies=2, rhs_per_thread=rhs))
                outs = list(_n(out))
            del out
            for k, o in enumerate(outs):
                for name, m in (("even", ~odd), ("odd", odd)):
                    d = np.linalg.norm((o[m] - refs[k][m]).reshape(-1, 12), axis=1)
                    scale = np.sqrt(np.mean(np.linalg.norm(refs[k][m].reshape(-1, 12), axis=1) ** 2))
                    _say("32^3x64 non-chiral operator", fmt, "rhs", rhs, red, "copy", k, name, "max",
                         d.max() / scale, "rms", np.sqrt(np.mean(d ** 2)) / scale)
                    assert d.max() / scale < 1e-2
                if red == "outx":
                    e = o[~odd].reshape(-1)
                    assert abs(dots[k, 2] - np.vdot(e, e).real) < 1e-2 * np.vdot(e, e).real
                if rhs >= 0:
                    alone, _ = wd.wd_apply_prec(g, kappa, _t(srcs[k]), p=p,
                                                v=wd.op_variant(red=red, rhs_per_thread=0, tile=0))
                    alone = _n(alone)
                    d = np.linalg.norm((o - alone).reshape(-1, 12), axis=1)
                    assert d.max() / np.sqrt(np.mean(np.linalg.norm(alone.reshape(-1, 12), axis=1) ** 2)) < 1e-2
                    del alone
    finally:
        g.close()


def test_mixed_solve_full_size_bench_config(big):
    """The benchmark's sequential mixed solve (FP32 spinors, FP16 links, delta 1e-3, poly guess)
    for the lightest and heaviest masses of the 8."""
    dims, U, b, g = big
    kappas = [0.120 + 0.002 * k for k in range(8)]
    xs, sts = wd.wd_multimass_solve(g, kappas, _t(b), p=wd.params(tol=1e-8, spinor="f32", links="f16", delta=1e-3))
    for i in (0, 7):
        res = oracle.true_residual(U, kappas[i], _n(xs[i]), b)
        _say("32^3x64 mixed", kappas[i], sts[i], "oracle residual", res)
        assert res < 1e-8
        assert abs(sts[i]["true_rel_res"] - res) < 1e-2 * res


def test_mixed_solve_full_size_8real_links(big):
    """The benchmark's sequential and batched mixed solves with 8-real FP16 links (recon = 8):
    oracle residual of the lightest and heaviest masses; iteration counts within two per mass of
    the 12-real links' (the rebuilt links are a small perturbation of the operator)."""
    dims, U, b, g = big
    kappas = [0.120 + 0.002 * k for k in range(8)]
    p8 = wd.params(tol=1e-8, spinor="f32", links="f16", recon=8, delta=1e-3)
    p12 = wd.params(tol=1e-8, spinor="f32", links="f16", delta=1e-3)
    _, s12 = wd.wd_multimass_solve(g, kappas, _t(b), p=p12)
    for method in (wd.WD_METHOD_SEQUENTIAL, wd.WD_METHOD_BATCHED):
        xs, sts = wd.wd_multimass_solve(g, kappas, _t(b), method=method, p=p8)
        for i in (0, 7):
            res = oracle.true_residual(U, kappas[i], _n(xs[i]), b)
            _say("32^3x64 8-real", method, kappas[i], sts[i], "oracle residual", res)
            assert res < 1e-8
            assert abs(sts[i]["true_rel_res"] - res) < 1e-2 * res
        if method == wd.WD_METHOD_SEQUENTIAL:
            assert all(a["iters"] <= c["iters"] + 2 for a, c in zip(sts, s12)), ([a["iters"] for a in sts],
                                                                               [c["iters"] for c in s12])


def test_mixed_solve_full_size_fp16_spinors(big):
    """The benchmark's sequential and batched mixed solves with FP16 spinors (per-site scale) and
    FP16 12-real links: oracle residual of the lightest and heaviest masses."""
    dims, U, b, g = big
    kappas = [0.120 + 0.002 * k for k in range(8)]
    p = wd.params(tol=1e-8, spinor="f16", links="f16", delta=1e-3)
    for method in (wd.WD_METHOD_SEQUENTIAL, wd.WD_METHOD_BATCHED):
        xs, sts = wd.wd_multimass_solve(g, kappas, _t(b), method=method, p=p)
        for i in (0, 7):
            res = oracle.true_residual(U, kappas[i], _n(xs[i]), b)
            _say("32^3x64 FP16 spinors", method, kappas[i], sts[i], "oracle residual", res)
            assert sts[i]["status"] == 0
            assert res < 1e-8
            assert abs(sts[i]["true_rel_res"] - res) < 1e-2 * res


def test_multishift_full_size(big):
    dims, U, b, g = big
    kappas = [0.120 + 0.002 * k for k in range(8)]
    xs, sts = wd.bicgstab_m_solve(g, kappas, _t(b), p=wd.params(tol=1e-8, mixed=False, eo=False))
    for i in (0, 7):
        res = oracle.true_residual(U, kappas[i], _n(xs[i]), b)
        _say("32^3x64 BiCGstab-M", kappas[i], sts[i], "oracle residual", res)
        assert res < 1e-8


def test_normal_equations_full_size(big):
    """CG-M and the sequential mixed CG on the 32^3x64 lattice, kappa 0.134, the 8 shifts the
    benchmark uses: the oracle's FP64 residual |b_e - (A + sigma) x| / |b_e| of the smallest and
    the largest shift of each method, and the two methods' solutions agree."""
    dims, U, b, g = big
    kappa = 0.134
    sig = [0.0] + [25.0 * 2 ** k for k in range(7)]
    be = oracle.even_part(b)
    xm, sm = wd.wd_normal_solve(g, kappa, sig, _t(b), method=wd.WD_METHOD_MULTISHIFT, p=wd.params(tol=1e-8, mixed=False))
    xq, sq = wd.wd_normal_solve(g, kappa, sig, _t(b), p=wd.params(tol=1e-8, spinor="f32", links="f16", delta=1e-3))
    for i in (0, 7):
        for xs, sts, name in ((xm, sm, "cg-m"), (xq, sq, "cg seq")):
            x = _n(xs[i])
            res = np.linalg.norm(be - oracle.normal_apply(U, kappa, sig[i], x)) / np.linalg.norm(be)
            _say("32^3x64", name, sig[i], sts[i], "oracle residual", res)
            assert res < 1.5e-8
            assert abs(sts[i]["true_rel_res"] - res) < 0.05 * res
        d = _n(xm[i]) - _n(xq[i])
        assert np.linalg.norm(d) / np.linalg.norm(_n(xm[i])) < 4e-7


def test_multimass_16x32_fp64_vs_mixed():
    """16^3x32, 6 masses: BiCGstab-M (FP64) and sequential even-odd mixed BiCGstab with FP16
    spinors and links, both to 1e-8 for every mass."""
    dims = (16, 16, 16, 32)
    U = li.random_links(dims, 1.0, 1001)
    b = li.gaussian_field(dims, 2001)
    kappas = [0.120, 0.122, 0.124, 0.126, 0.128, 0.130]
    g = wd.wd_gauge_create(_t(U))
    bd = _t(b)
    xm, stm = wd.bicgstab_m_solve(g, kappas, bd, p=wd.params(tol=1e-8, mixed=False, eo=False))
    xs, sts = wd.wd_multimass_solve(g, kappas, bd, p=wd.params(tol=1e-8, spinor="f16", links="f16"))
    for k, a, c in zip(kappas, xm, xs):
        ra = oracle.true_residual(U, k, _n(a), b)
        rc = oracle.true_residual(U, k, _n(c), b)
        assert ra < 1e-8 and rc < 1e-8, (k, ra, rc)
        # the two solutions agree within the condition number times the tolerance
        assert np.linalg.norm(_n(a) - _n(c)) / np.linalg.norm(_n(a)) < 1e-6
    # error against the oracle's own solution, per mass (its FP64 even-odd BiCGstab to 1e-12)
    for k, a, c in zip(kappas, xm, xs):
        xo = oracle.bicgstab(U, k, b, tol=1e-12, eo=True)[0]
        ea = np.linalg.norm(_n(a) - xo) / np.linalg.norm(xo)
        ec = np.linalg.norm(_n(c) - xo) / np.linalg.norm(xo)
        _say("16^3x32 kappa", k, "error vs oracle: BiCGstab-M", ea, "mixed sequential", ec)
        assert ea < 1e-7 and ec < 1e-7
    g.close()


def test_batched_full_config():
    """12 spin-colour point sources x 4 masses on 16^3x32, plus 8^4, 12^4 and 16^4 lattices with
    4 point sources x the same 4 masses each: 96 systems in one batched solve."""
    kappas = [0.124, 0.126, 0.128, 0.130]
    lattices = [((16, 16, 16, 32), 1100, 12), ((8, 8, 8, 8), 1101, 4), ((12, 12, 12, 12), 1102, 4),
                ((16, 16, 16, 16), 1103, 4)]
    systems, refs, gauges = [], [], []
    for dims, seed, nsrc in lattices:
        U = li.random_links(dims, 1.0, seed)
        g = wd.wd_gauge_create(_t(U), hint=wd.params(spinor="f16", links="f16"))
        gauges.append(g)
        for s in range(nsrc):
            b = li.point_source(dims, spin=s % 4, colour=s // 4)
            bd = _t(b)
            for k in kappas:
                systems.append((g, k, bd, torch.zeros(g.field_shape, dtype=torch.complex128, device=DEV)))
                refs.append((U, k, b))
    _say("batched systems:", len(systems))
    sts = wd.wd_batch_solve(systems, p=wd.params(tol=1e-8, spinor="f16", links="f16"))
    worst = 0.0
    for (g, k, bd, x), (U, kk, b), s in zip(systems, refs, sts):
        assert s["status"] == 0, s
        worst = max(worst, oracle.true_residual(U, kk, _n(x), b))
    _say("batched worst oracle residual", worst)
    assert worst < 1e-8
    for g in gauges:
        g.close()


def test_gradient_finite_differences_8444():
    """L = Re<eta, M(0.125)^{-1} b> on 8^4: the GPU gradient (autograd backward through the library)
    against central differences h = 1e-6 along +h and +ih of 20 random link entries, with the
    perturbed solves done by the CPU oracle."""
    dims = (8, 8, 8, 8)
    kappa = 0.125
    U = li.random_links(dims, 1.0, 1050)
    b = li.gaussian_field(dims, 2050)
    eta = li.gaussian_field(dims, 2051)
    Ud = _t(U).requires_grad_(True)
    x = wd.wilson_solve(Ud, _t(b), kappa, params=wd.params(tol=1e-14, mixed=False, max_iter=500))
    torch.real(torch.sum(torch.conj(_t(eta)) * x)).backward()
    G = _n(Ud.grad).reshape(-1)

    def loss(Uc):
        xs, _, _, _ = oracle.bicgstab(Uc, kappa, b, tol=1e-15, maxit=1000, eo=True)
        return float(np.real(np.vdot(eta, xs)))

    rng = np.random.default_rng(7)
    flat = U.reshape(-1)
    h = 1e-6
    for _ in range(20):
        j = int(rng.integers(0, flat.size))
        fd = []
        for step in (h, 1j * h):
            Up = flat.copy()
            Up[j] += step
            Um = flat.copy()
            Um[j] -= step
            fd.append((loss(Up.reshape(U.shape)) - loss(Um.reshape(U.shape))) / (2 * h))
        d = fd[0] + 1j * fd[1]
        assert abs(d - G[j]) < 1e-6 * max(1.0, abs(d)), (j, d, G[j])


def test_gradient_mixed_16x32():
    """Forward and backward in mixed precision on 16^3x32: grad_b solves the adjoint system to 1e-8."""
    dims = (16, 16, 16, 32)
    kappa = 0.125
    U = li.random_links(dims, 1.0, 1060)
    b = li.gaussian_field(dims, 2060)
    eta = li.gaussian_field(dims, 2061)
    Ud = _t(U).requires_grad_(True)
    bd = _t(b).requires_grad_(True)
    x = wd.wilson_solve(Ud, bd, kappa, params=wd.params(tol=1e-8))
    torch.real(torch.sum(torch.conj(_t(eta)) * x)).backward()
    lam = _n(bd.grad)
    r = eta - oracle.apply(U, kappa, lam, dag=True)
    assert np.linalg.norm(r) / np.linalg.norm(eta) < 1e-8
    assert oracle.true_residual(U, kappa, _n(x), b) < 1e-8
    assert np.isfinite(_n(Ud.grad)).all()
