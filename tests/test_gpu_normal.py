"""GPU parity of CG / CG-M on the shifted even-site normal equations (M_prec^dag M_prec + sigma) x = b_e
against the CPU oracle on the same seeded inputs.

The residual bar is the oracle's FP64 |b_e - (A + sigma) x| / |b_e| below the requested tolerance
(times 1.5 for rounding of the check itself); the distance to the oracle's own solution is bounded
by cond(A + sigma) x tol, and cond(M_prec^dag M_prec) < 4 on these near-Haar links (the spectrum of
M_prec lies within a factor < 2), so 20 x tol is a safe bound. Odd sites of every solution are zero.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import oracle
import paper_1103_5103_amd as wd

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
SIGMAS = [0.0, 25.0, 100.0, 400.0]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _n(t):
    return t.detach().cpu().numpy()


def _say(*a):
    print(*a, flush=True)


def _check(U, kappa, sigmas, b, xs, sts, tol, ref=None):
    be = oracle.even_part(b)
    odd = oracle.parity_mask((b.shape[3], b.shape[2], b.shape[1], b.shape[0]))
    for i, (s, xd, st) in enumerate(zip(sigmas, xs, sts)):
        x = _n(xd)
        assert st["status"] == 0, st
        assert np.abs(x[odd]).max() == 0.0
        res = np.linalg.norm(be - oracle.normal_apply(U, kappa, s, x)) / np.linalg.norm(be)
        assert res < 1.5 * tol, (s, res)
        assert abs(st["true_rel_res"] - res) < 0.05 * res + 1e-15, (st["true_rel_res"], res)
        if ref is not None:
            err = np.linalg.norm(x - ref[i]) / np.linalg.norm(ref[i])
            assert err < 20 * tol, (s, err)


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 4, 2), (6, 4, 2, 10), (16, 8, 8, 16)])
def test_cg_m_fp64(dims):
    _say("cg-m", dims)
    U = li.random_links(dims, 1.0, 1301)
    b = li.gaussian_field(dims, 2301)
    kappa, tol = 0.13, 1e-10
    g = wd.wd_gauge_create(_t(U))
    xs, sts = wd.wd_normal_solve(g, kappa, SIGMAS, _t(b), method=wd.WD_METHOD_MULTISHIFT,
                                 p=wd.params(tol=tol, mixed=False))
    ref, it, st, conv = oracle.cg_m(U, kappa, SIGMAS, b, tol=tol)
    _say("  iters", [s["iters"] for s in sts], "oracle", conv)
    _check(U, kappa, SIGMAS, b, xs, sts, tol, ref)
    for s, c in zip(sts, conv):
        assert abs(s["iters"] - c) <= 1
    g.close()


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 4, 2), (16, 8, 8, 16)])
@pytest.mark.parametrize("spinor,links", [("f32", "f16"), ("f16", "f16"), ("f32", "bf16"), ("f32", "f32")])
def test_cg_sequential_mixed(dims, spinor, links):
    _say("cg seq mixed", dims, spinor, links)
    U = li.random_links(dims, 1.0, 1302)
    b = li.gaussian_field(dims, 2302)
    kappa, tol = 0.128, 1e-8
    g = wd.wd_gauge_create(_t(U))
    p = wd.params(tol=tol, spinor=spinor, links=links, delta=0.1)
    xs, sts = wd.wd_normal_solve(g, kappa, SIGMAS, _t(b), p=p)
    ref = [oracle.cg(U, kappa, s, b, tol=1e-12)[0] for s in SIGMAS]
    _say("  iters", [s["iters"] for s in sts], "reliable", [s["reliable_updates"] for s in sts])
    _check(U, kappa, SIGMAS, b, xs, sts, tol, ref)
    g.close()


@pytest.mark.parametrize("method", ["sequential_fp64", "batched", "batched_dc", "sequential_dc", "no_guess"])
def test_cg_methods(method):
    dims = (8, 8, 4, 8)
    _say("cg", method)
    U = li.random_links(dims, 1.0, 1303)
    b = li.gaussian_field(dims, 2303)
    kappa = 0.13
    g = wd.wd_gauge_create(_t(U))
    tol = 1e-10 if method == "sequential_fp64" else 1e-8
    dc = method.endswith("_dc")
    p = wd.params(tol=tol, mixed=method != "sequential_fp64", defect_correction=dc, delta=1e-3 if dc else 0.1)
    m = wd.WD_METHOD_BATCHED if method.startswith("batched") else wd.WD_METHOD_SEQUENTIAL
    guess = wd.WD_GUESS_NONE if method == "no_guess" else wd.WD_GUESS_POLY
    xs, sts = wd.wd_normal_solve(g, kappa, SIGMAS, _t(b), method=m, guess=guess, p=p)
    ref = [oracle.cg(U, kappa, s, b, tol=1e-12)[0] for s in SIGMAS]
    _say("  iters", [s["iters"] for s in sts], "reliable", [s["reliable_updates"] for s in sts])
    _check(U, kappa, SIGMAS, b, xs, sts, tol, ref)
    g.close()


def test_cg_guess_reduces_iterations_and_matches_oracle_counts():
    """FP64 sequential CG with the Lagrange guess: the same iteration counts as the oracle's driver
    (within one), fewer in total than with zero start vectors."""
    dims = (8, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1304)
    b = li.gaussian_field(dims, 2304)
    kappa, tol = 0.128, 1e-10
    sig = [0.0, 25.0, 50.0, 100.0, 200.0]
    g = wd.wd_gauge_create(_t(U))
    p = wd.params(tol=tol, mixed=False)
    _, sg = wd.wd_normal_solve(g, kappa, sig, _t(b), p=p, guess=wd.WD_GUESS_POLY)
    _, sn = wd.wd_normal_solve(g, kappa, sig, _t(b), p=p, guess=wd.WD_GUESS_NONE)
    _, itg = oracle.normal_sequential(U, kappa, sig, b, tol=tol, guess="poly")
    ig = [s["iters"] for s in sg]
    _say("guess", ig, "oracle", itg, "none", [s["iters"] for s in sn])
    assert all(abs(a - c) <= 1 for a, c in zip(ig, itg))
    assert sum(ig) < sum(s["iters"] for s in sn)
    g.close()


def test_cg_temporal_gauge_and_repeated_and_zero():
    """A temporal-gauge handle gives the caller-gauge solutions; a repeated shift; a zero source."""
    dims = (8, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1305)
    b = li.gaussian_field(dims, 2305)
    kappa, tol = 0.125, 1e-8
    sig = [100.0, 0.0, 100.0]
    ref = [oracle.cg(U, kappa, s, b, tol=1e-12)[0] for s in sig]
    for tg in (False, True):
        g = wd.wd_gauge_create(_t(U), hint=wd.params(temporal_gauge=tg))
        for m in (wd.WD_METHOD_SEQUENTIAL, wd.WD_METHOD_MULTISHIFT, wd.WD_METHOD_BATCHED):
            p = wd.params(tol=tol, mixed=m != wd.WD_METHOD_MULTISHIFT)
            xs, sts = wd.wd_normal_solve(g, kappa, sig, _t(b), method=m, p=p)
            _say("tg", tg, "method", m, [s["iters"] for s in sts])
            _check(U, kappa, sig, b, xs, sts, tol, ref)
            z, zs = wd.wd_normal_solve(g, kappa, sig, _t(np.zeros_like(b)), method=m, p=p)
            assert all(float(torch.abs(v).max()) == 0.0 for v in z) and all(s["status"] == 0 for s in zs)
        g.close()


def test_cg_rejects_bad_arguments():
    dims = (4, 4, 4, 4)
    U = li.random_links(dims, 1.0, 1306)
    g = wd.wd_gauge_create(_t(U))
    b = _t(li.gaussian_field(dims, 2306))
    with pytest.raises(wd.WdError):
        wd.wd_normal_solve(g, 0.12, [-1.0], b)
    with pytest.raises(wd.WdError):
        wd.wd_normal_solve(g, 0.12, [1.0], b, guess=wd.WD_GUESS_MINRES)
    with pytest.raises(wd.WdError):
        wd.wd_normal_solve(g, 0.12, [1.0], b, p=wd.params(dagger=True))
    g.close()


@pytest.mark.parametrize("delta", [1e-4, 1e-5])
def test_cg_small_reliable_delta(delta):
    """Reliable updates far apart: the low-precision iterated residual falls below what the FP16
    operator resolves, so at an update the true residual exceeds the iterated one; the solver
    then restarts or rebuilds p from the true residual and still converges."""
    dims = (8, 8, 8, 8)
    U = li.random_links(dims, 1.0, 1307)
    b = li.gaussian_field(dims, 2307)
    kappa, tol = 0.134, 1e-8
    sig = [0.0, 100.0, 1600.0]
    g = wd.wd_gauge_create(_t(U))
    for m in (wd.WD_METHOD_SEQUENTIAL, wd.WD_METHOD_BATCHED):
        xs, sts = wd.wd_normal_solve(g, kappa, sig, _t(b), method=m,
                                     p=wd.params(tol=tol, spinor="f32", links="f16", delta=delta))
        _say("delta", delta, "method", m, [s["iters"] for s in sts], [s["reliable_updates"] for s in sts])
        _check(U, kappa, sig, b, xs, sts, tol)
        assert max(s["iters"] for s in sts) < 60
    g.close()


def test_cg_single_shift_and_iteration_cap():
    """CG-M with one shift is plain CG (its status is committed without the shift sweep); a cap on
    the iterations ends every method with WD_ERR_NOCONV and filled statistics."""
    dims = (8, 4, 4, 4)
    U = li.random_links(dims, 1.0, 1308)
    b = li.gaussian_field(dims, 2308)
    kappa, tol = 0.13, 1e-10
    g = wd.wd_gauge_create(_t(U))
    xs, sts = wd.wd_normal_solve(g, kappa, [50.0], _t(b), method=wd.WD_METHOD_MULTISHIFT,
                                 p=wd.params(tol=tol, mixed=False))
    ref, it, st, _ = oracle.cg(U, kappa, 50.0, b, tol=tol)
    _check(U, kappa, [50.0], b, xs, sts, tol, [ref])
    assert abs(sts[0]["iters"] - it) <= 1
    for m in (wd.WD_METHOD_MULTISHIFT, wd.WD_METHOD_SEQUENTIAL, wd.WD_METHOD_BATCHED):
        p = wd.params(tol=1e-12, max_iter=3, mixed=m != wd.WD_METHOD_MULTISHIFT)
        xs, sts = wd.wd_normal_solve(g, kappa, [0.0, 100.0], _t(b), method=m, p=p, raise_on_fail=False)
        _say("cap", m, sts)
        assert all(s["status"] == 4 for s in sts)  # WD_ERR_NOCONV
        assert all(1 <= s["iters"] <= 3 + 3 for s in sts) and all(s["true_rel_res"] > 0 for s in sts)
        assert all(np.isfinite(_n(x)).all() for x in xs)
    g.close()
