"""GPU parity of the mixed-precision solves with 8-real FP16 links (recon = 8) against the CPU oracle.

The 8-real format stores u01, u02, u10 and the phases of u00 and u20 of each SU(3) link and
rebuilds the rest from unitarity (the further link compression of Sec. 4). It only changes the
low-precision operator of the iteration; the FP64 reliable updates use the exact links, so every
solve must reach the oracle's FP64 residual bar. Rebuilding a link wrongly (a sign, a swapped
element, a phase in the wrong unit) makes the low-precision operator an O(1) perturbation of the
true one, which would stall the inner iteration between reliable updates: the iteration count is
therefore held to that of the 12-real format on the same system.
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


@pytest.mark.parametrize("spinor", ["f32", "f16"])
@pytest.mark.parametrize("dims,eps", [((8, 8, 8, 8), 1.0), ((6, 4, 4, 10), 1.0), ((72, 4, 4, 4), 1.0),
                                      ((16, 32, 4, 4), 1.0), ((8, 8, 8, 8), 0.3)])
def test_link8_mixed_solve(dims, eps, spinor):
    _say("link8 solve", dims, eps, spinor)
    U = li.random_links(dims, eps, 1501)
    b = li.gaussian_field(dims, 2501)
    kappa = 0.13
    g = wd.wd_gauge_create(_t(U))
    x8, st8 = wd.bicgstab_solve(g, kappa, _t(b), p=wd.params(tol=1e-8, spinor=spinor, links="f16", recon=8))
    x12, st12 = wd.bicgstab_solve(g, kappa, _t(b), p=wd.params(tol=1e-8, spinor=spinor, links="f16", recon=12))
    res = oracle.true_residual(U, kappa, _n(x8), b)
    _say("  8-real", st8, "oracle residual", res, "| 12-real iters", st12["iters"])
    assert st8["status"] == 0
    assert res < 1e-8
    assert abs(st8["true_rel_res"] - res) < 0.05 * res + 1e-15
    assert st8["iters"] <= 1.25 * st12["iters"] + 5
    g.close()


def test_link8_multimass_batched_and_normal_equations():
    dims = (8, 8, 8, 16)
    U = li.random_links(dims, 1.0, 1502)
    b = li.gaussian_field(dims, 2502)
    kappas = [0.120, 0.125, 0.130]
    g = wd.wd_gauge_create(_t(U), hint=wd.params(recon=8))
    p = wd.params(tol=1e-8, recon=8)
    xs, sts = wd.wd_multimass_solve(g, kappas, _t(b), method=wd.WD_METHOD_SEQUENTIAL, guess=wd.WD_GUESS_POLY, p=p)
    for k, x, st in zip(kappas, xs, sts):
        res = oracle.true_residual(U, k, _n(x), b)
        _say("  sequential", k, st, res)
        assert st["status"] == 0 and res < 1e-8
    bd = _t(b)
    outs = [torch.zeros_like(bd) for _ in kappas]
    sts = wd.wd_batch_solve([(g, k, bd, o) for k, o in zip(kappas, outs)], p=p)
    for k, x, st in zip(kappas, outs, sts):
        res = oracle.true_residual(U, k, _n(x), b)
        _say("  batched", k, st, res)
        assert st["status"] == 0 and res < 1e-8
    # the normal equations run the adjoint hop on the same 8-real links
    sigmas = [0.0, 100.0]
    be = oracle.even_part(b)
    xs, sts = wd.wd_normal_solve(g, 0.13, sigmas, bd, method=wd.WD_METHOD_SEQUENTIAL, p=p)
    for s, x, st in zip(sigmas, xs, sts):
        res = np.linalg.norm(be - oracle.normal_apply(U, 0.13, s, _n(x))) / np.linalg.norm(be)
        _say("  normal", s, st, res)
        assert st["status"] == 0 and res < 1.5e-8
    g.close()


def test_link8_refusals():
    dims = (4, 4, 4, 8)
    b = _t(li.gaussian_field(dims, 2503))
    p8 = wd.params(recon=8)
    # unit links: row 0 is (1, 0, 0) and row 1 cannot be rebuilt from u10 and the phases
    g = wd.wd_gauge_create(_t(li.unit_links(dims)))
    with pytest.raises(wd.WdError) as e:
        wd.bicgstab_solve(g, 0.12, b, p=p8)
    assert e.value.code == 7
    # the 12-real format still solves the same system
    x, st = wd.bicgstab_solve(g, 0.12, b)
    assert st["status"] == 0
    g.close()
    U = li.random_links(dims, 1.0, 1503)
    # the temporal gauge turns time links into unit matrices
    g = wd.wd_gauge_create(_t(U), hint=wd.params(temporal_gauge=True))
    with pytest.raises(wd.WdError) as e:
        wd.bicgstab_solve(g, 0.12, b, p=p8)
    assert e.value.code == 7
    g.close()
    g = wd.wd_gauge_create(_t(U))
    # 8-real links exist in FP16 only
    for links in ("f32", "bf16"):
        with pytest.raises(wd.WdError) as e:
            wd.bicgstab_solve(g, 0.12, b, p=wd.params(links=links, recon=8))
        assert e.value.code == 7
    g.close()
    # links that are not SU(3) would change the operator
    g = wd.wd_gauge_create(_t(U * 1.05))
    with pytest.raises(wd.WdError) as e:
        wd.bicgstab_solve(g, 0.12, b, p=p8)
    assert e.value.code == 7
    g.close()
