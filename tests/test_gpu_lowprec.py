"""GPU parity of the solvers' low-precision operator, site by site, against the FP64 oracle.

wd_apply_prec runs the same hop-kernel instantiations the solvers launch (storage formats, fused
epilogues and reductions, LDS staging on or off, non-temporal loads on or off, block orders,
temporal gauge, interleaved systems, the adjoint hops) and returns
    out_e = M_prec in_e      (Sec. 6.2.3, eq. eo4)
    out_o = D_oe in_e        (Sec. 2, eq. 3-4: the hopping term from even to odd sites)
which the oracle computes in FP64 as mprec(U, kappa, in_e) and hopping(U, in_e) on the odd sites.

Error measure: per site, |out(n) - ref(n)| / rms_n |ref(n)| (the 12-component site norm divided by
the field's RMS site norm, so a site whose value is small by chance is not over-weighted), max
over the sites of each parity. Tolerances follow from the storage formats:
    FP64 spinors and links              1e-13  (only the summation order differs)
    FP32 spinors, FP32 links            1e-6   (unit roundoff 6e-8, about a dozen rounded terms)
    FP16 links or FP16 spinors          1e-2   (unit roundoff 4.9e-4 per stored element)
    BF16 links                          2e-2   (unit roundoff 3.9e-3)
    8-real FP16 links                   5e-2 max, 5e-3 RMS (the rebuilt row 1 divides by
                                        1 - |u00|^2 and is coarser where that is small)
A defect confined to a subset of sites (a boundary slice, the LDS window, one system of an
interleaved group) shows up as an O(1) error on those sites.
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


FORMATS = {
    # name: (params kwargs, max per-site tolerance, rms tolerance)
    "f64": (dict(mixed=False), 1e-13, 1e-13),
    "f32/f32": (dict(spinor="f32", links="f32"), 1e-6, 1e-6),
    "f32/f16": (dict(spinor="f32", links="f16"), 1e-2, 1e-2),
    "f32/bf16": (dict(spinor="f32", links="bf16"), 2e-2, 2e-2),
    "f16/f32": (dict(spinor="f16", links="f32"), 1e-2, 1e-2),
    "f16/f16": (dict(spinor="f16", links="f16"), 1e-2, 1e-2),
    "f16/bf16": (dict(spinor="f16", links="bf16"), 2e-2, 2e-2),
    "f32/f16r8": (dict(spinor="f32", links="f16", recon=8), 5e-2, 5e-3),
    "f16/f16r8": (dict(spinor="f16", links="f16", recon=8), 5e-2, 5e-3),
}

# per-site agreement between hop variants (multi-RHS against single-system, staged against
# unstaged): they differ only in how the compiler contracts multiply-adds, i.e. in the last bit of
# FP32 intermediates, which can move a value stored in FP16 across one rounding step (2^-10
# relative to the site's scale)
MRHS_VS_SINGLE = {"f32": 1e-5, "f16": 2e-3, "f64": 1e-14}

SHAPES = [
    (8, 8, 8, 8),
    (6, 4, 4, 10),
    (72, 4, 4, 4),    # rows of 36 sites: wider than the LDS halo (x neighbours from memory)
    (64, 4, 2, 4),    # rows of 32 sites: the widest staged halo
    (16, 32, 4, 4),   # a 256-site block is one whole plane: the y wrap stays in the window
    (8, 4, 4, 2),     # T = 2: every site is on a boundary time slice
    (2, 2, 2, 2),     # forward and backward neighbours coincide
]


def reference(U, kappa, psi, dag, anti):
    """FP64 out: even sites M_prec in_e, odd sites the hopping term of in_e."""
    odd = oracle.parity_mask(U.shape[1:5][::-1])
    pe = psi.copy()
    pe[odd] = 0
    ref = oracle.mprec(U, kappa, pe, dag=dag, antiperiodic=anti)
    hop = oracle.hopping(U, pe, dag=dag, antiperiodic=anti)
    ref[odd] = hop[odd]
    return ref, pe, odd


def site_errors(out, ref, odd):
    """(max, rms) per-site error of each parity, relative to the RMS site norm of that parity."""
    res = {}
    for name, m in (("even", ~odd), ("odd", odd)):
        d = np.linalg.norm((out[m] - ref[m]).reshape(-1, 12), axis=1)
        r = np.linalg.norm(ref[m].reshape(-1, 12), axis=1)
        scale = np.sqrt(np.mean(r ** 2))
        res[name] = (float(d.max() / scale), float(np.sqrt(np.mean(d ** 2)) / scale))
    return res


def check(out, ref, odd, fmt, what):
    _, tmax, trms = FORMATS[fmt]
    e = site_errors(out, ref, odd)
    _say(what, fmt, {k: (f"{a:.2e}", f"{b:.2e}") for k, (a, b) in e.items()})
    for k, (emax, erms) in e.items():
        assert emax < tmax, (what, fmt, k, emax)
        assert erms < trms, (what, fmt, k, erms)
    return e


def check_dots(dots, out, pe, odd, red, tol):
    """The fused FP64 sums against the same sums of the returned field (what the kernel stored)
    and of the inputs; the kernel sums the values before they are rounded to the storage format,
    so the agreement is bounded by the format's unit roundoff."""
    ev = ~odd
    o, x = out[ev].reshape(-1), pe[ev].reshape(-1)
    scale = np.linalg.norm(o) * np.linalg.norm(x)
    if red == "zdot":
        ref = np.vdot(x, o)
        assert abs(complex(dots[0], dots[1]) - ref) < tol * scale, (dots, ref)
        assert dots[2] == 0.0
    elif red == "outx":
        ref = np.vdot(o, x)
        assert abs(complex(dots[0], dots[1]) - ref) < tol * scale, (dots, ref)
        assert abs(dots[2] - np.vdot(o, o).real) < tol * np.vdot(o, o).real
    elif red == "norm":
        assert dots[0] == 0.0 and dots[1] == 0.0
        assert abs(dots[2] - np.vdot(o, o).real) < tol * np.vdot(o, o).real
    else:
        assert np.all(dots == 0.0)


@pytest.mark.parametrize("dims", SHAPES)
@pytest.mark.parametrize("fmt", list(FORMATS))
def test_operator_formats(dims, fmt):
    """Every storage format on every lattice shape, with the solvers' default hop variants; the
    reduction kind rotates with the shape so that each format meets each epilogue."""
    red = ["none", "zdot", "outx", "norm"][SHAPES.index(dims) % 4]
    U = li.random_links(dims, 1.0, 1200 + SHAPES.index(dims))
    psi = li.gaussian_field(dims, 2200 + SHAPES.index(dims))
    kappa = 0.125
    g = wd.wd_gauge_create(_t(U))
    out, dots = wd.wd_apply_prec(g, kappa, _t(psi), p=wd.params(**FORMATS[fmt][0]), v=wd.op_variant(red=red))
    out = _n(out)
    ref, pe, odd = reference(U, kappa, psi, False, True)
    check(out, ref, odd, fmt, f"formats {dims} red={red}")
    check_dots(dots[0], out, pe, odd, red, FORMATS[fmt][1])
    g.close()


@pytest.mark.parametrize("dims", [(16, 32, 4, 4), (8, 4, 4, 2), (32, 16, 4, 4)])
@pytest.mark.parametrize("fmt", ["f32/f16", "f16/f16", "f64"])
def test_operator_hop_variants(dims, fmt):
    """Each hop variant the solvers can launch: every reduction, LDS staging on and off,
    non-temporal loads on and off, the adjoint hops, every block order valid on the lattice
    (32 x 16 x 4 x 4 allows t-fastest tiles of 2 and 4 z-planes). A block order changes the
    grouping of the reduction partial sums. Staging and the load policy change only the instruction schedule (and
    with it, in FP32, how multiply-adds are contracted): every variant is checked against the
    oracle and agrees with the others to the last rounding."""
    U = li.random_links(dims, 1.0, 1300)
    psi = li.gaussian_field(dims, 2300)
    kappa = 0.13
    anti = dims != (8, 4, 4, 2)
    g = wd.wd_gauge_create(_t(U), antiperiodic=anti)
    p = wd.params(**FORMATS[fmt][0])
    pd = _t(psi)
    refs = {dag: reference(U, kappa, psi, dag, anti) for dag in (False, True)}
    tol = MRHS_VS_SINGLE["f64" if fmt == "f64" else fmt.split("/")[0]]
    for dag in (False, True):
        for red in ("none", "zdot", "outx", "norm"):
            if dag and red == "outx" or (dag and red == "norm" and fmt != "f64"):
                with pytest.raises(wd.WdError) as e:
                    wd.wd_apply_prec(g, kappa, pd, p=p, v=wd.op_variant(red=red, dagger=True))
                assert e.value.code == 7
                continue
            ref, pe, odd = refs[dag]
            base = None
            for tile in (0, 2, 4):
                for stage in (0, 1):
                    for ntl in (0, 1):
                        v = wd.op_variant(red=red, stage=stage, nontemporal=ntl, tile=tile, dagger=dag, rhs_per_thread=0)
                        out, dots = wd.wd_apply_prec(g, kappa, pd, p=p, v=v)
                        out = _n(out)
                        what = f"variants {dims} dag={dag} red={red} tile={tile} stage={stage} ntl={ntl}"
                        check(out, ref, odd, fmt, what)
                        check_dots(dots[0], out, pe, odd, red, FORMATS[fmt][1])
                        if base is None:
                            base = (out, dots)
                            continue
                        # the variants differ only in scheduling and in the grouping of the
                        # reduction partials: results agree to the last rounding
                        e = site_errors(out, base[0], odd)
                        assert max(e["even"][0], e["odd"][0]) <= tol, (what, e)
                        assert np.allclose(dots, base[1], rtol=tol, atol=tol * np.abs(base[1]).max()), what
    g.close()


@pytest.mark.parametrize("dims", [(8, 4, 4, 2), (6, 4, 4, 10), (8, 8, 8, 8)])
@pytest.mark.parametrize("fmt", ["f32/f16", "f16/bf16", "f32/f32", "f64"])
def test_operator_temporal_gauge(dims, fmt):
    """A temporal-gauge handle: the hop skips the unit time links except on the boundary slices;
    with the source rotated by g(n) and the result by g(n)^dag the operator is the caller's."""
    U = li.random_links(dims, 1.0, 1400)
    psi = li.gaussian_field(dims, 2400)
    kappa = 0.12
    g = wd.wd_gauge_create(_t(U), hint=wd.params(temporal_gauge=True))
    for dag, red in ((False, "outx"), (False, "none"), (True, "zdot")):
        out, dots = wd.wd_apply_prec(g, kappa, _t(psi), p=wd.params(**FORMATS[fmt][0]),
                                     v=wd.op_variant(red=red, dagger=dag))
        ref, pe, odd = reference(U, kappa, psi, dag, True)
        out = _n(out)
        check(out, ref, odd, fmt, f"temporal gauge {dims} dag={dag} red={red}")
        # the sums are taken in the rotated gauge; inner products are invariant under g(n)
        check_dots(dots[0], out, pe, odd, red, max(FORMATS[fmt][1], 1e-12))
    g.close()




@pytest.mark.parametrize("rhs", [0, 2, 4])
@pytest.mark.parametrize("copies", [2, 3, 5])
@pytest.mark.parametrize("fmt", ["f32/f16", "f16/f16", "f32/f16r8", "f32/bf16", "f32/f32", "f16/bf16"])
def test_operator_many_systems_one_launch(copies, fmt, rhs):
    """Several systems on one gauge field in one launch, each with its own source: interleaved block
    pairs (rhs 0) or the multi-RHS hop with up to rhs systems per thread (5 systems make groups of
    4 + 1 and 2 + 2 + 1). Every system matches the oracle. Interleaving changes no arithmetic
    (bitwise equal to the system alone); the multi-RHS hop agrees with it to the last rounding."""
    dims = (16, 8, 8, 8)
    U = li.random_links(dims, 1.0, 1500)
    psis = np.stack([li.gaussian_field(dims, 2500 + k) for k in range(copies)])
    kappa = 0.128
    g = wd.wd_gauge_create(_t(U))
    p = wd.params(**FORMATS[fmt][0])
    for dag, red in ((False, "zdot"), (False, "outx"), (False, "none"), (True, "none"), (True, "zdot")):
        out, dots = wd.wd_apply_prec(g, kappa, _t(psis), p=p,
                                     v=wd.op_variant(red=red, copies=copies, rhs_per_thread=rhs, tile=0, dagger=dag))
        out = _n(out)
        for k in range(copies):
            ref, pe, odd = reference(U, kappa, psis[k], dag, True)
            check(out[k], ref, odd, fmt, f"copy {k}/{copies} rhs={rhs} dag={dag} red={red}")
            alone, dk = wd.wd_apply_prec(g, kappa, _t(psis[k]), p=p,
                                         v=wd.op_variant(red=red, rhs_per_thread=0, tile=0, dagger=dag))
            alone = _n(alone)
            if rhs == 0:
                assert np.array_equal(out[k], alone), (k, copies, red)
                assert np.array_equal(dots[k], dk[0])
            else:
                e = site_errors(out[k], alone, odd)
                tol = MRHS_VS_SINGLE[fmt.split("/")[0]]
                assert max(e["even"][0], e["odd"][0]) < tol, (k, copies, red, e)
                assert np.allclose(dots[k], dk[0], rtol=10 * tol, atol=10 * tol * np.abs(dk).max())
    g.close()


@pytest.mark.parametrize("fmt", ["f32/f16", "f16/f16", "f32/f32"])
def test_operator_multi_rhs_temporal_gauge_and_tiles(fmt):
    """The multi-RHS hop on a temporal-gauge handle (unit time links skipped inside the lattice)
    and in t-fastest block orders, against the oracle."""
    dims = (32, 16, 4, 6)
    U = li.random_links(dims, 1.0, 1510)
    psis = np.stack([li.gaussian_field(dims, 2510 + k) for k in range(3)])
    g = wd.wd_gauge_create(_t(U), hint=wd.params(temporal_gauge=True))
    for tile in (0, 2):
        for rhs in (2, 4):
            out, dots = wd.wd_apply_prec(g, 0.125, _t(psis), p=wd.params(**FORMATS[fmt][0]),
                                         v=wd.op_variant(red="outx", copies=3, rhs_per_thread=rhs, tile=tile))
            out = _n(out)
            for k in range(3):
                ref, pe, odd = reference(U, 0.125, psis[k], False, True)
                check(out[k], ref, odd, fmt, f"temporal gauge multi-RHS tile={tile} rhs={rhs} copy {k}")
                check_dots(dots[k], out[k], pe, odd, "outx", max(FORMATS[fmt][1], 1e-12))
    g.close()


def test_operator_argument_errors():
    dims = (4, 4, 4, 4)
    U = li.random_links(dims, 1.0, 1600)
    g = wd.wd_gauge_create(_t(U))
    psi = _t(li.gaussian_field(dims, 2600))
    with pytest.raises(wd.WdError) as e:
        wd.wd_apply_prec(g, -0.1, psi)
    assert e.value.code == 1
    with pytest.raises(wd.WdError) as e:
        wd.wd_apply_prec(g, 0.1, psi, v=wd.op_variant(rhs_per_thread=9))
    assert e.value.code == 1
    with pytest.raises(wd.WdError) as e:  # the multi-RHS hop has no FP64 form
        wd.wd_apply_prec(g, 0.1, psi, p=wd.params(mixed=False), v=wd.op_variant(rhs_per_thread=2))
    assert e.value.code == 7
    with pytest.raises(wd.WdError) as e:  # out and in overlap
        wd.wd_apply_prec(g, 0.1, psi, out=psi)
    assert e.value.code == 1
    g.close()
    # the 8-real format refuses unit links (row 1 cannot be rebuilt), 12-real refuses non-SU(3) links
    unit = np.zeros((4,) + dims[::-1] + (3, 3), dtype=np.complex128)
    unit[..., 0, 0] = unit[..., 1, 1] = unit[..., 2, 2] = 1.0
    g = wd.wd_gauge_create(_t(unit))
    with pytest.raises(wd.WdError) as e:
        wd.wd_apply_prec(g, 0.1, psi, p=wd.params(recon=8))
    assert e.value.code == 7
    g.close()
    g = wd.wd_gauge_create(_t(U * 1.05))
    with pytest.raises(wd.WdError) as e:
        wd.wd_apply_prec(g, 0.1, psi)
    assert e.value.code == 7
    out, _ = wd.wd_apply_prec(g, 0.1, psi, p=wd.params(mixed=False))  # 18-real FP64 operator
    ref, pe, odd = reference(U * 1.05, 0.1, _n(psi), False, True)
    check(_n(out), ref, odd, "f64", "non-SU(3) links, 18 reals")
    g.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 4, 10), (8, 4, 4, 2), (16, 32, 4, 4)])
@pytest.mark.parametrize("fmt", ["f64", "f32/f32", "f32/f16", "f16/f16", "f32/bf16", "f32/f16r8"])
def test_operator_nonchiral_basis(dims, fmt):
    """A handle in the non-chiral basis (gamma_4 diagonal: the time hops read two spin components
    of each neighbour): every reduction, the adjoint hops, with and without LDS staging, against
    the oracle's operator in the paper's chiral basis (the call rotates in and out)."""
    U = li.random_links(dims, 1.0, 1800)
    psi = li.gaussian_field(dims, 2800)
    kappa = 0.127
    g = wd.wd_gauge_create(_t(U), hint=wd.params(nonchiral=True))
    p = wd.params(**FORMATS[fmt][0])
    for dag, red in ((False, "zdot"), (False, "outx"), (False, "none"), (True, "none"), (True, "zdot")):
        for stage in (0, 1):
            out, dots = wd.wd_apply_prec(g, kappa, _t(psi), p=p, v=wd.op_variant(red=red, dagger=dag, stage=stage))
            out = _n(out)
            ref, pe, odd = reference(U, kappa, psi, dag, True)
            check(out, ref, odd, fmt, f"non-chiral {dims} dag={dag} red={red} stage={stage}")
            check_dots(dots[0], out, pe, odd, red, max(FORMATS[fmt][1], 1e-12))
    g.close()


@pytest.mark.parametrize("fmt", ["f32/f16", "f16/f16", "f32/f32"])
def test_operator_nonchiral_multi_rhs_and_temporal_gauge(fmt):
    """The non-chiral time hop inside the multi-RHS hop, and combined with the temporal gauge (unit
    time links skipped on the interior slices)."""
    dims = (16, 8, 8, 6)
    U = li.random_links(dims, 1.0, 1810)
    psis = np.stack([li.gaussian_field(dims, 2810 + k) for k in range(3)])
    for tg in (False, True):
        g = wd.wd_gauge_create(_t(U), hint=wd.params(nonchiral=True, temporal_gauge=tg))
        for rhs in (0, 2, 4):
            for dag, red in ((False, "outx"), (True, "zdot")):
                out, dots = wd.wd_apply_prec(g, 0.125, _t(psis), p=wd.params(**FORMATS[fmt][0]),
                                             v=wd.op_variant(red=red, copies=3, rhs_per_thread=rhs, dagger=dag))
                out = _n(out)
                for k in range(3):
                    ref, pe, odd = reference(U, 0.125, psis[k], dag, True)
                    check(out[k], ref, odd, fmt, f"non-chiral tg={tg} rhs={rhs} dag={dag} copy {k}")
                    check_dots(dots[k], out[k], pe, odd, red, max(FORMATS[fmt][1], 1e-12))
        g.close()
