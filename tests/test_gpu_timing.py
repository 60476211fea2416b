"""Per-launch kernel timing (wd_timing_*), the measurement behind the benchmark's roofline figure.

On one sequential mixed-precision multi-mass solve (16^4, FP32 spinors, FP16 12-real links, non-chiral
basis): every class that the solve launches is counted; the low-precision hops split exactly into
their fused-reduction classes; each counted launch carries the algorithmic bytes of its variant
(input and output spinor, 8 links, and one more spinor per epilogue field read); the launches of one
stream do not overlap, so the bracketed durations add up to less than the solve's wall time; and
nothing is counted while timing is off.
"""
import time

import pytest
import torch

import lattice_inputs as li
import paper_1103_5103_amd as wd

pytestmark = pytest.mark.gpu
DIMS = (16, 16, 16, 16)
VH = 16 ** 4 // 2
SPINOR_F32 = 96  # bytes per site
LINKS_F16_12 = 8 * 24  # 8 links of 12 FP16 reals per site


def _solve(g, b, p):
    return wd.wd_multimass_solve(g, [0.120, 0.124], b, method=wd.WD_METHOD_SEQUENTIAL, p=p)


def _classes():
    return [wd.timing_get(c) for c in range(8)]


def test_timing_classes_of_a_solve():
    U = torch.from_numpy(li.random_links(DIMS, 1.0, 1011)).cuda()
    b = torch.from_numpy(li.gaussian_field(DIMS, 2011)).cuda()
    g = wd.wd_gauge_create(U, hint=wd.params(nonchiral=True))
    p = wd.params(tol=1e-8, spinor="f32", links="f16", delta=1e-3)
    try:
        _solve(g, b, p)  # tuning and workspaces outside the measured solve
        torch.cuda.synchronize()
        wd.timing_reset()
        wd.timing_enable(True)
        t0 = time.perf_counter()
        _, sts = _solve(g, b, p)
        torch.cuda.synchronize()
        wall_ms = (time.perf_counter() - t0) * 1e3
        r = _classes()
        wd.timing_enable(False)
        print("classes", r, "wall ms", wall_ms, flush=True)
        assert all(s["status"] == 0 for s in sts)

        for c in range(4):  # lo hop, FP64 hop, sweeps, finishers
            ms, n, by = r[c]
            assert n > 0 and ms > 0.0, (c, r[c])
        assert r[3][2] == 0.0  # finishers move no field data
        # the reduction classes partition the low-precision hops
        assert sum(r[c][1] for c in range(4, 8)) == r[0][1]
        assert sum(r[c][0] for c in range(4, 8)) == pytest.approx(r[0][0], rel=1e-9)
        assert sum(r[c][2] for c in range(4, 8)) == pytest.approx(r[0][2], rel=1e-12)
        # algorithmic bytes per launch: plain hop, <z, out> (reads x0 and z), <out, x0> and |out|^2 (reads x0)
        for c, extra in ((4, 0), (5, 2), (6, 1)):
            ms, n, by = r[c]
            assert n > 0, c
            assert by / n == (2 + extra) * SPINOR_F32 * VH + LINKS_F16_12 * VH, (c, by / n)
        # one stream: the bracketed launches are disjoint intervals inside the wall time
        assert sum(r[c][0] for c in range(4)) <= wall_ms

        wd.timing_reset()
        _solve(g, b, p)
        torch.cuda.synchronize()
        assert all(n == 0 for _, n, _ in _classes())
    finally:
        wd.timing_enable(False)
        g.close()


def test_multishift_fp64_hop_bytes():
    """BiCGstab-M (FP64, full lattice, 12-real FP64 links for SU(3) input): per iteration one hop
    with <rhat, As> (reads the input, s and rhat: 4 spinors + 8 links per site) and one with
    <Aw, w>, |Aw|^2 (3 spinors + 8 links); at the end one launch forms every mass's true residual
    (reads x, b and the input: 4 spinors + 8 links per site and mass). Gated launches after
    convergence are not counted."""
    U = torch.from_numpy(li.random_links(DIMS, 1.0, 1012)).cuda()
    b = torch.from_numpy(li.gaussian_field(DIMS, 2012)).cuda()
    g = wd.wd_gauge_create(U)
    p = wd.params(tol=1e-8, mixed=False, eo=False)
    kappas = [0.120, 0.124]
    try:
        wd.bicgstab_m_solve(g, kappas, b, p=p)
        torch.cuda.synchronize()
        wd.timing_reset()
        wd.timing_enable(True)
        _, sts = wd.bicgstab_m_solve(g, kappas, b, p=p)
        torch.cuda.synchronize()
        ms, n, by = wd.timing_get(1)
        wd.timing_enable(False)
        iters = max(s["iters"] for s in sts)
        print("fp64 hop class", ms, n, by, "iterations", iters, flush=True)
        V = 2 * VH
        spinor64, links64 = 192, 8 * 96
        assert n == 2 * iters + 1
        assert by == iters * V * ((4 * spinor64 + links64) + (3 * spinor64 + links64)) + len(kappas) * V * (
            4 * spinor64 + links64)
    finally:
        wd.timing_enable(False)
        g.close()
