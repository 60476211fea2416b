"""wd_apply_noalloc, the operator application for callers that cannot allocate, against wd_apply.

The two run the same kernels with the same launch configuration, so the results must be bitwise
equal; the allocation-free entry point keeps its packed fields and job table in the library's
fixed per-GPU array, which holds the previous call's contents: two calls in a row, the second on a
smaller lattice, must each give wd_apply's result. Free device memory must not change across
calls once each kind of call has run (the library makes no allocation), and a lattice too large
for the array is refused.
"""
import numpy as np
import pytest
import torch

import lattice_inputs as li
import paper_1103_5103_amd as wd

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def test_noalloc_matches_wd_apply_on_consecutive_calls():
    cases = [((16, 16, 16, 32), 1.0, 0.125, True),   # 65,536 sites per parity: fills most of the array
             ((8, 4, 6, 4), 1.0, 0.13, False)]       # smaller, periodic in time
    gauges, psis, refs, outs = [], [], [], []
    for k, (dims, eps, kappa, anti) in enumerate(cases):
        print("case", dims, flush=True)
        U = li.random_links(dims, eps, 1700 + k)
        psi = _t(li.gaussian_field(dims, 2700 + k))
        g_ref = wd.wd_gauge_create(_t(U), antiperiodic=anti)
        refs.append((wd.wd_apply(g_ref, kappa, psi).clone(), wd.wd_apply_dag(g_ref, kappa, psi).clone()))
        g_ref.close()
        gauges.append((wd.wd_gauge_create(_t(U), antiperiodic=anti), kappa))
        psis.append(psi)
        outs.append((torch.empty_like(psi), torch.empty_like(psi)))
    torch.cuda.synchronize()
    def one_pass(rep):
        for (g, kappa), psi, (o, od), (r, rd) in zip(gauges, psis, outs, refs):
            o.zero_()
            od.zero_()
            wd.wd_apply_noalloc(g, kappa, psi, o)             # the big lattice, then the smaller one
            wd.wd_apply_noalloc(g, kappa, psi, od, dagger=True)
            torch.cuda.synchronize()
            assert torch.equal(o, r), rep
            assert torch.equal(od, rd), rep

    # the first pass also warms up: the library looks up the array's address on the device's first
    # call, and the runtime loads a kernel's code (torch's fill and compare kernels included) and
    # reserves its private memory when it first launches it. Later passes may not change the free
    # device memory.
    one_pass(0)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    one_pass(1)
    one_pass(2)
    assert torch.cuda.mem_get_info()[0] == free0
    for g, _ in gauges:
        g.close()


def test_noalloc_refuses_lattices_larger_than_its_array():
    dims = (16, 16, 16, 48)  # 98,304 sites per parity
    U = li.random_links(dims, 1.0, 1710)
    g = wd.wd_gauge_create(_t(U))
    psi = _t(li.gaussian_field(dims, 2710))
    with pytest.raises(wd.WdError) as e:
        wd.wd_apply_noalloc(g, 0.12, psi, torch.empty_like(psi))
    assert e.value.code == 1
    with pytest.raises(wd.WdError) as e:
        wd.wd_apply_noalloc(g, 0.12, psi, psi)
    assert e.value.code == 1
    g.close()
