"""CPU checks of the library's lattice index map and FP16 site scale (no GPU).

The hop kernels address sites through cb_coords / cb_index / nb_index and store FP16 spinors with
the scale rule f16_site_inv, all host-callable functions of wd_device.hpp. tests/index_map_probe.cpp
is built for the host with hipcc and prints them; they are checked here against the plain
definitions: the checkerboard index of parity p enumerates exactly the sites with
(x + y + z + t) mod 2 = p (the oracle's parity), every neighbour index is the periodic
lexicographic neighbour of Sec. 2, eq. 3, and the FP16 scale never turns a finite site into NaN.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PROBE = os.path.join(ROOT, "tests", "index_map_probe.cpp")
CSRC = os.path.join(ROOT, "paper_1103_5103_amd", "csrc")


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    if shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("probe") / "index_map_probe")
    subprocess.run(["hipcc", "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-I", CSRC, PROBE, "-o", exe],
                   check=True, capture_output=True)
    return exe


def run(exe, dims):
    out = subprocess.run([exe, *map(str, dims)], capture_output=True, text=True, check=True).stdout
    sites = np.array([[int(v) for v in l.split()[1:]] for l in out.splitlines() if l.startswith("S ")])
    scale = [(float(l.split()[1]), float(l.split()[2])) for l in out.splitlines() if l.startswith("F ")]
    return sites, scale


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4), (6, 4, 2, 10), (8, 4, 6, 2), (72, 4, 4, 4)])
def test_checkerboard_map_and_neighbours(probe, dims):
    X, Y, Z, T = dims
    V = X * Y * Z * T
    sites, _ = run(probe, dims)
    assert sites.shape == (V, 12)
    par, cb, n, cb_back = sites[:, 0], sites[:, 1], sites[:, 2], sites[:, 3]
    # bijection: every lexicographic site appears once, with its own parity
    assert sorted(n.tolist()) == list(range(V))
    dims_c = (np.ctypeslib.as_ctypes(np.array(dims, dtype=np.int32)))
    for p_, n_ in zip(par[:: max(1, V // 500)], n[:: max(1, V // 500)]):
        assert oracle.lib().oracle_parity(dims_c, int(n_)) == p_
    x, y, z, t = n % X, (n // X) % Y, (n // (X * Y)) % Z, n // (X * Y * Z)
    assert np.array_equal((x + y + z + t) % 2, par)
    assert np.array_equal(cb_back, cb)
    # the other parity's map from checkerboard index to lexicographic site
    lex = {q: np.empty(V // 2, dtype=np.int64) for q in (0, 1)}
    for q in (0, 1):
        m = par == q
        lex[q][cb[m]] = n[m]
    coords = np.stack([x, y, z, t])
    L = np.array(dims)[:, None]
    for mu in range(4):
        for d, step in ((0, 1), (1, -1)):
            c = coords.copy()
            c[mu] = (c[mu] + step) % L[mu, 0]
            want = c[0] + X * (c[1] + Y * (c[2] + Z * c[3]))
            got = np.array([lex[1 - p_][k] for p_, k in zip(par, sites[:, 4 + 2 * mu + d])])
            assert np.array_equal(got, want), (dims, mu, d)


def test_fp16_site_scale(probe):
    _, scale = run(probe, (2, 2, 2, 2))
    tiny = np.finfo(np.float32).tiny
    for m, inv in scale:
        if np.isfinite(m) and m >= tiny:
            assert inv > 0 and np.isfinite(inv) and abs(m * inv - 1.0) < 1e-6, (m, inv)
        else:
            # zero, subnormal, infinite or NaN maxima: no finite site value may become 0 * inf
            assert inv == 0.0, (m, inv)


def test_random_shapes(probe):
    """The same map checks on seeded random even shapes (rows from 1 to 40 checkerboard sites)."""
    rng = np.random.default_rng(7)
    for _ in range(6):
        dims = tuple(int(2 * rng.integers(1, 5)) for _ in range(3)) + (int(2 * rng.integers(1, 4)),)
        dims = (int(2 * rng.integers(1, 41)),) + dims[1:]
        test_checkerboard_map_and_neighbours(probe, dims)
