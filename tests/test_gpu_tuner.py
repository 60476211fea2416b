"""The hop tuner's choice cache ($WD_TUNE_CACHE): entries that are not candidates of their
configuration (a stale or hand-edited file) are ignored and the configuration is tuned again.

The cache file is read once per process, so the case runs in a child process of its own with
the variable set; the child solves four systems sharing one 8^4 gauge field (the tuner's
multi-system candidates), checks them with the oracle and prints the result.
"""
import os
import subprocess
import sys

import pytest
import torch

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import numpy as np, torch
import lattice_inputs as li, oracle
import paper_1103_5103_amd as wd
dims = (8, 8, 8, 8)
U = li.random_links(dims, 1.0, 1007)
g = wd.wd_gauge_create(torch.from_numpy(U).cuda(), hint=wd.params())
bs = [li.gaussian_field(dims, 2600 + k) for k in range(4)]
xs = [torch.zeros(g.field_shape, dtype=torch.complex128, device="cuda") for _ in bs]
systems = [(g, 0.124, torch.from_numpy(b).cuda(), x) for b, x in zip(bs, xs)]
sts = wd.wd_batch_solve(systems, p=wd.params(tol=1e-8, spinor="f32", links="f16"))
worst = max(oracle.true_residual(U, 0.124, x.cpu().numpy(), b) for x, b in zip(xs, bs))
print("statuses", [s["status"] for s in sts], "worst", worst, flush=True)
g.close()
"""


def test_invalid_cache_entry_is_retuned(tmp_path):
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    key = f"{arch}|8x8x8x8|sf1|lf3|tg0|n4"
    cache = tmp_path / "hop_tune.txt"
    cache.write_text(f"{key} 3 7\n")  # tz = 3 and 7 systems per thread are no candidates
    env = dict(os.environ, WD_TUNE_CACHE=str(cache))
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], env=env, capture_output=True, text=True,
                       timeout=240)
    print(r.stdout, r.stderr[-2000:], flush=True)
    assert r.returncode == 0
    line = [l for l in r.stdout.splitlines() if l.startswith("statuses")][0]
    assert "[0, 0, 0, 0]" in line
    assert float(line.split()[-1]) < 1e-8
    entries = [l.split() for l in cache.read_text().splitlines() if l.startswith(key)]
    # the invalid entry, then the tuned one, which is a candidate: tile order 0 (no tile divides
    # this lattice) and 0, 2 or 4 systems per thread
    assert len(entries) == 2, entries
    tz, rhs = int(entries[1][1]), int(entries[1][2])
    assert tz == 0 and rhs in (0, 2, 4)
