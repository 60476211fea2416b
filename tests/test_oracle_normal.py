"""Pins of the oracle's CG and CG-M on the shifted even-site normal equations
(M_prec^dag M_prec + sigma) x = b_e (Sec. 8 names CG / CG-M as the next Krylov pair; the shifted
family shares one Krylov space, Sec. 6.1).

The pins do not reuse the oracle's adjoint: the dense matrix of M_prec is built column by column
from the forward operator and its conjugate transpose goes to LAPACK; the adjoint identity and
positivity are checked on random fields; CG-M is checked against LAPACK and against independent
single-shift CG runs.
"""
import numpy as np
import pytest

import lattice_inputs as li
import oracle


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _even_index(dims):
    odd = oracle.parity_mask(dims)
    X, Y, Z, T = dims
    sites = np.flatnonzero(~odd.ravel())
    return np.concatenate([s * 12 + np.arange(12) for s in sites])


def _dense_mprec_even(U, kappa, dims):
    """M_prec restricted to the even sites, from the forward operator only."""
    X, Y, Z, T = dims
    idx = _even_index(dims)
    n = X * Y * Z * T * 12
    cols = []
    e = np.zeros(n, dtype=np.complex128)
    for j in idx:
        e[:] = 0
        e[j] = 1
        cols.append(oracle.mprec(U, kappa, e.reshape(T, Z, Y, X, 3, 4)).ravel()[idx])
    return np.stack(cols, axis=1), idx


def test_mprec_adjoint_identity_and_positivity():
    dims = (4, 4, 2, 4)
    U = li.random_links(dims, 1.0, 1201)
    kappa = 0.126
    u = oracle.even_part(li.gaussian_field(dims, 11))
    v = oracle.even_part(li.gaussian_field(dims, 12))
    lhs = np.vdot(u.ravel(), oracle.mprec(U, kappa, v).ravel())
    rhs = np.vdot(oracle.mprec(U, kappa, u, dag=True).ravel(), v.ravel())
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    sigma = 0.3
    Av = oracle.normal_apply(U, kappa, sigma, v)
    q = np.vdot(v.ravel(), Av.ravel())
    mv = oracle.mprec(U, kappa, v)
    expect = np.vdot(mv.ravel(), mv.ravel()).real + sigma * np.vdot(v.ravel(), v.ravel()).real
    assert abs(q.imag) < 1e-12 * q.real and abs(q.real - expect) < 1e-12 * expect
    assert np.abs(Av[oracle.parity_mask(dims)]).max() == 0.0


@pytest.mark.parametrize("sigmas", [(0.0, 5.0, 40.0, 300.0), (1.0, 1.1)])
def test_cg_and_cg_m_vs_lapack_2444(sigmas):
    """2^4 lattice (forward and backward neighbours coincide): CG and CG-M vs LAPACK on the dense
    conjugate-transpose product."""
    dims = (2, 2, 2, 2)
    U = li.random_links(dims, 1.0, 1202)
    b = li.gaussian_field(dims, 2202)
    kappa = 0.128
    Md, idx = _dense_mprec_even(U, kappa, dims)
    be = b.ravel()[idx]
    xs_m, it_m, st_m, conv = oracle.cg_m(U, kappa, sigmas, b, tol=1e-13)
    assert st_m == oracle.STATUS_OK
    for s, xm in zip(sigmas, xs_m):
        A = Md.conj().T @ Md + s * np.eye(len(idx))
        x_lu = np.linalg.solve(A, be)
        x, it, st, _ = oracle.cg(U, kappa, s, b, tol=1e-13)
        assert st == oracle.STATUS_OK
        assert _rel(x.ravel()[idx], x_lu) < 1e-10
        assert _rel(xm.ravel()[idx], x_lu) < 1e-10
        assert np.abs(xm[oracle.parity_mask(dims)]).max() == 0.0


def test_cg_m_against_single_shift_cg_4444():
    """Every CG-M solution equals a separate CG solve; its true residual meets the tolerance;
    larger shifts converge (freeze) no later than the base; CG-M takes the base's iterations."""
    dims = (4, 4, 4, 4)
    U = li.random_links(dims, 1.0, 1203)
    b = li.gaussian_field(dims, 2203)
    kappa = 0.13
    sigmas = [400.0, 0.0, 100.0, 20.0]  # the spectrum of M_prec^dag M_prec is ~ (1/(2 kappa))^4
    tol = 1e-10
    xs, it, st, conv = oracle.cg_m(U, kappa, sigmas, b, tol=tol)
    assert st == oracle.STATUS_OK
    be = oracle.even_part(b)
    its = []
    for s, x, c in zip(sigmas, xs, conv):
        xc, itc, stc, _ = oracle.cg(U, kappa, s, b, tol=tol)
        assert stc == oracle.STATUS_OK
        its.append(itc)
        r = be - oracle.normal_apply(U, kappa, s, x)
        assert np.linalg.norm(r) / np.linalg.norm(be) < 5 * tol
        assert _rel(x, xc) < 1e-7
        assert c <= it
    assert it == its[1]  # the base (smallest shift) is the single-shift CG run itself
    assert conv[0] <= conv[2] <= conv[3] <= conv[1] and conv[0] < conv[1]


def test_cg_start_vector_and_zero_source():
    dims = (4, 4, 2, 4)
    U = li.random_links(dims, 1.0, 1204)
    b = li.gaussian_field(dims, 2204)
    kappa, sigma = 0.125, 0.05
    x, it, st, _ = oracle.cg(U, kappa, sigma, b, tol=1e-12)
    # started at the solution: no iteration
    x2, it2, st2, _ = oracle.cg(U, kappa, sigma, b, tol=1e-10, x0=x)
    assert st2 == oracle.STATUS_OK and it2 == 0
    z, itz, stz, _ = oracle.cg(U, kappa, sigma, np.zeros_like(b))
    assert stz == oracle.STATUS_OK and itz == 0 and np.abs(z).max() == 0.0


def test_normal_sequential_with_guess():
    """Largest shift first with the Lagrange guess in sigma: same solutions as zero start vectors,
    fewer iterations in total."""
    dims = (4, 4, 4, 4)
    U = li.random_links(dims, 1.0, 1205)
    b = li.gaussian_field(dims, 2205)
    kappa = 0.128
    sigmas = [0.0, 25.0, 50.0, 100.0, 200.0]
    tol = 1e-10
    xg, itg = oracle.normal_sequential(U, kappa, sigmas, b, tol=tol, guess="poly")
    xn, itn = oracle.normal_sequential(U, kappa, sigmas, b, tol=tol, guess="none")
    be = oracle.even_part(b)
    for s, a, c in zip(sigmas, xg, xn):
        r = be - oracle.normal_apply(U, kappa, s, a)
        assert np.linalg.norm(r) / np.linalg.norm(be) < 5 * tol
        assert _rel(a, c) < 1e-7
    assert sum(itg) < sum(itn)
    assert itg[4] == itn[4]  # the first (largest) shift has no earlier solution
