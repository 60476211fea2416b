"""CPU pins of the compressed SU(3) link formats' reconstruction equations (no GPU).

The 12-real formats store rows 0 and 1 and rebuild row 2 = conj(row0 x row1); the 8-real format
stores u01, u02, u10 and the phases of u00 and u20, and rebuilds the rest from unitarity and
det U = 1 (U^-1 = U^dag is the adjugate): |u00|^2 = 1 - |u01|^2 - |u02|^2, |u20|^2 = 1 - |u00|^2 -
|u10|^2, and row 1 solves <row1, row0> = 0 together with conj(u20) = u01 u12 - u02 u11. Here the
equations are solved plainly (a 2 x 2 linear solve) on random SU(3) matrices from the input
generator and must give back the matrix to rounding; the GPU kernels that implement them in
closed form are checked site by site against the oracle's operator in the GPU tests.
"""
import numpy as np

import lattice_inputs as li


def su3_samples(n=400, seed=11):
    rng = np.random.default_rng(seed)
    return np.concatenate([li.random_su3(rng, n // 2, 1.0), li.random_su3(rng, n // 2, 0.3)])


def test_samples_are_su3():
    U = su3_samples()
    eye = np.eye(3)
    assert np.allclose(U @ np.conj(np.swapaxes(U, -1, -2)), eye, atol=1e-13)
    assert np.allclose(np.linalg.det(U), 1.0, atol=1e-13)


def test_row2_from_rows_0_and_1():
    for u in su3_samples():
        r2 = np.conj(np.cross(u[0], u[1]))
        assert np.allclose(r2, u[2], atol=1e-13)


def rebuild8(u01, u02, u10, ph00, ph20):
    """The 8-parameter reconstruction written out from the equations above."""
    n = abs(u01) ** 2 + abs(u02) ** 2
    u00 = np.sqrt(max(1 - n, 0.0)) * np.exp(1j * ph00)
    u20 = np.sqrt(max(n - abs(u10) ** 2, 0.0)) * np.exp(1j * ph20)
    # unknowns (u11, u12): conj(u01) u11 + conj(u02) u12 = -u10 conj(u00);  -u02 u11 + u01 u12 = conj(u20)
    A = np.array([[np.conj(u01), np.conj(u02)], [-u02, u01]])
    rhs = np.array([-u10 * np.conj(u00), np.conj(u20)])
    u11, u12 = np.linalg.solve(A, rhs)
    r0 = np.array([u00, u01, u02])
    r1 = np.array([u10, u11, u12])
    return np.array([r0, r1, np.conj(np.cross(r0, r1))])


def test_8real_reconstruction():
    worst = 0.0
    for u in su3_samples():
        if 1 - abs(u[0, 0]) ** 2 < 1e-6:
            continue  # the format refuses such links: row 1 is not determined there
        w = rebuild8(u[0, 1], u[0, 2], u[1, 0], np.angle(u[0, 0]), np.angle(u[2, 0]))
        worst = max(worst, np.abs(w - u).max())
    assert worst < 1e-10, worst


def test_8real_system_determinant():
    # the 2 x 2 system's determinant is |u01|^2 + |u02|^2 = 1 - |u00|^2
    for u in su3_samples(40):
        A = np.array([[np.conj(u[0, 1]), np.conj(u[0, 2])], [-u[0, 2], u[0, 1]]])
        assert np.isclose(np.linalg.det(A), 1 - abs(u[0, 0]) ** 2, atol=1e-13)
