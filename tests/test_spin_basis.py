"""CPU check of the non-chiral spin basis the solvers may work in (a bandwidth cut Sec. 4 names).

Spinor fields are 3 x 4 colour-by-spin matrices with the spin matrices acting from the right
(Sec. 2, eq. 4), so with psi' = psi S an operator psi -> psi G becomes psi' -> psi' S^dag G S. For
the rotation the library uses, S = [[1, 1], [-1, 1]] / sqrt(2) in 2 x 2 spin blocks, this pins
against the oracle's gamma matrices (themselves pinned to Table 1): the spatial gammas are
unchanged, gamma_4 becomes diag(1, 1, -1, -1), so the time projectors keep two spin components,
and gamma_5 becomes off-diagonal (the adjoint solves apply it before the rotation).
"""
import numpy as np

import oracle

R = 1 / np.sqrt(2)
# psi'_j = sum_i psi_i S_ij: psi'_0 = (psi_0 - psi_2) / sqrt 2, psi'_2 = (psi_0 + psi_2) / sqrt 2, and
# the same for spins 1 and 3
S = R * np.array([[1, 0, 1, 0],
                  [0, 1, 0, 1],
                  [-1, 0, 1, 0],
                  [0, -1, 0, 1]], dtype=np.complex128)


def rotate(g):
    return S.conj().T @ g @ S


def test_rotation_is_unitary():
    assert np.allclose(S.conj().T @ S, np.eye(4), atol=1e-15)


def test_spatial_gammas_unchanged():
    for mu in range(3):
        assert np.allclose(rotate(oracle.gamma(mu)), oracle.gamma(mu), atol=1e-15), mu


def test_gamma4_diagonal_and_time_projectors():
    g4 = rotate(oracle.gamma(3))
    assert np.allclose(g4, np.diag([1, 1, -1, -1]), atol=1e-15)
    # 1 - gamma_4 keeps spins 2, 3 and 1 + gamma_4 spins 0, 1, each times 2
    assert np.allclose(np.eye(4) - g4, np.diag([0, 0, 2, 2]), atol=1e-15)
    assert np.allclose(np.eye(4) + g4, np.diag([2, 2, 0, 0]), atol=1e-15)


def test_gamma5_off_diagonal():
    g5 = oracle.gamma(0) @ oracle.gamma(1) @ oracle.gamma(2) @ oracle.gamma(3)
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)  # chiral basis: diagonal
    g5r = rotate(g5)
    assert np.allclose(np.diag(np.diag(g5r)), 0, atol=1e-15)
    assert np.allclose(g5r @ g5r, np.eye(4), atol=1e-15)


def test_operator_on_a_field_commutes_with_the_rotation():
    # one site's spin part of a hop, psi -> psi (1 - gamma_mu), in either basis
    rng = np.random.default_rng(5)
    psi = rng.normal(size=(3, 4)) + 1j * rng.normal(size=(3, 4))
    for mu in range(4):
        p = np.eye(4) - oracle.gamma(mu)
        assert np.allclose((psi @ p) @ S, (psi @ S) @ rotate(p), atol=1e-14), mu
