"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

Each test ties an oracle function to something other than the oracle itself: the printed
Table 1, closed forms (free-field spectrum), symmetries (gamma5-hermiticity, gauge
covariance), LAPACK on a dense matrix, and finite differences. Chosen so that a plausible
mistake (a wrong projector sign, a link taken at the wrong site, a missing dagger, a dropped
boundary sign, a wrong diagonal, a wrong shift recurrence) fails at least one of them.
"""
import os

import numpy as np
import pytest

import lattice_inputs as li
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
G5 = np.diag([1, 1, -1, -1]).astype(np.complex128)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


# ------------------------------------------------------------------ gamma matrices, Table 1

def _table1():
    rows = []
    with open(os.path.join(GOLDEN, "table1_projector_vectors.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, v1, v2 = line.split("|")
            name, mu, sign = head.split()
            rows.append((int(mu) - 1, sign, np.array([complex(t) for t in v1.split()]),
                         np.array([complex(t) for t in v2.split()])))
    return rows


def test_table1_projectors_match_gammas():
    """(1 -/+ gamma_mu) = v1 v1^dag + v2 v2^dag for all eight rows of Table 1."""
    rows = _table1()
    assert len(rows) == 8
    for mu, sign, v1d, v2d in rows:
        v1, v2 = np.conj(v1d)[:, None], np.conj(v2d)[:, None]
        proj = v1 @ v1d[None, :] + v2 @ v2d[None, :]
        P = np.eye(4) - oracle.gamma(mu) if sign == "+" else np.eye(4) + oracle.gamma(mu)
        assert np.abs(proj - P).max() == 0.0


def test_gamma_algebra():
    g = [oracle.gamma(m) for m in range(4)]
    for m in range(4):
        assert np.abs(g[m] - g[m].conj().T).max() == 0.0  # Hermitian
        for n in range(4):
            anti = g[m] @ g[n] + g[n] @ g[m]
            assert np.abs(anti - 2.0 * (m == n) * np.eye(4)).max() == 0.0
    # gamma5 = gamma1 gamma2 gamma3 gamma4 is diagonal in the chiral basis
    assert np.abs(g[0] @ g[1] @ g[2] @ g[3] - G5).max() == 0.0


# ------------------------------------------------------------------ inputs

def test_link_generator_is_su3():
    U = li.random_links((4, 2, 2, 4), 1.0, 1234).reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.abs(np.einsum("nab,ncb->nac", U, U.conj()) - eye).max() < 1e-13
    assert np.abs(np.linalg.det(U) - 1.0).max() < 1e-13


# ------------------------------------------------------------------ operator

@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 2, 2, 2), (4, 2, 6, 4)])
def test_gamma5_hermiticity_and_adjoint(dims):
    U = li.random_links(dims, 1.0, 1000)
    kappa = 0.125
    p = li.gaussian_field(dims, 5)
    q = li.gaussian_field(dims, 6)
    Mq = oracle.apply(U, kappa, q)
    Mdp = oracle.apply(U, kappa, p, dag=True)
    # <p, M q> = <M^dag p, q>
    assert abs(np.vdot(p, Mq) - np.vdot(Mdp, q)) < 1e-12 * np.linalg.norm(p) * np.linalg.norm(Mq)
    # M^dag = gamma5 M gamma5 (gamma5 acts on the spin index from the right)
    assert _rel(oracle.apply(U, kappa, q, dag=True), oracle.apply(U, kappa, q @ G5) @ G5) < 1e-14


@pytest.mark.parametrize("antiperiodic", [True, False])
def test_gauge_covariance(antiperiodic):
    """M[U^g](g psi) = g M[U] psi with U^g_mu(n) = g(n) U_mu(n) g(n+mu)^dag."""
    dims = (4, 4, 2, 6)
    X, Y, Z, T = dims
    U = li.random_links(dims, 1.0, 1001)
    g = li.random_gauge_transform(dims, 77)
    psi = li.gaussian_field(dims, 8)
    Ug = np.empty_like(U)
    for mu in range(4):
        gs = np.roll(g, -1, axis=3 - mu)  # g(n + mu); axes (t, z, y, x)
        Ug[mu] = np.einsum("...ab,...bc,...dc->...ad", g, U[mu], gs.conj())
    lhs = oracle.apply(Ug, 0.13, np.einsum("...ab,...bs->...as", g, psi), antiperiodic=antiperiodic)
    rhs = np.einsum("...ab,...bs->...as", g, oracle.apply(U, 0.13, psi, antiperiodic=antiperiodic))
    assert _rel(lhs, rhs) < 1e-14


@pytest.mark.parametrize("dims,antiperiodic", [((4, 4, 4, 8), True), ((6, 4, 2, 4), True), ((4, 4, 4, 4), False)])
def test_free_field_plane_waves(dims, antiperiodic):
    """U = 1: a plane wave e^{ip.n} u is mapped to e^{ip.n} u K with
    K = W + i sum_mu sin(p_mu) gamma_mu, W = m a + sum_mu (1 - cos p_mu); the eigenvalues of K are
    W +- i sqrt(sum sin^2 p). Antiperiodic time shifts p_4 to pi (2k+1)/T."""
    X, Y, Z, T = dims
    U = li.unit_links(dims)
    kappa = 0.11
    ma = 1.0 / (2 * kappa) - 4.0
    rng = np.random.default_rng(3)
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    for trial in range(4):
        k = [rng.integers(0, L) for L in dims]
        p = [2 * np.pi * k[i] / dims[i] for i in range(3)]
        p.append((2 * k[3] + 1) * np.pi / T if antiperiodic else 2 * np.pi * k[3] / T)
        u = (rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4)))
        phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
        psi = phase[..., None, None] * u
        W = ma + sum(1 - np.cos(pm) for pm in p)
        K = W * np.eye(4) + 1j * sum(np.sin(p[m]) * oracle.gamma(m) for m in range(4))
        expect = phase[..., None, None] * (u @ K)
        assert _rel(oracle.apply(U, kappa, psi, antiperiodic=antiperiodic), expect) < 1e-13
        ev = np.linalg.eigvals(K)
        ev = ev[np.argsort(ev.imag)]
        s = np.sqrt(sum(np.sin(pm) ** 2 for pm in p))
        assert np.allclose(ev, np.array([W - 1j * s] * 2 + [W + 1j * s] * 2), atol=1e-13)


def test_free_field_spectrum_of_dense_matrix():
    """All eigenvalues of M on a free 4x2x2x4 lattice are W(p) +- i|sin p| with multiplicity 6 each."""
    dims = (4, 2, 2, 4)
    X, Y, Z, T = dims
    kappa = 0.1
    ma = 1 / (2 * kappa) - 4
    Md = oracle.dense_matrix(li.unit_links(dims), kappa)
    ev = np.linalg.eigvals(Md)
    ev = ev[np.lexsort((ev.real.round(8), ev.imag.round(8)))]
    expect = []
    for kx in range(X):
        for ky in range(Y):
            for kz in range(Z):
                for kt in range(T):
                    p = [2 * np.pi * kx / X, 2 * np.pi * ky / Y, 2 * np.pi * kz / Z, (2 * kt + 1) * np.pi / T]
                    W = ma + sum(1 - np.cos(v) for v in p)
                    s = np.sqrt(sum(np.sin(v) ** 2 for v in p))
                    expect += [W + 1j * s] * 6 + [W - 1j * s] * 6
    expect = np.array(expect)
    expect = expect[np.lexsort((expect.real.round(8), expect.imag.round(8)))]
    assert np.abs(ev - expect).max() < 1e-10


# ------------------------------------------------------------------ even-odd

def test_eo_operator_identities():
    """With b_o = 0, eq. eo2-eo3 give b_e = M_prec psi_e / (m a + 4) and psi_o = (1/2) D_oe psi_e / (m a + 4)."""
    dims = (4, 4, 2, 4)
    U = li.random_links(dims, 1.0, 1002)
    kappa = 0.124
    a = 1 / (2 * kappa)
    odd = oracle.parity_mask(dims)
    psi = li.gaussian_field(dims, 9)
    psi[odd] = 0
    full = psi.copy()
    h = oracle.hopping(U, psi)
    full[odd] = 0.5 * h[odd] / a
    b = oracle.apply(U, kappa, full)
    assert np.abs(b[odd]).max() < 1e-13
    mp = oracle.mprec(U, kappa, psi)
    assert _rel(b[~odd], mp[~odd] / a) < 1e-14
    assert np.abs(mp[odd]).max() == 0.0


# ------------------------------------------------------------------ solvers

def test_bicgstab_vs_dense_lu_2444():
    """2^4 lattice (forward and backward neighbours coincide): BiCGstab vs LAPACK."""
    dims = (2, 2, 2, 2)
    U = li.random_links(dims, 1.0, 1003)
    b = li.gaussian_field(dims, 2003)
    for kappa in (0.12, 0.13):
        Md = oracle.dense_matrix(U, kappa)
        x_lu = np.linalg.solve(Md, b.ravel()).reshape(b.shape)
        x, it, st, _ = oracle.bicgstab(U, kappa, b, tol=1e-14)
        assert st == oracle.STATUS_OK
        assert _rel(x, x_lu) < 1e-12
        xe, it2, st2, _ = oracle.bicgstab_eo(U, kappa, b, tol=1e-14)
        assert st2 == oracle.STATUS_OK
        assert _rel(xe, x_lu) < 1e-12
        # the dense matrix of M^dag is the conjugate transpose
        Mdag = oracle.dense_matrix(U, kappa)
        q = li.gaussian_field(dims, 4)
        assert _rel(oracle.apply(U, kappa, q, dag=True).ravel(), Mdag.conj().T @ q.ravel()) < 1e-14


def test_bicgstab_plain_config_4444():
    """Plain FP64 BiCGstab on 4^4, eps = 0.3, kappa = 0.12 to 1e-10 (the small parity case)."""
    dims = (4, 4, 4, 4)
    U = li.random_links(dims, 0.3, 1000)
    b = li.gaussian_field(dims, 2000)
    x, it, st, hist = oracle.bicgstab(U, 0.12, b, tol=1e-10)
    assert st == oracle.STATUS_OK
    assert oracle.true_residual(U, 0.12, x, b) < 1e-10 * 1.5
    assert 20 < it < 80
    # the recurrence residual tracks the true residual
    assert abs(hist[-1] - oracle.true_residual(U, 0.12, x, b)) < 1e-11


def test_free_field_solution_closed_form():
    """U = 1, plane-wave source b = e^{ip.n} u: x = e^{ip.n} u K^{-1}."""
    dims = (4, 4, 4, 8)
    X, Y, Z, T = dims
    kappa = 0.12
    ma = 1 / (2 * kappa) - 4
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    p = [2 * np.pi / X, 0.0, 2 * np.pi * 3 / Z, 3 * np.pi / T]
    u = np.arange(12).reshape(3, 4) + 1j
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    b = phase[..., None, None] * u
    K = (ma + sum(1 - np.cos(v) for v in p)) * np.eye(4) + 1j * sum(np.sin(p[m]) * oracle.gamma(m) for m in range(4))
    expect = phase[..., None, None] * (u @ np.linalg.inv(K))
    for eo in (False, True):
        xs, it, st, _ = oracle.bicgstab(li.unit_links(dims), kappa, b, tol=1e-13, eo=eo)
        assert _rel(xs, expect) < 1e-11


def test_even_odd_equals_full_solve():
    dims = (4, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1004)
    b = li.gaussian_field(dims, 2004)
    kappa = 0.13
    x, it, st, _ = oracle.bicgstab(U, kappa, b, tol=1e-12)
    xe, ite, ste, _ = oracle.bicgstab_eo(U, kappa, b, tol=1e-12)
    assert st == ste == oracle.STATUS_OK
    assert oracle.true_residual(U, kappa, xe, b) < 2e-12
    assert _rel(xe, x) < 1e-10
    assert ite < it


def test_bicgstab_m_shifted_solutions():
    """Each shifted iterate solves its own system (true FP64 residual), agrees with the single-mass
    solution, and shifts far from the base freeze earlier (Sec. 6.1)."""
    dims = (4, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1001)
    b = li.gaussian_field(dims, 2001)
    kappas = [0.120, 0.122, 0.124, 0.126, 0.128, 0.130]
    xs, it, st, conv = oracle.bicgstab_m(U, kappas, b, tol=1e-10)
    assert st == oracle.STATUS_OK
    for k, x in zip(kappas, xs):
        assert oracle.true_residual(U, k, x, b) < 2e-10
        xr, _, _, _ = oracle.bicgstab(U, k, b, tol=1e-12)
        assert _rel(x, xr) < 1e-8
    assert conv[-1] == it
    assert conv[0] <= conv[-1]
    assert conv == sorted(conv)


def test_bicgstab_m_single_mass_is_bicgstab():
    dims = (4, 4, 2, 4)
    U = li.random_links(dims, 1.0, 1005)
    b = li.gaussian_field(dims, 2005)
    xs, it, st, _ = oracle.bicgstab_m(U, [0.125], b, tol=1e-10)
    x, it2, st2, _ = oracle.bicgstab(U, 0.125, b, tol=1e-10)
    assert it == it2
    assert _rel(xs[0], x) < 1e-13


def test_poly_weights_exact_for_polynomials():
    """The Lagrange form reproduces any polynomial of degree < k from k points (Sec. 6.2.1)."""
    rng = np.random.default_rng(0)
    ms = [-0.2, -0.15, -0.1, -0.05]
    for deg in range(len(ms)):
        c = rng.standard_normal((deg + 1, 5))
        f = lambda m: sum(c[i] * m ** i for i in range(deg + 1))
        w = oracle.poly_weights(ms, -0.3)
        approx = sum(wj * f(mj) for wj, mj in zip(w, ms))
        assert np.allclose(approx, f(-0.3), atol=1e-12)
    assert oracle.poly_weights([0.1], 0.3) == [1.0]


def test_multimass_sequential_with_guess():
    dims = (4, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1001)
    b = li.gaussian_field(dims, 2001)
    kappas = [0.120, 0.122, 0.124, 0.126, 0.128, 0.130]
    sols, its = oracle.multimass_sequential(U, kappas, b, tol=1e-10, guess="poly")
    sols0, its0 = oracle.multimass_sequential(U, kappas, b, tol=1e-10, guess="none")
    for k, x in zip(kappas, sols):
        assert oracle.true_residual(U, k, x, b) < 2e-10
    assert sum(its) < sum(its0)


def _free_plane_wave_solution(dims, kappa, p, u):
    X, Y, Z, T = dims
    ma = 1 / (2 * kappa) - 4
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    phase = np.exp(1j * (p[0] * x + p[1] * y + p[2] * z + p[3] * t))
    K = (ma + sum(1 - np.cos(v) for v in p)) * np.eye(4) + 1j * sum(np.sin(p[m]) * oracle.gamma(m) for m in range(4))
    return phase[..., None, None] * u, phase[..., None, None] * (u @ np.linalg.inv(K))


def test_solution_space_guess_exact_in_free_field():
    """U = 1 and a plane-wave source: x(m) = e^{ip.n} u (W - iS)/(W^2 + s^2) with S = sum sin(p)
    gamma, S^2 = s^2, so every solution lies in the two-dimensional span of e^{ip.n} u and
    e^{ip.n} u S. From the exact solutions at two masses the minimising combination (Sec. 6.2.2)
    must reproduce the solution at any third mass; the two-point Lagrange guess (linear in m)
    cannot."""
    dims = (4, 4, 4, 8)
    p = [2 * np.pi / 4, 0.0, 2 * np.pi * 3 / 4, 3 * np.pi / 8]
    u = np.arange(12).reshape(3, 4) + 1j
    U = li.unit_links(dims)
    k_prev = [0.110, 0.115]
    b, _ = _free_plane_wave_solution(dims, 0.11, p, u)
    psis = [_free_plane_wave_solution(dims, k, p, u)[1] for k in k_prev]
    for kappa in (0.118, 0.122, 0.105):
        _, exact = _free_plane_wave_solution(dims, kappa, p, u)
        v, c = oracle.solution_space_guess(b, psis, k_prev, kappa)
        assert _rel(v, exact) < 1e-11
        assert oracle.true_residual(U, kappa, v, b) < 1e-12
        w = oracle.poly_weights([oracle.mass_of_kappa(k) for k in k_prev], oracle.mass_of_kappa(kappa))
        vp = sum(wj * pj for wj, pj in zip(w, psis))
        assert oracle.true_residual(U, kappa, vp, b) > 1e-4


def test_solution_space_guess_minimises_over_the_span():
    """Random links: the columns are M(kappa) psi_j (checked against the operator itself), and no
    other combination of the same solutions (the Lagrange guess, or each solution alone with its
    best scale) has a smaller residual."""
    dims = (4, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1012)
    b = li.gaussian_field(dims, 2012)
    k_prev = [0.120, 0.123, 0.126]
    psis = [oracle.bicgstab(U, k, b, tol=1e-13)[0] for k in k_prev]
    kappa = 0.129
    for k, ps in zip(k_prev, psis):
        d = b + (1 / (2 * kappa) - 1 / (2 * k)) * ps
        assert _rel(oracle.apply(U, kappa, ps), d) < 1e-11
    v, c = oracle.solution_space_guess(b, psis, k_prev, kappa)
    r_min = np.linalg.norm(b - oracle.apply(U, kappa, v))
    w = oracle.poly_weights([oracle.mass_of_kappa(k) for k in k_prev], oracle.mass_of_kappa(kappa))
    vp = sum(wj * pj for wj, pj in zip(w, psis))
    assert r_min <= np.linalg.norm(b - oracle.apply(U, kappa, vp)) * (1 + 1e-12)
    for ps in psis:
        mp = oracle.apply(U, kappa, ps).reshape(-1)
        alpha = np.vdot(mp, b.reshape(-1)) / np.vdot(mp, mp)
        assert r_min <= np.linalg.norm(b.reshape(-1) - alpha * mp) * (1 + 1e-12)
    # the normal equations hold: the residual is orthogonal to every M(kappa) psi_j
    r = (b - oracle.apply(U, kappa, v)).reshape(-1)
    for ps in psis:
        assert abs(np.vdot(oracle.apply(U, kappa, ps).reshape(-1), r)) < 1e-9 * np.linalg.norm(b) ** 2


def test_multimass_sequential_minres_guess_and_order():
    dims = (4, 4, 4, 8)
    U = li.random_links(dims, 1.0, 1001)
    b = li.gaussian_field(dims, 2001)
    kappas = [0.120, 0.122, 0.124, 0.126, 0.128, 0.130]
    sols0, its0 = oracle.multimass_sequential(U, kappas, b, tol=1e-10, guess="none")
    for guess in ("minres", "poly"):
        for order in (0, 1, 2):
            sols, its = oracle.multimass_sequential(U, kappas, b, tol=1e-10, guess=guess, order=order)
            for k, x in zip(kappas, sols):
                assert oracle.true_residual(U, k, x, b) < 2e-10
            assert sum(its) < sum(its0)


def test_multimass_sequential_repeated_mass():
    """A mass given twice: the Lagrange set keeps distinct masses, and the repeated mass starts
    from its own earlier solution (already converged)."""
    dims = (4, 4, 2, 4)
    U = li.random_links(dims, 1.0, 1015)
    b = li.gaussian_field(dims, 2015)
    kappas = [0.120, 0.126, 0.120, 0.130]
    sols, its = oracle.multimass_sequential(U, kappas, b, tol=1e-10, guess="poly")
    for k, x in zip(kappas, sols):
        assert oracle.true_residual(U, k, x, b) < 2e-10
    assert min(its[0], its[2]) <= 1


# ------------------------------------------------------------------ gradient

def _loss(U, kappa, eta, b):
    x, _, st, _ = oracle.bicgstab(U, kappa, b, tol=1e-15, maxit=2000)
    return float(np.real(np.vdot(eta, x)))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 4)])
def test_gauge_grad_central_differences(dims):
    """dL/dRe U + i dL/dIm U against central differences (h = 1e-6) on 20 random link entries,
    for L = Re<eta, M^{-1} b>; lam is obtained as gamma5 M^{-1} gamma5 eta."""
    kappa = 0.125
    U = li.random_links(dims, 1.0, 1006)
    b = li.gaussian_field(dims, 2006)
    eta = li.gaussian_field(dims, 2007)
    x, _, _, _ = oracle.bicgstab(U, kappa, b, tol=1e-15, maxit=2000)
    lg, _, _, _ = oracle.bicgstab(U, kappa, eta @ G5, tol=1e-15, maxit=2000)
    lam = lg @ G5
    # lam solves M^dag lam = eta
    assert _rel(oracle.apply(U, kappa, lam, dag=True), eta) < 1e-13
    G = oracle.gauge_grad(x, lam)
    rng = np.random.default_rng(11)
    h = 1e-6
    flat = U.reshape(-1)
    for _ in range(20):
        j = int(rng.integers(0, flat.size))
        vals = []
        for step in (h, 1j * h):
            Up = flat.copy(); Up[j] += step
            Um = flat.copy(); Um[j] -= step
            vals.append((_loss(Up.reshape(U.shape), kappa, eta, b) - _loss(Um.reshape(U.shape), kappa, eta, b)) / (2 * h))
        fd = vals[0] + 1j * vals[1]
        assert abs(fd - G.reshape(-1)[j]) < 1e-7 * max(1.0, abs(fd))


def test_su3_projected_gradient():
    """dL/de_a for U_mu(n) -> exp(i e_a T_a) U_mu(n) equals 2 tr(T_a F), T_a = Gell-Mann / 2."""
    dims = (2, 2, 2, 4)
    kappa = 0.125
    U = li.random_links(dims, 1.0, 1008)
    b = li.gaussian_field(dims, 2008)
    eta = li.gaussian_field(dims, 2009)
    x, _, _, _ = oracle.bicgstab(U, kappa, b, tol=1e-15, maxit=2000)
    lg, _, _, _ = oracle.bicgstab(U, kappa, eta @ G5, tol=1e-15, maxit=2000)
    F = oracle.su3_project(U, oracle.gauge_grad(x, lg @ G5))
    # F is Hermitian and traceless
    assert np.abs(F - np.conj(np.swapaxes(F, -1, -2))).max() < 1e-14
    assert np.abs(np.trace(F, axis1=-2, axis2=-1)).max() < 1e-14
    gm = np.zeros((8, 3, 3), dtype=np.complex128)
    gm[0][0, 1] = gm[0][1, 0] = 1
    gm[1][0, 1], gm[1][1, 0] = -1j, 1j
    gm[2][0, 0], gm[2][1, 1] = 1, -1
    gm[3][0, 2] = gm[3][2, 0] = 1
    gm[4][0, 2], gm[4][2, 0] = -1j, 1j
    gm[5][1, 2] = gm[5][2, 1] = 1
    gm[6][1, 2], gm[6][2, 1] = -1j, 1j
    gm[7] = np.diag([1, 1, -2]) / np.sqrt(3)
    Ta = gm / 2
    rng = np.random.default_rng(12)
    h = 1e-5
    for _ in range(6):
        mu, t, z, y, xx = (int(rng.integers(0, s)) for s in (4,) + U.shape[1:5])
        a = int(rng.integers(0, 8))
        w, v = np.linalg.eigh(Ta[a])
        vals = []
        for e in (h, -h):
            R = v @ np.diag(np.exp(1j * e * w)) @ v.conj().T
            Up = U.copy()
            Up[mu, t, z, y, xx] = R @ U[mu, t, z, y, xx]
            vals.append(_loss(Up, kappa, eta, b))
        fd = (vals[0] - vals[1]) / (2 * h)
        an = 2 * np.trace(Ta[a] @ F[mu, t, z, y, xx]).real
        assert abs(fd - an) < 1e-7 * max(1.0, abs(fd))
