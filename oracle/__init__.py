"""CPU oracle for the Wilson-Dirac multi-mass solve: TEST INFRASTRUCTURE ONLY.

Plain FP64 reference implementation (C library `liboracle.so` plus small numpy helpers) of
what the GPU path computes. Only `tests/`, `__graft_entry__.smoke()` and the benchmark's
`cpu_baseline` leg may import it; the GPU package never does, and the two share no code.

Layout: lexicographic, x fastest. Gauge U[4][T][Z][Y][X][3][3], fermions psi[T][Z][Y][X][3][4],
complex128. M(kappa) is the paper's M(m;U) with m*a + 4 = 1/(2 kappa) (Sec. 2, eq. 3).

Functions and the passages they follow:
  apply / hopping           Sec. 2, eq. 3 and eq. 4 (full 4x4 spin matrices)
  mprec / eo_source /
  eo_reconstruct            Sec. 6.2.3, eq. eo2-eo4
  bicgstab / bicgstab_eo    van der Vorst's BiCGstab (cited in Sec. 6), update x <- x - beta s + chi w (Sec. 5)
  bicgstab_m                BiCGstab-M (Jegerlehner, cited in Sec. 6.1), base = most singular mass,
                            frozen shifts (Sec. 6.1)
  poly_weights              Lagrange form of the Vandermonde solve (Sec. 6.2.1)
  multimass_sequential      heaviest mass first, highest-order polynomial guess (Sec. 7)
  gauge_grad / su3_project  derivative of Re<eta, M^{-1} b> with respect to the links
  normal_apply / cg / cg_m /
  normal_sequential         CG and multi-shift CG-M (Sec. 8 names them as the other Krylov pair the
                            findings carry over to) on the shifted even-site normal equations
                            (M_prec^dag M_prec + sigma) x = b_e, the family that shares one Krylov
                            space (Sec. 6.1); the single-shift driver mirrors Sec. 7 (largest
                            shift first, Lagrange guess in sigma)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIBPATH = os.path.join(_HERE, "liboracle.so")
_lib = None

STATUS_OK = 0
STATUS_NOCONV = 4
STATUS_BREAKDOWN = 5

_D = ctypes.POINTER(ctypes.c_double)
_I = ctypes.POINTER(ctypes.c_int)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIBPATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIBPATH)
        L.oracle_gamma.argtypes = [ctypes.c_int, _D]
        L.oracle_hopping.argtypes = [_I, ctypes.c_int, _D, _D, _D, ctypes.c_int]
        L.oracle_apply.argtypes = [_I, ctypes.c_int, _D, ctypes.c_double, _D, _D, ctypes.c_int]
        L.oracle_mprec.argtypes = [_I, ctypes.c_int, _D, ctypes.c_double, _D, _D, ctypes.c_int]
        L.oracle_eo_source.argtypes = [_I, ctypes.c_int, _D, ctypes.c_double, _D, _D]
        L.oracle_eo_reconstruct.argtypes = [_I, ctypes.c_int, _D, ctypes.c_double, _D, _D]
        L.oracle_bicgstab.argtypes = [_I, ctypes.c_int, _D, ctypes.c_double, _D, _D, ctypes.c_double,
                                      ctypes.c_int, ctypes.c_int, _I, _D]
        L.oracle_bicgstab.restype = ctypes.c_int
        L.oracle_bicgstab_eo.argtypes = L.oracle_bicgstab.argtypes
        L.oracle_bicgstab_eo.restype = ctypes.c_int
        L.oracle_bicgstab_m.argtypes = [_I, ctypes.c_int, _D, ctypes.c_int, _D, _D, _D, ctypes.c_double,
                                        ctypes.c_int, _I, _I]
        L.oracle_bicgstab_m.restype = ctypes.c_int
        L.oracle_gauge_grad.argtypes = [_I, ctypes.c_int, _D, _D, _D]
        L.oracle_parity.argtypes = [_I, ctypes.c_long]
        L.oracle_parity.restype = ctypes.c_int
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_get_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def get_threads() -> int:
    return int(lib().oracle_get_threads())


def _dp(a):
    return a.ctypes.data_as(_D)


def _dims_of_links(U):
    assert U.ndim == 7 and U.shape[0] == 4 and U.shape[-2:] == (3, 3)
    T, Z, Y, X = U.shape[1:5]
    return (X, Y, Z, T)


def _dims_arr(dims):
    return (ctypes.c_int * 4)(*dims)


def _c128(a):
    return np.ascontiguousarray(a, dtype=np.complex128)


def gamma(mu: int) -> np.ndarray:
    """gamma_mu (mu = 0..3 for the paper's 1..4) in the chiral basis of Sec. 2."""
    out = np.zeros((4, 4), dtype=np.complex128)
    lib().oracle_gamma(mu, _dp(out))
    return out


def hopping(U, psi, dag=False, antiperiodic=True):
    """sum over the 8 directions of T_mu psi (the bracket of eq. 3 without the -1/2)."""
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().oracle_hopping(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), _dp(psi), _dp(out), int(dag))
    return out


def apply(U, kappa, psi, dag=False, antiperiodic=True):
    """M(kappa) psi, or M(kappa)^dag psi (eq. 3)."""
    U = _c128(U)
    psi = _c128(psi)
    out = np.empty_like(psi)
    lib().oracle_apply(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), float(kappa), _dp(psi), _dp(out),
                       int(dag))
    return out


def parity_mask(dims):
    """Boolean [T, Z, Y, X] array, True on odd sites (parity of x+y+z+t, Sec. 6.2.3)."""
    X, Y, Z, T = dims
    t, z, y, x = np.meshgrid(np.arange(T), np.arange(Z), np.arange(Y), np.arange(X), indexing="ij")
    return ((x + y + z + t) % 2) == 1


def mprec(U, kappa, psi_e, dag=False, antiperiodic=True):
    """M_prec psi_e on full-length fields (odd sites of psi_e ignored, zero on return), eq. eo4."""
    U = _c128(U)
    psi = _c128(psi_e)
    out = np.empty_like(psi)
    lib().oracle_mprec(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), float(kappa), _dp(psi), _dp(out),
                       int(dag))
    return out


def eo_source(U, kappa, b, antiperiodic=True):
    U = _c128(U)
    b = _c128(b)
    out = np.empty_like(b)
    lib().oracle_eo_source(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), float(kappa), _dp(b), _dp(out))
    return out


def eo_reconstruct(U, kappa, b, x_even, antiperiodic=True):
    U = _c128(U)
    b = _c128(b)
    x = _c128(x_even).copy()
    lib().oracle_eo_reconstruct(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), float(kappa), _dp(b),
                                _dp(x))
    return x


def bicgstab(U, kappa, b, tol=1e-10, maxit=10000, x0=None, antiperiodic=True, eo=False):
    """Solve M(kappa) x = b; returns (x, iterations, status, relative-residual history)."""
    U = _c128(U)
    b = _c128(b)
    x = np.zeros_like(b) if x0 is None else _c128(x0).copy()
    it = ctypes.c_int(0)
    hist = np.zeros(maxit + 1)
    fn = lib().oracle_bicgstab_eo if eo else lib().oracle_bicgstab
    st = fn(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), float(kappa), _dp(b), _dp(x), float(tol),
            int(maxit), int(x0 is not None), ctypes.byref(it), _dp(hist))
    return x, it.value, st, hist[: it.value].copy()


def bicgstab_eo(U, kappa, b, tol=1e-10, maxit=10000, x0=None, antiperiodic=True):
    return bicgstab(U, kappa, b, tol, maxit, x0, antiperiodic, eo=True)


def bicgstab_m(U, kappas, b, tol=1e-10, maxit=10000, antiperiodic=True):
    """Multi-shift BiCGstab-M; returns (list of x_i in the order of kappas, iterations, status, freeze iterations)."""
    U = _c128(U)
    b = _c128(b)
    k = np.ascontiguousarray(kappas, dtype=np.float64)
    nk = len(k)
    assert 1 <= nk <= 64
    xs = np.zeros((nk,) + b.shape, dtype=np.complex128)
    it = ctypes.c_int(0)
    conv = (ctypes.c_int * nk)()
    st = lib().oracle_bicgstab_m(_dims_arr(_dims_of_links(U)), int(antiperiodic), _dp(U), nk, _dp(k), _dp(b), _dp(xs),
                                 float(tol), int(maxit), ctypes.byref(it), conv)
    return [xs[i] for i in range(nk)], it.value, st, list(conv)


def true_residual(U, kappa, x, b, antiperiodic=True):
    """|b - M x| / |b| in FP64."""
    r = b - apply(U, kappa, x, antiperiodic=antiperiodic)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def mass_of_kappa(kappa):
    """m a = 1/(2 kappa) - 4."""
    return 1.0 / (2.0 * np.asarray(kappa, dtype=np.float64)) - 4.0


def poly_weights(m_prev, m_new):
    """Lagrange weights c_j = prod_{i != j} (m - m_i)/(m_j - m_i) (Sec. 6.2.1), so that the
    extrapolated guess is psi(m) = sum_j c_j psi_j."""
    m_prev = [float(v) for v in m_prev]
    c = []
    for j, mj in enumerate(m_prev):
        w = 1.0
        for i, mi in enumerate(m_prev):
            if i != j:
                w *= (m_new - mi) / (mj - mi)
        c.append(w)
    return c


def solution_space_guess(b, psis, kappas_prev, kappa):
    """Solution-space minimisation (Sec. 6.2.2): the combination v = sum_j c_j psi_j of earlier
    solutions psi_j (of M(kappa_j) psi_j = b) that minimises |b - M(kappa) v|_2. Because the
    masses enter M only through the diagonal, M(kappa) psi_j = b + (m - m_j) a psi_j with
    (m - m_j) a = 1/(2 kappa) - 1/(2 kappa_j), so no operator is applied: the columns
    d_j = b + s_j psi_j go to a plain least-squares solve. Returns (v, c)."""
    b = _c128(b).reshape(-1)
    cols = [b + (1.0 / (2.0 * kappa) - 1.0 / (2.0 * kj)) * _c128(p).reshape(-1) for p, kj in zip(psis, kappas_prev)]
    D = np.stack(cols, axis=1)
    c = np.linalg.lstsq(D, b, rcond=None)[0]
    v = sum(cj * _c128(p) for cj, p in zip(c, psis))
    return v, c


def multimass_sequential(U, kappas, b, tol=1e-10, maxit=10000, guess="poly", eo=True, antiperiodic=True, order=0):
    """Single-mass BiCGstab once per mass, heaviest mass (smallest kappa) first; with
    guess='poly' each start vector is the Lagrange extrapolation in m a of the solutions found so
    far (Sec. 6.2.1, Sec. 7), with guess='minres' their residual-minimising combination (Sec.
    6.2.2); order > 0 uses only the most recent `order` solutions. Returns (solutions in the
    caller's order, iteration counts in the caller's order)."""
    seq = sorted(range(len(kappas)), key=lambda i: kappas[i])
    sols, its = [None] * len(kappas), [0] * len(kappas)
    done_m, done_x, done_k = [], [], []
    for i in seq:
        x0 = None
        m = float(mass_of_kappa(kappas[i]))
        k = len(done_x) if order <= 0 else min(order, len(done_x))
        if guess == "poly" and k:
            # distinct masses only (latest solution of a repeated mass); a repeated mass is its own guess
            ms, xs_ = [], []
            for mj, xj in zip(done_m[-k:], done_x[-k:]):
                if mj in ms:
                    i0 = ms.index(mj)
                    del ms[i0], xs_[i0]
                ms.append(mj)
                xs_.append(xj)
            if m in ms:
                x0 = xs_[ms.index(m)].copy()
            else:
                c = poly_weights(ms, m)
                x0 = sum(cj * xj for cj, xj in zip(c, xs_))
        elif guess == "minres" and k:
            x0, _ = solution_space_guess(b, done_x[-k:], done_k[-k:], kappas[i])
        x, it, st, _ = bicgstab(U, kappas[i], b, tol, maxit, x0=x0, antiperiodic=antiperiodic, eo=eo)
        sols[i], its[i] = x, it
        done_m.append(m)
        done_x.append(x)
        done_k.append(kappas[i])
    return sols, its


def gauge_grad(x, lam, antiperiodic=True):
    """G_mu(n) = dL/dRe U + i dL/dIm U for L = Re<eta, M^{-1} b>, given x = M^{-1} b and
    lam = M^{-dag} eta; shape [4, T, Z, Y, X, 3, 3]."""
    x = _c128(x)
    lam = _c128(lam)
    T, Z, Y, X = x.shape[:4]
    G = np.empty((4, T, Z, Y, X, 3, 3), dtype=np.complex128)
    lib().oracle_gauge_grad(_dims_arr((X, Y, Z, T)), int(antiperiodic), _dp(x), _dp(lam), _dp(G))
    return G


def su3_project(U, G):
    """F = (i/2) TA(U G^dag), TA(Y) = (Y - Y^dag)/2 - tr(Y - Y^dag)/6. For U -> exp(i e_a T_a) U
    with Hermitian traceless generators T_a, dL/de_a = 2 tr(T_a F)."""
    Y = np.einsum("...ab,...cb->...ac", U, np.conj(G))
    A = 0.5 * (Y - np.conj(np.swapaxes(Y, -1, -2)))
    tr = np.trace(A, axis1=-2, axis2=-1)[..., None, None] / 3.0
    return 0.5j * (A - tr * np.eye(3))


def dense_matrix(U, kappa, antiperiodic=True):
    """Dense M(kappa) built column by column from the oracle operator (tiny lattices only)."""
    T, Z, Y, X = U.shape[1:5]
    n = X * Y * Z * T * 12
    Mdense = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[:] = 0
        e[j] = 1
        Mdense[:, j] = apply(U, kappa, e.reshape(T, Z, Y, X, 3, 4), antiperiodic=antiperiodic).ravel()
    return Mdense


# ------------------------------------------------------------------ CG and CG-M (Sec. 8)

def even_part(psi):
    """psi with its odd sites set to zero."""
    out = _c128(psi).copy()
    out[parity_mask((out.shape[3], out.shape[2], out.shape[1], out.shape[0]))] = 0
    return out


def normal_apply(U, kappa, sigma, x_e, antiperiodic=True):
    """(M_prec^dag M_prec + sigma) x_e on the even sites (odd sites of x_e ignored, zero on return);
    M_prec of eq. eo4. Hermitian and positive definite for sigma >= 0."""
    x_e = even_part(x_e)
    y = mprec(U, kappa, x_e, antiperiodic=antiperiodic)
    return mprec(U, kappa, y, dag=True, antiperiodic=antiperiodic) + sigma * x_e


def _vdot(a, b):
    return complex(np.vdot(a.ravel(), b.ravel()))


def cg(U, kappa, sigma, b, tol=1e-10, maxit=10000, x0=None, antiperiodic=True):
    """Conjugate gradients (Hestenes-Stiefel) on (M_prec^dag M_prec + sigma) x = b_e:
        r = b_e - A x0, p = r
        repeat: alpha = |r|^2 / <p, A p>;  x += alpha p;  r -= alpha A p
                beta = |r_new|^2 / |r|^2;  p = r + beta p
        until |r| <= tol |b_e|.
    Returns (x, iterations, status, relative-residual history)."""
    be = even_part(b)
    x = np.zeros_like(be) if x0 is None else even_part(x0)
    r = be - normal_apply(U, kappa, sigma, x, antiperiodic) if x0 is not None else be.copy()
    p = r.copy()
    bn = np.linalg.norm(be)
    rr = np.vdot(r.ravel(), r.ravel()).real
    hist = []
    if bn == 0.0:
        return np.zeros_like(be), 0, STATUS_OK, hist
    it = 0
    while np.sqrt(rr) > tol * bn:
        if it >= maxit:
            return x, it, STATUS_NOCONV, hist
        Ap = normal_apply(U, kappa, sigma, p, antiperiodic)
        pAp = _vdot(p, Ap).real
        if pAp <= 0.0:
            return x, it, STATUS_BREAKDOWN, hist
        alpha = rr / pAp
        x = x + alpha * p
        r = r - alpha * Ap
        rr_new = np.vdot(r.ravel(), r.ravel()).real
        p = r + (rr_new / rr) * p
        rr = rr_new
        it += 1
        hist.append(np.sqrt(rr) / bn)
    return x, it, STATUS_OK, hist


def cg_m(U, kappa, sigmas, b, tol=1e-10, maxit=10000, antiperiodic=True):
    """Multi-shift CG-M on (M_prec^dag M_prec + sigma_i) x_i = b_e for all i at once, with x_i = 0
    to start (Sec. 6.1: the shifted systems share one Krylov space). The base system is the
    smallest shift sigma_0 (the slowest to converge); shift d_i = sigma_i - sigma_0 >= 0. The
    residual of system i is collinear with the base residual, r^i_n = zeta^i_n r_n, and matching
    the three-term residual recurrences of CG for A and A + d gives
        zeta_{n+1} = zeta_n zeta_{n-1} alpha_{n-1}
                     / (zeta_{n-1} alpha_{n-1} (1 + alpha_n d) + alpha_n beta_n (zeta_{n-1} - zeta_n))
        alpha^i_n = alpha_n zeta_{n+1} / zeta_n,   beta^i_{n+1} = beta_{n+1} (zeta_{n+1} / zeta_n)^2
        x^i += alpha^i_n p^i_n,   p^i_{n+1} = zeta_{n+1} r_{n+1} + beta^i_{n+1} p^i_n
    with zeta_{-1} = zeta_0 = 1, alpha_{-1} = 1, beta_0 = 0. System i is frozen once
    |zeta^i| |r| <= tol |b_e|; the solve stops when the base converges.
    Returns (list of x_i in the order of sigmas, iterations, status, freeze iterations)."""
    sig = [float(s) for s in sigmas]
    assert min(sig) >= 0.0
    base = int(np.argmin(sig))
    be = even_part(b)
    bn = np.linalg.norm(be)
    n = len(sig)
    xs = [np.zeros_like(be) for _ in range(n)]
    conv = [0] * n
    if bn == 0.0:
        return xs, 0, STATUS_OK, conv
    r = be.copy()
    ps = [be.copy() for _ in range(n)]   # p^i (the base's p is ps[base])
    z_prev = [1.0] * n
    z = [1.0] * n
    active = [True] * n
    alpha_prev, beta = 1.0, 0.0
    rr = np.vdot(r.ravel(), r.ravel()).real
    it = 0
    while np.sqrt(rr) > tol * bn:
        if it >= maxit:
            return xs, it, STATUS_NOCONV, conv
        p = ps[base]
        Ap = normal_apply(U, kappa, sig[base], p, antiperiodic)
        pAp = _vdot(p, Ap).real
        if pAp <= 0.0:
            return xs, it, STATUS_BREAKDOWN, conv
        alpha = rr / pAp
        z_next = [1.0] * n
        for i in range(n):
            if i == base or not active[i]:
                continue
            d = sig[i] - sig[base]
            z_next[i] = z[i] * z_prev[i] * alpha_prev / (
                z_prev[i] * alpha_prev * (1.0 + alpha * d) + alpha * beta * (z_prev[i] - z[i]))
        r = r - alpha * Ap
        rr_new = np.vdot(r.ravel(), r.ravel()).real
        beta_new = rr_new / rr
        for i in range(n):
            if not active[i]:
                continue
            if i == base:
                xs[i] = xs[i] + alpha * ps[i]
                ps[i] = r + beta_new * ps[i]
                continue
            a_i = alpha * z_next[i] / z[i]
            b_i = beta_new * (z_next[i] / z[i]) ** 2
            xs[i] = xs[i] + a_i * ps[i]
            ps[i] = z_next[i] * r + b_i * ps[i]
        it += 1
        for i in range(n):
            if i == base or not active[i]:
                continue
            z_prev[i], z[i] = z[i], z_next[i]
            if abs(z[i]) * np.sqrt(rr_new) <= tol * bn:
                active[i] = False
                conv[i] = it
        alpha_prev, beta, rr = alpha, beta_new, rr_new
    conv[base] = it
    for i in range(n):
        if active[i]:
            conv[i] = it
    return xs, it, STATUS_OK, conv


def normal_sequential(U, kappa, sigmas, b, tol=1e-10, maxit=10000, guess="poly", antiperiodic=True, order=0):
    """CG once per shift, largest shift (best conditioned) first; with guess='poly' each start
    vector is the Lagrange extrapolation in sigma of the solutions found so far (the analogue of
    Sec. 6.2.1 and Sec. 7 for this family); order > 0 keeps only the most recent `order`. Returns
    (solutions in the caller's order, iteration counts in the caller's order)."""
    seq = sorted(range(len(sigmas)), key=lambda i: -sigmas[i])
    sols, its = [None] * len(sigmas), [0] * len(sigmas)
    done_s, done_x = [], []
    for i in seq:
        x0 = None
        s = float(sigmas[i])
        k = len(done_x) if order <= 0 else min(order, len(done_x))
        if guess == "poly" and k:
            ss, xs_ = [], []
            for sj, xj in zip(done_s[-k:], done_x[-k:]):
                if sj in ss:
                    i0 = ss.index(sj)
                    del ss[i0], xs_[i0]
                ss.append(sj)
                xs_.append(xj)
            if s in ss:
                x0 = xs_[ss.index(s)].copy()
            else:
                c = poly_weights(ss, s)
                x0 = sum(cj * xj for cj, xj in zip(c, xs_))
        x, it, st, _ = cg(U, kappa, s, b, tol, maxit, x0=x0, antiperiodic=antiperiodic)
        sols[i], its[i] = x, it
        done_s.append(s)
        done_x.append(x)
    return sols, its

