"""Thin-film (Reynolds lubrication) pin of the elements of K that depend
only on the quadratic gap and on surface i's curvature: K33, K36 and the
rotation block K44, K45, K55 (Appendix).

The gap between the surfaces of Eqs. lub:surface-i and lub:surface-j is
H(x) = h + x^T M x to second order.  The Reynolds equation
    div(H^3 grad p) = 12 mu dH/dt
has exact solutions for the two motions needed here:
  * squeeze, dH/dt = -V:                p = 3 mu V / (tr M H^2)
  * tilt,    dH/dt = c.x (relative rotation about an in-plane axis):
                                        p = b.x / H^2,
                                        b = -6 mu (M + 2 tr M I)^{-1} c
(both checked below by finite differences).  Forces and torques on surface
i follow from the pressure acting along surface i's normal; the ln h
coefficient is extracted numerically from the moment integrals at two
small gaps.  None of this uses the appendix formulas.
"""
import numpy as np
import pytest


def M_of(S1, S2, iS1p, iS2p, cphi, sphi):
    """Quadratic gap matrix: surface i's curvature plus surface j's rotated
    by phi (x1' = cos phi x1 + sin phi x2)."""
    A = np.diag([1 / (2 * S1), 1 / (2 * S2)])
    R = np.array([[cphi, sphi], [-sphi, cphi]])
    B = R.T @ np.diag([iS1p / 2, iS2p / 2]) @ R
    return A, A + B


def quad_plane(f, M, h, tmin=-14.0, nt=4000, nth=256, rmax=None):
    """Integral of f(x1, x2) over the disc |u| < rmax of the rescaled
    coordinates u = sqrt(Lambda) X (H = h + |u|^2), polar grid in log
    radius (resolves both the sqrt(h) inner scale and the outer region)."""
    w, V = np.linalg.eigh(M)
    rmax = rmax or 1.0
    t = np.linspace(tmin, np.log(rmax), nt)
    rho = np.exp(t)
    th = np.linspace(0, 2 * np.pi, nth, endpoint=False)
    RH, TH = np.meshgrid(rho, th, indexing="ij")
    u1, u2 = RH * np.cos(TH), RH * np.sin(TH)
    X1, X2 = u1 / np.sqrt(w[0]), u2 / np.sqrt(w[1])
    x = V[:, 0][:, None, None] * X1 + V[:, 1][:, None, None] * X2
    val = f(x[0], x[1], h) * RH * RH   # dA = rho drho dtheta / sqrt(det)
    integ = np.trapezoid(val, t, axis=0).sum() * (2 * np.pi / nth)
    return integ / np.sqrt(w[0] * w[1])


def Hgap(M, h):
    return lambda x1, x2: h + M[0, 0] * x1 * x1 + 2 * M[0, 1] * x1 * x2 + M[1, 1] * x2 * x2


def reynolds_residual(p, H, src, x, eps=1e-4):
    """div(H^3 grad p) - src at point x by central differences."""
    def flux(xx, k):
        e = np.zeros(2)
        e[k] = eps
        dp = (p(*(xx + e)) - p(*(xx - e))) / (2 * eps)
        return H(*xx) ** 3 * dp
    tot = 0.0
    for k in range(2):
        e = np.zeros(2)
        e[k] = eps
        tot += (flux(x + e, k) - flux(x - e, k)) / (2 * eps)
    return tot - src(*x)


@pytest.mark.parametrize("seed", range(8))
def test_thin_film_elements(ref, seed):
    rng = np.random.default_rng(500 + seed)
    S1, S2 = rng.uniform(0.5, 8, size=2)
    iS1p, iS2p = rng.uniform(0.0, 1.5, size=2)
    ph = rng.uniform(0, 2 * np.pi)
    cphi, sphi = np.cos(ph), np.sin(ph)
    A, M = M_of(S1, S2, iS1p, iS2p, cphi, sphi)
    C, _ = ref.K_coeffs(S1, S2, iS1p, iS2p, np.zeros(4), np.zeros(4), cphi, sphi)
    mu, V = 1.0, 1.0
    trM = np.trace(M)
    h1, h2 = 1e-7, 1e-9

    # --- squeeze: K33 and K36 -------------------------------------------
    def p_sq(h):
        return lambda x1, x2: 3 * mu * V / (trM * Hgap(M, h)(x1, x2) ** 2)

    h0 = 1e-2
    for x in rng.normal(size=(3, 2)) * 0.3:
        res = reynolds_residual(p_sq(h0), Hgap(M, h0), lambda a, b: -12 * mu * V, x)
        assert abs(res) < 1e-5 * 12 * mu * V
    # normal force on i: -integral p (surface normal ~ e3), dU3 = -V
    F3 = -quad_plane(lambda a, b, h: p_sq(h)(a, b), M, h1, rmax=1e3)
    K33 = F3 / (mu * (-V))
    assert np.isclose(K33 * h1, C[2, 2], rtol=1e-4)

    # spin torque on i about e3 from the squeeze pressure acting along
    # surface i's normal (in-plane traction p grad H_i, H_i = -x^T A x)
    def t3(a, b, h):
        g1 = -2 * (A[0, 0] * a + A[0, 1] * b)
        g2 = -2 * (A[1, 0] * a + A[1, 1] * b)
        return p_sq(h)(a, b) * (a * g2 - b * g1)

    T1 = quad_plane(t3, M, h1)
    T2 = quad_plane(t3, M, h2)
    c63 = (T1 - T2) / np.log(h1 / h2) / (mu * (-V))
    scale = np.abs(C[3:5, 3:5]).max() + abs(C[2, 2]) * 1e-3
    assert abs(c63 - C[5, 2]) < 1e-4 * scale, (c63, C[5, 2])

    # --- tilt: rotation block ------------------------------------------
    for col in range(2):
        dW = np.zeros(2)
        dW[col] = 1.0
        # relative rotation of j about in-plane axes moves the surfaces
        # normally: dH/dt = (dOmega x x).e3 = dW1 x2 - dW2 x1
        cvec = np.array([-dW[1], dW[0]])
        b = -6 * mu * np.linalg.solve(M + 2 * trM * np.eye(2), cvec)

        def p_t(h, b=b):
            return lambda x1, x2: (b[0] * x1 + b[1] * x2) / Hgap(M, h)(x1, x2) ** 2

        for x in rng.normal(size=(3, 2)) * 0.3:
            res = reynolds_residual(p_t(h0), Hgap(M, h0),
                                    lambda a, bb: 12 * mu * (cvec[0] * a + cvec[1] * bb), x)
            assert abs(res) < 1e-5 * 12 * mu * (1 + np.abs(x).max())
        # torques about e1, e2 from the normal traction -p: (x2 f3, -x1 f3)
        tq = []
        for comp in range(2):
            def f(a, bb, h, comp=comp):
                pp = p_t(h)(a, bb)
                return -bb * pp if comp == 0 else a * pp
            tq.append((quad_plane(f, M, h1) - quad_plane(f, M, h2)) / np.log(h1 / h2))
        for comp in range(2):
            coeff = tq[comp] / mu
            assert abs(coeff - C[3 + comp, 3 + col]) < 1e-4 * np.abs(C[3:5, 3:5]).max(), \
                (comp, col, coeff, C[3 + comp, 3 + col])
