"""Pins of the oracle's tachyonic / hybrid potentials (negative mass terms
and the vacuum energy a^4 V0) against closed forms and independent RK4
integrations of the homogeneous equations."""
import numpy as np
import pytest

from oracle import Oracle, OracleParams

KAPPA = 8.0 * np.pi * 0.342 ** 2


def test_de_sitter_closed_form():
    # no field: rho = a^4 V0, a' = H a^2 with H = sqrt(kappa V0 / 3), so
    # a(tau) = 1 / (1 - H tau) exactly
    V0, tau = 0.1, 1.5
    H = np.sqrt(KAPPA * V0 / 3.0)
    a_ex = 1.0 / (1.0 - H * tau)
    errs = []
    for dt in (0.01, 0.005):
        p = OracleParams(dims=3, N=4, nfields=1, L=1.0, dt=dt, lam=1.0, expansion=True, kappa=KAPPA,
                         vacuum=V0)
        orc = Oracle(p, np.zeros((1, 4, 4, 4)), np.zeros((1, 4, 4, 4)))
        assert orc.state.adot == pytest.approx(H, rel=1e-15)
        assert orc.state.pot == pytest.approx(V0, rel=1e-15) and orc.state.rho == pytest.approx(V0, rel=1e-15)
        st = orc.step(int(round(tau / dt)), record=False)
        errs.append(abs(st.a - a_ex))
        assert st.pot == pytest.approx(V0 * st.a ** 4, rel=1e-14)
        assert abs(st.resid) < 1e-4
    assert a_ex > 1.8
    assert errs[0] < 1e-4 and 3.3 < errs[0] / errs[1] < 4.7


def _rk4(f0, v0, tau, h, lam, mu2, V0, kappa, expansion):
    """Homogeneous f with the double-well potential in conformal program
    variables: V = lam/4 f^4 + a^2 mu2/2 f^2 + a^4 V0."""
    def pot(f, a):
        return 0.25 * lam * f ** 4 + 0.5 * a * a * mu2 * f * f + a ** 4 * V0

    ap = np.sqrt(kappa * (0.5 * v0 * v0 + pot(f0, 1.0)) / 3.0) if expansion else 0.0
    y = np.array([f0, v0 + ap * f0, 1.0, ap])

    def rhs(y):
        f, fp, a, apr = y
        app = (-apr * apr / a + kappa * pot(f, a) / a) if expansion else 0.0
        return np.array([fp, -(lam * f ** 3 + a * a * mu2 * f) + app / a * f, apr, app])

    for _ in range(int(round(tau / h))):
        k1 = rhs(y); k2 = rhs(y + 0.5 * h * k1); k3 = rhs(y + 0.5 * h * k2); k4 = rhs(y + h * k3)
        y = y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


def test_double_well_static():
    # lam/4 (f^2 - v^2)^2 with v = 1: mu2 = -1, V0 = 1/4; inside one well
    lam, mu2, V0, f0, tau = 1.0, -1.0, 0.25, 0.2, 6.0
    E = 0.25 * lam * (f0 * f0 - 1.0) ** 2
    ref = _rk4(f0, 0.0, tau, 1e-4, lam, mu2, V0, KAPPA, False)
    errs, drift = [], []
    for dt in (0.01, 0.005):
        p = OracleParams(dims=2, N=4, nfields=1, L=1.0, dt=dt, lam=lam, mu2=(mu2,), vacuum=V0)
        orc = Oracle(p, np.full((1, 4, 4), f0), np.zeros((1, 4, 4)))
        orc.step(int(round(tau / dt)))
        errs.append(abs(orc.f[0, 0, 0] - ref[0]))
        # the energy including the vacuum term is the conserved double-well energy
        drift.append(max(abs(s.rho - E) for s in orc.log[1:]))
    assert ref[0] > 0.0   # stayed in the right-hand well
    assert errs[0] < 1e-4 and 3.3 < errs[0] / errs[1] < 4.7
    assert drift[0] < 1e-4 and 3.3 < drift[0] / drift[1] < 4.7


def test_tachyonic_expanding():
    lam, mu2, V0, f0, v0, tau = 1.0, -1.0, 0.25, 0.3, 0.1, 3.0
    ref = _rk4(f0, v0, tau, 1e-4, lam, mu2, V0, KAPPA, True)
    ef, ea, res = [], [], []
    for dt in (0.01, 0.005):
        p = OracleParams(dims=3, N=4, nfields=1, L=1.0, dt=dt, lam=lam, mu2=(mu2,), vacuum=V0, expansion=True,
                         kappa=KAPPA)
        orc = Oracle(p, np.full((1, 4, 4, 4), f0), np.full((1, 4, 4, 4), v0))
        st = orc.step(int(round(tau / dt)), record=False)
        ef.append(abs(orc.f[0].flat[0] - ref[0]))
        ea.append(abs(st.a - ref[2]))
        res.append(abs(st.resid))
    assert ref[2] > 1.5
    assert ef[0] < 1e-3 and ea[0] < 1e-3 and res[0] < 2e-4
    for e in (ef, ea, res):
        assert 3.3 < e[0] / e[1] < 4.7
