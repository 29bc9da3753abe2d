"""Pins of the oracle's user-defined polynomial potential.

A run may bring its own model potential (the paper's programs take the model
as a file with the potential and its derivatives, "Overview" section).  The
polynomial model V(phi) = sum_t coef_t prod_i phi_i^e_ti becomes, in the
program variables f = a phi, sum_t coef_t a^(4 - D_t) prod_i f_i^e_ti.  The
oracle evaluates it by that definition; these tests tie it to things fixed
independently of that code:
  - the quartic family written as polynomial terms reproduces the quartic
    oracle (itself pinned by closed forms and RK4) through whole runs,
    with masses, a vacuum energy and expansion;
  - the program-variable potential obeys V_pr(f; a) = a^4 V(f/a) for terms
    of every degree up to 8;
  - dV/df agrees with central differences of V at second order;
  - a homogeneous phi^6 field follows an RK4 integration of its ODE (static
    and with expansion) at second order;
  - a polynomial mass term alone follows the exact discrete dispersion;
  - energy is conserved to O(dt^2) for a model with phi^6 and trilinear terms.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams, dpotential_point, potential_point

KAPPA = 8.0 * np.pi * 0.342 ** 2


def quartic_as_terms(lam, G, mu2, vacuum, nfields):
    terms = [(0.25 * lam, (4, 0, 0))]
    for j in range(1, nfields):
        e = [2, 0, 0]
        e[j] = 2
        terms.append((0.5 * G[j], tuple(e)))
    for i in range(nfields):
        e = [0, 0, 0]
        e[i] = 2
        terms.append((0.5 * mu2[i], tuple(e)))
    terms.append((vacuum, (0, 0, 0)))
    return terms


@pytest.mark.parametrize("expansion", [False, True])
def test_quartic_family_written_as_terms_reproduces_the_quartic_oracle(expansion):
    rng = np.random.default_rng(11)
    G, mu2, vac = (0.0, 80.0, 300.0), (0.4, -0.2, 0.7), 0.3
    q = OracleParams(dims=3, N=8, nfields=3, L=2.5, dt=0.01, G=G, mu2=mu2, vacuum=vac, expansion=expansion,
                     kappa=KAPPA)
    p = OracleParams(dims=3, N=8, nfields=3, L=2.5, dt=0.01, lam=0.0, expansion=expansion, kappa=KAPPA,
                     terms=quartic_as_terms(1.0, G, mu2, vac, 3))
    phi = np.concatenate([1.0 + 1e-2 * rng.standard_normal((1, 8, 8, 8)), 1e-2 * rng.standard_normal((2, 8, 8, 8))])
    phid = 1e-2 * rng.standard_normal((3, 8, 8, 8))
    a, b = Oracle(q, phi, phid), Oracle(p, phi, phid)
    a.step(120)
    b.step(120)
    for i in range(3):
        scale = np.sqrt(np.mean(a.f[i] ** 2))
        assert np.max(np.abs(a.f[i] - b.f[i])) <= 1e-12 * scale
        assert np.max(np.abs(a.pi[i] - b.pi[i])) <= 1e-11 * max(np.sqrt(np.mean(a.pi[i] ** 2)), scale)
    for x, y in zip(a.log, b.log):
        for k in ("a", "rho", "pot", "adot"):
            assert abs(getattr(x, k) - getattr(y, k)) <= 1e-12 * max(abs(getattr(x, k)), abs(x.rho))


RANDOM_TERMS = [(0.7, (6, 0, 0)), (-1.3, (3, 2, 0)), (0.4, (1, 1, 1)), (2.1, (0, 4, 4)), (-0.5, (2, 0, 1)),
                (0.9, (0, 0, 3)), (1.5, (0, 0, 0)), (0.25, (5, 0, 3))]


def test_program_variables_scale_as_a_to_the_4_minus_degree():
    """V_pr(f; a) = a^4 V(f / a): the polynomial written in f = a phi."""
    p = OracleParams(dims=1, N=4, nfields=3, L=1.0, dt=0.01, lam=0.0, terms=RANDOM_TERMS)
    rng = np.random.default_rng(3)
    for _ in range(20):
        v = rng.uniform(-1.5, 1.5, 3)
        a = rng.uniform(0.3, 3.0)
        lhs = potential_point(p, v, a)
        rhs = a ** 4 * potential_point(p, v / a, 1.0)
        assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))
        # and term by term against the defining sum at a = 1
        ref = sum(c * np.prod([v[i] ** e[i] for i in range(3)]) for c, e in RANDOM_TERMS)
        assert abs(potential_point(p, v, 1.0) - ref) <= 1e-12 * max(1.0, abs(ref))


def test_derivative_is_the_derivative_of_the_potential():
    p = OracleParams(dims=1, N=4, nfields=3, L=1.0, dt=0.01, lam=0.0, terms=RANDOM_TERMS)
    rng = np.random.default_rng(4)
    for _ in range(10):
        v = rng.uniform(-1.2, 1.2, 3)
        a = rng.uniform(0.5, 2.0)
        for i in range(3):
            errs = []
            for h in (1e-3, 5e-4):
                e = np.zeros(3)
                e[i] = h
                fd = (potential_point(p, v + e, a) - potential_point(p, v - e, a)) / (2 * h)
                errs.append(abs(fd - dpotential_point(p, v, a, i)))
            assert errs[0] < 1e-4
            assert 3.0 < errs[0] / max(errs[1], 1e-300) < 5.0 or errs[0] < 1e-10  # second order


def _rk4(V, dV, kappa, f0, v0, tau, h, expansion):
    """Homogeneous field + scale factor in the program variables, RK4:
    f'' = -dV/df(f; a) + (a''/a) f and a'' = -a'^2/a + kappa V(f; a)/a, with
    a'(0) = sqrt(kappa rho_0 / 3) (radiation-like start) when expanding."""
    rho0 = 0.5 * v0 * v0 + V(f0, 1.0)
    ap = np.sqrt(kappa * rho0 / 3.0) if expansion else 0.0
    y = np.array([f0, v0 + ap * f0, 1.0, ap])

    def rhs(y):
        f, fp, a, apr = y
        app = (-apr * apr / a + kappa * V(f, a) / a) if expansion else 0.0
        return np.array([fp, -dV(f, a) + app / a * f, apr, app])

    for _ in range(int(round(tau / h))):
        k1 = rhs(y)
        k2 = rhs(y + 0.5 * h * k1)
        k3 = rhs(y + 0.5 * h * k2)
        k4 = rhs(y + h * k3)
        y = y + h / 6.0 * (k1 + 2 * k2 + 2 * k3 + k4)
    return y


@pytest.mark.parametrize("expansion", [False, True])
def test_homogeneous_phi6_matches_rk4(expansion):
    # V = g phi^6 / 6 + m^2 phi^2 / 2: degree 6 (a^-2) and degree 2 (a^2)
    g, m2 = 0.8, 0.3
    terms = [(g / 6.0, (6, 0, 0)), (0.5 * m2, (2, 0, 0))]
    V = lambda f, a: g / 6.0 * f ** 6 / a ** 2 + 0.5 * m2 * a * a * f * f
    dV = lambda f, a: g * f ** 5 / a ** 2 + m2 * a * a * f
    tau = 3.0
    ref = _rk4(V, dV, KAPPA, 1.2, 0.1, tau, 1e-4, expansion)
    errs = []
    for dt in (0.01, 0.005):
        p = OracleParams(dims=2, N=4, nfields=1, L=1.0, dt=dt, lam=0.0, expansion=expansion, kappa=KAPPA,
                         terms=terms)
        orc = Oracle(p, np.full((1, 4, 4), 1.2), np.full((1, 4, 4), 0.1))
        orc.step(int(round(tau / dt)), record=False)
        f = orc.f[0]
        assert np.all(f == f.flat[0])  # homogeneous stays homogeneous, bitwise
        errs.append((abs(f.flat[0] - ref[0]), abs(orc.state.a - ref[2])))
    assert errs[0][0] < 5e-4 and errs[0][1] < 5e-4
    assert 3.3 < errs[0][0] / errs[1][0] < 4.7  # second order in f
    if expansion:
        assert 3.3 < errs[0][1] / errs[1][1] < 4.7  # and in a


def test_polynomial_mass_term_follows_exact_dispersion():
    m2, dt, L, N, A = 0.7, 0.05, 6.0, 16, 0.3
    p = OracleParams(dims=2, N=N, nfields=1, L=L, dt=dt, lam=0.0, terms=[(0.5 * m2, (2, 0, 0))])
    idx = np.indices((N, N))
    n = (3, 5)
    f0 = A * np.cos(2 * np.pi * (n[0] * idx[0] + n[1] * idx[1]) / N)
    orc = Oracle(p, f0[None], np.zeros((1, N, N)))
    dx = L / N
    w2 = m2 + (4.0 / dx ** 2) * sum(np.sin(np.pi * k / N) ** 2 for k in n)
    wt = 2.0 / dt * np.arcsin(np.sqrt(w2) * dt / 2.0)
    for k in range(1, 301):
        orc.step(1, record=False)
        assert np.max(np.abs(orc.f[0] - f0 * np.cos(wt * k * dt))) < 1e-12


def test_energy_conserved_at_second_order_with_sixth_order_and_trilinear_terms():
    terms = [(0.25, (4, 0, 0)), (0.05, (6, 0, 0)), (40.0, (2, 2, 0)), (0.8, (1, 2, 0)), (0.3, (0, 2, 0))]
    rng = np.random.default_rng(8)
    phi = np.concatenate([1.0 + 0.02 * rng.standard_normal((1, 12, 12, 12)),
                          0.02 * rng.standard_normal((1, 12, 12, 12))])
    phid = 0.02 * rng.standard_normal((2, 12, 12, 12))
    drift = []
    for dt in (0.02, 0.01):
        p = OracleParams(dims=3, N=12, nfields=2, L=3.0, dt=dt, lam=0.0, terms=terms)
        orc = Oracle(p, phi, phid)
        orc.step(int(round(2.0 / dt)))
        rho = np.array([s.rho for s in orc.log])
        drift.append(np.max(np.abs(rho - rho[0])) / abs(rho[0]))
    # omega dt reaches ~0.2 for the chi mass at dt = 0.02: the bound is on
    # the order, not on the size
    assert drift[0] < 1e-2
    assert 3.0 < drift[0] / drift[1] < 5.0
