"""The GPU's rewriting of the step, replayed in FP64 NumPy against the oracle.

The device kernels do not store f and its half-step derivative as the
paper's order does.  They keep each field as an FP64 homogeneous reference
m plus a stored deviation d, and store p = fdot - beta f, where the c = a''/a
term of the kick (beta = dt c) is added one pass later, once the volume sums
that fix c are known.  This test restates that algebra (start-up pass, step
pass and the FP64 scalar tail, in the order the kernels use) with NumPy in
FP64, and checks that it reproduces the oracle's plain leapfrog per site and
in every diagnostic: the rewriting is exact up to rounding, in every model
the library accepts.  It needs no GPU and shares no code with either side.
"""
import numpy as np
import pytest

from oracle import Oracle, OracleParams, grf_initial

KAPPA = 8.0 * np.pi * 0.342 ** 2


def lap(g, dx):
    out = -2.0 * g.ndim * g
    for ax in range(g.ndim):
        out = out + (np.roll(g, 1, ax) + np.roll(g, -1, ax))
    return out / (dx * dx)


def dpot(v, i, p, a2):
    """dV/df_i at field values v (list of arrays), mass terms times a2."""
    G = p.G
    if i == 0:
        chi2 = sum(G[j] * v[j] * v[j] for j in range(1, p.nfields))
        out = p.lam * v[0] ** 3 + v[0] * chi2
    else:
        out = G[i] * v[0] * v[0] * v[i]
    return out + a2 * p.mu2[i] * v[i]


def pot(v, p, a2):
    out = 0.25 * p.lam * v[0] ** 4
    for j in range(1, p.nfields):
        out = out + 0.5 * p.G[j] * v[0] ** 2 * v[j] ** 2
    for i in range(p.nfields):
        out = out + 0.5 * a2 * p.mu2[i] * v[i] ** 2
    return out


class Deferred:
    """State (m_i, d_i, p_i) and the FP64 scalars of one lattice."""

    def __init__(self, p: OracleParams, phi, phidot):
        self.p = p
        nf, dt = p.nfields, p.dt
        self.dx = p.L / p.N
        Ns = float(p.N ** p.dims)
        # any reference works; the volume mean keeps d small
        self.m = [float(phi[i].mean()) for i in range(nf)]
        self.d = [phi[i] - self.m[i] for i in range(nf)]
        # start-up pass: derivative unchanged, half kick without the f terms
        v = [self.m[i] + self.d[i] for i in range(nf)]
        lp = [lap(self.d[i], self.dx) for i in range(nf)]
        self.p_ = [phidot[i] + 0.5 * dt * (lp[i] - dpot(v, i, p, 1.0)) for i in range(nf)]
        kin = [0.5 * np.sum(phidot[i] ** 2) / Ns for i in range(nf)]
        grad = [-0.5 * np.sum(self.d[i] * lp[i]) / Ns for i in range(nf)]
        V = np.sum(pot(v, p, 1.0)) / Ns + p.vacuum
        rho = sum(kin) + sum(grad) + V
        ap0 = np.sqrt(p.kappa * rho / 3.0) if p.expansion else 0.0
        app0 = (-ap0 * ap0 + p.kappa * (2.0 / 3.0 * sum(grad) + V)) if p.expansion else 0.0
        aph = ap0 + 0.5 * dt * app0
        self.beta = aph                       # a'(0) + dt/2 a''(0)
        mean = [self.m[i] + np.sum(self.d[i]) / Ns for i in range(nf)]
        self.fdot_mean = [np.sum(self.p_[i]) / Ns + self.beta * mean[i] for i in range(nf)]
        self.r = list(self.fdot_mean)
        self.a, self.y = 1.0, aph
        self.a_next = 1.0 + dt * aph if p.expansion else 1.0
        mean_sq = [(Ns * self.m[i] ** 2 + 2.0 * self.m[i] * np.sum(self.d[i]) + np.sum(self.d[i] ** 2)) / Ns
                   for i in range(nf)]
        self.log = [dict(a=1.0, adot=ap0, kin=kin, grad=grad, pot=V, rho=rho, mean=mean, mean_sq=mean_sq)]

    def f(self):
        return np.stack([self.m[i] + self.d[i] for i in range(self.p.nfields)])

    def pi(self):
        return np.stack([self.p_[i] + self.beta * (self.m[i] + self.d[i]) for i in range(self.p.nfields)])

    def step(self):
        p, nf, dt = self.p, self.p.nfields, self.p.dt
        Ns = float(p.N ** p.dims)
        a1 = self.a_next
        m1 = [self.m[i] + dt * self.r[i] for i in range(nf)]
        fdot = [self.beta * self.d[i] + self.p_[i] + self.beta * self.m[i] for i in range(nf)]
        d1 = [self.d[i] + dt * (fdot[i] - self.r[i]) for i in range(nf)]
        v = [m1[i] + d1[i] for i in range(nf)]
        lp = [lap(d1[i], self.dx) for i in range(nf)]
        pn = [fdot[i] + dt * (lp[i] - dpot(v, i, p, a1 * a1)) for i in range(nf)]
        ub = [0.5 * (fdot[i] + pn[i]) for i in range(nf)]
        t = [(np.sum(d1[i]), np.sum(d1[i] ** 2), np.sum(d1[i] * lp[i]), np.sum(ub[i] ** 2), np.sum(ub[i]),
              np.sum(ub[i] * d1[i])) for i in range(nf)]
        sumf2 = [Ns * m1[i] ** 2 + 2.0 * m1[i] * t[i][0] + t[i][1] for i in range(nf)]
        mean = [m1[i] + t[i][0] / Ns for i in range(nf)]
        grad = [-0.5 * t[i][2] / Ns for i in range(nf)]
        V = np.sum(pot(v, p, a1 * a1)) / Ns + a1 ** 4 * p.vacuum
        x = abar = c = 0.0
        y = self.y
        if p.expansion:
            S = p.kappa * (2.0 / 3.0 * sum(grad) + V) / a1
            A, B = dt / (4.0 * a1), 1.0 + dt * y / (2.0 * a1)
            C = dt * y * y / (4.0 * a1) - y - dt * S
            x = -2.0 * C / (B + np.sqrt(B * B - 4.0 * A * C))
            abar = 0.5 * (x + y)
            c = (S - abar * abar / a1) / a1
        beta1 = dt * c
        eta = 0.5 * dt * c - abar / a1
        kin = [0.5 * (t[i][3] + 2.0 * eta * (m1[i] * t[i][4] + t[i][5]) + eta * eta * sumf2[i]) / Ns
               for i in range(nf)]
        self.fdot_mean = [2.0 * t[i][4] / Ns - self.fdot_mean[i] + beta1 * mean[i] for i in range(nf)]
        self.r = list(self.fdot_mean)
        self.m, self.d, self.p_ = m1, d1, pn
        self.a, self.y, self.beta = a1, x, beta1
        self.a_next = a1 + dt * x if p.expansion else 1.0
        self.log.append(dict(a=a1, adot=abar, kin=kin, grad=grad, pot=V, rho=sum(kin) + sum(grad) + V,
                             mean=mean, mean_sq=[sumf2[i] / Ns for i in range(nf)]))


CASES = [
    ("3d_two_fields_expanding", OracleParams(3, 8, 2, 10.0 * 8 / 32, 0.01, G=(0.0, 100.0), expansion=True,
                                             kappa=KAPPA), (1.0, 100.0)),
    ("3d_two_fields_static", OracleParams(3, 8, 2, 2.5, 0.01, G=(0.0, 100.0)), (1.0, 100.0)),
    ("2d_three_fields_masses", OracleParams(2, 16, 3, 5.0, 0.01, G=(0.0, 40.0, 900.0), mu2=(0.3, 0.1, 0.0),
                                            expansion=True, kappa=KAPPA), (1.3, 40.0, 900.0)),
    ("1d_tachyonic_vacuum", OracleParams(1, 32, 1, 10.0, 0.01, mu2=(-1.0,), vacuum=0.25, expansion=True,
                                         kappa=0.05), (1.0,)),
]


@pytest.mark.parametrize("name,params,m_eff2", CASES, ids=[c[0] for c in CASES])
def test_deferred_split_form_reproduces_the_oracle(name, params, m_eff2):
    bg = (0.2, 0.0, 0.0) if params.vacuum else (1.0, 0.0, 0.0)
    phi, phid = grf_initial(7, params.dims, params.N, params.L, params.nfields, m_eff2, amp=1e-2,
                            background=bg)
    orc = Oracle(params, phi, phid)
    rep = Deferred(params, phi, phid)
    steps = 50
    orc.step(steps)
    for _ in range(steps):
        rep.step()
    for i in range(params.nfields):
        for got, want in ((rep.f()[i], orc.f[i]), (rep.pi()[i], orc.pi[i])):
            scale = max(np.sqrt(np.mean(want ** 2)), 1e-300)
            err = np.max(np.abs(got - want) / np.maximum(np.abs(want), scale))
            assert err <= 1e-12, (name, i, err)
    for k, (g, o) in enumerate(zip(rep.log, orc.log)):
        # energies relative to the total energy density, means to each
        # field's rms (a fluctuation field's mean is rounding noise)
        e_scale = abs(o.rho)
        pairs = [(g["a"], o.a, abs(o.a)), (g["rho"], o.rho, e_scale), (g["pot"], o.pot, e_scale)]
        if params.expansion:
            pairs.append((g["adot"], o.adot, abs(o.adot)))
        pairs += [(x, y, e_scale) for x, y in zip(g["kin"] + g["grad"], o.kin + o.grad)]
        pairs += [(x, y, np.sqrt(sq)) for x, y, sq in zip(g["mean"], o.mean, o.mean_sq)]
        pairs += [(x, y, abs(y)) for x, y in zip(g["mean_sq"], o.mean_sq)]
        for x, y, scale in pairs:
            assert abs(x - y) <= 1e-12 * max(abs(y), scale), (name, k, x, y)
