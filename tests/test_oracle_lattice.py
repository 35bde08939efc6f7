"""Pins of the oracle's kinetic model (paper Sec. II.C) against the
continuous Maxwell-Boltzmann moments, collision invariants and fixed points.

The reference moments are Gauss-Hermite integrals of the 2D Maxwellian with
C_v - 1 internal degrees of freedom per unit R; nothing here reuses the
oracle's formulas.
"""

import numpy as np
import pytest

from oracle import lattice as L

GAMMAS = (1.4, 5.0 / 3.0, 1.3)


def maxwell_moments(rho, ux, uy, T, gamma, order=12):
    """Moments of rho/(2 pi T) exp(-|v-u|^2/(2T)) by tensor Gauss-Hermite
    quadrature, for the f set (weight 1) and the g set (weight
    |v|^2 + 2 (C_v - 1) T, i.e. twice the total energy per particle)."""
    Cv = 1.0 / (gamma - 1.0)
    z, w = np.polynomial.hermite_e.hermegauss(order)
    w = w / np.sqrt(2.0 * np.pi)
    vx = ux + np.sqrt(T) * z[:, None]
    vy = uy + np.sqrt(T) * z[None, :]
    W = rho * w[:, None] * w[None, :]
    e2 = vx ** 2 + vy ** 2 + 2.0 * (Cv - 1.0) * T
    m = {}
    for name, weight in (("f", W), ("g", W * e2)):
        m[name + "0"] = weight.sum()
        m[name + "x"] = (weight * vx).sum()
        m[name + "y"] = (weight * vy).sum()
        m[name + "xx"] = (weight * vx * vx).sum()
        m[name + "xy"] = (weight * vx * vy).sum()
        m[name + "yy"] = (weight * vy * vy).sum()
        m[name + "xxx"] = (weight * vx ** 3).sum()
        m[name + "xxy"] = (weight * vx * vx * vy).sum()
        m[name + "xyy"] = (weight * vx * vy * vy).sum()
        m[name + "yyy"] = (weight * vy ** 3).sum()
    return m


def lattice_moments(pop):
    m = {}
    cx = np.array(L.CX, dtype=float)
    cy = np.array(L.CY, dtype=float)
    m["0"] = pop.sum()
    m["x"] = (pop * cx).sum()
    m["y"] = (pop * cy).sum()
    m["xx"] = (pop * cx * cx).sum()
    m["xy"] = (pop * cx * cy).sum()
    m["yy"] = (pop * cy * cy).sum()
    m["xxx"] = (pop * cx ** 3).sum()
    m["xxy"] = (pop * cx * cx * cy).sum()
    m["xyy"] = (pop * cx * cy * cy).sum()
    m["yyy"] = (pop * cy ** 3).sum()
    return m


def random_states(n=25, seed=7):
    rng = np.random.default_rng(seed)
    for _ in range(n):
        rho = rng.uniform(0.5, 2.0)
        T = rng.uniform(0.15, 0.6)
        umax = np.sqrt(max(1.0 - T, 0.0)) * 0.6
        ux, uy = rng.uniform(-umax, umax, 2)
        gamma = GAMMAS[rng.integers(len(GAMMAS))]
        yield rho, ux, uy, T, gamma


@pytest.mark.parametrize("state", list(random_states()))
def test_feq_moments_match_maxwellian_up_to_lattice_defect(state):
    """P1: zeroth, first, second and the mixed third moments of f^eq are the
    Maxwellian ones; the diagonal third moment is rho u (the D2Q9 defect) and
    the oracle's delta Q is exactly lattice minus Maxwellian."""
    rho, ux, uy, T, gamma = state
    lm = lattice_moments(L.feq(rho, ux, uy, T))
    mm = maxwell_moments(rho, ux, uy, T, gamma)
    for k in ("0", "x", "y", "xx", "xy", "yy", "xxy", "xyy"):
        assert lm[k] == pytest.approx(mm["f" + k], rel=1e-13, abs=1e-14), k
    assert lm["xxx"] == pytest.approx(rho * ux, rel=1e-13, abs=1e-15)
    dQx, dQy = L.momentum_defect(rho, ux, uy, T)
    assert dQx == pytest.approx(lm["xxx"] - mm["fxxx"], rel=1e-12, abs=1e-14)
    assert dQy == pytest.approx(lm["yyy"] - mm["fyyy"], rel=1e-12, abs=1e-14)


@pytest.mark.parametrize("state", list(random_states()))
def test_geq_moments_match_maxwellian(state):
    """P2: sum g^eq = 2 rho E, sum g^eq c = energy flux of the Maxwellian
    (2 rho u H), sum g^eq c c = R^eq of the Maxwellian, for any T and u.
    This pins the enthalpy, the 2 rho E T I term and the Psi placement."""
    rho, ux, uy, T, gamma = state
    Cv = 1.0 / (gamma - 1.0)
    E = Cv * T + 0.5 * (ux * ux + uy * uy)
    lm = lattice_moments(L.geq(rho, ux, uy, E, T))
    mm = maxwell_moments(rho, ux, uy, T, gamma)
    scale = mm["g0"]
    for k in ("0", "x", "y", "xx", "xy", "yy"):
        assert lm[k] == pytest.approx(mm["g" + k], abs=1e-13 * scale), k


def test_psi_is_needed_off_T_one_third():
    """Without Psi the diagonal second moment of g^eq is wrong unless T = 1/3."""
    rho, ux, uy, T, gamma = 1.1, 0.2, -0.1, 0.2, 1.4
    E = T / (gamma - 1) + 0.5 * (ux * ux + uy * uy)
    g_with = L.geq(rho, ux, uy, E, T)
    g_without = g_with - L.energy_correction(rho, ux, uy, E, T)
    mm = maxwell_moments(rho, ux, uy, T, gamma)
    assert lattice_moments(g_with)["xx"] == pytest.approx(mm["gxx"], rel=1e-13)
    assert abs(lattice_moments(g_without)["xx"] - mm["gxx"]) > 1e-3
    # and at T = 1/3 Psi vanishes identically
    T3 = 1.0 / 3.0
    E3 = T3 / (gamma - 1) + 0.5 * (ux * ux + uy * uy)
    assert np.max(np.abs(L.energy_correction(rho, ux, uy, E3, T3))) < 1e-15


def near_equilibrium_populations(rho, ux, uy, T, gamma, rng, eps=1e-3):
    Cv = 1.0 / (gamma - 1.0)
    E = Cv * T + 0.5 * (ux * ux + uy * uy)
    f = L.feq(rho, ux, uy, T)
    g = L.geq(rho, ux, uy, E, T)
    # perturbations that keep rho, rho u and 2 rho E (non-equilibrium parts)
    df = rng.normal(size=9) * eps
    dg = rng.normal(size=9) * eps
    cx = np.array(L.CX, float)
    cy = np.array(L.CY, float)
    basis = np.stack([np.ones(9), cx, cy])
    proj = basis.T @ np.linalg.solve(basis @ basis.T, basis @ df)
    df -= proj
    dg -= np.ones(9) * dg.mean()
    return f + df, g + dg


@pytest.mark.parametrize("seed", range(8))
def test_collision_invariants_and_relaxation(seed):
    """P3: mass and energy are conserved, momentum changes by -dt F; the stress
    relaxes with omega, the energy-flux moment R with omega_1, and the heat flux
    splits into a part relaxing with omega_1 and a viscous-heating part
    2 u.(P - P^eq) relaxing with omega (reading of q^*)."""
    rng = np.random.default_rng(seed)
    rho = rng.uniform(0.7, 1.5)
    T = rng.uniform(0.18, 0.5)
    ux, uy = rng.uniform(-0.25, 0.25, 2)
    gamma = GAMMAS[seed % len(GAMMAS)]
    mu, Pr, dt = rng.uniform(0.005, 0.1), rng.uniform(0.5, 2.0), rng.uniform(0.2, 1.0)
    f, g = near_equilibrium_populations(rho, ux, uy, T, gamma, rng)
    Fx, Fy = rng.normal(size=2) * 1e-3
    fpost, gpost = L.collide(f[:, None], g[:, None], gamma, mu, Pr, dt,
                             np.array([Fx]), np.array([Fy]))
    fpost, gpost = fpost[:, 0], gpost[:, 0]
    lf, lf2 = lattice_moments(f), lattice_moments(fpost)
    lg, lg2 = lattice_moments(g), lattice_moments(gpost)
    assert lf2["0"] == pytest.approx(lf["0"], rel=1e-14)
    assert lg2["0"] == pytest.approx(lg["0"], rel=1e-14)
    assert lf2["x"] == pytest.approx(lf["x"] - dt * Fx, abs=1e-14)
    assert lf2["y"] == pytest.approx(lf["y"] - dt * Fy, abs=1e-14)

    omega = 1.0 / (mu / (rho * T * dt) + 0.5)
    omega1 = 1.0 / ((1.0 / omega - 0.5) / Pr + 0.5)
    mm = maxwell_moments(rho, ux, uy, T, gamma)
    # f stress: P' - P^eq = (1 - omega)(P - P^eq) (phi has no second moment)
    for k in ("xx", "xy", "yy"):
        assert lf2[k] - mm["f" + k] == pytest.approx((1 - omega) * (lf[k] - mm["f" + k]),
                                                     abs=1e-14)
    # g second moment: g^eq and g^* share R^eq, so R relaxes with omega_1
    for k in ("xx", "xy", "yy"):
        assert lg2[k] - mm["g" + k] == pytest.approx((1 - omega1) * (lg[k] - mm["g" + k]),
                                                     abs=1e-13)
    # heat flux
    dP = {k: lf[k] - mm["f" + k] for k in ("xx", "xy", "yy")}
    visc = (2 * (ux * dP["xx"] + uy * dP["xy"]), 2 * (ux * dP["xy"] + uy * dP["yy"]))
    for a, k in enumerate(("x", "y")):
        neq = lg[k] - mm["g" + k]
        expect = (1 - omega1) * (neq - visc[a]) + (1 - omega) * visc[a]
        assert lg2[k] - mm["g" + k] == pytest.approx(expect, abs=1e-13)


def test_phi_moments():
    """P3: sum phi = 0, sum phi c = -F, sum phi c c = 0."""
    rng = np.random.default_rng(3)
    for _ in range(10):
        T = rng.uniform(0.1, 0.7)
        F = rng.normal(size=2)
        phi = L.momentum_correction(F[0], F[1], T)
        lm = lattice_moments(phi)
        assert abs(lm["0"]) < 1e-14
        assert lm["x"] == pytest.approx(-F[0], abs=1e-14)
        assert lm["y"] == pytest.approx(-F[1], abs=1e-14)
        for k in ("xx", "xy", "yy"):
            assert abs(lm[k]) < 1e-14


@pytest.mark.parametrize("T", [1.0 / 3.0, 0.2, 0.45])
def test_uniform_state_is_fixed_point(T):
    """P4: a uniform equilibrium with F = 0 is unchanged by the collision."""
    rho, ux, uy, gamma = 1.3, 0.12, -0.07, 1.4
    Cv = 1.0 / (gamma - 1.0)
    E = Cv * T + 0.5 * (ux * ux + uy * uy)
    f = L.feq(rho, ux, uy, T)[:, None]
    g = L.geq(rho, ux, uy, E, T)[:, None]
    fp, gp = L.collide(f, g, gamma, 0.02, 0.71, 0.5, np.zeros(1), np.zeros(1))
    assert np.max(np.abs(fp - f)) < 1e-15 * np.max(np.abs(f)) * 4
    assert np.max(np.abs(gp - g)) < 1e-15 * np.max(np.abs(g)) * 4


def test_macroscopic_roundtrip():
    rho, ux, uy, T, gamma = 0.9, -0.2, 0.15, 0.27, 1.4
    f, g = L.equilibrium_populations(np.array(rho), np.array(ux), np.array(uy),
                                     np.array(T), gamma)
    r, u, v, E, TT = L.macroscopic(f, g, gamma)
    assert (r, u, v, TT) == pytest.approx((rho, ux, uy, T), rel=1e-14)


@pytest.mark.parametrize("bad", [dict(T=1.0), dict(T=0.9, ux=0.4), dict(rho=-1.0),
                                 dict(T=-0.1), dict(rho=np.nan)])
def test_positivity_domain_raises(bad):
    """P5: states outside the D2Q9 positivity domain are rejected."""
    s = dict(rho=1.0, ux=0.0, uy=0.0, T=1.0 / 3.0)
    s.update(bad)
    with pytest.raises(L.NonPhysicalState):
        L.check_state(np.array([s["rho"]]), np.array([s["ux"]]), np.array([s["uy"]]),
                      np.array([s["T"]]))
