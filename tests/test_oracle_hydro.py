"""Hydrodynamic pins of the oracle: the Navier-Stokes-Fourier behaviour the
paper's Chapman-Enskog analysis fixes (Sec. II.C: mu = (1/omega - 1/2) p dt,
kappa = C_p (1/omega_1 - 1/2) p dt, P = p I - mu[grad u + grad u^T -
(1/C_v)(div u) I], c_s = sqrt(gamma T)).

Linear waves on a periodic mesh decay at rates given by those coefficients;
off T = 1/3 the rates are only right with both correction terms (phi for the
stress, Psi for the heat flux), which the mutation tests show.  The acoustic
pulse is compared with the closed-form 2D linear-acoustics solution.
"""

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import j0

import synth
import oracle.lattice as L
import oracle.solver as OS
from oracle.solver import OracleSolver


def wave_rate(kind, T0=1.0 / 3.0, dt=1.0, nu=0.05, N=64, steps=300, gamma=1.4,
              Pr=0.71, amp=1e-4, correction=True):
    """Measured (decay rate, angular frequency) of one Fourier mode."""
    mesh = synth.cartesian_mesh(N, 4)
    fluid = synth.FluidParams(gamma=gamma, Pr=Pr, mu=nu, rho_inf=1.0, T_inf=T0,
                              u_inf=(0.0, 0.0), dt=dt)
    k = 2 * np.pi / N
    x = mesh.X
    cs = np.sqrt(gamma * T0)
    rho = np.ones_like(x)
    ux = np.zeros_like(x)
    uy = np.zeros_like(x)
    T = np.full_like(x, T0)
    if kind == "shear":
        uy = amp * np.sin(k * x)
    elif kind == "thermal":          # entropy mode at constant pressure
        T = T0 * (1 + amp * np.cos(k * x))
        rho = T0 / T
    elif kind == "sound":            # right-running isentropic wave
        d = amp * np.cos(k * x)
        rho = 1 + d
        ux = cs * d
        T = T0 * (1 + (gamma - 1) * d)
    s = OracleSolver(mesh, fluid, [], rho, ux, uy, T, correction=correction)
    e = np.exp(-1j * k * x[0])
    hist = []
    for _ in range(steps):
        r, u, v, E, TT = s.macroscopic()
        pp = r[0] * TT[0]
        if kind == "shear":
            field = v[0]
        elif kind == "thermal":      # entropy variable: zero on acoustic modes
            field = (pp - T0) / T0 - gamma * (r[0] - 1.0)
        else:                        # right-running characteristic variable
            field = (pp - T0) / cs + u[0]
        hist.append((field * e).mean())
        s.step()
    hist = np.array(hist)
    t = np.arange(steps) * dt
    w = slice(steps // 3, None)
    rate = -np.polyfit(t[w], np.log(np.abs(hist[w])), 1)[0]
    omega = -np.polyfit(t[w], np.unwrap(np.angle(hist[w])), 1)[0]
    return rate, omega


def nsf_rates(kind, T0, nu, N=64, gamma=1.4, Pr=0.71):
    k = 2 * np.pi / N
    Cv = 1 / (gamma - 1)
    chi = nu / Pr                    # thermal diffusivity kappa / (rho C_p)
    if kind == "shear":
        return nu * k * k, 0.0
    if kind == "thermal":
        return chi * k * k, 0.0
    return 0.5 * k * k * (nu * (2 - 1 / Cv) + (gamma - 1) * chi), np.sqrt(gamma * T0) * k


@pytest.mark.parametrize("T0", [1.0 / 3.0, 0.2])
def test_shear_wave_viscosity(T0):
    """P10: shear-wave decay rate nu k^2 with nu = mu / rho."""
    rate, _ = wave_rate("shear", T0=T0)
    assert rate == pytest.approx(nsf_rates("shear", T0, 0.05)[0], rel=0.01)


@pytest.mark.parametrize("T0,dt", [(1.0 / 3.0, 1.0), (0.2, 1.0), (0.2, 0.5)])
def test_thermal_wave_diffusivity(T0, dt):
    """P11: entropy-wave decay rate chi k^2, chi = (1/omega_1 - 1/2) T dt = nu/Pr."""
    rate, _ = wave_rate("thermal", T0=T0, dt=dt)
    assert rate == pytest.approx(nsf_rates("thermal", T0, 0.05)[0], rel=0.05)


@pytest.mark.parametrize("T0,dt", [(1.0 / 3.0, 1.0), (0.2, 1.0), (0.2, 0.5)])
def test_sound_wave_speed_and_attenuation(T0, dt):
    """P12: sound speed sqrt(gamma T) and attenuation
    (k^2/2)[(2 - 1/C_v) nu + (gamma - 1) chi]."""
    rate, omega = wave_rate("sound", T0=T0, dt=dt)
    exp_rate, exp_omega = nsf_rates("sound", T0, 0.05)
    assert omega == pytest.approx(exp_omega, rel=0.003)
    assert rate == pytest.approx(exp_rate, rel=0.04)


def test_sound_attenuation_fails_without_momentum_correction():
    """Mutation: without phi the bulk stress carries the D2Q9 defect."""
    rate, _ = wave_rate("sound", T0=0.2, correction=False)
    exp_rate, _ = nsf_rates("sound", 0.2, 0.05)
    assert abs(rate / exp_rate - 1) > 0.3


def test_sound_attenuation_fails_without_dt_in_correction(monkeypatch):
    """Mutation: dropping the factor dt from the nested correction
    over-corrects by 1/dt at dt = 1/2."""
    orig = OS.correction_force

    def wrong(grid, f, g, x, y, gamma, mu, Pr, dt):
        Fx, Fy = orig(grid, f, g, x, y, gamma, mu, Pr, dt)
        return Fx / dt, Fy / dt

    monkeypatch.setattr(OS, "correction_force", wrong)
    rate, _ = wave_rate("sound", T0=0.2, dt=0.5)
    exp_rate, _ = nsf_rates("sound", 0.2, 0.05)
    assert abs(rate / exp_rate - 1) > 0.3


def test_heat_diffusivity_fails_without_energy_correction(monkeypatch):
    """Mutation: without Psi the D2Q9 defect of R^eq corrupts kappa off T = 1/3."""
    orig = L.energy_correction
    monkeypatch.setattr(L, "energy_correction", lambda *a: 0.0 * orig(*a))
    rate, _ = wave_rate("thermal", T0=0.2, steps=200)
    assert abs(rate / nsf_rates("thermal", 0.2, 0.05)[0] - 1) > 0.3


def test_unit_cfl_run_conserves_mass_momentum_energy():
    """On the undeformed unit-CFL mesh the scheme is a lattice shift plus a
    conservative collision: sum rho, sum rho u, sum rho E are constant (the
    correction force telescopes to zero over the periodic box)."""
    c = synth.acoustic_pulse_case(amp_mesh=0.0, dt=1.0, nu=0.05)
    fl = synth.configs.replace(c.fluid, u_inf=(0.0, 0.0))
    ux = 0.05 * np.sin(2 * np.pi * c.mesh.Y / 64)
    s = OracleSolver(c.mesh, fl, [], c.rho, ux, c.uy, c.T)
    def totals():
        r, u, v, E, T = s.macroscopic()
        return np.array([r.sum(), (r * u).sum(), (r * v).sum(), (r * E).sum()])
    t0 = totals()
    s.run(20)
    assert np.max(np.abs(totals() - t0) / np.maximum(np.abs(t0), 1.0)) < 1e-12


# ---- P13: acoustic pulse -----------------------------------------------------

def linear_acoustics_pressure(r, t, cs, A=1e-3 / 3, sigma=4.0, nu=0.01, gamma=1.4,
                              Pr=0.71):
    """p'(r, t) = A int_0^inf k sigma^2 exp(-k^2 sigma^2/2) J_0(k r) cos(c k t)
    exp(-Gamma(k) t) dk (Hankel transform of the 2D damped wave equation with
    a Gaussian initial pressure and zero velocity)."""
    Cv = 1 / (gamma - 1)

    def integrand(k):
        G = 0.5 * k * k * (nu * (2 - 1 / Cv) + (gamma - 1) * nu / Pr)
        return (A * sigma * sigma * k * np.exp(-0.5 * k * k * sigma * sigma) * j0(k * r)
                * np.cos(cs * k * t) * np.exp(-G * t))

    return quad(integrand, 0.0, 3.0, limit=400)[0]


def test_acoustic_pulse_matches_linear_acoustics():
    """P13 on the static 64x64 sine-deformed periodic mesh (dt = 1/3):
    pressure peak radius and amplitude follow the closed form with
    c_s = sqrt(gamma T); the pointwise profile error (dominated by the
    dispersion of quadratic semi-Lagrangian interpolation) stays below 20 % of
    the peak, while the isothermal speed sqrt(T) would miss by far more."""
    c = synth.acoustic_pulse_case()
    s = OracleSolver(c.mesh, c.fluid, c.bodies, c.rho, c.ux, c.uy, c.T)
    T0 = 1 / 3
    cs = np.sqrt(1.4 * T0)
    rs = np.linspace(0.0, 100.0, 801)
    for n in range(1, 101):
        s.step()
        if n not in (60, 100):
            continue
        r_, ux, uy, E, T = s.macroscopic()
        p = r_ * T - T0
        t = n * c.fluid.dt
        prof = {}
        for name, speed in (("adiabatic", cs), ("isothermal", np.sqrt(T0))):
            th = np.array([linear_acoustics_pressure(r, t, speed) for r in rs])
            field = 0.0
            for mx in (-1, 0, 1):          # periodic images superpose linearly
                for my in (-1, 0, 1):
                    R = np.hypot(c.mesh.X - 32 - 64 * mx, c.mesh.Y - 32 - 64 * my)
                    field = field + np.interp(R, rs, th)
            prof[name] = (th, field)
        th, field = prof["adiabatic"]
        peak = np.max(th)
        R0 = np.hypot(c.mesh.X - 32, c.mesh.Y - 32)
        r_peak_th = rs[np.argmax(th)]
        r_peak_sim = R0.ravel()[np.argmax(p)]
        assert r_peak_sim == pytest.approx(r_peak_th, rel=0.05)
        assert np.max(p) == pytest.approx(peak, rel=0.05)
        assert np.max(np.abs(p - field)) < 0.2 * peak
        assert np.max(np.abs(p - prof["isothermal"][1])) > 0.5 * peak
