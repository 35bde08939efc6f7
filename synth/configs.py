"""Workload definitions: meshes, physical parameters and initial fields.

Everything is in lattice units with the gas constant R = 1.  The conversion
from the non-dimensional groups (Mach, Reynolds, mass ratio, reduced
velocity) to dimensional lattice quantities follows the definitions of the
paper's validation section (1DOF spring-mass non-dimensionalisation and the
2DOF pitch-plunge parameters); they describe the problem being simulated,
not the lattice Boltzmann scheme.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace

import numpy as np

from .meshes import MeshSpec, ogrid_mesh, periodic_sine_mesh

DOF_PRESCRIBED = 0
DOF_HEAVE = 1
DOF_PITCH_PLUNGE = 2
DOF_FIXED = 3


@dataclass
class FluidParams:
    gamma: float = 1.4
    Pr: float = 0.71
    mu: float = 0.01          # dynamic viscosity (constant)
    rho_inf: float = 1.0
    T_inf: float = 1.0 / 3.0
    u_inf: tuple = (0.0, 0.0)
    dt: float = 1.0 / 3.0
    storage: int = 0          # 0 = FP32 populations, 1 = FP16 shifted


@dataclass
class BodyParams:
    dof: int = DOF_FIXED
    m: float = 1.0
    S_a: float = 0.0
    I_a: float = 1.0
    k_h: float = 0.0
    k_a: float = 0.0
    center: tuple = (0.0, 0.0)   # centre of the blending region (undeformed frame)
    ea: tuple = (0.0, 0.0)       # elastic axis / rotation centre (undeformed frame)
    r_rigid: float = 1.0
    r_blend: float = 2.0
    h0: float = 0.0
    a0: float = 0.0
    hd0: float = 0.0
    ad0: float = 0.0
    heave_amp: float = 0.0
    heave_freq: float = 0.0
    pitch_amp: float = 0.0
    pitch_freq: float = 0.0


@dataclass
class Case:
    name: str
    mesh: MeshSpec
    fluid: FluidParams
    bodies: list = field(default_factory=list)
    rho: np.ndarray | None = None
    ux: np.ndarray | None = None
    uy: np.ndarray | None = None
    T: np.ndarray | None = None
    steps: int = 0
    info: dict = field(default_factory=dict)


def sound_speed(gamma: float, T: float) -> float:
    return math.sqrt(gamma * T)


def gaussian_pulse_fields(mesh: MeshSpec, amp: float, sigma: float, center,
                          rho0: float = 1.0, T0: float = 1.0 / 3.0,
                          u0=(0.0, 0.0)):
    """rho = rho0 (1 + amp exp(-d^2 / (2 sigma^2))), T = T0, u = u0.

    d is the minimum-image distance on doubly periodic meshes.
    """
    dx = mesh.X - center[0]
    dy = mesh.Y - center[1]
    if mesh.shift_i[0] != 0.0:
        Lx = mesh.shift_i[0]
        dx = dx - Lx * np.round(dx / Lx)
    if mesh.shift_j[1] != 0.0:
        Ly = mesh.shift_j[1]
        dy = dy - Ly * np.round(dy / Ly)
    d2 = dx * dx + dy * dy
    rho = rho0 * (1.0 + amp * np.exp(-d2 / (2.0 * sigma * sigma)))
    shape = mesh.X.shape
    return (rho, np.full(shape, float(u0[0])), np.full(shape, float(u0[1])),
            np.full(shape, float(T0)))


def uniform_fields(mesh: MeshSpec, rho0: float, u0, T0: float):
    shape = mesh.X.shape
    return (np.full(shape, float(rho0)), np.full(shape, float(u0[0])),
            np.full(shape, float(u0[1])), np.full(shape, float(T0)))


def cylinder_start_fields(mesh: MeshSpec, D: float, U: float, rho0: float, T0: float,
                          delta: float, center=(0.0, 0.0), potential: bool = True):
    """Smooth start for flow past a cylinder of diameter D: incompressible
    potential flow (or a uniform stream) multiplied by tanh((r - R)/delta), so
    the velocity rises from zero at the wall over a layer of width delta;
    uniform density and temperature.  An impulsive start (free-stream velocity
    on the no-slip wall) drives the Grad wall populations negative when
    1/omega is large."""
    R = 0.5 * D
    dx = mesh.X - center[0]
    dy = mesh.Y - center[1]
    r = np.hypot(dx, dy)
    layer = np.tanh(np.maximum(r - R, 0.0) / delta)
    if potential:
        c = dx / r
        s = dy / r
        a = (R / r) ** 2
        ur = U * (1.0 - a) * c
        ut = -U * (1.0 + a) * s
        ux = (ur * c - ut * s) * layer
        uy = (ur * s + ut * c) * layer
    else:
        ux = U * layer
        uy = np.zeros_like(ux)
    shape = mesh.X.shape
    return np.full(shape, float(rho0)), ux, uy, np.full(shape, float(T0))


def start_layer_width(D: float, first_cell: float) -> float:
    return max(0.01 * D, 10.0 * first_cell)


def acoustic_pulse_case(n: int = 64, amp_mesh: float = 0.05, dt: float = 1.0 / 3.0,
                        nu: float = 0.01, steps: int = 100) -> Case:
    """Static 64x64 periodic sine-deformed mesh, gas at rest, Gaussian pulse.

    rho = 1 + 1e-3 exp(-d^2 / (2 * 4^2)) around the domain centre, T = 1/3,
    gamma = 1.4, nu = 0.01, Pr = 0.71.
    """
    mesh = periodic_sine_mesh(n, amp_mesh)
    fluid = FluidParams(gamma=1.4, Pr=0.71, mu=nu * 1.0, rho_inf=1.0,
                        T_inf=1.0 / 3.0, u_inf=(0.0, 0.0), dt=dt)
    rho, ux, uy, T = gaussian_pulse_fields(mesh, 1e-3, 4.0, (n / 2.0, n / 2.0))
    return Case("acoustic_pulse_64x64", mesh, fluid, [], rho, ux, uy, T, steps,
                info={"pulse_amp": 1e-3, "sigma": 4.0, "center": (n / 2, n / 2)})


def heave_body_params(D: float, rho: float, U: float, mstar: float, ustar: float,
                      r_rigid: float, r_blend: float, h0: float = 0.0) -> BodyParams:
    """1DOF spring-mounted cylinder: m = m* rho pi D^2 / 4, f_N = U / (U* D),
    k_h = m (2 pi f_N)^2 (undamped)."""
    m = mstar * rho * math.pi * D * D / 4.0
    fN = U / (ustar * D)
    k = m * (2.0 * math.pi * fN) ** 2
    return BodyParams(dof=DOF_HEAVE, m=m, S_a=0.0, I_a=1.0, k_h=k, k_a=0.0,
                      center=(0.0, 0.0), ea=(0.0, 0.0), r_rigid=r_rigid,
                      r_blend=r_blend, h0=h0)


def cylinder_viv_case(n_r: int = 256, n_theta: int = 512, D: float = 200.0,
                      first_cell_frac: float = 0.005, r_far_D: float = 30.0,
                      Ma: float = 0.2, Re: float = 100.0, T_inf: float = 1.0 / 3.0,
                      gamma: float = 1.4, Pr: float = 0.71, mstar: float = 10.0,
                      ustar: float = 5.0, blend_D: float = 10.0,
                      h0_frac: float = 0.0, dt: float | None = None,
                      steps: int = 20000, name: str | None = None) -> Case:
    """Single elastically mounted cylinder (1DOF cross-flow VIV) on an O-grid."""
    first = first_cell_frac * D
    mesh = ogrid_mesh(n_r, n_theta, D, first, r_far_D * D)
    U = Ma * sound_speed(gamma, T_inf)
    rho = 1.0
    mu = rho * U * D / Re
    if dt is None:
        h_min = min(first, math.pi * D / n_theta)
        dt = h_min / 3.0
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=mu, rho_inf=rho, T_inf=T_inf,
                        u_inf=(U, 0.0), dt=dt)
    body = heave_body_params(D, rho, U, mstar, ustar, r_rigid=0.5 * D,
                             r_blend=blend_D * D, h0=h0_frac * D)
    r, ux, uy, T = cylinder_start_fields(mesh, D, U, rho, T_inf, start_layer_width(D, first))
    return Case(name or f"cylinder_viv_{n_r}x{n_theta}", mesh, fluid, [body],
                r, ux, uy, T, steps,
                info={"D": D, "U": U, "Ma": Ma, "Re": Re, "mstar": mstar,
                      "ustar": ustar})


def large_heave_case(n_r: int = 2048, n_theta: int = 4096, D: float = 1600.0,
                     Ma: float = 0.5, Re: float = 1000.0, T_inf: float = 1.0 / 3.0,
                     gamma: float = 1.4, Pr: float = 0.71, steps: int = 5000,
                     storage: int = 0) -> Case:
    """Cylinder with a prescribed sinusoidal heave (amplitude 0.2 D, frequency
    0.2 U / D) on a large O-grid with square wall cells (first cell pi D / n_theta)
    stretched geometrically to 30 D."""
    first = math.pi * D / n_theta
    mesh = ogrid_mesh(n_r, n_theta, D, first, 30.0 * D)
    U = Ma * sound_speed(gamma, T_inf)
    rho = 1.0
    mu = rho * U * D / Re
    dt = first / 3.0
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=mu, rho_inf=rho, T_inf=T_inf,
                        u_inf=(U, 0.0), dt=dt, storage=storage)
    body = BodyParams(dof=DOF_PRESCRIBED, m=1.0, center=(0.0, 0.0), ea=(0.0, 0.0),
                      r_rigid=0.5 * D, r_blend=10.0 * D, heave_amp=0.2 * D,
                      heave_freq=0.2 * U / D)
    r, ux, uy, T = cylinder_start_fields(mesh, D, U, rho, T_inf, start_layer_width(D, first))
    return Case(f"cylinder_heave_{n_r}x{n_theta}", mesh, fluid, [body], r, ux, uy,
                T, steps, info={"D": D, "U": U, "Ma": Ma, "Re": Re})


def batched_sweep_cases(n_instances: int = 64, seed: int = 0, D: float = 200.0,
                        steps: int = 10000) -> list:
    """Independent 1DOF cylinder instances of uneven size for a parameter sweep.

    Drawn in order per instance with numpy.random.default_rng(seed):
    n_r ~ U_int[128, 384], n_theta = 2 n_r, U* ~ U[3, 8], m* ~ U[2, 20],
    Ma ~ U[0.1, 0.4]; Re = 100, T = 1/3, first cell 0.005 D, far field 30 D.
    """
    rng = np.random.default_rng(seed)
    cases = []
    for k in range(n_instances):
        n_r = int(rng.integers(128, 385))
        ustar = float(rng.uniform(3.0, 8.0))
        mstar = float(rng.uniform(2.0, 20.0))
        ma = float(rng.uniform(0.1, 0.4))
        cases.append(cylinder_viv_case(n_r=n_r, n_theta=2 * n_r, D=D, Ma=ma,
                                       Re=100.0, mstar=mstar, ustar=ustar,
                                       dt=1.0 / 3.0, steps=steps,
                                       name=f"sweep{k:02d}_{n_r}x{2 * n_r}"))
    return cases


def with_fluid(case: Case, **kw) -> Case:
    return replace(case, fluid=replace(case.fluid, **kw))
