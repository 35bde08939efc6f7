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

from .meshes import MeshSpec, cgrid_mesh, ogrid_mesh, periodic_sine_mesh, twin_mesh

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
    release_time: float = 0.0    # > 0: prescribed motion until then, free afterwards
    blend_mode: int = 0          # 0: radial from `center`; 1: distance to the wall
    link: int = -1               # >= 0: moves rigidly with that (earlier) body, no ODE of its own


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


def distance_to_polygon(X: np.ndarray, Y: np.ndarray, px: np.ndarray, py: np.ndarray,
                        chunk: int = 4096) -> np.ndarray:
    """Distance from every point (X, Y) to the closed polygon (px, py)."""
    ax, ay = px, py
    bx, by = np.roll(px, -1), np.roll(py, -1)
    ex, ey = bx - ax, by - ay
    ee = np.maximum(ex * ex + ey * ey, 1e-300)
    xf, yf = X.ravel(), Y.ravel()
    out = np.empty(xf.size)
    for k0 in range(0, xf.size, chunk):
        x = xf[k0:k0 + chunk, None]
        y = yf[k0:k0 + chunk, None]
        t = np.clip(((x - ax) * ex + (y - ay) * ey) / ee, 0.0, 1.0)
        dx = x - (ax + t * ex)
        dy = y - (ay + t * ey)
        out[k0:k0 + chunk] = np.sqrt(np.min(dx * dx + dy * dy, axis=1))
    return out.reshape(X.shape)


def airfoil_start_fields(mesh: MeshSpec, U: float, rho0: float, T0: float, delta: float):
    """Uniform stream along +x multiplied by tanh(d / delta), d the distance to
    the airfoil section (the wall row of the C-grid); uniform rho and T."""
    nw = mesh.n_wake
    px = mesh.X[0, nw:mesh.ni - nw - 1]
    py = mesh.Y[0, nw:mesh.ni - nw - 1]
    d = distance_to_polygon(mesh.X, mesh.Y, px, py)
    ux = U * np.tanh(d / delta)
    shape = mesh.X.shape
    return np.full(shape, float(rho0)), ux, np.zeros(shape), np.full(shape, float(T0))


def pitch_plunge_body_params(chord: float, rho: float, U: float, mstar: float,
                             freq_ratio: float, x_alpha: float, r_alpha: float, VR: float,
                             ea_frac: float, r_rigid: float, r_blend: float,
                             alpha0: float = 0.0, origin=(0.0, 0.0)) -> BodyParams:
    """2DOF pitch-plunge section (semi-chord b = chord / 2, leading edge at
    ``origin``): m = m* pi rho b^2, I_a = m r_a^2 b^2, S_a = m x_a b,
    omega_a = U / (b V_R sqrt(m*)), k_a = I_a omega_a^2, omega_h = ratio omega_a,
    k_h = m omega_h^2; the elastic axis at ea_frac * chord, the blending centre
    at mid-chord; alpha counter-clockwise, h along +y."""
    b = 0.5 * chord
    m = mstar * math.pi * rho * b * b
    I_a = m * r_alpha * r_alpha * b * b
    S_a = m * x_alpha * b
    om_a = U / (b * VR * math.sqrt(mstar))
    om_h = freq_ratio * om_a
    return BodyParams(dof=DOF_PITCH_PLUNGE, m=m, S_a=S_a, I_a=I_a, k_h=m * om_h * om_h,
                      k_a=I_a * om_a * om_a,
                      center=(origin[0] + 0.5 * chord, origin[1]),
                      ea=(origin[0] + ea_frac * chord, origin[1]),
                      r_rigid=r_rigid, r_blend=r_blend, a0=alpha0)


def airfoil_flutter_case(n_wake: int = 128, n_af: int = 512, nj: int = 256,
                         chord: float = 200.0, first_cell: float = 0.25,
                         far_chords: float = 20.0, Ma: float = 0.85, Re: float = 1.0e5,
                         T_inf: float = 0.2, gamma: float = 1.4, Pr: float = 0.71,
                         mstar: float = 60.0, freq_ratio: float = 0.34, x_alpha: float = 1.8,
                         r_alpha: float = 1.87, VR: float = 0.5025, ea_frac: float = 0.25,
                         alpha0_deg: float = 1.0, blend_chords: float = 10.0,
                         steps: int = 50000, storage: int = 0, forced_periods: int = 0,
                         name: str | None = None) -> Case:
    """Pitch-plunge NACA0012 section on a C-grid (768 x 256 with the defaults:
    128 + 512 + 128 nodes along the wrap-around index, far field 20 chords).

    dt is a third of the smallest wall spacing (first cell or wall-node
    spacing); the start is a uniform stream with a tanh layer at the wall.
    forced_periods > 0: the paper's protocol instead of an initial pitch: a
    sinusoidal pitching of amplitude alpha0 at the pitch natural frequency for
    that many periods, then release."""
    mesh = cgrid_mesh(n_wake, n_af, nj, chord, first_cell, far_chords)
    U = Ma * sound_speed(gamma, T_inf)
    rho = 1.0
    mu = rho * U * chord / Re
    wall = np.hypot(np.diff(mesh.X[0, n_wake:n_wake + n_af]),
                    np.diff(mesh.Y[0, n_wake:n_wake + n_af]))
    h_min = min(first_cell, float(wall.min()))
    dt = h_min / 3.0
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=mu, rho_inf=rho, T_inf=T_inf,
                        u_inf=(U, 0.0), dt=dt, storage=storage)
    body = pitch_plunge_body_params(chord, rho, U, mstar, freq_ratio, x_alpha, r_alpha, VR,
                                    ea_frac, r_rigid=0.55 * chord,
                                    r_blend=blend_chords * chord,
                                    alpha0=math.radians(alpha0_deg))
    if forced_periods > 0:
        om_a = math.sqrt(body.k_a / body.I_a)
        body = replace(body, a0=0.0, pitch_amp=math.radians(alpha0_deg),
                       pitch_freq=om_a / (2.0 * math.pi),
                       release_time=forced_periods * 2.0 * math.pi / om_a)
    r, ux, uy, T = airfoil_start_fields(mesh, U, rho, T_inf, start_layer_width(chord, first_cell))
    return Case(name or f"airfoil_flutter_{mesh.ni}x{nj}", mesh, fluid, [body], r, ux, uy, T,
                steps, info={"chord": chord, "U": U, "Ma": Ma, "Re": Re, "mstar": mstar})


def small_airfoil_case(n_wake: int = 16, n_af: int = 64, nj: int = 32, chord: float = 40.0,
                       first_cell: float = 0.5, far_chords: float = 4.0, Ma: float = 0.3,
                       Re: float = 200.0, T_inf: float = 1.0 / 3.0, mstar: float = 5.0,
                       alpha0_deg: float = 1.0, blend_chords: float = 2.5,
                       steps: int = 200) -> Case:
    """A small C-grid pitch-plunge case the oracle can run for many steps."""
    return airfoil_flutter_case(n_wake=n_wake, n_af=n_af, nj=nj, chord=chord,
                                first_cell=first_cell, far_chords=far_chords, Ma=Ma, Re=Re,
                                T_inf=T_inf, mstar=mstar, alpha0_deg=alpha0_deg,
                                blend_chords=blend_chords, steps=steps,
                                name=f"small_airfoil_{2 * n_wake + n_af}x{nj}")


def smallest_metric_scale(mesh: MeshSpec, rows: int = 4) -> float:
    """Smallest singular value of the index-space Jacobian d(x, y)/d(i, j)
    (centred in i, one-sided into the mesh from the wall row) over the first
    rows of a wall-bounded periodic mesh: the shortest physical step that one
    index step can take there.  A time step of a third of it keeps every
    departure point of a node within half a cell of it in index space."""
    X, Y = mesh.X[:rows + 2], mesh.Y[:rows + 2]
    xi = 0.5 * (np.roll(X, -1, 1) - np.roll(X, 1, 1))[:rows]
    yi = 0.5 * (np.roll(Y, -1, 1) - np.roll(Y, 1, 1))[:rows]
    xe = np.empty_like(xi)
    ye = np.empty_like(yi)
    xe[0] = -1.5 * X[0] + 2.0 * X[1] - 0.5 * X[2]
    ye[0] = -1.5 * Y[0] + 2.0 * Y[1] - 0.5 * Y[2]
    xe[1:] = 0.5 * (X[2:rows + 1] - X[:rows - 1])
    ye[1:] = 0.5 * (Y[2:rows + 1] - Y[:rows - 1])
    a = xi * xi + yi * yi
    c = xe * xe + ye * ye
    b = xi * xe + yi * ye
    lam_min = 0.5 * (a + c) - np.sqrt(0.25 * (a - c) ** 2 + b * b)
    return float(np.sqrt(np.min(lam_min)))


def tandem_start_fields(mesh: MeshSpec, D: float, centers, U: float, rho0: float, T0: float,
                        delta: float):
    """Uniform stream along +x multiplied by tanh(d / delta), d the distance to
    the nearer cylinder surface; uniform rho and T."""
    d = np.min([np.hypot(mesh.X - cx, mesh.Y - cy) for (cx, cy) in centers], axis=0) - 0.5 * D
    ux = U * np.tanh(np.maximum(d, 0.0) / delta)
    shape = mesh.X.shape
    return np.full(shape, float(rho0)), ux, np.zeros(shape), np.full(shape, float(T0))


def tandem_cylinders_case(linked: bool = False, n_wall: int = 512, n_slit: int = 640,
                          nj: int = 320, D: float = 200.0, L_D: float = 5.0,
                          first_cell: float = 1.0, far_D: float = 30.0, Ma: float = 0.1,
                          Re: float = 1000.0, T_inf: float = 1.0 / 3.0, gamma: float = 1.4,
                          Pr: float = 0.71, mstar: float = 4.0, ustar: float = 6.0,
                          rigid_gap_D: float = 0.25, blend_gap_D: float = 2.0,
                          h0_frac: float = 0.0, steps: int = 20000, storage: int = 0,
                          name: str | None = None) -> Case:
    """Two cylinders of diameter D in tandem (centres L_D * D apart on the x
    axis, the stream along +x) on a twin O-grid.

    Independent (linked=False, the 1+1DOF case): each cylinder is a 1DOF
    cross-flow oscillator with m = m* rho pi D^2 / 4 and f_N = U / (U* D).
    Linked (the 1DOF case of two rigidly connected cylinders on one spring):
    the downstream cylinder is linked to the upstream one, whose equation
    carries the assembly, m = m* rho 2 pi D^2 / 4 (reading: the mass ratio of
    the assembly to the fluid both cylinders displace), and the sum of the
    two loads.  Regions of influence: rigid to rigid_gap_D * D and blended to
    blend_gap_D * D from each surface (the paper's 50 and 400 lattice units at
    D = 200), capped at half the centre distance so they do not overlap.
    dt is a third of the smallest index-step length near the walls."""
    L = L_D * D
    mesh = twin_mesh(n_wall, n_slit, nj, D, L, first_cell, far_D)
    U = Ma * sound_speed(gamma, T_inf)
    rho = 1.0
    mu = rho * U * D / Re
    dt = smallest_metric_scale(mesh) / 3.0
    fluid = FluidParams(gamma=gamma, Pr=Pr, mu=mu, rho_inf=rho, T_inf=T_inf,
                        u_inf=(U, 0.0), dt=dt, storage=storage)
    R = 0.5 * D
    r_rigid = R + rigid_gap_D * D
    r_blend = min(R + blend_gap_D * D, 0.5 * L)
    centers = ((-0.5 * L, 0.0), (0.5 * L, 0.0))
    fN = U / (ustar * D)
    m1 = mstar * rho * math.pi * D * D / 4.0
    bodies = []
    for k, c in enumerate(centers):
        m = m1 * (2.0 if linked else 1.0)
        b = BodyParams(dof=DOF_HEAVE, m=m, k_h=m * (2.0 * math.pi * fN) ** 2, center=c, ea=c,
                       r_rigid=r_rigid, r_blend=r_blend, h0=h0_frac * D)
        if linked and k == 1:
            b = replace(b, link=0, m=1.0, k_h=0.0, h0=0.0)
        bodies.append(b)
    r, ux, uy, T = tandem_start_fields(mesh, D, centers, U, rho, T_inf,
                                       start_layer_width(D, first_cell))
    kind = "linked" if linked else "independent"
    return Case(name or f"tandem_{kind}_{mesh.ni}x{nj}", mesh, fluid, bodies, r, ux, uy, T,
                steps, info={"D": D, "L": L, "U": U, "Ma": Ma, "Re": Re, "mstar": mstar,
                             "ustar": ustar, "centers": centers})


def small_tandem_case(linked: bool = False, n_wall: int = 48, n_slit: int = 30, nj: int = 40,
                      D: float = 30.0, L_D: float = 3.0, first_cell: float = 0.5,
                      far_D: float = 8.0, Ma: float = 0.2, Re: float = 100.0,
                      mstar: float = 2.0, ustar: float = 4.0, h0_frac: float = 0.01,
                      steps: int = 100) -> Case:
    """A small tandem-cylinder twin O-grid case the oracle can run for many steps."""
    return tandem_cylinders_case(linked=linked, n_wall=n_wall, n_slit=n_slit, nj=nj, D=D,
                                 L_D=L_D, first_cell=first_cell, far_D=far_D, Ma=Ma, Re=Re,
                                 mstar=mstar, ustar=ustar, rigid_gap_D=0.1, blend_gap_D=0.5,
                                 h0_frac=h0_frac, steps=steps,
                                 name=f"small_tandem_{2 * n_wall + 2 * n_slit}x{nj}")


def with_fluid(case: Case, **kw) -> Case:
    return replace(case, fluid=replace(case.fluid, **kw))
