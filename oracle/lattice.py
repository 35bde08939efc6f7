"""D2Q9 two-population kinetic model in float64 (paper Sec. II.C, "Kinetic
Equations").  Test infrastructure only.

Population arrays are shaped [9, ...] (velocity first), fields [...].

Velocity order: 0:(0,0) 1:(1,0) 2:(0,1) 3:(-1,0) 4:(0,-1)
                5:(1,1) 6:(-1,1) 7:(-1,-1) 8:(1,-1)
"""

from __future__ import annotations

import numpy as np

Q = 9
CX = (0, 1, 0, -1, 0, 1, -1, -1, 1)
CY = (0, 0, 1, 0, -1, 1, 1, -1, -1)


class NonPhysicalState(ValueError):
    """rho <= 0, T <= 0, NaN, or outside the D2Q9 positivity domain
    (W_0 = 1 - T > 0 and Phi_0 = 1 - u_a^2 - T > 0)."""


def specific_heats(gamma: float):
    """R = 1, C_v = R / (gamma - 1), C_p = C_v + R (Sec. II.C)."""
    Cv = 1.0 / (gamma - 1.0)
    return Cv, Cv + 1.0


def weight_1d(c: int, T):
    """W_{-1} = T/2, W_0 = 1 - T, W_{+1} = T/2 (Sec. II.C, weights)."""
    if c == 0:
        return 1.0 - T
    return 0.5 * T


def weights(T):
    """W_i = W_{c_ix} W_{c_iy}, temperature dependent (Sec. II.C)."""
    return np.stack([weight_1d(CX[i], T) * weight_1d(CY[i], T) for i in range(Q)])


def phi_1d(c: int, u, T):
    """Phi_0 = 1 - (u_a^2 + T), Phi_{+-1} = (+-u_a + u_a^2 + T)/2 (Sec. II.C)."""
    if c == 0:
        return 1.0 - (u * u + T)
    return 0.5 * (c * u + u * u + T)


def feq(rho, ux, uy, T):
    """Product-form equilibrium f_i^eq = rho Phi_{c_ix}(u_x) Phi_{c_iy}(u_y)
    (Sec. II.C, Eq. for f^eq)."""
    return np.stack([rho * phi_1d(CX[i], ux, T) * phi_1d(CY[i], uy, T)
                     for i in range(Q)])


def macroscopic(f, g, gamma):
    """Density, velocity, energy and temperature from the populations.

    rho = sum f, rho u = sum f c, 2 rho E = sum g, T = (E - u^2/2) / C_v
    (Sec. II.C, conservation laws and definition of T).
    """
    Cv, _ = specific_heats(gamma)
    rho = np.zeros_like(f[0])
    jx = np.zeros_like(f[0])
    jy = np.zeros_like(f[0])
    two_rho_E = np.zeros_like(g[0])
    for i in range(Q):
        rho = rho + f[i]
        jx = jx + CX[i] * f[i]
        jy = jy + CY[i] * f[i]
        two_rho_E = two_rho_E + g[i]
    ux = jx / rho
    uy = jy / rho
    E = two_rho_E / (2.0 * rho)
    T = (E - 0.5 * (ux * ux + uy * uy)) / Cv
    return rho, ux, uy, E, T


def second_moment(f):
    """P = sum_i f_i c_i c_i as (P_xx, P_xy, P_yy)."""
    Pxx = np.zeros_like(f[0])
    Pxy = np.zeros_like(f[0])
    Pyy = np.zeros_like(f[0])
    for i in range(Q):
        Pxx = Pxx + CX[i] * CX[i] * f[i]
        Pxy = Pxy + CX[i] * CY[i] * f[i]
        Pyy = Pyy + CY[i] * CY[i] * f[i]
    return Pxx, Pxy, Pyy


def check_state(rho, ux, uy, T):
    """Raise NonPhysicalState outside the domain where the D2Q9 equilibria are
    positive-weight (W_0 > 0, Phi_0 > 0 in both directions)."""
    bad = ~np.isfinite(rho) | ~np.isfinite(ux) | ~np.isfinite(uy) | ~np.isfinite(T)
    bad |= (rho <= 0) | (T <= 0) | (1.0 - T <= 0)
    bad |= (1.0 - (ux * ux + T) <= 0) | (1.0 - (uy * uy + T) <= 0)
    if np.any(bad):
        k = int(np.flatnonzero(np.ravel(bad))[0])
        raise NonPhysicalState(f"non-physical state at flat node {k}")


def enthalpy(E, T):
    """Total enthalpy H = (C_v + 1) T + u^2/2 = E + T.

    The paper prints (C_v + 1)/T; the first moment of a Maxwellian with R = 1
    gives (C_v + 1) T, which is the reading taken here.
    """
    return E + T


def equilibrium_heat_flux(rho, ux, uy, E, T):
    """q^eq = 2 rho u H (Sec. II.C)."""
    H = enthalpy(E, T)
    return 2.0 * rho * ux * H, 2.0 * rho * uy * H


def equilibrium_R(rho, ux, uy, E, T):
    """R^eq = 2 rho E (T I + u u) + 2 rho T (T I + 2 u u) (Sec. II.C)."""
    Rxx = 2.0 * rho * E * (T + ux * ux) + 2.0 * rho * T * (T + 2.0 * ux * ux)
    Ryy = 2.0 * rho * E * (T + uy * uy) + 2.0 * rho * T * (T + 2.0 * uy * uy)
    Rxy = 2.0 * rho * E * (ux * uy) + 2.0 * rho * T * (2.0 * ux * uy)
    return Rxx, Rxy, Ryy


def energy_correction_deltaR(rho, ux, uy, E, T):
    """delta R_a = rho (1 - 3T)(T^2 + 2 u_a^2 T + E u_a^2) / T, the Hadamard
    argument of Psi (Sec. II.C, energy correction)."""
    dRx = rho * (1.0 - 3.0 * T) * (T * T + 2.0 * ux * ux * T + E * ux * ux) / T
    dRy = rho * (1.0 - 3.0 * T) * (T * T + 2.0 * uy * uy * T + E * uy * uy) / T
    return dRx, dRy


def B_matrix():
    """B_{i,a}: the vectors that place delta R on the lattice.

    The paper does not print B_i.  Reading: B_{0,a} = 1, B_{+-e_a, a} = -1/2,
    all other entries 0.  This has zero zeroth and first moments and
    sum_i B_{i,a} c_ib^2 = -delta_ab, so Psi removes exactly the diagonal
    error of the D2Q9 second moment of g^eq.
    """
    B = np.zeros((Q, 2))
    for i in range(Q):
        if CX[i] == 0 and CY[i] == 0:
            B[i] = (1.0, 1.0)
        elif CY[i] == 0:
            B[i] = (-0.5, 0.0)
        elif CX[i] == 0:
            B[i] = (0.0, -0.5)
    return B


def energy_correction(rho, ux, uy, E, T):
    """Psi_i = B_i . delta R (Sec. II.C, energy correction term)."""
    dRx, dRy = energy_correction_deltaR(rho, ux, uy, E, T)
    B = B_matrix()
    return np.stack([B[i, 0] * dRx + B[i, 1] * dRy for i in range(Q)])


def g_equilibrium_with_flux(rho, ux, uy, E, T, qx, qy):
    """W_i [2 rho E + q.c_i / T + (R^eq - 2 rho E T I):(c_i c_i - T I)/(2 T^2)]
    + Psi_i  (Sec. II.C, Eqs. for g^eq and g^*).

    The printed "(R^eq - rho E T I)" is read as (R^eq - 2 rho E T I): only then
    is the D2Q9 error of the second moment exactly the quantity Psi removes.
    """
    W = weights(T)
    Rxx, Rxy, Ryy = equilibrium_R(rho, ux, uy, E, T)
    Axx = Rxx - 2.0 * rho * E * T
    Ayy = Ryy - 2.0 * rho * E * T
    Axy = Rxy
    Psi = energy_correction(rho, ux, uy, E, T)
    out = []
    for i in range(Q):
        cx, cy = CX[i], CY[i]
        contraction = (Axx * (cx * cx - T) + 2.0 * Axy * cx * cy
                       + Ayy * (cy * cy - T))
        out.append(W[i] * (2.0 * rho * E + (qx * cx + qy * cy) / T
                           + contraction / (2.0 * T * T)) + Psi[i])
    return np.stack(out)


def geq(rho, ux, uy, E, T):
    """Energy equilibrium g_i^eq with q = q^eq (Sec. II.C)."""
    qx, qy = equilibrium_heat_flux(rho, ux, uy, E, T)
    return g_equilibrium_with_flux(rho, ux, uy, E, T, qx, qy)


def quasi_equilibrium_flux(rho, ux, uy, E, T, Pxx, Pxy, Pyy):
    """q^* = q^eq + 2 u . (P - P^eq), with P^eq = rho (T I + u u).

    The paper does not define q^*.  This reading makes the heat-flux part of
    the energy flux relax with omega_1 and its viscous-heating part with omega,
    which yields the Prandtl number (1/omega - 1/2)/(1/omega_1 - 1/2).
    """
    qx, qy = equilibrium_heat_flux(rho, ux, uy, E, T)
    dPxx = Pxx - rho * (T + ux * ux)
    dPxy = Pxy - rho * (ux * uy)
    dPyy = Pyy - rho * (T + uy * uy)
    return (qx + 2.0 * (ux * dPxx + uy * dPxy),
            qy + 2.0 * (ux * dPxy + uy * dPyy))


def gstar(rho, ux, uy, E, T, Pxx, Pxy, Pyy):
    """Quasi-equilibrium g_i^* (Sec. II.C, Eq. for g^*)."""
    qx, qy = quasi_equilibrium_flux(rho, ux, uy, E, T, Pxx, Pxy, Pyy)
    return g_equilibrium_with_flux(rho, ux, uy, E, T, qx, qy)


def relaxation_rates(rho, T, mu, Pr, dt):
    """omega from mu = (1/omega - 1/2) p dt with constant mu and p = rho T;
    omega_1 from Pr = (1/omega - 1/2) / (1/omega_1 - 1/2)
    (Sec. II.C, transport coefficients)."""
    p = rho * T
    omega = 1.0 / (mu / (p * dt) + 0.5)
    omega1 = 1.0 / ((1.0 / omega - 0.5) / Pr + 0.5)
    return omega, omega1


def momentum_defect(rho, ux, uy, T):
    """delta Q_a = rho u_a (1 - 3T) - rho u_a^3: the D2Q9 defect of the diagonal
    third moment of f^eq (argument of the momentum correction, Sec. II.C)."""
    return (rho * ux * (1.0 - 3.0 * T) - rho * ux ** 3,
            rho * uy * (1.0 - 3.0 * T) - rho * uy ** 3)


def momentum_correction(F_x, F_y, T):
    """phi_i = -(W_i / T) c_i . F, where F_a = d_a[(1/omega - 1/2) dt d_a dQ_a].

    The printed 1D factor -c_i/2 is taken with the transverse weight, so that
    sum phi = 0, sum phi c = -F and sum phi c c = 0 (Sec. II.C, phi_i).
    """
    W = weights(T)
    return np.stack([-(W[i] / T) * (CX[i] * F_x + CY[i] * F_y) for i in range(Q)])


def collide(f, g, gamma, mu, Pr, dt, F_x, F_y):
    """One BGK + quasi-equilibrium collision at every node (Sec. II.C, kinetic
    equations):

        f* = f + omega (f^eq - f) + dt phi
        g* = g + omega (g^eq - g) + (omega_1 - omega)(g^* - g)

    F_x, F_y are the nested correction gradients (see ``solver``).
    """
    rho, ux, uy, E, T = macroscopic(f, g, gamma)
    check_state(rho, ux, uy, T)
    Pxx, Pxy, Pyy = second_moment(f)
    omega, omega1 = relaxation_rates(rho, T, mu, Pr, dt)
    fe = feq(rho, ux, uy, T)
    ge = geq(rho, ux, uy, E, T)
    gs = gstar(rho, ux, uy, E, T, Pxx, Pxy, Pyy)
    phi = momentum_correction(F_x, F_y, T)
    f_post = np.stack([f[i] + omega * (fe[i] - f[i]) + dt * phi[i] for i in range(Q)])
    g_post = np.stack([g[i] + omega * (ge[i] - g[i]) + (omega1 - omega) * (gs[i] - g[i])
                       for i in range(Q)])
    return f_post, g_post


def equilibrium_populations(rho, ux, uy, T, gamma):
    """f^eq and g^eq (including Psi) of given macroscopic fields; E = C_v T + u^2/2."""
    Cv, _ = specific_heats(gamma)
    E = Cv * T + 0.5 * (ux * ux + uy * uy)
    return feq(rho, ux, uy, T), geq(rho, ux, uy, E, T)
