"""The staggered fluid-structure time step in float64 (paper Sec. III:
weak coupling; Sec. II: kinetic equations and semi-Lagrangian transport).
Test infrastructure only.

One step n -> n+1 (reading of the staggered order: the fluid step is followed
by the force evaluation, the structure update and the mesh update, so at the
start of step n the load F^n of the populations f^n is known):

 1. F^n      surface force and moment from f^n on the mesh x^n
 2. s^{n+1}  body state (RK4 with F^n frozen, or prescribed motion)
 3. x^{n+1}  blended mesh; V_G = (x^{n+1} - x^n) / dt
 4. collide  f^n at the nodes of x^n, with the correction F_a computed from
             nested FE gradients on x^n (zero at a C-grid's trailing edge):
                 D_a = (1/omega - 1/2) dt d_a dQ_a,   F_a = d_a D_a
             (reading: the factor dt makes the correction cancel the
             (1/omega - 1/2) dt scaled defect of the viscous stress for any
             time step, as the Chapman-Enskog expansion requires; the paper
             prints it for dt = 1)
 5. stream   ALE departure points with g and V_G at t^{n+1}; interpolation
 6. boundary far-field equilibria; Grad wall populations for the missing ones
 7. cut topologies (C-grid, twin O-grid): the duplicated nodes of row 0 are
    made single-valued (reading: the paper's unstructured meshes have no
    duplicated nodes).  The two copies of a trailing edge or of a junction of
    the slit with a body each see the cells of one side only, so population
    by population the point takes the streamed value of the copy that found
    its departure point, and the mean of the two copies where both or neither
    did; the mirror copy of every cut node takes the primary copy's values
    (the two are mirror-image evaluations of the same update).

Several bodies (Sec. II.D and the tandem-cylinder cases of Sec. V): each has
its own wall segment (body k <-> segment k of the mesh), its own region of
influence and its own load.  A body linked to another (a rigid assembly on
one spring, as the linked tandem cylinders) has no equation of its own: it
moves with that body, and its load joins that body's equation (forces
summed, moments about that body's elastic axis).
"""

from __future__ import annotations

import numpy as np

from . import lattice as L
from . import body as B
from .boundary import farfield_bc, wall_grad_bc
from .forces import wall_force
from .mesh import Grid, deformed_positions, master_of
from .stream import stream


def correction_force(grid, f, g, x, y, gamma, mu, Pr, dt):
    """F_a = d_a[(1/omega - 1/2) dt d_a dQ_a] with physical FE derivatives on
    the mesh (x, y) (Sec. II.C, momentum correction; Sec. II.B gradients)."""
    rho, ux, uy, E, T = L.macroscopic(f, g, gamma)
    omega, _ = L.relaxation_rates(rho, T, mu, Pr, dt)
    dQx, dQy = L.momentum_defect(rho, ux, uy, T)
    dQx_dx, _ = grid.grad(dQx, x, y)
    _, dQy_dy = grid.grad(dQy, x, y)
    Dx = (1.0 / omega - 0.5) * dt * dQx_dx
    Dy = (1.0 / omega - 0.5) * dt * dQy_dy
    Fx, _ = grid.grad(Dx, x, y)
    _, Fy = grid.grad(Dy, x, y)
    return Fx, Fy


def merge_cut_row(grid, f_new, g_new, missing):
    """Single-valued duplicated points of row 0 (step 7)."""
    for (i0, n, dup) in grid.segments:
        if not dup:
            continue
        a, b = i0, i0 + n - 1                 # the two copies of one point
        ma, mb = missing[:, 0, a], missing[:, 0, b]
        for F in (f_new, g_new):
            va, vb = F[:, 0, a].copy(), F[:, 0, b].copy()
            v = np.where(ma & ~mb, vb, np.where(mb & ~ma, va, 0.5 * (va + vb)))
            F[:, 0, a] = v
            F[:, 0, b] = v
    prim = grid.primary_cols
    for F in (f_new, g_new):
        F[:, 0, grid.mirror(prim)] = F[:, 0, prim]


def junction_columns(grid):
    """Columns of row 0 that are one copy of a duplicated wall point."""
    out = []
    for (i0, n, dup) in grid.segments:
        if dup:
            out += [i0, i0 + n - 1]
    return out


class OracleSolver:
    """Plain FP64 reference of the whole coupled step on one structured mesh."""

    def __init__(self, mesh, fluid, bodies=(), rho=None, ux=None, uy=None, T=None,
                 correction=True):
        self.mesh = mesh
        self.grid = Grid.from_mesh(mesh)
        self.X = mesh.X.astype(np.float64)
        self.Y = mesh.Y.astype(np.float64)
        self.fluid = fluid
        self.bodies = list(bodies)
        self.correction = correction
        self.n = 0
        for k, b in enumerate(self.bodies):
            link = getattr(b, "link", -1)
            assert link < k and (link < 0 or master_of(self.bodies, link) == link), \
                "a body links to an earlier body that is not linked itself"
        self.states = [B.initial_state(b) for b in self.bodies]
        self.states = [self.states[master_of(self.bodies, k)] for k in range(len(self.bodies))]
        self.history = []                     # body 0
        self.histories = [[] for _ in self.bodies]
        shape = self.X.shape
        if rho is None:
            rho = np.full(shape, fluid.rho_inf)
            ux = np.full(shape, fluid.u_inf[0])
            uy = np.full(shape, fluid.u_inf[1])
            T = np.full(shape, fluid.T_inf)
        self.f, self.g = L.equilibrium_populations(rho, ux, uy, T, fluid.gamma)
        self.has_wall = mesh.topo in (1, 2, 3)
        if self.bodies:
            assert len(self.bodies) <= max(1, len(self.grid.segments)), \
                "one wall segment per body"
        # undeformed wall polygons (distance-field blending), one per body
        self.walls = None
        if self.has_wall:
            from .forces import wall_polygon
            self.walls = []
            for k in range(len(self.grid.segments)):
                cols = wall_polygon(self.grid, k)
                self.walls.append((self.X[0, cols], self.Y[0, cols]))
        self.wall = self.walls[0] if self.walls else None
        self._r_cache = None
        self.subiterations = 1
        self.relaxation = 1.0
        self.residuals = []

    def coupling(self, subiterations=1, relaxation=1.0):
        """Strong coupling by sub-iterations (the alternative to the staggered
        scheme that Sec. III names for low mass ratios; the paper gives no
        algorithm).  Reading: each step starts from the staggered predictor
        (the structure advanced with the load at t^n frozen); a sub-iteration
        streams the post-collision populations of t^n onto the mesh of the
        current structure estimate, applies the boundary conditions, takes the
        load F^{n+1} of the result, re-solves the structure over the step with
        the load varying linearly from F^n to F^{n+1}, and relaxes the estimate
        towards that solution with the factor `relaxation`.  The last
        sub-iteration's fluid state and the structure state it was computed
        with are accepted (so populations and mesh stay consistent); the
        remaining change |solution - estimate| of each sub-iteration is kept in
        `residuals`.  One sub-iteration is the staggered scheme itself."""
        assert subiterations >= 1 and 0.0 < relaxation <= 1.0
        self.subiterations = int(subiterations)
        self.relaxation = float(relaxation)

    # ---- geometry ---------------------------------------------------------
    def positions(self, states):
        if self.bodies and self._r_cache is None:
            from .mesh import blend_factors
            walls = self.walls[:len(self.bodies)] if self.walls else None
            self._r_cache = blend_factors(self.X, self.Y, self.bodies, walls)
        return deformed_positions(self.X, self.Y, self.bodies, states, None, self._r_cache)

    def ea_position(self, states, k=0):
        """Physical elastic axis about which body k's moment is taken: the
        axis of the body it moves with."""
        m = master_of(self.bodies, k)
        b = self.bodies[m]
        return (b.ea[0], b.ea[1] + states[m][0])

    # ---- step pieces --------------------------------------------------------
    def body_forces(self):
        """(F_x, F_y, M) on the wall of every body at the current level."""
        if not (self.has_wall and self.bodies):
            return [(0.0, 0.0, 0.0) for _ in self.bodies]
        fl = self.fluid
        x, y = self.positions(self.states)
        return [wall_force(self.grid, self.f, self.g, x, y, fl.gamma, fl.mu, fl.Pr,
                           fl.dt, self.ea_position(self.states, k), seg=k)
                for k in range(len(self.bodies))]

    def forces(self):
        if not self.bodies:
            return (0.0, 0.0, 0.0)
        return self.body_forces()[0]

    def _advance_bodies(self, Fb, Fb1=None):
        """New states of all bodies over one step from the loads Fb at t^n
        (frozen), or varying linearly to Fb1 at t^{n+1}; linked bodies take
        the state of the body they move with, whose equation carries their
        loads."""
        dt = self.fluid.dt
        nb = len(self.bodies)
        new_states = [None] * nb
        for m in range(nb):
            if master_of(self.bodies, m) != m:
                continue
            Fy = Mz = 0.0
            Fy1 = Mz1 = None if Fb1 is None else 0.0
            for k in range(nb):                      # own load, then linked bodies'
                if master_of(self.bodies, k) == m:
                    Fy += Fb[k][1]
                    Mz += Fb[k][2]
                    if Fb1 is not None:
                        Fy1 += Fb1[k][1]
                        Mz1 += Fb1[k][2]
            new_states[m] = B.advance(self.bodies[m], self.states[m], Fy, Mz,
                                      (self.n + 1) * dt, dt, Fy1, Mz1)
        return [new_states[master_of(self.bodies, k)] for k in range(nb)]

    def _loads(self, f, g, states):
        """Loads of every body from populations (f, g) on the mesh of `states`."""
        if not (self.has_wall and self.bodies):
            return [(0.0, 0.0, 0.0) for _ in self.bodies]
        fl = self.fluid
        x, y = self.positions(states)
        return [wall_force(self.grid, f, g, x, y, fl.gamma, fl.mu, fl.Pr, fl.dt,
                           self.ea_position(states, k), seg=k)
                for k in range(len(self.bodies))]

    def _fluid(self, fpost, gpost, x0, y0, new_states):
        """Streaming onto the mesh of `new_states` and the boundary conditions
        (steps 3, 5-7) from the post-collision populations."""
        fl = self.fluid
        dt = fl.dt
        x1, y1 = self.positions(new_states)
        VGx = (x1 - x0) / dt
        VGy = (y1 - y0) / dt
        f_new, g_new, missing = stream(self.grid, self.X, self.Y, x1, y1, VGx, VGy,
                                       dt, fpost, gpost)
        if self.has_wall:
            farfield_bc(self.grid, self.X, self.Y, f_new, g_new, fl.gamma,
                        fl.rho_inf, fl.u_inf, fl.T_inf)
            wall_grad_bc(self.grid, self.X, self.Y, x1, y1, VGx, VGy, f_new, g_new,
                         missing, self.f, self.g, fl.gamma, fl.mu, fl.Pr, dt)
        if self.grid.cut:
            merge_cut_row(self.grid, f_new, g_new, missing)
        return f_new, g_new, missing

    def step(self):
        fl = self.fluid
        dt = fl.dt
        # 1-2: load at t^n, structure to t^{n+1}
        Fb = self.body_forces()
        nb = len(self.bodies)
        new_states = self._advance_bodies(Fb)
        for k in range(nb):
            s = self.states[k]
            self.histories[k].append((self.n, Fb[k][0], Fb[k][1], Fb[k][2], s[0], s[1]))
        if nb:
            self.history = self.histories[0]
        # 4: collision on x^n (it does not depend on the new mesh)
        x0, y0 = self.positions(self.states)
        if self.correction:
            Fx, Fy = correction_force(self.grid, self.f, self.g, x0, y0, fl.gamma,
                                      fl.mu, fl.Pr, dt)
        else:
            Fx = np.zeros_like(self.X)
            Fy = np.zeros_like(self.X)
        if self.grid.cut:
            # a duplicated point collides once: its two copies' one-sided nested
            # derivatives differ at the sharp edge, so the correction is dropped there
            te = junction_columns(self.grid)
            Fx[0, te] = 0.0
            Fy[0, te] = 0.0
        fpost, gpost = L.collide(self.f, self.g, fl.gamma, fl.mu, fl.Pr, dt, Fx, Fy)
        # 3, 5-7: mesh, streaming, boundaries; with strong coupling, repeated
        # with the structure re-solved against the new load (see `coupling`)
        self.residuals = []
        for it in range(self.subiterations):
            f_new, g_new, missing = self._fluid(fpost, gpost, x0, y0, new_states)
            if self.subiterations == 1:
                break
            Fb1 = self._loads(f_new, g_new, new_states)
            target = self._advance_bodies(Fb, Fb1)
            self.residuals.append(max((float(np.max(np.abs(np.asarray(t) - np.asarray(s))))
                                       for t, s in zip(target, new_states)), default=0.0))
            if it + 1 < self.subiterations:
                w = self.relaxation
                new_states = [np.asarray(s) + w * (np.asarray(t) - np.asarray(s))
                              for s, t in zip(new_states, target)]
        self.last_missing = missing
        self.f, self.g = f_new, g_new
        self.states = new_states
        self.n += 1

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    def macroscopic(self):
        return L.macroscopic(self.f, self.g, self.fluid.gamma)
