"""The step on an unstructured mesh of second-order (9-node) quadrilateral
elements, in float64 (paper Sec. II.B: the semi-Lagrangian method on
unstructured finite-element meshes).  Test infrastructure only.

Populations live at the mesh nodes.  One step on a static periodic mesh:

1. moments, delta Q_a and mu/p at every node (Sec. II.C);
2. nodal gradients by the finite-element derivative dC/dX = J^{-T} sum_s C_s
   grad_xi N_s of each element containing the node, evaluated at the node's
   own position in that element, and averaged over those elements (reading:
   the element derivatives are discontinuous across element edges; the paper
   does not say how a nodal value is formed from them); D_a = (mu/p) d_a
   delta Q_a, F_a = d_a D_a from the same recovery (Sec. II.C correction);
3. collision (Sec. II.C);
4. departure point X_dp = X - dt c_i, located among the elements that contain
   the node with the element's first-order (bilinear, corner-node) map,
   solved by Newton (Sec. II.B: the first-order element saves time);
5. f_i(X) = sum_s N_s(xi_dp) f*_i(X_s) with the element's nine quadratic
   Lagrange shape functions N_s (Sec. II.B).

Element node order and local positions: corners (-1,-1), (1,-1), (1,1),
(-1,1), edge midpoints (0,-1), (1,0), (0,1), (-1,0), centre (0,0).
"""

from __future__ import annotations

import numpy as np

from . import lattice as L

LOCAL = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1],
                  [0, -1], [1, 0], [0, 1], [-1, 0], [0, 0]], dtype=np.float64)
INSIDE_TOL = 1e-12
# Reading (as on the structured wall line; the paper does not say how a point
# on the boundary of the mesh is classified): a boundary node's departure point
# that lies in none of its elements but less than EDGE_TOL (in local
# coordinates) outside one of them counts as in it, so it is interpolated, not
# missing.  This makes the decision independent of rounding for points that lie
# on the boundary in exact arithmetic, or nearly so: the rest populations of a
# wall node whose mesh velocity is tangential or very small.
EDGE_TOL = 1e-4


def lagrange(p, a):
    """Quadratic Lagrange basis on {-1, 0, 1}: the polynomial of degree 2
    that is 1 at p and 0 at the other two nodes."""
    out = np.ones_like(a, dtype=np.float64)
    for m in (-1.0, 0.0, 1.0):
        if m != p:
            out = out * (a - m) / (p - m)
    return out


def dlagrange(p, a):
    """Derivative of `lagrange(p, .)` at a."""
    out = np.zeros_like(a, dtype=np.float64)
    others = [m for m in (-1.0, 0.0, 1.0) if m != p]
    den = (p - others[0]) * (p - others[1])
    return out + ((a - others[1]) + (a - others[0])) / den


def shape(xi, eta):
    """N_s(xi, eta), s = 0..8, stacked on the first axis."""
    return np.stack([lagrange(LOCAL[s, 0], xi) * lagrange(LOCAL[s, 1], eta) for s in range(9)])


def shape_grad(xi, eta):
    """(dN_s/dxi, dN_s/deta), each stacked on the first axis."""
    dxi = np.stack([dlagrange(LOCAL[s, 0], xi) * lagrange(LOCAL[s, 1], eta) for s in range(9)])
    deta = np.stack([lagrange(LOCAL[s, 0], xi) * dlagrange(LOCAL[s, 1], eta) for s in range(9)])
    return dxi, deta


class UGrid:
    """Connectivity and geometry of an unstructured periodic Q9 mesh."""

    def __init__(self, mesh):
        self.N = mesh.n_nodes
        self.E = mesh.n_elems
        self.elems = np.asarray(mesh.elems, dtype=np.int64)
        Lx, Ly = mesh.period
        sh = np.asarray(mesh.shifts, dtype=np.float64)
        # unwrapped node coordinates of every element
        self.ex = mesh.X[self.elems] + sh[..., 0] * Lx
        self.ey = mesh.Y[self.elems] + sh[..., 1] * Ly
        # patches: the (element, local node) pairs of every node, by element
        # index (a stable sort of all pairs by node)
        node = self.elems.ravel()
        elem = np.repeat(np.arange(self.E), 9)
        loc = np.tile(np.arange(9), self.E)
        order = np.lexsort((elem, node))
        node, elem, loc = node[order], elem[order], loc[order]
        self.count = np.bincount(node, minlength=self.N)
        start = np.concatenate([[0], np.cumsum(self.count)[:-1]])
        rank = np.arange(node.size) - start[node]
        self.P = int(self.count.max())
        self.pe = np.zeros((self.N, self.P), dtype=np.int64)
        self.pa = np.zeros((self.N, self.P), dtype=np.int64)
        self.pm = np.zeros((self.N, self.P), dtype=bool)
        self.pe[node, rank] = elem
        self.pa[node, rank] = loc
        self.pm[node, rank] = True
        self.Wx, self.Wy = self.operator(self.ex, self.ey)
        self.det_min = None

    @staticmethod
    def operator(ex, ey):
        """Element derivative operator at each element's own nodes for element
        node coordinates (ex, ey) [E, 9]: dC/dx at local node a of element e
        = sum_s Wx[e, a, s] C_s (and Wy for d/dy)."""
        E = ex.shape[0]
        Wx = np.zeros((E, 9, 9))
        Wy = np.zeros((E, 9, 9))
        for a in range(9):
            dxi, deta = shape_grad(np.array(LOCAL[a, 0]), np.array(LOCAL[a, 1]))
            x_xi = ex @ dxi
            x_eta = ex @ deta
            y_xi = ey @ dxi
            y_eta = ey @ deta
            det = x_xi * y_eta - y_xi * x_eta
            # [dC/dx, dC/dy] = J^{-T} [dC/dxi, dC/deta]
            Wx[:, a, :] = (y_eta[:, None] * dxi[None, :] - y_xi[:, None] * deta[None, :]) / det[:, None]
            Wy[:, a, :] = (-x_eta[:, None] * dxi[None, :] + x_xi[:, None] * deta[None, :]) / det[:, None]
        return Wx, Wy

    def grad(self, C, W=None):
        """Nodal gradient (dC/dx, dC/dy): the mean over the node's elements of
        the element derivative at the node; W = (Wx, Wy) an operator of other
        (deformed) element coordinates, else the mesh's own."""
        Wx, Wy = W if W is not None else (self.Wx, self.Wy)
        Ce = C[self.elems]                                    # [E, 9]
        gx_e = np.einsum("eas,es->ea", Wx, Ce)                # [E, 9] at each element node
        gy_e = np.einsum("eas,es->ea", Wy, Ce)
        gx = np.where(self.pm, gx_e[self.pe, self.pa], 0.0).sum(axis=1) / self.count
        gy = np.where(self.pm, gy_e[self.pe, self.pa], 0.0).sum(axis=1) / self.count
        return gx, gy

    def locate(self, dx, dy, nodes=None, allow_missing=None):
        """For every node n (or those listed in `nodes`), the element of its
        patch whose bilinear (corner) map holds the point at displacement
        (dx[n], dy[n]) from the node, and the local coordinates there.
        Returns (element, xi, eta).  A point in none of the node's elements
        raises ValueError, unless allow_missing[n] is set (a boundary node,
        whose point then lies outside the mesh: element -1 there, unless it
        lies within EDGE_TOL of one of its elements, which then holds it)."""
        nodes = np.arange(self.N) if nodes is None else np.asarray(nodes, dtype=np.int64)
        M = nodes.size
        found = np.zeros(M, dtype=bool)
        elem = np.full(M, -1, dtype=np.int64)
        XI = np.zeros(M)
        ETA = np.zeros(M)
        dx = np.broadcast_to(dx, (M,))
        dy = np.broadcast_to(dy, (M,))
        pm, pe, pa = self.pm[nodes], self.pe[nodes], self.pa[nodes]
        edge = np.zeros(M, dtype=bool) if allow_missing is None else \
            np.asarray(allow_missing)[nodes]
        for tol, among in ((INSIDE_TOL, np.ones(M, dtype=bool)), (EDGE_TOL, edge)):
            for k in range(self.P):
                # the k-th element of the patches of the nodes not yet placed
                todo = np.flatnonzero(pm[:, k] & ~found & among)
                if todo.size == 0:
                    continue
                e = pe[todo, k]
                a = pa[todo, k]
                # coordinates relative to the node (well conditioned)
                cx = self.ex[e, :4] - self.ex[e, a][:, None]
                cy = self.ey[e, :4] - self.ey[e, a][:, None]
                xi, eta = bilinear_local(cx, cy, dx[todo], dy[todo])
                inside = (np.abs(xi) <= 1 + tol) & (np.abs(eta) <= 1 + tol)
                hit = todo[inside]
                elem[hit] = e[inside]
                XI[hit] = xi[inside]
                ETA[hit] = eta[inside]
                found[hit] = True
        ok = found if allow_missing is None else (found | np.asarray(allow_missing)[nodes])
        if not np.all(ok):
            raise ValueError(f"departure point outside the patch of node {int(nodes[np.argmin(ok)])}")
        return elem, XI, ETA


def bilinear_local(cx, cy, px, py, iters=25):
    """Local (xi, eta) of points P under the bilinear map of quadrilaterals
    with corners (cx, cy)[:, 0..3] at (-1,-1), (1,-1), (1,1), (-1,1); Newton
    from the centre.  Inside a convex element it converges quadratically in a
    few steps; points where it has not settled after `iters` steps (far
    outside, where the extended map can fold) get NaN."""
    xi = np.zeros(px.shape)
    eta = np.zeros(px.shape)
    # the points still moving, with their data kept compact
    live = np.arange(px.size)
    cx, cy, px, py = cx, cy, px, py
    x_, e_ = xi.copy(), eta.copy()
    for _ in range(iters):
        if live.size == 0:
            break
        dxi, deta = _newton_update(cx, cy, px, py, x_, e_)
        x_ = x_ - dxi
        e_ = e_ - deta
        xi[live] = x_
        eta[live] = e_
        moving = ~(np.abs(dxi) + np.abs(deta) < 1e-13)   # quadratic convergence: error ~1e-26 after
        if not np.all(moving):
            live, cx, cy, px, py = live[moving], cx[moving], cy[moving], px[moving], py[moving]
            x_, e_ = x_[moving], e_[moving]
    xi[live] = np.nan
    eta[live] = np.nan
    return xi, eta


def _newton_update(cx, cy, px, py, xi, eta):
    """One Newton correction (dxi, deta) of the bilinear corner map."""
    n = [(1 - xi) * (1 - eta) / 4, (1 + xi) * (1 - eta) / 4,
         (1 + xi) * (1 + eta) / 4, (1 - xi) * (1 + eta) / 4]
    nxi = [-(1 - eta) / 4, (1 - eta) / 4, (1 + eta) / 4, -(1 + eta) / 4]
    neta = [-(1 - xi) / 4, -(1 + xi) / 4, (1 + xi) / 4, (1 - xi) / 4]
    rx = sum(n[c] * cx[:, c] for c in range(4)) - px
    ry = sum(n[c] * cy[:, c] for c in range(4)) - py
    a = sum(nxi[c] * cx[:, c] for c in range(4))
    b = sum(neta[c] * cx[:, c] for c in range(4))
    c_ = sum(nxi[c] * cy[:, c] for c in range(4))
    d = sum(neta[c] * cy[:, c] for c in range(4))
    det = a * d - b * c_
    return (d * rx - b * ry) / det, (-c_ * rx + a * ry) / det


class UnstructuredSolver:
    """Plain FP64 reference of the step on a static periodic Q9 mesh."""

    def __init__(self, mesh, fluid, rho=None, ux=None, uy=None, T=None, correction=True):
        self.grid = UGrid(mesh)
        self.fluid = fluid
        self.correction = correction
        N = self.grid.N
        if rho is None:
            rho = np.full(N, fluid.rho_inf)
            ux = np.full(N, fluid.u_inf[0])
            uy = np.full(N, fluid.u_inf[1])
            T = np.full(N, fluid.T_inf)
        self.f, self.g = L.equilibrium_populations(rho, ux, uy, T, fluid.gamma)
        self.n = 0
        # departure points: element and local coordinates per direction (static mesh)
        self.dep = [None] * L.Q
        for i in range(1, L.Q):
            self.dep[i] = self.grid.locate(-fluid.dt * L.CX[i], -fluid.dt * L.CY[i])

    def correction_force(self):
        fl = self.fluid
        rho, ux, uy, E, T = L.macroscopic(self.f, self.g, fl.gamma)
        omega, _ = L.relaxation_rates(rho, T, fl.mu, fl.Pr, fl.dt)
        dQx, dQy = L.momentum_defect(rho, ux, uy, T)
        gx, _ = self.grid.grad(dQx)
        _, gy = self.grid.grad(dQy)
        Dx = (1.0 / omega - 0.5) * fl.dt * gx
        Dy = (1.0 / omega - 0.5) * fl.dt * gy
        Fx, _ = self.grid.grad(Dx)
        _, Fy = self.grid.grad(Dy)
        return Fx, Fy

    def step(self):
        fl = self.fluid
        if self.correction:
            Fx, Fy = self.correction_force()
        else:
            Fx = Fy = np.zeros(self.grid.N)
        fpost, gpost = L.collide(self.f, self.g, fl.gamma, fl.mu, fl.Pr, fl.dt, Fx, Fy)
        f_new = np.empty_like(fpost)
        g_new = np.empty_like(gpost)
        f_new[0] = fpost[0]
        g_new[0] = gpost[0]
        els = self.grid.elems
        for i in range(1, L.Q):
            e, xi, eta = self.dep[i]
            Nw = shape(xi, eta)                                 # [9, N]
            nodes = els[e]                                       # [N, 9]
            f_new[i] = np.sum(Nw.T * fpost[i][nodes], axis=1)
            g_new[i] = np.sum(Nw.T * gpost[i][nodes], axis=1)
        self.f, self.g = f_new, g_new
        self.n += 1

    def run(self, nsteps):
        for _ in range(nsteps):
            self.step()

    def macroscopic(self):
        return L.macroscopic(self.f, self.g, self.fluid.gamma)


class UnstructuredWallSolver(UnstructuredSolver):
    """The step on an unstructured Q9 mesh round a body, in float64 (paper
    Sec. II.B on its own kind of mesh, with the boundary conditions of
    Sec. III.A, the wall force of Sec. III, the blended mesh of Sec. II.D and
    the rigid body of Sec. IV, staggered).  Test infrastructure only.

    The mesh carries `wall_nodes` (the body polygon, clockwise, so that a
    +90 degree rotation of its tangent points into the fluid) and
    `far_nodes` (the outer boundary).  Readings:

    * a population of a boundary node is missing when its departure point
      lies in none of the node's elements (outside the mesh);
    * far field: all populations of the far-field nodes are set to the
      free-stream equilibrium (the outer circle lies far from the body);
    * wall: missing populations take Grad's approximation (Sec. III.A.1) with
      u_t the wall node's mesh velocity, rho_t, T_t the 9-node interpolation
      at B = X + dt n in the undeformed frame (n the unit normal of the
      lumped wall polygon; the wall's elements lie in the rigid zone, where
      the deformed element is a rigid image of the undeformed one) in the
      wall node's element that holds B, the wall nodes of that element
      carrying the values of the previous level (their new populations are
      being built), and gradients of u, T, E at the wall node by the nodal
      finite-element derivative on the mesh of the new level, the wall nodes
      holding the targets;
    * force: sigma . (n ds) summed over the wall nodes in list order, with
      (n ds)_k = rot90(x_{k+1} - x_{k-1}) / 2 from the polygon neighbours on
      the mesh of the level, the moment about the body's displaced elastic
      axis (Sec. III);
    * a moving body (any dof but fixed): nodes move by the blending of
      Sec. II.D, x = X + (1 - r)(G'(X) - X), r of the distance to the body's
      centre or, with distance blending (the variant Sec. II.D suggests for
      slender bodies), to the closed wall polygon; the departure point of node X is
      X - dt g^{-1}(c_i - V_G) in the undeformed frame (g = dx/dX at the new
      level by the nodal finite-element derivative on the undeformed mesh,
      V_G = (x^{n+1} - x^n)/dt), located among the node's undeformed
      elements every step, for the rest populations (c_0 = 0) too: their
      point X + dt g^{-1} V_G is the node itself only where the mesh does not
      move (there they keep their value); a wall node's rest population whose
      point lies in the body is missing like any other; the correction's
      derivatives are taken on the mesh of level n.
    """

    def __init__(self, mesh, fluid, body, rho=None, ux=None, uy=None, T=None, correction=True):
        from . import body as B
        from .mesh import blend_factors
        self.grid = UGrid(mesh)
        self.fluid = fluid
        self.correction = correction
        self.body = body
        g = self.grid
        N = g.N
        if rho is None:
            rho = np.full(N, fluid.rho_inf)
            ux = np.full(N, fluid.u_inf[0])
            uy = np.full(N, fluid.u_inf[1])
            T = np.full(N, fluid.T_inf)
        self.f, self.g = L.equilibrium_populations(rho, ux, uy, T, fluid.gamma)
        self.n = 0
        self.X = np.asarray(mesh.X, dtype=np.float64)
        self.Y = np.asarray(mesh.Y, dtype=np.float64)
        self.moving = body.dof != B.DOF_FIXED
        self.state = B.initial_state(body)
        self.wall = np.asarray(mesh.wall_nodes, dtype=np.int64)
        # blending coordinate: distance to the centre, or (blend_mode 1) to the
        # closed wall polygon in the undeformed frame
        walls = [(self.X[self.wall], self.Y[self.wall])] if getattr(body, "blend_mode", 0) == 1 else None
        self.r = blend_factors(self.X[None], self.Y[None], [body], walls)[0][0]
        self.far = np.asarray(mesh.far_nodes, dtype=np.int64)
        self.bnd = np.zeros(N, dtype=bool)
        self.bnd[self.wall] = True
        self.bnd[self.far] = True
        self.dep = [None] * L.Q
        if not self.moving:
            for i in range(1, L.Q):
                self.dep[i] = g.locate(-fluid.dt * L.CX[i], -fluid.dt * L.CY[i], allow_missing=self.bnd)
        # lumped wall normals of the undeformed polygon and the points B
        self.xw, self.yw = self.X[self.wall], self.Y[self.wall]
        self.nds_x, self.nds_y = self._nds(self.xw, self.yw)
        nn = np.hypot(self.nds_x, self.nds_y)
        self.B = g.locate(fluid.dt * self.nds_x / nn, fluid.dt * self.nds_y / nn, nodes=self.wall)
        self.history = []
        self.subiterations = 1
        self.relaxation = 1.0
        self.residuals = []

    @staticmethod
    def _nds(xw, yw):
        return -0.5 * (np.roll(yw, -1) - np.roll(yw, 1)), 0.5 * (np.roll(xw, -1) - np.roll(xw, 1))

    def positions(self, state):
        """Node positions on the blended mesh of body state `state`."""
        from .mesh import rigid_displacement
        if not self.moving:
            return self.X.copy(), self.Y.copy()
        dx, dy = rigid_displacement(self.X, self.Y, self.body, state[0], state[1])
        return self.X + (1.0 - self.r) * dx, self.Y + (1.0 - self.r) * dy

    def _operator(self, x, y):
        if not self.moving:
            return None
        g = self.grid
        return g.operator(x[g.elems], y[g.elems])

    def missing(self, i):
        """Mask of the nodes whose population i is missing (last step's
        departure points on a moving mesh; a rest population is never missing
        on a fixed mesh)."""
        if self.dep[i] is None:
            return np.zeros(self.grid.N, dtype=bool)
        return self.dep[i][0] == -1

    def wall_force(self, x=None, y=None, state=None, f=None, gp=None):
        """(F_x, F_y, M_EA) on the body from the populations (f, gp) (default:
        the current ones) on the mesh (x, y) of the body state `state`
        (default: the current level)."""
        from .forces import wall_stress
        if state is None:
            state = self.state
        if x is None:
            x, y = self.positions(state)
        fl = self.fluid
        f = self.f if f is None else f
        gp = self.g if gp is None else gp
        sxx, sxy, syy = wall_stress(f[:, self.wall], gp[:, self.wall], fl.gamma, fl.mu, fl.Pr, fl.dt)
        xw, yw = x[self.wall], y[self.wall]
        nx, ny = self._nds(xw, yw)
        Fx_k = sxx * nx + sxy * ny
        Fy_k = sxy * nx + syy * ny
        rx = xw - self.body.ea[0]
        ry = yw - (self.body.ea[1] + state[0])
        Mz_k = rx * Fy_k - ry * Fx_k
        Fx = Fy = Mz = 0.0
        for k in range(self.wall.size):
            Fx += Fx_k[k]
            Fy += Fy_k[k]
            Mz += Mz_k[k]
        return Fx, Fy, Mz

    def coupling(self, subiterations=1, relaxation=1.0):
        """Strong coupling by sub-iterations, read as on the structured meshes
        (Sec. III names it for low mass ratios without giving an algorithm):
        the step starts from the staggered predictor; each sub-iteration
        streams the post-collision populations of t^n onto the mesh of the
        current body estimate and applies the boundary conditions, takes the
        load of the result, re-solves the body over the step with the load
        varying linearly from F^n to it, and relaxes the estimate towards that
        solution by `relaxation`; the last sub-iteration is accepted.  The
        change |solution - estimate| of each sub-iteration is kept in
        `residuals`.  One sub-iteration is the staggered scheme."""
        assert subiterations >= 1 and 0.0 < relaxation <= 1.0
        self.subiterations = int(subiterations)
        self.relaxation = float(relaxation)

    def step(self):
        from . import body as B
        fl = self.fluid
        g = self.grid
        dt = fl.dt
        x0, y0 = self.positions(self.state)
        Fx_b, Fy_b, Mz_b = self.wall_force(x0, y0, self.state)
        self.history.append([float(self.n), Fx_b, Fy_b, Mz_b, self.state[0], self.state[1]])
        new_state = B.advance(self.body, self.state, Fy_b, Mz_b, (self.n + 1) * dt, dt)
        rho0, _, _, _, T0 = L.macroscopic(self.f[:, self.wall], self.g[:, self.wall], fl.gamma)
        if self.correction:
            W0 = self._operator(x0, y0)
            rho, ux, uy, E, T = L.macroscopic(self.f, self.g, fl.gamma)
            omega, _ = L.relaxation_rates(rho, T, fl.mu, fl.Pr, dt)
            dQx, dQy = L.momentum_defect(rho, ux, uy, T)
            gx, _ = g.grad(dQx, W0)
            _, gy = g.grad(dQy, W0)
            Dx = (1.0 / omega - 0.5) * dt * gx
            Dy = (1.0 / omega - 0.5) * dt * gy
            Fx, _ = g.grad(Dx, W0)
            _, Fy = g.grad(Dy, W0)
        else:
            Fx = Fy = np.zeros(g.N)
        fpost, gpost = L.collide(self.f, self.g, fl.gamma, fl.mu, fl.Pr, dt, Fx, Fy)
        # streaming and boundaries on the mesh of the body estimate; with
        # strong coupling repeated with the structure re-solved against the
        # new load (the reading of `coupling`)
        self.residuals = []
        for it in range(self.subiterations):
            f_new, g_new, x1, y1 = self._fluid(fpost, gpost, x0, y0, rho0, T0, new_state)
            if self.subiterations == 1:
                break
            _, Fy1, M1 = self.wall_force(x1, y1, new_state, f_new, g_new)
            target = B.advance(self.body, self.state, Fy_b, Mz_b, (self.n + 1) * dt, dt, Fy1, M1)
            self.residuals.append(float(np.max(np.abs(target - new_state))))
            if it + 1 < self.subiterations:
                new_state = new_state + self.relaxation * (target - new_state)
        self.f, self.g = f_new, g_new
        self.state = new_state
        self.n += 1

    def _fluid(self, fpost, gpost, x0, y0, rho0, T0, new_state):
        """Streaming of the post-collision populations onto the mesh of body
        state `new_state`, far field and wall: the populations of the new
        level and that mesh."""
        from .boundary import grad_populations
        fl = self.fluid
        g = self.grid
        dt = fl.dt
        x1, y1 = self.positions(new_state)
        VGx, VGy = (x1 - x0) / dt, (y1 - y0) / dt
        f_new = np.full_like(fpost, np.nan)
        g_new = np.full_like(gpost, np.nan)
        # rest populations: their own value where the mesh does not move
        still = (VGx == 0.0) & (VGy == 0.0)
        f_new[0] = np.where(still, fpost[0], np.nan)
        g_new[0] = np.where(still, gpost[0], np.nan)
        if self.moving:
            # departure points in the undeformed frame: X - dt g^{-1}(c - V_G),
            # for the rest populations (c_0 = 0) at the nodes that move
            gxx, gxy = g.grad(x1)
            gyx, gyy = g.grad(y1)
            det = gxx * gyy - gxy * gyx
            for i in range(L.Q):
                ax, ay = L.CX[i] - VGx, L.CY[i] - VGy
                chx = (gyy * ax - gxy * ay) / det
                chy = (-gyx * ax + gxx * ay) / det
                if i == 0:
                    e, xi, eta = g.locate(-dt * chx, -dt * chy, allow_missing=self.bnd)
                    e = np.where(still, -2, e)          # -2: kept, not missing
                    self.dep[0] = (e, xi, eta)
                else:
                    self.dep[i] = g.locate(-dt * chx, -dt * chy, allow_missing=self.bnd)
        for i in range(L.Q):
            if self.dep[i] is None:
                continue
            e, xi, eta = self.dep[i]
            ok = e >= 0
            Nw = shape(xi[ok], eta[ok])
            nodes = g.elems[e[ok]]
            f_new[i, ok] = np.sum(Nw.T * fpost[i][nodes], axis=1)
            g_new[i, ok] = np.sum(Nw.T * gpost[i][nodes], axis=1)
        # far field: free-stream equilibrium
        nf = self.far.size
        fe, ge = L.equilibrium_populations(np.full(nf, fl.rho_inf), np.full(nf, fl.u_inf[0]),
                                           np.full(nf, fl.u_inf[1]), np.full(nf, fl.T_inf), fl.gamma)
        f_new[:, self.far] = fe
        g_new[:, self.far] = ge
        # wall: targets at B and gradients at the wall nodes on the new mesh
        Cv, _ = L.specific_heats(fl.gamma)
        with np.errstate(invalid="ignore", divide="ignore"):
            rho_s, ux_s, uy_s, E_s, T_s = L.macroscopic(np.nan_to_num(f_new), np.nan_to_num(g_new),
                                                        fl.gamma)
        R = rho_s.copy()
        R[self.wall] = rho0
        TT = T_s.copy()
        TT[self.wall] = T0
        eB, xiB, etaB = self.B
        NB = shape(xiB, etaB)                                 # [9, nw]
        nodesB = g.elems[eB]
        rho_t = np.sum(NB.T * R[nodesB], axis=1)
        T_t = np.sum(NB.T * TT[nodesB], axis=1)
        ux_t = VGx[self.wall]
        uy_t = VGy[self.wall]
        E_t = Cv * T_t + 0.5 * (ux_t ** 2 + uy_t ** 2)
        Ux, Uy, Tg, Eg = ux_s.copy(), uy_s.copy(), T_s.copy(), E_s.copy()
        Ux[self.wall] = ux_t
        Uy[self.wall] = uy_t
        Tg[self.wall] = T_t
        Eg[self.wall] = E_t
        W1 = self._operator(x1, y1)
        grads = []
        for F in (Ux, Uy, Tg, Eg):
            gx, gy = g.grad(F, W1)
            grads.append((gx[self.wall], gy[self.wall]))
        fw, gw = grad_populations(rho_t, ux_t, uy_t, T_t, E_t, *grads, fl.gamma, fl.mu, fl.Pr, dt)
        for i in range(L.Q):
            m = self.missing(i)[self.wall]
            f_new[i, self.wall[m]] = fw[i, m]
            g_new[i, self.wall[m]] = gw[i, m]
        assert not np.any(np.isnan(f_new)) and not np.any(np.isnan(g_new))
        return f_new, g_new, x1, y1

