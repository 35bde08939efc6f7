"""Unstructured 9-node quadrilateral meshes from and to Gmsh's ASCII format
(MSH 2.2), for the library's Q9 topology.

A mesh from a finite-element mesher carries second-order quadrilaterals
(Gmsh element type 10, nodes: the four corners counter-clockwise, the
midpoints of edges 0-1, 1-2, 2-3, 3-0, the centre: the library's element node
order) and, on its boundary, second-order lines (type 8: two end nodes, then
the midpoint) grouped by physical names.  `read_msh` returns a mesh the
library accepts: node coordinates, the elements (oriented counter-clockwise),
and, from the lines of the physical groups named for the wall and the far
field, the wall polygon as a closed clockwise node loop and the far-field
nodes.  The library needs straight-sided elements (edge and centre nodes where
the corners' bilinear map puts them; in Gmsh: Mesh.SecondOrderLinear = 1).
Periodic meshes are not read (their element shifts have no counterpart here).
"""

from __future__ import annotations

import numpy as np

TOPO_Q9 = 4
MSH_LINE3 = 8
MSH_QUAD9 = 10


class Q9Mesh:
    """A static unstructured 9-node mesh in the form `Simulation` takes."""

    topo = TOPO_Q9
    nj = 1

    def __init__(self, X, Y, elems, wall_nodes=None, far_nodes=None, info=None):
        self.X = np.ascontiguousarray(X, dtype=np.float64)
        self.Y = np.ascontiguousarray(Y, dtype=np.float64)
        self.elems = np.ascontiguousarray(elems, dtype=np.int32)
        self.shifts = np.zeros(self.elems.shape + (2,), dtype=np.int8)
        self.period = (0.0, 0.0)
        self.wall_nodes = None if wall_nodes is None else np.asarray(wall_nodes, dtype=np.int32)
        self.far_nodes = None if far_nodes is None else np.asarray(far_nodes, dtype=np.int32)
        self.info = dict(info or {})

    @property
    def n_nodes(self) -> int:
        return int(self.X.size)

    @property
    def n_elems(self) -> int:
        return int(self.elems.shape[0])

    @property
    def ni(self) -> int:
        return self.n_nodes

    shift_i = (0.0, 0.0)
    shift_j = (0.0, 0.0)

    def interleaved(self) -> np.ndarray:
        return np.stack([self.X, self.Y], axis=-1)[None]


def _corner_area(x, y, el):
    cx, cy = x[el[:, :4]], y[el[:, :4]]
    return 0.5 * np.sum(cx * np.roll(cy, -1, axis=1) - np.roll(cx, -1, axis=1) * cy, axis=1)


def _orient(x, y, el):
    """Elements with clockwise corners reversed (corners 0 3 2 1, edges 7 6 5
    4, centre 8), so that every element is counter-clockwise."""
    el = el.copy()
    flip = _corner_area(x, y, el) < 0
    el[flip] = el[flip][:, [0, 3, 2, 1, 7, 6, 5, 4, 8]]
    return el


def _loop(lines):
    """The closed node loop (end, mid, end, mid, ...) through second-order
    boundary lines [(a, b, mid), ...] that form one cycle."""
    adj = {}
    for a, b, m in lines:
        adj.setdefault(a, []).append((b, m))
        adj.setdefault(b, []).append((a, m))
    if any(len(v) != 2 for v in adj.values()):
        raise ValueError("wall lines do not form one closed loop")
    start = lines[0][0]
    loop, prev, cur = [], None, start
    for _ in range(len(lines)):
        (b0, m0), (b1, m1) = adj[cur]
        # on to the neighbour not come from (from the start: the first)
        b, m = (b0, m0) if prev is None or b0 != prev else (b1, m1)
        loop += [cur, m]
        prev, cur = cur, b
    if cur != start or len(set(loop)) != len(loop):
        raise ValueError("wall lines do not form one closed loop")
    return np.array(loop, dtype=np.int64)


def read_msh(path: str, wall: str = "wall", far: str = "farfield") -> Q9Mesh:
    """Read a Gmsh MSH 2.2 ASCII file: 9-node quadrilaterals and the
    second-order boundary lines of the physical groups `wall` and `far`
    (either may be absent; a mesh without both boundaries must close on
    itself, which only a periodic mesh does and this reader does not take)."""
    with open(path) as fh:
        lines = [ln.strip() for ln in fh]
    it = iter(range(len(lines)))
    names = {}
    node_ids, xs, ys = [], [], []
    quads, blines = [], []
    for i in it:
        ln = lines[i]
        if ln == "$MeshFormat":
            ver = lines[i + 1].split()
            if not ver[0].startswith("2") or ver[1] != "0":
                raise ValueError("only MSH 2.x ASCII files are read")
        elif ln == "$PhysicalNames":
            n = int(lines[i + 1])
            for k in range(n):
                dim, tag, name = lines[i + 2 + k].split(maxsplit=2)
                names[(int(dim), int(tag))] = name.strip('"')
        elif ln == "$Nodes":
            n = int(lines[i + 1])
            for k in range(n):
                p = lines[i + 2 + k].split()
                node_ids.append(int(p[0]))
                xs.append(float(p[1]))
                ys.append(float(p[2]))
        elif ln == "$Elements":
            n = int(lines[i + 1])
            for k in range(n):
                p = [int(v) for v in lines[i + 2 + k].split()]
                etype, ntags = p[1], p[2]
                tags, nodes = p[3:3 + ntags], p[3 + ntags:]
                if etype == MSH_QUAD9:
                    quads.append(nodes)
                elif etype == MSH_LINE3:
                    blines.append((names.get((1, tags[0]), str(tags[0])) if tags else "", nodes))
    if not quads:
        raise ValueError("no 9-node quadrilaterals (Gmsh element type 10) in the file")
    index = {nid: k for k, nid in enumerate(node_ids)}
    x, y = np.array(xs), np.array(ys)
    el = _orient(x, y, np.array([[index[v] for v in q] for q in quads], dtype=np.int64))
    wl = [(index[a], index[b], index[m]) for name, (a, b, m) in blines if name == wall]
    fl = [(index[a], index[b], index[m]) for name, (a, b, m) in blines if name == far]
    wall_nodes = far_nodes = None
    if wl:
        loop = _loop(wl)
        # clockwise: a +90 degree rotation of the tangent points away from the body
        if 0.5 * np.sum(x[loop] * np.roll(y[loop], -1) - np.roll(x[loop], -1) * y[loop]) > 0:
            loop = loop[::-1]
        wall_nodes = loop
    if fl:
        far_nodes = np.unique(np.array(fl).ravel())
    return Q9Mesh(x, y, el, wall_nodes, far_nodes, info={"source": str(path)})


def write_msh(path: str, mesh, wall: str = "wall", far: str = "farfield") -> None:
    """Write a bounded 9-node mesh (no element shifts) as Gmsh MSH 2.2 ASCII:
    its quadrilaterals, and its boundary edges as second-order lines in the
    physical groups `wall` (edges whose three nodes are wall nodes) and `far`
    (far-field nodes)."""
    el = np.asarray(mesh.elems, dtype=np.int64)
    if np.any(np.asarray(getattr(mesh, "shifts", np.zeros(1)))):
        raise ValueError("periodic meshes (element shifts) are not written")
    edges = {}
    for e in el:
        for a, b, m in ((0, 1, 4), (1, 2, 5), (2, 3, 6), (3, 0, 7)):
            key = (min(e[a], e[b]), max(e[a], e[b]))
            edges.setdefault(key, []).append((e[a], e[b], e[m]))
    wset = set(np.asarray(mesh.wall_nodes).tolist()) if getattr(mesh, "wall_nodes", None) is not None else set()
    fset = set(np.asarray(mesh.far_nodes).tolist()) if getattr(mesh, "far_nodes", None) is not None else set()
    bl = []
    for key, uses in edges.items():
        if len(uses) != 1:
            continue
        a, b, m = uses[0]
        if {a, b, m} <= wset:
            bl.append((1, (a, b, m)))
        elif {a, b, m} <= fset:
            bl.append((2, (a, b, m)))
    with open(path, "w") as fh:
        fh.write("$MeshFormat\n2.2 0 8\n$EndMeshFormat\n")
        fh.write(f'$PhysicalNames\n3\n1 1 "{wall}"\n1 2 "{far}"\n2 3 "fluid"\n$EndPhysicalNames\n')
        fh.write(f"$Nodes\n{mesh.n_nodes}\n")
        for k in range(mesh.n_nodes):
            fh.write(f"{k + 1} {mesh.X[k]:.17g} {mesh.Y[k]:.17g} 0\n")
        fh.write("$EndNodes\n")
        fh.write(f"$Elements\n{len(bl) + el.shape[0]}\n")
        k = 1
        for tag, (a, b, m) in bl:
            fh.write(f"{k} {MSH_LINE3} 2 {tag} {tag} {a + 1} {b + 1} {m + 1}\n")
            k += 1
        for e in el:
            fh.write(f"{k} {MSH_QUAD9} 2 3 3 " + " ".join(str(v + 1) for v in e) + "\n")
            k += 1
        fh.write("$EndElements\n")
