"""Gmsh MSH 2.2 reading and writing of unstructured 9-node meshes: a mesh
written and read back is the same mesh (coordinates, elements, the wall loop
up to its starting node, the far-field nodes), clockwise element input is
reoriented, and the library accepts what the reader returns."""

import numpy as np
import pytest

from paper_2107_01370_amd.meshio import read_msh, write_msh
from synth.unstructured import cylinder_q9_mesh


@pytest.fixture(scope="module")
def mesh():
    return cylinder_q9_mesh(16, 20.0, 4.0, seed=2)


def test_round_trip(tmp_path, mesh):
    p = tmp_path / "cyl.msh"
    write_msh(str(p), mesh)
    m = read_msh(str(p))
    assert np.array_equal(m.X, mesh.X) and np.array_equal(m.Y, mesh.Y)
    assert np.array_equal(m.elems, mesh.elems)
    # the same clockwise loop, possibly from another starting node
    w = np.asarray(mesh.wall_nodes)
    k = int(np.flatnonzero(w == m.wall_nodes[0])[0])
    assert np.array_equal(np.roll(w, -k), m.wall_nodes)
    assert set(m.far_nodes.tolist()) == set(np.asarray(mesh.far_nodes).tolist())


def test_clockwise_elements_are_reoriented(tmp_path, mesh):
    flipped = mesh.elems[:, [0, 3, 2, 1, 7, 6, 5, 4, 8]]
    bad = cylinder_q9_mesh(16, 20.0, 4.0, seed=2)
    bad.elems = flipped.astype(np.int32)
    p = tmp_path / "cw.msh"
    write_msh(str(p), bad)
    m = read_msh(str(p))
    assert np.array_equal(m.elems, mesh.elems)


def test_the_library_accepts_a_read_mesh(tmp_path, mesh):
    from paper_2107_01370_amd import fsilbm as F
    from synth.unstructured import q9_cylinder_case
    _, fl, body, _ = q9_cylinder_case(16, 20.0, 4.0, seed=2)
    p = tmp_path / "cyl.msh"
    write_msh(str(p), mesh)
    ctx = F.fsi_create(fl, read_msh(str(p)), [body], None)
    F.fsi_destroy(ctx)
