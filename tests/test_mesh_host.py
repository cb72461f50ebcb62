"""Host-side validation of triangle-mesh descriptions: cdem_create refuses
each malformed mesh input with CDEM_E_INVALID and a message naming it,
before it touches the device (these run without a GPU)."""
import numpy as np
import pytest

from paper_2307_03445_amd import inputs as I

MAT = (2e7, 0.25, 0.4, 0.6)
SQUARE = [((-0.05, -0.05, 0), (0.05, -0.05, 0), (0.05, 0.05, 0)), ((-0.05, -0.05, 0), (0.05, 0.05, 0), (-0.05, 0.05, 0))]


def _desc(meshes):
    t = I.sphere_template(1.5e-3)
    return I.assemble([t], [0], [(0, 0, 0.01)], [(1, 0, 0, 0)], [(0, 0, 0)], [(0, 0, 0)], [MAT], (0, 0, -9.81),
                      (-0.1, -0.1, -0.1, 0.1, 0.1, 0.1), 1e-6, meshes=meshes)


def _refused(desc, words):
    from paper_2307_03445_amd._lib import CdemError, Scene, load
    try:
        load()
    except OSError as e:  # pragma: no cover - the library is built by build()
        pytest.skip(f"library not built: {e}")
    with pytest.raises(CdemError) as e:
        Scene(desc, torch_allocator=False)
    assert e.value.code == -1 and words in str(e.value), str(e.value)


def test_too_many_meshes():
    _refused(_desc([dict(vertices=SQUARE, mat=MAT)] * 65), "mesh counts")


def test_triangle_of_no_mesh():
    d = _desc([dict(vertices=SQUARE, mat=MAT)])
    d.tri_mesh = np.array([0, 1], np.int32)
    _refused(d, "triangle mesh out of range")


def test_mesh_quaternion_must_be_unit():
    _refused(_desc([dict(vertices=SQUARE, mat=MAT, q=(1.0, 0.01, 0.0, 0.0))]), "mesh state")


def test_mesh_state_must_be_finite():
    _refused(_desc([dict(vertices=SQUARE, mat=MAT, v=(np.nan, 0.0, 0.0))]), "mesh state")


def test_mesh_material_range():
    _refused(_desc([dict(vertices=SQUARE, mat=(2e7, 0.6, 0.4, 0.6))]), "mesh material")


def test_mesh_scene_range():
    _refused(_desc([dict(vertices=SQUARE, mat=MAT, scene=1)]), "mesh scene")


def test_triangle_vertices_must_be_finite():
    d = _desc([dict(vertices=SQUARE, mat=MAT)])
    d.tri_vertex = d.tri_vertex.copy()
    d.tri_vertex[1, 2, 0] = np.inf
    _refused(d, "triangle vertices")
