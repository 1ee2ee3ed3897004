"""Host setup of general hex meshes in libpmg.so (no GPU needed) against the oracle:
patch vertices, DSATUR patch colors (bit-exact), Dirichlet nodes, patch cells and closure
nodes, a valid cell coloring, the closure layout in the common frame, and the errors of
invalid or unsupported meshes."""
import numpy as np
import pytest

from oracle.hexmesh import HexMesh
from paper_2512_02577_amd import pmg
from paper_2512_02577_amd.inputs import hex_mesh

CASES = [(2, 6, 3, "L"), (2, 8, 2, "hole"), (2, 5, 1, "box"), (3, 4, 2, "L"), (3, 8, 1, "hole"), (3, 4, 4, "box"),
         (3, 3, 7, "box")]


def setup(h, dim, p):
    return pmg.setup_hex(dim, p, h["vertices"], h["cell_vertices"], h["cell_dofs"], h["n_dofs"])


@pytest.mark.parametrize("dim,n,p,shape", CASES)
def test_maps_and_colors_match_the_oracle(dim, n, p, shape):
    h = hex_mesh(dim, n, p, 7, shape=shape, distortion=0.3)
    hp = setup(h, dim, p)
    ex = pmg.hex_export(hp)
    hm = HexMesh(dim, h["vertices"], h["cell_vertices"], p, h["cell_dofs"], h["n_dofs"])
    bnd = hm.boundary_dofs()
    assert np.array_equal(ex["patch_vertex"], hm.patch_vertices())
    assert np.array_equal(ex["patch_color"], hm.patch_colors())
    assert np.array_equal(ex["boundary"].astype(bool), bnd)
    cells = hm.patch_cells()
    assert hp.n_patches == len(cells)
    for j, cs in enumerate(cells):
        assert sorted(ex["patch_cells"][j]) == sorted(cs)
        cl = ex["patch_closure"][j]
        nodes = set(hm.cell_dofs[cs].reshape(-1).tolist())
        assert sorted(cl[cl >= 0].tolist()) == sorted(d for d in nodes if not bnd[d])
    # cells of one color share no vertex
    cc = ex["cell_color"]
    for c in range(hm.n_cells):
        same = np.nonzero(cc == cc[c])[0]
        for c2 in same[same != c]:
            assert not set(hm.cell_vertices[c]) & set(hm.cell_vertices[c2])


@pytest.mark.parametrize("dim,n,p,shape", [(2, 8, 3, "L"), (3, 8, 2, "L"), (3, 4, 3, "box")])
def test_closure_layout_is_a_tensor_grid(dim, n, p, shape):
    # in the common frame the closure is the (2p+1)^dim lattice block around the vertex:
    # its entry (i, j, k) sits at lattice position (vertex - 1 cell) * p + (i, j, k), up to
    # one symmetry of the block shared by the whole mesh
    h = hex_mesh(dim, n, p, 11, shape=shape, distortion=0.0)
    hp = setup(h, dim, p)
    ex = pmg.hex_export(hp)
    N = 2 * p + 1
    lat = h["dof_lattice"]
    seen_steps = set()
    for j in range(hp.n_patches):
        cl = ex["patch_closure"][j].reshape((N,) * dim)  # C order: last axis is x
        if (cl < 0).any():
            continue
        origin = lat[cl[(0,) * dim]]
        steps = []
        for a in range(dim):
            idx = [0] * dim
            idx[dim - 1 - a] = 1
            steps.append(tuple(lat[cl[tuple(idx)]] - origin))
        seen_steps.add(tuple(steps))
        for e in itertools_product(N, dim):
            pos = origin + sum(e[a] * np.array(steps[a]) for a in range(dim))
            assert np.array_equal(lat[cl[tuple(e[::-1])]], pos)
    assert len(seen_steps) == 1


def itertools_product(N, dim):
    import itertools
    return [t[::-1] for t in itertools.product(range(N), repeat=dim)]


def test_rejects_invalid_meshes():
    h = hex_mesh(3, 4, 2, 1, shape="box")
    cv, cd = h["cell_vertices"].copy(), h["cell_dofs"].copy()
    bad = cv.copy()
    bad[0, 0] = len(h["vertices"])
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_hex(3, 2, h["vertices"], bad, cd, h["n_dofs"])
    assert e.value.status == pmg.ERR_INVALID_ARG
    bad = cd.copy()
    bad[0, 13] = (bad[0, 13] + 1) % h["n_dofs"]  # the cell centre node collides with another node
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_hex(3, 2, h["vertices"], cv, bad, h["n_dofs"])
    assert e.value.status == pmg.ERR_INVALID_ARG
    bad = cv.copy()
    bad[0, [0, 1]] = bad[0, [1, 0]]  # two corners swapped: not a hexahedron's order
    with pytest.raises(pmg.PmgError):
        pmg.setup_hex(3, 2, h["vertices"], bad, cd, h["n_dofs"])
    c = pmg.default_config()
    c.local_solver = pmg.LOCAL_DIRECT
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_hex(3, 2, h["vertices"], cv, cd, h["n_dofs"], c)
    assert e.value.status == pmg.ERR_UNSUPPORTED


def test_rejects_a_vertex_without_a_full_patch():
    # a triangle split into three quadrilaterals: the centroid is an interior vertex with
    # three cells, which has no 2x2 vertex patch
    A, B, C = np.array([0.0, 0.0]), np.array([1.0, 0.0]), np.array([0.5, 0.9])
    O = (A + B + C) / 3
    verts = np.array([A, B, C, (A + B) / 2, (B + C) / 2, (C + A) / 2, O])
    # corners in each quad's lexicographic order: (0,0), (1,0), (0,1), (1,1)
    cells = np.array([[0, 3, 5, 6], [1, 4, 3, 6], [2, 5, 4, 6]], dtype=np.int32)
    with pytest.raises(pmg.PmgError) as e:
        pmg.setup_hex(2, 1, verts, cells, cells, 7)
    assert e.value.status == pmg.ERR_UNSUPPORTED


def test_a_domain_without_interior_vertices_has_no_patches():
    # a 3x3 grid without its centre cell: every vertex lies on a boundary face
    h = hex_mesh(2, 3, 2, 2, shape="box", permute=False, orient=False)
    keep = [c for c in range(9) if tuple(h["cell_lattice"][c]) != (1, 1)]
    hp = pmg.setup_hex(2, 2, h["vertices"], h["cell_vertices"][keep], h["cell_dofs"][keep], h["n_dofs"])
    assert hp.n_patches == 0 and hp.n_patch_colors == 0
