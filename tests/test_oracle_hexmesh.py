"""Pins of the oracle's general hex-mesh module (oracle/hexmesh.py) to things other than
itself: DSATUR on graphs whose chromatic number is known (and a coloring worked by hand),
the structured-mesh oracle on a box given as a cell list, invariance under renumbering,
rotation and reflection of the cells, and closed-form patch counts of an L-shaped domain."""
import itertools

import numpy as np
import pytest

from oracle.assembly import stiffness_matrix
from oracle.hexmesh import HexLevelSmoother, HexMesh, dsatur
from oracle.mesh import StructuredMesh, boundary_nodes, p_hierarchy, patch_index_sets
from oracle.smoother import LevelSmoother
from paper_2512_02577_amd.inputs import hex_mesh


def graph(n, edges):
    adj = [set() for _ in range(n)]
    for a, b in edges:
        adj[a].add(b)
        adj[b].add(a)
    return adj


def valid(adj, col):
    return all(col[a] != col[b] for a in range(len(adj)) for b in adj[a])


def test_dsatur_by_hand():
    # path 0-1-2-3: all saturations 0, uncolored degrees 1,2,2,1 -> vertex 1 gets color 0;
    # then 2 (saturation 1, one uncolored neighbour) gets 1; then 0 (lowest index among
    # saturation 1, degree 0) gets 1; then 3 gets 0
    assert dsatur(graph(4, [(0, 1), (1, 2), (2, 3)])).tolist() == [1, 0, 1, 0]
    # star with centre 2: the centre first (degree 3), then the leaves 0, 1, 3 in order
    assert dsatur(graph(4, [(2, 0), (2, 1), (2, 3)])).tolist() == [1, 1, 0, 1]


@pytest.mark.parametrize("seed", range(6))
def test_dsatur_exact_on_bipartite_graphs(seed):
    # Brelaz's DSATUR colors every bipartite graph with two colors
    rng = np.random.default_rng(seed)
    na, nb = rng.integers(3, 12, 2)
    edges = [(a, na + b) for a in range(na) for b in range(nb) if rng.random() < 0.4]
    edges.append((0, na))
    adj = graph(na + nb, edges)
    col = dsatur(adj)
    assert valid(adj, col) and col.max() == 1


@pytest.mark.parametrize("n", [3, 5, 7, 9])
def test_dsatur_odd_cycles_and_cliques(n):
    cyc = graph(n, [(i, (i + 1) % n) for i in range(n)])
    col = dsatur(cyc)
    assert valid(cyc, col) and col.max() == 2
    clique = graph(n, list(itertools.combinations(range(n), 2)))
    col = dsatur(clique)
    assert sorted(col.tolist()) == list(range(n))


@pytest.mark.parametrize("seed", range(4))
def test_dsatur_valid_on_random_graphs(seed):
    rng = np.random.default_rng(seed + 10)
    n = 40
    edges = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < 0.15]
    adj = graph(n, edges)
    col = dsatur(adj)
    assert valid(adj, col)
    assert col.max() + 1 <= max(len(a) for a in adj) + 1  # at most max degree + 1 colors


def mk(h, dim, p):
    return HexMesh(dim, h["vertices"], h["cell_vertices"], p, h["cell_dofs"], h["n_dofs"])


@pytest.mark.parametrize("dim,n,p", [(2, 4, 3), (2, 3, 7), (3, 3, 2), (3, 2, 4)])
def test_box_as_cell_list_matches_the_structured_oracle(dim, n, p):
    h = hex_mesh(dim, n, p, 5, shape="box", distortion=0.3, permute=False, orient=False)
    hm = mk(h, dim, p)
    sm = StructuredMesh(dim, n, h["vertices"])  # same vertices, lattice order
    assert abs(hm.stiffness() - stiffness_matrix(sm, p)).max() <= 1e-14
    assert np.array_equal(hm.boundary_dofs(), boundary_nodes(dim, n, p))
    hs = HexLevelSmoother(hm, p_hierarchy(p))
    ls = LevelSmoother(sm, p_hierarchy(p))
    interior = patch_index_sets(dim, n, p)[1]
    for j in range(len(interior)):
        assert np.array_equal(hs.interior[-1][j], np.sort(interior[j]))
    assert hs.n_colors == (2 ** dim if n >= 3 else 1)  # DSATUR finds the optimal coloring of the box
    rng = np.random.default_rng(1)
    u, b = rng.uniform(-1, 1, hm.n_dofs), rng.uniform(-1, 1, hm.n_dofs)
    order = hs.patch_order()
    assert abs(hs.smooth(u, b, order=order) - ls.smooth(u, b, order=order)).max() <= 1e-13


@pytest.mark.parametrize("dim,n,p,shape", [(2, 6, 3, "L"), (3, 4, 2, "L"), (2, 8, 2, "hole")])
def test_renumbered_rotated_mesh_gives_the_same_operator_and_smoother(dim, n, p, shape):
    ha = hex_mesh(dim, n, p, 9, shape=shape, distortion=0.3, permute=False, orient=False)
    hb = hex_mesh(dim, n, p, 9, shape=shape, distortion=0.3, permute=True, orient=True)
    ma, mb = mk(ha, dim, p), mk(hb, dim, p)
    m = p * n + 1

    def key(lat):
        return sum(lat[:, a] * m ** a for a in range(dim))

    # node ib of mesh b is node ia of mesh a when their lattice positions agree
    ka, kb = key(ha["dof_lattice"]), key(hb["dof_lattice"])
    a_of_b = np.argsort(ka)[np.searchsorted(np.sort(ka), kb)]
    Aa, Ab = ma.stiffness(), mb.stiffness()
    assert abs(Ab - Aa[a_of_b][:, a_of_b]).max() <= 1e-14
    assert np.array_equal(mb.boundary_dofs(), ma.boundary_dofs()[a_of_b])
    # patches matched by their cells' lattice positions; one sweep in the same order
    sa, sb = HexLevelSmoother(ma, p_hierarchy(p)), HexLevelSmoother(mb, p_hierarchy(p))

    def pkey(hh, cells):
        return tuple(sorted(tuple(x) for x in hh["cell_lattice"][cells]))

    pos_b = {pkey(hb, c): j for j, c in enumerate(sb.cells)}
    order_a = sa.patch_order()
    order_b = [pos_b[pkey(ha, sa.cells[j])] for j in order_a]
    rng = np.random.default_rng(3)
    u, b = rng.uniform(-1, 1, ma.n_dofs), rng.uniform(-1, 1, ma.n_dofs)
    ua = sa.smooth(u, b, order=order_a)
    ub = sb.smooth(u[a_of_b], b[a_of_b], order=order_b)
    assert abs(ub - ua[a_of_b]).max() <= 1e-13


@pytest.mark.parametrize("dim,n", [(2, 6), (2, 8), (3, 4), (3, 6)])
def test_l_shape_patch_count(dim, n):
    # interior lattice vertices of the L: (n-1)^2 - (n/2)^2 per plane, n-1 planes in 3D
    h = hex_mesh(dim, n, 1, 0, shape="L")
    hm = mk(h, dim, 1)
    per_plane = (n - 1) ** 2 - (n // 2) ** 2
    assert len(hm.patch_vertices()) == per_plane * ((n - 1) if dim == 3 else 1)
    assert hm.n_cells == (n ** 2 - (n // 2) ** 2) * (n if dim == 3 else 1)
