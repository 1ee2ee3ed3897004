"""Pins of the oracle's numbering, patch index sets, colors and level rules."""
import itertools
import os

import numpy as np
import pytest

from oracle.mesh import (boundary_nodes, cell_dofs, hlevel_sizes, p_hierarchy, patch_colors,
                         patch_index_sets, patch_vertices)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return [line.split() for line in f if line.strip() and not line.startswith("#")]


def lex(ranges):
    """Tuples of the product of ranges, x (first range) fastest."""
    return [tuple(reversed(t)) for t in itertools.product(*reversed(ranges))]


def node_index(ijk, m):
    idx, stride = 0, 1
    for a in ijk:
        idx += a * stride
        stride *= m
    return idx


@pytest.mark.parametrize("dim,n,p", [(2, 3, 1), (2, 4, 3), (3, 2, 2), (3, 3, 1), (3, 2, 4)])
def test_cell_dofs_follow_lexicographic_contract(dim, n, p):
    cd = cell_dofs(dim, n, p)
    m = p * n + 1
    assert cd.shape == (n**dim, (p + 1) ** dim)
    for c in range(n**dim):
        ci = [(c // n**a) % n for a in range(dim)]
        for loc in range(cd.shape[1]):
            li = [(loc // (p + 1) ** a) % (p + 1) for a in range(dim)]
            assert cd[c, loc] == node_index([p * ci[a] + li[a] for a in range(dim)], m)


@pytest.mark.parametrize("dim,n,p", [(2, 4, 3), (2, 5, 2), (3, 3, 2), (3, 4, 1)])
def test_patch_sets_follow_contract(dim, n, p):
    clo, inn = patch_index_sets(dim, n, p)
    verts = patch_vertices(dim, n)
    m = p * n + 1
    assert len(verts) == (n - 1) ** dim
    assert clo.shape[1] == (2 * p + 1) ** dim and inn.shape[1] == (2 * p - 1) ** dim
    for j, v in enumerate(verts):
        # patch index formula
        assert j == node_index([v[a] - 1 for a in range(dim)], n - 1)
        rng_c = [range(p * (v[a] - 1), p * (v[a] + 1) + 1) for a in range(dim)]
        assert list(clo[j]) == [node_index(t, m) for t in lex(rng_c)]
        rng_i = [range(p * (v[a] - 1) + 1, p * (v[a] + 1)) for a in range(dim)]
        exp_i = [node_index(t, m) for t in lex(rng_i)]
        assert list(inn[j]) == exp_i


def test_figure_p3_2d_patch_has_25_interior_dofs():
    # Figure (patch-smoother steps): a 2D Q3 vertex patch has 5 x 5 interior DoFs and
    # each of its four cells 4 x 4 DoFs
    _, inn = patch_index_sets(2, 2, 3)
    assert inn.shape == (1, 25)
    assert cell_dofs(2, 2, 3).shape[1] == 16


@pytest.mark.parametrize("dim", [2, 3])
def test_p1_patch_has_single_interior_dof(dim):
    # Sec. 3.2: at p = 1 the patch interior is the central vertex only
    _, inn = patch_index_sets(dim, 4, 1)
    assert inn.shape[1] == 1
    verts = patch_vertices(dim, 4)
    for j, v in enumerate(verts):
        assert inn[j, 0] == node_index(list(v), 5)


def test_paper_problem_sizes():
    # Tables 2 and 4: refinement r of one coarse patch (2^3 cells) gives n = 2^(r+1)
    for row in _rows("paper_problem_sizes.txt"):
        r, patches, *dofs = map(int, row)
        n = 2 ** (r + 1)
        assert len(patch_vertices(3, n)) == patches if n <= 16 else (n - 1) ** 3 == patches
        for p, nd in zip((2, 3, 4, 7), dofs):
            assert (p * n + 1) ** 3 == nd
    # brute-force node count on the smallest case
    assert len(boundary_nodes(3, 8, 2)) == 4913


def test_paper_p_hierarchy():
    for row in _rows("paper_p_hierarchy.txt"):
        p, *levels = map(int, row)
        assert p_hierarchy(p) == levels
    assert p_hierarchy(2) == [1, 2] and p_hierarchy(8) == [1, 3, 7, 8] and p_hierarchy(1) == [1]


def test_hlevel_sizes():
    assert hlevel_sizes(8) == [2, 4, 8]
    assert hlevel_sizes(32) == [2, 4, 8, 16, 32]
    assert hlevel_sizes(48) == [3, 6, 12, 24, 48]
    assert hlevel_sizes(5) == [5]
    assert hlevel_sizes(16, 2) == [8, 16]


@pytest.mark.parametrize("dim,n,p", [(2, 6, 2), (3, 4, 2), (3, 5, 1)])
def test_parity_colors_are_race_free(dim, n, p):
    # Sec. 4.4 colors patches so that patches of one color can be updated in parallel.
    # The condition for a parallel update to equal any sequential order is that no
    # patch's interior meets another same-color patch's closure.
    clo, inn = patch_index_sets(dim, n, p)
    col = patch_colors(dim, n)
    assert set(col.tolist()) == set(range(2**dim)) or n == 2
    for c in range(2**dim):
        js = np.nonzero(col == c)[0]
        for a in js:
            sa = set(inn[a].tolist())
            for b in js:
                if a != b:
                    assert not (sa & set(clo[b].tolist()))


def test_parity_coloring_is_minimal_in_the_interior_reading():
    # Two patches whose vertices differ by one in one direction conflict, so the
    # coloring needs at least 2^dim colors.
    clo, inn = patch_index_sets(2, 4, 2)
    verts = patch_vertices(2, 4)
    j0 = [j for j, v in enumerate(verts) if tuple(v) == (1, 1)][0]
    j1 = [j for j, v in enumerate(verts) if tuple(v) == (2, 2)][0]
    assert set(inn[j0].tolist()) & set(clo[j1].tolist())
