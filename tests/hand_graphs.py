"""Small hand-made graphs whose multilevel behaviour is traced by hand in the
tests that use them (inputs only: no step of the method is computed here)."""
import graphgen


def path_and_heavy_pairs(light, heavy_pairs, heavy_w=2):
    """A path of `light` unit-weight vertices (ids 0..light-1) plus `heavy_pairs`
    disjoint edges between vertices of weight `heavy_w` (ids after the path)."""
    n = light + 2 * heavy_pairs
    edges = [(i, i + 1) for i in range(light - 1)]
    edges += [(light + 2 * h, light + 2 * h + 1) for h in range(heavy_pairs)]
    vw = [1] * light + [heavy_w] * (2 * heavy_pairs)
    return graphgen.from_edges(n, edges, vwgt=vw)


def two_cliques(size):
    """Two disjoint cliques K_size: vertices 0..size-1 and size..2*size-1."""
    edges = [(i, j) for i in range(size) for j in range(i + 1, size)]
    edges += [(i + size, j + size) for i, j in edges]
    return graphgen.from_edges(2 * size, edges)


def star(leaves=7):
    """Centre 0 joined to leaves 1..leaves."""
    return graphgen.from_edges(leaves + 1, [(0, i) for i in range(1, leaves + 1)])


def spider():
    """Centre 0 with three legs 0-1-2-3, 0-4-5-6, 0-7-8-9."""
    return graphgen.from_edges(10, [(0, 1), (1, 2), (2, 3), (0, 4), (4, 5), (5, 6), (0, 7), (7, 8), (8, 9)])


def three_parts():
    """Three components: path 0-1-2-3-4, triangle 5-6-7, edge 8-9."""
    return graphgen.from_edges(10, [(0, 1), (1, 2), (2, 3), (3, 4), (5, 6), (6, 7), (5, 7), (8, 9)])


def path(n, vwgt=None):
    """Path 0-1-...-(n-1)."""
    return graphgen.from_edges(n, [(i, i + 1) for i in range(n - 1)], vwgt=vwgt)
