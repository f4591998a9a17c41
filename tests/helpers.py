"""Checks shared by the test modules (no solver arithmetic)."""
import numpy as np


def is_cover(g, cover) -> bool:
    """Every edge of g has an endpoint in cover."""
    c = np.zeros(g.n, bool)
    cover = np.asarray(cover, dtype=np.int64)
    if cover.size and (cover.min() < 0 or cover.max() >= g.n):
        return False
    c[cover] = True
    u, v = g.edges()
    return bool(np.all(c[u] | c[v]))


def assert_cover(g, cover, size=None, at_most=None):
    cover = np.asarray(cover, dtype=np.int64)
    assert np.unique(cover).size == cover.size, "cover repeats a vertex"
    assert is_cover(g, cover), "returned set leaves an edge uncovered"
    if size is not None:
        assert cover.size == size, (cover.size, size)
    if at_most is not None:
        assert cover.size <= at_most, (cover.size, at_most)
