"""Input generators (CPU): the orders the benchmark feeds the library."""
import numpy as np

from paper_1806_05713_amd import synth


def test_cell_sorted_is_a_stable_sort_by_cell():
    s = synth.small_fcc(6, 1.0, 0.1, 3)
    t = synth.cell_sorted(s)
    rs = s.rc + s.skin
    nc = np.floor(s.box / rs).astype(int)
    assert np.all(nc >= 1)
    # the same atoms (a permutation of the rows)
    a = s.pos[np.lexsort(s.pos.T)]
    b = t.pos[np.lexsort(t.pos.T)]
    assert np.array_equal(a, b)
    # cells non-decreasing in z-major order, x fastest
    c = np.minimum((t.pos / (s.box / nc)).astype(int), nc - 1)
    cid = (c[:, 2] * nc[1] + c[:, 1]) * nc[0] + c[:, 0]
    assert np.all(np.diff(cid) >= 0)
    # within a cell the previous (lattice) order is kept
    idx = np.array([np.flatnonzero(np.all(s.pos == p, axis=1))[0] for p in t.pos])
    for k in np.unique(cid):
        assert np.all(np.diff(idx[cid == k]) > 0)


def test_permuted_is_seeded():
    s = synth.small_fcc(4, 1.0, 0.1, 3)
    assert np.array_equal(synth.permuted(s, 5).pos, synth.permuted(s, 5).pos)
    assert not np.array_equal(synth.permuted(s, 5).pos, s.pos)
