"""Pins of the oracle's percolation model (Section 2.3): the medium draw
against its distribution and the threshold construction, the invasion
against library graph routines (connected-component labelling and
breadth-first shortest paths), a closed form on the 2 x 2 medium, and the
2D site-percolation threshold p_c ~ 0.592746 that Section 5 quotes."""
import itertools

import numpy as np
import pytest
from scipy import ndimage
from scipy.sparse import csgraph, csr_matrix

from tests.perc_checks import check_arrival_local


def _pore_graph(pore):
    """Sparse adjacency of pores (4-neighbour, open boundaries)."""
    L = pore.shape[0]
    idx = np.arange(L * L).reshape(L, L)
    rows, cols = [], []
    for a, b in ((idx[:, :-1], idx[:, 1:]), (idx[:-1, :], idx[1:, :])):
        m = (pore.ravel()[a.ravel()] == 1) & (pore.ravel()[b.ravel()] == 1)
        rows += [a.ravel()[m], b.ravel()[m]]
        cols += [b.ravel()[m], a.ravel()[m]]
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    return csr_matrix((np.ones(len(r)), (r, c)), shape=(L * L, L * L))


@pytest.mark.parametrize("L,P,seed", [(64, 0.3, 1), (97, 0.6, 2), (256, 0.5927, 3)])
def test_medium_fraction(oracle, L, P, seed):
    pore = oracle.perc_medium(L, P, seed)
    n = L * L
    assert abs(pore.sum() - P * n) < 5 * np.sqrt(n * P * (1 - P))


def test_medium_extremes_and_nesting(oracle):
    """P = 0 gives no pores, P = 1 only pores, and with one seed the pores
    at a lower porosity are a subset of those at a higher one (each site
    compares the same draw against a larger threshold)."""
    assert oracle.perc_medium(33, 0.0, 5).sum() == 0
    assert oracle.perc_medium(33, 1.0, 5).sum() == 33 * 33
    prev = oracle.perc_medium(40, 0.2, 9)
    for P in (0.4, 0.59, 0.6, 0.9):
        cur = oracle.perc_medium(40, P, 9)
        assert np.all(cur >= prev)
        prev = cur


def test_medium_keyed_by_row_major_index(oracle):
    """Draws are keyed by the row-major site index i*L + j, so row 0 of a
    16 x 16 medium equals the first 16 sites of row 0 of a 32 x 32 one."""
    a = oracle.perc_medium(16, 0.5, 7)
    b = oracle.perc_medium(32, 0.5, 7)
    assert np.array_equal(a[0], b[0, :16])
    assert not np.array_equal(a[1], b[1, :16])


@pytest.mark.parametrize("L,P,seed", [(8, 0.6, 1), (31, 0.59, 2), (64, 0.62, 3), (50, 0.7, 4), (40, 0.4, 5)])
def test_cluster_and_arrival_match_library(oracle, L, P, seed):
    """The invaded set is the union of the 4-connected pore components that
    touch row 0 (scipy.ndimage.label), and arrival passes are the
    breadth-first distances from the row-0 pores (scipy csgraph)."""
    pore = oracle.perc_medium(L, P, seed)
    arr = oracle.perc_invade(pore, 0)
    lab, _ = ndimage.label(pore, structure=[[0, 1, 0], [1, 1, 1], [0, 1, 0]])
    top = set(lab[0][lab[0] > 0].tolist())
    expect = np.isin(lab, list(top)) & (lab > 0)
    assert np.array_equal(arr >= 0, expect)
    src = np.flatnonzero(pore[0] == 1)
    if len(src):
        d = csgraph.shortest_path(_pore_graph(pore), unweighted=True, indices=src, directed=False).min(axis=0)
        d = np.where(np.isinf(d), -1, d).astype(np.int64).reshape(L, L)
        d[pore == 0] = -1
        assert np.array_equal(arr, d)
    else:
        assert np.all(arr == -1)


def test_point_source_matches_library(oracle):
    pore = oracle.perc_medium(45, 0.65, 8)
    i0, j0 = 22, 20
    pore[i0, j0] = 1
    arr = oracle.perc_invade(pore, 1, i0, j0)
    d = csgraph.shortest_path(_pore_graph(pore), unweighted=True, indices=[i0 * 45 + j0], directed=False)[0]
    d = np.where(np.isinf(d), -1, d).astype(np.int64).reshape(45, 45)
    assert np.array_equal(arr, d)
    pore[i0, j0] = 0
    assert np.all(oracle.perc_invade(pore, 1, i0, j0) == -1)


def test_two_by_two_spanning_closed_form(oracle):
    """On the 2 x 2 medium invaded from the top row, a pore path reaches the
    bottom row iff one of the two columns is all pore, so the spanning
    probability is 2 p^2 - p^4: summing the oracle's verdict over all 16
    media with their probabilities must give exactly that polynomial."""
    verdicts = {}
    for bits in itertools.product((0, 1), repeat=4):
        pore = np.array(bits, dtype=np.uint8).reshape(2, 2)
        verdicts[bits] = oracle.perc_summary(oracle.perc_invade(pore, 0))[2] & 1
    for p in (0.1, 0.35, 0.5, 0.8):
        prob = sum(v * np.prod([p if b else 1 - p for b in bits]) for bits, v in verdicts.items())
        assert abs(prob - (2 * p ** 2 - p ** 4)) < 1e-15


def test_summary(oracle):
    pore = np.zeros((5, 5), dtype=np.uint8)
    pore[:, 2] = 1  # one open column
    arr = oracle.perc_invade(pore, 0)
    assert oracle.perc_summary(arr) == (5, 4, 1)
    pore[2, :] = 1  # plus one open row
    arr = oracle.perc_invade(pore, 0)
    assert oracle.perc_summary(arr) == (9, 4, 3)
    assert oracle.perc_summary(oracle.perc_invade(np.zeros((5, 5), np.uint8), 0)) == (0, 0, 0)


def _span_threshold(oracle, L, seed, lo=0.3, hi=0.9, iters=14):
    """Smallest porosity at which the medium of this seed spans (the pore
    sets are nested in P, and spanning is monotone in the pore set)."""
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        sp = oracle.perc_summary(oracle.perc_invade(oracle.perc_medium(L, mid, seed), 0))[2] & 1
        lo, hi = (lo, mid) if sp else (mid, hi)
    return hi


def test_spanning_threshold_near_pc(oracle):
    """The porosity at which half of the 128 x 128 media span (the median of
    the per-seed spanning thresholds) lies near the 2D site-percolation
    threshold 0.592746."""
    th = [_span_threshold(oracle, 128, s) for s in range(120)]
    med = float(np.median(th))
    assert abs(med - 0.592746) < 0.008, med


def test_local_check_rejects_wrong_maps(oracle):
    """The local check itself: it passes the oracle's map and fails maps
    with one site off by one, one pore dropped, or one extra zero."""
    pore = oracle.perc_medium(200, 0.65, 3)
    arr = oracle.perc_invade(pore, 0)
    check_arrival_local(pore, arr, 0, rows=37)
    k = np.argwhere(arr > 3)[10]
    for mutate in (lambda a: a.__setitem__(tuple(k), a[tuple(k)] + 1),
                   lambda a: a.__setitem__(tuple(k), -1),
                   lambda a: a.__setitem__(tuple(k), 0)):
        bad = arr.copy()
        mutate(bad)
        with pytest.raises(AssertionError):
            check_arrival_local(pore, bad, 0, rows=37)
