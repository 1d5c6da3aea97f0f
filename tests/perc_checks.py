"""Checks of percolation arrival maps that hold at any size."""
import numpy as np


def check_arrival_local(pore, arr, source, i0=0, j0=0, rows=4096):
    """Arrival passes are the breadth-first distances iff: solid sites hold
    -1; the sources hold 0 and no other site does; every other invaded site
    is one more than its smallest invaded neighbour; and no pore next to an
    invaded site is left out. Checked in row blocks."""
    L = pore.shape[0]
    big = np.int64(1) << 40
    for r0 in range(0, L, rows):
        r1 = min(L, r0 + rows)
        lo, hi = max(0, r0 - 1), min(L, r1 + 1)
        a = arr[lo:hi].astype(np.int64)
        p = pore[lo:hi]
        av = np.where(a < 0, big, a)
        pad = np.full((a.shape[0] + 2, L + 2), big, dtype=np.int64)
        pad[1:-1, 1:-1] = av
        nbmin = np.minimum(np.minimum(pad[:-2, 1:-1], pad[2:, 1:-1]), np.minimum(pad[1:-1, :-2], pad[1:-1, 2:]))
        s0, s1 = r0 - lo, r0 - lo + (r1 - r0)
        a, p, nbmin = a[s0:s1], p[s0:s1], nbmin[s0:s1]
        assert np.all(a[p == 0] == -1), "solid site invaded"
        src = np.zeros(a.shape, dtype=bool)
        if source == 0 and r0 == 0:
            src[0] = p[0] == 1
        elif source == 1 and r0 <= i0 < r1:
            src[i0 - r0, j0] = p[i0 - r0, j0] == 1
        assert np.all(a[src] == 0) and not np.any((a == 0) & ~src), "sources"
        inv = (a > 0)
        assert np.all(nbmin[inv] + 1 == a[inv]), "arrival is not 1 + smallest neighbour"
        assert not np.any((p == 1) & (a < 0) & (nbmin < big)), "pore next to the cluster left out"
