"""Cross-checks between the C oracle, the NumPy oracle and the light-cone
window oracle. The two full oracles are independent codings of the same
reading of Section 2.2, so they must agree bit for bit."""
import numpy as np
import pytest

from oracle import mini


@pytest.mark.parametrize("L,J,h,T,seed,p_up", [
    (2, 1.0, 0.0, 2.269185, 1, 0.5),
    (4, 1.0, 0.1, 1.5, 7, 0.5),
    (8, 1.0, 0.0, 3.5, 11, 1.0),
    (10, 0.7, -0.2, 2.0, 2 ** 33 + 5, 0.3),
    (16, 1.0, 0.05, 2.269185, 123, 0.5),
    (64, 1.0, 0.0, 2.269185, 1, 0.5),
])
def test_c_and_numpy_oracles_agree(oracle, L, J, h, T, seed, p_up):
    a = oracle.init(L, seed, p_up)
    b = mini.initial_state(L, seed, p_up)
    assert np.array_equal(a, b)
    n = 60 if L <= 16 else 25
    Ba, Ma = oracle.run(a, J, h, T, seed, 3, n)
    Bb, Mb = mini.run(b, J, h, T, seed, 3, n)
    assert np.array_equal(a, b)
    assert np.array_equal(Ba, Bb) and np.array_equal(Ma, Mb)


@pytest.mark.parametrize("L,n,i0,j0,W", [(48, 3, 5, 40, 20), (40, 4, 30, 30, 25), (32, 2, 0, 0, 32)])
def test_window_oracle_matches_full_lattice(oracle, L, n, i0, j0, W):
    """The light-cone window run gives the true values wherever it reports
    them valid, and the valid region is the expected shrunken window."""
    J, h, T, seed = 1.0, 0.05, 2.269185, 77
    full = oracle.init(L, seed, 0.5)
    win = oracle.init_window(L, seed, 0.5, i0, j0, W)
    rows = (np.arange(W) + i0) % L
    cols = (np.arange(W) + j0) % L
    assert np.array_equal(win, full[np.ix_(rows, cols)])
    oracle.run(full, J, h, T, seed, 0, n)
    win, valid = oracle.window_run(L, J, h, T, seed, 0, n, i0, j0, win)
    truth = full[np.ix_(rows, cols)]
    assert np.array_equal(win[valid], truth[valid])
    core = slice(2 * n, W - 2 * n)
    if W > 4 * n:
        assert valid[core, core].all()


def test_hash_is_fnv1a_of_canonical_bytes(oracle):
    """FNV-1a 64 (Fowler, Noll, Vo): published test values for the empty
    string and "a", and the canonical byte encoding +1 -> 0x01, -1 -> 0xFF."""
    import ctypes
    lib = oracle.lib
    assert lib.oracle_fnv1a64(None, 0) == 0xcbf29ce484222325
    buf = (ctypes.c_uint8 * 1)(ord("a"))
    assert lib.oracle_fnv1a64(ctypes.cast(buf, ctypes.c_void_p), 1) == 0xaf63dc4c8601ec8c
    s = np.array([[1, -1], [-1, 1]], dtype=np.int8)
    h = 0xcbf29ce484222325
    for byte in (0x01, 0xFF, 0xFF, 0x01):
        h = ((h ^ byte) * 0x100000001b3) & 0xFFFFFFFFFFFFFFFF
    assert oracle.fnv1a64(s) == h
