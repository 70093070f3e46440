"""Window slicing of the sliding-window fitter (host logic, no GPU): every
window against a plain per-stream loop."""

import numpy as np

from paper_2411_10258_amd import stream


def _streams(seed, counts, M=5):
    g = np.random.default_rng(seed)
    off = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    t = np.concatenate([np.sort(g.uniform(0, 50, n)) for n in counts])
    dim = g.integers(0, M, off[-1]).astype(np.int32)
    return stream.Streams(M, off, t, dim)


def test_window_count():
    assert stream.n_windows(np.array([10, 25]), 4, 3) == 3
    assert stream.n_windows(np.array([10, 25]), 10, 3) == 1
    assert stream.n_windows(np.array([10, 25]), 11, 3) == 0
    assert stream.n_windows(np.array([], np.int64), 4, 3) == 0


def test_windows_match_plain_slicing():
    s = _streams(3, [40, 57, 33])
    L, stride = 12, 5
    K = stream.n_windows(s.counts(), L, stride)
    assert K == (33 - 12) // 5 + 1
    for k in range(K):
        off, t, dim, T = stream.window_batch(s, k, L, stride)
        assert list(off) == [0, L, 2 * L, 3 * L]
        for j in range(s.S):
            a = s.offsets[j] + k * stride
            ev_t = s.t[a:a + L]
            assert np.array_equal(t[j * L:(j + 1) * L], ev_t - ev_t[0])
            assert np.array_equal(dim[j * L:(j + 1) * L], s.dim[a:a + L])
            assert T[j] == ev_t[-1] - ev_t[0]
            assert np.all(np.diff(t[j * L:(j + 1) * L]) >= 0) and t[j * L] == 0.0


def test_degenerate_window_gets_positive_length():
    s = stream.Streams(2, np.array([0, 4]), np.full(4, 3.0), np.zeros(4, np.int32))
    off, t, dim, T = stream.window_batch(s, 0, 4, 1)
    assert np.all(t == 0.0) and T[0] == stream.MIN_SPAN
