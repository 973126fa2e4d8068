"""Host check of the wide-store generation kernel's stream mapping: workgroup
b (grids padded to a multiple of 8 workgroups) gives half-wave j (0..7) stream
(b div 8) * 64 + 8 j + (b mod 8), so that neighbouring rows are written from
different XCDs.  Every stream below n must be taken by exactly one half-wave,
and every half-wave past n must leave (its stream index is >= n)."""
import numpy as np
import pytest


def _streams(n):
    grid = ((n + 7) // 8 + 7) & ~7            # as the launch sizes it
    b = np.arange(grid, dtype=np.int64)[:, None]
    j = np.arange(8, dtype=np.int64)[None, :]
    return ((b >> 3) * 8 + j) * 8 + (b & 7)


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 63, 64, 65, 1000, 65536, 65537, 1 << 20, (1 << 20) + 13])
def test_every_stream_once(n):
    s = _streams(n).ravel()
    taken = s[s < n]
    assert taken.size == n
    assert np.array_equal(np.sort(taken), np.arange(n))
    assert s.max() < 8 * len(_streams(n))    # the padded grid's own range


def test_neighbouring_streams_on_different_xcds():
    s = _streams(1 << 12)
    b = np.repeat(np.arange(s.shape[0]), 8).reshape(s.shape)
    xcd = np.empty(1 << 12, dtype=np.int64)
    xcd[s.ravel()] = (b % 8).ravel()
    assert np.all(xcd[1:] != xcd[:-1])
