"""Host check of the wide-store generation kernel's stream mapping: with H
half-waves per workgroup (8 or 16) and grids padded to a multiple of 8
workgroups, workgroup b gives half-wave j (0..H-1) stream
8 ((b div 8) H + j) + (b mod 8), so that neighbouring rows are written from
different XCDs.  Every stream below n must be taken by exactly one half-wave,
and every half-wave past n must leave (its stream index is >= n)."""
import numpy as np
import pytest


def _streams(n, H):
    grid = ((n + H - 1) // H + 7) & ~7        # as the launch sizes it
    b = np.arange(grid, dtype=np.int64)[:, None]
    j = np.arange(H, dtype=np.int64)[None, :]
    return ((b >> 3) * H + j) * 8 + (b & 7)


@pytest.mark.parametrize("H", [8, 16])
@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 63, 64, 65, 127, 128, 129, 1000, 65536, 65537, 1 << 20, (1 << 20) + 13])
def test_every_stream_once(n, H):
    s = _streams(n, H).ravel()
    taken = s[s < n]
    assert taken.size == n
    assert np.array_equal(np.sort(taken), np.arange(n))
    assert s.max() < H * len(_streams(n, H))    # the padded grid's own range


@pytest.mark.parametrize("H", [8, 16])
def test_neighbouring_streams_on_different_xcds(H):
    s = _streams(1 << 12, H)
    b = np.repeat(np.arange(s.shape[0]), H).reshape(s.shape)
    xcd = np.empty(1 << 12, dtype=np.int64)
    xcd[s.ravel()] = (b % 8).ravel()
    assert np.all(xcd[1:] != xcd[:-1])
