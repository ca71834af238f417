"""Host checks of FP32 integer-division shortcuts used by the spreading
kernels, evaluated exhaustively with IEEE single precision (numpy float32
rounds add and multiply to nearest like the GPU's FP32 units)."""
import numpy as np


def test_tile_quotient_from_fp32_reciprocal_is_exact():
    """(i + 1/2) * fl(1/t) truncates to i // t for every cell index i <= 2048
    and tile edge 4 <= t <= 2048 (the grid limits)."""
    i = np.arange(0, 2049, dtype=np.int64)
    for t in range(4, 2049):
        inv = np.float32(1.0) / np.float32(t)
        q = ((i.astype(np.float32) + np.float32(0.5)) * inv).astype(np.int64)
        assert np.array_equal(q, i // t), t


def test_box_coordinates_from_fp32_reciprocals_are_exact():
    """The flush decodes a box node q < bx*by*bz into (lx, ly, lz) with the same
    trick, for every box shape the tiles allow (edges 7..19, a whole short
    periodic axis up to 16)."""
    for bx in range(4, 20):
        for by in range(4, 20):
            bz = 19
            q = np.arange(bx * by * bz, dtype=np.int64)
            inv_bx = np.float32(1.0) / np.float32(bx)
            inv_bxy = np.float32(1.0) / np.float32(bx * by)
            lz = ((q.astype(np.float32) + np.float32(0.5)) * inv_bxy).astype(np.int64)
            rq = q - lz * (bx * by)
            ly = ((rq.astype(np.float32) + np.float32(0.5)) * inv_bx).astype(np.int64)
            lx = rq - ly * bx
            assert np.array_equal(lz, q // (bx * by))
            assert np.array_equal(ly, (q // bx) % by)
            assert np.array_equal(lx, q % bx)


def test_support_window_and_wrap_rotation_give_the_wrapped_neighbours():
    """The interpolation loads the three x-neighbours of a row from the window
    i-1 .. i+1 clamped into the row, and a stencil that wraps round a periodic
    row (i = 0 or n-1) takes one extra value from the far end and rotates.
    Every row length 3 <= n <= 300 and home index 0 <= i < n gives the wrapped
    neighbours (i-1, i, i+1) mod n."""
    for n in range(3, 301):
        row = np.arange(n) * 7 + 1000          # distinct values
        for i in range(n):
            sx = min(max(i - 1, 0), n - 3)
            a0, a1, a2 = row[sx], row[sx + 1], row[sx + 2]
            lo, hi = i < 1, i > n - 2
            e = row[n - 1 if lo else 0]
            got = (e if lo else (a1 if hi else a0),
                   a0 if lo else (a2 if hi else a1),
                   a1 if lo else (e if hi else a2))
            want = tuple(row[(i + d) % n] for d in (-1, 0, 1))
            assert got == want, (n, i)
