"""Host-side model of the paired 16-bit PDF layout and of the paired sweeps'
pull (pidx / pull_idx for paired storage and k_sweep_pair, phase-field and
hydrodynamic, in lbm_kernels.hpp): cell c and cell c + half (half = ceil(N/2)) share one
32-bit word, the lower cell in the low 16 bits.  The mapping is a bijection
into the buffer; for even nz the two cells of a pair are (x, y, z) and
(x, y, z + nz/2), and a thread that pulls the pair's 32-bit word from the
pair upstream (swapping the halves where the z pull wraps across the half
domain) gets exactly the populations the one-cell-per-thread pull reads."""
import itertools

import numpy as np
import pytest

KB = 512
E27 = [(0, 0, 0), (1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
       (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1), (-1, 0, 1),
       (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1), (1, 1, 1), (-1, -1, -1), (1, 1, -1), (-1, -1, 1),
       (1, -1, 1), (-1, 1, -1), (-1, 1, 1), (1, -1, -1)]


def opp(i):
    return 0 if i == 0 else (i + 1 if i % 2 else i - 1)


def blocked(q, p, Q):
    return ((p >> 9) * Q + q) * KB + (p & (KB - 1))


def paired(q, c, Q, half):
    h = 1 if c >= half else 0
    return 2 * blocked(q, c - h * half, Q) + h


def size_elems(N, Q):
    half = (N + 1) // 2
    return 2 * ((half + KB - 1) // KB) * Q * KB


def cell_pull(nx, ny, nz, walls, x, y, z, i):
    """(source cell, direction) the one-cell-per-thread pull reads."""
    ex, ey, ez = E27[i]
    if walls and ((ey > 0 and y == 1) or (ey < 0 and y == ny - 2)):
        return x + nx * (y + ny * z), opp(i)
    xs, zs = (x - ex) % nx, (z - ez) % nz
    ys = y - ey if walls else (y - ey) % ny
    return xs + nx * (ys + ny * zs), i


@pytest.mark.parametrize("shape", [(13, 21, 9), (16, 16, 16), (1, 18, 1), (3, 5, 7), (1, 1, 1), (600, 2, 3)])
def test_paired_mapping_is_a_bijection(shape):
    N = int(np.prod(shape))
    half = (N + 1) // 2
    for Q in (15, 27):
        e = np.array([paired(q, c, Q, half) for q in range(Q) for c in range(N)])
        assert len(np.unique(e)) == e.size and e.min() >= 0 and e.max() < size_elems(N, Q)


@pytest.mark.parametrize("shape,walls", [((13, 21, 8), True), ((16, 16, 16), False), ((1, 18, 2), True),
                                         ((12, 3, 10), True), ((2, 2, 2), False), ((5, 4, 6), False)])
def test_pair_pull_matches_cell_pull(shape, walls):
    nx, ny, nz = shape
    assert nz % 2 == 0
    N = nx * ny * nz
    half = N // 2
    nz2 = nz // 2
    Q = 27
    for p in range(half):
        x, y, z2 = p % nx, (p // nx) % ny, p // (nx * ny)
        if walls and (y == 0 or y == ny - 1):
            continue
        for i in range(Q):
            ex, ey, ez = E27[i]
            bb = walls and ((ey > 0 and y == 1) or (ey < 0 and y == ny - 2))
            if bb:
                word, swap, d = p, False, opp(i)
            else:
                xs, zs = (x - ex) % nx, (z2 - ez) % nz2
                ys = y - ey if walls else (y - ey) % ny
                word, d = xs + nx * (ys + ny * zs), i
                swap = (z2 == 0 and ez > 0) or (z2 == nz2 - 1 and ez < 0)
            for h in (0, 1):
                c = p + h * half
                assert (x, y, z2 + h * nz2) == (c % nx, (c // nx) % ny, c // (nx * ny))
                src, di = cell_pull(nx, ny, nz, walls, x, y, z2 + h * nz2, i)
                assert d == di
                assert paired(di, src, Q, half) == 2 * blocked(d, word, Q) + (h ^ int(swap)), (p, i, h)
