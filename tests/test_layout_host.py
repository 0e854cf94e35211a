"""Host checks of the tiled population layout that the kernels rely on.

Moving flow population p of node m sits at element ((m >> 11) P + p - 1) 2048
+ (m mod 2048) of its region (P populations, tiles of 2048 nodes).  When tiles
hold whole rows and planes hold whole tiles (nx divides 2048 and 2048 / nx
divides ny, or nx is a multiple of 2048), that index is a sum of an x, a y and
a z part, so the odd step may form a link's target index as the node's own
index plus one delta per axis it moves along.  These tests check that identity
for every node and every D3Q27 direction (D3Q19 and D3Q15 are subsets), with
periodic wraps, on boxes the condition admits, and that it fails on boxes the
condition rejects."""
import itertools

import numpy as np
import pytest

TILE = 2048


def _index(m, P):
    return ((m >> 11) * P << 11) | (m & (TILE - 1))


def _separable(nx, ny):
    return nx % TILE == 0 or (TILE % nx == 0 and ny % (TILE // nx) == 0)


def _mismatches(nx, ny, nz, P):
    n = np.arange(nx * ny * nz, dtype=np.int64)
    c = [n % nx, (n // nx) % ny, n // (nx * ny)]
    dim, st = [nx, ny, nz], [1, nx, nx * ny]
    # offsets to the neighbour at -1 / +1 along each axis, wrapping at the faces
    off = [[np.where(c[a] > 0, -1, dim[a] - 1) * st[a], np.where(c[a] < dim[a] - 1, 1, -(dim[a] - 1)) * st[a]]
           for a in range(3)]
    base = _index(n, P)
    delta = [[_index(n + off[a][s], P) - base for s in range(2)] for a in range(3)]
    bad = 0
    for e in itertools.product((-1, 0, 1), repeat=3):
        if e == (0, 0, 0):
            continue
        o = sum(off[a][1 if e[a] > 0 else 0] for a in range(3) if e[a])
        d = sum(delta[a][1 if e[a] > 0 else 0] for a in range(3) if e[a])
        bad += int(np.sum(_index(n + o, P) - base != d))
    return bad


@pytest.mark.parametrize("shape", [(256, 8, 4), (2048, 2, 3), (4096, 2, 2), (64, 32, 5), (512, 4, 3), (8, 256, 5),
                                   (1, 2048, 2), (2, 1024, 3)])
def test_separable_tiles_split_the_index_by_axis(shape):
    assert _separable(shape[0], shape[1])
    for P in (18, 14):
        assert _mismatches(*shape, P) == 0


@pytest.mark.parametrize("shape", [(48, 40, 7), (96, 64, 4), (100, 30, 4)])
def test_other_boxes_do_not(shape):
    assert not _separable(shape[0], shape[1])
    assert _mismatches(*shape, 18) > 0
