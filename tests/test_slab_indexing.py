"""Index arithmetic of the time-slab hop, checked on the CPU: every read of a
rank's slab stays inside its own slices, every time neighbour outside them
is the matching site of the neighbour rank's packed face, and the ranks'
output sites tile the half field exactly once.  (The checkerboard index and
neighbour rules are restated here from the layout documented in wd.h.)"""
import itertools

import pytest


def coords_of(dims, i, parity):
    L1, L2, L3, L4 = dims
    L1h = L1 // 2
    x1h = i % L1h
    rest = i // L1h
    x2 = rest % L2
    r2 = rest // L2
    x3 = r2 % L3
    x4 = r2 // L3
    x1 = 2 * x1h + ((parity + x2 + x3 + x4) & 1)
    return x1, x2, x3, x4


def cb_index(dims, x):
    L1, L2, L3, L4 = dims
    x1, x2, x3, x4 = (v % L for v, L in zip(x, dims))
    return (x1 + L1 * (x2 + L2 * (x3 + L3 * x4))) >> 1


@pytest.mark.parametrize("dims,R", [((8, 8, 4, 16), 2), ((8, 8, 4, 16), 4), ((8, 4, 8, 12), 3), ((16, 4, 4, 8), 8)])
@pytest.mark.parametrize("parity", [0, 1])
def test_slab_reads_stay_in_range(dims, R, parity):
    L1, L2, L3, L4 = dims
    vs = L1 * L2 * L3 // 2
    assert vs % 64 == 0 and L4 % R == 0
    nt = L4 // R
    covered = []
    for r in range(R):
        t0 = r * nt
        base = t0 * vs
        for il in range(nt * vs):
            i = base + il
            covered.append(i)
            x = coords_of(dims, i, parity)
            x4 = x[3]
            j = i - x4 * vs
            assert 0 <= j < vs
            for mu, sgn in itertools.product(range(4), (1, -1)):
                y = list(x)
                y[mu] += sgn
                nb = cb_index(dims, y)
                if mu < 3:
                    # spatial neighbours: same slice, read from the slab
                    assert 0 <= nb - base < nt * vs
                elif sgn == 1 and x4 == t0 + nt - 1:
                    # face_hi = face 0 (first slice) of the rank above
                    ra = (r + 1) % R
                    assert nb == ra * nt * vs + j
                elif sgn == -1 and x4 == t0:
                    # face_lo = face 1 (last slice) of the rank below
                    rb = (r - 1) % R
                    assert nb == (rb * nt + nt - 1) * vs + j
                else:
                    assert 0 <= nb - base < nt * vs
    assert sorted(covered) == list(range(L1 * L2 * L3 * L4 // 2))
