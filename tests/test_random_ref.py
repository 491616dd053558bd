"""The Philox4x64-10 reference used to check the device random fields is
pinned to numpy's independent Philox bit generator (numpy advances its
counter before each block, so its first block is counter 1)."""
import numpy as np
import pytest

from philox_ref import box_muller, philox4x64_10


@pytest.mark.parametrize("key", [(0, 0), (5, 7), (2**64 - 1, 12345), (0x243F6A8885A308D3, 0x13198A2E03707344)])
@pytest.mark.parametrize("ctr", [(0, 0, 0, 0), (41, 3, 0, 0), (2**64 - 2, 2**64 - 1, 7, 9)])
def test_philox_matches_numpy(key, ctr):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    got = [int(v) for v in bg.random_raw(8)]
    # numpy: block 1 uses counter + 1, block 2 counter + 2 (carry into the next word)
    c = list(ctr)
    want = []
    for _ in range(2):
        c[0] += 1
        for w in range(3):
            if c[w] >> 64:
                c[w] &= (1 << 64) - 1
                c[w + 1] += 1
        want += philox4x64_10(c, key)
    assert got == want


def test_box_muller_moments():
    rng = np.random.Generator(np.random.PCG64(3))
    words = rng.integers(0, 2**63, size=(20000, 2), dtype=np.int64).astype(np.uint64) * 2
    z = np.array([box_muller(int(a), int(b)) for a, b in words])
    assert abs(z.real.mean()) < 0.03 and abs(z.imag.mean()) < 0.03
    assert abs(z.real.var() - 1) < 0.05 and abs(z.imag.var() - 1) < 0.05
    assert abs(np.mean(z.real * z.imag)) < 0.03
