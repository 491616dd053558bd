"""The global -> LDS copy micro-benchmark moves the right bytes (LDS checksum
against the host's sum of the same words) at every size and misalignment."""
import numpy as np
import pytest

import paper_0710_2442_amd as wd

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("nbytes,offset", [(16, 0), (128, 4), (1024, 128), (4096, 132), (32768, 252), (2048, 64)])
def test_lds_copy_checksums(nbytes, offset):
    rng = np.random.Generator(np.random.PCG64(7))
    pattern = rng.integers(0, 256, size=1 << 20, dtype=np.uint8)
    cyc, sums = wd.wd_micro_lds_copy(nbytes, offset, 4, pattern)
    want = int(pattern[offset:offset + nbytes].view(np.uint32).astype(np.uint64).sum() % (1 << 32))
    assert np.all(sums == want)
    assert np.all(cyc > 0)


def test_lds_copy_rejects_bad_arguments():
    for args in ((8, 0, 1), (32784, 0, 1), (64, 2, 1), (64, 256, 1), (64, 0, 0), (64, 0, 2000)):
        with pytest.raises(wd.WdError):
            wd.wd_micro_lds_copy(*args)


def test_resident_probe_orders_the_cache_levels():
    """Reads held by the XCDs' L2 (16 MiB) are faster than reads from the
    Infinity Cache (128 MiB), and both at least as fast as reads from HBM
    (2 GiB); HBM reads stay below the 8 TB/s data-sheet peak."""
    mib = 1 << 20
    l2 = 16 * mib / wd.wd_micro_resident(16 * mib, passes=50, reps=3)
    mall = 128 * mib / wd.wd_micro_resident(128 * mib, passes=5, reps=3)
    hbm = 2048 * mib / wd.wd_micro_resident(2048 * mib, passes=1, reps=2)
    print(f"resident reads: L2 {l2 / 1e12:.2f}, Infinity Cache {mall / 1e12:.2f}, HBM {hbm / 1e12:.2f} TB/s",
          flush=True)
    assert l2 > 1.5 * mall and mall >= 0.95 * hbm and hbm < 8.0e12
