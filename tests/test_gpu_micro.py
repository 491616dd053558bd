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
