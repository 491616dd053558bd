"""Reference of the library's device random fields, for the tests only:
Philox4x64-10 (Salmon et al., SC 2011) in plain Python integers and the
Box-Muller map, following the definition written in include/wd.h."""
import numpy as np

MASK = (1 << 64) - 1
M0, M1 = 0xD2E7470EE14C6C93, 0xCA5A826395121157
W0, W1 = 0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B


def philox4x64_10(counter, key):
    c = [int(v) & MASK for v in counter]
    k0, k1 = (int(v) & MASK for v in key)
    for _ in range(10):
        p0, p1 = M0 * c[0], M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k0, p1 & MASK, (p0 >> 64) ^ c[3] ^ k1, p0 & MASK]
        k0, k1 = (k0 + W0) & MASK, (k1 + W1) & MASK
    return c


def box_muller(a, b):
    u = ((a >> 11) + 1) * 2.0 ** -53
    v = (b >> 11) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u))
    return complex(r * np.cos(2 * np.pi * v), r * np.sin(2 * np.pi * v))


def gaussian_stored(vh, seed, stream, parities=(0, 1)):
    """Stored components [len(parities)][vh][12] as the library draws them."""
    out = np.zeros((len(parities), vh, 12), dtype=np.complex128)
    for n, q in enumerate(parities):
        for i in range(vh):
            for j in range(6):
                x = philox4x64_10(((q * vh + i) * 6 + j, stream, 0, 0), (seed, 0))
                out[n, i, 2 * j] = box_muller(x[0], x[1])
                out[n, i, 2 * j + 1] = box_muller(x[2], x[3])
    return out
