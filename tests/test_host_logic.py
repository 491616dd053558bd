"""Host-side logic without a GPU: weight marshalling of the network, the
near-identity start, the weight checkpoint, the timing model of Eqs. 1-2
with MI355X numbers, and the benchmark's one-GPU contract."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import paper_0710_2442_amd as wd
from paper_0710_2442_amd import learn, perf_model
from oracle import ptc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_ptc_weight_layout_round_trip():
    rng = np.random.Generator(np.random.PCG64(1))
    W1 = rng.standard_normal((9, 2, 1, 4, 4)) + 1j * rng.standard_normal((9, 2, 1, 4, 4))
    W2 = rng.standard_normal((9, 1, 2, 4, 4)) + 1j * rng.standard_normal((9, 1, 2, 4, 4))
    flat = wd.ptc_weights_to_flat(W1, W2)
    assert flat.dtype == np.float32 and flat.size == 1152
    # [layer][h][c'][c][4][4] complex, (re, im) interleaved
    assert flat[0] == np.float32(W1[0, 0, 0, 0, 0].real) and flat[1] == np.float32(W1[0, 0, 0, 0, 0].imag)
    assert flat[576] == np.float32(W2[0, 0, 0, 0, 0].real)
    a, b = wd.ptc_flat_to_weights(flat)
    assert np.array_equal(a, W1.astype(np.complex64)) and np.array_equal(b, W2.astype(np.complex64))


def test_near_identity_start_matches_the_oracle_network_at_h0():
    """With only W^(0) = I/sqrt 2 in both layers the network is the identity
    (1 -> 2 -> 1 channels: 2 * (1/sqrt 2)^2 = 1), checked with the oracle."""
    flat = learn.init_weights(3, scale=0.0)
    W1, W2 = wd.ptc_flat_to_weights(flat)
    assert np.allclose(W1[0, 0, 0], np.eye(4) / np.sqrt(2)) and np.all(W1[1:] == 0)
    dims = (2, 2, 2, 4)
    import synthetic as syn
    U = syn.gauge_field(dims, 0.3, 5)
    psi = syn.gaussian_spinor(dims, 6)
    y = ptc.network(U, psi, W1, W2)
    assert np.allclose(y, psi, rtol=1e-6, atol=1e-6)


def test_weight_checkpoint_round_trip_and_damage(tmp_path):
    flat = learn.init_weights(7, scale=0.1)
    meta = {"dims": [16, 16, 16, 16], "kappa": 0.124, "steps": 1250, "act": "bf16"}
    p = tmp_path / "w.wdptc"
    learn.save_weights(p, flat, meta)
    w, m = learn.load_weights(p)
    assert w.dtype == np.float32 and np.array_equal(w, flat) and m == meta
    assert p.stat().st_size == 24 + len(json.dumps(meta, sort_keys=True)) + 4 * 1152
    raw = bytearray(p.read_bytes())
    for pos, what in ((0, "not a PTC"), (8, "version"), (12, "size"), (len(raw) - 3, "checksum")):
        bad = bytearray(raw)
        bad[pos] ^= 0x01
        q = tmp_path / f"bad{pos}"
        q.write_bytes(bytes(bad))
        with pytest.raises(ValueError, match=what):
            learn.load_weights(q)
    with pytest.raises(ValueError):
        learn.save_weights(p, flat[:-1])


@pytest.mark.parametrize("n", ["2", "8"])
def test_bench_refuses_more_than_one_gpu(n):
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", n], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
