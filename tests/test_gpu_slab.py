"""Time-slab decomposition on one GPU: R ranks, each holding only its own
slices plus two packed faces, reproduce the full-lattice single-parity hop
bit for bit (FP64, FP32, D_W and D_W^dag, both parities), and the ranks'
outputs put together match the oracle's parity hop site by site."""
import numpy as np
import pytest
import torch

import paper_0710_2442_amd as wd
import synthetic as syn
from gpu_util import assert_close, from_field, round_c64, storage_round, to_field
from oracle import wilson

pytestmark = pytest.mark.gpu

SLOT = {"f64": 192, "f32": 96}


@pytest.mark.parametrize("dims,R", [((8, 8, 4, 16), 1), ((8, 8, 4, 16), 2), ((8, 8, 4, 16), 4), ((8, 4, 8, 12), 3)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_slabs_reproduce_the_hop(dims, R, prec, dagger):
    print(f"case: slab dims={dims} R={R} prec={prec} dagger={dagger}", flush=True)
    L1, L2, L3, L4 = dims
    vs = L1 * L2 * L3 // 2
    nt = L4 // R
    U = syn.gauge_field(dims, 0.3, 71)
    g = wd.Gauge(U, dims, -1, prec)
    psi = syn.gaussian_spinor(dims, 72)
    Ur = U if prec == "f64" else round_c64(U)
    pr = storage_round(psi, prec)
    fb = wd.wd_halo_face_bytes(dims, prec)
    assert fb == vs * SLOT[prec] // 2
    sb = nt * vs * SLOT[prec]  # bytes of one slab
    for parity in (0, 1):
        src = to_field(g, psi, prec, 1 - parity)
        full = wd.wd_new_field(dims, prec, 1, parity)
        wd.wd_dslash_ex(g, src, full, 0.8, parity, prec, wd.WD_DAGGER if dagger else 0)
        # each rank's input slab is its own buffer between two guard slabs of junk
        slabs = []
        for r in range(R):
            buf = torch.empty(3 * sb, dtype=torch.uint8, device="cuda")
            buf.fill_(0x7F)
            buf[sb:2 * sb].copy_(src[r * sb:(r + 1) * sb])
            slabs.append(buf)
        faces = [[torch.zeros(fb, dtype=torch.uint8, device="cuda") for _ in range(2)] for _ in range(R)]
        for r in range(R):
            for face in (0, 1):
                wd.wd_halo_pack(g, slabs[r][sb:2 * sb], nt, face, dagger, prec, faces[r][face])
        outs = []
        for r in range(R):
            out = torch.zeros(sb, dtype=torch.uint8, device="cuda")
            wd.wd_dslash_slab(g, slabs[r][sb:2 * sb], faces[(r - 1) % R][1], faces[(r + 1) % R][0], out, 0.8,
                              parity, r * nt, nt, dagger, prec)
            torch.cuda.synchronize()
            assert torch.equal(out, full[r * sb:(r + 1) * sb]), (parity, r)
            outs.append(out)
        # the slabs tile the half field in order: judge the whole by the oracle
        whole = torch.zeros_like(full)
        whole[:R * sb].copy_(torch.cat(outs))
        want = 0.8 * wilson.hop_parity(Ur, pr, parity, dagger=bool(dagger))
        assert_close(from_field(g, whole, prec, parity), want, prec, what=f"slabs {dims} R={R} {prec} p{parity}")
    g.close()


def test_slab_rejects_bad_arguments():
    dims = (8, 8, 4, 16)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 73), dims, -1, "f64")
    a = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    b = torch.zeros(1 << 20, dtype=torch.uint8, device="cuda")
    for args in ((a, a, a, b, 1.0, 0, 0, 17, 0, "f64"), (a, a, a, b, 1.0, 0, 12, 8, 0, "f64"),
                 (a, a, a, b, 1.0, 2, 0, 4, 0, "f64"), (a, a, a, b, 1.0, 0, 0, 4, 0, "bf16"),
                 (a, a, a, a, 1.0, 0, 0, 4, 0, "f64")):
        with pytest.raises(wd.WdError):
            wd.wd_dslash_slab(g, *args)
    g2 = wd.Gauge(syn.gauge_field((4, 4, 4, 4), 0.3, 74), (4, 4, 4, 4), -1, "f64")  # 32 sites per slice
    with pytest.raises(wd.WdError):
        wd.wd_halo_pack(g2, a, 2, 0, 0, "f64", a)
    g.close()
    g2.close()
