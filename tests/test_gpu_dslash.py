"""GPU parity of the single-parity hop, D_W, layouts and multi-RHS hop.

Bars: FP64 relative difference <= 1e-13, FP32 <= 1e-6 (the FP32 path is fed
the FP64 inputs rounded once to complex64 and the oracle uses the same
rounded inputs).  FP16 (+ per-site scale) and BF16 storage: the oracle sees
the same rounded inputs; the bar is set by the rounding of the stored output
(FP16: 1e-3, about 4x the RMS rounding error of 2^-11-ulp components;
BF16: 2^-8).
"""
import json
import os

import numpy as np
import pytest
import torch

import paper_0710_2442_amd as wd
import synthetic as syn
from gpu_util import (DEV, SITE_BARS, assert_close, from_field, half_view, rel_err, round_c64, site_err,
                      storage_round, to_field, to_storage_basis)
from oracle import free_field, solvers, wilson

pytestmark = pytest.mark.gpu

SMALL = [(8, 8, 8, 8), (6, 4, 6, 10), (2, 2, 2, 2), (4, 2, 2, 4), (2, 2, 2, 64)]
BARS = {"f64": 1e-13, "f32": 1e-6, "f16": 1e-3, "bf16": 2.0 ** -8}


def _inputs(dims, prec, seed=7):
    U = syn.gauge_field(dims, 0.3, 1000 + seed)
    psi = syn.gaussian_spinor(dims, 2000 + seed)
    if prec == "f64":
        return U, psi, U, psi
    Ur = round_c64(U)
    pr = storage_round(psi, prec)
    return U, psi, Ur, pr


@pytest.mark.parametrize("dims", SMALL)
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
@pytest.mark.parametrize("parity", [0, 1])
def test_parity_hop_matches_oracle(dims, prec, parity):
    print(f"case: hop dims={dims} prec={prec} parity={parity}", flush=True)
    U, psi, Ur, pr = _inputs(dims, prec)
    g = wd.Gauge(U, dims, -1, prec)
    src = to_field(g, psi, prec, 1 - parity)
    out = wd.wd_new_field(dims, prec, 1, parity)
    wd.wd_dslash(g, src, out, 1.0, dims, parity)
    got = from_field(g, out, prec, parity)
    want = wilson.hop_parity(Ur, pr, parity)
    assert_close(got, want, prec, what=f"hop {dims} {prec} p{parity}")
    g.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10), (2, 2, 2, 2)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_full_dirac_and_dagger(dims, prec):
    print(f"case: D_W dims={dims} prec={prec}", flush=True)
    kappa = 0.12
    U, psi, Ur, pr = _inputs(dims, prec, seed=9)
    g = wd.Gauge(U, dims, -1, prec)
    src = to_field(g, psi, prec)
    out = wd.wd_new_field(dims, prec)
    wd.wd_dslash(g, src, out, kappa, dims, wd.WD_FULL)
    assert_close(from_field(g, out, prec), wilson.dirac(Ur, pr, kappa), prec, what=f"D_W {dims} {prec}")
    for parity in (0, 1):
        o = wd.wd_new_field(dims, prec, 1, parity)
        wd.wd_dslash_ex(g, half_view(src, g, prec, 1 - parity), o, 1.0, parity, prec, wd.WD_DAGGER)
        want = wilson.hop_parity(Ur, pr, parity, dagger=True)
        assert_close(from_field(g, o, prec, parity), want, prec, what=f"H^dag {dims} {prec} p{parity}")
    g.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10), (2, 2, 2, 2), (2, 2, 2, 64), (16, 16, 16, 16)])
@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_one_launch_dirac_matches_oracle_and_two_pass(dims, prec):
    """The one-launch full-lattice D_W (backward links read from the
    neighbours' forward links, applied as U^dag) against the oracle, both for
    D_W and D_W^dag, and against the two single-parity launches."""
    print(f"case: one-launch D_W dims={dims} prec={prec}", flush=True)
    kappa = 0.12
    U, psi, Ur, pr = _inputs(dims, prec, seed=19)
    g = wd.Gauge(U, dims, -1, prec)
    src = to_field(g, psi, prec)
    for flags, dag in ((0, False), (wd.WD_DAGGER, True)):
        one = wd.wd_new_field(dims, prec)
        two = wd.wd_new_field(dims, prec)
        one.fill_(0xAB)
        wd.wd_dslash_ex(g, src, one, kappa, wd.WD_FULL, prec, flags | wd.WD_ONE_PASS)
        wd.wd_dslash_ex(g, src, two, kappa, wd.WD_FULL, prec, flags)
        want = wilson.dirac(Ur, pr, kappa) if not dag else wilson.gamma5(wilson.dirac(Ur, wilson.gamma5(pr), kappa))
        got = from_field(g, one, prec)
        assert_close(got, want, prec, what=f"one-launch D_W {dims} {prec} dag={dag}")
        # same operator, different link rounding only (U^dag rebuilt from U's rows vs stored rows of U^dag)
        assert rel_err(got, from_field(g, two, prec)) <= {"f64": 1e-14, "f32": 1e-6, "bf16": 1e-2}[prec]
    g.close()


@pytest.mark.parametrize("dims", [(6, 6, 10, 32), (4, 4, 4, 48), (8, 8, 8, 64), (16, 8, 4, 16), (8, 16, 6, 32)])
@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_marching_dirac_over_ranges_and_tiles(dims, prec):
    """The one-launch D_W marches each spatial tile (256 sites) through
    ranges of at least 8 time slices: several ranges here, so every range
    boundary (time link and half spinor fetched across it) and the
    antiperiodic wrap are crossed.  Tiles of consecutive sites, the last one
    ragged (6x6x10), and brick tiles of L1 x n2 x 2 sites (16x8x4: one brick
    per x3 pair; 8x16x6: three bricks along x3; FP64 and FP32 stage them in
    LDS with their side faces, FP16 and BF16 keep them in registers).
    Against the oracle, D_W and D_W^dag; the output's padding slots must
    come back zero.

    FP16 per-site bar 2^-10: the output's own rounding is bounded by 2^-11 of
    the site's largest component (half an FP16 ulp of each storage-basis real,
    two of which mix in each chiral-basis real), and the X term carries the
    input spinor at weight one, so a one-ulp difference between the oracle's
    emulated input rounding and the device packing adds up to another 2^-11."""
    print(f"case: marching D_W dims={dims} prec={prec}", flush=True)
    kappa = 0.124
    U, psi, Ur, pr = _inputs(dims, prec, seed=23)
    g = wd.Gauge(U, dims, -1, prec)
    src = to_field(g, psi, prec)
    for flags, dag in ((0, False), (wd.WD_DAGGER, True)):
        out = wd.wd_new_field(dims, prec)
        out.fill_(0xFF)  # NaN in every float format
        wd.wd_dslash_ex(g, src, out, kappa, wd.WD_FULL, prec, flags | wd.WD_ONE_PASS)
        want = wilson.dirac(Ur, pr, kappa) if not dag else wilson.gamma5(wilson.dirac(Ur, wilson.gamma5(pr), kappa))
        site = 2.0 ** -10 + 4e-6 if prec == "f16" else None
        assert_close(from_field(g, out, prec), want, prec, site=site, what=f"marching D_W {dims} {prec} dag={dag}")
        if prec in ("f64", "f32"):
            vh, vpad = int(np.prod(dims)) // 2, wd.wd_vh_pad(dims)
            nc = vpad // 64
            lanes = np.arange(vh, vpad)
            if prec == "f64":  # [parity][chunk][component][lane]
                dev = out.cpu().numpy().view(np.complex128).reshape(2, nc, 12, 64)
                pads = dev[:, lanes // 64, :, lanes % 64]
            else:  # [parity][chunk][packet][lane][2 components]
                dev = out.cpu().numpy().view(np.complex64).reshape(2, nc, 6, 64, 2)
                pads = dev[:, lanes // 64, :, lanes % 64, :]
            assert np.all(pads == 0), "padding slots not cleared"
    g.close()


def test_periodic_time_boundary():
    dims = (4, 4, 2, 6)
    U, psi, _, _ = _inputs(dims, "f64", seed=11)
    g = wd.Gauge(U, dims, +1, "f64")
    src = to_field(g, psi)
    out = wd.wd_new_field(dims, "f64")
    wd.wd_dslash(g, src, out, 0.13, dims, wd.WD_FULL)
    assert_close(from_field(g, out), wilson.dirac(U, psi, 0.13, tbc=+1), "f64", what="periodic-time D_W")
    g.close()


def test_pack_layout_is_documented_soa():
    """Device bytes equal the layout written in wd.h, built here index by index:
    packet k of checkerboard site i at packet (i // 64) * CHUNK + 64 k + i % 64."""
    dims = (6, 4, 2, 4)  # V_h = 96: two chunks, the second one ragged
    L1, L2, L3, L4 = dims
    psi = syn.gaussian_spinor(dims, 5)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 5), dims, -1, "f64")
    vpad = wd.wd_vh_pad(dims)
    nc = vpad // 64
    stored = to_storage_basis(psi)
    planes = np.zeros((2, 12, vpad), dtype=np.complex128)  # [parity][component][cb]
    for x4 in range(L4):
        for x3 in range(L3):
            for x2 in range(L2):
                for x1 in range(L1):
                    idx = x1 + L1 * (x2 + L2 * (x3 + L3 * x4))
                    p = (x1 + x2 + x3 + x4) % 2
                    for c in range(12):
                        planes[p, c, idx >> 1] = stored[x4, x3, x2, x1, c // 3, c % 3]
    chunked = planes.reshape(2, 12, nc, 64).transpose(0, 2, 1, 3)  # [parity][chunk][c][lane]
    # FP64: packet c holds component c
    f = to_field(g, psi, "f64")
    dev = f.cpu().numpy().view(np.complex128).reshape(2, nc, 12, 64)
    assert np.array_equal(dev, chunked)
    # FP32: packet k holds components 2k, 2k+1
    f32 = to_field(g, psi, "f32")
    d32 = f32.cpu().numpy().view(np.complex64).reshape(2, nc, 6, 64, 2)
    w32 = chunked.astype(np.complex64).reshape(2, nc, 6, 2, 64).transpose(0, 1, 2, 4, 3)
    assert np.array_equal(d32, w32)
    # BF16: packet k holds components 4k .. 4k+3, (re, im) interleaved
    fb = to_field(g, psi, "bf16")
    raw = fb.cpu().numpy().view(np.uint16).reshape(2, nc, 3, 64, 4, 2).astype(np.uint32) << 16
    vals = raw.view(np.float32)
    db = (vals[..., 0] + 1j * vals[..., 1]).transpose(0, 1, 2, 4, 3).reshape(2, nc, 12, 64)
    wb = solvers.round_storage(chunked, "bf16")
    assert np.array_equal(db, wb)
    # FP16: 3 packets of halves, then the chunk's 64 per-site scales
    fh = to_field(g, psi, "f16").cpu().numpy().view(np.uint8).reshape(2, nc, 208 * 16)
    halves = fh[:, :, :192 * 16].copy().view(np.float16).astype(np.float32).reshape(2, nc, 3, 64, 4, 2)
    scales = fh[:, :, 192 * 16:].copy().view(np.float32).reshape(2, nc, 1, 64)
    dh = (halves[..., 0] + 1j * halves[..., 1]).transpose(0, 1, 2, 4, 3).reshape(2, nc, 12, 64) * scales
    amax = np.maximum(np.abs(chunked.real), np.abs(chunked.imag)).max(axis=2, keepdims=True)
    assert np.allclose(scales, amax, rtol=1e-7, atol=0)
    assert np.max(np.abs(dh - chunked)) <= 2.0 ** -11 * amax.max() * 1.01
    # the round trip applies the basis map twice: exact up to rounding
    assert rel_err(from_field(g, f), psi) <= 1e-15
    g.close()


def test_bitwise_deterministic():
    dims = (8, 8, 8, 8)
    U, psi, _, _ = _inputs(dims, "f64", seed=13)
    g = wd.Gauge(U, dims, -1, "f64")
    src = to_field(g, psi)
    a = wd.wd_new_field(dims, "f64")
    b = wd.wd_new_field(dims, "f64")
    wd.wd_dslash(g, src, a, 0.12, dims, wd.WD_FULL)
    wd.wd_dslash(g, src, b, 0.12, dims, wd.WD_FULL)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
@pytest.mark.parametrize("nrhs", [1, 5, 12, 24])
def test_mrhs_equals_single_rhs_bitwise(prec, nrhs):
    dims = (8, 8, 8, 16)
    U = syn.gauge_field(dims, 0.3, 21)
    g = wd.Gauge(U, dims, -1, prec)
    psis = syn.gaussian_spinor(dims, 22, nrhs=nrhs)
    hb = wd.wd_field_bytes(dims, prec, 1, wd.WD_EVEN)
    src = torch.cat([to_field(g, psis[r], prec, wd.WD_ODD) for r in range(nrhs)])
    out = wd.wd_new_field(dims, prec, nrhs, wd.WD_EVEN)
    bs, gr, rp, us = wd.wd_tune_dslash_mrhs(g, prec, nrhs)  # any variant must give the same bits
    wd.wd_dslash_mrhs(g, src, out, 0.7, wd.WD_EVEN, prec, nrhs)
    for r in range(nrhs):
        one = wd.wd_new_field(dims, prec, 1, wd.WD_EVEN)
        wd.wd_dslash_ex(g, src[r * hb:(r + 1) * hb], one, 0.7, wd.WD_EVEN, prec)
        torch.cuda.synchronize()
        assert torch.equal(one, out[r * hb:(r + 1) * hb]), r
    g.close()


# (8, 4, 6, 16): V_h = 1536, 6, 12 or 24 tiles, no slice-aligned tile orders;
# (16, 8, 8, 8): 8 tiles of 64 per slice, every tile order; (8, 6, 8, 4): 3
# tiles of 64 per slice, 12 tiles (not a multiple of 8), orders 3, -2, -4
@pytest.mark.parametrize("dims", [(8, 4, 6, 16), (16, 8, 8, 8), (8, 6, 8, 4)])
@pytest.mark.parametrize("prec", ["f32", "f16", "bf16"])
def test_every_mrhs_variant_is_bitwise_identical(dims, prec):
    """Block size, tile order (box orders -101 .. -108 with tile-major RHS
    chunks included) and RHS per lane change only the schedule: every
    variant gives the bytes of the single-RHS hop, ragged RHS chunks and a
    ragged last tile included."""
    nrhs = 5
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 23), dims, -1, prec)
    psis = syn.gaussian_spinor(dims, 24, nrhs=nrhs)
    hb = wd.wd_field_bytes(dims, prec, 1, wd.WD_EVEN)
    src = torch.cat([to_field(g, psis[r], prec, wd.WD_ODD) for r in range(nrhs)])
    ref = wd.wd_new_field(dims, prec, nrhs, wd.WD_EVEN)
    for r in range(nrhs):
        wd.wd_dslash_ex(g, src[r * hb:(r + 1) * hb], ref[r * hb:(r + 1) * hb], 0.7, wd.WD_EVEN, prec)
    n = 0
    for bs in (64, 128, 256):
        for gr in (0, 2, 3, 4, 8, -2, -4, -8, -101, -102, -104, -108):
            for rpl in (1, 2, 3, 4, 12, 16):
                try:
                    wd.wd_set_dslash_mrhs_variant(g, prec, bs, gr, rpl)
                except wd.WdError:
                    assert gr != 0 or bs == 256  # only tile orders (or sizes) that do not fit are refused
                    continue
                assert wd.wd_get_dslash_mrhs_variant(g, prec) == (bs, gr, rpl)
                out = wd.wd_new_field(dims, prec, nrhs, wd.WD_EVEN)
                out.fill_(0xAB)
                wd.wd_dslash_mrhs(g, src, out, 0.7, wd.WD_EVEN, prec, nrhs)
                torch.cuda.synchronize()
                assert torch.equal(out, ref), (bs, gr, rpl)
                n += 1
    assert n >= 18
    for bad in ((96, 0, 4), (64, 0, 0), (64, 0, 17), (64, 5, 4), (64, 0, -1)):
        with pytest.raises(wd.WdError):
            wd.wd_set_dslash_mrhs_variant(g, prec, *bad)
    g.close()


@pytest.mark.parametrize("dims", [(16, 8, 8, 8), (8, 8, 8, 16)])
def test_every_fp64_mrhs_variant_is_bitwise_identical(dims):
    """FP64 multi-RHS: the 16-site x 4-RHS tiles in every tile order, and one
    RHS per block in every box order that fits, give the bytes of the
    single-RHS hop."""
    nrhs = 5
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 29), dims, -1, "f64")
    psis = syn.gaussian_spinor(dims, 30, nrhs=nrhs)
    hb = wd.wd_field_bytes(dims, "f64", 1, wd.WD_EVEN)
    src = torch.cat([to_field(g, psis[r], "f64", wd.WD_ODD) for r in range(nrhs)])
    ref = wd.wd_new_field(dims, "f64", nrhs, wd.WD_EVEN)
    for r in range(nrhs):
        wd.wd_dslash_ex(g, src[r * hb:(r + 1) * hb], ref[r * hb:(r + 1) * hb], 0.7, wd.WD_EVEN, "f64")
    n = 0
    for bs, rpl, groups in [(16, 4, gr) for gr in (0, 2, 4, 8, -2, -4, -8)] + \
            [(b, 1, gr) for b in (64, 128, 256) for gr in (-101, -102, -104, -108)]:
        try:
            wd.wd_set_dslash_mrhs_variant(g, "f64", bs, groups, rpl)
        except wd.WdError:
            continue
        out = wd.wd_new_field(dims, "f64", nrhs, wd.WD_EVEN)
        out.fill_(0xAB)
        wd.wd_dslash_mrhs(g, src, out, 0.7, wd.WD_EVEN, "f64", nrhs)
        torch.cuda.synchronize()
        assert torch.equal(out, ref), (bs, groups, rpl)
        n += 1
    assert n >= 6
    g.close()


def test_mrhs_solve_does_not_depend_on_rhs_per_lane():
    """The multi-RHS solver through its fused epilogues and per-RHS norms:
    1, 2 or all 3 right-hand sides per lane (same blocks, so the same norm
    partials), bit-identical x, and x solves D_W x = b to 1e-10."""
    dims = (8, 8, 4, 8)
    nrhs = 3
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 25), dims, -1, "f64")
    f = wd.wd_field_bytes(dims, "f64")
    B = torch.cat([to_field(g, syn.gaussian_spinor(dims, 26 + r), "f64", wd.WD_FULL) for r in range(nrhs)])
    xs = []
    for rpl in (1, 2, 3):
        wd.wd_set_dslash_mrhs_variant(g, "f32", 64, 0, rpl)
        x = wd.wd_new_field(dims, "f64", nrhs)
        prm = wd.wd_solve_params_default(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="f32", inner_tol=1e-4)
        rc, infos = wd.wd_solve_mrhs(g, B, x, nrhs, 0.12, 1e-10, prm)
        assert rc == 0 and all(i["status"] == 0 for i in infos)
        xs.append(x)
    assert torch.equal(xs[0], xs[1]) and torch.equal(xs[0], xs[2])
    U = syn.gauge_field(dims, 0.3, 25)
    for r in range(nrhs):
        b = syn.gaussian_spinor(dims, 26 + r)
        xr = from_field(g, xs[1][r * f:(r + 1) * f], "f64", wd.WD_FULL)
        res = b - wilson.dirac(U, xr, 0.12, -1)
        assert np.linalg.norm(res) / np.linalg.norm(b) <= 1e-10
    g.close()


def test_tuning_cache_round_trip(tmp_path):
    """Both tuners append their choice to the JSON-lines cache and take it
    back from there (same variant, the stored time) without timing again;
    force retunes; the multi-RHS key includes the number of RHS."""
    dims = (8, 8, 8, 16)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 27), dims, -1, "f64")
    path = str(tmp_path / "tune.jsonl")

    def lines():
        return open(path).read().splitlines()

    a = wd.wd_tune_dslash(g, "f32", path)
    assert len(lines()) == 1 and '"occ"' in lines()[0] and "/hop/p1/8x8x8x16" in lines()[0]
    b = wd.wd_tune_dslash(g, "f32", path)
    assert b[:3] == a[:3] and abs(b[3] - a[3]) < 1e-3 and len(lines()) == 1
    m = wd.wd_tune_dslash_mrhs(g, "bf16", 5, path)
    assert len(lines()) == 2 and '"rpl"' in lines()[1] and "/hop_mrhs5/p3/8x8x8x16" in lines()[1]
    wd.wd_set_dslash_mrhs_variant(g, "bf16", 256, 0, 1)
    m2 = wd.wd_tune_dslash_mrhs(g, "bf16", 5, path)
    assert m2[:3] == m[:3] and wd.wd_get_dslash_mrhs_variant(g, "bf16") == m[:3]
    assert abs(m2[3] - m[3]) < 1e-3 and len(lines()) == 2
    wd.wd_tune_dslash_mrhs(g, "bf16", 5, path, force=True)
    assert len(lines()) == 3
    wd.wd_tune_dslash_mrhs(g, "bf16", 3, path)
    assert len(lines()) == 4 and "/hop_mrhs3/" in lines()[3]
    g.close()


def test_one_launch_dirac_variants_and_tuning(tmp_path):
    """Every one-launch D_W variant (time slices per range; brick tiles,
    brick tiles staged in LDS with their side faces (FP64, FP32), or
    consecutive tiles) computes the same bytes, D_W and D_W^dag; the tuner
    keeps its choice in the JSON-lines cache and takes it back from there;
    variants that do not fit the lattice or precision are refused."""
    dims = (16, 8, 4, 16)  # bricks of 16 x 8 x 2 sites fit
    U = syn.gauge_field(dims, 0.3, 31)
    psi = syn.gaussian_spinor(dims, 32)
    for prec in ("f64", "f32", "bf16"):
        g = wd.Gauge(U, dims, -1, prec)
        src = to_field(g, psi, prec)
        assert wd.wd_get_dirac_variant(g, prec) == (0, 3 if prec != "bf16" else 2)
        staged = ((1, 3), (3, 3), (8, 3), (0, 3)) if prec != "bf16" else ()
        for flags in (0, wd.WD_DAGGER):
            ref = wd.wd_new_field(dims, prec)
            wd.wd_dslash_ex(g, src, ref, 0.124, wd.WD_FULL, prec, flags | wd.WD_ONE_PASS)
            for sl, tile in ((1, 0), (3, 2), (8, 0), (16, 2), (16, 0), (0, 0)) + staged:
                wd.wd_set_dirac_variant(g, prec, sl, tile)
                assert wd.wd_get_dirac_variant(g, prec) == (sl, tile)
                out = wd.wd_new_field(dims, prec)
                out.fill_(0xFF)
                wd.wd_dslash_ex(g, src, out, 0.124, wd.WD_FULL, prec, flags | wd.WD_ONE_PASS)
                assert torch.equal(out, ref), (prec, flags, sl, tile)
            wd.wd_set_dirac_variant(g, prec, 0, 3 if prec != "bf16" else 2)
        if prec == "bf16":
            with pytest.raises(wd.WdError):
                wd.wd_set_dirac_variant(g, prec, 8, 3)  # LDS staging: FP64 and FP32 storage only
        with pytest.raises(wd.WdError):
            wd.wd_set_dirac_variant(g, prec, 17, 2)
        with pytest.raises(wd.WdError):
            wd.wd_set_dirac_variant(g, prec, 8, 1)
        g.close()
    g = wd.Gauge(U, dims, -1, "f64")
    path = str(tmp_path / "tune.jsonl")
    a = wd.wd_tune_dirac(g, "f64", path)
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and '"slices"' in lines[0] and "/dirac/p0/16x8x4x16" in lines[0]
    wd.wd_set_dirac_variant(g, "f64", 1, 0)
    b = wd.wd_tune_dirac(g, "f64", path)
    assert b[:2] == a[:2] and abs(b[2] - a[2]) < 1e-3 and wd.wd_get_dirac_variant(g, "f64") == a[:2]
    assert len(open(path).read().splitlines()) == 1
    g.close()
    g = wd.Gauge(syn.gauge_field((6, 4, 6, 10), 0.3, 33), (6, 4, 6, 10), -1, "f32")
    assert wd.wd_get_dirac_variant(g, "f32") == (0, 0)  # 256 is not a multiple of 2 x 6: no bricks
    for tile in (2, 3):
        with pytest.raises(wd.WdError):
            wd.wd_set_dirac_variant(g, "f32", 4, tile)
    g.close()


def test_blas_against_numpy():
    dims = (6, 4, 6, 10)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 31), dims, -1, "f64")
    a = syn.gaussian_spinor(dims, 32)
    b = syn.gaussian_spinor(dims, 33)
    fa, fb = to_field(g, a), to_field(g, b)
    n = wd.wd_norm2(g, fa, 2, "f64")
    assert abs(n - np.vdot(a, a).real) <= 1e-13 * n
    d = wd.wd_cdot(g, fa, fb, 2, "f64")
    want = np.vdot(a, b)
    assert abs(d - want) <= 1e-13 * abs(want) * 10
    c = 0.3 - 1.7j
    wd.wd_caxpy(g, c, fa, fb, 2, "f64")
    assert rel_err(from_field(g, fb), c * a + b) <= 1e-15
    # caxpy in FP32 storage
    fa32, fb32 = to_field(g, a, "f32"), to_field(g, b, "f32")
    wd.wd_caxpy(g, c, fa32, fb32, 2, "f32")
    assert rel_err(from_field(g, fb32, "f32"), c * storage_round(a, "f32") + storage_round(b, "f32")) <= 1e-6
    g.close()


def test_argument_errors_do_not_launch():
    dims = (4, 4, 4, 4)
    g = wd.Gauge(syn.gauge_field(dims, 0.3, 41), dims, -1, "f64")
    f = wd.wd_new_field(dims, "f64")
    o = wd.wd_new_field(dims, "f64")
    with pytest.raises(wd.WdError) as e:
        wd.wd_dslash(g, f, o, 0.1, (4, 4, 4, 6), 0)
    assert e.value.status == -2
    with pytest.raises(wd.WdError):
        wd.wd_dslash(g, f, o, float("nan"), dims, 0)
    with pytest.raises(wd.WdError):
        wd.wd_dslash(g, f, o, 0.1, dims, 3)
    with pytest.raises(wd.WdError):
        wd.wd_dslash(g, f, f, 0.1, dims, 0)
    # the binding checks buffers on the host before the library sees them
    with pytest.raises(ValueError, match="bytes given"):
        wd.wd_dslash(g, f[:100], o, 0.1, dims, wd.WD_FULL)
    with pytest.raises(ValueError, match="bytes given"):
        wd.wd_solve(g, f, o[:-16], 0.1, 1e-10)
    with pytest.raises(ValueError, match="not in GPU memory"):
        wd.wd_dslash(g, f.cpu(), o, 0.1, dims, wd.WD_FULL)
    with pytest.raises(ValueError, match="not contiguous"):
        wd.wd_norm2(g, torch.stack([f, f], 1).reshape(-1)[::2], 2, "f64")
    g.close()


# ------------------------------------------------------------------ full size
@pytest.fixture(scope="module")
def big():
    dims = (32, 32, 32, 64)
    U = syn.gauge_field(dims, 0.3, 1002)
    psi = syn.gaussian_spinor(dims, 2002)
    return dims, U, psi


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_full_size_sampled_sites(big, prec):
    """32^3x64 in the benchmark's launch configuration (the committed tuned
    variant of each precision: for FP16/BF16 spinors that is link preloading,
    cached stores and a wave cap), checked against the oracle at sampled
    sites, element by element."""
    dims, U, psi = big
    print(f"case: 32^3x64 sampled prec={prec}", flush=True)
    g = wd.Gauge(U, dims, -1, prec)
    # the committed tuning table is what the benchmark loads: same variant here
    table = os.path.join(os.path.dirname(wd.__file__), "tuned", "mi355x_hop.jsonl")
    key = "gfx950/hop/p%d/32x32x32x64" % wd.PRECS[prec]
    entries = [json.loads(line) for line in open(table) if line.strip()]
    want = [e for e in entries if e["key"] == key][-1]
    b, gr, oc, us = wd.wd_tune_dslash(g, prec, table)
    assert (b, gr, oc) == (want["block"], want["groups"], want["occ"])
    assert wd.wd_get_dslash_variant(g, prec) == (b, gr, oc)
    rng = np.random.default_rng(3)
    Ur = U if prec == "f64" else round_c64(U)
    pr = storage_round(psi, prec)
    for parity in (0, 1):
        src = to_field(g, psi, prec, 1 - parity)
        out = wd.wd_new_field(dims, prec, 1, parity)
        wd.wd_dslash(g, src, out, 1.0, dims, parity)
        got = from_field(g, out, prec, parity)
        sites = [(0, 0, 0, 0), (31, 31, 31, 63), (1, 0, 0, 63), (0, 31, 5, 0), (30, 2, 31, 1)]
        sites += [tuple(int(rng.integers(0, L)) for L in dims) for _ in range(200)]
        sites = [s for s in sites if sum(s) % 2 == parity]
        want = wilson.hop_sites(Ur, pr, sites)
        g_s = np.stack([got[x4, x3, x2, x1] for (x1, x2, x3, x4) in sites])
        assert_close(g_s, want, prec, what=f"32^3x64 {prec} p{parity} ({len(sites)} sites)")
        # sites of the other parity were not written
        assert np.all(got[wilson.parity_field(dims) != parity] == 0)
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "f16", "bf16"])
def test_full_size_marching_dirac(big, prec):
    """The one-launch D_W at 32^3x64 in the benchmark's launch configuration
    (FP64, FP32: the committed tuned variant, range length and tile shape;
    FP16, BF16: the default register-brick form): the whole field against
    the two single-parity launches, and sampled sites of both parities
    against the oracle's D_W = 1 - kappa H, element by element (FP16
    per-site bar 2^-10, as in the marching test above)."""
    dims, U, psi = big
    print(f"case: 32^3x64 one-launch D_W prec={prec}", flush=True)
    kappa = 0.124
    g = wd.Gauge(U, dims, -1, prec)
    if prec in ("f64", "f32"):
        table = os.path.join(os.path.dirname(wd.__file__), "tuned", "mi355x_hop.jsonl")
        key = "gfx950/dirac/p%d/32x32x32x64" % wd.PRECS[prec]
        entry = [json.loads(line) for line in open(table) if line.strip() and key in line][-1]
        sl, tile, _ = wd.wd_tune_dirac(g, prec, table)
        assert (sl, tile) == (entry["slices"], entry["groups"]) == wd.wd_get_dirac_variant(g, prec)
    else:
        assert wd.wd_get_dirac_variant(g, prec) == (0, 2)
    src = to_field(g, psi, prec)
    one = wd.wd_new_field(dims, prec)
    two = wd.wd_new_field(dims, prec)
    wd.wd_dslash_ex(g, src, one, kappa, wd.WD_FULL, prec, wd.WD_ONE_PASS)
    wd.wd_dslash_ex(g, src, two, kappa, wd.WD_FULL, prec, 0)
    got = from_field(g, one, prec)
    assert rel_err(got, from_field(g, two, prec)) <= {"f64": 1e-14, "f32": 1e-6, "f16": 1e-3, "bf16": 2.0 ** -8}[prec]
    Ur = U if prec == "f64" else round_c64(U)
    pr = storage_round(psi, prec)
    rng = np.random.default_rng(5)
    sites = [(0, 0, 0, 0), (31, 31, 31, 63), (0, 0, 0, 31), (0, 0, 0, 32), (31, 3, 1, 63), (5, 7, 15, 16)]
    sites += [tuple(int(rng.integers(0, L)) for L in dims) for _ in range(200)]
    want = np.stack([pr[x4, x3, x2, x1] for (x1, x2, x3, x4) in sites]) - kappa * wilson.hop_sites(Ur, pr, sites)
    g_s = np.stack([got[x4, x3, x2, x1] for (x1, x2, x3, x4) in sites])
    site = 2.0 ** -10 + 4e-6 if prec == "f16" else None
    assert_close(g_s, want, prec, site=site, what=f"32^3x64 one-launch D_W {prec} ({len(sites)} sites)")
    g.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (6, 4, 6, 10)])
def test_fp64_hop_on_haar_and_gauge_transformed_links(dims):
    """Links that are not near the identity: Haar-random SU(3) on every link,
    and the eps = 0.3 field after a Haar-random gauge transformation.  The
    compressed storage rebuilds row 2 as conj(row0 x row1), which holds for
    any SU(3) matrix up to rounding, so FP64 still meets 1e-13 site by site;
    the transformed hop must also equal Omega times the original."""
    L1, L2, L3, L4 = dims
    V = L1 * L2 * L3 * L4
    Uh = syn.random_su3(4 * V, 51).reshape(L4, L3, L2, L1, 4, 3, 3)
    psi = syn.gaussian_spinor(dims, 52)
    for name, U in (("haar", Uh),):
        g = wd.Gauge(U, dims, -1, "f64")
        for parity in (0, 1):
            out = wd.wd_new_field(dims, "f64", 1, parity)
            wd.wd_dslash(g, to_field(g, psi, "f64", 1 - parity), out, 1.0, dims, parity)
            assert_close(from_field(g, out, "f64", parity), wilson.hop_parity(U, psi, parity), "f64",
                         what=f"{name} links {dims} p{parity}")
        g.close()
    U0 = syn.gauge_field(dims, 0.3, 53)
    Om = syn.random_su3(V, 54).reshape(L4, L3, L2, L1, 3, 3)
    Ut, pt = wilson.gauge_transform(U0, psi, Om)
    g0 = wd.Gauge(U0, dims, -1, "f64")
    gt = wd.Gauge(Ut, dims, -1, "f64")
    for parity in (0, 1):
        o0 = wd.wd_new_field(dims, "f64", 1, parity)
        ot = wd.wd_new_field(dims, "f64", 1, parity)
        wd.wd_dslash(g0, to_field(g0, psi, "f64", 1 - parity), o0, 1.0, dims, parity)
        wd.wd_dslash(gt, to_field(gt, pt, "f64", 1 - parity), ot, 1.0, dims, parity)
        got_t = from_field(gt, ot, "f64", parity)
        assert_close(got_t, wilson.hop_parity(Ut, pt, parity), "f64", what=f"transformed links {dims} p{parity}")
        # covariance on the GPU outputs themselves: H[U^Om](Om psi) = Om H[U] psi
        assert_close(got_t, wilson.colour_mul(Om, from_field(g0, o0, "f64", parity)), "f64",
                     what=f"covariance {dims} p{parity}")
    g0.close()
    gt.close()


def test_full_size_plane_wave():
    """Unit links at 32^3x64: D_W e^{ipx}u = symbol(p) u e^{ipx} at every site."""
    dims = (32, 32, 32, 64)
    U = syn.unit_gauge(dims)
    g = wd.Gauge(U, dims, -1, "f64")
    n = (3, 30, 1, 7)
    p = free_field.momentum_of(dims, n)  # p_4 = 2 pi (7 + 1/2) / 64
    u = syn.gaussian_spinor((2, 2, 2, 2), 5)[0, 0, 0, 0]
    # phases reduced exactly: unreduced, the rounding of p.x (up to ~260 here)
    # alone would put ~3e-14 into every site
    psi = free_field.plane_wave_n(dims, n, u)
    src = to_field(g, psi)
    out = wd.wd_new_field(dims, "f64")
    wd.wd_dslash(g, src, out, 0.124, dims, wd.WD_FULL)
    got = from_field(g, out)
    want = free_field.plane_wave_n(dims, n, free_field.symbol(p, 0.124) @ u)
    assert_close(got, want, "f64", what="32^3x64 plane wave")
    g.close()


# ------------------------------------------------------------ largest fields
@pytest.fixture(scope="module")
def largest():
    """32^3 x 384 (12,582,912 sites): one parity's FP64 hop links take 4.8 GB
    and FP32 2.4 GB, a full FP64 field 2.4 GB, so device offsets run past 2^31
    and 2^32 bytes.  The links are a random 32^3 x 8 block repeated along x4,
    each copy multiplied on the right by its own Haar SU(3) matrix (still
    SU(3), no two time blocks alike); the spinors are Gaussian everywhere."""
    dims = (32, 32, 32, 384)
    small = syn.gauge_field((32, 32, 32, 8), 0.3, 1004)
    R = syn.random_su3(48, 1005)
    U = np.empty((384,) + small.shape[1:], dtype=np.complex128)
    for b in range(48):
        U[8 * b:8 * b + 8] = small @ R[b]
    psi = syn.gaussian_spinor(dims, 2004)
    return dims, U, psi


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_largest_fields_sampled_sites(largest, prec):
    """The single-parity hop (both parities) and the one-launch D_W on the
    32^3 x 384 lattice, in their default launch configurations, against the
    oracle at sampled sites (the last time slice included, where the offsets
    are largest), element by element."""
    dims, U, psi = largest
    print(f"case: 32^3x384 largest fields prec={prec}", flush=True)
    kappa = 0.124
    g = wd.Gauge(U, dims, -1, prec)
    Ur = U if prec == "f64" else round_c64(U)
    pr = storage_round(psi, prec)
    rng = np.random.default_rng(7)
    edge = [(0, 0, 0, 0), (31, 31, 31, 383), (0, 0, 0, 383), (31, 31, 31, 382), (1, 0, 0, 383), (30, 31, 31, 191)]
    last = (wilson.parity_field(dims[:3] + (1,))[0] + dims[3] - 1) % 2  # parity of the last slice's sites
    for parity in (0, 1):
        src = to_field(g, psi, prec, 1 - parity)
        out = wd.wd_new_field(dims, prec, 1, parity)
        wd.wd_dslash(g, src, out, 1.0, dims, parity)
        got = from_field(g, out, prec, parity)
        del src, out
        sites = edge + [tuple(int(rng.integers(0, L)) for L in dims) for _ in range(200)]
        sites = [s for s in sites if sum(s) % 2 == parity]
        want = wilson.hop_sites(Ur, pr, sites)
        g_s = np.stack([got[x4, x3, x2, x1] for (x1, x2, x3, x4) in sites])
        assert_close(g_s, want, prec, what=f"32^3x384 hop {prec} p{parity} ({len(sites)} sites)")
        # the other parity's sites of the last slice were not written
        assert np.all(got[-1][last != parity] == 0)
        del got
    src = to_field(g, psi, prec)
    one = wd.wd_new_field(dims, prec)
    wd.wd_dslash_ex(g, src, one, kappa, wd.WD_FULL, prec, wd.WD_ONE_PASS)
    got = from_field(g, one, prec)
    del src, one
    sites = edge + [tuple(int(rng.integers(0, L)) for L in dims) for _ in range(200)]
    want = np.stack([pr[x4, x3, x2, x1] for (x1, x2, x3, x4) in sites]) - kappa * wilson.hop_sites(Ur, pr, sites)
    g_s = np.stack([got[x4, x3, x2, x1] for (x1, x2, x3, x4) in sites])
    assert_close(g_s, want, prec, what=f"32^3x384 one-launch D_W {prec} ({len(sites)} sites)")
    g.close()


@pytest.mark.parametrize("dims", [(8, 8, 8, 8), (16, 16, 16, 16), (6, 4, 6, 10)])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_every_hop_variant_is_bitwise_identical(dims, prec):
    """Block size, block -> tile order (box orders -101 .. -108 included) and
    the other schedule knobs (store policy, link preloading, sites per lane,
    LDS staging of the input tile) change only the schedule, never a result
    bit."""
    U, psi, _, _ = _inputs(dims, prec, seed=15)
    g = wd.Gauge(U, dims, -1, prec)
    src = to_field(g, psi, prec, wd.WD_ODD)
    ref = wd.wd_new_field(dims, prec, 1, wd.WD_EVEN)
    wd.wd_set_dslash_variant(g, prec, 256, 0, 0)
    wd.wd_dslash_ex(g, src, ref, 0.9, wd.WD_EVEN, prec)
    ref_dag = wd.wd_new_field(dims, prec, 1, wd.WD_EVEN)
    wd.wd_dslash_ex(g, src, ref_dag, 0.9, wd.WD_EVEN, prec, wd.WD_DAGGER)
    n = 0
    for bs, groups, occ in [(b, gr, o) for b in (64, 128, 256, 512) for gr in (0, 2, 4, 8, 16, -2, -4, -8, -16, -101, -102, -104, -108) for o in (0, 4, 256, 512, 516, 1024, 2048, 1536, 2308, 4096, 4100, 4352)]:
            try:
                wd.wd_set_dslash_variant(g, prec, bs, groups, occ)
            except wd.WdError:
                continue
            out = wd.wd_new_field(dims, prec, 1, wd.WD_EVEN)
            out.fill_(0xAB)
            wd.wd_dslash_ex(g, src, out, 0.9, wd.WD_EVEN, prec)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (bs, groups, occ)
            out.fill_(0xAB)
            wd.wd_dslash_ex(g, src, out, 0.9, wd.WD_EVEN, prec, wd.WD_DAGGER)
            torch.cuda.synchronize()
            assert torch.equal(out, ref_dag), ("dagger", bs, groups, occ)
            n += 1
    assert n >= 4
    b, gr, oc, us = wd.wd_tune_dslash(g, prec)
    assert wd.wd_get_dslash_variant(g, prec) == (b, gr, oc) and us > 0
    g.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_lds_staged_hop_in_a_solve_is_bitwise_the_default(prec):
    """The LDS-staged variant in every form a solver launches it (dagger,
    xpay and xmy epilogues, fused norms, FP64 true residual): an FP64 CG solve
    (prec f64) or an FP32 defect-correction solve (prec f32) gives the same
    bytes and iteration counts with the staged hop as with the default one."""
    dims, kappa = (8, 8, 8, 8), 0.124
    U = syn.gauge_field(dims, 0.3, 1701)
    b = syn.gaussian_spinor(dims, 1702)
    g = wd.Gauge(U, dims, -1, "f64")
    fb = to_field(g, b)
    kw = dict(solver=wd.WD_SOLVER_CG) if prec == "f64" else dict(solver=wd.WD_SOLVER_DEFECT_CG, inner_prec="f32",
                                                                   inner_tol=1e-4)
    outs = []
    for occ in (0, wd.WD_TUNE_STAGE_LDS):
        for p in ("f64", "f32"):
            wd.wd_set_dslash_variant(g, p, 128, 0, occ)
        fx = wd.wd_new_field(dims, "f64")
        rc, info = wd.wd_solve(g, fb, fx, kappa, 1e-10, wd.wd_solve_params_default(**kw))
        assert rc == 0
        outs.append((fx.clone(), info["iters"], info["outer_iters"]))
    assert outs[0][1:] == outs[1][1:]
    assert torch.equal(outs[0][0], outs[1][0])
    g.close()
