"""Device Gaussian fields (Philox4x64-10 + Box-Muller) against the Python
reference of the definition in include/wd.h, value by value."""
import numpy as np
import pytest
import torch

import paper_0710_2442_amd as wd
import synthetic as syn
from philox_ref import gaussian_stored

pytestmark = pytest.mark.gpu


def _stored(f, prec, vpad, nhalf):
    """Device bytes -> stored components [half][site][12] (chunked layout of wd.h)."""
    nc = vpad // 64
    if prec == "f64":
        a = f.cpu().numpy().view(np.complex128).reshape(nhalf, nc, 12, 64)
    else:
        a = f.cpu().numpy().view(np.complex64).reshape(nhalf, nc, 6, 64, 2).transpose(0, 1, 2, 4, 3)
        a = a.reshape(nhalf, nc, 12, 64)
    return a.transpose(0, 1, 3, 2).reshape(nhalf, vpad, 12)


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("parity", [wd.WD_FULL, wd.WD_EVEN, wd.WD_ODD])
def test_gaussian_field_matches_definition(prec, parity):
    dims = (6, 4, 2, 4)  # V_h = 96 in 256 slots: two chunks, padding
    g = wd.Gauge(syn.unit_gauge(dims), dims, -1, "f64")
    vh, vpad = 96, wd.wd_vh_pad(dims)
    f = wd.wd_new_field(dims, prec, 1, parity)
    f.fill_(0xAB)
    seed, stream = 0x1234_5678_9ABC_DEF0, 77
    wd.wd_gaussian_field(g, f, parity, prec, seed, stream)
    torch.cuda.synchronize()
    pars = (0, 1) if parity == wd.WD_FULL else (parity,)
    got = _stored(f, prec, vpad, len(pars))
    want = gaussian_stored(vh, seed, stream, pars)
    assert np.all(got[:, vh:] == 0)
    if prec == "f64":
        assert np.max(np.abs(got[:, :vh] - want)) <= 1e-13 * np.max(np.abs(want))
    else:
        assert np.max(np.abs(got[:, :vh] - want.astype(np.complex64))) <= 2 ** -22 * np.max(np.abs(want))
    g.close()


def test_gaussian_field_statistics_and_streams():
    dims = (16, 16, 16, 16)
    g = wd.Gauge(syn.unit_gauge(dims), dims, -1, "f64")
    a = wd.wd_new_field(dims, "f64")
    b = wd.wd_new_field(dims, "f64")
    wd.wd_gaussian_field(g, a, wd.WD_FULL, "f64", 9, 0)
    wd.wd_gaussian_field(g, b, wd.WD_FULL, "f64", 9, 1)
    torch.cuda.synchronize()
    va = a.cpu().numpy().view(np.float64)
    vb = b.cpu().numpy().view(np.float64)
    assert abs(va.mean()) < 5e-3 and abs(va.var() - 1) < 5e-3
    assert abs(np.corrcoef(va, vb)[0, 1]) < 5e-3
    c = wd.wd_new_field(dims, "f64")
    wd.wd_gaussian_field(g, c, wd.WD_FULL, "f64", 9, 0)
    torch.cuda.synchronize()
    assert torch.equal(a, c)
    g.close()
