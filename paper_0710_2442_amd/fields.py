"""Moving canonical numpy spinors in and out of device fields (marshalling only)."""
from __future__ import annotations

import numpy as np

from . import _lib as L


def canon_to_field(g, psi, prec="f64", parity=L.WD_FULL, device="cuda"):
    """Canonical complex128 spinor (numpy, host) -> new device field."""
    import torch

    canon = torch.from_numpy(np.ascontiguousarray(psi, dtype=np.complex128).reshape(-1)).to(device)
    f = L.wd_new_field(g.dims, prec, 1, parity, device)
    L.wd_spinor_pack(g, canon, f, parity, prec)
    return f


def field_to_canon(g, f, prec="f64", parity=L.WD_FULL, device="cuda"):
    """Device field -> canonical complex128 numpy spinor (unconverted sites = 0)."""
    import torch

    L1, L2, L3, L4 = g.dims
    canon = torch.zeros(L1 * L2 * L3 * L4 * 12, dtype=torch.complex128, device=device)
    L.wd_spinor_unpack(g, f, canon, parity, prec)
    torch.cuda.synchronize()
    return canon.cpu().numpy().reshape(L4, L3, L2, L1, 4, 3)


def half(f, g, prec, which):
    """View of the even (0) or odd (1) half of a full field buffer."""
    hb = L.wd_field_bytes(g.dims, prec, 1, L.WD_EVEN)
    return f[which * hb:(which + 1) * hb]
