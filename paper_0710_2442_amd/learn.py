"""Training driver of the learned preconditioner (orchestration only).

Pairs (r, e) come from the solver itself: for Gaussian sources b the
solutions x* are computed together by the multi-RHS defect-correction solver
(`nsrc` sources per call, BF16 inner storage, to 1e-6: the trained network's
own relative error is ~25%, so tighter targets buy nothing; 24 sources per
call with BF16 make pairs 30% faster than 12 with FP32 on 16^4); FP64 CG
stopped after k iterations (k in `ks`) gives x_k,
e_k = x* - x_k and r_k = b - D x_k = D e_k.  Each pair is normalised by
|r_k|.  The default uses k = 0 only (x_0 = 0: r = b, e = x*): residuals of
later CG iterates are dominated by the low modes, and a network trained on
them raised FGCR's iteration count (8^4, kappa 0.124: 88 with N = 1, 215-731
with such pairs, 35 with k = 0 pairs).  Every step of this runs in the
library's kernels (solves, hop, caxpy, conversion); this module only
sequences the calls; the Gaussian sources are drawn on the device by the
library's counter-based generator (seed, source index).

Training: Adam on L = mean |N(r) - e|^2 over mini-batches streamed from the
generator (pairs are not stored beyond a small pool).
"""
from __future__ import annotations

import time

import numpy as np

from . import _lib as L


class PairGenerator:
    """Streams normalised (r, e) pairs, FP32 full fields, on one lattice."""

    def __init__(self, g, kappa, seed, ks=(0,), target_tol=1e-6, nsrc=24, inner_prec="bf16", inner_tol=1e-2):
        import torch

        self.torch = torch
        self.g = g
        self.kappa = float(kappa)
        self.seed = int(seed)
        self.rng = np.random.Generator(np.random.PCG64(int(seed)))
        self.ks = tuple(int(k) for k in ks)
        self.target_tol = float(target_tol)
        self.nsrc = int(nsrc)
        self.inner_prec = inner_prec
        self.inner_tol = float(inner_tol)
        self.dims = g.dims
        self.f64 = L.wd_field_bytes(self.dims, "f64")
        self.f32 = L.wd_field_bytes(self.dims, "f32")
        self.pool_r, self.pool_e = [], []
        self.sources = 0
        self.solve_seconds = 0.0
        self._xs = L.wd_new_field(self.dims, "f64", self.nsrc)
        self._xk = L.wd_new_field(self.dims, "f64")
        self._dx = L.wd_new_field(self.dims, "f64")

    def _source(self):
        """A Gaussian source drawn on the device (counter-based generator:
        stream = the source's running index, so every source differs)."""
        f = L.wd_new_field(self.dims, "f64")
        L.wd_gaussian_field(self.g, f, L.WD_FULL, "f64", self.seed, self.sources)
        self.sources += 1
        return f

    def _push(self, r, e):
        """Normalise the pair by |r| and keep it as two FP32 full fields."""
        nr = np.sqrt(L.wd_norm2(self.g, r, 2, "f64"))
        r32 = L.wd_new_field(self.dims, "f32")
        e32 = L.wd_new_field(self.dims, "f32")
        L.wd_convert(self.g, r, "f64", r32, "f32", 2, 1.0 / nr)
        L.wd_convert(self.g, e, "f64", e32, "f32", 2, 1.0 / nr)
        self.pool_r.append(r32)
        self.pool_e.append(e32)

    def _refill(self):
        t = time.perf_counter()
        n = self.nsrc
        B = self.torch.cat([self._source() for _ in range(n)])
        prm = L.wd_solve_params_default(solver=L.WD_SOLVER_DEFECT_CG, inner_prec=self.inner_prec,
                                        inner_tol=self.inner_tol)
        rc, infos = L.wd_solve_mrhs(self.g, B, self._xs, n, self.kappa, self.target_tol, prm)
        if rc != 0:
            bad = [y for y, i in enumerate(infos) if i["status"] != 0]
            raise RuntimeError(f"pair generation: sources {bad} did not reach {self.target_tol}")
        f = self.f64
        for y in range(n):
            fb, xs = B[y * f:(y + 1) * f], self._xs[y * f:(y + 1) * f]
            for k in self.ks:
                if k == 0:  # x_0 = 0: r = b, e = x*
                    self._push(fb, xs)
                    continue
                L.wd_solve(self.g, fb, self._xk, self.kappa, 1e-14,
                           L.wd_solve_params_default(solver=L.WD_SOLVER_CG, max_iter=k))
                # r = b - D x_k  ;  e = x* - x_k
                L.wd_dslash(self.g, self._xk, self._dx, self.kappa, self.dims, L.WD_FULL)
                r = fb.clone()
                L.wd_caxpy(self.g, -1.0, self._dx, r, 2, "f64")
                e = xs.clone()
                L.wd_caxpy(self.g, -1.0, self._xk, e, 2, "f64")
                self._push(r, e)
        self.torch.cuda.synchronize()
        self.solve_seconds += time.perf_counter() - t

    def batch(self, B):
        """B pairs as two tensors of B consecutive FP32 full fields."""
        while len(self.pool_r) < B:
            self._refill()
        order = self.rng.permutation(len(self.pool_r))[:B]
        r = self.torch.cat([self.pool_r[i] for i in order])
        e = self.torch.cat([self.pool_e[i] for i in order])
        keep = [i for i in range(len(self.pool_r)) if i not in set(order.tolist())]
        self.pool_r = [self.pool_r[i] for i in keep]
        self.pool_e = [self.pool_e[i] for i in keep]
        return r, e


# Weight checkpoint: a small versioned binary (little-endian).
#   bytes 0-7   magic b"WDPTC\x00\x00\x00"
#   8-11        format version (uint32, 1)
#   12-15       number of float32 weights (uint32, 1152 = 576 complex)
#   16-19       length of the JSON metadata in bytes (uint32)
#   20-23       CRC-32 of everything after the header (metadata + weights)
#   then the UTF-8 JSON metadata, then the weights in the library's order
#   ([layer][h][c'][c][4][4] complex, (re, im) interleaved).
CKPT_MAGIC = b"WDPTC\x00\x00\x00"
CKPT_VERSION = 1
N_WEIGHTS = 1152


def save_weights(path, flat, meta=None):
    """Write the 1152 FP32 network weights and a JSON-able metadata dict."""
    import json
    import struct
    import zlib

    w = np.ascontiguousarray(np.asarray(flat, dtype="<f4").reshape(-1))
    if w.size != N_WEIGHTS:
        raise ValueError(f"PTC weights: {N_WEIGHTS} floats expected, got {w.size}")
    m = json.dumps(meta or {}, sort_keys=True).encode()
    body = m + w.tobytes()
    head = CKPT_MAGIC + struct.pack("<IIII", CKPT_VERSION, N_WEIGHTS, len(m), zlib.crc32(body) & 0xFFFFFFFF)
    with open(path, "wb") as f:
        f.write(head + body)


def load_weights(path):
    """Read a checkpoint written by save_weights: (float32 array of 1152, metadata dict).
    Raises ValueError for a wrong magic, version or size, or a damaged body."""
    import json
    import struct
    import zlib

    with open(path, "rb") as f:
        data = f.read()
    if len(data) < 24 or data[:8] != CKPT_MAGIC:
        raise ValueError("not a PTC weight checkpoint")
    version, n, mlen, crc = struct.unpack("<IIII", data[8:24])
    if version != CKPT_VERSION:
        raise ValueError(f"PTC checkpoint version {version}, this library reads {CKPT_VERSION}")
    if n != N_WEIGHTS or len(data) != 24 + mlen + 4 * n:
        raise ValueError("PTC checkpoint: wrong size")
    body = data[24:]
    if zlib.crc32(body) & 0xFFFFFFFF != crc:
        raise ValueError("PTC checkpoint: checksum mismatch")
    meta = json.loads(body[:mlen].decode())
    w = np.frombuffer(body[mlen:], dtype="<f4").astype(np.float32)
    return w, meta


def init_weights(seed, scale=1e-2):
    """Near-identity start: W^(0) = I/sqrt(2) in both layers, other hops N(0, scale^2)."""
    rng = np.random.Generator(np.random.PCG64(int(seed)))
    z1 = rng.standard_normal((9, 2, 1, 4, 4, 2))
    z2 = rng.standard_normal((9, 1, 2, 4, 4, 2))
    W1 = scale * (z1[..., 0] + 1j * z1[..., 1]) / np.sqrt(2)
    W2 = scale * (z2[..., 0] + 1j * z2[..., 1]) / np.sqrt(2)
    for W in (W1, W2):
        for co in range(W.shape[1]):
            for c in range(W.shape[2]):
                W[0, co, c] = np.eye(4) / np.sqrt(2)
    return L.ptc_weights_to_flat(W1, W2)


def train(g, kappa, steps=300, batch=8, lr=2e-3, seed=5, act="bf16", log_every=50, log=None, ks=(0,),
          checkpoint=None):
    """Train a PTC network on lattice g.  Returns (flat weights, history dict);
    with checkpoint (a path) the weights are also written by save_weights."""
    gen = PairGenerator(g, kappa, seed, ks)
    net = L.Ptc(g, init_weights(seed + 1), act)
    losses = []
    t0 = time.perf_counter()
    for s in range(steps):
        r, e = gen.batch(batch)
        want = (s % log_every == 0) or s == steps - 1
        loss = L.wd_ptc_train_step(net, r, e, batch, lr * (0.1 if s > 0.8 * steps else 1.0), want_loss=want)
        if want:
            losses.append((s, loss))
            if log:
                log(f"ptc step {s}: loss {loss:.4f}")
    import torch

    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    W = L.wd_ptc_get_weights(net)
    net.close()
    hist = {"losses": losses, "pairs": steps * batch, "sources": gen.sources, "seconds": wall,
            "pair_generation_seconds": gen.solve_seconds}
    if checkpoint:
        save_weights(checkpoint, W, {"dims": list(g.dims), "kappa": float(kappa), "steps": steps, "batch": batch,
                                     "lr": lr, "seed": seed, "act": act, "final_loss": losses[-1][1] if losses else None})
    return W, hist
