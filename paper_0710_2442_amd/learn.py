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
    """Streams normalised (r, e) pairs, FP32 full fields, on one lattice.

    Every buffer is allocated once: the sources of one solve call, and two
    rings of nsrc * len(ks) FP32 pair slots into which the library writes
    each normalised pair directly (in a random slot order, so a run of
    consecutive slots is a random sample of the call's pairs).  batch()
    hands out consecutive slots as views; they stay valid until the next
    call of batch() and are written only by work queued on the same stream
    after the caller's own use of them."""

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
        self.slots = self.nsrc * len(self.ks)
        self.sources = 0
        self.solve_seconds = 0.0
        self._B = L.wd_new_field(self.dims, "f64", self.nsrc)
        self._xs = L.wd_new_field(self.dims, "f64", self.nsrc)
        self._xk = L.wd_new_field(self.dims, "f64")
        self._dx = L.wd_new_field(self.dims, "f64")
        self._r1 = L.wd_new_field(self.dims, "f64")
        self._e1 = L.wd_new_field(self.dims, "f64")
        self._pr = L.wd_new_field(self.dims, "f32", self.slots)
        self._pe = L.wd_new_field(self.dims, "f32", self.slots)
        self._next = self.slots  # first slot not yet handed out
        self._perm = None

    def _field(self, buf, i, nbytes):
        return buf[i * nbytes:(i + 1) * nbytes]

    def _push(self, j, r, e):
        """Normalise pair j of this refill by |r| into its FP32 slot."""
        nr = np.sqrt(L.wd_norm2(self.g, r, 2, "f64"))
        slot = int(self._perm[j])
        L.wd_convert(self.g, r, "f64", self._field(self._pr, slot, self.f32), "f32", 2, 1.0 / nr)
        L.wd_convert(self.g, e, "f64", self._field(self._pe, slot, self.f32), "f32", 2, 1.0 / nr)

    def _refill(self):
        t = time.perf_counter()
        n = self.nsrc
        # Gaussian sources drawn on the device (counter-based generator:
        # stream = the source's running index, so every source differs)
        for y in range(n):
            L.wd_gaussian_field(self.g, self._field(self._B, y, self.f64), L.WD_FULL, "f64", self.seed, self.sources)
            self.sources += 1
        prm = L.wd_solve_params_default(solver=L.WD_SOLVER_DEFECT_CG, inner_prec=self.inner_prec,
                                        inner_tol=self.inner_tol)
        rc, infos = L.wd_solve_mrhs(self.g, self._B, self._xs, n, self.kappa, self.target_tol, prm)
        if rc != 0:
            bad = [y for y, i in enumerate(infos) if i["status"] != 0]
            raise RuntimeError(f"pair generation: sources {bad} did not reach {self.target_tol}")
        self._perm = self.rng.permutation(self.slots)
        j = 0
        for y in range(n):
            fb, xs = self._field(self._B, y, self.f64), self._field(self._xs, y, self.f64)
            for k in self.ks:
                if k == 0:  # x_0 = 0: r = b, e = x*
                    self._push(j, fb, xs)
                else:
                    L.wd_solve(self.g, fb, self._xk, self.kappa, 1e-14,
                               L.wd_solve_params_default(solver=L.WD_SOLVER_CG, max_iter=k))
                    # r = b - D x_k  ;  e = x* - x_k
                    L.wd_dslash(self.g, self._xk, self._dx, self.kappa, self.dims, L.WD_FULL)
                    self._r1.copy_(fb)
                    L.wd_caxpy(self.g, -1.0, self._dx, self._r1, 2, "f64")
                    self._e1.copy_(xs)
                    L.wd_caxpy(self.g, -1.0, self._xk, self._e1, 2, "f64")
                    self._push(j, self._r1, self._e1)
                j += 1
        self._next = 0
        self.torch.cuda.synchronize()
        self.solve_seconds += time.perf_counter() - t

    def batch(self, B):
        """B pairs as two views of B consecutive FP32 full fields each (valid
        until the next call).  A refill's last slots that cannot fill a whole
        batch are dropped."""
        B = int(B)
        if B > self.slots:
            raise ValueError(f"batch of {B} pairs, but one refill makes {self.slots}")
        if self._next + B > self.slots:
            self._refill()
        a, self._next = self._next, self._next + B
        return (self._pr[a * self.f32:(a + B) * self.f32], self._pe[a * self.f32:(a + B) * self.f32])


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
