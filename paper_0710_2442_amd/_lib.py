"""ctypes declarations of libwd.so and argument marshalling.

Only pointers, sizes and scalars cross into the library.  torch supplies
device memory and the current stream; nothing here computes on field data.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libwd.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first "
        "(python -c 'import __graft_entry__; __graft_entry__.build()')"
    )

# torch first: libwd.so then binds to the HIP runtime torch has already
# loaded (one runtime per process, the one that owns torch's device memory
# and streams) instead of loading a second copy of its own
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)

WD_F64, WD_F32, WD_F16, WD_BF16 = 0, 1, 2, 3
PRECS = {"f64": WD_F64, "f32": WD_F32, "f16": WD_F16, "bf16": WD_BF16}
WD_EVEN, WD_ODD, WD_FULL = 0, 1, 2
WD_DAGGER = 1
WD_ONE_PASS = 2
WD_TUNE_CACHED_STORE = 256
WD_TUNE_PRELOAD_LINKS = 512
WD_TUNE_SPL_SHIFT = 10
WD_TUNE_STAGE_LDS = 4096
WD_PTC_FP16_PRODUCTS = 1
WD_PTC_BF16_MFMA = 2
WD_SOLVER_CG, WD_SOLVER_DEFECT_CG, WD_SOLVER_FGCR, WD_SOLVER_DEFECT_FGCR, WD_SOLVER_CGLS_FULL = 0, 1, 2, 3, 4

_vp = C.c_void_p
_int4 = C.c_int * 4


class wd_solve_params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_size_t),
        ("solver", C.c_int),
        ("inner_prec", C.c_int),
        ("inner_tol", C.c_double),
        ("max_iter", C.c_int),
        ("check_every", C.c_int),
        ("use_graph", C.c_int),
        ("fgcr_m", C.c_int),
        ("precond", C.c_void_p),
        ("batch_tile", C.c_int),
        ("batch_blocks_per_cu", C.c_int),
    ]


class wd_solve_info(C.Structure):
    _fields_ = [
        ("iters", C.c_int),
        ("outer_iters", C.c_int),
        ("dslash_calls", C.c_int),
        ("true_rel_resid", C.c_double),
        ("seconds", C.c_double),
        ("fallback_used", C.c_int),
        ("status", C.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


def _decl(name, restype, argtypes):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


_decl("wd_gauge_create", C.c_int, [_vp, _int4, C.c_int, C.c_int, _vp, C.POINTER(_vp)])
_decl("wd_gauge_destroy", C.c_int, [_vp])
_decl("wd_gauge_set_stream", C.c_int, [_vp, _vp])
_decl("wd_vh_pad", C.c_size_t, [_int4])
_decl("wd_field_bytes", C.c_size_t, [_int4, C.c_int, C.c_int, C.c_int])
_decl("wd_spinor_pack", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int])
_decl("wd_spinor_unpack", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int])
_decl("wd_dslash", C.c_int, [_vp, _vp, _vp, C.c_double, _int4, C.c_int])
_decl("wd_dslash_ex", C.c_int, [_vp, _vp, _vp, C.c_double, C.c_int, C.c_int, C.c_int])
_decl("wd_dslash_mrhs", C.c_int, [_vp, _vp, _vp, C.c_double, C.c_int, C.c_int, C.c_int])
_decl("wd_caxpy", C.c_int, [_vp, C.c_double, C.c_double, _vp, _vp, C.c_int, C.c_int])
_decl("wd_cdot", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_int, C.POINTER(C.c_double)])
_decl("wd_norm2", C.c_int, [_vp, _vp, C.c_int, C.c_int, C.POINTER(C.c_double)])
_decl("wd_convert", C.c_int, [_vp, _vp, C.c_int, _vp, C.c_int, C.c_int, C.c_double])
_decl("wd_solve_params_default", None, [C.POINTER(wd_solve_params)])
_decl("wd_solve", C.c_int, [_vp, _vp, _vp, C.c_double, C.c_double, C.POINTER(wd_solve_params),
                             C.POINTER(wd_solve_info)])
_decl("wd_solve_noalloc", C.c_int, [_vp, _vp, _vp, C.c_double, C.c_double, C.POINTER(wd_solve_params),
                                     C.POINTER(wd_solve_info)])
_decl("wd_solve_mrhs", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, C.c_double,
                                  C.POINTER(wd_solve_params), C.POINTER(wd_solve_info)])
_decl("wd_solve_batch", C.c_int, [C.POINTER(_vp), C.c_int, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(C.c_double),
                                   C.c_double, C.POINTER(wd_solve_params), C.POINTER(wd_solve_info)])
_decl("wd_tune_batch", C.c_int, [C.POINTER(_vp), C.c_int, C.POINTER(_vp), C.POINTER(_vp), C.POINTER(C.c_double),
                                  C.c_double, C.POINTER(wd_solve_params), C.c_char_p, C.c_int, C.POINTER(C.c_int),
                                  C.POINTER(C.c_int), C.POINTER(C.c_double)])
_decl("wd_tune_dslash", C.c_int, [_vp, C.c_int, C.c_char_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                   C.POINTER(C.c_int), C.POINTER(C.c_double)])
_decl("wd_tune_dslash_mrhs", C.c_int, [_vp, C.c_int, C.c_int, C.c_char_p, C.c_int, C.POINTER(C.c_int),
                                       C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_double)])
_decl("wd_set_dslash_variant", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int])
_decl("wd_tune_dirac", C.c_int, [_vp, C.c_int, C.c_char_p, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                 C.POINTER(C.c_double)])
_decl("wd_set_dirac_variant", C.c_int, [_vp, C.c_int, C.c_int, C.c_int])
_decl("wd_get_dirac_variant", C.c_int, [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int)])
_decl("wd_get_dslash_variant", C.c_int, [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)])
_decl("wd_set_dslash_mrhs_variant", C.c_int, [_vp, C.c_int, C.c_int, C.c_int, C.c_int])
_decl("wd_get_dslash_mrhs_variant", C.c_int,
      [_vp, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(C.c_int)])
_decl("wd_ptc_create", C.c_int, [_vp, C.POINTER(C.c_float), C.c_int, C.POINTER(_vp)])
_decl("wd_ptc_destroy", C.c_int, [_vp])
_decl("wd_ptc_set_weights", C.c_int, [_vp, C.POINTER(C.c_float)])
_decl("wd_ptc_get_weights", C.c_int, [_vp, C.POINTER(C.c_float)])
_decl("wd_ptc_apply", C.c_int, [_vp, _vp, _vp])
_decl("wd_ptc_apply_even", C.c_int, [_vp, _vp, C.c_int, _vp, C.c_int, C.c_int])
_decl("wd_ptc_loss_grad", C.c_int, [_vp, _vp, _vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_float)])
_decl("wd_ptc_train_step", C.c_int, [_vp, _vp, _vp, C.c_int, C.c_double, C.POINTER(C.c_double)])
_decl("wd_gaussian_field", C.c_int, [_vp, _vp, C.c_int, C.c_int, C.c_ulonglong, C.c_ulonglong])
_decl("wd_micro_lds_copy", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, _vp, C.POINTER(C.c_ulonglong),
                                     C.POINTER(C.c_uint)])
_decl("wd_micro_stream", C.c_int, [C.c_int, C.c_int, C.c_int, C.c_int, C.c_size_t, C.c_int,
                                   C.POINTER(C.c_double)])
_decl("wd_micro_resident", C.c_int, [C.c_int, C.c_size_t, C.c_int, C.c_int, C.POINTER(C.c_double)])
_decl("wd_halo_face_bytes", C.c_size_t, [_int4, C.c_int])
_decl("wd_halo_pack", C.c_int, [_vp, _vp, C.c_int, C.c_int, C.c_int, C.c_int, _vp])
_decl("wd_dslash_slab", C.c_int, [_vp, _vp, _vp, _vp, _vp, C.c_double, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int])
_decl("wd_status_string", C.c_char_p, [C.c_int])
_decl("wd_last_error", C.c_char_p, [])


class WdError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = lib.wd_last_error().decode(errors="replace")
        super().__init__(f"{where}: {lib.wd_status_string(status).decode()} ({status}): {msg}")


def _check(rc, where, allow_not_converged=False):
    if rc < 0 or (rc > 0 and not allow_not_converged):
        raise WdError(rc, where)
    return rc


def _prec(p):
    if isinstance(p, str):
        return PRECS[p]
    return int(p)


def _dims(d):
    return _int4(*[int(x) for x in d])


def _need(dims, prec, nrhs, parity):
    """Bytes of nrhs fields (0 for arguments the library itself rejects)."""
    try:
        return int(lib.wd_field_bytes(_dims(dims), _prec(prec), int(nrhs), int(parity)))
    except (KeyError, ValueError, TypeError):
        return 0


def _buf(t, nbytes, what):
    """Address of a caller buffer for the library, after checking it on the
    host: a contiguous torch tensor on a GPU holding at least nbytes bytes.
    The library cannot see buffer sizes, so a short buffer would be read or
    written past its end on the device."""
    if t is None:
        return None
    import torch

    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{what}: a torch device tensor is expected, got {type(t).__name__}")
    if not t.is_cuda:
        raise ValueError(f"{what}: the tensor is not in GPU memory")
    if not t.is_contiguous():
        raise ValueError(f"{what}: the tensor is not contiguous")
    have = t.numel() * t.element_size()
    if have < nbytes:
        raise ValueError(f"{what}: {have} bytes given, {nbytes} needed")
    return t.data_ptr()


def _canon_bytes(dims):
    return int(np.prod([int(d) for d in dims])) * 12 * 16


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def wd_status_string(s):
    return lib.wd_status_string(int(s)).decode()


def wd_vh_pad(dims):
    return int(lib.wd_vh_pad(_dims(dims)))


def wd_field_bytes(dims, prec, nrhs=1, parity=WD_FULL):
    n = int(lib.wd_field_bytes(_dims(dims), _prec(prec), int(nrhs), int(parity)))
    if n == 0:
        raise WdError(-1, "wd_field_bytes")
    return n


def wd_new_field(dims, prec, nrhs=1, parity=WD_FULL, device="cuda"):
    """Allocate an (uninitialised) device field buffer of the documented size."""
    import torch
    return torch.empty(wd_field_bytes(dims, prec, nrhs, parity), dtype=torch.uint8, device=device)


class Gauge:
    """Owning wrapper of a wd_gauge handle."""

    def __init__(self, U, dims, t_bc=-1, prec="f64"):
        U = np.ascontiguousarray(U, dtype=np.complex128)
        dims = tuple(int(d) for d in dims)
        V = int(np.prod(dims))
        if U.size != V * 36:
            raise ValueError(f"gauge field has {U.size} complex entries, expected {V * 36}")
        self.dims = dims
        self.prec = _prec(prec)
        self.t_bc = int(t_bc)
        h = C.c_void_p()
        rc = lib.wd_gauge_create(U.ctypes.data, _dims(dims), int(t_bc), self.prec, _stream(), C.byref(h))
        _check(rc, "wd_gauge_create")
        self.handle = h

    def sync_stream(self):
        lib.wd_gauge_set_stream(self.handle, _stream())

    def close(self):
        if getattr(self, "handle", None):
            lib.wd_gauge_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wd_gauge_create(U, dims, t_bc=-1, prec="f64"):
    return Gauge(U, dims, t_bc, prec)


def wd_gauge_destroy(g):
    g.close()


def wd_gauge_set_stream(g, stream=None):
    """Bind the handle to a HIP stream (default: torch's current stream)."""
    _check(lib.wd_gauge_set_stream(g.handle, _stream() if stream is None else C.c_void_p(stream)),
           "wd_gauge_set_stream")


def wd_last_error():
    """Message of the calling thread's last failed library call."""
    m = lib.wd_last_error()
    return m.decode(errors="replace") if m else ""


def wd_spinor_pack(g, canon, field, parity=WD_FULL, prec=None):
    g.sync_stream()
    p = g.prec if prec is None else _prec(prec)
    _check(lib.wd_spinor_pack(g.handle, _buf(canon, _canon_bytes(g.dims), "canon"),
                              _buf(field, _need(g.dims, p, 1, parity), "field"), int(parity), p), "wd_spinor_pack")


def wd_gaussian_field(g, field, parity, prec, seed, stream):
    """Fill a field with i.i.d. N(0,1) stored components (Philox4x64-10 + Box-Muller, on the device)."""
    g.sync_stream()
    _check(lib.wd_gaussian_field(g.handle, _buf(field, _need(g.dims, prec, 1, parity), "field"), int(parity),
                                 _prec(prec), int(seed) & (2**64 - 1),
                                 int(stream) & (2**64 - 1)), "wd_gaussian_field")


def wd_micro_lds_copy(bytes_, offset, reps, pattern=None, device=0):
    """Global -> LDS copy micro-benchmark; returns (cycles per copy, LDS checksums), numpy arrays."""
    cyc = (C.c_ulonglong * int(reps))()
    sums = (C.c_uint * int(reps))()
    src = None
    if pattern is not None:
        src = np.ascontiguousarray(pattern, dtype=np.uint8)
        if src.nbytes != 1 << 20:
            raise ValueError("pattern must be 1 MiB")
    _check(lib.wd_micro_lds_copy(int(device), int(bytes_), int(offset), int(reps),
                                 None if src is None else src.ctypes.data_as(C.c_void_p), cyc, sums),
           "wd_micro_lds_copy")
    return np.array(cyc[:], dtype=np.uint64), np.array(sums[:], dtype=np.uint32)


def wd_micro_stream(nread, write, nontemporal, bytes_, reps=20, device=0):
    """Streaming probe; returns seconds per pass."""
    t = C.c_double()
    _check(lib.wd_micro_stream(int(device), int(nread), int(write), int(nontemporal), int(bytes_), int(reps),
                               C.byref(t)), "wd_micro_stream")
    return t.value


def wd_micro_resident(bytes_, passes=20, reps=5, device=0):
    """Resident-data probe; returns seconds per pass over `bytes_` bytes."""
    t = C.c_double()
    _check(lib.wd_micro_resident(int(device), int(bytes_), int(passes), int(reps), C.byref(t)), "wd_micro_resident")
    return t.value


def wd_halo_face_bytes(dims, prec):
    return int(lib.wd_halo_face_bytes(_dims(dims), _prec(prec)))


def _slab_bytes(g, nt, prec):
    slot = {WD_F64: 192, WD_F32: 96}.get(_prec(prec), 0)
    L1, L2, L3, _ = g.dims
    return max(int(nt), 0) * (L1 * L2 * L3 // 2) * slot


def wd_halo_pack(g, in_slab, nt, face, dagger, prec, face_buf):
    g.sync_stream()
    _check(lib.wd_halo_pack(g.handle, _buf(in_slab, _slab_bytes(g, nt, prec), "in_slab"), int(nt), int(face),
                            int(dagger), _prec(prec), _buf(face_buf, wd_halo_face_bytes(g.dims, prec), "face_buf")),
           "wd_halo_pack")


def wd_dslash_slab(g, in_slab, face_lo, face_hi, out_slab, a, parity, t0, nt, dagger, prec):
    g.sync_stream()
    sb, fb = _slab_bytes(g, nt, prec), wd_halo_face_bytes(g.dims, prec)
    _check(lib.wd_dslash_slab(g.handle, _buf(in_slab, sb, "in_slab"), _buf(face_lo, fb, "face_lo"),
                              _buf(face_hi, fb, "face_hi"), _buf(out_slab, sb, "out_slab"), float(a),
                              int(parity), int(t0), int(nt), int(dagger), _prec(prec)), "wd_dslash_slab")


def wd_spinor_unpack(g, field, canon, parity=WD_FULL, prec=None):
    g.sync_stream()
    p = g.prec if prec is None else _prec(prec)
    _check(lib.wd_spinor_unpack(g.handle, _buf(field, _need(g.dims, p, 1, parity), "field"),
                                _buf(canon, _canon_bytes(g.dims), "canon"), int(parity), p), "wd_spinor_unpack")


def _hop_fields(g, prec, parity, nrhs=1):
    """(input bytes, output bytes) of a hop of output parity `parity`."""
    if int(parity) in (WD_EVEN, WD_ODD):
        return _need(g.dims, prec, nrhs, 1 - int(parity)), _need(g.dims, prec, nrhs, parity)
    return _need(g.dims, prec, nrhs, parity), _need(g.dims, prec, nrhs, parity)


def wd_dslash(g, psi_in, psi_out, kappa, dims, parity):
    g.sync_stream()
    ni, no = _hop_fields(g, g.prec, parity)
    _check(lib.wd_dslash(g.handle, _buf(psi_in, ni, "psi_in"), _buf(psi_out, no, "psi_out"), float(kappa),
                         _dims(dims), int(parity)), "wd_dslash")


def wd_dslash_ex(g, psi_in, psi_out, kappa, parity, prec, flags=0):
    g.sync_stream()
    ni, no = _hop_fields(g, prec, parity)
    _check(lib.wd_dslash_ex(g.handle, _buf(psi_in, ni, "psi_in"), _buf(psi_out, no, "psi_out"), float(kappa),
                            int(parity), _prec(prec), int(flags)), "wd_dslash_ex")


def wd_dslash_mrhs(g, psi_in, psi_out, kappa, parity, prec, nrhs):
    g.sync_stream()
    ni, no = _hop_fields(g, prec, parity, max(int(nrhs), 1))
    _check(lib.wd_dslash_mrhs(g.handle, _buf(psi_in, ni, "psi_in"), _buf(psi_out, no, "psi_out"), float(kappa),
                              int(parity), _prec(prec), int(nrhs)), "wd_dslash_mrhs")


def _halves(g, prec, nhalf):
    return _need(g.dims, prec, max(int(nhalf), 1), WD_EVEN)


def wd_caxpy(g, c, x, y, nhalf, prec):
    g.sync_stream()
    c = complex(c)
    n = _halves(g, prec, nhalf)
    _check(lib.wd_caxpy(g.handle, c.real, c.imag, _buf(x, n, "x"), _buf(y, n, "y"), int(nhalf), _prec(prec)),
           "wd_caxpy")


def wd_cdot(g, x, y, nhalf, prec):
    g.sync_stream()
    out = (C.c_double * 2)()
    n = _halves(g, prec, nhalf)
    _check(lib.wd_cdot(g.handle, _buf(x, n, "x"), _buf(y, n, "y"), int(nhalf), _prec(prec), out), "wd_cdot")
    return complex(out[0], out[1])


def wd_norm2(g, x, nhalf, prec):
    g.sync_stream()
    out = C.c_double()
    _check(lib.wd_norm2(g.handle, _buf(x, _halves(g, prec, nhalf), "x"), int(nhalf), _prec(prec), C.byref(out)),
           "wd_norm2")
    return out.value


def wd_convert(g, x, pin, y, pout, nhalf, scale=1.0):
    g.sync_stream()
    _check(lib.wd_convert(g.handle, _buf(x, _halves(g, pin, nhalf), "in"), _prec(pin),
                          _buf(y, _halves(g, pout, nhalf), "out"), _prec(pout), int(nhalf), float(scale)),
           "wd_convert")


def wd_solve_params_default(**kw):
    p = wd_solve_params()
    lib.wd_solve_params_default(C.byref(p))
    for k, v in kw.items():
        if k == "inner_prec":
            v = _prec(v)
        if k == "precond":
            v = v.handle if hasattr(v, "handle") else v
        setattr(p, k, v)
    return p


def wd_solve(g, b, x, kappa, tol, params=None):
    """Solve D_W x = b (full FP64 fields).  Returns (status, info dict)."""
    g.sync_stream()
    info = wd_solve_info()
    pp = C.byref(params) if params is not None else None
    n = _need(g.dims, WD_F64, 1, WD_FULL)
    rc = lib.wd_solve(g.handle, _buf(b, n, "b"), _buf(x, n, "x"), float(kappa), float(tol), pp, C.byref(info))
    _check(rc, "wd_solve", allow_not_converged=True)
    return rc, info.as_dict()


def wd_solve_noalloc(g, b, x, kappa, tol, params=None):
    """wd_solve's FP64 CG with its workspace in the library's static device
    array (no device allocation).  Returns (status, info dict)."""
    g.sync_stream()
    info = wd_solve_info()
    pp = C.byref(params) if params is not None else None
    n = _need(g.dims, WD_F64, 1, WD_FULL)
    rc = lib.wd_solve_noalloc(g.handle, _buf(b, n, "b"), _buf(x, n, "x"), float(kappa), float(tol), pp,
                              C.byref(info))
    _check(rc, "wd_solve_noalloc", allow_not_converged=True)
    return rc, info.as_dict()


def wd_solve_mrhs(g, b, x, nrhs, kappa, tol, params):
    g.sync_stream()
    infos = (wd_solve_info * int(nrhs))()
    n = _need(g.dims, WD_F64, max(int(nrhs), 1), WD_FULL)
    rc = lib.wd_solve_mrhs(g.handle, _buf(b, n, "b"), _buf(x, n, "x"), int(nrhs), float(kappa), float(tol),
                           C.byref(params), infos)
    _check(rc, "wd_solve_mrhs", allow_not_converged=True)
    return rc, [i.as_dict() for i in infos]


def wd_tune_dslash(g, prec, cache_path=None, force=False):
    """Autotune the hop variant; returns (block, groups, occ, microseconds per launch)."""
    g.sync_stream()
    b, gr, oc, us = C.c_int(), C.c_int(), C.c_int(), C.c_double()
    cp = cache_path.encode() if cache_path else None
    _check(lib.wd_tune_dslash(g.handle, _prec(prec), cp, int(force), C.byref(b), C.byref(gr), C.byref(oc),
                              C.byref(us)), "wd_tune_dslash")
    return b.value, gr.value, oc.value, us.value


def wd_tune_dirac(g, prec, cache_path=None, force=False):
    """Tune the one-launch D_W (time slices per range, tile shape) or take the
    variant from the JSON-lines cache; returns (slices, tile, microseconds per
    launch)."""
    g.sync_stream()
    sl, ti, us = C.c_int(), C.c_int(), C.c_double()
    cp = cache_path.encode() if cache_path else None
    _check(lib.wd_tune_dirac(g.handle, _prec(prec), cp, int(force), C.byref(sl), C.byref(ti), C.byref(us)),
           "wd_tune_dirac")
    return sl.value, ti.value, us.value


def wd_set_dirac_variant(g, prec, slices, tile):
    _check(lib.wd_set_dirac_variant(g.handle, _prec(prec), int(slices), int(tile)), "wd_set_dirac_variant")


def wd_get_dirac_variant(g, prec):
    sl, ti = C.c_int(), C.c_int()
    _check(lib.wd_get_dirac_variant(g.handle, _prec(prec), C.byref(sl), C.byref(ti)), "wd_get_dirac_variant")
    return sl.value, ti.value


def wd_set_dslash_variant(g, prec, block, groups, occ=0):
    _check(lib.wd_set_dslash_variant(g.handle, _prec(prec), int(block), int(groups), int(occ)),
           "wd_set_dslash_variant")


def wd_get_dslash_variant(g, prec):
    b, gr, oc = C.c_int(), C.c_int(), C.c_int()
    _check(lib.wd_get_dslash_variant(g.handle, _prec(prec), C.byref(b), C.byref(gr), C.byref(oc)),
           "wd_get_dslash_variant")
    return b.value, gr.value, oc.value


def wd_set_dslash_mrhs_variant(g, prec, block, groups, rpl):
    """Multi-RHS hop variant (block, groups, right-hand sides per lane)."""
    _check(lib.wd_set_dslash_mrhs_variant(g.handle, _prec(prec), int(block), int(groups), int(rpl)),
           "wd_set_dslash_mrhs_variant")


def wd_get_dslash_mrhs_variant(g, prec):
    b, gr, rp = C.c_int(), C.c_int(), C.c_int()
    _check(lib.wd_get_dslash_mrhs_variant(g.handle, _prec(prec), C.byref(b), C.byref(gr), C.byref(rp)),
           "wd_get_dslash_mrhs_variant")
    return b.value, gr.value, rp.value


def _fptr(a):
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(C.POINTER(C.c_float))


def ptc_weights_to_flat(W1, W2):
    """Complex weight arrays (9,2,1,4,4) and (9,1,2,4,4) -> the 1152-float layout."""
    w = np.concatenate([np.asarray(W1, np.complex64).ravel(), np.asarray(W2, np.complex64).ravel()])
    return w.view(np.float32).copy()


def ptc_flat_to_weights(flat):
    c = np.asarray(flat, np.float32).view(np.complex64).astype(np.complex128)
    return c[:288].reshape(9, 2, 1, 4, 4), c[288:].reshape(9, 1, 2, 4, 4)


class Ptc:
    """Owning wrapper of a wd_ptc network handle."""

    def __init__(self, g, flat_weights, act_prec="bf16"):
        self.g = g
        a, p = _fptr(flat_weights)
        if a.size != 1152:
            raise ValueError("PTC weights: 1152 floats expected")
        h = C.c_void_p()
        _check(lib.wd_ptc_create(g.handle, p, _prec(act_prec), C.byref(h)), "wd_ptc_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib.wd_ptc_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def wd_ptc_create(g, flat_weights, act_prec="bf16"):
    return Ptc(g, flat_weights, act_prec)


def wd_ptc_destroy(n):
    n.close()


def wd_ptc_set_weights(n, flat):
    a, p = _fptr(flat)
    _check(lib.wd_ptc_set_weights(n.handle, p), "wd_ptc_set_weights")


def wd_ptc_get_weights(n):
    out = np.empty(1152, np.float32)
    _check(lib.wd_ptc_get_weights(n.handle, out.ctypes.data_as(C.POINTER(C.c_float))), "wd_ptc_get_weights")
    return out


def wd_ptc_apply(n, x, y):
    n.g.sync_stream()
    nb = _need(n.g.dims, WD_F32, 1, WD_FULL)
    _check(lib.wd_ptc_apply(n.handle, _buf(x, nb, "in"), _buf(y, nb, "out")), "wd_ptc_apply")


def wd_ptc_apply_even(n, x_even, pin, y_even, pout, flags=0):
    """y_e = [N(x_e, 0)]_e on even half fields (flags: 0, WD_PTC_FP16_PRODUCTS or WD_PTC_BF16_MFMA)."""
    n.g.sync_stream()
    _check(lib.wd_ptc_apply_even(n.handle, _buf(x_even, _need(n.g.dims, pin, 1, WD_EVEN), "in_even"), _prec(pin),
                                 _buf(y_even, _need(n.g.dims, pout, 1, WD_EVEN), "out_even"), _prec(pout),
                                 int(flags)), "wd_ptc_apply_even")


def wd_ptc_loss_grad(n, r, e, B):
    n.g.sync_stream()
    loss = C.c_double()
    grad = np.empty(1152, np.float32)
    nb = _need(n.g.dims, WD_F32, max(int(B), 1), WD_FULL)
    _check(lib.wd_ptc_loss_grad(n.handle, _buf(r, nb, "r"), _buf(e, nb, "e"), int(B), C.byref(loss),
                                grad.ctypes.data_as(C.POINTER(C.c_float))), "wd_ptc_loss_grad")
    return loss.value, grad


def wd_ptc_train_step(n, r, e, B, lr, want_loss=True):
    n.g.sync_stream()
    loss = C.c_double()
    nb = _need(n.g.dims, WD_F32, max(int(B), 1), WD_FULL)
    _check(lib.wd_ptc_train_step(n.handle, _buf(r, nb, "r"), _buf(e, nb, "e"), int(B), float(lr),
                                 C.byref(loss) if want_loss else None), "wd_ptc_train_step")
    return loss.value if want_loss else None


def wd_solve_batch(gauges, bs, xs, kappas, tol, params):
    """Solve D_W[l] x[l] = b[l] for every lattice l together (persistent launches)."""
    n, hs, pb, px, ks = _batch_args(gauges, bs, xs, kappas)
    infos = (wd_solve_info * n)()
    rc = lib.wd_solve_batch(hs, n, pb, px, ks, float(tol), C.byref(params), infos)
    _check(rc, "wd_solve_batch", allow_not_converged=True)
    return rc, [i.as_dict() for i in infos]


def _batch_args(gauges, bs, xs, kappas):
    n = len(gauges)
    for g in gauges:
        g.sync_stream()
    hs = (_vp * n)(*[g.handle for g in gauges])
    nbs = [_need(g.dims, WD_F64, 1, WD_FULL) for g in gauges]
    pb = (_vp * n)(*[_buf(b, k, "b") for b, k in zip(bs, nbs)])
    px = (_vp * n)(*[_buf(x, k, "x") for x, k in zip(xs, nbs)])
    ks = (C.c_double * n)(*[float(k) for k in kappas])
    return n, hs, pb, px, ks


def wd_tune_batch(gauges, bs, xs, kappas, tol, params, cache_path=None, force=False):
    """Tune the batched solve's tile size and persistent blocks per CU (x is
    overwritten); returns (tile, blocks_per_cu, seconds per solve).  Put the
    choice into params.batch_tile / batch_blocks_per_cu to use it."""
    n, hs, pb, px, ks = _batch_args(gauges, bs, xs, kappas)
    t, c, sec = C.c_int(), C.c_int(), C.c_double()
    cp = cache_path.encode() if cache_path else None
    _check(lib.wd_tune_batch(hs, n, pb, px, ks, float(tol), C.byref(params), cp, int(force), C.byref(t), C.byref(c),
                             C.byref(sec)), "wd_tune_batch")
    return t.value, c.value, sec.value


def wd_tune_dslash_mrhs(g, prec, nrhs, cache_path=None, force=False):
    """Tune the multi-RHS hop (block size, tile order, RHS per lane), or take
    the variant from the JSON-lines cache; returns (block, groups, rpl,
    microseconds per launch)."""
    g.sync_stream()
    bs, gr, rp, us = C.c_int(), C.c_int(), C.c_int(), C.c_double()
    cp = cache_path.encode() if cache_path else None
    _check(lib.wd_tune_dslash_mrhs(g.handle, _prec(prec), int(nrhs), cp, int(force), C.byref(bs), C.byref(gr),
                                   C.byref(rp), C.byref(us)), "wd_tune_dslash_mrhs")
    return bs.value, gr.value, rp.value, us.value
