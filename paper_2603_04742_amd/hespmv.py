"""Encrypted sparse matrix-vector multiplication over the CSSC format on MI355X (gfx950).

Thin ctypes binding of ``libhespmv.so`` (C ABI declared in ``include/hespmv.h``).  Every step of
the computation runs in the library's HIP kernels; this module only marshals arguments.  Device
arrays are passed as torch CUDA tensors (torch is used for device memory and streams only).
The library must have been built (``python -m paper_2603_04742_amd.build`` or
``__graft_entry__.build()``); importing the binding without it raises ImportError.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhespmv.so")

HS_OK, HS_EINVAL, HS_EPARAM, HS_ECAPACITY, HS_EKEY, HS_ENOMEM, HS_EDEVICE = 0, -1, -2, -3, -4, -5, -6


class HespmvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("hespmv error %d: %s" % (code, msg))
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("log_n", ctypes.c_uint32), ("n_q", ctypes.c_uint32), ("q_bits", ctypes.c_uint32),
                ("n_p", ctypes.c_uint32), ("p_bits", ctypes.c_uint32), ("t", ctypes.c_uint64),
                ("sigma", ctypes.c_double), ("agg_mode", ctypes.c_uint32), ("slot_rows", ctypes.c_uint32),
                ("relin_mode", ctypes.c_uint32)]


_vp = ctypes.c_void_p
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_int = ctypes.c_int
_pp = ctypes.POINTER(ctypes.c_void_p)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)
_i32p = ctypes.POINTER(ctypes.c_int32)

# name -> (restype, argtypes); the names are those of include/hespmv.h
SIGNATURES = {
    "hs_last_error": (ctypes.c_char_p, []),
    "hs_ctx_create": (_int, [ctypes.POINTER(Params), _pp]),
    "hs_ctx_destroy": (None, [_vp]),
    "hs_ctx_moduli": (_int, [_vp, _u64p, _int, ctypes.POINTER(ctypes.c_int)]),
    "hs_cdt_table": (_int, [_u64p]),
    "hs_keygen": (_int, [_vp, _u64, _vp, _pp]),
    "hs_keyset_destroy": (None, [_vp]),
    "hs_keyset_export": (_int, [_vp, _int, _int, _u64p, _i64]),
    "hs_keyset_add_rotation_keys": (_int, [_vp, _vp, _i64p, _i64, _vp]),
    "hs_keyset_add_right_rotation_keys": (_int, [_vp, _vp, _vp]),
    "hs_matrix_rotation_steps": (_int, [_vp, _i64p, _i64, _i64p]),
    "hs_cssc_pack": (_int, [_vp, _i64, _i64, _vp, _vp, _vp, _int, _vp, _u64, _vp, _pp]),
    "hs_matrix_destroy": (None, [_vp]),
    "hs_matrix_info": (_int, [_vp, _i64p, _i64p]),
    "hs_matrix_chunk": (_int, [_vp, _i64, _i64p]),
    "hs_matrix_column_index": (_int, [_vp, _i32p, _i64, _i64p]),
    "hs_matrix_cssc": (_int, [_vp, _i64, _i32p, _i64, _i64p, _i64, _i64p]),
    "hs_matrix_groups": (_int, [_vp, _i64p]),
    "hs_matrix_export": (_int, [_vp, _int, _i64, _u64p, _i64]),
    "hs_encrypt": (_int, [_vp, _vp, _vp, _vp, _i64, _u64, _vp, _pp]),
    "hs_he_spmv": (_int, [_vp, _vp, _vp, _vp, _vp, _pp]),
    "hs_he_spmv_batch": (_int, [_vp, _int, _pp, _pp, _pp, _vp, _pp]),
    "hs_decrypt": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    "hs_ctvec_count": (_int, [_vp, _i64p]),
    "hs_ct_export": (_int, [_vp, _i64, _u64p, _i64]),
    "hs_ctvec_import": (_int, [_vp, _u64p, _i64, _pp]),
    "hs_ct_export_coeff": (_int, [_vp, _i64, _u64p, _i64, _vp]),
    "hs_ctvec_wrap": (_int, [_vp, _vp, _i64, _pp]),
    "hs_ctx_tensor_widths": (_int, [_vp, _i64p]),
    "hs_he_spmv_noalloc": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    "hs_ctx_set_option": (_int, [_vp, _int, _i64]),
    "hs_ctvec_destroy": (None, [_vp]),
    "hs_ntt": (_int, [_vp, _vp, _i64, _int, _int, _int, _vp]),
    "hs_mul_plain": (_int, [_vp, _vp, _vp, _vp, _pp]),
    "hs_rotate": (_int, [_vp, _vp, _vp, _i64, _vp, _pp]),
    "hs_mul_ct": (_int, [_vp, _vp, _vp, _vp, _vp, _pp]),
    "hs_last_counters": (_int, [_i64p]),
    "hs_profile": (_int, [_int]),
    "hs_set_option": (_int, [_int, _i64]),
    "hs_server_create": (_int, [_vp, _i64, _int, _vp, _pp]),
    "hs_server_submit": (_int, [_vp, _vp, _vp, _vp, _i64p]),
    "hs_server_wait": (_int, [_vp, _i64, _pp, ctypes.POINTER(ctypes.c_double)]),
    "hs_server_stats": (_int, [_vp, _i64p, ctypes.POINTER(ctypes.c_double)]),
    "hs_server_destroy": (None, [_vp]),
    "hs_profile_summary": (_int, [ctypes.c_char_p, _i64, _i64p]),
    "hs_batch_plan_create": (_int, [_vp, _int, _pp, _pp, _pp, _vp, _pp]),
    "hs_batch_plan_run": (_int, [_vp, _vp]),
    "hs_batch_plan_output": (_int, [_vp, _int, _pp]),
    "hs_batch_plan_destroy": (None, [_vp]),
    "hs_ctvec_copy": (_int, [_vp, _vp, _vp]),
    "hs_autotune": (_int, [_vp, _vp, _vp, ctypes.POINTER(ctypes.c_double), _int, ctypes.POINTER(ctypes.c_int)]),
    "hs_tuning": (_int, [_vp, _i64p]),
    "hs_diag_pack": (_int, [_vp, _i64, _i64, _vp, _vp, _vp, _vp, _pp]),
    "hs_diag_destroy": (None, [_vp]),
    "hs_diag_info": (_int, [_vp, _i64p]),
    "hs_diag_keys": (_int, [_vp, _i64p, _i64]),
    "hs_diag_export": (_int, [_vp, _i64, _u64p, _i64]),
    "hs_diag_rotation_steps": (_int, [_vp, _i64p, _i64, _i64p]),
    "hs_diag_encrypt": (_int, [_vp, _vp, _vp, _vp, _i64, _u64, _vp, _pp]),
    "hs_diag_spmv": (_int, [_vp, _vp, _vp, _vp, _vp, _pp]),
    "hs_diag_decrypt": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp]),
    "hs_set_tuning": (_int, [_vp, _i64p]),
}

if not os.path.exists(LIB_PATH):
    raise ImportError("libhespmv.so is not built (%s); run paper_2603_04742_amd/build.py" % LIB_PATH)
lib = ctypes.CDLL(LIB_PATH)
for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args


def _check(rc):
    if rc != HS_OK:
        msg = lib.hs_last_error()
        raise HespmvError(rc, msg.decode() if msg else "")


def _stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dptr(t):
    """Device address of a contiguous torch CUDA tensor (None for an empty tensor)."""
    if t is None or t.numel() == 0:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return ctypes.c_void_p(t.data_ptr())


def _np(a, dt, ptr):
    a = np.ascontiguousarray(a, dt)
    return a, a.ctypes.data_as(ptr)


class Context:
    """hs_ctx: parameter set, primes, tables."""

    def __init__(self, log_n, n_q, q_bits, n_p, t=65537, agg_mode=0, sigma=3.2, slot_rows=1, lazy_relin=0):
        self.params = Params(log_n, n_q, q_bits, n_p, q_bits, t, sigma, agg_mode, slot_rows, int(lazy_relin))
        h = ctypes.c_void_p()
        _check(lib.hs_ctx_create(ctypes.byref(self.params), ctypes.byref(h)))
        self.h = h
        self.N, self.L, self.K, self.t = 1 << log_n, n_q, n_p, t
        self.dnum = (n_q + n_p - 1) // n_p

    def close(self):
        if getattr(self, "h", None) and lib is not None:  # lib is None during interpreter shutdown
            lib.hs_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def moduli(self):
        n = ctypes.c_int()
        buf = np.zeros(256, np.uint64)
        _check(lib.hs_ctx_moduli(self.h, buf.ctypes.data_as(_u64p), 256, ctypes.byref(n)))
        return [int(x) for x in buf[:n.value]]

    def tensor_widths(self):
        """{T, WQ, WM, WD, WMU, WA, KW}: word widths of the exact ciphertext product (zeros without one)."""
        out = np.zeros(7, np.int64)
        _check(lib.hs_ctx_tensor_widths(self.h, out.ctypes.data_as(_i64p)))
        return dict(zip(["T", "WQ", "WM", "WD", "WMU", "WA", "KW"], (int(v) for v in out)))

    def ct_words(self):
        return 2 * self.L * self.N

    def ntt(self, limbs, mod0, n_limbs, inverse=False):
        """In place on a CUDA uint64 tensor [n_polys][n_limbs][N] (torch int64 dtype)."""
        n_polys = limbs.numel() // (n_limbs * self.N)
        _check(lib.hs_ntt(self.h, _dptr(limbs), n_polys, mod0, n_limbs, int(inverse), _stream()))

    def keygen(self, seed):
        return Keyset(self, seed)

    def set_option(self, key, value):
        """hs_ctx_set_option: this context's own setting of an execution option (-1: unset)."""
        _check(lib.hs_ctx_set_option(self.h, key, value))


def cdt_table():
    out = np.zeros(20, np.uint64)
    _check(lib.hs_cdt_table(out.ctypes.data_as(_u64p)))
    return out


class Keyset:
    def __init__(self, ctx, seed):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib.hs_keygen(ctx.h, seed, _stream(), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and lib is not None:  # lib is None during interpreter shutdown
            lib.hs_keyset_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def export(self, which, index=0):
        c = self.ctx
        n = {0: len(c.moduli()) * c.N, 1: 2 * c.L * c.N}.get(which, 2 * c.dnum * (c.L + c.K) * c.N)
        out = np.zeros(n, np.uint64)
        _check(lib.hs_keyset_export(self.h, which, index, out.ctypes.data_as(_u64p), n))
        return out

    def add_rotation_keys(self, steps):
        """hs_keyset_add_rotation_keys: exact-step rotation keys for these steps (host ints)."""
        st = np.ascontiguousarray(np.asarray(steps, np.int64).reshape(-1))
        _check(lib.hs_keyset_add_rotation_keys(self.ctx.h, self.h, st.ctypes.data_as(_i64p), st.size, _stream()))

    def add_right_rotation_keys(self):
        """hs_keyset_add_right_rotation_keys: right rotations by 2^i; rotations then apply the
        signed digits of the non-adjacent form."""
        _check(lib.hs_keyset_add_right_rotation_keys(self.ctx.h, self.h, _stream()))


class CtVec:
    def __init__(self, ctx, h, owner=None):
        # owner: the object that owns a borrowed handle (a BatchPlan); such a vector is not destroyed
        self.ctx, self.h, self.owner = ctx, h, owner

    @classmethod
    def from_host(cls, ctx, limbs, n):
        arr, ptr = _np(limbs, np.uint64, _u64p)
        h = ctypes.c_void_p()
        _check(lib.hs_ctvec_import(ctx.h, ptr, n, ctypes.byref(h)))
        return cls(ctx, h)

    @classmethod
    def wrap(cls, ctx, tensor, n):
        """hs_ctvec_wrap: n ciphertexts held in a caller-owned CUDA tensor (int64 view of the u64
        limbs, [n][2][L][N]), without copying; the tensor must outlive the handle."""
        if tensor.numel() < n * ctx.ct_words():
            raise ValueError("tensor smaller than n ciphertexts")
        h = ctypes.c_void_p()
        _check(lib.hs_ctvec_wrap(ctx.h, _dptr(tensor), n, ctypes.byref(h)))
        v = cls(ctx, h)
        v.backing = tensor
        return v

    def close(self):
        if getattr(self, "h", None) and lib is not None and getattr(self, "owner", None) is None:  # lib: None at shutdown
            lib.hs_ctvec_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()

    def copy_from(self, src):
        """Overwrite this vector's ciphertexts with src's (same count), on the current stream."""
        _check(lib.hs_ctvec_copy(self.h, src.h, _stream()))

    def count(self):
        n = ctypes.c_int64()
        _check(lib.hs_ctvec_count(self.h, ctypes.byref(n)))
        return n.value

    def export(self, i):
        out = np.zeros(self.ctx.ct_words(), np.uint64)
        _check(lib.hs_ct_export(self.h, i, out.ctypes.data_as(_u64p), out.size))
        return out

    def export_all(self):
        return np.concatenate([self.export(i) for i in range(self.count())]) if self.count() else np.zeros(0, np.uint64)

    def export_coeff(self, i):
        """Ciphertext i in coefficient form, residues in [0, q) ([2][L][N])."""
        out = np.zeros(self.ctx.ct_words(), np.uint64)
        _check(lib.hs_ct_export_coeff(self.h, i, out.ctypes.data_as(_u64p), out.size, _stream()))
        return out


class Matrix:
    """Client A: hs_cssc_pack of a CSR matrix given as CUDA tensors (int64 row_ptr, int32 col,
    int64 vals)."""

    def __init__(self, ctx, rows, cols, row_ptr, col, val, encrypt_values=False, keyset=None, seed=0):
        self.ctx, self.R, self.C = ctx, rows, cols
        h = ctypes.c_void_p()
        _check(lib.hs_cssc_pack(ctx.h, rows, cols, _dptr(row_ptr), _dptr(col), _dptr(val), int(encrypt_values),
                                keyset.h if keyset is not None else None, seed, _stream(), ctypes.byref(h)))
        self.h = h
        self.encrypted = bool(encrypt_values)

    def close(self):
        if getattr(self, "h", None) and lib is not None:  # lib is None during interpreter shutdown
            lib.hs_matrix_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def info(self):
        p, c = ctypes.c_int64(), ctypes.c_int64()
        _check(lib.hs_matrix_info(self.h, ctypes.byref(p), ctypes.byref(c)))
        return p.value, c.value

    def groups(self):
        n = ctypes.c_int64()
        _check(lib.hs_matrix_groups(self.h, ctypes.byref(n)))
        return n.value

    def chunk(self, k):
        out = np.zeros(4, np.int64)
        _check(lib.hs_matrix_chunk(self.h, k, out.ctypes.data_as(_i64p)))
        return tuple(int(x) for x in out)

    def rotation_steps(self):
        n = ctypes.c_int64()
        lib.hs_matrix_rotation_steps(self.h, None, 0, ctypes.byref(n))
        out = np.zeros(max(n.value, 1), np.int64)
        _check(lib.hs_matrix_rotation_steps(self.h, out.ctypes.data_as(_i64p), out.size, ctypes.byref(n)))
        return [int(x) for x in out[:n.value]]

    def cssc(self, part):
        """(RM, CP) of row partition `part` (local row indices; CP[0..Lw])."""
        lens = (ctypes.c_int64 * 2)()
        lib.hs_matrix_cssc(self.h, part, None, 0, None, 0, lens)
        rm = np.zeros(max(lens[0], 1), np.int32)
        cp = np.zeros(max(lens[1], 1), np.int64)
        _check(lib.hs_matrix_cssc(self.h, part, rm.ctypes.data_as(_i32p), rm.size, cp.ctypes.data_as(_i64p), cp.size, lens))
        return rm[:lens[0]], cp[:lens[1]]

    def column_index(self):
        n = ctypes.c_int64()
        lib.hs_matrix_column_index(self.h, None, 0, ctypes.byref(n))
        out = np.zeros(max(n.value, 1), np.int32)
        _check(lib.hs_matrix_column_index(self.h, out.ctypes.data_as(_i32p), out.size, ctypes.byref(n)))
        return out[:n.value]

    def export(self, which, k):
        c = self.ctx
        n = c.ct_words() if (which == 0 and self.encrypted) else c.L * c.N
        out = np.zeros(n, np.uint64)
        _check(lib.hs_matrix_export(self.h, which, k, out.ctypes.data_as(_u64p), n))
        return out


class DiagMatrix:
    """The diagonal method (the paper's baseline): hs_diag_pack of a CSR matrix given as CUDA
    tensors (int64 row_ptr, int32 col, int64 vals)."""

    def __init__(self, ctx, rows, cols, row_ptr, col, val):
        self.ctx, self.R, self.C = ctx, rows, cols
        h = ctypes.c_void_p()
        _check(lib.hs_diag_pack(ctx.h, rows, cols, _dptr(row_ptr), _dptr(col), _dptr(val), _stream(), ctypes.byref(h)))
        self.h = h

    def close(self):
        if getattr(self, "h", None) and lib is not None:
            lib.hs_diag_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def info(self):
        """(B, block rows, block columns, diagonals)."""
        out = np.zeros(4, np.int64)
        _check(lib.hs_diag_info(self.h, out.ctypes.data_as(_i64p)))
        return tuple(int(x) for x in out)

    def keys(self):
        n = self.info()[3]
        out = np.zeros(max(3 * n, 1), np.int64)
        _check(lib.hs_diag_keys(self.h, out.ctypes.data_as(_i64p), out.size))
        return out[:3 * n].reshape(n, 3)

    def export(self, k):
        c = self.ctx
        out = np.zeros(c.L * c.N, np.uint64)
        _check(lib.hs_diag_export(self.h, k, out.ctypes.data_as(_u64p), out.size))
        return out

    def rotation_steps(self):
        n = ctypes.c_int64()
        lib.hs_diag_rotation_steps(self.h, None, 0, ctypes.byref(n))
        out = np.zeros(max(n.value, 1), np.int64)
        _check(lib.hs_diag_rotation_steps(self.h, out.ctypes.data_as(_i64p), out.size, ctypes.byref(n)))
        return [int(x) for x in out[:n.value]]


def diag_encrypt(ctx, ks, d, v, seed):
    """Client B of the diagonal method: one ciphertext per block column (CUDA int64 vector v)."""
    h = ctypes.c_void_p()
    _check(lib.hs_diag_encrypt(ctx.h, ks.h, d.h, _dptr(v), v.numel(), seed, _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


def diag_spmv(ctx, ks, d, x):
    h = ctypes.c_void_p()
    _check(lib.hs_diag_spmv(ctx.h, ks.h, d.h, x.h, _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


def diag_decrypt(ctx, ks, d, y, out):
    _check(lib.hs_diag_decrypt(ctx.h, ks.h, d.h, y.h, _dptr(out), d.R, _stream()))
    return out


def encrypt(ctx, ks, m, v, seed):
    """Client B: reorganise, encode and encrypt the CUDA int64 vector v."""
    h = ctypes.c_void_p()
    _check(lib.hs_encrypt(ctx.h, ks.h, m.h, _dptr(v), v.numel(), seed, _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


def he_spmv(ctx, ks, m, x):
    h = ctypes.c_void_p()
    _check(lib.hs_he_spmv(ctx.h, ks.h, m.h, x.h, _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


def he_spmv_noalloc(ctx, ks, m, x, y):
    """hs_he_spmv_noalloc: the result written into the caller's CUDA tensor y (int64 view of the
    u64 limbs, at least m.groups() ciphertexts), intermediates in the library's fixed scratch
    array; returns y wrapped as a vector handle (no copy)."""
    _check(lib.hs_he_spmv_noalloc(ctx.h, ks.h, m.h, x.h, _dptr(y), y.numel(), _stream()))
    return CtVec.wrap(ctx, y, m.groups())


def he_spmv_batch(ctx, kss, ms, xs):
    """n independent encrypted SpMVs in one call (rotations merged into shared batched launches)."""
    n = len(ms)
    arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[h.h for h in hs])
    ys = (ctypes.c_void_p * max(n, 1))()
    _check(lib.hs_he_spmv_batch(ctx.h, n, arr(kss), arr(ms), arr(xs), _stream(), ys))
    return [CtVec(ctx, ctypes.c_void_p(ys[i])) for i in range(n)]


def autotune(ctx, ks):
    """Time the launch variants on this context and keep the faster ones; returns the report:
    {"variant": v, "variant_ms": [v0, v1], "ntt_variant": v, "ntt_variant_ms": [v0, v1],
     "pipelines": [(B, ms one-workgroup, ms two-pass), ...]}."""
    buf = (ctypes.c_double * 64)()
    n = ctypes.c_int()
    _check(lib.hs_autotune(ctx.h, ks.h, _stream(), buf, 64, ctypes.byref(n)))
    r = list(buf[:n.value])
    return {"variant": int(r[0]), "variant_ms": r[1:3], "ntt_variant": int(r[3]), "ntt_variant_ms": r[4:6],
            "pipelines": [(int(r[6 + 3 * i]), r[7 + 3 * i], r[8 + 3 * i]) for i in range((len(r) - 6) // 3)]}


def tuning(ctx):
    """[key-switch transform variant, plain transform variant, pipeline pick per batch bucket x 8]."""
    out = (ctypes.c_int64 * 10)()
    _check(lib.hs_tuning(ctx.h, out))
    return list(out)


def set_tuning(ctx, table):
    arr = (ctypes.c_int64 * 10)(*[int(v) for v in table])
    _check(lib.hs_set_tuning(ctx.h, arr))


class BatchPlan:
    """hs_he_spmv_batch recorded as a HIP graph: built (and run once) at construction, replayed by
    run() on the current stream.  outputs() are borrowed from the plan."""

    def __init__(self, ctx, kss, ms, xs):
        self.ctx, self._refs = ctx, (list(kss), list(ms), list(xs))
        n = len(ms)
        arr = lambda hs: (ctypes.c_void_p * max(n, 1))(*[h.h for h in hs])
        h = ctypes.c_void_p()
        _check(lib.hs_batch_plan_create(ctx.h, n, arr(kss), arr(ms), arr(xs), _stream(), ctypes.byref(h)))
        self.h, self.n = h, n

    def run(self):
        _check(lib.hs_batch_plan_run(self.h, _stream()))

    def outputs(self):
        out = []
        for i in range(self.n):
            y = ctypes.c_void_p()
            _check(lib.hs_batch_plan_output(self.h, i, ctypes.byref(y)))
            out.append(CtVec(self.ctx, y, owner=self))
        return out

    def close(self):
        if getattr(self, "h", None) and lib is not None:
            lib.hs_batch_plan_destroy(self.h)
        self.h = None

    def __del__(self):
        self.close()


def decrypt(ctx, ks, m, y, out):
    """Key holder: decrypt into the CUDA int64 tensor out[rows]."""
    _check(lib.hs_decrypt(ctx.h, ks.h, m.h, y.h, _dptr(out), m.R, _stream()))
    return out


def mul_plain(ctx, x, pt):
    h = ctypes.c_void_p()
    _check(lib.hs_mul_plain(ctx.h, x.h, _dptr(pt), _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


def rotate(ctx, ks, x, k):
    h = ctypes.c_void_p()
    _check(lib.hs_rotate(ctx.h, ks.h, x.h, k, _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


OPT_KS_PIPELINE, OPT_NTT_PATH, OPT_KS_THRESHOLD, OPT_AUX_PATH, OPT_MODUP_GROUP, OPT_NTT_PIPE, OPT_KS_BLOCK, OPT_MODUP_ACC, \
    OPT_KS_FUSE = 1, 2, 3, 4, 5, 6, 7, 8, 9


def set_option(key, value):
    _check(lib.hs_set_option(key, value))


def profile(enable):
    """Start (clearing earlier records) or stop HIP-event timing of every kernel launch."""
    _check(lib.hs_profile(int(bool(enable))))


def profile_summary(units=False):
    """{kernel name: (launches, total ms)} of the launches recorded since profile(True); with
    units=True also the work those launches processed (key switches for the key-switch kernels,
    limbs for k_ntt15): (launches, total ms, units)."""
    n = ctypes.c_int64()
    lib.hs_profile_summary(None, 0, ctypes.byref(n))
    buf = ctypes.create_string_buffer(n.value + 1)
    _check(lib.hs_profile_summary(buf, n.value + 1, ctypes.byref(n)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms, u = line.split()
        out[name] = (int(cnt), float(ms), int(u)) if units else (int(cnt), float(ms))
    return out


def mul_ct(ctx, ks, a, b):
    """Slot-wise product of two ciphertext vectors (exact scaled tensor + relinearisation)."""
    h = ctypes.c_void_p()
    _check(lib.hs_mul_ct(ctx.h, ks.h, a.h, b.h, _stream(), ctypes.byref(h)))
    return CtVec(ctx, h)


class Server:
    """Continuous-batching server (hs_server_*): submit() queues a request, wait() returns its
    result and (submit, admit, done) times."""

    def __init__(self, ctx, hbm_budget_bytes=64 << 30, max_active=256):
        self.ctx = ctx
        h = ctypes.c_void_p()
        _check(lib.hs_server_create(ctx.h, hbm_budget_bytes, max_active, _stream(), ctypes.byref(h)))
        self.h = h
        self._keep = {}

    def submit(self, ks, m, x):
        rid = ctypes.c_int64()
        _check(lib.hs_server_submit(self.h, ks.h, m.h, x.h, ctypes.byref(rid)))
        self._keep[rid.value] = (ks, m, x)
        return rid.value

    def wait(self, rid):
        y = ctypes.c_void_p()
        t = (ctypes.c_double * 3)()
        try:
            _check(lib.hs_server_wait(self.h, rid, ctypes.byref(y), t))
        finally:
            self._keep.pop(rid, None)
        return CtVec(self.ctx, y), (t[0], t[1], t[2])

    def stats(self):
        out = np.zeros(8, np.int64)
        now = ctypes.c_double()
        _check(lib.hs_server_stats(self.h, out.ctypes.data_as(_i64p), ctypes.byref(now)))
        return dict(zip(["ticks", "max_active", "admitted", "completed", "bytes_in_use", "held_by_budget", "held_by_slots",
                         "requests_waited"], (int(v) for v in out)), now=now.value)

    def close(self):
        if getattr(self, "h", None) and lib is not None:  # lib is None during interpreter shutdown
            lib.hs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()


def last_counters():
    out = np.zeros(5, np.int64)
    _check(lib.hs_last_counters(out.ctypes.data_as(_i64p)))
    return dict(zip(["key_switches", "rotations", "launches", "products", "mask_products"], (int(x) for x in out)))
