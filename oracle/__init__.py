"""CPU oracle for encrypted SpMV over CSSC -- TEST INFRASTRUCTURE ONLY.

ctypes binding of ``oracle/liboracle.so`` (built from ``oracle/oracle.cpp`` with g++).  Only the
tests, ``__graft_entry__.smoke()`` and the benchmark's ``cpu_baseline`` leg may import this
module.  It shares no code with the GPU library (``paper_2603_04742_amd``).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.cpp")

u64p = ctypes.POINTER(ctypes.c_uint64)
i64p = ctypes.POINTER(ctypes.c_int64)
i32p = ctypes.POINTER(ctypes.c_int32)
u32p = ctypes.POINTER(ctypes.c_uint32)
vp = ctypes.c_void_p


def build(force=False):
    """Compile the oracle (plain g++, -O2, no OpenMP; no GPU code)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", _SO, _SRC])
    return _SO


def build_native(out_dir):
    """Compile the same source with -O3 -march=native -fopenmp into out_dir (for timing the oracle
    on the machine that runs it: the instruction set is that host's, so the library is built
    there, never shipped).  Returns the library path."""
    so = os.path.join(out_dir, "liboracle_native.so")
    subprocess.check_call(["g++", "-O3", "-march=native", "-fopenmp", "-std=c++17", "-shared", "-fPIC", "-o", so, _SRC])
    return so


_lib = None
_lib_path = None


def use_library(path):
    """Load the oracle from `path` (e.g. build_native's output) instead of the plain build; only
    before the first call into the oracle in this process."""
    global _lib_path
    if _lib is not None and path != (_lib_path or _SO):
        raise RuntimeError("the oracle library is already loaded in this process")
    _lib_path = path


def set_threads(n):
    """Threads of the OpenMP build (the plain build always runs one); returns the count in effect."""
    return lib().orc_set_threads(n)


def lib():
    global _lib
    if _lib is None:
        if _lib_path is None:
            build()
        L = ctypes.CDLL(_lib_path or _SO)
        sig = {
            "orc_set_threads": (ctypes.c_int, [ctypes.c_int]),
            "orc_ctx_new": (vp, [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                 ctypes.c_int]),
            "orc_ctx_free": (None, [vp]),
            "orc_n_moduli": (ctypes.c_int, [vp]),
            "orc_n_aux": (ctypes.c_int, [vp]),
            "orc_moduli": (None, [vp, u64p]),
            "orc_psi": (ctypes.c_uint64, [vp, ctypes.c_int]),
            "orc_slot_pos": (None, [vp, u32p]),
            "orc_is_prime": (ctypes.c_int, [ctypes.c_uint64]),
            "orc_mulmod": (ctypes.c_uint64, [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint64]),
            "orc_chacha20_block": (None, [u32p, ctypes.c_uint32, u32p, u32p]),
            "orc_cdt": (None, [u64p]),
            "orc_sample": (None, [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, ctypes.c_uint64, i64p]),
            "orc_ntt": (None, [vp, ctypes.c_int, u64p]),
            "orc_intt": (None, [vp, ctypes.c_int, u64p]),
            "orc_encode": (None, [vp, u64p, u64p]),
            "orc_decode": (None, [vp, u64p, u64p]),
            "orc_plain_ntt": (None, [vp, u64p, u64p]),
            "orc_galois_elt": (ctypes.c_uint64, [vp, ctypes.c_int]),
            "orc_rotation_digits": (ctypes.c_int, [vp, ctypes.c_uint64, i64p]),
            "orc_add_right_keys": (None, [vp]),
            "orc_n_rotation_keys": (ctypes.c_int, [vp]),
            "orc_keygen": (None, [vp, ctypes.c_uint64]),
            "orc_export_sk": (None, [vp, i64p]),
            "orc_export_sk_ntt": (None, [vp, u64p]),
            "orc_export_pk": (None, [vp, u64p]),
            "orc_export_ksk": (None, [vp, ctypes.c_int, u64p]),
            "orc_encrypt": (None, [vp, u64p, ctypes.c_uint64, ctypes.c_uint64, u64p]),
            "orc_decrypt": (None, [vp, u64p, u64p]),
            "orc_noise_log2": (ctypes.c_double, [vp, u64p, u64p]),
            "orc_ct_mul_plain": (None, [vp, u64p, u64p, u64p]),
            "orc_ct_mul_ct": (ctypes.c_int, [vp, u64p, u64p, u64p]),
            "orc_ct_tensor": (ctypes.c_int, [vp, u64p, u64p, u64p]),
            "orc_has_tensor": (ctypes.c_int, [vp]),
            "orc_keyswitch": (None, [vp, u64p, ctypes.c_int, u64p]),
            "orc_automorph_ntt": (None, [vp, u64p, ctypes.c_uint64, u64p]),
            "orc_rotate": (None, [vp, u64p, ctypes.c_uint64, u64p]),
            "orc_add_step_keys": (None, [vp, i64p, ctypes.c_int64]),
            "orc_export_step_key": (ctypes.c_int, [vp, ctypes.c_uint64, u64p]),
            "orc_total_sum_steps": (ctypes.c_int, [vp, ctypes.c_int64, ctypes.c_int64, u64p]),
            "orc_total_sum": (None, [vp, u64p, ctypes.c_int64, ctypes.c_int64, u64p]),
            "orc_cssc_lw": (ctypes.c_int, [ctypes.c_int64, i64p]),
            "orc_cssc": (None, [ctypes.c_int64, i64p, i32p, i64p, i64p, i32p, i32p, i64p]),
            "orc_chunks": (ctypes.c_int, [ctypes.c_int, i64p, ctypes.c_int64, ctypes.c_int, i64p]),
            "orc_matrix_new": (vp, [vp, ctypes.c_int64, ctypes.c_int64, i64p, i32p, i64p, ctypes.c_int, ctypes.c_uint64]),
            "orc_matrix_free": (None, [vp]),
            "orc_matrix_n_parts": (ctypes.c_int, [vp]),
            "orc_matrix_n_groups": (ctypes.c_int, [vp]),
            "orc_matrix_n_chunks": (ctypes.c_int, [vp]),
            "orc_matrix_chunk": (None, [vp, ctypes.c_int, i64p]),
            "orc_matrix_pt": (None, [vp, ctypes.c_int, u64p]),
            "orc_matrix_mask": (None, [vp, ctypes.c_int, u64p]),
            "orc_encrypt_vector": (None, [vp, vp, i64p, ctypes.c_uint64, u64p]),
            "orc_he_spmv": (None, [vp, vp, u64p, u64p, i64p]),
            "orc_decrypt_result": (None, [vp, vp, u64p, i64p]),
            "orc_diag_new": (vp, [vp, ctypes.c_int64, ctypes.c_int64, i64p, i32p, i64p]),
            "orc_diag_free": (None, [vp]),
            "orc_diag_count": (ctypes.c_int, [vp]),
            "orc_diag_info": (None, [vp, i64p]),
            "orc_diag_key": (None, [vp, ctypes.c_int, i64p]),
            "orc_diag_pt": (None, [vp, ctypes.c_int, u64p]),
            "orc_diag_encrypt_vector": (None, [vp, vp, i64p, ctypes.c_uint64, u64p]),
            "orc_diag_spmv": (None, [vp, vp, u64p, u64p, i64p]),
            "orc_diag_decrypt": (None, [vp, vp, u64p, i64p]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a, t):
    return a.ctypes.data_as(t)


def cdt():
    out = np.zeros(20, np.uint64)
    lib().orc_cdt(_p(out, u64p))
    return out


def chacha20_block(key_words, counter, nonce_words):
    k = np.ascontiguousarray(key_words, np.uint32)
    n = np.ascontiguousarray(nonce_words, np.uint32)
    out = np.zeros(16, np.uint32)
    lib().orc_chacha20_block(_p(k, u32p), counter, _p(n, u32p), _p(out, u32p))
    return out


def sample(seed, purpose, index, n, kind, q=0):
    """kind 0 = ternary, 1 = Gaussian, 2 = uniform mod q."""
    out = np.zeros(n, np.int64)
    lib().orc_sample(seed, purpose, index, n, kind, q, _p(out, i64p))
    return out


def is_prime(n):
    return bool(lib().orc_is_prime(n))


def cssc(R, row_ptr, col, val):
    row_ptr = np.ascontiguousarray(row_ptr, np.int64)
    col = np.ascontiguousarray(col, np.int32)
    val = np.ascontiguousarray(val, np.int64)
    Lw = lib().orc_cssc_lw(R, _p(row_ptr, i64p))
    nnz = int(row_ptr[R])
    VA = np.zeros(max(nnz, 1), np.int64)
    CI = np.zeros(max(nnz, 1), np.int32)
    RM = np.zeros(max(R, 1), np.int32)
    CP = np.zeros(Lw + 1, np.int64)
    lib().orc_cssc(R, _p(row_ptr, i64p), _p(col, i32p), _p(val, i64p), _p(VA, i64p), _p(CI, i32p), _p(RM, i32p), _p(CP, i64p))
    return VA[:nnz], CI[:nnz], RM[:R], CP


def chunks(CP, s, uniform=False):
    CP = np.ascontiguousarray(CP, np.int64)
    Lw = len(CP) - 1
    out = np.zeros(3 * max(Lw, 1), np.int64)
    n = lib().orc_chunks(Lw, _p(CP, i64p), s, int(uniform), _p(out, i64p))
    return [tuple(int(x) for x in out[3 * i:3 * i + 3]) for i in range(n)]


class Context:
    """Scheme parameters + keys (single key-set)."""

    def __init__(self, logn, L, qbits, K, pbits=None, t=65537, agg_mode=0, slot_rows=1, lazy_relin=0):
        self.logn, self.N, self.L, self.K, self.t = logn, 1 << logn, L, K, t
        self.slot_rows, self.lazy_relin = slot_rows, lazy_relin
        self._free = lib().orc_ctx_free
        self.h = lib().orc_ctx_new(logn, L, qbits, K, pbits or qbits, t, agg_mode, slot_rows, int(lazy_relin))
        if not self.h:
            raise ValueError("oracle: unsupported parameters")
        self.agg_mode = agg_mode
        self.dnum = (L + K - 1) // K

    def __del__(self):
        # the free function is looked up while the module is alive (not at interpreter shutdown)
        free = getattr(self, "_free", None)
        if getattr(self, "h", None) and free is not None:
            free(self.h)
            self.h = None

    # --- parameters
    def moduli(self):
        out = np.zeros(lib().orc_n_moduli(self.h), np.uint64)
        lib().orc_moduli(self.h, _p(out, u64p))
        return [int(x) for x in out]

    def n_aux(self):
        return lib().orc_n_aux(self.h)

    def psi(self, m):
        return int(lib().orc_psi(self.h, m))

    def slot_pos(self):
        out = np.zeros(self.N, np.uint32)
        lib().orc_slot_pos(self.h, _p(out, u32p))
        return out

    def galois_elt(self, i):
        """Galois element of rotation key index i: left by 2^i for i < log2 N - 1, else right
        by 2^(i - log2 N + 1)."""
        return int(lib().orc_galois_elt(self.h, i))

    def add_right_rotation_keys(self):
        """The optional right rotation keys (index log2 N - 1 + i rotates right by 2^i); rotations
        then apply the signed digits of the non-adjacent form."""
        lib().orc_add_right_keys(self.h)

    def rotation_digits(self, k):
        """Power-of-two steps (lowest first) that a rotation by k mod N/2 applies when no
        exact-step key is held: the binary digits of k, or with the right keys the signed digits
        +-2^i of the non-adjacent form of k without a digit of N/2."""
        out = np.zeros(64, np.int64)
        n = lib().orc_rotation_digits(self.h, k % (self.N // 2), _p(out, i64p))
        return [int(v) for v in out[:n]]

    # --- transforms
    def ntt(self, m, a):
        a = np.array(a, np.uint64)
        lib().orc_ntt(self.h, m, _p(a, u64p))
        return a

    def intt(self, m, a):
        a = np.array(a, np.uint64)
        lib().orc_intt(self.h, m, _p(a, u64p))
        return a

    def encode(self, slots):
        s = np.ascontiguousarray(np.asarray(slots, np.int64) % self.t, np.uint64)
        out = np.zeros(self.N, np.uint64)
        lib().orc_encode(self.h, _p(s, u64p), _p(out, u64p))
        return out

    def decode(self, m):
        m = np.ascontiguousarray(m, np.uint64)
        out = np.zeros(self.N, np.uint64)
        lib().orc_decode(self.h, _p(m, u64p), _p(out, u64p))
        return out

    def plain_ntt(self, m):
        m = np.ascontiguousarray(m, np.uint64)
        out = np.zeros(self.L * self.N, np.uint64)
        lib().orc_plain_ntt(self.h, _p(m, u64p), _p(out, u64p))
        return out

    # --- keys
    def keygen(self, seed):
        lib().orc_keygen(self.h, seed)

    def sk(self):
        out = np.zeros(self.N, np.int64)
        lib().orc_export_sk(self.h, _p(out, i64p))
        return out

    def sk_ntt(self):
        out = np.zeros(len(self.moduli()) * self.N, np.uint64)
        lib().orc_export_sk_ntt(self.h, _p(out, u64p))
        return out

    def pk(self):
        out = np.zeros(2 * self.L * self.N, np.uint64)
        lib().orc_export_pk(self.h, _p(out, u64p))
        return out

    def ksk(self, key_id):
        """Key-switching key: key_id < 0 the relinearisation key, else rotation key index key_id
        (left by 2^key_id below log2 N - 1, else right by 2^(key_id - log2 N + 1))."""
        if key_id >= lib().orc_n_rotation_keys(self.h):
            raise IndexError("no rotation key with index %d" % key_id)
        out = np.zeros(2 * self.dnum * (self.L + self.K) * self.N, np.uint64)
        lib().orc_export_ksk(self.h, key_id, _p(out, u64p))
        return out

    def add_step_keys(self, steps):
        """Rotation keys for left rotations by exactly these steps (mod N/2); powers of two and
        steps already held are skipped."""
        st = np.ascontiguousarray(np.asarray(steps, np.int64).reshape(-1))
        lib().orc_add_step_keys(self.h, _p(st, i64p), len(st))

    def step_key(self, k):
        out = np.zeros(2 * self.dnum * (self.L + self.K) * self.N, np.uint64)
        return out if lib().orc_export_step_key(self.h, k, _p(out, u64p)) else None

    def total_sum_steps(self, r, c):
        out = np.zeros(128, np.uint64)
        n = lib().orc_total_sum_steps(self.h, r, c, _p(out, u64p))
        return [int(x) for x in out[:n]]

    # --- HE ops (ciphertexts: flat uint64 [2][L][N], NTT form)
    def ct_size(self):
        return 2 * self.L * self.N

    def encrypt(self, m, seed, idx=0):
        m = np.ascontiguousarray(m, np.uint64)
        out = np.zeros(self.ct_size(), np.uint64)
        lib().orc_encrypt(self.h, _p(m, u64p), seed, idx, _p(out, u64p))
        return out

    def decrypt(self, ct):
        ct = np.ascontiguousarray(ct, np.uint64)
        out = np.zeros(self.N, np.uint64)
        lib().orc_decrypt(self.h, _p(ct, u64p), _p(out, u64p))
        return out

    def noise_log2(self, ct, m):
        ct = np.ascontiguousarray(ct, np.uint64)
        m = np.ascontiguousarray(m, np.uint64)
        return lib().orc_noise_log2(self.h, _p(ct, u64p), _p(m, u64p))

    def ct_mul_plain(self, ct, pt_ntt):
        ct = np.ascontiguousarray(ct, np.uint64)
        pt = np.ascontiguousarray(pt_ntt, np.uint64)
        out = np.zeros(self.ct_size(), np.uint64)
        lib().orc_ct_mul_plain(self.h, _p(ct, u64p), _p(pt, u64p), _p(out, u64p))
        return out

    def ct_mul_ct(self, a, b):
        a = np.ascontiguousarray(a, np.uint64)
        b = np.ascontiguousarray(b, np.uint64)
        out = np.zeros(self.ct_size(), np.uint64)
        if lib().orc_ct_mul_ct(self.h, _p(a, u64p), _p(b, u64p), _p(out, u64p)) != 0:
            raise ValueError("oracle: the primes of this ring cannot hold the exact ciphertext product")
        return out

    def ct_tensor(self, a, b):
        """The exact three-component product (d0, d1, d2) before relinearisation, [3][L][N] NTT form."""
        a = np.ascontiguousarray(a, np.uint64)
        b = np.ascontiguousarray(b, np.uint64)
        out = np.zeros(3 * self.L * self.N, np.uint64)
        if lib().orc_ct_tensor(self.h, _p(a, u64p), _p(b, u64p), _p(out, u64p)) != 0:
            raise ValueError("oracle: the primes of this ring cannot hold the exact ciphertext product")
        return out

    def has_tensor(self):
        return bool(lib().orc_has_tensor(self.h))

    def keyswitch(self, d, key_id):
        """Key switch of d ([L][N], NTT form) with the relinearisation key (key_id < 0) or rotation
        key index key_id (as ksk)."""
        if key_id >= lib().orc_n_rotation_keys(self.h):
            raise IndexError("no rotation key with index %d" % key_id)
        d = np.ascontiguousarray(d, np.uint64)
        out = np.zeros(self.ct_size(), np.uint64)
        lib().orc_keyswitch(self.h, _p(d, u64p), key_id, _p(out, u64p))
        return out

    def automorph_ntt(self, a, g):
        a = np.ascontiguousarray(a, np.uint64)
        out = np.zeros(self.L * self.N, np.uint64)
        lib().orc_automorph_ntt(self.h, _p(a, u64p), g, _p(out, u64p))
        return out

    def rotate(self, ct, k):
        ct = np.ascontiguousarray(ct, np.uint64)
        out = np.zeros(self.ct_size(), np.uint64)
        lib().orc_rotate(self.h, _p(ct, u64p), k, _p(out, u64p))
        return out

    def total_sum(self, ct, r, c):
        ct = np.ascontiguousarray(ct, np.uint64)
        out = np.zeros(self.ct_size(), np.uint64)
        lib().orc_total_sum(self.h, _p(ct, u64p), r, c, _p(out, u64p))
        return out


class Matrix:
    """Client A's packed matrix (plaintext or encrypted values) for one Context."""

    def __init__(self, ctx, R, C, row_ptr, col, val, encrypted=False, mat_seed=0):
        self.ctx, self.R, self.C = ctx, R, C
        self.row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        self.col = np.ascontiguousarray(col, np.int32)
        self.val = np.ascontiguousarray(val, np.int64)
        self._free = lib().orc_matrix_free
        self.h = lib().orc_matrix_new(ctx.h, R, C, _p(self.row_ptr, i64p), _p(self.col, i32p), _p(self.val, i64p), int(encrypted), mat_seed)
        if not self.h:
            raise ValueError("oracle: encrypted matrix values need the exact ciphertext product, which this ring cannot hold")

    def __del__(self):
        # the free function is looked up while the module is alive (not at interpreter shutdown)
        free = getattr(self, "_free", None)
        if getattr(self, "h", None) and free is not None:
            free(self.h)
            self.h = None

    def n_parts(self):
        return lib().orc_matrix_n_parts(self.h)

    def n_chunks(self):
        return lib().orc_matrix_n_chunks(self.h)

    def n_groups(self):
        """Result ciphertexts: one per row partition, or per pair of partitions (two slot rows)."""
        return lib().orc_matrix_n_groups(self.h)

    def chunk(self, k):
        out = np.zeros(4, np.int64)
        lib().orc_matrix_chunk(self.h, k, _p(out, i64p))
        return tuple(int(x) for x in out)

    def pt(self, k, encrypted=False):
        n = self.ctx.ct_size() if encrypted else self.ctx.L * self.ctx.N
        out = np.zeros(n, np.uint64)
        lib().orc_matrix_pt(self.h, k, _p(out, u64p))
        return out

    def mask(self, k):
        out = np.zeros(self.ctx.L * self.ctx.N, np.uint64)
        lib().orc_matrix_mask(self.h, k, _p(out, u64p))
        return out

    def encrypt_vector(self, v, seed):
        v = np.ascontiguousarray(v, np.int64)
        out = np.zeros(self.n_chunks() * self.ctx.ct_size(), np.uint64)
        lib().orc_encrypt_vector(self.ctx.h, self.h, _p(v, i64p), seed, _p(out, u64p))
        return out

    def he_spmv(self, x):
        x = np.ascontiguousarray(x, np.uint64)
        out = np.zeros(self.n_groups() * self.ctx.ct_size(), np.uint64)
        stats = np.zeros(2, np.int64)
        lib().orc_he_spmv(self.ctx.h, self.h, _p(x, u64p), _p(out, u64p), _p(stats, i64p))
        return out, {"key_switches": int(stats[0]), "rotations": int(stats[1])}

    def decrypt_result(self, res):
        res = np.ascontiguousarray(res, np.uint64)
        y = np.zeros(self.R, np.int64)
        lib().orc_decrypt_result(self.ctx.h, self.h, _p(res, u64p), _p(y, i64p))
        return y


class DiagMatrix:
    """The paper's diagonal baseline: generalised diagonals of B x B blocks as plaintexts."""

    def __init__(self, ctx, R, C, row_ptr, col, val):
        self.ctx, self.R, self.C = ctx, R, C
        self.row_ptr = np.ascontiguousarray(row_ptr, np.int64)
        self.col = np.ascontiguousarray(col, np.int32)
        self.val = np.ascontiguousarray(val, np.int64)
        self._free = lib().orc_diag_free
        self.h = lib().orc_diag_new(ctx.h, R, C, _p(self.row_ptr, i64p), _p(self.col, i32p), _p(self.val, i64p))

    def __del__(self):
        # the free function is looked up while the module is alive (not at interpreter shutdown)
        free = getattr(self, "_free", None)
        if getattr(self, "h", None) and free is not None:
            free(self.h)
            self.h = None

    def info(self):
        out = np.zeros(5, np.int64)
        lib().orc_diag_info(self.h, _p(out, i64p))
        return dict(B=int(out[0]), row_blocks=int(out[1]), col_blocks=int(out[2]), diagonals=int(out[3]))

    def key(self, k):
        out = np.zeros(3, np.int64)
        lib().orc_diag_key(self.h, k, _p(out, i64p))
        return tuple(int(x) for x in out)

    def pt(self, k):
        out = np.zeros(self.ctx.L * self.ctx.N, np.uint64)
        lib().orc_diag_pt(self.h, k, _p(out, u64p))
        return out

    def encrypt_vector(self, v, seed):
        v = np.ascontiguousarray(v, np.int64)
        out = np.zeros(self.info()["col_blocks"] * self.ctx.ct_size(), np.uint64)
        lib().orc_diag_encrypt_vector(self.ctx.h, self.h, _p(v, i64p), seed, _p(out, u64p))
        return out

    def spmv(self, x):
        x = np.ascontiguousarray(x, np.uint64)
        out = np.zeros(self.info()["row_blocks"] * self.ctx.ct_size(), np.uint64)
        stats = np.zeros(1, np.int64)
        lib().orc_diag_spmv(self.ctx.h, self.h, _p(x, u64p), _p(out, u64p), _p(stats, i64p))
        return out

    def decrypt_result(self, res):
        res = np.ascontiguousarray(res, np.uint64)
        y = np.zeros(self.R, np.int64)
        lib().orc_diag_decrypt(self.ctx.h, self.h, _p(res, u64p), _p(y, i64p))
        return y
