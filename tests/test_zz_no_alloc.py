"""The allocation-free encrypted SpMV (hs_he_spmv_noalloc) against hs_he_spmv, through the C ABI:
two calls in a row on one context, the second with a smaller matrix, each bit for bit equal to
the allocating entry point's result and decrypting to the integer SpMV; an encrypted-matrix
SpMV (exact ciphertext products, eager and lazy relinearisation); the error paths (short output,
intermediates beyond the fixed array)."""
import numpy as np
import pytest

from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402


def dev(a, dtype):
    npd = {torch.int64: np.int64, torch.int32: np.int32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(npd))).cuda()


def matrix(g, kg, w, encrypted=False, seed=0):
    return H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64),
                    encrypted, kg if encrypted else None, seed)


def check_against_he_spmv(g, kg, w, encrypted=False, poison=None):
    """One SpMV through both entry points; the no-alloc result lands in a fresh tensor filled with
    `poison` first (so nothing of it may be left over)."""
    M = matrix(g, kg, w, encrypted, 31)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    want = H.he_spmv(g, kg, M, x).export_all()
    y = torch.full((M.groups() * g.ct_words(),), -1 if poison is None else poison, dtype=torch.int64, device="cuda")
    print("no-alloc SpMV %d x %d, %d chunks, %d groups" % (w["R"], w["C"], M.info()[1], M.groups()), flush=True)
    yv = H.he_spmv_noalloc(g, kg, M, x, y)
    got = yv.export_all()
    assert got.shape == want.shape and np.array_equal(got, want)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, yv, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))
    return M


def test_noalloc_two_calls_second_smaller():
    """zipf16k at full size (16384 x 16384, N = 16384, 6 + 1 primes, masked aggregation) and then a
    2048 x 2048 Zipf matrix on the same context: each equals hs_he_spmv's result limb for limb."""
    g = H.Context(14, 6, 50, 1, agg_mode=0)
    kg = g.keygen(7)
    check_against_he_spmv(g, kg, W.zipf16k())
    check_against_he_spmv(g, kg, W.zipf16k(idx=1, R=2048), poison=0x5A5A)


@pytest.mark.parametrize("relin", [0, 1], ids=["eager", "lazy"])
def test_noalloc_encrypted_matrix(relin):
    """Both operands encrypted (exact ciphertext products + relinearisation, masks) on a small
    ring, then a smaller Laplacian: equal to hs_he_spmv's results."""
    g = H.Context(10, 3, 50, 1, agg_mode=0, lazy_relin=relin)
    kg = g.keygen(23)
    check_against_he_spmv(g, kg, W.laplace256(n=30), encrypted=True)
    check_against_he_spmv(g, kg, W.laplace256(n=12), encrypted=True)


def test_noalloc_errors():
    """A short output buffer is refused (HS_ECAPACITY); an SpMV whose intermediates exceed the
    fixed array is refused (HS_ENOMEM) and leaves the library usable."""
    g = H.Context(12, 2, 30, 1, agg_mode=1)
    kg = g.keygen(11)
    w = W.small()
    M = matrix(g, kg, w)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 12)
    short = torch.zeros(M.groups() * g.ct_words() - 1, dtype=torch.int64, device="cuda")
    with pytest.raises(H.HespmvError) as e:
        H.he_spmv_noalloc(g, kg, M, x, short)
    assert e.value.code == H.HS_ECAPACITY
    big = H.Context(15, 12, 50, 2, agg_mode=0)
    kb = big.keygen(29)
    wl = W.laplace256(n=128)
    Ml = matrix(big, kb, wl, True, 31)
    xl = H.encrypt(big, kb, Ml, dev(wl["v"], torch.int64), 41)
    yl = torch.zeros(Ml.groups() * big.ct_words(), dtype=torch.int64, device="cuda")
    with pytest.raises(H.HespmvError) as e:
        H.he_spmv_noalloc(big, kb, Ml, xl, yl)
    assert e.value.code == H.HS_ENOMEM and "scratch" in str(e.value)
    check_against_he_spmv(g, kg, w)
