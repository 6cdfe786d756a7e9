"""GPU checks of boundary calls: caller-owned ciphertext buffers (hs_ctvec_wrap), the canonical
coefficient-form export (hs_ct_export_coeff) and per-context execution options
(hs_ctx_set_option), each through the C ABI against the CPU oracle."""
import numpy as np
import pytest

import oracle as O
from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402

P = (11, 3, 50, 1, 0)


def _dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a).astype(dt)).cuda()


def _setup(p=P, seed=13):
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    o = O.Context(logn, L, bits, K, agg_mode=agg)
    kg = g.keygen(seed)
    o.keygen(seed)
    rng = np.random.default_rng(seed)
    R = 700
    rp, col, val = W.uniform_matrix(R, R, 4000, 15, rng)
    w = dict(R=R, C=R, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, R))
    return g, kg, o, w


def test_wrapped_vector_is_read_in_place():
    """hs_ctvec_wrap over a torch tensor: he_spmv reads the caller's buffer (the oracle's
    encryption copied into it), gives the oracle's result limbs, and a change of the tensor's
    contents is seen by the next call without re-wrapping; destroying the handle leaves the tensor."""
    g, kg, o, w = _setup()
    M = H.Matrix(g, w["R"], w["C"], _dev(w["row_ptr"], np.int64), _dev(w["col"], np.int32), _dev(w["val"], np.int64))
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"])
    n = OM.n_chunks()
    ox1 = OM.encrypt_vector(w["v"], 5)
    buf = torch.from_numpy(ox1.view(np.int64).copy()).cuda()
    x = H.CtVec.wrap(g, buf, n)
    assert x.count() == n
    assert np.array_equal(x.export_all(), ox1)
    y = H.he_spmv(g, kg, M, x)
    oy1, _ = OM.he_spmv(ox1)
    assert np.array_equal(y.export_all(), oy1)
    v2 = -w["v"]
    ox2 = OM.encrypt_vector(v2, 6)
    buf.copy_(torch.from_numpy(ox2.view(np.int64)))
    y2 = H.he_spmv(g, kg, M, x)
    oy2, _ = OM.he_spmv(ox2)
    assert np.array_equal(y2.export_all(), oy2)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y2, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(dict(w, v=v2)))
    x.close()
    assert np.array_equal(buf.cpu().numpy().view(np.uint64), ox2)


def test_wrap_rejects_bad_arguments():
    g, kg, o, w = _setup()
    t = torch.zeros(2 * g.ct_words(), dtype=torch.int64, device="cuda")
    h = H.ctypes.c_void_p()
    assert H.lib.hs_ctvec_wrap(g.h, None, 1, H.ctypes.byref(h)) == H.HS_EINVAL
    assert H.lib.hs_ctvec_wrap(g.h, H.ctypes.c_void_p(t.data_ptr()), 0, H.ctypes.byref(h)) == H.HS_EINVAL
    assert H.lib.hs_ctvec_wrap(g.h, H.ctypes.c_void_p(t.data_ptr() + 4), 1, H.ctypes.byref(h)) == H.HS_EINVAL


@pytest.mark.parametrize("p", [P, (14, 6, 50, 1, 0), (15, 12, 50, 2, 0)])
def test_coefficient_form_export_is_the_inverse_transform(p):
    """hs_ct_export_coeff gives the canonical form: each limb is the oracle's inverse NTT of the
    NTT-form limb (the oracle's transform is pinned to direct evaluation), residues in [0, q);
    the vector itself is left in NTT form."""
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    o = O.Context(logn, L, bits, K, agg_mode=agg)
    N = 1 << logn
    mods = o.moduli()[:L]
    rng = np.random.default_rng(logn)
    cts = np.concatenate([rng.integers(0, mods[i], N, dtype=np.uint64) for _ in range(2 * 2) for i in range(L)])
    v = H.CtVec.from_host(g, cts, 2)
    for i in range(2):
        got = v.export_coeff(i).reshape(2, L, N)
        ntt = cts[i * 2 * L * N:(i + 1) * 2 * L * N].reshape(2, L, N)
        for c in range(2):
            for l in range(L):
                assert np.array_equal(got[c, l], o.intt(l, ntt[c, l].copy())), (i, c, l)
                assert int(got[c, l].max()) < mods[l]
        assert np.array_equal(v.export(i), cts[i * 2 * L * N:(i + 1) * 2 * L * N])


def test_per_context_options_override_the_process_default():
    """Two contexts of one ring: one forced to the one-workgroup key switch by its own option, the
    other to the two-pass one, while the process-wide default says the opposite; both give the
    oracle's limbs, and hs_ctx_set_option rejects unknown keys and values."""
    p = (11, 3, 50, 1, 0)
    g1, kg1, o, w = _setup(p, 17)
    g2 = H.Context(*p[:4], agg_mode=p[4])
    kg2 = g2.keygen(17)
    g1.set_option(H.OPT_KS_PIPELINE, 1)
    g2.set_option(H.OPT_KS_PIPELINE, 2)
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"])
    ox = OM.encrypt_vector(w["v"], 9)
    oy, _ = OM.he_spmv(ox)
    try:
        for default in (2, 1):
            H.set_option(H.OPT_KS_PIPELINE, default)
            for g, kg in ((g1, kg1), (g2, kg2)):
                M = H.Matrix(g, w["R"], w["C"], _dev(w["row_ptr"], np.int64), _dev(w["col"], np.int32), _dev(w["val"], np.int64))
                y = H.he_spmv(g, kg, M, H.CtVec.from_host(g, ox, OM.n_chunks()))
                assert np.array_equal(y.export_all(), oy)
    finally:
        H.set_option(H.OPT_KS_PIPELINE, 0)
    with pytest.raises(H.HespmvError):
        g1.set_option(99, 1)
    with pytest.raises(H.HespmvError):
        g1.set_option(H.OPT_KS_PIPELINE, 7)
    g1.set_option(H.OPT_KS_PIPELINE, -1)
