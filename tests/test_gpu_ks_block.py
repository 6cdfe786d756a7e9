"""GPU: the block sizes of the two-pass key switch at N = 2^14 (HS_OPT_KS_BLOCK) change only the
launch shape: rotations equal the oracle's (digits of one and of two primes) and the zipf16k
he_spmv result is bit-identical under every choice, on the two-pass pipeline."""
import numpy as np
import pytest

import oracle as O
from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402

MODES = (0, 1, 2, 3)


@pytest.fixture
def two_pass():
    H.set_option(H.OPT_KS_PIPELINE, 2)
    yield
    H.set_option(H.OPT_KS_PIPELINE, 0)
    H.set_option(H.OPT_KS_BLOCK, 0)


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


@pytest.mark.parametrize("p", [(14, 6, 50, 1), (14, 4, 50, 2)], ids=["K1", "K2"])
def test_rotations_match_oracle_under_every_block_size(two_pass, p):
    g = H.Context(*p, agg_mode=0)
    o = O.Context(*p, agg_mode=0)
    kg = g.keygen(8)
    o.keygen(8)
    N = 1 << p[0]
    rng = np.random.default_rng(3)
    m = rng.integers(0, 65537, N).astype(np.uint64)
    ct = np.concatenate([o.encrypt(m, 9, i) for i in range(3)])
    want = [o.rotate(ct[i * o.ct_size():(i + 1) * o.ct_size()], 5) for i in range(3)]
    for mode in MODES:
        H.set_option(H.OPT_KS_BLOCK, mode)
        r = H.rotate(g, kg, H.CtVec.from_host(g, ct, 3), 5)   # two levels of three items
        for i in range(3):
            assert np.array_equal(r.export(i), want[i]), (mode, i)


def test_zipf16k_spmv_is_bit_identical_under_every_block_size(two_pass):
    g = H.Context(14, 6, 50, 1, agg_mode=0)
    kg = g.keygen(8)
    w = W.zipf16k()
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"].astype(np.int32), torch.int32),
                 dev(w["val"], torch.int64))
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    ys = []
    for mode in MODES:
        H.set_option(H.OPT_KS_BLOCK, mode)
        ys.append(H.he_spmv(g, kg, M, x).export_all())
    assert all(np.array_equal(ys[0], y) for y in ys[1:])
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.set_option(H.OPT_KS_BLOCK, 0)
    H.decrypt(g, kg, M, H.he_spmv(g, kg, M, x), out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))
