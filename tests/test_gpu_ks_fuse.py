"""GPU: consecutive two-pass rotation levels with the next level's first key-switch step (Galois
gather + inverse low pass of c1) run inside the previous level's last kernel (HS_OPT_KS_FUSE = 0)
and as a kernel of its own (1): rotations equal the oracle's under both, on every block geometry,
and the zipf16k SpMV and a batch are bit-identical with fewer launches when fused."""
import numpy as np
import pytest

import oracle as O
from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402


@pytest.fixture
def two_pass():
    H.set_option(H.OPT_KS_PIPELINE, 2)
    yield
    for k in (H.OPT_KS_PIPELINE, H.OPT_KS_BLOCK, H.OPT_KS_FUSE):
        H.set_option(k, 0)


def dev(a, dt):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dt)


@pytest.mark.parametrize("p", [(14, 6, 50, 1), (14, 4, 50, 2), (12, 3, 50, 1), (15, 4, 50, 1)], ids=["16k", "16k-K2", "4k", "32k"])
def test_chained_rotations_match_oracle_fused_and_not(two_pass, p):
    g = H.Context(*p, agg_mode=0)
    o = O.Context(*p, agg_mode=0)
    kg = g.keygen(8)
    o.keygen(8)
    N = 1 << p[0]
    rng = np.random.default_rng(4)
    cts = [o.encrypt(rng.integers(0, 65537, N).astype(np.uint64), 9, i) for i in range(3)]
    x = H.CtVec.from_host(g, np.concatenate(cts), 3)
    modes = (0, 1, 2, 3) if p[0] == 14 else (0,)
    for step in (5, 13):   # two and three levels of three items
        want = [o.rotate(ct, step) for ct in cts]
        for blk in modes:
            H.set_option(H.OPT_KS_BLOCK, blk)
            for fuse in (0, 1):
                H.set_option(H.OPT_KS_FUSE, fuse)
                print("p=%s step=%d block=%d fuse=%d" % (p, step, blk, fuse), flush=True)
                r = H.rotate(g, kg, x, step)
                for i in range(3):
                    assert np.array_equal(r.export(i), want[i]), (step, blk, fuse, i)


def test_zipf16k_and_batch_identical_fused_and_not():
    g = H.Context(14, 6, 50, 1, agg_mode=0)
    kg = g.keygen(8)
    w = W.zipf16k()
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"].astype(np.int32), torch.int32),
                 dev(w["val"], torch.int64))
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    ws = W.batch64(count=4, rmax=2048)
    ms = [H.Matrix(g, v["R"], v["C"], dev(v["row_ptr"], torch.int64), dev(v["col"].astype(np.int32), torch.int32),
                   dev(v["val"], torch.int64)) for v in ws]
    xs = [H.encrypt(g, kg, m, dev(v["v"], torch.int64), 60 + i) for i, (m, v) in enumerate(zip(ms, ws))]
    res = {}
    try:
        for fuse in (0, 1):
            H.set_option(H.OPT_KS_FUSE, fuse)
            print("fuse=%d" % fuse, flush=True)
            y = H.he_spmv(g, kg, M, x).export_all()
            launches = H.last_counters()["launches"]
            ys = [t.export_all() for t in H.he_spmv_batch(g, [kg] * len(ms), ms, xs)]
            res[fuse] = (y, launches, ys)
    finally:
        H.set_option(H.OPT_KS_FUSE, 0)
    assert np.array_equal(res[0][0], res[1][0])
    assert all(np.array_equal(a, b) for a, b in zip(res[0][2], res[1][2]))
    assert res[0][1] < res[1][1], (res[0][1], res[1][1])
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, H.he_spmv(g, kg, M, x), out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))
