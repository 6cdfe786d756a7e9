"""GPU: two row partitions per ciphertext (slot rows 0 and 1) against the oracle, bit for bit.

With slot_rows = 2 a pair of row partitions shares every chunk ciphertext (chunks on the joint
column heights), so the matrix has about half the chunks, products and rotations; the plaintexts,
masks, encrypted vector, every result limb (one ciphertext per pair) and the decrypted product must
equal the oracle's.
"""
import numpy as np
import pytest

import oracle as O
from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402


def dev(a, dtype):
    npd = {torch.int64: np.int64, torch.int32: np.int32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(npd, copy=False))).cuda()


@pytest.fixture(params=[1, 2], ids=["ks_limb", "ks_2pass"])
def pipeline(request):
    H.set_option(H.OPT_KS_PIPELINE, request.param)
    yield request.param
    H.set_option(H.OPT_KS_PIPELINE, 0)


def workload(case):
    rng = np.random.default_rng({"three_parts": 1, "uniform": 2, "empty_second": 3, "zipf": 4, "ragged": 5}[case])
    if case == "zipf":
        return (14, 6, 50, 1, 0), W.zipf16k()
    p, (R, C, nnz) = {"three_parts": ((9, 3, 50, 1, 0), (700, 300, 2500)), "uniform": ((12, 2, 30, 1, 1), (5000, 2000, 12000)),
                      "empty_second": ((9, 3, 50, 1, 0), (300, 300, 600)), "ragged": ((11, 3, 50, 1, 0), (3000, 1500, 9000))}[case]
    rp, col, val = W.uniform_matrix(R, C, nnz, 15, rng)
    if case == "empty_second":   # rows 256.. (the second partition) without nonzeros
        rows = np.repeat(np.arange(R), np.diff(rp))
        keep = rows < 256
        rp, col, val = W._csr_from_rows_cols(R, rows[keep], col[keep], val[keep])
    return p, dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, C))


@pytest.mark.parametrize("case", ["three_parts", "uniform", "empty_second", "ragged", "zipf"])
def test_two_slot_rows_protocol(case, pipeline):
    (logn, L, bits, K, agg), w = workload(case)
    g = H.Context(logn, L, bits, K, agg_mode=agg, slot_rows=2)
    o = O.Context(logn, L, bits, K, agg_mode=agg, slot_rows=2)
    kg = g.keygen(13)
    o.keygen(13)
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64))
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], False, 31)
    assert M.info() == (OM.n_parts(), OM.n_chunks())
    assert M.groups() == OM.n_groups() == (OM.n_parts() + 1) // 2
    for k in range(OM.n_chunks()):
        assert M.chunk(k) == OM.chunk(k), k
        assert np.array_equal(M.export(0, k), OM.pt(k)), ("plaintext", k)
        if agg == 0:
            assert np.array_equal(M.export(1, k), OM.mask(k)), ("mask", k)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    ox = OM.encrypt_vector(w["v"], 41)
    assert np.array_equal(x.export_all(), ox)
    y = H.he_spmv(g, kg, M, x)
    oy, stats = OM.he_spmv(ox)
    cnt = H.last_counters()
    assert cnt["key_switches"] == stats["key_switches"] and cnt["rotations"] == stats["rotations"]
    assert y.count() == OM.n_groups()
    assert np.array_equal(y.export_all(), oy)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


def test_two_slot_rows_batch_plan_and_server():
    """Matrices of one, two and three partitions in one batch, graph plan and server."""
    p = (10, 3, 50, 1, 0)
    g = H.Context(*p[:4], agg_mode=p[4], slot_rows=2)
    o = O.Context(*p[:4], agg_mode=p[4], slot_rows=2)
    kg = g.keygen(17)
    o.keygen(17)
    rng = np.random.default_rng(6)
    reqs = []
    for i, (R, C, nnz) in enumerate([(300, 200, 1200), (1000, 600, 4000), (1400, 900, 5000)]):
        rp, col, val = W.uniform_matrix(R, C, nnz, 15, rng)
        w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, C))
        M = H.Matrix(g, R, C, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.int64))
        OM = O.Matrix(o, R, C, rp, col, val, False, 0)
        x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 70 + i)
        oy, _ = OM.he_spmv(OM.encrypt_vector(w["v"], 70 + i))
        reqs.append((w, M, x, oy))
    ms, xs = [r[1] for r in reqs], [r[2] for r in reqs]
    for y, r in zip(H.he_spmv_batch(g, [kg] * 3, ms, xs), reqs):
        assert np.array_equal(y.export_all(), r[3])
    plan = H.BatchPlan(g, [kg] * 3, ms, xs)
    plan.run()
    torch.cuda.synchronize()
    for y, r in zip(plan.outputs(), reqs):
        assert np.array_equal(y.export_all(), r[3])
    plan.close()
    srv = H.Server(g, 1 << 30, 8)
    ids = [srv.submit(kg, r[1], r[2]) for r in reqs]
    for rid, r in zip(ids, reqs):
        y, _ = srv.wait(rid)
        assert np.array_equal(y.export_all(), r[3])
        out = torch.zeros(r[0]["R"], dtype=torch.int64, device="cuda")
        H.decrypt(g, kg, r[1], y, out)
        assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(r[0]))
    srv.close()
