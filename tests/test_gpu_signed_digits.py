"""GPU: right rotation keys and signed-digit rotations against the oracle, bit for bit, through
the C ABI.

With the optional right keys (hs_keyset_add_right_rotation_keys; right rotations by 2^i, Galois
element 3^(-2^i) mod 2N) a rotation by k without an exact-step key applies the signed digits
+-2^i of the non-adjacent form of k mod N/2, lowest first, one key switch each (the power-of-two
keys of Sec. 5 read as common BFV libraries generate and apply them; the paper-reading default is
left keys and binary digits).  The right keys, every rotated limb, the he_spmv result (single,
batched, graph replay and server), the diagonal method and the decrypted products must equal the
oracle's with the same option.
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

SMALL = (12, 2, 30, 1, 1)
RING16K = (14, 6, 50, 1, 0)
TINY = (9, 3, 50, 1, 0)
TINY11 = (11, 3, 50, 1, 0)


def dev(a, dtype):
    npd = {torch.int64: np.int64, torch.int32: np.int32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(npd, copy=False))).cuda()


@pytest.fixture(params=[1, 2], ids=["ks_limb", "ks_2pass"])
def pipeline(request):
    H.set_option(H.OPT_KS_PIPELINE, request.param)
    yield request.param
    H.set_option(H.OPT_KS_PIPELINE, 0)


def fresh(p, seed=8, right=True):
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    o = O.Context(logn, L, bits, K, agg_mode=agg)
    kg = g.keygen(seed)
    o.keygen(seed)
    if right:
        kg.add_right_rotation_keys()
        o.add_right_rotation_keys()
    return g, kg, o


@pytest.mark.parametrize("p", [TINY, SMALL, RING16K], ids=["ring512", "ring4096", "ring16k"])
def test_right_keys_and_rotations_match_oracle(p):
    g, kg, o = fresh(p, right=False)
    nl = p[0] - 1
    with pytest.raises(H.HespmvError):
        kg.export(2, nl)
    kg.add_right_rotation_keys()
    kg.add_right_rotation_keys()   # a second call adds nothing
    o.add_right_rotation_keys()
    for i in (range(2 * nl) if p != RING16K else (0, 12, nl, nl + 5, 2 * nl - 1)):
        assert np.array_equal(kg.export(2, i), o.ksk(i)), i
    with pytest.raises(H.HespmvError):
        kg.export(2, 2 * nl)
    N, h = 1 << p[0], (1 << p[0]) // 2
    rng = np.random.default_rng(5)
    m = rng.integers(0, 65537, N).astype(np.uint64)
    ct = np.concatenate([o.encrypt(m, 9, 0), o.encrypt(m, 9, 1)])
    x = H.CtVec.from_host(g, ct, 2)
    for k in (1, 3, 11, 37, h - 1, h - 6, -5):
        assert len(o.rotation_digits(k)) <= len([b for b in bin(k % h) if b == "1"])
        r = H.rotate(g, kg, x, k)
        assert np.array_equal(r.export(0), o.rotate(ct[:o.ct_size()], k % h)), k
        assert np.array_equal(r.export(1), o.rotate(ct[o.ct_size():], k % h)), k
    sl = o.decode(m)
    want = np.concatenate([np.roll(sl[:h], 5), np.roll(sl[h:], 5)])
    assert np.array_equal(o.decode(o.decrypt(H.rotate(g, kg, x, -5).export(0))), want)


def workload(case):
    rng = np.random.default_rng({"tiny": 17, "ragged": 18, "zipf": 19}[case])
    if case == "zipf":
        return RING16K, W.zipf16k()
    p, (R, C, nnz) = (TINY, (300, 200, 1200)) if case == "tiny" else (TINY11, (3000, 1500, 9000))
    rp, col, val = W.uniform_matrix(R, C, nnz, 15, rng)
    return p, dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, C))


@pytest.mark.parametrize("case", ["tiny", "ragged", "zipf"])
def test_protocol_with_signed_digits(case, pipeline):
    p, w = workload(case)
    g, kg, o = fresh(p)
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64))
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], False, 0)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    ox = OM.encrypt_vector(w["v"], 41)
    assert np.array_equal(x.export_all(), ox)
    y = H.he_spmv(g, kg, M, x)
    oy, stats = OM.he_spmv(ox)
    cnt = H.last_counters()
    want = sum(len(o.rotation_digits(k)) for c in range(OM.n_chunks())
               for k in o.total_sum_steps(OM.chunk(c)[3], OM.chunk(c)[2]))
    assert cnt["key_switches"] == stats["key_switches"] == want
    assert cnt["rotations"] == stats["rotations"]
    assert np.array_equal(y.export_all(), oy)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


def test_batch_plan_and_server_with_signed_digits():
    """Two key-sets, one with right keys and one without, in one batch, one graph plan and the
    server: each request's result equals the oracle's for its own key-set."""
    p = TINY11
    g = H.Context(*p[:4], agg_mode=p[4])
    oa, ob = O.Context(*p[:4], agg_mode=p[4]), O.Context(*p[:4], agg_mode=p[4])
    ka, kb = g.keygen(21), g.keygen(22)
    oa.keygen(21)
    ob.keygen(22)
    ka.add_right_rotation_keys()
    oa.add_right_rotation_keys()
    rng = np.random.default_rng(23)
    reqs = []
    for i, (R, C, nnz) in enumerate([(300, 200, 1200), (1500, 900, 5000), (40, 40, 100)]):
        rp, col, val = W.uniform_matrix(R, C, nnz, 15, rng)
        w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, C))
        M = H.Matrix(g, R, C, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.int64))
        ks, o = (ka, oa) if i != 1 else (kb, ob)
        OM = O.Matrix(o, R, C, rp, col, val, False, 0)
        x = H.encrypt(g, ks, M, dev(w["v"], torch.int64), 60 + i)
        oy, _ = OM.he_spmv(OM.encrypt_vector(w["v"], 60 + i))
        reqs.append((w, ks, M, x, oy))
    kss, ms, xs = [r[1] for r in reqs], [r[2] for r in reqs], [r[3] for r in reqs]
    for y, r in zip(H.he_spmv_batch(g, kss, ms, xs), reqs):
        assert np.array_equal(y.export_all(), r[4])
    plan = H.BatchPlan(g, kss, ms, xs)
    for _ in range(2):
        plan.run()
        torch.cuda.synchronize()
        for y, r in zip(plan.outputs(), reqs):
            assert np.array_equal(y.export_all(), r[4])
    plan.close()
    srv = H.Server(g, 1 << 30, 8)
    ids = [srv.submit(r[1], r[2], r[3]) for r in reqs]
    for rid, r in zip(ids, reqs):
        y, _ = srv.wait(rid)
        assert np.array_equal(y.export_all(), r[4])
    srv.close()


def test_diagonal_method_with_signed_digits():
    """The diagonal method with right keys: every result limb equals the oracle's, with one key
    switch per distinct partial sum of the offsets' signed digits per block column."""
    p = TINY
    g, kg, o = fresh(p)
    rng = np.random.default_rng(31)
    R, C = 300, 200
    rp, col, val = W.uniform_matrix(R, C, 1200, 15, rng)
    v = rng.integers(-15, 16, C)
    D = H.DiagMatrix(g, R, C, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.int64))
    OD = O.DiagMatrix(o, R, C, rp, col, val)
    x = H.diag_encrypt(g, kg, D, dev(v, torch.int64), 41)
    ox = OD.encrypt_vector(v, 41)
    assert np.array_equal(x.export_all(), ox)
    y = H.diag_spmv(g, kg, D, x)
    cnt = H.last_counters()
    assert np.array_equal(y.export_all(), OD.spmv(ox))
    keys = D.keys()
    want = 0
    for bj in range(D.info()[2]):
        nodes = set()
        for d in {int(k[2]) for k in keys if k[1] == bj} - {0}:
            s_ = 0
            for z in o.rotation_digits(d):
                s_ += z
                nodes.add(s_)
        want += len(nodes)
    assert cnt["key_switches"] == want
    out = torch.full((R,), 12345, dtype=torch.int64, device="cuda")
    H.diag_decrypt(g, kg, D, y, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=v)))
