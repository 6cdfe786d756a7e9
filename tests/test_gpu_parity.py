"""GPU parity: every stage of the HIP path against the CPU oracle, bit for bit, through the C ABI.

Inputs come from the seeded generators in paper_2603_04742_amd.workloads; randomness the method
draws (keys, encryption noise) comes from the same ChaCha20 streams on both sides.
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

# (log_n, L, bits, K, agg_mode): the small ring of the 256 x 256 workload, the 16384 ring, and
# small rings with several partitions and ragged sizes
SMALL = (12, 2, 30, 1, 1)
RING16K = (14, 6, 50, 1, 0)
TINY = (9, 3, 50, 1, 0)
TINY11 = (11, 3, 50, 1, 0)


def dev(a, dtype):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    npd = {torch.int64: np.int64, torch.int32: np.int32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(a.astype(npd, copy=False))).cuda()


_cache = {}


@pytest.fixture(params=[1, 2], ids=["ks_limb", "ks_2pass"])
def pipeline(request):
    """Run the test under both key-switch pipelines (results must be identical)."""
    H.set_option(H.OPT_KS_PIPELINE, request.param)
    yield request.param
    H.set_option(H.OPT_KS_PIPELINE, 0)


def contexts(p, seed=7):
    key = (p, seed)
    if key not in _cache:
        logn, L, bits, K, agg = p
        g = H.Context(logn, L, bits, K, agg_mode=agg)
        o = O.Context(logn, L, bits, K, agg_mode=agg)
        kg = g.keygen(seed)
        o.keygen(seed)
        _cache[key] = (g, kg, o)
    return _cache[key]


@pytest.mark.parametrize("p", [SMALL, RING16K, TINY, (15, 12, 50, 2, 0)])
def test_moduli_match_oracle(p):
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    o = O.Context(logn, L, bits, K, agg_mode=agg)
    assert g.moduli() == o.moduli()


@pytest.fixture(params=[1, 2], ids=["ntt_limb", "ntt_2pass"])
def ntt_path(request):
    H.set_option(H.OPT_NTT_PATH, request.param)
    yield request.param
    H.set_option(H.OPT_NTT_PATH, 0)


@pytest.mark.parametrize("p", [(3, 2, 30, 1, 0), (6, 2, 30, 1, 0), (10, 3, 50, 1, 0), (11, 2, 40, 1, 0), SMALL, (13, 2, 50, 1, 0), RING16K])
def test_ntt_parity(p, ntt_path):
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    o = O.Context(logn, L, bits, K, agg_mode=agg)
    N = 1 << logn
    mods = o.moduli()[:L + K]
    rng = np.random.default_rng(logn)
    npoly = 3
    x = np.stack([np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in mods]) for _ in range(npoly)])
    d = dev(x.reshape(-1), torch.int64)
    g.ntt(d, 0, len(mods), inverse=False)
    got = d.cpu().numpy().view(np.uint64).reshape(npoly, len(mods), N)
    for pi in range(npoly):
        for m in range(len(mods)):
            assert np.array_equal(got[pi, m], o.ntt(m, x[pi, m])), (p, pi, m)
    g.ntt(d, 0, len(mods), inverse=True)
    assert np.array_equal(d.cpu().numpy().view(np.uint64).reshape(x.shape), x)
    # plaintext modulus t
    y = rng.integers(0, 65537, N, dtype=np.uint64)
    dt = dev(y, torch.int64)
    g.ntt(dt, -1, 1, inverse=True)
    assert np.array_equal(dt.cpu().numpy().view(np.uint64), o.intt(-1, y))


@pytest.mark.parametrize("p", [SMALL, TINY])
def test_keygen_parity(p):
    g, kg, o = contexts(p)
    assert np.array_equal(kg.export(0), o.sk_ntt())
    assert np.array_equal(kg.export(1), o.pk())
    for i in range(p[0] - 1):
        assert np.array_equal(kg.export(2, i), o.ksk(i)), i
    assert np.array_equal(kg.export(3), o.ksk(-1))


def test_keygen_parity_16k():
    g, kg, o = contexts(RING16K)
    assert np.array_equal(kg.export(0), o.sk_ntt())
    assert np.array_equal(kg.export(1), o.pk())
    for i in (0, 5, 12):
        assert np.array_equal(kg.export(2, i), o.ksk(i)), i
    assert np.array_equal(kg.export(3), o.ksk(-1))


def gpu_matrix(g, kg, w, encrypted=False, seed=31):
    return H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32),
                    dev(w["val"], torch.int64), encrypted, kg if encrypted else None, seed)


def check_protocol(p, w, mat_seed=31, vec_seed=41):
    """Every stage of the protocol, GPU vs oracle, bit for bit; returns the decrypted result."""
    g, kg, o = contexts(p)
    M = gpu_matrix(g, kg, w, seed=mat_seed)
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], False, mat_seed)
    nparts, nchunks = M.info()
    assert (nparts, nchunks) == (OM.n_parts(), OM.n_chunks())
    for k in range(nchunks):
        assert M.chunk(k) == OM.chunk(k)
        assert np.array_equal(M.export(0, k), OM.pt(k)), ("plaintext", k)
        if p[4] == 0:
            assert np.array_equal(M.export(1, k), OM.mask(k)), ("mask", k)
    # column index array (Client A -> Client B): the CSSC CI of every partition in order
    # and the row map and column pointers of every partition (built on the device)
    s = (1 << p[0]) // 2
    ci = []
    for part, r0 in enumerate(range(0, w["R"], s)):
        r1 = min(w["R"], r0 + s)
        rp = w["row_ptr"][r0:r1 + 1] - w["row_ptr"][r0]
        sl = slice(w["row_ptr"][r0], w["row_ptr"][r1])
        _, CI, RM, CP = O.cssc(r1 - r0, rp, w["col"][sl], w["val"][sl])
        grm, gcp = M.cssc(part)
        assert np.array_equal(grm, RM) and np.array_equal(gcp, CP), ("cssc", part)
        ci.append(CI)
    ci = np.concatenate(ci) if ci else np.zeros(0, np.int32)
    assert np.array_equal(M.column_index(), ci)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), vec_seed)
    ox = OM.encrypt_vector(w["v"], vec_seed)
    assert np.array_equal(x.export_all(), ox), "encrypted vector"
    y = H.he_spmv(g, kg, M, x)
    oy, stats = OM.he_spmv(ox)
    cnt = H.last_counters()
    assert cnt["key_switches"] == stats["key_switches"] and cnt["rotations"] == stats["rotations"]
    assert np.array_equal(y.export_all(), oy), "he_spmv result"
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y, out)
    res = out.cpu().numpy()
    assert np.array_equal(res, OM.decrypt_result(oy))
    assert np.array_equal(res, W.spmv_mod_t(w))
    return res


def test_protocol_small_workload(pipeline):
    check_protocol(SMALL, W.small())


@pytest.mark.parametrize("case", ["empty", "one", "emptyrows", "rect", "partitions", "dense_row", "ragged"])
def test_protocol_edge_cases(case, pipeline):
    rng = np.random.default_rng(abs(hash(case)) % 1000)
    p = TINY
    if case == "empty":
        R, C, nnz = 10, 10, 0
    elif case == "one":
        R, C, nnz = 1, 1, 1
    elif case == "emptyrows":
        R, C, nnz = 100, 50, 60
    elif case == "rect":
        R, C, nnz = 30, 200, 500
    elif case == "partitions":
        R, C, nnz = 700, 300, 2500
    elif case == "ragged":
        p = TINY11
        R, C, nnz = 3000, 1500, 9000   # three partitions of <= 1024 rows, last one ragged
    else:
        R, C, nnz = 20, 256, 0
    if case == "dense_row":
        rows = np.concatenate([np.zeros(256, np.int64), rng.integers(1, R, 19)])
        cols = np.concatenate([np.arange(256), rng.integers(0, C, 19)])
        key = np.unique(rows * C + cols)
        rows, cols = key // C, key % C
        rp, col, val = W._csr_from_rows_cols(R, rows, cols, rng.integers(-15, 16, len(rows)))
    else:
        rp, col, val = W.uniform_matrix(R, C, nnz, 15, rng)
    w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, C))
    check_protocol(p, w)


def test_rotation_parity(pipeline):
    for p in (SMALL, TINY):
        g, kg, o = contexts(p)
        N = 1 << p[0]
        rng = np.random.default_rng(5)
        m = rng.integers(0, 65537, N).astype(np.uint64)
        ct = np.concatenate([o.encrypt(m, 9, 0), o.encrypt(m, 9, 1)])
        x = H.CtVec.from_host(g, ct, 2)
        for k in (1, 6, 11, 37, N // 2 - 1):
            r = H.rotate(g, kg, x, k)
            assert np.array_equal(r.export(0), o.rotate(ct[:o.ct_size()], k)), (p, k)
            assert np.array_equal(r.export(1), o.rotate(ct[o.ct_size():], k)), (p, k)


def test_mul_plain_parity():
    g, kg, o = contexts(TINY)
    N = 1 << TINY[0]
    rng = np.random.default_rng(6)
    m = rng.integers(0, 65537, N).astype(np.uint64)
    ct = o.encrypt(m, 3, 0)
    pt = o.plain_ntt(o.encode(rng.integers(0, 65537, N)))
    r = H.mul_plain(g, H.CtVec.from_host(g, ct, 1), dev(pt, torch.int64))
    assert np.array_equal(r.export(0), o.ct_mul_plain(ct, pt))


def test_protocol_zipf16k_full_size(pipeline):
    """The 16384 x 16384 Zipf workload at full size (two partitions, ~22 chunks, ~56 key
    switches): every ciphertext limb and the decrypted result against the oracle."""
    check_protocol(RING16K, W.zipf16k())


def test_repeated_runs_are_bit_identical(pipeline):
    """A race in the batched kernels would show up as a limb mismatch between runs."""
    g, kg, o = contexts(SMALL)
    w = W.small(1)
    M = gpu_matrix(g, kg, w)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 5)
    a = H.he_spmv(g, kg, M, x).export_all()
    for _ in range(3):
        assert np.array_equal(H.he_spmv(g, kg, M, x).export_all(), a)


def test_ntt_32768_two_pass():
    """N = 32768 (limb larger than LDS): a handful of limbs takes the two-pass transform."""
    g = H.Context(15, 2, 50, 1)
    o = O.Context(15, 2, 50, 1)
    rng = np.random.default_rng(15)
    mods = o.moduli()[:3]
    x = np.stack([rng.integers(0, q, 1 << 15, dtype=np.uint64) for q in mods])
    d = dev(x.reshape(-1), torch.int64)
    g.ntt(d, 0, 3)
    got = d.cpu().numpy().view(np.uint64).reshape(3, -1)
    for m in range(3):
        assert np.array_equal(got[m], o.ntt(m, x[m]))
    g.ntt(d, 0, 3, inverse=True)
    assert np.array_equal(d.cpu().numpy().view(np.uint64).reshape(3, -1), x)


@pytest.mark.parametrize("path", [0, 1], ids=["auto_300_limbs", "forced_3_limbs"])
def test_ntt_32768_one_workgroup_per_limb(path):
    """N = 32768 with one workgroup per limb on half-limb LDS (k_ntt15): a batch of 300 limbs (the
    automatic choice from 256 on) and 3 limbs with the path forced; sampled limbs equal the
    oracle's transform, and the inverse restores every limb."""
    g = H.Context(15, 12, 50, 2)
    o = O.Context(15, 12, 50, 2)
    rng = np.random.default_rng(16)
    nl = 14
    mods = o.moduli()[:nl]
    npoly = 22 if path == 0 else 1   # 308 limbs, or 14
    base = np.stack([rng.integers(0, q, 1 << 15, dtype=np.uint64) for q in mods])
    x = np.concatenate([np.roll(base, p, axis=1) for p in range(npoly)])
    if path == 1:
        x = x[:3]
        nl = 3
        H.set_option(H.OPT_NTT_PATH, 1)
    try:
        d = dev(x.reshape(-1), torch.int64)
        g.ntt(d, 0, nl)
        got = d.cpu().numpy().view(np.uint64).reshape(x.shape[0], -1)
        for r in sorted({0, 1, x.shape[0] // 2, x.shape[0] - 1}):
            assert np.array_equal(got[r], o.ntt(r % nl, x[r])), r
        g.ntt(d, 0, nl, inverse=True)
        assert np.array_equal(d.cpu().numpy().view(np.uint64).reshape(x.shape[0], -1), x)
    finally:
        H.set_option(H.OPT_NTT_PATH, 0)


def test_ntt_32768_extreme_residues():
    """k_ntt15 (8-byte twiddles in its LDS rounds) on residues at the top of [0, q): all q - 1 and
    alternating q - 1 / 0 limbs equal the oracle's transform; the inverse restores them."""
    g = H.Context(15, 12, 50, 2)
    o = O.Context(15, 12, 50, 2)
    nl = 14
    mods = o.moduli()[:nl]
    H.set_option(H.OPT_NTT_PATH, 1)
    try:
        for kind in (0, 1):
            x = np.stack([np.full(1 << 15, q - 1, np.uint64) if kind == 0 else
                          np.where(np.arange(1 << 15) % 2 == 0, q - 1, 0).astype(np.uint64) for q in mods[:3]])
            d = dev(x.reshape(-1), torch.int64)
            g.ntt(d, 0, 3)
            got = d.cpu().numpy().view(np.uint64).reshape(3, -1)
            for r in range(3):
                assert np.array_equal(got[r], o.ntt(r, x[r])), (kind, r)
            g.ntt(d, 0, 3, inverse=True)
            assert np.array_equal(d.cpu().numpy().view(np.uint64).reshape(3, -1), x)
    finally:
        H.set_option(H.OPT_NTT_PATH, 0)


def test_options_rejected():
    with pytest.raises(H.HespmvError):
        H.set_option(99, 1)
    with pytest.raises(H.HespmvError):
        H.set_option(H.OPT_KS_PIPELINE, 7)


def test_invalid_csr_rejected():
    g, kg, o = contexts(TINY)
    rp = np.array([0, 2, 1], np.int64)   # decreasing row pointer
    with pytest.raises(H.HespmvError) as e:
        H.Matrix(g, 2, 4, dev(rp, torch.int64), dev(np.array([0, 1], np.int32), torch.int32), dev(np.array([1, 1]), torch.int64))
    assert e.value.code == H.HS_EINVAL
    rp = np.array([0, 2], np.int64)       # column out of range
    with pytest.raises(H.HespmvError):
        H.Matrix(g, 1, 4, dev(rp, torch.int64), dev(np.array([0, 9], np.int32), torch.int32), dev(np.array([1, 1]), torch.int64))
    rp = np.array([0, 2], np.int64)       # columns not ascending within the row
    with pytest.raises(H.HespmvError):
        H.Matrix(g, 1, 4, dev(rp, torch.int64), dev(np.array([2, 1], np.int32), torch.int32), dev(np.array([1, 1]), torch.int64))


def _pack_and_encrypt(g, kg, w, seed):
    M = gpu_matrix(g, kg, w)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), seed)
    return M, x


@pytest.mark.parametrize("n_keysets", [1, 2])
def test_batch_equals_individual_calls(pipeline, n_keysets):
    """hs_he_spmv_batch over requests of mixed sizes (including an empty matrix and several
    partitions) and key-sets returns, per request, exactly its own hs_he_spmv result."""
    p = TINY
    g, kg0, o = contexts(p)
    kgs = [kg0] + ([g.keygen(8)] if n_keysets == 2 else [])
    rng = np.random.default_rng(21)
    reqs = []
    for i, (R, C, nnz) in enumerate([(40, 30, 200), (10, 10, 0), (300, 300, 1500), (700, 200, 2000), (5, 80, 60), (256, 256, 2500)]):
        rp, col, val = W.uniform_matrix(R, C, nnz, 7, rng)
        w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-7, 8, C))
        ks = kgs[i % len(kgs)]
        M, x = _pack_and_encrypt(g, ks, w, 100 + i)
        reqs.append((w, ks, M, x))
    ys = H.he_spmv_batch(g, [r[1] for r in reqs], [r[2] for r in reqs], [r[3] for r in reqs])
    for (w, ks, M, x), y in zip(reqs, ys):
        solo = H.he_spmv(g, ks, M, x)
        assert np.array_equal(y.export_all(), solo.export_all())
        out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
        H.decrypt(g, ks, M, y, out)
        assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


def test_batch64_workload_sample():
    """Eight matrices of the 64-matrix batch generator on the 16384 ring: batch == individual,
    and the decrypted results equal the integer SpMV."""
    g, kg, o = contexts(RING16K)
    ws = W.batch64(count=8, rmax=4096)
    pairs = [_pack_and_encrypt(g, kg, w, 7 + i) for i, w in enumerate(ws)]
    ys = H.he_spmv_batch(g, [kg] * len(ws), [p[0] for p in pairs], [p[1] for p in pairs])
    for w, (M, x), y in zip(ws, pairs, ys):
        assert np.array_equal(y.export_all(), H.he_spmv(g, kg, M, x).export_all())
        out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
        H.decrypt(g, kg, M, y, out)
        assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


def test_batch64_full_batch_against_oracle():
    """The whole 64-matrix batch (rows log-uniform in [512, 16384], densities log-uniform in
    [0.05 %, 1 %]) on the 16384 ring in one hs_he_spmv_batch call, rotation levels merged across all
    requests; three of its requests (the two smallest and a mid-size one) equal the oracle's
    he_spmv limb for limb, and every request equals its own hs_he_spmv."""
    g, kg, o = contexts(RING16K)
    ws = W.batch64()
    pairs = [_pack_and_encrypt(g, kg, w, 50 + i) for i, w in enumerate(ws)]
    print("batch64: %d requests" % len(ws), flush=True)
    ys = H.he_spmv_batch(g, [kg] * len(ws), [p[0] for p in pairs], [p[1] for p in pairs])
    order = sorted(range(len(ws)), key=lambda i: ws[i]["R"])
    for i in (order[0], order[1], order[20]):
        w = ws[i]
        print("batch64 request %d: %d x %d, %d nnz" % (i, w["R"], w["C"], int(w["row_ptr"][-1])), flush=True)
        OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], False, 31)
        ox = OM.encrypt_vector(w["v"], 50 + i)
        assert np.array_equal(pairs[i][1].export_all(), ox)
        oy, _ = OM.he_spmv(ox)
        assert np.array_equal(ys[i].export_all(), oy)
    for (M, x), y in zip(pairs[::8], ys[::8]):
        assert np.array_equal(y.export_all(), H.he_spmv(g, kg, M, x).export_all())


@pytest.fixture
def split_path():
    """Force keygen/encoding/encryption/decryption onto the elementwise + two-pass-NTT path (the
    path every N = 32768 ring takes), at ring sizes the oracle handles quickly."""
    H.set_option(H.OPT_AUX_PATH, 2)
    H.set_option(H.OPT_NTT_PATH, 2)
    yield
    H.set_option(H.OPT_AUX_PATH, 0)
    H.set_option(H.OPT_NTT_PATH, 0)


@pytest.mark.parametrize("p", [SMALL, TINY, (10, 3, 50, 2, 0)])
def test_split_path_keygen_and_protocol(p, split_path, pipeline):
    g = H.Context(*p[:4], agg_mode=p[4])
    o = O.Context(*p[:4], agg_mode=p[4])
    kg = g.keygen(19)
    o.keygen(19)
    assert np.array_equal(kg.export(0), o.sk_ntt())
    assert np.array_equal(kg.export(1), o.pk())
    for i in (0, p[0] - 2):
        assert np.array_equal(kg.export(2, i), o.ksk(i))
    assert np.array_equal(kg.export(3), o.ksk(-1))
    _cache[(p, 19)] = (g, kg, o)
    rng = np.random.default_rng(3)
    R = 3 * (1 << p[0]) // 4
    rp, col, val = W.uniform_matrix(R, R, 6 * R, 7, rng)
    check_protocol_seeded(p, 19, dict(R=R, C=R, row_ptr=rp, col=col, val=val, v=rng.integers(-7, 8, R)))


def check_protocol_seeded(p, seed, w):
    saved = _cache.get((p, 7))
    _cache[(p, 7)] = _cache[(p, seed)]
    try:
        check_protocol(p, w)
    finally:
        if saved is None:
            del _cache[(p, 7)]
        else:
            _cache[(p, 7)] = saved


@pytest.mark.parametrize("p", [(6, 3, 50, 1, 0), (8, 4, 40, 2, 0), (10, 3, 50, 2, 0), (13, 4, 50, 2, 0), (10, 12, 50, 2, 0),
                               (10, 11, 50, 2, 0), (10, 14, 45, 2, 0)])
def test_mul_ct_parity(p):
    """Exact scaled tensor + relinearisation against the oracle, bit for bit (K = 1 and K = 2
    digits).  The multiword kernels come in word capacities of 8, 16 and 24; the 24-word rings
    cover the instance with the widths of 12 x 50-bit primes fixed at compile time (12 primes),
    the runtime-width 24-word kernels (11 x 50-bit primes) and a ring whose CRT lift takes the fixed
    instance while its scaled rounding takes the runtime-width one (14 x 45-bit).  The product
    decrypts to the slot-wise product."""
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    o = O.Context(logn, L, bits, K, agg_mode=agg)
    assert g.moduli() == o.moduli()
    kg = g.keygen(5)
    o.keygen(5)
    N = 1 << logn
    rng = np.random.default_rng(logn)
    x, y = rng.integers(-40, 40, N), rng.integers(-40, 40, N)
    ca = np.concatenate([o.encrypt(o.encode(x), 1, i) for i in range(2)])
    cb = np.concatenate([o.encrypt(o.encode(y), 2, i) for i in range(2)])
    r = H.mul_ct(g, kg, H.CtVec.from_host(g, ca, 2), H.CtVec.from_host(g, cb, 2))
    cs = o.ct_size()
    for i in range(2):
        want = o.ct_mul_ct(ca[i * cs:(i + 1) * cs], cb[i * cs:(i + 1) * cs])
        assert np.array_equal(r.export(i), want), i
    assert np.array_equal(o.decode(o.decrypt(r.export(0))), (x * y) % 65537)


@pytest.mark.parametrize("p", [(10, 3, 50, 1, 0), (10, 4, 50, 2, 0)])
def test_protocol_both_encrypted(p, pipeline):
    """Matrix values encrypted too (HE-Mult + relinearisation, then masks): every stage bit for
    bit against the oracle, on a small 5-point Laplacian."""
    g = H.Context(*p[:4], agg_mode=p[4])
    o = O.Context(*p[:4], agg_mode=p[4])
    kg = g.keygen(23)
    o.keygen(23)
    w = W.laplace256(n=30)   # 900 rows: two partitions of <= 512
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64), True, kg, 31)
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], True, 31)
    assert M.info() == (OM.n_parts(), OM.n_chunks())
    for k in range(M.info()[1]):
        assert np.array_equal(M.export(0, k), OM.pt(k, encrypted=True))
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    ox = OM.encrypt_vector(w["v"], 41)
    assert np.array_equal(x.export_all(), ox)
    y = H.he_spmv(g, kg, M, x)
    oy, _ = OM.he_spmv(ox)
    assert np.array_equal(y.export_all(), oy)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


def test_mul_ct_refused_without_a_large_enough_basis():
    """N = 2^14 with two 20-bit data primes: the NTT-friendly 20-bit primes run out before their
    product exceeds 4 N Q^2, so the exact ciphertext product and encrypted matrices are refused
    (HS_EPARAM) instead of wrapping; the same ring still runs the plaintext-matrix path."""
    g = H.Context(14, 2, 20, 1, agg_mode=0)
    o = O.Context(14, 2, 20, 1, agg_mode=0)
    assert g.moduli() == o.moduli() and not o.has_tensor()
    kg = g.keygen(3)
    z = H.CtVec.from_host(g, np.zeros(o.ct_size(), np.uint64), 1)
    with pytest.raises(H.HespmvError) as e:
        H.mul_ct(g, kg, z, z)
    assert e.value.code == H.HS_EPARAM
    w = W.laplace256(n=8)
    with pytest.raises(H.HespmvError) as e:
        H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64), True, kg, 1)
    assert e.value.code == H.HS_EPARAM


_lap = {}


def _laplace_contexts(relin):
    """Library and oracle contexts of the laplace256 ring (N = 32768, 12 x 50-bit data primes, 2
    special primes), keys from seed 29 (the oracle's keys are made once and shared)."""
    p = (15, 12, 50, 2)
    if "o" not in _lap:
        _lap["o"] = O.Context(*p, agg_mode=0)
        _lap["o"].keygen(29)
        _lap["o_lazy"] = O.Context(*p, agg_mode=0, lazy_relin=1)
        _lap["o_lazy"].keygen(29)
    if relin not in _lap:
        g = H.Context(*p, agg_mode=0, lazy_relin=relin)
        _lap[relin] = (g, g.keygen(29))
    g, kg = _lap[relin]
    return g, kg, _lap["o_lazy" if relin else "o"]


@pytest.mark.parametrize("relin", [0, 1], ids=["eager", "lazy"])
def test_laplace256_full_size_result_limbs(relin):
    """The whole both-encrypted laplace256 SpMV at its full size (65536 rows, 4 partitions of 5
    one-column chunks, N = 32768 with 12 + 2 primes), relinearising after every product (eager)
    and once per result ciphertext (lazy): every limb of the 4 result ciphertexts equals the
    oracle's, and the result decrypts to the integer SpMV."""
    g, kg, o = _laplace_contexts(relin)
    w = W.laplace256()
    print("laplace256 full size, relin_mode %d" % relin, flush=True)
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64), True, kg, 31)
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    y = H.he_spmv(g, kg, M, x)
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], True, 31)
    assert M.info() == (OM.n_parts(), OM.n_chunks()) == (4, 20)
    oy, _ = OM.he_spmv(OM.encrypt_vector(w["v"], 41))
    assert np.array_equal(y.export_all(), oy)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


@pytest.mark.parametrize("relin", [0, 1], ids=["eager", "lazy"])
def test_laplace_full_ring_mixed_chunks(relin):
    """A 64 x 64-grid Laplacian on the same N = 32768 ring: one partition whose first chunk has four
    columns (totalSum rotations by 4096 and 8192 slots on the two-pass transforms) and whose
    second has one (lazy relinearisation applies to it alone): every result limb against the
    oracle."""
    g, kg, o = _laplace_contexts(relin)
    w = W.laplace256(n=64)
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64), True, kg, 32)
    OM = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], True, 32)
    assert [M.chunk(k)[2] for k in range(M.info()[1])] == [OM.chunk(k)[2] for k in range(OM.n_chunks())] == [4, 1]
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 42)
    y = H.he_spmv(g, kg, M, x)
    oy, _ = OM.he_spmv(OM.encrypt_vector(w["v"], 42))
    assert np.array_equal(y.export_all(), oy)


def test_laplace256_full_size():
    """The both-encrypted 5-point Laplacian on a 256 x 256 grid at N = 32768 (12 x 50-bit data
    primes, 2 special): keys sampled against the oracle, the decrypted result equal to the
    integer SpMV, and the first chunk's encryption and exact product + relinearisation against
    the oracle, limb for limb."""
    g, kg, o = _laplace_contexts(0)
    assert g.moduli() == o.moduli()
    assert np.array_equal(kg.export(0), o.sk_ntt())
    assert np.array_equal(kg.export(2, 3), o.ksk(3))
    assert np.array_equal(kg.export(3), o.ksk(-1))
    w = W.laplace256()
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64), True, kg, 31)
    nparts, nchunks = M.info()
    assert nparts == 4
    x = H.encrypt(g, kg, M, dev(w["v"], torch.int64), 41)
    y = H.he_spmv(g, kg, M, x)
    out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
    H.decrypt(g, kg, M, y, out)
    assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))
    # sampled limb parity: chunk 0 of partition 0 (matrix ciphertext, vector ciphertext, product)
    s = (1 << 15) // 2
    rp = w["row_ptr"][:s + 1]
    VA, CI, RM, CP = O.cssc(s, rp, w["col"][:rp[-1]], w["val"][:rp[-1]])
    ch = O.chunks(CP, s)
    start, c, h = ch[0]
    assert M.chunk(0) == (0, start, c, h)
    slots_a = np.zeros(1 << 15, np.int64)
    slots_v = np.zeros(1 << 15, np.int64)
    for b in range(c):
        col_ = start + b
        cnt = min(CP[col_ + 1] - CP[col_], h)
        slots_a[b * h:b * h + cnt] = VA[CP[col_]:CP[col_] + cnt]
        slots_v[b * h:b * h + cnt] = w["v"][CI[CP[col_]:CP[col_] + cnt]]
    ca = o.encrypt(o.encode(slots_a), 31, 0)
    cv = o.encrypt(o.encode(slots_v), 41, 0)
    assert np.array_equal(M.export(0, 0), ca)
    assert np.array_equal(x.export(0), cv)
    got = H.mul_ct(g, kg, H.CtVec.from_host(g, ca, 1), H.CtVec.from_host(g, cv, 1)).export(0)
    assert np.array_equal(got, o.ct_mul_ct(ca, cv))


def _serve_mix(budget, max_active, stagger_s):
    import time as _t
    p = TINY
    g, kg0, o = contexts(p)
    kgs = [kg0, g.keygen(9)]
    rng = np.random.default_rng(77)
    reqs = []
    for i, (R, nnz) in enumerate([(200, 900), (600, 3000), (50, 100), (300, 2000), (1000, 3000), (90, 400), (256, 2500), (700, 1400)]):
        rp, col, val = W.uniform_matrix(R, R, nnz, 15, rng)
        w = dict(R=R, C=R, row_ptr=rp, col=col, val=val, v=rng.integers(-15, 16, R))
        ks = kgs[i % 2]
        M, x = _pack_and_encrypt(g, ks, w, 300 + i)
        reqs.append((w, ks, M, x))
    srv = H.Server(g, budget, max_active)
    ids = []
    for w, ks, M, x in reqs:
        ids.append(srv.submit(ks, M, x))
        _t.sleep(stagger_s)
    outs = [srv.wait(i) for i in ids]
    stats = srv.stats()
    srv.close()
    for (w, ks, M, x), (y, times) in zip(reqs, outs):
        assert times[0] <= times[1] <= times[2]
        solo = H.he_spmv(g, ks, M, x)
        assert np.array_equal(y.export_all(), solo.export_all())
        out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
        H.decrypt(g, ks, M, y, out)
        assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))
    return stats


def test_server_results_equal_solo_in_the_mix():
    """Continuous batching: requests arriving while others run are admitted at the next tick and
    share rotation launches; each result equals the request's own hs_he_spmv, bit for bit."""
    stats = _serve_mix(64 << 30, 64, 0.0)
    assert stats["completed"] == 8 and stats["max_active"] >= 2


def test_server_staggered_arrivals():
    stats = _serve_mix(64 << 30, 64, 0.001)
    assert stats["completed"] == 8


def test_server_admission_by_footprint():
    """A budget below any two requests' footprint admits one request at a time."""
    stats = _serve_mix(1, 64, 0.0)
    assert stats["completed"] == 8 and stats["max_active"] == 1
    assert stats["held_by_budget"] >= 1 and stats["requests_waited"] >= 1 and stats["held_by_slots"] == 0
    stats = _serve_mix(64 << 30, 1, 0.0)   # one slot: requests wait for max_active instead
    assert stats["completed"] == 8 and stats["max_active"] == 1
    assert stats["held_by_slots"] >= 1 and stats["held_by_budget"] == 0
