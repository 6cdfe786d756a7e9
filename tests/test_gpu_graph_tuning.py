"""GPU: the graph-recorded batch and the autotuner change launches only, never results.

A BatchPlan replay must reproduce the eager hs_he_spmv_batch result bit for bit on every replay
(with eager work and synchronisations in between, and after new vectors are copied into its
inputs), and every tuning table (transform variant x key-switch pipeline) must give the same
ciphertext limbs as the default launches.  Decrypted results are checked against the integer SpMV.
"""
import numpy as np
import pytest

from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402

SMALL = (12, 2, 30, 1, 1)  # the ring of the 256 x 256 workload: uniform aggregation, 30-bit primes
TINY = (9, 3, 50, 1, 0)
TINY11 = (11, 3, 50, 1, 0)
RING16K = (14, 6, 50, 1, 0)


def dev(a, dtype):
    npd = {torch.int64: np.int64, torch.int32: np.int32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(npd, copy=False))).cuda()


def fresh(p, seed=11):
    logn, L, bits, K, agg = p
    g = H.Context(logn, L, bits, K, agg_mode=agg)
    return g, g.keygen(seed)


def pack(g, w):
    return H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64))


def requests(g, kss, shapes, seed):
    rng = np.random.default_rng(seed)
    out = []
    for i, (R, C, nnz) in enumerate(shapes):
        rp, col, val = W.uniform_matrix(R, C, nnz, 7, rng)
        w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=rng.integers(-7, 8, C))
        ks = kss[i % len(kss)]
        M = pack(g, w)
        out.append([w, ks, M, H.encrypt(g, ks, M, dev(w["v"], torch.int64), 500 + i)])
    return out


def check_decrypt(g, reqs, ys):
    for (w, ks, M, _), y in zip(reqs, ys):
        out = torch.zeros(w["R"], dtype=torch.int64, device="cuda")
        H.decrypt(g, ks, M, y, out)
        assert np.array_equal(out.cpu().numpy(), W.spmv_mod_t(w))


@pytest.mark.parametrize("p", [TINY, SMALL, RING16K], ids=["tiny", "ring4096", "ring16k"])
def test_batch_plan_replays_match_eager(p):
    g, kg = fresh(p)
    kg2 = g.keygen(12)
    shapes = [(40, 30, 200), (10, 10, 0), (300, 300, 1500), (700, 200, 2000), (5, 80, 60)]
    if p == RING16K:
        shapes = [(2000, 2000, 9000), (9000, 4000, 20000), (64, 64, 300)]
    reqs = requests(g, [kg, kg2], shapes, 3)
    kss, ms, xs = [r[1] for r in reqs], [r[2] for r in reqs], [r[3] for r in reqs]
    eager = [y.export_all() for y in H.he_spmv_batch(g, kss, ms, xs)]
    plan = H.BatchPlan(g, kss, ms, xs)
    outs = plan.outputs()
    for y, e in zip(outs, eager):  # the eager pass made at construction
        assert np.array_equal(y.export_all(), e)
    for rep in range(3):
        # eager work of the program between replays
        solo = H.he_spmv(g, kss[0], ms[0], xs[0])
        torch.cuda.synchronize()
        plan.run()
        torch.cuda.synchronize()
        for y, e in zip(outs, eager):
            assert np.array_equal(y.export_all(), e), "replay %d differs from the eager batch" % rep
        assert np.array_equal(solo.export_all(), eager[0])
    check_decrypt(g, reqs, outs)
    # new vectors copied into the plan's inputs
    rng = np.random.default_rng(99)
    for i, r in enumerate(reqs):
        r[0] = dict(r[0], v=rng.integers(-7, 8, r[0]["C"]))
        xs[i].copy_from(H.encrypt(g, r[1], r[2], dev(r[0]["v"], torch.int64), 900 + i))
    plan.run()
    torch.cuda.synchronize()
    eager2 = [y.export_all() for y in H.he_spmv_batch(g, kss, ms, xs)]
    for y, e in zip(outs, eager2):
        assert np.array_equal(y.export_all(), e)
    check_decrypt(g, reqs, outs)
    plan.close()


def test_batch_plan_rejects_encrypted_matrix():
    g, kg = fresh((10, 3, 50, 1, 0))
    rng = np.random.default_rng(5)
    rp, col, val = W.uniform_matrix(20, 20, 60, 3, rng)
    M = H.Matrix(g, 20, 20, dev(rp, torch.int64), dev(col, torch.int32), dev(val, torch.int64), True, kg, 3)
    x = H.encrypt(g, kg, M, dev(rng.integers(-3, 4, 20), torch.int64), 4)
    with pytest.raises(H.HespmvError):
        H.BatchPlan(g, [kg], [M], [x])


@pytest.mark.parametrize("p", [TINY11, SMALL, RING16K], ids=["ring2048", "ring4096", "ring16k"])
def test_autotune_and_every_tuning_give_identical_limbs(p):
    g, kg = fresh(p)
    shapes = [(9000, 4000, 20000), (64, 64, 300)] if p == RING16K else [(300, 300, 1500), (700, 200, 2000)]
    reqs = requests(g, [kg], shapes, 8)
    kss, ms, xs = [r[1] for r in reqs], [r[2] for r in reqs], [r[3] for r in reqs]
    ref = [y.export_all() for y in H.he_spmv_batch(g, kss, ms, xs)]
    rep = H.autotune(g, kg)
    assert rep["variant"] in (0, 1)
    assert [b for b, _, _ in rep["pipelines"]] == [1, 2, 4, 8, 16, 32, 64]
    assert all(t2 > 0 for _, _, t2 in rep["pipelines"])
    tab = H.tuning(g)
    assert tab[0] == rep["variant"] and tab[1] == rep["ntt_variant"] and all(v in (0, 1) for v in tab[2:])
    for y, e in zip(H.he_spmv_batch(g, kss, ms, xs), ref):
        assert np.array_equal(y.export_all(), e)
    for variant in (0, 1):
        for pick in (0, 1):
            H.set_tuning(g, [variant, 1 - variant] + [pick] * 8)
            for y, e in zip(H.he_spmv_batch(g, kss, ms, xs), ref):
                assert np.array_equal(y.export_all(), e), "variant %d pipeline %d" % (variant, pick)
            # the standalone transform under this variant round-trips
            lim = torch.randint(0, min(g.moduli()[: p[1]]), (3, p[1], 1 << p[0]), dtype=torch.int64, device="cuda")
            back = lim.clone()
            g.ntt(back, 0, p[1])
            g.ntt(back, 0, p[1], inverse=True)
            assert torch.equal(back, lim)
    check_decrypt(g, reqs, H.he_spmv_batch(g, kss, ms, xs))
    with pytest.raises(H.HespmvError):
        H.set_tuning(g, [2, 0] + [0] * 8)


@pytest.mark.parametrize("p", [TINY11, SMALL, RING16K, (10, 3, 50, 2, 0)], ids=["ring2048", "ring4096", "ring16k", "two_prime_digits"])
def test_modup_grouping_gives_identical_limbs(p):
    """The two-pass ModUp with one, two or three targets per workgroup computes the same limbs."""
    g, kg = fresh(p)
    shapes = [(9000, 4000, 20000), (64, 64, 300)] if p == RING16K else [(300, 300, 1500), (700, 200, 2000)]
    reqs = requests(g, [kg], shapes, 9)
    kss, ms, xs = [r[1] for r in reqs], [r[2] for r in reqs], [r[3] for r in reqs]
    H.set_option(H.OPT_KS_PIPELINE, 2)
    try:
        ref = [y.export_all() for y in H.he_spmv_batch(g, kss, ms, xs)]
        for tg in (2, 3, 1, 0):
            H.set_option(H.OPT_MODUP_GROUP, tg)
            for y, e in zip(H.he_spmv_batch(g, kss, ms, xs), ref):
                assert np.array_equal(y.export_all(), e), "targets per workgroup %d" % tg
        check_decrypt(g, reqs, H.he_spmv_batch(g, kss, ms, xs))
    finally:
        H.set_option(H.OPT_MODUP_GROUP, 0)
        H.set_option(H.OPT_KS_PIPELINE, 0)
