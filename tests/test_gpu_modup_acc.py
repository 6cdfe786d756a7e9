"""GPU: ModUp + key inner product of the one-workgroup-per-limb key switch at N = 2^14 with the
accumulators in registers (HS_OPT_MODUP_ACC = 2, one workgroup per half of the target limb; 3, one
workgroup of 1024 threads per target limb) and in memory (1): rotations equal the oracle's under
all three, for one-prime and two-prime digits, at level sizes with six, two and one digit
groups."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402


@pytest.fixture
def one_wg():
    H.set_option(H.OPT_KS_PIPELINE, 1)
    yield
    H.set_option(H.OPT_KS_PIPELINE, 0)
    H.set_option(H.OPT_MODUP_ACC, 0)


@pytest.mark.parametrize("p", [(14, 6, 50, 1), (14, 4, 50, 2)], ids=["K1", "K2"])
def test_rotations_match_oracle_under_both_accumulator_forms(one_wg, p):
    g = H.Context(*p, agg_mode=0)
    o = O.Context(*p, agg_mode=0)
    kg = g.keygen(8)
    o.keygen(8)
    N = 1 << p[0]
    rng = np.random.default_rng(11)
    n_distinct = 4
    cts = [o.encrypt(rng.integers(0, 65537, N).astype(np.uint64), 9, i) for i in range(n_distinct)]
    want = {}
    for step in (1, 5):
        for i in range(n_distinct):
            want[step, i] = o.rotate(cts[i], step)
    for B in (3, 40, 80):   # digit groups per level: dnum, two, one (one-prime digits)
        idx = [i % n_distinct for i in range(B)]
        x = H.CtVec.from_host(g, np.concatenate([cts[i] for i in idx]), B)
        for mode in (1, 2, 3):
            H.set_option(H.OPT_MODUP_ACC, mode)
            for step in (1, 5):
                print("B=%d mode=%d step=%d" % (B, mode, step), flush=True)
                r = H.rotate(g, kg, x, step)
                for b in sorted({0, 1, B // 2, B - 1}):
                    assert np.array_equal(r.export(b), want[step, idx[b]]), (B, mode, step, b)
