"""CSR -> CSSC on the device (App. B) against the oracle's conversion, partition by partition:
the row map RM (descending nonzero count, ties in ascending row order), the column pointers CP
and the column-index array CI, bit for bit, on matrices that exercise the radix passes (a row of
70000 nonzeros needs three 8-bit passes), ragged and empty partitions, an empty matrix, and
malformed row pointers (rejected before any kernel reads through them)."""
import numpy as np
import pytest

import oracle as O
from paper_2603_04742_amd import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402

_ctx = {}


def ctx(logn=9, L=3, slot_rows=1):
    key = (logn, L, slot_rows)
    if key not in _ctx:
        _ctx[key] = H.Context(logn, L, 50, 1, agg_mode=0, slot_rows=slot_rows)
    return _ctx[key]


def dev(a, dtype):
    npd = {torch.int64: np.int64, torch.int32: np.int32}[dtype]
    return torch.from_numpy(np.ascontiguousarray(np.asarray(a).astype(npd))).cuda()


def csr_from_rows(R, C, rows, g):
    """CSR with row r holding rows[r] distinct ascending columns, values in [-7, 7]."""
    rp = np.zeros(R + 1, np.int64)
    rp[1:] = np.cumsum(rows)
    col = np.concatenate([np.sort(g.choice(C, size=k, replace=False)) if k else np.zeros(0, np.int64) for k in rows]).astype(np.int32)
    val = g.integers(-7, 8, size=int(rp[-1]))
    return dict(R=R, C=C, row_ptr=rp, col=col, val=val)


def check_structure(g, w):
    print("cssc %d x %d, nnz %d" % (w["R"], w["C"], int(w["row_ptr"][-1])), flush=True)
    M = H.Matrix(g, w["R"], w["C"], dev(w["row_ptr"], torch.int64), dev(w["col"], torch.int32), dev(w["val"], torch.int64))
    s = g.N // 2
    ci = []
    for part, r0 in enumerate(range(0, w["R"], s)):
        r1 = min(w["R"], r0 + s)
        rp = w["row_ptr"][r0:r1 + 1] - w["row_ptr"][r0]
        sl = slice(int(w["row_ptr"][r0]), int(w["row_ptr"][r1]))
        _, CI, RM, CP = O.cssc(r1 - r0, rp, w["col"][sl], w["val"][sl])
        grm, gcp = M.cssc(part)
        assert np.array_equal(grm, RM), ("RM", part)
        assert np.array_equal(gcp, CP), ("CP", part)
        ci.append(CI)
    want = np.concatenate(ci) if ci else np.zeros(0, np.int32)
    assert np.array_equal(M.column_index(), want)
    return M


def test_zipf16k_structure():
    check_structure(ctx(14, 6), W.zipf16k())


def test_ragged_partitions_and_empty_rows():
    """1300 rows on N = 512 (partitions of 256 rows, the last of 20), a third of the rows empty,
    ties everywhere (counts 0..6)."""
    g = np.random.default_rng(3)
    rows = g.integers(0, 7, size=1300)
    rows[g.random(1300) < 0.33] = 0
    check_structure(ctx(), csr_from_rows(1300, 900, rows, g))


def test_long_row_needs_three_radix_passes():
    """One row of 70000 nonzeros beside short rows: Lw = 70000 is a 17-bit key (three passes)."""
    g = np.random.default_rng(4)
    rows = g.integers(0, 4, size=300)
    rows[137] = 70000
    rows[5] = 300
    check_structure(ctx(), csr_from_rows(300, 70000, rows, g))


def test_empty_and_single_row_matrices():
    g = np.random.default_rng(5)
    check_structure(ctx(), csr_from_rows(300, 40, np.zeros(300, np.int64), g))
    check_structure(ctx(), csr_from_rows(1, 40, np.array([7]), g))


def test_two_slot_rows_keep_each_partitions_structure():
    """With two slot rows the CP arrays are padded to the joint width on the device; the
    partitions' own RM and CP are unchanged."""
    g = np.random.default_rng(6)
    rows = g.integers(0, 9, size=700)
    check_structure(ctx(slot_rows=2), csr_from_rows(700, 500, rows, g))


def test_malformed_row_pointers_rejected():
    g = ctx()
    bad = [np.array([1, 2, 3], np.int64),        # row_ptr[0] != 0
           np.array([0, 3, 2], np.int64)]        # decreasing
    for rp in bad:
        with pytest.raises(H.HespmvError) as e:
            H.Matrix(g, 2, 4, dev(rp, torch.int64), dev(np.array([0, 1, 2], np.int32), torch.int32), dev(np.array([1, 1, 1]), torch.int64))
        assert e.value.code == H.HS_EINVAL
    # the library stays usable
    check_structure(g, csr_from_rows(10, 10, np.arange(10) % 3, np.random.default_rng(7)))
