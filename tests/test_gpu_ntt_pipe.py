"""GPU: the software-pipelined forward transform of many N = 2^14 limbs (a persistent grid of two
workgroups per CU, each reading its next limb while it finishes the current one) against the oracle
and against the one-workgroup-per-limb kernel, bit for bit, through the C ABI."""
import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2603_04742_amd import hespmv as H  # noqa: E402


def test_pipelined_forward_ntt_matches_oracle_and_plain_kernel():
    logn, L, K = 14, 6, 1
    g = H.Context(logn, L, 50, K)
    o = O.Context(logn, L, 50, K)
    N, nl = 1 << logn, L + K
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    npoly = (4 * cus + 3) // nl + 3        # at least two limbs per workgroup of the grid, ragged tail
    rng = np.random.default_rng(5)
    mods = o.moduli()[:nl]
    x = np.stack([np.stack([rng.integers(0, q, N, dtype=np.uint64) for q in mods]) for _ in range(npoly)])
    base = torch.from_numpy(x.reshape(-1).view(np.int64)).cuda()
    outs = {}
    try:
        for opt in (0, 1):                 # 0: pipelined (automatic), 1: one workgroup per limb
            H.set_option(H.OPT_NTT_PIPE, opt)
            d = base.clone()
            H.profile(True)
            g.ntt(d, 0, nl, inverse=False)
            torch.cuda.synchronize()
            names = H.profile_summary()
            H.profile(False)
            assert ("k_ntt_fwd_pipe" in names) == (opt == 0), names
            outs[opt] = d.cpu().numpy().view(np.uint64).reshape(npoly, nl, N)
    finally:
        H.set_option(H.OPT_NTT_PIPE, 0)
    assert np.array_equal(outs[0], outs[1])
    for pi in (0, 1, npoly // 2, npoly - 1):   # first, a middle and the last limbs of the grid loop
        for m in range(nl):
            assert np.array_equal(outs[0][pi, m], o.ntt(m, x[pi, m])), (pi, m)


def test_forward_ntt_extreme_residues():
    """Residues at the top of [0, q) (all q - 1, alternating q - 1 and 0, a half of q - 1, values
    within 2^20 of q) through both forward kernels, whose LDS rounds use the 8-byte twiddle
    table: every checked limb equals the oracle's transform."""
    logn, L, K = 14, 6, 1
    g = H.Context(logn, L, 50, K)
    o = O.Context(logn, L, 50, K)
    N, nl = 1 << logn, L + K
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    npoly = (4 * cus + 3) // nl + 3
    rng = np.random.default_rng(9)
    mods = o.moduli()[:nl]

    def limb(p, q):
        q = np.uint64(q)
        kind = p % 4
        if kind == 0:
            return np.full(N, q - np.uint64(1), np.uint64)
        if kind == 1:
            return np.where(np.arange(N) % 2 == 0, q - np.uint64(1), np.uint64(0)).astype(np.uint64)
        if kind == 2:
            return np.where(np.arange(N) < N // 2, q - np.uint64(1), np.uint64(0)).astype(np.uint64)
        return q - np.uint64(1) - rng.integers(0, 1 << 20, N, dtype=np.uint64)

    x = np.stack([np.stack([limb(p, q) for q in mods]) for p in range(npoly)])
    base = torch.from_numpy(x.reshape(-1).view(np.int64)).cuda()
    try:
        for opt in (0, 1):
            H.set_option(H.OPT_NTT_PIPE, opt)
            d = base.clone()
            g.ntt(d, 0, nl, inverse=False)
            got = d.cpu().numpy().view(np.uint64).reshape(npoly, nl, N)
            for pi in (0, 1, 2, 3, npoly - 1):
                for m in (0, 3, nl - 1):
                    assert np.array_equal(got[pi, m], o.ntt(m, x[pi, m])), (opt, pi, m)
    finally:
        H.set_option(H.OPT_NTT_PIPE, 0)
