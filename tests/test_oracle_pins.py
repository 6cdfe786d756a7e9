"""Pins of the CPU oracle against facts fixed by the paper and by mathematics (no GPU).

Each test checks the oracle against something other than itself: values printed in the paper
(tests/golden), published test vectors, closed forms, direct definitions evaluated with Python
big integers, brute force on tiny inputs, and invariants.  A plausible slip in the oracle (a
dropped term, a wrong sign or index, a transposed operand) fails at least one of them.
"""
import collections
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2603_04742_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")
T = 65537


# ----------------------------------------------------------------- independent helpers
def mr_prime(n):
    if n < 2:
        return False
    for p in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def bitrev(x, bits):
    return int(format(x, "0%db" % bits)[::-1], 2) if bits else 0


def negacyclic(a, b, q):
    n = len(a)
    out = [0] * n
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n):
            k = i + j
            if k < n:
                out[k] = (out[k] + a[i] * b[j]) % q
            else:
                out[k - n] = (out[k - n] - a[i] * b[j]) % q
    return out


def coeff_automorph(a, g, q):
    n = len(a)
    out = [0] * n
    for i, v in enumerate(a):
        e = g * i % (2 * n)
        if e < n:
            out[e] = (out[e] + v) % q
        else:
            out[e - n] = (out[e - n] - v) % q
    return out


# ----------------------------------------------------------------- arithmetic and primes
def test_mulmod_matches_python_ints():
    g = np.random.default_rng(1)
    for q in (1125899904679937, 1073692673, (1 << 61) - 1, 65537):
        for _ in range(300):
            a, b = int(g.integers(0, q)), int(g.integers(0, q))
            assert O.lib().orc_mulmod(a, b, q) == a * b % q


@pytest.mark.parametrize("logn,L,K,bits", [(12, 2, 1, 30), (14, 6, 1, 50), (15, 12, 2, 50)])
def test_primes_are_the_largest_ntt_friendly_ones(logn, L, K, bits):
    c = O.Context(logn, L, bits, K)
    N = 1 << logn
    mods = c.moduli()
    # independent downward scan with its own primality test
    want, q = [], ((1 << bits) - 1) // (2 * N) * (2 * N) + 1
    while len(want) < len(mods):
        if q < (1 << bits) and mr_prime(q):
            want.append(q)
        q -= 2 * N
    special, data, aux = want[:K], want[K:K + L], want[K + L:]
    assert mods[:L] == data and mods[L:L + K] == special and mods[L + K:] == aux
    # the tensor basis is large enough for exact ct x ct products: prod > 4 N Q^2
    Q = math.prod(data)
    assert math.prod(mods) > 4 * N * Q * Q
    assert math.prod(mods[:-1]) <= 4 * N * Q * Q or c.n_aux() == 0


@pytest.mark.parametrize("logn,bits", [(4, 30), (12, 30), (14, 50)])
def test_psi_is_the_smallest_primitive_2n_th_root(logn, bits):
    c = O.Context(logn, 2, bits, 1)
    N = 1 << logn
    for m, q in enumerate(c.moduli()[:3]):
        psi = c.psi(m)
        assert pow(psi, N, q) == q - 1
        roots = [pow(psi, 2 * k + 1, q) for k in range(N)]
        assert psi == min(roots)
        assert len(set(roots)) == N
    z = c.psi(-1)  # plaintext modulus
    assert pow(z, N, T) == T - 1 and z == min(pow(z, 2 * k + 1, T) for k in range(N))


# ----------------------------------------------------------------- NTT
@pytest.mark.parametrize("logn", [3, 4, 6])
def test_ntt_is_evaluation_at_odd_powers_in_bitreversed_order(logn):
    c = O.Context(logn, 2, 30, 1)
    N = 1 << logn
    g = np.random.default_rng(logn)
    for m, q in enumerate(c.moduli()[:3]):
        psi = c.psi(m)
        a = [int(x) for x in g.integers(0, q, N)]
        A = c.ntt(m, a)
        for k in range(N):
            e = 2 * bitrev(k, logn) + 1
            assert int(A[k]) == sum(a[i] * pow(psi, e * i, q) for i in range(N)) % q
        assert [int(x) for x in c.intt(m, A)] == a


def test_ntt_product_is_negacyclic_convolution():
    c = O.Context(6, 2, 30, 1)
    g = np.random.default_rng(5)
    for m, q in enumerate(c.moduli()[:2]):
        a = g.integers(0, q, 64)
        b = g.integers(0, q, 64)
        A, B = c.ntt(m, a), c.ntt(m, b)
        prod = np.array([int(x) * int(y) % q for x, y in zip(A, B)], np.uint64)
        got = [int(x) for x in c.intt(m, prod)]
        assert got == negacyclic([int(x) for x in a], [int(x) for x in b], q)


def test_ntt_roundtrip_full_size():
    c = O.Context(14, 6, 50, 1)
    g = np.random.default_rng(7)
    for m, q in enumerate(c.moduli()):
        a = g.integers(0, q, 1 << 14, dtype=np.uint64)
        assert np.array_equal(c.intt(m, c.ntt(m, a)), a)


# ----------------------------------------------------------------- randomness
def test_chacha20_rfc8439_vectors():
    n = 0
    for line in open(os.path.join(GOLD, "chacha20_rfc8439.txt")):
        if not line.strip() or line.startswith("#"):
            continue
        key, ctr, nonce, out = [p.split() for p in line.split("|")]
        got = O.chacha20_block([int(x, 16) for x in key], int(ctr[0]), [int(x, 16) for x in nonce])
        assert [int(x) for x in got] == [int(x, 16) for x in out]
        n += 1
    assert n == 2


def test_cdt_table_closed_form_and_shape():
    tab = [int(x) for x in O.cdt()]
    assert tab[-1] == 1 << 63 and all(a < b for a, b in zip(tab, tab[1:]))
    rho = [math.exp(-j * j / (2 * 3.2 * 3.2)) for j in range(20)]
    S = rho[0] + 2 * sum(rho[1:])
    acc = 0.0
    for k in range(19):
        acc += rho[k] if k == 0 else 2 * rho[k]
        assert abs(tab[k] / 2.0 ** 63 - acc / S) < 1e-12


def test_samplers_statistics():
    n = 1 << 17
    e = O.sample(11, 3, 0, n, 1)
    assert abs(e.mean()) < 0.05 and abs(e.var() - 3.2 ** 2) < 0.15 and np.abs(e).max() <= 19
    assert abs((e == 0).mean() - 1 / (math.sqrt(2 * math.pi) * 3.2)) < 0.005
    s = O.sample(11, 1, 0, n, 0)
    assert set(np.unique(s)) == {-1, 0, 1} and all(abs((s == v).mean() - 1 / 3) < 0.01 for v in (-1, 0, 1))
    q = 1125899904679937
    u = O.sample(11, 2, 0, n, 2, q).astype(np.uint64)
    assert int(u.max()) < q and abs(u.astype(np.float64).mean() / q - 0.5) < 0.01
    # distinct (purpose, index) give independent streams; same ones repeat
    assert not np.array_equal(O.sample(11, 3, 0, 64, 1), O.sample(11, 3, 1, 64, 1))
    assert np.array_equal(O.sample(11, 3, 5, 64, 1), O.sample(11, 3, 5, 64, 1))


# ----------------------------------------------------------------- batch encoding (slots)
def slot_exponents(N):
    e = [pow(3, j, 2 * N) for j in range(N // 2)]
    return e + [(2 * N - x) % (2 * N) for x in e]


@pytest.mark.parametrize("logn", [3, 5])
def test_decode_is_evaluation_at_slot_roots(logn):
    c = O.Context(logn, 2, 30, 1)
    N = 1 << logn
    z = c.psi(-1)
    g = np.random.default_rng(3)
    m = [int(x) for x in g.integers(0, T, N)]
    got = [int(x) for x in c.decode(np.array(m, np.uint64))]
    for j, e in enumerate(slot_exponents(N)):
        assert got[j] == sum(m[i] * pow(z, e * i, T) for i in range(N)) % T
    slots = g.integers(0, T, N)
    assert np.array_equal(c.decode(c.encode(slots)), slots.astype(np.uint64))


def test_encode_is_multiplicative():
    c = O.Context(6, 2, 30, 1)
    g = np.random.default_rng(4)
    x, y = g.integers(0, T, 64), g.integers(0, T, 64)
    mx, my = c.encode(x), c.encode(y)
    prod = negacyclic([int(v) for v in mx], [int(v) for v in my], T)
    assert np.array_equal(c.decode(np.array(prod, np.uint64)), (x * y) % T)


@pytest.mark.parametrize("k", [1, 2, 5, 13])
def test_galois_3k_rotates_rows_left(k):
    c = O.Context(5, 2, 30, 1)
    N, h = 32, 16
    x = np.arange(N) * 7 % T
    m = [int(v) for v in c.encode(x)]
    rot = c.decode(np.array(coeff_automorph(m, pow(3, k, 2 * N), T), np.uint64))
    want = np.concatenate([np.roll(x[:h], -k), np.roll(x[h:], -k)])
    assert np.array_equal(rot, want)


# ----------------------------------------------------------------- encryption
def small_ctx(agg_mode=0, logn=6, L=2, bits=30, K=1, seed=77):
    c = O.Context(logn, L, bits, K, agg_mode=agg_mode)
    c.keygen(seed)
    return c


def phase_python(c, ct):
    """[c0 + c1 s]_Q as exact integers, from the exported secret key (schoolbook products)."""
    N, L = c.N, c.L
    qs = c.moduli()[:L]
    s = [int(v) for v in c.sk()]
    res = []
    for i, q in enumerate(qs):
        c0 = [int(v) for v in c.intt(i, ct[i * N:(i + 1) * N])]
        c1 = [int(v) for v in c.intt(i, ct[(L + i) * N:(L + i + 1) * N])]
        prod = negacyclic(c1, [v % q for v in s], q)
        res.append([(a + b) % q for a, b in zip(c0, prod)])
    Q = math.prod(qs)
    xs = []
    for k in range(N):
        x = 0
        for i, q in enumerate(qs):
            Qi = Q // q
            x += res[i][k] * pow(Qi, -1, q) * Qi
        xs.append(x % Q)
    return xs, Q


def test_encrypt_decrypt_against_big_integer_definition():
    c = small_ctx()
    g = np.random.default_rng(9)
    m = g.integers(0, T, c.N).astype(np.uint64)
    ct = c.encrypt(m, 1234, 0)
    xs, Q = phase_python(c, ct)
    for k in range(c.N):
        assert (T * xs[k] * 2 + Q) // (2 * Q) % T == int(m[k])
        # noise: x - round(Q m / t) is small (fresh encryption, sigma = 3.2, N = 64)
        d = (xs[k] - (Q * int(m[k]) * 2 + T) // (2 * T)) % Q
        d = d - Q if d > Q // 2 else d
        assert abs(d) < 2 ** 12
    assert np.array_equal(c.decrypt(ct), m)


def test_public_key_relation():
    c = small_ctx()
    N, L = c.N, c.L
    pk = c.pk()
    s = [int(v) for v in c.sk()]
    for i, q in enumerate(c.moduli()[:L]):
        b = [int(v) for v in c.intt(i, pk[i * N:(i + 1) * N])]
        a = [int(v) for v in c.intt(i, pk[(L + i) * N:(L + i + 1) * N])]
        e = [(x + y) % q for x, y in zip(b, negacyclic(a, [v % q for v in s], q))]
        e = [v - q if v > q // 2 else v for v in e]
        assert max(abs(v) for v in e) <= 19


def test_homomorphic_add_cmult_rotate_keyswitch():
    c = small_ctx(logn=7, L=3, bits=50, K=1)
    N, h = c.N, c.N // 2
    g = np.random.default_rng(2)
    x, y = g.integers(0, T, N), g.integers(0, T, N)
    cx, cy = c.encrypt(c.encode(x), 5, 0), c.encrypt(c.encode(y), 5, 1)
    # HE-Add
    s = (cx.astype(object) + cy.astype(object))
    mods = c.moduli()
    qv = np.repeat(np.array(mods[:c.L] * 2, dtype=object), N)
    s = np.array([int(a) % int(q) for a, q in zip(s, qv)], np.uint64)
    assert np.array_equal(c.decode(c.decrypt(s)), (x + y) % T)
    # HE-CMult
    prod = c.ct_mul_plain(cx, c.plain_ntt(c.encode(y)))
    assert np.array_equal(c.decode(c.decrypt(prod)), (x * y) % T)
    # HE-Rot: left rotation within each row of N/2 slots, for several amounts
    for k in (1, 3, 6, 37, h - 1):
        r = c.rotate(cx, k)
        want = np.concatenate([np.roll(x[:h], -k), np.roll(x[h:], -k)])
        assert np.array_equal(c.decode(c.decrypt(r)), want)
    # key switching alone: c0' + KS(c1') decrypts like (c0, c1) under the rotated key s'
    gelt = c.galois_elt(2)
    a0 = c.automorph_ntt(cx[:c.L * N], gelt)
    a1 = c.automorph_ntt(cx[c.L * N:], gelt)
    ks = c.keyswitch(a1, 2)
    out = np.concatenate([(a0.astype(object) + ks[:c.L * N].astype(object)), ks[c.L * N:].astype(object)])
    out = np.array([int(a) % int(q) for a, q in zip(out, qv)], np.uint64)
    assert np.array_equal(out, c.rotate(cx, 4))


def test_exact_step_rotation_keys():
    """Sec. 2.1 HE-Rot with a key for the whole step: one key switch whose key satisfies
    b + a s = e + P sigma_g(s) on its digit (g = 3^k mod 2N, e small), and whose rotation decrypts
    to the slot rows rotated left by k; power-of-two steps and 0 get no extra key."""
    c = small_ctx(logn=6, L=2, bits=30, K=1)
    N, h, L, K = c.N, c.N // 2, c.L, c.K
    c.add_step_keys([3, 5, -1, 4, 0, 3, h + 6])
    assert c.step_key(4) is None and c.step_key(0) is None and c.step_key(7) is None
    mods = c.moduli()
    P = math.prod(mods[L:L + K])
    s = [int(v) for v in c.sk()]
    for k in (3, 5, h - 1, 6):
        key = c.step_key(k).reshape(2, c.dnum, L + K, N)
        sp = coeff_automorph(s, pow(3, k, 2 * N), 2 ** 62)
        sp = [v - 2 ** 62 if v > 2 ** 61 else v for v in sp]
        for j in range(c.dnum):
            for m in range(L + K):
                q = mods[m]
                b = [int(v) for v in c.intt(m, key[0, j, m].copy())]
                a = [int(v) for v in c.intt(m, key[1, j, m].copy())]
                e = [(x + y) % q for x, y in zip(b, negacyclic(a, [v % q for v in s], q))]
                if m < L and m // K == j:  # digits of K data primes
                    e = [(x - P * v) % q for x, v in zip(e, sp)]
                e = [v - q if v > q // 2 else v for v in e]
                assert max(abs(v) for v in e) <= 19, (k, j, m)
    g = np.random.default_rng(21)
    x = g.integers(0, T, N)
    cx = c.encrypt(c.encode(x), 8, 0)
    for k in (3, 5, h - 1, 6, 7):
        want = np.concatenate([np.roll(x[:h], -k), np.roll(x[h:], -k)])
        assert np.array_equal(c.decode(c.decrypt(c.rotate(cx, k))), want), k


def test_rotation_keys_both_directions():
    """Power-of-two rotation keys (Sec. 5): key index i < log2 N - 1 has Galois element 3^(2^i)
    mod 2N; the optional right keys, index log2 N - 1 + i, the inverse of 3^(2^i).  Each key holds
    b + a s = e + P sigma_g(s) on its digit, and one key switch with a right key rotates the slot
    rows right by 2^i."""
    c = small_ctx(logn=6, L=2, bits=30, K=1)
    N, h, L, K = c.N, c.N // 2, c.L, c.K
    nl = c.logn - 1
    with pytest.raises(IndexError):
        c.ksk(nl)
    c.add_right_rotation_keys()
    c.add_right_rotation_keys()   # a second call adds nothing
    mods = c.moduli()
    P = math.prod(mods[L:L + K])
    s = [int(v) for v in c.sk()]
    for idx in (0, 2, nl - 1, nl, nl + 1, 2 * nl - 1):
        g = c.galois_elt(idx)
        want = pow(3, 1 << idx, 2 * N) if idx < nl else pow(pow(3, 1 << (idx - nl), 2 * N), -1, 2 * N)
        assert g == want, idx
        key = c.ksk(idx).reshape(2, c.dnum, L + K, N)
        sp = coeff_automorph(s, g, 2 ** 62)
        sp = [v - 2 ** 62 if v > 2 ** 61 else v for v in sp]
        for j in range(c.dnum):
            for m in range(L + K):
                q = mods[m]
                b = [int(v) for v in c.intt(m, key[0, j, m].copy())]
                a = [int(v) for v in c.intt(m, key[1, j, m].copy())]
                e = [(x + y) % q for x, y in zip(b, negacyclic(a, [v % q for v in s], q))]
                if m < L and m // K == j:
                    e = [(x - P * v) % q for x, v in zip(e, sp)]
                e = [v - q if v > q // 2 else v for v in e]
                assert max(abs(v) for v in e) <= 19, (idx, j, m)
    with pytest.raises(IndexError):
        c.ksk(2 * nl)
    g = np.random.default_rng(4)
    x = g.integers(0, T, N)
    cx = c.encrypt(c.encode(x), 6, 0)
    qv = np.repeat(np.array(mods[:L] * 2, dtype=object), N)
    for i in (0, 3):
        gelt = c.galois_elt(nl + i)
        a0 = c.automorph_ntt(cx[:L * N], gelt)
        ks = c.keyswitch(c.automorph_ntt(cx[L * N:], gelt), nl + i)
        out = np.concatenate([a0.astype(object) + ks[:L * N].astype(object), ks[L * N:].astype(object)])
        out = np.array([int(a) % int(q) for a, q in zip(out, qv)], np.uint64)
        assert np.array_equal(out, c.rotate(cx, h - (1 << i))), i
        want = np.concatenate([np.roll(x[:h], 1 << i), np.roll(x[h:], 1 << i)])
        assert np.array_equal(c.decode(c.decrypt(out)), want), i


@pytest.mark.parametrize("logn", [6, 9])
def test_rotation_digits_fewest_key_switches(logn):
    """Left keys only (the paper reading): a rotation by k applies the binary digits of k, lowest
    first.  With the right keys: signed powers of two below N/2, lowest first, that sum to k mod N/2
    with no two at adjacent positions (the non-adjacent form), and no sequence of power-of-two keys
    in either direction reaches k in fewer key switches (breadth-first search over the N/2 slot-row
    rotations)."""
    c = small_ctx(logn=logn, L=2, bits=30, K=1)
    h = c.N // 2
    for k in range(h):
        assert c.rotation_digits(k) == [1 << i for i in range(logn - 1) if (k >> i) & 1], k
    c.add_right_rotation_keys()
    gens = [1 << i for i in range(logn - 1)] + [-(1 << i) for i in range(logn - 1)]
    dist = {0: 0}
    frontier = [0]
    while frontier:
        nxt = []
        for v in frontier:
            for s_ in gens:
                w = (v + s_) % h
                if w not in dist:
                    dist[w] = dist[v] + 1
                    nxt.append(w)
        frontier = nxt
    for k in range(h):
        d = c.rotation_digits(k)
        assert sum(d) % h == k, k
        assert all(v in gens for v in d), k
        pos = [abs(v).bit_length() - 1 for v in d]
        assert all(b - a >= 2 for a, b in zip(pos, pos[1:])), (k, d)
        assert len(d) == dist[k], (k, d, dist[k])
    assert c.rotation_digits(h - 1) == [-1] and c.rotation_digits(3) == [-1, 4] and c.rotation_digits(0) == []


@pytest.mark.parametrize("right", [False, True])
def test_rotation_by_every_amount_decrypts(right):
    """Every left rotation amount at N = 64 (binary digits with left keys; signed digits of the
    non-adjacent form with the right keys too) decrypts to the slot rows rotated left by k."""
    c = small_ctx(logn=6, L=2, bits=30, K=1)
    if right:
        c.add_right_rotation_keys()
    N, h = c.N, c.N // 2
    g = np.random.default_rng(12)
    x = g.integers(0, T, N)
    cx = c.encrypt(c.encode(x), 9, 0)
    for k in range(h):
        want = np.concatenate([np.roll(x[:h], -k), np.roll(x[h:], -k)])
        assert np.array_equal(c.decode(c.decrypt(c.rotate(cx, k))), want), k


def test_total_sum_steps_follow_the_recurrence():
    c = small_ctx(logn=8)
    h = c.N // 2
    for r, cc in ((5, 6), (3, 1), (7, 13), (1, 16), (40, 5)):
        steps, e = [], 1
        for j in range(cc.bit_length() - 2, -1, -1):
            steps.append(e * r % h)
            e *= 2
            if (cc >> j) & 1:
                steps.append(r % h)
                e += 1
        assert c.total_sum_steps(r, cc) == steps
    assert c.total_sum_steps(5, 6) == [5, 5, 15]


def test_ct_times_ct_with_relinearisation():
    c = small_ctx(logn=6, L=3, bits=50, K=1)
    g = np.random.default_rng(8)
    x, y = g.integers(-50, 50, c.N), g.integers(-50, 50, c.N)
    cx, cy = c.encrypt(c.encode(x), 3, 0), c.encrypt(c.encode(y), 3, 1)
    p = c.ct_mul_ct(cx, cy)
    assert np.array_equal(c.decode(c.decrypt(p)), (x * y) % T)
    assert c.noise_log2(p, c.encode((x * y) % T)) < math.log2(math.prod(c.moduli()[:3]) / (2 * T)) - 20
    # and a ct x ct product followed by a mask multiply (depth 1M + 1C)
    mask = np.zeros(c.N, np.int64)
    mask[:10] = 1
    pm = c.ct_mul_plain(p, c.plain_ntt(c.encode(mask)))
    assert np.array_equal(c.decode(c.decrypt(pm)), (x * y * mask) % T)


@pytest.mark.parametrize("agg", [0, 1])
@pytest.mark.parametrize("kind", ["laplace", "mixed"])
def test_lazy_relinearisation_protocol(kind, agg):
    """Both-encrypted SpMV with lazy relinearisation: the decrypted product is the integer SpMV.
    A group's limbs equal those of relinearising after every product when it has no one-column
    chunk, or a single one and no mask (then the same key switch of the same d2 is added); they
    differ when several one-column products are summed, or masked, before their key switch (the
    key switch is not linear in the limbs), which shows the lazy sum ran."""
    eager = O.Context(8, 3, 50, 1, agg_mode=agg)
    lazy = O.Context(8, 3, 50, 1, agg_mode=agg, lazy_relin=1)
    eager.keygen(3)
    lazy.keygen(3)
    if kind == "laplace":
        w = W.laplace256(n=10)   # 100 x 100: every chunk one column wide
        w["v"] = w["v"][:100]
    else:
        g = np.random.default_rng(77)
        rp, col, val = W.uniform_matrix(150, 90, 500, 7, g)   # chunks of one and of several columns
        w = dict(R=150, C=90, row_ptr=rp, col=col, val=val, v=g.integers(-7, 8, 90))
    runs = []
    for c in (eager, lazy):
        M = O.Matrix(c, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], True, 31)
        res, stats = M.he_spmv(M.encrypt_vector(w["v"], 41))
        assert np.array_equal(M.decrypt_result(res), W.spmv_mod_t(w))
        runs.append((M, res))
    M = runs[0][0]
    cs = [M.chunk(k) for k in range(M.n_chunks())]
    n1 = collections.Counter(k[0] for k in cs if k[2] == 1)
    if kind == "mixed":
        assert any(k[2] > 1 for k in cs) and n1
    ct = lazy.ct_size()
    for gi in range(M.n_groups()):
        same = np.array_equal(runs[0][1][gi * ct:(gi + 1) * ct], runs[1][1][gi * ct:(gi + 1) * ct])
        assert same == (n1[gi] == 0 or (n1[gi] == 1 and agg == 1)), gi


def test_ct_times_ct_exact_tensor_definition_tiny():
    """The scaled tensor round(t/Q * c (x) d) of centered lifts, computed with Python integers at
    N = 8, equals the oracle's product before relinearisation, checked through decryption with
    the s^2 term (a relinearisation-free decryption of the 3-component product)."""
    c = small_ctx(logn=3, L=2, bits=30, K=1)
    N, L = c.N, c.L
    qs = c.moduli()[:L]
    Q = math.prod(qs)
    g = np.random.default_rng(1)
    x, y = g.integers(0, T, N), g.integers(0, T, N)
    cx, cy = c.encrypt(c.encode(x), 4, 0), c.encrypt(c.encode(y), 4, 1)

    def lift(ct, p):
        limbs = [[int(v) for v in c.intt(i, ct[(p * L + i) * N:(p * L + i + 1) * N])] for i in range(L)]
        out = []
        for k in range(N):
            v = sum(limbs[i][k] * pow(Q // q, -1, q) * (Q // q) for i, q in enumerate(qs)) % Q
            out.append(v - Q if v > Q // 2 else v)
        return out

    def negint(a, b):
        n = len(a)
        o = [0] * n
        for i in range(n):
            for j in range(n):
                if i + j < n:
                    o[i + j] += a[i] * b[j]
                else:
                    o[i + j - n] -= a[i] * b[j]
        return o

    c0, c1, d0, d1 = lift(cx, 0), lift(cx, 1), lift(cy, 0), lift(cy, 1)

    def sr(v):  # round(t v / Q), symmetric (no ties: t, Q odd)
        return (2 * T * v + Q) // (2 * Q) if v >= 0 else -((2 * T * (-v) + Q) // (2 * Q))

    e0 = [sr(v) for v in negint(c0, d0)]
    e1 = [sr(a + b) for a, b in zip(negint(c0, d1), negint(c1, d0))]
    e2 = [sr(v) for v in negint(c1, d1)]
    s = [int(v) for v in c.sk()]
    s2 = negint(s, s)
    ph = [(a + b + cc) % Q for a, b, cc in zip(e0, negint(e1, s), negint(e2, s2))]
    m = [(2 * T * v + Q) // (2 * Q) % T for v in ph]
    assert np.array_equal(c.decode(np.array(m, np.uint64)), (x * y) % T)
    # the oracle (with relinearisation) decrypts to the same plaintext
    assert np.array_equal(c.decrypt(c.ct_mul_ct(cx, cy)), np.array(m, np.uint64))


def _negint(a, b):
    """Exact integer negacyclic product in Z[X]/(X^n + 1) (schoolbook)."""
    n = len(a)
    o = [0] * n
    for i in range(n):
        if a[i] == 0:
            continue
        for j in range(n):
            if i + j < n:
                o[i + j] += a[i] * b[j]
            else:
                o[i + j - n] -= a[i] * b[j]
    return o


@pytest.mark.parametrize("logn,L,bits,K", [(3, 2, 30, 1), (3, 3, 30, 2), (4, 2, 50, 1), (4, 3, 50, 1),
                                           (4, 3, 50, 2), (3, 2, 50, 2)])
def test_ct_tensor_limbs_equal_the_scaled_exact_product(logn, L, bits, K):
    """Sec. 2.1 HE-Mult, limb by limb: every residue of the oracle's three-component product equals
    [round(t/Q * (c0 d0, c0 d1 + c1 d0, c1 d1))]_{q_i}, where the c's and d's are the centered lifts
    of the inputs (coefficients in (-Q/2, Q/2]), the products are exact integer negacyclic
    convolutions and the rounding is to the nearest integer (t, Q odd: no ties).  Inputs are
    uniform residues, so about half of every polynomial's coefficients lift to negative values and
    the scaled products take both signs; a floor in place of the rounding, a non-centered lift or a
    swapped cross term changes limbs here."""
    c = O.Context(logn, L, bits, K)
    N = c.N
    qs = c.moduli()[:L]
    Q = math.prod(qs)
    g = np.random.default_rng(1000 * logn + 10 * L + K)
    coef = [[int.from_bytes(g.bytes(32), "little") % Q for _ in range(N)] for _ in range(4)]
    # a few coefficients at the edges of the lift: 0, (Q-1)/2 (positive), (Q+1)/2 and Q - 1 (negative)
    coef[0][:4] = [0, (Q - 1) // 2, (Q + 1) // 2, Q - 1]

    def to_ct(p0, p1):   # two coefficient-form polynomials -> [2][L][N] NTT form (pinned transform)
        out = []
        for poly in (p0, p1):
            for i, q in enumerate(qs):
                out.append(c.ntt(i, np.array([v % q for v in poly], np.uint64)))
        return np.concatenate(out)

    x, y = to_ct(coef[0], coef[1]), to_ct(coef[2], coef[3])
    got = c.ct_tensor(x, y).reshape(3, L, N)
    lift = [[v - Q if v > Q // 2 else v for v in poly] for poly in coef]
    c0, c1, d0, d1 = lift

    def sr(v):
        return (2 * T * v + Q) // (2 * Q) if v >= 0 else -((2 * T * (-v) + Q) // (2 * Q))

    want = [[sr(v) for v in _negint(c0, d0)],
            [sr(a + b) for a, b in zip(_negint(c0, d1), _negint(c1, d0))],
            [sr(v) for v in _negint(c1, d1)]]
    for w in range(3):
        for i, q in enumerate(qs):
            coeff = [int(v) for v in c.intt(i, got[w, i].copy())]
            assert coeff == [v % q for v in want[w]], (w, i)


def test_ct_tensor_needs_a_basis_above_4nq2():
    """The exact products need a CRT basis above 4 N Q^2; on a ring whose NTT-friendly primes of the
    given width run out first (N = 2^14, two 20-bit data primes) the oracle refuses the product
    instead of wrapping, while a ring with room keeps it."""
    assert O.Context(4, 2, 30, 1).has_tensor()
    c = O.Context(14, 2, 20, 1)
    assert not c.has_tensor()
    z = np.zeros(c.ct_size(), np.uint64)
    with pytest.raises(ValueError):
        c.ct_tensor(z, z)
    with pytest.raises(ValueError):
        c.ct_mul_ct(z, z)


def test_plaintext_modulus_bound():
    """t must be a prime = 1 mod 2N below 2^26 (the encoding's integer numerator then stays exact)."""
    assert O.Context(3, 2, 30, 1, t=65537).L == 2
    big = next(p for p in range((1 << 26) + 1, (1 << 26) + 10 ** 6, 16) if mr_prime(p))
    assert big % 16 == 1
    with pytest.raises(ValueError):
        O.Context(3, 2, 30, 1, t=big)


@pytest.mark.parametrize("logn,L,bits,K", [(4, 2, 30, 1), (4, 3, 50, 2), (5, 3, 30, 1)])
def test_relinearisation_key_relation(logn, L, bits, K):
    """The relinearisation key is a key-switching key for s^2 -> s in the hybrid form: on every
    modulus m of the digit j, b_j + a_j s = e_j + P [s^2]_m, and on the other moduli
    b_j + a_j s = e_j, with |e_j| <= 19 (the Gaussian tail) -- s^2 the exact negacyclic square of
    the ternary secret, P the product of the special primes."""
    c = small_ctx(logn=logn, L=L, bits=bits, K=K, seed=5)
    N = c.N
    mods = c.moduli()
    P = math.prod(mods[L:L + K])
    s = [int(v) for v in c.sk()]
    s2 = _negint(s, s)
    key = c.ksk(-1).reshape(2, c.dnum, L + K, N)
    for j in range(c.dnum):
        for m in range(L + K):
            q = mods[m]
            b = [int(v) for v in c.intt(m, key[0, j, m].copy())]
            a = [int(v) for v in c.intt(m, key[1, j, m].copy())]
            e = [(x + y) % q for x, y in zip(b, negacyclic(a, [v % q for v in s], q))]
            if m < L and m // K == j:
                e = [(x - P * v) % q for x, v in zip(e, s2)]
            e = [v - q if v > q // 2 else v for v in e]
            assert max(abs(v) for v in e) <= 19, (j, m)
            # and the key is not trivially zero on the digit
            if m < L and m // K == j:
                assert any(v % q for v in b)


# ----------------------------------------------------------------- CSSC (Sec. 4.3, App. B)
def dense_from_csr(R, C, rp, col, val):
    D = np.zeros((R, C), np.int64)
    for i in range(R):
        for k in range(rp[i], rp[i + 1]):
            D[i, col[k]] = val[k]
    return D


def random_csr(R, C, nnz, seed):
    g = np.random.default_rng(seed)
    rp, col, val = W.uniform_matrix(R, C, nnz, 9, g)
    return rp, col, val


@pytest.mark.parametrize("R,C,nnz,seed", [(1, 1, 1, 0), (7, 5, 0, 1), (12, 9, 30, 2), (40, 33, 200, 3), (64, 64, 4096, 4)])
def test_cssc_roundtrip_and_invariants(R, C, nnz, seed):
    rp, col, val = random_csr(R, C, nnz, seed)
    VA, CI, RM, CP = O.cssc(R, rp, col, val)
    nnz_row = np.diff(rp)
    Lw = len(CP) - 1
    assert Lw == (nnz_row.max() if R else 0)
    # CP[0] = 0, CP[j+1] = CP[j] + nnz of aligned column j, CP[L] = nnz
    assert CP[0] == 0 and CP[-1] == nnz
    for j in range(Lw):
        assert CP[j + 1] - CP[j] == (nnz_row > j).sum()
    # RM: a permutation, rows by descending nonzero count, ties in ascending row order
    assert sorted(RM) == list(range(R))
    keys = [(-nnz_row[r], r) for r in RM]
    assert keys == sorted(keys)
    # column-major scan of the left-aligned sorted rows; back to dense exactly
    D = np.zeros((R, C), np.int64)
    for j in range(Lw):
        for p in range(CP[j + 1] - CP[j]):
            r = RM[p]
            k = rp[r] + j
            assert CI[CP[j] + p] == col[k] and VA[CP[j] + p] == val[k]
            D[r, CI[CP[j] + p]] += VA[CP[j] + p]
    assert np.array_equal(D, dense_from_csr(R, C, rp, col, val))


def test_cssc_brute_force_tiny():
    """All 3 x 3 0/1 patterns: CSSC rebuilt by brute force from the definition."""
    for bits in range(1 << 9):
        M = np.array([(bits >> k) & 1 for k in range(9)]).reshape(3, 3) * np.arange(1, 10).reshape(3, 3)
        rows, cols = np.nonzero(M)
        rp = np.zeros(4, np.int64)
        np.add.at(rp, rows + 1, 1)
        rp = np.cumsum(rp)
        VA, CI, RM, CP = O.cssc(3, rp, cols.astype(np.int32), M[rows, cols])
        order = sorted(range(3), key=lambda r: (-np.count_nonzero(M[r]), r))
        aligned = [[(int(M[r, c]), c) for c in range(3) if M[r, c]] for r in order]
        va, ci = [], []
        for j in range(3):
            for row in aligned:
                if j < len(row):
                    va.append(row[j][0])
                    ci.append(row[j][1])
        assert list(RM) == order and list(VA) == va and list(CI) == ci


# ----------------------------------------------------------------- chunks (Alg. generateChunk)
def test_chunk_example_from_paper():
    lines = {l.split()[0]: l for l in open(os.path.join(GOLD, "chunk_example.txt")) if l.strip() and not l.startswith("#")}
    s = int(lines["s"].split()[1])
    nnz = [int(v) for v in lines["nnz_per_column"].split()[1:]]
    want = [tuple(int(v) for v in part.split()[-3:]) for part in lines["chunks"].split("|")]
    CP = np.concatenate([[0], np.cumsum(nnz)])
    assert O.chunks(CP, s) == want


@pytest.mark.parametrize("seed", range(6))
def test_chunks_fit_and_tile(seed):
    g = np.random.default_rng(seed)
    s = int(g.integers(8, 200))
    nnz = np.sort(g.integers(1, s + 1, size=int(g.integers(1, 40))))[::-1]
    CP = np.concatenate([[0], np.cumsum(nnz)])
    for uniform in (False, True):
        ch = O.chunks(CP, s, uniform)
        covered = []
        for start, c, h in ch:
            assert c >= 1 and h * c <= s                       # padded rectangle fits
            assert h == (nnz[0] if uniform else nnz[start])    # height rule
            assert all(nnz[j] <= h for j in range(start, start + c))
            covered += list(range(start, start + c))
        assert covered == list(range(len(nnz)))                # every column exactly once, in order
        if not uniform:  # greedy: the next column would not have fit
            for start, c, h in ch[:-1]:
                assert h * (c + 1) > s


def test_padded_fit_rule_differs_from_unpadded_count():
    # unpadded counting (10 + 6 + 5 = 21 <= s) would pack a 10 x 3 = 30-slot rectangle into 21
    CP = np.array([0, 10, 16, 21])
    assert O.chunks(CP, 21) == [(0, 2, 10), (2, 1, 5)]


def test_numbits_and_reorg_examples_from_paper():
    facts = [l.split() for l in open(os.path.join(GOLD, "paper_small_facts.txt")) if l.strip() and not l.startswith("#")]
    for f in facts:
        if f[0] == "numBits":
            assert int(f[1]).bit_length() == int(f[2])
    # reorgVector: slot k of a chunk holds v[CI[k]] (or 0 for padding); exercised through the
    # oracle's encrypted vector: a one-chunk matrix whose CI[3] == 1
    (k, idx) = [(int(f[1]), int(f[2])) for f in facts if f[0] == "reorg_index"][0]
    c = small_ctx(logn=5, L=2, bits=30, K=1, agg_mode=1)
    # 4 x 3 matrix with one nonzero per row; column indices by sorted row: 0, 2, 2, 1
    rp = np.array([0, 1, 2, 3, 4])
    col = np.array([0, 2, 2, 1], np.int32)
    M = O.Matrix(c, 4, 3, rp, col, np.ones(4, np.int64))
    v = np.array([1, 2, 3])
    x = M.encrypt_vector(v, 5)
    slots = c.decode(c.decrypt(x[:c.ct_size()]))
    assert int(slots[k]) == v[idx] == 2


# ----------------------------------------------------------------- aggregation (Alg. Aggregation)
def total_sum_plain(vec, r, c, fixed=True):
    """Alg. Aggregation's intra-chunk loop on a plain integer array of one slot row."""
    w = vec.copy()
    e = 1
    rots = 0
    for j in range(c.bit_length() - 2, -1, -1):
        w = w + np.roll(w, -e * r)
        rots += 1
        e *= 2
        if (c >> j) & 1:
            w = (vec if fixed else w) + np.roll(w, -r)
            rots += 1
            e += 1
    return w, rots


@pytest.mark.parametrize("c", range(1, 17))
def test_total_sum_plain_simulation(c):
    r, n = 5, 128
    g = np.random.default_rng(c)
    vec = np.zeros(n, np.int64)
    vec[:r * c] = g.integers(-9, 10, r * c)
    w, rots = total_sum_plain(vec, r, c)
    assert np.array_equal(w[:r], vec[:r * c].reshape(c, r).sum(0))
    assert rots == (c.bit_length() - 1) + (bin(c).count("1") - 1)


def test_total_sum_as_printed_double_counts():
    """The printed line w <- w + Rot(w, r) for a set bit counts block 1 twice for c = 3, which is
    why the oracle adds the original chunk ciphertext instead (the HElib totalSum it cites)."""
    vec = np.zeros(64, np.int64)
    vec[:6] = [1, 1, 10, 10, 100, 100]
    w, _ = total_sum_plain(vec, 2, 3, fixed=False)
    assert list(w[:2]) == [121, 121]   # = b0 + 2 b1 + b2
    w, _ = total_sum_plain(vec, 2, 3, fixed=True)
    assert list(w[:2]) == [111, 111]


def test_total_sum_homomorphic_matches_simulation():
    c = small_ctx(logn=7, L=3, bits=50, K=1)
    N, h = c.N, c.N // 2
    g = np.random.default_rng(3)
    for r, cc in ((5, 3), (4, 7), (9, 6)):
        x = np.zeros(N, np.int64)
        x[:r * cc] = g.integers(0, 100, r * cc)
        ct = c.encrypt(c.encode(x), 6, 0)
        got = c.decode(c.decrypt(c.total_sum(ct, r, cc)))
        want, _ = total_sum_plain(x[:h], r, cc)
        assert np.array_equal(got[:r], want[:r] % T)


# ----------------------------------------------------------------- whole protocol
def run_protocol(c, w, encrypted=False):
    M = O.Matrix(c, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], encrypted, 31)
    x = M.encrypt_vector(w["v"], 41)
    res, stats = M.he_spmv(x)
    return M, M.decrypt_result(res), stats


def test_spmv_small_workload_uniform_aggregation():
    c = O.Context(12, 2, 30, 1, agg_mode=1)
    c.keygen(101)
    w = W.small()
    M, y, stats = run_protocol(c, w)
    assert np.array_equal(y, W.spmv_mod_t(w))
    # op counts of Table "Time complexity": n_ct products, rotations within the log bound
    n_ct = M.n_chunks()
    cs = [M.chunk(k)[2] for k in range(n_ct)]
    assert stats["rotations"] == sum((x.bit_length() - 1) + (bin(x).count("1") - 1) for x in cs)
    assert stats["rotations"] <= 2 * n_ct * math.log2(max(cs))


def test_spmv_with_exact_step_keys_one_key_switch_per_rotation():
    """With a key for every totalSum step the decrypted product is unchanged and every logical
    rotation costs one key switch instead of one per binary digit of its step."""
    g = np.random.default_rng(17)
    rp, col, val = W.uniform_matrix(300, 200, 1200, 15, g)
    w = dict(R=300, C=200, row_ptr=rp, col=col, val=val, v=g.integers(-15, 16, 200))
    res = []
    for steps in (False, True):
        c = O.Context(9, 3, 50, 1, agg_mode=0)   # s = 256: two row partitions, several chunks
        c.keygen(101)
        M = O.Matrix(c, w["R"], w["C"], w["row_ptr"], w["col"], w["val"], False, 31)
        if steps:
            need = sorted({k for g in range(M.n_chunks()) for k in c.total_sum_steps(M.chunk(g)[3], M.chunk(g)[2])})
            c.add_step_keys(need)
        x = M.encrypt_vector(w["v"], 41)
        out, stats = M.he_spmv(x)
        assert np.array_equal(M.decrypt_result(out), W.spmv_mod_t(w))
        res.append(stats)
    assert res[1]["rotations"] == res[0]["rotations"] == res[1]["key_switches"]
    assert res[0]["key_switches"] > res[0]["rotations"]


def joint_chunks_python(cssc_a, cssc_b, s, uniform):
    """generateChunk (padded fit rule) on the column heights max(NNZ_A[j], NNZ_B[j])."""
    def heights(cp):
        return [cp[j + 1] - cp[j] for j in range(len(cp) - 1)]
    ha, hb = heights(cssc_a[3]), heights(cssc_b[3])
    nc = max(len(ha), len(hb))
    hj = [max(ha[j] if j < len(ha) else 0, hb[j] if j < len(hb) else 0) for j in range(nc)]
    out, i = [], 0
    while i < nc:
        start, h = i, (hj[0] if uniform else hj[i])
        while i < nc and h * (i - start + 1) <= s:
            i += 1
        out.append((start, i - start, h))
    return out


@pytest.mark.parametrize("agg,R,C,nnz", [(0, 700, 300, 2500), (0, 512, 400, 1800), (1, 600, 200, 1500), (0, 300, 300, 600)])
def test_two_slot_rows_protocol(agg, R, C, nnz):
    """Two row partitions per ciphertext (slot rows 0 and 1, joint chunks): the decrypted product is
    the integer SpMV, with one result ciphertext per pair of partitions and no more chunks than the
    one-row layout needs."""
    g = np.random.default_rng(R + C + agg)
    rp, col, val = W.uniform_matrix(R, C, nnz, 15, g)
    if R == 300:   # second partition without nonzeros: rows 256.. empty
        keep = np.repeat(np.arange(R), np.diff(rp)) < 256
        rows = np.repeat(np.arange(R), np.diff(rp))[keep]
        rp, col, val = W._csr_from_rows_cols(R, rows, col[keep], val[keep])
    w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=g.integers(-15, 16, C))
    res = {}
    for rows_ in (1, 2):
        c = O.Context(9, 3, 50, 1, agg_mode=agg, slot_rows=rows_)
        c.keygen(5)
        M = O.Matrix(c, R, C, rp, col, val, False, 31)
        x = M.encrypt_vector(w["v"], 41)
        out, stats = M.he_spmv(x)
        assert np.array_equal(M.decrypt_result(out), W.spmv_mod_t(w)), rows_
        res[rows_] = (M.n_parts(), M.n_groups(), M.n_chunks(), stats)
        if rows_ == 2:
            s = c.N // 2
            parts = []
            for r0 in range(0, R, s):
                r1 = min(R, r0 + s)
                prp = rp[r0:r1 + 1] - rp[r0]
                sl = slice(rp[r0], rp[r1])
                parts.append(O.cssc(r1 - r0, prp, col[sl], val[sl]))
            want = []
            for p in range(0, len(parts), 2):
                if p + 1 < len(parts):
                    want += [(p // 2,) + ch for ch in joint_chunks_python(parts[p], parts[p + 1], s, agg == 1)]
                else:
                    want += [(p // 2,) + tuple(ch) for ch in O.chunks(parts[p][3], s, agg == 1)]
            assert [M.chunk(k) for k in range(M.n_chunks())] == want
    (p1, g1, n1, s1), (p2, g2, n2, s2) = res[1], res[2]
    assert p1 == p2 and g1 == p1 and g2 == (p1 + 1) // 2
    assert n2 <= n1 and s2["rotations"] <= s1["rotations"]


@pytest.mark.parametrize("R,C,nnz", [(100, 100, 400), (200, 150, 600), (64, 300, 500), (1, 1, 1)])
def test_diagonal_baseline(R, C, nnz):
    """The diagonal method (the paper's baseline): the plaintext diagonals rebuild the dense matrix
    (decoded slot by slot), and the decrypted product is the integer SpMV."""
    c = O.Context(9, 3, 50, 1)
    c.keygen(3)
    g = np.random.default_rng(R * 7 + C)
    rp, col, val = W.uniform_matrix(R, C, nnz, 15, g)
    w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=g.integers(-15, 16, C))
    D = O.DiagMatrix(c, R, C, rp, col, val)
    inf = D.info()
    B = inf["B"]
    assert B == min(c.N // 4, max(R, C))
    dense = np.zeros((inf["row_blocks"] * B, inf["col_blocks"] * B), np.int64)
    q0 = c.moduli()[0]
    for k in range(inf["diagonals"]):
        bi, bj, d = D.key(k)
        coef = c.intt(0, D.pt(k)[:c.N].copy()).astype(object)
        m = np.array([(int(x) - q0 if int(x) > q0 // 2 else int(x)) % T for x in coef], np.uint64)
        sl = c.decode(m).astype(np.int64)
        sl = np.where(sl > T // 2, sl - T, sl)
        assert not sl[B:].any()
        for i in range(B):
            dense[bi * B + i, bj * B + (i + d) % B] += sl[i]
    want = np.zeros_like(dense)
    for r in range(R):
        for k in range(rp[r], rp[r + 1]):
            want[r, col[k]] = ((int(val[k]) + T // 2) % T) - T // 2
    assert np.array_equal(dense, want)
    y = D.decrypt_result(D.spmv(D.encrypt_vector(w["v"], 7)))
    assert np.array_equal(y, W.spmv_mod_t(w))


@pytest.mark.parametrize("case", ["empty", "one", "emptyrows", "rect", "partitions", "dense_row"])
def test_spmv_edge_cases_paper_aggregation(case):
    c = O.Context(9, 3, 50, 1, agg_mode=0)   # s = 256 slots per chunk
    c.keygen(5)
    g = np.random.default_rng(hash(case) & 0xFFFF)
    if case == "empty":
        R, C, nnz = 10, 10, 0
    elif case == "one":
        R, C, nnz = 1, 1, 1
    elif case == "emptyrows":
        R, C, nnz = 100, 50, 60
    elif case == "rect":
        R, C, nnz = 30, 200, 500
    elif case == "partitions":
        R, C, nnz = 700, 300, 2500     # three row partitions of <= 256 rows
    else:
        R, C, nnz = 20, 256, 256 + 19  # one full row of 256 nonzeros
    if case == "dense_row":
        rows = np.concatenate([np.zeros(256, np.int64), g.integers(1, R, 19)])
        cols = np.concatenate([np.arange(256), g.integers(0, C, 19)])
        key = np.unique(rows * C + cols)
        rows, cols = key // C, key % C
        rp, col, val = W._csr_from_rows_cols(R, rows, cols, g.integers(-15, 16, len(rows)))
    else:
        rp, col, val = W.uniform_matrix(R, C, nnz, 15, g)
    w = dict(R=R, C=C, row_ptr=rp, col=col, val=val, v=g.integers(-15, 16, C))
    M, y, _ = run_protocol(c, w)
    assert np.array_equal(y, W.spmv_mod_t(w))


def test_spmv_both_encrypted_small():
    c = O.Context(8, 3, 50, 1, agg_mode=0)
    c.keygen(3)
    w = W.laplace256(n=10)   # 100 x 100 Laplacian: two partitions of <= 128 rows
    w["v"] = w["v"][:100]
    M, y, stats = run_protocol(c, w, encrypted=True)
    assert np.array_equal(y, W.spmv_mod_t(w))
    assert stats["rotations"] == 0   # every chunk of a 5-point stencil is one column wide here
