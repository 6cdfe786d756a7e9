"""Seeded synthetic inputs for encrypted SpMV (matrices in CSR form, vectors, request streams).

This module holds no homomorphic-encryption arithmetic: it only draws integer matrices, vectors
and arrival times with numpy.  Both the GPU tests and the CPU oracle tests take their inputs from
here, so the two sides see identical data.

The SuiteSparse matrices the paper evaluates on (Sec. 5) are not available; these generators
stand in for them with the shapes, value ranges and degree structure of the five workloads:

  small      256 x 256, 2% density, uniform positions, values and vector in [-7, 7]   (N = 4096)
  zipf16k    16384 x 16384, Zipf(1.2) column degrees, mean 8 nnz per column (131072 nnz),
             values and vector in [-15, 15]                                             (N = 16384)
  laplace256 5-point Laplacian on a 256 x 256 grid (65536 rows, 326656 nnz; 4 and -1),
             vector in [-3, 3]; matrix values encrypted too                             (N = 32768)
  batch64    64 square matrices, rows log-uniform in [512, 16384], density log-uniform in
             [0.05%, 1%], uniform positions, values and vectors in [-7, 7]               (N = 16384)
  serve10k   request stream: exponential inter-arrivals (mean 5 ms), key-set uniform over 8,
             rows = cols log-uniform in [1024, 32768], Zipf(1.2) with 8 nnz per column,
             values and vectors in [-15, 15]                                             (N = 16384)
"""
import numpy as np

BASE_SEED = 0x2603047420260000


def rng(tag, sub=0):
    return np.random.default_rng([BASE_SEED & 0xFFFFFFFF, BASE_SEED >> 32, tag, sub])


def _csr_from_rows_cols(R, rows, cols, vals):
    """CSR with columns ascending inside each row."""
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(R + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return row_ptr, cols.astype(np.int32), vals.astype(np.int64)


def uniform_matrix(R, C, nnz, vmax, g):
    """nnz distinct positions uniform over the R x C grid; values uniform in [-vmax, vmax]."""
    pos = g.choice(R * C, size=nnz, replace=False)
    rows, cols = pos // C, pos % C
    vals = g.integers(-vmax, vmax + 1, size=nnz)
    return _csr_from_rows_cols(R, rows, cols, vals)


def zipf_degrees(R, C, total, alpha, g):
    """Column degrees: the column of rank k (ranks a seeded permutation) gets weight k^-alpha;
    `total` nonzeros are spread by water-filling with a cap of R per column and largest-remainder
    rounding."""
    w = np.arange(1, C + 1, dtype=np.float64) ** (-alpha)
    cap = np.full(C, float(R))
    deg = np.zeros(C)
    free = np.ones(C, bool)
    remaining = float(total)
    while remaining > 1e-9 and free.any():
        share = remaining * w * free / (w * free).sum()
        over = free & (deg + share >= cap)
        if over.any():
            remaining -= (cap[over] - deg[over]).sum()
            deg[over] = cap[over]
            free &= ~over
        else:
            deg += share
            remaining = 0.0
    base = np.floor(deg).astype(np.int64)
    short = int(total - base.sum())
    if short > 0:
        frac = deg - base
        frac[base >= R] = -1.0
        idx = np.argsort(-frac, kind="stable")[:short]
        base[idx] += 1
    perm = g.permutation(C)
    out = np.zeros(C, np.int64)
    out[perm] = base
    return out


def zipf_matrix(R, C, nnz_per_col, alpha, vmax, g):
    deg = zipf_degrees(R, C, nnz_per_col * C, alpha, g)
    rows = np.concatenate([g.choice(R, size=int(d), replace=False) for d in deg]) if deg.sum() else np.zeros(0, np.int64)
    cols = np.repeat(np.arange(C), deg)
    vals = g.integers(-vmax, vmax + 1, size=len(rows))
    return _csr_from_rows_cols(R, rows, cols, vals)


def laplace_2d(n):
    """5-point stencil on an n x n grid, natural ordering: 4 on the diagonal, -1 to neighbours."""
    R = n * n
    rows, cols, vals = [], [], []
    idx = np.arange(R)
    i, j = idx // n, idx % n
    for di, dj, v in ((0, 0, 4), (-1, 0, -1), (1, 0, -1), (0, -1, -1), (0, 1, -1)):
        ok = (i + di >= 0) & (i + di < n) & (j + dj >= 0) & (j + dj < n)
        rows.append(idx[ok]); cols.append(((i + di) * n + (j + dj))[ok]); vals.append(np.full(ok.sum(), v))
    return _csr_from_rows_cols(R, np.concatenate(rows), np.concatenate(cols), np.concatenate(vals))


def small(idx=0):
    g = rng(0, idx)
    R = C = 256
    row_ptr, col, val = uniform_matrix(R, C, round(0.02 * R * C), 7, g)
    v = g.integers(-7, 8, size=C)
    return dict(R=R, C=C, row_ptr=row_ptr, col=col, val=val, v=v)


def zipf16k(idx=0, R=16384):
    g = rng(1, idx)
    row_ptr, col, val = zipf_matrix(R, R, 8, 1.2, 15, g)
    v = g.integers(-15, 16, size=R)
    return dict(R=R, C=R, row_ptr=row_ptr, col=col, val=val, v=v)


def laplace256(n=256):
    g = rng(2)
    row_ptr, col, val = laplace_2d(n)
    v = g.integers(-3, 4, size=n * n)
    return dict(R=n * n, C=n * n, row_ptr=row_ptr, col=col, val=val, v=v)


def batch64(count=64, rmin=512, rmax=16384):
    g = rng(3)
    out = []
    for b in range(count):
        R = int(round(np.exp(g.uniform(np.log(rmin), np.log(rmax)))))
        d = float(np.exp(g.uniform(np.log(5e-4), np.log(1e-2))))
        nnz = max(1, int(round(d * R * R)))
        row_ptr, col, val = uniform_matrix(R, R, nnz, 7, g)
        v = g.integers(-7, 8, size=R)
        out.append(dict(R=R, C=R, row_ptr=row_ptr, col=col, val=val, v=v))
    return out


def serve_stream(n_requests=10000, rate=200.0, n_keysets=8, rmin=1024, rmax=32768):
    """Arrival times (s), key-set ids and matrix sizes; matrices are drawn lazily by serve_request."""
    g = rng(4)
    gaps = g.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    keyset = g.integers(0, n_keysets, size=n_requests)
    sizes = np.round(np.exp(g.uniform(np.log(rmin), np.log(rmax), size=n_requests))).astype(np.int64)
    return arrivals, keyset, sizes


def serve_request(i, R):
    g = rng(5, i)
    row_ptr, col, val = zipf_matrix(R, R, 8, 1.2, 15, g)
    v = g.integers(-15, 16, size=R)
    return dict(R=R, C=R, row_ptr=row_ptr, col=col, val=val, v=v)


def spmv_mod_t(w, t=65537):
    """Integer SpMV y = A v reduced to the centered range (-t/2, t/2] (the plain definition of
    the decrypted result)."""
    R = w["R"]
    y = np.zeros(R, dtype=object)
    rp, col, val, v = w["row_ptr"], w["col"], w["val"], w["v"]
    rows = np.repeat(np.arange(R), np.diff(rp))
    prod = val.astype(np.int64) * v[col].astype(np.int64)
    y = np.zeros(R, np.int64)
    np.add.at(y, rows, prod)
    y = np.mod(y, t)
    return np.where(y > t // 2, y - t, y)
