"""The oracle's OpenMP build (-O3 -march=native -fopenmp, threads over independent limbs and
coefficients; the timing leg of the benchmark) gives the same ciphertext limbs as the plain
one-thread build: a plaintext-matrix SpMV with rotations and masks, and an encrypted-matrix SpMV
(exact tensor, relinearisation) on small rings.  The OpenMP library runs in a child process, since
one process loads one oracle library."""
import os
import subprocess
import sys
import textwrap

import numpy as np

import oracle as O
from paper_2603_04742_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CASES = textwrap.dedent("""
    import numpy as np
    from paper_2603_04742_amd import workloads as W
    def cases(O):
        out = []
        o = O.Context(10, 3, 50, 1, agg_mode=0)
        o.keygen(5)
        w = W.zipf16k(idx=2, R=1500)
        M = O.Matrix(o, w["R"], w["C"], w["row_ptr"], w["col"], w["val"])
        out.append(M.he_spmv(M.encrypt_vector(w["v"], 9))[0])
        o2 = O.Context(9, 3, 50, 1, agg_mode=0, lazy_relin=1)
        o2.keygen(6)
        w2 = W.laplace256(n=20)
        M2 = O.Matrix(o2, w2["R"], w2["C"], w2["row_ptr"], w2["col"], w2["val"], True, 3)
        out.append(M2.he_spmv(M2.encrypt_vector(w2["v"], 4))[0])
        return out
""")


def test_openmp_build_gives_the_same_limbs(tmp_path):
    ns = {}
    exec(CASES, ns)
    want = ns["cases"](O)
    script = CASES + textwrap.dedent("""
        import sys
        import oracle as O
        O.use_library(O.build_native(sys.argv[1]))
        assert O.set_threads(4) == 4
        for i, a in enumerate(cases(O)):
            np.save("%s/limbs%d.npy" % (sys.argv[1], i), a)
    """)
    env = dict(os.environ, PYTHONPATH=ROOT)
    subprocess.run([sys.executable, "-c", script, str(tmp_path)], check=True, env=env, cwd=ROOT, timeout=600)
    for i, a in enumerate(want):
        got = np.load(tmp_path / ("limbs%d.npy" % i))
        assert got.shape == a.shape and np.array_equal(got, a), i
    assert len(want) == 2 and W is not None
