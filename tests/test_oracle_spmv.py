"""Pins of the oracle's threaded CSR product (oracle/cpu_spmv.c), the CPU
baseline's matrix-based operator application (Sec. 3.2).

Each row of y = A u is a plain sum of a_ij u_j over the row's stored
entries; the C product sums them in storage order, so a Python loop that
does the same is equal to it bitwise, a dense product agrees to rounding, and
the result does not depend on the thread count."""
import os
import subprocess
import sys

import numpy as np
import pytest
import scipy.sparse as sp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _spmv():
    from oracle.cpu_spmv import LIB_PATH, CsrSpmv
    if not os.path.exists(LIB_PATH):
        pytest.skip("oracle/libcpu_spmv.so not built")
    return CsrSpmv


def _matrix(n, density, seed, empty_rows=()):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=density, random_state=rng, format="lil")
    for i in empty_rows:
        A[i, :] = 0
    A = sp.csr_matrix(A)
    A.sort_indices()
    return A, rng.uniform(-1, 1, n)


def _loop(A, u):
    y = np.zeros(A.shape[0])
    for i in range(A.shape[0]):
        s = 0.0
        for k in range(A.indptr[i], A.indptr[i + 1]):
            s += A.data[k] * u[A.indices[k]]
        y[i] = s
    return y


@pytest.mark.parametrize("n,density,empty", [(1, 1.0, ()), (7, 0.5, (0, 3)), (300, 0.05, (5, 299))])
def test_spmv_equals_row_sums_in_storage_order(n, density, empty):
    CsrSpmv = _spmv()
    A, u = _matrix(n, density, n, empty)
    y = CsrSpmv(A, u).apply()
    assert np.array_equal(y, _loop(A, u))
    dense = A.toarray() @ u
    scale = np.abs(A.toarray()) @ np.abs(u)
    assert np.all(np.abs(y - dense) <= 1e-14 * scale)
    for i in empty:
        assert y[i] == 0.0


def test_spmv_unsorted_columns_and_timing():
    CsrSpmv = _spmv()
    A, u = _matrix(200, 0.1, 3)
    # reverse the column order inside every row: still the same matrix
    idx = np.concatenate([np.arange(A.indptr[i], A.indptr[i + 1])[::-1] for i in range(200)])
    B = sp.csr_matrix((A.data[idx], A.indices[idx], A.indptr), shape=A.shape)
    m = CsrSpmv(B, u)
    assert np.array_equal(m.apply(), _loop(B, u))
    t = m.time(1, 5)
    assert t.shape == (5,) and np.all(t >= 0)


def test_spmv_independent_of_thread_count(tmp_path):
    tmp = str(tmp_path)
    _spmv()
    code = ("import sys, numpy as np, scipy.sparse as sp; sys.path.insert(0, %r)\n"
            "from oracle.cpu_spmv import CsrSpmv\n"
            "rng = np.random.default_rng(11); A = sp.random(5000, 5000, density=0.002, random_state=rng, "
            "format='csr'); u = rng.uniform(-1, 1, 5000)\n"
            "m = CsrSpmv(A, u); print(CsrSpmv.threads()); np.save(sys.argv[1], m.apply())\n") % ROOT
    outs = []
    for nt in (1, 3):
        f = os.path.join(tmp, f"spmv_nt{nt}.npy")
        env = dict(os.environ, OMP_NUM_THREADS=str(nt))
        r = subprocess.run([sys.executable, "-c", code, f], env=env, capture_output=True, text=True, check=True)
        assert int(r.stdout.strip()) == nt
        outs.append(np.load(f))
    assert np.array_equal(outs[0], outs[1])
