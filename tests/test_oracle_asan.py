"""The oracle under host AddressSanitizer and UndefinedBehaviorSanitizer: a C driver
(oracle/check_main.c) runs the build, the fixed-pattern re-solve, the adjoint and both
BiCGStab forms on matrices that reach every branch of the column loop (drops,
zero diagonals, rows bringing many columns, iteration limits); any memory error or
undefined behaviour aborts it. Its results must equal the oracle library's."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
from paper_1503_04500_amd import gen

HERE = os.path.dirname(os.path.abspath(__file__))
ODIR = os.path.join(HERE, "..", "oracle")


@pytest.fixture(scope="module")
def driver():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    d = tempfile.mkdtemp(prefix="rsai_asan_")
    exe = os.path.join(d, "check_main")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-fopenmp", "-std=c11",
           os.path.join(ODIR, "rsai_oracle.c"), os.path.join(ODIR, "check_main.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("sanitizer build unavailable: " + r.stderr[-300:])
    yield d, exe
    shutil.rmtree(d, ignore_errors=True)


def _arrow(n):
    rows, cols, vals = [], [], []
    for k in range(n):
        rows.append(k); cols.append(k); vals.append(4.0 if k else 2.0 * n)
        if k:
            rows += [0, k]; cols += [k, 0]; vals += [3.0, 1.0]
    return gen.from_coo(n, np.array(rows), np.array(cols), np.array(vals))


def _zero_diag():
    A = gen.cd2d(10, seed=2)
    perm = np.random.default_rng(5).permutation(A.n)
    inv = np.empty(A.n, np.int64)
    inv[perm] = np.arange(A.n)
    return gen.from_coo(A.n, inv[A.rowidx], A.col_of_entry(), A.val)


CASES = [
    ("cd2d", lambda: gen.cd2d(12, seed=1), (3, 8, 0.4, 1, 1e-3)),
    ("adaptive", lambda: gen.cd2d(10, seed=4), (2, 6, 0.2, 2, 1e-3)),
    ("nodrop", lambda: gen.cd3d(5, seed=3), (3, 5, 0.1, 0, 1e-3)),
    ("powerlaw", lambda: gen.powerlaw(400, seed=2, lmax=30), (3, 4, 0.4, 1, 1e-3)),
    ("denserows", lambda: gen.dense_rows(10, 4, 20), (3, 6, 0.3, 1, 1e-2)),
    ("zerodiag", _zero_diag, (3, 8, 0.4, 1, 1e-3)),
    ("arrow", lambda: _arrow(60), (3, 2, 0.4, 1, 1e-3)),
]


@pytest.mark.parametrize("name,make,prm", CASES, ids=[c[0] for c in CASES])
def test_oracle_clean_under_sanitizers(driver, name, make, prm):
    d, exe = driver
    A = make()
    path = os.path.join(d, name + ".bin")
    with open(path, "wb") as f:
        np.array([A.n, A.nnz], np.int64).tofile(f)
        np.asarray(A.colptr, np.int64).tofile(f)
        np.asarray(A.rowidx, np.int32).tofile(f)
        np.asarray(A.val, np.float64).tofile(f)
    c, lmax, eps, drop, tol = prm
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="2")
    r = subprocess.run([exe, path, str(c), str(lmax), repr(eps), str(drop), repr(tol)], capture_output=True,
                       text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    out = {ln.split()[0]: ln.split()[1:] for ln in r.stdout.splitlines()}
    R = oracle.rsai(A, c=c, lmax=lmax, eps=eps, drop=drop, tol=tol)
    rs = out["rsai"]
    assert int(rs[1]) == int(R["colptr"][-1])
    assert int(rs[3]) == int(np.asarray(R["rowidx"], np.int64).sum())
    assert abs(float(rs[5]) - R["val"].sum()) <= 1e-12 * max(1.0, np.abs(R["val"]).sum())
    assert int(rs[9]) == int(R["nJmax"].sum())
    assert out["fixed"][1] == "0" and float(out["fixed"][3]) <= 1e-10
    b = 1.0 + (np.arange(A.n) % 5)
    Mt = (R["colptr"], R["rowidx"], R["val"])
    its = out["bicgstab"]
    assert int(its[1]) == oracle.bicgstab(A, b, Mt, maxit=500)[0]
    assert int(its[3]) == oracle.bicgstab(A, b, None, maxit=500)[0]
    assert int(its[5]) == oracle.bicgstab(A, b, Mt, maxit=500, left=True)[0]
