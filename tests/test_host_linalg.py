"""Host linear algebra of the library's state assembly (host_linalg.h), on the
CPU: the Hermitian eigensolver (Householder tridiagonalisation + implicit QL)
against numpy's eigh, eigenvector residuals and orthonormality, and the
tridiagonal form's spectrum."""
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "host", "linalg_check.cpp")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("linalg") / "linalg_check")
    subprocess.check_call(["g++", "-O2", "-std=c++17", SRC, "-o", exe])
    return exe


def _run(exe, A):
    n = A.shape[0]
    with tempfile.TemporaryDirectory() as d:
        fi, fo = os.path.join(d, "in"), os.path.join(d, "out")
        with open(fi, "wb") as f:
            np.array([n], np.float64).tofile(f)
            np.ascontiguousarray(A, np.complex128).tofile(f)
        subprocess.check_call([exe, fi, fo])
        out = np.fromfile(fo, np.float64)
    flags, out = out[:2], out[2:]
    lam, out = out[:n], out[n:]
    V, out = out[:2 * n * n].view(np.complex128).reshape(n, n), out[2 * n * n:]
    lam2, d, e = out[:n], out[n:2 * n], out[2 * n:3 * n]
    return flags, lam, V, lam2, d, e


def _hermitian(n, rng, kind):
    if kind == "random":
        Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        return (Z + Z.conj().T) / 2
    if kind == "degenerate":  # repeated eigenvalues
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        lam = np.repeat(rng.standard_normal((n + 2) // 3), 3)[:n]
        return (Q * lam) @ Q.conj().T
    if kind == "diagonal":
        return np.diag(rng.standard_normal(n)).astype(np.complex128)
    if kind == "state":  # H = I - Sigma^-1 of a lossy squeezed state (spectrum in (-1, 1))
        import workloads as W
        from oracle import state as st
        m = n // 2
        U = W.haar_unitary(m, rng)
        S = st.assemble(W.make_instance(np.sqrt(0.6) * U, rng.uniform(0.2, 1.0, m), bin_of=np.zeros(m), cutoff=[3]))
        return np.eye(2 * m) - np.linalg.inv(S["Sigma"])
    if kind == "lowrank":  # the same with one squeezed input: rank 2, a cluster of n - 2 zeros
        import workloads as W
        from oracle import state as st
        m = n // 2
        r = np.zeros(m)
        r[rng.integers(m)] = rng.uniform(0.4, 1.2)
        S = st.assemble(W.make_instance(np.sqrt(0.3) * W.haar_unitary(m, rng), r, bin_of=np.zeros(m), cutoff=[3]))
        return np.eye(2 * m) - np.linalg.inv(S["Sigma"])
    raise ValueError(kind)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 16, 33, 96, 288])
@pytest.mark.parametrize("kind", ["random", "degenerate", "diagonal", "state", "lowrank"])
def test_hermitian_eigensolver_matches_numpy(driver, n, kind):
    if kind in ("state", "lowrank") and n % 2:
        pytest.skip("state matrices have even order")
    rng = np.random.default_rng(1000 * n + len(kind))
    A = _hermitian(n, rng, kind)
    flags, lam, V, lam2, d, e = _run(driver, A)
    assert flags.tolist() == [1.0, 1.0]
    ref = np.linalg.eigvalsh(A)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(np.sort(lam) - ref).max() <= 1e-12 * scale * n
    assert np.abs(np.sort(lam2) - ref).max() <= 1e-12 * scale * n
    assert np.abs(A @ V - V * lam[None, :]).max() <= 1e-12 * scale * n
    assert np.abs(V.conj().T @ V - np.eye(n)).max() <= 1e-12 * n
    T = np.diag(d) + np.diag(e[:-1], 1) + np.diag(e[:-1], -1) if n > 1 else np.diag(d)
    assert np.all(e[:-1] >= 0)
    assert np.abs(np.linalg.eigvalsh(T) - ref).max() <= 1e-12 * scale * n
