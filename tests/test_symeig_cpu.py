"""The host eigensolver of the factored build (csrc/symeig.h: Householder
tridiagonalisation + implicit-shift QL with the transform accumulated),
compiled on its own with the host C++ compiler and checked against LAPACK
(numpy.linalg.eigh) on symmetric matrices with flat, graded (Gram-like,
eigenvalues over 15 decades) and repeated spectra: eigenvalues, A V = V diag(w),
V^T V = I, descending order."""
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_2511_12894_amd", "csrc", "symeig.h")

DRIVER = r"""
#include <cstdio>
#include <vector>
#include "%s"
int main(int argc, char** argv) {
  FILE* f = std::fopen(argv[1], "rb");
  int n = 0;
  if (std::fread(&n, sizeof(int), 1, f) != 1) return 2;
  std::vector<double> A(size_t(n) * n), w, V;
  if (std::fread(A.data(), sizeof(double), A.size(), f) != A.size()) return 2;
  std::fclose(f);
  rf::sym_eig(A, n, w, V);
  FILE* o = std::fopen(argv[2], "wb");
  std::fwrite(w.data(), sizeof(double), n, o);
  std::fwrite(V.data(), sizeof(double), V.size(), o);
  std::fclose(o);
  return 0;
}
"""


@pytest.fixture(scope="module")
def solver(tmp_path_factory):
    d = tmp_path_factory.mktemp("symeig")
    src = d / "drv.cpp"
    src.write_text(DRIVER % HEADER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-o", str(exe), str(src)], check=True)

    def run(A):
        n = A.shape[0]
        fin, fout = d / "in.bin", d / "out.bin"
        with open(fin, "wb") as f:
            f.write(np.int32(n).tobytes())
            f.write(np.ascontiguousarray(A, dtype=np.float64).tobytes())
        subprocess.run([str(exe), str(fin), str(fout)], check=True)
        raw = np.fromfile(fout, dtype=np.float64)
        return raw[:n], raw[n:].reshape(n, n)
    return run


def _check(A, w, V):
    n = A.shape[0]
    ref = np.sort(np.linalg.eigvalsh(A))[::-1]
    scale = np.abs(ref).max()
    assert np.all(np.diff(w) <= 0)
    np.testing.assert_allclose(w, ref, rtol=0, atol=1e-12 * scale)
    np.testing.assert_allclose(V.T @ V, np.eye(n), rtol=0, atol=1e-12 * np.sqrt(n))
    np.testing.assert_allclose(A @ V, V * w, rtol=0, atol=1e-11 * scale)


@pytest.mark.parametrize("n", [1, 2, 5, 64, 301])
def test_random_symmetric(solver, n):
    rng = np.random.default_rng(100 + n)
    B = rng.standard_normal((n, n))
    A = (B + B.T) / 2
    w, V = solver(A)
    _check(A, w, V)


def test_gram_like_graded_spectrum(solver):
    """Gram matrix of 200 smooth, strongly correlated vectors: eigenvalues
    falling over many decades, as for a kernel set."""
    rng = np.random.default_rng(7)
    t = np.linspace(0, 1, 3000)
    X = np.stack([np.cos(2 * np.pi * (20 + 0.01 * k) * t ** 1.5 + rng.uniform()) for k in range(200)])
    A = X @ X.T
    w, V = solver(A)
    _check(A, w, V)
    assert w[0] / max(abs(w[-1]), 1e-300) > 1e10


def test_repeated_eigenvalues(solver):
    rng = np.random.default_rng(9)
    Qm, _ = np.linalg.qr(rng.standard_normal((40, 40)))
    lam = np.repeat([5.0, 2.0, 2.0, 1e-3], 10)
    A = (Qm * lam) @ Qm.T
    A = (A + A.T) / 2
    w, V = solver(A)
    _check(A, w, V)
