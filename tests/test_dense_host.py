"""The host-side dense routines of the eigensolver (csrc/dense_host.h:
Cholesky, inverse adjoint, Hermitian Jacobi, general eigenproblem by
Hessenberg reduction and shifted QR), built with g++ alone and checked
against numpy/LAPACK on random and structured matrices.  No GPU needed."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_0912_4457_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstring>
#include "dense_host.h"
using namespace nks::dense;
int main(int argc, char** argv) {
    FILE* f = std::fopen(argv[1], "r");
    char op[16];
    int p;
    if (std::fscanf(f, "%15s %d", op, &p) != 2) return 2;
    Mat A((size_t)p * p);
    for (int j = 0; j < p; ++j)
        for (int i = 0; i < p; ++i) {
            double re, im;
            if (std::fscanf(f, "%lf %lf", &re, &im) != 2) return 2;
            A[i + (size_t)j * p] = cd(re, im);
        }
    std::fclose(f);
    auto dump = [&](const Mat& M) {
        for (int j = 0; j < p; ++j)
            for (int i = 0; i < p; ++i) std::printf("%.17g %.17g\n", M[i + (size_t)j * p].real(), M[i + (size_t)j * p].imag());
    };
    if (!std::strcmp(op, "chol")) {
        if (!cholesky(A, p)) { std::printf("FAIL\n"); return 0; }
        dump(A);
        dump(inverse_adjoint(A, p));
    } else if (!std::strcmp(op, "jacobi")) {
        symmetrise(A, p);
        std::vector<double> w;
        Mat W;
        jacobi(A, p, w, W);
        for (double x : w) std::printf("%.17g 0\n", x);
        dump(W);
    } else {
        std::vector<cd> lam;
        Mat V;
        if (!eig_general(A, p, lam, V)) { std::printf("FAIL\n"); return 0; }
        for (auto x : lam) std::printf("%.17g %.17g\n", x.real(), x.imag());
        dump(V);
    }
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("dense")
    (d / "drv.cpp").write_text(DRIVER)
    exe = d / "drv"
    subprocess.run([gxx, "-O2", "-std=c++17", "-I", CSRC, "-o", str(exe), str(d / "drv.cpp")], check=True,
                   capture_output=True)

    def run(op, A):
        p = A.shape[0]
        inp = d / "in.txt"
        with open(inp, "w") as fh:
            fh.write(f"{op} {p}\n")
            for j in range(p):
                for i in range(p):
                    fh.write(f"{A[i, j].real:.17g} {A[i, j].imag:.17g}\n")
        out = subprocess.run([str(exe), str(inp)], capture_output=True, text=True, check=True).stdout.split()
        if out and out[0] == "FAIL":
            return None
        v = np.array(out, dtype=float).reshape(-1, 2)
        return v[:, 0] + 1j * v[:, 1]
    return run


def _mat(v, p, off=0):
    return v[off:off + p * p].reshape(p, p, order="F")


@pytest.mark.parametrize("p", [1, 2, 7, 40])
def test_cholesky_and_inverse_adjoint(driver, p):
    rng = np.random.default_rng(p)
    X = rng.standard_normal((3 * p, p)) + 1j * rng.standard_normal((3 * p, p))
    G = X.conj().T @ X
    out = driver("chol", G)
    L, Z = _mat(out, p), _mat(out, p, p * p)
    assert np.allclose(np.triu(L, 1), 0)
    assert np.abs(L @ L.conj().T - G).max() <= 1e-12 * np.abs(G).max()
    assert np.abs(L.conj().T @ Z - np.eye(p)).max() <= 1e-10
    assert driver("chol", -G) is None              # not positive definite


@pytest.mark.parametrize("p", [1, 2, 9, 48])
def test_jacobi_hermitian(driver, p):
    rng = np.random.default_rng(10 + p)
    B = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    H = B + B.conj().T
    out = driver("jacobi", H)
    w, W = out[:p].real, _mat(out, p, p)
    assert np.allclose(np.sort(w), np.linalg.eigvalsh(H), rtol=0, atol=1e-12 * np.abs(H).max())
    assert np.abs(W.conj().T @ W - np.eye(p)).max() <= 1e-12
    assert np.abs(H @ W - W * w).max() <= 1e-11 * np.abs(H).max()


@pytest.mark.parametrize("kind", ["random", "normal", "jordan_near", "real_pairs", "hessenberg"])
@pytest.mark.parametrize("p", [1, 2, 5, 33])
def test_eig_general(driver, kind, p):
    rng = np.random.default_rng(hash((kind, p)) % 2**32)
    if kind == "random":
        A = rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p))
    elif kind == "normal":                          # unitary similarity of a diagonal
        Q, _ = np.linalg.qr(rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)))
        A = Q @ np.diag(rng.standard_normal(p) + 1j * rng.standard_normal(p)) @ Q.conj().T
    elif kind == "jordan_near":                     # distinct but close eigenvalues, non-normal
        A = np.diag(np.linspace(1.0, 1.0 + 1e-3 * p, p)).astype(complex) + np.diag(np.ones(p - 1), 1) * 0.5
    elif kind == "real_pairs":                      # real matrix: conjugate pairs
        A = rng.standard_normal((p, p)).astype(complex)
    else:                                           # already upper Hessenberg
        A = np.triu(rng.standard_normal((p, p)) + 1j * rng.standard_normal((p, p)), -1)
    out = driver("eig", A)
    assert out is not None
    lam, V = out[:p], _mat(out, p, p)
    ref = np.linalg.eigvals(A)
    # every eigenvalue matches one of LAPACK's
    for l_ in lam:
        assert np.min(np.abs(ref - l_)) <= 1e-9 * max(1.0, np.abs(A).max())
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0)
    res = np.abs(A @ V - V * lam).max()
    assert res <= 1e-9 * max(1.0, np.abs(A).max())
