"""Host dense linear algebra of the Krylov solvers (csrc/dense.cpp) against
numpy: the general complex eigen-solver (harmonic Ritz pairs of deflated
restarting), the complex Schur form with reordering and the shifted
Hessenberg solves (thick restarts of the multi-shift solver), the Hermitian
Jacobi eigen-solver (eigenbasis of H for the block
preconditioner), the pivoted LU solve and the column orthonormalisation.

dense.cpp is plain C++ with no HIP dependency; the test builds it with g++
together with a small C wrapper, so these checks run without a GPU."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2306_07522_amd", "csrc")

WRAPPER = r"""
#include <complex>
#include <vector>
#include "dense.h"
using heom::cd;
extern "C" {
int t_eig(int n, const double *a, double *w, double *v) {
  std::vector<cd> A(n * n), W, V;
  for (int i = 0; i < n * n; ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
  if (!heom::eig_general(n, A, W, V)) return 1;
  for (int i = 0; i < n; ++i) { w[2 * i] = W[i].real(); w[2 * i + 1] = W[i].imag(); }
  for (int i = 0; i < n * n; ++i) { v[2 * i] = V[i].real(); v[2 * i + 1] = V[i].imag(); }
  return 0;
}
int t_eigh(int n, const double *a, double *e, double *u) {
  std::vector<cd> A(n * n), U;
  std::vector<double> E;
  for (int i = 0; i < n * n; ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
  if (!heom::eigh_jacobi(n, A, E, U)) return 1;
  for (int i = 0; i < n; ++i) e[i] = E[i];
  for (int i = 0; i < n * n; ++i) { u[2 * i] = U[i].real(); u[2 * i + 1] = U[i].imag(); }
  return 0;
}
int t_solve(int n, const double *a, double *x) {
  std::vector<cd> A(n * n), X(n);
  for (int i = 0; i < n * n; ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
  for (int i = 0; i < n; ++i) X[i] = cd(x[2 * i], x[2 * i + 1]);
  if (!heom::lu_solve(n, A, X)) return 1;
  for (int i = 0; i < n; ++i) { x[2 * i] = X[i].real(); x[2 * i + 1] = X[i].imag(); }
  return 0;
}
int t_schur(int n, const double *a, const char *sel, double *t, double *z, int reorder) {
  std::vector<cd> A(n * n), T, Z;
  for (int i = 0; i < n * n; ++i) A[i] = cd(a[2 * i], a[2 * i + 1]);
  if (!heom::schur_complex(n, A, T, Z)) return 1;
  if (reorder) heom::schur_reorder(n, T, Z, std::vector<char>(sel, sel + n));
  for (int i = 0; i < n * n; ++i) {
    t[2 * i] = T[i].real(); t[2 * i + 1] = T[i].imag();
    z[2 * i] = Z[i].real(); z[2 * i + 1] = Z[i].imag();
  }
  return 0;
}
int t_hess(int n, double *a, double *z) {
  std::vector<cd> H(n * n), Z(n * n, cd(0));
  for (int i = 0; i < n * n; ++i) H[i] = cd(a[2 * i], a[2 * i + 1]);
  for (int i = 0; i < n; ++i) Z[i + i * n] = 1.0;
  heom::hessenberg_reduce(n, H, Z);
  for (int i = 0; i < n * n; ++i) {
    a[2 * i] = H[i].real(); a[2 * i + 1] = H[i].imag();
    z[2 * i] = Z[i].real(); z[2 * i + 1] = Z[i].imag();
  }
  return 0;
}
int t_hsolve(int k, const double *h, double sr, double si, const double *rhs, double *y) {
  std::vector<cd> H(k * k), R(k), Y;
  for (int i = 0; i < k * k; ++i) H[i] = cd(h[2 * i], h[2 * i + 1]);
  for (int i = 0; i < k; ++i) R[i] = cd(rhs[2 * i], rhs[2 * i + 1]);
  heom::HessSolver hs;
  if (!hs.solve(H, k, k, cd(sr, si), R, Y)) return 1;
  for (int i = 0; i < k; ++i) { y[2 * i] = Y[i].real(); y[2 * i + 1] = Y[i].imag(); }
  return 0;
}
int t_orth(int rows, int cols, double *p, double tol) {
  std::vector<cd> P(rows * cols);
  for (int i = 0; i < rows * cols; ++i) P[i] = cd(p[2 * i], p[2 * i + 1]);
  const int k = heom::orthonormalise_columns(rows, cols, P, tol);
  for (int i = 0; i < rows * cols; ++i) { p[2 * i] = P[i].real(); p[2 * i + 1] = P[i].imag(); }
  return k;
}
}
"""


@pytest.fixture(scope="module")
def dense(tmp_path_factory):
    d = tmp_path_factory.mktemp("dense")
    src = d / "wrap.cpp"
    src.write_text(WRAPPER)
    so = d / "libdense_test.so"
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-I", CSRC, str(src),
                    os.path.join(CSRC, "dense.cpp"), "-o", str(so)], check=True)
    lib = C.CDLL(str(so))
    dp = C.POINTER(C.c_double)
    lib.t_eig.argtypes = [C.c_int, dp, dp, dp]
    lib.t_eigh.argtypes = [C.c_int, dp, dp, dp]
    lib.t_solve.argtypes = [C.c_int, dp, dp]
    lib.t_orth.argtypes = [C.c_int, C.c_int, dp, C.c_double]
    lib.t_schur.argtypes = [C.c_int, dp, C.c_char_p, dp, dp, C.c_int]
    lib.t_hess.argtypes = [C.c_int, dp, dp]
    lib.t_hsolve.argtypes = [C.c_int, dp, C.c_double, C.c_double, dp, dp]
    return lib


def _ptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _colmajor(A):
    return np.ascontiguousarray(np.asfortranarray(A).ravel(order="F").view(np.float64))


def _eig(lib, A):
    n = A.shape[0]
    a = _colmajor(A.astype(np.complex128))
    w = np.zeros(2 * n)
    v = np.zeros(2 * n * n)
    assert lib.t_eig(n, _ptr(a), _ptr(w), _ptr(v)) == 0
    return w.view(np.complex128), v.view(np.complex128).reshape(n, n, order="F")


def _match(a, b):
    """Largest distance after pairing every value of a with its nearest in b."""
    b = list(b)
    worst = 0.0
    for x in a:
        k = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[k]))
        b.pop(k)
    return worst


def _cases():
    rng = np.random.default_rng(11)
    out = []
    for n in (1, 2, 3, 7, 30, 90):
        out.append(("random", rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))))
    H = np.triu(rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40)), -1)
    out.append(("hessenberg", H))
    T = np.triu(rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12)))
    out.append(("triangular", T))
    Q, _ = np.linalg.qr(rng.standard_normal((16, 16)) + 1j * rng.standard_normal((16, 16)))
    D = np.diag(np.repeat([1.0, -2.0 + 1j, 0.5j, 3.0], 4))
    out.append(("repeated", Q @ D @ Q.conj().T))
    # the shape that deflated restarting solves: Hessenberg plus a last-column update
    Hm = np.triu(rng.standard_normal((25, 25)) + 1j * rng.standard_normal((25, 25)), -1)
    f = np.linalg.solve(Hm.conj().T, np.eye(25)[:, -1])
    out.append(("harmonic", Hm + 0.3 * np.outer(f, np.eye(25)[-1])))
    return out


@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] + str(c[1].shape[0]) for c in _cases()])
def test_eig_general_against_numpy(dense, name, A):
    w, V = _eig(dense, A)
    scale = max(1.0, np.abs(A).max())
    assert _match(np.linalg.eigvals(A), w) <= 1e-8 * scale * A.shape[0]
    if name != "repeated":  # eigenvectors of a repeated eigenvalue are a subspace; residuals still hold
        res = np.linalg.norm(A @ V - V * w[None, :], axis=0)
        assert res.max() <= 1e-9 * scale * A.shape[0]
    assert np.allclose(np.linalg.norm(V, axis=0), 1.0)


@pytest.mark.parametrize("n,degenerate", [(1, False), (2, False), (6, False), (16, False), (16, True), (20, True)])
def test_eigh_jacobi_against_numpy(dense, n, degenerate):
    rng = np.random.default_rng(n + 100 * degenerate)
    if degenerate:  # spin-degenerate spectrum, as in the Anderson models
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        ev = np.repeat(rng.standard_normal(n // 2), 2)
        A = Q @ np.diag(ev) @ Q.conj().T
    else:
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = A + A.conj().T
    a = _colmajor(A)
    e = np.zeros(n)
    u = np.zeros(2 * n * n)
    assert dense.t_eigh(n, _ptr(a), _ptr(e), _ptr(u)) == 0
    U = u.view(np.complex128).reshape(n, n, order="F")
    assert np.allclose(e, np.linalg.eigvalsh(A), atol=1e-12 * max(1.0, np.abs(A).max()))
    assert np.abs(U.conj().T @ U - np.eye(n)).max() <= 1e-13
    assert np.abs(U @ np.diag(e) @ U.conj().T - A).max() <= 1e-12 * max(1.0, np.abs(A).max())


def test_lu_solve_against_numpy(dense):
    rng = np.random.default_rng(5)
    for n in (1, 4, 33):
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        if n > 1:
            A[0, 0] = 0.0  # needs a pivot
        b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
        x = np.ascontiguousarray(b.copy().view(np.float64))
        assert dense.t_solve(n, _ptr(_colmajor(A)), _ptr(x)) == 0
        assert np.allclose(x.view(np.complex128), np.linalg.solve(A, b), rtol=1e-10, atol=1e-12)
    S = np.zeros((3, 3), complex)
    x = np.zeros(6)
    assert dense.t_solve(3, _ptr(_colmajor(S)), _ptr(x)) == 1


def test_orthonormalise_columns(dense):
    rng = np.random.default_rng(8)
    P = rng.standard_normal((30, 6)) + 1j * rng.standard_normal((30, 6))
    P[:, 3] = 2.0 * P[:, 0] - 1j * P[:, 1]          # dependent: dropped
    p = _colmajor(P)
    k = dense.t_orth(30, 6, _ptr(p), 1e-10)
    assert k == 5
    Q = p.view(np.complex128).reshape(30, 6, order="F")[:, :k]
    assert np.abs(Q.conj().T @ Q - np.eye(k)).max() <= 1e-13
    # every original column lies in the span of Q
    for c in range(6):
        r = P[:, c] - Q @ (Q.conj().T @ P[:, c])
        assert np.linalg.norm(r) <= 1e-10 * np.linalg.norm(P[:, c])


def _schur(lib, A, sel=None):
    n = A.shape[0]
    a = _colmajor(A.astype(np.complex128))
    t = np.zeros(2 * n * n)
    z = np.zeros(2 * n * n)
    flags = bytes(bytearray([1 if (sel is not None and sel[i]) else 0 for i in range(n)]))
    assert lib.t_schur(n, _ptr(a), flags, _ptr(t), _ptr(z), int(sel is not None)) == 0
    return (t.view(np.complex128).reshape(n, n, order="F"), z.view(np.complex128).reshape(n, n, order="F"))


@pytest.mark.parametrize("name,A", _cases(), ids=[c[0] + str(c[1].shape[0]) for c in _cases()])
def test_schur_complex(dense, name, A):
    """A = Z T Z^H with Z unitary and T upper triangular; diag(T) are the
    eigenvalues."""
    n = A.shape[0]
    T, Z = _schur(dense, A)
    scale = max(1.0, np.abs(A).max())
    assert np.abs(np.tril(T, -1)).max(initial=0.0) == 0.0
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-13 * n
    assert np.abs(Z @ T @ Z.conj().T - A).max() <= 1e-13 * scale * n
    assert _match(np.linalg.eigvals(A), np.diag(T)) <= 1e-8 * scale * n


@pytest.mark.parametrize("n,pick", [(2, [1]), (6, [5, 2]), (20, [19, 3, 11, 7]), (30, list(range(0, 30, 3)))])
def test_schur_reorder_moves_selected_eigenvalues_first(dense, n, pick):
    """After reordering, the flagged eigenvalues lead the diagonal in their
    original order, the form is still a Schur form of A, and the leading
    columns of Z span an invariant subspace: A Z_k = Z_k T_k."""
    rng = np.random.default_rng(n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    T0, _ = _schur(dense, A)
    sel = np.zeros(n, bool)
    sel[pick] = True
    T, Z = _schur(dense, A, sel)
    k = len(pick)
    want = np.diag(T0)[np.sort(pick)]
    assert np.abs(np.diag(T)[:k] - want).max() <= 1e-12 * np.abs(A).max()
    assert _match(np.diag(T)[k:], np.diag(T0)[~sel]) <= 1e-10 * np.abs(A).max()
    assert np.abs(np.tril(T, -1)).max(initial=0.0) == 0.0
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-13 * n
    assert np.abs(Z @ T @ Z.conj().T - A).max() <= 1e-12 * np.abs(A).max() * n
    Zk = Z[:, :k]
    assert np.abs(A @ Zk - Zk @ T[:k, :k]).max() <= 1e-12 * np.abs(A).max() * n


def test_schur_reorder_with_equal_eigenvalues(dense):
    """Swapping equal diagonal entries is a no-op rotation, not a division by
    zero."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((8, 8)) + 1j * rng.standard_normal((8, 8)))
    A = Q @ np.diag([1.0, 1.0, 2.0, 2.0, 1.0, 3.0, 3.0, 2.0]).astype(complex) @ Q.conj().T
    sel = np.zeros(8, bool)
    sel[[4, 6, 7]] = True
    T, Z = _schur(dense, A, sel)
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(Z))
    assert np.abs(Z @ T @ Z.conj().T - A).max() <= 1e-12 * 8


@pytest.mark.parametrize("n", [1, 2, 3, 9, 25])
def test_hessenberg_reduce(dense, n):
    """H <- Q^H H Q is upper Hessenberg, Q unitary, and the similarity holds;
    an already Hessenberg input keeps its moduli (only phases change)."""
    rng = np.random.default_rng(40 + n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    a = _colmajor(A)
    z = np.zeros(2 * n * n)
    dense.t_hess(n, _ptr(a), _ptr(z))
    H = a.view(np.complex128).reshape(n, n, order="F")
    Q = z.view(np.complex128).reshape(n, n, order="F")
    assert np.abs(np.tril(H, -2)).max(initial=0.0) == 0.0
    assert np.abs(Q.conj().T @ Q - np.eye(n)).max() <= 1e-13 * n
    assert np.abs(Q @ H @ Q.conj().T - A).max() <= 1e-13 * n * np.abs(A).max()
    Hh = np.triu(A, -1)
    a = _colmajor(Hh)
    dense.t_hess(n, _ptr(a), _ptr(z))
    H2 = a.view(np.complex128).reshape(n, n, order="F")
    assert np.allclose(np.abs(H2), np.abs(Hh), atol=1e-13 * n)


@pytest.mark.parametrize("k", [1, 2, 5, 20, 40])
def test_shifted_hessenberg_solve(dense, k):
    """(H + sigma I) y = rhs for upper-Hessenberg H at several complex shifts
    (the per-frequency projected systems of the multi-shift solver), against
    numpy; entries below the subdiagonal are ignored; a zero pivot is
    reported."""
    rng = np.random.default_rng(70 + k)
    H = np.triu(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k)), -1)
    Hfull = H + np.tril(rng.standard_normal((k, k)), -2)   # junk below the subdiagonal: must not be read
    rhs = rng.standard_normal(k) + 1j * rng.standard_normal(k)
    for sigma in (0.0, 0.7j, -1.3 + 2.0j, 1e-3):
        y = np.zeros(2 * k)
        st = dense.t_hsolve(k, _ptr(_colmajor(Hfull)), sigma.real if isinstance(sigma, complex) else sigma,
                            sigma.imag if isinstance(sigma, complex) else 0.0,
                            _ptr(np.ascontiguousarray(rhs.view(np.float64))), _ptr(y))
        assert st == 0
        ref = np.linalg.solve(H + sigma * np.eye(k), rhs)
        assert np.abs(y.view(np.complex128) - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())
    # neighbouring-row pivoting: a zero diagonal entry with a nonzero subdiagonal one
    if k >= 2:
        Hp = H.copy()
        Hp[0, 0] = 0.0
        y = np.zeros(2 * k)
        assert dense.t_hsolve(k, _ptr(_colmajor(Hp)), 0.0, 0.0, _ptr(np.ascontiguousarray(rhs.view(np.float64))), _ptr(y)) == 0
        assert np.allclose(y.view(np.complex128), np.linalg.solve(Hp, rhs), rtol=1e-9, atol=1e-11)
    Z = np.zeros((k, k), complex)
    y = np.zeros(2 * k)
    assert dense.t_hsolve(k, _ptr(_colmajor(Z)), 0.0, 0.0, _ptr(np.ascontiguousarray(rhs.view(np.float64))), _ptr(y)) == 1
