// Host dense complex kernels for the projected Krylov matrices.
#include "dense.h"

#include <algorithm>
#include <cmath>
#include <limits>

namespace heom {

namespace {

// Plane rotation G = [[c, s], [-conj(s), c]] (c real) that maps (a, b) to
// (r, 0).
struct Rot {
  double c;
  cd s;
};

Rot make_rot(cd a, cd b) {
  const double na = std::abs(a), nb = std::abs(b);
  if (nb == 0.0) return {1.0, cd(0)};
  if (na == 0.0) return {0.0, std::conj(b) / nb};
  const double nrm = std::hypot(na, nb);
  return {na / nrm, (a / na) * std::conj(b) / nrm};
}

// rows i, i+1 of A (columns c0..c1-1) <- G * rows
void rot_rows(std::vector<cd> &A, int lda, int i, int c0, int c1, const Rot &g) {
  for (int j = c0; j < c1; ++j) {
    cd &x = A[i + (size_t)j * lda];
    cd &y = A[i + 1 + (size_t)j * lda];
    const cd t = g.c * x + g.s * y;
    y = -std::conj(g.s) * x + g.c * y;
    x = t;
  }
}

// columns i, i+1 of A (rows r0..r1-1) <- columns * G^H
void rot_cols(std::vector<cd> &A, int lda, int i, int r0, int r1, const Rot &g) {
  for (int r = r0; r < r1; ++r) {
    cd &x = A[r + (size_t)i * lda];
    cd &y = A[r + (size_t)(i + 1) * lda];
    const cd t = x * g.c + y * std::conj(g.s);
    y = -x * g.s + y * g.c;
    x = t;
  }
}

}  // namespace

void hessenberg_reduce(int n, std::vector<cd> &H, std::vector<cd> &Z) {
  auto h = [&](int i, int j) -> cd & { return H[i + (size_t)j * n]; };
  // Householder reflections I - 2 v v^H on rows/columns j+1..n-1
  std::vector<cd> v(n);
  for (int j = 0; j + 2 < n; ++j) {
    double xn = 0.0;
    for (int i = j + 1; i < n; ++i) xn += std::norm(h(i, j));
    xn = std::sqrt(xn);
    if (xn == 0.0) continue;
    const cd x0 = h(j + 1, j);
    const cd phase = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1);
    const cd alpha = -phase * xn;
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = j + 1; i < n; ++i) v[i] = h(i, j);
    v[j + 1] -= alpha;
    double vn = 0.0;
    for (int i = j + 1; i < n; ++i) vn += std::norm(v[i]);
    vn = std::sqrt(vn);
    if (vn == 0.0) continue;
    for (int i = j + 1; i < n; ++i) v[i] /= vn;
    // rows: H <- (I - 2 v v^H) H
    for (int c = 0; c < n; ++c) {
      cd s(0);
      for (int i = j + 1; i < n; ++i) s += std::conj(v[i]) * h(i, c);
      for (int i = j + 1; i < n; ++i) h(i, c) -= 2.0 * v[i] * s;
    }
    // columns: H <- H (I - 2 v v^H), Z likewise
    for (int r = 0; r < n; ++r) {
      cd s(0), t(0);
      for (int i = j + 1; i < n; ++i) {
        s += h(r, i) * v[i];
        t += Z[r + (size_t)i * n] * v[i];
      }
      for (int i = j + 1; i < n; ++i) {
        h(r, i) -= 2.0 * s * std::conj(v[i]);
        Z[r + (size_t)i * n] -= 2.0 * t * std::conj(v[i]);
      }
    }
    for (int i = j + 2; i < n; ++i) h(i, j) = 0.0;
  }
}

bool schur_complex(int n, const std::vector<cd> &A, std::vector<cd> &H, std::vector<cd> &Z) {
  H.assign(A.begin(), A.begin() + (size_t)n * n);
  Z.assign((size_t)n * n, cd(0));
  for (int i = 0; i < n; ++i) Z[i + (size_t)i * n] = 1.0;
  if (n <= 1) return true;
  auto h = [&](int i, int j) -> cd & { return H[i + (size_t)j * n]; };
  hessenberg_reduce(n, H, Z);

  // implicitly shifted QR on the active window [lo, hi]
  double anorm = 0.0;
  for (const cd &z : H) anorm = std::max(anorm, std::abs(z));
  const double eps = std::numeric_limits<double>::epsilon();
  int hi = n - 1, iter = 0, total = 0;
  const int max_total = 60 * n + 100;
  while (hi > 0) {
    int lo = hi;
    while (lo > 0) {
      const double s = std::abs(h(lo - 1, lo - 1)) + std::abs(h(lo, lo));
      if (std::abs(h(lo, lo - 1)) <= eps * (s > 0 ? s : anorm)) {
        h(lo, lo - 1) = 0.0;
        break;
      }
      --lo;
    }
    if (lo == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > max_total) return false;
    ++iter;
    // Wilkinson shift: the eigenvalue of the trailing 2x2 block nearer h(hi, hi)
    cd mu;
    if (iter % 11 == 10) {
      mu = h(hi, hi) + std::abs(h(hi, hi - 1));  // exceptional shift
    } else {
      const cd a = h(hi - 1, hi - 1), b = h(hi - 1, hi), c = h(hi, hi - 1), d = h(hi, hi);
      const cd half = 0.5 * (a - d);
      const cd disc = std::sqrt(half * half + b * c);
      const cd m1 = 0.5 * (a + d) + disc, m2 = 0.5 * (a + d) - disc;
      mu = std::abs(m1 - d) < std::abs(m2 - d) ? m1 : m2;
    }
    // chase the bulge through the window; rows and columns outside it are
    // updated too so that H converges to the full Schur form
    for (int k = lo; k < hi; ++k) {
      const Rot g = (k == lo) ? make_rot(h(lo, lo) - mu, h(lo + 1, lo)) : make_rot(h(k, k - 1), h(k + 1, k - 1));
      rot_rows(H, n, k, k == lo ? lo : k - 1, n, g);
      if (k > lo) h(k + 1, k - 1) = 0.0;
      rot_cols(H, n, k, 0, std::min(k + 3, hi + 1), g);
      rot_cols(Z, n, k, 0, n, g);
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) h(i, j) = 0.0;
  return true;
}

void schur_reorder(int n, std::vector<cd> &T, std::vector<cd> &Z, const std::vector<char> &sel) {
  auto t = [&](int i, int j) -> cd & { return T[i + (size_t)j * n]; };
  std::vector<char> flag(sel.begin(), sel.begin() + n);
  int next = 0;  // first position not yet holding a selected eigenvalue
  for (int i = 0; i < n; ++i) {
    if (!flag[i]) continue;
    // bubble the eigenvalue at i up to position next
    for (int q = i - 1; q >= next; --q) {
      // swap the diagonal entries a = T(q,q), b = T(q+1,q+1): the plane
      // rotation that maps the eigenvector (t_q,q+1, b - a) of the 2 x 2
      // block for b onto e_1 makes T(q,q) = b and T(q+1,q) = 0
      const cd a = t(q, q), b = t(q + 1, q + 1);
      const Rot g = make_rot(t(q, q + 1), b - a);
      rot_rows(T, n, q, q, n, g);
      rot_cols(T, n, q, 0, q + 2, g);
      rot_cols(Z, n, q, 0, n, g);
      t(q + 1, q) = 0.0;
      t(q, q) = b;
      t(q + 1, q + 1) = a;
      std::swap(flag[q], flag[q + 1]);
    }
    ++next;
  }
}

bool eig_general(int n, const std::vector<cd> &A, std::vector<cd> &w, std::vector<cd> &vecs) {
  w.assign(n, cd(0));
  vecs.assign((size_t)n * n, cd(0));
  if (n <= 0) return true;
  std::vector<cd> H, Z;
  if (!schur_complex(n, A, H, Z)) return false;
  auto h = [&](int i, int j) -> cd & { return H[i + (size_t)j * n]; };
  double anorm = 0.0;
  for (const cd &z : A) anorm = std::max(anorm, std::abs(z));
  const double eps = std::numeric_limits<double>::epsilon();

  for (int i = 0; i < n; ++i) w[i] = h(i, i);
  // eigenvectors of the triangular T, then through Z
  const double small = eps * std::max(anorm, 1e-300);
  std::vector<cd> y(n);
  for (int p = 0; p < n; ++p) {
    for (int i = 0; i < n; ++i) y[i] = 0.0;
    y[p] = 1.0;
    for (int i = p - 1; i >= 0; --i) {
      cd s(0);
      for (int l = i + 1; l <= p; ++l) s += h(i, l) * y[l];
      cd den = h(i, i) - w[p];
      if (std::abs(den) < small) den = small;
      y[i] = -s / den;
    }
    double nrm = 0.0;
    for (int r = 0; r < n; ++r) {
      cd s(0);
      for (int l = 0; l <= p; ++l) s += Z[r + (size_t)l * n] * y[l];
      vecs[r + (size_t)p * n] = s;
      nrm += std::norm(s);
    }
    nrm = std::sqrt(nrm);
    if (nrm > 0)
      for (int r = 0; r < n; ++r) vecs[r + (size_t)p * n] /= nrm;
  }
  return true;
}

bool eigh_jacobi(int n, const std::vector<cd> &A0, std::vector<double> &E, std::vector<cd> &U) {
  std::vector<cd> A(A0.begin(), A0.begin() + (size_t)n * n);
  auto a = [&](int i, int j) -> cd & { return A[i + (size_t)j * n]; };
  U.assign((size_t)n * n, cd(0));
  for (int i = 0; i < n; ++i) U[i + (size_t)i * n] = 1.0;
  for (int i = 0; i < n; ++i)  // symmetrise: use the Hermitian part
    for (int j = i; j < n; ++j) {
      const cd h = 0.5 * (a(i, j) + std::conj(a(j, i)));
      a(i, j) = h;
      a(j, i) = std::conj(h);
    }
  double fro = 0.0;
  for (const cd &z : A) fro += std::norm(z);
  fro = std::sqrt(fro);
  bool ok = false;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) off += std::norm(a(i, j));
    if (std::sqrt(2.0 * off) <= 1e-15 * fro || fro == 0.0) {
      ok = true;
      break;
    }
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        const cd apq = a(p, q);
        const double mag = std::abs(apq);
        if (mag == 0.0) continue;
        // rotation in the (p, q) plane zeroing a(p, q): with apq = mag e^{i phi},
        // the real symmetric 2x2 problem [[app, mag], [mag, aqq]]
        const cd ph = apq / mag;
        const double app = a(p, p).real(), aqq = a(q, q).real();
        const double tau = (aqq - app) / (2.0 * mag);
        const double t = (tau >= 0 ? 1.0 : -1.0) / (std::abs(tau) + std::sqrt(1.0 + tau * tau));
        const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
        // J: columns p, q of the identity replaced by (c, -sn conj(ph)) and (sn ph, c)
        for (int k = 0; k < n; ++k) {  // A <- A J
          const cd akp = a(k, p), akq = a(k, q);
          a(k, p) = c * akp - sn * std::conj(ph) * akq;
          a(k, q) = sn * ph * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {  // A <- J^H A
          const cd apk = a(p, k), aqk = a(q, k);
          a(p, k) = c * apk - sn * ph * aqk;
          a(q, k) = sn * std::conj(ph) * apk + c * aqk;
        }
        a(p, q) = 0.0;
        a(q, p) = 0.0;
        for (int k = 0; k < n; ++k) {  // U <- U J
          const cd ukp = U[k + (size_t)p * n], ukq = U[k + (size_t)q * n];
          U[k + (size_t)p * n] = c * ukp - sn * std::conj(ph) * ukq;
          U[k + (size_t)q * n] = sn * ph * ukp + c * ukq;
        }
      }
  }
  // ascending eigenvalues
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int x, int y) { return a(x, x).real() < a(y, y).real(); });
  E.assign(n, 0.0);
  std::vector<cd> Us((size_t)n * n);
  for (int c = 0; c < n; ++c) {
    E[c] = a(order[c], order[c]).real();
    for (int r = 0; r < n; ++r) Us[r + (size_t)c * n] = U[r + (size_t)order[c] * n];
  }
  U.swap(Us);
  return ok;
}

bool lu_solve(int n, const std::vector<cd> &A0, std::vector<cd> &x) {
  std::vector<cd> A(A0.begin(), A0.begin() + (size_t)n * n);
  auto a = [&](int i, int j) -> cd & { return A[i + (size_t)j * n]; };
  for (int k = 0; k < n; ++k) {
    int p = k;
    for (int i = k + 1; i < n; ++i)
      if (std::abs(a(i, k)) > std::abs(a(p, k))) p = i;
    if (std::abs(a(p, k)) == 0.0) return false;
    if (p != k) {
      for (int j = 0; j < n; ++j) std::swap(a(k, j), a(p, j));
      std::swap(x[k], x[p]);
    }
    for (int i = k + 1; i < n; ++i) {
      const cd f = a(i, k) / a(k, k);
      if (f == cd(0)) continue;
      for (int j = k + 1; j < n; ++j) a(i, j) -= f * a(k, j);
      x[i] -= f * x[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    cd s = x[i];
    for (int j = i + 1; j < n; ++j) s -= a(i, j) * x[j];
    x[i] = s / a(i, i);
  }
  return true;
}

int orthonormalise_columns(int rows, int cols, std::vector<cd> &P, double drop_tol) {
  int kept = 0;
  std::vector<cd> h(cols);
  for (int c = 0; c < cols; ++c) {
    cd *col = &P[(size_t)c * rows];
    double n0 = 0.0;
    for (int r = 0; r < rows; ++r) n0 += std::norm(col[r]);
    n0 = std::sqrt(n0);
    if (n0 == 0.0) continue;
    for (int pass = 0; pass < 2; ++pass) {
      for (int q = 0; q < kept; ++q) {
        const cd *u = &P[(size_t)q * rows];
        cd s(0);
        for (int r = 0; r < rows; ++r) s += std::conj(u[r]) * col[r];
        h[q] = s;
      }
      for (int q = 0; q < kept; ++q) {
        const cd *u = &P[(size_t)q * rows];
        for (int r = 0; r < rows; ++r) col[r] -= h[q] * u[r];
      }
    }
    double nn = 0.0;
    for (int r = 0; r < rows; ++r) nn += std::norm(col[r]);
    nn = std::sqrt(nn);
    if (nn <= drop_tol * n0) continue;
    cd *dst = &P[(size_t)kept * rows];
    for (int r = 0; r < rows; ++r) dst[r] = col[r] / nn;
    ++kept;
  }
  return kept;
}

bool HessSolver::solve(const std::vector<cd> &H, int ld, int k, cd sigma, const std::vector<cd> &rhs, std::vector<cd> &y) {
  ar.resize((size_t)k * k);
  ai.resize((size_t)k * k);
  br.resize(k);
  bi.resize(k);
  for (int c = 0; c < k; ++c)
    for (int r = 0; r <= std::min(c + 1, k - 1); ++r) {  // rows below c + 1 are never read
      const cd v = H[(size_t)c * ld + r];
      ar[(size_t)c * k + r] = v.real();
      ai[(size_t)c * k + r] = v.imag();
    }
  for (int i = 0; i < k; ++i) {
    ar[(size_t)i * k + i] += sigma.real();
    ai[(size_t)i * k + i] += sigma.imag();
    br[i] = rhs[i].real();
    bi[i] = rhs[i].imag();
  }
  for (int i = 0; i + 1 < k; ++i) {
    // rows i and i+1 only (Hessenberg); pivot on the larger modulus
    const size_t d0 = (size_t)i * k + i, d1 = d0 + 1;
    if (ar[d1] * ar[d1] + ai[d1] * ai[d1] > ar[d0] * ar[d0] + ai[d0] * ai[d0]) {
      for (int c = i; c < k; ++c) {
        std::swap(ar[(size_t)c * k + i], ar[(size_t)c * k + i + 1]);
        std::swap(ai[(size_t)c * k + i], ai[(size_t)c * k + i + 1]);
      }
      std::swap(br[i], br[i + 1]);
      std::swap(bi[i], bi[i + 1]);
    }
    const double pr = ar[d0], pi = ai[d0], pn = pr * pr + pi * pi;
    if (pn == 0.0) return false;
    // f = A[i+1][i] / p
    const double fr = (ar[d1] * pr + ai[d1] * pi) / pn, fi = (ai[d1] * pr - ar[d1] * pi) / pn;
    if (fr != 0.0 || fi != 0.0) {
      for (int c = i; c < k; ++c) {
        const size_t u = (size_t)c * k + i;
        ar[u + 1] -= fr * ar[u] - fi * ai[u];
        ai[u + 1] -= fr * ai[u] + fi * ar[u];
      }
      br[i + 1] -= fr * br[i] - fi * bi[i];
      bi[i + 1] -= fr * bi[i] + fi * br[i];
    }
  }
  y.resize(k);
  for (int i = k - 1; i >= 0; --i) {
    double sr = br[i], si = bi[i];
    for (int c = i + 1; c < k; ++c) {
      const size_t u = (size_t)c * k + i;
      sr -= ar[u] * y[c].real() - ai[u] * y[c].imag();
      si -= ar[u] * y[c].imag() + ai[u] * y[c].real();
    }
    const size_t dd = (size_t)i * k + i;
    const double pr = ar[dd], pi = ai[dd], pn = pr * pr + pi * pi;
    if (pn == 0.0) return false;
    const double yr = (sr * pr + si * pi) / pn, yi = (si * pr - sr * pi) / pn;
    if (!std::isfinite(yr) || !std::isfinite(yi)) return false;
    y[i] = cd(yr, yi);
  }
  return true;
}

}  // namespace heom
