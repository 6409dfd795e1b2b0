// Complex Schur decomposition of a small dense matrix: Householder reduction
// to Hessenberg form, then single-shift QR with Wilkinson shifts and Givens
// rotations (Golub & Van Loan, Ch. 7), plus adjacent swaps of the triangular
// factor for reordering.  Used for the m x m Rayleigh quotient of the
// Krylov-Schur restart (the paper uses ARPACK's implicitly restarted Arnoldi,
// Sec. 4; Krylov-Schur is an equivalent restart built on this Schur form).
#include "dense.h"

#include <cmath>
#include <limits>

namespace fq {

namespace {

// Givens rotation G = [[c, s], [-conj(s), c]] with c real and
// G [x; y] = [r; 0].
void givens(zd x, zd y, double* c, zd* s) {
  const double ax = std::abs(x), ay = std::abs(y);
  if (ay == 0.0) {
    *c = 1.0;
    *s = zd(0, 0);
    return;
  }
  if (ax == 0.0) {
    *c = 0.0;
    *s = std::conj(y) / ay;
    return;
  }
  const double r = std::hypot(ax, ay);
  *c = ax / r;
  *s = (x / ax) * std::conj(y) / r;
}

// The rotations work on the interleaved (re, im) doubles of the column-major
// storage, written out in real arithmetic so that the compiler emits plain
// FMAs (and vectorises the column form over rows).

// rows k, k+1 of A, columns [j0, j1):  A <- G A
void rot_rows(ZMat& A, int k, int j0, int j1, double c, zd s) {
  const double sr = s.real(), si = s.imag();
  double* p = reinterpret_cast<double*>(A.a.data()) + 2 * (size_t(j0) * A.ld + k);
  const size_t step = 2 * size_t(A.ld);
  for (int j = j0; j < j1; ++j, p += step) {
    const double ar = p[0], ai = p[1], br = p[2], bi = p[3];
    p[0] = c * ar + (sr * br - si * bi);  // c a + s b
    p[1] = c * ai + (sr * bi + si * br);
    p[2] = c * br - (sr * ar + si * ai);  // -conj(s) a + c b
    p[3] = c * bi - (sr * ai - si * ar);
  }
}

// columns k, k+1 of A, rows [i0, i1):  A <- A G^H
void rot_cols(ZMat& A, int k, int i0, int i1, double c, zd s) {
  const double sr = s.real(), si = s.imag();
  double* __restrict__ pa = reinterpret_cast<double*>(A.a.data()) + 2 * (size_t(k) * A.ld);
  double* __restrict__ pb = pa + 2 * size_t(A.ld);
  for (int i = i0; i < i1; ++i) {
    const double ar = pa[2 * i], ai = pa[2 * i + 1], br = pb[2 * i], bi = pb[2 * i + 1];
    pa[2 * i] = c * ar + (sr * br + si * bi);  // c a + conj(s) b
    pa[2 * i + 1] = c * ai + (sr * bi - si * br);
    pb[2 * i] = c * br - (sr * ar - si * ai);  // -s a + c b
    pb[2 * i + 1] = c * bi - (sr * ai + si * ar);
  }
}

// A rotation of columns (k, k+1) of Z, recorded during the QR sweeps.
struct ZRot {
  int k;
  double c;
  zd s;
};

// Z <- Z G_1^H G_2^H ... for the recorded rotations in order.  Applied
// after the iteration on a copy of Z with the real and imaginary parts in
// separate arrays (the rotation of two columns is then four contiguous
// streams, which the compiler vectorises), a block of 64 rows at a time (the
// block's two columns of each rotation stay in cache across the rotations).
void apply_z_rotations(ZMat& Z, const std::vector<ZRot>& rots) {
  const int n = Z.n;
  std::vector<double> re(size_t(n) * n), im(size_t(n) * n);
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) {
      re[size_t(j) * n + i] = Z(i, j).real();
      im[size_t(j) * n + i] = Z(i, j).imag();
    }
  for (int r0 = 0; r0 < n; r0 += 64) {
    const int r1 = r0 + 64 < n ? r0 + 64 : n;
    for (const ZRot& g : rots) {
      const double c = g.c, sr = g.s.real(), si = g.s.imag();
      double* __restrict__ ar = re.data() + size_t(g.k) * n;
      double* __restrict__ ai = im.data() + size_t(g.k) * n;
      double* __restrict__ br = ar + n;
      double* __restrict__ bi = ai + n;
      for (int i = r0; i < r1; ++i) {
        const double xr = ar[i], xi = ai[i], yr = br[i], yi = bi[i];
        ar[i] = c * xr + (sr * yr + si * yi);  // c a + conj(s) b
        ai[i] = c * xi + (sr * yi - si * yr);
        br[i] = c * yr - (sr * xr - si * xi);  // -s a + c b
        bi[i] = c * yi - (sr * xi + si * xr);
      }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = 0; i < n; ++i) Z(i, j) = zd(re[size_t(j) * n + i], im[size_t(j) * n + i]);
}

void hessenberg(ZMat& A, ZMat& Z) {
  const int n = A.n;
  std::vector<zd> v(n), p(n), q(n);
  std::vector<int> nz;  // rows where the reflector is non-zero
  nz.reserve(n);
  for (int k = 0; k + 2 < n; ++k) {
    // nothing below the subdiagonal (the Arnoldi part of a projected
    // matrix is Hessenberg already): no reflection
    double tail = 0.0;
    for (int i = k + 2; i < n; ++i) tail += std::norm(A(i, k));
    if (tail == 0.0) continue;
    const double xn = std::sqrt(tail + std::norm(A(k + 1, k)));
    const zd x0 = A(k + 1, k);
    const zd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : zd(1, 0);
    // v = x + ph*||x|| e1, P = I - 2 v v^H / (v^H v), P x = -ph ||x|| e1
    nz.clear();
    v[k + 1] = x0 + ph * xn;
    nz.push_back(k + 1);
    for (int i = k + 2; i < n; ++i) {
      v[i] = A(i, k);
      if (v[i] != zd(0, 0)) nz.push_back(i);
    }
    double vn = 0.0;
    for (int i : nz) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    const double tau = 2.0 / vn;
    // Only the rows (and columns) in nz change.  A Krylov-Schur restart
    // matrix (triangular block, one coupling row, Hessenberg rest) gives
    // two-entry reflectors, so these steps are O(n) instead of O(n^2).
    // A <- P A
    for (int j = 0; j < n; ++j) {
      zd s = 0;
      for (int i : nz) s += std::conj(v[i]) * A(i, j);
      s *= tau;
      for (int i : nz) A(i, j) -= v[i] * s;
    }
    // A <- A P, Z <- Z P, column by column (contiguous in memory):
    // p = A v, q = Z v, then column j -= tau * conj(v_j) * p (resp. q)
    for (int i = 0; i < n; ++i) {
      p[i] = 0;
      q[i] = 0;
    }
    for (int j : nz) {
      const zd vj = v[j];
      const zd* a = &A(0, j);
      const zd* z = &Z(0, j);
      for (int i = 0; i < n; ++i) {
        p[i] += a[i] * vj;
        q[i] += z[i] * vj;
      }
    }
    for (int j : nz) {
      const zd f = tau * std::conj(v[j]);
      zd* a = &A(0, j);
      zd* z = &Z(0, j);
      for (int i = 0; i < n; ++i) {
        a[i] -= p[i] * f;
        z[i] -= q[i] * f;
      }
    }
    for (int i = k + 2; i < n; ++i) A(i, k) = 0;
  }
}

}  // namespace

bool schur(ZMat& A, ZMat& Z) {
  const int n = A.n;
  Z = ZMat(n, n);
  for (int i = 0; i < n; ++i) Z(i, i) = 1;
  if (n <= 1) return true;
  hessenberg(A, Z);
  const double eps = std::numeric_limits<double>::epsilon();
  double anorm = 0.0;
  for (const zd& x : A.a) anorm = std::max(anorm, std::abs(x));
  const double tiny = anorm * eps * 1e-3 + std::numeric_limits<double>::min();
  int hi = n - 1;
  int iter = 0;
  const int max_iter = 60 * n;
  int total = 0;
  // Z does not enter the iteration: its rotations are recorded and applied
  // once at the end
  std::vector<ZRot> zrots;
  zrots.reserve(size_t(n) * 8);
  while (hi > 0) {
    // find the start l of the unreduced block ending at hi
    int l = hi;
    while (l > 0) {
      const double s = std::abs(A(l - 1, l - 1)) + std::abs(A(l, l));
      if (std::abs(A(l, l - 1)) <= eps * (s > 0 ? s : anorm) || std::abs(A(l, l - 1)) <= tiny) {
        A(l, l - 1) = 0;
        break;
      }
      --l;
    }
    if (l == hi) {
      --hi;
      iter = 0;
      continue;
    }
    if (++total > max_iter) {
      apply_z_rotations(Z, zrots);
      return false;
    }
    ++iter;
    // Wilkinson shift from the trailing 2x2 of the active block
    zd mu;
    if (iter % 11 == 0) {
      // exceptional shift
      mu = A(hi, hi) + zd(std::abs(A(hi, hi - 1)) * 0.75, std::abs(A(hi, hi - 1)) * 0.5);
    } else {
      const zd a = A(hi - 1, hi - 1), b = A(hi - 1, hi), c = A(hi, hi - 1), d = A(hi, hi);
      const zd tr = a + d, det = a * d - b * c;
      const zd disc = std::sqrt(tr * tr * 0.25 - det);
      const zd e1 = tr * 0.5 + disc, e2 = tr * 0.5 - disc;
      mu = std::abs(e1 - d) < std::abs(e2 - d) ? e1 : e2;
    }
    zd x = A(l, l) - mu, y = A(l + 1, l);
    for (int k = l; k < hi; ++k) {
      double c;
      zd s;
      givens(x, y, &c, &s);
      rot_rows(A, k, k > l ? k - 1 : l, n, c, s);
      rot_cols(A, k, 0, std::min(k + 3, hi + 1), c, s);
      zrots.push_back({k, c, s});
      if (k > l) A(k + 1, k - 1) = 0;
      if (k + 1 < hi) {
        x = A(k + 1, k);
        y = A(k + 2, k);
      }
    }
  }
  apply_z_rotations(Z, zrots);
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) A(i, j) = 0;
  return true;
}

void schur_swap(ZMat& T, ZMat& Z, int k) {
  const int n = T.n;
  const zd t11 = T(k, k), t22 = T(k + 1, k + 1), t12 = T(k, k + 1);
  const zd y = t22 - t11;
  if (std::abs(t12) == 0.0 && std::abs(y) == 0.0) return;
  double c;
  zd s;
  givens(t12, y, &c, &s);
  rot_rows(T, k, k, n, c, s);
  rot_cols(T, k, 0, k + 2, c, s);
  rot_cols(Z, k, 0, n, c, s);
  T(k, k) = t22;
  T(k + 1, k + 1) = t11;
  T(k + 1, k) = 0;
}

std::vector<zd> tri_eigvec(const ZMat& T, int i) {
  const int n = T.n;
  std::vector<zd> y(n, zd(0, 0));
  y[i] = 1;
  double tn = 0.0;
  for (const zd& x : T.a) tn = std::max(tn, std::abs(x));
  const double small = std::max(tn, 1e-300) * std::numeric_limits<double>::epsilon();
  const zd lam = T(i, i);
  for (int j = i - 1; j >= 0; --j) {
    zd s = 0;
    for (int l = j + 1; l <= i; ++l) s += T(j, l) * y[l];
    zd den = T(j, j) - lam;
    if (std::abs(den) < small) den = small;
    y[j] = -s / den;
  }
  return y;
}

}  // namespace fq
