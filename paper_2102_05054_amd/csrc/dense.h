// Small dense complex linear algebra on the host (the m x m projected matrix
// of the Krylov-Schur restart, m <= a few hundred).  Column-major storage.
#pragma once

#include <complex>
#include <vector>

namespace fq {

using zd = std::complex<double>;

struct ZMat {
  // Columns are ld = rows + 2 apart: with a power-of-two stride the row
  // rotations of the QR sweeps (two adjacent entries in each of many columns)
  // map every column onto the same cache sets (measured 1.5x slower Schur
  // form at 256 x 256).  Padding entries stay zero.
  int n = 0, m = 0, ld = 0;  // rows, cols, leading dimension
  std::vector<zd> a;
  ZMat() = default;
  ZMat(int rows, int cols) : n(rows), m(cols), ld(rows + 2), a(size_t(rows + 2) * cols, zd(0, 0)) {}
  zd& operator()(int i, int j) { return a[size_t(j) * ld + i]; }
  const zd& operator()(int i, int j) const { return a[size_t(j) * ld + i]; }
};

// Complex Schur form A = Z T Z^H (A: n x n, overwritten by T).  Z starts as
// identity.  Returns false if the QR iteration fails to converge.
bool schur(ZMat& A, ZMat& Z);

// Reorder the Schur form so that positions 0..nsel-1 hold the eigenvalues
// chosen by `better` (a strict weak order: better(x, y) = x goes first),
// greedily: position i receives the best remaining eigenvalue.
template <class Better>
void schur_sort(ZMat& T, ZMat& Z, int nsel, Better better);

// Swap diagonal entries k and k+1 of the upper-triangular T (and update Z).
void schur_swap(ZMat& T, ZMat& Z, int k);

// Eigenvector y (length n) of upper-triangular T for eigenvalue index i:
// y_i = 1, y_j = 0 for j > i, back substitution above.
std::vector<zd> tri_eigvec(const ZMat& T, int i);

template <class Better>
void schur_sort(ZMat& T, ZMat& Z, int nsel, Better better) {
  const int n = T.n;
  for (int pos = 0; pos < nsel && pos < n; ++pos) {
    int best = pos;
    for (int j = pos + 1; j < n; ++j)
      if (better(T(j, j), T(best, best))) best = j;
    for (int j = best; j > pos; --j) schur_swap(T, Z, j - 1);
  }
}

}  // namespace fq
