// Host dense real Schur decomposition with reordering, for the small p x p
// projected matrix of the Krylov-Schur restart (p <= a few hundred).
#pragma once

namespace dcgs2 {

// Real Schur form of a general p x p matrix A (column-major, lda): A = Z T Z^T.
// T overwrites A (quasi-upper-triangular, 2x2 blocks only for complex pairs, in
// standard form a = d, b c < 0); Z (ldz) receives the orthogonal factor.
// Returns 0 on success, 1 if the QR iteration failed to converge.
int real_schur(int p, double* A, int lda, double* Z, int ldz);

// Reorder a real Schur form so that the `count` eigenvalues of largest magnitude
// lead, by decreasing magnitude.  The cut moves down past every eigenvalue whose
// magnitude is within cut_gap * |lambda_max| of the last selected one (so a
// complex pair is never split).  T and Z are updated in place (T <- G^T T G,
// Z <- Z G).  Returns the size of the leading block, or -1 on failure.
int reorder_schur_by_magnitude(int p, double* T, int ldt, double* Z, int ldz, int count,
                               double cut_gap);

// Eigenvalues of a standardised real quasi-triangular T, in diagonal order.
void schur_eigenvalues(int p, const double* T, int ldt, double* re, double* im);

}  // namespace dcgs2
