// Test-only C wrapper around the host Schur routines (compiled with g++ by
// tests/test_schur_host.py; not part of the library).
#include "schur.h"
extern "C" {
int shim_real_schur(int p, double* A, int lda, double* Z, int ldz) {
  return dcgs2::real_schur(p, A, lda, Z, ldz);
}
int shim_reorder(int p, double* T, int ldt, double* Z, int ldz, int count, double gap) {
  return dcgs2::reorder_schur_by_magnitude(p, T, ldt, Z, ldz, count, gap);
}
void shim_eigs(int p, const double* T, int ldt, double* re, double* im) {
  dcgs2::schur_eigenvalues(p, T, ldt, re, im);
}
}
