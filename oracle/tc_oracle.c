/*
 * Reference CPU contraction -- TEST INFRASTRUCTURE ONLY.
 *
 * This file is the oracle that the GPU library is checked against.  It is
 * plain, slow and written to be read against the paper ("Towards an
 * Efficient Use of the BLAS Library for Multilinear Tensor Contractions",
 * Di Napoli, Fabregat-Traver, Quintana-Orti, Bientinesi): a contraction is
 * the sum, over every value of the repeated (contracted) indices, of the
 * product of the two operands' entries (Sec. 2.3 and Appendix A, the
 * Einstein convention; Sec. 2.2 for the matrix product c_ij = sum_h a_ih b_hj).
 * The BLAS convention C <- alpha*op + beta*C (Sec. 2.1, GEMM definition) is
 * applied on top; beta == 0 never reads C.
 *
 * Nothing here is shared with the GPU path: labels are parsed again, every
 * output entry is a nested loop over the contracted multi-index, and the
 * accumulation is a plain running sum in FP64 (compiled with
 * -ffp-contract=off so that no FMA is formed).  A compensated variant (Dot2:
 * error-free TwoProduct via fma and TwoSum, Ogita, Rump and Oishi 2005) is
 * the accuracy reference for tolerance checks, and an |A||B| variant gives
 * the denominator of componentwise error bounds.
 *
 * Only tests, the smoke check and the CPU leg of the benchmark may use it.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TCO_MAX_RANK 24

enum { TCO_PLAIN = 0, TCO_DOT2 = 1, TCO_ABS = 2 };

typedef struct {
  int ncontr;                      /* number of contracted labels            */
  int64_t cext[TCO_MAX_RANK];      /* extent of each contracted label        */
  int64_t cstrA[TCO_MAX_RANK];     /* its stride in A                        */
  int64_t cstrB[TCO_MAX_RANK];     /* its stride in B                        */
  int rC;
  int64_t oext[TCO_MAX_RANK];      /* extents of C's modes                   */
  int64_t ostrA[TCO_MAX_RANK];     /* stride in A of C's mode (0 if absent)  */
  int64_t ostrB[TCO_MAX_RANK];     /* stride in B of C's mode (0 if absent)  */
  int64_t ostrC[TCO_MAX_RANK];     /* stride in C                            */
} tco_layout;

static int find_label(int rank, const int32_t* lab, int32_t l) {
  for (int i = 0; i < rank; ++i)
    if (lab[i] == l) return i;
  return -1;
}

static int has_repeats(int rank, const int32_t* lab) {
  for (int i = 0; i < rank; ++i)
    for (int j = i + 1; j < rank; ++j)
      if (lab[i] == lab[j]) return 1;
  return 0;
}

/* Sort the labels into output modes and contracted modes.  Every label of A
 * must occur in B or C, every label of B in A or C, every label of C in A or
 * B, equal labels must have equal extents, and no tensor repeats a label. */
static int build_layout(int rA, const int64_t* eA, const int64_t* sA, const int32_t* lA,
                        int rB, const int64_t* eB, const int64_t* sB, const int32_t* lB,
                        int rC, const int64_t* eC, const int64_t* sC, const int32_t* lC,
                        tco_layout* L) {
  if (rA < 0 || rB < 0 || rC < 0 || rA > TCO_MAX_RANK || rB > TCO_MAX_RANK || rC > TCO_MAX_RANK)
    return -1;
  if (has_repeats(rA, lA) || has_repeats(rB, lB) || has_repeats(rC, lC)) return -2;
  memset(L, 0, sizeof(*L));
  for (int i = 0; i < rA; ++i) {
    int jb = find_label(rB, lB, lA[i]), jc = find_label(rC, lC, lA[i]);
    if (jb < 0 && jc < 0) return -3;
    if (jb >= 0 && eB[jb] != eA[i]) return -4;
    if (jc >= 0 && eC[jc] != eA[i]) return -4;
    if (jb >= 0 && jc < 0) {            /* contracted: in A and B, not in C */
      L->cext[L->ncontr] = eA[i];
      L->cstrA[L->ncontr] = sA[i];
      L->cstrB[L->ncontr] = sB[jb];
      L->ncontr++;
    }
  }
  for (int i = 0; i < rB; ++i) {
    int ja = find_label(rA, lA, lB[i]), jc = find_label(rC, lC, lB[i]);
    if (ja < 0 && jc < 0) return -3;
    if (jc >= 0 && eC[jc] != eB[i]) return -4;
  }
  L->rC = rC;
  for (int i = 0; i < rC; ++i) {
    int ja = find_label(rA, lA, lC[i]), jb = find_label(rB, lB, lC[i]);
    if (ja < 0 && jb < 0) return -3;
    L->oext[i] = eC[i];
    L->ostrC[i] = sC[i];
    L->ostrA[i] = ja >= 0 ? sA[ja] : 0;
    L->ostrB[i] = jb >= 0 ? sB[jb] : 0;
  }
  return 0;
}

static void two_sum(double a, double b, double* s, double* e) {
  double x = a + b, z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}

/* Sum over the contracted multi-index for one output entry whose A and B
 * base offsets are baseA and baseB.  The odometer runs over the contracted
 * labels in the order they appear in A (first label fastest). */
static double contracted_sum(const tco_layout* L, const double* A, const double* B,
                             int64_t baseA, int64_t baseB, int mode) {
  int64_t total = 1;
  for (int q = 0; q < L->ncontr; ++q) total *= L->cext[q];
  if (total == 0) return 0.0;
  int64_t idx[TCO_MAX_RANK] = {0};
  int64_t oa = baseA, ob = baseB;
  double s = 0.0, c = 0.0;
  for (int64_t t = 0; t < total; ++t) {
    double a = A[oa], b = B[ob];
    if (mode == TCO_PLAIN) {
      s = s + a * b;
    } else if (mode == TCO_ABS) {
      s = s + fabs(a) * fabs(b);
    } else {
      double p = a * b;
      double pe = fma(a, b, -p);
      double e;
      two_sum(s, p, &s, &e);
      c = c + (e + pe);
    }
    /* advance the odometer */
    for (int q = 0; q < L->ncontr; ++q) {
      idx[q]++;
      oa += L->cstrA[q];
      ob += L->cstrB[q];
      if (idx[q] < L->cext[q]) break;
      oa -= L->cstrA[q] * L->cext[q];
      ob -= L->cstrB[q] * L->cext[q];
      idx[q] = 0;
    }
  }
  return mode == TCO_DOT2 ? s + c : s;
}

/* Full contraction: C <- alpha * sum(A*B) + beta * C over every entry of C.
 * mode: 0 plain FP64 sum, 1 compensated (Dot2), 2 sum of |a||b| (alpha and
 * beta then ignored: C receives the raw |A||B| contraction).  Returns 0 on
 * success and a negative code on an invalid label or extent set. */
int tco_contract(int rA, const int64_t* eA, const int64_t* sA, const int32_t* lA,
                 int rB, const int64_t* eB, const int64_t* sB, const int32_t* lB,
                 int rC, const int64_t* eC, const int64_t* sC, const int32_t* lC,
                 const double* A, const double* B, double* C,
                 double alpha, double beta, int mode, int nthreads) {
  tco_layout L;
  int rc = build_layout(rA, eA, sA, lA, rB, eB, sB, lB, rC, eC, sC, lC, &L);
  if (rc) return rc;
  int64_t nout = 1;
  for (int i = 0; i < rC; ++i) nout *= eC[i];
  if (nout == 0) return 0;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 64)
#endif
  for (int64_t lin = 0; lin < nout; ++lin) {
    int64_t rem = lin, oa = 0, ob = 0, oc = 0;
    for (int i = 0; i < L.rC; ++i) {      /* column-major decode of C's index */
      int64_t v = rem % L.oext[i];
      rem /= L.oext[i];
      oa += v * L.ostrA[i];
      ob += v * L.ostrB[i];
      oc += v * L.ostrC[i];
    }
    double s = contracted_sum(&L, A, B, oa, ob, mode);
    if (mode == TCO_ABS)
      C[oc] = s;
    else
      C[oc] = beta == 0.0 ? alpha * s : alpha * s + beta * C[oc];
  }
  return 0;
}

/* Selected entries only: for each of the n output multi-indices in cidx
 * (row-major n x rC array, one row per entry, in C's label order) return the
 * plain or compensated sum in sum[] and the |A||B| sum in abssum[] (either
 * pointer may be NULL).  Used where the full contraction is too large. */
int tco_contract_entries(int rA, const int64_t* eA, const int64_t* sA, const int32_t* lA,
                         int rB, const int64_t* eB, const int64_t* sB, const int32_t* lB,
                         int rC, const int64_t* eC, const int32_t* lC,
                         const double* A, const double* B, int64_t n, const int64_t* cidx,
                         double* sum, double* abssum, int compensated, int nthreads) {
  int64_t dummyC[TCO_MAX_RANK];
  for (int i = 0; i < rC && i < TCO_MAX_RANK; ++i) dummyC[i] = 0;
  tco_layout L;
  int rc = build_layout(rA, eA, sA, lA, rB, eB, sB, lB, rC, eC, dummyC, lC, &L);
  if (rc) return rc;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 16)
#endif
  for (int64_t e = 0; e < n; ++e) {
    int64_t oa = 0, ob = 0;
    for (int i = 0; i < L.rC; ++i) {
      int64_t v = cidx[e * rC + i];
      oa += v * L.ostrA[i];
      ob += v * L.ostrB[i];
    }
    if (sum) sum[e] = contracted_sum(&L, A, B, oa, ob, compensated ? TCO_DOT2 : TCO_PLAIN);
    if (abssum) abssum[e] = contracted_sum(&L, A, B, oa, ob, TCO_ABS);
  }
  return 0;
}

/* Out-of-place reordering of a tensor's storage: Y[addrY(idx)] = X[addrX(idx)]
 * for every multi-index idx over the given extents (the copy step that the
 * paper places before GEMM when a slice has no unit-stride mode, Sec. 3.1 F1). */
int tco_permute(int rank, const int64_t* ext, const int64_t* sX, const int64_t* sY,
                const double* X, double* Y) {
  if (rank < 0 || rank > TCO_MAX_RANK) return -1;
  int64_t total = 1;
  for (int i = 0; i < rank; ++i) total *= ext[i];
  for (int64_t lin = 0; lin < total; ++lin) {
    int64_t rem = lin, ox = 0, oy = 0;
    for (int i = 0; i < rank; ++i) {
      int64_t v = rem % ext[i];
      rem /= ext[i];
      ox += v * sX[i];
      oy += v * sY[i];
    }
    Y[oy] = X[ox];
  }
  return 0;
}

int tco_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
