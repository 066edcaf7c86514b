/* Host driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of
 * the library's host code (exponents, hierarchy enumeration and pruning,
 * neighbour tables, dictionary, argument checks, error plumbing).  Calls
 * the C ABI only; prints one line per check and exits non-zero on the first
 * wrong result.  Several host threads query one handle at once. */
#include <math.h>
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "heom.h"

static int failures = 0;
#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      printf("FAIL %s:%d: ", __FILE__, __LINE__); \
      printf(__VA_ARGS__);                     \
      printf("\n");                            \
      failures++;                              \
    }                                          \
  } while (0)

static long binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  long r = 1;
  for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
  return r;
}

/* Jordan-Wigner annihilation operators of `modes` fermionic modes, d = 2^modes,
 * basis |n_0 n_1 ...> with index bits n_k. */
static void jw_annihilation(int modes, int k, double *out) {
  int d = 1 << modes;
  memset(out, 0, sizeof(double) * 2 * d * d);
  for (int col = 0; col < d; ++col) {
    if (!(col >> k & 1)) continue;
    int row = col & ~(1 << k);
    int s = 0;
    for (int j = 0; j < k; ++j) s += col >> j & 1;
    out[2 * (row * d + col)] = (s & 1) ? -1.0 : 1.0;
  }
}

typedef struct {
  heom_hier *h;
  int64_t n;
  int tid;
  int ok;
} thread_arg;

/* Queries one shared handle; each thread also provokes its own error and
 * checks that heom_last_error() reports that error, not another thread's. */
static void *query_thread(void *p) {
  thread_arg *a = (thread_arg *)p;
  a->ok = 1;
  for (int it = 0; it < 200; ++it) {
    heom_info info;
    if (heom_hierarchy_info(a->h, &info) != HEOM_OK || info.n_ado != a->n) a->ok = 0;
    int32_t ids[3] = {(a->tid + it) % 8, 8 + (it % 8), 30};
    int64_t idx = -2;
    int32_t sign = 0;
    if (heom_ado_index(a->h, NULL, ids, 3, &idx, &sign) != HEOM_OK || idx < 0 || (sign != 1 && sign != -1)) a->ok = 0;
    double kappa[4], zeta[4];
    int bad = 65 + a->tid;
    if (heom_pade_params(HEOM_FERMION, HEOM_PADE, bad, kappa, zeta) != HEOM_ERR_ARG) a->ok = 0;
    const char *msg = heom_last_error();
    if (!msg || !strstr(msg, "pade_params")) a->ok = 0;
  }
  return NULL;
}

long stub_device_allocations(void);

typedef struct {
  heom_hier *h;
  int ok;
} prep_arg;

/* The first heom_prepare on a fresh handle, from several threads at once. */
static void *prepare_thread(void *p) {
  prep_arg *a = (prep_arg *)p;
  a->ok = heom_prepare(a->h) == HEOM_OK;
  return NULL;
}

int main(void) {
  /* ---- exponents */
  double kappa[8], zeta[8];
  CHECK(heom_pade_params(HEOM_FERMION, HEOM_PADE, 1, kappa, zeta) == HEOM_OK, "pade n=1");
  CHECK(fabs(kappa[0] - 1.5) < 1e-12 && fabs(zeta[0] - sqrt(12.0)) < 1e-12, "fermi pade N=1: %g %g", kappa[0], zeta[0]);
  CHECK(heom_pade_params(HEOM_BOSON, HEOM_PADE, 1, kappa, zeta) == HEOM_OK, "bose pade n=1");
  CHECK(fabs(kappa[0] - 2.5) < 1e-12 && fabs(zeta[0] - sqrt(60.0)) < 1e-12, "bose pade N=1: %g %g", kappa[0], zeta[0]);
  CHECK(heom_pade_params(HEOM_FERMION, HEOM_PADE, 8, kappa, zeta) == HEOM_OK, "pade n=8");
  CHECK(heom_pade_params(HEOM_FERMION, HEOM_PADE, 65, kappa, zeta) == HEOM_ERR_ARG, "pade n=65 rejected");
  CHECK(heom_pade_params(7, HEOM_PADE, 2, kappa, zeta) == HEOM_ERR_ARG, "bad kind rejected");
  CHECK(heom_pade_params(HEOM_FERMION, 9, 2, kappa, zeta) == HEOM_ERR_ARG, "bad method rejected");
  double xi[6], chi[6];
  CHECK(heom_exponents_drude_lorentz(0.1, 0.5, 0.5, 3, HEOM_MATSUBARA, xi, chi) == HEOM_OK, "DL exponents");
  CHECK(fabs(xi[0] - 0.0915243860856226) < 1e-12 && fabs(xi[1] + 0.05) < 1e-15, "DL xi_0 %g %g", xi[0], xi[1]);
  CHECK(heom_exponents_drude_lorentz(0.1, 0.5, 0.5, 0, HEOM_MATSUBARA, xi, chi) == HEOM_ERR_ARG, "DL n=0");
  CHECK(heom_exponents_drude_lorentz(0.1, 0.5, -1.0, 3, HEOM_MATSUBARA, xi, chi) == HEOM_ERR_ARG, "DL T<0");
  double ep[10], gp[10], em[10], gm[10];
  CHECK(heom_exponents_lorentz(2.0, 10.0, 1.0, 0.5, 5, HEOM_PADE, ep, gp, em, gm) == HEOM_OK, "Lorentz exponents");
  CHECK(heom_exponents_lorentz(2.0, 10.0, 1.0, 0.5, 0, HEOM_PADE, ep, gp, em, gm) == HEOM_ERR_ARG, "Lorentz n=0");
  CHECK(heom_exponents_lorentz(2.0, 10.0, 1.0, 0.5, 5, HEOM_PADE, NULL, gp, em, gm) == HEOM_ERR_ARG, "Lorentz NULL");

  /* ---- spin-boson: d = 2, 3 RI exponents, m_max = 4 -> 35 ADOs */
  double H2[8] = {0.5, 0, 0.5, 0, 0.5, 0, -0.5, 0};
  double sz[8] = {1, 0, 0, 0, 0, 0, -1, 0};
  int32_t u3[3] = {HEOM_U_RI, HEOM_U_RI, HEOM_U_RI};
  heom_bath sb = {HEOM_BOSON, sz, 3, u3, xi, chi, NULL, NULL, NULL, NULL};
  heom_hier *h = NULL;
  CHECK(heom_build_hierarchy(2, H2, 1, &sb, 4, 0, 1, NULL, &h) == HEOM_OK, "spin-boson build: %s", heom_last_error());
  heom_info info;
  CHECK(heom_hierarchy_info(h, &info) == HEOM_OK && info.n_ado == 35, "spin-boson N = %lld", (long long)info.n_ado);
  {
    int64_t N = info.n_ado, E = info.n_edges;
    int32_t *occ = malloc(sizeof(int32_t) * N * 3), *lev = malloc(sizeof(int32_t) * N * 2);
    uint64_t *mask = malloc(sizeof(uint64_t) * N);
    double *dec = malloc(sizeof(double) * 2 * N);
    int64_t *rp = malloc(sizeof(int64_t) * (N + 1));
    int32_t *col = malloc(sizeof(int32_t) * E), *kind = malloc(sizeof(int32_t) * E), *ex = malloc(sizeof(int32_t) * E),
            *mult = malloc(sizeof(int32_t) * E);
    CHECK(heom_hierarchy_ados(h, occ, mask, lev) == HEOM_OK, "ados");
    CHECK(heom_hierarchy_tables(h, dec, rp, col, kind, ex, mult) == HEOM_OK, "tables");
    CHECK(rp[0] == 0 && rp[N] == E, "row_ptr ends");
    for (int64_t a = 0; a < N; ++a) {
      int64_t idx = -2;
      int32_t sign = 0;
      CHECK(heom_ado_index(h, occ + 3 * a, NULL, 0, &idx, &sign) == HEOM_OK && idx == a && sign == 1, "lookup %lld", (long long)a);
      for (int64_t e = rp[a]; e < rp[a + 1]; ++e) CHECK(col[e] >= 0 && col[e] < N && (kind[e] == 0 || kind[e] == 1), "edge");
    }
    int32_t beyond[3] = {5, 0, 0};
    int64_t idx = 0;
    int32_t sign = 0;
    CHECK(heom_ado_index(h, beyond, NULL, 0, &idx, &sign) == HEOM_OK && idx == -1, "outside the hierarchy");
    free(occ); free(lev); free(mask); free(dec); free(rp); free(col); free(kind); free(ex); free(mult);
  }
  double x[8], y[8];
  CHECK(heom_apply(h, HEOM_FP64, x, y, 1, NULL, NULL) != HEOM_OK, "apply fails without device code");
  CHECK(heom_apply(h, HEOM_FP64, x, x, 1, NULL, NULL) == HEOM_ERR_ARG, "aliasing rejected");
  heom_free(h);

  /* ---- Anderson impurity: d = 4, 2 leads x 2 spins x 5 h x 2 nu = 40 exponents, n_max = 3 */
  double d4[2][32], H4[32];
  memset(H4, 0, sizeof(H4));
  H4[2 * (1 * 4 + 1)] = -5; H4[2 * (2 * 4 + 2)] = -5; H4[2 * (3 * 4 + 3)] = 0;  /* eps = -5, U = 10 */
  jw_annihilation(2, 0, d4[0]);
  jw_annihilation(2, 1, d4[1]);
  double epL[10], gpL[10], emL[10], gmL[10], epR[10], gpR[10], emR[10], gmR[10];
  CHECK(heom_exponents_lorentz(2.0, 10.0, 1.0, 0.5, 5, HEOM_PADE, epL, gpL, emL, gmL) == HEOM_OK, "left lead");
  CHECK(heom_exponents_lorentz(2.0, 10.0, -1.0, 0.5, 5, HEOM_PADE, epR, gpR, emR, gmR) == HEOM_OK, "right lead");
  heom_bath fb[4] = {
      {HEOM_FERMION, d4[0], 5, NULL, NULL, NULL, epL, gpL, emL, gmL},
      {HEOM_FERMION, d4[1], 5, NULL, NULL, NULL, epL, gpL, emL, gmL},
      {HEOM_FERMION, d4[0], 5, NULL, NULL, NULL, epR, gpR, emR, gmR},
      {HEOM_FERMION, d4[1], 5, NULL, NULL, NULL, epR, gpR, emR, gmR},
  };
  double P4[32];
  memset(P4, 0, sizeof(P4));
  for (int i = 0; i < 4; ++i) P4[2 * (i * 4 + i)] = (__builtin_popcount(i) & 1) ? -1.0 : 1.0;
  for (int parity = -1; parity <= 1; parity += 2) {
    CHECK(heom_build_hierarchy(4, H4, 4, fb, 0, 3, parity, P4, &h) == HEOM_OK, "SIAM build: %s", heom_last_error());
    CHECK(heom_hierarchy_info(h, &info) == HEOM_OK && info.n_ado == 10701, "SIAM N = %lld", (long long)info.n_ado);
    long expect = 0;
    for (int k = 0; k <= 3; ++k) expect += binom(40, k);
    CHECK(info.n_ado == expect, "binomial count");
    /* dictionary with an unsorted exponent list: sign of the reordering */
    int32_t ids[3] = {7, 2, 30};
    int64_t i1 = -2, i2 = -2;
    int32_t s1 = 0, s2 = 0;
    CHECK(heom_ado_index(h, NULL, ids, 3, &i1, &s1) == HEOM_OK && i1 >= 0, "lookup unsorted");
    int32_t ids2[3] = {2, 7, 30};
    CHECK(heom_ado_index(h, NULL, ids2, 3, &i2, &s2) == HEOM_OK && i2 == i1 && s1 == -s2, "one swap flips the sign");
    int32_t dup[2] = {3, 3};
    CHECK(heom_ado_index(h, NULL, dup, 2, &i1, &s1) != HEOM_OK || i1 == -1, "repeated exponent is no ADO");
    /* the table upload: once, whatever the number of threads asking */
    if (parity == 1) {
      long before = stub_device_allocations();
      CHECK(heom_prepare(h) == HEOM_OK, "prepare: %s", heom_last_error());
      long one = stub_device_allocations() - before;
      CHECK(one > 0, "prepare allocated the tables");
      CHECK(heom_prepare(h) == HEOM_OK && stub_device_allocations() - before == one, "second prepare is free");
      heom_hier *h2 = NULL;
      CHECK(heom_build_hierarchy(4, H4, 4, fb, 0, 3, parity, P4, &h2) == HEOM_OK, "second handle");
      before = stub_device_allocations();
      pthread_t tp[4];
      prep_arg pa[4];
      for (int t = 0; t < 4; ++t) {
        pa[t].h = h2; pa[t].ok = 0;
        pthread_create(&tp[t], NULL, prepare_thread, &pa[t]);
      }
      for (int t = 0; t < 4; ++t) {
        pthread_join(tp[t], NULL);
        CHECK(pa[t].ok, "concurrent prepare %d: %s", t, heom_last_error());
      }
      CHECK(stub_device_allocations() - before == one, "concurrent first prepares upload once: %ld vs %ld",
            stub_device_allocations() - before, one);
      heom_free(h2);
    }
    CHECK(heom_prepare(NULL) == HEOM_ERR_ARG, "prepare NULL");
    /* several threads on one handle */
    pthread_t th[4];
    thread_arg ta[4];
    for (int t = 0; t < 4; ++t) {
      ta[t].h = h; ta[t].n = info.n_ado; ta[t].tid = t; ta[t].ok = 0;
      pthread_create(&th[t], NULL, query_thread, &ta[t]);
    }
    for (int t = 0; t < 4; ++t) {
      pthread_join(th[t], NULL);
      CHECK(ta[t].ok, "thread %d", t);
    }
    heom_free(h);
  }
  /* pruned: eq:importance keeps fewer ADOs */
  CHECK(heom_build_hierarchy_pruned(4, H4, 4, fb, 0, 3, 1, P4, 3e-3, &h) == HEOM_OK, "pruned build");
  CHECK(heom_hierarchy_info(h, &info) == HEOM_OK && info.n_ado > 81 && info.n_ado < 10701, "pruned N = %lld",
        (long long)info.n_ado);
  heom_free(h);
  CHECK(heom_build_hierarchy_pruned(4, H4, 4, fb, 0, 3, 1, P4, -1.0, &h) == HEOM_ERR_ARG, "negative threshold");

  /* ---- argument checks */
  double Hbad[8] = {0, 0, 1, 0, 0, 0, 0, 0};  /* not Hermitian */
  CHECK(heom_build_hierarchy(2, Hbad, 1, &sb, 2, 0, 1, NULL, &h) == HEOM_ERR_ARG, "non-Hermitian H");
  CHECK(strstr(heom_last_error(), "Hermitian") != NULL, "message: %s", heom_last_error());
  CHECK(heom_build_hierarchy(2, NULL, 1, &sb, 2, 0, 1, NULL, &h) == HEOM_ERR_ARG, "NULL H");
  CHECK(heom_build_hierarchy(0, H2, 1, &sb, 2, 0, 1, NULL, &h) == HEOM_ERR_ARG, "d = 0");
  CHECK(heom_build_hierarchy(2, H2, 1, &sb, 2, 0, 3, NULL, &h) == HEOM_ERR_ARG, "parity 3");
  CHECK(heom_build_hierarchy(2, H2, 1, NULL, 2, 0, 1, NULL, &h) == HEOM_ERR_ARG, "NULL baths");
  heom_bath badb = sb;
  badb.kind = 5;
  CHECK(heom_build_hierarchy(2, H2, 1, &badb, 2, 0, 1, NULL, &h) == HEOM_ERR_ARG, "bad bath kind");
  int32_t ubad[3] = {HEOM_U_RI, 7, HEOM_U_RI};
  badb = sb;
  badb.u_type = ubad;
  CHECK(heom_build_hierarchy(2, H2, 1, &badb, 2, 0, 1, NULL, &h) == HEOM_ERR_ARG, "bad exponent type");
  /* parity operator: a fermionic operator that is not odd is rejected */
  heom_bath even_d = fb[0];
  even_d.op = H4;
  CHECK(heom_build_hierarchy(4, H4, 1, &even_d, 0, 2, 1, P4, &h) == HEOM_ERR_ARG, "even fermionic op");
  CHECK(heom_status_string(HEOM_ERR_NAN) != NULL, "status string");
  heom_free(NULL);

  printf(failures ? "host driver: %d failures\n" : "host driver: all checks passed\n", failures);
  return failures ? 1 : 0;
}
