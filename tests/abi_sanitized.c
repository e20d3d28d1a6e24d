/* Drives every entry point of the C ABI, for a build of the library whose host code carries
 * AddressSanitizer and UndefinedBehaviorSanitizer checks (built by build.py's build_sanitized;
 * run by tests/test_host_sanitizers.py and tests/test_gpu_host_sanitizers.py).
 *
 *   abi_sanitized          argument checks and error paths only (no device needed)
 *   abi_sanitized gpu      the same, then small solves on every path: restricted singlet and
 *                          triplet in each sigma precision, Davidson (pp and hh channels, warm
 *                          start, log callback, caller-driven iterations), direct solve,
 *                          correlation energy (both entry points), NTOs, the alpha-beta sector
 *                          (dense and density fitted) and the serving queue.
 *
 * Inputs are synthetic (a fixed linear congruential sequence): orbital energies with a gap and
 * small symmetric three-centre integrals, so that M - 2 mu W is definite. The numbers are checked
 * against each other (direct vs Davidson roots, the two correlation-energy entry points), not
 * against the oracle: the parity tests do that. Exit status 0 when every check holds; the
 * sanitizers abort the process on the first error they find. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pprpa.h"

static int fails = 0;

#define EXPECT(call, want)                                                                  \
  do {                                                                                      \
    pprpa_status s_ = (call);                                                               \
    if (s_ != (want)) {                                                                     \
      fprintf(stderr, "line %d: %s -> %d (%s), want %d\n", __LINE__, #call, (int)s_,         \
              pprpa_last_error(), (int)(want));                                             \
      ++fails;                                                                              \
    }                                                                                       \
  } while (0)

#define CHECK(cond)                                                        \
  do {                                                                     \
    if (!(cond)) {                                                         \
      fprintf(stderr, "line %d: check failed: %s\n", __LINE__, #cond);     \
      ++fails;                                                             \
    }                                                                      \
  } while (0)

static unsigned long long lcg_state = 12345;
static double uniform(void) { /* [0, 1) */
  lcg_state = lcg_state * 6364136223846793005ULL + 1442695040888963407ULL;
  return (double)(lcg_state >> 11) * (1.0 / 9007199254740992.0);
}

/* Occupied energies ascending below -0.4, virtual ascending above 0.2. */
static double* energies(int nmo, int nocc, double shift) {
  double* e = malloc(sizeof(double) * nmo);
  for (int i = 0; i < nocc; ++i) e[i] = -1.0 - 0.1 * (nocc - 1 - i) + shift;
  for (int a = 0; a < nmo - nocc; ++a) e[nocc + a] = 0.2 + 0.07 * a + shift;
  return e;
}

/* [naux][nmo][nmo], symmetric in (p, q), entries in [-scale/2, scale/2). */
static double* integrals(int naux, int nmo, double scale) {
  double* L = malloc(sizeof(double) * (size_t)naux * nmo * nmo);
  for (int P = 0; P < naux; ++P)
    for (int p = 0; p < nmo; ++p)
      for (int q = 0; q <= p; ++q) {
        double v = scale * (uniform() - 0.5);
        L[((size_t)P * nmo + p) * nmo + q] = v;
        L[((size_t)P * nmo + q) * nmo + p] = v;
      }
  return L;
}

static void cpu_checks(void) {
  for (int s = 0; s <= 8; ++s) CHECK(pprpa_strerror((pprpa_status)s) != NULL);
  CHECK(pprpa_last_error() != NULL);

  EXPECT(pprpa_build(NULL, NULL), PPRPA_EINVAL);
  pprpa_ctx* ctx = NULL;
  EXPECT(pprpa_build(NULL, &ctx), PPRPA_EINVAL);
  CHECK(ctx == NULL);

  const int nmo = 12, nocc = 4, naux = 10;
  double* eps = energies(nmo, nocc, 0.0);
  double* L = integrals(naux, nmo, 0.1);
  pprpa_build_args a;
  memset(&a, 0, sizeof a);
  a.nmo = nmo; a.nocc = nocc; a.naux = naux; a.eps = eps; a.Lpq = L;
  a.naux = 0;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  a.naux = naux; a.nocc = nmo + 1;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  a.nocc = nocc; a.mult = 7;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  a.mult = PPRPA_SINGLET; a.prec = 9;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  a.prec = PPRPA_FP64;
  double keep = eps[1];
  eps[1] = NAN;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  eps[1] = eps[0] - 1.0; /* occupied block out of order */
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  eps[1] = keep;
  a.nocc_act = nocc + 1;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  a.nocc_act = 0;
  a.Lpq = NULL;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_EINVAL);
  CHECK(ctx == NULL);

  pprpa_build_ab_args b;
  memset(&b, 0, sizeof b);
  EXPECT(pprpa_build_ab(NULL, &ctx), PPRPA_EINVAL);
  EXPECT(pprpa_build_ab(&b, NULL), PPRPA_EINVAL);
  b.nmo = nmo; b.naux = naux; b.nocc_a = nmo; b.nocc_b = 2;
  b.eps_a = eps; b.eps_b = eps; b.Lpq_a = L; b.Lpq_b = L;
  EXPECT(pprpa_build_ab(&b, &ctx), PPRPA_EINVAL);
  b.nocc_a = 3; b.density_fitted = 2;
  EXPECT(pprpa_build_ab(&b, &ctx), PPRPA_EINVAL);
  b.density_fitted = 1; b.prec = 9;
  EXPECT(pprpa_build_ab(&b, &ctx), PPRPA_EINVAL);
  b.prec = -1;
  EXPECT(pprpa_build_ab(&b, &ctx), PPRPA_EINVAL);

  double buf[4];
  int64_t npp, nhh;
  pprpa_davidson_args d;
  memset(&d, 0, sizeof d);
  pprpa_corr_energy ce;
  pprpa_kernel_stats ks;
  EXPECT(pprpa_dims(NULL, &npp, &nhh), PPRPA_EINVAL);
  EXPECT(pprpa_matvec(NULL, 1, buf, buf, 0), PPRPA_EINVAL);
  EXPECT(pprpa_dense_matrix(NULL, buf, 0), PPRPA_EINVAL);
  EXPECT(pprpa_davidson(NULL, &d, buf, NULL, NULL, NULL), PPRPA_EINVAL);
  EXPECT(pprpa_correlation_energy(NULL, &ce), PPRPA_EINVAL);
  EXPECT(pprpa_correlation_energy_noalloc(NULL, &ce), PPRPA_EINVAL);
  EXPECT(pprpa_nto(NULL, 1, buf, 0, buf, buf, NULL, NULL), PPRPA_EINVAL);
  EXPECT(pprpa_nto_vectors(NULL, 1, buf, 0, 1, buf, buf, buf, buf), PPRPA_EINVAL);
  EXPECT(pprpa_sigma_stats(NULL, &ks, 0), PPRPA_EINVAL);
  pprpa_solve* sv = NULL;
  EXPECT(pprpa_solve_begin(NULL, &d, &sv), PPRPA_EINVAL);
  EXPECT(pprpa_solve_iterate(NULL, 1, NULL, NULL), PPRPA_EINVAL);
  EXPECT(pprpa_solve_stats(NULL, &ks, 0), PPRPA_EINVAL);
  pprpa_free(NULL);

  pprpa_server* srv = NULL;
  EXPECT(pprpa_server_create(1 << 30, 0, &srv), PPRPA_EINVAL);
  EXPECT(pprpa_server_create(1 << 30, 65, &srv), PPRPA_EINVAL);
  EXPECT(pprpa_server_create(1000, 4, &srv), PPRPA_EINVAL);
  EXPECT(pprpa_server_create(1 << 30, 4, NULL), PPRPA_EINVAL);
  uint64_t ticket;
  EXPECT(pprpa_server_submit(NULL, &a, &d, &ticket), PPRPA_EINVAL);
  pprpa_request_info info;
  EXPECT(pprpa_server_poll(NULL, 1, &info, NULL, NULL, NULL), PPRPA_EINVAL);
  EXPECT(pprpa_server_wait(NULL, 1, 0.0), PPRPA_EINVAL);
  pprpa_serving_stats st;
  EXPECT(pprpa_server_stats(NULL, &st), PPRPA_EINVAL);
  pprpa_server_destroy(NULL);
  free(eps);
  free(L);
}

static int log_lines = 0;
static void count_log(void* user, const char* line) {
  (void)user;
  if (line && line[0] == '{') ++log_lines;
}

static int ascending_finite(const double* w, int n) {
  for (int i = 0; i < n; ++i) {
    if (!isfinite(w[i])) return 0;
    if (i > 0 && w[i] < w[i - 1]) return 0;
  }
  return 1;
}

/* Restricted context: matvec, Davidson (pp, hh, warm start, log, caller-driven), direct solve,
 * correlation energy, NTOs. */
static void gpu_restricted(int mult, pprpa_prec prec) {
  const int nmo = 25, nocc = 5, naux = 60, nroot = 4;
  double* eps = energies(nmo, nocc, 0.0);
  double* L = integrals(naux, nmo, 0.06);
  pprpa_build_args a;
  memset(&a, 0, sizeof a);
  a.nmo = nmo; a.nocc = nocc; a.naux = naux; a.eps = eps; a.Lpq = L;
  a.mult = mult; a.prec = prec; a.dense = prec == PPRPA_FP64; a.max_block = 8;
  pprpa_ctx* ctx = NULL;
  EXPECT(pprpa_build(&a, &ctx), PPRPA_OK);
  if (!ctx) goto out;
  int64_t npp = 0, nhh = 0;
  EXPECT(pprpa_dims(ctx, &npp, &nhh), PPRPA_OK);
  const int64_t n = npp + nhh;
  CHECK(n > 0);

  double* z = malloc(sizeof(double) * 3 * n);
  double* s = malloc(sizeof(double) * 3 * n);
  for (int64_t i = 0; i < 3 * n; ++i) z[i] = uniform() - 0.5;
  EXPECT(pprpa_matvec(ctx, 3, z, s, 0), PPRPA_OK);
  EXPECT(pprpa_matvec(ctx, 0, z, s, 0), PPRPA_EINVAL);
  for (int64_t i = 0; i < 3 * n; ++i) CHECK(isfinite(s[i]));
  pprpa_kernel_stats ks;
  EXPECT(pprpa_sigma_stats(ctx, &ks, 1), PPRPA_OK);
  CHECK(ks.launches >= 1);

  double om[8], rs[8];
  double* vecs = malloc(sizeof(double) * nroot * n);
  pprpa_report rep;
  pprpa_davidson_args d;
  memset(&d, 0, sizeof d);
  d.nroot = nroot; d.block = 8; d.tol = prec == PPRPA_FP64 ? 1e-8 : 1e-5; d.log = count_log;
  log_lines = 0;
  EXPECT(pprpa_davidson(ctx, &d, om, vecs, rs, &rep), PPRPA_OK);
  CHECK(ascending_finite(om, nroot));
  CHECK(rep.n_conv == nroot);
  CHECK(log_lines == rep.iters);

  /* warm start from the converged vectors: converges at once */
  pprpa_davidson_args w = d;
  w.guess = vecs; w.nguess = nroot; w.log = NULL;
  double om2[8];
  EXPECT(pprpa_davidson(ctx, &w, om2, NULL, NULL, &rep), PPRPA_OK);
  for (int r = 0; r < nroot; ++r) CHECK(fabs(om2[r] - om[r]) < 1e-6);

  /* caller-driven iterations */
  pprpa_solve* sv = NULL;
  d.log = NULL;
  EXPECT(pprpa_solve_begin(ctx, &d, &sv), PPRPA_OK);
  if (sv) {
    int done = 0;
    pprpa_status it = PPRPA_OK;
    for (int k = 0; k < 200 && !done && it == PPRPA_OK; ++k) it = pprpa_solve_iterate(sv, 2, NULL, &done);
    CHECK(it == PPRPA_OK && done);
    EXPECT(pprpa_solve_stats(sv, &ks, 0), PPRPA_OK);
    EXPECT(pprpa_solve_end(sv, om2, NULL, rs, &rep), PPRPA_OK);
    for (int r = 0; r < nroot; ++r) CHECK(fabs(om2[r] - om[r]) < 1e-6);
  }

  /* hh channel */
  pprpa_davidson_args h = d;
  h.channel = 1; h.nroot = 3;
  EXPECT(pprpa_davidson(ctx, &h, om2, NULL, rs, &rep), PPRPA_OK);
  for (int r = 0; r < 3; ++r) CHECK(isfinite(om2[r]));
  h.channel = 2;
  EXPECT(pprpa_davidson(ctx, &h, om2, NULL, rs, &rep), PPRPA_EINVAL);

  /* NTO weights, densities and vectors of the pp roots */
  const int nv = nmo - nocc, no = nocc;
  double* lp = malloc(sizeof(double) * nroot * nv);
  double* lh = malloc(sizeof(double) * nroot * no);
  double* dvv = malloc(sizeof(double) * nroot * nv * nv);
  double* doo = malloc(sizeof(double) * nroot * no * no);
  EXPECT(pprpa_nto(ctx, nroot, vecs, 0, lp, lh, dvv, doo), PPRPA_OK);
  const int nvec = 3;
  double* c1 = malloc(sizeof(double) * nroot * nvec * nv);
  double* c2 = malloc(sizeof(double) * nroot * nvec * nv);
  double* c3 = malloc(sizeof(double) * nroot * nvec * no);
  double* c4 = malloc(sizeof(double) * nroot * nvec * no);
  EXPECT(pprpa_nto_vectors(ctx, nroot, vecs, 0, nvec, c1, c2, c3, c4), PPRPA_OK);
  EXPECT(pprpa_nto_vectors(ctx, nroot, vecs, 0, 65, c1, c2, c3, c4), PPRPA_EINVAL);

  if (a.dense) {
    double* M = malloc(sizeof(double) * n * n);
    EXPECT(pprpa_dense_matrix(ctx, M, 0), PPRPA_OK);
    for (int64_t i = 0; i < n; ++i)
      for (int64_t j = 0; j < i; ++j) CHECK(fabs(M[i * n + j] - M[j * n + i]) < 1e-12);
    free(M);
    pprpa_davidson_args dd = d;
    dd.direct = 1;
    EXPECT(pprpa_davidson(ctx, &dd, om2, vecs, rs, &rep), PPRPA_OK);
    for (int r = 0; r < nroot; ++r) CHECK(fabs(om2[r] - om[r]) < 1e-7);
    pprpa_corr_energy e1, e2;
    EXPECT(pprpa_correlation_energy(ctx, &e1), PPRPA_OK);
    EXPECT(pprpa_correlation_energy_noalloc(ctx, &e2), PPRPA_OK);
    CHECK(e1.ec_pp == e2.ec_pp && e1.ec_hh == e2.ec_hh);
    CHECK(fabs(e1.ec_pp - e1.ec_hh) < 1e-9);
  } else {
    pprpa_corr_energy e1;
    EXPECT(pprpa_correlation_energy(ctx, &e1), PPRPA_EUNSUPPORTED);
  }
  free(lp); free(lh); free(dvv); free(doo); free(c1); free(c2); free(c3); free(c4);
  free(vecs); free(z); free(s);
  pprpa_free(ctx);
out:
  free(eps);
  free(L);
}

/* Alpha-beta sector, dense and density fitted, with its NTOs. */
static void gpu_alpha_beta(int density_fitted, pprpa_prec prec) {
  const int nmo = 14, noa = 4, nob = 3, naux = 40, nroot = 3;
  double* ea = energies(nmo, noa, 0.0);
  double* eb = energies(nmo, nob, 0.03);
  double* La = integrals(naux, nmo, 0.06);
  double* Lb = integrals(naux, nmo, 0.06);
  pprpa_build_ab_args b;
  memset(&b, 0, sizeof b);
  b.nmo = nmo; b.nocc_a = noa; b.nocc_b = nob; b.naux = naux;
  b.eps_a = ea; b.eps_b = eb; b.Lpq_a = La; b.Lpq_b = Lb;
  b.density_fitted = density_fitted; b.prec = prec; b.max_block = 8;
  pprpa_ctx* ctx = NULL;
  EXPECT(pprpa_build_ab(&b, &ctx), PPRPA_OK);
  if (ctx) {
    int64_t npp = 0, nhh = 0;
    EXPECT(pprpa_dims(ctx, &npp, &nhh), PPRPA_OK);
    const int64_t n = npp + nhh;
    CHECK(npp == (int64_t)(nmo - noa) * (nmo - nob) && nhh == (int64_t)noa * nob);
    double om[8], rs[8];
    double* vecs = malloc(sizeof(double) * nroot * n);
    pprpa_report rep;
    pprpa_davidson_args d;
    memset(&d, 0, sizeof d);
    d.nroot = nroot; d.block = 6; d.tol = prec == PPRPA_FP64 ? 1e-8 : 1e-5;
    EXPECT(pprpa_davidson(ctx, &d, om, vecs, rs, &rep), PPRPA_OK);
    CHECK(ascending_finite(om, nroot));
    const int nva = nmo - noa, nvb = nmo - nob;
    double* lp = malloc(sizeof(double) * nroot * nva);
    double* lh = malloc(sizeof(double) * nroot * noa);
    double* dvv = malloc(sizeof(double) * nroot * (nva * nva + nvb * nvb));
    double* doo = malloc(sizeof(double) * nroot * (noa * noa + nob * nob));
    EXPECT(pprpa_nto(ctx, nroot, vecs, 0, lp, lh, dvv, doo), PPRPA_OK);
    double* c1 = malloc(sizeof(double) * nroot * 2 * nva);
    double* c2 = malloc(sizeof(double) * nroot * 2 * nvb);
    double* c3 = malloc(sizeof(double) * nroot * 2 * noa);
    double* c4 = malloc(sizeof(double) * nroot * 2 * nob);
    EXPECT(pprpa_nto_vectors(ctx, nroot, vecs, 0, 2, c1, c2, c3, c4), PPRPA_OK);
    free(lp); free(lh); free(dvv); free(doo); free(c1); free(c2); free(c3); free(c4);
    free(vecs);
    pprpa_free(ctx);
  }
  free(ea); free(eb); free(La); free(Lb);
}

/* Serving queue: three requests of different shapes and precisions, one too large for the
 * arena (finishes with ENOMEM). */
static void gpu_server(void) {
  pprpa_server* srv = NULL;
  EXPECT(pprpa_server_create((size_t)64 << 20, 3, &srv), PPRPA_OK);
  if (!srv) return;
  const int nreq = 4;
  int nmo[4] = {25, 30, 20, 160}, nocc[4] = {5, 6, 4, 40}, naux[4] = {60, 70, 50, 1200};
  double* eps[4];
  double* L[4];
  uint64_t ticket[4];
  pprpa_build_args a[4];
  pprpa_davidson_args d;
  memset(&d, 0, sizeof d);
  d.nroot = 3; d.tol = 1e-6;
  for (int r = 0; r < nreq; ++r) {
    eps[r] = energies(nmo[r], nocc[r], 0.0);
    L[r] = integrals(naux[r], nmo[r], 0.05);
    memset(&a[r], 0, sizeof a[r]);
    a[r].nmo = nmo[r]; a[r].nocc = nocc[r]; a[r].naux = naux[r];
    a[r].eps = eps[r]; a[r].Lpq = L[r];
    a[r].mult = r % 2; a[r].prec = r == 1 ? PPRPA_FP32 : PPRPA_FP64;
    EXPECT(pprpa_server_submit(srv, &a[r], &d, &ticket[r]), PPRPA_OK);
  }
  for (int r = 0; r < nreq; ++r) {
    EXPECT(pprpa_server_wait(srv, ticket[r], 120.0), PPRPA_OK);
    pprpa_request_info info;
    double om[3], rs[3];
    pprpa_report rep;
    EXPECT(pprpa_server_poll(srv, ticket[r], &info, om, rs, &rep), PPRPA_OK);
    CHECK(info.state == 2);
    if (info.status != (r < 3 ? PPRPA_OK : PPRPA_ENOMEM))
      fprintf(stderr, "request %d: status %d (%s)\n", r, info.status, info.message);
    if (r < 3) {
      CHECK(info.status == PPRPA_OK);
      CHECK(info.footprint < ((uint64_t)16 << 20)); /* staging sized by the request's own L */
      CHECK(ascending_finite(om, 3));
    } else {
      CHECK(info.status == PPRPA_ENOMEM);
    }
    EXPECT(pprpa_server_poll(srv, ticket[r], &info, NULL, NULL, NULL), PPRPA_EINVAL);
  }
  pprpa_serving_stats st;
  EXPECT(pprpa_server_stats(srv, &st), PPRPA_OK);
  pprpa_server_destroy(srv);
  for (int r = 0; r < nreq; ++r) {
    free(eps[r]);
    free(L[r]);
  }
}

int main(int argc, char** argv) {
  cpu_checks();
  printf("cpu checks done (%d failures)\n", fails);
  fflush(stdout);
  if (argc > 1 && strcmp(argv[1], "gpu") == 0) {
    const pprpa_prec precs[4] = {PPRPA_FP64, PPRPA_FP32, PPRPA_BF16X6, PPRPA_BF16X3};
    for (int p = 0; p < 4; ++p)
      for (int mult = 0; mult < 2; ++mult) {
        gpu_restricted(mult, precs[p]);
        printf("restricted mult %d prec %d done (%d failures)\n", mult, (int)precs[p], fails);
        fflush(stdout);
      }
    gpu_alpha_beta(0, PPRPA_FP64);
    for (int p = 0; p < 4; ++p) gpu_alpha_beta(1, precs[p]);
    printf("alpha-beta done (%d failures)\n", fails);
    fflush(stdout);
    gpu_server();
    printf("server done (%d failures)\n", fails);
  }
  printf("%s\n", fails ? "FAILED" : "ALL OK");
  return fails ? 1 : 0;
}
