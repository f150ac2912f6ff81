/* Host-side checks of the C ABI under AddressSanitizer, UndefinedBehavior-
 * Sanitizer or ThreadSanitizer, on a machine without a GPU: argument
 * validation and error paths of every entry point, the checkpoint parser on
 * damaged images, the host gate builder from several threads at once, the
 * footprint planner, and the serving scheduler's admission threads (each
 * request fails at its first device allocation, so every thread runs its
 * error path concurrently).
 * Prints one line per group and "host checks: ok" at the end; any check
 * that fails prints its line and the program exits with status 1. */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "ptebd.h"
#include "ptebd_diag.h"

static int failures = 0;

#define CHECK(cond, what)                                                   \
  do {                                                                      \
    if (!(cond)) {                                                          \
      fprintf(stderr, "FAILED: %s (%s:%d) last error: %s\n", what, __FILE__, \
              __LINE__, tebd_last_error());                                 \
      ++failures;                                                           \
    }                                                                       \
  } while (0)

static tebd_model model(int L, int d) {
  tebd_model m;
  m.L = L;
  m.d = d;
  m.U = 2.0;
  m.J = 1.0;
  m.Jnnn = 0.1;
  m.K = 0.02;
  m.jc = 0.5 * (L - 1);
  return m;
}

static void validation(void) {
  tebd_opts o;
  tebd_opts_default(&o);
  tebd_mps* h = NULL;
  tebd_model m = model(8, 3);
  tebd_model bad = model(2, 3);
  CHECK(mps_init_cdw(&bad, &o, 1, &h) == TEBD_EINVAL && h == NULL, "L < 3 refused");
  bad = model(8, 1);
  CHECK(mps_init_cdw(&bad, &o, 1, &h) == TEBD_EINVAL, "d < 2 refused");
  bad = model(8, 3);
  bad.U = NAN;
  CHECK(mps_init_cdw(&bad, &o, 1, &h) == TEBD_EINVAL, "non-finite coupling refused");
  o.chi_max = 0;
  CHECK(mps_init_cdw(&m, &o, 1, &h) == TEBD_EINVAL, "chi_max < 1 refused");
  tebd_opts_default(&o);
  o.svd = TEBD_SVD_GRAM_EIG;
  o.trunc_rel = 1e-12;
  CHECK(mps_init_cdw(&m, &o, 1, &h) == TEBD_EINVAL, "Gram route eps below its floor refused");
  size_t bytes = 0;
  CHECK(mps_footprint(&m, &o, &bytes) == TEBD_EINVAL, "footprint refuses the same eps");
  o.trunc_rel = TEBD_GRAM_EPS_MIN;
  CHECK(mps_footprint(&m, &o, &bytes) == TEBD_OK && bytes > 0, "footprint of a valid request");
  tebd_opts_default(&o);
  o.workers = -1;
  CHECK(mps_init_cdw(&m, &o, 1, &h) == TEBD_EINVAL, "negative workers refused");
  tebd_opts_default(&o);
  int32_t occ[8] = {0, 1, 2, 3, 0, 1, 2, 0};
  CHECK(mps_init_product(&m, &o, occ, &h) == TEBD_EINVAL, "occupation >= d refused");
  CHECK(mps_init_product(&m, &o, NULL, &h) == TEBD_EINVAL, "NULL occupations refused");
  /* calls on a NULL handle */
  CHECK(tebd_step(NULL, 0.01) != TEBD_OK, "step on NULL handle");
  CHECK(tebd_layer(NULL, 0, 0.01) != TEBD_OK, "layer on NULL handle");
  CHECK(measure_local(NULL, NULL, NULL, NULL) != TEBD_OK, "measure on NULL handle");
  double w = 0.0;
  CHECK(mps_discarded_weight(NULL, &w) != TEBD_OK, "ledger of NULL handle");
  CHECK(tebd_step_many(NULL, 2, NULL) == TEBD_EINVAL, "step_many without handles");
  CHECK(tebd_step_many(NULL, 0, NULL) == TEBD_OK, "step_many of nothing");
  CHECK(tebd_serve(NULL, -1, NULL, NULL, NULL, NULL, NULL) == TEBD_EINVAL, "serve with n < 0");
  CHECK(tebd_diag_svd(1, 4, 4, NULL, 4, 0.0, 1e-6, NULL, NULL, NULL, NULL, NULL, NULL) == TEBD_EINVAL,
        "diag svd without buffers");
  CHECK(strlen(tebd_last_error()) > 0, "an error message is set");
  printf("validation: %s\n", failures ? "FAILED" : "ok");
}

/* The checkpoint parser on hostile input: random bytes, images with a
 * plausible header (right tag, version and sizes, random payload size and
 * checksum), cut at every length up to 4 KiB and read from an odd address;
 * each is refused with TEBD_EINVAL before any device call. */
static uint32_t lcg(uint32_t* s) {
  *s = *s * 1664525u + 1013904223u;
  return *s >> 8;
}

static void checkpoint_images(void) {
  tebd_model m = model(6, 3);
  tebd_opts o;
  tebd_opts_default(&o);
  o.chi_max = 8;
  enum { N = 4096 };
  unsigned char* raw = (unsigned char*)malloc(N + 1);
  uint32_t seed = 12345u;
  int bad = 0;
  for (int rep = 0; rep < 3000; ++rep) {
    const size_t len = lcg(&seed) % N;
    unsigned char* img = raw + 1;   /* misaligned on purpose */
    for (size_t i = 0; i < len; ++i) img[i] = (unsigned char)lcg(&seed);
    if (rep % 2 == 0 && len >= 64) {
      const uint32_t version = 1;
      const int32_t sizes[7] = {6, 3, 6, 3, 0, 0, 0};
      const uint64_t payload = (rep % 4 == 0) ? (uint64_t)(len - 64) : (uint64_t)lcg(&seed);
      memcpy(img, "ptebdck", 8);
      memcpy(img + 8, &version, 4);
      memcpy(img + 12, sizes, sizeof sizes);
      memcpy(img + 48, &payload, 8);
    }
    tebd_mps* h = NULL;
    const tebd_status st = mps_restore(&m, &o, img, len, &h);
    bad |= st != TEBD_EINVAL || h != NULL;
  }
  size_t bytes = 0;
  tebd_mps* h = NULL;
  CHECK(!bad, "damaged checkpoint images refused");
  CHECK(mps_checkpoint(NULL, NULL, 0, &bytes) == TEBD_EINVAL, "checkpoint of a NULL handle");
  CHECK(mps_restore(&m, &o, NULL, 64, &h) == TEBD_EINVAL && h == NULL, "restore from NULL");
  printf("checkpoint images: %s\n", bad ? "FAILED" : "ok");
  free(raw);
}

/* The host gate builder (sector-wise Jacobi eigensolver) from several threads. */
typedef struct {
  int j;
  double err;
} gate_job;

static void* gate_thread(void* arg) {
  gate_job* g = (gate_job*)arg;
  tebd_model m = model(9, 3);
  const int n = 27;
  double* G = (double*)malloc(sizeof(double) * 2 * n * n);
  double* H = (double*)malloc(sizeof(double) * 2 * n * n);
  g->err = -1.0;
  for (int rep = 0; rep < 20; ++rep) {
    if (tebd_diag_gate(&m, 0, g->j, 0.05, G) != TEBD_OK) break;
    /* unitarity: G G^+ = 1 (planar: real parts then imaginary parts) */
    double e = 0.0;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double re = 0.0, im = 0.0;
        for (int c = 0; c < n; ++c) {
          const double xr = G[a * n + c], xi = G[n * n + a * n + c];
          const double yr = G[b * n + c], yi = -G[n * n + b * n + c];
          re += xr * yr - xi * yi;
          im += xr * yi + xi * yr;
        }
        H[a * n + b] = re;
        e = fmax(e, fabs(re - (a == b ? 1.0 : 0.0)) + fabs(im));
      }
    g->err = e;
  }
  free(G);
  free(H);
  return NULL;
}

static void gates(void) {
  enum { NT = 6 };
  pthread_t th[NT];
  gate_job job[NT];
  for (int t = 0; t < NT; ++t) {
    job[t].j = t % 7;
    pthread_create(&th[t], NULL, gate_thread, &job[t]);
  }
  for (int t = 0; t < NT; ++t) pthread_join(th[t], NULL);
  int bad = 0;
  for (int t = 0; t < NT; ++t) bad |= !(job[t].err >= 0.0 && job[t].err < 1e-12);
  CHECK(!bad, "gates built concurrently are unitary");
  printf("gates from %d threads: %s\n", NT, bad ? "FAILED" : "ok");
}

/* Serving: every request fails at its first device allocation on a machine
 * without a GPU; the admission loop and the per-request threads still run. */
static void serving(void) {
  enum { N = 12 };
  tebd_request req[N];
  tebd_serve_result res[N];
  memset(res, 0, sizeof(res));
  for (int i = 0; i < N; ++i) {
    req[i].model = model(6 + (i % 4), 3);
    req[i].chi_max = 8 << (i % 3);
    req[i].dt = 0.01;
    req[i].steps = 2;
    req[i].arrival = 0.002 * i;
    req[i].first_occupied = i & 1;
  }
  tebd_serve_opts so;
  memset(&so, 0, sizeof(so));
  so.max_active = 3;
  so.hbm_budget = 1e9;
  so.prec = TEBD_FP64;
  so.svd = TEBD_SVD_JACOBI;
  so.trunc_weight = 1e-12;
  so.trunc_rel = 1e-12;
  so.workers_per_request = 1;
  double* n_out = (double*)calloc(N * 16, sizeof(double));
  const tebd_status st = tebd_serve(req, N, &so, res, n_out, NULL, NULL);
  int finished = 1;
  for (int i = 0; i < N; ++i) finished &= res[i].finished >= res[i].admitted && res[i].admitted >= res[i].arrival;
  CHECK(finished, "every request admitted after arrival and finished after admission");
  printf("serving %d requests (status %d without a device): %s\n", N, (int)st, finished ? "ok" : "FAILED");
  /* continuous batching: one scheduler thread, the same admission rule */
  memset(res, 0, sizeof(res));
  so.batched = 1;
  so.workers_per_request = 0;
  const tebd_status st2 = tebd_serve(req, N, &so, res, n_out, NULL, NULL);
  finished = 1;
  for (int i = 0; i < N; ++i) finished &= res[i].finished >= res[i].admitted && res[i].admitted >= res[i].arrival;
  CHECK(finished && st2 != TEBD_OK, "batched serving admits and retires every request");
  so.svd = TEBD_SVD_GRAM_EIG;
  so.trunc_rel = TEBD_GRAM_EPS_MIN;
  CHECK(tebd_serve(req, N, &so, res, n_out, NULL, NULL) == TEBD_EINVAL, "batched serving needs the Jacobi route");
  printf("batched serving (status %d without a device): %s\n", (int)st2, finished ? "ok" : "FAILED");
  free(n_out);
}

int main(void) {
  validation();
  checkpoint_images();
  gates();
  serving();
  if (failures) {
    printf("host checks: %d failures\n", failures);
    return 1;
  }
  printf("host checks: ok\n");
  return 0;
}
