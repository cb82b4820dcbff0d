/* Host-side checks of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Runs only entry points that return before touching a GPU: the default
 * schedule for every edge length up to 4096, the autotuner cache reader on
 * well-formed, malformed and hostile files, descriptor validation of plans,
 * batches and particle objects, and the resource hooks.  Built and run by
 * tests/test_host_sanitizers.py against a host-instrumented build of the library.
 * Exit status 0 = every check held (the sanitizers abort on their own findings). */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "psatd.h"

static int failures = 0;
#define CHECK(cond)                                                   \
  do {                                                                \
    if (!(cond)) {                                                    \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      ++failures;                                                     \
    }                                                                 \
  } while (0)

static void write_file(const char* path, const char* text) {
  FILE* f = fopen(path, "w");
  if (!f) {
    perror(path);
    exit(2);
  }
  fputs(text, f);
  fclose(f);
}

static psatd_plan_desc good_desc(void) {
  psatd_plan_desc d;
  memset(&d, 0, sizeof d);
  d.nx = d.ny = d.nz = 8;
  d.ngx = d.ngy = d.ngz = 1;
  d.order = 4;
  d.dx = d.dy = d.dz = 1.0;
  d.dt = 0.5;
  d.c = d.eps0 = 1.0;
  return d;
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : ".";
  char path[4096];

  /* default schedules: product of the radices equals the transform length */
  for (int n = 1; n <= 4096; ++n) {
    int r[32], m = 0;
    const int k = psatd_default_schedule(n, r, 32, &m);
    CHECK(k >= 0);
    long long prod = 1;
    for (int i = 0; i < k; ++i) prod *= r[i];
    CHECK(prod == m || (n == 1 && k == 0));
    CHECK(m == n || m >= 2 * n - 1);
  }
  {
    int r[2], m = 0;
    CHECK(psatd_default_schedule(0, r, 2, &m) < 0);
    CHECK(psatd_default_schedule(-5, r, 2, &m) < 0);
    CHECK(psatd_default_schedule(4096, r, 0, &m) < 0 || 1); /* too few slots: an error or a count, never a write */
    CHECK(psatd_default_schedule(64, NULL, 4, &m) < 0);
  }

  /* autotuner cache reader on hostile text */
  static const char* files[] = {
      "",
      "{",
      "{\"schema\": 3, \"entries\": [",
      "{\"schema\": 3, \"entries\": [{\"key\": \"f,0,320,320,1,1\", \"radices\": [20, 16], \"tile\": 256}]}",
      "{\"schema\": 3, \"entries\": [{\"key\": \"f,0,320,320,1,1\", \"radices\": [20, 16, 99999999999], \"tile\": 1}]}",
      "{\"schema\": 3, \"entries\": [{\"key\": \"\", \"radices\": [], \"tile\": -7}]}",
      "{\"schema\": 99, \"entries\": []}",
      "[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[[",
      "{\"schema\": 3, \"entries\": [{\"key\": \"f,0,320,320,1,1\", \"radices\": [2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2,2], \"tile\": 8}]}",
      "{\"schema\": 3, \"entries\": [{\"key\": \"\\\"\\\\\\u0000\", \"radices\": [-2, 0], \"tile\": 2147483647}]}",
  };
  for (size_t i = 0; i < sizeof files / sizeof files[0]; ++i) {
    snprintf(path, sizeof path, "%s/cache_%zu.json", dir, i);
    write_file(path, files[i]);
    int acc = -1, rej = -1;
    const int rc = psatd_tune_cache_load(path, &acc, &rej);
    CHECK(rc == PSATD_OK || rc == PSATD_EINVAL);
    CHECK(acc >= 0 && rej >= 0);
  }
  {
    /* a long line of one token */
    const size_t big = 1 << 20;
    char* text = (char*)malloc(big + 1);
    memset(text, '9', big);
    text[big] = 0;
    snprintf(path, sizeof path, "%s/cache_big.json", dir);
    write_file(path, text);
    free(text);
    int acc = -1, rej = -1;
    (void)psatd_tune_cache_load(path, &acc, &rej);
    snprintf(path, sizeof path, "%s/does_not_exist.json", dir);
    CHECK(psatd_tune_cache_load(path, &acc, &rej) == PSATD_OK && acc == 0 && rej == 0);
    CHECK(psatd_tune_cache_load(path, NULL, NULL) == PSATD_OK);
  }

  /* descriptor validation (all rejected on the host) */
  {
    psatd_plan* p = NULL;
    psatd_plan_desc d = good_desc();
    d.nx = 0;
    CHECK(psatd_plan_create_ex(&d, &p) == PSATD_EINVAL && p == NULL);
    d = good_desc();
    d.order = 3;
    CHECK(psatd_plan_create_ex(&d, &p) == PSATD_EINVAL);
    d = good_desc();
    d.flags = 1 << 20;
    CHECK(psatd_plan_create_ex(&d, &p) == PSATD_EINVAL);
    CHECK(psatd_plan_create_ex(NULL, &p) == PSATD_EINVAL);
    CHECK(psatd_plan_create(0, 8, 8, 0, 0, 1.0, 0.5) == NULL);
    CHECK(strlen(psatd_last_error()) > 0);
    psatd_plan_destroy(NULL);
  }
  {
    /* two boxes whose interiors overlap: refused before any allocation */
    psatd_plan_desc subs[2] = {good_desc(), good_desc()};
    int origins[6] = {0, 0, 0, 4, 4, 4};
    int gdims[3] = {16, 16, 16};
    psatd_batch* b = NULL;
    CHECK(psatd_batch_create(2, subs, origins, gdims, &b) == PSATD_EINVAL && b == NULL);
    CHECK(psatd_batch_create(0, subs, origins, gdims, &b) == PSATD_EINVAL);
    psatd_batch_destroy(NULL);
  }
  {
    psatd_pic_desc d;
    memset(&d, 0, sizeof d);
    d.gx = d.gy = d.gz = 16;
    d.dx = d.dy = d.dz = 1.0;
    d.dt = 2.0; /* c dt above the cell size */
    d.c = 1.0;
    d.max_particles = 10;
    d.tile = 8;
    psatd_pic* o = NULL;
    CHECK(psatd_pic_create(&d, &o) == PSATD_EUNSUPPORTED && o == NULL);
    d.dt = 0.5;
    d.shape = 4; /* no B-spline of degree 4 */
    CHECK(psatd_pic_create(&d, &o) == PSATD_EINVAL && o == NULL);
    d.shape = 2;
    d.tile = 0;
    CHECK(psatd_pic_create(&d, &o) == PSATD_EINVAL);
    psatd_pic_destroy(NULL);
  }
  {
    int w[3] = {1, 1, 1};
    CHECK(psatd_pml_set(NULL, w, 1.0, 2.0) == PSATD_EINVAL);
    CHECK(psatd_pml_step(NULL, NULL, NULL, NULL) == PSATD_EINVAL);
    CHECK(psatd_pic_push(NULL, NULL, NULL, NULL, NULL, 0, NULL) == PSATD_EINVAL);
    CHECK(psatd_pic_deposit(NULL, NULL, NULL, NULL, NULL, 0, NULL) == PSATD_EINVAL);
  }
  {
    const long long before = psatd_device_bytes_in_use();
    CHECK(psatd_set_device_budget(1 << 20) == PSATD_OK);
    CHECK(psatd_set_device_budget(-1) == PSATD_OK);
    CHECK(psatd_device_bytes_in_use() == before);
  }
  if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
  else printf("host ABI checks passed\n");
  return failures ? 1 : 0;
}
