/* Host-code checks of librsk under AddressSanitizer and UndefinedBehaviorSanitizer.
 *
 * Linked against the library sources built with both sanitizers on their host code, this program
 * drives every host path that needs no kernel: argument validation of each entry point (Algorithm
 * 1's Require line: eta >= 1, lambda >= 0, alpha > 0, the sizes and pointers the kernels take), the
 * planners, the workspace queries and the tuning table with its text cache file. No call here
 * launches a kernel: each solve call carries one invalid argument and must return its status code
 * before any device work, and every device pointer is a made-up address that the host code must
 * never dereference. Calls whose outcome depends on whether a GPU is present (planners, workspace
 * queries) are checked for a code in the documented set only. Exit status: 0 when every
 * expectation holds (the sanitizers abort on their own findings).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include "rsk.h"

static int n_calls, n_fail;

static void expect(const char* what, int got, int want) {
  ++n_calls;
  if (got != want) {
    ++n_fail;
    fprintf(stderr, "FAIL %s: got %d (%s), want %d\n", what, got, rsk_status_string(got), want);
  }
}

/* got must be one of the codes in the bit mask */
static void expect_in(const char* what, int got, unsigned mask) {
  ++n_calls;
  if (got < 0 || got > 31 || !((mask >> got) & 1u)) {
    ++n_fail;
    fprintf(stderr, "FAIL %s: got %d (%s), not in mask 0x%x\n", what, got, rsk_status_string(got), mask);
  }
}

#define BIT(c) (1u << (c))
#define DEV(a) ((void*)(uintptr_t)(a))

static rsk_dense dense(int64_t m, int64_t n, int64_t ld, int32_t dt) {
  rsk_dense d;
  d.m = m; d.n = n; d.ld = ld; d.dtype = dt; d.val = DEV(0x100000);
  return d;
}

static rsk_params params(int32_t eta, int64_t K) {
  rsk_params p;
  memset(&p, 0, sizeof p);
  p.lambda = 1.0; p.eta = eta; p.alpha = 1.0; p.K = K;
  p.index_stream = (const int32_t*)DEV(0x200000);
  p.rownorm2 = DEV(0x300000);
  p.status_dev = (int32_t*)DEV(0x400000);
  return p;
}

static void check_status_strings(void) {
  expect("abi version", rsk_abi_version(), RSK_ABI_VERSION);
  for (int s = -3; s < 12; ++s) {
    const char* t = rsk_status_string(s);
    ++n_calls;
    if (!t || !t[0]) { ++n_fail; fprintf(stderr, "FAIL status string %d\n", s); }
  }
}

static rsk_tune_entry tune(int32_t path, int32_t dt, int64_t m, int64_t n, int32_t eta, int32_t R, int64_t v0,
                           int64_t v1) {
  rsk_tune_entry e;
  memset(&e, 0, sizeof e);
  e.path = path; e.dtype = dt; e.m = m; e.n = n; e.eta = eta; e.R = R; e.v0 = v0; e.v1 = v1; e.us = 1.5;
  return e;
}

static void check_tune_table(const char* dir) {
  char f1[512], f2[512], f3[512];
  snprintf(f1, sizeof f1, "%s/tune_saved.txt", dir);
  snprintf(f2, sizeof f2, "%s/tune_hostile.txt", dir);
  snprintf(f3, sizeof f3, "%s/no_such_dir/tune.txt", dir);
  expect("tune clear all", rsk_tune_clear(-1), RSK_OK);
  rsk_tune_entry d = tune(RSK_TUNE_DENSE, RSK_F32, 100000, 20000, 1024, 0, 2, 256);
  rsk_tune_entry out;
  int32_t found = -1;
  expect("tune set dense", rsk_tune_set(&d), RSK_OK);
  expect("tune set null", rsk_tune_set(NULL), RSK_ERR_INVALID_ARG);
  rsk_tune_entry bad = tune(7, 0, 1, 1, 1, 0, 1, 1);
  expect("tune set bad path", rsk_tune_set(&bad), RSK_ERR_INVALID_ARG);
  bad = tune(RSK_TUNE_BATCHED, 0, 0, 0, 0, 0, 4096, 0);
  expect("tune set batched zero bound", rsk_tune_set(&bad), RSK_ERR_INVALID_ARG);
  expect("tune get", rsk_tune_get(&d, &out, &found), RSK_OK);
  expect("tune get found", found, 1);
  expect("tune get null key", rsk_tune_get(NULL, &out, &found), RSK_ERR_INVALID_ARG);
  expect("tune get null out", rsk_tune_get(&d, NULL, &found), RSK_ERR_INVALID_ARG);
  expect("tune get null found", rsk_tune_get(&d, &out, NULL), RSK_ERR_INVALID_ARG);
  /* more batched classes than the planner's table holds: it keeps the lowest bounds */
  for (int i = 0; i < 40; ++i) {
    rsk_tune_entry b = tune(RSK_TUNE_BATCHED, RSK_F32, (int64_t)(i + 1) << 14, 0, 0, i % 3 == 0 ? 2 : 0,
                            (int64_t)(16 + i) << 10, 0);
    expect("tune set batched class", rsk_tune_set(&b), RSK_OK);
  }
  for (int i = 0; i < 300; ++i) {
    rsk_tune_entry e = tune(i % 2 ? RSK_TUNE_MULTIRHS : RSK_TUNE_DENSE, i % 2, 1000 + i, 500, 10 + i, 4 * (i % 5),
                            i, i + 1);
    expect("tune set many", rsk_tune_set(&e), RSK_OK);
  }
  expect("tune save", rsk_tune_save(f1), RSK_OK);
  expect("tune save null", rsk_tune_save(NULL), RSK_ERR_INVALID_ARG);
  expect("tune save into a missing directory", rsk_tune_save(f3), RSK_ERR_INVALID_ARG);
  expect("tune clear dense", rsk_tune_clear(RSK_TUNE_DENSE), RSK_OK);
  expect("tune get after clear", rsk_tune_get(&d, &out, &found), RSK_OK);
  expect("tune get after clear found", found, 0);
  expect("tune load saved", rsk_tune_load(f1), RSK_OK);
  found = -1;
  expect("tune get reloaded", rsk_tune_get(&d, &out, &found), RSK_OK);
  expect("tune get reloaded found", found, 1);
  expect("tune erase", rsk_tune_erase(&d), RSK_OK);
  expect("tune erase again", rsk_tune_erase(&d), RSK_OK);
  expect("tune erase null", rsk_tune_erase(NULL), RSK_ERR_INVALID_ARG);

  /* a hostile cache file: lines longer than the reader's buffer, truncated and out-of-range
     fields, numbers that overflow, no final newline */
  FILE* h = fopen(f2, "w");
  if (!h) { ++n_fail; fprintf(stderr, "FAIL cannot write %s\n", f2); return; }
  fprintf(h, "# header\n\n");
  for (int i = 0; i < 3000; ++i) fputc('7', h);
  fputc('\n', h);
  fprintf(h, "0 0 1 2 3\n");
  fprintf(h, "9 0 1 2 3 4 5 6 7 8.0\n");
  fprintf(h, "-1 0 1 2 3 4 5 6 7 8.0\n");
  fprintf(h, "0 0 99999999999999999999999 1 1 0 1 1 1 nan\n");
  fprintf(h, "2 0 -5 0 0 0 -7 0 0 inf\n");
  fprintf(h, "1 1 2147483648 3 2147483647 -2147483648 1 1 1 1e308\n");
  fprintf(h, "0 1 1000 500 10 0 1 4 0 12.5");
  fclose(h);
  expect("tune load hostile", rsk_tune_load(f2), RSK_OK);
  rsk_tune_entry k = tune(RSK_TUNE_DENSE, RSK_F64, 1000, 500, 10, 0, 0, 0);
  found = -1;
  expect("tune get last line", rsk_tune_get(&k, &out, &found), RSK_OK);
  expect("tune get last line found", found, 1);
  expect("tune load missing", rsk_tune_load(f3), RSK_ERR_INVALID_ARG);
  expect("tune load null", rsk_tune_load(NULL), RSK_ERR_INVALID_ARG);
  /* the planners read the batched classes (including the hostile file's negative ones) */
  rsk_batch_item it;
  memset(&it, 0, sizeof it);
  it.A = DEV(0x10000000); it.m = 4000; it.n = 2000; it.ld = 2000; it.b = DEV(0x2000); it.rownorm2 = DEV(0x3000);
  it.index_stream = (const int32_t*)DEV(0x4000); it.K = 10; it.eta = 201; it.alpha = 1.0; it.lambda = 0.5;
  it.x_star = DEV(0x5000); it.x = DEV(0x6000); it.status_dev = (int32_t*)DEV(0x7000);
  int32_t kout = -1, g = -1;
  expect_in("plan batched with tuned classes", rsk_plan_batched(1, RSK_F32, &it, 0, 0, &kout, &g),
            BIT(RSK_OK) | BIT(RSK_ERR_UNSUPPORTED) | BIT(RSK_ERR_HIP));
  expect("tune clear batched", rsk_tune_clear(RSK_TUNE_BATCHED), RSK_OK);
  expect("tune clear all again", rsk_tune_clear(-1), RSK_OK);
  remove(f1);
  remove(f2);
}

static void check_dense(void) {
  rsk_dense d = dense(10, 5, 5, RSK_F32);
  rsk_params p = params(2, 3);
  size_t nb = 0;
  void* b = DEV(0x500000);
  void* xs = DEV(0x600000);
  void* x = DEV(0x700000);
  void* ws = DEV(0x800000);
#define SOLVE() rsk_avg_solve_dense(&d, b, &p, xs, x, ws, (size_t)1 << 20, NULL)
  /* each bad field alone */
  p.eta = 0; expect("dense eta 0", SOLVE(), RSK_ERR_INVALID_ARG); p.eta = 2;
  p.K = -1; expect("dense K < 0", SOLVE(), RSK_ERR_INVALID_ARG); p.K = 3;
  p.lambda = -1.0; expect("dense lambda < 0", SOLVE(), RSK_ERR_INVALID_ARG); p.lambda = 1.0;
  p.lambda = NAN; expect("dense lambda nan", SOLVE(), RSK_ERR_INVALID_ARG); p.lambda = 1.0;
  p.alpha = 0.0; expect("dense alpha 0", SOLVE(), RSK_ERR_INVALID_ARG); p.alpha = 1.0;
  p.alpha = NAN; expect("dense alpha nan", SOLVE(), RSK_ERR_INVALID_ARG); p.alpha = 1.0;
  p.alpha = INFINITY; expect("dense alpha inf", SOLVE(), RSK_ERR_INVALID_ARG); p.alpha = 1.0;
  p.index_stream = NULL; expect("dense no stream", SOLVE(), RSK_ERR_INVALID_ARG);
  p.index_stream = (const int32_t*)DEV(0x200000);
  p.rownorm2 = NULL; expect("dense no norms", SOLVE(), RSK_ERR_INVALID_ARG); p.rownorm2 = DEV(0x300000);
  p.status_dev = NULL; expect("dense no status", SOLVE(), RSK_ERR_INVALID_ARG);
  p.status_dev = (int32_t*)DEV(0x400000);
  p.stream_offset = -3; expect("dense negative offset", SOLVE(), RSK_ERR_INVALID_ARG); p.stream_offset = 0;
  d.m = 0; expect("dense m 0", SOLVE(), RSK_ERR_INVALID_ARG); d.m = 10;
  d.n = -1; expect("dense n < 0", SOLVE(), RSK_ERR_INVALID_ARG); d.n = 5;
  d.ld = 4; expect("dense ld < n", SOLVE(), RSK_ERR_INVALID_ARG); d.ld = 5;
  d.val = NULL; expect("dense no values", SOLVE(), RSK_ERR_INVALID_ARG); d.val = DEV(0x100000);
  d.dtype = 3; expect("dense dtype", SOLVE(), RSK_ERR_UNSUPPORTED);
  expect("dense ws dtype", rsk_workspace_size_dense(&d, &p, &nb), RSK_ERR_UNSUPPORTED);
  d.dtype = RSK_F32;
  expect("dense null A", rsk_avg_solve_dense(NULL, b, &p, xs, x, ws, 1 << 20, NULL), RSK_ERR_INVALID_ARG);
  expect("dense null b", rsk_avg_solve_dense(&d, NULL, &p, xs, x, ws, 1 << 20, NULL), RSK_ERR_INVALID_ARG);
  expect("dense null p", rsk_avg_solve_dense(&d, b, NULL, xs, x, ws, 1 << 20, NULL), RSK_ERR_INVALID_ARG);
  expect("dense null x", rsk_avg_solve_dense(&d, b, &p, xs, NULL, ws, 1 << 20, NULL), RSK_ERR_INVALID_ARG);
  expect("dense ws null out", rsk_workspace_size_dense(&d, &p, NULL), RSK_ERR_INVALID_ARG);
  expect("dense ws null A", rsk_workspace_size_dense(NULL, &p, &nb), RSK_ERR_INVALID_ARG);
  expect("noalloc eta 0", (p.eta = 0, rsk_avg_solve_dense_noalloc(&d, b, &p, xs, x, NULL)), RSK_ERR_INVALID_ARG);
  p.eta = 2;
  expect("noalloc null A", rsk_avg_solve_dense_noalloc(NULL, b, &p, xs, x, NULL), RSK_ERR_INVALID_ARG);
  int32_t plan[16];
  expect("plan dense null out", rsk_plan_dense(&d, &p, NULL), RSK_ERR_INVALID_ARG);
  /* planners and workspace sizes over a sweep of shapes and kernels (GPU-dependent outcome) */
  static const int64_t ms[] = {1, 7, 1000, 100000};
  static const int64_t ns[] = {1, 5, 20000, 1 << 20};
  static const int32_t etas[] = {1, 16, 88, 1024, 16384, 16385};
  for (int a = 0; a < 4; ++a)
    for (int c = 0; c < 4; ++c)
      for (int e = 0; e < 6; ++e)
        for (int kern = 0; kern < 6; ++kern)
          for (int dt = 0; dt < 2; ++dt) {
            rsk_dense dd = dense(ms[a], ns[c], ns[c] + (c & 1), dt);
            rsk_params pp = params(etas[e], 100);
            pp.kernel = kern;
            pp.grid = (a + e) % 3 == 0 ? 0 : 64 * (a + 1);
            const unsigned ok = BIT(RSK_OK) | BIT(RSK_ERR_INVALID_ARG) | BIT(RSK_ERR_UNSUPPORTED) | BIT(RSK_ERR_HIP);
            expect_in("plan dense sweep", rsk_plan_dense(&dd, &pp, plan), ok);
            expect_in("workspace dense sweep", rsk_workspace_size_dense(&dd, &pp, &nb), ok);
          }
#undef SOLVE
}

static void check_csr(void) {
  rsk_csr c;
  c.m = 100; c.n = 50; c.nnz = 300; c.dtype = RSK_F32;
  c.row_ptr = (const int64_t*)DEV(0x1000); c.col = (const int32_t*)DEV(0x2000); c.val = DEV(0x3000);
  rsk_params p = params(8, 10);
  size_t nb = 0;
  expect_in("csr ws", rsk_workspace_size_csr(&c, &p, &nb), BIT(RSK_OK) | BIT(RSK_ERR_UNSUPPORTED));
  p.y_out = DEV(0x9000);
  expect_in("csr ws with y", rsk_workspace_size_csr(&c, &p, &nb), BIT(RSK_OK) | BIT(RSK_ERR_UNSUPPORTED));
  p.eta = 4097; expect("csr eta > 4096", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_UNSUPPORTED); p.eta = 8;
  p.kernel = 3; expect("csr dense kernel", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_INVALID_ARG); p.kernel = 0;
  p.kernel = 4; expect("csr dense kernel 4", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_INVALID_ARG); p.kernel = 0;
  c.row_ptr = NULL; expect("csr no row_ptr", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_INVALID_ARG);
  c.row_ptr = (const int64_t*)DEV(0x1000);
  c.m = 0; expect("csr m 0", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_INVALID_ARG); c.m = 100;
  c.nnz = -1; expect("csr nnz < 0", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_INVALID_ARG); c.nnz = 300;
  c.n = (int64_t)INT32_MAX + 1; expect("csr n too big", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_UNSUPPORTED);
  c.n = 50;
  c.dtype = 9; expect("csr dtype", rsk_workspace_size_csr(&c, &p, &nb), RSK_ERR_UNSUPPORTED); c.dtype = RSK_F32;
  expect("csr ws null out", rsk_workspace_size_csr(&c, &p, NULL), RSK_ERR_INVALID_ARG);
  expect("csr solve small ws", rsk_avg_solve_csr(&c, DEV(0x4000), &p, DEV(0x5000), DEV(0x6000), DEV(0x7000), 8, NULL),
         RSK_ERR_WORKSPACE);
  expect("csr solve misaligned ws",
         rsk_avg_solve_csr(&c, DEV(0x4000), &p, DEV(0x5000), DEV(0x6000), DEV(0x7008), (size_t)1 << 30, NULL),
         RSK_ERR_WORKSPACE);
  p.alpha = -2.0;
  expect("csr alpha < 0", rsk_avg_solve_csr(&c, DEV(0x4000), &p, DEV(0x5000), DEV(0x6000), DEV(0x7000), 1 << 20, NULL),
         RSK_ERR_INVALID_ARG);
  expect("rownorm2 csr null A", rsk_rownorm2_csr(NULL, DEV(0x8000), NULL), RSK_ERR_INVALID_ARG);
  rsk_dense d = dense(10, 5, 5, RSK_F32);
  expect("rownorm2 dense null out", rsk_rownorm2_dense(&d, NULL, NULL), RSK_ERR_INVALID_ARG);
}

static void check_multirhs_adjoint(void) {
  rsk_dense d = dense(32768, 8192, 8192, RSK_F32);
  rsk_params p = params(820, 10);
  size_t nb = 0;
  int32_t plan[16];
  const unsigned ok = BIT(RSK_OK) | BIT(RSK_ERR_UNSUPPORTED) | BIT(RSK_ERR_HIP);
  expect_in("multirhs ws", rsk_workspace_size_multirhs(&d, 256, &p, &nb), ok);
  expect_in("multirhs plan", rsk_plan_multirhs(&d, 256, &p, plan), ok);
  expect("multirhs R 0", rsk_workspace_size_multirhs(&d, 0, &p, &nb), RSK_ERR_INVALID_ARG);
  expect("multirhs R 6", rsk_workspace_size_multirhs(&d, 6, &p, &nb), RSK_ERR_UNSUPPORTED);
  p.eta = 4097; expect("multirhs eta", rsk_workspace_size_multirhs(&d, 256, &p, &nb), RSK_ERR_UNSUPPORTED);
  p.eta = 820;
  p.y_out = DEV(0x1000); expect("multirhs y", rsk_workspace_size_multirhs(&d, 256, &p, &nb), RSK_ERR_UNSUPPORTED);
  p.y_out = NULL;
  d.dtype = RSK_F64; expect("multirhs f64", rsk_workspace_size_multirhs(&d, 256, &p, &nb), RSK_ERR_UNSUPPORTED);
  d.dtype = RSK_F32;
  d.n = 8190; d.ld = 8190;
  expect("multirhs n % 4", rsk_workspace_size_multirhs(&d, 256, &p, &nb), RSK_ERR_UNSUPPORTED);
  d.n = 8192; d.ld = 8192;
  for (int R = 4; R <= 512; R *= 2)
    for (int eta = 1; eta <= 4096; eta *= 4)
      for (int kern = 0; kern < 5; ++kern) {
        rsk_params q = params(eta, 50);
        q.kernel = kern;
        expect_in("multirhs sweep", rsk_plan_multirhs(&d, R, &q, plan), ok | BIT(RSK_ERR_INVALID_ARG));
        expect_in("adjoint ws sweep", rsk_workspace_size_adjoint(&d, R, &q, 1 + (eta % 20), &nb),
                  ok | BIT(RSK_ERR_INVALID_ARG));
      }
  expect("adjoint ckpt 0", rsk_workspace_size_adjoint(&d, 64, &p, 0, &nb), RSK_ERR_INVALID_ARG);
  expect("adjoint null out", rsk_workspace_size_adjoint(&d, 64, &p, 20, NULL), RSK_ERR_INVALID_ARG);
  double lb = 0.0;
  expect("adjoint null A",
         rsk_avg_adjoint(NULL, DEV(1 << 12), 64, &p, 20, DEV(2 << 12), DEV(3 << 12), DEV(4 << 12), DEV(5 << 12), &lb,
                         DEV(6 << 12), DEV(7 << 12), 1 << 20, NULL),
         RSK_ERR_INVALID_ARG);
}

static void check_batched(void) {
  enum { NS = 3000 };
  rsk_batch_item* items = (rsk_batch_item*)calloc(NS, sizeof(rsk_batch_item));
  int32_t* groups = (int32_t*)calloc(NS, sizeof(int32_t));
  if (!items || !groups) { ++n_fail; return; }
  uint64_t s = 12345;
  for (int i = 0; i < NS; ++i) {
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    const int64_t m = 500 + (int64_t)((s >> 33) % 7501);
    const int64_t n = 200 + (int64_t)((s >> 13) % (uint64_t)(m / 2 - 199));
    rsk_batch_item* it = &items[i];
    it->A = DEV(0x10000000 + (uint64_t)i * 0x100000);
    it->m = m; it->n = n; it->ld = (n + 3) & ~3ll;
    it->b = DEV(0x2000); it->rownorm2 = DEV(0x3000); it->index_stream = (const int32_t*)DEV(0x4000);
    it->K = 100 + i; it->eta = 1 + (int32_t)((s >> 40) % 600); it->alpha = 1.0; it->lambda = 0.5;
    it->x_star = DEV(0x5000); it->x = DEV(0x6000); it->status_dev = (int32_t*)DEV(0x7000);
  }
  const unsigned ok = BIT(RSK_OK) | BIT(RSK_ERR_UNSUPPORTED) | BIT(RSK_ERR_HIP);
  size_t nb = 0;
  int32_t kout = -1;
  static const int64_t wgs[] = {0, 4096, 16 << 10, 1 << 20, (int64_t)1 << 40};
  for (int w = 0; w < 5; ++w)
    for (int kern = 0; kern < 3; ++kern)
      for (int dt = 0; dt < 2; ++dt) {
        for (int nsys = 1; nsys <= NS; nsys *= 7) {
          expect_in("plan batched sweep", rsk_plan_batched(nsys, dt, items, wgs[w], kern, &kout, groups),
                    ok | BIT(RSK_ERR_INVALID_ARG));
          expect_in("ws batched sweep", rsk_workspace_size_batched(nsys, dt, items, wgs[w], kern, &nb),
                    ok | BIT(RSK_ERR_INVALID_ARG));
        }
      }
  expect("batched nsys 0", rsk_workspace_size_batched(0, RSK_F32, items, 0, 0, &nb), RSK_OK);  /* documented */
  expect("batched nsys < 0", rsk_workspace_size_batched(-1, RSK_F32, items, 0, 0, &nb), RSK_ERR_INVALID_ARG);
  expect("batched null items", rsk_workspace_size_batched(4, RSK_F32, NULL, 0, 0, &nb), RSK_ERR_INVALID_ARG);
  expect("batched null out", rsk_workspace_size_batched(4, RSK_F32, items, 0, 0, NULL), RSK_ERR_INVALID_ARG);
  expect("batched dtype", rsk_workspace_size_batched(4, 7, items, 0, 0, &nb), RSK_ERR_UNSUPPORTED);
  rsk_batch_item keep = items[2];
  items[2].m = 0; expect("batched m 0", rsk_workspace_size_batched(4, RSK_F32, items, 0, 0, &nb), RSK_ERR_INVALID_ARG);
  items[2] = keep;
  items[2].eta = 0;
  expect("batched eta 0", rsk_workspace_size_batched(4, RSK_F32, items, 0, 0, &nb), RSK_ERR_INVALID_ARG);
  items[2] = keep;
  items[2].ld = items[2].n - 1;
  expect("batched ld < n", rsk_workspace_size_batched(4, RSK_F32, items, 0, 0, &nb), RSK_ERR_INVALID_ARG);
  items[2] = keep;
  items[2].status_dev = NULL;
  expect("batched no status", rsk_workspace_size_batched(4, RSK_F32, items, 0, 0, &nb), RSK_ERR_INVALID_ARG);
  items[2] = keep;
  expect("batched solve null device items",
         rsk_avg_solve_batched(4, RSK_F32, items, NULL, NULL, 0, 0, DEV(0x8000), 1 << 20, NULL), RSK_ERR_INVALID_ARG);
  expect("batched plan null kernel out", rsk_plan_batched(4, RSK_F32, items, 0, 0, NULL, groups), RSK_ERR_INVALID_ARG);
  free(items);
  free(groups);
}

static void check_sampler_lb_bsk_gather(void) {
  size_t nb = 0;
  expect("cdf ws m 0", rsk_workspace_size_sampling_cdf(0, &nb), RSK_ERR_INVALID_ARG);
  expect("cdf ws null out", rsk_workspace_size_sampling_cdf(10, NULL), RSK_ERR_INVALID_ARG);
  expect_in("cdf ws", rsk_workspace_size_sampling_cdf((int64_t)1 << 30, &nb), BIT(RSK_OK));
  rsk_dense d = dense(1000, 500, 500, RSK_F64);
  expect("cdf dense null cdf", rsk_sampling_cdf_dense(&d, NULL, DEV(0x1000), 1 << 20, NULL), RSK_ERR_INVALID_ARG);
  expect("cdf weights m 0", rsk_sampling_cdf_weights((const double*)DEV(0x1000), 0, (double*)DEV(0x2000), DEV(0x3000),
                                                     1 << 20, NULL),
         RSK_ERR_INVALID_ARG);
  expect("cdf weighted null w", rsk_sampling_cdf_dense_weighted(&d, NULL, (double*)DEV(0x2000), DEV(0x3000), 1 << 20,
                                                                NULL),
         RSK_ERR_INVALID_ARG);
  int32_t* out = (int32_t*)DEV(0x5000);
  const double* cdf = (const double*)DEV(0x6000);
  expect("sample null cdf", rsk_sample_stream(NULL, 10, 1, 0, 5, 2, out, NULL), RSK_ERR_INVALID_ARG);
  expect("sample m 0", rsk_sample_stream(cdf, 0, 1, 0, 5, 2, out, NULL), RSK_ERR_INVALID_ARG);
  expect("sample eta 0", rsk_sample_stream(cdf, 10, 1, 0, 5, 0, out, NULL), RSK_ERR_INVALID_ARG);
  expect("sample K < 0", rsk_sample_stream(cdf, 10, 1, 0, -5, 2, out, NULL), RSK_ERR_INVALID_ARG);
  expect("sample null out", rsk_sample_stream(cdf, 10, 1, 0, 5, 2, NULL, NULL), RSK_ERR_INVALID_ARG);
  expect("sample k0 < 0", rsk_sample_stream(cdf, 10, 1, -1, 5, 2, out, NULL), RSK_ERR_INVALID_ARG);

  rsk_lb_params lp;
  memset(&lp, 0, sizeof lp);
  lp.lambda = 1.0; lp.step = 1e-3; lp.K = 10; lp.status_dev = (int32_t*)DEV(0x7000);
  expect_in("lb ws", rsk_workspace_size_lb_dense(&d, &nb), BIT(RSK_OK) | BIT(RSK_ERR_HIP));
  expect("lb ws null out", rsk_workspace_size_lb_dense(&d, NULL), RSK_ERR_INVALID_ARG);
#define LB() rsk_lb_solve_dense(&d, DEV(0x1000), &lp, DEV(0x2000), DEV(0x3000), DEV(0x4000), (size_t)1 << 24, NULL)
  lp.step = 0.0; expect("lb step 0", LB(), RSK_ERR_INVALID_ARG); lp.step = 1e-3;
  lp.step = NAN; expect("lb step nan", LB(), RSK_ERR_INVALID_ARG); lp.step = 1e-3;
  lp.lambda = -1.0; expect("lb lambda < 0", LB(), RSK_ERR_INVALID_ARG); lp.lambda = 1.0;
  lp.K = -1; expect("lb K < 0", LB(), RSK_ERR_INVALID_ARG); lp.K = 10;
  lp.status_dev = NULL; expect("lb no status", LB(), RSK_ERR_INVALID_ARG); lp.status_dev = (int32_t*)DEV(0x7000);
#undef LB
  double est = 0.0;
  expect("spectral iters 0", rsk_spectral_norm2_dense(&d, 0, DEV(0x1000), &est, DEV(0x2000), 1 << 20, NULL),
         RSK_ERR_INVALID_ARG);
  expect("spectral null est", rsk_spectral_norm2_dense(&d, 10, DEV(0x1000), NULL, DEV(0x2000), 1 << 20, NULL),
         RSK_ERR_INVALID_ARG);

  rsk_params p = params(64, 10);
  expect_in("bsk ws", rsk_workspace_size_bsk_dense(&d, &p, &nb), BIT(RSK_OK) | BIT(RSK_ERR_UNSUPPORTED));
  expect("bsk ws null out", rsk_workspace_size_bsk_dense(&d, &p, NULL), RSK_ERR_INVALID_ARG);
  p.eta = 0;
  expect("bsk eta 0", rsk_bsk_solve_dense(&d, DEV(0x1000), &p, DEV(0x2000), DEV(0x3000), (double*)DEV(0x4000),
                                          DEV(0x5000), 1 << 24, NULL),
         RSK_ERR_INVALID_ARG);

  rsk_dense g = dense(100000, 20000, 20000, RSK_F32);
  float* sink = (float*)DEV(0x9000);
  const int32_t* idx = (const int32_t*)DEV(0xa000);
  expect("gather layout 2", rsk_gather_rate_dense(&g, idx, 1024, 10, 256, 1, 2, sink, NULL), RSK_ERR_INVALID_ARG);
  expect("gather grid 0", rsk_gather_rate_dense(&g, idx, 1024, 10, 0, 1, 0, sink, NULL), RSK_ERR_INVALID_ARG);
  expect("gather eta 0", rsk_gather_rate_dense(&g, idx, 0, 10, 256, 1, 0, sink, NULL), RSK_ERR_INVALID_ARG);
  expect("gather null sink", rsk_gather_rate_dense(&g, idx, 1024, 10, 256, 1, 0, NULL, NULL), RSK_ERR_INVALID_ARG);
  expect("gather groups 3", rsk_gather_rate_dense(&g, idx, 1024, 10, 255, 3, 0, sink, NULL), RSK_ERR_INVALID_ARG);
  expect("gather layout 1 wide slices", rsk_gather_rate_dense(&g, idx, 1024, 10, 64, 1, 1, sink, NULL),
         RSK_ERR_UNSUPPORTED);
  expect("gather K 0", rsk_gather_rate_dense(&g, idx, 1024, 0, 256, 1, 1, sink, NULL), RSK_OK);
  g.dtype = RSK_F64;
  expect("gather f64", rsk_gather_rate_dense(&g, idx, 1024, 10, 256, 1, 0, sink, NULL), RSK_ERR_UNSUPPORTED);
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : ".";
  check_status_strings();
  check_tune_table(dir);
  check_dense();
  check_csr();
  check_multirhs_adjoint();
  check_batched();
  check_sampler_lb_bsk_gather();
  printf("rsk_host_check: %d checks, %d failed\n", n_calls, n_fail);
  return n_fail ? 1 : 0;
}
