// C ABI of librsk: validation, planning, workspace layout and launches.
// The operation every entry point performs is documented in include/rsk.h.
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "rsk.h"
#include "rsk_kernels.hpp"

using rsk::u64;

namespace {

// ---------------------------------------------------------------------------
// Tuning table: the choices kernel = 0 / grid = 0 (dense), the split of the multi-RHS products and
// the batched workgroup targets read, written by a tuner (rsk_tune_set) or a cache file
// (rsk_tune_load; RSK_TUNE_CACHE names one read at the first lookup). Process-global; a lookup
// holds the lock only while it copies an entry.
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::vector<rsk_tune_entry> g_tune;
bool g_tune_env_done = false;

bool tune_same_key(const rsk_tune_entry& a, const rsk_tune_entry& b) {
  return a.path == b.path && a.dtype == b.dtype && a.m == b.m && a.n == b.n && a.eta == b.eta && a.R == b.R;
}

int32_t tune_load_locked(const char* path);

void tune_env_locked() {
  if (g_tune_env_done) return;
  g_tune_env_done = true;
  const char* f = getenv("RSK_TUNE_CACHE");
  if (f && *f) tune_load_locked(f);
}

bool tune_find(int32_t path, int32_t dtype, int64_t m, int64_t n, int32_t eta, int32_t R, rsk_tune_entry* out) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_env_locked();
  rsk_tune_entry key{};
  key.path = path; key.dtype = dtype; key.m = m; key.n = n; key.eta = eta; key.R = R;
  for (const rsk_tune_entry& e : g_tune)
    if (tune_same_key(e, key)) { *out = e; return true; }
  return false;
}

void tune_put_locked(const rsk_tune_entry& e) {
  for (rsk_tune_entry& x : g_tune)
    if (tune_same_key(x, e)) { x = e; return; }
  g_tune.push_back(e);
}

// the batched classes of one dtype and launch kind (key R: 0 general kernel, 2 register tile),
// ascending by their step-byte bound
rsk::BatchWgTable tune_batch_table(int32_t dtype, int kind) {
  rsk::BatchWgTable t{};
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_env_locked();
  std::vector<rsk_tune_entry> cls;
  const int32_t key_r = kind == 2 ? 2 : 0;
  for (const rsk_tune_entry& e : g_tune)
    if (e.path == RSK_TUNE_BATCHED && e.dtype == dtype && e.R == key_r && e.v0 > 0) cls.push_back(e);
  std::sort(cls.begin(), cls.end(), [](const rsk_tune_entry& a, const rsk_tune_entry& b) { return a.m < b.m; });
  for (const rsk_tune_entry& e : cls) {
    if (t.nc == rsk::kBatchClasses) break;
    t.hi[t.nc] = e.m;
    t.wg[t.nc] = e.v0;
    ++t.nc;
  }
  return t;
}

// Cache file: one entry per line, whitespace-separated:
//   path dtype m n eta R v0 v1 v2 us
// '#' starts a comment line. Unknown paths and malformed lines are skipped.
int32_t tune_load_locked(const char* path) {
  FILE* f = fopen(path, "r");
  if (!f) return RSK_ERR_INVALID_ARG;
  char line[512];
  while (fgets(line, sizeof line, f)) {
    if (line[0] == '#') continue;
    rsk_tune_entry e{};
    long long m, n, v0, v1, v2;
    int pth, dt, eta, R;
    double us;
    if (sscanf(line, "%d %d %lld %lld %d %d %lld %lld %lld %lf", &pth, &dt, &m, &n, &eta, &R, &v0, &v1, &v2, &us) != 10)
      continue;
    if (pth < RSK_TUNE_DENSE || pth > RSK_TUNE_BATCHED) continue;
    e.path = pth; e.dtype = dt; e.m = m; e.n = n; e.eta = eta; e.R = R; e.v0 = v0; e.v1 = v1; e.v2 = v2; e.us = us;
    tune_put_locked(e);
  }
  fclose(f);
  return RSK_OK;
}

constexpr int kMaxEtaDense = 16384;
constexpr size_t kTileCacheBytes = 96 * 1024;
// both tiles of the pipelined row tile (the next step's rows loaded during the step)
constexpr size_t kPipeTileBytes = 128 * 1024;
// General-kernel grid for grid = 0. A step is a chain of dependent round trips, so below a few MB
// it is bound by latency, not bytes: one workgroup (no exchange) while the step and its rows are
// small, else about 4 KB of rows per workgroup on 16..128 workgroups, the whole chip for big steps.
constexpr size_t kOneWgStepBytes = 32 * 1024, kOneWgRowBytes = 16 * 1024;
// the one-workgroup register kernel (kernel 4) is the float64 default for steps up to this size
constexpr double kSmallStepBytes = 64.0 * 1024;
constexpr size_t kBytesPerWg = 4 * 1024;
constexpr int kMinSpreadG = 16, kMaxSpreadG = 128;
constexpr size_t kFullGridStepBytes = size_t(8) << 20;
using rsk::kOneHopWords;
// the automatic choice takes two row groups of the register-tile kernel for eta in this range
// (measured on 20000 columns: below it one group is as fast, the step being bound by the
// exchange; above it the third exchange hop costs more than the wider row pieces save), unless one
// group's whole next-step tile fits the kernel's LDS prefetch (kRtPfBytes of LDS): then one group
// is faster (20000 columns, eta = 96 ... 256: 4-7% shorter steps)
constexpr int kRtTwoGroupMinEta = 88, kRtTwoGroupMaxEta = 800;
constexpr int kRtPfBytes = 147456;

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }
size_t elem_size(int32_t dt) { return dt == RSK_F64 ? 8 : 4; }

int device_cus() {
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return cus;
}

int next_pow2(int v) {
  int p = 1;
  while (p < v) p <<= 1;
  return p;
}

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

int32_t check_params(const rsk_params* p, int64_t m) {
  if (!p) return RSK_ERR_INVALID_ARG;
  if (p->eta < 1 || p->K < 0 || p->K >= (int64_t(1) << 31) || p->stream_offset < 0) return RSK_ERR_INVALID_ARG;
  if (!(p->lambda >= 0.0) || !isfinite(p->lambda)) return RSK_ERR_INVALID_ARG;
  if (!p->alpha_k && !finite_pos(p->alpha)) return RSK_ERR_INVALID_ARG;
  if (p->K > 0 && !p->index_stream) return RSK_ERR_INVALID_ARG;
  if (!p->rownorm2 || !p->status_dev) return RSK_ERR_INVALID_ARG;
  if (p->check_every < 0 || !(p->tol >= 0.0) || p->grid < 0) return RSK_ERR_INVALID_ARG;
  if (p->kernel < 0 || p->kernel > 4) return RSK_ERR_INVALID_ARG;
  if (p->x_ref && p->check_every > 0 && p->err_hist == nullptr && p->tol <= 0.0) return RSK_ERR_INVALID_ARG;
  (void)m;
  return RSK_OK;
}

struct DensePlan {
  int kernel;  // 1 general, 2 register tile, 4 one workgroup with the step in registers
  int nt, rp, cpl, rg;
  int vec, G, two_hop, tile_cache, wq_max, lpr, W;
  int64_t nchunks;
  size_t offP, offC, offM, offU, bytes;
};

// uwords: words of the register-tile kernel's third exchange hop (0 with one row group)
size_t dense_ws_layout(int Gmax, int eta, int W, size_t uwords, DensePlan* pl) {
  size_t o = 0;
  pl->offP = o; o = align256(o + 2 * (size_t)Gmax * eta * W * sizeof(u64));
  pl->offC = o; o = align256(o + (size_t)eta * W * sizeof(u64));
  pl->offM = o; o = align256(o + (size_t)Gmax * 4 * sizeof(u64));
  pl->offU = o; o = align256(o + uwords * sizeof(u64));
  pl->bytes = o;
  return o;
}

int dense_grid_cap(const rsk_dense* A, const rsk_params* p) {
  const int cus = device_cus();
  int cap = p->grid > 0 ? p->grid : (cus > 0 ? cus : 1);
  if (cap > A->n) cap = (int)A->n;
  return cap < 1 ? 1 : cap;
}

int32_t check_dense(const rsk_dense* A) {
  if (!A || !A->val) return RSK_ERR_INVALID_ARG;
  if (A->m <= 0 || A->n <= 0 || A->ld < A->n) return RSK_ERR_INVALID_ARG;
  if (A->m > INT32_MAX) return RSK_ERR_UNSUPPORTED;
  if (A->dtype != RSK_F32 && A->dtype != RSK_F64) return RSK_ERR_UNSUPPORTED;
  return RSK_OK;
}

// float32 register-tile plan: one 1024-thread workgroup per CU (512 for eta > 768), eta <= 1024,
// rg row groups of G/rg column slices, each slice at most 5*rg units of 16 floats. Returns false,
// with *pl unchanged, if it does not apply.
bool plan_dense_rt(const rsk_dense* A, const rsk_params* p, int rg, DensePlan* pl) {
  if (A->dtype != RSK_F32 || (A->n % 4) != 0 || (A->ld % 4) != 0 || (((uintptr_t)A->val) % 16) != 0) return false;
  const int64_t nchunks = (A->n + 3) / 4;
  const int64_t nunits = (nchunks + 3) / 4;
  const int cus = device_cus();
  int G = p->grid > 0 ? p->grid : cus;
  if (G > nunits * rg) G = (int)(nunits * rg);
  if (rg > 1 && G >= 16) G -= G % 8;  // whole XCD rounds keep a slice's groups on one XCD
  G -= G % rg;
  if (G > 256) return false;
  if (G < rg) return false;
  const int C = G / rg;
  const int64_t upm = (nunits + C - 1) / C;  // units of the widest slice
  const int cpl = (int)((upm + rg - 1) / rg);
  if (cpl > rsk::kRtMaxCPL || p->eta > rsk::kRtMaxEta) return false;
  const int nt = p->eta <= 768 ? 1024 : 512;
  const int etaR = (p->eta + rg - 1) / rg;
  const int rpp = nt / (4 * rg);  // group rows of one pass
  const int rp = (etaR + rpp - 1) / rpp;
  if (rsk::dense_rt_max_grid(nt, rp, cpl, rg) < G) return false;
  int two_hop = ((int64_t)C * etaR) > rsk::kRtOneHopWords;
  // each wave reduces at most kRtOwnMax rows per step
  const int own = rsk::kRtOwnMax * (nt / 64);
  if (!two_hop && etaR > own) two_hop = 1;
  if (two_hop && (etaR + C - 1) / C > own) return false;
  // the plan is written only once the kernel applies: a caller falls back to the general
  // kernel with *pl as it was
  pl->kernel = 2; pl->nt = nt; pl->rp = rp; pl->cpl = cpl; pl->rg = rg;
  pl->vec = 4; pl->W = 1; pl->nchunks = nchunks; pl->G = G;
  pl->wq_max = 4 * rg * cpl; pl->lpr = 4; pl->tile_cache = 0;
  pl->two_hop = two_hop;
  const int cap = dense_grid_cap(A, p);
  const size_t uwords = rg > 1 ? 2 * (size_t)G * 16 * rg * cpl : 0;
  dense_ws_layout(cap > G ? cap : G, p->eta, 1, uwords, pl);
  return true;
}

template <typename T>
int32_t plan_dense_fixed(const rsk_dense* A, const rsk_params* p, DensePlan* pl);

// kernel = 0 and grid = 0: a tuned (kernel, grid) for this (dtype, m, n, eta), if the table has one
// that applies to this matrix (alignment and leading dimension are not part of the key); else the
// built-in choice.
template <typename T>
int32_t plan_dense(const rsk_dense* A, const rsk_params* p, DensePlan* pl) {
  rsk_tune_entry e;
  if (p->kernel == 0 && p->grid == 0 &&
      tune_find(RSK_TUNE_DENSE, A->dtype, A->m, A->n, p->eta, 0, &e) && e.v0 >= 1 && e.v0 <= 4 && e.v1 >= 1) {
    rsk_params q = *p;
    q.kernel = (int32_t)e.v0;
    q.grid = (int32_t)e.v1;
    DensePlan t;
    if (plan_dense_fixed<T>(A, &q, &t) == RSK_OK) {
      *pl = t;
      return RSK_OK;
    }
  }
  return plan_dense_fixed<T>(A, p, pl);
}

template <typename T>
int32_t plan_dense_fixed(const rsk_dense* A, const rsk_params* p, DensePlan* pl) {
  const size_t s = sizeof(T);
  pl->kernel = 1; pl->nt = pl->rp = pl->cpl = 0; pl->rg = 1;
  // one workgroup, the step in registers: asked for, or by default for a small system whose step
  // is bound by latency (a float64 step of at most kSmallStepBytes)
  const int cpt = rsk::dense_small_cpt(A->n, p->eta);
  if (p->kernel == 4 || (p->kernel == 0 && p->grid <= 1 && cpt && A->dtype == RSK_F64 &&
                         (double)p->eta * (double)A->n * (double)s <= kSmallStepBytes)) {
    if (!cpt || p->grid > 1) return RSK_ERR_UNSUPPORTED;
    pl->kernel = 4; pl->nt = 256; pl->cpl = cpt; pl->vec = 1; pl->W = (int)(s / 4);
    pl->nchunks = A->n; pl->G = 1; pl->wq_max = (int)A->n; pl->lpr = 1; pl->tile_cache = 0; pl->two_hop = 0;
    dense_ws_layout(1, p->eta, pl->W, 0, pl);
    return RSK_OK;
  }
  // float32: the register-tile kernel wherever its shape limits allow; its exchange is cheaper
  // than the general kernel's at every step size measured, one row per step included
  if (p->kernel == 3) return plan_dense_rt(A, p, 2, pl) ? RSK_OK : RSK_ERR_UNSUPPORTED;
  if (p->kernel == 2 || (p->kernel == 0 && A->dtype == RSK_F32)) {
    if (p->kernel == 0 && p->eta >= kRtTwoGroupMinEta && p->eta <= kRtTwoGroupMaxEta) {
      DensePlan one = *pl;
      const bool whole = plan_dense_rt(A, p, 1, &one) && one.rp * one.cpl <= kRtPfBytes / (one.nt * 16);
      if (!whole && plan_dense_rt(A, p, 2, pl)) return RSK_OK;
    }
    if (plan_dense_rt(A, p, 1, pl)) return RSK_OK;
    if (p->kernel == 2) return RSK_ERR_UNSUPPORTED;
  }
  const int vmax = (int)(16 / s);
  pl->vec = ((A->ld % vmax) == 0 && (((uintptr_t)A->val) % 16) == 0) ? vmax : 1;
  pl->W = (int)(s / 4);
  pl->nchunks = (A->n + pl->vec - 1) / pl->vec;
  const int cap = dense_grid_cap(A, p);
  int G;
  if (p->grid > 0) {
    G = p->grid;
  } else {
    const double row_bytes = (double)A->n * (double)s, step_bytes = (double)p->eta * row_bytes;
    if (step_bytes <= kOneWgStepBytes && row_bytes <= kOneWgRowBytes) {
      G = 1;
    } else if (step_bytes >= kFullGridStepBytes) {
      G = cap;
    } else {
      const double g = ceil(step_bytes / (double)kBytesPerWg);
      G = g < kMinSpreadG ? kMinSpreadG : g > kMaxSpreadG ? kMaxSpreadG : (int)g;
    }
    if (G >= 16) G -= G % 8;
  }
  if (G > cap) G = cap;
  if (G > pl->nchunks) G = (int)pl->nchunks;
  if (G < 1) G = 1;
  for (;;) {
    pl->G = G;
    pl->wq_max = (int)((pl->nchunks + G - 1) / G);
    pl->lpr = next_pow2(pl->wq_max) < 64 ? next_pow2(pl->wq_max) : 64;
    const size_t tile_bytes = (size_t)p->eta * pl->wq_max * pl->vec * s;
    pl->tile_cache = tile_bytes <= kTileCacheBytes;
    pl->two_hop = ((int64_t)G * p->eta * pl->W) > kOneHopWords;
    size_t lds = 0;
    const int64_t xr = pl->two_hop ? 0 : rsk::onehop_lds_elems(G, p->eta);
    // the pipelined tile (next step's rows loaded during the step) for one workgroup, where two
    // tiles fit: with an exchange its step is no faster (measured on 1000x500 float64, eta = 10,
    // 16 workgroups: 8.4 against 6.9 us), as the exchange, not the row loads, sets the pace
    if (G == 1 && rsk::dense_pipe_ok(s, pl->vec, p->eta, pl->wq_max) && 2 * tile_bytes <= kPipeTileBytes &&
        rsk::dense_max_grid<T>(pl->vec, p->eta, pl->wq_max, 2, xr, &lds) >= G) {
      pl->tile_cache = 2;
      break;
    }
    int maxg = rsk::dense_max_grid<T>(pl->vec, p->eta, pl->wq_max, pl->tile_cache, xr, &lds);
    if (maxg == 0 && pl->tile_cache) {
      pl->tile_cache = 0;
      maxg = rsk::dense_max_grid<T>(pl->vec, p->eta, pl->wq_max, 0, xr, &lds);
    }
    if (maxg >= G) break;
    if (maxg == 0) {
      if (G >= cap) return RSK_ERR_UNSUPPORTED;  // slice too wide for LDS even at the largest grid
      G = cap;  // wider grid, narrower slices
      continue;
    }
    if (p->grid > 0) return RSK_ERR_UNSUPPORTED;
    G = maxg;
  }
  dense_ws_layout(cap > pl->G ? cap : pl->G, p->eta, pl->W, 0, pl);
  return RSK_OK;
}

template <typename T>
int32_t solve_dense_t(const rsk_dense* A, const void* b, const rsk_params* p, void* x_star, void* x,
                      void* ws, size_t ws_bytes, hipStream_t stream, bool zero_status = true) {
  DensePlan pl;
  int32_t st = plan_dense<T>(A, p, &pl);
  if (st) return st;
  if (!ws || ws_bytes < pl.bytes) return RSK_ERR_WORKSPACE;
  if (((uintptr_t)ws) % 256) return RSK_ERR_WORKSPACE;
  unsigned char* w = (unsigned char*)ws;
  rsk::DenseArgs<T> a;
  a.A = (const T*)A->val; a.m = A->m; a.n = A->n; a.ld = A->ld;
  a.b = (const T*)b; a.r2 = (const T*)p->rownorm2; a.row_w = (const T*)p->row_w;
  a.lambda = (T)p->lambda; a.alpha = (T)p->alpha; a.alpha_k = (const T*)p->alpha_k;
  a.eta = p->eta; a.K = p->K;
  a.idx = p->index_stream ? p->index_stream + p->stream_offset : nullptr;
  a.x_star = (T*)x_star; a.x = (T*)x; a.warm = p->warm_start ? 1 : 0;
  a.y = (T*)p->y_out;
  a.xref = (const T*)p->x_ref; a.check_every = p->x_ref ? p->check_every : 0; a.tol = p->tol;
  a.err_hist = p->err_hist; a.status = p->status_dev;
  a.xP = (u64*)(w + pl.offP); a.xC = (u64*)(w + pl.offC); a.xM = (u64*)(w + pl.offM);
  a.xU = pl.rg > 1 ? (u64*)(w + pl.offU) : nullptr;
  a.G = pl.G; a.two_hop = pl.two_hop; a.tile_cache = pl.tile_cache;
  a.nchunks = pl.nchunks; a.wq_max = pl.wq_max; a.lpr = pl.lpr;
  if (rsk::launch_zero_words((u64*)w, pl.bytes / sizeof(u64), stream) != hipSuccess) return RSK_ERR_HIP;
  if (zero_status && rsk::launch_zero_status(p->status_dev, stream) != hipSuccess) return RSK_ERR_HIP;
  if (pl.kernel == 2) {
    if (rsk::launch_dense_rt(*reinterpret_cast<rsk::DenseArgs<float>*>(&a), pl.nt, pl.rp, pl.cpl, pl.rg, stream) !=
        hipSuccess)
      return RSK_ERR_HIP;
    return RSK_OK;
  }
  if (pl.kernel == 4) return rsk::launch_dense_small<T>(a, stream) == hipSuccess ? RSK_OK : RSK_ERR_HIP;
  int maxg = 0;
  if (rsk::launch_dense<T>(a, pl.vec, stream, &maxg) != hipSuccess) return RSK_ERR_HIP;
  return RSK_OK;
}

int32_t check_csr(const rsk_csr* A) {
  if (!A || !A->row_ptr || !A->col || !A->val) return RSK_ERR_INVALID_ARG;
  if (A->m <= 0 || A->n <= 0 || A->nnz < 0) return RSK_ERR_INVALID_ARG;
  if (A->m > INT32_MAX || A->n > INT32_MAX) return RSK_ERR_UNSUPPORTED;
  if (A->dtype != RSK_F32 && A->dtype != RSK_F64) return RSK_ERR_UNSUPPORTED;
  return RSK_OK;
}

// CSR plan: one workgroup (small steps) or the multi-workgroup kernel.
// Workspace: n + 1 int64 column accumulators (the last a spare slot); with a
// dual output, m per-row slot counters and (grid kernel) the step's eta
// coefficients; then for the grid kernel the barrier counter, the step-parity
// exponent words and the monitor words.
struct CsrPlan {
  int kernel, G;
  size_t offYcnt, offCy, offBar, offEmax, offM, bytes;
};

template <typename T>
int32_t plan_csr(const rsk_csr* A, const rsk_params* p, CsrPlan* pl) {
  const int cus = device_cus() > 0 ? device_cus() : 1;
  const int rpp = rsk::kCsrGridRowsPerPass;
  if (p->kernel == 3 || p->kernel == 4) return RSK_ERR_INVALID_ARG;  // dense kernels
  const bool grid = p->kernel == 2 || (p->kernel == 0 && p->eta >= 4);
  pl->kernel = grid ? 2 : 1;
  pl->G = 1;
  size_t o = align256((size_t)(A->n + 1) * sizeof(long long));
  pl->offYcnt = pl->offCy = 0;
  if (p->y_out) {
    pl->offYcnt = o; o = align256(o + (size_t)A->m * sizeof(int));
    if (grid) { pl->offCy = o; o = align256(o + (size_t)p->eta * sizeof(T)); }
  }
  pl->offBar = pl->offEmax = pl->offM = o;
  if (grid) {
    int G = p->grid > 0 ? p->grid : (p->eta + rpp - 1) / rpp;
    if (p->grid <= 0 && G > cus) G = cus;
    const int maxres = rsk::csr_grid_max_resident<T>();
    if (G < 1 || (maxres > 0 && G > maxres)) return RSK_ERR_UNSUPPORTED;
    if ((p->eta + rpp * G - 1) / (rpp * G) > rsk::kCsrGridMaxPasses) return RSK_ERR_UNSUPPORTED;
    pl->G = G;
    pl->offBar = o; o += 9 * 128;  // global barrier counter and 8 group counters, 128 bytes apart
    pl->offEmax = o; o += 64;
    pl->offM = o; o = align256(o + (size_t)G * 4 * sizeof(u64));
  }
  pl->bytes = o;
  return RSK_OK;
}

template <typename T>
int32_t solve_csr_t(const rsk_csr* A, const void* b, const rsk_params* p, void* x_star, void* x, void* ws,
                    size_t ws_bytes, hipStream_t stream) {
  CsrPlan pl;
  int32_t st = plan_csr<T>(A, p, &pl);
  if (st) return st;
  if (!ws || ws_bytes < pl.bytes || ((uintptr_t)ws) % 256) return RSK_ERR_WORKSPACE;
  unsigned char* w = (unsigned char*)ws;
  rsk::CsrArgs<T> a;
  a.row_ptr = A->row_ptr; a.col = A->col; a.val = (const T*)A->val; a.m = A->m; a.n = A->n;
  a.b = (const T*)b; a.r2 = (const T*)p->rownorm2; a.row_w = (const T*)p->row_w;
  a.lambda = (T)p->lambda; a.alpha = (T)p->alpha; a.alpha_k = (const T*)p->alpha_k;
  a.eta = p->eta; a.K = p->K;
  a.idx = p->index_stream ? p->index_stream + p->stream_offset : nullptr;
  a.x_star = (T*)x_star; a.x = (T*)x; a.warm = p->warm_start ? 1 : 0;
  a.y = (T*)p->y_out;
  a.xref = (const T*)p->x_ref; a.check_every = p->x_ref ? p->check_every : 0; a.tol = p->tol;
  a.err_hist = p->err_hist; a.status = p->status_dev;
  a.acc = (long long*)ws;
  a.ycnt = p->y_out ? (int*)(w + pl.offYcnt) : nullptr;
  a.cy = p->y_out && pl.offCy ? (T*)(w + pl.offCy) : nullptr;
  a.G = pl.G;
  a.bar = (u64*)(w + pl.offBar);
  a.emax = (int*)(w + pl.offEmax);
  a.xM = (u64*)(w + pl.offM);
  if (rsk::launch_zero_words((u64*)ws, pl.bytes / sizeof(u64), stream) != hipSuccess) return RSK_ERR_HIP;
  if (rsk::launch_zero_status(p->status_dev, stream) != hipSuccess) return RSK_ERR_HIP;
  const hipError_t e = pl.kernel == 2 ? rsk::launch_csr_grid<T>(a, stream) : rsk::launch_csr<T>(a, stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

struct MultiPlan {
  int S, eta_pad, S2;
  int64_t kspan;
  int kernel;       // 1: step kernels (four per step), 2: one persistent launch for all K steps,
                    // 3: the step kernels with wide product tiles (128 x 128, or 128 x 64 for R <= 64)
  int tile;         // 64 (kernels 1, 2) or 128 (kernel 3): the tile edge of the products
  int pS;           // persistent launch: its split of the n columns (kspan rounded up to 64)
  int64_t pkspan;
  size_t offY, offC, offW, offCnt, cnt_words, bytes;
};

int32_t plan_multirhs(const rsk_dense* A, int32_t R, const rsk_params* p, MultiPlan* pl) {
  if (A->dtype != RSK_F32) return RSK_ERR_UNSUPPORTED;
  if (R <= 0) return RSK_ERR_INVALID_ARG;
  if ((R % 4) || (A->n % 4) || (A->ld % 4) || (((uintptr_t)A->val) % 16)) return RSK_ERR_UNSUPPORTED;
  if (p->x_ref || p->y_out || p->check_every) return RSK_ERR_UNSUPPORTED;
  if (p->eta > 4096) return RSK_ERR_UNSUPPORTED;  // the sampled rows of a step are staged in LDS
  if (p->kernel < 0 || p->kernel > 3) return RSK_ERR_INVALID_ARG;
  const int cus = device_cus() > 0 ? device_cus() : 256;
  rsk_tune_entry te;
  const bool tuned = tune_find(RSK_TUNE_MULTIRHS, A->dtype, A->m, A->n, p->eta, R, &te);
  // the kernel: p->kernel 1, 2 or 3 as asked, else a tuned choice, else the wide-tile step kernels
  // when R and eta each fill at least one 128 tile, the 64 x 64 ones below that
  pl->kernel = p->kernel >= 1 ? p->kernel
             : (tuned && te.v2 >= 1 && te.v2 <= 3 ? (int)te.v2 : (R > 64 && p->eta >= 128 ? 3 : 1));
  pl->tile = pl->kernel == 3 ? 128 : 64;
  const int tn = pl->tile == 128 && R <= 64 ? 64 : pl->tile;  // the R edge of a product tile
  pl->eta_pad = (p->eta + pl->tile - 1) / pl->tile * pl->tile;
  const int tiles = (pl->eta_pad / pl->tile) * ((R + tn - 1) / tn);
  // about three 256-thread workgroups per CU for the n-long products, in whole XCD rounds (the
  // tiles of a split share one L2); or one 512-thread wide-tile workgroup per CU, rounded down (a
  // second round on some CUs costs more than a few idle CUs or the L2 sharing)
  int S = pl->tile == 128 ? cus / tiles : (3 * cus + tiles - 1) / tiles;
  if (S >= 8 && pl->tile != 128) S = (S + 7) / 8 * 8;
  if (tuned && te.v0 >= 1) S = (int)(te.v0 < 4096 ? te.v0 : 4096);
  // at least 256 columns a split by the built-in rule, at least 64 (one stage) for a tuned split
  const int64_t max_s = tuned && te.v0 >= 1 ? (A->n + 63) / 64 : (A->n + 255) / 256;
  if (S > max_s) S = (int)max_s;
  if (S < 1) S = 1;
  pl->kspan = (A->n + S - 1) / S;
  pl->kspan = (pl->kspan + 15) / 16 * 16;
  pl->S = (int)((A->n + pl->kspan - 1) / pl->kspan);
  // the A_tau^T products write n x R: with fewer 64 x 64 tiles than CUs their sampled rows
  // are split over S2 workgroups (at least 64 rows each) and summed in a second kernel
  const int att_tiles = (int)((A->n + pl->tile - 1) / pl->tile) * ((R + tn - 1) / tn);
  int S2 = cus / att_tiles;
  // the wide tiles' fused update (no row split) runs 128 x 64 tiles: when those fill the device
  // there is nothing to split
  if (pl->tile == 128 && R > 64 && ((A->n + 127) / 128) * ((R + 63) / 64) >= cus) S2 = 1;
  // at least 64 rows a split by the built-in rule, at least 16 for a tuned split
  const int max_s2 = tuned && te.v1 >= 1 ? (p->eta + 15) / 16 : (p->eta + 63) / 64;
  if (S2 > max_s2) S2 = max_s2;
  if (tuned && te.v1 >= 1) S2 = (int)(te.v1 < 8 ? te.v1 : 8);
  if (S2 > max_s2) S2 = max_s2;
  S2 = S2 >= 8 ? 8 : S2 >= 4 ? 4 : S2 >= 2 ? 2 : 1;  // the reduction kernels take 2, 4 or 8
  pl->S2 = S2;
  pl->pkspan = (pl->kspan + 63) / 64 * 64;
  pl->pS = (int)((A->n + pl->pkspan - 1) / pl->pkspan);
  const int64_t gt = pl->eta_pad / 64, gr = (R + 63) / 64, gn = (A->n + 63) / 64;
  pl->cnt_words = (size_t)(gt * gr + gr + (int64_t)pl->S * gr + gn * gr);
  size_t o = 0;
  pl->offY = o; o = align256(o + (size_t)pl->S * pl->eta_pad * R * sizeof(float));
  pl->offC = o; o = align256(o + (size_t)pl->eta_pad * R * sizeof(float));
  pl->offW = o; o = align256(o + (S2 > 1 ? (size_t)S2 * A->n * R * sizeof(float) : 0));
  pl->offCnt = o; o = align256(o + pl->cnt_words * sizeof(unsigned));
  pl->bytes = o;
  return RSK_OK;
}

int32_t check_batch_item(const rsk_batch_item& it) {
  if (!it.A || !it.b || !it.rownorm2 || !it.x_star || !it.x || !it.status_dev) return RSK_ERR_INVALID_ARG;
  if (it.m <= 0 || it.n <= 0 || it.ld < it.n || it.eta < 1 || it.K < 0 || it.K >= (int64_t(1) << 31))
    return RSK_ERR_INVALID_ARG;
  if (it.K > 0 && !it.index_stream) return RSK_ERR_INVALID_ARG;
  if (!(it.lambda >= 0.0) || !isfinite(it.lambda) || !finite_pos(it.alpha)) return RSK_ERR_INVALID_ARG;
  if (it.check_every < 0 || !(it.tol >= 0.0)) return RSK_ERR_INVALID_ARG;
  if (it.x_ref && it.check_every > 0 && !it.err_hist && it.tol <= 0.0) return RSK_ERR_INVALID_ARG;
  if (it.m > INT32_MAX || it.eta > kMaxEtaDense) return RSK_ERR_UNSUPPORTED;
  return RSK_OK;
}

// Workspace of a batch: [256 B: ticket counter][ticket starts, nsys+1 int64]
// [region offsets, nsys int64][one exchange region per system].
struct BatchLayout {
  int kind;  // 1 general kernel, 2 register tile
  int vec, gmax;
  rsk::BatchWgTable tab;
  int64_t tickets, words;
  size_t lds, off_t0, off_woff, off_region, bytes;
};

rsk::BatchWgTable batch_table(int32_t dtype, int kind, int64_t wg_bytes) {
  if (wg_bytes > 0) {
    rsk::BatchWgTable t{};
    t.nc = 1;
    t.hi[0] = INT64_MAX;
    t.wg[0] = wg_bytes;
    return t;
  }
  return tune_batch_table(dtype, kind);  // no classes: every system takes the kind's default target
}

// The launch of a batch: kernel 1 (general), 2 (register tile: float32, every system's rows 16-byte
// aligned and its plan within the tile's limits, else RSK_ERR_UNSUPPORTED) or 0 (the register tile
// where every system takes it, else the general kernel); each system's plan and the workspace.
int32_t batch_layout(int32_t nsys, int32_t dtype, const rsk_batch_item* items, int64_t wg_bytes, int32_t kernel,
                     BatchLayout* L, int32_t* g_out = nullptr) {
  if (nsys < 0 || (nsys > 0 && !items) || wg_bytes < 0 || kernel < 0 || kernel > 2) return RSK_ERR_INVALID_ARG;
  if (dtype != RSK_F32 && dtype != RSK_F64) return RSK_ERR_UNSUPPORTED;
  const size_t es = elem_size(dtype);
  const int vmax = (int)(16 / es);
  L->vec = vmax;
  for (int32_t i = 0; i < nsys; ++i) {
    const int32_t st = check_batch_item(items[i]);
    if (st) return st;
    if ((items[i].ld % vmax) != 0 || ((uintptr_t)items[i].A) % 16 != 0) L->vec = 1;
  }
  L->kind = 1;
  if (kernel != 1 && dtype == RSK_F32 && L->vec == 4 && nsys > 0) {
    const rsk::BatchWgTable tab = batch_table(dtype, 2, wg_bytes);
    bool all = true;
    for (int32_t i = 0; i < nsys && all; ++i) {
      rsk::BatchPlan pl;
      all = rsk::batched_rt_plan(items[i].n, items[i].eta, tab, &pl);
    }
    if (all) L->kind = 2;
  }
  if (kernel == 2 && L->kind != 2) return RSK_ERR_UNSUPPORTED;
  L->tab = batch_table(dtype, L->kind, wg_bytes);
  L->gmax = 0; L->tickets = 0; L->words = 0; L->lds = 0;
  for (int32_t i = 0; i < nsys; ++i) {
    rsk::BatchPlan pl;
    const bool ok = L->kind == 2 ? rsk::batched_rt_plan(items[i].n, items[i].eta, L->tab, &pl)
                                 : rsk::batched_plan(items[i].n, items[i].eta, (int)es, L->vec, L->tab, &pl);
    if (!ok) return RSK_ERR_UNSUPPORTED;
    if (g_out) g_out[i] = pl.G;
    if (pl.G > L->gmax) L->gmax = pl.G;
    if (pl.lds > L->lds) L->lds = pl.lds;
    L->tickets += pl.G;
    L->words += pl.words;
  }
  size_t o = 256;
  L->off_t0 = o; o = align256(o + (size_t)(nsys + 1) * sizeof(int64_t));
  L->off_woff = o; o = align256(o + (size_t)nsys * sizeof(int64_t));
  L->off_region = o; o = align256(o + (size_t)L->words * sizeof(u64));
  L->bytes = o;
  return RSK_OK;
}

void fill_multirhs(const rsk_dense* A, const void* B, int32_t R, const rsk_params* p, void* X_star, void* X,
                   const MultiPlan* plp, void* workspace, rsk::MultiRhsArgs* ap) {
  const MultiPlan& pl = *plp;
  rsk::MultiRhsArgs& a = *ap;
  unsigned char* w = (unsigned char*)workspace;
  a.A = (const float*)A->val; a.m = A->m; a.n = A->n; a.ld = A->ld;
  a.B = (const float*)B; a.R = R; a.r2 = (const float*)p->rownorm2; a.row_w = (const float*)p->row_w;
  a.lambda = (float)p->lambda; a.alpha = (float)p->alpha; a.alpha_k = (const float*)p->alpha_k;
  a.eta = p->eta; a.K = p->K;
  a.idx = p->index_stream ? p->index_stream + p->stream_offset : nullptr;
  a.x_star = (float*)X_star; a.x = (float*)X; a.warm = p->warm_start ? 1 : 0;
  a.status = p->status_dev;
  a.Y = (float*)(w + pl.offY); a.C = (float*)(w + pl.offC);
  a.S = pl.S; a.eta_pad = pl.eta_pad; a.kspan = pl.kspan; a.tile = pl.tile;
  // the row-split epilogue moves float4 of X* and X: used only when both are 16-byte aligned
  const bool al = ((uintptr_t)X_star) % 16 == 0 && ((uintptr_t)X) % 16 == 0;
  a.S2 = (pl.S2 > 1 && al) ? pl.S2 : 1;
  a.Wp = a.S2 > 1 ? (float*)(w + pl.offW) : nullptr;
  // tile counters of the split-K fix-ups: [gt * gr] for R_tau, then [gr], [S * gr], [gn * gr] for A_tau^T C
  const int64_t gt = pl.eta_pad / 64, gr = (R + 63) / 64;
  a.ycnt = (unsigned*)(w + pl.offCnt);
  a.wcnt = a.ycnt + gt * gr + gr + (int64_t)pl.S * gr;
}

// One multi-RHS forward solve on the planned kernel (the persistent one zeroes its counters first).
int32_t launch_multirhs_planned(const rsk_dense* A, int32_t R, const MultiPlan& pl, const rsk::MultiRhsArgs& a,
                                void* workspace, hipStream_t s, float* ckpt, int64_t ckpt_every) {
  if (pl.kernel != 2) {
    if (rsk::launch_zero_words((u64*)((unsigned char*)workspace + pl.offCnt), (pl.cnt_words * sizeof(unsigned) + 7) / 8,
                               s) != hipSuccess)
      return RSK_ERR_HIP;
  }
  if (pl.kernel == 2) {
    const int grid = rsk::multirhs_persistent_grid();
    if (grid < 1) return RSK_ERR_UNSUPPORTED;
    unsigned char* w = (unsigned char*)workspace;
    unsigned* cnt = (unsigned*)(w + pl.offCnt);
    rsk::MrpWork mw;
    mw.gt = pl.eta_pad / 64;
    mw.gr = (R + 63) / 64;
    mw.gn = (int)((A->n + 63) / 64);
    mw.S = pl.pS;
    mw.kspan = pl.pkspan;
    mw.ycnt = cnt;
    mw.ccnt = mw.ycnt + mw.gt * mw.gr;
    mw.xcnt = mw.ccnt + mw.gr;
    mw.wcnt = mw.xcnt + (size_t)pl.S * mw.gr;
    if (rsk::launch_zero_words((u64*)(w + pl.offCnt), (pl.cnt_words * sizeof(unsigned) + 7) / 8, s) != hipSuccess)
      return RSK_ERR_HIP;
    return rsk::launch_multirhs_persistent(a, mw, grid, s, ckpt, ckpt_every) == hipSuccess ? RSK_OK : RSK_ERR_HIP;
  }
  return rsk::launch_multirhs(a, s, ckpt, ckpt_every) == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

// Adjoint workspace: the forward's (Y, C) then Zh, Rh, x, zbar and the partial sums.
struct AdjLayout {
  size_t offZh, offRh, offX, offZbar, offAbar, offLam, bytes;
};

int32_t adj_layout(const rsk_dense* A, int32_t R, const rsk_params* p, int32_t ckpt_every, const MultiPlan& pl,
                   AdjLayout* L) {
  if (ckpt_every < 1) return RSK_ERR_INVALID_ARG;
  if (p->K > 0 && !p->alpha_k) return RSK_ERR_INVALID_ARG;
  if (p->row_w) return RSK_ERR_UNSUPPORTED;  // the reverse pass has no per-row weights
  if (p->eta > rsk::kAdjMaxEtaHost) return RSK_ERR_UNSUPPORTED;
  const size_t nr = (size_t)A->n * R * sizeof(float), er = (size_t)pl.eta_pad * R * sizeof(float);
  const int64_t C = ckpt_every < p->K ? ckpt_every : (p->K > 0 ? p->K : 1);
  size_t o = pl.bytes;
  L->offZh = o; o = align256(o + (size_t)(C + 1) * nr);
  L->offRh = o; o = align256(o + (size_t)C * er);
  L->offX = o; o = align256(o + nr);
  L->offZbar = o; o = align256(o + nr);
  L->offAbar = o; o = align256(o + rsk::adjoint_abar_parts(p->K, pl.eta_pad, R) * sizeof(double));
  L->offLam = o; o = align256(o + rsk::adjoint_lam_parts(A->n, R, p->K) * sizeof(double));
  L->bytes = o;
  return RSK_OK;
}

struct LbLayout {
  int vec, cpt, G;
  size_t lds, bytes, offPart, offR;
  int64_t nstride;
};

template <typename T>
int32_t lb_layout(const rsk_dense* A, LbLayout* L) {
  constexpr int V = rsk::kLbVec<T>;
  L->vec = (((uintptr_t)A->val) % 16 == 0 && A->ld % V == 0) ? V : 1;
  const int planned = rsk::lb_plan<T>(A->n, L->vec, &L->cpt, &L->lds, &L->G, &L->nstride);
  if (planned < 0) return RSK_ERR_HIP;
  if (planned == 0) return RSK_ERR_UNSUPPORTED;
  L->offPart = 0;
  L->offR = align256((size_t)L->G * L->nstride * sizeof(T));
  L->bytes = L->offR + align256((size_t)L->G * sizeof(double));
  return RSK_OK;
}

template <typename T>
rsk::LbArgs<T> lb_args(const rsk_dense* A, const LbLayout& L, void* ws) {
  rsk::LbArgs<T> a{};
  a.A = (const T*)A->val;
  a.m = A->m;
  a.n = A->n;
  a.ld = A->ld;
  a.part = (T*)((char*)ws + L.offPart);
  a.rpart = (double*)((char*)ws + L.offR);
  a.nstride = L.nstride;
  a.G = L.G;
  a.vec = L.vec;
  a.cpt = L.cpt;
  a.lds = L.lds;
  return a;
}

template <typename T>
int32_t lb_solve_t(const rsk_dense* A, const void* b, const rsk_lb_params* p, void* x_star, void* x, void* ws,
                   size_t ws_bytes, hipStream_t s) {
  LbLayout L;
  int32_t st = lb_layout<T>(A, &L);
  if (st) return st;
  if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws) % 256) return RSK_ERR_WORKSPACE;
  rsk::LbArgs<T> a = lb_args<T>(A, L, ws);
  a.b = (const T*)b;
  a.lambda = (T)p->lambda;
  a.step = (T)p->step;
  a.K = p->K;
  a.z = (T*)x_star;
  a.x = (T*)x;
  a.warm = p->warm_start ? 1 : 0;
  a.xref = (const T*)p->x_ref;
  a.check_every = p->check_every;
  a.err_hist = p->err_hist;
  a.res_hist = p->res_hist;
  a.status = p->status_dev;
  if (rsk::launch_zero_status(p->status_dev, s) != hipSuccess) return RSK_ERR_HIP;
  return rsk::launch_lb<T>(a, s) == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t check_bsk(const rsk_dense* A, const rsk_params* p) {
  if (!p || !p->status_dev) return RSK_ERR_INVALID_ARG;
  if (p->eta < 1 || p->K < 0 || p->K >= (int64_t(1) << 31) || p->stream_offset < 0) return RSK_ERR_INVALID_ARG;
  if (!(p->lambda >= 0.0) || !isfinite(p->lambda) || !finite_pos(p->alpha)) return RSK_ERR_INVALID_ARG;
  if (p->K > 0 && !p->index_stream) return RSK_ERR_INVALID_ARG;
  if (p->alpha_k || p->row_w) return RSK_ERR_UNSUPPORTED;
  if (p->eta > rsk::kBskMaxEta || A->m > INT32_MAX) return RSK_ERR_UNSUPPORTED;
  return RSK_OK;
}

// The bsk workspace: per-step relaxations [K], unit row norms [m], then the RSKA solve's own.
struct BskLayout {
  size_t offAlpha, offOnes, offSolve, bytes;
  rsk_params p2;
};

template <typename T>
int32_t bsk_layout(const rsk_dense* A, const rsk_params* p, BskLayout* L) {
  L->offAlpha = 0;
  L->offOnes = align256((size_t)(p->K > 0 ? p->K : 1) * sizeof(T));
  L->offSolve = L->offOnes + align256((size_t)A->m * sizeof(T));
  L->p2 = *p;
  L->p2.alpha = 1.0;
  L->p2.alpha_k = (const void*)1;  // placeholders with the solve's validity; set at launch
  L->p2.rownorm2 = (const void*)1;
  size_t solve_bytes = 0;
  int32_t st = rsk_workspace_size_dense(A, &L->p2, &solve_bytes);
  if (st) return st;
  L->bytes = L->offSolve + solve_bytes;
  return RSK_OK;
}

template <typename T>
int32_t bsk_solve_t(const rsk_dense* A, const void* b, const rsk_params* p, void* x_star, void* x, double* norm2,
                    void* ws, size_t ws_bytes, hipStream_t s) {
  BskLayout L;
  int32_t st = bsk_layout<T>(A, p, &L);
  if (st) return st;
  if (!ws || ws_bytes < L.bytes || ((uintptr_t)ws) % 256) return RSK_ERR_WORKSPACE;
  char* w = (char*)ws;
  rsk::BskArgs<T> a{};
  a.A = (const T*)A->val;
  a.m = A->m;
  a.n = A->n;
  a.ld = A->ld;
  a.tau = p->index_stream ? p->index_stream + p->stream_offset : nullptr;
  a.eta = p->eta;
  a.K = p->K;
  a.w = p->alpha;
  a.alpha_k = (T*)(w + L.offAlpha);
  a.ones = (T*)(w + L.offOnes);
  a.norm2_hist = norm2;
  a.status = p->status_dev;
  if (rsk::launch_zero_status(p->status_dev, s) != hipSuccess) return RSK_ERR_HIP;
  if (rsk::launch_bsk_norms<T>(a, s) != hipSuccess) return RSK_ERR_HIP;
  L.p2.alpha_k = a.alpha_k;
  L.p2.rownorm2 = a.ones;
  // the status stays as the block norms left it: the first error wins
  return solve_dense_t<T>(A, b, &L.p2, x_star, x, w + L.offSolve, ws_bytes - L.offSolve, s, false);
}

// Static exchange scratch of rsk_avg_solve_dense_noalloc: one copy per GPU (each device holds its
// own instance of this array until the process ends). Host code never uses the array's name as a
// device address: the address is looked up once per device with hipGetSymbolAddress.
constexpr size_t kNoAllocScratchBytes = size_t(RSK_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The current device's copy of the scratch array (set up on the first call on that device).
int32_t noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return RSK_ERR_HIP;
  if (dev < 0 || dev >= kMaxDevices) return RSK_ERR_UNSUPPORTED;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return RSK_ERR_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return RSK_OK;
}

}  // namespace

extern "C" {

int32_t rsk_workspace_size_batched(int32_t nsys, int32_t dtype, const rsk_batch_item* items, int64_t wg_bytes,
                                   int32_t kernel, size_t* bytes) {
  if (!bytes) return RSK_ERR_INVALID_ARG;
  BatchLayout L;
  const int32_t st = batch_layout(nsys, dtype, items, wg_bytes, kernel, &L);
  if (st) return st;
  *bytes = L.bytes;
  return RSK_OK;
}

int32_t rsk_plan_batched(int32_t nsys, int32_t dtype, const rsk_batch_item* items, int64_t wg_bytes, int32_t kernel,
                         int32_t* kernel_out, int32_t* groups_out) {
  if (!kernel_out || (nsys > 0 && !groups_out)) return RSK_ERR_INVALID_ARG;
  BatchLayout L;
  const int32_t st = batch_layout(nsys, dtype, items, wg_bytes, kernel, &L, groups_out);
  if (st) return st;
  *kernel_out = L.kind;
  return RSK_OK;
}

int32_t rsk_avg_solve_batched(int32_t nsys, int32_t dtype, const rsk_batch_item* items,
                              const rsk_batch_item* items_dev, const int32_t* order, int64_t wg_bytes,
                              int32_t kernel, void* workspace, size_t ws_bytes, void* stream) {
  BatchLayout L;
  const int32_t st = batch_layout(nsys, dtype, items, wg_bytes, kernel, &L);
  if (st) return st;
  if (nsys == 0) return RSK_OK;
  if (!items_dev) return RSK_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < L.bytes || ((uintptr_t)workspace) % 256) return RSK_ERR_WORKSPACE;
  const int maxg = L.kind == 2 ? rsk::batched_rt_max_resident() : rsk::batched_max_resident(dtype, L.vec, L.lds);
  if (maxg < L.gmax) return RSK_ERR_UNSUPPORTED;
  const int grid = L.tickets < maxg ? (int)L.tickets : maxg;
  unsigned char* w = (unsigned char*)workspace;
  hipStream_t s = (hipStream_t)stream;
  if (rsk::launch_zero_words((u64*)w, L.bytes / sizeof(u64), s) != hipSuccess) return RSK_ERR_HIP;
  int64_t* t0 = (int64_t*)(w + L.off_t0);
  int64_t* wo = (int64_t*)(w + L.off_woff);
  if (rsk::launch_batched_prep(L.kind, items_dev, order, nsys, (int)elem_size(dtype), L.vec, L.tab, L.lds,
                               L.words, t0, wo, s) != hipSuccess)
    return RSK_ERR_HIP;
  const hipError_t e = L.kind == 2
      ? rsk::launch_batched_rt(items_dev, order, nsys, t0, wo, (u64*)w, (u64*)(w + L.off_region), L.tab, grid, s)
      : rsk::launch_batched(items_dev, order, nsys, t0, wo, (u64*)w, (u64*)(w + L.off_region), L.tab, dtype,
                            L.vec, L.lds, grid, s);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_workspace_size_multirhs(const rsk_dense* A, int32_t R, const rsk_params* p, size_t* bytes) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!bytes) return RSK_ERR_INVALID_ARG;
  st = check_params(p, A->m);
  if (st) return st;
  MultiPlan pl;
  st = plan_multirhs(A, R, p, &pl);
  if (st) return st;
  *bytes = pl.bytes;
  return RSK_OK;
}

int32_t rsk_plan_multirhs(const rsk_dense* A, int32_t R, const rsk_params* p, int32_t* out) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!out) return RSK_ERR_INVALID_ARG;
  st = check_params(p, A->m);
  if (st) return st;
  MultiPlan pl;
  st = plan_multirhs(A, R, p, &pl);
  if (st) return st;
  out[0] = pl.kernel == 2 ? pl.pS : pl.S;
  out[1] = (int32_t)(pl.kernel == 2 ? pl.pkspan : pl.kspan);
  out[2] = pl.S2;
  out[3] = pl.eta_pad;
  out[4] = pl.kernel;
  return RSK_OK;
}

int32_t rsk_avg_solve_multirhs(const rsk_dense* A, const void* B, int32_t R, const rsk_params* p, void* X_star,
                               void* X, void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  st = check_params(p, A->m);
  if (st) return st;
  if (!B || !X_star || !X) return RSK_ERR_INVALID_ARG;
  MultiPlan pl;
  st = plan_multirhs(A, R, p, &pl);
  if (st) return st;
  if (!workspace || ws_bytes < pl.bytes || ((uintptr_t)workspace) % 256) return RSK_ERR_WORKSPACE;
  rsk::MultiRhsArgs a;
  fill_multirhs(A, B, R, p, X_star, X, &pl, workspace, &a);
  if (rsk::launch_zero_status(p->status_dev, (hipStream_t)stream) != hipSuccess) return RSK_ERR_HIP;
  return launch_multirhs_planned(A, R, pl, a, workspace, (hipStream_t)stream, nullptr, 1);
}


int32_t rsk_avg_solve_multirhs_ckpt(const rsk_dense* A, const void* B, int32_t R, const rsk_params* p,
                                    int32_t ckpt_every, void* X_star, void* X, void* ckpt, void* workspace,
                                    size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  st = check_params(p, A->m);
  if (st) return st;
  if (!B || !X_star || !X || !ckpt || ckpt_every < 1) return RSK_ERR_INVALID_ARG;
  MultiPlan pl;
  st = plan_multirhs(A, R, p, &pl);
  if (st) return st;
  if (!workspace || ws_bytes < pl.bytes || ((uintptr_t)workspace) % 256) return RSK_ERR_WORKSPACE;
  rsk::MultiRhsArgs a;
  fill_multirhs(A, B, R, p, X_star, X, &pl, workspace, &a);
  if (rsk::launch_zero_status(p->status_dev, (hipStream_t)stream) != hipSuccess) return RSK_ERR_HIP;
  return launch_multirhs_planned(A, R, pl, a, workspace, (hipStream_t)stream, (float*)ckpt, ckpt_every);
}

int32_t rsk_workspace_size_adjoint(const rsk_dense* A, int32_t R, const rsk_params* p, int32_t ckpt_every,
                                   size_t* bytes) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!bytes) return RSK_ERR_INVALID_ARG;
  st = check_params(p, A->m);
  if (st) return st;
  MultiPlan pl;
  st = plan_multirhs(A, R, p, &pl);
  if (st) return st;
  AdjLayout L;
  st = adj_layout(A, R, p, ckpt_every, pl, &L);
  if (st) return st;
  *bytes = L.bytes;
  return RSK_OK;
}

int32_t rsk_avg_adjoint(const rsk_dense* A, const void* B, int32_t R, const rsk_params* p, int32_t ckpt_every,
                        const void* ckpt, const void* X_star_K, const void* Xbar_K, void* Bbar, double* lambda_bar,
                        void* alpha_bar, void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  st = check_params(p, A->m);
  if (st) return st;
  if (!B || !X_star_K || !Xbar_K || !Bbar || !lambda_bar || (p->K > 0 && (!ckpt || !alpha_bar)))
    return RSK_ERR_INVALID_ARG;
  MultiPlan pl;
  st = plan_multirhs(A, R, p, &pl);
  if (st) return st;
  AdjLayout L;
  st = adj_layout(A, R, p, ckpt_every, pl, &L);
  if (st) return st;
  if (!workspace || ws_bytes < L.bytes || ((uintptr_t)workspace) % 256) return RSK_ERR_WORKSPACE;
  unsigned char* w = (unsigned char*)workspace;
  rsk::AdjointArgs d;
  fill_multirhs(A, B, R, p, w + L.offZh, w + L.offX, &pl, workspace, &d.f);
  d.f.warm = 1;
  d.ckpt = (const float*)ckpt;
  d.ckpt_every = ckpt_every;
  d.zK = (const float*)X_star_K;
  d.xbarK = (const float*)Xbar_K;
  d.Bbar = (float*)Bbar;
  d.lambda_bar = lambda_bar;
  d.alpha_bar = (float*)alpha_bar;
  d.Zh = (float*)(w + L.offZh);
  d.Rh = (float*)(w + L.offRh);
  d.zbar = (float*)(w + L.offZbar);
  d.abar_part = (double*)(w + L.offAbar);
  d.lam_part = (double*)(w + L.offLam);
  if (rsk::launch_zero_words((u64*)(w + pl.offCnt), (pl.cnt_words * sizeof(unsigned) + 7) / 8, (hipStream_t)stream) !=
      hipSuccess)
    return RSK_ERR_HIP;
  if (rsk::launch_zero_status(p->status_dev, (hipStream_t)stream) != hipSuccess) return RSK_ERR_HIP;
  if (rsk::launch_adjoint(d, (hipStream_t)stream) != hipSuccess) return RSK_ERR_HIP;
  return RSK_OK;
}

int32_t rsk_rownorm2_csr(const rsk_csr* A, void* rownorm2, void* stream) {
  int32_t st = check_csr(A);
  if (st) return st;
  if (!rownorm2) return RSK_ERR_INVALID_ARG;
  hipError_t e = A->dtype == RSK_F64
      ? rsk::launch_rownorm2_csr<double>(A->row_ptr, (const double*)A->val, A->m, (double*)rownorm2, (hipStream_t)stream)
      : rsk::launch_rownorm2_csr<float>(A->row_ptr, (const float*)A->val, A->m, (float*)rownorm2, (hipStream_t)stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_workspace_size_csr(const rsk_csr* A, const rsk_params* p, size_t* bytes) {
  int32_t st = check_csr(A);
  if (st) return st;
  if (!bytes) return RSK_ERR_INVALID_ARG;
  st = check_params(p, A->m);
  if (st) return st;
  if (p->eta > rsk::kCsrMaxEta) return RSK_ERR_UNSUPPORTED;
  CsrPlan pl;
  st = A->dtype == RSK_F64 ? plan_csr<double>(A, p, &pl) : plan_csr<float>(A, p, &pl);
  if (st) return st;
  *bytes = pl.bytes;
  return RSK_OK;
}

int32_t rsk_avg_solve_csr(const rsk_csr* A, const void* b, const rsk_params* p, void* x_star, void* x,
                          void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_csr(A);
  if (st) return st;
  st = check_params(p, A->m);
  if (st) return st;
  if (!b || !x_star || !x) return RSK_ERR_INVALID_ARG;
  if (p->eta > rsk::kCsrMaxEta) return RSK_ERR_UNSUPPORTED;
  return A->dtype == RSK_F64
      ? solve_csr_t<double>(A, b, p, x_star, x, workspace, ws_bytes, (hipStream_t)stream)
      : solve_csr_t<float>(A, b, p, x_star, x, workspace, ws_bytes, (hipStream_t)stream);
}


int32_t rsk_workspace_size_sampling_cdf(int64_t m, size_t* bytes) {
  if (m <= 0 || !bytes) return RSK_ERR_INVALID_ARG;
  *bytes = rsk::sampling_cdf_ws_bytes(m);
  return RSK_OK;
}

int32_t rsk_sampling_cdf_dense(const rsk_dense* A, double* cdf, void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!cdf) return RSK_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < rsk::sampling_cdf_ws_bytes(A->m) || ((uintptr_t)workspace) % 256)
    return RSK_ERR_WORKSPACE;
  const hipError_t e = A->dtype == RSK_F64
      ? rsk::launch_sampling_cdf<double>((const double*)A->val, A->m, A->n, A->ld, nullptr, cdf, workspace,
                                         (hipStream_t)stream)
      : rsk::launch_sampling_cdf<float>((const float*)A->val, A->m, A->n, A->ld, nullptr, cdf, workspace,
                                        (hipStream_t)stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_sampling_cdf_dense_weighted(const rsk_dense* A, const void* row_w, double* cdf, void* workspace,
                                        size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!cdf || !row_w) return RSK_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < rsk::sampling_cdf_ws_bytes(A->m) || ((uintptr_t)workspace) % 256)
    return RSK_ERR_WORKSPACE;
  const hipError_t e = A->dtype == RSK_F64
      ? rsk::launch_sampling_cdf<double>((const double*)A->val, A->m, A->n, A->ld, (const double*)row_w, cdf,
                                         workspace, (hipStream_t)stream)
      : rsk::launch_sampling_cdf<float>((const float*)A->val, A->m, A->n, A->ld, (const float*)row_w, cdf, workspace,
                                        (hipStream_t)stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_sampling_cdf_weights(const double* weights, int64_t m, double* cdf, void* workspace, size_t ws_bytes,
                                 void* stream) {
  if (!weights || !cdf || m <= 0) return RSK_ERR_INVALID_ARG;
  if (!workspace || ws_bytes < rsk::sampling_cdf_ws_bytes(m) || ((uintptr_t)workspace) % 256) return RSK_ERR_WORKSPACE;
  return rsk::launch_sampling_cdf_weights(weights, m, cdf, workspace, (hipStream_t)stream) == hipSuccess
             ? RSK_OK
             : RSK_ERR_HIP;
}

int32_t rsk_sample_stream(const double* cdf, int64_t m, uint64_t seed, int64_t k0, int64_t K, int32_t eta,
                          int32_t* out, void* stream) {
  if (!cdf || m <= 0 || m > INT32_MAX || k0 < 0 || K < 0 || eta < 1 || (K > 0 && !out)) return RSK_ERR_INVALID_ARG;
  const hipError_t e = rsk::launch_sample_stream(cdf, m, seed, k0, K, eta, out, (hipStream_t)stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_workspace_size_lb_dense(const rsk_dense* A, size_t* bytes) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!bytes) return RSK_ERR_INVALID_ARG;
  LbLayout L;
  st = A->dtype == RSK_F64 ? lb_layout<double>(A, &L) : lb_layout<float>(A, &L);
  if (st) return st;
  *bytes = L.bytes;
  return RSK_OK;
}

int32_t rsk_lb_solve_dense(const rsk_dense* A, const void* b, const rsk_lb_params* p, void* x_star, void* x,
                           void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!p || !b || !x_star || !x || !p->status_dev || p->K < 0 || p->K >= (int64_t(1) << 31)) return RSK_ERR_INVALID_ARG;
  if (!(p->lambda >= 0.0) || !isfinite(p->lambda) || !finite_pos(p->step)) return RSK_ERR_INVALID_ARG;
  if (p->check_every < 0 || (p->x_ref && p->check_every > 0 && !p->err_hist)) return RSK_ERR_INVALID_ARG;
  return A->dtype == RSK_F64 ? lb_solve_t<double>(A, b, p, x_star, x, workspace, ws_bytes, (hipStream_t)stream)
                             : lb_solve_t<float>(A, b, p, x_star, x, workspace, ws_bytes, (hipStream_t)stream);
}

int32_t rsk_spectral_norm2_dense(const rsk_dense* A, int64_t iters, void* v, double* est, void* workspace,
                                 size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (iters < 1 || !v || !est) return RSK_ERR_INVALID_ARG;
  LbLayout L;
  st = A->dtype == RSK_F64 ? lb_layout<double>(A, &L) : lb_layout<float>(A, &L);
  if (st) return st;
  if (!workspace || ws_bytes < L.bytes || ((uintptr_t)workspace) % 256) return RSK_ERR_WORKSPACE;
  hipError_t e;
  if (A->dtype == RSK_F64)
    e = rsk::launch_power<double>(lb_args<double>(A, L, workspace), iters, (double*)v, est, (hipStream_t)stream);
  else
    e = rsk::launch_power<float>(lb_args<float>(A, L, workspace), iters, (float*)v, est, (hipStream_t)stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_workspace_size_bsk_dense(const rsk_dense* A, const rsk_params* p, size_t* bytes) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!bytes) return RSK_ERR_INVALID_ARG;
  st = check_bsk(A, p);
  if (st) return st;
  BskLayout L;
  st = A->dtype == RSK_F64 ? bsk_layout<double>(A, p, &L) : bsk_layout<float>(A, p, &L);
  if (st) return st;
  *bytes = L.bytes;
  return RSK_OK;
}

int32_t rsk_bsk_solve_dense(const rsk_dense* A, const void* b, const rsk_params* p, void* x_star, void* x,
                            double* block_norm2, void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  st = check_bsk(A, p);
  if (st) return st;
  if (!b || !x_star || !x) return RSK_ERR_INVALID_ARG;
  return A->dtype == RSK_F64
      ? bsk_solve_t<double>(A, b, p, x_star, x, block_norm2, workspace, ws_bytes, (hipStream_t)stream)
      : bsk_solve_t<float>(A, b, p, x_star, x, block_norm2, workspace, ws_bytes, (hipStream_t)stream);
}

int32_t rsk_tune_set(const rsk_tune_entry* e) {
  if (!e || e->path < RSK_TUNE_DENSE || e->path > RSK_TUNE_BATCHED) return RSK_ERR_INVALID_ARG;
  if (e->dtype != RSK_F32 && e->dtype != RSK_F64) return RSK_ERR_INVALID_ARG;
  if (e->path == RSK_TUNE_BATCHED && (e->m <= 0 || e->v0 <= 0)) return RSK_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_env_locked();
  tune_put_locked(*e);
  return RSK_OK;
}

int32_t rsk_tune_get(const rsk_tune_entry* key, rsk_tune_entry* out, int32_t* found) {
  if (!key || !out || !found) return RSK_ERR_INVALID_ARG;
  *found = tune_find(key->path, key->dtype, key->m, key->n, key->eta, key->R, out) ? 1 : 0;
  return RSK_OK;
}

int32_t rsk_tune_erase(const rsk_tune_entry* key) {
  if (!key) return RSK_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  tune_env_locked();
  g_tune.erase(std::remove_if(g_tune.begin(), g_tune.end(), [&](const rsk_tune_entry& e) { return tune_same_key(e, *key); }),
               g_tune.end());
  return RSK_OK;
}

int32_t rsk_tune_clear(int32_t path) {
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_env_done = true;  // a cleared table is not refilled from RSK_TUNE_CACHE
  if (path < 0) {
    g_tune.clear();
  } else {
    g_tune.erase(std::remove_if(g_tune.begin(), g_tune.end(), [&](const rsk_tune_entry& e) { return e.path == path; }),
                 g_tune.end());
  }
  return RSK_OK;
}

int32_t rsk_tune_load(const char* path) {
  if (!path) return RSK_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  g_tune_env_done = true;
  return tune_load_locked(path);
}

int32_t rsk_tune_save(const char* path) {
  if (!path) return RSK_ERR_INVALID_ARG;
  std::lock_guard<std::mutex> lock(g_tune_mu);
  FILE* f = fopen(path, "w");
  if (!f) return RSK_ERR_INVALID_ARG;
  fprintf(f, "# librsk tuning cache: path dtype m n eta R v0 v1 v2 us\n");
  for (const rsk_tune_entry& e : g_tune)
    fprintf(f, "%d %d %lld %lld %d %d %lld %lld %lld %.3f\n", e.path, e.dtype, (long long)e.m, (long long)e.n, e.eta,
            e.R, (long long)e.v0, (long long)e.v1, (long long)e.v2, e.us);
  const bool ok = fclose(f) == 0;
  return ok ? RSK_OK : RSK_ERR_INVALID_ARG;
}

int32_t rsk_gather_rate_dense(const rsk_dense* A, const int32_t* index_stream, int32_t eta, int64_t K, int32_t grid,
                              int32_t row_groups, int32_t layout, float* sink, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (A->dtype != RSK_F32 || (A->n % 4) || (A->ld % 4) || (((uintptr_t)A->val) % 16)) return RSK_ERR_UNSUPPORTED;
  if (!sink || (K > 0 && !index_stream) || eta < 1 || eta > 4096 || K < 0) return RSK_ERR_INVALID_ARG;
  if (row_groups != 1 && row_groups != 2 && row_groups != 4 && row_groups != 8) return RSK_ERR_INVALID_ARG;
  if (grid < row_groups || grid > 1024 || grid % row_groups || (layout != 0 && layout != 1)) return RSK_ERR_INVALID_ARG;
  if (layout == 1) {
    // the register tile's lanes: one row group, slices of at most 5 units of 16 floats, eta <= 1024
    const int64_t nunits = (A->n / 4 + 3) / 4;
    if (row_groups != 1 || eta > 1024 || (nunits + grid - 1) / grid > 5) return RSK_ERR_UNSUPPORTED;
  }
  if (K == 0) return RSK_OK;
  return rsk::launch_gather_rate((const float*)A->val, A->m, A->ld, A->n, index_stream, eta, K, grid, row_groups,
                                 layout, sink, (hipStream_t)stream) == hipSuccess
             ? RSK_OK
             : RSK_ERR_HIP;
}

int32_t rsk_abi_version(void) { return RSK_ABI_VERSION; }

const char* rsk_status_string(int32_t s) {
  switch (s) {
    case RSK_OK: return "RSK_OK";
    case RSK_ERR_INVALID_ARG: return "RSK_ERR_INVALID_ARG";
    case RSK_ERR_UNSUPPORTED: return "RSK_ERR_UNSUPPORTED";
    case RSK_ERR_WORKSPACE: return "RSK_ERR_WORKSPACE";
    case RSK_ERR_HIP: return "RSK_ERR_HIP";
    case RSK_ERR_ZERO_ROW: return "RSK_ERR_ZERO_ROW";
    case RSK_ERR_INDEX_RANGE: return "RSK_ERR_INDEX_RANGE";
    case RSK_ERR_NONFINITE: return "RSK_ERR_NONFINITE";
    case RSK_ERR_ABORTED: return "RSK_ERR_ABORTED";
    default: return "RSK_ERR_UNKNOWN";
  }
}

int32_t rsk_rownorm2_dense(const rsk_dense* A, void* rownorm2, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!rownorm2) return RSK_ERR_INVALID_ARG;
  hipError_t e = A->dtype == RSK_F64
      ? rsk::launch_rownorm2_dense<double>((const double*)A->val, A->m, A->n, A->ld, (double*)rownorm2, (hipStream_t)stream)
      : rsk::launch_rownorm2_dense<float>((const float*)A->val, A->m, A->n, A->ld, (float*)rownorm2, (hipStream_t)stream);
  return e == hipSuccess ? RSK_OK : RSK_ERR_HIP;
}

int32_t rsk_workspace_size_dense(const rsk_dense* A, const rsk_params* p, size_t* bytes) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!bytes) return RSK_ERR_INVALID_ARG;
  st = check_params(p, A->m);
  if (st) return st;
  if (p->eta > kMaxEtaDense) return RSK_ERR_UNSUPPORTED;
  DensePlan pl;
  st = A->dtype == RSK_F64 ? plan_dense<double>(A, p, &pl) : plan_dense<float>(A, p, &pl);
  if (st) return st;
  *bytes = pl.bytes;
  return RSK_OK;
}

int32_t rsk_avg_solve_dense_noalloc(const rsk_dense* A, const void* b, const rsk_params* p, void* x_star, void* x,
                                    void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  st = check_params(p, A->m);
  if (st) return st;
  if (!b || !x_star || !x) return RSK_ERR_INVALID_ARG;
  if (p->eta > kMaxEtaDense) return RSK_ERR_UNSUPPORTED;
  DensePlan pl;
  st = A->dtype == RSK_F64 ? plan_dense<double>(A, p, &pl) : plan_dense<float>(A, p, &pl);
  if (st) return st;
  if (pl.bytes > kNoAllocScratchBytes) return RSK_ERR_WORKSPACE;
  void* ws = nullptr;
  st = noalloc_scratch(&ws);
  if (st) return st;
  return A->dtype == RSK_F64
      ? solve_dense_t<double>(A, b, p, x_star, x, ws, kNoAllocScratchBytes, (hipStream_t)stream)
      : solve_dense_t<float>(A, b, p, x_star, x, ws, kNoAllocScratchBytes, (hipStream_t)stream);
}

int32_t rsk_plan_dense(const rsk_dense* A, const rsk_params* p, int32_t* out) {
  int32_t st = check_dense(A);
  if (st) return st;
  if (!out) return RSK_ERR_INVALID_ARG;
  st = check_params(p, A->m);
  if (st) return st;
  if (p->eta > kMaxEtaDense) return RSK_ERR_UNSUPPORTED;
  DensePlan pl;
  st = A->dtype == RSK_F64 ? plan_dense<double>(A, p, &pl) : plan_dense<float>(A, p, &pl);
  if (st) return st;
  const bool rt = pl.kernel == 2;
  out[0] = rt ? (pl.rg > 1 ? 3 : 2) : pl.kernel;
  out[1] = pl.G;
  out[2] = rt ? pl.nt : rsk::kDenseThreads;
  out[3] = rt ? pl.rp : 0;
  out[4] = rt || pl.kernel == 4 ? pl.cpl : 0;
  out[5] = pl.rg;
  out[6] = pl.two_hop ? 2 : 1;
  out[7] = pl.vec;
  out[8] = rt ? 0 : pl.tile_cache;
  return RSK_OK;
}

int32_t rsk_avg_solve_dense(const rsk_dense* A, const void* b, const rsk_params* p, void* x_star, void* x,
                            void* workspace, size_t ws_bytes, void* stream) {
  int32_t st = check_dense(A);
  if (st) return st;
  st = check_params(p, A->m);
  if (st) return st;
  if (!b || !x_star || !x) return RSK_ERR_INVALID_ARG;
  if (p->eta > kMaxEtaDense) return RSK_ERR_UNSUPPORTED;
  return A->dtype == RSK_F64
      ? solve_dense_t<double>(A, b, p, x_star, x, workspace, ws_bytes, (hipStream_t)stream)
      : solve_dense_t<float>(A, b, p, x_star, x, workspace, ws_bytes, (hipStream_t)stream);
}

}  // extern "C"
