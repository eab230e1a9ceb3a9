// Argument blocks and launch entry points of the RSKA kernels (host + device).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsk.h"

namespace rsk {

typedef unsigned long long u64;

// One dense persistent solve (eq. (rska) / Algorithm 1) over K steps.
template <typename T>
struct DenseArgs {
  const T* A;
  int64_t m, n, ld;
  const T* b;
  const T* r2;            // ||a_i||^2
  const T* row_w = nullptr;  // nullable per-row weights w_i (row i relaxed by alpha w_i)
  T lambda, alpha;
  const T* alpha_k;       // nullable, per-step relaxation
  int eta;
  int64_t K;
  const int32_t* idx;     // stream, already advanced by stream_offset
  T* x_star;              // in/out
  T* x;                   // out
  int warm;
  T* y;                   // nullable dual, y[tau_t] -= c_t
  const T* xref;          // nullable monitor target
  int64_t check_every;
  double tol;
  double* err_hist;
  int* status;            // [0] status, [1] steps done
  u64* xP;                // partial dots  [2][G][eta][words] (step parity)
  u64* xC;                // coefficients  [eta][words]
  u64* xM;                // monitor sums  [G][2][2]
  u64* xU = nullptr;      // register-tile kernel with RG > 1 row groups: update parts [2][G][slice floats]
  int G;
  int two_hop;            // 1: owners reduce rows, then everyone gathers; 0: everyone reduces everything
  int tile_cache;         // 1: keep the step's row tile in LDS between dot and scatter;
                          // 2: two LDS tiles, the next step's rows loaded (into registers)
                          // while the step runs on the other (see dense_pipe_ok)
                          // (two_hop == 0 requires G*eta*words <= kOneHopWords)
  int64_t nchunks;        // ceil(n / VEC)
  int wq_max;             // max chunks per workgroup slice
  int lpr;                // lanes per row in the dot phase (power of two <= 64)
};

constexpr int kDenseThreads = 256;

// The pipelined tile (tile_cache == 2) loads the next step's rows into
// registers during the step (at most pipe_reg_chunks 16-byte chunks a thread:
// 8 for float, 4 for double, whose other values take twice the registers) and
// keeps the next step's b and ||a||^2 in registers (at most 4 rows a thread):
// it needs whole 16-byte vectors, eta <= 4 * kDenseThreads and a tile of at
// most pipe_reg_chunks * kDenseThreads chunks.
__host__ __device__ constexpr int pipe_reg_chunks(size_t esize) { return esize == 8 ? 4 : 8; }
__host__ __device__ inline bool dense_pipe_ok(size_t esize, int vec, int eta, int wq) {
  return esize * (size_t)vec == 16 && eta >= 1 && eta <= 4 * kDenseThreads && wq >= 1 &&
         (int64_t)eta * wq <= (int64_t)pipe_reg_chunks(esize) * kDenseThreads;
}

// LDS layout of one workgroup of the general dense kernel (byte offsets):
// own slices of x* and x, the step's coefficients, the rows' indices (three
// buffers: the pipelined tile fetches them two steps ahead), b and ||a||^2 (two
// buffers: the next step's are prefetched during the current one), the
// update's row-group partials, monitor scratch and, optionally, the step's row
// tile (two tiles when pipelined); with the one-hop exchange also the G*eta
// partials of the step.
struct DenseSmem {
  size_t xs, xv, cs, tau, bq, rq, red, xr, flags, tile, total;
  __host__ __device__ static size_t al16(size_t v) { return (v + 15) & ~size_t(15); }

  __host__ __device__ DenseSmem(size_t esize, int vec, int wq_max, int eta, int nt, int tile_cache, int64_t xr_elems) {
    size_t o = 0;
    xs = o; o += al16(esize * (size_t)wq_max * vec);
    xv = o; o += al16(esize * (size_t)wq_max * vec);
    cs = o; o += al16(esize * (size_t)eta);
    tau = o; o += al16(sizeof(int) * 3 * (size_t)eta);
    bq = o; o += al16(esize * 2 * (size_t)eta);
    rq = o; o += al16(esize * 2 * (size_t)eta);
    red = o; o += al16(esize * (size_t)nt * vec);
    xr = o; o += al16(esize * (size_t)xr_elems);
    flags = o; o += 128;
    tile = o;
    if (tile_cache == 2) o += 2 * al16(esize * (size_t)eta * wq_max * vec);
    else if (tile_cache) o += al16(esize * (size_t)eta * wq_max * vec);
    total = o;
  }
};

// LDS values of the one-hop gather: the G*eta partials and the per-row sums
// of their segments of kOneHopSeg workgroups.
constexpr int kOneHopSeg = 16;
__host__ __device__ inline int64_t onehop_lds_elems(int64_t G, int64_t eta) {
  return G * eta + (G + kOneHopSeg - 1) / kOneHopSeg * eta;
}

// Exchange words per step (G*eta*words per value) at or below which every
// workgroup gathers all partials (one flat poll of at most 16 words per
// thread of a 256-thread workgroup, then per-row sums in LDS).
constexpr int64_t kOneHopWords = 4096;

// The register-tile kernel gathers all C*eta partials in one hop only up to this many words per
// step: above it the flat poll costs more than the two-hop exchange (measured on 8000- and
// 20000-column slices over 256 workgroups).
constexpr int64_t kRtOneHopWords = 2048;

// One CSR persistent solve (single workgroup).
constexpr int kCsrMaxEta = 4096;  // rows per step of the CSR kernel
template <typename T>
struct CsrArgs {
  const int64_t* row_ptr;
  const int32_t* col;
  const T* val;
  int64_t m, n;
  const T* b;
  const T* r2;
  const T* row_w = nullptr;  // nullable per-row weights
  T lambda, alpha;
  const T* alpha_k;
  int eta;
  int64_t K;
  const int32_t* idx;
  T* x_star;
  T* x;
  int warm;
  T* y;
  const T* xref;
  int64_t check_every;
  double tol;
  double* err_hist;
  int* status;
  long long* acc;         // n + 1 int64 accumulators (the last a spare), zero on entry and on exit
  int* ycnt;              // [m] slots of the current step per row (y only; zero on entry and between steps)
  T* cy;                  // [eta] the step's coefficients by slot (grid kernel, y only)
  // grid kernel only
  int G;                  // workgroups
  u64* bar;               // grid barrier counter (zero on entry)
  int* emax;              // [2] biased max exponent of a step's contributions (zero on entry)
  u64* xM;                // monitor words [G][4]
};

template <typename T>
hipError_t launch_csr(CsrArgs<T>& a, hipStream_t stream);
// Multi-workgroup CSR kernel (one lane per nonzero, three grid barriers per step).
constexpr int kCsrGridRowsPerPass = 8;   // rows per workgroup and pass (256 threads, 32 lanes a row)
constexpr int kCsrGridMaxPasses = 8;
template <typename T>
int csr_grid_max_resident();
template <typename T>
hipError_t launch_csr_grid(CsrArgs<T>& a, hipStream_t stream);

// Multi-RHS (shared A and stream), float32 MFMA GEMMs per step.
struct MultiRhsArgs {
  const float* A;
  int64_t m, n, ld;
  const float* B;         // m x R row-major
  int R;
  const float* r2;
  const float* row_w = nullptr;  // nullable per-row weights
  float lambda, alpha;
  const float* alpha_k;   // nullable, device
  int eta;
  int64_t K;
  const int32_t* idx;
  float* x_star;          // n x R row-major, in/out
  float* x;               // n x R row-major, out
  int warm;
  int* status;
  float* Y;               // S x eta_pad x R split-K partials
  float* C;               // eta_pad x R coefficients
  int S, eta_pad;
  int64_t kspan;
  int S2 = 1;             // row splits of the A_tau^T products (small n x R outputs)
  float* Wp = nullptr;    // S2 x n x R partials of A_tau^T C when S2 > 1
  unsigned* ycnt = nullptr;  // per 64 x 64 tile of R_tau: split partials counted (zero before a solve)
  unsigned* wcnt = nullptr;  // per 64 x 64 tile of A_tau^T C: row-split partials counted (zero before a solve)
  int tile = 64;          // product tile edge of the step kernels: 64, or 128 (eta_pad a multiple of 128)
};
// ckpt (nullable): x*_k is copied to ckpt[k / ckpt_every] before every step k with k % ckpt_every == 0.
hipError_t launch_multirhs(const MultiRhsArgs& a, hipStream_t stream, float* ckpt = nullptr, int64_t ckpt_every = 1);

// Persistent multi-RHS forward (one cooperative launch for all K steps): its own split of the n
// columns (kspan a multiple of 64, S = ceil(n / kspan)) and the tile counters, zeroed before the
// launch: ycnt [gt * gr], ccnt [gr], xcnt [S * gr], wcnt [gn * gr].
struct MrpWork {
  int gt, gr, gn, S;
  int64_t kspan;
  unsigned *ycnt, *ccnt, *xcnt, *wcnt;
};
int multirhs_persistent_grid();
hipError_t launch_multirhs_persistent(const MultiRhsArgs& a, const MrpWork& w, int grid, hipStream_t stream,
                                      float* ckpt = nullptr, int64_t ckpt_every = 1);

// Reverse mode of K multi-RHS steps. f holds the forward's arguments (alpha_k required);
// workspace pieces: Zh (ckpt_every+1) n x R, Rh ckpt_every eta_pad x R, zbar n x R, partial sums.
struct AdjointArgs {
  MultiRhsArgs f;
  const float* ckpt;      // ceil(K / ckpt_every) x n x R, x* at steps 0, C, 2C, ...
  int64_t ckpt_every;
  const float* zK;        // x*_K of the forward
  const float* xbarK;     // dL/dx_K, n x R
  float* Bbar;            // m x R, out
  double* lambda_bar;     // 1, out
  float* alpha_bar;       // K, out
  float* Zh;
  float* Rh;
  float* zbar;
  double* abar_part;
  double* lam_part;
};
constexpr int kAdjMaxEtaHost = 4096;
size_t adjoint_lam_parts(int64_t n, int R, int64_t K);
size_t adjoint_abar_parts(int64_t K, int eta_pad, int R);
hipError_t launch_adjoint(const AdjointArgs& d, hipStream_t stream);

// Batched independent systems. System s is solved by G_s workgroups running
// the dense kernel's per-workgroup code on its own workspace region. The plan
// of a system depends only on (n, eta, element size, vector width, target
// bytes per workgroup) and is computed by the same function on the host
// (workspace and LDS sizing) and on the device (tickets and offsets).
constexpr int kBatchGcap = 256;                 // most workgroups one system may use
constexpr size_t kBatchLdsCap = 80 * 1024;      // LDS of one workgroup: two fit a CU
constexpr int64_t kBatchWgBytes = 56 * 1024;    // default row bytes per workgroup per step (swept: 16-96 KiB)
constexpr int64_t kBatchRegionHead = 32;        // words: join counter + padding

struct BatchPlan {
  int G, two_hop, tile_cache, lpr, wq_max;
  int cpl;  // register-tile launch: float4 chunks a lane (units of 16 floats of the widest slice)
  int64_t nchunks, words;
  size_t lds;
};

// Row bytes per workgroup by size class of a system's step (eta * n * element bytes): system s
// takes the first class with step bytes <= hi[c] (classes ascend), else the default. Either one
// class of every size (an explicit target) or the tuned classes of the library's tuning table.
constexpr int kBatchClasses = 8;
struct BatchWgTable {
  int nc;
  int64_t hi[kBatchClasses];
  int64_t wg[kBatchClasses];
  __host__ __device__ int64_t lookup(int64_t step_bytes, int64_t dflt = kBatchWgBytes) const {
    for (int c = 0; c < nc; ++c)
      if (step_bytes <= hi[c]) return wg[c];
    return dflt;
  }
};

__host__ __device__ inline bool batched_plan(int64_t n, int eta, int esize, int vec, const BatchWgTable& tab,
                                             BatchPlan* p) {
  if (n <= 0 || eta <= 0 || vec <= 0) return false;
  const int64_t wg_bytes = tab.lookup((int64_t)eta * n * esize);
  if (wg_bytes <= 0) return false;
  const int64_t nchunks = (n + vec - 1) / vec;
  const int64_t gmax = nchunks < kBatchGcap ? nchunks : kBatchGcap;
  int64_t G = ((int64_t)eta * n * esize + wg_bytes - 1) / wg_bytes;
  if (G < 1) G = 1;
  if (G > gmax) G = gmax;
  for (;;) {
    const int wq = (int)((nchunks + G - 1) / G);
    const int64_t xr = G * eta * (esize / 4) > kOneHopWords ? 0 : onehop_lds_elems(G, eta);
    const DenseSmem piped(esize, vec, wq, eta, kDenseThreads, 2, xr);
    const DenseSmem with_tile(esize, vec, wq, eta, kDenseThreads, 1, xr);
    const DenseSmem no_tile(esize, vec, wq, eta, kDenseThreads, 0, xr);
    if (dense_pipe_ok(esize, vec, eta, wq) && piped.total <= kBatchLdsCap) {
      p->tile_cache = 2;
      p->lds = piped.total;
      p->wq_max = wq;
      break;
    }
    if (with_tile.total <= kBatchLdsCap || no_tile.total <= kBatchLdsCap) {
      p->tile_cache = with_tile.total <= kBatchLdsCap;
      p->lds = p->tile_cache ? with_tile.total : no_tile.total;
      p->wq_max = wq;
      break;
    }
    if (G >= gmax) return false;
    G = 2 * G < gmax ? 2 * G : gmax;
  }
  int lpr = 1;
  while (lpr < p->wq_max && lpr < 64) lpr <<= 1;
  const int W = esize / 4;
  p->G = (int)G;
  p->lpr = lpr;
  p->cpl = 0;
  p->nchunks = nchunks;
  p->two_hop = G * eta * W > kOneHopWords;
  const int64_t body = 2 * G * eta * W + (int64_t)eta * W + 4 * G;
  p->words = kBatchRegionHead + (body + 31) / 32 * 32;
  return true;
}

// kind 1: general kernel plans (batched_plan); kind 2: register-tile plans (batched_rt_plan)
hipError_t launch_batched_prep(int kind, const rsk_batch_item* items, const int32_t* order, int nsys, int esize, int vec,
                               const BatchWgTable& tab, size_t lds_launch, int64_t cap_words, int64_t* ticket0,
                               int64_t* woff, hipStream_t stream);
// Largest co-resident grid of the batched kernel with this LDS size (0 if none).
int batched_max_resident(int dtype, int vec, size_t lds);
hipError_t launch_batched(const rsk_batch_item* items, const int32_t* order, int nsys, const int64_t* ticket0,
                          const int64_t* woff, u64* queue, u64* regions, const BatchWgTable& tab, int dtype, int vec,
                          size_t lds, int grid, hipStream_t stream);

struct DenseLaunch {
  int threads;
  size_t lds_bytes;
  int vec;
};

// Plans and launches; returns a hipError_t.
template <typename T>
hipError_t launch_dense(DenseArgs<T>& a, int vec, hipStream_t stream, int* max_grid_out);

template <typename T>
hipError_t launch_rownorm2_dense(const T* A, int64_t m, int64_t n, int64_t ld, T* r2, hipStream_t stream);

template <typename T>
hipError_t launch_rownorm2_csr(const int64_t* row_ptr, const T* val, int64_t m, T* r2, hipStream_t stream);

hipError_t launch_zero_words(u64* p, size_t nwords, hipStream_t stream);

// One-workgroup dense kernel with the step in registers (rsk_dense_small.hip): columns a thread
// (1, 2, 4 or 8) for n columns and eta rows a step, 0 where it does not apply.
int dense_small_cpt(int64_t n, int eta);
template <typename T>
hipError_t launch_dense_small(DenseArgs<T>& a, hipStream_t stream);

// Launch of a persistent kernel whose workgroups wait for one another. Cooperative by default:
// the runtime guarantees that all of them are resident at once. With the environment variable
// RSK_COOPERATIVE=0 (read once per process) the same grid goes out as a plain launch: the callers
// have already checked that it fits the device's resident capacity, so on an otherwise idle GPU
// every workgroup is resident all the same, and the bounded waits turn anything else into
// RSK_ERR_ABORTED. It exists for tools that do not follow a process with a cooperative launch
// to a clean end (under the profiler of this ROCm release such processes have ended with a
// segmentation fault in their exit path, after the profiler had written its results), and for
// several processes on one GPU (a cooperative launch has failed in one process while another
// process that had made cooperative launches was alive).
hipError_t launch_persistent(const void* fn, dim3 grid, dim3 block, void** args, unsigned lds, hipStream_t stream);

// float32 register-tile kernel: NT threads, RP row passes of NT/(4 RG) rows, CPL float4 chunks
// per lane, RG row groups (1 or 2) of G/RG column slices
int dense_rt_max_grid(int nt, int rp, int cpl, int rg);
hipError_t launch_dense_rt(DenseArgs<float>& a, int nt, int rp, int cpl, int rg, hipStream_t stream);
// kRtOwnMax: rows of a step one wave of the register-tile kernel reduces
constexpr int kRtMaxEta = 1024, kRtMaxCPL = 5, kRtOwnMax = 4;

// Batched launch on the register tile (float32): kBrtThreads threads a workgroup, one per CU,
// kBrtPasses row passes of kBrtThreads / 4 rows (eta <= 512) and at most kBrtCpl float4 chunks a
// lane, i.e. column slices of up to 16 * kBrtCpl floats (640-byte pieces of each sampled row).
constexpr int kBrtThreads = 512, kBrtPasses = 4, kBrtCpl = 10;
// LDS of the next-step prefetch (one workgroup a CU)
constexpr int kBrtPfBytes = 147456;
constexpr int kBrtMaxEta = kBrtPasses * (kBrtThreads / 4);
// default row bytes per workgroup per step of the register-tile launch (a tuned class overrides it)
constexpr int64_t kBrtWgBytes = 256 * 1024;

// Plan of one system on the batched register tile (the same function on host and device):
// G_s from the row bytes per workgroup of the system's size class, at least enough slices for
// kBrtCpl chunks a lane and, with two exchange hops, for kRtOwnMax rows per wave; the
// exchange region has the layout of the general batched kernel (4-byte words); at most one
// workgroup per 16-float unit of a row. False if the system does not fit (eta > kBrtMaxEta, or
// more workgroups needed than it has units or than kBatchGcap).
__host__ __device__ inline bool batched_rt_plan(int64_t n, int eta, const BatchWgTable& tab, BatchPlan* p) {
  if (n <= 0 || eta <= 0 || eta > kBrtMaxEta) return false;
  const int64_t wg_bytes = tab.lookup((int64_t)eta * n * 4, kBrtWgBytes);
  if (wg_bytes <= 0) return false;
  const int64_t nchunks = (n + 3) / 4, nunits = (nchunks + 3) / 4;
  const int64_t gmax = nunits < kBatchGcap ? nunits : kBatchGcap;
  int64_t G = ((int64_t)eta * n * 4 + wg_bytes - 1) / wg_bytes;
  if (G > gmax) G = gmax;  // a small target: one 16-float unit a slice
  const int64_t gcpl = (nunits + kBrtCpl - 1) / kBrtCpl;
  if (G < gcpl) G = gcpl;
  if (G < 1) G = 1;
  const int own = kRtOwnMax * (kBrtThreads / 64);
  if (G * eta > kRtOneHopWords || eta > own) {
    const int64_t gown = (eta + own - 1) / own;
    if (G < gown) G = gown;
  }
  if (G > gmax) return false;
  p->G = (int)G;
  p->two_hop = (G * eta > kRtOneHopWords || eta > own) ? 1 : 0;
  p->tile_cache = 0;
  p->lds = 0;
  p->nchunks = nchunks;
  p->cpl = (int)((nunits + G - 1) / G);
  p->wq_max = 4 * p->cpl;
  p->lpr = 4;
  const int64_t body = 2 * G * eta + (int64_t)eta + 4 * G;
  p->words = kBatchRegionHead + (body + 31) / 32 * 32;
  return true;
}
// Largest co-resident grid of the batched register-tile kernel (0 if none).
int batched_rt_max_resident();
hipError_t launch_batched_rt(const rsk_batch_item* items, const int32_t* order, int nsys, const int64_t* ticket0,
                             const int64_t* woff, u64* queue, u64* regions, const BatchWgTable& tab, int grid,
                             hipStream_t stream);
hipError_t launch_zero_status(int* status, hipStream_t stream);
// the gather of the register-tile solve alone (rsk_gather_rate_dense); sink: G * 512 floats
hipError_t launch_gather_rate(const float* A, int64_t m, int64_t ld, int64_t n, const int32_t* idx, int eta, int64_t K,
                              int G, int rg, int layout, float* sink, hipStream_t stream);

// Linearized Bregman (full batch) and power iteration on A^T A. One pass reads A once with
// kLbThreads threads a workgroup, chunks of vec elements (16 bytes, or 1 element when A is not
// 16-byte aligned or ld not a multiple of kLbVec), at most 12 chunks a thread: n <= 6144 vec.
constexpr int kLbThreads = 512;
template <typename T>
constexpr int kLbVec = 16 / (int)sizeof(T);
constexpr int kLbMaxChunksPerThread = 12;
template <typename T>
struct LbArgs {
  const T* A;
  int64_t m, n, ld;
  const T* b;
  T lambda, step;
  int64_t K;
  T* z;                   // x*: in when warm, out
  T* x;                   // out (in when warm: S_lambda(z))
  int warm;
  const T* xref;
  int64_t check_every;
  double* err_hist;
  double* res_hist;       // ||A x_k - b|| before step k (nullable)
  int* status;
  T* part;                // [G][nstride] per-workgroup partial A^T r
  double* rpart;          // [G] per-workgroup sum of r_i^2
  int64_t nstride;        // nchunks * vec
  int G, vec, cpt;
  size_t lds;
};
template <typename T>
int lb_plan(int64_t n, int vec, int* cpt, size_t* lds, int* grid, int64_t* nstride);
template <typename T>
hipError_t launch_lb(const LbArgs<T>& a, hipStream_t stream);
template <typename T>
hipError_t launch_power(const LbArgs<T>& a, int64_t iters, T* v, double* est, hipStream_t stream);

// Block sparse Kaczmarz, eq. (bsk): per-step block norms (eta <= kBskMaxEta) computed up front,
// written as the relaxations alpha_k = eta w / ||A_tau_k||_2^2 of an RSKA solve with unit row norms.
constexpr int kBskMaxEta = 64;
constexpr int kBskThreads = 256;
template <typename T>
struct BskArgs {
  const T* A;
  int64_t m, n, ld;
  const int* tau;         // index stream at the first step (K * eta entries)
  int eta;
  int64_t K;
  double w;               // relaxation of eq. (bsk)
  T* alpha_k;             // out: K relaxations
  T* ones;                // out: m unit row norms
  double* norm2_hist;     // nullable, K entries: ||A_tau_k||_2^2
  int* status;
};
template <typename T>
hipError_t launch_bsk_norms(const BskArgs<T>& a, hipStream_t stream);

// Row sampler (Philox4x32-10 + inverse CDF) and the FP64 cdf of the row norms.
size_t sampling_cdf_ws_bytes(int64_t m);
template <typename T>
hipError_t launch_sampling_cdf(const T* A, int64_t m, int64_t n, int64_t ld, const T* row_w, double* cdf, void* ws,
                               hipStream_t stream);
hipError_t launch_sampling_cdf_weights(const double* w, int64_t m, double* cdf, void* ws, hipStream_t stream);
hipError_t launch_sample_stream(const double* cdf, int64_t m, uint64_t seed, int64_t k0, int64_t K, int eta,
                                int32_t* out, hipStream_t stream);

// Largest co-resident grid for the dense kernel with these sizes (0 if none).
template <typename T>
int dense_max_grid(int vec, int eta, int wq_max, int tile_cache, int64_t xr_elems, size_t* lds_bytes);

}  // namespace rsk
