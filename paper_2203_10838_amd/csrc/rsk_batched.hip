// Batched RSKA: many independent dense systems of uneven shape in one launch.
//
// System s is solved by a group of G_s workgroups that split its columns the
// way the single-system dense kernel does, with the same device code
// (dense_run), exchanging partial dots through the system's own region of the
// workspace. G_s follows the system's row bytes per step (a target of row
// bytes per workgroup, per size class of the step: one explicit target, or the
// tuned classes of the library's tuning table), so a large system gets many
// CUs and a small one a single workgroup (whose exchange then stays in LDS).
//
// A float32 batch whose systems all fit the register tile (rows 16-byte aligned, eta <= 512)
// can instead run on rska_batched_rt: one 512-thread workgroup per CU, each system on G_s of
// them with the single-system register-tile step (rt_run), column slices of up to 160 floats
// held in VGPRs through the step, the next step's rows partly prefetched into LDS during the
// exchange. Same tickets, join and exchange regions as the general launch.
//
// Scheduling. The systems, in the caller's order, own consecutive ranges of
// G_s tickets. Persistent workgroups draw tickets from one atomic counter;
// ticket q in the range of system s makes its drawer rank q - start_s of that
// system's group. A workgroup runs its system to the end before it draws
// again, so all groups before the one holding the counter are complete and
// finish, which frees workgroups for the incomplete one: a group waits only
// until enough workgroups are free (it never waits on a later group). Each
// group still joins on a counter before its first step, with the wait
// bounded in wall-clock time.
#include "rsk_dense_run.hpp"
#include "rsk_dense_rt.hpp"

namespace rsk {

namespace {

constexpr int kPrepThreads = 1024;

__device__ bool item_ok(const rsk_batch_item& it) {
  if (!it.A || !it.b || !it.rownorm2 || !it.x_star || !it.x || !it.status_dev) return false;
  if (it.m <= 0 || it.m > INT32_MAX || it.n <= 0 || it.ld < it.n || it.eta < 1 || it.K < 0) return false;
  if (it.K > 0 && !it.index_stream) return false;
  return true;
}

// the plan of one system for the launch kind (1 general, 2 register tile), as the host made it
__device__ bool item_plan(int kind, const rsk_batch_item& it, int esize, int vec, const BatchWgTable& tab,
                          size_t lds_launch, BatchPlan* pl) {
  if (!item_ok(it)) return false;
  if (kind == 2)
    return esize == 4 && (it.ld % 4) == 0 && ((uintptr_t)it.A) % 16 == 0 && batched_rt_plan(it.n, it.eta, tab, pl);
  return batched_plan(it.n, it.eta, esize, vec, tab, pl) && pl->lds <= lds_launch;
}

// The next ticket t of the launch and the position p of the system whose range holds it (every
// thread gets both); false once the tickets are gone.
__device__ bool take_ticket(const int64_t* __restrict__ ticket0, int nsys, u64* queue, int64_t* sh, int64_t* t_out,
                            int* p_out) {
  const int64_t total = ticket0[nsys];
  if (threadIdx.x == 0) {
    const int64_t t = (int64_t)__hip_atomic_fetch_add(queue, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // last position p with ticket0[p] <= t
    int lo = 0, hi = nsys - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ticket0[mid] <= t) lo = mid;
      else hi = mid - 1;
    }
    sh[0] = t;
    sh[1] = lo;
  }
  __syncthreads();
  *t_out = sh[0];
  *p_out = (int)sh[1];
  __syncthreads();
  return *t_out < total;
}

// Join: wait until all G ranks of the system hold a workgroup, the wait bounded by join_ticks of
// the wall clock (expired: the system reports RSK_ERR_ABORTED and this workgroup skips it).
__device__ bool join_group(u64* region, int G, int* status_dev, uint64_t join_ticks, int64_t* sh) {
  if (threadIdx.x == 0) {
    __hip_atomic_fetch_add(region, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint64_t t0 = wall_clock64();
    int ok = 1;
    while (xload(region) < (u64)G) {
      if (wall_clock64() - t0 > join_ticks) { ok = 0; break; }
      __builtin_amdgcn_s_sleep(2);
    }
    if (!ok) set_status(status_dev, ST_ABORTED);
    sh[2] = ok;
  }
  __syncthreads();
  const bool joined = sh[2] != 0;
  __syncthreads();
  return joined;
}

template <typename T>
__device__ void fill_args(DenseArgs<T>& a, const rsk_batch_item& it, const BatchPlan& pl, u64* region) {
  a.A = (const T*)it.A; a.m = it.m; a.n = it.n; a.ld = it.ld;
  a.b = (const T*)it.b; a.r2 = (const T*)it.rownorm2; a.row_w = nullptr;
  a.lambda = (T)it.lambda; a.alpha = (T)it.alpha; a.alpha_k = nullptr;
  a.eta = it.eta; a.K = it.K; a.idx = it.index_stream;
  a.x_star = (T*)it.x_star; a.x = (T*)it.x; a.warm = it.warm_start ? 1 : 0; a.y = nullptr;
  a.xref = (const T*)it.x_ref; a.check_every = it.x_ref ? it.check_every : 0; a.tol = it.tol;
  a.err_hist = it.err_hist; a.status = it.status_dev;
  a.xP = region + kBatchRegionHead;
  a.xC = a.xP + (size_t)2 * pl.G * it.eta * Words<T>::N;
  a.xM = a.xC + (size_t)it.eta * Words<T>::N;
  a.xU = nullptr;
  a.G = pl.G; a.two_hop = pl.two_hop; a.tile_cache = pl.tile_cache;
  a.nchunks = pl.nchunks; a.wq_max = pl.wq_max; a.lpr = pl.lpr;
}

}  // namespace

// One workgroup: per-system plans in the caller's order, exclusive prefix
// sums of tickets and region words, status words reset. A system whose
// descriptor or plan does not fit the launch gets no tickets and
// RSK_ERR_INVALID_ARG; if the regions overflow the workspace no system runs
// and every system reports RSK_ERR_WORKSPACE.
__global__ __launch_bounds__(kPrepThreads) void batched_prep(int kind, const rsk_batch_item* __restrict__ items,
                                                             const int32_t* __restrict__ order, int nsys, int esize,
                                                             int vec, BatchWgTable tab, size_t lds_launch,
                                                             int64_t cap_words, int64_t* ticket0, int64_t* woff) {
  __shared__ int64_t sg[kPrepThreads], sw[kPrepThreads];
  const int tid = threadIdx.x;
  const int per = (nsys + kPrepThreads - 1) / kPrepThreads;
  const int p0 = tid * per, p1 = p0 + per < nsys ? p0 + per : nsys;
  int64_t tg = 0, tw = 0;
  for (int p = p0; p < p1; ++p) {
    const int s = order ? order[p] : p;
    int64_t G = 0, words = 0;
    if (s >= 0 && s < nsys) {
      const rsk_batch_item it = items[s];
      BatchPlan pl;
      const bool ok = item_plan(kind, it, esize, vec, tab, lds_launch, &pl);
      if (ok) { G = pl.G; words = pl.words; }
      if (it.status_dev) {
        it.status_dev[0] = ok ? 0 : 1;
        it.status_dev[1] = 0;
      }
    }
    tg += G;
    tw += words;
  }
  sg[tid] = tg;
  sw[tid] = tw;
  __syncthreads();
  // inclusive scan of the per-thread sums (Hillis-Steele)
  for (int off = 1; off < kPrepThreads; off <<= 1) {
    const int64_t ag = tid >= off ? sg[tid - off] : 0, aw = tid >= off ? sw[tid - off] : 0;
    __syncthreads();
    sg[tid] += ag;
    sw[tid] += aw;
    __syncthreads();
  }
  int64_t rg = tid ? sg[tid - 1] : 0, rw = tid ? sw[tid - 1] : 0;
  const bool fits = sw[kPrepThreads - 1] <= cap_words;
  for (int p = p0; p < p1; ++p) {
    const int s = order ? order[p] : p;
    int64_t G = 0, words = 0;
    if (s >= 0 && s < nsys) {
      const rsk_batch_item it = items[s];
      BatchPlan pl;
      if (item_plan(kind, it, esize, vec, tab, lds_launch, &pl)) {
        G = pl.G;
        words = pl.words;
      }
    }
    ticket0[p] = fits ? rg : 0;
    woff[p] = rw;
    if (!fits && s >= 0 && s < nsys && items[s].status_dev) items[s].status_dev[0] = RSK_ERR_WORKSPACE;
    rg += G;
    rw += words;
  }
  if (tid == kPrepThreads - 1) ticket0[nsys] = fits ? sg[tid] : 0;
}

template <typename T, int VEC>
__global__ __launch_bounds__(kDenseThreads, 2) void rska_batched(const rsk_batch_item* __restrict__ items,
                                                              const int32_t* __restrict__ order, int nsys,
                                                              const int64_t* __restrict__ ticket0,
                                                              const int64_t* __restrict__ woff, u64* queue,
                                                              u64* regions, BatchWgTable tab, uint64_t join_ticks) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int64_t sh[3];
  for (;;) {
    int64_t t;
    int p;
    if (!take_ticket(ticket0, nsys, queue, sh, &t, &p)) break;  // every workgroup ends here once the tickets are gone
    const int s = order ? order[p] : p;
    const rsk_batch_item it = items[s];
    BatchPlan pl;
    batched_plan(it.n, it.eta, sizeof(T), VEC, tab, &pl);  // succeeded in the prep kernel
    const int rank = (int)(t - ticket0[p]);
    u64* region = regions + woff[p];
    if (!join_group(region, pl.G, it.status_dev, join_ticks, sh)) continue;
    DenseArgs<T> a;
    fill_args(a, it, pl, region);
    if (a.tile_cache == 2 && dense_pipe_ok(sizeof(T), VEC, a.eta, a.wq_max))
      dense_run<T, VEC, kDenseThreads, true>(a, rank, rank, smem);
    else
      dense_run<T, VEC, kDenseThreads, false>(a, rank, rank, smem);
  }
}

// Register-tile batched launch (float32): the same tickets and join; a system's ranks run
// rt_run on the system's plan (slices in rank order, cpl chunk slots a lane).
__global__ __launch_bounds__(kBrtThreads) void rska_batched_rt(const rsk_batch_item* __restrict__ items,
                                                               const int32_t* __restrict__ order, int nsys,
                                                               const int64_t* __restrict__ ticket0,
                                                               const int64_t* __restrict__ woff, u64* queue,
                                                               u64* regions, BatchWgTable tab, uint64_t join_ticks) {
  __shared__ int64_t sh[3];
  for (;;) {
    int64_t t;
    int p;
    if (!take_ticket(ticket0, nsys, queue, sh, &t, &p)) break;
    const int s = order ? order[p] : p;
    const rsk_batch_item it = items[s];
    BatchPlan pl;
    batched_rt_plan(it.n, it.eta, tab, &pl);  // succeeded in the prep kernel
    const int rank = (int)(t - ticket0[p]);
    u64* region = regions + woff[p];
    if (!join_group(region, pl.G, it.status_dev, join_ticks, sh)) continue;
    DenseArgs<float> a;
    fill_args(a, it, pl, region);
    rt_run<kBrtThreads, kBrtPasses, kBrtCpl, 1, true, kBrtPfBytes>(a, rank, pl.cpl);
    __syncthreads();  // the body's LDS is reused by the next ticket's system
  }
}

hipError_t launch_batched_prep(int kind, const rsk_batch_item* items, const int32_t* order, int nsys, int esize,
                               int vec, const BatchWgTable& tab, size_t lds_launch, int64_t cap_words,
                               int64_t* ticket0, int64_t* woff, hipStream_t stream) {
  hipLaunchKernelGGL(batched_prep, dim3(1), dim3(kPrepThreads), 0, stream, kind, items, order, nsys, esize, vec, tab,
                     lds_launch, cap_words, ticket0, woff);
  return hipGetLastError();
}

int batched_rt_max_resident() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&rska_batched_rt, kBrtThreads, 0) !=
      hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

static uint64_t join_ticks_minute() {
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0) khz = 100000;
  return (uint64_t)khz * 1000ull * 60ull;
}

hipError_t launch_batched_rt(const rsk_batch_item* items, const int32_t* order, int nsys, const int64_t* ticket0,
                             const int64_t* woff, u64* queue, u64* regions, const BatchWgTable& tab, int grid,
                             hipStream_t stream) {
  uint64_t join_ticks = join_ticks_minute();
  BatchWgTable t = tab;
  void* args[] = {&items, &order, &nsys, &ticket0, &woff, &queue, &regions, &t, &join_ticks};
  return launch_persistent((const void*)&rska_batched_rt, dim3(grid), dim3(kBrtThreads), args, 0, stream);
}

static void* batched_fn(int dtype, int vec) {
  if (dtype == RSK_F64) return vec == 2 ? (void*)&rska_batched<double, 2> : (void*)&rska_batched<double, 1>;
  return vec == 4 ? (void*)&rska_batched<float, 4> : (void*)&rska_batched<float, 1>;
}

int batched_max_resident(int dtype, int vec, size_t lds) {
  if (lds > 160 * 1024) return 0;
  void* fn = batched_fn(dtype, vec);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kDenseThreads, lds) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_batched(const rsk_batch_item* items, const int32_t* order, int nsys, const int64_t* ticket0,
                          const int64_t* woff, u64* queue, u64* regions, const BatchWgTable& tab, int dtype, int vec,
                          size_t lds, int grid, hipStream_t stream) {
  void* fn = batched_fn(dtype, vec);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess)
    return hipErrorInvalidValue;
  uint64_t join_ticks = join_ticks_minute();
  BatchWgTable t = tab;
  void* args[] = {&items, &order, &nsys, &ticket0, &woff, &queue, &regions, &t, &join_ticks};
  // co-residency of the whole grid: a group forms only from running workgroups
  return launch_persistent(fn, dim3(grid), dim3(kDenseThreads), args, (unsigned)lds, stream);
}

}  // namespace rsk
