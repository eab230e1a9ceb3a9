// Dense RSKA: one persistent launch runs K steps of eq. (rska) / Algorithm 1.
//
// Work split. Workgroup g owns a contiguous column slice of x* and x for the
// whole run (kept in LDS), so the transposed update x* -= sum_t c_t a_t and
// S_lambda touch only the owner's columns: the scatter needs no atomics.
// Per step:
//   1. read tau_k (eta indices) and check their range;
//   2. partial dots p_{g,t} = sum_{j in slice} A[tau_t, j] x_j, the slice of
//      each row read once, coalesced, and (when it fits) kept in LDS;
//   3. all-reduce of the eta partials across workgroups through tagged
//      64-bit words (see rsk_device.hpp): either every workgroup sums all of
//      them (small G*eta), or row owners sum and publish c_t, then everyone
//      gathers; the sum order is the same in both, so results are identical;
//   4. c_t = (alpha_k/eta) (r_t - b_{tau_t}) / ||a_{tau_t}||^2;
//   5. x*_j -= sum_t c_t A[tau_t, j] for the own columns, x_j = S_lambda(x*_j);
//   6. every check_every steps, ||x - x_ref|| / ||x_ref|| (monitor).
#include <cstdlib>

#include "rsk_dense_run.hpp"

namespace rsk {

template <typename T, int VEC, int NT>
__global__ __launch_bounds__(NT, 2) void rska_dense_persistent(DenseArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  if (a.tile_cache == 2 && dense_pipe_ok(sizeof(T), VEC, a.eta, a.wq_max))
    dense_run<T, VEC, NT, true>(a, blockIdx.x, xcd_slice(blockIdx.x, a.G), smem);
  else
    dense_run<T, VEC, NT, false>(a, blockIdx.x, xcd_slice(blockIdx.x, a.G), smem);
}

template <typename T>
__global__ void rownorm2_dense_kernel(const T* __restrict__ A, int64_t m, int64_t n, int64_t ld, T* __restrict__ r2) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < m; i += nwaves) {
    const T* rowp = A + i * ld;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) { const double v = (double)rowp[j]; s += v * v; }
    s = wave_sum(s);
    if (lane == 0) r2[i] = (T)s;
  }
}

template <typename T>
__global__ void rownorm2_csr_kernel(const int64_t* __restrict__ rp, const T* __restrict__ val, int64_t m, T* __restrict__ r2) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < m; i += nwaves) {
    double s = 0.0;
    for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += 64) { const double v = (double)val[p]; s += v * v; }
    s = wave_sum(s);
    if (lane == 0) r2[i] = (T)s;
  }
}

__global__ void zero_words_kernel(u64* p, size_t nwords) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < nwords; i += (size_t)gridDim.x * blockDim.x) p[i] = 0ull;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <typename T, int VEC>
static void* dense_kernel_ptr() {
  return reinterpret_cast<void*>(&rska_dense_persistent<T, VEC, kDenseThreads>);
}

template <typename T>
static void* dense_kernel_for(int vec) {
  if constexpr (sizeof(T) == 4) {
    if (vec == 4) return dense_kernel_ptr<T, 4>();
    return dense_kernel_ptr<T, 1>();
  } else {
    if (vec == 2) return dense_kernel_ptr<T, 2>();
    return dense_kernel_ptr<T, 1>();
  }
}

template <typename T>
static size_t dense_smem(int vec, int eta, int wq_max, int tile_cache, int64_t xr_elems) {
  return DenseSmem(sizeof(T), vec, wq_max, eta, kDenseThreads, tile_cache, xr_elems).total;
}

template <typename T>
int dense_max_grid(int vec, int eta, int wq_max, int tile_cache, int64_t xr_elems, size_t* lds_bytes) {
  const size_t lds = dense_smem<T>(vec, eta, wq_max, tile_cache, xr_elems);
  if (lds_bytes) *lds_bytes = lds;
  if (lds > 160 * 1024) return 0;
  void* fn = dense_kernel_for<T>(vec);
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds) != hipSuccess) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kDenseThreads, lds) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_persistent(const void* fn, dim3 grid, dim3 block, void** args, unsigned lds, hipStream_t stream) {
  static const bool coop = [] {
    const char* e = getenv("RSK_COOPERATIVE");
    return !(e && e[0] == '0' && e[1] == 0);
  }();
  return coop ? hipLaunchCooperativeKernel(fn, grid, block, args, lds, stream)
              : hipLaunchKernel(fn, grid, block, args, lds, stream);
}

template <typename T>
hipError_t launch_dense(DenseArgs<T>& a, int vec, hipStream_t stream, int* max_grid_out) {
  size_t lds = 0;
  const int maxg = dense_max_grid<T>(vec, a.eta, a.wq_max, a.tile_cache,
                                     a.two_hop ? 0 : onehop_lds_elems(a.G, a.eta), &lds);
  if (max_grid_out) *max_grid_out = maxg;
  if (maxg < a.G) return hipErrorCooperativeLaunchTooLarge;
  void* fn = dense_kernel_for<T>(vec);
  void* args[] = {&a};
  return launch_persistent(fn, dim3(a.G), dim3(kDenseThreads), args, (unsigned)lds, stream);
}

template <typename T>
hipError_t launch_rownorm2_dense(const T* A, int64_t m, int64_t n, int64_t ld, T* r2, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  const int64_t waves = m < 65536 ? m : 65536;
  const int blocks = (int)((waves * 64 + 255) / 256);
  hipLaunchKernelGGL(rownorm2_dense_kernel<T>, dim3(blocks), dim3(256), 0, stream, A, m, n, ld, r2);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_rownorm2_csr(const int64_t* row_ptr, const T* val, int64_t m, T* r2, hipStream_t stream) {
  if (m <= 0) return hipSuccess;
  const int64_t waves = m < 65536 ? m : 65536;
  const int blocks = (int)((waves * 64 + 255) / 256);
  hipLaunchKernelGGL(rownorm2_csr_kernel<T>, dim3(blocks), dim3(256), 0, stream, row_ptr, val, m, r2);
  return hipGetLastError();
}

__global__ void zero_status_kernel(int* s) {
  if (threadIdx.x < 2) s[threadIdx.x] = 0;
}

hipError_t launch_zero_status(int* status, hipStream_t stream) {
  hipLaunchKernelGGL(zero_status_kernel, dim3(1), dim3(64), 0, stream, status);
  return hipGetLastError();
}

hipError_t launch_zero_words(u64* p, size_t nwords, hipStream_t stream) {
  if (nwords == 0) return hipSuccess;
  size_t blocks = (nwords + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  hipLaunchKernelGGL(zero_words_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, p, nwords);
  return hipGetLastError();
}

template hipError_t launch_dense<float>(DenseArgs<float>&, int, hipStream_t, int*);
template hipError_t launch_dense<double>(DenseArgs<double>&, int, hipStream_t, int*);
template int dense_max_grid<float>(int, int, int, int, int64_t, size_t*);
template int dense_max_grid<double>(int, int, int, int, int64_t, size_t*);
template hipError_t launch_rownorm2_dense<float>(const float*, int64_t, int64_t, int64_t, float*, hipStream_t);
template hipError_t launch_rownorm2_dense<double>(const double*, int64_t, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_rownorm2_csr<float>(const int64_t*, const float*, int64_t, float*, hipStream_t);
template hipError_t launch_rownorm2_csr<double>(const int64_t*, const double*, int64_t, double*, hipStream_t);

}  // namespace rsk
