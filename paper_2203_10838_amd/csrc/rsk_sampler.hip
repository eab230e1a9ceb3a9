// Row sampler on the device: the index stream tau_k (Sec. 1.1: eta rows per
// step, with replacement, p_i proportional to ||a_i||^2) drawn from the
// counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11)
// and an inverse-CDF search, so long streams need neither host generation
// nor a host-to-device copy.
//
// Index t of step k: Philox4x32-10 of the counter (t, k mod 2^32, k div 2^32, 0)
// under the key (seed mod 2^32, seed div 2^32) gives words w0, w1;
// u = ((w0 >> 5) 2^26 + (w1 >> 6)) 2^-53 in [0, 1); the row is the first i with
// cdf_i > u cdf_{m-1}. Given the same cdf array the stream is bit-for-bit a
// function of (seed, k, t) alone, whatever the launch shape.
//
// The cdf (running sums of the FP64 row norms) is built by a three-pass scan:
// chunk sums, one fixed-order scan of the chunk sums, chunk-local scans.
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 8;                       // elements per thread
constexpr int kScanChunk = kScanThreads * kScanPer;

__device__ __forceinline__ void philox4x32_10(uint32_t (&c)[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(0xD2511F53u, c[0]), lo0 = 0xD2511F53u * c[0];
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c[2]), lo1 = 0xCD9E8D57u * c[2];
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

}  // namespace

__global__ __launch_bounds__(256) void sample_stream_kernel(const double* __restrict__ cdf, int64_t m, uint32_t key0,
                                                            uint32_t key1, int64_t k0, int64_t K, int eta,
                                                            int32_t* __restrict__ out) {
  const double total = cdf[m - 1];
  const int64_t N = K * (int64_t)eta;
  for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < N; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = k0 + e / eta;
    const uint32_t t = (uint32_t)(e % eta);
    uint32_t c[4] = {t, (uint32_t)k, (uint32_t)((uint64_t)k >> 32), 0u};
    philox4x32_10(c, key0, key1);
    const uint64_t bits = ((uint64_t)(c[0] >> 5) << 26) | (uint64_t)(c[1] >> 6);
    const double target = (double)bits * (1.0 / 9007199254740992.0) * total;
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (cdf[mid] > target) hi = mid;
      else lo = mid + 1;
    }
    out[e] = (int32_t)(lo < m ? lo : m - 1);
  }
}

// ||a_i||^2 in double (row i read once, coalesced), divided by row_w[i] when given (the
// sampling weights ||a_i||^2 / w_i of variant v4, Sec. 5).
template <typename T>
__global__ void rownorm2_f64_kernel(const T* __restrict__ A, int64_t m, int64_t n, int64_t ld,
                                    const T* __restrict__ row_w, double* __restrict__ w) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t i = wave; i < m; i += nwaves) {
    const T* rowp = A + i * ld;
    double s = 0.0;
    for (int64_t j = lane; j < n; j += 64) {
      const double v = (double)rowp[j];
      s += v * v;
    }
    s = wave_sum(s);
    if (lane == 0) w[i] = row_w ? s / (double)row_w[i] : s;
  }
}

// Chunk c covers [c * kScanChunk, (c + 1) * kScanChunk): its sum (thread-sequential, then threads in order).
__global__ __launch_bounds__(kScanThreads) void scan_chunk_sums(const double* __restrict__ w, int64_t m,
                                                                double* __restrict__ csum) {
  __shared__ double part[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j)
    if (base + j < m) s += w[base + j];
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < kScanThreads; ++i) t += part[i];
    csum[blockIdx.x] = t;
  }
}

// Exclusive prefix of the chunk sums, in chunk order (one thread).
__global__ void scan_chunk_prefix(double* csum, int64_t nchunks) {
  if (threadIdx.x != 0) return;
  double s = 0.0;
  for (int64_t c = 0; c < nchunks; ++c) {
    const double v = csum[c];
    csum[c] = s;
    s += v;
  }
}

// Inclusive scan inside each chunk, offset by the chunk's prefix.
__global__ __launch_bounds__(kScanThreads) void scan_chunk_apply(const double* __restrict__ w, int64_t m,
                                                                 const double* __restrict__ cpre,
                                                                 double* __restrict__ cdf) {
  __shared__ double part[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  double v[kScanPer];
  double s = 0.0;
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    v[j] = base + j < m ? w[base + j] : 0.0;
    s += v[j];
  }
  part[threadIdx.x] = s;
  __syncthreads();
  if (threadIdx.x == 0) {  // exclusive prefix of the thread sums, in thread order
    double t = 0.0;
    for (int i = 0; i < kScanThreads; ++i) {
      const double x = part[i];
      part[i] = t;
      t += x;
    }
  }
  __syncthreads();
  double r = cpre[blockIdx.x] + part[threadIdx.x];
#pragma unroll
  for (int j = 0; j < kScanPer; ++j) {
    r += v[j];
    if (base + j < m) cdf[base + j] = r;
  }
}

size_t sampling_cdf_ws_bytes(int64_t m) {
  const int64_t nch = (m + kScanChunk - 1) / kScanChunk;
  return ((size_t)m * sizeof(double) + 255) / 256 * 256 + ((size_t)nch * sizeof(double) + 255) / 256 * 256;
}

static void launch_scan(const double* w, int64_t m, double* cdf, double* csum, hipStream_t stream) {
  const int64_t nch = (m + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(scan_chunk_sums, dim3((unsigned)nch), dim3(kScanThreads), 0, stream, w, m, csum);
  hipLaunchKernelGGL(scan_chunk_prefix, dim3(1), dim3(64), 0, stream, csum, nch);
  hipLaunchKernelGGL(scan_chunk_apply, dim3((unsigned)nch), dim3(kScanThreads), 0, stream, w, m, csum, cdf);
}

template <typename T>
hipError_t launch_sampling_cdf(const T* A, int64_t m, int64_t n, int64_t ld, const T* row_w, double* cdf, void* ws,
                               hipStream_t stream) {
  double* w = (double*)ws;
  double* csum = (double*)((unsigned char*)ws + ((size_t)m * sizeof(double) + 255) / 256 * 256);
  const int64_t waves = m < 65536 ? m : 65536;
  hipLaunchKernelGGL(rownorm2_f64_kernel<T>, dim3((unsigned)((waves * 64 + 255) / 256)), dim3(256), 0, stream, A, m,
                     n, ld, row_w, w);
  launch_scan(w, m, cdf, csum, stream);
  return hipGetLastError();
}

hipError_t launch_sampling_cdf_weights(const double* w, int64_t m, double* cdf, void* ws, hipStream_t stream) {
  double* csum = (double*)((unsigned char*)ws + ((size_t)m * sizeof(double) + 255) / 256 * 256);
  launch_scan(w, m, cdf, csum, stream);
  return hipGetLastError();
}

hipError_t launch_sample_stream(const double* cdf, int64_t m, uint64_t seed, int64_t k0, int64_t K, int eta,
                                int32_t* out, hipStream_t stream) {
  const int64_t N = K * (int64_t)eta;
  if (N == 0) return hipSuccess;
  int64_t blocks = (N + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(sample_stream_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, cdf, m, (uint32_t)seed,
                     (uint32_t)(seed >> 32), k0, K, eta, out);
  return hipGetLastError();
}

template hipError_t launch_sampling_cdf<float>(const float*, int64_t, int64_t, int64_t, const float*, double*,
                                               void*, hipStream_t);
template hipError_t launch_sampling_cdf<double>(const double*, int64_t, int64_t, int64_t, const double*, double*,
                                                void*, hipStream_t);

}  // namespace rsk
