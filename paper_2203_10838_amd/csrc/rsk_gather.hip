// Gather-rate measurement: the HBM reads of the float32 register-tile solve alone.
//
// Workgroup g of G (the solve's XCD-aware slice order, row group h of rg) reads, for each of K
// steps, the part of the step's sampled rows that it reads in a solve on G workgroups: rows
// h * ceil(eta / rg) .. of the step, its column slice of whole 16-float units. There is no
// exchange and no update; each thread adds what it loads and writes its sum to sink (so that the
// loads are used). The time of K steps against their eta * n * 4 bytes a step is the rate at
// which HBM serves this pattern of row pieces: the ceiling of the solve's own rate.
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

constexpr int kGatherThreads = 512;
constexpr int kGatherMaxEta = 4096;
constexpr int kGatherInFlight = 16;  // float4 loads a thread issues before it adds them

// LAYOUT 0: thread e of a step's (row, chunk) items reads chunk e % wq of row e / wq (consecutive
// lanes cover a row's slice, so one instruction reads whole pieces of few rows). LAYOUT p > 0: the
// register tile's lanes over p passes of 128 rows (one row group, slices of at most 80 floats):
// lane l of wave w reads row 128 p + 16 w + l % 16 of pass p and chunks l / 16 + 4 r, r < 5 (one
// instruction: 64 bytes of each of 16 rows); chunks past the slice are clamped into it and rows
// past the step read row 0, as in the solve, and neither is added.
template <int LAYOUT>
__global__ __launch_bounds__(kGatherThreads) void gather_rate(const float* __restrict__ A, int64_t m, int64_t ld,
                                                              int64_t nchunks, const int32_t* __restrict__ idx,
                                                              int eta, int64_t K, int rg, float* __restrict__ sink) {
  __shared__ int rows[kGatherMaxEta];
  const int g = blockIdx.x, G = gridDim.x, tid = threadIdx.x;
  const int C = G / rg;
  const int sx = xcd_slice(g, G);
  const int s = sx / rg, h = sx % rg;
  const int etaR = (eta + rg - 1) / rg, hr0 = h * etaR;
  const int etaH = hr0 >= eta ? 0 : (eta - hr0 < etaR ? eta - hr0 : etaR);
  const int64_t nunits = (nchunks + 3) / 4;
  const int64_t q0 = (int64_t)s * nunits / C * 4;
  int64_t q1 = (int64_t)(s + 1) * nunits / C * 4;
  if (q1 > nchunks) q1 = nchunks;
  const int wq = (int)(q1 - q0);
  const int items = etaH * wq;  // (row, chunk) pairs a step
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t k = 0; k < K; ++k) {
    __syncthreads();  // the previous step's rows are read
    for (int t = tid; t < etaH; t += kGatherThreads) {
      const int i = idx[k * eta + hr0 + t];
      rows[t] = (i >= 0 && (int64_t)i < m) ? i : 0;  // a bad index reads row 0
    }
    __syncthreads();
    if constexpr (LAYOUT > 0) {
      // LAYOUT = passes (1 .. 8): every slot of the step is loaded before any is added, as in the
      // solve (rows past the step read row 0, chunks past the slice the slice's last chunk)
      constexpr int RP = LAYOUT, CPL = 5;
      const int lane = tid & 63, wave = tid >> 6;
      float4 v[RP][CPL];
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const int t = 128 * p + 16 * wave + (lane & 15);
        const float* rowp = A + (int64_t)(t < etaH ? rows[t] : 0) * ld + 4 * q0;
#pragma unroll
        for (int r = 0; r < CPL; ++r) {
          const int q = (lane >> 4) + 4 * r;
          v[p][r] = *reinterpret_cast<const float4*>(rowp + 4 * (q < wq ? q : wq - 1));
        }
      }
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const int t = 128 * p + 16 * wave + (lane & 15);
#pragma unroll
        for (int r = 0; r < CPL; ++r) {
          const int q = (lane >> 4) + 4 * r;
          if (t < etaH && q < wq) {
            acc.x += v[p][r].x;
            acc.y += v[p][r].y;
            acc.z += v[p][r].z;
            acc.w += v[p][r].w;
          }
        }
      }
      continue;
    }
    for (int e0 = tid; e0 < items; e0 += kGatherInFlight * kGatherThreads) {
      float4 v[kGatherInFlight];
#pragma unroll
      for (int u = 0; u < kGatherInFlight; ++u) {
        const int e = e0 + u * kGatherThreads;
        const int r = e < items ? e / wq : 0, q = e < items ? e % wq : 0;
        v[u] = *reinterpret_cast<const float4*>(A + (int64_t)rows[r] * ld + 4 * (q0 + q));
        if (e >= items) v[u] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int u = 0; u < kGatherInFlight; ++u) {
        acc.x += v[u].x;
        acc.y += v[u].y;
        acc.z += v[u].z;
        acc.w += v[u].w;
      }
    }
  }
  sink[(size_t)g * kGatherThreads + tid] = (acc.x + acc.y) + (acc.z + acc.w);
}

hipError_t launch_gather_rate(const float* A, int64_t m, int64_t ld, int64_t n, const int32_t* idx, int eta, int64_t K,
                              int G, int rg, int layout, float* sink, hipStream_t stream) {
  void (*fn)(const float*, int64_t, int64_t, int64_t, const int32_t*, int, int64_t, int, float*) = gather_rate<0>;
  if (layout == 1) {
    const int passes = (eta + 127) / 128;
    fn = passes <= 1 ? gather_rate<1> : passes == 2 ? gather_rate<2> : passes == 3 ? gather_rate<3>
       : passes == 4 ? gather_rate<4> : passes == 5 ? gather_rate<5> : passes == 6 ? gather_rate<6>
       : passes == 7 ? gather_rate<7> : gather_rate<8>;
  }
  hipLaunchKernelGGL(fn, dim3(G), dim3(kGatherThreads), 0, stream, A, m, ld, (n + 3) / 4, idx, eta, K, rg, sink);
  return hipGetLastError();
}

}  // namespace rsk
