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
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

template <typename T, int VEC>
__device__ __forceinline__ Vec<T, VEC> load_chunk(const T* __restrict__ rowp, int64_t col, int64_t n) {
  Vec<T, VEC> v;
  if (col + VEC <= n) {
    v = *reinterpret_cast<const Vec<T, VEC>*>(rowp + col);
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = (col + e < n) ? rowp[col + e] : T(0);
  }
  return v;
}

template <typename T>
__device__ __forceinline__ T coef_of(T s, int i, const DenseArgs<T>& a, T ak, int& zero_row) {
  const T rn = a.r2[i];
  if (rn == T(0)) { zero_row = 1; return T(NAN); }
  return (ak / T(a.eta)) * (s - a.b[i]) / rn;
}

constexpr int align16(size_t v) { return (int)((v + 15) & ~size_t(15)); }

template <typename T, int VEC>
struct DenseSmem {
  size_t xs, xv, cs, tau, red, flags, tile, total;
  __host__ __device__ DenseSmem(int wq_max, int eta, int nt, int tile_cache) {
    size_t o = 0;
    xs = o; o += align16(sizeof(T) * (size_t)wq_max * VEC);
    xv = o; o += align16(sizeof(T) * (size_t)wq_max * VEC);
    cs = o; o += align16(sizeof(T) * (size_t)eta);
    tau = o; o += align16(sizeof(int) * (size_t)eta);
    red = o; o += align16(sizeof(T) * (size_t)nt * VEC);
    flags = o; o += 128;
    tile = o; o += tile_cache ? align16(sizeof(T) * (size_t)eta * wq_max * VEC) : 0;
    total = o;
  }
};

template <typename T, int VEC, int NT>
__global__ __launch_bounds__(NT) void rska_dense_persistent(DenseArgs<T> a) {
  extern __shared__ __align__(16) unsigned char smem[];
  using V = Vec<T, VEC>;
  constexpr int NW = NT / 64;
  constexpr int W = Words<T>::N;
  const int g = blockIdx.x, G = a.G, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int eta = a.eta;

  DenseSmem<T, VEC> L(a.wq_max, eta, NT, a.tile_cache);
  T* xs = reinterpret_cast<T*>(smem + L.xs);
  T* xv = reinterpret_cast<T*>(smem + L.xv);
  T* cs = reinterpret_cast<T*>(smem + L.cs);
  int* tau = reinterpret_cast<int*>(smem + L.tau);
  V* red = reinterpret_cast<V*>(smem + L.red);
  double* mon = reinterpret_cast<double*>(smem + L.flags);
  V* tile = reinterpret_cast<V*>(smem + L.tile);

  const int s = xcd_slice(g, G);
  const int64_t q0 = (int64_t)s * a.nchunks / G, q1 = (int64_t)(s + 1) * a.nchunks / G;
  const int wq = (int)(q1 - q0);
  const int64_t c0 = q0 * VEC;
  const int wcols = wq * VEC;

  // x*_0, x_0 = S_lambda(x*_0)
  for (int j = tid; j < wcols; j += NT) {
    const int64_t c = c0 + j;
    T z = (a.warm && c < a.n) ? a.x_star[c] : T(0);
    xs[j] = z;
    xv[j] = shrink(z, a.lambda);
  }
  __syncthreads();

  const int lpr = a.lpr, rpw = 64 / lpr;
  const int rs = lane / lpr, cl = lane % lpr;
  int64_t k_done = 0;
  int stop_code = 0;

  for (int64_t k = 0; k < a.K; ++k) {
    const unsigned tag = (unsigned)(k + 1);
    const T ak = a.alpha_k ? a.alpha_k[k] : a.alpha;
    // partials are double-buffered by step parity: with every workgroup
    // reducing every row, a fast workgroup may publish step k+1 while a slow
    // one still reads step k
    u64* xP = a.xP + (size_t)(k & 1) * G * eta * W;
    int lerr = 0;

    // 1. the step's indices (every workgroup reads all of them, so a bad
    //    index stops every workgroup at the same step)
    const int32_t* tk = a.idx + k * (int64_t)eta;
    for (int t = tid; t < eta; t += NT) {
      const int i = tk[t];
      if (i < 0 || (int64_t)i >= a.m) lerr = ST_INDEX;
      tau[t] = i;
    }
    if (__syncthreads_or(lerr)) { stop_code = ST_INDEX; break; }

    // 2. partial dots over the own columns
    for (int tb = wave * rpw; tb < eta; tb += NW * rpw) {
      const int t = tb + rs;
      T acc = T(0);
      if (t < eta) {
        const T* rowp = a.A + (int64_t)tau[t] * a.ld;
        for (int q = cl; q < wq; q += lpr) {
          const V v = load_chunk<T, VEC>(rowp, c0 + (int64_t)q * VEC, a.n);
          if (a.tile_cache) tile[(size_t)t * wq + q] = v;
          const V xx = reinterpret_cast<const V*>(xv)[q];
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc += v.v[e] * xx.v[e];
        }
      }
      acc = group_sum(acc, lpr);
      if (t < eta && cl == 0) put_tagged(&xP[((size_t)g * eta + t) * W], acc, tag);
    }

    // 3./4. all-reduce of the partials, coefficients into cs[]
    int zero_row = 0;
    if (!a.two_hop) {
      for (int t = wave; t < eta; t += NW) {
        T sum = T(0);
        for (int q = lane; q < G; q += 64) sum += wait_tagged<T>(&xP[((size_t)q * eta + t) * W], tag, lerr);
        sum = wave_sum(sum);
        if (lane == 0) cs[t] = coef_of(sum, tau[t], a, ak, zero_row);
      }
    } else {
      for (int t = g + wave * G; t < eta; t += NW * G) {
        T sum = T(0);
        for (int q = lane; q < G; q += 64) sum += wait_tagged<T>(&xP[((size_t)q * eta + t) * W], tag, lerr);
        sum = wave_sum(sum);
        if (lane == 0) {
          const T c = coef_of(sum, tau[t], a, ak, zero_row);
          if (zero_row) set_status(a.status, ST_ZERO_ROW);
          put_tagged(&a.xC[(size_t)t * W], c, tag);
        }
      }
      for (int t = tid; t < eta; t += NT) cs[t] = wait_tagged<T>(&a.xC[(size_t)t * W], tag, lerr);
    }
    if (zero_row) set_status(a.status, ST_ZERO_ROW);
    __syncthreads();
    int bad = 0;
    for (int t = tid; t < eta; t += NT) bad |= !isfinite(cs[t]);
    if (lerr) set_status(a.status, lerr);
    const int any_err = __syncthreads_or(lerr);
    if (__syncthreads_or(bad) || any_err) { stop_code = any_err ? ST_ABORTED : ST_NONFINITE; break; }

    if (a.y && g == 0)
      for (int t = tid; t < eta; t += NT) atomicAdd(&a.y[tau[t]], -cs[t]);

    // 5. transposed update of the own columns, fused with S_lambda
    if (wq <= NT) {
      const int nrg = NT / wq, rg = tid / wq, q = tid % wq;
      if (rg < nrg) {
        V acc;
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc.v[e] = T(0);
        for (int t = rg; t < eta; t += nrg) {
          const T c = cs[t];
          V v;
          if (a.tile_cache) v = tile[(size_t)t * wq + q];
          else v = load_chunk<T, VEC>(a.A + (int64_t)tau[t] * a.ld, c0 + (int64_t)q * VEC, a.n);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc.v[e] += c * v.v[e];
        }
        red[rg * wq + q] = acc;
      }
      __syncthreads();
      if (tid < wq) {
        V d = red[tid];
        for (int r = 1; r < nrg; ++r) {
          const V o = red[r * wq + tid];
#pragma unroll
          for (int e = 0; e < VEC; ++e) d.v[e] += o.v[e];
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int j = tid * VEC + e;
          const T z = xs[j] - d.v[e];
          xs[j] = z;
          xv[j] = shrink(z, a.lambda);
        }
      }
    } else {
      for (int q = tid; q < wq; q += NT) {
        V d;
#pragma unroll
        for (int e = 0; e < VEC; ++e) d.v[e] = T(0);
        for (int t = 0; t < eta; ++t) {
          const T c = cs[t];
          V v;
          if (a.tile_cache) v = tile[(size_t)t * wq + q];
          else v = load_chunk<T, VEC>(a.A + (int64_t)tau[t] * a.ld, c0 + (int64_t)q * VEC, a.n);
#pragma unroll
          for (int e = 0; e < VEC; ++e) d.v[e] += c * v.v[e];
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int j = q * VEC + e;
          const T z = xs[j] - d.v[e];
          xs[j] = z;
          xv[j] = shrink(z, a.lambda);
        }
      }
    }
    // columns past n inside the last chunk stay zero: their tile entries are zero
    __syncthreads();
    k_done = k + 1;

    // 6. monitor
    if (a.xref && a.check_every > 0 && (k + 1) % a.check_every == 0) {
      const unsigned mtag = (unsigned)((k + 1) / a.check_every);
      double e2 = 0.0, r2s = 0.0;
      for (int j = tid; j < wcols; j += NT) {
        const int64_t c = c0 + j;
        if (c < a.n) {
          const double rf = (double)a.xref[c];
          const double d = (double)xv[j] - rf;
          e2 += d * d;
          r2s += rf * rf;
        }
      }
      e2 = wave_sum(e2);
      r2s = wave_sum(r2s);
      if (lane == 0) { mon[2 * wave] = e2; mon[2 * wave + 1] = r2s; }
      __syncthreads();
      if (tid == 0) {
        double se = 0.0, sr = 0.0;
        for (int w = 0; w < NW; ++w) { se += mon[2 * w]; sr += mon[2 * w + 1]; }
        put_tagged(&a.xM[(size_t)g * 4], se, mtag);
        put_tagged(&a.xM[(size_t)g * 4 + 2], sr, mtag);
      }
      __syncthreads();
      if (wave == 0) {
        double se = 0.0, sr = 0.0;
        for (int q = lane; q < G; q += 64) {
          se += wait_tagged<double>(&a.xM[(size_t)q * 4], mtag, lerr);
          sr += wait_tagged<double>(&a.xM[(size_t)q * 4 + 2], mtag, lerr);
        }
        se = wave_sum(se);
        sr = wave_sum(sr);
        if (lane == 0) {
          const double err = sr > 0.0 ? sqrt(se / sr) : sqrt(se);
          if (g == 0 && a.err_hist) a.err_hist[mtag - 1] = err;
          mon[2 * NW] = err;
        }
      }
      if (lerr) set_status(a.status, lerr);
      if (__syncthreads_or(lerr)) { stop_code = ST_ABORTED; break; }
      const double err = mon[2 * NW];
      if (a.tol > 0.0 && err <= a.tol) break;
    }
  }
  if (stop_code && tid == 0) set_status(a.status, stop_code);

  __syncthreads();
  for (int j = tid; j < wcols; j += NT) {
    const int64_t c = c0 + j;
    if (c < a.n) { a.x_star[c] = xs[j]; a.x[c] = xv[j]; }
  }
  if (g == 0 && tid == 0) a.status[1] = (int)k_done;
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

constexpr int kDenseThreads = 256;

template <typename T, int VEC>
static void* dense_kernel_ptr() {
  return reinterpret_cast<void*>(&rska_dense_persistent<T, VEC, kDenseThreads>);
}

template <typename T>
static void* dense_kernel_for(int vec) {
  if (sizeof(T) == 4) {
    if (vec == 4) return dense_kernel_ptr<T, 4>();
    return dense_kernel_ptr<T, 1>();
  }
  if (vec == 2) return dense_kernel_ptr<T, 2>();
  return dense_kernel_ptr<T, 1>();
}

template <typename T>
static size_t dense_smem(int vec, int eta, int wq_max, int tile_cache) {
  switch (vec) {
    case 4: return DenseSmem<T, 4>(wq_max, eta, kDenseThreads, tile_cache).total;
    case 2: return DenseSmem<T, 2>(wq_max, eta, kDenseThreads, tile_cache).total;
    default: return DenseSmem<T, 1>(wq_max, eta, kDenseThreads, tile_cache).total;
  }
}

template <typename T>
int dense_max_grid(int vec, int eta, int wq_max, int tile_cache, size_t* lds_bytes) {
  const size_t lds = dense_smem<T>(vec, eta, wq_max, tile_cache);
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

template <typename T>
hipError_t launch_dense(DenseArgs<T>& a, int vec, hipStream_t stream, int* max_grid_out) {
  size_t lds = 0;
  const int maxg = dense_max_grid<T>(vec, a.eta, a.wq_max, a.tile_cache, &lds);
  if (max_grid_out) *max_grid_out = maxg;
  if (maxg < a.G) return hipErrorCooperativeLaunchTooLarge;
  void* fn = dense_kernel_for<T>(vec);
  void* args[] = {&a};
  return hipLaunchCooperativeKernel(fn, dim3(a.G), dim3(kDenseThreads), args, (unsigned)lds, stream);
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
template int dense_max_grid<float>(int, int, int, int, size_t*);
template int dense_max_grid<double>(int, int, int, int, size_t*);
template hipError_t launch_rownorm2_dense<float>(const float*, int64_t, int64_t, int64_t, float*, hipStream_t);
template hipError_t launch_rownorm2_dense<double>(const double*, int64_t, int64_t, int64_t, double*, hipStream_t);
template hipError_t launch_rownorm2_csr<float>(const int64_t*, const float*, int64_t, float*, hipStream_t);
template hipError_t launch_rownorm2_csr<double>(const int64_t*, const double*, int64_t, double*, hipStream_t);

}  // namespace rsk
