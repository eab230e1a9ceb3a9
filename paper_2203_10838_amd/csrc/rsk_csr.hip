// CSR RSKA: one persistent workgroup runs K steps of eq. (rska) / Algorithm 1
// on a sparse A (row_ptr int64, col int32, val).
//
// A step of the sparse workloads moves little data (eta rows of a few dozen
// nonzeros), so it is bound by latency, not bandwidth. One workgroup on one CU
// keeps every access to x* and x inside one XCD's caches and needs no
// cross-CU exchange at all.
//
// Per step, one thread per sampled row (chunks of 32 nonzeros held in registers):
//   1. r_t = sum_p val_p x[col_p] - b_{tau_t};  c_t = (alpha_k/eta) r_t / ||a_{tau_t}||^2
//   2. contributions v_p = c_t val_p are added into x*[col_p]. Columns hit by
//      several sampled rows must sum in a fixed order to stay reproducible, so
//      the contributions are accumulated as int64 fixed point with the step's
//      power-of-two quantum q = 2^(e-40), e = exponent of max |v_p| (integer
//      adds commute), and every column's total is applied once by the lane
//      that swaps it out of the accumulator: x*_j -= total*q, x_j = S_lambda(x*_j).
//      The quantisation error is below 2^-41 of the step's largest
//      contribution, far under float32 resolution of the update.
//   3. the optional dual output y (y_i -= c_t for every slot t of row i, the
//      dual update at the start of Sec. 4) is applied once per row and step:
//      each slot counts itself on an integer per-row counter, and the slot
//      whose increment found zero applies all of the row's coefficients in
//      slot order, so y is bitwise reproducible however the slots race.
// x*, x and the accumulators live in global memory and are shared only within
// the workgroup, so workgroup-scope atomics order them (device-scope atomics
// would cost a serialized memory round trip each).
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

namespace {

constexpr int kCsrThreads = 512;
constexpr int kCsrWaves = kCsrThreads / 64;
constexpr int kRowChunk = 32;   // nonzeros of a row a thread holds in registers
constexpr int kSub = 8;         // swaps in flight per thread when applying totals
static_assert(kCsrMaxEta <= 32 * kCsrThreads, "a thread's y-owner bits fit one word");

template <typename T>
__device__ __forceinline__ T ld_wg(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <typename T>
__device__ __forceinline__ void st_wg(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The update loops below are branch-free: every slot issues its atomic, an
// empty slot (-1) on the spare accumulator acc[n] with value 0, so the
// compiler issues all of them back to back instead of waiting on each.

// Add the chunk's quantised contributions c*val into the column accumulators.
template <typename T>
__device__ __forceinline__ void accumulate(long long* acc, int64_t n, const int (&jc)[kRowChunk],
                                           const T (&vv)[kRowChunk], T c, int e) {
#pragma unroll
  for (int i = 0; i < kRowChunk; ++i) {
    const bool on = jc[i] >= 0;
    const long long v = on ? (long long)llrint(ldexp((double)(c * vv[i]), 40 - e)) : 0ll;
    __hip_atomic_fetch_add(&acc[on ? (int64_t)jc[i] : n], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
  }
}

// Apply each touched column's total once: the thread that swaps a non-zero
// total out of the accumulator updates x*_j and x_j.
template <typename T>
__device__ __forceinline__ void apply(const CsrArgs<T>& a, const int (&jc)[kRowChunk], int e) {
#pragma unroll
  for (int i0 = 0; i0 < kRowChunk; i0 += kSub) {
    long long tot[kSub];
#pragma unroll
    for (int i = 0; i < kSub; ++i) {
      const int j = jc[i0 + i];
      tot[i] = __hip_atomic_exchange(&a.acc[j >= 0 ? (int64_t)j : a.n], 0ll, __ATOMIC_RELAXED,
                                     __HIP_MEMORY_SCOPE_WORKGROUP);
    }
    T zo[kSub];
#pragma unroll
    for (int i = 0; i < kSub; ++i) zo[i] = ld_wg(a.x_star + (tot[i] != 0 ? jc[i0 + i] : 0));
#pragma unroll
    for (int i = 0; i < kSub; ++i) {
      if (tot[i] != 0) {
        const T z = (T)((double)zo[i] - ldexp((double)tot[i], e - 40));
        st_wg(a.x_star + jc[i0 + i], z);
        st_wg(a.x + jc[i0 + i], shrink(z, a.lambda));
      }
    }
  }
}

// Columns and values of nonzeros [q, q+32) of a row (extent p0..p1, p1 > p0);
// -1 marks past the end (the load itself is clamped into the row).
template <typename T>
__device__ __forceinline__ void load_chunk(const CsrArgs<T>& a, int64_t p0, int64_t p1, int64_t q,
                                           int (&jc)[kRowChunk], T (&vv)[kRowChunk]) {
#pragma unroll
  for (int i = 0; i < kRowChunk; ++i) {
    const int64_t p = p0 + q + i;
    const int64_t pc = p < p1 ? p : p1 - 1;
    const int c = a.col[pc];
    const T v = a.val[pc];
    jc[i] = p < p1 ? c : -1;
    vv[i] = p < p1 ? v : T(0);
  }
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kCsrThreads) void rska_csr_single(CsrArgs<T> a) {
  __shared__ T cs[kCsrMaxEta];
  __shared__ double wmax[kCsrWaves];
  __shared__ double mon[2 * kCsrWaves];
  __shared__ int orw[2];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int eta = a.eta;
  // one sampled row per thread; eta <= 512 keeps each thread's row in registers
  const bool resident = eta <= kCsrThreads;
  if (tid < 2) orw[tid] = 0;

  for (int64_t j = tid; j < a.n; j += kCsrThreads) {
    const T z = a.warm ? a.x_star[j] : T(0);
    if (!a.warm) st_wg(a.x_star + j, z);
    st_wg(a.x + j, shrink(z, a.lambda));
  }
  __syncthreads();

  int64_t k_done = 0;
  int stop_code = 0;
  for (int64_t k = 0; k < a.K; ++k) {
    const T ak = a.alpha_k ? a.alpha_k[k] : a.alpha;
    const int32_t* tk = a.idx + k * (int64_t)eta;
    int lerr = 0;
    unsigned yown = 0;  // bit s: this thread's slot tid + s * kCsrThreads applies its row's y update

    // 1. residual and coefficient of each sampled row: r_t = sum_p val_p x[col_p] - b, c_t
    int jc[kRowChunk];
    T vv[kRowChunk];
    int64_t p0 = 0, p1 = 0;
    double vmax = 0.0;
    for (int t = tid, s = 0; t < eta; t += kCsrThreads, ++s) {
      const int i = tk[t];
      if (i < 0 || (int64_t)i >= a.m) { lerr = ST_INDEX; continue; }
      p0 = a.row_ptr[i];
      p1 = a.row_ptr[i + 1];
      T dot = T(0);
      for (int64_t q = 0; q < p1 - p0; q += kRowChunk) {
        load_chunk(a, p0, p1, q, jc, vv);
        T xg[kRowChunk];
#pragma unroll
        for (int u = 0; u < kRowChunk; ++u) {
          const bool ok = jc[u] >= 0 && (int64_t)jc[u] < a.n;
          if (!ok && jc[u] != -1) lerr = ST_INDEX;
          xg[u] = ld_wg(a.x + (ok ? jc[u] : 0));
          if (!ok) xg[u] = T(0);
        }
#pragma unroll
        for (int u = 0; u < kRowChunk; ++u) dot += vv[u] * xg[u];
      }
      const T rn = weighted_rn(a.r2, a.row_w, i);
      T c;
      if (rn == T(0)) { c = T(NAN); lerr = ST_ZERO_ROW; }
      else c = (ak / T(eta)) * (dot - a.b[i]) / rn;
      cs[t] = c;
      if (a.y && __hip_atomic_fetch_add(a.ycnt + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) == 0)
        yown |= 1u << s;
      // the step's largest contribution fixes the quantum
      for (int64_t q = 0; q < p1 - p0; q += kRowChunk) {
        if (!(resident && q == 0)) load_chunk(a, p0, p1, q, jc, vv);
#pragma unroll
        for (int u = 0; u < kRowChunk; ++u)
          if (jc[u] >= 0) vmax = fmax(vmax, fabs((double)(c * vv[u])));
      }
      if (resident && p1 - p0 > kRowChunk) load_chunk(a, p0, p1, 0, jc, vv);
    }
    if (lerr) set_status(a.status, lerr);
    // each thread checks the coefficients it wrote; one barrier publishes cs[] and wmax[] and
    // agrees on a fault (the thread that found it set the exact code first) or a non-finite c_t
    int bad = 0;
    for (int t = tid; t < eta; t += kCsrThreads) bad |= !isfinite(cs[t]);
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
    if (lane == 0) wmax[wave] = vmax;
    const int fl = block_or(orw, (lerr ? 1 : 0) | (bad ? 2 : 0), k);
    if (fl & 1) { stop_code = ST_INDEX; break; }
    if (fl & 2) { stop_code = ST_NONFINITE; break; }
    // dual output: the counters are final after the barrier; the owner takes the row's count
    // (resetting it for the next step) and subtracts its coefficients in slot order
    if (a.y) {
      for (int t = tid, s = 0; t < eta; t += kCsrThreads, ++s) {
        if (!((yown >> s) & 1u)) continue;
        const int i = tk[t];
        const int cnt = __hip_atomic_exchange(a.ycnt + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        T yi = ld_wg(a.y + i);
        if (cnt == 1) {
          yi -= cs[t];
        } else {
          for (int u = 0; u < eta; ++u)
            if (tk[u] == i) yi -= cs[u];
        }
        st_wg(a.y + i, yi);
      }
    }
    double gmax = 0.0;
    for (int w = 0; w < kCsrWaves; ++w) gmax = fmax(gmax, wmax[w]);
    // power-of-two quantum q = 2^(e-40): |v/q| < 2^41
    const int e = gmax > 0.0 ? ilogb(gmax) : 0;

    // 2. integer accumulation (integer adds commute: atomic order does not matter)
    if (gmax > 0.0) {
      for (int t = tid; t < eta; t += kCsrThreads) {
        const int i = tk[t];
        const int64_t r0 = a.row_ptr[i], r1 = a.row_ptr[i + 1];
        for (int64_t q = 0; q < r1 - r0; q += kRowChunk) {
          if (!(resident && q == 0)) load_chunk(a, r0, r1, q, jc, vv);
          accumulate(a.acc, a.n, jc, vv, cs[t], e);
        }
        if (resident && r1 - r0 > kRowChunk) load_chunk(a, r0, r1, 0, jc, vv);
      }
    }
    __syncthreads();
    // 3. apply every touched column once
    if (gmax > 0.0) {
      for (int t = tid; t < eta; t += kCsrThreads) {
        const int i = tk[t];
        const int64_t r0 = a.row_ptr[i], r1 = a.row_ptr[i + 1];
        for (int64_t q = 0; q < r1 - r0; q += kRowChunk) {
          if (!(resident && q == 0)) load_chunk(a, r0, r1, q, jc, vv);
          apply(a, jc, e);
        }
      }
    }
    __syncthreads();
    k_done = k + 1;

    if (a.xref && a.check_every > 0 && (k + 1) % a.check_every == 0) {
      double e2 = 0.0, r2s = 0.0;
      for (int64_t j = tid; j < a.n; j += kCsrThreads) {
        const double rf = (double)a.xref[j];
        const double d = (double)ld_wg(a.x + j) - rf;
        e2 += d * d;
        r2s += rf * rf;
      }
      e2 = wave_sum(e2);
      r2s = wave_sum(r2s);
      if (lane == 0) { mon[2 * wave] = e2; mon[2 * wave + 1] = r2s; }
      __syncthreads();
      double se = 0.0, sr = 0.0;
      for (int w = 0; w < kCsrWaves; ++w) { se += mon[2 * w]; sr += mon[2 * w + 1]; }
      const double err = sr > 0.0 ? sqrt(se / sr) : sqrt(se);
      if (tid == 0 && a.err_hist) a.err_hist[(k + 1) / a.check_every - 1] = err;
      __syncthreads();
      if (a.tol > 0.0 && err <= a.tol) break;
    }
  }
  if (stop_code && tid == 0) set_status(a.status, stop_code);
  if (tid == 0) a.status[1] = (int)k_done;
}

template <typename T>
hipError_t launch_csr(CsrArgs<T>& a, hipStream_t stream) {
  hipLaunchKernelGGL(rska_csr_single<T>, dim3(1), dim3(kCsrThreads), 0, stream, a);
  return hipGetLastError();
}

template hipError_t launch_csr<float>(CsrArgs<float>&, hipStream_t);
template hipError_t launch_csr<double>(CsrArgs<double>&, hipStream_t);

// ---------------------------------------------------------------------------
// Multi-workgroup CSR kernel.
//
// One sampled row per 32 lanes, one nonzero per lane (longer rows loop), so a
// step's 16K nonzeros spread over G workgroups instead of one CU's request
// queue. x*, x and the column accumulators are shared by all workgroups, so
// every access to them is an agent-scope atomic (coherent across the XCDs
// without cache maintenance). Per step, three grid barriers on one monotonic
// counter (each workgroup first waits for all of its own memory operations):
//   A. dots r_t (x gathered), c_t, contributions c_t a_{t,j}; the largest
//      exponent goes to a step-parity word by atomicMax;      barrier
//   B. int64 fixed-point accumulation with the step's quantum 2^(e-40)
//      (integer adds commute: the totals do not depend on atomic order);  barrier
//   C. every touched column applied once, by the lane that swaps its nonzero
//      total out of the accumulator: x*_j -= total q, x_j = S_lambda(x*_j); barrier
// x* and x are bitwise reproducible (the dots use a fixed lane order). The optional dual y
// is too: after barrier A, one slot per sampled row (the one whose increment of the row's
// integer counter found zero) subtracts the coefficients of all the row's slots, gathered by
// its 32 lanes in a fixed order from the step's coefficient array.
// ---------------------------------------------------------------------------

namespace {

constexpr int kGridThreads = 256;
constexpr int kEBias = 4096;  // biased exponent stored in emax (0 = no contribution)

template <typename T>
__device__ __forceinline__ T ld_ag(const T* p) {
  return __hip_atomic_load(const_cast<T*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_ag(T* p, T v) {
  // an exchange returns, so the write is complete before the workgroup arrives at the next barrier
  (void)__hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int CTRL>
__device__ __forceinline__ int dpp32(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dppf(float v) { return __int_as_float(dpp32<CTRL>(__float_as_int(v))); }
template <int CTRL>
__device__ __forceinline__ double dppf(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp32<CTRL>((int)b), hi = dpp32<CTRL>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ float swap16f(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ double swap16f(double v) {
  const long long b = __double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane16_swap((int)b, (int)b, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((int)(b >> 32), (int)(b >> 32), false, false);
  return __longlong_as_double((long long)(unsigned)l[0] | ((long long)h[0] << 32)) +
         __longlong_as_double((long long)(unsigned)l[1] | ((long long)h[1] << 32));
}
// Sum over an aligned group of 32 lanes (DPP within 16 lanes, then the 16-lane swap).
template <typename T>
__device__ __forceinline__ T sum32(T v) {
  v += dppf<0xB1>(v);
  v += dppf<0x4E>(v);
  v += dppf<0x141>(v);
  v += dppf<0x140>(v);
  return swap16f(v);
}

// Grid barrier number `nbar` (1, 2, ...; the counters only grow). Two levels, so that no
// counter takes more than a group's worth of atomics: workgroup g arrives on the counter of
// group g % 8 (workgroups are dispatched to the XCDs in turn), the last arriver of a group
// moves the global counter on, and every workgroup waits for all groups. Counters are 128
// bytes apart. Returns false if the bounded wait expired.
constexpr int kBarGroups = 8;
constexpr int kBarStride = 16;  // u64 words between counters
__device__ __forceinline__ bool grid_sync(u64* bar, u64 nbar, int G) {
  __builtin_amdgcn_s_waitcnt(0);  // this thread's memory operations are complete
  __syncthreads();
  __shared__ int ok;
  if (threadIdx.x == 0) {
    const int grp = (int)(blockIdx.x % kBarGroups);
    const int ngroups = G < kBarGroups ? G : kBarGroups;
    const u64 members = (u64)((G - grp + kBarGroups - 1) / kBarGroups);
    u64* gbar = bar + (size_t)kBarStride * (1 + grp);
    const u64 old = __hip_atomic_fetch_add(gbar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == members * nbar) __hip_atomic_fetch_add(bar, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const u64 target = (u64)ngroups * nbar;
    unsigned spins = 0;
    int good = 1;
    while (xload(bar) < target) {
      if (++spins > kSpinLimit) { good = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    ok = good;
  }
  __syncthreads();
  return ok != 0;
}

}  // namespace

template <typename T>
__global__ __launch_bounds__(kGridThreads) void rska_csr_grid(CsrArgs<T> a) {
  constexpr int RPP = kCsrGridRowsPerPass;
  __shared__ T cl[kCsrGridMaxPasses * RPP];
  __shared__ int il[kCsrGridMaxPasses * RPP];
  __shared__ int yo[kCsrGridMaxPasses * RPP];  // the slot applies its row's y update
  __shared__ double wmax[kGridThreads / 64];
  __shared__ double mon[2 * (kGridThreads / 64) + 2];
  const int g = blockIdx.x, G = a.G, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int hw = tid >> 5, p = tid & 31;
  const int eta = a.eta;
  const int passes = (eta + RPP * G - 1) / (RPP * G);
  u64 nbar = 0;
  int stop_code = 0;

  // x*_0, x_0 over this workgroup's column block
  const int64_t j0 = (int64_t)g * a.n / G, j1 = (int64_t)(g + 1) * a.n / G;
  for (int64_t j = j0 + tid; j < j1; j += kGridThreads) {
    const T z = a.warm ? ld_ag(a.x_star + j) : T(0);
    if (!a.warm) st_ag(a.x_star + j, z);
    st_ag(a.x + j, shrink(z, a.lambda));
  }
  if (!grid_sync(a.bar, ++nbar, G)) stop_code = ST_ABORTED;

  int64_t k_done = 0;
  for (int64_t k = 0; k < a.K && !stop_code; ++k) {
    const T ak = a.alpha_k ? a.alpha_k[k] : a.alpha;
    const int32_t* tk = a.idx + k * (int64_t)eta;
    int lerr = 0;
    double vmax = 0.0;

    // A. residuals, coefficients, largest contribution
    for (int ps = 0; ps < passes; ++ps) {
      const int t = ps * RPP * G + g * RPP + hw;
      if (t < eta) {
        int i = tk[t];
        if (i < 0 || (int64_t)i >= a.m) { lerr = ST_INDEX; i = -1; }
        T dot = T(0);
        int64_t r0 = 0, r1 = 0;
        if (i >= 0) { r0 = a.row_ptr[i]; r1 = a.row_ptr[i + 1]; }
        for (int64_t q = r0 + p; q < r1; q += 32) {
          const int j = a.col[q];
          const T v = a.val[q];
          if (j < 0 || (int64_t)j >= a.n) { lerr = ST_INDEX; continue; }
          dot += v * ld_ag(a.x + j);
        }
        dot = sum32(dot);
        T c = T(0);
        if (i >= 0) {
          const T rn = weighted_rn(a.r2, a.row_w, i);
          if (rn == T(0)) { lerr = ST_ZERO_ROW; c = T(NAN); }
          else c = (ak / T(eta)) * (dot - a.b[i]) / rn;
          if (!isfinite(c) && !lerr) lerr = ST_NONFINITE;
        }
        for (int64_t q = r0 + p; q < r1; q += 32) vmax = fmax(vmax, fabs((double)(c * a.val[q])));
        if (p == 0) {
          cl[ps * RPP + hw] = c;
          il[ps * RPP + hw] = i;
          if (a.y) {
            int own = 0;
            if (i >= 0) {
              st_ag(a.cy + t, c);
              own = __hip_atomic_fetch_add(a.ycnt + i, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0;
            }
            yo[ps * RPP + hw] = own;
          }
        }
      }
    }
    if (lerr) set_status(a.status, lerr);
    for (int off = 32; off > 0; off >>= 1) vmax = fmax(vmax, __shfl_xor(vmax, off));
    if (lane == 0) wmax[wave] = vmax;
    __syncthreads();
    if (tid == 0) {
      double m = 0.0;
      for (int w = 0; w < kGridThreads / 64; ++w) m = fmax(m, wmax[w]);
      if (m > 0.0 && isfinite(m))
        __hip_atomic_fetch_max(a.emax + (k & 1), ilogb(m) + kEBias, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!grid_sync(a.bar, ++nbar, G)) { stop_code = ST_ABORTED; break; }
    if (ld_ag(a.status)) { stop_code = -1; break; }  // the fault was recorded by the workgroup that saw it
    const int eb = ld_ag(a.emax + (k & 1));
    if (g == 0 && tid == 0) st_ag(a.emax + ((k + 1) & 1), 0);  // read by everyone two barriers ago

    // dual output (the counters and coefficients are complete after barrier A): the owning
    // slot takes its row's count, resetting it for the next step; a repeated row's 32 lanes
    // collect the coefficients of its slots, each lane in slot order, then a fixed-order sum
    if (a.y) {
      for (int ps = 0; ps < passes; ++ps) {
        const int t = ps * RPP * G + g * RPP + hw;
        if (t < eta && yo[ps * RPP + hw]) {  // uniform over the row's 32 lanes
          const int i = il[ps * RPP + hw];
          int cnt = 0;
          if (p == 0) cnt = __hip_atomic_exchange(a.ycnt + i, 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          cnt = __shfl(cnt, lane & 32);
          T sc = T(0);
          if (cnt == 1) {
            if (p == 0) sc = cl[ps * RPP + hw];
          } else {
            for (int u = p; u < eta; u += 32)
              if (tk[u] == i) sc += ld_ag(a.cy + u);
          }
          sc = sum32(sc);
          if (p == 0) st_ag(a.y + i, ld_ag(a.y + i) - sc);
        }
      }
    }

    if (eb > 0) {
      const int e = eb - kEBias;
      // B. integer accumulation
      for (int ps = 0; ps < passes; ++ps) {
        const int t = ps * RPP * G + g * RPP + hw;
        if (t < eta) {
          const int i = il[ps * RPP + hw];
          const T c = cl[ps * RPP + hw];
          const int64_t r0 = a.row_ptr[i], r1 = a.row_ptr[i + 1];
          for (int64_t q = r0 + p; q < r1; q += 32) {
            const long long v = (long long)llrint(ldexp((double)(c * a.val[q]), 40 - e));
            __hip_atomic_fetch_add(a.acc + a.col[q], v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      if (!grid_sync(a.bar, ++nbar, G)) { stop_code = ST_ABORTED; break; }
      // C. apply each touched column once
      for (int ps = 0; ps < passes; ++ps) {
        const int t = ps * RPP * G + g * RPP + hw;
        if (t < eta) {
          const int i = il[ps * RPP + hw];
          const int64_t r0 = a.row_ptr[i], r1 = a.row_ptr[i + 1];
          for (int64_t q = r0 + p; q < r1; q += 32) {
            const int j = a.col[q];
            const long long tot = __hip_atomic_exchange(a.acc + j, 0ll, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (tot != 0) {
              const T z = (T)((double)ld_ag(a.x_star + j) - ldexp((double)tot, e - 40));
              st_ag(a.x_star + j, z);
              st_ag(a.x + j, shrink(z, a.lambda));
            }
          }
        }
      }
    } else {
      ++nbar;  // keep the barrier count of the skipped accumulation phase
      if (!grid_sync(a.bar, nbar, G)) { stop_code = ST_ABORTED; break; }
    }
    if (!grid_sync(a.bar, ++nbar, G)) { stop_code = ST_ABORTED; break; }
    k_done = k + 1;

    if (a.xref && a.check_every > 0 && (k + 1) % a.check_every == 0) {
      const unsigned mtag = (unsigned)((k + 1) / a.check_every);
      double e2 = 0.0, r2s = 0.0;
      for (int64_t j = j0 + tid; j < j1; j += kGridThreads) {
        const double rf = (double)a.xref[j];
        const double d = (double)ld_ag(a.x + j) - rf;
        e2 += d * d;
        r2s += rf * rf;
      }
      e2 = wave_sum(e2);
      r2s = wave_sum(r2s);
      if (lane == 0) { mon[2 * wave] = e2; mon[2 * wave + 1] = r2s; }
      __syncthreads();
      if (tid == 0) {
        double se = 0.0, sr = 0.0;
        for (int w = 0; w < kGridThreads / 64; ++w) { se += mon[2 * w]; sr += mon[2 * w + 1]; }
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
          mon[2 * (kGridThreads / 64)] = err;
        }
      }
      if (lerr) set_status(a.status, lerr);
      if (__syncthreads_or(lerr)) { stop_code = ST_ABORTED; break; }
      if (a.tol > 0.0 && mon[2 * (kGridThreads / 64)] <= a.tol) break;
    }
  }
  if (stop_code > 0 && tid == 0) set_status(a.status, stop_code);
  if (g == 0 && tid == 0) a.status[1] = (int)k_done;
}

template <typename T>
int csr_grid_max_resident() {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void*)&rska_csr_grid<T>, kGridThreads, 0) !=
      hipSuccess)
    return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

template <typename T>
hipError_t launch_csr_grid(CsrArgs<T>& a, hipStream_t stream) {
  if (a.G < 1 || a.G > csr_grid_max_resident<T>()) return hipErrorCooperativeLaunchTooLarge;
  void* args[] = {&a};
  return launch_persistent((const void*)&rska_csr_grid<T>, dim3(a.G), dim3(kGridThreads), args, 0, stream);
}

template int csr_grid_max_resident<float>();
template int csr_grid_max_resident<double>();
template hipError_t launch_csr_grid<float>(CsrArgs<float>&, hipStream_t);
template hipError_t launch_csr_grid<double>(CsrArgs<double>&, hipStream_t);

}  // namespace rsk
