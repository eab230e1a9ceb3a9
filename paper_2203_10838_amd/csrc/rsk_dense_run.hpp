// Per-workgroup code of the general dense RSKA kernel (eq. (rska) /
// Algorithm 1), shared by the single-system and the batched launches.
#pragma once
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

// Chunk [col, col+VEC) of a row with the elements at or past n set to zero.
// The load itself is always a whole aligned vector (VEC > 1 requires a 16-byte
// aligned A and ld a multiple of VEC), so it never leaves the 16-byte block
// that holds element col; the elements past n are discarded by a select.
template <typename T, int VEC>
__device__ __forceinline__ Vec<T, VEC> load_vec(const T* __restrict__ rowp, int64_t col, int64_t n) {
  Vec<T, VEC> v;
  load_global_vec<T, VEC>(rowp + col, v.v);
  if constexpr (VEC > 1) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) v.v[e] = col + e < n ? v.v[e] : T(0);
  }
  return v;
}

// Chunk v of a row read from LDS, columns [col, col+VEC) relative to the
// slice: the elements at or past nrel (past n) set to zero, as load_vec does.
template <typename T, int VEC>
__device__ __forceinline__ void mask_tail(Vec<T, VEC>& v, int64_t col, int64_t nrel) {
#pragma unroll
  for (int e = 0; e < VEC; ++e) v.v[e] = col + e < nrel ? v.v[e] : T(0);
}

// One-hop gather: the n_slots tagged partials of a step (slot s = q*eta + t)
// into LDS, thread `tid` of `nt` taking slots tid, tid+nt, ... (at most 16
// words, i.e. 16 float or 8 double slots). All of a thread's slots are loaded
// before any is checked.
template <typename T>
__device__ __forceinline__ void poll_flat(const u64* xP, int n_slots, int tid, int nt, unsigned tag, T* out,
                                          int& err) {
  constexpr int W = Words<T>::N;
  constexpr int N = 16 / W;
  unsigned pending = 0;
#pragma unroll
  for (int j = 0; j < N; ++j)
    if (tid + j * nt < n_slots) pending |= 1u << j;
  if (err) return;
  unsigned spins = 0;
  while (pending) {
    u64 w[N][W];
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int i = 0; i < W; ++i)
        w[j][i] = ((pending >> j) & 1u) ? xload(xP + (size_t)(tid + j * nt) * W + i) : 0ull;
#pragma unroll
    for (int j = 0; j < N; ++j) {
      if (!((pending >> j) & 1u)) continue;
      bool ok = true;
#pragma unroll
      for (int i = 0; i < W; ++i) ok = ok && (unsigned)(w[j][i] >> 32) == tag;
      if (!ok) continue;
      if constexpr (W == 1) {
        out[tid + j * nt] = __uint_as_float((unsigned)w[j][0]);
      } else {
        out[tid + j * nt] = __longlong_as_double((long long)((w[j][1] << 32) | (w[j][0] & 0xffffffffull)));
      }
      pending &= ~(1u << j);
    }
    if (!pending) break;
    if (++spins > kSpinLimit) { err = ST_ABORTED; break; }
    __builtin_amdgcn_s_sleep(1);
  }
}

// Butterfly sums within aligned groups of `width` lanes (a power of two <= 64)
// without the LDS crossbar: DPP quad permutes for offsets 1 and 2, the row
// half-mirror and row mirror for 4 and 8 (each pairs a lane with one of the
// other, already uniform, half-group), and the gfx950 permlane16/32 swaps for
// 16 and 32 (the two swapped outputs are the lane's own and its partner's
// value). Every lane of a group ends with the same, fixed-order sum.
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
  return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
  return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = dpp_i<CTRL>((int)b), hi = dpp_i<CTRL>((int)(b >> 32));
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ float swap16_sum(float v) {
  const auto r = __builtin_amdgcn_permlane16_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ float swap32_sum(float v) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_int(v), __float_as_int(v), false, false);
  return __int_as_float(r[0]) + __int_as_float(r[1]);
}
__device__ __forceinline__ double join_d(int lo, int hi) {
  return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
}
__device__ __forceinline__ double swap16_sum(double v) {
  const long long b = __double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane16_swap((int)b, (int)b, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap((int)(b >> 32), (int)(b >> 32), false, false);
  return join_d(l[0], h[0]) + join_d(l[1], h[1]);
}
__device__ __forceinline__ double swap32_sum(double v) {
  const long long b = __double_as_longlong(v);
  const auto l = __builtin_amdgcn_permlane32_swap((int)b, (int)b, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap((int)(b >> 32), (int)(b >> 32), false, false);
  return join_d(l[0], h[0]) + join_d(l[1], h[1]);
}
template <typename T>
__device__ __forceinline__ T lane_sum(T v, int width) {
  if (width > 1) v += dpp_move<0xB1>(v);   // quad_perm [1,0,3,2]
  if (width > 2) v += dpp_move<0x4E>(v);   // quad_perm [2,3,0,1]
  if (width > 4) v += dpp_move<0x141>(v);  // row_half_mirror
  if (width > 8) v += dpp_move<0x140>(v);  // row_mirror
  if (width > 16) v = swap16_sum(v);
  if (width > 32) v = swap32_sum(v);
  return v;
}

// c_t = (alpha_k/eta) (r_t - b_t) / ||a_t||^2 from the row's prefetched b and norm.
template <typename T>
__device__ __forceinline__ T coef_of(T s, T bt, T rn, T ak, int eta, int& zero_row) {
  if (rn == T(0)) { zero_row = 1; return T(NAN); }
  return (ak / T(eta)) * (s - bt) / rn;
}

// Wait for the partials of workgroup q for rows t0 + u*tstep (u < N, rows <
// eta) of the step tagged `tag`; all pending slots are loaded before any is
// checked, so the N round trips overlap. Lanes with !qok get zeros.
template <typename T, int N>
__device__ __forceinline__ void wait_rows(const u64* xP, int eta, int q, bool qok, int t0, int tstep, unsigned tag,
                                          T (&v)[N], int& err) {
  constexpr int W = Words<T>::N;
  unsigned pending = 0;
#pragma unroll
  for (int u = 0; u < N; ++u) {
    v[u] = T(0);
    if (qok && t0 + u * tstep < eta) pending |= 1u << u;
  }
  if (err) return;
  unsigned spins = 0;
  while (pending) {
    u64 w[N][W];
#pragma unroll
    for (int u = 0; u < N; ++u)
#pragma unroll
      for (int i = 0; i < W; ++i)
        w[u][i] = ((pending >> u) & 1u) ? xload(xP + ((size_t)q * eta + t0 + u * tstep) * W + i) : 0ull;
#pragma unroll
    for (int u = 0; u < N; ++u) {
      if (!((pending >> u) & 1u)) continue;
      bool ok = true;
#pragma unroll
      for (int i = 0; i < W; ++i) ok = ok && (unsigned)(w[u][i] >> 32) == tag;
      if (!ok) continue;
      if constexpr (W == 1) {
        v[u] = __uint_as_float((unsigned)w[u][0]);
      } else {
        v[u] = __longlong_as_double((long long)((w[u][1] << 32) | (w[u][0] & 0xffffffffull)));
      }
      pending &= ~(1u << u);
    }
    if (!pending) break;
    if (++spins > kSpinLimit) { err = ST_ABORTED; break; }
    __builtin_amdgcn_s_sleep(1);
  }
}

// One workgroup's part of a dense solve: rank g of the a.G workgroups that
// share the system, owning column slice `slice`. The single-system kernel
// calls it once per workgroup, the batched kernel once per (system, rank)
// ticket. With a.G == 1 the exchange stays in LDS.
//
// Latency. A step is a chain of dependent memory round trips, so each phase
// keeps many of them in flight: a lane loads the chunks of U rows before it
// uses any, a wave polls the partials of UR rows at once, and the next step's
// indices, b and ||a||^2 are fetched while the current step runs (into the
// second of two LDS buffers). The row sample of every step is known in
// advance (it does not depend on x), so with the pipelined tile (PIPE, for
// a.tile_cache == 2) the next step's rows are loaded into registers while the
// step runs on the LDS tile of its own rows, and written to the other tile at
// its end: no HBM round trip is left on a step's critical path but the
// exchange's. The indices are then fetched two steps ahead. None of this
// changes any summation order: the pipelined tile gives the same bits as the
// single one. PIPE is a template argument so that the other variant's
// register loads never share a code path with it (the compiler would wait for
// them, and with them for the prefetch, where the paths join).
template <typename T, int VEC, int NT, bool PIPE>
__device__ __forceinline__ void dense_run(const DenseArgs<T>& a, const int g, const int slice, unsigned char* smem) {
  using V = Vec<T, VEC>;
  constexpr int NW = NT / 64;
  constexpr int W = Words<T>::N;
  constexpr int U = 8, UR = 4, PF = 4;
  constexpr int QU = VEC == 1 ? 2 : 1;  // chunks per row a lane loads together
  const int G = a.G, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int eta = a.eta;
  const bool solo = G == 1;
  const bool pf_regs = eta <= PF * NT;

  DenseSmem L(sizeof(T), VEC, a.wq_max, eta, NT, a.tile_cache, a.two_hop ? 0 : onehop_lds_elems(G, eta));
  T* xs = reinterpret_cast<T*>(smem + L.xs);
  T* xv = reinterpret_cast<T*>(smem + L.xv);
  T* cs = reinterpret_cast<T*>(smem + L.cs);
  int* taub = reinterpret_cast<int*>(smem + L.tau);
  T* bqb = reinterpret_cast<T*>(smem + L.bq);
  T* rqb = reinterpret_cast<T*>(smem + L.rq);
  V* red = reinterpret_cast<V*>(smem + L.red);
  double* mon = reinterpret_cast<double*>(smem + L.flags);
  static_assert((2 * NW + 1) * sizeof(double) <= 96, "monitor words overlap the block-OR words");
  int* orA = reinterpret_cast<int*>(smem + L.flags + 96);   // after the exchange: 1 aborted, 2 non-finite
  int* orB = orA + 2;                                        // end of step: 4 bad index in the next step
  V* tile = reinterpret_cast<V*>(smem + L.tile);
  T* xr = reinterpret_cast<T*>(smem + L.xr);
  constexpr bool pipe = PIPE && VEC * sizeof(T) == 16;
  constexpr int PR = pipe_reg_chunks(sizeof(T));
  const size_t tslots = (size_t)eta * a.wq_max;  // chunks of one pipelined tile

  const int64_t q0 = (int64_t)slice * a.nchunks / G, q1 = (int64_t)(slice + 1) * a.nchunks / G;
  const int wq = (int)(q1 - q0);
  const int64_t c0 = q0 * VEC;
  const int wcols = wq * VEC;
  const bool ragged = c0 + wcols > a.n;  // the last chunk holds columns past n

  // pipelined tile: chunk e = t*wq + q of row tsrc[t] of this slice, thread tid taking
  // e = tid + p*NT (coalesced: consecutive threads read consecutive chunks of a row); whole
  // 16-byte chunks, the columns past n masked where the tile is read. Every thread issues all
  // PR loads, unconditionally, so that they leave back to back
  auto load_tile = [&](const int* tsrc, V (&nv)[PR]) {
    const int total = eta * wq;
#pragma unroll
    for (int p = 0; p < PR; ++p) {
      // past the tile: its last chunk again (unused)
      const int e = tid + p * NT < total ? tid + p * NT : total - 1;
      const int t = e / wq, q = e - t * wq;
      load_global_vec<T, VEC>(a.A + (int64_t)tsrc[t] * a.ld + c0 + (int64_t)q * VEC, nv[p].v);
    }
  };
  auto store_tile = [&](V* dst, const V (&nv)[PR]) {
    const int total = eta * wq;
#pragma unroll
    for (int p = 0; p < PR; ++p) {
      const int e = tid + p * NT;
      if (e < total) dst[e] = nv[p];
    }
  };

  // x*_0, x_0 = S_lambda(x*_0)
  for (int j = tid; j < wcols; j += NT) {
    const int64_t c = c0 + j;
    T z = (a.warm && c < a.n) ? a.x_star[c] : T(0);
    xs[j] = z;
    xv[j] = shrink(z, a.lambda);
  }
  // rows of step 0 (an index outside [0, m) is reported at that step and never dereferenced)
  int row_err = 0;
  if (a.K > 0) {
    for (int t = tid; t < eta; t += NT) {
      const int i = load_global(a.idx + t);
      const bool ok = i >= 0 && (int64_t)i < a.m;
      if (!ok) row_err = ST_INDEX;
      const int ic = ok ? i : 0;
      taub[t] = ic;
      bqb[t] = load_global(a.b + ic);
      rqb[t] = weighted_rn(a.r2, a.row_w, ic);
    }
  }
  // pipelined: the indices of step 1 as well (its rows, b and ||a||^2 follow during step 0)
  int row_err1 = 0;
  if (pipe && a.K > 1) {
    for (int t = tid; t < eta; t += NT) {
      const int i = load_global(a.idx + eta + t);
      const bool ok = i >= 0 && (int64_t)i < a.m;
      if (!ok) row_err1 = ST_INDEX;
      taub[eta + t] = ok ? i : 0;
    }
  }

  const int lpr = a.lpr, rpw = 64 / lpr;
  const int rs = lane / lpr, cl = lane % lpr;
  const int rstride = NW * rpw;
  int64_t k_done = 0;
  int stop_code = 0;
  if (tid < 4) orA[tid] = 0;  // orA[0..1] and orB[0..1]
  // step 0's rows were fetched above; every workgroup checks all of them (this barrier also
  // orders the clearing of the flag words)
  int row_bad = __syncthreads_or(row_err);
  int row_bad1 = pipe ? __syncthreads_or(row_err1) : 0;  // pipelined: the next step's verdict
  if (pipe && a.K > 0 && !row_bad) {
    V nv[PR];
    load_tile(taub, nv);
    store_tile(tile, nv);
    __syncthreads();
  }

  for (int64_t k = 0; k < a.K; ++k) {
    const unsigned tag = (unsigned)(k + 1);
    const T ak = a.alpha_k ? a.alpha_k[k] : a.alpha;
    const int buf = (int)(k & 1);
    const int* tau = taub + (pipe ? (int)(k % 3) : buf) * eta;
    const V* tcur = tile + (size_t)buf * tslots;  // pipelined: this step's tile
    // chunk q of the step's row t: from the tile (masked past n when pipelined) or from HBM
    auto tile_at = [&](int t, int q) -> V {
      if (pipe) {
        V v = tcur[(size_t)t * wq + q];
        if (ragged && q == wq - 1) mask_tail<T, VEC>(v, (int64_t)q * VEC, a.n - c0);
        return v;
      }
      return a.tile_cache ? tile[(size_t)t * wq + q]
                          : load_vec<T, VEC>(a.A + (int64_t)tau[t] * a.ld + c0, (int64_t)q * VEC, a.n - c0);
    };
    const T* bq = bqb + buf * eta;
    const T* rq = rqb + buf * eta;
    // partials are double-buffered by step parity: with every workgroup
    // reducing every row, a fast workgroup may publish step k+1 while a slow
    // one still reads step k
    u64* xP = a.xP + (size_t)(k & 1) * G * eta * W;
    int lerr = 0;

    // 1. the step's rows were fetched in the previous step; every workgroup
    //    checks all of them, so a bad index stops every workgroup at this step
    if (row_bad) { stop_code = ST_INDEX; break; }
    const bool has_next = k + 1 < a.K;
    const int32_t* tk1 = a.idx + (k + 1) * (int64_t)eta;
    const bool has_next2 = k + 2 < a.K;
    int ni[PF];
    T nb[PF], nr[PF];
    V nv[PR];  // pipelined: the next step's chunks of this slice
    if (pipe) {
      // the next step's rows, b and ||a||^2 (its indices were checked a step ago) and the raw
      // indices of the step after it, all into registers: nothing waits for them before the
      // step's end
      // (every lane loads, the rows past eta as row eta-1: straight-line loads, which the
      // compiler does not guard with waits for earlier ones)
      if (has_next) {
        const int* t1 = taub + (int)((k + 1) % 3) * eta;
        load_tile(t1, nv);
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          const int t = tid + p * NT < eta ? tid + p * NT : eta - 1;
          nb[p] = load_global(a.b + t1[t]);
          nr[p] = weighted_rn(a.r2, a.row_w, t1[t]);
        }
      }
      if (has_next2) {
        const int32_t* tk2 = a.idx + (k + 2) * (int64_t)eta;
#pragma unroll
        for (int p = 0; p < PF; ++p) ni[p] = load_global(tk2 + (tid + p * NT < eta ? tid + p * NT : eta - 1));
      }
    } else if (pf_regs && has_next) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int t = tid + p * NT;
        ni[p] = t < eta ? load_global(tk1 + t) : 0;
      }
    }

    // 2. partial dots over the own columns: every lane issues the loads of
    //    U rows x QU chunks before it uses any (rows past eta load a valid
    //    row and are discarded), so a batch costs one memory round trip
    if (pipe) {
      // the tile is in LDS: lane group rs of a wave takes U rows at once, its lpr lanes the
      // chunks of each in ascending order (the order of the loads from HBM below)
      for (int tb = wave * rpw; tb < eta; tb += rstride * U) {
        T acc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) acc[u] = T(0);
        for (int q = cl; q < wq; q += lpr) {
          V v[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int t = tb + u * rstride + rs;
            v[u] = tile_at(t < eta ? t : eta - 1, q);
          }
          const V xx = reinterpret_cast<const V*>(xv)[q];
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (tb + u * rstride + rs < eta) {
#pragma unroll
              for (int e = 0; e < VEC; ++e) acc[u] += v[u].v[e] * xx.v[e];
            }
        }
        T sum[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sum[u] = lane_sum(acc[u], lpr);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = tb + u * rstride + rs;
          if (t < eta && cl == 0) cs[t] = sum[u];
        }
      }
    } else if (eta <= rstride) {
      // at most one row per lane group: keep 8 chunks of that row in flight instead
      constexpr int QC = 8;
      const int t = wave * rpw + rs;
      if (t < eta) {
        const T* rowp = a.A + (int64_t)tau[t] * a.ld + c0;
        T acc = T(0);
        for (int qb = cl; qb < wq; qb += lpr * QC) {
          V v[QC];
#pragma unroll
          for (int h = 0; h < QC; ++h) {
            const int q = qb + h * lpr < wq ? qb + h * lpr : wq - 1;
            v[h] = load_vec<T, VEC>(rowp, (int64_t)q * VEC, a.n - c0);
          }
#pragma unroll
          for (int h = 0; h < QC; ++h) {
            const int q = qb + h * lpr;
            if (q < wq) {
              if (a.tile_cache) tile[(size_t)t * wq + q] = v[h];
              const V xx = reinterpret_cast<const V*>(xv)[q];
#pragma unroll
              for (int e = 0; e < VEC; ++e) acc += v[h].v[e] * xx.v[e];
            }
          }
        }
        acc = lane_sum(acc, lpr);
        if (cl == 0) cs[t] = acc;
      }
    } else {
      for (int tb = wave * rpw; tb < eta; tb += rstride * U) {
        T acc[U];
        const T* rowp[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
          acc[u] = T(0);
          const int t = tb + u * rstride + rs;
          rowp[u] = a.A + (int64_t)tau[t < eta ? t : eta - 1] * a.ld + c0;
        }
        for (int qb = cl; qb < wq; qb += lpr * QU) {
          V v[QU][U];
#pragma unroll
          for (int h = 0; h < QU; ++h) {
            const int q = qb + h * lpr < wq ? qb + h * lpr : wq - 1;
#pragma unroll
            for (int u = 0; u < U; ++u) v[h][u] = load_vec<T, VEC>(rowp[u], (int64_t)q * VEC, a.n - c0);
          }
#pragma unroll
          for (int h = 0; h < QU; ++h) {
            const int q = qb + h * lpr;
            if (q < wq) {
              const V xx = reinterpret_cast<const V*>(xv)[q];
#pragma unroll
              for (int u = 0; u < U; ++u) {
                const int t = tb + u * rstride + rs;
                if (t < eta) {
                  if (a.tile_cache) tile[(size_t)t * wq + q] = v[h][u];
#pragma unroll
                  for (int e = 0; e < VEC; ++e) acc[u] += v[h][u].v[e] * xx.v[e];
                }
              }
            }
          }
        }
        T sum[U];
#pragma unroll
        for (int u = 0; u < U; ++u) sum[u] = lane_sum(acc[u], lpr);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int t = tb + u * rstride + rs;
          if (t < eta && cl == 0) cs[t] = sum[u];
        }
      }
    }
    // publish the partials in one coalesced pass: on this architecture a
    // store holds the in-order memory counter until it is acknowledged, so
    // one pass costs one store latency where a store per row costs one each
    if (!solo) {
      __syncthreads();
      for (int t = tid; t < eta; t += NT) put_tagged(&xP[((size_t)g * eta + t) * W], cs[t], tag);
    }

    // 2b. b and ||a||^2 of the next step's rows (indices checked first)
    int next_err = 0;
    if (!pipe && pf_regs && has_next) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        const int t = tid + p * NT;
        if (t < eta) {
          const bool ok = ni[p] >= 0 && (int64_t)ni[p] < a.m;
          if (!ok) next_err = ST_INDEX;
          ni[p] = ok ? ni[p] : 0;
          nb[p] = load_global(a.b + ni[p]);
          nr[p] = weighted_rn(a.r2, a.row_w, ni[p]);
        }
      }
    }

    // 3./4. all-reduce of the partials, coefficients into cs[]
    int zero_row = 0;
    if (solo) {
      __syncthreads();
      for (int t = tid; t < eta; t += NT) cs[t] = coef_of(cs[t], bq[t], rq[t], ak, eta, zero_row);
    } else if (!a.two_hop) {
      // every workgroup gathers all G*eta partials in one round, then sums
      // each row in a fixed order: segments of kOneHopSeg workgroups in
      // ascending q (loads unrolled), then the segment sums in ascending order
      poll_flat<T>(xP, G * eta, tid, NT, tag, xr, lerr);
      __syncthreads();
      constexpr int SG = kOneHopSeg;
      const int nseg = (G + SG - 1) / SG;
      T* part = xr + G * eta;
      for (int p = tid; p < eta * nseg; p += NT) {
        const int t = p % eta, q0 = (p / eta) * SG;
        T v[SG];
#pragma unroll
        for (int u = 0; u < SG; ++u) v[u] = q0 + u < G ? xr[(q0 + u) * eta + t] : T(0);
        T sum = T(0);
#pragma unroll
        for (int u = 0; u < SG; ++u)
          if (q0 + u < G) sum += v[u];
        part[p] = sum;
      }
      __syncthreads();
      for (int t = tid; t < eta; t += NT) {
        T sum = T(0);
        for (int j0 = 0; j0 < nseg; j0 += SG) {
          T v[SG];
#pragma unroll
          for (int u = 0; u < SG; ++u) v[u] = j0 + u < nseg ? part[(j0 + u) * eta + t] : T(0);
#pragma unroll
          for (int u = 0; u < SG; ++u)
            if (j0 + u < nseg) sum += v[u];
        }
        cs[t] = coef_of(sum, bq[t], rq[t], ak, eta, zero_row);
      }
    } else {
      for (int tb = g + wave * G; tb < eta; tb += NW * G * UR) {
        T part[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) part[u] = T(0);
        for (int qb = 0; qb < G; qb += 64) {
          T v[UR];
          wait_rows<T, UR>(xP, eta, qb + lane, qb + lane < G, tb, NW * G, tag, v, lerr);
#pragma unroll
          for (int u = 0; u < UR; ++u) part[u] += v[u];
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
          const T sum = lane_sum(part[u], 64);
          const int t = tb + u * NW * G;
          if (lane == 0 && t < eta) {
            const T c = coef_of(sum, bq[t], rq[t], ak, eta, zero_row);
            if (zero_row) set_status(a.status, ST_ZERO_ROW);
            put_tagged(&a.xC[(size_t)t * W], c, tag);
          }
        }
      }
      for (int t = tid; t < eta; t += NT) cs[t] = wait_tagged<T>(&a.xC[(size_t)t * W], tag, lerr);
    }
    if (zero_row) set_status(a.status, ST_ZERO_ROW);
    // every path above wrote cs[t] for t = tid, tid + NT, ...: each thread checks its own
    int bad = 0;
    for (int t = tid; t < eta; t += NT) bad |= !isfinite(cs[t]);
    if (lerr) set_status(a.status, lerr);
    // one barrier publishes cs[] and agrees on an expired wait or a non-finite coefficient
    const int fl = block_or(orA, (lerr ? 1 : 0) | (bad ? 2 : 0), k);
    if (fl) { stop_code = (fl & 1) ? ST_ABORTED : ST_NONFINITE; break; }

    // the dual (x* = A^T y): float atomics, so a row drawn twice in a step adds in either order
    if (a.y && g == 0)
      for (int t = tid; t < eta; t += NT) atomicAdd(&a.y[tau[t]], -cs[t]);

    // 5. transposed update of the own columns, fused with S_lambda; rows in
    //    ascending order, the chunks of UB rows loaded before they are used
    constexpr int UB = 8;
    if (wq <= NT) {
      const int nrg = NT / wq, rg = tid / wq, q = tid % wq;
      if (rg < nrg) {
        V acc;
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc.v[e] = T(0);
        for (int tb = rg; tb < eta; tb += nrg * UB) {
          V v[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const int t = tb + u * nrg < eta ? tb + u * nrg : eta - 1;
            v[u] = tile_at(t, q);
          }
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const int t = tb + u * nrg;
            if (t < eta) {
              const T c = cs[t];
#pragma unroll
              for (int e = 0; e < VEC; ++e) acc.v[e] += c * v[u].v[e];
            }
          }
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
        for (int tb = 0; tb < eta; tb += UB) {
          V v[UB];
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            const int t = tb + u < eta ? tb + u : eta - 1;
            v[u] = tile_at(t, q);
          }
#pragma unroll
          for (int u = 0; u < UB; ++u) {
            if (tb + u < eta) {
              const T c = cs[tb + u];
#pragma unroll
              for (int e = 0; e < VEC; ++e) d.v[e] += c * v[u].v[e];
            }
          }
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
    // next step's rows into the other buffer (last read by the previous
    // step, which ended at a barrier)
    if (pipe) {
      if (has_next) {
        store_tile(tile + (size_t)(buf ^ 1) * tslots, nv);
        T* bn = bqb + (buf ^ 1) * eta;
        T* rn = rqb + (buf ^ 1) * eta;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          const int t = tid + p * NT;
          if (t < eta) { bn[t] = nb[p]; rn[t] = nr[p]; }
        }
      }
      if (has_next2) {
        // the indices of step k+2, checked (their verdict is agreed below), into the buffer
        // that held those of step k-1
        int* tn = taub + (int)((k + 2) % 3) * eta;
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          const int t = tid + p * NT;
          if (t < eta) {
            const bool ok = ni[p] >= 0 && (int64_t)ni[p] < a.m;
            if (!ok) next_err = ST_INDEX;
            tn[t] = ok ? ni[p] : 0;
          }
        }
      }
      // every prefetch has landed (the stores above used them); said explicitly, so that the
      // next step's prefetch, whose loads are conditional, is not made to wait for this one's
      __builtin_amdgcn_s_waitcnt(0);
    } else if (has_next) {
      int* tn = taub + (buf ^ 1) * eta;
      T* bn = bqb + (buf ^ 1) * eta;
      T* rn = rqb + (buf ^ 1) * eta;
      if (pf_regs) {
#pragma unroll
        for (int p = 0; p < PF; ++p) {
          const int t = tid + p * NT;
          if (t < eta) { tn[t] = ni[p]; bn[t] = nb[p]; rn[t] = nr[p]; }
        }
      } else {
        for (int t = tid; t < eta; t += NT) {
          const int i = load_global(tk1 + t);
          const bool ok = i >= 0 && (int64_t)i < a.m;
          if (!ok) next_err = ST_INDEX;
          const int ic = ok ? i : 0;
          tn[t] = ic;
          bn[t] = load_global(a.b + ic);
          rn[t] = weighted_rn(a.r2, a.row_w, ic);
        }
      }
    }
    // columns past n inside the last chunk stay zero: their tile entries are zero; the
    // barrier agrees on a bad index among the next step's rows
    const int nbad = block_or(orB, next_err ? 4 : 0, k) & 4;
    if (pipe) {
      row_bad = row_bad1;  // checked a step ago
      row_bad1 = nbad;
    } else {
      row_bad = nbad;
    }
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
      e2 = lane_sum(e2, 64);
      r2s = lane_sum(r2s, 64);
      if (lane == 0) { mon[2 * wave] = e2; mon[2 * wave + 1] = r2s; }
      __syncthreads();
      if (solo) {
        if (tid == 0) {
          double se = 0.0, sr = 0.0;
          for (int w = 0; w < NW; ++w) { se += mon[2 * w]; sr += mon[2 * w + 1]; }
          const double err = sr > 0.0 ? sqrt(se / sr) : sqrt(se);
          if (a.err_hist) a.err_hist[mtag - 1] = err;
          mon[2 * NW] = err;
        }
      } else {
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
          se = lane_sum(se, 64);
          sr = lane_sum(sr, 64);
          if (lane == 0) {
            const double err = sr > 0.0 ? sqrt(se / sr) : sqrt(se);
            if (g == 0 && a.err_hist) a.err_hist[mtag - 1] = err;
            mon[2 * NW] = err;
          }
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
  // nothing of this task stays in flight: the caller may reuse the LDS and the registers for
  // its next task (the compiler then need not guard the next task's writes with waits)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

}  // namespace rsk
