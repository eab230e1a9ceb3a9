// Dense RSKA, float32, register-tile persistent kernel (the throughput path).
//
// Same iteration and exchange protocol as rska_dense_persistent, laid out for
// HBM streaming on gfx950:
//  * NT threads per workgroup (1024, or 512 for eta > 768), one workgroup per
//    CU. The G workgroups form RG row groups of G/RG column slices: the
//    workgroup of slice s and group h owns the slice's x (at most 4*RG*CPL
//    float4 chunks, whole 64-byte units) and reads the slice of the rows
//    h*etaR .. (h+1)*etaR - 1 of each step, etaR = ceil(eta/RG). Wider
//    slices (RG = 2) make longer contiguous pieces of each row, which HBM
//    serves faster; the RG workgroups of a slice then add their parts of the
//    update in a third exchange hop, in a fixed order, so that they keep
//    identical copies of x.
//  * With RL = 16/RG, lane l of wave w holds group row p*(NT/64)*RL + RL*w +
//    (l % RL) of pass p and chunks q = (l / RL) + 4*RG*r, r < CPL. The RL
//    lanes that hold one chunk column are adjacent, so the column sums of the
//    update reduce with DPP adds within a row; the lanes that hold one row
//    reduce with swaps.
//  * All RP*CPL float4 loads of a step are issued before the first is used
//    (up to 20 KB in flight per CU). The addresses never depend on a
//    predicate: a chunk outside the slice is clamped into the row and meets a
//    zero x entry in the dot, and its column sum is discarded.
//  * The step's tile stays in VGPRs from the dots to the transposed update:
//    A is read from HBM exactly once per step.
//  * The first NPF (pass, chunk) slots of the next step's tile (up to 144 KB
//    a workgroup; all slots for tiles that fit) are loaded straight into LDS
//    (global_load_lds, no VGPRs) by the waves that take no part in the
//    exchange, while the exchange runs; the next step reads them from LDS, so
//    only the other slots load from HBM on the step's critical path.
//  * Each pass publishes its partial dots as soon as its own loads have
//    landed; the next step's indices, and b and ||a||^2 of the rows this
//    workgroup reduces, are fetched a step ahead.
//  * Summation orders are fixed, so x* and x are bitwise reproducible (the
//    optional dual y is summed with atomics: reproducible to rounding).
#include "rsk_device.hpp"
#include "rsk_kernels.hpp"

namespace rsk {

namespace {

constexpr int kMaxG = 256;  // workgroups the exchange code is unrolled for (4 slots per lane)

__device__ __forceinline__ float dot4(float4 a, float4 b) {
  float s = a.x * b.x;
  s += a.y * b.y;
  s += a.z * b.z;
  s += a.w * b.w;
  return s;
}

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

// Sum over aligned groups of RL adjacent lanes (RL = 16: a DPP row; 8: half a
// row); every lane of the group gets the sum.
template <int RL>
__device__ __forceinline__ float lanes_sum(float v) {
  if constexpr (RL == 16) {
    v += dpp<0x128>(v);  // row_ror:8
    v += dpp<0x124>(v);  // row_ror:4
    v += dpp<0x122>(v);  // row_ror:2
    v += dpp<0x121>(v);  // row_ror:1
  } else {
    static_assert(RL == 8, "row groups of 16 or 8 lanes");
    v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
    v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
    v += dpp<0x141>(v);  // row_half_mirror: quad 0 <-> quad 1 of each half row
  }
  return v;
}

}  // namespace

template <int NT, int RP, int CPL, int RG>
__global__ __launch_bounds__(NT) void rska_dense_rt(DenseArgs<float> a) {
  constexpr int kRtThreads = NT;
  constexpr int kRtWaves = NT / 64;
  constexpr int RL = 16 / RG;                     // rows a wave holds per pass
  constexpr int CL = 4 * RG;                      // lanes of one row
  constexpr int kRtRowsPerPass = kRtWaves * RL;
  constexpr int SW = 4 * CL * CPL;                // floats of the widest slice
  constexpr int kOwnMax = kRtOwnMax;              // rows one wave reduces per step
  constexpr int kPollWaves = RG > 1 ? (SW + 63) / 64 : 0;  // waves holding the third hop's pollers
  static_assert(kPollWaves <= kRtWaves / 2, "the pollers of the third hop do not issue the LDS prefetch");
  __shared__ float4 xs4[CL * CPL];                // x* slice
  __shared__ float4 xv4[CL * CPL];                // x slice
  __shared__ float4 red[kRtWaves][CL * CPL];      // per-wave column sums
  __shared__ float cs[RP * kRtRowsPerPass];        // step coefficients
  __shared__ double mon[2 * kRtWaves + 2];
  __shared__ int orflag[2];  // step-parity flag words of the block OR
  __shared__ int hop3_bad[2];  // step-parity: a non-finite sum of the slice's update parts
  // next-step tile slots prefetched into LDS: (p, r) with s = p * CPL + r < NPF; LDS slot s * NT + tid
  // holds tile[p][r] of thread tid. PL passes hold prefetched slots.
  constexpr int kPfBudget = 147456 / (NT * 16);
  // (1024-thread tiles wider than 12 slots leave no registers for the prefetch loop)
  constexpr int NPF = (NT == 1024 && RP * CPL > 12) ? 0 : (RP * CPL < kPfBudget ? RP * CPL : kPfBudget);
  constexpr int PL = (NPF + CPL - 1) / CPL;
  // s_waitcnt immediate with vmcnt = kHbmSlots (bits 3:0 and 15:14), expcnt and lgkmcnt not waited on
  constexpr int kHbmSlots = RP * CPL - NPF;
  static_assert(kHbmSlots < 64, "vmcnt holds at most 63");
  constexpr int kWaitPrefetch = (kHbmSlots & 15) | ((kHbmSlots >> 4) << 14) | (7 << 4) | (15 << 8);
  // When the LDS prefetch holds the whole next tile, it is issued after the first exchange hop
  // instead of under it: the hop's polls then do not queue behind the prefetch's HBM reads, and
  // the prefetch still lands under the second hop and the update (measured on 100000 x 20000:
  // eta = 16, 64 and 256 steps 7-10% shorter). With slots left to load from HBM the prefetch
  // needs the whole exchange to hide it, and is issued right after the dots.
  constexpr bool kPfAfterHop1 = kHbmSlots == 0;
  __shared__ float4 pf[NPF > 0 ? NPF * NT : 1];
  __shared__ int nrow[PL > 0 ? PL * kRtRowsPerPass : 1];  // rows of the passes holding prefetched slots

  const int g = blockIdx.x, G = a.G, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int eta = a.eta;
  const int sl = lane / RL, ri = lane % RL;

  // column slice s of C = G / RG and row group h (the RG workgroups of a slice are adjacent in
  // the XCD-aware order); the group's rows of a step are h * etaR .. h * etaR + etaH - 1
  const int C = G / RG;
  const int sx = xcd_slice(g, G);
  const int s = sx / RG, h = sx % RG;
  const int etaR = (eta + RG - 1) / RG;
  const int hr0 = h * etaR;
  const int etaH = hr0 >= eta ? 0 : (eta - hr0 < etaR ? eta - hr0 : etaR);
  // slice in 4-chunk (64-byte) units
  const int64_t nunits = (a.nchunks + 3) / 4;
  const int64_t u0 = (int64_t)s * nunits / C, u1 = (int64_t)(s + 1) * nunits / C;
  const int64_t q0 = u0 * 4;
  int64_t q1 = u1 * 4;
  if (q1 > a.nchunks) q1 = a.nchunks;
  const int wq = (int)(q1 - q0);
  const int64_t c0 = q0 * 4;
  // last chunk of the row reachable from this slice (clamp target)
  const int qlast = (int)(a.nchunks - 1 - q0);
  float* xs = reinterpret_cast<float*>(xs4);
  float* xv = reinterpret_cast<float*>(xv4);

  // group rows this workgroup reduces: a contiguous block (two hops) or all (one hop)
  const int per = a.two_hop ? (etaR + C - 1) / C : etaR;
  const int ot0 = a.two_hop ? s * per : 0;
  const int ot1 = (ot0 + per < etaH) ? ot0 + per : etaH;

  if (tid < 2) orflag[tid] = hop3_bad[tid] = 0;
  for (int j = tid; j < SW; j += kRtThreads) {
    const int64_t c = c0 + j;
    const float z = (a.warm && j < wq * 4 && c < a.n) ? a.x_star[c] : 0.f;
    xs[j] = z;
    xv[j] = shrink(z, a.lambda);
  }

  // Prefetched per-step inputs: the lane's rows of the step (tile rows), and
  // for the rows this wave reduces, b and ||a||^2 (over w) of the sampled rows.
  // The row indices load at fixed in-range positions with no branch, all before
  // the first is checked: a load inside a branch is waited for at once, one
  // round trip each.
  int rowi[RP];
  float ob[kOwnMax], orn[kOwnMax];
  int lerr = 0;
  auto fetch_rows = [&](int64_t k, int (&ri_out)[RP], int& err) {
    const int32_t* tk = a.idx + k * (int64_t)eta;
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const int t = p * kRtRowsPerPass + RL * wave + ri;
      ri_out[p] = tk[t < etaH ? hr0 + t : 0];
    }
    int xo[RG > 1 ? RP : 1];
    if constexpr (RG > 1) {
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const int t = p * kRtRowsPerPass + RL * wave + ri;
        const int tt = (1 - h) * etaR + t;
        xo[p] = tk[(t < etaR && tt < eta) ? tt : 0];
      }
    }
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const int t = p * kRtRowsPerPass + RL * wave + ri;
      int i = ri_out[p];
      if (t >= etaH) i = -1;
      else if (i < 0 || (int64_t)i >= a.m) { err = ST_INDEX; i = -1; }
      ri_out[p] = i;
      if constexpr (RG > 1) {
        // the other group's rows are checked too: every workgroup stops at the same step
        if (xo[p] < 0 || (int64_t)xo[p] >= a.m) err = ST_INDEX;
      }
    }
  };
  auto fetch_owned = [&](int64_t k) {
    const int32_t* tk = a.idx + k * (int64_t)eta + hr0;
#pragma unroll
    for (int j = 0; j < kOwnMax; ++j) {
      const int t = ot0 + wave + kRtWaves * j;
      ob[j] = 0.f;
      orn[j] = 1.f;
      if (lane == 0 && t < ot1) {
        const int i = tk[t];
        if (i >= 0 && (int64_t)i < a.m) { ob[j] = a.b[i]; orn[j] = weighted_rn(a.r2, a.row_w, i); }
      }
    }
  };
  if (a.K > 0) {
    fetch_rows(0, rowi, lerr);
    fetch_owned(0);
  }
  int64_t k_done = 0;
  int stop_code = 0;
  // every workgroup read the same indices, so all skip the loop alike
  if (__syncthreads_or(lerr)) stop_code = ST_INDEX;

  // LDS prefetch of slots s < NPF: the issuing waves (the upper half) load, for consumer wave j,
  // tile slot (p, r) of each of its 64 lanes; lane l of the issuing wave stands for lane l of
  // wave j, so the 64 x 16 B that one global_load_lds writes are the 64 consumers' slots in order.
  auto publish_rows = [&](const int (&rows)[RP]) {
    if constexpr (NPF > 0) {
#pragma unroll
      for (int p = 0; p < PL; ++p)
        if (sl == 0) nrow[p * kRtRowsPerPass + RL * wave + ri] = rows[p];
    }
  };
  auto issue_prefetch = [&]() {
    if constexpr (NPF > 0) {
      if (wave >= kRtWaves / 2) {
        for (int I = wave - kRtWaves / 2; I < NPF * kRtWaves; I += kRtWaves / 2) {
          const int j = I % kRtWaves, sp = I / kRtWaves, r = sp % CPL, p = sp / CPL;
          const int row = nrow[p * kRtRowsPerPass + RL * j + ri];
          const int q = sl + CL * r;
          const float* gp = a.A + (int64_t)(row < 0 ? 0 : row) * a.ld + c0 + 4 * (q < qlast ? q : qlast);
          __builtin_amdgcn_global_load_lds(gp, (__attribute__((address_space(3))) void*)&pf[(p * CPL + r) * NT + 64 * j],
                                           16, 0, 0);
        }
      }
    }
  };
  if constexpr (NPF > 0) {
    if (!stop_code && a.K > 0) {
      publish_rows(rowi);
      __syncthreads();
      issue_prefetch();
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
    }
  }

  // The step's tile. Slots p * CPL + r < NPF come from the LDS prefetch; the others load from
  // HBM: for step 0 here, for step k + 1 at the end of step k's update (rows past eta read row 0
  // and are never used).
  float4 tile[RP][CPL];
  if (!stop_code && a.K > 0) {
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const float* rowp = a.A + (int64_t)(rowi[p] < 0 ? 0 : rowi[p]) * a.ld + c0;
#pragma unroll
      for (int r = 0; r < CPL; ++r) {
        if (p * CPL + r < NPF) continue;
        const int q = sl + CL * r;  // clamped into the row: past the slice it meets x = 0
        tile[p][r] = *reinterpret_cast<const float4*>(rowp + 4 * (q < qlast ? q : qlast));
      }
    }
  }

  for (int64_t k = 0; k < a.K && !stop_code; ++k) {
    // Re-derive the lane coordinates from an opaque copy of the thread id each
    // step: otherwise the compiler hoists every lane-dependent address out of
    // the loop and keeps it in VGPRs that the register tile needs.
    int tidl = threadIdx.x;
    asm volatile("" : "+v"(tidl));
    const int tid = tidl, lane = tidl & 63, wave = tidl >> 6, sl = lane / RL, ri = lane % RL;
    const unsigned tag = (unsigned)(k + 1);
    const float ak = a.alpha_k ? a.alpha_k[k] : a.alpha;
    u64* xP = a.xP + (size_t)(k & 1) * G * eta;
    const bool has_next = k + 1 < a.K;

#pragma unroll
    for (int p = 0; p < PL; ++p)
#pragma unroll
      for (int r = 0; r < CPL; ++r)
        if (p * CPL + r < NPF) tile[p][r] = pf[(p * CPL + r) * NT + tid];
    int rown[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) rown[p] = -1;
    int nerr = 0;
    if (has_next) fetch_rows(k + 1, rown, nerr);

    // partial dots, published pass by pass
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      float acc = 0.f;
#pragma unroll
      for (int r = 0; r < CPL; ++r) acc += dot4(tile[p][r], xv4[sl + CL * r]);
#pragma unroll
      for (int o = RL; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
      const int t = p * kRtRowsPerPass + RL * wave + ri;
      if (sl == 0 && t < etaH) put_tagged(&xP[(size_t)s * eta + hr0 + t], acc, tag);
      __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (NPF > 0 && !kPfAfterHop1) {
      // every wave has consumed its LDS slots (the dots used them): the next step's may land
      if (has_next) {
        publish_rows(rown);
        __syncthreads();
        issue_prefetch();
      }
    } else if constexpr (NPF > 0) {
      if (has_next) publish_rows(rown);
    }
    int bad = 0;
    // reduce the owned rows over the C slices; c_t = (alpha/eta)(r_t - b)/||a||^2
#pragma unroll
    for (int j = 0; j < kOwnMax; ++j) {
      const int t = ot0 + wave + kRtWaves * j;
      if (t < ot1) {
        float v[kMaxG / 64];
        wait_tagged_batch(&xP[(size_t)lane * eta + hr0 + t], (size_t)64 * eta, (C - lane + 63) / 64, tag, v, lerr);
        float sum = 0.f;
#pragma unroll
        for (int i = 0; i < kMaxG / 64; ++i) sum += v[i];
        sum = wave_sum(sum);
        if (lane == 0) {
          float c;
          const float rn = orn[j];
          if (rn == 0.f) { c = NAN; set_status(a.status, ST_ZERO_ROW); }
          else c = (ak / (float)eta) * (sum - ob[j]) / rn;
          if (a.two_hop) {
            put_tagged(&a.xC[hr0 + t], c, tag);
          } else {
            cs[t] = c;
            bad |= !isfinite(c);
          }
        }
      }
    }
    if constexpr (NPF > 0 && kPfAfterHop1) {
      if (has_next) {
        __syncthreads();  // publishes nrow[]; every wave's LDS slots were read before the dots
        issue_prefetch();
      }
    }
    if (has_next) fetch_owned(k + 1);
    if (a.two_hop && tid < kRtRowsPerPass) {
      float v[RP];
      wait_tagged_batch(&a.xC[hr0 + tid], kRtRowsPerPass, (etaH - tid + kRtRowsPerPass - 1) / kRtRowsPerPass, tag,
                        v, lerr);
#pragma unroll
      for (int i = 0; i < RP; ++i)
        if (tid + kRtRowsPerPass * i < etaH) {
          cs[tid + kRtRowsPerPass * i] = v[i];
          bad |= !isfinite(v[i]);
        }
    }
    if (lerr) set_status(a.status, lerr);
    // One or-barrier agrees on every condition of the step (an expired wait, a non-finite
    // coefficient, a bad index in the next step), so that the barriers after the update are
    // plain ones, which do not wait for the next step's loads; every workgroup holds the same
    // c_t and the same indices, so all stop at the same step.
    // Block OR in one barrier: the flag word of this step's parity collects the bits, the other
    // word (last read before the previous step's final barrier) is cleared for the next step.
    const int flag = (lerr ? 1 : 0) | (bad ? 2 : 0) | (nerr ? 4 : 0);
    if (flag) atomicOr(&orflag[k & 1], flag);
    __syncthreads();
    const int fl = orflag[k & 1];
    if (tid == 0) orflag[(k + 1) & 1] = hop3_bad[(k + 1) & 1] = 0;
    if (fl & 1) { stop_code = ST_ABORTED; break; }
    if (fl & 2) {
      if constexpr (RG > 1) {
        // the other group of the slice (whose coefficients may be finite) takes a NaN update
        // part from this one and stops at the end of this step
        if (tid < 4 * wq)
          put_tagged(&a.xU[(((size_t)(k & 1) * C + s) * RG + h) * SW + tid], __builtin_nanf(""), tag);
      }
      stop_code = ST_NONFINITE;
      break;
    }
    const int next_bad = fl & 4;

    // transposed update: per chunk slot, sum over own rows, then the RL lanes
    // holding that chunk, then the waves
    float cp[RP];
#pragma unroll
    for (int p = 0; p < RP; ++p) {
      const int t = p * kRtRowsPerPass + RL * wave + ri;
      cp[p] = t < etaH ? cs[t] : 0.f;
    }
    const bool load_next = has_next && !next_bad;
    if (a.y && s == 0)
      for (int t = tid; t < etaH; t += kRtThreads) atomicAdd(&a.y[a.idx[k * (int64_t)eta + hr0 + t]], -cs[t]);
#pragma unroll
    for (int r = 0; r < CPL; ++r) {
      float4 d = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        d.x += cp[p] * tile[p][r].x;
        d.y += cp[p] * tile[p][r].y;
        d.z += cp[p] * tile[p][r].z;
        d.w += cp[p] * tile[p][r].w;
      }
      d.x = lanes_sum<RL>(d.x);
      d.y = lanes_sum<RL>(d.y);
      d.z = lanes_sum<RL>(d.z);
      d.w = lanes_sum<RL>(d.w);
      if (ri == 0) red[wave][sl + CL * r] = d;
    }
    // the tile is used up: the next step's HBM slots load now, row by row (a row's chunks issued
    // back to back keep the DRAM pages open), and stay in flight across the plain barriers. The
    // waves that poll the third hop issue theirs after it: a poll waits for all of its wave's loads.
    auto load_tile = [&]() {
#pragma unroll
      for (int p = 0; p < RP; ++p) {
        const float* rowp = a.A + (int64_t)(rown[p] < 0 ? 0 : rown[p]) * a.ld + c0;
#pragma unroll
        for (int r = 0; r < CPL; ++r) {
          if (p * CPL + r < NPF) continue;
          const int q = sl + CL * r;
          tile[p][r] = *reinterpret_cast<const float4*>(rowp + 4 * (q < qlast ? q : qlast));
        }
      }
    };
    if (load_next && wave >= kPollWaves) load_tile();
    __syncthreads();  // publishes red[]
    if (tid < 4 * wq) {  // chunks past the slice carry clamped data: discarded
      const int q = tid >> 2, e = tid & 3;
      float dsum = 0.f;
      for (int w = 0; w < kRtWaves; ++w) {
        const float4 v = red[w][q];
        dsum += e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w;
      }
      if constexpr (RG > 1) {
        // third hop: the slice's RG groups add their parts in group order, so every copy of the
        // slice gets the same x (the next step's HBM loads are in flight meanwhile)
        u64* xU = a.xU + ((size_t)(k & 1) * C + s) * RG * SW;
        put_tagged(&xU[(size_t)h * SW + tid], dsum, tag);
        float tot = 0.f;
#pragma unroll
        for (int hh = 0; hh < RG; ++hh) tot += hh == h ? dsum : wait_tagged<float>(&xU[(size_t)hh * SW + tid], tag, lerr);
        if (lerr) set_status(a.status, ST_ABORTED);
        if (!isfinite(tot)) atomicOr(&hop3_bad[k & 1], 1);
        dsum = tot;
      }
      const float z = xs[tid] - dsum;
      xs[tid] = z;
      xv[tid] = shrink(z, a.lambda);
    }
    if constexpr (RG > 1) {
      if (load_next && wave < kPollWaves) load_tile();
    }
    k_done = k + 1;
    if constexpr (NPF > 0) {
      // the LDS prefetch has landed before the barrier: the only loads this wave issued after
      // it are the update's kHbmSlots next-step slots (older ones are done at vmcnt <= kHbmSlots)
      if (wave >= kRtWaves / 2) {
        if (load_next) __builtin_amdgcn_s_waitcnt(kWaitPrefetch);
        else __builtin_amdgcn_s_waitcnt(0);
      }
    }
    __syncthreads();
    if constexpr (RG > 1) {
      // a group that stopped on a non-finite coefficient sent NaN parts: every copy stops here
      if (hop3_bad[k & 1]) { stop_code = ST_NONFINITE; break; }
    }

    if (a.xref && a.check_every > 0 && (k + 1) % a.check_every == 0) {
      const unsigned mtag = (unsigned)((k + 1) / a.check_every);
      double e2 = 0.0, r2s = 0.0;
      for (int j = tid; j < wq * 4; j += kRtThreads) {
        const int64_t c = c0 + j;
        if (c < a.n && h == 0) {  // one copy of each slice counts
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
        for (int w = 0; w < kRtWaves; ++w) { se += mon[2 * w]; sr += mon[2 * w + 1]; }
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
          mon[2 * kRtWaves] = err;
        }
      }
      if (lerr) set_status(a.status, lerr);
      if (__syncthreads_or(lerr)) { stop_code = ST_ABORTED; break; }
      if (a.tol > 0.0 && mon[2 * kRtWaves] <= a.tol) break;
    }
    if (next_bad) { stop_code = ST_INDEX; break; }
#pragma unroll
    for (int p = 0; p < RP; ++p) rowi[p] = rown[p];
  }
  if (stop_code && tid == 0) set_status(a.status, stop_code);
  __builtin_amdgcn_s_waitcnt(0);  // no load of a step that will not run stays in flight
  __syncthreads();
  if (h == 0)
    for (int j = tid; j < wq * 4; j += kRtThreads) {
      const int64_t c = c0 + j;
      if (c < a.n) { a.x_star[c] = xs[j]; a.x[c] = xv[j]; }
    }
  if (g == 0 && tid == 0) a.status[1] = (int)k_done;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

template <int NT, int RP, int CPL, int RG>
static void* rt_ptr() {
  return reinterpret_cast<void*>(&rska_dense_rt<NT, RP, CPL, RG>);
}

// 1024 threads for eta <= 768 (RP <= 3), 512 threads (256 VGPRs a lane) for 768 < eta <= 1024.
static void* rt_kernel(int nt, int rp, int cpl, int rg) {
#define RT_CASE(N, R, C, H) if (nt == N && rp == R && cpl == C && rg == H) return rt_ptr<N, R, C, H>();
#define RT_CPL(N, R, H) RT_CASE(N, R, 1, H) RT_CASE(N, R, 2, H) RT_CASE(N, R, 3, H) RT_CASE(N, R, 4, H) RT_CASE(N, R, 5, H)
  RT_CPL(1024, 1, 1) RT_CPL(1024, 2, 1) RT_CPL(1024, 3, 1)
  RT_CPL(512, 7, 1) RT_CPL(512, 8, 1)
  RT_CPL(1024, 1, 2) RT_CPL(1024, 2, 2) RT_CPL(1024, 3, 2)
  RT_CPL(512, 7, 2) RT_CPL(512, 8, 2)
#undef RT_CPL
#undef RT_CASE
  return nullptr;
}

int dense_rt_max_grid(int nt, int rp, int cpl, int rg) {
  void* fn = rt_kernel(nt, rp, cpl, rg);
  if (!fn) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, nt, 0) != hipSuccess) return 0;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  return per_cu * cus;
}

hipError_t launch_dense_rt(DenseArgs<float>& a, int nt, int rp, int cpl, int rg, hipStream_t stream) {
  void* fn = rt_kernel(nt, rp, cpl, rg);
  if (!fn) return hipErrorInvalidValue;
  if (a.G % rg != 0 || (rg > 1 && !a.xU)) return hipErrorInvalidValue;
  if (a.G > kMaxG || dense_rt_max_grid(nt, rp, cpl, rg) < a.G) return hipErrorCooperativeLaunchTooLarge;
  void* args[] = {&a};
  return launch_persistent(fn, dim3(a.G), dim3(nt), args, 0, stream);
}

}  // namespace rsk
