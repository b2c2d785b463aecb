// Device code shared by the single-graph kernels and the batched kernels:
// union-find, the sort + LPT body, the per-component walk and the packed
// base access.  Each part names the step of Algorithm 2 it serves.
#pragma once

#include "cg_internal.h"

namespace cg {

// ---------------------------------------------------------------------------
// BranchRemoval: flags of a vertex whose row starts at b and has `deg`
// entries: bit0 branch (deg >= 3); bit1 / bit2 entry 0 / 1 kept (neither end
// is a branch vertex).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t vertex_flags(const int32_t *__restrict__ row_ptr,
                                                 const int32_t *__restrict__ col, int32_t b,
                                                 int32_t deg) {
  if (deg >= 3) return 1u;
  uint32_t f = 0;
  if (deg > 0) {
    const int32_t u0 = col[b];
    if (row_ptr[u0 + 1] - row_ptr[u0] < 3) f |= 2;
    if (deg == 2) {
      const int32_t u1 = col[b + 1];
      if (row_ptr[u1 + 1] - row_ptr[u1] < 3) f |= 4;
    }
  }
  return f;
}

// ---------------------------------------------------------------------------
// ConnectedComponent: union-find with min-id roots
// ---------------------------------------------------------------------------
__device__ __forceinline__ int32_t uf_find(int32_t *P, int32_t x) {
  while (true) {
    int32_t p = ld_relaxed(P + x);
    if (p == x) return x;
    int32_t gp = ld_relaxed(P + p);
    if (gp == p) return p;
    st_relaxed(P + x, gp);  // path halving: gp is an ancestor of x
    x = gp;
  }
}

__device__ __forceinline__ void uf_union(int32_t *P, int32_t a, int32_t b) {
  a = uf_find(P, a);
  b = uf_find(P, b);
  while (a != b) {
    if (a < b) {
      int32_t old = atomicCAS(P + b, b, a);  // link the larger root under the smaller
      if (old == b) return;
      b = old;
    } else {
      int32_t old = atomicCAS(P + a, a, b);
      if (old == a) return;
      a = old;
    }
  }
}

// Tagged forest: each entry holds (tag << 32) | parent, and an entry whose
// tag is not the current run's stands for "no parent".  Bumping the tag
// between runs therefore resets the whole forest without touching it, so
// the hooks can run in the same pass that finds the kept entries.  Parents
// are always smaller than their children, so every root is its tree's
// minimum id.
__device__ __forceinline__ uint64_t ld_relaxed64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_relaxed64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t tf_entry(uint32_t tag, int32_t parent) {
  return ((uint64_t)tag << 32) | (uint32_t)parent;
}
__device__ __forceinline__ int32_t tf_parent(const uint64_t *F, uint32_t tag, int32_t x) {
  const uint64_t e = ld_relaxed64(F + x);
  return (uint32_t)(e >> 32) == tag ? (int32_t)(uint32_t)e : x;
}

__device__ __forceinline__ int32_t tf_find(uint64_t *F, uint32_t tag, int32_t x) {
  while (true) {
    const int32_t p = tf_parent(F, tag, x);
    if (p == x) return x;
    const int32_t gp = tf_parent(F, tag, p);
    if (gp == p) return p;
    st_relaxed64(F + x, tf_entry(tag, gp));  // path halving
    x = gp;
  }
}

__device__ __forceinline__ void tf_union(uint64_t *F, uint32_t tag, int32_t a, int32_t b) {
  a = tf_find(F, tag, a);
  b = tf_find(F, tag, b);
  while (a != b) {
    const int32_t hi = a > b ? a : b, lo = a > b ? b : a;
    const uint64_t e = ld_relaxed64(F + hi);
    if ((uint32_t)(e >> 32) == tag) {  // hi got a parent meanwhile: climb
      const int32_t p = (int32_t)(uint32_t)e;
      if (a == hi) a = p;
      else b = p;
      continue;
    }
    // link the larger root under the smaller one
    if (atomicCAS((unsigned long long *)(F + hi), (unsigned long long)e,
                  (unsigned long long)tf_entry(tag, lo)) == e)
      return;
  }
}

// ---------------------------------------------------------------------------
// GreedyPartitioning: sort + LPT on one workgroup
// ---------------------------------------------------------------------------
constexpr int kLptBlock = 1024;
constexpr int kSortCapLds = 8192;  // components sorted in LDS
constexpr int kBinCapLds = 2048;   // bins kept in LDS

__device__ __forceinline__ int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Exclusive prefix minimum over the lanes of the wave (lane 0 gets
// 0xFFFFFFFF): row shifts 1, 2, 4, 8 within rows of 16 lanes, then the row
// broadcasts of lanes 15 and 31 (lanes without a source take the identity).
// Every lane of the wave must be active.
__device__ __forceinline__ uint32_t wave_excl_min_u32(uint32_t x) {
  const int id = -1;  // 0xFFFFFFFF
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x111, 0xF, 0xF, false));  // row_shr:1
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x112, 0xF, 0xF, false));  // row_shr:2
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x114, 0xF, 0xF, false));  // row_shr:4
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x118, 0xF, 0xF, false));  // row_shr:8
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x142, 0xA, 0xF, false));  // row_bcast:15
  x = min(x, (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x143, 0xC, 0xF, false));  // row_bcast:31
  return (uint32_t)__builtin_amdgcn_update_dpp(id, (int)x, 0x138, 0xF, 0xF, false);       // wave_shr:1
}

// x of lane l ^ J: quad permutes for J = 1, 2, row shifts by 4 for J = 4, a
// rotation of each 16-lane row by 8 for J = 8, a swizzle for J = 16 and a
// bpermute for J = 32.  Every lane of the wave must be active.
template <int J>
__device__ __forceinline__ uint32_t wave_xor_u32(uint32_t x) {
  const int v = (int)x;
  if constexpr (J == 1) {
    return (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);  // quad_perm [1,0,3,2]
  } else if constexpr (J == 2) {
    return (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);  // quad_perm [2,3,0,1]
  } else if constexpr (J == 4) {
    const uint32_t up = (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0x104, 0xF, 0xF, false);  // row_shl:4
    const uint32_t dn = (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0x114, 0xF, 0xF, false);  // row_shr:4
    return (lane_id() & 4) ? dn : up;
  } else if constexpr (J == 8) {
    return (uint32_t)__builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else if constexpr (J == 16) {
    return (uint32_t)__builtin_amdgcn_ds_swizzle(v, 0x401F);  // lanes of 32: xor 16
  } else {
    static_assert(J == 32, "partner distance");
    return (uint32_t)__shfl_xor(v, 32);
  }
}

// Bitonic sort of one value per lane across the wave, ascending in lane
// order: stage (K, J) for K = 2..64, J = K/2..1.  All lanes active.
template <int K = 2, int J = 1>
__device__ __forceinline__ uint32_t wave_sort_u32(uint32_t x, int l) {
  const uint32_t p = wave_xor_u32<J>(x);
  const bool keep_min = ((l & J) == 0) == ((l & K) == 0);
  x = keep_min ? min(x, p) : max(x, p);
  if constexpr (J > 1) return wave_sort_u32<K, J / 2>(x, l);
  else if constexpr (K < kWave) return wave_sort_u32<2 * K, K>(x, l);
  else return x;
}

// One compare-exchange of a bitonic stage (k, J), J < 64, in registers: x is
// element i of the array, held by lane i % 64, and its partner i ^ J is held
// by lane (i % 64) ^ J of the same wave.  Every lane of the wave takes part.
template <int J, typename K>
__device__ __forceinline__ K bitonic_lane_step(K x, int i, int k) {
  K p;
  if constexpr (sizeof(K) == 8)
    p = ((K)wave_xor_u32<J>((uint32_t)(x >> 32)) << 32) | wave_xor_u32<J>((uint32_t)x);
  else
    p = (K)wave_xor_u32<J>((uint32_t)x);
  const bool keep_min = ((i & J) == 0) == ((i & k) == 0);
  const K mn = x < p ? x : p, mx = x < p ? p : x;
  return keep_min ? mn : mx;
}

// Stages (k, j) for j = min(k/2, 32) down to 1 on two independent elements
// (k wave-uniform, so each test is a scalar branch)
template <typename K>
__device__ __forceinline__ void bitonic_lane_merge(K &x0, K &x1, int i0, int i1, int k) {
  if (k >= 64) {
    x0 = bitonic_lane_step<32>(x0, i0, k);
    x1 = bitonic_lane_step<32>(x1, i1, k);
  }
  if (k >= 32) {
    x0 = bitonic_lane_step<16>(x0, i0, k);
    x1 = bitonic_lane_step<16>(x1, i1, k);
  }
  if (k >= 16) {
    x0 = bitonic_lane_step<8>(x0, i0, k);
    x1 = bitonic_lane_step<8>(x1, i1, k);
  }
  if (k >= 8) {
    x0 = bitonic_lane_step<4>(x0, i0, k);
    x1 = bitonic_lane_step<4>(x1, i1, k);
  }
  if (k >= 4) {
    x0 = bitonic_lane_step<2>(x0, i0, k);
    x1 = bitonic_lane_step<2>(x1, i1, k);
  }
  x0 = bitonic_lane_step<1>(x0, i0, k);
  x1 = bitonic_lane_step<1>(x1, i1, k);
}

// Stages (k, j) of every k in [k0, k1] with j < 64, in registers, two
// 64-element segments per wave at a time (independent chains, so their lane
// shuffles overlap); no barrier: a wave only touches its own segments.
// Elements past N2 (N2 < 64, or a missing second segment) are held as the
// largest key and never meet a real one.
template <typename K>
__device__ __forceinline__ void bitonic_segments(K *a, int N2, int k0, int k1) {
  const int nw = (int)(blockDim.x / kWave);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWave));
  const int l = lane_id();
  const int nseg = (N2 + kWave - 1) / kWave;
  for (int sgm = w; sgm < nseg; sgm += 2 * nw) {
    const int i0 = sgm * kWave + l, i1 = (sgm + nw) * kWave + l;
    K x0 = i0 < N2 ? a[i0] : ~K(0);
    K x1 = i1 < N2 ? a[i1] : ~K(0);
    for (int k = k0; k <= k1; k <<= 1) bitonic_lane_merge(x0, x1, i0, i1, k);
    if (i0 < N2) a[i0] = x0;
    if (i1 < N2) a[i1] = x1;
  }
}

// Sort a[0, N2) ascending (N2 a power of two) with every thread of the
// workgroup.  Only the stages whose pairs lie 64 or more apart go through
// memory, two per pass and barrier; the stages inside 64-element segments
// run in registers (for N2 = 512: 4 passes through memory, 45 stages).
// kLdsOnly: the barriers order LDS only, so the caller's global loads stay
// in flight through the sort.
template <typename K, bool kLdsOnly = false>
__device__ __forceinline__ void bitonic_sort(K *a, int N2) {
  auto bar = [] {
    if constexpr (kLdsOnly) lds_barrier();
    else __syncthreads();
  };
  bitonic_segments(a, N2, 2, N2 < kWave ? N2 : kWave);
  bar();
  for (int k = 2 * kWave; k <= N2; k <<= 1) {
    int j = k >> 1;
    // two stages (j, j/2) per barrier: each thread takes the four elements
    // i, i + j/2, i + j, i + 3j/2 (bits j and j/2 of i clear), all sorted in
    // the same direction since they differ only below k
    for (; j >= 2 * kWave; j >>= 2) {
      const int h = j >> 1;
      for (int t = threadIdx.x; t < N2 / 4; t += blockDim.x) {
        const int i = ((t & ~(h - 1)) << 2) | (t & (h - 1));
        const bool up = (i & k) == 0;
        K x0 = a[i], x1 = a[i + h], x2 = a[i + j], x3 = a[i + j + h];
        if ((x0 > x2) == up) { const K tmp = x0; x0 = x2; x2 = tmp; }
        if ((x1 > x3) == up) { const K tmp = x1; x1 = x3; x3 = tmp; }
        if ((x0 > x1) == up) { const K tmp = x0; x0 = x1; x1 = tmp; }
        if ((x2 > x3) == up) { const K tmp = x2; x2 = x3; x3 = tmp; }
        a[i] = x0;
        a[i + h] = x1;
        a[i + j] = x2;
        a[i + j + h] = x3;
      }
      bar();
    }
    if (j >= kWave) {  // one stage left above the register stages
      for (int t = threadIdx.x; t < N2 / 2; t += blockDim.x) {
        const int i = ((t & ~(j - 1)) << 1) | (t & (j - 1));  // pair (i, i + j)
        const K x = a[i], y = a[i + j];
        if ((x > y) == ((i & k) == 0)) {
          a[i] = y;
          a[i + j] = x;
        }
      }
      bar();
    }
    bitonic_segments(a, N2, k, k);
    bar();
  }
}

// Stable sort of a[0, n) by bits 16 and up of its 32-bit keys, whose low 16
// bits are each key's index (the input is in index order), so the result is
// the order of the whole keys.  LSD radix sort over `passes` 8-bit digits
// from bit 16.  Each wave takes a contiguous run of keys, 64 per round in
// order: the lanes holding the same digit are found by eight ballots, and a
// key's rank is the wave's running count of its digit (in LDS) plus the
// lanes below it with the same digit.  One block scan over the counts in
// (digit, wave) order gives every digit's start for every wave.  tmp holds
// n keys, cnt 256 counters per wave (LDS), sh the block scan's words.
// n <= kRadixRounds * BLOCK.  Returns the array holding the result (a after
// an even number of passes, else tmp).
constexpr int kRadixRounds = 8;
template <int BLOCK>
__device__ __forceinline__ uint32_t *radix_sort_hi16(uint32_t *a, uint32_t *tmp, int n, int passes,
                                                     uint32_t *cnt, uint32_t *sh) {
  constexpr int NW = BLOCK / kWave;
  constexpr int E = 256 * NW / BLOCK;  // (digit, wave) counters per thread in the scan
  static_assert(E * BLOCK == 256 * NW, "whole counters per thread");
  const int w = threadIdx.x / kWave, l = lane_id();
  const int per_w = ((n + NW - 1) / NW + kWave - 1) & ~(kWave - 1);
  const int rounds = per_w / kWave;  // uniform, at most kRadixRounds
  const uint64_t below = (1ull << l) - 1ull;
  uint32_t *my = cnt + w * 256;
  uint32_t *src = a, *dst = tmp;
  for (int p = 0; p < passes; ++p) {
    const int s = 16 + 8 * p;
    for (int d = l; d < 256; d += kWave) my[d] = 0;
    uint32_t x[kRadixRounds];
    int pos[kRadixRounds];
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
      x[r] = 0;
      pos[r] = 0;
      if (r >= rounds) continue;
      const int i = w * per_w + r * kWave + l;
      const bool v = i < n;
      x[r] = v ? src[i] : 0u;
      const uint32_t d = (x[r] >> s) & 255u;
      uint64_t peers = __ballot(v);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(v && bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t c = my[d];  // the digit's count before this round
      pos[r] = (int)c + __popcll(peers & below);
      // the lowest lane holding the digit adds the round's keys of it
      if (v && (peers & below) == 0) my[d] = c + (uint32_t)__popcll(peers);
    }
    __syncthreads();
    // every (digit, wave) count to its start: exclusive scan in digit-major
    // order
    uint32_t c[E], sum = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = (int)threadIdx.x * E + k;
      c[k] = cnt[(e % NW) * 256 + e / NW];
      sum += c[k];
    }
    uint32_t tot;
    uint32_t ex = block_excl_scan<uint32_t, BLOCK>(sum, sh, &tot);
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const int e = (int)threadIdx.x * E + k;
      cnt[(e % NW) * 256 + e / NW] = ex;
      ex += c[k];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kRadixRounds; ++r) {
      if (r >= rounds) continue;
      const int i = w * per_w + r * kWave + l;
      if (i < n) dst[my[(x[r] >> s) & 255u] + pos[r]] = x[r];
    }
    __syncthreads();
    uint32_t *t = src;
    src = dst;
    dst = t;
  }
  return src;
}

// number of elements of the sorted array a[0..len) that are < x
__device__ __forceinline__ int lower_bound_u64(const uint64_t *a, int len, uint64_t x) {
  int lo = 0, hi = len;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (a[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// x of lane l + 1 in lane l, by a DPP wave shift (wave_shl:1); lane 63,
// which has no source, keeps its own x
__device__ __forceinline__ uint64_t wave_next_u64(uint64_t x) {
  const int lo = (int)(uint32_t)x, hi = (int)(uint32_t)(x >> 32);
  const uint32_t nlo = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, 0x130, 0xF, 0xF, false);
  const uint32_t nhi = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, 0x130, 0xF, 0xF, false);
  return ((uint64_t)nhi << 32) | nlo;
}

// x of lane l - 1 in lane l, by a DPP wave shift (wave_shr:1); lane 0 keeps
// its own x
__device__ __forceinline__ uint32_t wave_prev_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x138, 0xF, 0xF, false);
}
// x of lane l + 1 in lane l (wave_shl:1); lane 63 keeps its own x
__device__ __forceinline__ uint32_t wave_next_u32(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)x, (int)x, 0x130, 0xF, 0xF, false);
}

// weight of the t-th item in LPT order, from the sorted keys (32-bit keys
// (2^16-1 - w) << 16 | index, or 64-bit (2^32-1 - w) << 32 | index)
__device__ __forceinline__ uint32_t lpt_item_weight(const uint32_t *srt, const uint64_t *keys,
                                                    bool k32, int t) {
  return 0xFFFFFFFFu - (k32 ? 0xFFFF0000u | (srt[t] >> 16) : (uint32_t)(keys[t] >> 32));
}

// Bin keys are (load << 16) | bin: ascending key order is ascending
// (load, bin), i.e. the least loaded bin with the lowest index first.
constexpr int kBinBits = 16;
constexpr int kLptRoundMin = 6;   // equal items taken as one round from this many
constexpr int kLptPrefixMin = 8;  // prefix rounds (any weights) from this many items

// With comp_kind and comp_estart given, it also writes each component's
// first local CSR entry (2(q-1) entries for a path, 2q for a cycle, none for
// a single read, in (bin, label) order) and returns their total.  bin_reads
// (global memory, read back with atomic loads) gets the reads of each bin.
template <int BLOCK>
__device__ __forceinline__ int lpt_body(int nc, int P, const int32_t *__restrict__ comp_size,
                                        const uint64_t *__restrict__ weight,
                                        uint64_t *keys, int32_t *bin_of, uint64_t *binA,
                                        uint64_t *binB, int32_t *__restrict__ comp_bin,
                                        int32_t *__restrict__ comp_rank,
                                        int32_t *__restrict__ comp_start,
                                        uint64_t *__restrict__ bin_load,
                                        uint64_t *__restrict__ bin_reads,
                                        unsigned int *status,
                                        const uint8_t *__restrict__ comp_kind = nullptr,
                                        int32_t *__restrict__ comp_estart = nullptr) {
  static_assert(BLOCK > 2 * kWave, "the pipelined windows' merge needs threads beyond two waves");
  __shared__ uint64_t win[2][kWave];  // a window's raised keys, alternating buffers
  __shared__ uint32_t s_cnt[BLOCK >= 1024 ? BLOCK / kWave * 256 : 1];  // the radix sorts' counters
  __shared__ int32_t sh_scan[BLOCK / kWave + 1];
  __shared__ int64_t sh_scan64[BLOCK / kWave + 1];
  __shared__ unsigned long long s_wsum;
  __shared__ unsigned int s_wmax;
  const int tid = threadIdx.x;
  const int N2 = next_pow2(nc > 0 ? nc : 1);
  if (tid == 0) {
    s_wsum = 0;
    s_wmax = 0;
  }
  __syncthreads();

  // 1. sort by (weight desc, label asc); components are indexed in label
  // order.  The weight is the read count, or the given weights (below 2^32).
  // Keys are ((2^32-1 - w) << 32) | i, or, when every weight and index fits
  // 16 bits, ((2^16-1 - w) << 16) | i in 32 bits (k32: the first half of
  // keys holds them); ~0 pads to N2.
  unsigned long long wsum = 0;
  uint32_t wmax = 0;
  for (int i = tid; i < nc; i += blockDim.x) {
    uint64_t w = weight ? weight[i] : (uint64_t)comp_size[i];
    if (w > 0xFFFFFFFFull) {
      atomicOr(status, CG_STATUS_WEIGHT_RANGE);
      w = 0xFFFFFFFFull;
    }
    wsum += w;
    wmax = w > wmax ? (uint32_t)w : wmax;
  }
  for (int off = kWave / 2; off > 0; off >>= 1) {
    wsum += __shfl_xor(wsum, off);
    const uint32_t o = (uint32_t)__shfl_xor((int)wmax, off);
    wmax = o > wmax ? o : wmax;
  }
  if (lane_id() == 0 && wsum) {
    atomicAdd(&s_wsum, wsum);
    atomicMax(&s_wmax, wmax);
  }
  for (int b = tid; b < P; b += blockDim.x) binA[b] = (uint64_t)b;  // load 0, sorted
  __syncthreads();
  const bool k32 = nc <= 0xFFFF && s_wmax <= 0xFFFFu;
  uint32_t *keys32 = reinterpret_cast<uint32_t *>(keys);
  for (int i = tid; i < N2; i += blockDim.x) {
    uint64_t w = 0;
    if (i < nc) {
      w = weight ? weight[i] : (uint64_t)comp_size[i];
      w = w > 0xFFFFFFFFull ? 0xFFFFFFFFull : w;
    }
    if (k32)
      keys32[i] = i < nc ? ((0xFFFFu - (uint32_t)w) << 16) | (uint32_t)i : ~0u;
    else
      keys[i] = i < nc ? ((uint64_t)(0xFFFFFFFFu - (uint32_t)w) << 32) | (uint32_t)i : ~0ull;
  }
  __syncthreads();
  // the keys in LPT order: with a 1024-thread workgroup, radix passes over
  // the weight's bytes (one when every weight is below 256); else (fewer
  // waves, whose rounds of the radix sort run one after another, wide keys,
  // or more keys than the radix sort holds) a bitonic sort
  constexpr bool kRadix = BLOCK >= 1024;
  const uint32_t *srt = keys32;
  if (kRadix && k32 && nc <= kRadixRounds * BLOCK)
    srt = radix_sort_hi16<BLOCK>(keys32, keys32 + N2, nc, s_wmax < 256u ? 1 : 2, s_cnt,
                                 reinterpret_cast<uint32_t *>(sh_scan));
  else if (k32)
    bitonic_sort(keys32, N2);
  else
    bitonic_sort(keys, N2);

  // 2. LPT.  The bins are kept sorted by (load, bin).  A window holds the W
  // least loaded bins in the lanes of wave 0 (sorted across lanes): each
  // component goes to lane 0's bin, whose new key is then re-inserted by
  // ballot + shift.  Within W steps of a window only its W bins can be the
  // minimum (step t picks a bin of initial rank <= t), so after W steps the
  // window is merged back into the sorted bin list.
  const int W = P < kWave ? P : kWave;
  const bool single_window = P <= kWave;
  // Narrow keys: with kb bits for the bin index (2^kb >= P) and a total
  // weight below 2^(32 - kb) - 1, a bin's key (load << kb) | bin fits 32 bits
  // below the padding value 0xFFFFFFFF, and a step needs about 12 vector
  // instructions instead of 17.  Same order, same choices.  The bin lists
  // hold narrow keys zero-extended, so the window merge is unchanged.
  int kb = 0;
  while ((1 << kb) < P) ++kb;
  const bool narrow = kb <= 16 && s_wsum + 1 < (1ull << (32 - kb));
  int i0 = 0;
  if (!single_window && nc > P) {
    // The first round in one pass.  Every weight is at least 1, so item t
    // (t < P) finds bins 0..t-1 loaded and bin t empty, the least loaded one
    // with the lowest index: items 0..P-1 go to bins 0..P-1.  The weights do
    // not increase along the items, so in the bin list sorted by (load, bin)
    // bin t comes after the bins of smaller load (those past its run of
    // equal weights) and in bin order within its run.
    for (int t = tid; t < P; t += blockDim.x) {
      const uint32_t wt = lpt_item_weight(srt, keys, k32, t);
      int lo = 0, hi = t;  // the run's first item: the first of weight <= wt
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lpt_item_weight(srt, keys, k32, mid) > wt) lo = mid + 1;
        else hi = mid;
      }
      const int g0 = lo;
      lo = t;
      hi = P;  // one past the run's last item (within the first round)
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lpt_item_weight(srt, keys, k32, mid) < wt) hi = mid;
        else lo = mid + 1;
      }
      const int pos = (P - lo) + (t - g0);
      binA[pos] = narrow ? (uint64_t)(((uint32_t)wt << kb) | (uint32_t)t)
                         : ((uint64_t)wt << kBinBits) | (uint64_t)t;
      bin_of[k32 ? (srt[t] & 0xFFFFu) : (uint32_t)keys[t]] = t;
    }
    i0 = P;
  }
  __syncthreads();  // (outside the branch: inside it, the compiler kept a stack frame)
  // Above 64 bins the windows are pipelined (the workgroup has more than
  // 2 * 64 threads): after a window's steps, wave 0
  // forms the next window in its lanes as the W least of the raised keys and
  // the next W keys of the list (a bitonic merge in registers) and goes on,
  // while the other waves merge the raised keys back into the list.  One
  // barrier per window; the raised keys alternate between two buffers, so a
  // window's keys are written while the other waves still merge the last
  // ones, and the list alternates between binA and binB.
  uint32_t key32 = 0xFFFFFFFFu;  // wave 0: the window's keys (narrow or wide)
  uint64_t key64 = ~0ull;
  if (tid < kWave) {
    if (narrow) key32 = tid < W ? (uint32_t)binA[tid] : 0xFFFFFFFFu;
    else key64 = tid < W ? binA[tid] : ~0ull;
  }
  int cur = 0;
  while (i0 < nc) {
    const int T = single_window ? nc - i0 : (nc - i0 < W ? nc - i0 : W);
    if (tid < kWave && narrow) {
      const int l = tid;
      const uint32_t bmask = (1u << kb) - 1u;
      uint32_t key = key32;
      for (int base = 0; base < T; base += kWave) {
        const int cnt = __builtin_amdgcn_readfirstlane(T - base < kWave ? T - base : kWave);
        uint64_t item = 0;
        if (l < cnt) {
          const int at = i0 + base + l;
          item = k32 ? ((uint64_t)(0xFFFF0000u | (srt[at] >> 16)) << 32) | (srt[at] & 0xFFFFu)
                     : keys[at];
        }
        int32_t mine = 0;  // bin of item l
        const uint32_t iw = (uint32_t)(item >> 32);
        for (int t = 0; t < cnt;) {
          const uint32_t wt = (uint32_t)__builtin_amdgcn_readlane((int)iw, t);
          const uint32_t q = 0xFFFFFFFFu - wt;
          const uint32_t k0 = (uint32_t)__builtin_amdgcn_readlane((int)key, 0);
          const uint32_t nk = k0 + (q << kb);
          const uint64_t below = __ballot(key < nk);  // lane 0 and the lanes below nk
          // items t, t+1, ... of the same weight (within this batch)
          const uint64_t same = __ballot(l < cnt && iw == wt) >> t;
          const int run = ~same ? (int)__builtin_ctzll(~same) : kWave;
          const int m = __popcll(below);
          const int c = run < m ? run : m;
          // A prefix round: items t, t+1, ... go to lanes 0, 1, ... for as
          // long as each lane's key is below every key the earlier items of
          // the round raised (lane j is then the least loaded bin when item
          // t + j comes), whatever the weights.  Only lanes below nk can
          // qualify, so it is tried when m allows a long enough round and an
          // equal run does not already take all m.
          int cp = 0;
          uint32_t r = 0xFFFFFFFFu;
          if (m >= kLptPrefixMin && c < m) {
            const bool has = l < cnt - t && l < W;
            const uint32_t ql = 0xFFFFFFFFu - (uint32_t)__shfl((int)iw, (l + t) & (kWave - 1));
            r = has ? key + (ql << kb) : 0xFFFFFFFFu;  // lane l's key after item t + l
            const uint32_t lower = wave_excl_min_u32(r);
            const uint64_t ok = __ballot(has && key < lower);
            cp = ~ok ? (int)__builtin_ctzll(~ok) : kWave;
          }
          if (cp >= kLptPrefixMin) {
            const uint32_t src = (uint32_t)__shfl((int)key, (l - t) & (kWave - 1));
            if (l >= t && l < t + cp) mine = (int32_t)(src & bmask);
            // raised keys in lanes 0..cp-1, the rest unchanged: sort the wave
            key = wave_sort_u32(l < cp ? r : key, l);
            t += cp;
          } else if (c >= kLptRoundMin) {
            // a round: c equal items go to lanes 0..c-1 in order (each of
            // those bins is below lane 0's raised key, so the steps would pick
            // them one after another); the raised keys of lanes 0..c-1 and
            // the keys of lanes c.. are two sorted runs, merged by rank
            const uint32_t src = (uint32_t)__shfl((int)key, (l - t) & (kWave - 1));
            if (l >= t && l < t + c) mine = (int32_t)(src & bmask);
            const uint32_t x = l < c ? key + (q << kb) : key;
            // rank in the other run: lanes 0..c-1 search lanes c..63, the
            // others lanes 0..c-1 (every lane runs every step)
            int lo = l < c ? c : 0, hi = l < c ? kWave : c;
            for (int it = 0; it < 7; ++it) {
              const int mid = (lo + hi) >> 1;
              const uint32_t v = (uint32_t)__shfl((int)x, mid & (kWave - 1));
              if (lo < hi) {
                if (v < x) lo = mid + 1;
                else hi = mid;
              }
            }
            const int pos = l < c ? l + (lo - c) : (l - c) + lo;
            key = (uint32_t)__builtin_amdgcn_ds_permute(pos * 4, (int)x);
            t += c;
          } else {
            mine = l == t ? (int32_t)(k0 & bmask) : mine;
            const int p = __popcll(below) - 1;  // lanes 1.. below nk
            const uint32_t nxt = wave_next_u32(key);
            key = l < p ? nxt : (l == p ? nk : key);
            t += 1;
          }
        }
        if (l < cnt) bin_of[(uint32_t)item] = mine;
      }
      if (l < W) win[cur][l] = key;
      key32 = key;
    } else if (tid < kWave) {
      const int l = tid;
      uint64_t key = key64;
      for (int base = 0; base < T; base += kWave) {
        const int cnt = __builtin_amdgcn_readfirstlane(T - base < kWave ? T - base : kWave);
        uint64_t item = 0;
        if (l < cnt) {
          const int at = i0 + base + l;
          item = k32 ? ((uint64_t)(0xFFFF0000u | (srt[at] >> 16)) << 32) | (srt[at] & 0xFFFFu)
                     : keys[at];
        }
        int32_t mine = 0;  // bin of item l, kept in lane l until the batch ends
        for (int t = 0; t < cnt; ++t) {
          // t is uniform: broadcasts are lane reads into scalar registers
          const uint64_t q =
              0xFFFFFFFFu - (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(item >> 32), t);
          const uint64_t k0 =
              ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(key >> 32), 0) << 32) |
              (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)key, 0);
          mine = l == t ? (int32_t)(k0 & ((1u << kBinBits) - 1)) : mine;
          const uint64_t nk = k0 + (q << kBinBits);
          const int p = __popcll(__ballot(key < nk)) - 1;  // lanes 1.. below nk
          // the key of lane l + 1 (a wave-wide DPP shift; lane 63 keeps its own)
          const uint64_t nxt = wave_next_u64(key);
          key = l < p ? nxt : (l == p ? nk : key);
        }
        if (l < cnt) bin_of[(uint32_t)item] = mine;
      }
      if (l < W) win[cur][l] = key;
      key64 = key;
    }
    // the window's raised keys are out, and the previous window's merge (by
    // the other waves, during these steps) is done
    __syncthreads();
    if (single_window) {
      if (tid < W) binA[tid] = win[cur][tid];
    } else {
      if (tid < kWave) {
        if (i0 + T < nc) {
          // the next window: the W (= 64) least of the raised keys and
          // binA[W..2W), as min(raised key l, binA[2W-1-l]) (a bitonic run
          // holding exactly those) sorted by the bitonic merge's stages
          const int l = tid, j = W + (kWave - 1) - l;
          if (narrow) {
            const uint32_t b = j < P ? (uint32_t)binA[j] : 0xFFFFFFFFu;
            uint32_t c = key32 < b ? key32 : b;
            c = bitonic_lane_step<32>(c, l, kWave);
            c = bitonic_lane_step<16>(c, l, kWave);
            c = bitonic_lane_step<8>(c, l, kWave);
            c = bitonic_lane_step<4>(c, l, kWave);
            c = bitonic_lane_step<2>(c, l, kWave);
            key32 = bitonic_lane_step<1>(c, l, kWave);
          } else {
            const uint64_t b = j < P ? binA[j] : ~0ull;
            uint64_t c = key64 < b ? key64 : b;
            c = bitonic_lane_step<32>(c, l, kWave);
            c = bitonic_lane_step<16>(c, l, kWave);
            c = bitonic_lane_step<8>(c, l, kWave);
            c = bitonic_lane_step<4>(c, l, kWave);
            c = bitonic_lane_step<2>(c, l, kWave);
            key64 = bitonic_lane_step<1>(c, l, kWave);
          }
        }
      } else {
        // the other waves: the raised keys (sorted) merged with binA[W..P)
        // (sorted) into binB.  Merge thread t < W places raised key t (its
        // rank in binA[W..P) by binary search); the others place the list's
        // keys, two at once (each one's rank among the W = 64 raised keys by
        // six fixed steps, the two searches interleaved)
        const uint64_t *wk = win[cur];
        const int t = tid - kWave, mt = (int)blockDim.x - kWave - W;  // list threads
        if (t < W) {
          const uint64_t x = wk[t];
          binB[t + lower_bound_u64(binA + W, P - W, x)] = x;
        } else {
          for (int j0 = t - W; j0 < P - W; j0 += 2 * mt) {
            const int j1 = j0 + mt;
            const bool two = j1 < P - W;
            const uint64_t x0 = binA[W + j0], x1 = two ? binA[W + j1] : 0ull;
            int r0 = 0, r1 = 0;
#pragma unroll
            for (int step = kWave / 2; step > 0; step >>= 1) {
              r0 += wk[r0 + step - 1] < x0 ? step : 0;
              r1 += wk[r1 + step - 1] < x1 ? step : 0;
            }
            r0 += wk[r0] < x0 ? 1 : 0;
            r1 += wk[r1] < x1 ? 1 : 0;
            binB[j0 + r0] = x0;
            if (two) binB[j1 + r1] = x1;
          }
        }
      }
      uint64_t *t = binA;
      binA = binB;
      binB = t;
      cur ^= 1;
    }
    i0 += T;
  }
  __syncthreads();  // the last merge is done: binA holds the final bin list
  // 3. (bin, label) order, read offsets and the reads of each bin; keys
  // (bin << 16) | i in 32 bits when bin and index fit 16 bits
  const bool b32 = nc <= 0xFFFF && P <= 0x10000;
  for (int i = tid; i < N2; i += blockDim.x) {
    if (b32)
      keys32[i] = i < nc ? ((uint32_t)bin_of[i] << 16) | (uint32_t)i : ~0u;
    else
      keys[i] = i < nc ? ((uint64_t)(uint32_t)bin_of[i] << 32) | (uint32_t)i : ~0ull;
  }
  // the reads of each bin are summed in binB (free once the loads are out;
  // in LDS when the bins are), then written once per bin
  for (int b = tid; b < P; b += blockDim.x) binB[b] = 0;
  __syncthreads();
  for (int i = tid; i < nc; i += blockDim.x)
    atomicAdd((unsigned long long *)binB + bin_of[i], (unsigned long long)comp_size[i]);
  __syncthreads();
  // (bin, label) order: radix passes over the bin's bytes (one up to 256
  // bins) as above, else a bitonic sort
  const uint32_t *srt2 = keys32;
  if (kRadix && b32 && nc <= kRadixRounds * BLOCK)
    srt2 = radix_sort_hi16<BLOCK>(keys32, keys32 + N2, nc, P <= 256 ? 1 : 2, s_cnt,
                                  reinterpret_cast<uint32_t *>(sh_scan));
  else if (b32)
    bitonic_sort(keys32, N2);
  else
    bitonic_sort(keys, N2);
  int carry = 0, ecarry = 0;
  for (int base = 0; base < nc; base += BLOCK) {
    const int i = base + tid;
    const uint32_t c = i < nc ? (b32 ? srt2[i] & 0xFFFFu : (uint32_t)keys[i]) : 0u;
    const int32_t sz = i < nc ? comp_size[c] : 0;
    if (comp_estart) {
      // reads and local entries in one scan: (reads << 32) | entries, each
      // field's total below 2^32 (entries <= 2 * reads, reads < 2^31)
      int64_t e2 = 0;
      if (i < nc) {
        const uint8_t kd = comp_kind[c];
        e2 = kd == CG_KIND_PATH ? 2 * (sz - 1) : (kd == CG_KIND_CYCLE ? 2 * sz : 0);
      }
      int64_t tot;
      const int64_t ex = block_excl_scan<int64_t, BLOCK>(((int64_t)sz << 32) | e2, sh_scan64, &tot);
      if (i < nc) {
        comp_start[c] = carry + (int32_t)(ex >> 32);
        comp_estart[c] = ecarry + (int32_t)(uint32_t)ex;
        comp_rank[c] = i;
      }
      carry += (int32_t)(tot >> 32);
      ecarry += (int32_t)(uint32_t)tot;
    } else {
      int32_t tot;
      const int32_t ex = block_excl_scan<int32_t, BLOCK>(sz, sh_scan, &tot);
      if (i < nc) {
        comp_start[c] = carry + ex;
        comp_rank[c] = i;
      }
      carry += tot;
    }
  }
  // the per-bin and per-component results, stored after the last barrier
  // (a barrier waits for the stores issued before it); binA still holds the
  // final bin list and binB the reads of each bin
  {
    const int bb = narrow ? kb : kBinBits;
    for (int b = tid; b < P; b += blockDim.x) {
      const uint64_t k = binA[b];
      bin_load[k & ((1ull << bb) - 1)] = k >> bb;
      bin_reads[b] = binB[b];
    }
  }
  for (int i = tid; i < nc; i += blockDim.x) comp_bin[i] = bin_of[i];
  return ecarry;
}

// ---------------------------------------------------------------------------
// InducedSubgraph: sort one component's block of reads by id (local numbers
// follow (bin, label, id)); one workgroup of kIndBlock threads
// ---------------------------------------------------------------------------
constexpr int kIndBlock = 256;
constexpr int kIndLocalCap = 1024;

// lidx (the local number of each read) is written for every component when
// lidx_always, else only for components above CAP reads (the ones whose
// neighbours are then numbered through it instead of the sorted block).
// Member i's id is members[MS * i].
template <int BLOCK, int CAP, int MS = 1>
__device__ __forceinline__ void sort_component_block(int q, int st,
                                                     const int32_t *__restrict__ members,
                                                     int32_t *__restrict__ perm,
                                                     int32_t *__restrict__ lidx, int32_t *a,
                                                     bool lidx_always = true) {
  if (q <= CAP) {
    int N2 = 1;
    while (N2 < q) N2 <<= 1;
    for (int i = threadIdx.x; i < N2; i += BLOCK) a[i] = i < q ? members[MS * i] : 0x7FFFFFFF;
    __syncthreads();
    // non-negative ids padded with the largest int32: the same order as uint32
    bitonic_sort(reinterpret_cast<uint32_t *>(a), N2);
    for (int i = threadIdx.x; i < q; i += BLOCK) {
      const int32_t v = a[i];
      perm[st + i] = v;
      if (lidx_always) lidx[v] = st + i;
    }
  } else {
    // large component: the rank of a read is the number of smaller ids in
    // its block (ids are distinct)
    for (int i = threadIdx.x; i < q; i += BLOCK) {
      const int32_t x = members[MS * i];
      int r = 0;
      for (int t = 0; t < q; ++t) r += members[MS * t] < x;
      perm[st + r] = x;
      lidx[x] = st + r;
    }
  }
  __syncthreads();
}

// InducedSubgraph for one component, all in one workgroup: sort its reads
// (members, in any order) by id, number them st, st+1, ..., and write their
// local CSR rows (kept entries in row order of S, neighbours renumbered,
// entry index kept)
// starting at entry estart.  Neighbours of a kept entry lie in the same
// component, so their local numbers come from the sorted block itself.
template <int BLOCK, int CAP, int MS = 1>
__device__ __forceinline__ void induce_component(
    int q, int st, int estart, const int32_t *__restrict__ members,
    const uint8_t *__restrict__ flags,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col,
    int32_t *__restrict__ perm, int32_t *__restrict__ lidx, int32_t *__restrict__ loc_row_ptr,
    int32_t *__restrict__ loc_col, int32_t *__restrict__ loc_eid, int32_t *a,
    int32_t *sh_scan) {
  sort_component_block<BLOCK, CAP, MS>(q, st, members, perm, lidx, a, false);  // ends with a barrier
  const bool in_lds = q <= CAP;
  int carry = 0;
  for (int base = 0; base < q; base += BLOCK) {
    const int i = base + threadIdx.x;
    int32_t v = -1, b = 0;
    uint32_t f = 0;
    if (i < q) {
      v = in_lds ? a[i] : perm[st + i];
      f = flags[v];
      b = row_ptr[v];  // with the flags, before the scan
    }
    const int32_t deg = (int32_t)(((f >> 1) & 1) + ((f >> 2) & 1));
    int32_t tot;
    const int32_t ex = block_excl_scan<int32_t, BLOCK>(deg, sh_scan, &tot);
    if (i < q) {
      int32_t r = estart + carry + ex;
      loc_row_ptr[st + i] = r;
      for (int j = 0; j < 2; ++j) {
        if (!(f & (2u << j))) continue;
        const int32_t u = col[b + j];
        int32_t li;
        if (in_lds) {
          int lo = 0, hi = q - 1;  // u is in the sorted block
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a[mid] < u) lo = mid + 1;
            else hi = mid;
          }
          li = st + lo;
        } else {
          li = lidx[u];
        }
        loc_col[r] = li;
        loc_eid[r] = b + j;
        ++r;
      }
    }
    carry += tot;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// LocalAssembly: chain walk of one component, packed base access
// ---------------------------------------------------------------------------
constexpr int kWalkBlock = 256;
constexpr int kWalkCap = 1024;               // reads per component handled in LDS
// small components: one wave each, so many more are walked at once
constexpr int kWalkSmallBlock = 64;
constexpr int kWalkSmallCap = 128;

// Where a piece starts in the store, as the copy needs it (Section 4.4: the
// piece is bases [skip, skip + plen) of its read in walking orientation).
// Bits 0-62: forward, the stored base of the piece's first base; reverse,
// one past the stored base of its first base (the piece is read backwards
// from there).  Bit 63: the read is walked reverse-complemented.  A read
// ends inside the store (read_off + read_len <= 16 seq_words), so the base
// offset stays below 2^63.
__device__ __forceinline__ uint64_t piece_anchor(uint64_t roff, uint32_t rlen, uint32_t skip,
                                                 bool rev) {
  return rev ? ((roff + rlen - skip) | (1ull << 63)) : roff + skip;
}

struct WalkArrays {
  int32_t *nb;     // [2q] local neighbour of slot k of read i (-1: none / cut)
  int32_t *eid;    // [2q] entry index in S of that slot
  int32_t *nxt;    // [2q] ray successor
  int32_t *dist;   // [2q] ray length
  int32_t *endv;   // [2q] ray end
  // the LDS form also keeps what the pieces need, loaded before the doubling:
  int32_t *vid;    // [q] read id of local read i
  uint32_t *rlen;  // [q] its length
  uint64_t *roff;  // [q] its first base in the store
  uint8_t *es;     // [2q] strand bits of the entry of slot k
  uint32_t *eo;    // [2q] its pre (explicit coordinates) or overlap length
  uint32_t *ep;    // [2q] its post (explicit coordinates)
};

template <int BLOCK, int CAP, bool kLds>
__device__ __forceinline__ void walk_component(
    int c, int q, int st, WalkArrays w, const cg_graph &g, const cg_parts &parts,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ loc_row_ptr,
    const int32_t *__restrict__ loc_col, const int32_t *__restrict__ loc_eid,
    const cg_contigs &out, const Scratch &s, int32_t *sh_small, uint32_t *sh_scan);

// What a component's contig record takes from the component table: its
// record index (the component's (bin, label) rank), label and bin.  Loaded
// when the component's work starts, so that no load waits at its end.
struct CompRec {
  int32_t rank, label, bin;
};
__device__ __forceinline__ CompRec comp_rec(const cg_parts &parts, int c, int32_t rank) {
  return CompRec{rank, ((const CG_GLOBAL int32_t *)parts.comp_label)[c],
                 ((const CG_GLOBAL int32_t *)parts.comp_bin)[c]};
}
__device__ __forceinline__ CompRec comp_rec(const cg_parts &parts, int c) {
  return comp_rec(parts, c, ((const CG_GLOBAL int32_t *)parts.comp_rank)[c]);
}

// Steps 2-5 of the walk, from the component's rows in w (nb, eid; and in the
// LDS form vid, rlen, roff, es, eo, ep).
template <int BLOCK, int CAP, bool kLds>
__device__ __forceinline__ void walk_chain(const CompRec &cr, int q, int st, WalkArrays w,
                                           const cg_graph &g, const int32_t *__restrict__ perm,
                                           const cg_contigs &out, const Scratch &s,
                                           uint32_t *sh_scan);

template <int BLOCK, int CAP, bool kLds>
__device__ __forceinline__ void walk_component(
    int c, int q, int st, WalkArrays w, const cg_graph &g, const cg_parts &parts,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ loc_row_ptr,
    const int32_t *__restrict__ loc_col, const int32_t *__restrict__ loc_eid,
    const cg_contigs &out, const Scratch &s, int32_t *sh_small, uint32_t *sh_scan) {
  const int tid = threadIdx.x;
  const CompRec cr = comp_rec(parts, c);
  // 1. local rows of the component's block
  if constexpr (kLds) {
    // and, in three rounds of loads issued together, the read ids and
    // lengths and the entries' strand bits and overlaps (or coordinates)
    constexpr int R = CAP / BLOCK;
    const CG_GLOBAL int32_t *lrp = (const CG_GLOBAL int32_t *)loc_row_ptr;
    const CG_GLOBAL int32_t *lcol = (const CG_GLOBAL int32_t *)loc_col;
    const CG_GLOBAL int32_t *leid = (const CG_GLOBAL int32_t *)loc_eid;
    const CG_GLOBAL int32_t *gperm = (const CG_GLOBAL int32_t *)perm;
    const CG_GLOBAL uint32_t *glen = (const CG_GLOBAL uint32_t *)g.read_len;
    const CG_GLOBAL uint64_t *goff = (const CG_GLOBAL uint64_t *)g.read_off;
    const CG_GLOBAL uint8_t *gstr = (const CG_GLOBAL uint8_t *)g.strand;
    const CG_GLOBAL uint32_t *gov =
        (const CG_GLOBAL uint32_t *)(g.pre ? g.pre : g.ovl);
    const CG_GLOBAL uint32_t *gpost = (const CG_GLOBAL uint32_t *)g.post;
    int ra[R], rd[R], rv[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = tid + u * BLOCK;
      ra[u] = rd[u] = rv[u] = 0;
      if (i < q) {
        ra[u] = lrp[st + i];
        rd[u] = lrp[st + i + 1];
        rv[u] = gperm[st + i];
      }
    }
    int c0[R], c1[R], e0[R], e1[R];
    uint32_t rl[R];
    uint64_t ro[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = tid + u * BLOCK;
      const int deg = i < q ? rd[u] - ra[u] : 0;
      c0[u] = c1[u] = e0[u] = e1[u] = -1;
      rl[u] = 0;
      ro[u] = 0;
      if (i < q) {
        rl[u] = glen[rv[u]];
        ro[u] = goff[rv[u]];
      }
      if (deg >= 1) {
        c0[u] = lcol[ra[u]];
        e0[u] = leid[ra[u]];
      }
      if (deg >= 2) {
        c1[u] = lcol[ra[u] + 1];
        e1[u] = leid[ra[u] + 1];
      }
    }
    uint32_t s0[R], s1[R], o0[R], o1[R], p0[R], p1[R];
#pragma unroll
    for (int u = 0; u < R; ++u) {
      s0[u] = s1[u] = o0[u] = o1[u] = p0[u] = p1[u] = 0;
      if (e0[u] >= 0) {
        s0[u] = gstr[e0[u]];
        o0[u] = gov[e0[u]];
        if (gpost) p0[u] = gpost[e0[u]];
      }
      if (e1[u] >= 0) {
        s1[u] = gstr[e1[u]];
        o1[u] = gov[e1[u]];
        if (gpost) p1[u] = gpost[e1[u]];
      }
    }
#pragma unroll
    for (int u = 0; u < R; ++u) {
      const int i = tid + u * BLOCK;
      if (i >= q) continue;
      w.nb[2 * i] = c0[u] >= 0 ? c0[u] - st : -1;
      w.nb[2 * i + 1] = c1[u] >= 0 ? c1[u] - st : -1;
      w.eid[2 * i] = e0[u];
      w.eid[2 * i + 1] = e1[u];
      w.vid[i] = rv[u];
      w.rlen[i] = rl[u];
      w.roff[i] = ro[u];
      w.es[2 * i] = (uint8_t)s0[u];
      w.es[2 * i + 1] = (uint8_t)s1[u];
      w.eo[2 * i] = o0[u];
      w.eo[2 * i + 1] = o1[u];
      w.ep[2 * i] = p0[u];
      w.ep[2 * i + 1] = p1[u];
    }
  } else {
    for (int i = tid; i < q; i += BLOCK) {
      const int a = loc_row_ptr[st + i], b = loc_row_ptr[st + i + 1];
      const int deg = b - a;
      w.nb[2 * i] = deg >= 1 ? loc_col[a] - st : -1;
      w.nb[2 * i + 1] = deg >= 2 ? loc_col[a + 1] - st : -1;
      w.eid[2 * i] = deg >= 1 ? loc_eid[a] : -1;
      w.eid[2 * i + 1] = deg >= 2 ? loc_eid[a + 1] : -1;
    }
  }
  __syncthreads();
  walk_chain<BLOCK, CAP, kLds>(cr, q, st, w, g, perm, out, s, sh_scan);
  (void)sh_small;
}

template <int BLOCK, int CAP, bool kLds>
__device__ __forceinline__ void walk_chain(const CompRec &cr, int q, int st, WalkArrays w,
                                           const cg_graph &g, const int32_t *__restrict__ perm,
                                           const cg_contigs &out, const Scratch &s,
                                           uint32_t *sh_scan) {
  const int tid = threadIdx.x;
  // the LDS form orders LDS only at its barriers (its global stores stay in
  // flight; nothing it reads back from global memory was written here); the
  // global form's arrays are global memory
  auto wbar = [] {
    if constexpr (kLds) lds_barrier();
    else __syncthreads();
  };
  __shared__ int s_start, s_cyc, s_sej;
  __shared__ uint64_t s_carry;
  if (tid == 0) {
    s_start = 0x7FFFFFFF;
    s_cyc = 0;
    s_sej = 0;
    s_carry = 0;
  }
  wbar();
  // 2. start: the first read of local degree 1 (the smaller-id root, since
  // the block is in id order); a cycle starts at its first read and loses
  // the edge to the larger-numbered neighbour of it
  for (int i = tid; i < q; i += BLOCK)
    if ((w.nb[2 * i] >= 0) != (w.nb[2 * i + 1] >= 0)) atomicMin(&s_start, i);
  wbar();
  if (tid == 0) {
    if (s_start == 0x7FFFFFFF) {
      s_start = 0;
      if (q > 1) {
        s_cyc = 1;
        const int x = w.nb[0], y = w.nb[1];
        const int t = x > y ? x : y;  // closing neighbour
        if (x > y) w.nb[0] = -1; else w.nb[1] = -1;
        if (w.nb[2 * t] == 0) w.nb[2 * t] = -1; else w.nb[2 * t + 1] = -1;
      }
    }
  }
  wbar();
  const int s0 = s_start;
  // 3. rays (i, k): leave read i through slot k.  A ray jumps along the
  // chain; after ceil(log2 q) doublings it knows the chain end it reaches and
  // how many steps away that end is.
  for (int r = tid; r < 2 * q; r += BLOCK) {
    const int y = w.nb[r];
    if (y < 0) {
      w.nxt[r] = -1;
      w.dist[r] = 0;
      w.endv[r] = -1;
    } else {
      const int i = r >> 1;
      const int k2 = w.nb[2 * y] == i ? 1 : 0;  // y's slot that does not lead back
      const int z = w.nb[2 * y + k2];
      w.nxt[r] = z >= 0 ? 2 * y + k2 : -1;
      w.dist[r] = 1;
      w.endv[r] = y;
    }
  }
  wbar();
  for (int span = 1; span < q; span <<= 1) {
    if (kLds && BLOCK == kWave) {
      // one wave: the rays' successors, then the successors' fields, each
      // round of a lane's LDS loads issued together (indices in bounds,
      // results selected after), so a doubling step waits for two rounds of
      // loads (in a 256-thread workgroup this measured no better)
      constexpr int U = 2 * CAP / BLOCK;
      int xr[U], rn[U], rd[U], re[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = tid + u * BLOCK;
        xr[u] = r < 2 * q ? w.nxt[r] : -1;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = tid + u * BLOCK;
        const int x = xr[u] >= 0 ? xr[u] : 0;
        rn[u] = w.nxt[x];
        rd[u] = w.dist[r] + w.dist[x];
        re[u] = w.endv[x];
      }
      wbar();
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int r = tid + u * BLOCK;
        if (xr[u] >= 0) {
          w.nxt[r] = rn[u];
          w.dist[r] = rd[u];
          w.endv[r] = re[u];
        }
      }
      wbar();
    } else if (kLds) {
      int rn[(2 * CAP / BLOCK)], rd[(2 * CAP / BLOCK)], re[(2 * CAP / BLOCK)];
#pragma unroll
      for (int u = 0; u < (2 * CAP / BLOCK); ++u) {
        const int r = tid + u * BLOCK;
        rn[u] = -2;
        if (r < 2 * q) {
          const int x = w.nxt[r];
          if (x >= 0) {
            rn[u] = w.nxt[x];
            rd[u] = w.dist[r] + w.dist[x];
            re[u] = w.endv[x];
          }
        }
      }
      wbar();
#pragma unroll
      for (int u = 0; u < (2 * CAP / BLOCK); ++u) {
        const int r = tid + u * BLOCK;
        if (rn[u] != -2) {
          w.nxt[r] = rn[u];
          w.dist[r] = rd[u];
          w.endv[r] = re[u];
        }
      }
      wbar();
    } else {
      // large component (global arrays): ray r's successor x is only
      // rewritten by its own owner, so read all then write all in two passes
      // with the new values parked in the endv/dist of the high half
      for (int r = tid; r < 2 * q; r += BLOCK) {
        const int x = w.nxt[r];
        if (x >= 0) {
          // encode the update next to the ray: (new nxt, new dist, new end)
          w.nxt[2 * q + r] = w.nxt[x];
          w.dist[2 * q + r] = w.dist[r] + w.dist[x];
          w.endv[2 * q + r] = w.endv[x];
        } else {
          w.nxt[2 * q + r] = -2;
        }
      }
      wbar();
      for (int r = tid; r < 2 * q; r += BLOCK) {
        const int x = w.nxt[2 * q + r];
        if (x != -2) {
          w.nxt[r] = x;
          w.dist[r] = w.dist[2 * q + r];
          w.endv[r] = w.endv[2 * q + r];
        }
      }
      wbar();
    }
  }
  // 4. rank, predecessor, successor, orientation and piece of every read
  int32_t *R_vid = out.layout_vid + st;
  uint8_t *R_rev = out.layout_rev + st;
  uint32_t *R_len = s.piece_len + st;
  uint64_t *R_src = s.piece_src + st;
  const int rank_c = cr.rank;
  for (int i = tid; i < q; i += BLOCK) {
    int rank = 0, pred = -1, succ = -1, succ_e = -1;
    int ss = -1;  // slot of i leading to its successor
    if (i == s0) {
      if (w.nb[2 * i] >= 0) ss = 2 * i;
      else if (w.nb[2 * i + 1] >= 0) ss = 2 * i + 1;
    } else {
      for (int k = 0; k < 2; ++k) {
        if (w.nb[2 * i + k] >= 0 && w.endv[2 * i + k] == s0) {
          rank = w.dist[2 * i + k];
          pred = w.nb[2 * i + k];
          const int o = 1 - k;
          if (w.nb[2 * i + o] >= 0) ss = 2 * i + o;
        }
      }
    }
    if (ss >= 0) {
      succ = w.nb[ss];
      succ_e = w.eid[ss];
    }
    int ps = -1;  // slot of pred leading to i (its entry pred -> i)
    if (i != s0 && pred >= 0) ps = w.nb[2 * pred] == i ? 2 * pred : 2 * pred + 1;
    // strand bits, overlap or coordinates of the two entries, and the read
    const int32_t v = kLds ? w.vid[i] : perm[st + i];
    const uint32_t L = kLds ? w.rlen[i] : g.read_len[v];
    const uint64_t roff = kLds ? w.roff[i] : g.read_off[v];
    const uint32_t ses = ss < 0 ? 0u : (kLds ? w.es[ss] : (uint32_t)g.strand[succ_e]);
    const uint32_t pes = ps < 0 ? 0u : (kLds ? w.es[ps] : (uint32_t)g.strand[w.eid[ps]]);
    int orient;
    if (i == s0) orient = ss >= 0 ? (int)(ses & 1) : 0;
    else if (ps >= 0) orient = (int)((pes >> 1) & 1);
    else orient = 0;  // unreachable for a chain: every read but the start has a predecessor
    // the piece: walking offsets [skip, end] of the read (Section 4.4: from
    // post of the entering entry to pre of the leaving one, in stored
    // coordinates; from overlap lengths: the read minus its overlap with the
    // successor)
    uint32_t skip = 0, plen = L;
    if (g.pre) {
      const uint32_t post_in = ps < 0 ? 0u : (kLds ? w.ep[ps] : g.post[w.eid[ps]]);
      const uint32_t pre_out = ss < 0 ? 0u : (kLds ? w.eo[ss] : g.pre[succ_e]);
      const int64_t first = ps >= 0 ? (orient ? (int64_t)L - 1 - post_in : post_in) : 0;
      const int64_t last =
          ss >= 0 ? (orient ? (int64_t)L - 1 - pre_out : pre_out) : (int64_t)L - 1;
      skip = (uint32_t)first;
      plen = last >= first ? (uint32_t)(last - first + 1) : 0u;
    } else if (ss >= 0) {
      plen -= kLds ? w.eo[ss] : g.ovl[succ_e];
    }
    if (ss >= 0 && (int)(ses & 1) != orient) s_sej = 1;
    R_vid[rank] = v;
    R_rev[rank] = (uint8_t)orient;
    R_len[rank] = plen;
    if constexpr (kLds) w.nxt[rank] = (int32_t)plen;  // nxt is free after the rays
    R_src[rank] = piece_anchor(roff, L, skip, orient != 0);
    s.lay_contig[st + rank] = rank_c;
    (void)succ;
  }
  wbar();
  // 5. piece offsets in walk order
  for (int base = 0; base < q; base += BLOCK) {
    const int i = base + tid;
    const uint32_t x = i < q ? (kLds ? (uint32_t)w.nxt[i] : R_len[i]) : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t, BLOCK, kLds>(x, sh_scan, &tot);
    if (i < q) s.piece_off[st + i] = s_carry + ex;
    wbar();
    if (tid == 0) s_carry += tot;
    wbar();
  }
  if (tid == 0) {
    out.label[rank_c] = cr.label;
    out.bin[rank_c] = cr.bin;
    out.start[rank_c] = kLds ? w.vid[s0] : perm[st + s0];
    out.n_reads[rank_c] = q;
    out.len[rank_c] = s_carry;
    out.cflags[rank_c] = (q == 1 ? CG_CONTIG_SINGLE : 0u) | (s_cyc ? CG_CONTIG_CIRCULAR : 0u) |
                         (s_sej ? CG_CONTIG_SAME_END_JOIN : 0u);
    out.layout_off[rank_c] = st;
  }
  wbar();
}

// ---------------------------------------------------------------------------
// Packed base copy
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t rev_fields32(uint32_t v) {
  const uint32_t y = __builtin_bitreverse32(v);
  return ((y >> 1) & 0x55555555u) | ((y & 0x55555555u) << 1);
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// One piece as the copy needs it.
struct PieceD {
  uint64_t a;     // piece_anchor without its strand bit
  uint64_t poff;  // first base of the piece in its contig
  uint64_t L;     // contig length
  uint64_t cb;    // first output word of the contig
  uint32_t plen;  // piece length
  int32_t rev;    // read walked reverse-complemented
};

// The per-piece arrays are read in piece order (coalesced across a wave's
// lanes); only the two per-contig arrays are gathered.
struct PieceArrays {
  const CG_GLOBAL int32_t *lay_contig;
  const CG_GLOBAL uint64_t *piece_off;
  const CG_GLOBAL uint32_t *piece_len;
  const CG_GLOBAL uint64_t *piece_src;
  const CG_GLOBAL uint64_t *clen;
  const CG_GLOBAL uint64_t *cbase;
};

__device__ __forceinline__ PieceArrays piece_arrays(const int32_t *lay_contig,
                                                    const uint64_t *piece_off,
                                                    const uint32_t *piece_len,
                                                    const uint64_t *piece_src,
                                                    const uint64_t *clen, const uint64_t *cbase) {
  return PieceArrays{(const CG_GLOBAL int32_t *)lay_contig, (const CG_GLOBAL uint64_t *)piece_off,
                     (const CG_GLOBAL uint32_t *)piece_len, (const CG_GLOBAL uint64_t *)piece_src,
                     (const CG_GLOBAL uint64_t *)clen,      (const CG_GLOBAL uint64_t *)cbase};
}

__device__ __forceinline__ PieceD load_piece(const PieceArrays &A, int32_t p) {
  PieceD d;
  const int32_t k = A.lay_contig[p];
  const uint64_t a = A.piece_src[p];
  d.a = a & ~(1ull << 63);
  d.rev = (int32_t)(a >> 63);
  d.plen = A.piece_len[p];
  d.poff = A.piece_off[p];
  d.L = A.clen[k];
  d.cb = A.cbase[k] >> 4;
  return d;
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int t) {
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, t);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), t);
  return ((uint64_t)hi << 32) | lo;
}

// Store word index clamped into [0, nwords - 1]; a window may start before
// the store (reverse pieces of the first reads) or end after it, and the
// words it then reads are never used.
__device__ __forceinline__ uint64_t clamp_word(int64_t w, uint64_t nwords) {
  return w < 0 ? 0 : ((uint64_t)w >= nwords ? nwords - 1 : (uint64_t)w);
}

// 16 stored bases starting at base b (any alignment, b taken as signed) as
// one word: a 64-bit funnel shift of two store words.
__device__ __forceinline__ uint32_t window16(const CG_GLOBAL uint32_t *__restrict__ seq,
                                             uint64_t nwords, uint64_t b) {
  const int64_t w = (int64_t)b >> 4;
  const uint32_t lo = seq[clamp_word(w, nwords)];
  const uint32_t hi = seq[clamp_word(w + 1, nwords)];
  return __builtin_amdgcn_alignbit(hi, lo, 2u * (uint32_t)(b & 15));
}

// reverse the 16 2-bit fields of a word and complement them
__device__ __forceinline__ uint32_t revcomp16(uint32_t x) { return ~rev_fields32(x); }

__device__ __forceinline__ uint32_t low_fields(int k) {
  return k >= 16 ? 0xFFFFFFFFu : ((1u << (2 * k)) - 1u);
}

// Stored base where the 16-base window holding a piece's first 16 bases (in
// walking orientation) starts: forward at the piece's first base, reverse 15
// bases below it (the window is then read backwards).  a is the piece's
// anchor without its strand bit.
__device__ __forceinline__ uint64_t head_src(uint64_t a, bool rev) { return rev ? a - 16 : a; }

// The first k (<= 16) bases of a piece in walking orientation, in fields 0..k-1
// (fields above k are not cleared).
__device__ __forceinline__ uint32_t piece_head16(const CG_GLOBAL uint32_t *__restrict__ seq,
                                                 uint64_t nwords, const PieceD &f) {
  const uint32_t x = window16(seq, nwords, head_src(f.a, f.rev != 0));
  return f.rev ? revcomp16(x) : x;
}

// Copy descriptor of one piece: output words [w0, w0 + nw) of the bases
// array are the words whose first base lies in the piece.
//   sw0   store word at which the window of the piece's first group (output
//         word w0) starts; the group at word w0 + k starts at sw0 + k
//         (forward) or sw0 - k (reverse).  Signed: a reverse window may start
//         before the store.  Forward, output word w begins at stored base
//         16 sw0 + sh/2 + 16 (w - w0); reverse, the (16 kGroupWords)-base
//         window of the group at word w begins there with w0 - w in place of
//         w - w0.
//   info  bits 0-4: bases of the piece in its last owned word (1..16);
//         bit 5: reverse; bit 6: the piece ends its contig; bits 8-11: the
//         window's first base within its first store word (the funnel shift
//         is twice that)
struct CopyD {
  int64_t sw0;
  uint64_t w0;
  uint32_t nw, info;
};

// words per group: a lane's share of one row of a step
constexpr int kGroupWords = 4;
static_assert(kGroupWords % 4 == 0, "groups are moved in 16-byte units");
// What a word straddling into the next piece needs of it.
struct CopyE {
  uint64_t hsrc;   // head_src of the piece
  uint32_t info;   // plen | reverse << 30 | ends its contig << 31
};

__device__ __forceinline__ CopyD copy_desc(const PieceD &d) {
  CopyD c;
  const uint64_t pend = d.poff + d.plen;
  const uint64_t j0 = (d.poff + 15) >> 4, j1 = (pend + 15) >> 4;
  c.w0 = d.cb + j0;
  c.nw = (uint32_t)(j1 - j0);
  const uint32_t fs = (uint32_t)(pend - 16 * (j1 - 1));
  // stored base where the window of the first group begins (modulo 2^64)
  const uint64_t sb0 = d.rev ? d.a - 16 * kGroupWords + d.poff - 16 * j0 : d.a - d.poff + 16 * j0;
  c.sw0 = (int64_t)sb0 >> 4;
  c.info = fs | (d.rev ? 32u : 0u) | (pend == d.L ? 64u : 0u) | ((uint32_t)(sb0 & 15) << 8);
  return c;
}

__device__ __forceinline__ CopyE copy_next(const PieceD &e) {
  CopyE c;
  c.hsrc = head_src(e.a, e.rev != 0);
  c.info = e.plen | (e.rev ? (1u << 30) : 0u) | (e.poff + e.plen == e.L ? (1u << 31) : 0u);
  return c;
}

constexpr int kCopyUnroll = 2;  // groups per lane per step

// One step of the copy: kCopyUnroll groups per lane (groups g, g + 64, ...),
// their pieces' descriptors and store windows.
struct CopyStage {
  uint32_t win[kCopyUnroll][kGroupWords + 1];  // the last word only where the neighbouring
                                               // lane lacks it (nb)
  uint32_t hlo[kCopyUnroll], hhi[kCopyUnroll];  // store words of the next piece's head
  CopyD d[kCopyUnroll];
  CopyE e[kCopyUnroll];
  uint32_t k[kCopyUnroll];
  int t[kCopyUnroll];
  bool ok[kCopyUnroll];
  bool nb[kCopyUnroll];  // the last word is word 0 of the next group's window, held by
                         // lane l + 1 (forward) or l - 1 (reverse)
};


// Find the pieces of a step's groups and start its loads.
__device__ __forceinline__ void copy_fetch(CopyStage &S, uint32_t gb, uint32_t G, uint32_t gstart,
                                           const CopyD &my, const CopyE &nx,
                                           const CG_GLOBAL uint32_t *__restrict__ seq,
                                           uint64_t nwords, int lane) {
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) S.t[u] = 0;
  // piece of group g: the last lane t with gstart[t] <= g (gstart is
  // non-decreasing and equals G from lane cnt on, so t < cnt when g < G).
  // Six fixed steps, every lane shuffling in every step: a shuffle must
  // never run with part of the wave switched off.
#pragma unroll
  for (int step = kWave / 2; step > 0; step >>= 1) {
#pragma unroll
    for (int u = 0; u < kCopyUnroll; ++u) {
      const uint32_t g = gb + lane + kWave * u;
      const uint32_t sm = __shfl(gstart, S.t[u] + step);
      if (sm <= g) S.t[u] += step;
    }
  }
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const int t = S.t[u];
    S.d[u].sw0 = __shfl(my.sw0, t);
    S.d[u].w0 = __shfl(my.w0, t);
    S.d[u].nw = __shfl(my.nw, t);
    S.d[u].info = __shfl(my.info, t);
    S.e[u].hsrc = __shfl(nx.hsrc, t);
    S.e[u].info = __shfl(nx.info, t);
    const uint32_t gs = __shfl(gstart, t);
    const uint32_t g = gb + lane + kWave * u;
    S.ok[u] = g < G;
    S.k[u] = S.ok[u] ? kGroupWords * (g - gs) : 0;  // first owned word of the group
  }
  // loads only, so that nothing here waits for memory and the step's loads
  // stay in flight while the previous step is finished
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    const CopyD &d = S.d[u];
    const bool rev = d.info & 32u;
    // the piece's window: kGroupWords + 1 store words covering the group's
    // bases, as 16-byte loads (dword aligned) and a dword; clamped word by
    // word at the ends of the store, where the words outside it are never used
    const int64_t sw = S.ok[u] ? (rev ? d.sw0 - (int64_t)S.k[u] : d.sw0 + (int64_t)S.k[u]) : 0;
    // the neighbouring lane's group is the next one of the same piece: its
    // window starts at the last word of this one
    // (both shifts by every lane, then the choice: a shift must never run
    // with part of the wave switched off)
    const uint32_t tk = (uint32_t)S.t[u] | (S.ok[u] ? 0x80000000u : 0u);
    const uint32_t tprev = wave_prev_u32(tk), tnext = wave_next_u32(tk);
    const uint32_t tnb = rev ? tprev : tnext;
    const int tn = (int)(tnb & 0x7FFFFFFFu);
    const bool okn = (tnb >> 31) != 0u;
    const bool edge = rev ? lane == 0 : lane == kWave - 1;
    S.nb[u] = false;
    if (sw >= 0 && sw + kGroupWords + 1 <= (int64_t)nwords) {
#pragma unroll
      for (int v = 0; v < kGroupWords / 4; ++v) {
        u32x4 a;
        __builtin_memcpy(&a, seq + sw + 4 * v, 16);
        S.win[u][4 * v] = a.x;
        S.win[u][4 * v + 1] = a.y;
        S.win[u][4 * v + 2] = a.z;
        S.win[u][4 * v + 3] = a.w;
      }
      S.nb[u] = S.ok[u] && okn && !edge && tn == S.t[u];
      S.win[u][kGroupWords] = S.nb[u] ? 0u : seq[sw + kGroupWords];
    } else {
#pragma unroll
      for (int i = 0; i <= kGroupWords; ++i) S.win[u][i] = seq[clamp_word(sw + i, nwords)];
    }
    // the next piece's first 16 bases, for the group holding the piece's
    // last word
    S.hlo[u] = S.hhi[u] = 0;
    if (S.ok[u] && S.k[u] + kGroupWords >= d.nw) {
      const int64_t hw = (int64_t)S.e[u].hsrc >> 4;
      S.hlo[u] = seq[clamp_word(hw, nwords)];
      S.hhi[u] = seq[clamp_word(hw + 1, nwords)];
    }
  }
}

// Finish a step: words from the windows, the pieces' last words, stores.
__device__ __forceinline__ void copy_emit(const CopyStage &S, const PieceArrays &A, int32_t c0,
                                          int32_t n_e, const CG_GLOBAL uint32_t *__restrict__ seq,
                                          uint64_t nwords, CG_GLOBAL uint32_t *__restrict__ bases) {
#pragma unroll
  for (int u = 0; u < kCopyUnroll; ++u) {
    // the last window word from the neighbouring lane, while every lane is
    // still active
    const uint32_t up = wave_next_u32(S.win[u][0]), dn = wave_prev_u32(S.win[u][0]);
    if (!S.ok[u]) continue;
    const CopyD &d = S.d[u];
    const bool rev = d.info & 32u;
    uint32_t win[kGroupWords + 1];
#pragma unroll
    for (int i = 0; i < kGroupWords; ++i) win[i] = S.win[u][i];
    win[kGroupWords] = S.nb[u] ? (rev ? dn : up) : S.win[u][kGroupWords];
    const uint32_t sh = 2u * ((d.info >> 8) & 15u);
    const uint32_t nw = d.nw - S.k[u] < kGroupWords ? d.nw - S.k[u] : kGroupWords;
    uint32_t out[kGroupWords];
#pragma unroll
    for (int i = 0; i < kGroupWords; ++i)
      out[i] = rev ? revcomp16(__builtin_amdgcn_alignbit(win[kGroupWords - i],
                                                         win[kGroupWords - 1 - i], sh))
                   : __builtin_amdgcn_alignbit(win[i + 1], win[i], sh);
    const int fs = (int)(d.info & 31u);
    if (S.k[u] + nw == d.nw && fs < 16) {
      // the piece's last word: its own fs bases, then the next piece(s) or
      // zero padding at the contig's end
      uint32_t x = out[nw - 1] & low_fields(fs);
      if (!(d.info & 64u)) {
        const CopyE &e = S.e[u];
        const int pl = (int)(e.info & 0x3FFFFFFFu);
        const int k2 = 16 - fs < pl ? 16 - fs : pl;
        const bool erev = e.info & (1u << 30);
        uint32_t head =
            __builtin_amdgcn_alignbit(S.hhi[u], S.hlo[u], 2u * (uint32_t)(e.hsrc & 15));
        if (erev) head = revcomp16(head);
        x |= (head & low_fields(k2)) << (2 * fs);
        int filled = fs + k2;
        // pieces shorter than the rest of the word: take the following ones
        if (filled < 16 && !(e.info & (1u << 31))) {
          for (int32_t pp = c0 + S.t[u] + 2; filled < 16 && pp < n_e; ++pp) {
            const PieceD f = load_piece(A, pp);
            const int k3 = 16 - filled < (int)f.plen ? 16 - filled : (int)f.plen;
            const uint32_t y = piece_head16(seq, nwords, f);
            x |= (y & low_fields(k3)) << (2 * filled);
            filled += k3;
            if (f.poff + f.plen == f.L) break;
          }
        }
      }
      out[nw - 1] = x;
    }
    CG_GLOBAL uint32_t *o = bases + d.w0 + S.k[u];
    if (nw == kGroupWords) {
#pragma unroll
      for (int v = 0; v < kGroupWords / 4; ++v) {
        const u32x4 x4 = {out[4 * v], out[4 * v + 1], out[4 * v + 2], out[4 * v + 3]};
        __builtin_memcpy(o + 4 * v, &x4, 16);  // 16-byte stores, dword aligned
      }
    } else {
#pragma unroll
      for (int i = 0; i < kGroupWords; ++i)
        if (i < (int)nw) o[i] = out[i];
    }
  }
}

// One wave copies the chunk of cnt (<= 64) consecutive pieces starting at
// piece c0 of a graph with n_e pieces.  Lane l gathers piece c0+l's
// descriptor; the chunk's kGroupWords-word groups (each owned by the piece holding
// the first base of its words) are then spread over the lanes, 64 groups per
// row, so lanes of one row work on different pieces.  Every word is a
// funnel shift of two store words, reverse-complemented in registers for a
// reverse piece; only a piece's last word can run into the next piece(s).
// Steps are software-pipelined: the loads of step s + 1 are issued before
// step s is finished, so a wave always has loads in flight.
// c0, cnt and n_e are wave-uniform; every lane runs every step.
__device__ __forceinline__ void copy_chunk(const uint32_t *seq_, uint64_t nwords, uint32_t *bases_,
                                           const PieceArrays &A, int32_t c0, int cnt,
                                           int32_t n_e, int lane) {
  const CG_GLOBAL uint32_t *seq = (const CG_GLOBAL uint32_t *)seq_;
  CG_GLOBAL uint32_t *bases = (CG_GLOBAL uint32_t *)bases_;
  CopyD my{};
  uint32_t ng = 0;
  PieceD pd{};
  if (lane < cnt) {
    pd = load_piece(A, c0 + lane);
    my = copy_desc(pd);
    ng = (my.nw + kGroupWords - 1) / kGroupWords;
  }
  // the next piece of every lane's piece: from the next lane, or loaded for
  // the chunk's last piece
  CopyE nx;
  {
    const CopyE mine = copy_next(pd);
    nx.hsrc = __shfl_down(mine.hsrc, 1);
    nx.info = __shfl_down(mine.info, 1);
    if (lane == cnt - 1 && c0 + lane + 1 < n_e) nx = copy_next(load_piece(A, c0 + lane + 1));
  }
  const uint32_t gincl = wave_incl_scan(ng);
  const uint32_t gstart = gincl - ng;
  const uint32_t G = __shfl(gincl, kWave - 1);
  constexpr uint32_t kStep = kWave * kCopyUnroll;
  CopyStage S0, S1;
  if (G > 0) copy_fetch(S0, 0, G, gstart, my, nx, seq, nwords, lane);
  for (uint32_t gb = 0; gb < G; gb += 2 * kStep) {
    if (gb + kStep < G) copy_fetch(S1, gb + kStep, G, gstart, my, nx, seq, nwords, lane);
    copy_emit(S0, A, c0, n_e, seq, nwords, bases);
    if (gb + kStep < G) {
      if (gb + 2 * kStep < G) copy_fetch(S0, gb + 2 * kStep, G, gstart, my, nx, seq, nwords, lane);
      copy_emit(S1, A, c0, n_e, seq, nwords, bases);
    }
  }
}

}  // namespace cg
