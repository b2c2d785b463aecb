// Contig sizes and GreedyPartitioning (Sections 4.2 and 4.3).
//
//  k_part_zero / k_part_count  per-label counter (4 per read, +1 per read of
//                              degree 1 in L): size q = c >> 2, roots of degree
//                              one = c & 3 (2 for a path, 0 for a cycle)
//  k_part_compact              eligible components in ascending label order
//                              (single-pass look-back scan), label -> index map
//  k_part_lpt                  one workgroup: sort by (size desc, label asc),
//                              exact LPT, sort by (bin, label), read offsets
#include "cg_internal.h"

namespace cg {

constexpr int kPartBlock = 256;

__global__ __launch_bounds__(kPartBlock) void k_part_zero(int32_t n, int32_t *__restrict__ cnt) {
  const int64_t v = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
  if (v < n) cnt[v] = 0;
}

__global__ __launch_bounds__(kPartBlock) void k_part_count(int32_t n, const uint8_t *__restrict__ flags,
                                                           const int32_t *__restrict__ label,
                                                           int32_t *cnt) {
  const int64_t v = (int64_t)blockIdx.x * kPartBlock + threadIdx.x;
  if (v >= n) return;
  const uint32_t f = flags[v];
  const uint32_t degL = ((f >> 1) & 1) + ((f >> 2) & 1);
  atomicAdd((uint32_t *)cnt + label[v], 4u + (degL == 1 ? 1u : 0u));
}

__global__ __launch_bounds__(kScanBlock) void k_part_compact(
    int32_t n, const uint8_t *__restrict__ flags, int32_t *label_comp, int32_t min_reads,
    int32_t *__restrict__ comp_label, int32_t *__restrict__ comp_size,
    uint8_t *__restrict__ comp_kind, int32_t *__restrict__ d_n_comp, ScanCtx sc, int nblocks) {
  const int blk = lookback_ticket(sc);
  const int64_t v = (int64_t)blk * kScanBlock + threadIdx.x;
  const uint32_t c = v < n ? (uint32_t)label_comp[v] : 0u;
  const uint32_t q = c >> 2;
  const bool elig = v < n && q >= (uint32_t)min_reads && !(flags[v] & 1);
  unsigned long long incl_end;
  const unsigned long long ex = lookback_block_scan(sc, blk, elig ? 1ull : 0ull, &incl_end);
  if (v < n) {
    if (elig) {
      comp_label[ex] = (int32_t)v;
      comp_size[ex] = (int32_t)q;
      comp_kind[ex] = q == 1 ? CG_KIND_SINGLE : ((c & 3u) ? CG_KIND_PATH : CG_KIND_CYCLE);
      label_comp[v] = (int32_t)ex;
    } else {
      label_comp[v] = -1;
    }
  }
  if (blk == nblocks - 1 && threadIdx.x == 0) *d_n_comp = (int32_t)incl_end;
  lookback_finish(sc, nblocks);
}

// ---------------------------------------------------------------------------
// Single-workgroup sort + LPT.
// ---------------------------------------------------------------------------
constexpr int kLptBlock = 1024;
constexpr int kSortCapLds = 8192;  // components sorted in LDS
constexpr int kBinCapLds = 2048;   // bins kept in LDS

__device__ __forceinline__ int next_pow2(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

template <typename K>
__device__ __forceinline__ void bitonic_sort(K *a, int N2) {
  for (int k = 2; k <= N2; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < N2; i += blockDim.x) {
        int ixj = i ^ j;
        if (ixj > i) {
          K x = a[i], y = a[ixj];
          bool up = (i & k) == 0;
          if ((x > y) == up) {
            a[i] = y;
            a[ixj] = x;
          }
        }
      }
      __syncthreads();
    }
  }
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

// Bin keys are (load << 16) | bin: ascending key order is ascending
// (load, bin), i.e. the least loaded bin with the lowest index first.
constexpr int kBinBits = 16;

__device__ __forceinline__ void lpt_body(int nc, int P, const int32_t *__restrict__ comp_size,
                                         uint64_t *keys, int32_t *bin_of, uint64_t *binA,
                                         uint64_t *binB, int32_t *__restrict__ comp_bin,
                                         int32_t *__restrict__ comp_rank,
                                         int32_t *__restrict__ comp_start,
                                         uint64_t *__restrict__ bin_load) {
  __shared__ uint64_t win[kWave];
  __shared__ int32_t sh_scan[kLptBlock / kWave + 1];
  const int tid = threadIdx.x;
  const int N2 = next_pow2(nc > 0 ? nc : 1);

  // 1. sort by (size desc, label asc); components are indexed in label order
  for (int i = tid; i < N2; i += blockDim.x)
    keys[i] = i < nc ? ((uint64_t)(0xFFFFFFFFu - (uint32_t)comp_size[i]) << 32) | (uint32_t)i
                     : ~0ull;
  for (int b = tid; b < P; b += blockDim.x) binA[b] = (uint64_t)b;  // load 0, sorted
  __syncthreads();
  bitonic_sort(keys, N2);

  // 2. LPT.  The bins are kept sorted by (load, bin).  A window holds the W
  // least loaded bins in the lanes of wave 0 (sorted across lanes): each
  // component goes to lane 0's bin, whose new key is then re-inserted by
  // ballot + shift.  Within W steps of a window only its W bins can be the
  // minimum (step t picks a bin of initial rank <= t), so after W steps the
  // window is merged back into the sorted bin list.
  const int W = P < kWave ? P : kWave;
  const bool single_window = P <= kWave;
  int i0 = 0;
  while (i0 < nc) {
    const int T = single_window ? nc - i0 : (nc - i0 < W ? nc - i0 : W);
    if (tid < kWave) {
      const int l = tid;
      uint64_t key = l < W ? binA[l] : ~0ull;
      for (int base = 0; base < T; base += kWave) {
        const int cnt = T - base < kWave ? T - base : kWave;
        const uint64_t item = l < cnt ? keys[i0 + base + l] : 0ull;
        for (int t = 0; t < cnt; ++t) {
          const uint64_t it = __shfl(item, t);
          const uint32_t c = (uint32_t)it;
          const uint64_t q = 0xFFFFFFFFu - (uint32_t)(it >> 32);
          const uint64_t k0 = __shfl(key, 0);
          if (l == 0) bin_of[c] = (int32_t)(k0 & ((1u << kBinBits) - 1));
          const uint64_t nk = k0 + (q << kBinBits);
          const int p = __popcll(__ballot(key < nk)) - 1;  // lanes 1.. below nk
          const uint64_t nxt = __shfl_down(key, 1);
          key = l < p ? nxt : (l == p ? nk : key);
        }
      }
      if (l < W) win[l] = key;
    }
    __syncthreads();
    if (single_window) {
      if (tid < W) binA[tid] = win[tid];
    } else {
      // merge the window (sorted) with binA[W..P) (sorted) into binB
      for (int idx = tid; idx < P; idx += blockDim.x) {
        uint64_t x;
        int pos;
        if (idx < W) {
          x = win[idx];
          pos = idx + lower_bound_u64(binA + W, P - W, x);
        } else {
          x = binA[idx];
          pos = (idx - W) + lower_bound_u64(win, W, x);
        }
        binB[pos] = x;
      }
      __syncthreads();
      uint64_t *t = binA;
      binA = binB;
      binB = t;
    }
    __syncthreads();
    i0 += T;
  }
  for (int b = tid; b < P; b += blockDim.x) {
    const uint64_t k = binA[b];
    bin_load[k & ((1u << kBinBits) - 1)] = k >> kBinBits;
  }

  // 3. (bin, label) order and read offsets
  for (int i = tid; i < N2; i += blockDim.x)
    keys[i] = i < nc ? ((uint64_t)(uint32_t)bin_of[i] << 32) | (uint32_t)i : ~0ull;
  __syncthreads();
  bitonic_sort(keys, N2);
  for (int i = tid; i < nc; i += blockDim.x) comp_bin[i] = bin_of[i];
  int carry = 0;
  for (int base = 0; base < nc; base += kLptBlock) {
    const int i = base + tid;
    const uint32_t c = i < nc ? (uint32_t)keys[i] : 0u;
    const int32_t sz = i < nc ? comp_size[c] : 0;
    int32_t tot;
    const int32_t ex = block_excl_scan<int32_t, kLptBlock>(sz, sh_scan, &tot);
    if (i < nc) {
      comp_start[c] = carry + ex;
      comp_rank[c] = i;
    }
    carry += tot;
  }
}

__global__ __launch_bounds__(kLptBlock) void k_part_lpt(int32_t P, const int32_t *__restrict__ d_n_comp,
                                                        const int32_t *__restrict__ comp_size,
                                                        int32_t *__restrict__ comp_bin,
                                                        int32_t *__restrict__ comp_rank,
                                                        int32_t *__restrict__ comp_start,
                                                        uint64_t *__restrict__ bin_load,
                                                        uint64_t *g_keys, int32_t *g_bin,
                                                        uint64_t *g_bins) {
  __shared__ uint64_t s_keys[kSortCapLds];
  __shared__ int32_t s_bin[kSortCapLds];
  __shared__ uint64_t s_binA[kBinCapLds], s_binB[kBinCapLds];
  const int nc = *d_n_comp;
  if (nc <= kSortCapLds && P <= kBinCapLds)
    lpt_body(nc, P, comp_size, s_keys, s_bin, s_binA, s_binB, comp_bin, comp_rank, comp_start,
             bin_load);
  else
    lpt_body(nc, P, comp_size, g_keys, g_bin, g_bins, g_bins + P, comp_bin, comp_rank, comp_start,
             bin_load);
}

int launch_partition(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const uint8_t *flags,
                     const int32_t *label, int32_t P, int32_t min_reads, const cg_parts &out,
                     hipStream_t st) {
  const int32_t n = g.n;
  if (min_reads < 1) min_reads = 1;
  const int grid = n > 0 ? (int)((n + kPartBlock - 1) / kPartBlock) : 1;
  if (n > 0) {
    CG_LAUNCH(ctx, k_part_zero, dim3(grid), dim3(kPartBlock), st, n, out.label_comp);
    CG_LAUNCH(ctx, k_part_count, dim3(grid), dim3(kPartBlock), st, n, flags, label,
                       out.label_comp);
  }
  const int nb = scan_blocks(n > 0 ? n : 1);
  CG_LAUNCH(ctx, k_part_compact, dim3(nb), dim3(kScanBlock), st, n, flags, out.label_comp,
                     min_reads, out.comp_label, out.comp_size, out.comp_kind, out.d_n_comp,
                     scan_ctx(ctx, s), nb);
  CG_LAUNCH(ctx, k_part_lpt, dim3(1), dim3(kLptBlock), st, P, out.d_n_comp, out.comp_size,
                     out.comp_bin, out.comp_rank, out.comp_start, out.bin_load, s.keys, s.aux,
                     s.bins);
  return hip_check(hipGetLastError(), "k_part");
}

}  // namespace cg
