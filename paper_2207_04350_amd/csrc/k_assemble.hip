// LocalAssembly (Section 4.4).  A contig is the concatenation
//   l_r[alpha:pre(e0)] + l_c1[post(e0):pre(e1)] + ... + l_r'[post(e_{q-2}):beta]
// over the chain r, c1, ..., r' of a component: every read but the last
// contributes the part of its walking orientation that precedes its overlap
// with the next read (len - ovl bases), the last read all its bases.
//
//  k_asm_walk_small  one wave per component of at most kWalkSmallCap reads
//                 (small LDS arrays, so many are walked at once per CU)
//  k_asm_walk     one workgroup per larger component: start read, walk order
//                 by pointer jumping over the chain's arcs (Wyllie list
//                 ranking), orientation from the strand bits, piece lengths
//                 and offsets, layout and contig record
//  k_asm_offsets  contig base offsets (16-base aligned) in (bin, label) order
//  k_asm_copy     chunks of consecutive pieces, one wave each: every output
//                 word is written by the piece holding its first base, 2-bit
//                 funnel shifts for unaligned starts, reverse + complement in
//                 registers
#include "cg_device.h"

namespace cg {

constexpr int32_t kWalkSplitReads = 1 << 19;  // reads from which the walk takes two passes

__global__ __launch_bounds__(kWalkSmallBlock) void k_asm_walk_small(cg_graph g, cg_parts parts,
                                                                   cg_local local, cg_contigs out,
                                                                   Scratch s) {
  __shared__ int32_t s_nb[2 * kWalkSmallCap], s_eid[2 * kWalkSmallCap], s_nxt[2 * kWalkSmallCap],
      s_dist[2 * kWalkSmallCap], s_endv[2 * kWalkSmallCap], s_vid[kWalkSmallCap];
  __shared__ uint32_t s_rlen[kWalkSmallCap], s_eo[2 * kWalkSmallCap], s_ep[2 * kWalkSmallCap];
  __shared__ uint64_t s_roff[kWalkSmallCap];
  __shared__ uint8_t s_es[2 * kWalkSmallCap];
  __shared__ uint32_t sh_scan[kWalkSmallBlock / kWave + 1];
  const int nc = *parts.d_n_comp;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const int q = parts.comp_size[c];
    if (q > kWalkSmallCap) continue;  // k_asm_walk's
    const int st = parts.comp_start[c];
    WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_roff, s_es, s_eo, s_ep};
    walk_component<kWalkSmallBlock, kWalkSmallCap, true>(c, q, st, w, g, parts, local.perm,
                                                         local.loc_row_ptr, local.loc_col,
                                                         local.loc_eid, out, s, nullptr, sh_scan);
  }
}

// skip_to: components of at most this many reads are k_asm_walk_small's (0:
// every component is this kernel's).  Components of up to kAsmWalkCap reads
// are walked in LDS, larger ones in global scratch: LDS arrays for 512 reads
// let four workgroups share a compute unit (two with arrays for 1024), and
// a component's walk is mostly latency, so more of them at once pays.
constexpr int kAsmWalkCap = 512;
static_assert(kAsmWalkCap % kWalkBlock == 0, "whole members per thread");
__global__ __launch_bounds__(kWalkBlock) void k_asm_walk(cg_graph g, cg_parts parts, cg_local local,
                                                         cg_contigs out, Scratch s,
                                                         int32_t *gbuf, int32_t skip_to) {
  __shared__ int32_t s_nb[2 * kAsmWalkCap], s_eid[2 * kAsmWalkCap], s_nxt[2 * kAsmWalkCap],
      s_dist[2 * kAsmWalkCap], s_endv[2 * kAsmWalkCap], s_vid[kAsmWalkCap];
  __shared__ uint32_t s_rlen[kAsmWalkCap], s_eo[2 * kAsmWalkCap], s_ep[2 * kAsmWalkCap];
  __shared__ uint64_t s_roff[kAsmWalkCap];
  __shared__ uint8_t s_es[2 * kAsmWalkCap];
  __shared__ uint32_t sh_scan[kWalkBlock / kWave + 1];
  const int nc = *parts.d_n_comp;
  const int n = g.n;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const int q = parts.comp_size[c];
    if (q <= skip_to) continue;  // k_asm_walk_small's
    const int st = parts.comp_start[c];
    if (q <= kAsmWalkCap) {
      WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv, s_vid, s_rlen, s_roff, s_es, s_eo, s_ep};
      walk_component<kWalkBlock, kAsmWalkCap, true>(c, q, st, w, g, parts, local.perm, local.loc_row_ptr, local.loc_col,
                           local.loc_eid, out, s, nullptr, sh_scan);
    } else {
      // per-component slices of global scratch: the blocks of different
      // components are disjoint, so slices never overlap
      WalkArrays w{gbuf + 2 * (int64_t)st, gbuf + 2 * (int64_t)n + 2 * (int64_t)st,
                   gbuf + 4 * (int64_t)n + 4 * (int64_t)st,
                   gbuf + 8 * (int64_t)n + 4 * (int64_t)st,
                   gbuf + 12 * (int64_t)n + 4 * (int64_t)st};
      walk_component<kWalkBlock, kWalkCap, false>(c, q, st, w, g, parts, local.perm, local.loc_row_ptr, local.loc_col,
                            local.loc_eid, out, s, nullptr, sh_scan);
    }
  }
}

// contig word offsets: one workgroup, scan of ceil(len/16) in record order
constexpr int kOffRun = 8;  // contigs per thread k_asm_offsets holds in registers
__global__ __launch_bounds__(kScanBlock) void k_asm_offsets(const int32_t *__restrict__ d_n_comp,
                                                            const uint64_t *__restrict__ len,
                                                            uint64_t *__restrict__ base_off,
                                                            uint64_t cap_words,
                                                            uint64_t *__restrict__ d_total_words,
                                                            Fixed *fx) {
  __shared__ unsigned long long sh[kScanBlock / kWave + 1];
  const int nc = *d_n_comp;
  unsigned long long carry = 0;
  if (nc <= kOffRun * kScanBlock) {
    // thread t takes contigs t*E .. t*E + E-1: their lengths loaded at once,
    // one block scan of the thread sums (a loop over blocks of contigs
    // waited for a load and a scan per block)
    const int E = (nc + kScanBlock - 1) / kScanBlock;
    const int k0 = (int)threadIdx.x * E;
    unsigned long long w[kOffRun], x = 0;
#pragma unroll
    for (int r = 0; r < kOffRun; ++r) {
      w[r] = r < E && k0 + r < nc ? (len[k0 + r] + 15) / 16 : 0;
      x += w[r];
    }
    unsigned long long ex = block_excl_scan<unsigned long long, kScanBlock>(x, sh, &carry);
#pragma unroll
    for (int r = 0; r < kOffRun; ++r) {
      if (r < E && k0 + r < nc) base_off[k0 + r] = 16 * ex;
      ex += w[r];
    }
  } else {
    for (int base = 0; base < nc; base += kScanBlock) {
      const int k = base + threadIdx.x;
      const unsigned long long wds = k < nc ? (len[k] + 15) / 16 : 0;
      unsigned long long tot;
      const unsigned long long ex = block_excl_scan<unsigned long long, kScanBlock>(wds, sh, &tot);
      if (k < nc) base_off[k] = 16 * (carry + ex);
      carry += tot;
    }
  }
  if (threadIdx.x == 0) {
    *d_total_words = carry;
    if (carry > cap_words) atomicOr(&fx->status, CG_STATUS_BASES_OVERFLOW);
  }
}

constexpr int kCopyBlock = 256;
constexpr int kCopyWavesPerCU = 16;  // resident copy waves per compute unit (4 per SIMD)
constexpr int kCopyRounds = 4;       // copy chunks per resident wave slot
constexpr int kCopyMinPieces = 2;    // pieces per copy chunk at least

__global__ __launch_bounds__(kCopyBlock) void k_asm_copy(const uint32_t *__restrict__ seq,
                                                         uint64_t seq_words,
                                                         const int32_t *__restrict__ bin_vptr,
                                                         int32_t P,
                                                         const uint64_t *__restrict__ piece_off,
                                                         const uint32_t *__restrict__ piece_len,
                                                         const uint64_t *__restrict__ piece_src,
                                                         const int32_t *__restrict__ lay_contig,
                                                         const uint64_t *__restrict__ clen,
                                                         const uint64_t *__restrict__ cbase,
                                                         const uint64_t *__restrict__ d_total_words,
                                                         uint64_t cap_words,
                                                         uint32_t *__restrict__ bases,
                                                         int32_t chunk_target) {
  if (*d_total_words > cap_words) return;
  const int32_t n_e = bin_vptr[P];
  const PieceArrays A = piece_arrays(lay_contig, piece_off, piece_len, piece_src, clen, cbase);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
  const int32_t gw = blockIdx.x * (blockDim.x / kWave) + wave;
  const int32_t nwv = gridDim.x * (blockDim.x / kWave);
  // pieces per chunk: about chunk_target chunks (a few per wave slot of the
  // device, so the slots drain evenly while each chunk's setup, a chain of
  // dependent descriptor loads, is paid for enough pieces), at least
  // kCopyMinPieces, at most one piece per lane
  int32_t C = (n_e + chunk_target - 1) / chunk_target;
  C = C < kCopyMinPieces ? kCopyMinPieces : (C > kWave ? kWave : C);
  const int32_t n_chunks = (n_e + C - 1) / C;
  for (int32_t ch = gw; ch < n_chunks; ch += nwv) {
    const int32_t c0 = ch * C;
    const int cnt = n_e - c0 < C ? n_e - c0 : C;
    copy_chunk(seq, seq_words, bases, A, c0, cnt, n_e, lane_id());
  }
}

int launch_assemble(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const cg_parts &parts,
                    const cg_local &local, int32_t P, const cg_contigs &out, hipStream_t st) {
  const PhaseRange range("cg: LocalAssembly");
  const int32_t n = g.n;
  if (n == 0) {
    CG_LAUNCH(ctx, k_asm_offsets, dim3(1), dim3(kScanBlock), st, parts.d_n_comp, out.len,
                       out.base_off, out.cap_words, out.d_total_words, ctx->fixed);
    return hip_check(hipGetLastError(), "k_asm");
  }
  const int wgrid = n < 4096 ? n : 4096;
  // A large graph has thousands of components, most of them small: those of
  // at most kWalkSmallCap reads go one wave each to a pass of their own with
  // small LDS arrays (many per CU).  On a smaller graph the second launch
  // costs more than it saves (on 125,000 reads: 26 us against 17).
  const bool split = n >= kWalkSplitReads;
  if (split)
    CG_LAUNCH(ctx, k_asm_walk_small, dim3(n < 8192 ? n : 8192), dim3(kWalkSmallBlock), st, g,
              parts, local, out, s);
  CG_LAUNCH(ctx, k_asm_walk, dim3(wgrid), dim3(kWalkBlock), st, g, parts, local, out, s,
                     s.walk, split ? kWalkSmallCap : 0);
  CG_LAUNCH(ctx, k_asm_offsets, dim3(1), dim3(kScanBlock), st, parts.d_n_comp, out.len,
                     out.base_off, out.cap_words, out.d_total_words, ctx->fixed);
  // about eight pieces per wave, so a small graph still spreads over the chip
  const int cgrid = (n + 31) / 32 < 8192 ? (n + 31) / 32 : 8192;
  // chunks: kCopyRounds per resident wave slot (kCopyWavesPerCU per compute
  // unit at the copy's register use), and never fewer than the grid's waves
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess ||
      cus < 1)
    cus = 1;
  const int64_t tgt = (int64_t)kCopyRounds * kCopyWavesPerCU * cus;
  const int64_t gw = (int64_t)cgrid * (kCopyBlock / kWave);
  const int32_t chunk_target = (int32_t)(tgt > gw ? gw : tgt);
  CG_LAUNCH(ctx, k_asm_copy, dim3(cgrid), dim3(kCopyBlock), st, g.seq, g.seq_words,
                     local.bin_vptr, P, s.piece_off, s.piece_len, s.piece_src, s.lay_contig,
                     out.len, out.base_off, out.d_total_words, out.cap_words, out.bases,
                     chunk_target);
  return hip_check(hipGetLastError(), "k_asm");
}

}  // namespace cg
