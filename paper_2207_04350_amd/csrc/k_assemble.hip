// LocalAssembly (Section 4.4).  A contig is the concatenation
//   l_r[alpha:pre(e0)] + l_c1[post(e0):pre(e1)] + ... + l_r'[post(e_{q-2}):beta]
// over the chain r, c1, ..., r' of a component: every read but the last
// contributes the part of its walking orientation that precedes its overlap
// with the next read (len - ovl bases), the last read all its bases.
//
//  k_asm_walk     one workgroup per component: start read, walk order by
//                 pointer jumping over the chain's arcs (Wyllie list
//                 ranking), orientation from the strand bits, piece lengths
//                 and offsets, layout and contig record
//  k_asm_offsets  contig base offsets (16-base aligned) in (bin, label) order
//  k_asm_copy     one workgroup per piece: every output word is written by
//                 the piece holding its first base, 2-bit funnel shifts for
//                 unaligned starts, reverse + complement in registers
#include "cg_internal.h"

namespace cg {

constexpr int kWalkBlock = 256;
constexpr int kWalkCap = 1024;               // reads per component handled in LDS
constexpr int kRaysPerThread = 2 * kWalkCap / kWalkBlock;

struct WalkArrays {
  int32_t *nb;     // [2q] local neighbour of slot k of read i (-1: none / cut)
  int32_t *eid;    // [2q] entry index in S of that slot
  int32_t *nxt;    // [2q] ray successor
  int32_t *dist;   // [2q] ray length
  int32_t *endv;   // [2q] ray end
};

template <bool kLds>
__device__ __forceinline__ void walk_component(
    int c, int q, int st, WalkArrays w, const cg_graph &g, const cg_parts &parts,
    const int32_t *__restrict__ perm, const int32_t *__restrict__ loc_row_ptr,
    const int32_t *__restrict__ loc_col, const int32_t *__restrict__ loc_eid,
    const cg_contigs &out, const Scratch &s, int32_t *sh_small, uint32_t *sh_scan) {
  const int tid = threadIdx.x;
  __shared__ int s_start, s_cyc, s_sej;
  __shared__ uint64_t s_carry;
  if (tid == 0) {
    s_start = 0x7FFFFFFF;
    s_cyc = 0;
    s_sej = 0;
    s_carry = 0;
  }
  // 1. local rows of the component's block
  for (int i = tid; i < q; i += kWalkBlock) {
    const int a = loc_row_ptr[st + i], b = loc_row_ptr[st + i + 1];
    const int deg = b - a;
    w.nb[2 * i] = deg >= 1 ? loc_col[a] - st : -1;
    w.nb[2 * i + 1] = deg >= 2 ? loc_col[a + 1] - st : -1;
    w.eid[2 * i] = deg >= 1 ? loc_eid[a] : -1;
    w.eid[2 * i + 1] = deg >= 2 ? loc_eid[a + 1] : -1;
  }
  __syncthreads();
  // 2. start: the first read of local degree 1 (the smaller-id root, since
  // the block is in id order); a cycle starts at its first read and loses
  // the edge to the larger-numbered neighbour of it
  for (int i = tid; i < q; i += kWalkBlock)
    if ((w.nb[2 * i] >= 0) != (w.nb[2 * i + 1] >= 0)) atomicMin(&s_start, i);
  __syncthreads();
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
  __syncthreads();
  const int s0 = s_start;
  // 3. rays (i, k): leave read i through slot k.  A ray jumps along the
  // chain; after ceil(log2 q) doublings it knows the chain end it reaches and
  // how many steps away that end is.
  for (int r = tid; r < 2 * q; r += kWalkBlock) {
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
  __syncthreads();
  for (int span = 1; span < q; span <<= 1) {
    if (kLds) {
      int rn[kRaysPerThread], rd[kRaysPerThread], re[kRaysPerThread];
#pragma unroll
      for (int u = 0; u < kRaysPerThread; ++u) {
        const int r = tid + u * kWalkBlock;
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
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kRaysPerThread; ++u) {
        const int r = tid + u * kWalkBlock;
        if (rn[u] != -2) {
          w.nxt[r] = rn[u];
          w.dist[r] = rd[u];
          w.endv[r] = re[u];
        }
      }
      __syncthreads();
    } else {
      // large component (global arrays): ray r's successor x is only
      // rewritten by its own owner, so read all then write all in two passes
      // with the new values parked in the endv/dist of the high half
      for (int r = tid; r < 2 * q; r += kWalkBlock) {
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
      __syncthreads();
      for (int r = tid; r < 2 * q; r += kWalkBlock) {
        const int x = w.nxt[2 * q + r];
        if (x != -2) {
          w.nxt[r] = x;
          w.dist[r] = w.dist[2 * q + r];
          w.endv[r] = w.endv[2 * q + r];
        }
      }
      __syncthreads();
    }
  }
  // 4. rank, predecessor, successor, orientation and piece of every read
  int32_t *R_vid = out.layout_vid + st;
  uint8_t *R_rev = out.layout_rev + st;
  uint32_t *R_len = s.piece_len + st;
  const int rank_c = parts.comp_rank[c];
  for (int i = tid; i < q; i += kWalkBlock) {
    int rank = 0, pred = -1, succ = -1, succ_e = -1;
    if (i == s0) {
      if (w.nb[2 * i] >= 0) { succ = w.nb[2 * i]; succ_e = w.eid[2 * i]; }
      else if (w.nb[2 * i + 1] >= 0) { succ = w.nb[2 * i + 1]; succ_e = w.eid[2 * i + 1]; }
    } else {
      for (int k = 0; k < 2; ++k) {
        if (w.nb[2 * i + k] >= 0 && w.endv[2 * i + k] == s0) {
          rank = w.dist[2 * i + k];
          pred = w.nb[2 * i + k];
          const int o = 1 - k;
          if (w.nb[2 * i + o] >= 0) { succ = w.nb[2 * i + o]; succ_e = w.eid[2 * i + o]; }
        }
      }
    }
    const int32_t v = perm[st + i];
    int orient;
    if (i == s0) {
      orient = succ_e >= 0 ? (g.strand[succ_e] & 1) : 0;
    } else if (pred >= 0) {
      // the entry pred -> i, read in pred's row
      const int pe = w.nb[2 * pred] == i ? w.eid[2 * pred] : w.eid[2 * pred + 1];
      orient = (g.strand[pe] >> 1) & 1;
    } else {
      orient = 0;  // unreachable for a chain: every read but the start has a predecessor
    }
    uint32_t plen = g.read_len[v];
    if (succ_e >= 0) {
      plen -= g.ovl[succ_e];
      if ((int)(g.strand[succ_e] & 1) != orient) s_sej = 1;
    }
    R_vid[rank] = v;
    R_rev[rank] = (uint8_t)orient;
    R_len[rank] = plen;
    s.lay_contig[st + rank] = rank_c;
    (void)succ;
  }
  __syncthreads();
  // 5. piece offsets in walk order
  for (int base = 0; base < q; base += kWalkBlock) {
    const int i = base + tid;
    const uint32_t x = i < q ? R_len[i] : 0u;
    uint32_t tot;
    const uint32_t ex = block_excl_scan<uint32_t, kWalkBlock>(x, sh_scan, &tot);
    if (i < q) s.piece_off[st + i] = s_carry + ex;
    __syncthreads();
    if (tid == 0) s_carry += tot;
    __syncthreads();
  }
  if (tid == 0) {
    out.label[rank_c] = parts.comp_label[c];
    out.bin[rank_c] = parts.comp_bin[c];
    out.start[rank_c] = perm[st + s0];
    out.n_reads[rank_c] = q;
    out.len[rank_c] = s_carry;
    out.cflags[rank_c] = (q == 1 ? CG_CONTIG_SINGLE : 0u) | (s_cyc ? CG_CONTIG_CIRCULAR : 0u) |
                         (s_sej ? CG_CONTIG_SAME_END_JOIN : 0u);
    out.layout_off[rank_c] = st;
  }
  (void)sh_small;
  __syncthreads();
}

__global__ __launch_bounds__(kWalkBlock) void k_asm_walk(cg_graph g, cg_parts parts, cg_local local,
                                                         cg_contigs out, Scratch s,
                                                         int32_t *gbuf) {
  __shared__ int32_t s_nb[2 * kWalkCap], s_eid[2 * kWalkCap], s_nxt[2 * kWalkCap],
      s_dist[2 * kWalkCap], s_endv[2 * kWalkCap];
  __shared__ uint32_t sh_scan[kWalkBlock / kWave + 1];
  const int nc = *parts.d_n_comp;
  const int n = g.n;
  for (int c = blockIdx.x; c < nc; c += gridDim.x) {
    const int q = parts.comp_size[c];
    const int st = parts.comp_start[c];
    if (q <= kWalkCap) {
      WalkArrays w{s_nb, s_eid, s_nxt, s_dist, s_endv};
      walk_component<true>(c, q, st, w, g, parts, local.perm, local.loc_row_ptr, local.loc_col,
                           local.loc_eid, out, s, nullptr, sh_scan);
    } else {
      // per-component slices of global scratch: the blocks of different
      // components are disjoint, so slices never overlap
      WalkArrays w{gbuf + 2 * (int64_t)st, gbuf + 2 * (int64_t)n + 2 * (int64_t)st,
                   gbuf + 4 * (int64_t)n + 4 * (int64_t)st,
                   gbuf + 8 * (int64_t)n + 4 * (int64_t)st,
                   gbuf + 12 * (int64_t)n + 4 * (int64_t)st};
      walk_component<false>(c, q, st, w, g, parts, local.perm, local.loc_row_ptr, local.loc_col,
                            local.loc_eid, out, s, nullptr, sh_scan);
    }
  }
}

// contig word offsets: one workgroup, scan of ceil(len/16) in record order
__global__ __launch_bounds__(kScanBlock) void k_asm_offsets(const int32_t *__restrict__ d_n_comp,
                                                            const uint64_t *__restrict__ len,
                                                            uint64_t *__restrict__ base_off,
                                                            uint64_t cap_words,
                                                            uint64_t *__restrict__ d_total_words,
                                                            Fixed *fx) {
  __shared__ unsigned long long sh[kScanBlock / kWave + 1];
  const int nc = *d_n_comp;
  unsigned long long carry = 0;
  for (int base = 0; base < nc; base += kScanBlock) {
    const int k = base + threadIdx.x;
    const unsigned long long wds = k < nc ? (len[k] + 15) / 16 : 0;
    unsigned long long tot;
    const unsigned long long ex = block_excl_scan<unsigned long long, kScanBlock>(wds, sh, &tot);
    if (k < nc) base_off[k] = 16 * (carry + ex);
    carry += tot;
  }
  if (threadIdx.x == 0) {
    *d_total_words = carry;
    if (carry > cap_words) atomicOr(&fx->status, CG_STATUS_BASES_OVERFLOW);
  }
}

// k bases (1..16) starting at base index b of the store, LSB first; words
// past the end of the store read as zero
__device__ __forceinline__ uint32_t fetch_bases(const uint32_t *__restrict__ seq, uint64_t nwords,
                                                uint64_t b, int k) {
  const uint64_t wi = b >> 4;
  const int sh = (int)(b & 15) * 2;
  uint64_t x = wi < nwords ? seq[wi] : 0u;
  if (sh + 2 * k > 32 && wi + 1 < nwords) x |= (uint64_t)seq[wi + 1] << 32;
  x >>= sh;
  return k == 16 ? (uint32_t)x : (uint32_t)x & ((1u << (2 * k)) - 1u);
}

// reverse the order of the k low 2-bit fields and complement them
__device__ __forceinline__ uint32_t revcomp_fields(uint32_t x, int k) {
  uint32_t y = __builtin_bitreverse32(x);
  y = ((y >> 1) & 0x55555555u) | ((y & 0x55555555u) << 1);
  y >>= 32 - 2 * k;
  return y ^ (k == 16 ? 0xFFFFFFFFu : ((1u << (2 * k)) - 1u));
}

constexpr int kCopyBlock = 256;

__global__ __launch_bounds__(kCopyBlock) void k_asm_copy(const uint32_t *__restrict__ seq,
                                                         uint64_t seq_words,
                                                         const uint32_t *__restrict__ read_len,
                                                         const uint64_t *__restrict__ read_off,
                                                         const int32_t *__restrict__ bin_vptr,
                                                         int32_t P,
                                                         const int32_t *__restrict__ layout_vid,
                                                         const uint8_t *__restrict__ layout_rev,
                                                         const uint64_t *__restrict__ piece_off,
                                                         const uint32_t *__restrict__ piece_len,
                                                         const int32_t *__restrict__ lay_contig,
                                                         const uint64_t *__restrict__ clen,
                                                         const uint64_t *__restrict__ cbase,
                                                         const uint64_t *__restrict__ d_total_words,
                                                         uint64_t cap_words,
                                                         uint32_t *__restrict__ bases) {
  if (*d_total_words > cap_words) return;
  const int32_t n_e = bin_vptr[P];
  for (int32_t p = blockIdx.x; p < n_e; p += gridDim.x) {
    const int32_t k = lay_contig[p];
    const uint64_t L = clen[k];
    const uint64_t cb = cbase[k] >> 4;
    const uint64_t poff = piece_off[p];
    const uint32_t plen = piece_len[p];
    const uint64_t j0 = (poff + 15) >> 4, j1 = (poff + plen + 15) >> 4;
    for (uint64_t j = j0 + threadIdx.x; j < j1; j += kCopyBlock) {
      uint64_t pos = j << 4;
      int32_t pp = p;
      uint64_t o_off = poff;
      uint32_t o_len = plen;
      int32_t v = layout_vid[pp];
      int rev = layout_rev[pp];
      uint32_t out = 0;
      int filled = 0;
      while (filled < 16 && pos < L) {
        while (pos >= o_off + o_len && pp + 1 < n_e) {  // continue into the next piece
          o_off += o_len;
          ++pp;
          o_len = piece_len[pp];
          v = layout_vid[pp];
          rev = layout_rev[pp];
        }
        const uint64_t t = pos - o_off;
        const uint64_t avail = o_off + o_len > pos ? o_off + o_len - pos : 0;
        int kk = 16 - filled;
        if (avail < (uint64_t)kk) kk = (int)avail;
        if (kk <= 0) break;  // only on inconsistent pieces
        uint32_t x;
        if (!rev) {
          x = fetch_bases(seq, seq_words, read_off[v] + t, kk);
        } else {
          const uint64_t Lr = read_len[v];
          x = revcomp_fields(fetch_bases(seq, seq_words, read_off[v] + Lr - t - kk, kk), kk);
        }
        out |= x << (2 * filled);
        filled += kk;
        pos += kk;
      }
      bases[cb + j] = out;
    }
  }
}

int launch_assemble(cg_ctx *ctx, const cg_graph &g, const Scratch &s, const cg_parts &parts,
                    const cg_local &local, int32_t P, const cg_contigs &out, hipStream_t st) {
  const int32_t n = g.n;
  if (n == 0) {
    CG_LAUNCH(ctx, k_asm_offsets, dim3(1), dim3(kScanBlock), st, parts.d_n_comp, out.len,
                       out.base_off, out.cap_words, out.d_total_words, ctx->fixed);
    return hip_check(hipGetLastError(), "k_asm");
  }
  const int wgrid = n < 4096 ? n : 4096;
  CG_LAUNCH(ctx, k_asm_walk, dim3(wgrid), dim3(kWalkBlock), st, g, parts, local, out, s,
                     s.walk);
  CG_LAUNCH(ctx, k_asm_offsets, dim3(1), dim3(kScanBlock), st, parts.d_n_comp, out.len,
                     out.base_off, out.cap_words, out.d_total_words, ctx->fixed);
  const int cgrid = n < 8192 ? n : 8192;
  CG_LAUNCH(ctx, k_asm_copy, dim3(cgrid), dim3(kCopyBlock), st, g.seq, g.seq_words,
                     g.read_len,
                     g.read_off, local.bin_vptr, P, out.layout_vid, out.layout_rev, s.piece_off,
                     s.piece_len, s.lay_contig, out.len, out.base_off, out.d_total_words,
                     out.cap_words, out.bases);
  return hip_check(hipGetLastError(), "k_asm");
}

}  // namespace cg
