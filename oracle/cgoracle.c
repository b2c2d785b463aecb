/*
 * CPU oracle for the contig-generation path.  TEST INFRASTRUCTURE ONLY: see
 * cgoracle.h.  Plain single-threaded C99; each function follows one step of
 * the paper's Algorithm 2 in the paper's order, without blocking, fusion or
 * reordering, so that it can be checked against the text by eye.
 *
 * Readings of passages the paper leaves open are marked "reading:".
 */
#include "cgoracle.h"

#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* O-0  Input checks                                                         */
/* ------------------------------------------------------------------------ */

static int64_t find_entry(const int32_t *row_ptr, const int32_t *col, int32_t u, int32_t v)
{
    for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
        if (col[j] == v) return j;
    return -1;
}

int64_t cgo_validate(int32_t n, int32_t m, const int32_t *row_ptr, const int32_t *col,
                     const uint32_t *ovl, const uint8_t *strand, const uint32_t *read_len,
                     const uint64_t *read_off, uint64_t seq_words, const uint32_t *pre,
                     const uint32_t *post, int32_t *why)
{
    *why = 0;
    if (n < 0 || m < 0 || row_ptr[0] != 0 || row_ptr[n] != m) { *why = 1; return -2; }
    for (int32_t v = 0; v < n; ++v)
        if (row_ptr[v + 1] < row_ptr[v]) { *why = 1; return v; }
    for (int32_t v = 0; v < n; ++v) {
        if (read_len[v] < 1) { *why = 9; return v; }
        if (read_off[v] % 16 != 0) { *why = 10; return v; }
        if (read_off[v] + read_len[v] > seq_words * 16) { *why = 11; return v; }
    }
    for (int32_t u = 0; u < n; ++u) {
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            int32_t v = col[j];
            if (v < 0 || v >= n) { *why = 2; return j; }
            if (v == u) { *why = 3; return j; }
            if (j > row_ptr[u] && col[j - 1] >= v) { *why = 4; return j; }
            int64_t t = find_entry(row_ptr, col, v, u);
            if (t < 0) { *why = 5; return j; }
            if (ovl[t] != ovl[j]) { *why = 6; return j; }
            /* twin of (s, d) is (not d, not s): S is symmetric as a bidirected graph */
            uint8_t s = strand[j] & 1, d = (strand[j] >> 1) & 1;
            uint8_t want = (uint8_t)((1 - d) | ((1 - s) << 1));
            if ((strand[t] & 3) != want || (strand[j] & ~3u)) { *why = 7; return j; }
            uint32_t lmin = read_len[u] < read_len[v] ? read_len[u] : read_len[v];
            if (ovl[j] < 1 || ovl[j] >= lmin) { *why = 8; return j; }
            /* Section 4.4: pre indexes read u, post indexes read v */
            if (pre && pre[j] >= read_len[u]) { *why = 12; return j; }
            if (post && post[j] >= read_len[v]) { *why = 13; return j; }
        }
    }
    return -1;
}

/* ------------------------------------------------------------------------ */
/* O-1  BranchRemoval(S) -> L                                                 */
/* ------------------------------------------------------------------------ */

void cgo_mask(int32_t n, const int32_t *row_ptr, const int32_t *col, uint8_t *flags,
              int32_t *counts)
{
    /* d = row sums of the pattern of S (reading: count of nonzeros, not the
     * weights); b = {v : d[v] >= 3}.  One pass on S's degrees: neighbours of
     * a branch vertex merely lose that edge. */
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) d[v] = row_ptr[v + 1] - row_ptr[v];
    counts[0] = 0;
    counts[1] = 0;
    for (int32_t v = 0; v < n; ++v) {
        uint8_t f = 0;
        if (d[v] >= 3) {
            f = 1;
            counts[0]++;
        } else {
            for (int32_t j = 0; j < d[v]; ++j) {
                int32_t u = col[row_ptr[v] + j];
                if (d[u] < 3) {
                    f |= (uint8_t)(2 << j);
                    counts[1]++;
                }
            }
        }
        flags[v] = f;
    }
    free(d);
}

/* ------------------------------------------------------------------------ */
/* O-2  ConnectedComponent(L) -> v                                            */
/* ------------------------------------------------------------------------ */

static int32_t uf_find(int32_t *parent, int32_t x)
{
    int32_t r = x;
    while (parent[r] != r) r = parent[r];
    while (parent[x] != r) {
        int32_t nx = parent[x];
        parent[x] = r;
        x = nx;
    }
    return r;
}

void cgo_components(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint8_t *flags,
                    int32_t *label)
{
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) parent[v] = v;
    for (int32_t v = 0; v < n; ++v) {
        for (int32_t j = 0; j < 2; ++j) {
            if (!(flags[v] & (2 << j))) continue;
            int32_t u = col[row_ptr[v] + j];
            int32_t a = uf_find(parent, v), b = uf_find(parent, u);
            if (a != b) parent[a] = b;
        }
    }
    /* canonical component id: the smallest vertex id in the component */
    int32_t *minid = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t v = 0; v < n; ++v) minid[v] = n;
    for (int32_t v = 0; v < n; ++v) {
        int32_t r = uf_find(parent, v);
        if (v < minid[r]) minid[r] = v;
    }
    for (int32_t v = 0; v < n; ++v) label[v] = minid[uf_find(parent, v)];
    free(minid);
    free(parent);
}

/* ------------------------------------------------------------------------ */
/* O-3  Component sizes and kinds                                             */
/* ------------------------------------------------------------------------ */

static int popcount2(uint8_t f) { return ((f >> 1) & 1) + ((f >> 2) & 1); }

int32_t cgo_table(int32_t n, const int32_t *row_ptr, const uint8_t *flags, const int32_t *label,
                  int32_t min_reads, int32_t *comp_label, int32_t *comp_size, uint8_t *comp_kind,
                  int32_t *label_comp)
{
    (void)row_ptr;
    int64_t *q = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    int64_t *e2 = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    for (int32_t v = 0; v < n; ++v) {
        q[label[v]] += 1;
        e2[label[v]] += popcount2(flags[v]);   /* each undirected edge counted twice */
    }
    if (min_reads < 1) min_reads = 1;
    int32_t k = 0;
    for (int32_t r = 0; r < n; ++r) {
        label_comp[r] = -1;
        if (q[r] == 0) continue;                /* r is not a component label */
        int64_t e = e2[r] / 2;
        uint8_t kind;
        if (q[r] == 1) kind = CGO_SINGLE;
        else if (e == q[r] - 1) kind = CGO_PATH;
        else if (e == q[r]) kind = CGO_CYCLE;
        else { free(q); free(e2); return -1; }
        int branch = flags[r] & 1;
        if (branch || q[r] < min_reads) continue;
        comp_label[k] = r;
        comp_size[k] = (int32_t)q[r];
        comp_kind[k] = kind;
        label_comp[r] = k;
        ++k;
    }
    free(q);
    free(e2);
    return k;
}

/* ------------------------------------------------------------------------ */
/* O-4  GreedyPartitioning(v, P) -> p   (LPT)                                 */
/* ------------------------------------------------------------------------ */

static const uint64_t *g_sort_weight;
static const int32_t *g_sort_label;

static int cmp_size_desc(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_sort_weight[x] != g_sort_weight[y]) return g_sort_weight[x] > g_sort_weight[y] ? -1 : 1;
    if (g_sort_label[x] != g_sort_label[y]) return g_sort_label[x] < g_sort_label[y] ? -1 : 1;
    return 0;
}

void cgo_lpt(int32_t n_comp, const uint64_t *weight, const int32_t *comp_label, int32_t P,
             int32_t *comp_bin, uint64_t *bin_load)
{
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_comp > 0 ? n_comp : 1));
    for (int32_t i = 0; i < n_comp; ++i) order[i] = i;
    g_sort_weight = weight;
    g_sort_label = comp_label;
    qsort(order, (size_t)n_comp, sizeof(int32_t), cmp_size_desc);
    for (int32_t j = 0; j < P; ++j) bin_load[j] = 0;
    for (int32_t i = 0; i < n_comp; ++i) {
        int32_t c = order[i];
        int32_t best = 0;                       /* least loaded set, lowest index on ties */
        for (int32_t j = 1; j < P; ++j)
            if (bin_load[j] < bin_load[best]) best = j;
        comp_bin[c] = best;
        bin_load[best] += weight[c];
    }
    free(order);
}

static const int32_t *g_ord_bin, *g_ord_label;

static int cmp_bin_label(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    if (g_ord_bin[x] != g_ord_bin[y]) return g_ord_bin[x] < g_ord_bin[y] ? -1 : 1;
    if (g_ord_label[x] != g_ord_label[y]) return g_ord_label[x] < g_ord_label[y] ? -1 : 1;
    return 0;
}

void cgo_order(int32_t n_comp, const int32_t *comp_label, const int32_t *comp_bin,
               const int32_t *comp_size, int32_t *comp_rank, int32_t *comp_start)
{
    int32_t *order = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_comp > 0 ? n_comp : 1));
    for (int32_t i = 0; i < n_comp; ++i) order[i] = i;
    g_ord_bin = comp_bin;
    g_ord_label = comp_label;
    qsort(order, (size_t)n_comp, sizeof(int32_t), cmp_bin_label);
    int32_t acc = 0;
    for (int32_t r = 0; r < n_comp; ++r) {
        comp_rank[order[r]] = r;
        comp_start[order[r]] = acc;
        acc += comp_size[order[r]];
    }
    free(order);
}

/* ------------------------------------------------------------------------ */
/* O-5  InducedSubgraph(L, p)                                                 */
/* ------------------------------------------------------------------------ */

void cgo_induce(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint8_t *flags,
                const int32_t *label, int32_t n_comp, const int32_t *label_comp,
                const int32_t *comp_bin, const int32_t *comp_start, int32_t P,
                const int32_t *comp_size, int32_t *perm, int32_t *bin_vptr,
                int32_t *loc_row_ptr, int32_t *loc_col, int32_t *loc_eid, int32_t *sizes)
{
    /* V_i = {v : owner(v) = i}; vertices numbered by (bin, label, id): the
     * component blocks come in (bin, label) order (comp_start), and inside a
     * block the vertices keep ascending id order. */
    int32_t *fill = (int32_t *)calloc((size_t)(n_comp > 0 ? n_comp : 1), sizeof(int32_t));
    int32_t *local = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t n_e = 0;
    for (int32_t v = 0; v < n; ++v) {
        local[v] = -1;
        int32_t c = label_comp[label[v]];
        if (c < 0) continue;
        int32_t pos = comp_start[c] + fill[c]++;
        perm[pos] = v;
        local[v] = pos;
        ++n_e;
    }
    /* bin boundaries: the reads of each bin, counted from the components */
    for (int32_t b = 0; b <= P; ++b) bin_vptr[b] = 0;
    for (int32_t c = 0; c < n_comp; ++c) bin_vptr[comp_bin[c] + 1] += comp_size[c];
    for (int32_t b = 0; b < P; ++b) bin_vptr[b + 1] += bin_vptr[b];
    /* E_i = {(u, v) in L : u, v in V_i}: each kept entry of a local vertex, in
     * the row order of S, with its column renumbered and its entry index kept */
    int32_t m_e = 0;
    for (int32_t i = 0; i < n_e; ++i) {
        int32_t v = perm[i];
        loc_row_ptr[i] = m_e;
        for (int32_t j = 0; j < 2; ++j) {
            if (!(flags[v] & (2 << j))) continue;
            int32_t e = row_ptr[v] + j;
            loc_col[m_e] = local[col[e]];
            loc_eid[m_e] = e;
            ++m_e;
        }
    }
    loc_row_ptr[n_e] = m_e;
    sizes[0] = n_e;
    sizes[1] = m_e;
    free(local);
    free(fill);
}

/* ------------------------------------------------------------------------ */
/* O-6 / O-7  LocalAssembly(P, sequences) -> cset                             */
/* ------------------------------------------------------------------------ */

static uint8_t base_at(const uint32_t *seq, uint64_t i)
{
    return (uint8_t)((seq[i / 16] >> (2 * (i % 16))) & 3u);
}

/* l[i:j] of the paper with inclusive ends: forward bases i..j when the read
 * is walked forward, else the reverse complement l[i]^c, l[i-1]^c, ...,
 * l[j]^c.  Reading: the direction comes from the strand bits rather than from
 * comparing i and j, which also settles one-base pieces (i == j). */
static uint64_t emit_piece(const uint32_t *seq, uint64_t off, int64_t i, int64_t j, int rev,
                           uint8_t *out, uint64_t at)
{
    if (!rev) {
        for (int64_t t = i; t <= j; ++t) out[at++] = base_at(seq, off + (uint64_t)t);
    } else {
        for (int64_t t = i; t >= j; --t) out[at++] = (uint8_t)(3u - base_at(seq, off + (uint64_t)t));
    }
    return at;
}

/* The piece of the t-th read v of a walk of q reads, oriented o, as stored
 * indices [from .. to] (increasing for o = 0, decreasing for o = 1; an
 * empty piece when to lies before from).  Section 4.4: the piece runs from
 * post(e_{t-1}), the first base of v inside its overlap with the
 * predecessor, to pre(e_t), the last base of v before its overlap with the
 * successor; alpha / beta (the read's first / last base in walking order)
 * stand in at the walk's ends.  Without explicit values they follow from the
 * overlap length: post = 0 or |l|-1 and pre = |l|-ovl-1 or ovl. */
static void piece_bounds(int32_t t, int32_t q, int o, int32_t v, const int32_t *edge,
                         const uint32_t *ovl, const uint32_t *read_len, const uint32_t *pre,
                         const uint32_t *post, int64_t *from, int64_t *to)
{
    int64_t L = (int64_t)read_len[v];
    if (t == 0) *from = o == 0 ? 0 : L - 1;                    /* alpha */
    else if (post) *from = (int64_t)post[edge[t - 1]];
    else *from = o == 0 ? 0 : L - 1;
    if (t == q - 1) *to = o == 0 ? L - 1 : 0;                  /* beta */
    else if (pre) *to = (int64_t)pre[edge[t]];
    else {
        int64_t ov = (int64_t)ovl[edge[t]];
        *to = o == 0 ? L - ov - 1 : ov;
    }
}

int32_t cgo_assemble(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *ovl,
                     const uint8_t *strand, const uint32_t *read_len, const uint64_t *read_off,
                     const uint32_t *seq, const uint32_t *pre, const uint32_t *post, int32_t n_comp, const int32_t *comp_label,
                     const int32_t *comp_size, const uint8_t *comp_kind, const int32_t *comp_bin,
                     const int32_t *comp_rank, const int32_t *comp_start, const int32_t *perm,
                     const int32_t *loc_row_ptr, const int32_t *loc_col, const int32_t *loc_eid,
                     int32_t *rec_label, int32_t *rec_bin, int32_t *rec_start,
                     int32_t *rec_nreads, uint64_t *rec_len, uint64_t *rec_base_off,
                     uint32_t *rec_flags, int32_t *rec_layout_off, int32_t *layout_vid,
                     uint8_t *layout_rev, uint32_t *bases, uint64_t cap_words,
                     uint64_t *total_words)
{
    (void)n;
    (void)row_ptr;
    (void)col;
    int32_t n_e = 0;
    for (int32_t c = 0; c < n_comp; ++c) n_e += comp_size[c];
    uint8_t *visited = (uint8_t *)calloc((size_t)(n_e > 0 ? n_e : 1), 1);
    int32_t *walk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_e > 0 ? n_e : 1));
    int32_t *edge = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_e > 0 ? n_e : 1));
    int32_t *by_rank = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n_comp > 0 ? n_comp : 1));
    for (int32_t c = 0; c < n_comp; ++c) by_rank[comp_rank[c]] = c;

    /* pass 1: walk every chain (layout, orientation, length); pass 2: bases */
    uint64_t words = 0;
    for (int pass = 0; pass < 2; ++pass) {
        uint64_t woff = 0;
        for (int32_t k = 0; k < n_comp; ++k) {
            int32_t c = by_rank[k];
            int32_t q = comp_size[c];
            int32_t lo = comp_start[c], hi = lo + q;      /* the component's local block */

            /* choose the start: the first root (local degree 1) in local
             * scan order; a cycle has none and starts at its first local
             * vertex (its smallest id), stepping to the smaller-numbered
             * neighbour; a single read starts at itself */
            int32_t s = -1;
            for (int32_t i = lo; i < hi && s < 0; ++i)
                if (loc_row_ptr[i + 1] - loc_row_ptr[i] == 1) s = i;
            int cyclic = 0;
            if (s < 0) {
                s = lo;
                cyclic = q > 1;
            }
            /* DFS on a graph of maximum degree 2: the frontier holds one
             * vertex; at each step take the unvisited neighbour */
            int32_t len_walk = 0;
            int32_t cur = s;
            visited[cur] = (uint8_t)(pass + 1);
            walk[lo + len_walk++] = cur;
            while (1) {
                int32_t nxt = -1, e = -1;
                int32_t a = loc_row_ptr[cur], b = loc_row_ptr[cur + 1];
                if (cyclic && cur == s && b - a == 2) {
                    /* first step of a cycle: toward the smaller local number */
                    int32_t t = loc_col[a] < loc_col[a + 1] ? a : a + 1;
                    nxt = loc_col[t];
                    e = loc_eid[t];
                } else {
                    for (int32_t t = a; t < b; ++t) {
                        if (visited[loc_col[t]] != (uint8_t)(pass + 1)) {
                            nxt = loc_col[t];
                            e = loc_eid[t];
                            break;
                        }
                    }
                }
                if (nxt < 0) break;
                edge[lo + len_walk - 1] = e;        /* e_{k} joins walk[k] -> walk[k+1] */
                visited[nxt] = (uint8_t)(pass + 1);
                walk[lo + len_walk++] = nxt;
                cur = nxt;
            }
            /* a valid induced chain visits every vertex of its component */
            if (len_walk != q) {
                free(visited); free(walk); free(edge); free(by_rank);
                return -1;
            }

            /* orientation: the start takes the s bit of e0, every later read
             * the d bit of the edge it is entered by */
            uint32_t cflags = 0;
            if (q == 1) cflags |= CGO_SINGLE_READ;
            if (cyclic) cflags |= CGO_CIRCULAR;
            uint64_t total = 0;
            for (int32_t t = 0; t < q; ++t) {
                int32_t v = perm[walk[lo + t]];
                int o;
                if (t == 0) o = q > 1 ? (strand[edge[lo]] & 1) : 0;
                else o = (strand[edge[lo + t - 1]] >> 1) & 1;
                int64_t from, to;
                piece_bounds(t, q, o, v, edge + lo, ovl, read_len, pre, post, &from, &to);
                if (t < q - 1 && (int)(strand[edge[lo + t]] & 1) != o) cflags |= CGO_SAME_END_JOIN;
                if (pass == 1) {
                    layout_vid[lo + t] = v;
                    layout_rev[lo + t] = (uint8_t)o;
                }
                int64_t plen = (o == 0 ? to - from : from - to) + 1;
                total += (uint64_t)(plen > 0 ? plen : 0);
            }
            if (pass == 0) {
                rec_label[k] = comp_label[c];
                rec_bin[k] = comp_bin[c];
                rec_start[k] = perm[s];
                rec_nreads[k] = q;
                rec_len[k] = total;
                rec_base_off[k] = woff * 16;
                rec_flags[k] = cflags;
                rec_layout_off[k] = lo;
                (void)comp_kind;
                woff += (total + 15) / 16;
            } else {
                /* concatenate the pieces into a byte buffer, then pack */
                uint8_t *buf = (uint8_t *)malloc((size_t)(total > 0 ? total : 1));
                uint64_t at = 0;
                for (int32_t t = 0; t < q; ++t) {
                    int32_t v = perm[walk[lo + t]];
                    int o = layout_rev[lo + t];
                    int64_t from, to;
                    piece_bounds(t, q, o, v, edge + lo, ovl, read_len, pre, post, &from, &to);
                    at = emit_piece(seq, read_off[v], from, to, o, buf, at);
                }
                uint64_t base = rec_base_off[k] / 16;
                uint64_t nw = (total + 15) / 16;
                for (uint64_t w = 0; w < nw; ++w) {
                    uint32_t word = 0;
                    for (uint64_t i = 0; i < 16 && w * 16 + i < total; ++i)
                        word |= (uint32_t)buf[w * 16 + i] << (2 * i);
                    bases[base + w] = word;
                }
                free(buf);
            }
        }
        if (pass == 0) {
            words = woff;
            *total_words = words;
            if (words > cap_words) {
                free(visited); free(walk); free(edge); free(by_rank);
                return -4;
            }
        }
    }
    free(visited);
    free(walk);
    free(edge);
    free(by_rank);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Before the path: Prune(IsContainedRead) and TransitiveReduction           */
/* (Algorithm 1; Section 2: redundant vertices and redundant edges)          */
/* ------------------------------------------------------------------------ */

int64_t cgo_reduce(int32_t n, const int32_t *row_ptr, const int32_t *col, const uint32_t *ovl,
                   const uint8_t *strand, const uint32_t *read_len, uint32_t fuzz,
                   uint8_t *contained, uint8_t *kept, int32_t *s_row_ptr, int32_t *s_col,
                   uint32_t *s_ovl, uint8_t *s_strand)
{
    const int64_t m = row_ptr[n];
    /* redundant vertices: a read whose every base lies in an overlap with a
     * longer read (of equal reads, all but the smallest id) */
    for (int32_t v = 0; v < n; ++v) {
        contained[v] = 0;
        for (int64_t j = row_ptr[v]; j < row_ptr[v + 1]; ++j) {
            const int32_t u = col[j];
            if (ovl[j] >= read_len[v] &&
                (read_len[u] > read_len[v] || (read_len[u] == read_len[v] && u < v)))
                contained[v] = 1;
        }
    }
    /* redundant edges: entries with a parallel two-edge walk of the same
     * overhang */
    uint8_t *trans = (uint8_t *)calloc((size_t)(m > 0 ? m : 1), 1);
    for (int32_t u = 0; u < n; ++u) {
        if (contained[u]) continue;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t w = col[e];
            if (contained[w]) continue;
            const int64_t sfx_uw = (int64_t)read_len[w] - ovl[e];
            for (int64_t f = row_ptr[u]; f < row_ptr[u + 1] && !trans[e]; ++f) {
                const int32_t v = col[f];
                if (v == w || contained[v]) continue;
                const int64_t g = find_entry(row_ptr, col, v, w);
                if (g < 0) continue;
                const int s_uv = strand[f] & 1, d_uv = (strand[f] >> 1) & 1;
                const int s_vw = strand[g] & 1, d_vw = (strand[g] >> 1) & 1;
                const int s_uw = strand[e] & 1, d_uw = (strand[e] >> 1) & 1;
                if (s_uv != s_uw || d_uv != s_vw || d_vw != d_uw) continue;
                const int64_t sum = ((int64_t)read_len[v] - ovl[f]) + ((int64_t)read_len[w] - ovl[g]);
                const int64_t diff = sum > sfx_uw ? sum - sfx_uw : sfx_uw - sum;
                if (diff <= (int64_t)fuzz) trans[e] = 1;
            }
        }
    }
    /* S: the pairs with neither entry transitive and no contained read */
    int64_t at = 0;
    for (int32_t u = 0; u < n; ++u) {
        s_row_ptr[u] = (int32_t)at;
        for (int64_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
            const int32_t w = col[e];
            const int64_t twin = find_entry(row_ptr, col, w, u);
            const int keep = !contained[u] && !contained[w] && !trans[e] &&
                             !(twin >= 0 && trans[twin]);
            kept[e] = (uint8_t)keep;
            if (keep) {
                s_col[at] = w;
                s_ovl[at] = ovl[e];
                s_strand[at] = strand[e];
                ++at;
            }
        }
    }
    s_row_ptr[n] = (int32_t)at;
    free(trans);
    return at;
}
