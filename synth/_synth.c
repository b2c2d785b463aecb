/*
 * Bulk read extraction for the synthetic workload generator.
 *
 * Input synthesis only: this file simulates sequencing (copying a read's
 * interval out of a genome, on the forward or the reverse strand) and writes
 * the reads in the 2-bit packed store layout the path consumes (16 bases per
 * 32-bit word, base i of a word at bits 2*i, A=0 C=1 G=2 T=3, each read at a
 * 16-base-aligned offset).  It computes nothing the contig-generation method
 * computes and is shared, as an input source only, by the oracle tests and
 * the GPU path.
 */
#include <stdint.h>
#include <string.h>

/* Fill `out` (zeroed by the caller, `out_words` long) with n reads.
 * Read r covers genome[start[r], start[r] + len[r]); when rc[r] is set the
 * stored read is the other strand of that interval (last genome base first,
 * each base complemented).  Read r's first base lands at base offset off[r]
 * (a multiple of 16) of the store.  Reads are independent, so the loop is
 * split across threads when OpenMP is enabled. */
void synth_extract_reads(const uint8_t *genome, int64_t n, const int64_t *start,
                         const int64_t *len, const uint8_t *rc, const int64_t *off,
                         uint32_t *out, int64_t out_words)
{
    (void)out_words;
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t r = 0; r < n; ++r) {
        const uint8_t *g = genome + start[r];
        const int64_t L = len[r];
        uint32_t *w = out + (off[r] >> 4);
        int64_t i = 0;
        while (i < L) {
            uint32_t word = 0;
            int64_t k = L - i < 16 ? L - i : 16;
            if (!rc[r]) {
                for (int64_t j = 0; j < k; ++j)
                    word |= (uint32_t)(g[i + j] & 3u) << (2 * j);
            } else {
                for (int64_t j = 0; j < k; ++j)
                    word |= (uint32_t)(3u - (g[L - 1 - (i + j)] & 3u)) << (2 * j);
            }
            w[i >> 4] = word;
            i += k;
        }
    }
}
