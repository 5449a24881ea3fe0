/*
 * ppc_oracle.h -- CPU oracle for the positional population count.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links
 * or calls this header or its implementation; only the test suite, the smoke
 * check and the CPU-baseline leg of the benchmark do.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * Definition followed (Klarqvist, Mula, Lemire, "Efficient Computation of
 * Positional Population Counts Using SIMD Instructions", Sec. 1 and Sec. 4,
 * Fig. 3): for a stream of n words of k bits, counts[p] is the number of words
 * whose bit p is set, p = 0 .. k-1.  The shift-mask-add reference of Fig. 3 is
 * generalised to k in {8, 16, 32, 64}, to any byte address (a word is the k/8
 * bytes starting at bytes + j*k/8, read little-endian) and to 64-bit counters.
 * Counters are accumulated into (+=), never overwritten (Sec. 4 and Fig. 3
 * start from zeroed counters and only add).
 */
#ifndef PPC_ORACLE_H
#define PPC_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Plain definition, single thread.  bytes: host memory, n*k/8 bytes, any
 * alignment.  counts: host array of k uint64, accumulated into.
 * Returns 0, or -1 if k is not 8, 16, 32 or 64. */
int ppc_oracle_count(const uint8_t* bytes, uint64_t n, int k, uint64_t* counts);

/* Same definition split over `threads` POSIX threads on contiguous word
 * ranges; the partial count vectors are summed.  Exact because the count of a
 * concatenation is the sum of the counts of its parts (every step of Fig. 3
 * only adds).  threads <= 0 means one thread per online CPU.  Returns the
 * number of threads used, or -1 on a bad k. */
int ppc_oracle_count_mt(const uint8_t* bytes, uint64_t n, int k, uint64_t* counts,
                        int threads);

/* Carry-save adder of Sec. 2 (Fig. "csacpp"): three 64-bit words in, the
 * sum bit l = a^b^c and the carry bit h = majority(a,b,c) out, using five
 * logical operations. */
void ppc_oracle_csa(uint64_t a, uint64_t b, uint64_t c, uint64_t* h, uint64_t* l);

/* Model of the Sec. 4.1 algorithm for 16-bit words, in the paper's own terms:
 * 512-bit registers (32 words each), a Harley-Seal circuit over 2^N registers
 * built by the recursion of Sec. 2 (F_{N+1} from two F_N and one CSA), running
 * registers B0..B_{N-1}, the carry register B_N counted per position with a
 * deferred weight 2^N, the final flush of B0..B_{N-1} with weights 1,2,..,
 * 2^{N-1}, and the scalar shift-mask-add routine for the residual words that do
 * not fill a whole 2^N-register block.  N in 1..6 (N = 2, 3, 4 are the 256 B,
 * 512 B and 1 kB circuits).  data: n little-endian uint16 words (any
 * alignment).  counts[16] accumulated into.  *csa_calls (if not NULL) receives
 * the number of CSA evaluations made.  Returns 0 or -1 on a bad N. */
int ppc_oracle_hs16(const uint8_t* data, uint64_t n, int N, uint64_t* counts,
                    uint64_t* csa_calls);

/* Histogram of categorical ids -- the paper's motivating use (Sec. 1, Table 1):
 * category c is bit c of a one-hot word, and the positional population count
 * of the one-hot stream is the frequency histogram.  Computed here directly
 * from the ids: ids are n little-endian unsigned integers of id_bytes (1 or 2)
 * bytes each, at any alignment; counts[c] += number of ids equal to c for
 * c < bins, and counts[bins] += number of ids >= bins (ids with no one-hot code
 * of `bins` bits).  bins in 1..64.  Returns 0 or -1 on bad arguments. */
int ppc_oracle_histogram(const uint8_t* ids, uint64_t n, int id_bytes, int bins,
                         uint64_t* counts);

/* Wider words as several streams of 16-bit words (Sec. 4): a word of k = 16*m
 * bits is held as m planes, plane j holding its 16-bit limb j (word bits 16j ..
 * 16j+15) as n little-endian uint16 words at any alignment.  counts[16j + p] +=
 * number of words whose limb j has bit p set, which is the count of word bit
 * 16j + p.  planes: m host pointers.  m in 1..64.  Returns 0 or -1 on a bad m. */
int ppc_oracle_count_planes(const uint8_t* const* planes, int m, uint64_t n, uint64_t* counts);

#ifdef __cplusplus
}
#endif

#endif /* PPC_ORACLE_H */
