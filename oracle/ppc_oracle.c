/*
 * ppc_oracle.c -- CPU oracle for the positional population count.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
 * benchmark's CPU-baseline leg.  The product library never links it, and it
 * shares no code with the GPU path.  Plain C99 + POSIX threads, built with gcc.
 *
 * Sources in the paper (Klarqvist, Mula, Lemire):
 *   - the problem statement: abstract and Sec. 1 (k sums, one per bit index;
 *     a frequency histogram when the words are one-hot);
 *   - the plain definition: Sec. 4, Fig. 3 (shift, mask, add per bit index);
 *   - the carry-save adder: Sec. 2, Fig. "csacpp", and its truth tables,
 *     Sec. 3, Table 2;
 *   - the Harley-Seal recursion: Sec. 2 (a 2^N-input circuit from two
 *     2^(N-1)-input circuits plus one CSA, 2^N - 1 CSAs in all);
 *   - the counting of the carry register, the deferred weight and the final
 *     flush of the running registers: Sec. 4.1 and Fig. 6;
 *   - the scalar residual: end of Sec. 4.1;
 *   - wider words as several 16-bit streams: Sec. 4, opening paragraph.
 *
 * Mutation hooks: building with -DPPC_ORACLE_PLANT=<id> plants one known
 * mistake (used only by the test that shows the pins catch such mistakes).
 * A normal build defines nothing and compiles none of them.
 */
#include "ppc_oracle.h"

#include <pthread.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#ifndef PPC_ORACLE_PLANT
#define PPC_ORACLE_PLANT 0
#endif
#define PLANT(id) (PPC_ORACLE_PLANT == (id))

static int valid_k(int k) { return k == 8 || k == 16 || k == 32 || k == 64; }

/* Word j: the k/8 bytes at bytes + j*k/8, least significant byte first. */
static uint64_t load_word(const uint8_t* bytes, uint64_t j, int k) {
    const uint64_t wb = (uint64_t)(k / 8);
    const uint8_t* src = bytes + j * wb;
    uint64_t w = 0;
    for (uint64_t b = 0; b < wb; ++b) {
        if (PLANT(1))
            w |= (uint64_t)src[b] << (8 * (wb - 1 - b)); /* planted: big-endian */
        else
            w |= (uint64_t)src[b] << (8 * b);
    }
    return w;
}

int ppc_oracle_count(const uint8_t* bytes, uint64_t n, int k, uint64_t* counts) {
    if (!valid_k(k)) return -1;
    uint64_t end = n;
    if (PLANT(2) && end > 0) end -= 1; /* planted: last word dropped */
    for (uint64_t j = 0; j < end; ++j) {
        const uint64_t w = load_word(bytes, j, k);
        for (int p = 0; p < k; ++p) {
            /* Fig. 3: shift the word right by p, keep the lowest bit, add. */
            if (PLANT(3))
                counts[p] += (w >> ((p + 1) % k)) & 1u; /* planted: index off by one */
            else if (PLANT(4))
                counts[p] = (w >> p) & 1u; /* planted: overwrite instead of add */
            else
                counts[p] += (w >> p) & 1u;
        }
    }
    return 0;
}

typedef struct {
    const uint8_t* bytes;
    uint64_t first, count;
    int k;
    uint64_t partial[64];
} chunk_job;

static void* chunk_main(void* arg) {
    chunk_job* job = (chunk_job*)arg;
    memset(job->partial, 0, sizeof(job->partial));
    ppc_oracle_count(job->bytes + job->first * (uint64_t)(job->k / 8), job->count, job->k,
                     job->partial);
    return NULL;
}

int ppc_oracle_count_mt(const uint8_t* bytes, uint64_t n, int k, uint64_t* counts,
                        int threads) {
    if (!valid_k(k)) return -1;
    if (threads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        threads = c > 0 ? (int)c : 1;
    }
    if ((uint64_t)threads > n) threads = n > 0 ? (int)n : 1;
    chunk_job* jobs = (chunk_job*)calloc((size_t)threads, sizeof(chunk_job));
    pthread_t* tid = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1;
    }
    /* Contiguous word ranges; the first n % threads ranges get one extra word. */
    const uint64_t base = n / (uint64_t)threads, extra = n % (uint64_t)threads;
    uint64_t first = 0;
    for (int t = 0; t < threads; ++t) {
        uint64_t cnt = base + ((uint64_t)t < extra ? 1 : 0);
        if (PLANT(5) && t > 0 && cnt > 0) { /* planted: a word lost at each split */
            first += 1;
            cnt -= 1;
        }
        jobs[t].bytes = bytes;
        jobs[t].first = first;
        jobs[t].count = cnt;
        jobs[t].k = k;
        first += cnt;
    }
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, chunk_main, &jobs[t]) != 0) break;
        started = t;
    }
    chunk_main(&jobs[0]);
    for (int t = started + 1; t < threads; ++t) chunk_main(&jobs[t]); /* not started */
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    for (int t = 0; t < threads; ++t)
        for (int p = 0; p < k; ++p) counts[p] += jobs[t].partial[p];
    free(jobs);
    free(tid);
    return threads;
}

/* Sec. 2, Fig. "csacpp": l = (a xor b) xor c; h = (a and b) or ((a xor b) and c). */
void ppc_oracle_csa(uint64_t a, uint64_t b, uint64_t c, uint64_t* h, uint64_t* l) {
    const uint64_t u = a ^ b;
    if (PLANT(6))
        *h = a & b; /* planted: carry term (a xor b) and c dropped */
    else
        *h = (a & b) | (u & c);
    *l = u ^ c;
}

/* ---- Model of the Sec. 4.1 algorithm (16-bit words, 512-bit registers) ---- */

enum { REG_LIMBS = 8, REG_BYTES = 64, REG_WORDS = 32 };
typedef struct {
    uint64_t limb[REG_LIMBS]; /* bits 64*i .. 64*i+63 of the 512-bit register */
} reg512;

typedef struct {
    uint64_t csa_calls;
} hs_ctx;

/* The CSA applied limb by limb: a 512-bit CSA is 8 independent 64-bit CSAs
 * (bitwise operations act on each bit position independently). */
static void csa512(hs_ctx* ctx, reg512* h, reg512* l, const reg512* a, const reg512* b,
                   const reg512* c) {
    for (int i = 0; i < REG_LIMBS; ++i)
        ppc_oracle_csa(a->limb[i], b->limb[i], c->limb[i], &h->limb[i], &l->limb[i]);
    ctx->csa_calls += 1;
}

static void load_reg(reg512* r, const uint8_t* src) {
    for (int i = 0; i < REG_LIMBS; ++i) {
        uint64_t v = 0;
        for (int b = 0; b < 8; ++b) v |= (uint64_t)src[8 * i + b] << (8 * b);
        r->limb[i] = v;
    }
}

/* F_N(d_0 .. d_{2^N - 1}; B_0 .. B_{N-1}) -> updated B_0 .. B_{N-1} and the new
 * B_N, returned in *carry.  Sec. 2: F_1 is one CSA of B_0 with two inputs; F_{N+1}
 * runs F_N on the first 2^N inputs, passes the updated B_0 .. B_{N-1} to a second
 * F_N on the next 2^N inputs, and combines the incoming B_N with the two B_N
 * values the two calls produced, using one more CSA. */
static void hs_circuit(hs_ctx* ctx, int N, const reg512* d, reg512* B, reg512* carry) {
    if (N == 1) {
        reg512 h, l;
        csa512(ctx, &h, &l, &B[0], &d[0], &d[1]);
        B[0] = l;
        *carry = h;
        return;
    }
    reg512 x, y, h, l;
    hs_circuit(ctx, N - 1, d, B, &x);
    hs_circuit(ctx, N - 1, d + (1 << (N - 1)), B, &y);
    csa512(ctx, &h, &l, &B[N - 1], &x, &y);
    B[N - 1] = l;
    *carry = h;
}

/* Fig. 6 (scalar form given beside it): for each position p, add bit p of every
 * 16-bit word of the register to counter p. */
static void count_positions(const reg512* r, uint64_t weight, uint64_t* counts) {
    for (int w = 0; w < REG_WORDS; ++w) {
        const uint64_t word = (r->limb[w / 4] >> (16 * (w % 4))) & 0xFFFFu;
        for (int p = 0; p < 16; ++p) counts[p] += weight * ((word >> p) & 1u);
    }
}

int ppc_oracle_hs16(const uint8_t* data, uint64_t n, int N, uint64_t* counts,
                    uint64_t* csa_calls) {
    if (N < 1 || N > 6) return -1;
    hs_ctx ctx = {0};
    const uint64_t block_regs = (uint64_t)1 << N;
    const uint64_t block_words = block_regs * REG_WORDS;
    const uint64_t blocks = n / block_words;

    reg512 B[6];
    memset(B, 0, sizeof(B));
    uint64_t carry_counts[16] = {0}; /* counts of B_N, weight 2^N applied at the end */
    reg512* d = (reg512*)malloc(sizeof(reg512) * (size_t)block_regs);
    if (!d) return -1;
    for (uint64_t blk = 0; blk < blocks; ++blk) {
        for (uint64_t r = 0; r < block_regs; ++r)
            load_reg(&d[r], data + (blk * block_regs + r) * REG_BYTES);
        reg512 carry;
        hs_circuit(&ctx, N, d, B, &carry);
        count_positions(&carry, 1, carry_counts);
    }
    free(d);
    /* Deferred multiplication of the carry counts by 2^N (Sec. 4.1). */
    for (int p = 0; p < 16; ++p)
        counts[p] += (PLANT(7) ? ((uint64_t)1 << (N - 1)) : ((uint64_t)1 << N)) * carry_counts[p];
    /* Remaining bits of the running registers, with weights 1, 2, 4, ... */
    for (int i = 0; i < N; ++i) count_positions(&B[i], (uint64_t)1 << i, counts);
    /* Scalar residual for the words after the last whole block. */
    const uint64_t done = blocks * block_words;
    ppc_oracle_count(data + done * 2, n - done, 16, counts);
    if (csa_calls) *csa_calls = ctx.csa_calls;
    return 0;
}

/* ---- Histogram of categorical ids (Sec. 1, Table 1) ---- */

int ppc_oracle_histogram(const uint8_t* ids, uint64_t n, int id_bytes, int bins,
                         uint64_t* counts) {
    if ((id_bytes != 1 && id_bytes != 2) || bins < 1 || bins > 64) return -1;
    for (uint64_t j = 0; j < n; ++j) {
        uint64_t id = ids[j * (uint64_t)id_bytes];
        if (id_bytes == 2) id |= (uint64_t)ids[j * 2 + 1] << 8;
        const uint64_t limit = PLANT(8) ? (uint64_t)bins - 1 : (uint64_t)bins;
        if (id < limit)  /* planted: the last category treated as out of range */
            counts[id] += 1;
        else
            counts[bins] += 1;
    }
    return 0;
}

/* ---- Wider words held as 16-bit planes (Sec. 4) ---- */

int ppc_oracle_count_planes(const uint8_t* const* planes, int m, uint64_t n, uint64_t* counts) {
    if (m < 1 || m > 64) return -1;
    for (int j = 0; j < m; ++j) {
        /* limb j of every word counts toward word bits 16j .. 16j+15 */
        const int first = PLANT(9) ? 16 * (m - 1 - j) : 16 * j; /* planted: planes reversed */
        if (ppc_oracle_count(planes[j], n, 16, counts + first) != 0) return -1;
    }
    return 0;
}
