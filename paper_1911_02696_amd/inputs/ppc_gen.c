/*
 * ppc_gen.c -- seeded synthetic inputs for the positional population count.
 *
 * This module only draws bytes; it computes nothing of the counting method and
 * is shared by the tests, the benchmark and the serving demo.  It is built
 * into its own library, apart from the GPU library and from the oracle.
 *
 * Generator: counter-based SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014): output i of a stream with key
 * K is mix(K + (i + 1) * GOLDEN), where mix is the published 64-bit finaliser
 * (shift-xor 30, multiply, shift-xor 27, multiply, shift-xor 31).  Being
 * counter-based, any byte range of a stream can be generated on its own and in
 * parallel, and the bytes do not depend on the chunking or thread count.
 *
 * Distributions (the paper generates random words, Sec. 5; the one-hot case is
 * its motivating example, Sec. 1):
 *   UNIFORM   : every byte uniform (each bit Bernoulli(1/2)); byte j is byte
 *               j % 8 of output j / 8.
 *   BERNOULLI : bit g (bit g % 8 of byte g / 8) is set iff u_g < threshold,
 *               where u_g is the low (g even) or high (g odd) 32-bit half of
 *               output g / 2 and threshold = floor(p * 2^32) in [0, 2^32].
 *   ONEHOT    : word w (k bits, little-endian) is 1 << c, where u = high half
 *               of output w and c is the largest index with cdf[c] <= u
 *               (cdf[0] = 0 < cdf[1] <= ... <= cdf[k] = 2^32).
 *   IDS       : word w (k = 8 or 16 bits) is the category index c itself, drawn
 *               as for ONEHOT over ncat categories (cdf[0..ncat]); with
 *               threshold > 0, a word whose low output half is below threshold
 *               is instead an id >= ncat (ncat + low half mod 7): an id with no
 *               category.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

enum { PPCGEN_UNIFORM = 0, PPCGEN_BERNOULLI = 1, PPCGEN_ONEHOT = 2, PPCGEN_IDS = 3 };

typedef struct {
    int32_t kind;
    int32_t k;           /* word bits for ONEHOT (8, 16, 32, 64) and IDS (8, 16) */
    uint64_t key;        /* stream key, see ppcgen_key */
    uint64_t threshold;  /* BERNOULLI; IDS: share of ids without a category, scaled to 2^32 */
    uint64_t cdf[65];    /* ONEHOT, IDS */
    int32_t ncat;        /* IDS: number of categories (1 .. 64) */
    int32_t unused;
} ppcgen_spec;

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t draw(uint64_t key, uint64_t i) { return mix64(key + (i + 1) * GOLDEN); }

/* Key of sub-stream `stream` of a seed: output `stream` of the stream keyed by the seed. */
uint64_t ppcgen_key(uint64_t seed, uint64_t stream) { return draw(seed, stream); }

uint64_t ppcgen_draw(uint64_t key, uint64_t i) { return draw(key, i); }

static uint8_t bernoulli_byte(uint64_t key, uint64_t j, uint64_t thr) {
    uint8_t v = 0;
    for (int q = 0; q < 4; ++q) {
        const uint64_t x = draw(key, 4 * j + (uint64_t)q);
        v |= (uint8_t)(((x & 0xFFFFFFFFu) < thr) << (2 * q));
        v |= (uint8_t)(((x >> 32) < thr) << (2 * q + 1));
    }
    return v;
}

static int category(const ppcgen_spec* s, uint64_t x, int ncat) {
    const uint64_t u = x >> 32;
    int lo = 0, hi = ncat; /* invariant: cdf[lo] <= u < cdf[hi] */
    while (hi - lo > 1) {
        const int mid = (lo + hi) / 2;
        if (s->cdf[mid] <= u) lo = mid; else hi = mid;
    }
    return lo;
}

static uint64_t onehot_word(const ppcgen_spec* s, uint64_t w) {
    return (uint64_t)1 << category(s, draw(s->key, w), s->k);
}

static uint64_t id_word(const ppcgen_spec* s, uint64_t w) {
    const uint64_t x = draw(s->key, w);
    if ((x & 0xFFFFFFFFu) < s->threshold) return (uint64_t)s->ncat + (x & 0xFFFFFFFFu) % 7;
    return (uint64_t)category(s, x, s->ncat);
}

static void fill_range(uint8_t* out, uint64_t first, uint64_t nbytes, const ppcgen_spec* s) {
    uint64_t j = first;
    const uint64_t end = first + nbytes;
    switch (s->kind) {
    case PPCGEN_UNIFORM:
        while (j < end) {
            const uint64_t x = draw(s->key, j / 8);
            for (uint64_t b = j % 8; b < 8 && j < end; ++b, ++j) out[j - first] = (uint8_t)(x >> (8 * b));
        }
        break;
    case PPCGEN_BERNOULLI:
        for (; j < end; ++j) out[j - first] = bernoulli_byte(s->key, j, s->threshold);
        break;
    case PPCGEN_ONEHOT:
    case PPCGEN_IDS: {
        const uint64_t wb = (uint64_t)(s->k / 8);
        while (j < end) {
            const uint64_t w = j / wb;
            const uint64_t word = s->kind == PPCGEN_ONEHOT ? onehot_word(s, w) : id_word(s, w);
            for (uint64_t b = j % wb; b < wb && j < end; ++b, ++j)
                out[j - first] = (uint8_t)(word >> (8 * b));
        }
        break;
    }
    default:
        memset(out, 0, (size_t)nbytes);
    }
}

typedef struct {
    uint8_t* out;
    uint64_t first, nbytes;
    const ppcgen_spec* spec;
} fill_job;

static void* fill_main(void* arg) {
    fill_job* f = (fill_job*)arg;
    fill_range(f->out, f->first, f->nbytes, f->spec);
    return NULL;
}

/* Writes bytes [first, first + nbytes) of the stream described by spec to out.
 * threads <= 0: one per online CPU.  Returns 0, or -1 on a bad spec. */
int ppcgen_fill(uint8_t* out, uint64_t first, uint64_t nbytes, const ppcgen_spec* spec,
                int threads) {
    if (spec->kind < 0 || spec->kind > 3) return -1;
    if (spec->kind == PPCGEN_ONEHOT &&
        !(spec->k == 8 || spec->k == 16 || spec->k == 32 || spec->k == 64))
        return -1;
    if (spec->kind == PPCGEN_IDS &&
        (!(spec->k == 8 || spec->k == 16) || spec->ncat < 1 || spec->ncat > 64))
        return -1;
    if (threads <= 0) {
        long c = sysconf(_SC_NPROCESSORS_ONLN);
        threads = c > 0 ? (int)c : 1;
    }
    const uint64_t grain = 1 << 20;
    if ((uint64_t)threads > nbytes / grain) threads = (int)(nbytes / grain);
    if (threads < 1) threads = 1;
    fill_job* jobs = (fill_job*)calloc((size_t)threads, sizeof(fill_job));
    pthread_t* tid = (pthread_t*)calloc((size_t)threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        return -1;
    }
    /* Split at multiples of 64 bytes (a whole number of words for every k). */
    uint64_t per = (nbytes / (uint64_t)threads + 63) & ~(uint64_t)63, off = 0;
    for (int t = 0; t < threads; ++t) {
        const uint64_t len = off >= nbytes ? 0 : (nbytes - off < per ? nbytes - off : per);
        jobs[t].out = out + off;
        jobs[t].first = first + off;
        jobs[t].nbytes = len;
        jobs[t].spec = spec;
        off += len;
    }
    int started = 0;
    for (int t = 1; t < threads; ++t) {
        if (pthread_create(&tid[t], NULL, fill_main, &jobs[t]) != 0) break;
        started = t;
    }
    fill_main(&jobs[0]);
    for (int t = started + 1; t < threads; ++t) fill_main(&jobs[t]);
    for (int t = 1; t <= started; ++t) pthread_join(tid[t], NULL);
    free(jobs);
    free(tid);
    return 0;
}
