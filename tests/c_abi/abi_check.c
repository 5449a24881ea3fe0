/* A C caller of include/pospopcnt.h: the library's boundary used from C, with no
 * Python or C++ in between.  Test infrastructure, built by build.py beside it.
 *
 *   abi_check cpu   argument checks that return before any device call, the status
 *                   strings and the constants of the header
 *   abi_check gpu   counts of device buffers against closed forms: all-ones words
 *                   set every position once per word, all-zero words none, and a
 *                   constant id stream falls in that id's category (or outside)
 *   abi_check calls N   host time per call of N back-to-back pospopcnt_u16 calls on
 *                   2^20 words (2 MiB) on the null stream, after 100 untimed calls;
 *                   prints {"c_us_per_call": ...} (the per-call cost of the boundary
 *                   itself, with no Python in between)
 *
 * Prints one line and exits 0 when every check holds, 1 otherwise. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <time.h>

#include <hip/hip_runtime_api.h>

#include "pospopcnt.h"

static int failures = 0;

#define EXPECT(cond)                                                      \
    do {                                                                  \
        if (!(cond)) {                                                    \
            fprintf(stderr, "%s:%d: check failed: %s\n", __FILE__, __LINE__, #cond); \
            ++failures;                                                   \
        }                                                                 \
    } while (0)

static int cpu_checks(void) {
    uint64_t fake_counts[64];
    EXPECT(PPC_OK == 0 && PPC_ERR_NULL == 1 && PPC_ERR_ALIGN == 2 && PPC_ERR_WIDTH == 3);
    EXPECT(PPC_ERR_RANGE == 4 && PPC_ERR_HIP == 5 && PPC_ERR_ARG == 7 && PPC_ERR_OVERLAP == 8);
    EXPECT(PPC_VARIANT_CSA == 0 && PPC_VARIANT_BALLOT == 1 && PPC_VARIANT_HYBRID == 2);
    EXPECT(sizeof(ppc_desc) == 32);
    /* n = 0 does nothing, whatever the pointers */
    EXPECT(pospopcnt_u8(NULL, 0, NULL, NULL) == PPC_OK);
    EXPECT(pospopcnt_u16(NULL, 0, NULL, NULL) == PPC_OK);
    EXPECT(pospopcnt_u32(NULL, 0, NULL, NULL) == PPC_OK);
    EXPECT(pospopcnt_u64(NULL, 0, NULL, NULL) == PPC_OK);
    /* missing pointers, a width with no kernel, a misaligned counts array */
    EXPECT(pospopcnt_u16(NULL, 10, fake_counts, NULL) == PPC_ERR_NULL);
    EXPECT(pospopcnt_u16((const void*)0x1000, 10, NULL, NULL) == PPC_ERR_NULL);
    EXPECT(pospopcnt((const void*)0x1000, 10, 12, fake_counts, NULL) == PPC_ERR_WIDTH);
    EXPECT(pospopcnt_u16((const void*)0x1000, 10, (uint64_t*)((char*)fake_counts + 4), NULL) ==
           PPC_ERR_ALIGN);
    EXPECT(pospopcnt_u64((const void*)0x1000, (uint64_t)1 << 61, fake_counts, NULL) ==
           PPC_ERR_RANGE);
    EXPECT(ppc_histogram_u8(NULL, 10, 8, fake_counts, NULL) == PPC_ERR_NULL);
    EXPECT(ppc_histogram_u8((const void*)0x1000, 10, 33, fake_counts, NULL) == PPC_ERR_WIDTH);
    EXPECT(ppc_histogram_u8((const void*)0x1000, 10, 0, fake_counts, NULL) == PPC_ERR_WIDTH);
    EXPECT(PPC_ERR_TIMEOUT == 11 && PPC_ERR_CANCELLED == 12);
    for (int st = 0; st <= 12; ++st) {
        const char* s = ppc_status_string(st);
        EXPECT(s != NULL && strlen(s) > 0);
    }
    return failures;
}

static int read_counts(const uint64_t* d_counts, uint64_t* h, int k) {
    return hipMemcpy(h, d_counts, sizeof(uint64_t) * (size_t)k, hipMemcpyDeviceToHost) ==
           hipSuccess;
}

static int gpu_checks(void) {
    const uint64_t bytes = (16u << 20) + 77; /* a ragged length */
    void* buf = NULL;
    uint64_t* d_counts = NULL;
    uint64_t h[65];
    if (hipMalloc(&buf, bytes + 64) != hipSuccess || hipMalloc((void**)&d_counts, 8 * 65) != hipSuccess) {
        fprintf(stderr, "hipMalloc failed\n");
        return 1;
    }
    const char* p = (const char*)buf + 3; /* an unaligned start */
    /* all-ones words: every position set once per word */
    EXPECT(hipMemset(buf, 0xFF, bytes + 64) == hipSuccess);
    const int ks[4] = {8, 16, 32, 64};
    for (int i = 0; i < 4; ++i) {
        const int k = ks[i];
        const uint64_t n = bytes / (uint64_t)(k / 8);
        EXPECT(hipMemset(d_counts, 0, 8 * 65) == hipSuccess);
        EXPECT(pospopcnt(p, n, k, d_counts, NULL) == PPC_OK);
        EXPECT(hipDeviceSynchronize() == hipSuccess && read_counts(d_counts, h, k));
        for (int q = 0; q < k; ++q) EXPECT(h[q] == n);
    }
    /* every variant adds into the counters: three calls, three times n */
    {
        const uint64_t n = bytes / 4;
        EXPECT(hipMemset(d_counts, 0, 8 * 65) == hipSuccess);
        for (int v = 0; v < 3; ++v) {
            ppc_launch_config cfg;
            memset(&cfg, 0, sizeof cfg);
            cfg.variant = v;
            EXPECT(pospopcnt_ex(p, n, 32, d_counts, NULL, &cfg) == PPC_OK);
        }
        EXPECT(hipDeviceSynchronize() == hipSuccess && read_counts(d_counts, h, 32));
        for (int q = 0; q < 32; ++q) EXPECT(h[q] == 3 * n);
    }
    /* all-zero words: nothing */
    EXPECT(hipMemset(buf, 0, bytes + 64) == hipSuccess);
    EXPECT(hipMemset(d_counts, 0, 8 * 65) == hipSuccess);
    EXPECT(pospopcnt_u16(p, bytes / 2, d_counts, NULL) == PPC_OK);
    EXPECT(hipDeviceSynchronize() == hipSuccess && read_counts(d_counts, h, 16));
    for (int q = 0; q < 16; ++q) EXPECT(h[q] == 0);
    /* a constant id stream: all n ids in that id's category, or outside */
    const unsigned ids[3] = {5, 31, 200};
    for (int i = 0; i < 3; ++i) {
        EXPECT(hipMemset(buf, (int)ids[i], bytes + 64) == hipSuccess);
        EXPECT(hipMemset(d_counts, 0, 8 * 65) == hipSuccess);
        EXPECT(ppc_histogram_u8(p, bytes, 32, d_counts, NULL) == PPC_OK);
        EXPECT(hipDeviceSynchronize() == hipSuccess && read_counts(d_counts, h, 33));
        for (unsigned c = 0; c <= 32; ++c) EXPECT(h[c] == (c == (ids[i] < 32 ? ids[i] : 32) ? bytes : 0));
    }
    /* counts inside the input are refused before anything is launched */
    EXPECT(pospopcnt_u16(buf, 1000, (uint64_t*)buf + 8, NULL) == PPC_ERR_OVERLAP);
    EXPECT(hipFree(buf) == hipSuccess && hipFree(d_counts) == hipSuccess);
    return failures;
}

static double now_s(void) {
    struct timespec t;
    clock_gettime(CLOCK_MONOTONIC, &t);
    return (double)t.tv_sec + 1e-9 * (double)t.tv_nsec;
}

static int time_calls(long calls) {
    const uint64_t n = 1u << 20;
    void* buf = NULL;
    uint64_t* d_counts = NULL;
    if (calls < 1 || hipMalloc(&buf, 2 * n) != hipSuccess ||
        hipMalloc((void**)&d_counts, 8 * 16) != hipSuccess) {
        fprintf(stderr, "bad call count or hipMalloc failed\n");
        return 1;
    }
    EXPECT(hipMemset(buf, 0x5A, 2 * n) == hipSuccess && hipMemset(d_counts, 0, 128) == hipSuccess);
    for (int i = 0; i < 100; ++i) EXPECT(pospopcnt_u16(buf, n, d_counts, NULL) == PPC_OK);
    EXPECT(hipDeviceSynchronize() == hipSuccess);
    const double t0 = now_s();
    for (long i = 0; i < calls; ++i)
        if (pospopcnt_u16(buf, n, d_counts, NULL) != PPC_OK) ++failures;
    EXPECT(hipDeviceSynchronize() == hipSuccess);
    const double dt = now_s() - t0;
    uint64_t h[16];
    EXPECT(read_counts(d_counts, h, 16));
    /* 0x5A5A = bits 1, 3, 4, 6 of each byte set: positions 1,3,4,6,9,11,12,14 */
    for (int q = 0; q < 16; ++q)
        EXPECT(h[q] == (((0x5A5Au >> q) & 1u) ? n * (uint64_t)(calls + 100) : 0));
    EXPECT(hipFree(buf) == hipSuccess && hipFree(d_counts) == hipSuccess);
    printf("{\"c_us_per_call\": %.3f, \"calls\": %ld, \"words\": %llu, \"ok\": %s}\n",
           1e6 * dt / (double)calls, calls, (unsigned long long)n, failures ? "false" : "true");
    return failures ? 1 : 0;
}

int main(int argc, char** argv) {
    if (argc == 3 && strcmp(argv[1], "calls") == 0) return time_calls(atol(argv[2]));
    if (argc != 2 || (strcmp(argv[1], "cpu") != 0 && strcmp(argv[1], "gpu") != 0)) {
        fprintf(stderr, "usage: %s cpu|gpu|calls N\n", argv[0]);
        return 2;
    }
    const int gpu = strcmp(argv[1], "gpu") == 0;
    const int bad = gpu ? gpu_checks() : cpu_checks();
    printf("c abi %s: %s (%d failed checks)\n", argv[1], bad ? "FAILED" : "ok", bad);
    return bad ? 1 : 0;
}
