// ppc_api.hip -- status codes, argument checks, stream splitting, device facts.
#include <stdlib.h>
#include <string.h>

#include <mutex>

#include "ppc_internal.h"

namespace ppc {

static thread_local int g_last_hip = 0;

int fail_hip(hipError_t e) {
    g_last_hip = (int)e;
    return PPC_ERR_HIP;
}

int current_device(const DeviceFacts** out) {
    static std::mutex mu;
    static DeviceFacts facts[64];
    int dev = 0;
    PPC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return PPC_ERR_ARG;
    std::lock_guard<std::mutex> lock(mu);
    DeviceFacts& f = facts[dev];
    if (f.device != dev) {
        hipDeviceProp_t prop;
        PPC_HIP(hipGetDeviceProperties(&prop, dev));
        f.cus = prop.multiProcessorCount;
        f.clock_khz = prop.clockRate;
        f.l2_bytes = prop.l2CacheSize;
        f.global_mem = (int64_t)prop.totalGlobalMem;
        strncpy(f.name, prop.name, sizeof(f.name) - 1);
        strncpy(f.arch, prop.gcnArchName, sizeof(f.arch) - 1);
        f.device = dev;
    }
    *out = &f;
    return PPC_OK;
}

bool parse_kv(const char* text, int (*apply)(void*, const char*, const char*), void* ctx) {
    char buf[512];
    if (!text || strlen(text) >= sizeof(buf)) return false;
    strcpy(buf, text);
    char* save = nullptr;
    for (char* tok = strtok_r(buf, ",", &save); tok; tok = strtok_r(nullptr, ",", &save)) {
        while (*tok == ' ') ++tok;
        char* eq = strchr(tok, '=');
        if (!eq || eq == tok || !eq[1]) return false;
        *eq = 0;
        if (!apply(ctx, tok, eq + 1)) return false;
    }
    return true;
}

static bool to_int(const char* v, long long* out) {
    char* end = nullptr;
    const long long x = strtoll(v, &end, 10);
    if (!end || end == v || *end) return false;
    *out = x;
    return true;
}

static int apply_launch(void* ctx, const char* key, const char* value) {
    ppc_launch_config& c = *(ppc_launch_config*)ctx;
    long long x = 0;
    if (!strcmp(key, "variant")) {
        if (!strcmp(value, "csa")) c.variant = PPC_VARIANT_CSA;
        else if (!strcmp(value, "ballot")) c.variant = PPC_VARIANT_BALLOT;
        else if (!strcmp(value, "hybrid")) c.variant = PPC_VARIANT_HYBRID;
        else if (to_int(value, &x) && x >= 0 && x <= 2) c.variant = (int32_t)x;
        else return 0;
        return 1;
    }
    if (!to_int(value, &x) || x < 0 || x > 0x7fffffff) return 0;
    if (!strcmp(key, "depth")) c.depth = (int32_t)x;
    else if (!strcmp(key, "block_threads")) c.block_threads = (int32_t)x;
    else if (!strcmp(key, "blocks_per_cu")) c.blocks_per_cu = (int32_t)x;
    else if (!strcmp(key, "grid")) c.grid = x;
    else return 0;
    return 1;
}

const EnvLaunch& env_launch(int k) {
    static EnvLaunch table[4];
    static std::once_flag once;
    std::call_once(once, [] {
        const char* names[4] = {"PPC_LAUNCH_U8", "PPC_LAUNCH_U16", "PPC_LAUNCH_U32",
                                "PPC_LAUNCH_U64"};
        const char* all = getenv("PPC_LAUNCH");
        for (int i = 0; i < 4; ++i) {
            const char* v = getenv(names[i]);
            if (!v) v = all;
            if (!v) continue;
            table[i].set = true;
            table[i].bad = !parse_kv(v, apply_launch, &table[i].cfg);
        }
    });
    return table[k == 8 ? 0 : k == 16 ? 1 : k == 32 ? 2 : 3];
}

static int apply_batch(void* ctx, const char* key, const char* value) {
    ppc_batch_config& c = *(ppc_batch_config*)ctx;
    long long x = 0;
    if (!to_int(value, &x) || x < 0 || x > 0x7fffffff) return 0;
    if (!strcmp(key, "depth")) c.depth = (int32_t)x;
    else if (!strcmp(key, "block_threads")) c.block_threads = (int32_t)x;
    else if (!strcmp(key, "blocks_per_cu")) c.blocks_per_cu = (int32_t)x;
    else if (!strcmp(key, "stream_weight")) c.stream_weight = (int32_t)x;
    else return 0;
    return 1;
}

const EnvBatch& env_batch() {
    static EnvBatch e;
    static std::once_flag once;
    std::call_once(once, [] {
        const char* v = getenv("PPC_BATCH_CONFIG");
        if (!v) return;
        e.set = true;
        e.bad = !parse_kv(v, apply_batch, &e.cfg);
    });
    return e;
}

Split split_stream(const void* ptr, uint64_t nbytes, int k) {
    const uintptr_t p = (uintptr_t)ptr, end = p + nbytes;
    const uintptr_t a0 = (p + 15) & ~(uintptr_t)15;
    Split s;
    s.rot = 8u * (uint32_t)(p % (uintptr_t)(k / 8));
    s.head = (const uint8_t*)ptr;
    if (a0 >= end) {  // fits before the first 16-byte boundary
        s.head_len = (uint32_t)nbytes;
        s.body = (const void*)a0;
        s.units = 0;
        s.tail = (const uint8_t*)end;
        s.tail_len = 0;
        return s;
    }
    const uintptr_t a1 = end & ~(uintptr_t)15;
    s.head_len = (uint32_t)(a0 - p);
    s.body = (const void*)a0;
    s.units = (uint64_t)(a1 - a0) / 16;
    s.tail = (const uint8_t*)a1;
    s.tail_len = (uint32_t)(end - a1);
    return s;
}

int check_stream_args(const void* ptr, uint64_t n, int k, const uint64_t* counts,
                      uint64_t* nbytes_out) {
    if (k != 8 && k != 16 && k != 32 && k != 64) return PPC_ERR_WIDTH;
    *nbytes_out = 0;
    if (n == 0) return PPC_OK;
    const uint64_t wb = (uint64_t)(k / 8);
    if (n > UINT64_MAX / wb) return PPC_ERR_RANGE;
    const uint64_t nbytes = n * wb;
    if (!ptr || !counts) return PPC_ERR_NULL;
    if ((uintptr_t)counts & 7u) return PPC_ERR_ALIGN;
    const uintptr_t p = (uintptr_t)ptr;
    if (p + nbytes < p) return PPC_ERR_RANGE;
    const uintptr_t c0 = (uintptr_t)counts, c1 = c0 + 8u * (uintptr_t)k;
    if (c0 < p + nbytes && p < c1) return PPC_ERR_OVERLAP;
    *nbytes_out = nbytes;
    return PPC_OK;
}

}  // namespace ppc

using namespace ppc;

extern "C" {

const char* ppc_status_string(int status) {
    switch (status) {
    case PPC_OK: return "PPC_OK";
    case PPC_ERR_NULL: return "PPC_ERR_NULL: required pointer is NULL";
    case PPC_ERR_ALIGN: return "PPC_ERR_ALIGN: counts or descriptors not 8-byte aligned";
    case PPC_ERR_WIDTH:
        return "PPC_ERR_WIDTH: word width must be 8, 16, 32 or 64 (8, 16 or 32 in batches and "
               "serving)";
    case PPC_ERR_RANGE: return "PPC_ERR_RANGE: byte length overflows 64 bits";
    case PPC_ERR_HIP: return "PPC_ERR_HIP: a HIP runtime call failed";
    case PPC_ERR_BUDGET: return "PPC_ERR_BUDGET: request exceeds the memory budget";
    case PPC_ERR_ARG: return "PPC_ERR_ARG: argument out of range";
    case PPC_ERR_OVERLAP: return "PPC_ERR_OVERLAP: counts overlaps the input";
    case PPC_ERR_STATE: return "PPC_ERR_STATE: call not allowed in the object's state";
    case PPC_ERR_CAPACITY:
        return "PPC_ERR_CAPACITY: more than the library's fixed capacity (streams or blocks)";
    case PPC_ERR_TIMEOUT: return "PPC_ERR_TIMEOUT: the request waited longer than its timeout";
    case PPC_ERR_CANCELLED: return "PPC_ERR_CANCELLED: the request was cancelled before its launch";
    default: return "unknown pospopcnt status";
    }
}

int ppc_last_hip_error(void) { return g_last_hip; }

int ppc_get_device_info(ppc_device_info* info) {
    if (!info) return PPC_ERR_NULL;
    const DeviceFacts* f = nullptr;
    int st = current_device(&f);
    if (st) return st;
    memset(info, 0, sizeof(*info));
    info->device = f->device;
    info->compute_units = f->cus;
    info->clock_khz = f->clock_khz;
    info->l2_bytes = f->l2_bytes;
    info->global_mem_bytes = f->global_mem;
    memcpy(info->name, f->name, sizeof(info->name));
    memcpy(info->arch, f->arch, sizeof(info->arch));
    return PPC_OK;
}

}  // extern "C"
