// ppc_internal.h -- host-side helpers shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pospopcnt.h"

namespace ppc {

// Remember a failed HIP call for ppc_last_hip_error() and map it to a status.
int fail_hip(hipError_t e);

#define PPC_HIP(call)                                   \
    do {                                                \
        hipError_t e_ = (call);                         \
        if (e_ != hipSuccess) return ::ppc::fail_hip(e_); \
    } while (0)

struct DeviceFacts {
    int device = -1;
    int cus = 0;
    int clock_khz = 0;
    int l2_bytes = 0;
    int64_t global_mem = 0;
    char name[64] = {0};
    char arch[64] = {0};
};

// Facts of the current device (cached per device id).  Returns PPC_OK or an error.
int current_device(const DeviceFacts** out);

// Byte-range split of a stream: a head before the first 16-byte boundary, a
// 16-byte aligned body of `units` dwordx4 units, and a tail after the last one.
struct Split {
    const uint8_t* head;  // first head byte (== ptr)
    const uint8_t* tail;  // first tail byte
    uint32_t head_len;    // 0 .. 15
    uint32_t tail_len;    // 0 .. 15
    const void* body;     // 16-byte aligned
    uint64_t units;       // body length / 16
    uint32_t rot;         // 8 * (ptr mod (k/8)): dword bit i is word bit (i - rot) mod k
};

Split split_stream(const void* ptr, uint64_t nbytes, int k);

// Argument checks common to the single-stream entry points.
int check_stream_args(const void* ptr, uint64_t n, int k, const uint64_t* counts,
                      uint64_t* nbytes_out);

// Launch configuration after defaults and validation.
struct Launch {
    int variant;
    int logd;      // circuit of 2^logd dwords per lane per step
    int threads;   // block size
    int64_t grid;  // blocks
};

// Validate and launch the single-stream kernel (the body of pospopcnt_ex).
// k = 64 single stream (ppc_wide.hip); launch_stream routes k = 64 here.
int launch_wide64(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream,
                  const ppc_launch_config* cfg);

int launch_stream(const void* ptr, uint64_t n, int k, uint64_t* counts, ppc_stream stream,
                  const ppc_launch_config* cfg);

// pospopcnt_batch without graph capture, clearing each valid descriptor's
// counters before counting (the descriptors must own distinct counters).  bytes:
// the batch's input bytes if known (sizes the grid for small batches), else 0.
// dsts: NULL, or per descriptor the address its input bytes are also copied to
// while they are counted (congruent to the input's address modulo 16, and not
// overlapping any input or counter); the array lives where descs does.
int batch_fresh(ppc_plan* plan, const ppc_desc* d_descs, uint32_t m, hipStream_t stream,
                uint64_t bytes, uint8_t* const* dsts = nullptr);

// As batch_fresh for callers whose counters are zero already (the serving
// executor clears them after reading them back): up to kSmallBatch descriptors run
// as one kernel that prepares its own shares, larger batches as batch_fresh.  Up to
// kSmallBatch, descs may also be pinned host memory (each block reads them once).
constexpr uint32_t kSmallBatch = 1024;
int batch_zeroed(ppc_plan* plan, const ppc_desc* descs, uint32_t m, hipStream_t stream,
                 uint64_t bytes, uint8_t* const* dsts = nullptr);
// The grid batch_zeroed launches for m <= kSmallBatch descriptors and `bytes` of input.
uint32_t small_batch_grid(const ppc_plan* plan, uint32_t m, uint64_t bytes);
// Descriptors a launch may read from pinned host memory, summed over its blocks,
// before one small host-to-device copy is the cheaper way.
constexpr uint64_t kDirectReads = 2048;

int resolve_launch(const ppc_launch_config* cfg, int k, uint64_t units, bool has_edges,
                   uint64_t nbytes, Launch* out);

// Launch-shape overrides from the environment, read once per process.
//   PPC_LAUNCH_U8 / _U16 / _U32 / _U64, else PPC_LAUNCH: "key=value,..." with keys
//   variant (csa, ballot, hybrid or 0..2), depth, block_threads, blocks_per_cu and
//   grid.  They fill the fields a call leaves at zero (an explicit configuration
//   wins).  *bad is set when the variable does not parse.
struct EnvLaunch {
    ppc_launch_config cfg{};
    bool set = false, bad = false;
};
const EnvLaunch& env_launch(int k);
// PPC_BATCH_CONFIG: "depth=..,block_threads=..,blocks_per_cu=..,stream_weight=..", the
// initial configuration of every new plan (absent fields keep the default).
struct EnvBatch {
    ppc_batch_config cfg{};
    bool set = false, bad = false;
};
const EnvBatch& env_batch();
// Parses "key=value,key=value" into (key, value) pairs; false on a syntax error.
bool parse_kv(const char* text, int (*apply)(void* ctx, const char* key, const char* value),
              void* ctx);

// Blocks a launch needs for `tiles` wave tiles with `wpb` waves per block: at least
// two tiles per wave, both in flight at once.  Every block ends with one atomic per
// counter on the same few counters, and those atomics serialise, so on a small input
// one tile per wave costs more in flushes than it saves in latency: 2 MiB of uint16
// words took 4.3 us per back-to-back call on 128 four-wave blocks (one tile each),
// 3.7 us on 64 (two each), 3.75 us on 32 (four each).  Large inputs are unaffected:
// their grids stop at the blocks that fit on the chip.
inline uint64_t blocks_needed(uint64_t tiles, int wpb) {
    const uint64_t per = 2 * (uint64_t)wpb;
    return (tiles + per - 1) / per;
}

// log2 of a circuit depth of 4, 8, 16 or 32 dwords per lane; -1 for any other.
inline int logd_of_depth(int depth) {
    return depth == 4 ? 2 : depth == 8 ? 3 : depth == 16 ? 4 : depth == 32 ? 5 : -1;
}

}  // namespace ppc
