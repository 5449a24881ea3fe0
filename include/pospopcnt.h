/*
 * pospopcnt.h -- C ABI of the MI355X (gfx950) positional population count.
 *
 * Operation (Klarqvist, Mula, Lemire, "Efficient Computation of Positional
 * Population Counts Using SIMD Instructions", abstract, Sec. 1 and Sec. 4,
 * Fig. 3): given n words of k bits, counts[p] += number of words whose bit p is
 * set, for p = 0 .. k-1.  For one-hot words the k sums are a frequency
 * histogram (Sec. 1, Table 1).
 *
 * Conventions shared by every entry point:
 *   - Word j of a stream at byte address ptr is the k/8 bytes at ptr + j*k/8,
 *     least significant byte first.  ptr may be any byte address.
 *   - Counts are 64-bit and are ADDED INTO (the paper's counters start at zero
 *     and are only incremented, Sec. 4, Fig. 3): zero them for a fresh count.
 *     Splitting a stream into pieces and counting each piece into the same
 *     counts gives the count of the whole stream.
 *   - Input and counts live in device memory (hipMalloc or equivalent); the
 *     caller owns them.  Unless stated otherwise no call allocates memory.
 *   - Calls are asynchronous on `stream` (a hipStream_t, NULL = null stream):
 *     arguments are validated synchronously, and on any error nothing is
 *     launched and a status is returned.  Faults inside a kernel surface at the
 *     caller's next synchronisation, as usual in HIP.
 *   - n = 0 returns PPC_OK and launches nothing.
 *   - Calls on distinct streams may be made from several host threads.
 *   - Results are exact integers: identical on every run and for every launch
 *     configuration.
 */
#ifndef POSPOPCNT_H
#define POSPOPCNT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* A hipStream_t passed as an opaque pointer; NULL is the null stream. */
typedef void* ppc_stream;

/* Status codes returned by every entry point. */
enum {
    PPC_OK = 0,
    PPC_ERR_NULL = 1,     /* a required pointer is NULL (input or counts with n > 0) */
    PPC_ERR_ALIGN = 2,    /* counts (or a descriptor array) not 8-byte aligned */
    PPC_ERR_WIDTH = 3,    /* k is not 8, 16, 32 or 64 (8, 16 or 32 in batches and serving) */
    PPC_ERR_RANGE = 4,    /* n * k / 8 does not fit in 64 bits */
    PPC_ERR_HIP = 5,      /* a HIP runtime call failed: see ppc_last_hip_error() */
    PPC_ERR_BUDGET = 6,   /* serving: request larger than the memory budget */
    PPC_ERR_ARG = 7,      /* another argument is out of range (configuration, size) */
    PPC_ERR_OVERLAP = 8,  /* counts overlaps the input bytes */
    PPC_ERR_STATE = 9,    /* object used in a state that does not allow the call */
    PPC_ERR_CAPACITY = 10, /* a fixed capacity of the library is exceeded (see
                              pospopcnt_batch_static) */
    PPC_ERR_TIMEOUT = 11,  /* serving: the request waited longer than its timeout */
    PPC_ERR_CANCELLED = 12 /* serving: the request was cancelled before its launch */
};

/* Human-readable name of a status code (static storage, never NULL). */
const char* ppc_status_string(int status);

/* The hipError_t of the last failed HIP call made by this library on the
 * calling host thread (0 if none). */
int ppc_last_hip_error(void);

/* ------------------------------------------------------------------------
 * Single stream.
 *
 * pospopcnt_u8 / _u16 / _u32 / _u64: counts has 8 / 16 / 32 / 64 entries.
 *   ptr    device pointer to n*k/8 bytes, any alignment; may be NULL if n = 0.
 *   n      number of k-bit words (64-bit: inputs of 2^32 words and more are
 *          allowed, unlike the paper's uint32_t length, Fig. 3).
 *   counts device pointer, 8-byte aligned, k uint64 entries, added into; must
 *          not overlap the input.  Several concurrent calls may add into the
 *          same counts (the kernels flush with 64-bit device-scope atomics).
 * Errors: PPC_ERR_NULL, PPC_ERR_ALIGN, PPC_ERR_RANGE, PPC_ERR_OVERLAP,
 * PPC_ERR_HIP (launch failure).  Nothing is launched on error.
 * The work is the Harley-Seal carry-save-adder method of Sec. 4.1 (circuits of
 * Sec. 2), with the carry counted per bit position as in Fig. 6.  64-bit words
 * are the generalisation to wider words named at the start of Sec. 4: two
 * circuits per lane, one for the low and one for the high halves.
 * ---------------------------------------------------------------------- */
int pospopcnt_u8(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream);
int pospopcnt_u16(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream);
int pospopcnt_u32(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream);
int pospopcnt_u64(const void* ptr, uint64_t n, uint64_t* counts, ppc_stream stream);

/* Same, with the width k in {8, 16, 32, 64} as an argument (PPC_ERR_WIDTH otherwise). */
int pospopcnt(const void* ptr, uint64_t n, int k, uint64_t* counts, ppc_stream stream);

/* Kernel variants. */
enum {
    PPC_VARIANT_CSA = 0,     /* per-lane Harley-Seal circuit + masked popcount (Sec. 4.1) */
    PPC_VARIANT_BALLOT = 1,  /* wave-wide bit transposition: ballot per bit, popcount */
    PPC_VARIANT_HYBRID = 2   /* the CSA circuit, its carry planes counted by the ballot
                                transposition instead of per-lane class counters */
};

/* Launch configuration for pospopcnt_ex.  Zero in any field selects the
 * library's default for that field. */
typedef struct {
    int32_t variant;        /* PPC_VARIANT_CSA, or PPC_VARIANT_BALLOT or _HYBRID (k <= 32
                               only) */
    int32_t depth;          /* CSA, HYBRID: inputs per lane per circuit, 4, 8, 16 or 32
                               dwords (the 2^N-input circuits of Sec. 2, N = 2 .. 5; the
                               paper's 256 B / 512 B / 1 kB circuits have the same
                               input counts as N = 2, 3, 4: 3 / 7 / 15 CSAs per step) */
    int32_t block_threads;  /* 64 .. 256, multiple of 64 */
    int32_t blocks_per_cu;  /* resident blocks per compute unit used to size the grid */
    int64_t grid;           /* explicit number of blocks (overrides blocks_per_cu) */
} ppc_launch_config;

/* pospopcnt with an explicit launch configuration (NULL = defaults).  Same
 * contract and errors as pospopcnt, plus PPC_ERR_ARG for a field out of range.
 * Every configuration gives the same counts.
 * Overrides: the environment variable PPC_LAUNCH_U8, _U16, _U32 or _U64 (per
 * width), else PPC_LAUNCH, read once per process, as "key=value,..." with keys
 * variant (csa, ballot, hybrid), depth, block_threads, blocks_per_cu and grid,
 * fills the fields a call leaves at zero, for pospopcnt_ex and for every
 * single-stream call without a configuration.  A variable that does not parse
 * makes every such call with n > 0 return PPC_ERR_ARG. */
int pospopcnt_ex(const void* ptr, uint64_t n, int k, uint64_t* counts, ppc_stream stream,
                 const ppc_launch_config* config);

/* ------------------------------------------------------------------------
 * Wider words as several streams of 16-bit words (Sec. 4: a word of k = 16*m
 * bits held as m planes, plane j holding every word's 16-bit limb j, i.e. word
 * bits 16j .. 16j+15).
 *   planes host array of m device pointers, plane j pointing at n little-endian
 *          uint16 limbs, any alignment; the array is read during the call only.
 *   m      1 .. PPC_MAX_PLANES (PPC_ERR_ARG otherwise): k = 16m up to 512 bits.
 *   n      words (limbs per plane); all planes hold n.
 *   counts device, 8-byte aligned, 16*m uint64 entries, added into:
 *          counts[16j + p] += number of words whose bit 16j + p is set.  Must not
 *          overlap any plane.
 * One launch counts every plane (the chip's blocks are shared out over them).
 * Errors: PPC_ERR_NULL (planes, a plane or counts NULL with n > 0),
 * PPC_ERR_ALIGN, PPC_ERR_RANGE, PPC_ERR_OVERLAP, PPC_ERR_ARG, PPC_ERR_HIP.
 * pospopcnt_planes16_ex takes a launch configuration as pospopcnt_ex does (CSA
 * only; blocks_per_cu and grid count blocks per plane row of the grid).
 * ---------------------------------------------------------------------- */
#define PPC_MAX_PLANES 32
int pospopcnt_planes16(const void* const* planes, uint32_t m, uint64_t n, uint64_t* counts,
                       ppc_stream stream);
int pospopcnt_planes16_ex(const void* const* planes, uint32_t m, uint64_t n, uint64_t* counts,
                          ppc_stream stream, const ppc_launch_config* config);

/* Read-only bandwidth reference: reads the nbytes at ptr (any alignment) with
 * the same loads, tiling and grid as the CSA kernel, XOR-reduces them, and
 * XORs the result into *sink (device, 8-byte aligned).  It computes no count;
 * it measures the memory ceiling the counting kernels run against.
 * config: NULL or as for pospopcnt_ex (depth sets loads per lane). */
int ppc_read_ceiling(const void* ptr, uint64_t nbytes, uint64_t* sink, ppc_stream stream,
                     const ppc_launch_config* config);

/* ------------------------------------------------------------------------
 * Histogram of categorical ids, through their one-hot codes.
 *
 * With `bins` categories, category c is bit c of a bins-bit one-hot word, and the
 * positional population count of the one-hot encoded stream is the frequency
 * histogram (Sec. 1, Table 1).  These calls take the ids themselves and count
 * their one-hot codes in registers, so the encoded stream is never written.
 *   ids    device pointer to n unsigned ids of 1 (u8) or 2 (u16) bytes,
 *          little-endian; u16 ids must be 2-byte aligned (PPC_ERR_ALIGN).
 *   bins   1 .. 32 (PPC_ERR_WIDTH otherwise); the codes are 8, 16 or 32 bits, the
 *          narrowest that holds bins categories.
 *   counts device, 8-byte aligned, bins + 1 uint64 entries, added into:
 *          counts[c] += number of ids equal to c (c < bins) and
 *          counts[bins] += number of ids >= bins (ids without a code).
 * Other errors and conventions as for pospopcnt.
 * ---------------------------------------------------------------------- */
int ppc_histogram_u8(const void* ids, uint64_t n, uint32_t bins, uint64_t* counts,
                     ppc_stream stream);
int ppc_histogram_u16(const void* ids, uint64_t n, uint32_t bins, uint64_t* counts,
                      ppc_stream stream);
/* id_bytes 1 or 2; config as for pospopcnt_ex except that depth must be 0 (the
 * circuit spans one tile: 64 u8 or 32 u16 ids per lane).  NULL = defaults. */
int ppc_histogram_ex(const void* ids, uint64_t n, int id_bytes, uint32_t bins, uint64_t* counts,
                     ppc_stream stream, const ppc_launch_config* config);

/* ------------------------------------------------------------------------
 * Many streams in one launch.
 *
 * A descriptor names one stream (same conventions as the single-stream calls).
 * Descriptor arrays passed to pospopcnt_batch live in device memory, 8-byte
 * aligned, caller-owned, and must stay valid until the call's work on the
 * stream has completed.  Streams may have any length (including 0), any start
 * address and mixed widths; several descriptors may share counts (the flush
 * uses atomics).  A descriptor with k not in {8, 16, 32}, reserved != 0, a
 * NULL or misaligned pointer while n > 0, a length overflowing 64 bits, or
 * counts overlapping its own input is skipped (nothing is added for it) and
 * counted in the plan's rejected count.
 * ---------------------------------------------------------------------- */
typedef struct {
    const void* ptr;   /* device pointer to the first byte of the stream */
    uint64_t n;        /* number of k-bit words */
    uint32_t k;        /* 8, 16 or 32 */
    uint32_t reserved; /* must be 0 */
    uint64_t* counts;  /* device, 8-byte aligned, k entries, added into */
} ppc_desc;

/* Launch configuration of the batched kernel (chosen by ppc_plan_autotune, or
 * set explicitly).  The work of a call is split into equal shares of
 * "weighted units": every stream weighs stream_weight + (its 16-byte body
 * units), the stream_weight standing for the fixed cost of its edge bytes and
 * its flush.  Block b of the grid takes exactly the b-th share. */
typedef struct {
    int32_t depth;          /* circuit inputs per lane per step: 4, 8, 16 or 32 dwords */
    int32_t block_threads;  /* 64, 128 or 256 */
    int32_t blocks_per_cu;  /* 1 .. 16; grid = blocks_per_cu * compute units */
    int32_t stream_weight;  /* weighted units charged per stream, 1 .. 65536 */
} ppc_batch_config;

/* Sizing hints for a plan. */
typedef struct {
    uint32_t max_streams;   /* largest m any call on this plan will pass (>= 1) */
    uint32_t flags;         /* PPC_PLAN_GRAPH: see pospopcnt_batch */
} ppc_workload_hint;

enum { PPC_PLAN_GRAPH = 1 };

typedef struct ppc_plan ppc_plan;

/* Creates a plan on the current device.  The plan owns device scratch for
 * max_streams descriptors (a prefix array of 8 bytes per stream, 12 bytes per
 * 2048 streams for the split preparation, a per-block start table and an
 * autotuning sink of 256 bytes per block of the largest grid, 1 MiB on 256
 * compute units) and a default configuration.  This is the only batched call
 * that allocates.  The environment variable PPC_BATCH_CONFIG
 * ("depth=16,block_threads=64,blocks_per_cu=4,stream_weight=2048", any subset of
 * the keys) overrides the default configuration of every new plan.
 * Errors: PPC_ERR_NULL, PPC_ERR_ARG (max_streams = 0 or > 2^26, or a
 * PPC_BATCH_CONFIG that does not parse or is out of range), PPC_ERR_HIP. */
int ppc_plan_create(const ppc_workload_hint* hint, ppc_plan** plan);

/* Releases the plan's scratch and graphs, after waiting for the plan's device to
 * finish its work (so that work enqueued with the plan completes first; the call
 * synchronises that device).  NULL is accepted. */
int ppc_plan_destroy(ppc_plan* plan);

/* Counts every stream of the m descriptors at d_descs (device memory) with a
 * preparation kernel (two above 4096 streams: one block per 2048 streams) and
 * one persistent counting kernel, asynchronously on stream.  With
 * PPC_PLAN_GRAPH the kernels are captured into a HIP graph on the first
 * call for a given (d_descs, m, configuration) and replayed by later calls; the
 * graph reads the descriptors when it runs, so their contents may change between
 * calls.  Calls sharing a plan must not overlap in time (the plan's scratch is
 * reused); use one plan per concurrent stream.  To record the call into a graph of
 * the caller's own (stream capture), use a plan made without PPC_PLAN_GRAPH: the
 * call then only enqueues kernels, which read the plan's scratch when the graph
 * runs, so the plan must outlive the graph and its replays count as calls on the
 * plan.  m = 0 is a no-op.
 * Errors: PPC_ERR_NULL, PPC_ERR_ALIGN, PPC_ERR_ARG (m > max_streams), PPC_ERR_HIP. */
int pospopcnt_batch(ppc_plan* plan, const ppc_desc* d_descs, uint32_t m, ppc_stream stream);

/* Times candidate configurations on the given workload (counts are redirected
 * to plan scratch, so the descriptors' counters are not touched), keeps the
 * fastest in the plan and returns its time per call in *best_ms (may be NULL).
 * Every candidate (144 shapes: depth 4, 8, 16 or 32, and per depth 28 shapes of
 * one-wave blocks, 1 .. 16 per CU, times four stream weights, and 8 of
 * four-wave blocks) is timed 3 times; the 4 with the lowest medians are then
 * timed 5 times more, in turn, and the lowest median of those decides.  Synchronises
 * `stream`; on an error the plan keeps its previous configuration. */
int ppc_plan_autotune(ppc_plan* plan, const ppc_desc* d_descs, uint32_t m, ppc_stream stream,
                      float* best_ms);

int ppc_plan_get_config(const ppc_plan* plan, ppc_batch_config* config);
/* Errors: PPC_ERR_ARG for a field out of range. */
int ppc_plan_set_config(ppc_plan* plan, const ppc_batch_config* config);

/* Writes the plan's configuration as a small JSON object (with the device
 * architecture, e.g. "gfx950") to path / reads it back.  ppc_plan_load returns
 * PPC_ERR_STATE if the file was written for another device architecture and
 * PPC_ERR_ARG if it cannot be parsed; the plan is then unchanged. */
int ppc_plan_save(const ppc_plan* plan, const char* path);
int ppc_plan_load(ppc_plan* plan, const char* path);

/* A file of tuned configurations keyed by workload, for reuse across runs: the key
 * is (device architecture, compute units, floor(log2 m), floor(log2 bytes)), where m
 * is the number of streams and bytes their total input size.  The file holds one
 * JSON object per line.
 * ppc_plan_cache_put stores the plan's configuration under the key of (m, bytes),
 * replacing an entry with the same key; the file is rewritten through path.tmp and
 * a rename.  ppc_plan_cache_get sets the plan's configuration from the entry with
 * that key.  Errors: PPC_ERR_NULL, PPC_ERR_ARG (m or bytes 0, a file that cannot be
 * written, or a line that does not parse), and for get PPC_ERR_STATE when there is
 * no entry for the key (a missing file is an empty cache); the plan is then
 * unchanged.  Neither call touches the device. */
int ppc_plan_cache_put(const ppc_plan* plan, const char* path, uint32_t m, uint64_t bytes);
int ppc_plan_cache_get(ppc_plan* plan, const char* path, uint32_t m, uint64_t bytes);

/* Number of descriptors the last completed pospopcnt_batch call on this plan
 * skipped as invalid.  Enqueues a 4-byte copy on stream and waits for it. */
int ppc_plan_rejected(ppc_plan* plan, ppc_stream stream, uint32_t* rejected);

/* For callers that cannot allocate device memory: code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc.  The batched count of
 * pospopcnt_batch without a plan: the same kernels, with their scratch (prefix
 * array, per-block start table, preparation partials) in one file-scope device
 * array of the library, about 530 KiB, which each device holds from the first
 * call on it until the process ends.  Nothing is allocated, by this call or by
 * its kernels.
 *   d_descs  device array of m descriptors, as for pospopcnt_batch; invalid
 *            descriptors are skipped (their number is not reported).
 *   m        0 .. PPC_STATIC_MAX_STREAMS; more returns PPC_ERR_CAPACITY and
 *            launches nothing.
 *   config   launch configuration (as for ppc_plan_set_config), or NULL for the
 *            plan's default; blocks_per_cu x compute units may not exceed 4096
 *            (PPC_ERR_CAPACITY).  No graph, no autotuning.
 * The first call on a device looks the array's address up (a runtime query, no
 * allocation); make that call outside stream capture if the capture mode
 * forbids such queries.  Every call on a device shares that device's array:
 * calls on one device must not overlap in time (enqueue them on one stream, or
 * order the streams); overlapping calls race and give wrong counts.
 * Errors: PPC_ERR_NULL, PPC_ERR_ALIGN, PPC_ERR_CAPACITY, PPC_ERR_ARG (config),
 * PPC_ERR_HIP. */
#define PPC_STATIC_MAX_STREAMS 65536
int pospopcnt_batch_static(const ppc_desc* d_descs, uint32_t m, const ppc_batch_config* config,
                           ppc_stream stream);

/* One single-stream launch per descriptor, from a HOST array of m descriptors
 * (each launch as pospopcnt with default configuration).  The per-launch form
 * the batched kernel is measured against; also handy when descriptors are
 * built on the host.  Validation is per descriptor, before any launch: the
 * first invalid descriptor's status is returned and nothing is launched; as in
 * the batched form, k must be 8, 16 or 32 (PPC_ERR_WIDTH for 64). */
int pospopcnt_each(const ppc_desc* h_descs, uint32_t m, ppc_stream stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * Requests name a stream already in device memory (src, n, k).  The server
 * admits them in arrival order while its memory budget and request slots allow:
 * an admitted request gets a slab of its input size in the server's device
 * arena and joins the next launch.  Unless PPC_SERVE_IN_PLACE, its bytes are
 * copied into the slab by the count itself (each input byte is read once and
 * stored once); the copy starts (src mod 16) bytes into the slab, which is sized
 * for that.  Each progress step reaps finished launches (their slabs and
 * slots free up), admits waiting requests and launches every newly admitted one
 * as one batched count on the next of the server's HIP streams, so launches
 * overlap on the device while earlier ones still run.  Counts come back to the
 * host with the launch and are reported per request with its timestamps.  The
 * counting is the batched kernel's, so a request's counts are the same alone and
 * in any mix.  A server is used from one host thread at a time.
 * ---------------------------------------------------------------------- */
typedef struct {
    uint64_t arena_bytes;   /* device memory budget for admitted requests' inputs */
    uint32_t max_requests;  /* requests admitted at once (1 .. 2^20) */
    uint32_t max_batch;     /* requests per launch (1 .. 65536) */
    uint32_t streams;       /* HIP streams launches rotate over (1 .. 8) */
    uint32_t flags;         /* PPC_SERVE_IN_PLACE, PPC_SERVE_FIFO_BYPASS */
} ppc_server_config;

enum {
    /* count at the request's own src (its slab is reserved for accounting only) */
    PPC_SERVE_IN_PLACE = 1,
    /* when the oldest waiting request does not fit, later ones that fit may pass it */
    PPC_SERVE_FIFO_BYPASS = 2
};

typedef struct {
    const void* src;    /* device pointer of the request's input, any alignment */
    uint64_t n;         /* words */
    uint32_t k;         /* 8, 16 or 32 */
    uint32_t reserved;  /* must be 0 */
    double arrival;     /* arrival time in seconds (server clock for ppc_server_submit,
                           offset from the start of the replay for ppc_server_run_trace) */
    uint64_t tag;       /* caller's identifier, returned with the completion */
    double timeout;     /* seconds after arrival by which the request must be admitted;
                           a request still waiting then completes with PPC_ERR_TIMEOUT
                           and is never counted.  0 = no limit (negative or NaN:
                           PPC_ERR_ARG) */
} ppc_request;

typedef struct {
    uint64_t tag;
    int32_t status;     /* PPC_OK, PPC_ERR_BUDGET (larger than the arena), PPC_ERR_WIDTH,
                           PPC_ERR_NULL, PPC_ERR_ARG, PPC_ERR_OVERLAP (the input lies in
                           the server's arena), PPC_ERR_TIMEOUT, PPC_ERR_CANCELLED, or
                           PPC_ERR_HIP if its launch failed */
    uint32_t batch;     /* requests in the launch that counted it */
    double arrival, admitted, launched, completed;  /* server clock, seconds */
    uint64_t counts[32];                            /* first k entries used */
    uint64_t arena_offset; /* where the request's bytes were in the arena (copy mode: the
                              copy's first byte; in place: the reserved slab), UINT64_MAX
                              if it was never launched.  The slab is free again once the
                              completion is reported. */
} ppc_completion;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, launches;
    uint64_t queued_now, inflight_now, max_queued, max_inflight;
    uint64_t arena_used_now, arena_peak, bytes_counted;
    uint64_t expired, cancelled; /* completed with PPC_ERR_TIMEOUT / PPC_ERR_CANCELLED */
} ppc_server_stats;

/* Executor callbacks, for driving the scheduler with something other than the
 * GPU (tests use the CPU oracle).  launch receives the admitted requests of one
 * launch, each with the offset of its slab in a virtual arena; poll reports
 * whether a launch has finished; results fills n x 32 counts in launch order;
 * release forgets the launch.  Every callback returns a status (PPC_OK or an
 * error, which fails the requests of that launch with that status). */
typedef struct {
    const void* src;
    uint64_t n;
    uint32_t k;
    uint32_t reserved;
    uint64_t arena_offset;
    uint64_t tag;
} ppc_exec_item;

typedef struct {
    int (*launch)(void* user, const ppc_exec_item* items, uint32_t n, uint64_t* handle);
    int (*poll)(void* user, uint64_t handle, int* done);
    int (*results)(void* user, uint64_t handle, uint64_t* counts);
    int (*release)(void* user, uint64_t handle);
} ppc_executor_ops;

typedef struct ppc_server ppc_server;

/* Creates a server on the current device: allocates the arena, the streams, one
 * plan per stream and pinned staging for launches (the only serving call that
 * allocates).  Errors: PPC_ERR_NULL, PPC_ERR_ARG, PPC_ERR_HIP.
 * Fault injection for tests: with the environment variable PPC_FAULT_LAUNCH=N
 * set when the server is created, its N-th launch (counted from 1) fails with
 * PPC_ERR_HIP after its count was enqueued, as a failure to enqueue the
 * collection of its results would; the launch's requests complete with that
 * status and the server goes on serving. */
int ppc_server_create(const ppc_server_config* config, ppc_server** server);

/* Same scheduler over caller-supplied executor callbacks (no device memory is
 * allocated; arena offsets are virtual).  ops and user must outlive the server. */
int ppc_server_create_with_executor(const ppc_server_config* config,
                                    const ppc_executor_ops* ops, void* user,
                                    ppc_server** server);

/* Waits for launches in flight, then releases everything.  NULL is accepted. */
int ppc_server_destroy(ppc_server* server);

/* Seconds since the server was created (steady clock). */
double ppc_server_now(const ppc_server* server);

/* Queues n requests (their arrival times are taken as given).  Requests that can
 * never be served complete at once with an error status (larger than the arena:
 * PPC_ERR_BUDGET).  Never blocks and never launches. */
int ppc_server_submit(ppc_server* server, const ppc_request* requests, uint32_t n);

/* One scheduling step: reap finished launches, admit, launch.  Optional outputs:
 * requests launched and completed in this step. */
int ppc_server_progress(ppc_server* server, uint32_t* launched, uint32_t* completed);

/* Moves up to cap completions (oldest first) to out; *n_out receives how many. */
int ppc_server_take_completions(ppc_server* server, ppc_completion* out, uint32_t cap,
                                uint32_t* n_out);

int ppc_server_get_stats(const ppc_server* server, ppc_server_stats* stats);

/* Cancels every request with this tag that is waiting or admitted but not yet
 * launched: each completes with PPC_ERR_CANCELLED (an admitted one gives its
 * slab back).  A launched request is not stopped; it completes as usual.
 * *cancelled (optional) receives how many were cancelled. */
int ppc_server_cancel(ppc_server* server, uint64_t tag, uint32_t* cancelled);

/* The server's device arena: *base its device address (NULL in place, where no
 * arena memory is allocated, and for callback executors) and *bytes its size.
 * Completions give each request's offset in it. */
int ppc_server_arena(const ppc_server* server, void** base, uint64_t* bytes);

/* Replays n requests in real time: request i is submitted when
 * (now - start) >= requests[i].arrival (arrivals must be non-decreasing), and
 * the server is progressed continuously until all n have completed.  out[i]
 * receives request i's completion (out holds n entries); arrival times in out are
 * on the server clock.  Returns PPC_OK when every request has completed, whatever
 * their individual statuses.  The server must be idle at the call: no request
 * queued or in flight and no completion left to take (else PPC_ERR_STATE, and
 * nothing is submitted).  PPC_ERR_STATE also when nothing has progressed for
 * 120 s (a launch that never finished); the requests still held stay in the server. */
int ppc_server_run_trace(ppc_server* server, const ppc_request* requests, uint32_t n,
                         ppc_completion* out);

/* Device facts used to size launches (for the current HIP device). */
typedef struct {
    int32_t device;
    int32_t compute_units;
    int32_t clock_khz;
    int32_t l2_bytes;
    int64_t global_mem_bytes;
    char name[64];
    char arch[64];
} ppc_device_info;

int ppc_get_device_info(ppc_device_info* info);

#ifdef __cplusplus
}
#endif

#endif /* POSPOPCNT_H */
