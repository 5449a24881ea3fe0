// ppc_serve.hip -- request loop with continuous batching over the batched count.
//
// Scheduler (host): requests wait in arrival order; a request is admitted when a
// request slot is free and a slab of its input size fits in the device arena
// (first fit, 256-byte granules).  Every progress step
//   1. reaps finished launches: their completions are recorded with the counts
//      and timestamps, their slabs and slots are released;
//   2. admits waiting requests while slots and memory allow;
//   3. launches the admitted requests not yet launched as one batch, if the
//      executor has a launch slot free.
// So requests that arrive while earlier launches run join the next launch, and
// launches on different streams overlap on the device.
//
// GPU executor: a launch on stream s (launch slots rotate over the streams, two
// per stream) enqueues, in order: one host-to-device copy of the descriptor table
// (and, in copy mode, of where each request's copy goes), unless the launch is
// small enough for its kernel to read them from pinned host memory; the batched
// count, which in copy mode also stores every byte it reads into the request's
// slab, so that each input byte is read once and written once; a small kernel that
// moves the counts to pinned host memory and clears them for the slot's next
// launch; and an event the scheduler polls.
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "ppc_device.h"
#include "ppc_internal.h"

namespace ppc {

constexpr uint64_t kGranule = 256;
constexpr uint32_t kMaxServerRequests = 1u << 20;
constexpr uint32_t kMaxServerBatch = 65536;
constexpr double kStallSeconds = 120.0;  // run_trace gives up after this long without progress

// ------------------------------------------------------------------ arena

class Arena {
  public:
    explicit Arena(uint64_t size) : size_(size) {
        if (size_) free_[0] = size_;
    }
    static uint64_t granules(uint64_t bytes) {
        return ((bytes ? bytes : 1) + kGranule - 1) & ~(kGranule - 1);
    }
    bool alloc(uint64_t bytes, uint64_t* off) {
        const uint64_t need = granules(bytes);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < need) continue;
            *off = it->first;
            const uint64_t rest = it->second - need, noff = it->first + need;
            free_.erase(it);
            if (rest) free_[noff] = rest;
            used_ += need;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        uint64_t need = granules(bytes), start = off;
        used_ -= need;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + need) {
            need += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                need += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = need;
    }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t size() const { return size_; }

  private:
    uint64_t size_, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> length of free runs
};

// ------------------------------------------------------------------ executors

// In copy mode a request's copy starts at its source's address modulo 16 inside
// its slab: the slab holds copy_shift(src) + bytes.
__host__ __device__ inline uint64_t copy_shift(const void* src) { return (uintptr_t)src & 15u; }

struct Admitted {
    ppc_request r;
    uint64_t bytes;  // input bytes
    uint64_t slab;   // bytes reserved in the arena (input plus the copy's shift)
    uint64_t off;    // slab offset in the arena
    double admitted;
};

class Executor {
  public:
    virtual ~Executor() = default;
    virtual int launch(const std::vector<Admitted>& items, uint64_t* handle) = 0;
    virtual int poll(uint64_t handle, bool* done) = 0;
    virtual int results(uint64_t handle, uint64_t* counts) = 0;
    virtual int release(uint64_t handle) = 0;
    virtual size_t capacity() const = 0;  // launches in flight at most
    virtual void wait_all() {}
};

class CallbackExecutor : public Executor {
  public:
    CallbackExecutor(const ppc_executor_ops& ops, void* user, size_t cap)
        : ops_(ops), user_(user), cap_(cap) {}
    int launch(const std::vector<Admitted>& items, uint64_t* handle) override {
        std::vector<ppc_exec_item> v(items.size());
        for (size_t i = 0; i < items.size(); ++i)
            v[i] = {items[i].r.src, items[i].r.n, items[i].r.k, 0, items[i].off, items[i].r.tag};
        return ops_.launch(user_, v.data(), (uint32_t)v.size(), handle);
    }
    int poll(uint64_t h, bool* done) override {
        int d = 0;
        const int st = ops_.poll(user_, h, &d);
        *done = d != 0;
        return st;
    }
    int results(uint64_t h, uint64_t* counts) override { return ops_.results(user_, h, counts); }
    int release(uint64_t h) override { return ops_.release(user_, h); }
    size_t capacity() const override { return cap_; }

  private:
    ppc_executor_ops ops_;
    void* user_;
    size_t cap_;
};

// After a launch's count: its rows of counters go to the pinned results buffer, and the
// counters are cleared for the slot's next launch.  One small kernel in place of a copy
// and a fill: one launch call instead of two on the host.  It runs after the count
// kernel on the same stream, so every flush of the count is visible to it.
__global__ void __launch_bounds__(256) collect_counts(unsigned long long* __restrict__ dev,
                                                      unsigned long long* __restrict__ host,
                                                      uint32_t words) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += gridDim.x * blockDim.x) {
        host[i] = dev[i];
        dev[i] = 0;
    }
}

class HipExecutor : public Executor {
  public:
    // One launch's buffers.  The descriptors and, in copy mode, the destination of
    // each request's copy share one staging area (and one device area), so that a
    // single host-to-device copy carries both.
    struct Slot {
        int stream = 0;
        bool busy = false;
        uint32_t n = 0;
        char* d_meta = nullptr;  // [descs: n][destinations: n], each part 256-byte aligned
        uint64_t* d_counts = nullptr;
        char* h_meta = nullptr;
        uint64_t* h_counts = nullptr;
        hipEvent_t done = nullptr;
        ppc_desc* h_descs() { return (ppc_desc*)h_meta; }
        ppc_desc* d_descs() { return (ppc_desc*)d_meta; }
    };

    int init(const ppc_server_config& c) {
        cfg_ = c;
        const DeviceFacts* dev = nullptr;
        int st = current_device(&dev);
        if (st) return st;
        device_ = dev->device;
        cus_ = dev->cus;
        in_place_ = (c.flags & PPC_SERVE_IN_PLACE) != 0;
        // Test hook: PPC_FAULT_LAUNCH=N makes the N-th launch (counted from 1) fail
        // after its count was enqueued, as if the collection of its results had failed.
        if (const char* f = getenv("PPC_FAULT_LAUNCH")) fault_launch_ = strtoull(f, nullptr, 10);
        if (!in_place_ && c.arena_bytes) PPC_HIP(hipMalloc(&arena_, c.arena_bytes));
        streams_.resize(c.streams, nullptr);
        plans_.resize(c.streams, nullptr);
        for (uint32_t i = 0; i < c.streams; ++i) {
            PPC_HIP(hipStreamCreateWithFlags(&streams_[i], hipStreamNonBlocking));
            ppc_workload_hint hint{c.max_batch, 0};
            st = ppc_plan_create(&hint, &plans_[i]);
            if (st) return st;
            // Four-wave blocks, one per compute unit: a request split over the grid
            // then flushes from a quarter as many blocks (the waves of a block sum
            // in LDS first), and the flush atomics on its counters queue less.
            const ppc_batch_config serve_cfg{16, 256, 1, 4096};
            st = ppc_plan_set_config(plans_[i], &serve_cfg);
            if (st) return st;
        }
        slots_.resize((size_t)c.streams * 2);
        const size_t meta = dst_offset(c.max_batch) + (in_place_ ? 0 : 8ull * c.max_batch);
        for (size_t i = 0; i < slots_.size(); ++i) {
            Slot& s = slots_[i];
            s.stream = (int)(i % c.streams);
            PPC_HIP(hipMalloc(&s.d_meta, meta));
            PPC_HIP(hipMalloc(&s.d_counts, 256ull * c.max_batch));
            // counters start at zero; each launch clears the ones it used after its
            // results have been copied back (see launch)
            PPC_HIP(hipMemset(s.d_counts, 0, 256ull * c.max_batch));
            // Small launches are read by the counting kernel straight from this pinned
            // buffer (see launch), which the host rewrites before every launch of the
            // slot: fine-grained (coherent) memory, so that the device never holds a
            // stale copy of it.
            PPC_HIP(hipHostMalloc(&s.h_meta, meta, hipHostMallocCoherent));
            // written by collect_counts: fine-grained, so that the host sees the kernel's
            // stores once the launch's event has completed
            PPC_HIP(hipHostMalloc(&s.h_counts, 256ull * c.max_batch, hipHostMallocCoherent));
            PPC_HIP(hipEventCreateWithFlags(&s.done, hipEventDisableTiming));
        }
        return PPC_OK;
    }

    ~HipExecutor() override {
        wait_all();
        for (Slot& s : slots_) {
            if (s.done) (void)hipEventDestroy(s.done);
            if (s.d_meta) (void)hipFree(s.d_meta);
            if (s.d_counts) (void)hipFree(s.d_counts);
            if (s.h_meta) (void)hipHostFree(s.h_meta);
            if (s.h_counts) (void)hipHostFree(s.h_counts);
        }
        for (ppc_plan* p : plans_) ppc_plan_destroy(p);
        for (hipStream_t s : streams_)
            if (s) (void)hipStreamDestroy(s);
        if (arena_) (void)hipFree(arena_);
    }

    void wait_all() override {
        for (hipStream_t s : streams_)
            if (s) (void)hipStreamSynchronize(s);
    }

    size_t capacity() const override { return slots_.size(); }

    void* arena() const { return arena_; }

    int launch(const std::vector<Admitted>& items, uint64_t* handle) override {
        size_t si = slots_.size();
        for (size_t j = 0; j < slots_.size(); ++j) {
            const size_t i = (next_ + j) % slots_.size();
            if (!slots_[i].busy) {
                si = i;
                break;
            }
        }
        if (si == slots_.size()) return PPC_ERR_STATE;
        next_ = (si + 1) % slots_.size();
        Slot& s = slots_[si];
        const uint32_t n = (uint32_t)items.size();
        hipStream_t st = streams_[s.stream];
        // The destinations follow this batch's own descriptors, so that the one
        // host-to-device copy stays small (large ones go through a DMA engine, whose
        // hand-over to the compute queue costs tens of microseconds).  A request's
        // copy starts at its source's address modulo 16 inside its slab (the
        // scheduler sized the slab for that), so the count stores each aligned
        // 16-byte unit it reads to one aligned unit of the slab.
        const size_t dst_off = dst_offset(n);
        uint8_t** h_dsts = (uint8_t**)(s.h_meta + dst_off);
        uint64_t bytes = 0;
        for (uint32_t i = 0; i < n; ++i) {
            const Admitted& a = items[i];
            if (!in_place_) h_dsts[i] = (uint8_t*)arena_ + a.off + copy_shift(a.r.src);
            s.h_descs()[i] = {a.r.src, a.r.n, a.r.k, 0, s.d_counts + 32ull * i};
            bytes += a.bytes;
        }
        // One copy of the descriptors (and the destinations right after them), except
        // for launches small enough for the counting kernel to read them from the
        // pinned buffer itself, every block once (kDirectReads descriptors in all at
        // most): that saves the copy and the queue's gap after it.
        const bool direct = n <= kSmallBatch &&
                            (uint64_t)small_batch_grid(plans_[s.stream], n, bytes) * n <=
                                kDirectReads;
        // A failure once work is queued: wait for that work, so that no kernel still
        // writes into the slabs the scheduler frees when it fails these requests, and
        // clear the counters it may have added to, which the slot's next launch
        // expects at zero.
        auto abandon = [&](int status) {
            (void)hipStreamSynchronize(st);
            (void)hipMemsetAsync(s.d_counts, 0, 256ull * n, st);
            (void)hipStreamSynchronize(st);
            return status;
        };
#define PPC_HIP_QUEUED(call)                                       \
    do {                                                           \
        const hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) return abandon(::ppc::fail_hip(e_)); \
    } while (0)
        if (!direct) {
            const size_t meta = in_place_ ? sizeof(ppc_desc) * n : dst_off + 8ull * n;
            PPC_HIP_QUEUED(hipMemcpyAsync(s.d_meta, s.h_meta, meta, hipMemcpyHostToDevice, st));
        }
        char* meta = direct ? s.h_meta : s.d_meta;
        uint8_t* const* dsts = in_place_ ? nullptr : (uint8_t* const*)(meta + dst_off);
        // the slot's counters are zero here (cleared after the slot's previous use)
        const int bst = batch_zeroed(plans_[s.stream], (const ppc_desc*)meta, n, st, bytes, dsts);
        if (bst) return abandon(bst);
        if (++launches_ == fault_launch_) return abandon(fail_hip(hipErrorLaunchFailure));
        // the counts to the pinned buffer, the counters cleared for the slot's next launch
        {
            unsigned long long* dev = (unsigned long long*)s.d_counts;
            unsigned long long* host = (unsigned long long*)s.h_counts;
            uint32_t words = 32u * n;
            const uint32_t grid = std::min<uint32_t>((words + 255) / 256, 64);
            void* cargs[] = {(void*)&dev, (void*)&host, &words};
            PPC_HIP_QUEUED(
                hipLaunchKernel((const void*)collect_counts, dim3(grid), dim3(256), cargs, 0, st));
        }
        PPC_HIP_QUEUED(hipEventRecord(s.done, st));
#undef PPC_HIP_QUEUED
        s.busy = true;
        s.n = n;
        *handle = si;
        return PPC_OK;
    }

    int poll(uint64_t h, bool* done) override {
        const hipError_t e = hipEventQuery(slots_[h].done);
        if (e == hipSuccess) {
            *done = true;
            return PPC_OK;
        }
        *done = false;
        if (e == hipErrorNotReady) return PPC_OK;
        return fail_hip(e);
    }

    int results(uint64_t h, uint64_t* counts) override {
        memcpy(counts, slots_[h].h_counts, 256ull * slots_[h].n);
        return PPC_OK;
    }

    int release(uint64_t h) override {
        slots_[h].busy = false;
        return PPC_OK;
    }

  private:
    static size_t dst_offset(uint32_t n) { return (sizeof(ppc_desc) * n + 255) & ~(size_t)255; }

    ppc_server_config cfg_{};
    int device_ = -1, cus_ = 0;
    bool in_place_ = false;
    void* arena_ = nullptr;
    uint64_t launches_ = 0, fault_launch_ = 0;
    std::vector<hipStream_t> streams_;
    std::vector<ppc_plan*> plans_;
    std::vector<Slot> slots_;
    size_t next_ = 0;
};

static int check_server_config(const ppc_server_config& c) {
    if (c.max_requests < 1 || c.max_requests > kMaxServerRequests) return PPC_ERR_ARG;
    if (c.max_batch < 1 || c.max_batch > kMaxServerBatch) return PPC_ERR_ARG;
    if (c.streams < 1 || c.streams > 8) return PPC_ERR_ARG;
    if (c.flags & ~(uint32_t)(PPC_SERVE_IN_PLACE | PPC_SERVE_FIFO_BYPASS)) return PPC_ERR_ARG;
    return PPC_OK;
}

}  // namespace ppc

using namespace ppc;

struct ppc_server {
    struct Inflight {
        uint64_t handle;
        std::vector<Admitted> items;
        double launched;
    };
    struct Waiting {
        ppc_request r;
        uint64_t bytes, slab;
    };

    ppc_server_config cfg{};
    std::unique_ptr<Executor> exec;
    void* arena_base = nullptr;  // the executor's device arena (NULL in place or virtual)
    Arena arena{0};
    std::deque<Waiting> queue;
    uint64_t queued_with_timeout = 0;  // waiting requests that carry a timeout
    std::vector<Admitted> admitted;    // admitted, not yet launched
    std::vector<Inflight> inflight;
    std::deque<ppc_completion> done;
    uint64_t slots = 0;  // requests admitted and not yet completed
    ppc_server_stats stats{};
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::vector<uint64_t> counts;

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }

    bool copies() const { return (cfg.flags & PPC_SERVE_IN_PLACE) == 0; }

    // A source that overlaps the arena could be overwritten by another request's copy
    // while it is read.
    bool inside_arena(const void* src, uint64_t bytes) const {
        if (!arena_base || !bytes) return false;
        const uintptr_t a0 = (uintptr_t)arena_base, a1 = a0 + arena.size();
        const uintptr_t s0 = (uintptr_t)src, s1 = s0 + bytes;
        return s1 < s0 || (s0 < a1 && a0 < s1);
    }

    // Slab of a request: its bytes, plus in copy mode the shift of its copy.
    uint64_t slab_of(const ppc_request& r, uint64_t bytes) const {
        return bytes + (copies() ? copy_shift(r.src) : 0);
    }

    void complete(const ppc_request& r, int status, uint32_t batch, double admitted_t,
                  double launched_t, const uint64_t* c, uint64_t arena_off = UINT64_MAX) {
        ppc_completion x;
        memset(&x, 0, sizeof(x));
        x.tag = r.tag;
        x.status = status;
        x.batch = batch;
        x.arrival = r.arrival;
        x.admitted = admitted_t;
        x.launched = launched_t;
        x.completed = now();
        if (c && status == PPC_OK) memcpy(x.counts, c, sizeof(uint64_t) * r.k);
        x.arena_offset = arena_off;
        done.push_back(x);
        ++stats.completed;
    }

    // Where the request's bytes sit in the arena: the copy's first byte in copy
    // mode, the reserved slab in place.
    uint64_t copy_offset(const Admitted& a) const {
        return a.off + (copies() ? copy_shift(a.r.src) : 0);
    }

    void finish(Inflight& f, int status) {
        const uint32_t n = (uint32_t)f.items.size();
        if (!status) {
            counts.resize(32ull * n);
            status = exec->results(f.handle, counts.data());
        }
        for (uint32_t i = 0; i < n; ++i) {
            const Admitted& a = f.items[i];
            complete(a.r, status, n, a.admitted, f.launched, status ? nullptr : &counts[32ull * i],
                     copy_offset(a));
            arena.release(a.off, a.slab);
            if (!status) stats.bytes_counted += a.bytes;
        }
        slots -= n;
        exec->release(f.handle);
    }

    uint32_t reap() {
        uint32_t n = 0;
        for (size_t i = 0; i < inflight.size();) {
            bool fin = false;
            const int st = exec->poll(inflight[i].handle, &fin);
            if (st || fin) {
                n += (uint32_t)inflight[i].items.size();
                finish(inflight[i], st);
                inflight.erase(inflight.begin() + (long)i);
            } else {
                ++i;
            }
        }
        return n;
    }

    // Waiting requests whose timeout has passed complete with PPC_ERR_TIMEOUT.
    uint32_t expire() {
        if (!queued_with_timeout) return 0;
        const double t = now();
        uint32_t n = 0;
        for (auto it = queue.begin(); it != queue.end();) {
            const ppc_request& r = it->r;
            if (r.timeout > 0 && t > r.arrival + r.timeout) {
                complete(r, PPC_ERR_TIMEOUT, 0, 0.0, 0.0, nullptr);
                ++stats.expired;
                --queued_with_timeout;
                ++n;
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
        return n;
    }

    void admit() {
        const double t = now();
        const bool bypass = (cfg.flags & PPC_SERVE_FIFO_BYPASS) != 0;
        for (auto it = queue.begin(); it != queue.end() && slots < cfg.max_requests;) {
            uint64_t off = 0;
            if (arena.alloc(it->slab, &off)) {
                admitted.push_back({it->r, it->bytes, it->slab, off, t});
                if (it->r.timeout > 0) --queued_with_timeout;
                ++slots;
                ++stats.admitted;
                it = queue.erase(it);
            } else if (bypass) {
                ++it;
            } else {
                break;
            }
        }
    }

    // Requests with this tag that have not been launched complete with
    // PPC_ERR_CANCELLED (an admitted one gives its slab back).
    uint32_t cancel(uint64_t tag) {
        uint32_t n = 0;
        for (auto it = queue.begin(); it != queue.end();) {
            if (it->r.tag == tag) {
                if (it->r.timeout > 0) --queued_with_timeout;
                complete(it->r, PPC_ERR_CANCELLED, 0, 0.0, 0.0, nullptr);
                ++n;
                it = queue.erase(it);
            } else {
                ++it;
            }
        }
        for (auto it = admitted.begin(); it != admitted.end();) {
            if (it->r.tag == tag) {
                complete(it->r, PPC_ERR_CANCELLED, 0, it->admitted, 0.0, nullptr);
                arena.release(it->off, it->slab);
                --slots;
                ++n;
                it = admitted.erase(it);
            } else {
                ++it;
            }
        }
        stats.cancelled += n;
        return n;
    }

    uint32_t launch() {
        if (admitted.empty() || inflight.size() >= exec->capacity()) return 0;
        const size_t n = std::min<size_t>(admitted.size(), cfg.max_batch);
        Inflight f;
        f.items.assign(admitted.begin(), admitted.begin() + (long)n);
        admitted.erase(admitted.begin(), admitted.begin() + (long)n);
        f.launched = now();
        const int st = exec->launch(f.items, &f.handle);
        ++stats.launches;
        if (st) {
            for (const Admitted& a : f.items) {
                complete(a.r, st, (uint32_t)n, a.admitted, f.launched, nullptr, copy_offset(a));
                arena.release(a.off, a.slab);
            }
            slots -= n;
            return (uint32_t)n;
        }
        inflight.push_back(std::move(f));
        return (uint32_t)n;
    }

    void note() {
        stats.queued_now = queue.size();
        stats.inflight_now = slots;
        stats.max_queued = std::max<uint64_t>(stats.max_queued, queue.size());
        stats.max_inflight = std::max<uint64_t>(stats.max_inflight, slots);
        stats.arena_used_now = arena.used();
        stats.arena_peak = arena.peak();
    }
};

static int server_init(const ppc_server_config* config, ppc_server** out) {
    if (!config || !out) return PPC_ERR_NULL;
    *out = nullptr;
    return check_server_config(*config);
}

extern "C" {

int ppc_server_create(const ppc_server_config* config, ppc_server** out) {
    int st = server_init(config, out);
    if (st) return st;
    auto ex = std::make_unique<HipExecutor>();
    st = ex->init(*config);
    if (st) return st;  // the executor's destructor frees what init allocated
    ppc_server* s = new ppc_server();
    s->cfg = *config;
    s->arena = Arena(config->arena_bytes);
    s->arena_base = ex->arena();
    s->exec = std::move(ex);
    *out = s;
    return PPC_OK;
}

int ppc_server_create_with_executor(const ppc_server_config* config, const ppc_executor_ops* ops,
                                    void* user, ppc_server** out) {
    int st = server_init(config, out);
    if (st) return st;
    if (!ops || !ops->launch || !ops->poll || !ops->results || !ops->release) return PPC_ERR_NULL;
    ppc_server* s = new ppc_server();
    s->cfg = *config;
    s->arena = Arena(config->arena_bytes);
    s->exec = std::make_unique<CallbackExecutor>(*ops, user, (size_t)config->streams * 2);
    *out = s;
    return PPC_OK;
}

int ppc_server_destroy(ppc_server* s) {
    if (!s) return PPC_OK;
    s->exec->wait_all();
    delete s;
    return PPC_OK;
}

double ppc_server_now(const ppc_server* s) { return s ? s->now() : 0.0; }

int ppc_server_submit(ppc_server* s, const ppc_request* reqs, uint32_t n) {
    if (!s) return PPC_ERR_NULL;
    if (n && !reqs) return PPC_ERR_NULL;
    for (uint32_t i = 0; i < n; ++i) {
        const ppc_request& r = reqs[i];
        ++s->stats.submitted;
        int st = PPC_OK;
        uint64_t bytes = 0, slab = 0;
        if (r.k != 8 && r.k != 16 && r.k != 32) st = PPC_ERR_WIDTH;
        else if (r.reserved) st = PPC_ERR_ARG;
        else if (!(r.timeout >= 0.0)) st = PPC_ERR_ARG;  // negative or NaN
        else if (r.n > UINT64_MAX / (r.k / 8)) st = PPC_ERR_ARG;
        else if (r.n && !r.src) st = PPC_ERR_NULL;
        else if (s->inside_arena(r.src, r.n * (r.k / 8))) st = PPC_ERR_OVERLAP;
        else {
            bytes = r.n * (r.k / 8);
            slab = bytes <= s->arena.size() ? s->slab_of(r, bytes) : 0;
            if (bytes > s->arena.size() || Arena::granules(slab) > s->arena.size())
                st = PPC_ERR_BUDGET;
        }
        if (st) {
            ++s->stats.rejected;
            s->complete(r, st, 0, 0.0, 0.0, nullptr);
        } else if (bytes == 0) {
            static const uint64_t zeros[32] = {0};
            s->complete(r, PPC_OK, 0, r.arrival, r.arrival, zeros);
        } else {
            s->queue.push_back({r, bytes, slab});
            if (r.timeout > 0) ++s->queued_with_timeout;
        }
    }
    s->note();
    return PPC_OK;
}

int ppc_server_progress(ppc_server* s, uint32_t* launched, uint32_t* completed) {
    if (!s) return PPC_ERR_NULL;
    const uint32_t c = s->reap() + s->expire();
    s->admit();
    const uint32_t l = s->launch();
    s->note();
    if (launched) *launched = l;
    if (completed) *completed = c;
    return PPC_OK;
}

int ppc_server_take_completions(ppc_server* s, ppc_completion* out, uint32_t cap,
                                uint32_t* n_out) {
    if (!s || !n_out) return PPC_ERR_NULL;
    if (cap && !out) return PPC_ERR_NULL;
    uint32_t n = 0;
    while (n < cap && !s->done.empty()) {
        out[n++] = s->done.front();
        s->done.pop_front();
    }
    *n_out = n;
    return PPC_OK;
}

int ppc_server_get_stats(const ppc_server* s, ppc_server_stats* out) {
    if (!s || !out) return PPC_ERR_NULL;
    *out = s->stats;
    return PPC_OK;
}

int ppc_server_cancel(ppc_server* s, uint64_t tag, uint32_t* cancelled) {
    if (!s) return PPC_ERR_NULL;
    const uint32_t n = s->cancel(tag);
    s->note();
    if (cancelled) *cancelled = n;
    return PPC_OK;
}

int ppc_server_arena(const ppc_server* s, void** base, uint64_t* bytes) {
    if (!s || !base || !bytes) return PPC_ERR_NULL;
    *base = s->arena_base;
    *bytes = s->arena.size();
    return PPC_OK;
}

int ppc_server_run_trace(ppc_server* s, const ppc_request* reqs, uint32_t n, ppc_completion* out) {
    if (!s) return PPC_ERR_NULL;
    if (n && (!reqs || !out)) return PPC_ERR_NULL;
    for (uint32_t i = 1; i < n; ++i)
        if (reqs[i].arrival < reqs[i - 1].arrival) return PPC_ERR_ARG;
    // Requests are submitted with their index as tag; completions are put back in
    // place with the caller's tag.  Completions of requests submitted before would
    // carry other tags, so the server must hold none.
    if (!s->queue.empty() || !s->admitted.empty() || !s->inflight.empty() || !s->done.empty())
        return PPC_ERR_STATE;
    const double start = s->now();
    uint32_t next = 0, finished = 0;
    double last_change = start;
    std::vector<ppc_completion> buf(256);
    while (finished < n) {
        const double t = s->now();
        uint32_t sub = 0;
        while (next < n && reqs[next].arrival <= t - start) {
            ppc_request r = reqs[next];
            r.arrival += start;
            r.tag = next;
            ppc_server_submit(s, &r, 1);
            ++next;
            ++sub;
        }
        uint32_t l = 0, c = 0;
        ppc_server_progress(s, &l, &c);
        uint32_t got = 0;
        ppc_server_take_completions(s, buf.data(), (uint32_t)buf.size(), &got);
        for (uint32_t i = 0; i < got; ++i) {
            const uint64_t idx = buf[i].tag;
            out[idx] = buf[i];
            out[idx].tag = reqs[idx].tag;
        }
        finished += got;
        if (sub || l || c || got) {
            last_change = s->now();
        } else if (s->now() - last_change > kStallSeconds) {
            return PPC_ERR_STATE;  // nothing moved for too long: a launch never finished
        } else if (next < n && s->slots == 0 && s->queue.empty()) {
            // idle until the next arrival: yield instead of spinning hard
            const double wait = reqs[next].arrival - (s->now() - start);
            if (wait > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
    }
    return PPC_OK;
}

}  // extern "C"
