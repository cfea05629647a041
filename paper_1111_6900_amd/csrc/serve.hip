// Serving: a request loop with continuous batching over the persistent
// plane-product kernel.
//
// A scheduler thread owns a HIP stream, a device arena of `memory_budget`
// bytes for resident bit-planes, and `max_inflight` descriptor slots.  Each
// round of its loop
//   1. retires requests whose completion event has fired (frees arena + slot),
//   2. admits waiting requests in arrival order while their plane footprint
//      fits the arena and a slot is free, slicing A and B into planes that stay
//      resident on the device until the request completes.  When the oldest
//      waiting request does not fit, later ones that do may be admitted ahead
//      of it, at most `bypass_limit` times per oldest request, so that a large
//      request delays small ones only boundedly and is never starved,
//   3. issues one iteration: up to `quantum_macs` of plane-product tiles taken
//      from the admitted requests oldest first, as one persistent launch per
//      tile class; a request whose last tiles are in the iteration gets its
//      combine launch and completion event right behind it.
// Requests that arrive while others run join the next iteration, so their
// work shares launches with the requests already on the GPU.  The arithmetic
// is the same as gf2e_mul's, so every result is identical to the product
// computed alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "ctx.hpp"

namespace gf2e {

namespace {

using Clock = std::chrono::steady_clock;

// Tile classes: {large, small} x {fp4 (k <= 2^23), int8}.
constexpr int kNumClasses = 4;
constexpr int kClassKinds[kNumClasses] = {GEMM_FP4_256x256_W8, GEMM_FP4_128x128, GEMM_MFMA_256x256_W8,
                                          GEMM_MFMA_128x128};
constexpr int kIterBuffers = 3;  // iterations that may be in flight at once

int64_t footprint_of(const Plan& p)
{
    auto a = [](int64_t x) { return (x + 255) / 256 * 256; };
    return a(p.a_bytes) + a(p.b_bytes) + a(p.p_bytes);
}

// First-fit allocator over [0, size) with 256-byte granules.
class Arena {
public:
    explicit Arena(int64_t size) { free_[0] = size; }
    int64_t alloc(int64_t bytes)
    {
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= bytes) {
                const int64_t off = it->first, len = it->second;
                free_.erase(it);
                if (len > bytes) free_[off + bytes] = len - bytes;
                return off;
            }
        return -1;
    }
    void release(int64_t off, int64_t bytes)
    {
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }

private:
    std::map<int64_t, int64_t> free_;  // offset -> length
};

enum ReqState { PENDING = 0, ADMITTED = 1, ISSUED = 2, DONE = 3 };

struct Request {
    uint64_t ticket = 0;
    BatchProduct d{};
    Plan plan{};
    int64_t footprint = 0, arena_off = -1;
    int slot = -1, cls = 0, tm = 0, tn = 0;
    int group = 1;  // planes per work item
    int64_t total_items = 0, next_item = 0;
    std::atomic<int> state{PENDING};
    int status = GF2E_OK;
    int overtaken = 0;        // admissions of later requests while this one was the oldest waiting
    bool waited_mem = false;  // found the arena full at least once
    hipEvent_t ready_ev = nullptr;  // recorded on the submitter's stream: inputs are written
    hipEvent_t done_ev = nullptr;
    int64_t t_submit = 0, t_admit = 0, t_done = 0;
};

}  // namespace

struct Server {
    Ctx* ctx = nullptr;
    gf2e_server_config cfg{};
    hipStream_t stream = nullptr;
    uint8_t* arena_base = nullptr;
    Arena* arena = nullptr;
    BatchProduct* d_slots = nullptr;  // device descriptor table, one per slot
    BatchProduct* h_slots = nullptr;  // pinned staging for it
    int* d_err = nullptr;             // per-slot range-error flags
    int* h_err = nullptr;             // pinned copies read at completion
    std::vector<int> free_slots;
    WorkItem* d_items[kIterBuffers] = {};
    WorkItem* h_items[kIterBuffers] = {};
    int* d_counters = nullptr;        // kNumClasses per iteration buffer
    hipEvent_t iter_ev[kIterBuffers] = {};
    bool iter_busy[kIterBuffers] = {};
    int grid[kNumClasses] = {};
    int64_t max_items = 0;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request*> incoming;    // submitted, not yet seen by the scheduler
    std::map<uint64_t, Request*> all; // every live request by ticket
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    Clock::time_point t0;

    // scheduler-thread state
    std::deque<Request*> pending, admitted;
    std::vector<Request*> issued;

    // statistics
    std::atomic<int64_t> completed{0}, iterations{0}, element_macs{0};
    std::atomic<int64_t> arena_used{0}, peak_arena{0};
    std::atomic<int> inflight{0}, peak_inflight{0};
    std::atomic<int64_t> memory_waits{0}, bypass_admissions{0}, shared_iterations{0};
    std::atomic<int> max_iteration_requests{0};

    int64_t now_ns() const
    {
        return std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count();
    }
    void run();
    bool retire();
    bool admit();
    void start(Request* r, int64_t off);
    bool issue_iteration();
};

bool Server::retire()
{
    bool any = false;
    for (size_t i = 0; i < issued.size();) {
        Request* r = issued[i];
        const hipError_t q = hipEventQuery(r->done_ev);
        if (q == hipErrorNotReady) { ++i; continue; }
        r->status = q != hipSuccess ? GF2E_EDEVICE : (h_err[r->slot] ? GF2E_ERANGE : GF2E_OK);
        arena->release(r->arena_off, r->footprint);
        arena_used -= r->footprint;
        free_slots.push_back(r->slot);
        completed += 1;
        element_macs += r->d.m * r->d.k * r->d.n;
        inflight -= 1;
        {
            std::lock_guard<std::mutex> lk(mu);
            r->t_done = now_ns();
            r->state = DONE;
        }
        cv_done.notify_all();
        issued[i] = issued.back();
        issued.pop_back();
        any = true;
    }
    return any;
}

// Scan depth past the oldest waiting request when it does not fit.
constexpr size_t kBypassWindow = 64;

bool Server::admit()
{
    bool any = false;
    while (!pending.empty() && !free_slots.empty() &&
           (cfg.max_inflight <= 0 || inflight < cfg.max_inflight)) {
        Request* head = pending.front();
        int64_t off = arena->alloc(head->footprint);
        if (off >= 0) {
            pending.pop_front();
            start(head, off);
            any = true;
            continue;
        }
        if (!head->waited_mem) {
            head->waited_mem = true;
            memory_waits += 1;
        }
        if (head->overtaken >= cfg.bypass_limit) break;  // arrival order from here on
        // The oldest request waits for memory: admit the first later one that fits.
        size_t pick = 0;
        const size_t end = std::min(pending.size(), kBypassWindow + 1);
        for (size_t i = 1; i < end && pick == 0; ++i) {
            off = arena->alloc(pending[i]->footprint);
            if (off >= 0) {
                pick = i;
            } else if (!pending[i]->waited_mem) {
                pending[i]->waited_mem = true;
                memory_waits += 1;
            }
        }
        if (pick == 0) break;
        Request* r = pending[pick];
        pending.erase(pending.begin() + std::ptrdiff_t(pick));
        head->overtaken += 1;
        bypass_admissions += 1;
        start(r, off);
        any = true;
    }
    return any;
}

// Admits r into the arena range at `off`: slot, descriptor and slicing of its
// inputs, after the submitter's stream has written them.
void Server::start(Request* r, int64_t off)
{
    r->arena_off = off;
    r->slot = free_slots.back();
    free_slots.pop_back();
    arena_used += r->footprint;
    peak_arena = std::max<int64_t>(peak_arena, arena_used);
    inflight += 1;
    peak_inflight = std::max<int>(peak_inflight, inflight);
    uint8_t* base = arena_base + off;
    auto a256 = [](int64_t x) { return (x + 255) / 256 * 256; };
    r->d.Apl = reinterpret_cast<uint64_t*>(base);
    r->d.Bpl = reinterpret_cast<uint64_t*>(base + a256(r->plan.a_bytes));
    r->d.P = reinterpret_cast<uint64_t*>(base + a256(r->plan.a_bytes) + a256(r->plan.b_bytes));
    h_slots[r->slot] = r->d;
    (void)hipStreamWaitEvent(stream, r->ready_ev, 0);
    (void)hipMemcpyAsync(d_slots + r->slot, h_slots + r->slot, sizeof(BatchProduct), hipMemcpyHostToDevice,
                         stream);
    int* err = d_err + r->slot;
    if (r->d.k > 0) {
        (void)launch_slice_rows(r->d.e, r->d.sid, r->d.A, r->d.lda, r->d.m, r->d.k, r->d.Apl, r->d.Mp,
                                r->d.K64p, err, stream);
        (void)launch_slice_cols(r->d.e, r->d.sid, r->d.B, r->d.ldb, r->d.k, r->d.n, r->d.Bpl, r->d.Np,
                                r->d.K64p, err, stream);
    }
    r->t_admit = now_ns();
    r->state = ADMITTED;
    admitted.push_back(r);
}

bool Server::issue_iteration()
{
    if (admitted.empty()) return false;
    int buf = -1;
    for (int b = 0; b < kIterBuffers; ++b) {
        if (iter_busy[b] && hipEventQuery(iter_ev[b]) != hipErrorNotReady) iter_busy[b] = false;
        if (!iter_busy[b] && buf < 0) buf = b;
    }
    if (buf < 0) return false;

    // Take tiles oldest request first until the quantum is used.
    std::vector<WorkItem> cls_items[kNumClasses];
    std::vector<Request*> finishing;
    int64_t budget = cfg.quantum_macs > 0 ? cfg.quantum_macs : INT64_MAX;
    int64_t room = max_items;
    int contributors = 0;
    for (Request* r : admitted) {
        if (budget <= 0 || room <= 0) break;
        if (r->next_item < r->total_items) contributors += 1;
        const GemmShape sh = gemm_shape(kClassKinds[r->cls]);
        const int64_t plane_macs = int64_t(sh.bm) * sh.bn * r->d.K64p * 64;
        while (r->next_item < r->total_items && budget > 0 && room > 0) {
            const int64_t it = r->next_item++;
            const int64_t per_group = int64_t(r->tm) * r->tn;
            const int s = int(it / per_group) * r->group, rem = int(it % per_group);
            const int np = std::min(r->group, r->d.T - s);
            cls_items[r->cls].push_back({int32_t(r->slot), s, rem / r->tn, rem % r->tn, np});
            budget -= plane_macs * np;
            room -= 1;
        }
        if (r->next_item == r->total_items) finishing.push_back(r);
    }
    size_t total = 0, off[kNumClasses] = {};
    for (int c = 0; c < kNumClasses; ++c) {
        off[c] = total;
        total += cls_items[c].size();
    }
    if (total > 0) {
        for (int c = 0; c < kNumClasses; ++c)
            std::memcpy(h_items[buf] + off[c], cls_items[c].data(), cls_items[c].size() * sizeof(WorkItem));
        (void)hipMemcpyAsync(d_items[buf], h_items[buf], total * sizeof(WorkItem), hipMemcpyHostToDevice,
                             stream);
        int* ctr = d_counters + kNumClasses * buf;
        (void)launch_reset_counters(ctr, kNumClasses, stream);
        for (int c = 0; c < kNumClasses; ++c)
            if (!cls_items[c].empty())
                (void)launch_persistent_gemm(kClassKinds[c], d_slots, d_items[buf] + off[c],
                                             int(cls_items[c].size()), ctr + c, grid[c], stream);
    }
    for (Request* r : finishing) {
        if (r->d.k == 0)
            (void)launch_zero(r->d.C, r->d.m, r->d.n, r->d.ldc, elem_bytes(r->d.e), stream);
        else
            (void)launch_combine(r->d.e, r->d.sid, r->d.f, r->d.P, r->d.Mp * (r->d.Np / 64), r->d.Np / 64, r->d.m, r->d.n, r->d.C,
                                 r->d.ldc, stream);
        (void)hipMemcpyAsync(h_err + r->slot, d_err + r->slot, sizeof(int), hipMemcpyDeviceToHost, stream);
        (void)launch_reset_counters(d_err + r->slot, 1, stream);
        (void)hipEventRecord(r->done_ev, stream);
        r->state = ISSUED;
        issued.push_back(r);
        admitted.erase(std::find(admitted.begin(), admitted.end(), r));
    }
    (void)hipEventRecord(iter_ev[buf], stream);
    iter_busy[buf] = true;
    iterations += 1;
    if (contributors >= 2) shared_iterations += 1;
    max_iteration_requests = std::max<int>(max_iteration_requests, contributors);
    return true;
}

void Server::run()
{
    (void)hipSetDevice(ctx->device);
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(mu);
            if (pending.empty() && admitted.empty() && issued.empty() && incoming.empty()) {
                if (stop) break;
                cv_work.wait(lk, [&] { return stop || !incoming.empty(); });
                if (stop && incoming.empty()) break;
            }
            while (!incoming.empty()) {
                pending.push_back(incoming.front());
                incoming.pop_front();
            }
        }
        bool progress = retire();
        progress |= admit();
        progress |= issue_iteration();
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

}  // namespace gf2e

using namespace gf2e;

extern "C" {

int gf2e_server_create(gf2e_ctx* handle, const gf2e_server_config* cfg, gf2e_server** out)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !out || !cfg || cfg->memory_budget <= 0 || cfg->max_inflight <= 0 ||
        cfg->max_inflight > 4096 || cfg->bypass_limit < 0)
        return GF2E_EINVAL;
    *out = nullptr;
    DeviceGuard guard(c->device);
    auto s = std::make_unique<Server>();
    s->ctx = c;
    s->cfg = *cfg;
    s->max_items = cfg->max_items_per_iteration > 0 ? cfg->max_items_per_iteration : 1 << 18;
    const int slots = cfg->max_inflight;
    bool ok = hipStreamCreateWithFlags(&s->stream, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(reinterpret_cast<void**>(&s->arena_base), size_t(cfg->memory_budget)) == hipSuccess &&
              hipMalloc(&s->d_slots, sizeof(BatchProduct) * slots) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&s->h_slots), sizeof(BatchProduct) * slots, 0) == hipSuccess &&
              hipMalloc(&s->d_err, sizeof(int) * slots) == hipSuccess &&
              hipMemset(s->d_err, 0, sizeof(int) * slots) == hipSuccess &&
              hipHostMalloc(reinterpret_cast<void**>(&s->h_err), sizeof(int) * slots, 0) == hipSuccess &&
              hipMalloc(&s->d_counters, sizeof(int) * kNumClasses * kIterBuffers) == hipSuccess;
    for (int b = 0; ok && b < kIterBuffers; ++b)
        ok = hipMalloc(&s->d_items[b], sizeof(WorkItem) * s->max_items) == hipSuccess &&
             hipHostMalloc(reinterpret_cast<void**>(&s->h_items[b]), sizeof(WorkItem) * s->max_items, 0) ==
                 hipSuccess &&
             hipEventCreateWithFlags(&s->iter_ev[b], hipEventDisableTiming) == hipSuccess;
    for (int c = 0; ok && c < kNumClasses; ++c) {
        s->grid[c] = persistent_grid(kClassKinds[c]);
        ok = s->grid[c] > 0;
    }
    if (!ok) {
        (void)hipGetLastError();
        gf2e_server_destroy(reinterpret_cast<gf2e_server*>(s.release()));
        return GF2E_ENOMEM;
    }
    s->arena = new Arena(cfg->memory_budget);
    for (int i = slots - 1; i >= 0; --i) s->free_slots.push_back(i);
    std::memset(s->h_err, 0, sizeof(int) * slots);
    s->t0 = Clock::now();
    Server* raw = s.release();
    raw->worker = std::thread([raw] { raw->run(); });
    *out = reinterpret_cast<gf2e_server*>(raw);
    return GF2E_OK;
}

void gf2e_server_destroy(gf2e_server* handle)
{
    Server* s = reinterpret_cast<Server*>(handle);
    if (!s) return;
    if (s->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->stop = true;
        }
        s->cv_work.notify_all();
        s->worker.join();  // the loop drains every submitted request first
    }
    DeviceGuard guard(s->ctx->device);
    if (s->stream) (void)hipStreamSynchronize(s->stream);
    for (auto& kv : s->all) {
        if (kv.second->ready_ev) (void)hipEventDestroy(kv.second->ready_ev);
        if (kv.second->done_ev) (void)hipEventDestroy(kv.second->done_ev);
        delete kv.second;
    }
    for (int b = 0; b < kIterBuffers; ++b) {
        if (s->d_items[b]) (void)hipFree(s->d_items[b]);
        if (s->h_items[b]) (void)hipHostFree(s->h_items[b]);
        if (s->iter_ev[b]) (void)hipEventDestroy(s->iter_ev[b]);
    }
    if (s->d_counters) (void)hipFree(s->d_counters);
    if (s->d_err) (void)hipFree(s->d_err);
    if (s->h_err) (void)hipHostFree(s->h_err);
    if (s->d_slots) (void)hipFree(s->d_slots);
    if (s->h_slots) (void)hipHostFree(s->h_slots);
    if (s->arena_base) (void)hipFree(s->arena_base);
    if (s->stream) (void)hipStreamDestroy(s->stream);
    delete s->arena;
    delete s;
}

int gf2e_server_submit(gf2e_server* handle, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                       uint32_t f, void* stream, uint64_t* ticket)
{
    Server* s = reinterpret_cast<Server*>(handle);
    if (!s || !ticket) return GF2E_EINVAL;
    int rc = validate_mul(A, B, C, e, f);
    if (rc) return rc;
    const int64_t m = A->rows, k = A->cols, n = B->cols;
    auto r = std::make_unique<Request>();
    r->plan = make_plan(e, f, std::max<int64_t>(m, 1), std::max<int64_t>(k, 1), std::max<int64_t>(n, 1));
    r->footprint = footprint_of(r->plan);
    if (r->footprint > s->cfg.memory_budget) return GF2E_EBUSY;  // can never be admitted
    BatchProduct& d = r->d;
    d.A = A->data; d.B = B->data; d.C = C->data;
    d.lda = A->ld; d.ldb = B->ld; d.ldc = C->ld;
    d.m = m; d.k = k; d.n = n;
    d.Mp = r->plan.Mp; d.Np = r->plan.Np; d.K64p = r->plan.K64p;
    d.e = e; d.T = r->plan.T; d.f = f; d.sid = r->plan.sid;
    r->cls = (std::min(m, n) >= s->ctx->batch_threshold ? 0 : 1) +
             (r->plan.K64p * 64 <= kFp4MaxK ? 0 : 2);
    const GemmShape sh = gemm_shape(kClassKinds[r->cls]);
    r->tm = int(ceil_div(std::max<int64_t>(m, 1), sh.bm));
    r->tn = int(ceil_div(std::max<int64_t>(n, 1), sh.bn));
    // One plane per item: an iteration's quantum then splits into many items,
    // which keeps the device full and the latency of small requests low.
    r->group = 1;
    r->total_items = (m > 0 && n > 0 && k > 0) ? ceil_div(r->plan.T, r->group) * r->tm * r->tn : 0;
    {
        DeviceGuard guard(s->ctx->device);
        if (hipEventCreateWithFlags(&r->ready_ev, hipEventDisableTiming) != hipSuccess) return GF2E_EDEVICE;
        if (hipEventCreateWithFlags(&r->done_ev, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(r->ready_ev, static_cast<hipStream_t>(stream)) != hipSuccess) {
            (void)hipEventDestroy(r->ready_ev);
            if (r->done_ev) (void)hipEventDestroy(r->done_ev);
            return GF2E_EDEVICE;
        }
    }
    Request* raw = r.release();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        raw->ticket = s->next_ticket++;
        raw->t_submit = s->now_ns();
        s->all[raw->ticket] = raw;
        s->incoming.push_back(raw);
        *ticket = raw->ticket;
    }
    s->cv_work.notify_one();
    return GF2E_OK;
}

static void fill_times(const Request* r, gf2e_req_times* t)
{
    if (!t) return;
    t->t_submit_ns = r->t_submit;
    t->t_admit_ns = r->t_admit;
    t->t_done_ns = r->t_done;
    t->status = r->status;
}

int gf2e_server_poll(gf2e_server* handle, uint64_t ticket, int* done, gf2e_req_times* times)
{
    Server* s = reinterpret_cast<Server*>(handle);
    if (!s || !done) return GF2E_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->all.find(ticket);
    if (it == s->all.end()) return GF2E_EINVAL;
    *done = it->second->state == DONE;
    if (*done) fill_times(it->second, times);
    return GF2E_OK;
}

// Waits for the request, reports its times and status, and forgets it.
int gf2e_server_wait(gf2e_server* handle, uint64_t ticket, gf2e_req_times* times)
{
    Server* s = reinterpret_cast<Server*>(handle);
    if (!s) return GF2E_EINVAL;
    Request* r = nullptr;
    {
        std::unique_lock<std::mutex> lk(s->mu);
        auto it = s->all.find(ticket);
        if (it == s->all.end()) return GF2E_EINVAL;
        r = it->second;
        s->cv_done.wait(lk, [&] { return r->state == DONE; });
        s->all.erase(it);
    }
    fill_times(r, times);
    const int status = r->status;
    {
        DeviceGuard guard(s->ctx->device);
        (void)hipEventDestroy(r->ready_ev);
        (void)hipEventDestroy(r->done_ev);
    }
    delete r;
    return status;
}

int gf2e_server_stats(gf2e_server* handle, gf2e_server_counters* out)
{
    Server* s = reinterpret_cast<Server*>(handle);
    if (!s || !out) return GF2E_EINVAL;
    out->completed = s->completed;
    out->iterations = s->iterations;
    out->element_macs = s->element_macs;
    out->peak_arena_bytes = s->peak_arena;
    out->peak_inflight = s->peak_inflight;
    out->memory_waits = s->memory_waits;
    out->bypass_admissions = s->bypass_admissions;
    out->shared_iterations = s->shared_iterations;
    out->max_iteration_requests = s->max_iteration_requests;
    return GF2E_OK;
}

// Open-loop driver: request i is submitted at arrival_s[i] seconds after the
// call starts (sleeping until then), then every request is awaited.  Times
// are reported relative to the start of the call.
int gf2e_server_run_trace(gf2e_server* handle, int count, const gf2e_mat* A, const gf2e_mat* B,
                          gf2e_mat* C, const int* e, const uint32_t* f, const double* arrival_s,
                          void* stream, gf2e_req_times* out)
{
    Server* s = reinterpret_cast<Server*>(handle);
    if (!s || count < 0 || (count > 0 && (!A || !B || !C || !e || !f || !arrival_s || !out)))
        return GF2E_EINVAL;
    std::vector<uint64_t> tickets(size_t(count), 0);
    const int64_t base = s->now_ns();
    const auto start = Clock::now();
    int first_error = GF2E_OK;
    for (int i = 0; i < count; ++i) {
        std::this_thread::sleep_until(start + std::chrono::nanoseconds(int64_t(arrival_s[i] * 1e9)));
        const int rc = gf2e_server_submit(handle, &A[i], &B[i], &C[i], e[i], f[i], stream, &tickets[i]);
        if (rc) {
            tickets[i] = 0;
            out[i] = {0, 0, 0, rc};
            if (!first_error) first_error = rc;
        }
    }
    for (int i = 0; i < count; ++i) {
        if (!tickets[i]) continue;
        gf2e_req_times t{};
        gf2e_server_wait(handle, tickets[i], &t);
        out[i] = {t.t_submit_ns - base, t.t_admit_ns - base, t.t_done_ns - base, t.status};
        if (t.status && !first_error) first_error = t.status;
    }
    return first_error;
}

}  // extern "C"
