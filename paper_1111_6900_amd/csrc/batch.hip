// Batched products: many independent C_p = A_p * B_p over F_{2^e_p} of
// uneven shapes and mixed e in three launches, captured once into a HIP
// graph and replayed.
//
// After slicing, a product over any F_{2^e} is t(e) GF(2) plane products of
// the same (m, n, k) (Section 5), so one persistent grouped kernel serves
// every field: its work list holds (product, planes, tile) items, sorted by
// decreasing work so the longest start first, and workgroups take items
// from a global counter until the list is exhausted.  Slicing and combining
// run as one grouped launch each, dispatching on e per product.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include "ctx.hpp"
#include "field.hpp"

namespace gf2e {

namespace {
// Tile classes: {large, small} x {fp4 (k <= 2^23), int8}, and the fused
// class: fp4 128x128 tiles of every plane of a product with the
// recombination in the epilogue (e <= kFusedMaxE).
constexpr int kNumPlainClasses = 4;
constexpr int kNumClasses = 5;
constexpr int kFusedClass = 4;
constexpr int kClassKinds[kNumPlainClasses] = {GEMM_FP4_256x256_W8, GEMM_FP4_128x128, GEMM_MFMA_256x256_W8,
                                               GEMM_MFMA_128x128};
// Tile shape of a class.
GemmShape class_shape(int cls) { return gemm_shape(cls == kFusedClass ? GEMM_FP4_128x128 : kClassKinds[cls]); }

// omask[s] for the fused epilogue: bit c set when plane product s enters
// result plane c.  A folded field schedule gives it directly; for a
// Karatsuba schedule, product s enters coefficient plane d when s is in
// w[d], and plane d enters result plane c when bit c of x^d mod f is set.
void result_masks(int e, uint32_t f, int sid, uint32_t* out)
{
    const KernelSchedule S = kernel_schedule(e, sid);
    for (int s = 0; s < S.t; ++s) {
        if (S.folded) {
            out[s] = S.c[s];
            continue;
        }
        uint32_t m = 0;
        for (int d = 0; d < 2 * e - 1; ++d)
            if ((S.w[d] >> s) & 1u) m ^= x_pow_mod(d, f, e);
        out[s] = m;
    }
}
}  // namespace

struct BatchGraph {
    std::vector<uint8_t> key;
    int count = 0;
    void* arena = nullptr;
    int64_t arena_bytes = 0;
    BatchProduct* d_prods = nullptr;
    WorkItem* d_items = nullptr;
    int* d_counters = nullptr;
    uint32_t* d_masks = nullptr;  // omask tables of the fused products
    int n_items[kNumClasses] = {};
    int grid[kNumClasses] = {};
    int* d_jobs = nullptr;  // job lists of the slicing and combining launches
    JobList slice_jobs[2], combine_jobs[2];
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~BatchGraph()
    {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (cap) (void)hipStreamDestroy(cap);
        if (d_counters) (void)hipFree(d_counters);
        if (d_masks) (void)hipFree(d_masks);
        if (d_jobs) (void)hipFree(d_jobs);
        if (d_items) (void)hipFree(d_items);
        if (d_prods) (void)hipFree(d_prods);
        if (arena) (void)hipFree(arena);
    }
};

namespace {

constexpr int kMaxCachedBatches = 8;


template <class T>
void put(std::vector<uint8_t>& key, const T& v)
{
    const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
    key.insert(key.end(), p, p + sizeof(T));
}

int64_t align256(int64_t x) { return (x + 255) / 256 * 256; }

}  // namespace

void Ctx::release_batches()
{
    if (!batches.empty()) (void)hipDeviceSynchronize();
    for (BatchGraph* b : batches) delete b;
    batches.clear();
}

static int build_batch(Ctx* c, int count, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C,
                       const int* e, const uint32_t* f, std::vector<uint8_t>&& key, BatchGraph** out)
{
    auto bg = std::make_unique<BatchGraph>();
    bg->key = std::move(key);
    const int TPB = batch_threads_per_block();

    // Plans and the arena layout.
    std::vector<BatchProduct> prods;
    std::vector<int64_t> offs;
    int64_t total = 0;
    for (int p = 0; p < count; ++p) {
        const int64_t m = A[p].rows, k = A[p].cols, n = B[p].cols;
        if (m == 0 || n == 0) continue;
        const Plan pl = make_plan(e[p], f[p], m, k, n);
        BatchProduct d{};
        d.A = A[p].data; d.B = B[p].data; d.C = C[p].data;
        d.lda = A[p].ld; d.ldb = B[p].ld; d.ldc = C[p].ld;
        d.m = m; d.k = k; d.n = n;
        d.Mp = pl.Mp; d.Np = pl.Np; d.K64p = pl.K64p;
        d.e = e[p]; d.T = pl.T; d.f = f[p]; d.sid = pl.sid;
        d.slice_a_blocks = k > 0 ? int32_t(pl.Mp / TPB * pl.K64p) : 0;
        d.slice_b_blocks = k > 0 ? int32_t(pl.Np / TPB * pl.K64p) : 0;
        d.combine_blocks = int32_t(ceil_div(m * ceil_div(n, 64), TPB));
        // Fused: fp4 128x128 class, e small enough for the epilogue's result planes.
        d.fused = c->batch_fused && k > 0 && e[p] <= kFusedMaxE && pl.K64p * 64 <= kFp4MaxK &&
                  std::min(m, n) < c->batch_threshold;
        offs.push_back(total);
        if (k > 0) total += align256(pl.a_bytes) + align256(pl.b_bytes) + (d.fused ? 0 : align256(pl.p_bytes));
        prods.push_back(d);
    }
    bg->count = int(prods.size());
    if (bg->count > 65535) return GF2E_EINVAL;
    if (total > 0 && hipMalloc(&bg->arena, size_t(total)) != hipSuccess) {
        (void)hipGetLastError();
        return GF2E_ENOMEM;
    }
    bg->arena_bytes = total;
    for (size_t i = 0; i < prods.size(); ++i) {
        BatchProduct& d = prods[i];
        if (d.k == 0) continue;
        uint8_t* base = static_cast<uint8_t*>(bg->arena) + offs[i];
        const Plan pl = make_plan(d.e, d.f, d.m, d.k, d.n);
        d.Apl = reinterpret_cast<uint64_t*>(base);
        d.Bpl = reinterpret_cast<uint64_t*>(base + align256(pl.a_bytes));
        d.P = d.fused ? nullptr : reinterpret_cast<uint64_t*>(base + align256(pl.a_bytes) + align256(pl.b_bytes));
    }
    // omask tables of the fused products, one device array.
    {
        std::vector<uint32_t> masks;
        std::vector<int64_t> at(prods.size(), -1);
        for (size_t i = 0; i < prods.size(); ++i) {
            if (!prods[i].fused) continue;
            at[i] = int64_t(masks.size());
            masks.resize(masks.size() + size_t(prods[i].T));
            result_masks(prods[i].e, prods[i].f, prods[i].sid, masks.data() + at[i]);
        }
        if (!masks.empty()) {
            if (hipMalloc(&bg->d_masks, masks.size() * sizeof(uint32_t)) != hipSuccess) {
                (void)hipGetLastError();
                return GF2E_ENOMEM;
            }
            if (hipMemcpy(bg->d_masks, masks.data(), masks.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
                hipSuccess)
                return GF2E_EDEVICE;
            for (size_t i = 0; i < prods.size(); ++i)
                if (at[i] >= 0) prods[i].omask = bg->d_masks + at[i];
        }
    }

    // Work lists: size class by the smaller output dimension.
    std::vector<WorkItem> items[kNumClasses];
    for (size_t i = 0; i < prods.size(); ++i) {
        const BatchProduct& d = prods[i];
        if (d.k == 0) continue;
        const int cls = d.fused ? kFusedClass
                                : (std::min(d.m, d.n) >= c->batch_threshold ? 0 : 1) +
                                      (d.K64p * 64 <= kFp4MaxK ? 0 : 2);
        const GemmShape sh = class_shape(cls);
        const int tm = int(ceil_div(d.m, sh.bm)), tn = int(ceil_div(d.n, sh.bn));
        if (d.fused) {  // one item per tile, all planes
            for (int a = 0; a < tm; ++a)
                for (int b = 0; b < tn; ++b) items[cls].push_back({int32_t(i), 0, a, b, d.T});
            continue;
        }
        // Planes of one tile per item: as many as keep an item below
        // kItemKWords k-words in all, so that items stay comparable.
        const int group = int(std::clamp<int64_t>(kItemKWords / d.K64p, 1, d.T));
        for (int s = 0; s < d.T; s += group)
            for (int a = 0; a < tm; ++a)
                for (int b = 0; b < tn; ++b)
                    items[cls].push_back({int32_t(i), s, a, b, std::min(group, d.T - s)});
    }
    const char* shuffle = std::getenv("GF2E_BATCH_SHUFFLE");
    for (int cls = 0; cls < kNumClasses; ++cls) {
        auto& v = items[cls];
        if (shuffle && *shuffle) {
            std::mt19937_64 rng(std::strtoull(shuffle, nullptr, 10));
            std::shuffle(v.begin(), v.end(), rng);
        } else {
            std::stable_sort(v.begin(), v.end(), [&](const WorkItem& x, const WorkItem& y) {
                return prods[x.prod].K64p * x.nplanes > prods[y.prod].K64p * y.nplanes;
            });
        }
        bg->n_items[cls] = int(v.size());
        bg->grid[cls] = v.empty() ? 0 : cls == kFusedClass ? fused_persistent_grid() : persistent_grid(kClassKinds[cls]);
        if (!v.empty() && bg->grid[cls] <= 0) return GF2E_EDEVICE;
    }

    // Device copies of the descriptors and work lists.
    size_t nall = 0, item_off[kNumClasses] = {};
    for (int cls = 0; cls < kNumClasses; ++cls) {
        item_off[cls] = nall;
        nall += items[cls].size();
    }
    if (hipMalloc(&bg->d_prods, sizeof(BatchProduct) * std::max<size_t>(prods.size(), 1)) != hipSuccess ||
        hipMalloc(&bg->d_items, sizeof(WorkItem) * std::max<size_t>(nall, 1)) != hipSuccess ||
        hipMalloc(&bg->d_counters, kNumClasses * sizeof(int)) != hipSuccess) {
        (void)hipGetLastError();
        return GF2E_ENOMEM;
    }
    if (!prods.empty() && hipMemcpy(bg->d_prods, prods.data(), sizeof(BatchProduct) * prods.size(),
                                    hipMemcpyHostToDevice) != hipSuccess)
        return GF2E_EDEVICE;
    for (int cls = 0; cls < kNumClasses; ++cls)
        if (!items[cls].empty() &&
            hipMemcpy(bg->d_items + item_off[cls], items[cls].data(), sizeof(WorkItem) * items[cls].size(),
                      hipMemcpyHostToDevice) != hipSuccess)
            return GF2E_EDEVICE;

    // Job lists of the slicing and combining launches, per e-range: the
    // products of the range and the prefix sums of their blocks, laid out as
    // four lists of (first[n + 1], owner[n]) in one device array.
    {
        std::vector<int> host;
        int64_t at[4] = {}, totals[4] = {};
        int ns[4] = {};
        for (int list = 0; list < 4; ++list) {
            const bool combine = list >= 2, large = list & 1;
            std::vector<int> own;
            std::vector<int64_t> first{0};
            for (size_t i = 0; i < prods.size(); ++i) {
                const BatchProduct& d = prods[i];
                if ((d.e > kBatchSmallE) != large) continue;
                if (combine && d.fused) continue;  // its product kernel writes C
                const int64_t blocks = combine ? d.combine_blocks : int64_t(d.slice_a_blocks) + d.slice_b_blocks;
                if (blocks == 0) continue;
                own.push_back(int(i));
                first.push_back(first.back() + blocks);
            }
            if (first.back() > INT32_MAX) return GF2E_EINVAL;  // one launch's grid
            at[list] = int64_t(host.size());
            for (int64_t v : first) host.push_back(int(v));
            host.insert(host.end(), own.begin(), own.end());
            ns[list] = int(own.size());
            totals[list] = first.back();
        }
        if (hipMalloc(&bg->d_jobs, host.size() * sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            return GF2E_ENOMEM;
        }
        if (hipMemcpy(bg->d_jobs, host.data(), host.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return GF2E_EDEVICE;
        for (int list = 0; list < 4; ++list) {
            JobList& jl = list >= 2 ? bg->combine_jobs[list & 1] : bg->slice_jobs[list & 1];
            jl.first = bg->d_jobs + at[list];
            jl.owner = bg->d_jobs + at[list] + ns[list] + 1;
            jl.n = ns[list];
            jl.total = int(totals[list]);
        }
    }

    // Capture: reset counters, grouped slicing, the persistent products of
    // each size class, grouped combining.
    if (hipStreamCreateWithFlags(&bg->cap, hipStreamNonBlocking) != hipSuccess) return GF2E_EDEVICE;
    if (hipStreamBeginCapture(bg->cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return GF2E_EDEVICE;
    hipError_t err = launch_reset_counters(bg->d_counters, kNumClasses, bg->cap);
    if (err == hipSuccess)
        err = launch_batched_slice(bg->d_prods, bg->slice_jobs, c->d_err, bg->cap);
    for (int cls = 0; cls < kNumClasses && err == hipSuccess; ++cls)
        err = cls == kFusedClass
                  ? launch_fused_persistent(bg->d_prods, bg->d_items + item_off[cls], bg->n_items[cls],
                                            bg->d_counters + cls, bg->grid[cls], bg->cap)
                  : launch_persistent_gemm(kClassKinds[cls], bg->d_prods, bg->d_items + item_off[cls],
                                           bg->n_items[cls], bg->d_counters + cls, bg->grid[cls], bg->cap);
    if (err == hipSuccess)
        err = launch_batched_combine(bg->d_prods, bg->combine_jobs, bg->cap);
    hipGraph_t graph = nullptr;
    const hipError_t end = hipStreamEndCapture(bg->cap, &graph);
    bg->graph = graph;
    if (err != hipSuccess || end != hipSuccess || !graph) return GF2E_EDEVICE;
    if (hipGraphInstantiate(&bg->exec, bg->graph, nullptr, nullptr, 0) != hipSuccess) return GF2E_EDEVICE;
    *out = bg.release();
    return GF2E_OK;
}

}  // namespace gf2e

using namespace gf2e;

extern "C" {

int gf2e_mul_batched(gf2e_ctx* handle, int count, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C,
                     const int* e, const uint32_t* f, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || count < 0) return GF2E_EINVAL;
    if (count == 0) return GF2E_OK;
    if (!A || !B || !C || !e || !f) return GF2E_EINVAL;
    for (int p = 0; p < count; ++p) {
        int rc = validate_mul(&A[p], &B[p], &C[p], e[p], f[p]);
        if (rc) return rc;
    }
    // Outputs must not overlap each other either: sort their byte ranges by
    // start and compare each start with the furthest end seen so far.
    {
        std::vector<std::pair<uintptr_t, uintptr_t>> ranges;
        for (int p = 0; p < count; ++p) {
            if (C[p].rows <= 0 || C[p].cols <= 0) continue;
            const uintptr_t lo = reinterpret_cast<uintptr_t>(C[p].data);
            ranges.push_back(
                {lo, lo + uintptr_t(((C[p].rows - 1) * C[p].ld + C[p].cols) * elem_bytes(e[p]))});
        }
        std::sort(ranges.begin(), ranges.end());
        uintptr_t end = 0;
        for (size_t i = 0; i < ranges.size(); ++i) {
            if (i > 0 && ranges[i].first < end) return GF2E_EALIAS;
            end = std::max(end, ranges[i].second);
        }
    }
    std::vector<uint8_t> key;
    put(key, c->batch_threshold);
    put(key, c->batch_fused);
    put(key, count);
    for (int p = 0; p < count; ++p) {
        put(key, A[p]); put(key, B[p]); put(key, C[p]); put(key, e[p]); put(key, f[p]);
    }
    if (const char* sh = std::getenv("GF2E_BATCH_SHUFFLE")) key.insert(key.end(), sh, sh + std::strlen(sh));

    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchGraph* bg = nullptr;
    for (size_t i = 0; i < c->batches.size(); ++i)
        if (c->batches[i]->key == key) {
            bg = c->batches[i];
            // most recently used goes last
            c->batches.erase(c->batches.begin() + long(i));
            c->batches.push_back(bg);
            break;
        }
    if (!bg) {
        if (int(c->batches.size()) >= kMaxCachedBatches) {
            (void)hipDeviceSynchronize();
            delete c->batches.front();
            c->batches.erase(c->batches.begin());
        }
        int rc = build_batch(c, count, A, B, C, e, f, std::move(key), &bg);
        if (rc) return rc;
        c->batches.push_back(bg);
        c->batch_builds += 1;
    }
    c->order_stream(s);
    hipError_t err;
    {
        StageTimer t(c, GF2E_STAGE_BATCH, s);
        err = hipGraphLaunch(bg->exec, s);
    }
    c->mark_used(s);
    c->last_batch_items[0] = bg->n_items[0] + bg->n_items[2];
    c->last_batch_items[1] = bg->n_items[1] + bg->n_items[3];
    c->last_batch_items[2] = bg->n_items[kFusedClass];
    c->last_batch_arena = bg->arena_bytes;
    return err == hipSuccess ? GF2E_OK : GF2E_EDEVICE;
}

int gf2e_set_batch_threshold(gf2e_ctx* handle, int64_t min_dim)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || min_dim < 0) return GF2E_EINVAL;
    c->batch_threshold = min_dim;
    return GF2E_OK;
}

int gf2e_set_batch_fusion(gf2e_ctx* handle, int on)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || on < 0 || on > 1) return GF2E_EINVAL;
    c->batch_fused = on == 1;
    return GF2E_OK;
}

int gf2e_batch_info(gf2e_ctx* handle, gf2e_batch_stats* out)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !out) return GF2E_EINVAL;
    out->items_large = c->last_batch_items[0];
    out->items_small = c->last_batch_items[1];
    out->items_fused = c->last_batch_items[2];
    out->fusion = c->batch_fused ? 1 : 0;
    out->arena_bytes = c->last_batch_arena;
    out->graphs_cached = int(c->batches.size());
    out->graph_builds = c->batch_builds;
    out->threshold = c->batch_threshold;
    return GF2E_OK;
}

int gf2e_tune_batched(gf2e_ctx* handle, int count, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C,
                      const int* e, const uint32_t* f, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    // (threshold, fusion) pairs: with fusion on, the products below the
    // threshold take the fused class, the rest 256x256 tiles.
    static const int64_t thresholds[] = {0, 256, 384, 512, 768, INT64_MAX};
    hipStream_t s = static_cast<hipStream_t>(stream);
    DeviceGuard guard(c->device);
    hipEvent_t e0 = c->get_event(), e1 = c->get_event();
    if (!e0 || !e1) return GF2E_EDEVICE;
    int64_t best = c->batch_threshold;
    bool best_fused = c->batch_fused;
    float best_ms = -1;
    auto restore = [&] {
        c->batch_threshold = best;
        c->batch_fused = best_fused;
    };
    for (int fused = 1; fused >= 0; --fused)
        for (int64_t th : thresholds) {
            if (fused && th == 0) continue;  // the same as th = 0 without fusion
            c->batch_threshold = th;
            c->batch_fused = fused == 1;
            int rc = gf2e_mul_batched(handle, count, A, B, C, e, f, stream);  // build + warm-up
            if (rc) { restore(); return rc; }
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < 3 && rc == GF2E_OK; ++r) rc = gf2e_mul_batched(handle, count, A, B, C, e, f, stream);
            (void)hipEventRecord(e1, s);
            if (rc || hipEventSynchronize(e1) != hipSuccess) { restore(); return rc ? rc : GF2E_EDEVICE; }
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            if (best_ms < 0 || ms < best_ms) {
                best_ms = ms;
                best = th;
                best_fused = fused == 1;
            }
            c->release_batches();  // each candidate holds its own plane arena
        }
    c->event_pool.push_back(e0);
    c->event_pool.push_back(e1);
    restore();
    return GF2E_OK;
}

}  // extern "C"
