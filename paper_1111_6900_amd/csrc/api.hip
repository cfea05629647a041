// C ABI of the library: validation, planning, workspace, stage launches,
// autotuning and stage timers.  See include/gf2e.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ctx.hpp"
#include "field.hpp"
#include "gf2e.h"

namespace gf2e {

DeviceGuard::DeviceGuard(int dev)
{
    if (hipGetDevice(&prev_) != hipSuccess) prev_ = -1;
    if (prev_ != dev) (void)hipSetDevice(dev);
}
DeviceGuard::~DeviceGuard()
{
    int cur = -1;
    if (prev_ >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev_) (void)hipSetDevice(prev_);
}

int elem_bytes(int e) { return e <= 8 ? 1 : 2; }

// Plane workspace of gf2e_mul_noalloc_async: a fixed array in device memory,
// one per GPU, held until the process ends and shared by every call on that
// GPU.  Host code never passes `scratch` itself to a kernel (on the host it
// names a stand-in, not the device array); it uses the address that
// hipGetSymbolAddress reports for the current device, kept per device.
static __device__ __align__(256) uint64_t scratch[GF2E_NOALLOC_MAX_BYTES / 8];

namespace {
std::mutex scratch_mu;
std::vector<void*> scratch_addr;  // per device; nullptr until looked up
}  // namespace

// Looks up the device address of `scratch` on `dev` (which must be current)
// once; later calls return the kept address.  nullptr if the lookup failed.
static void* scratch_on(int dev)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (dev < 0) return nullptr;
    if (size_t(dev) >= scratch_addr.size()) scratch_addr.resize(size_t(dev) + 1, nullptr);
    if (!scratch_addr[size_t(dev)]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        scratch_addr[size_t(dev)] = ptr;
    }
    return scratch_addr[size_t(dev)];
}

static void* scratch_known(int dev)
{
    std::lock_guard<std::mutex> lk(scratch_mu);
    return dev >= 0 && size_t(dev) < scratch_addr.size() ? scratch_addr[size_t(dev)] : nullptr;
}

bool field_ok(int e, uint32_t f)
{
    if (e < 2 || e > kMaxE) return false;
    // f must have degree exactly e; this also rejects f = 0, which would
    // otherwise match an empty cache slot below.
    if ((f >> e) != 1u) return false;
    // The last irreducible f seen per degree (per thread): batches repeat a
    // few fields many times.  A slot holds 0 until a valid f is cached.
    thread_local uint32_t known[kMaxE + 1] = {};
    if (known[e] == f) return true;
    if (!is_irreducible(e, f)) return false;
    known[e] = f;
    return true;
}

int check_mat(const gf2e_mat* M)
{
    if (!M) return GF2E_EINVAL;
    if (M->rows < 0 || M->cols < 0) return GF2E_ESHAPE;
    if (M->rows > 0 && M->cols > 0) {
        if (M->ld < M->cols) return GF2E_ESHAPE;
        if (!M->data) return GF2E_EINVAL;
    }
    return GF2E_OK;
}

// Byte range [lo, hi) touched by a matrix (empty when it has no entries).
static void extent(const gf2e_mat* M, int esz, uintptr_t* lo, uintptr_t* hi)
{
    *lo = *hi = 0;
    if (M->rows <= 0 || M->cols <= 0) return;
    *lo = reinterpret_cast<uintptr_t>(M->data);
    *hi = *lo + uintptr_t(((M->rows - 1) * M->ld + M->cols) * esz);
}

bool overlaps(const gf2e_mat* X, const gf2e_mat* Y, int esz)
{
    uintptr_t a0, a1, b0, b1;
    extent(X, esz, &a0, &a1);
    extent(Y, esz, &b0, &b1);
    if (a0 == a1 || b0 == b1) return false;
    return a0 < b1 && b0 < a1;
}

int validate_mul(const gf2e_mat* A, const gf2e_mat* B, const gf2e_mat* C, int e, uint32_t f)
{
    int rc;
    if ((rc = check_mat(A)) || (rc = check_mat(B)) || (rc = check_mat(C))) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (A->rows != C->rows || A->cols != B->rows || B->cols != C->cols) return GF2E_ESHAPE;
    const int esz = elem_bytes(e);
    if (overlaps(C, A, esz) || overlaps(C, B, esz)) return GF2E_EALIAS;
    return GF2E_OK;
}

int schedule_id(int e, uint32_t f)
{
    static const bool karatsuba_only = [] {
        const char* v = std::getenv("GF2E_SCHEDULE");
        return v && std::strcmp(v, "karatsuba") == 0;
    }();
    return karatsuba_only ? -1 : find_field_schedule(e, f);
}

Plan make_plan(int e, uint32_t f, int64_t m, int64_t k, int64_t n, int form, bool short_k)
{
    Plan p{};
    p.e = e;
    p.f = f;
    p.form = form;
    p.m = m; p.k = k; p.n = n;
    p.Mp = round_up(std::max<int64_t>(m, 1), kRowAlign);
    p.Np = round_up(std::max<int64_t>(n, 1), kRowAlign);
    p.K64p = short_k && k <= 128 ? 2 : kwords_padded(std::max<int64_t>(k, 1));
    // The alpha form's product has e blocks of K64p words along k; with
    // k <= 64 and e even one word per block keeps that a whole number of
    // 128-bit stages and halves the product.
    if (form == kFormAlpha && short_k && k <= 64 && e % 2 == 0) p.K64p = 1;
    if (form == kFormAlpha) {
        p.sid = kIdentitySchedule;
        p.T = e;
        p.gT = 1;
        p.gNp = int64_t(e) * p.Np;
        p.gn = int64_t(e - 1) * p.Np + std::max<int64_t>(n, 1);
        p.gK64p = int64_t(e) * p.K64p;
        p.a_bytes = int64_t(e) * p.K64p * p.Mp * 8;
        p.b_bytes = p.gK64p * p.gNp * 8;
        p.p_bytes = p.Mp * (p.gNp / 64) * 8;
    } else {
        p.sid = schedule_id(e, f);
        p.T = p.sid >= 0 ? kFieldSchedules[p.sid].t : best_count(e);
        p.gT = p.T;
        p.gn = std::max<int64_t>(n, 1);
        p.gNp = p.Np;
        p.gK64p = p.K64p;
        p.a_bytes = int64_t(p.T) * p.K64p * p.Mp * 8;
        p.b_bytes = int64_t(p.T) * p.K64p * p.Np * 8;
        p.p_bytes = int64_t(p.T) * p.Mp * (p.Np / 64) * 8;
    }
    return p;
}

// ---------------------------------------------------------------------------
// Context helpers
// ---------------------------------------------------------------------------

hipEvent_t Ctx::get_event()
{
    if (!event_pool.empty()) {
        hipEvent_t ev = event_pool.back();
        event_pool.pop_back();
        return ev;
    }
    hipEvent_t ev = nullptr;
    if (hipEventCreate(&ev) != hipSuccess) return nullptr;
    return ev;
}

void Ctx::order_stream(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    if (have_last && s != last_stream && cs == hipStreamCaptureStatusNone)
        (void)hipStreamWaitEvent(s, ws_done, 0);
}

void Ctx::mark_used(hipStream_t s)
{
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone) return;
    (void)hipEventRecord(ws_done, s);
    last_stream = s;
    have_last = true;
}

int Ctx::ensure_workspace(int64_t bytes, hipStream_t s)
{
    if (bytes <= ws_bytes) return GF2E_OK;
    if (cfg.workspace_limit > 0 && bytes > cfg.workspace_limit) return GF2E_ENOMEM;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone) return GF2E_ENOMEM;  // cannot allocate while capturing
    if (ws) {
        if (hipDeviceSynchronize() != hipSuccess) return GF2E_EDEVICE;
        (void)hipFree(ws);
        ws = nullptr;
        ws_bytes = 0;
    }
    void* p = nullptr;
    if (hipMalloc(&p, size_t(bytes)) != hipSuccess) {
        (void)hipGetLastError();
        return GF2E_ENOMEM;
    }
    ws = p;
    ws_bytes = bytes;
    return GF2E_OK;
}

StageTimer::StageTimer(Ctx* c, int stage, hipStream_t s, bool on) : ctx_(c), stage_(stage), s_(s)
{
    if (!on || !ctx_->prof) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    if (cs != hipStreamCaptureStatusNone) return;
    a_ = ctx_->get_event();
    b_ = ctx_->get_event();
    if (a_ && b_) (void)hipEventRecord(a_, s_);
}

StageTimer::~StageTimer()
{
    if (a_ && b_) {
        (void)hipEventRecord(b_, s_);
        ctx_->prof_pending[stage_].push_back({a_, b_});
    }
}

static uint64_t bucket_key(int T, int64_t m, int64_t k, int64_t n)
{
    auto lg = [](int64_t x) { return uint64_t(std::lround(std::log2(double(std::max<int64_t>(x, 1))) * 2.0)); };
    return (uint64_t(T) << 48) | (lg(m) << 32) | (lg(n) << 16) | lg(k);
}

// A size bucket is keyed by the schedule form's product count (which depends
// on e and f) and the rounded log sizes.  Its tuned choice packs the best
// kernel of each form and the faster form.
static uint64_t bucket_of(int e, uint32_t f, int64_t m, int64_t k, int64_t n)
{
    return bucket_key(make_plan(e, f, m, k, n).T, m, k, n);
}
static int pack_choice(int kind0, int kind1, int form) { return (kind0 & 0xFF) | ((kind1 & 0xFF) << 8) | (form << 16); }
static int choice_kind(int choice, int form) { return (choice >> (8 * form)) & 0xFF; }
static int choice_form(int choice) { return (choice >> 16) & 0xFF; }

int default_kind(int T, int64_t m, int64_t n)
{
    const int64_t t256 = int64_t(T) * ceil_div(m, 256) * ceil_div(n, 256);
    const int64_t t128 = int64_t(T) * ceil_div(m, 128) * ceil_div(n, 128);
    if (t256 >= 512) return GEMM_MFMA_256x256_W8;
    if (t128 >= 256) return GEMM_MFMA_128x128;
    return GEMM_MFMA_64x64;
}

bool kind_supports(int kind, const Plan& p)
{
    if (p.gK64p % 4) return kind == GEMM_FP4_128x128_PLANES;  // only it steps 128-bit stages
    const bool fp4 = kind == GEMM_FP4_256x256_W8 || kind == GEMM_FP4_128x128 || kind == GEMM_FP4_128x128_PLANES;
    return !fp4 || p.gK64p * 64 <= kFp4MaxK;
}

int supported_kind(int kind, const Plan& p)
{
    if (kind_supports(kind, p)) return kind;
    // k of 128 bits or less, or f32 counts that would not be exact
    return p.gK64p % 4 ? GEMM_FP4_128x128_PLANES : GEMM_MFMA_256x256_W8;
}

int Ctx::choose_form(int e, uint32_t f, int64_t m, int64_t k, int64_t n)
{
    if (forced_form >= 0) return forced_form;
    auto it = tune.find(bucket_of(e, f, m, k, n));
    if (it != tune.end()) return choice_form(it->second);
    return kFormSchedule;
}

int Ctx::choose_kind(const Plan& p)
{
    if (forced_kind >= 0) return forced_kind;
    auto it = tune.find(bucket_of(p.e, p.f, p.m, p.k, p.n));
    if (it != tune.end()) {
        const int kind = choice_kind(it->second, p.form);
        if (kind < GEMM_NUM_KINDS) return kind;
    }
    return default_kind(p.gT, p.m, p.gn);
}

void Ctx::load_tune_cache()
{
    const char* path = std::getenv("GF2E_TUNE_CACHE");
    if (!path) return;
    FILE* fp = std::fopen(path, "r");
    if (!fp) return;
    char line[256];
    while (std::fgets(line, sizeof line, fp)) {
        unsigned long long key = 0;
        int choice = -1;
        if (std::sscanf(line, "{\"arch\": \"gfx950\", \"key\": %llu, \"choice\": %d", &key, &choice) == 2 &&
            choice >= 0 && choice_form(choice) < kNumForms)
            tune[key] = choice;
    }
    std::fclose(fp);
}

void Ctx::save_tune_entry(uint64_t key, int choice)
{
    const char* path = std::getenv("GF2E_TUNE_CACHE");
    if (!path) return;
    FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    const int form = choice_form(choice);
    std::fprintf(fp, "{\"arch\": \"gfx950\", \"key\": %llu, \"choice\": %d, \"form\": \"%s\", \"kernel\": \"%s\"}\n",
                 static_cast<unsigned long long>(key), choice, form == kFormAlpha ? "alpha" : "schedule",
                 gemm_name(choice_kind(choice, form)));
    std::fclose(fp);
}

int Ctx::exec_plan(const Plan& p, int kind, const void* A, int64_t lda, const void* B, int64_t ldb, void* C,
                   int64_t ldc, hipStream_t s, bool acc, void* planes)
{
    uint64_t* Apl = static_cast<uint64_t*>(planes ? planes : ws);
    uint64_t* Bpl = Apl + p.a_bytes / 8;
    uint64_t* P = Bpl + p.b_bytes / 8;
    // No stage timers on caller-provided planes (the path that must not
    // create events or allocate).
    const bool timed = planes == nullptr;
    hipError_t err;
    {
        StageTimer t(this, GF2E_STAGE_SLICE_A, s, timed);
        err = launch_slice_rows(p.e, p.sid, A, lda, p.m, p.k, Apl, p.Mp, p.K64p, d_err, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    {
        StageTimer t(this, GF2E_STAGE_SLICE_B, s, timed);
        err = p.form == kFormAlpha
                  ? launch_slice_cols_alpha(p.e, p.f, B, ldb, p.k, p.n, Bpl, p.Np, p.K64p, d_err, s)
                  : launch_slice_cols(p.e, p.sid, B, ldb, p.k, p.n, Bpl, p.Np, p.K64p, d_err, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    // Alpha form on an fp4 kernel: the product clings its result into C.
    const bool fp4 = kind == GEMM_FP4_256x256_W8 || kind == GEMM_FP4_128x128 || kind == GEMM_FP4_128x128_PLANES;
    if (p.form == kFormAlpha && fp4 && p.e <= kFusedMaxE && p.gK64p * 64 <= kFp4MaxK) {
        StageTimer t(this, GF2E_STAGE_PRODUCTS, s, timed);
        err = launch_fused_alpha(p.e, Apl, Bpl, p.m, p.n, p.Mp, p.Np, p.gK64p, C, ldc, acc, s);
        return err == hipSuccess ? GF2E_OK : GF2E_EDEVICE;
    }
    {
        StageTimer t(this, GF2E_STAGE_PRODUCTS, s, timed);
        err = launch_gemm(kind, p.gT, Apl, Bpl, P, p.m, p.gn, p.Mp, p.gNp, p.gK64p, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    {
        StageTimer t(this, GF2E_STAGE_COMBINE, s, timed);
        // Alpha form: result plane c is the column block c of the one product.
        err = p.form == kFormAlpha
                  ? launch_combine(p.e, p.sid, p.f, P, p.Np / 64, p.gNp / 64, p.m, p.n, C, ldc, s, acc)
                  : launch_combine(p.e, p.sid, p.f, P, p.Mp * (p.Np / 64), p.Np / 64, p.m, p.n, C, ldc, s, acc);
    }
    return err == hipSuccess ? GF2E_OK : GF2E_EDEVICE;
}

int Ctx::tune_now(int e, uint32_t f, int64_t m, int64_t k, int64_t n, hipStream_t s)
{
    const Plan plans[kNumForms] = {make_plan(e, f, m, k, n, kFormSchedule, true),
                                   make_plan(e, f, m, k, n, kFormAlpha, true)};
    int64_t planes = 0;
    for (const Plan& p : plans) planes = std::max(planes, p.a_bytes + p.b_bytes + p.p_bytes);
    const int esz = elem_bytes(e);
    const int64_t a_in = round_up(m * k * esz, 256), b_in = round_up(k * n * esz, 256);
    const int64_t c_out = round_up(m * n * esz, 256);
    int rc = ensure_workspace(planes + a_in + b_in + c_out, s);
    if (rc) return rc;
    // Inputs of the timings live in the workspace after the planes: random
    // field elements (all-zero data runs the matrix cores at lower power and
    // would time them too fast).
    uint8_t* in = static_cast<uint8_t*>(ws) + planes;
    void* dA = in;
    void* dB = in + a_in;
    void* dC = in + a_in + b_in;
    if (launch_fill_elements(dA, m * k, e, 1, s) != hipSuccess ||
        launch_fill_elements(dB, k * n, e, 2, s) != hipSuccess)
        return GF2E_EDEVICE;
    hipEvent_t e0 = get_event(), e1 = get_event();
    if (!e0 || !e1) return GF2E_EDEVICE;
    const bool verbose = std::getenv("GF2E_TUNE_LOG") != nullptr;
    auto timed = [&](auto&& launch, int reps, float* ms) -> bool {
        (void)hipEventRecord(e0, s);
        for (int r = 0; r < reps; ++r)
            if (!launch()) return false;
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) != hipSuccess) return false;
        (void)hipEventElapsedTime(ms, e0, e1);
        *ms /= reps;
        return true;
    };
    int best_kind[kNumForms] = {-1, -1};
    float pipe_ms[kNumForms] = {-1.f, -1.f};
    for (int form = 0; form < kNumForms; ++form) {
        const Plan& p = plans[form];
        uint64_t* Apl = static_cast<uint64_t*>(ws);
        uint64_t* Bpl = Apl + p.a_bytes / 8;
        uint64_t* P = Bpl + p.b_bytes / 8;
        // Operand planes of this form from the random inputs.
        if (exec_plan(p, supported_kind(default_kind(p.gT, p.m, p.gn), p), dA, k, dB, n, dC, n, s) != GF2E_OK)
            return GF2E_EDEVICE;
        // Two rounds over all product kernels (the first also brings the
        // clocks up); each keeps its best round.
        float best_ms[GEMM_NUM_KINDS];
        for (int kind = 0; kind < GEMM_NUM_KINDS; ++kind) best_ms[kind] = -1.f;
        for (int round = 0; round < 2; ++round)
            for (int kind = 0; kind < GEMM_NUM_KINDS; ++kind) {
                if (!kind_supports(kind, p)) continue;
                auto gemm = [&] {
                    return launch_gemm(kind, p.gT, Apl, Bpl, P, p.m, p.gn, p.Mp, p.gNp, p.gK64p, s) == hipSuccess;
                };
                if (!gemm()) {
                    (void)hipGetLastError();
                    continue;  // not applicable to this shape
                }
                float ms = 0;
                if (!timed(gemm, 1, &ms)) return GF2E_EDEVICE;
                if (!timed(gemm, std::clamp(int(1.0f / std::max(ms, 1e-3f)), 3, 100), &ms)) return GF2E_EDEVICE;
                if (verbose)
                    std::fprintf(stderr, "[gf2e tune] e=%d m=%lld k=%lld n=%lld form %d round %d %s %.4f ms\n", e,
                                 static_cast<long long>(m), static_cast<long long>(k), static_cast<long long>(n),
                                 form, round, gemm_name(kind), ms);
                if (best_ms[kind] < 0 || ms < best_ms[kind]) best_ms[kind] = ms;
            }
        for (int kind = 0; kind < GEMM_NUM_KINDS; ++kind)
            if (best_ms[kind] >= 0 && (best_kind[form] < 0 || best_ms[kind] < best_ms[best_kind[form]]))
                best_kind[form] = kind;
        if (best_kind[form] < 0) continue;
        // The whole pipeline of this form with its best kernel, repeated
        // for about 2 ms so that short pipelines are not timed on noise.
        auto pipe = [&] {
            return exec_plan(p, best_kind[form], dA, k, dB, n, dC, n, s) == GF2E_OK;
        };
        float once = 0;
        if (!pipe() || !timed(pipe, 1, &once)) return GF2E_EDEVICE;
        const int reps = std::clamp(int(2.0f / std::max(once, 1e-3f)), 3, 200);
        if (!timed(pipe, reps, &pipe_ms[form])) return GF2E_EDEVICE;
        if (verbose)
            std::fprintf(stderr, "[gf2e tune] e=%d m=%lld k=%lld n=%lld form %d pipeline %s %.4f ms\n", e,
                         static_cast<long long>(m), static_cast<long long>(k), static_cast<long long>(n), form,
                         gemm_name(best_kind[form]), pipe_ms[form]);
    }
    event_pool.push_back(e0);
    event_pool.push_back(e1);
    if (best_kind[kFormSchedule] < 0 && best_kind[kFormAlpha] < 0) return GF2E_EDEVICE;
    int form = kFormSchedule;
    if (best_kind[kFormSchedule] < 0 || (best_kind[kFormAlpha] >= 0 && pipe_ms[kFormAlpha] < pipe_ms[kFormSchedule]))
        form = kFormAlpha;
    const int choice = pack_choice(best_kind[kFormSchedule] < 0 ? 0xFF : best_kind[kFormSchedule],
                                   best_kind[kFormAlpha] < 0 ? 0xFF : best_kind[kFormAlpha], form);
    const uint64_t key = bucket_of(e, f, m, k, n);
    tune[key] = choice;
    save_tune_entry(key, choice);
    return GF2E_OK;
}

int Ctx::mul(int e, uint32_t f, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, hipStream_t s, bool acc)
{
    const int64_t m = A->rows, k = A->cols, n = B->cols;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    (void)hipStreamIsCapturing(s, &cs);
    int rc;
    if (cfg.autotune && (forced_kind < 0 || forced_form < 0) && cs == hipStreamCaptureStatusNone &&
        !tune.count(bucket_of(e, f, m, k, n))) {
        if ((rc = tune_now(e, f, m, k, n, s))) return rc;
    }
    const Plan p = make_plan(e, f, m, k, n, choose_form(e, f, m, k, n), true);
    const int kind = supported_kind(choose_kind(p), p);
    if ((rc = ensure_workspace(p.a_bytes + p.b_bytes + p.p_bytes, s))) return rc;
    return exec_plan(p, kind, A->data, A->ld, B->data, B->ld, C->data, C->ld, s, acc);
}

}  // namespace gf2e

using namespace gf2e;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* gf2e_strerror(int code)
{
    switch (code) {
        case GF2E_OK: return "ok";
        case GF2E_EINVAL: return "invalid argument";
        case GF2E_EFIELD: return "e must be in 2..16 and f an irreducible polynomial of degree e";
        case GF2E_ESHAPE: return "matrix shapes or leading dimensions do not fit";
        case GF2E_EALIAS: return "output overlaps an input";
        case GF2E_ERANGE: return "an input entry is not an element of F_{2^e} (>= 2^e)";
        case GF2E_ENOMEM: return "workspace allocation failed or exceeds the limit";
        case GF2E_EDEVICE: return "HIP runtime error";
        case GF2E_EBUSY: return "request does not fit the memory budget now";
        case GF2E_ESINGULAR: return "triangular matrix has a zero on its diagonal";
        default: return "unknown error";
    }
}

int gf2e_field_check(int e, uint32_t f) { return field_ok(e, f) ? GF2E_OK : GF2E_EFIELD; }

int gf2e_num_products(int e, uint32_t f)
{
    if (!field_ok(e, f)) return GF2E_EFIELD;
    return make_plan(e, f, 1, 1, 1).T;
}

int gf2e_schedule(int e, uint32_t f, int* t, uint32_t* u, uint32_t* v, uint8_t* w, uint8_t* m)
{
    if (!field_ok(e, f)) return GF2E_EFIELD;
    const KernelSchedule S = kernel_schedule(e, schedule_id(e, f));
    const int T = S.t;
    if (t) *t = T;
    for (int s = 0; s < T; ++s) {
        if (u) u[s] = S.u[s];
        if (v) v[s] = S.v[s];
    }
    for (int d = 0; d < 2 * e - 1; ++d)
        for (int s = 0; s < T; ++s)
            if (w) w[d * T + s] = uint8_t((S.w[d] >> s) & 1u);  // zero for a field schedule
    if (m) {
        for (int c = 0; c < e; ++c)
            for (int s = 0; s < T; ++s) m[c * T + s] = 0;
        if (S.folded) {
            for (int s = 0; s < T; ++s)
                for (int c = 0; c < e; ++c)
                    if ((S.c[s] >> c) & 1u) m[c * T + s] = 1;
        } else {
            for (int d = 0; d < 2 * e - 1; ++d) {
                const uint32_t col = x_pow_mod(d, f, e);
                for (int c = 0; c < e; ++c)
                    if ((col >> c) & 1u)
                        for (int s = 0; s < T; ++s) m[c * T + s] ^= uint8_t((S.w[d] >> s) & 1u);
            }
        }
    }
    return GF2E_OK;
}

int gf2e_plane_geometry(int e, uint32_t f, int64_t m, int64_t k, int64_t n, gf2e_geometry* g)
{
    if (!g) return GF2E_EINVAL;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (m < 0 || k < 0 || n < 0) return GF2E_ESHAPE;
    const Plan p = make_plan(e, f, m, k, n);
    g->t = p.T;
    g->Mp = p.Mp;
    g->Np = p.Np;
    g->K64p = p.K64p;
    g->a_bytes = p.a_bytes;
    g->b_bytes = p.b_bytes;
    g->p_bytes = p.p_bytes;
    return GF2E_OK;
}

int gf2e_create(gf2e_ctx** out, int device, const gf2e_config* cfg)
{
    if (!out) return GF2E_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
        (void)hipGetLastError();
        return GF2E_EDEVICE;
    }
    DeviceGuard guard(device);
    Ctx* c = new (std::nothrow) Ctx();
    if (!c) return GF2E_ENOMEM;
    c->device = device;
    if (cfg) c->cfg = *cfg;
    else {
        c->cfg.kernel = GF2E_KERNEL_AUTO;
        c->cfg.autotune = 0;
        c->cfg.workspace_limit = 0;
    }
    if (c->cfg.kernel >= GEMM_NUM_KINDS) { delete c; return GF2E_EINVAL; }
    c->forced_kind = c->cfg.kernel >= 0 ? c->cfg.kernel : -1;
    if (const char* kenv = std::getenv("GF2E_KERNEL")) {
        for (int kk = 0; kk < GEMM_NUM_KINDS; ++kk)
            if (std::strcmp(kenv, gemm_name(kk)) == 0) c->forced_kind = kk;
    }
    if (hipMalloc(&c->d_err, sizeof(int)) != hipSuccess ||
        hipMemset(c->d_err, 0, sizeof(int)) != hipSuccess ||
        hipEventCreateWithFlags(&c->ws_done, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        if (c->d_err) (void)hipFree(c->d_err);
        delete c;
        return GF2E_EDEVICE;
    }
    c->load_tune_cache();
    // The no-allocation entry point's scratch array: its address on this
    // device, looked up once per device with the device current.
    if (!scratch_on(device)) {
        (void)hipFree(c->d_err);
        (void)hipEventDestroy(c->ws_done);
        delete c;
        return GF2E_EDEVICE;
    }
    *out = reinterpret_cast<gf2e_ctx*>(c);
    return GF2E_OK;
}

void gf2e_destroy(gf2e_ctx* handle)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return;
    DeviceGuard guard(c->device);
    (void)hipDeviceSynchronize();
    c->release_batches();
    if (c->ws) (void)hipFree(c->ws);
    if (c->aux) (void)hipFree(c->aux);
    for (auto& kv : c->ftabs) (void)hipFree(kv.second);
    if (c->pinned) (void)hipHostFree(c->pinned);
    if (c->side) (void)hipStreamDestroy(c->side);
    if (c->d_err) (void)hipFree(c->d_err);
    for (int st = 0; st < GF2E_NUM_STAGES; ++st)
        for (auto& pr : c->prof_pending[st]) {
            (void)hipEventDestroy(pr.first);
            (void)hipEventDestroy(pr.second);
        }
    for (hipEvent_t ev : c->event_pool) (void)hipEventDestroy(ev);
    if (c->ws_done) (void)hipEventDestroy(c->ws_done);
    delete c;
}

int gf2e_mul_async(gf2e_ctx* handle, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                   uint32_t f, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    int rc = validate_mul(A, B, C, e, f);
    if (rc) return rc;
    const int64_t m = A->rows, k = A->cols, n = B->cols;
    if (m == 0 || n == 0) return GF2E_OK;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    c->order_stream(s);
    if (k == 0) {
        if (launch_zero(C->data, m, n, C->ld, elem_bytes(e), s) != hipSuccess) return GF2E_EDEVICE;
        c->mark_used(s);
        return GF2E_OK;
    }
    rc = c->mul(e, f, A, B, C, s);
    c->mark_used(s);
    return rc;
}

int gf2e_mul_noalloc_async(gf2e_ctx* handle, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                           uint32_t f, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    int rc = validate_mul(A, B, C, e, f);
    if (rc) return rc;
    const int64_t m = A->rows, k = A->cols, n = B->cols;
    if (m == 0 || n == 0) return GF2E_OK;
    void* planes = scratch_known(c->device);
    if (!planes) return GF2E_EDEVICE;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (k == 0)
        return launch_zero(C->data, m, n, C->ld, elem_bytes(e), s) == hipSuccess ? GF2E_OK : GF2E_EDEVICE;
    // Form and kernel: forced, or tuned earlier, or the planner's default;
    // this entry point never tunes (tuning allocates its inputs).
    Plan p = make_plan(e, f, m, k, n, c->choose_form(e, f, m, k, n), true);
    if (p.a_bytes + p.b_bytes + p.p_bytes > GF2E_NOALLOC_MAX_BYTES) {
        p = make_plan(e, f, m, k, n, kFormSchedule, true);
        if (p.a_bytes + p.b_bytes + p.p_bytes > GF2E_NOALLOC_MAX_BYTES) return GF2E_ENOMEM;
    }
    const int kind = supported_kind(c->choose_kind(p), p);
    return c->exec_plan(p, kind, A->data, A->ld, B->data, B->ld, C->data, C->ld, s, false, planes);
}

int gf2e_sync(gf2e_ctx* handle, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    DeviceGuard guard(c->device);
    if (hipStreamSynchronize(static_cast<hipStream_t>(stream)) != hipSuccess) return GF2E_EDEVICE;
    int flag = 0;
    if (hipMemcpy(&flag, c->d_err, sizeof(int), hipMemcpyDeviceToHost) != hipSuccess)
        return GF2E_EDEVICE;
    if (flag) {
        const int zero = 0;
        if (hipMemcpy(c->d_err, &zero, sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
            return GF2E_EDEVICE;
        return (flag & 1) ? GF2E_ERANGE : GF2E_ESINGULAR;
    }
    return GF2E_OK;
}

int gf2e_mul(gf2e_ctx* handle, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e, uint32_t f)
{
    int rc = gf2e_mul_async(handle, A, B, C, e, f, nullptr);
    if (rc) return rc;
    return gf2e_sync(handle, nullptr);
}

int gf2e_slice_a(gf2e_ctx* handle, const gf2e_mat* A, int e, uint32_t f, uint64_t* planes, int64_t Mp,
                 int64_t K64p, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !planes) return GF2E_EINVAL;
    int rc = check_mat(A);
    if (rc) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (Mp < A->rows || Mp % kRowAlign || K64p < kwords_padded(A->cols) || K64p % 4) return GF2E_ESHAPE;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageTimer t(c, GF2E_STAGE_SLICE_A, s);
    return launch_slice_rows(e, schedule_id(e, f), A->data, A->ld, A->rows, A->cols, planes, Mp, K64p,
                             c->d_err, s) ==
                   hipSuccess
               ? GF2E_OK
               : GF2E_EDEVICE;
}

int gf2e_slice_b(gf2e_ctx* handle, const gf2e_mat* B, int e, uint32_t f, uint64_t* planes, int64_t Np,
                 int64_t K64p, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !planes) return GF2E_EINVAL;
    int rc = check_mat(B);
    if (rc) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (Np < B->cols || Np % kRowAlign || K64p < kwords_padded(B->rows) || K64p % 4) return GF2E_ESHAPE;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageTimer t(c, GF2E_STAGE_SLICE_B, s);
    return launch_slice_cols(e, schedule_id(e, f), B->data, B->ld, B->rows, B->cols, planes, Np, K64p,
                             c->d_err, s) ==
                   hipSuccess
               ? GF2E_OK
               : GF2E_EDEVICE;
}

int gf2e_plane_products(gf2e_ctx* handle, int kernel, int t, const uint64_t* a_planes,
                        const uint64_t* b_planes, uint64_t* p_planes, int64_t m, int64_t n,
                        int64_t Mp, int64_t Np, int64_t K64p, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !a_planes || !b_planes || !p_planes || t <= 0 || t > kMaxT) return GF2E_EINVAL;
    // the fp4 kernels move operand rows in 16-byte pairs straight into LDS
    auto aligned16 = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
    if (!aligned16(a_planes) || !aligned16(b_planes) || !aligned16(p_planes)) return GF2E_EINVAL;
    if (m < 0 || n < 0 || Mp < m || Np < n || Mp % kRowAlign || Np % kRowAlign || K64p <= 0 ||
        K64p % 4)
        return GF2E_ESHAPE;
    if (kernel < GF2E_KERNEL_AUTO || kernel >= GEMM_NUM_KINDS) return GF2E_EINVAL;
    const int kind = kernel >= 0 ? kernel : default_kind(t, m, n);
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageTimer tm(c, GF2E_STAGE_PRODUCTS, s);
    return launch_gemm(kind, t, a_planes, b_planes, p_planes, m, n, Mp, Np, K64p, s) == hipSuccess
               ? GF2E_OK
               : GF2E_EDEVICE;
}

int gf2e_combine(gf2e_ctx* handle, int e, uint32_t f, const uint64_t* p_planes, int64_t Mp,
                 int64_t Np, gf2e_mat* C, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || !p_planes) return GF2E_EINVAL;
    int rc = check_mat(C);
    if (rc) return rc;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (Mp < C->rows || Np < C->cols || Mp % kRowAlign || Np % kRowAlign) return GF2E_ESHAPE;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    StageTimer t(c, GF2E_STAGE_COMBINE, s);
    return launch_combine(e, schedule_id(e, f), f, p_planes, Mp * (Np / 64), Np / 64, C->rows, C->cols, C->data,
                          C->ld, s) ==
                   hipSuccess
               ? GF2E_OK
               : GF2E_EDEVICE;
}

int gf2e_kernel_count(void) { return GEMM_NUM_KINDS; }

const char* gf2e_kernel_name(int kernel) { return gemm_name(kernel); }

int gf2e_set_kernel(gf2e_ctx* handle, int kernel)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || kernel < GF2E_KERNEL_AUTO || kernel >= GEMM_NUM_KINDS) return GF2E_EINVAL;
    c->forced_kind = kernel;
    return GF2E_OK;
}

int gf2e_chosen_kernel(gf2e_ctx* handle, int e, uint32_t f, int64_t m, int64_t k, int64_t n)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    const Plan p = make_plan(e, f, m, k, n, c->choose_form(e, f, m, k, n), true);
    return supported_kind(c->choose_kind(p), p);
}

int gf2e_set_form(gf2e_ctx* handle, int form)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || form < GF2E_FORM_AUTO || form >= kNumForms) return GF2E_EINVAL;
    c->forced_form = form;
    return GF2E_OK;
}

int gf2e_chosen_form(gf2e_ctx* handle, int e, uint32_t f, int64_t m, int64_t k, int64_t n)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    return c->choose_form(e, f, m, k, n);
}

int gf2e_tune(gf2e_ctx* handle, int e, uint32_t f, int64_t m, int64_t k, int64_t n, void* stream)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    if (!field_ok(e, f)) return GF2E_EFIELD;
    if (m <= 0 || k <= 0 || n <= 0) return GF2E_ESHAPE;
    DeviceGuard guard(c->device);
    hipStream_t s = static_cast<hipStream_t>(stream);
    c->order_stream(s);
    int rc = c->tune_now(e, f, m, k, n, s);
    c->mark_used(s);
    return rc;
}

int gf2e_profile(gf2e_ctx* handle, int enable)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    c->prof = enable != 0;
    return GF2E_OK;
}

int gf2e_profile_read(gf2e_ctx* handle, int stage, double* total_ms, int64_t* launches)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c || stage < 0 || stage >= GF2E_NUM_STAGES) return GF2E_EINVAL;
    DeviceGuard guard(c->device);
    for (auto& pr : c->prof_pending[stage]) {
        if (hipEventSynchronize(pr.second) != hipSuccess) return GF2E_EDEVICE;
        float ms = 0;
        if (hipEventElapsedTime(&ms, pr.first, pr.second) != hipSuccess) return GF2E_EDEVICE;
        c->prof_ms[stage] += ms;
        c->prof_n[stage] += 1;
        c->event_pool.push_back(pr.first);
        c->event_pool.push_back(pr.second);
    }
    c->prof_pending[stage].clear();
    if (total_ms) *total_ms = c->prof_ms[stage];
    if (launches) *launches = c->prof_n[stage];
    return GF2E_OK;
}

int gf2e_profile_reset(gf2e_ctx* handle)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    if (!c) return GF2E_EINVAL;
    for (int st = 0; st < GF2E_NUM_STAGES; ++st) {
        double ms;
        int64_t n;
        int rc = gf2e_profile_read(handle, st, &ms, &n);
        if (rc) return rc;
        c->prof_ms[st] = 0;
        c->prof_n[st] = 0;
    }
    return GF2E_OK;
}

int64_t gf2e_workspace_bytes(gf2e_ctx* handle)
{
    Ctx* c = reinterpret_cast<Ctx*>(handle);
    return c ? c->ws_bytes : 0;
}

}  // extern "C"
