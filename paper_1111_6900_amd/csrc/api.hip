// C ABI of the library: validation, planning, workspace, stage launches,
// autotuning and stage timers.  See include/gf2e.h for the contract.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
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

bool field_ok(int e, uint32_t f) { return e >= 2 && e <= kMaxE && is_irreducible(e, f); }

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

Plan make_plan(int e, uint32_t f, int64_t m, int64_t k, int64_t n)
{
    Plan p{};
    p.e = e;
    p.f = f;
    p.sid = schedule_id(e, f);
    p.T = p.sid >= 0 ? kFieldSchedules[p.sid].t : best_count(e);
    p.m = m; p.k = k; p.n = n;
    p.Mp = round_up(std::max<int64_t>(m, 1), kRowAlign);
    p.Np = round_up(std::max<int64_t>(n, 1), kRowAlign);
    p.K64p = kwords_padded(std::max<int64_t>(k, 1));
    p.a_bytes = int64_t(p.T) * p.K64p * p.Mp * 8;
    p.b_bytes = int64_t(p.T) * p.K64p * p.Np * 8;
    p.p_bytes = int64_t(p.T) * p.Mp * (p.Np / 64) * 8;
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

StageTimer::StageTimer(Ctx* c, int stage, hipStream_t s) : ctx_(c), stage_(stage), s_(s)
{
    if (!ctx_->prof) return;
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
    const bool fp4 = kind == GEMM_FP4_256x256_W8 || kind == GEMM_FP4_128x128;
    return !fp4 || p.K64p * 64 <= (int64_t(1) << 24);
}

int Ctx::choose_kind(const Plan& p)
{
    if (forced_kind >= 0) return forced_kind;
    auto it = tune.find(bucket_key(p.T, p.m, p.k, p.n));
    if (it != tune.end()) return it->second;
    return default_kind(p.T, p.m, p.n);
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
        int kind = -1;
        if (std::sscanf(line, "{\"arch\": \"gfx950\", \"key\": %llu, \"kernel\": %d", &key, &kind) == 2 &&
            kind >= 0 && kind < GEMM_NUM_KINDS)
            tune[key] = kind;
    }
    std::fclose(fp);
}

void Ctx::save_tune_entry(uint64_t key, int kind)
{
    const char* path = std::getenv("GF2E_TUNE_CACHE");
    if (!path) return;
    FILE* fp = std::fopen(path, "a");
    if (!fp) return;
    std::fprintf(fp, "{\"arch\": \"gfx950\", \"key\": %llu, \"kernel\": %d, \"name\": \"%s\"}\n",
                 static_cast<unsigned long long>(key), kind, gemm_name(kind));
    std::fclose(fp);
}

int Ctx::tune_now(const Plan& p, hipStream_t s)
{
    int rc = ensure_workspace(p.a_bytes + p.b_bytes + p.p_bytes, s);
    if (rc) return rc;
    uint64_t* Apl = static_cast<uint64_t*>(ws);
    uint64_t* Bpl = Apl + p.a_bytes / 8;
    uint64_t* P = Bpl + p.b_bytes / 8;
    hipEvent_t e0 = get_event(), e1 = get_event();
    if (!e0 || !e1) return GF2E_EDEVICE;
    // Two rounds over all candidates (the first also brings the clocks up);
    // each candidate keeps its best round.
    float best_ms[GEMM_NUM_KINDS];
    for (int kind = 0; kind < GEMM_NUM_KINDS; ++kind) best_ms[kind] = -1.f;
    const bool verbose = std::getenv("GF2E_TUNE_LOG") != nullptr;
    for (int round = 0; round < 2; ++round)
        for (int kind = 0; kind < GEMM_NUM_KINDS; ++kind) {
            if (launch_gemm(kind, p.T, Apl, Bpl, P, p.m, p.n, p.Mp, p.Np, p.K64p, s) != hipSuccess) {
                (void)hipGetLastError();
                continue;  // not applicable to this shape
            }
            const int reps = 3;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps; ++r)
                (void)launch_gemm(kind, p.T, Apl, Bpl, P, p.m, p.n, p.Mp, p.Np, p.K64p, s);
            (void)hipEventRecord(e1, s);
            if (hipEventSynchronize(e1) != hipSuccess) return GF2E_EDEVICE;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= reps;
            if (verbose)
                std::fprintf(stderr, "[gf2e tune] T=%d m=%lld k=%lld n=%lld round %d %s %.4f ms\n", p.T,
                             static_cast<long long>(p.m), static_cast<long long>(p.k),
                             static_cast<long long>(p.n), round, gemm_name(kind), ms);
            if (best_ms[kind] < 0 || ms < best_ms[kind]) best_ms[kind] = ms;
        }
    int best = -1;
    for (int kind = 0; kind < GEMM_NUM_KINDS; ++kind)
        if (best_ms[kind] >= 0 && (best < 0 || best_ms[kind] < best_ms[best])) best = kind;
    event_pool.push_back(e0);
    event_pool.push_back(e1);
    if (best < 0) return GF2E_EDEVICE;
    const uint64_t key = bucket_key(p.T, p.m, p.k, p.n);
    tune[key] = best;
    save_tune_entry(key, best);
    return GF2E_OK;
}

int Ctx::run_plan(const Plan& p, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, uint32_t f,
                  hipStream_t s)
{
    int rc = ensure_workspace(p.a_bytes + p.b_bytes + p.p_bytes, s);
    if (rc) return rc;
    if (cfg.autotune && forced_kind < 0 && !tune.count(bucket_key(p.T, p.m, p.k, p.n))) {
        if ((rc = tune_now(p, s))) return rc;
    }
    int kind = choose_kind(p);
    if (!kind_supports(kind, p)) kind = GEMM_MFMA_256x256_W8;  // f32 counts would not be exact
    uint64_t* Apl = static_cast<uint64_t*>(ws);
    uint64_t* Bpl = Apl + p.a_bytes / 8;
    uint64_t* P = Bpl + p.b_bytes / 8;
    hipError_t err;
    {
        StageTimer t(this, GF2E_STAGE_SLICE_A, s);
        err = launch_slice_rows(p.e, p.sid, A->data, A->ld, p.m, p.k, Apl, p.Mp, p.K64p, d_err, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    {
        StageTimer t(this, GF2E_STAGE_SLICE_B, s);
        err = launch_slice_cols(p.e, p.sid, B->data, B->ld, p.k, p.n, Bpl, p.Np, p.K64p, d_err, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    {
        StageTimer t(this, GF2E_STAGE_PRODUCTS, s);
        err = launch_gemm(kind, p.T, Apl, Bpl, P, p.m, p.n, p.Mp, p.Np, p.K64p, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    {
        StageTimer t(this, GF2E_STAGE_COMBINE, s);
        err = launch_combine(p.e, p.sid, f, P, p.Mp, p.Np / 64, p.m, p.n, C->data, C->ld, s);
    }
    if (err != hipSuccess) return GF2E_EDEVICE;
    return GF2E_OK;
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
        case GF2E_EFIELD: return "e must be in 2..10 and f an irreducible polynomial of degree e";
        case GF2E_ESHAPE: return "matrix shapes or leading dimensions do not fit";
        case GF2E_EALIAS: return "output overlaps an input";
        case GF2E_ERANGE: return "an input entry is not an element of F_{2^e} (>= 2^e)";
        case GF2E_ENOMEM: return "workspace allocation failed or exceeds the limit";
        case GF2E_EDEVICE: return "HIP runtime error";
        case GF2E_EBUSY: return "request does not fit the memory budget now";
        default: return "unknown error";
    }
}

int gf2e_field_check(int e, uint32_t f) { return field_ok(e, f) ? GF2E_OK : GF2E_EFIELD; }

int gf2e_num_products(int e, uint32_t f)
{
    if (!field_ok(e, f)) return GF2E_EFIELD;
    return make_plan(e, f, 1, 1, 1).T;
}

int gf2e_schedule(int e, uint32_t f, int* t, uint32_t* u, uint32_t* v, uint64_t* w, uint64_t* m)
{
    if (!field_ok(e, f)) return GF2E_EFIELD;
    const KernelSchedule S = kernel_schedule(e, schedule_id(e, f));
    if (t) *t = S.t;
    for (int s = 0; s < S.t; ++s) {
        if (u) u[s] = S.u[s];
        if (v) v[s] = S.v[s];
    }
    for (int d = 0; d < 2 * e - 1; ++d)
        if (w) w[d] = S.w[d];  // zero for a field schedule (reduction folded in)
    if (m) {
        for (int c = 0; c < e; ++c) m[c] = 0;
        if (S.folded) {
            for (int s = 0; s < S.t; ++s)
                for (int c = 0; c < e; ++c)
                    if ((S.c[s] >> c) & 1u) m[c] |= uint64_t(1) << s;
        } else {
            for (int d = 0; d < 2 * e - 1; ++d) {
                const uint32_t col = x_pow_mod(d, f, e);
                for (int c = 0; c < e; ++c)
                    if ((col >> c) & 1u) m[c] ^= S.w[d];
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
    const Plan p = make_plan(e, f, m, k, n);
    rc = c->run_plan(p, A, B, C, f, s);
    c->mark_used(s);
    return rc;
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
        return GF2E_ERANGE;
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
    return launch_combine(e, schedule_id(e, f), f, p_planes, Mp, Np / 64, C->rows, C->cols, C->data, C->ld,
                          s) ==
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
    return c->choose_kind(make_plan(e, f, m, k, n));
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
    int rc = c->tune_now(make_plan(e, f, m, k, n), s);
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
