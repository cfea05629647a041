// Host-side context of the library (the object behind gf2e_ctx*).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <memory>
#include <utility>
#include <vector>

#include "gf2e.h"
#include "gf2e_internal.hpp"

namespace gf2e {

struct DeviceGuard {
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
    DeviceGuard(const DeviceGuard&) = delete;
    DeviceGuard& operator=(const DeviceGuard&) = delete;

private:
    int prev_ = -1;
};

// How the plain path computes one product.  kFormSchedule: T GF(2) plane
// products of the bilinear schedule (Section 5), then recombination and
// reduction.  kFormAlpha: one GF(2) product of the e A-planes (m x ek) with
// the ek x en matrix of the planes of alpha^i B (reduction folded in), then
// clinging of its e result planes; e^2 bit products per element product
// instead of T, but a single larger launch and no recombination.
enum Form : int { kFormSchedule = 0, kFormAlpha = 1, kNumForms = 2 };

// Sizes of one product's planes (see the layout notes in gf2e_internal.hpp).
struct Plan {
    int e = 0, T = 0;
    int form = kFormSchedule;
    int sid = -1;  // schedule: -1 Karatsuba + run-time reduction, >= 0 field schedule, -2 identity
    uint32_t f = 0;
    int64_t m = 0, k = 0, n = 0;
    int64_t Mp = 0, Np = 0, K64p = 0;
    // Geometry of the product launch: gT planes of an m x gn result with
    // padded width gNp and gK64p words of k.
    int gT = 0;
    int64_t gn = 0, gNp = 0, gK64p = 0;
    int64_t a_bytes = 0, b_bytes = 0, p_bytes = 0;
};

int elem_bytes(int e);
bool field_ok(int e, uint32_t f);
int check_mat(const gf2e_mat* M);
bool overlaps(const gf2e_mat* X, const gf2e_mat* Y, int esz);
int validate_mul(const gf2e_mat* A, const gf2e_mat* B, const gf2e_mat* C, int e, uint32_t f);
// Schedule for (e, f): the field schedule if one is compiled in (and not
// disabled with GF2E_SCHEDULE=karatsuba), else -1.
int schedule_id(int e, uint32_t f);
// short_k: the plain path's plans, where k <= 128 takes K64p = 2 (run by the
// kernel with 128-bit stages); the stage entry points, batches and served
// requests keep K64p a multiple of 4.
Plan make_plan(int e, uint32_t f, int64_t m, int64_t k, int64_t n, int form = kFormSchedule, bool short_k = false);
int default_kind(int T, int64_t m, int64_t n);
bool kind_supports(int kind, const Plan& p);
int supported_kind(int kind, const Plan& p);  // kind, or a kernel that can run plan p

struct BatchGraph;  // defined in batch.hip

struct DevTables {
    const uint16_t* exp;
    const uint32_t* log;
};

struct Ctx {
    int device = 0;
    gf2e_config cfg{};
    int forced_kind = -1;
    int forced_form = -1;  // GF2E_FORM_AUTO
    int* d_err = nullptr;  // sticky device flag: an entry >= 2^e was seen

    void* ws = nullptr;  // plane workspace of the plain path
    int64_t ws_bytes = 0;
    hipEvent_t ws_done = nullptr;
    hipStream_t last_stream = nullptr;
    bool have_last = false;

    bool prof = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending[GF2E_NUM_STAGES];
    double prof_ms[GF2E_NUM_STAGES] = {};
    int64_t prof_n[GF2E_NUM_STAGES] = {};
    std::vector<hipEvent_t> event_pool;

    // size bucket -> tuned choice: product kernel | (form << 8)
    std::map<uint64_t, int> tune;

    std::vector<BatchGraph*> batches;  // cached batched graphs (owned), least recent first
    int64_t batch_threshold = 384;     // min(m, n) at which a product takes 256x256 tiles
    int64_t batch_builds = 0;
    bool batch_fused = true;           // fused recombination for the 128x128 class (e <= kFusedMaxE)
    int64_t last_batch_items[3] = {0, 0, 0};
    int64_t last_batch_arena = 0;

    hipEvent_t get_event();
    void order_stream(hipStream_t s);
    void mark_used(hipStream_t s);
    int ensure_workspace(int64_t bytes, hipStream_t s);
    // Form and product kernel for a product (forced, tuned or default).
    int choose_form(int e, uint32_t f, int64_t m, int64_t k, int64_t n);
    int choose_kind(const Plan& p);
    // Times the product kernels for the plans of both forms and then both
    // whole pipelines (on inputs it allocates), and records the faster.
    int tune_now(int e, uint32_t f, int64_t m, int64_t k, int64_t n, hipStream_t s);
    void load_tune_cache();
    void save_tune_entry(uint64_t key, int choice);
    // C = A*B, or C += A*B with acc (shapes already validated).  C may
    // overlap B: B is sliced into its planes before the last kernel writes
    // C, all in stream order (the library's own callers use that).
    int mul(int e, uint32_t f, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, hipStream_t s,
            bool acc = false);
    // Launches the stages of plan p with product kernel kind; planes in
    // `planes` (a_bytes + b_bytes + p_bytes of device memory), else in ws.
    int exec_plan(const Plan& p, int kind, const void* A, int64_t lda, const void* B, int64_t ldb,
                  void* C, int64_t ldc, hipStream_t s, bool acc = false, void* planes = nullptr);

    // Buffers of the triangular solver (inverted diagonal blocks) and of
    // the echelon driver, kept apart from the product workspace.
    void* aux = nullptr;
    int64_t aux_bytes = 0;
    int ensure_aux(int64_t bytes, hipStream_t s);
    int trsm(int lower, int unit, const gf2e_mat* T, gf2e_mat* B, int e, uint32_t f, hipStream_t s);

    // Log/antilog tables of F_2[x]/<f> in device memory, built on first use
    // and kept per (e, f): exp[4q + 1] (uint16, g^i for i < 2q, then zeros)
    // and log[q + 1] (uint32, log 0 = 2q), so that exp[log a + log b] = a*b.
    std::map<uint64_t, void*> ftabs;
    DevTables field_tables(int e, uint32_t f);  // {nullptr, nullptr} on failure
    // Mapped, coherent host buffer that the final pivot-search kernel of an
    // echelon panel writes its state into; the host reads it once the launch
    // has completed (no copy launch in between).
    void* pinned = nullptr;
    size_t pinned_bytes = 0;
    void* ensure_pinned(size_t bytes);
    // A second stream of the context (default priority, created on first
    // use): the echelon driver runs the next panel's pivot search on it.
    hipStream_t side = nullptr;
    hipStream_t side_stream();
    // Row echelon form in place (reduced when full); host-synchronous.  With
    // ple (full = 0) it also returns the PLE decomposition's L (m x min(m, n),
    // device) and P (m row indices, host).
    struct PleOut {
        gf2e_mat* L;
        int64_t* P;
    };
    int echelon(gf2e_mat* A, int e, uint32_t f, int full, int64_t* rank, int64_t* pivots, hipStream_t s,
                PleOut* ple = nullptr);
    void release_batches();
};

// Brackets one stage launch with HIP events when the context's timers are on.
class StageTimer {
public:
    StageTimer(Ctx* c, int stage, hipStream_t s, bool on = true);
    ~StageTimer();

private:
    Ctx* ctx_;
    int stage_;
    hipStream_t s_;
    hipEvent_t a_ = nullptr, b_ = nullptr;
};

}  // namespace gf2e
