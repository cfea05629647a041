/*
 * gf2e.h -- C ABI of the MI355X (gfx950) library for dense matrix
 * multiplication over F_{2^e}, 2 <= e <= 16.
 *
 * What is computed: C = A * B with A m x k and B k x n over
 * F_{2^e} = F_2[x]/<f> (M4RIE paper, Section 2 for the field and the element
 * encoding, Section 4 Algorithm 1 for the product).  An element is the
 * polynomial sum a_i x^i, stored as the integer sum a_i 2^i: one uint8_t per
 * element when e <= 8, one uint16_t when e is 9..16.  f is the full
 * polynomial with bit e set (x^2+x+1 = 0x7, x^8+x^4+x^3+x^2+1 = 0x11D) and
 * must be irreducible of degree e.
 *
 * How: the Bradshaw-Boothby reduction of Section 5.  Each operand is sliced
 * into e GF(2) bit-planes (Section 3.2), the Karatsuba schedule forms t(e)
 * products of plane sums over GF(2) (t = 3, 6, 9, 15, 18, 24, 27, 36, 45, 51,
 * 54, 66, 72, 78, 81 for e = 2..16; fewer for the fields with a schedule
 * compiled in), the products are recombined into the 2e-1 coefficients of the
 * polynomial product, reduced modulo f, and clung back into elements.  Every
 * step runs as a HIP kernel on the device; the result is exact and unique.
 *
 * Conventions for every entry point below:
 *   - matrix data pointers are DEVICE pointers, row-major, with a leading
 *     dimension `ld` counted in elements (ld >= cols);
 *   - the caller owns A, B and C; the library never frees them.  A context
 *     owns its workspace (bit-planes), tuning cache and graph cache;
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream);
 *   - errors are returned as status codes; nothing is thrown or aborted
 *     across the ABI.  Host-detectable errors are returned before anything is
 *     enqueued.  Entries >= 2^e are detected on the device and reported by
 *     the next gf2e_sync (or by the blocking call) as GF2E_ERANGE; the
 *     offending product's output is then unspecified;
 *   - C must not overlap A or B (GF2E_EALIAS);
 *   - m = 0 or n = 0 is a no-op; k = 0 sets C to zero (the empty sum);
 *   - a context may be used from one host thread at a time.  Calls on one
 *     context are ordered: a call on a different stream than the previous one
 *     first waits for that call to finish using the workspace.
 */
#ifndef GF2E_H
#define GF2E_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    GF2E_OK = 0,
    GF2E_EINVAL = -1,  /* null pointer, bad argument */
    GF2E_EFIELD = -2,  /* e outside 2..16, or f not an irreducible polynomial of degree e */
    GF2E_ESHAPE = -3,  /* inner/outer dimensions disagree, ld < cols, negative size */
    GF2E_EALIAS = -4,  /* C overlaps A or B */
    GF2E_ERANGE = -5,  /* an input entry is >= 2^e (found on the device) */
    GF2E_ENOMEM = -6,  /* workspace could not be allocated or exceeds the limit */
    GF2E_EDEVICE = -7, /* a HIP runtime call failed */
    GF2E_EBUSY = -8,   /* serving: request does not fit the memory budget right now */
    GF2E_ESINGULAR = -9 /* triangular solve: a zero on the diagonal (found on the device) */
};

typedef struct gf2e_ctx gf2e_ctx;

typedef struct {
    void* data;      /* device pointer to element (0, 0) */
    int64_t rows;
    int64_t cols;
    int64_t ld;      /* elements between the starts of consecutive rows */
} gf2e_mat;

/* Product-kernel choice (gf2e_config.kernel, gf2e_set_kernel). */
enum {
    GF2E_KERNEL_AUTO = -1,        /* autotuned (or planner default) per size bucket */
    GF2E_KERNEL_MFMA_256 = 0,     /* int8 MFMA, 256x256 tiles */
    GF2E_KERNEL_MFMA_128 = 1,     /* int8 MFMA, 128x128 tiles */
    GF2E_KERNEL_MFMA_256x128 = 2, /* int8 MFMA, 256x128 tiles */
    GF2E_KERNEL_MFMA_64 = 3,      /* int8 MFMA, 64x64 tiles */
    GF2E_KERNEL_VALU_128 = 4,     /* AND/XOR on packed words, 128x128 tiles */
    GF2E_KERNEL_MFMA_256_W8 = 5,  /* int8 MFMA, 256x256 tiles, 8 waves of 128x64 */
    GF2E_KERNEL_FP4_256_W8 = 6,   /* fp4 MFMA (0/1 nibbles, exact count in f32), 256x256, k <= 2^23 */
    GF2E_KERNEL_FP4_128 = 7,      /* fp4 MFMA, 128x128 tiles, k <= 2^23 */
    GF2E_KERNEL_FP4_128_PLANES = 8 /* as FP4_128 with 128-bit k stages and several planes per
                                      workgroup; the only kernel for products with k <= 128,
                                      which the plain path pads to 128 bits instead of 256 */
};

typedef struct {
    int kernel;              /* GF2E_KERNEL_*; GF2E_KERNEL_AUTO by default */
    int autotune;            /* 1: time every candidate kernel on first use of a size bucket */
    int64_t workspace_limit; /* bytes of plane workspace allowed; 0 = no limit */
} gf2e_config;

/* Context on HIP device `device`.  cfg may be NULL (defaults).  The tuning
 * cache is read from / written to the file named by GF2E_TUNE_CACHE if set. */
int gf2e_create(gf2e_ctx** ctx, int device, const gf2e_config* cfg);
void gf2e_destroy(gf2e_ctx* ctx);

/* C = A * B over F_{2^e} (Section 5 reduction), enqueued on `stream`. */
int gf2e_mul_async(gf2e_ctx* ctx, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                   uint32_t f, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as gf2e_mul_async, bit for bit, computed with no hipMalloc, hipFree
 * or event creation.  Its bit-planes live in a fixed device array of
 * GF2E_NOALLOC_MAX_BYTES bytes, one per GPU, which the library holds until
 * the process ends (its address is looked up by gf2e_create).  Products whose
 * planes do not fit return GF2E_ENOMEM before anything is enqueued (for
 * e = 8 that allows m = k = n = 2048; the plane bytes of a shape are
 * gf2e_plane_geometry's a_bytes + b_bytes + p_bytes).  It never autotunes:
 * it uses the context's forced or already tuned kernel, else the default.
 * Every call on one GPU shares that array, so calls that overlap in time on
 * one GPU (different streams, threads or contexts) race and give wrong
 * results: order them on one stream or synchronise between them.  Entries
 * >= 2^e are reported by gf2e_sync like gf2e_mul_async's. */
#define GF2E_NOALLOC_MAX_BYTES ((int64_t)64 << 20)
int gf2e_mul_noalloc_async(gf2e_ctx* ctx, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                           uint32_t f, void* stream);

/* Many independent products C[p] = A[p] * B[p] over F_{2^e[p]} (f[p]), of
 * any shapes and fields, enqueued on `stream` as one captured HIP graph:
 * grouped slicing, one persistent grouped launch of all GF(2) plane
 * products per tile-size class, grouped combining.  After slicing every
 * product is t(e) GF(2) products of the same shape (Section 5), so one
 * e-agnostic product kernel serves the whole batch.  A, B, C, e, f are
 * host arrays of `count` entries; outputs must not overlap any input of
 * their own product nor each other.  The graph, its plane arena and its
 * work list are built on the first call with a given set of descriptors
 * (pointers, shapes, fields) and replayed by later identical calls, which
 * read the current contents of the same buffers.  Results are bit-identical
 * to gf2e_mul on each product. */
int gf2e_mul_batched(gf2e_ctx* ctx, int count, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C,
                     const int* e, const uint32_t* f, void* stream);

/* Products with min(m, n) >= min_dim take 256x256 tiles in a batch, the rest
 * 128x128 (default 384). */
int gf2e_set_batch_threshold(gf2e_ctx* ctx, int64_t min_dim);
/* on = 1 (the default): products of the 128x128 class with e <= 10 and
 * k <= 2^23 run fused, one work item per tile covering all t(e) planes, whose
 * epilogue folds each plane's parity words into the e result planes (the
 * recombination and reduction of Section 5 as one merged map) and clings
 * them to C; they write no product planes and skip the combining pass.
 * on = 0: every product writes its planes and is combined afterwards.
 * Results are the same either way.  GF2E_EINVAL for other values. */
int gf2e_set_batch_fusion(gf2e_ctx* ctx, int on);
/* Autotune the threshold and the fusion: build and time the batch for each
 * candidate pair and keep the fastest (the batch is computed several times). */
int gf2e_tune_batched(gf2e_ctx* ctx, int count, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C,
                      const int* e, const uint32_t* f, void* stream);

typedef struct {
    int64_t items_large, items_small; /* work items of the last batch, per tile class */
    int64_t arena_bytes;              /* plane arena of the last batch */
    int graphs_cached;
    int64_t graph_builds;
    int64_t threshold;
    int64_t items_fused; /* work items of the last batch in the fused class */
    int fusion;          /* the context's fusion setting */
} gf2e_batch_stats;
int gf2e_batch_info(gf2e_ctx* ctx, gf2e_batch_stats* out);

/* ---- Serving ------------------------------------------------------------
 * A request loop with continuous batching.  A scheduler thread admits
 * submitted products in arrival order while their bit-plane footprint fits
 * `memory_budget` bytes of device memory and a descriptor slot is free,
 * slices them into planes that stay resident until the request completes,
 * and runs iterations of the persistent plane-product kernel over the tiles
 * of every admitted request (at most `quantum_macs` bit-MACs per iteration),
 * so requests that arrive while others are on the GPU share its launches.
 * When the oldest waiting request does not fit the free memory, later
 * requests that fit may be admitted ahead of it, at most `bypass_limit`
 * times for each oldest request (0: strict arrival order).  Results are
 * identical to gf2e_mul of the same product.
 *
 * Input readiness: submit records an event on `stream` (a hipStream_t as
 * void*, NULL = the null stream), and the server's own stream waits for that
 * event before it reads A and B, so the inputs may still be being written by
 * work enqueued on `stream` before the call.  A, B, C must stay valid, and
 * A and B unchanged, until the request is waited for; C is complete when
 * gf2e_server_wait returns (or poll reports done). */
typedef struct gf2e_server gf2e_server;

typedef struct {
    int64_t memory_budget;           /* device bytes for resident planes (admission limit) */
    int max_inflight;                /* admitted requests at once (1..4096) */
    int64_t quantum_macs;            /* plane-product bit-MACs per iteration; 0 = no limit */
    int64_t max_items_per_iteration; /* tile items per iteration; 0 = 262144 */
    int bypass_limit;                /* admissions past a waiting oldest request (>= 0) */
} gf2e_server_config;

typedef struct {
    int64_t t_submit_ns; /* times since the server (or run_trace call) started */
    int64_t t_admit_ns;
    int64_t t_done_ns;   /* when the scheduler saw the completion event */
    int status;          /* GF2E_OK, GF2E_ERANGE, ... */
} gf2e_req_times;

typedef struct {
    int64_t completed, iterations, element_macs, peak_arena_bytes;
    int peak_inflight;
    int64_t memory_waits;      /* requests that found the memory budget full at least once */
    int64_t bypass_admissions; /* admissions ahead of an older request waiting for memory */
    int64_t shared_iterations; /* iterations holding tiles of two or more requests */
    int max_iteration_requests; /* most requests with tiles in one iteration */
} gf2e_server_counters;

int gf2e_server_create(gf2e_ctx* ctx, const gf2e_server_config* cfg, gf2e_server** out);
/* Drains every submitted request, then frees the server. */
void gf2e_server_destroy(gf2e_server* srv);
/* Validates and queues a request (never blocks on the GPU).  GF2E_EBUSY: its
 * footprint exceeds the whole budget, so it could never be admitted. */
int gf2e_server_submit(gf2e_server* srv, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                       uint32_t f, void* stream, uint64_t* ticket);
int gf2e_server_poll(gf2e_server* srv, uint64_t ticket, int* done, gf2e_req_times* times);
/* Blocks until the request is done; returns its status and forgets it. */
int gf2e_server_wait(gf2e_server* srv, uint64_t ticket, gf2e_req_times* times);
int gf2e_server_stats(gf2e_server* srv, gf2e_server_counters* out);
/* Open-loop driver: submits request i at arrival_s[i] seconds after the call
 * starts (inputs ordered after `stream` as in submit), then waits for all;
 * out[i] gets times relative to that start. */
int gf2e_server_run_trace(gf2e_server* srv, int count, const gf2e_mat* A, const gf2e_mat* B,
                          gf2e_mat* C, const int* e, const uint32_t* f, const double* arrival_s,
                          void* stream, gf2e_req_times* out);

/* Blocking form: enqueue on the null stream, wait, report device errors. */
int gf2e_mul(gf2e_ctx* ctx, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
             uint32_t f);

/* Wait for `stream`; return GF2E_ERANGE (once) if any call enqueued since
 * the previous sync found an entry >= 2^e, else GF2E_ESINGULAR (once) if a
 * triangular solve found a zero on its diagonal, else GF2E_OK. */
int gf2e_sync(gf2e_ctx* ctx, void* stream);

/* C += A * B over F_{2^e} (the accumulating form of gf2e_mul_async; the
 * combine step adds to C instead of replacing it).  Same rules as
 * gf2e_mul_async; k = 0 leaves C unchanged. */
int gf2e_mul_add_async(gf2e_ctx* ctx, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e,
                       uint32_t f, void* stream);
int gf2e_mul_add(gf2e_ctx* ctx, const gf2e_mat* A, const gf2e_mat* B, gf2e_mat* C, int e, uint32_t f);

/* Triangular solving with matrices (Section 4.3): B <- T^{-1} B, where T is
 * an m x m upper (lower = 0) or lower (lower = 1) triangular matrix and B is
 * m x n.  Only T's triangle is read; unit = 1 takes its diagonal as ones
 * (the diagonal entries are then not read).  The diagonal 128 x 128 blocks
 * of T are inverted on the device, and the remaining work is gf2e products
 * (C += A*B) over a recursion on block ranges.  B must not overlap T
 * (GF2E_EALIAS).  A zero on a non-unit diagonal is reported by gf2e_sync as
 * GF2E_ESINGULAR (B is then unspecified).  The context's triangular-solve
 * buffers (inverted blocks and one block row of B) are owned by the
 * context.  Enqueued on `stream`. */
int gf2e_trsm_async(gf2e_ctx* ctx, int lower, int unit, const gf2e_mat* T, gf2e_mat* B, int e,
                    uint32_t f, void* stream);
int gf2e_trsm(gf2e_ctx* ctx, int lower, int unit, const gf2e_mat* T, gf2e_mat* B, int e, uint32_t f);

/* Row echelon form of A (m x n) in place (Sections 4.1 and 6): with full = 1
 * the reduced row echelon form (unique: every pivot is 1 and the only
 * nonzero of its column), with full = 0 a row echelon form whose pivots are
 * 1 with zeros below them.  *rank receives the rank; pivots (may be NULL,
 * else room for min(m, n) entries) receives the pivot column of rows
 * 0..rank-1.  Blocking (the null stream; the host reads each panel's pivot
 * count).  GF2E_ERANGE if an entry is >= 2^e (A is then unchanged).  The
 * context's buffers hold two copies of a 64-column panel and room for the
 * rows below the current rank (about m*n elements). */
int gf2e_echelonize(gf2e_ctx* ctx, gf2e_mat* A, int e, uint32_t f, int full, int64_t* rank,
                    int64_t* pivots);

/* PLE decomposition (Section 4.2, Definition PLE, in the paper's variant
 * whose L is not unit and whose E has leading ones): A = P * L * E.
 *   A (m x n): in place; on return rows 0..rank-1 hold E in row echelon form
 *     (row t has its leading 1 in column Q[t], zeros below it; entries above
 *     the pivots are not cleared) and rows rank..m-1 are zero.
 *   L (m x min(m, n), device, caller-owned, must not overlap A): on return
 *     L[i][t] for t < rank, lower trapezoidal (zero for t > i) with the
 *     pivots on its diagonal, and zero in columns rank..min(m, n)-1.
 *   P (host, m entries): row i of L * E equals row P[i] of the input A.
 *   Q (host, min(m, n) entries, may be NULL): pivot column of row t < rank;
 *     the pivot columns are the column rank profile of A, unique.
 * P and L depend on which rows the pivot search picks (several valid
 * decompositions exist); E's row space, the rank and Q do not.  Blocking
 * (the null stream).  GF2E_ERANGE if an entry of A is >= 2^e (A and L are
 * then unchanged), GF2E_ESHAPE if L's shape differs, GF2E_EALIAS if L
 * overlaps A.  Computed panel by panel like gf2e_echelonize, with each
 * panel's pivot block factored as Lk Uk on the device. */
int gf2e_ple(gf2e_ctx* ctx, gf2e_mat* A, gf2e_mat* L, int e, uint32_t f, int64_t* rank, int64_t* P,
             int64_t* Q);

const char* gf2e_strerror(int code);

/* ---- Field and schedule queries (host only; need no GPU) ---------------- */

/* GF2E_OK when 2 <= e <= 16 and f is irreducible of degree e. */
int gf2e_field_check(int e, uint32_t f);

/* Number t of GF(2) products in the schedule used for (e, f), or < 0. */
int gf2e_num_products(int e, uint32_t f);

/* The product schedule used for (e, f): product s multiplies
 * (XOR_{i in u[s]} A_i) by (XOR_{j in v[s]} B_j); plane c of the reduced
 * result is XOR_{s in m[c]} P_s (c < e).  For the Karatsuba schedule of
 * Section 5, coefficient d of the polynomial product is XOR_{s in w[d]} P_s
 * (d < 2e-1) before reduction modulo f; for a schedule compiled in for this
 * particular f (fewer products, reduction folded in) w is all zero.  w and m
 * are 0/1 matrices, one byte per entry, row-major with t columns:
 * w[d*t + s] = 1 iff s is in w[d], m[c*t + s] = 1 iff s is in m[c].  Arrays:
 * u, v of length >= t, w of length >= (2e-1)*t, m of length >= e*t, where
 * t <= 96 (t(16) = 81); any may be NULL.  GF2E_SCHEDULE=karatsuba in the
 * environment selects Karatsuba for every field. */
int gf2e_schedule(int e, uint32_t f, int* t, uint32_t* u, uint32_t* v, uint8_t* w, uint8_t* m);

/* ---- Stage entry points (the steps of gf2e_mul, for tests and composition).
 * Plane layouts (64-bit words, bit b of a word = index 64*word + b):
 *   A-side operand planes: t planes of K64p x Mp words, word (kw, r) = row r,
 *     k-bits [64kw, 64kw+64);
 *   B-side operand planes: t planes of K64p x Np words, word (kw, j) =
 *     column j, k-bits [64kw, 64kw+64) in B-side bit order: inside each
 *     aligned group of four, bits 4g, 4g+1, 4g+2, 4g+3 hold k = 4g+2, 4g+1,
 *     4g, 4g+3 (the first and third k trade places; the fp4 kernels then
 *     expand both sides with four masks and one shift);
 *   product planes: t planes of Mp x (Np/64) words, row-major.
 * Mp, Np must be multiples of 256 and >= m, n; K64p = 4*ceil(k/256).
 * All plane pointers are device pointers owned by the caller. */

typedef struct {
    int t;             /* products */
    int64_t Mp, Np;    /* padded rows of A-side / B-side planes */
    int64_t K64p;      /* words along k */
    int64_t a_bytes, b_bytes, p_bytes; /* sizes of the three plane buffers */
} gf2e_geometry;

int gf2e_plane_geometry(int e, uint32_t f, int64_t m, int64_t k, int64_t n, gf2e_geometry* g);

/* Slice A (m x k) into the t operand planes of the A side of the (e, f)
 * schedule (Section 3.2 slicing fused with the operand sums of Section 5). */
int gf2e_slice_a(gf2e_ctx* ctx, const gf2e_mat* A, int e, uint32_t f, uint64_t* planes, int64_t Mp,
                 int64_t K64p, void* stream);
/* Slice B (k x n) column-wise into the t transposed operand planes. */
int gf2e_slice_b(gf2e_ctx* ctx, const gf2e_mat* B, int e, uint32_t f, uint64_t* planes, int64_t Np,
                 int64_t K64p, void* stream);
/* P_s = Ahat_s * Bhat_s^T over GF(2) for s < t, one grouped launch of the
 * given kernel (GF2E_KERNEL_*, AUTO allowed).  The three plane buffers must
 * be 16-byte aligned (GF2E_EINVAL otherwise). */
int gf2e_plane_products(gf2e_ctx* ctx, int kernel, int t, const uint64_t* a_planes,
                        const uint64_t* b_planes, uint64_t* p_planes, int64_t m, int64_t n,
                        int64_t Mp, int64_t Np, int64_t K64p, void* stream);
/* Recombine the t products, reduce modulo f, cling into C (m x n). */
int gf2e_combine(gf2e_ctx* ctx, int e, uint32_t f, const uint64_t* p_planes, int64_t Mp,
                 int64_t Np, gf2e_mat* C, void* stream);

/* ---- Kernels, tuning, profiling ----------------------------------------- */

int gf2e_kernel_count(void);
const char* gf2e_kernel_name(int kernel);
int gf2e_set_kernel(gf2e_ctx* ctx, int kernel);
/* Kernel the planner would use now for an (e, f, m, k, n) product (for the
 * form it would use). */
int gf2e_chosen_kernel(gf2e_ctx* ctx, int e, uint32_t f, int64_t m, int64_t k, int64_t n);
/* Time every candidate kernel for this shape, for both forms, then both
 * whole pipelines, and cache the fastest form and kernel.  Runs on inputs
 * of zeros in the context's workspace; the caller's data is not touched. */
int gf2e_tune(gf2e_ctx* ctx, int e, uint32_t f, int64_t m, int64_t k, int64_t n, void* stream);

/* How gf2e_mul computes a product (gf2e_set_form).
 *  SCHEDULE: slice A and B into the t(e) operand planes of the bilinear
 *    schedule, t(e) GF(2) products, recombine and reduce modulo f (Section 5).
 *  ALPHA: write the product as C_c = sum_i A_i * (plane c of x^i B) over the
 *    bit-planes A_i of A, with x^i B computed in F_2[x]/<f>; that is one GF(2)
 *    product of the m x ek matrix [A_0 .. A_{e-1}] with the ek x en matrix of
 *    the planes of x^i B, whose column blocks are the e result planes.  The
 *    reduction modulo f is folded into the B side: the rows x^k B, k < e, are
 *    the first table that Section 4 builds for its Newton-John tables
 *    (Algorithm MakeTable), here on bit-planes.  It costs e^2 bit products per
 *    element product instead of t(e), in one launch with no recombination;
 *    the autotuner keeps it for sizes where that is faster.
 *  AUTO: the tuned form for the size bucket (SCHEDULE until tuned).
 * Results are identical for every form. */
enum { GF2E_FORM_AUTO = -1, GF2E_FORM_SCHEDULE = 0, GF2E_FORM_ALPHA = 1 };
int gf2e_set_form(gf2e_ctx* ctx, int form);
/* Form the planner would use now for an (e, f, m, k, n) product. */
int gf2e_chosen_form(gf2e_ctx* ctx, int e, uint32_t f, int64_t m, int64_t k, int64_t n);

/* Stage timers: when enabled, every launch of a stage is bracketed by HIP
 * events on the stream it runs on.  Stages: 0 slice A, 1 slice B,
 * 2 plane products, 3 combine, 4 a whole batched graph. */
enum { GF2E_STAGE_SLICE_A = 0, GF2E_STAGE_SLICE_B = 1, GF2E_STAGE_PRODUCTS = 2,
       GF2E_STAGE_COMBINE = 3, GF2E_STAGE_BATCH = 4, GF2E_NUM_STAGES = 5 };
int gf2e_profile(gf2e_ctx* ctx, int enable);
/* Waits for the recorded events; total milliseconds and launch count. */
int gf2e_profile_read(gf2e_ctx* ctx, int stage, double* total_ms, int64_t* launches);
int gf2e_profile_reset(gf2e_ctx* ctx);

/* Bytes of plane workspace currently held by the context. */
int64_t gf2e_workspace_bytes(gf2e_ctx* ctx);

#ifdef __cplusplus
}
#endif

#endif /* GF2E_H */
