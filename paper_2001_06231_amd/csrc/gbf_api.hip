// C ABI of the gbf solver: loader, single and batched solve drivers, policy
// extraction.  All device work is issued on the handle's HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "gbf.h"
#include "gbf_internal.h"

using namespace gbf;

static thread_local std::string t_err;

// Blocks per CU of the persistent kernel: below the occupancy limit, so that
// the cooperative grid is co-resident with margin.
#ifndef GBF_PBLOCKS
#define GBF_PBLOCKS 2
#endif
constexpr int kPersistentBlocksPerCU = GBF_PBLOCKS;

// AUTO solves a single instance with at most this many (x,u) pairs in one
// workgroup (measured crossover on MI355X).
#ifndef GBF_SINGLE_BLOCK_MAX_PAIRS
#define GBF_SINGLE_BLOCK_MAX_PAIRS 65536
#endif
constexpr int64_t kSingleBlockMaxPairs = GBF_SINGLE_BLOCK_MAX_PAIRS;

// Bucket order: extra rounds allowed beyond the plain cap (one per possible
// bucket key), a window spanning every bucket, and the work budget: at most
// the pair evaluations and twice the rounds of the handle's last plain
// solve, or without one 16 evaluations per pair.  Past the budget the solve
// continues in plain order; the switch happens by round kBucketRounds at
// the latest, so the continuation keeps at least the plain cap.
constexpr int64_t kBucketRounds = 65536;
constexpr int32_t kBucketsAll = 65536;
constexpr double kBucketEvalFactor = 1.0;
constexpr double kBucketRoundFactor = 2.0;
constexpr int64_t kBucketEvalsPerPair = 16;
// Progress test against the last plain solve's per-round profile: from
// round kProgressRound on, a bucket order whose pair evaluations so far are
// below kProgressFactor times the plain order's at the same round is taken
// to be falling behind (keys that do not follow V), and the solve finishes
// in plain order.  Measured on the 32 held-out learned-order instances:
// untrained keys drop to 0.3-0.5 of the plain profile by round 24; at 0.6
// the untrained control takes 1.25x the plain solve time (1.33x at 0.5)
// and the trained keys keep a 1.13x speedup (1.14x), their switches coming
// late in the solve.
#ifndef GBF_PROGRESS_ROUND
#define GBF_PROGRESS_ROUND 24
#endif
#ifndef GBF_PROGRESS_PCT
#define GBF_PROGRESS_PCT 60
#endif
constexpr int64_t kProgressRound = GBF_PROGRESS_ROUND;
constexpr double kProgressFactor = GBF_PROGRESS_PCT / 100.0;

static int fail(int code, const std::string& msg) {
    t_err = msg;
    return code;
}

int gbf::set_error(int code, const std::string& msg) { return fail(code, msg); }

#define HIPC(expr)                                                                                 \
    do {                                                                                           \
        hipError_t e_ = (expr);                                                                    \
        if (e_ != hipSuccess) return fail(GBF_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------ device memory
struct DevMem {
    std::vector<void*> ptrs;
    size_t bytes = 0;
    int alloc(void** out, size_t sz) {
        *out = nullptr;
        if (sz == 0) sz = 16;
        hipError_t e = hipMalloc(out, sz);
        if (e != hipSuccess) {
            *out = nullptr;
            return fail(GBF_ENOMEM, std::string("hipMalloc of ") + std::to_string(sz) + " bytes failed: " +
                                        hipGetErrorString(e));
        }
        ptrs.push_back(*out);
        bytes += sz;
        return GBF_OK;
    }
    void release(void* p, size_t sz) {
        auto it = std::find(ptrs.begin(), ptrs.end(), p);
        if (it != ptrs.end()) {
            (void)hipFree(p);
            ptrs.erase(it);
            bytes -= sz;
        }
    }
    ~DevMem() {
        for (void* p : ptrs) (void)hipFree(p);
    }
};

// Solver scratch: frontier bitmaps, list, per-round counts, counters.
struct Scratch {
    int64_t total_pairs = 0;
    int64_t counts_cap = 0;
    int64_t list_bytes = 0, counts_bytes = 0;  // allocated sizes (ids are 4 or 8 bytes)
    uint8_t* dirty[2] = {nullptr, nullptr};
    uint32_t* list = nullptr;
    uint32_t* counts = nullptr;
    unsigned long long* ctr = nullptr;
    unsigned long long* slots = nullptr;
    int32_t* inst_status = nullptr;
    uint32_t* barrier = nullptr;
    int32_t* error = nullptr;
    int32_t* result = nullptr;
    uint8_t* occ = nullptr;   // bucket order: occupancy per bucket [65536]
    uint32_t* thr = nullptr;  // bucket order: selected bucket
    Inst* dinst = nullptr;
    int ninst_cap = 0;
    void* host = nullptr;  // pinned readback area
    size_t host_bytes = 0;
    std::vector<hipEvent_t> events;
    DevMem mem;
    // A view of the library's static device scratch (gbf_solve_noalloc): its
    // buffers are carved from that array, nothing is allocated or released,
    // and no events exist.
    bool fixed = false;
    ~Scratch() {
        if (fixed) return;
        if (host) (void)hipHostFree(host);
        for (auto e : events) (void)hipEventDestroy(e);
    }
};

// Default memory budget of expand_box 3: this fraction of the device
// memory free at load (plus what the handle already holds), the threshold
// the paper's implementation used for its cache of images.
constexpr double kDefaultBudgetFraction = 0.68;

struct gbf_graph {
    int64_t budget_bytes = 0;  // expand_box 3: the budget applied
    int64_t budget_need = 0;   // expand_box 3: load bytes the predecessor images would have needed
    int64_t n = 0;
    int32_t K = 0;
    int32_t dtype = 0;
    int32_t enc = 0;
    int32_t dims[4] = {1, 1, 1, 1};
    int64_t m = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    int cus = 0;
    int clock_khz = 100000;
    DevMem mem;
    Inst inst{};
    bool solved = false;
    bool wide = false;  // 64-bit pair ids
    int64_t rev_bytes = 0, rptr_bytes = 0;  // predecessor images (reverse CSR)
    // the last plain-order solve of this handle (0 = none): the reference
    // of the bucket order's work budget, and (host-loop solves) its pair
    // evaluations accumulated round by round
    int64_t ref_evals = 0, ref_rounds = 0;
    std::vector<int64_t> ref_profile;
    Scratch scratch;
};

static int ensure_scratch(Scratch& S, int64_t total_pairs, int64_t max_rounds, int ninst, int nevents,
                          int idbytes = 4) {
    if (S.fixed) {
        if (total_pairs > S.total_pairs || max_rounds + 2 > S.counts_cap || ninst > S.ninst_cap || idbytes != 4)
            return fail(GBF_EINVAL, "problem exceeds the static scratch of the no-allocation solve");
        return GBF_OK;
    }
    const int64_t nchunks = (total_pairs + 15) / 16;
    if (S.total_pairs < total_pairs) {
        const int64_t old = (S.total_pairs + 15) / 16 * 16;
        if (S.dirty[0]) S.mem.release(S.dirty[0], old), S.mem.release(S.dirty[1], old);
        int rc;
        if ((rc = S.mem.alloc((void**)&S.dirty[0], nchunks * 16))) return rc;
        if ((rc = S.mem.alloc((void**)&S.dirty[1], nchunks * 16))) return rc;
        S.total_pairs = total_pairs;
    }
    if (S.list_bytes < total_pairs * idbytes) {
        if (S.list) S.mem.release(S.list, S.list_bytes);
        S.list = nullptr;
        S.list_bytes = 0;
        int rc;
        if ((rc = S.mem.alloc((void**)&S.list, total_pairs * idbytes))) return rc;
        S.list_bytes = total_pairs * idbytes;
    }
    if (S.counts_bytes < (max_rounds + 2) * idbytes) {
        if (S.counts) S.mem.release(S.counts, S.counts_bytes);
        S.counts = nullptr;
        S.counts_bytes = 0;
        int rc;
        if ((rc = S.mem.alloc((void**)&S.counts, (max_rounds + 2) * idbytes))) return rc;
        S.counts_bytes = (max_rounds + 2) * idbytes;
        S.counts_cap = S.counts_bytes / 4;
    }
    if (!S.ctr) {
        int rc;
        if ((rc = S.mem.alloc((void**)&S.ctr, 8 * sizeof(unsigned long long)))) return rc;
        if ((rc = S.mem.alloc((void**)&S.slots, (size_t)kMaxGrid * 8 * sizeof(unsigned long long)))) return rc;
        if ((rc = S.mem.alloc((void**)&S.barrier, kBarrierBytes))) return rc;
        if ((rc = S.mem.alloc((void**)&S.error, 64))) return rc;
        if ((rc = S.mem.alloc((void**)&S.result, 64))) return rc;
        if ((rc = S.mem.alloc((void**)&S.occ, 65536))) return rc;
        if ((rc = S.mem.alloc((void**)&S.thr, 64))) return rc;
    }
    if (S.ninst_cap < ninst) {
        if (S.dinst) S.mem.release(S.dinst, sizeof(Inst) * S.ninst_cap), S.mem.release(S.inst_status, 4 * S.ninst_cap);
        int rc;
        if ((rc = S.mem.alloc((void**)&S.dinst, sizeof(Inst) * ninst))) return rc;
        if ((rc = S.mem.alloc((void**)&S.inst_status, 4 * ninst))) return rc;
        S.ninst_cap = ninst;
    }
    const size_t hb = 16384 + 4 * (size_t)ninst;
    if (S.host_bytes < hb) {
        if (S.host) (void)hipHostFree(S.host);
        S.host = nullptr;
        if (hipHostMalloc(&S.host, hb, hipHostMallocDefault) != hipSuccess)
            return fail(GBF_ENOMEM, "hipHostMalloc failed");
        S.host_bytes = hb;
    }
    while ((int)S.events.size() < nevents) {
        // events 0 and 1 bracket a solve (1 is also waited on before the
        // host reads results); the others only time launches, so they skip
        // the system-scope fence (its cache write-back would be timed too)
        hipEvent_t e;
        HIPC(hipEventCreateWithFlags(&e, S.events.size() < 2 ? hipEventDefault : hipEventDisableSystemFence));
        S.events.push_back(e);
    }
    return GBF_OK;
}

// Per-input predecessor windows of a box problem (Sect. V-B: pred may be
// replaced by a superset): for input u and axis a the range of lo_a - x_a
// and hi_a - x_a over the live pairs.  Copied to `host` if it is not NULL.
static int make_windows(Inst& I, DevMem& M, hipStream_t s, std::vector<int32_t>* host) {
    const int64_t K = I.K;
    int32_t* win;
    int rc;
    if ((rc = M.alloc((void**)&win, K * 8 * 4))) return rc;
    std::vector<int32_t> hw(K * 8);
    for (int64_t u = 0; u < K; ++u)
        for (int a = 0; a < 4; ++a) {
            hw[u * 8 + a] = 0x7fffffff;
            hw[u * 8 + 4 + a] = (int32_t)0x80000000;
        }
    HIPC(hipMemcpyAsync(win, hw.data(), K * 8 * 4, hipMemcpyHostToDevice, s));
    HIPC(launch_box_window(I, win, s));
    if (host) {
        host->resize(K * 8);
        HIPC(hipMemcpyAsync(host->data(), win, K * 8 * 4, hipMemcpyDeviceToHost, s));
    }
    HIPC(hipStreamSynchronize(s));
    I.win = win;
    return GBF_OK;
}

// ------------------------------------------------------------------ load
// The part of the loader after validation for 64-bit pair ids (GBF_BOX):
// pruning, the per-input predecessor windows, and for expand_box 2 (or 3
// within the memory budget) a reverse CSR built straight from the boxes,
// whose entries are the predecessor pair ids relative to y*K (int32).
static int load_wide(gbf_graph* gr, const gbf_problem* p, int eb, int32_t* err) {
    Inst& I = gr->inst;
    DevMem& M = gr->mem;
    hipStream_t s = gr->stream;
    const int64_t n = I.n, K = I.K;
    int rc;
    HIPC(launch_prune(I, p->dtype, s));
    std::vector<int32_t> hw;
    if ((rc = make_windows(I, M, s, &hw))) return rc;
    M.release(err, 64);
    if (eb != 2 && eb != 3) return GBF_OK;
    // a reverse entry is (x - y)*K + u for y in F(x,u): bound |x - y| by the
    // windows' offsets so that it fits int32
    int64_t maxoff = 0;
    for (int64_t u = 0; u < K; ++u) {
        if (hw[u * 8] > hw[u * 8 + 4]) continue;  // no live pair with this input
        int64_t off = 0;
        for (int a = 0; a < 4; ++a)
            off += std::max<int64_t>(std::abs((int64_t)hw[u * 8 + a]), std::abs((int64_t)hw[u * 8 + 4 + a])) *
                   I.strides[a];
        maxoff = std::max(maxoff, off);
    }
    if ((maxoff + 1) * K >= ((int64_t)1 << 31)) {
        if (eb == 2) return fail(GBF_EINVAL, "64-bit pair ids with expand_box 2 need predecessor offsets below 2^31 pairs");
        return GBF_OK;  // stays implicit
    }
    uint32_t* cnt;
    uint64_t *rptr, *tmp;
    const int64_t nb = (n + 1023) / 1024 + 1;
    if ((rc = M.alloc((void**)&cnt, (n + 1) * 4)) || (rc = M.alloc((void**)&rptr, (n + 1) * 8)) ||
        (rc = M.alloc((void**)&tmp, nb * 8)))
        return rc;
    HIPC(launch_fill_u32(cnt, 0, n + 1, s));
    HIPC(launch_rev_count_box(I, cnt, s));
    HIPC(launch_scan64(cnt, rptr, n, tmp, s));
    uint64_t total = 0;
    HIPC(hipMemcpyAsync(&total, rptr + n, 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    const int64_t need = (int64_t)total * 4 + n * 8;  // entries + fill cursors
    if (eb == 3) {
        int64_t budget = p->mem_budget;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            HIPC(hipMemGetInfo(&fr, &tot));
            budget = (int64_t)(kDefaultBudgetFraction * (double)(fr + M.bytes));
        }
        gr->budget_bytes = budget;
        gr->budget_need = (int64_t)M.bytes + need;
        if ((int64_t)M.bytes + need > budget) {
            M.release(cnt, (n + 1) * 4);
            M.release(rptr, (n + 1) * 8);
            M.release(tmp, nb * 8);
            return GBF_OK;  // stays implicit
        }
    }
    int32_t* rel;
    unsigned long long* cursor;
    if ((rc = M.alloc((void**)&rel, (size_t)total * 4)) || (rc = M.alloc((void**)&cursor, n * 8))) return rc;
    HIPC(hipMemcpyAsync(cursor, rptr, n * 8, hipMemcpyDeviceToDevice, s));
    HIPC(launch_rev_fill_box(I, cursor, rel, s));
    HIPC(launch_sort_rows64(rptr, rel, n, s));
    HIPC(hipStreamSynchronize(s));
    M.release(cursor, n * 8);
    M.release(cnt, (n + 1) * 4);
    M.release(tmp, nb * 8);
    gr->rev_bytes = (int64_t)total * 4;
    gr->rptr_bytes = (n + 1) * 8;
    I.rptr64 = rptr;
    I.rrel = rel;
    I.enc = 2;
    gr->enc = 2;
    gr->m = (int64_t)total;
    return GBF_OK;
}

extern "C" int gbf_load_graph(const gbf_problem* p, void* hip_stream, gbf_graph** out) {
    if (!out) return fail(GBF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(GBF_EINVAL, "problem is NULL");
    if (p->n_states <= 0 || p->n_inputs <= 0) return fail(GBF_EINVAL, "n_states and n_inputs must be positive");
    if (p->dtype != GBF_I32 && p->dtype != GBF_F32) return fail(GBF_EINVAL, "dtype must be GBF_I32 or GBF_F32");
    if (p->encoding != GBF_CSR && p->encoding != GBF_BOX) return fail(GBF_EINVAL, "bad encoding");
    if (p->encoding == GBF_BOX && (p->expand_box < 0 || p->expand_box > 3))
        return fail(GBF_EINVAL, "expand_box must be 0, 1, 2 or 3");
    if (p->mem_budget < 0) return fail(GBF_EINVAL, "mem_budget must be >= 0");
    if (p->memspace != GBF_HOST && p->memspace != GBF_DEVICE) return fail(GBF_EINVAL, "bad memspace");
    if (!p->G || !p->g) return fail(GBF_EINVAL, "G and g are required");
    if (p->g_edge && p->encoding != GBF_CSR) return fail(GBF_EINVAL, "per-edge costs need GBF_CSR");
    const int64_t n = p->n_states, K = p->n_inputs, np = n * K;
    if (p->pair_ids64 != 0 && p->pair_ids64 != 1) return fail(GBF_EINVAL, "pair_ids64 must be 0 or 1");
    // 64-bit pair ids: by request, or when the 32-bit ids would not reach
    const bool wide = p->pair_ids64 == 1 || np >= ((int64_t)1 << 31);
    if (wide && (p->encoding != GBF_BOX || p->expand_box == 1))
        return fail(GBF_EINVAL, "64-bit pair ids (n_states * n_inputs >= 2^31, or pair_ids64) need GBF_BOX with "
                                "expand_box 0, 2 or 3");
    if (n >= ((int64_t)1 << 32) - 1) return fail(GBF_EINVAL, "n_states must be < 2^32 - 1");
    const hipMemcpyKind kind = p->memspace == GBF_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;

    std::unique_ptr<gbf_graph> gr(new gbf_graph());
    gr->n = n;
    gr->K = (int32_t)K;
    gr->dtype = p->dtype;
    gr->enc = p->encoding;
    gr->stream = (hipStream_t)hip_stream;
    HIPC(hipGetDevice(&gr->device));
    HIPC(hipDeviceGetAttribute(&gr->cus, hipDeviceAttributeMultiprocessorCount, gr->device));
    if (hipDeviceGetAttribute(&gr->clock_khz, hipDeviceAttributeWallClockRate, gr->device) != hipSuccess ||
        gr->clock_khz <= 0)
        gr->clock_khz = 100000;
    hipStream_t s = gr->stream;
    DevMem& M = gr->mem;
    Inst& I = gr->inst;
    I.n = n;
    I.K = (int32_t)K;
    I.enc = p->encoding;
    I.dtype = p->dtype;
    I.pair_base = 0;
    I.max_rounds = n;
    I.wide = wide ? 1 : 0;
    gr->wide = wide;
    for (int a = 0; a < 4; ++a) I.dims[a] = 1;

    int64_t m = 0;
    if (p->encoding == GBF_CSR) {
        if (!p->succ_ptr || !p->succ_idx) return fail(GBF_EINVAL, "CSR needs succ_ptr and succ_idx");
        int64_t last = 0;
        if (p->memspace == GBF_HOST) last = p->succ_ptr[np];
        else HIPC(hipMemcpy(&last, p->succ_ptr + np, 8, hipMemcpyDeviceToHost));
        if (last < np) return fail(GBF_EINVAL, "succ_ptr[n*K] < n*K: some F(x,u) is empty (F must be strict)");
        if (last >= ((int64_t)1 << 31)) return fail(GBF_EINVAL, "m must be < 2^31");
        m = last;
    } else {
        if (!p->box) return fail(GBF_EINVAL, "BOX needs box");
        int64_t prod = 1;
        for (int a = 0; a < 4; ++a) {
            if (p->dims[a] <= 0) return fail(GBF_EINVAL, "dims must be positive");
            prod *= p->dims[a];
            I.dims[a] = p->dims[a];
        }
        if (prod != n) return fail(GBF_EINVAL, "prod(dims) != n_states");
    }
    I.strides[0] = 1;
    I.strides[1] = I.dims[0];
    I.strides[2] = I.dims[0] * I.dims[1];
    I.strides[3] = I.dims[0] * I.dims[1] * I.dims[2];
    gr->m = m;
    for (int a = 0; a < 4; ++a) gr->dims[a] = I.dims[a];

    int rc;
    int32_t *G, *g, *err;
    uint8_t* avoid;
    void* V;
    if ((rc = M.alloc((void**)&G, n * 4)) || (rc = M.alloc((void**)&g, np * 4)) ||
        (rc = M.alloc((void**)&avoid, n)) || (rc = M.alloc(&V, n * 4)) ||
        (rc = M.alloc((void**)&err, 64)))
        return rc;
    HIPC(hipMemcpyAsync(G, p->G, n * 4, kind, s));
    HIPC(hipMemcpyAsync(g, p->g, np * 4, kind, s));
    if (p->avoid) HIPC(hipMemcpyAsync(avoid, p->avoid, n, kind, s));
    else HIPC(hipMemsetAsync(avoid, 0, n, s));
    HIPC(hipMemsetAsync(err, 0, 64, s));
    I.G = G;
    I.g = g;
    I.avoid = avoid;
    I.V = V;

    int64_t* sptr64 = nullptr;
    if (p->encoding == GBF_CSR) {
        uint32_t* sptr;
        int32_t* sidx;
        if ((rc = M.alloc((void**)&sptr, (np + 1) * 4)) || (rc = M.alloc((void**)&sidx, m * 4)) ||
            (rc = M.alloc((void**)&sptr64, (np + 1) * 8)))
            return rc;
        HIPC(hipMemcpyAsync(sptr64, p->succ_ptr, (np + 1) * 8, kind, s));
        HIPC(hipMemcpyAsync(sidx, p->succ_idx, m * 4, kind, s));
        I.sidx = sidx;
        I.sptr = sptr;
        if (p->g_edge) {
            int32_t* ge;
            if ((rc = M.alloc((void**)&ge, m * 4))) return rc;
            HIPC(hipMemcpyAsync(ge, p->g_edge, m * 4, kind, s));
            I.ge = ge;
        }
    } else {
        uint64_t* box;
        if ((rc = M.alloc((void**)&box, np * 8))) return rc;
        HIPC(hipMemcpyAsync(box, p->box, np * 8, kind, s));
        I.box = box;
    }
    HIPC(launch_validate(I, sptr64, m, p->dtype, err, s));
    int32_t herr = 0;
    HIPC(hipMemcpyAsync(&herr, err, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (herr) {
        std::string msg = "invalid problem:";
        if (herr & 1) msg += " empty F(x,u) or non-monotone succ_ptr;";
        if (herr & 2) msg += " successor index out of range;";
        if (herr & 4) msg += " NaN or -inf cost;";
        if (herr & 8) msg += " finite G on an avoid cell;";
        if (herr & 16) msg += " box outside the grid;";
        if (herr & 32) msg += " non-finite per-edge cost;";
        return fail(GBF_EINVAL, msg);
    }

    int eb = p->encoding == GBF_BOX ? p->expand_box : 0;
    if (wide) {
        if ((rc = load_wide(gr.get(), p, eb, err))) return rc;
        *out = gr.release();
        return GBF_OK;
    }
    // expand_box 3: keep the predecessor images (HYB) if their peak at load
    // fits the memory budget, else stay implicit (BOX)
    if (eb == 3) {
        uint32_t* sizes;
        unsigned long long* tot64;
        if ((rc = M.alloc((void**)&sizes, (np + 1) * 4)) || (rc = M.alloc((void**)&tot64, 8))) return rc;
        HIPC(hipMemsetAsync(tot64, 0, 8, s));
        HIPC(launch_box_sizes(I, sizes, tot64, s));
        unsigned long long total64 = 0;
        HIPC(hipMemcpyAsync(&total64, tot64, 8, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        M.release(sizes, (np + 1) * 4);
        M.release(tot64, 8);
        int64_t budget = p->mem_budget;
        if (budget == 0) {
            size_t fr = 0, tot = 0;
            HIPC(hipMemGetInfo(&fr, &tot));
            budget = (int64_t)(kDefaultBudgetFraction * (double)(fr + M.bytes));
        }
        // peak of the HYB build: temporary successor lists and row pointers,
        // box sizes, reverse lists, reverse row pointers and counts, scans
        const int64_t msucc = (int64_t)total64;
        const int64_t need = msucc * 4 * 2 + (np + 1) * 4 * 3 + (n + 1) * 4 * 2 + ((np + 1023) / 1024 + 2) * 8;
        eb = (msucc < ((int64_t)1 << 31) && (int64_t)M.bytes + need <= budget) ? 2 : 0;
        gr->budget_bytes = budget;
        gr->budget_need = (int64_t)M.bytes + need;
    }
    // expand_box 2 (HYB): successors stay boxes, predecessors become a
    // reverse CSR built from a temporary expansion
    const bool hyb = p->encoding == GBF_BOX && eb == 2;
    if (p->encoding == GBF_BOX && eb) {
        // materialise F as successor lists on the device (then as CSR below)
        uint32_t *sizes, *sptr, *tmp;
        unsigned long long* tot64;
        const int64_t nb = (np + 1023) / 1024 + 1;
        if ((rc = M.alloc((void**)&sizes, (np + 1) * 4)) || (rc = M.alloc((void**)&sptr, (np + 1) * 4)) ||
            (rc = M.alloc((void**)&tmp, nb * 4)) || (rc = M.alloc((void**)&tot64, 8)))
            return rc;
        HIPC(hipMemsetAsync(tot64, 0, 8, s));
        HIPC(launch_box_sizes(I, sizes, tot64, s));
        unsigned long long total64 = 0;
        HIPC(hipMemcpyAsync(&total64, tot64, 8, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        // exact 64-bit total first: the 32-bit scan below must not wrap
        if (total64 >= (1ull << 31))
            return fail(GBF_EINVAL, "expanded successor lists must hold < 2^31 entries");
        HIPC(launch_scan(sizes, sptr, np, tmp, s));
        const uint32_t mtot = (uint32_t)total64;
        int32_t* sidx;
        if ((rc = M.alloc((void**)&sidx, (size_t)mtot * 4))) return rc;
        HIPC(launch_box_fill(I, sptr, sidx, s));
        M.release(sizes, (np + 1) * 4);
        M.release(tmp, nb * 4);
        M.release(tot64, 8);
        if (!hyb) {
            M.release((void*)I.box, np * 8);
            I.box = nullptr;
        }
        I.sptr = sptr;
        I.sidx = sidx;
        I.enc = GBF_CSR;
        gr->enc = GBF_CSR;
        gr->m = mtot;
        m = mtot;
    }
    if (I.enc == GBF_CSR) {
        if (sptr64) HIPC(launch_convert_ptr(sptr64, const_cast<uint32_t*>(I.sptr), np + 1, s));
        HIPC(launch_prune(I, p->dtype, s));
        uint32_t *cnt, *rptr, *tmp, *rev;
        const int64_t nb = (n + 1023) / 1024 + 1;
        if ((rc = M.alloc((void**)&cnt, (n + 1) * 4)) || (rc = M.alloc((void**)&rptr, (n + 1) * 4)) ||
            (rc = M.alloc((void**)&tmp, nb * 4)))
            return rc;
        HIPC(hipMemsetAsync(cnt, 0, (n + 1) * 4, s));
        HIPC(launch_rev_count(I, cnt, s));
        HIPC(launch_scan(cnt, rptr, n, tmp, s));
        uint32_t total = 0;
        HIPC(hipMemcpyAsync(&total, rptr + n, 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if ((rc = M.alloc((void**)&rev, (size_t)total * 4))) return rc;
        HIPC(hipMemcpyAsync(cnt, rptr, n * 4, hipMemcpyDeviceToDevice, s));
        HIPC(launch_rev_fill(I, cnt, rev, s));
        HIPC(launch_sort_rows(rptr, rev, n, s));
        I.rptr = rptr;
        I.rev = rev;
        HIPC(hipStreamSynchronize(s));
        if (sptr64) M.release(sptr64, (np + 1) * 8);
        M.release(cnt, (n + 1) * 4);
        M.release(tmp, nb * 4);
        gr->rev_bytes = (int64_t)total * 4;
        gr->rptr_bytes = (n + 1) * 4;
        if (hyb) {
            M.release(const_cast<uint32_t*>(I.sptr), (np + 1) * 4);
            M.release(const_cast<int32_t*>(I.sidx), (size_t)m * 4);
            I.sptr = nullptr;
            I.sidx = nullptr;
            I.enc = 2;
            gr->enc = 2;
            // the windows, for a solve that drops the predecessor images
            if ((rc = make_windows(I, M, s, nullptr))) return rc;
        }
    } else {
        HIPC(launch_prune(I, p->dtype, s));
        if ((rc = make_windows(I, M, s, nullptr))) return rc;
    }
    M.release(err, 64);
    *out = gr.release();
    return GBF_OK;
}

// ------------------------------------------------------------------ aircraft
// Checks a scenario and fills the kernels' numeric view of it.
static int ac_spec(const gbf_aircraft* a, AcSpec& S, AcSets* sets) {
    if (!a) return fail(GBF_EINVAL, "scenario is NULL");
    int64_t n = 1;
    for (int k = 0; k < 4; ++k) {
        if (a->dims[k] < 1) return fail(GBF_EINVAL, "dims must be positive");
        n *= a->dims[k];
        S.dims[k] = a->dims[k];
    }
    if (a->dims[2] > 255 || a->dims[3] > 255) return fail(GBF_EINVAL, "dims[2] and dims[3] must be <= 255");
    if (n >= ((int64_t)1 << 32) - 1) return fail(GBF_EINVAL, "the grid must have fewer than 2^32 - 1 cells");
    if (a->x_max[0] <= 0 || a->x_max[1] <= 0) return fail(GBF_EINVAL, "x_max must be positive");
    if (a->v_range[0] <= 0 || a->v_range[1] <= a->v_range[0]) return fail(GBF_EINVAL, "bad v_range");
    if (!(a->mass > 0) || !(a->tau > 0) || !(a->p_D >= 0) || !(a->p_L >= 0) || !(a->thrust_max >= 0) ||
        !(a->bank_max_deg >= 0 && a->bank_max_deg < 90) || !std::isfinite(a->mass) || !std::isfinite(a->tau) ||
        !std::isfinite(a->p_D) || !std::isfinite(a->p_L) || !std::isfinite(a->thrust_max))
        return fail(GBF_EINVAL, "bad model constants");
    if (a->steps < 1 || a->steps > 64) return fail(GBF_EINVAL, "steps must be 1..64");
    if (a->n_thrust < 1 || a->n_bank < 1 || a->n_thrust * a->n_bank > 255)
        return fail(GBF_EINVAL, "need 1 <= n_thrust * n_bank <= 255");
    if (!std::isfinite(a->reward_cost)) return fail(GBF_EINVAL, "reward_cost must be finite");
    if (a->pair_ids64 != 0 && a->pair_ids64 != 1) return fail(GBF_EINVAL, "pair_ids64 must be 0 or 1");
    for (int k = 0; k < 2; ++k) S.x_max[k] = a->x_max[k], S.v_range[k] = a->v_range[k];
    S.mass = a->mass;
    S.p_D = a->p_D;
    S.p_L = a->p_L;
    S.tau = a->tau;
    S.steps = a->steps;
    S.n_thrust = a->n_thrust;
    S.n_bank = a->n_bank;
    S.thrust_max = a->thrust_max;
    S.bank_max_deg = a->bank_max_deg;
    if (sets) {
        const gbf_ac_box* lists[3] = {a->target, a->avoid, a->reward};
        const int32_t counts[3] = {a->n_target, a->n_avoid, a->n_reward};
        std::memset(sets, 0, sizeof(*sets));
        for (int k = 0; k < 3; ++k) {
            if (counts[k] < 0 || counts[k] > kAcMaxBoxes || (counts[k] > 0 && !lists[k]))
                return fail(GBF_EINVAL, "at most 16 boxes per set, with a non-NULL array");
            sets->count[k] = counts[k];
            for (int b = 0; b < counts[k]; ++b)
                for (int c = 0; c < 4; ++c) {
                    sets->box[k][b][c] = lists[k][b].lo[c];
                    sets->box[k][b][4 + c] = lists[k][b].hi[c];
                }
        }
    }
    return GBF_OK;
}

// Bank angle of input column b in radians, as the kernels compute it.
static double ac_bank_rad(const AcSpec& S, int b) {
    if (S.n_bank == 1) return 0.0;
    double t = (double)(2 * b - (S.n_bank - 1)) * S.bank_max_deg;
    t = t / (double)(S.n_bank - 1);
    return t * (3.141592653589793 / 180.0);
}

extern "C" int gbf_aircraft_table(const gbf_aircraft* a, int32_t* table, void* hip_stream) {
    AcSpec S;
    int rc = ac_spec(a, S, nullptr);
    if (rc) return rc;
    if (!table) return fail(GBF_EINVAL, "table is NULL");
    hipStream_t s = (hipStream_t)hip_stream;
    DevMem M;
    unsigned long long* bad;
    if ((rc = M.alloc((void**)&bad, 16))) return rc;
    HIPC(launch_fill_u32((uint32_t*)bad, 0, 4, s));
    HIPC(launch_ac_table(S, table, nullptr, bad, s));
    unsigned long long hb[2] = {0, 0};
    HIPC(hipMemcpyAsync(hb, bad, 16, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hb[0]) return fail(GBF_EINVAL, std::to_string(hb[0]) + " enclosures without an a priori enclosure");
    return GBF_OK;
}

extern "C" int gbf_load_aircraft(const gbf_aircraft* a, void* hip_stream, gbf_graph** out) {
    if (!out) return fail(GBF_EINVAL, "out is NULL");
    *out = nullptr;
    AcSpec S;
    AcSets sets;
    int rc = ac_spec(a, S, &sets);
    if (rc) return rc;
    const int64_t n = (int64_t)S.dims[0] * S.dims[1] * S.dims[2] * S.dims[3];
    const int K = S.n_thrust * S.n_bank;
    const int64_t rows = (int64_t)S.dims[2] * S.dims[3] * K;  // table entries
    const int64_t rrows = (int64_t)S.dims[2] * S.dims[3];     // reverse rows
    const int stage = a->n_reward > 0 ? 2 : 1;

    std::unique_ptr<gbf_graph> gr(new gbf_graph());
    gr->n = n;
    gr->K = K;
    gr->dtype = GBF_F32;
    gr->enc = 3;
    gr->stream = (hipStream_t)hip_stream;
    HIPC(hipGetDevice(&gr->device));
    HIPC(hipDeviceGetAttribute(&gr->cus, hipDeviceAttributeMultiprocessorCount, gr->device));
    if (hipDeviceGetAttribute(&gr->clock_khz, hipDeviceAttributeWallClockRate, gr->device) != hipSuccess ||
        gr->clock_khz <= 0)
        gr->clock_khz = 100000;
    hipStream_t s = gr->stream;
    DevMem& M = gr->mem;
    Inst& I = gr->inst;
    I.n = n;
    I.K = K;
    I.enc = 3;
    I.dtype = GBF_F32;
    I.pair_base = 0;
    I.max_rounds = n;
    gr->wide = a->pair_ids64 == 1 || n * K >= ((int64_t)1 << 31);
    I.wide = gr->wide ? 1 : 0;
    for (int k = 0; k < 4; ++k) I.dims[k] = gr->dims[k] = S.dims[k];
    I.strides[0] = 1;
    I.strides[1] = I.dims[0];
    I.strides[2] = I.dims[0] * I.dims[1];
    I.strides[3] = I.dims[0] * I.dims[1] * I.dims[2];
    I.ac_stage = stage;

    int32_t *G, *gu;
    uint8_t *avoid, *reward = nullptr;
    void* V;
    uint2* tab;
    uint32_t* rptr;
    unsigned long long* bad;
    AcInst* dac;
    uint8_t* imp;
    if ((rc = M.alloc((void**)&imp, (n + 15) / 16 * 16))) return rc;
    HIPC(launch_fill_u32((uint32_t*)imp, 0, (n + 15) / 16 * 4, s));
    if ((rc = M.alloc((void**)&G, n * 4)) || (rc = M.alloc((void**)&avoid, n)) || (rc = M.alloc(&V, n * 4)) ||
        (rc = M.alloc((void**)&tab, rows * 8)) || (rc = M.alloc((void**)&rptr, (rrows + 1) * 4)) ||
        (rc = M.alloc((void**)&gu, K * 4)) || (rc = M.alloc((void**)&bad, 16)) ||
        (rc = M.alloc((void**)&dac, sizeof(AcInst))))
        return rc;
    if (stage == 2 && (rc = M.alloc((void**)&reward, n))) return rc;
    // the enclosure table and the cell sets
    HIPC(launch_fill_u32((uint32_t*)bad, 0, 4, s));
    HIPC(launch_ac_table(S, nullptr, tab, bad, s));
    HIPC(launch_ac_sets(S, sets, a->G, G, avoid, reward, s));
    // reverse rows: counts, scan, fill
    HIPC(launch_fill_u32(rptr, 0, rrows + 1, s));
    HIPC(launch_ac_rev_count(S, tab, rptr, s));
    HIPC(launch_ac_scan(rptr, rrows, s));
    unsigned long long hb[2] = {0, 0};
    uint32_t total = 0;
    HIPC(hipMemcpyAsync(hb, bad, 16, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(&total, rptr + rrows, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (hb[0]) return fail(GBF_EINVAL, std::to_string(hb[0]) + " enclosures without an a priori enclosure");
    if (hb[1]) return fail(GBF_EINVAL, "table offsets beyond +-127 cells (cells too small for the sampling time)");
    uint2* rent;
    uint32_t* cursor;
    if ((rc = M.alloc((void**)&rent, (size_t)total * 8)) || (rc = M.alloc((void**)&cursor, rrows * 4))) return rc;
    HIPC(launch_fill_u32(cursor, 0, rrows, s));
    HIPC(launch_ac_rev_fill(S, tab, rptr, cursor, rent, s));
    HIPC(launch_ac_sort(rptr, rent, rrows, s));
    // running costs per input: tau + u2^2 rounded to fp32
    std::vector<int32_t> hgu(K);
    for (int u = 0; u < K; ++u) {
        const double b = ac_bank_rad(S, u % S.n_bank);
        const float c = (float)(S.tau + b * b);
        std::memcpy(&hgu[u], &c, 4);
    }
    HIPC(hipMemcpyAsync(gu, hgu.data(), K * 4, hipMemcpyHostToDevice, s));
    AcInst A{};
    A.tab = tab;
    A.rptr = rptr;
    A.rent = rent;
    A.reward = reward;
    A.gu = gu;
    A.imp = imp;  // zero here; every round's expansion clears what its relax step set
    std::memcpy(&A.rc, &a->reward_cost, 4);
    A.stage = stage;
    HIPC(hipMemcpyAsync(dac, &A, sizeof(A), hipMemcpyHostToDevice, s));
    HIPC(hipStreamSynchronize(s));  // the host copies above must finish before they go out of scope
    M.release(cursor, rrows * 4);
    I.G = G;
    I.g = nullptr;
    I.avoid = avoid;
    I.V = V;
    I.ac = dac;
    *out = gr.release();
    return GBF_OK;
}

static void forget_batches_of(gbf_graph* g);

extern "C" void gbf_free_graph(gbf_graph* g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    // batch contexts (and their captured graphs) that refer to this handle
    // would otherwise be reused for a new handle at the same address
    forget_batches_of(g);
    delete g;
}

extern "C" const char* gbf_last_error(void) { return t_err.c_str(); }

// ------------------------------------------------------------------ solve core
struct SolveOut {
    int64_t rounds = 0;
    unsigned long long ctr[6] = {0, 0, 0, 0, 0, 0};
    double solve_ms = 0, relax_ms = 0, barrier_ms = 0;
    int64_t relax_launches = 0;
    int mode = 0, grid = 0, block = 0, lanes = 0, graph = 0, sweeps = 0;
    int switched = 0;  // bucket order: 1 = the work budget moved the rest of the solve to the plain order
    int dropped = 0;   // 1 = the predecessor images were released during the solve
    int32_t inst_status[kMaxBatch] = {};  // per instance: 1 = round cap reached with work left
};

// Everything needed to enqueue one solve over a table of instances.
struct Plan {
    Run R{};
    int ninst = 0;
    int64_t max_rounds = 0, max_states = 0;
    int enc_mask = 0, lanes = 4, mode = GBF_MODE_HOSTLOOP, grid = 0, dtype = 0;
    int block = 0, compact_grid = 0;  // host loop: relax block (threads), compaction grid; 0 = defaults
    bool bucket = false;
    bool wide = false;  // 64-bit pair ids
    int ac_stage = 0;   // aircraft abstraction: 1 or 2 (costs per pair or per transition)
    // bucket order: work budget (pair evaluations, rounds) after which the
    // remaining rounds list every dirty pair, i.e. continue in plain order
    int64_t budget_evals = INT64_MAX, budget_rounds = INT64_MAX;
    const std::vector<int64_t>* ref_profile = nullptr;  // bucket order: plain profile to keep up with
    std::vector<int64_t>* record = nullptr;             // plain order: per-round profile out
    // memory floor: the handle whose predecessor images are released when
    // the device's free memory falls below mem_floor bytes
    gbf_graph* owner = nullptr;
    int64_t mem_floor = 0;
};

// Releases the predecessor images (reverse CSR) of a handle with box
// successors; later expansions search the per-input windows.  The caller
// has synchronised the stream, so no launch still reads them.
static void drop_images(gbf_graph* g) {
    Inst& I = g->inst;
    if (I.rev) g->mem.release(const_cast<uint32_t*>(I.rev), g->rev_bytes);
    if (I.rptr) g->mem.release(const_cast<uint32_t*>(I.rptr), g->rptr_bytes);
    if (I.rrel) g->mem.release(const_cast<int32_t*>(I.rrel), g->rev_bytes);
    if (I.rptr64) g->mem.release(const_cast<uint64_t*>(I.rptr64), g->rptr_bytes);
    I.rev = nullptr;
    I.rptr = nullptr;
    I.rrel = nullptr;
    I.rptr64 = nullptr;
    I.enc = 1;
    g->enc = 1;
    g->rev_bytes = g->rptr_bytes = 0;
}

static int plan_solve(Scratch& S, const Inst* insts, int ninst, int dtype, const gbf_opts& o, int cus,
                      int clock_khz, Plan& P) {
    P.ninst = ninst;
    P.dtype = dtype;
    int64_t total_pairs = 0;
    for (int i = 0; i < ninst; ++i) {
        const Inst& I = insts[i];
        total_pairs = std::max<int64_t>(total_pairs, I.pair_base + I.n * I.K);
        P.max_rounds = std::max<int64_t>(P.max_rounds, I.max_rounds);
        P.max_states = std::max<int64_t>(P.max_states, I.n);
        P.enc_mask |= I.enc == 0 ? (I.ge ? 8 : 1) : I.enc == 1 ? 2 : I.enc == 3 ? 16 : 4;
    }
    P.wide = insts[0].wide != 0;
    if (P.enc_mask & 16) {
        // the aircraft abstraction: one instance, host loop, plain order
        if (ninst != 1) return fail(GBF_EINVAL, "an aircraft abstraction is solved on its own, not in a batch");
        if (o.order != GBF_ORDER_PLAIN) return fail(GBF_EINVAL, "an aircraft abstraction uses the plain order");
        if (o.mode == GBF_MODE_PERSISTENT || o.mode == GBF_MODE_SINGLE_BLOCK)
            return fail(GBF_EINVAL, "an aircraft abstraction runs in host-loop mode");
        P.ac_stage = insts[0].ac_stage;
    }
    if (P.wide) {
        // 64-bit pair ids: one instance, host loop, plain order
        if (ninst != 1) return fail(GBF_EINVAL, "a problem with 64-bit pair ids is solved on its own, not in a batch");
        if (o.order != GBF_ORDER_PLAIN) return fail(GBF_EINVAL, "64-bit pair ids use the plain order");
        if (o.mode == GBF_MODE_PERSISTENT || o.mode == GBF_MODE_SINGLE_BLOCK)
            return fail(GBF_EINVAL, "64-bit pair ids run in host-loop mode");
    }
    const int nevents = o.profile ? 2 * (int)std::min<int64_t>(P.max_rounds + 2, 4096) + 2 : 4;
    int rc = ensure_scratch(S, total_pairs, P.max_rounds, P.ninst, nevents, P.wide ? 8 : 4);
    if (rc) return rc;
    Run& R = P.R;
    R.dirty[0] = S.dirty[0];
    R.dirty[1] = S.dirty[1];
    R.list = P.wide ? nullptr : S.list;
    R.counts = P.wide ? nullptr : S.counts;
    R.list64 = P.wide ? reinterpret_cast<uint64_t*>(S.list) : nullptr;
    R.counts64 = P.wide ? reinterpret_cast<unsigned long long*>(S.counts) : nullptr;
    R.ctr = S.ctr;
    R.slots = S.slots;
    R.inst_status = S.inst_status;
    R.barrier = S.barrier;
    R.error = S.error;
    R.result = S.result;
    R.occ = S.occ;
    R.thr = S.thr;
    R.key = nullptr;
    R.keyK = 1;
    if (o.order == GBF_ORDER_BUCKETS) {
        // one byte map: the selection leaves unlisted pairs in place and the
        // relax step marks into the same map
        if (P.ninst != 1) return fail(GBF_EINVAL, "bucket order is for single solves");
        if (o.mode == GBF_MODE_PERSISTENT || o.mode == GBF_MODE_SINGLE_BLOCK)
            return fail(GBF_EINVAL, "bucket order runs in host-loop mode");
        if (o.bucket_span < -1) return fail(GBF_EINVAL, "bucket_span must be >= -1");
        R.dirty[1] = R.dirty[0];
        R.key = insts[0].key;
        R.keyK = insts[0].K;
        R.bspan = o.bucket_span == 0 ? GBF_BUCKET_SPAN_DEFAULT : o.bucket_span;
        P.bucket = true;
    }
    R.nchunks = (total_pairs + 15) / 16;
    R.total_pairs = total_pairs;
    R.max_rounds = P.max_rounds;
    R.ninst = P.ninst;
    R.dtype = dtype;
    // a single barrier wait longer than 250 ms means the blocks are not
    // co-resident (or the device is stuck): give up instead of hanging
    R.timeout_ticks = (uint64_t)clock_khz * 250;
    P.lanes = (o.lanes == 1 || o.lanes == 2 || o.lanes == 4 || o.lanes == 8 || o.lanes == 16 || o.lanes == 32)
                  ? o.lanes
                  : 4;
    if (o.block != 0 && (o.block < 64 || o.block > 1024 || o.block % 64 != 0))
        return fail(GBF_EINVAL, "block must be 0 or a multiple of 64 from 64 to 1024");
    if (o.compact_grid < 0) return fail(GBF_EINVAL, "compact_grid must be >= 0");
    P.block = o.block;
    P.compact_grid = o.compact_grid;
    P.mode = (P.bucket || P.wide || (P.enc_mask & 16)) ? GBF_MODE_HOSTLOOP : o.mode;
    if (P.mode == GBF_MODE_SINGLE_BLOCK && P.ninst != 1)
        return fail(GBF_EINVAL, "single-block mode solves one instance");
    if (P.mode == GBF_MODE_AUTO && P.ninst == 1 && total_pairs <= kSingleBlockMaxPairs)
        P.mode = GBF_MODE_SINGLE_BLOCK;  // measured: fastest below this size
    if (P.mode == GBF_MODE_SINGLE_BLOCK) {
        P.grid = 1;
        return GBF_OK;
    }
    if (P.mode != GBF_MODE_HOSTLOOP) {
        const int per_cu = persistent_blocks_per_cu(R, P.lanes, dtype, P.enc_mask);
        if (per_cu <= 0) {
            if (P.mode == GBF_MODE_PERSISTENT) return fail(GBF_EHIP, "occupancy query failed");
            P.mode = GBF_MODE_HOSTLOOP;
        } else {
            if (P.mode == GBF_MODE_AUTO) {
                // measured on MI355X: one launch pair per round is as fast as
                // the cooperative kernel on single CSR instances and faster
                // on box instances (whose round kernel runs one block per
                // CU); the persistent form serves callers that want one
                // graph-capturable launch, and the autotuner times both
                P.mode = GBF_MODE_HOSTLOOP;
            }
            // co-residency is required; stay below the occupancy limit
            const int cap = std::min(per_cu, kPersistentBlocksPerCU) * cus;
            P.grid = o.grid > 0 ? std::min(o.grid, cap) : cap;
        }
    }
    if (P.mode == GBF_MODE_HOSTLOOP) P.grid = o.grid > 0 ? std::min(o.grid, kMaxGrid) : 8 * cus;
    return GBF_OK;
}

// Fills, W <- G, seed.  Kernels only (no memset), so it can be captured.
static int enqueue_init(Scratch& S, const Plan& P, const Inst* insts, hipStream_t s) {
    const Run& R = P.R;
    HIPC(launch_fill_u32((uint32_t*)R.dirty[0], 0, R.nchunks * 4, s));
    HIPC(launch_fill_u32((uint32_t*)R.dirty[1], 0, R.nchunks * 4, s));
    HIPC(launch_fill_u32(P.wide ? reinterpret_cast<uint32_t*>(R.counts64) : R.counts, 0,
                         (P.max_rounds + 2) * (P.wide ? 2 : 1), s));
    HIPC(launch_fill_u32((uint32_t*)R.ctr, 0, 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.slots, 0, (int64_t)kMaxGrid * 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.inst_status, 0, P.ninst, s));
    HIPC(launch_fill_u32(R.barrier, 0, kBarrierBytes / 4, s));
    HIPC(launch_fill_u32((uint32_t*)R.error, 0, 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.result, 0, 16, s));
    if (P.bucket) HIPC(launch_fill_u32((uint32_t*)R.occ, 0, 65536 / 4, s));
    for (int i = 0; i < P.ninst; ++i) HIPC(launch_init(S.dinst, insts[i], P.dtype, s));
    if (P.enc_mask == 16) HIPC(launch_ac_seed(S.dinst, R, P.max_states, s, P.wide));
    else HIPC(launch_seed(S.dinst, P.ninst, R, P.max_states, P.dtype, P.enc_mask, s, P.wide));
    return GBF_OK;
}

// Statistics reduction and read-back of the status words into pinned host
// memory (all capturable).  Layout of S.host: [0] rounds, [1] barrier error,
// [8] bucket sweeps, [16..27] counters (6 x u64), [64..] per-instance status.
static int enqueue_readback(Scratch& S, const Plan& P, hipStream_t s) {
    int32_t* host = (int32_t*)S.host;
    HIPC(launch_sum_slots(S.slots, kMaxGrid, S.ctr, s));
    HIPC(hipMemcpyAsync(host, S.result, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(host + 1, S.error, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(host + 4, S.result + 2, 8, hipMemcpyDeviceToHost, s));
    if (P.bucket) HIPC(hipMemcpyAsync(host + 8, S.thr + 2, 4, hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(host + 16, S.ctr, 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(host + 64, S.inst_status, 4 * P.ninst, hipMemcpyDeviceToHost, s));
    return GBF_OK;
}

static void read_host(const Scratch& S, const Plan& P, SolveOut& out, bool rounds_from_host, int clock_khz) {
    const int32_t* host = (const int32_t*)S.host;
    if (rounds_from_host) {
        out.rounds = host[0];
        uint64_t ticks;
        std::memcpy(&ticks, host + 4, 8);
        out.barrier_ms = (double)ticks / (double)clock_khz;
    }
    std::memcpy(out.ctr, host + 16, 6 * sizeof(unsigned long long));
    for (int i = 0; i < P.ninst; ++i) out.inst_status[i] = host[64 + i];
    out.sweeps = P.bucket ? host[8] : 0;
    out.mode = P.mode;
    out.grid = P.grid;
    out.block = P.mode == GBF_MODE_HOSTLOOP ? (P.block > 0 ? P.block : kRelaxBlock) : 1024;
    out.lanes = P.lanes;
}

// Host-loop rounds: compact + relax per round; the host reads the per-round
// frontier sizes after each batch of rounds (rounds launched after the
// frontier drained exit at once).
static int enqueue_hostloop(Scratch& S, const Plan& P, const gbf_opts& o, hipStream_t s, SolveOut& out) {
    Run R = P.R;
    int32_t* host = (int32_t*)S.host;
    int64_t r = 0;
    int64_t batch = o.batch_hint > 0 ? o.batch_hint : 8;
    int ev = 2;
    bool done = false;
    int64_t evals = 0;  // pairs listed so far (bucket order's work budget)
    // the round after the last allowed one only flags capped instances, so a
    // zero count appears at round max_rounds + 1 at the latest
    int enc_mask = P.enc_mask;
    while (!done && r <= P.max_rounds + 1) {
        const int64_t nb = std::min<int64_t>(batch, P.max_rounds + 2 - r);
        if (P.owner && P.mem_floor > 0 && enc_mask == 4 && r > 0 && !out.dropped) {
            // the stream is idle here: the previous batch was synchronised
            size_t fr = 0, tot = 0;
            HIPC(hipMemGetInfo(&fr, &tot));
            if ((int64_t)fr < P.mem_floor) {
                drop_images(P.owner);
                enc_mask = 2;  // box successors, predecessor windows
                out.dropped = 1;
            }
        }
        bool behind = false;
        if (P.bucket && P.ref_profile && !P.ref_profile->empty() && r >= kProgressRound) {
            const auto& pr = *P.ref_profile;
            const int64_t ref = pr[(size_t)std::min<int64_t>(r - 1, (int64_t)pr.size() - 1)];
            behind = (double)evals < kProgressFactor * (double)ref;
        }
        if (P.bucket && !out.switched && (behind || evals > P.budget_evals || r + nb > P.budget_rounds)) {
            // over budget: every later round lists all dirty pairs (a
            // window over every bucket), which is the plain order continued
            // from the current iterate; any order reaches the same fixed
            // point, so only the work changes
            R.bspan = kBucketsAll;
            out.switched = 1;
        }
        for (int64_t k = 0; k < nb; ++k) {
            if (P.bucket) HIPC(launch_bucket_compact(R, (int)(r + k), P.compact_grid, s));
            else HIPC(launch_compact(R, (int)(r + k), P.compact_grid, s, P.wide));
            const bool timed = o.profile && ev + 1 < (int)S.events.size();
            if (timed) HIPC(hipEventRecord(S.events[ev], s));
            if (enc_mask == 16) {
                HIPC(launch_ac_relax(S.dinst, R, (int)(r + k), P.grid, s, P.wide, P.ac_stage));
                HIPC(launch_ac_expand(S.dinst, R, (int)(r + k), P.max_states, s, P.wide));
            } else {
                HIPC(launch_relax(S.dinst, R, (int)(r + k), P.grid, P.lanes, P.dtype, enc_mask, s, P.wide, P.block));
            }
            if (timed) {
                HIPC(hipEventRecord(S.events[ev + 1], s));
                ev += 2;
            }
        }
        const int64_t nread = std::min<int64_t>(nb, 1000);
        if (P.wide) HIPC(hipMemcpyAsync(host + 256, R.counts64 + r, nread * 8, hipMemcpyDeviceToHost, s));
        else HIPC(hipMemcpyAsync(host + 256, R.counts + r, nread * 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        for (int64_t k = 0; k < nread; ++k) {
            uint64_t c;
            if (P.wide) std::memcpy(&c, host + 256 + 2 * k, 8);
            else c = (uint32_t)host[256 + k];
            if (c == 0) {
                out.rounds = r + k;
                done = true;
                break;
            }
            evals += (int64_t)c;
            if (P.record && (int64_t)P.record->size() == r + k) P.record->push_back(evals);
        }
        r += nb;
        // speculative rounds after the frontier drains cost a launch each,
        // host reads a round trip: grow the batch moderately
        batch = std::min<int64_t>(batch * 2, 16);
    }
    if (!done) return fail(GBF_EHIP, "internal: frontier did not drain after the round cap");
    if (o.profile) {
        for (int e = 2; e < ev; e += 2) {
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, S.events[e], S.events[e + 1]));
            out.relax_ms += ms;
            out.relax_launches++;
        }
    }
    return GBF_OK;
}

// Runs one solve over `insts`, not captured.
static int run_rounds(Scratch& S, const Inst* insts, int ninst, int dtype, const gbf_opts& o, hipStream_t s,
                      int cus, int clock_khz, SolveOut& out, int64_t budget_evals = INT64_MAX,
                      int64_t budget_rounds = INT64_MAX, const std::vector<int64_t>* ref_profile = nullptr,
                      std::vector<int64_t>* record = nullptr, gbf_graph* owner = nullptr) {
    Plan P;
    int rc = plan_solve(S, insts, ninst, dtype, o, cus, clock_khz, P);
    if (rc) return rc;
    P.budget_evals = budget_evals;
    P.budget_rounds = budget_rounds;
    P.ref_profile = ref_profile;
    P.record = record;
    if (owner && ninst == 1 && o.mem_floor_mib > 0) {
        P.owner = owner;
        P.mem_floor = (int64_t)o.mem_floor_mib << 20;
    }
    if (!S.events.empty()) HIPC(hipEventRecord(S.events[0], s));
    HIPC(hipMemcpyAsync(S.dinst, insts, sizeof(Inst) * P.ninst, hipMemcpyHostToDevice, s));
    if ((rc = enqueue_init(S, P, insts, s))) return rc;
    if (P.mode == GBF_MODE_SINGLE_BLOCK) {
        if (o.profile) HIPC(hipEventRecord(S.events[2], s));
        HIPC(launch_single(S.dinst, P.R, P.lanes, dtype, P.enc_mask, P.max_states, s));
        if (o.profile) HIPC(hipEventRecord(S.events[3], s));
        if ((rc = enqueue_readback(S, P, s))) return rc;
        HIPC(hipStreamSynchronize(s));
        read_host(S, P, out, true, clock_khz);
        if (o.profile) {
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, S.events[2], S.events[3]));
            out.relax_ms = ms;
            out.relax_launches = 1;
        }
        return GBF_OK;
    }
    if (P.mode == GBF_MODE_PERSISTENT) {
        if (o.profile) HIPC(hipEventRecord(S.events[2], s));
        HIPC(launch_persistent(S.dinst, P.R, P.grid, P.lanes, dtype, P.enc_mask, false, s));
        if (o.profile) HIPC(hipEventRecord(S.events[3], s));
        if ((rc = enqueue_readback(S, P, s))) return rc;
        HIPC(hipStreamSynchronize(s));
        if (((int32_t*)S.host)[1] != 0) {
            if (o.mode == GBF_MODE_AUTO) {
                // retry the whole solve with one launch sequence per round
                gbf_opts o2 = o;
                o2.mode = GBF_MODE_HOSTLOOP;
                out = SolveOut();
                return run_rounds(S, insts, ninst, dtype, o2, s, cus, clock_khz, out, budget_evals, budget_rounds,
                                  ref_profile, record, owner);
            }
            return fail(GBF_ETIMEOUT, "grid barrier timed out (blocks not co-resident?)");
        }
        read_host(S, P, out, true, clock_khz);
        if (o.profile) {
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, S.events[2], S.events[3]));
            out.relax_ms = ms;
            out.relax_launches = 1;
        }
        return GBF_OK;
    }
    if ((rc = enqueue_hostloop(S, P, o, s, out))) return rc;
    if ((rc = enqueue_readback(S, P, s))) return rc;
    HIPC(hipStreamSynchronize(s));
    read_host(S, P, out, false, clock_khz);
    return GBF_OK;
}

static gbf_opts default_opts() {
    gbf_opts o;
    std::memset(&o, 0, sizeof(o));
    return o;
}

static void fill_stats(gbf_stats* st, int status, const SolveOut& so, int64_t rounds_cap, size_t bytes, int enc) {
    if (!st) return;
    std::memset(st, 0, sizeof(*st));
    st->status = status;
    st->rounds = std::min<int64_t>(so.rounds, rounds_cap);
    st->pair_evals = (int64_t)so.ctr[0];
    st->edge_relax = (int64_t)so.ctr[1];
    st->improvements = (int64_t)so.ctr[2];
    st->saturations = (int64_t)so.ctr[3];
    st->expansions = (int64_t)so.ctr[4];
    st->marks = (int64_t)so.ctr[5];
    st->solve_ms = so.solve_ms;
    st->relax_ms = so.relax_ms;
    st->relax_launches = so.relax_launches;
    st->barrier_ms = so.barrier_ms;
    st->device_bytes = (int64_t)bytes;
    st->mode_used = so.mode;
    st->grid_used = so.grid;
    st->block_used = so.block;
    st->lanes_used = so.lanes;
    st->graph_used = so.graph;
    st->sweeps = so.sweeps;
    st->enc_used = enc;
    st->images_dropped = so.dropped;
}

static int write_values(gbf_graph* g, void* V_out, int memspace, hipStream_t s) {
    if (!V_out) return GBF_OK;
    if (memspace == GBF_DEVICE) {
        HIPC(launch_decode(g->inst, g->dtype, V_out, s));
    } else {
        // decode into the scratch list buffer, then copy out
        HIPC(launch_decode(g->inst, g->dtype, g->scratch.list, s));
        HIPC(hipMemcpyAsync(V_out, g->scratch.list, g->n * 4, hipMemcpyDeviceToHost, s));
    }
    return GBF_OK;
}

extern "C" int gbf_solve(gbf_graph* g, const gbf_opts* opts, void* V_out, gbf_stats* st) {
    if (!g) return fail(GBF_EINVAL, "graph is NULL");
    gbf_opts o = opts ? *opts : default_opts();
    if (o.order == GBF_ORDER_BUCKETS && !o.bucket_key) return fail(GBF_EINVAL, "BUCKETS order needs bucket_key");
    if (o.order != GBF_ORDER_PLAIN && o.order != GBF_ORDER_BUCKETS) return fail(GBF_EINVAL, "bad order");
    if (o.v_memspace != GBF_HOST && o.v_memspace != GBF_DEVICE) return fail(GBF_EINVAL, "bad v_memspace");
    hipStream_t s = g->stream;
    g->solved = false;
    Inst I = g->inst;
    I.pair_base = 0;
    I.max_rounds = o.max_rounds > 0 ? o.max_rounds : g->n;
    const bool bucket = o.order == GBF_ORDER_BUCKETS;
    if (bucket) {
        // the bucket schedule may split a plain round into several: its cap
        // is the plain cap plus one round per possible bucket; hitting it
        // reruns the plain order (which decides the status)
        int rc = ensure_scratch(g->scratch, g->n * g->K, 1, 1, 4);
        if (rc) return rc;
        I.key = o.bucket_key;
        I.occ = g->scratch.occ;
        I.max_rounds += kBucketRounds;
    }
    // bucket order: the work budget, from the handle's last plain solve
    int64_t budget_evals = INT64_MAX, budget_rounds = INT64_MAX;
    if (bucket && o.bucket_budget < -1) return fail(GBF_EINVAL, "bucket_budget must be >= -1");
    if (bucket && o.bucket_budget != -1) {
        const double pct = (o.bucket_budget == 0 ? 100.0 : (double)o.bucket_budget) / 100.0;
        budget_evals = (int64_t)(pct * (g->ref_evals > 0 ? kBucketEvalFactor * (double)g->ref_evals
                                                         : (double)(kBucketEvalsPerPair * g->n * g->K)));
        budget_rounds = kBucketRounds;
        if (g->ref_rounds > 0)
            budget_rounds =
                std::min<int64_t>(budget_rounds, (int64_t)(pct * kBucketRoundFactor * (double)g->ref_rounds) + 1);
    }
    // the switch to the plain order comes by round kBucketRounds at the
    // latest, so the continuation keeps at least the plain cap
    if (bucket) budget_rounds = std::min<int64_t>(budget_rounds, kBucketRounds);
    const Inst insts[1] = {I};
    SolveOut so;
    std::vector<int64_t> profile;
    const bool use_ref = bucket && o.bucket_budget != -1 && !g->ref_profile.empty();
    if (o.mem_floor_mib < 0) return fail(GBF_EINVAL, "mem_floor_mib must be >= 0");
    int rc = run_rounds(g->scratch, insts, 1, g->dtype, o, s, g->cus, g->clock_khz, so, budget_evals, budget_rounds,
                        use_ref ? &g->ref_profile : nullptr, bucket ? nullptr : &profile, g);
    if (rc) return rc;
    int fallback = so.switched ? 1 : 0;
    if (bucket && so.inst_status[0]) {
        gbf_opts o2 = o;
        o2.order = GBF_ORDER_PLAIN;
        o2.bucket_key = nullptr;
        gbf_stats st2;
        rc = gbf_solve(g, &o2, V_out, &st2);
        if (st) {
            *st = st2;
            st->fallback = 2;
        }
        return rc;
    }
    if ((rc = write_values(g, V_out, o.v_memspace, s))) return rc;
    HIPC(hipEventRecord(g->scratch.events[1], s));
    HIPC(hipEventSynchronize(g->scratch.events[1]));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, g->scratch.events[0], g->scratch.events[1]));
    so.solve_ms = ms;
    const int status = so.inst_status[0] ? GBF_ENEGCYCLE : GBF_OK;
    fill_stats(st, status, so, I.max_rounds, g->mem.bytes + g->scratch.mem.bytes, g->enc);
    if (st) st->fallback = fallback;
    g->solved = true;
    if (!bucket && status == GBF_OK) {
        g->ref_evals = (int64_t)so.ctr[0];
        g->ref_rounds = so.rounds;
        g->ref_profile.swap(profile);  // empty unless the solve ran in host-loop mode
    }
    if (status != GBF_OK) fail(status, "round cap reached with a non-empty frontier");
    return status;
}

// ------------------------------------------------------------------ no-allocation solve
// One static device array holds every scratch buffer of a solve (frontier
// byte maps, list, per-round counts, statistics, barrier and status words,
// the instance table).  Each device the library runs on holds its own copy
// for the life of the process.  Host code never passes the array's name to
// a kernel (in host code it names a host-side stand-in): the device address
// of each device's copy is taken once with hipGetSymbolAddress and kept.
constexpr int64_t kNaPairs = GBF_NOALLOC_MAX_PAIRS;
constexpr int64_t kNaRounds = (int64_t)GBF_NOALLOC_MAX_ROUNDS + 2;  // round-count slots (round cap + 2)
constexpr int kNaMaxDevices = 64;
constexpr size_t kNaAlign = 256;
constexpr size_t na_up(size_t v) { return (v + kNaAlign - 1) / kNaAlign * kNaAlign; }
constexpr size_t kNaOffDirty0 = 0;
constexpr size_t kNaOffDirty1 = kNaOffDirty0 + na_up((size_t)kNaPairs);
constexpr size_t kNaOffList = kNaOffDirty1 + na_up((size_t)kNaPairs);
constexpr size_t kNaOffCounts = kNaOffList + na_up((size_t)kNaPairs * 4);
constexpr size_t kNaOffCtr = kNaOffCounts + na_up((size_t)kNaRounds * 4);
constexpr size_t kNaOffSlots = kNaOffCtr + na_up(8 * sizeof(unsigned long long));
constexpr size_t kNaOffBarrier = kNaOffSlots + na_up((size_t)kMaxGrid * 8 * sizeof(unsigned long long));
constexpr size_t kNaOffError = kNaOffBarrier + na_up(kBarrierBytes);
constexpr size_t kNaOffResult = kNaOffError + na_up(64);
constexpr size_t kNaOffOcc = kNaOffResult + na_up(64);
constexpr size_t kNaOffThr = kNaOffOcc + na_up(65536);
constexpr size_t kNaOffInst = kNaOffThr + na_up(64);
constexpr size_t kNaOffStatus = kNaOffInst + na_up(sizeof(Inst));
constexpr size_t kNaBytes = kNaOffStatus + na_up(64);

static __device__ __align__(256) uint8_t scratch[kNaBytes];

static std::mutex g_na_lock;
static void* g_na_ptr[kNaMaxDevices];
// host readback words (pageable: the copies into it complete before use)
static int32_t g_na_host[kNaMaxDevices][2048];

// Device address of `scratch` on `device` (looked up once per device, with
// that device current).
static int na_scratch(int device, void** out) {
    if (device < 0 || device >= kNaMaxDevices) return fail(GBF_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lk(g_na_lock);
    if (!g_na_ptr[device]) {
        int cur = -1;
        HIPC(hipGetDevice(&cur));
        if (cur != device) HIPC(hipSetDevice(device));
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (cur != device) (void)hipSetDevice(cur);
        if (e != hipSuccess || !ptr)
            return fail(GBF_EHIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_na_ptr[device] = ptr;
    }
    *out = g_na_ptr[device];
    return GBF_OK;
}

extern "C" int gbf_solve_noalloc(gbf_graph* g, const gbf_opts* opts, void* V_out, gbf_stats* st) {
    const auto t0 = std::chrono::steady_clock::now();
    if (!g) return fail(GBF_EINVAL, "graph is NULL");
    gbf_opts o = opts ? *opts : default_opts();
    if (g->wide) return fail(GBF_EINVAL, "the no-allocation solve takes 32-bit pair ids only");
    if (g->enc == 3) return fail(GBF_EINVAL, "an aircraft abstraction is solved with gbf_solve");
    if (o.order != GBF_ORDER_PLAIN) return fail(GBF_EINVAL, "the no-allocation solve uses the plain order");
    if (o.v_memspace != GBF_HOST && o.v_memspace != GBF_DEVICE) return fail(GBF_EINVAL, "bad v_memspace");
    o.profile = 0;  // per-launch timing needs events, which are allocated
    const int64_t npairs = g->n * g->K;
    const int64_t max_rounds = o.max_rounds > 0 ? o.max_rounds : g->n;
    if (npairs > kNaPairs)
        return fail(GBF_EINVAL, "the no-allocation solve takes at most " + std::to_string(kNaPairs) + " pairs");
    if (max_rounds > kNaRounds - 2)
        return fail(GBF_EINVAL, "the no-allocation solve takes a round cap of at most " +
                                    std::to_string(kNaRounds - 2) + " (pass a smaller max_rounds)");
    void* base = nullptr;
    int rc = na_scratch(g->device, &base);
    if (rc) return rc;
    uint8_t* b = static_cast<uint8_t*>(base);
    hipStream_t s = g->stream;
    Scratch S;
    S.fixed = true;
    S.total_pairs = kNaPairs;
    S.counts_cap = kNaRounds;
    S.ninst_cap = 1;
    S.dirty[0] = b + kNaOffDirty0;
    S.dirty[1] = b + kNaOffDirty1;
    S.list = reinterpret_cast<uint32_t*>(b + kNaOffList);
    S.counts = reinterpret_cast<uint32_t*>(b + kNaOffCounts);
    S.ctr = reinterpret_cast<unsigned long long*>(b + kNaOffCtr);
    S.slots = reinterpret_cast<unsigned long long*>(b + kNaOffSlots);
    S.barrier = reinterpret_cast<uint32_t*>(b + kNaOffBarrier);
    S.error = reinterpret_cast<int32_t*>(b + kNaOffError);
    S.result = reinterpret_cast<int32_t*>(b + kNaOffResult);
    S.occ = b + kNaOffOcc;
    S.thr = reinterpret_cast<uint32_t*>(b + kNaOffThr);
    S.dinst = reinterpret_cast<Inst*>(b + kNaOffInst);
    S.inst_status = reinterpret_cast<int32_t*>(b + kNaOffStatus);
    S.host = g_na_host[g->device];
    S.host_bytes = sizeof(g_na_host[0]);
    g->solved = false;
    Inst I = g->inst;
    I.pair_base = 0;
    I.max_rounds = max_rounds;
    const Inst insts[1] = {I};
    SolveOut so;
    rc = run_rounds(S, insts, 1, g->dtype, o, s, g->cus, g->clock_khz, so);
    if (rc) return rc;
    if (V_out) {
        if (o.v_memspace == GBF_DEVICE) {
            HIPC(launch_decode(g->inst, g->dtype, V_out, s));
        } else {
            HIPC(launch_decode(g->inst, g->dtype, S.list, s));
            HIPC(hipMemcpyAsync(V_out, S.list, g->n * 4, hipMemcpyDeviceToHost, s));
        }
    }
    HIPC(hipStreamSynchronize(s));
    so.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    const int status = so.inst_status[0] ? GBF_ENEGCYCLE : GBF_OK;
    fill_stats(st, status, so, I.max_rounds, g->mem.bytes, g->enc);
    g->solved = true;
    if (status != GBF_OK) fail(status, "round cap reached with a non-empty frontier");
    return status;
}

extern "C" int gbf_extract_policy(gbf_graph* g, int32_t* policy_out, int32_t memspace, int64_t* residual) {
    if (!g) return fail(GBF_EINVAL, "graph is NULL");
    if (!g->solved) return fail(GBF_ENOTSOLVED, "no solve on this handle");
    if (!policy_out) return fail(GBF_EINVAL, "policy_out is NULL");
    hipStream_t s = g->stream;
    Scratch& S = g->scratch;
    int rc = ensure_scratch(S, g->n * g->K, 1, 1, 2);
    if (rc) return rc;
    unsigned long long* bad = S.ctr + 6;
    HIPC(launch_fill_u32((uint32_t*)bad, 0, 2, s));
    int32_t* dst = memspace == GBF_DEVICE ? policy_out : (int32_t*)S.list;
    if (g->enc == 3) HIPC(launch_ac_policy(g->inst, dst, bad, s));
    else HIPC(launch_policy(g->inst, g->dtype, dst, bad, s));
    if (memspace != GBF_DEVICE) HIPC(hipMemcpyAsync(policy_out, dst, g->n * 4, hipMemcpyDeviceToHost, s));
    unsigned long long* hb = (unsigned long long*)((char*)S.host + 64);
    HIPC(hipMemcpyAsync(hb, bad, 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (residual) *residual = (int64_t)*hb;
    return GBF_OK;
}

// ------------------------------------------------------------------ batch
// A batch context is kept per set of handles: its scratch, its instance
// table and, for the persistent form with device outputs, a HIP graph of the
// whole solve (fills, W <- G, seed, the cooperative round kernel, statistics,
// decode into the outputs, status read-back) that later calls replay.
struct BatchCtx {
    std::vector<gbf_graph*> graphs;
    Scratch scratch;
    hipGraphExec_t exec = nullptr;
    hipStream_t priv = nullptr;  // capture and replay stream (default priority)
    std::vector<void*> vouts;
    gbf_opts key_opts{};
    bool graph_failed = false;
    ~BatchCtx() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (priv) (void)hipStreamDestroy(priv);
    }
};
// Batch contexts by the ordered set of handles.  One lock guards the map;
// a batch call holds it for its whole duration (a context's scratch and
// graph are not shared between concurrent calls).
// The map is created on first use and never destroyed by a static
// destructor: destructors of library-scope objects run at process exit,
// possibly after the HIP runtime (or a profiler attached to it) has shut
// down, and a HIP call from there faults.  gbf_shutdown releases the
// contexts explicitly while the runtime is still up.
using BatchMap = std::map<std::vector<gbf_graph*>, std::unique_ptr<BatchCtx>>;
static BatchMap& g_batches_map() {
    static BatchMap* m = new BatchMap();
    return *m;
}
#define g_batches (g_batches_map())
static std::mutex g_batches_lock;

extern "C" void gbf_shutdown(void) {
    std::lock_guard<std::mutex> lk(g_batches_lock);
    for (auto& kv : g_batches)
        if (kv.second->priv) (void)hipStreamSynchronize(kv.second->priv);
    g_batches.clear();
}

static void forget_batches_of(gbf_graph* g) {
    std::lock_guard<std::mutex> lk(g_batches_lock);
    for (auto it = g_batches.begin(); it != g_batches.end();) {
        if (std::find(it->first.begin(), it->first.end(), g) != it->first.end()) {
            if (it->second->priv) (void)hipStreamSynchronize(it->second->priv);
            it = g_batches.erase(it);
        } else {
            ++it;
        }
    }
}

static bool same_opts(const gbf_opts& a, const gbf_opts& b) {
    return a.mode == b.mode && a.max_rounds == b.max_rounds && a.lanes == b.lanes && a.grid == b.grid &&
           a.v_memspace == b.v_memspace;
}

static int capture_batch(BatchCtx& ctx, const Plan& P, const Inst* insts, void* const* V_outs,
                         hipStream_t s) {
    Scratch& S = ctx.scratch;
    hipGraph_t graph = nullptr;
    HIPC(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    int rc = enqueue_init(S, P, insts, s);
    hipError_t e = hipSuccess;
    if (!rc) e = launch_persistent(S.dinst, P.R, P.grid, P.lanes, P.dtype, P.enc_mask, true, s);
    if (!rc && e == hipSuccess) rc = enqueue_readback(S, P, s);
    if (!rc && e == hipSuccess)
        for (int i = 0; i < P.ninst; ++i)
            if (V_outs && V_outs[i]) {
                e = launch_decode(insts[i], P.dtype, V_outs[i], s);
                if (e != hipSuccess) break;
            }
    hipError_t e2 = hipStreamEndCapture(s, &graph);
    if (rc || e != hipSuccess || e2 != hipSuccess || !graph) {
        if (graph) (void)hipGraphDestroy(graph);
        (void)hipGetLastError();
        return fail(GBF_EHIP, std::string("graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    }
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(GBF_EHIP, std::string("graph instantiation failed: ") + hipGetErrorString(e));
    if (ctx.exec) (void)hipGraphExecDestroy(ctx.exec);
    ctx.exec = exec;
    return GBF_OK;
}

extern "C" int gbf_solve_batch(gbf_graph* const* graphs, int32_t count, const gbf_opts* opts, void* const* V_outs,
                               gbf_stats* st) {
    if (!graphs || count <= 0) return fail(GBF_EINVAL, "empty batch");
    if (count > kMaxBatch) return fail(GBF_EINVAL, "batch larger than " + std::to_string(kMaxBatch));
    for (int i = 0; i < count; ++i)
        if (graphs[i] && graphs[i]->enc == 3)
            return fail(GBF_EINVAL, "an aircraft abstraction is solved with gbf_solve");
    gbf_opts o = opts ? *opts : default_opts();
    if (o.order != GBF_ORDER_PLAIN) return fail(GBF_EINVAL, "batched solves use the plain order");
    if (o.v_memspace != GBF_HOST && o.v_memspace != GBF_DEVICE) return fail(GBF_EINVAL, "bad v_memspace");
    for (int i = 0; i < count; ++i)
        if (!graphs[i]) return fail(GBF_EINVAL, "NULL graph in batch");
    const int dtype = graphs[0]->dtype;
    hipStream_t s = graphs[0]->stream;
    for (int i = 0; i < count; ++i) {
        if (graphs[i]->dtype != dtype) return fail(GBF_EINVAL, "batch mixes value types");
        if (graphs[i]->stream != s || graphs[i]->device != graphs[0]->device)
            return fail(GBF_EINVAL, "batch spans streams or devices");
    }
    std::vector<gbf_graph*> key(graphs, graphs + count);
    std::lock_guard<std::mutex> lk(g_batches_lock);
    auto& ctx = g_batches[key];
    if (!ctx) {
        ctx.reset(new BatchCtx());
        ctx->graphs = key;
    }
    std::vector<Inst> insts;
    int64_t base = 0;
    for (int i = 0; i < count; ++i) {
        Inst I = graphs[i]->inst;
        I.pair_base = base;
        I.index = i;
        I.max_rounds = o.max_rounds > 0 ? o.max_rounds : I.n;
        base += I.n * I.K;
        insts.push_back(I);
        graphs[i]->solved = false;
    }
    if (base >= ((int64_t)1 << 32)) return fail(GBF_EINVAL, "batch has >= 2^32 pairs");
    Scratch& S = ctx->scratch;
    SolveOut so;
    Plan P;
    int rc = plan_solve(S, insts.data(), count, dtype, o, graphs[0]->cus, graphs[0]->clock_khz, P);
    if (rc) return rc;
    const bool graphable = P.mode == GBF_MODE_PERSISTENT && o.v_memspace == GBF_DEVICE && !o.profile;
    bool replayed = false;
    if (graphable && !ctx->graph_failed && !ctx->priv) {
        // the caller's stream may be the legacy default stream, which cannot
        // be captured: capture and replay on a stream of our own
        if (hipStreamCreateWithFlags(&ctx->priv, hipStreamNonBlocking) != hipSuccess) {
            ctx->priv = nullptr;
            ctx->graph_failed = true;
        }
    }
    if (graphable && !ctx->graph_failed) {
        hipStream_t gs = ctx->priv;
        // inputs and outputs are ordered on the caller's stream
        HIPC(hipStreamSynchronize(s));
        std::vector<void*> vo(V_outs ? V_outs : nullptr, V_outs ? V_outs + count : nullptr);
        const bool fresh = !ctx->exec || vo != ctx->vouts || !same_opts(o, ctx->key_opts);
        if (fresh) {
            HIPC(hipMemcpyAsync(S.dinst, insts.data(), sizeof(Inst) * count, hipMemcpyHostToDevice, gs));
            HIPC(hipStreamSynchronize(gs));
            if (capture_batch(*ctx, P, insts.data(), V_outs, gs) != GBF_OK) {
                ctx->graph_failed = true;  // fall back to direct launches
                (void)hipGetLastError();
            } else {
                ctx->vouts = vo;
                ctx->key_opts = o;
            }
        }
        if (!ctx->graph_failed) {
            HIPC(hipEventRecord(S.events[0], gs));
            HIPC(hipGraphLaunch(ctx->exec, gs));
            HIPC(hipEventRecord(S.events[1], gs));
            HIPC(hipStreamSynchronize(gs));
            if (((int32_t*)S.host)[1] != 0) {
                if (o.mode != GBF_MODE_AUTO) return fail(GBF_ETIMEOUT, "grid barrier timed out");
            } else {
                read_host(S, P, so, true, graphs[0]->clock_khz);
                so.graph = 1;
                replayed = true;
            }
        }
    }
    if (!replayed) {
        gbf_opts o2 = o;
        if (graphable && o.mode == GBF_MODE_AUTO && ((int32_t*)S.host)[1] != 0) o2.mode = GBF_MODE_HOSTLOOP;
        rc = run_rounds(S, insts.data(), count, dtype, o2, s, graphs[0]->cus, graphs[0]->clock_khz, so);
        if (rc) return rc;
        for (int i = 0; i < count; ++i) {
            if (!V_outs || !V_outs[i]) continue;
            if (o.v_memspace == GBF_DEVICE) {
                HIPC(launch_decode(insts[i], dtype, V_outs[i], s));
            } else {
                HIPC(launch_decode(insts[i], dtype, S.list, s));
                HIPC(hipMemcpyAsync(V_outs[i], S.list, insts[i].n * 4, hipMemcpyDeviceToHost, s));
            }
        }
        HIPC(hipEventRecord(S.events[1], s));
        HIPC(hipEventSynchronize(S.events[1]));
    }
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, S.events[0], S.events[1]));
    so.solve_ms = ms;
    int worst = GBF_OK;
    for (int i = 0; i < count; ++i) {
        const int status = so.inst_status[i] ? GBF_ENEGCYCLE : GBF_OK;
        if (status != GBF_OK) worst = status;
        graphs[i]->solved = true;
        if (st) fill_stats(st + i, status, so, insts[i].max_rounds, graphs[i]->mem.bytes, graphs[i]->enc);
    }
    if (worst != GBF_OK) fail(worst, "round cap reached in some instance");
    return worst;
}

// ------------------------------------------------------------------ autotuner
// Times every candidate launch configuration on the given handles and keeps
// the fastest: lanes per listed pair {2, 4, 8} x relax grid {4, 8, 16}
// blocks per CU in host-loop mode, and lanes {2, 4, 8} in persistent mode
// (its grid is fixed by co-residency).  Each candidate runs one untimed and
// `reps` timed solves; the median HIP-event solve time decides.  Candidates
// that fail (e.g. a persistent grid that is not co-resident) are skipped.
extern "C" int gbf_tune(gbf_graph* const* graphs, int32_t count, const gbf_opts* base, int32_t reps,
                        gbf_opts* best, double* best_ms) {
    if (!graphs || count <= 0 || !best) return fail(GBF_EINVAL, "NULL graphs or output, or empty set");
    for (int i = 0; i < count; ++i) {
        if (!graphs[i]) return fail(GBF_EINVAL, "NULL graph");
        if (graphs[i]->enc == 3) return fail(GBF_EINVAL, "an aircraft abstraction has no launch options to tune");
    }
    if (reps <= 0) reps = 3;
    gbf_opts o = base ? *base : default_opts();
    o.profile = 0;
    o.v_memspace = GBF_DEVICE;
    const int cus = graphs[0]->cus;
    struct Cand {
        int mode, lanes, grid, block, cgrid;
    };
    if (o.mode != GBF_MODE_AUTO && o.mode != GBF_MODE_HOSTLOOP && o.mode != GBF_MODE_PERSISTENT &&
        o.mode != GBF_MODE_SINGLE_BLOCK)
        return fail(GBF_EINVAL, "unknown mode");
    const bool any = o.mode == GBF_MODE_AUTO;
    std::vector<Cand> cands;
    if (any || o.mode == GBF_MODE_HOSTLOOP)
        for (int lanes : {2, 4, 8})
            for (int per_cu : {4, 8, 16})
                for (int block : {256, 512, 1024}) cands.push_back({GBF_MODE_HOSTLOOP, lanes, per_cu * cus, block, 0});
    if (o.order == GBF_ORDER_PLAIN && (any || o.mode == GBF_MODE_PERSISTENT))
        for (int lanes : {2, 4, 8}) cands.push_back({GBF_MODE_PERSISTENT, lanes, 0, 0, 0});
    // one workgroup is only worth timing on small single instances
    if (o.order == GBF_ORDER_PLAIN && count == 1 && graphs[0]->n * graphs[0]->K <= 4 * kSingleBlockMaxPairs &&
        (any || o.mode == GBF_MODE_SINGLE_BLOCK))
        for (int lanes : {2, 4, 8}) cands.push_back({GBF_MODE_SINGLE_BLOCK, lanes, 0, 0, 0});
    if (cands.empty()) return fail(GBF_EINVAL, "no candidate configuration for this mode and order");
    double best_t = 1e300;
    gbf_opts bo = o;
    bool found = false;
    std::vector<gbf_stats> st(count);
    // second pass: the compaction grid of the best host-loop configuration
    bool second = false;
    for (size_t ci = 0; ci < cands.size(); ++ci) {
        const Cand c = cands[ci];  // a copy: the second pass appends to cands
        gbf_opts t = o;
        t.mode = c.mode;
        t.lanes = c.lanes;
        t.grid = c.grid;
        t.block = c.block;
        t.compact_grid = c.cgrid;
        std::vector<double> ms;
        bool ok = true;
        for (int r = 0; r <= reps && ok; ++r) {
            int rc = count == 1 ? gbf_solve(graphs[0], &t, nullptr, st.data())
                                : gbf_solve_batch(graphs, count, &t, nullptr, st.data());
            if (rc < 0) ok = false;
            else if (r > 0) ms.push_back(st[0].solve_ms);
        }
        if (!ok) continue;
        std::sort(ms.begin(), ms.end());
        const double med = ms[ms.size() / 2];
        if (med < best_t) {
            best_t = med;
            bo = t;
            found = true;
        }
        if (ci + 1 == cands.size() && !second && found && bo.mode == GBF_MODE_HOSTLOOP) {
            second = true;
            for (int cg : {256, 1024}) cands.push_back({GBF_MODE_HOSTLOOP, bo.lanes, bo.grid, bo.block, cg});
        }
    }
    if (!found) return fail(GBF_EHIP, "no candidate configuration ran");
    bo.v_memspace = base ? base->v_memspace : GBF_HOST;
    bo.profile = base ? base->profile : 0;
    *best = bo;
    if (best_ms) *best_ms = best_t;
    return GBF_OK;
}
