// C ABI of the gbf solver: loader, single and batched solve drivers, policy
// extraction.  All device work is issued on the handle's HIP stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "gbf.h"
#include "gbf_internal.h"

using namespace gbf;

static thread_local std::string t_err;

// Blocks per CU of the persistent kernel: below the occupancy limit, so that
// the cooperative grid is co-resident with margin.
constexpr int kPersistentBlocksPerCU = 1;

static int fail(int code, const std::string& msg) {
    t_err = msg;
    return code;
}

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
    uint8_t* dirty[2] = {nullptr, nullptr};
    uint32_t* list = nullptr;
    uint32_t* counts = nullptr;
    unsigned long long* ctr = nullptr;
    unsigned long long* slots = nullptr;
    int32_t* inst_status = nullptr;
    uint32_t* barrier = nullptr;
    int32_t* error = nullptr;
    int32_t* result = nullptr;
    Inst* dinst = nullptr;
    int ninst_cap = 0;
    void* host = nullptr;  // pinned readback area
    size_t host_bytes = 0;
    std::vector<hipEvent_t> events;
    DevMem mem;
    ~Scratch() {
        if (host) (void)hipHostFree(host);
        for (auto e : events) (void)hipEventDestroy(e);
    }
};

struct gbf_graph {
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
    Scratch scratch;
};

static int ensure_scratch(Scratch& S, int64_t total_pairs, int64_t max_rounds, int ninst, int nevents) {
    const int64_t nchunks = (total_pairs + 15) / 16;
    if (S.total_pairs < total_pairs) {
        if (S.dirty[0]) S.mem.release(S.dirty[0], 0), S.mem.release(S.dirty[1], 0), S.mem.release(S.list, 0);
        int rc;
        if ((rc = S.mem.alloc((void**)&S.dirty[0], nchunks * 16))) return rc;
        if ((rc = S.mem.alloc((void**)&S.dirty[1], nchunks * 16))) return rc;
        if ((rc = S.mem.alloc((void**)&S.list, total_pairs * 4))) return rc;
        S.total_pairs = total_pairs;
    }
    if (S.counts_cap < max_rounds + 2) {
        if (S.counts) S.mem.release(S.counts, 0);
        int rc;
        if ((rc = S.mem.alloc((void**)&S.counts, (max_rounds + 2) * 4))) return rc;
        S.counts_cap = max_rounds + 2;
    }
    if (!S.ctr) {
        int rc;
        if ((rc = S.mem.alloc((void**)&S.ctr, 8 * sizeof(unsigned long long)))) return rc;
        if ((rc = S.mem.alloc((void**)&S.slots, (size_t)kMaxGrid * 8 * sizeof(unsigned long long)))) return rc;
        if ((rc = S.mem.alloc((void**)&S.barrier, 64))) return rc;
        if ((rc = S.mem.alloc((void**)&S.error, 64))) return rc;
        if ((rc = S.mem.alloc((void**)&S.result, 64))) return rc;
    }
    if (S.ninst_cap < ninst) {
        if (S.dinst) S.mem.release(S.dinst, 0), S.mem.release(S.inst_status, 0);
        int rc;
        if ((rc = S.mem.alloc((void**)&S.dinst, sizeof(Inst) * ninst))) return rc;
        if ((rc = S.mem.alloc((void**)&S.inst_status, 4 * ninst))) return rc;
        S.ninst_cap = ninst;
    }
    const size_t hb = 4096 + 4 * (size_t)ninst + 1024;
    if (S.host_bytes < hb) {
        if (S.host) (void)hipHostFree(S.host);
        S.host = nullptr;
        if (hipHostMalloc(&S.host, hb, hipHostMallocDefault) != hipSuccess)
            return fail(GBF_ENOMEM, "hipHostMalloc failed");
        S.host_bytes = hb;
    }
    while ((int)S.events.size() < nevents) {
        hipEvent_t e;
        HIPC(hipEventCreate(&e));
        S.events.push_back(e);
    }
    return GBF_OK;
}

// ------------------------------------------------------------------ load
extern "C" int gbf_load_graph(const gbf_problem* p, void* hip_stream, gbf_graph** out) {
    if (!out) return fail(GBF_EINVAL, "out is NULL");
    *out = nullptr;
    if (!p) return fail(GBF_EINVAL, "problem is NULL");
    if (p->n_states <= 0 || p->n_inputs <= 0) return fail(GBF_EINVAL, "n_states and n_inputs must be positive");
    if (p->dtype != GBF_I32 && p->dtype != GBF_F32) return fail(GBF_EINVAL, "dtype must be GBF_I32 or GBF_F32");
    if (p->encoding != GBF_CSR && p->encoding != GBF_BOX) return fail(GBF_EINVAL, "bad encoding");
    if (p->memspace != GBF_HOST && p->memspace != GBF_DEVICE) return fail(GBF_EINVAL, "bad memspace");
    if (!p->G || !p->g) return fail(GBF_EINVAL, "G and g are required");
    const int64_t n = p->n_states, K = p->n_inputs, np = n * K;
    if (np >= (int64_t)1 << 31) return fail(GBF_EINVAL, "n_states * n_inputs must be < 2^31");
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
    int32_t *G, *g, *stamp, *err;
    uint8_t* avoid;
    void* V;
    if ((rc = M.alloc((void**)&G, n * 4)) || (rc = M.alloc((void**)&g, np * 4)) ||
        (rc = M.alloc((void**)&avoid, n)) || (rc = M.alloc(&V, n * 4)) || (rc = M.alloc((void**)&stamp, n * 4)) ||
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
    I.stamp = stamp;

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
        return fail(GBF_EINVAL, msg);
    }

    if (p->encoding == GBF_CSR) {
        HIPC(launch_convert_ptr(sptr64, const_cast<uint32_t*>(I.sptr), np + 1, s));
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
        M.release(sptr64, (np + 1) * 8);
        M.release(cnt, (n + 1) * 4);
        M.release(tmp, nb * 4);
    } else {
        HIPC(launch_prune(I, p->dtype, s));
        int32_t* win;
        if ((rc = M.alloc((void**)&win, K * 8 * 4))) return rc;
        std::vector<int32_t> init(K * 8);
        for (int64_t u = 0; u < K; ++u)
            for (int a = 0; a < 4; ++a) {
                init[u * 8 + a] = 0x7fffffff;
                init[u * 8 + 4 + a] = (int32_t)0x80000000;
            }
        HIPC(hipMemcpyAsync(win, init.data(), K * 8 * 4, hipMemcpyHostToDevice, s));
        HIPC(launch_box_window(I, win, s));
        HIPC(hipStreamSynchronize(s));
        I.win = win;
    }
    M.release(err, 64);
    *out = gr.release();
    return GBF_OK;
}

extern "C" void gbf_free_graph(gbf_graph* g) {
    if (!g) return;
    (void)hipStreamSynchronize(g->stream);
    delete g;
}

extern "C" const char* gbf_last_error(void) { return t_err.c_str(); }

// ------------------------------------------------------------------ solve core
struct SolveOut {
    int64_t rounds = 0;
    unsigned long long ctr[6] = {0, 0, 0, 0, 0, 0};
    double solve_ms = 0, relax_ms = 0;
    int64_t relax_launches = 0;
    int mode = 0, grid = 0, block = 0, lanes = 0;
    std::vector<int32_t> inst_status;
};

// Runs the frontier iteration over `insts` (already initialised device
// table `S.dinst`).  Host-loop mode: compact + relax per round, the host reads
// the per-round frontier sizes in growing batches.  Persistent mode: one
// cooperative launch runs every round with grid barriers.
static int run_rounds(Scratch& S, const std::vector<Inst>& insts, int dtype, const gbf_opts& o, hipStream_t s,
                      int cus, int clock_khz, SolveOut& out) {
    const int ninst = (int)insts.size();
    int64_t total_pairs = 0, max_rounds = 0, max_states = 0;
    int enc_mask = 0;
    for (const Inst& I : insts) {
        total_pairs = std::max<int64_t>(total_pairs, I.pair_base + I.n * I.K);
        max_rounds = std::max<int64_t>(max_rounds, I.max_rounds);
        max_states = std::max<int64_t>(max_states, I.n);
        enc_mask |= I.enc == 0 ? 1 : 2;
    }
    const int nevents = o.profile ? 2 * (int)std::min<int64_t>(max_rounds + 2, 4096) + 2 : 2;
    int rc = ensure_scratch(S, total_pairs, max_rounds, ninst, nevents);
    if (rc) return rc;
    Run R{};
    R.dirty[0] = S.dirty[0];
    R.dirty[1] = S.dirty[1];
    R.list = S.list;
    R.counts = S.counts;
    R.ctr = S.ctr;
    R.slots = S.slots;
    R.inst_status = S.inst_status;
    R.barrier = S.barrier;
    R.error = S.error;
    R.result = S.result;
    R.nchunks = (total_pairs + 15) / 16;
    R.total_pairs = total_pairs;
    R.max_rounds = max_rounds;
    R.ninst = ninst;
    R.dtype = dtype;
    // a single barrier wait longer than 250 ms means the blocks are not
    // co-resident (or the device is stuck): give up instead of hanging
    R.timeout_ticks = (uint64_t)clock_khz * 250;

    HIPC(hipEventRecord(S.events[0], s));
    HIPC(hipMemcpyAsync(S.dinst, insts.data(), sizeof(Inst) * ninst, hipMemcpyHostToDevice, s));
    HIPC(launch_fill_u32((uint32_t*)R.dirty[0], 0, R.nchunks * 4, s));
    HIPC(launch_fill_u32((uint32_t*)R.dirty[1], 0, R.nchunks * 4, s));
    HIPC(launch_fill_u32(R.counts, 0, max_rounds + 2, s));
    HIPC(launch_fill_u32((uint32_t*)R.ctr, 0, 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.slots, 0, (int64_t)kMaxGrid * 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.inst_status, 0, ninst, s));
    HIPC(launch_fill_u32(R.barrier, 0, 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.error, 0, 16, s));
    HIPC(launch_fill_u32((uint32_t*)R.result, 0, 16, s));
    for (const Inst& I : insts) HIPC(launch_init(S.dinst, I, dtype, s));
    HIPC(launch_seed(S.dinst, ninst, R, max_states, dtype, enc_mask, s));

    int mode = o.mode;
    int per_cu = 0;
    const int lanes = (o.lanes == 1 || o.lanes == 2 || o.lanes == 4 || o.lanes == 8 || o.lanes == 16 ||
                       o.lanes == 32)
                          ? o.lanes
                          : 4;
    out.lanes = lanes;
    if (mode != GBF_MODE_HOSTLOOP) {
        per_cu = persistent_blocks_per_cu(R, lanes, dtype, enc_mask);
        if (per_cu <= 0) {
            if (mode == GBF_MODE_PERSISTENT) return fail(GBF_EHIP, "occupancy query failed");
            mode = GBF_MODE_HOSTLOOP;
        } else if (mode == GBF_MODE_AUTO) {
            // measured on MI355X: one launch pair per round beats the
            // cooperative kernel for single instances (its grid barriers
            // write back and invalidate L2); batches use the persistent form
            mode = ninst > 1 ? GBF_MODE_PERSISTENT : GBF_MODE_HOSTLOOP;
        }
    }
    int32_t* host = (int32_t*)S.host;
    if (mode == GBF_MODE_PERSISTENT) {
        // co-residency is required; stay below the occupancy limit
        const int cap = std::min(per_cu, kPersistentBlocksPerCU) * cus;
        int grid = o.grid > 0 ? std::min(o.grid, cap) : cap;
        out.grid = grid;
        out.block = 256;
        if (o.profile) HIPC(hipEventRecord(S.events[2], s));
        HIPC(launch_persistent(S.dinst, R, grid, lanes, dtype, enc_mask, s));
        if (o.profile) HIPC(hipEventRecord(S.events[3], s));
        HIPC(hipMemcpyAsync(host, S.result, 4, hipMemcpyDeviceToHost, s));
        HIPC(hipMemcpyAsync(host + 1, S.error, 4, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        if (host[1] != 0) {
            if (o.mode == GBF_MODE_AUTO) {
                // retry the whole solve with one launch sequence per round
                gbf_opts o2 = o;
                o2.mode = GBF_MODE_HOSTLOOP;
                out = SolveOut();
                return run_rounds(S, insts, dtype, o2, s, cus, clock_khz, out);
            }
            return fail(GBF_ETIMEOUT, "grid barrier timed out (blocks not co-resident?)");
        }
        out.rounds = host[0];
        if (o.profile) {
            float ms = 0;
            HIPC(hipEventElapsedTime(&ms, S.events[2], S.events[3]));
            out.relax_ms = ms;
            out.relax_launches = 1;
        }
    } else {
        const int grid = o.grid > 0 ? std::min(o.grid, kMaxGrid) : 8 * cus;
        out.grid = grid;
        out.block = 256;
        int64_t r = 0;
        int64_t batch = o.batch_hint > 0 ? o.batch_hint : 8;
        int ev = 2;
        bool done = false;
        // the round after the last allowed one only flags capped instances,
        // so a zero count appears at round max_rounds + 1 at the latest
        while (!done && r <= max_rounds + 1) {
            const int64_t nb = std::min<int64_t>(batch, max_rounds + 2 - r);
            for (int64_t k = 0; k < nb; ++k) {
                HIPC(launch_compact(R, (int)(r + k), 0, s));
                const bool timed = o.profile && ev + 1 < (int)S.events.size();
                if (timed) HIPC(hipEventRecord(S.events[ev], s));
                HIPC(launch_relax(S.dinst, R, (int)(r + k), grid, lanes, dtype, enc_mask, s));
                if (timed) {
                    HIPC(hipEventRecord(S.events[ev + 1], s));
                    ev += 2;
                }
            }
            const int64_t nread = std::min<int64_t>(nb, 1000);
            HIPC(hipMemcpyAsync(host, R.counts + r, nread * 4, hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            for (int64_t k = 0; k < nread; ++k)
                if (host[k] == 0) {
                    out.rounds = r + k;
                    done = true;
                    break;
                }
            r += nb;
            // speculative rounds after the frontier drains cost a launch
            // each, host reads cost a round trip: grow the batch moderately
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
    }
    out.mode = mode;
    out.inst_status.assign(ninst, 0);
    HIPC(launch_sum_slots(S.slots, kMaxGrid, S.ctr, s));
    HIPC(hipMemcpyAsync(host + 16, S.ctr, 6 * sizeof(unsigned long long), hipMemcpyDeviceToHost, s));
    HIPC(hipMemcpyAsync(host + 64, S.inst_status, 4 * ninst, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    std::memcpy(out.ctr, host + 16, 6 * sizeof(unsigned long long));
    for (int i = 0; i < ninst; ++i) out.inst_status[i] = host[64 + i];
    return GBF_OK;
}

static gbf_opts default_opts() {
    gbf_opts o;
    std::memset(&o, 0, sizeof(o));
    return o;
}

static void fill_stats(gbf_stats* st, int status, const SolveOut& so, int64_t rounds_cap, size_t bytes) {
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
    st->device_bytes = (int64_t)bytes;
    st->mode_used = so.mode;
    st->grid_used = so.grid;
    st->block_used = so.block;
    st->lanes_used = so.lanes;
}

static int write_values(gbf_graph* g, void* V_out, int memspace, hipStream_t s) {
    if (!V_out) return GBF_OK;
    if (memspace == GBF_DEVICE) {
        HIPC(launch_decode(g->inst, g->dtype, V_out, s));
    } else {
        // decode in place into the scratch list buffer, then copy out
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
    std::vector<Inst> insts{I};
    SolveOut so;
    int rc = run_rounds(g->scratch, insts, g->dtype, o, s, g->cus, g->clock_khz, so);
    if (rc) return rc;
    if ((rc = write_values(g, V_out, o.v_memspace, s))) return rc;
    HIPC(hipEventRecord(g->scratch.events[1], s));
    HIPC(hipEventSynchronize(g->scratch.events[1]));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, g->scratch.events[0], g->scratch.events[1]));
    so.solve_ms = ms;
    const int status = so.inst_status[0] ? GBF_ENEGCYCLE : GBF_OK;
    fill_stats(st, status, so, I.max_rounds, g->mem.bytes + g->scratch.mem.bytes);
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
    unsigned long long* bad = S.ctr + 4;
    HIPC(launch_fill_u32((uint32_t*)bad, 0, 2, s));
    int32_t* dst = memspace == GBF_DEVICE ? policy_out : (int32_t*)S.list;
    HIPC(launch_policy(g->inst, g->dtype, dst, bad, s));
    if (memspace != GBF_DEVICE) HIPC(hipMemcpyAsync(policy_out, dst, g->n * 4, hipMemcpyDeviceToHost, s));
    unsigned long long* hb = (unsigned long long*)((char*)S.host + 64);
    HIPC(hipMemcpyAsync(hb, bad, 8, hipMemcpyDeviceToHost, s));
    HIPC(hipStreamSynchronize(s));
    if (residual) *residual = (int64_t)*hb;
    return GBF_OK;
}

// ------------------------------------------------------------------ batch
struct BatchCtx {
    std::vector<gbf_graph*> graphs;
    Scratch scratch;
};
static std::map<std::vector<gbf_graph*>, std::unique_ptr<BatchCtx>> g_batches;

extern "C" int gbf_solve_batch(gbf_graph* const* graphs, int32_t count, const gbf_opts* opts, void* const* V_outs,
                               gbf_stats* st) {
    if (!graphs || count <= 0) return fail(GBF_EINVAL, "empty batch");
    if (count > kMaxBatch) return fail(GBF_EINVAL, "batch larger than " + std::to_string(kMaxBatch));
    gbf_opts o = opts ? *opts : default_opts();
    if (o.order != GBF_ORDER_PLAIN) return fail(GBF_EINVAL, "batched solves use the plain order");
    const int dtype = graphs[0]->dtype;
    hipStream_t s = graphs[0]->stream;
    for (int i = 0; i < count; ++i) {
        if (!graphs[i]) return fail(GBF_EINVAL, "NULL graph in batch");
        if (graphs[i]->dtype != dtype) return fail(GBF_EINVAL, "batch mixes value types");
        if (graphs[i]->stream != s || graphs[i]->device != graphs[0]->device)
            return fail(GBF_EINVAL, "batch spans streams or devices");
    }
    std::vector<gbf_graph*> key(graphs, graphs + count);
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
    SolveOut so;
    int rc = run_rounds(ctx->scratch, insts, dtype, o, s, graphs[0]->cus, graphs[0]->clock_khz, so);
    if (rc) return rc;
    for (int i = 0; i < count; ++i) {
        if (!V_outs || !V_outs[i]) continue;
        if (o.v_memspace == GBF_DEVICE) {
            HIPC(launch_decode(insts[i], dtype, V_outs[i], s));
        } else {
            HIPC(launch_decode(insts[i], dtype, ctx->scratch.list, s));
            HIPC(hipMemcpyAsync(V_outs[i], ctx->scratch.list, insts[i].n * 4, hipMemcpyDeviceToHost, s));
        }
    }
    HIPC(hipEventRecord(ctx->scratch.events[1], s));
    HIPC(hipEventSynchronize(ctx->scratch.events[1]));
    float ms = 0;
    HIPC(hipEventElapsedTime(&ms, ctx->scratch.events[0], ctx->scratch.events[1]));
    so.solve_ms = ms;
    int worst = GBF_OK;
    for (int i = 0; i < count; ++i) {
        const int status = so.inst_status[i] ? GBF_ENEGCYCLE : GBF_OK;
        if (status != GBF_OK) worst = status;
        graphs[i]->solved = true;
        if (st) {
            SolveOut si = so;
            fill_stats(st + i, status, si, insts[i].max_rounds, graphs[i]->mem.bytes);
        }
    }
    if (worst != GBF_OK) fail(worst, "round cap reached in some instance");
    return worst;
}
