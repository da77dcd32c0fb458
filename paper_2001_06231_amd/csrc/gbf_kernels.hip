// HIP kernels of the gbf solver for gfx950 (CDNA4, wave64).
//
// The hot path is one pass of the while loop of Algorithm 1 (Sect. IV-A),
// restated for a data-parallel machine:
//   compact : the dirty-pair byte map of the active frontier is turned into
//             an ascending list of pair ids (per-thread 16-byte chunks, wave
//             prefix sums staged in LDS, one global atomic per block) and
//             the listed bytes are cleared;
//   relax   : G lanes per listed pair (x,u) form the max of W over F(x,u)
//             (a CSR row, or the rows of a box along axis 0) and reduce it
//             with lane shuffles; d = g(x,u) + max is reduced to one
//             candidate per state of a wave step and applied by atomicMin on
//             order-preserving words (the strict-improvement update);
//   expand  : every improved state marks, with plain byte stores, each pair
//             (x',u') that has it in F(x',u') in the next frontier's byte map
//             (the reverse CSR row of the state, or the per-input predecessor
//             windows of the box encoding; pair-level pred of Sect. IV-A).
// Pairs are the frontier's unit (not states as in the paper's F1 x U): a pair
// whose successors did not change cannot improve, so only pairs with a
// changed successor are evaluated.  Any evaluation order reaches the same
// maximal fixed point (Sect. IV-A: the processing order is irrelevant; the
// operator is monotone and every pair is re-evaluated after its last
// successor change).  That is also what lets the bucket order (a schedule
// over the byte map driven by per-state keys) change only the work, never
// the result.
#include <cstring>
#include <type_traits>

#include "gbf_device.h"
#include "gbf_internal.h"

// Compile-time tuning knobs (measured defaults).
#ifndef GBF_NT_ROWS
#define GBF_NT_ROWS 0  // streaming (non-temporal) loads for successor rows
#endif
#ifndef GBF_NT_MISC
#define GBF_NT_MISC 0  // ... for list entries, row bounds, costs, reverse rows
#endif
#ifndef GBF_PBLOCKS
#define GBF_PBLOCKS 2  // persistent kernel: 1024-thread blocks per CU
#endif
#ifndef GBF_PHYB
#define GBF_PHYB 2  // persistent kernel, box successors with a reverse CSR: 1024-thread blocks per CU
#endif
#ifndef GBF_PEDGE
#define GBF_PEDGE 2  // persistent kernel, CSR with per-edge costs: 1024-thread blocks per CU
#endif
#ifndef GBF_EXP_BATCH
#define GBF_EXP_BATCH 4  // reverse-row slices of 64 loaded together when expanding a state
#endif
#ifndef GBF_ROW_BATCH
#define GBF_ROW_BATCH 6  // successor indices loaded together per lane at most (CSR relax)
#endif
#ifndef GBF_SMALL_LDS
#define GBF_SMALL_LDS 1  // single-block mode on small CSR instances keeps V, frontiers and list in LDS
#endif
#ifndef GBF_ILP
#define GBF_ILP 1  // wave steps whose gathers a host-loop relax wave keeps in flight together (2+ measured slower)
#endif
#ifndef GBF_XCD_MAP
#define GBF_XCD_MAP 1  // host-loop relax: the blocks of each XCD take one contiguous part of the list
#endif
#ifndef GBF_PERSIST_MAP
#define GBF_PERSIST_MAP 1  // persistent kernel, one instance: the host-loop relax's mapping of the list
#endif
#ifndef GBF_EDGE_BATCH
#define GBF_EDGE_BATCH 4  // successor indices and edge costs loaded together per lane (per-edge costs)
#endif
#ifndef GBF_XCD_BARRIER
#define GBF_XCD_BARRIER 1  // persistent kernel: one L2 write-back per XCD and barrier
#endif
#ifndef GBF_COMPACT_GRID
#define GBF_COMPACT_GRID 512  // blocks of a host-loop compaction
#endif

namespace gbf {

constexpr int kExpBatch = GBF_EXP_BATCH;
constexpr int kRowBatch = GBF_ROW_BATCH;
constexpr int kEdgeBatch = GBF_EDGE_BATCH;
constexpr int kXcdParts = 8;  // XCDs of an MI355X
constexpr int kILP = GBF_ILP;

template <bool NT, class P>
__device__ __forceinline__ P ldx(const GBF_GLOBAL P* p) {
    if (NT) return __builtin_nontemporal_load(p);
    return *p;
}

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;


// Per-lane statistics (32-bit; folded into the wave's 64-bit LDS slot after
// every round, so they cannot overflow).
struct Acc {
    uint32_t pairs = 0, edges = 0, impr = 0, sat = 0, expanded = 0, marks = 0;
};

// Statistics: each block owns kCtrSlot counters in R.slots (block index
// slot), reduced once at the end of a solve; no two blocks of one launch
// touch the same slot, so no atomics (and no contention) are needed.
constexpr int kCtrSlot = 8;

constexpr int kMaxWavesPerBlock = 16;

// Pair-id width.  32-bit ids serve every workload below 2^31 pairs (and
// batches below 2^32); one instance with more pairs runs with 64-bit ids
// (host loop, BOX or HYB encoding): its frontier list and per-round counts
// are R.list64 / R.counts64.
template <bool WIDE>
struct Ids {
    using id_t = uint32_t;
    using cnt_t = uint32_t;
    __device__ static __forceinline__ id_t* list(const Run& R) { return R.list; }
    __device__ static __forceinline__ cnt_t* counts(const Run& R) { return R.counts; }
};
template <>
struct Ids<true> {
    using id_t = uint64_t;
    using cnt_t = unsigned long long;
    __device__ static __forceinline__ id_t* list(const Run& R) { return R.list64; }
    __device__ static __forceinline__ cnt_t* counts(const Run& R) { return R.counts64; }
};

struct AccLds {
    unsigned long long v[kMaxWavesPerBlock][6];
};

__device__ __forceinline__ void acc_init(AccLds& L) {
    if (lane_id() < 6) L.v[threadIdx.x / kWave][lane_id()] = 0;
}

// Adds this wave's lane counters to its LDS slot and clears them.
__device__ __forceinline__ void fold_acc(Acc& a, AccLds& L) {
    const uint32_t v[6] = {a.pairs, a.edges, a.impr, a.sat, a.expanded, a.marks};
    const int w = threadIdx.x / kWave;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const unsigned long long t = wave_sum64((unsigned long long)v[k]);
        if (lane_id() == 0) L.v[w][k] += t;
    }
    a = Acc();
}

// Block total into the block's slot (the only writer of that slot).
__device__ __forceinline__ void flush_acc(Acc& a, AccLds& L, unsigned long long* slots) {
    fold_acc(a, L);
    __syncthreads();
    if (threadIdx.x < 6) {
        unsigned long long t = 0;
        const int nw = blockDim.x / kWave;
        for (int k = 0; k < nw; ++k) t += L.v[k][threadIdx.x];
        if (t) slots[blockIdx.x * kCtrSlot + threadIdx.x] += t;
    }
}

__global__ void k_sum_slots(const unsigned long long* slots, int nslots, unsigned long long* ctr) {
    __shared__ unsigned long long s[kBlock];
    for (int k = 0; k < 6; ++k) {
        unsigned long long t = 0;
        for (int b = threadIdx.x; b < nslots; b += blockDim.x) t += slots[b * kCtrSlot + k];
        s[threadIdx.x] = t;
        __syncthreads();
        for (int h = kBlock / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) s[threadIdx.x] += s[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) ctr[k] = s[0];
        __syncthreads();
    }
}

hipError_t launch_sum_slots(const unsigned long long* slots, int nslots, unsigned long long* ctr, hipStream_t s) {
    k_sum_slots<<<1, kBlock, 0, s>>>(slots, nslots, ctr);
    return hipGetLastError();
}

template <bool MULTI>
__device__ __forceinline__ int find_inst(const int64_t* bases, int ninst, int64_t q) {
    if (!MULTI) return 0;
    int lo = 0, hi = ninst - 1;
    while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (q >= bases[mid]) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// ------------------------------------------------------------------ fills
__global__ void k_fill_u32(uint32_t* p, uint32_t v, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static int grid_for(int64_t n, int block, int cap = 8192) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (int)b;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_fill_u32<<<grid_for(n, 256), 256, 0, s>>>(p, v, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ loader
// error bits: 1 empty row / bad row pointer, 2 index out of range, 4 NaN or
// -inf cost, 8 finite G on an avoid cell, 16 box outside the grid
__global__ void k_validate(Inst I, const int64_t* sptr64, int64_t m, int dtype, int32_t* err) {
    const int64_t npairs = I.n * I.K;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    int e = 0;
    for (int64_t p = t0; p < npairs; p += stride) {
        if (I.enc == 0) {
            int64_t a = sptr64[p], b = sptr64[p + 1];
            if (b <= a || a < 0 || b > m) {
                e |= 1;
            } else {
                for (int64_t j = a; j < b; ++j) {
                    int32_t y = I.sidx[j];
                    if (y < 0 || y >= I.n) e |= 2;
                    if (I.ge) {
                        const int32_t hr = I.ge[j];
                        // per-edge costs must be finite
                        if (dtype == 1 ? (hr & 0x7f800000) == 0x7f800000 : hr == 0x7fffffff) e |= 32;
                    }
                }
            }
        } else {
            uint64_t bx = I.box[p];
            int64_t lo = (int64_t)(bx & 0xffffffffu);
            if (lo >= I.n) {
                e |= 16;
            } else {
                int64_t r = lo;
                for (int a = 0; a < 4; ++a) {
                    int c = (int)(r % I.dims[a]);
                    r /= I.dims[a];
                    int ex = (int)((bx >> (32 + 8 * a)) & 0xffu);
                    if (c + ex >= I.dims[a]) e |= 16;
                }
            }
        }
        int32_t graw = I.g[p];
        if (dtype == 1) {
            float gv = __int_as_float(graw);
            if (gv != gv || gv == -__builtin_inff()) e |= 4;
        }
    }
    for (int64_t x = t0; x < I.n; x += stride) {
        int32_t Graw = I.G[x];
        bool fin;
        if (dtype == 1) {
            float Gv = __int_as_float(Graw);
            if (Gv != Gv || Gv == -__builtin_inff()) e |= 4;
            fin = Gv != __builtin_inff();
        } else {
            fin = Graw != TI32::INF;
        }
        if (I.avoid && I.avoid[x] && fin) e |= 8;
    }
    if (t0 == 0 && I.enc == 0 && sptr64[0] != 0) e |= 1;
    if (e) atomicOr(err, e);
}

hipError_t launch_validate(const Inst& I, const int64_t* sptr64, int64_t m, int dtype, int32_t* err,
                           hipStream_t s) {
    k_validate<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, sptr64, m, dtype, err);
    return hipGetLastError();
}

__global__ void k_convert_ptr(const int64_t* in, uint32_t* out, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (uint32_t)in[i];
}

hipError_t launch_convert_ptr(const int64_t* in, uint32_t* out, int64_t n, hipStream_t s) {
    k_convert_ptr<<<grid_for(n, 256), 256, 0, s>>>(in, out, n);
    return hipGetLastError();
}

// Box decode helpers
struct BoxDec {
    int64_t lo;
    int e[4];
};
__device__ __forceinline__ BoxDec decode_box(uint64_t b) {
    BoxDec d;
    d.lo = (int64_t)(b & 0xffffffffu);
    d.e[0] = (int)((b >> 32) & 0xffu);
    d.e[1] = (int)((b >> 40) & 0xffu);
    d.e[2] = (int)((b >> 48) & 0xffu);
    d.e[3] = (int)((b >> 56) & 0xffu);
    return d;
}

// Pruning: a pair can improve a value only if g < INF, its state is not an
// avoid cell and no successor is an avoid cell (an avoid successor has
// W = INF forever, so the max over F(x,u) is INF).  Pruned pairs get g = INF.
__global__ void k_prune(Inst I, int dtype) {
    const int64_t npairs = I.n * I.K;
    int32_t* g = const_cast<int32_t*>(I.g);
    const int32_t ginf = dtype == 1 ? 0x7f800000 : TI32::INF;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        if (g[p] == ginf) continue;
        int64_t x = p / I.K;
        bool kill = I.avoid[x] != 0;
        if (!kill) {
            if (I.enc == 0) {
                for (uint32_t j = I.sptr[p]; j < I.sptr[p + 1] && !kill; ++j) kill = I.avoid[I.sidx[j]] != 0;
            } else {
                BoxDec d = decode_box(I.box[p]);
                for (int j3 = 0; j3 <= d.e[3] && !kill; ++j3)
                    for (int j2 = 0; j2 <= d.e[2] && !kill; ++j2)
                        for (int j1 = 0; j1 <= d.e[1] && !kill; ++j1)
                            for (int j0 = 0; j0 <= d.e[0] && !kill; ++j0)
                                kill = I.avoid[d.lo + j0 + (int64_t)j1 * I.strides[1] + (int64_t)j2 * I.strides[2] +
                                               (int64_t)j3 * I.strides[3]] != 0;
            }
        }
        if (kill) g[p] = ginf;
    }
}

hipError_t launch_prune(const Inst& I, int dtype, hipStream_t s) {
    if (!I.avoid) return hipSuccess;
    k_prune<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, dtype);
    return hipGetLastError();
}

__device__ __forceinline__ bool pair_live(const Inst& I, int64_t p, int dtype) {
    int32_t v = I.g[p];
    return dtype == 1 ? v != 0x7f800000 : v != TI32::INF;
}

// reverse CSR, pass 1: in-degree of every state over live pairs
__global__ void k_rev_count(Inst I, int dtype, uint32_t* cnt) {
    const int64_t npairs = I.n * I.K;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        if (!pair_live(I, p, dtype)) continue;
        for (uint32_t j = I.sptr[p]; j < I.sptr[p + 1]; ++j) atomicAdd(cnt + I.sidx[j], 1u);
    }
}

hipError_t launch_rev_count(const Inst& I, uint32_t* cnt, hipStream_t s) {
    k_rev_count<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, I.dtype, cnt);
    return hipGetLastError();
}

// reverse CSR, pass 3: scatter pair ids
__global__ void k_rev_fill(Inst I, int dtype, uint32_t* cursor, uint32_t* rev) {
    const int64_t npairs = I.n * I.K;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        if (!pair_live(I, p, dtype)) continue;
        for (uint32_t j = I.sptr[p]; j < I.sptr[p + 1]; ++j) {
            uint32_t pos = atomicAdd(cursor + I.sidx[j], 1u);
            rev[pos] = (uint32_t)p;
        }
    }
}

hipError_t launch_rev_fill(const Inst& I, uint32_t* cursor, uint32_t* rev, hipStream_t s) {
    k_rev_fill<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, I.dtype, cursor, rev);
    return hipGetLastError();
}

// Sorts every reverse row ascending (bitonic network in LDS, one wave per
// row) so that the pairs a state marks are visited in ascending order and
// marks to the same bitmap word can be combined.  Rows longer than
// kSortCap stay unsorted, which only costs combining, not correctness.
constexpr int kSortCap = 1024;
__global__ __launch_bounds__(kBlock) void k_sort_rows(const uint32_t* __restrict__ rptr, uint32_t* __restrict__ rev,
                                                     int64_t n) {
    __shared__ uint32_t buf[kWavesPerBlock][kSortCap];
    uint32_t* B = buf[threadIdx.x / kWave];
    const int lane = lane_id();
    for (int64_t row = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; row < n;
         row += (int64_t)gridDim.x * kWavesPerBlock) {
        const uint32_t s0 = rptr[row], len = rptr[row + 1] - s0;
        if (len <= 1 || len > (uint32_t)kSortCap) continue;
        uint32_t np2 = 2;
        while (np2 < len) np2 <<= 1;
        for (uint32_t i = lane; i < np2; i += kWave) B[i] = i < len ? rev[s0 + i] : 0xffffffffu;
        wave_sync();
        for (uint32_t k = 2; k <= np2; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = lane; i < np2; i += kWave) {
                    const uint32_t ixj = i ^ j;
                    if (ixj > i) {
                        const uint32_t a = B[i], b = B[ixj];
                        const bool asc = (i & k) == 0;
                        if ((a > b) == asc) {
                            B[i] = b;
                            B[ixj] = a;
                        }
                    }
                }
                wave_sync();
            }
        }
        for (uint32_t i = lane; i < len; i += kWave) rev[s0 + i] = B[i];
        wave_sync();
    }
}

hipError_t launch_sort_rows(const uint32_t* rptr, uint32_t* rev, int64_t n, hipStream_t s) {
    k_sort_rows<<<grid_for((n + kWavesPerBlock - 1) / kWavesPerBlock, 1, 4096), kBlock, 0, s>>>(rptr, rev, n);
    return hipGetLastError();
}


// Exclusive scan of n uint32 into out[0..n] (out[n] = total), three phases.
constexpr int kScanBlock = 1024;
__global__ void k_scan_local(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* blocksum) {
    __shared__ uint32_t s[kScanBlock / kWave];
    const int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
    const uint32_t v = i < n ? in[i] : 0u;
    const uint32_t incl = (uint32_t)wave_incl_scan((int)v);
    const int w = threadIdx.x / kWave;
    if (lane_id() == kWave - 1) s[w] = incl;
    __syncthreads();
    uint32_t wofs = 0;
    for (int k = 0; k < w; ++k) wofs += s[k];
    const uint32_t excl = wofs + incl - v;
    if (i < n) out[i] = excl;
    if (threadIdx.x == kScanBlock - 1) blocksum[blockIdx.x] = excl + v;
}

// single block: exclusive scan of the block sums, in chunks of kScanBlock
__global__ void k_scan_blocks(uint32_t* blocksum, int64_t nb) {
    __shared__ uint32_t s[kScanBlock / kWave];
    __shared__ uint32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        const int64_t i = base + threadIdx.x;
        const uint32_t v = i < nb ? blocksum[i] : 0u;
        const uint32_t incl = (uint32_t)wave_incl_scan((int)v);
        const int w = threadIdx.x / kWave;
        if (lane_id() == kWave - 1) s[w] = incl;
        __syncthreads();
        uint32_t wofs = 0;
        for (int k = 0; k < w; ++k) wofs += s[k];
        const uint32_t excl = carry + wofs + incl - v;
        if (i < nb) blocksum[i] = excl;
        __syncthreads();
        if (threadIdx.x == kScanBlock - 1) carry = excl + v;
        __syncthreads();
    }
}

__global__ void k_scan_add(uint32_t* out, int64_t n, const uint32_t* blocksum, const uint32_t* in) {
    const int64_t i = blockIdx.x * (int64_t)kScanBlock + threadIdx.x;
    if (i < n) out[i] += blocksum[blockIdx.x];
    if (i == n - 1) out[n] = out[i] + in[i];
}

hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s) {
    int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    k_scan_local<<<(unsigned)nb, kScanBlock, 0, s>>>(in, out, n, tmp);
    k_scan_blocks<<<1, kScanBlock, 0, s>>>(tmp, nb);
    k_scan_add<<<(unsigned)nb, kScanBlock, 0, s>>>(out, n, tmp, in);
    return hipGetLastError();
}

// BOX predecessor windows: for every input u and axis a the range of
// (lo_a - x_a) and (hi_a - x_a) over all live pairs with input u.  Then
// pred(y,u) is contained in { x : y_a - hi_off <= x_a <= y_a - lo_off }, a
// superset of pred (Sect. V-B allows pred to be replaced by a superset);
// candidates are filtered exactly by decoding their box.
// The window table of up to kWinLds inputs is reduced in LDS first (one
// global atomic per entry and block instead of eight per pair).
constexpr int kWinLds = 512;
__global__ __launch_bounds__(256) void k_box_window(Inst I, int dtype, int32_t* win) {
    __shared__ int32_t s_win[kWinLds * 8];
    const int64_t npairs = I.n * I.K;
    const bool lds = I.K <= kWinLds;
    if (lds) {
        for (int i = threadIdx.x; i < I.K * 8; i += blockDim.x) s_win[i] = (i & 4) ? (int32_t)0x80000000 : 0x7fffffff;
        __syncthreads();
    }
    int32_t* w = lds ? s_win : win;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        if (!pair_live(I, p, dtype)) continue;
        const int u = (int)(p % I.K);
        int64_t x = p / I.K;
        BoxDec d = decode_box(I.box[p]);
        int64_t lo = d.lo;
        for (int a = 0; a < 4; ++a) {
            int xc = (int)(x % I.dims[a]);
            int lc = (int)(lo % I.dims[a]);
            x /= I.dims[a];
            lo /= I.dims[a];
            atomicMin(w + u * 8 + a, lc - xc);
            atomicMax(w + u * 8 + 4 + a, lc + d.e[a] - xc);
        }
    }
    if (lds) {
        __syncthreads();
        for (int i = threadIdx.x; i < I.K * 8; i += blockDim.x) {
            const int32_t v = s_win[i];
            if (i & 4) {
                if (v != (int32_t)0x80000000) atomicMax(win + i, v);
            } else if (v != 0x7fffffff) {
                atomicMin(win + i, v);
            }
        }
    }
}

hipError_t launch_box_window(const Inst& I, int32_t* win32, hipStream_t s) {
    k_box_window<<<grid_for(I.n * I.K, 256, 4096), 256, 0, s>>>(I, I.dtype, win32);
    return hipGetLastError();
}

// BOX -> CSR on the device: sizes, then (after a scan) each pair writes its
// box's cells in ascending linear order.
__global__ void k_box_sizes(Inst I, uint32_t* sizes, unsigned long long* total) {
    const int64_t npairs = I.n * I.K;
    unsigned long long acc = 0;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        const BoxDec d = decode_box(I.box[p]);
        const unsigned long long k = (unsigned long long)(d.e[0] + 1) * (d.e[1] + 1) * (d.e[2] + 1) * (d.e[3] + 1);
        sizes[p] = (uint32_t)(k > 0xffffffffull ? 0xffffffffull : k);
        acc += k;
    }
    acc = wave_sum64(acc);
    if (lane_id() == 0 && acc) atomicAdd(total, acc);
}

hipError_t launch_box_sizes(const Inst& I, uint32_t* sizes, unsigned long long* total, hipStream_t s) {
    k_box_sizes<<<grid_for(I.n * I.K, 256, 1024), 256, 0, s>>>(I, sizes, total);
    return hipGetLastError();
}

__global__ void k_box_fill(Inst I, const uint32_t* sptr, int32_t* sidx) {
    const int64_t npairs = I.n * I.K;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        const BoxDec d = decode_box(I.box[p]);
        uint32_t pos = sptr[p];
        for (int j3 = 0; j3 <= d.e[3]; ++j3)
            for (int j2 = 0; j2 <= d.e[2]; ++j2)
                for (int j1 = 0; j1 <= d.e[1]; ++j1) {
                    const int64_t r0 = d.lo + (int64_t)j1 * I.strides[1] + (int64_t)j2 * I.strides[2] +
                                       (int64_t)j3 * I.strides[3];
                    for (int j0 = 0; j0 <= d.e[0]; ++j0) sidx[pos++] = (int32_t)(r0 + j0);
                }
    }
}

hipError_t launch_box_fill(const Inst& I, const uint32_t* sptr, int32_t* sidx, hipStream_t s) {
    k_box_fill<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, sptr, sidx);
    return hipGetLastError();
}

// ------------------------------------------------------------------ loader, 64-bit pair ids
// HYB with 64-bit pair ids: the reverse CSR is built straight from the boxes
// (no temporary successor lists).  Each live pair visits the cells of its
// box; pass 1 counts the in-degree of every state, a 64-bit scan gives the
// row pointers, pass 2 writes each predecessor pair as its id minus y*K
// (a small signed offset: the loader checks that the predecessor windows
// keep it within int32), and the rows are sorted ascending.
template <class F>
__device__ __forceinline__ void for_box_cells(const Inst& I, uint64_t bx, F f) {
    const BoxDec d = decode_box(bx);
    for (int j3 = 0; j3 <= d.e[3]; ++j3)
        for (int j2 = 0; j2 <= d.e[2]; ++j2)
            for (int j1 = 0; j1 <= d.e[1]; ++j1) {
                const int64_t r0 =
                    d.lo + (int64_t)j1 * I.strides[1] + (int64_t)j2 * I.strides[2] + (int64_t)j3 * I.strides[3];
                for (int j0 = 0; j0 <= d.e[0]; ++j0) f(r0 + j0);
            }
}

__global__ void k_rev_count_box(Inst I, int dtype, uint32_t* cnt) {
    const int64_t npairs = I.n * I.K;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        if (!pair_live(I, p, dtype)) continue;
        for_box_cells(I, I.box[p], [&](int64_t y) { atomicAdd(cnt + y, 1u); });
    }
}

hipError_t launch_rev_count_box(const Inst& I, uint32_t* cnt, hipStream_t s) {
    k_rev_count_box<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, I.dtype, cnt);
    return hipGetLastError();
}

__global__ void k_rev_fill_box(Inst I, int dtype, unsigned long long* cursor, int32_t* rel) {
    const int64_t npairs = I.n * I.K;
    for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < npairs; p += (int64_t)gridDim.x * blockDim.x) {
        if (!pair_live(I, p, dtype)) continue;
        for_box_cells(I, I.box[p], [&](int64_t y) {
            const unsigned long long pos = atomicAdd(cursor + y, 1ull);
            rel[pos] = (int32_t)(p - y * I.K);
        });
    }
}

hipError_t launch_rev_fill_box(const Inst& I, unsigned long long* cursor, int32_t* rel, hipStream_t s) {
    k_rev_fill_box<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, I.dtype, cursor, rel);
    return hipGetLastError();
}

// Exclusive scan of n uint32 into uint64 out[0..n] (out[n] = total).
__global__ void k_scan64_local(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* blocksum) {
    __shared__ uint64_t s[1024 / kWave];
    const int64_t i = blockIdx.x * (int64_t)1024 + threadIdx.x;
    const uint64_t v = i < n ? in[i] : 0u;
    uint64_t incl = v;
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const uint64_t t = __shfl_up(incl, d, kWave);
        if (lane >= d) incl += t;
    }
    const int w = threadIdx.x / kWave;
    if (lane == kWave - 1) s[w] = incl;
    __syncthreads();
    uint64_t wofs = 0;
    for (int k = 0; k < w; ++k) wofs += s[k];
    const uint64_t excl = wofs + incl - v;
    if (i < n) out[i] = excl;
    if (threadIdx.x == 1023) blocksum[blockIdx.x] = excl + v;
}

__global__ void k_scan64_blocks(uint64_t* blocksum, int64_t nb) {
    __shared__ uint64_t s[1024 / kWave];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = lane_id();
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const uint64_t v = i < nb ? blocksum[i] : 0u;
        uint64_t incl = v;
#pragma unroll
        for (int d = 1; d < kWave; d <<= 1) {
            const uint64_t t = __shfl_up(incl, d, kWave);
            if (lane >= d) incl += t;
        }
        const int w = threadIdx.x / kWave;
        if (lane == kWave - 1) s[w] = incl;
        __syncthreads();
        uint64_t wofs = 0;
        for (int k = 0; k < w; ++k) wofs += s[k];
        const uint64_t excl = carry + wofs + incl - v;
        if (i < nb) blocksum[i] = excl;
        __syncthreads();
        if (threadIdx.x == 1023) carry = excl + v;
        __syncthreads();
    }
}

__global__ void k_scan64_add(uint64_t* out, int64_t n, const uint64_t* blocksum, const uint32_t* in) {
    const int64_t i = blockIdx.x * (int64_t)1024 + threadIdx.x;
    if (i < n) out[i] += blocksum[blockIdx.x];
    if (i == n - 1) out[n] = out[i] + in[i];
}

hipError_t launch_scan64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, hipStream_t s) {
    const int64_t nb = (n + 1023) / 1024;
    k_scan64_local<<<(unsigned)nb, 1024, 0, s>>>(in, out, n, tmp);
    k_scan64_blocks<<<1, 1024, 0, s>>>(tmp, nb);
    k_scan64_add<<<(unsigned)nb, 1024, 0, s>>>(out, n, tmp, in);
    return hipGetLastError();
}

// Sorts every 64-bit-indexed reverse row ascending (as k_sort_rows).
__global__ __launch_bounds__(kBlock) void k_sort_rows64(const uint64_t* __restrict__ rptr, int32_t* __restrict__ rel,
                                                       int64_t n) {
    __shared__ int32_t buf[kWavesPerBlock][kSortCap];
    int32_t* B = buf[threadIdx.x / kWave];
    const int lane = lane_id();
    for (int64_t row = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; row < n;
         row += (int64_t)gridDim.x * kWavesPerBlock) {
        const uint64_t s0 = rptr[row];
        const uint64_t len = rptr[row + 1] - s0;
        if (len <= 1 || len > (uint64_t)kSortCap) continue;
        uint32_t np2 = 2;
        while (np2 < len) np2 <<= 1;
        for (uint32_t i = lane; i < np2; i += kWave) B[i] = i < len ? rel[s0 + i] : 0x7fffffff;
        wave_sync();
        for (uint32_t k = 2; k <= np2; k <<= 1) {
            for (uint32_t j = k >> 1; j > 0; j >>= 1) {
                for (uint32_t i = lane; i < np2; i += kWave) {
                    const uint32_t ixj = i ^ j;
                    if (ixj > i) {
                        const int32_t a = B[i], b = B[ixj];
                        const bool asc = (i & k) == 0;
                        if ((a > b) == asc) {
                            B[i] = b;
                            B[ixj] = a;
                        }
                    }
                }
                wave_sync();
            }
        }
        for (uint32_t i = lane; i < len; i += kWave) rel[s0 + i] = B[i];
        wave_sync();
    }
}

hipError_t launch_sort_rows64(const uint64_t* rptr, int32_t* rel, int64_t n, hipStream_t s) {
    k_sort_rows64<<<grid_for((n + kWavesPerBlock - 1) / kWavesPerBlock, 1, 4096), kBlock, 0, s>>>(rptr, rel, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ init
// W <- G (Algorithm 1 initialisation), avoid cells pinned to INF.
template <class T>
__global__ void k_init(Inst I) {
    auto* V = static_cast<typename T::key_t*>(I.V);
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < I.n; x += (int64_t)gridDim.x * blockDim.x)
        V[x] = (I.avoid && I.avoid[x]) ? T::INF : T::from_raw(I.G[x]);
}

hipError_t launch_init(const Inst* dI, const Inst& I, int dtype, hipStream_t s) {
    (void)dI;
    if (dtype == 1) k_init<TF32><<<grid_for(I.n, 256), 256, 0, s>>>(I);
    else k_init<TI32><<<grid_for(I.n, 256), 256, 0, s>>>(I);
    return hipGetLastError();
}

// ------------------------------------------------------------------ expand
// Marks a pair dirty in the upcoming frontier: one byte per pair, set with a
// plain store.  Marking is idempotent, so no read-modify-write is needed; on
// this multi-XCD device every device-scope atomic executes at the memory
// side (it bypasses L2), while a byte store is write-combined in L2 and
// merged by byte mask on write-back.  A plain read skips pairs already
// marked (a stale read only misses marks, never invents them).
// Bucket order: the first mark of a pair also flags its state's bucket as
// occupied (another idempotent byte store).
template <class IdT>
__device__ __forceinline__ void mark_pair(const Inst& I, uint8_t* __restrict__ dirty, IdT base, IdT q, bool valid) {
    if (valid) {
        GBF_GLOBAL uint8_t* b = gp(dirty) + base + q;
        if (*b == 0) {
            *b = 1;
            if (I.key) gp(I.occ)[gp(I.key)[q / (IdT)I.K]] = 1;
        }
    }
}

// Encodings.  Template ENC: 1 = CSR, 2 = BOX, 4 = box successors with a
// reverse CSR for the predecessors (HYB), 5 = CSR with per-edge costs,
// 3 = decided per instance from Inst.enc (0 CSR, 1 BOX, 2 HYB) and Inst.ge.
template <int ENC>
__device__ __forceinline__ bool fwd_csr(const Inst& I) {
    return ENC == 1 || ENC == 5 || (ENC == 3 && I.enc == 0);
}
template <int ENC>
__device__ __forceinline__ bool rev_csr(const Inst& I) {
    return ENC == 1 || ENC == 4 || ENC == 5 || (ENC == 3 && I.enc != 1);
}
template <int ENC>
__device__ __forceinline__ bool has_edge(const Inst& I) {
    return ENC == 5 || (ENC == 3 && I.enc == 0 && I.ge != nullptr);
}
// Kernels that may meet per-edge costs.
template <int ENC>
constexpr bool kMayEdge = ENC == 5 || ENC == 3;

// NS slices of 64 reverse entries of one state, starting at entry t0.
// Every load is unconditional -- lanes past the row end read its last entry
// again -- so all NS entry loads, then all NS dirty-byte loads, issue back
// to back before one wait each (a load under a lane condition would be
// followed by its own wait); the marks stay guarded.  entry(t) gives the
// pair id of entry t.
template <int NS, class Id, class Entry>
__device__ __forceinline__ void mark_slices(const Inst& I, uint8_t* __restrict__ dirty, Id base, uint32_t t0,
                                            uint32_t len, Entry entry) {
    const int lane = lane_id();
    Id q[NS];
    bool v[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) {
        const uint32_t t = t0 + (uint32_t)(k * kWave + lane);
        v[k] = t < len;
        q[k] = entry(min(t, len - 1u));
    }
    uint8_t b[NS];
#pragma unroll
    for (int k = 0; k < NS; ++k) b[k] = gp(dirty)[base + q[k]];
#pragma unroll
    for (int k = 0; k < NS; ++k)
        if (v[k] && b[k] == 0) {
            gp(dirty)[base + q[k]] = 1;
            if (I.key) gp(I.occ)[gp(I.key)[q[k] / (Id)I.K]] = 1;
        }
}

// Streams a reverse row of `len` entries, kExpBatch slices per step.
template <class Id, class Entry>
__device__ __forceinline__ void mark_row(const Inst& I, uint8_t* __restrict__ dirty, Id base, uint32_t len,
                                         Entry entry) {
    for (uint32_t t0 = 0; t0 < len; t0 += kWave * kExpBatch) mark_slices<kExpBatch, Id>(I, dirty, base, t0, len, entry);
}

// Bounds of the reverse row of state y: 64-bit rows start at a 64-bit
// offset.
template <bool WIDE>
struct RevRow {
    typename std::conditional<WIDE, uint64_t, uint32_t>::type s0;
    uint32_t len;
};
template <bool WIDE>
__device__ __forceinline__ RevRow<WIDE> rev_bounds(const Inst& I, int64_t y) {
    RevRow<WIDE> r;
    if constexpr (WIDE) {
        const GBF_GLOBAL uint64_t* rptr = gp(I.rptr64);
        r.s0 = rptr[y];
        r.len = (uint32_t)(rptr[y + 1] - r.s0);
    } else {
        const GBF_GLOBAL uint32_t* rptr = gp(I.rptr);
        r.s0 = rptr[y];
        r.len = rptr[y + 1] - r.s0;
    }
    return r;
}

// Marks every pair of the reverse row of y (wave-uniform arguments).
// 64-bit reverse rows hold each predecessor pair as its id minus y*K.
template <bool WIDE>
__device__ __forceinline__ void expand_rev(const Inst& I, int64_t y, const RevRow<WIDE>& rr,
                                           uint8_t* __restrict__ dirty, Acc& acc) {
    using Id = typename Ids<WIDE>::id_t;
    const Id base = (Id)I.pair_base;
    const auto s0 = rr.s0;
    const uint32_t len = rr.len;
    if (lane_id() == 0) {
        acc.expanded += 1;
        acc.marks += len;
    }
    if constexpr (WIDE) {
        const GBF_GLOBAL int32_t* rel = gp(I.rrel);
        const int64_t yK = y * (int64_t)I.K;
        mark_row<Id>(I, dirty, base, len,
                     [&](uint32_t t) { return (Id)(yK + (int64_t)ldx<GBF_NT_MISC>(rel + s0 + t)); });
    } else {
        // kExpBatch slices of 64 entries per step: all their reverse
        // entries, then all their dirty bytes, are loaded before any store
        const GBF_GLOBAL uint32_t* rev = gp(I.rev);
        mark_row<uint32_t>(I, dirty, (uint32_t)base, len,
                           [&](uint32_t t) { return ldx<GBF_NT_MISC>(rev + s0 + t); });
    }
}

// Whole-wave expansion of one state y (wave-uniform arguments): every live
// pair (x',u') with y in F(x',u') is marked.  CSR: the (sorted) reverse row
// of y is streamed by the wave.  BOX: for every input the predecessor
// window is streamed and each candidate's box is decoded to filter it.
template <int ENC, bool WIDE = false>
__device__ __forceinline__ void expand_state(const Inst& I, int64_t y, uint8_t* __restrict__ dirty, Acc& acc) {
    using Id = typename Ids<WIDE>::id_t;
    const int lane = lane_id();
    const Id base = (Id)I.pair_base;
    if (rev_csr<ENC>(I)) {
        const RevRow<WIDE> rr = rev_bounds<WIDE>(I, y);
        expand_rev<WIDE>(I, y, rr, dirty, acc);
        return;
    }
    int yc[4];
    int64_t r = y;
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        yc[a] = (int)(r % I.dims[a]);
        r /= I.dims[a];
    }
    if (lane == 0) acc.expanded += 1;
    const int dt = I.dtype;
    for (int u = 0; u < I.K; ++u) {
        const int32_t* w = I.win + u * 8;
        int lo[4], sz[4];
        bool empty = false;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            lo[a] = max(0, yc[a] - w[4 + a]);
            const int hi = min(I.dims[a] - 1, yc[a] - w[a]);
            sz[a] = hi - lo[a] + 1;
            empty |= sz[a] <= 0;
        }
        if (empty) continue;
        const uint32_t total = (uint32_t)(sz[0] * sz[1] * sz[2] * sz[3]);
        if (lane == 0) acc.marks += total;
        for (uint32_t t0 = 0; t0 < total; t0 += kWave) {
            const uint32_t t = t0 + (uint32_t)lane;
            bool hit = false;
            Id q = 0;
            if (t < total) {
                uint32_t rr = t;
                const int c0 = (int)(rr % (uint32_t)sz[0]);
                rr /= (uint32_t)sz[0];
                const int c1 = (int)(rr % (uint32_t)sz[1]);
                rr /= (uint32_t)sz[1];
                const int c2 = (int)(rr % (uint32_t)sz[2]);
                const int c3 = (int)(rr / (uint32_t)sz[2]);
                const int64_t x = (lo[0] + c0) + (int64_t)(lo[1] + c1) * I.strides[1] +
                                  (int64_t)(lo[2] + c2) * I.strides[2] + (int64_t)(lo[3] + c3) * I.strides[3];
                const int64_t qq = x * I.K + u;
                if (pair_live(I, qq, dt)) {
                    const BoxDec d = decode_box(I.box[qq]);
                    int64_t lr = d.lo;
                    bool in = true;
#pragma unroll
                    for (int a = 0; a < 4; ++a) {
                        const int lc = (int)(lr % I.dims[a]);
                        lr /= I.dims[a];
                        in &= (yc[a] >= lc) && (yc[a] <= lc + d.e[a]);
                    }
                    hit = in;
                    q = (Id)qq;
                }
            }
            mark_pair<Id>(I, dirty, base, q, hit);
        }
    }
}

// Seed: F1 <- union of pred(y) over states with G(y) < INF (Algorithm 1
// initialisation), at pair level.  Each wave looks at 64 states and expands
// the targets among them one after the other.
template <class T, int ENC, bool WIDE = false>
__global__ __launch_bounds__(kBlock) void k_seed(const Inst* __restrict__ It, int ninst, Run R) {
    Acc acc;
    for (int ii = 0; ii < ninst; ++ii) {
        const Inst& I = It[ii];
        const int64_t nw = (I.n + kWave - 1) / kWave;
        for (int64_t w = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; w < nw;
             w += (int64_t)gridDim.x * kWavesPerBlock) {
            const int64_t y = w * kWave + lane_id();
            bool act = false;
            if (y < I.n) act = T::from_raw(I.G[y]) != T::INF && !I.avoid[y];
            unsigned long long bal = __ballot(act);
            while (bal) {
                const int l = __ffsll(bal) - 1;
                bal &= bal - 1;
                expand_state<ENC, WIDE>(I, w * kWave + l, R.dirty[0], acc);
            }
        }
    }
}

// ------------------------------------------------------------------ compact
// A tile = one 16-byte chunk of the dirty byte map per thread of a block.
// Each thread turns its chunk into a 16-bit mask of dirty pairs; a
// block-wide scan of the mask popcounts (wave prefix sums staged in LDS)
// places the pair ids, ascending, in the frontier list.  Listed bytes are
// cleared.

// Inverse of nonzero_bytes4 for 0/1 bytes: bit b of the low nibble -> byte b.
__device__ __forceinline__ uint32_t spread_bytes4(uint32_t m) {
    return (m & 1u) | ((m & 2u) << 7) | ((m & 4u) << 14) | ((m & 8u) << 21);
}

__device__ __forceinline__ uint32_t nonzero_bytes4(uint32_t w) {
    const uint32_t hb = (((w & 0x7f7f7f7fu) + 0x7f7f7f7fu) | w) & 0x80808080u;
    return ((hb >> 7) & 1u) | ((hb >> 14) & 2u) | ((hb >> 21) & 4u) | ((hb >> 28) & 8u);
}

// Bucket order: only dirty pairs whose state key lies in [lo, hi] are
// listed and cleared; the others stay in the map for a later round.
constexpr uint32_t kNoBucket = 0xFFFFFFFFu;
constexpr int kBuckets = 65536;

struct BucketSel {
    const uint16_t* key;
    uint32_t lo, hi;
    uint32_t K;
};

// Persistent-kernel compaction of one super-tile of C tiles of NB chunks:
// the counts of all C tiles are scanned first, then one global atomicAdd
// reserves the super-tile's slots, then the ids are written in ascending
// order and the chunks cleared.
// LOCAL: the whole map is compacted by this one block, tile after tile, so
// the slots are reserved from a running total in LDS (*s_base, which the
// caller zeroes) instead of a device-scope atomic on `cnt`.
template <int NB, int C, bool LOCAL = false>
__device__ __forceinline__ void compact_tile(uint8_t* __restrict__ dirty, int64_t nchunks, int64_t stile,
                                             uint32_t* __restrict__ list, uint32_t* cnt, int* s_w, uint32_t* s_base) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    constexpr int NW = NB / kWave;
    const int t = threadIdx.x;
    const int w = t / kWave;
    GBF_GLOBAL u32x4* chunks = reinterpret_cast<GBF_GLOBAL u32x4*>(gp(dirty));
    uint32_t mask[C];
    int loc[C];
#pragma unroll
    for (int i = 0; i < C; ++i) {
        const int64_t ci = (stile * C + i) * NB + t;
        u32x4 v = {0u, 0u, 0u, 0u};
        if (ci < nchunks) v = chunks[ci];
        mask[i] = nonzero_bytes4(v.x) | (nonzero_bytes4(v.y) << 4) | (nonzero_bytes4(v.z) << 8) |
                  (nonzero_bytes4(v.w) << 12);
        const int c = __popc(mask[i]);
        const int incl = wave_incl_scan(c);
        loc[i] = incl - c;
        if (lane_id() == kWave - 1) s_w[i * NW + w] = incl;
    }
    __syncthreads();
    int run = 0;
#pragma unroll
    for (int i = 0; i < C; ++i) {
        int wofs = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int vv = s_w[i * NW + k];
            wofs += k < w ? vv : 0;
            tot += vv;
        }
        loc[i] += run + wofs;
        run += tot;
    }
    if (run != 0) {
        if (!LOCAL && t == 0) *s_base = atomicAdd(cnt, (uint32_t)run);
        __syncthreads();
        const uint32_t base = *s_base;
        GBF_GLOBAL uint32_t* out = gp(list);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            uint32_t m = mask[i];
            if (m) {
                const int64_t ci = (stile * C + i) * NB + t;
                const u32x4 zero = {0u, 0u, 0u, 0u};
                chunks[ci] = zero;
                uint32_t pos = base + (uint32_t)loc[i];
                const uint32_t pbase = (uint32_t)(ci * 16);
                while (m) {
                    const int b = __ffs(m) - 1;
                    out[pos++] = pbase + (uint32_t)b;
                    m &= m - 1u;
                }
            }
        }
        if (LOCAL) {
            __syncthreads();  // every thread has read the base
            if (t == 0) *s_base = base + (uint32_t)run;
        }
    }
    __syncthreads();
}

constexpr int kPCompactC = 1;  // tiles per super-tile, 1024-thread blocks

// Selected pairs of one 16-byte chunk (bit b = pair 16*ci + b); BK: `keep`
// receives the dirty pairs that stay in the map.
template <bool BK>
__device__ __forceinline__ uint32_t chunk_select(const uint32_t v4[4], int64_t ci, const BucketSel& bs,
                                                 uint32_t* keep) {
    uint32_t m = nonzero_bytes4(v4[0]) | (nonzero_bytes4(v4[1]) << 4) | (nonzero_bytes4(v4[2]) << 8) |
                 (nonzero_bytes4(v4[3]) << 12);
    *keep = 0;
    if (BK && m) {
        // the 16 pairs belong to consecutive states: one key load per state
        const uint32_t p0 = (uint32_t)(ci * 16);
        uint32_t x = p0 / bs.K, r = p0 - x * bs.K;
        const GBF_GLOBAL uint16_t* key = gp(bs.key);
        uint32_t sel = 0;
        int b = 0;
        while (b < 16) {
            const uint32_t run = min(16u - (uint32_t)b, bs.K - r);  // pairs of state x in this chunk
            const uint32_t bits = ((1u << run) - 1u) << b;
            if (m & bits) {
                const uint32_t k = key[x];
                if (k >= bs.lo && k <= bs.hi) sel |= m & bits;
            }
            b += (int)run;
            r = 0;
            ++x;
        }
        *keep = m & ~sel;
        m = sel;
    }
    return m;
}

// Host-loop compaction.  Block b owns the contiguous tiles [t0, t1) of
// kBlock chunks.  Pass 1 counts the pairs it will list; one atomicAdd per
// block reserves their slots (device-scope atomics serialise at the memory
// side, so the grid is kept small); pass 2 re-reads the chunks, now in L2,
// and writes the ids in ascending order, clearing the listed bytes.
template <bool BK, bool WIDE = false>
__device__ __forceinline__ void compact_range(uint8_t* __restrict__ dirty, int64_t nchunks, int64_t t0, int64_t t1,
                                              typename Ids<WIDE>::id_t* __restrict__ list,
                                              typename Ids<WIDE>::cnt_t* cnt, const BucketSel& bs) {
    using Id = typename Ids<WIDE>::id_t;
    using Cnt = typename Ids<WIDE>::cnt_t;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    __shared__ int s_w[kWavesPerBlock];
    __shared__ Cnt s_base;
    const int t = threadIdx.x;
    const int w = t / kWave;
    GBF_GLOBAL u32x4* chunks = reinterpret_cast<GBF_GLOBAL u32x4*>(gp(dirty));
    int c = 0;
#pragma unroll 4
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t ci = tile * kBlock + t;
        if (ci < nchunks) {
            const u32x4 v = chunks[ci];
            const uint32_t v4[4] = {v.x, v.y, v.z, v.w};
            uint32_t keep;
            c += __popc(chunk_select<BK>(v4, ci, bs, &keep));
        }
    }
    c = wave_sum(c);
    if (lane_id() == 0) s_w[w] = c;
    __syncthreads();
    int total = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) total += s_w[k];
    if (total == 0) return;  // block-uniform
    if (t == 0) s_base = atomicAdd(cnt, (Cnt)total);
    __syncthreads();
    Id off = (Id)s_base;
    GBF_GLOBAL Id* out = gp(list);
    for (int64_t tile = t0; tile < t1; ++tile) {
        const int64_t ci = tile * kBlock + t;
        uint32_t m = 0, keep = 0;
        if (ci < nchunks) {
            const u32x4 v = chunks[ci];
            const uint32_t v4[4] = {v.x, v.y, v.z, v.w};
            m = chunk_select<BK>(v4, ci, bs, &keep);
        }
        const int cc = __popc(m);
        const int incl = wave_incl_scan(cc);
        __syncthreads();  // s_w of the previous tile has been read
        if (lane_id() == kWave - 1) s_w[w] = incl;
        __syncthreads();
        int wofs = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < kWavesPerBlock; ++k) {
            const int vv = s_w[k];
            wofs += k < w ? vv : 0;
            tot += vv;
        }
        if (m) {
            u32x4 rest = {0u, 0u, 0u, 0u};
            if (BK) {
                rest.x = spread_bytes4(keep);
                rest.y = spread_bytes4(keep >> 4);
                rest.z = spread_bytes4(keep >> 8);
                rest.w = spread_bytes4(keep >> 12);
            }
            chunks[ci] = rest;
            Id pos = off + (Id)(wofs + incl - cc);
            const Id pbase = (Id)(ci * 16);
            while (m) {
                const int b = __ffs(m) - 1;
                out[pos++] = pbase + (Id)b;
                m &= m - 1u;
            }
        }
        off += (Id)tot;
    }
}

constexpr int kCompactGrid = GBF_COMPACT_GRID;

template <bool WIDE>
__global__ __launch_bounds__(kBlock) void k_compact(Run R, int round) {
    auto* counts = Ids<WIDE>::counts(R);
    if (round > 0 && counts[round - 1] == 0) return;  // frontier already empty
    const int64_t ntiles = (R.nchunks + kBlock - 1) / kBlock;
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = blockIdx.x * per, t1 = min(ntiles, t0 + per);
    compact_range<false, WIDE>(R.dirty[round & 1], R.nchunks, t0, t1, Ids<WIDE>::list(R), counts + round,
                               BucketSel{nullptr, 0u, 0u, 1u});
}

// Bucket order, one round: picks the range of buckets [lo, hi] whose dirty
// pairs the compaction lists (all of them, so those buckets are empty
// afterwards: their occupancy flags are cleared here, and a later mark sets
// a flag again).  Two schedules (R.bspan):
//   bspan >= 1: window.  lo = the lowest occupied bucket, hi = lo + bspan - 1.
//     Pairs marked below the window are taken in the next round.
//   bspan == -1: sweeps.  One bucket per round, the lowest occupied one at or
//     above the previous round's; pairs marked in lower buckets wait for
//     the next sweep, which starts again at the lowest occupied bucket.
// Past the round cap every pair is listed, so the remaining pairs are
// dropped and flagged in one round.  No bucket occupied: lo = kNoBucket and
// nothing is listed.  Words: thr[0] lo, thr[1] sweep position, thr[2]
// number of sweeps (window: rounds that found the range empty below the
// previous one), thr[3] hi.
__global__ __launch_bounds__(1024) void k_bucket_select(Run R, int round) {
    __shared__ uint32_t s_up, s_all;
    if (round > 0 && R.counts[round - 1] == 0) return;  // frontier already empty
    if (threadIdx.x == 0) {
        s_up = kNoBucket;
        s_all = kNoBucket;
    }
    __syncthreads();
    GBF_GLOBAL uint32_t* thr = gp(R.thr);
    const uint32_t pos = round == 0 ? 0u : thr[1];
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    const GBF_GLOBAL u32x4* occ = reinterpret_cast<const GBF_GLOBAL u32x4*>(gp(R.occ));
    uint32_t up = kNoBucket, all = kNoBucket;
    for (int i = threadIdx.x; i < kBuckets / 16; i += blockDim.x) {
        const u32x4 v = occ[i];
        uint32_t m = nonzero_bytes4(v.x) | (nonzero_bytes4(v.y) << 4) | (nonzero_bytes4(v.z) << 8) |
                     (nonzero_bytes4(v.w) << 12);
        if (!m) continue;
        const uint32_t b = (uint32_t)i * 16u;
        if (all == kNoBucket) all = b + (uint32_t)(__ffs(m) - 1);
        if (b + 15u < pos) continue;
        if (b < pos) m &= ~((1u << (pos - b)) - 1u);
        if (m) {
            up = b + (uint32_t)(__ffs(m) - 1);
            break;  // i only grows: the thread's smallest at or above pos
        }
    }
    if (up != kNoBucket) atomicMin(&s_up, up);
    if (all != kNoBucket) atomicMin(&s_all, all);
    __syncthreads();
    uint32_t lo, hi;
    if (R.bspan < 0) {
        lo = s_up != kNoBucket ? s_up : s_all;
        hi = lo;
    } else {
        lo = s_all;
        hi = lo == kNoBucket ? lo : min(lo + (uint32_t)R.bspan - 1u, (uint32_t)kBuckets - 1u);
    }
    const bool cap = round >= R.max_rounds;
    if (lo != kNoBucket && !cap)
        for (uint32_t b = lo + threadIdx.x; b <= hi; b += blockDim.x) gp(R.occ)[b] = 0;
    if (threadIdx.x == 0) {
        const bool wrap = R.bspan < 0 ? (s_up == kNoBucket && s_all != kNoBucket) : (round > 0 && lo < pos);
        thr[2] = (round == 0 ? 1u : thr[2]) + (wrap ? 1u : 0u);
        if (cap) {
            lo = 0;
            hi = kBuckets - 1;  // list everything
        } else if (lo != kNoBucket) {
            thr[1] = lo;
        }
        thr[0] = lo;
        thr[3] = hi;
    }
}

__global__ __launch_bounds__(kBlock) void k_compact_bucket(Run R, int round) {
    if (round > 0 && R.counts[round - 1] == 0) return;
    const uint32_t lo = gp(R.thr)[0], hi = gp(R.thr)[3];
    if (lo == kNoBucket) return;
    const BucketSel bs{R.key, lo, hi, (uint32_t)R.keyK};
    const int64_t ntiles = (R.nchunks + kBlock - 1) / kBlock;
    const int64_t per = (ntiles + gridDim.x - 1) / gridDim.x;
    const int64_t t0 = blockIdx.x * per, t1 = min(ntiles, t0 + per);
    compact_range<true>(R.dirty[0], R.nchunks, t0, t1, R.list, R.counts + round, bs);
}

hipError_t launch_bucket_compact(const Run& R, int round, int grid, hipStream_t s) {
    k_bucket_select<<<1, 1024, 0, s>>>(R, round);
    const int64_t ntiles = (R.nchunks + kBlock - 1) / kBlock;
    int g = (int)std::min<int64_t>(ntiles, grid > 0 ? std::min(grid, kMaxGrid) : kCompactGrid);
    if (g < 1) g = 1;
    k_compact_bucket<<<g, kBlock, 0, s>>>(R, round);
    return hipGetLastError();
}

hipError_t launch_compact(const Run& R, int round, int grid, hipStream_t s, bool wide) {
    const int64_t ntiles = (R.nchunks + kBlock - 1) / kBlock;
    int g = (int)std::min<int64_t>(ntiles, grid > 0 ? std::min(grid, kMaxGrid) : kCompactGrid);
    if (g < 1) g = 1;
    if (wide) k_compact<true><<<g, kBlock, 0, s>>>(R, round);
    else k_compact<false><<<g, kBlock, 0, s>>>(R, round);
    return hipGetLastError();
}

// ------------------------------------------------------------------ relax
// G lanes per listed pair: the group streams the pair's successor row (CSR,
// coalesced) or walks its box (BOX), folds V[y] into a running max and
// reduces it across the group with lane shuffles.  The group leader forms
// d = g(x,u) + max and applies the strict improvement with atomicMin.  Each
// improved state of a wave step is then expanded by the whole wave.
template <class T, int G>
__device__ __forceinline__ typename T::key_t group_max(typename T::key_t v) {
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) v = T::max2(v, __shfl_xor(v, d, kWave));
    return v;
}

template <class T, int G>
__device__ __forceinline__ typename T::wide_t group_wmax(typename T::wide_t v) {
#pragma unroll
    for (int d = G / 2; d > 0; d >>= 1) v = T::wmax2(v, __shfl_xor(v, d, kWave));
    return v;
}

// Per-lane view of the listed pair that a lane group works on.
template <class IdT>
struct PairCtxT {
    uint32_t s0, len;  // CSR row of the pair (BOX: unused)
    IdT p;             // instance-local pair id
    int ii;            // instance
    bool valid;
};
template <bool WIDE>
using PairCtx = PairCtxT<typename Ids<WIDE>::id_t>;

template <bool MULTI, int ENC, int G, bool WIDE = false>
__device__ __forceinline__ PairCtx<WIDE> load_pair(const Inst* __restrict__ It, const int64_t* bases, const Run& R,
                                                   typename Ids<WIDE>::id_t count, typename Ids<WIDE>::id_t first,
                                                   int round) {
    using Id = typename Ids<WIDE>::id_t;
    PairCtx<WIDE> c;
    const int sub = lane_id() & (G - 1);
    const Id i = first + (Id)(lane_id() / G);
    c.valid = i < count;
    const Id q = c.valid ? ldx<GBF_NT_MISC>(gp(Ids<WIDE>::list(R)) + i) : (Id)0;
    c.ii = find_inst<MULTI>(bases, R.ninst, (int64_t)q);
    const Inst& I = It[c.ii];
    c.p = q - (MULTI ? (Id)I.pair_base : (Id)0);
    if (c.valid && round >= I.max_rounds) {
        // the instance's round cap (second condition of Algorithm 1's while
        // loop) is reached with work left: drop the pair, flag the instance
        if (sub == 0) R.inst_status[c.ii] = 1;
        c.valid = false;
    }
    c.s0 = 0;
    c.len = 0;
    if (c.valid && fwd_csr<ENC>(I)) {
        const GBF_GLOBAL uint32_t* sptr = gp(I.sptr);
        c.s0 = ldx<GBF_NT_MISC>(sptr + c.p);
        c.len = ldx<GBF_NT_MISC>(sptr + c.p + 1) - c.s0;
    }
    return c;
}

// What a lane group gathered for its pair: the running max over the
// successors (this lane's share), W(x), the raw cost and |F(x,u)|.
template <class T>
struct PairVal {
    typename T::key_t mx, cur;
    typename T::wide_t mw;  // per-edge costs: this lane's max of h + W(y)
    int32_t graw;
    uint32_t len;
};

// NK loads per lane of a successor row segment starting at entry t (lane
// stride G), then the NK values: all unconditional -- lanes past the row
// end take its last entry again, a real successor, so the max does not
// change -- so the loads of a batch issue back to back before one wait.
// EDGE: per-edge costs h stream beside the indices.
template <class T, int NK, int G, bool EDGE>
__device__ __forceinline__ void row_batch(const GBF_GLOBAL int32_t* row, const GBF_GLOBAL int32_t* hrow,
                                          const GBF_GLOBAL typename T::key_t* V, uint32_t t, uint32_t len,
                                          typename T::key_t& mx, typename T::wide_t& mw) {
    using K = typename T::key_t;
    int32_t y[NK], hv[NK];
    K w[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        const uint32_t tk = min(t + (uint32_t)(k * G), len - 1u);
        y[k] = ldx<GBF_NT_ROWS>(row + tk);
        if constexpr (EDGE) hv[k] = ldx<GBF_NT_ROWS>(hrow + tk);
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) w[k] = V[y[k]];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
        if constexpr (EDGE) mw = T::wmax2(mw, T::edge(hv[k], w[k]));
        else mx = T::max2(mx, w[k]);
    }
}

// The batch size is the largest number of entries any lane of the wave has
// left in this step (wave-uniform), so that no load instruction is issued
// for lanes that all ran past their rows.
template <class T, int NK, int G, bool EDGE>
__device__ __forceinline__ void row_step(const GBF_GLOBAL int32_t* row, const GBF_GLOBAL int32_t* hrow,
                                         const GBF_GLOBAL typename T::key_t* V, uint32_t t, uint32_t len,
                                         typename T::key_t& mx, typename T::wide_t& mw) {
    if constexpr (NK > 1) {
        if (!__ballot(t + (uint32_t)((NK - 1) * G) < len)) {
            row_step<T, NK - 1, G, EDGE>(row, hrow, V, t, len, mx, mw);
            return;
        }
    }
    row_batch<T, NK, G, EDGE>(row, hrow, V, t, len, mx, mw);
}

// Gather phase of one wave step (64/G pairs, G lanes each): loads only, so
// the gathers of several wave steps can be in flight together.
template <class T, bool MULTI, int ENC, int G, bool WIDE = false>
__device__ __forceinline__ PairVal<T> pair_gather(const Inst* __restrict__ It, const PairCtx<WIDE>& c) {
    using K = typename T::key_t;
    using Id = typename Ids<WIDE>::id_t;
    const int sub = lane_id() & (G - 1);
    const Inst& I = It[c.ii];
    const GBF_GLOBAL K* V = gp(static_cast<const K*>(I.V));
    const uint32_t x = (uint32_t)(c.p / (Id)I.K);
    K cur = (K)T::INF;
    int32_t graw = 0;
    if (c.valid) {
        cur = V[x];
        graw = ldx<GBF_NT_MISC>(gp(I.g) + c.p);
    }
    K mx = (K)T::LOWEST;
    typename T::wide_t mw = T::WLOWEST;
    uint32_t len = c.len;
    if (c.valid) {
        if (has_edge<ENC>(I)) {
            // per-edge costs: the row's h values stream beside its indices
            const GBF_GLOBAL int32_t* row = gp(I.sidx) + c.s0;
            const GBF_GLOBAL int32_t* hrow = gp(I.ge) + c.s0;
            for (uint32_t t = (uint32_t)sub; t < len; t += kEdgeBatch * G)
                row_batch<T, kEdgeBatch, G, true>(row, hrow, V, t, len, mx, mw);
        } else if (fwd_csr<ENC>(I)) {
            // kRowBatch successor indices per lane in flight, then their values
            const GBF_GLOBAL int32_t* row = gp(I.sidx) + c.s0;
            for (uint32_t t = (uint32_t)sub; t < len; t += kRowBatch * G)
                row_step<T, kRowBatch, G, false>(row, nullptr, V, t, len, mx, mw);
        } else {
            // the box is w1*w2*w3 rows of w0 consecutive cells along axis 0;
            // the G lanes of the group take the rows in turn
            const BoxDec d = decode_box(ldx<GBF_NT_MISC>(gp(I.box) + c.p));
            const uint32_t w0 = d.e[0] + 1, w1 = d.e[1] + 1, w2 = d.e[2] + 1;
            const uint32_t lo = (uint32_t)d.lo, st1 = (uint32_t)I.strides[1], st2 = (uint32_t)I.strides[2],
                           st3 = (uint32_t)I.strides[3];
            const uint32_t nrows = w1 * w2 * (uint32_t)(d.e[3] + 1);
            len = w0 * nrows;
            // the first three cells of a row are read with clamped offsets (a
            // repeated cell leaves the max unchanged), so that the three loads
            // carry no branch and issue together
            const uint32_t c1 = min(1u, w0 - 1u), c2 = min(2u, w0 - 1u);
            for (uint32_t r = (uint32_t)sub; r < nrows; r += G) {
                const uint32_t r2 = r / w1;
                const uint32_t j1 = r - r2 * w1;
                const uint32_t j3 = r2 / w2;
                const uint32_t j2 = r2 - j3 * w2;
                const GBF_GLOBAL K* row = V + (lo + j1 * st1 + j2 * st2 + j3 * st3);
                const K a0 = row[0], a1 = row[c1], a2 = row[c2];
                K m0 = T::max2(a0, T::max2(a1, a2));
                for (uint32_t j0 = 3; j0 < w0; ++j0) m0 = T::max2(m0, row[j0]);
                mx = T::max2(mx, m0);
            }
        }
    }
    return PairVal<T>{mx, cur, mw, graw, len};
}

// Commit phase: max over the group, backup, one candidate per state, strict
// improvement, expansion.
template <class T, bool MULTI, int ENC, int G, int SCOPE = __HIP_MEMORY_SCOPE_AGENT, bool WIDE = false>
__device__ __forceinline__ void pair_commit(const Inst* __restrict__ It, const PairCtx<WIDE>& c,
                                            const PairVal<T>& pv, uint8_t* __restrict__ next, Acc& acc) {
    using K = typename T::key_t;
    using Id = typename Ids<WIDE>::id_t;
    constexpr int W = kWave / G;
    const int lane = lane_id();
    const int sub = lane & (G - 1);
    const int grp = lane / G;
    const Inst& I = It[c.ii];
    GBF_GLOBAL K* V = gp(static_cast<K*>(I.V));
    const uint32_t x = (uint32_t)(c.p / (Id)I.K);
    const K cur = pv.cur;
    const int32_t graw = pv.graw;
    const uint32_t len = pv.len;
    const K mx = group_max<T, G>(pv.mx);
    typename T::wide_t mw = T::WLOWEST;
    if constexpr (kMayEdge<ENC>) mw = group_wmax<T, G>(pv.mw);
    // candidate value of this pair (INF if it cannot improve V(x))
    K d = (K)T::INF;
    if (c.valid) {
        int sat = 0;
        K dd;
        const bool ok = has_edge<ENC>(I) ? T::backupw(graw, mw, dd, sat) : T::backup(graw, mx, dd, sat);
        if (ok && T::less(dd, cur)) d = dd;
        if (sub == 0) {
            acc.pairs += 1;
            acc.edges += len;
            acc.sat += (unsigned)sat;
        }
    }
    // The pairs of one state are adjacent in the (ascending) list: take the
    // min over the run of groups with the same state so that one atomic and
    // one expansion per state and wave step suffice.
    const uint32_t key = c.valid ? x : 0xffffffffu;
    const int ikey = c.valid ? c.ii : -1;
#pragma unroll
    for (int st = 1; st < W; st <<= 1) {
        const K od = __shfl_down(d, st * G, kWave);
        const uint32_t ok = __shfl_down(key, st * G, kWave);
        const int oi = MULTI ? __shfl_down(ikey, st * G, kWave) : ikey;
        if (grp + st < W && ok == key && oi == ikey) d = T::less(od, d) ? od : d;
    }
    const uint32_t pkey = __shfl_up(key, G, kWave);
    const int pi = MULTI ? __shfl_up(ikey, G, kWave) : ikey;
    const bool head = c.valid && sub == 0 && (grp == 0 || pkey != key || pi != ikey);
    // strict improvement (Algorithm 1: d < W(x)): a non-returning atomicMin;
    // the plain read above decided that it lowers V(x) (if a concurrent
    // update lowered it further, the expansion below is redundant, never
    // wrong: marks are idempotent)
    bool expand = false;
    if (head && T::less(d, cur)) {
        __hip_atomic_fetch_min(V + x, d, __ATOMIC_RELAXED, SCOPE);
        acc.impr += 1;
        expand = true;
    }
    unsigned long long bal = __ballot(expand);
    if (!bal) return;
    while (bal) {
        const int l = __ffsll(bal) - 1;
        bal &= bal - 1;
        const uint32_t xl = __shfl(x, l, kWave);
        if (MULTI) {
            const int il = __shfl(c.ii, l, kWave);
            expand_state<ENC, WIDE>(It[il], xl, next, acc);
        } else {
            expand_state<ENC, WIDE>(It[0], xl, next, acc);
        }
    }
}

// One round over the listed pairs.  Each wave takes ILP consecutive wave
// steps at a time: their loads are issued before any commit, so ILP times
// as many gathers are in flight per wave.
template <class T, bool MULTI, int ENC, int G, int ILP, int SCOPE = __HIP_MEMORY_SCOPE_AGENT, bool WIDE = false,
          bool XMAP = false>
__device__ __forceinline__ void relax_round(const Inst* __restrict__ It, const int64_t* bases, const Run& R,
                                            typename Ids<WIDE>::id_t count, int round, Acc& acc) {
    using Id = typename Ids<WIDE>::id_t;
    constexpr Id W = kWave / G;  // pairs per wave and step
    uint8_t* next = R.dirty[(round + 1) & 1];
    const Id wpb = blockDim.x / kWave;
    if constexpr (XMAP) {
        // Blocks b with b % kXcdParts == k take the k-th contiguous part of
        // the (ascending) list.  The hardware deals consecutive blocks to the
        // XCDs in turn (block b runs on XCD b % 8, read back from the XCC id
        // register on MI355X), so each XCD's L2 sees about one part of V and
        // of the maps.  Every pair is taken by exactly one wave whatever the
        // placement of the blocks.
        const Id part = (Id)(blockIdx.x % kXcdParts);
        const Id plo = (Id)((uint64_t)count * (uint64_t)part / kXcdParts);
        const Id phi = (Id)((uint64_t)count * (uint64_t)(part + 1) / kXcdParts);
        const Id nbp = (Id)(gridDim.x / kXcdParts);
        const Id lb = (Id)(blockIdx.x / kXcdParts);
        const Id w = threadIdx.x / kWave;
        Id c0, c1, step;
        if constexpr (!MULTI) {
            // One instance: each block takes one contiguous chunk of whole
            // wave steps, its waves the steps in turn, so that the block moves
            // through neighbouring states whose boxes and predecessor pairs
            // share lines of V and of the maps, which stay in the CU's L1
            // (measured 7-9% faster than dealing single steps; splitting the
            // chunk further gives it back).
            const uint64_t nst = ((uint64_t)(phi - plo) + W - 1) / W;
            c0 = plo + W * (Id)(nst * (uint64_t)lb / (uint64_t)nbp);
            const Id e1 = plo + W * (Id)(nst * (uint64_t)(lb + 1) / (uint64_t)nbp);
            c1 = e1 < phi ? e1 : phi;
            c0 += w * W;
            step = wpb * W;
        } else {
            // a batch: instances differ widely in cost per pair, so the
            // part's waves take its steps in turn, which balances them
            c0 = plo + (lb * wpb + w) * W;
            c1 = phi;
            step = nbp * wpb * W;
        }
        for (Id first = c0; first < c1; first += step) {
            const PairCtx<WIDE> c = load_pair<MULTI, ENC, G, WIDE>(It, bases, R, c1, first, round);
            const PairVal<T> v = pair_gather<T, MULTI, ENC, G, WIDE>(It, c);
            pair_commit<T, MULTI, ENC, G, SCOPE, WIDE>(It, c, v, next, acc);
        }
        return;
    }
    const Id wave = (Id)blockIdx.x * wpb + threadIdx.x / kWave;
    const Id stride = (Id)gridDim.x * wpb * W * ILP;
    for (Id first = wave * W * ILP; first < count; first += stride) {
        PairCtx<WIDE> c[ILP];
        PairVal<T> v[ILP];
#pragma unroll
        for (int i = 0; i < ILP; ++i)
            c[i] = load_pair<MULTI, ENC, G, WIDE>(It, bases, R, count, first + (Id)(i * W), round);
#pragma unroll
        for (int i = 0; i < ILP; ++i) v[i] = pair_gather<T, MULTI, ENC, G, WIDE>(It, c[i]);
#pragma unroll
        for (int i = 0; i < ILP; ++i) pair_commit<T, MULTI, ENC, G, SCOPE, WIDE>(It, c[i], v[i], next, acc);
    }
}

// The CSR, HYB and per-edge variants are built for 64 VGPRs: 8 waves per
// SIMD, so that the default grid (8 x 256 threads per CU) is resident in
// one pass.  The variants that decode forward boxes need about twice that
// and run at 4.  Blocks of any multiple of 64 threads up to 1024 (the
// waves of a block are read from blockDim).
template <class T, bool MULTI, int ENC, int G, bool WIDE = false>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(ENC == 2 || ENC == 3 ? 4 : 8)))
void k_relax(const Inst* __restrict__ It, Run R, int round) {
    __shared__ int64_t s_bases[MULTI ? kMaxBatch : 1];
    const typename Ids<WIDE>::id_t count = Ids<WIDE>::counts(R)[round];
    if (count == 0) return;
    if (MULTI) {
        for (int k = threadIdx.x; k < R.ninst; k += blockDim.x) s_bases[k] = It[k].pair_base;
        __syncthreads();
    }
    __shared__ AccLds s_acc;
    acc_init(s_acc);
    Acc acc;
    if (GBF_XCD_MAP && gridDim.x % kXcdParts == 0)
        relax_round<T, MULTI, ENC, G, kILP, __HIP_MEMORY_SCOPE_AGENT, WIDE, true>(It, s_bases, R, count, round, acc);
    else
        relax_round<T, MULTI, ENC, G, kILP, __HIP_MEMORY_SCOPE_AGENT, WIDE>(It, s_bases, R, count, round, acc);
    flush_acc(acc, s_acc, R.slots);
}

// ------------------------------------------------------------------ persistent
// All rounds in one launch.  Every wait is bounded in wall-clock time: a
// barrier that does not complete within R.timeout_ticks of the constant-rate
// device clock sets R.error, and every block leaves the loop (blocks that
// start after an error leave at once).
// Barrier words, each counter on its own 128-byte line (uint32 index * 32):
//   line 0: top-level arrival counter, line 1: generation,
//   line 2 + g: arrival counter of group g (blocks b with b % kBarGroups == g),
//   line 18: blocks per XCD (word k for XCD k) and, word 16, the number of
//            XCDs with blocks,
//   line 19: arrival counter of the XCD leaders,
//   lines 20..27: arrival counter of XCD k at word 20*32 + 16*k.
// Arrivals are device-scope atomics, which execute at the memory side and
// serialise per address; spreading them over groups keeps each chain short.
constexpr int kBarGroups = 16;
constexpr int kBarLine = 32;
constexpr int kMaxXcd = 16;
constexpr int kBarXcdInfo = 18 * kBarLine;
constexpr int kBarXcdTop = 19 * kBarLine;
constexpr int kBarXcdCtr = 20 * kBarLine;
static_assert(kBarXcdCtr + kMaxXcd * 16 <= 1024, "barrier words exceed their 4 KiB allocation");

// The accelerator complex (XCD) this wave runs on.  Each XCD has its own L2.
__device__ __forceinline__ uint32_t xcd_id() {
    return (uint32_t)__builtin_amdgcn_s_getreg((20) | (0 << 6) | ((4 - 1) << 11)) & (kMaxXcd - 1);
}

// Waits (thread 0 of the block) until the generation word moves past
// `gen`, with relaxed loads: an acquire load would invalidate the XCD's L2
// on every poll and evict the data the blocks still working there use.
__device__ __forceinline__ int wait_generation(uint32_t* gen_w, uint32_t gen, int32_t* err, uint64_t timeout_ticks) {
    const uint64_t t0 = wall_clock64();
    while (__hip_atomic_load(gen_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(4);
        if (wall_clock64() - t0 > timeout_ticks ||
            __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
            atomicOr(err, 1);
            return 0;
        }
    }
    return 1;
}

// Grid barrier over all blocks, arrivals combined in groups of blocks.
__device__ __forceinline__ bool grid_barrier(uint32_t* bar, int32_t* err, uint32_t nblocks, uint64_t timeout_ticks) {
    __shared__ int s_ok;
    // the block barrier orders every wave's stores before thread 0's
    // agent-scope release fence, which publishes them device-wide; one
    // acquire fence after the wait makes the other blocks' stores visible
    __syncthreads();
    if (threadIdx.x == 0) {
        // release: this block's stores are written back to memory before
        // the arrival is seen
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        int ok = 1;
        uint32_t* top = bar;
        uint32_t* gen_w = bar + kBarLine;
        const uint32_t ng = nblocks < (uint32_t)kBarGroups ? nblocks : (uint32_t)kBarGroups;
        const uint32_t grp = blockIdx.x % ng;
        uint32_t* gctr = bar + (2 + grp) * kBarLine;
        const uint32_t gsize = nblocks / ng + (grp < nblocks % ng ? 1u : 0u);
        const uint32_t gen = __hip_atomic_load(gen_w, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t a = __hip_atomic_fetch_add(gctr, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        bool released = false;
        if (a == gsize - 1) {
            __hip_atomic_store(gctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t t = __hip_atomic_fetch_add(top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            if (t == ng - 1) {
                __hip_atomic_store(top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(gen_w, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) ok = wait_generation(gen_w, gen, err, timeout_ticks);
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        s_ok = ok;
        // acquire: stale lines of other blocks' data are dropped before the
        // block reads again
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_ok != 0;
}

// Registers the block with the XCD it runs on (once, before the first
// grid barrier; after that barrier the counts are final).
__device__ __forceinline__ void xcd_register(uint32_t* bar) {
    if (threadIdx.x == 0) {
        const uint32_t x = xcd_id();
        const uint32_t a = __hip_atomic_fetch_add(bar + kBarXcdInfo + x, 1u, __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_AGENT);
        if (a == 0) __hip_atomic_fetch_add(bar + kBarXcdInfo + kMaxXcd, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Grid barrier with one L2 write-back per XCD: every wave waits until its
// own stores have completed (they are then in its XCD's L2), the blocks of
// an XCD count their arrivals, and the last block of each XCD writes that
// L2 back to memory (one agent-scope release) and arrives at the top
// level.  The last XCD leader advances the generation; every block then
// drops its stale cache lines (agent-scope acquire) before reading again.
// xsize: blocks on this block's XCD; nx: XCDs holding blocks (both from
// xcd_register).
__device__ __forceinline__ bool xcd_barrier(uint32_t* bar, int32_t* err, uint32_t xsize, uint32_t nx,
                                            uint64_t timeout_ticks) {
    __shared__ int s_ok;
    __builtin_amdgcn_s_waitcnt(0);  // this wave's stores have completed
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        uint32_t* gen_w = bar + kBarLine;
        uint32_t* xtop = bar + kBarXcdTop;
        uint32_t* xctr = bar + kBarXcdCtr + 16 * xcd_id();
        const uint32_t gen = __hip_atomic_load(gen_w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t a = __hip_atomic_fetch_add(xctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bool released = false;
        if (a == xsize - 1) {
            __hip_atomic_store(xctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // every block of this XCD has arrived with its stores in this
            // L2: write it back once for all of them
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t t = __hip_atomic_fetch_add(xtop, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == nx - 1) {
                __hip_atomic_store(xtop, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(gen_w, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                released = true;
            }
        }
        if (!released) ok = wait_generation(gen_w, gen, err, timeout_ticks);
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        s_ok = ok;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
    return s_ok != 0;
}

constexpr int kPBlock = 1024;  // persistent kernel: one 16-wave block per CU

// The CSR and HYB variants and CSR with per-edge costs are built for 64
// VGPRs (two 16-wave blocks per CU; a few bytes of spill in the wider lane
// groups); the variants that decode forward boxes (BOX, mixed) would spill
// some 300 bytes per lane at that budget and run one block per CU.
template <class T, bool MULTI, int ENC, int G>
__global__ __launch_bounds__(kPBlock) __attribute__((amdgpu_waves_per_eu(
    4 * (ENC == 1 ? GBF_PBLOCKS : ENC == 4 ? GBF_PHYB : ENC == 5 ? GBF_PEDGE : 1))))
void k_persistent(const Inst* __restrict__ It, Run R) {
    __shared__ int64_t s_bases[MULTI ? kMaxBatch : 1];
    __shared__ int s_w[kPCompactC * (kPBlock / kWave)];
    __shared__ uint32_t s_base;
    if (MULTI) {
        for (int k = threadIdx.x; k < R.ninst; k += blockDim.x) s_bases[k] = It[k].pair_base;
        __syncthreads();
    }
    if (__hip_atomic_load(R.error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) return;
    __shared__ AccLds s_acc;
    acc_init(s_acc);
    Acc acc;
    uint64_t t_bar = 0;  // block 0: device-clock ticks spent in barriers
    const int64_t ntiles = (R.nchunks + kPBlock * kPCompactC - 1) / (kPBlock * kPCompactC);
#if GBF_XCD_BARRIER
    __shared__ uint32_t s_xsize, s_nx;
    xcd_register(R.barrier);
    if (!grid_barrier(R.barrier, R.error, gridDim.x, R.timeout_ticks)) {
        flush_acc(acc, s_acc, R.slots);
        return;
    }
    if (threadIdx.x == 0) {
        s_xsize = __hip_atomic_load(R.barrier + kBarXcdInfo + xcd_id(), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_nx = __hip_atomic_load(R.barrier + kBarXcdInfo + kMaxXcd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t xsize = s_xsize, nx = s_nx;
#define GBF_PBARRIER() xcd_barrier(R.barrier, R.error, xsize, nx, R.timeout_ticks)
#else
#define GBF_PBARRIER() grid_barrier(R.barrier, R.error, gridDim.x, R.timeout_ticks)
#endif
    for (int round = 0;; ++round) {
        uint8_t* cur = R.dirty[round & 1];
        for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            compact_tile<kPBlock, kPCompactC>(cur, R.nchunks, tile, R.list, R.counts + round, s_w, &s_base);
        uint64_t t0 = wall_clock64();
        const bool ok1 = GBF_PBARRIER();
        t_bar += wall_clock64() - t0;
        if (!ok1) break;
        const uint32_t count = __hip_atomic_load(R.counts + round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (count == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) R.result[0] = round;
            break;
        }
        // one instance: the host-loop relax's mapping of the list (each
        // block one contiguous chunk of its XCD's part; measured 2-7%
        // faster); a batch keeps every wave stepping through the whole list
        if (!MULTI && GBF_PERSIST_MAP && gridDim.x % kXcdParts == 0)
            relax_round<T, MULTI, ENC, G, 1, __HIP_MEMORY_SCOPE_AGENT, false, true>(It, s_bases, R, count, round, acc);
        else
            relax_round<T, MULTI, ENC, G, 1>(It, s_bases, R, count, round, acc);
        fold_acc(acc, s_acc);
        t0 = wall_clock64();
        const bool ok2 = GBF_PBARRIER();
        t_bar += wall_clock64() - t0;
        if (!ok2) break;
    }
#undef GBF_PBARRIER
    if (blockIdx.x == 0 && threadIdx.x == 0) reinterpret_cast<uint64_t*>(R.result)[1] = t_bar;
    flush_acc(acc, s_acc, R.slots);
}

// ------------------------------------------------------------------ single block
// Small instances: all rounds in one 1024-thread workgroup.  The rounds are
// separated by block barriers only (workgroup-scope ordering; V is updated
// with workgroup-scope atomics, so the whole solve stays inside one CU's
// caches), which makes a round cost a few microseconds instead of two
// kernel launches or a grid barrier.
template <class T, int ENC, int G>
__global__ __launch_bounds__(kPBlock) void k_single(const Inst* __restrict__ It, Run R) {
    __shared__ int s_w[kPBlock / kWave];
    __shared__ uint32_t s_base;
    __shared__ AccLds s_acc;
    acc_init(s_acc);
    Acc acc;
    const int64_t ntiles = (R.nchunks + kPBlock - 1) / kPBlock;
    for (int round = 0;; ++round) {
        uint8_t* cur = R.dirty[round & 1];
        if (threadIdx.x == 0) s_base = 0;
        __syncthreads();
        for (int64_t tile = 0; tile < ntiles; ++tile)
            compact_tile<kPBlock, 1, true>(cur, R.nchunks, tile, R.list, R.counts + round, s_w, &s_base);
        const uint32_t count = s_base;  // compact_tile ends with a block barrier
        if (threadIdx.x == 0) R.counts[round] = count;
        if (count == 0) {
            if (threadIdx.x == 0) R.result[0] = round;
            break;
        }
        relax_round<T, false, ENC, G, 1, __HIP_MEMORY_SCOPE_WORKGROUP>(It, nullptr, R, count, round, acc);
        fold_acc(acc, s_acc);
        __syncthreads();
    }
    flush_acc(acc, s_acc, R.slots);
}

// Small instances (CSR with or without per-edge costs, or HYB; one instance, at most kSmallPairs pairs and
// kSmallStates states): the single-block solver with V, both frontiers (as
// bitmaps) and the frontier list in LDS.  Only the read-only successor and
// reverse rows, costs and row bounds come from global memory; a round's
// dependent accesses to V, the marks and the list stay on the CU.  V is
// loaded from (and at the end written back to) global memory; the seeded
// byte map is converted once.
constexpr int kSmallPairs = 16384;
constexpr int kSmallStates = 6144;
constexpr int kSmallWords = kSmallPairs / 32;

template <class T, int G, bool EDGE, bool HYB>
__global__ __launch_bounds__(kPBlock) void k_small(const Inst* __restrict__ It, Run R) {
    using K = typename T::key_t;
    constexpr int NW = kPBlock / kWave;
    constexpr int W = kWave / G;  // pairs per wave step
    __shared__ K s_V[kSmallStates];
    __shared__ uint16_t s_list[kSmallPairs];
    __shared__ uint32_t s_bits[2][kSmallWords];
    __shared__ int s_w[NW];
    __shared__ AccLds s_acc;
    acc_init(s_acc);
    Acc acc;
    const Inst& I = It[0];
    const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
    const int sub = lane & (G - 1), grp = lane / G;
    const int n = (int)I.n, KK = I.K, np = n * KK;
    const int nwords = (np + 31) / 32;  // <= kSmallWords <= kPBlock
    GBF_GLOBAL K* Vg = gp(static_cast<K*>(I.V));
    const GBF_GLOBAL uint32_t* sptr = gp(I.sptr);
    const GBF_GLOBAL int32_t* sidx = gp(I.sidx);
    const GBF_GLOBAL int32_t* gc = gp(I.g);
    const GBF_GLOBAL uint32_t* rptr = gp(I.rptr);
    const GBF_GLOBAL uint32_t* rev = gp(I.rev);
    const GBF_GLOBAL int32_t* hc = gp(I.ge);  // EDGE: per-edge costs
    for (int i = t; i < n; i += kPBlock) s_V[i] = Vg[i];
    {
        const GBF_GLOBAL uint8_t* d0 = gp(R.dirty[0]);
        if (t < nwords) {
            uint32_t bits = 0;
            for (int b = 0; b < 32; ++b) {
                const int q = t * 32 + b;
                if (q < np && d0[q]) bits |= 1u << b;
            }
            s_bits[0][t] = bits;
            s_bits[1][t] = 0u;
        }
    }
    __syncthreads();
    for (int round = 0;; ++round) {
        uint32_t* cur = s_bits[round & 1];
        uint32_t* nxt = s_bits[(round + 1) & 1];
        // frontier list, ascending, from the bits (one word per thread)
        uint32_t word = t < nwords ? cur[t] : 0u;
        const int c = __popc(word);
        const int incl = wave_incl_scan(c);
        if (lane == kWave - 1) s_w[w] = incl;
        __syncthreads();
        int wofs = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < NW; ++k) {
            const int v = s_w[k];
            wofs += k < w ? v : 0;
            tot += v;
        }
        uint32_t pos = (uint32_t)(wofs + incl - c);
        while (word) {
            const int b = __ffs(word) - 1;
            s_list[pos++] = (uint16_t)(t * 32 + b);
            word &= word - 1u;
        }
        if (t < nwords) cur[t] = 0u;
        const uint32_t count = (uint32_t)tot;
        if (t == 0) R.counts[round] = count;
        __syncthreads();  // list complete; s_w read by every thread
        if (count == 0) {
            if (t == 0) R.result[0] = round;
            break;
        }
        if (round >= I.max_rounds) {
            // the round cap (second condition of Algorithm 1's while loop)
            // with work left: drop the frontier, flag the instance
            if (t == 0) R.inst_status[0] = 1;
            continue;
        }
        for (uint32_t first = (uint32_t)(w * W); first < count; first += (uint32_t)(NW * W)) {
            const uint32_t i = first + (uint32_t)grp;
            const bool valid = i < count;
            const uint32_t q = valid ? (uint32_t)s_list[i] : 0u;
            const uint32_t x = q / (uint32_t)KK;
            K mx = (K)T::LOWEST, cv = (K)T::INF;
            typename T::wide_t mw = T::WLOWEST;
            uint32_t len = 0;
            int32_t graw = 0;
            if (valid && HYB) {
                // the box is w1*w2*w3 rows of w0 consecutive cells along axis 0
                graw = gc[q];
                cv = s_V[x];
                const BoxDec bd = decode_box(gp(I.box)[q]);
                const uint32_t w0 = bd.e[0] + 1, w1 = bd.e[1] + 1, w2 = bd.e[2] + 1;
                const uint32_t nrows = w1 * w2 * (uint32_t)(bd.e[3] + 1);
                len = w0 * nrows;
                for (uint32_t r = (uint32_t)sub; r < nrows; r += G) {
                    const uint32_t r2 = r / w1, j1 = r - r2 * w1, j3 = r2 / w2, j2 = r2 - j3 * w2;
                    const uint32_t b0 = (uint32_t)bd.lo + j1 * (uint32_t)I.strides[1] + j2 * (uint32_t)I.strides[2] +
                                        j3 * (uint32_t)I.strides[3];
                    for (uint32_t j0 = 0; j0 < w0; ++j0) mx = T::max2(mx, s_V[b0 + j0]);
                }
            } else if (valid) {
                const uint32_t s0 = sptr[q];
                len = sptr[q + 1] - s0;
                graw = gc[q];
                cv = s_V[x];
                if (EDGE) {
                    for (uint32_t e = (uint32_t)sub; e < len; e += G)
                        mw = T::wmax2(mw, T::edge(hc[s0 + e], s_V[sidx[s0 + e]]));
                } else {
                    for (uint32_t e = (uint32_t)sub; e < len; e += G) mx = T::max2(mx, s_V[sidx[s0 + e]]);
                }
            }
            if (EDGE) mw = group_wmax<T, G>(mw);
            else mx = group_max<T, G>(mx);
            K d = (K)T::INF;
            if (valid) {
                int sat = 0;
                K dd;
                const bool ok = EDGE ? T::backupw(graw, mw, dd, sat) : T::backup(graw, mx, dd, sat);
                if (ok && T::less(dd, cv)) d = dd;
                if (sub == 0) {
                    acc.pairs += 1;
                    acc.edges += len;
                    acc.sat += (unsigned)sat;
                }
            }
            // one candidate per state and wave step (its pairs are adjacent)
            const uint32_t key = valid ? x : 0xffffffffu;
#pragma unroll
            for (int st = 1; st < W; st <<= 1) {
                const K od = __shfl_down(d, st * G, kWave);
                const uint32_t ok = __shfl_down(key, st * G, kWave);
                if (grp + st < W && ok == key) d = T::less(od, d) ? od : d;
            }
            const uint32_t pkey = __shfl_up(key, G, kWave);
            const bool head = valid && sub == 0 && (grp == 0 || pkey != key);
            bool expand = false;
            if (head && T::less(d, cv)) {
                atomicMin(&s_V[x], d);
                acc.impr += 1;
                expand = true;
            }
            unsigned long long bal = __ballot(expand);
            while (bal) {
                const int l = __ffsll(bal) - 1;
                bal &= bal - 1;
                const uint32_t xl = __shfl(x, l, kWave);
                const uint32_t r0 = rptr[xl], rl = rptr[xl + 1] - r0;
                if (lane == 0) {
                    acc.expanded += 1;
                    acc.marks += rl;
                }
                for (uint32_t e = (uint32_t)lane; e < rl; e += kWave) {
                    const uint32_t qp = rev[r0 + e];
                    atomicOr(&nxt[qp >> 5], 1u << (qp & 31u));
                }
            }
        }
        fold_acc(acc, s_acc);
        __syncthreads();  // every mark of the round is in nxt
    }
    __syncthreads();
    for (int i = t; i < n; i += kPBlock) Vg[i] = s_V[i];
    flush_acc(acc, s_acc, R.slots);
}

// ------------------------------------------------------------------ dispatch
// Kernel variants: value type (int32 / fp32 key), single or batched
// instance table, encoding (1 CSR, 2 BOX, 3 mixed batch) and lanes per pair.
using RelaxFn = void (*)(const Inst*, Run, int);
using PersistFn = void (*)(const Inst*, Run);
using SeedFn = void (*)(const Inst*, int, Run);

template <class T, bool MULTI, int ENC>
static void pick(int G, RelaxFn* rf, PersistFn* pf) {
    switch (G) {
        case 1: *rf = k_relax<T, MULTI, ENC, 1>; *pf = k_persistent<T, MULTI, ENC, 1>; break;
        case 2: *rf = k_relax<T, MULTI, ENC, 2>; *pf = k_persistent<T, MULTI, ENC, 2>; break;
        case 4: *rf = k_relax<T, MULTI, ENC, 4>; *pf = k_persistent<T, MULTI, ENC, 4>; break;
        case 16: *rf = k_relax<T, MULTI, ENC, 16>; *pf = k_persistent<T, MULTI, ENC, 16>; break;
        case 32: *rf = k_relax<T, MULTI, ENC, 32>; *pf = k_persistent<T, MULTI, ENC, 32>; break;
        default: *rf = k_relax<T, MULTI, ENC, 8>; *pf = k_persistent<T, MULTI, ENC, 8>; break;
    }
}

// enc_mask: bit 0 = some instance uses CSR, bit 1 = BOX, bit 2 = HYB,
// bit 3 = CSR with per-edge costs.
template <class T>
static void pick_t(bool multi, int enc_mask, int G, RelaxFn* rf, PersistFn* pf) {
    if (multi) {
        if (enc_mask == 1) pick<T, true, 1>(G, rf, pf);
        else if (enc_mask == 2) pick<T, true, 2>(G, rf, pf);
        else if (enc_mask == 4) pick<T, true, 4>(G, rf, pf);
        else if (enc_mask == 8) pick<T, true, 5>(G, rf, pf);
        else pick<T, true, 3>(G, rf, pf);
    } else {
        if (enc_mask == 2) pick<T, false, 2>(G, rf, pf);
        else if (enc_mask == 4) pick<T, false, 4>(G, rf, pf);
        else if (enc_mask == 8) pick<T, false, 5>(G, rf, pf);
        else pick<T, false, 1>(G, rf, pf);
    }
}

static void pick_all(const Run& R, int dtype, int enc_mask, int G, RelaxFn* rf, PersistFn* pf) {
    if (dtype == 1) pick_t<TF32>(R.ninst > 1, enc_mask, G, rf, pf);
    else pick_t<TI32>(R.ninst > 1, enc_mask, G, rf, pf);
}

hipError_t launch_seed(const Inst* dI, int ninst, const Run& R, int64_t max_states, int dtype, int enc_mask,
                       hipStream_t s, bool wide) {
    const int grid = grid_for((max_states + kWave - 1) / kWave, kWavesPerBlock, 4096);
    SeedFn f;
    if (wide) {
        // the seed marks pairs only: the value type does not matter
        f = enc_mask == 2 ? k_seed<TI32, 2, true> : k_seed<TI32, 4, true>;
        f<<<grid, kBlock, 0, s>>>(dI, ninst, R);
        return hipGetLastError();
    }
    // the seed reads only the successor structure: per-edge costs do not matter
    if (enc_mask == 8) enc_mask = 1;
    if (dtype == 1)
        f = enc_mask == 1 ? k_seed<TF32, 1> : enc_mask == 2 ? k_seed<TF32, 2> : enc_mask == 4 ? k_seed<TF32, 4>
                                                                                         : k_seed<TF32, 3>;
    else
        f = enc_mask == 1 ? k_seed<TI32, 1> : enc_mask == 2 ? k_seed<TI32, 2> : enc_mask == 4 ? k_seed<TI32, 4>
                                                                                         : k_seed<TI32, 3>;
    f<<<grid, kBlock, 0, s>>>(dI, ninst, R);
    return hipGetLastError();
}

using SingleFn = void (*)(const Inst*, Run);

template <class T, int ENC>
static SingleFn pick_single(int G) {
    switch (G) {
        case 1: return k_single<T, ENC, 1>;
        case 2: return k_single<T, ENC, 2>;
        case 8: return k_single<T, ENC, 8>;
        case 16: return k_single<T, ENC, 16>;
        case 32: return k_single<T, ENC, 32>;
        default: return k_single<T, ENC, 4>;
    }
}

template <class T>
static SingleFn pick_single_t(int enc_mask, int G) {
    if (enc_mask == 2) return pick_single<T, 2>(G);
    if (enc_mask == 4) return pick_single<T, 4>(G);
    if (enc_mask == 8) return pick_single<T, 5>(G);
    return pick_single<T, 1>(G);
}

template <class T, bool EDGE, bool HYB>
static SingleFn pick_small(int G) {
    switch (G) {
        case 1: return k_small<T, 1, EDGE, HYB>;
        case 2: return k_small<T, 2, EDGE, HYB>;
        case 8: return k_small<T, 8, EDGE, HYB>;
        case 16: return k_small<T, 16, EDGE, HYB>;
        case 32: return k_small<T, 32, EDGE, HYB>;
        default: return k_small<T, 4, EDGE, HYB>;
    }
}

hipError_t launch_single(const Inst* dI, const Run& R, int lanes, int dtype, int enc_mask, int64_t n_states,
                         hipStream_t s) {
    SingleFn f;
    if (GBF_SMALL_LDS && (enc_mask == 1 || enc_mask == 4 || enc_mask == 8) && R.ninst == 1 &&
        R.total_pairs <= kSmallPairs && n_states <= kSmallStates) {
        if (enc_mask == 8) f = dtype == 1 ? pick_small<TF32, true, false>(lanes) : pick_small<TI32, true, false>(lanes);
        else if (enc_mask == 4) f = dtype == 1 ? pick_small<TF32, false, true>(lanes) : pick_small<TI32, false, true>(lanes);
        else f = dtype == 1 ? pick_small<TF32, false, false>(lanes) : pick_small<TI32, false, false>(lanes);
    } else
        f = dtype == 1 ? pick_single_t<TF32>(enc_mask, lanes) : pick_single_t<TI32>(enc_mask, lanes);
    f<<<1, kPBlock, 0, s>>>(dI, R);
    return hipGetLastError();
}

// 64-bit pair ids: one instance, BOX (2) or HYB (4), lanes 2, 4 or 8.
template <class T, int ENC>
static RelaxFn pick_wide_enc(int G) {
    switch (G) {
        case 2: return k_relax<T, false, ENC, 2, true>;
        case 8: return k_relax<T, false, ENC, 8, true>;
        default: return k_relax<T, false, ENC, 4, true>;
    }
}

static RelaxFn pick_wide(int dtype, int enc_mask, int G) {
    if (dtype == 1) return enc_mask == 2 ? pick_wide_enc<TF32, 2>(G) : pick_wide_enc<TF32, 4>(G);
    return enc_mask == 2 ? pick_wide_enc<TI32, 2>(G) : pick_wide_enc<TI32, 4>(G);
}

hipError_t launch_relax(const Inst* dI, const Run& R, int round, int grid, int lanes, int dtype, int enc_mask,
                        hipStream_t s, bool wide, int block) {
    RelaxFn rf;
    PersistFn pf;
    if (wide) rf = pick_wide(dtype, enc_mask, lanes);
    else pick_all(R, dtype, enc_mask, lanes, &rf, &pf);
    // `grid` counts kBlock-thread blocks; the relax kernel runs `block`
    // threads per block (any multiple of 64 up to 1024, default kRelaxBlock)
    // in at most kMaxGrid blocks (one statistics slot each)
    const int b = block > 0 ? block : kRelaxBlock;
    const int g = grid > 0 ? std::min(grid, kMaxGrid) : 1024;
    const int nb = (int)std::min<int64_t>(kMaxGrid, std::max<int64_t>(1, (int64_t)g * kBlock / b));
    rf<<<nb, b, 0, s>>>(dI, R, round);
    return hipGetLastError();
}

int persistent_blocks_per_cu(const Run& R, int lanes, int dtype, int enc_mask) {
    RelaxFn rf;
    PersistFn pf;
    pick_all(R, dtype, enc_mask, lanes, &rf, &pf);
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(pf), kPBlock, 0) !=
        hipSuccess)
        return 0;
    return nb;
}

hipError_t launch_persistent(const Inst* dI, const Run& R, int grid, int lanes, int dtype, int enc_mask,
                             bool attr_launch, hipStream_t s) {
    RelaxFn rf;
    PersistFn pf;
    pick_all(R, dtype, enc_mask, lanes, &rf, &pf);
    Run r = R;
    const Inst* di = dI;
    void* args[] = {(void*)&di, (void*)&r};
    if (attr_launch) {
        hipLaunchAttribute attr;
        std::memset(&attr, 0, sizeof(attr));
        attr.id = hipLaunchAttributeCooperative;
        attr.val.cooperative = 1;
        hipLaunchConfig_t cfg;
        std::memset(&cfg, 0, sizeof(cfg));
        cfg.gridDim = dim3(grid);
        cfg.blockDim = dim3(kPBlock);
        cfg.dynamicSmemBytes = 0;
        cfg.stream = s;
        cfg.attrs = &attr;
        cfg.numAttrs = 1;
        return hipLaunchKernelExC(&cfg, reinterpret_cast<const void*>(pf), args);
    }
    return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(pf), dim3(grid), dim3(kPBlock), args, 0, s);
}

// ------------------------------------------------------------------ outputs
template <class T>
__global__ void k_decode(Inst I, int32_t* out) {
    const auto* V = static_cast<const typename T::key_t*>(I.V);
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < I.n; x += (int64_t)gridDim.x * blockDim.x)
        out[x] = T::out_word(V[x]);
}

hipError_t launch_decode(const Inst& I, int dtype, void* out, hipStream_t s) {
    if (dtype == 1) k_decode<TF32><<<grid_for(I.n, 256), 256, 0, s>>>(I, (int32_t*)out);
    else k_decode<TI32><<<grid_for(I.n, 256), 256, 0, s>>>(I, (int32_t*)out);
    return hipGetLastError();
}

// Canonical controller and fixed-point residual: one application of P to
// the final V.  One lane per pair; a wave holds 64/K whole states, so the
// scan over a state's inputs (ascending u, first strict improvement over
// G, hand over on ties with G) reads the K backups from LDS.
template <class T, int ENC>
__global__ __launch_bounds__(kBlock) void k_policy(Inst I, int32_t* pol, unsigned long long* bad) {
    using K = typename T::key_t;
    __shared__ K s_d[kBlock];
    const GBF_GLOBAL K* V = gp(static_cast<const K*>(I.V));
    const int lane = lane_id();
    const int K_ = I.K;
    const int spw = kWave / K_;  // whole states per wave
    const int64_t nsteps = (I.n + spw - 1) / spw;
    unsigned long long nb = 0;
    K* sd = s_d + (threadIdx.x / kWave) * kWave;
    for (int64_t st = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; st < nsteps;
         st += (int64_t)gridDim.x * kWavesPerBlock) {
        const int si = lane / K_, u = lane - si * K_;
        const int64_t x = st * spw + si;
        const bool valid = si < spw && x < I.n;
        K d = (K)T::INF;
        if (valid) {
            const int64_t p = x * K_ + u;
            K m = (K)T::LOWEST;
            typename T::wide_t mw = T::WLOWEST;
            if (ENC == 5) {
                const GBF_GLOBAL uint32_t* sptr = gp(I.sptr);
                const GBF_GLOBAL int32_t* sidx = gp(I.sidx);
                const GBF_GLOBAL int32_t* h = gp(I.ge);
                const uint32_t e1 = ldx<GBF_NT_MISC>(sptr + p + 1);
                for (uint32_t j = ldx<GBF_NT_MISC>(sptr + p); j < e1; ++j)
                    mw = T::wmax2(mw, T::edge(ldx<GBF_NT_ROWS>(h + j), V[ldx<GBF_NT_ROWS>(sidx + j)]));
            } else if (ENC == 1) {
                const GBF_GLOBAL uint32_t* sptr = gp(I.sptr);
                const GBF_GLOBAL int32_t* sidx = gp(I.sidx);
                const uint32_t e1 = ldx<GBF_NT_MISC>(sptr + p + 1);
                uint32_t j = ldx<GBF_NT_MISC>(sptr + p);
                // four independent gathers in flight per lane
                for (; j + 4 <= e1; j += 4) {
                    const int32_t y0 = ldx<GBF_NT_ROWS>(sidx + j), y1 = ldx<GBF_NT_ROWS>(sidx + j + 1),
                                  y2 = ldx<GBF_NT_ROWS>(sidx + j + 2), y3 = ldx<GBF_NT_ROWS>(sidx + j + 3);
                    m = T::max2(T::max2(m, T::max2(V[y0], V[y1])), T::max2(V[y2], V[y3]));
                }
                for (; j < e1; ++j) m = T::max2(m, V[ldx<GBF_NT_ROWS>(sidx + j)]);
            } else {
                const BoxDec bd = decode_box(ldx<GBF_NT_MISC>(gp(I.box) + p));
                for (int j3 = 0; j3 <= bd.e[3]; ++j3)
                    for (int j2 = 0; j2 <= bd.e[2]; ++j2)
                        for (int j1 = 0; j1 <= bd.e[1]; ++j1) {
                            const int64_t r0 = bd.lo + (int64_t)j1 * I.strides[1] + (int64_t)j2 * I.strides[2] +
                                               (int64_t)j3 * I.strides[3];
                            for (int j0 = 0; j0 <= bd.e[0]; ++j0) m = T::max2(m, V[r0 + j0]);
                        }
            }
            K dd;
            int sat = 0;
            if (ENC == 5 ? T::backupw(gp(I.g)[p], mw, dd, sat) : T::backup(gp(I.g)[p], m, dd, sat)) d = dd;
        }
        sd[lane] = d;
        wave_sync();
        if (valid && u == 0) {
            const K vx = V[x];
            if (I.avoid[x]) {
                pol[x] = -2;
                nb += vx != T::INF;
            } else {
                K best = T::from_raw(gp(I.G)[x]);
                int pu = -1;
                for (int k = 0; k < K_; ++k) {
                    const K dk = sd[si * K_ + k];
                    if (T::less(dk, best)) {
                        best = dk;
                        pu = k;
                    }
                }
                if (best == T::INF) pu = -2;
                pol[x] = pu;
                nb += best != vx;
            }
        }
        wave_sync();
    }
    nb = wave_sum64(nb);
    if (lane_id() == 0 && nb) atomicAdd(bad, nb);
}

// States with more than 64 inputs: one thread per state.
template <class T>
__global__ void k_policy_wide(Inst I, int32_t* pol, unsigned long long* bad) {
    using K = typename T::key_t;
    const K* V = static_cast<const K*>(I.V);
    unsigned long long nb = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < I.n; x += (int64_t)gridDim.x * blockDim.x) {
        const K vx = V[x];
        if (I.avoid[x]) {
            pol[x] = -2;
            nb += vx != T::INF;
            continue;
        }
        K best = T::from_raw(I.G[x]);
        int pu = -1;
        for (int u = 0; u < I.K; ++u) {
            const int64_t p = x * I.K + u;
            K m = (K)T::LOWEST;
            typename T::wide_t mw = T::WLOWEST;
            if (I.enc == 0 && I.ge) {
                for (uint32_t j = I.sptr[p]; j < I.sptr[p + 1]; ++j) mw = T::wmax2(mw, T::edge(I.ge[j], V[I.sidx[j]]));
            } else if (I.enc == 0) {
                for (uint32_t j = I.sptr[p]; j < I.sptr[p + 1]; ++j) m = T::max2(m, V[I.sidx[j]]);
            } else {
                const BoxDec d = decode_box(I.box[p]);
                for (int j3 = 0; j3 <= d.e[3]; ++j3)
                    for (int j2 = 0; j2 <= d.e[2]; ++j2)
                        for (int j1 = 0; j1 <= d.e[1]; ++j1)
                            for (int j0 = 0; j0 <= d.e[0]; ++j0)
                                m = T::max2(m, V[d.lo + j0 + (int64_t)j1 * I.strides[1] +
                                                 (int64_t)j2 * I.strides[2] + (int64_t)j3 * I.strides[3]]);
            }
            K d;
            int sat = 0;
            const bool ok = (I.enc == 0 && I.ge) ? T::backupw(I.g[p], mw, d, sat) : T::backup(I.g[p], m, d, sat);
            if (ok && T::less(d, best)) {
                best = d;
                pu = u;
            }
        }
        if (best == T::INF) pu = -2;
        pol[x] = pu;
        nb += best != vx;
    }
    nb = wave_sum64(nb);
    if (lane_id() == 0 && nb) atomicAdd(bad, nb);
}

hipError_t launch_policy(const Inst& I, int dtype, int32_t* pol, unsigned long long* bad, hipStream_t s) {
    if (I.K > kWave) {
        if (dtype == 1) k_policy_wide<TF32><<<grid_for(I.n, 256), 256, 0, s>>>(I, pol, bad);
        else k_policy_wide<TI32><<<grid_for(I.n, 256), 256, 0, s>>>(I, pol, bad);
        return hipGetLastError();
    }
    const int64_t steps = (I.n + (kWave / I.K) - 1) / (kWave / I.K);
    const int grid = grid_for(steps, kWavesPerBlock, 8192);
    if (dtype == 1) {
        if (I.enc == 0 && I.ge) k_policy<TF32, 5><<<grid, kBlock, 0, s>>>(I, pol, bad);
        else if (I.enc == 0) k_policy<TF32, 1><<<grid, kBlock, 0, s>>>(I, pol, bad);
        else k_policy<TF32, 2><<<grid, kBlock, 0, s>>>(I, pol, bad);
    } else {
        if (I.enc == 0 && I.ge) k_policy<TI32, 5><<<grid, kBlock, 0, s>>>(I, pol, bad);
        else if (I.enc == 0) k_policy<TI32, 1><<<grid, kBlock, 0, s>>>(I, pol, bad);
        else k_policy<TI32, 2><<<grid, kBlock, 0, s>>>(I, pol, bad);
    }
    return hipGetLastError();
}

}  // namespace gbf
