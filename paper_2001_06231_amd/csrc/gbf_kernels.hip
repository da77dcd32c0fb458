// HIP kernels of the gbf solver for gfx950 (CDNA4, wave64).
//
// The hot path is one pass of the while loop of Algorithm 1 (Sect. IV-A),
// restated for a data-parallel machine:
//   compact : the dirty-pair bitmap of the active frontier is turned into a
//             list of pair ids (ballot-free popcount scan per block, one
//             global atomic per block) and cleared;
//   relax   : for every listed pair (x,u) the max of W over F(x,u) is formed
//             with all 64 lanes of a wave streaming the concatenated
//             successor rows of 64 pairs (coalesced reads, per-segment max in
//             LDS), then d = g(x,u) + max is compared with W(x) and applied
//             by atomicMin (the strict-improvement update);
//   expand  : the first improvement of a state in a round marks every pair
//             (x',u') with that state in F(x',u') in the upcoming frontier's
//             bitmap (pair-level refinement of pred(x,u), Sect. IV-A).
// Pairs are the frontier's unit (not states as in the paper's F1 x U): a pair
// whose successors did not change cannot improve, so only pairs with a
// changed successor are evaluated.  Any evaluation order reaches the same
// maximal fixed point (Sect. IV-A: the processing order is irrelevant; the
// operator is monotone and every pair is re-evaluated after its last
// successor change).
#include "gbf_device.h"
#include "gbf_internal.h"

namespace gbf {

constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

struct Acc {
    unsigned long long pairs = 0, edges = 0, impr = 0, sat = 0;
};

struct WaveLds {
    int off[kWave];
    const int32_t* row[kWave];
    void* vbase[kWave];
    uint32_t mx[kWave];
    int64_t qbase[kWave];
};

__device__ __forceinline__ void flush_acc(const Acc& a, unsigned long long* ctr) {
    unsigned long long p = wave_sum64(a.pairs), e = wave_sum64(a.edges), i = wave_sum64(a.impr),
                       s = wave_sum64(a.sat);
    if (lane_id() == 0) {
        if (p) atomicAdd(ctr + 0, p);
        if (e) atomicAdd(ctr + 1, e);
        if (i) atomicAdd(ctr + 2, i);
        if (s) atomicAdd(ctr + 3, s);
    }
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
__global__ void k_box_window(Inst I, int dtype, int32_t* win) {
    const int64_t npairs = I.n * I.K;
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
            atomicMin(win + u * 8 + a, lc - xc);
            atomicMax(win + u * 8 + 4 + a, lc + d.e[a] - xc);
        }
    }
}

hipError_t launch_box_window(const Inst& I, int32_t* win32, hipStream_t s) {
    k_box_window<<<grid_for(I.n * I.K, 256), 256, 0, s>>>(I, I.dtype, win32);
    return hipGetLastError();
}

// ------------------------------------------------------------------ init
// W <- G (Algorithm 1 initialisation), avoid cells pinned to INF; stamps
// cleared.
template <class T>
__global__ void k_init(Inst I) {
    auto* V = static_cast<typename T::key_t*>(I.V);
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < I.n; x += (int64_t)gridDim.x * blockDim.x) {
        V[x] = (I.avoid && I.avoid[x]) ? T::INF : T::from_raw(I.G[x]);
        I.stamp[x] = -1;
    }
}

hipError_t launch_init(const Inst* dI, const Inst& I, int dtype, hipStream_t s) {
    (void)dI;
    if (dtype == 1) k_init<TF32><<<grid_for(I.n, 256), 256, 0, s>>>(I);
    else k_init<TI32><<<grid_for(I.n, 256), 256, 0, s>>>(I);
    return hipGetLastError();
}

// ------------------------------------------------------------------ expand
// Marks in `bits` every live pair (x',u') with y in F(x',u'), for the
// states y of the lanes with `active` set.  CSR: the 64 reverse rows are
// streamed by the whole wave.
__device__ __forceinline__ void expand_wave_csr(const Inst& I, bool active, int64_t y, uint32_t* bits, WaveLds& S) {
    const int lane = lane_id();
    uint32_t s0 = 0, len = 0;
    if (active) {
        s0 = I.rptr[y];
        len = I.rptr[y + 1] - s0;
    }
    const int incl = wave_incl_scan((int)len);
    const int total = __shfl(incl, kWave - 1, kWave);
    if (total == 0) return;
    wave_sync();
    S.off[lane] = incl - (int)len;
    S.row[lane] = reinterpret_cast<const int32_t*>(I.rev + s0);
    S.qbase[lane] = I.pair_base;
    wave_sync();
    for (int j = lane; j < total; j += kWave) {
        const int k = seg_search(S.off, j);
        const uint32_t q = (uint32_t)S.row[k][j - S.off[k]];
        set_bit(bits, (uint32_t)S.qbase[k] + q);
    }
    wave_sync();
}

// BOX: every input's predecessor window is scanned and filtered by
// decoding the candidate's box (lane per state).
__device__ __forceinline__ void expand_lane_box(const Inst& I, int64_t y, uint32_t* bits, int dtype) {
    int yc[4];
    int64_t r = y;
    for (int a = 0; a < 4; ++a) {
        yc[a] = (int)(r % I.dims[a]);
        r /= I.dims[a];
    }
    const uint32_t base = (uint32_t)I.pair_base;
    for (int u = 0; u < I.K; ++u) {
        const int32_t* w = I.win + u * 8;
        int lo[4], hi[4];
        bool empty = false;
        for (int a = 0; a < 4; ++a) {
            lo[a] = max(0, yc[a] - w[4 + a]);
            hi[a] = min(I.dims[a] - 1, yc[a] - w[a]);
            empty |= lo[a] > hi[a];
        }
        if (empty) continue;
        for (int c3 = lo[3]; c3 <= hi[3]; ++c3)
            for (int c2 = lo[2]; c2 <= hi[2]; ++c2)
                for (int c1 = lo[1]; c1 <= hi[1]; ++c1)
                    for (int c0 = lo[0]; c0 <= hi[0]; ++c0) {
                        const int64_t x = c0 + (int64_t)c1 * I.strides[1] + (int64_t)c2 * I.strides[2] +
                                          (int64_t)c3 * I.strides[3];
                        const int64_t q = x * I.K + u;
                        if (!pair_live(I, q, dtype)) continue;
                        BoxDec d = decode_box(I.box[q]);
                        int64_t rr = d.lo;
                        bool in = true;
                        for (int a = 0; a < 4; ++a) {
                            int lc = (int)(rr % I.dims[a]);
                            rr /= I.dims[a];
                            in &= (yc[a] >= lc) && (yc[a] <= lc + d.e[a]);
                        }
                        if (in) set_bit(bits, base + (uint32_t)q);
                    }
    }
}

// Seed: F1 <- union of pred(y) over states with G(y) < INF (Algorithm 1
// initialisation), at pair level.
template <class T>
__global__ __launch_bounds__(kBlock) void k_seed(const Inst* __restrict__ It, int ninst, Run R) {
    __shared__ WaveLds lds[kWavesPerBlock];
    WaveLds& S = lds[threadIdx.x / kWave];
    for (int ii = 0; ii < ninst; ++ii) {
        const Inst I = It[ii];
        const int64_t nw = (I.n + kWave - 1) / kWave;
        for (int64_t w = blockIdx.x * (int64_t)kWavesPerBlock + threadIdx.x / kWave; w < nw;
             w += (int64_t)gridDim.x * kWavesPerBlock) {
            const int64_t y = w * kWave + lane_id();
            bool act = false;
            if (y < I.n) {
                const auto Gk = T::from_raw(I.G[y]);
                act = Gk != T::INF && !(I.avoid && I.avoid[y]);
            }
            if (I.enc == 0) expand_wave_csr(I, act, y, R.bits[0], S);
            else if (act) expand_lane_box(I, y, R.bits[0], R.dtype);
        }
    }
}

hipError_t launch_seed(const Inst* dI, int ninst, const Run& R, int64_t max_states, int dtype, hipStream_t s) {
    const int grid = grid_for((max_states + kWave - 1) / kWave, kWavesPerBlock, 4096);
    if (dtype == 1) k_seed<TF32><<<grid, kBlock, 0, s>>>(dI, ninst, R);
    else k_seed<TI32><<<grid, kBlock, 0, s>>>(dI, ninst, R);
    return hipGetLastError();
}

// ------------------------------------------------------------------ compact
// One tile = kBlock bitmap words.  Each thread owns one word; a block scan
// of the popcounts places the set bits (ascending within the tile) after a
// single global atomicAdd per tile.  Words are cleared as they are read.
__device__ __forceinline__ void compact_tile(uint32_t* __restrict__ bits, int64_t nwords, int64_t tile,
                                             uint32_t* __restrict__ list, uint32_t* cnt, int* s_w, uint32_t* s_base) {
    const int t = threadIdx.x;
    const int64_t wi = tile * kBlock + t;
    uint32_t word = wi < nwords ? bits[wi] : 0u;
    const int c = __popc(word);
    const int incl = wave_incl_scan(c);
    const int w = t / kWave;
    if (lane_id() == kWave - 1) s_w[w] = incl;
    __syncthreads();
    int wofs = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < kWavesPerBlock; ++k) {
        const int v = s_w[k];
        wofs += k < w ? v : 0;
        tot += v;
    }
    if (tot != 0) {
        if (t == 0) *s_base = atomicAdd(cnt, (uint32_t)tot);
        __syncthreads();
        uint32_t pos = *s_base + (uint32_t)(wofs + incl - c);
        if (word) {
            bits[wi] = 0u;
            const uint32_t bitbase = (uint32_t)(wi * 32);
            while (word) {
                const int b = __ffs(word) - 1;
                list[pos++] = bitbase + (uint32_t)b;
                word &= word - 1u;
            }
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(kBlock) void k_compact(Run R, int round) {
    __shared__ int s_w[kWavesPerBlock];
    __shared__ uint32_t s_base;
    if (round > 0 && R.counts[round - 1] == 0) return;  // frontier already empty
    uint32_t* bits = R.bits[round & 1];
    const int64_t ntiles = (R.nwords + kBlock - 1) / kBlock;
    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
        compact_tile(bits, R.nwords, tile, R.list, R.counts + round, s_w, &s_base);
}

hipError_t launch_compact(const Run& R, int round, int grid, hipStream_t s) {
    const int64_t ntiles = (R.nwords + kBlock - 1) / kBlock;
    int g = (int)std::min<int64_t>(ntiles, grid > 0 ? grid : 2048);
    if (g < 1) g = 1;
    k_compact<<<g, kBlock, 0, s>>>(R, round);
    return hipGetLastError();
}

// ------------------------------------------------------------------ relax
// One wave handles list entries [base, base+64).  CSR: the successor rows of
// the 64 pairs are concatenated and streamed by all lanes (coalesced), each
// lane folding V[y] into its pair's LDS max; BOX: each lane decodes its own
// box and walks it.
template <class T, bool MULTI>
__device__ __forceinline__ void relax_chunk(const Inst* __restrict__ It, const int64_t* bases, int ninst,
                                            const Run& R, uint32_t count, uint32_t base, int round,
                                            uint32_t* __restrict__ next, WaveLds& S, Acc& acc, int enc_mask) {
    using K = typename T::key_t;
    const int lane = lane_id();
    const uint32_t i = base + (uint32_t)lane;
    bool valid = i < count;
    const uint32_t q = valid ? R.list[i] : 0u;
    const int ii = find_inst<MULTI>(bases, ninst, (int64_t)q);
    const Inst& I = It[ii];
    const int64_t p = (int64_t)q - (MULTI ? I.pair_base : 0);
    if (valid && round >= I.max_rounds) {
        // this instance's round cap is reached with work left (Algorithm 1's
        // second loop condition): its pairs are dropped and it is flagged
        R.inst_status[ii] = 1;
        valid = false;
    }
    K* V = static_cast<K*>(I.V);
    K m = T::INF;
    if (enc_mask & 1) {  // some CSR instance present
        const bool csr = valid && I.enc == 0;
        uint32_t s0 = 0, len = 0;
        if (csr) {
            s0 = I.sptr[p];
            len = I.sptr[p + 1] - s0;
        }
        const int incl = wave_incl_scan((int)len);
        const int total = __shfl(incl, kWave - 1, kWave);
        S.off[lane] = incl - (int)len;
        S.row[lane] = I.sidx + s0;
        S.vbase[lane] = I.V;
        S.mx[lane] = (uint32_t)T::LOWEST;
        wave_sync();
        for (int j = lane; j < total; j += kWave) {
            const int k = seg_search(S.off, j);
            const int32_t y = S.row[k][j - S.off[k]];
            const K v = MULTI ? static_cast<const K*>(S.vbase[k])[y] : V[y];
            T::lds_max(reinterpret_cast<K*>(&S.mx[k]), v);
        }
        wave_sync();
        if (csr) {
            m = (K)S.mx[lane];
            acc.edges += len;
        }
        wave_sync();
    }
    if ((enc_mask & 2) && valid && I.enc == 1) {
        const BoxDec d = decode_box(I.box[p]);
        K mx = (K)T::LOWEST;
        for (int j3 = 0; j3 <= d.e[3]; ++j3)
            for (int j2 = 0; j2 <= d.e[2]; ++j2)
                for (int j1 = 0; j1 <= d.e[1]; ++j1) {
                    const K* row = V + d.lo + (int64_t)j1 * I.strides[1] + (int64_t)j2 * I.strides[2] +
                                   (int64_t)j3 * I.strides[3];
                    for (int j0 = 0; j0 <= d.e[0]; ++j0) mx = T::max2(mx, row[j0]);
                }
        m = mx;
        acc.edges += (unsigned long long)(d.e[0] + 1) * (d.e[1] + 1) * (d.e[2] + 1) * (d.e[3] + 1);
    }
    bool improved = false;
    int64_t x = 0;
    if (valid) {
        acc.pairs += 1;
        x = p / I.K;
        K d;
        int sat = 0;
        if (T::backup(I.g[p], m, d, sat)) {
            acc.sat += (unsigned)sat;
            const K cur = __hip_atomic_load(V + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (T::less(d, cur)) {
                const K old = T::amin(V + x, d);
                if (T::less(d, old)) {
                    improved = true;
                    acc.impr += 1;
                }
            }
        }
    }
    // first improvement of x in this round expands it (one expansion per
    // state and round suffices: pairs marked now re-read V(x) next round)
    const bool expand = improved && (atomicExch(I.stamp + x, round) != round);
    if (enc_mask & 1) expand_wave_csr(I, expand && I.enc == 0, x, next, S);
    if ((enc_mask & 2) && expand && I.enc == 1) expand_lane_box(I, x, next, R.dtype);
}

template <class T, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_relax(const Inst* __restrict__ It, Run R, int round, int enc_mask) {
    __shared__ WaveLds lds[kWavesPerBlock];
    __shared__ int64_t s_bases[MULTI ? kMaxBatch : 1];
    const uint32_t count = R.counts[round];
    if (count == 0) return;
    if (MULTI) {
        for (int k = threadIdx.x; k < R.ninst; k += blockDim.x) s_bases[k] = It[k].pair_base;
        __syncthreads();
    }
    WaveLds& S = lds[threadIdx.x / kWave];
    Acc acc;
    uint32_t* next = R.bits[(round + 1) & 1];
    const uint32_t nchunks = (count + kWave - 1) / kWave;
    for (uint32_t c = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; c < nchunks;
         c += gridDim.x * kWavesPerBlock)
        relax_chunk<T, MULTI>(It, s_bases, R.ninst, R, count, c * kWave, round, next, S, acc, enc_mask);
    flush_acc(acc, R.ctr);
}

hipError_t launch_relax(const Inst* dI, const Run& R, int round, int grid, int block, int dtype, int enc_mask,
                        hipStream_t s) {
    (void)block;
    const int g = grid > 0 ? grid : 1024;
    const bool multi = R.ninst > 1;
    if (dtype == 1) {
        if (multi) k_relax<TF32, true><<<g, kBlock, 0, s>>>(dI, R, round, enc_mask);
        else k_relax<TF32, false><<<g, kBlock, 0, s>>>(dI, R, round, enc_mask);
    } else {
        if (multi) k_relax<TI32, true><<<g, kBlock, 0, s>>>(dI, R, round, enc_mask);
        else k_relax<TI32, false><<<g, kBlock, 0, s>>>(dI, R, round, enc_mask);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ persistent
// All rounds in one launch.  Every wait is bounded: a barrier that does not
// complete within ~2 s sets R.error and every block leaves the loop.
constexpr uint64_t kSpinLimit = 1ull << 25;

__device__ __forceinline__ bool grid_barrier(uint32_t* bar, int32_t* err, uint32_t nblocks) {
    __shared__ int s_ok;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        int ok = 1;
        const uint32_t gen = __hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t arrived = __hip_atomic_fetch_add(bar, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (arrived == nblocks - 1) {
            __hip_atomic_store(bar, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(bar + 1, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint64_t spins = 0;
            while (__hip_atomic_load(bar + 1, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                __builtin_amdgcn_s_sleep(2);
                if (++spins > kSpinLimit) {
                    atomicOr(err, 1);
                    ok = 0;
                    break;
                }
            }
        }
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) ok = 0;
        s_ok = ok;
    }
    __syncthreads();
    __threadfence();
    return s_ok != 0;
}

template <class T, bool MULTI>
__global__ __launch_bounds__(kBlock) void k_persistent(const Inst* __restrict__ It, Run R, int enc_mask) {
    __shared__ WaveLds lds[kWavesPerBlock];
    __shared__ int64_t s_bases[MULTI ? kMaxBatch : 1];
    __shared__ int s_w[kWavesPerBlock];
    __shared__ uint32_t s_base;
    if (MULTI) {
        for (int k = threadIdx.x; k < R.ninst; k += blockDim.x) s_bases[k] = It[k].pair_base;
        __syncthreads();
    }
    WaveLds& S = lds[threadIdx.x / kWave];
    Acc acc;
    const int64_t ntiles = (R.nwords + kBlock - 1) / kBlock;
    for (int round = 0;; ++round) {
        uint32_t* cur = R.bits[round & 1];
        for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x)
            compact_tile(cur, R.nwords, tile, R.list, R.counts + round, s_w, &s_base);
        if (!grid_barrier(R.barrier, R.error, gridDim.x)) break;
        const uint32_t count = __hip_atomic_load(R.counts + round, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (count == 0) {
            if (blockIdx.x == 0 && threadIdx.x == 0) R.result[0] = round;
            break;
        }
        uint32_t* next = R.bits[(round + 1) & 1];
        const uint32_t nchunks = (count + kWave - 1) / kWave;
        for (uint32_t c = blockIdx.x * kWavesPerBlock + threadIdx.x / kWave; c < nchunks;
             c += gridDim.x * kWavesPerBlock)
            relax_chunk<T, MULTI>(It, s_bases, R.ninst, R, count, c * kWave, round, next, S, acc, enc_mask);
        if (!grid_barrier(R.barrier, R.error, gridDim.x)) break;
    }
    flush_acc(acc, R.ctr);
}

template <class T, bool MULTI>
static int occ_of() {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent<T, MULTI>, kBlock, 0) != hipSuccess) return 0;
    return nb;
}

int persistent_blocks_per_cu(int block, int dtype, int enc_mask) {
    (void)block;
    (void)enc_mask;
    return dtype == 1 ? std::min(occ_of<TF32, false>(), occ_of<TF32, true>())
                      : std::min(occ_of<TI32, false>(), occ_of<TI32, true>());
}

hipError_t launch_persistent(const Inst* dI, const Run& R, int grid, int block, int dtype, int enc_mask,
                             hipStream_t s) {
    (void)block;
    const bool multi = R.ninst > 1;
    Run r = R;
    int em = enc_mask;
    void* args[] = {(void*)&dI, (void*)&r, (void*)&em};
    const void* fn;
    if (dtype == 1) fn = multi ? (const void*)k_persistent<TF32, true> : (const void*)k_persistent<TF32, false>;
    else fn = multi ? (const void*)k_persistent<TI32, true> : (const void*)k_persistent<TI32, false>;
    return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
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

// Canonical controller and fixed-point residual: per state, one application
// of P to the final V, scanning inputs in ascending order and keeping the
// first strict improvement over G (hand over on ties with G).
template <class T>
__global__ void k_policy(Inst I, int32_t* pol, unsigned long long* bad) {
    using K = typename T::key_t;
    const K* V = static_cast<const K*>(I.V);
    unsigned long long nb = 0;
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < I.n; x += (int64_t)gridDim.x * blockDim.x) {
        const K vx = V[x];
        if (I.avoid && I.avoid[x]) {
            pol[x] = -2;
            nb += vx != T::INF;
            continue;
        }
        K best = T::from_raw(I.G[x]);
        int pu = -1;
        for (int u = 0; u < I.K; ++u) {
            const int64_t p = x * I.K + u;
            K m = (K)T::LOWEST;
            if (I.enc == 0) {
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
            if (T::backup(I.g[p], m, d, sat) && T::less(d, best)) {
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
    if (dtype == 1) k_policy<TF32><<<grid_for(I.n, 256), 256, 0, s>>>(I, pol, bad);
    else k_policy<TI32><<<grid_for(I.n, 256), 256, 0, s>>>(I, pol, bad);
    return hipGetLastError();
}

}  // namespace gbf
