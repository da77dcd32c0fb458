// Device-side building blocks of the gbf solver (gfx950, wave64).
//
// Value types.  V lives in device memory as 32-bit words that order like the
// values, so one integer atomicMin implements the strict-improvement update
// of Algorithm 1 (Sect. IV-A: if d < W(x) then W(x) <- d) without locks:
//   - int32 costs: the int32 value itself, INF = INT32_MAX;
//   - fp32 costs:  an order-preserving key of the float (sign bit flipped
//     for non-negatives, all bits inverted for negatives), INF = key(+inf).
// A backup d = g(x,u) + max_{y in F(x,u)} W(y) (Sect. III-C operator P with
// per-pair costs) is INF if either operand is INF.  int32 sums are formed in
// 64 bits: >= INT32_MAX is INF, below -INT32_MAX saturates (and is counted).
// fp32 sums are a single IEEE round-to-nearest-even addition.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gbf {

constexpr int kWave = 64;
constexpr uint32_t kNoList = 0xffffffffu;

// Global address space.  Pointers read from the instance table are generic
// to the compiler, which would otherwise emit flat loads (these wait on both
// the vector-memory and the LDS counters and serialise the memory pipeline).
#define GBF_GLOBAL __attribute__((address_space(1)))
template <class P>
__device__ __forceinline__ GBF_GLOBAL P* gp(P* p) {
    return (GBF_GLOBAL P*)p;
}
template <class P>
__device__ __forceinline__ const GBF_GLOBAL P* gp(const P* p) {
    return (const GBF_GLOBAL P*)p;
}

struct TI32 {
    using key_t = int32_t;
    static constexpr int32_t INF = 0x7fffffff;
    static constexpr int32_t LOWEST = (int32_t)0x80000000;
    __device__ static __forceinline__ int32_t from_raw(int32_t raw) { return raw; }
    __device__ static __forceinline__ bool less(int32_t a, int32_t b) { return a < b; }
    __device__ static __forceinline__ int32_t max2(int32_t a, int32_t b) { return a > b ? a : b; }
    __device__ static __forceinline__ bool backup(int32_t g, int32_t m, int32_t& d, int& sat) {
        if (g == INF || m == INF) return false;
        int64_t s = (int64_t)g + (int64_t)m;
        if (s >= (int64_t)INF) return false;
        if (s < -(int64_t)INF) {
            s = -(int64_t)INF;
            sat = 1;
        }
        d = (int32_t)s;
        return true;
    }
    __device__ static __forceinline__ int32_t amin(GBF_GLOBAL int32_t* p, int32_t v) {
        return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static __forceinline__ int32_t out_word(int32_t k) { return k; }
    // per-edge costs: h + W(y) exactly in int64; INF stays far above every
    // finite sum so that a row max is INF if any W(y) is
    using wide_t = int64_t;
    static constexpr int64_t WINF = (int64_t)1 << 62;
    static constexpr int64_t WLOWEST = -((int64_t)1 << 62);
    __device__ static __forceinline__ int64_t edge(int32_t h, int32_t v) {
        return v == INF ? WINF : (int64_t)h + (int64_t)v;
    }
    __device__ static __forceinline__ int64_t wmax2(int64_t a, int64_t b) { return a > b ? a : b; }
    __device__ static __forceinline__ bool backupw(int32_t g, int64_t m, int32_t& d, int& sat) {
        if (g == INF || m >= WINF) return false;
        int64_t s = (int64_t)g + m;
        if (s >= (int64_t)INF) return false;
        if (s < -(int64_t)INF) {
            s = -(int64_t)INF;
            sat = 1;
        }
        d = (int32_t)s;
        return true;
    }
};

struct TF32 {
    using key_t = uint32_t;
    static constexpr uint32_t INF = 0xff800000u;  // key(+inf)
    static constexpr uint32_t LOWEST = 0u;
    __device__ static __forceinline__ uint32_t key(float f) {
        uint32_t b = __float_as_uint(f);
        if ((b & 0x7fffffffu) == 0) b = 0;  // -0 -> +0
        return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    }
    __device__ static __forceinline__ float unkey(uint32_t k) {
        uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
        return __uint_as_float(b);
    }
    __device__ static __forceinline__ uint32_t from_raw(int32_t raw) { return key(__int_as_float(raw)); }
    __device__ static __forceinline__ bool less(uint32_t a, uint32_t b) { return a < b; }
    __device__ static __forceinline__ uint32_t max2(uint32_t a, uint32_t b) { return a > b ? a : b; }
    __device__ static __forceinline__ bool backup(int32_t graw, uint32_t m, uint32_t& d, int& sat) {
        (void)sat;
        const float g = __int_as_float(graw);
        if (m == INF || g == __builtin_inff()) return false;
        const float s = __fadd_rn(g, unkey(m));
        if (s == __builtin_inff()) return false;
        d = key(s);
        return true;
    }
    __device__ static __forceinline__ uint32_t amin(GBF_GLOBAL uint32_t* p, uint32_t v) {
        return __hip_atomic_fetch_min(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __device__ static __forceinline__ int32_t out_word(uint32_t k) { return __float_as_int(unkey(k)); }
    // per-edge costs: one round-to-nearest-even addition h + W(y), kept as
    // a key (+inf, from W(y) = INF or an overflow, is INF)
    using wide_t = uint32_t;
    static constexpr uint32_t WINF = INF;
    static constexpr uint32_t WLOWEST = LOWEST;
    __device__ static __forceinline__ uint32_t edge(int32_t hraw, uint32_t v) {
        return key(__fadd_rn(__int_as_float(hraw), unkey(v)));
    }
    __device__ static __forceinline__ uint32_t wmax2(uint32_t a, uint32_t b) { return a > b ? a : b; }
    __device__ static __forceinline__ bool backupw(int32_t graw, uint32_t m, uint32_t& d, int& sat) {
        return backup(graw, m, d, sat);
    }
};

// ---------------------------------------------------------------- wave helpers
__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }

// Compiler fence at wavefront scope: orders this wave's LDS writes before
// later LDS reads by other lanes of the same wave.
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        int t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v) {
#pragma unroll
    for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

}  // namespace gbf
