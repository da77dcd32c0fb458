// The aircraft abstraction on the device: F'(Omega, u) and its predecessors
// computed from the ODE instead of stored per pair (Sect. V-B: discrete
// abstractions of sampled systems, with attainable sets over-approximated by
// hyper-rectangles and pred replaced by a superset; Sect. VI-A: the
// point-mass aircraft x1' = x4 cos x3, x2' = x4 sin x3,
// x3' = p_L x4 sin(u2) / m, x4' = (u1 - p_D x4^2) / m).
//
// Enclosures: the first-order interval Taylor method (R. E. Moore, Interval
// Analysis, 1966) in double precision.  Every interval operation rounds to
// nearest and moves each bound one unit in the last place outward; a step
// of length h from the box X first finds a box E with X + [0,h] f(E) inside
// E (every solution then stays in B = X + [0,h] f(E) over the step) and
// ends in (X + h f(B)) intersected with B.  sin and cos of an interval come
// from the values at its ends, widened by an error bound of the evaluation,
// and the extrema it contains.  The dynamics do not depend on x1 and x2, so
// the enclosure of a cell is that of the cell moved to the origin in
// (x1, x2), shifted back by whole cells: one table entry per (heading cell,
// speed cell, input) serves every position.  At the paper's grid that is
// 354,375 entries (2.8 MB) in place of about 5 G stored images.
//
// The solver kernels walk the entry's box (the heading wraps) for the
// maximum of W, and find predecessors from reverse rows of the table:
// (x, u) has y in F(x, u) exactly when the entry of (x's heading and speed
// cells, u) holds y's heading and speed cells and x1, x2 lie in the window
// its offsets give.  Pairs whose box leaves the grid on x1, x2 or the speed
// leave the operating range: infinite cost, never evaluated or marked.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "gbf_device.h"
#include "gbf_internal.h"

namespace gbf {
namespace {

// ------------------------------------------------------------ interval maths
struct Iv {
    double lo, hi;
};

// the neighbouring doubles toward -inf and +inf (finite arguments; both
// zeros step to the smallest subnormal)
__device__ __forceinline__ double below(double x) {
    uint64_t b = (uint64_t)__double_as_longlong(x);
    if ((b << 1) == 0) b = 0x8000000000000001ull;
    else if (b >> 63) b += 1;
    else b -= 1;
    return __longlong_as_double((long long)b);
}
__device__ __forceinline__ double above(double x) { return -below(-x); }

__device__ __forceinline__ Iv point(double c) { return Iv{c, c}; }
__device__ __forceinline__ Iv operator+(Iv a, Iv b) { return Iv{below(a.lo + b.lo), above(a.hi + b.hi)}; }
__device__ __forceinline__ Iv operator-(Iv a, Iv b) { return Iv{below(a.lo - b.hi), above(a.hi - b.lo)}; }
__device__ __forceinline__ Iv operator*(Iv a, Iv b) {
    const double p0 = a.lo * b.lo, p1 = a.lo * b.hi, p2 = a.hi * b.lo, p3 = a.hi * b.hi;
    double mn = p0, mx = p0;
    if (p1 < mn) mn = p1;
    if (p1 > mx) mx = p1;
    if (p2 < mn) mn = p2;
    if (p2 > mx) mx = p2;
    if (p3 < mn) mn = p3;
    if (p3 > mx) mx = p3;
    return Iv{below(mn), above(mx)};
}
// by a positive double
__device__ __forceinline__ Iv times(Iv a, double c) { return Iv{below(a.lo * c), above(a.hi * c)}; }
__device__ __forceinline__ Iv over(Iv a, double c) { return Iv{below(a.lo / c), above(a.hi / c)}; }
__device__ __forceinline__ Iv square(Iv a) {
    if (a.lo >= 0) return Iv{below(a.lo * a.lo), above(a.hi * a.hi)};
    if (a.hi <= 0) return Iv{below(a.hi * a.hi), above(a.lo * a.lo)};
    const double s = a.lo * a.lo, t = a.hi * a.hi;
    return Iv{0.0, above(s > t ? s : t)};
}
// [0, h] a for h > 0
__device__ __forceinline__ Iv sweep(Iv a, double h) {
    const double l = below(a.lo * h), u = above(a.hi * h);
    return Iv{l < 0 ? l : 0.0, u > 0 ? u : 0.0};
}

// sin / cos of a double: x = k pi/2 + r with pi/2 as a 33-bit head (exact
// products k * head) plus the double nearest the rest, then the Taylor
// polynomials in r to degree 17 (sin) and 18 (cos) in Horner form.  Their
// error over |x| < 16 stays far below kTrigErr.
constexpr double kPio2Head = 1.5707963267341256;   // 0x3ff921fb54400000
constexpr double kPio2Tail = 6.077100506506192e-11;  // 0x3dd0b4611a626331
constexpr double kTwoOverPi = 0.6366197723675814;
constexpr double kPiBelow = 3.141592653589793;  // the double just below pi
constexpr double kTrigErr = 1e-14;

__device__ __forceinline__ double sin_poly(double r) {
    const double z = r * r;
    double p = 1.0 / 355687428096000.0;
    p = -1.0 / 1307674368000.0 + z * p;
    p = 1.0 / 6227020800.0 + z * p;
    p = -1.0 / 39916800.0 + z * p;
    p = 1.0 / 362880.0 + z * p;
    p = -1.0 / 5040.0 + z * p;
    p = 1.0 / 120.0 + z * p;
    p = -1.0 / 6.0 + z * p;
    return r + r * (z * p);
}
__device__ __forceinline__ double cos_poly(double r) {
    const double z = r * r;
    double p = 1.0 / 6402373705728000.0;
    p = -1.0 / 20922789888000.0 + z * p;
    p = 1.0 / 87178291200.0 + z * p;
    p = -1.0 / 479001600.0 + z * p;
    p = 1.0 / 3628800.0 + z * p;
    p = -1.0 / 40320.0 + z * p;
    p = 1.0 / 720.0 + z * p;
    p = -1.0 / 24.0 + z * p;
    p = 0.5 + z * p;
    return 1.0 - z * p;
}
// shift 0: sin, 1: cos
__device__ __forceinline__ double trig(double x, int shift) {
    const double k = floor(x * kTwoOverPi + 0.5);
    const double r = (x - k * kPio2Head) - k * kPio2Tail;
    const int quad = (int)(((long long)k + shift) & 3);
    const double v = (quad & 1) ? cos_poly(r) : sin_poly(r);
    return quad >= 2 ? -v : v;
}
// [a, b] holds c + 2 pi j for an integer j (with a margin of 1e-9)
__device__ __forceinline__ bool holds(double a, double b, double c) {
    const double turn = 2.0 * kPiBelow;
    const double j0 = floor((a - c) / turn) - 1.0;
    for (int t = 0; t < 4; ++t) {
        const double p = c + (j0 + t) * turn;
        if (p >= a - 1e-9 && p <= b + 1e-9) return true;
    }
    return false;
}
__device__ __forceinline__ Iv trig(Iv a, int shift) {
    if (!(a.hi - a.lo < 3.0)) return Iv{-1.0, 1.0};
    const double fa = trig(a.lo, shift), fb = trig(a.hi, shift);
    const double mn = fa < fb ? fa : fb, mx = fa < fb ? fb : fa;
    Iv r{below(mn - kTrigErr), above(mx + kTrigErr)};
    const double top = shift == 0 ? 0.5 * kPiBelow : 0.0;  // a maximum; the minima lie half a turn away
    if (holds(a.lo, a.hi, top)) r.hi = 1.0;
    if (holds(a.lo, a.hi, top - kPiBelow)) r.lo = -1.0;
    if (r.hi > 1.0) r.hi = 1.0;
    if (r.lo < -1.0) r.lo = -1.0;
    return r;
}

struct Input {
    double u1;  // thrust
    Iv k3;      // p_L sin(u2) / m
    double mass, p_D;
};

__device__ __forceinline__ void field(const Iv* x, const Input& in, Iv* f) {
    const Iv c = trig(x[2], 1), s = trig(x[2], 0);
    f[0] = x[3] * c;
    f[1] = x[3] * s;
    f[2] = x[3] * in.k3;
    f[3] = over(point(in.u1) - times(square(x[3]), in.p_D), in.mass);
}

// One step of length h; false if no a priori enclosure was found.
__device__ bool step(Iv* X, const Input& in, double h) {
    Iv f[4], E[4], C[4], B[4];
    field(X, in, f);
    for (int a = 0; a < 4; ++a) E[a] = X[a] + sweep(f[a], h);
    for (int it = 0; it < 12; ++it) {
        for (int a = 0; a < 4; ++a) {
            const double d = (E[a].hi - E[a].lo) * 0.125 + 1e-10;
            C[a] = Iv{E[a].lo - d, E[a].hi + d};
        }
        field(C, in, f);
        bool inside = true;
        for (int a = 0; a < 4; ++a) {
            B[a] = X[a] + sweep(f[a], h);
            if (B[a].lo < C[a].lo || B[a].hi > C[a].hi) inside = false;
        }
        if (inside) {
            field(B, in, f);
            for (int a = 0; a < 4; ++a) {
                const Iv y = X[a] + times(f[a], h);
                X[a].lo = y.lo > B[a].lo ? y.lo : B[a].lo;
                X[a].hi = y.hi < B[a].hi ? y.hi : B[a].hi;
            }
            return true;
        }
        for (int a = 0; a < 4; ++a) E[a] = B[a];
    }
    return false;
}

// cells [j eta, (j+1) eta] meeting [ylo, yhi] (eta > 0 an interval)
__device__ __forceinline__ void cells(double ylo, double yhi, Iv eta, int& jlo, int& jhi) {
    const double q = ylo >= 0 ? below(ylo / eta.hi) : below(ylo / eta.lo);
    const double p = yhi >= 0 ? above(yhi / eta.lo) : above(yhi / eta.hi);
    jlo = (int)ceil(below(q - 1.0));
    jhi = (int)floor(p);
}

// input u = a * n_bank + b: thrust a * thrust_max / (n_thrust - 1), bank
// angle ((2 b - (n_bank - 1)) * bank_max / (n_bank - 1)) degrees
__device__ __forceinline__ double thrust_of(const AcSpec& S, int a) {
    return S.n_thrust == 1 ? 0.0 : (double)a * S.thrust_max / (double)(S.n_thrust - 1);
}
__device__ __forceinline__ double bank_of(const AcSpec& S, int b) {
    if (S.n_bank == 1) return 0.0;
    double t = (double)(2 * b - (S.n_bank - 1)) * S.bank_max_deg;
    t = t / (double)(S.n_bank - 1);
    return t * (kPiBelow / 180.0);
}

__global__ __launch_bounds__(128) void k_ac_table(AcSpec S, int32_t* full, uint2* packed,
                                                  unsigned long long* bad) {
    const int N3 = S.dims[2], N4 = S.dims[3], K = S.n_thrust * S.n_bank;
    const int64_t total = (int64_t)N3 * N4 * K;
    const Iv pi{kPiBelow, above(kPiBelow)};
    const Iv eta1 = over(point((double)S.x_max[0]), (double)S.dims[0]);
    const Iv eta2 = over(point((double)S.x_max[1]), (double)S.dims[1]);
    const Iv eta3 = over(times(pi, 2.0), (double)N3);
    const Iv eta4 = over(point((double)(S.v_range[1] - S.v_range[0])), (double)N4);
    const Iv lo3{-pi.hi, -pi.lo};
    const double v0 = (double)S.v_range[0];
    const double h = S.tau / (double)S.steps;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const int u = (int)(e % K);
        const int i3 = (int)((e / K) % N3), i4 = (int)(e / K / N3);
        Input in;
        in.u1 = thrust_of(S, u / S.n_bank);
        in.mass = S.mass;
        in.p_D = S.p_D;
        const double s2 = trig(bank_of(S, u % S.n_bank), 0);
        in.k3 = over(Iv{below(s2 - kTrigErr), above(s2 + kTrigErr)} * point(S.p_L), S.mass);
        Iv X[4];
        X[0] = Iv{0.0, eta1.hi};
        X[1] = Iv{0.0, eta2.hi};
        X[2] = Iv{(lo3 + times(eta3, (double)i3)).lo, (lo3 + times(eta3, (double)(i3 + 1))).hi};
        X[3] = Iv{(point(v0) + times(eta4, (double)i4)).lo, (point(v0) + times(eta4, (double)(i4 + 1))).hi};
        bool ok = true;
        for (int t = 0; t < S.steps && ok; ++t) ok = step(X, in, h);
        int r[8];
        if (ok) {
            cells(X[0].lo, X[0].hi, eta1, r[0], r[1]);
            cells(X[1].lo, X[1].hi, eta2, r[2], r[3]);
            cells(below(X[2].lo - lo3.hi), above(X[2].hi - lo3.lo), eta3, r[4], r[5]);
            cells(below(X[3].lo - v0), above(X[3].hi - v0), eta4, r[6], r[7]);
        } else {
            atomicAdd(bad, 1ull);
            for (int t = 0; t < 8; t += 2) r[t] = 1, r[t + 1] = 0;
        }
        if (full)
            for (int t = 0; t < 8; ++t) full[e * 8 + t] = r[t];
        if (packed) {
            bool fits = true;
            for (int t = 0; t < 4; ++t) fits &= r[t] >= -128 && r[t] <= 127;
            int n3 = r[5] - r[4] + 1;
            if (n3 > N3) n3 = N3;
            const bool live = ok && r[0] <= r[1] && r[2] <= r[3] && n3 > 0 && r[6] >= 0 && r[7] < N4 && r[6] <= r[7];
            if (!fits) atomicAdd(bad + 1, 1ull);
            const int j3 = ((r[4] % N3) + N3) % N3;
            uint2 w;
            w.x = (uint32_t)(r[0] & 0xff) | (uint32_t)(r[1] & 0xff) << 8 | (uint32_t)(r[2] & 0xff) << 16 |
                  (uint32_t)(r[3] & 0xff) << 24;
            w.y = live && fits ? (uint32_t)j3 | (uint32_t)n3 << 8 | (uint32_t)r[6] << 16 | (uint32_t)r[7] << 24 : 0u;
            packed[e] = w;
        }
    }
}

// ------------------------------------------------------------ cell sets
// Cell i of an axis [A, B] split into N is [A + i (B-A)/N, A + (i+1) (B-A)/N];
// against [lo, hi] with integer bounds both tests are exact in integers.
__device__ __forceinline__ bool axis_inside(int64_t A, int64_t B, int64_t N, int64_t i, int64_t lo, int64_t hi) {
    return N * (lo - A) <= i * (B - A) && (i + 1) * (B - A) <= N * (hi - A);
}
__device__ __forceinline__ bool axis_meets(int64_t A, int64_t B, int64_t N, int64_t i, int64_t lo, int64_t hi) {
    return i * (B - A) <= N * (hi - A) && (i + 1) * (B - A) >= N * (lo - A);
}

__global__ __launch_bounds__(256) void k_ac_sets(AcSpec S, AcSets sets, const float* G_in, int32_t* G, uint8_t* avoid,
                                                uint8_t* reward) {
    const int64_t n = (int64_t)S.dims[0] * S.dims[1] * S.dims[2] * S.dims[3];
    const int64_t A[4] = {0, 0, -180, S.v_range[0]};
    const int64_t B[4] = {S.x_max[0], S.x_max[1], 180, S.v_range[1]};
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x) {
        int64_t c[4], r = x;
        for (int a = 0; a < 4; ++a) {
            c[a] = r % S.dims[a];
            r /= S.dims[a];
        }
        bool in_set[3] = {false, false, false};
        for (int k = 0; k < 3; ++k)
            for (int b = 0; b < sets.count[k]; ++b) {
                const int32_t* bx = sets.box[k][b];
                bool all = true;
                for (int a = 0; a < 4; ++a)
                    all &= k == 1 ? axis_meets(A[a], B[a], S.dims[a], c[a], bx[a], bx[4 + a])
                                  : axis_inside(A[a], B[a], S.dims[a], c[a], bx[a], bx[4 + a]);
                in_set[k] |= all;
            }
        G[x] = G_in ? __float_as_int(G_in[x]) : (in_set[0] ? 0 : 0x7f800000);
        avoid[x] = in_set[1] ? 1 : 0;
        if (reward) reward[x] = in_set[2] ? 1 : 0;
    }
}

// ------------------------------------------------------------ reverse rows
struct Entry {
    int o1lo, o1hi, o2lo, o2hi, j3, n3, j4lo, j4hi;
};
__device__ __forceinline__ Entry unpack(uint2 w) {
    Entry e;
    e.o1lo = (int)(int8_t)(w.x & 0xff);
    e.o1hi = (int)(int8_t)((w.x >> 8) & 0xff);
    e.o2lo = (int)(int8_t)((w.x >> 16) & 0xff);
    e.o2hi = (int)(int8_t)(w.x >> 24);
    e.j3 = (int)(w.y & 0xff);
    e.n3 = (int)((w.y >> 8) & 0xff);
    e.j4lo = (int)((w.y >> 16) & 0xff);
    e.j4hi = (int)(w.y >> 24);
    return e;
}

template <bool FILL>
__global__ __launch_bounds__(256) void k_ac_rev(AcSpec S, const uint2* tab, const uint32_t* rptr, uint32_t* cnt,
                                               uint2* rent) {
    const int N3 = S.dims[2], N4 = S.dims[3], K = S.n_thrust * S.n_bank;
    const int64_t total = (int64_t)N3 * N4 * K;
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        const uint2 w = tab[e];
        const Entry t = unpack(w);
        if (t.n3 == 0) continue;
        const int u = (int)(e % K);
        const int i3 = (int)((e / K) % N3), i4 = (int)(e / K / N3);
        for (int k4 = t.j4lo; k4 <= t.j4hi; ++k4)
            for (int d = 0; d < t.n3; ++d) {
                int k3 = t.j3 + d;
                if (k3 >= N3) k3 -= N3;
                const int64_t row = (int64_t)k4 * N3 + k3;
                if (FILL) {
                    const uint32_t at = rptr[row] + atomicAdd(cnt + row, 1u);
                    rent[at] = uint2{w.x, (uint32_t)i3 | (uint32_t)i4 << 8 | (uint32_t)u << 16};
                } else {
                    atomicAdd(cnt + row + 1, 1u);
                }
            }
    }
}

// scan in place over rows + 1 words (one block; at most 255 * 255 rows)
__global__ __launch_bounds__(1024) void k_ac_scan(uint32_t* p, int64_t n) {
    __shared__ uint32_t s[1024];
    const int64_t per = (n + 1023) / 1024;
    const int64_t a = threadIdx.x * per, b = min(n, a + per);
    uint32_t sum = 0;
    for (int64_t i = a; i < b; ++i) sum += p[i];
    s[threadIdx.x] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = threadIdx.x >= (unsigned)d ? s[threadIdx.x - d] : 0u;
        __syncthreads();
        s[threadIdx.x] += v;
        __syncthreads();
    }
    // inclusive scan: the counts sit one word after their row (p[0] = 0),
    // so p[row] becomes the start of the row
    uint32_t run = threadIdx.x ? s[threadIdx.x - 1] : 0u;
    for (int64_t i = a; i < b; ++i) {
        run += p[i];
        p[i] = run;
    }
}

// Each reverse row sorted by source (speed cell, heading cell, input), one
// thread per row (a row holds a few hundred entries): the entries of one
// predecessor cell's inputs sit side by side, so the lanes that take them
// mark neighbouring bytes x K + u of the frontier map.
__global__ __launch_bounds__(256) void k_ac_sort(const uint32_t* rptr, uint2* rent, int64_t rows) {
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t a = rptr[r], b = rptr[r + 1];
        for (uint32_t i = a + 1; i < b; ++i) {
            const uint2 v = rent[i];
            const uint32_t key = ((v.y >> 8) & 0xffu) << 16 | (v.y & 0xffu) << 8 | (v.y >> 16);
            uint32_t j = i;
            while (j > a) {
                const uint2 w = rent[j - 1];
                const uint32_t kw = ((w.y >> 8) & 0xffu) << 16 | (w.y & 0xffu) << 8 | (w.y >> 16);
                if (kw <= key) break;
                rent[j] = w;
                --j;
            }
            rent[j] = v;
        }
    }
}

// ------------------------------------------------------------ the solver
// Lanes per listed pair: problem 1 (costs per pair) and problem 2 (a
// reward flag per successor as well).  Measured at the paper's grid: 4 and
// 8 (problem 1: 6.1-6.4 s against 7.1-7.4 s with 8; problem 2: 2.25 s
// against 2.39 s with 4).
#ifndef GBF_AC_LANES1
#define GBF_AC_LANES1 4
#endif
#ifndef GBF_AC_LANES2
#define GBF_AC_LANES2 8
#endif
#ifndef GBF_AC_MARK
#define GBF_AC_MARK 4
#endif
// Successor values in flight per lane.  Batches of 2 and 4 were measured
// slower at the paper's grid (10.0 and 11.6 s for problem 1): the faster
// gathers evaluate pairs before their successors' improvements of the same
// round land, and the solve then makes 33-52% more pair evaluations.
#ifndef GBF_AC_GATHER
#define GBF_AC_GATHER 1
#endif
constexpr int kGatherBatch = GBF_AC_GATHER;
constexpr int kMarkBatch = GBF_AC_MARK;  // predecessor marks in flight per lane
constexpr int kSlotWords = 8;  // Run.slots: 8 counters per block, the first 6 used

struct Grid4 {
    int n1, n2, n3, n4;
};
__device__ __forceinline__ Grid4 grid_of(const Inst& I) { return Grid4{I.dims[0], I.dims[1], I.dims[2], I.dims[3]}; }

// The successor cell t (0 <= t < n1 n2 n3 n4) of the box with lower cells
// c1, c2, heading j3 (wrapping), speed j4.
__device__ __forceinline__ uint32_t succ_cell(const Grid4& g, int c1, int c2, const Entry& e, int n1, int n2,
                                              uint32_t t) {
    const int t1 = (int)(t % (uint32_t)n1);
    t /= (uint32_t)n1;
    const int t2 = (int)(t % (uint32_t)n2);
    t /= (uint32_t)n2;
    const int t3 = (int)(t % (uint32_t)e.n3);
    const int t4 = (int)(t / (uint32_t)e.n3);
    int k3 = e.j3 + t3;
    if (k3 >= g.n3) k3 -= g.n3;
    return (uint32_t)(c1 + t1) + (uint32_t)g.n1 * ((uint32_t)(c2 + t2) + (uint32_t)g.n2 * ((uint32_t)k3 + (uint32_t)g.n3 * (uint32_t)(e.j4lo + t4)));
}

// A pair's box, or false if its successors leave the operating range.
__device__ __forceinline__ bool pair_box(const Grid4& g, const AcInst& A, int K, uint32_t x, int u, int& c1, int& c2,
                                         int& n1, int& n2, Entry& e) {
    const int i1 = (int)(x % (uint32_t)g.n1);
    uint32_t r = x / (uint32_t)g.n1;
    const int i2 = (int)(r % (uint32_t)g.n2);
    r /= (uint32_t)g.n2;
    const int i3 = (int)(r % (uint32_t)g.n3);
    const int i4 = (int)(r / (uint32_t)g.n3);
    e = unpack(A.tab[((int64_t)i4 * g.n3 + i3) * K + u]);
    c1 = i1 + e.o1lo;
    c2 = i2 + e.o2lo;
    n1 = e.o1hi - e.o1lo + 1;
    n2 = e.o2hi - e.o2lo + 1;
    return e.n3 > 0 && c1 >= 0 && i1 + e.o1hi < g.n1 && c2 >= 0 && i2 + e.o2hi < g.n2;
}

struct Counts {
    uint32_t pairs = 0, edges = 0, impr = 0, sat = 0, expanded = 0, marks = 0;
};

// Marks every pair (x, u) with y in F(x, u) (whole wave, y wave-uniform).
template <class Id>
__device__ __forceinline__ void expand(const Inst& I, const AcInst& A, const Grid4& g, uint32_t y,
                                       uint8_t* __restrict__ dirty, Counts& c) {
    const int K = I.K;
    const int k1 = (int)(y % (uint32_t)g.n1);
    uint32_t r = y / (uint32_t)g.n1;
    const int k2 = (int)(r % (uint32_t)g.n2);
    r /= (uint32_t)g.n2;
    const int k3 = (int)(r % (uint32_t)g.n3);
    const int k4 = (int)(r / (uint32_t)g.n3);
    const int64_t row = (int64_t)k4 * g.n3 + k3;
    const uint32_t r0 = A.rptr[row], r1 = A.rptr[row + 1];
    if (lane_id() == 0) c.expanded += 1;
    for (uint32_t t0 = r0; t0 < r1; t0 += kWave) {
        const uint32_t t = t0 + (uint32_t)lane_id();
        if (t >= r1) continue;
        const uint2 w = A.rent[t];
        const int o1lo = (int)(int8_t)(w.x & 0xff), o1hi = (int)(int8_t)((w.x >> 8) & 0xff);
        const int o2lo = (int)(int8_t)((w.x >> 16) & 0xff), o2hi = (int)(int8_t)(w.x >> 24);
        const int i3 = (int)(w.y & 0xff), i4 = (int)((w.y >> 8) & 0xff), u = (int)(w.y >> 16);
        // x1 with k1 in [x1 + o1lo, x1 + o1hi] whose box stays in the grid
        const int a1 = max(max(k1 - o1hi, -o1lo), 0), b1 = min(min(k1 - o1lo, g.n1 - 1 - o1hi), g.n1 - 1);
        const int a2 = max(max(k2 - o2hi, -o2lo), 0), b2 = min(min(k2 - o2lo, g.n2 - 1 - o2hi), g.n2 - 1);
        const uint32_t hi = (uint32_t)g.n1 * (uint32_t)g.n2 * ((uint32_t)i3 + (uint32_t)g.n3 * (uint32_t)i4);
        const int w1 = b1 - a1 + 1, w2 = b2 - a2 + 1;
        const int cnt = (w1 > 0 && w2 > 0) ? w1 * w2 : 0;
        c.marks += (uint32_t)cnt;
        // kMarkBatch window cells at a time: every byte load issues before
        // the first wait (positions past the window repeat its last cell)
        for (int w0 = 0; w0 < cnt; w0 += kMarkBatch) {
            Id q[kMarkBatch];
            uint8_t v[kMarkBatch];
#pragma unroll
            for (int k = 0; k < kMarkBatch; ++k) {
                const int w = min(w0 + k, cnt - 1);
                const int x2 = a2 + w / w1, x1 = a1 + w - (w / w1) * w1;
                q[k] = (Id)((uint32_t)x1 + (uint32_t)g.n1 * (uint32_t)x2 + hi) * (Id)K + (Id)u;
            }
#pragma unroll
            for (int k = 0; k < kMarkBatch; ++k) v[k] = gp(dirty)[q[k]];
#pragma unroll
            for (int k = 0; k < kMarkBatch; ++k)
                if (w0 + k < cnt && v[k] == 0) gp(dirty)[q[k]] = 1;
        }
    }
}

__device__ __forceinline__ void flush(Counts& c, unsigned long long* s_c, unsigned long long* slots) {
    const uint32_t v[6] = {c.pairs, c.edges, c.impr, c.sat, c.expanded, c.marks};
    for (int k = 0; k < 6; ++k) {
        const unsigned long long t = wave_sum64((unsigned long long)v[k]);
        if (lane_id() == 0 && t) atomicAdd(s_c + k, t);
    }
    __syncthreads();
    if (threadIdx.x < 6 && s_c[threadIdx.x]) slots[blockIdx.x * kSlotWords + threadIdx.x] += s_c[threadIdx.x];
}

// One round: every listed pair is evaluated by kLanes lanes, which split its
// box; the group's first lane forms the backup, updates W(x) and flags x as
// improved for the round's expansion (k_ac_expand).
template <class T, bool WIDE, bool STAGE2>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(8)))
void k_ac_relax(const Inst* __restrict__ It, Run R, int round) {
    using Id = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
    using Key = typename T::key_t;
    const Id count = WIDE ? (Id)R.counts64[round] : (Id)R.counts[round];
    if (count == 0) return;
    const Inst& I = It[0];
    if (round >= I.max_rounds) {
        // the round cap is reached with work left (Algorithm 1's second
        // loop condition): nothing is evaluated, the instance is flagged
        if (blockIdx.x == 0 && threadIdx.x == 0) R.inst_status[0] = 1;
        return;
    }
    __shared__ unsigned long long s_c[6];
    if (threadIdx.x < 6) s_c[threadIdx.x] = 0;
    __syncthreads();
    const AcInst A = *I.ac;
    const Grid4 g = grid_of(I);
    const int K = I.K;
    Key* V = static_cast<Key*>(I.V);
    const Id* list = WIDE ? (const Id*)R.list64 : (const Id*)R.list;
    constexpr int kLanes = STAGE2 ? GBF_AC_LANES2 : GBF_AC_LANES1;
    const int lane = lane_id(), sub = lane & (kLanes - 1);
    Counts c;
    const Id waves = (Id)gridDim.x * (blockDim.x / kWave);
    for (Id first = ((Id)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave) * (kWave / kLanes); first < count;
         first += waves * (kWave / kLanes)) {
        const Id i = first + (Id)(lane / kLanes);
        bool live = i < count;
        const Id q = live ? list[i] : (Id)0;
        const uint32_t x = (uint32_t)(q / (Id)K);
        const int u = (int)(q - (Id)x * (Id)K);
        int c1 = 0, c2 = 0, n1 = 1, n2 = 1;
        Entry e{};
        if (live) live = !I.avoid[x] && pair_box(g, A, K, x, u, c1, c2, n1, n2, e);
        const uint32_t vol = live ? (uint32_t)(n1 * n2 * e.n3 * (e.j4hi - e.j4lo + 1)) : 0u;
        const int32_t gu = live ? A.gu[u] : 0;
        Key m = (Key)T::LOWEST;
        typename T::wide_t mw = T::WLOWEST;
        // kGatherBatch cells per lane at a time, all their loads issued
        // before the first wait (positions past the box repeat its last
        // cell, which leaves the maximum unchanged)
        for (uint32_t t0 = (uint32_t)sub; t0 < vol; t0 += kLanes * kGatherBatch) {
            uint32_t y[kGatherBatch];
#pragma unroll
            for (int k = 0; k < kGatherBatch; ++k)
                y[k] = succ_cell(g, c1, c2, e, n1, n2, min(t0 + (uint32_t)(k * kLanes), vol - 1u));
            Key vy[kGatherBatch];
#pragma unroll
            for (int k = 0; k < kGatherBatch; ++k) vy[k] = gp(V)[y[k]];
            if (STAGE2) {
                uint8_t rw[kGatherBatch];
#pragma unroll
                for (int k = 0; k < kGatherBatch; ++k) rw[k] = gp(A.reward)[y[k]];
#pragma unroll
                for (int k = 0; k < kGatherBatch; ++k) mw = T::wmax2(mw, T::edge(rw[k] ? A.rc : gu, vy[k]));
            } else {
#pragma unroll
                for (int k = 0; k < kGatherBatch; ++k) m = T::max2(m, vy[k]);
            }
        }
#pragma unroll
        for (int d = 1; d < kLanes; d <<= 1) {
            if (STAGE2) mw = T::wmax2(mw, __shfl_xor(mw, d, kWave));
            else m = T::max2(m, __shfl_xor(m, d, kWave));
        }
        bool improved = false;
        if (live && sub == 0) {
            c.pairs += 1;
            c.edges += vol;
            Key d;
            int sat = 0;
            const bool ok = STAGE2 ? T::backupw(0, mw, d, sat) : T::backup(gu, m, d, sat);
            c.sat += sat;
            if (ok && T::less(d, V[x])) {
                const Key old = T::amin(gp(V) + x, d);
                improved = T::less(d, old);
                c.impr += improved;
            }
        }
        // the expansion waits for the end of the round (k_ac_expand): marks
        // only feed the next round, so one expansion per improved state and
        // round gives the same next frontier as one per improvement
        if (improved) gp(A.imp)[x] = 1;
    }
    flush(c, s_c, R.slots);
}

// The round's improved states, each expanded once by a whole wave; the
// flags are cleared for the next round.  Lanes read 16 flags at a time.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_ac_expand(const Inst* __restrict__ It, Run R, int round) {
    using Id = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
    const Id count = WIDE ? (Id)R.counts64[round] : (Id)R.counts[round];
    if (count == 0) return;
    __shared__ unsigned long long s_c[6];
    if (threadIdx.x < 6) s_c[threadIdx.x] = 0;
    __syncthreads();
    const Inst& I = It[0];
    const AcInst A = *I.ac;
    const Grid4 g = grid_of(I);
    uint8_t* next = R.dirty[(round + 1) & 1];
    Counts c;
    const int64_t nchunk = (I.n + 15) / 16;
    const int64_t nw = (nchunk + kWave - 1) / kWave;
    for (int64_t w = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; w < nw;
         w += (int64_t)gridDim.x * (blockDim.x / kWave)) {
        const int64_t ch = w * kWave + lane_id();
        uint4 f = make_uint4(0u, 0u, 0u, 0u);
        uint4* flags = reinterpret_cast<uint4*>(A.imp);
        if (ch < nchunk) f = flags[ch];
        const bool any = (f.x | f.y | f.z | f.w) != 0u;
        if (!__ballot(any)) continue;
        if (any) flags[ch] = make_uint4(0u, 0u, 0u, 0u);
        const uint32_t word[4] = {f.x, f.y, f.z, f.w};
        for (int b = 0; b < 16; ++b) {
            unsigned long long bal = __ballot(((word[b >> 2] >> (8 * (b & 3))) & 0xffu) != 0u);
            while (bal) {
                const int l = __ffsll((long long)bal) - 1;
                bal &= bal - 1;
                expand<Id>(I, A, g, (uint32_t)((w * kWave + l) * 16 + b), next, c);
            }
        }
    }
    flush(c, s_c, R.slots);
}

// Algorithm 1's start: F1 = the predecessors of every state with G < inf.
template <bool WIDE>
__global__ __launch_bounds__(256) void k_ac_seed(const Inst* __restrict__ It, Run R) {
    using Id = typename std::conditional<WIDE, uint64_t, uint32_t>::type;
    __shared__ unsigned long long s_c[6];
    if (threadIdx.x < 6) s_c[threadIdx.x] = 0;
    __syncthreads();
    const Inst& I = It[0];
    const AcInst A = *I.ac;
    const Grid4 g = grid_of(I);
    Counts c;
    const int64_t nw = (I.n + kWave - 1) / kWave;
    for (int64_t w = blockIdx.x * (int64_t)(blockDim.x / kWave) + threadIdx.x / kWave; w < nw;
         w += (int64_t)gridDim.x * (blockDim.x / kWave)) {
        const int64_t y = w * kWave + lane_id();
        const bool act = y < I.n && TF32::from_raw(I.G[y]) != TF32::INF && !I.avoid[y];
        unsigned long long bal = __ballot(act);
        while (bal) {
            const int l = __ffsll((long long)bal) - 1;
            bal &= bal - 1;
            expand<Id>(I, A, g, (uint32_t)(w * kWave + l), R.dirty[0], c);
        }
    }
    c.expanded = 0;  // seeding is not an expansion of an improved state
    c.marks = 0;
    flush(c, s_c, R.slots);
}

// The canonical policy (smallest input attaining the minimum) and a count of
// states whose backup differs from V, one thread per state.
template <class T, bool STAGE2>
__global__ __launch_bounds__(256) void k_ac_policy(Inst I, int32_t* pol, unsigned long long* bad) {
    using Key = typename T::key_t;
    const Key* V = static_cast<const Key*>(I.V);
    const AcInst A = *I.ac;
    const Grid4 g = grid_of(I);
    unsigned long long nb = 0;
    for (int64_t xi = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; xi < I.n;
         xi += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t x = (uint32_t)xi;
        const Key vx = V[x];
        if (I.avoid[x]) {
            pol[x] = -2;
            nb += vx != T::INF;
            continue;
        }
        Key best = T::from_raw(I.G[x]);
        int pu = -1;
        for (int u = 0; u < I.K; ++u) {
            int c1, c2, n1, n2;
            Entry e;
            if (!pair_box(g, A, I.K, x, u, c1, c2, n1, n2, e)) continue;
            const uint32_t vol = (uint32_t)(n1 * n2 * e.n3 * (e.j4hi - e.j4lo + 1));
            Key m = (Key)T::LOWEST;
            typename T::wide_t mw = T::WLOWEST;
            for (uint32_t t = 0; t < vol; ++t) {
                const uint32_t y = succ_cell(g, c1, c2, e, n1, n2, t);
                if (STAGE2) mw = T::wmax2(mw, T::edge(A.reward[y] ? A.rc : A.gu[u], V[y]));
                else m = T::max2(m, V[y]);
            }
            Key d;
            int sat = 0;
            const bool ok = STAGE2 ? T::backupw(0, mw, d, sat) : T::backup(A.gu[u], m, d, sat);
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

int blocks_for(int64_t n, int block, int cap) {
    const int64_t b = (n + block - 1) / block;
    return (int)std::max<int64_t>(1, std::min<int64_t>(b, cap));
}

}  // namespace

hipError_t launch_ac_table(const AcSpec& S, int32_t* full, uint2* packed, unsigned long long* bad, hipStream_t s) {
    const int64_t total = (int64_t)S.dims[2] * S.dims[3] * S.n_thrust * S.n_bank;
    k_ac_table<<<blocks_for(total, 128, 8192), 128, 0, s>>>(S, full, packed, bad);
    return hipGetLastError();
}

hipError_t launch_ac_sets(const AcSpec& S, const AcSets& sets, const float* G_in, int32_t* G, uint8_t* avoid,
                          uint8_t* reward, hipStream_t s) {
    const int64_t n = (int64_t)S.dims[0] * S.dims[1] * S.dims[2] * S.dims[3];
    k_ac_sets<<<blocks_for(n, 256, 8192), 256, 0, s>>>(S, sets, G_in, G, avoid, reward);
    return hipGetLastError();
}

hipError_t launch_ac_rev_count(const AcSpec& S, const uint2* tab, uint32_t* rptr, hipStream_t s) {
    const int64_t total = (int64_t)S.dims[2] * S.dims[3] * S.n_thrust * S.n_bank;
    k_ac_rev<false><<<blocks_for(total, 256, 4096), 256, 0, s>>>(S, tab, nullptr, rptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_ac_rev_fill(const AcSpec& S, const uint2* tab, const uint32_t* rptr, uint32_t* cursor,
                              uint2* rent, hipStream_t s) {
    const int64_t total = (int64_t)S.dims[2] * S.dims[3] * S.n_thrust * S.n_bank;
    k_ac_rev<true><<<blocks_for(total, 256, 4096), 256, 0, s>>>(S, tab, rptr, cursor, rent);
    return hipGetLastError();
}

hipError_t launch_ac_scan(uint32_t* rptr, int64_t rows, hipStream_t s) {
    k_ac_scan<<<1, 1024, 0, s>>>(rptr, rows + 1);
    return hipGetLastError();
}

hipError_t launch_ac_sort(const uint32_t* rptr, uint2* rent, int64_t rows, hipStream_t s) {
    k_ac_sort<<<blocks_for(rows, 256, 4096), 256, 0, s>>>(rptr, rent, rows);
    return hipGetLastError();
}

hipError_t launch_ac_relax(const Inst* dI, const Run& R, int round, int grid, hipStream_t s, bool wide, int stage) {
    const bool stage2 = stage == 2;
    const int nb = std::max(1, std::min(grid > 0 ? grid : 2048, kMaxGrid));
    if (wide) {
        if (stage2) k_ac_relax<TF32, true, true><<<nb, 256, 0, s>>>(dI, R, round);
        else k_ac_relax<TF32, true, false><<<nb, 256, 0, s>>>(dI, R, round);
    } else {
        if (stage2) k_ac_relax<TF32, false, true><<<nb, 256, 0, s>>>(dI, R, round);
        else k_ac_relax<TF32, false, false><<<nb, 256, 0, s>>>(dI, R, round);
    }
    return hipGetLastError();
}

hipError_t launch_ac_expand(const Inst* dI, const Run& R, int round, int64_t n, hipStream_t s, bool wide) {
    const int nb = blocks_for(((n + 15) / 16 + kWave - 1) / kWave, 4, 4096);
    if (wide) k_ac_expand<true><<<nb, 256, 0, s>>>(dI, R, round);
    else k_ac_expand<false><<<nb, 256, 0, s>>>(dI, R, round);
    return hipGetLastError();
}

hipError_t launch_ac_seed(const Inst* dI, const Run& R, int64_t n, hipStream_t s, bool wide) {
    const int nb = blocks_for((n + kWave - 1) / kWave, 4, 4096);
    if (wide) k_ac_seed<true><<<nb, 256, 0, s>>>(dI, R);
    else k_ac_seed<false><<<nb, 256, 0, s>>>(dI, R);
    return hipGetLastError();
}

hipError_t launch_ac_policy(const Inst& I, int32_t* pol, unsigned long long* bad, hipStream_t s) {
    if (I.ac_stage == 2) k_ac_policy<TF32, true><<<blocks_for(I.n, 256, 8192), 256, 0, s>>>(I, pol, bad);
    else k_ac_policy<TF32, false><<<blocks_for(I.n, 256, 8192), 256, 0, s>>>(I, pol, bad);
    return hipGetLastError();
}

}  // namespace gbf
