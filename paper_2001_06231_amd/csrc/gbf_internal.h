// Internal interface between the host driver (gbf_api.hip) and the kernels
// (gbf_kernels.hip).  Not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace gbf {

struct AcInst;

// One problem instance as the kernels see it.  Pair ids are global: pair p
// of this instance has id pair_base + p, state x is instance-local.
struct Inst {
    const uint32_t* sptr;   // CSR row pointers [nK+1]
    const int32_t* sidx;    // CSR successors [m]
    const uint32_t* rptr;   // reverse CSR row pointers [n+1]
    const uint32_t* rev;    // reverse CSR: local pair ids whose box/row holds the state
    const uint64_t* box;    // BOX encoding [nK]
    const int32_t* G;       // terminal cost bits [n]
    const int32_t* g;       // running cost bits [nK] (pruned pairs = INF)
    const int32_t* ge;      // CSR only: per-edge cost bits [m] (succ_idx order), or NULL
    const uint8_t* avoid;   // [n]
    void* V;                // value words [n] (int32 or fp32 key)
    const int32_t* win;     // BOX: per input 8 ints: min (lo-x) per axis, max (hi-x) per axis
    const uint64_t* rptr64; // 64-bit pair ids: reverse CSR row pointers [n+1]
    const int32_t* rrel;    // 64-bit pair ids: reverse CSR entries, pair id minus y*K of row y
    const uint16_t* key;    // bucket order: bucket key of each state [n], else NULL
    uint8_t* occ;           // bucket order: occupancy flag per bucket [65536]
    int64_t n;
    int64_t pair_base;      // first global pair id
    int64_t max_rounds;     // round cap of this instance
    int32_t K;
    int32_t enc;            // 0 CSR, 1 BOX, 2 HYB (box successors, reverse CSR)
    int32_t dims[4];
    int32_t strides[4];
    int32_t index;          // position in the batch
    int32_t dtype;          // 0 int32, 1 fp32
    int32_t wide;           // 1 = 64-bit pair ids (Run.list64 / counts64; HYB: rptr64 / rrel)
    const AcInst* ac;       // enc 3 (aircraft abstraction): its tables (device), else NULL
    int32_t ac_stage;       // enc 3: 1 = costs per pair, 2 = per transition (reward cells)
};

// The aircraft abstraction (enc 3): F(x,u) and pred come from a table of
// enclosures per (heading cell, speed cell, input) instead of per-pair
// images; positions shift the table's boxes by whole cells.
//   tab[(i4 * N3 + i3) * K + u], two words:
//     .x = o1lo | o1hi << 8 | o2lo << 16 | o2hi << 24  (int8 cell offsets on x1, x2)
//     .y = j3lo | n3 << 8 | j4lo << 16 | j4hi << 24   (uint8: first heading
//          cell, mod N3, and the number of heading cells; speed cells;
//          n3 = 0: the enclosure leaves the speed range or was not found)
//   reverse rows, key k4 * N3 + k3: the entries whose box holds heading
//   cell k3 and speed cell k4, sorted by (i4, i3, u), as
//     .x = the entry's offsets (as in tab), .y = i3 | i4 << 8 | u << 16.
struct AcInst {
    const uint2* tab;
    const uint32_t* rptr;   // [N4 * N3 + 1]
    const uint2* rent;
    const uint8_t* reward;  // [n] transitions into these cells cost rc (problem 2), or NULL
    const int32_t* gu;      // [K] running cost bits (fp32) per input
    uint8_t* imp;           // [n rounded up to 16] 1 = the state improved in this round (cleared by the expansion)
    int32_t rc;             // reward cost bits (fp32)
    int32_t stage;          // 1: costs per pair gu[u]; 2: per transition (gu[u] or rc)
};

// The numeric part of an aircraft scenario (see gbf_aircraft in gbf.h).
struct AcSpec {
    int32_t dims[4];
    int32_t x_max[2], v_range[2];
    double mass, p_D, p_L, tau;
    int32_t steps, n_thrust, n_bank;
    double thrust_max, bank_max_deg;
};

// Closed boxes with integer bounds per axis (x1, x2 metres, heading
// degrees in [-180, 180], speed m/s): 0 target, 1 avoid, 2 reward.
constexpr int kAcMaxBoxes = 16;
struct AcSets {
    int32_t count[3];
    int32_t box[3][kAcMaxBoxes][8];  // lo[4], hi[4]
};

// Device-side solver state shared by all instances of one solve.
struct Run {
    uint8_t* dirty[2];          // dirty-pair byte maps (frontiers F1 / F2), 1 = pair is dirty
    uint32_t* list;             // compacted frontier (global pair ids)
    uint32_t* counts;           // frontier size per round [max_rounds + 2]
    uint64_t* list64;           // 64-bit pair ids: compacted frontier
    unsigned long long* counts64;  // 64-bit pair ids: frontier size per round
    unsigned long long* ctr;    // [8]: pair evals, edges, improvements, saturations, expansions, marks
    unsigned long long* slots;  // per-block statistics [kMaxGrid * 8]
    int32_t* inst_status;       // per instance: 1 = cap reached with work left
    uint32_t* barrier;          // persistent mode: barrier words (see the grid barriers), kBarrierBytes
    int32_t* error;             // persistent mode: barrier timeout flag
    int32_t* result;            // persistent mode: [0] rounds executed
    uint64_t timeout_ticks;     // persistent mode: bound of one barrier wait (device clock ticks)
    const uint16_t* key;        // bucket order (single instance): state keys [n]
    uint8_t* occ;               // bucket order: occupancy flag per bucket [65536]
    uint32_t* thr;              // bucket order: bucket selected for the current round
    int64_t nchunks;            // 16-byte chunks per byte map
    int64_t total_pairs;
    int64_t max_rounds;         // global cap (max over instances)
    int32_t ninst;
    int32_t dtype;              // 0 int32, 1 fp32
    int32_t keyK;               // bucket order: inputs per state
    int32_t bspan;              // bucket order: buckets per round (>= 1), or -1 = sweeps
};

// Records `msg` as the calling thread's last error (gbf_last_error) and
// returns `code`.
int set_error(int code, const std::string& msg);

constexpr int kMaxBatch = 1024;
constexpr int kBarrierBytes = 4096;  // persistent mode: barrier words (see the grid barriers)
constexpr int kMaxGrid = 8192;  // most blocks of any solver launch
#ifndef GBF_RELAX_BLOCK
#define GBF_RELAX_BLOCK 512  // default threads per block of the host-loop relax kernel (measured: 256 and 1024 3-5% slower)
#endif
constexpr int kRelaxBlock = GBF_RELAX_BLOCK;

// Launch wrappers (all asynchronous on `s`).
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_validate(const Inst& I, const int64_t* sptr64, int64_t m, int dtype, int32_t* err,
                           hipStream_t s);
hipError_t launch_convert_ptr(const int64_t* in, uint32_t* out, int64_t n, hipStream_t s);
hipError_t launch_prune(const Inst& I, int dtype, hipStream_t s);
hipError_t launch_rev_count(const Inst& I, uint32_t* cnt, hipStream_t s);
hipError_t launch_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s);
hipError_t launch_rev_fill(const Inst& I, uint32_t* cursor, uint32_t* rev, hipStream_t s);
hipError_t launch_box_window(const Inst& I, int32_t* win32, hipStream_t s);
hipError_t launch_box_sizes(const Inst& I, uint32_t* sizes, unsigned long long* total, hipStream_t s);
hipError_t launch_box_fill(const Inst& I, const uint32_t* sptr, int32_t* sidx, hipStream_t s);

hipError_t launch_init(const Inst* dI, const Inst& I, int dtype, hipStream_t s);
// `wide`: 64-bit pair ids (one instance, host loop, BOX or HYB encoding):
// the list and counts are R.list64 / R.counts64, the reverse CSR of HYB is
// rptr64 / rrel
hipError_t launch_seed(const Inst* dI, int ninst, const Run& R, int64_t max_states, int dtype, int enc_mask,
                       hipStream_t s, bool wide = false);
hipError_t launch_compact(const Run& R, int round, int grid, hipStream_t s, bool wide = false);
// bucket order: bucket selection + compaction of the selected pairs (one
// byte map, R.dirty[0] == R.dirty[1])
hipError_t launch_bucket_compact(const Run& R, int round, int grid, hipStream_t s);
// `lanes`: lanes per listed pair in the relax step (4, 8, 16 or 32)
hipError_t launch_relax(const Inst* dI, const Run& R, int round, int grid, int lanes, int dtype, int enc_mask,
                        hipStream_t s, bool wide = false, int block = 0);
// `attr_launch`: launch through hipLaunchKernelExC with the cooperative
// attribute (the form that stream capture records as a graph node)
hipError_t launch_persistent(const Inst* dI, const Run& R, int grid, int lanes, int dtype, int enc_mask,
                             bool attr_launch, hipStream_t s);
int persistent_blocks_per_cu(const Run& R, int lanes, int dtype, int enc_mask);
// all rounds of one instance in a single 1024-thread workgroup
hipError_t launch_single(const Inst* dI, const Run& R, int lanes, int dtype, int enc_mask, int64_t n_states,
                         hipStream_t s);
hipError_t launch_sum_slots(const unsigned long long* slots, int nslots, unsigned long long* ctr, hipStream_t s);
hipError_t launch_sort_rows(const uint32_t* rptr, uint32_t* rev, int64_t n, hipStream_t s);
// 64-bit pair ids, HYB: the reverse CSR built straight from the boxes
// (counts per state, a 64-bit scan, relative entries, rows sorted)
hipError_t launch_rev_count_box(const Inst& I, uint32_t* cnt, hipStream_t s);
hipError_t launch_scan64(const uint32_t* in, uint64_t* out, int64_t n, uint64_t* tmp, hipStream_t s);
hipError_t launch_rev_fill_box(const Inst& I, unsigned long long* cursor, int32_t* rel, hipStream_t s);
hipError_t launch_sort_rows64(const uint64_t* rptr, int32_t* rel, int64_t n, hipStream_t s);
hipError_t launch_decode(const Inst& I, int dtype, void* out, hipStream_t s);

// Aircraft abstraction (gbf_aircraft.hip).
// The enclosure table: `full` (or NULL) gets 8 int32 per entry (o1lo, o1hi,
// o2lo, o2hi, j3lo, j3hi unwrapped, j4lo, j4hi), `packed` (or NULL) the
// solver's form; bad[0] counts entries without an a priori enclosure,
// bad[1] entries that do not fit the packed form.
hipError_t launch_ac_table(const AcSpec& S, int32_t* full, uint2* packed, unsigned long long* bad, hipStream_t s);
// G bits (fp32: 0 on target cells, +inf elsewhere; skipped if G_in is
// given, which is copied instead), avoid and reward flags per state.
hipError_t launch_ac_sets(const AcSpec& S, const AcSets& sets, const float* G_in, int32_t* G, uint8_t* avoid,
                          uint8_t* reward, hipStream_t s);
// Reverse rows of the packed table: counts into rptr[1..], scan, fill,
// sort.  `cursor` has N4 * N3 words.
hipError_t launch_ac_rev_count(const AcSpec& S, const uint2* tab, uint32_t* rptr, hipStream_t s);
hipError_t launch_ac_rev_fill(const AcSpec& S, const uint2* tab, const uint32_t* rptr, uint32_t* cursor,
                              uint2* rent, hipStream_t s);
hipError_t launch_ac_scan(uint32_t* rptr, int64_t rows, hipStream_t s);
hipError_t launch_ac_sort(const uint32_t* rptr, uint2* rent, int64_t rows, hipStream_t s);
hipError_t launch_ac_relax(const Inst* dI, const Run& R, int round, int grid, hipStream_t s, bool wide, int stage);
hipError_t launch_ac_seed(const Inst* dI, const Run& R, int64_t n, hipStream_t s, bool wide);
// After a round's relax step: every state flagged as improved is expanded
// once into the next frontier and its flag cleared.
hipError_t launch_ac_expand(const Inst* dI, const Run& R, int round, int64_t n, hipStream_t s, bool wide);
hipError_t launch_ac_policy(const Inst& I, int32_t* pol, unsigned long long* bad, hipStream_t s);
hipError_t launch_policy(const Inst& I, int dtype, int32_t* pol, unsigned long long* bad, hipStream_t s);

}  // namespace gbf
