// Internal interface between the host runtime and the HIP kernels of the
// Lottery BP (+OSD) decoder.  gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace lbp {

// Padded row width of the per-shot edge array: check c owns slots c*DEG .. c*DEG+DEG-1.
constexpr int DEG = 8;
// Column table: up to CDEG edge slots per column packed as u16 into one u64.
constexpr int CDEG = 4;
constexpr uint32_t NOPOS = 0xFFFFu;
// Codes whose slot positions c*DEG+k do not fit 16 bits (m > 8191) keep them as
// four u32 per column instead (all-ones for an unused entry).
constexpr int MAX_M_NARROW = 8191;
constexpr uint32_t NOPOS32 = 0xFFFFFFFFu;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
// Magnitude sent by a degree-1 check (empty minimum) in float modes.
constexpr float CAP_FLOAT = 1024.0f;
// Hard-decision threshold in float modes: e = [lambda <= TAU].
constexpr float TAU_FLOAT = 1.0f / 4096.0f;

enum { MSG_FP32 = 0, MSG_FP16 = 1, MSG_INT8 = 2 };
enum { FLIP_MSG = 0, FLIP_LLR = 1 };
enum { OSD_NONE = 0, OSD_0 = 1, OSD_CS = 2 };
enum { FLAG_CONVERGED = 1, FLAG_OSD = 2, FLAG_OSD_INCONSISTENT = 4 };

struct DevCode {
    int32_t m, n, mw, nw;     // mw = ceil(m/32), nw = ceil(n/32)
    const uint16_t *cn_cols;  // [m*DEG]   column of each slot, NOPOS for padding
    const uint8_t *cn_deg;    // [m]       row weight
    const uint64_t *vn_tab;   // [n]       CDEG x u16 slot positions, ascending check, NOPOS-filled
    const u32x4 *vn_tab4;     // [n]       the same as u32 (NOPOS32-filled) when the code is wide, else null
    const float *mu_f32;      // [n]       prior LLR rounded to fp32
    const float *mu_f16;      // [n]       prior LLR rounded to fp16 (held as float)
    const int32_t *mu_q;      // [n]       Int3.4 prior
    int32_t mu_q_uniform;     // the Int3.4 prior when every column has the same one, else INT32_MIN
    // Eq. 1 structure when H is a space-time matrix [I_r (x) H0 | D (x) I_m0] (0 otherwise):
    // check t*m0 + s touches data columns t*n0 + cols(s) and measurement columns
    // r*n0 + t*m0 + s and, for t >= 1, r*n0 + (t-1)*m0 + s.
    int32_t st_r, st_m0, st_n0;
    const uint32_t *st_tab;   // compact space-time offset table of the Int x.y kernel, or null
};

// Access to a column's slot positions in either table layout: load(C, v)
// returns the column's entry, pos(t, j) its j-th position (j < CDEG, ascending
// check), NONE marks an unused entry.
struct ColTab16 {
    using T = uint64_t;
    static constexpr uint32_t NONE = NOPOS;
    __device__ static T load(const DevCode &C, int v) { return C.vn_tab[v]; }
    __device__ static T empty() { return ~0ull; }
    __device__ static uint32_t pos(T t, int j) { return (uint32_t)(t >> (16 * j)) & 0xFFFFu; }
};
struct ColTab32 {
    using T = u32x4;
    static constexpr uint32_t NONE = NOPOS32;
    __device__ static T load(const DevCode &C, int v) { return C.vn_tab4[v]; }
    __device__ static T empty() { return T{NOPOS32, NOPOS32, NOPOS32, NOPOS32}; }
    __device__ static uint32_t pos(T t, int j) { return t[j]; }
};

// Slot positions of column v in either layout, NOPOS32 for an unused entry
// (for paths where the layout test per column costs nothing that matters).
__device__ inline u32x4 col_positions(const DevCode &C, int v) {
    if (C.vn_tab4) return C.vn_tab4[v];
    const uint64_t t = C.vn_tab[v];
    u32x4 r;
#pragma unroll
    for (int j = 0; j < CDEG; ++j) {
        const uint32_t p = (uint32_t)(t >> (16 * j)) & 0xFFFFu;
        r[j] = p == NOPOS ? NOPOS32 : p;
    }
    return r;
}

struct BpParams {
    int32_t max_iter;
    int32_t scale_mode;  // 0 paper schedule, 1 constant
    float scale_f;       // constant (float modes)
    int32_t scale_k;     // constant k of k/8 (Int3.4)
    int32_t lottery, skip, flip, osd;
    int32_t rule;        // lottery selection rule: CN rule | VN rule << 4
    int32_t qmax;        // fixed point: messages saturate at +-qmax (127 for Int3.4)
    uint64_t seed;
};

// Lottery selection rules (Sec. III-B, Table I).
enum { LOT_CN_RANDOM = 0, LOT_CN_WORST = 1 };
enum { LOT_VN_PROPOSED = 0, LOT_VN_Q_FIRST = 1, LOT_VN_UNRELIABLE = 2, LOT_VN_RANDOM = 3 };

// Candidate order of the neighbour rules: is (cnt, q, v) ahead of (bc, bq, bv)?
// PROPOSED: more checks in U, then smaller Q, then smaller column; Q_FIRST:
// smaller Q, then more checks in U, then column; UNRELIABLE: smaller Q, then column.
template <typename Q>
__device__ __forceinline__ bool lottery_key_less(int vn_rule, int cnt, Q q, int v, int bc, Q bq, int bv) {
    if (vn_rule == LOT_VN_Q_FIRST)
        return q < bq || (q == bq && (cnt > bc || (cnt == bc && v < bv)));
    if (vn_rule == LOT_VN_UNRELIABLE) return q < bq || (q == bq && v < bv);
    return cnt > bc || (cnt == bc && (q < bq || (q == bq && v < bv)));
}

// Serving rings of one code slot.  Host memory is pinned, fine-grained
// (coherent) and read or written by the kernels directly.
struct ServeRing {
    const uint32_t *syn;            // host [R][mw]: syndrome of item k in slot k & mask
    const uint64_t *keys;           // host [R][2]: (lottery seed, shot_id)
    const uint64_t *host_tail;      // host: number of items published
    const uint32_t *host_stop;      // host: nonzero asks idle waves to exit
    uint32_t *corr;                 // host [R][nw]
    uint8_t *flags;                 // host [R]
    int32_t *iters;                 // host [R]
    uint64_t *cq;                   // host [R]: completion queue; position p holds cq_entry(p, item)
    unsigned long long *cq_tail;    // device: next completion-queue position
    unsigned long long *head;       // device: next item to claim
    unsigned long long *tail;       // device: copy of host_tail (raised by the polling wave)
    uint32_t *token;                // device: 1 while a wave polls host memory
    unsigned long long *last_claim; // device: clock of the latest claim by any wave
    uint32_t *exiting;              // device: set by the first wave that finds the ring idle; every wave then exits
    float *llr;                     // device [R][2n]: lambda (hi, lo) of items left to OSD (float kernels)
    int16_t *llr16;                 // device [R][n]: the same buffer as int16 lambda (Int x.y check-centric kernel)
    int64_t mask;                   // R - 1 (R a power of two)
    uint64_t idle_ticks;            // the grid exits after this long without a claim (100 MHz ticks)
    uint32_t claim_max;             // items a wave may claim at once (>= 1)
    uint32_t claim_backlog;         // ... one more per this many items waiting beyond the claim
};
// flags bit of a ring item whose BP failed and whose OSD has not run yet
constexpr uint8_t FLAG_OSD_PENDING = 0x80;

struct BpArgs {
    DevCode code;
    BpParams prm;
    int64_t n_work;             // work items in this launch
    uint64_t first_shot_id;
    const uint64_t *shot_keys;  // nullable: [shots][2] = (lottery seed, shot_id) per shot
    const int32_t *work_list;   // nullable: work item -> shot index
    const uint32_t *synd;       // [shots][mw]
    uint32_t *corr;             // [shots][nw]
    uint8_t *flags;             // [shots]
    int32_t *iters;             // [shots] or null
    float *llr_out;             // [shots][n] or null
    uint32_t *counters;         // [0] next work item, [1] failed shots
    int32_t *fail_list;         // [n_work]
    float *fail_llr;            // [fail_cap][2n]: lambda as hi[n], lo[n] (value = hi + lo) (float kernels)
    int16_t *fail_q;            // [fail_cap][n]: the same buffer as int16 lambda (Int x.y check-centric kernel)
    int64_t fail_cap;
    float *stage;               // [grid waves][2n] (float kernels)
    int32_t wave_bytes;         // LDS bytes of one shot's state
    int32_t group;              // nonzero: a block decodes one shot (bp_kernel), else each wave its own
    const ServeRing *ring;      // device copy; non-null: take items from the ring, not the batch arrays
};

// Claim the next published ring item for the calling lane (call from one lane
// per wave).  Returns -1 when the host asked to stop, or once no wave of the
// grid has claimed anything for idle_ticks.  The grid winds down as a whole:
// the first wave to see the ring idle raises `exiting`, and every wave stops
// claiming once it is raised, so a grid never keeps serving with part of its
// waves gone (the host relaunches a full grid when items wait and the old
// one has drained).  Only the wave holding the token reads host memory; the
// others watch the device copy of the tail.
__device__ inline int64_t serve_claim(const ServeRing &r, uint32_t max_claim, uint32_t *count) {
    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    int idle_rounds = 0;
    for (;;) {
        if (__hip_atomic_load(r.exiting, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) return -1;
        unsigned long long t = __hip_atomic_load(r.tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long h = __hip_atomic_load(r.head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        while (h < t) {
            // every claim is one CAS on the shared head, a device-wide round trip: with a
            // deep backlog a wave takes several items at once (every wave is busy then)
            const unsigned long long waiting = t - h;
            unsigned long long want = 1;  // no division: a handful of scalar compares
            while (want < max_claim && waiting > want * r.claim_backlog) ++want;
            const unsigned long long old = atomicCAS(r.head, h, h + want);
            if (old == h) {
                __hip_atomic_fetch_max(r.last_claim, (unsigned long long)__builtin_amdgcn_s_memrealtime(),
                                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *count = (uint32_t)want;
                return (int64_t)h;
            }
            h = old;
        }
        // test before test-and-set: idle waves mostly read, and only one polls the host
        if (__hip_atomic_load(r.token, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
            atomicCAS(r.token, 0u, 1u) == 0u) {
            const uint64_t ht = __hip_atomic_load(r.host_tail, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
            const uint32_t stop = __hip_atomic_load(r.host_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (ht > t) __hip_atomic_fetch_max(r.tail, (unsigned long long)ht, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            atomicExch(r.token, 0u);
            if (ht > t) continue;
            if (stop) return -1;
        }
        const uint64_t now = __builtin_amdgcn_s_memrealtime();
        const uint64_t last = __hip_atomic_load(r.last_claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // signed: the real-time counters of different XCDs need not agree, and a
        // claim stamped on an XCD whose clock runs ahead must not read as idle time
        if ((int64_t)(now - (last > t_start ? last : t_start)) > (int64_t)r.idle_ticks) {
            atomicExch(r.exiting, 1u);
            return -1;
        }
        // back off while nothing arrives (s_sleep k waits about 64 k cycles)
        if (idle_rounds < 6) ++idle_rounds;
        for (int z = 0; z < (1 << idle_rounds); ++z) __builtin_amdgcn_s_sleep(2);
    }
}

// Claim for one wave through its workgroup: one wave of the block at a time
// talks to the ring (an LDS lock), the others wait on the CU.  This keeps the
// polling and the head CAS to one wave per block instead of every resident
// wave.  A claim may take several consecutive items (serve_claim); the wave's
// unclaimed remainder waits in LDS, so that the next call returns it without
// touching the ring.  Call from every lane; returns the item (wave-uniform) or
// -1.  The LDS state must start zeroed (ClaimLds::clear).
struct ClaimLds {
    uint32_t lock;
    int64_t next[16], end[16];  // per wave of the block
    __device__ void clear(int tid) {
        if (tid == 0) lock = 0u;
        if (tid < 16) next[tid] = end[tid] = 0;
    }
};

__device__ inline int64_t serve_claim_block(const ServeRing &r, ClaimLds *cs, int wave, int lane) {
    int64_t item = 0;
    if (lane == 0) {
        if (cs->next[wave] < cs->end[wave]) {
            item = cs->next[wave]++;
        } else {
            // the lock is held while its wave waits for the ring: test before the CAS and
            // back off, so that waiting waves leave the CU's LDS and issue slots to the
            // waves decoding
            int back = 0;
            while (__hip_atomic_load(&cs->lock, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0u ||
                   atomicCAS(&cs->lock, 0u, 1u) != 0u) {
                for (int z = 0; z < (1 << back); ++z) __builtin_amdgcn_s_sleep(2);
                if (back < 5) ++back;
            }
            uint32_t cnt = 1;
            item = serve_claim(r, r.claim_max, &cnt);
            __hip_atomic_store(&cs->lock, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
            if (item >= 0) {
                cs->next[wave] = item + 1;
                cs->end[wave] = item + (int64_t)cnt;
            }
        }
    }
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)item);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)item >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// A completion-queue entry names its position's lap and the item in one word,
// so the reader can tell a fresh entry from an old one with a single load.
constexpr int CQ_ITEM_BITS = 40;
__host__ __device__ inline uint64_t cq_entry(uint64_t pos, uint64_t item, int64_t mask) {
    return ((pos / ((uint64_t)mask + 1) + 1) << CQ_ITEM_BITS) | (item & ((1ull << CQ_ITEM_BITS) - 1));
}

// Publish a finished ring item: every lane's stores first, then an entry of
// the completion queue (at most R items are in flight, so it never laps the
// host's reader).
__device__ inline void serve_publish(const ServeRing &r, int64_t item, int lane) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) {
        const unsigned long long p = atomicAdd(r.cq_tail, 1ull);
        __hip_atomic_store(r.cq + (p & r.mask), cq_entry(p, (uint64_t)item, r.mask), __ATOMIC_RELEASE,
                           __HIP_MEMORY_SCOPE_SYSTEM);
    }
}

__device__ inline int64_t uniform64(int64_t x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

struct OsdArgs {
    int32_t m, n, mw, nw, mws;  // mws: G row stride in words (odd)
    const uint64_t *vn_tab;
    const u32x4 *vn_tab4;       // wide codes (m > 8191): u32 slot positions, else null
    int32_t mode, order;
    const uint32_t *synd;
    uint32_t *corr;
    uint8_t *flags;
    const uint32_t *counters;   // [1] failed shots
    const int32_t *fail_list;
    const float *fail_llr;      // [fail_cap][2n]: lambda hi[n], lo[n]; or, with llr_i16, int16 lambda [fail_cap][n]
    int64_t fail_cap;
    int32_t llr_i16;            // fail_llr holds int16 lambda (the Int x.y check-centric kernel)
    uint32_t *gscratch;         // per-block scratch: G in global memory, or column ballots
    int32_t sort_p;             // power of two >= n
    int32_t g_in_lds;
    int32_t has_lo;             // lambda carries a non-zero low part (fp32 messages)
    int32_t llr_by_shot;        // fail_llr indexed by the shot (ring slot) instead of the list position
    int32_t cols_global;        // G-in-global variant: the per-column arrays live in the block's scratch too
    int64_t scratch_words;      // per-block stride of gscratch in 32-bit words
    int64_t cs_offset_words;    // OSD-CS column ballots in the block's scratch (kernels for m > 1024)
    // How blocks take failures: 0 strided over [0, counters[1]) (the list is complete);
    // 1 (alongside BP) and 2 (after BP) claim list positions from *claim in order, a
    // position once BP has published its entry (fail_list[q] >= 0, written after the
    // staged lambda).  Mode 1 waits for entries only while every one of BP's bp_grid
    // blocks is resident (counters[3] counts the started blocks, counters[4] the
    // finished ones), so it never holds resources BP needs; otherwise it exits.
    int32_t claim_mode;
    int32_t bp_grid;
    uint32_t *claim;            // counters + 2
};

// One group of a multi-group launch (lbp_plan): a code with its format and
// parameters, and the group's own input, output and OSD buffers.
struct GroupDesc {
    DevCode code;               // tables and priors (Int x.y prior of the group's format)
    BpParams prm;
    int32_t msg;                // MSG_FP32 / MSG_FP16 / MSG_INT8 (any Int x.y)
    int32_t pad0;
    int64_t first_item;         // work items [first_item, first_item + n_shots) are this group's shots
    int64_t n_shots;
    uint64_t first_shot_id;     // lottery counter of shot 0
    const uint32_t *synd;       // [n_shots][mw]
    uint32_t *corr;             // [n_shots][nw]
    uint8_t *flags;             // [n_shots]
    int32_t *iters;             // [n_shots] or null
    uint32_t *counters;         // [16]: [1] failed shots of the group
    int32_t *fail_list;         // [n_shots]
    float *fail_llr;            // [n_shots][2n]: staging for every shot (no overflow pass)
};

struct MultiArgs {
    const GroupDesc *groups;    // device table, ascending first_item
    int32_t n_groups;
    int32_t wave_bytes;         // LDS per wave: the largest group's shot state
    int64_t n_work;             // shots of all groups
    uint32_t *counter;          // next work item
    float *stage;               // [launched waves][stage_stride]
    int64_t stage_stride;       // floats per wave: 2 n of the widest group
};
hipError_t launch_bp_multi(const MultiArgs &a, int blocks, int wpb, hipStream_t s);
hipError_t bp_multi_prepare(int lds_bytes);
hipError_t bp_multi_max_blocks_per_cu(int wpb, int lds, int *out);

// Global-memory comparison path (one launch per half-iteration).
struct BlArgs {
    DevCode code;
    BpParams prm;
    int32_t msg;                // MSG_FP32 or MSG_FP16 storage
    int64_t shots;
    uint64_t first_shot_id;
    const uint64_t *shot_keys;  // nullable, as in BpArgs
    const uint32_t *synd;       // [shots][mw]
    uint32_t *corr;             // [shots][nw]
    uint8_t *flags;             // [shots]
    int32_t *iters;             // [shots] or null
    float *alpha, *beta;        // [shots][m*DEG]
    float *lam;                 // [shots][2][n]: lambda as an exact pair, hi[n] then lo[n]
    uint32_t *ehat;             // [shots][nw]
    uint32_t *shat;             // [shots][2][mw]: estimate of iteration i in slot i&1
    int32_t *flipv;             // [shots] column whose messages the next CN update negates, or -1
    uint8_t *active;            // [shots]
    uint32_t *counters;         // [0] shots still running after an iteration, [1] failed shots
    int32_t *fail_list;         // [shots]
};
hipError_t baseline_init(const BlArgs &a, hipStream_t s);
hipError_t baseline_iteration(const BlArgs &a, int i, hipStream_t s);
hipError_t baseline_stage(const BlArgs &a, int64_t from, int64_t count, float *dst, uint32_t *ocounters,
                          hipStream_t s);

// Set the thread-local message returned by lbp_last_error.
void set_error(const char *msg);

// LDS bytes the BP kernel needs per wave for a code.
int bp_wave_bytes(int msg, int m, int n);
// OSD kernel choice for a code: variant > 0 keeps G in registers (m < 1024;
// variant = 100 * rows per lane + NW words per row; rows_per_lane 1, else 2),
// 0 keeps G in LDS, -1 in global memory, -2 also keeps the per-column arrays
// (sort keys, order, non-basis list) in global memory (large n).  Returns LDS
// bytes per block for lambda staged as int16 (i16 = 1) or as fp32 pairs (0);
// *threads is the block size.
int osd_block_bytes(int m, int n, int lds_limit, int rows_per_lane, int i16, int *variant, int *mws, int *sort_p,
                    int *threads);
// Per-block global scratch of the OSD kernel.
size_t osd_scratch_bytes(int variant, int m, int n, int mws, int sort_p, int cs);
size_t osd_scratch_layout(int variant, int m, int n, int mws, int sort_p, int cs, size_t *cs_off);
hipError_t osd_max_blocks_per_cu(int variant, int threads, int lds, int *out);

// Int3.4 check-centric kernel (codes with <= 1024 checks): slots per lane
// (0 = not applicable), block-shared table bytes, per-wave LDS bytes.
// table: 0 per-check offset table in LDS, 1 compact space-time table in LDS, 2 compact
// table in global memory (codes with the Eq. 1 structure, 8 / 14 / 16 slots).
int bp_int8_slots(int m, int n);
int bp_int8_table_bytes(int table, int slots, int m0);
int bp_int8_wave_bytes(int m, int n);
hipError_t launch_bp_int8(int slots, int table, const BpArgs &a, int blocks, int waves_per_block, hipStream_t s);
hipError_t bp_int8_max_blocks_per_cu(int slots, int table, int waves_per_block, int lds_bytes, int *out);
// Compact space-time table of a code with the Eq. 1 structure (cols: padded rows,
// [m][DEG]); false when the code does not qualify.
bool bp_int8_build_st_table(const uint16_t *cols, int m, int n, int r, int m0, int n0, std::vector<uint32_t> &out);

hipError_t launch_reset(uint32_t *counters, int count, hipStream_t s);
// buf[0, count) = value
hipError_t launch_fill_i32(int32_t *buf, int32_t value, int64_t count, hipStream_t s);
hipError_t launch_bp(int msg, const BpArgs &a, int blocks, int waves_per_block, hipStream_t s);
hipError_t bp_max_blocks_per_cu(int msg, bool wide, bool group, int waves_per_block, int lds_bytes, int *out);
hipError_t launch_osd(const OsdArgs &a, int variant, int blocks, int threads, int lds_bytes, hipStream_t s);
hipError_t launch_gather_list(const uint32_t *counters, const int32_t *fail_list, int64_t from, int32_t *out,
                              int64_t count, hipStream_t s);

}  // namespace lbp
