/*
 * lbp.h -- C ABI of the MI355X Lottery BP (+OSD) decoder.
 *
 * The library decodes batches of syndromes of a sparse GF(2) parity-check
 * matrix H (m checks x n columns) with normalized min-sum belief propagation
 * (Algorithm 1 of "Lottery BP: Unlocking Quantum Error Decoding at Scale"),
 * the lottery sign-flip policy of Algorithm 3, and ordered-statistics
 * decoding (OSD-0 of Algorithm 2, or the OSD-CS combination sweep) for the
 * shots whose BP run does not converge.
 *
 * Conventions
 *  - Bit vectors (syndromes, corrections) are packed LSB-first into uint32
 *    words, ceil(bits/32) words per shot, shots stored back to back:
 *    bit b of shot k is word (k*W + b/32), bit (b % 32).
 *  - Functions return an lbp_status; on failure lbp_last_error() returns a
 *    thread-local message.  No C++ exception crosses the boundary.
 *  - Handles are not thread-safe: one thread at a time per handle.
 *  - Every result of shot k depends only on (code, params, seed,
 *    first_shot_id + k, syndrome k): never on batch size or composition.
 */
#ifndef LBP_H
#define LBP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBP_OK = 0,
    LBP_EINVAL = -1,        /* malformed argument (bad CSR, prior outside (0,1), size, NULL) */
    LBP_ENOMEM = -2,        /* device or host allocation failed */
    LBP_EDEVICE = -3,       /* HIP runtime error (message says which call) */
    LBP_EBUSY = -4,         /* serving: admission refused, or no free slot */
    LBP_ENOTREADY = -5,     /* serving: result not available yet */
    LBP_EUNSUPPORTED = -6   /* valid input outside what the kernels handle (see lbp_code_create) */
} lbp_status;

typedef struct lbp_code_s *lbp_code;       /* immutable Tanner graph + priors (device copy) */
typedef struct lbp_decoder_s *lbp_decoder; /* parameters + device workspace for up to max_batch shots */
typedef struct lbp_server_s *lbp_server;   /* continuous-batching serving loop (one device) */

/* Message storage format.  INT8 is the paper's Int3.4 fixed point (Sec. VII-A):
 * signed 8-bit, LSB = 1/16, saturated symmetrically to +-127; column LLRs are
 * accumulated exactly in 32-bit integers.  FP16 / FP32 store V2C and C2V
 * messages (and the prior) rounded to nearest even, saturating at the largest
 * finite value, and accumulate in fp32. */
typedef enum { LBP_MSG_FP32 = 0, LBP_MSG_FP16 = 1, LBP_MSG_INT8 = 2 } lbp_msg;
/* Fixed point Int x.y for the quantization study (Sec. VII-A, Fig. 15): a sign
 * bit, x integer and y fraction bits (1 <= x + y <= 7), i.e. integers in units
 * of 2^-y saturated symmetrically to +-(2^(x+y) - 1).  The prior is 2^y mu
 * rounded to nearest even, then saturated; a degree-1 check sends the largest
 * magnitude.  LBP_MSG_FIXED(3, 4) is LBP_MSG_INT8.  Other formats (x + y > 7,
 * bits above 0x1FF) are rejected with LBP_EINVAL. */
#define LBP_MSG_FIXED(x, y) (0x100 | ((x) << 4) | (y))

/* Check-node scale (Algorithm 1, CN update).  PAPER: sigma_i = 1 - 2^-(i+1),
 * evaluated in fp32 (exactly 1.0 from i = 24); Int3.4 applies it as
 * mag - (mag >> (i+1)).  CONST: a fixed factor (Int3.4 requires k/8, applied as
 * (k*mag) >> 3). */
typedef enum { LBP_SCALE_PAPER = 0, LBP_SCALE_CONST = 1 } lbp_scale;

/* What the lottery flips (Algorithm 3, last step).  MSG: the messages v* sends
 * into the next check-node update are negated for that one update (the
 * hardware's sign-flip stage in front of the CNU, Sec. IV-B).  LLR: lambda_v*
 * itself is negated before the next VN update (the literal Algorithm 3). */
typedef enum { LBP_FLIP_MSG = 0, LBP_FLIP_LLR = 1 } lbp_flip;

/* Lottery selection rule (the design space of Sec. III-B and Table I):
 * lottery_rule = CN rule | (VN rule << 4).  Let r0 and r1 be the upper 32 bits
 * of words 0 and 1 of the Philox block of (shot_id, i), divided by 2^32.
 *   LBP_CN_RANDOM: c* = the floor(r0 |U|)-th check of U in ascending order
 *                  (Algorithm 3).
 *   LBP_CN_WORST:  c* = the check of U with the most neighbours whose current
 *                  hard decision is 1; the smallest index among equals.
 *   LBP_VN_PROPOSED:   v* = the neighbour of c* with the most checks in U, then
 *                      the smallest Q(|lambda|), then the smallest column
 *                      (Algorithm 3, Sec. IV-B).
 *   LBP_VN_Q_FIRST:    smallest Q first, then most checks in U, then column (the
 *                      order in which Sec. III-B words the proposed key).
 *   LBP_VN_UNRELIABLE: smallest Q, then smallest column.
 *   LBP_VN_RANDOM:     the floor(r1 deg(c*))-th neighbour of c* in ascending order.
 * Q(|lambda|) is |lambda| for INT8 and floor(|lambda| 2^12) for float formats. */
enum { LBP_CN_RANDOM = 0, LBP_CN_WORST = 1 };
enum { LBP_VN_PROPOSED = 0, LBP_VN_Q_FIRST = 1, LBP_VN_UNRELIABLE = 2, LBP_VN_RANDOM = 3 };
#define LBP_LOTTERY_RULE(cn, vn) ((cn) | ((vn) << 4))

/* Fallback for shots whose BP run ends without matching the syndrome. */
typedef enum { LBP_OSD_NONE = 0, LBP_OSD_0 = 1, LBP_OSD_CS = 2 } lbp_osd;

typedef struct {
    int32_t max_iter;     /* I >= 1 (Algorithm 1 input) */
    int32_t scale_mode;   /* lbp_scale */
    float scale;          /* constant scale for LBP_SCALE_CONST */
    int32_t msg;          /* lbp_msg */
    int32_t lottery;      /* 0 = plain NMS BP, 1 = Lottery BP */
    int32_t lottery_skip; /* K: the lottery runs after iterations K..I-2 (0-based); paper uses 6 */
    int32_t flip;         /* lbp_flip */
    int32_t osd;          /* lbp_osd */
    int32_t osd_order;    /* OSD-CS: weight-2 patterns among the first osd_order non-basis columns */
    int32_t lottery_rule; /* LBP_LOTTERY_RULE(cn, vn); 0 = Algorithm 3; other values rejected (LBP_EINVAL) */
    uint64_t seed;        /* lottery key: Philox4x64-10, key (seed, 0), counter (shot_id, i, 0, 0) */
} lbp_params;

/* flags[k] bits */
enum {
    LBP_FLAG_CONVERGED = 1,        /* BP matched the syndrome */
    LBP_FLAG_OSD = 2,              /* BP did not converge; OSD was run */
    LBP_FLAG_OSD_INCONSISTENT = 4  /* s is not in the column space of H; correction = BP hard decision */
};

/* Fill *p with the defaults: I = 100, PAPER scale, INT8, lottery on, K = 6,
 * MSG flip, OSD-0, order 10, rule 0 (Algorithm 3), seed 0. */
void lbp_params_default(lbp_params *p);

/* Load a parity-check matrix and per-column priors (Algorithm 1 inputs H and p).
 * row_ptr[m+1], col_idx[row_ptr[m]] (host pointers): CSR with strictly
 * increasing column indices per row; p[n] (host): error probability of each
 * column, 0 < p < 1.  The library copies everything; the caller may free its
 * arrays on return.  The prior LLR mu_v = ln((1-p_v)/p_v) is evaluated in
 * fp64 on the host (Algorithm 1, prior).
 * Limits (LBP_EUNSUPPORTED otherwise): 1 <= row weight <= 8, column weight
 * <= 4, m <= 32767, n <= 65535.  Empty rows and malformed CSR: LBP_EINVAL.
 * Whether a decoder fits the device is decided by lbp_decoder_create (the
 * per-shot messages of the chosen format must fit one CU's LDS: for
 * space-time surface codes Int x.y reaches about 18000 checks, FP16 about
 * 9500, FP32 about 4900).
 * The column table keeps each edge's slot position (8 check + slot) in 16
 * bits when m <= 8191 and in 32 bits above; the environment variable
 * LBP_WIDE_COLUMN_TABLE=1, read here, selects the 32-bit layout for any code
 * (it changes no result; it exists to test that layout on small codes).
 * The code lives on the device that is current when it is created. */
lbp_status lbp_code_create(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                           const double *p, lbp_code *out);
void lbp_code_destroy(lbp_code code);
/* Shape queries (never fail on a valid handle). */
int32_t lbp_code_rows(lbp_code code);
int32_t lbp_code_cols(lbp_code code);

/* Create a decoder for `code` with parameters *prm, able to decode up to
 * max_batch shots per call.  *prm fixes Algorithm 1's remaining input, the
 * iteration limit I, and the choices the paper leaves to the decoder: the
 * message format (Sec. VII-A), the check-node scale (Algorithm 1, CN update),
 * the lottery and its rule (Algorithm 3, Sec. III-B) and the OSD fallback
 * (Algorithm 2, or the OSD-CS sweep).  Allocates the device workspace (on the code's
 * device).  OSD-CS requires a uniform prior (LBP_EUNSUPPORTED otherwise): its
 * candidate cost is the Hamming weight.  The decoder holds a reference to the
 * code: lbp_code_destroy may come before lbp_decoder_destroy (in any order);
 * the code's device memory is released with its last user.
 * The launch shape is chosen here from the per-shot state and the device: a
 * wavefront per shot, or a workgroup of 2-16 waves per shot when fewer than 32
 * one-wave shots fit a CU.  The environment variable LBP_BP_GROUP=g, read
 * here, forces workgroups of g waves (it changes no result; it exists to test
 * that variant on small codes).  OSD keeps G in registers for codes with
 * fewer than 1024 checks, two rows per lane; LBP_OSD_ROWS_PER_LANE=1, read
 * here, selects one row per lane (same results; for tests). */
lbp_status lbp_decoder_create(lbp_code code, const lbp_params *prm, int64_t max_batch, lbp_decoder *out);
void lbp_decoder_destroy(lbp_decoder dec);

/* Decode n_shots syndromes, asynchronously on `stream` (a hipStream_t; NULL =
 * the default stream): per shot, Algorithm 1 (with Algorithm 3 when the lottery
 * is on) maps the syndrome s to the estimate e_hat; a shot whose run ends
 * without H e_hat = s goes to Algorithm 2 (OSD) with the lambda of the last
 * iteration, which replaces e_hat.  All array arguments are DEVICE pointers owned by the
 * caller, which must keep them alive until the stream has passed this call:
 *   syndromes   [n_shots][ceil(m/32)]  in
 *   corrections [n_shots][ceil(n/32)]  out: e_hat (BP hard decision, or OSD result)
 *   flags       [n_shots]              out: LBP_FLAG_*
 *   iters       [n_shots]              out, may be NULL: BP iterations executed
 *   llr_out     [n_shots][n]           out, may be NULL: lambda of the last BP
 *               iteration executed (Int3.4: integer units of 1/16)
 * Shot k uses lottery counter shot_id = first_shot_id + k.  0 <= n_shots <=
 * max_batch.  The call may synchronize `stream` when more shots fail BP than
 * the decoder's OSD staging capacity (lbp_decoder_osd_capacity). */
lbp_status lbp_decode(lbp_decoder dec, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                      uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out, void *stream);

/* lbp_decode with a lottery key per shot instead of (params seed, first_shot_id + k):
 * shot_keys [n_shots][2] (DEVICE) holds (seed, shot_id) of each shot, as
 * Algorithm 3's random draw for shot k at iteration i uses Philox4x64-10 with
 * key (seed, 0) and counter (shot_id, i, 0, 0).  Used to pack shots of
 * different requests into one launch without changing any result. */
lbp_status lbp_decode_keyed(lbp_decoder dec, int64_t n_shots, const uint64_t *shot_keys, const uint32_t *syndromes,
                            uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): lbp_decode with the
 * same arguments, kernels and results, that allocates nothing and never
 * synchronizes.  Every buffer besides the caller's inputs and outputs (work
 * and failure counters, the failure list, the staged lambda of failed shots,
 * the float kernels' per-wave staging, the OSD blocks' scratch) is carved from
 * one static device array of LBP_NOALLOC_SCRATCH_BYTES that the library holds
 * on each GPU it runs on until the process ends; its address is looked up once
 * per device (at lbp_decoder_create).  The counters are cleared by a kernel at
 * the start of each call.  Staging is reserved for every shot, so n_shots is
 * bounded by that array: a larger n_shots returns LBP_EINVAL and the message
 * names the largest batch of this decoder that fits (e.g. about 14000 shots of
 * BB[[144,12,12]] over 12 rounds with Int3.4 and OSD-CS).  n_shots is not
 * bounded by the decoder's max_batch, and the decoder's own workspace is not
 * used.  All calls on one GPU share the array, which keeps the last call's
 * contents: calls that overlap on one GPU (other streams, other threads) race
 * and must be serialized by the caller.  Timing (lbp_decoder_set_timing) does
 * not record these calls. */
#define LBP_NOALLOC_SCRATCH_BYTES ((uint64_t)128 << 20)
lbp_status lbp_decode_noalloc(lbp_decoder dec, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                              uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out, void *stream);

/* Comparison path: the same decoding as lbp_decode (FP32 or FP16 message
 * storage; LBP_EUNSUPPORTED for INT8) written the plain way, with every
 * message in global memory, one thread per check or per column and a kernel
 * launch per half-iteration (Algorithm 1's CN update, then LLR update + hard
 * decision + next VN update, then syndrome check + Algorithm 3).  Sums are
 * taken in fp64 in ascending check order and rounded once to the storage
 * format.  Same arguments and outputs as lbp_decode (no llr_out).  Allocates
 * its message arrays on first use (n_shots * (8*m*8 + 8*n) bytes, kept until
 * the decoder is destroyed) and synchronizes `stream` every 4 iterations to
 * stop once all shots have finished. */
lbp_status lbp_decode_baseline(lbp_decoder dec, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                               uint32_t *corrections, uint8_t *flags, int32_t *iters, void *stream);

/* Same contract as lbp_decode (Algorithm 1 with Algorithm 3, then Algorithm 2
 * on the shots BP leaves unsolved) with HOST pointers; synchronous.  Allocates and
 * frees device staging buffers internally. */
lbp_status lbp_decode_host(lbp_decoder dec, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                           uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out);

/* The decoder's launch shapes, chosen at creation (any output may be NULL):
 * BP waves per workgroup and resident workgroups of the persistent grid, BP
 * group size (waves that decode one shot together; 1 = a wavefront per shot),
 * and the OSD kernel: variant (> 0: G in registers, 100 * rows per lane + words
 * per row; 0: G in LDS; -1: G in global memory; -2: G and the per-column arrays
 * in global memory), threads per workgroup and workgroups. */
lbp_status lbp_decoder_shape(lbp_decoder dec, int32_t *bp_waves_per_block, int32_t *bp_blocks, int32_t *bp_group,
                             int32_t *osd_variant, int32_t *osd_threads, int32_t *osd_blocks);

/* Device bytes held by the decoder's workspace, and its max_batch. */
int64_t lbp_decoder_device_bytes(lbp_decoder dec);
int64_t lbp_decoder_max_batch(lbp_decoder dec);

/* Number of failed shots whose lambda one OSD pass can stage (2n bytes each as
 * int16 for Int x.y codes of at most 1024 checks, else 8n bytes as an fp32
 * (hi, lo) pair; initially 256 MiB worth).  Failures beyond it are re-decoded (BP is
 * deterministic) and handled in a further pass; when the overflow exceeds the
 * capacity, lbp_decode first grows the staging to the overflow, bounded by
 * max_batch and a quarter of the free device memory, so a high OSD invoke rate
 * costs one extra BP pass once, not one per capacity's worth of failures. */
int64_t lbp_decoder_osd_capacity(lbp_decoder dec);
/* Testing aid: lower the staging capacity (>= 1) to exercise the overflow path;
 * a lowered capacity is never grown again. */
lbp_status lbp_decoder_set_osd_capacity(lbp_decoder dec, int64_t cap);

/* Kernel timing (tracing aid).  While enabled, lbp_decode records a pair of HIP
 * events around every BP and every OSD kernel launch on the call's stream.
 * lbp_decoder_kernel_times waits for the recorded events, returns the
 * accumulated GPU milliseconds and launch counts since the last query, and
 * resets them.  Any output pointer may be NULL. */
lbp_status lbp_decoder_set_timing(lbp_decoder dec, int32_t enable);
lbp_status lbp_decoder_kernel_times(lbp_decoder dec, double *bp_ms, int64_t *bp_launches, double *osd_ms,
                                    int64_t *osd_launches);

/* ---- Multi-group plans: shots of several codes in one launch.  A plan decodes
 * groups of shots whose codes, message formats and parameters differ (each
 * group is one decoder's code and lbp_params) with one persistent BP launch:
 * every wavefront claims the next shot of any group from a device descriptor
 * table and decodes it with that group's code, format and parameters, in an LDS
 * slice sized for the largest group; then each group with OSD gets its OSD
 * launch (Algorithm 1 and 3 for BP, Algorithm 2 for OSD-0; OSD-CS as for
 * lbp_decode).  Every shot's result equals lbp_decode of its group alone (same
 * seed and shot ids): per-shot results never depend on what shares the launch.
 * The groups' buffers are bound when the plan is created, and the launch
 * sequence is captured once into a HIP graph: a caller writes new syndromes
 * into the same buffers and replays the graph with lbp_plan_launch.  The plan
 * reserves failure staging for every shot of every group (8n bytes per shot of
 * a group with OSD), so a replay never needs a second pass.  Codes above 8191
 * checks are not supported in plans (LBP_EUNSUPPORTED). */
typedef struct lbp_plan_s *lbp_plan;
typedef struct {
    lbp_decoder dec;            /* code, format and parameters of the group (its workspace is not used);
                                   it must outlive the plan */
    int64_t n_shots;            /* >= 0 */
    uint64_t first_shot_id;     /* lottery counter of the group's shot 0 (shot k uses first_shot_id + k) */
    const uint32_t *syndromes;  /* DEVICE [n_shots][ceil(m/32)] */
    uint32_t *corrections;      /* DEVICE [n_shots][ceil(n/32)] */
    uint8_t *flags;             /* DEVICE [n_shots] */
    int32_t *iters;             /* DEVICE [n_shots] or NULL */
} lbp_group;
/* Autotuning: time every feasible launch shape (waves per block, with the
 * resident blocks the occupancy allows) on the device, on the groups' own
 * buffers, and keep the fastest; without it the shape with the most resident
 * waves is used. */
enum { LBP_PLAN_AUTOTUNE = 1 };
/* Build a plan over n_groups (1..64) groups on one device (the decoders'):
 * allocates its descriptor table and workspace, runs the sequence eagerly
 * (with LBP_PLAN_AUTOTUNE, three times per candidate shape), so the groups'
 * outputs then hold the results of their current syndromes, and captures the
 * sequence into a graph.  Synchronous. */
lbp_status lbp_plan_create(int32_t n_groups, const lbp_group *groups, int32_t options, lbp_plan *out);
/* Decode every group again (replay of the captured graph) on `stream`
 * (hipStream_t, NULL = default), asynchronously.  Replays on one plan must not
 * overlap (they share the plan's workspace). */
lbp_status lbp_plan_launch(lbp_plan plan, void *stream);
/* The launch shape in use and, after autotuning, the measured milliseconds of
 * each candidate (candidate_ms: room for 8 values; any output may be NULL). */
lbp_status lbp_plan_info(lbp_plan plan, int32_t *waves_per_block, int32_t *blocks, int32_t *n_candidates,
                         double *candidate_ms);
void lbp_plan_destroy(lbp_plan plan);

/* ---- Serving (real-time decoding of a stream of requests, Sec. I and VI-B:
 * the decoder must keep up with syndromes as they arrive, and its tail
 * latency matters).  A server owns one worker thread on the device current
 * at creation, its queues and all device buffers; the caller owns its host
 * arrays.  lbp_server_* calls are thread-safe.
 *
 * Streaming: every code slot has a ring of R shots in pinned host memory and
 * a persistent BP grid that claims published shots one per wavefront (or
 * workgroup, for large codes), so each shot's result is visible as soon as
 * that shot is done (no batch boundaries).  Shots whose BP run fails are
 * handed to OSD launches.  A slot's BP and OSD streams are CU-masked to 20 and
 * 12 of every 32 CUs, so OSD never holds the CUs BP needs; with several slots
 * their BP grids split the BP CUs.  The worker publishes queued shots first
 * come first served, splitting large requests, with at most R shots in flight
 * per slot; a request completes when all of its shots have.  Each shot is
 * decoded with the key (seed, first_shot_id + j) of its request, so results
 * equal a lone lbp_decode of the request with that seed, whatever else is in
 * flight.  The BP grid exits after 2 ms without work (20 us when the server
 * holds several slots) and is relaunched when shots arrive.  CU-masked
 * streams synchronize with the legacy default stream: work the caller
 * enqueues there waits for a running grid to exit. */

/* device_mem_budget_bytes: cap on the device memory all slots may hold (0 =
 * 16 GiB); max_slots: number of codes (1..64). */
lbp_status lbp_server_create(int64_t device_mem_budget_bytes, int32_t max_slots, lbp_server *out);
/* Register a code with its decoding parameters (params.seed is ignored: each
 * request brings its own).  Picks the largest ring (power of two, 1024 ..
 * 65536 shots; per shot 2n bytes of device memory for Int x.y codes of at most
 * 1024 checks, else 8n, for the lambda of shots left to OSD) that fits the remaining
 * budget: LBP_ENOMEM if none does, LBP_EBUSY if all slots are taken.  The
 * slot holds a reference to the code (as a decoder does). */
lbp_status lbp_server_add_code(lbp_server srv, lbp_code code, const lbp_params *prm, int32_t *code_slot);
/* Queue n_shots >= 1 syndromes (HOST, [n_shots][ceil(m/32)], copied before
 * return).  Admission: LBP_EBUSY when the slot would hold more than 16 rings'
 * worth of queued shots.  *ticket identifies the request. */
lbp_status lbp_server_submit(lbp_server srv, int32_t code_slot, int64_t n_shots, uint64_t seed,
                             uint64_t first_shot_id, const uint32_t *host_syndromes, uint64_t *ticket);
/* LBP_ENOTREADY while the request is pending.  Once complete, copies the
 * results into the HOST arrays (corrections [n_shots][ceil(n/32)], flags
 * [n_shots], iters [n_shots]; any may be NULL), releases the ticket and
 * returns LBP_OK (or the error that stopped the request).  Unknown or
 * released ticket: LBP_EINVAL. */
lbp_status lbp_server_poll(lbp_server srv, uint64_t ticket, uint32_t *corrections, uint8_t *flags, int32_t *iters);
/* lbp_server_poll that blocks up to timeout_us microseconds (< 0: no limit). */
lbp_status lbp_server_wait(lbp_server srv, uint64_t ticket, int64_t timeout_us, uint32_t *corrections,
                           uint8_t *flags, int32_t *iters);
/* Drop a request: its queued shots are never published, results of shots
 * already in flight are discarded, and the ticket is released. */
lbp_status lbp_server_cancel(lbp_server srv, uint64_t ticket);
/* Slot statistics: ring size, BP grid launches, shots completed, most shots
 * in flight at once, shots queued now.  Any output may be NULL. */
lbp_status lbp_server_slot_info(lbp_server srv, int32_t code_slot, int64_t *ring_items, int64_t *bp_launches,
                                int64_t *shots, int64_t *max_inflight, int64_t *queued_shots);
/* Benchmarking aid: drive the server with an open-loop stream of n_requests
 * requests of shots_per_request syndromes each.  Request q goes to
 * code_slots[k], k uniform in [0, n_codes) (request_code[q] = k, may be
 * NULL), and takes the next shots_per_request rows of host_syndromes[k]
 * ([pool[k]][ceil(m_k/32)], HOST, cycled), with lottery key (seed,
 * q * shots_per_request + j).  Arrivals form a Poisson process of rate
 * requests_per_s (0: submit back to back, retrying while admission refuses:
 * the saturation load).  latency_us[q] = time from request q's scheduled
 * arrival to the moment its result is visible to lbp_server_poll;
 * *elapsed_s (may be NULL) = first arrival to last completion.  Returns when
 * every request has completed. */
lbp_status lbp_server_run_load(lbp_server srv, int32_t n_codes, const int32_t *code_slots,
                               const uint32_t *const *host_syndromes, const int64_t *pool, int64_t n_requests,
                               int64_t shots_per_request, double requests_per_s, uint64_t seed,
                               int32_t *request_code, double *latency_us, double *elapsed_s);
/* Stop the worker (pending requests are dropped) and free everything. */
void lbp_server_destroy(lbp_server srv);

/* Thread-local description of the last error (empty string if none). */
const char *lbp_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int32_t lbp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LBP_H */
