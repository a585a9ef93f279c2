// Host runtime of the C ABI in include/lbp.h: validation, device tables,
// workspace sizing, launch configuration and the OSD overflow loop.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/lbp.h"
#include "lbp_internal.h"
#include "serve_internal.h"

using namespace lbp;

namespace {

thread_local std::string g_err;

lbp_status fail(lbp_status s, const std::string &msg) {
    g_err = msg;
    return s;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess) {                                                               \
            lbp_status st_ = e_ == hipErrorOutOfMemory ? LBP_ENOMEM : LBP_EDEVICE;            \
            return fail(st_, std::string(#call) + ": " + hipGetErrorString(e_));              \
        }                                                                                     \
    } while (0)

struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) == hipSuccess && prev != dev) hipSetDevice(dev);
        else prev = -1;
    }
    ~DeviceGuard() {
        if (prev >= 0) hipSetDevice(prev);
    }
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Round a double to the nearest binary16 value (ties to even), saturating at 65504.
float to_fp16_value(double x) {
    _Float16 h = (_Float16)x;
    float f = (float)h;
    if (std::isinf(f)) f = x > 0 ? 65504.0f : -65504.0f;
    return f;
}

}  // namespace

void lbp::set_error(const char *msg) { g_err = msg ? msg : ""; }

// Scratch of lbp_decode_noalloc: a static device array that the library holds on
// every GPU it runs on until the process ends (LBP_NOALLOC_SCRATCH_BYTES).  In
// host code `scratch` names a host-side stand-in, never the device memory: its
// device address is looked up once per device with hipGetSymbolAddress (each GPU
// has its own copy at its own address) and only that pointer is used.
static __device__ __align__(256) unsigned char scratch[LBP_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];

// Device address of `scratch` on device `dev`, which must be current; nullptr
// with the error message set when the lookup fails.
void *scratch_on(int dev) {
    if (dev < 0 || dev >= kMaxDevices) {
        g_err = "lbp_decode_noalloc: device index out of range";
        return nullptr;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            g_err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
            return nullptr;
        }
        g_scratch_dev[dev] = ptr;
    }
    return g_scratch_dev[dev];
}
}  // namespace

struct lbp_code_s {
    int m = 0, n = 0, nnz = 0, device = 0;
    bool uniform = true;
    std::vector<double> mu;  // prior LLRs (fp64, host): fixed-point decoders quantize their own copy
    void *dmem = nullptr;
    DevCode dc{};
    std::atomic<int> refs{1};  // the creator's reference plus one per decoder using the code
};

struct lbp_decoder_s {
    lbp_code code = nullptr;
    lbp_params prm{};
    int msgk = 0;       // message storage the kernels run: MSG_FP32 / MSG_FP16 / MSG_INT8 (any Int x.y)
    DevCode dc{};       // the code's tables, with this decoder's fixed-point prior
    int32_t *d_muq = nullptr;
    int64_t max_batch = 0;
    BpParams bp{};
    int wpb = 1, bp_blocks = 1, wave_bytes = 0, int8_slots = 0, table_bytes = 0, group = 0;
    int int8_table = 0;  // where the Int x.y kernel takes its column offsets from (bp_int8_table_bytes)
    int osd_blocks = 0, osd_lds = 0, osd_variant = 0, osd_threads = 1024, mws = 1, sort_p = 1;
    int osd_lds_pairs = 0;  // OSD LDS per block when lambda is staged as fp32 pairs (general BP kernel)
    int64_t fail_cap = 0;
    int64_t llr_bytes = 0;         // staged lambda per failed shot: 2n (int16, Int x.y kernel) or 8n (hi, lo floats)
    bool fail_cap_pinned = false;  // set by lbp_decoder_set_osd_capacity: never grown
    int64_t dev_bytes = 0;  // device workspace held by the decoder
    uint32_t *d_counters = nullptr;
    int32_t *d_fail_list = nullptr;
    int32_t *d_list2 = nullptr;
    float *d_fail_llr = nullptr;
    float *d_stage = nullptr;
    uint32_t *d_gscratch = nullptr;
    uint32_t *d_gscratch2 = nullptr;  // OSD scratch of the grid that runs alongside BP (allocated on first use)
    bool early_osd = false;           // Int x.y kernel + OSD: an OSD grid takes failures while BP runs
    hipEvent_t ev_early = nullptr;
    uint32_t *h_count = nullptr;  // pinned
    // global-memory comparison path, allocated on first use
    int64_t bl_cap = 0;
    float *bl_alpha = nullptr, *bl_beta = nullptr;
    float *bl_lam = nullptr;   // [shots][2][n] exact pairs
    uint32_t *bl_ehat = nullptr, *bl_shat = nullptr;
    int32_t *bl_flipv = nullptr;
    uint8_t *bl_active = nullptr;
    // kernel timing: event pairs per launch, kind 0 = BP, 1 = OSD
    bool timing = false;
    struct Rec {
        hipEvent_t a, b;
        int kind;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    // pipelined decode of large batches: BP of chunk i + 1 on the caller's stream
    // while OSD of chunk i runs on `side`; chunks alternate over two failure
    // workspaces, each sized for a whole chunk (no chunk can overflow its staging)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_bp[2] = {nullptr, nullptr}, ev_osd[2] = {nullptr, nullptr};
    int64_t pipe_chunk = 0;  // shots per chunk the workspaces hold (0: none yet)
    uint32_t *pipe_counters[2] = {nullptr, nullptr};
    int32_t *pipe_list[2] = {nullptr, nullptr};
    float *pipe_llr[2] = {nullptr, nullptr};
};

static hipEvent_t take_event(lbp_decoder d) {
    if (!d->pool.empty()) {
        hipEvent_t e = d->pool.back();
        d->pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

lbp_status lbp::serve_shape(lbp_decoder d, double osd_fraction, ServeShape *out) {
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, d->code->device) != hipSuccess)
        return fail(LBP_EDEVICE, "serve_shape: device query failed");
    const int bpc = std::max(1, d->bp_blocks / std::max(1, ncu));
    const int osd_cus = d->prm.osd ? std::max(1, (int)(ncu * osd_fraction)) : 0;
    out->bp_blocks = std::max(1, std::min(d->bp_blocks, bpc * (ncu - osd_cus)));
    out->osd_blocks = d->prm.osd ? std::max(1, std::min(d->osd_blocks, osd_cus * std::max(1, d->osd_blocks / ncu))) : 0;
    return LBP_OK;
}

int64_t lbp::serve_llr_bytes(lbp_decoder d) { return (int64_t)d->code->n * (d->int8_slots ? 2 : 8); }

lbp_status lbp::serve_launch_bp(lbp_decoder d, const ServeRing *ring_dev, uint32_t *exiting, int blocks,
                                hipStream_t s) {
    HIPCHK(launch_reset(exiting, 1, s));  // the previous grid has drained: stream order
    BpArgs a{};
    a.code = d->dc;
    a.prm = d->bp;
    a.ring = ring_dev;
    a.stage = d->d_stage;
    a.wave_bytes = d->wave_bytes;
    a.group = d->group;
    blocks = std::max(1, std::min(blocks, d->bp_blocks));  // d_stage holds bp_blocks * wpb waves
    HIPCHK(d->int8_slots ? launch_bp_int8(d->int8_slots, d->int8_table, a, blocks, d->wpb, s)
                         : launch_bp(d->msgk, a, blocks, d->wpb, s));
    return LBP_OK;
}

// OSD arguments that depend only on the decoder (code tables, variant, formats).
static OsdArgs osd_args(lbp_decoder d) {
    lbp_code C = d->code;
    OsdArgs o{};
    o.m = C->m;
    o.n = C->n;
    o.mw = C->dc.mw;
    o.nw = C->dc.nw;
    o.mws = d->mws;
    o.vn_tab = C->dc.vn_tab;
    o.vn_tab4 = C->dc.vn_tab4;
    o.mode = d->prm.osd;
    o.order = d->prm.osd_order;
    o.sort_p = d->sort_p;
    o.g_in_lds = d->osd_variant == 0;
    o.cols_global = d->osd_variant == -2;
    size_t cs_off = 0;
    o.scratch_words = (int64_t)(osd_scratch_layout(d->osd_variant, C->m, C->n, d->mws, d->sort_p,
                                                   d->prm.osd == LBP_OSD_CS, &cs_off) / 4);
    o.cs_offset_words = (int64_t)(cs_off / 4);
    o.has_lo = d->msgk != LBP_MSG_INT8;  // float lambda is an exact (hi, lo) pair
    o.llr_i16 = d->int8_slots != 0;
    return o;
}

lbp_status lbp::serve_launch_osd(lbp_decoder d, const ServeRing &ring, const int32_t *d_list,
                                 const uint32_t *d_counters, int blocks, hipStream_t s) {
    OsdArgs o = osd_args(d);
    o.synd = ring.syn;
    o.corr = ring.corr;
    o.flags = ring.flags;
    o.counters = d_counters;
    o.fail_list = d_list;
    o.fail_llr = o.llr_i16 ? (const float *)ring.llr16 : ring.llr;
    o.fail_cap = (int64_t)1 << 40;
    o.gscratch = d->d_gscratch;
    o.llr_by_shot = 1;
    blocks = std::max(1, std::min(blocks, d->osd_blocks));  // d_gscratch holds osd_blocks blocks
    HIPCHK(launch_osd(o, d->osd_variant, blocks, d->osd_threads, d->osd_lds, s));
    return LBP_OK;
}

lbp_status lbp::decoder_view(lbp_decoder d, DecoderView *out) {
    if (!d || !out) return fail(LBP_EINVAL, "NULL decoder");
    lbp_code C = d->code;
    out->dc = d->dc;
    out->bp = d->bp;
    out->msgk = d->msgk;
    out->osd = d->prm.osd;
    out->device = C->device;
    out->osd_blocks = d->osd_blocks;
    out->osd_scratch = d->prm.osd ? osd_scratch_bytes(d->osd_variant, C->m, C->n, d->mws, d->sort_p,
                                                      d->prm.osd == LBP_OSD_CS)
                                  : 0;
    return LBP_OK;
}

lbp_status lbp::decoder_launch_osd(lbp_decoder d, const uint32_t *synd, uint32_t *corr, uint8_t *flags,
                                   const uint32_t *counters, const int32_t *fail_list, const float *fail_llr,
                                   int64_t fail_cap, uint32_t *gscratch, int blocks, hipStream_t s) {
    OsdArgs o = osd_args(d);
    o.synd = synd;
    o.corr = corr;
    o.flags = flags;
    o.counters = counters;
    o.fail_list = fail_list;
    o.fail_llr = fail_llr;
    o.fail_cap = fail_cap;
    o.gscratch = gscratch;
    o.llr_i16 = 0;  // the general kernel stages every format as fp32 pairs
    HIPCHK(launch_osd(o, d->osd_variant, blocks, d->osd_threads, d->osd_lds_pairs, s));
    return LBP_OK;
}

extern "C" {

const char *lbp_last_error(void) { return g_err.c_str(); }

int32_t lbp_version(void) { return 100; }

void lbp_params_default(lbp_params *p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->max_iter = 100;
    p->scale_mode = LBP_SCALE_PAPER;
    p->scale = 0.625f;
    p->msg = LBP_MSG_INT8;
    p->lottery = 1;
    p->lottery_skip = 6;
    p->flip = LBP_FLIP_MSG;
    p->osd = LBP_OSD_0;
    p->osd_order = 10;
    p->seed = 0;
}

lbp_status lbp_code_create(int32_t m, int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *p,
                           lbp_code *out) {
    g_err.clear();
    if (!out || !row_ptr || !col_idx || !p) return fail(LBP_EINVAL, "lbp_code_create: NULL argument");
    *out = nullptr;
    if (m < 1 || n < 1) return fail(LBP_EINVAL, "lbp_code_create: m and n must be >= 1");
    if (m > 32767 || n > 65535) return fail(LBP_EUNSUPPORTED, "lbp_code_create: m <= 32767 and n <= 65535 supported");
    if (row_ptr[0] != 0) return fail(LBP_EINVAL, "lbp_code_create: row_ptr[0] must be 0");
    for (int c = 0; c < m; ++c) {
        int w = row_ptr[c + 1] - row_ptr[c];
        if (w < 1) return fail(LBP_EINVAL, "lbp_code_create: row " + std::to_string(c) + " is empty or row_ptr decreases");
        if (w > DEG) return fail(LBP_EUNSUPPORTED, "lbp_code_create: row weight > 8 at row " + std::to_string(c));
        for (int e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
            if (col_idx[e] < 0 || col_idx[e] >= n)
                return fail(LBP_EINVAL, "lbp_code_create: column index out of range in row " + std::to_string(c));
            if (e > row_ptr[c] && col_idx[e] <= col_idx[e - 1])
                return fail(LBP_EINVAL, "lbp_code_create: column indices not strictly increasing in row " + std::to_string(c));
        }
    }
    for (int v = 0; v < n; ++v)
        if (!(p[v] > 0.0 && p[v] < 1.0)) return fail(LBP_EINVAL, "lbp_code_create: prior outside (0,1) at column " + std::to_string(v));
    const int nnz = row_ptr[m];
    // column tables: slot positions c*DEG + k in ascending check order
    std::vector<int> cw(n, 0);
    std::vector<uint64_t> tab(n, ~0ull);
    // wide layout (u32 positions) when c*DEG+k can exceed 16 bits, or on request
    const char *force_wide = std::getenv("LBP_WIDE_COLUMN_TABLE");
    const bool wide = m > MAX_M_NARROW || (force_wide && force_wide[0] == '1');
    std::vector<uint32_t> tab4(wide ? (size_t)n * CDEG : 0, NOPOS32);
    std::vector<uint16_t> cols((size_t)m * DEG, (uint16_t)NOPOS);
    std::vector<uint8_t> deg(m);
    for (int c = 0; c < m; ++c) {
        deg[c] = (uint8_t)(row_ptr[c + 1] - row_ptr[c]);
        for (int e = row_ptr[c]; e < row_ptr[c + 1]; ++e) {
            int v = col_idx[e], k = e - row_ptr[c];
            cols[(size_t)c * DEG + k] = (uint16_t)v;
            if (cw[v] >= CDEG) return fail(LBP_EUNSUPPORTED, "lbp_code_create: column weight > 4 at column " + std::to_string(v));
            const uint32_t pos = (uint32_t)(c * DEG + k);
            if (wide) tab4[(size_t)v * CDEG + cw[v]] = pos;
            if (m <= MAX_M_NARROW) {  // the narrow table serves the kernels limited to m <= 1024 in any case
                tab[v] &= ~(0xFFFFull << (16 * cw[v]));
                tab[v] |= (uint64_t)pos << (16 * cw[v]);
            }
            cw[v]++;
        }
    }
    std::vector<float> mu32(n), mu16(n);
    std::vector<int32_t> muq(n);
    bool uniform = true;
    for (int v = 0; v < n; ++v) {
        double mu = std::log((1.0 - p[v]) / p[v]);  // prior LLR of Algorithm 1 (fp64, host)
        mu32[v] = (float)mu;
        mu16[v] = to_fp16_value(mu);
        double q = std::nearbyint(16.0 * mu);
        muq[v] = (int32_t)(q > 127 ? 127 : (q < -127 ? -127 : q));
        if (p[v] != p[0]) uniform = false;
    }
    // Eq. 1 structure: the largest r (>= 2) for which every row of H is the row of
    // a space-time matrix [I_r (x) H0 | D (x) I_m0] with D lower bidiagonal
    int st_r = 0, st_m0 = 0, st_n0 = 0;
    for (int r = m; r >= 2 && !st_r; --r) {
        if (m % r || (n - m) % r) continue;
        const int m0 = m / r, n0 = (n - m) / r;
        bool ok = n0 > 0;
        for (int t = 0; t < r && ok; ++t)
            for (int s0 = 0; s0 < m0 && ok; ++s0) {
                const int c = t * m0 + s0, b0 = row_ptr[s0], w0 = row_ptr[s0 + 1] - b0;
                int nd0 = 0;  // data columns of the round-0 row
                while (nd0 < w0 && col_idx[b0 + nd0] < n0) ++nd0;
                const int want = nd0 + (t ? 2 : 1);
                if (w0 != nd0 + 1 || row_ptr[c + 1] - row_ptr[c] != want) {
                    ok = false;
                    break;
                }
                const int *cc = col_idx + row_ptr[c];
                for (int k = 0; k < nd0 && ok; ++k) ok = cc[k] == t * n0 + col_idx[b0 + k];
                if (!ok) break;
                if (t) ok = cc[nd0] == r * n0 + (t - 1) * m0 + s0 && cc[nd0 + 1] == r * n0 + t * m0 + s0;
                else ok = cc[nd0] == r * n0 + s0;
            }
        if (ok) {
            st_r = r;
            st_m0 = m0;
            st_n0 = n0;
        }
    }
    lbp_code code = new lbp_code_s();
    code->m = m;
    code->n = n;
    code->nnz = nnz;
    code->uniform = uniform;
    code->mu.resize(n);
    for (int v = 0; v < n; ++v) code->mu[v] = std::log((1.0 - p[v]) / p[v]);
    hipGetDevice(&code->device);
    // compact space-time offset table of the Int x.y kernel (codes with the Eq. 1 structure)
    std::vector<uint32_t> sttab;
    if (st_r && !bp_int8_build_st_table(cols.data(), m, n, st_r, st_m0, st_n0, sttab)) sttab.clear();
    size_t o_cols = 0, o_deg = align256(o_cols + cols.size() * 2), o_tab = align256(o_deg + (size_t)m),
           o_m32 = align256(o_tab + (size_t)n * 8), o_m16 = align256(o_m32 + (size_t)n * 4),
           o_mq = align256(o_m16 + (size_t)n * 4), o_t4 = align256(o_mq + (size_t)n * 4),
           o_st = align256(o_t4 + tab4.size() * 4), total = align256(o_st + sttab.size() * 4);
    hipError_t e = hipMalloc(&code->dmem, total);
    if (e != hipSuccess) {
        delete code;
        return fail(LBP_ENOMEM, std::string("lbp_code_create: hipMalloc: ") + hipGetErrorString(e));
    }
    char *b = (char *)code->dmem;
    std::vector<char> host(total, 0);
    std::memcpy(host.data() + o_cols, cols.data(), cols.size() * 2);
    std::memcpy(host.data() + o_deg, deg.data(), (size_t)m);
    std::memcpy(host.data() + o_tab, tab.data(), (size_t)n * 8);
    std::memcpy(host.data() + o_m32, mu32.data(), (size_t)n * 4);
    std::memcpy(host.data() + o_m16, mu16.data(), (size_t)n * 4);
    std::memcpy(host.data() + o_mq, muq.data(), (size_t)n * 4);
    if (wide) std::memcpy(host.data() + o_t4, tab4.data(), tab4.size() * 4);
    if (!sttab.empty()) std::memcpy(host.data() + o_st, sttab.data(), sttab.size() * 4);
    e = hipMemcpy(code->dmem, host.data(), total, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        hipFree(code->dmem);
        delete code;
        return fail(LBP_EDEVICE, std::string("lbp_code_create: hipMemcpy: ") + hipGetErrorString(e));
    }
    DevCode &dc = code->dc;
    dc.m = m;
    dc.n = n;
    dc.mw = (m + 31) / 32;
    dc.nw = (n + 31) / 32;
    dc.cn_cols = (const uint16_t *)(b + o_cols);
    dc.cn_deg = (const uint8_t *)(b + o_deg);
    dc.vn_tab = (const uint64_t *)(b + o_tab);
    dc.vn_tab4 = wide ? (const u32x4 *)(b + o_t4) : nullptr;
    dc.mu_f32 = (const float *)(b + o_m32);
    dc.mu_f16 = (const float *)(b + o_m16);
    dc.mu_q = (const int32_t *)(b + o_mq);
    dc.mu_q_uniform = uniform ? muq[0] : INT32_MIN;
    dc.st_tab = sttab.empty() ? nullptr : (const uint32_t *)(b + o_st);
    dc.st_r = st_r;
    dc.st_m0 = st_m0;
    dc.st_n0 = st_n0;
    *out = code;
    return LBP_OK;
}

static void code_release(lbp_code code) {
    if (code->refs.fetch_sub(1, std::memory_order_acq_rel) != 1) return;
    DeviceGuard g(code->device);
    hipFree(code->dmem);
    delete code;
}

void lbp_code_destroy(lbp_code code) {
    if (code) code_release(code);
}

int32_t lbp_code_rows(lbp_code code) { return code ? code->m : 0; }
int32_t lbp_code_cols(lbp_code code) { return code ? code->n : 0; }

static void free_decoder(lbp_decoder d) {
    for (auto &r : d->recs) {
        hipEventDestroy(r.a);
        hipEventDestroy(r.b);
    }
    for (auto e : d->pool) hipEventDestroy(e);
    d->recs.clear();
    d->pool.clear();
    hipFree(d->d_counters);
    hipFree(d->d_fail_list);
    hipFree(d->d_list2);
    hipFree(d->d_fail_llr);
    hipFree(d->d_stage);
    hipFree(d->d_gscratch);
    hipFree(d->d_gscratch2);
    if (d->ev_early) hipEventDestroy(d->ev_early);
    if (d->h_count) hipHostFree(d->h_count);
    hipFree(d->bl_alpha);
    hipFree(d->bl_beta);
    hipFree(d->bl_lam);
    hipFree(d->bl_ehat);
    hipFree(d->bl_shat);
    hipFree(d->bl_flipv);
    hipFree(d->bl_active);
    hipFree(d->d_muq);
    for (int c = 0; c < 2; ++c) {
        hipFree(d->pipe_counters[c]);
        hipFree(d->pipe_list[c]);
        hipFree(d->pipe_llr[c]);
        if (d->ev_bp[c]) hipEventDestroy(d->ev_bp[c]);
        if (d->ev_osd[c]) hipEventDestroy(d->ev_osd[c]);
    }
    if (d->ev_fork) hipEventDestroy(d->ev_fork);
    if (d->side) hipStreamDestroy(d->side);
    if (d->code) code_release(d->code);
    d->code = nullptr;
}

lbp_status lbp_decoder_create(lbp_code code, const lbp_params *prm, int64_t max_batch, lbp_decoder *out) {
    g_err.clear();
    if (!code || !prm || !out) return fail(LBP_EINVAL, "lbp_decoder_create: NULL argument");
    *out = nullptr;
    if (max_batch < 1 || max_batch > (int64_t)1 << 31) return fail(LBP_EINVAL, "lbp_decoder_create: 1 <= max_batch <= 2^31");
    if (prm->max_iter < 1) return fail(LBP_EINVAL, "lbp_decoder_create: max_iter must be >= 1");
    // message storage: FP32, FP16, or fixed point Int x.y (LBP_MSG_INT8 = Int3.4)
    int fx = 3, fy = 4;
    if (prm->msg & 0x100) {
        fx = (prm->msg >> 4) & 15;
        fy = prm->msg & 15;
        if ((prm->msg & ~0x1FF) != 0 || fx + fy < 1 || fx + fy > 7)
            return fail(LBP_EINVAL, "lbp_decoder_create: fixed point Int x.y needs 1 <= x + y <= 7");
    } else if (prm->msg < 0 || prm->msg > 2) {
        return fail(LBP_EINVAL, "lbp_decoder_create: unknown message format");
    }
    const int msgk = (prm->msg & 0x100) ? LBP_MSG_INT8 : prm->msg;
    if (prm->scale_mode != 0 && prm->scale_mode != 1) return fail(LBP_EINVAL, "lbp_decoder_create: unknown scale mode");
    if (prm->flip != 0 && prm->flip != 1) return fail(LBP_EINVAL, "lbp_decoder_create: unknown flip mode");
    if (prm->osd < 0 || prm->osd > 2) return fail(LBP_EINVAL, "lbp_decoder_create: unknown OSD mode");
    if (prm->lottery_skip < 0) return fail(LBP_EINVAL, "lbp_decoder_create: lottery_skip must be >= 0");
    if (prm->osd == LBP_OSD_CS && prm->osd_order < 0) return fail(LBP_EINVAL, "lbp_decoder_create: osd_order must be >= 0");
    if ((prm->lottery_rule & ~0x33) != 0 || (prm->lottery_rule & 3) > LBP_CN_WORST)
        return fail(LBP_EINVAL, "lbp_decoder_create: unknown lottery_rule");
    int k = 0;
    if (prm->scale_mode == 1) {
        if (!(prm->scale > 0.0f && prm->scale <= 1.0f)) return fail(LBP_EINVAL, "lbp_decoder_create: constant scale must be in (0,1]");
        if (msgk == LBP_MSG_INT8) {
            double kk = (double)prm->scale * 8.0;
            k = (int)std::lround(kk);
            if (std::fabs(kk - k) > 1e-6) return fail(LBP_EINVAL, "lbp_decoder_create: Int3.4 constant scale must be k/8");
        }
    }
    if (prm->osd == LBP_OSD_CS && !code->uniform)
        return fail(LBP_EUNSUPPORTED, "lbp_decoder_create: OSD-CS needs a uniform prior (Hamming-weight cost)");
    DeviceGuard g(code->device);
    lbp_decoder d = new lbp_decoder_s();
    d->code = code;
    code->refs.fetch_add(1, std::memory_order_relaxed);
    d->prm = *prm;
    d->msgk = msgk;
    d->dc = code->dc;
    d->max_batch = max_batch;
    BpParams &bp = d->bp;
    bp.qmax = (1 << (fx + fy)) - 1;
    bp.max_iter = prm->max_iter;
    bp.scale_mode = prm->scale_mode;
    bp.scale_f = prm->scale;
    bp.scale_k = k;
    bp.lottery = prm->lottery ? 1 : 0;
    bp.skip = prm->lottery_skip;
    bp.flip = prm->flip;
    bp.osd = prm->osd;
    bp.rule = prm->lottery_rule;
    bp.seed = prm->seed;

    int dev = code->device, ncu = 0, lds_block = 0;
    auto cleanup_fail = [&](lbp_status s, const std::string &msg) {
        free_decoder(d);
        delete d;
        return fail(s, msg);
    };
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_block, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return cleanup_fail(LBP_EDEVICE, "lbp_decoder_create: device query failed");
    // ---- BP launch shape: the waves-per-block choice with the most resident waves per CU
    d->int8_slots = msgk == LBP_MSG_INT8 ? bp_int8_slots(code->m, code->n) : 0;
    d->wave_bytes = d->int8_slots ? bp_int8_wave_bytes(code->m, code->n) : bp_wave_bytes(msgk, code->m, code->n);
    // LBP_INT8_TABLE=1 / 2 (read here) selects the compact space-time offset table in LDS /
    // global memory for codes with the Eq. 1 structure (same results; for measurements)
    if (d->int8_slots && code->dc.st_tab && (d->int8_slots == 8 || d->int8_slots >= 14)) {
        const char *te = std::getenv("LBP_INT8_TABLE");
        const int tv = te ? std::atoi(te) : 0;
        if (tv == 1 || tv == 2) d->int8_table = tv;
    }
    d->table_bytes = d->int8_slots ? bp_int8_table_bytes(d->int8_table, d->int8_slots, code->dc.st_m0) : 0;
    if (d->table_bytes + d->wave_bytes > lds_block)
        return cleanup_fail(LBP_EUNSUPPORTED, "lbp_decoder_create: per-shot state exceeds LDS");
    // A workgroup per shot when a shot per wave would leave a CU with fewer than 32
    // waves (the per-shot state fits fewer than 32 times in LDS): the smallest
    // group of 2..8 waves that brings the CU to 32, or 16 when only one shot fits.
    // Measured best or within 10 % on BB144 FP16/FP32, BB288 and surface d=13..27
    // in Int3.4; larger groups cost more in barriers than they gain in waves once
    // they leave fewer shots per CU.  LBP_BP_GROUP=g (read here) forces groups of
    // g waves, for tests.
    const bool wide = code->dc.vn_tab4 != nullptr;
    int group = 1;
    if (!d->int8_slots) {
        const int per_cu = (lds_block - 64) / d->wave_bytes;
        const char *force = std::getenv("LBP_BP_GROUP");
        const int fg = force ? std::atoi(force) : 0;
        if (fg > 0) {
            group = fg >= 16 ? 16 : fg >= 8 ? 8 : fg >= 4 ? 4 : fg >= 2 ? 2 : 1;
        } else if (per_cu < 32) {
            group = 2;
            while (group < 8 && per_cu * group < 32) group *= 2;
            if (per_cu <= 1) group = 16;
        }
    }
    d->group = group > 1;
    int best_waves = 0;
    if (d->group) {
        int bpc = 0;
        if (bp_max_blocks_per_cu(msgk, wide, true, group, d->wave_bytes, &bpc) == hipSuccess && bpc > 0) {
            best_waves = bpc * group;
            d->wpb = group;
            d->bp_blocks = bpc * ncu;
        }
    } else {
        for (int wpb : {16, 15, 14, 13, 12, 11, 10, 9, 8, 7, 6, 5, 4, 3, 2, 1}) {
            int lds = d->table_bytes + d->wave_bytes * wpb;
            if (lds + 64 > lds_block) continue;  // plus the kernels' static LDS
            int bpc = 0;
            hipError_t oe = d->int8_slots ? bp_int8_max_blocks_per_cu(d->int8_slots, d->int8_table, wpb, lds, &bpc)
                                          : bp_max_blocks_per_cu(msgk, wide, false, wpb, lds, &bpc);
            if (oe != hipSuccess) continue;
            // most resident waves; among equals a multiple of 4 waves per block, whose
            // waves spread evenly over the CU's four SIMDs (10-wave blocks of a 20-wave
            // shape ran 15-25 % slower than 4-wave ones on BB144 code capacity)
            const bool even = wpb % 4 == 0, best_even = d->wpb % 4 == 0;
            if (bpc * wpb > best_waves || (bpc * wpb == best_waves && even && !best_even)) {
                best_waves = bpc * wpb;
                d->wpb = wpb;
                d->bp_blocks = bpc * ncu;
            }
        }
    }
    if (best_waves == 0) return cleanup_fail(LBP_EDEVICE, "lbp_decoder_create: no feasible BP launch shape");
    // ---- OSD workspace
    d->llr_bytes = (int64_t)code->n * (d->int8_slots ? 2 : 8);
    d->fail_cap = prm->osd ? std::min<int64_t>(max_batch, std::max<int64_t>(1024, ((int64_t)256 << 20) / d->llr_bytes))
                           : 0;
    // the OSD kernel also holds a little static LDS (block-wide reductions).  Codes
    // with < 1024 checks keep G in registers, two rows per lane unless
    // LBP_OSD_ROWS_PER_LANE=1 (read here) asks for one, for tests.
    const char *rpl_env = std::getenv("LBP_OSD_ROWS_PER_LANE");
    const int rpl = rpl_env && std::atoi(rpl_env) == 1 ? 1 : 2;
    d->osd_lds_pairs = osd_block_bytes(code->m, code->n, lds_block - 1024, rpl, 0, &d->osd_variant, &d->mws,
                                       &d->sort_p, &d->osd_threads);
    d->osd_lds = d->int8_slots ? osd_block_bytes(code->m, code->n, lds_block - 1024, rpl, 1, &d->osd_variant, &d->mws,
                                                 &d->sort_p, &d->osd_threads)
                               : d->osd_lds_pairs;
    if (d->osd_lds_pairs > lds_block - 1024)
        return cleanup_fail(LBP_EUNSUPPORTED, "lbp_decoder_create: OSD sort does not fit LDS");
    int obpc = 0;
    if (prm->osd && (osd_max_blocks_per_cu(d->osd_variant, d->osd_threads, d->osd_lds, &obpc) != hipSuccess || obpc < 1))
        return cleanup_fail(LBP_EDEVICE, "lbp_decoder_create: no feasible OSD launch shape");
    d->osd_blocks = ncu * std::max(1, obpc);
    {
        // An OSD grid alongside the Int x.y kernel's BP grid fills BP's tail (BB144 r=12,
        // 10^6 shots: 31.8 -> 29.8 ms per decode), where BP's blocks leave no room for an
        // OSD block in a CU's LDS: the side grid's blocks then start as BP's blocks leave.
        // Where one fits beside them (small codes), the side grid's blocks would be
        // resident from the start, polling the counters that BP claims its shots with (a
        // 72-check code at p = 0.06: 70 ms -> 3.6 s per 2^20 shots), so OSD runs after BP
        // there.  LBP_EARLY_OSD=0 (read here) turns it off everywhere.
        int lds_cu = 0;
        if (hipDeviceGetAttribute(&lds_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, dev) != hipSuccess)
            lds_cu = lds_block;
        const int64_t bp_lds_cu = (int64_t)(d->bp_blocks / std::max(1, ncu)) *
                                  ((int64_t)d->table_bytes + (int64_t)d->wave_bytes * d->wpb + 64);
        const bool osd_waits_for_bp = (int64_t)lds_cu - bp_lds_cu < (int64_t)d->osd_lds;
        const char *eo = std::getenv("LBP_EARLY_OSD");
        d->early_osd = d->int8_slots && prm->osd && osd_waits_for_bp && !(eo && std::atoi(eo) == 0);
    }
    hipError_t e;
#define ALLOC(ptr, bytes)                                                                                     \
    do {                                                                                                      \
        d->dev_bytes += (int64_t)align256((bytes) > 0 ? (bytes) : 16);                                          \
        e = hipMalloc((void **)&(ptr), (bytes) > 0 ? (bytes) : 16);                                            \
        if (e != hipSuccess) return cleanup_fail(LBP_ENOMEM, std::string("lbp_decoder_create: hipMalloc: ") + \
                                                                 hipGetErrorString(e));                        \
    } while (0)
    ALLOC(d->d_counters, 64);
    if (msgk == LBP_MSG_INT8 && !(fx == 3 && fy == 4)) {
        // this format's prior: 2^y mu rounded to nearest even, saturated to +-qmax
        std::vector<int32_t> muq(code->n);
        bool uni = true;
        for (int v = 0; v < code->n; ++v) {
            double q = std::nearbyint(std::ldexp(code->mu[v], fy));
            muq[v] = (int32_t)(q > bp.qmax ? bp.qmax : (q < -bp.qmax ? -bp.qmax : q));
            uni = uni && muq[v] == muq[0];
        }
        ALLOC(d->d_muq, (size_t)code->n * 4);
        e = hipMemcpy(d->d_muq, muq.data(), (size_t)code->n * 4, hipMemcpyHostToDevice);
        if (e != hipSuccess) return cleanup_fail(LBP_EDEVICE, "lbp_decoder_create: hipMemcpy of the prior failed");
        d->dc.mu_q = d->d_muq;
        d->dc.mu_q_uniform = uni ? muq[0] : INT32_MIN;
    }
    // the float kernels stage lambda of the last iteration per wave; the Int x.y
    // check-centric kernel reads it from LDS once the shot is done
    if (!d->int8_slots) ALLOC(d->d_stage, (size_t)d->bp_blocks * d->wpb * code->n * 8);
    if (prm->osd) {
        ALLOC(d->d_fail_list, (size_t)max_batch * 4);
        ALLOC(d->d_list2, (size_t)max_batch * 4);
        ALLOC(d->d_fail_llr, (size_t)d->fail_cap * d->llr_bytes);
        ALLOC(d->d_gscratch, (size_t)d->osd_blocks * osd_scratch_bytes(d->osd_variant, code->m, code->n, d->mws, d->sort_p,
                                                                       prm->osd == LBP_OSD_CS));
    }
#undef ALLOC
    e = hipHostMalloc((void **)&d->h_count, 64, hipHostMallocDefault);
    if (e != hipSuccess) return cleanup_fail(LBP_ENOMEM, "lbp_decoder_create: hipHostMalloc failed");
    // set-up of lbp_decode_noalloc on this device (its scratch address), while the device is current
    if (!scratch_on(dev)) return cleanup_fail(LBP_EDEVICE, "lbp_decoder_create: " + g_err);
    *out = d;
    return LBP_OK;
}

void lbp_decoder_destroy(lbp_decoder d) {
    if (!d) return;
    DeviceGuard g(d->code->device);
    free_decoder(d);
    delete d;
}

int64_t lbp_decoder_osd_capacity(lbp_decoder d) { return d ? d->fail_cap : 0; }

lbp_status lbp_decoder_set_osd_capacity(lbp_decoder d, int64_t cap) {
    if (!d) return fail(LBP_EINVAL, "lbp_decoder_set_osd_capacity: NULL decoder");
    if (cap < 1 || cap > d->fail_cap) return fail(LBP_EINVAL, "lbp_decoder_set_osd_capacity: 1 <= cap <= current capacity");
    d->fail_cap = cap;
    d->fail_cap_pinned = true;
    return LBP_OK;
}

// Device buffers one decode pass works in: the decoder's own workspace, or the
// library's static scratch (lbp_decode_noalloc).
struct PassBufs {
    uint32_t *counters;     // [16]: next work item, failed shots, ...
    int32_t *fail_list;     // [n_work]
    float *fail_llr;        // [fail_cap] staged lambda, llr_bytes each
    int64_t fail_cap;
    float *stage;           // float kernels: [launched BP waves or blocks][2n]
    int max_bp_blocks;      // BP blocks the stage rows cover
    uint32_t *gscratch;     // [osd_blocks] OSD per-block scratch
    int osd_blocks;
    bool timing;            // record the decoder's timing events (they may be created here)
};

static PassBufs own_bufs(lbp_decoder d) {
    return PassBufs{d->d_counters, d->d_fail_list, d->d_fail_llr, d->fail_cap, d->d_stage, d->bp_blocks,
                    d->d_gscratch, d->osd_blocks, d->timing};
}

// Algorithm 1 (with Algorithm 3) over n_work shots; the failures are listed and
// their lambda staged in w for bp_pass's OSD.
static lbp_status bp_pass(lbp_decoder d, const PassBufs &w, int64_t n_work, const int32_t *work_list,
                          uint64_t first_shot_id, const uint64_t *keys, const uint32_t *syn, uint32_t *corr,
                          uint8_t *flags, int32_t *iters, float *llr, hipStream_t s, bool fork_side = false,
                          int *grid_out = nullptr) {
    HIPCHK(launch_reset(w.counters, 16, s));
    if (fork_side) {
        // the grid alongside BP tells published list entries from unwritten ones
        HIPCHK(launch_fill_i32(w.fail_list, -1, std::min<int64_t>(n_work, w.fail_cap), s));
        HIPCHK(hipEventRecord(d->ev_fork, s));
        HIPCHK(hipStreamWaitEvent(d->side, d->ev_fork, 0));
    }
    BpArgs a{};
    a.code = d->dc;
    a.prm = d->bp;
    a.n_work = n_work;
    a.first_shot_id = first_shot_id;
    a.shot_keys = keys;
    a.work_list = work_list;
    a.synd = syn;
    a.corr = corr;
    a.flags = flags;
    a.iters = iters;
    a.llr_out = llr;
    a.counters = w.counters;
    a.fail_list = w.fail_list;
    a.fail_llr = w.fail_llr;
    a.fail_q = (int16_t *)w.fail_llr;
    a.fail_cap = w.fail_cap;
    a.stage = w.stage;
    a.wave_bytes = d->wave_bytes;
    a.group = d->group;
    const int shots_per_block = d->group ? 1 : d->wpb;
    int64_t need_blocks = (n_work + shots_per_block - 1) / shots_per_block;
    int blocks = (int)std::min<int64_t>(std::min(d->bp_blocks, w.max_bp_blocks), std::max<int64_t>(1, need_blocks));
    if (grid_out) *grid_out = blocks;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (w.timing && (e0 = take_event(d)) && (e1 = take_event(d))) HIPCHK(hipEventRecord(e0, s));
    HIPCHK(d->int8_slots ? launch_bp_int8(d->int8_slots, d->int8_table, a, blocks, d->wpb, s)
                         : launch_bp(d->msgk, a, blocks, d->wpb, s));
    if (e1) {
        HIPCHK(hipEventRecord(e1, s));
        d->recs.push_back({e0, e1, 0});
    }
    return LBP_OK;
}

// Algorithm 2 (or OSD-CS) on the failures a bp_pass listed in w.
static lbp_status osd_pass(lbp_decoder d, const PassBufs &w, const uint32_t *syn, uint32_t *corr, uint8_t *flags,
                           hipStream_t s, int claim_mode = 0, int bp_grid = 0, uint32_t *gscratch = nullptr) {
    if (d->prm.osd) {
        OsdArgs o = osd_args(d);
        o.synd = syn;
        o.corr = corr;
        o.flags = flags;
        o.counters = w.counters;
        o.fail_list = w.fail_list;
        o.fail_llr = w.fail_llr;
        o.fail_cap = w.fail_cap;
        o.gscratch = gscratch ? gscratch : w.gscratch;
        o.claim_mode = claim_mode;
        o.bp_grid = bp_grid;
        o.claim = w.counters + 2;
        hipEvent_t f0 = nullptr, f1 = nullptr;
        if (w.timing && (f0 = take_event(d)) && (f1 = take_event(d))) HIPCHK(hipEventRecord(f0, s));
        HIPCHK(launch_osd(o, d->osd_variant, w.osd_blocks, d->osd_threads, d->osd_lds, s));
        if (f1) {
            HIPCHK(hipEventRecord(f1, s));
            d->recs.push_back({f0, f1, 1});
        }
    }
    return LBP_OK;
}

static lbp_status early_prepare(lbp_decoder d);
constexpr int64_t kEarlyOsdMinShots = 65536;

// BP, then OSD.  With early_osd (Int x.y kernel), a second OSD grid on the side
// stream takes failures while BP runs: BP's grid holds every CU's LDS until its
// last shots, so that grid's blocks start in BP's tail and fill it; the launch
// after BP takes what is left (the two claim list positions from one counter).
static lbp_status run_pass(lbp_decoder d, const PassBufs &w, int64_t n_work, const int32_t *work_list,
                           uint64_t first_shot_id, const uint64_t *keys, const uint32_t *syn, uint32_t *corr,
                           uint8_t *flags, int32_t *iters, float *llr, hipStream_t s) {
    // (only for batches that keep BP's grid busy long enough to have a tail worth filling)
    const bool early = d->early_osd && n_work >= kEarlyOsdMinShots && w.gscratch == d->d_gscratch &&
                       early_prepare(d) == LBP_OK;
    int grid = 0;
    lbp_status st = bp_pass(d, w, n_work, work_list, first_shot_id, keys, syn, corr, flags, iters, llr, s, early, &grid);
    if (st != LBP_OK) return st;
    if (!early) return osd_pass(d, w, syn, corr, flags, s);
    st = osd_pass(d, w, syn, corr, flags, d->side, 1, grid, d->d_gscratch2);
    if (st != LBP_OK) return st;
    HIPCHK(hipEventRecord(d->ev_early, d->side));
    st = osd_pass(d, w, syn, corr, flags, s, 2, grid);
    if (st != LBP_OK) return st;
    HIPCHK(hipStreamWaitEvent(s, d->ev_early, 0));
    return LBP_OK;
}

// Chunks of a pipelined decode (LBP_PIPELINE_CHUNKS, read at each call: 0 or 1 =
// one pass); only batches of at least 2^17 shots with OSD are split.
static int pipeline_chunks(lbp_decoder d, int64_t n_shots) {
    if (!d->prm.osd || n_shots < ((int64_t)1 << 17)) return 1;
    const char *e = std::getenv("LBP_PIPELINE_CHUNKS");
    const int k = e ? std::atoi(e) : 0;
    return k >= 2 && k <= 64 ? k : 1;
}

// Workspaces and the side stream of a pipelined decode with chunks of `chunk`
// shots (grown, never shrunk).
static lbp_status pipeline_prepare(lbp_decoder d, int64_t chunk) {
    if (!d->side) {
        HIPCHK(hipStreamCreateWithFlags(&d->side, hipStreamNonBlocking));
        HIPCHK(hipEventCreateWithFlags(&d->ev_fork, hipEventDisableTiming));
        for (int c = 0; c < 2; ++c) {
            HIPCHK(hipEventCreateWithFlags(&d->ev_bp[c], hipEventDisableTiming));
            HIPCHK(hipEventCreateWithFlags(&d->ev_osd[c], hipEventDisableTiming));
        }
    }
    if (chunk <= d->pipe_chunk) return LBP_OK;
    for (int c = 0; c < 2; ++c) {
        hipFree(d->pipe_counters[c]);
        hipFree(d->pipe_list[c]);
        hipFree(d->pipe_llr[c]);
        d->pipe_counters[c] = nullptr;
        d->pipe_list[c] = nullptr;
        d->pipe_llr[c] = nullptr;
    }
    d->pipe_chunk = 0;
    for (int c = 0; c < 2; ++c) {
        if (hipMalloc((void **)&d->pipe_counters[c], 64) != hipSuccess ||
            hipMalloc((void **)&d->pipe_list[c], (size_t)chunk * 4) != hipSuccess ||
            hipMalloc((void **)&d->pipe_llr[c], (size_t)chunk * d->llr_bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(LBP_ENOMEM, "pipelined decode: workspace allocation failed");
        }
    }
    d->pipe_chunk = chunk;
    return LBP_OK;
}

// The side stream, its events and the second OSD scratch of the early grid.
static lbp_status early_prepare(lbp_decoder d) {
    lbp_status st = pipeline_prepare(d, 0);
    if (st != LBP_OK) return st;
    if (!d->ev_early) HIPCHK(hipEventCreateWithFlags(&d->ev_early, hipEventDisableTiming));
    if (!d->d_gscratch2) {
        const size_t b = (size_t)d->osd_blocks * osd_scratch_bytes(d->osd_variant, d->code->m, d->code->n, d->mws,
                                                                   d->sort_p, d->prm.osd == LBP_OSD_CS);
        if (hipMalloc((void **)&d->d_gscratch2, b > 0 ? b : 16) != hipSuccess) {
            (void)hipGetLastError();
            d->d_gscratch2 = nullptr;
            return fail(LBP_ENOMEM, "OSD alongside BP: scratch allocation failed");
        }
        d->dev_bytes += (int64_t)align256(b > 0 ? b : 16);
    }
    return LBP_OK;
}

// BP of chunk i + 1 overlaps OSD of chunk i: BP runs in order on s, each chunk's
// OSD on the side stream after that chunk's BP; a chunk reuses the workspace of
// chunk i - 2 only after that chunk's OSD.  The side stream joins s at the end.
static lbp_status decode_pipelined(lbp_decoder d, int k, int64_t n_shots, uint64_t first_shot_id,
                                   const uint64_t *keys, const uint32_t *syndromes, uint32_t *corrections,
                                   uint8_t *flags, int32_t *iters, float *llr_out, hipStream_t s) {
    const int64_t chunk = (n_shots + k - 1) / k;
    lbp_status st = pipeline_prepare(d, chunk);
    if (st != LBP_OK) return st;
    const size_t mw = d->code->dc.mw, nw = d->code->dc.nw, n = d->code->n;
    HIPCHK(hipEventRecord(d->ev_fork, s));
    HIPCHK(hipStreamWaitEvent(d->side, d->ev_fork, 0));
    for (int i = 0; i * chunk < n_shots; ++i) {
        const int c = i & 1;
        const int64_t off = (int64_t)i * chunk, cnt = std::min(chunk, n_shots - off);
        PassBufs w = own_bufs(d);
        w.counters = d->pipe_counters[c];
        w.fail_list = d->pipe_list[c];
        w.fail_llr = d->pipe_llr[c];
        w.fail_cap = chunk;
        if (i >= 2) HIPCHK(hipStreamWaitEvent(s, d->ev_osd[c], 0));
        const uint32_t *syn = syndromes + (size_t)off * mw;
        uint32_t *corr = corrections + (size_t)off * nw;
        st = bp_pass(d, w, cnt, nullptr, first_shot_id + (keys ? 0 : (uint64_t)off), keys ? keys + 2 * off : nullptr, syn,
                     corr, flags + off, iters ? iters + off : nullptr, llr_out ? llr_out + (size_t)off * n : nullptr, s);
        if (st != LBP_OK) return st;
        HIPCHK(hipEventRecord(d->ev_bp[c], s));
        HIPCHK(hipStreamWaitEvent(d->side, d->ev_bp[c], 0));
        st = osd_pass(d, w, syn, corr, flags + off, d->side);
        if (st != LBP_OK) return st;
        HIPCHK(hipEventRecord(d->ev_osd[c], d->side));
    }
    HIPCHK(hipEventRecord(d->ev_fork, d->side));
    HIPCHK(hipStreamWaitEvent(s, d->ev_fork, 0));
    return LBP_OK;
}

lbp_status lbp_decoder_set_timing(lbp_decoder d, int32_t enable) {
    if (!d) return fail(LBP_EINVAL, "lbp_decoder_set_timing: NULL decoder");
    d->timing = enable != 0;
    return LBP_OK;
}

lbp_status lbp_decoder_kernel_times(lbp_decoder d, double *bp_ms, int64_t *bp_launches, double *osd_ms,
                                    int64_t *osd_launches) {
    if (!d) return fail(LBP_EINVAL, "lbp_decoder_kernel_times: NULL decoder");
    DeviceGuard g(d->code->device);
    double t[2] = {0, 0};
    int64_t c[2] = {0, 0};
    for (auto &r : d->recs) {
        HIPCHK(hipEventSynchronize(r.b));
        float ms = 0.f;
        HIPCHK(hipEventElapsedTime(&ms, r.a, r.b));
        t[r.kind] += ms;
        c[r.kind] += 1;
        d->pool.push_back(r.a);
        d->pool.push_back(r.b);
    }
    d->recs.clear();
    if (bp_ms) *bp_ms = t[0];
    if (bp_launches) *bp_launches = c[0];
    if (osd_ms) *osd_ms = t[1];
    if (osd_launches) *osd_launches = c[1];
    return LBP_OK;
}

// Enlarge the OSD staging of failed shots' lambda to `want` shots, bounded by
// max_batch and a quarter of the free device memory; on any failure the old
// buffer stays (the caller then needs more passes, never wrong results).  The
// stream is idle here (the caller has synchronized it).
static void grow_fail_cap(lbp_decoder d, int64_t want) {
    const int64_t per = d->llr_bytes;
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) return;
    const int64_t cap = std::min<int64_t>(std::min<int64_t>(want, d->max_batch), (int64_t)(free_b / 4) / per);
    if (cap <= d->fail_cap) return;
    float *nb = nullptr;
    if (hipMalloc((void **)&nb, (size_t)cap * per) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    hipFree(d->d_fail_llr);
    d->d_fail_llr = nb;
    d->dev_bytes += (int64_t)align256((size_t)cap * per) - (int64_t)align256((size_t)d->fail_cap * per);
    d->fail_cap = cap;
}

static lbp_status decode_impl(const char *who, lbp_decoder d, int64_t n_shots, uint64_t first_shot_id,
                              const uint64_t *keys, const uint32_t *syndromes, uint32_t *corrections, uint8_t *flags,
                              int32_t *iters, float *llr_out, void *stream) {
    g_err.clear();
    if (!d) return fail(LBP_EINVAL, std::string(who) + ": NULL decoder");
    if (n_shots < 0 || n_shots > d->max_batch) return fail(LBP_EINVAL, std::string(who) + ": 0 <= n_shots <= max_batch");
    if (n_shots == 0) return LBP_OK;
    if (!syndromes || !corrections || !flags) return fail(LBP_EINVAL, std::string(who) + ": NULL buffer");
    DeviceGuard g(d->code->device);
    hipStream_t s = (hipStream_t)stream;
    const int k = pipeline_chunks(d, n_shots);
    if (k > 1) return decode_pipelined(d, k, n_shots, first_shot_id, keys, syndromes, corrections, flags, iters,
                                       llr_out, s);
    lbp_status st = run_pass(d, own_bufs(d), n_shots, nullptr, first_shot_id, keys, syndromes, corrections, flags,
                             iters, llr_out, s);
    if (st != LBP_OK || !d->prm.osd || n_shots <= d->fail_cap) return st;
    // More shots may have failed BP than one OSD pass can stage: re-decode the
    // overflow (BP is deterministic per shot) and run OSD on it, until done.
    for (;;) {
        HIPCHK(hipMemcpyAsync(d->h_count, d->d_counters + 1, 4, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        const int64_t total = d->h_count[0];
        if (total <= d->fail_cap) return LBP_OK;
        // entries [0, staged) of the failure list went through OSD in the pass that just ran
        const int64_t staged = d->fail_cap;
        const int64_t rest = total - staged;
        // grow the staging (once) so that the overflow takes one more pass, not
        // rest / capacity passes that each re-decode everything still pending
        if (!d->fail_cap_pinned && rest > d->fail_cap) grow_fail_cap(d, rest);
        HIPCHK(launch_gather_list(d->d_counters, d->d_fail_list, staged, d->d_list2, rest, s));
        st = run_pass(d, own_bufs(d), rest, d->d_list2, first_shot_id, keys, syndromes, corrections, flags, iters,
                      llr_out, s);
        if (st != LBP_OK) return st;
    }
}

lbp_status lbp_decode(lbp_decoder d, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                      uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out, void *stream) {
    return decode_impl("lbp_decode", d, n_shots, first_shot_id, nullptr, syndromes, corrections, flags, iters, llr_out,
                       stream);
}

lbp_status lbp_decode_keyed(lbp_decoder d, int64_t n_shots, const uint64_t *shot_keys, const uint32_t *syndromes,
                            uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out, void *stream) {
    if (n_shots > 0 && !shot_keys) return fail(LBP_EINVAL, "lbp_decode_keyed: NULL shot_keys");
    return decode_impl("lbp_decode_keyed", d, n_shots, 0, shot_keys, syndromes, corrections, flags, iters, llr_out,
                       stream);
}

// Scratch layout of a no-allocation decode of n shots, in bytes from the start
// of the array (0 when it does not fit).  Every shot gets failure staging, so a
// pass never overflows and needs no second pass or host synchronisation.
static size_t noalloc_layout(lbp_decoder d, int64_t n, PassBufs *w, unsigned char *base) {
    lbp_code C = d->code;
    const size_t cap = LBP_NOALLOC_SCRATCH_BYTES;
    size_t off = 0;
    const size_t o_cnt = off;
    off += 256;
    const size_t o_list = off;
    off += align256((size_t)n * 4);
    const size_t o_llr = off;
    if (d->prm.osd) off += align256((size_t)n * (size_t)d->llr_bytes);
    // BP blocks the launch uses; the float kernels stage lambda per wave (or per block in groups)
    const int64_t per_block_shots = d->group ? 1 : d->wpb;
    int blocks = (int)std::min<int64_t>(d->bp_blocks, std::max<int64_t>(1, (n + per_block_shots - 1) / per_block_shots));
    const size_t stage_row = (size_t)C->n * 8 * (d->group ? 1 : d->wpb);
    const size_t o_stage = off;
    if (!d->int8_slots) {
        if (off > cap) return 0;
        blocks = (int)std::min<size_t>((size_t)blocks, (cap - off) / stage_row);
        if (blocks < 1) return 0;
        off += align256((size_t)blocks * stage_row);
    }
    const size_t o_g = off;
    int ob = 0;
    if (d->prm.osd) {
        const size_t per = align256(osd_scratch_bytes(d->osd_variant, C->m, C->n, d->mws, d->sort_p,
                                                      d->prm.osd == LBP_OSD_CS));
        if (off > cap) return 0;
        ob = (int)std::min<int64_t>(std::min<int64_t>(d->osd_blocks, std::max<int64_t>(1, n)),
                                    (int64_t)((cap - off) / per));
        if (ob < 1) return 0;
        off += (size_t)ob * per;
    }
    if (off > cap) return 0;
    if (w) {
        *w = PassBufs{(uint32_t *)(base + o_cnt), (int32_t *)(base + o_list), (float *)(base + o_llr), n,
                      d->int8_slots ? nullptr : (float *)(base + o_stage), blocks, (uint32_t *)(base + o_g), ob,
                      false};
    }
    return off;
}

lbp_status lbp_decode_noalloc(lbp_decoder d, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                              uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out, void *stream) {
    g_err.clear();
    if (!d) return fail(LBP_EINVAL, "lbp_decode_noalloc: NULL decoder");
    if (n_shots < 0) return fail(LBP_EINVAL, "lbp_decode_noalloc: n_shots < 0");
    if (n_shots == 0) return LBP_OK;
    if (!syndromes || !corrections || !flags) return fail(LBP_EINVAL, "lbp_decode_noalloc: NULL buffer");
    if (n_shots > (int64_t)1 << 31) return fail(LBP_EINVAL, "lbp_decode_noalloc: n_shots > 2^31");
    if (!noalloc_layout(d, n_shots, nullptr, nullptr)) {
        int64_t lo = 0, hi = n_shots;  // largest batch that fits, for the message
        while (lo + 1 < hi) {
            const int64_t mid = lo + (hi - lo) / 2;
            (noalloc_layout(d, mid, nullptr, nullptr) ? lo : hi) = mid;
        }
        return fail(LBP_EINVAL, "lbp_decode_noalloc: " + std::to_string(n_shots) + " shots exceed the " +
                                    std::to_string(LBP_NOALLOC_SCRATCH_BYTES >> 20) +
                                    " MiB static scratch; at most " + std::to_string(lo) +
                                    " shots of this code and format fit one call");
    }
    DeviceGuard g(d->code->device);
    unsigned char *base = (unsigned char *)scratch_on(d->code->device);
    if (!base) return fail(LBP_EDEVICE, "lbp_decode_noalloc: " + g_err);
    PassBufs w{};
    noalloc_layout(d, n_shots, &w, base);
    return run_pass(d, w, n_shots, nullptr, first_shot_id, nullptr, syndromes, corrections, flags, iters, llr_out,
                    (hipStream_t)stream);
}

lbp_status lbp_decode_baseline(lbp_decoder d, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                               uint32_t *corrections, uint8_t *flags, int32_t *iters, void *stream) {
    g_err.clear();
    if (!d) return fail(LBP_EINVAL, "lbp_decode_baseline: NULL decoder");
    if (n_shots < 0 || n_shots > d->max_batch) return fail(LBP_EINVAL, "lbp_decode_baseline: 0 <= n_shots <= max_batch");
    if (d->msgk == LBP_MSG_INT8)
        return fail(LBP_EUNSUPPORTED, "lbp_decode_baseline: FP32 or FP16 message storage only");
    if (n_shots == 0) return LBP_OK;
    if (!syndromes || !corrections || !flags) return fail(LBP_EINVAL, "lbp_decode_baseline: NULL buffer");
    DeviceGuard g(d->code->device);
    hipStream_t s = (hipStream_t)stream;
    lbp_code C = d->code;
    const size_t slots = (size_t)C->m * DEG;
    if (d->bl_cap < n_shots) {
        HIPCHK(hipStreamSynchronize(s));
        hipFree(d->bl_alpha); hipFree(d->bl_beta); hipFree(d->bl_lam); hipFree(d->bl_ehat);
        hipFree(d->bl_shat); hipFree(d->bl_flipv); hipFree(d->bl_active);
        d->bl_alpha = d->bl_beta = nullptr; d->bl_lam = nullptr; d->bl_ehat = d->bl_shat = nullptr;
        d->bl_flipv = nullptr; d->bl_active = nullptr;
        d->bl_cap = 0;
        const size_t S = (size_t)n_shots;
        HIPCHK(hipMalloc((void **)&d->bl_alpha, S * slots * 4));
        HIPCHK(hipMalloc((void **)&d->bl_beta, S * slots * 4));
        HIPCHK(hipMalloc((void **)&d->bl_lam, S * C->n * 8));  // hi and lo floats
        HIPCHK(hipMalloc((void **)&d->bl_ehat, S * C->dc.nw * 4));
        HIPCHK(hipMalloc((void **)&d->bl_shat, S * 2 * C->dc.mw * 4));
        HIPCHK(hipMalloc((void **)&d->bl_flipv, S * 4));
        HIPCHK(hipMalloc((void **)&d->bl_active, S));
        d->bl_cap = n_shots;
    }
    BlArgs a{};
    a.code = d->dc;
    a.prm = d->bp;
    a.msg = d->msgk;
    a.shots = n_shots;
    a.first_shot_id = first_shot_id;
    a.synd = syndromes;
    a.corr = corrections;
    a.flags = flags;
    a.iters = iters;
    a.alpha = d->bl_alpha;
    a.beta = d->bl_beta;
    a.lam = d->bl_lam;
    a.ehat = d->bl_ehat;
    a.shat = d->bl_shat;
    a.flipv = d->bl_flipv;
    a.active = d->bl_active;
    a.counters = d->d_counters;
    a.fail_list = d->d_fail_list;
    HIPCHK(launch_reset(d->d_counters, 16, s));
    HIPCHK(baseline_init(a, s));
    for (int i = 0; i < d->prm.max_iter; ++i) {
        HIPCHK(launch_reset(d->d_counters, 1, s));
        HIPCHK(baseline_iteration(a, i, s));
        if ((i & 3) == 3 && i + 1 < d->prm.max_iter) {  // stop launching once every shot has finished
            HIPCHK(hipMemcpyAsync(d->h_count, d->d_counters, 4, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            if (d->h_count[0] == 0) break;
        }
    }
    if (!d->prm.osd) return LBP_OK;
    HIPCHK(hipMemcpyAsync(d->h_count, d->d_counters + 1, 4, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const int64_t total = d->h_count[0];
    for (int64_t from = 0; from < total; from += d->fail_cap) {
        const int64_t cnt = std::min<int64_t>(d->fail_cap, total - from);
        uint32_t *oc = d->d_counters + 8;
        HIPCHK(baseline_stage(a, from, cnt, d->d_fail_llr, oc, s));
        OsdArgs o = osd_args(d);
        o.synd = syndromes;
        o.corr = corrections;
        o.flags = flags;
        o.counters = oc;
        o.fail_list = d->d_fail_list + from;
        o.fail_llr = d->d_fail_llr;
        o.fail_cap = d->fail_cap;
        o.gscratch = d->d_gscratch;
        o.has_lo = 1;     // the comparison path stages lambda as an fp32 (hi, lo) pair
        o.llr_i16 = 0;
        HIPCHK(launch_osd(o, d->osd_variant, d->osd_blocks, d->osd_threads, d->osd_lds_pairs, s));
    }
    return LBP_OK;
}

lbp_status lbp_decoder_shape(lbp_decoder d, int32_t *bp_waves_per_block, int32_t *bp_blocks, int32_t *bp_group,
                             int32_t *osd_variant, int32_t *osd_threads, int32_t *osd_blocks) {
    if (!d) return fail(LBP_EINVAL, "lbp_decoder_shape: NULL decoder");
    if (bp_waves_per_block) *bp_waves_per_block = d->wpb;
    if (bp_blocks) *bp_blocks = d->bp_blocks;
    if (bp_group) *bp_group = d->group ? d->wpb : 1;
    if (osd_variant) *osd_variant = d->osd_variant;
    if (osd_threads) *osd_threads = d->osd_threads;
    if (osd_blocks) *osd_blocks = d->osd_blocks;
    return LBP_OK;
}

int64_t lbp_decoder_device_bytes(lbp_decoder d) { return d ? d->dev_bytes : 0; }
int64_t lbp_decoder_max_batch(lbp_decoder d) { return d ? d->max_batch : 0; }

lbp_status lbp_decode_host(lbp_decoder d, int64_t n_shots, uint64_t first_shot_id, const uint32_t *syndromes,
                           uint32_t *corrections, uint8_t *flags, int32_t *iters, float *llr_out) {
    g_err.clear();
    if (!d) return fail(LBP_EINVAL, "lbp_decode_host: NULL decoder");
    if (n_shots < 0 || n_shots > d->max_batch) return fail(LBP_EINVAL, "lbp_decode_host: 0 <= n_shots <= max_batch");
    if (n_shots == 0) return LBP_OK;
    if (!syndromes || !corrections || !flags) return fail(LBP_EINVAL, "lbp_decode_host: NULL buffer");
    DeviceGuard g(d->code->device);
    const size_t mw = d->code->dc.mw, nw = d->code->dc.nw, n = d->code->n;
    uint32_t *ds = nullptr, *dc = nullptr;
    uint8_t *df = nullptr;
    int32_t *di = nullptr;
    float *dl = nullptr;
    hipStream_t s = nullptr;
    lbp_status st = LBP_OK;
    auto cleanup = [&]() {
        if (s) hipStreamDestroy(s);
        hipFree(ds); hipFree(dc); hipFree(df); hipFree(di); hipFree(dl);
    };
    auto chk = [&](hipError_t e, const char *what) {
        if (e != hipSuccess && st == LBP_OK)
            st = fail(e == hipErrorOutOfMemory ? LBP_ENOMEM : LBP_EDEVICE, std::string("lbp_decode_host: ") + what + ": " + hipGetErrorString(e));
        return e == hipSuccess;
    };
    bool ok = chk(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "hipStreamCreate") &&
              chk(hipMalloc(&ds, n_shots * mw * 4), "hipMalloc") && chk(hipMalloc(&dc, n_shots * nw * 4), "hipMalloc") &&
              chk(hipMalloc(&df, n_shots), "hipMalloc") && (!iters || chk(hipMalloc(&di, n_shots * 4), "hipMalloc")) &&
              (!llr_out || chk(hipMalloc(&dl, n_shots * n * 4), "hipMalloc")) &&
              chk(hipMemcpyAsync(ds, syndromes, n_shots * mw * 4, hipMemcpyHostToDevice, s), "hipMemcpyAsync");
    if (ok) {
        st = lbp_decode(d, n_shots, first_shot_id, ds, dc, df, di, dl, s);
        ok = st == LBP_OK && chk(hipMemcpyAsync(corrections, dc, n_shots * nw * 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync") &&
             chk(hipMemcpyAsync(flags, df, n_shots, hipMemcpyDeviceToHost, s), "hipMemcpyAsync") &&
             (!iters || chk(hipMemcpyAsync(iters, di, n_shots * 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync")) &&
             (!llr_out || chk(hipMemcpyAsync(llr_out, dl, n_shots * n * 4, hipMemcpyDeviceToHost, s), "hipMemcpyAsync")) &&
             chk(hipStreamSynchronize(s), "hipStreamSynchronize");
    }
    (void)ok;
    cleanup();
    return st;
}

}  // extern "C"
