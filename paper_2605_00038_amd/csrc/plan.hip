// Multi-group plans (lbp_plan_*): groups of shots from codes of different sizes,
// formats and parameters decoded by one persistent BP launch over a device
// descriptor table, followed by each group's OSD launch; the launch shape is
// picked by timing candidate shapes on the device, and the whole sequence is
// captured once into a HIP graph that every lbp_plan_launch replays.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbp.h"
#include "lbp_internal.h"
#include "serve_internal.h"

using namespace lbp;

namespace {

lbp_status pfail(lbp_status s, const std::string &msg) {
    set_error(msg.c_str());
    return s;
}

size_t al256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Shape {
    int wpb, blocks;
};

}  // namespace

struct lbp_plan_s {
    int device = 0;
    int n_groups = 0;
    std::vector<lbp_group> groups;
    std::vector<DecoderView> views;
    std::vector<GroupDesc> desc;   // host copy of the device table
    void *dmem = nullptr;          // one allocation: table, counters, failure lists, staging, OSD scratch, stage
    GroupDesc *d_desc = nullptr;
    uint32_t *d_counters = nullptr;  // [16 (global) + 16 per group]
    std::vector<uint32_t *> gscratch;
    float *d_stage = nullptr;
    int wave_bytes = 0;
    int64_t stage_stride = 0;
    int64_t n_work = 0;
    Shape shape{1, 1};
    std::vector<Shape> cands;
    std::vector<double> cand_ms;
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

// The launch sequence of one decode of every group: clear the counters (a kernel:
// no memset node in the graph), the persistent multi-group BP launch, then the
// OSD launch of each group that has one.
static lbp_status plan_enqueue(lbp_plan P, const Shape &sh, hipStream_t s) {
    const int nc = 16 * (P->n_groups + 1);
    hipError_t e = launch_reset(P->d_counters, nc, s);
    if (e != hipSuccess) return pfail(LBP_EDEVICE, std::string("lbp_plan: reset launch: ") + hipGetErrorString(e));
    MultiArgs a{};
    a.groups = P->d_desc;
    a.n_groups = P->n_groups;
    a.wave_bytes = P->wave_bytes;
    a.n_work = P->n_work;
    a.counter = P->d_counters;
    a.stage = P->d_stage;
    a.stage_stride = P->stage_stride;
    e = launch_bp_multi(a, sh.blocks, sh.wpb, s);
    if (e != hipSuccess) return pfail(LBP_EDEVICE, std::string("lbp_plan: BP launch: ") + hipGetErrorString(e));
    for (int g = 0; g < P->n_groups; ++g) {
        const GroupDesc &G = P->desc[(size_t)g];
        if (G.prm.osd == OSD_NONE || G.n_shots == 0) continue;
        const int blocks = (int)std::min<int64_t>(P->views[(size_t)g].osd_blocks, G.n_shots);
        lbp_status st = decoder_launch_osd(P->groups[(size_t)g].dec, G.synd, G.corr, G.flags, G.counters,
                                           G.fail_list, G.fail_llr, G.n_shots, P->gscratch[(size_t)g], blocks, s);
        if (st != LBP_OK) return st;
    }
    return LBP_OK;
}

static void plan_free(lbp_plan P) {
    if (P->exec) hipGraphExecDestroy(P->exec);
    if (P->graph) hipGraphDestroy(P->graph);
    if (P->cap) hipStreamDestroy(P->cap);
    hipFree(P->dmem);
}

extern "C" {

lbp_status lbp_plan_create(int32_t n_groups, const lbp_group *groups, int32_t options, lbp_plan *out) {
    set_error("");
    if (!out || (n_groups > 0 && !groups)) return pfail(LBP_EINVAL, "lbp_plan_create: NULL argument");
    *out = nullptr;
    if (n_groups < 1 || n_groups > 64) return pfail(LBP_EINVAL, "lbp_plan_create: 1 <= n_groups <= 64");
    if (options & ~LBP_PLAN_AUTOTUNE) return pfail(LBP_EINVAL, "lbp_plan_create: unknown option bits");
    lbp_plan P = new lbp_plan_s();
    auto bail = [&](lbp_status st, const std::string &msg) {
        plan_free(P);
        delete P;
        return pfail(st, msg);
    };
    P->n_groups = n_groups;
    P->groups.assign(groups, groups + n_groups);
    P->views.resize((size_t)n_groups);
    int64_t items = 0;
    size_t max_n = 1;
    for (int g = 0; g < n_groups; ++g) {
        const lbp_group &q = groups[g];
        if (!q.dec) return bail(LBP_EINVAL, "lbp_plan_create: group " + std::to_string(g) + " has no decoder");
        if (q.n_shots < 0 || q.n_shots > ((int64_t)1 << 31))
            return bail(LBP_EINVAL, "lbp_plan_create: group " + std::to_string(g) + ": 0 <= n_shots <= 2^31");
        if (q.n_shots > 0 && (!q.syndromes || !q.corrections || !q.flags))
            return bail(LBP_EINVAL, "lbp_plan_create: group " + std::to_string(g) + " has a NULL buffer");
        DecoderView &v = P->views[(size_t)g];
        lbp_status st = decoder_view(q.dec, &v);
        if (st != LBP_OK) return bail(st, "lbp_plan_create: " + std::string(lbp_last_error()));
        if (g == 0) P->device = v.device;
        if (v.device != P->device) return bail(LBP_EINVAL, "lbp_plan_create: groups on different devices");
        if (v.dc.vn_tab4) return bail(LBP_EUNSUPPORTED, "lbp_plan_create: codes above 8191 checks are not supported");
        P->wave_bytes = std::max(P->wave_bytes, bp_wave_bytes(v.msgk, v.dc.m, v.dc.n));
        max_n = std::max(max_n, (size_t)v.dc.n);
        items += q.n_shots;
    }
    if (items > ((int64_t)1 << 32) - 1) return bail(LBP_EINVAL, "lbp_plan_create: more than 2^32 - 1 shots in all");
    P->n_work = items;
    P->stage_stride = (int64_t)(2 * max_n);
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != P->device) hipSetDevice(P->device);
    struct Restore {
        int d;
        ~Restore() {
            if (d >= 0) hipSetDevice(d);
        }
    } restore{prev != P->device ? prev : -1};

    // ---- launch shapes the multi-group kernel can run: waves per block x resident blocks
    int ncu = 0, lds_max = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, P->device) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, P->device) != hipSuccess)
        return bail(LBP_EDEVICE, "lbp_plan_create: device query failed");
    for (int wpb : {1, 2, 4, 8, 16}) {
        const int lds = P->wave_bytes * wpb;
        if (lds > lds_max) continue;
        int bpc = 0;
        if (bp_multi_max_blocks_per_cu(wpb, lds, &bpc) != hipSuccess || bpc < 1) continue;
        P->cands.push_back(Shape{wpb, bpc * ncu});
    }
    if (P->cands.empty()) return bail(LBP_EUNSUPPORTED, "lbp_plan_create: a shot's state exceeds LDS");
    // without tuning: the most resident waves, ties to the larger block
    P->shape = P->cands[0];
    for (const Shape &c : P->cands)
        if (c.wpb * c.blocks >= P->shape.wpb * P->shape.blocks) P->shape = c;
    size_t stage_waves = 0;
    for (const Shape &c : P->cands) stage_waves = std::max(stage_waves, (size_t)c.wpb * (size_t)c.blocks);

    // ---- one allocation: table, counters, and per group failure list, staging for
    // every shot (the graph has no overflow pass) and OSD scratch; then the stage
    size_t off = 0;
    const size_t o_desc = off;
    off += al256(sizeof(GroupDesc) * (size_t)n_groups);
    const size_t o_cnt = off;
    off += al256((size_t)16 * 4 * (size_t)(n_groups + 1));
    std::vector<size_t> o_list((size_t)n_groups), o_llr((size_t)n_groups), o_g((size_t)n_groups);
    for (int g = 0; g < n_groups; ++g) {
        const DecoderView &v = P->views[(size_t)g];
        const int64_t ns = groups[g].n_shots;
        o_list[(size_t)g] = off;
        o_llr[(size_t)g] = off;
        o_g[(size_t)g] = off;
        if (v.osd == OSD_NONE || ns == 0) continue;
        off += al256((size_t)ns * 4);
        o_llr[(size_t)g] = off;
        off += al256((size_t)ns * 8 * (size_t)v.dc.n);
        o_g[(size_t)g] = off;
        off += al256((size_t)std::min<int64_t>(v.osd_blocks, ns) * v.osd_scratch);
    }
    const size_t o_stage = off;
    off += al256(stage_waves * (size_t)P->stage_stride * 4);
    hipError_t e = hipMalloc(&P->dmem, off);
    if (e != hipSuccess) return bail(LBP_ENOMEM, std::string("lbp_plan_create: hipMalloc: ") + hipGetErrorString(e));
    unsigned char *b = (unsigned char *)P->dmem;
    P->d_desc = (GroupDesc *)(b + o_desc);
    P->d_counters = (uint32_t *)(b + o_cnt);
    P->d_stage = (float *)(b + o_stage);
    P->desc.resize((size_t)n_groups);
    P->gscratch.resize((size_t)n_groups);
    int64_t first = 0;
    for (int g = 0; g < n_groups; ++g) {
        const DecoderView &v = P->views[(size_t)g];
        GroupDesc &G = P->desc[(size_t)g];
        std::memset(&G, 0, sizeof(G));
        G.code = v.dc;
        G.prm = v.bp;
        G.msg = v.msgk;
        G.first_item = first;
        G.n_shots = groups[g].n_shots;
        G.first_shot_id = groups[g].first_shot_id;
        G.synd = groups[g].syndromes;
        G.corr = groups[g].corrections;
        G.flags = groups[g].flags;
        G.iters = groups[g].iters;
        G.counters = P->d_counters + 16 * (g + 1);
        G.fail_list = (int32_t *)(b + o_list[(size_t)g]);
        G.fail_llr = (float *)(b + o_llr[(size_t)g]);
        P->gscratch[(size_t)g] = (uint32_t *)(b + o_g[(size_t)g]);
        first += G.n_shots;
    }
    e = hipMemcpy(P->d_desc, P->desc.data(), sizeof(GroupDesc) * (size_t)n_groups, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(LBP_EDEVICE, std::string("lbp_plan_create: hipMemcpy: ") + hipGetErrorString(e));
    e = hipStreamCreateWithFlags(&P->cap, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(LBP_EDEVICE, std::string("lbp_plan_create: hipStreamCreate: ") + hipGetErrorString(e));

    // ---- autotuner: time every candidate shape on the device (one warm-up run,
    // then the best of two timed runs on the groups' own buffers)
    if (options & LBP_PLAN_AUTOTUNE) {
        hipEvent_t t0 = nullptr, t1 = nullptr;
        if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
            return bail(LBP_EDEVICE, "lbp_plan_create: hipEventCreate failed");
        double best = 1e300;
        lbp_status st = LBP_OK;
        for (const Shape &c : P->cands) {
            double ms_best = 1e300;
            for (int rep = 0; rep < 3 && st == LBP_OK; ++rep) {
                if (rep > 0 && hipEventRecord(t0, P->cap) != hipSuccess) st = LBP_EDEVICE;
                if (st == LBP_OK) st = plan_enqueue(P, c, P->cap);
                if (st == LBP_OK && rep > 0) {
                    float ms = 0.f;
                    if (hipEventRecord(t1, P->cap) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                        hipEventElapsedTime(&ms, t0, t1) != hipSuccess)
                        st = LBP_EDEVICE;
                    ms_best = std::min(ms_best, (double)ms);
                }
            }
            if (st != LBP_OK) break;
            P->cand_ms.push_back(ms_best);
            if (ms_best < best) {
                best = ms_best;
                P->shape = c;
            }
        }
        hipEventDestroy(t0);
        hipEventDestroy(t1);
        if (st != LBP_OK) return bail(LBP_EDEVICE, "lbp_plan_create: autotuning run failed");
    } else {
        // one eager run sets the kernels' LDS attributes outside the capture
        lbp_status st = plan_enqueue(P, P->shape, P->cap);
        if (st != LBP_OK) return bail(st, lbp_last_error());
    }
    if (hipStreamSynchronize(P->cap) != hipSuccess) return bail(LBP_EDEVICE, "lbp_plan_create: eager run failed");

    // ---- capture the sequence once; lbp_plan_launch replays it
    e = bp_multi_prepare(P->wave_bytes * P->shape.wpb);
    if (e == hipSuccess) e = hipStreamBeginCapture(P->cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return bail(LBP_EDEVICE, std::string("lbp_plan_create: capture: ") + hipGetErrorString(e));
    lbp_status st = plan_enqueue(P, P->shape, P->cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(P->cap, &graph);
    P->graph = graph;
    if (st != LBP_OK) return bail(st, lbp_last_error());
    if (e != hipSuccess) return bail(LBP_EDEVICE, std::string("lbp_plan_create: end capture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&P->exec, P->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return bail(LBP_EDEVICE, std::string("lbp_plan_create: instantiate: ") + hipGetErrorString(e));
    *out = P;
    return LBP_OK;
}

lbp_status lbp_plan_launch(lbp_plan P, void *stream) {
    set_error("");
    if (!P) return pfail(LBP_EINVAL, "lbp_plan_launch: NULL plan");
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != P->device) hipSetDevice(P->device);
    const hipError_t e = hipGraphLaunch(P->exec, (hipStream_t)stream);
    if (prev != P->device) hipSetDevice(prev);
    if (e != hipSuccess) return pfail(LBP_EDEVICE, std::string("lbp_plan_launch: ") + hipGetErrorString(e));
    return LBP_OK;
}

lbp_status lbp_plan_info(lbp_plan P, int32_t *waves_per_block, int32_t *blocks, int32_t *n_candidates,
                         double *candidate_ms) {
    if (!P) return pfail(LBP_EINVAL, "lbp_plan_info: NULL plan");
    if (waves_per_block) *waves_per_block = P->shape.wpb;
    if (blocks) *blocks = P->shape.blocks;
    if (n_candidates) *n_candidates = (int32_t)P->cand_ms.size();
    if (candidate_ms)
        for (size_t k = 0; k < P->cand_ms.size() && k < 8; ++k) candidate_ms[k] = P->cand_ms[k];
    return LBP_OK;
}

void lbp_plan_destroy(lbp_plan P) {
    if (!P) return;
    int prev = -1;
    hipGetDevice(&prev);
    if (prev != P->device) hipSetDevice(P->device);
    plan_free(P);
    if (prev != P->device) hipSetDevice(prev);
    delete P;
}

}  // extern "C"
