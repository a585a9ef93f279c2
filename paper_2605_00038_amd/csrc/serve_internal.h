// Helpers the serving loop and the multi-group plans use on a decoder's
// kernels, tables and workspace.
#pragma once

#include "../../include/lbp.h"
#include "lbp_internal.h"

namespace lbp {

struct ServeShape {
    int bp_blocks;   // BP grid while serving (leaves CUs for OSD launches)
    int osd_blocks;  // OSD grid per launch
};

// Split the device between the persistent BP grid and OSD launches:
// osd_fraction of the CUs are left to OSD.
lbp_status serve_shape(lbp_decoder d, double osd_fraction, ServeShape *out);
// Device bytes of one ring item's staged lambda (for OSD): 2n for the Int x.y
// check-centric kernel (int16), 8n for the others (hi, lo floats).
int64_t serve_llr_bytes(lbp_decoder d);
// Persistent BP kernel over the ring described by ring_dev (device copy).
// Clears `exiting` (stream-ordered) and launches the persistent BP grid.
lbp_status serve_launch_bp(lbp_decoder d, const ServeRing *ring_dev, uint32_t *exiting, int blocks, hipStream_t s);
// OSD of the ring slots d_list[0 .. d_counters[1]) (lambda in ring.llr, by slot).
lbp_status serve_launch_osd(lbp_decoder d, const ServeRing &ring, const int32_t *d_list, const uint32_t *d_counters,
                            int blocks, hipStream_t s);

// What a multi-group plan needs of a decoder: its tables and parameters, and the
// size of its OSD blocks' scratch.
struct DecoderView {
    DevCode dc;          // tables, with the decoder's Int x.y prior
    BpParams bp;
    int msgk;            // MSG_FP32 / MSG_FP16 / MSG_INT8
    int osd;             // OSD_NONE / OSD_0 / OSD_CS
    int device;
    int osd_blocks;      // OSD grid of the decoder
    size_t osd_scratch;  // OSD scratch bytes per block
};
lbp_status decoder_view(lbp_decoder d, DecoderView *out);
// OSD of fail_list[0 .. counters[1]) whose lambda was staged as fp32 pairs
// (hi[n], lo[n]) by the general BP kernel, on gscratch (blocks OSD blocks).
lbp_status decoder_launch_osd(lbp_decoder d, const uint32_t *synd, uint32_t *corr, uint8_t *flags,
                              const uint32_t *counters, const int32_t *fail_list, const float *fail_llr,
                              int64_t fail_cap, uint32_t *gscratch, int blocks, hipStream_t s);

}  // namespace lbp
