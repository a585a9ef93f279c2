// Launch helpers the serving loop uses on a decoder's kernels and workspace.
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

}  // namespace lbp
