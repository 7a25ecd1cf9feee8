// Launchers of the setup kernels that build the segment layout's per-surfel
// part on the device (see setup.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace swgn {

// out[r] = key[run_start[r]]: the node set of each run of equal keys.
void launch_set_keys(int nsets, const uint64_t* key, const int* run_start, uint64_t* out, hipStream_t st);

// pos4[i]: positions (3 bits each, slot order) of surfel i's nodes among the
// 5 nodes of its segment (seg_start[nseg + 1], seg_nodes[5 nseg]); *bad is set
// if a node is missing.
void launch_seg_pos4(int ns, int nseg, const int* seg_start, const int* seg_nodes, const int4* idx, uint16_t* pos4,
                     int* bad, hipStream_t st);

}  // namespace swgn
