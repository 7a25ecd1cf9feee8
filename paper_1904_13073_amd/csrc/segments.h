// Host-side layout of the segment Gram storage (plain C++, no HIP).
//
// Surfels sorted by node set are cut into segments: greedy runs of at most
// `max_surfels` surfels whose node sets together name at most 5 nodes. Each
// surfel gets the positions (3 bits each) of its 4 nodes among its segment's
// nodes; each segment gets a 15-bit mask of the node pairs (pa <= pb) that
// share a surfel, bit first(pa) + pb - pa with first(pa) = 5 pa - pa (pa-1)/2,
// and a float offset. A segment keeps 36 floats per pair of its mask, then
// J^T r (5 x 6 floats) and r^T r plus one pad float. The entries of an upper
// block of J^T J are the float offsets of its sub-blocks (and, for a diagonal
// block, of the matching 6-float J^T r piece) in segment order. Packs are
// greedy runs of whole segments with at most `max_surfels` surfels.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace swgn {

struct SegmentLayout {
    std::vector<int> seg_start;         // [nseg + 1]
    std::vector<int> seg_nodes;         // [5 nseg] the segment's nodes, ascending, -1 padded
    std::vector<uint16_t> pos4;         // [ns] (segment_layout only)
    std::vector<uint16_t> mask;         // [nseg]
    std::vector<uint32_t> off;          // [nseg + 1] float offsets
    std::vector<int> ent_ptr;           // [nb + 1]
    std::vector<uint32_t> ent_sub;      // [entries]
    std::vector<uint32_t> ent_grad;     // [entries], 0xffffffff for off-diagonal blocks
    std::vector<int> pack_start;        // [npack + 1] first surfel of each pack
    std::vector<int> pack_seg;          // [npack + 1] first segment of each pack
    uint64_t total = 0;                 // floats of all segments
};

// key[i]: the 4 node ids of surfel i in ascending order, 16 bits each, most
// significant first; keys ascend with i. idx4[4 i .. 4 i + 3]: the same nodes
// in the surfel's own slot order. (row_ptr, col_idx): the upper block pattern
// (CSR, columns ascending), which holds every pair of every node set.
// Returns false with `why` set when the input breaks these rules or the
// storage would exceed 2^32 floats.
bool segment_layout(int ns, int nn, int nb, const uint64_t* key, const int32_t* idx4, const int* row_ptr,
                    const int* col_idx, int max_surfels, SegmentLayout& out, std::string& why);

// The same layout from the runs of equal node sets alone (everything but
// pos4, which depends on each surfel's slot order): run r holds surfels
// set_start[r] .. set_start[r + 1] - 1 (non-empty, set_start[0] = 0), all with
// node set set_key[r]; keys strictly ascend. The work is per run and per
// segment, not per surfel.
bool segment_layout_sets(int nsets, const uint64_t* set_key, const int* set_start, int nn, int nb,
                         const int* row_ptr, const int* col_idx, int max_surfels, SegmentLayout& out,
                         std::string& why);

}  // namespace swgn
