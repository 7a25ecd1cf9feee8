// Launchers of the setup kernels that build the segment layout on the device
// (setup.hip, segwalk.hip).
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

// Successor chains: for next[i] with i < next[i] <= min(n, i + M) (M at most
// chain_max_hop()), out[0 .. *count) = 0, next[0], next[next[0]], ... (every
// position below n the chain from 0 visits). work holds chain_work_ints(n, M)
// ints; *bad is set if next breaks the rule (out and *count are then not the
// chain).
size_t chain_work_ints(int n, int M);
int chain_max_hop();
void chain_from_zero(const int* next, int n, int M, int* out, int* count, int* work, int* bad, hipStream_t st);

// next[s]: the surfel where the greedy segment opening at surfel s ends (at
// most M surfels, at most 5 nodes; runs of equal node sets set_start[nsets +
// 1] with node sets set_key[nsets]; run_pos[ns + 1] the exclusive scan of the
// run-start flags).
void launch_seg_next(int ns, int nsets, const uint64_t* set_key, const int* set_start, const int* run_pos, int M,
                     int* next, hipStream_t st);

// next[g]: the segment where the greedy pack of at most M surfels opening at
// segment g ends.
void launch_pack_next(int nseg, const int* seg_start, int M, int* next, hipStream_t st);

// Per segment: nodes (5, ascending, -1 padded), pair mask, Gram output size
// in 4-float units and pair count; *total_units accumulates the sizes (64-bit);
// *bad is set for a segment of more than 5 nodes.
void launch_seg_info(int nseg, const int* seg_start, const int* run_pos, const uint64_t* set_key, int* seg_nodes,
                     uint16_t* mask, int* units, int* npairs, unsigned long long* total_units, int* bad,
                     hipStream_t st);

// off[g] = 4 off_units[g] for g <= nseg (float offsets from 4-float units).
void launch_seg_off(int nseg, const int* off_units, uint32_t* off, hipStream_t st);

// The block fold's entries, unsorted: ne = sum of the pair counts, entry e of
// segment g at ebase[g] + rank; ekey/eval padded to npad (a power of two) for
// sort_pairs; bcount[nb] counts entries per block (zeroed by the caller).
void launch_seg_entries(int nseg, int nb, int npad, const int* seg_nodes, const uint16_t* mask, const uint32_t* off,
                        const int* ebase, int ne, const int* row_ptr, const int* col_idx, uint64_t* ekey,
                        uint32_t* eval, uint32_t* esub, uint32_t* egrad, int* bcount, int* bad, hipStream_t st);

// ent_sub/ent_grad[i] = esub/egrad[order[i]] (entries in block order).
void launch_ent_gather(int ne, const uint32_t* order, const uint32_t* esub, const uint32_t* egrad, uint32_t* ent_sub,
                       uint32_t* ent_grad, hipStream_t st);

// pack_start[i] = seg_start[pack_seg[i]] for i < npack; pack_seg[npack] = nseg,
// pack_start[npack] = ns.
void launch_pack_arrays(int npack, int nseg, int ns, const int* seg_start, int* pack_seg, int* pack_start,
                        hipStream_t st);

}  // namespace swgn
