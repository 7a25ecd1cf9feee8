// Host-side launchers of the setup kernels and the node-state helpers; the
// per-frame stages are launched through swgn_frame.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace swgn {

// setup
// 4 nearest nodes (caller indices) and weights of every surfel; nodes in the
// library's order with their caller indices; boxes holds knn_box_count(nn)
// float4 of scratch.
size_t knn_box_count(int nn);
void launch_knn_skin(int ns, const float* pos_aos, int nn, const float4* nodes, const int* caller, float4* boxes,
                     float inv_two_sigma2, int4* idx, float4* w, hipStream_t st);
void launch_node_graph(int nn, const float4* nodes, int* nbr, hipStream_t st);
void sort_pairs(uint64_t* key, uint32_t* val, int n_pow2, hipStream_t st);
void exclusive_scan(const int* in, int* out, int n, int* tmp, hipStream_t st);
size_t scan_tmp_size(int n);
void launch_tuple_keys(int ns, int npad, const int4* idx, uint64_t* key, uint32_t* val, hipStream_t st);
void launch_permute_surfels(int ns, int seg_len, const uint64_t* key, const uint32_t* val, const float* ipos, const float* inrm,
                            const int4* iidx, const float4* iw, float* px, float* py, float* pz, float* nx,
                            float* ny, float* nz, int4* oidx, float4* ow, int* orig, int* flag, hipStream_t st);
void launch_run_starts(int ns, const int* flag, const int* pos, int* run_start, hipStream_t st);
void launch_pattern(int nruns, const uint64_t* key, const int* run_start, int nn, const int* nbr, uint32_t* bm,
                    int words, hipStream_t st);
void launch_row_counts(int nn, const uint32_t* bm, int words, int* cnt, hipStream_t st);
void launch_row_fill(int nn, const uint32_t* bm, int words, const int* row_ptr, int* col_idx, int* blk_row,
                     hipStream_t st);
void launch_transpose_keys(int nb, int npad, const int* blk_row, const int* col_idx, uint64_t* tkey, uint32_t* tval,
                           int* tcount, hipStream_t st);
void launch_full_counts(int nn, const int* row_ptr, const int* tcount, int* fcount, hipStream_t st);
void launch_full_rows(int nn, int ntr, const int* row_ptr, const int* col_idx, const int* tcount, const int* tstart,
                      const int* frow_ptr, const uint64_t* tkey, const uint32_t* tval, uint32_t* fblk, int* fcol,
                      hipStream_t st);

void launch_in_edge_keys(int nn, int npad, const int* nbr, uint64_t* key, uint32_t* val, int* icount, hipStream_t st);
void launch_in_edge_store(int n, const uint32_t* val, int* in_list, hipStream_t st);
void launch_ell_slots(int nn, int ell_w, const uint32_t* ell_blk, int* slot_u, int* slot_t, hipStream_t st);
void launch_ell(int nn, int ell_w, const int* frow_ptr, const uint32_t* fblk, const int* fcol, uint32_t* ell_blk,
                int* ell_col, hipStream_t st);

// node state and capture helpers
void launch_offlist(int nb, const int* blk_row, const int* col_idx, int* offlist, hipStream_t st);
void launch_nodes_from_se3(int nn, const float* se3, const float4* pref, float4* rq, float4* tt, float4* dq,
                           float4* cl, hipStream_t st);
void launch_node_se3_out(int nn, const float4* rq, const float4* tt, float* out, hipStream_t st);
void launch_export_index_map(int npx, const unsigned long long* z, int* out, hipStream_t st);
void launch_positions_to_f4(int n, const float* pos, float4* out, hipStream_t st);

}  // namespace swgn

namespace swgn {
void launch_fill_i32(int* p, int n, int v, hipStream_t st);
// p[i] <- map[p[i]] for i < n (indices from one numbering to another)
void launch_map_ids(int* p, int n, const int* map, hipStream_t st);
void launch_tables_from_state(int nn, const float4* pref, const float4* rq, const float4* tt, float4* dq, float4* cl,
                              hipStream_t st);
}  // namespace swgn
