// Host-side launchers of the setup and per-frame kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace swgn {

struct Cam;

struct SurfelView {
    const float *px, *py, *pz, *nx, *ny, *nz;
    const int4* idx;
    const float4* w;
    const int* orig;
};

constexpr int kSegLen = 128;      // surfels per segment at most (one node set)
constexpr int kSegSlots = 400;    // per segment: 10 upper 6x6 blocks, J^T r (24), r^T r

struct AssembleArgs {
    int nb, nn, noff, pitch, nseg;
    const int* blk_row;
    const int* col_idx;
    const int* row_ptr;
    const int* offlist;
    const int* seg_start;    // [nseg + 1] surfel ranges sharing one node set
    const int* ent_ptr;      // [nb + 1] per block: its (segment, pos_a, pos_b) entries
    const uint32_t* ent;     // (segment << 4 | pos_a << 2 | pos_b)
    const int* in_ptr;       // node -> in-edges (j with the node in N_j)
    const int* in_list;
    const float* J;          // [pitch][32]: J (24), r, zero padding
    const int* nbr;
    const float4* pref;
    const float4* rq;
    const float4* cl;
    float lambda, mu;
    float* part;             // [nseg][kSegSlots] segment Gram sub-blocks
    float* H;
    float* g;
    float* ereg;
};

struct SolveStepArgs {
    int nn, npx;
    const int* row_ptr;
    const float* H;
    const float* g;
    int ell_w;
    const uint32_t* ell_blk;
    const int* ell_col;
    double* Minv;
    float *x, *r, *z, *q, *p0, *p1;
    double *sc, *part_rho, *part_rr, *part_pq;
    int* flags;
    const double* part_e;
    const int* part_n;
    int nparts;
    const float* ereg;
    void* stats;
    const float4* pref;
    float4 *rq, *tt, *dq, *cl;
    unsigned long long* zbuf;
};

// setup
void launch_knn_skin(int ns, const float* pos_aos, int nn, const float4* nodes, float inv_two_sigma2, int4* idx,
                     float4* w, hipStream_t st);
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
void launch_run_entries(int nruns, int npad, const uint64_t* key, const int* run_start, const int* row_ptr,
                        const int* col_idx, uint64_t* ekey, uint32_t* eval, int* ecount, hipStream_t st);
void launch_entries_store(int ne, const uint64_t* ekey, uint32_t* ent, hipStream_t st);
void launch_transpose_keys(int nb, int npad, const int* blk_row, const int* col_idx, uint64_t* tkey, uint32_t* tval,
                           int* tcount, hipStream_t st);
void launch_full_counts(int nn, const int* row_ptr, const int* tcount, int* fcount, hipStream_t st);
void launch_full_rows(int nn, int ntr, const int* row_ptr, const int* col_idx, const int* tcount, const int* tstart,
                      const int* frow_ptr, const uint64_t* tkey, const uint32_t* tval, uint32_t* fblk, int* fcol,
                      hipStream_t st);

void launch_in_edge_keys(int nn, int npad, const int* nbr, uint64_t* key, uint32_t* val, int* icount, hipStream_t st);
void launch_in_edge_store(int n, const uint32_t* val, int* in_list, hipStream_t st);
void launch_ell(int nn, int ell_w, const int* frow_ptr, const uint32_t* fblk, const int* fcol, uint32_t* ell_blk,
                int* ell_col, hipStream_t st);

// per frame
void launch_depth_prep(const Cam& cam, const float* depth, float gate, float4* nmap, unsigned long long* zbuf,
                       int* flags, hipStream_t st);
void launch_clear_z(unsigned long long* z, int n, hipStream_t st);
void launch_warp_zbuf(int ns, const SurfelView& sv, const float4* dq, const Cam& cam, unsigned long long* z,
                      hipStream_t st);
int corr_blocks(int ns);
void launch_corr_jac(int ns, const SurfelView& sv, const float4* dq, const float4* cl, const Cam& cam,
                     const unsigned long long* z, const float4* nmap, float dist2, float cosn, float* J, int pitch,
                     double* part_e, int* part_n, int* corr_map, float* live_pos, hipStream_t st);
void launch_offlist(int nb, const int* blk_row, const int* col_idx, int* offlist, hipStream_t st);
void launch_assemble_segments(const AssembleArgs& a, hipStream_t st);
void launch_assemble_fold(const AssembleArgs& a, hipStream_t st);
int solve_partials_size(int nn);
void launch_pcg_init(const SolveStepArgs& a, hipStream_t st);
void launch_pcg_spmv(const SolveStepArgs& a, int it, hipStream_t st);
void launch_pcg_update(const SolveStepArgs& a, int it, hipStream_t st);
void launch_node_update(const SolveStepArgs& a, int pcg_iters, hipStream_t st);
void launch_nodes_from_se3(int nn, const float* se3, const float4* pref, float4* rq, float4* tt, float4* dq,
                           float4* cl, hipStream_t st);
void launch_node_se3_out(int nn, const float4* rq, const float4* tt, float* out, hipStream_t st);
void launch_export_index_map(int npx, const unsigned long long* z, int* out, hipStream_t st);
void launch_positions_to_f4(int n, const float* pos, float4* out, hipStream_t st);

}  // namespace swgn

namespace swgn {
void launch_fill_i32(int* p, int n, int v, hipStream_t st);
void launch_tables_from_state(int nn, const float4* pref, const float4* rq, const float4* tt, float4* dq, float4* cl,
                              hipStream_t st);
}  // namespace swgn
