/*
 * swgn -- per-frame Gauss-Newton estimate of a node-graph warp field on
 * AMD Instinct MI355X (gfx950).
 *
 * The operation is the non-rigid solve of SurfelWarp (Gao and Tedrake, RSS
 * 2019), Sec. 7 "Non-Rigid Warp Field Estimation": given a new depth image D,
 * the previous warp field W_prev and the reference surfels S_ref, estimate the
 * node transforms T_j of W by minimising E_depth + lambda E_regulation with
 * Gauss-Newton (Sec. 7 energy equation; Sec. 8: build J^T J, then solve; at
 * most 10 iterations). The warp of a surfel is the dual-quaternion blend of
 * its K = 4 nearest nodes (Sec. 3, Eq. 1 and Eq. 2); skinning and node graph
 * are computed once per node set (Sec. 6.5).
 *
 * All entry points are C, take plain pointers and sizes and never throw or
 * abort. Each returns an sw_status; on failure sw_last_error() gives a
 * message. A stream handle owns all of its device memory; it is not
 * thread-safe, distinct handles are independent.
 *
 * Coordinates are metres in the camera frame (x right, y down, z forward),
 * pixel centres at integer coordinates: pixel (u, v) sees
 * ((u - cx) / fx, (v - cy) / fy, 1) * depth.
 */
#ifndef SWGN_H
#define SWGN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sw_status;
#define SW_OK        0
#define SW_EINVAL   -1   /* bad argument */
#define SW_ESTATE   -2   /* call order (e.g. solve before surfels and nodes) */
#define SW_ENOMEM   -3   /* device or host allocation failed */
#define SW_EHIP     -4   /* HIP runtime error */
#define SW_ENUMERIC -5   /* non-finite energy or a non-positive-definite 6x6 block */

typedef struct sw_stream_s* sw_stream;

/* Solver configuration. sw_config_default() fills the defaults given below. */
typedef struct sw_config {
    int32_t width, height;     /* depth image size, 640 x 480 */
    float fx, fy, cx, cy;      /* pinhole intrinsics, 570 570 320 240 */
    int32_t gn_iters;          /* Gauss-Newton iterations per frame, 10 (0..16) */
    int32_t pcg_iters;         /* PCG iterations per Gauss-Newton step, 10 (0..4096) */
    float lambda_reg;          /* regulariser weight lambda, 5 (Table 1) */
    float node_sigma;          /* node radius sigma in the blend weights, 0.025 m (Table 1) */
    float corr_dist;           /* correspondence distance gate, 0.05 m */
    float corr_normal;         /* correspondence normal gate (cosine), 0.5 */
    float edge_gate;           /* normal-map depth-discontinuity gate, 0.03 m */
    float damping;             /* mu added to every diagonal entry of J^T J, 1e-4 */
    int32_t jac_dtype;         /* Jacobian storage: 0 = fp32 */
    int32_t dot_fp64;          /* 1 = accumulate PCG dot products in fp64 (default 1) */
    int32_t debug_iter;        /* -1 = capture nothing; k = capture GN iteration k */
    int32_t stage_timing;      /* 1 = time every kernel with HIP events into stage_us */
} sw_config;

/* Per-frame statistics, one entry per Gauss-Newton iteration (<= 16). */
typedef struct sw_frame_stats {
    int32_t iters;             /* Gauss-Newton iterations run */
    float e_data[16];          /* E_depth at the iteration's linearisation point */
    float e_reg[16];           /* E_regulation (unweighted) at the same point */
    int32_t n_corr[16];        /* correspondences |P| */
    float pcg_resid[16];       /* |r| of the linear system when PCG stops */
    float stage_us[12];        /* with stage_timing: microseconds per kernel, summed
                                  over the frame: [0] depth preprocessing, [1] warp +
                                  index map, [2] correspondence + Jacobians,
                                  [3] assembly of chunk partials, [4] block-Jacobi +
                                  PCG start, [5] PCG products, [6] PCG updates,
                                  [7] node update, [8] assembly of the blocks;
                                  measured with HIP events */
    double alg_bytes;          /* algorithmic bytes moved by the frame (model) */
} sw_frame_stats;

/* Fill *cfg with the defaults listed in sw_config. */
void sw_config_default(sw_config* cfg);

/* Static description of a status code. */
const char* sw_status_string(sw_status st);

/* Message of the last failed call on s (empty if none; never NULL). */
const char* sw_last_error(sw_stream s);

/* Create a stream. hip_stream is the hipStream_t all work is queued on, or
 * NULL for a stream the library creates and destroys. The config is copied.
 * SW_EINVAL: image size <= 0, non-finite or non-positive focal lengths,
 * iteration counts out of range, non-positive sigma, negative weights. */
sw_status sw_create_stream(const sw_config* cfg, void* hip_stream, sw_stream* out);

/* Destroy a stream and free its device memory. NULL is a no-op. */
sw_status sw_destroy_stream(sw_stream s);

/* Reference surfels S_ref (Sec. 4): n positions and unit normals, each n x 3
 * row-major fp32 (AoS), host (on_device = 0) or device (on_device = 1)
 * pointers readable on the stream until the call returns. The data is copied;
 * the caller keeps ownership. Setting surfels invalidates the skinning:
 * sw_set_node_graph must follow before a solve. n in [1, 2^28). */
sw_status sw_set_reference_surfels(sw_stream s, int64_t n, const float* pos_xyz,
                                   const float* nrm_xyz, int32_t on_device);

/* Node graph (Sec. 3 and Sec. 6.5): n_nodes positions p_j (n x 3 fp32) in the
 * reference frame and their transforms (n x 12 fp32, row-major [R | t],
 * x_live = R x + t), or NULL for the identity. Runs the skinning (each surfel's
 * 4 nearest nodes by squared distance, ties to the lower node index, and the
 * blend weights exp(-d^2 / (2 sigma^2)) normalised), the node graph (each
 * node's 8 nearest other nodes) and the block pattern of J^T J. The node order
 * defines the node indices. n_nodes in [9, 32768]; surfels must be set
 * (SW_ESTATE otherwise). */
sw_status sw_set_node_graph(sw_stream s, int32_t n_nodes, const float* node_pos_xyz,
                            const float* node_se3, int32_t on_device);

/* Replace the node transforms (n x 12 [R | t]) without redoing skinning:
 * restores a snapshot taken with sw_get_node_se3. n must equal n_nodes. */
sw_status sw_set_node_se3(sw_stream s, const float* node_se3, int32_t n, int32_t on_device);

/* Solve one frame: depth is H x W fp32 row-major metres (<= 0 or non-finite
 * = no measurement), host or device. Runs gn_iters Gauss-Newton iterations
 * from the current node transforms (the previous frame's warp field, Sec. 4)
 * and returns after the transforms are updated. stats may be NULL. On
 * SW_ENUMERIC the transforms keep their values from before the call. */
sw_status sw_solve_frame(sw_stream s, const float* depth, int32_t on_device,
                         sw_frame_stats* stats);

/* Copy the node transforms to host memory out (n_nodes x 12 fp32 [R | t]).
 * SW_EINVAL if capacity (in nodes) < n_nodes. */
sw_status sw_get_node_se3(sw_stream s, float* out, int32_t capacity);

/* Sizes of the current problem (any pointer may be NULL). */
sw_status sw_get_sizes(sw_stream s, int64_t* n_surfels, int32_t* n_nodes, int32_t* n_blocks);

/* ---- parity and debug exports (host pointers, caller's surfel order) ---- */

/* Skinning: idx4 (n_surfels x 4, nearest first) and weights w4 (n_surfels x 4). */
sw_status sw_get_skinning(sw_stream s, int32_t* idx4, float* w4);

/* Node graph: nbr8 (n_nodes x 8, nearest first). */
sw_status sw_get_node_graph(sw_stream s, int32_t* nbr8);

/* Upper block pattern of J^T J: row_ptr (n_nodes + 1), col_idx (n_blocks),
 * node indices, columns ascending, the diagonal first in every row. */
sw_status sw_get_pattern(sw_stream s, int32_t* row_ptr, int32_t* col_idx);

/* Maps of the captured Gauss-Newton iteration (config debug_iter): index map
 * and correspondence map (H x W surfel indices, -1 = none), live positions
 * (n_surfels x 3, NaN where the blend is undefined) and the depth normal map
 * (3 x H x W planes, 0 where undefined). Any pointer may be NULL.
 * SW_ESTATE if nothing was captured. */
sw_status sw_get_last_maps(sw_stream s, int32_t* index_map, int32_t* corr_map,
                           float* live_pos, float* depth_normals);

/* Linear system of the captured iteration: blocks (n_blocks x 36, row-major
 * 6x6 blocks of J^T J + mu I in the order of sw_get_pattern; unknowns of node k
 * are (w_k, tau_k)), g = J^T r (n_nodes x 6) and the PCG solution delta of
 * (J^T J + mu I) delta = -g (n_nodes x 6). Any pointer may be NULL. */
sw_status sw_get_last_system(sw_stream s, float* blocks, float* g, float* delta);

/* Data-term residuals r (n_surfels; 0 where no correspondence) and Jacobians
 * J (n_surfels x 4 x 6, node slots nearest first) of the captured iteration. */
sw_status sw_get_last_jacobian(sw_stream s, float* r, float* J);

#ifdef __cplusplus
}
#endif

#endif /* SWGN_H */
