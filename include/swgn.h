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
#define SW_EPENDING  1   /* sw_server_poll: the frame is not done yet (not an error) */

typedef struct sw_stream_s* sw_stream;
typedef struct sw_server_s* sw_server;

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
    int32_t jac_dtype;         /* Jacobian entries kept as 0 = fp32, 1 = bf16, 2 = fp16
                                  (rounded to nearest even; r, J^T J, J^T r, PCG stay
                                  fp32, block inverses and PCG dots fp64) */
    int32_t dot_fp64;          /* 1 = accumulate PCG dot products in fp64 (default 1) */
    int32_t debug_iter;        /* -1 = capture nothing; k = capture GN iteration k */
    int32_t stage_timing;      /* 1 = time every kernel with HIP events into stage_us */
    int32_t rigid_iters;       /* rigid alignment steps before the non-rigid ones (Sec. 7,
                                  as in KinectFusion): projective point-to-plane ICP of one
                                  rigid transform applied after the warp field, then
                                  composed into every node; 0 = none (default), <= 16 */
    int32_t visibility;        /* surfels rendered into the solver's index map (Sec. 7):
                                  0 = all (default), 1 = only stable ones (confidence >
                                  stable_conf) or recently observed ones (t_now - t_observed
                                  <= recent_frames); unsized points either way */
    float stable_conf;         /* delta_stable, 10 (Table 1) */
    int32_t recent_frames;     /* delta_recent, 2 (Table 1); -1 = the recent clause off, only
                                  stable surfels render (Sec. 7 adds the recent ones only in
                                  the first frames and after a reinitialisation) */
    float fusion_dist;         /* depth fusion distance gate delta_distance, 0.001 m (Table 1) */
    float fusion_normal;       /* depth fusion normal gate delta_normal, 0.85 (Table 1) */
    float warp_eps;            /* intrinsic deformation bound epsilon of live skinning and of
                                  the compressive-warp test (Eq. 7, Eq. 8), 0.2 (Table 1) */
    float append_nn;           /* delta_nn: append candidates whose kept nearest-node weight
                                  sum is below it are dropped (Sec. 6.4); the paper gives no
                                  value, 0.3 */
    int32_t t_low_confid;      /* frames a surfel may stay below stable_conf after its
                                  initialisation before the geometry update drops it, 30
                                  (Table 1) */
    int32_t splat;             /* solver index map (Sec. 7): 0 = unsized points (default);
                                  1 = opaque disc splats of the surfels' radii: a surfel whose
                                  centre projects into the image is tried on the pixels within
                                  min(4, ceil(fx r / z)) of its centre pixel, pixel u is covered
                                  when its centre ray meets the disc (n.d != 0, t = n.v / n.d
                                  > 0, |t d - v|^2 <= r^2) at depth t, nearest depth wins,
                                  ties to the lower index; radius 0 renders a point. Every
                                  pixel with a normal then pairs with its winner under the
                                  correspondence gates, so a surfel may hold several pairs
                                  (each a data row; n_corr counts pairs). The rigid
                                  pre-alignment keeps points. A captured iteration's Jacobian
                                  row of a surfel with several pairs is the first row of their
                                  4 x 4 factor (the sum of the pairs' Gram matrices is that of
                                  the factor's rows) */
} sw_config;

/* Statistics of one depth-map fusion (sw_fuse_frame). */
typedef struct sw_fusion_stats {
    int32_t n_fused;           /* depth surfels fused into a live surfel */
    int32_t n_candidates;      /* pixels with a normal that found no surfel (append candidates) */
} sw_fusion_stats;

/* Statistics of one append-candidate selection (sw_append_candidates). */
typedef struct sw_append_stats {
    int32_t n_candidates;      /* pixels with a normal that fusion matched to no surfel */
    int32_t n_far;             /* dropped: kept nearest-node weight sum below append_nn */
    int32_t n_compressive;     /* dropped: the warp back stretches by more than 1 + warp_eps */
    int32_t n_appended;        /* survivors */
    int32_t n_written;         /* survivors written (at most max_out) */
} sw_append_stats;

/* Statistics of one geometry update (sw_update_geometry). */
typedef struct sw_geometry_stats {
    int32_t n_removed;         /* existing surfels dropped as unstable */
    int32_t n_surfels;         /* surfels after the update */
    sw_append_stats append;    /* the append selection (all survivors appended) */
} sw_geometry_stats;

/* Per-frame statistics, one entry per Gauss-Newton iteration (<= 16). */
typedef struct sw_frame_stats {
    int32_t iters;             /* Gauss-Newton iterations run */
    float e_data[16];          /* E_depth at the iteration's linearisation point */
    float e_reg[16];           /* E_regulation (unweighted) at the same point */
    int32_t n_corr[16];        /* correspondences |P| */
    float pcg_resid[16];       /* |r| of the linear system when PCG stops */
    float stage_us[12];        /* with stage_timing: microseconds per kernel, summed
                                  over the frame: [0] depth preprocessing, [1] warp +
                                  index map, [2] correspondence + Jacobians +
                                  segment Gram matrices, [3] fused PCG steps
                                  (the last of an iteration also moves the
                                  nodes), [4] block-Jacobi + PCG start (0: it
                                  runs inside the assembly), [5] PCG products,
                                  [6] PCG finishes, [7] node update of streams
                                  without PCG iterations, [8] assembly of the
                                  blocks with the block-Jacobi + PCG start,
                                  [9] rigid warp + index map, [10] rigid 6x6 sums,
                                  [11] rigid solve + composition; measured with HIP
                                  events */
    double alg_bytes;          /* algorithmic bytes moved by the frame (model) */
    int32_t rigid_steps;       /* rigid alignment steps run */
    float rigid_e[16];         /* point-to-plane energy at each rigid step */
    int32_t rigid_n[16];       /* correspondences at each rigid step */
} sw_frame_stats;

/* Fill *cfg with the defaults listed in sw_config. */
void sw_config_default(sw_config* cfg);

/* Static description of a status code. */
const char* sw_status_string(sw_status st);

/* Message of the last failed call on s (empty if none; never NULL). */
const char* sw_last_error(sw_stream s);

/* Create a stream: the state of one depth camera's reconstruction, its
 * reference surfels and node-graph warp field (Sec. 3, Sec. 4), solved once
 * per depth frame (Sec. 7, Sec. 8) with the camera intrinsics and solver
 * parameters of the config (Table 1). hip_stream is the hipStream_t all work
 * is queued on, or NULL for a stream the library creates and destroys. The
 * config is copied. SW_EINVAL: image size <= 0, non-finite or non-positive
 * focal lengths, iteration counts out of range, non-positive sigma, negative
 * weights. */
sw_status sw_create_stream(const sw_config* cfg, void* hip_stream, sw_stream* out);

/* Destroy a stream and free its device memory (if it is attached to a
 * server, after its submitted frames are done). NULL is a no-op. */
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
 * node's 8 nearest other nodes) and the block pattern of J^T J with its
 * segment layout, all on the device. The node order defines the node
 * indices. n_nodes in [9, 32768]; surfels must be set (SW_ESTATE otherwise).
 * A repeated call reuses the device memory of the stream's previous node set
 * and so first waits for all work on the device (as freeing it would). */
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

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * solve as sw_solve_frame, with the same results bit for bit, whose per-frame
 * workspace (normal map, index map, Gram partials, blocks, PCG vectors,
 * statistics) is taken from a static device array of 64 MiB held by the
 * library on each GPU it runs on until the process ends, instead of the
 * stream's own workspace. The call allocates nothing. Inputs and outputs
 * are as for sw_solve_frame; the stream's resident state (surfels, nodes,
 * graph) is its own as always. Returns SW_EINVAL if the stream's frame
 * workspace (sw_get_footprint) exceeds 64 MiB, SW_EHIP if the array's
 * device address cannot be found. Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (each call initialises what it
 * reads): calls that overlap on one GPU (from several host threads or on
 * several HIP streams at once) race and must not be made. Synchronous. */
sw_status sw_solve_frame_noalloc(sw_stream s, const float* depth, int32_t on_device,
                                 sw_frame_stats* stats);

/* ---- surfel attributes and depth-map fusion (Sec. 5, Sec. 6.1, Sec. 6.4) ---- */

/* Radius (m), confidence, last observed frame and initialisation frame of
 * every surfel, in the caller's surfel order (n = the count given to
 * sw_set_reference_surfels); any pointer may be NULL to keep that attribute.
 * Defaults after sw_set_reference_surfels: radius 0, confidence 1,
 * t_observed 0, t_init 0. Setting surfels again resets them. The data is
 * copied. A radius must be finite and >= 0 (0 = an unsized point): any other
 * value returns SW_EINVAL and leaves every attribute unchanged. */
sw_status sw_set_surfel_attributes(sw_stream s, int64_t n, const float* radius, const float* confidence,
                                   const int32_t* t_observed, const int32_t* t_init, int32_t on_device);

/* Read the attributes (caller order, host arrays of n entries; NULL skips). */
sw_status sw_get_surfel_attributes(sw_stream s, float* radius, float* confidence, int32_t* t_observed,
                                   int32_t* t_init);

/* Read the reference surfels (n x 3 positions and normals, caller order, host):
 * the ones given, as updated by sw_fuse_frame. */
sw_status sw_get_reference_surfels(sw_stream s, float* pos, float* nrm);

/* Current frame time t_now, used by visibility = 1 (recently observed
 * surfels). sw_fuse_frame also sets it. */
sw_status sw_set_frame_time(sw_stream s, int32_t t_now);

/* Fuse a depth image into the surfels at the current warp field (call after
 * sw_solve_frame on the same depth). Every pixel with a normal gives a depth
 * surfel: position V(u), normal N(u), confidence exp(-gamma^2 / (2 * 0.6^2)),
 * gamma = |u - c| / |c| (c the principal point), radius
 * sqrt(2) d / (fx max(|n_z|, cos 75 deg)). The live surfels are rendered as
 * points into an index map super-sampled 4 x 4 (nearest z, then lower
 * index); each pixel takes the surfels of its 4 x 4 block that lie within
 * fusion_dist of V(u) with n . N(u) >= fusion_normal, and the one with the
 * highest confidence, then the closest, then the lowest index, receives the
 * depth surfel: confidence adds, t_observed = t_now, position, normal
 * (renormalised) and radius become confidence-weighted means. Fused surfels
 * return to the reference frame through the inverse of their blended
 * transform (skinning kept). Synchronous. stats may be NULL. SW_ESTATE
 * without a node graph or while attached to a server. */
sw_status sw_fuse_frame(sw_stream s, const float* depth, int32_t on_device, int32_t t_now,
                        sw_fusion_stats* stats);

/* Parity export of the last fusion: per pixel the caller index of the surfel
 * fused there or -1 (H x W), and the live positions and normals the match
 * used (n x 3 each, caller order; NaN positions for surfels without a valid
 * blend). Any pointer may be NULL. SW_ESTATE before the first fusion. */
sw_status sw_get_last_fusion(sw_stream s, int32_t* match_map, float* live_pos, float* live_nrm);

/* Append candidates of the last fusion (Sec. 6.2 - 6.4), at the current warp
 * field. A candidate is a pixel with a normal that the fusion matched to no
 * surfel. It is skinned to its 4 nearest live node positions c_j = T_j p_j
 * (ties to the lower index); node i of the set stays only if
 * (1 - warp_eps)^2 |p_i - p_0|^2 < |c_i - c_0|^2 < (1 + warp_eps)^2 |p_i - p_0|^2
 * (Eq. 7; the nearest node always stays). It is dropped if the Gaussian
 * weights exp(-|V - c_j|^2 / (2 node_sigma^2)) of the kept nodes sum to less
 * than append_nn, or if the warp back to the reference frame (the inverse of
 * the normalised blend of the kept nodes, weights at the point) has a
 * derivative, taken by central differences with a 1 mm step, whose largest
 * singular value exceeds 1 + warp_eps (Eq. 8). Survivors come in row-major
 * pixel order: pixel index y * W + x, reference position and normal
 * (3 floats each), the depth surfel's radius and confidence (as in
 * sw_fuse_frame). At most max_out are written (host arrays with on_device = 0,
 * device arrays on the stream's HIP stream with 1); stats->n_appended counts
 * all. They are not added to the stream: the caller appends them to its
 * surfels (sw_set_reference_surfels, sw_set_surfel_attributes with
 * t_observed = t_now, then sw_set_node_graph with the current transforms).
 * Synchronous. SW_ESTATE unless the stream's last depth frame was fused (a
 * solve in between replaces the frame) or while attached to a server. */
sw_status sw_append_candidates(sw_stream s, int32_t max_out, int32_t on_device, int32_t* pixel, float* pos,
                               float* nrm, float* radius, float* confidence, sw_append_stats* stats);

/* Live node positions T_k p_k at the current transforms (n_nodes x 3, host). */
sw_status sw_get_live_nodes(sw_stream s, float* pos);

/* Geometry update after a fusion (Sec. 6.4 and the GPU selection of Sec. 6.7),
 * on the device: existing surfels whose confidence is below stable_conf more
 * than t_low_confid frames after their t_init are dropped; the survivors of
 * the append selection of the last fusion (as sw_append_candidates) are
 * appended with t_init = t_observed = t_now; the surfel array becomes the
 * kept surfels in their caller order followed by the appended ones in pixel
 * order, and every surfel is skinned again to the same nodes, whose
 * transforms are kept bit for bit (the node graph itself is not extended).
 * Caller indices change accordingly; read the new surfels with
 * sw_get_reference_surfels / sw_get_surfel_attributes. Synchronous. SW_ESTATE
 * as sw_append_candidates; SW_EINVAL if no surfel would remain or the count
 * would exceed the library's limit (nothing is changed then). */
sw_status sw_update_geometry(sw_stream s, sw_geometry_stats* stats);

/* ---- batches: frames of several streams solved together ----
 *
 * A batch executor launches each Gauss-Newton stage once for all the streams
 * of a call: the grid is the concatenation of every stream's tiles and each
 * workgroup reads its stream's descriptor, so a stream's result does not
 * depend on what it is batched with. Streams may differ in image size,
 * surfel and node counts and iteration counts. An executor owns a HIP stream
 * (or uses the caller's), a small statistics buffer and timing events; it is
 * not thread-safe, and a stream must not be solved by two calls at once. */
typedef struct sw_batch_s* sw_batch;

#define SW_BATCH_TIMING 1   /* time every launch with HIP events into stage_us */
#define SW_BATCH_GRAPH  2   /* replay a batch's Gauss-Newton iterations as one HIP graph */
#define SW_BATCH_PCG_SPLIT 4   /* every PCG iteration as a product and a finish launch */
#define SW_BATCH_PCG_FUSED 8   /* every PCG iteration as one fused step launch */

/* Create an executor. hip_stream as in sw_create_stream; flags: 0,
 * SW_BATCH_TIMING (then every stream's stage_us holds the times of the
 * batch's launches, summed over the frame) or SW_BATCH_GRAPH: the launches
 * of all Gauss-Newton iterations and the statistics copy are captured as one
 * HIP graph the first time a batch (the same streams in the same order) is
 * solved, and the graph is replayed while the batch and its streams'
 * buffers are unchanged (a new batch, or sw_set_reference_surfels /
 * sw_set_node_graph on a member, captures anew). Results are identical to
 * the launch-by-launch path. Not combinable with SW_BATCH_TIMING (EINVAL);
 * streams that capture an iteration (debug_iter) run launch by launch.
 * SW_BATCH_PCG_SPLIT or SW_BATCH_PCG_FUSED (not both) fix the PCG schedule,
 * which is otherwise chosen per batch shape (the autotuner's choice, else
 * fused steps up to 8192 nodes in all); both give identical results. */
sw_status sw_create_batch(void* hip_stream, int32_t flags, sw_batch* out);

/* Destroy an executor (NULL is a no-op). Streams are not affected. */
sw_status sw_destroy_batch(sw_batch b);

/* Message of the last failed call on b (never NULL). */
const char* sw_batch_last_error(sw_batch b);

/* Solve one frame for each of n distinct streams (1 <= n <= 64): depths[i]
 * is stream i's H_i x W_i image, all host (on_device = 0) or all device
 * memory readable on the executor's HIP stream. Synchronous. Each stream
 * ends exactly as sw_solve_frame would leave it. stats (n entries) and
 * status (n entries, per-stream result) may be NULL. Returns SW_OK, or
 * SW_ENUMERIC when one or more streams failed numerically (those keep their
 * transforms from before the call, the others are updated), or an argument /
 * state / runtime error before or during the launches. */
sw_status sw_solve_batch(sw_batch b, const sw_stream* streams, int32_t n,
                         const float* const* depths, int32_t on_device,
                         sw_frame_stats* stats, sw_status* status);

/* Measurement: launch one per-frame stage of the batch reps times back to
 * back (after one untimed launch) between two HIP events and return the mean
 * time per launch in microseconds. The streams' frame workspaces are
 * overwritten (their warp fields are not); use after a solve, so that the
 * stage's inputs hold a real frame. stage numbers as in stage_us: 1 warp +
 * index map, 2 correspondence + Jacobians + segment Gram matrices,
 * 4 block-Jacobi + PCG start as a launch of its own (a solve runs it inside
 * the fold), 5 PCG products (u = A z, v = A p_prev),
 * 6 PCG finish (scalars, x, r, z, p), 8 block fold, 13 fused PCG step
 * (finish of iteration pcg_it - 1 and products of pcg_it in one launch,
 * pcg_it >= 1); others give SW_EINVAL. pcg_it selects the PCG iteration for
 * 5, 6 and 13. */
sw_status sw_profile_stage(sw_batch b, const sw_stream* streams, int32_t n, int32_t stage,
                           int32_t pcg_it, int32_t reps, float* us_per_launch);

/* Autotuner: for the shape bucket of this batch (stream count and the
 * powers of two of its total surfels and nodes) time each per-frame stage
 * (1 warp, 2 correspondence, 8 fold, 5 product, 6 finish, 13 fused step)
 * reps times back to back in each launch variant and keep the
 * fastest for later solves of batches in that bucket on this executor.
 * Variants: the tile order — linear, or XCD-contiguous (the workgroups an XCD
 * runs take one contiguous range of tiles, keeping a stream's data in few L2
 * caches) — and, for the product and the finish, 1 or 2 block rows per wave
 * / nodes per lane group; then the PCG schedule — one fused step per
 * iteration, or a product and a finish launch — by the faster sum. Every
 * variant computes the same tiles with the same reductions, so results do
 * not change. Use after a solve of the batch (the stages replay its last
 * frame; workspaces are overwritten, warp fields are not). variants (NULL or
 * 12 entries, indexed like stage_us) receives the choices: bit 0 =
 * XCD-contiguous order, bit 1 = 2 rows / nodes, bit 2 (entry 5) = fused PCG
 * steps. */
sw_status sw_batch_autotune(sw_batch b, const sw_stream* streams, int32_t n, int32_t reps,
                            int32_t* variants);

/* ---- serving: frames of many streams arriving at any time ----
 *
 * A server owns a HIP stream (or uses the caller's), one device slab for the
 * workspaces of frames in flight and a worker thread. Streams are attached
 * to it; frames are submitted with sw_server_submit and collected with
 * sw_server_poll. A frame is admitted when its stream has no frame in flight,
 * a batch slot is free and the stream's workspace (its footprint) fits in a
 * free range of the slab; frames are admitted in arrival order as slots and
 * memory free up. Every step runs one Gauss-Newton iteration of all frames in
 * flight in the same launches, so a frame that arrives while others are on
 * the GPU joins them at the next iteration. A frame's result is the same as
 * sw_solve_frame's alone. The server's functions are thread-safe. */
typedef struct sw_server_config {
    int32_t max_batch;          /* frames in flight at most, 1..64 (default 32) */
    int32_t reserved;
    int64_t workspace_bytes;    /* device slab for frame workspaces (default 4 GiB) */
} sw_server_config;

typedef struct sw_ticket_info {
    sw_status status;           /* the frame's result (as sw_solve_frame's) */
    int32_t reserved;
    double t_submit, t_admit, t_done;   /* seconds since the server was created
                                           (monotonic clock) */
} sw_ticket_info;

typedef struct sw_server_info {
    int64_t steps;              /* Gauss-Newton steps run */
    int64_t frames_done;
    int32_t max_in_flight;      /* most frames in flight at once so far */
    int32_t pending;            /* frames waiting for admission now */
    int32_t in_flight;          /* frames in flight now */
    int32_t reserved;
    int64_t workspace_bytes;    /* slab size */
    int64_t workspace_peak;     /* most slab bytes in use at once so far */
} sw_server_info;

void sw_server_config_default(sw_server_config* cfg);

/* Create a server on the current device. SW_EINVAL for max_batch outside
 * 1..64 or a slab under 4 KiB; SW_ENOMEM if the slab cannot be allocated. */
sw_status sw_create_server(const sw_server_config* cfg, void* hip_stream, sw_server* out);

/* Wait for every submitted frame, stop the worker, give attached streams
 * their own workspace back and free the slab. NULL is a no-op. */
sw_status sw_destroy_server(sw_server sv);

const char* sw_server_last_error(sw_server sv);

/* Attach a stream (surfels and node graph set): its own frame workspace is
 * freed and its frames run in the slab from now on. While attached the
 * stream's sw_set_* and sw_solve_frame calls return SW_ESTATE, and its
 * readers wait until its submitted frames are done. SW_EINVAL if its
 * workspace exceeds the slab. */
sw_status sw_server_attach(sw_server sv, sw_stream s);

/* Wait for the stream's frames, then give it its own workspace back. */
sw_status sw_server_detach(sw_server sv, sw_stream s);

/* Queue one frame of an attached stream. A host image is copied before the
 * call returns; a device image must stay readable and unchanged until the
 * frame is done. *ticket identifies the frame for sw_server_poll. */
sw_status sw_server_submit(sw_server sv, sw_stream s, const float* depth, int32_t on_device,
                           uint64_t* ticket);

/* Result of a frame: waits up to wait_ms (0 = do not wait, -1 = until done).
 * SW_OK when done (stats and info filled, either may be NULL; the ticket is
 * then released), SW_EPENDING while not done, SW_EINVAL for an unknown
 * ticket. */
sw_status sw_server_poll(sw_server sv, uint64_t ticket, int32_t wait_ms, sw_frame_stats* stats,
                         sw_ticket_info* info);

/* Counters of the server so far. */
sw_status sw_server_counters(sw_server sv, sw_server_info* out);

/* Copy the node transforms T_j of the warp field (Sec. 3; the result of the
 * last solve, Sec. 7) to host memory out (n_nodes x 12 fp32 [R | t], caller's
 * node order). SW_EINVAL if capacity (in nodes) < n_nodes. */
sw_status sw_get_node_se3(sw_stream s, float* out, int32_t capacity);

/* Sizes of the current problem (any pointer may be NULL). */
sw_status sw_get_sizes(sw_stream s, int64_t* n_surfels, int32_t* n_nodes, int32_t* n_blocks);

/* Device memory of the stream: resident state (surfels, skinning, node state,
 * graph, block pattern, work lists, capture buffers, and the temporaries of
 * the last node-set build, whose memory the next build reuses) and the
 * workspace one frame in flight needs (the admission footprint of
 * sw_server_attach).
 * SW_ESTATE before sw_set_node_graph. */
sw_status sw_get_footprint(sw_stream s, int64_t* resident_bytes, int64_t* workspace_bytes);

/* Work layout chosen at sw_set_node_graph: distinct node sets; segments (runs
 * of surfels with at most 5 nodes in all, each summed into one Gram matrix);
 * packs (runs of whole segments, at most 232 surfels, one workgroup each);
 * the ELL width of the product's rows; the block fold's entries (one per
 * node pair of a segment); the floats of all segments' Gram output. */
typedef struct sw_layout {
    int32_t node_sets, segments, packs, ell_width;
    int64_t fold_entries, gram_floats;
} sw_layout;

sw_status sw_get_layout(sw_stream s, sw_layout* out);

/* Self-check of the segment layout, for tests: sw_set_node_graph cuts the
 * sorted surfels into segments and packs on the device (greedy cuts walked as
 * successor chains); this call redoes the cut with the plain sequential walk
 * on the host, from the same sorted surfels and block pattern, and writes
 * into differ[9] the number of differing elements (plus any difference in
 * length) of: segment starts, pair masks, Gram offsets (and their total),
 * block entry pointers, entry sub-block offsets, entry J^T r offsets, pack
 * starts, pack first segments, per-surfel node positions. All zero means the
 * two agree exactly. Synchronises the stream; host memory of order the
 * surfel count. */
sw_status sw_check_layout(sw_stream s, int64_t* differ);

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

/* Live normals of the captured iteration (Sec. 3, Eq. 2: the blended rotation
 * applied to each reference normal): n_surfels x 3 fp32 in the caller's
 * surfel order, NaN where the blend is undefined. These, with the live
 * positions above, are the inputs of every decision the correspondence step
 * takes (Sec. 7: the normal-angle gate). live_nrm is a host array owned by
 * the caller. SW_ESTATE if nothing was captured. */
sw_status sw_get_last_live_normals(sw_stream s, float* live_nrm);

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
