// Arguments of the depth-map fusion kernels of one stream (see fusion.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "swgn_impl.h"

namespace swgn {

constexpr float kFusePhi = 0.6f;      // depth-surfel confidence exp(-gamma^2 / (2 phi^2))

struct FuseArgs {
    int ns;
    int t_now;
    Cam cam;
    float dist2;                  // (float)delta_d * (float)delta_d
    float cosn;                   // delta_n
    float cos_max;                // cos 75 deg: the radius clamp
    // resident, sorted by node set (orig = caller index, inv its inverse)
    const int4* idx;
    const float4* w;
    const float4* dq;
    const int* orig;
    const int* inv;
    float *px, *py, *pz, *nx, *ny, *nz;     // reference surfels, updated where fused
    float *radius, *conf;
    int* t_obs;
    // frame
    const float4* nmap;           // (normal, depth) per pixel; depth 0 = no normal
    unsigned long long* zmap4;    // [4H][4W] index map
    float *lx, *ly, *lz, *lnx, *lny, *lnz;  // live surfels before fusion
    int* match;                   // [H][W] caller index fused at the pixel, -1
    int* counts;                  // [0] fused, [1] append candidates
    // caller-order copies kept current (the inputs a later node graph sorts from)
    float *cpos, *cnrm, *crad, *cconf;
    int* ctobs;
};

void launch_fuse(const FuseArgs& a, hipStream_t st);

// Arguments of the append-candidate kernels (see append.hip).
struct AppendArgs {
    Cam cam;
    int nn;
    int max_out;                  // capacity of the out_ arrays
    float eps;                    // intrinsic deformation bound of Eq. 7 / Eq. 8
    float delta_nn;               // weight-sum threshold
    float inv2s2;                 // 1 / (2 sigma^2)
    float cos_max;                // cos 75 deg: the radius clamp
    const float4* nmap;           // (normal, depth) per pixel of the fused frame
    const int* match;             // [H][W] fused surfel per pixel, -1
    const float4* cl;             // live node positions
    const float4* pref;           // reference node positions
    const float4* dq;             // node dual quaternions
    const int* node_id;           // [nn] the caller's index of each node (ties go to the lower)
    const int* node_inv;          // [nn] the library's index of each caller index
    int* flag;                    // [npx + 1] survivor flags (the last stays 0)
    float4 *sv, *sn;              // [npx] reference position / normal of survivors
    int* counts;                  // [0] candidates, [1] far, [2] compressive
    int* out_pixel;
    float *out_pos, *out_nrm, *out_rad, *out_conf;
};

// Evaluation, exclusive scan of the flags into pos[npx + 1] (pos[npx] = the
// number of survivors) and compaction.
void launch_append(const AppendArgs& a, int* pos, int* scan_tmp, hipStream_t st);

// flag[i] = 1 for the existing surfels a geometry update keeps (caller order).
void launch_keep_mark(int ns, const float* conf, const int* tinit, int t_now, float stable, int t_low, int* flag,
                      hipStream_t st);

// Arguments of the compaction of a geometry update: the kept surfels (flag,
// exclusive-scan positions pos) and napp appended ones into fresh arrays.
struct CompactArgs {
    int ns, nkeep, napp, t_now;
    const int *flag, *pos;
    const float *spos, *snrm, *srad, *sconf;
    const int *stobs, *stinit;
    const float *apos, *anrm, *arad, *aconf;
    float *dpos, *dnrm, *drad, *dconf;
    int *dtobs, *dtinit;
};

void launch_compact_surfels(const CompactArgs& c, hipStream_t st);

// Node positions as float4 -> packed x, y, z.
void launch_f4_to_positions(int n, const float4* in, float* out, hipStream_t st);

// Sorted copies of the caller-order attributes (sorted i takes caller
// orig[i]) and the inverse permutation inv[orig[i]] = i.
void launch_fuse_gather(int ns, const int* orig, const float* crad, const float* cconf, const int* ctobs,
                        float* rad, float* conf, int* tobs, int* inv, hipStream_t st);

}  // namespace swgn
