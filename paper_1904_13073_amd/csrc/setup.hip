// Setup kernels, run once per node set (Sec. 6.5, Initialization): skinning of
// every surfel to its nearest nodes, the node graph, and the block pattern of
// J^T J with the per-block lists the assembly walks.
//
// Every integer result is deterministic: nearest-node order is decided by an
// FP32 key with a fixed operation order and ties to the lower index; sorts
// compare full (key, value) pairs that are unique; the only atomics are
// integer OR / ADD whose results do not depend on order.
#include "swgn_impl.h"
#include "swgn_launch.h"
#include "swgn_setup.h"

namespace swgn {

// ---------------------------------------------------------------------------
// Nearest nodes. Key ((dx*dx + dy*dy) + dz*dz), dx = x_query - x_node; the 4
// nearest are the 4 smallest (key, caller index) pairs, which is what a scan
// in ascending caller index that admits a candidate only strictly below the
// current fourth key gives. Here the nodes are scanned in the library's
// (Morton) order with candidates ordered by (key, caller index), so the
// result is the same whatever the order, and whole runs of 32 nodes are
// skipped when no lane of the wave can admit any of them: the wave first
// takes the runs whose bounding box meets its surfels' box (else the nearest
// one), then skips every other run whose box distance, less a margin above
// FP32 rounding, exceeds every lane's current fourth key (a candidate enters
// only at or below it).
// A non-finite position enters no list (its keys are NaN or infinite).
// ---------------------------------------------------------------------------
constexpr int kKnnTile = 1024;          // nodes staged in LDS per round
constexpr int kKnnRun = 32;             // nodes per bounding box

__global__ void k_node_boxes(int nn, const float4* __restrict__ nodes, float4* __restrict__ boxes) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q * kKnnRun >= nn) return;
    float3 lo = make_float3(INFINITY, INFINITY, INFINITY), hi = make_float3(-INFINITY, -INFINITY, -INFINITY);
    for (int t = q * kKnnRun; t < min(nn, (q + 1) * kKnnRun); ++t) {
        const float4 p = nodes[t];
        lo.x = fminf(lo.x, p.x); lo.y = fminf(lo.y, p.y); lo.z = fminf(lo.z, p.z);
        hi.x = fmaxf(hi.x, p.x); hi.y = fmaxf(hi.y, p.y); hi.z = fmaxf(hi.z, p.z);
    }
    boxes[2 * q] = make_float4(lo.x, lo.y, lo.z, 0.f);
    boxes[2 * q + 1] = make_float4(hi.x, hi.y, hi.z, 0.f);
}

__device__ __forceinline__ float wave_minf(float v) {
    v = fminf(v, xchg<32>(v)); v = fminf(v, xchg<16>(v)); v = fminf(v, xchg<8>(v));
    v = fminf(v, xchg<4>(v)); v = fminf(v, xchg<2>(v)); v = fminf(v, xchg<1>(v));
    return v;
}
__device__ __forceinline__ float wave_maxf(float v) {
    v = fmaxf(v, xchg<32>(v)); v = fmaxf(v, xchg<16>(v)); v = fmaxf(v, xchg<8>(v));
    v = fmaxf(v, xchg<4>(v)); v = fmaxf(v, xchg<2>(v)); v = fmaxf(v, xchg<1>(v));
    return v;
}

// A lower bound of every key between the wave's box (lo, hi) and a node box:
// each point pair is at least the boxes' gap apart per axis; the computed key
// is within 5 roundings of the exact sum of squares and so is this bound, so
// shrinking it by 2^-20 (and 1e-30 for tiny values) keeps it below every key.
__device__ __forceinline__ float box_key_bound(float3 lo, float3 hi, float4 blo, float4 bhi) {
    const float gx = fmaxf(fmaxf(lo.x - bhi.x, blo.x - hi.x), 0.f);
    const float gy = fmaxf(fmaxf(lo.y - bhi.y, blo.y - hi.y), 0.f);
    const float gz = fmaxf(fmaxf(lo.z - bhi.z, blo.z - hi.z), 0.f);
    const float d2 = (gx * gx + gy * gy) + gz * gz;
    return d2 * (1.0f - 0x1p-20f) - 1e-30f;
}

// A candidate as one 64-bit word, (key bits, index): keys are >= +0 or +inf
// or NaN, whose bit patterns order as the values do and sort NaN last, so
// comparing words compares (key, index) pairs, ties to the lower index.
__device__ __forceinline__ uint64_t knn_word(float key, int j) {
    return ((uint64_t)__float_as_uint(key) << 32) | (uint32_t)j;
}

// A word into the 4 smallest kept ascending, by selects only (the list stays
// in registers): the words below it stay, it takes the first place above
// them, the rest move down one.
__device__ __forceinline__ void admit4(uint64_t (&kk)[4], uint64_t c) {
    if (c >= kk[3]) return;
    const bool c0 = c < kk[0], c1 = c < kk[1], c2 = c < kk[2];
    kk[3] = c2 ? kk[2] : c;
    kk[2] = c1 ? kk[1] : (c2 ? c : kk[2]);
    kk[1] = c0 ? kk[0] : (c1 ? c : kk[1]);
    kk[0] = c0 ? c : kk[0];
}

__global__ void __launch_bounds__(256) k_knn_skin(int ns, const float* __restrict__ pos, int nn,
        const float4* __restrict__ nodes, const int* __restrict__ caller, const float4* __restrict__ boxes,
        float inv_two_sigma2, int4* __restrict__ out_idx, float4* __restrict__ out_w) {
    __shared__ float4 tile[kKnnTile];
    __shared__ int tid[kKnnTile];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    float x = 0.f, y = 0.f, z = 0.f;
    if (i < ns) { x = pos[3 * i]; y = pos[3 * i + 1]; z = pos[3 * i + 2]; }
    const bool fin = i < ns && isfinite(x) && isfinite(y) && isfinite(z);
    // (INFINITY, 0) admits no infinite key
    uint64_t kk[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) kk[q] = knn_word(INFINITY, 0);
    // the box of the wave's finite surfels (empty: every run is skipped)
    const float3 lo = make_float3(wave_minf(fin ? x : INFINITY), wave_minf(fin ? y : INFINITY),
                                  wave_minf(fin ? z : INFINITY));
    const float3 hi = make_float3(wave_maxf(fin ? x : -INFINITY), wave_maxf(fin ? y : -INFINITY),
                                  wave_maxf(fin ? z : -INFINITY));
    const int nruns = (nn + kKnnRun - 1) / kKnnRun;
    // first the runs whose box meets the wave's (or the nearest one)
    int seed = 0;
    float sb = INFINITY;
    for (int q = 0; q < nruns; ++q) {
        const float b = box_key_bound(lo, hi, boxes[2 * q], boxes[2 * q + 1]);
        if (b < sb) { sb = b; seed = q; }
        if (b > 0.f) continue;
        for (int t = q * kKnnRun; t < min(nn, (q + 1) * kKnnRun); ++t) {
            const float4 p = nodes[t];
            const float dx = x - p.x, dy = y - p.y, dz = z - p.z;
            admit4(kk, knn_word((dx * dx + dy * dy) + dz * dz, caller[t]));
        }
    }
    if (sb > 0.f) {
        for (int t = seed * kKnnRun; t < min(nn, (seed + 1) * kKnnRun); ++t) {
            const float4 p = nodes[t];
            const float dx = x - p.x, dy = y - p.y, dz = z - p.z;
            admit4(kk, knn_word((dx * dx + dy * dy) + dz * dz, caller[t]));
        }
    } else {
        seed = -1;                          // (the meeting runs are done)
    }
    for (int base = 0; base < nn; base += kKnnTile) {
        const int cnt = min(kKnnTile, nn - base);
        __syncthreads();
        for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
            tile[t] = nodes[base + t];
            tid[t] = caller[base + t];
        }
        __syncthreads();
        for (int r0 = 0; r0 < cnt; r0 += kKnnRun) {
            const int q = (base + r0) / kKnnRun;
            const float b = box_key_bound(lo, hi, boxes[2 * q], boxes[2 * q + 1]);
            if (q == seed || b <= 0.f) continue;
            // every lane's fourth key bounds what it could still admit
            const float worst = wave_maxf(fin ? __uint_as_float((uint32_t)(kk[3] >> 32)) : -INFINITY);
            if (b > worst) continue;
            for (int t = r0; t < min(cnt, r0 + kKnnRun); ++t) {
                const float4 p = tile[t];
                const float dx = x - p.x, dy = y - p.y, dz = z - p.z;
                admit4(kk, knn_word((dx * dx + dy * dy) + dz * dz, tid[t]));
            }
        }
    }
    float kd[4];
    int ki[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        kd[q] = __uint_as_float((uint32_t)(kk[q] >> 32));
        ki[q] = (int)(uint32_t)kk[q];
    }
    if (i >= ns) return;
    // weights exp(-(d_k^2 - d_0^2) / (2 sigma^2)), normalised
    float e0 = 1.0f;
    float e1 = expf(-(kd[1] - kd[0]) * inv_two_sigma2);
    float e2 = expf(-(kd[2] - kd[0]) * inv_two_sigma2);
    float e3 = expf(-(kd[3] - kd[0]) * inv_two_sigma2);
    float inv = 1.0f / (((e0 + e1) + e2) + e3);
    out_idx[i] = make_int4(ki[0], ki[1], ki[2], ki[3]);
    out_w[i] = make_float4(e0 * inv, e1 * inv, e2 * inv, e3 * inv);
}

// One wave per node j: lane l keeps the 8 nearest of the nodes l, l + 64, ...
// (ascending index, so equal keys keep the lower index first), then the wave
// merges its 64 sorted lists by taking, 8 times, the smallest (key, index)
// head: the same set and order as one sequential scan.
constexpr int kGraphNodesPerBlock = 4;

__global__ void __launch_bounds__(64 * kGraphNodesPerBlock) k_node_graph(int nn, const float4* __restrict__ nodes,
                                                                         int* __restrict__ nbr) {
    const int lane = threadIdx.x % kWave;
    const int j = blockIdx.x * kGraphNodesPerBlock + threadIdx.x / kWave;
    if (j >= nn) return;                     // whole waves: no barrier follows
    const float4 me = nodes[j];
    float kd[8];
    int ki[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) { kd[q] = INFINITY; ki[q] = 0x7fffffff; }
    for (int t = lane; t < nn; t += kWave) {
        if (t == j) continue;
        const float4 p = nodes[t];
        const float dx = me.x - p.x, dy = me.y - p.y, dz = me.z - p.z;
        knn_insert<8>(kd, ki, (dx * dx + dy * dy) + dz * dz, t);
    }
    int out = 0;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        float bk = kd[0];
        int bi = ki[0];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const float ok = __shfl_xor(bk, o, kWave);
            const int oi = __shfl_xor(bi, o, kWave);
            if (ok < bk || (ok == bk && oi < bi)) { bk = ok; bi = oi; }
        }
        if (lane == r) out = bi;
        if (ki[0] == bi) {                   // this lane's head was taken: shift its list
#pragma unroll
            for (int q = 0; q < 7; ++q) { kd[q] = kd[q + 1]; ki[q] = ki[q + 1]; }
            kd[7] = INFINITY;
            ki[7] = 0x7fffffff;
        }
    }
    if (lane < 8) nbr[8 * j + lane] = out;
}

// ---------------------------------------------------------------------------
// Bitonic sort of (u64 key, u32 val) pairs, ascending in (key, val).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool pair_less(uint64_t ka, uint32_t va, uint64_t kb, uint32_t vb) {
    return ka < kb || (ka == kb && va < vb);
}

// S consecutive stages j, j/2, ..., j/2^(S-1) of block size k in one pass:
// each thread holds the 2^S elements whose indices differ only in those S
// bits (all in one k-block, so one direction) and applies the stages to them
// in order, as the one-stage passes would.
template <int S>
__global__ void k_bitonic_global(uint64_t* __restrict__ key, uint32_t* __restrict__ val, int n, int k, int jlow) {
    constexpr int E = 1 << S;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (n >> S)) return;
    // insert S zero bits at the stage bits (jlow is the lowest stage)
    const int a = ((t & ~(jlow - 1)) << S) | (t & (jlow - 1));
    const bool asc = (a & k) == 0;
    uint64_t kk[E];
    uint32_t vv[E];
#pragma unroll
    for (int m = 0; m < E; ++m) {
        kk[m] = key[a + m * jlow];
        vv[m] = val[a + m * jlow];
    }
#pragma unroll
    for (int st = S - 1; st >= 0; --st) {
        const int d = 1 << st;              // partner offset in units of jlow
#pragma unroll
        for (int m = 0; m < E; ++m) {
            if (m & d) continue;
            const uint64_t ka = kk[m], kb = kk[m | d];
            const uint32_t va = vv[m], vb = vv[m | d];
            const bool sw = asc ? pair_less(kb, vb, ka, va) : pair_less(ka, va, kb, vb);
            kk[m] = sw ? kb : ka; kk[m | d] = sw ? ka : kb;
            vv[m] = sw ? vb : va; vv[m | d] = sw ? va : vb;
        }
    }
#pragma unroll
    for (int m = 0; m < E; ++m) {
        key[a + m * jlow] = kk[m];
        val[a + m * jlow] = vv[m];
    }
}

constexpr int kSortLds = 1024;  // elements per block in the LDS stages

// All stages with j < kSortLds for a given k (and, when k <= kSortLds, all k
// up to it) on one 1024-element slice held in LDS, 512 threads.
static_assert(kSortLds == 2 * 512, "one compare-exchange per thread and stage");
__global__ void __launch_bounds__(512) k_bitonic_lds(uint64_t* __restrict__ key,
        uint32_t* __restrict__ val, int n, int k_from, int k_to) {
    __shared__ uint64_t sk[kSortLds];
    __shared__ uint32_t sv[kSortLds];
    int base = blockIdx.x * kSortLds;
    for (int t = threadIdx.x; t < kSortLds; t += blockDim.x) {
        sk[t] = key[base + t];
        sv[t] = val[base + t];
    }
    __syncthreads();
    for (int k = k_from; k <= k_to; k <<= 1) {
        int jstart = min(k >> 1, kSortLds >> 1);
        for (int j = jstart; j > 0; j >>= 1) {
            // one pair per thread: the lower index has a 0 at bit j
            const int q = threadIdx.x;
            const int t = ((q & ~(j - 1)) << 1) | (q & (j - 1)), p = t + j;
            const bool asc = ((base + t) & k) == 0;
            const uint64_t ka = sk[t], kb = sk[p];
            const uint32_t va = sv[t], vb = sv[p];
            const bool sw = asc ? pair_less(kb, vb, ka, va) : pair_less(ka, va, kb, vb);
            if (sw) { sk[t] = kb; sk[p] = ka; sv[t] = vb; sv[p] = va; }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < kSortLds; t += blockDim.x) {
        key[base + t] = sk[t];
        val[base + t] = sv[t];
    }
}

void sort_pairs(uint64_t* key, uint32_t* val, int n_pow2, hipStream_t st) {
    // n_pow2 is a power of two >= kSortLds
    int blocks = n_pow2 / kSortLds;
    hipLaunchKernelGGL(k_bitonic_lds, dim3(blocks), dim3(512), 0, st, key, val, n_pow2, 2, kSortLds);
    for (int k = 2 * kSortLds; k <= n_pow2; k <<= 1) {
        // the stages j >= kSortLds, up to three per pass
        for (int j = k >> 1; j >= kSortLds;) {
            if (j >= 4 * kSortLds) {
                hipLaunchKernelGGL(k_bitonic_global<3>, dim3((n_pow2 / 8 + 255) / 256), dim3(256), 0, st,
                                   key, val, n_pow2, k, j / 4);
                j /= 8;
            } else if (j >= 2 * kSortLds) {
                hipLaunchKernelGGL(k_bitonic_global<2>, dim3((n_pow2 / 4 + 255) / 256), dim3(256), 0, st,
                                   key, val, n_pow2, k, j / 2);
                j /= 4;
            } else {
                hipLaunchKernelGGL(k_bitonic_global<1>, dim3((n_pow2 / 2 + 255) / 256), dim3(256), 0, st,
                                   key, val, n_pow2, k, j);
                j /= 2;
            }
        }
        hipLaunchKernelGGL(k_bitonic_lds, dim3(blocks), dim3(512), 0, st, key, val, n_pow2, k, k);
    }
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32 (n elements -> out[0..n], out[n] = total).
// ---------------------------------------------------------------------------
constexpr int kScanBlock = 1024;

__global__ void __launch_bounds__(kScanBlock) k_scan_block(const int* __restrict__ in, int* __restrict__ out,
                                                           int* __restrict__ sums, int n) {
    __shared__ int s[kScanBlock];
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    int v = i < n ? in[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int t = threadIdx.x >= off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = s[threadIdx.x] - v;
    if (threadIdx.x == kScanBlock - 1) sums[blockIdx.x] = s[threadIdx.x];
}

__global__ void k_scan_add(int* __restrict__ out, const int* __restrict__ offs, int n) {
    int i = blockIdx.x * kScanBlock + threadIdx.x;
    if (i < n) out[i] += offs[blockIdx.x];
}

__global__ void k_scan_total(int* __restrict__ out, const int* __restrict__ in, int n) {
    out[n] = (n > 0 ? out[n - 1] + in[n - 1] : 0);
}

void exclusive_scan(const int* in, int* out, int n, int* tmp, hipStream_t st) {
    // tmp must hold scan_tmp_size(n) ints
    int nb = (n + kScanBlock - 1) / kScanBlock;
    if (n <= 0) {
        hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, in, 0);
        return;
    }
    int* sums = tmp;
    int* sums_scan = tmp + nb;
    hipLaunchKernelGGL(k_scan_block, dim3(nb), dim3(kScanBlock), 0, st, in, out, sums, n);
    if (nb > 1) {
        exclusive_scan(sums, sums_scan, nb, tmp + 2 * nb + 1, st);
        hipLaunchKernelGGL(k_scan_add, dim3(nb), dim3(kScanBlock), 0, st, out, sums_scan, n);
    }
    hipLaunchKernelGGL(k_scan_total, dim3(1), dim3(1), 0, st, out, in, n);
}

size_t scan_tmp_size(int n) {
    size_t total = 0;
    while (n > 1) {
        int nb = (n + kScanBlock - 1) / kScanBlock;
        total += 2 * (size_t)nb + 1;
        n = nb;
    }
    return total + 4;
}

// ---------------------------------------------------------------------------
// Surfel ordering by node set
// ---------------------------------------------------------------------------
__device__ __forceinline__ void sort4(int& a, int& b, int& c, int& d) {
    int t;
#define SWGN_CS(p, q) if (p > q) { t = p; p = q; q = t; }
    SWGN_CS(a, b) SWGN_CS(c, d) SWGN_CS(a, c) SWGN_CS(b, d) SWGN_CS(b, c)
#undef SWGN_CS
}

__global__ void k_tuple_keys(int ns, int npad, const int4* __restrict__ idx, uint64_t* __restrict__ key,
                             uint32_t* __restrict__ val) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npad) return;
    if (i >= ns) {
        key[i] = ~0ull;
        val[i] = 0xffffffffu;
        return;
    }
    int4 q = idx[i];
    int a = q.x, b = q.y, c = q.z, d = q.w;
    sort4(a, b, c, d);
    key[i] = ((uint64_t)a << 48) | ((uint64_t)b << 32) | ((uint64_t)c << 16) | (uint64_t)d;
    val[i] = (uint32_t)i;
}

// Gather surfel arrays into sorted order; flag run starts.
__global__ void k_permute_surfels(int ns, int seg_len, const uint64_t* __restrict__ key, const uint32_t* __restrict__ val,
        const float* __restrict__ ipos, const float* __restrict__ inrm, const int4* __restrict__ iidx,
        const float4* __restrict__ iw, float* __restrict__ px, float* __restrict__ py, float* __restrict__ pz,
        float* __restrict__ nx, float* __restrict__ ny, float* __restrict__ nz, int4* __restrict__ oidx,
        float4* __restrict__ ow, int* __restrict__ orig, int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    int o = (int)val[i];
    px[i] = ipos[3 * o + 0]; py[i] = ipos[3 * o + 1]; pz[i] = ipos[3 * o + 2];
    nx[i] = inrm[3 * o + 0]; ny[i] = inrm[3 * o + 1]; nz[i] = inrm[3 * o + 2];
    oidx[i] = iidx[o];
    ow[i] = iw[o];
    orig[i] = o;
    // run starts: a new node set (or, with seg_len > 0, every seg_len-th surfel)
    flag[i] = (i == 0 || key[i] != key[i - 1] || (seg_len > 0 && (i % seg_len) == 0)) ? 1 : 0;
}

__global__ void k_run_starts(int ns, const int* __restrict__ flag, const int* __restrict__ pos,
                             int* __restrict__ run_start) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ns && flag[i]) run_start[pos[i]] = i;
    if (i == 0) run_start[pos[ns]] = ns;
}

// The node set of every run (its first surfel's key).
__global__ void k_set_keys(int nsets, const uint64_t* __restrict__ key, const int* __restrict__ run_start,
                           uint64_t* __restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nsets) out[r] = key[run_start[r]];
}

// Positions (3 bits each) of surfel i's 4 nodes, in its slot order, among
// its segment's nodes; the segment is found by binary search over the
// segment starts. A node missing from the segment sets *bad.
__global__ void k_seg_pos4(int ns, int nseg, const int* __restrict__ seg_start, const int* __restrict__ seg_nodes,
                           const int4* __restrict__ idx, uint16_t* __restrict__ pos4, int* __restrict__ bad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ns) return;
    int lo = 0, hi = nseg - 1;                 // largest g with seg_start[g] <= i
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (seg_start[mid] <= i) lo = mid;
        else hi = mid - 1;
    }
    int nd[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) nd[q] = seg_nodes[5 * lo + q];
    const int4 t = idx[i];
    const int id[4] = {t.x, t.y, t.z, t.w};
    int code = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        int p = 5;
#pragma unroll
        for (int q = 4; q >= 0; --q)
            if (nd[q] == id[k]) p = q;
        ok = ok && p < 5;
        code |= (p < 5 ? p : 0) << (3 * k);
    }
    pos4[i] = (uint16_t)code;
    if (!ok) atomicOr(bad, 1);
}

// ---------------------------------------------------------------------------
// Block pattern: bitmap of the upper triangle, one row of nn bits per node.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void set_bit(uint32_t* bm, int words, int r, int c) {
    atomicOr(&bm[(size_t)r * words + (c >> 5)], 1u << (c & 31));
}

__global__ void k_pattern_runs(int nruns, const uint64_t* __restrict__ key, const int* __restrict__ run_start,
                               uint32_t* __restrict__ bm, int words) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nruns) return;
    uint64_t k = key[run_start[r]];
    int t[4] = {(int)(k >> 48), (int)((k >> 32) & 0xffff), (int)((k >> 16) & 0xffff), (int)(k & 0xffff)};
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = a + 1; b < 4; ++b) set_bit(bm, words, t[a], t[b]);
}

__global__ void k_pattern_nodes(int nn, const int* __restrict__ nbr, uint32_t* __restrict__ bm, int words) {
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nn) return;
    set_bit(bm, words, j, j);
    for (int q = 0; q < 8; ++q) {
        int m = nbr[8 * j + q];
        set_bit(bm, words, min(j, m), max(j, m));
    }
}

__global__ void k_row_counts(int nn, const uint32_t* __restrict__ bm, int words, int* __restrict__ cnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nn) return;
    int c = 0;
    for (int w = 0; w < words; ++w) c += __popc(bm[(size_t)r * words + w]);
    cnt[r] = c;
}

__global__ void k_row_fill(int nn, const uint32_t* __restrict__ bm, int words, const int* __restrict__ row_ptr,
                           int* __restrict__ col_idx, int* __restrict__ blk_row) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nn) return;
    int p = row_ptr[r];
    for (int w = 0; w < words; ++w) {
        uint32_t m = bm[(size_t)r * words + w];
        while (m) {
            int b = __ffs(m) - 1;
            m &= m - 1;
            col_idx[p] = w * 32 + b;
            blk_row[p] = r;
            ++p;
        }
    }
}

__global__ void k_pad_keys(uint64_t* __restrict__ key, uint32_t* __restrict__ val, int from, int to) {
    int i = from + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= to) return;
    key[i] = ~0ull;
    val[i] = 0xffffffffu;
}

// Transposed uses of the upper off-diagonal blocks, keyed by (col, row).
__global__ void k_transpose_keys(int nb, const int* __restrict__ blk_row, const int* __restrict__ col_idx,
                                 uint64_t* __restrict__ tkey, uint32_t* __restrict__ tval,
                                 int* __restrict__ tcount) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    int r = blk_row[b], c = col_idx[b];
    if (r == c) {
        tkey[b] = ~0ull;
        tval[b] = 0xffffffffu;
        return;
    }
    tkey[b] = ((uint64_t)c << 32) | (uint64_t)r;
    tval[b] = (uint32_t)b;
    atomicAdd(&tcount[c], 1);
}

__global__ void k_full_counts(int nn, const int* __restrict__ row_ptr, const int* __restrict__ tcount,
                              int* __restrict__ fcount) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nn) fcount[r] = tcount[r] + (row_ptr[r + 1] - row_ptr[r]);
}

// Fill full rows: first the transposed blocks (ascending row), then the upper ones.
__global__ void k_full_fill_t(int ntr, const uint64_t* __restrict__ tkey, const uint32_t* __restrict__ tval,
                              const int* __restrict__ tstart, const int* __restrict__ frow_ptr,
                              uint32_t* __restrict__ fblk, int* __restrict__ fcol) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ntr) return;
    int c = (int)(tkey[i] >> 32);
    int r = (int)(tkey[i] & 0xffffffffull);
    int slot = frow_ptr[c] + (i - tstart[c]);
    fblk[slot] = tval[i] | kTransposed;
    fcol[slot] = r;
}

__global__ void k_full_fill_u(int nn, const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                              const int* __restrict__ tcount, const int* __restrict__ frow_ptr,
                              uint32_t* __restrict__ fblk, int* __restrict__ fcol) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nn) return;
    int p = frow_ptr[r] + tcount[r];
    for (int b = row_ptr[r]; b < row_ptr[r + 1]; ++b) {
        fblk[p] = (uint32_t)b;
        fcol[p] = col_idx[b];
        ++p;
    }
}

// ---------------------------------------------------------------------------
// Node-graph in-edges and ELL rows
// ---------------------------------------------------------------------------
// in-edges of every node: (m << 32 | j) keys for every edge j -> m
__global__ void k_in_edge_keys(int nn, int npad, const int* __restrict__ nbr, uint64_t* __restrict__ key,
                               uint32_t* __restrict__ val, int* __restrict__ icount) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= npad) return;
    if (e >= 8 * nn) {
        key[e] = ~0ull;
        val[e] = 0xffffffffu;
        return;
    }
    int j = e / 8, m = nbr[e];
    key[e] = ((uint64_t)m << 32) | (uint64_t)j;
    val[e] = (uint32_t)j;
    atomicAdd(&icount[m], 1);
}

__global__ void k_in_edge_store(int n, const uint32_t* __restrict__ val, int* __restrict__ in_list) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < n) in_list[e] = (int)val[e];
}

// Full rows in ELL layout (width ell_w, left-aligned, ~0 padding).
__global__ void k_ell(int nn, int ell_w, const int* __restrict__ frow_ptr, const uint32_t* __restrict__ fblk,
                      const int* __restrict__ fcol, uint32_t* __restrict__ ell_blk, int* __restrict__ ell_col) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * ell_w) return;
    int k = t / ell_w, i = t % ell_w;
    int f = frow_ptr[k] + i;
    bool in = f < frow_ptr[k + 1];
    ell_blk[t] = in ? fblk[f] : 0xffffffffu;
    ell_col[t] = in ? fcol[f] : 0;
}

// Where each upper block is stored in the explicit full rows of the product:
// slot_u[b] = ELL slot of block b in its row, slot_t[b] = ELL slot of its
// transpose in the column's row (-1 for a diagonal block, set by the caller).
__global__ void k_ell_slots(int nn, int ell_w, const uint32_t* __restrict__ ell_blk, int* __restrict__ slot_u,
                            int* __restrict__ slot_t) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nn * ell_w) return;
    const uint32_t bb = ell_blk[t];
    if (bb == 0xffffffffu) return;
    if (bb & 0x80000000u) slot_t[bb & 0x7fffffffu] = t;
    else slot_u[bb] = t;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
size_t knn_box_count(int nn) { return 2 * (size_t)((nn + kKnnRun - 1) / kKnnRun); }

void launch_knn_skin(int ns, const float* pos_aos, int nn, const float4* nodes, const int* caller, float4* boxes,
                     float inv_two_sigma2, int4* idx, float4* w, hipStream_t st) {
    if (ns <= 0 || nn <= 0) return;
    const int nruns = (nn + kKnnRun - 1) / kKnnRun;
    hipLaunchKernelGGL(k_node_boxes, dim3((nruns + 255) / 256), dim3(256), 0, st, nn, nodes, boxes);
    hipLaunchKernelGGL(k_knn_skin, dim3((ns + 255) / 256), dim3(256), 0, st, ns, pos_aos, nn, nodes, caller, boxes,
                       inv_two_sigma2, idx, w);
}

void launch_node_graph(int nn, const float4* nodes, int* nbr, hipStream_t st) {
    hipLaunchKernelGGL(k_node_graph, dim3((nn + kGraphNodesPerBlock - 1) / kGraphNodesPerBlock),
                       dim3(64 * kGraphNodesPerBlock), 0, st, nn, nodes, nbr);
}

void launch_tuple_keys(int ns, int npad, const int4* idx, uint64_t* key, uint32_t* val, hipStream_t st) {
    hipLaunchKernelGGL(k_tuple_keys, dim3((npad + 255) / 256), dim3(256), 0, st, ns, npad, idx, key, val);
}

void launch_permute_surfels(int ns, int seg_len, const uint64_t* key, const uint32_t* val, const float* ipos,
                            const float* inrm, const int4* iidx, const float4* iw, float* px, float* py,
                            float* pz, float* nx, float* ny, float* nz, int4* oidx, float4* ow, int* orig,
                            int* flag, hipStream_t st) {
    hipLaunchKernelGGL(k_permute_surfels, dim3((ns + 255) / 256), dim3(256), 0, st, ns, seg_len, key, val, ipos, inrm,
                       iidx, iw, px, py, pz, nx, ny, nz, oidx, ow, orig, flag);
}

void launch_set_keys(int nsets, const uint64_t* key, const int* run_start, uint64_t* out, hipStream_t st) {
    if (nsets > 0)
        hipLaunchKernelGGL(k_set_keys, dim3((nsets + 255) / 256), dim3(256), 0, st, nsets, key, run_start, out);
}

void launch_seg_pos4(int ns, int nseg, const int* seg_start, const int* seg_nodes, const int4* idx, uint16_t* pos4,
                     int* bad, hipStream_t st) {
    if (ns > 0 && nseg > 0)
        hipLaunchKernelGGL(k_seg_pos4, dim3((ns + 255) / 256), dim3(256), 0, st, ns, nseg, seg_start, seg_nodes, idx,
                           pos4, bad);
}

void launch_run_starts(int ns, const int* flag, const int* pos, int* run_start, hipStream_t st) {
    hipLaunchKernelGGL(k_run_starts, dim3((ns + 255) / 256), dim3(256), 0, st, ns, flag, pos, run_start);
}

void launch_pattern(int nruns, const uint64_t* key, const int* run_start, int nn, const int* nbr,
                    uint32_t* bm, int words, hipStream_t st) {
    if (nruns > 0)
        hipLaunchKernelGGL(k_pattern_runs, dim3((nruns + 255) / 256), dim3(256), 0, st, nruns, key,
                           run_start, bm, words);
    hipLaunchKernelGGL(k_pattern_nodes, dim3((nn + 255) / 256), dim3(256), 0, st, nn, nbr, bm, words);
}

void launch_row_counts(int nn, const uint32_t* bm, int words, int* cnt, hipStream_t st) {
    hipLaunchKernelGGL(k_row_counts, dim3((nn + 255) / 256), dim3(256), 0, st, nn, bm, words, cnt);
}

void launch_row_fill(int nn, const uint32_t* bm, int words, const int* row_ptr, int* col_idx, int* blk_row,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_row_fill, dim3((nn + 255) / 256), dim3(256), 0, st, nn, bm, words, row_ptr,
                       col_idx, blk_row);
}

void launch_transpose_keys(int nb, int npad, const int* blk_row, const int* col_idx, uint64_t* tkey,
                           uint32_t* tval, int* tcount, hipStream_t st) {
    hipLaunchKernelGGL(k_transpose_keys, dim3((nb + 255) / 256), dim3(256), 0, st, nb, blk_row, col_idx,
                       tkey, tval, tcount);
    if (npad > nb)
        hipLaunchKernelGGL(k_pad_keys, dim3((npad - nb + 255) / 256), dim3(256), 0, st, tkey, tval, nb, npad);
}

void launch_full_rows(int nn, int ntr, const int* row_ptr, const int* col_idx, const int* tcount,
                      const int* tstart, const int* frow_ptr, const uint64_t* tkey, const uint32_t* tval,
                      uint32_t* fblk, int* fcol, hipStream_t st) {
    if (ntr > 0)
        hipLaunchKernelGGL(k_full_fill_t, dim3((ntr + 255) / 256), dim3(256), 0, st, ntr, tkey, tval, tstart,
                           frow_ptr, fblk, fcol);
    hipLaunchKernelGGL(k_full_fill_u, dim3((nn + 255) / 256), dim3(256), 0, st, nn, row_ptr, col_idx, tcount,
                       frow_ptr, fblk, fcol);
}

void launch_full_counts(int nn, const int* row_ptr, const int* tcount, int* fcount, hipStream_t st) {
    hipLaunchKernelGGL(k_full_counts, dim3((nn + 255) / 256), dim3(256), 0, st, nn, row_ptr, tcount, fcount);
}

void launch_in_edge_keys(int nn, int npad, const int* nbr, uint64_t* key, uint32_t* val, int* icount, hipStream_t st) {
    hipLaunchKernelGGL(k_in_edge_keys, dim3((npad + 255) / 256), dim3(256), 0, st, nn, npad, nbr, key, val, icount);
}

void launch_ell(int nn, int ell_w, const int* frow_ptr, const uint32_t* fblk, const int* fcol, uint32_t* ell_blk,
                int* ell_col, hipStream_t st) {
    int n = nn * ell_w;
    hipLaunchKernelGGL(k_ell, dim3((n + 255) / 256), dim3(256), 0, st, nn, ell_w, frow_ptr, fblk, fcol, ell_blk,
                       ell_col);
}

void launch_ell_slots(int nn, int ell_w, const uint32_t* ell_blk, int* slot_u, int* slot_t, hipStream_t st) {
    const int n = nn * ell_w;
    hipLaunchKernelGGL(k_ell_slots, dim3((n + 255) / 256), dim3(256), 0, st, nn, ell_w, ell_blk, slot_u, slot_t);
}

void launch_in_edge_store(int n, const uint32_t* val, int* in_list, hipStream_t st) {
    hipLaunchKernelGGL(k_in_edge_store, dim3((n + 255) / 256), dim3(256), 0, st, n, val, in_list);
}

}  // namespace swgn
