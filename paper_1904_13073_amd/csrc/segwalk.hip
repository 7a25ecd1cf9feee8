// The segment layout on the device (Sec. 6.5, Initialization: the per-node-set
// structures the assembly of J^T J walks every iteration).
//
// Surfels sorted by node set are cut into segments: greedy runs of at most M
// consecutive surfels whose node sets together name at most 5 nodes, so that
// a segment's Gram matrix fits one 32x32 MFMA tile; packs are greedy runs of
// whole segments with at most M surfels. A greedy cut is a chain: a segment
// that opens at surfel s always starts with the node set of s's run, so the
// next opening after s is a function next(s) of s alone, with
// s < next(s) <= s + M. next is formed for every surfel at once; the chain
// from surfel 0 is then walked in chunks of C positions, M <= C <= kChainChunk
// (each chunk from each of the M positions a chain can enter it by, in
// parallel; the chunks linked by one thread; the chosen walk of each chunk
// written out).
// Packs are the same chain over segments. Every result is an integer that
// does not depend on the order of any atomic.
#include "swgn_impl.h"
#include "swgn_launch.h"
#include "swgn_setup.h"

namespace swgn {

namespace {

constexpr int kChainChunk = 8192;   // most positions per workgroup of the chain walk (LDS ints)
constexpr int kChainBlock = 256;    // threads per workgroup; >= M

__device__ __forceinline__ void set_nodes(uint64_t k, int (&t)[4]) {
    t[0] = (int)(k >> 48);
    t[1] = (int)((k >> 32) & 0xffff);
    t[2] = (int)((k >> 16) & 0xffff);
    t[3] = (int)(k & 0xffff);
}

// Adds the 4 distinct nodes t to the set cur (cn entries, 5 slots); returns
// the new size, or 6 once it would exceed 5 (cur is then no longer used).
__device__ __forceinline__ int merge_set(int (&cur)[5], int cn, const int (&t)[4]) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        bool have = false;
#pragma unroll
        for (int q = 0; q < 5; ++q) have = have || (q < cn && cur[q] == t[k]);
        if (!have) {
            if (cn == 5) return 6;
#pragma unroll
            for (int q = 0; q < 5; ++q)
                if (q == cn) cur[q] = t[k];
            ++cn;
        }
    }
    return cn;
}

__device__ __forceinline__ int first_pair(int pa) { return 5 * pa - pa * (pa - 1) / 2; }

// next(s): where the segment opening at surfel s ends. run_pos is the
// exclusive scan of the run-start flags (s lies in run run_pos[s + 1] - 1).
// Within s's run only the length cuts; each following run joins while the
// node union stays within 5 nodes and the segment within M surfels, and a run
// that would take it past M surfels cuts it at s + M.
__global__ void k_seg_next(int ns, int nsets, const uint64_t* __restrict__ set_key, const int* __restrict__ set_start,
                           const int* __restrict__ run_pos, int M, int* __restrict__ next) {
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= ns) return;
    const int r = run_pos[s + 1] - 1;
    int nx = ns;
    if (set_start[r + 1] - s > M) {
        nx = s + M;
    } else {
        int t[4];
        set_nodes(set_key[r], t);
        int cur[5] = {t[0], t[1], t[2], t[3], -1};
        int cn = 4;
        for (int r2 = r + 1; r2 < nsets; ++r2) {
            const int a2 = set_start[r2];
            if (a2 - s >= M) { nx = a2; break; }
            set_nodes(set_key[r2], t);
            cn = merge_set(cur, cn, t);
            if (cn > 5) { nx = a2; break; }
            if (set_start[r2 + 1] - s > M) { nx = s + M; break; }
        }
    }
    next[s] = nx;
}

// next over segments for packs: the first segment g2 > g whose end lies more
// than M surfels past the start of g (binary search), else nseg.
__global__ void k_pack_next(int nseg, const int* __restrict__ seg_start, int M, int* __restrict__ next) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nseg) return;
    const int lim = seg_start[g] + M;
    int lo = g + 2, hi = nseg + 1;            // smallest k in [g + 2, nseg] with seg_start[k] > lim, else nseg + 1
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (seg_start[mid] > lim) hi = mid;
        else lo = mid + 1;
    }
    next[g] = lo <= nseg ? lo - 1 : nseg;
}

__device__ __forceinline__ void stage_chunk(const int* __restrict__ next, int lo, int hi, int* nx) {
    for (int i = lo + (int)threadIdx.x; i < hi; i += kChainBlock) nx[i - lo] = next[i];
    __syncthreads();
}

// Per chunk q and entry position lo + t (t < M): where the walk from it leaves
// the chunk and how many positions it visits inside. A successor that does not
// move forward ends the walk and flags the input.
__global__ void __launch_bounds__(kChainBlock) k_chain_chunks(const int* __restrict__ next, int n, int M, int C,
                                                               int* __restrict__ exit_pos, int* __restrict__ hops,
                                                               int* __restrict__ bad) {
    __shared__ int nx[kChainChunk];
    const int q = blockIdx.x, lo = q * C, hi = min(n, lo + C);
    stage_chunk(next, lo, hi, nx);
    const int t = threadIdx.x;
    if (t >= M) return;
    int pos = lo + t, cnt = 0;
    while (pos < hi) {
        const int np = nx[pos - lo];
        if (np <= pos) { atomicOr(bad, 1); break; }
        pos = np;
        ++cnt;
    }
    exit_pos[q * M + t] = pos;
    hops[q * M + t] = cnt;
}

// The chunks linked in order from position 0 (one thread): each chunk's entry
// position and the number of chain positions before it; *count = the chain's
// length. An entry outside the chunk's M entry positions flags the input and
// marks the remaining chunks unused (entry -1).
__global__ void k_chain_link(int nchunks, int n, int M, int C, const int* __restrict__ exit_pos,
                             const int* __restrict__ hops, int* __restrict__ entry, int* __restrict__ base,
                             int* __restrict__ count, int* __restrict__ bad) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    int e = 0, b = 0;
    bool ok = true;
    for (int q = 0; q < nchunks; ++q) {
        const int t = e - q * C;
        ok = ok && t >= 0 && t < M;
        entry[q] = ok ? e : -1;
        base[q] = b;
        if (ok) {
            b += hops[q * M + t];
            e = exit_pos[q * M + t];
        }
    }
    if (!ok || e != n) *bad = 1;
    *count = ok ? b : 0;
}

// The chain's positions inside each chunk, from its entry, at out[base ...].
__global__ void __launch_bounds__(kChainBlock) k_chain_emit(const int* __restrict__ next, int n, int C,
                                                             const int* __restrict__ entry,
                                                             const int* __restrict__ base, int* __restrict__ out) {
    __shared__ int nx[kChainChunk];
    const int q = blockIdx.x, lo = q * C, hi = min(n, lo + C);
    stage_chunk(next, lo, hi, nx);
    if (threadIdx.x != 0 || entry[q] < 0) return;
    int pos = entry[q], j = base[q];
    while (pos < hi && j < n) {
        out[j++] = pos;
        const int np = nx[pos - lo];
        if (np <= pos) break;
        pos = np;
    }
}

// Per segment: its nodes (ascending, -1 padded), the mask of its node pairs
// that share a surfel (bit first(pa) + pb - pa, pa <= pb positions in the
// node list), its Gram output in 4-float units (36 per pair + 32) and its
// pair count; the units' 64-bit total. More than 5 nodes flags the input.
__global__ void __launch_bounds__(256) k_seg_info(int nseg, const int* __restrict__ seg_start,
                                                  const int* __restrict__ run_pos, const uint64_t* __restrict__ set_key,
                                                  int* __restrict__ seg_nodes, uint16_t* __restrict__ mask,
                                                  int* __restrict__ units, int* __restrict__ npairs,
                                                  unsigned long long* __restrict__ total_units, int* __restrict__ bad) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    int u = 0;
    if (g < nseg) {
        const int r0 = run_pos[seg_start[g] + 1] - 1, r1 = run_pos[seg_start[g + 1]] - 1;
        int t[4];
        set_nodes(set_key[r0], t);
        int cur[5] = {t[0], t[1], t[2], t[3], 0x7fffffff};
        int cn = 4;
        for (int r = r0 + 1; r <= r1 && cn <= 5; ++r) {
            set_nodes(set_key[r], t);
            cn = merge_set(cur, cn, t);
        }
        if (cn > 5) {
            atomicOr(bad, 1);
            cn = 4;
            set_nodes(set_key[r0], t);
            cur[0] = t[0]; cur[1] = t[1]; cur[2] = t[2]; cur[3] = t[3]; cur[4] = 0x7fffffff;
        }
        // ascending (an unused slot holds the largest int and sorts last)
        int tmp;
#define SWGN_CS(p, q) if (cur[p] > cur[q]) { tmp = cur[p]; cur[p] = cur[q]; cur[q] = tmp; }
        SWGN_CS(0, 1) SWGN_CS(3, 4) SWGN_CS(2, 4) SWGN_CS(2, 3) SWGN_CS(0, 3)
        SWGN_CS(0, 2) SWGN_CS(1, 4) SWGN_CS(1, 3) SWGN_CS(1, 2)
#undef SWGN_CS
        uint32_t m = 0;
        for (int r = r0; r <= r1; ++r) {
            set_nodes(set_key[r], t);
            int p[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                p[k] = 0;
#pragma unroll
                for (int q = 0; q < 5; ++q) p[k] += cur[q] < t[k] ? 1 : 0;
            }
#pragma unroll
            for (int x = 0; x < 4; ++x)
#pragma unroll
                for (int y = x; y < 4; ++y) m |= 1u << (first_pair(p[x]) + p[y] - p[x]);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) seg_nodes[5 * g + q] = q < cn ? cur[q] : -1;
        mask[g] = (uint16_t)m;
        const int np = __popc(m);
        u = 9 * np + 8;
        units[g] = u;
        npairs[g] = np;
    }
    u = wave_sumi(u);
    if ((threadIdx.x % kWave) == 0 && u != 0) atomicAdd(total_units, (unsigned long long)u);
}

__global__ void k_seg_off(int nseg, const int* __restrict__ off_units, uint32_t* __restrict__ off) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g <= nseg) off[g] = 4u * (uint32_t)off_units[g];
}

// Per segment, one entry per pair of its mask (in mask order): the block of
// the pair (binary search in the node's row of the upper pattern), the float
// offsets of its sub-block and, on the diagonal, of the J^T r piece; keyed
// (block, entry index) for a stable sort by block, and counted per block. A
// pair missing from the pattern flags the input and keys past every block.
__global__ void k_seg_entries(int nseg, int nb, const int* __restrict__ seg_nodes, const uint16_t* __restrict__ mask,
                              const uint32_t* __restrict__ off, const int* __restrict__ ebase,
                              const int* __restrict__ row_ptr, const int* __restrict__ col_idx,
                              uint64_t* __restrict__ ekey, uint32_t* __restrict__ eval, uint32_t* __restrict__ esub,
                              uint32_t* __restrict__ egrad, int* __restrict__ bcount, int* __restrict__ bad) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nseg) return;
    const uint32_t m = mask[g], np = (uint32_t)__popc(m), o = off[g];
    int e = ebase[g];
    uint32_t rank = 0;
    for (int pa = 0; pa < 5; ++pa)
        for (int pb = pa; pb < 5; ++pb) {
            if (!((m >> (first_pair(pa) + pb - pa)) & 1u)) continue;
            const int ra = seg_nodes[5 * g + pa], cb = seg_nodes[5 * g + pb];
            int lo = row_ptr[ra], hi = row_ptr[ra + 1];
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (col_idx[mid] < cb) lo = mid + 1;
                else hi = mid;
            }
            int blk = lo;
            if (lo >= row_ptr[ra + 1] || col_idx[lo] != cb) {
                atomicOr(bad, 1);
                blk = nb;
            } else {
                atomicAdd(&bcount[blk], 1);
            }
            ekey[e] = ((uint64_t)(uint32_t)blk << 32) | (uint32_t)e;
            eval[e] = (uint32_t)e;
            esub[e] = o + 36u * rank;
            egrad[e] = pa == pb ? o + 36u * np + 6u * (uint32_t)pa : 0xffffffffu;
            ++e;
            ++rank;
        }
}

__global__ void k_key_tail(uint64_t* __restrict__ key, uint32_t* __restrict__ val, int from, int to) {
    const int i = from + blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= to) return;
    key[i] = ~0ull;
    val[i] = 0xffffffffu;
}

__global__ void k_ent_gather(int ne, const uint32_t* __restrict__ order, const uint32_t* __restrict__ esub,
                             const uint32_t* __restrict__ egrad, uint32_t* __restrict__ ent_sub,
                             uint32_t* __restrict__ ent_grad) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const uint32_t v = order[i];
    ent_sub[i] = esub[v];
    ent_grad[i] = egrad[v];
}

// pack_start[i] = seg_start[pack_seg[i]]; the closing entries ns and nseg.
__global__ void k_pack_arrays(int npack, int nseg, int ns, const int* __restrict__ seg_start, int* __restrict__ pack_seg,
                              int* __restrict__ pack_start) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npack) pack_start[i] = seg_start[pack_seg[i]];
    if (i == npack) {
        pack_seg[npack] = nseg;
        pack_start[npack] = ns;
    }
}

inline int grid_of(int64_t n, int block) { return (int)((n + block - 1) / block); }

}  // namespace

// Chunk size: a walk inside a chunk costs a dependent LDS read per step and
// the link a dependent global read per chunk, so C ~ sqrt(32 n) (a power of
// two in [256, kChainChunk]; at least M, so that a chain enters every chunk).
int chain_chunk(int n, int M) {
    int c = 256;
    while (c < kChainChunk && (int64_t)c * c < 32 * (int64_t)n) c <<= 1;
    return c < M ? kChainChunk : c;
}

size_t chain_work_ints(int n, int M) {
    const int64_t nchunks = (n + 255) / 256;
    return (size_t)(nchunks * (2 * (int64_t)M + 2) + 1);
}

void chain_from_zero(const int* next, int n, int M, int* out, int* count, int* work, int* bad, hipStream_t st) {
    const int C = chain_chunk(n, M);
    const int nchunks = (n + C - 1) / C;
    int* exit_pos = work;
    int* hops = exit_pos + (size_t)nchunks * M;
    int* entry = hops + (size_t)nchunks * M;
    int* base = entry + nchunks;
    hipLaunchKernelGGL(k_chain_chunks, dim3(nchunks), dim3(kChainBlock), 0, st, next, n, M, C, exit_pos, hops, bad);
    hipLaunchKernelGGL(k_chain_link, dim3(1), dim3(kWave), 0, st, nchunks, n, M, C, exit_pos, hops, entry, base,
                       count, bad);
    hipLaunchKernelGGL(k_chain_emit, dim3(nchunks), dim3(kChainBlock), 0, st, next, n, C, entry, base, out);
}

int chain_max_hop() { return kChainBlock; }

void launch_seg_next(int ns, int nsets, const uint64_t* set_key, const int* set_start, const int* run_pos, int M,
                     int* next, hipStream_t st) {
    hipLaunchKernelGGL(k_seg_next, dim3(grid_of(ns, 256)), dim3(256), 0, st, ns, nsets, set_key, set_start, run_pos, M,
                       next);
}

void launch_pack_next(int nseg, const int* seg_start, int M, int* next, hipStream_t st) {
    hipLaunchKernelGGL(k_pack_next, dim3(grid_of(nseg, 256)), dim3(256), 0, st, nseg, seg_start, M, next);
}

void launch_seg_info(int nseg, const int* seg_start, const int* run_pos, const uint64_t* set_key, int* seg_nodes,
                     uint16_t* mask, int* units, int* npairs, unsigned long long* total_units, int* bad,
                     hipStream_t st) {
    hipLaunchKernelGGL(k_seg_info, dim3(grid_of(nseg, 256)), dim3(256), 0, st, nseg, seg_start, run_pos, set_key,
                       seg_nodes, mask, units, npairs, total_units, bad);
}

void launch_seg_off(int nseg, const int* off_units, uint32_t* off, hipStream_t st) {
    hipLaunchKernelGGL(k_seg_off, dim3(grid_of(nseg + 1, 256)), dim3(256), 0, st, nseg, off_units, off);
}

void launch_seg_entries(int nseg, int nb, int npad, const int* seg_nodes, const uint16_t* mask, const uint32_t* off,
                        const int* ebase, int ne, const int* row_ptr, const int* col_idx, uint64_t* ekey,
                        uint32_t* eval, uint32_t* esub, uint32_t* egrad, int* bcount, int* bad, hipStream_t st) {
    hipLaunchKernelGGL(k_seg_entries, dim3(grid_of(nseg, 256)), dim3(256), 0, st, nseg, nb, seg_nodes, mask, off,
                       ebase, row_ptr, col_idx, ekey, eval, esub, egrad, bcount, bad);
    if (npad > ne)
        hipLaunchKernelGGL(k_key_tail, dim3(grid_of(npad - ne, 256)), dim3(256), 0, st, ekey, eval, ne, npad);
}

void launch_ent_gather(int ne, const uint32_t* order, const uint32_t* esub, const uint32_t* egrad, uint32_t* ent_sub,
                       uint32_t* ent_grad, hipStream_t st) {
    if (ne > 0)
        hipLaunchKernelGGL(k_ent_gather, dim3(grid_of(ne, 256)), dim3(256), 0, st, ne, order, esub, egrad, ent_sub,
                           ent_grad);
}

void launch_pack_arrays(int npack, int nseg, int ns, const int* seg_start, int* pack_seg, int* pack_start,
                        hipStream_t st) {
    hipLaunchKernelGGL(k_pack_arrays, dim3(grid_of(npack + 1, 256)), dim3(256), 0, st, npack, nseg, ns, seg_start,
                       pack_seg, pack_start);
}

}  // namespace swgn
