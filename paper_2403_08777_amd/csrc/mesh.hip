// Mesh preprocessing: validation, Hilbert element order, first-touch node
// renumbering, element patches; plus the user <-> mesh order helpers.
//
// The paper's kernels gather nodal values and scatter RHS entries through the
// connectivity, and after removing intermediates those indirect accesses are
// what remains (Sec. V-C); their reuse happens in the shared cache.  On a
// chip with eight L2 caches (one per XCD) that reuse depends on the order of
// elements and on node numbering, so the mesh is reordered here once:
//   1. elements sorted along a Hilbert curve of their centroids;
//   2. nodes renumbered in order of first use by that element sequence, so the
//      nodes of consecutive elements have nearby ids (coalesced gathers);
//   3. the sequence cut into patches of E consecutive elements; for each patch
//      the ascending list of its distinct nodes and one-byte local ids per
//      element, so a workgroup can stage the patch's nodes through LDS.
#include <algorithm>
#include <cfloat>
#include <climits>
#include <new>
#include <vector>

#include "internal.hpp"

namespace nsasm {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kBadRange = 1u, kBadRepeat = 2u, kBadDet = 4u;
constexpr int kBboxBlocks = 512;
constexpr double kDetRelTol = 64.0 * DBL_EPSILON;

struct CreateFlags {
    uint32_t bits;
    int32_t first_bad;
};

__global__ __launch_bounds__(kThreads) void k_validate_ids(const int32_t *conn, int64_t ne, int64_t nn,
                                                            CreateFlags *flags) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= ne) return;
    const int4 c = reinterpret_cast<const int4 *>(conn)[e];
    uint32_t bad = 0;
    const int ids[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int a = 0; a < 4; ++a)
        if (ids[a] < 0 || ids[a] >= nn) bad |= kBadRange;
    if (c.x == c.y || c.x == c.z || c.x == c.w || c.y == c.z || c.y == c.w || c.z == c.w) bad |= kBadRepeat;
    if (bad) {
        atomicOr(&flags->bits, bad);
        atomicMin(&flags->first_bad, static_cast<int32_t>(e));
    }
}

__global__ __launch_bounds__(kThreads) void k_bbox_partial(const double *x, int64_t nn, double *part) {
    __shared__ double red[6][kThreads];
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; k < nn;
         k += static_cast<int64_t>(gridDim.x) * kThreads) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const double v = x[3 * k + i];
            lo[i] = fmin(lo[i], v);
            hi[i] = fmax(hi[i], v);
        }
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        red[i][threadIdx.x] = lo[i];
        red[3 + i][threadIdx.x] = hi[i];
    }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                red[i][threadIdx.x] = fmin(red[i][threadIdx.x], red[i][threadIdx.x + s]);
                red[3 + i][threadIdx.x] = fmax(red[3 + i][threadIdx.x], red[3 + i][threadIdx.x + s]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[threadIdx.x * gridDim.x + blockIdx.x] = red[threadIdx.x][0];
}

__global__ __launch_bounds__(kThreads) void k_bbox_final(const double *part, int nparts, double *box) {
    __shared__ double red[6][kThreads];
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double v = (i < 3) ? INFINITY : -INFINITY;
        for (int k = threadIdx.x; k < nparts; k += kThreads) {
            const double w = part[i * nparts + k];
            v = (i < 3) ? fmin(v, w) : fmax(v, w);
        }
        red[i][threadIdx.x] = v;
    }
    __syncthreads();
    for (int s = kThreads / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
#pragma unroll
            for (int i = 0; i < 6; ++i)
                red[i][threadIdx.x] = (i < 3) ? fmin(red[i][threadIdx.x], red[i][threadIdx.x + s])
                                              : fmax(red[i][threadIdx.x], red[i][threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) box[threadIdx.x] = red[threadIdx.x][0];
}

// Spread the low 21 bits of v to every third bit (the 3-D bit interleave).
__device__ inline uint64_t spread_bits3(uint64_t v) {
    v &= 0x1fffffull;
    v = (v | (v << 32)) & 0x1f00000000ffffull;
    v = (v | (v << 16)) & 0x1f0000ff0000ffull;
    v = (v | (v << 8)) & 0x100f00f00f00f00full;
    v = (v | (v << 4)) & 0x10c30c30c30c30c3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
}

// Index of cell (q0, q1, q2), 0 <= q < 2^21, along the 3-D Hilbert curve of
// 2^21 cells per axis (63 bits), by Skilling's method (J. Skilling,
// "Programming the Hilbert curve", AIP Conf. Proc. 707, 2004): the axes are
// turned into the curve's transposed index level by level from the top
// (reflect the lower bits of axis 0 where a coordinate's bit is set, else
// exchange them between axis 0 and that axis), Gray-decoded, and the bits of
// the three transposed words are interleaved, most significant level first,
// axis 0 highest.  Consecutive indices are face-adjacent cells, so a run of
// consecutive elements stays compact where a Morton curve would jump.
__device__ inline uint64_t hilbert_key3(uint32_t q0, uint32_t q1, uint32_t q2) {
    uint32_t X[3] = {q0, q1, q2};
    constexpr uint32_t kTop = 1u << 20;
    for (uint32_t Q = kTop; Q > 1; Q >>= 1) {
        const uint32_t P = Q - 1;
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (X[i] & Q) {
                X[0] ^= P;
            } else {
                const uint32_t t = (X[0] ^ X[i]) & P;
                X[0] ^= t;
                X[i] ^= t;
            }
        }
    }
    X[1] ^= X[0];
    X[2] ^= X[1];
    uint32_t t = 0;
    for (uint32_t Q = kTop; Q > 1; Q >>= 1)
        if (X[2] & Q) t ^= Q - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) X[i] ^= t;
    return (spread_bits3(X[0]) << 2) | (spread_bits3(X[1]) << 1) | spread_bits3(X[2]);
}

// Hilbert key of each element's centroid (63 bits) and the degenerate-element check.
__global__ __launch_bounds__(kThreads) void k_element_keys(const double *x, const int32_t *conn,
                                                            int64_t ne, const double *box,
                                                            uint64_t *keys, int32_t *vals,
                                                            CreateFlags *flags) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (e >= ne) return;
    const int4 c = reinterpret_cast<const int4 *>(conn)[e];
    const int ids[4] = {c.x, c.y, c.z, c.w};
    double xe[4][3];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int i = 0; i < 3; ++i) xe[a][i] = x[3 * static_cast<int64_t>(ids[a]) + i];
    // The determinant the assembly kernels invert, rejected when it is not a
    // normal number or is within rounding of zero: below 64 eps |d_1||d_2||d_3|
    // (Hadamard's bound is |d_1||d_2||d_3|) the kernels' sign and value of
    // det J would be rounding noise, and 1/det could overflow.
    double c1[3], c2[3], c3[3], d1[3];
    const double det = tet_adjugate(xe, c1, c2, c3, d1);
    double len2[3] = {0.0, 0.0, 0.0};  // squared edge lengths |d_k|^2
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) len2[k] += (xe[k + 1][i] - xe[0][i]) * (xe[k + 1][i] - xe[0][i]);
    const double bound = kDetRelTol * sqrt(len2[0]) * sqrt(len2[1]) * sqrt(len2[2]);
    if (!isfinite(det) || !(fabs(det) >= DBL_MIN) || !(fabs(det) > bound)) {
        atomicOr(&flags->bits, kBadDet);
        atomicMin(&flags->first_bad, static_cast<int32_t>(e));
    }
    const double ext = fmax(fmax(box[3] - box[0], box[4] - box[1]), box[5] - box[2]);
    const double scale = (ext > 0.0) ? 2097151.0 / ext : 0.0;
    uint32_t cell[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const double cen = 0.25 * (xe[0][i] + xe[1][i] + xe[2][i] + xe[3][i]);
        double q = (cen - box[i]) * scale;
        q = fmin(fmax(q, 0.0), 2097151.0);
        cell[i] = static_cast<uint32_t>(q);
    }
    keys[e] = hilbert_key3(cell[0], cell[1], cell[2]);
    vals[e] = static_cast<int32_t>(e);
}

__global__ __launch_bounds__(kThreads) void k_iota(int32_t *v, int64_t n) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (k < n) v[k] = static_cast<int32_t>(k);
}

// first[n] = smallest (4 * position + local vertex) at which node n is used.
__global__ __launch_bounds__(kThreads) void k_first_touch(const int32_t *conn, const int32_t *order,
                                                           int64_t ne, uint32_t *first) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (s >= ne) return;
    const int4 c = reinterpret_cast<const int4 *>(conn)[order[s]];
    const uint32_t k = static_cast<uint32_t>(4 * s);
    atomicMin(&first[c.x], k);
    atomicMin(&first[c.y], k + 1);
    atomicMin(&first[c.z], k + 2);
    atomicMin(&first[c.w], k + 3);
}

__global__ __launch_bounds__(kThreads) void k_invert(const int32_t *iperm, int64_t n, int32_t *perm) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (k < n) perm[iperm[k]] = static_cast<int32_t>(k);
}

__global__ __launch_bounds__(kThreads) void k_remap_conn(const int32_t *conn, const int32_t *order,
                                                          const int32_t *perm, int64_t ne, int4 *out) {
    const int64_t s = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (s >= ne) return;
    const int4 c = reinterpret_cast<const int4 *>(conn)[order[s]];
    out[s] = make_int4(perm[c.x], perm[c.y], perm[c.z], perm[c.w]);
}

// dst[k] = src[map[k]] for rows of ncomp elements.
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather_rows(const T *src, const int32_t *map, int64_t n,
                                                           int ncomp, T *dst) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (k >= n * ncomp) return;
    const int64_t row = k / ncomp;
    const int c = static_cast<int>(k - row * ncomp);
    dst[k] = src[static_cast<int64_t>(map[row]) * ncomp + c];
}

// Bitonic sort of kN keys in LDS (kN a power of two), 256 threads.
template <typename K, int kN>
__device__ void lds_bitonic_sort(K *keys) {
    for (int len = 2; len <= kN; len <<= 1) {
        for (int j = len >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < kN; i += kThreads) {
                const int partner = i ^ j;
                if (partner > i) {
                    const bool ascending = (i & len) == 0;
                    const K a = keys[i], b = keys[partner];
                    if ((a > b) == ascending) {
                        keys[i] = b;
                        keys[partner] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

constexpr int kPatchSlots = 4 * kMaxPatchElems;   // 1024 (element, vertex) pairs
constexpr uint64_t kNoKey = ~0ull;

// Keys (node id << 10 | slot) of one patch, slot = 4 * local element + vertex;
// padded with kNoKey.  Sorted, they list each node's slots contiguously, in
// slot order.
__device__ void patch_sorted_pairs(const int4 *conn, int64_t ne, int64_t first_elem, int elems,
                                   uint64_t *keys /*LDS, kPatchSlots*/) {
    const int32_t *flat = reinterpret_cast<const int32_t *>(conn);
    const int nslots = 4 * static_cast<int>(min<int64_t>(elems, ne - first_elem));
    for (int k = threadIdx.x; k < kPatchSlots; k += kThreads)
        keys[k] = (k < nslots) ? ((static_cast<uint64_t>(flat[4 * first_elem + k]) << 10) | static_cast<uint64_t>(k))
                               : kNoKey;
    __syncthreads();
    lds_bitonic_sort<uint64_t, kPatchSlots>(keys);
}

__device__ inline bool run_head(const uint64_t *keys, int k) {
    return keys[k] != kNoKey && (k == 0 || (keys[k] >> 10) != (keys[k - 1] >> 10));
}

// Pass 1: number of distinct nodes per patch.
__global__ __launch_bounds__(kThreads) void k_patch_count(const int4 *conn, int64_t ne, int elems,
                                                           uint32_t *count) {
    __shared__ uint64_t keys[kPatchSlots];
    __shared__ uint32_t lds4[4];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * elems;
    patch_sorted_pairs(conn, ne, first, elems, keys);
    uint32_t heads = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) heads += run_head(keys, 4 * threadIdx.x + r) ? 1u : 0u;
    uint32_t total;
    (void)block_exclusive_scan_256(heads, lds4, &total);
    if (threadIdx.x == 0) count[blockIdx.x] = total;
}

// Pass 2: for each patch write its distinct nodes (ascending), where each
// node's run of slots lies, and for every element the positions of its four
// (element, vertex) slots.  An assembly workgroup stores element
// contributions at those positions and then sums each node's run (one thread
// per node, records ordered by decreasing run length): a deterministic
// in-LDS reduction without atomics.  Where runs and positions lie is free;
// both are chosen to spread the LDS banks (a double's bank pair is its slot
// modulo 32, and the LDS serves the 32 lanes of a half-wave together):
//  - runs are placed one after another, each time taking, among the runs not
//    yet placed and in record order, the first whose half-wave of summing
//    threads has no run starting at the current position modulo 32 yet, so
//    that the run reads of a half-wave start in different banks;
//  - each (element, vertex) pair takes the free position of its node's run
//    whose bank the store instruction of its half-wave and vertex has used
//    least (the lowest such position on ties), half-wave by half-wave and
//    vertex by vertex.
// node_start receives each run as first | length << 11.  Patches with more
// than kMaxPatchNodes nodes are rejected (from pass 1) on the host before
// this runs.
__global__ __launch_bounds__(kThreads) void k_patch_fill(const int4 *conn, int64_t ne, int elems,
                                                          const uint32_t *offset, int32_t *nodes,
                                                          int32_t *node_start, ushort4 *elem_pos) {
    __shared__ uint64_t keys[kPatchSlots];
    __shared__ uint16_t pos_of_slot[kPatchSlots];
    __shared__ uint16_t run_of_slot[kPatchSlots];  // by element slot: its node's index in the patch
    __shared__ uint16_t run_sorted[kMaxPatchNodes];  // per node: its first position in sorted order
    __shared__ uint16_t run_len[kMaxPatchNodes];
    __shared__ uint16_t run_place[kMaxPatchNodes];   // per node: first slot of its run
    __shared__ uint8_t node_of_rank[kMaxPatchNodes]; // record order: longer runs first, then node order
    __shared__ uint32_t used[kPatchSlots / 32];      // slots already taken
    __shared__ uint32_t bank_use[32];                // stores per bank in the current instruction
    __shared__ uint32_t left[kMaxPatchNodes / 32];   // record ranks not yet placed
    __shared__ uint32_t half_used[kMaxPatchNodes / 32];  // per half-wave of records: starts taken modulo 32
    __shared__ uint32_t lds4[4];
    const int64_t first = static_cast<int64_t>(blockIdx.x) * elems;
    const int nel = static_cast<int>(min<int64_t>(elems, ne - first));
    const int t = threadIdx.x;
    patch_sorted_pairs(conn, ne, first, elems, keys);
    bool head[4];
    uint32_t heads = 0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        head[r] = run_head(keys, 4 * t + r);
        heads += head[r] ? 1u : 0u;
    }
    uint32_t nruns;
    uint32_t u = block_exclusive_scan_256(heads, lds4, &nruns);
    if (t < kPatchSlots / 32) used[t] = 0u;
    if (t < 32) bank_use[t] = 0u;
    if (t < kMaxPatchNodes / 32) {
        const int n = static_cast<int>(nruns) - 32 * t;
        left[t] = n >= 32 ? ~0u : (n > 0 ? (1u << n) - 1u : 0u);
        half_used[t] = 0u;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int k = 4 * t + r;
        if (head[r]) {
            int e = k + 1;
            while (e < kPatchSlots && keys[e] != kNoKey && !run_head(keys, e)) ++e;
            nodes[offset[blockIdx.x] + u] = static_cast<int32_t>(keys[k] >> 10);
            run_sorted[u] = static_cast<uint16_t>(k);
            run_len[u] = static_cast<uint16_t>(e - k);
            ++u;
        }
    }
    __syncthreads();
    if (static_cast<uint32_t>(t) < nruns) {
        const int mine = run_len[t];
        int rank = 0;
        for (int v = 0; v < static_cast<int>(nruns); ++v) {
            const int lv = run_len[v];
            rank += (lv > mine || (lv == mine && v < t)) ? 1 : 0;
        }
        node_of_rank[rank] = static_cast<uint8_t>(t);
        for (int k = run_sorted[t]; k < run_sorted[t] + mine; ++k) run_of_slot[keys[k] & 1023u] = static_cast<uint16_t>(t);
    }
    __syncthreads();
    // run placement and position choice by the first wave (only it runs
    // these loops; the fences make lane 0's LDS writes visible to the wave)
    if (t < 64) {
        const int lane = t;
        int cursor = 0;
        for (uint32_t step = 0; step < nruns; ++step) {
            const int res = cursor & 31;
            int pick = -1, fallback = -1;
#pragma unroll
            for (int w = 0; w < kMaxPatchNodes / 64; ++w) {
                const int rank = 64 * w + lane;
                const bool here = ((left[rank >> 5] >> (rank & 31)) & 1u) != 0u;
                const bool fits = here && !((half_used[rank >> 5] >> res) & 1u);
                const uint64_t fb = __ballot(fits), lb = __ballot(here);
                if (pick < 0 && fb) pick = 64 * w + __ffsll(static_cast<long long>(fb)) - 1;
                if (fallback < 0 && lb) fallback = 64 * w + __ffsll(static_cast<long long>(lb)) - 1;
            }
            if (pick < 0) pick = fallback;
            const int v = node_of_rank[pick];
            if (lane == 0) {
                left[pick >> 5] &= ~(1u << (pick & 31));
                half_used[pick >> 5] |= 1u << res;
                run_place[v] = static_cast<uint16_t>(cursor);
            }
            cursor += run_len[v];
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
        for (int h = 0; 32 * h < nel; ++h) {
            const int hn = min(32, nel - 32 * h);
            for (int a = 0; a < 4; ++a) {
                for (int i = 0; i < hn; ++i) {
                    const int slot = 4 * (32 * h + i) + a;
                    const int v = run_of_slot[slot];
                    const int rf = run_place[v], rl = run_len[v];
                    uint32_t best = 0xffffffffu;
                    for (int k = lane; k < rl; k += 64) {
                        const int q = rf + k;
                        if (!((used[q >> 5] >> (q & 31)) & 1u)) best = min(best, (bank_use[q & 31] << 16) | k);
                    }
                    for (int o = 32; o > 0; o >>= 1)
                        best = min(best, static_cast<uint32_t>(__shfl_xor(static_cast<int>(best), o, 64)));
                    if (lane == 0) {
                        const int q = rf + static_cast<int>(best & 0xffffu);
                        used[q >> 5] |= 1u << (q & 31);
                        bank_use[q & 31] += 1u;
                        pos_of_slot[slot] = static_cast<uint16_t>(q);
                    }
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                }
                if (lane < 32) bank_use[lane] = 0u;
                __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __syncthreads();
    if (static_cast<uint32_t>(t) < nruns)
        node_start[offset[blockIdx.x] + t] = static_cast<int32_t>(run_place[t]) | (static_cast<int32_t>(run_len[t]) << 11);
    const int64_t s = first + t;
    if (t < elems && s < ne) {
        const int b = 4 * t;
        elem_pos[s] = make_ushort4(pos_of_slot[b], pos_of_slot[b + 1], pos_of_slot[b + 2], pos_of_slot[b + 3]);
    }
}

// LDS placement of each patch node, chosen so that the element gathers of
// the assembly kernels are free of LDS bank conflicts where possible.  An
// assembly workgroup reads vertex a of its elements, lane = element, in one
// instruction per field; the hardware serves lanes in groups, and two lanes
// of a group that read different nodes whose LDS words fall in the same bank
// wait for each other.  Node data sits in arrays indexed by the position, so
// the bank of a node is its position modulo the bank count (in 4-byte words
// for float fields, 8-byte pairs for double).  Nodes read together by a group
// of 16, 32 or 64 consecutive elements (for one vertex slot) get positions
// distinct modulo 16, 32 or 64, by greedy colouring in node order: class
// c in [0, 64) with at most 4 nodes, position c + 64 * (rank in class).  When
// no class satisfies every level the coarser levels are dropped in turn.
// Any placement is correct; this one only saves LDS cycles.
constexpr int kColorLevels = 3;           // groups of 64, 32, 16 lanes
constexpr int kAdjWords = kMaxPatchNodes * kMaxPatchNodes / 32;

__global__ __launch_bounds__(kThreads) void k_patch_color(const uint32_t *off, const int32_t *start,
                                                           const ushort4 *elem_pos, int64_t ne, int elems,
                                                           uint8_t *position, uchar4 *elem_loc) {
    __shared__ uint32_t adj[kColorLevels][kAdjWords];  // 24 KB: adjacency bit matrices
    __shared__ uint8_t node_of_slot[kPatchSlots];
    __shared__ uint8_t la[4][kMaxPatchElems];
    __shared__ uint8_t cls[kMaxPatchNodes];
    __shared__ uint8_t posn[kMaxPatchNodes];
    __shared__ uint32_t used[64];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t beg = off[p], cnt = off[p + 1] - beg;
    const int64_t first = p * static_cast<int64_t>(elems);
    const int nel = static_cast<int>(min<int64_t>(elems, ne - first));
    for (int k = t; k < kColorLevels * kAdjWords; k += kThreads) (&adj[0][0])[k] = 0u;
    if (t < 64) used[t] = 0u;
    if (static_cast<uint32_t>(t) < cnt) {
        const int sb = start[beg + t] & 0x7ff;
        const int se = sb + (start[beg + t] >> 11);
        for (int k = sb; k < se; ++k) node_of_slot[k] = static_cast<uint8_t>(t);
    }
    __syncthreads();
    if (t < nel) {
        const ushort4 ps = elem_pos[first + t];
        la[0][t] = node_of_slot[ps.x];
        la[1][t] = node_of_slot[ps.y];
        la[2][t] = node_of_slot[ps.z];
        la[3][t] = node_of_slot[ps.w];
    }
    __syncthreads();
    if (t < nel) {
#pragma unroll
        for (int lvl = 0; lvl < kColorLevels; ++lvl) {
            const int lanes = 64 >> lvl;
            const int g0 = t & ~(lanes - 1);
            const int g1 = min(g0 + lanes, nel);
            for (int a = 0; a < 4; ++a) {
                const int x = la[a][t];
                for (int e = g0; e < g1; ++e) {
                    const int y = la[a][e];
                    if (y != x) atomicOr(&adj[lvl][(x * kMaxPatchNodes + y) >> 5], 1u << (y & 31));
                }
            }
        }
    }
    __syncthreads();
    // greedy colouring by the first wave, nodes in ascending order
    if (t < 64) {
        for (uint32_t x = 0; x < cnt; ++x) {
            uint64_t m64 = 0;
            uint32_t m32 = 0, m16 = 0;
            for (int y = t; y < static_cast<int>(x); y += 64) {
                const int c = cls[y];
                const int w = (static_cast<int>(x) * kMaxPatchNodes + y) >> 5, b = y & 31;
                if ((adj[0][w] >> b) & 1u) m64 |= uint64_t(1) << c;
                if ((adj[1][w] >> b) & 1u) m32 |= 1u << (c & 31);
                if ((adj[2][w] >> b) & 1u) m16 |= 1u << (c & 15);
            }
            for (int o = 32; o > 0; o >>= 1) {
                m64 |= static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(m64), o, 64));
                m32 |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(m32), o, 64));
                m16 |= static_cast<uint32_t>(__shfl_xor(static_cast<int>(m16), o, 64));
            }
            const int c = t;  // this lane's candidate class
            const bool room = used[c] < 4u;
            const bool f16 = (m16 >> (c & 15)) & 1u, f32 = (m32 >> (c & 31)) & 1u, f64 = (m64 >> c) & 1u;
            uint64_t ok = __ballot(room && !f64 && !f32 && !f16);
            if (!ok) ok = __ballot(room && !f32 && !f16);
            if (!ok) ok = __ballot(room && !f32);
            if (!ok) ok = __ballot(room);
            const int choice = __ffsll(static_cast<long long>(ok)) - 1;
            if (t == 0) {
                const uint8_t pos = static_cast<uint8_t>(choice + 64 * used[choice]);
                cls[x] = static_cast<uint8_t>(choice);
                posn[x] = pos;
                position[beg + x] = pos;
                used[choice] += 1u;
            }
            // only the first wave runs this loop: make lane 0's LDS writes
            // visible to the wave before the next node
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
            __builtin_amdgcn_wave_barrier();
        }
    }
    __syncthreads();
    if (t < nel)
        elem_loc[first + t] = make_uchar4(posn[la[0][t]], posn[la[1][t]], posn[la[2][t]], posn[la[3][t]]);
}

// Fixed-stride patch records: entry t of patch p at p * stride + t, so an
// assembly workgroup finds its nodes without first reading the patch offset.
// rec.y packs the node's slot run [first, end) and its LDS position:
// first | end << 11 | position << 22.  Records are ordered by decreasing run
// length (ties by node): the assembly thread of record t sums that run, and a
// wave loops as long as its longest run, so similar lengths share a wave.
__global__ __launch_bounds__(kThreads) void k_patch_pad(const uint32_t *off, const int32_t *nodes,
                                                         const int32_t *start, const uint8_t *position,
                                                         const int32_t *ref_slot, int64_t ne, int elems,
                                                         int stride, int2 *rec, int32_t *ref) {
    __shared__ int len[kMaxPatchNodes];
    const int64_t p = blockIdx.x;
    const int t = threadIdx.x;
    const uint32_t beg = off[p], cnt = off[p + 1] - beg;
    const bool real = static_cast<uint32_t>(t) < cnt;
    int sb = 0, se = 0;
    if (real) {
        sb = start[beg + t] & 0x7ff;
        se = sb + (start[beg + t] >> 11);
        len[t] = se - sb;
    }
    __syncthreads();
    if (real) {
        const int mine = se - sb;
        int slot = 0;  // this record's place: longer runs first, then node order
        for (int u = 0; u < static_cast<int>(cnt); ++u) {
            const int lu = len[u];
            slot += (lu > mine || (lu == mine && u < t)) ? 1 : 0;
        }
        rec[p * stride + slot] =
            make_int2(nodes[beg + t], sb | (se << 11) | (static_cast<int>(position[beg + t]) << 22));
        if (ref) ref[p * stride + slot] = ref_slot ? ref_slot[beg + t] : 0;
    } else if (t < stride) {
        rec[p * stride + t] = make_int2(-1, 0);
        if (ref) ref[p * stride + t] = 0;
    }
}

// Number of patch references of every node (patch_nodes entries equal to it).
__global__ __launch_bounds__(kThreads) void k_count_refs(const int32_t *nodes, int64_t refs, uint32_t *count) {
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (r < refs) atomicAdd(&count[nodes[r]], 1u);
}

inline unsigned blocks_for(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

nsasm_status check_launch(const char *what) {
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? NSASM_OK : hip_fail(err, what);
}

void free_mesh(nsasm_mesh *m) {
    if (!m) return;
    device_free(m->perm);
    device_free(m->iperm);
    device_free(m->user_elem);
    device_free(m->conn);
    device_free(m->x);
    device_free(m->patch_off);
    device_free(m->patch_nodes);
    device_free(m->patch_node_start);
    device_free(m->elem_pos);
    device_free(m->elem_loc);
    device_free(m->node_ref_off);
    device_free(m->ref_slot);
    device_free(m->patch_rec);
    device_free(m->patch_ref);
    device_free(m->partial);
    device_free(m->lumped);
    delete m;
}

// Free the compact patch lists once the padded records exist.
void free_compact_patches(nsasm_mesh *m) {
    device_free(m->patch_off);
    device_free(m->patch_nodes);
    device_free(m->patch_node_start);
    device_free(m->ref_slot);
    m->patch_off = m->patch_nodes = m->patch_node_start = m->ref_slot = nullptr;
}

nsasm_status read_flags(const CreateFlags *d_flags, hipStream_t stream, CreateFlags *h) {
    NSASM_HIP(hipMemcpyAsync(h, d_flags, sizeof(CreateFlags), hipMemcpyDeviceToHost, stream));
    NSASM_HIP(hipStreamSynchronize(stream));
    return NSASM_OK;
}

// Build patches of `elems` consecutive mesh-order elements.  Returns
// UNSUPPORTED (leaving m without patches) when a patch has too many distinct
// nodes.
nsasm_status build_patches(nsasm_mesh *m, int elems, hipStream_t stream) {
    const int64_t np = (m->n_elems + elems - 1) / elems;
    if (np >= INT_MAX) return fail(NSASM_ERR_UNSUPPORTED, "too many patches");
    uint32_t *count = nullptr;
    NSASM_TRY(device_alloc(&count, static_cast<size_t>(np + 1), "patch counts"));
    k_patch_count<<<static_cast<unsigned>(np), kThreads, 0, stream>>>(m->conn, m->n_elems, elems, count);
    nsasm_status st = check_launch("k_patch_count");
    std::vector<uint32_t> host(static_cast<size_t>(np));
    if (st == NSASM_OK) {
        hipError_t err = hipMemcpyAsync(host.data(), count, sizeof(uint32_t) * np, hipMemcpyDeviceToHost, stream);
        if (err == hipSuccess) err = hipStreamSynchronize(stream);
        if (err != hipSuccess) st = hip_fail(err, "patch counts");
    }
    uint32_t max_nodes = 0;
    if (st == NSASM_OK) max_nodes = *std::max_element(host.begin(), host.end());
    if (st == NSASM_OK && max_nodes > static_cast<uint32_t>(kMaxPatchNodes))
        st = fail(NSASM_ERR_UNSUPPORTED,
                  "a patch of %d elements touches %u distinct nodes (limit %d); use a smaller "
                  "patch, renumbering, or atomic scatter",
                  elems, max_nodes, kMaxPatchNodes);
    uint32_t total = 0;
    if (st == NSASM_OK) st = exclusive_scan_u32(count, count, np, &total, stream);
    if (st == NSASM_OK) {
        hipError_t err = hipMemcpyAsync(count + np, &total, sizeof(uint32_t), hipMemcpyHostToDevice, stream);
        if (err != hipSuccess) st = hip_fail(err, "patch offsets");
    }
    if (st == NSASM_OK) st = device_alloc(&m->patch_nodes, total, "patch nodes");
    // one padding entry so that reading the successor of the last reference stays in bounds
    if (st == NSASM_OK) st = device_alloc(&m->patch_node_start, static_cast<size_t>(total) + 1, "patch slot starts");
    if (st == NSASM_OK) {
        hipError_t err = hipMemsetAsync(m->patch_node_start + total, 0, sizeof(int32_t), stream);
        if (err != hipSuccess) st = hip_fail(err, "patch slot padding");
    }
    if (st == NSASM_OK) st = device_alloc(&m->elem_pos, static_cast<size_t>(m->n_elems), "element slots");
    if (st == NSASM_OK) {
        k_patch_fill<<<static_cast<unsigned>(np), kThreads, 0, stream>>>(
            m->conn, m->n_elems, elems, count, m->patch_nodes, m->patch_node_start, m->elem_pos);
        st = check_launch("k_patch_fill");
    }
    if (st == NSASM_OK) {
        hipError_t err = hipStreamSynchronize(stream);
        if (err != hipSuccess) st = hip_fail(err, "patch build");
    }
    if (st != NSASM_OK) {
        device_free(count);
        device_free(m->patch_nodes);
        device_free(m->patch_node_start);
        device_free(m->elem_pos);
        m->patch_nodes = nullptr;
        m->patch_node_start = nullptr;
        m->elem_pos = nullptr;
        return st;
    }
    m->patch_off = reinterpret_cast<int32_t *>(count);
    m->n_patches = static_cast<int32_t>(np);
    m->patch_elems = elems;
    m->max_patch_nodes = static_cast<int32_t>(max_nodes);
    m->patch_node_refs = total;
    return NSASM_OK;
}

// Node-major index of the patch references (for the deterministic gather of
// per-patch partial sums) and the partial-sum buffer itself.
nsasm_status build_node_gather(nsasm_mesh *m, hipStream_t stream) {
    const int64_t nn = m->n_nodes, refs = m->patch_node_refs;
    uint32_t *off = nullptr, *keys = nullptr;
    NSASM_TRY(device_alloc(&off, static_cast<size_t>(nn + 1), "node reference offsets"));
    nsasm_status st = device_alloc(&keys, static_cast<size_t>(refs), "node reference keys");
    int32_t *refs_sorted = nullptr;
    if (st == NSASM_OK) st = device_alloc(&refs_sorted, static_cast<size_t>(refs), "node references");
    if (st == NSASM_OK) st = device_alloc(&m->ref_slot, static_cast<size_t>(refs), "reference slots");
    if (st == NSASM_OK) st = device_alloc(&m->partial, static_cast<size_t>(3 * refs), "patch partial sums");
    if (st == NSASM_OK) {
        hipError_t err = hipMemsetAsync(off, 0, sizeof(uint32_t) * (nn + 1), stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(keys, m->patch_nodes, sizeof(uint32_t) * refs, hipMemcpyDeviceToDevice, stream);
        if (err != hipSuccess) st = hip_fail(err, "node reference setup");
    }
    if (st == NSASM_OK) {
        k_count_refs<<<blocks_for(refs), kThreads, 0, stream>>>(m->patch_nodes, refs, off);
        st = check_launch("k_count_refs");
    }
    if (st == NSASM_OK) st = exclusive_scan_u32(off, off, nn + 1, nullptr, stream);
    if (st == NSASM_OK) {
        k_iota<<<blocks_for(refs), kThreads, 0, stream>>>(refs_sorted, refs);
        st = check_launch("k_iota");
    }
    int bits = 1;
    while (bits < 31 && (int64_t(1) << bits) < nn) ++bits;
    // stable: each node's references stay in patch order
    if (st == NSASM_OK) st = radix_sort_pairs_u32(keys, refs_sorted, refs, bits, stream);
    if (st == NSASM_OK) {
        k_invert<<<blocks_for(refs), kThreads, 0, stream>>>(refs_sorted, refs, m->ref_slot);
        st = check_launch("k_invert");
    }
    if (st == NSASM_OK) {
        hipError_t err = hipStreamSynchronize(stream);
        if (err != hipSuccess) st = hip_fail(err, "node gather build");
    }
    device_free(keys);
    device_free(refs_sorted);
    if (st != NSASM_OK) {
        device_free(off);
        device_free(m->ref_slot);
        device_free(m->partial);
        m->ref_slot = nullptr;
        m->partial = nullptr;
        return st;
    }
    m->node_ref_off = reinterpret_cast<int32_t *>(off);
    return NSASM_OK;
}

// Padded patch records (and partial-sum positions with the gather scatter)
// from the compact lists, which are then freed.
nsasm_status build_patch_records(nsasm_mesh *m, hipStream_t stream) {
    const int stride = (m->max_patch_nodes + 7) / 8 * 8;
    const size_t n = static_cast<size_t>(m->n_patches) * stride;
    NSASM_TRY(device_alloc(&m->patch_rec, n, "patch records"));
    const bool gather = m->scatter == NSASM_SCATTER_PATCH_GATHER;
    if (gather) NSASM_TRY(device_alloc(&m->patch_ref, n, "patch partial positions"));
    NSASM_TRY(device_alloc(&m->elem_loc, static_cast<size_t>(m->n_elems), "element LDS positions"));
    uint8_t *position = nullptr;
    NSASM_TRY(device_alloc(&position, static_cast<size_t>(m->patch_node_refs), "patch node positions"));
    const uint32_t *off = reinterpret_cast<const uint32_t *>(m->patch_off);
    k_patch_color<<<static_cast<unsigned>(m->n_patches), kThreads, 0, stream>>>(
        off, m->patch_node_start, m->elem_pos, m->n_elems, m->patch_elems, position, m->elem_loc);
    nsasm_status st = check_launch("k_patch_color");
    if (st == NSASM_OK) {
        k_patch_pad<<<static_cast<unsigned>(m->n_patches), kThreads, 0, stream>>>(
            off, m->patch_nodes, m->patch_node_start, position, gather ? m->ref_slot : nullptr, m->n_elems,
            m->patch_elems, stride, m->patch_rec, m->patch_ref);
        st = check_launch("k_patch_pad");
    }
    if (st == NSASM_OK) {
        hipError_t err = hipStreamSynchronize(stream);
        if (err != hipSuccess) st = hip_fail(err, "patch records");
    }
    device_free(position);
    NSASM_TRY(st);
    m->patch_stride = stride;
    free_compact_patches(m);
    return NSASM_OK;
}

nsasm_status create(const double *coords, int64_t nn, const int32_t *conn, int64_t ne,
                    const nsasm_mesh_options &opt, hipStream_t stream, nsasm_mesh *m) {
    m->n_nodes = nn;
    m->n_elems = ne;
    NSASM_HIP(hipGetDevice(&m->device));

    CreateFlags *d_flags = nullptr;
    NSASM_TRY(device_alloc(&d_flags, 1, "create flags"));
    struct Scratch {
        CreateFlags *flags;
        double *box = nullptr;
        uint64_t *keys = nullptr;
        uint32_t *first = nullptr;
        ~Scratch() {
            device_free(flags);
            device_free(box);
            device_free(keys);
            device_free(first);
        }
    } scratch{d_flags};

    const CreateFlags init{0u, INT_MAX};
    NSASM_HIP(hipMemcpyAsync(d_flags, &init, sizeof init, hipMemcpyHostToDevice, stream));
    k_validate_ids<<<blocks_for(ne), kThreads, 0, stream>>>(conn, ne, nn, d_flags);
    NSASM_TRY(check_launch("k_validate_ids"));
    CreateFlags h{};
    NSASM_TRY(read_flags(d_flags, stream, &h));
    if (h.bits & kBadRange)
        return fail(NSASM_ERR_BAD_CONNECTIVITY, "node id out of [0, %lld) (first bad element %d)",
                    static_cast<long long>(nn), h.first_bad);
    if (h.bits & kBadRepeat)
        return fail(NSASM_ERR_BAD_CONNECTIVITY, "repeated node in a tetrahedron (first bad element %d)",
                    h.first_bad);

    NSASM_TRY(device_alloc(&scratch.box, 6 + 6 * kBboxBlocks, "bounding box"));
    k_bbox_partial<<<kBboxBlocks, kThreads, 0, stream>>>(coords, nn, scratch.box + 6);
    NSASM_TRY(check_launch("k_bbox_partial"));
    k_bbox_final<<<1, kThreads, 0, stream>>>(scratch.box + 6, kBboxBlocks, scratch.box);
    NSASM_TRY(check_launch("k_bbox_final"));

    NSASM_TRY(device_alloc(&scratch.keys, static_cast<size_t>(ne), "element keys"));
    NSASM_TRY(device_alloc(&m->user_elem, static_cast<size_t>(ne), "element order"));
    k_element_keys<<<blocks_for(ne), kThreads, 0, stream>>>(coords, conn, ne, scratch.box, scratch.keys,
                                                             m->user_elem, d_flags);
    NSASM_TRY(check_launch("k_element_keys"));
    NSASM_TRY(read_flags(d_flags, stream, &h));
    if (h.bits & kBadDet)
        return fail(NSASM_ERR_DEGENERATE_ELEMENT,
                    "element %d has det J within rounding of zero (|det J| <= 64 eps |d1||d2||d3|), "
                    "a subnormal det J or a non-finite vertex",
                    h.first_bad);

    NSASM_TRY(device_alloc(&m->perm, static_cast<size_t>(nn), "node permutation"));
    NSASM_TRY(device_alloc(&m->iperm, static_cast<size_t>(nn), "inverse node permutation"));
    if (opt.renumber) {
        NSASM_TRY(radix_sort_pairs_u64(scratch.keys, m->user_elem, ne, 63, stream));
        NSASM_TRY(device_alloc(&scratch.first, static_cast<size_t>(nn), "first touch"));
        NSASM_HIP(hipMemsetAsync(scratch.first, 0xff, sizeof(uint32_t) * nn, stream));
        k_first_touch<<<blocks_for(ne), kThreads, 0, stream>>>(conn, m->user_elem, ne, scratch.first);
        NSASM_TRY(check_launch("k_first_touch"));
        k_iota<<<blocks_for(nn), kThreads, 0, stream>>>(m->iperm, nn);
        NSASM_TRY(check_launch("k_iota"));
        // stable: nodes used by no element keep their relative order at the end
        NSASM_TRY(radix_sort_pairs_u32(scratch.first, m->iperm, nn, 32, stream));
        k_invert<<<blocks_for(nn), kThreads, 0, stream>>>(m->iperm, nn, m->perm);
        NSASM_TRY(check_launch("k_invert"));
        m->renumbered = 1;
    } else {
        k_iota<<<blocks_for(ne), kThreads, 0, stream>>>(m->user_elem, ne);
        NSASM_TRY(check_launch("k_iota"));
        k_iota<<<blocks_for(nn), kThreads, 0, stream>>>(m->iperm, nn);
        NSASM_TRY(check_launch("k_iota"));
        k_iota<<<blocks_for(nn), kThreads, 0, stream>>>(m->perm, nn);
        NSASM_TRY(check_launch("k_iota"));
        m->renumbered = 0;
    }

    NSASM_TRY(device_alloc(&m->conn, static_cast<size_t>(ne), "mesh connectivity"));
    k_remap_conn<<<blocks_for(ne), kThreads, 0, stream>>>(conn, m->user_elem, m->perm, ne, m->conn);
    NSASM_TRY(check_launch("k_remap_conn"));
    NSASM_TRY(device_alloc(&m->x, static_cast<size_t>(3 * nn), "mesh coordinates"));
    k_gather_rows<double><<<blocks_for(3 * nn), kThreads, 0, stream>>>(coords, m->iperm, nn, 3, m->x);
    NSASM_TRY(check_launch("k_gather_rows"));

    m->scatter = NSASM_SCATTER_ATOMIC;
    if (opt.scatter != NSASM_SCATTER_ATOMIC) {
        // default size: kMaxPatchElems, halved once if a patch touches too many
        // nodes (a mesh without locality fits neither and keeps atomic scatter)
        int elems = opt.patch_elems > 0 ? opt.patch_elems : kMaxPatchElems;
        nsasm_status st = build_patches(m, elems, stream);
        if (st == NSASM_ERR_UNSUPPORTED && opt.patch_elems == 0) {
            elems /= 2;
            st = build_patches(m, elems, stream);
        }
        if (st == NSASM_OK) {
            m->scatter = (opt.scatter == NSASM_SCATTER_PATCH) ? NSASM_SCATTER_PATCH : NSASM_SCATTER_PATCH_GATHER;
            if (m->scatter == NSASM_SCATTER_PATCH_GATHER) NSASM_TRY(build_node_gather(m, stream));
            NSASM_TRY(build_patch_records(m, stream));
        } else if (!(st == NSASM_ERR_UNSUPPORTED && opt.scatter == NSASM_SCATTER_AUTO)) {
            return st;
        }
    }
    NSASM_TRY(compute_lumped_volume(m, stream));
    NSASM_HIP(hipStreamSynchronize(stream));
    clear_error();
    return NSASM_OK;
}

template <typename T>
nsasm_status reorder(const nsasm_mesh *m, int32_t ncomp, const void *src, void *dst, bool to_mesh,
                     hipStream_t stream) {
    const int32_t *map = to_mesh ? m->iperm : m->perm;
    k_gather_rows<T><<<blocks_for(m->n_nodes * ncomp), kThreads, 0, stream>>>(
        static_cast<const T *>(src), map, m->n_nodes, ncomp, static_cast<T *>(dst));
    return check_launch("k_gather_rows");
}

nsasm_status reorder_entry(const nsasm_mesh *m, int32_t ncomp, nsasm_precision prec, const void *src,
                           void *dst, void *stream, bool to_mesh) {
    if (!m) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    if (ncomp < 1 || ncomp > 16) return fail(NSASM_ERR_INVALID_ARGUMENT, "ncomp must be in 1..16");
    if (prec != NSASM_FP64 && prec != NSASM_MIXED)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown precision %d", static_cast<int>(prec));
    NSASM_TRY(check_device_ptr(src, to_mesh ? "user" : "mesh_ordered"));
    NSASM_TRY(check_device_ptr(dst, to_mesh ? "mesh_ordered" : "user"));
    if (src == dst) return fail(NSASM_ERR_INVALID_ARGUMENT, "source and destination must differ");
    hipStream_t s = static_cast<hipStream_t>(stream);
    nsasm_status st = (prec == NSASM_FP64) ? reorder<double>(m, ncomp, src, dst, to_mesh, s)
                                           : reorder<float>(m, ncomp, src, dst, to_mesh, s);
    if (st == NSASM_OK) clear_error();
    return st;
}

}  // namespace
}  // namespace nsasm

extern "C" nsasm_status nsasm_mesh_create(const double *coords, int64_t n_nodes, const int32_t *conn,
                                          int64_t n_elems, const nsasm_mesh_options *opts, void *stream,
                                          nsasm_mesh **out) {
    using namespace nsasm;
    if (!out) return fail(NSASM_ERR_INVALID_ARGUMENT, "out is NULL");
    *out = nullptr;
    if (!coords) return fail(NSASM_ERR_INVALID_ARGUMENT, "coords is NULL");
    if (!conn) return fail(NSASM_ERR_INVALID_ARGUMENT, "conn is NULL");
    if (n_nodes <= 0 || n_nodes >= (int64_t(1) << 31))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "n_nodes must be in [1, 2^31)");
    if (n_elems <= 0 || n_elems >= (int64_t(1) << 29))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "n_elems must be in [1, 2^29)");
    nsasm_mesh_options opt{1, NSASM_SCATTER_AUTO, 0, 0};
    if (opts) opt = *opts;
    if (opt.renumber != 0 && opt.renumber != 1)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "renumber must be 0 or 1");
    if (opt.scatter < NSASM_SCATTER_AUTO || opt.scatter > NSASM_SCATTER_PATCH_GATHER)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown scatter mode %d", opt.scatter);
    if (opt.patch_elems != 0 &&
        (opt.patch_elems < 32 || opt.patch_elems > kMaxPatchElems || opt.patch_elems % 32 != 0))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "patch_elems must be 0 or a multiple of 32 in [32, 256]");
    if (opt.reserved != 0) return fail(NSASM_ERR_INVALID_ARGUMENT, "reserved option must be 0");
    NSASM_TRY(check_device_ptr(coords, "coords"));
    NSASM_TRY(check_device_ptr(conn, "conn"));

    nsasm_mesh *m = new (std::nothrow) nsasm_mesh();
    if (!m) return fail(NSASM_ERR_OUT_OF_MEMORY, "host allocation of the mesh handle failed");
    nsasm_status st = create(coords, n_nodes, conn, n_elems, opt, static_cast<hipStream_t>(stream), m);
    if (st != NSASM_OK) {
        std::string msg = nsasm_last_error();
        (void)hipStreamSynchronize(static_cast<hipStream_t>(stream));
        free_mesh(m);
        fail(st, "%s", msg.c_str());
        return st;
    }
    *out = m;
    return NSASM_OK;
}

extern "C" nsasm_status nsasm_mesh_destroy(nsasm_mesh *mesh) {
    if (!mesh) return NSASM_OK;
    hipError_t err = hipDeviceSynchronize();
    nsasm::free_mesh(mesh);
    if (err != hipSuccess) return nsasm::hip_fail(err, "hipDeviceSynchronize in nsasm_mesh_destroy");
    nsasm::clear_error();
    return NSASM_OK;
}

extern "C" nsasm_status nsasm_mesh_info(const nsasm_mesh *mesh, nsasm_mesh_info_t *info) {
    using namespace nsasm;
    if (!mesh) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    if (!info) return fail(NSASM_ERR_INVALID_ARGUMENT, "info is NULL");
    *info = nsasm_mesh_info_t{};
    info->n_nodes = mesh->n_nodes;
    info->n_elems = mesh->n_elems;
    info->scatter = mesh->scatter;
    info->renumbered = mesh->renumbered;
    info->n_patches = mesh->n_patches;
    info->patch_elems = mesh->patch_elems;
    info->max_patch_nodes = mesh->max_patch_nodes;
    info->patch_node_refs = mesh->patch_node_refs;
    clear_error();
    return NSASM_OK;
}

extern "C" nsasm_status nsasm_mesh_permutation(const nsasm_mesh *mesh, int32_t *mesh_id_of_user,
                                               void *stream) {
    using namespace nsasm;
    if (!mesh) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    NSASM_TRY(check_device_ptr(mesh_id_of_user, "mesh_id_of_user"));
    NSASM_HIP(hipMemcpyAsync(mesh_id_of_user, mesh->perm, sizeof(int32_t) * mesh->n_nodes,
                             hipMemcpyDeviceToDevice, static_cast<hipStream_t>(stream)));
    clear_error();
    return NSASM_OK;
}

extern "C" nsasm_status nsasm_mesh_connectivity(const nsasm_mesh *mesh, int32_t *conn_mesh,
                                                int32_t *user_elem, void *stream) {
    using namespace nsasm;
    if (!mesh) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (conn_mesh) {
        NSASM_TRY(check_device_ptr(conn_mesh, "conn_mesh"));
        NSASM_HIP(hipMemcpyAsync(conn_mesh, mesh->conn, sizeof(int4) * mesh->n_elems,
                                 hipMemcpyDeviceToDevice, s));
    }
    if (user_elem) {
        NSASM_TRY(check_device_ptr(user_elem, "user_elem"));
        NSASM_HIP(hipMemcpyAsync(user_elem, mesh->user_elem, sizeof(int32_t) * mesh->n_elems,
                                 hipMemcpyDeviceToDevice, s));
    }
    clear_error();
    return NSASM_OK;
}

extern "C" nsasm_status nsasm_to_mesh_order(const nsasm_mesh *mesh, int32_t ncomp,
                                            nsasm_precision precision, const void *user,
                                            void *mesh_ordered, void *stream) {
    return nsasm::reorder_entry(mesh, ncomp, precision, user, mesh_ordered, stream, true);
}

extern "C" nsasm_status nsasm_from_mesh_order(const nsasm_mesh *mesh, int32_t ncomp,
                                              nsasm_precision precision, const void *mesh_ordered,
                                              void *user, void *stream) {
    return nsasm::reorder_entry(mesh, ncomp, precision, mesh_ordered, user, stream, false);
}

extern "C" nsasm_status nsasm_mesh_lumped_volume(const nsasm_mesh *mesh, double *lumped, void *stream) {
    using namespace nsasm;
    if (!mesh) return fail(NSASM_ERR_INVALID_ARGUMENT, "mesh is NULL");
    NSASM_TRY(check_device_ptr(lumped, "lumped"));
    NSASM_HIP(hipMemcpyAsync(lumped, mesh->lumped, sizeof(double) * mesh->n_nodes, hipMemcpyDeviceToDevice,
                             static_cast<hipStream_t>(stream)));
    clear_error();
    return NSASM_OK;
}
