// Internal declarations shared by the nsasm library sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "nsasm.h"

namespace nsasm {

// ------------------------------------------------------------------ errors

// Record `status` with a printf-style message for nsasm_last_error(); returns status.
nsasm_status fail(nsasm_status status, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
void clear_error();

// Caller-owned HIP events that time the kernels of the next assembly call on
// a thread (nsasm_set_kernel_events); any may be null.
struct KernelEvents {
    hipEvent_t element_start = nullptr;
    hipEvent_t element_stop = nullptr;
    hipEvent_t gather_start = nullptr;
    hipEvent_t gather_stop = nullptr;
};

// The events set by nsasm_set_kernel_events on this thread (all null if
// none); the pending events are cleared.
KernelEvents take_kernel_events();

// Map a HIP error to NSASM_ERR_DEVICE (or OUT_OF_MEMORY) with context.
nsasm_status hip_fail(hipError_t err, const char *what);

#define NSASM_HIP(call)                                               \
    do {                                                              \
        hipError_t e_ = (call);                                       \
        if (e_ != hipSuccess) return ::nsasm::hip_fail(e_, #call);    \
    } while (0)

#define NSASM_TRY(expr)                                               \
    do {                                                              \
        nsasm_status s_ = (expr);                                     \
        if (s_ != NSASM_OK) return s_;                                \
    } while (0)

// NSASM_OK if p is a device (or managed) allocation visible to the current device.
nsasm_status check_device_ptr(const void *p, const char *name);

// hipMalloc with a test hook: NSASM_TEST_FAIL_ALLOC=k makes the k-th call (1-based,
// counted per process) report out-of-memory.
nsasm_status device_alloc(void **p, size_t bytes, const char *what);
template <typename T>
nsasm_status device_alloc(T **p, size_t count, const char *what) {
    return device_alloc(reinterpret_cast<void **>(p), count * sizeof(T), what);
}
void device_free(void *p);

// ------------------------------------------------------------------- mesh

constexpr int kMaxPatchNodes = 256;  // local node ids are one byte
constexpr int kMaxPatchElems = 256;
constexpr int kNumXcd = 8;           // MI355X: 8 XCDs, workgroups dealt round-robin

}  // namespace nsasm

struct nsasm_mesh {
    int device = 0;
    int64_t n_nodes = 0;
    int64_t n_elems = 0;
    int32_t renumbered = 0;
    int32_t scatter = NSASM_SCATTER_ATOMIC;

    int32_t *perm = nullptr;      // [n_nodes] mesh id of user node
    int32_t *iperm = nullptr;     // [n_nodes] user id of mesh node
    int32_t *user_elem = nullptr; // [n_elems] user element of mesh element
    int4 *conn = nullptr;         // [n_elems] mesh node ids, mesh element order
    double *x = nullptr;          // [n_nodes * 3] coordinates, mesh order

    // element patches (scatter == PATCH or PATCH_GATHER)
    int32_t n_patches = 0;
    int32_t patch_elems = 0;
    int32_t max_patch_nodes = 0;
    int32_t patch_stride = 0;       // entries per patch in patch_rec / patch_ref (>= max_patch_nodes)
    int64_t patch_node_refs = 0;
    // [n_patches * patch_stride]: the patch's distinct nodes, ascending, as
    // {mesh node id, first slot | end slot << 11 | LDS position << 22};
    // {-1, 0} pads each patch
    int2 *patch_rec = nullptr;
    ushort4 *elem_pos = nullptr;    // [n_elems] slot of each (element, vertex)
    uchar4 *elem_loc = nullptr;     // [n_elems] LDS position of each vertex's node in its patch

    // deterministic gather of per-patch partial sums (scatter == PATCH_GATHER)
    int32_t *node_ref_off = nullptr;  // [n_nodes + 1] each node's run in the partial buffer
    int32_t *patch_ref = nullptr;     // as patch_rec: node-major partial-sum position of each entry
    double *partial = nullptr;        // [3 * patch_node_refs] partial sums (float or double)

    // compact patch lists, used while the mesh is built and freed after
    int32_t *patch_off = nullptr;          // [n_patches + 1] offsets into patch_nodes
    int32_t *patch_nodes = nullptr;        // distinct mesh node ids of each patch, ascending
    int32_t *patch_node_start = nullptr;   // first slot of each patch node (same indexing, +1 padding)
    int32_t *ref_slot = nullptr;           // [patch_node_refs] node-major position of each reference

    double *lumped = nullptr;         // [n_nodes] lumped volume V^L, mesh order
};

namespace nsasm {

// Device-wide primitives (sort.hip).  All asynchronous on `stream`; scratch
// buffers are allocated and freed inside (so these synchronise on return).
// Stable LSD radix sort of (key, value) pairs; key_bits <= 64 bits are sorted.
nsasm_status radix_sort_pairs_u64(uint64_t *keys, int32_t *vals, int64_t n, int key_bits,
                                  hipStream_t stream);
nsasm_status radix_sort_pairs_u32(uint32_t *keys, int32_t *vals, int64_t n, int key_bits,
                                  hipStream_t stream);
// out[i] = sum_{k<i} in[i]; out may alias in.  n < 2^31.  Returns the total in *total
// (host, after a synchronisation) if total != nullptr.
nsasm_status exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                                hipStream_t stream);

// Fill m->lumped (allocated here) with the lumped volume of every node
// (assemble.hip); asynchronous on `stream`.
nsasm_status compute_lumped_volume(nsasm_mesh *m, hipStream_t stream);

// Grid of `n_tiles` workgroups padded to a multiple of the XCD count; see xcd_tile().
inline unsigned xcd_grid(int64_t n_tiles) {
    int64_t per = (n_tiles + kNumXcd - 1) / kNumXcd;
    return static_cast<unsigned>(per * kNumXcd);
}

}  // namespace nsasm

// Exclusive scan of one value per thread over a 256-thread block; lds4 holds
// 4 words of scratch.  Every thread of the block must call it.
__device__ inline uint32_t block_exclusive_scan_256(uint32_t v, uint32_t *lds4, uint32_t *total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds4[w] = x;
    __syncthreads();
    uint32_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        uint32_t s = lds4[k];
        before += (k < w) ? s : 0u;
        all += s;
    }
    __syncthreads();
    *total = all;
    return before + x - v;
}

// Rows of adj(J) for J = [d_1 | d_2 | d_3], d_k = x_k - x_0: c_1 = d_2 x d_3,
// c_2 = d_3 x d_1, c_3 = d_1 x d_2; returns det J = d_1 . c_1.  The assembly
// kernels and the mesh validation both call this, so the determinant a mesh
// is validated with is the one the kernels invert.
__device__ inline double tet_adjugate(const double (&xe)[4][3], double (&c1)[3], double (&c2)[3],
                                      double (&c3)[3], double (&d1)[3]) {
    double d2[3], d3[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        d1[i] = xe[1][i] - xe[0][i];
        d2[i] = xe[2][i] - xe[0][i];
        d3[i] = xe[3][i] - xe[0][i];
    }
    c1[0] = d2[1] * d3[2] - d2[2] * d3[1];
    c1[1] = d2[2] * d3[0] - d2[0] * d3[2];
    c1[2] = d2[0] * d3[1] - d2[1] * d3[0];
    c2[0] = d3[1] * d1[2] - d3[2] * d1[1];
    c2[1] = d3[2] * d1[0] - d3[0] * d1[2];
    c2[2] = d3[0] * d1[1] - d3[1] * d1[0];
    c3[0] = d1[1] * d2[2] - d1[2] * d2[1];
    c3[1] = d1[2] * d2[0] - d1[0] * d2[2];
    c3[2] = d1[0] * d2[1] - d1[1] * d2[0];
    return d1[0] * c1[0] + d1[1] * c1[1] + d1[2] * c1[2];
}

// Workgroup b runs on XCD (b mod 8).  Give each XCD one contiguous run of
// tiles so that tiles sharing nodes (neighbours along the element curve) share one L2.
// Valid only for grids built by xcd_grid(); returns a tile index that may be
// >= the real tile count (the caller exits).
__device__ inline int64_t xcd_tile(unsigned b, unsigned grid) {
    const unsigned per = grid / nsasm::kNumXcd;
    return static_cast<int64_t>(b % nsasm::kNumXcd) * per + b / nsasm::kNumXcd;
}
