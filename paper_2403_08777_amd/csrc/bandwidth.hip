// Machine measurements the roofline analysis rests on.
//
// Attainable HBM bandwidth: the Scale kernel b = s a over FP64 arrays, the
// streaming measurement the paper prices its machine balance with (Sec. III-C:
// the measured Scale bandwidth against the FP64 peak, 7 flop/B on its GPU).  One
// read and one write stream per element, no reuse, so with arrays much larger
// than the last-level cache its rate is the bandwidth a kernel can draw.
//
// Atomic scatter rate: out[index[k]][c] += value with device-scope atomic
// adds, the immediate scatter of the paper's final kernel (Sec. V-D: each
// element adds its local RHS straight into the global vector) on its own,
// without the element arithmetic, so its cost can be priced per atomic.
#include <cstdint>

#include "internal.hpp"

namespace nsasm {
namespace {

constexpr int kThreads = 256;
constexpr int kUnroll = 4;  // 16-byte loads in flight per thread before the stores

// b[k] = s a[k] over n2 16-byte pairs; every load of a thread is issued
// before its first store.  The odd last element of the FP64 array (when n is
// odd) is done by thread 0 of block 0 through the scalar pointers.
__global__ __launch_bounds__(kThreads) void k_scale_pairs(const double2 *__restrict__ a, double2 *__restrict__ b,
                                                          int64_t n2, double s, const double *__restrict__ a_tail,
                                                          double *__restrict__ b_tail) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kUnroll * kThreads) + threadIdx.x;
    double2 v[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
        const int64_t k = base + j * kThreads;
        v[j] = k < n2 ? a[k] : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
        const int64_t k = base + j * kThreads;
        if (k < n2) b[k] = make_double2(s * v[j].x, s * v[j].y);
    }
    if (a_tail && blockIdx.x == 0 && threadIdx.x == 0) *b_tail = s * *a_tail;
}

// The same for arrays that are not both 16-byte aligned, one double a lane.
__global__ __launch_bounds__(kThreads) void k_scale(const double *__restrict__ a, double *__restrict__ b, int64_t n,
                                                    double s) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * (kUnroll * kThreads) + threadIdx.x;
    double v[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
        const int64_t k = base + j * kThreads;
        v[j] = k < n ? a[k] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j) {
        const int64_t k = base + j * kThreads;
        if (k < n) b[k] = s * v[j];
    }
}

// One thread per index entry: ncomp device-scope atomic adds of `value`
// (entries outside [0, rows) are skipped).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scatter_add(const int32_t *__restrict__ index, int64_t n, int ncomp,
                                                          T value, T *out, int64_t rows) {
    const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
    if (k >= n) return;
    const int64_t row = index[k];
    if (row < 0 || row >= rows) return;
    T *dst = out + row * ncomp;
    for (int c = 0; c < ncomp; ++c) __hip_atomic_fetch_add(dst + c, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace
}  // namespace nsasm

extern "C" nsasm_status nsasm_scatter_add(const int32_t *index, int64_t n, int32_t ncomp, nsasm_precision precision,
                                          double value, void *out, int64_t n_out_rows, void *stream) {
    using namespace nsasm;
    clear_error();
    if (n < 0 || n_out_rows < 0)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "n and n_out_rows must be >= 0 (got %lld, %lld)",
                    static_cast<long long>(n), static_cast<long long>(n_out_rows));
    if (ncomp < 1 || ncomp > 16) return fail(NSASM_ERR_INVALID_ARGUMENT, "ncomp must be in [1, 16] (got %d)", ncomp);
    if (precision != NSASM_FP64 && precision != NSASM_MIXED)
        return fail(NSASM_ERR_INVALID_ARGUMENT, "unknown precision %d", static_cast<int>(precision));
    if (n == 0) return NSASM_OK;
    if ((n + kThreads - 1) / kThreads > int64_t(0x7fffffff))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "n = %lld is too large", static_cast<long long>(n));
    NSASM_TRY(check_device_ptr(index, "index"));
    NSASM_TRY(check_device_ptr(out, "out"));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const unsigned blocks = static_cast<unsigned>((n + kThreads - 1) / kThreads);
    if (precision == NSASM_FP64)
        k_scatter_add<double><<<blocks, kThreads, 0, st>>>(index, n, ncomp, value, static_cast<double *>(out),
                                                           n_out_rows);
    else
        k_scatter_add<float><<<blocks, kThreads, 0, st>>>(index, n, ncomp, static_cast<float>(value),
                                                          static_cast<float *>(out), n_out_rows);
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? NSASM_OK : hip_fail(err, "k_scatter_add launch");
}

extern "C" nsasm_status nsasm_stream_scale(const double *a, double *b, int64_t n, double s, void *stream) {
    using namespace nsasm;
    clear_error();
    if (n < 0) return fail(NSASM_ERR_INVALID_ARGUMENT, "n must be >= 0 (got %lld)", static_cast<long long>(n));
    if (n == 0) return NSASM_OK;
    constexpr int64_t kPerBlock = int64_t(kUnroll) * kThreads;
    // blocks of the scalar kernel (the larger grid) must fit a 32-bit grid
    if ((n + kPerBlock - 1) / kPerBlock > int64_t(0x7fffffff))
        return fail(NSASM_ERR_INVALID_ARGUMENT, "n = %lld is too large", static_cast<long long>(n));
    NSASM_TRY(check_device_ptr(a, "a"));
    NSASM_TRY(check_device_ptr(b, "b"));
    const char *pa = reinterpret_cast<const char *>(a), *pb = reinterpret_cast<const char *>(b);
    const size_t bytes = sizeof(double) * static_cast<size_t>(n);
    if (pa < pb + bytes && pb < pa + bytes) return fail(NSASM_ERR_INVALID_ARGUMENT, "a and b overlap");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const bool paired = ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15u) == 0;
    if (paired) {
        const int64_t n2 = n / 2;
        const bool odd = (n & 1) != 0;
        const int64_t blocks = n2 > 0 ? (n2 + kPerBlock - 1) / kPerBlock : 1;
        k_scale_pairs<<<static_cast<unsigned>(blocks), kThreads, 0, st>>>(
            reinterpret_cast<const double2 *>(a), reinterpret_cast<double2 *>(b), n2, s, odd ? a + (n - 1) : nullptr,
            odd ? b + (n - 1) : nullptr);
    } else {
        const int64_t blocks = (n + kPerBlock - 1) / kPerBlock;
        k_scale<<<static_cast<unsigned>(blocks), kThreads, 0, st>>>(a, b, n, s);
    }
    hipError_t err = hipGetLastError();
    return err == hipSuccess ? NSASM_OK : hip_fail(err, "k_scale launch");
}
