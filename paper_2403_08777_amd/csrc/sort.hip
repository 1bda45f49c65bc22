// Device-wide exclusive scan and stable LSD radix sort (key/value pairs) used by
// mesh preprocessing.  Plain hand-written HIP for wave64: ballots for in-wave
// digit matching, LDS for block-level counts.
#include <utility>

#include "internal.hpp"

namespace nsasm {
namespace {

constexpr int kThreads = 256;
constexpr int kScanItems = 4;                         // per thread
constexpr int kScanTile = kThreads * kScanItems;      // 1024
constexpr int kSortItems = 8;                         // per thread
constexpr int kSortTile = kThreads * kSortItems;      // 2048
constexpr int kRadix = 256;                           // 8-bit digits

__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t *lds4, uint32_t *total) {
    return block_exclusive_scan_256(v, lds4, total);
}

__global__ __launch_bounds__(kThreads) void k_scan_block_sums(const uint32_t *in, int64_t n,
                                                               uint32_t *sums) {
    __shared__ uint32_t lds4[4];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    uint32_t total;
    (void)block_exclusive_scan(s, lds4, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// Exclusive scan of each 1024-item tile plus the tile's offset (offsets may be
// null for a single tile); writes the grand total when `total_out` is set.
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const uint32_t *in, uint32_t *out,
                                                          int64_t n, const uint32_t *offsets,
                                                          uint32_t *total_out) {
    __shared__ uint32_t lds4[4];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = (base + i < n) ? in[base + i] : 0u;
        s += v[i];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, lds4, &total);
    if (offsets) run += offsets[blockIdx.x];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (total_out && threadIdx.x == 0) *total_out = total;
}

nsasm_status scan_recursive(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *d_total,
                            hipStream_t stream) {
    const int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles <= 1) {
        k_scan_tiles<<<1, kThreads, 0, stream>>>(in, out, n, nullptr, d_total);
        NSASM_HIP(hipGetLastError());
        return NSASM_OK;
    }
    uint32_t *sums = nullptr;
    NSASM_TRY(device_alloc(&sums, static_cast<size_t>(tiles), "scan partials"));
    k_scan_block_sums<<<static_cast<unsigned>(tiles), kThreads, 0, stream>>>(in, n, sums);
    nsasm_status st = NSASM_OK;
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) st = hip_fail(err, "k_scan_block_sums");
    if (st == NSASM_OK) st = scan_recursive(sums, sums, tiles, d_total, stream);
    if (st == NSASM_OK) {
        k_scan_tiles<<<static_cast<unsigned>(tiles), kThreads, 0, stream>>>(in, out, n, sums, nullptr);
        err = hipGetLastError();
        if (err != hipSuccess) st = hip_fail(err, "k_scan_tiles");
    }
    // the partials must outlive the kernels that read them
    if (st == NSASM_OK) {
        err = hipStreamSynchronize(stream);
        if (err != hipSuccess) st = hip_fail(err, "scan synchronize");
    }
    device_free(sums);
    return st;
}

// ------------------------------------------------------------- radix sort

template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_histogram(const K *keys, int64_t n, int shift,
                                                               uint32_t *hist, int64_t n_tiles) {
    __shared__ uint32_t h[kRadix];
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
#pragma unroll
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t idx = base + i * kThreads + t;
        if (idx < n) atomicAdd(&h[static_cast<uint32_t>(keys[idx] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[static_cast<int64_t>(t) * n_tiles + blockIdx.x] = h[t];
}

// Stable scatter of one tile.  Items are visited in tile order (round i holds
// positions i*256 .. i*256+255, thread t position i*256+t); an item's rank is
// the count of same-digit items before it: earlier rounds (run[]), lower waves
// of this round (wave_count[][]) and lower lanes of its wave (ballot match).
template <typename K>
__global__ __launch_bounds__(kThreads) void k_radix_scatter(const K *kin, const int32_t *vin,
                                                             K *kout, int32_t *vout, int64_t n,
                                                             int shift, const uint32_t *offsets,
                                                             int64_t n_tiles) {
    __shared__ uint32_t base_off[kRadix];
    __shared__ uint32_t run[kRadix];
    __shared__ uint32_t wave_count[kThreads / 64][kRadix];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    base_off[t] = offsets[static_cast<int64_t>(t) * n_tiles + blockIdx.x];
    run[t] = 0;
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k) wave_count[k][t] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kSortTile;
    const uint64_t lanes_below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int i = 0; i < kSortItems; ++i) {
        const int64_t idx = base + i * kThreads + t;
        const bool valid = idx < n;
        // Items past the end carry digit 255 and are not written.  They sit
        // after every valid item of the tile, so they shift no valid rank.
        const K key = valid ? kin[idx] : K(0);
        const int32_t val = valid ? vin[idx] : 0;
        const uint32_t d = valid ? (static_cast<uint32_t>(key >> shift) & (kRadix - 1)) : kRadix - 1;
        uint64_t peers = ~0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            peers &= bit ? bal : ~bal;
        }
        const uint32_t lower = static_cast<uint32_t>(__popcll(peers & lanes_below));
        if (lower == 0) wave_count[w][d] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        uint32_t pos = base_off[d] + run[d] + lower;
        for (int k = 0; k < w; ++k) pos += wave_count[k][d];
        if (valid) {
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int k = 0; k < kThreads / 64; ++k) {
            add += wave_count[k][t];
            wave_count[k][t] = 0;
        }
        run[t] += add;
        __syncthreads();
    }
}

template <typename K>
nsasm_status radix_sort_pairs(K *keys, int32_t *vals, int64_t n, int key_bits, hipStream_t stream) {
    if (n <= 1) return NSASM_OK;
    if (n >= (int64_t(1) << 31)) return fail(NSASM_ERR_INVALID_ARGUMENT, "sort of %lld items", (long long)n);
    const int passes = (key_bits + 7) / 8;
    const int64_t n_tiles = (n + kSortTile - 1) / kSortTile;
    K *k_alt = nullptr;
    int32_t *v_alt = nullptr;
    uint32_t *hist = nullptr;
    nsasm_status st = device_alloc(&k_alt, static_cast<size_t>(n), "sort keys");
    if (st == NSASM_OK) st = device_alloc(&v_alt, static_cast<size_t>(n), "sort values");
    if (st == NSASM_OK) st = device_alloc(&hist, static_cast<size_t>(n_tiles * kRadix), "sort histogram");
    K *ka = keys, *kb = k_alt;
    int32_t *va = vals, *vb = v_alt;
    for (int pass = 0; pass < passes && st == NSASM_OK; ++pass) {
        const int shift = 8 * pass;
        k_radix_histogram<K><<<static_cast<unsigned>(n_tiles), kThreads, 0, stream>>>(ka, n, shift, hist, n_tiles);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) { st = hip_fail(err, "k_radix_histogram"); break; }
        st = scan_recursive(hist, hist, n_tiles * kRadix, nullptr, stream);
        if (st != NSASM_OK) break;
        k_radix_scatter<K><<<static_cast<unsigned>(n_tiles), kThreads, 0, stream>>>(ka, va, kb, vb, n, shift, hist, n_tiles);
        err = hipGetLastError();
        if (err != hipSuccess) { st = hip_fail(err, "k_radix_scatter"); break; }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (st == NSASM_OK && ka != keys) {
        hipError_t err = hipMemcpyAsync(keys, ka, sizeof(K) * n, hipMemcpyDeviceToDevice, stream);
        if (err == hipSuccess)
            err = hipMemcpyAsync(vals, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, stream);
        if (err != hipSuccess) st = hip_fail(err, "radix sort copy-back");
    }
    hipError_t err = hipStreamSynchronize(stream);
    if (st == NSASM_OK && err != hipSuccess) st = hip_fail(err, "radix sort synchronize");
    device_free(k_alt);
    device_free(v_alt);
    device_free(hist);
    return st;
}

}  // namespace

nsasm_status radix_sort_pairs_u64(uint64_t *keys, int32_t *vals, int64_t n, int key_bits,
                                  hipStream_t stream) {
    return radix_sort_pairs<uint64_t>(keys, vals, n, key_bits, stream);
}

nsasm_status radix_sort_pairs_u32(uint32_t *keys, int32_t *vals, int64_t n, int key_bits,
                                  hipStream_t stream) {
    return radix_sort_pairs<uint32_t>(keys, vals, n, key_bits, stream);
}

nsasm_status exclusive_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                                hipStream_t stream) {
    if (n <= 0) {
        if (total) *total = 0;
        return NSASM_OK;
    }
    if (n >= (int64_t(1) << 31)) return fail(NSASM_ERR_INVALID_ARGUMENT, "scan of %lld items", (long long)n);
    uint32_t *d_total = nullptr;
    NSASM_TRY(device_alloc(&d_total, 1, "scan total"));
    nsasm_status st = scan_recursive(in, out, n, d_total, stream);
    if (st == NSASM_OK) {
        hipError_t err = hipStreamSynchronize(stream);
        if (err == hipSuccess && total)
            err = hipMemcpy(total, d_total, sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (err != hipSuccess) st = hip_fail(err, "scan total");
    }
    device_free(d_total);
    return st;
}

}  // namespace nsasm
