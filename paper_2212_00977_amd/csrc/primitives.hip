// Device-wide exclusive scan and stable LSD radix sort (gfx950, wave64).
#include "spc_internal.h"

namespace spc {

namespace {

constexpr int kItems = 8;
constexpr uint64_t kTile = (uint64_t)kBlock * kItems;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_sums(const T *in, uint64_t n, uint64_t *sums) {
    __shared__ uint64_t lds4[kWaves];
    uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++)
        if (base + j < n) s += (uint64_t)in[base + j];
    uint64_t total;
    (void)block_excl_scan<uint64_t>(s, lds4, total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_tile_scan(const T *in, uint64_t *out, uint64_t n,
                                                      const uint64_t *tile_prefix) {
    __shared__ uint64_t lds4[kWaves];
    uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
    uint64_t v[kItems];
    uint64_t s = 0;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        v[j] = (base + j < n) ? (uint64_t)in[base + j] : 0;
        s += v[j];
    }
    uint64_t total;
    uint64_t pre = block_excl_scan<uint64_t>(s, lds4, total);
    uint64_t tp = tile_prefix ? tile_prefix[blockIdx.x] : 0;
    uint64_t run = tp + pre;
#pragma unroll
    for (int j = 0; j < kItems; j++) {
        if (base + j < n) out[base + j] = run;
        run += v[j];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[n] = tp + total;
}

__global__ void k_set_zero_u64(uint64_t *p) { *p = 0; }

template <typename T>
spc_status scan_rec(const T *in, uint64_t *out, uint64_t n, uint64_t *ws, hipStream_t st) {
    if (n == 0) {
        hipLaunchKernelGGL(k_set_zero_u64, dim3(1), dim3(1), 0, st, out);
        SPC_LAUNCHED();
        return SPC_OK;
    }
    uint64_t tiles = (n + kTile - 1) / kTile;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_tile_scan<T>, dim3(1), dim3(kBlock), 0, st, in, out, n,
                           (const uint64_t *)nullptr);
        SPC_LAUNCHED();
        return SPC_OK;
    }
    uint64_t *sums = ws, *sums_scan = ws + tiles, *rest = ws + 2 * tiles + 1;
    hipLaunchKernelGGL(k_tile_sums<T>, dim3((uint32_t)tiles), dim3(kBlock), 0, st, in, n, sums);
    SPC_LAUNCHED();
    SPC_TRY(scan_rec<uint64_t>(sums, sums_scan, tiles, rest, st));
    hipLaunchKernelGGL(k_tile_scan<T>, dim3((uint32_t)tiles), dim3(kBlock), 0, st, in, out, n,
                       (const uint64_t *)sums_scan);
    SPC_LAUNCHED();
    return SPC_OK;
}

// ---------------------------------------------------------------------------
// Radix sort: 8-bit digits, tiles of 2048 keys; per pass one histogram
// kernel, one scan of the digit-major histogram, one stable scatter.  Within
// a tile the keys are ranked in index order (round-major, lane-minor), with
// wave ballots matching equal digits, so the sort is stable.
// ---------------------------------------------------------------------------
constexpr int kRadix = 256;

__global__ __launch_bounds__(kBlock) void k_radix_hist(const uint64_t *keys, uint64_t n, int shift,
                                                       uint64_t *hist, uint32_t nblocks) {
    __shared__ uint32_t h[kRadix];
    h[threadIdx.x] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int r = 0; r < kItems; r++) {
        uint64_t i = base + (uint64_t)r * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void k_radix_scatter(const uint64_t *keys, const uint32_t *vals,
                                                          uint64_t *okeys, uint32_t *ovals,
                                                          uint64_t n, int shift,
                                                          const uint64_t *hist_scan,
                                                          uint32_t nblocks) {
    __shared__ uint64_t run[kRadix];
    __shared__ uint32_t wcnt[kWaves][kRadix];
    __shared__ uint64_t wpre[kWaves][kRadix];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    run[t] = hist_scan[(uint64_t)t * nblocks + blockIdx.x];
    for (int i = 0; i < kWaves; i++) wcnt[i][t] = 0;
    __syncthreads();
    uint64_t base = (uint64_t)blockIdx.x * kTile;
    for (int r = 0; r < kItems; r++) {
        uint64_t i = base + (uint64_t)r * kBlock + t;
        bool valid = i < n;
        uint64_t key = valid ? keys[i] : 0;
        uint32_t val = (valid && vals) ? vals[i] : 0;
        uint32_t dg = (uint32_t)(key >> shift) & 0xFF;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bb = __ballot((dg >> b) & 1);
            peers &= ((dg >> b) & 1) ? bb : ~bb;
        }
        uint32_t rank = __popcll(peers & lanemask_lt());
        bool leader = valid && (peers & lanemask_lt()) == 0;
        if (leader) wcnt[w][dg] = __popcll(peers);
        __syncthreads();
        {
            uint64_t acc = run[t];
            for (int k = 0; k < kWaves; k++) {
                wpre[k][t] = acc;
                acc += wcnt[k][t];
            }
            run[t] = acc;
        }
        __syncthreads();
        if (valid) {
            uint64_t pos = wpre[w][dg] + rank;
            okeys[pos] = key;
            if (vals) ovals[pos] = val;
        }
        for (int k = 0; k < kWaves; k++) wcnt[k][t] = 0;
        __syncthreads();
    }
}

}  // namespace

size_t scan_ws_elems(uint64_t n) {
    size_t total = 4;
    while (n > kTile) {
        uint64_t tiles = (n + kTile - 1) / kTile;
        total += 2 * tiles + 1;
        n = tiles;
    }
    return total;
}

spc_status scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, uint64_t *ws, hipStream_t st) {
    return scan_rec<uint32_t>(in, out, n, ws, st);
}
spc_status scan_u64(const uint64_t *in, uint64_t *out, uint64_t n, uint64_t *ws, hipStream_t st) {
    return scan_rec<uint64_t>(in, out, n, ws, st);
}

size_t radix_ws_elems(uint64_t n) {
    uint64_t nblocks = (n + kTile - 1) / kTile;
    uint64_t h = nblocks * kRadix;
    return 2 * h + 1 + scan_ws_elems(h);
}

spc_status radix_sort_pairs(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                            uint64_t n, int bits, uint64_t *ws, hipStream_t st) {
    if (n <= 1 || bits <= 0) return SPC_OK;
    uint32_t nblocks = (uint32_t)((n + kTile - 1) / kTile);
    uint64_t h = (uint64_t)nblocks * kRadix;
    uint64_t *hist = ws, *hist_scan = ws + h, *rest = ws + 2 * h + 1;
    uint64_t *ka = keys, *kb = keys_alt;
    uint32_t *va = vals, *vb = vals_alt;
    int passes = (bits + 7) / 8;
    for (int p = 0; p < passes; p++) {
        int shift = 8 * p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblocks), dim3(kBlock), 0, st, ka, n, shift, hist,
                           nblocks);
        SPC_LAUNCHED();
        SPC_TRY(scan_u64(hist, hist_scan, h, rest, st));
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblocks), dim3(kBlock), 0, st, ka, va, kb, vb, n,
                           shift, hist_scan, nblocks);
        SPC_LAUNCHED();
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        SPC_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, st));
        if (vals) SPC_HIP(hipMemcpyAsync(vals, va, n * sizeof(uint32_t), hipMemcpyDeviceToDevice, st));
    }
    return SPC_OK;
}

}  // namespace spc
