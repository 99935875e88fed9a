// Exclusive prefix sum of uint32 arrays (bucket offsets, rank tables,
// cumulative step counts). Three phases per level: block scans writing block
// totals, a recursive scan of the totals, and a uniform add.
#include "ibip_internal.h"

namespace ibip {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanPer = 4;
constexpr int kScanBlock = kScanThreads * kScanPer;  // 1024 elements per block

__device__ inline uint32_t wave_incl_scan(uint32_t x, int lane) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t t = __shfl_up(x, o, 64);
        if (lane >= o) x += t;
    }
    return x;
}

// Exclusive scan of each 1024-element block in place; block totals to `sums`.
__global__ __launch_bounds__(kScanThreads) void scan_blocks(uint32_t* data, int64_t n, uint32_t* sums) {
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)tid * kScanPer;
    uint32_t v[kScanPer];
    uint32_t tsum = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; j++) {
        v[j] = (base + j < n) ? data[base + j] : 0u;
        tsum += v[j];
    }
    uint32_t incl = wave_incl_scan(tsum, lane);
    if (lane == 63) wsum[wid] = incl;
    __syncthreads();
    uint32_t wpre = 0, total = 0;
#pragma unroll
    for (int w = 0; w < kScanThreads / 64; w++) {
        if (w < wid) wpre += wsum[w];
        total += wsum[w];
    }
    uint32_t run = wpre + incl - tsum;
#pragma unroll
    for (int j = 0; j < kScanPer; j++) {
        if (base + j < n) data[base + j] = run;
        run += v[j];
    }
    if (tid == 0) sums[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void scan_add(uint32_t* data, int64_t n, const uint32_t* sums) {
    const uint32_t add = sums[blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kScanBlock;
    for (int j = threadIdx.x; j < kScanBlock; j += kScanThreads) {
        int64_t i = base + j;
        if (i < n) data[i] += add;
    }
}

__global__ void copy_total(const uint32_t* sums, uint32_t* total) { *total = sums[0]; }

hipError_t scan_rec(uint32_t* data, int64_t n, uint32_t* partials, uint32_t* total, hipStream_t s) {
    const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
    uint32_t* sums = partials;
    hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    if (nb == 1) {
        hipLaunchKernelGGL(copy_total, dim3(1), dim3(1), 0, s, sums, total);
        return hipGetLastError();
    }
    hipError_t e = scan_rec(sums, nb, partials + nb, total, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n, sums);
    return hipGetLastError();
}

__global__ void k_sum_slots(const uint32_t* slots, uint32_t* dst) {
    uint32_t v = threadIdx.x < kCountSlots ? slots[threadIdx.x] : 0u;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (threadIdx.x == 0) *dst = v;
}

__global__ void k_sum_copies(const uint32_t* in, int copies, int64_t K, uint32_t* out) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    uint32_t v = 0;
    for (int c = 0; c < copies; c++) v += in[c * K + k];
    out[k] = v;
}

}  // namespace

hipError_t launch_sum_copies(const uint32_t* in, int copies, int64_t K, uint32_t* out, hipStream_t s) {
    if (K <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sum_copies, dim3((unsigned)((K + 255) / 256)), dim3(256), 0, s, in, copies, K, out);
    return hipGetLastError();
}

hipError_t launch_sum_slots(const uint32_t* slots, uint32_t* dst, hipStream_t s) {
    hipLaunchKernelGGL(k_sum_slots, dim3(1), dim3(64), 0, s, slots, dst);
    return hipGetLastError();
}

// `partials` must hold at least n / 1023 + 8 entries.
hipError_t launch_scan_u32(uint32_t* data, int64_t n, uint32_t* partials, uint32_t* total, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    return scan_rec(data, n, partials, total, s);
}

}  // namespace ibip
