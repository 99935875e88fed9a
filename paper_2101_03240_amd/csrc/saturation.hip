// Saturation map and per-step arrays of any step labelling (Sections 2.2.1,
// 2.2.2; Figure 5 left), and the squared radii that survive trapping
// (Section 2.2.3), so that the capillary pressure curve can be drawn with or
// without trapping.
#include <algorithm>
#include <cmath>

#include "ibip_internal.h"

namespace ibip {

namespace {

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// counts[k-1] = voxels labelled k; n_pore slots += pore voxels (label >= 0). Lanes
// of a wave are grouped by label with ballots, and each group adds its size
// with one atomic (labels of neighbouring voxels repeat).
// Per-step counts into copy blockIdx % ncopies (copy c at copies + c * K),
// each block summing its chunk of kCntChunk voxels in LDS first; the pore
// count into the slots; *bad set if a step exceeds K.
__global__ __launch_bounds__(256) void k_count_steps(const int32_t* __restrict__ seq, int64_t n, int64_t K,
                                                     uint32_t* copies, int ncopies, uint32_t* n_pore, uint32_t* bad) {
    __shared__ CountTable tab;
    count_table_clear(tab);
    __syncthreads();
    uint32_t* copy = copies + (int64_t)(blockIdx.x % (unsigned)ncopies) * K;
    const int64_t base = (int64_t)blockIdx.x * kCntChunk;
    uint32_t pore = 0;
    bool over = false;
    for (int j = 0; j < kCntChunk; j += 256) {
        const int64_t v = base + j + threadIdx.x;
        const int32_t s = v < n ? seq[v] : -1;
        over |= s > 0 && (int64_t)s > K;
        pore += s >= 0 ? 1u : 0u;
        count_table_add(tab, s > 0 && (int64_t)s <= K, s, copy);
    }
    if (over) atomicOr(bad, 1u);
    __syncthreads();
    count_table_flush(tab, copy);
    block_add_slots(n_pore, pore);
}

__global__ void k_curves(const uint32_t* counts, const uint32_t* excl, const uint32_t* M, int64_t K,
                         const uint32_t* n_pore, double c0, int64_t* n_new, double* sat, double* pc) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    const uint32_t c = counts[k];
    const double s = (double)(excl[k] + c) / (double)*n_pore;
    if (n_new) n_new[k] = c;
    if (sat) sat[k] = s;
    if (pc) pc[k] = c0 / sqrt((double)M[k]);
}

__global__ __launch_bounds__(256) void k_satmap(const int32_t* __restrict__ seq, int64_t n, const uint32_t* counts,
                                                const uint32_t* excl, const uint32_t* n_pore, double* satmap) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t s = seq[v];
    double m = s < 0 ? -1.0 : 0.0;
    if (s > 0) m = (double)(excl[s - 1] + counts[s - 1]) / (double)*n_pore;
    satmap[v] = m;
}

// M_after[seq_after[v]-1] = M[seq[v]-1]: every voxel of a re-ranked step
// carries the same original step, so the writes agree; a mismatch is flagged.
__global__ __launch_bounds__(256) void k_remap(const int32_t* __restrict__ seq, const int32_t* __restrict__ after,
                                               int64_t n, const uint32_t* M, int64_t K, int64_t K_after,
                                               uint32_t* M_after, uint32_t* bad) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t a = after[v];
    if (a <= 0) return;
    const int32_t s = seq[v];
    if ((int64_t)a > K_after || s <= 0 || (int64_t)s > K) {
        atomicOr(bad, 1u);
        return;
    }
    M_after[a - 1] = M[s - 1];
}

__global__ __launch_bounds__(256) void k_remap_check(const int32_t* __restrict__ seq,
                                                     const int32_t* __restrict__ after, int64_t n, const uint32_t* M,
                                                     int64_t K, const uint32_t* M_after, uint32_t* bad) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t a = after[v], s = seq[v];
    if (a > 0 && s > 0 && (int64_t)s <= K && M_after[a - 1] != M[s - 1]) atomicOr(bad, 1u);
}

// Equal-saturation comparison with the opening. Voxel v is in the IBIP
// configuration of level i when 0 < satmap[v] <= sat_T[i] (sat_T increasing),
// i.e. from level a = first i with sat_T[i] >= satmap[v] on, and in the
// opening's from level b = first i with mio_r2[v] >= T[i] (T decreasing) on.
// It disagrees on the levels between min(a, b) and max(a, b): +1 at the first,
// -1 at the second of a difference array over levels (n = no such level),
// whose prefix sum is the disagreement per level. A trapped voxel adds +1 at
// b to the second array (held by the opening from level b on).
constexpr int32_t kCmpLdsLevels = 2048;

__device__ __forceinline__ int32_t first_level_sat(const double* sat_T, int32_t nl, double m) {
    int32_t lo = 0, hi = nl;  // first level whose saturation reaches m
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (sat_T[mid] >= m) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

__device__ __forceinline__ int32_t first_level_r2(const uint32_t* T, int32_t nl, uint32_t r) {
    int32_t lo = 0, hi = nl;  // first level whose threshold r reaches
    while (lo < hi) {
        const int32_t mid = (lo + hi) >> 1;
        if (r >= T[mid]) hi = mid;
        else lo = mid + 1;
    }
    return lo;
}

// kLds: the difference arrays are binned per block in LDS (nl <= kCmpLdsLevels)
// and flushed with one global atomic per non-zero bin; else straight to HBM.
template <bool kLds>
__global__ __launch_bounds__(256) void k_compare_opening(const double* __restrict__ satmap,
                                                         const uint32_t* __restrict__ mio_r2,
                                                         const uint8_t* __restrict__ trapped, int64_t n,
                                                         const uint32_t* T, const double* sat_T, int32_t nl,
                                                         int32_t* diff, int32_t* tdiff) {
    __shared__ int32_t bins[kLds ? 2 * kCmpLdsLevels : 1];
    int32_t* ld = kLds ? bins : diff;
    int32_t* lt = kLds ? bins + kCmpLdsLevels : tdiff;
    if (kLds) {
        for (int32_t i = threadIdx.x; i < 2 * kCmpLdsLevels; i += 256) bins[i] = 0;
        __syncthreads();
    }
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x; v < n; v += stride) {
        const double m = satmap[v];
        const uint32_t r = mio_r2[v];
        const int32_t a = m > 0 ? first_level_sat(sat_T, nl, m) : nl;
        const int32_t b = r > 0 ? first_level_r2(T, nl, r) : nl;
        const int32_t x = min(a, b), y = max(a, b);
        if (x < y) {
            atomicAdd(&ld[x], 1);
            if (y < nl) atomicAdd(&ld[y], -1);
        }
        if (trapped && trapped[v] && b < nl) atomicAdd(&lt[b], 1);
    }
    if (kLds) {
        __syncthreads();
        for (int32_t i = threadIdx.x; i < nl; i += 256) {
            if (bins[i]) atomicAdd(&diff[i], bins[i]);
            if (bins[kCmpLdsLevels + i]) atomicAdd(&tdiff[i], bins[kCmpLdsLevels + i]);
        }
    }
}

__global__ void k_prefix_levels(const int32_t* diff, int32_t nl, int64_t* out) {
    // nl is small (the opening's levels): one thread
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        int64_t acc = 0;
        for (int32_t i = 0; i < nl; i++) {
            acc += diff[i];
            out[i] = acc;
        }
    }
}

}  // namespace

}  // namespace ibip

using namespace ibip;

extern "C" {

ibip_status ibip_saturation(ibip_ctx* ctx, const int32_t* seq, ibip_dims dims, const uint32_t* M, int64_t K,
                            const ibip_invade_opts* opts, int64_t* n_new, double* sat, double* pc,
                            double* satmap) {
    if (!ctx) return IBIP_EINVAL;
    if (!seq || !dims_ok(dims) || K < 0 || (K > 0 && pc && !M))
        return fail(ctx, IBIP_EINVAL, "saturation: bad arguments");
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    const int64_t n = nvox(dims);
    const double sigma = opts ? opts->sigma : 1.0, theta = opts ? opts->theta_rad : 0.0;
    const double vs = opts ? opts->voxel_size : 1.0;
    if (!(vs > 0)) return fail(ctx, IBIP_EINVAL, "saturation: voxel_size must be positive");
    const double c0 = 2.0 * sigma * cos(theta) / vs;
    const int S = count_copies(K, n);
    const size_t ncopy = S > 1 ? (size_t)S * (size_t)K : 0;
    uint32_t* w = (uint32_t*)ensure(ctx, B_SATW, sizeof(uint32_t) * (2 * (size_t)K + 64 + kCountSlots + ncopy));
    uint32_t* partials = (uint32_t*)ensure(ctx, B_SCAN, sizeof(uint32_t) * (K / 1000 + n / 1000 + 64));
    uint32_t* h = (uint32_t*)pinned(ctx, 4096);
    if (!w || !partials || !h) return fail(ctx, IBIP_ENOMEM, "saturation: allocation failed");
    uint32_t* ctl = w;                // [0] n_pore, [1] bad label, [2] scan total
    uint32_t* slots = w + 64;         // n_pore, by block
    uint32_t* counts = slots + kCountSlots;  // K
    uint32_t* excl = counts + K;      // K
    uint32_t* copies = S > 1 ? excl + K : counts;  // S * K
    ibip_status rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(w, 0, sizeof(uint32_t) * (64 + kCountSlots + (size_t)K), s), "memset")) !=
        IBIP_OK)
        return rc;
    if (S > 1 && (rc = hip_check(ctx, hipMemsetAsync(copies, 0, sizeof(uint32_t) * ncopy, s), "memset")) != IBIP_OK)
        return rc;
    hipLaunchKernelGGL(k_count_steps, dim3((unsigned)((n + kCntChunk - 1) / kCntChunk)), dim3(256), 0, s, seq, n, K,
                       copies, S, slots, ctl + 1);
    if ((rc = hip_check(ctx, launch_sum_slots(slots, ctl, s), "sum")) != IBIP_OK) return rc;
    if (S > 1 && (rc = hip_check(ctx, launch_sum_copies(copies, S, K, counts, s), "sum")) != IBIP_OK) return rc;
    if (K > 0) {
        if ((rc = hip_check(ctx, hipMemcpyAsync(excl, counts, sizeof(uint32_t) * K, hipMemcpyDeviceToDevice, s),
                            "copy")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, launch_scan_u32(excl, K, partials, ctl + 2, s), "scan")) != IBIP_OK) return rc;
        if (n_new || sat || pc)
            hipLaunchKernelGGL(k_curves, dim3(blocks(K)), dim3(256), 0, s, counts, excl, M, K, ctl, c0, n_new, sat,
                               pc);
    }
    if (satmap) hipLaunchKernelGGL(k_satmap, dim3(blocks(n)), dim3(256), 0, s, seq, n, counts, excl, ctl, satmap);
    if ((rc = hip_check(ctx, hipMemcpyAsync(h, ctl, sizeof(uint32_t) * 2, hipMemcpyDeviceToHost, s), "copy")) !=
        IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (h[1]) return fail(ctx, IBIP_EINVAL, "saturation: a label exceeds K");
    if (h[0] == 0 && K > 0) return fail(ctx, IBIP_EINVAL, "saturation: no pore voxel");
    return IBIP_OK;
}

ibip_status ibip_remap_steps(ibip_ctx* ctx, const int32_t* seq, const int32_t* seq_after, ibip_dims dims,
                             const uint32_t* M, int64_t K, int64_t K_after, uint32_t* M_after) {
    if (!ctx) return IBIP_EINVAL;
    if (!seq || !seq_after || !M_after || !dims_ok(dims) || K < 0 || K_after < 0 || (K > 0 && !M))
        return fail(ctx, IBIP_EINVAL, "remap_steps: bad arguments");
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    const int64_t n = nvox(dims);
    uint32_t* w = (uint32_t*)ensure(ctx, B_SATW, sizeof(uint32_t) * 64);
    uint32_t* h = (uint32_t*)pinned(ctx, 4096);
    if (!w || !h) return fail(ctx, IBIP_ENOMEM, "remap_steps: allocation failed");
    ibip_status rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(w, 0, sizeof(uint32_t) * 4, s), "memset")) != IBIP_OK) return rc;
    if (K_after > 0 &&
        (rc = hip_check(ctx, hipMemsetAsync(M_after, 0, sizeof(uint32_t) * K_after, s), "memset")) != IBIP_OK)
        return rc;
    hipLaunchKernelGGL(k_remap, dim3(blocks(n)), dim3(256), 0, s, seq, seq_after, n, M, K, K_after, M_after, w);
    hipLaunchKernelGGL(k_remap_check, dim3(blocks(n)), dim3(256), 0, s, seq, seq_after, n, M, K, M_after, w);
    if ((rc = hip_check(ctx, hipMemcpyAsync(h, w, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (h[0]) return fail(ctx, IBIP_EINVAL, "remap_steps: labels do not come from one trapping of this sequence");
    return IBIP_OK;
}

ibip_status ibip_compare_opening(ibip_ctx* ctx, const double* satmap, const uint32_t* mio_r2,
                                 const uint8_t* trapped, ibip_dims dims, const uint32_t* T, const double* sat_T,
                                 int32_t n_levels, int64_t* disagree, int64_t* mio_trapped) {
    if (!ctx) return IBIP_EINVAL;
    if (!satmap || !mio_r2 || !T || !sat_T || !disagree || !dims_ok(dims) || n_levels <= 0 ||
        n_levels > (1 << 20) || (trapped && !mio_trapped))
        return fail(ctx, IBIP_EINVAL, "compare_opening: bad arguments");
    if (T[n_levels - 1] < 1) return fail(ctx, IBIP_EINVAL, "compare_opening: radii must be >= 1");
    for (int32_t i = 1; i < n_levels; i++)
        if (T[i] >= T[i - 1] || sat_T[i] < sat_T[i - 1])
            return fail(ctx, IBIP_EINVAL, "compare_opening: T must decrease and sat_T must not");
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    const int64_t n = nvox(dims);
    const size_t nl = (size_t)n_levels;
    // device copies of the levels, and two difference arrays
    uint8_t* w = (uint8_t*)ensure(ctx, B_SATW, 256 + nl * (4 + 8 + 4 + 4) + 256);
    if (!w) return fail(ctx, IBIP_ENOMEM, "compare_opening: allocation failed");
    uint32_t* dT = (uint32_t*)w;
    double* dS = (double*)(w + align256(4 * nl));
    int32_t* diff = (int32_t*)((uint8_t*)dS + 8 * nl);
    int32_t* tdiff = diff + nl;
    ibip_status rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(dT, T, 4 * nl, hipMemcpyHostToDevice, s), "copy")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(dS, sat_T, 8 * nl, hipMemcpyHostToDevice, s), "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(diff, 0, 8 * nl, s), "memset")) != IBIP_OK) return rc;
    // enough blocks to fill the chip; each strides over the volume
    const int64_t nb = std::max<int64_t>(1, std::min<int64_t>(blocks(n), 2048));
    if (n_levels <= kCmpLdsLevels)
        hipLaunchKernelGGL(k_compare_opening<true>, dim3(nb), dim3(256), 0, s, satmap, mio_r2, trapped, n, dT, dS,
                           (int32_t)n_levels, diff, tdiff);
    else
        hipLaunchKernelGGL(k_compare_opening<false>, dim3(nb), dim3(256), 0, s, satmap, mio_r2, trapped, n, dT, dS,
                           (int32_t)n_levels, diff, tdiff);
    hipLaunchKernelGGL(k_prefix_levels, dim3(1), dim3(64), 0, s, diff, (int32_t)n_levels, disagree);
    if (trapped) hipLaunchKernelGGL(k_prefix_levels, dim3(1), dim3(64), 0, s, tdiff, (int32_t)n_levels, mio_trapped);
    if ((rc = hip_check(ctx, hipGetLastError(), "compare launch")) != IBIP_OK) return rc;
    return hip_check(ctx, hipStreamSynchronize(s), "sync");
}

}  // extern "C"
