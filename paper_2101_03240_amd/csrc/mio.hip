// Pressure-based drainage by morphological image opening (Section 2.4.1),
// used for the equal-saturation comparison of Section 3.1.1.
//
// For a squared radius T: eroding the pore space by B(., T) leaves the
// centres c with dt2[c] >= T (a ball around c is free of solid exactly when
// the nearest solid is at squared distance >= T); trimming keeps the eroded
// components that touch the inlet candidates Q0 (inlets and their face
// neighbours, pore only); dilating by B(., T) gives
//   D_T = {v : some kept c has |v - c|^2 < T}.
// The kept sets are nested in T, and c is kept at T exactly when
// K(c) >= T, where K(c) is the maximin of dt2 over paths from Q0 to c. So one
// maximin reconstruction gives every trim at once, and each dilation is a
// distance transform of {K >= T} thresholded at T.
#include "ibip_internal.h"

namespace ibip {

namespace {

// K0(v) = dt2(v) on Q0, 0 elsewhere; also counts pore voxels.
// Seeds of the opening: pore voxels in Q0 (an inlet voxel or a face
// neighbour of one); with mask, only pore inlet voxels count.
__global__ __launch_bounds__(256) void k_mio_seed(const uint8_t* img, const uint8_t* inlets, const uint32_t* dt2,
                                                  int X, int Y, int Z, FastDiv divZ, FastDiv divY, uint32_t* k0,
                                                  uint32_t* n_pore, bool mask) {
    const int64_t yz = (int64_t)Y * Z;
    const int64_t n = (int64_t)X * yz;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool pore = false;
    if (v < n) {
        // the seven positions are loaded together (an outside neighbour reads
        // v itself): a chain of conditional loads would wait for each in turn
        // coordinates by multiplicative division (indices fit 31 bits)
        const uint32_t t = fdiv((uint32_t)v, divZ), xx = fdiv(t, divY);
        const int z = (int)((uint32_t)v - t * (uint32_t)Z), y = (int)(t - xx * (uint32_t)Y), x = (int)xx;
        const int64_t nb[7] = {v, x > 0 ? v - yz : v, x < X - 1 ? v + yz : v, y > 0 ? v - Z : v,
                               y < Y - 1 ? v + Z : v, z > 0 ? v - 1 : v, z < Z - 1 ? v + 1 : v};
        const uint32_t d = dt2[v];
        uint8_t in[7], im[7];
#pragma unroll
        for (int j = 0; j < 7; j++) {
            in[j] = inlets[nb[j]];
            im[j] = img[nb[j]];
        }
        bool any = false;
#pragma unroll
        for (int j = 0; j < 7; j++) any |= in[j] != 0 && (!mask || im[j] != 0);
        pore = im[0] != 0;
        k0[v] = pore && any ? d : 0u;
    }
    block_add_slots(n_pore, pore ? 1u : 0u);
}

// First write in decreasing T; count voxels with mio_r2 >= T.
__global__ __launch_bounds__(256) void k_mio_update(const uint32_t* d2, uint32_t T, int64_t n, uint32_t* mio_r2,
                                                    uint32_t* count) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    bool hit = false;
    if (v < n) {
        uint32_t r = mio_r2[v];
        if (r == 0 && d2[v] < T) { r = T; mio_r2[v] = T; }
        hit = r >= T;
    }
    block_add_slots(count, hit ? 1u : 0u);
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

ibip_status run_mio(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims d, const uint32_t* T,
                    int32_t nT, uint32_t* mio_r2, double* mio_sat) {
    hipStream_t s = ctx->stream;
    const int64_t n = nvox(d);
    uint32_t* dt2 = (uint32_t*)ensure(ctx, B_KEY, sizeof(uint32_t) * n);
    uint32_t* kmap = (uint32_t*)ensure(ctx, B_STATE, sizeof(uint32_t) * n);
    uint16_t* g16 = (uint16_t*)ensure(ctx, B_TMP0, sizeof(uint16_t) * n);
    uint32_t* tmp32 = (uint32_t*)ensure(ctx, B_TMP1, sizeof(uint32_t) * n);
    uint32_t* d2 = (uint32_t*)ensure(ctx, B_TMP2, sizeof(uint32_t) * n);
    // per-level counts and the pore count, kCountSlots words each
    const size_t ncount = (size_t)kCountSlots * ((size_t)nT + 1);
    uint32_t* counts = (uint32_t*)ensure(ctx, B_MIOCNT, sizeof(uint32_t) * ncount);
    uint8_t* misc = (uint8_t*)ensure(ctx, B_MISC, 4096);
    uint32_t* h = (uint32_t*)pinned(ctx, 4096 + sizeof(uint32_t) * ncount);
    if (!dt2 || !kmap || !g16 || !tmp32 || !d2 || !counts || !misc || !h)
        return fail(ctx, IBIP_ENOMEM, "opening_drainage: allocation failed");
    uint32_t* flags = (uint32_t*)(misc + 3584);  // [0] solid seen, [2] scratch flag
    uint32_t* pore_slots = counts + (size_t)kCountSlots * nT;
    ibip_status rc;
    ctx->timer.mark(10, s);
    if ((rc = hip_check(ctx, hipMemsetAsync(flags, 0, 16, s), "memset")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(counts, 0, sizeof(uint32_t) * ncount, s), "memset")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(mio_r2, 0, sizeof(uint32_t) * n, s), "memset")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, launch_edt(image, nullptr, 0, 0, d, g16, tmp32, dt2, &flags[0], s, nullptr, nullptr,
                                        edt_tiles(ctx->tuning)), "edt")) != IBIP_OK)
        return rc;
    hipLaunchKernelGGL(k_mio_seed, dim3(blocks(n)), dim3(256), 0, s, image, inlets, dt2, d.X, d.Y, d.Z,
                       make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y), kmap, pore_slots, (ctx->readings & IBIP_READ_MASK_INLETS) != 0);
    if ((rc = hip_check(ctx, hipMemcpyAsync(h, flags, 4, hipMemcpyDeviceToHost, s), "copy")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(h + 64, pore_slots, sizeof(uint32_t) * kCountSlots,
                                            hipMemcpyDeviceToHost, s), "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (!h[0]) return fail(ctx, IBIP_ENOSOLID, "opening_drainage: image holds no solid voxel");
    uint64_t n_pore = 0;
    for (int q = 0; q < kCountSlots; q++) n_pore += h[64 + q];
    int iters = 0;
    if ((rc = reconstruct(ctx, nullptr, dt2, false, d, kmap, &iters)) != IBIP_OK) return rc;
    for (int32_t i = 0; i < nT; i++) {
        // distance to the kept centres, capped at T; the last pass writes T
        // into mio_r2 where it is still 0 and the distance is below T
        if ((rc = hip_check(ctx, launch_edt(nullptr, kmap, T[i], T[i], d, g16, tmp32, nullptr, &flags[2], s, mio_r2,
                                            counts + (size_t)kCountSlots * i, edt_tiles(ctx->tuning)),
                                 "edt")) != IBIP_OK)
            return rc;
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "mio launch")) != IBIP_OK) return rc;
    uint32_t* hc = h + 1024;
    if ((rc = hip_check(ctx, hipMemcpyAsync(hc, counts, sizeof(uint32_t) * kCountSlots * nT, hipMemcpyDeviceToHost,
                                            s), "copy")) != IBIP_OK)
        return rc;
    ctx->timer.mark(11, s);
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (ctx->timer.on) {
        ctx->timing.mio_ms += ctx->timer.ms(10, 11);
        ctx->timing.relax_sweeps += iters;
    }
    if (mio_sat)
        for (int32_t i = 0; i < nT; i++) {
            uint64_t c = 0;
            for (int q = 0; q < kCountSlots; q++) c += hc[(size_t)kCountSlots * i + q];
            mio_sat[i] = n_pore ? (double)c / (double)n_pore : 0.0;
        }
    return IBIP_OK;
}

}  // namespace ibip
