// Exact squared Euclidean distance transform (Section 2.1, Figure 2(b)).
//
// dt2(v) = min over feature voxels s of |v - s|^2, computed separably:
//   pass z: g(v)  = distance along z to the nearest feature voxel in the row
//                   (uint16, 0xFFFF = none), by a wave-wide max/min scan;
//   pass y: h(v)  = min over y' of g(x, y', z)^2 + (y - y')^2;
//   pass x: dt2(v)= min over x' of h(x', y, z) + (x - x')^2.
// The y and x passes evaluate the lower envelope of the parabolas
// f(i) + (u - i)^2 at u by an outward search from i = u that stops once
// o^2 >= best (every farther i adds at least o^2), which is exact; its cost is
// O(distance) per voxel, small in porous media.
// Threads of a wave own consecutive z, so every global access of the y and x
// passes is a contiguous 64-element segment.
#include "ibip_internal.h"

namespace ibip {

namespace {

constexpr uint16_t kInf16 = 0xFFFFu;

struct FeatImage {
    const uint8_t* img;
    __device__ bool operator()(int64_t v) const { return img[v] == 0; }
};
struct FeatThreshold {
    const uint32_t* w;
    uint32_t thr;
    __device__ bool operator()(int64_t v) const { return w[v] >= thr; }
};

// One wave per row along z. The row is walked in segments of 64 * kPer voxels;
// each lane owns kPer consecutive voxels of a segment.
constexpr int kPer = 8;
constexpr int kSeg = 64 * kPer;

template <class Feat>
__global__ __launch_bounds__(256) void edt_pass_z(Feat feat, int64_t rows, int Z, uint64_t cap, uint16_t* g,
                                                  uint32_t* solid_flag) {
    const int lane = threadIdx.x & 63;
    const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (row >= rows) return;
    const int64_t base = row * Z;
    bool any = false;
    // forward: distance to the nearest feature at or before z
    int carry = -1;  // last feature position before this segment, -1 = none
    for (int s0 = 0; s0 < Z; s0 += kSeg) {
        int z0 = s0 + lane * kPer;
        int last = -1;
        unsigned fbits = 0;
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            int z = z0 + j;
            if (z < Z && feat(base + z)) { fbits |= 1u << j; last = z; }
        }
        any |= fbits != 0;
        // inclusive max-scan of `last` over lanes
        int incl = last;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_up(incl, o, 64);
            if (lane >= o) incl = max(incl, t);
        }
        int prev = __shfl_up(incl, 1, 64);
        if (lane == 0) prev = -1;
        prev = max(prev, carry);
#pragma unroll
        for (int j = 0; j < kPer; j++) {
            int z = z0 + j;
            if (z >= Z) break;
            if (fbits & (1u << j)) prev = z;
            const uint64_t dz = (uint64_t)(z - prev);
            g[base + z] = (prev < 0 || dz * dz >= cap) ? kInf16 : (uint16_t)dz;
        }
        carry = max(carry, __shfl(incl, 63, 64));
    }
    // backward: distance to the nearest feature at or after z, min with forward
    int carryn = 0x7FFFFFFF;
    const int nseg = (Z + kSeg - 1) / kSeg;
    for (int si = nseg - 1; si >= 0; si--) {
        int s0 = si * kSeg;
        int z0 = s0 + lane * kPer;
        int first = 0x7FFFFFFF;
        unsigned fbits = 0;
#pragma unroll
        for (int j = kPer - 1; j >= 0; j--) {
            int z = z0 + j;
            if (z < Z && feat(base + z)) { fbits |= 1u << j; first = z; }
        }
        int incl = first;  // inclusive min-scan from the right
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            int t = __shfl_down(incl, o, 64);
            if (lane + o < 64) incl = min(incl, t);
        }
        int next = __shfl_down(incl, 1, 64);
        if (lane == 63) next = 0x7FFFFFFF;
        next = min(next, carryn);
#pragma unroll
        for (int j = kPer - 1; j >= 0; j--) {
            int z = z0 + j;
            if (z >= Z) continue;
            if (fbits & (1u << j)) next = z;
            if (next != 0x7FFFFFFF) {
                const uint32_t d = (uint32_t)(next - z);
                const uint16_t f = g[base + z];
                if (d < f && (uint64_t)d * d < cap) g[base + z] = (uint16_t)d;
            }
        }
        carryn = min(carryn, __shfl(incl, 0, 64));
    }
    // the flag only needs setting once: read before writing
    if (lane == 0 && any && __hip_atomic_load(solid_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(solid_flag, 1u);
}

// pass y: lines along y at fixed (x, z). One thread per voxel.
__global__ __launch_bounds__(256) void edt_pass_y(const uint16_t* __restrict__ g, int X, int Y, int Z, uint64_t cap,
                                                  uint32_t* __restrict__ h) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t n = (int64_t)X * Y * Z;
    if (v >= n) return;
    const int y = (int)((v / Z) % Y);
    uint64_t best;
    {
        uint16_t f = g[v];
        best = f == kInf16 ? cap : (uint64_t)f * f;
    }
    const int far = max(y, Y - 1 - y);
    for (int o = 1; o <= far; o++) {
        uint64_t oo = (uint64_t)o * o;
        if (oo >= best) break;
        if (y - o >= 0) {
            uint16_t f = g[v - (int64_t)o * Z];
            if (f != kInf16) { uint64_t c = (uint64_t)f * f + oo; best = c < best ? c : best; }
        }
        if (y + o < Y) {
            uint16_t f = g[v + (int64_t)o * Z];
            if (f != kInf16) { uint64_t c = (uint64_t)f * f + oo; best = c < best ? c : best; }
        }
    }
    h[v] = best >= cap ? kInf32 : (uint32_t)best;
}

// pass x: lines along x at fixed (y, z).
__global__ __launch_bounds__(256) void edt_pass_x(const uint32_t* __restrict__ h, int X, int Y, int Z, uint64_t cap,
                                                  uint32_t* __restrict__ out) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t yz = (int64_t)Y * Z;
    const int64_t n = (int64_t)X * yz;
    if (v >= n) return;
    const int x = (int)(v / yz);
    uint64_t best;
    {
        uint32_t f = h[v];
        best = f == kInf32 ? cap : (uint64_t)f;
    }
    const int far = max(x, X - 1 - x);
    for (int o = 1; o <= far; o++) {
        uint64_t oo = (uint64_t)o * o;
        if (oo >= best) break;
        if (x - o >= 0) {
            uint32_t f = h[v - (int64_t)o * yz];
            if (f != kInf32) { uint64_t c = (uint64_t)f + oo; best = c < best ? c : best; }
        }
        if (x + o < X) {
            uint32_t f = h[v + (int64_t)o * yz];
            if (f != kInf32) { uint64_t c = (uint64_t)f + oo; best = c < best ? c : best; }
        }
    }
    out[v] = best >= cap ? kInf32 : (uint32_t)best;
}

// LDS-tiled passes. A workgroup owns consecutive z columns of one plane:
// pass y loads the whole (Y x 64) tile of g, pass x the whole (X x 32) tile of
// h, in 128-byte row segments, and evaluates the envelope for every voxel
// of the tile by the same bounded outward search, reading LDS instead of
// global memory. Used when a whole line fits in LDS (L <= kMaxTileLine).
constexpr int kW = 64;             // pass y: 64 uint16 columns = 128 B row segments
constexpr int kWx = 32;            // pass x: 32 uint32 columns = 128 B row segments
constexpr int kMaxTileLine = 512;  // at most 64 KB of LDS per tile

__global__ __launch_bounds__(256) void edt_pass_y_tile(const uint16_t* __restrict__ g, int X, int Y, int Z,
                                                       uint64_t cap, uint32_t* __restrict__ h) {
    extern __shared__ uint16_t tile16[];  // [Y][kW]
    const int nzc = (Z + kW - 1) / kW;
    const int x = blockIdx.x / nzc;
    const int z0 = (blockIdx.x - x * nzc) * kW;
    const int lz = threadIdx.x & (kW - 1);
    const int r0 = threadIdx.x / kW;          // 0..3
    const int z = z0 + lz;
    const bool zin = z < Z;
    const int64_t plane = (int64_t)x * Y * Z;
    for (int y = r0; y < Y; y += 256 / kW) tile16[y * kW + lz] = zin ? g[plane + (int64_t)y * Z + z] : kInf16;
    __syncthreads();
    if (!zin) return;
    for (int y = r0; y < Y; y += 256 / kW) {
        const uint16_t f0 = tile16[y * kW + lz];
        uint64_t best = f0 == kInf16 ? cap : (uint64_t)f0 * f0;
        const int far = max(y, Y - 1 - y);
        for (int o = 1; o <= far; o++) {
            const uint64_t oo = (uint64_t)o * o;
            if (oo >= best) break;
            if (y - o >= 0) {
                const uint16_t f = tile16[(y - o) * kW + lz];
                if (f != kInf16) { const uint64_t c = (uint64_t)f * f + oo; best = c < best ? c : best; }
            }
            if (y + o < Y) {
                const uint16_t f = tile16[(y + o) * kW + lz];
                if (f != kInf16) { const uint64_t c = (uint64_t)f * f + oo; best = c < best ? c : best; }
            }
        }
        h[plane + (int64_t)y * Z + z] = best >= cap ? kInf32 : (uint32_t)best;
    }
}

// Epilogue of pass x: write dt2, or (opening) first-write T into mio_r2 where
// dt2 < T and count the voxels with mio_r2 >= T.
struct OutPlain {
    uint32_t* out;
    __device__ void put(int64_t v, uint64_t best, uint64_t cap) const {
        out[v] = best >= cap ? kInf32 : (uint32_t)best;
    }
    __device__ uint32_t hit(int64_t, uint64_t) const { return 0; }
};
struct OutOpening {
    uint32_t* mio_r2;
    uint32_t T;
    __device__ void put(int64_t, uint64_t, uint64_t) const {}
    __device__ uint32_t hit(int64_t v, uint64_t best) const {
        uint32_t r = mio_r2[v];
        if (r == 0 && best < T) {
            r = T;
            mio_r2[v] = T;
        }
        return r >= T ? 1u : 0u;
    }
};

template <class Out>
__global__ __launch_bounds__(256) void edt_pass_x_tile(const uint32_t* __restrict__ hin, int X, int Y, int Z,
                                                       uint64_t cap, Out outp, uint32_t* count) {
    extern __shared__ uint32_t tile32[];  // [X][kWx]
    const int nzc = (Z + kWx - 1) / kWx;
    const int y = blockIdx.x / nzc;
    const int z0 = (blockIdx.x - y * nzc) * kWx;
    const int lz = threadIdx.x & (kWx - 1);
    const int r0 = threadIdx.x / kWx;
    const int z = z0 + lz;
    const bool zin = z < Z;
    const int64_t yz = (int64_t)Y * Z;
    const int64_t col = (int64_t)y * Z + z;
    for (int x = r0; x < X; x += 256 / kWx) tile32[x * kWx + lz] = zin ? hin[x * yz + col] : kInf32;
    __syncthreads();
    uint32_t hits = 0;
    if (zin) {
        for (int x = r0; x < X; x += 256 / kWx) {
            const uint32_t f0 = tile32[x * kWx + lz];
            uint64_t best = f0 == kInf32 ? cap : (uint64_t)f0;
            const int far = max(x, X - 1 - x);
            for (int o = 1; o <= far; o++) {
                const uint64_t oo = (uint64_t)o * o;
                if (oo >= best) break;
                if (x - o >= 0) {
                    const uint32_t f = tile32[(x - o) * kWx + lz];
                    if (f != kInf32) { const uint64_t c = (uint64_t)f + oo; best = c < best ? c : best; }
                }
                if (x + o < X) {
                    const uint32_t f = tile32[(x + o) * kWx + lz];
                    if (f != kInf32) { const uint64_t c = (uint64_t)f + oo; best = c < best ? c : best; }
                }
            }
            outp.put(x * yz + col, best, cap);
            hits += outp.hit(x * yz + col, best);
        }
    }
    if (count) block_add_u32(count, hits);
}

// Non-tiled pass x with the opening epilogue (lines longer than the tile).
__global__ __launch_bounds__(256) void edt_pass_x_opening(const uint32_t* __restrict__ h, int X, int Y, int Z,
                                                          uint64_t cap, OutOpening outp, uint32_t* count) {
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const int64_t yz = (int64_t)Y * Z;
    const int64_t n = (int64_t)X * yz;
    uint32_t hits = 0;
    if (v < n) {
        const int x = (int)(v / yz);
        const uint32_t f0 = h[v];
        uint64_t best = f0 == kInf32 ? cap : (uint64_t)f0;
        const int far = max(x, X - 1 - x);
        for (int o = 1; o <= far; o++) {
            const uint64_t oo = (uint64_t)o * o;
            if (oo >= best) break;
            if (x - o >= 0) {
                const uint32_t f = h[v - (int64_t)o * yz];
                if (f != kInf32) { const uint64_t c = (uint64_t)f + oo; best = c < best ? c : best; }
            }
            if (x + o < X) {
                const uint32_t f = h[v + (int64_t)o * yz];
                if (f != kInf32) { const uint64_t c = (uint64_t)f + oo; best = c < best ? c : best; }
            }
        }
        hits = outp.hit(v, best);
    }
    block_add_u32(count, hits);
}

}  // namespace

hipError_t launch_edt(const uint8_t* image, const uint32_t* w, uint32_t thr, uint32_t cap, ibip_dims d,
                      uint16_t* g16, uint32_t* tmp32, uint32_t* out, uint32_t* solid_flag, hipStream_t s,
                      uint32_t* mio_r2, uint32_t* mio_count) {
    // cap == 0: exact everywhere; else exact where dt2 < cap, 0xFFFFFFFF elsewhere
    const uint64_t c64 = cap ? (uint64_t)cap : 0xFFFFFFFFull;
    const int64_t n = nvox(d);
    const int64_t rows = (int64_t)d.X * d.Y;
    const unsigned gz = (unsigned)((rows + 3) / 4);
    if (image)
        hipLaunchKernelGGL(edt_pass_z<FeatImage>, dim3(gz), dim3(256), 0, s, FeatImage{image}, rows, d.Z,
                           c64, g16, solid_flag);
    else
        hipLaunchKernelGGL(edt_pass_z<FeatThreshold>, dim3(gz), dim3(256), 0, s, FeatThreshold{w, thr},
                           rows, d.Z, c64, g16, solid_flag);
    const unsigned gv = (unsigned)((n + 255) / 256);
    const int nzc = (d.Z + kW - 1) / kW;
    const int nzcx = (d.Z + kWx - 1) / kWx;
    if (d.Y <= kMaxTileLine)
        hipLaunchKernelGGL(edt_pass_y_tile, dim3((unsigned)(d.X * nzc)), dim3(256), sizeof(uint16_t) * kW * d.Y, s,
                           g16, d.X, d.Y, d.Z, c64, tmp32);
    else
        hipLaunchKernelGGL(edt_pass_y, dim3(gv), dim3(256), 0, s, g16, d.X, d.Y, d.Z, c64, tmp32);
    const bool tile_x = d.X <= kMaxTileLine;
    if (mio_r2) {
        OutOpening o{mio_r2, cap};
        if (tile_x)
            hipLaunchKernelGGL(edt_pass_x_tile<OutOpening>, dim3((unsigned)(d.Y * nzcx)), dim3(256),
                               sizeof(uint32_t) * kWx * d.X, s, tmp32, d.X, d.Y, d.Z, c64, o, mio_count);
        else
            hipLaunchKernelGGL(edt_pass_x_opening, dim3(gv), dim3(256), 0, s, tmp32, d.X, d.Y, d.Z, c64, o,
                               mio_count);
    } else if (tile_x) {
        hipLaunchKernelGGL(edt_pass_x_tile<OutPlain>, dim3((unsigned)(d.Y * nzcx)), dim3(256),
                           sizeof(uint32_t) * kWx * d.X, s, tmp32, d.X, d.Y, d.Z, c64, OutPlain{out},
                           (uint32_t*)nullptr);
    } else {
        hipLaunchKernelGGL(edt_pass_x, dim3(gv), dim3(256), 0, s, tmp32, d.X, d.Y, d.Z, c64, out);
    }
    return hipGetLastError();
}

}  // namespace ibip
