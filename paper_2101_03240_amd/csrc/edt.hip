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
// passes is a contiguous segment. Pass y, and pass x on lines long enough
// that its 32-bit tile would leave a compute unit a single workgroup, run in
// packed 16-bit arithmetic with two columns per lane: exact for results
// below 65535, searched again exactly from HBM above. Pass z works in 16-bit
// halves too (its two distance chains in one packed word). Where pass x runs
// its 32-bit tiles, h travels between passes y and x as 16 bits per voxel,
// the exact values at 65535 and above kept aside in the output array.
#include <cmath>

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
    // r: the result, kInf32 at or above the cap
    __device__ uint32_t put_hit(int64_t v, uint32_t r) const {
        out[v] = r;
        return 0;
    }
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
    __device__ uint32_t put_hit(int64_t v, uint32_t r) const { return hit(v, r); }
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
    if (count) block_add_slots(count, hits);
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
    block_add_slots(count, hits);
}

// ---------------------------------------------------------------------------
// Vectorised passes (lines of at most 1024 voxels): pass z with each row in
// registers, loaded and stored with vectors when the rows are aligned;
// passes y and x from LDS tiles, loaded with 16-byte vectors when the rows
// allow it. Each row or tile is read once. Longer lines take the passes above.
// ---------------------------------------------------------------------------
struct FeatImage8 {
    const uint8_t* img;
    // feature bits of voxels v..v+7 (v % 8 == 0): bit j set iff voxel v+j is solid
    __device__ uint32_t bits8(int64_t v) const {
        const uint2 w = *reinterpret_cast<const uint2*>(img + v);
        uint32_t b = 0;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            b |= (((w.x >> (8 * j)) & 0xFFu) == 0u ? 1u : 0u) << j;
            b |= (((w.y >> (8 * j)) & 0xFFu) == 0u ? 1u : 0u) << (j + 4);
        }
        return b;
    }
    __device__ bool bit(int64_t v) const { return img[v] == 0; }
    // the bytes of voxels v..v+7 (v % 8 == 0)
    __device__ uint2 bytes8(int64_t v) const { return *reinterpret_cast<const uint2*>(img + v); }
    static constexpr bool kBytes = true;
};
struct FeatThreshold8 {
    const uint32_t* w;
    uint32_t thr;
    __device__ uint32_t bits8(int64_t v) const {
        const uint4 a = *reinterpret_cast<const uint4*>(w + v);
        const uint4 c = *reinterpret_cast<const uint4*>(w + v + 4);
        return (a.x >= thr ? 1u : 0u) | (a.y >= thr ? 2u : 0u) | (a.z >= thr ? 4u : 0u) | (a.w >= thr ? 8u : 0u) |
               (c.x >= thr ? 16u : 0u) | (c.y >= thr ? 32u : 0u) | (c.z >= thr ? 64u : 0u) |
               (c.w >= thr ? 128u : 0u);
    }
    __device__ bool bit(int64_t v) const { return w[v] >= thr; }
    __device__ uint2 bytes8(int64_t) const { return make_uint2(0u, 0u); }
    static constexpr bool kBytes = false;
};

// Pass z with the whole row in registers: a lane owns P = 8 (rows of at most
// 512 voxels) or 16 (at most 1024) consecutive voxels, a row spans lpr = Z / P
// lanes, a wave holds 64 / lpr rows. The nearest feature before / after each
// lane's voxels comes from a max / min scan over the row's lanes (DPP moves
// when the row fills the wave, lane shuffles otherwise); within the lane, the
// distances to them run as two packed 16-bit chains. Everything a voxel needs
// is 16-bit (distances below 1024, 65535 for none), so no 32- or 64-bit
// product is formed: the cap d^2 >= cap becomes d >= dcap, the least such d.
constexpr int kZGroups = 4;  // row groups per wave, their loads issued together
constexpr int kMaxVecLine = 1024;  // longest row or line of the vectorised passes

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ inline u16x2 as_u16x2(uint32_t v) { return __builtin_bit_cast(u16x2, v); }
__device__ inline uint32_t as_u32(u16x2 v) { return __builtin_bit_cast(uint32_t, v); }

// DPP moves within the wave: a lane without a source keeps `idle`
template <int kCtrl, int kRowMask = 0xf>
__device__ inline int dpp_or(int idle, int v) {
    return __builtin_amdgcn_update_dpp(idle, v, kCtrl, kRowMask, 0xf, false);
}

// Over a wave holding one row (64 lanes): the maximum of v over the lanes at
// or below this one (row shifts within rows of 16, then the last lane of a
// row broadcast to the rows above), and the minimum of w over the lanes at or
// above this one (row shifts the other way, then the first lanes of the rows
// above, read as scalars). A lane without a source takes the operation's
// identity, so each move folds into the max or min that takes it.
__device__ inline void wave_scans(int& v, int& w) {
    constexpr int kLo = INT_MIN, kHi = INT_MAX;
    v = max(v, dpp_or<0x111>(kLo, v));  // row_shr:1
    w = min(w, dpp_or<0x101>(kHi, w));  // row_shl:1
    v = max(v, dpp_or<0x112>(kLo, v));
    w = min(w, dpp_or<0x102>(kHi, w));
    v = max(v, dpp_or<0x114>(kLo, v));
    w = min(w, dpp_or<0x104>(kHi, w));
    v = max(v, dpp_or<0x118>(kLo, v));
    w = min(w, dpp_or<0x108>(kHi, w));
    v = max(v, dpp_or<0x142, 0xa>(kLo, v));  // row_bcast:15 into rows 1 and 3
    v = max(v, dpp_or<0x143, 0xc>(kLo, v));  // row_bcast:31 into rows 2 and 3
    const int m3 = __builtin_amdgcn_readlane(w, 48), m2 = min(__builtin_amdgcn_readlane(w, 32), m3),
              m1 = min(__builtin_amdgcn_readlane(w, 16), m2);
    const int lane = threadIdx.x & 63;
    int t = lane < 48 ? m3 : kHi;
    t = lane < 32 ? m2 : t;
    t = lane < 16 ? m1 : t;
    w = min(w, t);
}

// The chains' step factors from the lane's P image bytes (nonzero: not a
// feature), without going through single bits: tj[j] holds 1 in its low half
// where voxel j is not a feature and 1 in its high half where voxel P-1-j is
// not, 0 elsewhere; fb gets the feature bits.
template <int P>
__device__ inline void byte_factors(const uint32_t (&raw)[P / 4], uint32_t (&tj)[P], uint32_t& fb) {
    // nz[2q + e]: voxels 4q + e and 4q + e + 2 (the bytes e and e + 2 of raw[q])
    uint32_t nz[P / 2];
#pragma unroll
    for (int q = 0; q < P / 4; q++) {
        // bit 7 of each byte of y: that byte is nonzero (no carry crosses a byte)
        const uint32_t y = ((raw[q] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | raw[q];
        nz[2 * q] = y >> 7 & 0x00010001u;
        nz[2 * q + 1] = y >> 15 & 0x00010001u;
    }
#pragma unroll
    for (int j = 0; j < P; j++) {
        const int k = P - 1 - j;
        // byte 0 or 2 of voxel j's word into byte 0, of voxel k's word into byte 2
        const uint32_t sel = (uint32_t)(2 * ((j >> 1) & 1)) | 0x0C00u | (uint32_t)(4 + 2 * ((k >> 1) & 1)) << 16 |
                             0x0C000000u;
        tj[j] = __builtin_amdgcn_perm(nz[2 * (k >> 2) + (k & 1)], nz[2 * (j >> 2) + (j & 1)], sel);
    }
    // voxels 4q, 4q+1 to bits 4q, 4q+1 and voxels 4q+2, 4q+3 to bits 4q+16,
    // 4q+17, folded down by 14
    uint32_t c = 0;
#pragma unroll
    for (int q = 0; q < P / 4; q++) c |= (nz[2 * q] | nz[2 * q + 1] << 1) << (4 * q);
    fb = ~(c | c >> 14) & ((1u << P) - 1u);
}

// pass z of one row group: lane li of lpr holds feature bits fb of voxels
// v0..v0+P-1 of its row (the first nv of them inside the row); writes their
// distances along z, kInf16 for a distance of dcap or more (capped when
// dcap < Z), with 16-byte stores when the rows are aligned (Al). The distances
// to the nearest feature before and after each voxel run as two chains in
// the halves of one packed 16-bit word: the first forward from the lane's
// first voxel, the second backward from its last, each step adding one
// (saturating at 65535 where no feature lies on that side) and resetting to
// zero at a feature.
template <int P, bool Al, bool Bytes>
__device__ inline uint32_t pass_z_rows(uint32_t fb, const uint32_t (&raw)[P / 4], bool act, int64_t v0, int li,
                                       int lpr, int nv, uint32_t dcap, int Z, uint16_t* g) {
    constexpr int kNone = 0x10000;  // a feature position that no row reaches
    const int zb = li * P;
    uint32_t tj[P];
    if (Bytes) {
        byte_factors<P>(raw, tj, fb);
    } else {
        // step j's factors from the feature bits: bit j of the not-feature
        // bits in the low half, bit P-1-j in the high one
        const uint32_t nf = ~fb & ((1u << P) - 1u);
        const uint32_t nfr = nf | (__builtin_bitreverse32(nf) >> (16 - P));
#pragma unroll
        for (int j = 0; j < P; j++) tj[j] = (nfr >> j) & 0x00010001u;
    }
    // nearest feature at or before the end of this lane's voxels
    int incl = fb ? zb + 31 - __clz(fb) : -kNone;
    // nearest feature at or after the start of this lane's voxels
    int incr = fb ? zb + __ffs(fb) - 1 : 2 * kNone;
    int prev, next;
    if (lpr == 64) {
        // one row per wave: scans and the one-lane shifts by DPP
        wave_scans(incl, incr);
        prev = dpp_or<0x138>(-kNone, incl);     // wave_shr:1
        next = dpp_or<0x130>(2 * kNone, incr);  // wave_shl:1
    } else {
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int a = __shfl_up(incl, o, 64);
            const int b = __shfl_down(incr, o, 64);
            if (o < lpr) {
                if (li >= o) incl = max(incl, a);
                if (li + o < lpr) incr = min(incr, b);
            }
        }
        prev = __shfl_up(incl, 1, 64);
        next = __shfl_down(incr, 1, 64);
    }
    if (li == 0) prev = -kNone;
    if (li == lpr - 1) next = 2 * kNone;
    // the chains' values one voxel before this lane's first and one after its last
    const uint32_t l0 = (uint32_t)min(zb - 1 - prev, 0xFFFF), r0 = (uint32_t)min(next - zb - P, 0xFFFF);
    u16x2 st = as_u16x2(l0 | r0 << 16);
    u16x2 ch[P];
#pragma unroll
    for (int j = 0; j < P; j++) {
        st = __builtin_elementwise_add_sat(st, as_u16x2(0x00010001u)) * as_u16x2(tj[j]);
        ch[j] = st;
    }
    // ch[j] holds (before-distance of voxel j, after-distance of voxel P-1-j):
    // the minimum with ch[P-1-j] swapped gives (d_j, d_{P-1-j})
    uint32_t dp[P / 2];
#pragma unroll
    for (int j = 0; j < P / 2; j++) {
        const uint32_t o = as_u32(ch[P - 1 - j]);
        dp[j] = as_u32(__builtin_elementwise_min(ch[j], as_u16x2(o >> 16 | o << 16)));
    }
    uint32_t pk[P / 2];
#pragma unroll
    for (int i = 0; i < P / 4; i++) {
        pk[i] = (dp[2 * i] & 0xFFFFu) | dp[2 * i + 1] << 16;
        pk[P / 4 + i] = dp[P / 2 - 1 - 2 * i] >> 16 | (dp[P / 2 - 2 - 2 * i] & 0xFFFF0000u);
    }
    if (dcap < (uint32_t)Z) {
        // kInf16 where d >= dcap: (dcap - d) saturates to 0 there
        const u16x2 dc = as_u16x2(dcap | dcap << 16);
#pragma unroll
        for (int i = 0; i < P / 2; i++) {
            const u16x2 keep = __builtin_elementwise_sub_sat(dc, as_u16x2(pk[i]));
            const u16x2 over = __builtin_elementwise_sub_sat(as_u16x2(0x00010001u), keep);
            pk[i] |= as_u32(over * as_u16x2(0xFFFFFFFFu));
        }
    }
    if (act && Al) {
#pragma unroll
        for (int j = 0; j < P / 8; j++)
            *reinterpret_cast<uint4*>(g + v0 + 8 * j) =
                make_uint4(pk[4 * j], pk[4 * j + 1], pk[4 * j + 2], pk[4 * j + 3]);
    } else if (act) {
#pragma unroll
        for (int j = 0; j < P; j++)
            if (j < nv) g[v0 + j] = (uint16_t)(pk[j >> 1] >> (16 * (j & 1)));
    }
    return fb;
}

// Al: rows of a multiple of P voxels from an aligned input, loaded and
// stored with vectors; otherwise (rows of any length up to 64 * P) voxel by
// voxel, the last lane of a row holding fewer than P.
template <class Feat, int P, bool Al>
__global__ __launch_bounds__(256) void edt_pass_z_vec(Feat feat, int64_t rows, int Z, uint32_t dcap, uint16_t* g,
                                                      uint32_t* solid_flag) {
    const int lane = threadIdx.x & 63;
    const int lpr = (Z + P - 1) / P;
    const int rpw = 64 / lpr;
    const int r = lane / lpr;
    const int li = lane - r * lpr;
    const int64_t wave = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    // voxels of this lane inside its row (a lane of the partial row group
    // past the last whole row computes a phantom row and stores nothing)
    const int nv = min(P, Z - li * P);
    // the image's bytes go to the chains directly; other inputs through bits
    constexpr bool Bytes = Al && Feat::kBytes;
    uint32_t fb[kZGroups];
    uint32_t raw[kZGroups][P / 4];
    bool act[kZGroups];
    int64_t v0[kZGroups];
#pragma unroll
    for (int q = 0; q < kZGroups; q++) {
        const int64_t row = (wave * kZGroups + q) * rpw + r;
        act[q] = r < rpw && row < rows;
        // unconditional loads (a lane past the last row reads row 0, a voxel
        // past its row's end rereads the row's last voxel): a load under a
        // lane condition would be waited for before the next one
        v0[q] = (act[q] ? row : 0) * Z + li * P;
        uint32_t b = 0;
        if (Bytes) {
#pragma unroll
            for (int k = 0; k < P / 8; k++) {
                const uint2 x = feat.bytes8(v0[q] + 8 * k);
                raw[q][2 * k] = x.x;
                raw[q][2 * k + 1] = x.y;
            }
        } else if (Al) {
            b = feat.bits8(v0[q]);
            if (P == 16) b |= feat.bits8(v0[q] + 8) << 8;
        } else {
#pragma unroll
            for (int j = 0; j < P; j++) b |= (feat.bit(v0[q] + min(j, nv - 1)) && j < nv ? 1u : 0u) << j;
        }
        fb[q] = b;
    }
    bool any = false;
#pragma unroll
    for (int q = 0; q < kZGroups; q++) {
        const uint32_t f = pass_z_rows<P, Al, Bytes>(fb[q], raw[q], act[q], v0[q], li, lpr, nv, dcap, Z, g);
        any |= __ballot(act[q] && f != 0) != 0;
    }
    if (lane == 0 && any && __hip_atomic_load(solid_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        atomicOr(solid_flag, 1u);
}

// Tiled passes y and x: a workgroup loads a whole tile of lines (every line
// of one plane, 32 z columns wide) into LDS with 16-byte vectors, then
// evaluates the envelope min over i of f(i) + (u - i)^2 at every voxel by the
// outward search, four offsets per side at a time, stopping once o^2 >= best
// (every farther i adds at least o^2; reading a whole group before the test
// only adds candidates, so the result is exact). The tile carries kPad rows
// of a sentinel above and below the line, and a side that has run past its
// end reads the sentinel rows, so a group is eight unconditional LDS reads at
// fixed offsets. Each side keeps a pointer to its group's lowest row, moved
// by four rows and held at the pad rows in one add and one unsigned min/max;
// with 8 pad rows the held pointer lies at least one move above LDS address
// 0, so the move never wraps. The sentinel stands for "no feature": it is larger than any
// real value and small enough that sentinel + o^2 cannot overflow. The two
// sides at one offset share o^2, so a candidate pair costs a min of the two
// tile values, one add and one min. Lines are at most 1024 voxels, so every
// real sum stays below 3 * 1023^2.
//
// Between the passes, h (pass y's result) is either one 32-bit word per voxel
// (HPlain) or, where pass x runs its 32-bit tiles and a 32-bit output array is
// there, split (HSplit): min(h, 65535) as 16 bits per voxel, and the exact h
// of the voxels at 65535 or above (no feature in the plane included) in the
// output array at the voxel's own index. Pass x reads those while loading its
// tile, before any of its workgroups writes the output of its columns, which
// are the only voxels whose exact h it reads. 2 bytes per voxel are written
// and read instead of 4 (plus 4 per voxel at a 2D distance of 256 or more).
constexpr int kPad = 8;
constexpr uint32_t kSent16 = 0x7FFFu;                // pass y: sentinel distance
constexpr uint32_t kSentSq = kSent16 * kSent16;      // its square (+ o^2 < 2^31)
constexpr uint32_t kSent32 = 0x40000000u;            // pass x: sentinel value
constexpr int kThreadsY = 512, kThreadsX = 1024;

// Pass y in packed 16-bit arithmetic, two columns per lane. The tile holds
// min(g^2, 65535) (g < 256 squares exactly; a larger g and the sentinel
// become 65535), so one 32-bit LDS read gives a lane both of its columns and
// each candidate costs one saturating packed add (v_pk_add_u16 with clamp)
// and one packed min for two voxels. A result below 65535 is exact: the
// minimum's candidate is then below 65535 itself, and every candidate that
// saturated is at least 65535. A result of 65535 where the cap allows more is
// searched again exactly, from the distances in HBM (a 2D distance of 256
// voxels or more; none on the workloads here). The search of a pair of
// columns goes on until both are settled, and at most to offset 256 (every
// candidate farther out is at least 65536). The packed type and its casts
// are the ones of pass z.

// pass y's result h: one 32-bit word per voxel
struct HPlain {
    static constexpr bool kSplit = false;
    uint32_t* h;
    __device__ void put(int64_t v, uint32_t val) const { h[v] = val; }
    // voxels v and v+1 (v even: one 32-bit store in the split form)
    __device__ void put2(int64_t v, uint32_t a, uint32_t b) const {
        h[v] = a;
        h[v + 1] = b;
    }
    __device__ uint32_t get(int64_t v) const { return h[v]; }
    __device__ uint4 get4(int64_t v) const { return *reinterpret_cast<const uint4*>(h + v); }
};

// pass y's result h split: min(h, 65535) in h16, the exact h of the voxels at
// 65535 or above in hx
struct HSplit {
    static constexpr bool kSplit = true;
    uint16_t* h16;
    uint32_t* hx;
    __device__ void put(int64_t v, uint32_t val) const {
        h16[v] = (uint16_t)min(val, 65535u);
        if (val >= 65535u) hx[v] = val;
    }
    __device__ void put2(int64_t v, uint32_t a, uint32_t b) const {
        *reinterpret_cast<uint32_t*>(h16 + v) = min(a, 65535u) | min(b, 65535u) << 16;
        if (a >= 65535u) hx[v] = a;
        if (b >= 65535u) hx[v + 1] = b;
    }
    __device__ uint32_t get(int64_t v) const {
        const uint32_t u = h16[v];
        return u < 65535u ? u : hx[v];
    }
    // voxels v..v+3 (v % 4 == 0)
    __device__ uint4 get4(int64_t v) const {
        const uint2 r = *reinterpret_cast<const uint2*>(h16 + v);
        uint4 w = make_uint4(r.x & 0xFFFFu, r.x >> 16, r.y & 0xFFFFu, r.y >> 16);
        if (w.x == 65535u) w.x = hx[v];
        if (w.y == 65535u) w.y = hx[v + 1];
        if (w.z == 65535u) w.z = hx[v + 2];
        if (w.w == 65535u) w.w = hx[v + 3];
        return w;
    }
};

// min(g^2, 65535) of a distance along z (0x7FFF = no feature)
__device__ inline uint32_t sq16(uint32_t gv) { return gv < 256u ? gv * gv : 65535u; }

// the exact search of pass y for one voxel, reading the distances in HBM
__device__ inline uint32_t pass_y_exact(const uint16_t* g, int64_t v, int y, int Y, int Z, uint64_t cap) {
    const uint16_t f = g[v];
    uint64_t best = f == kInf16 ? cap : (uint64_t)f * f;
    const int far = max(y, Y - 1 - y);
    for (int o = 1; o <= far; o++) {
        const uint64_t oo = (uint64_t)o * o;
        if (oo >= best) break;
        if (y - o >= 0) {
            const uint16_t fl = g[v - (int64_t)o * Z];
            if (fl != kInf16) best = min(best, (uint64_t)fl * fl + oo);
        }
        if (y + o < Y) {
            const uint16_t fr = g[v + (int64_t)o * Z];
            if (fr != kInf16) best = min(best, (uint64_t)fr * fr + oo);
        }
    }
    return (uint32_t)min(best, (uint64_t)0xFFFFFFFFu);
}

template <int TW, bool V, class H>
__global__ __launch_bounds__(kThreadsY) void edt_pass_y_pk(const uint16_t* __restrict__ g, int X, int Y, int Z,
                                                          uint64_t cap, H h) {
    extern __shared__ uint16_t t16[];  // [kPad + Y + kPad][TW]: min(g^2, 65535)
    constexpr int kSegs = TW / 8, kRows = kThreadsY / kSegs;
    const int nzc = (Z + TW - 1) / TW;
    const int x = blockIdx.x / nzc;
    const int z0 = (blockIdx.x - x * nzc) * TW;
    const int64_t plane = (int64_t)x * Y * Z;
    if (!V) {
        for (int i = threadIdx.x; i < Y * TW; i += kThreadsY) {
            const int y = i / TW, lz = i - y * TW, zc = z0 + lz;
            t16[(y + kPad) * TW + lz] =
                (uint16_t)(zc < Z ? sq16(g[plane + (int64_t)y * Z + zc] & 0x7FFFu) : 65535u);
        }
    } else {
        const int seg = threadIdx.x % kSegs;
        const int zc = z0 + seg * 8;
        for (int y = threadIdx.x / kSegs; y < Y; y += kRows) {
            uint4 w = make_uint4(0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu, 0xFFFFFFFFu);
            if (zc < Z) {
                const uint4 r = *reinterpret_cast<const uint4*>(g + plane + (int64_t)y * Z + zc);
                w.x = sq16(r.x & 0x7FFFu) | sq16((r.x >> 16) & 0x7FFFu) << 16;
                w.y = sq16(r.y & 0x7FFFu) | sq16((r.y >> 16) & 0x7FFFu) << 16;
                w.z = sq16(r.z & 0x7FFFu) | sq16((r.z >> 16) & 0x7FFFu) << 16;
                w.w = sq16(r.w & 0x7FFFu) | sq16((r.w >> 16) & 0x7FFFu) << 16;
            }
            *reinterpret_cast<uint4*>(t16 + (y + kPad) * TW + seg * 8) = w;
        }
    }
    for (int i = threadIdx.x; i < 2 * kPad * TW; i += kThreadsY) {
        const int r = i / TW;
        t16[(r < kPad ? r : Y + r) * TW + (i - r * TW)] = (uint16_t)65535u;
    }
    __syncthreads();
    constexpr int LC = TW / 2;             // lanes per tile row
    constexpr int RPI = kThreadsY / LC;    // rows per round
    const int lc = threadIdx.x % LC;
    const int z = z0 + 2 * lc;
    if (z >= Z) return;
    const uint32_t capv = (uint32_t)cap;
    const uint32_t lim = min(capv, kSentSq);
    const uint32_t c16 = min(capv, 65535u);
    const u16x2 capp = as_u16x2(c16 | c16 << 16);
    const uint32_t* col = reinterpret_cast<const uint32_t*>(t16 + kPad * TW) + lc;  // row i at col[i * LC]
    // the voxel's index runs with y (no 64-bit product per voxel)
    int64_t v = plane + (int64_t)(threadIdx.x / LC) * Z + z;
    for (int y = threadIdx.x / LC; y < Y; y += RPI, v += (int64_t)RPI * Z) {
        u16x2 best = __builtin_elementwise_min(as_u16x2(col[y * LC]), capp);
        uint32_t bb = as_u32(best);
        uint32_t bmax = max(bb & 0xFFFFu, bb >> 16);
        if (bmax > 1) {
            const int far = min(max(y, Y - 1 - y), 256);
            // rows y - o - 3 (the lowest of the group on the left, so that
            // every read has a positive offset) and y + o, each stepped and
            // held at the pad rows in one move, so neither leaves the tile
            const uint32_t* const ltop = col - 4 * LC;
            const uint32_t* const rbot = col + Y * LC;
            const uint32_t* lp = col + (y - 4) * LC;
            const uint32_t* rp = col + (y + 1) * LC;
            for (int o = 1; o <= far && (uint32_t)(o * o) < bmax;
                 o += 4, lp = lp - 4 * LC < ltop ? ltop : lp - 4 * LC, rp = rp + 4 * LC > rbot ? rbot : rp + 4 * LC) {
#pragma unroll
                for (int j = 0; j < 4; j++) {
                    const uint32_t oo = min((uint32_t)((o + j) * (o + j)), 65535u);
                    const u16x2 oop = as_u16x2(oo | oo << 16);
                    best = __builtin_elementwise_min(
                        best, __builtin_elementwise_add_sat(
                                  __builtin_elementwise_min(as_u16x2(lp[(3 - j) * LC]), as_u16x2(rp[j * LC])), oop));
                }
                bb = as_u32(best);
                bmax = max(bb & 0xFFFFu, bb >> 16);
            }
        }
        bb = as_u32(best);
        uint32_t r0 = bb & 0xFFFFu, r1 = bb >> 16;
        if (r0 == 65535u && capv > 65535u) r0 = pass_y_exact(g, v, y, Y, Z, cap);
        r0 = r0 >= lim ? kInf32 : r0;
        if (z + 1 < Z) {
            if (r1 == 65535u && capv > 65535u) r1 = pass_y_exact(g, v + 1, y, Y, Z, cap);
            r1 = r1 >= lim ? kInf32 : r1;
            if (V) h.put2(v, r0, r1);
            else {
                h.put(v, r0);
                h.put(v + 1, r1);
            }
        } else {
            h.put(v, r0);
        }
    }
}

// TW: z columns per tile (16: 64-byte tile rows; 32: whole 128-byte lines).
// V: rows of Z % 4 == 0 voxels, loaded with 16-byte vectors; otherwise the
// tile is loaded element by element.
template <class Out, int TW, bool V, class H>
__global__ __launch_bounds__(kThreadsX) void edt_pass_x_vec(H hin, int X, int Y, int Z, uint64_t cap, Out outp,
                                                           uint32_t* count) {
    extern __shared__ uint32_t t32[];  // [kPad + X + kPad][TW]
    constexpr int kSegs = TW / 4, kRows = kThreadsX / kSegs;
    const int nzc = (Z + TW - 1) / TW;
    const int y = blockIdx.x / nzc;
    const int z0 = (blockIdx.x - y * nzc) * TW;
    const int64_t yz = (int64_t)Y * Z;
    const int64_t col0 = (int64_t)y * Z + z0;
    if (!V) {
        for (int i = threadIdx.x; i < X * TW; i += kThreadsX) {
            const int x = i / TW, lz = i - x * TW;
            uint32_t w = kSent32;
            if (z0 + lz < Z) {
                w = hin.get(x * yz + col0 + lz);
                w = w == kInf32 ? kSent32 : w;
            }
            t32[(x + kPad) * TW + lz] = w;
        }
    } else {
        const int seg = threadIdx.x % kSegs;
        const int zc = z0 + seg * 4;
        for (int x = threadIdx.x / kSegs; x < X; x += kRows) {
            uint4 w = make_uint4(kSent32, kSent32, kSent32, kSent32);
            if (zc < Z) {
                w = hin.get4(x * yz + col0 + seg * 4);
                w.x = w.x == kInf32 ? kSent32 : w.x;
                w.y = w.y == kInf32 ? kSent32 : w.y;
                w.z = w.z == kInf32 ? kSent32 : w.z;
                w.w = w.w == kInf32 ? kSent32 : w.w;
            }
            *reinterpret_cast<uint4*>(t32 + (x + kPad) * TW + seg * 4) = w;
        }
    }
    for (int i = threadIdx.x; i < 2 * kPad * TW; i += kThreadsX) {
        const int r = i / TW;
        t32[(r < kPad ? r : X + r) * TW + (i - r * TW)] = kSent32;
    }
    __syncthreads();
    const int lz = threadIdx.x % TW;
    const int z = z0 + lz;
    uint32_t hits = 0;
    if (z < Z) {
        const uint32_t capv = (uint32_t)cap;
        const uint32_t lim = min(capv, kSent32);
        const uint32_t* col = t32 + kPad * TW + lz;
        // the voxel's index runs with x (no 64-bit product per voxel)
        int64_t v = (int64_t)(threadIdx.x / TW) * yz + col0 + lz;
        const int64_t dv = (int64_t)(kThreadsX / TW) * yz;
        for (int x = threadIdx.x / TW; x < X; x += kThreadsX / TW, v += dv) {
            const uint32_t f0 = col[x * TW];
            uint32_t best = f0 == kSent32 ? capv : f0;
            if (best) {
                const int far = max(x, X - 1 - x);
                // rows x - o - 3 (the lowest of the group on the left, so that
                // every read has a positive offset) and x + o, each stepped and
                // held at the pad rows in one move, so neither leaves the tile
                const uint32_t* const ltop = col - 4 * TW;
                const uint32_t* const rbot = col + X * TW;
                const uint32_t* lp = col + (x - 4) * TW;
                const uint32_t* rp = col + (x + 1) * TW;
                for (int o = 1; o <= far;
                     o += 4, lp = lp - 4 * TW < ltop ? ltop : lp - 4 * TW, rp = rp + 4 * TW > rbot ? rbot : rp + 4 * TW) {
                    if ((uint32_t)(o * o) >= best) break;
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const uint32_t oo = (uint32_t)((o + j) * (o + j));
                        best = min(best, min(lp[(3 - j) * TW], rp[j * TW]) + oo);
                    }
                }
            }
            hits += outp.put_hit(v, best >= lim ? kInf32 : best);
        }
    }
    if (count) block_add_slots(count, hits);
}

// Pass x in packed 16-bit arithmetic, as pass y above: the tile holds
// min(h, 65535) (h = 0xFFFFFFFF, no feature in the plane, becomes 65535),
// two columns per lane; a result of 65535 where the cap allows more is
// searched again exactly from h in HBM.
__device__ inline uint32_t pass_x_exact(const uint32_t* hin, int64_t v, int x, int X, int64_t yz, uint64_t cap) {
    const uint32_t f = hin[v];
    uint64_t best = f == kInf32 ? cap : (uint64_t)f;
    const int far = max(x, X - 1 - x);
    for (int o = 1; o <= far; o++) {
        const uint64_t oo = (uint64_t)o * o;
        if (oo >= best) break;
        if (x - o >= 0) {
            const uint32_t fl = hin[v - (int64_t)o * yz];
            if (fl != kInf32) best = min(best, (uint64_t)fl + oo);
        }
        if (x + o < X) {
            const uint32_t fr = hin[v + (int64_t)o * yz];
            if (fr != kInf32) best = min(best, (uint64_t)fr + oo);
        }
    }
    return (uint32_t)min(best, (uint64_t)0xFFFFFFFFu);
}

template <class Out, int TW, bool V>
__global__ __launch_bounds__(kThreadsX) void edt_pass_x_pk(const uint32_t* __restrict__ hin, int X, int Y, int Z,
                                                          uint64_t cap, Out outp, uint32_t* count) {
    extern __shared__ uint16_t t16[];  // [kPad + X + kPad][TW]: min(h, 65535)
    constexpr int kSegs = TW / 4, kRows = kThreadsX / kSegs;
    const int nzc = (Z + TW - 1) / TW;
    const int y = blockIdx.x / nzc;
    const int z0 = (blockIdx.x - y * nzc) * TW;
    const int64_t yz = (int64_t)Y * Z;
    const int64_t col0 = (int64_t)y * Z + z0;
    if (!V) {
        for (int i = threadIdx.x; i < X * TW; i += kThreadsX) {
            const int x = i / TW, lz = i - x * TW;
            t16[(x + kPad) * TW + lz] = (uint16_t)(z0 + lz < Z ? min(hin[x * yz + col0 + lz], 65535u) : 65535u);
        }
    } else {
        const int seg = threadIdx.x % kSegs;
        const int zc = z0 + seg * 4;
        for (int x = threadIdx.x / kSegs; x < X; x += kRows) {
            uint2 w = make_uint2(0xFFFFFFFFu, 0xFFFFFFFFu);
            if (zc < Z) {
                const uint4 r = *reinterpret_cast<const uint4*>(hin + x * yz + col0 + seg * 4);
                w.x = min(r.x, 65535u) | min(r.y, 65535u) << 16;
                w.y = min(r.z, 65535u) | min(r.w, 65535u) << 16;
            }
            *reinterpret_cast<uint2*>(t16 + (x + kPad) * TW + seg * 4) = w;
        }
    }
    for (int i = threadIdx.x; i < 2 * kPad * TW; i += kThreadsX) {
        const int r = i / TW;
        t16[(r < kPad ? r : X + r) * TW + (i - r * TW)] = (uint16_t)65535u;
    }
    __syncthreads();
    constexpr int LC = TW / 2;             // lanes per tile row
    constexpr int RPI = kThreadsX / LC;    // rows per round
    const int lc = threadIdx.x % LC;
    const int z = z0 + 2 * lc;
    uint32_t hits = 0;
    if (z < Z) {
        const uint32_t capv = (uint32_t)cap;
        const uint32_t lim = min(capv, kSent32);
        const uint32_t c16 = min(capv, 65535u);
        const u16x2 capp = as_u16x2(c16 | c16 << 16);
        const uint32_t* col = reinterpret_cast<const uint32_t*>(t16 + kPad * TW) + lc;  // row i at col[i * LC]
        for (int x = threadIdx.x / LC; x < X; x += RPI) {
            u16x2 best = __builtin_elementwise_min(as_u16x2(col[x * LC]), capp);
            uint32_t bb = as_u32(best);
            uint32_t bmax = max(bb & 0xFFFFu, bb >> 16);
            if (bmax > 1) {
                const int far = min(max(x, X - 1 - x), 256);
                // rows x - o - 3 and x + o, stepped and held at the pad rows
                // in one move each (as in pass y)
                const uint32_t* const ltop = col - 4 * LC;
                const uint32_t* const rbot = col + X * LC;
                const uint32_t* lp = col + (x - 4) * LC;
                const uint32_t* rp = col + (x + 1) * LC;
                for (int o = 1; o <= far && (uint32_t)(o * o) < bmax;
                     o += 4, lp = lp - 4 * LC < ltop ? ltop : lp - 4 * LC, rp = rp + 4 * LC > rbot ? rbot : rp + 4 * LC) {
#pragma unroll
                    for (int j = 0; j < 4; j++) {
                        const uint32_t oo = min((uint32_t)((o + j) * (o + j)), 65535u);
                        const u16x2 oop = as_u16x2(oo | oo << 16);
                        best = __builtin_elementwise_min(
                            best, __builtin_elementwise_add_sat(
                                      __builtin_elementwise_min(as_u16x2(lp[(3 - j) * LC]), as_u16x2(rp[j * LC])), oop));
                    }
                    bb = as_u32(best);
                    bmax = max(bb & 0xFFFFu, bb >> 16);
                }
            }
            bb = as_u32(best);
#pragma unroll
            for (int e = 0; e < 2; e++) {
                if (z + e >= Z) break;
                const int64_t v = x * yz + col0 + 2 * lc + e;
                uint32_t r = e ? bb >> 16 : bb & 0xFFFFu;
                if (r == 65535u && capv > 65535u) r = pass_x_exact(hin, v, x, X, yz, cap);
                const uint64_t b = r >= lim ? (uint64_t)cap : (uint64_t)r;
                outp.put(v, b, cap);
                hits += outp.hit(v, b);
            }
        }
    }
    if (count) block_add_slots(count, hits);
}

// LDS a workgroup may use on the current device (the pass-x tile of a
// 512-voxel line takes 66.5 KB, of a 1024-voxel line 132 KB).
size_t max_lds_per_block() {
    static size_t cached[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 65536;
    if (!cached[dev]) {
        int v = 0;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
            v = 65536;
        cached[dev] = (size_t)v;
    }
    return cached[dev];
}

// the packed pass x with tiles of tx z columns and 16-byte loads (xv) or not
template <class Out>
void launch_pass_x_pk(int tx, bool xv, dim3 gx, size_t lds_bytes, hipStream_t s, const uint32_t* h, ibip_dims d,
                      uint64_t c64, Out o, uint32_t* count) {
    const dim3 b(kThreadsX);
    if (tx == 16) {
        if (xv) hipLaunchKernelGGL((edt_pass_x_pk<Out, 16, true>), gx, b, lds_bytes, s, h, d.X, d.Y, d.Z, c64, o, count);
        else hipLaunchKernelGGL((edt_pass_x_pk<Out, 16, false>), gx, b, lds_bytes, s, h, d.X, d.Y, d.Z, c64, o, count);
    } else {
        if (xv) hipLaunchKernelGGL((edt_pass_x_pk<Out, 32, true>), gx, b, lds_bytes, s, h, d.X, d.Y, d.Z, c64, o, count);
        else hipLaunchKernelGGL((edt_pass_x_pk<Out, 32, false>), gx, b, lds_bytes, s, h, d.X, d.Y, d.Z, c64, o, count);
    }
}

// Pass x: packed (pk) or 32-bit tiles of tx z columns, 16-byte loads (xv) or
// not. The packed kernels read h as one word per voxel (their exact search
// reads it in HBM), so the split form only ever comes with the 32-bit ones.
template <class Out, class H>
void launch_pass_x(bool pk, int tx, bool xv, dim3 gx, size_t lds_bytes, hipStream_t s, H in, ibip_dims d,
                   uint64_t c64, Out o, uint32_t* count) {
    if constexpr (!H::kSplit) {
        if (pk) return launch_pass_x_pk(tx, xv, gx, lds_bytes, s, in.h, d, c64, o, count);
    }
    const dim3 b(kThreadsX);
    if (tx == 16) {
        if (xv) hipLaunchKernelGGL((edt_pass_x_vec<Out, 16, true, H>), gx, b, lds_bytes, s, in, d.X, d.Y, d.Z, c64, o, count);
        else hipLaunchKernelGGL((edt_pass_x_vec<Out, 16, false, H>), gx, b, lds_bytes, s, in, d.X, d.Y, d.Z, c64, o, count);
    } else {
        if (xv) hipLaunchKernelGGL((edt_pass_x_vec<Out, 32, true, H>), gx, b, lds_bytes, s, in, d.X, d.Y, d.Z, c64, o, count);
        else hipLaunchKernelGGL((edt_pass_x_vec<Out, 32, false, H>), gx, b, lds_bytes, s, in, d.X, d.Y, d.Z, c64, o, count);
    }
}

// pass y with tiles of ty z columns and 16-byte loads (yv) or not
template <class H>
void launch_pass_y(int ty, bool yv, dim3 gy, size_t lds_bytes, hipStream_t s, const uint16_t* g16, ibip_dims d,
                   uint64_t c64, H h) {
    const dim3 b(kThreadsY);
    if (ty == 64 && yv) hipLaunchKernelGGL((edt_pass_y_pk<64, true, H>), gy, b, lds_bytes, s, g16, d.X, d.Y, d.Z, c64, h);
    else if (ty == 64) hipLaunchKernelGGL((edt_pass_y_pk<64, false, H>), gy, b, lds_bytes, s, g16, d.X, d.Y, d.Z, c64, h);
    else if (yv) hipLaunchKernelGGL((edt_pass_y_pk<32, true, H>), gy, b, lds_bytes, s, g16, d.X, d.Y, d.Z, c64, h);
    else hipLaunchKernelGGL((edt_pass_y_pk<32, false, H>), gy, b, lds_bytes, s, g16, d.X, d.Y, d.Z, c64, h);
}

}  // namespace

hipError_t launch_edt(const uint8_t* image, const uint32_t* w, uint32_t thr, uint32_t cap, ibip_dims d,
                      uint16_t* g16, uint32_t* tmp32, uint32_t* out, uint32_t* solid_flag, hipStream_t s,
                      uint32_t* mio_r2, uint32_t* mio_count, EdtTiles tiles) {
    // cap == 0: exact everywhere; else exact where dt2 < cap, 0xFFFFFFFF elsewhere
    const uint64_t c64 = cap ? (uint64_t)cap : 0xFFFFFFFFull;
    const int64_t n = nvox(d);
    // tile widths in z columns: pass y 32 or 64 (uint16), pass x 16 or 32 (uint32)
    const int ty = tiles.y == 64 ? 64 : 32, tx = tiles.x == 16 ? 16 : 32;
    // each pass takes its vectorised form where it can: pass z with the row in
    // registers for rows up to 1024 voxels; the LDS-tiled passes y and x when every
    // line the pass has read so far is at most 1024 voxels long (so each
    // distance along z is below 1024, each h below 2 * 1023^2, and 32-bit sums
    // with the sentinels cannot reach 2^31) and the tile fits in LDS, loading
    // their tiles with 16-byte vectors when the rows allow it. The other forms
    // read and write the same layouts.
    const size_t ly = sizeof(uint16_t) * ty * (d.Y + 2 * kPad), lx32 = sizeof(uint32_t) * tx * (d.X + 2 * kPad),
                 lx16 = sizeof(uint16_t) * tx * (d.X + 2 * kPad);
    const size_t lds = max_lds_per_block();
    const bool in_al = image ? ((uintptr_t)image & 7) == 0 : ((uintptr_t)w & 15) == 0;
    // pass z: P voxels per lane (8 for rows up to 512, else 16), vectors when
    // the rows are a multiple of P and the input is aligned
    const int zp = d.Z <= 512 ? 8 : d.Z <= kMaxVecLine ? 16 : 0;
    const bool zal = zp && in_al && d.Z % zp == 0;
    const bool yvec = d.Z <= kMaxVecLine && d.Y <= kMaxVecLine && ly <= lds;
    // pass x packed (16-bit tile) when two 1024-thread workgroups' 32-bit tiles
    // would not fit in a compute unit's LDS: on 512-voxel lines the 32-bit
    // kernel is faster (two columns per lane search as long as the longer of
    // the two), on 768 the packed one (twice the workgroups per unit)
    const bool xpk = 2 * lx32 > lds;
    const size_t lx = xpk ? lx16 : lx32;
    const bool xvec = yvec && d.X <= kMaxVecLine && lx <= lds;
    const bool yv = d.Z % 8 == 0, xv = d.Z % 4 == 0;  // rows that 16-byte loads can take
    const int64_t rows = (int64_t)d.X * d.Y;
    // h between passes y and x split in two (16 bits per voxel, the exact
    // values at 65535 and above in the output array) where pass x runs its
    // 32-bit tiles, which read all of it while loading, and writes an output
    const bool split = yvec && xvec && !xpk && out != nullptr && mio_r2 == nullptr;
    const HPlain hp{tmp32};
    const HSplit hs{reinterpret_cast<uint16_t*>(tmp32), out};
    if (zp) {
        // the distance cap of pass z: the least d with d^2 >= cap
        uint64_t dz64 = (uint64_t)std::sqrt((double)c64);
        while (dz64 * dz64 < c64) dz64++;
        while (dz64 > 0 && (dz64 - 1) * (dz64 - 1) >= c64) dz64--;
        const uint32_t dz = (uint32_t)std::min<uint64_t>(dz64, 0xFFFFu);
        const int64_t rows_per_block = 4LL * (64 / ((d.Z + zp - 1) / zp)) * kZGroups;
        const unsigned gz = (unsigned)((rows + rows_per_block - 1) / rows_per_block);
        const dim3 gzd(gz);
        const int form = (image ? 4 : 0) + (zp == 16 ? 2 : 0) + (zal ? 1 : 0);
        const FeatImage8 fi{image};
        const FeatThreshold8 ft{w, thr};
        switch (form) {
            case 7:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatImage8, 16, true>), gzd, dim3(256), 0, s, fi, rows, d.Z,
                                   dz, g16, solid_flag);
                break;
            case 6:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatImage8, 16, false>), gzd, dim3(256), 0, s, fi, rows, d.Z,
                                   dz, g16, solid_flag);
                break;
            case 5:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatImage8, 8, true>), gzd, dim3(256), 0, s, fi, rows, d.Z,
                                   dz, g16, solid_flag);
                break;
            case 4:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatImage8, 8, false>), gzd, dim3(256), 0, s, fi, rows, d.Z,
                                   dz, g16, solid_flag);
                break;
            case 3:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatThreshold8, 16, true>), gzd, dim3(256), 0, s, ft, rows, d.Z,
                                   dz, g16, solid_flag);
                break;
            case 2:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatThreshold8, 16, false>), gzd, dim3(256), 0, s, ft, rows,
                                   d.Z, dz, g16, solid_flag);
                break;
            case 1:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatThreshold8, 8, true>), gzd, dim3(256), 0, s, ft, rows, d.Z,
                                   dz, g16, solid_flag);
                break;
            default:
                hipLaunchKernelGGL((edt_pass_z_vec<FeatThreshold8, 8, false>), gzd, dim3(256), 0, s, ft, rows,
                                   d.Z, dz, g16, solid_flag);
                break;
        }
    } else {
        const unsigned gz = (unsigned)((rows + 3) / 4);
        if (image)
            hipLaunchKernelGGL(edt_pass_z<FeatImage>, dim3(gz), dim3(256), 0, s, FeatImage{image}, rows, d.Z, c64,
                               g16, solid_flag);
        else
            hipLaunchKernelGGL(edt_pass_z<FeatThreshold>, dim3(gz), dim3(256), 0, s, FeatThreshold{w, thr}, rows,
                               d.Z, c64, g16, solid_flag);
    }
    const unsigned gv = (unsigned)((n + 255) / 256);
    if (yvec) {
        const unsigned nzy = (unsigned)((d.Z + ty - 1) / ty);
        const dim3 gy((unsigned)d.X * nzy);
        if (split) launch_pass_y(ty, yv, gy, ly, s, g16, d, c64, hs);
        else launch_pass_y(ty, yv, gy, ly, s, g16, d, c64, hp);
    } else if (d.Y <= kMaxTileLine) {
        const int nzc = (d.Z + kW - 1) / kW;
        hipLaunchKernelGGL(edt_pass_y_tile, dim3((unsigned)(d.X * nzc)), dim3(256), sizeof(uint16_t) * kW * d.Y, s,
                           g16, d.X, d.Y, d.Z, c64, tmp32);
    } else {
        hipLaunchKernelGGL(edt_pass_y, dim3(gv), dim3(256), 0, s, g16, d.X, d.Y, d.Z, c64, tmp32);
    }
    if (xvec) {
        const unsigned nzx = (unsigned)((d.Z + tx - 1) / tx);
        const dim3 gx((unsigned)d.Y * nzx);
        const OutOpening oo{mio_r2, cap};
        const OutPlain op{out};
        uint32_t* const nocount = nullptr;
        if (mio_r2) launch_pass_x(xpk, tx, xv, gx, lx, s, hp, d, c64, oo, mio_count);
        else if (split) launch_pass_x(xpk, tx, xv, gx, lx, s, hs, d, c64, op, nocount);
        else launch_pass_x(xpk, tx, xv, gx, lx, s, hp, d, c64, op, nocount);
        return hipGetLastError();
    }
    const int nzcx = (d.Z + kWx - 1) / kWx;
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
