// Defender trapping and re-ranking (Section 2.2.3, Figure 7), and the
// maximin reconstruction it shares with the opening drainage.
//
// A voxel v invaded at step k is trapped when the defender region D_k =
// {pore u : seq[u] == 0 or seq[u] >= k} holds no path from v to an outlet.
// With node capacities cap(u) = infinity for uninvaded pore and seq[u] for
// invaded voxels, a path lies in D_k exactly when its smallest capacity is
// >= k. So with W(v) = max over paths from the outlets to v of the smallest
// capacity on the path (a maximin, or widest-path, value), v is free iff
// W(v) >= seq[v]. The paper's reverse sweep over thresholds computes the same
// predicate one level at a time; W gives it for every level at once and is
// computed here by data-parallel relaxation to the fixed point
//   W(v) = max(W0(v), min(cap(v), max over face neighbours u of W(u))).
//
// Relaxation runs per 8 x 16 x 32 tile: the tile and a one-voxel halo sit in
// LDS and are relaxed until nothing changes (6-connected: rounds of forward and
// backward scans along the lines of each axis; 26-connected: neighbour sweeps). Sweeps repeat over the active
// tiles (all at first, then those whose face-neighbour changed its boundary
// layer) until no tile changes. W only grows and is bounded, so this ends at
// the unique fixed point.
#include <climits>

#include "ibip_internal.h"

namespace ibip {

namespace {

constexpr int TX = 8, TY = 16, TZ = 32;  // 4096 voxels per tile, 16 per thread
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;

struct CapSeq {
    const int32_t* seq;
    __device__ uint32_t operator()(int64_t v) const {
        int32_t s = seq[v];
        return s < 0 ? 0u : (s == 0 ? kInf32 : (uint32_t)s);
    }
};
struct CapU32 {
    const uint32_t* cap;
    __device__ uint32_t operator()(int64_t v) const { return cap[v]; }
};

// One sweep over the active tiles, in ascending tile order or (rev) in
// descending order. Tiles update w in place, so a tile that starts after a
// neighbour has written reads the neighbour's new boundary in the same sweep;
// alternating the order lets values travel several tiles per sweep towards
// either end of the image (any order reaches the same fixed point: w only
// grows). A tile whose boundary layer changed
// activates the face-neighbour tiles across the changed faces for the next
// sweep (act_out); *changed is set when a tile changed anything. Each active
// tile clears its own act_in flag, so act_in is all zero afterwards and
// serves as act_out of the next sweep. kConn26: the
// neighbours of a voxel are the 26 that share a face, an edge or a corner,
// and the edge and corner tiles are activated too (a tile across an edge or
// a corner when every face it lies across changed, which covers every
// changed voxel on that edge or corner).
template <class Cap, bool kConn26>
__global__ __launch_bounds__(256) void k_relax_tiles(Cap cap, int X, int Y, int Z, int ntx, int nty, int ntz,
                                                     uint32_t* w, uint8_t* act_in, uint8_t* act_out,
                                                     uint32_t* changed, bool rev) {
    __shared__ uint32_t hw[HX * HY * HZ];
    __shared__ uint32_t hc[kConn26 ? 1 : TX * TY * TZ];  // capacities, for the line scans
    __shared__ uint32_t face[6];
    const int tid = threadIdx.x;
    const int64_t tile = rev ? (int64_t)gridDim.x - 1 - blockIdx.x : (int64_t)blockIdx.x;
    if (!act_in[tile]) return;
    __syncthreads();  // every thread has read the flag
    if (tid == 0) act_in[tile] = 0;
    const int tz = (int)(tile % ntz);
    const int ty = (int)((tile / ntz) % nty);
    const int tx = (int)(tile / ((int64_t)ntz * nty));
    const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
    const int64_t yz = (int64_t)Y * Z;
    if (tid < 6) face[tid] = 0;
    // Tile, halo and capacities: every load is issued before the first is
    // used. Coordinates are clamped into the image and out-of-image values
    // replaced afterwards, so no load sits under a lane condition (such a
    // load is waited for at once, one round trip each).
    constexpr int HN = HX * HY * HZ, HPER = (HN + 255) / 256;
    uint32_t hv[HPER];
#pragma unroll
    for (int q = 0; q < HPER; q++) {
        const int i = min(tid + q * 256, HN - 1);
        const int hz = i % HZ, hy = (i / HZ) % HY, hx = i / (HZ * HY);
        const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
        const bool in = gx >= 0 && gx < X && gy >= 0 && gy < Y && gz >= 0 && gz < Z;
        const int cx = min(max(gx, 0), X - 1), cy = min(max(gy, 0), Y - 1), cz = min(max(gz, 0), Z - 1);
        const uint32_t val = w[cx * yz + (int64_t)cy * Z + cz];
        hv[q] = in ? val : 0u;
    }
    const int lz = tid & 31, ly = tid >> 5;  // ly in [0, 8): rows ly and ly + 8
    constexpr int NV = TX * 2;
    uint32_t c[NV], orig[NV];
    const int gz = z0 + lz;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        const int gx = x0 + (j >> 1), gy = y0 + ly + 8 * (j & 1);
        const bool in = gx < X && gy < Y && gz < Z;
        const uint32_t cv = cap(min(gx, X - 1) * yz + (int64_t)min(gy, Y - 1) * Z + min(gz, Z - 1));
        c[j] = in ? cv : 0u;
    }
#pragma unroll
    for (int q = 0; q < HPER; q++)
        if (tid + q * 256 < HN) hw[tid + q * 256] = hv[q];
    __syncthreads();
#pragma unroll
    for (int j = 0; j < NV; j++) orig[j] = hw[(((j >> 1) + 1) * HY + (ly + 8 * (j & 1) + 1)) * HZ + (lz + 1)];
    bool any_change = false;
    if (!kConn26) {
        // Rounds of line scans: along each axis every line is relaxed forward
        // and backward in registers, w[i] = max(w[i], min(cap[i], w[i -+ 1])),
        // so a value travels the whole line in one scan and a round moves it
        // around as many corners as a path takes in the tile, where a
        // neighbour-by-neighbour sweep needs as many rounds as the path has
        // voxels. Each update only raises w towards the fixed point, so the
        // result is the same.
#pragma unroll
        for (int j = 0; j < NV; j++) hc[((j >> 1) * TY + (ly + 8 * (j & 1))) * TZ + lz] = c[j];
        __syncthreads();
        for (;;) {
            bool ch = false;
            if (tid < TX * TY) {  // lines along z (waves 0 and 1)
                const int lx = tid >> 4, lyy = tid & 15;
                const int base = ((lx + 1) * HY + (lyy + 1)) * HZ;
                const int cb = (lx * TY + lyy) * TZ;
                uint32_t v[HZ], cc[TZ];
#pragma unroll
                for (int i = 0; i < HZ; i++) v[i] = hw[base + i];
#pragma unroll
                for (int i = 0; i < TZ; i++) cc[i] = hc[cb + i];
                bool lc = false;
#pragma unroll
                for (int i = 1; i <= TZ; i++) {
                    const uint32_t nv = max(v[i], min(cc[i - 1], v[i - 1]));
                    lc |= nv != v[i];
                    v[i] = nv;
                }
#pragma unroll
                for (int i = TZ; i >= 1; i--) {
                    const uint32_t nv = max(v[i], min(cc[i - 1], v[i + 1]));
                    lc |= nv != v[i];
                    v[i] = nv;
                }
                if (lc) {
#pragma unroll
                    for (int i = 1; i <= TZ; i++) hw[base + i] = v[i];
                }
                ch |= lc;
            }
            __syncthreads();
            {  // lines along y: one per thread
                const int lx = tid >> 5, lzz = tid & 31;
                const int base = (lx + 1) * HY * HZ + (lzz + 1);
                uint32_t v[HY], cc[TY];
#pragma unroll
                for (int i = 0; i < HY; i++) v[i] = hw[base + i * HZ];
#pragma unroll
                for (int i = 0; i < TY; i++) cc[i] = hc[(lx * TY + i) * TZ + lzz];
                bool lc = false;
#pragma unroll
                for (int i = 1; i <= TY; i++) {
                    const uint32_t nv = max(v[i], min(cc[i - 1], v[i - 1]));
                    lc |= nv != v[i];
                    v[i] = nv;
                }
#pragma unroll
                for (int i = TY; i >= 1; i--) {
                    const uint32_t nv = max(v[i], min(cc[i - 1], v[i + 1]));
                    lc |= nv != v[i];
                    v[i] = nv;
                }
                if (lc) {
#pragma unroll
                    for (int i = 1; i <= TY; i++) hw[base + i * HZ] = v[i];
                }
                ch |= lc;
            }
            __syncthreads();
#pragma unroll
            for (int hh = 0; hh < 2; hh++) {  // lines along x: two per thread
                const int line = tid + 256 * hh;
                const int lyy = line >> 5, lzz = line & 31;
                const int base = (lyy + 1) * HZ + (lzz + 1);
                uint32_t v[HX], cc[TX];
#pragma unroll
                for (int i = 0; i < HX; i++) v[i] = hw[base + i * HY * HZ];
#pragma unroll
                for (int i = 0; i < TX; i++) cc[i] = hc[(i * TY + lyy) * TZ + lzz];
                bool lc = false;
#pragma unroll
                for (int i = 1; i <= TX; i++) {
                    const uint32_t nv = max(v[i], min(cc[i - 1], v[i - 1]));
                    lc |= nv != v[i];
                    v[i] = nv;
                }
#pragma unroll
                for (int i = TX; i >= 1; i--) {
                    const uint32_t nv = max(v[i], min(cc[i - 1], v[i + 1]));
                    lc |= nv != v[i];
                    v[i] = nv;
                }
                if (lc) {
#pragma unroll
                    for (int i = 1; i <= TX; i++) hw[base + i * HY * HZ] = v[i];
                }
                ch |= lc;
            }
            // wave-uniform exit (see the note on loop control in invade.hip)
            if (!__builtin_amdgcn_readfirstlane(__syncthreads_or(ch))) break;
            any_change = true;
        }
    } else {
        for (;;) {
            bool ch = false;
#pragma unroll
            for (int j = 0; j < NV; j++) {
                if (c[j] == 0) continue;
                const int idx = (((j >> 1) + 1) * HY + (ly + 8 * (j & 1) + 1)) * HZ + (lz + 1);
                const uint32_t cur = hw[idx];
                if (cur >= c[j]) continue;
                uint32_t nb;
                if (kConn26) {
                    nb = 0;
#pragma unroll
                    for (int dx = -1; dx <= 1; dx++)
#pragma unroll
                        for (int dy = -1; dy <= 1; dy++)
#pragma unroll
                            for (int dz = -1; dz <= 1; dz++)
                                if (dx || dy || dz) nb = max(nb, hw[idx + (dx * HY + dy) * HZ + dz]);
                } else {
                    nb = max(max(hw[idx - 1], hw[idx + 1]), max(hw[idx - HZ], hw[idx + HZ]));
                    nb = max(nb, max(hw[idx - HY * HZ], hw[idx + HY * HZ]));
                }
                const uint32_t cand = min(c[j], nb);
                if (cand > cur) { hw[idx] = cand; ch = true; }
            }
            // wave-uniform exit (see the note on loop control in invade.hip)
            if (!__builtin_amdgcn_readfirstlane(__syncthreads_or(ch))) break;
            any_change = true;
        }
    }
    if (!any_change) return;
    bool wrote = false;
#pragma unroll
    for (int j = 0; j < NV; j++) {
        const int lx = j >> 1, lyy = ly + 8 * (j & 1);
        const int gx = x0 + lx, gy = y0 + lyy;
        if (gx >= X || gy >= Y || gz >= Z) continue;
        const uint32_t nv = hw[((lx + 1) * HY + (lyy + 1)) * HZ + (lz + 1)];
        if (nv != orig[j]) {
            w[gx * yz + (int64_t)gy * Z + gz] = nv;
            wrote = true;
            if (lx == 0) face[0] = 1;
            if (lx == TX - 1) face[1] = 1;
            if (lyy == 0) face[2] = 1;
            if (lyy == TY - 1) face[3] = 1;
            if (lz == 0) face[4] = 1;
            if (lz == TZ - 1) face[5] = 1;
        }
    }
    if (__builtin_amdgcn_readfirstlane(__syncthreads_or(wrote))) {
        // a flag, read first: one word taking an atomic from every tile that
        // changed would queue them all at one place
        if (tid == 0 && __hip_atomic_load(changed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
            atomicOr(changed, 1u);
        if (kConn26) {
            if (tid < 27 && tid != 13) {
                const int dx = tid / 9 - 1, dy = (tid / 3) % 3 - 1, dz = tid % 3 - 1;
                const bool cross = (dx == 0 || face[dx < 0 ? 0 : 1]) && (dy == 0 || face[dy < 0 ? 2 : 3]) &&
                                   (dz == 0 || face[dz < 0 ? 4 : 5]);
                const int nx = tx + dx, ny = ty + dy, nz = tz + dz;
                if (cross && nx >= 0 && nx < ntx && ny >= 0 && ny < nty && nz >= 0 && nz < ntz)
                    act_out[((int64_t)nx * nty + ny) * ntz + nz] = 1;
            }
        } else if (tid < 6 && face[tid]) {
            int nx = tx, ny = ty, nz = tz;
            if (tid == 0) nx--;
            if (tid == 1) nx++;
            if (tid == 2) ny--;
            if (tid == 3) ny++;
            if (tid == 4) nz--;
            if (tid == 5) nz++;
            if (nx >= 0 && nx < ntx && ny >= 0 && ny < nty && nz >= 0 && nz < ntz)
                act_out[((int64_t)nx * nty + ny) * ntz + nz] = 1;
        }
    }
}

// ---- trapping ----
// w[v] = the seed of the maximin reconstruction (the step on outlet voxels,
// kInf32 on uninvaded outlet pore, 0 elsewhere), and the largest step of the
// image into max_slots[block % kCountSlots]: each block covers a contiguous
// chunk of kCntChunk voxels and adds one atomic.
__global__ __launch_bounds__(256) void k_trap_init(const int32_t* seq, const uint8_t* outlets, int64_t n,
                                                   uint32_t* w, int32_t* max_slots) {
    __shared__ int32_t part[4];
    int32_t m = 0;
    const int64_t base = (int64_t)blockIdx.x * kCntChunk;
    for (int j = 0; j < kCntChunk; j += 256) {
        const int64_t v = base + j + threadIdx.x;
        if (v < n) {
            const int32_t s = seq[v];
            m = max(m, s);
            uint32_t val = 0;
            if (s >= 0 && outlets[v]) val = s == 0 ? kInf32 : (uint32_t)s;
            w[v] = val;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        m = max(max(part[0], part[1]), max(part[2], part[3]));
        if (m > 0) atomicMax(&max_slots[blockIdx.x % kCountSlots], m);
    }
}

__global__ __launch_bounds__(256) void k_trap_mark(const int32_t* seq, const uint32_t* w, int64_t n,
                                                   uint8_t* trapped, uint32_t* present) {
    int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t s = seq[v];
    const bool t = s > 0 && w[v] < (uint32_t)s;
    trapped[v] = t ? 1 : 0;
    // most voxels of a step find its flag already set: read before writing
    if (s > 0 && !t && __hip_atomic_load(&present[s - 1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        present[s - 1] = 1u;
}

__global__ __launch_bounds__(256) void k_trap_rank(const int32_t* seq, const uint8_t* trapped,
                                                   const uint32_t* rank_excl, int64_t n, int32_t* out) {
    int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    const int32_t s = seq[v];
    int32_t r;
    if (s < 0) r = -1;
    else if (s == 0 || trapped[v]) r = 0;
    else r = (int32_t)rank_excl[s - 1] + 1;
    out[v] = r;
}

inline unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

ibip_status reconstruct(ibip_ctx* ctx, const int32_t* seq, const uint32_t* cap32, bool conn26, ibip_dims d,
                        uint32_t* w, int* n_iter) {
    hipStream_t s = ctx->stream;
    const int ntx = (d.X + TX - 1) / TX, nty = (d.Y + TY - 1) / TY, ntz = (d.Z + TZ - 1) / TZ;
    const int64_t ntiles = (int64_t)ntx * nty * ntz;
    constexpr int kBatch = 16;  // sweeps per host check
    uint8_t* misc = (uint8_t*)ensure(ctx, B_MISC, 4096);
    uint8_t* act = (uint8_t*)ensure(ctx, B_ACT, 2 * (size_t)ntiles + 64);
    uint32_t* cnt = (uint32_t*)ensure(ctx, B_CNT, sizeof(uint32_t) * kBatch);
    uint32_t* h = (uint32_t*)pinned(ctx, 4096);
    if (!misc || !act || !cnt || !h) return fail(ctx, IBIP_ENOMEM, "reconstruct: allocation failed");
    uint8_t* a0 = act;
    uint8_t* a1 = act + ntiles;
    uint32_t* h_changed = h + 512;
    ibip_status rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(a0, 1, ntiles, s), "memset")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(a1, 0, ntiles, s), "memset")) != IBIP_OK) return rc;
    int it = 0;
    const int limit = 4 * (d.X + d.Y + d.Z) + 100000;
    for (;;) {
        if ((rc = hip_check(ctx, hipMemsetAsync(cnt, 0, sizeof(uint32_t) * kBatch, s), "memset")) != IBIP_OK) return rc;
        for (int b = 0; b < kBatch; b++, it++) {
            uint8_t* in = (it & 1) ? a1 : a0;
            uint8_t* out = (it & 1) ? a0 : a1;  // all zero: cleared by the sweep that read it
            const bool rev = (it & 1) != 0;     // alternate the tile order
            if (cap32)
                hipLaunchKernelGGL((k_relax_tiles<CapU32, false>), dim3((unsigned)ntiles), dim3(256), 0, s,
                                   CapU32{cap32}, d.X, d.Y, d.Z, ntx, nty, ntz, w, in, out, cnt + b, rev);
            else if (conn26)
                hipLaunchKernelGGL((k_relax_tiles<CapSeq, true>), dim3((unsigned)ntiles), dim3(256), 0, s,
                                   CapSeq{seq}, d.X, d.Y, d.Z, ntx, nty, ntz, w, in, out, cnt + b, rev);
            else
                hipLaunchKernelGGL((k_relax_tiles<CapSeq, false>), dim3((unsigned)ntiles), dim3(256), 0, s,
                                   CapSeq{seq}, d.X, d.Y, d.Z, ntx, nty, ntz, w, in, out, cnt + b, rev);
        }
        if ((rc = hip_check(ctx, hipGetLastError(), "relax launch")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipMemcpyAsync(h_changed, cnt + kBatch - 1, sizeof(uint32_t), hipMemcpyDeviceToHost,
                                                s), "copy")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
        if (*h_changed == 0) break;
        if (it > limit) return fail(ctx, IBIP_EDEVICE, "reconstruct: no fixed point after the iteration limit");
    }
    if (n_iter) *n_iter = it;
    return IBIP_OK;
}

ibip_status run_trap(ibip_ctx* ctx, const int32_t* seq, const uint8_t* outlets, ibip_dims d, uint8_t* trapped,
                     int32_t* seq_trapped, int64_t* n_steps_after) {
    hipStream_t s = ctx->stream;
    const int64_t n = nvox(d);
    uint32_t* w = (uint32_t*)ensure(ctx, B_KEY, sizeof(uint32_t) * n);
    uint8_t* misc = (uint8_t*)ensure(ctx, B_MISC, 4096);
    uint32_t* h = (uint32_t*)pinned(ctx, 4096);
    if (!w || !misc || !h) return fail(ctx, IBIP_ENOMEM, "trap: allocation failed");
    int32_t* dmax = (int32_t*)(misc + 2048);  // kCountSlots words
    uint32_t* dtotal = (uint32_t*)(misc + 3076);
    ibip_status rc;
    ctx->timer.mark(10, s);
    if ((rc = hip_check(ctx, hipMemsetAsync(dmax, 0, sizeof(int32_t) * kCountSlots, s), "memset")) != IBIP_OK)
        return rc;
    hipLaunchKernelGGL(k_trap_init, dim3((unsigned)((n + kCntChunk - 1) / kCntChunk)), dim3(256), 0, s, seq, outlets,
                       n, w, dmax);
    if ((rc = hip_check(ctx, hipMemcpyAsync(h, dmax, sizeof(int32_t) * kCountSlots, hipMemcpyDeviceToHost, s),
                        "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    int32_t kmax = 0;
    for (int q = 0; q < kCountSlots; q++) kmax = std::max(kmax, (int32_t)h[q]);
    const int64_t K = kmax;
    int iters = 0;
    if ((rc = reconstruct(ctx, seq, nullptr, (ctx->readings & IBIP_READ_TRAP26) != 0, d, w, &iters)) != IBIP_OK)
        return rc;
    uint32_t* present = (uint32_t*)ensure(ctx, B_TMP2, sizeof(uint32_t) * (K + 1));
    uint32_t* partials = (uint32_t*)ensure(ctx, B_SCAN, sizeof(uint32_t) * (K / 1000 + n / 1000 + 64));
    if (!present || !partials) return fail(ctx, IBIP_ENOMEM, "trap: allocation failed");
    if ((rc = hip_check(ctx, hipMemsetAsync(present, 0, sizeof(uint32_t) * (K + 1), s), "memset")) != IBIP_OK)
        return rc;
    hipLaunchKernelGGL(k_trap_mark, dim3(blocks(n)), dim3(256), 0, s, seq, w, n, trapped, present);
    if (K > 0) {
        if ((rc = hip_check(ctx, launch_scan_u32(present, K, partials, dtotal, s), "scan")) != IBIP_OK) return rc;
    }
    if (seq_trapped) hipLaunchKernelGGL(k_trap_rank, dim3(blocks(n)), dim3(256), 0, s, seq, trapped, present, n,
                                        seq_trapped);
    if ((rc = hip_check(ctx, hipGetLastError(), "trap launch")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(h + 1, dtotal, sizeof(uint32_t), hipMemcpyDeviceToHost, s), "copy")) !=
        IBIP_OK)
        return rc;
    ctx->timer.mark(11, s);
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (ctx->timer.on) {
        ctx->timing.trap_ms += ctx->timer.ms(10, 11);
        ctx->timing.relax_sweeps += iters;
    }
    if (n_steps_after) *n_steps_after = K > 0 ? (int64_t)h[1] : 0;
    return IBIP_OK;
}

}  // namespace ibip
