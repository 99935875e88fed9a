// The invasion loop of Section 2.1 (Figure 2(e)-(l)) and its per-step
// post-processing (Sections 2.2.1-2.2.2).
//
// Data layout in HBM (N voxels, N_pore pore voxels, R distinct dt2 values):
//   key[N]      uint32  bits 0..23: rank of dt2 among the distinct pore values
//               (1..R), 0 on solid; bits 24..29: which of the six face
//               neighbours lie inside the image (pore voxels only); bit 31:
//               claimed as a candidate (one atomicOr claims a neighbour and
//               returns its rank and its in-image neighbours)
//   state[N]    int32   k > 0: centre of step k; 0 otherwise
//   bucket[N_pore] uint32  candidates grouped by rank; rank r owns the slice
//               [off[r], off[r+1]) whose length is the number of pore voxels
//               of that rank, so every pore voxel fits exactly once
//   head/tail[R+1]  the live part of each slice
//
// One step (a "round") pops the whole live part of the highest non-empty
// slice (every candidate holding the maximum -- the all-maxima rule), marks
// those voxels as centres of the step and appends their unseen pore face
// neighbours to the slices of their ranks. Entries appended during a step are
// popped from the next step on, which reproduces the rescan of the dilated
// inlets image step by step.
//
// Steps are a chain of dependent rounds, mostly tiny, so the loop runs inside
// ONE workgroup with the slice heads, tails and a two-level occupancy bitmap
// in LDS: a round costs one workgroup barrier and a few L2 round trips. A
// step with more than kWideRound centres exits to the host, which runs that
// step with the whole GPU and resumes the loop.
//
// Sphere insertion is decoupled from selection (selection never reads what
// was painted): after the loop, seq[v] = min over centres c whose ball
// B(c, M) = {|v - c|^2 < M} holds v of step(c), as an atomicMin per stamp --
// this equals first-write-wins in step order. A centre c with a face
// neighbour p that was a centre of an earlier step with a ball at least as
// large stamps only the part of its ball outside B(p): the one-voxel cap
// S = {o : |o|^2 < M <= |o - n|^2} (n = p - c), filtered by every other such
// neighbour. This is exact: the smallest step covering a voxel always stamps
// it, since a ball it skipped is covered by an earlier ball.
#include <chrono>
#include <climits>
#include <thread>
#include <vector>

#include "ibip_internal.h"

namespace ibip {

namespace {

// largest q with q * q <= a. Below 2^24 a is exact as a float and the float
// square root is within one of the answer, so one step each way corrects it
// in 32-bit arithmetic; larger a take 64-bit correction loops.
__device__ inline uint32_t isqrt_u32(uint32_t a) {
    if (a < (1u << 24)) {
        uint32_t q = (uint32_t)sqrtf((float)a);
        q -= q * q > a ? 1u : 0u;
        q += (q + 1u) * (q + 1u) <= a ? 1u : 0u;
        return q;
    }
    uint64_t q = (uint64_t)sqrtf((float)a);
    while (q * q > a) q--;
    while ((q + 1) * (q + 1) <= a) q++;
    return (uint32_t)q;
}

// Key words: bits 0..23 hold the rank of dt2 among the distinct pore values
// (0 on solid); bit 24 + d is set when the face neighbour in direction d
// (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z) lies inside the image; bit 31 marks
// a voxel claimed as a candidate. A claim thus returns, with the rank, what a
// later step needs to claim the voxel's own neighbours without dividing its
// index into coordinates.
constexpr uint32_t kClaim = 0x80000000u;
constexpr uint32_t kRankMask = 0x00FFFFFFu;
constexpr int kNbShift = 24;

// in-image neighbour bits of the voxel at (x, y, z)
__device__ inline uint32_t nb_bits(uint32_t x, uint32_t y, uint32_t z, int X, int Y, int Z) {
    return (x > 0 ? 1u : 0u) | (x + 1 < (uint32_t)X ? 2u : 0u) | (y > 0 ? 4u : 0u) |
           (y + 1 < (uint32_t)Y ? 8u : 0u) | (z > 0 ? 16u : 0u) | (z + 1 < (uint32_t)Z ? 32u : 0u);
}

// number of set bits of m in the lanes below this one
__device__ inline uint32_t lanes_below(uint64_t m) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

__device__ inline uint64_t lanemask_lt() {
    const int lane = threadIdx.x & 63;
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// ---------------------------------------------------------------------------
// Setup
// ---------------------------------------------------------------------------

// Histogram of dt2 over pore voxels, pore count, largest value.
constexpr int kHistLds = 2048;
// k_hist's grid: every block adds each of its non-empty bins to the global
// histogram, so the common distances take one atomic per block
constexpr int kHistBlocks = 1024;
// Values >= vlimit (the no-solid sentinel) are skipped; the host rejects such
// images before anything reads the tables.
__global__ __launch_bounds__(256) void k_hist(const uint32_t* __restrict__ dt2,
                                              int64_t n, uint32_t vlimit, uint32_t* hist, LoopState* st) {
    __shared__ uint32_t h[kHistLds];
    __shared__ uint32_t s_pore, s_max;
    for (int i = threadIdx.x; i < kHistLds; i += 256) h[i] = 0;
    if (threadIdx.x == 0) { s_pore = 0; s_max = 0; }
    __syncthreads();
    uint32_t pore = 0, mx = 0;
    // dt2 is 0 exactly on solid, so the image itself is not read; four
    // voxels per thread and round, their loads issued together
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t v0 = (int64_t)blockIdx.x * 256 + threadIdx.x; v0 < n; v0 += 4 * stride) {
        uint32_t d[4];
#pragma unroll
        for (int j = 0; j < 4; j++) d[j] = v0 + j * stride < n ? dt2[v0 + j * stride] : 0u;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            if (d[j] == 0 || d[j] >= vlimit) continue;
            pore++;
            mx = d[j] > mx ? d[j] : mx;
            if (d[j] < kHistLds) atomicAdd(&h[d[j]], 1u);
            else atomicAdd(&hist[d[j]], 1u);
        }
    }
    atomicAdd(&s_pore, pore);
    atomicMax(&s_max, mx);
    __syncthreads();
    for (int i = threadIdx.x; i < kHistLds; i += 256)
        if (h[i]) atomicAdd(&hist[i], h[i]);
    if (threadIdx.x == 0) {
        atomicAdd(&st->n_pore, s_pore);
        atomicMax(&st->maxval, s_max);
    }
}

// present[v] = 1 if some pore voxel has dt2 == v (v >= 1)
__global__ void k_present(const uint32_t* hist, uint32_t* present, int64_t V) {
    int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v < V) present[v] = (v >= 1 && hist[v] > 0) ? 1u : 0u;
}

// After the scans: offv[v] = bucket offset of value v, rk[v] = rank - 1 of v.
// rcap: the largest rank the tables hold (a job of a batch or of the server
// has room for kMaxRanks; beyond that its loop rejects the image).
__global__ void k_rank_tables(const uint32_t* cnt_scanned, const uint32_t* present_scanned,
                              const uint32_t* hist_raw_flag, int64_t V, uint32_t* val, uint32_t* off,
                              uint32_t* head, uint32_t* tail, uint32_t rcap) {
    int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= V || v == 0 || !hist_raw_flag[v]) return;
    uint32_t r = present_scanned[v] + 1;
    if (r > rcap + 1) return;  // too many ranks: the loop rejects the image
    val[r] = (uint32_t)v;
    off[r] = cnt_scanned[v];
    head[r] = cnt_scanned[v];
    tail[r] = cnt_scanned[v];
}

// key = rank and in-image neighbour bits (0 on solid); state = 0;
// seq = INT_MAX on pore, -1 on solid.
__global__ __launch_bounds__(256) void k_convert(const uint8_t* __restrict__ img, uint32_t* key,
                                                 const uint32_t* __restrict__ present_scanned, int64_t n,
                                                 uint32_t vlimit, int32_t* state, int32_t* seq, int X, int Y, int Z,
                                                 FastDiv divZ, FastDiv divY, uint32_t rcap) {
    int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (v >= n) return;
    state[v] = 0;
    if (img[v]) {
        const uint32_t d = key[v];
        // d >= vlimit only without any solid voxel; such images are rejected
        const uint32_t rk = d < vlimit ? present_scanned[d] + 1 : 0u;
        const uint32_t t = fdiv((uint32_t)v, divZ), xx = fdiv(t, divY);
        const uint32_t nb = nb_bits(xx, t - xx * (uint32_t)Y, (uint32_t)v - t * (uint32_t)Z, X, Y, Z);
        key[v] = rk > rcap ? 0u : rk | (nb << kNbShift);
        seq[v] = INT_MAX;
    } else {
        key[v] = 0;
        seq[v] = -1;
    }
}

// Groups the active lanes of a wave by rank with ballots only (no memory
// access): `lead` = the group's first lane, `off` = the lane's place in its
// group, `cnt` = the group's size on the first lane, 0 elsewhere.
struct RankGroup {
    uint32_t lead = 0, off = 0, cnt = 0;
};
__device__ inline RankGroup group_by_rank(bool active, uint32_t rr) {
    const int lane = threadIdx.x & 63;
    const uint64_t lt = lanemask_lt();
    RankGroup g;
    uint64_t pending = __ballot(active);
    while (pending) {
        const int leader = __ffsll((unsigned long long)pending) - 1;
        const uint32_t lr = __builtin_amdgcn_readlane(rr, leader);
        const uint64_t same = __ballot(active && rr == lr) & pending;
        if ((same >> lane) & 1) {
            g.lead = (uint32_t)leader;
            g.off = (uint32_t)__popcll(same & lt);
        }
        if (lane == leader) g.cnt = (uint32_t)__popcll(same);
        pending &= ~same;
    }
    return g;
}

// Append u to the slice of rank rr with one atomic per distinct rank in the
// wave (many waves hitting one slice tail lane by lane contend at L2).
__device__ inline void push_global(bool active, uint32_t u, uint32_t rr, uint32_t* tail, uint32_t* bucket) {
    const RankGroup g = group_by_rank(active, rr);
    uint32_t base = g.cnt ? atomicAdd(&tail[rr], g.cnt) : 0u;
    base = __shfl(base, (int)g.lead, 64);
    if (active) bucket[base + g.off] = u;
}

// Seeds: Q0 = (inlets U their face neighbours) restricted to pore.
// mask: a solid inlet voxel (rank 0) seeds nothing (the masked reading).
__global__ __launch_bounds__(256) void k_seed(const uint8_t* __restrict__ inlets, uint32_t* key, int X, int Y,
                                              int Z, uint32_t* tail, uint32_t* bucket, bool mask, uint32_t rcap) {
    const int64_t n = (int64_t)X * Y * Z;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool inl = v < n && inlets[v] != 0 && (!mask || (key[v] & kRankMask) != 0);
    if (!__any(inl)) return;
    const int64_t yz = (int64_t)Y * Z;
    int z = 0, y = 0, x = 0;
    if (inl) { z = (int)(v % Z); y = (int)((v / Z) % Y); x = (int)(v / yz); }
#pragma unroll
    for (int j = 0; j < 7; j++) {
        bool ok = inl;
        int64_t u = v;
        if (j == 1) { ok &= x > 0; u = v - yz; }
        if (j == 2) { ok &= x < X - 1; u = v + yz; }
        if (j == 3) { ok &= y > 0; u = v - Z; }
        if (j == 4) { ok &= y < Y - 1; u = v + Z; }
        if (j == 5) { ok &= z > 0; u = v - 1; }
        if (j == 6) { ok &= z < Z - 1; u = v + 1; }
        bool won = false;
        uint32_t rr = 0;
        if (ok && key[u] < kClaim) {
            const uint32_t old = atomicOr(&key[u], kClaim);
            rr = old & kRankMask;
            won = !(old & kClaim) && rr != 0 && rr <= rcap;
        }
        push_global(won, (uint32_t)u, rr, tail, bucket);
    }
}

// Resumption from a checkpoint (ibip_invade_resume): cs_in holds the step at
// which each voxel was a centre in steps 1..k_done (0 if it was not). Every
// pore voxel that was a centre, a seed of Q0 or a face neighbour of a centre
// has been claimed; the claimed voxels that were not centres are the
// candidates of step k_done + 1 and go into the slices of their ranks (the
// order inside a slice never matters); the maximum of each earlier step is
// the rank of its centres. A value outside 0..k_done, or a centre on solid,
// sets *bad.
__global__ __launch_bounds__(256) void k_resume_seed(const uint8_t* __restrict__ inlets,
                                                     const int32_t* __restrict__ cs_in, int64_t k_done, uint32_t* key,
                                                     int32_t* state, uint32_t* M, int X, int Y, int Z, uint32_t* tail,
                                                     uint32_t* bucket, bool mask, uint32_t* bad) {
    const int64_t n = (int64_t)X * Y * Z;
    const int64_t v = (int64_t)blockIdx.x * 256 + threadIdx.x;
    const bool in = v < n;
    const uint32_t kv = in ? key[v] : 0u;
    const uint32_t rk = kv & kRankMask;
    const bool pore = rk != 0;
    const int32_t c = in ? cs_in[v] : 0;
    if (in) {
        state[v] = c;
        if (c < 0 || (int64_t)c > k_done || (c > 0 && !pore)) atomicOr(bad, 1u);
    }
    const bool popped = pore && c > 0 && (int64_t)c <= k_done;
    bool seed = false, touched = false;
    if (pore) {
        const int64_t yz = (int64_t)Y * Z;
        const int z = (int)(v % Z), y = (int)((v / Z) % Y), x = (int)(v / yz);
        seed = inlets[v] != 0;  // v itself is pore
        const bool inb[6] = {x > 0, x < X - 1, y > 0, y < Y - 1, z > 0, z < Z - 1};
        const int64_t off[6] = {-yz, yz, -(int64_t)Z, (int64_t)Z, -1, 1};
#pragma unroll
        for (int j = 0; j < 6; j++) {
            if (!inb[j]) continue;
            const int64_t u = v + off[j];
            seed |= inlets[u] != 0 && (!mask || (key[u] & kRankMask) != 0);
            touched |= cs_in[u] > 0;
        }
    }
    const bool claimed = popped || seed || touched;
    if (claimed) key[v] = kv | kClaim;
    if (popped) M[c - 1] = rk;  // every centre of a step holds the step's rank
    push_global(claimed && !popped, (uint32_t)v, rk, tail, bucket);
}

// ---------------------------------------------------------------------------
// The step loop: one workgroup.
// ---------------------------------------------------------------------------
struct LoopArgs {
    LoopState* st;
    uint32_t* head;
    uint32_t* tail;
    const uint32_t* val;
    uint32_t* bucket;
    int32_t* state;
    uint32_t* key;
    uint32_t* M;
    int X, Y, Z;
    uint32_t wide;    // steps with more centres go to the whole-GPU kernel
    uint32_t small;   // steps with at most this many centres run in wave 0 alone
    FastDiv divZ, divY;
    // a batch job's completion record in host memory (done, k, err), or null
    uint32_t* done = nullptr;
    // a served job's cancel flag in host memory, read every 1024 steps, or null
    const uint32_t* cancel = nullptr;
    // the occupancy bitmap of k_loop_global (more ranks than LDS holds), or null
    uint32_t* gbits = nullptr;
};

// true when the job's cancel flag is set (wave-uniform)
__device__ inline bool cancel_requested(const LoopArgs& a) {
    return a.cancel && __builtin_amdgcn_readfirstlane(
                           __hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) != 0u;
}

constexpr int kLoopThreads = 1024;
constexpr int kBitWords = (kMaxRanks >> 5) + 2;
constexpr int kSumWords = (kBitWords >> 5) + 1;
constexpr uint32_t kLog = 2048;  // entries of the per-step push log
constexpr uint32_t kRunCentres = 21;  // steps of at most two passes of 64 (centre, direction) pairs

struct LoopShared {
    uint32_t head[kMaxRanks + 1];
    uint32_t tail[kMaxRanks + 1 + 64];  // + one dummy word per lane (see slice_pos)
    uint32_t bits[kBitWords];   // rank r non-empty
    uint32_t sum[kSumWords];    // bits word w non-zero
    // pushes of the last two steps (voxel, rank), double-buffered
    uint32_t logu[2][kLog];
    uint32_t logr[2][kLog];
    uint32_t logn[2];           // pushes counted (more than kLog = log incomplete)
    uint32_t cl[kSmallRound];   // centres of a small step gathered from the log
    uint8_t clb[kSmallRound];   // their in-image neighbour bits
    // descriptor of a step run by all waves
    uint32_t d_exit, d_h, d_cnt, d_k, d_r, d_fromlog, d_sel, d_up;
};

__device__ inline uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

// in-image neighbour bits of voxel c, from its coordinates
__device__ inline uint32_t nb_of(uint32_t c, const LoopArgs& a) {
    const uint32_t t = fdiv(c, a.divZ), x = fdiv(t, a.divY);
    return nb_bits(x, t - x * (uint32_t)a.Y, c - t * (uint32_t)a.Z, a.X, a.Y, a.Z);
}


// Position of a push into the LDS slice of rank rr, and that slice's head.
// Every lane issues the atomic and the read: a lane that does not push adds 0
// to a dummy word of its own. (An LDS atomic under a lane condition makes the
// compiler wait for its result before the next one, serialising a lane's
// several pushes into one LDS round trip each.)
__device__ inline void slice_pos(LoopShared& s, bool push, uint32_t rr, uint32_t& pos, uint32_t& hd) {
    const uint32_t lane = threadIdx.x & 63;
    pos = atomicAdd(&s.tail[push ? rr : (uint32_t)kMaxRanks + 1u + lane], push ? 1u : 0u);
    hd = s.head[push ? rr : 0u];
}

__device__ inline void lds_set(LoopShared& s, uint32_t r) {
    atomicOr(&s.bits[r >> 5], 1u << (r & 31));
    atomicOr(&s.sum[r >> 10], 1u << ((r >> 5) & 31));
}

// highest set rank strictly below r (0 = none), with every loaded word made
// wave-uniform so the search runs on scalar branches. A summary bit may
// outlive its word (a rank bit cleared without a read-back of the word): such
// a word reads zero, its summary bit is dropped and the search goes on. Only
// wave 0 calls this, while no other wave touches the bitmap.
__device__ inline uint32_t lds_highest_below_uni(LoopShared& s, uint32_t r) {
    uint32_t w = r >> 5, b = r & 31;
    uint32_t m = uni(s.bits[w]) & ((1u << b) - 1u);
    if (m) return (w << 5) + 31 - __clz(m);
    uint32_t sw = w >> 5, sb = w & 31;
    uint32_t ms = uni(s.sum[sw]) & ((1u << sb) - 1u);
    for (;;) {
        while (ms) {
            const uint32_t wb = 31 - __clz(ms);
            const uint32_t ww = (sw << 5) + wb;
            const uint32_t bw = uni(s.bits[ww]);
            if (bw) return (ww << 5) + 31 - __clz(bw);
            ms &= ~(1u << wb);
            atomicAnd(&s.sum[sw], ~(1u << wb));
        }
        if (sw == 0) return 0;
        sw--;
        ms = uni(s.sum[sw]);
    }
}

// Maximum of v over the 64 lanes of a wave (every lane active), by DPP row
// shifts within rows of 16 lanes and row broadcasts across rows.
__device__ inline uint32_t wave_max_u32(uint32_t v) {
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, true));  // row_shr:1
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, true));  // row_shr:2
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, true));  // row_shr:4
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, true));  // row_shr:8
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false)); // row_bcast:15
    v = max(v, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false)); // row_bcast:31
    return __builtin_amdgcn_readlane(v, 63);
}

// After step r: clear the occupancy bit of r if its slice stayed empty. If a
// rank above r was pushed (`up`), the new maximum is the highest set bit,
// since every rank above r was empty when the step began; otherwise it is r
// itself if its slice refilled, else the highest non-empty rank below it.
// `refilled`: whether the step pushed into slice r (known from the pushes
// when wave 0 ran the step alone).
__device__ inline uint32_t next_top_known(LoopShared& s, uint32_t r, bool up, bool refilled, uint32_t R) {
    if (!refilled) {
        const uint32_t wv = uni(s.bits[r >> 5]) & ~(1u << (r & 31));
        s.bits[r >> 5] = wv;
        if (wv == 0) s.sum[r >> 10] = uni(s.sum[r >> 10]) & ~(1u << ((r >> 5) & 31));
    }
    if (up) return lds_highest_below_uni(s, R + 1);
    return refilled ? r : lds_highest_below_uni(s, r);
}

__device__ inline uint32_t next_top(LoopShared& s, uint32_t r, bool up, uint32_t R) {
    return next_top_known(s, r, up, uni(s.tail[r]) > uni(s.head[r]), R);
}

// Claims of a wide step (run over the whole GPU): each key is read first
// (from L2, not the CU cache, which atomics do not update) and the atomic
// goes only to voxels that read unclaimed pore. A voxel claimed earlier, or
// solid, costs a load instead of an atomic; the atomic still decides every
// race. Wide steps issue millions of claims and are bound by the atomic rate;
// steps run inside one workgroup are bound by latency, and the extra round
// trip made them slower, so they claim directly.
template <int N>
__device__ inline void claim_filtered(const uint32_t* key_ro, uint32_t* key, const int64_t (&uu)[N],
                                      const bool (&okd)[N], uint32_t c, uint32_t (&old)[N]) {
    uint32_t pre[N];
#pragma unroll
    for (int j = 0; j < N; j++)
        pre[j] = __hip_atomic_load(&key_ro[okd[j] ? uu[j] : (int64_t)c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
    for (int j = 0; j < N; j++) {
        const bool go = okd[j] && !(pre[j] & kClaim) && (pre[j] & kRankMask) != 0;
        old[j] = go ? atomicOr(&key[uu[j]], kClaim) : kClaim;
    }
}

// Make c a centre of step k and claim its unseen pore face neighbours: one
// atomicOr per neighbour sets the claim bit and returns the rank, so a claim
// costs one round trip; the six claims are in flight together. The claimed
// voxels are then appended to the slices of their ranks in LDS with one
// independent atomicAdd per push on the slice tail (no serial per-rank loop).
// Only the push that finds its slice empty (position == head) sets the
// occupancy bit, so the bitmap sees no same-address atomics. Push-log entries
// are reserved per wave: from the scalar running count `logn` when wave 0
// runs the step alone (kSingle), else with one LDS atomic per wave. Returns
// the largest rank this lane pushed (0 if none).
template <bool kSingle, int NC>
__device__ inline uint32_t expand_lds(const bool (&have)[NC], const uint32_t (&c)[NC], uint32_t k, const LoopArgs& a,
                                      LoopShared& s, uint32_t sel, uint32_t& logn) {
    constexpr int ND = 6 * NC;
    const int64_t yz = (int64_t)a.Y * a.Z;
    int64_t uu[ND];
    bool okd[ND];
#pragma unroll
    for (int q = 0; q < NC; q++) {
        int z = 0, y = 0, x = 0;
        if (have[q]) {
            a.state[c[q]] = (int32_t)k;
            const uint32_t t = fdiv(c[q], a.divZ);
            z = (int)(c[q] - t * (uint32_t)a.Z);
            x = (int)fdiv(t, a.divY);
            y = (int)(t - (uint32_t)x * (uint32_t)a.Y);
        }
        const int64_t cc = (int64_t)c[q];
        uu[6 * q + 0] = cc - yz; okd[6 * q + 0] = have[q] && x > 0;
        uu[6 * q + 1] = cc + yz; okd[6 * q + 1] = have[q] && x < a.X - 1;
        uu[6 * q + 2] = cc - a.Z; okd[6 * q + 2] = have[q] && y > 0;
        uu[6 * q + 3] = cc + a.Z; okd[6 * q + 3] = have[q] && y < a.Y - 1;
        uu[6 * q + 4] = cc - 1; okd[6 * q + 4] = have[q] && z > 0;
        uu[6 * q + 5] = cc + 1; okd[6 * q + 5] = have[q] && z < a.Z - 1;
    }
    uint32_t old[ND];
#pragma unroll
    for (int j = 0; j < ND; j++) old[j] = okd[j] ? atomicOr(&a.key[uu[j]], kClaim) : kClaim;
    bool won[ND];
    uint32_t rr[ND], pos[ND], hd[ND];
    uint32_t mymax = 0;
#pragma unroll
    for (int j = 0; j < ND; j++) {
        rr[j] = old[j] & kRankMask;
        won[j] = !(old[j] & kClaim) && rr[j] != 0;
        mymax = won[j] && rr[j] > mymax ? rr[j] : mymax;
    }
    // slice positions: independent LDS atomics, all in flight together, with
    // the slice heads read alongside
#pragma unroll
    for (int j = 0; j < ND; j++) {
        slice_pos(s, won[j], rr[j], pos[j], hd[j]);
    }
    // push-log entries
    uint64_t m[ND];
    uint32_t before[ND], total = 0;
#pragma unroll
    for (int j = 0; j < ND; j++) {
        m[j] = __ballot(won[j]);
        before[j] = total;
        total += (uint32_t)__popcll(m[j]);
    }
    uint32_t lbase = 0;
    if (total) {
        if (kSingle) {
            lbase = logn;
            logn += total;
        } else {
            uint32_t b = 0;
            if ((threadIdx.x & 63) == 0) b = atomicAdd(&s.logn[sel], total);
            lbase = __builtin_amdgcn_readlane(b, 0);
        }
    }
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int j = 0; j < ND; j++) {
        if (!won[j]) continue;
        a.bucket[pos[j]] = (uint32_t)uu[j];
        if (pos[j] == hd[j]) lds_set(s, rr[j]);
        const uint32_t li = lbase + before[j] + (uint32_t)__popcll(m[j] & lt);
        if (li < kLog) {
            s.logu[sel][li] = (uint32_t)uu[j];
            s.logr[sel][li] = old[j] & ~kClaim;  // rank and in-image neighbour bits
        }
    }
    return mymax;
}

// A step with at most kSmallRound centres, run by wave 0 alone. The centres
// sit in s.cl; each lane takes one (centre, direction) pair per pass of 64
// pairs. The direction becomes a stride and a bounds test by selects, not
// branches, so the claims of the first two passes (21 centres) are issued
// back to back and waited for once; steps with more centres run their further
// passes one at a time.
__device__ inline void claim_pair(uint32_t p, uint32_t np, uint32_t k, const LoopArgs& a, const LoopShared& s,
                                  uint32_t& old, uint32_t& u) {
    const uint32_t i = p * 64 + (threadIdx.x & 63);
    const bool act = i < np;
    const uint32_t ci = act ? i / 6u : 0u;
    const uint32_t dir = i - ci * 6u;
    // slot ci (0 on idle lanes) lies inside s.cl: the reads need no lane condition
    const uint32_t c = s.cl[ci];
    const uint32_t nb = s.clb[ci];  // the centre's in-image neighbours
    const uint32_t axis = dir >> 1;
    const bool up = dir & 1u;
    const uint32_t stride = axis == 0 ? (uint32_t)a.Y * (uint32_t)a.Z : axis == 1 ? (uint32_t)a.Z : 1u;
    const bool ok = act && ((nb >> dir) & 1u);
    u = up ? c + stride : c - stride;
    old = kClaim;
    if (ok) old = atomicOr(&a.key[u], kClaim);
    // stores go after the claims: a wait for the claims then leaves them in
    // flight. Every lane stores (the lanes of one centre the same value; an
    // idle lane that of centre 0, also a centre of this step), so the number
    // of memory operations after the claims is fixed.
    a.state[c] = (int32_t)k;
}

// Pairs of a wave-0 step, fixed per lane: pass p takes pair 64p + lane,
// that is centre (64p + lane) / 6 of the step's list and direction
// (64p + lane) % 6, with its neighbour bit and signed index offset. Three
// passes are 192 pairs, 32 whole centres: pass p + 3 takes the direction of
// pass p and the centre 32 further.
struct RunLane {
    uint32_t ci[3], bit[3];
    int32_t off[3];
};

__device__ inline RunLane run_lanes(const LoopArgs& a) {
    RunLane L;
#pragma unroll
    for (int p = 0; p < 3; p++) {
        const uint32_t i = (uint32_t)(p * 64) + (threadIdx.x & 63);
        const uint32_t d = i % 6u;
        const int32_t stride = d < 2 ? a.Y * a.Z : d < 4 ? a.Z : 1;
        L.ci[p] = i / 6u;
        L.bit[p] = 1u << d;
        L.off[p] = d & 1u ? stride : -stride;
    }
    return L;
}

// The claims of both passes of a run step of np / 6 centres listed in s.cl,
// as claim_pair with the pairs' constants from L: the four list reads are
// issued together (unconditionally: an idle lane reads slot 0), then the
// claims, then the state stores.
__device__ inline void claim_run(uint32_t np, uint32_t k, const LoopArgs& a, const LoopShared& s, const RunLane& L,
                                 uint32_t& o0, uint32_t& u0, uint32_t& o1, uint32_t& u1) {
    const uint32_t lane = threadIdx.x & 63;
    const bool act0 = lane < np, act1 = lane + 64u < np;
    const uint32_t ci0 = act0 ? L.ci[0] : 0u, ci1 = act1 ? L.ci[1] : 0u;
    const uint32_t c0 = s.cl[ci0], c1 = s.cl[ci1];
    const uint32_t nb0 = s.clb[ci0], nb1 = s.clb[ci1];
    const bool ok0 = act0 & ((nb0 & L.bit[0]) != 0u), ok1 = act1 & ((nb1 & L.bit[1]) != 0u);
    u0 = c0 + (uint32_t)L.off[0];
    u1 = c1 + (uint32_t)L.off[1];
    o0 = kClaim;
    o1 = kClaim;
    if (ok0) o0 = atomicOr(&a.key[u0], kClaim);
    if (ok1) o1 = atomicOr(&a.key[u1], kClaim);
    a.state[c0] = (int32_t)k;
    a.state[c1] = (int32_t)k;
}

// Rank of a won claim (0 if the claim lost or hit solid).
__device__ inline uint32_t won_rank(uint32_t old) {
    const uint32_t rr = old & kRankMask;
    return !(old & kClaim) && rr != 0 ? rr : 0u;
}

// Entries of the slice a step may pop next, read ahead. When a small step
// pushes nothing at or above the highest non-empty rank below its own
// (`below`), that rank is the next maximum and its centres come from the
// bucket in HBM: a global round trip ahead of the next claims. Reading them
// while the current step's claims are in flight takes it off the chain. The
// entries of a slice between its head and tail never change, so the next
// step takes them if its rank, head and tail are the ones read here.
struct SliceAhead {
    uint32_t r = 0, h = 0, t = 0;  // wave-uniform; r = 0: nothing read
    uint32_t c = 0;                // entry h + lane, clamped into the slice
};

// The load is issued in every case (entry 0 of the bucket when there is
// nothing to read): with a fixed number of memory operations after the claims,
// the wait for the claims leaves it in flight.
__device__ inline void read_ahead(const LoopArgs& a, const LoopShared& s, uint32_t below, SliceAhead& ah) {
    const uint32_t h = uni(s.head[below]), t = uni(s.tail[below]);
    const bool ok = below != 0 && t != h && t - h <= 64u;
    ah.r = ok ? below : 0u;
    ah.h = h;
    ah.t = t;
    ah.c = a.bucket[ok ? h + min((uint32_t)(threadIdx.x & 63), t - h - 1u) : 0u];
}

// Push of one (centre, direction) pair of a step of the run below, from the
// won rank w (0: nothing to push) and the neighbour bits nb of the claimed
// voxel u, into the LDS slice of its rank; a push of rank rd (the next
// step's rank, when every live entry of its slice comes from this step) is
// also listed in s.cl for the next step. The bucket store is issued by every
// lane: one without a push writes the step's rank r into M[k - 1], which
// holds it anyway. (A store under a lane condition leaves the number of
// memory operations in flight unknown to the compiler, which then waits for
// all of them wherever it needs a load's result, as the next step's centres
// read ahead.)
__device__ inline void push_won(uint32_t w, uint32_t u, uint32_t nb, const LoopArgs& a, LoopShared& s,
                                uint32_t rd, uint32_t& dn, uint32_t k, uint32_t r) {
    const bool won = w != 0;
    uint32_t pos, hd;
    slice_pos(s, won, w, pos, hd);
    const bool nx = won && w == rd;
    const uint64_t mn = __ballot(nx);
    const uint32_t di = dn + lanes_below(mn);
    dn += (uint32_t)__popcll(mn);
    *(won ? &a.bucket[pos] : &a.M[k - 1]) = won ? u : r;
    if (won) {
        if (pos == hd) lds_set(s, w);
        if (nx && di < kSmallRound) {
            s.cl[di] = u;
            s.clb[di] = (uint8_t)nb;
        }
    }
}

// One small step of more than kRunCentres centres (3 to 12 passes), wave 0
// alone; returns the next maximum rank: the highest pushed rank if above r
// (every rank above r was empty), else r if its slice refilled, else the
// larger of the highest pushed rank and the highest non-empty rank below r
// (`below`, found while the claims are in flight). Every pass's claims are
// issued first, four passes at a time with their list reads together; once
// they are all back the pushes go four passes at a time, their slice-tail
// atomics together, and are logged for the next step.
__device__ inline uint32_t small_step(uint32_t cnt, uint32_t k, uint32_t r, uint32_t t, const LoopArgs& a,
                                      LoopShared& s, uint32_t sel, uint32_t& logn, SliceAhead& ah,
                                      const RunLane& L) {
    constexpr int kMaxPasses = (6 * kSmallRound + 63) / 64;  // 12
    const uint32_t np = 6 * cnt;
    const uint32_t passes = (np + 63) >> 6;
    const uint32_t lane = threadIdx.x & 63;
    uint32_t o[kMaxPasses], u[kMaxPasses];
#pragma unroll
    for (int g = 0; g < kMaxPasses; g += 4) {
        o[g] = o[g + 1] = o[g + 2] = o[g + 3] = kClaim;
        u[g] = u[g + 1] = u[g + 2] = u[g + 3] = 0;
        if ((uint32_t)g < passes) {
            uint32_t cc[4], nbv[4];
            bool act[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int p = g + j;
                act[j] = (uint32_t)(64 * p) + lane < np;
                const uint32_t ci = act[j] ? L.ci[p % 3] + 32u * (uint32_t)(p / 3) : 0u;
                cc[j] = s.cl[ci];
                nbv[j] = s.clb[ci];
            }
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int p = g + j;
                const bool ok = act[j] & ((nbv[j] & L.bit[p % 3]) != 0u);
                u[p] = cc[j] + (uint32_t)L.off[p % 3];
                if (ok) o[p] = atomicOr(&a.key[u[p]], kClaim);
            }
            // (every lane stores: an idle lane that of centre 0)
#pragma unroll
            for (int j = 0; j < 4; j++) a.state[cc[j]] = (int32_t)k;
        }
    }
    // pop slice r (its head moves to tail t) once the claims are out
    s.head[r] = t;
    const uint32_t below = lds_highest_below_uni(s, r);
    read_ahead(a, s, below, ah);
    uint32_t lm = 0;
    bool same = false;
    const uint64_t lt = lanemask_lt();
#pragma unroll
    for (int g = 0; g < kMaxPasses; g += 4) {
        if ((uint32_t)g < passes) {
            uint32_t w[4], pos[4], hd[4];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                w[j] = won_rank(o[g + j]);
                lm = max(lm, w[j]);
                same |= w[j] == r;
            }
#pragma unroll
            for (int j = 0; j < 4; j++) slice_pos(s, w[j] != 0, w[j], pos[j], hd[j]);
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const bool won = w[j] != 0;
                const uint64_t m = __ballot(won);
                const uint32_t li = logn + (uint32_t)__popcll(m & lt);
                logn += (uint32_t)__popcll(m);
                // (every lane stores, as in push_won)
                *(won ? &a.bucket[pos[j]] : &a.M[k - 1]) = won ? u[g + j] : r;
                if (won) {
                    if (pos[j] == hd[j]) lds_set(s, w[j]);
                    if (li < kLog) {
                        s.logu[sel][li] = u[g + j];
                        s.logr[sel][li] = o[g + j] & ~kClaim;  // rank and in-image neighbour bits
                    }
                }
            }
        }
    }
    const uint32_t pmax = wave_max_u32(lm);
    const bool refilled = __ballot(same) != 0;
    if (!refilled) atomicAnd(&s.bits[r >> 5], ~(1u << (r & 31)));
    return pmax > r ? pmax : refilled ? r : max(below, pmax);
}

// Control flow: the step decisions run in all 64 lanes of wave 0 on values
// made uniform with readfirstlane (duplicate stores of one value from several
// lanes are harmless). Wave 0 runs steps of up to `small` centres alone, with
// no barrier; larger steps are run by all waves between two barriers, and the
// barriers stay in wave-uniform control flow. (A lane-divergent `tid == 0`
// region in a barrier loop can be restructured so that lanes 1..63 of wave 0
// loop back to a barrier while lane 0 waits outside the loop.)
//
// When the new maximum rank is at least the previous step's, its live entries
// are exactly the previous step's pushes of that rank (the slice was either
// popped empty by that step or empty before it), so they are read from the
// LDS push log instead of global memory, if the log did not overflow.
// kCancel: the loop checks the job's cancel flag every 1024 steps (served
// jobs only; the check costs the other paths about 3 % of their loop time)
template <bool kCancel>
__device__ inline void loop_body(const LoopArgs& a, LoopShared& s) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const bool wave0 = uni((uint32_t)tid >> 6) == 0;
    const uint32_t R = a.st->R;
    // an image without solid, or with more distinct distances than the LDS
    // tables hold, is rejected before anything is read (its setup kernels
    // skipped the offending values)
    if (!a.st->solid_seen || R > (uint32_t)kMaxRanks) {
        if (tid == 0) {
            a.st->err = !a.st->solid_seen ? 2u : 3u;
            a.st->status = LS_DONE;
        }
        return;
    }
    for (uint32_t q = tid; q <= R; q += kLoopThreads) {
        s.head[q] = a.head[q];
        s.tail[q] = a.tail[q];
    }
    for (int w = tid; w < kBitWords; w += kLoopThreads) s.bits[w] = 0;
    for (int w = tid; w < kSumWords; w += kLoopThreads) s.sum[w] = 0;
    if (tid < 2) s.logn[tid] = 0;
    __syncthreads();
    for (uint32_t q = 1 + tid; q <= R; q += kLoopThreads)
        if (s.tail[q] > s.head[q]) lds_set(s, q);
    __syncthreads();
    const int64_t max_steps = a.st->max_steps;
    const uint32_t n_pore = a.st->n_pore;
    // one bound for both stops: steps past max_steps, or more steps than pore
    // voxels (every step takes at least one new pore voxel)
    const uint32_t klim =
        max_steps > 0 && max_steps < (int64_t)n_pore ? (uint32_t)max_steps : n_pore;
    // driver state, live in wave 0
    uint32_t r = 0, k = 0, prev_r = 0, sel = 0, nlog = 0, npop = 0;
    bool log_ok = false, direct = false;
    SliceAhead ah;
    const RunLane L = run_lanes(a);
    if (wave0) {
        r = lds_highest_below_uni(s, R + 1);
        k = uni(a.st->k);
    }
    for (;;) {
        if (wave0) {
            for (;;) {
                const bool cancelled = kCancel && r != 0 && k <= klim && (k & 1023u) == 0 && cancel_requested(a);
                if (r == 0 || k > klim || cancelled) {
                    if (r == 0) {
                        a.st->status = LS_DONE;
                    } else if (k > n_pore) {
                        // more steps than pore voxels means corrupted state; stop
                        // instead of looping
                        a.st->err = 1;
                        a.st->status = LS_DONE;
                    } else if (cancelled) {
                        a.st->status = LS_CANCEL;
                    } else {
                        a.st->status = LS_MAXSTEPS;
                    }
                    s.d_exit = 1;
                    break;
                }
                const uint32_t h = uni(s.head[r]), t = uni(s.tail[r]);
                const uint32_t cnt = t - h;
                const bool fromlog = log_ok && (direct || r >= prev_r);
                if (cnt > a.small) {
                    s.head[r] = t;
                    a.M[k - 1] = r;  // rank; k_rank_to_value turns it into dt2 after the loop
                    if (cnt > a.wide) {  // its centres are counted by the host
                        a.st->big_r = r;
                        a.st->big_h = h;
                        a.st->big_t = t;
                        a.st->big_k = k;
                        a.st->status = LS_WIDE;
                        k = k + 1;
                        s.d_exit = 1;
                        break;
                    }
                    npop += cnt;
                    s.logn[sel] = nlog;    // the log this step may gather from
                    s.logn[sel ^ 1u] = 0;  // the waves count their pushes there
                    s.d_up = 0;
                    s.d_exit = 0;
                    s.d_h = h;
                    s.d_cnt = cnt;
                    s.d_k = k;
                    s.d_r = r;
                    s.d_fromlog = fromlog ? 1u : 0u;
                    s.d_sel = sel;
                    break;
                }
                npop += cnt;
                const uint32_t nsel = sel ^ 1u;
                // a small step, wave 0 alone: its centres are listed in s.cl by the
                // previous step, or gathered there from the log or the bucket
                uint32_t ln = 0;  // entries in the new push log
                if (direct) {
                } else if (fromlog) {
                    const uint32_t n = nlog;
                    uint32_t got = 0;
                    for (uint32_t b0 = 0; b0 < n; b0 += 64) {
                        const uint32_t i = b0 + lane;
                        const uint32_t lr = i < n ? s.logr[sel][i] : 0u;
                        const bool match = (lr & kRankMask) == r;
                        const uint64_t mm = __ballot(match);
                        const uint32_t slot = got + (uint32_t)__popcll(mm & lanemask_lt());
                        if (match && slot < kSmallRound) {
                            s.cl[slot] = s.logu[sel][i];
                            s.clb[slot] = (uint8_t)(lr >> kNbShift);
                        }
                        got += (uint32_t)__popcll(mm);
                    }
                } else {
                    // unconditional loads (clamped into the slice) and LDS stores:
                    // entries past cnt are never read. A load under a lane
                    // condition would leave its register pending past this
                    // block, and the compiler would then wait for every
                    // outstanding store before the claims.
                    // (the bucket holds voxel indices only: their neighbour bits
                    // come from their coordinates)
                    // (the entries read ahead by the previous step, if they are
                    // this slice's: same rank, head and tail)
                    uint32_t c0 = ah.c;
                    if (!(ah.r == r && ah.h == h && ah.t == t)) c0 = a.bucket[h + min((uint32_t)lane, cnt - 1u)];
                    s.cl[lane] = c0;
                    s.clb[lane] = (uint8_t)nb_of(c0, a);
                    if (cnt > 64) {
                        const uint32_t c1 = a.bucket[h + min((uint32_t)lane + 64u, cnt - 1u)];
                        s.cl[lane + 64] = c1;
                        s.clb[lane + 64] = (uint8_t)nb_of(c1, a);
                    }
                }
                if (cnt <= kRunCentres) {
                    // A run of steps of at most kRunCentres centres (at most
                    // two passes of 64 pairs). Once a step's claims return and
                    // the next maximum is decided, the next step's centres are
                    // often known already: this step's pushes of that rank
                    // (`direct`: they are every live entry of its slice), or
                    // the entries of the slice below, read ahead while the
                    // claims were in flight, if this step pushed none of that
                    // rank. The run then lists them in s.cl and issues the
                    // next step's claims at once; while they are in flight it
                    // does this step's pushes, pops the next slice, finds the
                    // rank below it and reads that slice's entries ahead. The
                    // run ends at a step whose successor is not known that
                    // way or has more centres, at the step limit, or (a job
                    // that can be cancelled) every 1024 steps; the last step
                    // pushes as a step of the general path and lists its
                    // direct pushes in s.cl for it.
                    // (the second pass is issued in every step, with no lane
                    // active in a step of at most 10 centres: its claim words
                    // then stay in the same registers from step to step)
                    uint32_t c1 = cnt;
                    uint32_t o0, u0, o1, u1;
                    claim_run(6 * c1, k, a, s, L, o0, u0, o1, u1);
                    s.head[r] = t;
                    uint32_t below = lds_highest_below_uni(s, r);
                    read_ahead(a, s, below, ah);
                    for (;;) {
                        // the claim words are not used past this point: the empty
                        // asm makes the compiler take their ranks and neighbour
                        // bits here, so the next step's claims can reuse their
                        // registers (a copy into them would wait for those claims)
                        uint32_t w0 = won_rank(o0), w1 = won_rank(o1);
                        uint32_t b0 = o0 >> kNbShift, b1 = o1 >> kNbShift;
                        asm volatile("" : "+v"(w0), "+v"(w1), "+v"(b0), "+v"(b1));
                        const uint32_t pmax = wave_max_u32(max(w0, w1));
                        const bool refilled = __ballot(w0 == r || w1 == r) != 0;
                        if (!refilled) atomicAnd(&s.bits[r >> 5], ~(1u << (r & 31)));
                        const uint32_t rn = pmax > r ? pmax : refilled ? r : max(below, pmax);
                        const bool dir = rn != 0 && rn != below;
                        // won pushes of rank rn (a lane that won nothing has w = 0)
                        const bool x0 = rn != 0 && w0 == rn, x1 = rn != 0 && w1 == rn;
                        const uint64_t m0 = __ballot(x0), m1 = __ballot(x1);
                        const uint32_t n0 = (uint32_t)__popcll(m0);
                        const uint32_t nrn = n0 + (uint32_t)__popcll(m1);
                        const bool hit = !dir && rn != 0 && rn == ah.r && nrn == 0;
                        const uint32_t cn = dir ? nrn : hit ? ah.t - ah.h : 0u;
                        const bool go = cn != 0 && cn <= kRunCentres && k + 1 <= klim &&
                                        !(kCancel && ((k + 1) & 1023u) == 0);
                        if (go) {
                            if (dir) {
                                if (x0) {
                                    const uint32_t i = lanes_below(m0);
                                    s.cl[i] = u0;
                                    s.clb[i] = (uint8_t)b0;
                                }
                                if (x1) {
                                    const uint32_t i = n0 + lanes_below(m1);
                                    s.cl[i] = u1;
                                    s.clb[i] = (uint8_t)b1;
                                }
                            } else if ((uint32_t)lane < cn) {
                                s.cl[lane] = ah.c;
                                s.clb[lane] = (uint8_t)nb_of(ah.c, a);
                            }
                            uint32_t p0, v0, p1, v1;
                            claim_run(6 * cn, k + 1, a, s, L, p0, v0, p1, v1);
                            // This step's pushes: slice positions, and the
                            // occupancy bit of every pushed rank (a step pushes
                            // few voxels, so few same-address atomics), which
                            // the search for the rank below the next one reads;
                            // the bucket stores once the positions are back,
                            // ahead of the read-ahead, which may read them.
                            const bool g0 = w0 != 0, g1 = w1 != 0;
                            uint32_t q0, h0, q1, h1;
                            slice_pos(s, g0, w0, q0, h0);
                            slice_pos(s, g1, w1, q1, h1);
                            const uint32_t hrn = s.head[rn];  // (the next slice was empty: its tail is hrn + nrn)
                            if (g0) lds_set(s, w0);
                            if (g1) lds_set(s, w1);
                            const uint32_t nbelow = lds_highest_below_uni(s, rn);
                            const uint32_t t_next = dir ? hrn + nrn : ah.t;
                            *(g0 ? &a.bucket[q0] : &a.M[k - 1]) = g0 ? u0 : r;
                            *(g1 ? &a.bucket[q1] : &a.M[k - 1]) = g1 ? u1 : r;
                            a.M[k - 1] = r;
                            read_ahead(a, s, nbelow, ah);
                            s.head[rn] = t_next;  // the pop of the next step
                            prev_r = r;
                            r = rn;
                            below = nbelow;
                            k = k + 1;
                            npop += cn;
                            c1 = cn;
                            o0 = p0;
                            u0 = v0;
                            o1 = p1;
                            u1 = v1;
                            continue;
                        }
                        uint32_t dn = 0;
                        const uint32_t rd = dir ? rn : 0u;
                        push_won(w0, u0, b0, a, s, rd, dn, k, r);
                        if (c1 > 10) push_won(w1, u1, b1, a, s, rd, dn, k, r);
                        a.M[k - 1] = r;
                        prev_r = r;
                        r = rn;
                        k = k + 1;
                        direct = dir;
                        break;
                    }
                    log_ok = false;  // no push log was written
                    nlog = kLog + 1;
                    continue;
                }
                const uint32_t rn = small_step(cnt, k, r, t, a, s, nsel, ln, ah, L);
                a.M[k - 1] = r;
                prev_r = r;
                r = rn;
                direct = false;
                k = k + 1;
                sel = nsel;
                log_ok = ln <= kLog;
                nlog = ln;
            }
        }
        __syncthreads();
        if (uni(s.d_exit)) break;
        {
            // a step with many centres, all waves
            const uint32_t h = uni(s.d_h), cnt = uni(s.d_cnt), kk = uni(s.d_k), rr0 = uni(s.d_r);
            const uint32_t osel = uni(s.d_sel), nsel = osel ^ 1u;
            uint32_t unused = 0, lm = 0;
            if (uni(s.d_fromlog)) {
                const uint32_t n = uni(s.logn[osel]);
                for (uint32_t b0 = 0; b0 < n; b0 += kLoopThreads) {
                    const uint32_t i = b0 + tid;
                    bool have = false;
                    uint32_t c = 0;
                    if (i < n) {
                        have = (s.logr[osel][i] & kRankMask) == rr0;
                        c = s.logu[osel][i];
                    }
                    const bool hv[1] = {have};
                    const uint32_t cv[1] = {c};
                    const uint32_t m = expand_lds<false, 1>(hv, cv, kk, a, s, nsel, unused);
                    lm = m > lm ? m : lm;
                }
            } else {
                for (uint32_t b0 = 0; b0 < cnt; b0 += kLoopThreads) {
                    const uint32_t i = b0 + tid;
                    const bool have = i < cnt;
                    const bool hv[1] = {have};
                    const uint32_t cv[1] = {have ? a.bucket[h + i] : 0u};
                    const uint32_t m = expand_lds<false, 1>(hv, cv, kk, a, s, nsel, unused);
                    lm = m > lm ? m : lm;
                }
            }
            if (__ballot(lm > rr0) != 0 && lane == 0) s.d_up = 1;
        }
        __syncthreads();
        if (wave0) {
            const uint32_t r_done = r;
            r = next_top(s, r, uni(s.d_up) != 0, R);
            prev_r = r_done;
            direct = false;
            k = k + 1;
            sel ^= 1u;
            nlog = uni(s.logn[sel]);
            log_ok = nlog <= kLog;
        }
    }
    if (wave0) {
        a.st->k = k;
        a.st->popped = uni(a.st->popped) + npop;
    }
    for (uint32_t q = tid; q <= R; q += kLoopThreads) {
        a.head[q] = s.head[q];
        a.tail[q] = s.tail[q];
    }
    if (a.done) {
        // a batch job: tell the host, which starts the job's post-processing
        // (or, after a stop at a wide step, runs that step over the whole GPU
        // and resumes the job's loop) while other jobs' loops still run. The barrier orders every
        // thread's writes before thread 0's fence, which makes them visible
        // before the record; the record's fields precede its flag.
        __syncthreads();
        if (tid == 0) {
            __threadfence_system();
            a.done[1] = k;
            a.done[2] = a.st->err;
            a.done[3] = a.st->status;
            __threadfence_system();
            a.done[0] = 1u;
        }
    }
}

// The host queues each launch before it knows whether the previous one
// finished the loop: a launch after the end does nothing.
template <bool kCancel>
__global__ __launch_bounds__(kLoopThreads) void k_loop(LoopArgs a) {
    __shared__ LoopShared s;
    const uint32_t status = a.st->status;
    if (status != LS_RUN && status != LS_WIDE) return;
    loop_body<kCancel>(a, s);
}

// Many images in one launch: workgroup j runs the whole step loop of job j
// (jobs are ordered largest first, so the longest loops start first).
template <bool kCancel>
__global__ __launch_bounds__(kLoopThreads) void k_loop_batch(const LoopArgs* __restrict__ all) {
    __shared__ LoopShared s;
    const LoopArgs a = all[blockIdx.x];
    loop_body<kCancel>(a, s);
}

// ---------------------------------------------------------------------------
// The step loop for images with more distinct distance values than the LDS
// tables hold (R > kMaxRanks). The same steps on the slice tables in global
// memory, with a two-level occupancy bitmap there (bits: rank r non-empty;
// sum: bits word w non-zero), rebuilt from the tables at every launch: every
// step is run by all waves between barriers, thread 0 takes the decisions.
// Slices and the bitmap are updated with atomics and read with device-scope
// loads; each pop is followed by a barrier before its slice grows again.
// ---------------------------------------------------------------------------
struct GlobalLoopShared {
    uint32_t exit, r, k, h, t, up, refill;
};

__device__ inline uint32_t gload(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline void gbits_set(uint32_t* bits, uint32_t* sum, uint32_t r) {
    atomicOr(&bits[r >> 5], 1u << (r & 31));
    atomicOr(&sum[r >> 10], 1u << ((r >> 5) & 31));
}

// highest set rank strictly below r (0 = none); a summary bit whose word
// reads zero is dropped on the way (thread 0 only)
__device__ inline uint32_t gbits_highest_below(uint32_t* bits, uint32_t* sum, uint32_t r) {
    uint32_t w = r >> 5;
    const uint32_t m = gload(&bits[w]) & ((1u << (r & 31)) - 1u);
    if (m) return (w << 5) + 31 - __clz(m);
    uint32_t sw = w >> 5;
    uint32_t ms = gload(&sum[sw]) & ((1u << (w & 31)) - 1u);
    for (;;) {
        while (ms) {
            const uint32_t wb = 31 - __clz(ms);
            const uint32_t ww = (sw << 5) + wb;
            const uint32_t bw = gload(&bits[ww]);
            if (bw) return (ww << 5) + 31 - __clz(bw);
            ms &= ~(1u << wb);
            atomicAnd(&sum[sw], ~(1u << wb));
        }
        if (sw == 0) return 0;
        sw--;
        ms = gload(&sum[sw]);
    }
}

template <bool kCancel>
__global__ __launch_bounds__(kLoopThreads) void k_loop_global(LoopArgs a) {
    __shared__ GlobalLoopShared s;
    const int tid = threadIdx.x;
    const uint32_t status0 = a.st->status;
    if (status0 != LS_RUN && status0 != LS_WIDE) return;
    const uint32_t R = a.st->R;
    uint32_t* bits = a.gbits;
    const uint32_t nbw = (R >> 5) + 2;
    uint32_t* sum = a.gbits + nbw;
    const uint32_t nsw = (nbw >> 5) + 2;
    for (uint32_t w = tid; w < nbw; w += kLoopThreads) bits[w] = 0;
    for (uint32_t w = tid; w < nsw; w += kLoopThreads) sum[w] = 0;
    __syncthreads();
    for (uint32_t q = 1 + tid; q <= R; q += kLoopThreads)
        if (gload(&a.tail[q]) > a.head[q]) gbits_set(bits, sum, q);
    __syncthreads();
    const int64_t max_steps = a.st->max_steps;
    const uint32_t n_pore = a.st->n_pore;
    const uint32_t klim = max_steps > 0 && max_steps < (int64_t)n_pore ? (uint32_t)max_steps : n_pore;
    uint32_t npop = 0;  // thread 0
    // thread 0: start step k at rank r, or stop (exit set)
    auto decide = [&](uint32_t r, uint32_t k) {
        const bool cancelled = kCancel && r != 0 && k <= klim && (k & 1023u) == 0 && cancel_requested(a);
        s.exit = 1;
        s.k = k;
        if (r == 0 || k > klim || cancelled) {
            if (r == 0) {
                a.st->status = LS_DONE;
            } else if (k > n_pore) {
                a.st->err = 1;
                a.st->status = LS_DONE;
            } else {
                a.st->status = cancelled ? LS_CANCEL : LS_MAXSTEPS;
            }
            return;
        }
        const uint32_t h = a.head[r], t = gload(&a.tail[r]);
        a.head[r] = t;
        a.M[k - 1] = r;  // rank; k_rank_to_value turns it into dt2 after the loop
        if (t - h > a.wide) {  // its centres are counted by the host
            a.st->big_r = r;
            a.st->big_h = h;
            a.st->big_t = t;
            a.st->big_k = k;
            a.st->status = LS_WIDE;
            s.k = k + 1;
            return;
        }
        npop += t - h;
        s.r = r;
        s.h = h;
        s.t = t;
        s.up = 0;
        s.refill = 0;
        s.exit = 0;
    };
    if (tid == 0) decide(gbits_highest_below(bits, sum, R + 1), a.st->k);
    __syncthreads();
    const int64_t yz = (int64_t)a.Y * a.Z;
    while (!uni(s.exit)) {
        const uint32_t r = uni(s.r), k = uni(s.k), h = uni(s.h), cnt = uni(s.t) - h;
        for (uint32_t i = tid; i < cnt; i += kLoopThreads) {
            const uint32_t c = a.bucket[h + i];
            a.state[c] = (int32_t)k;
            const uint32_t tt = fdiv(c, a.divZ);
            const int z = (int)(c - tt * (uint32_t)a.Z);
            const int x = (int)fdiv(tt, a.divY);
            const int y = (int)(tt - (uint32_t)x * (uint32_t)a.Y);
            const int64_t uu[6] = {(int64_t)c - yz, (int64_t)c + yz, (int64_t)c - a.Z, (int64_t)c + a.Z,
                                   (int64_t)c - 1, (int64_t)c + 1};
            const bool okd[6] = {x > 0, x < a.X - 1, y > 0, y < a.Y - 1, z > 0, z < a.Z - 1};
            uint32_t old[6];
#pragma unroll
            for (int j = 0; j < 6; j++) old[j] = okd[j] ? atomicOr(&a.key[uu[j]], kClaim) : kClaim;
#pragma unroll
            for (int j = 0; j < 6; j++) {
                const uint32_t rr = won_rank(old[j]);
                if (!rr) continue;
                const uint32_t pos = atomicAdd(&a.tail[rr], 1u);
                a.bucket[pos] = (uint32_t)uu[j];
                // the push that finds its slice empty marks it non-empty
                // (slice heads other than r's do not move during the step)
                if (pos == a.head[rr]) gbits_set(bits, sum, rr);
                if (rr > r) atomicMax(&s.up, rr);
                else if (rr == r) s.refill = 1;
            }
        }
        __syncthreads();
        if (tid == 0) {
            // every rank above r was empty when the step began: a push above r
            // makes its largest rank the maximum; else r if its slice refilled,
            // else the highest non-empty rank below r
            if (!s.refill) atomicAnd(&bits[r >> 5], ~(1u << (r & 31)));  // slice r stayed empty
            const uint32_t rn = s.up > r ? s.up : s.refill ? r : gbits_highest_below(bits, sum, r);
            decide(rn, k + 1);
        }
        __syncthreads();
    }
    if (tid == 0) {
        a.st->k = s.k;
        a.st->popped = a.st->popped + npop;
    }
    if (a.done) {
        // a batch job's completion record, as in loop_body
        __syncthreads();
        if (tid == 0) {
            __threadfence_system();
            a.done[1] = s.k;
            a.done[2] = a.st->err;
            a.done[3] = a.st->status;
            __threadfence_system();
            a.done[0] = 1u;
        }
    }
}

// One step with many centres, spread over the whole GPU. Claims as in the
// loop (filtered by a read of the key first). The pushes of a block are
// counted per rank in LDS, each rank then takes one slice-tail atomic per
// block, and every push lands at that base plus its place in the block's
// count: slice tails are few and hot, and one atomic per wave and rank
// queued thousands of atomics on each of them.
// It is queued after every loop launch and does nothing unless that launch
// stopped at a wide step.
// With more ranks than its LDS counts hold, a block pushes with one slice-tail
// atomic per wave and distinct rank instead.
__global__ __launch_bounds__(256) void k_wide(LoopArgs a) {
    __shared__ uint32_t lcnt[kMaxRanks + 1];  // per rank: the block's pushes, then their base
    if (a.st->status != LS_WIDE) return;
    const uint32_t h = a.st->big_h, t = a.st->big_t, k = a.st->big_k, R = a.st->R;
    const bool lds = R <= (uint32_t)kMaxRanks;
    const uint32_t cnt = t - h;
    const uint32_t stride = gridDim.x * 256;
    const uint32_t ntrip = (cnt + stride - 1) / stride;
    const int64_t yz = (int64_t)a.Y * a.Z;
    for (uint32_t it = 0; it < ntrip; it++) {
        if (lds) {
            for (uint32_t q = threadIdx.x; q <= R; q += 256) lcnt[q] = 0;
            __syncthreads();
        }
        const uint32_t i = it * stride + blockIdx.x * 256 + threadIdx.x;
        const bool have = i < cnt;
        const uint32_t c = have ? a.bucket[h + i] : 0u;
        int z = 0, y = 0, x = 0;
        if (have) {
            a.state[c] = (int32_t)k;
            const uint32_t tt = fdiv(c, a.divZ);
            z = (int)(c - tt * (uint32_t)a.Z);
            x = (int)fdiv(tt, a.divY);
            y = (int)(tt - (uint32_t)x * (uint32_t)a.Y);
        }
        const int64_t uu[6] = {(int64_t)c - yz, (int64_t)c + yz, (int64_t)c - a.Z, (int64_t)c + a.Z,
                               (int64_t)c - 1, (int64_t)c + 1};
        const bool okd[6] = {have && x > 0, have && x < a.X - 1, have && y > 0, have && y < a.Y - 1,
                             have && z > 0, have && z < a.Z - 1};
        uint32_t old[6];
        claim_filtered<6>(a.key, a.key, uu, okd, c, old);
        uint32_t rr[6], off[6];
#pragma unroll
        for (int j = 0; j < 6; j++) {
            rr[j] = old[j] & kRankMask;
            if ((old[j] & kClaim) || rr[j] > R) rr[j] = 0;  // 0: no push (ranks above R do not occur)
        }
        if (!lds) {
#pragma unroll
            for (int j = 0; j < 6; j++) push_global(rr[j] != 0, (uint32_t)uu[j], rr[j], a.tail, a.bucket);
            continue;
        }
#pragma unroll
        for (int j = 0; j < 6; j++) off[j] = rr[j] ? atomicAdd(&lcnt[rr[j]], 1u) : 0u;
        __syncthreads();
        for (uint32_t q = threadIdx.x; q <= R; q += 256) {
            const uint32_t nq = lcnt[q];
            if (nq) lcnt[q] = atomicAdd(&a.tail[q], nq);
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < 6; j++)
            if (rr[j]) a.bucket[lcnt[rr[j]] + off[j]] = (uint32_t)uu[j];
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Sphere insertion
// ---------------------------------------------------------------------------
struct PaintArgs {
    const int32_t* state;
    const uint32_t* key;
    const uint32_t* val;
    int32_t* seq;
    uint32_t* full;
    uint32_t* n_full;
    int X, Y, Z;
    bool integer_ball;  // footnote 1's integer sphere instead of the strict ball
    FastDiv divZ, divY;  // voxel index -> coordinates (indices fit 31 bits)
    // the centres of steps k_lo..k_hi only (insertion is order-free, so the
    // steps can be inserted in passes); the full-ball list from *full_lo on
    int32_t k_lo = 1, k_hi = INT_MAX;
    const uint32_t* full_lo = nullptr;
    // leave the first XCD to the step loop: workgroups b with b % 8 == 0 (the
    // ones dispatched to XCD 0) return at once and the others take all the
    // work (a pass run while the loop's single workgroup, on XCD 0, runs)
    bool skip_xcd0 = false;
};

// The workgroup's index among those that take work (all of them, or the ones
// outside XCD 0), and their number; -1 for a workgroup that takes none.
__device__ inline int64_t paint_block(const PaintArgs& a, int64_t& nblocks) {
    if (!a.skip_xcd0) {
        nblocks = gridDim.x;
        return blockIdx.x;
    }
    nblocks = (int64_t)(gridDim.x >> 3) * 7;
    if ((blockIdx.x & 7u) == 0) return -1;
    return (int64_t)(blockIdx.x >> 3) * 7 + (blockIdx.x & 7u) - 1;
}

// Coordinates of voxel c (c < 2^31) by two multiplicative divisions.
__device__ inline void coords(uint32_t c, const PaintArgs& a, int& x, int& y, int& z) {
    const uint32_t t = fdiv(c, a.divZ);
    z = (int)(c - t * (uint32_t)a.Z);
    const uint32_t xx = fdiv(t, a.divY);
    y = (int)(t - xx * (uint32_t)a.Y);
    x = (int)xx;
}

// The painted ball of a centre of squared distance m is {|o|^2 < ball_m(m)}:
// m itself (the strict ball), or floor(sqrt(m))^2 + 1, i.e. the integer sphere
// {|o|^2 <= floor(sqrt(m))^2}. The integer ball can reach solid voxels when m
// is a perfect square; they hold -1, below every step, so atomicMin leaves
// them. The shell trick holds for any non-decreasing ball_m.
__device__ inline uint32_t ball_m(const PaintArgs& a, uint32_t m) {
    if (!a.integer_ball) return m;
    const uint32_t q = isqrt_u32(m);
    return q * q + 1;
}

// Stamps go out in groups of kStampGroup: the current values of the whole
// group are loaded together (a slot with nothing to stamp loads a valid
// address instead of branching), then an atomicMin, whose result is not
// used, goes only where the value is still larger. Most stamps land on
// voxels that already hold a smaller step, so the loads save L2 atomics; one
// load per stamp taken in turn would cost a round trip each.
constexpr int kStampGroup = 4;

__device__ inline void stamp_group(int32_t* seq, const uint32_t (&v)[kStampGroup], const bool (&ok)[kStampGroup],
                                   int32_t k) {
    int32_t cur[kStampGroup];
#pragma unroll
    for (int t = 0; t < kStampGroup; t++) cur[t] = seq[v[t]];
#pragma unroll
    for (int t = 0; t < kStampGroup; t++)
        if (ok[t] && cur[t] > k) atomicMin(&seq[v[t]], k);
}

// The cap of centre c (step k, painted ball {|o|^2 < m}) away from its first
// preceding neighbour in qmask, filtered by the other preceding neighbours:
// for each point (p, q) of the disk p^2 + q^2 <= m - 1 across the cap's axis,
// one stamp at the ball's outermost voxel along that axis.
struct CapGeom {
    int sgn, posA, posB, posC, dimA, dimB, dimC, sA, sB, sC, Rb;
    uint32_t rest0;
    int comp[6];
};

__device__ inline CapGeom cap_geom(const PaintArgs& a, uint32_t m, uint32_t qmask, int x, int y, int z) {
    CapGeom g;
    const int j0 = __ffs(qmask) - 1;
    const int A = j0 >> 1;              // axis of the cap
    g.sgn = (j0 & 1) ? -1 : 1;          // cap on the side away from the neighbour
    const int B = (A + 1) % 3, C = (A + 2) % 3;
    // per-axis values of A, B and C (indices fit 31 bits, so the stamp
    // addresses are 32-bit sums)
    const int yzi = a.Y * a.Z;
    g.posA = A == 0 ? x : A == 1 ? y : z;
    g.posB = B == 0 ? x : B == 1 ? y : z;
    g.posC = C == 0 ? x : C == 1 ? y : z;
    g.dimA = A == 0 ? a.X : A == 1 ? a.Y : a.Z;
    g.dimB = B == 0 ? a.X : B == 1 ? a.Y : a.Z;
    g.dimC = C == 0 ? a.X : C == 1 ? a.Y : a.Z;
    g.sA = A == 0 ? yzi : A == 1 ? a.Z : 1;
    g.sB = B == 0 ? yzi : B == 1 ? a.Z : 1;
    g.sC = C == 0 ? yzi : C == 1 ? a.Z : 1;
    // the other preceding neighbours filter the cap: neighbour j tests
    // |o - n_j|^2 = |o|^2 - 2 s_j o_(axis j) + 1 < mp[j], where o_(axis j) is
    // the cap offset along A (0), B (1) or C (2)
    g.rest0 = qmask & ~(1u << j0);
#pragma unroll
    for (int j = 0; j < 6; j++) g.comp[j] = (j >> 1) == A ? 0 : (j >> 1) == B ? 1 : 2;
    g.Rb = (int)isqrt_u32(m - 1);
    return g;
}

// The stamp of point (p, q) (in the disk when ok), false if none.
__device__ inline bool cap_point(const CapGeom& g, int c, uint32_t m, const uint32_t (&mp)[6], int p, int q, bool ok,
                                 uint32_t& tv) {
    const int pb = g.posB + p, pc = g.posC + q;
    const int rem = (int)(m - 1) - p * p - q * q;
    ok = ok && rem >= 0 && pb >= 0 && pb < g.dimB && pc >= 0 && pc < g.dimC;
    const int w = ok ? (int)isqrt_u32((uint32_t)rem) : 0;
    const int oa = g.sgn * w;
    const int pa = g.posA + oa;
    ok = ok && pa >= 0 && pa < g.dimA;
    const uint32_t oo = (uint32_t)(w * w + p * p + q * q);
    // (unrolled over the six neighbours: a loop over the set bits indexes
    // the arrays at run time, which puts them in scratch memory)
#pragma unroll
    for (int j = 0; j < 6; j++) {
        if (!((g.rest0 >> j) & 1u)) continue;
        const int sj = (j & 1) ? 1 : -1;      // n_j component
        const int oj = g.comp[j] == 0 ? oa : g.comp[j] == 1 ? p : q;
        const uint32_t d = oo - 2 * sj * oj + 1;  // |o - n_j|^2
        ok = ok && d >= mp[j];
    }
    tv = ok ? (uint32_t)(c + oa * g.sA + p * g.sB + q * g.sC) : (uint32_t)c;
    return ok;
}

// A lane stamps its own cap: rows p, and along each row groups of q.
__device__ inline void stamp_cap_lane(const PaintArgs& a, int c, int32_t k, uint32_t m, uint32_t qmask, int x, int y,
                                      int z, const uint32_t (&mp)[6]) {
    const CapGeom g = cap_geom(a, m, qmask, x, y, z);
    for (int p = -g.Rb; p <= g.Rb; p++) {
        if (g.posB + p < 0 || g.posB + p >= g.dimB) continue;
        const int U = (int)isqrt_u32(m - 1 - (uint32_t)(p * p));
        for (int q0 = -U; q0 <= U; q0 += kStampGroup) {
            uint32_t tv[kStampGroup];
            bool tok[kStampGroup];
#pragma unroll
            for (int t = 0; t < kStampGroup; t++) tok[t] = cap_point(g, c, m, mp, p, q0 + t, q0 + t <= U, tv[t]);
            stamp_group(a.seq, tv, tok, k);
        }
    }
}

// The whole wave stamps one cap (arguments uniform): the rows of the
// square holding the disk side by side, a lane per (row, column) point.
__device__ inline void stamp_cap_wave(const PaintArgs& a, int c, int32_t k, uint32_t m, uint32_t qmask, int x, int y,
                                      int z, const uint32_t (&mp)[6]) {
    const int lane = threadIdx.x & 63;
    const CapGeom g = cap_geom(a, m, qmask, x, y, z);
    const int L = 2 * g.Rb + 1;
    if (L <= 64) {
        const int rpr = 64 / L;  // rows per round
        const int r0 = lane / L, q = lane - r0 * L - g.Rb;
        const bool lane_ok = r0 < rpr;
        for (int p0 = -g.Rb; p0 <= g.Rb; p0 += kStampGroup * rpr) {
            uint32_t tv[kStampGroup];
            bool tok[kStampGroup];
#pragma unroll
            for (int t = 0; t < kStampGroup; t++) {
                const int p = p0 + r0 + t * rpr;
                tok[t] = cap_point(g, c, m, mp, p, q, lane_ok && p <= g.Rb, tv[t]);
            }
            stamp_group(a.seq, tv, tok, k);
        }
    } else {
        for (int p = -g.Rb; p <= g.Rb; p++) {
            if (g.posB + p < 0 || g.posB + p >= g.dimB) continue;
            for (int q0 = -g.Rb; q0 <= g.Rb; q0 += 64 * kStampGroup) {
                uint32_t tv[kStampGroup];
                bool tok[kStampGroup];
#pragma unroll
                for (int t = 0; t < kStampGroup; t++) {
                    const int q = q0 + lane + 64 * t;
                    tok[t] = cap_point(g, c, m, mp, p, q, q <= g.Rb, tv[t]);
                }
                stamp_group(a.seq, tv, tok, k);
            }
        }
    }
}

// Caps up to this radius are stamped by their own lane, larger ones by the
// whole wave.
constexpr int kSmallCap = 2;

// One thread per voxel finds its centre's cap: centres with an earlier,
// at-least-as-large face neighbour stamp a cap, the others are listed for the
// full-ball pass. Caps differ widely in size, and with one lane per centre
// most lanes of a wave idled while the largest cap among them was stamped:
// small caps stay with their lane, large ones are stamped one centre at a
// time by all 64 lanes, lanes over the points of the cap's disk.
__global__ __launch_bounds__(256) void k_paint_shell(PaintArgs a) {
    const int64_t yz = (int64_t)a.Y * a.Z;
    const int64_t n = (int64_t)a.X * yz;
    int64_t nb_unused;
    const int64_t b = paint_block(a, nb_unused);
    if (b < 0) return;
    const int64_t c = b * 256 + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int32_t k = 0;
    uint32_t m = 0, qmask = 0;
    uint32_t mp[6] = {0u, 0u, 0u, 0u, 0u, 0u};
    int x = 0, y = 0, z = 0;
    if (c < n) k = a.state[c];
    if (k < a.k_lo || k > a.k_hi) k = 0;
    if (k > 0) {
        const uint32_t rc = a.key[c] & kRankMask;
        m = ball_m(a, a.val[rc]);
        coords((uint32_t)c, a, x, y, z);
        // neighbour j sits at c + n_j: axis j >> 1, sign (j & 1) ? +1 : -1
        const bool inb[6] = {x > 0, x < a.X - 1, y > 0, y < a.Y - 1, z > 0, z < a.Z - 1};
        const int64_t off[6] = {-yz, yz, -(int64_t)a.Z, (int64_t)a.Z, -1, 1};
        // the six neighbours read together (an outside neighbour reads c itself)
        int32_t kp[6];
        uint32_t rp[6];
#pragma unroll
        for (int j = 0; j < 6; j++) {
            const int64_t nb = inb[j] ? c + off[j] : c;
            kp[j] = a.state[nb];
            rp[j] = a.key[nb] & kRankMask;
        }
        uint32_t vp[6];
#pragma unroll
        for (int j = 0; j < 6; j++) vp[j] = a.val[rp[j]];
#pragma unroll
        for (int j = 0; j < 6; j++) {
            const bool q = inb[j] && kp[j] > 0 && kp[j] < k && rp[j] >= rc;
            qmask |= q ? 1u << j : 0u;
            mp[j] = q ? ball_m(a, vp[j]) : 0u;
        }
    }
    // full balls: listed with one atomic per wave
    const bool full = k > 0 && qmask == 0;
    const uint64_t mf = __ballot(full);
    if (mf) {
        const int leader = __ffsll((unsigned long long)mf) - 1;
        uint32_t base = 0;
        if (lane == leader) base = atomicAdd(a.n_full, (uint32_t)__popcll(mf));
        base = __shfl(base, leader, 64);
        if (full) a.full[base + (uint32_t)__popcll(mf & lanemask_lt())] = (uint32_t)c;
    }
    // small caps: each lane stamps its own (the wave runs as long as its
    // largest small cap); large caps: the whole wave on one cap at a time
    const bool cap = k > 0 && qmask != 0;
    const uint32_t rbl = cap ? isqrt_u32(m - 1) : 0u;
    if (cap && rbl <= (uint32_t)kSmallCap)
        stamp_cap_lane(a, (int)c, k, m, qmask, x, y, z, mp);
    uint64_t pending = __ballot(cap && rbl > (uint32_t)kSmallCap);
    while (pending) {
        const int src = __ffsll((unsigned long long)pending) - 1;
        pending &= pending - 1;
        uint32_t mps[6];
#pragma unroll
        for (int j = 0; j < 6; j++) mps[j] = __builtin_amdgcn_readlane(mp[j], src);
        stamp_cap_wave(a, __builtin_amdgcn_readlane((int)c, src), __builtin_amdgcn_readlane(k, src),
                       __builtin_amdgcn_readlane(m, src), __builtin_amdgcn_readlane(qmask, src),
                       __builtin_amdgcn_readlane(x, src), __builtin_amdgcn_readlane(y, src),
                       __builtin_amdgcn_readlane(z, src), mps);
    }
}

// One wave per listed centre: the whole ball, lanes over (x, y) columns,
// each lane writing a contiguous run along z.
__global__ __launch_bounds__(256) void k_paint_full(PaintArgs a) {
    const int lane = threadIdx.x & 63;
    const uint32_t nf = *a.n_full;
    const uint32_t f0 = a.full_lo ? *a.full_lo : 0u;
    int64_t nblocks;
    const int64_t b = paint_block(a, nblocks);
    if (b < 0) return;
    for (uint32_t i = f0 + (uint32_t)b * 4 + (threadIdx.x >> 6); i < nf; i += (uint32_t)nblocks * 4) {
        const int64_t c = a.full[i];
        const int32_t k = a.state[c];
        const uint32_t m = ball_m(a, a.val[a.key[c] & kRankMask]);
        int x, y, z;
        coords((uint32_t)c, a, x, y, z);
        const int Rb = (int)isqrt_u32(m - 1);
        for (int dx = -Rb; dx <= Rb; dx++) {
            const int xx = x + dx;
            if (xx < 0 || xx >= a.X) continue;
            const uint32_t rem = m - 1 - (uint32_t)(dx * dx);
            const int U = (int)isqrt_u32(rem);
            for (int dy = -U + lane; dy <= U; dy += 64) {
                const int yy = y + dy;
                if (yy < 0 || yy >= a.Y) continue;
                const int W = (int)isqrt_u32(rem - (uint32_t)(dy * dy));
                const int z0 = max(z - W, 0), z1 = min(z + W, a.Z - 1);
                const uint32_t rowv = ((uint32_t)xx * (uint32_t)a.Y + (uint32_t)yy) * (uint32_t)a.Z;
                for (int zz = z0; zz <= z1; zz += kStampGroup) {
                    uint32_t tv[kStampGroup];
                    bool tok[kStampGroup];
#pragma unroll
                    for (int t = 0; t < kStampGroup; t++) {
                        tok[t] = zz + t <= z1;
                        tv[t] = rowv + (uint32_t)min(zz + t, z1);
                    }
                    stamp_group(a.seq, tv, tok, k);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Finalise and per-step accounting
// ---------------------------------------------------------------------------
// M held ranks during the loop; turn them into squared radii.
// After an insertion pass: the full-ball list entries so far are painted.
__global__ void k_full_mark(uint32_t* full_done, const uint32_t* n_full) { *full_done = *n_full; }

__global__ void k_rank_to_value(uint32_t* M, int64_t K, const uint32_t* val) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < K) M[k] = val[M[k]];
}

// Each block finalises a contiguous chunk of kCntChunk voxels. With `copies`
// given, the per-step counts of painted voxels go to copy blockIdx % ncopies
// (copy c at copies + c * K), summed per block in LDS first.
__global__ __launch_bounds__(256) void k_finalise(int32_t* seq, int32_t* state_io, bool map_state, int64_t n,
                                                  const uint32_t* M, uint32_t* rad2, uint32_t* copies, int64_t K,
                                                  int ncopies) {
    __shared__ CountTable tab;
    const bool counting = copies != nullptr;
    if (counting) count_table_clear(tab);
    __syncthreads();
    uint32_t* copy = counting ? copies + (int64_t)(blockIdx.x % (unsigned)ncopies) * K : nullptr;
    const int64_t base = (int64_t)blockIdx.x * kCntChunk;
    for (int j = 0; j < kCntChunk; j += 256) {
        const int64_t v = base + j + threadIdx.x;
        const bool have = v < n;
        int32_t s = 0;
        if (have) {
            s = seq[v];
            if (s == INT_MAX) { s = 0; seq[v] = 0; }
            if (rad2) rad2[v] = s > 0 ? M[s - 1] : 0u;
            const int32_t t = state_io[v];
            if (map_state && t < 0) state_io[v] = 0;
        }
        if (counting) count_table_add(tab, have && s > 0, s, copy);
    }
    if (counting) {
        __syncthreads();
        count_table_flush(tab, copy);
    }
}

__global__ void k_copy_u32(const uint32_t* src, uint32_t* dst, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) dst[i] = src[i];
}

// count_excl: exclusive scan of counts; counts: raw counts.
__global__ void k_steps(const uint32_t* counts, const uint32_t* count_excl, const uint32_t* M, int64_t K,
                        const LoopState* st, double c0, int64_t* n_new, double* sat, double* pc) {
    int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k >= K) return;
    const uint32_t c = counts[k];
    n_new[k] = c;
    const double np = (double)st->n_pore;
    sat[k] = (double)(count_excl[k] + c) / np;
    pc[k] = c0 / sqrt((double)M[k]);
}

inline unsigned blocks(int64_t n, int t = 256) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// k_finalise over n voxels. With counts given (K > 0), counts[0..K) receives
// the number of voxels of each step; `spare` holds the copies when there is
// more than one (kCntCopies * K words, see count_copies).
hipError_t launch_finalise(int32_t* seq, int32_t* state, int64_t n, const uint32_t* M, uint32_t* rad2,
                           uint32_t* counts, uint32_t* spare, int64_t K, hipStream_t s) {
    const unsigned g = (unsigned)((n + kCntChunk - 1) / kCntChunk);
    if (!counts || K <= 0) {
        hipLaunchKernelGGL(k_finalise, dim3(g), dim3(256), 0, s, seq, state, true, n, M, rad2, (uint32_t*)nullptr,
                           (int64_t)0, 1);
        return hipGetLastError();
    }
    const int S = count_copies(K, n);
    uint32_t* dst = S > 1 ? spare : counts;
    hipError_t e = hipMemsetAsync(dst, 0, sizeof(uint32_t) * (size_t)S * (size_t)K, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_finalise, dim3(g), dim3(256), 0, s, seq, state, true, n, M, rad2, dst, K, S);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return S > 1 ? launch_sum_copies(spare, S, K, counts, s) : hipSuccess;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
ibip_status run_invade(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims d,
                       const ibip_invade_opts* opts, int32_t* seq, uint32_t* rad2, int32_t* centre_step,
                       int64_t* n_steps, const int32_t* resume_cs, int64_t k_done) {
    hipStream_t s = ctx->stream;
    const int64_t n = nvox(d);
    const int64_t V = (int64_t)(d.X - 1) * (d.X - 1) + (int64_t)(d.Y - 1) * (d.Y - 1) +
                      (int64_t)(d.Z - 1) * (d.Z - 1) + 2;
    ctx->have_steps = false;
    uint32_t* key = (uint32_t*)ensure(ctx, B_KEY, sizeof(uint32_t) * n);
    int32_t* state = centre_step ? centre_step : (int32_t*)ensure(ctx, B_STATE, sizeof(int32_t) * n);
    uint32_t* bucket = (uint32_t*)ensure(ctx, B_BUCKET, sizeof(uint32_t) * n);
    uint32_t* hist = (uint32_t*)ensure(ctx, B_HIST, sizeof(uint32_t) * 3 * V);
    uint16_t* g16 = (uint16_t*)ensure(ctx, B_TMP0, sizeof(uint16_t) * n);
    uint32_t* tmp32 = (uint32_t*)ensure(ctx, B_TMP1, sizeof(uint32_t) * n);
    uint32_t* partials = (uint32_t*)ensure(ctx, B_SCAN, sizeof(uint32_t) * (V / 1000 + n / 1000 + 64));
    uint8_t* misc = (uint8_t*)ensure(ctx, B_MISC, 4096);
    LoopState* h_st = (LoopState*)pinned(ctx, 4096);
    if (!key || !state || !bucket || !hist || !g16 || !tmp32 || !partials || !misc || !h_st)
        return fail(ctx, IBIP_ENOMEM, "invade: scratch allocation failed");
    LoopState* st = (LoopState*)misc;
    uint32_t* solid_flag = &st->solid_seen;
    uint32_t* dummy_total = (uint32_t*)(misc + 1024);
    uint32_t* present = hist + V;
    uint32_t* flags = hist + 2 * V;  // raw presence (kept unscanned)

    ibip_status rc;
    Timer& tm = ctx->timer;
    tm.mark(0, s);
    if ((rc = hip_check(ctx, hipMemsetAsync(misc, 0, 4096, s), "memset")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(hist, 0, sizeof(uint32_t) * V, s), "memset")) != IBIP_OK) return rc;
    // a1: distance transform into key[]
    if ((rc = hip_check(ctx, launch_edt(image, nullptr, 0, 0, d, g16, tmp32, key, solid_flag, s, nullptr, nullptr,
                                        edt_tiles(ctx->tuning)), "edt")) != IBIP_OK)
        return rc;
    tm.mark(1, s);
    // a2: histogram -> ranks and bucket slices
    hipLaunchKernelGGL(k_hist, dim3(std::min<int64_t>(blocks(n), kHistBlocks)), dim3(256), 0, s, key, n,
                       (uint32_t)(V - 1), hist, st);
    hipLaunchKernelGGL(k_present, dim3(blocks(V)), dim3(256), 0, s, hist, present, V);
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks(V)), dim3(256), 0, s, present, flags, V);
    if ((rc = hip_check(ctx, launch_scan_u32(hist, V, partials, dummy_total, s), "scan")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, launch_scan_u32(present, V, partials, &st->R, s), "scan")) != IBIP_OK) return rc;
    // sync once: the rank count sizes the per-rank arrays and picks the loop variant
    if ((rc = hip_check(ctx, hipMemcpyAsync(h_st, st, sizeof(LoopState), hipMemcpyDeviceToHost, s), "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (!h_st->solid_seen) return fail(ctx, IBIP_ENOSOLID, "invade: image holds no solid voxel");
    const uint32_t R = h_st->R;
    if (R > kRankMask)
        return fail(ctx, IBIP_ECAPACITY, "invade: more distinct distance values than the 24-bit rank field holds");
    // more ranks than the LDS tables of k_loop hold: the global-memory loop
    const bool big = R > (uint32_t)kMaxRanks;
    const int64_t n_pore = h_st->n_pore;
    uint32_t* val = (uint32_t*)ensure(ctx, B_VAL, sizeof(uint32_t) * (R + 2));
    uint32_t* off = (uint32_t*)ensure(ctx, B_OFF, sizeof(uint32_t) * (R + 2));
    uint32_t* head = (uint32_t*)ensure(ctx, B_HEAD, sizeof(uint32_t) * (R + 2));
    uint32_t* tail = (uint32_t*)ensure(ctx, B_TAIL, sizeof(uint32_t) * (R + 2));
    uint32_t* M = (uint32_t*)ensure(ctx, B_M, sizeof(uint32_t) * (n_pore + 1));
    uint32_t* full = (uint32_t*)ensure(ctx, B_FULL, sizeof(uint32_t) * (n_pore + 1));
    uint32_t* gbits =
        big ? (uint32_t*)ensure(ctx, B_GBITS, sizeof(uint32_t) * (((size_t)R >> 5) + ((size_t)R >> 10) + 8)) : nullptr;
    if (!val || !off || !head || !tail || !M || !full || (big && !gbits))
        return fail(ctx, IBIP_ENOMEM, "invade: scratch allocation failed");
    if ((rc = hip_check(ctx, hipMemsetAsync(head, 0, sizeof(uint32_t) * (R + 2), s), "memset")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(tail, 0, sizeof(uint32_t) * (R + 2), s), "memset")) != IBIP_OK) return rc;
    hipLaunchKernelGGL(k_rank_tables, dim3(blocks(V)), dim3(256), 0, s, hist, present, flags, V, val, off, head, tail,
                       R);
    hipLaunchKernelGGL(k_convert, dim3(blocks(n)), dim3(256), 0, s, image, key, present, n, (uint32_t)(V - 1), state,
                       seq, d.X, d.Y, d.Z, make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y), R);
    if (resume_cs) {
        if (k_done > n_pore) return fail(ctx, IBIP_EINVAL, "invade_resume: more steps done than pore voxels");
        hipLaunchKernelGGL(k_resume_seed, dim3(blocks(n)), dim3(256), 0, s, inlets, resume_cs, k_done, key, state, M,
                           d.X, d.Y, d.Z, tail, bucket, (ctx->readings & IBIP_READ_MASK_INLETS) != 0, &st->pad2);
    } else {
        hipLaunchKernelGGL(k_seed, dim3(blocks(n)), dim3(256), 0, s, inlets, key, d.X, d.Y, d.Z, tail, bucket,
                           (ctx->readings & IBIP_READ_MASK_INLETS) != 0, R);
    }
    tm.mark(2, s);
    // loop control
    h_st->k = 1 + (uint32_t)(resume_cs ? k_done : 0);
    h_st->status = LS_RUN;
    h_st->max_steps = opts ? opts->max_steps : 0;
    {
        // k, status and max_steps only; the rest stays as computed on the device
        LoopState init = *h_st;
        if ((rc = hip_check(ctx, hipMemcpyAsync(&st->k, &init.k, sizeof(uint32_t) * 2, hipMemcpyHostToDevice, s),
                            "copy")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipMemcpyAsync(&st->max_steps, &init.max_steps, sizeof(int64_t),
                                                hipMemcpyHostToDevice, s), "copy")) != IBIP_OK)
            return rc;
        if (resume_cs &&
            (rc = hip_check(ctx, hipMemcpyAsync(&h_st->pad2, &st->pad2, sizeof(uint32_t), hipMemcpyDeviceToHost, s),
                            "copy")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
        if (resume_cs && h_st->pad2)
            return fail(ctx, IBIP_EINVAL, "invade_resume: the checkpoint has a step outside 1..k_done or a centre on solid");
    }
    LoopArgs la{st,     head, tail, val, bucket, state, key, M, d.X, d.Y, d.Z, kWideRound, kSmallRound,
                make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y)};
    la.gbits = gbits;
    auto launch_loop = [&]() {
        if (big) hipLaunchKernelGGL(k_loop_global<false>, dim3(1), dim3(kLoopThreads), 0, s, la);
        else hipLaunchKernelGGL(k_loop<false>, dim3(1), dim3(kLoopThreads), 0, s, la);
    };
    // The loop kernel stops at each wide step; the host reads the loop state
    // after each stop. The wide step and the next loop segment are queued
    // before that read (each does nothing if the loop had ended), so the GPU
    // does not wait for the host between segments. Timing events alternate
    // between two slots, since a launch's events are read only after the
    // launch queued behind it was recorded.
    // at least one block: an image with no pore voxel still takes the launches
    const unsigned gw = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n_pore + 255) / 256, 4096));
    if (!ctx->copy_ev &&
        (rc = hip_check(ctx, hipEventCreateWithFlags(&ctx->copy_ev, hipEventDisableTiming), "event")) != IBIP_OK)
        return rc;
    auto loop_ev = [](int p, int e) { return p ? 12 + e : 3 + e; };  // e = 0 start, 1 end
    auto wide_ev = [](int p, int e) { return p ? 14 + e : 5 + e; };
    int64_t segments = 0, wide_centres = 0;
    // a5, in passes: insertion is order-free and selection never reads it,
    // so the steps finished so far are inserted on a second stream while the
    // loop runs: at a wide-step stop, a pass once the previous one has ended
    // and a 32nd of the pore voxels (at least 2^21) have become centres since
    // it; the rest after the loop
    PaintArgs pa{state, key, val, seq, full, &st->n_full, d.X, d.Y, d.Z,
                 (ctx->readings & IBIP_READ_INTEGER_BALL) != 0, make_fastdiv((uint32_t)d.Z),
                 make_fastdiv((uint32_t)d.Y)};
    pa.full_lo = &st->full_done;
    auto paint_pass = [&](hipStream_t ps, int32_t lo, int32_t hi) {
        pa.k_lo = lo;
        pa.k_hi = hi;
        // a pass under the loop keeps off XCD 0: 8 workgroups for every 7
        pa.skip_xcd0 = ps != s;
        const int64_t gb = pa.skip_xcd0 ? (blocks(n) + 6) / 7 * 8 : blocks(n);
        hipLaunchKernelGGL(k_paint_shell, dim3((unsigned)gb), dim3(256), 0, ps, pa);
        hipLaunchKernelGGL(k_paint_full, dim3(pa.skip_xcd0 ? 2048 / 7 * 8 : 2048), dim3(256), 0, ps, pa);
        hipLaunchKernelGGL(k_full_mark, dim3(1), dim3(1), 0, ps, &st->full_done, (const uint32_t*)&st->n_full);
    };
    int32_t painted = 0;  // steps 1..painted inserted by passes on the second stream
    int64_t painted_centres = 0;
    const int64_t pass_centres = std::max<int64_t>(n_pore / 32, (int64_t)1 << 21);
    // an early return leaves no pass running on buffers the next call reuses
    struct PaintJoin {
        hipStream_t ps = nullptr;
        ~PaintJoin() {
            if (ps) (void)hipStreamSynchronize(ps);
        }
    } pjoin;
    int p = 0;
    bool wide_ran = false;  // the wide launch read this round ran a wide step
    tm.mark(loop_ev(p, 0), s);
    launch_loop();
    tm.mark(loop_ev(p, 1), s);
    for (;;) {
        if ((rc = hip_check(ctx, hipGetLastError(), "loop launch")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipMemcpyAsync(h_st, st, sizeof(LoopState), hipMemcpyDeviceToHost, s), "copy")) !=
            IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipEventRecord(ctx->copy_ev, s), "event")) != IBIP_OK) return rc;
        tm.mark(wide_ev(p, 0), s);
        hipLaunchKernelGGL(k_wide, dim3(gw), dim3(256), 0, s, la);
        tm.mark(wide_ev(p, 1), s);
        tm.mark(loop_ev(p ^ 1, 0), s);
        launch_loop();
        tm.mark(loop_ev(p ^ 1, 1), s);
        if ((rc = hip_check(ctx, hipGetLastError(), "wide launch")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipEventSynchronize(ctx->copy_ev), "sync")) != IBIP_OK) return rc;
        if (tm.on) {
            ctx->timing.loop_kernel_ms += tm.ms(loop_ev(p, 0), loop_ev(p, 1));
            ctx->timing.loop_launches++;
            if (wide_ran) {
                ctx->timing.wide_kernel_ms += tm.ms(wide_ev(p ^ 1, 0), wide_ev(p ^ 1, 1));
                ctx->timing.wide_launches++;
            }
        }
        if (++segments > n_pore + 2) return fail(ctx, IBIP_EDEVICE, "invade: too many loop segments");
        if (h_st->status != LS_WIDE) break;
        {
            // steps before the pending wide step are finished; their centres:
            // the loop kernels' and the earlier wide steps'
            const int32_t done = (int32_t)h_st->big_k - 1;
            const int64_t centres = (int64_t)h_st->popped + wide_centres;
            bool idle = true;  // no pass yet, or the last one has ended
            if (pjoin.ps) {
                const hipError_t qe = hipEventQuery(ctx->paint_ev);
                if (qe != hipSuccess && qe != hipErrorNotReady) return hip_check(ctx, qe, "event query");
                idle = qe == hipSuccess;
            }
            if (idle && centres - painted_centres >= pass_centres && done > painted) {
                if (!ctx->paint_stream &&
                    (rc = hip_check(ctx, hipStreamCreateWithFlags(&ctx->paint_stream, hipStreamNonBlocking),
                                    "stream")) != IBIP_OK)
                    return rc;
                if ((rc = hip_check(ctx, hipStreamWaitEvent(ctx->paint_stream, ctx->copy_ev, 0), "wait")) != IBIP_OK)
                    return rc;
                pjoin.ps = ctx->paint_stream;
                paint_pass(ctx->paint_stream, painted + 1, done);
                if ((rc = hip_check(ctx, hipGetLastError(), "paint launch")) != IBIP_OK) return rc;
                if (!ctx->paint_ev &&
                    (rc = hip_check(ctx, hipEventCreateWithFlags(&ctx->paint_ev, hipEventDisableTiming), "event")) !=
                        IBIP_OK)
                    return rc;
                if ((rc = hip_check(ctx, hipEventRecord(ctx->paint_ev, ctx->paint_stream), "event")) != IBIP_OK)
                    return rc;
                painted = done;
                painted_centres = centres;
            }
        }
        const uint32_t cnt = h_st->big_t - h_st->big_h;
        wide_centres += cnt;
        if (tm.on) ctx->timing.wide_centres += cnt;
        wide_ran = true;
        p ^= 1;
    }
    if (h_st->err) return fail(ctx, IBIP_EDEVICE, "invade: step loop exceeded the pore count");
    const int64_t K = (int64_t)h_st->k - 1;
    tm.mark(7, s);
    if (K > 0) hipLaunchKernelGGL(k_rank_to_value, dim3(blocks(K)), dim3(256), 0, s, M, K, val);
    // a5: the steps not inserted yet, after the passes on the second stream
    if (pjoin.ps) {
        if (!ctx->paint_ev &&
            (rc = hip_check(ctx, hipEventCreateWithFlags(&ctx->paint_ev, hipEventDisableTiming), "event")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipEventRecord(ctx->paint_ev, ctx->paint_stream), "event")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipStreamWaitEvent(s, ctx->paint_ev, 0), "wait")) != IBIP_OK) return rc;
    }
    paint_pass(s, painted + 1, INT_MAX);
    tm.mark(8, s);
    // a6: finalise and per-step arrays
    int64_t* n_new = (int64_t*)ensure(ctx, B_NNEW, sizeof(int64_t) * (K + 1));
    double* sat = (double*)ensure(ctx, B_SAT, sizeof(double) * (K + 1));
    double* pc = (double*)ensure(ctx, B_PC, sizeof(double) * (K + 1));
    // counts (K + 1), their exclusive scan (K + 1), then the count copies
    const size_t ncopy = count_copies(K, n) > 1 ? (size_t)kCntCopies * (size_t)K : 0;
    uint32_t* counts = (uint32_t*)ensure(ctx, B_TMP2, sizeof(uint32_t) * (2 * (K + 1) + ncopy));
    partials = (uint32_t*)ensure(ctx, B_SCAN, sizeof(uint32_t) * (V / 1000 + n / 1000 + 64));
    if (!n_new || !sat || !pc || !counts || !partials) return fail(ctx, IBIP_ENOMEM, "invade: scratch allocation failed");
    if ((rc = hip_check(ctx, launch_finalise(seq, state, n, M, rad2, counts, counts + 2 * (K + 1), K, s),
                        "finalise")) != IBIP_OK)
        return rc;
    if (K > 0) {
        uint32_t* excl = counts + (K + 1);
        hipLaunchKernelGGL(k_copy_u32, dim3(blocks(K)), dim3(256), 0, s, counts, excl, K);
        if ((rc = hip_check(ctx, launch_scan_u32(excl, K, partials, dummy_total, s), "scan")) != IBIP_OK) return rc;
        const double sigma = (opts && opts->sigma != 0.0) ? opts->sigma : 1.0;
        const double theta = opts ? opts->theta_rad : 0.0;
        const double vs = (opts && opts->voxel_size != 0.0) ? opts->voxel_size : 1.0;
        const double c0 = 2.0 * sigma * cos(theta) / vs;
        hipLaunchKernelGGL(k_steps, dim3(blocks(K)), dim3(256), 0, s, counts, excl, M, K, st, c0, n_new, sat, pc);
    }
    if ((rc = hip_check(ctx, hipGetLastError(), "post launch")) != IBIP_OK) return rc;
    tm.mark(9, s);
    if ((rc = hip_check(ctx, hipMemcpyAsync(h_st, st, sizeof(LoopState), hipMemcpyDeviceToHost, s), "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(s), "sync")) != IBIP_OK) return rc;
    if (tm.on) {
        ibip_timing& T = ctx->timing;
        T.edt_ms += tm.ms(0, 1);
        T.setup_ms += tm.ms(1, 2);
        T.loop_ms += tm.ms(2, 7);
        T.paint_ms += tm.ms(7, 8);
        T.steps_ms += tm.ms(8, 9);
        T.steps += K;
        T.popped += h_st->popped + wide_centres;
    }
    ctx->last_K = K;
    ctx->last_n_pore = n_pore;
    ctx->have_steps = true;
    if (n_steps) *n_steps = K;
    return IBIP_OK;
}


// ---------------------------------------------------------------------------
// Batches: many images of uneven size in one call.
// ---------------------------------------------------------------------------
int64_t value_range(ibip_dims d) {
    return (int64_t)(d.X - 1) * (d.X - 1) + (int64_t)(d.Y - 1) * (d.Y - 1) + (int64_t)(d.Z - 1) * (d.Z - 1) + 2;
}


// bytes of one job's scratch; carve() lays the same regions out in order
size_t job_bytes(ibip_dims d, bool own_state, bool want_sat) {
    const size_t n = (size_t)nvox(d), V = (size_t)value_range(d);
    size_t b = 0;
    b += align256(4 * n);                                 // key
    if (own_state) b += align256(4 * n);                  // state
    b += align256(4 * n);                                 // bucket
    b += align256(4 * 3 * V);                             // hist
    b += align256(2 * n);                                 // g16
    b += align256(4 * n);                                 // tmp32
    b += align256(4 * (V / 1000 + n / 1000 + 64));        // partials
    b += 4 * align256(4 * ((size_t)kMaxRanks + 2));       // val, off, head, tail
    b += align256(4 * (n + 1));                           // M
    b += align256(4 * (n + 1));                           // full
    if (want_sat) b += align256(4 * 2 * (n + 1));         // counts
    b += 256;                                             // scan total
    return b;
}

JobBufs carve(uint8_t* base, ibip_dims d, int32_t* caller_state, bool want_sat) {
    const size_t n = (size_t)nvox(d), V = (size_t)value_range(d);
    JobBufs j{};
    auto take = [&](size_t bytes) {
        uint8_t* p = base;
        base += align256(bytes);
        return p;
    };
    j.key = (uint32_t*)take(4 * n);
    j.state = caller_state ? caller_state : (int32_t*)take(4 * n);
    j.bucket = (uint32_t*)take(4 * n);
    j.hist = (uint32_t*)take(4 * 3 * V);
    j.g16 = (uint16_t*)take(2 * n);
    j.tmp32 = (uint32_t*)take(4 * n);
    j.partials = (uint32_t*)take(4 * (V / 1000 + n / 1000 + 64));
    j.val = (uint32_t*)take(4 * ((size_t)kMaxRanks + 2));
    j.off = (uint32_t*)take(4 * ((size_t)kMaxRanks + 2));
    j.head = (uint32_t*)take(4 * ((size_t)kMaxRanks + 2));
    j.tail = (uint32_t*)take(4 * ((size_t)kMaxRanks + 2));
    j.M = (uint32_t*)take(4 * (n + 1));
    j.full = (uint32_t*)take(4 * (n + 1));
    j.counts = want_sat ? (uint32_t*)take(4 * 2 * (n + 1)) : nullptr;
    j.scan_total = (uint32_t*)take(256);
    return j;
}

// n words of p set to v (a kernel, not a memset: the batch's setup is
// captured into a graph, where memset nodes are avoided)
static __global__ void k_fill_u32(uint32_t* p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) p[i] = v;
}

static hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks(n), 1024))),
                       dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

static __global__ void k_loopstate_init(LoopState* st, int64_t max_steps) {
    st->k = 1;
    st->status = LS_RUN;
    st->max_steps = max_steps;
}

// saturation after each step: (counts up to k) / n_pore
static __global__ void k_sat(const uint32_t* counts, const uint32_t* count_excl, int64_t K, const LoopState* st,
                      double* sat) {
    const int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (k < K) sat[k] = (double)(count_excl[k] + counts[k]) / (double)st->n_pore;
}

hipError_t job_setup(const JobBufs& j, LoopState* st, const uint8_t* image, const uint8_t* inlets, ibip_dims d,
                     int64_t max_steps, int32_t* seq, hipStream_t s, EdtTiles tiles) {
    const int64_t n = nvox(d), V = value_range(d);
    hipError_t e;
    static_assert(sizeof(LoopState) % 4 == 0, "LoopState is cleared as words");
    if ((e = fill_u32((uint32_t*)st, sizeof(LoopState) / 4, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(j.hist, V, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(j.head, kMaxRanks + 2, 0u, s)) != hipSuccess) return e;
    if ((e = fill_u32(j.tail, kMaxRanks + 2, 0u, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_loopstate_init, dim3(1), dim3(1), 0, s, st, max_steps);
    if ((e = launch_edt(image, nullptr, 0, 0, d, j.g16, j.tmp32, j.key, &st->solid_seen, s, nullptr, nullptr, tiles)) != hipSuccess) return e;
    uint32_t* present = j.hist + V;
    uint32_t* flags = j.hist + 2 * V;
    hipLaunchKernelGGL(k_hist, dim3(std::min<int64_t>(blocks(n), kHistBlocks)), dim3(256), 0, s, j.key, n,
                       (uint32_t)(V - 1), j.hist, st);
    hipLaunchKernelGGL(k_present, dim3(blocks(V)), dim3(256), 0, s, j.hist, present, V);
    hipLaunchKernelGGL(k_copy_u32, dim3(blocks(V)), dim3(256), 0, s, present, flags, V);
    if ((e = launch_scan_u32(j.hist, V, j.partials, j.scan_total, s)) != hipSuccess) return e;
    if ((e = launch_scan_u32(present, V, j.partials, &st->R, s)) != hipSuccess) return e;
    // a job's tables hold kMaxRanks ranks; its loop rejects an image with more
    hipLaunchKernelGGL(k_rank_tables, dim3(blocks(V)), dim3(256), 0, s, j.hist, present, flags, V, j.val, j.off,
                       j.head, j.tail, (uint32_t)kMaxRanks);
    hipLaunchKernelGGL(k_convert, dim3(blocks(n)), dim3(256), 0, s, image, j.key, present, n, (uint32_t)(V - 1),
                       j.state, seq, d.X, d.Y, d.Z, make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y),
                       (uint32_t)kMaxRanks);
    hipLaunchKernelGGL(k_seed, dim3(blocks(n)), dim3(256), 0, s, inlets, j.key, d.X, d.Y, d.Z, j.tail, j.bucket,
                       false, (uint32_t)kMaxRanks);
    return hipGetLastError();
}

hipError_t job_post(const JobBufs& j, LoopState* st, ibip_dims d, int64_t K, int32_t* seq, uint32_t* rad2,
                    uint32_t* M_out, double* sat_out, hipStream_t s) {
    const int64_t n = nvox(d);
    hipError_t e;
    if (K > 0) hipLaunchKernelGGL(k_rank_to_value, dim3(blocks(K)), dim3(256), 0, s, j.M, K, j.val);
    PaintArgs pa{j.state, j.key, j.val, seq, j.full, &st->n_full, d.X, d.Y, d.Z, false,
                 make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y)};
    hipLaunchKernelGGL(k_paint_shell, dim3(blocks(n)), dim3(256), 0, s, pa);
    hipLaunchKernelGGL(k_paint_full, dim3(std::min<int64_t>(blocks(n), 2048)), dim3(256), 0, s, pa);
    // the job's counts region holds 2 (n + 1) words: counts, their scan and,
    // when used, the copies (at most n words, and then 2 K <= n)
    uint32_t* counts = j.counts;
    if ((e = launch_finalise(seq, j.state, n, j.M, rad2, counts, counts ? counts + 2 * (K + 1) : nullptr,
                             counts ? K : 0, s)) != hipSuccess)
        return e;
    if (K > 0 && M_out)
        if ((e = hipMemcpyAsync(M_out, j.M, sizeof(uint32_t) * K, hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
    if (K > 0 && sat_out && counts) {
        uint32_t* excl = counts + (K + 1);
        hipLaunchKernelGGL(k_copy_u32, dim3(blocks(K)), dim3(256), 0, s, counts, excl, K);
        if ((e = launch_scan_u32(excl, K, j.partials, j.scan_total, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(k_sat, dim3(blocks(K)), dim3(256), 0, s, counts, excl, K, st, sat_out);
    }
    return hipGetLastError();
}

// Post-processing when K is only known on the device (the server path):
// grid-stride kernels read K from the loop state.
static __global__ void k_rank_to_value_dev(uint32_t* M, const LoopState* st, const uint32_t* val, uint32_t* M_out) {
    const int64_t K = (int64_t)st->k - 1;
    if (st->err) return;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < K; k += (int64_t)gridDim.x * 256) {
        const uint32_t v = val[M[k]];
        M[k] = v;
        if (M_out) M_out[k] = v;
    }
}

hipError_t job_post_devk(const JobBufs& j, LoopState* st, ibip_dims d, int32_t* seq, uint32_t* rad2,
                         uint32_t* M_out, hipStream_t s) {
    const int64_t n = nvox(d);
    hipLaunchKernelGGL(k_rank_to_value_dev, dim3((unsigned)std::min<int64_t>(blocks(n), 1024)), dim3(256), 0, s,
                       j.M, st, j.val, M_out);
    PaintArgs pa{j.state, j.key, j.val, seq, j.full, &st->n_full, d.X, d.Y, d.Z, false,
                 make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y)};
    hipLaunchKernelGGL(k_paint_shell, dim3(blocks(n)), dim3(256), 0, s, pa);
    hipLaunchKernelGGL(k_paint_full, dim3(std::min<int64_t>(blocks(n), 2048)), dim3(256), 0, s, pa);
    return launch_finalise(seq, j.state, n, j.M, rad2, nullptr, nullptr, 0, s);
}

hipError_t launch_loop_jobs(const void* d_args, int32_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_loop_batch<true>, dim3((unsigned)n), dim3(kLoopThreads), 0, s, (const LoopArgs*)d_args);
    return hipGetLastError();
}

// wide: a step with more centres stops the job's loop, to be run over the
// whole GPU (0xFFFFFFFF: every step inside the job's workgroup)
LoopArgs job_loop_args(const JobBufs& j, LoopState* st, ibip_dims d, uint32_t wide = 0xFFFFFFFFu) {
    return LoopArgs{st,  j.head, j.tail, j.val, j.bucket, j.state, j.key, j.M, d.X, d.Y, d.Z, wide,
                    kSmallRound, make_fastdiv((uint32_t)d.Z), make_fastdiv((uint32_t)d.Y)};
}

uint32_t wide_threshold(int64_t tuned) {
    return tuned < 0 ? 0xFFFFFFFFu : tuned == 0 ? kWideRound : (uint32_t)std::min<int64_t>(tuned, 0xFFFFFFFEll);
}

// The wide step a job's loop stopped at, over the whole GPU, then the job's
// loop again in one workgroup (to its next wide step or its end), on s; with
// `cancellable` the loop checks the job's cancel flag.
hipError_t launch_wide_and_loop(const LoopArgs& la, int64_t n, hipStream_t s, bool cancellable = false) {
    const unsigned gw = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
    hipLaunchKernelGGL(k_wide, dim3(gw), dim3(256), 0, s, la);
    if (cancellable) hipLaunchKernelGGL(k_loop<true>, dim3(1), dim3(kLoopThreads), 0, s, la);
    else hipLaunchKernelGGL(k_loop<false>, dim3(1), dim3(kLoopThreads), 0, s, la);
    return hipGetLastError();
}

hipError_t launch_wide_and_loop_host(const void* host_args, int64_t n, hipStream_t s) {
    LoopArgs la = *(const LoopArgs*)host_args;
    la.done = nullptr;
    return launch_wide_and_loop(la, n, s, true);
}

size_t loop_args_bytes() { return sizeof(LoopArgs); }

void set_loop_cancel(void* args, const uint32_t* flag) { ((LoopArgs*)args)->cancel = flag; }

void fill_loop_args(void* out, const JobBufs& j, LoopState* st, ibip_dims d, uint32_t wide) {
    *(LoopArgs*)out = job_loop_args(j, st, d, wide);
}

ibip_status run_invade_batch(ibip_ctx* ctx, ibip_job* jobs, int32_t nj) {
    hipStream_t s0 = ctx->stream;
    // largest jobs first: their loops are the longest
    std::vector<int32_t> order(nj);
    for (int32_t i = 0; i < nj; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int32_t a, int32_t b) { return nvox(jobs[a].dims) > nvox(jobs[b].dims); });
    std::vector<size_t> offs(nj);
    size_t total = 0;
    for (int32_t q = 0; q < nj; q++) {
        const ibip_job& jb = jobs[order[q]];
        offs[q] = total;
        total += job_bytes(jb.dims, jb.centre_step == nullptr, jb.sat != nullptr);
    }
    const size_t st_off = total;
    total += align256(sizeof(LoopState) * (size_t)nj);
    const size_t la_off = total;
    total += align256(sizeof(LoopArgs) * (size_t)nj);
    uint8_t* arena = (uint8_t*)ensure(ctx, B_BATCH, total);
    // pinned: the states after the launch, the loop arguments, and each
    // continued job's state after its latest segment
    LoopState* h_st =
        (LoopState*)pinned(ctx, std::max<size_t>(4096, (2 * sizeof(LoopState) + sizeof(LoopArgs)) * (size_t)nj));
    if (!arena || !h_st) return fail(ctx, IBIP_ENOMEM, "invade_batch: scratch allocation failed");
    LoopState* states = (LoopState*)(arena + st_off);
    LoopArgs* d_args = (LoopArgs*)(arena + la_off);
    LoopArgs* h_args = (LoopArgs*)(h_st + nj);
    LoopState* h_cont = (LoopState*)(h_args + nj);
    // a job that leaves the batched launch continues in launches of its own
    // on a batch stream, where it serialises with the other jobs of that
    // stream: by default every step stays in the job's workgroup
    const uint32_t wide = ctx->tuning.batch_wide == 0 ? 0xFFFFFFFFu : wide_threshold(ctx->tuning.batch_wide);
    ibip_status rc;
    if ((rc = batch_streams(ctx)) != IBIP_OK) return rc;
    const int S = kBatchStreams;
    std::vector<JobBufs> bufs(nj);
    const EdtTiles tiles = edt_tiles(ctx->tuning);
    // the per-job setup (EDT, histogram, ranks, slices, seeds) depends only on
    // the jobs' buffers, dims and step limits and the arena: each batch
    // stream's share of it is captured once into a graph of its own and
    // replayed on that stream while the same batch comes back (one graph
    // for the whole setup would replay its branches without the streams'
    // concurrency)
    std::vector<uint64_t> key = {(uint64_t)nj, (uint64_t)(uintptr_t)arena, (uint64_t)tiles.y, (uint64_t)tiles.x};
    for (int32_t q = 0; q < nj; q++) {
        const ibip_job& jb = jobs[order[q]];
        bufs[q] = carve(arena + offs[q], jb.dims, jb.centre_step, jb.sat != nullptr);
        h_args[q] = job_loop_args(bufs[q], states + q, jb.dims, wide);
        key.insert(key.end(), {(uint64_t)(uintptr_t)jb.image, (uint64_t)(uintptr_t)jb.inlets,
                               (uint64_t)(uintptr_t)jb.seq, (uint64_t)(uintptr_t)jb.centre_step,
                               (uint64_t)(uintptr_t)jb.sat, (uint64_t)jb.max_steps, (uint64_t)jb.dims.X,
                               ((uint64_t)jb.dims.Y << 32) | (uint32_t)jb.dims.Z});
    }
    // The first job of each stream (the S largest jobs) is set up by direct
    // launches, so that those jobs' loops can start while the other setups
    // run: replays of the graphs below do not overlap each other (measured:
    // the 8 streams' replays ran one after another), while direct launches on
    // the streams do. The other jobs' setups are captured per stream.
    if (ctx->batch_key != key) {
        for (int i = 0; i < S; i++)
            if (ctx->batch_exec[i]) {
                (void)hipGraphExecDestroy(ctx->batch_exec[i]);
                ctx->batch_exec[i] = nullptr;
            }
        ctx->batch_key.clear();
        for (int i = 0; i < S && i + S < nj; i++) {
            hipStream_t bs = ctx->bstream[i];
            if ((rc = hip_check(ctx, hipStreamBeginCapture(bs, hipStreamCaptureModeThreadLocal), "begin capture")) !=
                IBIP_OK)
                return rc;
            hipError_t e = hipSuccess;
            for (int32_t q = i + S; q < nj && e == hipSuccess; q += S) {
                const ibip_job& jb = jobs[order[q]];
                e = job_setup(bufs[q], states + q, jb.image, jb.inlets, jb.dims, jb.max_steps, jb.seq, bs, tiles);
            }
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(bs, &graph);
            if (e == hipSuccess) e = ee;
            if (e == hipSuccess) e = hipGraphInstantiate(&ctx->batch_exec[i], graph, nullptr, nullptr, 0);
            if (graph) (void)hipGraphDestroy(graph);
            if (e != hipSuccess) {
                ctx->batch_exec[i] = nullptr;
                return hip_check(ctx, e, "setup graph");
            }
        }
        ctx->batch_key = key;
    }
    const int32_t G = std::min<int32_t>(nj, S);  // jobs of the early launch
    // Each job's workgroup writes a completion record to host memory when its
    // loop ends, and the host starts that job's post-processing on the batch
    // streams while the launches still run the other (larger) jobs; the jobs
    // left when the launches end take their results from the state copy.
    if (!done_records(ctx, 4 * (size_t)nj)) return fail(ctx, IBIP_ENOMEM, "invade_batch: pinned allocation failed");
    for (int32_t q = 0; q < nj; q++) h_args[q].done = ctx->done_dev + 4 * q;
    while (ctx->job_ev.size() < (size_t)nj) {
        hipEvent_t e = nullptr;
        if ((rc = hip_check(ctx, hipEventCreateWithFlags(&e, hipEventDisableTiming), "event")) != IBIP_OK) return rc;
        ctx->job_ev.push_back(e);
    }
    Timer& tm = ctx->timer;
    hipStream_t sf = ctx->bfirst;
    // fork: every batch stream and the early-launch stream wait for the
    // caller's stream (inputs ready); the loop arguments go over first
    if ((rc = hip_check(ctx, hipEventRecord(ctx->bev[S], s0), "event")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipStreamWaitEvent(sf, ctx->bev[S], 0), "wait")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(d_args, h_args, sizeof(LoopArgs) * nj, hipMemcpyHostToDevice, sf),
                        "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipEventRecord(ctx->bev_first[S], sf), "event")) != IBIP_OK) return rc;
    // the first job of each stream (the S largest), set up directly; their
    // loops start on the early-launch stream as soon as those setups end
    for (int i = 0; i < G; i++) {
        hipStream_t bs = ctx->bstream[i];
        const ibip_job& jb = jobs[order[i]];
        if ((rc = hip_check(ctx, hipStreamWaitEvent(bs, ctx->bev[S], 0), "wait")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, job_setup(bufs[i], states + i, jb.image, jb.inlets, jb.dims, jb.max_steps, jb.seq,
                                           bs, tiles), "setup")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipEventRecord(ctx->bev_first[i], bs), "event")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipStreamWaitEvent(sf, ctx->bev_first[i], 0), "wait")) != IBIP_OK) return rc;
    }
    tm.mark(3, sf);
    hipLaunchKernelGGL(k_loop_batch<false>, dim3((unsigned)G), dim3(kLoopThreads), 0, sf, d_args);
    if ((rc = hip_check(ctx, hipGetLastError(), "batch loop launch")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipEventRecord(ctx->bev_first[S + 1], sf), "event")) != IBIP_OK) return rc;
    // the other jobs' setups (graph replays, after the first job's on each
    // stream), then their loops in a second launch; the state copy follows both
    for (int i = 0; i < G; i++) {
        hipStream_t bs = ctx->bstream[i];
        if (ctx->batch_exec[i] &&
            (rc = hip_check(ctx, hipGraphLaunch(ctx->batch_exec[i], bs), "setup graph launch")) != IBIP_OK)
            return rc;
        if ((rc = hip_check(ctx, hipEventRecord(ctx->bev[i], bs), "event")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipStreamWaitEvent(s0, ctx->bev[i], 0), "wait")) != IBIP_OK) return rc;
    }
    if ((rc = hip_check(ctx, hipStreamWaitEvent(s0, ctx->bev_first[S], 0), "wait")) != IBIP_OK) return rc;
    if (nj > G)
        hipLaunchKernelGGL(k_loop_batch<false>, dim3((unsigned)(nj - G)), dim3(kLoopThreads), 0, s0, d_args + G);
    if ((rc = hip_check(ctx, hipStreamWaitEvent(s0, ctx->bev_first[S + 1], 0), "wait")) != IBIP_OK) return rc;
    tm.mark(4, s0);
    if ((rc = hip_check(ctx, hipGetLastError(), "batch loop launch")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipMemcpyAsync(h_st, states, sizeof(LoopState) * nj, hipMemcpyDeviceToHost, s0),
                        "copy")) != IBIP_OK)
        return rc;
    if (!ctx->copy_ev &&
        (rc = hip_check(ctx, hipEventCreateWithFlags(&ctx->copy_ev, hipEventDisableTiming), "event")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipEventRecord(ctx->copy_ev, s0), "event")) != IBIP_OK) return rc;
    ibip_status first = IBIP_OK;
    // jobs with more distinct distance values than a job's rank tables hold
    // (their loop stopped before its first step): run alone afterwards
    std::vector<int32_t> alone;
    auto post = [&](int32_t q, uint32_t k, uint32_t err) -> ibip_status {
        ibip_job& jb = jobs[order[q]];
        jb.status = IBIP_OK;
        jb.n_steps = 0;
        if (err == 2) jb.status = IBIP_ENOSOLID;
        else if (err == 3) jb.status = IBIP_ECAPACITY;
        else if (err) jb.status = IBIP_EDEVICE;
        if (err == 3) {
            alone.push_back(q);
            return IBIP_OK;
        }
        if (jb.status != IBIP_OK) {
            if (first == IBIP_OK) first = (ibip_status)jb.status;
            return IBIP_OK;
        }
        const int64_t K = (int64_t)k - 1;
        jb.n_steps = K;
        return hip_check(ctx, job_post(bufs[q], states + q, jb.dims, K, jb.seq, jb.rad2, jb.M, jb.sat,
                                       ctx->bstream[q % S]), "post");
    };
    // per job: 0 = in the launch, 1 = continued on its batch stream after a
    // stop at a wide step, 2 = post-processing queued
    std::vector<uint8_t> phase(nj, 0);
    auto cont = [&](int32_t q) -> ibip_status {
        hipStream_t bs = ctx->bstream[q % S];
        LoopArgs la = h_args[q];
        la.done = nullptr;  // the continued loop reports through its state copy
        ibip_status r;
        if (tm.on) ctx->timing.wide_launches++;
        if ((r = hip_check(ctx, launch_wide_and_loop(la, nvox(jobs[order[q]].dims), bs), "wide launch")) != IBIP_OK)
            return r;
        if ((r = hip_check(ctx, hipMemcpyAsync(h_cont + q, states + q, sizeof(LoopState), hipMemcpyDeviceToHost, bs),
                           "copy")) != IBIP_OK)
            return r;
        phase[q] = 1;
        return hip_check(ctx, hipEventRecord(ctx->job_ev[q], bs), "event");
    };
    int32_t left = nj;
    bool launch_done = false;
    for (;;) {
        bool progress = false;
        for (int32_t q = 0; q < nj; q++) {
            if (phase[q] == 0) {
                if (__atomic_load_n(&ctx->done_host[4 * q], __ATOMIC_ACQUIRE) == 0) {
                    if (!launch_done) continue;
                    // the launch ended without a record: rejected before its loop
                    if ((rc = post(q, h_st[q].k, h_st[q].err)) != IBIP_OK) return rc;
                    phase[q] = 2;
                } else if (ctx->done_host[4 * q + 3] == LS_WIDE && ctx->done_host[4 * q + 2] == 0) {
                    if ((rc = cont(q)) != IBIP_OK) return rc;
                    progress = true;
                    continue;
                } else {
                    if ((rc = post(q, ctx->done_host[4 * q + 1], ctx->done_host[4 * q + 2])) != IBIP_OK) return rc;
                    phase[q] = 2;
                }
                left--;
                progress = true;
            } else if (phase[q] == 1) {
                const hipError_t qe = hipEventQuery(ctx->job_ev[q]);
                if (qe == hipErrorNotReady) continue;
                if ((rc = hip_check(ctx, qe, "event query")) != IBIP_OK) return rc;
                progress = true;
                if (h_cont[q].status == LS_WIDE && h_cont[q].err == 0) {
                    if ((rc = cont(q)) != IBIP_OK) return rc;
                    continue;
                }
                if ((rc = post(q, h_cont[q].k, h_cont[q].err)) != IBIP_OK) return rc;
                phase[q] = 2;
                left--;
            }
        }
        if (left == 0) break;
        if (!launch_done) {
            const hipError_t qe = hipEventQuery(ctx->copy_ev);
            if (qe == hipSuccess) {
                launch_done = true;
                if (tm.on) {
                    ctx->timing.loop_kernel_ms += tm.ms(3, 4);
                    ctx->timing.loop_launches++;
                }
                continue;  // a last pass over the records
            }
            if (qe != hipErrorNotReady) return hip_check(ctx, qe, "event query");
        }
        if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    if ((rc = hip_check(ctx, hipEventSynchronize(ctx->copy_ev), "sync")) != IBIP_OK) return rc;
    if (!launch_done && tm.on) {
        ctx->timing.loop_kernel_ms += tm.ms(3, 4);
        ctx->timing.loop_launches++;
    }
    for (int i = 0; i < S; i++) {
        if ((rc = hip_check(ctx, hipEventRecord(ctx->bev[i], ctx->bstream[i]), "event")) != IBIP_OK) return rc;
        if ((rc = hip_check(ctx, hipStreamWaitEvent(s0, ctx->bev[i], 0), "wait")) != IBIP_OK) return rc;
    }
    if ((rc = hip_check(ctx, hipStreamSynchronize(s0), "sync")) != IBIP_OK) return rc;
    // the jobs with too many ranks for the batch's tables take the
    // single-image path (its global-memory loop), one after another on the
    // context's stream, with the batch's readings (none); that replaces the
    // context's per-step arrays, so ibip_get_steps then refers to no call
    if (!alone.empty()) {
        const uint32_t readings = ctx->readings;
        ctx->readings = 0;
        for (int32_t q : alone) {
            ibip_job& jb = jobs[order[q]];
            ibip_invade_opts o{};
            o.max_steps = jb.max_steps;
            int64_t K = 0;
            ibip_status r = run_invade(ctx, jb.image, jb.inlets, jb.dims, &o, jb.seq, jb.rad2, jb.centre_step, &K);
            if (r == IBIP_OK && K > 0 && jb.M)
                r = hip_check(ctx, hipMemcpyAsync(jb.M, ctx->buf[B_M].p, sizeof(uint32_t) * K,
                                                  hipMemcpyDeviceToDevice, s0), "copy");
            if (r == IBIP_OK && K > 0 && jb.sat)
                r = hip_check(ctx, hipMemcpyAsync(jb.sat, ctx->buf[B_SAT].p, sizeof(double) * K,
                                                  hipMemcpyDeviceToDevice, s0), "copy");
            if (r == IBIP_OK) r = hip_check(ctx, hipStreamSynchronize(s0), "sync");
            jb.status = r;
            jb.n_steps = r == IBIP_OK ? K : 0;
            if (r != IBIP_OK && first == IBIP_OK) first = r;
        }
        ctx->readings = readings;
        ctx->have_steps = false;
    }
    if (first != IBIP_OK) return fail(ctx, first, "invade_batch: at least one job failed (see its status)");
    return IBIP_OK;
}

}  // namespace ibip
