// Internal declarations of the HIP library: context, scratch arena, error
// plumbing and the host-side launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/ibip.h"

namespace ibip {

// Distinct distance values the invasion loop keeps in LDS (bucket heads and
// tails of 4 bytes each, plus a two-level occupancy bitmap).
constexpr int kMaxRanks = 8192;
// A step with more centres than this is handed to the whole-GPU kernel.
constexpr uint32_t kWideRound = 8192;
// A step with at most this many centres runs in one wave, without barriers.
constexpr uint32_t kSmallRound = 128;
constexpr uint32_t kInf32 = 0xFFFFFFFFu;
// Streams a batch spreads its per-job setup and post-processing over.
constexpr int kBatchStreams = 8;

// Division of 32-bit values by a fixed divisor with a precomputed multiplier
// (Granlund & Montgomery, "Division by invariant integers using
// multiplication", 1994): q = (t + ((n - t) >> s1)) >> s2, t = mulhi(m, n).
struct FastDiv {
    uint32_t d, m, s1, s2;
};
inline FastDiv make_fastdiv(uint32_t d) {
    uint32_t l = 0;
    while (((uint64_t)1 << l) < d) l++;
    const uint64_t m = (((uint64_t)1 << 32) * (((uint64_t)1 << l) - d)) / d + 1;
    return FastDiv{d, (uint32_t)m, l < 1 ? l : 1u, l > 1 ? l - 1 : 0u};
}
__device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
    const uint32_t t = __umulhi(f.m, n);
    return (t + ((n - t) >> f.s1)) >> f.s2;
}

// Adds each thread's `v` into *dst with one global atomic per block (a
// single counter hit by every wave serialises at L2). Every thread of the
// block must call it; blockDim.x must be a multiple of 64 and <= 1024.
__device__ inline void block_add_u32(uint32_t* dst, uint32_t v) {
    __shared__ uint32_t part[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += part[w];
        if (t) atomicAdd(dst, t);
    }
}

// Sum of v over the block, added to one of kCountSlots words chosen by the
// block index: one word taking an atomic from every block of a large grid
// queues them all at one L2 channel. The count is the sum of the slots.
constexpr int kCountSlots = 64;
__device__ inline void block_add_slots(uint32_t* slots, uint32_t v) {
    __shared__ uint32_t part[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    if (lane == 0) part[wid] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); w++) t += part[w];
        if (t) atomicAdd(&slots[blockIdx.x % kCountSlots], t);
    }
}

// Per-key counts (keys >= 1, e.g. step numbers) over a grid whose blocks each
// cover a contiguous chunk of voxels. A block first sums its chunk in an LDS
// hash table and then adds each distinct key once, to one of kCntCopies
// copies of the count array (chosen by the block index; copy c starts at
// c * stride). Atomics on one global word, or on neighbouring words of one
// cache line, from every wave of a large grid serialise at one place; here a
// line takes at most one atomic per key from the blocks of its copy.
constexpr int kCntHash = 2048;  // table entries (power of two)
constexpr int kCntProbes = 16;  // a key that finds no slot goes straight to the copy
constexpr int kCntChunk = 4096; // voxels per block
constexpr int kCntCopies = 16;
struct CountTable {
    int32_t key[kCntHash];  // 0 = empty
    uint32_t cnt[kCntHash];
};

__device__ inline void count_table_clear(CountTable& t) {
    for (int i = threadIdx.x; i < kCntHash; i += blockDim.x) {
        t.key[i] = 0;
        t.cnt[i] = 0;
    }
}

// Adds 1 for every active lane to the count of its key. Runs of equal keys
// in consecutive lanes are added once, by the run's first lane.
__device__ inline void count_table_add(CountTable& t, bool act, int32_t key, uint32_t* copy) {
    const int lane = threadIdx.x & 63;
    const int32_t prev = __shfl_up(key, 1, 64);
    const bool prev_act = __shfl_up(act ? 1 : 0, 1, 64) != 0;
    const bool head = act && (lane == 0 || !prev_act || prev != key);
    const uint64_t brk = __ballot(!act || head);
    if (!head) return;
    // the run ends at the next lane that is inactive or starts another run
    const uint64_t after = lane == 63 ? 0ull : brk & (~0ull << (lane + 1));
    const uint32_t len = (uint32_t)((after ? __ffsll((unsigned long long)after) - 1 : 64) - lane);
    uint32_t h = ((uint32_t)key * 2654435761u) >> 21;  // 11 bits: kCntHash slots
    for (int p = 0; p < kCntProbes; p++) {
        const int32_t old = atomicCAS(&t.key[h], 0, key);
        if (old == 0 || old == key) {
            atomicAdd(&t.cnt[h], len);
            return;
        }
        h = (h + 1) & (kCntHash - 1);
    }
    atomicAdd(&copy[key - 1], len);
}

// After a barrier: each distinct key of the table is added to the copy.
__device__ inline void count_table_flush(const CountTable& t, uint32_t* copy) {
    for (int i = threadIdx.x; i < kCntHash; i += blockDim.x) {
        const int32_t k = t.key[i];
        if (k != 0) atomicAdd(&copy[k - 1], t.cnt[i]);
    }
}

// Makes `dev` current for a scope and restores the previous device after.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) prev = -1;
        if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
    }
    ~DeviceGuard() {
        if (prev >= 0) (void)hipSetDevice(prev);
    }
};

// One grow-only device allocation.
struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

enum BufId {
    B_KEY = 0,     // uint32[N]   dt2, then the rank of dt2 (0 = solid)
    B_STATE,       // int32[N]    k > 0 centre of step k, else 0
    B_BUCKET,      // uint32[N]   candidate voxel indices grouped by rank
    B_HIST,        // uint32[V]   histogram of dt2 values, then value -> rank
    B_OFF,         // uint32[R+2] bucket offsets by rank
    B_HEAD,        // uint32[R+1]
    B_TAIL,        // uint32[R+1]
    B_VAL,         // uint32[R+1] rank -> dt2 value
    B_M,           // uint32[K]   squared radius per step
    B_NNEW,        // int64[K]
    B_SAT,         // double[K]
    B_PC,          // double[K]
    B_FULL,        // uint32[N]   centres that need a full ball
    B_MISC,        // small control block (LoopState and counters)
    B_TMP0,        // generic N-sized scratch
    B_TMP1,
    B_TMP2,
    B_SCAN,        // scan partials
    B_ACT,         // uint8[2 * tiles] active-tile flags of the reconstruction
    B_CNT,         // uint32 per-sweep change counters
    B_BATCH,       // arena of a batch of jobs
    B_SATW,        // counts and scan of ibip_saturation
    B_MIOCNT,      // per-level counts of the opening (kept apart from B_M, which ibip_get_steps reads)
    B_GBITS,       // occupancy bitmap of the global-memory step loop (more ranks than LDS holds)
    B_NUM
};

// Device-side control block of the invasion loop (lives in B_MISC).
struct LoopState {
    uint32_t k;        // next step number
    uint32_t status;   // LoopStatus
    uint32_t R;        // number of ranks
    uint32_t big_r;    // pending wide step: rank, bucket range [big_h, big_t)
    uint32_t big_h;
    uint32_t big_t;
    uint32_t n_pore;
    uint32_t maxval;   // largest dt2 value
    uint32_t solid_seen;
    uint32_t n_full;   // centres that need a full ball
    uint32_t err;
    uint32_t big_k;    // step number of the pending wide step
    uint32_t popped;   // centres of the steps the loop kernels ran (wide steps not included)
    uint32_t pad2;     // resumption: set when the checkpoint is not a valid one
    int64_t max_steps;
    uint32_t full_done;  // full-ball list entries painted by earlier insertion passes
    uint32_t pad3;
};

enum LoopStatus : uint32_t { LS_RUN = 0, LS_DONE = 1, LS_WIDE = 2, LS_MAXSTEPS = 3, LS_CANCEL = 4 };

}  // namespace ibip

namespace ibip {
// Optional event-based phase timer (see ibip_timing).
struct Timer {
    bool on = false;
    hipEvent_t ev[16] = {};
    bool made = false;
    // record event i on stream s (no-op when off)
    void mark(int i, hipStream_t s) {
        if (!on) return;
        if (!made) {
            for (auto& e : ev) (void)hipEventCreate(&e);
            made = true;
        }
        (void)hipEventRecord(ev[i], s);
    }
    // elapsed ms between events a and b (both recorded and complete)
    double ms(int a, int b) const {
        float t = 0.f;
        if (!on || !made) return 0.0;
        if (hipEventElapsedTime(&t, ev[a], ev[b]) != hipSuccess) return 0.0;
        return (double)t;
    }
};
}  // namespace ibip

struct ibip_ctx {
    ibip::Timer timer;
    hipStream_t bstream[ibip::kBatchStreams] = {};
    hipEvent_t bev[ibip::kBatchStreams + 1] = {};
    // the batch's first jobs (one per batch stream, the largest) start their
    // loops on their own stream as soon as their setups are done
    hipStream_t bfirst = nullptr;
    hipEvent_t bev_first[ibip::kBatchStreams + 2] = {};
    // the batch's setup captured as one graph per batch stream, and the
    // batch it was captured for
    hipGraphExec_t batch_exec[ibip::kBatchStreams] = {};  // each stream's setups after its first job's
    std::vector<uint64_t> batch_key;
    bool have_bstreams = false;
    ibip_timing timing = {};
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    ibip::Buf buf[ibip::B_NUM];
    void* host_pinned = nullptr;   // pinned mirror of LoopState and small results
    hipEvent_t copy_ev = nullptr;  // the loop state's copy to the host (no timing)
    // sphere insertion of finished steps while the step loop runs (ibip_invade)
    hipStream_t paint_stream = nullptr;
    hipEvent_t paint_ev = nullptr;
    std::vector<hipEvent_t> job_ev;  // per batch job: its continued loop's state copy
    // per-job completion records of a batch (4 words each: done, k, err,
    // loop status) in
    // coherent pinned host memory that the loop kernel writes directly
    uint32_t* done_host = nullptr;
    uint32_t* done_dev = nullptr;
    size_t done_words = 0;
    size_t host_pinned_bytes = 0;
    // results of the last invade
    int64_t last_K = -1;
    int64_t last_n_pore = 0;
    bool have_steps = false;
    uint32_t readings = 0;         // IBIP_READ_* flags for the following calls
    ibip_tuning tuning = {};       // launch parameters (zero: defaults)
};

namespace ibip {

// Set ctx->err and return `st`.
ibip_status fail(ibip_ctx* ctx, ibip_status st, const std::string& what);
// Map a HIP error to IBIP_EDEVICE with a message; IBIP_OK if e == hipSuccess.
ibip_status hip_check(ibip_ctx* ctx, hipError_t e, const char* what);
// Ensure buffer `id` holds at least `bytes`; returns its pointer or nullptr.
void* ensure(ibip_ctx* ctx, BufId id, size_t bytes);
void* pinned(ibip_ctx* ctx, size_t bytes);
// ctx->done_host/done_dev with at least `words` words, zeroed; false on failure.
bool done_records(ibip_ctx* ctx, size_t words);
bool dims_ok(ibip_dims d);
inline int64_t nvox(ibip_dims d) { return (int64_t)d.X * d.Y * d.Z; }

// ---- launchers (each returns hipSuccess or the first launch error) ----
// EDT: dt2 = squared distance to the nearest voxel with feature != 0, where
// feature(v) = (image[v] == 0) when `image` is given, else (w[v] >= thr).
// With cap > 0 the result is exact where it is below cap and 0xFFFFFFFF
// elsewhere (the searches stop at cap). Sets *solid_flag (device) to 1 if any
// feature voxel exists.
// With mio_r2 given (opening drainage), the last pass writes no distances:
// it sets mio_r2[v] = cap where mio_r2[v] == 0 and dt2 < cap, and adds the
// number of voxels with mio_r2 >= cap to *mio_count.
// Tile widths (z columns) of the LDS-tiled passes y and x.
struct EdtTiles {
    int y = 32;  // 32 or 64
    int x = 32;  // 16 or 32
};
hipError_t launch_edt(const uint8_t* image, const uint32_t* w, uint32_t thr, uint32_t cap, ibip_dims d,
                      uint16_t* g16, uint32_t* tmp32, uint32_t* out, uint32_t* solid_flag,
                      hipStream_t s, uint32_t* mio_r2 = nullptr, uint32_t* mio_count = nullptr,
                      EdtTiles tiles = EdtTiles{});

// *dst = the sum of kCountSlots slot words (see block_add_slots).
hipError_t launch_sum_slots(const uint32_t* slots, uint32_t* dst, hipStream_t s);
// out[k] = sum over c < copies of in[c * K + k], for k < K (see count_table_flush).
hipError_t launch_sum_copies(const uint32_t* in, int copies, int64_t K, uint32_t* out, hipStream_t s);
// Number of count copies for K keys over n voxels: kCntCopies when the
// copies take at most 4 B per voxel, else 1.
inline int count_copies(int64_t K, int64_t n) { return K > 0 && (int64_t)kCntCopies * K <= n ? kCntCopies : 1; }
// Exclusive scan of n uint32 values in place; returns the total in *total (device).
hipError_t launch_scan_u32(uint32_t* data, int64_t n, uint32_t* partials, uint32_t* total,
                           hipStream_t s);

// Maximin reconstruction: w[v] = max over face-connected paths from the seeds
// to v of the smallest cap along the path. On entry w holds the seed values
// (w <= cap) and 0 elsewhere. cap(v) is cap32[v] when cap32 is given, else it
// is derived from a step image: 0 on solid (seq < 0), 0xFFFFFFFF on uninvaded
// pore (seq == 0), seq[v] on invaded voxels. Iterates to the fixed point;
// *n_iter receives the number of sweeps.
ibip_status reconstruct(ibip_ctx* ctx, const int32_t* seq, const uint32_t* cap32, bool conn26, ibip_dims d,
                        uint32_t* w, int* n_iter);

// resume_cs / k_done: a checkpoint (the centres of steps 1..k_done) to resume from, or null
ibip_status run_invade(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims d,
                       const ibip_invade_opts* opts, int32_t* seq, uint32_t* rad2, int32_t* centre_step,
                       int64_t* n_steps, const int32_t* resume_cs = nullptr, int64_t k_done = 0);
ibip_status run_invade_batch(ibip_ctx* ctx, ibip_job* jobs, int32_t n);

// ---- one job of the batch / server paths (invade.hip) ----
// Per-job scratch carved from one region, so jobs run concurrently.
struct JobBufs {
    uint32_t* key;
    int32_t* state;
    uint32_t* bucket;
    uint32_t* hist;
    uint16_t* g16;
    uint32_t* tmp32;
    uint32_t* partials;
    uint32_t* val;
    uint32_t* off;
    uint32_t* head;
    uint32_t* tail;
    uint32_t* M;
    uint32_t* full;
    uint32_t* counts;  // 2 (N + 1) entries, only when saturation is requested
    uint32_t* scan_total;
};
inline size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
int64_t value_range(ibip_dims d);
// bytes of one job's scratch (own_state: no caller centre_step buffer)
size_t job_bytes(ibip_dims d, bool own_state, bool want_sat);
JobBufs carve(uint8_t* base, ibip_dims d, int32_t* caller_state, bool want_sat);
// EDT, ranks, slices and seeds; loop state initialised on the device
hipError_t job_setup(const JobBufs& j, LoopState* st, const uint8_t* image, const uint8_t* inlets, ibip_dims d,
                     int64_t max_steps, int32_t* seq, hipStream_t s, EdtTiles tiles = EdtTiles{});
// EDT tile widths from a tuning (defaults where it holds 0)
inline EdtTiles edt_tiles(const ibip_tuning& t) {
    EdtTiles e;
    if (t.edt_tile_y) e.y = t.edt_tile_y;
    if (t.edt_tile_x) e.x = t.edt_tile_x;
    return e;
}
// true when the tuning's values are among the accepted ones
inline bool tuning_ok(const ibip_tuning& t) {
    return (t.edt_tile_y == 0 || t.edt_tile_y == 32 || t.edt_tile_y == 64) &&
           (t.edt_tile_x == 0 || t.edt_tile_x == 16 || t.edt_tile_x == 32);
}
// post-processing with K read on the device (no host sync)
hipError_t job_post_devk(const JobBufs& j, LoopState* st, ibip_dims d, int32_t* seq, uint32_t* rad2,
                         uint32_t* M_out, hipStream_t s);
size_t loop_args_bytes();
// fills `out` (loop_args_bytes() of host memory) with the loop arguments of a job
void fill_loop_args(void* out, const JobBufs& j, LoopState* st, ibip_dims d, uint32_t wide);
// the loop of `args` stops with LS_CANCEL when *flag (device-visible host
// memory) is nonzero at one of its checks (every 1024 steps)
void set_loop_cancel(void* args, const uint32_t* flag);
// the step-count threshold above which a batch or served job's step runs over
// the whole GPU, from a tuning value (0: kWideRound; negative: never)
uint32_t wide_threshold(int64_t tuned);
// after a job's loop stopped at a wide step (its state on the device says
// so): that step over the whole GPU, then the job's loop in one workgroup to
// its next wide step or its end, stream-ordered on s. host_args: the job's
// loop arguments (fill_loop_args); n: its voxel count.
hipError_t launch_wide_and_loop_host(const void* host_args, int64_t n, hipStream_t s);
// one workgroup per job, every step loop to completion (served jobs: each loop
// checks its cancel flag)
hipError_t launch_loop_jobs(const void* d_args, int32_t n, hipStream_t s);
// create the batch streams and events once per context
ibip_status batch_streams(ibip_ctx* ctx);
ibip_status run_trap(ibip_ctx* ctx, const int32_t* seq, const uint8_t* outlets, ibip_dims d,
                     uint8_t* trapped, int32_t* seq_trapped, int64_t* n_steps_after);
ibip_status run_mio(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims d,
                    const uint32_t* T, int32_t n, uint32_t* mio_r2, double* mio_sat);

}  // namespace ibip
