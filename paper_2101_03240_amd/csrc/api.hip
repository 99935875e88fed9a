// C ABI of the library (declared in include/ibip.h): context, scratch arena,
// argument checks and error plumbing around the kernels of edt.hip,
// invade.hip, trap.hip and mio.hip.
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>

#include "ibip_internal.h"

namespace ibip {

// Scratch of ibip_edt_noalloc: the z pass's uint16 distances (2 B per voxel)
// followed by the y pass's uint32 values (4 B per voxel) of one image of at
// most kNoAllocMaxVoxels voxels. Every device the library runs on holds one
// copy for the life of the process. Host code never passes `scratch` itself
// to a kernel (in host code the name is only a stand-in): it uses the
// device address that hipGetSymbolAddress returned for the current device.
constexpr int64_t kNoAllocMaxVoxels = (int64_t)1 << 24;
constexpr size_t kNoAllocScratchBytes = (size_t)6 << 24;
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[kMaxDevices];
std::atomic<int> g_scratch_state[kMaxDevices];  // 0 not looked up, 1 ok, -1 lookup failed

// The address of `scratch` on `device`, looked up once per device with that
// device current (the caller's DeviceGuard makes it current).
void* scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) return nullptr;
    if (g_scratch_state[device].load(std::memory_order_acquire) == 0) {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_state[device].load(std::memory_order_relaxed) == 0) {
            void* p = nullptr;
            const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                g_scratch_state[device].store(-1, std::memory_order_release);
            } else {
                g_scratch_ptr[device].store(p, std::memory_order_relaxed);
                g_scratch_state[device].store(1, std::memory_order_release);
            }
        }
    }
    return g_scratch_state[device].load(std::memory_order_acquire) == 1
               ? g_scratch_ptr[device].load(std::memory_order_relaxed)
               : nullptr;
}

__global__ void k_clear_word(uint32_t* w) { *w = 0u; }
}  // namespace

ibip_status fail(ibip_ctx* ctx, ibip_status st, const std::string& what) {
    if (ctx) ctx->err = what;
    return st;
}

ibip_status hip_check(ibip_ctx* ctx, hipError_t e, const char* what) {
    if (e == hipSuccess) return IBIP_OK;
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(ctx, e == hipErrorOutOfMemory ? IBIP_ENOMEM : IBIP_EDEVICE, m);
}

void* ensure(ibip_ctx* ctx, BufId id, size_t bytes) {
    Buf& b = ctx->buf[id];
    if (bytes == 0) bytes = 16;
    if (b.bytes >= bytes) return b.p;
    if (b.p) {
        // the old buffer may still be in use by queued work on our stream
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return nullptr;
        (void)hipFree(b.p);
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes + bytes / 8;  // some headroom for slightly larger calls
    void* p = nullptr;
    if (hipMalloc(&p, want) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    b.p = p;
    b.bytes = want;
    return p;
}

bool done_records(ibip_ctx* ctx, size_t words) {
    if (ctx->done_words < words) {
        if (ctx->done_host) {
            if (hipStreamSynchronize(ctx->stream) != hipSuccess) return false;
            (void)hipHostFree(ctx->done_host);
            ctx->done_host = ctx->done_dev = nullptr;
            ctx->done_words = 0;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, words * sizeof(uint32_t), hipHostMallocCoherent | hipHostMallocMapped) != hipSuccess) {
            (void)hipGetLastError();
            return false;
        }
        void* d = nullptr;
        if (hipHostGetDevicePointer(&d, p, 0) != hipSuccess) {
            (void)hipGetLastError();
            (void)hipHostFree(p);
            return false;
        }
        ctx->done_host = (uint32_t*)p;
        ctx->done_dev = (uint32_t*)d;
        ctx->done_words = words;
    }
    std::memset(ctx->done_host, 0, words * sizeof(uint32_t));
    return true;
}

void* pinned(ibip_ctx* ctx, size_t bytes) {
    if (ctx->host_pinned_bytes >= bytes) return ctx->host_pinned;
    if (ctx->host_pinned) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return nullptr;
        (void)hipHostFree(ctx->host_pinned);
        ctx->host_pinned = nullptr;
        ctx->host_pinned_bytes = 0;
    }
    void* p = nullptr;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    std::memset(p, 0, bytes);
    ctx->host_pinned = p;
    ctx->host_pinned_bytes = bytes;
    return p;
}

ibip_status batch_streams(ibip_ctx* ctx) {
    if (ctx->have_bstreams) return IBIP_OK;
    for (auto& st : ctx->bstream)
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess)
            return fail(ctx, IBIP_EDEVICE, "cannot create batch streams");
    for (auto& e : ctx->bev)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(ctx, IBIP_EDEVICE, "cannot create batch events");
    for (auto& e : ctx->bev_first)
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess)
            return fail(ctx, IBIP_EDEVICE, "cannot create batch events");
    if (hipStreamCreateWithFlags(&ctx->bfirst, hipStreamNonBlocking) != hipSuccess)
        return fail(ctx, IBIP_EDEVICE, "cannot create batch streams");
    ctx->have_bstreams = true;
    return IBIP_OK;
}

bool dims_ok(ibip_dims d) {
    if (d.X <= 0 || d.Y <= 0 || d.Z <= 0) return false;
    if (d.X > 65535 || d.Y > 65535 || d.Z > 65535) return false;
    return nvox(d) < ((int64_t)1 << 31);
}

}  // namespace ibip

using namespace ibip;

extern "C" {

ibip_status ibip_ctx_set_readings(ibip_ctx* ctx, uint32_t flags) {
    if (!ctx) return IBIP_EINVAL;
    if (flags & ~(IBIP_READ_INTEGER_BALL | IBIP_READ_MASK_INLETS | IBIP_READ_TRAP26))
        return fail(ctx, IBIP_EINVAL, "set_readings: unknown flag");
    ctx->readings = flags;
    return IBIP_OK;
}

ibip_status ibip_ctx_create(ibip_ctx** out, int32_t device, void* stream) {
    if (!out) return IBIP_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return IBIP_EDEVICE;
    ibip_ctx* ctx = new (std::nothrow) ibip_ctx();
    if (!ctx) return IBIP_ENOMEM;
    {
        // the device address of the no-allocation scratch, looked up once
        // per device while that device is current (a failed lookup is
        // reported by ibip_edt_noalloc)
        DeviceGuard g(device);
        if (g.ok) (void)scratch_on(device);
    }
    ctx->device = device;
    ctx->stream = (hipStream_t)stream;
    *out = ctx;
    return IBIP_OK;
}

ibip_status ibip_ctx_set_tuning(ibip_ctx* ctx, const ibip_tuning* t) {
    if (!ctx) return IBIP_EINVAL;
    if (!t) {
        ctx->tuning = ibip_tuning{};
        return IBIP_OK;
    }
    if (!tuning_ok(*t)) return fail(ctx, IBIP_EINVAL, "set_tuning: tile width not among 32/64 (y) and 16/32 (x)");
    ctx->tuning = *t;
    return IBIP_OK;
}

ibip_status ibip_ctx_get_tuning(const ibip_ctx* ctx, ibip_tuning* out) {
    if (!ctx || !out) return IBIP_EINVAL;
    *out = ctx->tuning;
    return IBIP_OK;
}

ibip_status ibip_ctx_enable_timing(ibip_ctx* ctx, int32_t enable) {
    if (!ctx) return IBIP_EINVAL;
    ctx->timer.on = enable != 0;
    return IBIP_OK;
}

ibip_status ibip_ctx_get_timing(const ibip_ctx* ctx, ibip_timing* out) {
    if (!ctx || !out) return IBIP_EINVAL;
    *out = ctx->timing;
    return IBIP_OK;
}

ibip_status ibip_ctx_reset_timing(ibip_ctx* ctx) {
    if (!ctx) return IBIP_EINVAL;
    ctx->timing = ibip_timing{};
    return IBIP_OK;
}

ibip_status ibip_ctx_destroy(ibip_ctx* ctx) {
    if (!ctx) return IBIP_EINVAL;
    DeviceGuard g(ctx->device);
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->have_bstreams) {
        for (auto& st : ctx->bstream) (void)hipStreamDestroy(st);
        for (auto& e : ctx->bev) (void)hipEventDestroy(e);
        for (auto& e : ctx->bev_first) (void)hipEventDestroy(e);
        if (ctx->bfirst) (void)hipStreamDestroy(ctx->bfirst);
    }
    if (ctx->timer.made)
        for (auto& e : ctx->timer.ev) (void)hipEventDestroy(e);
    if (ctx->copy_ev) (void)hipEventDestroy(ctx->copy_ev);
    if (ctx->paint_ev) (void)hipEventDestroy(ctx->paint_ev);
    if (ctx->paint_stream) (void)hipStreamDestroy(ctx->paint_stream);
    for (auto& e : ctx->job_ev) (void)hipEventDestroy(e);
    for (auto& g : ctx->batch_exec)
        if (g) (void)hipGraphExecDestroy(g);
    for (auto& b : ctx->buf)
        if (b.p) (void)hipFree(b.p);
    if (ctx->host_pinned) (void)hipHostFree(ctx->host_pinned);
    if (ctx->done_host) (void)hipHostFree(ctx->done_host);
    delete ctx;
    return IBIP_OK;
}

ibip_status ibip_ctx_set_stream(ibip_ctx* ctx, void* stream) {
    if (!ctx) return IBIP_EINVAL;
    ctx->stream = (hipStream_t)stream;
    return IBIP_OK;
}

const char* ibip_last_error(const ibip_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

namespace {

// buf[i] = the next index of the chain: a fixed odd stride of more than a
// cache line, so consecutive claims touch different lines
__global__ void k_probe_fill(uint32_t* buf, uint32_t span) {
    const uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < span) buf[i] = (uint32_t)((i + 32673u) % span);
}

__global__ void k_probe_chase(uint32_t* buf, int32_t n, uint32_t* out) {
    uint32_t i = 0;
    for (int32_t j = 0; j < n; j++) i = atomicOr(&buf[i], 0u);
    *out = i;
}

}  // namespace

ibip_status ibip_probe_claim_latency(ibip_ctx* ctx, int64_t span_bytes, int32_t n_chain, double* ns_per_claim) {
    if (!ctx) return IBIP_EINVAL;
    if (!ns_per_claim || span_bytes < 4096 || span_bytes >= ((int64_t)1 << 34) || n_chain < 1)
        return fail(ctx, IBIP_EINVAL, "probe: bad arguments");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "probe: cannot select device");
    const uint32_t span = (uint32_t)(span_bytes / 4);
    uint32_t* buf = (uint32_t*)ensure(ctx, B_TMP0, (size_t)span * 4 + 256);
    if (!buf) return fail(ctx, IBIP_ENOMEM, "probe: allocation failed");
    hipStream_t s = ctx->stream;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ibip_status rc;
    if ((rc = hip_check(ctx, hipEventCreate(&e0), "event")) != IBIP_OK) return rc;
    if ((rc = hip_check(ctx, hipEventCreate(&e1), "event")) != IBIP_OK) {
        (void)hipEventDestroy(e0);
        return rc;
    }
    hipLaunchKernelGGL(k_probe_fill, dim3((span + 255) / 256), dim3(256), 0, s, buf, span);
    // one short chase first, so that the timed one finds the code and the
    // buffer's pages ready
    hipLaunchKernelGGL(k_probe_chase, dim3(1), dim3(1), 0, s, buf, std::min(n_chain, 64), buf + span);
    (void)hipEventRecord(e0, s);
    hipLaunchKernelGGL(k_probe_chase, dim3(1), dim3(1), 0, s, buf, n_chain, buf + span);
    (void)hipEventRecord(e1, s);
    rc = hip_check(ctx, hipGetLastError(), "probe launch");
    if (rc == IBIP_OK) rc = hip_check(ctx, hipEventSynchronize(e1), "sync");
    float ms = 0.f;
    if (rc == IBIP_OK) rc = hip_check(ctx, hipEventElapsedTime(&ms, e0, e1), "event");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != IBIP_OK) return rc;
    *ns_per_claim = (double)ms * 1e6 / (double)n_chain;
    return IBIP_OK;
}

int64_t ibip_ctx_scratch_bytes(const ibip_ctx* ctx) {
    if (!ctx) return -1;
    int64_t t = 0;
    for (const auto& b : ctx->buf) t += (int64_t)b.bytes;
    return t;
}

ibip_status ibip_edt(ibip_ctx* ctx, const uint8_t* image, ibip_dims dims, uint32_t* dt2) {
    if (!ctx) return IBIP_EINVAL;
    if (!image || !dt2) return fail(ctx, IBIP_EINVAL, "edt: null pointer");
    if (!dims_ok(dims)) return fail(ctx, IBIP_EINVAL, "edt: bad dims");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "edt: cannot select device");
    const int64_t n = nvox(dims);
    uint16_t* g16 = (uint16_t*)ensure(ctx, B_TMP0, sizeof(uint16_t) * n);
    uint32_t* tmp = (uint32_t*)ensure(ctx, B_TMP1, sizeof(uint32_t) * n);
    uint8_t* misc = (uint8_t*)ensure(ctx, B_MISC, 4096);
    uint32_t* h = (uint32_t*)pinned(ctx, 4096);
    if (!g16 || !tmp || !misc || !h) return fail(ctx, IBIP_ENOMEM, "edt: allocation failed");
    uint32_t* flag = (uint32_t*)(misc + 3600);
    ibip_status rc;
    if ((rc = hip_check(ctx, hipMemsetAsync(flag, 0, 4, ctx->stream), "memset")) != IBIP_OK) return rc;
    ctx->timer.mark(0, ctx->stream);
    if ((rc = hip_check(ctx, launch_edt(image, nullptr, 0, 0, dims, g16, tmp, dt2, flag, ctx->stream, nullptr, nullptr,
                                         edt_tiles(ctx->tuning)), "edt launch")) !=
        IBIP_OK)
        return rc;
    ctx->timer.mark(1, ctx->stream);
    if ((rc = hip_check(ctx, hipMemcpyAsync(h, flag, 4, hipMemcpyDeviceToHost, ctx->stream), "copy")) != IBIP_OK)
        return rc;
    if ((rc = hip_check(ctx, hipStreamSynchronize(ctx->stream), "sync")) != IBIP_OK) return rc;
    if (ctx->timer.on) ctx->timing.edt_ms += ctx->timer.ms(0, 1);  // the three passes' kernels
    if (!h[0]) return fail(ctx, IBIP_ENOSOLID, "edt: image holds no solid voxel");
    return IBIP_OK;
}

ibip_status ibip_edt_noalloc(ibip_ctx* ctx, const uint8_t* image, ibip_dims dims, uint32_t* dt2,
                             uint32_t* solid_flag) {
    if (!ctx) return IBIP_EINVAL;
    if (!image || !dt2 || !solid_flag) return fail(ctx, IBIP_EINVAL, "edt_noalloc: null pointer");
    if (!dims_ok(dims)) return fail(ctx, IBIP_EINVAL, "edt_noalloc: bad dims");
    const int64_t n = nvox(dims);
    if (n > kNoAllocMaxVoxels)
        return fail(ctx, IBIP_ECAPACITY,
                    "edt_noalloc: the image has more than 2^24 voxels, the limit of the fixed scratch");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "edt_noalloc: cannot select device");
    uint8_t* base = (uint8_t*)scratch_on(ctx->device);
    if (!base) return fail(ctx, IBIP_EDEVICE, "edt_noalloc: no device address for the fixed scratch");
    uint16_t* g16 = (uint16_t*)base;
    uint32_t* tmp = (uint32_t*)(base + align256(sizeof(uint16_t) * (size_t)n));
    hipLaunchKernelGGL(k_clear_word, dim3(1), dim3(1), 0, ctx->stream, solid_flag);
    return hip_check(ctx, launch_edt(image, nullptr, 0, 0, dims, g16, tmp, dt2, solid_flag, ctx->stream, nullptr, nullptr,
                                      edt_tiles(ctx->tuning)),
                     "edt_noalloc launch");
}

ibip_status ibip_invade(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims dims,
                        const ibip_invade_opts* opts, int32_t* seq, uint32_t* rad2, int32_t* centre_step,
                        int64_t* n_steps) {
    if (!ctx) return IBIP_EINVAL;
    if (!image || !inlets || !seq) return fail(ctx, IBIP_EINVAL, "invade: null pointer");
    if (!dims_ok(dims)) return fail(ctx, IBIP_EINVAL, "invade: bad dims");
    if (opts && opts->max_steps < 0) return fail(ctx, IBIP_EINVAL, "invade: max_steps < 0");
    if (opts && (opts->voxel_size < 0.0)) return fail(ctx, IBIP_EINVAL, "invade: voxel_size < 0");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "invade: cannot select device");
    return run_invade(ctx, image, inlets, dims, opts, seq, rad2, centre_step, n_steps);
}

ibip_status ibip_invade_resume(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims dims,
                               const ibip_invade_opts* opts, const int32_t* centre_step_in, int64_t k_done,
                               int32_t* seq, uint32_t* rad2, int32_t* centre_step, int64_t* n_steps) {
    if (!ctx) return IBIP_EINVAL;
    if (!image || !inlets || !seq || !centre_step_in) return fail(ctx, IBIP_EINVAL, "invade_resume: null pointer");
    if (!dims_ok(dims)) return fail(ctx, IBIP_EINVAL, "invade_resume: bad dims");
    if (k_done < 0) return fail(ctx, IBIP_EINVAL, "invade_resume: k_done < 0");
    if (centre_step == centre_step_in)
        return fail(ctx, IBIP_EINVAL, "invade_resume: centre_step must not be the checkpoint's buffer");
    if (opts && opts->max_steps < 0) return fail(ctx, IBIP_EINVAL, "invade_resume: max_steps < 0");
    if (opts && opts->max_steps > 0 && opts->max_steps < k_done)
        return fail(ctx, IBIP_EINVAL, "invade_resume: max_steps below the steps already done");
    if (opts && (opts->voxel_size < 0.0)) return fail(ctx, IBIP_EINVAL, "invade_resume: voxel_size < 0");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "invade_resume: cannot select device");
    return run_invade(ctx, image, inlets, dims, opts, seq, rad2, centre_step, n_steps, centre_step_in, k_done);
}

ibip_status ibip_invade_batch(ibip_ctx* ctx, ibip_job* jobs, int32_t n) {
    if (!ctx) return IBIP_EINVAL;
    if (n < 0 || (n > 0 && !jobs)) return fail(ctx, IBIP_EINVAL, "invade_batch: bad job list");
    for (int32_t i = 0; i < n; i++) {
        const ibip_job& j = jobs[i];
        if (!j.image || !j.inlets || !j.seq) return fail(ctx, IBIP_EINVAL, "invade_batch: null pointer in a job");
        if (!dims_ok(j.dims)) return fail(ctx, IBIP_EINVAL, "invade_batch: bad dims in a job");
        if (j.max_steps < 0) return fail(ctx, IBIP_EINVAL, "invade_batch: max_steps < 0");
    }
    if (n == 0) return IBIP_OK;
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "invade_batch: cannot select device");
    return run_invade_batch(ctx, jobs, n);
}

ibip_status ibip_get_steps(ibip_ctx* ctx, uint32_t* M, int64_t* n_new, double* sat, double* pc, int64_t capacity) {
    if (!ctx) return IBIP_EINVAL;
    if (!ctx->have_steps) return fail(ctx, IBIP_EINVAL, "get_steps: no completed invade on this context");
    const int64_t K = ctx->last_K;
    if (capacity < K) return fail(ctx, IBIP_ECAPACITY, "get_steps: capacity below the number of steps");
    if (K == 0) return IBIP_OK;
    DeviceGuard g(ctx->device);
    hipStream_t s = ctx->stream;
    ibip_status rc;
    struct { void* dst; BufId id; size_t sz; } items[4] = {
        {M, B_M, sizeof(uint32_t)}, {n_new, B_NNEW, sizeof(int64_t)}, {sat, B_SAT, sizeof(double)},
        {pc, B_PC, sizeof(double)}};
    for (auto& it : items) {
        if (!it.dst) continue;
        if ((rc = hip_check(ctx, hipMemcpyAsync(it.dst, ctx->buf[it.id].p, it.sz * K, hipMemcpyDeviceToDevice, s),
                            "get_steps copy")) != IBIP_OK)
            return rc;
    }
    return IBIP_OK;
}

ibip_status ibip_trap(ibip_ctx* ctx, const int32_t* seq, const uint8_t* outlets, ibip_dims dims, uint8_t* trapped,
                      int32_t* seq_trapped, int64_t* n_steps_after) {
    if (!ctx) return IBIP_EINVAL;
    if (!seq || !outlets || !trapped) return fail(ctx, IBIP_EINVAL, "trap: null pointer");
    if (!dims_ok(dims)) return fail(ctx, IBIP_EINVAL, "trap: bad dims");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "trap: cannot select device");
    return run_trap(ctx, seq, outlets, dims, trapped, seq_trapped, n_steps_after);
}

ibip_status ibip_opening_drainage(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims dims,
                                  const uint32_t* r2_thresholds, int32_t n, uint32_t* mio_r2, double* mio_sat) {
    if (!ctx) return IBIP_EINVAL;
    if (!image || !inlets || !mio_r2 || (n > 0 && !r2_thresholds))
        return fail(ctx, IBIP_EINVAL, "opening_drainage: null pointer");
    if (n < 0) return fail(ctx, IBIP_EINVAL, "opening_drainage: n < 0");
    if (!dims_ok(dims)) return fail(ctx, IBIP_EINVAL, "opening_drainage: bad dims");
    for (int32_t i = 0; i < n; i++)
        if (r2_thresholds[i] == 0 || (i > 0 && r2_thresholds[i] >= r2_thresholds[i - 1]))
            return fail(ctx, IBIP_EINVAL, "opening_drainage: thresholds must be >= 1 and strictly decreasing");
    DeviceGuard g(ctx->device);
    if (!g.ok) return fail(ctx, IBIP_EDEVICE, "opening_drainage: cannot select device");
    return run_mio(ctx, image, inlets, dims, r2_thresholds, n, mio_r2, mio_sat);
}

}  // extern "C"
