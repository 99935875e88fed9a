/*
 * ibip.h -- C ABI of the MI355X (gfx950) image-based invasion percolation
 * library: exact squared Euclidean distance transform, volume-controlled
 * invasion of a non-wetting fluid, defender trapping and pressure-based
 * morphological-opening drainage on binary voxel images, after Gostick, Yang
 * & Boek, "Simulating volume-controlled invasion of a non-wetting fluid in
 * volumetric images using basic image processing tools" (arXiv 2101.03240).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Grid: dims {X, Y, Z}, C order, voxel v = (x*Y + y)*Z + z, x slowest.
 *    2D images are X = 1. N = X*Y*Z must be below 2^31.
 *  - image: uint8, nonzero = pore (void), zero = solid.
 *  - Every N-sized array is a caller-owned DEVICE buffer on the context's
 *    device (e.g. a torch tensor's data pointer), contiguous in C order.
 *    Inputs are never written. Outputs are fully overwritten.
 *  - Calls are ordered on the context's stream (ibip_ctx_set_stream); calls
 *    that return a host-side count (n_steps, n_steps_after) synchronise that
 *    stream before returning, the others do not.
 *  - A context is used by one host thread at a time. The library owns only
 *    the context and its scratch arena, which grows on demand and is freed by
 *    ibip_ctx_destroy.
 *  - Every call returns an ibip_status; on error the outputs are unspecified
 *    and ibip_last_error() describes the failure. No C++ exception crosses
 *    this ABI.
 *  - Connectivity is 6 (face neighbours; 4 in 2D) everywhere.
 */
#ifndef IBIP_H
#define IBIP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IBIP_OK = 0,
    IBIP_EINVAL = -1,     /* null pointer, bad dims, bad option or threshold list */
    IBIP_ENOMEM = -2,     /* device or pinned host allocation failed */
    IBIP_ENOSOLID = -3,   /* image holds no solid voxel: the distance transform is undefined */
    IBIP_EDEVICE = -4,    /* a HIP runtime call or kernel launch failed */
    IBIP_ECAPACITY = -5,  /* caller array too short, or an internal limit exceeded */
    IBIP_ECANCELLED = -6  /* a job was cancelled before it ran */
} ibip_status;

typedef struct { int32_t X, Y, Z; } ibip_dims;

/* Options of ibip_invade. Zero-initialise, then set what you need; a NULL
   options pointer means all defaults. */
typedef struct {
    int64_t max_steps;   /* stop after this many steps; 0 = run until no candidate is left */
    double sigma;        /* interfacial tension for the Washburn pressure (0 -> 1.0) */
    double theta_rad;    /* contact angle through the defending phase, radians (default 0) */
    double voxel_size;   /* length of one voxel (0 -> 1.0) */
} ibip_invade_opts;

typedef struct ibip_ctx ibip_ctx;

/* Create a context on HIP device `device`, ordered on `stream` (a hipStream_t;
   NULL = the null stream). */
ibip_status ibip_ctx_create(ibip_ctx** out, int32_t device, void* stream);
ibip_status ibip_ctx_destroy(ibip_ctx* ctx);
ibip_status ibip_ctx_set_stream(ibip_ctx* ctx, void* stream);
/* Text of the last error on this context ("" if none). Owned by the context. */
const char* ibip_last_error(const ibip_ctx* ctx);
/* Bytes of device scratch the context currently holds. */
int64_t ibip_ctx_scratch_bytes(const ibip_ctx* ctx);

/* Phase timing, for measurement. When enabled, the calls record HIP events
   on the context's stream around each phase and each launch of the step
   loop, and add the elapsed times (milliseconds) to the counters below. */
typedef struct {
    double edt_ms;          /* distance transform kernels (ibip_edt, and inside ibip_invade) */
    double setup_ms;        /* histogram, ranks, buckets, seeding */
    double loop_ms;         /* the whole step loop, host round trips included */
    double loop_kernel_ms;  /* sum of the single-workgroup loop kernel durations */
    double wide_kernel_ms;  /* sum of the whole-GPU step kernel durations */
    double paint_ms;        /* sphere insertion */
    double steps_ms;        /* finalisation and per-step arrays */
    double trap_ms;         /* ibip_trap */
    double mio_ms;          /* ibip_opening_drainage */
    int64_t loop_launches;  /* launches of the loop kernel */
    int64_t wide_launches;  /* launches of the whole-GPU step kernel */
    int64_t steps;          /* steps K summed over ibip_invade calls */
    int64_t popped;         /* centres summed over ibip_invade calls */
    int64_t relax_sweeps;   /* reconstruction sweeps (trapping and MIO) */
    int64_t wide_centres;   /* centres of the steps run by the whole-GPU kernel */
} ibip_timing;

/* Readings of passages the paper leaves ambiguous, for the following calls
   on this context (default 0: the strict sphere, literal inlets, 6-connected
   trapping).
   IBIP_READ_INTEGER_BALL  footnote 1 of Section 2.1: a sphere of integer
       radius floor(sqrt(M)), ball {|v - c|^2 <= floor(sqrt(M))^2} restricted to
       pore, instead of {|v - c|^2 < M} (ibip_invade painting).
   IBIP_READ_MASK_INLETS   solid inlet voxels contribute no neighbours to the
       seed set (ibip_invade and the seeds of ibip_opening_drainage).
   IBIP_READ_TRAP26        ibip_trap connects voxels sharing a face, an edge or
       a corner (26-connectivity) instead of a face only.
   Batches and the server always use the default readings. */
#define IBIP_READ_INTEGER_BALL 1u
#define IBIP_READ_MASK_INLETS 2u
#define IBIP_READ_TRAP26 4u
ibip_status ibip_ctx_set_readings(ibip_ctx* ctx, uint32_t flags);

/* Launch parameters, for the following calls on this context (chosen per
   size class by the package's autotuner; results never depend on them).
   edt_tile_y  z columns per LDS tile of the EDT's pass y: 32 or 64 (0: 32)
   edt_tile_x  z columns per LDS tile of the EDT's pass x: 16 or 32 (0: 32)
   batch_wide  a batch job's step with more centres than this leaves the job's
               workgroup: the step runs over the whole GPU and the job's loop
               resumes in its own launch (0: never for ibip_invade_batch, 8192
               for the server's jobs; negative: never).
   Errors: EINVAL (a tile width not listed). NULL restores the defaults. */
typedef struct {
    int32_t edt_tile_y;
    int32_t edt_tile_x;
    int64_t batch_wide;
} ibip_tuning;
ibip_status ibip_ctx_set_tuning(ibip_ctx* ctx, const ibip_tuning* t);
ibip_status ibip_ctx_get_tuning(const ibip_ctx* ctx, ibip_tuning* out);

ibip_status ibip_ctx_enable_timing(ibip_ctx* ctx, int32_t enable);
ibip_status ibip_ctx_get_timing(const ibip_ctx* ctx, ibip_timing* out);
ibip_status ibip_ctx_reset_timing(ibip_ctx* ctx);

/* Measurement aid for the step loop, whose steps each wait for at least one
   claim (an atomic that returns the claimed word) before the next step's
   maximum is known. One lane follows a chain of n_chain dependent atomics
   through a device buffer of span_bytes (each atomic's result is the next
   address, consecutive ones on different cache lines); *ns_per_claim (host)
   receives the average time of one. A small span stays in the L2 cache, a
   large one goes to memory. The buffer is context scratch.
   Errors: EINVAL (span_bytes < 4096 or >= 2^34, n_chain < 1), ENOMEM. */
ibip_status ibip_probe_claim_latency(ibip_ctx* ctx, int64_t span_bytes, int32_t n_chain, double* ns_per_claim);

/*
 * ibip_edt -- distance transform of the pore space (Section 2.1, Figure 2(b)).
 * dt2[v] = min over solid voxels s of |v - s|^2 (exact, integer), 0 on solid.
 * Only voxels inside the image count as solid; the border is not solid.
 * dt2 (caller-owned DEVICE buffer, one uint32 per voxel) also holds
 * intermediate values while the call's kernels run (pass y's exact values at
 * 65535 and above, read back by pass x), so it is meaningful only once they
 * have finished on the context's stream.
 * Errors: EINVAL, ENOSOLID (checked on device, reported after a sync).
 */
ibip_status ibip_edt(ibip_ctx* ctx, const uint8_t* image, ibip_dims dims, uint32_t* dt2);

/*
 * ibip_edt_noalloc -- ibip_edt for callers that cannot allocate memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same dt2 as ibip_edt, but the call allocates nothing: its
 * intermediate distances (6 bytes per voxel) live in one fixed scratch array
 * of the library, 96 MiB per device, held from the first context created on
 * that device until the process ends. It does not synchronise: the solid
 * check is returned on the device instead of as ENOSOLID.
 * image, dt2:  as for ibip_edt, caller-owned DEVICE buffers.
 * solid_flag:  DEVICE uint32 out, set to 1 when the image holds a solid
 *              voxel, 0 when it holds none (dt2 is then unspecified).
 * Every call on one device shares that device's scratch: two calls that
 * overlap on the device (on different streams or contexts) race and give
 * wrong results. Calls ordered on one stream are safe.
 * Errors: EINVAL, ECAPACITY (more than 2^24 voxels), EDEVICE (launch failure,
 * or the scratch has no address on this device).
 */
ibip_status ibip_edt_noalloc(ibip_ctx* ctx, const uint8_t* image, ibip_dims dims, uint32_t* dt2,
                             uint32_t* solid_flag);

/*
 * ibip_invade -- the invasion loop of Section 2.1 (Figure 2(e)-(l)).
 * Step k takes the candidates (inlets, plus the face neighbours of the inlets
 * and of every earlier centre, pore only, not yet a centre), finds the
 * largest distance-transform value M_k among them, makes every candidate
 * holding M_k a centre of step k, and inserts at each centre c the sphere
 * B(c, M_k) = {v : |v - c|^2 < M_k} (which lies in pore space), writing k only
 * where nothing was written before (first write wins). The loop stops when no
 * candidate is left or after max_steps steps.
 *
 * inlets: uint8 mask, nonzero = inlet voxel (anywhere in the image; inlet
 *         voxels on solid still contribute their neighbours).
 * seq:    int32 out. -1 solid, 0 uninvaded pore, k >= 1 = step of invasion.
 * rad2:   uint32 out or NULL. M_{seq[v]} for invaded voxels (the squared
 *         radius of the sphere that invaded v), 0 elsewhere.
 * centre_step: int32 out or NULL. The step at which v was a centre, 0 if never.
 * n_steps: host out, the number of steps K.
 * The per-step arrays of this call stay in the context until the next
 * ibip_invade on it; read them with ibip_get_steps.
 * An image with more than 8192 distinct distance values in its pore space
 * (a pore whose largest inscribed ball has a radius near 100 voxels or more)
 * runs a slower form of the step loop whose per-rank tables live in device
 * memory instead of LDS; the results are the same.
 * Errors: EINVAL, ENOSOLID, ENOMEM, EDEVICE, ECAPACITY (more than 2^24 - 1
 * distinct distance values).
 */
ibip_status ibip_invade(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims dims,
                        const ibip_invade_opts* opts, int32_t* seq, uint32_t* rad2,
                        int32_t* centre_step, int64_t* n_steps);

/*
 * ibip_invade_resume -- continue an invasion from a checkpoint taken at a
 * step boundary (Section 2.1; the sequence image holds the whole history of
 * the invasion, Section 2.2.1). A call of ibip_invade with max_steps = k_done
 * that returned K = k_done leaves, in its centre_step output, the step at
 * which every voxel was a centre; that map and k_done are the checkpoint.
 * The candidates of step k_done + 1 are rebuilt from it (every pore voxel that
 * is a seed of the inlets, a centre, or a face neighbour of a centre, minus
 * the centres), and the loop continues from there. The outputs cover the
 * whole invasion (steps 1..K) and equal those of one uninterrupted
 * ibip_invade on the same inputs and readings; ibip_get_steps then returns
 * all K steps.
 * centre_step_in: int32 DEVICE in, the checkpoint (values 0..k_done); it must
 *                 not be the same buffer as centre_step.
 * k_done:         steps taken before the checkpoint (>= 0; 0 = a fresh start).
 * opts:           as for ibip_invade; max_steps counts every step from step 1
 *                 and must be 0 or at least k_done.
 * Other arguments and outputs as for ibip_invade.
 * Errors: as ibip_invade, and EINVAL for a checkpoint with a value outside
 * 0..k_done or a centre on solid.
 */
ibip_status ibip_invade_resume(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets, ibip_dims dims,
                               const ibip_invade_opts* opts, const int32_t* centre_step_in, int64_t k_done,
                               int32_t* seq, uint32_t* rad2, int32_t* centre_step, int64_t* n_steps);

/*
 * ibip_invade_batch -- ibip_invade (Section 2.1) over many images of uneven
 * size in one call, with the same results as one ibip_invade per image.
 * Each job names its own device buffers, dims and step limit; per-job setup
 * runs concurrently, the step loops of all jobs run in ONE launch (one
 * workgroup per job, largest first) and the call synchronises once between
 * the loops and the post-processing.
 * Per job: status receives the job's ibip_status (OK, ENOSOLID, ECAPACITY,
 * EDEVICE) and n_steps its K. M (uint32) and sat (double) are optional DEVICE
 * outputs of the per-step squared radius and saturation, each with capacity
 * for at least as many entries as the image has pore voxels.
 * A job whose image has more than 8192 distinct distance values in its pore
 * space (more than a job's rank tables hold) runs after the batched launch,
 * alone, through the path of ibip_invade on the context's stream (same
 * results); that call replaces the context's per-step arrays, so
 * ibip_get_steps afterwards reports EINVAL until the next ibip_invade.
 * Returns IBIP_OK when every job succeeded, else the first failing job's code.
 */
typedef struct {
    const uint8_t* image;   /* device, image mask as in ibip_invade */
    const uint8_t* inlets;  /* device */
    ibip_dims dims;
    int64_t max_steps;      /* 0 = run until no candidate is left */
    int32_t* seq;           /* device out */
    uint32_t* rad2;         /* device out or NULL */
    int32_t* centre_step;   /* device out or NULL */
    uint32_t* M;            /* device out or NULL */
    double* sat;            /* device out or NULL */
    int64_t n_steps;        /* out */
    int32_t status;         /* out */
} ibip_job;

ibip_status ibip_invade_batch(ibip_ctx* ctx, ibip_job* jobs, int32_t n);

/*
 * Continuous-batching server for invasion jobs (the serving pattern of the
 * invasion loop of Section 2.1). Jobs are submitted at any time; a worker
 * thread admits a pending job as soon as an execution slot is free and the
 * job's scratch (about 26 bytes per voxel) fits in the server's HBM pool, and
 * runs it on its slot's stream: setup, the step loop in one workgroup, sphere
 * insertion and finalisation, without host synchronisation, so admitted jobs
 * overlap on the device. A job behind one that does not fit yet may start
 * first (within `lookahead` places), so a huge job does not block the queue.
 * A job's results are those of ibip_invade on the same inputs.
 * The job's input buffers must hold their data when it is submitted, and its
 * output buffers must stay valid until ibip_server_wait returns for it.
 * ibip_job.M, when given, receives the per-step squared radii; sat is not
 * produced by the server. Latency = submission to completion.
 */
typedef struct ibip_server ibip_server;

typedef struct {
    int64_t hbm_budget_bytes;  /* device pool for job scratch (0 -> 8 GiB) */
    int32_t max_inflight;      /* execution slots (0 -> 16) */
    int32_t lookahead;         /* pending jobs scanned for one that fits (0 -> 8) */
} ibip_server_opts;

typedef struct {
    int64_t submitted, completed, cancelled, pending, running;
    int64_t bytes_in_use, peak_bytes, peak_running;
} ibip_server_stats;

ibip_status ibip_server_create(ibip_server** out, int32_t device, const ibip_server_opts* opts);
/* Queue a job (copied); *ticket identifies it. ECAPACITY if its scratch
   exceeds the whole pool, EINVAL for a bad job. A job whose image has more
   than 8192 distinct distance values in its pore space completes with status
   ECAPACITY (a served job's rank tables hold 8192 ranks; ibip_invade takes
   such images). */
ibip_status ibip_server_submit(ibip_server* s, const ibip_job* job, int64_t* ticket);
/* *done = 1 once the job completed (or was cancelled). */
ibip_status ibip_server_poll(ibip_server* s, int64_t ticket, int32_t* done);
/* Block until the job completes; copy it (status, n_steps) into *result and
   its latency into *latency_ms (either may be NULL), then forget the ticket.
   Returns the job's status. */
ibip_status ibip_server_wait(ibip_server* s, int64_t ticket, ibip_job* result, double* latency_ms);
/* Cancel a job. A pending job is dropped at once; a running one stops at the
   next check of its step loop (every 1024 steps, and between its loop
   segments) and nothing more is queued for it. Its status becomes ECANCELLED
   (its outputs are unspecified) unless it had finished before the request
   took effect. EINVAL if the job is done or unknown. */
ibip_status ibip_server_cancel(ibip_server* s, int64_t ticket);
ibip_status ibip_server_stats_get(ibip_server* s, ibip_server_stats* out);
/* Launch parameters of the jobs admitted from now on (ibip_tuning:
   edt_tile_y, edt_tile_x, and batch_wide for the served jobs' wide steps).
   NULL restores the defaults. Errors: EINVAL. */
ibip_status ibip_server_set_tuning(ibip_server* s, const ibip_tuning* t);
const char* ibip_server_last_error(const ibip_server* s);
/* Cancel pending jobs, let running ones finish, free everything. */
ibip_status ibip_server_destroy(ibip_server* s);

/*
 * ibip_get_steps -- per-step arrays of the last ibip_invade (Sections 2.2.1,
 * 2.2.2). For k = 1..K, entry k-1 holds:
 *   M      uint32  squared radius inserted at step k
 *   n_new  int64   voxels first invaded at step k
 *   sat    double  saturation after step k = (voxels invaded at steps <= k) / (pore voxels)
 *   pc     double  Washburn capillary pressure 2 sigma cos(theta) / (sqrt(M_k) voxel_size)
 * Each pointer is a DEVICE buffer of at least `capacity` entries, or NULL to
 * skip it. Errors: EINVAL (no invade yet), ECAPACITY (capacity < K).
 */
ibip_status ibip_get_steps(ibip_ctx* ctx, uint32_t* M, int64_t* n_new, double* sat, double* pc,
                           int64_t capacity);

/*
 * ibip_saturation -- per-step arrays and the saturation map of any step
 * labelling (Sections 2.2.1, 2.2.2; Figure 5 left): the sequence written by
 * ibip_invade, or the re-ranked one of ibip_trap for the trapping-aware curve.
 * seq:     int32[N] in (-1 solid, 0 uninvaded, 1..K step).
 * M:       uint32[K] in, squared radius of each step's spheres (needed for pc;
 *          after trapping, from ibip_remap_steps).
 * opts:    sigma, theta_rad, voxel_size for pc (NULL: 1, 0, 1); max_steps unused.
 * n_new, sat, pc: as for ibip_get_steps, K entries each, saturation over all
 *          pore voxels (seq >= 0). satmap: double[N], -1 on solid, 0 on
 *          uninvaded pore, else the saturation after the voxel's step, so that
 *          {0 < satmap <= s} is the invaded configuration at saturation s.
 * Every array is a caller-owned DEVICE buffer; any output may be NULL.
 * Errors: EINVAL (a label above K, no pore voxel), ENOMEM.
 */
ibip_status ibip_saturation(ibip_ctx* ctx, const int32_t* seq, ibip_dims dims, const uint32_t* M, int64_t K,
                            const ibip_invade_opts* opts, int64_t* n_new, double* sat, double* pc,
                            double* satmap);

/*
 * ibip_remap_steps -- squared radii of the steps that survive trapping
 * (Section 2.2.3): re-ranked step k' keeps the spheres of the original step
 * it came from, M_after[k'-1] = M[seq[v]-1] for any voxel v with
 * seq_after[v] = k'. seq: the sequence before trapping (K steps); seq_after:
 * the re-ranked sequence of ibip_trap (K_after steps). All DEVICE buffers.
 * Errors: EINVAL (labels that do not come from one trapping of seq), ENOMEM.
 */
ibip_status ibip_remap_steps(ibip_ctx* ctx, const int32_t* seq, const int32_t* seq_after, ibip_dims dims,
                             const uint32_t* M, int64_t K, int64_t K_after, uint32_t* M_after);

/*
 * ibip_compare_opening -- equal-saturation comparison of IBIP with the
 * opening drainage (Section 3.1.1, Figures 8 and 9). At level i (one per
 * opening radius) the IBIP configuration is {0 < satmap <= sat_T[i]} and the
 * opening's is {mio_r2 >= T[i]}.
 * satmap:      double[N] DEVICE, from ibip_saturation (of ibip_invade's seq).
 * mio_r2:      uint32[N] DEVICE, from ibip_opening_drainage at the radii T.
 * trapped:     uint8[N] DEVICE or NULL, from ibip_trap.
 * T, sat_T:    HOST arrays of n_levels entries: the opening's squared radii
 *              (strictly decreasing, >= 1) and its saturations (non-decreasing).
 * disagree:    int64[n_levels] DEVICE out: voxels in exactly one configuration.
 * mio_trapped: int64[n_levels] DEVICE out (needed with trapped): voxels the
 *              opening holds that IBIP leaves trapped.
 * Errors: EINVAL, ENOMEM.
 */
ibip_status ibip_compare_opening(ibip_ctx* ctx, const double* satmap, const uint32_t* mio_r2,
                                 const uint8_t* trapped, ibip_dims dims, const uint32_t* T, const double* sat_T,
                                 int32_t n_levels, int64_t* disagree, int64_t* mio_trapped);

/*
 * ibip_trap -- defender trapping and re-ranking (Section 2.2.3, Figure 7).
 * A voxel invaded at step k (seq[v] = k > 0) is trapped when the defender
 * region just before step k, {pore u : seq[u] == 0 or seq[u] >= k}, holds no
 * path of face neighbours from v to a pore voxel with outlets[u] != 0.
 * seq:          int32 in, as written by ibip_invade (-1 solid, 0 uninvaded).
 * outlets:      uint8 mask in.
 * trapped:      uint8 out, 1 for trapped invaded voxels, else 0.
 * seq_trapped:  int32 out or NULL. -1 solid, 0 uninvaded or trapped, else the
 *               dense rank (1..K') of seq[v] among the surviving step values.
 * n_steps_after: host out or NULL, K'.
 * Errors: EINVAL, ENOMEM, EDEVICE.
 */
ibip_status ibip_trap(ibip_ctx* ctx, const int32_t* seq, const uint8_t* outlets, ibip_dims dims,
                      uint8_t* trapped, int32_t* seq_trapped, int64_t* n_steps_after);

/*
 * ibip_opening_drainage -- pressure-based drainage by morphological image
 * opening (Section 2.4.1), the comparison of Section 3.1.1.
 * For each squared radius T_i (HOST array, strictly decreasing, >= 1): erode
 * the pore space by B(., T_i) (the centres c with dt2[c] >= T_i), keep the
 * eroded components that touch the inlet candidates (inlets and their face
 * neighbours, pore only), and dilate the kept centres by B(., T_i).
 * mio_r2:  uint32 DEVICE out. The first (largest) T_i whose opening holds v, 0 if none.
 * mio_sat: double HOST out or NULL, n entries: |{v : mio_r2[v] >= T_i}| / (pore voxels).
 * Errors: EINVAL, ENOSOLID, ENOMEM, EDEVICE.
 */
ibip_status ibip_opening_drainage(ibip_ctx* ctx, const uint8_t* image, const uint8_t* inlets,
                                  ibip_dims dims, const uint32_t* r2_thresholds, int32_t n,
                                  uint32_t* mio_r2, double* mio_sat);

#ifdef __cplusplus
}
#endif

#endif /* IBIP_H */
