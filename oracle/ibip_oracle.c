/*
 * CPU oracle for image-based invasion percolation (IBIP) and morphological
 * image opening (MIO) drainage -- Gostick, Yang & Boek, "Simulating
 * volume-controlled invasion of a non-wetting fluid in volumetric images
 * using basic image processing tools" (arXiv 2101.03240).
 *
 * THIS IS TEST INFRASTRUCTURE. It exists only to check the HIP path. Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * it. It shares no code, header, table or constant with the HIP library.
 *
 * Plain single-threaded C99, integer arithmetic, written for clarity over
 * speed. Every function follows a definition or the steps of the paper:
 *
 *   ibipref_edt_brute     squared Euclidean distance to the nearest solid voxel,
 *                         by definition (minimum over all solid voxels).
 *   ibipref_edt           the same quantity, computed as the exact separable
 *                         decomposition of that minimum (three 1D minima, each
 *                         taken over the whole line; no envelope algorithm).
 *   ibipref_invade_literal  Section 2.1 step by step: dilate the inlets image
 *                         with a cross, take the maximum of dt under it, insert
 *                         spheres at every maximum (first write wins), add the
 *                         centres to the inlets image and zero dt there; the
 *                         whole image is rescanned every step.
 *   ibipref_invade        the same loop with the dilated inlets image kept as
 *                         an explicit candidate set grouped by dt value (with
 *                         seq NULL: the selection alone, centres and M, no
 *                         spheres inserted).
 *   ibipref_steps         Sections 2.2.1-2.2.2: per-step newly invaded counts,
 *                         saturation and Washburn capillary pressure.
 *   ibipref_satmap        Section 2.2.1, Figure 5 (left): each invaded voxel
 *                         labelled with the saturation after its step.
 *   ibipref_remap_steps   Section 2.2.3: the squared radius of every step that
 *                         survives trapping, in re-ranked order.
 *   ibipref_trap          Section 2.2.3: reverse sweep over the sequence with
 *                         union-find (Masson-style), then dense re-ranking.
 *   ibipref_trap_brute    trapping by definition: one breadth-first search per
 *                         invaded voxel.
 *   ibipref_mio           Section 2.4.1: for decreasing radii, erode, trim to
 *                         inlet-connected, dilate; first write wins.
 *
 * Conventions (readings of passages where the paper is silent or ambiguous):
 *   - grid (X, Y, Z) in C order, v = (x*Y + y)*Z + z; image != 0 is pore.
 *   - dt2 = squared distance to the nearest solid voxel centre inside the
 *     image; the image border is not solid; dt2 = 0 on solid.
 *   - a sphere of squared radius m centred at c is B(c, m) = {v : |v-c|^2 < m}
 *     clipped to the grid (this ball always lies in pore space).
 *   - candidates = (inlets U cross-dilation(inlets)) restricted to pore.
 *   - all maxima are inserted in the same step; the step counter starts at 1
 *     and advances every step; the loop ends when no candidate is left or the
 *     step limit is reached.
 *   - seq = -1 on solid, 0 on uninvaded pore, k >= 1 = step of invasion.
 *   - 6-connectivity (face neighbours) throughout.
 *
 * Variants (the other readings of ambiguous passages, selected by flags):
 *   IBIPREF_INTEGER_BALL  footnote 1's integer sphere: radius floor(sqrt(M)),
 *                         ball {|v-c|^2 <= floor(sqrt(M))^2} restricted to pore.
 *   IBIPREF_MASK_INLETS   solid inlet voxels contribute no neighbours to the
 *                         seeds: Q0 = ((I & P) U N6(I & P)) & P (also for MIO).
 *   connectivity 26       trapping connects voxels that share a face, an edge
 *                         or a corner.
 *
 * Status codes: 0 ok, -1 invalid argument, -3 no solid voxel (the distance
 * transform is undefined), -5 capacity (output array too short),
 * -2 out of memory.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define REF_OK 0
#define REF_EINVAL (-1)
#define REF_ENOMEM (-2)
#define REF_ENOSOLID (-3)
#define REF_ECAPACITY (-5)

static const uint64_t REF_INF = (uint64_t)1 << 62;

#define IBIPREF_INTEGER_BALL 1
#define IBIPREF_MASK_INLETS 2

static int dims_ok(int X, int Y, int Z) {
    return X > 0 && Y > 0 && Z > 0 && (int64_t)X * Y * Z < ((int64_t)1 << 32);
}

/* face neighbours of voxel (x, y, z); returns how many were written */
static int neighbours6(int X, int Y, int Z, int64_t v, int64_t out[6]) {
    int64_t z = v % Z, y = (v / Z) % Y, x = v / ((int64_t)Y * Z);
    int n = 0;
    if (x > 0) out[n++] = v - (int64_t)Y * Z;
    if (x < X - 1) out[n++] = v + (int64_t)Y * Z;
    if (y > 0) out[n++] = v - Z;
    if (y < Y - 1) out[n++] = v + Z;
    if (z > 0) out[n++] = v - 1;
    if (z < Z - 1) out[n++] = v + 1;
    return n;
}

/* the (up to) 26 voxels sharing a face, an edge or a corner with v */
static int neighbours26(int X, int Y, int Z, int64_t v, int64_t out[26]) {
    int64_t z = v % Z, y = (v / Z) % Y, x = v / ((int64_t)Y * Z);
    int n = 0;
    for (int dx = -1; dx <= 1; dx++)
        for (int dy = -1; dy <= 1; dy++)
            for (int dz = -1; dz <= 1; dz++) {
                if (!dx && !dy && !dz) continue;
                int64_t a = x + dx, b = y + dy, c = z + dz;
                if (a < 0 || a >= X || b < 0 || b >= Y || c < 0 || c >= Z) continue;
                out[n++] = (a * Y + b) * Z + c;
            }
    return n;
}

/* face neighbours (conn 6) or all 26 neighbours (conn 26) */
static int neighbours(int conn, int X, int Y, int Z, int64_t v, int64_t out[26]) {
    return conn == 26 ? neighbours26(X, Y, Z, v, out) : neighbours6(X, Y, Z, v, out);
}

/* largest integer q with q*q <= a */
static int64_t isqrt64(int64_t a) {
    if (a <= 0) return 0;
    int64_t q = (int64_t)sqrt((double)a);
    while (q * q > a) q--;
    while ((q + 1) * (q + 1) <= a) q++;
    return q;
}

/* ------------------------------------------------------------------------- */
/* Distance transform of the pore space (Section 2.1; Figure 2(b)).          */
/* ------------------------------------------------------------------------- */

/* By definition: dt2[v] = min over solid s of |v - s|^2. O(N * N_solid). */
int ibipref_edt_brute(const uint8_t* img, int X, int Y, int Z, uint32_t* dt2) {
    if (!img || !dt2 || !dims_ok(X, Y, Z)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    int64_t ns = 0;
    for (int64_t i = 0; i < N; i++) ns += (img[i] == 0);
    if (ns == 0) return REF_ENOSOLID;
    int32_t* sx = (int32_t*)malloc(sizeof(int32_t) * 3 * (size_t)ns);
    if (!sx) return REF_ENOMEM;
    int64_t k = 0;
    for (int x = 0; x < X; x++)
        for (int y = 0; y < Y; y++)
            for (int z = 0; z < Z; z++)
                if (img[((int64_t)x * Y + y) * Z + z] == 0) {
                    sx[3 * k] = x; sx[3 * k + 1] = y; sx[3 * k + 2] = z; k++;
                }
    for (int x = 0; x < X; x++)
        for (int y = 0; y < Y; y++)
            for (int z = 0; z < Z; z++) {
                int64_t best = INT64_MAX;
                for (int64_t s = 0; s < ns; s++) {
                    int64_t dx = x - sx[3 * s], dy = y - sx[3 * s + 1], dz = z - sx[3 * s + 2];
                    int64_t d = dx * dx + dy * dy + dz * dz;
                    if (d < best) best = d;
                }
                dt2[((int64_t)x * Y + y) * Z + z] = (uint32_t)best;
            }
    free(sx);
    return REF_OK;
}

/*
 * Separable form of the same minimum. Since |v-s|^2 = dx^2 + dy^2 + dz^2,
 *   min_s |v-s|^2 = min_x' [ (x-x')^2 + min_y' [ (y-y')^2 + min_{z': solid} (z-z')^2 ] ],
 * an exact identity. Each 1D minimum is taken over the whole line, O(N * L).
 */
int ibipref_edt(const uint8_t* img, int X, int Y, int Z, uint32_t* dt2) {
    if (!img || !dt2 || !dims_ok(X, Y, Z)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    int64_t ns = 0;
    for (int64_t i = 0; i < N; i++) ns += (img[i] == 0);
    if (ns == 0) return REF_ENOSOLID;
    uint64_t* a = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    uint64_t* b = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    if (!a || !b) { free(a); free(b); return REF_ENOMEM; }
    /* Lines are independent: built with OpenMP (the CPU data-parallel
       baseline), each pass splits its lines over the threads; the plain build
       ignores the pragmas. */
    /* along z: nearest solid in the same row */
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < (int64_t)X * Y; r++) {
        const uint8_t* row = img + r * Z;
        for (int z = 0; z < Z; z++) {
            uint64_t best = REF_INF;
            for (int zp = 0; zp < Z; zp++)
                if (row[zp] == 0) {
                    uint64_t d = (uint64_t)((int64_t)(z - zp) * (z - zp));
                    if (d < best) best = d;
                }
            a[r * Z + z] = best;
        }
    }
    /* along y */
    int fail = 0;
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int64_t xz = 0; xz < (int64_t)X * Z; xz++) {
        const int x = (int)(xz / Z), z = (int)(xz % Z);
        uint64_t* line = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)Y);
        if (!line) { fail = 1; continue; }
        for (int y = 0; y < Y; y++) line[y] = a[((int64_t)x * Y + y) * Z + z];
        for (int y = 0; y < Y; y++) {
            uint64_t best = REF_INF;
            for (int yp = 0; yp < Y; yp++) {
                if (line[yp] >= REF_INF) continue;
                uint64_t d = line[yp] + (uint64_t)((int64_t)(y - yp) * (y - yp));
                if (d < best) best = d;
            }
            b[((int64_t)x * Y + y) * Z + z] = best;
        }
        free(line);
    }
    /* along x */
#pragma omp parallel for schedule(static) reduction(| : fail)
    for (int64_t yz = 0; yz < (int64_t)Y * Z; yz++) {
        const int y = (int)(yz / Z), z = (int)(yz % Z);
        uint64_t* line = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)X);
        if (!line) { fail = 1; continue; }
        for (int x = 0; x < X; x++) line[x] = b[((int64_t)x * Y + y) * Z + z];
        for (int x = 0; x < X; x++) {
            uint64_t best = REF_INF;
            for (int xp = 0; xp < X; xp++) {
                if (line[xp] >= REF_INF) continue;
                uint64_t d = line[xp] + (uint64_t)((int64_t)(x - xp) * (x - xp));
                if (d < best) best = d;
            }
            dt2[((int64_t)x * Y + y) * Z + z] = (uint32_t)best;
        }
        free(line);
    }
    free(a); free(b);
    return fail ? REF_ENOMEM : REF_OK;
}

/*
 * Exact squared distance at a single voxel by searching cubic shells of
 * growing half-width h around it; stops once h*h >= best, since every voxel
 * outside the searched cube is at squared distance > h*h. Returns -1 if the
 * image holds no solid voxel.
 */
/* threads the OpenMP build uses (1 for the plain build) */
int ibipref_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

int64_t ibipref_edt_at(const uint8_t* img, int X, int Y, int Z, int x, int y, int z) {
    int64_t best = INT64_MAX;
    int Lmax = X > Y ? X : Y; if (Z > Lmax) Lmax = Z;
    for (int h = 0; h <= Lmax; h++) {
        if (best != INT64_MAX && (int64_t)h * h >= best) break;
        for (int dx = -h; dx <= h; dx++) {
            int xx = x + dx; if (xx < 0 || xx >= X) continue;
            for (int dy = -h; dy <= h; dy++) {
                int yy = y + dy; if (yy < 0 || yy >= Y) continue;
                int onface = (dx == -h || dx == h || dy == -h || dy == h);
                for (int dz = -h; dz <= h; dz += (onface ? 1 : (2 * h > 0 ? 2 * h : 1))) {
                    int zz = z + dz; if (zz < 0 || zz >= Z) continue;
                    if (img[((int64_t)xx * Y + yy) * Z + zz] == 0) {
                        int64_t d = (int64_t)dx * dx + (int64_t)dy * dy + (int64_t)dz * dz;
                        if (d < best) best = d;
                    }
                }
            }
        }
    }
    return best == INT64_MAX ? -1 : best;
}

/* ------------------------------------------------------------------------- */
/* Sphere insertion (Section 2.1, footnote 1; Figure 2(h), (l)).             */
/* ------------------------------------------------------------------------- */

/* write `step` (and `m` into rad2) into every uninvaded voxel of B(c, m);
   with the integer rule, into every uninvaded pore voxel with |v - c|^2 <=
   floor(sqrt(m))^2 instead (solid voxels hold -1 and are never written) */
static void insert_sphere(int X, int Y, int Z, int64_t c, uint32_t m, int32_t step,
                          int32_t* seq, uint32_t* rad2, int integer_ball) {
    int cz = (int)(c % Z), cy = (int)((c / Z) % Y), cx = (int)(c / ((int64_t)Y * Z));
    int64_t R = integer_ball ? isqrt64((int64_t)m) : isqrt64((int64_t)m - 1);
    int64_t lim = integer_ball ? R * R + 1 : (int64_t)m; /* ball = {d^2 < lim} */
    /* under OpenMP the x-planes of a large sphere go to different threads
       (they write disjoint voxels); the plain build ignores the pragma */
#pragma omp parallel for schedule(static) if (R >= 8)
    for (int64_t dx = -R; dx <= R; dx++) {
        int64_t x = cx + dx; if (x < 0 || x >= X) continue;
        for (int64_t dy = -R; dy <= R; dy++) {
            int64_t y = cy + dy; if (y < 0 || y >= Y) continue;
            for (int64_t dz = -R; dz <= R; dz++) {
                int64_t z = cz + dz; if (z < 0 || z >= Z) continue;
                if (dx * dx + dy * dy + dz * dz >= lim) continue;
                int64_t v = (x * Y + y) * Z + z;
                if (seq[v] == 0) { seq[v] = step; if (rad2) rad2[v] = m; }
            }
        }
    }
}

static void init_seq(const uint8_t* img, int64_t N, int32_t* seq, uint32_t* rad2, int32_t* cs) {
    for (int64_t i = 0; i < N; i++) {
        if (seq) seq[i] = img[i] ? 0 : -1;
        if (rad2) rad2[i] = 0;
        if (cs) cs[i] = 0;
    }
}

/* ------------------------------------------------------------------------- */
/* The invasion loop, literally (Section 2.1; Figure 2(e)-(l)).              */
/* Returns the number of steps K (>= 0) or a negative status.                */
/* M_out[k-1] receives the squared radius inserted at step k.                */
/* ------------------------------------------------------------------------- */
int64_t ibipref_invade_literal_v(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z,
                                 int64_t max_steps, int flags, int32_t* seq, uint32_t* rad2,
                                 int32_t* centre_step, uint32_t* M_out, int64_t M_cap) {
    if (!img || !inlets || !seq || !dims_ok(X, Y, Z)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    uint32_t* dt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
    uint8_t* inl = (uint8_t*)malloc((size_t)N);
    uint8_t* cand = (uint8_t*)malloc((size_t)N);
    int64_t* C = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!dt || !inl || !cand || !C) { free(dt); free(inl); free(cand); free(C); return REF_ENOMEM; }
    int st = ibipref_edt(img, X, Y, Z, dt);
    if (st != REF_OK) { free(dt); free(inl); free(cand); free(C); return st; }
    for (int64_t i = 0; i < N; i++) inl[i] = inlets[i] != 0 && (!(flags & IBIPREF_MASK_INLETS) || img[i]);
    init_seq(img, N, seq, rad2, centre_step);
    int64_t step = 0;
    for (;;) {
        if (max_steps > 0 && step >= max_steps) break;
        /* (e) dilate the inlets image with a cross */
        for (int64_t v = 0; v < N; v++) {
            cand[v] = inl[v];
            if (!cand[v]) {
                int64_t nb[6]; int n = neighbours6(X, Y, Z, v, nb);
                for (int j = 0; j < n; j++) if (inl[nb[j]]) { cand[v] = 1; break; }
            }
        }
        /* (f), (g) value and locations of the maximum of dt under the dilated inlets */
        uint32_t M = 0;
        for (int64_t v = 0; v < N; v++) if (cand[v] && dt[v] > M) M = dt[v];
        if (M == 0) break; /* no pore candidate left */
        int64_t nc = 0;
        for (int64_t v = 0; v < N; v++) if (cand[v] && dt[v] == M) C[nc++] = v;
        step++;
        if (M_out) {
            if (step > M_cap) { free(dt); free(inl); free(cand); free(C); return REF_ECAPACITY; }
            M_out[step - 1] = M;
        }
        /* (h) insert spheres at every maximum, only into uninvaded voxels */
        for (int64_t i = 0; i < nc; i++)
            insert_sphere(X, Y, Z, C[i], M, (int32_t)step, seq, rad2, flags & IBIPREF_INTEGER_BALL);
        /* (i) add the centres to the inlets image and zero dt there */
        for (int64_t i = 0; i < nc; i++) {
            inl[C[i]] = 1; dt[C[i]] = 0;
            if (centre_step) centre_step[C[i]] = (int32_t)step;
        }
    }
    free(dt); free(inl); free(cand); free(C);
    return step;
}

int64_t ibipref_invade_literal(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z,
                               int64_t max_steps, int32_t* seq, uint32_t* rad2,
                               int32_t* centre_step, uint32_t* M_out, int64_t M_cap) {
    return ibipref_invade_literal_v(img, inlets, X, Y, Z, max_steps, 0, seq, rad2, centre_step, M_out, M_cap);
}

/* ------------------------------------------------------------------------- */
/* The same loop with the dilated inlets image kept as a candidate set.      */
/* Candidates are grouped by dt value (one list per value), so the maximum    */
/* of dt under the dilated inlets is the highest non-empty group. Each step   */
/* takes every member of that group present at the start of the step; the     */
/* neighbours of the new centres join the candidate set for the next step.    */
/* ------------------------------------------------------------------------- */
typedef struct { int64_t* v; int64_t n, cap; } vlist;

static int vlist_push(vlist* l, int64_t v) {
    if (l->n == l->cap) {
        int64_t nc = l->cap ? 2 * l->cap : 16;
        int64_t* p = (int64_t*)realloc(l->v, sizeof(int64_t) * (size_t)nc);
        if (!p) return 0;
        l->v = p; l->cap = nc;
    }
    l->v[l->n++] = v;
    return 1;
}

int64_t ibipref_invade_v(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z,
                         int64_t max_steps, int flags, int32_t* seq, uint32_t* rad2,
                         int32_t* centre_step, uint32_t* M_out, int64_t M_cap) {
    /* seq may be NULL: the selection alone (painting never feeds back into it) */
    if (!img || !inlets || !dims_ok(X, Y, Z)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    uint32_t* dt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
    uint8_t* seen = (uint8_t*)calloc((size_t)N, 1);
    if (!dt || !seen) { free(dt); free(seen); return REF_ENOMEM; }
    int st = ibipref_edt(img, X, Y, Z, dt);
    if (st != REF_OK) { free(dt); free(seen); return st; }
    uint32_t maxdt = 0;
    for (int64_t v = 0; v < N; v++) if (dt[v] > maxdt) maxdt = dt[v];
    vlist* group = (vlist*)calloc((size_t)maxdt + 1, sizeof(vlist));
    if (!group) { free(dt); free(seen); return REF_ENOMEM; }
    init_seq(img, N, seq, rad2, centre_step);
    int64_t rc = 0;
    /* initial candidates: inlets and their face neighbours, pore only */
    for (int64_t v = 0; v < N; v++) {
        if (!inlets[v] || ((flags & IBIPREF_MASK_INLETS) && !img[v])) continue;
        int64_t nb[7]; int n = neighbours6(X, Y, Z, v, nb); nb[n++] = v;
        for (int j = 0; j < n; j++) {
            int64_t u = nb[j];
            if (img[u] && !seen[u]) {
                seen[u] = 1;
                if (!vlist_push(&group[dt[u]], u)) { rc = REF_ENOMEM; goto done; }
            }
        }
    }
    int64_t top = maxdt;
    int64_t step = 0;
    vlist cur = {0, 0, 0};
    for (;;) {
        if (max_steps > 0 && step >= max_steps) break;
        while (top > 0 && group[top].n == 0) top--;
        if (top == 0) break;
        uint32_t M = (uint32_t)top;
        /* the centres of this step: the whole group as it stands now */
        vlist tmp = cur; cur = group[M]; group[M] = tmp; group[M].n = 0;
        step++;
        if (M_out) {
            if (step > M_cap) { rc = REF_ECAPACITY; free(cur.v); goto done; }
            M_out[step - 1] = M;
        }
        for (int64_t i = 0; i < cur.n; i++) {
            int64_t c = cur.v[i];
            if (centre_step) centre_step[c] = (int32_t)step;
            if (seq) insert_sphere(X, Y, Z, c, M, (int32_t)step, seq, rad2, flags & IBIPREF_INTEGER_BALL);
        }
        for (int64_t i = 0; i < cur.n; i++) {
            int64_t nb[6]; int n = neighbours6(X, Y, Z, cur.v[i], nb);
            for (int j = 0; j < n; j++) {
                int64_t u = nb[j];
                if (img[u] && !seen[u]) {
                    seen[u] = 1;
                    if (!vlist_push(&group[dt[u]], u)) { rc = REF_ENOMEM; free(cur.v); goto done; }
                    if ((int64_t)dt[u] > top) top = dt[u];
                }
            }
        }
        cur.n = 0;
    }
    free(cur.v);
    rc = step;
done:
    for (uint32_t g = 0; g <= maxdt; g++) free(group[g].v);
    free(group); free(dt); free(seen);
    return rc;
}

int64_t ibipref_invade(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z,
                       int64_t max_steps, int32_t* seq, uint32_t* rad2,
                       int32_t* centre_step, uint32_t* M_out, int64_t M_cap) {
    return ibipref_invade_v(img, inlets, X, Y, Z, max_steps, 0, seq, rad2, centre_step, M_out, M_cap);
}

/* ------------------------------------------------------------------------- */
/* Steps -> saturation and capillary pressure (Sections 2.2.1, 2.2.2).       */
/* n_new[k-1] = voxels with seq == k; sat[k-1] = (voxels with 1 <= seq <= k) */
/* / (all pore voxels); pc[k-1] = c0 / sqrt(M[k-1]) with c0 = 2 sigma        */
/* cos(theta) / voxel_size supplied by the caller (Washburn relation).       */
/* ------------------------------------------------------------------------- */
int ibipref_steps(const int32_t* seq, int64_t N, int64_t K, const uint32_t* M, double c0,
                  int64_t* n_new, double* sat, double* pc) {
    if (!seq || N <= 0 || K < 0) return REF_EINVAL;
    int64_t n_pore = 0;
    int64_t* cnt = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
    if (!cnt) return REF_ENOMEM;
    for (int64_t v = 0; v < N; v++) {
        if (seq[v] >= 0) n_pore++;
        if (seq[v] > 0) {
            if (seq[v] > K) { free(cnt); return REF_EINVAL; }
            cnt[seq[v]]++;
        }
    }
    int64_t cum = 0;
    for (int64_t k = 1; k <= K; k++) {
        cum += cnt[k];
        if (n_new) n_new[k - 1] = cnt[k];
        if (sat) sat[k - 1] = n_pore ? (double)cum / (double)n_pore : 0.0;
        if (pc && M) pc[k - 1] = c0 / sqrt((double)M[k - 1]);
    }
    free(cnt);
    return REF_OK;
}

/* Saturation map (Section 2.2.1, Figure 5 left): satmap[v] = sat[seq[v]-1]
 * for an invaded voxel, 0 for uninvaded pore, -1 on solid, where sat is the
 * per-step saturation of ibipref_steps for the same labelling. Thresholding
 * the map as 0 < satmap <= s gives the invaded configuration at saturation s. */
int ibipref_satmap(const int32_t* seq, int64_t N, int64_t K, const double* sat, double* satmap) {
    if (!seq || !satmap || N <= 0 || K < 0) return REF_EINVAL;
    for (int64_t v = 0; v < N; v++) {
        const int32_t s = seq[v];
        if (s < 0) satmap[v] = -1.0;
        else if (s == 0) satmap[v] = 0.0;
        else if (s > K) return REF_EINVAL;
        else satmap[v] = sat[s - 1];
    }
    return REF_OK;
}

/* Squared radii after trapping (Section 2.2.3): a re-ranked step k' holds the
 * voxels of one surviving original step s, and keeps that step's spheres, so
 * M_after[k'-1] = M[s-1]. seq is the sequence before trapping, seq_after the
 * re-ranked one (0 where trapped). */
int ibipref_remap_steps(const int32_t* seq, const int32_t* seq_after, int64_t N, const uint32_t* M, int64_t K,
                        int64_t K_after, uint32_t* M_after) {
    if (!seq || !seq_after || !M || !M_after || N <= 0 || K < 0 || K_after < 0) return REF_EINVAL;
    for (int64_t j = 0; j < K_after; j++) M_after[j] = 0;
    for (int64_t v = 0; v < N; v++) {
        const int32_t a = seq_after[v];
        if (a <= 0) continue;
        const int32_t s = seq[v];
        if (a > K_after || s <= 0 || s > K) return REF_EINVAL;
        if (M_after[a - 1] != 0 && M_after[a - 1] != M[s - 1]) return REF_EINVAL;  /* one step per rank */
        M_after[a - 1] = M[s - 1];
    }
    return REF_OK;
}

/* ------------------------------------------------------------------------- */
/* Trapping of the defending phase (Section 2.2.3; Figure 7).                */
/* A voxel invaded at step k is trapped when, just before step k, the        */
/* defender region D_k = {pore u : seq[u] == 0 or seq[u] >= k} has no path   */
/* from it to an outlet voxel. Trapped voxels are reset to uninvaded and the */
/* surviving step values are re-ranked to 1..K'.                            */
/* ------------------------------------------------------------------------- */
static int64_t uf_find(int64_t* parent, int64_t a) {
    while (parent[a] != a) { parent[a] = parent[parent[a]]; a = parent[a]; }
    return a;
}

static void uf_union(int64_t* parent, uint8_t* flag, int64_t a, int64_t b) {
    a = uf_find(parent, a); b = uf_find(parent, b);
    if (a == b) return;
    if (a < b) { int64_t t = a; a = b; b = t; }
    parent[a] = b;
    flag[b] |= flag[a];
}

static int rerank(const int32_t* seq, const uint8_t* trapped, int64_t N, int64_t K,
                  int32_t* seq_trapped, int64_t* K_after) {
    uint8_t* present = (uint8_t*)calloc((size_t)K + 2, 1);
    int32_t* rank = (int32_t*)calloc((size_t)K + 2, sizeof(int32_t));
    if (!present || !rank) { free(present); free(rank); return REF_ENOMEM; }
    for (int64_t v = 0; v < N; v++) if (seq[v] > 0 && !trapped[v]) present[seq[v]] = 1;
    int32_t r = 0;
    for (int64_t k = 1; k <= K; k++) if (present[k]) rank[k] = ++r;
    if (seq_trapped)
        for (int64_t v = 0; v < N; v++) {
            if (seq[v] < 0) seq_trapped[v] = -1;
            else if (seq[v] == 0 || trapped[v]) seq_trapped[v] = 0;
            else seq_trapped[v] = rank[seq[v]];
        }
    if (K_after) *K_after = r;
    free(present); free(rank);
    return REF_OK;
}

int ibipref_trap_c(const int32_t* seq, const uint8_t* outlets, int X, int Y, int Z, int conn,
                   uint8_t* trapped, int32_t* seq_trapped, int64_t* K_after) {
    if (!seq || !outlets || !trapped || !dims_ok(X, Y, Z) || (conn != 6 && conn != 26)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    int64_t K = 0;
    for (int64_t v = 0; v < N; v++) if (seq[v] > K) K = seq[v];
    int64_t* parent = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    uint8_t* flag = (uint8_t*)calloc((size_t)N, 1);
    int64_t* start = (int64_t*)calloc((size_t)K + 2, sizeof(int64_t));
    int64_t* order = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!parent || !flag || !start || !order) {
        free(parent); free(flag); free(start); free(order); return REF_ENOMEM;
    }
    /* group the invaded voxels by step (counting sort) */
    for (int64_t v = 0; v < N; v++) if (seq[v] > 0) start[seq[v] + 1]++;
    for (int64_t k = 1; k <= K; k++) start[k + 1] += start[k];
    {
        int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(K + 2));
        if (!fill) { free(parent); free(flag); free(start); free(order); return REF_ENOMEM; }
        memcpy(fill, start, sizeof(int64_t) * (size_t)(K + 2));
        for (int64_t v = 0; v < N; v++) if (seq[v] > 0) order[fill[seq[v]]++] = v;
        free(fill);
    }
    for (int64_t v = 0; v < N; v++) {
        parent[v] = v;
        flag[v] = (seq[v] >= 0 && outlets[v]) ? 1 : 0;
        trapped[v] = 0;
    }
    /* the never-invaded pore is defender at every step */
    for (int64_t v = 0; v < N; v++) {
        if (seq[v] != 0) continue;
        int64_t nb[26]; int n = neighbours(conn, X, Y, Z, v, nb);
        for (int j = 0; j < n; j++) if (seq[nb[j]] == 0) uf_union(parent, flag, v, nb[j]);
    }
    /* thresholds in decreasing order: at level k the defender region gains
       the voxels invaded at step k */
    for (int64_t k = K; k >= 1; k--) {
        for (int64_t i = start[k]; i < start[k + 1]; i++) {
            int64_t v = order[i];
            int64_t nb[26]; int n = neighbours(conn, X, Y, Z, v, nb);
            for (int j = 0; j < n; j++) {
                int32_t s = seq[nb[j]];
                if (s == 0 || s >= k) uf_union(parent, flag, v, nb[j]);
            }
        }
        for (int64_t i = start[k]; i < start[k + 1]; i++) {
            int64_t v = order[i];
            trapped[v] = flag[uf_find(parent, v)] ? 0 : 1;
        }
    }
    int st = rerank(seq, trapped, N, K, seq_trapped, K_after);
    free(parent); free(flag); free(start); free(order);
    return st;
}

int ibipref_trap(const int32_t* seq, const uint8_t* outlets, int X, int Y, int Z,
                 uint8_t* trapped, int32_t* seq_trapped, int64_t* K_after) {
    return ibipref_trap_c(seq, outlets, X, Y, Z, 6, trapped, seq_trapped, K_after);
}

/* Trapping by definition: for every invaded voxel v, a breadth-first search
   inside D_{seq[v]} from v; trapped if it reaches no outlet voxel. */
int ibipref_trap_brute_c(const int32_t* seq, const uint8_t* outlets, int X, int Y, int Z, int conn,
                         uint8_t* trapped) {
    if (!seq || !outlets || !trapped || !dims_ok(X, Y, Z) || (conn != 6 && conn != 26)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    uint8_t* vis = (uint8_t*)malloc((size_t)N);
    if (!queue || !vis) { free(queue); free(vis); return REF_ENOMEM; }
    for (int64_t v = 0; v < N; v++) {
        trapped[v] = 0;
        if (seq[v] <= 0) continue;
        int32_t k = seq[v];
        memset(vis, 0, (size_t)N);
        int64_t qh = 0, qt = 0;
        queue[qt++] = v; vis[v] = 1;
        int reached = 0;
        while (qh < qt && !reached) {
            int64_t u = queue[qh++];
            if (outlets[u]) { reached = 1; break; }
            int64_t nb[26]; int n = neighbours(conn, X, Y, Z, u, nb);
            for (int j = 0; j < n; j++) {
                int64_t w = nb[j];
                if (vis[w]) continue;
                if (seq[w] == 0 || seq[w] >= k) { vis[w] = 1; queue[qt++] = w; }
            }
        }
        trapped[v] = reached ? 0 : 1;
    }
    free(queue); free(vis);
    return REF_OK;
}

int ibipref_trap_brute(const int32_t* seq, const uint8_t* outlets, int X, int Y, int Z, uint8_t* trapped) {
    return ibipref_trap_brute_c(seq, outlets, X, Y, Z, 6, trapped);
}

/* Dense re-ranking for a given trapped mask (exposed for tests). */
int ibipref_rerank(const int32_t* seq, const uint8_t* trapped, int64_t N,
                   int32_t* seq_trapped, int64_t* K_after) {
    if (!seq || !trapped || N <= 0) return REF_EINVAL;
    int64_t K = 0;
    for (int64_t v = 0; v < N; v++) if (seq[v] > K) K = seq[v];
    return rerank(seq, trapped, N, K, seq_trapped, K_after);
}

/* ------------------------------------------------------------------------- */
/* Morphological image opening drainage (Section 2.4.1).                     */
/* For each squared radius T (given in decreasing order): erode the pore     */
/* space by B(., T) -- the centres c whose ball B(c, T) holds no solid, i.e. */
/* dt2[c] >= T --; keep only the eroded components that touch the inlet      */
/* candidates (inlets and their face neighbours, pore only); dilate the kept */
/* centres by B(., T). mio_r2[v] = the first (largest) T whose opening holds */
/* v, 0 if none, and mio_sat[i] = |{v : mio_r2[v] >= T_i}| / N_pore.         */
/* `brute_erosion` != 0 checks each ball voxel by voxel instead of reading   */
/* the distance transform (tiny images only).                                */
/* ------------------------------------------------------------------------- */
/* inlet seed test of the opening (the same Q0 as the invasion) */
static int mio_seed(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z, int64_t v, int flags) {
    const int mask = flags & IBIPREF_MASK_INLETS;
    if (inlets[v] && (!mask || img[v])) return 1;
    int64_t nb[6]; int nn = neighbours6(X, Y, Z, v, nb);
    for (int j = 0; j < nn; j++) if (inlets[nb[j]] && (!mask || img[nb[j]])) return 1;
    return 0;
}

int ibipref_mio_v(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z,
                  const uint32_t* T, int32_t n, int brute_erosion, int flags,
                  uint32_t* mio_r2, double* mio_sat) {
    if (!img || !inlets || !T || n < 0 || !mio_r2 || !dims_ok(X, Y, Z)) return REF_EINVAL;
    for (int32_t i = 0; i < n; i++) if (T[i] == 0 || (i > 0 && T[i] >= T[i - 1])) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    uint32_t* dt = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)N);
    uint8_t* er = (uint8_t*)malloc((size_t)N);
    uint8_t* kept = (uint8_t*)malloc((size_t)N);
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!dt || !er || !kept || !queue) { free(dt); free(er); free(kept); free(queue); return REF_ENOMEM; }
    int st = ibipref_edt(img, X, Y, Z, dt);
    if (st != REF_OK) { free(dt); free(er); free(kept); free(queue); return st; }
    int64_t n_pore = 0;
    for (int64_t v = 0; v < N; v++) { mio_r2[v] = 0; n_pore += img[v] != 0; }
    for (int32_t i = 0; i < n; i++) {
        uint32_t t = T[i];
        int64_t R = isqrt64((int64_t)t - 1);
        /* erosion */
        for (int64_t v = 0; v < N; v++) {
            if (!img[v]) { er[v] = 0; continue; }
            if (!brute_erosion) { er[v] = dt[v] >= t; continue; }
            int cz = (int)(v % Z), cy = (int)((v / Z) % Y), cx = (int)(v / ((int64_t)Y * Z));
            int ok = 1;
            for (int64_t dx = -R; dx <= R && ok; dx++) {
                int64_t x = cx + dx; if (x < 0 || x >= X) continue;
                for (int64_t dy = -R; dy <= R && ok; dy++) {
                    int64_t y = cy + dy; if (y < 0 || y >= Y) continue;
                    for (int64_t dz = -R; dz <= R; dz++) {
                        int64_t z = cz + dz; if (z < 0 || z >= Z) continue;
                        if (dx * dx + dy * dy + dz * dz >= (int64_t)t) continue;
                        if (!img[(x * Y + y) * Z + z]) { ok = 0; break; }
                    }
                }
            }
            er[v] = (uint8_t)ok;
        }
        /* trim: breadth-first search from the eroded voxels among the inlet candidates */
        int64_t qh = 0, qt = 0;
        memset(kept, 0, (size_t)N);
        for (int64_t v = 0; v < N; v++) {
            if (!er[v] || kept[v]) continue;
            if (mio_seed(img, inlets, X, Y, Z, v, flags)) { kept[v] = 1; queue[qt++] = v; }
        }
        while (qh < qt) {
            int64_t u = queue[qh++];
            int64_t nb[6]; int nn = neighbours6(X, Y, Z, u, nb);
            for (int j = 0; j < nn; j++) {
                int64_t w = nb[j];
                if (er[w] && !kept[w]) { kept[w] = 1; queue[qt++] = w; }
            }
        }
        /* dilation of the kept centres; first write wins */
        for (int64_t q = 0; q < qt; q++) {
            int64_t c = queue[q];
            int cz = (int)(c % Z), cy = (int)((c / Z) % Y), cx = (int)(c / ((int64_t)Y * Z));
            for (int64_t dx = -R; dx <= R; dx++) {
                int64_t x = cx + dx; if (x < 0 || x >= X) continue;
                for (int64_t dy = -R; dy <= R; dy++) {
                    int64_t y = cy + dy; if (y < 0 || y >= Y) continue;
                    for (int64_t dz = -R; dz <= R; dz++) {
                        int64_t z = cz + dz; if (z < 0 || z >= Z) continue;
                        if (dx * dx + dy * dy + dz * dz >= (int64_t)t) continue;
                        int64_t v = (x * Y + y) * Z + z;
                        if (mio_r2[v] == 0) mio_r2[v] = t;
                    }
                }
            }
        }
        if (mio_sat) {
            int64_t cnt = 0;
            for (int64_t v = 0; v < N; v++) cnt += mio_r2[v] >= t;
            mio_sat[i] = n_pore ? (double)cnt / (double)n_pore : 0.0;
        }
    }
    free(dt); free(er); free(kept); free(queue);
    return REF_OK;
}

int ibipref_mio(const uint8_t* img, const uint8_t* inlets, int X, int Y, int Z,
                const uint32_t* T, int32_t n, int brute_erosion,
                uint32_t* mio_r2, double* mio_sat) {
    return ibipref_mio_v(img, inlets, X, Y, Z, T, n, brute_erosion, 0, mio_r2, mio_sat);
}

/* The MIO kept set at one squared radius T: eroded pore voxels 6-connected
   (inside the eroded set) to the inlet candidates. Exposed for the exact
   IBIP / MIO invariant tests. Returns the number of kept voxels. */
int64_t ibipref_mio_kept_v(const uint8_t* img, const uint8_t* inlets, const uint32_t* dt2,
                           int X, int Y, int Z, uint32_t T, int flags, uint8_t* kept) {
    if (!img || !inlets || !dt2 || !kept || !dims_ok(X, Y, Z)) return REF_EINVAL;
    int64_t N = (int64_t)X * Y * Z;
    int64_t* queue = (int64_t*)malloc(sizeof(int64_t) * (size_t)N);
    if (!queue) return REF_ENOMEM;
    memset(kept, 0, (size_t)N);
    int64_t qh = 0, qt = 0;
    for (int64_t v = 0; v < N; v++) {
        if (!img[v] || dt2[v] < T) continue;
        if (mio_seed(img, inlets, X, Y, Z, v, flags)) { kept[v] = 1; queue[qt++] = v; }
    }
    while (qh < qt) {
        int64_t u = queue[qh++];
        int64_t nb[6]; int nn = neighbours6(X, Y, Z, u, nb);
        for (int j = 0; j < nn; j++) {
            int64_t w = nb[j];
            if (img[w] && dt2[w] >= T && !kept[w]) { kept[w] = 1; queue[qt++] = w; }
        }
    }
    free(queue);
    return qt;
}

int64_t ibipref_mio_kept(const uint8_t* img, const uint8_t* inlets, const uint32_t* dt2,
                         int X, int Y, int Z, uint32_t T, uint8_t* kept) {
    return ibipref_mio_kept_v(img, inlets, dt2, X, Y, Z, T, 0, kept);
}
