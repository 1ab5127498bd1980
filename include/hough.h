/*
 * hough.h -- C ABI of the MI355X (gfx950) Hough-transform track finder.
 *
 * The library computes the data-parallel part of the Hough track finder
 * (Section 3): every track hypothesis of a binned parameter space starts with
 * zero votes, every detector hit adds one vote to each hypothesis it is
 * compatible with, and the local maxima above a threshold become track
 * candidates.  Section 3 notes that prompt curved tracks need two parameters
 * (phi0, kappa) and displaced curved tracks three (d0, phi0, kappa); both are
 * served here.  Section 4 points out that no hit's votes depend on any other
 * hit: that independence is the parallelism the kernels use.
 *
 * Track model (transverse plane, cm).  Hypothesis (d0, phi0, kappa) is the
 * circle whose point of closest approach to the origin is
 * P0 = (-d0 sin phi0, d0 cos phi0), tangent there to (cos phi0, sin phi0),
 * with signed curvature kappa (> 0: counter-clockwise).  A hit (x, y) votes,
 * for each d0 bin l and phi0 bin j, the kappa of the circle through it:
 *     r2 = x*x + y*y;   u = y*cos_phi[j] - x*sin_phi[j];   d = d0[l]
 *     kappa = 2*(u - d) / ((r2 - (2*d)*u) + d*d)
 *     kf = (kappa - kappa_min) * kappa_scale
 *     if (kf >= 0 && kf < n_kappa) acc[l][j][(int)kf] += 1
 * Every operation is one IEEE binary32 operation rounded to nearest even, in
 * exactly this order (no FMA contraction, correctly rounded division,
 * denormals kept).  NaN/Inf kf casts no vote.  A 2D grid is the d0 = +0 case.
 * Results (accumulators, vote counts, candidate lists) are therefore exact
 * integers and do not depend on launch shape, tiling or batching.
 *
 * Peak rule.  Cell p = (l, j, k) with v = acc[p] >= threshold is a candidate
 * when for every neighbour w at offset o in {-1,0,1}^3 \ {0} (order d0, phi0,
 * kappa; phi0 periodic; d0 and kappa neighbours outside the grid ignored)
 * v > w if o is lexicographically negative and v >= w otherwise.  Candidates
 * are sorted by votes descending then cell ascending, with
 * cell = (l*n_phi + j)*n_kappa + k.
 *
 * Conventions for every call:
 *   - [dev] marks device memory (e.g. a torch tensor's data_ptr()); all other
 *     pointers are host memory read during the call only.
 *   - The caller owns every buffer; the context owns only its workspace,
 *     allocated in hough_ctx_create.  No other call allocates device memory.
 *   - Work is enqueued on `stream` (a hipStream_t, NULL = default stream) and
 *     is asynchronous; results are valid once the stream reaches that point.
 *   - Argument errors are reported synchronously as HOUGH_EINVAL and enqueue
 *     nothing.  HIP runtime failures return HOUGH_EDEVICE and
 *     hough_last_error() describes them.  Calls never throw.
 *   - Device-side conditions are not errors: a candidate list longer than its
 *     capacity reports its full length in n_found and writes the first `cap`
 *     entries of the sorted list.
 *   - A context may be used by one host thread at a time.  Calls on one
 *     context must not overlap on different streams (they share workspace).
 */
#ifndef HOUGH_H
#define HOUGH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HOUGH_OK = 0,
    HOUGH_EINVAL = -1,   /* invalid argument; nothing was enqueued */
    HOUGH_ENOMEM = -2,   /* workspace allocation failed (context creation only) */
    HOUGH_EDEVICE = -3,  /* a HIP runtime call failed; see hough_last_error() */
    HOUGH_EBUSY = -4     /* the server's pending queue is full; the event was not taken */
} hough_status;

typedef enum {
    HOUGH_ACC_I32 = 0,   /* int32 cells */
    HOUGH_ACC_U16 = 1    /* uint16 cells; requires n_hits <= 65535 per event and even n_kappa */
} hough_acc_type;

typedef enum {
    HOUGH_CURVED = 0,    /* circles (d0, phi0, kappa): the vote formula above */
    HOUGH_STRAIGHT = 1   /* straight lines (phi0, d0), the kappa = 0 family: n_d0 == 1, d0 == NULL, and
                            the last axis holds d0 -- kappa_min is the d0 lower edge (cm) and
                            kappa_scale the bins per cm.  A hit votes, for every phi0 bin,
                                u = y*c - x*s;  fd = (u - kappa_min) * kappa_scale;
                                if (fd >= 0 && fd < n_kappa) acc[j][(int)fd] += 1
                            (binary32, in this order): the d0 of the line through the hit. */
} hough_family;

/* The binned parameter space.  Bin tables are shared inputs computed once by
 * the caller (fp32), so no transcendental is evaluated on the device. */
typedef struct {
    int32_t n_d0;            /* d0 bins; 1 with d0 == NULL for the 2D grid */
    int32_t n_phi;           /* phi0 bins (periodic); >= 3 */
    int32_t n_kappa;         /* kappa bins; >= 1 */
    float kappa_min;         /* lower edge of the kappa range (cm^-1) */
    float kappa_scale;       /* bins per unit kappa (cm) */
    const float *cos_phi;    /* [dev][n_phi] cos of the phi0 bin centres */
    const float *sin_phi;    /* [dev][n_phi] sin of the phi0 bin centres */
    const float *d0;         /* [dev][n_d0] d0 bin centres (cm), or NULL for 2D */
    int32_t acc_type;        /* hough_acc_type */
    int32_t family;          /* hough_family (0: curved tracks) */
    int32_t forward;         /* 0: every phi0 bin.  1, the forward-hemisphere option (an addition to the
                                paper's method): a hit votes for phi0 bin j only when it lies ahead of P0,
                                    x*cos_phi[j] + y*sin_phi[j] > 0   (binary32, in this order),
                                which drops each hit's mirror solution (the direction of travel pointing
                                back at the origin) and about half of the votes; both families */
} hough_grid;

typedef struct {
    int32_t votes;           /* votes of the cell */
    int32_t cell;            /* (l*n_phi + j)*n_kappa + k */
} hough_cand;

/* Context sizing.  Zero fields take the defaults noted. */
typedef struct {
    int32_t max_events;      /* largest n_events of hough_event_batch (default 1) */
    int64_t max_hits;        /* largest total hit count of one call (default 1<<20, at most 1<<30) */
    const char *tune_cache;  /* JSON file of tuned launch shapes, or NULL */
} hough_ctx_opts;

typedef struct hough_ctx hough_ctx;

/* Create a context for one grid on the current HIP device.  The bin tables
 * must stay valid for the context's lifetime.  Allocates all workspace.
 * EINVAL: null pointers, n_phi < 3, n_kappa < 1, n_d0 < 1, n_d0 > 1 without a
 * d0 table, u16 with odd n_kappa, more than 2^31 - 1 cells, max_hits < 0 or
 * above 2^30. */
hough_status hough_ctx_create(hough_ctx **ctx, const hough_grid *grid, const hough_ctx_opts *opts);
void hough_ctx_destroy(hough_ctx *ctx);

/* Vote one event (Section 3: zero the parameter space, then every hit adds its
 * votes).  x, y: [dev][n_hits] fp32, cm.  acc: [dev] n_d0*n_phi*n_kappa cells
 * of the grid's type, 4-byte aligned, overwritten.  n_votes: [dev] one
 * uint64, overwritten with the number of votes cast (sum of acc), or NULL.
 * EINVAL: null x/y/acc with n_hits > 0, n_hits < 0, n_hits > max_hits, u16
 * with n_hits > 65535. */
hough_status hough_vote(hough_ctx *ctx, const float *x, const float *y, int32_t n_hits,
                        void *acc, uint64_t *n_votes, void *stream);

/* Find the local maxima of an accumulator (Section 3: once all hits have
 * voted, the local maxima of the votes are the candidates).  acc: [dev] as
 * produced by hough_vote
 * (any values are accepted).  out: [dev][cap] sorted candidates (may be NULL
 * when cap == 0).  n_found: [dev] one int32, the full number of candidates.
 * EINVAL: null acc/n_found, cap < 0, threshold < 1 for u16 is allowed. */
hough_status hough_peaks(hough_ctx *ctx, const void *acc, int32_t threshold,
                         hough_cand *out, int32_t cap, int32_t *n_found, void *stream);

/* ------------------------------------------------------------------------
 * Displaced vertices: the second Hough transform (Section 5).
 *
 * A vertex V is the sinusoid d0 = V_y cos(phi0) - V_x sin(phi0) of the
 * (phi0, d0) plane.  Every first-transform candidate with votes >=
 * track_threshold is read as the straight line of vertices V with
 * V_y c - V_x s = d0 (c, s, d0 the bin centres of its cell in the context's
 * grid) and votes into a binned (x, y) vertex grid, one binary32 operation at
 * a time with no contraction:
 *   |c| >= |s|: for every column ix
 *       y = (d0 + x_centre[ix] * s) / c;  fy = (y - y_min) * y_scale;
 *       if (fy >= 0 && fy < n_y) vacc[ix][(int)fy] += 1
 *   otherwise:  for every row iy
 *       x = (y_centre[iy] * c - d0) / s;  fx = (x - x_min) * x_scale;
 *       if (fx >= 0 && fx < n_x) vacc[(int)fx][iy] += 1
 * Vertex candidates are cells with vacc >= vertex_threshold that pass the
 * asymmetric 3x3 local-maximum rule (earlier offsets in (dx, dy) order must
 * be exceeded, later ones reached; neither axis is periodic), sorted by votes
 * descending then cell = ix * n_y + iy ascending.
 * ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_x, n_y;            /* bins per axis: n_x*n_y <= 16384, ceil(n_x/2)*ceil(n_y/2) <= 4096,
                                    and n_x*(n_y+1) cells of LDS with the sort keys within 160 KB */
    float x_min, x_scale;        /* fx = (x - x_min) * x_scale */
    float y_min, y_scale;        /* fy = (y - y_min) * y_scale */
    const float *x_centre;       /* [dev][n_x] fp32 column centres */
    const float *y_centre;       /* [dev][n_y] fp32 row centres */
} hough_vertex_grid;

/* Second transform for n_events events whose first-transform candidates are
 * in cands (e.g. the output of hough_event_batch on this context):
 *   cands:      [dev] hough_cand lists; event e's list is cands[cand_off[e] ..
 *               cand_off[e] + min(n_found[e], cand_off[e+1] - cand_off[e])).
 *   cand_off:   [dev][n_events+1] int64 list offsets (nondecreasing).
 *   n_found:    [dev][n_events] int32 candidates found per event.
 *   sorted_lists: nonzero when every list is sorted by votes descending (as
 *               hough_event_batch and hough_peaks write them): the voting
 *               candidates are then a prefix and the scan stops at the first
 *               one below track_threshold.  Zero scans whole lists.
 *   vout:       [dev] vertex candidates; event e gets the first
 *               vout_off[e+1] - vout_off[e] of its sorted list at vout_off[e].
 *   vout_off:   [dev][n_events+1] int64 (nondecreasing).
 *   n_vertices: [dev][n_events] int32, the full number of vertex candidates.
 *   vacc:       [dev][n_events][n_x*n_y] int32 accumulators (overwritten), or NULL.
 * Candidate cells outside the context's grid are skipped.  Allocates
 * nothing; asynchronous on stream.  EINVAL: null required pointers,
 * n_events < 1, a vertex grid beyond the limits above. */
hough_status hough_vertices(hough_ctx *ctx, const hough_vertex_grid *vgrid, int32_t n_events,
                            const hough_cand *cands, const int64_t *cand_off, const int32_t *n_found,
                            int32_t sorted_lists, int32_t track_threshold, int32_t vertex_threshold,
                            hough_cand *vout, const int64_t *vout_off, int32_t *n_vertices, int32_t *vacc,
                            void *stream);

/* Hit association (Section 3: a track candidate is made by the hits
 * compatible with it) for one event.  Hit h belongs to candidate c when c has
 * votes >= min_votes and h votes -- the vote of hough_vote, with the grid's
 * family and forward option -- into a cell of c's window, the cells within
 * one bin of c's on every axis (phi0 modulo n_phi; d0 and kappa inside the
 * grid): the window of the peak rule.
 *   x, y:      [dev][n_hits] fp32 hits of the event.
 *   cands:     [dev][cands_cap] the event's candidates (e.g. hough_peaks' list);
 *              the first min(*n_cands, cands_cap) are used, and their cells must
 *              be distinct (a repeated cell keeps one of its indices).
 *   n_cands:   [dev] int32 candidate count (e.g. hough_peaks' n_found).
 *   pairs:     [dev][cap][2] int32 (candidate index, hit index), each pair once,
 *              in no particular order; the first min(*n_pairs, cap) are written.
 *   n_pairs:   [dev] uint64 (8-byte aligned), the full number of pairs.
 * Uses the context's cell map (cells int32) and hit records: calls on one
 * context must not overlap.  Allocates nothing; asynchronous on stream.
 * EINVAL: null required pointers, negative sizes, n_hits above the context's
 * max_hits, a misaligned n_pairs. */
hough_status hough_associate(hough_ctx *ctx, const float *x, const float *y, int32_t n_hits,
                             const hough_cand *cands, const int32_t *n_cands, int32_t cands_cap, int32_t min_votes,
                             int32_t *pairs, int64_t cap, uint64_t *n_pairs, void *stream);

/* Vote and find peaks for a batch of independent events in one pass
 * (Section 4: hits, and so events, are independent).  Equivalent, bit for bit,
 * to hough_vote followed by hough_peaks on each event.
 *   hit_off:  host [n_events+1] CSR offsets into x, y (hit_off[0] == 0).
 *   x, y:     [dev][hit_off[n_events]] fp32 hits of all events, packed.
 *   acc:      [dev][n_events * cells] accumulators, or NULL to skip storing them.
 *   cands:    [dev] candidate storage; event e owns [cand_off[e], cand_off[e+1]).
 *   cand_off: host [n_events+1] nondecreasing capacity offsets.
 *   n_found:  [dev][n_events] int32 full candidate counts.
 *   n_votes:  [dev][n_events] uint64 vote counts, or NULL.
 * The launch sequence is captured once as a HIP graph per stream and
 * replayed; the per-batch descriptors travel inside the graph.
 * EINVAL: n_events < 1 or > max_events, bad offsets, total hits > max_hits,
 * u16 with an event of more than 65535 hits, null required pointers. */
hough_status hough_event_batch(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off,
                               const float *x, const float *y, int32_t threshold,
                               void *acc, hough_cand *cands, const int64_t *cand_off,
                               int32_t *n_found, uint64_t *n_votes, void *stream);

/* hough_event_batch with the stored lists packed back to back, so that one
 * copy moves a whole batch's candidates (Section 4's per-event independence
 * leaves the lists' order to the caller).  Event e's list -- the first
 * min(n_found[e], cand_off[e+1] - cand_off[e]) candidates of its sorted list,
 * exactly what hough_event_batch stores at cands[cand_off[e]] -- is written at
 * cands[cand_start[e]], with cand_start[e] the sum of the earlier events'
 * stored counts; cand_start[n_events] is the total.  Every list lies inside
 * [0, cand_off[n_events]), so cands needs no more room than for
 * hough_event_batch.
 *   cand_start: [dev][n_events+1] int64 (8-byte aligned), overwritten.
 * Everything else, including EINVAL, as for hough_event_batch (also for a
 * null or misaligned cand_start). */
hough_status hough_event_batch_packed(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off,
                                      const float *x, const float *y, int32_t threshold,
                                      void *acc, hough_cand *cands, const int64_t *cand_off,
                                      int64_t *cand_start, int32_t *n_found, uint64_t *n_votes,
                                      void *stream);

/* Vote a batch of independent events (the vote half of hough_event_batch,
 * without the peak search and without a captured graph): acc receives every
 * event's accumulator back to back, exactly as hough_vote would write it.
 *   hit_off: host [n_events+1] CSR offsets; x, y: [dev] packed hits;
 *   acc: [dev][n_events * cells]; n_votes: [dev][n_events] uint64 or NULL.
 * EINVAL as for hough_event_batch. */
hough_status hough_vote_batch(hough_ctx *ctx, int32_t n_events, const int64_t *hit_off,
                              const float *x, const float *y, void *acc, uint64_t *n_votes,
                              void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one event's
 * vote, peak search and sort without a context -- bit for bit hough_vote then
 * hough_peaks on a context of this grid.
 *   grid:     as for hough_ctx_create (its tables are read by this call's
 *             kernels only); x, y: [dev][n_hits] fp32 hits.
 *   acc:      [dev] n_d0*n_phi*n_kappa cells of the grid's type, 4-byte
 *             aligned, overwritten (the peak search reads it back).
 *   out:      [dev][cap] sorted candidates (NULL when cap == 0); n_found: [dev]
 *             int32 full count; n_votes: [dev] uint64 (8-byte aligned) or NULL.
 * Scratch (hit records, tile words or ranges, per-event state, sort buffers)
 * is one fixed device array of HOUGH_NOALLOC_SCRATCH_BYTES inside the library,
 * held on every device it runs on until the process ends; the call allocates
 * and frees nothing.  It needs about 16 + 8*n_d0 bytes per hit plus 16 bytes
 * per candidate the grid can hold (cells/4 for 2D, cells/8 for 3D): the
 * workload grids fit with their events (a 1024x512 event of 64k hits uses
 * about 4 MiB, a 64x512x256 event of 35k hits about 50 MiB).  Every call on a
 * device shares that device's array and leaves its contents behind (each call
 * rewrites what it reads); calls that overlap in time on one device -- on two
 * streams or from two threads -- race on it and give wrong results.  The first
 * call on each device looks the array's address up there (a symbol query, no
 * allocation).  Asynchronous on stream.
 * EINVAL (nothing enqueued; hough_last_error says which): the grid rules of
 * hough_ctx_create, null pointers, negative sizes, misaligned acc or n_votes,
 * uint16 with more than 65535 hits, or an event and grid whose scratch exceeds
 * HOUGH_NOALLOC_SCRATCH_BYTES.  EDEVICE on a HIP failure. */
#define HOUGH_NOALLOC_SCRATCH_BYTES (64u << 20)
hough_status hough_event_noalloc(const hough_grid *grid, const float *x, const float *y, int32_t n_hits,
                                 int32_t threshold, void *acc, hough_cand *out, int32_t cap,
                                 int32_t *n_found, uint64_t *n_votes, void *stream);

/* Launch-shape controls (used by the autotuner and tests; results never
 * depend on them).  which: 0 = single-event vote, 1 = batched vote.
 * rows: phi0 rows per workgroup tile; threads: workgroup size (256/512/1024);
 * split: hit chunks per tile for the single-event vote (>= 1; 1 for the
 * batch).  Invalid combinations (a shape whose tile does not fit in LDS, a
 * batch work list longer than the context holds) return EINVAL. */
hough_status hough_set_launch(hough_ctx *ctx, int32_t which, int32_t rows, int32_t threads,
                              int32_t split);
hough_status hough_get_launch(const hough_ctx *ctx, int32_t which, int32_t *rows, int32_t *threads,
                              int32_t *split);

/* Autotuner (launch shapes only; results never depend on them).  Times every
 * supported shape of `which` on the caller's resident hits and keeps the
 * fastest on the context:
 *   which 1: whole hough_event_batch calls (tile rows x workgroup size), with
 *            the arguments of hough_event_batch (acc may be NULL);
 *   which 0: hough_vote of event 0 (hits [hit_off[0], hit_off[1])) into acc
 *            (required), over tile rows x workgroup size x hit split.
 * Each shape runs reps + 1 times (the first warms up); the median decides.
 * The candidates, counts and accumulators written are those of the last run,
 * exactly as the plain calls write them.  With a cache path (else
 * $HOUGH_TUNE_CACHE, else none) the winner is appended there as one JSON line
 * keyed by device, grid dimensions, accumulator type, which and
 * ceil(log2(hits)); hough_ctx_create applies the entry nearest to its
 * max_hits.  best_ms (nullable) receives the winner's median time.
 * Synchronous.  EINVAL as for the timed call, reps outside [1, 1000], or an
 * unwritable cache file. */
hough_status hough_autotune(hough_ctx *ctx, int32_t which, int32_t n_events, const int64_t *hit_off,
                            const float *x, const float *y, int32_t threshold, void *acc,
                            hough_cand *cands, const int64_t *cand_off, int32_t *n_found, int32_t reps,
                            const char *cache_path, void *stream, float *best_ms);

/* Host-only cache query (no device needed): the shape recorded for device tag
 * `device` (e.g. "gfx950/256"), the grid's dimensions and accumulator type,
 * `which` and the hit bucket nearest to ceil(log2(hits)).  *found = 0 when the
 * file or an entry is missing.  Only the grid's sizes and acc_type are read. */
hough_status hough_tune_lookup(const char *cache_path, const char *device, const hough_grid *grid,
                               int32_t which, int64_t hits, int32_t *found, int32_t *rows,
                               int32_t *threads, int32_t *split);

/* Timing mode (for benchmarks and profiling; results are unchanged).  When
 * enabled (enable 1 or 2), hough_event_batch enqueues its kernels directly on
 * the stream instead of replaying a graph and records HIP events around the
 * whole batch and around its vote kernel; with 2 the vote kernel also counts
 * the (hit, row) pairs it evaluates (one global atomic per wavefront and tile,
 * which lengthens the vote: time with 1, count with 2).  hough_get_timing
 * waits for the last timed batch and returns the two durations in
 * milliseconds (EINVAL before any timed batch).  EINVAL for enable outside
 * 0..2. */
hough_status hough_set_timing(hough_ctx *ctx, int32_t enable);
hough_status hough_get_timing(hough_ctx *ctx, float *vote_ms, float *total_ms);
/* Work of the last timed batch (measurement only): the (hit, phi0 row) pairs
 * its vote kernel evaluated -- each hit staged into a tile times the rows of
 * that tile, halo rows included.  The culling arcs leave out the rows where a
 * hit cannot vote, so this is less than hits * n_d0 * n_phi.  Waits for the
 * batch.  EINVAL unless the last batch ran in timing mode 2. */
hough_status hough_get_work(hough_ctx *ctx, uint64_t *evaluated_pairs);

/* ------------------------------------------------------------------------
 * Served stream (a trigger-farm node; Sections 1-2: events arrive
 * continuously; Section 4: they are independent).  A server owns, per grid
 * and per lane, a context, a stream and device-resident hit and candidate
 * pools, and batches continuously: a free lane takes the events waiting for
 * its grid as one hough_event_batch call while other lanes' batches run.
 * Results are the ones hough_vote + hough_peaks give each event alone.
 * ------------------------------------------------------------------------ */
typedef struct hough_server hough_server;

typedef struct {
    int32_t n_grids;                 /* 1..8 */
    const hough_grid *grids;         /* [n_grids]; tables must outlive the server */
    const int32_t *thresholds;       /* [n_grids] peak thresholds */
    int32_t lanes;                   /* batches in flight per grid (default 2, at most 8) */
    const int32_t *batch_events;     /* [n_grids] event slots per batch, or NULL (64) */
    const int64_t *batch_hits;       /* [n_grids] hit pool per lane, or NULL (1<<22) */
    const int64_t *event_candidates; /* [n_grids] candidates kept per event, or NULL (the grid's bound) */
    double deadline_ms;              /* longest wait to fill a batch while others run (default 2) */
    int32_t queue_limit;             /* pending events before submit refuses (default 4096) */
    int32_t keep_candidates;         /* 0: results carry counts only */
    const char *tune_cache;          /* passed to every lane's context */
    double batch_timeout_ms;         /* longest wait for a batch to complete (default 10000): past it
                                        the batch's events are returned with HOUGH_EDEVICE and the
                                        lane takes new work behind it on its stream */
} hough_server_opts;

typedef struct {
    int64_t tag;                     /* the caller's tag from submit */
    int32_t grid;
    int32_t status;                  /* HOUGH_OK, or HOUGH_EDEVICE if its batch failed */
    int32_t n_hits;
    int32_t n_found;                 /* full candidate count */
    int32_t n_stored;                /* candidates copied to the poll buffer */
    int32_t batch_events;            /* events in the batch it ran in */
    uint64_t n_votes;
    int64_t cand_offset;             /* first candidate in the poll buffer */
    double t_submit, t_launch, t_done;   /* seconds on the server clock */
} hough_served;

/* Create a server on the current device (allocates every pool; starts a
 * dispatcher thread and one completion thread per lane).  EINVAL for bad
 * options, ENOMEM when the pools do not fit. */
hough_status hough_server_create(hough_server **server, const hough_server_opts *opts);
/* Launch what is still pending, wait for every batch and free the server. */
void hough_server_destroy(hough_server *server);
/* Seconds since the server was created (the clock of every time stamp). */
double hough_server_clock(const hough_server *server);
/* Hand one event to the server: x, y are host fp32 arrays, copied before the
 * call returns.  t_submit: its arrival time on the server clock, or < 0 for
 * now (latency is measured from it).  EINVAL: bad grid or pointers, or an
 * event that can never be admitted (more hits than a lane's pool, or more
 * than 65535 for a uint16 grid); EBUSY: the pending queue is full. */
hough_status hough_server_submit(hough_server *server, int64_t tag, int32_t grid, const float *x,
                                 const float *y, int32_t n_hits, double t_submit);
/* Open-loop replay from a pool of events: arrival i is pool event pick[i]
 * (hits [pool_hit_off[k], pool_hit_off[k+1]) of pool_x, pool_y, grid
 * pool_grid[k]), submitted with tag i at arrival_s[i] seconds after the call
 * starts and stamped with that scheduled time.  Writes each submit's status
 * to status[i] and returns when all are submitted; poll concurrently.
 * EINVAL: null arrays, arrivals out of order, pick outside the pool. */
hough_status hough_server_replay(hough_server *server, int32_t n, const double *arrival_s,
                                 const int32_t *pick, int32_t n_pool, const int32_t *pool_grid,
                                 const int64_t *pool_hit_off, const float *pool_x, const float *pool_y,
                                 int32_t *status);
/* Take up to max_out finished events (waiting up to wait_ms for the first),
 * copying their candidates back to back into cand_buf[cand_cap].  EDEVICE
 * if a batch failed on the device (the failed events carry that status). */
hough_status hough_server_poll(hough_server *server, hough_served *out, int32_t max_out,
                               hough_cand *cand_buf, int64_t cand_cap, int32_t *n_out, int32_t wait_ms);
/* Pending events, events refused so far and lanes with a batch in flight. */
hough_status hough_server_stats(hough_server *server, int64_t *pending, int64_t *refused,
                                int32_t *busy_lanes);

/* Diagnostic: on the current device, compare the vote's division fast path
 * (the correctly rounded fp32 quotient with its reciprocal refinement done
 * once per hit) with the division operator, bit for bit, over n pseudo-random
 * operand pairs of the range where the fast path is used.  Writes the number
 * of mismatches (must be 0) and of pairs checked.  Allocates and frees a
 * 16-byte device buffer; synchronous. */
hough_status hough_selftest_divide(int64_t n, uint64_t seed, uint64_t *mismatches, uint64_t *checked);

/* Diagnostic: on the current device, the largest absolute error (radians) of
 * the fp32 angle functions that bound the culling arcs (the hit angle atan2f
 * over hits with r in [2^-30, 2^30], and asinf over [-1, 1] with extra
 * arguments near +-1) against fp64, over n pseudo-random arguments.  The arcs
 * are widened by 1e-4 rad, which assumes both errors stay below 1e-6.
 * Allocates and frees an 8-byte device buffer; synchronous. */
hough_status hough_selftest_angles(int64_t n, uint64_t seed, float *max_err_atan2, float *max_err_asin);

/* Diagnostic: on the current device, check the vote's approximate bins (one
 * FMA per evaluation, exact redo inside a band above each integer) for a
 * grid's kappa_min, kappa_scale and n_kappa.  form 0: the 3D quotient
 * 2 (u - d) / den by one reciprocal; form 1: the 2D quotient u / (r2/2) from
 * the hit's scaled reciprocal (straight-line records included).  Over n
 * pseudo-random operand pairs of the fast-path range, with quotients placed
 * across the kappa band (half of them within a few bound-widths of a bin
 * edge), every approximate bin outside the band must be the exact kf's bin or
 * miss.  Writes the mismatches (must be 0), the flagged pairs (which the vote
 * redoes exactly) and the pairs checked.  EINVAL for another form or when the
 * grid does not take approximate bins.  Allocates and frees a 24-byte device
 * buffer; synchronous. */
hough_status hough_selftest_near(int64_t n, uint64_t seed, float kappa_min, float kappa_scale, int32_t n_kappa,
                                 int32_t form, uint64_t *mismatches, uint64_t *redone, uint64_t *checked);

/* Diagnostics (measurement only; no part of the method).  Saturating probes
 * on the current device: the rate of conflict-free, no-return 32-bit LDS
 * atomic adds (the vote's one memory operation) and of plain fp32 VALU
 * operations (unpacked and unfused, as in the vote), both per second over the
 * whole device.  Allocates and frees 64 bytes of device memory; synchronous.
 * EINVAL for null outputs, EDEVICE on a HIP failure. */
hough_status hough_diag_rates(double *lds_atomics_per_s, double *valu_ops_per_s);

const char *hough_status_str(hough_status status);
/* Text of the last HIP failure seen by this thread (empty if none). */
const char *hough_last_error(void);
/* Library version string. */
const char *hough_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HOUGH_H */
