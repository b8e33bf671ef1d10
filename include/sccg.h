/* sccg — exact pixel areas of intersection and union of rectilinear polygon
 * pairs on AMD MI355X (gfx950), by PixelBox sampling-box subdivision.
 *
 * Method (Section 3 of "Accelerating Pathology Image Data Cross-Comparison
 * on CPU-GPU Hybrid Systems", Wang et al.):
 *   - polygons have integer vertices and axis-aligned edges (Section 3.1,
 *     Figure 3), so a pixel is either wholly inside or wholly outside;
 *   - |p ∩ q| counts the pixels inside both; |p ∪ q| = |p| + |q| − |p ∩ q|
 *     with |p| from the shoelace formula (Section 3.2);
 *   - the pair box is recursively split into sampling boxes; a box is
 *     inside / outside / hovering each polygon (Lemma 1); boxes decided for
 *     both polygons contribute at once, hovering boxes are split again until
 *     they fall under the pixelization threshold, where every pixel is
 *     tested by an even-odd ray-crossing count (Sections 3.1–3.3,
 *     Algorithm 1);
 *   - two polygon sets are compared by the Jaccard ratio of summed
 *     intersections over summed unions (Section 2.1), and by the mean of the
 *     per-pair ratios over pairs that intersect (Equation 1).
 *
 * Conventions for every entry point:
 *   - All array pointers are DEVICE pointers owned by the caller; the library
 *     borrows them until the work queued on the context's stream completes.
 *   - Calls are asynchronous on the context's stream.  Argument errors are
 *     returned at once and nothing is queued.  Errors found on the device
 *     (see SCCG_E_RANGE) are latched in a device error word and returned by
 *     sccg_sync().
 *   - Return 0 (SCCG_OK) or a negative error code; sccg_last_error() gives a
 *     message.  A context is used by one host thread at a time.
 *
 * Polygon storage (CSR): polygon k is the ring
 *   xy[2*offsets[k]], xy[2*offsets[k]+1], ..., up to 2*offsets[k+1]-1
 * as interleaved int32 (x, y) vertices.  The ring is implicitly closed,
 * either orientation; a repeated closing vertex or collinear vertices are
 * allowed (zero-length or split edges do not change any count).  Polygons
 * must be simple, hole-free, with axis-aligned edges (sccg_validate_polys
 * checks the last two); |x|, |y| <= 2^30.  Pixel (x, y) is the unit square
 * [x, x+1) x [y, y+1).
 */
#ifndef SCCG_H
#define SCCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ errors ---- */
#define SCCG_OK 0
#define SCCG_E_ARG -1    /* null pointer with a non-zero count, negative count, bad mode/flag/param */
#define SCCG_E_RANGE -2  /* (device) pair index out of range, pair-box side > 32767, |coord| > 2^30 */
#define SCCG_E_POLY -3   /* (validate) non-axis-aligned edge or ring of fewer than 4 vertices */
#define SCCG_E_HIP -4    /* a HIP runtime call failed; message carries hipGetErrorString */
#define SCCG_E_NOMEM -5  /* device allocation failed */
#define SCCG_E_DEVICE -6 /* (device) a kernel's bounded wait ran out (watchdog) */
#define SCCG_E_STATE -7  /* call not allowed in the context's current state */

/* ------------------------------------------------------------- modes ---- */
/* PLAIN: the direct GPU form of Section 3.3's method (the paper's Algorithm
 * 1): one pair per workgroup, a stack of live sampling boxes in LDS, one
 * sub-box per thread placed by Lemma 1 against every edge, one pixel per
 * thread at the leaves tested against every edge. */
#define SCCG_PLAIN 0u
/* BATCHED: a sweep over all pairs, then one persistent launch over the
 * pairs whose box is larger than a leaf tile, with a device task queue that
 * spreads the hovering sampling boxes of large pairs over workgroups.
 * Leaves are bit-sliced 64x64-pixel tiles: a prefix XOR over the columns of
 * per-column row masks gives the crossing parities.  The sweep counts a
 * pair whose MBR union fits one tile directly there (every ring vertex with
 * one vertical edge XORs the rows at or above it into the column left of
 * it); the persistent kernel classifies boxes edge-parallel and XORs each
 * band edge's row mask into one column slot. */
#define SCCG_BATCHED 1u

/* sccg_params.flags (ablation switches; none changes any count) */
#define SCCG_F_NO_LPT 0x1u          /* batched: no heavy-first ordering (heavy pairs are swept) */
#define SCCG_F_NO_KNOWN_INSIDE 0x2u /* batched: re-test a polygon already known to contain a box */
#define SCCG_F_NO_SPLIT_QUEUE 0x4u  /* batched: a large pair's boxes stay with the wave that split it */
#define SCCG_F_NO_GRAPH 0x8u        /* batched: launch the kernels directly, no HIP graph      */
/* The two baselines of Section 5.2 (Figure 8), as ablations of BATCHED mode.
 * Both count the union directly, pixel by pixel, over the bounding box of
 * MBR(p) ∪ MBR(q), instead of deriving it from the polygon areas:
 *   PIXEL_ONLY: no sampling boxes, every pixel of that box is tested;
 *   NO_SEP:     sampling boxes, but a box stops only when it is decided for
 *               both the intersection and the union.
 * Counts are identical to the default; only the work differs. */
#define SCCG_F_PIXEL_ONLY 0x10u
#define SCCG_F_NO_SEP 0x20u
/* batched: by default a pair (not shared through the queue, rings of at most
 * 128 vertices) whose MBR(p) ∪ MBR(q) fits one 64 x 64 leaf tile is counted
 * directly on that tile: the intersection and the union are popcounts of the
 * AND and the OR of the two row masks, so the ring areas are not needed.
 * This flag turns that off (every pair derives U from the areas). */
#define SCCG_F_NO_UNION_TILE 0x40u

/* sccg_jaccard_sets flags */
#define SCCG_J_NONZERO_ONLY 0u /* default: only pairs with I > 0 contribute (Equation 1's filter) */
#define SCCG_J_INCLUDE_ZERO 1u /* every pair contributes                                          */

typedef struct sccg_ctx sccg_ctx;

typedef struct {
  int64_t n_polys;
  const int64_t* offsets; /* [n_polys+1], offsets[0] = 0, non-decreasing (device)   */
  const int32_t* xy;      /* [2*offsets[n_polys]] interleaved x, y (device)          */
} sccg_polys;

/* Tuning parameters.  0 in any field means "default or autotuned".  No value
 * changes any count; out-of-range values give SCCG_E_ARG. */
typedef struct {
  int32_t wg_size;        /* PLAIN: threads per workgroup, 64/128/256 (default 64)                  */
  int32_t box_threshold;  /* PLAIN: pixelize when BOXSIZE < T (default wg_size^2/2, Section 3.4)     */
  int32_t split_gx;       /* PLAIN: sub-box grid; split_gx*split_gy == wg_size (default square-ish) */
  int32_t split_gy;
  int32_t queue_chunk;    /* BATCHED: pairs claimed per counter access, 1..64 (default 16)            */
  int32_t lds_vertex_cap; /* PLAIN: vertices of both rings staged in LDS, 1..4096 (default 1024; above
                             it the rings are read from global memory)                               */
  uint32_t flags;         /* SCCG_F_*                                                                 */
  int32_t grid;           /* workgroups of the persistent (BATCHED) or grid-stride (PLAIN) launch    */
  int32_t queue_cap;      /* BATCHED: slots per task queue, 1..2^26 (default 2^20); a full queue makes
                             the producing wave process its boxes itself                             */
  int32_t waves_per_wg;   /* BATCHED: waves per workgroup, 1..8 (default 4)                          */
  int32_t min_queue_cells;/* BATCHED: a split publishes its boxes to the queue only when at least this
                             many continue (default 8); fewer stay with the splitting wave          */
  int32_t n_queues;       /* BATCHED: device queues, 1..8 (default 8, one per XCD)                   */
  int32_t heavy_verts;    /* BATCHED: pairs with at least this many vertices (both rings) are claimed
                             first and may share their boxes through the queue (default 512)        */
  int32_t min_classify_cells; /* BATCHED: a split into 64-pixel leaf tiles classifies its tiles (Lemma
                             1) only when it has at least this many, 1..65; a smaller split pixelizes
                             every tile of a polygon not known to contain it (default 26)           */
  int32_t sweep_pair_box; /* BATCHED: 2 = the union sweep also counts, on its pair box MBR(p) ∩ MBR(q)
                             (Section 3.2), a pair whose union box exceeds a 64 x 64 leaf tile but
                             whose pair box fits one, from the rings it already holds; pays on mixes
                             with many such pairs (densely packed sets).  1 = it leaves them to the
                             medium sweep, which loads the rings again (default 1)                  */
} sccg_params;

/* Create a context on HIP device `hip_device` using stream `hip_stream`
 * (a hipStream_t; NULL = the device's null stream).  `params` may be NULL.
 * The context owns its scratch (polygon metadata, queues, counters). */
int sccg_create(sccg_ctx** out, int hip_device, void* hip_stream, const sccg_params* params);

/* Synchronize the context's stream and free everything the context owns. */
int sccg_destroy(sccg_ctx* ctx);

/* Replace the tuning parameters (same rules as sccg_create). */
int sccg_set_params(sccg_ctx* ctx, const sccg_params* params);
int sccg_get_params(const sccg_ctx* ctx, sccg_params* out);

/* Pre-size the scratch so that later calls up to these sizes allocate
 * nothing (needed before capturing calls into a HIP graph).  Growing the
 * scratch frees the old buffers, so it also drops the context's captured
 * batched graph, which is captured again on the next call. */
int sccg_reserve(sccg_ctx* ctx, int64_t max_polys_a, int64_t max_polys_b, int64_t max_pairs);

/* Per pair k: out_inter[k] = |A[pair_a[k]] ∩ B[pair_b[k]]| and
 * out_union[k] = |A[pair_a[k]] ∪ B[pair_b[k]]| in pixels (int64), exactly.
 * Section 3's problem statement: an array of polygon pairs in, areas of
 * intersection and union out.  mode = SCCG_PLAIN or SCCG_BATCHED; both give
 * identical counts.  A pair whose index is out of range or whose pair box
 * (MBR(p) ∩ MBR(q)) has a side above 32767 gets 0, 0 and latches
 * SCCG_E_RANGE.  Output arrays must not alias inputs. */
int sccg_area_pairs(sccg_ctx* ctx, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs,
                    const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter, int64_t* out_union,
                    uint32_t mode);

/* Per set s over pairs [set_pair_off[s], set_pair_off[s+1]) (Section 2.1 and
 * Equation 1):
 *   out_sum_i[s], out_sum_u[s] = sums of inter / union over contributing pairs (int64),
 *   out_n_contrib[s]           = number of contributing pairs,
 *   out_j[s]                   = (double)sum_i / (double)sum_u, one IEEE division (0 if sum_u == 0),
 *   out_jprime[s] (nullable)   = mean of inter/union over contributing pairs: each ratio is one
 *                                IEEE division, their sum is formed exactly and rounded once to
 *                                binary64, then divided by n (0 if n == 0).
 * Contributing = inter > 0 unless flags has SCCG_J_INCLUDE_ZERO.  set_pair_off
 * must be non-decreasing with set_pair_off[0] >= 0 (all device pointers). */
int sccg_jaccard_sets(sccg_ctx* ctx, int64_t n_sets, const int64_t* set_pair_off, const int64_t* inter,
                      const int64_t* uni, uint32_t flags, int64_t* out_sum_i, int64_t* out_sum_u,
                      int64_t* out_n_contrib, double* out_j, double* out_jprime);

/* The filter stage of Section 4.1 on the device: candidate pairs of two
 * polygon sets are the pairs whose MBRs intersect.  For each set s, every
 * (a, b) with a in [a_set_off[s], a_set_off[s+1]) and b in
 * [b_set_off[s], b_set_off[s+1]) whose MBRs (the pixel extents
 * [min x, max x) x [min y, max y) of their vertices) share at least one
 * pixel, each once, ordered by set, then b, then a: the input that
 * sccg_area_pairs and sccg_jaccard_sets take.
 *   a_set_off, b_set_off: device int64 [n_sets+1], non-decreasing, within
 *     [0, n_polys] of A and B.
 *   cell: side in pixels of the uniform grid that indexes each set's A
 *     polygons (0 = 64); a set whose grid would exceed 2^24 cells latches
 *     SCCG_E_RANGE and yields no pairs.
 *   out_pa, out_pb: device int32 [cap]; written only if the total fits.
 *   out_set_off: device int64 [n_sets+1], offsets of each set's pairs
 *     (always written, counting every pair).
 *   *out_total (host): the number of pairs; if it exceeds cap, no pair is
 *     written: call again with cap >= *out_total.
 * The call waits for the context's stream three times (to size its scratch
 * and to read the total), so it cannot be captured in a HIP graph. */
int sccg_join_sets(sccg_ctx* ctx, const sccg_polys* A, const sccg_polys* B, int64_t n_sets,
                   const int64_t* a_set_off, const int64_t* b_set_off, int32_t cell, int64_t cap,
                   int32_t* out_pa, int32_t* out_pb, int64_t* out_set_off, int64_t* out_total);

/* sccg_relate_pairs result bits (Section 3.4's other spatial operators) */
#define SCCG_REL_INTERSECTS 0x1u /* a common pixel: I > 0                                        */
#define SCCG_REL_CONTAINS 0x2u   /* A contains B: I == |B| > 0 (ST_Contains from the counts)       */
#define SCCG_REL_WITHIN 0x4u     /* A within B: I == |A| > 0                                       */
#define SCCG_REL_EQUALS 0x8u     /* the same pixels: I == |A| == |B| > 0                           */
#define SCCG_REL_TOUCHES 0x10u   /* no common pixel, but the boundaries share a point (ST_Touches) */

/* Per pair k, the bits above for (A[pair_a[k]], B[pair_b[k]]), from
 * inter[k] (the intersection counts of the same pairs, as sccg_area_pairs
 * writes them), the polygon areas, and, for pairs with no common pixel whose
 * closed MBRs meet, a test of every edge of one ring against every edge of
 * the other (axis-parallel closed segments) -- Section 3.4's suggestion for
 * ST_Contains and ST_Touches.  out_rel: device uint32 [n_pairs].  A pair
 * index out of range gives 0 and latches SCCG_E_RANGE. */
int sccg_relate_pairs(sccg_ctx* ctx, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs,
                      const int32_t* pair_a, const int32_t* pair_b, const int64_t* inter, uint32_t* out_rel);

/* PixelBox on the host CPU (the PixelBox-CPU of Section 4.2): the same
 * counts as sccg_area_pairs, from HOST arrays, on n_threads threads (< 1 =
 * 1), synchronously; no context or GPU is needed.  Sampling boxes split in
 * four down to boxes of at most 64 x 64 pixels below 4096 pixels, whose rows
 * are tested as 64-bit masks.  The serving path runs it on jobs it moves
 * off a congested device.  A pair index out of range returns SCCG_E_RANGE
 * before any work.  A pair box side above 32767 gives (0, 0) and a ring with
 * a coordinate magnitude above 2^30 covers nothing; either makes the call
 * return SCCG_E_RANGE after every count has been written. */
int sccg_host_area_pairs(const sccg_polys* A, const sccg_polys* B, int64_t n_pairs, const int32_t* pair_a,
                         const int32_t* pair_b, int64_t* out_inter, int64_t* out_union, int n_threads);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * BATCHED mode of sccg_area_pairs, with the same arguments and the same
 * results, that calls no hipMalloc, hipFree or other allocating routine.
 * Its scratch (batched state, task queues, per-pair records and lists) is a
 * static device array of about 19 MiB that every GPU the library runs on
 * holds until the process ends; its device address is taken once per device
 * by sccg_create.  Limits: at most 2^18 = 262144 pairs per call (more gives
 * SCCG_E_ARG with a message naming the limit), task queues of at most 2^17
 * slots in all (queue_cap is lowered to fit, which changes no count), device
 * ordinals below 64.  Work counters and timing are not collected and no HIP
 * graph is used (the kernels are launched on the context's stream).  Every
 * call on one GPU uses that GPU's one array and leaves its state there for
 * the next call, which clears what must start at zero: calls that overlap on
 * one GPU (on different streams or contexts, without ordering between them)
 * race and give wrong results. */
int sccg_area_pairs_noalloc(sccg_ctx* ctx, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs,
                            const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter, int64_t* out_union);

/* Check the input form the method assumes (Section 3.1 and Figure 3: a
 * segmented object's boundary follows pixel sides, so a polygon has integer
 * vertices and only horizontal and vertical edges): every ring of P has at
 * least 4 vertices and every edge, the closing one included, is axis-aligned
 * (a repeated vertex, i.e. an edge of length 0, passes).  Simplicity and the
 * absence of holes are not checked.  Writes the smallest bad polygon index,
 * or -1, to *out_first_bad (device int64, caller-owned).  Asynchronous on the
 * context's stream; read the value after sccg_sync.  SCCG_E_ARG for a NULL
 * context, polygon set or output. */
int sccg_validate_polys(sccg_ctx* ctx, const sccg_polys* P, int64_t* out_first_bad);

/* Wait for the context's stream; return SCCG_E_RANGE / SCCG_E_DEVICE if the
 * device latched an error since the last sync (and clear it), else SCCG_OK. */
int sccg_sync(sccg_ctx* ctx);

/* Work counters of the last sccg_area_pairs call, valid after sccg_sync.
 * Counting costs a few atomics per box and is on only while
 * sccg_set_stats(ctx, flags) has bit 0 set; bit 1 turns on the per-wave
 * stamps of sccg_get_wave_times (no atomics), other bits give SCCG_E_ARG
 * (the HIP graph is rebuilt on a change).
 *   [0] leaf pixel tests: pixels of leaf boxes x polygons tested there
 *   [1] leaf boxes       [2] split boxes
 *   [3] boxes published to the device queue (BATCHED)
 *   [4] boxes kept by the splitting wave although enough to publish (BATCHED)
 *   [5] small pairs (one leaf tile)   [6] large pairs   [7] pairs with an empty
 *       or rejected pair box (BATCHED)
 *   [8] leaf edge updates: BATCHED, staged band edges x leaf tiles;
 *       PLAIN, leaf pixels x ring edges tested
 *   [9] classification edge visits: BATCHED, ring edges x splits;
 *       PLAIN, sub-boxes x ring edges tested
 *   [10] ring edges read while staging leaf tiles (BATCHED)
 *   [11] covered pixels: sum of the non-empty pair-box areas (BATCHED)
 *   [12] vertices reduced for MBRs and areas: by the prepass of listed pairs
 *        and by the medium sweep (BATCHED)
 *   [13] vertices reduced for union boxes only, of pairs counted on one leaf tile (BATCHED)
 *   [14] leaf vertex updates: vertices XORed into a leaf slot by the union
 *        tile's vertex form of the crossing test (BATCHED)
 * Writes min(n, 16) values to out; returns that count (or an error < 0). */
int sccg_set_stats(sccg_ctx* ctx, int enable);
int sccg_get_stats(sccg_ctx* ctx, int64_t* out, int n);

/* Load balance of BATCHED mode (Algorithm 1's pairs spread over the grid):
 * while stamps are on (sccg_set_stats bit 1), every wave of the union sweep (kernel 0), the
 * medium sweep (1) and the persistent kernel (2) stamps its start and its
 * end with the device's constant-rate 100 MHz counter.  Waits for the
 * context's stream, writes min(waves, max_waves) (start, end) pairs of the
 * last such call's kernel to out (host int64 [2 * max_waves]) and returns
 * the kernel's wave count (0 before any such call), or an error < 0
 * (SCCG_E_ARG for a kernel outside [0, 2] or a NULL out with max_waves > 0). */
int64_t sccg_get_wave_times(sccg_ctx* ctx, int kernel, int64_t* out, int64_t max_waves);

/* Time the kernels of every sccg_area_pairs call (the plain kernel, or every
 * launch of BATCHED mode, from the reset of its state to the persistent
 * kernel, back to back) with HIP events recorded on the context's stream
 * around them.  While timing is on, BATCHED mode
 * launches its kernels directly instead of through the HIP graph.
 * sccg_get_timing waits for the stream, returns the summed milliseconds and
 * the number of timed launches since the last sccg_get_timing (or since
 * timing was enabled), and starts a new sum. */
int sccg_set_timing(sccg_ctx* ctx, int enable);
int sccg_get_timing(sccg_ctx* ctx, double* out_ms, int64_t* out_launches);

/* Message of the last error on this context ("" if none). */
const char* sccg_last_error(const sccg_ctx* ctx);

/* Number of BATCHED sccg_area_pairs calls on this context that ran as a
 * replay of its captured HIP graph (on a non-null stream, without
 * SCCG_F_NO_GRAPH and with timing off); -1 for a NULL context. */
int64_t sccg_graph_launches(const sccg_ctx* ctx);

/* ------------------------------------------------------------ serving ---- */
/* A server answers a stream of jobs, each one cross-comparison of two
 * polygon sets over a list of candidate pairs (the unit of work of Section
 * 4.1's pipeline: a tile's two result sets after the MBR filter).  Jobs
 * are copied into resident device arenas when they are admitted, run
 * together in bounded persistent launches (every admitted job that has not
 * run yet joins the next launch: the aggregator stage of Section 4.1, which
 * groups small tile tasks and is the only one to launch kernels), and
 * retired in submission order.  A job is admitted once its
 * footprint fits in all three arenas; until then it waits, and later jobs
 * wait behind it.  Results are identical to sccg_area_pairs (BATCHED) plus
 * sccg_jaccard_sets over the job's pairs, whatever else runs beside it.
 *
 * Unlike the calls above, sccg_server_submit takes HOST pointers.  They are
 * borrowed until the job's result has been returned by sccg_server_poll.
 * Offsets and pair indices are copied on admission into pinned mirrors of
 * the arenas and sent from there; vertices are sent straight from the
 * caller's memory, so they should be pinned (hipHostMalloc): a copy from
 * pageable memory holds the scheduler until the copy stream reaches it.  A
 * server runs its own scheduler thread and two streams on its device;
 * submit, poll, stats and clock may be called from any thread. */
typedef struct sccg_server sccg_server;

typedef struct {
  int64_t vertex_cap;     /* resident vertex arena, in vertices (8 B each); 0 = 2^28                  */
  int64_t slot_cap;       /* resident offset arena, in entries (8 B of device and 8 B of pinned host
                             memory each): a job takes n_polys(A) + n_polys(B) + 2; 0 = 2^24, at most
                             2^31 - 1                                                                 */
  int64_t pair_cap;       /* resident pair arena, in pairs (24 B of device and 24 B of pinned host
                             memory each); 0 = 2^23                                                   */
  int64_t max_step_pairs; /* pairs per launch; a larger job runs alone in its launch; 0 = 2^21        */
  int32_t max_inflight;   /* launches queued on the device at once, 1..4; 0 = 2                      */
  uint32_t jaccard_flags; /* SCCG_J_* for the per-job sums                                            */
  /* Migration to the host CPU (Section 4.2's GPU-to-CPU direction): while at
   * least cpu_trigger jobs wait for admission (the arenas, the device's input
   * buffer, are full), the scheduler moves the waiting job with the fewest
   * pairs, if it has at most cpu_max_pairs, to a migration thread that runs
   * it with the host PixelBox on cpu_threads threads (a pool kept for the
   * server's life), one job at a time.  Its result is bit-identical to the
   * device's, with jobs_in_launch 0.                                         */
  int32_t cpu_threads;    /* 0 = no migration; at most 256                                            */
  int32_t cpu_trigger;    /* waiting jobs that wake the migration; 0 = 1                              */
  int64_t cpu_max_pairs;  /* largest job that migrates; 0 = 2^20                                      */
} sccg_server_config;

typedef struct {
  uint64_t job_id;       /* as returned by sccg_server_submit                                        */
  int32_t status;        /* SCCG_OK, or SCCG_E_RANGE / SCCG_E_DEVICE for the job's own pairs (a launch
                            that latches an error runs each of its jobs again alone to attribute it),
                            or SCCG_E_HIP if the server failed; the same alone and in a mix          */
  int32_t jobs_in_launch;/* jobs that shared the job's launch; 0 = run on host threads (migrated)     */
  int64_t n_pairs;
  int64_t sum_i, sum_u, n_contrib; /* as sccg_jaccard_sets over the job's pairs                      */
  double j, jprime;
  double t_submit, t_admit, t_launch, t_done; /* seconds on the server's clock: submitted, copied
                             into the arenas (migrated: handed to the migration thread), launched
                             (migrated: started on the host), results on the host                    */
} sccg_job_result;

/* Create a server on HIP device `hip_device`.  `config` and `params` may be
 * NULL (defaults); `params` tunes the batched launches (SCCG_F_NO_GRAPH is
 * implied).  All device and pinned memory is allocated here. */
int sccg_server_create(sccg_server** out, int hip_device, const sccg_server_config* config,
                       const sccg_params* params);

/* Queue one job: pairs (A[pair_a[k]], B[pair_b[k]]), k < n_pairs, with A and
 * B given as host CSR (here offsets[0] need not be 0: polygon k's vertices
 * are xy[2*offsets[k]] ... xy[2*offsets[k+1]-1]).  out_inter / out_union
 * (host, [n_pairs], nullable) receive the per-pair counts before the job is
 * reported done.  Offsets and pair indices are checked here (SCCG_E_ARG); a
 * job larger than an arena gives SCCG_E_NOMEM; a failed server gives
 * SCCG_E_STATE.  A job with no pairs completes at once.  *out_job_id gets
 * the job's id (ids count up from 1). */
int sccg_server_submit(sccg_server* srv, const sccg_polys* A, const sccg_polys* B, int64_t n_pairs,
                       const int32_t* pair_a, const int32_t* pair_b, int64_t* out_inter, int64_t* out_union,
                       uint64_t* out_job_id);

/* Move up to max_results finished jobs into out (in completion order),
 * waiting up to timeout_us microseconds for the first one (0 = do not wait,
 * < 0 = wait without limit).  Returns the number written. */
int sccg_server_poll(sccg_server* srv, sccg_job_result* out, int max_results, int64_t timeout_us);

/* Server counters: [0] jobs submitted [1] jobs done [2] launches [3] pairs
 * done [4] peak resident vertices [5] peak resident offset entries [6] peak
 * resident pairs [7] admission waits (the oldest queued job did not fit)
 * [8] most jobs in one launch [9] jobs rejected at submit [10] jobs run on
 * host threads (migrated) [11] pairs run on host threads.  Writes
 * min(n, 12) values; returns that count. */
int sccg_server_get_stats(sccg_server* srv, int64_t* out, int n);

/* Seconds since the server was created, on the clock of sccg_job_result. */
double sccg_server_clock(const sccg_server* srv);

/* Message of the last error of this server ("" if none). */
const char* sccg_server_last_error(sccg_server* srv);

/* Finish every submitted job, stop the scheduler and free everything.
 * Results not yet polled are dropped. */
int sccg_server_destroy(sccg_server* srv);

/* Diagnostic: the device's sustained integer VALU rate, the peak against
 * which the persistent kernel's work is measured.  Runs a kernel in which
 * every lane of 8 waves per SIMD on every compute unit issues independent
 * 32-bit integer adds and XORs (32 per loop trip, `iters` trips, 1..2^24),
 * once untimed and once timed with HIP events on the context's stream, and
 * waits for it.  *out_lane_ops_per_s = lane-operations per second of the
 * timed launch, *out_ms its duration.  The nominal figure is 256 CUs x 64
 * lanes x 2.4 GHz = 39.3e12. */
int sccg_valu_peak(sccg_ctx* ctx, int32_t iters, double* out_lane_ops_per_s, double* out_ms);

/* Library version string. */
const char* sccg_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SCCG_H */
