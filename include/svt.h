/*
 * svt.h -- C ABI of the SVT linearized track fitter for AMD Instinct MI355X (gfx950).
 *
 * The method (Gianelle et al., IEEE NSS 2013, arXiv:1312.0917):
 *   section II   : every one-hit-per-layer combination of hits inside a road is fitted; each
 *                  track parameter is a scalar product of pre-defined constants with the hit
 *                  coordinates plus an offset, p_i = f_i . x_i + q_i, evaluated with table
 *                  lookups and integer additions and multiplications, together with the
 *                  chi-square of the fitted track;
 *   section II-A : the serial code is three stages -- unpack the input words and fill the
 *                  data structures, compute all hit combinations of each road, fit each
 *                  combination -- inside loops over events, roads and combinations.
 * svt_unpack, svt_combine and svt_fit are those three stages; svt_select applies the
 * chi-square cut and picks the best track of every road; svt_process_batch runs all four as
 * one persistent fused pass (optionally replayed from a captured HIP graph).
 *
 * Exact definitions where the paper is silent (all arithmetic is integer and exact):
 *   hit word (uint32, LSB first): coord 13 bits two's complement | layer 3 | road tag 8 |
 *     event tag 8.  A new event starts where the event tag changes, a new road where either
 *     tag changes (tags are delimiters, roads and events are numbered in stream order).
 *   constant set of a road = its road tag.  Hits of a road are grouped by layer, stream order
 *     kept inside a layer.  Combination k of a road is mixed-radix over the layers with layer 0
 *     most significant (k = ((((h0*n1 + h1)*n2 + h2)*n3 + h3)*n4 + h4).
 *   v_j = floor((sum_l f[j][l] * x_l + q[j]) / 2^shift), j = 0..5, computed exactly;
 *     p = v_0..2 (track parameters), c = v_3..5 (chi-square components),
 *     chi2 = c0^2 + c1^2 + c2^2 (int64).  A combination is accepted when chi2 <= chi2_cut.
 *   best track of a road: its accepted combination of smallest chi2, the smallest k among
 *     equal chi2.  A road with none: k = -1, p = INT32_MIN, chi2 = INT64_MAX, n_accept = 0.
 *
 * Conventions shared by every entry point:
 *   - Pointers to device memory are written d_* or are fields of the svt_roads / svt_fitrec /
 *     svt_best structs; the caller allocates and owns all of them.  Structs themselves and
 *     svt_config / svt_tune are read from host memory during the call only.
 *   - The library allocates no device memory.  Scratch comes from the caller's workspace
 *     (d_work, work_bytes; size from the matching *_workspace function, 256-byte aligned), or
 *     for svt_process_batch_static from a static array in the library's code object.  The
 *     only other library-owned objects are the HIP graphs cached by svt_process_batch, freed
 *     by svt_release_graphs().
 *   - Every call only enqueues work on `stream` and returns; nothing synchronises.
 *   - The return value reports host-side checks: SVT_OK, SVT_ERR_ARG (null pointer, negative
 *     size, bad configuration, misaligned output), SVT_ERR_HIP (a launch failed).  On an error
 *     nothing is enqueued.
 *   - Errors found in the data are written on the device to the error word *d_err (uint64):
 *     SVT_NO_ERROR (all ones) or (class << 56) | index, and the smallest such value wins, so
 *     the reported error is deterministic: layer-field errors first (index = word), then too
 *     many hits in a layer (index = road), then a road tag without a constant set (index =
 *     road), then capacity (index 0 roads, 1 combinations, 2 kept list).  svt_error_decode()
 *     turns the word into an svt_status and index.  After a data error the outputs are
 *     unspecified except the sizes: *d_n_roads and *d_n_combos are always the sizes the input
 *     needs (a road with too many hits in a layer counts no combination), so a caller can grow
 *     its buffers and retry; *d_n_kept is the accepted count when the fit ran, -1 otherwise.
 *   - Kernels never write past a capacity and never read outside the given arrays, whatever
 *     the input words contain.
 *   - Output arrays of the fused pass must be 16-byte aligned (accept: 4-byte aligned).
 */
#ifndef SVT_H
#define SVT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SVT_ABI_VERSION 1

typedef int32_t svt_status;
#define SVT_OK 0
#define SVT_ERR_ARG (-1)
#define SVT_ERR_LAYER (-2)
#define SVT_ERR_HITS (-3)
#define SVT_ERR_CAPACITY (-4)
#define SVT_ERR_HIP (-5)
#define SVT_ERR_SET (-6)

#define SVT_NO_ERROR UINT64_MAX
#define SVT_ERRCLASS_LAYER 1u
#define SVT_ERRCLASS_HITS 2u
#define SVT_ERRCLASS_SET 3u
#define SVT_ERRCLASS_CAPACITY 4u
#define SVT_ERRCLASS_INDEX 5u /* svt_fit / svt_select given an out-of-range road or hit index */

#define SVT_N_LAYERS 5
#define SVT_MAX_HITS 8

/* One constant set (88 bytes): rows 0-2 track parameters, rows 3-5 chi-square components;
 * column = layer; q is in the scale of f . x (2^shift per unit of the result). */
typedef struct svt_fconst {
    int16_t f[6][5];
    int16_t pad[2];
    int32_t q[6];
} svt_fconst;

typedef struct svt_config {
    int32_t n_layers; /* must be 5 */
    int32_t shift;    /* fixed-point shift, 1..30 (10 for the benchmark) */
    int64_t chi2_cut; /* accept when chi2 <= chi2_cut */
    int32_t max_hits; /* most hits allowed in one layer of a road, 1..8 */
    int32_t n_sets;   /* constant sets in the bank, 1..256 */
} svt_config;

/* Road table, structure of arrays, one entry per road in stream order (device memory). */
typedef struct svt_roads {
    int32_t *event;       /* event ordinal */
    int32_t *set;         /* road tag = constant set */
    int64_t *hit_begin;   /* index of the road's first word (also its first hit_coord) */
    uint32_t *nhits;      /* hits per layer, 4 bits per layer, layer l in bits 4l..4l+3 */
    int64_t *combo_begin; /* index of the road's first combination */
    int32_t *ncombo;      /* number of combinations = product of the hits per layer */
} svt_roads;

/* Per-combination fit records, structure of arrays (device memory). c0..c2 may be NULL. */
typedef struct svt_fitrec {
    int32_t *p0, *p1, *p2;
    int64_t *chi2;
    int32_t *c0, *c1, *c2;
} svt_fitrec;

/* Best track per road (device memory). */
typedef struct svt_best {
    int32_t *n_accept;
    int32_t *k; /* combination index inside the road, -1 when none */
    int32_t *p0, *p1, *p2;
    int64_t *chi2;
} svt_best;

/* Launch parameters of the batched pass; zeros pick the built-in defaults. */
typedef struct svt_tune {
    int32_t tile_combos;  /* two-kernel schedule: combinations per work tile, 4096 or 8192 */
    int32_t chunk_roads;  /* two-kernel schedule: roads staged in LDS at once at most: 16, 32
                             or 64 (fewer when their hits or pair tables fill the stage) */
    int32_t wg_size;      /* two-kernel schedule: 256 or 512 (one loader wave, the rest fit) */
    int32_t wgs_per_cu;   /* persistent workgroups per compute unit, 1..8 (one pass: 1..3);
                             the two-kernel schedule launches no more workgroups than
                             combo_cap has tiles */
    int32_t schedule;     /* SVT_SCHEDULE_*; 0 chooses per call from word_cap: the one-pass
                             kernel up to 2^19 words, the two-kernel schedule above (0 must
                             then suit both: wgs_per_cu 1..3).  The fields a schedule does
                             not use only have to be valid values. */
} svt_tune;
/* One persistent kernel that unpacks, combines, fits and selects units of 1024 words, each
 * workgroup holding its unit's roads, pair tables and best tracks in LDS (the loop nest of
 * section II-A per unit); the pass is that kernel and a reset of its look-back state. */
#define SVT_SCHEDULE_ONEPASS 2
/* One event per workgroup at a time (the multi-core scheme of section II-A, an ablation). */
#define SVT_SCHEDULE_EVENTS 1
/* A single-pass pre-pass writes the road table and grouped coordinates, then a persistent
 * kernel fits flat tiles of tile_combos combinations and a last launch finalizes the best
 * tracks (four launches per pass). */
#define SVT_SCHEDULE_TILES 3

/* ---- sizes of the caller-provided scratch ------------------------------------------------ */
int64_t svt_unpack_workspace(int64_t n_words);
int64_t svt_combine_workspace(int64_t n_roads);
int64_t svt_select_workspace(int64_t n_combos);
int64_t svt_batch_workspace(int64_t word_cap, int64_t road_cap, int64_t combo_cap,
                            const svt_tune *tune);

/* Stage 1, unpack (section II-A, first function): decode words[0..n_words) and fill the road
 * table fields event, set, hit_begin, nhits for at most road_cap roads; hit_coord[n_words]
 * receives the int13 coordinates regrouped by layer inside each road (stream order inside a
 * layer), so road r's layer-l hits start at hit_begin[r] + (hits of layers < l).  Writes the
 * number of roads to *d_n_roads.  Resets *d_err, then reports layer, hit-count, road-tag
 * (tag >= n_sets) and road-capacity errors in it.  words: uint32 device array (any alignment). */
svt_status svt_unpack(const uint32_t *words, int64_t n_words, const svt_config *cfg,
                      const svt_roads *roads, int64_t road_cap, int16_t *hit_coord,
                      int64_t *d_n_roads, uint64_t *d_err, void *d_work, int64_t work_bytes,
                      hipStream_t stream);

/* Stage 2, combine (section II-A, second function): for roads[0..n_roads) set ncombo (product
 * of the hits per layer) and combo_begin (exclusive prefix sum), write the total to
 * *d_n_combos and, when combo_road / combo_hits are non-NULL and the total fits combo_cap,
 * list every combination: its road and its hit index in each layer (4 bits per layer, layer l
 * in bits 4l..4l+3).  Reports combination-capacity errors in *d_err (not reset). */
svt_status svt_combine(const svt_roads *roads, int64_t n_roads, const svt_config *cfg,
                       int32_t *combo_road, uint32_t *combo_hits, int64_t combo_cap,
                       int64_t *d_n_combos, uint64_t *d_err, void *d_work, int64_t work_bytes,
                       hipStream_t stream);

/* Stage 3, fit (section II, the scalar-product equation): one fit per listed combination.
 * bank[n_sets] device array of svt_fconst; hit_coord[n_hits] from svt_unpack; combo_road /
 * combo_hits[n_combos] from svt_combine.  Writes out->p0..p2, out->chi2 and, when non-NULL,
 * out->c0..c2.  Indices outside the road table or the hit array are reported in *d_err (class
 * INDEX, index = combination) and that combination is skipped. */
svt_status svt_fit(const svt_fconst *bank, const svt_config *cfg, const svt_roads *roads,
                   int64_t n_roads, const int16_t *hit_coord, int64_t n_hits,
                   const int32_t *combo_road, const uint32_t *combo_hits, int64_t n_combos,
                   const svt_fitrec *out, uint64_t *d_err, hipStream_t stream);

/* Stage 4, select (section II: the fit yields the chi-square of each fitted track, and that
 * chi-square is what a trigger keeps or rejects a track by).  The paper prints no cut and no
 * rule for a road's best track; this library's readings are: accept[i] = (rec->chi2[i] <=
 * chi2_cut), inclusive; the best track of a road is its accepted combination of smallest
 * chi2, the first in enumeration order (smallest k) among equal chi2, which is what the serial
 * loop nest of section II-A keeps with a strict "<".  Per road: n_accept and that best track
 * (k, p0..p2, chi2; none: k = -1, p = INT32_MIN, chi2 = INT64_MAX).  combo_road[n_combos]
 * (from svt_combine) names each record's road; rec holds the records of svt_fit.  When kept is
 * non-NULL, the ascending indices of accepted combinations (at most kept_cap written, the
 * count in *d_n_kept; d_n_kept alone gives the count without the list).  Indices outside the
 * road table are reported in *d_err (class INDEX, index = combination) and skipped. */
svt_status svt_select(const svt_config *cfg, const svt_roads *roads, int64_t n_roads,
                      const int32_t *combo_road, const svt_fitrec *rec, int64_t n_combos,
                      uint8_t *accept, const svt_best *best, int64_t *kept, int64_t kept_cap,
                      int64_t *d_n_kept, uint64_t *d_err, void *d_work, int64_t work_bytes,
                      hipStream_t stream);

/* The whole path in one pass (sections II and II-A: unpack, combine, fit, plus the chi-square
 * selection), writing the same records, accept flags, road table and best tracks as stages 1-4
 * (bit for bit) with one of two schedules (svt_tune.schedule; 0 chooses from word_cap, see
 * svt_tune_for_batch):
 *   - SVT_SCHEDULE_ONEPASS: one persistent kernel unpacks, combines, fits and selects units of
 *     1024 words, each workgroup holding its unit's roads in LDS (plus a reset launch);
 *   - SVT_SCHEDULE_TILES: a single-pass pre-pass reads every word once and writes the road
 *     table, the layer-grouped coordinates and each road's combination range (decoupled
 *     look-back over blocks of 2048 words); a persistent fused kernel then takes tiles of
 *     tile_combos consecutive combinations, stages the roads' hits and constants in LDS and fits
 *     every combination with integer VALU arithmetic; a last launch writes the best tracks.  The word count is read on the device from *d_n_words, so
 * a captured graph can be replayed for any batch up to word_cap (at most 2^31 - 1 words;
 * larger capacities are SVT_ERR_ARG, and svt_batch_workspace returns -1 for them).
 * flags: SVT_BATCH_GRAPH
 * captures the launch sequence in a HIP graph on first use (keyed by every argument) and
 * replays it afterwards.  kept may be NULL; with d_n_kept also NULL no accepted count and no
 * kept list are produced.  Resets *d_err. */
#define SVT_BATCH_GRAPH 1
/* flags: SVT_BATCH_KEPT_ONLY writes no per-combination records -- the output a trigger
 * consumes (section II: the fit's chi-square decides which tracks are kept).  accept[] is still
 * written per combination and best[] per road; kept (required, with d_n_kept) receives the
 * ascending indices of the accepted combinations and rec their fit values, compacted: entry i
 * of rec->p0..p2, chi2 (and c0..c2 when non-NULL) belongs to combination kept[i], kept_cap
 * entries each.  The values are fitted again for the accepted combinations only, with the
 * same integer arithmetic, so they equal the records of the default mode bit for bit. */
#define SVT_BATCH_KEPT_ONLY 2
svt_status svt_process_batch(const svt_fconst *bank, const svt_config *cfg, const svt_tune *tune,
                             const uint32_t *words, const int64_t *d_n_words, int64_t word_cap,
                             const svt_roads *roads, int64_t road_cap, const svt_fitrec *rec,
                             uint8_t *accept, int64_t combo_cap, const svt_best *best,
                             int64_t *kept, int64_t kept_cap, int64_t *d_n_roads,
                             int64_t *d_n_combos, int64_t *d_n_kept, uint64_t *d_err,
                             void *d_work, int64_t work_bytes, int32_t flags, hipStream_t stream);

/* For callers that cannot allocate device memory -- code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc: svt_process_batch with the same arguments but no
 * d_work / work_bytes.  Its workspace is one static array of SVT_STATIC_WORK_BYTES bytes per
 * GPU, part of the library's code object and held until the process ends; the call allocates
 * nothing.  Capacities whose workspace (svt_batch_workspace) exceeds that size return
 * SVT_ERR_CAPACITY before anything is enqueued (svt_static_workspace_need reports both
 * numbers); SVT_BATCH_GRAPH is SVT_ERR_ARG (instantiating a graph allocates -- capture the
 * call in a graph of your own instead).  Every call on one GPU uses that GPU's array, and each
 * pass clears what must start at zero: calls whose passes overlap on one GPU (other streams,
 * other threads) race and give wrong results; serialise them.  Outputs and the device-side
 * error word are exactly those of svt_process_batch. */
#define SVT_STATIC_WORK_BYTES (32ll << 20)
svt_status svt_process_batch_static(const svt_fconst *bank, const svt_config *cfg,
                                    const svt_tune *tune, const uint32_t *words,
                                    const int64_t *d_n_words, int64_t word_cap,
                                    const svt_roads *roads, int64_t road_cap,
                                    const svt_fitrec *rec, uint8_t *accept, int64_t combo_cap,
                                    const svt_best *best, int64_t *kept, int64_t kept_cap,
                                    int64_t *d_n_roads, int64_t *d_n_combos, int64_t *d_n_kept,
                                    uint64_t *d_err, int32_t flags, hipStream_t stream);
/* *need = the workspace these capacities take (svt_batch_workspace), *limit =
 * SVT_STATIC_WORK_BYTES; SVT_OK if svt_process_batch_static accepts them, SVT_ERR_CAPACITY if
 * they are too large, SVT_ERR_ARG for invalid capacities or tune. */
svt_status svt_static_workspace_need(int64_t word_cap, int64_t road_cap, int64_t combo_cap,
                                     const svt_tune *tune, int64_t *need, int64_t *limit);

/* When both are non-NULL, svt_process_batch calls without SVT_BATCH_GRAPH record `start`
 * right before and `stop` right after the fused kernel, on the call's stream (for timing). */
void svt_set_fused_timing_events(hipEvent_t start, hipEvent_t stop);

/* Device-side address of page-locked host memory (from hipHostMalloc, e.g. a pinned torch
 * tensor), so kernels can read it in place over the bus ("zero-copy" input).  Returns
 * SVT_ERR_ARG for NULL arguments and SVT_ERR_HIP when the runtime does not know the pointer.
 * Host call, no allocation. */
svt_status svt_mapped_pointer(void *host, void **dev);

/* Host plumbing for callers that drive batches from a host loop (the serving form), so that a
 * binding needs no runtime handle of its own: an asynchronous copy on `stream` between
 * page-locked host memory and device memory (kind SVT_COPY_H2D or SVT_COPY_D2H; bytes >= 0;
 * the host side must stay untouched until the copy has run), an event recorded on a stream,
 * and a poll of such an event (1 done, 0 pending, SVT_ERR_HIP on a runtime error). */
#define SVT_COPY_H2D 1
#define SVT_COPY_D2H 2
svt_status svt_copy_async(void *dst, const void *src, int64_t bytes, int32_t kind,
                          hipStream_t stream);
svt_status svt_event_record(hipEvent_t event, hipStream_t stream);
int32_t svt_event_done(hipEvent_t event);

/* The results of one batch gathered into one buffer, for host loops that read them with no
 * copy call (the serving form: `out` is then the device address of page-locked host memory from
 * svt_mapped_pointer; device memory works as well).  Writes the header int64[8] = {*d_n_words,
 * *d_n_roads, *d_n_combos, *d_n_kept (-1 when d_n_kept is NULL), *d_err, 0, 0, 0}; then, when
 * 0 <= n_roads <= min(out_roads, road_cap), the first n_roads entries of best->chi2 (int64),
 * then those of best->n_accept, best->k, best->p0, best->p1, best->p2, roads->event and
 * roads->set (int32 each), back to back; otherwise the header only.  out must be 8-byte aligned
 * and hold 64 + 36 * out_roads bytes; out_roads >= 0.  Values written to host memory are
 * visible to the host once work enqueued after this call has completed (an event recorded
 * after it).  SVT_ERR_ARG for NULL pointers (except d_n_kept) or a bad size. */
svt_status svt_gather_results(const svt_roads *roads, const svt_best *best, int64_t road_cap,
                              const int64_t *d_n_words, const int64_t *d_n_roads,
                              const int64_t *d_n_combos, const int64_t *d_n_kept,
                              const uint64_t *d_err, void *out, int64_t out_roads,
                              hipStream_t stream);

/* Destroy every cached graph (call before freeing buffers a cached graph refers to). */
void svt_release_graphs(void);

/* Write to `out` the launch parameters svt_process_batch uses for `tune` (NULL or zero fields
 * take the built-in defaults).  Returns SVT_ERR_ARG when `out` is NULL or the resolved set is
 * not one the fused kernel is built for, SVT_OK otherwise.  Host memory only. */
svt_status svt_tune_resolve(const svt_tune *tune, svt_tune *out);
/* The launch parameters svt_process_batch uses for `tune` at word capacity word_cap: as
 * svt_tune_resolve, with a zero schedule replaced by the one chosen for that capacity. */
svt_status svt_tune_for_batch(const svt_tune *tune, int64_t word_cap, svt_tune *out);

/* Turn an error word into a status (SVT_OK when none) and its index (-1 when none). */
svt_status svt_error_decode(uint64_t err, int64_t *index);

const char *svt_status_name(svt_status s);
int32_t svt_abi_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SVT_H */
