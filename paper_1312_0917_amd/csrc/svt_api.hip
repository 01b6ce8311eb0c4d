// Host side of the libsvt C ABI: argument checks, workspace layout, launch sequences and the
// HIP-graph cache of svt_process_batch.  Every function only enqueues on the given stream.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <mutex>
#include <tuple>
#include <vector>

#include "svt_common.h"

namespace svt {
// launcher of k_gather (svt_stages.hip), used by svt_gather_results only
hipError_t launch_gather(const svt_roads &roads, const svt_best &best, int64_t road_cap,
                         const int64_t *d_n_words, const int64_t *d_n_roads,
                         const int64_t *d_n_combos, const int64_t *d_n_kept,
                         const uint64_t *d_err, void *out, int64_t out_roads, hipStream_t s);
}  // namespace svt

using namespace svt;

namespace {

constexpr int64_t kAlign = 256;
inline int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

bool config_ok(const svt_config *c) {
    return c && c->n_layers == SVT_N_LAYERS && c->shift >= 1 && c->shift <= 30 &&
           c->max_hits >= 1 && c->max_hits <= SVT_MAX_HITS && c->n_sets >= 1 && c->n_sets <= 256;
}

bool aligned(const void *p, uintptr_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Workspace carving: a bump allocator over the caller's buffer.
struct Carver {
    char *base;
    int64_t used = 0;
    template <typename T>
    T *take(int64_t count) {
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += align_up(static_cast<int64_t>(sizeof(T)) * (count > 0 ? count : 1));
        return p;
    }
};

struct UnpackWs {
    int64_t *scalars;  // [0] event total
    int64_t *wb;       // [2][nb]
    int64_t nb;
};
UnpackWs carve_unpack(Carver &c, int64_t n_words) {
    UnpackWs w;
    w.nb = ceil_div(n_words > 0 ? n_words : 1, kSegBlockWords);
    w.scalars = c.take<int64_t>(4);
    w.wb = c.take<int64_t>(2 * w.nb);
    return w;
}

struct BatchWs {
    uint32_t *tickets;  // [0] fused-kernel tiles (or events of the event schedule); rest spare
    int64_t *n_events;  // events of the batch
    int32_t *efr;       // first road of every event
    int64_t events_cap;
    int64_t *status;    // look-back status words
    int64_t status_words;
    int64_t nb;         // one-pass units of the capacity
    int32_t *tfr;
    int64_t tiles_cap;
    int64_t *kb;
    int64_t kbn;
    int16_t *coords;
    int64_t *nw_copy;   // the batch's word count, copied to device memory by the reset
};
BatchWs carve_batch(Carver &c, int64_t word_cap, int64_t road_cap, int64_t combo_cap,
                    int64_t tile) {
    BatchWs w;
    w.tickets = c.take<uint32_t>(4);
    w.n_events = c.take<int64_t>(2);
    w.events_cap = road_cap > 0 ? road_cap : 1;  // every event holds at least one road
    w.efr = c.take<int32_t>(w.events_cap);
    // status words for the one-pass units or for the pre-pass blocks and their groups
    w.nb = ceil_div(word_cap > 0 ? word_cap : 1, kOnepassUnitWords);
    const int64_t pre = prepass_status_words(ceil_div(word_cap > 0 ? word_cap : 1,
                                                      kPrepassBlockWords));
    w.status_words = 2 * w.nb > pre ? 2 * w.nb : pre;
    w.status = c.take<int64_t>(w.status_words);
    // tile marks at the smaller of the tile and the kept block (the one-pass kernel marks
    // kept blocks)
    w.tiles_cap = ceil_div(combo_cap > 0 ? combo_cap : 1, tile < kKeptBlock ? tile : kKeptBlock) + 1;
    w.tfr = c.take<int32_t>(w.tiles_cap);
    w.kbn = ceil_div(combo_cap > 0 ? combo_cap : 1, kKeptBlock);
    w.kb = c.take<int64_t>(w.kbn);
    w.coords = c.take<int16_t>(word_cap + 16);  // slack for 16-byte reads of the last span
    w.nw_copy = c.take<int64_t>(1);
    return w;
}

// Batches of at most this many words (capacity) run the one-pass kernel by default, larger ones
// the pre-pass and fused kernels: per-unit latency dominates the one-pass kernel once every
// workgroup has several units of small roads (on 3000 events of 64 roads the two tie at the
// default tile, and the pre-pass path leads with 8192-combination tiles).
constexpr int64_t kOnepassDefaultWords = 1 << 19;

// Launch parameters for `t` (zero fields take the defaults).  A zero schedule stays zero when
// no capacity is given (word_cap < 0), and is chosen from the capacity otherwise.
svt_tune resolve_tune(const svt_tune *t, int64_t word_cap = -1) {
    svt_tune r{4096, 64, 256, 3, 0};
    if (t) {
        if (t->tile_combos) r.tile_combos = t->tile_combos;
        if (t->chunk_roads) r.chunk_roads = t->chunk_roads;
        if (t->wg_size) r.wg_size = t->wg_size;
        if (t->wgs_per_cu) r.wgs_per_cu = t->wgs_per_cu;
        if (t->schedule) r.schedule = t->schedule;
    }
    if (r.schedule == 0 && word_cap >= 0)
        r.schedule = word_cap <= kOnepassDefaultWords ? SVT_SCHEDULE_ONEPASS : SVT_SCHEDULE_TILES;
    return r;
}

// A tune is valid when its fields are, before the capacity picks a zero schedule (which must
// then suit both schedules), and after.
bool tune_ok(const svt_tune *t, int64_t word_cap) {
    return fused_tune_supported(resolve_tune(t)) &&
           fused_tune_supported(resolve_tune(t, word_cap));
}

int num_cus() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    static std::mutex mu;
    static std::map<int, int> cache;
    std::lock_guard<std::mutex> lock(mu);
    auto it = cache.find(dev);
    if (it != cache.end()) return it->second;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) n = 0;
    cache[dev] = n;
    return n;
}

#define SVT_TRY(x)                                  \
    do {                                            \
        if ((x) != hipSuccess) return SVT_ERR_HIP;  \
    } while (0)

hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;
std::mutex g_graph_mu;

using GraphKey = std::vector<uint64_t>;
struct GraphEntry {
    hipGraph_t graph;
    hipGraphExec_t exec;
};
std::map<GraphKey, GraphEntry> &graph_cache() {
    static std::map<GraphKey, GraphEntry> m;
    return m;
}

}  // namespace

extern "C" {

int32_t svt_abi_version(void) { return SVT_ABI_VERSION; }

svt_status svt_copy_async(void *dst, const void *src, int64_t bytes, int32_t kind,
                          hipStream_t stream) {
    if (bytes < 0 || (bytes > 0 && (!dst || !src))) return SVT_ERR_ARG;
    if (kind != SVT_COPY_H2D && kind != SVT_COPY_D2H) return SVT_ERR_ARG;
    if (bytes == 0) return SVT_OK;
    const hipMemcpyKind k = kind == SVT_COPY_H2D ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
    return hipMemcpyAsync(dst, src, static_cast<size_t>(bytes), k, stream) == hipSuccess
               ? SVT_OK
               : SVT_ERR_HIP;
}

svt_status svt_event_record(hipEvent_t event, hipStream_t stream) {
    if (!event) return SVT_ERR_ARG;
    return hipEventRecord(event, stream) == hipSuccess ? SVT_OK : SVT_ERR_HIP;
}

int32_t svt_event_done(hipEvent_t event) {
    if (!event) return SVT_ERR_ARG;
    const hipError_t e = hipEventQuery(event);
    if (e == hipSuccess) return 1;
    if (e == hipErrorNotReady) return 0;
    return SVT_ERR_HIP;
}

svt_status svt_mapped_pointer(void *host, void **dev) {
    if (!host || !dev) return SVT_ERR_ARG;
    *dev = nullptr;
    return hipHostGetDevicePointer(dev, host, 0) == hipSuccess && *dev ? SVT_OK : SVT_ERR_HIP;
}

svt_status svt_gather_results(const svt_roads *roads, const svt_best *best, int64_t road_cap,
                              const int64_t *d_n_words, const int64_t *d_n_roads,
                              const int64_t *d_n_combos, const int64_t *d_n_kept,
                              const uint64_t *d_err, void *out, int64_t out_roads,
                              hipStream_t stream) {
    if (!roads || !best || !d_n_words || !d_n_roads || !d_n_combos || !d_err || !out)
        return SVT_ERR_ARG;
    if (!roads->event || !roads->set || !best->n_accept || !best->k || !best->p0 || !best->p1 ||
        !best->p2 || !best->chi2)
        return SVT_ERR_ARG;
    if (road_cap < 0 || out_roads < 0 || out_roads > (INT64_MAX - 64) / 36) return SVT_ERR_ARG;
    if (reinterpret_cast<uintptr_t>(out) % 8 != 0) return SVT_ERR_ARG;
    return launch_gather(*roads, *best, road_cap, d_n_words, d_n_roads, d_n_combos, d_n_kept, d_err,
                         out, out_roads, stream) == hipSuccess
               ? SVT_OK
               : SVT_ERR_HIP;
}

svt_status svt_tune_resolve(const svt_tune *tune, svt_tune *out) {
    if (!out) return SVT_ERR_ARG;
    *out = resolve_tune(tune);
    return fused_tune_supported(*out) ? SVT_OK : SVT_ERR_ARG;
}

svt_status svt_tune_for_batch(const svt_tune *tune, int64_t word_cap, svt_tune *out) {
    if (!out || word_cap < 0) return SVT_ERR_ARG;
    *out = resolve_tune(tune, word_cap);
    return tune_ok(tune, word_cap) ? SVT_OK : SVT_ERR_ARG;
}

const char *svt_status_name(svt_status s) {
    switch (s) {
        case SVT_OK: return "SVT_OK";
        case SVT_ERR_ARG: return "SVT_ERR_ARG";
        case SVT_ERR_LAYER: return "SVT_ERR_LAYER";
        case SVT_ERR_HITS: return "SVT_ERR_HITS";
        case SVT_ERR_CAPACITY: return "SVT_ERR_CAPACITY";
        case SVT_ERR_HIP: return "SVT_ERR_HIP";
        case SVT_ERR_SET: return "SVT_ERR_SET";
        default: return "SVT_ERR_UNKNOWN";
    }
}

svt_status svt_error_decode(uint64_t err, int64_t *index) {
    if (err == SVT_NO_ERROR) {
        if (index) *index = -1;
        return SVT_OK;
    }
    const uint32_t cls = static_cast<uint32_t>(err >> 56);
    if (index) *index = static_cast<int64_t>(err & ((1ull << 56) - 1));
    switch (cls) {
        case SVT_ERRCLASS_LAYER: return SVT_ERR_LAYER;
        case SVT_ERRCLASS_HITS: return SVT_ERR_HITS;
        case SVT_ERRCLASS_SET: return SVT_ERR_SET;
        case SVT_ERRCLASS_CAPACITY: return SVT_ERR_CAPACITY;
        default: return SVT_ERR_ARG;
    }
}

int64_t svt_unpack_workspace(int64_t n_words) {
    if (n_words < 0) return -1;
    Carver c{nullptr};
    carve_unpack(c, n_words);
    return c.used;
}

int64_t svt_combine_workspace(int64_t n_roads) {
    if (n_roads < 0) return -1;
    return align_up(8 * ceil_div(n_roads > 0 ? n_roads : 1, kRoadBlock));
}

int64_t svt_select_workspace(int64_t n_combos) {
    if (n_combos < 0) return -1;
    return align_up(8 * ceil_div(n_combos > 0 ? n_combos : 1, kKeptBlock));
}

int64_t svt_batch_workspace(int64_t word_cap, int64_t road_cap, int64_t combo_cap,
                            const svt_tune *tune) {
    if (word_cap < 0 || word_cap > kMaxBatchWords || road_cap < 0 || combo_cap < 0) return -1;
    const svt_tune t = resolve_tune(tune, word_cap);
    if (!tune_ok(tune, word_cap)) return -1;
    Carver c{nullptr};
    carve_batch(c, word_cap, road_cap, combo_cap, t.tile_combos);
    return c.used;
}

svt_status svt_unpack(const uint32_t *words, int64_t n_words, const svt_config *cfg,
                      const svt_roads *roads, int64_t road_cap, int16_t *hit_coord,
                      int64_t *d_n_roads, uint64_t *d_err, void *d_work, int64_t work_bytes,
                      hipStream_t stream) {
    if (!config_ok(cfg) || !roads || n_words < 0 || road_cap < 0 || !d_n_roads || !d_err)
        return SVT_ERR_ARG;
    if (n_words > 0 && (!words || !hit_coord)) return SVT_ERR_ARG;
    if (road_cap > 0 && (!roads->event || !roads->set || !roads->hit_begin || !roads->nhits))
        return SVT_ERR_ARG;
    if (!d_work || work_bytes < svt_unpack_workspace(n_words) || !aligned(d_work, kAlign))
        return SVT_ERR_ARG;
    Carver c{static_cast<char *>(d_work)};
    UnpackWs w = carve_unpack(c, n_words);
    const Sizes nw{n_words, nullptr, n_words};
    SVT_TRY(launch_init_err(d_err, stream));
    SVT_TRY(launch_seg_count(words, nw, w.nb, cfg->n_layers, w.wb, d_err, stream));
    SVT_TRY(launch_scan(w.wb, w.nb, 2, nw, kSegBlockWords, d_n_roads, w.scalars, road_cap, 0,
                        d_err, false, stream));
    SVT_TRY(launch_seg_emit(words, nw, w.nb, w.wb, *roads, road_cap, d_err, stream));
    SVT_TRY(launch_road_fill(words, nw, d_n_roads, road_cap, *roads, *cfg, hit_coord, nullptr,
                             d_err, stream));
    return SVT_OK;
}

svt_status svt_combine(const svt_roads *roads, int64_t n_roads, const svt_config *cfg,
                       int32_t *combo_road, uint32_t *combo_hits, int64_t combo_cap,
                       int64_t *d_n_combos, uint64_t *d_err, void *d_work, int64_t work_bytes,
                       hipStream_t stream) {
    if (!config_ok(cfg) || !roads || n_roads < 0 || combo_cap < 0 || !d_n_combos || !d_err)
        return SVT_ERR_ARG;
    if (n_roads > 0 && (!roads->nhits || !roads->ncombo || !roads->combo_begin))
        return SVT_ERR_ARG;
    if (!d_work || work_bytes < svt_combine_workspace(n_roads) || !aligned(d_work, kAlign))
        return SVT_ERR_ARG;
    int64_t *rb = static_cast<int64_t *>(d_work);
    const int64_t rbn = ceil_div(n_roads > 0 ? n_roads : 1, kRoadBlock);
    const Sizes nr{n_roads, nullptr, n_roads};
    const bool listing = combo_road || combo_hits;
    SVT_TRY(launch_combo_count(*roads, nr, rbn, rb, d_err, stream));
    SVT_TRY(launch_scan(rb, 0, 1, nr, kRoadBlock, d_n_combos, nullptr, listing ? combo_cap : -1,
                        1, d_err, true, stream));
    SVT_TRY(launch_combo_begin(*roads, nr, rbn, rb, 0, nullptr, 0, nullptr, d_err, stream));
    if (listing)
        SVT_TRY(launch_materialize(*roads, n_roads, d_n_combos, combo_cap, combo_road, combo_hits,
                                   d_err, stream));
    return SVT_OK;
}

svt_status svt_fit(const svt_fconst *bank, const svt_config *cfg, const svt_roads *roads,
                   int64_t n_roads, const int16_t *hit_coord, int64_t n_hits,
                   const int32_t *combo_road, const uint32_t *combo_hits, int64_t n_combos,
                   const svt_fitrec *out, uint64_t *d_err, hipStream_t stream) {
    if (!config_ok(cfg) || !roads || !out || !d_err || n_roads < 0 || n_hits < 0 || n_combos < 0)
        return SVT_ERR_ARG;
    if (n_combos > 0 && (!bank || !hit_coord || !combo_road || !combo_hits || !out->p0 ||
                         !out->p1 || !out->p2 || !out->chi2 || !roads->nhits ||
                         !roads->hit_begin || !roads->set))
        return SVT_ERR_ARG;
    SVT_TRY(launch_fit_plain(bank, *cfg, *roads, n_roads, hit_coord, n_hits, combo_road,
                             combo_hits, n_combos, *out, d_err, stream));
    return SVT_OK;
}

svt_status svt_select(const svt_config *cfg, const svt_roads *roads, int64_t n_roads,
                      const int32_t *combo_road, const svt_fitrec *rec, int64_t n_combos,
                      uint8_t *accept, const svt_best *best, int64_t *kept, int64_t kept_cap,
                      int64_t *d_n_kept, uint64_t *d_err, void *d_work, int64_t work_bytes,
                      hipStream_t stream) {
    if (!config_ok(cfg) || !roads || !rec || !best || !d_err || n_roads < 0 || n_combos < 0 ||
        kept_cap < 0)
        return SVT_ERR_ARG;
    if (n_combos > 0 && (!combo_road || !rec->chi2 || !rec->p0 || !rec->p1 || !rec->p2 ||
                         !accept || !roads->combo_begin))
        return SVT_ERR_ARG;
    if (n_roads > 0 && (!best->n_accept || !best->k || !best->p0 || !best->p1 || !best->p2 ||
                        !best->chi2 || !roads->combo_begin || !roads->ncombo))
        return SVT_ERR_ARG;
    if (kept && !d_n_kept) return SVT_ERR_ARG;
    if (!d_work || work_bytes < svt_select_workspace(n_combos) || !aligned(d_work, kAlign))
        return SVT_ERR_ARG;
    int64_t *kb = static_cast<int64_t *>(d_work);
    const int64_t kbn = ceil_div(n_combos > 0 ? n_combos : 1, kKeptBlock);
    SVT_TRY(launch_select(*cfg, *roads, n_roads, combo_road, *rec, n_combos, accept, *best, kb,
                          d_err, stream));
    if (d_n_kept) {
        const Sizes nc{n_combos, nullptr, n_combos};
        SVT_TRY(launch_scan(kb, 0, 1, nc, kKeptBlock, d_n_kept, nullptr, kept ? kept_cap : -1, 2,
                            d_err, true, stream));
        if (kept && n_combos > 0)
            SVT_TRY(launch_kept_write(accept, nc, kbn, kb, kept, kept_cap, d_err, stream));
    }
    return SVT_OK;
}

void svt_set_fused_timing_events(hipEvent_t start, hipEvent_t stop) {
    g_ev_start = start;
    g_ev_stop = stop;
}

static svt_status batch_sequence(const FusedLaunch &f, const BatchWs &w, int64_t word_cap,
                                 int64_t road_cap, int64_t combo_cap, int64_t *kept,
                                 int64_t kept_cap, int64_t *d_n_kept, bool timing,
                                 hipStream_t stream) {
    const Sizes nw{0, f.d_n_words, word_cap};
    // after the reset the kernels read the word count from its copy in device memory
    const Sizes nw_dev{0, w.nw_copy, word_cap};
    const Sizes nr{0, f.d_n_roads, road_cap};
    const Sizes nc{0, f.d_n_combos, combo_cap};
    PrepassLaunch p{};
    p.words = f.words;
    p.nw = nw;
    p.cfg = f.cfg;
    p.roads = f.roads;
    p.road_cap = road_cap;
    p.coords = const_cast<int16_t *>(f.coords);
    p.best = f.best;
    p.tile_combos = f.tune.tile_combos;
    p.tile_first_road = w.tfr;
    p.tiles_cap = w.tiles_cap;
    p.combo_cap = combo_cap;
    p.d_n_roads = const_cast<int64_t *>(f.d_n_roads);
    p.d_n_combos = const_cast<int64_t *>(f.d_n_combos);
    p.status = w.status;
    p.nb_cap = w.nb;
    p.tickets = w.tickets;
    p.err = f.err;
    p.event_first_road = w.efr;
    p.event_cap = w.events_cap;
    p.d_n_events = w.n_events;
    uint64_t *err = f.err;
    if (f.tune.schedule == SVT_SCHEDULE_ONEPASS) {
        // reset, the one-pass kernel, and with a kept list its scan and compaction
        p.nb_cap = w.nb;
        p.status_words = 2 * w.nb;
        SVT_TRY(launch_batch_reset(p, w.nw_copy, d_n_kept, d_n_kept ? w.kb : nullptr,
                                   d_n_kept ? w.kbn : 0, stream));
        OnepassLaunch o{};
        o.bank = f.bank;
        o.cfg = f.cfg;
        o.words = f.words;
        o.nw = nw_dev;
        o.roads = f.roads;
        o.road_cap = road_cap;
        o.rec = f.rec;
        o.accept = f.accept;
        o.best = f.best;
        o.combo_cap = combo_cap;
        o.d_n_roads = p.d_n_roads;
        o.d_n_combos = p.d_n_combos;
        o.kb_counts = d_n_kept ? w.kb : nullptr;
        o.status = w.status;
        o.nb_cap = w.nb;
        o.tickets = w.tickets;
        o.err = err;
        o.kept_only = f.kept_only;
        o.coords = w.coords;
        o.tile_first_road = w.tfr;
        o.tiles_cap = w.tiles_cap;
        o.num_cus = f.num_cus;
        o.wgs_per_cu = f.tune.wgs_per_cu;
        if (timing) SVT_TRY(hipEventRecord(g_ev_start, stream));
        SVT_TRY(launch_onepass(o, stream));
        if (timing) SVT_TRY(hipEventRecord(g_ev_stop, stream));
        if (d_n_kept) {
            SVT_TRY(launch_scan(w.kb, 0, 1, nc, kKeptBlock, d_n_kept, nullptr,
                                kept ? kept_cap : -1, 2, err, true, stream));
            if (kept && f.kept_only)
                SVT_TRY(launch_kept_refit(f.accept, nc, nr, w.kbn, w.kb, f.roads, w.tfr,
                                          kKeptBlock, f.bank, f.cfg.n_sets, f.coords,
                                          f.cfg.shift, kept, f.rec, kept_cap, err, stream));
            else if (kept)
                SVT_TRY(launch_kept_write(f.accept, nc, w.kbn, w.kb, kept, kept_cap, err,
                                          stream));
        }
        return SVT_OK;
    }
    // (the kept-list block counts are cleared with the rest: the fused kernel adds to them)
    p.nb_cap = ceil_div(word_cap > 0 ? word_cap : 1, kPrepassBlockWords);
    p.status_words = prepass_status_words(p.nb_cap);
    SVT_TRY(launch_batch_reset(p, w.nw_copy, d_n_kept, d_n_kept ? w.kb : nullptr,
                               d_n_kept ? w.kbn : 0, stream));
    p.nw = nw_dev;
    SVT_TRY(launch_prepass(p, stream));
    if (timing) SVT_TRY(hipEventRecord(g_ev_start, stream));
    if (f.tune.schedule == SVT_SCHEDULE_EVENTS)
        SVT_TRY(launch_fit_events(f, w.efr, w.n_events, w.events_cap, stream));
    else
        SVT_TRY(launch_fused(f, stream));
    if (timing) SVT_TRY(hipEventRecord(g_ev_stop, stream));
    // the kept list's block counts are scanned by one extra workgroup of the finalize launch
    ScanJob job;
    if (d_n_kept) {
        job.data = w.kb;
        job.n = nc;
        job.div = kKeptBlock;
        job.tot = d_n_kept;
        job.cap = kept ? kept_cap : -1;
        job.cap_index = 2;
    }
    SVT_TRY(launch_best_finalize(f.roads, nr, f.kept_only ? svt_fitrec{} : f.rec, nc, f.best,
                                 f.cfg.chi2_cut, err, true, f.bank, f.coords, f.cfg.shift, job,
                                 stream));
    if (d_n_kept) {
        if (kept && f.kept_only)
            SVT_TRY(launch_kept_refit(f.accept, nc, nr, w.kbn, w.kb, f.roads, w.tfr,
                                      f.tune.tile_combos, f.bank, f.cfg.n_sets, f.coords,
                                      f.cfg.shift, kept, f.rec, kept_cap, err, stream));
        else if (kept)
            SVT_TRY(launch_kept_write(f.accept, nc, w.kbn, w.kb, kept, kept_cap, err, stream));
    }
    return SVT_OK;
}

}  // extern "C"

namespace {

// ---- the workspace of svt_process_batch_static ----------------------------------------------
// One array per GPU in this library's code object, held until the process ends.  In host code
// its name is only the runtime's handle for it: the device address is taken once per device
// with hipGetSymbolAddress and used everywhere instead.
static __device__ __align__(256) char scratch[SVT_STATIC_WORK_BYTES];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

svt_status static_workspace(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return SVT_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SVT_ERR_HIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return SVT_OK;
}

// work_bytes value that selects the static workspace (d_work is then ignored)
constexpr int64_t kStaticWork = -2;

// svt_process_batch on the caller's workspace, or on the static one (work_bytes == kStaticWork).
svt_status process_batch(const svt_fconst *bank, const svt_config *cfg, const svt_tune *tune,
                         const uint32_t *words, const int64_t *d_n_words, int64_t word_cap,
                         const svt_roads *roads, int64_t road_cap, const svt_fitrec *rec,
                         uint8_t *accept, int64_t combo_cap, const svt_best *best, int64_t *kept,
                         int64_t kept_cap, int64_t *d_n_roads, int64_t *d_n_combos,
                         int64_t *d_n_kept, uint64_t *d_err, void *d_work, int64_t work_bytes,
                         int32_t flags, hipStream_t stream) {
    if (!config_ok(cfg) || !bank || !words || !d_n_words || !roads || !rec || !best ||
        !d_n_roads || !d_n_combos || !d_err || word_cap < 0 || word_cap > kMaxBatchWords ||
        road_cap < 0 || combo_cap < 0 ||
        kept_cap < 0)
        return SVT_ERR_ARG;
    if (kept && !d_n_kept) return SVT_ERR_ARG;
    const bool kept_only = (flags & SVT_BATCH_KEPT_ONLY) != 0;
    if (kept_only && (!kept || !d_n_kept)) return SVT_ERR_ARG;
    if (!roads->event || !roads->set || !roads->hit_begin || !roads->nhits ||
        !roads->combo_begin || !roads->ncombo)
        return SVT_ERR_ARG;
    if (!best->n_accept || !best->k || !best->p0 || !best->p1 || !best->p2 || !best->chi2)
        return SVT_ERR_ARG;
    if (!rec->p0 || !rec->p1 || !rec->p2 || !rec->chi2 || !accept) return SVT_ERR_ARG;
    const void *a16[] = {rec->p0, rec->p1, rec->p2, rec->chi2, rec->c0, rec->c1, rec->c2};
    for (const void *p : a16)
        if (p && !aligned(p, 16)) return SVT_ERR_ARG;
    if (!aligned(accept, 4)) return SVT_ERR_ARG;
    const svt_tune t = resolve_tune(tune, word_cap);
    if (!tune_ok(tune, word_cap)) return SVT_ERR_ARG;
    if (work_bytes == kStaticWork) {  // svt_process_batch_static
        if (flags & SVT_BATCH_GRAPH) return SVT_ERR_ARG;  // instantiating a graph allocates
        if (svt_batch_workspace(word_cap, road_cap, combo_cap, &t) > SVT_STATIC_WORK_BYTES)
            return SVT_ERR_CAPACITY;
        const svt_status st = static_workspace(&d_work);
        if (st != SVT_OK) return st;
        work_bytes = SVT_STATIC_WORK_BYTES;
    } else if (!d_work || work_bytes < svt_batch_workspace(word_cap, road_cap, combo_cap, &t) ||
               !aligned(d_work, kAlign)) {
        return SVT_ERR_ARG;
    }
    const int cus = num_cus();
    if (cus <= 0) return SVT_ERR_HIP;

    Carver c{static_cast<char *>(d_work)};
    const BatchWs w = carve_batch(c, word_cap, road_cap, combo_cap, t.tile_combos);
    FusedLaunch f{};
    f.bank = bank;
    f.cfg = *cfg;
    f.tune = t;
    f.words = words;
    f.d_n_words = d_n_words;
    f.coords = w.coords;
    f.roads = *roads;
    f.d_n_roads = d_n_roads;
    f.d_n_combos = d_n_combos;
    f.rec = *rec;
    f.accept = accept;
    f.best = *best;
    f.tile_first_road = w.tfr;
    f.kb_counts = d_n_kept ? w.kb : nullptr;
    f.tile_counter = w.tickets;
    f.err = d_err;
    f.tiles_cap = w.tiles_cap;
    f.road_cap = road_cap;
    f.combo_cap = combo_cap;
    f.num_cus = cus;
    f.kept_only = kept_only;

    if (!(flags & SVT_BATCH_GRAPH)) {
        const bool timing = g_ev_start && g_ev_stop;
        return batch_sequence(f, w, word_cap, road_cap, combo_cap, kept, kept_cap, d_n_kept,
                              timing, stream);
    }

    // graph path: key on every value the launch sequence bakes in
    int dev = 0;
    SVT_TRY(hipGetDevice(&dev));
    auto u = [](const void *p) { return static_cast<uint64_t>(reinterpret_cast<uintptr_t>(p)); };
    GraphKey key = {static_cast<uint64_t>(dev), u(stream), u(bank), u(words), u(d_n_words),
                    static_cast<uint64_t>(word_cap), static_cast<uint64_t>(road_cap),
                    static_cast<uint64_t>(combo_cap), static_cast<uint64_t>(kept_cap),
                    u(roads->event), u(roads->set), u(roads->hit_begin), u(roads->nhits),
                    u(roads->combo_begin), u(roads->ncombo), u(rec->p0), u(rec->p1), u(rec->p2),
                    u(rec->chi2), u(rec->c0), u(rec->c1), u(rec->c2), u(accept), u(best->n_accept),
                    u(best->k), u(best->p0), u(best->p1), u(best->p2), u(best->chi2), u(kept),
                    u(d_n_roads), u(d_n_combos), u(d_n_kept), u(d_err), u(d_work),
                    static_cast<uint64_t>(work_bytes), static_cast<uint64_t>(cfg->shift),
                    static_cast<uint64_t>(cfg->chi2_cut), static_cast<uint64_t>(cfg->max_hits),
                    static_cast<uint64_t>(cfg->n_sets), static_cast<uint64_t>(t.tile_combos),
                    static_cast<uint64_t>(t.chunk_roads), static_cast<uint64_t>(t.wg_size),
                    static_cast<uint64_t>(t.wgs_per_cu), static_cast<uint64_t>(t.schedule),
                    static_cast<uint64_t>(flags)};
    std::lock_guard<std::mutex> lock(g_graph_mu);
    auto &cache = graph_cache();
    auto it = cache.find(key);
    if (it == cache.end()) {
        SVT_TRY(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
        svt_status st = batch_sequence(f, w, word_cap, road_cap, combo_cap, kept, kept_cap,
                                       d_n_kept, false, stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(stream, &g);
        if (st != SVT_OK || e != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return st != SVT_OK ? st : SVT_ERR_HIP;
        }
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
            (void)hipGraphDestroy(g);
            return SVT_ERR_HIP;
        }
        it = cache.emplace(key, GraphEntry{g, ex}).first;
    }
    SVT_TRY(hipGraphLaunch(it->second.exec, stream));
    return SVT_OK;
}


}  // namespace

extern "C" {

svt_status svt_process_batch(const svt_fconst *bank, const svt_config *cfg, const svt_tune *tune,
                             const uint32_t *words, const int64_t *d_n_words, int64_t word_cap,
                             const svt_roads *roads, int64_t road_cap, const svt_fitrec *rec,
                             uint8_t *accept, int64_t combo_cap, const svt_best *best,
                             int64_t *kept, int64_t kept_cap, int64_t *d_n_roads,
                             int64_t *d_n_combos, int64_t *d_n_kept, uint64_t *d_err,
                             void *d_work, int64_t work_bytes, int32_t flags,
                             hipStream_t stream) {
    if (work_bytes < 0) return SVT_ERR_ARG;
    return process_batch(bank, cfg, tune, words, d_n_words, word_cap, roads, road_cap, rec, accept,
                         combo_cap, best, kept, kept_cap, d_n_roads, d_n_combos, d_n_kept, d_err,
                         d_work, work_bytes, flags, stream);
}

svt_status svt_process_batch_static(const svt_fconst *bank, const svt_config *cfg,
                                    const svt_tune *tune, const uint32_t *words,
                                    const int64_t *d_n_words, int64_t word_cap,
                                    const svt_roads *roads, int64_t road_cap,
                                    const svt_fitrec *rec, uint8_t *accept, int64_t combo_cap,
                                    const svt_best *best, int64_t *kept, int64_t kept_cap,
                                    int64_t *d_n_roads, int64_t *d_n_combos, int64_t *d_n_kept,
                                    uint64_t *d_err, int32_t flags, hipStream_t stream) {
    return process_batch(bank, cfg, tune, words, d_n_words, word_cap, roads, road_cap, rec, accept,
                         combo_cap, best, kept, kept_cap, d_n_roads, d_n_combos, d_n_kept, d_err,
                         nullptr, kStaticWork, flags, stream);
}

svt_status svt_static_workspace_need(int64_t word_cap, int64_t road_cap, int64_t combo_cap,
                                     const svt_tune *tune, int64_t *need, int64_t *limit) {
    if (!need || !limit) return SVT_ERR_ARG;
    *limit = SVT_STATIC_WORK_BYTES;
    *need = svt_batch_workspace(word_cap, road_cap, combo_cap, tune);
    return *need < 0 ? SVT_ERR_ARG : *need > *limit ? SVT_ERR_CAPACITY : SVT_OK;
}
void svt_release_graphs(void) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (auto &kv : graph_cache()) {
        (void)hipGraphExecDestroy(kv.second.exec);
        (void)hipGraphDestroy(kv.second.graph);
    }
    graph_cache().clear();
}

}  // extern "C"
