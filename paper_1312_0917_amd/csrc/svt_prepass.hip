// Single-pass unpack + combine of the batched path: one kernel reads every hit word once and
// writes the whole road table (event, set, hit_begin, nhits, ncombo, combo_begin), the
// layer-grouped coordinates, the first road of every fit tile and the initial best-track keys.
//
// Section II-A of the paper: the serial code first unpacks the input and fills its data
// structures, then counts the hit combinations of every road.  Both need running counts over
// the whole stream (which road and event a word belongs to, where a road's combinations start);
// here they come from one decoupled look-back over blocks of 2048 words instead of separate
// count / scan / emit launches.
//
// Ownership: a block owns the roads that *start* among its 2048 words.  A road may run past the
// block's last word; the block stages 64 more words, which covers every legal road (at most
// n_layers * max_hits = 40 words), and a road still running after them is reported as a hit-count
// error (some layer must then hold more than max_hits hits).
//
// Everything a block needs from its own words (road list, hits per layer, combinations,
// grouped coordinates, even their coalesced store) is done before it looks back, so the only
// wait is one look-back.  Two 64-bit status words per block carry the running counts -- roads
// and events packed in one (31 bits each: a batch holds fewer than 2^31 words), combinations in
// the other: the top two bits say "aggregate" or "inclusive prefix", the rest hold the value.
// The look-back has two levels (look_back_grouped): a block sums the aggregates of the blocks
// before it in its group of 64 and the values of the groups before that, which the groups'
// last blocks publish.  The status words are cleared by the batch-reset kernel before every
// pass.
//
// LDS per block stays near 21 KB, so that seven blocks fit on a compute unit: the grouped
// coordinates go into the high halves of the staged words of their own road, the road list
// holds 16-bit starts, and a road's event index comes from the same block scan as its first
// combination.
//
// Blocks are numbered by their index in the grid, with no ticket: every block fetching an
// ordered ticket from one counter at the start serialises on that counter (about 12 ns per
// block, 11 us for the last of 940 blocks).  A ticket would guarantee that a block only waits
// on blocks already running; without it, a look-back round that has waited too long computes
// the aggregates it is missing from the words themselves (block_aggregate), so no block can
// wait forever on one that has not been scheduled, and the wait stays bounded.
#include <cstdlib>

#include "svt_lookback_block.h"

namespace svt {
namespace {

constexpr int kPT = 256;                  // threads per block
constexpr int kPB = kPrepassBlockWords;   // 2048 words per block
constexpr int kPW = kPB / kPT;            // 8 words per thread
constexpr int kTail = kRoadTail;          // words staged past the block's own
constexpr int kOff = 4;                   // sw[kOff - 1] = word before the block; the body
                                          // starts 16-byte aligned
struct PArgs {
    const uint32_t *words;
    Sizes nw;
    svt_config cfg;
    svt_roads roads;
    int64_t road_cap;
    int16_t *coords;
    svt_best best;
    int64_t tile_combos;
    int32_t *tile_first_road;
    int64_t tiles_cap;
    int64_t combo_cap;
    int64_t *d_n_roads;
    int64_t *d_n_combos;
    int64_t *status;  // [2][nb_cap]: roads | events << 31, combinations
    int64_t nb_cap;
    uint64_t lookback_timeout;  // wall-clock ticks a look-back waits before computing itself
    uint64_t *err;
    int32_t *event_first_road;
    int64_t event_cap;
    int64_t *d_n_events;
};

// Per owned road, in LDS: s_road[rl] = first local word (12 bits) | the word starts an event
// << 12; s_info[rl] = hits per layer (4 bits each) | road tag << 20 | too-many-hits << 28 |
// no-constant-set << 29.  The road that starts at s_road[rl] ends where road rl + 1 starts, the
// last one at s_tail_end.
constexpr uint32_t kInfoOver = 1u << 28;
constexpr uint32_t kInfoSet = 1u << 29;

__device__ inline int road_end(const uint16_t *s_road, int rl, int nroads, int tail_end) {
    return rl + 1 < nroads ? (s_road[rl + 1] & 0xFFF) : tail_end;
}

__global__ __launch_bounds__(kPT) void k_prepass(PArgs a) {
    // sw[kOff + j] = word base + j.  Once a road's hits are counted, the high halves of its own
    // words receive its coordinates grouped by layer (the low halves, coordinate and layer,
    // stay as read): 16-bit store k of the road goes to the high half of its word k.
    __shared__ __align__(16) uint32_t sw[kOff + kPB + kTail];
    __shared__ uint16_t s_road[kPB];
    __shared__ uint32_t s_info[kPB];
    __shared__ int64_t tmp[kPT / kWaveSize + 1];
    __shared__ GroupLookShared s_look;
    __shared__ int32_t s_tail_end;
    uint16_t *sh16 = reinterpret_cast<uint16_t *>(sw);

    const int tid = threadIdx.x;
    const int64_t n = load_size(a.nw);
    const int64_t b = blockIdx.x;
    const LookbackCtx lc{a.words, n, a.cfg.n_layers, a.cfg.max_hits, a.status, a.nb_cap,
                         a.lookback_timeout};
    const int64_t nb = (n + kPB - 1) / kPB;
    if (b == 0 && tid == 0 && a.nw.dev && *a.nw.dev > a.nw.cap)
        report(a.err, SVT_ERRCLASS_CAPACITY, 3);
    if (b >= nb) {
        if (b == 0 && tid == 0) {  // empty batch
            *a.d_n_roads = 0;
            *a.d_n_combos = 0;
            if (a.d_n_events) *a.d_n_events = 0;
        }
        return;
    }

    // ---- stage the block's words, 64 more, and the word before ------------------------------
    const int64_t base = b * kPB;
    const int nloc = static_cast<int>(n - base < kPB + kTail ? n - base : kPB + kTail);
    const int nown = nloc < kPB ? nloc : kPB;
    const int j0 = tid * kPW;
    const bool aligned16 = (reinterpret_cast<uintptr_t>(a.words) & 15) == 0;
    uint32_t wv[kPW];  // this thread's words, kept for the flags below
    if (aligned16 && j0 + kPW <= nown) {
        const uint4 *p = reinterpret_cast<const uint4 *>(a.words + base + j0);
        uint4 *q = reinterpret_cast<uint4 *>(sw + kOff + j0);
#pragma unroll
        for (int v = 0; v < kPW / 4; ++v) {
            const uint4 u = p[v];
            q[v] = u;
            wv[4 * v] = u.x;
            wv[4 * v + 1] = u.y;
            wv[4 * v + 2] = u.z;
            wv[4 * v + 3] = u.w;
        }
    } else {
#pragma unroll
        for (int e = 0; e < kPW; ++e) {
            wv[e] = (j0 + e < nloc) ? a.words[base + j0 + e] : 0u;
            sw[kOff + j0 + e] = wv[e];
        }
    }
    if (tid < kTail) sw[kOff + kPB + tid] = (kPB + tid < nloc) ? a.words[base + kPB + tid] : 0u;
    if (tid == 0) sw[kOff - 1] = base > 0 ? a.words[base - 1] : 0u;
    __syncthreads();

    // ---- road and event starts of this thread's words ---------------------------------------
    uint32_t rmask = 0, emask = 0;
    int nr = 0, ne = 0;
    int64_t bad = -1;
#pragma unroll
    for (int e = 0; e < kPW; ++e) {
        const int j = j0 + e;
        if (j < nown) {
            const uint32_t x = wv[e];
            const uint32_t px = e == 0 ? sw[kOff + j - 1] : wv[e - 1];
            const bool first = (base + j == 0);
            const bool r = first || w_tags(x) != w_tags(px);
            const bool v = first || w_etag(x) != w_etag(px);
            rmask |= (r ? 1u : 0u) << e;
            emask |= (v ? 1u : 0u) << e;
            nr += r;
            ne += v;
            if (bad < 0 && static_cast<int32_t>(w_layer(x)) >= a.cfg.n_layers) bad = base + j;
        }
    }
    if (bad >= 0) report(a.err, SVT_ERRCLASS_LAYER, static_cast<uint64_t>(bad));
    if (tid < kWaveSize) {
        // end of the last owned road: the first road start among the staged words past the
        // block, else the end of the staged words (the end of the input, or a road longer than
        // any legal one)
        const int j = kPB + tid;
        const bool start = j < nloc && w_tags(sw[kOff + j]) != w_tags(sw[kOff + j - 1]);
        const uint64_t m = __ballot(start);
        if (tid == 0) s_tail_end = nloc <= kPB ? nloc : (m ? kPB + __builtin_ctzll(m) : nloc);
    }
    int64_t tre;  // roads and events of the block, scanned together (each at most 2048)
    const int64_t rel0 = block_excl_scan<int64_t, kPT>(static_cast<int64_t>(nr) |
                                                       (static_cast<int64_t>(ne) << 32), tmp, tre);
    const int64_t tr = tre & 0xFFFFFFFF, te = tre >> 32;
    const int nroads = static_cast<int>(tr);

    // ---- list of owned roads (every event start is a road start: the tags hold both) --------
    {
        int rl = static_cast<int>(rel0 & 0xFFFFFFFF);
#pragma unroll
        for (int e = 0; e < kPW; ++e)
            if ((rmask >> e) & 1u)
                s_road[rl++] = static_cast<uint16_t>((j0 + e) | (((emask >> e) & 1u) << 12));
    }
    __syncthreads();
    const int tail_end = s_tail_end;

    // ---- one road per thread: hits per layer, checks, combinations --------------------------
    // Counts and, below, write offsets per layer are packed 6 bits a layer in one word: a road
    // that is not too long has at most 40 hits.
    const int max_len = a.cfg.n_layers * a.cfg.max_hits;
    int64_t csum = 0;
    for (int rl = tid; rl < nroads; rl += kPT) {
        const int j = s_road[rl] & 0xFFF;
        const int len = road_end(s_road, rl, nroads, tail_end) - j;
        const uint32_t w0 = sw[kOff + j];
        bool over = len > max_len;
        uint32_t cnt = 0;
        if (!over) {
            for (int i0 = 0; i0 < len; i0 += 8) {
                uint32_t x[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) x[u] = i0 + u < len ? sw[kOff + j + i0 + u] : 0xE000u;
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    const uint32_t l = w_layer(x[u]);  // 7 for the padding
                    if (l < SVT_N_LAYERS) cnt += 1u << (6 * l);
                }
            }
        }
        uint32_t packed = 0;
#pragma unroll
        for (int l = 0; l < SVT_N_LAYERS; ++l) {
            const uint32_t c = (cnt >> (6 * l)) & 0x3F;
            over |= c > static_cast<uint32_t>(a.cfg.max_hits);
            packed |= (c & 0xFu) << (4 * l);
        }
        if (!over) csum += combos_of(packed);
        const bool noset = w_rtag(w0) >= static_cast<uint32_t>(a.cfg.n_sets);
        s_info[rl] = packed | (w_rtag(w0) << 20) | (over ? kInfoOver : 0u) |
                     (noset ? kInfoSet : 0u);
    }
    const int64_t tc = block_sum<int64_t, kPT>(csum, tmp);  // (its barrier publishes s_info)
    const uint64_t agg0 = static_cast<uint64_t>(tr) | (static_cast<uint64_t>(te) << 31);
    const uint64_t agg1 = static_cast<uint64_t>(tc);
    // the aggregate is all that later blocks need from this one: publish it before grouping
    if (tid == 0) publish_aggregate(lc, b, agg0, agg1);

    // ---- grouped coordinates of the roads with combinations (while predecessors finish) ----
    for (int rl = tid; rl < nroads; rl += kPT) {
        const uint32_t info = s_info[rl];
        if (info & kInfoOver) continue;
        const int j = s_road[rl] & 0xFFF;
        const int len = road_end(s_road, rl, nroads, tail_end) - j;
        uint32_t off = 0;  // next write position per layer, 6 bits a layer
        uint32_t run = 0;
#pragma unroll
        for (int l = 0; l < SVT_N_LAYERS; ++l) {
            off |= run << (6 * l);
            run += nh_of(info, l);
        }
        for (int i0 = 0; i0 < len; i0 += 8) {
            uint32_t x[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) x[u] = i0 + u < len ? sw[kOff + j + i0 + u] : 0xE000u;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const uint32_t l = w_layer(x[u]);
                if (l >= SVT_N_LAYERS) continue;
                const uint32_t o = (off >> (6 * l)) & 0x3F;
                off += 1u << (6 * l);
                sh16[2 * (kOff + j + static_cast<int>(o)) + 1] = static_cast<uint16_t>(x[u]);
            }
        }
    }
    __syncthreads();

    // ---- grouped coordinates of the owned roads: contiguous, coalesced (no prefix needed) ---
    if (nroads > 0) {
        const int lo = s_road[0] & 0xFFF;
        for (int j = lo + tid; j < tail_end; j += kPT)
            a.coords[base + j] = static_cast<int16_t>(static_cast<int32_t>(
                                     static_cast<uint32_t>(sh16[2 * (kOff + j) + 1]) << 19) >> 19);
    }

    // ---- running counts of the blocks before this one (roads and events share a word: both
    // stay below 2^31) --------------------------------------------------------------------------
    uint64_t p0, p1;
    look_back_grouped<kPB>(lc, b, agg0, agg1, s_look, p0, p1);
    const int64_t R0 = static_cast<int64_t>(p0 & 0x7FFFFFFFull);
    const int64_t E0 = static_cast<int64_t>(p0 >> 31);

    // ---- road table, combo_begin and event index (one scan over the road list), tiles, best
    // keys ---------------------------------------------------------------------------------------
    {
        constexpr int kEvShift = 48;  // a block's combinations stay far below 2^48
        int64_t carry = static_cast<int64_t>(p1);
        int64_t ecarry = E0 - 1;  // the event of the block's first word, before its own starts
        const int64_t T = a.tile_combos;
        uint64_t *keys = reinterpret_cast<uint64_t *>(a.best.chi2);
        for (int q0 = 0; q0 < nroads; q0 += kPT) {
            const int rl = q0 + tid;
            const bool mine = rl < nroads;
            const uint32_t info = mine ? s_info[rl] : kInfoOver;
            const uint32_t rd = mine ? s_road[rl] : 0u;
            const int64_t evs = (rd >> 12) & 1u;
            const int64_t c = (info & kInfoOver) ? 0 : combos_of(info);
            int64_t tot;
            const int64_t sc = block_excl_scan<int64_t, kPT>(c | (evs << kEvShift), tmp, tot);
            const int64_t cb = carry + (sc & ((1ll << kEvShift) - 1));
            const int64_t ev = ecarry + (sc >> kEvShift) + evs;
            carry += tot & ((1ll << kEvShift) - 1);
            ecarry += tot >> kEvShift;
            if (!mine) continue;
            const int64_t r = R0 + rl;
            if (info & kInfoOver) report(a.err, SVT_ERRCLASS_HITS, static_cast<uint64_t>(r));
            if (info & kInfoSet) report(a.err, SVT_ERRCLASS_SET, static_cast<uint64_t>(r));
            if (r >= a.road_cap) continue;
            a.roads.event[r] = static_cast<int32_t>(ev);
            if (a.event_first_road && evs && ev < a.event_cap)
                a.event_first_road[ev] = static_cast<int32_t>(r);
            a.roads.set[r] = static_cast<int32_t>((info >> 20) & 0xFFu);
            a.roads.hit_begin[r] = base + (rd & 0xFFF);
            a.roads.nhits[r] = info & 0xFFFFFu;
            a.roads.ncombo[r] = static_cast<int32_t>(c);
            a.roads.combo_begin[r] = cb;
            keys[r] = UINT64_MAX;
            a.best.n_accept[r] = 0;
            if (T > 0 && c > 0) {
                for (int64_t t = (cb + T - 1) / T; t * T < cb + c; ++t)
                    if (t < a.tiles_cap) a.tile_first_road[t] = static_cast<int32_t>(r);
            }
        }
    }

    if (b == nb - 1 && tid == 0) {
        const int64_t n_roads = R0 + tr;
        const int64_t n_combos = static_cast<int64_t>(p1) + tc;
        *a.d_n_roads = n_roads;
        *a.d_n_combos = n_combos;
        if (a.d_n_events) *a.d_n_events = E0 + te;
        if (n_roads > a.road_cap) report(a.err, SVT_ERRCLASS_CAPACITY, 0);
        if (n_combos > a.combo_cap) report(a.err, SVT_ERRCLASS_CAPACITY, 1);
    }
}

// Clears the error word, the work tickets (the fused kernel's tile counter is the first), the
// kept count, the look-back status words in use and, when given, zero[0 .. n_zero) (the kept
// list's per-block counts, which the fused kernel adds to); copies the word count into
// *nw_copy, where the pass's later kernels read it (the count may live in page-locked host
// memory, and one read of it beats one per wave across the bus).
__global__ void k_batch_reset(uint64_t *err, uint32_t *tickets, int64_t *d_n_kept,
                              int64_t *status, int64_t n_status, Sizes nw, int64_t *nw_copy,
                              int64_t *zero, int64_t n_zero) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *err = SVT_NO_ERROR;
        tickets[0] = 0;
        tickets[1] = 0;
        if (d_n_kept) *d_n_kept = 0;
        *nw_copy = nw.dev ? *nw.dev : nw.host;  // the one read of a (possibly host-side) count
    }
    for (int64_t i = gtid(); i < n_status; i += gstride()) status[i] = 0;
    if (zero)
        for (int64_t i = gtid(); i < n_zero; i += gstride()) zero[i] = 0;
}

}  // namespace

hipError_t launch_prepass(const PrepassLaunch &p, hipStream_t s) {
    PArgs a;
    a.words = p.words;
    a.nw = p.nw;
    a.cfg = p.cfg;
    a.roads = p.roads;
    a.road_cap = p.road_cap;
    a.coords = p.coords;
    a.best = p.best;
    a.tile_combos = p.tile_combos;
    a.tile_first_road = p.tile_first_road;
    a.tiles_cap = p.tiles_cap;
    a.combo_cap = p.combo_cap;
    a.d_n_roads = p.d_n_roads;
    a.d_n_combos = p.d_n_combos;
    a.status = p.status;
    a.nb_cap = p.nb_cap;
    a.lookback_timeout = kLookbackTimeout;
    if (const char *e = std::getenv("SVT_LOOKBACK_TIMEOUT_TICKS"))  // test hook: 0 forces the
        a.lookback_timeout = std::strtoull(e, nullptr, 10);        // computed aggregates
    a.err = p.err;
    a.event_first_road = p.event_first_road;
    a.event_cap = p.event_cap;
    a.d_n_events = p.d_n_events;
    const int64_t grid = p.nb_cap > 0 ? p.nb_cap : 1;
    hipLaunchKernelGGL(k_prepass, dim3(static_cast<unsigned>(grid)), dim3(kPT), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_reset(const PrepassLaunch &p, int64_t *nw_copy, int64_t *d_n_kept,
                              int64_t *zero, int64_t n_zero, hipStream_t s) {
    const int64_t items = zero && n_zero > p.status_words ? n_zero : p.status_words;
    int64_t blocks = (items + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_batch_reset, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                       p.err, p.tickets, d_n_kept, p.status, p.status_words, p.nw, nw_copy, zero,
                       zero ? n_zero : 0);
    return hipGetLastError();
}

}  // namespace svt
