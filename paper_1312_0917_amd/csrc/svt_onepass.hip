// One-pass batched kernel: unpack, combine, fit and select in a single persistent launch.
//
// Section II-A of the paper runs its three functions -- unpack the input and fill the data
// structures, compute all combinations of hits of each road, fit each combination -- as one loop
// nest over events, roads and combinations.  This kernel keeps that shape per unit of work: a
// workgroup takes a unit of 1024 consecutive hit words and, in its own LDS,
//   1. stages the words (plus 64 words past the unit, enough for any road that starts in it,
//      and the word before it), flags road and event starts, lists the roads that start among
//      its words and counts their hits per layer and combinations;
//   2. publishes those counts for the units after it, groups each road's coordinates by layer,
//      and takes its own running offsets (first road, event and combination) from one
//      decoupled look-back over the units before it (svt_lookback.h);
//   3. writes the road table of its roads;
//   4. fits every combination of its roads in chunks: per chunk, the coordinate-pair tables of
//      the chunk's roads are built in LDS and every lane fits four consecutive combinations with
//      packed 16-bit dot products (svt_fit.h), writing the records with 16-byte stores;
//   5. keeps each road's accepted count and best key in LDS (a road is owned by one unit), so
//      the best tracks are written straight from the unit -- no global atomics and no second
//      pass over the roads.
// The words are read from HBM once and the grouped coordinates and road table never go back
// to HBM to be read again; the only other launch of a pass is the reset of the look-back state.
//
// Units: workgroup w takes unit w first, then units gridDim.x + t from a ticket counter,
// fetched while it finishes the previous unit (a ticket taken earlier reserves a unit that later
// units' look-backs then wait on until it starts).  Units taken from tickets run in ticket order,
// so a unit only waits on units already taken; the first units are numbered by the grid, and a
// look-back that has waited too long on one of them computes that unit's counts itself.
//
// The constant bank (at most 256 sets) is staged into LDS once per workgroup, packed for the
// dot products; a 112-byte stride puts the sets one wave reads in different LDS banks.
#include <cstdlib>
#include <type_traits>

#include "svt_fit.h"
#include "svt_lookback.h"

namespace svt {
namespace {

constexpr int kOT = 256;                      // threads per workgroup
constexpr int kUW = kOnepassUnitWords;        // 1024 words per unit
constexpr int kUPW = kUW / kOT;               // 4 words staged per thread
constexpr int kUT = kRoadTail;                // words staged past the unit
constexpr int kUOff = 4;                      // sw[kUOff - 1] = word before the unit
constexpr int kFitCap = 224;                  // roads with combinations starting in a unit:
                                              // each has >= 5 words, (kUW + 40) / 5 < 224
constexpr int kXTCap = 2048;                  // coordinate-pair table entries per chunk
constexpr int kGrpCap = 2048;                 // groups of 4 combinations per chunk
constexpr int kMaxLayerHits = SVT_MAX_HITS;
constexpr int32_t kListedMaxMean = 48;        // mean combinations per road below which the
                                              // groups spanning a road boundary are listed
constexpr uint32_t kInfoOver = 1u << 20;      // too many hits on a layer, or too long a road
constexpr uint32_t kInfoSet = 1u << 21;       // road tag without a constant set
static_assert(kUPW == 4, "one 16-byte load of words per thread");

struct OArgs {
    const svt_fconst *bank;
    svt_config cfg;
    const uint32_t *words;
    Sizes nw;
    svt_roads roads;
    int64_t road_cap;
    svt_fitrec rec;
    uint8_t *accept;
    svt_best best;
    int64_t combo_cap;
    int64_t *d_n_roads;
    int64_t *d_n_combos;
    unsigned long long *kb_counts;  // accepted count per kKeptBlock combinations (nullable)
    int64_t *status;                // look-back status words, 2 * nb_cap
    int64_t nb_cap;
    uint32_t *tickets;              // [1]: units past the grid
    uint64_t lookback_timeout;
    uint64_t *err;
    int16_t *coords;                // kept-only mode: grouped coordinates for the refit pass
    int32_t *tile_first_road;       // kept-only mode: first road of every kKeptBlock block
    int64_t tiles_cap;
};

// A constant set packed for the dot products, with the offset's low part folded into the
// layer-4 pair (shift <= 15): (f_j4, ql_j) . (x4, 1).
struct alignas(16) BankSetF {
    int32_t F01[6];
    int32_t F23[6];
    int32_t F4[6];
    int32_t qh[6];
    int32_t pad[4];
};
static_assert(sizeof(BankSetF) == 112, "LDS bank spread of the staged constant sets");

template <bool FOLD>
using BankT = typename std::conditional<FOLD, BankSetF, RoadConst>::type;

template <bool FOLD>
struct OLds {
    BankT<FOLD> bank[256];
    alignas(16) int16_t sc[kUW + kUT + 16];  // grouped coordinates at the words' local positions
    // the unit's roads with combinations, in stream order
    uint16_t fr_hb[kFitCap];             // local index of the road's first word
    uint16_t fr_rl[kFitCap];             // index among the roads that start in the unit
    uint32_t fr_info[kFitCap];           // hits per layer (4 bits each) | constant set << 20
    int32_t fr_cb[kFitCap];              // first combination, from the unit's first
    unsigned long long fr_key[kFitCap];  // best key (chi2 << 15 | k) of the accepted ones
    uint32_t fr_nacc[kFitCap];
    union {
        struct {  // unpacking
            uint32_t sw[kUOff + kUW + kUT];  // word base + j at sw[kUOff + j]
            uint32_t road[kUW + 1];          // first local word (12 bits) | events started in
                                             // the unit up to it (12 bits) << 12 | event start
                                             // << 24; [n_owned] = end of the last road
            uint32_t info[kUW];              // hits per layer | kInfoOver | kInfoSet
        } u;
        struct {  // fitting one chunk
            int32_t XT[kXTCap];              // coordinate-pair tables of the chunk's roads
            RoadMeta meta[kFitCap];
            uint32_t crs[kFitCap];           // road begin (24 bits, unit coordinates) | set << 24
            uint8_t M[kGrpCap];              // group of 4 -> chunk road of its first combination
            uint16_t X[kFitCap];             // groups spanning a road boundary (from g_lo)
        } f;
    };
    int64_t tmp[kOT / kWaveSize + 1];
    int64_t pre[3];
    int32_t tail_end;
    int32_t next_unit;
    int32_t c_fa, c_nr, c_cs, c_ce, c_g_lo, c_g_hi, c_nx;
    int32_t work[2];
};

template <bool FOLD>
__device__ __forceinline__ void pack_set(const svt_fconst &F, BankT<FOLD> &B, int32_t shift,
                                         uint32_t qlmask) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        const int32_t q = F.q[j];
        const int32_t ql = static_cast<int32_t>(static_cast<uint32_t>(q) & qlmask);
        B.F01[j] = pack16(F.f[j][0], F.f[j][1]);
        B.F23[j] = pack16(F.f[j][2], F.f[j][3]);
        B.F4[j] = pack16(F.f[j][4], FOLD ? ql : 0);
        B.qh[j] = q >> shift;
        if constexpr (!FOLD) B.ql[j] = ql;
    }
}

// Fit combination k of a road from the grouped coordinates and the road's packed constant set in
// LDS, with the records' own arithmetic (so the values equal the records bit for bit).
template <bool FOLD>
__device__ __forceinline__ Fit refit_packed(const BankT<FOLD> &c, const int16_t *sc, uint32_t nh,
                                            int32_t hb, uint32_t k, int32_t shift) {
    uint32_t h[SVT_N_LAYERS];
#pragma unroll
    for (int l = SVT_N_LAYERS - 1; l >= 0; --l) {  // layer 0 most significant
        const uint32_t nl = nh_of(nh, l);
        h[l] = k % nl;
        k /= nl;
    }
    int32_t off = hb;
    int32_t x[SVT_N_LAYERS];
#pragma unroll
    for (int l = 0; l < SVT_N_LAYERS; ++l) {
        x[l] = sc[off + static_cast<int32_t>(h[l])];
        off += static_cast<int32_t>(nh_of(nh, l));
    }
    return fit_xyz<FOLD>(c, pack16(x[0], x[1]), pack16(x[2], x[3]), pack16(x[4], 1), shift);
}

// ---- one chunk of the unit's combinations ---------------------------------------------------
// Coordinates "local" below count combinations from GB = the unit's first combination rounded
// down to a multiple of 4, so that groups of 4 are aligned with the records' 16-byte stores.

// Wave 0: choose the chunk that starts at group g0 -- the fit roads from the first one still
// unfinished at the chunk's start, as many as the pair-table capacity and the group capacity
// allow -- and write its per-road indexing data, road begins and listed groups.
template <bool FOLD>
__device__ void chunk_params(OLds<FOLD> &S, int32_t &fa, int32_t g0, int32_t g_end, int32_t o,
                             int32_t TC, int32_t nfit) {
    const int lane = lane_id();
    const int32_t cs = 4 * g0 > o ? 4 * g0 : o;
    // roads that end at or before the chunk's first combination are done
    while (fa < nfit) {
        const int32_t r = fa + lane;
        bool done = false;
        if (r < nfit) {
            const uint32_t info = S.fr_info[r];
            done = o + S.fr_cb[r] + static_cast<int32_t>(combos_of(info)) <= cs;
        }
        const uint64_t m = __ballot(done);
        const int cnt = __popcll(m);  // a prefix of the lanes
        fa += cnt;
        if (cnt < kWaveSize) break;
    }
    const int32_t gcap_end = 4 * (g0 + kGrpCap);
    int32_t nr = 0, xt = 0;
    bool stopped = false;
    for (int32_t b0 = fa; !stopped && b0 < nfit; b0 += kWaveSize) {
        const int32_t r = b0 + lane;
        const bool valid = r < nfit;
        uint32_t info = 0;
        int32_t rb = 0;
        if (valid) {
            info = S.fr_info[r];
            rb = o + S.fr_cb[r];
        }
        const int32_t n0 = nh_of(info, 0), n1 = nh_of(info, 1), n2 = nh_of(info, 2),
                      n3 = nh_of(info, 3), n4 = nh_of(info, 4);
        const int32_t ntab = valid ? n0 * n1 + n2 * n3 + n4 : 0;
        const int32_t tend = xt + wave_incl_scan(ntab);
        const bool inc = valid && rb < gcap_end && tend <= kXTCap && r - fa < kFitCap;
        const uint64_t m = __ballot(inc);  // a prefix of the lanes
        const int cnt = __popcll(m);
        if (inc) {
            const int32_t ri = r - fa;
            const int32_t to = tend - ntab;
            const uint32_t n23 = static_cast<uint32_t>(n2 * n3);
            const int32_t C = n0 * n1 * n2 * n3 * n4;
            RoadMeta mm;
            mm.w4 = magic_of(n4 > 0 ? n4 : 1) | (static_cast<uint32_t>(n4) << 24);
            mm.w23 = magic_of(n23 > 0 ? n23 : 1) | (n23 << 24);
            mm.b0123 = static_cast<uint32_t>(to) | (static_cast<uint32_t>(to + n0 * n1) << 16);
            mm.b4c = static_cast<uint32_t>(to + n0 * n1 + n2 * n3) |
                     (static_cast<uint32_t>(C) << 16);
            S.f.meta[ri] = mm;
            S.f.crs[ri] = static_cast<uint32_t>(rb) | ((info >> 20) << 24);
        }
        nr += cnt;
        xt = __shfl(tend, kWaveSize - 1);
        stopped = cnt < kWaveSize;
    }
    // the chunk ends at the group cap, at the batch's end, or where the first road left out
    // starts (the groups before it are complete without it)
    int32_t g_hi = g0 + kGrpCap;
    const int32_t g_last = g_end;
    if (g_hi > g_last) g_hi = g_last;
    if (fa + nr < nfit) {
        const int32_t next_start = (o + S.fr_cb[fa + nr]) >> 2;
        if (next_start < g_hi) g_hi = next_start;
    }
    const int32_t ce = 4 * g_hi < o + TC ? 4 * g_hi : o + TC;
    __builtin_amdgcn_wave_barrier();  // crs written by this wave above
    // groups that span a road boundary: a road starts inside the group (not at a multiple of
    // 4) after the chunk's first combination and before its end; one entry per group
    int32_t nx = 0;
    int32_t prev_g = -1;  // group of the last cut road of the previous 64 (carried)
    for (int32_t b0 = 0; b0 < nr; b0 += kWaveSize) {
        const int32_t ri = b0 + lane;
        int32_t rb = 0;
        if (ri < nr) rb = static_cast<int32_t>(S.f.crs[ri] & 0xFFFFFFu);
        const int32_t g = rb >> 2;
        const bool cut = ri < nr && (rb & 3) != 0 && rb > cs && rb < ce;
        int32_t pg = __shfl_up(cut ? g : -1, 1);
        if (lane == 0) pg = prev_g;
        const bool head = cut && pg != g;
        const uint64_t hm = __ballot(head);
        if (head) S.f.X[nx + __popcll(hm & ((1ull << lane) - 1))] = static_cast<uint16_t>(g - g0);
        nx += __popcll(hm);
        // the last lane's cut group carries into the next 64 roads
        const uint64_t cm = __ballot(cut);
        const int32_t last = cm ? 63 - __builtin_clzll(cm) : -1;
        const int32_t lg = __shfl(g, last < 0 ? 0 : last);
        // a cut in lane 63 is what the next batch's lane 0 compares with
        prev_g = (last == kWaveSize - 1) ? lg : -1;
    }
    if (lane == 0) {
        S.c_fa = fa;
        S.c_nr = nr;
        S.c_cs = cs;
        S.c_ce = ce;
        S.c_g_lo = g0;
        S.c_g_hi = g_hi;
        S.c_nx = nx;
        S.work[0] = 0;
        S.work[1] = 0;
    }
}

// All threads: the pair tables and the group -> road map of the chunk, one road per thread.
template <bool FOLD>
__device__ __forceinline__ void chunk_tables(OLds<FOLD> &S) {
    const int32_t nr = S.c_nr, fa = S.c_fa, cs = S.c_cs, g_lo = S.c_g_lo, g_hi = S.c_g_hi;
    for (int32_t ri = threadIdx.x; ri < nr; ri += kOT) {
        const uint32_t info = S.fr_info[fa + ri];
        const int32_t g0w = S.fr_hb[fa + ri];
        const int32_t n0 = nh_of(info, 0), n1 = nh_of(info, 1), n2 = nh_of(info, 2),
                      n3 = nh_of(info, 3), n4 = nh_of(info, 4);
        const RoadMeta m = S.f.meta[ri];
        const int32_t off1 = g0w + n0, off2 = off1 + n1, off3 = off2 + n2, off4 = off3 + n3;
        const int32_t b01 = m.b01(), b23 = m.b23(), b4 = m.b4();
        // the hits of layers 1, 3 and 4 in registers first (at most kMaxLayerHits each; reads
        // past a layer stay inside sc's slack)
        int32_t y1[kMaxLayerHits], y3[kMaxLayerHits], y4[kMaxLayerHits];
#pragma unroll
        for (int i = 0; i < kMaxLayerHits; ++i) {
            y1[i] = S.sc[off1 + i];
            y3[i] = S.sc[off3 + i];
            y4[i] = S.sc[off4 + i];
        }
        int32_t t = b01;
        for (int32_t h0 = 0; h0 < n0; ++h0, t += n1) {
            const int32_t x0 = S.sc[g0w + h0];
#pragma unroll
            for (int h1 = 0; h1 < kMaxLayerHits; ++h1)
                if (h1 < n1) S.f.XT[t + h1] = pack16(x0, y1[h1]);
        }
        t = b23;
        for (int32_t h2 = 0; h2 < n2; ++h2, t += n3) {
            const int32_t x2 = S.sc[off2 + h2];
#pragma unroll
            for (int h3 = 0; h3 < kMaxLayerHits; ++h3)
                if (h3 < n3) S.f.XT[t + h3] = pack16(x2, y3[h3]);
        }
#pragma unroll
        for (int h4 = 0; h4 < kMaxLayerHits; ++h4)
            if (h4 < n4) S.f.XT[b4 + h4] = pack16(y4[h4], 1);
        // groups whose first combination inside [cs, ce) belongs to this road
        const int32_t rb = static_cast<int32_t>(S.f.crs[ri] & 0xFFFFFFu);
        const int32_t glo = rb <= cs ? g_lo : (rb + 3) >> 2;
        int32_t ghi = g_hi;
        if (ri + 1 < nr) {
            const int32_t nrb = static_cast<int32_t>(S.f.crs[ri + 1] & 0xFFFFFFu);
            ghi = nrb <= cs ? g_lo : (nrb + 3) >> 2;
        }
        if (ghi > g_hi) ghi = g_hi;
        for (int32_t g = glo; g < ghi; ++g) S.f.M[g - g_lo] = static_cast<uint8_t>(ri);
    }
}

__device__ __forceinline__ int32_t claim64(int32_t *counter) {
    int32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, kWaveSize);
    return __shfl(base, 0);
}

// Accepted combinations of one road in one group: the unit's per-road count and best key (LDS
// atomics), and the kept list's block count (global, only when a kept list is wanted).
template <bool FOLD>
__device__ __forceinline__ void note_accepts(const OArgs &a, OLds<FOLD> &S, int32_t fi,
                                             int64_t gi, uint32_t acc_bits,
                                             unsigned long long kmin) {
    if (a.kb_counts)
        atomicAdd(a.kb_counts + gi / kKeptBlock,
                  static_cast<unsigned long long>(__popc(acc_bits)));
    atomicMin(&S.fr_key[fi], kmin);
    atomicAdd(&S.fr_nacc[fi], static_cast<uint32_t>(__popc(acc_bits)));
}

// A group whose valid slots all lie in chunk road ri: four fits with one set of constants.
template <bool FOLD, int REC>
__device__ __forceinline__ void fit_group(const OArgs &a, OLds<FOLD> &S, int ri, int32_t rel0,
                                          uint32_t slots, int64_t GB, int32_t shift) {
    const RoadMeta m = S.f.meta[ri];
    const uint32_t rs = S.f.crs[ri];
    const int32_t rbase = static_cast<int32_t>(rs & 0xFFFFFFu);
    const BankT<FOLD> &c = S.bank[rs >> 24];
    int32_t vp0[4], vp1[4], vp2[4], vc0[4], vc1[4], vc2[4];
    int64_t vchi[4];
    Fit f4r[4];
    fit4<FOLD>(m, c, rel0 - rbase, S.f.XT, shift, f4r);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const Fit &f = f4r[e];
        vp0[e] = f.v[0]; vp1[e] = f.v[1]; vp2[e] = f.v[2];
        vc0[e] = f.v[3]; vc1[e] = f.v[4]; vc2[e] = f.v[5];
        vchi[e] = f.chi2;
    }
    uint32_t acc_bits = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        acc_bits |= ((slots >> e) & 1u) && vchi[e] <= a.cfg.chi2_cut ? (1u << e) : 0u;
    const int64_t gi = GB + rel0;
    if (acc_bits) {  // rare
        unsigned long long kmin = ~0ull;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if ((acc_bits >> e) & 1u) {
                const unsigned long long kv =
                    best_key(vchi[e], static_cast<uint32_t>(rel0 + e - rbase));
                kmin = kv < kmin ? kv : kmin;
            }
        note_accepts(a, S, S.c_fa + ri, gi, acc_bits, kmin);
    }
    store_group<REC>(a.rec, a.accept, gi, slots, acc_bits, vp0, vp1, vp2, vc0, vc1, vc2, vchi);
}

// One combination ci (local) of a group that spans a road boundary, fitted with its own road's
// constants (the group's first road is ri; later roads follow in order) and written on its own.
template <bool FOLD, int REC>
__device__ __forceinline__ void fit_slot(const OArgs &a, OLds<FOLD> &S, int ri, int32_t ci,
                                         int64_t GB, int32_t shift) {
    const int nr = S.c_nr;
    while (ri + 1 < nr &&
           ci >= static_cast<int32_t>(S.f.crs[ri] & 0xFFFFFFu) + S.f.meta[ri].C())
        ++ri;
    const uint32_t rs = S.f.crs[ri];
    const int32_t k = ci - static_cast<int32_t>(rs & 0xFFFFFFu);
    const Fit f = fit_combo<FOLD>(S.f.meta[ri], S.bank[rs >> 24], static_cast<uint32_t>(k),
                                  S.f.XT, shift);
    const bool acc = f.chi2 <= a.cfg.chi2_cut;
    const int64_t gi = GB + ci;
    if (REC != kRecNone) {
        a.rec.p0[gi] = f.v[0];
        a.rec.p1[gi] = f.v[1];
        a.rec.p2[gi] = f.v[2];
        a.rec.chi2[gi] = f.chi2;
    }
    if (REC == kRecRows) {
        if (a.rec.c0) a.rec.c0[gi] = f.v[3];
        if (a.rec.c1) a.rec.c1[gi] = f.v[4];
        if (a.rec.c2) a.rec.c2[gi] = f.v[5];
    }
    a.accept[gi] = acc ? 1 : 0;
    if (acc)
        note_accepts(a, S, S.c_fa + ri, gi, 1u,
                     static_cast<unsigned long long>(best_key(f.chi2, static_cast<uint32_t>(k))));
}

// Small roads: the listed groups first, one combination per lane, then every other group of
// the chunk on the uniform one-road path (see the fused kernel for why in this order).
template <bool FOLD, int REC>
__device__ void consume_listed(const OArgs &a, OLds<FOLD> &S, int64_t GB, int32_t shift) {
    const int32_t cs = S.c_cs, ce = S.c_ce, g_lo = S.c_g_lo, g_hi = S.c_g_hi, nx = S.c_nx;
    const int32_t ng = g_hi - g_lo;
    const int lane = lane_id();
    while (true) {
        const int32_t base = claim64(&S.work[1]);
        if (base >= 4 * nx) break;
        const int32_t j = base + lane;
        if (j < 4 * nx) {
            const int32_t off = S.f.X[j >> 2];
            const int32_t ci = ((g_lo + off) << 2) + (j & 3);
            if (ci >= cs && ci < ce) fit_slot<FOLD, REC>(a, S, S.f.M[off], ci, GB, shift);
        }
    }
    while (true) {
        const int32_t base = claim64(&S.work[0]);
        if (base >= ng) break;
        const int32_t it = base + lane;
        if (it < ng) {
            const int32_t rel0 = (g_lo + it) << 2;
            const int ri = S.f.M[it];
            const int32_t end = static_cast<int32_t>(S.f.crs[ri] & 0xFFFFFFu) + S.f.meta[ri].C();
            uint32_t valid = 0, in_ri = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                valid |= (rel0 + e >= cs && rel0 + e < ce) ? (1u << e) : 0u;
                in_ri |= (rel0 + e < end) ? (1u << e) : 0u;
            }
            // a group spanning a road boundary is a listed group, fitted above
            if (!(valid & ~in_ri)) fit_group<FOLD, REC>(a, S, ri, rel0, valid, GB, shift);
        }
    }
}

// Large roads: each lane fits its group of 4 itself, a group that spans a road boundary slot
// by slot.
template <bool FOLD, int REC>
__device__ void consume_inline(const OArgs &a, OLds<FOLD> &S, int64_t GB, int32_t shift) {
    const int nr = S.c_nr;
    const int32_t cs = S.c_cs, ce = S.c_ce, g_lo = S.c_g_lo, g_hi = S.c_g_hi, fa = S.c_fa;
    const int32_t ng = g_hi - g_lo;
    while (true) {
        const int32_t base = claim64(&S.work[0]);
        if (base >= ng) break;
        if (base + lane_id() >= ng) continue;
        const int32_t it = base + lane_id();
        const int32_t rel0 = (g_lo + it) << 2;
        const int32_t first = rel0 > cs ? rel0 : cs;
        const int32_t last = (rel0 + 3 < ce - 1) ? rel0 + 3 : ce - 1;
        int ri = S.f.M[it];
        RoadMeta m = S.f.meta[ri];
        uint32_t rs = S.f.crs[ri];
        const int32_t rbase = static_cast<int32_t>(rs & 0xFFFFFFu);
        uint32_t valid_bits = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            valid_bits |= (rel0 + e >= cs && rel0 + e < ce) ? (1u << e) : 0u;
        if (last - rbase < m.C()) {
            fit_group<FOLD, REC>(a, S, ri, rel0, valid_bits, GB, shift);
            continue;
        }
        int32_t vp0[4], vp1[4], vp2[4], vc0[4], vc1[4], vc2[4];
        int64_t vchi[4];
        int32_t kk[4];
        int rr4[4];
        int32_t k = first - rbase;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            vp0[e] = vp1[e] = vp2[e] = vc0[e] = vc1[e] = vc2[e] = 0;
            vchi[e] = 0;
            kk[e] = 0;
            rr4[e] = ri;
            if ((valid_bits >> e) & 1u) {
                while (k >= m.C() && ri + 1 < nr) {  // bounded by the chunk
                    k -= m.C();
                    ++ri;
                    m = S.f.meta[ri];
                    rs = S.f.crs[ri];
                }
                const Fit f = fit_combo<FOLD>(m, S.bank[rs >> 24], static_cast<uint32_t>(k),
                                              S.f.XT, shift);
                vp0[e] = f.v[0]; vp1[e] = f.v[1]; vp2[e] = f.v[2];
                vc0[e] = f.v[3]; vc1[e] = f.v[4]; vc2[e] = f.v[5];
                vchi[e] = f.chi2;
                kk[e] = k;
                rr4[e] = ri;
                ++k;
            }
        }
        uint32_t acc_bits = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            acc_bits |= ((valid_bits >> e) & 1u) && vchi[e] <= a.cfg.chi2_cut ? (1u << e) : 0u;
        const int64_t gi = GB + rel0;
        if (acc_bits) {
#pragma unroll
            for (int e = 0; e < 4; ++e)
                if ((acc_bits >> e) & 1u)
                    note_accepts(a, S, fa + rr4[e], gi, 1u,
                                 static_cast<unsigned long long>(
                                     best_key(vchi[e], static_cast<uint32_t>(kk[e]))));
        }
        store_group<REC>(a.rec, a.accept, gi, valid_bits, acc_bits, vp0, vp1, vp2, vc0, vc1,
                         vc2, vchi);
    }
}

template <bool FOLD, int REC>
__global__ __launch_bounds__(kOT) __attribute__((amdgpu_waves_per_eu(FOLD ? 3 : 2))) void k_onepass(
    OArgs a) {
    __shared__ OLds<FOLD> S;
    const int tid = threadIdx.x;
    const int wave = tid / kWaveSize;
    const int64_t n = load_size(a.nw);
    const int64_t nb = (n + kUW - 1) / kUW;
    if (blockIdx.x == 0 && tid == 0 && a.nw.dev && *a.nw.dev > a.nw.cap)
        report(a.err, SVT_ERRCLASS_CAPACITY, 3);
    if (nb == 0) {
        if (blockIdx.x == 0 && tid == 0) {  // empty batch
            *a.d_n_roads = 0;
            *a.d_n_combos = 0;
        }
        return;
    }
    if (static_cast<int64_t>(blockIdx.x) >= nb) return;
    const LookbackCtx lc{a.words, n, a.cfg.n_layers, a.cfg.max_hits, a.status, a.nb_cap,
                         a.lookback_timeout};
    const int32_t shift = a.cfg.shift;
    const uint32_t qlmask = (1u << shift) - 1u;
    const int32_t n_sets = a.cfg.n_sets;
    for (int s = tid; s < n_sets; s += kOT) pack_set<FOLD>(a.bank[s], S.bank[s], shift, qlmask);
    const bool aligned16 = (reinterpret_cast<uintptr_t>(a.words) & 15) == 0;
    const int max_len = a.cfg.n_layers * a.cfg.max_hits;

    int64_t u = blockIdx.x;
    while (u < nb) {
        // ---- stage the unit's words, 64 more, and the word before ---------------------------
        const int64_t base = u * kUW;
        const int nloc = static_cast<int>(n - base < kUW + kUT ? n - base : kUW + kUT);
        const int nown = nloc < kUW ? nloc : kUW;
        const int j0 = tid * kUPW;
        uint32_t wv[kUPW];
        if (aligned16 && j0 + kUPW <= nown) {
            const uint4 v = *reinterpret_cast<const uint4 *>(a.words + base + j0);
            *reinterpret_cast<uint4 *>(S.u.sw + kUOff + j0) = v;
            wv[0] = v.x;
            wv[1] = v.y;
            wv[2] = v.z;
            wv[3] = v.w;
        } else {
#pragma unroll
            for (int e = 0; e < kUPW; ++e) {
                wv[e] = (j0 + e < nloc) ? a.words[base + j0 + e] : 0u;
                S.u.sw[kUOff + j0 + e] = wv[e];
            }
        }
        if (tid < kUT) S.u.sw[kUOff + kUW + tid] = (kUW + tid < nloc) ? a.words[base + kUW + tid] : 0u;
        if (tid == 0) S.u.sw[kUOff - 1] = base > 0 ? a.words[base - 1] : 0u;
        __syncthreads();

        // ---- road and event starts of this thread's words ----------------------------------
        uint32_t rmask = 0, emask = 0;
        int nr = 0, ne = 0;
        int64_t bad = -1;
#pragma unroll
        for (int e = 0; e < kUPW; ++e) {
            const int j = j0 + e;
            if (j < nown) {
                const uint32_t x = wv[e];
                const uint32_t px = e == 0 ? S.u.sw[kUOff + j - 1] : wv[e - 1];
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
            // unit, else the end of the staged words
            const int j = kUW + tid;
            const bool start = j < nloc && w_tags(S.u.sw[kUOff + j]) != w_tags(S.u.sw[kUOff + j - 1]);
            const uint64_t m = __ballot(start);
            if (tid == 0) S.tail_end = nloc <= kUW ? nloc : (m ? kUW + __builtin_ctzll(m) : nloc);
        }
        int64_t tre;
        const int64_t rel0 = block_excl_scan<int64_t, kOT>(
            static_cast<int64_t>(nr) | (static_cast<int64_t>(ne) << 32), S.tmp, tre);
        const int rl0 = static_cast<int>(rel0 & 0xFFFFFFFF), el0 = static_cast<int>(rel0 >> 32);
        const int nroads = static_cast<int>(tre & 0xFFFFFFFF);
        const int64_t te = tre >> 32;
        {
            int rl = rl0;
            int ev = el0;
#pragma unroll
            for (int e = 0; e < kUPW; ++e) {
                ev += (emask >> e) & 1u;
                if ((rmask >> e) & 1u)
                    S.u.road[rl++] = static_cast<uint32_t>(j0 + e) |
                                     (static_cast<uint32_t>(ev) << 12) |
                                     (((emask >> e) & 1u) << 24);
            }
            if (tid == 0) S.u.road[nroads] = static_cast<uint32_t>(S.tail_end);
        }
        __syncthreads();

        // ---- one road per thread: hits per layer, checks, combinations ---------------------
        int64_t csum = 0;
        for (int rl = tid; rl < nroads; rl += kOT) {
            const int j = S.u.road[rl] & 0xFFF;
            const int len = static_cast<int>(S.u.road[rl + 1] & 0xFFF) - j;
            bool over = len > max_len;
            uint64_t cnt = 0;  // 8 bits per layer
            if (!over) {
                for (int i0 = 0; i0 < len; i0 += 8) {
                    uint32_t x[8];
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        x[q] = i0 + q < len ? S.u.sw[kUOff + j + i0 + q] : 0xE000u;
#pragma unroll
                    for (int q = 0; q < 8; ++q) {
                        const uint32_t l = w_layer(x[q]);  // 7 for the padding
                        if (l < SVT_N_LAYERS) cnt += 1ull << (8 * l);
                    }
                }
            }
            uint32_t packed = 0;
#pragma unroll
            for (int l = 0; l < SVT_N_LAYERS; ++l) {
                const uint32_t c = static_cast<uint32_t>((cnt >> (8 * l)) & 0xFF);
                over |= c > static_cast<uint32_t>(a.cfg.max_hits);
                packed |= (c & 0xFu) << (4 * l);
            }
            if (!over) csum += combos_of(packed);
            const bool noset = w_rtag(S.u.sw[kUOff + j]) >= static_cast<uint32_t>(n_sets);
            S.u.info[rl] = packed | (over ? kInfoOver : 0u) | (noset ? kInfoSet : 0u);
        }
        const int64_t tc = block_sum<int64_t, kOT>(csum, S.tmp);  // its barrier publishes info
        const uint64_t agg0 = static_cast<uint64_t>(nroads) | (static_cast<uint64_t>(te) << 31);
        const uint64_t agg1 = static_cast<uint64_t>(tc);
        if (tid == 0) publish_aggregate(lc, u, agg0, agg1);

        // ---- grouped coordinates of the roads with combinations (predecessors finish) ------
        for (int rl = tid; rl < nroads; rl += kOT) {
            const uint32_t info = S.u.info[rl];
            if (info & kInfoOver) continue;
            const int j = S.u.road[rl] & 0xFFF;
            const int len = static_cast<int>(S.u.road[rl + 1] & 0xFFF) - j;
            uint32_t off[SVT_N_LAYERS];
            uint32_t run = 0;
#pragma unroll
            for (int l = 0; l < SVT_N_LAYERS; ++l) {
                off[l] = run;
                run += nh_of(info, l);
            }
            for (int i0 = 0; i0 < len; i0 += 8) {
                uint32_t x[8];
#pragma unroll
                for (int q = 0; q < 8; ++q)
                    x[q] = i0 + q < len ? S.u.sw[kUOff + j + i0 + q] : 0xE000u;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const uint32_t l = w_layer(x[q]);
                    if (l >= SVT_N_LAYERS) continue;
                    uint32_t o = 0;
#pragma unroll
                    for (int k = 0; k < SVT_N_LAYERS; ++k)
                        if (static_cast<uint32_t>(k) == l) { o = off[k]; off[k] = o + 1; }
                    S.sc[j + o] = static_cast<int16_t>(w_coord(x[q]));
                }
            }
        }

        // ---- running counts of the units before this one ------------------------------------
        if (wave == 0) {
            uint64_t p0, p1;
            look_back2<kUW>(lc, u, agg0, agg1, p0, p1);
            if (tid == 0) {
                S.pre[0] = static_cast<int64_t>(p0 & 0x7FFFFFFFull);
                S.pre[1] = static_cast<int64_t>(p0 >> 31);
                S.pre[2] = static_cast<int64_t>(p1);
            }
        }
        __syncthreads();
        const int64_t R0 = S.pre[0], E0 = S.pre[1], CB0 = S.pre[2];

        // ---- road table, the list of roads with combinations, errors -----------------------
        int64_t carry_c = 0;
        int32_t carry_f = 0;
        for (int q0 = 0; q0 < nroads; q0 += kOT) {
            const int rl = q0 + tid;
            const bool mine = rl < nroads;
            const uint32_t info = mine ? S.u.info[rl] : kInfoOver;
            const int64_t c = (info & kInfoOver) ? 0 : combos_of(info);
            const bool fit = mine && c > 0;
            int64_t tot;
            const int64_t ex = block_excl_scan<int64_t, kOT>((c << 12) | (fit ? 1 : 0), S.tmp,
                                                             tot);
            const int64_t cb_loc = carry_c + (ex >> 12);
            const int32_t fi = carry_f + static_cast<int32_t>(ex & 0xFFF);
            carry_c += tot >> 12;
            carry_f += static_cast<int32_t>(tot & 0xFFF);
            if (!mine) continue;
            const int64_t r = R0 + rl;
            if (info & kInfoOver) report(a.err, SVT_ERRCLASS_HITS, static_cast<uint64_t>(r));
            if (info & kInfoSet) report(a.err, SVT_ERRCLASS_SET, static_cast<uint64_t>(r));
            const uint32_t rd = S.u.road[rl];
            const int j = rd & 0xFFF;
            const uint32_t tag = w_rtag(S.u.sw[kUOff + j]);
            if (fit && fi < kFitCap) {
                // a road without a constant set fits with set 0: its outputs are unspecified
                // (the error is reported), and no read leaves the bank
                const uint32_t set = tag < static_cast<uint32_t>(n_sets) ? tag : 0u;
                S.fr_hb[fi] = static_cast<uint16_t>(j);
                S.fr_rl[fi] = static_cast<uint16_t>(rl);
                S.fr_info[fi] = (info & 0xFFFFFu) | (set << 20);
                S.fr_cb[fi] = static_cast<int32_t>(cb_loc);
                S.fr_key[fi] = ~0ull;
                S.fr_nacc[fi] = 0;
            }
            if (r >= a.road_cap) continue;
            a.roads.event[r] = static_cast<int32_t>(E0 + ((rd >> 12) & 0xFFF) - 1);
            a.roads.set[r] = static_cast<int32_t>(tag);
            a.roads.hit_begin[r] = base + j;
            a.roads.nhits[r] = info & 0xFFFFFu;
            a.roads.ncombo[r] = static_cast<int32_t>(c);
            a.roads.combo_begin[r] = CB0 + cb_loc;
            if (!fit) {
                a.best.n_accept[r] = 0;
                a.best.k[r] = -1;
                a.best.p0[r] = INT32_MIN;
                a.best.p1[r] = INT32_MIN;
                a.best.p2[r] = INT32_MIN;
                a.best.chi2[r] = INT64_MAX;
            }
            if (a.tile_first_road && c > 0) {  // kept-only mode: first road of each block
                const int64_t cb = CB0 + cb_loc;
                for (int64_t t = (cb + kKeptBlock - 1) / kKeptBlock; t * kKeptBlock < cb + c; ++t)
                    if (t < a.tiles_cap) a.tile_first_road[t] = static_cast<int32_t>(r);
            }
        }
        const int32_t nfit = carry_f < kFitCap ? carry_f : kFitCap;
        const int64_t TC = carry_c;
        if (a.coords && nroads > 0) {  // kept-only mode: the refit pass reads these
            const int lo = S.u.road[0] & 0xFFF, hi = S.u.road[nroads] & 0xFFF;
            for (int j = lo + tid; j < hi; j += kOT) a.coords[base + j] = S.sc[j];
        }
        if (u == nb - 1 && tid == 0) {
            const int64_t n_roads = R0 + nroads;
            const int64_t n_combos = CB0 + TC;
            *a.d_n_roads = n_roads;
            *a.d_n_combos = n_combos;
            if (n_roads > a.road_cap) report(a.err, SVT_ERRCLASS_CAPACITY, 0);
            if (n_combos > a.combo_cap) report(a.err, SVT_ERRCLASS_CAPACITY, 1);
        }
        __syncthreads();  // the fit-road list is complete; the LDS union turns to the fit layout

        // ---- fit every combination of the unit, chunk by chunk -----------------------------
        // (a unit whose combinations do not fit the records' capacity writes none: the last
        // unit reports the capacity error)
        const bool can_fit = CB0 + TC <= a.combo_cap && carry_f <= kFitCap;
        if (can_fit && TC > 0) {
            const int64_t GB = CB0 & ~static_cast<int64_t>(3);
            const int32_t o = static_cast<int32_t>(CB0 - GB);
            const int32_t tc32 = static_cast<int32_t>(TC);
            const int32_t g_end = (o + tc32 + 3) >> 2;
            const bool listed = tc32 < kListedMaxMean * nfit;
            int32_t g0 = 0, fa = 0;
            while (g0 < g_end) {
                if (wave == 0) chunk_params(S, fa, g0, g_end, o, tc32, nfit);
                __syncthreads();
                chunk_tables(S);
                __syncthreads();
                if (listed)
                    consume_listed<FOLD, REC>(a, S, GB, shift);
                else
                    consume_inline<FOLD, REC>(a, S, GB, shift);
                g0 = S.c_g_hi;
                fa = S.c_fa;
                __syncthreads();
            }
        }

        // ---- best track of every road with combinations ------------------------------------
        if (tid == 0) S.next_unit = static_cast<int32_t>(gridDim.x) +
                                    static_cast<int32_t>(atomicAdd(a.tickets + 1, 1u));
        for (int fi = tid; fi < nfit; fi += kOT) {
            const int64_t r = R0 + S.fr_rl[fi];
            if (r >= a.road_cap) continue;
            const uint32_t info = S.fr_info[fi];
            const uint32_t nh = info & 0xFFFFFu;
            const BankT<FOLD> &F = S.bank[info >> 20];
            const int32_t hb = S.fr_hb[fi];
            unsigned long long key = can_fit ? S.fr_key[fi] : ~0ull;
            int32_t bk = -1;
            int64_t bchi = INT64_MAX;
            if (key != ~0ull && (key >> kKeyKBits) == kKeyChiMax) {
                // saturated key (chi2 >= 2^49 - 1, extreme constants only): exact rescan
                const int64_t C = combos_of(nh);
                for (int64_t k = 0; k < C; ++k) {
                    const int64_t c2 =
                        refit_packed<FOLD>(F, S.sc, nh, hb, static_cast<uint32_t>(k), shift).chi2;
                    if (c2 <= a.cfg.chi2_cut && c2 < bchi) {
                        bchi = c2;
                        bk = static_cast<int32_t>(k);
                    }
                }
            } else if (key != ~0ull) {
                bk = static_cast<int32_t>(key & ((1u << kKeyKBits) - 1));
                bchi = static_cast<int64_t>(key >> kKeyKBits);
            }
            a.best.n_accept[r] = can_fit ? static_cast<int32_t>(S.fr_nacc[fi]) : 0;
            a.best.k[r] = bk;
            a.best.chi2[r] = bchi;
            if (bk >= 0) {
                const Fit f = refit_packed<FOLD>(F, S.sc, nh, hb, static_cast<uint32_t>(bk), shift);
                a.best.p0[r] = f.v[0];
                a.best.p1[r] = f.v[1];
                a.best.p2[r] = f.v[2];
            } else {
                a.best.p0[r] = INT32_MIN;
                a.best.p1[r] = INT32_MIN;
                a.best.p2[r] = INT32_MIN;
            }
        }
        __syncthreads();  // next unit's ticket visible; LDS free for the next unit
        u = S.next_unit;
    }
}

template <bool FOLD>
hipError_t launch_fold(const OArgs &a, bool kept_only, bool rows, int grid, hipStream_t s) {
    if (kept_only)
        hipLaunchKernelGGL((k_onepass<FOLD, kRecNone>), dim3(grid), dim3(kOT), 0, s, a);
    else if (rows)
        hipLaunchKernelGGL((k_onepass<FOLD, kRecRows>), dim3(grid), dim3(kOT), 0, s, a);
    else
        hipLaunchKernelGGL((k_onepass<FOLD, kRecFit>), dim3(grid), dim3(kOT), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_onepass(const OnepassLaunch &p, hipStream_t s) {
    OArgs a;
    a.bank = p.bank;
    a.cfg = p.cfg;
    a.words = p.words;
    a.nw = p.nw;
    a.roads = p.roads;
    a.road_cap = p.road_cap;
    a.rec = p.kept_only ? svt_fitrec{} : p.rec;
    a.accept = p.accept;
    a.best = p.best;
    a.combo_cap = p.combo_cap;
    a.d_n_roads = p.d_n_roads;
    a.d_n_combos = p.d_n_combos;
    a.kb_counts = reinterpret_cast<unsigned long long *>(p.kb_counts);
    a.status = p.status;
    a.nb_cap = p.nb_cap;
    a.tickets = p.tickets;
    a.lookback_timeout = kLookbackTimeout;
    if (const char *e = std::getenv("SVT_LOOKBACK_TIMEOUT_TICKS"))  // test hook: 0 forces the
        a.lookback_timeout = std::strtoull(e, nullptr, 10);        // computed aggregates
    a.err = p.err;
    a.coords = p.kept_only ? p.coords : nullptr;
    a.tile_first_road = p.kept_only ? p.tile_first_road : nullptr;
    a.tiles_cap = p.tiles_cap;
    // a shift above 15 needs the larger constant layout: two workgroups fit a CU, not three,
    // and every workgroup of the persistent grid should be resident
    const bool fold = p.cfg.shift <= 15;
    const int per_cu = !fold && p.wgs_per_cu > 2 ? 2 : p.wgs_per_cu;
    int64_t grid = static_cast<int64_t>(p.num_cus) * per_cu;
    if (grid > p.nb_cap) grid = p.nb_cap;
    if (grid < 1) grid = 1;
    const bool rows = p.rec.c0 || p.rec.c1 || p.rec.c2;
    if (fold) return launch_fold<true>(a, p.kept_only, rows, static_cast<int>(grid), s);
    return launch_fold<false>(a, p.kept_only, rows, static_cast<int>(grid), s);
}

}  // namespace svt
