// Persistent fused combine + fit + select kernel of libsvt.
//
// The fit of section II is p_j = sum_l f[j][l] x_l + q_j followed by the fixed-point shift.
// Constants are int16 and coordinates int13, so the five products of one parameter are three
// packed 16-bit dot products (v_dot2_i32_i16) once the coordinates of layers (0,1) and (2,3)
// are paired: each road's hits are staged in LDS as small tables of coordinate pairs, and one
// combination is three LDS reads plus eighteen dot products.  The offset is split exactly as
// q = qh * 2^s + ql with 0 <= ql < 2^s: ql seeds the accumulator, so the sum stays inside
// int32, and
//     floor((S + q) / 2^s) = qh + floor((S + ql) / 2^s)       (exact for every integer S).
// A chunk whose every road's constant set has small enough bounds (narrow_ok) takes the narrow
// form instead: the whole offset seeds the accumulator and chi-square is summed in 32 bits.
//
// Work distribution: combinations are numbered globally (road-major, combo_begin from the
// pre-pass); each workgroup of a persistent grid walks tiles of tile_combos consecutive
// combinations taken from an atomic counter, and stages the roads of a tile in LDS in chunks
// of up to chunk_roads (16, 32 or 64) roads.  Wave 0 of the workgroup is a loader: while the other waves fit chunk i
// from one LDS buffer, it stages chunk i+1 in the other (road table, constants, one coalesced
// copy of the chunk's layer-grouped coordinates, pair tables, group-to-road map), so global
// latency hides behind arithmetic.  Compute lanes fit 4 consecutive combinations each and
// write every record array with 16-byte coalesced stores.  Per-road best tracks, accept
// counts and the kept-list block counts are reduced with global atomics from the (rare)
// accepted combinations, which needs no synchronisation between compute waves; a small pass
// after the kernel turns the per-road keys into best tracks.
#include <algorithm>

#include "svt_fit.h"

namespace svt {
namespace {

constexpr int kChunk = 64;             // roads staged per chunk at most: one loader lane each
constexpr int kWordCap = 2048;         // coordinates staged per chunk (a road has at most 40)
constexpr int kTabCap = 2048;          // coordinate-pair table entries per chunk (<= 136/road)
constexpr int kMapCap = kMaxTile / 4;  // groups of 4 combinations in a tile
constexpr int kMaxLayerHits = SVT_MAX_HITS;  // hits on one layer of a road with combinations
constexpr int kListedBit = 0x80;        // group map entry of a group listed in X (index below)
constexpr int64_t kStashMinMean = 48;   // mean combinations per road from which the listed
                                        // groups' records wait in LDS (consume_listed)

struct FArgs {
    const svt_fconst *bank;
    int32_t shift;
    int32_t n_sets;
    int64_t cut;
    const int16_t *coords;  // hit coordinates grouped by layer inside each road
    svt_roads roads;
    const int64_t *d_n_roads;
    const int64_t *d_n_combos;
    svt_fitrec rec;
    uint8_t *accept;
    svt_best best;          // best.chi2 holds the per-road key during the pass
    const int32_t *tile_first_road;
    unsigned long long *kb_counts;
    uint32_t *tile_counter;
    uint64_t *err;
    int64_t tile_combos;
    int64_t tiles_cap;
    int64_t road_cap;
    int64_t combo_cap;
    int32_t records;        // 0: kept-only mode, no per-combination records
    int32_t fold;           // shift <= 15: ql packed with f_j4 (see fit_xyz)
    int32_t chunk_roads;    // roads staged per chunk (16, 32 or kChunk)
    int32_t num_cus;        // CUs of the device (the grid holds wgs_per_cu workgroups per CU)
};

// One staged chunk: up to 64 consecutive roads of a tile.
struct Stage {
    // layer-grouped coordinates; the slack covers the 16-byte copies (up to 7 words past the
    // chunk's last) and the table build's reads of kMaxLayerHits words from a layer's start
    alignas(16) int16_t G[kWordCap + 32];
    int32_t XT[kTabCap];                   // coordinate-pair tables
    uint8_t M[kMapCap];                    // group of 4 combinations -> road of its first one,
                                           // or kListedBit | its index in X
    uint16_t X[kChunk];                    // groups that span a road boundary (from g_lo)
    uint8_t XR[kChunk];                    // road of the first combination of each group in X
    uint8_t ready[kChunk];                 // group X[x]'s records are in the stash (see Stash)
    RoadMeta meta[kChunk];
    RoadConst rc[kChunk];
    int32_t rb[kChunk];                    // road begin relative to the tile start
    int64_t tile_start;
    int64_t r_first;                       // global index of staged road 0
    int32_t nr, cs, ce, g_lo, g_hi, nx, done;
    int32_t narrow;                        // every staged road allows kFitNarrow (its rc too)
    int32_t work[2];                       // next unclaimed group / listed group (LDS atomics)
};

struct Loader {
    int64_t t, tile_start, tile_end, r_next;
    // lane 0: ticket of the next tile, fetched only when there are more tiles than workgroups,
    // and then once the tile's first chunk has arrived, not when the tile starts: memory
    // results return in issue order, so a fetch issued first would hold up the chunk's loads
    // behind the counter every workgroup hits at once.
    uint32_t ticket;
    bool need_ticket;
    // road-table entries of roads r_next + lane, loaded one chunk ahead
    bool pf;
    int64_t pcb, phb;
    int32_t pC, ps;
    uint32_t pnh;
};

__device__ __forceinline__ void load_roads(const FArgs &a, Loader &L, int64_t n_roads) {
    const int64_t r = L.r_next + lane_id();
    L.pcb = INT64_MAX;  // roads past the end are never valid
    L.phb = 0;
    L.pC = 0;
    L.ps = 0;
    L.pnh = 0;
    if (r < n_roads) {
        L.pcb = a.roads.combo_begin[r];
        L.pC = a.roads.ncombo[r];
        L.pnh = a.roads.nhits[r];
        L.phb = a.roads.hit_begin[r];
        L.ps = a.roads.set[r];
    }
    L.pf = true;
}

// first_road: the tile's first road when already read (< 0: read it here)
__device__ __forceinline__ void start_tile(const FArgs &a, Loader &L, int64_t n_tiles,
                                           int64_t n_combos, int64_t T, int64_t first_road = -1) {
    L.pf = false;
    if (L.t < n_tiles) {
        L.tile_start = L.t * T;
        L.tile_end = (L.tile_start + T < n_combos) ? L.tile_start + T : n_combos;
        L.r_next = first_road >= 0 ? first_road : a.tile_first_road[L.t];
        // tiles past the grid exist only when there are more tiles than workgroups
        L.need_ticket = n_tiles > static_cast<int64_t>(gridDim.x);
    }
}


// Wave 0: stage the next chunk into S (or mark the end of the work).
__device__ void produce(const FArgs &a, Stage &S, Loader &L, int64_t n_roads, int64_t n_combos,
                        int64_t n_tiles, int64_t T, uint32_t qlmask) {
    const int lane = lane_id();
    while (true) {
        if (L.t >= n_tiles) {
            if (lane == 0) S.done = 1;
            return;
        }
        if (!L.pf) load_roads(a, L, n_roads);
        // ---- sizes and capacities of up to 64 candidate roads
        const int64_t cb = L.pcb, hb = L.phb;
        const int32_t C = L.pC, s = L.ps;
        const uint32_t nh = L.pnh;
        const bool valid = cb < L.tile_end;
        const int32_t n0 = nh_of(nh, 0), n1 = nh_of(nh, 1), n2 = nh_of(nh, 2),
                      n3 = nh_of(nh, 3), n4 = nh_of(nh, 4);
        const int32_t nwords = valid ? n0 + n1 + n2 + n3 + n4 : 0;
        const int32_t ntab = (valid && C > 0) ? n0 * n1 + n2 * n3 + n4 : 0;
        const int32_t wend = wave_incl_scan(nwords), tend = wave_incl_scan(ntab);
        const int32_t wo = wend - nwords, to = tend - ntab;
        const bool fits = valid && lane < a.chunk_roads && wend <= kWordCap &&
                          tend <= kTabCap;  // a prefix of lanes
        const int nr = __popcll(__ballot(fits));
        if (nr == 0) {  // tile finished: continue with the ticket fetched during it
            if (L.need_ticket) {  // (never set when no tile lies past the grid: the ticket then
                                  // stays 0 and gridDim.x + 0 is past the last tile)
                if (lane == 0) L.ticket = atomicAdd(a.tile_counter, 1u);
                L.need_ticket = false;
            }
            const uint32_t tk = __shfl(L.ticket, 0);
            L.t = static_cast<int64_t>(gridDim.x) + tk;
            start_tile(a, L, n_tiles, n_combos, T);
            continue;
        }
        const int32_t tile_len = static_cast<int32_t>(L.tile_end - L.tile_start);
        const int32_t rb = static_cast<int32_t>(cb - L.tile_start);
        const int64_t span = __shfl(hb, 0);
        const int32_t nw = __shfl(wend, nr - 1);
        const int32_t first_rb = __shfl(rb, 0);
        const int32_t last_end = __shfl(rb + C, nr - 1);
        const int32_t cs = first_rb > 0 ? first_rb : 0;
        const int32_t ce = last_end < tile_len ? last_end : tile_len;
        const int32_t g_lo = cs >> 2, g_hi = (ce + 3) >> 2;
        const int32_t next_rb = __shfl_down(rb, 1);
        const int64_t r_first = L.r_next;

        // ---- issue every global read of this chunk before waiting on any: constant sets,
        //      the coordinate span (aligned 16-byte pieces), the next chunk's road table
        uint2 fw[8];
        uint2 qw[3];
        if (fits) {
            const uint2 *src = reinterpret_cast<const uint2 *>(a.bank + s);
#pragma unroll
            for (int i = 0; i < 8; ++i) fw[i] = src[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) qw[i] = src[8 + i];  // q[6] at byte 64
        }
        const int64_t base = span & ~static_cast<int64_t>(7);
        const int32_t goff = static_cast<int32_t>(span - base);
        const int32_t n16 = (goff + nw + 7) >> 3;  // <= 257
        uint4 v[5];
        {
            const uint4 *src = reinterpret_cast<const uint4 *>(a.coords + base);
#pragma unroll
            for (int u = 0; u < 5; ++u) {
                const int i = lane + 64 * u;
                v[u] = i < n16 ? src[i] : make_uint4(0, 0, 0, 0);
            }
        }
        L.r_next += nr;
        load_roads(a, L, n_roads);

        // ---- stage: coordinates, per-road indexing data and packed constants
        {
            uint4 *dst = reinterpret_cast<uint4 *>(S.G);
#pragma unroll
            for (int u = 0; u < 5; ++u) {
                const int i = lane + 64 * u;
                if (i < n16) dst[i] = v[u];
            }
        }
        if (L.need_ticket) {  // the chunk's loads are in: ask for the next tile now
            if (lane == 0) L.ticket = atomicAdd(a.tile_counter, 1u);
            L.need_ticket = false;
        }
        if (fits) {
            RoadMeta m;
            const uint32_t n23 = static_cast<uint32_t>(n2 * n3);
            m.w4 = magic_of(n4 > 0 ? n4 : 1) | (static_cast<uint32_t>(n4) << 24);
            m.w23 = magic_of(n23 > 0 ? n23 : 1) | (n23 << 24);
            m.b0123 = static_cast<uint32_t>(to) | (static_cast<uint32_t>(to + n0 * n1) << 16);
            m.b4c = static_cast<uint32_t>(to + n0 * n1 + n2 * n3) | (static_cast<uint32_t>(C) << 16);
            S.meta[lane] = m;
            S.rb[lane] = rb;
        }
        // the narrow form for the whole chunk when every staged road's constants allow it
        int32_t qv[6], fv[30];
#pragma unroll
        for (int i = 0; i < 30; ++i) fv[i] = f_el(fw, i);
        qv[0] = static_cast<int32_t>(qw[0].x);
        qv[1] = static_cast<int32_t>(qw[0].y);
        qv[2] = static_cast<int32_t>(qw[1].x);
        qv[3] = static_cast<int32_t>(qw[1].y);
        qv[4] = static_cast<int32_t>(qw[2].x);
        qv[5] = static_cast<int32_t>(qw[2].y);
        const bool narrow = __ballot(fits && !narrow_ok(fv, qv, a.shift)) == 0;
        if (fits) {
            RoadConst rc;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                rc.F01[j] = pack16(fv[5 * j + 0], fv[5 * j + 1]);
                rc.F23[j] = pack16(fv[5 * j + 2], fv[5 * j + 3]);
                const int32_t ql = static_cast<int32_t>(static_cast<uint32_t>(qv[j]) & qlmask);
                rc.F4[j] = pack16(fv[5 * j + 4], (a.fold && !narrow) ? ql : 0);
                rc.qh[j] = narrow ? 0 : qv[j] >> a.shift;
                rc.ql[j] = narrow ? qv[j] : ql;
            }
#pragma unroll
            for (int j = 0; j < 6; ++j) rc.pad[j] = 0;
            S.rc[lane] = rc;
        }
        __builtin_amdgcn_wave_barrier();  // one wave: its LDS writes precede its later reads

        // ---- per staged road: coordinate-pair tables and the group -> road map
        if (fits) {
            const int32_t g0 = goff + wo;
            if (C > 0) {
                const int32_t off1 = g0 + n0, off2 = off1 + n1, off3 = off2 + n2,
                              off4 = off3 + n3;
                const int32_t b01 = to, b23 = to + n0 * n1, b4 = b23 + n2 * n3;
                // the hits of layers 1, 3 and 4 in registers first (a layer of a road with
                // combinations holds at most kMaxLayerHits; reads past a layer stay inside
                // G's slack), so that the table writes wait on no LDS read of their own
                int32_t y1[kMaxLayerHits], y3[kMaxLayerHits], y4[kMaxLayerHits];
#pragma unroll
                for (int i = 0; i < kMaxLayerHits; ++i) {
                    y1[i] = S.G[off1 + i];
                    y3[i] = S.G[off3 + i];
                    y4[i] = S.G[off4 + i];
                }
                int32_t t = b01;
                for (int32_t h0 = 0; h0 < n0; ++h0, t += n1) {
                    const int32_t x0 = S.G[g0 + h0];
#pragma unroll
                    for (int h1 = 0; h1 < kMaxLayerHits; ++h1)
                        if (h1 < n1) S.XT[t + h1] = pack16(x0, y1[h1]);
                }
                t = b23;
                for (int32_t h2 = 0; h2 < n2; ++h2, t += n3) {
                    const int32_t x2 = S.G[off2 + h2];
#pragma unroll
                    for (int h3 = 0; h3 < kMaxLayerHits; ++h3)
                        if (h3 < n3) S.XT[t + h3] = pack16(x2, y3[h3]);
                }
#pragma unroll
                for (int h4 = 0; h4 < kMaxLayerHits; ++h4)
                    if (h4 < n4) S.XT[b4 + h4] = pack16(y4[h4], 1);
            }
            // groups whose first combination inside [cs, ce) belongs to this road
            const int32_t glo = rb <= cs ? g_lo : (rb + 3) >> 2;
            int32_t ghi = g_hi;
            if (lane + 1 < nr) ghi = next_rb <= cs ? g_lo : (next_rb + 3) >> 2;
            if (ghi > g_hi) ghi = g_hi;
            for (int32_t g = glo; g < ghi; ++g) S.M[g - g_lo] = static_cast<uint8_t>(lane);
        }
        // groups that span a road boundary: a road with combinations starts inside the group
        // (not at a multiple of 4) after the chunk's first combination; one entry per group
        {
            const int32_t g = rb >> 2;
            const bool cut = fits && C > 0 && (rb & 3) != 0 && rb > cs && rb < ce;
            const bool pcut = __shfl_up(cut ? 1 : 0, 1) != 0 && lane > 0;
            const int32_t pg = __shfl_up(g, 1);
            const bool head = cut && !(pcut && pg == g);
            const uint64_t hm = __ballot(head);
            if (head) {
                const int xi = __popcll(hm & ((1ull << lane) - 1));
                S.X[xi] = static_cast<uint16_t>(g - g_lo);
                S.XR[xi] = S.M[g - g_lo];  // written above by the road of the group's start
                S.M[g - g_lo] = static_cast<uint8_t>(kListedBit | xi);
            }
            if (lane == 0) S.nx = __popcll(hm);
        }
        if (lane == 0) {
            S.tile_start = L.tile_start;
            S.r_first = r_first;
            S.nr = nr;
            S.cs = cs;
            S.ce = ce;
            S.g_lo = g_lo;
            S.g_hi = g_hi;
            S.done = 0;
            S.narrow = narrow ? 1 : 0;
            S.work[0] = 0;
            S.work[1] = 0;
        }
        S.ready[lane] = 0;  // kChunk lanes
        return;
    }
}

// First of the next 64 work items of a staged chunk for the calling wave (wave-uniform); lane i
// takes item base + i.  Waves claim work as they become free, the loader wave included once it
// has staged the next chunk, so no wave waits at the chunk barrier for a slower one.
__device__ __forceinline__ int32_t claim64(int32_t *counter) {
    int32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, kWaveSize);
    return __shfl(base, 0);
}

// A group whose valid slots all lie in staged road ri: four fits with one road's constants
// (slots outside `slots` compute a harmless dummy, k = 0).  Returns the records and the accept
// bits; the caller writes them.
template <int MODE>
__device__ __forceinline__ uint32_t fit_group(const FArgs &a, const Stage &S, int ri, int32_t rel0,
                                              uint32_t slots, int64_t tile_start, int64_t r_first,
                                              int32_t *vp0, int32_t *vp1, int32_t *vp2,
                                              int32_t *vc0, int32_t *vc1, int32_t *vc2,
                                              int64_t *vchi) {
    const RoadMeta m = S.meta[ri];
    const RoadConst c = S.rc[ri];
    const int32_t rbase = S.rb[ri];
    int32_t kk[4];
    Fit f4r[4];
    fit4<MODE>(m, c, rel0 - rbase, S.XT, a.shift, f4r);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const Fit &f = f4r[e];
        vp0[e] = f.v[0]; vp1[e] = f.v[1]; vp2[e] = f.v[2];
        vc0[e] = f.v[3]; vc1[e] = f.v[4]; vc2[e] = f.v[5];
        vchi[e] = f.chi2;
        kk[e] = rel0 + e - rbase;
    }
    uint32_t acc_bits = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e)
        acc_bits |= ((slots >> e) & 1u) && vchi[e] <= a.cut ? (1u << e) : 0u;
    const int64_t gi = tile_start + rel0;
    if (acc_bits) {  // rare: one global atomic pair per road and group
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(a.best.chi2);
        if (a.kb_counts)
            atomicAdd(a.kb_counts + gi / kKeptBlock,
                      static_cast<unsigned long long>(__popc(acc_bits)));
        unsigned long long kmin = ~0ull;
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if ((acc_bits >> e) & 1u) {
                const unsigned long long kv = best_key(vchi[e], static_cast<uint32_t>(kk[e]));
                kmin = kv < kmin ? kv : kmin;
            }
        atomicMin(keys + r_first + ri, kmin);
        atomicAdd(a.best.n_accept + r_first + ri, __popc(acc_bits));
    }
    return acc_bits;
}

// The records of the groups that span a road boundary wait in LDS until the main pass writes
// them with the same store instructions as their neighbours' records.  A 128-byte line whose
// parts are written by different instructions at different times can reach memory in parts,
// at a large cost (fitting those groups in a second round of the chunk instead raised the
// written bytes by 16 % and the kernel time by 59 % on 3000 events of 2048 roads).  The stash
// takes the staged coordinates' LDS, which no fit reads: per listed group its records
// (REC > kRecNone), then 4 accept bytes per group.  A listed group past the capacity is written
// by the listed pass itself.
template <int REC>
struct Stash {
    static constexpr int kRecBytes = REC == kRecNone ? 0 : (REC == kRecFit ? 80 : 128);
    static constexpr int kBytes = static_cast<int>(sizeof(Stage::G));
    static constexpr int kCap = kBytes / (kRecBytes + 4) < kChunk ? kBytes / (kRecBytes + 4)
                                                                  : kChunk;
    // record layout: p0[4], p1[4], p2[4] (int32), chi2[4] (int64), then c0[4], c1[4], c2[4]
    __device__ static int32_t *rec32(Stage &S, int x) {
        return reinterpret_cast<int32_t *>(reinterpret_cast<uint8_t *>(S.G) + x * kRecBytes);
    }
    __device__ static int64_t *chi(Stage &S, int x) {
        return reinterpret_cast<int64_t *>(reinterpret_cast<uint8_t *>(S.G) + x * kRecBytes + 48);
    }
    __device__ static uint8_t *acc(Stage &S, int x) {
        return reinterpret_cast<uint8_t *>(S.G) + kCap * kRecBytes + 4 * x;
    }
};
static_assert(Stash<kRecRows>::kCap >= 16 && Stash<kRecNone>::kCap == kChunk, "stash room");
static_assert(kChunk <= kListedBit && kChunk == kWaveSize, "listed index; one loader lane per road");

// A listed group's ready flag as an LDS address: a volatile access through a generic pointer
// becomes a flat access, which also waits for every outstanding global store of the wave.
typedef __attribute__((address_space(3))) volatile uint8_t lds_flag;
__device__ __forceinline__ lds_flag *ready_flag(Stage &S, int x) {
    return (lds_flag *)(&S.ready[x]);
}

// One combination ci (relative to the tile start) of listed group x (slot e), fitted with the
// constants of its own road (the group's first road is r; later roads follow in staging order).
// Its records go to the stash, or to memory past the stash's capacity.  Such groups are few (at
// most one per road), but at small roads one chunk holds dozens of them; one lane per
// combination rather than per group spreads them over four times as many lanes.
template <int MODE, int REC>
__device__ void fit_slot(const FArgs &a, Stage &S, int r, int32_t ci, int64_t tile_start,
                         int64_t r_first, int x, int e, int xcap) {
    const int nr = S.nr;
    while (r + 1 < nr && ci >= S.rb[r] + S.meta[r].C()) ++r;  // skips empty roads
    const int32_t k = ci - S.rb[r];
    const Fit f = fit_combo<MODE>(S.meta[r], S.rc[r], static_cast<uint32_t>(k), S.XT, a.shift);
    const bool acc = f.chi2 <= a.cut;
    const int64_t gi = tile_start + ci;
    if (x < xcap) {
        if (REC != kRecNone) {
            int32_t *q = Stash<REC>::rec32(S, x);
            q[e] = f.v[0];
            q[4 + e] = f.v[1];
            q[8 + e] = f.v[2];
            Stash<REC>::chi(S, x)[e] = f.chi2;
        }
        if (REC == kRecRows) {
            int32_t *q = Stash<REC>::rec32(S, x);
            q[20 + e] = f.v[3];
            q[24 + e] = f.v[4];
            q[28 + e] = f.v[5];
        }
        Stash<REC>::acc(S, x)[e] = acc ? 1 : 0;
    } else {
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
    }
    if (acc) {
        unsigned long long *keys = reinterpret_cast<unsigned long long *>(a.best.chi2);
        if (a.kb_counts) atomicAdd(a.kb_counts + gi / kKeptBlock, 1ull);
        atomicMin(keys + r_first + r,
                  static_cast<unsigned long long>(best_key(f.chi2, static_cast<uint32_t>(k))));
        atomicAdd(a.best.n_accept + r_first + r, 1);
    }
}

// Compute waves: fit every combination of a staged chunk that lies inside its tile.  A lane
// takes a group of 4 consecutive combinations.  The groups that span a road boundary are listed
// by the loader and fitted first, one combination per lane with its own road's constants.  In
// the main pass every other group takes the uniform path (one road's constants, 16-byte stores).
// With STASH (roads of 48 combinations or more on average) the listed groups' records wait in
// the stash and each main-pass lane writes its group's records, fitted or from the stash, with
// one set of store instructions for the whole wave.  Without it (small roads, where a chunk
// holds many listed groups and the main pass would wait on them) the listed pass writes them
// itself, before the main pass, so that the main pass completes their lines while they are
// still in L2 (the other order wrote 1.37x the algorithmic bytes against 1.18x on 3000 events of
// 64 roads of about 32 combinations).
template <int MODE, int REC, bool STASH>
__device__ void consume_listed(const FArgs &a, Stage &S) {
    constexpr int xcap = STASH ? Stash<REC>::kCap : 0;
    const int32_t cs = S.cs, ce = S.ce, g_lo = S.g_lo, g_hi = S.g_hi;
    const int64_t tile_start = S.tile_start, r_first = S.r_first;
    const int32_t ng = g_hi - g_lo;
    const int lane = lane_id();
    const int32_t nx = S.nx;
    while (true) {  // the listed groups, one combination per lane
        const int32_t base = claim64(&S.work[1]);
        if (base >= 4 * nx) break;
        const int32_t j = base + lane;
        if (j < 4 * nx) {
            // a claim holds whole groups (base is a multiple of 64), so the lanes of slots 0..3
            // of group x make their stash writes in one instruction stream
            const int x = j >> 2, e = j & 3;
            const int32_t ci = ((g_lo + S.X[x]) << 2) + e;
            if (ci >= cs && ci < ce)
                fit_slot<MODE, REC>(a, S, S.XR[x], ci, tile_start, r_first, x, e, xcap);
            if (x < xcap) {
                asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // the stash writes landed
                if (e == 0) *ready_flag(S, x) = 1;
            }
        }
    }
    if constexpr (!STASH) {
        // the listed groups are written; the main pass fits and writes every other group
        while (true) {
            const int32_t base = claim64(&S.work[0]);
            if (base >= ng) break;
            const int32_t it = base + lane;
            if (it < ng) {
                const int mv = S.M[it];
                if (!(mv & kListedBit)) {
                    const int32_t rel0 = (g_lo + it) << 2;
                    uint32_t valid = 0;
#pragma unroll
                    for (int e = 0; e < 4; ++e)
                        valid |= (rel0 + e >= cs && rel0 + e < ce) ? (1u << e) : 0u;
                    int32_t vp0[4], vp1[4], vp2[4], vc0[4], vc1[4], vc2[4];
                    int64_t vchi[4];
                    const uint32_t acc_bits = fit_group<MODE>(a, S, mv, rel0, valid, tile_start,
                                                              r_first, vp0, vp1, vp2, vc0, vc1,
                                                              vc2, vchi);
                    store_group<REC>(a.rec, a.accept, tile_start + rel0, valid, acc_bits, vp0,
                                     vp1, vp2, vc0, vc1, vc2, vchi);
                }
            }
        }
        return;
    }
    while (true) {
        const int32_t base = claim64(&S.work[0]);
        if (base >= ng) break;
        const int32_t it = base + lane;
        if (it < ng) {
            const int32_t g = g_lo + it;
            const int32_t rel0 = g << 2;
            const int mv = S.M[it];
            uint32_t valid = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) valid |= (rel0 + e >= cs && rel0 + e < ce) ? (1u << e) : 0u;
            int32_t vp0[4], vp1[4], vp2[4], vc0[4], vc1[4], vc2[4];
            int64_t vchi[4];
            uint32_t acc_bits = 0, slots = 0;
            if (mv & kListedBit) {
                const int x = mv & (kListedBit - 1);
                if (x < xcap) {
                    // its slots were claimed before any main-pass work, by waves that finish
                    // them without waiting on anything
                    while (*ready_flag(S, x) == 0) __builtin_amdgcn_s_sleep(1);
                    asm volatile("" ::: "memory");
                    if (REC != kRecNone) {
                        const int32_t *q = Stash<REC>::rec32(S, x);
                        const int64_t *qc = Stash<REC>::chi(S, x);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            vp0[e] = q[e];
                            vp1[e] = q[4 + e];
                            vp2[e] = q[8 + e];
                            vchi[e] = qc[e];
                        }
                    }
                    if (REC == kRecRows) {
                        const int32_t *q = Stash<REC>::rec32(S, x);
#pragma unroll
                        for (int e = 0; e < 4; ++e) {
                            vc0[e] = q[20 + e];
                            vc1[e] = q[24 + e];
                            vc2[e] = q[28 + e];
                        }
                    }
                    const uint32_t w =
                        *reinterpret_cast<const uint32_t *>(Stash<REC>::acc(S, x));
                    acc_bits = ((w & 1u) | ((w >> 7) & 2u) | ((w >> 14) & 4u) | ((w >> 21) & 8u)) &
                               valid;
                    slots = valid;
                }
            } else {
                acc_bits = fit_group<MODE>(a, S, mv, rel0, valid, tile_start, r_first, vp0, vp1,
                                           vp2, vc0, vc1, vc2, vchi);
                slots = valid;
            }
            if (slots)
                store_group<REC>(a.rec, a.accept, tile_start + rel0, slots, acc_bits, vp0, vp1,
                                 vp2, vc0, vc1, vc2, vchi);
        }
    }
}

template <int WG, bool FOLD, int REC>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(WG == 256 ? 3 : 2))) void k_fused(FArgs a) {
    static_assert(WG > kWaveSize, "one loader wave plus compute waves");
    __shared__ Stage S[2];

    // The error word, the two sizes and the first road of this workgroup's first tile do not
    // depend on each other: one vector load brings all of them, lanes 0-5 the 32-bit halves of
    // the three 64-bit words and lane 6 the first road, so they share one round trip (as
    // uniform scalar loads the compiler serialises them, one wait each).  Errors of the earlier
    // kernels of the pass are what matters here, so a plain load of the error word suffices.
    int64_t first_road, n_roads, n_combos;
    uint64_t err0;
    {
        const int ln = lane_id();
        const uint32_t *p = reinterpret_cast<const uint32_t *>(a.err);
        p = (ln == 2 || ln == 3) ? reinterpret_cast<const uint32_t *>(a.d_n_roads) : p;
        p = (ln == 4 || ln == 5) ? reinterpret_cast<const uint32_t *>(a.d_n_combos) : p;
        p = (ln == 6 && blockIdx.x < a.tiles_cap)
                ? reinterpret_cast<const uint32_t *>(a.tile_first_road + blockIdx.x)
                : p;
        const int w = static_cast<int>(p[(ln < 6 && (ln & 1)) ? 1 : 0]);
        auto word64 = [&](int l) {
            return static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(w, l))) |
                   (static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readlane(w, l + 1)))
                    << 32);
        };
        err0 = word64(0);
        n_roads = static_cast<int64_t>(word64(2));
        n_combos = static_cast<int64_t>(word64(4));
        first_road = blockIdx.x < a.tiles_cap ? __builtin_amdgcn_readlane(w, 6) : 0;
    }
    if ((err0 != SVT_NO_ERROR) | (n_roads < 0) | (n_roads > a.road_cap) | (n_combos < 0) |
        (n_combos > a.combo_cap))
        return;
    const int64_t T = a.tile_combos;
    const int64_t n_tiles = (n_combos + T - 1) / T;
    if (n_tiles > a.tiles_cap) return;
    const int wave = threadIdx.x / kWaveSize;
    const uint32_t qlmask = (1u << a.shift) - 1u;
    // where the listed groups' records wait, from the batch's mean combinations per road
    const bool stash = n_combos >= kStashMinMean * n_roads;

    Loader L;
    L.t = blockIdx.x;
    L.tile_start = L.tile_end = L.r_next = 0;
    L.ticket = 0;
    L.need_ticket = false;
    L.pf = false;
    L.pcb = L.phb = 0;
    L.pC = L.ps = 0;
    L.pnh = 0;
    if (wave == 0) {
        start_tile(a, L, n_tiles, n_combos, T, first_road);
        produce(a, S[0], L, n_roads, n_combos, n_tiles, T, qlmask);
    }
    __syncthreads();
    int cur = 0;
    // Workgroups sharing a CU: equal priorities issue oldest first, and the dispatcher hands
    // out blocks 0 .. num_cus - 1 one per CU before the next num_cus, so the last-dispatched
    // workgroup of a CU (slot = blockIdx.x / num_cus) fitted its chunks about 20 % slower and
    // ended 4-5 us after the first on 3000 events of 64 roads; the kernel waits for it.  The
    // compute priority rotates over the slots from chunk to chunk (youngest highest first), so
    // the workgroups of a CU take turns; all waves of a workgroup share one level.
    const int slot = static_cast<int>(blockIdx.x) / (a.num_cus > 0 ? a.num_cus : 1);
    int iter = 0;
    while (!S[cur].done) {
        // The loader runs at the top priority while it stages: its chain of dependent loads
        // and LDS writes sets the pace of the pipeline, and on its SIMD it would otherwise wait
        // for issue slots behind the compute waves' arithmetic (about 2 % with roads of ~32 and
        // of ~100 combinations).
        if (wave == 0) {
            __builtin_amdgcn_s_setprio(3);
            produce(a, S[cur ^ 1], L, n_roads, n_combos, n_tiles, T, qlmask);
        }
        set_prio((slot + iter) % 3);
        // every wave, the loader once it has staged the next chunk
        constexpr int kWide = FOLD ? kFitFold : kFitSplit;
        if (S[cur].narrow) {
            if (stash)
                consume_listed<kFitNarrow, REC, true>(a, S[cur]);
            else
                consume_listed<kFitNarrow, REC, false>(a, S[cur]);
        } else if (stash) {
            consume_listed<kWide, REC, true>(a, S[cur]);
        } else {
            consume_listed<kWide, REC, false>(a, S[cur]);
        }
        __syncthreads();
        cur ^= 1;
        ++iter;
    }
}

FArgs make_args(const FusedLaunch &f) {
    FArgs a;
    a.bank = f.bank;
    a.shift = f.cfg.shift;
    a.n_sets = f.cfg.n_sets;
    a.cut = f.cfg.chi2_cut;
    a.coords = f.coords;
    a.roads = f.roads;
    a.d_n_roads = f.d_n_roads;
    a.d_n_combos = f.d_n_combos;
    a.rec = f.rec;
    a.accept = f.accept;
    a.best = f.best;
    a.tile_first_road = f.tile_first_road;
    a.kb_counts = reinterpret_cast<unsigned long long *>(f.kb_counts);
    a.tile_counter = f.tile_counter;
    a.err = f.err;
    a.tile_combos = f.tune.tile_combos;
    a.tiles_cap = f.tiles_cap;
    a.road_cap = f.road_cap;
    a.combo_cap = f.combo_cap;
    a.records = f.kept_only ? 0 : 1;
    a.fold = f.cfg.shift <= 15 ? 1 : 0;
    a.chunk_roads = f.tune.chunk_roads;
    a.num_cus = f.num_cus;
    return a;
}

template <int WG, int REC>
void launch_fused_r(const FArgs &a, int grid, hipStream_t s) {
    if (a.fold)
        hipLaunchKernelGGL((k_fused<WG, true, REC>), dim3(grid), dim3(WG), 0, s, a);
    else
        hipLaunchKernelGGL((k_fused<WG, false, REC>), dim3(grid), dim3(WG), 0, s, a);
}

template <int WG>
hipError_t launch_fused_t(const FArgs &a, int grid, hipStream_t s) {
    if (a.records == 0)
        launch_fused_r<WG, kRecNone>(a, grid, s);
    else if (a.rec.c0 || a.rec.c1 || a.rec.c2)
        launch_fused_r<WG, kRecRows>(a, grid, s);
    else
        launch_fused_r<WG, kRecFit>(a, grid, s);
    return hipGetLastError();
}

}  // namespace

bool fused_tune_supported(const svt_tune &t) {
    const bool wg_ok = t.wg_size == 256 || t.wg_size == 512;
    const bool ch_ok = t.chunk_roads == 16 || t.chunk_roads == 32 || t.chunk_roads == kChunk;
    const bool tile_ok = t.tile_combos >= kKeptBlock && t.tile_combos <= kMaxTile &&
                         t.tile_combos % kKeptBlock == 0;
    // the one-pass kernel's LDS holds three workgroups per CU: more would not be resident
    // (schedule 0, chosen per batch, may become the one-pass kernel)
    const int occ_max = (t.schedule == SVT_SCHEDULE_ONEPASS || t.schedule == 0) ? 3 : 8;
    const bool occ_ok = t.wgs_per_cu >= 1 && t.wgs_per_cu <= occ_max;
    const bool sched_ok = t.schedule == 0 || t.schedule == SVT_SCHEDULE_TILES ||
                          t.schedule == SVT_SCHEDULE_EVENTS || t.schedule == SVT_SCHEDULE_ONEPASS;
    return wg_ok && ch_ok && tile_ok && occ_ok && sched_ok;
}

hipError_t launch_fused(const FusedLaunch &f, hipStream_t s) {
    const FArgs a = make_args(f);
    // persistent grid: wgs_per_cu per CU, but no more workgroups than the capacity has tiles
    const int64_t tiles = (f.combo_cap + f.tune.tile_combos - 1) / f.tune.tile_combos;
    const int grid = static_cast<int>(
        std::max<int64_t>(1, std::min<int64_t>(int64_t{f.num_cus} * f.tune.wgs_per_cu, tiles)));
    if (f.tune.wg_size == 256) return launch_fused_t<256>(a, grid, s);
    if (f.tune.wg_size == 512) return launch_fused_t<512>(a, grid, s);
    return hipErrorInvalidValue;
}

}  // namespace svt
