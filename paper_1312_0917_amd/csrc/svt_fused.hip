// Persistent fused combine + fit + select kernel of libsvt, and its split-road fixup.
//
// The fit of section II is p_j = sum_l f[j][l] x_l + q_j followed by the fixed-point shift.
// Constants are int16 and coordinates int13, so the five products of one parameter are three
// packed 16-bit dot products (v_dot2_i32_i16) once the coordinates of layers (0,1) and (2,3)
// are paired: each road's hits are staged in LDS as small tables of coordinate pairs, and one
// combination is three LDS reads plus eighteen dot products.  The offset is split exactly as
// q = qh * 2^s + ql with 0 <= ql < 2^s: ql seeds the accumulator, so the sum stays inside
// int32, and
//     floor((S + q) / 2^s) = qh + floor((S + ql) / 2^s)       (exact for every integer S).
//
// Work distribution: combinations are numbered globally (road-major, combo_begin from the
// pre-pass); workgroups of a persistent grid take tiles of tile_combos consecutive
// combinations from an atomic counter.  A tile stages its roads in LDS in chunks of up to
// CHUNK roads (bounded by the LDS word and table capacities): the chunk's hit words are one
// contiguous span of the input, copied with coalesced loads.  Each lane fits 4 consecutive
// combinations so that every record array is written with 16-byte coalesced stores.  Roads
// entirely inside a tile get their best track from LDS atomics; roads cut by tile boundaries
// leave partial (key, count) pairs per tile that the fixup kernel merges.
#include "svt_common.h"

namespace svt {
namespace {

constexpr int kWordCap = 2048;         // hit words staged per chunk (a road has at most 40)
constexpr int kTabCap = 2048;          // coordinate-pair table entries per chunk (<= 136 per road)
constexpr int kMaxKb = 4;              // kept-count blocks per tile (tile_combos <= 16384)
constexpr uint32_t kKMask = (1u << kKeyKBits) - 1;

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
    svt_best best;
    const int32_t *tile_first_road;
    Partial *part;
    int64_t *kb_counts;
    uint32_t *tile_counter;
    uint64_t *err;
    int64_t tile_combos;
    int64_t tiles_cap;
    int64_t road_cap;
    int64_t combo_cap;
};

// Per-road indexing data of the current chunk, in LDS (32 bytes).
struct alignas(16) RoadMeta {
    int32_t C;      // combinations
    uint32_t m4;    // division magic of n4 (0 when n4 == 1)
    uint32_t m23;   // division magic of n2 * n3 (0 when 1)
    uint32_t nn;    // n4 | (n2 * n3) << 8
    int32_t b01;    // table index of the (h0, h1) coordinate pairs
    int32_t b23;    // table index of the (h2, h3) pairs
    int32_t b4;     // table index of the layer-4 coordinates
    int32_t wo;     // first staged word of the road
};

// Per-road constants of the current chunk, packed for the dot products (128 bytes).
struct alignas(16) RoadConst {
    int32_t F01[6];  // (f[j][0], f[j][1]) as an int16 pair
    int32_t F23[6];  // (f[j][2], f[j][3])
    int32_t F4[6];   // (f[j][4], 0)
    int32_t ql[6];   // q[j] mod 2^shift
    int32_t qh[6];   // floor(q[j] / 2^shift)
    int32_t pad[2];
};

typedef short v2s __attribute__((ext_vector_type(2)));

// a.lo * b.lo + a.hi * b.hi + c on signed 16-bit halves (v_dot2_i32_i16, no clamping).
__device__ __forceinline__ int32_t dot2(int32_t a, int32_t b, int32_t c) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(v2s, a), __builtin_bit_cast(v2s, b), c,
                                  false);
}

// floor(k / n) for 0 <= k < 2^15 and 1 <= n <= 64 with m = ceil(2^32 / n) (m = 0 for n = 1):
// k * (m * n - 2^32) < 2^15 * 64 < 2^32, so the high word of k * m is exact.
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t m) {
    return m ? __umulhi(k, m) : k;
}

__host__ __device__ constexpr uint32_t magic_of(uint32_t n) {
    return n <= 1 ? 0u : static_cast<uint32_t>((0x100000000ull + n - 1) / n);
}

__device__ __forceinline__ int32_t pack16(int32_t lo, int32_t hi) {
    return static_cast<int32_t>((static_cast<uint32_t>(lo) & 0xFFFFu) |
                                (static_cast<uint32_t>(hi) << 16));
}

struct Fit {
    int32_t v[6];
    int64_t chi2;
};

// Fit combination k of a road.  k = (i01 * n23 + i23) * n4 + h4, where i01 = h0 * n1 + h1
// and i23 = h2 * n3 + h3 index the coordinate-pair tables.  Each sum
//     ql_j + f_j0 x0 + f_j1 x1 + f_j2 x2 + f_j3 x3 + f_j4 x4
// is three packed 16-bit dot products; |sum| < 2^30 + 5 * 2^27 < 2^31, so int32 is exact.
__device__ __forceinline__ Fit fit_combo(const RoadMeta &m, const RoadConst &c, uint32_t k,
                                         const int32_t *XT, int32_t shift) {
    const uint32_t n4 = m.nn & 0xFFu, n23 = m.nn >> 8;
    const uint32_t q4 = div_small(k, m.m4);
    const uint32_t h4 = k - q4 * n4;
    const uint32_t i01 = div_small(q4, m.m23);
    const uint32_t i23 = q4 - i01 * n23;
    const int32_t x01 = XT[m.b01 + static_cast<int32_t>(i01)];
    const int32_t x23 = XT[m.b23 + static_cast<int32_t>(i23)];
    const int32_t x4 = XT[m.b4 + static_cast<int32_t>(h4)];
    Fit f;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        int32_t acc = dot2(c.F01[j], x01, c.ql[j]);
        acc = dot2(c.F23[j], x23, acc);
        acc = dot2(c.F4[j], x4, acc);
        f.v[j] = (acc >> shift) + c.qh[j];
    }
    f.chi2 = static_cast<int64_t>(f.v[3]) * f.v[3] + static_cast<int64_t>(f.v[4]) * f.v[4] +
             static_cast<int64_t>(f.v[5]) * f.v[5];
    return f;
}

// int16 element i of a constant set's f[6][5] read as 8-byte words
__device__ __forceinline__ int32_t f_at(const uint2 *fw, int i) {
    const uint2 w = fw[i >> 2];
    const uint32_t d = ((i >> 1) & 1) ? w.y : w.x;
    return static_cast<int32_t>(static_cast<int16_t>((i & 1) ? (d >> 16) : (d & 0xFFFFu)));
}

template <int WG, int CHUNK>
__global__ __launch_bounds__(WG) void k_fused(FArgs a) {
    static_assert(CHUNK <= WG && CHUNK <= 256, "one thread per staged road, road index in a byte");
    constexpr int kMapCap = kKeptBlock * kMaxKb / 4;  // groups of 4 combinations in a tile
    constexpr int kCopy = (kWordCap + WG - 1) / WG;
    __shared__ int16_t G[kWordCap];           // layer-grouped coordinates of the staged roads
    __shared__ int32_t XT[kTabCap];           // coordinate-pair tables
    __shared__ uint8_t M[kMapCap];            // group of 4 combinations -> staged road
    __shared__ RoadMeta meta[CHUNK];
    __shared__ RoadConst rcst[CHUNK];
    __shared__ int32_t s_rb[CHUNK];           // road begin relative to the tile start
    __shared__ unsigned long long s_key[CHUNK];
    __shared__ uint32_t s_nacc[CHUNK];
    __shared__ uint32_t s_kb[kMaxKb];
    __shared__ int64_t s_scan[WG / kWaveSize + 1];
    __shared__ int64_t s_tile, s_first, s_span;
    __shared__ int32_t s_nr, s_nwords;

    if (has_error(a.err)) return;
    const int64_t n_roads = *a.d_n_roads;
    const int64_t n_combos = *a.d_n_combos;
    if (n_roads < 0 || n_roads > a.road_cap || n_combos < 0 || n_combos > a.combo_cap) return;
    const int64_t T = a.tile_combos;
    const int64_t n_tiles = (n_combos + T - 1) / T;
    if (n_tiles > a.tiles_cap) return;
    const int tid = threadIdx.x;
    const uint32_t qlmask = (1u << a.shift) - 1u;

    int64_t t = blockIdx.x;  // first tile by block index, the rest from the counter
    int64_t r_first = t < n_tiles ? a.tile_first_road[t] : 0;
    while (t < n_tiles) {
        uint32_t ticket = 0;
        if (tid == 0) ticket = atomicAdd(a.tile_counter, 1u);  // next tile, fetched early
        if (tid < kMaxKb) s_kb[tid] = 0;
        const int64_t tile_start = t * T;
        const int64_t tile_end = (tile_start + T < n_combos) ? tile_start + T : n_combos;
        const int32_t tile_len = static_cast<int32_t>(tile_end - tile_start);
        int64_t r_next = r_first;
        int64_t next_first = 0;
        bool prefetched = false;

        while (true) {
            // ---- A1: one thread per candidate road: sizes, capacity, indexing, constants
            const int64_t r = r_next + tid;
            bool valid = false;
            int64_t cb = 0, hb = 0;
            int32_t C = 0, s = 0;
            uint32_t nh = 0;
            if (tid < CHUNK && r < n_roads) {
                cb = a.roads.combo_begin[r];
                valid = cb < tile_end;
                if (valid) {
                    C = a.roads.ncombo[r];
                    nh = a.roads.nhits[r];
                    hb = a.roads.hit_begin[r];
                    s = a.roads.set[r];
                }
            }
            const int32_t n0 = nh_of(nh, 0), n1 = nh_of(nh, 1), n2 = nh_of(nh, 2),
                          n3 = nh_of(nh, 3), n4 = nh_of(nh, 4);
            const int32_t nwords = n0 + n1 + n2 + n3 + n4;
            const int32_t ntab = (valid && C > 0) ? n0 * n1 + n2 * n3 + n4 : 0;
            const int64_t packed = static_cast<int64_t>(valid ? nwords : 0) |
                                   (static_cast<int64_t>(ntab) << 32);
            if (tid == 0) {
                s_nr = 0;
                s_nwords = 0;
            }
            int64_t total;
            const int64_t ex = block_excl_scan<int64_t, WG>(packed, s_scan, total);
            const int32_t wo = static_cast<int32_t>(ex & 0xFFFFFFFF);
            const int32_t to = static_cast<int32_t>(ex >> 32);
            const bool fits = valid && wo + nwords <= kWordCap && to + ntab <= kTabCap;
            if (fits) {
                atomicMax(&s_nr, tid + 1);
                atomicMax(&s_nwords, wo + nwords);
                RoadMeta m;
                m.C = C;
                m.m4 = magic_of(n4);
                m.m23 = magic_of(n2 * n3);
                m.nn = static_cast<uint32_t>(n4) | (static_cast<uint32_t>(n2 * n3) << 8);
                m.b01 = to;
                m.b23 = to + n0 * n1;
                m.b4 = to + n0 * n1 + n2 * n3;
                m.wo = wo;
                meta[tid] = m;
                s_rb[tid] = static_cast<int32_t>(cb - tile_start);
                s_key[tid] = ~0ull;
                s_nacc[tid] = 0;
                if (tid == 0) s_span = hb;
                // constant set: f[6][5] int16 (60 bytes), 4 bytes pad, q[6] int32
                const uint2 *fw = reinterpret_cast<const uint2 *>(a.bank + s);
                RoadConst rc;
#pragma unroll
                for (int j = 0; j < 6; ++j) {
                    rc.F01[j] = pack16(f_at(fw, 5 * j + 0), f_at(fw, 5 * j + 1));
                    rc.F23[j] = pack16(f_at(fw, 5 * j + 2), f_at(fw, 5 * j + 3));
                    rc.F4[j] = pack16(f_at(fw, 5 * j + 4), 0);
                    const int32_t q = a.bank[s].q[j];
                    rc.qh[j] = q >> a.shift;
                    rc.ql[j] = static_cast<int32_t>(static_cast<uint32_t>(q) & qlmask);
                }
                rc.pad[0] = rc.pad[1] = 0;
                rcst[tid] = rc;
            }
            __syncthreads();
            const int nr = s_nr;
            if (nr == 0) break;
            if (tid == 0 && !prefetched) {  // first road of the next tile, while this one runs
                const int64_t nt = static_cast<int64_t>(gridDim.x) + ticket;
                next_first = nt < n_tiles ? a.tile_first_road[nt] : 0;
                prefetched = true;
            }

            // ---- A2: copy the chunk's grouped coordinates (one contiguous span) into LDS
            {
                const int32_t nw = s_nwords;
                const int16_t *src = a.coords + s_span;
                int16_t v[kCopy];
#pragma unroll
                for (int u = 0; u < kCopy; ++u) {
                    const int i = tid + u * WG;
                    v[u] = i < nw ? src[i] : static_cast<int16_t>(0);
                }
#pragma unroll
                for (int u = 0; u < kCopy; ++u) {
                    const int i = tid + u * WG;
                    if (i < nw) G[i] = v[u];
                }
            }
            const int32_t first_rb = s_rb[0];
            const int32_t last_end = s_rb[nr - 1] + meta[nr - 1].C;
            const int32_t cs = first_rb > 0 ? first_rb : 0;
            const int32_t ce = last_end < tile_len ? last_end : tile_len;
            const int32_t g_lo = cs >> 2, g_hi = (ce + 3) >> 2;
            __syncthreads();

            // ---- A3: per road, coordinate-pair tables and the group -> road map
            if (tid < nr) {
                if (C > 0) {
                    const int32_t off1 = wo + n0, off2 = off1 + n1, off3 = off2 + n2,
                                  off4 = off3 + n3;
                    const int32_t b01 = to, b23 = to + n0 * n1, b4 = b23 + n2 * n3;
                    for (int32_t h0 = 0; h0 < n0; ++h0) {
                        const int32_t x0 = G[wo + h0];
                        for (int32_t h1 = 0; h1 < n1; ++h1)
                            XT[b01 + h0 * n1 + h1] = pack16(x0, G[off1 + h1]);
                    }
                    for (int32_t h2 = 0; h2 < n2; ++h2) {
                        const int32_t x2 = G[off2 + h2];
                        for (int32_t h3 = 0; h3 < n3; ++h3)
                            XT[b23 + h2 * n3 + h3] = pack16(x2, G[off3 + h3]);
                    }
                    for (int32_t h4 = 0; h4 < n4; ++h4) XT[b4 + h4] = pack16(G[off4 + h4], 0);
                }
                // groups whose first combination inside [cs, ce) belongs to this road
                const int32_t rb = s_rb[tid];
                int32_t glo = rb <= cs ? g_lo : (rb + 3) >> 2;
                int32_t ghi = g_hi;
                if (tid + 1 < nr) {
                    const int32_t nb = s_rb[tid + 1];
                    ghi = nb <= cs ? g_lo : (nb + 3) >> 2;
                }
                if (ghi > g_hi) ghi = g_hi;
                for (int32_t g = glo; g < ghi; ++g) M[g - g_lo] = static_cast<uint8_t>(tid);
            }
            __syncthreads();

            // ---- B: fit every combination of the chunk that lies inside the tile
            for (int32_t g = g_lo + tid; g < g_hi; g += WG) {
                const int32_t rel0 = g << 2;
                const int32_t first = rel0 > cs ? rel0 : cs;
                const int32_t last = (rel0 + 3 < ce - 1) ? rel0 + 3 : ce - 1;
                int ri = M[g - g_lo];
                RoadMeta m = meta[ri];
                int32_t rbase = s_rb[ri];
                uint32_t valid_bits = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    valid_bits |= (rel0 + e >= cs && rel0 + e < ce) ? (1u << e) : 0u;
                int32_t vp0[4], vp1[4], vp2[4], vc0[4], vc1[4], vc2[4];
                int64_t vchi[4];
                int32_t kk[4];
                int rr4[4];
                if (last - rbase < m.C) {
                    // common case: every valid combination of the group is in road ri; the
                    // four fits are independent (invalid slots compute a dummy k = 0)
                    const RoadConst c = rcst[ri];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        const int32_t k = (valid_bits >> e) & 1u ? rel0 + e - rbase : 0;
                        const Fit f = fit_combo(m, c, static_cast<uint32_t>(k), XT, a.shift);
                        vp0[e] = f.v[0]; vp1[e] = f.v[1]; vp2[e] = f.v[2];
                        vc0[e] = f.v[3]; vc1[e] = f.v[4]; vc2[e] = f.v[5];
                        vchi[e] = f.chi2;
                        kk[e] = k;
                        rr4[e] = ri;
                    }
                } else {
                    int32_t k = first - rbase;
                    RoadConst c = rcst[ri];
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        vp0[e] = vp1[e] = vp2[e] = vc0[e] = vc1[e] = vc2[e] = 0;
                        vchi[e] = 0;
                        kk[e] = 0;
                        rr4[e] = ri;
                        if ((valid_bits >> e) & 1u) {
                            if (k >= m.C) {
                                while (k >= m.C && ri + 1 < nr) {  // bounded by the chunk
                                    k -= m.C;
                                    ++ri;
                                    m = meta[ri];
                                }
                                c = rcst[ri];
                            }
                            const Fit f = fit_combo(m, c, static_cast<uint32_t>(k), XT, a.shift);
                            vp0[e] = f.v[0]; vp1[e] = f.v[1]; vp2[e] = f.v[2];
                            vc0[e] = f.v[3]; vc1[e] = f.v[4]; vc2[e] = f.v[5];
                            vchi[e] = f.chi2;
                            kk[e] = k;
                            rr4[e] = ri;
                            ++k;
                        }
                    }
                }
                uint32_t acc_bits = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc_bits |= ((valid_bits >> e) & 1u) && vchi[e] <= a.cut ? (1u << e) : 0u;
                if (acc_bits) {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if ((acc_bits >> e) & 1u) {
                            atomicMin(&s_key[rr4[e]], static_cast<unsigned long long>(
                                                          best_key(vchi[e], static_cast<uint32_t>(kk[e]))));
                            atomicAdd(&s_nacc[rr4[e]], 1u);
                            atomicAdd(&s_kb[(rel0 + e) >> 12], 1u);
                        }
                    }
                }
                const int64_t gi = tile_start + rel0;
                if (valid_bits == 0xF) {
                    *reinterpret_cast<int4 *>(a.rec.p0 + gi) = make_int4(vp0[0], vp0[1], vp0[2], vp0[3]);
                    *reinterpret_cast<int4 *>(a.rec.p1 + gi) = make_int4(vp1[0], vp1[1], vp1[2], vp1[3]);
                    *reinterpret_cast<int4 *>(a.rec.p2 + gi) = make_int4(vp2[0], vp2[1], vp2[2], vp2[3]);
                    longlong2 *c2p = reinterpret_cast<longlong2 *>(a.rec.chi2 + gi);
                    c2p[0] = make_longlong2(vchi[0], vchi[1]);
                    c2p[1] = make_longlong2(vchi[2], vchi[3]);
                    if (a.rec.c0) *reinterpret_cast<int4 *>(a.rec.c0 + gi) = make_int4(vc0[0], vc0[1], vc0[2], vc0[3]);
                    if (a.rec.c1) *reinterpret_cast<int4 *>(a.rec.c1 + gi) = make_int4(vc1[0], vc1[1], vc1[2], vc1[3]);
                    if (a.rec.c2) *reinterpret_cast<int4 *>(a.rec.c2 + gi) = make_int4(vc2[0], vc2[1], vc2[2], vc2[3]);
                    const uint32_t accw = (acc_bits & 1u) | ((acc_bits & 2u) << 7) |
                                          ((acc_bits & 4u) << 14) | ((acc_bits & 8u) << 21);
                    *reinterpret_cast<uint32_t *>(a.accept + gi) = accw;
                } else {
#pragma unroll
                    for (int e = 0; e < 4; ++e) {
                        if (valid_bits & (1u << e)) {
                            a.rec.p0[gi + e] = vp0[e];
                            a.rec.p1[gi + e] = vp1[e];
                            a.rec.p2[gi + e] = vp2[e];
                            a.rec.chi2[gi + e] = vchi[e];
                            if (a.rec.c0) a.rec.c0[gi + e] = vc0[e];
                            if (a.rec.c1) a.rec.c1[gi + e] = vc1[e];
                            if (a.rec.c2) a.rec.c2[gi + e] = vc2[e];
                            a.accept[gi + e] = (acc_bits >> e) & 1u;
                        }
                    }
                }
            }
            __syncthreads();

            // ---- C: best track of roads inside the tile, exact partials otherwise
            if (tid < nr) {
                const RoadMeta m = meta[tid];
                const RoadConst c = rcst[tid];
                const int32_t rb = s_rb[tid];
                const int64_t rr = r_next + tid;
                if (m.C > 0) {
                    const unsigned long long key = s_key[tid];
                    const uint32_t nacc = s_nacc[tid];
                    // this road's combinations inside the tile: k in [k_lo, k_hi)
                    const int32_t k_lo = rb < 0 ? -rb : 0;
                    const int32_t k_hi = (rb + m.C <= tile_len) ? m.C : tile_len - rb;
                    uint64_t bchi = ~0ull;
                    uint32_t bk = 0xFFFFFFFFu;
                    if (key != ~0ull) {
                        bchi = key >> kKeyKBits;
                        bk = static_cast<uint32_t>(key) & kKMask;
                        if (bchi == kKeyChiMax) {  // saturated key: exact rescan of the part
                            bchi = ~0ull;
                            for (int32_t k = k_lo; k < k_hi; ++k) {
                                const Fit f = fit_combo(m, c, static_cast<uint32_t>(k), XT, a.shift);
                                if (f.chi2 <= a.cut && static_cast<uint64_t>(f.chi2) < bchi) {
                                    bchi = static_cast<uint64_t>(f.chi2);
                                    bk = static_cast<uint32_t>(k);
                                }
                            }
                        }
                    }
                    if (rb >= 0 && rb + m.C <= tile_len) {
                        a.best.n_accept[rr] = static_cast<int32_t>(nacc);
                        if (bchi == ~0ull) {
                            a.best.k[rr] = -1;
                            a.best.p0[rr] = INT32_MIN;
                            a.best.p1[rr] = INT32_MIN;
                            a.best.p2[rr] = INT32_MIN;
                            a.best.chi2[rr] = INT64_MAX;
                        } else {
                            const Fit f = fit_combo(m, c, bk, XT, a.shift);
                            a.best.k[rr] = static_cast<int32_t>(bk);
                            a.best.p0[rr] = f.v[0];
                            a.best.p1[rr] = f.v[1];
                            a.best.p2[rr] = f.v[2];
                            a.best.chi2[rr] = static_cast<int64_t>(bchi);
                        }
                    } else {
                        const int slot = rb < 0 ? 0 : 1;
                        a.part[2 * t + slot] = Partial{bchi, bk, nacc};
                    }
                }
            }
            r_next += nr;
        }

        // tile end: accepted counts per block of 4096 combinations (kept-list compaction)
        if (tid < (tile_len + kKeptBlock - 1) / kKeptBlock)
            a.kb_counts[tile_start / kKeptBlock + tid] = s_kb[tid];
        if (tid == 0) {
            s_tile = static_cast<int64_t>(gridDim.x) + ticket;
            s_first = next_first;
        }
        __syncthreads();
        t = s_tile;
        r_first = s_first;
    }
}

// Merge the per-tile partials of roads cut by tile boundaries and write their best tracks.
__global__ void k_fixup(FArgs a) {
    if (has_error(a.err)) return;
    const int64_t n_combos = *a.d_n_combos;
    if (n_combos < 0 || n_combos > a.combo_cap) return;
    const int64_t T = a.tile_combos;
    const int64_t n_tiles = (n_combos + T - 1) / T;
    if (n_tiles > a.tiles_cap) return;
    for (int64_t t = gtid() + 1; t < n_tiles; t += gstride()) {
        const int64_t r = a.tile_first_road[t];
        const int64_t cb = a.roads.combo_begin[r];
        if (!(cb < t * T && cb >= (t - 1) * T)) continue;  // the road began in tile t-1
        const int64_t C = a.roads.ncombo[r];
        const int64_t te = (cb + C - 1) / T;
        Partial b = a.part[2 * (t - 1) + 1];
        for (int64_t u = t; u <= te && u < n_tiles; ++u) {
            const Partial p = a.part[2 * u];
            b.nacc += p.nacc;
            if (p.chi2 < b.chi2 || (p.chi2 == b.chi2 && p.k < b.k)) {
                b.chi2 = p.chi2;
                b.k = p.k;
            }
        }
        a.best.n_accept[r] = static_cast<int32_t>(b.nacc);
        if (b.chi2 == ~0ull) {
            a.best.k[r] = -1;
            a.best.p0[r] = INT32_MIN;
            a.best.p1[r] = INT32_MIN;
            a.best.p2[r] = INT32_MIN;
            a.best.chi2[r] = INT64_MAX;
        } else {
            const int64_t k = static_cast<int64_t>(b.k);
            const int64_t g = cb + k;
            a.best.k[r] = static_cast<int32_t>(k);
            a.best.chi2[r] = static_cast<int64_t>(b.chi2);
            a.best.p0[r] = a.rec.p0[g];
            a.best.p1[r] = a.rec.p1[g];
            a.best.p2[r] = a.rec.p2[g];
        }
    }
}

__global__ void k_batch_init(uint64_t *err, uint32_t *tile_counter, int64_t *d_n_kept) {
    *err = SVT_NO_ERROR;
    *tile_counter = 0;
    if (d_n_kept) *d_n_kept = 0;
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
    a.part = f.tile_part;
    a.kb_counts = f.kb_counts;
    a.tile_counter = f.tile_counter;
    a.err = f.err;
    a.tile_combos = f.tune.tile_combos;
    a.tiles_cap = f.tiles_cap;
    a.road_cap = f.road_cap;
    a.combo_cap = f.combo_cap;
    return a;
}

template <int WG, int CHUNK>
hipError_t launch_fused_t(const FArgs &a, int grid, hipStream_t s) {
    hipLaunchKernelGGL((k_fused<WG, CHUNK>), dim3(grid), dim3(WG), 0, s, a);
    return hipGetLastError();
}

}  // namespace

bool fused_tune_supported(const svt_tune &t) {
    const bool wg_ok = t.wg_size == 256 || t.wg_size == 512;
    const bool ch_ok = (t.chunk_roads == 64 || t.chunk_roads == 128 || t.chunk_roads == 256) &&
                       t.chunk_roads <= t.wg_size;
    const bool tile_ok = t.tile_combos >= kKeptBlock && t.tile_combos <= kKeptBlock * kMaxKb &&
                         t.tile_combos % kKeptBlock == 0;
    const bool occ_ok = t.wgs_per_cu >= 1 && t.wgs_per_cu <= 8;
    return wg_ok && ch_ok && tile_ok && occ_ok;
}

hipError_t launch_fused(const FusedLaunch &f, hipStream_t s) {
    const FArgs a = make_args(f);
    const int grid = f.num_cus * f.tune.wgs_per_cu;
    const int wg = f.tune.wg_size, ch = f.tune.chunk_roads;
    if (wg == 256 && ch == 64) return launch_fused_t<256, 64>(a, grid, s);
    if (wg == 256 && ch == 128) return launch_fused_t<256, 128>(a, grid, s);
    if (wg == 256 && ch == 256) return launch_fused_t<256, 256>(a, grid, s);
    if (wg == 512 && ch == 64) return launch_fused_t<512, 64>(a, grid, s);
    if (wg == 512 && ch == 128) return launch_fused_t<512, 128>(a, grid, s);
    if (wg == 512 && ch == 256) return launch_fused_t<512, 256>(a, grid, s);
    return hipErrorInvalidValue;
}

hipError_t launch_fixup(const FusedLaunch &f, hipStream_t s) {
    const FArgs a = make_args(f);
    int64_t blocks = (f.tiles_cap + 255) / 256;
    if (blocks < 1) blocks = 1;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fixup, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_batch_init(uint64_t *err, uint32_t *tile_counter, int64_t *d_n_kept,
                             hipStream_t s) {
    hipLaunchKernelGGL(k_batch_init, dim3(1), dim3(1), 0, s, err, tile_counter, d_n_kept);
    return hipGetLastError();
}

}  // namespace svt
