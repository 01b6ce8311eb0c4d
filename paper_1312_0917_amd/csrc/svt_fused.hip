// Persistent fused combine + fit + select kernel of libsvt, and its split-road fixup.
//
// The fit of section II is p_j = sum_l f[j][l] x_l + q_j followed by the fixed-point shift.
// Because the sum is linear in the hits, each hit's contribution f[j][l] * x_l (six int32 per
// hit, the "partial-product vector") is computed once per road and staged in LDS; every
// combination then costs five LDS vector reads and integer adds instead of thirty multiplies.
// The offset is split exactly as q = qh * 2^s + ql with 0 <= ql < 2^s: ql is folded into the
// layer-0 vectors, so the five-term sum stays inside int32, and
//     floor((S + q) / 2^s) = qh + floor((S + ql) / 2^s)       (exact for every integer S).
//
// Work distribution: combinations are numbered globally (road-major, combo_begin from the
// pre-pass); workgroups of a persistent grid take tiles of tile_combos consecutive
// combinations from an atomic counter.  A tile stages its roads in LDS in chunks of up to
// CHUNK roads (bounded by the LDS hit capacity), and each lane fits 4 consecutive
// combinations so that every record array is written with 16-byte coalesced stores.  Roads
// entirely inside a tile get their best track from LDS atomics; roads cut by tile boundaries
// leave partial (key, count) pairs per tile that the fixup kernel merges.
#include "svt_common.h"

namespace svt {
namespace {

constexpr int kHitCap = 1024;          // hits staged per chunk (a road has at most 5 * 8 = 40)
constexpr int kMaxKb = 16;             // kept-count blocks per tile (tile_combos <= 65536)
constexpr uint32_t kKMask = (1u << kKeyKBits) - 1;

struct FArgs {
    const svt_fconst *bank;
    int32_t shift;
    int32_t n_sets;
    int64_t cut;
    const uint32_t *words;
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

// Per-road data of the current chunk, in LDS (96 bytes).
struct alignas(16) RoadMeta {
    int32_t C;         // combinations
    uint32_t nh;       // packed hits per layer
    uint32_t mg[4];    // division magics for n1..n4 (0 when n == 1)
    int32_t base[5];   // LDS vector index of the first hit of each layer
    int32_t qh[6];     // offsets >> shift
    int32_t pad[7];
};
static_assert(sizeof(RoadMeta) == 96, "RoadMeta layout");

// floor(k / n) for 0 <= k < 2^15 and 1 <= n <= 8 with m = ceil(2^32 / n) (m = 0 for n = 1):
// k * (m * n - 2^32) < 2^15 * 8 < 2^32, so the high word of k * m is exact.
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t m) {
    return m ? __umulhi(k, m) : k;
}

__host__ __device__ constexpr uint32_t magic_of(uint32_t n) {
    return n <= 1 ? 0u : static_cast<uint32_t>((0x100000000ull + n - 1) / n);
}

struct Fit {
    int32_t v[6];
    int64_t chi2;
};

// Fit combination k of the road described by m, from the partial-product vectors P.
__device__ __forceinline__ Fit fit_combo(const RoadMeta &m, uint32_t k, const int2 *P,
                                         int32_t shift) {
    uint32_t h[5];
    uint32_t rest = k;
#pragma unroll
    for (int l = 4; l >= 1; --l) {
        const uint32_t n = nh_of(m.nh, l);
        const uint32_t q = div_small(rest, m.mg[l - 1]);
        h[l] = rest - q * n;
        rest = q;
    }
    h[0] = rest;
    int32_t a[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int l = 0; l < 5; ++l) {
        const int2 *v = P + 3 * (m.base[l] + static_cast<int32_t>(h[l]));
        const int2 x0 = v[0], x1 = v[1], x2 = v[2];
        a[0] += x0.x; a[1] += x0.y; a[2] += x1.x; a[3] += x1.y; a[4] += x2.x; a[5] += x2.y;
    }
    Fit f;
#pragma unroll
    for (int j = 0; j < 6; ++j) f.v[j] = (a[j] >> shift) + m.qh[j];
    f.chi2 = static_cast<int64_t>(f.v[3]) * f.v[3] + static_cast<int64_t>(f.v[4]) * f.v[4] +
             static_cast<int64_t>(f.v[5]) * f.v[5];
    return f;
}

template <int WG, int CHUNK>
__global__ __launch_bounds__(WG) void k_fused(FArgs a) {
    static_assert(CHUNK <= kWaveSize, "chunk roads are staged by one wave");
    __shared__ int2 P[3 * kHitCap];           // 6 int32 per staged hit
    __shared__ RoadMeta meta[CHUNK];
    __shared__ int32_t s_rb[CHUNK + 1];       // road begin relative to the tile start
    __shared__ unsigned long long s_key[CHUNK];
    __shared__ uint32_t s_nacc[CHUNK];
    __shared__ uint32_t s_kb[kMaxKb];
    __shared__ int64_t s_tile;
    __shared__ int32_t s_nr;

    if (has_error(a.err)) return;
    const int64_t n_roads = *a.d_n_roads;
    const int64_t n_combos = *a.d_n_combos;
    if (n_roads < 0 || n_roads > a.road_cap || n_combos < 0 || n_combos > a.combo_cap) return;
    const int64_t T = a.tile_combos;
    const int64_t n_tiles = (n_combos + T - 1) / T;
    if (n_tiles > a.tiles_cap) return;
    const int tid = threadIdx.x;
    const int wave = tid / kWaveSize;
    const int lane = tid % kWaveSize;
    const uint32_t qlmask = (1u << a.shift) - 1u;

    while (true) {
        if (tid == 0) s_tile = static_cast<int64_t>(atomicAdd(a.tile_counter, 1u));
        if (tid < kMaxKb) s_kb[tid] = 0;
        __syncthreads();
        const int64_t t = s_tile;
        if (t >= n_tiles) break;
        const int64_t tile_start = t * T;
        const int64_t tile_end = (tile_start + T < n_combos) ? tile_start + T : n_combos;
        const int32_t tile_len = static_cast<int32_t>(tile_end - tile_start);
        int64_t r_next = a.tile_first_road[t];

        while (true) {
            // ---- phase A (wave 0): chunk road table, hit grouping, partial-product vectors
            if (wave == 0) {
                const int64_t r = r_next + lane;
                bool valid = false;
                int64_t cb = 0, hb = 0;
                int32_t C = 0, s = 0;
                uint32_t nh = 0;
                if (lane < CHUNK && r < n_roads) {
                    cb = a.roads.combo_begin[r];
                    valid = cb < tile_end;
                    if (valid) {
                        C = a.roads.ncombo[r];
                        nh = a.roads.nhits[r];
                        hb = a.roads.hit_begin[r];
                        s = a.roads.set[r];
                    }
                }
                int32_t nhit = 0;
                if (valid && C > 0)
                    for (int l = 0; l < 5; ++l) nhit += static_cast<int32_t>(nh_of(nh, l));
                const int32_t incl = wave_incl_scan(nhit);
                const bool fits = valid && incl <= kHitCap;
                const int nr = __popcll(__ballot(fits));
                if (lane < nr) {
                    RoadMeta m;
                    m.C = C;
                    m.nh = nh;
                    int32_t base = incl - nhit;
#pragma unroll
                    for (int l = 0; l < 5; ++l) {
                        m.base[l] = base;
                        base += static_cast<int32_t>(nh_of(nh, l));
                    }
#pragma unroll
                    for (int l = 1; l < 5; ++l) m.mg[l - 1] = magic_of(nh_of(nh, l));
                    const svt_fconst *F = a.bank + s;
                    int32_t ql[6];
#pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        const int32_t q = F->q[j];
                        m.qh[j] = q >> a.shift;
                        ql[j] = static_cast<int32_t>(static_cast<uint32_t>(q) & qlmask);
                    }
                    meta[lane] = m;
                    s_rb[lane] = static_cast<int32_t>(cb - tile_start);
                    s_key[lane] = ~0ull;
                    s_nacc[lane] = 0;
                    // group the road's hits by layer (stream order kept) and stage f.x
                    uint64_t seen = 0;  // 8 bits per layer (5 layers: 40 bits)
                    for (int32_t i = 0; i < nhit; ++i) {
                        const uint32_t w = a.words[hb + i];
                        const uint32_t l = w_layer(w);
                        if (l >= 5) continue;  // excluded by the layer check of the pre-pass
                        const int32_t x = w_coord(w);
                        int32_t pos = 0;
#pragma unroll
                        for (int ll = 0; ll < 5; ++ll)
                            if (static_cast<uint32_t>(ll) == l) pos = m.base[ll];
                        pos += static_cast<int32_t>((seen >> (8 * l)) & 0xFF);
                        seen += 1ull << (8 * l);
                        if (pos >= kHitCap) continue;
                        const int16_t *fc = &F->f[0][0] + l;  // column l: stride 5
                        int32_t v[6];
#pragma unroll
                        for (int j = 0; j < 6; ++j)
                            v[j] = static_cast<int32_t>(fc[5 * j]) * x + (l == 0 ? ql[j] : 0);
                        int2 *dst = P + 3 * pos;
                        dst[0] = make_int2(v[0], v[1]);
                        dst[1] = make_int2(v[2], v[3]);
                        dst[2] = make_int2(v[4], v[5]);
                    }
                }
                if (lane == 0) {
                    s_nr = nr;
                    // sentinel: end of the last staged road
                    s_rb[nr] = 0x7FFFFFFF;
                }
            }
            __syncthreads();
            const int nr = s_nr;
            if (nr == 0) break;

            // ---- phase B (all waves): fit every combination of the chunk inside the tile
            const int32_t first_rb = s_rb[0];
            const int32_t last_end = s_rb[nr - 1] + meta[nr - 1].C;
            const int32_t cs = first_rb > 0 ? first_rb : 0;
            const int32_t ce = last_end < tile_len ? last_end : tile_len;
            const int32_t g_lo = cs >> 2, g_hi = (ce + 3) >> 2;
            for (int32_t g = g_lo + tid; g < g_hi; g += WG) {
                const int32_t rel0 = g << 2;
                const int32_t first = rel0 > cs ? rel0 : cs;
                // last staged road whose begin <= first
                int ri = 0;
#pragma unroll
                for (int step = CHUNK / 2; step > 0; step >>= 1)
                    if (ri + step < nr && s_rb[ri + step] <= first) ri += step;
                RoadMeta m = meta[ri];
                int32_t k = first - s_rb[ri];
                int32_t vp0[4], vp1[4], vp2[4], vc0[4], vc1[4], vc2[4];
                int64_t vchi[4];
                uint32_t acc_bits = 0, valid_bits = 0;
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int32_t rel = rel0 + e;
                    vp0[e] = vp1[e] = vp2[e] = vc0[e] = vc1[e] = vc2[e] = 0;
                    vchi[e] = 0;
                    if (rel >= cs && rel < ce) {
                        while (k >= m.C && ri + 1 < nr) {  // bounded: never past the chunk
                            k -= m.C;
                            ++ri;
                            m = meta[ri];
                        }
                        const Fit f = fit_combo(m, static_cast<uint32_t>(k), P, a.shift);
                        vp0[e] = f.v[0]; vp1[e] = f.v[1]; vp2[e] = f.v[2];
                        vc0[e] = f.v[3]; vc1[e] = f.v[4]; vc2[e] = f.v[5];
                        vchi[e] = f.chi2;
                        valid_bits |= 1u << e;
                        if (f.chi2 <= a.cut) {
                            acc_bits |= 1u << e;
                            const unsigned long long key =
                                best_key(f.chi2, static_cast<uint32_t>(k));
                            atomicMin(&s_key[ri], key);
                            atomicAdd(&s_nacc[ri], 1u);
                            atomicAdd(&s_kb[rel >> 12], 1u);
                        }
                        ++k;
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

            // ---- phase C (wave 0): best track of roads inside the tile, partials otherwise
            if (wave == 0 && lane < nr) {
                const RoadMeta m = meta[lane];
                const int32_t rb = s_rb[lane];
                const int64_t r = r_next + lane;
                if (m.C > 0) {
                    const unsigned long long key = s_key[lane];
                    const uint32_t nacc = s_nacc[lane];
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
                                const Fit f = fit_combo(m, static_cast<uint32_t>(k), P, a.shift);
                                if (f.chi2 <= a.cut && static_cast<uint64_t>(f.chi2) < bchi) {
                                    bchi = static_cast<uint64_t>(f.chi2);
                                    bk = static_cast<uint32_t>(k);
                                }
                            }
                        }
                    }
                    if (rb >= 0 && rb + m.C <= tile_len) {
                        a.best.n_accept[r] = static_cast<int32_t>(nacc);
                        if (bchi == ~0ull) {
                            a.best.k[r] = -1;
                            a.best.p0[r] = INT32_MIN;
                            a.best.p1[r] = INT32_MIN;
                            a.best.p2[r] = INT32_MIN;
                            a.best.chi2[r] = INT64_MAX;
                        } else {
                            const Fit f = fit_combo(m, bk, P, a.shift);
                            a.best.k[r] = static_cast<int32_t>(bk);
                            a.best.p0[r] = f.v[0];
                            a.best.p1[r] = f.v[1];
                            a.best.p2[r] = f.v[2];
                            a.best.chi2[r] = static_cast<int64_t>(bchi);
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
        __syncthreads();
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
    a.words = f.words;
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
    const bool ch_ok = t.chunk_roads == 16 || t.chunk_roads == 32 || t.chunk_roads == 64;
    const bool tile_ok = t.tile_combos >= kKeptBlock && t.tile_combos <= kKeptBlock * kMaxKb &&
                         t.tile_combos % kKeptBlock == 0;
    const bool occ_ok = t.wgs_per_cu >= 1 && t.wgs_per_cu <= 8;
    return wg_ok && ch_ok && tile_ok && occ_ok;
}

hipError_t launch_fused(const FusedLaunch &f, hipStream_t s) {
    const FArgs a = make_args(f);
    const int grid = f.num_cus * f.tune.wgs_per_cu;
    const int wg = f.tune.wg_size, ch = f.tune.chunk_roads;
    if (wg == 256 && ch == 16) return launch_fused_t<256, 16>(a, grid, s);
    if (wg == 256 && ch == 32) return launch_fused_t<256, 32>(a, grid, s);
    if (wg == 256 && ch == 64) return launch_fused_t<256, 64>(a, grid, s);
    if (wg == 512 && ch == 16) return launch_fused_t<512, 16>(a, grid, s);
    if (wg == 512 && ch == 32) return launch_fused_t<512, 32>(a, grid, s);
    if (wg == 512 && ch == 64) return launch_fused_t<512, 64>(a, grid, s);
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
