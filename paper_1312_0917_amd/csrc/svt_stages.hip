// Stage kernels of libsvt: unpack (segment, emit, road fill), combine (count, scan, list),
// plain fit (one lane per listed combination), select (cut, best track, kept list).
//
// Section II-A of the paper splits the serial code into unpack / combine / fit; these are the
// one-launch-per-stage GPU forms of those functions, kept simple: they are the baseline the
// fused persistent pass is compared with and share none of its code beyond the field
// decoders and scans in svt_common.h.
#include "svt_common.h"

namespace svt {
namespace {

__global__ void k_init_err(uint64_t *err) { *err = SVT_NO_ERROR; }

// ---- unpack 1: per 4096-word block, count road starts and event starts ------------------
// A new event starts where the event tag changes, a new road where either tag changes.
__global__ __launch_bounds__(kSegThreads) void k_seg_count(const uint32_t *__restrict__ words,
                                                           Sizes n_words_s, int32_t n_layers,
                                                           int64_t *wb_counts, int64_t nb_stride,
                                                           uint64_t *err) {
    __shared__ int64_t tmp[kSegThreads / kWaveSize + 1];
    const int64_t n = load_size(n_words_s);
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_words_s.dev && *n_words_s.dev > n_words_s.cap)
        report(err, SVT_ERRCLASS_CAPACITY, 3);
    const int64_t nb = (n + kSegBlockWords - 1) / kSegBlockWords;
    const bool aligned = (reinterpret_cast<uintptr_t>(words) & 15) == 0;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t base =
            b * kSegBlockWords + static_cast<int64_t>(threadIdx.x) * kSegWordsPerThread;
        uint32_t w[kSegWordsPerThread];
        if (aligned && base + kSegWordsPerThread <= n) {
            const uint4 *p = reinterpret_cast<const uint4 *>(words + base);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                uint4 t = p[v];
                w[4 * v] = t.x; w[4 * v + 1] = t.y; w[4 * v + 2] = t.z; w[4 * v + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int e = 0; e < kSegWordsPerThread; ++e)
                w[e] = (base + e < n) ? words[base + e] : 0u;
        }
        uint32_t prev = (base > 0 && base <= n) ? words[base - 1] : 0u;
        int64_t nr = 0, ne = 0;
        int64_t bad = -1;
#pragma unroll
        for (int e = 0; e < kSegWordsPerThread; ++e) {
            const int64_t i = base + e;
            if (i < n) {
                const uint32_t x = w[e];
                const bool first = (i == 0);
                nr += (first || w_tags(x) != w_tags(prev)) ? 1 : 0;
                ne += (first || w_etag(x) != w_etag(prev)) ? 1 : 0;
                if (bad < 0 && static_cast<int32_t>(w_layer(x)) >= n_layers) bad = i;
                prev = x;
            }
        }
        if (bad >= 0) report(err, SVT_ERRCLASS_LAYER, static_cast<uint64_t>(bad));
        const int64_t br = block_sum<int64_t, kSegThreads>(nr, tmp);
        const int64_t be = block_sum<int64_t, kSegThreads>(ne, tmp);
        if (threadIdx.x == 0) {
            wb_counts[b] = br;
            wb_counts[nb_stride + b] = be;
        }
    }
}

// ---- single-workgroup in-place exclusive scan ---------------------------------------------
// Exclusive scan of col[0 .. n) in place by one workgroup of NT threads; the total goes to *tot
// (nullable).  tmp holds NT / 64 + 1 values.
template <int NT>
__device__ int64_t scan_column(int64_t *col, int64_t n, int64_t *tot, int64_t *tmp) {
    constexpr int kItems = 4;
    int64_t carry = 0;
    for (int64_t base = 0; base < n; base += static_cast<int64_t>(NT) * kItems) {
        const int64_t i0 = base + static_cast<int64_t>(threadIdx.x) * kItems;
        int64_t v[kItems];
        int64_t s = 0;
#pragma unroll
        for (int e = 0; e < kItems; ++e) {
            v[e] = (i0 + e < n) ? col[i0 + e] : 0;
            s += v[e];
        }
        int64_t total;
        int64_t ex = block_excl_scan<int64_t, NT>(s, tmp, total);
        int64_t run = carry + ex;
#pragma unroll
        for (int e = 0; e < kItems; ++e) {
            if (i0 + e < n) col[i0 + e] = run;
            run += v[e];
        }
        carry += total;
    }
    if (threadIdx.x == 0 && tot) *tot = carry;
    return carry;
}

// One workgroup per column; column 0's total is checked against cap0 (class CAPACITY, index
// cap_index) when cap0 >= 0.
__global__ __launch_bounds__(kScanThreads) void k_scan(int64_t *data, int64_t col_stride,
                                                       Sizes n_s, int64_t div, int64_t *tot0,
                                                       int64_t *tot1, int64_t cap0,
                                                       uint32_t cap_index, uint64_t *err,
                                                       int32_t skip_if_error) {
    __shared__ int64_t tmp[kScanThreads / kWaveSize + 1];
    int64_t *tot = blockIdx.x == 0 ? tot0 : tot1;
    if (skip_if_error && has_error(err)) {
        if (threadIdx.x == 0 && tot) *tot = -1;
        return;
    }
    const int64_t n = (load_size(n_s) + div - 1) / div;
    const int64_t carry = scan_column<kScanThreads>(data + blockIdx.x * col_stride, n, tot, tmp);
    if (threadIdx.x == 0 && blockIdx.x == 0 && cap0 >= 0 && carry > cap0)
        report(err, SVT_ERRCLASS_CAPACITY, cap_index);
}

// ---- unpack 2: write each road's first word, tag and event ordinal -----------------------
__global__ __launch_bounds__(kSegThreads) void k_seg_emit(const uint32_t *__restrict__ words,
                                                          Sizes n_words_s,
                                                          const int64_t *__restrict__ wb_prefix,
                                                          int64_t nb_stride, svt_roads roads,
                                                          int64_t road_cap, uint64_t *err) {
    __shared__ int64_t tmp[kSegThreads / kWaveSize + 1];
    if (has_error(err)) return;
    const int64_t n = load_size(n_words_s);
    const int64_t nb = (n + kSegBlockWords - 1) / kSegBlockWords;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t base =
            b * kSegBlockWords + static_cast<int64_t>(threadIdx.x) * kSegWordsPerThread;
        uint32_t w[kSegWordsPerThread];
#pragma unroll
        for (int e = 0; e < kSegWordsPerThread; ++e) w[e] = (base + e < n) ? words[base + e] : 0u;
        const uint32_t prev0 = (base > 0 && base <= n) ? words[base - 1] : 0u;
        uint32_t flags = 0;  // bit 2e: new road, bit 2e+1: new event
        int64_t nr = 0, ne = 0;
        uint32_t prev = prev0;
#pragma unroll
        for (int e = 0; e < kSegWordsPerThread; ++e) {
            const int64_t i = base + e;
            if (i < n) {
                const bool first = (i == 0);
                const bool r = first || w_tags(w[e]) != w_tags(prev);
                const bool v = first || w_etag(w[e]) != w_etag(prev);
                flags |= (r ? 1u : 0u) << (2 * e);
                flags |= (v ? 1u : 0u) << (2 * e + 1);
                nr += r;
                ne += v;
                prev = w[e];
            }
        }
        int64_t tr, te;
        int64_t rc = block_excl_scan<int64_t, kSegThreads>(nr, tmp, tr) + wb_prefix[b];
        int64_t ec = block_excl_scan<int64_t, kSegThreads>(ne, tmp, te) + wb_prefix[nb_stride + b];
#pragma unroll
        for (int e = 0; e < kSegWordsPerThread; ++e) {
            const int64_t i = base + e;
            if (i < n) {
                if (flags & (2u << (2 * e))) ++ec;
                if (flags & (1u << (2 * e))) {
                    const int64_t r = rc++;
                    if (r < road_cap) {
                        roads.hit_begin[r] = i;
                        roads.set[r] = static_cast<int32_t>(w_rtag(w[e]));
                        roads.event[r] = static_cast<int32_t>(ec - 1);
                    }
                }
            }
        }
    }
}

// ---- unpack 3: per road, count hits per layer, check, regroup coordinates by layer -------
__global__ __launch_bounds__(kRoadBlock) void k_road_fill(const uint32_t *__restrict__ words,
                                                          Sizes n_words_s,
                                                          const int64_t *d_n_roads,
                                                          int64_t road_cap, svt_roads roads,
                                                          svt_config cfg, int16_t *hit_coord,
                                                          uint64_t *err) {
    if (has_error(err)) return;
    const int64_t n = load_size(n_words_s);
    const int64_t nr_all = *d_n_roads;
    if (nr_all > road_cap || nr_all < 0) return;  // capacity error already reported
    const int64_t nr = nr_all;
    const int64_t max_len = static_cast<int64_t>(cfg.n_layers) * cfg.max_hits;
    for (int64_t r = gtid(); r < nr; r += gstride()) {
        const int64_t b = roads.hit_begin[r];
        const int64_t e = (r + 1 < nr_all) ? roads.hit_begin[r + 1] : n;
        const int64_t len = e - b;
        if (len <= 0 || len > max_len || b < 0 || e > n) {
            report(err, SVT_ERRCLASS_HITS, static_cast<uint64_t>(r));
            continue;
        }
        uint64_t cnt = 0;  // 8 bits per layer
        for (int64_t i = b; i < e; ++i) {
            const uint32_t l = w_layer(words[i]);
            if (l < SVT_N_LAYERS) cnt += 1ull << (8 * l);
        }
        bool over = false;
        uint32_t packed = 0;
        for (int l = 0; l < SVT_N_LAYERS; ++l) {
            const uint32_t c = static_cast<uint32_t>((cnt >> (8 * l)) & 0xFF);
            over |= c > static_cast<uint32_t>(cfg.max_hits);
            packed |= (c & 0xFu) << (4 * l);
        }
        if (over) {
            report(err, SVT_ERRCLASS_HITS, static_cast<uint64_t>(r));
            continue;
        }
        if (static_cast<uint32_t>(roads.set[r]) >= static_cast<uint32_t>(cfg.n_sets))
            report(err, SVT_ERRCLASS_SET, static_cast<uint64_t>(r));
        roads.nhits[r] = packed;
        if (hit_coord) {
            uint32_t off[SVT_N_LAYERS];
            uint32_t run = 0;
            for (int l = 0; l < SVT_N_LAYERS; ++l) {
                off[l] = run;
                run += nh_of(packed, l);
            }
            for (int64_t i = b; i < e; ++i) {
                const uint32_t w = words[i];
                const uint32_t l = w_layer(w);
                if (l >= SVT_N_LAYERS) continue;
                uint32_t o = 0;
                // select off[l] without dynamic register indexing
                for (int k = 0; k < SVT_N_LAYERS; ++k)
                    if (static_cast<uint32_t>(k) == l) { o = off[k]; off[k] = o + 1; }
                hit_coord[b + o] = static_cast<int16_t>(w_coord(w));
            }
        }
    }
}

// ---- combine 1: combinations per road and per-block sums ---------------------------------
__global__ __launch_bounds__(kRoadBlock) void k_combo_count(svt_roads roads, Sizes n_roads_s,
                                                            int64_t *rb_sums, uint64_t *err) {
    __shared__ int64_t tmp[kRoadBlock / kWaveSize + 1];
    if (has_error(err)) return;
    const int64_t nr = load_size(n_roads_s);
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRoadBlock + threadIdx.x;
    if (static_cast<int64_t>(blockIdx.x) * kRoadBlock >= nr) return;
    int64_t c = 0;
    if (r < nr) {
        const uint32_t p = roads.nhits[r];
        c = 1;
        for (int l = 0; l < SVT_N_LAYERS; ++l) c *= nh_of(p, l);
        roads.ncombo[r] = static_cast<int32_t>(c);
    }
    const int64_t s = block_sum<int64_t, kRoadBlock>(c, tmp);
    if (threadIdx.x == 0) rb_sums[blockIdx.x] = s;
}

// ---- combine 2: combo_begin, tile marks, defaults of roads without combinations ----------
__global__ __launch_bounds__(kRoadBlock) void k_combo_begin(svt_roads roads, Sizes n_roads_s,
                                                            const int64_t *rb_prefix,
                                                            int64_t tile_combos,
                                                            int32_t *tile_first_road,
                                                            int64_t tiles_cap, svt_best best,
                                                            int32_t init_best,
                                                            uint64_t *err) {
    __shared__ int64_t tmp[kRoadBlock / kWaveSize + 1];
    if (has_error(err)) return;
    const int64_t nr = load_size(n_roads_s);
    if (static_cast<int64_t>(blockIdx.x) * kRoadBlock >= nr) return;
    const int64_t r = static_cast<int64_t>(blockIdx.x) * kRoadBlock + threadIdx.x;
    const int64_t c = (r < nr) ? roads.ncombo[r] : 0;
    int64_t tot;
    const int64_t begin = block_excl_scan<int64_t, kRoadBlock>(c, tmp, tot) + rb_prefix[blockIdx.x];
    if (r >= nr) return;
    roads.combo_begin[r] = begin;
    if (tile_combos > 0 && c > 0) {
        // this road holds the first combination of every tile that starts inside it
        for (int64_t t = (begin + tile_combos - 1) / tile_combos; t * tile_combos < begin + c; ++t)
            if (t < tiles_cap) tile_first_road[t] = static_cast<int32_t>(r);
    }
    if (init_best) {  // best-track key "none" (all ones) and no accepted combination yet
        reinterpret_cast<uint64_t *>(best.chi2)[r] = UINT64_MAX;
        best.n_accept[r] = 0;
    }
}

// ---- combine 3 (plain path): list every combination --------------------------------------
__global__ __launch_bounds__(kRoadBlock) void k_materialize(svt_roads roads, int64_t n_roads,
                                                            const int64_t *d_n_combos,
                                                            int64_t combo_cap,
                                                            int32_t *combo_road,
                                                            uint32_t *combo_hits,
                                                            uint64_t *err) {
    __shared__ int64_t s_begin[kRoadBlock + 1];
    __shared__ uint32_t s_nh[kRoadBlock];
    if (has_error(err)) return;
    const int64_t total = *d_n_combos;
    if (total > combo_cap) return;
    const int64_t r0 = static_cast<int64_t>(blockIdx.x) * kRoadBlock;
    if (r0 >= n_roads) return;
    const int nloc = static_cast<int>((n_roads - r0) < kRoadBlock ? (n_roads - r0) : kRoadBlock);
    if (threadIdx.x < nloc) {
        s_begin[threadIdx.x] = roads.combo_begin[r0 + threadIdx.x];
        s_nh[threadIdx.x] = roads.nhits[r0 + threadIdx.x];
    }
    if (threadIdx.x == 0) {
        const int64_t rl = r0 + nloc - 1;
        s_begin[nloc] = roads.combo_begin[rl] + roads.ncombo[rl];
    }
    __syncthreads();
    const int64_t c_lo = s_begin[0], c_hi = s_begin[nloc];
    for (int64_t c = c_lo + threadIdx.x; c < c_hi; c += kRoadBlock) {
        int lo = 0, hi = nloc - 1;  // last road with begin <= c
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_begin[mid] <= c) lo = mid; else hi = mid - 1;
        }
        uint32_t k = static_cast<uint32_t>(c - s_begin[lo]);
        const uint32_t p = s_nh[lo];
        uint32_t h[SVT_N_LAYERS];
        for (int l = SVT_N_LAYERS - 1; l >= 0; --l) {  // layer 0 most significant
            const uint32_t nl = nh_of(p, l);
            h[l] = k % nl;
            k /= nl;
        }
        uint32_t packed = 0;
        for (int l = 0; l < SVT_N_LAYERS; ++l) packed |= h[l] << (4 * l);
        if (combo_road) combo_road[c] = static_cast<int32_t>(r0 + lo);
        if (combo_hits) combo_hits[c] = packed;
    }
}

// ---- plain fit: one lane per listed combination, 64-bit accumulation -----------------------
__global__ __launch_bounds__(256) void k_fit_plain(const svt_fconst *__restrict__ bank,
                                                   svt_config cfg, svt_roads roads,
                                                   int64_t n_roads,
                                                   const int16_t *__restrict__ hit_coord,
                                                   int64_t n_hits,
                                                   const int32_t *__restrict__ combo_road,
                                                   const uint32_t *__restrict__ combo_hits,
                                                   int64_t n_combos, svt_fitrec out,
                                                   uint64_t *err) {
    for (int64_t i = gtid(); i < n_combos; i += gstride()) {
        const int32_t r = combo_road[i];
        if (r < 0 || r >= n_roads) { report(err, SVT_ERRCLASS_INDEX, i); continue; }
        const uint32_t ph = combo_hits[i];
        const uint32_t pn = roads.nhits[r];
        const int64_t hb = roads.hit_begin[r];
        const int32_t s = roads.set[r];
        bool ok = (s >= 0 && s < cfg.n_sets);
        int32_t x[SVT_N_LAYERS];
        int64_t off = hb;
        for (int l = 0; l < SVT_N_LAYERS; ++l) {
            const uint32_t d = (ph >> (4 * l)) & 0xFu;
            const uint32_t nl = nh_of(pn, l);
            const int64_t idx = off + d;
            ok &= (d < nl) && idx >= 0 && idx < n_hits;
            x[l] = ok ? hit_coord[idx] : 0;
            off += nl;
        }
        if (!ok) { report(err, SVT_ERRCLASS_INDEX, i); continue; }
        const svt_fconst &F = bank[s];
        int32_t v[6];
        for (int j = 0; j < 6; ++j) {
            int64_t a = 0;
            for (int l = 0; l < SVT_N_LAYERS; ++l)
                a += static_cast<int64_t>(F.f[j][l]) * static_cast<int64_t>(x[l]);
            a += static_cast<int64_t>(F.q[j]);
            v[j] = static_cast<int32_t>(a >> cfg.shift);  // arithmetic shift = floor
        }
        const int64_t chi2 = static_cast<int64_t>(v[3]) * v[3] +
                             static_cast<int64_t>(v[4]) * v[4] +
                             static_cast<int64_t>(v[5]) * v[5];
        out.p0[i] = v[0];
        out.p1[i] = v[1];
        out.p2[i] = v[2];
        out.chi2[i] = chi2;
        if (out.c0) out.c0[i] = v[3];
        if (out.c1) out.c1[i] = v[4];
        if (out.c2) out.c2[i] = v[5];
    }
}

// ---- select: cut, per-road best key (chi2 << 15 | k) and counts, kept-block counts -------
__global__ void k_best_init(svt_best best, int64_t n_roads) {
    for (int64_t r = gtid(); r < n_roads; r += gstride()) {
        reinterpret_cast<uint64_t *>(best.chi2)[r] = UINT64_MAX;
        best.n_accept[r] = 0;
    }
}

__global__ __launch_bounds__(kSegThreads) void k_select_mark(svt_config cfg, svt_roads roads,
                                                             int64_t n_roads,
                                                             const int32_t *__restrict__ combo_road,
                                                             const int64_t *__restrict__ chi2,
                                                             int64_t n_combos, uint8_t *accept,
                                                             svt_best best, int64_t *kb_counts,
                                                             uint64_t *err) {
    __shared__ int64_t tmp[kSegThreads / kWaveSize + 1];
    const int64_t nb = (n_combos + kKeptBlock - 1) / kKeptBlock;
    uint64_t *key = reinterpret_cast<uint64_t *>(best.chi2);
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t base = b * kKeptBlock + static_cast<int64_t>(threadIdx.x) * 16;
        int64_t cnt = 0;
        for (int e = 0; e < 16; ++e) {
            const int64_t i = base + e;
            if (i >= n_combos) break;
            const int64_t c2 = chi2[i];
            const bool acc = c2 <= cfg.chi2_cut;
            accept[i] = acc ? 1 : 0;
            if (acc) {
                ++cnt;
                const int32_t r = combo_road[i];
                if (r < 0 || r >= n_roads) { report(err, SVT_ERRCLASS_INDEX, i); continue; }
                const int64_t k = i - roads.combo_begin[r];
                if (k < 0 || k >= (1 << kKeyKBits) || c2 < 0) {
                    report(err, SVT_ERRCLASS_INDEX, i);
                    continue;
                }
                const uint64_t kv = best_key(c2, static_cast<uint32_t>(k));
                atomicMin(reinterpret_cast<unsigned long long *>(key + r), kv);
                atomicAdd(best.n_accept + r, 1);
            }
        }
        const int64_t s = block_sum<int64_t, kSegThreads>(cnt, tmp);
        if (threadIdx.x == 0 && kb_counts) kb_counts[b] = s;
    }
}

// Parameters of combination k of road r, fitted again from the grouped coordinates and the
// road's constant set (the same integer arithmetic as the records, so the same values).
__device__ inline int64_t refit_combo(const svt_fconst *__restrict__ bank,
                                     const int16_t *__restrict__ coords, int32_t shift,
                                     uint32_t nh, int64_t hb, int32_t set, uint32_t k, int32_t *v,
                                     int rows) {
    uint32_t h[SVT_N_LAYERS];
#pragma unroll
    for (int l = SVT_N_LAYERS - 1; l >= 0; --l) {  // layer 0 most significant
        const uint32_t nl = nh_of(nh, l);
        h[l] = k % nl;
        k /= nl;
    }
    int64_t off = hb;
    int32_t x[SVT_N_LAYERS];
#pragma unroll
    for (int l = 0; l < SVT_N_LAYERS; ++l) {
        x[l] = coords[off + h[l]];
        off += nh_of(nh, l);
    }
    const svt_fconst &F = bank[set];
    for (int j = 0; j < rows; ++j) {
        int64_t acc = F.q[j];
#pragma unroll
        for (int l = 0; l < SVT_N_LAYERS; ++l)
            acc += static_cast<int64_t>(F.f[j][l]) * static_cast<int64_t>(x[l]);
        v[j] = static_cast<int32_t>(acc >> shift);
    }
    if (rows < 6) return 0;
    return static_cast<int64_t>(v[3]) * v[3] + static_cast<int64_t>(v[4]) * v[4] +
           static_cast<int64_t>(v[5]) * v[5];
}

// With bank and coords (batched path), the best track's parameters are fitted again from its
// hits instead of gathered from the three record arrays: one coordinate line per road instead
// of three scattered reads.
// With a scan job (job.data non-null), the grid's last block does that scan instead of roads:
// the kept list's per-block counts, in the same launch (it reads nothing the roads write).
__global__ __launch_bounds__(256) void k_best_finalize(svt_roads roads, Sizes n_roads_s,
                                                       svt_fitrec rec, Sizes n_combos_s,
                                                       svt_best best, int64_t cut, uint64_t *err,
                                                       int32_t skip_if_error,
                                                       const svt_fconst *bank,
                                                       const int16_t *coords, int32_t shift,
                                                       ScanJob job) {
    const int64_t road_blocks = job.data ? gridDim.x - 1 : gridDim.x;
    if (job.data && blockIdx.x == road_blocks) {
        __shared__ int64_t tmp[256 / kWaveSize + 1];
        if (skip_if_error && has_error(err)) {
            if (threadIdx.x == 0 && job.tot) *job.tot = -1;
            return;
        }
        const int64_t n = (load_size(job.n) + job.div - 1) / job.div;
        const int64_t carry = scan_column<256>(job.data, n, job.tot, tmp);
        if (threadIdx.x == 0 && job.cap >= 0 && carry > job.cap)
            report(err, SVT_ERRCLASS_CAPACITY, job.cap_index);
        return;
    }
    if (skip_if_error && has_error(err)) return;
    const int64_t n_roads = load_size(n_roads_s);
    const int64_t n_combos = load_size(n_combos_s);
    const int64_t stride = road_blocks * blockDim.x;
    for (int64_t r = gtid(); r < n_roads; r += stride) {
        uint64_t key = reinterpret_cast<uint64_t *>(best.chi2)[r];
        const int64_t cb = roads.combo_begin[r];
        const int64_t nc = roads.ncombo[r];
        if (key != UINT64_MAX && (key >> kKeyKBits) == kKeyChiMax && cb >= 0 &&
            nc <= (1 << kKeyKBits)) {
            // saturated key: exact scan of the road's records (chi2 >= 2^49 - 1 only)
            uint64_t bchi = UINT64_MAX;
            int64_t bk = 0;
            for (int64_t k = 0; k < nc && cb + k < n_combos; ++k) {
                int32_t vv[6];
                const int64_t c2 = rec.chi2 ? rec.chi2[cb + k]
                                            : refit_combo(bank, coords, shift, roads.nhits[r],
                                                          roads.hit_begin[r], roads.set[r],
                                                          static_cast<uint32_t>(k), vv, 6);
                if (c2 <= cut && c2 >= 0 && static_cast<uint64_t>(c2) < bchi) {
                    bchi = static_cast<uint64_t>(c2);
                    bk = k;
                }
            }
            if (bchi != UINT64_MAX) {
                const int64_t g = cb + bk;
                best.k[r] = static_cast<int32_t>(bk);
                best.chi2[r] = static_cast<int64_t>(bchi);
                if (rec.p0) {
                    best.p0[r] = rec.p0[g];
                    best.p1[r] = rec.p1[g];
                    best.p2[r] = rec.p2[g];
                } else {
                    int32_t vv[6];
                    refit_combo(bank, coords, shift, roads.nhits[r], roads.hit_begin[r],
                                roads.set[r], static_cast<uint32_t>(bk), vv, 3);
                    best.p0[r] = vv[0];
                    best.p1[r] = vv[1];
                    best.p2[r] = vv[2];
                }
                continue;
            }
            key = UINT64_MAX;
        }
        if (key == UINT64_MAX) {
            best.k[r] = -1;
            best.p0[r] = INT32_MIN;
            best.p1[r] = INT32_MIN;
            best.p2[r] = INT32_MIN;
            best.chi2[r] = INT64_MAX;
        } else {
            const int32_t k = static_cast<int32_t>(key & ((1u << kKeyKBits) - 1));
            const int64_t g = cb + k;
            best.k[r] = k;
            best.chi2[r] = static_cast<int64_t>(key >> kKeyKBits);
            const bool in = g >= 0 && g < n_combos && k < nc;
            if (bank && coords && in) {
                int32_t p[6];
                refit_combo(bank, coords, shift, roads.nhits[r], roads.hit_begin[r],
                            roads.set[r], static_cast<uint32_t>(k), p, 3);
                best.p0[r] = p[0];
                best.p1[r] = p[1];
                best.p2[r] = p[2];
            } else {
                best.p0[r] = in ? rec.p0[g] : INT32_MIN;
                best.p1[r] = in ? rec.p1[g] : INT32_MIN;
                best.p2[r] = in ? rec.p2[g] : INT32_MIN;
            }
        }
    }
}

// Accept flags of combinations base .. base + 15 as a bit mask (one 16-byte load when aligned).
__device__ inline uint32_t accept_bits16(const uint8_t *__restrict__ accept, int64_t base,
                                         int64_t n) {
    uint32_t bits = 0;
    if (base + 16 <= n && (reinterpret_cast<uintptr_t>(accept + base) & 15) == 0) {
        const uint4 v = *reinterpret_cast<const uint4 *>(accept + base);
        const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int c = 0; c < 4; ++c)
                bits |= ((w[q] >> (8 * c)) & 0xFFu) ? (1u << (4 * q + c)) : 0u;
    } else {
        for (int e = 0; e < 16; ++e) {
            const int64_t i = base + e;
            if (i < n && accept[i]) bits |= 1u << e;
        }
    }
    return bits;
}

// ---- kept list: ascending indices of accepted combinations -------------------------------
__global__ __launch_bounds__(kSegThreads) void k_kept_write(const uint8_t *__restrict__ accept,
                                                            Sizes n_s,
                                                            const int64_t *__restrict__ kb_prefix,
                                                            int64_t *kept, int64_t kept_cap,
                                                            uint64_t *err) {
    __shared__ int64_t tmp[kSegThreads / kWaveSize + 1];
    const int64_t n = load_size(n_s);
    const int64_t nb = (n + kKeptBlock - 1) / kKeptBlock;
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const int64_t base = b * kKeptBlock + static_cast<int64_t>(threadIdx.x) * 16;
        uint32_t bits = accept_bits16(accept, base, n);
        int64_t tot;
        int64_t pos = block_excl_scan<int64_t, kSegThreads>(__popc(bits), tmp, tot) + kb_prefix[b];
        while (bits) {
            const int e = __ffs(bits) - 1;
            bits &= bits - 1;
            if (pos < kept_cap) kept[pos] = base + e;
            ++pos;
        }
    }
    (void)err;
}

// Kept-only mode: per block of kKeptBlock combinations, the accepted ones in ascending order.
// One wave per block (lane i reads the flags of combinations 64 i .. 64 i + 63 of the block), so
// that many blocks are in flight at once: the work per block is a short chain of dependent
// reads.  The block's accepted offsets are compacted in LDS and then spread evenly over the
// lanes.  The
// block's roads lie between the first road of its fit tile and the first road of the next tile;
// their combo_begin values are staged in the wave's LDS slice (up to kKeptRoads of them, else
// searched in place), each accepted combination finds its road by binary search and is fitted
// again from the grouped coordinates.
constexpr int kKeptRoads = 512;
__global__ __launch_bounds__(kSegThreads) void k_kept_refit(
    const uint8_t *__restrict__ accept, Sizes n_s, Sizes nr_s,
    const int64_t *__restrict__ kb_prefix, svt_roads roads,
    const int32_t *__restrict__ tile_first_road, int64_t tile_combos,
    const svt_fconst *__restrict__ bank, int32_t n_sets, const int16_t *__restrict__ coords,
    int32_t shift, int64_t *kept, svt_fitrec rec, int64_t kept_cap, uint64_t *err) {
    constexpr int kWaves = kSegThreads / kWaveSize;
    // After a data or capacity error the accept flags, the tile marks and the road table are
    // not (all) written: nothing here may be read.
    if (has_error(err)) return;
    __shared__ int64_t s_cb[kWaves][kKeptRoads];
    __shared__ uint16_t s_acc[kWaves][kKeptBlock];  // accepted offsets inside the block, in order
    const int wv = threadIdx.x / kWaveSize;
    const int lane = lane_id();
    const int64_t n = load_size(n_s);
    const int64_t n_roads = load_size(nr_s);
    const int64_t nb = (n + kKeptBlock - 1) / kKeptBlock;
    const int64_t n_tiles = (n + tile_combos - 1) / tile_combos;
    for (int64_t b = static_cast<int64_t>(blockIdx.x) * kWaves + wv; b < nb;
         b += static_cast<int64_t>(gridDim.x) * kWaves) {
        const int64_t base = b * kKeptBlock + static_cast<int64_t>(lane) * 64;
        uint64_t bits = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            bits |= static_cast<uint64_t>(accept_bits16(accept, base + 16 * q, n)) << (16 * q);
        const int cnt = __popcll(bits);
        const int incl = wave_incl_scan(cnt);
        const int tot = __shfl(incl, kWaveSize - 1);
        if (tot == 0) continue;  // uniform within the wave
        const int64_t pos0 = kb_prefix[b];
        uint16_t *acc_l = s_acc[wv];
        {
            int o = incl - cnt;
            uint64_t m = bits;
            while (m) {
                acc_l[o++] = static_cast<uint16_t>(lane * 64 + __builtin_ctzll(m));
                m &= m - 1;
            }
        }
        const int64_t t0 = (b * kKeptBlock) / tile_combos;
        const int64_t t1 = ((b + 1) * kKeptBlock - 1) / tile_combos + 1;
        const int64_t r_lo = tile_first_road[t0];
        const int64_t r_hi = t1 < n_tiles ? tile_first_road[t1] : n_roads - 1;
        if (r_lo < 0 || r_hi < r_lo || r_hi >= n_roads) {  // marks inconsistent with the roads
            if (lane == 0) report(err, SVT_ERRCLASS_INDEX, static_cast<uint64_t>(b * kKeptBlock));
            continue;
        }
        const int64_t nloc = r_hi - r_lo + 1;
        const bool staged = nloc <= kKeptRoads;
        int64_t *cb_l = s_cb[wv];
        if (staged)
            for (int64_t j = lane; j < nloc; j += kWaveSize) cb_l[j] = roads.combo_begin[r_lo + j];
        __builtin_amdgcn_wave_barrier();  // one wave: its LDS writes precede its reads
        // the block's accepted combinations, spread evenly over the lanes
        for (int j = lane; j < tot; j += kWaveSize) {
            const int64_t i = b * kKeptBlock + acc_l[j];
            const int64_t pos = pos0 + j;
            int64_t lo = 0, hi = nloc - 1;  // last road with combo_begin <= i
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                const int64_t cb = staged ? cb_l[mid] : roads.combo_begin[r_lo + mid];
                if (cb <= i) lo = mid; else hi = mid - 1;
            }
            const int64_t r = r_lo + lo;
            const int64_t k = i - (staged ? cb_l[lo] : roads.combo_begin[r]);
            const int32_t set = roads.set[r];
            if (k < 0 || k >= roads.ncombo[r] || set < 0 || set >= n_sets) {
                report(err, SVT_ERRCLASS_INDEX, static_cast<uint64_t>(i));
                continue;
            }
            if (pos < kept_cap) {
                int32_t v[6];
                const int64_t c2 = refit_combo(bank, coords, shift, roads.nhits[r],
                                               roads.hit_begin[r], set,
                                               static_cast<uint32_t>(k), v, 6);
                kept[pos] = i;
                if (rec.p0) rec.p0[pos] = v[0];
                if (rec.p1) rec.p1[pos] = v[1];
                if (rec.p2) rec.p2[pos] = v[2];
                if (rec.chi2) rec.chi2[pos] = c2;
                if (rec.c0) rec.c0[pos] = v[3];
                if (rec.c1) rec.c1[pos] = v[4];
                if (rec.c2) rec.c2[pos] = v[5];
            }
        }
        __builtin_amdgcn_wave_barrier();  // the slice is reused by the wave's next block
    }
}

// The header and the first n_roads per-road results of a batch, back to back in one buffer
// (layout in svt_gather_results).  When the buffer is host memory every store crosses the bus
// once; a closing system-scope fence in every thread that stored makes them visible to the
// host with the kernel's end (the grid is sized for the capacity, and the threads past the
// batch's roads store nothing and skip the costly fence).
__global__ void k_gather(svt_roads roads, svt_best best, int64_t road_cap, const int64_t *n_words,
                         const int64_t *n_roads, const int64_t *n_combos, const int64_t *n_kept,
                         const uint64_t *err, int64_t *out, int64_t out_roads) {
    const int64_t nr = *n_roads;
    if (gtid() == 0) {
        out[0] = *n_words;
        out[1] = nr;
        out[2] = *n_combos;
        out[3] = n_kept ? *n_kept : -1;
        out[4] = static_cast<int64_t>(*err);
        out[5] = out[6] = out[7] = 0;
    }
    if (nr >= 0 && nr <= out_roads && nr <= road_cap) {
        int64_t *chi2 = out + 8;
        int32_t *col = reinterpret_cast<int32_t *>(chi2 + nr);
        const int32_t *src[7] = {best.n_accept, best.k, best.p0, best.p1, best.p2, roads.event,
                                 roads.set};
        for (int64_t i = gtid(); i < nr; i += gstride()) {
            chi2[i] = best.chi2[i];
#pragma unroll
            for (int a = 0; a < 7; ++a) col[a * nr + i] = src[a][i];
        }
    }
    if (gtid() == 0 || gtid() < nr) __threadfence_system();
}

inline int64_t clamp_grid(int64_t blocks, int64_t maxb) {
    if (blocks < 1) return 1;
    return blocks < maxb ? blocks : maxb;
}

}  // namespace

// ---------------------------------------------------------------------------------------------
hipError_t launch_init_err(uint64_t *d_err, hipStream_t s) {
    hipLaunchKernelGGL(k_init_err, dim3(1), dim3(1), 0, s, d_err);
    return hipGetLastError();
}

hipError_t launch_seg_count(const uint32_t *words, Sizes n_words, int64_t grid_blocks,
                            int32_t n_layers, int64_t *wb_counts, uint64_t *err, hipStream_t s) {
    const int64_t g = clamp_grid(grid_blocks, 1 << 16);
    hipLaunchKernelGGL(k_seg_count, dim3(g), dim3(kSegThreads), 0, s, words, n_words, n_layers,
                       wb_counts, grid_blocks, err);
    return hipGetLastError();
}

hipError_t launch_scan(int64_t *data, int64_t col_stride, int ncols, Sizes n, int64_t div,
                       int64_t *tot0, int64_t *tot1, int64_t cap0, uint32_t cap_index,
                       uint64_t *err, bool skip_if_error, hipStream_t s) {
    hipLaunchKernelGGL(k_scan, dim3(ncols), dim3(kScanThreads), 0, s, data, col_stride, n, div,
                       tot0, tot1, cap0, cap_index, err, static_cast<int32_t>(skip_if_error));
    return hipGetLastError();
}

hipError_t launch_seg_emit(const uint32_t *words, Sizes n_words, int64_t grid_blocks,
                           const int64_t *wb_prefix, const svt_roads &roads, int64_t road_cap,
                           uint64_t *err, hipStream_t s) {
    const int64_t g = clamp_grid(grid_blocks, 1 << 16);
    hipLaunchKernelGGL(k_seg_emit, dim3(g), dim3(kSegThreads), 0, s, words, n_words, wb_prefix,
                       grid_blocks, roads, road_cap, err);
    return hipGetLastError();
}

hipError_t launch_road_fill(const uint32_t *words, Sizes n_words, const int64_t *d_n_roads,
                            int64_t road_cap, const svt_roads &roads, const svt_config &cfg,
                            int16_t *hit_coord, int64_t *rb_sums, uint64_t *err,
                            hipStream_t s) {
    (void)rb_sums;
    const int64_t g = clamp_grid((road_cap + kRoadBlock - 1) / kRoadBlock, 8192);
    hipLaunchKernelGGL(k_road_fill, dim3(g), dim3(kRoadBlock), 0, s, words, n_words, d_n_roads,
                       road_cap, roads, cfg, hit_coord, err);
    return hipGetLastError();
}

hipError_t launch_combo_count(const svt_roads &roads, Sizes n_roads, int64_t grid_blocks,
                              int64_t *rb_sums, uint64_t *err, hipStream_t s) {
    const int64_t g = grid_blocks < 1 ? 1 : grid_blocks;
    hipLaunchKernelGGL(k_combo_count, dim3(g), dim3(kRoadBlock), 0, s, roads, n_roads, rb_sums,
                       err);
    return hipGetLastError();
}

hipError_t launch_combo_begin(const svt_roads &roads, Sizes n_roads, int64_t grid_blocks,
                              const int64_t *rb_prefix, int64_t tile_combos,
                              int32_t *tile_first_road, int64_t tiles_cap,
                              const svt_best *best_defaults, uint64_t *err, hipStream_t s) {
    const int64_t g = grid_blocks < 1 ? 1 : grid_blocks;
    svt_best b = best_defaults ? *best_defaults : svt_best{};
    hipLaunchKernelGGL(k_combo_begin, dim3(g), dim3(kRoadBlock), 0, s, roads, n_roads, rb_prefix,
                       tile_combos, tile_first_road, tiles_cap, b,
                       static_cast<int32_t>(best_defaults != nullptr), err);
    return hipGetLastError();
}

hipError_t launch_materialize(const svt_roads &roads, int64_t n_roads, const int64_t *d_n_combos,
                              int64_t combo_cap, int32_t *combo_road, uint32_t *combo_hits,
                              uint64_t *err, hipStream_t s) {
    if (n_roads <= 0 || (!combo_road && !combo_hits)) return hipSuccess;
    const int64_t g = (n_roads + kRoadBlock - 1) / kRoadBlock;
    hipLaunchKernelGGL(k_materialize, dim3(g), dim3(kRoadBlock), 0, s, roads, n_roads, d_n_combos,
                       combo_cap, combo_road, combo_hits, err);
    return hipGetLastError();
}

hipError_t launch_fit_plain(const svt_fconst *bank, const svt_config &cfg,
                            const svt_roads &roads, int64_t n_roads, const int16_t *hit_coord,
                            int64_t n_hits, const int32_t *combo_road,
                            const uint32_t *combo_hits, int64_t n_combos, const svt_fitrec &out,
                            uint64_t *err, hipStream_t s) {
    if (n_combos <= 0) return hipSuccess;
    const int64_t g = clamp_grid((n_combos + 255) / 256, 1 << 20);
    hipLaunchKernelGGL(k_fit_plain, dim3(g), dim3(256), 0, s, bank, cfg, roads, n_roads,
                       hit_coord, n_hits, combo_road, combo_hits, n_combos, out, err);
    return hipGetLastError();
}

hipError_t launch_select(const svt_config &cfg, const svt_roads &roads, int64_t n_roads,
                         const int32_t *combo_road, const svt_fitrec &rec, int64_t n_combos,
                         uint8_t *accept, const svt_best &best, int64_t *kb_counts,
                         uint64_t *err, hipStream_t s) {
    if (n_roads > 0) {
        const int64_t g = clamp_grid((n_roads + 255) / 256, 1 << 16);
        hipLaunchKernelGGL(k_best_init, dim3(g), dim3(256), 0, s, best, n_roads);
    }
    if (n_combos > 0) {
        const int64_t g = clamp_grid((n_combos + kKeptBlock - 1) / kKeptBlock, 1 << 16);
        hipLaunchKernelGGL(k_select_mark, dim3(g), dim3(kSegThreads), 0, s, cfg, roads, n_roads,
                           combo_road, rec.chi2, n_combos, accept, best, kb_counts, err);
    }
    if (n_roads > 0)
        return launch_best_finalize(roads, Sizes{n_roads, nullptr, n_roads}, rec,
                                    Sizes{n_combos, nullptr, n_combos}, best, cfg.chi2_cut, err,
                                    false, nullptr, nullptr, 0, ScanJob{}, s);
    return hipGetLastError();
}

hipError_t launch_best_finalize(const svt_roads &roads, Sizes n_roads, const svt_fitrec &rec,
                                Sizes n_combos, const svt_best &best, int64_t cut,
                                uint64_t *err, bool skip_if_error, const svt_fconst *bank,
                                const int16_t *coords, int32_t shift, const ScanJob &job,
                                hipStream_t s) {
    const int64_t g = clamp_grid((n_roads.cap + 255) / 256, 1 << 14) + (job.data ? 1 : 0);
    hipLaunchKernelGGL(k_best_finalize, dim3(g), dim3(256), 0, s, roads, n_roads, rec, n_combos,
                       best, cut, err, static_cast<int32_t>(skip_if_error), bank, coords, shift,
                       job);
    return hipGetLastError();
}

hipError_t launch_kept_write(const uint8_t *accept, Sizes n_combos, int64_t grid_blocks,
                             const int64_t *kb_prefix, int64_t *kept, int64_t kept_cap,
                             uint64_t *err, hipStream_t s) {
    const int64_t g = clamp_grid(grid_blocks, 1 << 16);
    hipLaunchKernelGGL(k_kept_write, dim3(g), dim3(kSegThreads), 0, s, accept, n_combos,
                       kb_prefix, kept, kept_cap, err);
    return hipGetLastError();
}

hipError_t launch_gather(const svt_roads &roads, const svt_best &best, int64_t road_cap,
                         const int64_t *d_n_words, const int64_t *d_n_roads,
                         const int64_t *d_n_combos, const int64_t *d_n_kept,
                         const uint64_t *d_err, void *out, int64_t out_roads, hipStream_t s) {
    const int64_t g = clamp_grid((out_roads + 255) / 256, 1024);
    hipLaunchKernelGGL(k_gather, dim3(g), dim3(256), 0, s, roads, best, road_cap, d_n_words,
                       d_n_roads, d_n_combos, d_n_kept, d_err, static_cast<int64_t *>(out),
                       out_roads);
    return hipGetLastError();
}

}  // namespace svt

namespace svt {
hipError_t launch_kept_refit(const uint8_t *accept, Sizes n_combos, Sizes n_roads,
                             int64_t grid_blocks, const int64_t *kb_prefix, const svt_roads &roads,
                             const int32_t *tile_first_road, int64_t tile_combos,
                             const svt_fconst *bank, int32_t n_sets, const int16_t *coords,
                             int32_t shift, int64_t *kept, const svt_fitrec &rec,
                             int64_t kept_cap, uint64_t *err, hipStream_t s) {
    // one wave per kept block, four per workgroup
    const int64_t g = clamp_grid((grid_blocks + 3) / 4, 1 << 16);
    hipLaunchKernelGGL(k_kept_refit, dim3(g), dim3(kSegThreads), 0, s, accept, n_combos, n_roads,
                       kb_prefix, roads, tile_first_road, tile_combos, bank, n_sets, coords,
                       shift, kept, rec, kept_cap, err);
    return hipGetLastError();
}
}  // namespace svt
