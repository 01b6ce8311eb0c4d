// One event per workgroup: the multi-core scheme of section II-A (each core takes whole events
// and runs the combine and fit loops of each of them), as schedule 1 of the batched pass.  It
// writes exactly the outputs of the persistent fused kernel -- records (or, in kept-only mode,
// only the accept flags), the per-road best keys and accept counts -- and is kept as the
// ablation against flat combination tiles: an event's work is not split between workgroups,
// so the batch is balanced only at event granularity.
//
// A workgroup takes the next event from an atomic ticket, stages its roads' combo_begin in
// LDS, and its threads walk the event's combinations; each finds its road by binary search,
// decodes the hit of every layer from the combination index (layer 0 most significant), reads
// the coordinates and fits them with 64-bit integer arithmetic.
#include "svt_common.h"

namespace svt {
namespace {

constexpr int kEvThreads = 256;
constexpr int kEvRoads = 2048;  // roads of an event staged in LDS; more are searched in place

struct EArgs {
    const svt_fconst *bank;
    int32_t shift;
    int64_t cut;
    const int16_t *coords;
    svt_roads roads;
    const int64_t *d_n_roads;
    const int64_t *d_n_combos;
    const int64_t *d_n_events;
    const int32_t *event_first_road;
    svt_fitrec rec;
    uint8_t *accept;
    svt_best best;  // best.chi2 holds the per-road key during the pass
    unsigned long long *kb_counts;
    uint32_t *ticket;
    uint64_t *err;
    int64_t road_cap, combo_cap, event_cap;
    int32_t records;
};

__global__ __launch_bounds__(kEvThreads) void k_fit_events(EArgs a) {
    __shared__ int64_t s_cb[kEvRoads];
    __shared__ int64_t s_e;
    if (has_error(a.err)) return;
    const int64_t n_roads = *a.d_n_roads;
    const int64_t n_combos = *a.d_n_combos;
    const int64_t n_events = *a.d_n_events;
    if (n_roads < 0 || n_roads > a.road_cap || n_combos < 0 || n_combos > a.combo_cap ||
        n_events < 0 || n_events > a.event_cap)
        return;
    unsigned long long *keys = reinterpret_cast<unsigned long long *>(a.best.chi2);
    const int tid = threadIdx.x;
    while (true) {
        if (tid == 0) s_e = atomicAdd(a.ticket, 1u);
        __syncthreads();
        const int64_t e = s_e;
        __syncthreads();  // s_e is written again next round
        if (e >= n_events) break;
        const int64_t r0 = a.event_first_road[e];
        const int64_t r1 = e + 1 < n_events ? a.event_first_road[e + 1] : n_roads;
        if (r0 < 0 || r1 > n_roads || r0 >= r1) {
            if (tid == 0) report(a.err, SVT_ERRCLASS_INDEX, static_cast<uint64_t>(e));
            continue;
        }
        const int64_t nr = r1 - r0;
        const int64_t c0 = a.roads.combo_begin[r0];
        const int64_t c1 = r1 < n_roads ? a.roads.combo_begin[r1] : n_combos;
        const bool staged = nr <= kEvRoads;
        if (staged)
            for (int64_t j = tid; j < nr; j += kEvThreads) s_cb[j] = a.roads.combo_begin[r0 + j];
        __syncthreads();
        for (int64_t c = c0 + tid; c < c1; c += kEvThreads) {
            int64_t lo = 0, hi = nr - 1;  // last road of the event with combo_begin <= c
            while (lo < hi) {
                const int64_t mid = (lo + hi + 1) >> 1;
                const int64_t cb = staged ? s_cb[mid] : a.roads.combo_begin[r0 + mid];
                if (cb <= c) lo = mid; else hi = mid - 1;
            }
            const int64_t r = r0 + lo;
            const uint32_t nh = a.roads.nhits[r];
            const int64_t hb = a.roads.hit_begin[r];
            const int32_t s = a.roads.set[r];
            uint32_t k = static_cast<uint32_t>(c - (staged ? s_cb[lo] : a.roads.combo_begin[r]));
            const uint32_t kk = k;
            uint32_t h[SVT_N_LAYERS];
            for (int l = SVT_N_LAYERS - 1; l >= 0; --l) {  // layer 0 most significant
                const uint32_t nl = nh_of(nh, l);
                h[l] = k % nl;
                k /= nl;
            }
            int64_t off = hb;
            int32_t x[SVT_N_LAYERS];
            for (int l = 0; l < SVT_N_LAYERS; ++l) {
                x[l] = a.coords[off + h[l]];
                off += nh_of(nh, l);
            }
            const svt_fconst &F = a.bank[s];
            int32_t v[6];
            for (int j = 0; j < 6; ++j) {
                int64_t acc = F.q[j];
                for (int l = 0; l < SVT_N_LAYERS; ++l)
                    acc += static_cast<int64_t>(F.f[j][l]) * static_cast<int64_t>(x[l]);
                v[j] = static_cast<int32_t>(acc >> a.shift);
            }
            const int64_t chi2 = static_cast<int64_t>(v[3]) * v[3] +
                                 static_cast<int64_t>(v[4]) * v[4] +
                                 static_cast<int64_t>(v[5]) * v[5];
            const bool acc = chi2 <= a.cut;
            if (a.records) {
                a.rec.p0[c] = v[0];
                a.rec.p1[c] = v[1];
                a.rec.p2[c] = v[2];
                a.rec.chi2[c] = chi2;
                if (a.rec.c0) a.rec.c0[c] = v[3];
                if (a.rec.c1) a.rec.c1[c] = v[4];
                if (a.rec.c2) a.rec.c2[c] = v[5];
            }
            a.accept[c] = acc ? 1 : 0;
            if (acc) {
                atomicMin(keys + r, static_cast<unsigned long long>(best_key(chi2, kk)));
                atomicAdd(a.best.n_accept + r, 1);
                if (a.kb_counts) atomicAdd(a.kb_counts + c / kKeptBlock, 1ull);
            }
        }
        __syncthreads();  // s_cb is reused by the next event
    }
}

}  // namespace

hipError_t launch_fit_events(const FusedLaunch &f, const int32_t *event_first_road,
                             const int64_t *d_n_events, int64_t event_cap, hipStream_t s) {
    EArgs a;
    a.bank = f.bank;
    a.shift = f.cfg.shift;
    a.cut = f.cfg.chi2_cut;
    a.coords = f.coords;
    a.roads = f.roads;
    a.d_n_roads = f.d_n_roads;
    a.d_n_combos = f.d_n_combos;
    a.d_n_events = d_n_events;
    a.event_first_road = event_first_road;
    a.rec = f.rec;
    a.accept = f.accept;
    a.best = f.best;
    a.kb_counts = reinterpret_cast<unsigned long long *>(f.kb_counts);
    a.ticket = f.tile_counter;
    a.err = f.err;
    a.road_cap = f.road_cap;
    a.combo_cap = f.combo_cap;
    a.event_cap = event_cap;
    a.records = f.kept_only ? 0 : 1;
    const int grid = f.num_cus * f.tune.wgs_per_cu;
    hipLaunchKernelGGL(k_fit_events, dim3(grid > 0 ? grid : 1), dim3(kEvThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace svt
