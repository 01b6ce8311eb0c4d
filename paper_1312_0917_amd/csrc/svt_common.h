// Internal helpers shared by the HIP kernels of libsvt (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "svt.h"

namespace svt {

constexpr int kWaveSize = 64;
constexpr int kSegThreads = 256;          // threads of the word-segmentation kernels
constexpr int kSegWordsPerThread = 16;
constexpr int kSegBlockWords = kSegThreads * kSegWordsPerThread;  // 4096 words per block
constexpr int kPrepassBlockWords = 2048;  // words per block of the batched single-pass pre-pass
constexpr int kLookGroup = 64;            // pre-pass blocks per group of its two-level look-back
// look-back status words of the pre-pass: two per block, then two per group of kLookGroup blocks
inline int64_t prepass_status_words(int64_t nb_cap) {
    return 2 * nb_cap + 2 * ((nb_cap + kLookGroup - 1) / kLookGroup);
}
constexpr int kOnepassUnitWords = 1024;   // words per unit of the one-pass kernel
constexpr int kRoadBlock = 256;           // roads per block in road-table kernels
constexpr int kKeptBlock = 4096;          // combinations per block of the kept-list compaction
constexpr int kScanThreads = 1024;        // single-workgroup scan
constexpr int kKeyKBits = 15;             // best-track key: chi2 << 15 | k  (k < 8^5 = 2^15)
constexpr uint64_t kKeyChiMax = (1ull << 49) - 1;  // chi2 part of a key saturates here

// Order-preserving key of an accepted combination for one 64-bit atomicMin: exact whenever
// the smallest chi2 of the road is below kKeyChiMax; a saturated minimum means "rescan".
__device__ inline uint64_t best_key(int64_t chi2, uint32_t k) {
    uint64_t c = static_cast<uint64_t>(chi2);
    if (c > kKeyChiMax) c = kKeyChiMax;
    return (c << kKeyKBits) | k;
}
constexpr int kMaxTile = 8192;  // combinations per tile of the fused kernel, at most
constexpr int64_t kMaxBatchWords = (1ll << 31) - 1;  // batched path: road and event counts fit 31 bits

// ---- error word: (class << 56) | index, smallest wins, all ones = none ------------------
__device__ inline void report(uint64_t *err, uint32_t cls, uint64_t index) {
    uint64_t v = (static_cast<uint64_t>(cls) << 56) | (index & ((1ull << 56) - 1));
    atomicMin(reinterpret_cast<unsigned long long *>(err), static_cast<unsigned long long>(v));
}

__device__ inline bool has_error(const uint64_t *err) {
    return *reinterpret_cast<const volatile uint64_t *>(err) != SVT_NO_ERROR;
}

// ---- hit word fields (coord int13 | layer 3 | road tag 8 | event tag 8) -------------------
__device__ inline int32_t w_coord(uint32_t w) {
    return static_cast<int32_t>(w << 19) >> 19;  // sign-extend the low 13 bits
}
__device__ inline uint32_t w_layer(uint32_t w) { return (w >> 13) & 7u; }
__device__ inline uint32_t w_rtag(uint32_t w) { return (w >> 16) & 0xFFu; }
__device__ inline uint32_t w_etag(uint32_t w) { return w >> 24; }
__device__ inline uint32_t w_tags(uint32_t w) { return w >> 16; }  // road and event tag together

__device__ inline uint32_t nh_of(uint32_t packed, int l) { return (packed >> (4 * l)) & 0xFu; }

// ---- wave64 / block scans -----------------------------------------------------------------
__device__ inline int lane_id() { return __lane_id(); }

template <typename T>
__device__ inline T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int d = 1; d < kWaveSize; d <<= 1) {
        T t = __shfl_up(v, d, kWaveSize);
        if (lane >= d) v += t;
    }
    return v;
}

template <typename T>
__device__ inline T wave_sum(T v) {
#pragma unroll
    for (int d = kWaveSize / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWaveSize);
    return v;
}

// Exclusive block scan for blockDim.x = NT threads; returns the exclusive prefix and the
// block total.  `tmp` must hold NT/64 + 1 elements of T in LDS.  Contains barriers.
template <typename T, int NT>
__device__ inline T block_excl_scan(T v, T *tmp, T &total) {
    constexpr int NW = NT / kWaveSize;
    const int lane = lane_id();
    const int wave = threadIdx.x / kWaveSize;
    T incl = wave_incl_scan(v);
    if (lane == kWaveSize - 1) tmp[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < NW; ++w) {
            T t = tmp[w];
            tmp[w] = run;
            run += t;
        }
        tmp[NW] = run;
    }
    __syncthreads();
    T res = incl - v + tmp[wave];
    total = tmp[NW];
    __syncthreads();
    return res;
}

template <typename T, int NT>
__device__ inline T block_sum(T v, T *tmp) {
    constexpr int NW = NT / kWaveSize;
    T s = wave_sum(v);
    const int wave = threadIdx.x / kWaveSize;
    if (lane_id() == 0) tmp[wave] = s;
    __syncthreads();
    T tot = 0;
    for (int w = 0; w < NW; ++w) tot += tmp[w];
    __syncthreads();
    return tot;
}

// Grid-stride helpers
__device__ inline int64_t gtid() {
    return static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
}
__device__ inline int64_t gstride() { return static_cast<int64_t>(gridDim.x) * blockDim.x; }

}  // namespace svt

// ---- host-side launchers (defined in the .hip files) --------------------------------------
namespace svt {

struct Sizes {  // counts that can live on the host (plain path) or on the device (batch path)
    int64_t host;            // used when dev == nullptr
    const int64_t *dev;      // device scalar
    int64_t cap;             // kernels never use more than this many items
};

__device__ inline int64_t load_size(const Sizes &s) {
    int64_t v = s.dev ? *s.dev : s.host;
    if (v > s.cap) v = s.cap;
    return v < 0 ? 0 : v;
}

hipError_t launch_init_err(uint64_t *d_err, hipStream_t s);
hipError_t launch_seg_count(const uint32_t *words, Sizes n_words, int64_t grid_blocks,
                            int32_t n_layers, int64_t *wb_counts, uint64_t *err, hipStream_t s);
// In-place exclusive scan of ncols (1 or 2) int64 columns of ceil(n / items_div) entries,
// one workgroup per column; column c's total goes to tot[c] (may be null).  When the total
// of column 0 exceeds cap0 (>= 0), a capacity error with index cap_index is reported.  With
// skip_if_error, an error already in *err makes it write -1 totals and do nothing else.
hipError_t launch_scan(int64_t *data, int64_t col_stride, int ncols, Sizes n,
                       int64_t items_div, int64_t *tot0, int64_t *tot1, int64_t cap0,
                       uint32_t cap_index, uint64_t *err, bool skip_if_error, hipStream_t s);
hipError_t launch_seg_emit(const uint32_t *words, Sizes n_words, int64_t grid_blocks,
                           const int64_t *wb_prefix, const svt_roads &roads, int64_t road_cap,
                           uint64_t *err, hipStream_t s);
hipError_t launch_road_fill(const uint32_t *words, Sizes n_words, const int64_t *d_n_roads,
                            int64_t road_cap, const svt_roads &roads, const svt_config &cfg,
                            int16_t *hit_coord, int64_t *rb_sums, uint64_t *err,
                            hipStream_t s);
hipError_t launch_combo_count(const svt_roads &roads, Sizes n_roads, int64_t grid_blocks,
                              int64_t *rb_sums, uint64_t *err, hipStream_t s);
// best_init (nullable): every road's best key := none, n_accept := 0
hipError_t launch_combo_begin(const svt_roads &roads, Sizes n_roads, int64_t grid_blocks,
                              const int64_t *rb_prefix, int64_t tile_combos,
                              int32_t *tile_first_road, int64_t tiles_cap,
                              const svt_best *best_init, uint64_t *err, hipStream_t s);
hipError_t launch_materialize(const svt_roads &roads, int64_t n_roads, const int64_t *d_n_combos,
                              int64_t combo_cap, int32_t *combo_road, uint32_t *combo_hits,
                              uint64_t *err, hipStream_t s);
hipError_t launch_fit_plain(const svt_fconst *bank, const svt_config &cfg,
                            const svt_roads &roads, int64_t n_roads, const int16_t *hit_coord,
                            int64_t n_hits, const int32_t *combo_road,
                            const uint32_t *combo_hits, int64_t n_combos, const svt_fitrec &out,
                            uint64_t *err, hipStream_t s);
hipError_t launch_select(const svt_config &cfg, const svt_roads &roads, int64_t n_roads,
                         const int32_t *combo_road, const svt_fitrec &rec, int64_t n_combos,
                         uint8_t *accept, const svt_best &best, int64_t *kb_counts,
                         uint64_t *err, hipStream_t s);
hipError_t launch_kept_write(const uint8_t *accept, Sizes n_combos, int64_t grid_blocks,
                             const int64_t *kb_prefix, int64_t *kept, int64_t kept_cap,
                             uint64_t *err, hipStream_t s);
// Kept-only mode: the ascending indices of accepted combinations into kept[] and their fit
// values, compacted, into rec (entry i for combination kept[i]), fitted again from the grouped
// coordinates and the constant bank.  tile_first_road / tile_combos locate each block's roads.
// Does nothing when *err already holds an error (the inputs it reads are then incomplete).
hipError_t launch_kept_refit(const uint8_t *accept, Sizes n_combos, Sizes n_roads,
                             int64_t grid_blocks, const int64_t *kb_prefix, const svt_roads &roads,
                             const int32_t *tile_first_road, int64_t tile_combos,
                             const svt_fconst *bank, int32_t n_sets, const int16_t *coords,
                             int32_t shift, int64_t *kept, const svt_fitrec &rec,
                             int64_t kept_cap, uint64_t *err, hipStream_t s);

struct FusedLaunch {
    const svt_fconst *bank;
    svt_config cfg;
    svt_tune tune;
    const uint32_t *words;
    const int64_t *d_n_words;
    const int16_t *coords;     // workspace: coordinates grouped by layer inside each road
    svt_roads roads;
    const int64_t *d_n_roads;
    const int64_t *d_n_combos;
    svt_fitrec rec;
    uint8_t *accept;
    svt_best best;
    int32_t *tile_first_road;
    int64_t *kb_counts;        // per kKeptBlock combinations (null: kept list not wanted)
    uint32_t *tile_counter;
    uint64_t *err;
    int64_t tiles_cap;
    int64_t road_cap;
    int64_t combo_cap;
    int num_cus;
    bool kept_only;            // no per-combination records (accept flags still written)
};
hipError_t launch_fused(const FusedLaunch &f, hipStream_t s);
// One event per workgroup at a time (schedule 1 of svt_tune): the same outputs as the fused
// kernel, for the ablation against flat combination tiles.
hipError_t launch_fit_events(const FusedLaunch &f, const int32_t *event_first_road,
                             const int64_t *d_n_events, int64_t event_cap, hipStream_t s);
// Per road: turn the best-track key left in best.chi2 into (k, chi2, p0..p2), reading the
// parameters from the records, or fitting them again from the grouped coordinates when bank
// and coords are given (exact rescan of the records for a road whose key saturated).
// An in-place exclusive scan of ceil(n / div) counts with its total written to *tot and checked
// against cap (class CAPACITY, index cap_index) when cap >= 0; data == nullptr: no job.
struct ScanJob {
    int64_t *data = nullptr;
    Sizes n{};
    int64_t div = 1;
    int64_t *tot = nullptr;
    int64_t cap = -1;
    uint32_t cap_index = 0;
};
// Best track per road from the keys; with a scan job, one extra workgroup does that scan.
hipError_t launch_best_finalize(const svt_roads &roads, Sizes n_roads, const svt_fitrec &rec,
                                Sizes n_combos, const svt_best &best, int64_t cut,
                                uint64_t *err, bool skip_if_error, const svt_fconst *bank,
                                const int16_t *coords, int32_t shift, const ScanJob &job,
                                hipStream_t s);
bool fused_tune_supported(const svt_tune &t);

// Single-pass unpack + combine of the batched path (decoupled look-back over word blocks).
struct PrepassLaunch {
    const uint32_t *words;
    Sizes nw;                  // device word count, capacity word_cap
    svt_config cfg;
    svt_roads roads;
    int64_t road_cap;
    int16_t *coords;           // grouped coordinates, word_cap entries
    svt_best best;             // best keys and n_accept are initialised here
    int64_t tile_combos;
    int32_t *tile_first_road;
    int64_t tiles_cap;
    int64_t combo_cap;
    int64_t *d_n_roads;
    int64_t *d_n_combos;
    int64_t *status;           // look-back status words (prepass_status_words(nb_cap))
    int64_t nb_cap;            // ceil(word_cap / kPrepassBlockWords)
    int64_t status_words;      // status words the reset clears
    uint32_t *tickets;         // [0] fused-kernel tiles, [1] pre-pass blocks
    uint64_t *err;
    int32_t *event_first_road; // first road of every event (event_cap entries)
    int64_t event_cap;
    int64_t *d_n_events;
};
// Clears the error word, both tickets, *d_n_kept (nullable), status[0 .. status_words) and
// zero[0 .. n_zero) (the kept-list block counts; nullable).
hipError_t launch_batch_reset(const PrepassLaunch &p, int64_t *nw_copy, int64_t *d_n_kept,
                              int64_t *zero, int64_t n_zero, hipStream_t s);
hipError_t launch_prepass(const PrepassLaunch &p, hipStream_t s);

// The whole batched pass in one persistent kernel (unpack, combine, fit, select; road table,
// records and best tracks written from LDS).  Needs the reset of launch_batch_reset (with
// nb_cap status words for units of kOnepassUnitWords) first.
struct OnepassLaunch {
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
    int64_t *kb_counts;        // accepted count per kKeptBlock combinations (null: no kept list)
    int64_t *status;           // 2 * nb_cap look-back status words
    int64_t nb_cap;            // ceil(word_cap / kOnepassUnitWords)
    uint32_t *tickets;
    uint64_t *err;
    bool kept_only;            // no records; grouped coordinates and block marks for the refit
    int16_t *coords;           // kept-only: grouped coordinates (word_cap entries)
    int32_t *tile_first_road;  // kept-only: first road of every kKeptBlock block
    int64_t tiles_cap;
    int num_cus;
    int wgs_per_cu;
};
hipError_t launch_onepass(const OnepassLaunch &p, hipStream_t s);

}  // namespace svt
