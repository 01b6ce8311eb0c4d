// Decoupled look-back over fixed-size blocks of hit words, shared by the batched pre-pass and
// the one-pass kernel of libsvt.
//
// Unpacking (section II-A of the paper, the serial code's first function) needs running counts
// over the whole stream: which road and event a word belongs to, where a road's combinations
// start.  Each block of BW words publishes what it found among its own words -- the roads that
// start there, the events that start there, and the combinations of those roads -- as soon as
// it knows them, then adds up the published values of the blocks before it.
//
// Two 64-bit status words per block carry the running counts -- roads and events packed in one
// (31 bits each: a batch holds fewer than 2^31 words), combinations in the other: the top two
// bits say "aggregate of this block" or "inclusive prefix up to this block", the rest hold the
// value.  The status words are read and written with relaxed agent-scope atomics; each word
// carries its own flag, so no release/acquire ordering is needed.  They must be zero before a
// pass (the batch-reset kernel clears them).
//
// A block that waits too long for a predecessor computes that predecessor's aggregate from the
// words itself (block_aggregate), by the rules the predecessor applies to its own words, and
// publishes it with a compare-and-swap from "empty": no block waits forever on one that has not
// been scheduled, whatever order the hardware runs blocks in.
#pragma once

#include "svt_common.h"

namespace svt {

constexpr uint64_t kStAgg = 1ull << 62;
constexpr uint64_t kStIncl = 2ull << 62;
constexpr uint64_t kStMask = 3ull << 62;
// a look-back round computes missing aggregates itself after this long (wall-clock ticks of
// 10 ns): far beyond any wait on a predecessor that is running
constexpr uint64_t kLookbackTimeout = 20000;
constexpr int kLookWindows = 8;  // predecessors read per round: 64 per window
constexpr int kRoadTail = 64;    // words past a block that a road starting in it may use
                                 // (a road with combinations has at most 5 * 8 = 40 words)

struct LookbackCtx {
    const uint32_t *words;
    int64_t n;             // words in the batch
    int32_t n_layers;
    int32_t max_hits;
    int64_t *status;       // [2][nb_cap]: roads | events << 31, combinations
    int64_t nb_cap;
    uint64_t timeout;      // wall-clock ticks a look-back round waits before computing itself
};

__device__ inline void status_publish(int64_t *p, uint64_t v) {
    __hip_atomic_store(reinterpret_cast<uint64_t *>(p), v, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

// publish v for a block that has published nothing yet (no effect otherwise)
__device__ inline void status_claim(int64_t *p, uint64_t v) {
    uint64_t expected = 0;
    __hip_atomic_compare_exchange_strong(reinterpret_cast<uint64_t *>(p), &expected, v,
                                         __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline uint64_t status_read(int64_t *p) {
    return __hip_atomic_load(reinterpret_cast<uint64_t *>(p), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
}

__device__ inline int64_t combos_of(uint32_t packed) {
    int64_t c = 1;
#pragma unroll
    for (int l = 0; l < SVT_N_LAYERS; ++l) c *= nh_of(packed, l);
    return c;
}

// The aggregate of block p -- roads that start among its words | events that start there << 31,
// and the combinations of those roads -- computed from the words in global memory by the rules
// a block applies to its own staged words (a road runs to the next road start among the block's
// words and its kRoadTail-word tail, else to the end of them; longer than n_layers * max_hits
// words, or more than max_hits hits on a layer, and it has no combinations).  One wave; lane i
// takes the block's words BW/64 * i .. BW/64 * (i + 1) - 1.
template <int BW>
__device__ void block_aggregate(const LookbackCtx &a, int64_t p, uint64_t &agg0,
                                uint64_t &agg1) {
    constexpr int kPerLane = BW / kWaveSize;
    const int lane = lane_id();
    const int64_t base = p * BW;
    const int64_t n = a.n;
    const int nloc = static_cast<int>(n - base < BW + kRoadTail ? n - base : BW + kRoadTail);
    const int nown = nloc < BW ? nloc : BW;
    const int max_len = a.n_layers * a.max_hits;
    int64_t nr = 0, ne = 0, nc = 0;
    for (int e = 0; e < kPerLane; ++e) {
        const int j = lane * kPerLane + e;
        if (j >= nown) break;
        const uint32_t x = a.words[base + j];
        const bool first = base + j == 0;
        const uint32_t px = first ? 0u : a.words[base + j - 1];
        ne += (first || w_etag(x) != w_etag(px)) ? 1 : 0;
        if (!(first || w_tags(x) != w_tags(px))) continue;
        ++nr;
        uint64_t cnt = 0;  // 8 bits per layer
        bool over = false;
        uint32_t prev = x;
        for (int k = j, len = 0; k < nloc; ++k) {
            const uint32_t y = a.words[base + k];
            if (k > j && w_tags(y) != w_tags(prev)) break;  // next road starts
            if (++len > max_len) {
                over = true;
                break;
            }
            const uint32_t l = w_layer(y);
            if (l < SVT_N_LAYERS) cnt += 1ull << (8 * l);
            prev = y;
        }
        uint32_t packed = 0;
#pragma unroll
        for (int l = 0; l < SVT_N_LAYERS; ++l) {
            const uint32_t c = static_cast<uint32_t>((cnt >> (8 * l)) & 0xFF);
            over |= c > static_cast<uint32_t>(a.max_hits);
            packed |= (c & 0xFu) << (4 * l);
        }
        if (!over) nc += combos_of(packed);
    }
    agg0 = static_cast<uint64_t>(wave_sum(nr)) | (static_cast<uint64_t>(wave_sum(ne)) << 31);
    agg1 = static_cast<uint64_t>(wave_sum(nc));
}

// A block's own counts, published as soon as they are known: an aggregate, or for block 0
// directly its inclusive prefix.  One thread.
__device__ inline void publish_aggregate(const LookbackCtx &a, int64_t b, uint64_t agg0,
                                         uint64_t agg1) {
    const uint64_t flag = b == 0 ? kStIncl : kStAgg;
    status_publish(a.status + b, flag | agg0);
    status_publish(a.status + a.nb_cap + b, flag | agg1);
}

// Exclusive prefixes over blocks 0..b-1 of two status columns at once (col0[i], col1[i] =
// column 0 and 1 of block i), for a block whose aggregates are already published
// (publish_aggregate); publishes its inclusive prefixes once known.  Executed by one whole
// wave; the results are valid in every lane.  One round reads kLookWindows * 64 predecessors
// of both columns (lane i of window k inspects block top - 64 k - i, so position 0 is the
// nearest predecessor); each column sums its values up to its nearest block that already has
// an inclusive value.  Values are opaque sums: counts packed in one word add field by field as
// long as no field overflows.  A round that has waited a.timeout wall-clock ticks for
// predecessors to publish computes their aggregates from the words instead (block_aggregate)
// and goes on.
template <int BW>
__device__ void look_back2(const LookbackCtx &a, int64_t b, uint64_t agg0, uint64_t agg1,
                           uint64_t &ex0, uint64_t &ex1) {
    int64_t *col0 = a.status, *col1 = a.status + a.nb_cap;
    const int lane = lane_id();
    ex0 = 0;
    ex1 = 0;
    if (b == 0) return;  // its inclusive prefix is its aggregate, already published
    bool done0 = false, done1 = false;
    int64_t top = b - 1;
    uint64_t wait_since = 0;  // start of this round's wait (0: not waiting)
    while (!(done0 && done1)) {
        uint64_t v0[kLookWindows], v1[kLookWindows];
#pragma unroll
        for (int k = 0; k < kLookWindows; ++k) {
            const int64_t idx = top - 64 * k - lane;
            v0[k] = (idx >= 0 && !done0) ? status_read(col0 + idx) : kStIncl;
            v1[k] = (idx >= 0 && !done1) ? status_read(col1 + idx) : kStIncl;
        }
        int f0 = 64 * kLookWindows, f1 = 64 * kLookWindows;  // nearest inclusive positions
#pragma unroll
        for (int k = kLookWindows - 1; k >= 0; --k) {
            const uint64_t m0 = __ballot((v0[k] & kStMask) == kStIncl);
            const uint64_t m1 = __ballot((v1[k] & kStMask) == kStIncl);
            if (m0) f0 = 64 * k + __builtin_ctzll(m0);
            if (m1) f1 = 64 * k + __builtin_ctzll(m1);
        }
        bool wait = false;
#pragma unroll
        for (int k = 0; k < kLookWindows; ++k) {
            const int pos = 64 * k + lane;
            wait |= __ballot(((v0[k] & kStMask) == 0 && pos <= f0) ||
                             ((v1[k] & kStMask) == 0 && pos <= f1)) != 0;
        }
        if (wait) {  // a block at or before a nearest inclusive one has not published yet
            const uint64_t now = wall_clock64();
            if (wait_since == 0) wait_since = now;
            if (now - wait_since < a.timeout) {
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            // Waited long enough: publish every aggregate this round still misses, computed
            // from the words, then read the round again.  A compare-and-swap from "nothing"
            // never overwrites what the block itself has published meanwhile (and what it
            // publishes later is the same aggregate, or its inclusive prefix).
            int need = (done0 ? -1 : f0) > (done1 ? -1 : f1) ? f0 : f1;  // farthest position
            need = need < 64 * kLookWindows ? need : 64 * kLookWindows - 1;  // of this round
            for (int64_t idx = top; idx >= 0 && top - idx <= need; --idx) {
                const uint64_t s0 = status_read(col0 + idx), s1 = status_read(col1 + idx);
                if ((s0 & kStMask) != 0 && (s1 & kStMask) != 0) continue;
                uint64_t g0, g1;
                block_aggregate<BW>(a, idx, g0, g1);
                if (lane == 0) {
                    status_claim(col0 + idx, kStAgg | g0);
                    status_claim(col1 + idx, kStAgg | g1);
                }
            }
            wait_since = 0;
            continue;
        }
        wait_since = 0;
        uint64_t m0 = 0, m1 = 0;
#pragma unroll
        for (int k = 0; k < kLookWindows; ++k) {
            const int pos = 64 * k + lane;
            if (!done0 && pos <= f0) m0 += v0[k] & ~kStMask;
            if (!done1 && pos <= f1) m1 += v1[k] & ~kStMask;
        }
        ex0 += wave_sum(m0);
        ex1 += wave_sum(m1);
        done0 |= f0 < 64 * kLookWindows;
        done1 |= f1 < 64 * kLookWindows;
        top -= 64 * kLookWindows;
    }
    if (lane == 0) {
        status_publish(col0 + b, kStIncl | (ex0 + agg0));
        status_publish(col1 + b, kStIncl | (ex1 + agg1));
    }
}

}  // namespace svt
