// Two-level decoupled look-back of the batched pre-pass.
//
// With a thousand or more blocks in flight, the nearest block that already knows its inclusive
// prefix is several hundred blocks back, and a one-level look-back (look_back2) makes every block
// read that many status words per round.  Those reads bypass the non-coherent L2 and all land
// on the few kilobytes of status words of the blocks in flight, so they queue behind each other
// and behind every other memory access of the kernel.  Grouping the blocks keeps each read short:
//
//   level 1: per block, its aggregate (the status words of look_back2, written by
//            publish_aggregate);
//   level 2: per group of kLookGroup consecutive blocks, "aggregate of the group" or "inclusive
//            prefix up to the group's end", both published by the group's last block: the
//            aggregate once it has summed the aggregates of the blocks before it in the group,
//            the inclusive prefix once its own look-back is done.
//
// Block b, at position i of group g, sums the level-1 aggregates of blocks gG .. b - 1 (wave 0,
// one lane per block) and the level-2 values of groups g - 1, g - 2, ... back to the nearest
// inclusive one (wave 1, 64 groups per round).  The two reads share a round, and the waves'
// results meet in LDS at one barrier per round.  At most a few dozen groups are in flight, so
// one round usually suffices.  Waiting and the fallback follow look_back2: a round that has
// waited `timeout` ticks computes the missing block aggregates from the words (block_aggregate),
// sums a missing group from its blocks, and claims both with compare-and-swap from "empty".
#pragma once

#include "svt_lookback.h"

namespace svt {

constexpr int kLookNone = 1 << 30;
static_assert(kLookGroup == kWaveSize, "one lane per block of a group");

// Per-round results of look_back_grouped, kept twice (by round parity) so that one barrier per
// round suffices.
struct GroupLookShared {
    uint64_t s1[2][2];  // level 1: sum of the aggregates of the earlier blocks of the group
    uint32_t z1[2];     // level 1: bit c: one of them has published nothing in column c
    uint64_t s2[2][2];  // level 2: sum of the group values up to the nearest inclusive one
    int32_t f2[2][2];   // level 2: position of that group (0 = group g - 1), or kLookNone
    uint32_t z2[2];     // level 2: bit c: a group up to there has published nothing in column c
    uint64_t now[2];    // thread 0's clock: every wave decides alike on waiting
};

// Exclusive prefixes over blocks 0..b-1 of both status columns for the pre-pass block b, whose
// aggregate is already published.  status holds prepass_status_words(nb_cap) words: columns 0
// and 1 of the blocks, then columns 0 and 1 of the groups.  Must be called by every thread of
// the block (at least two waves); contains barriers.  The results are valid in every thread.
template <int BW>
__device__ void look_back_grouped(const LookbackCtx &a, int64_t b, uint64_t agg0, uint64_t agg1,
                                  GroupLookShared &sh, uint64_t &ex0, uint64_t &ex1) {
    constexpr int G = kLookGroup;
    int64_t *col0 = a.status, *col1 = a.status + a.nb_cap;
    const int64_t ng = (a.nb_cap + G - 1) / G;
    int64_t *gcol0 = a.status + 2 * a.nb_cap, *gcol1 = gcol0 + ng;
    const int lane = lane_id();
    const int wave = static_cast<int>(threadIdx.x) / kWaveSize;
    const int64_t g = b / G;
    const int i = static_cast<int>(b - g * G);
    const bool last = i == G - 1;
    bool d1 = i == 0;  // level 1 done
    bool dg0 = g == 0, dg1 = g == 0;
    uint64_t e10 = 0, e11 = 0, e20 = 0, e21 = 0;
    int64_t top = g - 1;      // nearest group not yet summed
    uint64_t wait_since = 0;  // start of the current wait (0: not waiting)
    int par = 0;
    while (!(d1 && dg0 && dg1)) {
        if (wave == 0 && !d1) {
            uint64_t v0 = kStAgg, v1 = kStAgg;  // lanes past the block: published zeros
            if (lane < i) {
                v0 = status_read(col0 + g * G + lane);
                v1 = status_read(col1 + g * G + lane);
            }
            const uint64_t s0 = wave_sum(v0 & ~kStMask), s1 = wave_sum(v1 & ~kStMask);
            const uint32_t z = (__ballot((v0 & kStMask) == 0) ? 1u : 0u) |
                               (__ballot((v1 & kStMask) == 0) ? 2u : 0u);
            if (lane == 0) {
                sh.s1[par][0] = s0;
                sh.s1[par][1] = s1;
                sh.z1[par] = z;
            }
        }
        if (wave == 1 && !(dg0 && dg1)) {
            const int64_t idx = top - lane;
            const uint64_t v0 = (idx >= 0 && !dg0) ? status_read(gcol0 + idx) : kStIncl;
            const uint64_t v1 = (idx >= 0 && !dg1) ? status_read(gcol1 + idx) : kStIncl;
            const uint64_t m0 = __ballot((v0 & kStMask) == kStIncl);
            const uint64_t m1 = __ballot((v1 & kStMask) == kStIncl);
            const int f0 = m0 ? __builtin_ctzll(m0) : kLookNone;
            const int f1 = m1 ? __builtin_ctzll(m1) : kLookNone;
            const uint64_t s0 = wave_sum(lane <= f0 ? v0 & ~kStMask : 0ull);
            const uint64_t s1 = wave_sum(lane <= f1 ? v1 & ~kStMask : 0ull);
            const uint32_t z = (__ballot((v0 & kStMask) == 0 && lane <= f0) ? 1u : 0u) |
                               (__ballot((v1 & kStMask) == 0 && lane <= f1) ? 2u : 0u);
            if (lane == 0) {
                sh.s2[par][0] = s0;
                sh.s2[par][1] = s1;
                sh.f2[par][0] = f0;
                sh.f2[par][1] = f1;
                sh.z2[par] = z;
            }
        }
        if (threadIdx.x == 0) sh.now[par] = wall_clock64();
        __syncthreads();
        bool wait = false;
        if (!d1) {
            if (sh.z1[par]) {
                wait = true;
            } else {
                d1 = true;
                e10 = sh.s1[par][0];
                e11 = sh.s1[par][1];
                if (last && threadIdx.x == 0) {  // the group's aggregate, for later groups
                    status_publish(gcol0 + g, kStAgg | (e10 + agg0));
                    status_publish(gcol1 + g, kStAgg | (e11 + agg1));
                }
            }
        }
        if (!(dg0 && dg1)) {
            const uint32_t z = sh.z2[par];
            if ((!dg0 && (z & 1u)) || (!dg1 && (z & 2u))) {
                wait = true;
            } else {
                if (!dg0) {
                    e20 += sh.s2[par][0];
                    dg0 = sh.f2[par][0] != kLookNone;
                }
                if (!dg1) {
                    e21 += sh.s2[par][1];
                    dg1 = sh.f2[par][1] != kLookNone;
                }
                top -= kWaveSize;
            }
        }
        const uint64_t now = sh.now[par];
        // the farthest group position this round needs (its fallback stops there)
        int f2max = -1;
        if (!dg0) f2max = sh.f2[par][0];
        if (!dg1 && sh.f2[par][1] > f2max) f2max = sh.f2[par][1];
        par ^= 1;
        if (!wait) {
            wait_since = 0;
            continue;
        }
        if (wait_since == 0) wait_since = now;
        if (now - wait_since < a.timeout) {
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        // Waited long enough: wave 0 publishes what this round still misses, computed from the
        // words, then every wave reads the round again.  A compare-and-swap from "nothing" never
        // overwrites what a block or a group's last block has published meanwhile (and what it
        // publishes later is the same aggregate, or the inclusive prefix).
        if (wave == 0) {
            // range r = -1: the earlier blocks of the own group; r >= 0: group top - r, up to
            // the farthest group this round needs
            const int need = f2max < kWaveSize ? f2max : kWaveSize - 1;
            for (int r = d1 ? 0 : -1; r <= need; ++r) {
                const int64_t q = top - r;
                if (r >= 0) {
                    if ((dg0 && dg1) || q < 0) break;
                    if ((status_read(gcol0 + q) & kStMask) != 0 &&
                        (status_read(gcol1 + q) & kStMask) != 0)
                        continue;
                }
                const int64_t lo = r < 0 ? g * G : q * G, hi = r < 0 ? b : lo + G;
                uint64_t t0 = 0, t1 = 0;  // the range's aggregate
                for (int64_t p = lo; p < hi; ++p) {
                    uint64_t x0 = status_read(col0 + p), x1 = status_read(col1 + p);
                    if ((x0 & kStMask) == 0 || (x1 & kStMask) == 0) {
                        block_aggregate<BW>(a, p, x0, x1);
                        if (lane == 0) {
                            status_claim(col0 + p, kStAgg | x0);
                            status_claim(col1 + p, kStAgg | x1);
                        }
                    }
                    t0 += x0 & ~kStMask;
                    t1 += x1 & ~kStMask;
                }
                if (r >= 0 && lane == 0) {
                    status_claim(gcol0 + q, kStAgg | t0);
                    status_claim(gcol1 + q, kStAgg | t1);
                }
            }
        }
        __syncthreads();
        wait_since = 0;
    }
    ex0 = e20 + e10;
    ex1 = e21 + e11;
    if (last && threadIdx.x == 0) {
        status_publish(gcol0 + g, kStIncl | (ex0 + agg0));
        status_publish(gcol1 + g, kStIncl | (ex1 + agg1));
    }
}

}  // namespace svt
