// Fit helpers shared by the persistent kernels of libsvt: packed 16-bit dot products, the
// exact split offset, mixed-radix stepping over a road's combinations and the record stores.
//
// The fit of section II is p_j = sum_l f[j][l] x_l + q_j followed by the fixed-point shift.
// Constants are int16 and coordinates int13, so the five products of one row are three packed
// 16-bit dot products (v_dot2_i32_i16) once the coordinates of layers (0,1) and (2,3) are
// paired.  The offset is split exactly as q = qh * 2^s + ql with 0 <= ql < 2^s: ql seeds the
// accumulator, so the sum stays inside int32, and
//     floor((S + q) / 2^s) = qh + floor((S + ql) / 2^s)       (exact for every integer S).
#pragma once

#include "svt_common.h"

namespace svt {

constexpr int kRecNone = 0;  // no per-combination records (kept-only output)
constexpr int kRecFit = 1;   // p0..p2 and chi2
constexpr int kRecRows = 2;  // also the constraint rows c0..c2 (each pointer may be null)

// Wave issue priority from a run-time level 0..2 (the instruction takes an immediate).
__device__ __forceinline__ void set_prio(int p) {
    if (p <= 0)
        __builtin_amdgcn_s_setprio(0);
    else if (p == 1)
        __builtin_amdgcn_s_setprio(1);
    else
        __builtin_amdgcn_s_setprio(2);
}

// Per-road indexing data of the current chunk, in LDS, packed into 16 bytes so that the reads
// of the roads one wave works on fall in different banks.  Field widths: n4 <= 8 and
// n2 * n3 <= 64 fit the top byte above a 24-bit division magic; table indices are below
// kTabCap and C <= 8^5, so each fits 16 bits.
struct alignas(16) RoadMeta {
    uint32_t w4;     // division magic of n4 (low 24 bits) | n4 << 24
    uint32_t w23;    // division magic of n2 * n3 (low 24 bits) | (n2 * n3) << 24
    uint32_t b0123;  // table index of the (h0, h1) coordinate pairs | that of the (h2, h3)
                     // pairs << 16
    uint32_t b4c;    // table index of the layer-4 coordinates | combinations << 16
    __device__ int32_t C() const { return static_cast<int32_t>(b4c >> 16); }
    __device__ uint32_t n4() const { return w4 >> 24; }
    __device__ uint32_t n23() const { return w23 >> 24; }
    __device__ int32_t b01() const { return static_cast<int32_t>(b0123 & 0xFFFFu); }
    __device__ int32_t b23() const { return static_cast<int32_t>(b0123 >> 16); }
    __device__ int32_t b4() const { return static_cast<int32_t>(b4c & 0xFFFFu); }
};
static_assert(sizeof(RoadMeta) == 16, "LDS bank spread of the per-road indexing data");

// Per-road constants of the current chunk, packed for the dot products.  144 bytes: with a
// stride of 36 dwords the 16-byte reads of the (up to 8) roads one wave works on start in
// different LDS banks; a 128-byte stride puts them all in the same few banks.
struct alignas(16) RoadConst {
    int32_t F01[6];  // (f[j][0], f[j][1]) as an int16 pair
    int32_t F23[6];  // (f[j][2], f[j][3])
    int32_t F4[6];   // (f[j][4], 0)
    int32_t ql[6];   // q[j] mod 2^shift
    int32_t qh[6];   // floor(q[j] / 2^shift)
    int32_t pad[6];
};
static_assert(sizeof(RoadConst) == 144, "LDS bank spread of the per-road constants");

typedef short v2s __attribute__((ext_vector_type(2)));

// a.lo * b.lo + a.hi * b.hi + c on signed 16-bit halves (v_dot2_i32_i16, no clamping).
__device__ __forceinline__ int32_t dot2(int32_t a, int32_t b, int32_t c) {
    return __builtin_amdgcn_sdot2(__builtin_bit_cast(v2s, a), __builtin_bit_cast(v2s, b), c,
                                  false);
}

// a.lo * b.lo + a.hi * b.hi, the VOP3P form with an inline zero accumulator: the compiler
// otherwise picks the accumulate-in-place encoding and copies a zero into every accumulator.
__device__ __forceinline__ int32_t dot2_zero(int32_t a, int32_t b) {
    int32_t r;
    asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

// floor(k / n) for 0 <= k < 2^15 and 1 <= n <= 64 with m = ceil(2^23 / n) < 2^24, using the
// full-rate 24-bit multiply: (k * 2^9) * m / 2^32 = k * m / 2^23 and k * (m * n - 2^23) <
// 2^15 * 64 < 2^23, so the high word is exactly floor(k / n) (n = 1 included).
__device__ __forceinline__ uint32_t div_small(uint32_t k, uint32_t m) {
    const uint64_t p = static_cast<uint64_t>((k << 9) & 0xFFFFFFu) * static_cast<uint64_t>(m & 0xFFFFFFu);
    return static_cast<uint32_t>(p >> 32);  // v_mul_hi_u32_u24
}

// a * b for a, b < 2^24 (low 32 bits) on the full-rate 24-bit multiplier
__device__ __forceinline__ uint32_t mul_u24(uint32_t a, uint32_t b) {
    uint32_t r;
    asm("v_mul_u32_u24 %0, %1, %2" : "=v"(r) : "v"(a), "v"(b));
    return r;
}

__host__ __device__ constexpr uint32_t magic_of(uint32_t n) {
    return static_cast<uint32_t>(((1u << 23) + n - 1) / n);
}

// 16-byte stores marked non-temporal: the per-combination records are written once and read
// by nothing later in the pass, so they should not displace the staged inputs in the caches.
typedef int32_t nt_i32x4 __attribute__((ext_vector_type(4)));
typedef int64_t nt_i64x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_nt(int32_t *p, const int32_t *v) {
    const nt_i32x4 x = {v[0], v[1], v[2], v[3]};
    __builtin_nontemporal_store(x, reinterpret_cast<nt_i32x4 *>(p));
}
__device__ __forceinline__ void store_nt(int64_t *p, int64_t a, int64_t b) {
    const nt_i64x2 x = {a, b};
    __builtin_nontemporal_store(x, reinterpret_cast<nt_i64x2 *>(p));
}

__device__ __forceinline__ int32_t pack16(int32_t lo, int32_t hi) {
    return static_cast<int32_t>((static_cast<uint32_t>(lo) & 0xFFFFu) |
                                (static_cast<uint32_t>(hi) << 16));
}

struct Fit {
    int32_t v[6];
    int64_t chi2;
};

// Arithmetic forms of the fit, all exact (same values as the int64 definition):
//   kFitSplit  q = qh * 2^s + ql, ql seeds each row, qh is added after the shift;
//   kFitFold   the same with ql carried in the layer-4 pair (shift <= 15, see fit_xyz);
//   kFitNarrow the whole offset seeds each row and the chi-square is summed in 32 bits.  Valid
//              for a constant set whose bounds narrow_ok() accepts: every row's sum stays in
//              int32 for any int13 coordinates, and every chi-square component has |c| < 2^15,
//              so c^2 < 2^30 and the sum of three is below 2^32.
constexpr int kFitSplit = 0;
constexpr int kFitFold = 1;
constexpr int kFitNarrow = 2;

// Whether a constant set allows kFitNarrow: with |x_l| <= 2^12 the row sum S_j + q_j lies in
// [-B_j, B_j] for B_j = 2^12 * sum_l |f_jl| + |q_j|; int32 needs B_j < 2^31, and the shifted
// value floor((S_j + q_j) / 2^s) then has magnitude at most (B_j >> s) + 1, which must stay
// below 2^15 for the chi-square rows (j = 3..5).  f holds the set's 30 constants row-major.
__device__ __forceinline__ bool narrow_ok(const int32_t *f, const int32_t *q, int32_t shift) {
    bool ok = true;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        int64_t sf = 0;
#pragma unroll
        for (int l = 0; l < 5; ++l) sf += f[5 * j + l] < 0 ? -f[5 * j + l] : f[5 * j + l];
        const int64_t b = (sf << 12) + (q[j] < 0 ? -static_cast<int64_t>(q[j]) : q[j]);
        ok &= b < (1ll << 31);
        if (j >= 3) ok &= (b >> shift) + 1 < (1ll << 15);
    }
    return ok;
}

// a * b + c on the full-rate 24-bit signed multiplier (low 32 bits of the result)
__device__ __forceinline__ int32_t mad_i24(int32_t a, int32_t b, int32_t c) {
    int32_t r;
    asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// The six rows of one combination from its three coordinate pairs.  Each sum
//     ql_j + f_j0 x0 + f_j1 x1 + f_j2 x2 + f_j3 x3 + f_j4 x4
// is three packed 16-bit dot products; |sum| < 2^30 + 5 * 2^27 < 2^31, so int32 is exact.
// With FOLD (shift <= 15, so 0 <= ql < 2^15) ql rides in the layer-4 pair, (f_j4, ql_j) .
// (x4, 1), and every row starts from zero instead of from a copy of ql.
// With kFitNarrow the constants hold the whole offset in ql and (f_j4, 0) in F4, and each row
// is three dot products and a shift.
template <int MODE, typename CT>
__device__ __forceinline__ Fit fit_xyz(const CT &c, int32_t x01, int32_t x23, int32_t x4,
                                       int32_t shift) {
    Fit f;
    if constexpr (MODE == kFitNarrow) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            int32_t acc = dot2(c.F01[j], x01, c.ql[j]);
            acc = dot2(c.F23[j], x23, acc);
            acc = dot2(c.F4[j], x4, acc);
            f.v[j] = acc >> shift;
        }
        // each square < 2^30: the 32-bit sum wraps past 2^31 but stays below 2^32
        const int32_t s2 = mad_i24(f.v[3], f.v[3], mad_i24(f.v[4], f.v[4], 0));
        f.chi2 = static_cast<int64_t>(
            static_cast<uint32_t>(mad_i24(f.v[5], f.v[5], s2)));
        return f;
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        int32_t acc;
        if constexpr (MODE == kFitFold) {
            acc = dot2_zero(c.F4[j], x4);
            acc = dot2(c.F01[j], x01, acc);
            acc = dot2(c.F23[j], x23, acc);
        } else {
            acc = dot2(c.F01[j], x01, c.ql[j]);
            acc = dot2(c.F23[j], x23, acc);
            acc = dot2(c.F4[j], x4, acc);
        }
        f.v[j] = (acc >> shift) + c.qh[j];
    }
    f.chi2 = static_cast<int64_t>(f.v[3]) * f.v[3] + static_cast<int64_t>(f.v[4]) * f.v[4] +
             static_cast<int64_t>(f.v[5]) * f.v[5];
    return f;
}

// Fit combination k of a road.  k = (i01 * n23 + i23) * n4 + h4, where i01 = h0 * n1 + h1
// and i23 = h2 * n3 + h3 index the coordinate-pair tables.
template <int MODE, typename CT>
__device__ __forceinline__ Fit fit_combo(const RoadMeta &m, const CT &c, uint32_t k,
                                         const int32_t *XT, int32_t shift) {
    const uint32_t n4 = m.n4(), n23 = m.n23();
    const uint32_t q4 = div_small(k, m.w4);
    const uint32_t h4 = k - mul_u24(q4, n4);
    const uint32_t i01 = div_small(q4, m.w23);
    const uint32_t i23 = q4 - mul_u24(i01, n23);
    return fit_xyz<MODE, CT>(c, XT[m.b01() + static_cast<int32_t>(i01)],
                         XT[m.b23() + static_cast<int32_t>(i23)],
                         XT[m.b4() + static_cast<int32_t>(h4)], shift);
}

// Four consecutive combinations k0, k0 + 1, k0 + 2, k0 + 3 of one road (k0 may lie up to 3
// outside [0, C); those slots get a harmless dummy).  The table indices of the first are
// divided out once and the others stepped from it, carrying h4 -> i23 -> i01.
//
// From a start inside the road (k0 >= 0) the steps need no bounds: past the road's last
// combination h4 and i23 keep wrapping and i01 passes n01 by at most 2 (when n23 * n4 = 1),
// so a read lands in the road's own (h2, h3) or layer-4 table or one entry past the road's
// tables -- still LDS of the staging buffer; such slots are not written.
template <int MODE, typename CT>
__device__ __forceinline__ void fit4(const RoadMeta &m, const CT &c, int32_t k0,
                                     const int32_t *XT, int32_t shift, Fit *out) {
    const int32_t C = m.C();
    const uint32_t n4 = m.n4(), n23 = m.n23();
    if (MODE == kFitNarrow && k0 >= 0) {
        const uint32_t k = static_cast<uint32_t>(k0);
        const uint32_t q4 = div_small(k, m.w4);
        uint32_t h4 = k - mul_u24(q4, n4);
        uint32_t i01 = div_small(q4, m.w23);
        uint32_t i23 = q4 - mul_u24(i01, n23);
        const int32_t *t01 = XT + m.b01(), *t23 = XT + m.b23(), *t4 = XT + m.b4();
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            out[e] = fit_xyz<MODE, CT>(c, t01[i01], t23[i23], t4[h4], shift);
            if (e < 3) {
                ++h4;
                const bool w4 = h4 == n4;
                h4 = w4 ? 0u : h4;
                i23 += w4 ? 1u : 0u;
                const bool w23 = i23 == n23;
                i23 = w23 ? 0u : i23;
                i01 += w23 ? 1u : 0u;
            }
        }
        return;
    }
    const uint32_t k = static_cast<uint32_t>(k0 < 0 ? 0 : (k0 > C - 1 ? C - 1 : k0));
    const uint32_t q4 = div_small(k, m.w4);
    uint32_t h4 = k - mul_u24(q4, n4);
    uint32_t i01 = div_small(q4, m.w23);
    uint32_t i23 = q4 - mul_u24(i01, n23);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        out[e] = fit_xyz<MODE, CT>(c, XT[m.b01() + static_cast<int32_t>(i01)],
                               XT[m.b23() + static_cast<int32_t>(i23)],
                               XT[m.b4() + static_cast<int32_t>(h4)], shift);
        if (e < 3 && k0 + e >= 0 && k0 + e + 1 < C) {  // step to k0 + e + 1
            ++h4;
            const bool w4 = h4 == n4;
            h4 = w4 ? 0u : h4;
            i23 += w4 ? 1u : 0u;
            const bool w23 = i23 == n23;
            i23 = w23 ? 0u : i23;
            i01 += w23 ? 1u : 0u;
        }
    }
}

// int16 element i of a constant set's f[6][5], from its first 64 bytes held as 8-byte words
__device__ __forceinline__ int32_t f_el(const uint2 *fw, int i) {
    const uint2 w = fw[i >> 2];
    const uint32_t d = ((i >> 1) & 1) ? w.y : w.x;
    return static_cast<int32_t>(static_cast<int16_t>((i & 1) ? (d >> 16) : (d & 0xFFFFu)));
}

// Write the records of one group of 4 consecutive combinations (global index gi of slot 0):
// one 16-byte store per array when all four slots are written, else one store per slot.
template <int REC>
__device__ __forceinline__ void store_group(const svt_fitrec &rec, uint8_t *accept, int64_t gi,
                                            uint32_t slots,
                                            uint32_t acc_bits, const int32_t *vp0,
                                            const int32_t *vp1, const int32_t *vp2,
                                            const int32_t *vc0, const int32_t *vc1,
                                            const int32_t *vc2, const int64_t *vchi) {
    if (slots == 0xF) {
        if (REC != kRecNone) {  // per-combination records (not in kept-only mode)
            store_nt(rec.p0 + gi, vp0);
            store_nt(rec.p1 + gi, vp1);
            store_nt(rec.p2 + gi, vp2);
            store_nt(rec.chi2 + gi, vchi[0], vchi[1]);
            store_nt(rec.chi2 + gi + 2, vchi[2], vchi[3]);
        }
        if (REC == kRecRows) {
            if (rec.c0) store_nt(rec.c0 + gi, vc0);
            if (rec.c1) store_nt(rec.c1 + gi, vc1);
            if (rec.c2) store_nt(rec.c2 + gi, vc2);
        }
        const uint32_t accw = (acc_bits & 1u) | ((acc_bits & 2u) << 7) |
                              ((acc_bits & 4u) << 14) | ((acc_bits & 8u) << 21);
        *reinterpret_cast<uint32_t *>(accept + gi) = accw;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            if (slots & (1u << e)) {
                if (REC != kRecNone) {
                    rec.p0[gi + e] = vp0[e];
                    rec.p1[gi + e] = vp1[e];
                    rec.p2[gi + e] = vp2[e];
                    rec.chi2[gi + e] = vchi[e];
                }
                if (REC == kRecRows) {
                    if (rec.c0) rec.c0[gi + e] = vc0[e];
                    if (rec.c1) rec.c1[gi + e] = vc1[e];
                    if (rec.c2) rec.c2[gi + e] = vc2[e];
                }
                accept[gi + e] = (acc_bits >> e) & 1u;
            }
        }
    }
}

}  // namespace svt
