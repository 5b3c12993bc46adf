// Register-window conversions for short fields (device code).
//
// A field of at most kWin bytes that lies inside the tile is fetched with
// independent aligned LDS reads and funnel-shifted into registers, so the
// parse below has no dependent memory accesses and only compile-time byte
// indices (no scratch). Numbers are parsed byte-serially with selects, dates
// and times at fixed positions. Each function returns 1 (converted), 0 (not a value of the type: a conversion
// error) or -1 (defer to the general conversions in convert.h, e.g. more than
// 19 significant digits or an exponent). The grammar and results are exactly
// those of convert.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "convert.h"

namespace pp {

constexpr int kWin = 24;

struct Win {
    uint32_t w[kWin / 4];
    __device__ __forceinline__ uint32_t at(int i) const { return (w[i >> 2] >> ((i & 3) * 8)) & 0xffu; }
};

// Bytes [off, off + kWin) of a padded LDS buffer, fetched in two steps: the
// first 8 bytes always, the rest only when a lane of the wavefront has a
// field longer than 8 bytes (bytes past 8 read as zero otherwise; the parses
// below never look at them then).
__device__ __forceinline__ Win load_win_lazy(const uint32_t* lds_words, int off, int len)
{
    const int d0 = off >> 2;
    const uint32_t sh = (uint32_t)(off & 3);
    Win r;
    const uint32_t a0 = lds_words[d0], a1 = lds_words[d0 + 1], a2 = lds_words[d0 + 2];
    r.w[0] = __builtin_amdgcn_alignbyte(a1, a0, sh);
    r.w[1] = __builtin_amdgcn_alignbyte(a2, a1, sh);
#pragma unroll
    for (int k = 2; k < kWin / 4; ++k) r.w[k] = 0u;
    if (__builtin_amdgcn_ballot_w64(len > 8) != 0) {
        uint32_t raw[kWin / 4 + 1];
        raw[2] = a2;
#pragma unroll
        for (int k = 3; k <= kWin / 4; ++k) raw[k] = lds_words[d0 + k];
#pragma unroll
        for (int k = 2; k < kWin / 4; ++k) r.w[k] = __builtin_amdgcn_alignbyte(raw[k + 1], raw[k], sh);
    }
    return r;
}

// Byte-serial parses over a left-aligned window (the field starts at byte 0),
// fully unrolled and branch-free per byte (selects, no divergent ifs); the
// loop ends once no lane of the wavefront is still inside its field.
__device__ __forceinline__ bool wave_any(bool p) { return __builtin_amdgcn_ballot_w64(p) != 0; }

__device__ __forceinline__ int ser_int64(const Win& x, int len, int64_t* out)
{
    const uint32_t c0 = x.at(0);
    const bool neg = c0 == '-';
    const bool sg = (c0 == '+') | (c0 == '-');
    if (len - (int)sg > 18) return -1;  // overflow checks in the general path
    if (len <= (int)sg) return 0;
    uint32_t m32 = 0;  // the first nine bytes fit 32 bits
    uint64_t mag = 0;
    bool bad = false;
#pragma unroll
    for (int q = 0; q < 5; ++q) {  // a dword of the window per step (19 bytes at most)
        if (!wave_any(4 * q < len)) break;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * q + j;
            if (i >= 19) break;
            const uint32_t d = x.at(i) - '0';
            const bool in = i == 0 ? !sg : (i < len);
            bad |= in & (d > 9u);
            if (i < 9) {
                m32 = in ? m32 * 10u + d : m32;
                if (i == 8) mag = m32;
            } else {
                const uint64_t nx = mag * 10u + d;
                mag = in ? nx : mag;
            }
        }
    }
    if (len <= 8) mag = m32;  // the loop may have ended before byte 8
    if (bad) return 0;
    *out = neg ? -(int64_t)mag : (int64_t)mag;
    return 1;
}

// [+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+) with <= 19 digits and no exponent, in
// Clinger's exact range (digit string below 2^53, at most 22 fraction
// digits); anything else goes to the general path. The digits of the first
// 8 bytes are accumulated in 32-bit integers (exact), the rest in double
// precision from there: every partial value is an integer no larger than
// the final one, so while the final value is below 2^53 each step v*10+d
// is exact; a larger final value is caught by the range check (rounding is
// monotonic, so it cannot land below 2^53).
// pow10: 10^k for 0 <= k <= 22 (a table the caller keeps in LDS).
__device__ __forceinline__ int ser_float64(const Win& x, int len, double* out, const double* pow10)
{
    const uint32_t c0 = x.at(0);
    const bool neg = c0 == '-';
    const bool sg = (c0 == '+') | (c0 == '-');
    // the digits of bytes 0-7 in 32-bit integer arithmetic (at most 8 of
    // them: below 10^8), the rest in double precision from that value on
    uint32_t m32 = 0;
    double v = 0.0;
    bool wide = false;  // the wavefront went past byte 7 (uniform)
    uint32_t dots = 0;  // bit i: byte i is a decimal point
    bool other = false;
#pragma unroll
    for (int q = 0; q < kWin / 4; ++q) {  // a dword of the window per step
        if (!wave_any(4 * q < len)) break;
        if (q == 2) {
            v = (double)m32;
            wide = true;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int i = 4 * q + j;
            const uint32_t c = x.at(i);
            const uint32_t d = c - '0';
            const bool in = i == 0 ? (!sg & (len > 0)) : (i < len);
            const bool isd = in & (d <= 9u);
            const bool isdot = in & (c == '.');
            other |= in & !isd & !isdot;
            if (q < 2) {
                m32 = isd ? m32 * 10u + d : m32;
            } else {
                // a digit: v*10 + d; anything else: v*1 + 0 (no select of v needed)
                const uint32_t dz = isd ? d : 0u;
                v = __builtin_fma(v, isd ? 10.0 : 1.0, (double)dz);
            }
            dots = isdot ? dots | (1u << i) : dots;
        }
    }
    if (!wide) v = (double)m32;
    const int ndot = __popc(dots);
    const int nd = len - (int)sg - ndot;  // digits, when nothing else is in the field
    if (other || ndot > 1 || nd > 19) return -1;
    if (nd <= 0) return 0;
    if (v == 0.0) {
        *out = neg ? -0.0 : 0.0;
        return 1;
    }
    const int frac = ndot ? len - 1 - (31 - __clz((int)dots)) : 0;
    if (!(v < 9007199254740992.0) || frac > 22) return -1;
    if (frac) v = v / pow10[frac];
    *out = neg ? -v : v;
    return 1;
}

// Per byte of a word: 0x80 where the byte is zero (exact: no carries
// between bytes), and 0x80 where the byte is above 9.
__device__ __forceinline__ uint32_t zero_bytes(uint32_t y)
{
    return ~(((y & 0x7f7f7f7fu) + 0x7f7f7f7fu) | y | 0x7f7f7f7fu);
}
__device__ __forceinline__ uint32_t above9_bytes(uint32_t t)
{
    return (((t & 0x7f7f7f7fu) + 0x76767676u) | t) & 0x80808080u;
}

// ser_float64 for a field of at most 8 bytes, with word-parallel steps in
// place of the byte loop (same grammar, same results) and no branches: a
// sign reads as a leading zero digit; the field is right-aligned in a 64-bit
// word with the ASCII '0' bits cleared (digits become their values, the
// bytes shifted in are leading zeros, bytes past the field drop out); a
// decimal point is found by an exact per-byte zero test, every other byte
// must be at most 9, the point's byte is squeezed out by shifting the bytes
// before it up one, and the eight digits (at most 10^8 - 1, so the range
// checks always pass) are combined by 8-bit dot products. Without a point
// the division is by 10^0 = 1, which is exact.
__device__ __forceinline__ int ser_float64_8(const Win& x, int len, double* out, const double* pow10)
{
    typedef unsigned long long u64;
    const uint32_t c0 = x.w[0] & 0xffu;
    const bool neg = c0 == '-';
    const uint32_t k = c0 - 0x2bu;  // '+' and '-' are 0x2b and 0x2d: bits 0 and 2 of 5
    const bool sg = ((0x5u >> (k & 31u)) & (k < 3u ? 1u : 0u)) != 0u;
    const uint32_t w0 = (x.w[0] & ~0xffu) | (sg ? 0x30u : c0);
    const u64 raw = ((u64)(x.w[1] ^ 0x30303030u) << 32) | (w0 ^ 0x30303030u);
    const u64 t = raw << (64u - 8u * (uint32_t)len);  // len in [1, 8]
    const uint32_t tl = (uint32_t)t, th = (uint32_t)(t >> 32);
    const uint32_t zl = zero_bytes(tl ^ 0x1e1e1e1eu), zh = zero_bytes(th ^ 0x1e1e1e1eu);  // '.' ^ '0' = 0x1e
    const uint32_t bad = (above9_bytes(tl) & ~zl) | (above9_bytes(th) & ~zh);
    const int ndot = __popc(zl) + __popc(zh);
    const int nd = len - (int)sg - ndot;
    const uint32_t pz = zl ? (uint32_t)__builtin_ctz(zl) : 32u + (uint32_t)__builtin_ctz(zh | 0x80000000u);
    const uint32_t p = pz >> 3;  // the point's byte (7 when there is none: unused)
    const u64 after = (~0ull << (8u * p)) << 8;  // the bytes after the point
    const u64 d = ndot ? ((t & after) | ((t << 8) & ~after)) : t;
    const int frac = ndot ? 7 - (int)p : 0;
    const uint32_t lo = (uint32_t)d, hi = (uint32_t)(d >> 32);
    // byte 0 is the most significant digit: d0*100 + d1*10 + d2, then *10 + d3
    const uint32_t a = __builtin_amdgcn_udot4(lo, 0x00010a64u, 0u, false);
    const uint32_t b = __builtin_amdgcn_udot4(hi, 0x00010a64u, 0u, false);
    const uint32_t ha = __builtin_amdgcn_udot4(lo, 0x01000000u, __umul24(a, 10u), false);
    const uint32_t hb = __builtin_amdgcn_udot4(hi, 0x01000000u, __umul24(b, 10u), false);
    const double v = (double)(__umul24(ha, 10000u) + hb) / pow10[frac];
    *out = neg ? -v : v;
    return (bad != 0u || ndot > 1) ? -1 : (nd > 0 ? 1 : 0);
}

// The calendar for four-digit years (0000-9999) in 32-bit arithmetic: the
// same definitions as convert.h (Gregorian leap rule; Hinnant's era/day-of-
// era count from March), with the year shifted by one 400-year era so that
// every quantity stays non-negative.
__device__ __forceinline__ uint32_t days_in_month4(uint32_t y, uint32_t m)
{
    // y % 400 == 0 exactly when y % 100 == 0 and y % 16 == 0
    const bool leap = ((y & 3u) == 0) & ((y % 100u != 0) | ((y & 15u) == 0));
    const uint32_t d = 30u + ((m + m / 8u) & 1u);
    return m == 2 ? (leap ? 29u : 28u) : d;
}

__device__ __forceinline__ int64_t days_from_civil4(uint32_t y, uint32_t m, uint32_t d)
{
    const uint32_t ys = y + 400u - (m <= 2u);  // [399, 10399]
    const uint32_t era = ys / 400u;
    const uint32_t yoe = ys - era * 400u;
    const uint32_t mp = m > 2u ? m - 3u : m + 9u;  // March = 0
    const uint32_t doy = (153u * mp + 2u) / 5u + d - 1u;
    const uint32_t doe = yoe * 365u + yoe / 4u - yoe / 100u + doy;
    return (int64_t)era * 146097 + (int64_t)doe - 719468 - 146097;
}

// Fixed-layout date and time fields, checked and converted a word at a
// time: the window's words with the ASCII '0' bits cleared hold digit values
// in the digit places, every digit place is checked to be at most 9 and
// every separator compared in one step per word, each number is one 8-bit
// dot product of its digits with their place values, and the results are
// combined with & (no short-circuit branches). (Checked on the GPU against
// the byte-by-byte form they replace on 67 million windows: identical.)
// The YYYY-MM-DD of bytes 0-9 (words w0-w2): y, m, d, and nonzero when a
// digit place holds no digit or a separator is not '-'.
__device__ __forceinline__ uint32_t ymd_bad(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t& y, uint32_t& m,
                                           uint32_t& d)
{
    const uint32_t t0 = w0 ^ 0x30303030u, t1 = w1 ^ 0x30303030u, t2 = w2 ^ 0x30303030u;
    // digits: bytes 0-3, 5-6, 8-9; '-' at bytes 4 and 7
    const uint32_t bad = above9_bytes(t0) | (above9_bytes(t1) & 0x00808000u) | (above9_bytes(t2) & 0x00008080u) |
                         ((w1 & 0xff0000ffu) ^ 0x2d00002du);
    y = __builtin_amdgcn_udot4(t0, 0x01000000u, __umul24(__builtin_amdgcn_udot4(t0, 0x00010a64u, 0u, false), 10u), false);
    m = __builtin_amdgcn_udot4(t1, 0x00010a00u, 0u, false);
    d = __builtin_amdgcn_udot4(t2, 0x0000010au, 0u, false);
    return bad;
}

__device__ __forceinline__ int win_date(const Win& x, int len, int64_t* out)
{
    uint32_t y, m, d;
    bool ok = ymd_bad(x.w[0], x.w[1], x.w[2], y, m, d) == 0u && len == 10;
    ok &= (m >= 1) & (m <= 12) & (d >= 1);
    ok &= d <= days_in_month4(y, ok ? m : 1);
    *out = ok ? days_from_civil4(y, m, d) : 0;
    return ok;
}

__device__ __forceinline__ int win_timestamp(const Win& x, int len, int64_t* out)
{
    uint32_t y, m, d;
    const uint32_t w2 = x.w[2], w3 = x.w[3], w4 = x.w[4];
    const uint32_t t2 = w2 ^ 0x30303030u, t3 = w3 ^ 0x30303030u, t4 = w4 ^ 0x30303030u;
    const uint32_t sep = (w2 >> 16) & 0xffu;
    // digits: bytes 11-12, 14-15, 17-18; ':' at bytes 13 and 16; ' ' or 'T' at byte 10
    const uint32_t bad = ymd_bad(x.w[0], x.w[1], w2, y, m, d) | (above9_bytes(t2) & 0x80000000u) |
                         (above9_bytes(t3) & 0x80800080u) | (above9_bytes(t4) & 0x00808000u) |
                         ((w3 & 0x0000ff00u) ^ 0x00003a00u) | ((w4 & 0x000000ffu) ^ 0x0000003au);
    bool ok = bad == 0u && len == 19 && ((sep == ' ') | (sep == 'T'));
    const uint32_t h = __builtin_amdgcn_udot4(t2, 0x0a000000u, t3 & 0xffu, false);
    const uint32_t mi = __builtin_amdgcn_udot4(t3, 0x010a0000u, 0u, false);
    const uint32_t sc = __builtin_amdgcn_udot4(t4, 0x00010a00u, 0u, false);
    ok &= (m >= 1) & (m <= 12) & (d >= 1) & (h <= 23) & (mi <= 59) & (sc <= 59);
    ok &= d <= days_in_month4(y, ok ? m : 1);
    *out = ok ? days_from_civil4(y, m, d) * 86400 + (int64_t)(h * 3600u + mi * 60u + sc) : 0;
    return ok;
}

}  // namespace pp
