// Field conversions for the typed columns (Sec. 3.3: a thread converts a
// field's symbol string to its column's type). The paper fixes no grammar;
// the one implemented here:
//   INT64        [+-]?[0-9]+ that fits int64
//   FLOAT64      [+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+)([eE][+-]?[0-9]+)?, the
//                binary64 nearest to the decimal value, ties to even
//   TIMESTAMP_S  YYYY-MM-DD[ T]hh:mm:ss, seconds 0..59, UTC
//   DATE_DAYS    YYYY-MM-DD
// Device code only. Bytes are fetched through a functor so a field can be read
// from the tile staged in LDS or, for the part before the tile, from HBM.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pp {

__device__ inline bool is_dig(uint32_t c) { return c - '0' < 10u; }

// ---- INT64 ----------------------------------------------------------------
template <class Src>
__device__ inline bool conv_int64(const Src& src, int64_t b, int64_t e, int64_t* out)
{
    int64_t i = b;
    uint32_t c0 = src(i);
    bool neg = false;
    if (c0 == '+' || c0 == '-') { neg = c0 == '-'; ++i; }
    if (i == e) return false;
    const uint64_t limit = neg ? (1ull << 63) : (1ull << 63) - 1;
    uint64_t mag = 0;
    for (; i < e; ++i) {
        uint32_t d = src(i) - '0';
        if (d > 9u) return false;
        if (mag > (limit - d) / 10u) return false;
        mag = mag * 10u + d;
    }
    *out = neg ? (int64_t)(0ull - mag) : (int64_t)mag;
    return true;
}

// ---- calendar ----------------------------------------------------------------
__device__ __forceinline__ bool is_leap(int64_t y) { return (y % 4 == 0 && y % 100 != 0) || y % 400 == 0; }

__device__ __forceinline__ int days_in_month(int64_t y, int64_t m)
{
    // 30 + (m + m/8) % 2 gives 31/30 alternating with the July/August switch;
    // February is fixed up below.
    int d = 30 + (int)((m + m / 8) & 1);
    if (m == 2) d = is_leap(y) ? 29 : 28;
    return d;
}

// Days since 1970-01-01 of a proleptic Gregorian date, by Hinnant's
// era/day-of-era method ("chrono-compatible low-level date algorithms"):
// shift the year to start in March so the leap day is last, split into
// 400-year eras of 146097 days, and count within the era.
__device__ __forceinline__ int64_t days_from_civil(int64_t y, int64_t m, int64_t d)
{
    y -= m <= 2;
    const int64_t era = (y >= 0 ? y : y - 399) / 400;
    const int64_t yoe = y - era * 400;                      // [0, 399]
    const int64_t mp = (m + 9) % 12;                        // March = 0
    const int64_t doy = (153 * mp + 2) / 5 + d - 1;         // [0, 365]
    const int64_t doe = yoe * 365 + yoe / 4 - yoe / 100 + doy;  // [0, 146096]
    return era * 146097 + doe - 719468;
}

template <class Src>
__device__ inline bool digits_at(const Src& src, int64_t p, int n, int64_t* v)
{
    int64_t x = 0;
    for (int k = 0; k < n; ++k) {
        uint32_t d = src(p + k) - '0';
        if (d > 9u) return false;
        x = x * 10 + d;
    }
    *v = x;
    return true;
}

template <class Src>
__device__ inline bool conv_date(const Src& src, int64_t b, int64_t e, int64_t* out)
{
    if (e - b != 10 || src(b + 4) != '-' || src(b + 7) != '-') return false;
    int64_t y, m, d;
    if (!digits_at(src, b, 4, &y) || !digits_at(src, b + 5, 2, &m) || !digits_at(src, b + 8, 2, &d))
        return false;
    if (m < 1 || m > 12 || d < 1 || d > days_in_month(y, m)) return false;
    *out = days_from_civil(y, m, d);
    return true;
}

template <class Src>
__device__ inline bool conv_timestamp(const Src& src, int64_t b, int64_t e, int64_t* out)
{
    if (e - b != 19) return false;
    uint32_t sep = src(b + 10);
    if ((sep != ' ' && sep != 'T') || src(b + 13) != ':' || src(b + 16) != ':') return false;
    int64_t days, h, mi, s;
    if (!conv_date(src, b, b + 10, &days)) return false;
    if (!digits_at(src, b + 11, 2, &h) || !digits_at(src, b + 14, 2, &mi) || !digits_at(src, b + 17, 2, &s))
        return false;
    if (h > 23 || mi > 59 || s > 59) return false;
    *out = days * 86400 + h * 3600 + mi * 60 + s;
    return true;
}

// ---- FLOAT64 ------------------------------------------------------------------
// Tier 1 (Clinger 1990): at most 19 significant digits giving a mantissa
// w <= 2^53 and a decimal exponent in [-22, 22]. Then w and 10^|e| are both
// exact binary64 values and one IEEE multiply or divide rounds correctly.
// Tier 2: exact decimal scaling by powers of two on a digit buffer, then
// rounding to 53 bits with ties to even (the "simple decimal conversion"
// method; 800 retained digits plus a sticky flag decide every halfway case).

__device__ __forceinline__ double exact_pow10(int k)
{
    // 10^k for 0 <= k <= 22 by binary exponentiation. Every partial product
    // is some 10^j with j <= 22, exactly representable in binary64, so each
    // multiplication is exact and no table in memory is needed.
    double r = 1.0;
    if (k & 1) r *= 1e1;
    if (k & 2) r *= 1e2;
    if (k & 4) r *= 1e4;
    if (k & 8) r *= 1e8;
    if (k & 16) r *= 1e16;
    return r;
}

constexpr int kDecCap = 800;
constexpr int kDecRoom = 19;  // 2^60 < 10^19: a left shift by <= 60 adds <= 19 digits

struct Decimal {
    uint8_t d[kDecCap + kDecRoom];
    int nd;      // number of digits in d
    int dp;      // value = 0.d[0]d[1]... * 10^dp
    bool trunc;  // nonzero digits were dropped past kDecCap
};

__device__ inline void dec_trim(Decimal& a)
{
    while (a.nd > 0 && a.d[a.nd - 1] == 0) --a.nd;
    if (a.nd == 0) a.dp = 0;
}

// a /= 2^k for 1 <= k <= 60: long division of the digit string.
__device__ inline void dec_shr(Decimal& a, int k)
{
    const uint64_t mask = (1ull << k) - 1;
    uint64_t rem = 0;
    int r = 0, w = 0, dp = a.dp;
    bool started = false;
    while (r < a.nd || rem != 0) {
        rem = rem * 10 + (r < a.nd ? a.d[r] : 0);
        ++r;
        uint32_t q = (uint32_t)(rem >> k);
        rem &= mask;
        if (!started) {
            if (q == 0) { --dp; continue; }
            started = true;
        }
        if (w < kDecCap) a.d[w++] = (uint8_t)q;
        else if (q) a.trunc = true;
    }
    a.nd = w;
    a.dp = dp;
    dec_trim(a);
}

// a *= 2^k for 1 <= k <= 60.
__device__ inline void dec_shl(Decimal& a, int k)
{
    for (int i = a.nd - 1; i >= 0; --i) a.d[i + kDecRoom] = a.d[i];
    uint64_t carry = 0;
    for (int i = kDecRoom + a.nd - 1; i >= kDecRoom; --i) {
        uint64_t v = ((uint64_t)a.d[i] << k) + carry;
        a.d[i] = (uint8_t)(v % 10);
        carry = v / 10;
    }
    int p = kDecRoom - 1;
    while (carry) {
        a.d[p--] = (uint8_t)(carry % 10);
        carry /= 10;
    }
    const int start = p + 1;
    int nd = kDecRoom + a.nd - start;
    a.dp += kDecRoom - start;
    for (int i = 0; i < nd; ++i) a.d[i] = a.d[start + i];
    if (nd > kDecCap) {
        for (int i = kDecCap; i < nd; ++i)
            if (a.d[i]) a.trunc = true;
        nd = kDecCap;
    }
    a.nd = nd;
    dec_trim(a);
}

__device__ __forceinline__ double dec_to_double(Decimal& a, bool neg);

template <class Src>
__device__ __noinline__ double float_slow(const Src& src, int64_t b, int64_t e)
{
    Decimal a;
    a.nd = 0;
    a.dp = 0;
    a.trunc = false;
    int64_t i = b;
    bool neg = false;
    uint32_t c = src(i);
    if (c == '+' || c == '-') { neg = c == '-'; ++i; }
    bool dot = false;
    for (; i < e; ++i) {
        c = src(i);
        if (c == '.') { dot = true; continue; }
        if (!is_dig(c)) break;
        uint32_t d = c - '0';
        if (a.nd == 0 && d == 0) {
            if (dot) --a.dp;
            continue;
        }
        if (!dot) ++a.dp;
        if (a.nd < kDecCap) a.d[a.nd++] = (uint8_t)d;
        else if (d) a.trunc = true;
    }
    if (i < e) {  // exponent part (grammar already checked)
        ++i;
        bool eneg = false;
        c = src(i);
        if (c == '+' || c == '-') { eneg = c == '-'; ++i; }
        int64_t ex = 0;
        for (; i < e; ++i)
            if (ex < 100000000) ex = ex * 10 + (src(i) - '0');
        a.dp += (int)(eneg ? -ex : ex);
    }
    return dec_to_double(a, neg);
}

// The binary64 nearest to the decimal a (ties to even), negated if neg. a
// holds the significant digits as read (trailing zeros included).
__device__ __forceinline__ double dec_to_double(Decimal& a, bool neg)
{
    dec_trim(a);
    const double sgn = neg ? -1.0 : 1.0;
    if (a.nd == 0) return sgn * 0.0;
    if (a.dp > 310) return sgn * __builtin_huge_val();
    if (a.dp < -330) return sgn * 0.0;
    int e2 = 0;
    while (a.dp > 0) {
        int n = a.dp >= 20 ? 60 : 3 * a.dp;
        dec_shr(a, n);
        e2 += n;
    }
    while (a.dp < 0 || (a.dp == 0 && a.d[0] < 5)) {
        int n = a.dp < 0 ? (-a.dp >= 20 ? 60 : 3 * -a.dp) : 1;
        dec_shl(a, n);
        e2 -= n;
    }
    // value = 0.d.. * 2^e2 with 0.d.. in [0.5, 1), i.e. (2 * 0.d..) * 2^(e2-1)
    int E = e2 - 1;
    if (E < -1022) {
        int s = -1022 - E;
        while (s > 0) {
            int n = s > 60 ? 60 : s;
            dec_shr(a, n);
            s -= n;
        }
        E = -1022;
    }
    if (E > 1023) return sgn * __builtin_huge_val();
    dec_shl(a, 53);
    uint64_t m = 0;
    if (a.dp >= 0) {
        for (int k = 0; k < a.dp; ++k) m = m * 10 + (k < a.nd ? a.d[k] : 0);
        if (a.dp < a.nd) {
            uint32_t rd = a.d[a.dp];
            bool more = a.trunc || a.dp + 1 < a.nd;
            if (rd > 5 || (rd == 5 && (more || (m & 1)))) ++m;
        }
    }
    if (m == (1ull << 53)) {
        m >>= 1;
        ++E;
        if (E > 1023) return sgn * __builtin_huge_val();
    }
    uint64_t bits;
    if (m < (1ull << 52)) bits = m;  // subnormal (or zero)
    else bits = ((uint64_t)(E + 1023) << 52) | (m & ((1ull << 52) - 1));
    if (neg) bits |= 1ull << 63;
    return __builtin_bit_cast(double, bits);
}

// [+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+)([eE][+-]?[0-9]+)?: the grammar alone
// (what conv_float64 accepts), without the conversion.
template <class Src>
__device__ inline bool float_grammar(const Src& src, int64_t b, int64_t e)
{
    int64_t i = b, nd = 0;
    if (i < e && (src(i) == '+' || src(i) == '-')) ++i;
    for (; i < e && is_dig(src(i)); ++i) ++nd;
    if (i < e && src(i) == '.')
        for (++i; i < e && is_dig(src(i)); ++i) ++nd;
    if (nd == 0) return false;
    if (i < e && (src(i) | 0x20u) == 'e') {
        ++i;
        if (i < e && (src(i) == '+' || src(i) == '-')) ++i;
        int64_t ne = 0;
        for (; i < e && is_dig(src(i)); ++i) ++ne;
        if (ne == 0) return false;
    }
    return i == e;
}

template <class Src>
__device__ inline bool conv_float64(const Src& src, int64_t b, int64_t e, double* out)
{
    int64_t i = b;
    bool neg = false;
    uint32_t c = src(i);
    if (c == '+' || c == '-') { neg = c == '-'; ++i; }
    uint64_t w = 0;
    int nsig = 0;
    int64_t nint = 0, nfrac = 0, dropped_int = 0, kept_frac = 0;
    bool trunc = false;
    for (; i < e; ++i) {
        c = src(i);
        if (!is_dig(c)) break;
        uint32_t d = c - '0';
        ++nint;
        if (nsig == 0 && d == 0) continue;
        if (nsig < 19) { w = w * 10 + d; ++nsig; }
        else { ++dropped_int; trunc |= d != 0; }
    }
    if (i < e && src(i) == '.') {
        for (++i; i < e; ++i) {
            c = src(i);
            if (!is_dig(c)) break;
            uint32_t d = c - '0';
            ++nfrac;
            if (nsig == 0 && d == 0) { ++kept_frac; continue; }
            if (nsig < 19) { w = w * 10 + d; ++nsig; ++kept_frac; }
            else trunc |= d != 0;
        }
    }
    if (nint + nfrac == 0) return false;
    int64_t ex = 0;
    if (i < e && (src(i) | 0x20u) == 'e') {
        ++i;
        bool eneg = false;
        if (i < e && (src(i) == '+' || src(i) == '-')) { eneg = src(i) == '-'; ++i; }
        int64_t ne = 0;
        for (; i < e; ++i) {
            c = src(i);
            if (!is_dig(c)) break;
            if (ex < 100000000) ex = ex * 10 + (c - '0');
            ++ne;
        }
        if (ne == 0) return false;
        if (eneg) ex = -ex;
    }
    if (i != e) return false;
    if (w == 0) { *out = neg ? -0.0 : 0.0; return true; }
    const int64_t e10 = ex + dropped_int - kept_frac;
    if (!trunc && w <= (1ull << 53) && e10 >= -22 && e10 <= 22) {
        double v = (double)w;
        v = e10 < 0 ? v / exact_pow10((int)-e10) : v * exact_pow10((int)e10);
        *out = neg ? -v : v;
        return true;
    }
    *out = float_slow(src, b, e);
    return true;
}

}  // namespace pp
