// Register-window conversions for short fields (device code).
//
// A field of at most kWin bytes that lies inside the tile is fetched with
// independent aligned LDS reads and funnel-shifted into registers, so the
// parse below has no dependent memory accesses and only compile-time byte
// indices (no scratch). Each function returns 1 (converted), 0 (not a value
// of the type: a conversion error) or -1 (defer to the general conversions in
// convert.h, e.g. more than 19 significant digits or an exponent). The
// grammar and results are exactly those of convert.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "convert.h"

namespace pp {

constexpr int kWin = 24;

struct Win {
    uint32_t w[kWin / 4];
    __device__ uint32_t at(int i) const { return (w[i >> 2] >> ((i & 3) * 8)) & 0xffu; }
};

// Bytes [off, off + kWin) of an LDS byte array of `size` bytes (dword
// aligned); bytes past `size` read as zero.
__device__ inline Win load_win(const uint32_t* lds_words, int size, int off)
{
    const int d0 = off >> 2;
    const uint32_t sh = (uint32_t)(off & 3);
    const int nw = size >> 2;
    uint32_t raw[kWin / 4 + 1];
#pragma unroll
    for (int k = 0; k <= kWin / 4; ++k) raw[k] = (d0 + k < nw) ? lds_words[d0 + k] : 0u;
    Win r;
#pragma unroll
    for (int k = 0; k < kWin / 4; ++k) r.w[k] = __builtin_amdgcn_alignbyte(raw[k + 1], raw[k], sh);
    return r;
}

__device__ inline int win_int64(const Win& x, int len, int64_t* out)
{
    const uint32_t c0 = x.at(0);
    const bool neg = c0 == '-';
    const int s = (c0 == '+' || c0 == '-') ? 1 : 0;
    if (len - s > 18 || len <= s) return len <= s ? 0 : -1;  // > 18 digits: overflow checks in the general path
    uint64_t mag = 0;
    bool bad = false;
#pragma unroll
    for (int i = 0; i < kWin; ++i) {
        if (i >= s && i < len) {
            const uint32_t d = x.at(i) - '0';
            bad |= d > 9u;
            mag = mag * 10u + d;
        }
    }
    if (bad) return 0;
    *out = neg ? -(int64_t)mag : (int64_t)mag;
    return 1;
}

// [+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+) without exponent, <= 19 significant
// digits, decimal exponent within Clinger's exact range.
__device__ inline int win_float64(const Win& x, int len, double* out)
{
    const uint32_t c0 = x.at(0);
    const bool neg = c0 == '-';
    const int s = (c0 == '+' || c0 == '-') ? 1 : 0;
    uint64_t w = 0;
    int nsig = 0, ndig = 0, frac = 0;
    bool dot = false, other = false;
#pragma unroll
    for (int i = 0; i < kWin; ++i) {
        if (i >= s && i < len) {
            const uint32_t c = x.at(i);
            const uint32_t d = c - '0';
            if (d <= 9u) {
                ++ndig;
                frac += dot;
                nsig += (w != 0 || d != 0);
                w = w * 10u + d;
            } else if (c == '.' && !dot) {
                dot = true;
            } else {
                other = true;  // exponent or a stray byte: the general path decides
            }
        }
    }
    if (other || nsig > 19) return -1;
    if (ndig == 0) return 0;  // "", "+", ".", "-."
    if (w == 0) {
        *out = neg ? -0.0 : 0.0;
        return 1;
    }
    if (w > (1ull << 53) || frac > 22) return -1;
    double v = (double)w;
    if (frac) v = v / exact_pow10(frac);
    *out = neg ? -v : v;
    return 1;
}

__device__ inline bool win_digits(const Win& x, int p, int n, int64_t* v)
{
    int64_t r = 0;
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < n) {
            const uint32_t d = x.at(p + k) - '0';
            ok &= d <= 9u;
            r = r * 10 + d;
        }
    }
    *v = r;
    return ok;
}

__device__ inline int win_date(const Win& x, int len, int64_t* out)
{
    if (len != 10 || x.at(4) != '-' || x.at(7) != '-') return 0;
    int64_t y, m, d;
    if (!win_digits(x, 0, 4, &y) || !win_digits(x, 5, 2, &m) || !win_digits(x, 8, 2, &d)) return 0;
    if (m < 1 || m > 12 || d < 1 || d > days_in_month(y, m)) return 0;
    *out = days_from_civil(y, m, d);
    return 1;
}

__device__ inline int win_timestamp(const Win& x, int len, int64_t* out)
{
    if (len != 19) return 0;
    const uint32_t sep = x.at(10);
    if ((sep != ' ' && sep != 'T') || x.at(13) != ':' || x.at(16) != ':') return 0;
    int64_t days, h, mi, s;
    if (!win_date(x, 10, &days)) return 0;
    if (!win_digits(x, 11, 2, &h) || !win_digits(x, 14, 2, &mi) || !win_digits(x, 17, 2, &s)) return 0;
    if (h > 23 || mi > 59 || s > 59) return 0;
    *out = days * 86400 + h * 3600 + mi * 60 + s;
    return 1;
}

}  // namespace pp
