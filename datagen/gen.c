/*
 * Seeded synthetic inputs: delimiter-separated text shaped like the paper's
 * workloads (a numeric taxi-trip-like CSV, a text-heavy review-like CSV with
 * quoted free text, mixed dialects, and an extended web-server log). None of
 * the paper's datasets is used; only their shapes are imitated.
 *
 * This file holds no parsing arithmetic. It draws values, formats them as
 * text, and records what it wrote (field starts, content spans, the drawn
 * values) as ground truth for tests.
 *
 * Randomness: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014), one independent stream per block of
 * records, keyed by (seed, block index), so a block's bytes do not depend on
 * how many threads generate the buffer.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct { uint64_t s; } rng_t;

static uint64_t splitmix64(rng_t* r)
{
    uint64_t z = (r->s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static rng_t rng_for(uint64_t seed, uint64_t block)
{
    rng_t r = {seed * 0x2545F4914F6CDD1Dull + block * 0x9E3779B97F4A7C15ull + 1};
    splitmix64(&r);
    return r;
}

static uint64_t below(rng_t* r, uint64_t n) { return splitmix64(r) % n; }
static double unit(rng_t* r) { return (double)(splitmix64(r) >> 11) * (1.0 / 9007199254740992.0); }
static int64_t uniform_i(rng_t* r, int64_t lo, int64_t hi) { return lo + (int64_t)below(r, (uint64_t)(hi - lo + 1)); }
static int bern(rng_t* r, double p) { return unit(r) < p; }

static double normal(rng_t* r)
{
    double u1 = unit(r), u2 = unit(r);
    if (u1 < 1e-300) u1 = 1e-300;
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ---- truth ------------------------------------------------------------ */
/* Per (record, column) of a block, indexes rec*ncols + col:
 *   fbeg: raw first byte of the field, relative to the block start
 *   vbeg, vend: content span (inside enclosing quotes/brackets)
 *   ival: drawn integer / epoch value / float mantissa; aux: float decimals
 *   kind: 0 absent/null-text, 1 int-like (ival), 2 float (ival/10^aux), 3 text */
typedef struct {
    int64_t* fbeg;
    int64_t* vbeg;
    int64_t* vend;
    int64_t* ival;
    int32_t* aux;
    int8_t* kind;
} truth_t;

typedef struct {
    uint8_t* out;
    int64_t cap;
    int64_t pos;
    int overflow;
    truth_t* t;
    int64_t tidx; /* rec*ncols + col of the field being written */
} wr_t;

static void put(wr_t* w, uint8_t c)
{
    if (w->pos < w->cap) w->out[w->pos] = c;
    else w->overflow = 1;
    w->pos++;
}

static void puts_n(wr_t* w, const char* s, int n) { for (int i = 0; i < n; i++) put(w, (uint8_t)s[i]); }

static void put_uint(wr_t* w, uint64_t v, int min_digits)
{
    char tmp[24];
    int n = 0;
    do { tmp[n++] = (char)('0' + v % 10); v /= 10; } while (v);
    while (n < min_digits) tmp[n++] = '0';
    while (n) put(w, (uint8_t)tmp[--n]);
}

static void put_int(wr_t* w, int64_t v)
{
    if (v < 0) { put(w, '-'); put_uint(w, (uint64_t)0 - (uint64_t)v, 1); }
    else put_uint(w, (uint64_t)v, 1);
}

static void field_begin(wr_t* w, int kind)
{
    if (!w->t) return;
    w->t->fbeg[w->tidx] = w->pos;
    w->t->vbeg[w->tidx] = w->pos;
    w->t->kind[w->tidx] = (int8_t)kind;
}
static void content_begin(wr_t* w) { if (w->t) w->t->vbeg[w->tidx] = w->pos; }
static void content_end(wr_t* w) { if (w->t) w->t->vend[w->tidx] = w->pos; }
static void truth_int(wr_t* w, int64_t v) { if (w->t) w->t->ival[w->tidx] = v; }
static void truth_float(wr_t* w, int64_t m, int dec) { if (w->t) { w->t->ival[w->tidx] = m; w->t->aux[w->tidx] = dec; } }

/* ---- calendar (formatting direction: epoch -> civil, by counting) ------ */
static int leap(int64_t y) { return (y % 4 == 0 && y % 100 != 0) || y % 400 == 0; }

static void civil(int64_t days, int64_t* y, int64_t* m, int64_t* d)
{
    static const int dm[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    int64_t yy = 1970;
    while (days < 0) { yy--; days += 365 + leap(yy); }
    while (days >= 365 + leap(yy)) { days -= 365 + leap(yy); yy++; }
    int64_t mm = 0;
    while (days >= dm[mm] + (mm == 1 && leap(yy))) { days -= dm[mm] + (mm == 1 && leap(yy)); mm++; }
    *y = yy;
    *m = mm + 1;
    *d = days + 1;
}

static void put_date(wr_t* w, int64_t days)
{
    int64_t y, m, d;
    civil(days, &y, &m, &d);
    put_uint(w, (uint64_t)y, 4); put(w, '-'); put_uint(w, (uint64_t)m, 2); put(w, '-'); put_uint(w, (uint64_t)d, 2);
}

static void put_ts(wr_t* w, int64_t t, char sep)
{
    int64_t days = t >= 0 ? t / 86400 : -((-t + 86399) / 86400);
    int64_t sod = t - days * 86400;
    put_date(w, days);
    put(w, (uint8_t)sep);
    put_uint(w, (uint64_t)(sod / 3600), 2); put(w, ':');
    put_uint(w, (uint64_t)(sod / 60 % 60), 2); put(w, ':');
    put_uint(w, (uint64_t)(sod % 60), 2);
}

/* value m / 10^dec written with exactly dec decimals */
static void put_fixed(wr_t* w, int64_t m, int dec)
{
    uint64_t p = 1;
    for (int i = 0; i < dec; i++) p *= 10;
    uint64_t a = m < 0 ? (uint64_t)0 - (uint64_t)m : (uint64_t)m;
    if (m < 0) put(w, '-');
    put_uint(w, a / p, 1);
    if (dec) { put(w, '.'); put_uint(w, a % p, dec); }
}

static uint8_t printable_except(rng_t* r, uint8_t a, uint8_t b, uint8_t c)
{
    for (;;) {
        uint8_t ch = (uint8_t)(0x20 + below(r, 0x5F));
        if (ch != a && ch != b && ch != c) return ch;
    }
}

/* ---- C1: mixed CSV, 8 columns, 20% of strings quoted with specials ------ */
static void c1_string(wr_t* w, rng_t* r, uint8_t delim)
{
    int len = (int)uniform_i(r, 0, 40);
    if (bern(r, 0.20)) {
        if (len < 4) len = 4;
        uint8_t buf[48];
        for (int i = 0; i < len; i++) buf[i] = printable_except(r, '"', delim, '"');
        /* at least one delimiter, one LF and one doubled quote */
        int pq = (int)below(r, (uint64_t)(len - 1)), pc, pl;
        do { pc = (int)below(r, (uint64_t)len); } while (pc == pq || pc == pq + 1);
        do { pl = (int)below(r, (uint64_t)len); } while (pl == pq || pl == pq + 1 || pl == pc);
        buf[pc] = delim;
        buf[pl] = '\n';
        buf[pq] = '"';
        buf[pq + 1] = '"';
        field_begin(w, 3);
        put(w, '"');
        content_begin(w);
        for (int i = 0; i < len; i++) put(w, buf[i]);
        content_end(w);
        put(w, '"');
    } else {
        field_begin(w, 3);
        for (int i = 0; i < len; i++) put(w, printable_except(r, '"', delim, '"'));
        content_end(w);
    }
}

static void c1_record(wr_t* w, rng_t* r, uint8_t delim, int ncols_base)
{
    for (int c = 0; c < 8; c++) {
        w->tidx = ncols_base + c;
        if (c) put(w, delim);
        if (c < 2) {
            int64_t v = uniform_i(r, -1000000000, 1000000000);
            field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v);
        } else if (c < 4) {
            int64_t m = uniform_i(r, -1000000000000ll, 1000000000000ll);
            field_begin(w, 2); put_fixed(w, m, 6); content_end(w); truth_float(w, m, 6);
        } else if (c == 4) {
            int64_t t = uniform_i(r, 946684800ll, 1893455999ll);
            field_begin(w, 1); put_ts(w, t, 'T'); content_end(w); truth_int(w, t);
        } else {
            c1_string(w, r, delim);
        }
    }
    put(w, '\n');
}

/* ---- C2: numeric CSV, 18 columns, ~130 B per record --------------------- */
#define C2_MU 7.6
static void c2_record(wr_t* w, rng_t* r, int base)
{
    int c = 0;
    for (int k = 0; k < 4; k++, c++) {
        w->tidx = base + c;
        if (c) put(w, ',');
        int64_t v = uniform_i(r, 1, 300);
        field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v);
    }
    for (int k = 0; k < 2; k++, c++) {
        w->tidx = base + c;
        put(w, ',');
        int64_t t = uniform_i(r, 1514764800ll, 1546300799ll);
        field_begin(w, 1); put_ts(w, t, ' '); content_end(w); truth_int(w, t);
    }
    for (int k = 0; k < 8; k++, c++) {
        w->tidx = base + c;
        put(w, ',');
        double x = exp(C2_MU + normal(r));
        int64_t m = (int64_t)floor(x * 100.0 + 0.5);
        if (m > 99999999999ll) m = 99999999999ll;
        field_begin(w, 2); put_fixed(w, m, 2); content_end(w); truth_float(w, m, 2);
    }
    for (int k = 0; k < 4; k++, c++) {
        w->tidx = base + c;
        put(w, ',');
        int len = (int)uniform_i(r, 1, 3);
        field_begin(w, 3);
        for (int i = 0; i < len; i++) put(w, (uint8_t)('A' + below(r, 26)));
        content_end(w);
    }
    put(w, '\n');
}

/* ---- C3: text-heavy CSV, 9 columns, ~700 B per record ------------------- */
static const char B62[] = "0123456789ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz";

static void c3_text(wr_t* w, rng_t* r)
{
    double x = exp(log(300.0) - 0.5 + normal(r));
    int64_t len = (int64_t)x;
    if (len < 1) len = 1;
    if (len > 65536) len = 65536;
    int has_comma = bern(r, 0.05), has_lf = bern(r, 0.01), has_q = bern(r, 0.005);
    field_begin(w, 3);
    put(w, '"');
    content_begin(w);
    int64_t start = w->pos;
    /* random words of 1..12 lowercase letters separated by spaces */
    int64_t i = 0;
    while (i < len) {
        int wl = (int)uniform_i(r, 1, 12);
        for (int k = 0; k < wl && i < len; k++, i++) put(w, (uint8_t)('a' + below(r, 26)));
        if (i < len) { put(w, ' '); i++; }
    }
    /* overwrite positions with the special symbols (inside the content) */
    if (w->pos <= w->cap) {
        if (has_comma) w->out[start + (int64_t)below(r, (uint64_t)len)] = ',';
        if (has_lf) w->out[start + (int64_t)below(r, (uint64_t)len)] = '\n';
        if (has_q && len >= 2) {
            int64_t q = (int64_t)below(r, (uint64_t)(len - 1));
            w->out[start + q] = '"';
            w->out[start + q + 1] = '"';
            /* a doubled quote must not touch a lone quote elsewhere: none exist */
        }
    }
    content_end(w);
    put(w, '"');
}

static void c3_record(wr_t* w, rng_t* r, int base)
{
    for (int c = 0; c < 9; c++) {
        w->tidx = base + c;
        if (c) put(w, ',');
        if (c < 3) {
            field_begin(w, 3);
            for (int k = 0; k < 22; k++) put(w, (uint8_t)B62[below(r, 62)]);
            content_end(w);
        } else if (c < 6) {
            int64_t v = uniform_i(r, 0, 5);
            field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v);
        } else if (c == 6) {
            int64_t d = uniform_i(r, 12418, 18261); /* 2004-01-01 .. 2019-12-31 */
            field_begin(w, 1); put_date(w, d); content_end(w); truth_int(w, d);
        } else {
            c3_text(w, r);
        }
    }
    put(w, '\n');
}

/* ---- mixed dialects: 8 C1-like columns, quoting style by dialect --------
 * qstyle 0: no quoting, no escapes (delimiter and LF never in data)
 * qstyle 1: RFC-4180 quotes (doubled quote inside)
 * qstyle 2: quotes with backslash escapes inside and in unquoted fields
 * qstyle 3: no quotes, backslash escapes the next byte */
static void mixed_string(wr_t* w, rng_t* r, uint8_t delim, int qstyle)
{
    int len = (int)uniform_i(r, 0, 24);
    field_begin(w, 3);
    if ((qstyle == 1 || qstyle == 2) && bern(r, 0.2)) {
        put(w, '"');
        content_begin(w);
        for (int i = 0; i < len; i++) {
            int k = (int)below(r, 16);
            if (k == 0) put(w, delim);
            else if (k == 1) put(w, '\n');
            else if (k == 2 && qstyle == 1) { put(w, '"'); put(w, '"'); }
            else if (k == 2) { put(w, '\\'); put(w, bern(r, 0.5) ? '"' : '\\'); }
            else put(w, printable_except(r, '"', '\\', delim));
        }
        content_end(w);
        put(w, '"');
        return;
    }
    for (int i = 0; i < len; i++) {
        if (qstyle == 3 && below(r, 10) == 0) { put(w, '\\'); put(w, bern(r, 0.5) ? delim : '\\'); }
        else put(w, printable_except(r, '"', '\\', delim));
    }
    content_end(w);
}

static void mixed_record(wr_t* w, rng_t* r, int base, uint8_t delim, int qstyle)
{
    for (int c = 0; c < 8; c++) {
        w->tidx = base + c;
        if (c) put(w, delim);
        if (c < 2) {
            int64_t v = uniform_i(r, -1000000000, 1000000000);
            field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v);
        } else if (c < 4) {
            int64_t m = uniform_i(r, -100000000ll, 100000000ll);
            field_begin(w, 2); put_fixed(w, m, 3); content_end(w); truth_float(w, m, 3);
        } else if (c == 4) {
            int64_t t = uniform_i(r, 946684800ll, 1893455999ll);
            field_begin(w, 1); put_ts(w, t, 'T'); content_end(w); truth_int(w, t);
        } else {
            mixed_string(w, r, delim, qstyle);
        }
    }
    put(w, '\n');
}

/* ---- extended web-server log, 12 space-separated columns ----------------
 * host ident user [time] "request" status bytes "referer" "agent" taken port server */
static const char* MONTHS[12] = {"Jan", "Feb", "Mar", "Apr", "May", "Jun", "Jul", "Aug", "Sep", "Oct", "Nov", "Dec"};
static const char* METHODS[4] = {"GET", "POST", "PUT", "HEAD"};
static const int STATUS[6] = {200, 200, 200, 304, 404, 500};

static void put_word(wr_t* w, rng_t* r, int lo, int hi)
{
    int n = (int)uniform_i(r, lo, hi);
    for (int i = 0; i < n; i++) put(w, (uint8_t)('a' + below(r, 26)));
}

static void log_quoted_text(wr_t* w, rng_t* r, int lo, int hi, int escapes)
{
    put(w, '"');
    content_begin(w);
    int n = (int)uniform_i(r, lo, hi);
    for (int i = 0; i < n; i++) {
        if (escapes && below(r, 40) == 0) { put(w, '\\'); put(w, bern(r, 0.5) ? '"' : '\\'); continue; }
        int k = (int)below(r, 8);
        put(w, k == 0 ? ' ' : k == 1 ? '/' : (uint8_t)('a' + below(r, 26)));
    }
    content_end(w);
    put(w, '"');
}

static void log_record(wr_t* w, rng_t* r, int base, uint8_t delim)
{
    int c = 0;
#define NEXTCOL() do { w->tidx = base + c; if (c) put(w, delim); } while (0)
    NEXTCOL(); field_begin(w, 3);
    put_uint(w, below(r, 256), 1); put(w, '.'); put_uint(w, below(r, 256), 1); put(w, '.');
    put_uint(w, below(r, 256), 1); put(w, '.'); put_uint(w, below(r, 256), 1); content_end(w); c++;
    NEXTCOL(); field_begin(w, 3); put(w, '-'); content_end(w); c++;
    NEXTCOL(); field_begin(w, 3); if (bern(r, 0.5)) put(w, '-'); else put_word(w, r, 3, 10); content_end(w); c++;
    NEXTCOL(); field_begin(w, 3); put(w, '[');
    {
        content_begin(w);
        int64_t t = uniform_i(r, 1514764800ll, 1546300799ll);
        int64_t days = t / 86400, sod = t % 86400, y, m, d;
        civil(days, &y, &m, &d);
        put_uint(w, (uint64_t)d, 2); put(w, '/'); puts_n(w, MONTHS[m - 1], 3); put(w, '/'); put_uint(w, (uint64_t)y, 4);
        put(w, ':'); put_uint(w, (uint64_t)(sod / 3600), 2); put(w, ':'); put_uint(w, (uint64_t)(sod / 60 % 60), 2);
        put(w, ':'); put_uint(w, (uint64_t)(sod % 60), 2); put(w, ' '); put(w, '+'); put_uint(w, 0, 4);
        content_end(w);
    }
    put(w, ']'); c++;
    NEXTCOL(); field_begin(w, 3); put(w, '"');
    {
        content_begin(w);
        const char* mth = METHODS[below(r, 4)];
        puts_n(w, mth, (int)strlen(mth)); put(w, ' '); put(w, '/');
        int segs = (int)uniform_i(r, 1, 6);
        for (int i = 0; i < segs; i++) {
            put_word(w, r, 1, 12);
            if (below(r, 30) == 0) { put(w, '\\'); put(w, bern(r, 0.5) ? '"' : '\\'); }
            if (i + 1 < segs) put(w, '/');
        }
        puts_n(w, " HTTP/1.1", 9);
        content_end(w);
    }
    put(w, '"'); c++;
    NEXTCOL(); { int64_t v = STATUS[below(r, 6)]; field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v); } c++;
    NEXTCOL();
    if (bern(r, 0.05)) { field_begin(w, 0); put(w, '-'); content_end(w); }
    else { int64_t v = uniform_i(r, 0, 5000000); field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v); }
    c++;
    NEXTCOL(); field_begin(w, 3); log_quoted_text(w, r, 0, 60, 1); c++;
    NEXTCOL(); field_begin(w, 3); log_quoted_text(w, r, 10, 120, 1); c++;
    NEXTCOL(); { int64_t m = uniform_i(r, 0, 9999999); field_begin(w, 2); put_fixed(w, m, 3); content_end(w); truth_float(w, m, 3); } c++;
    NEXTCOL(); { int64_t v = bern(r, 0.7) ? 443 : uniform_i(r, 1024, 65535); field_begin(w, 1); put_int(w, v); content_end(w); truth_int(w, v); } c++;
    NEXTCOL(); field_begin(w, 3); puts_n(w, "srv", 3); put_uint(w, below(r, 64), 2); content_end(w); c++;
#undef NEXTCOL
    put(w, '\n');
}

/* ---- entry point -------------------------------------------------------- */
enum { K_C1 = 1, K_C2 = 2, K_C3 = 3, K_MIXED = 4, K_LOG = 5 };

int dg_ncols(int kind)
{
    switch (kind) {
    case K_C1: return 8;
    case K_C2: return 18;
    case K_C3: return 9;
    case K_MIXED: return 8;
    case K_LOG: return 12;
    }
    return -1;
}

/*
 * Generate up to max_records records of one block into out[0..cap): whole
 * records only, stopping before the record that would pass max_bytes.
 * Returns bytes written; *nrec_out = records written. Truth arrays (nullable)
 * must hold max_records * ncols entries.
 */
int64_t dg_block(int kind, uint64_t seed, uint64_t block, int64_t max_records, int64_t max_bytes,
                 int delim, int qstyle, uint8_t* out, int64_t cap,
                 int64_t* fbeg, int64_t* vbeg, int64_t* vend, int64_t* ival, int32_t* aux, int8_t* tkind,
                 int64_t* nrec_out)
{
    rng_t r = rng_for(seed, block);
    truth_t t = {fbeg, vbeg, vend, ival, aux, tkind};
    wr_t w = {out, cap, 0, 0, fbeg ? &t : NULL, 0};
    int ncols = dg_ncols(kind);
    if (ncols < 0) return -1;
    int64_t nrec = 0;
    if (max_bytes > cap) max_bytes = cap;
    while (nrec < max_records) {
        int64_t save = w.pos;
        rng_t rsave = r;
        int base = (int)(nrec * ncols);
        switch (kind) {
        case K_C1: c1_record(&w, &r, (uint8_t)delim, base); break;
        case K_C2: c2_record(&w, &r, base); break;
        case K_C3: c3_record(&w, &r, base); break;
        case K_MIXED: mixed_record(&w, &r, base, (uint8_t)delim, qstyle); break;
        case K_LOG: log_record(&w, &r, base, (uint8_t)delim); break;
        }
        if (w.pos > max_bytes || w.overflow) {
            w.pos = save;
            r = rsave;
            break;
        }
        nrec++;
    }
    *nrec_out = nrec;
    return w.pos;
}
