/*
 * The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (built and
 * run by test_oracle_sanitized.py, on the CPU): every entry point on
 * adversarial inputs -- bytes of every value, soups of quotes and delimiters,
 * ragged and long records, numbers, dates and times of every shape, fields
 * far longer than a line -- with every output buffer allocated to its exact
 * size (so an access one element past it is caught) and with capacities
 * below the counts, and the UTF-16 entry point on the same inputs widened to
 * code units (with units outside ASCII and surrogates mixed in). Also checks that the counting run, the full run and the
 * capacity-limited runs agree on the counts. Prints "ok <checks>" at the end.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

enum { T_INT64 = 0, T_FLOAT64 = 1, T_TIMESTAMP = 2, T_DATE = 3, T_STRING = 4, T_SKIP = 5 };
enum { TAG_D = 0, TAG_C = 1, TAG_F = 2, TAG_R = 3 };

static uint64_t g_rng = 0x1905134150ull;
static uint64_t rnd(void) /* splitmix64 (Steele, Lea, Flood 2014) */
{
    uint64_t z = (g_rng += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
static int64_t rnd_below(int64_t k) { return k > 0 ? (int64_t)(rnd() % (uint64_t)k) : 0; }

static long g_checks = 0;
#define CHECK(c)                                                                  \
    do {                                                                          \
        ++g_checks;                                                               \
        if (!(c)) {                                                               \
            fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #c);       \
            exit(2);                                                              \
        }                                                                         \
    } while (0)

static void* xmalloc(size_t n)
{
    void* p = malloc(n ? n : 1);
    if (!p) exit(3);
    return p;
}

/* A DFA from rows of (next, tag) per group; groups: 0 line feed, 1 quote,
 * 2 the field delimiter, 3 everything else. */
static void make_dfa(orc_dfa* d, int ns, const int next[4][8], const int tag[4][8], uint32_t accept, int invalid)
{
    memset(d, 0, sizeof *d);
    d->num_states = ns;
    d->num_groups = 4;
    d->start_state = 0;
    d->invalid_state = invalid;
    d->accept_mask = accept;
    for (int b = 0; b < 256; ++b) d->group_of[b] = 3;
    d->group_of['\n'] = 0;
    d->group_of['"'] = 1;
    d->group_of[','] = 2;
    for (int g = 0; g < 4; ++g)
        for (int s = 0; s < ns; ++s) {
            d->next[g][s] = (uint8_t)next[g][s];
            d->tag[g][s] = (uint8_t)tag[g][s];
        }
}

static void dfa_csv4(orc_dfa* d) /* FB UQ QT QE */
{
    static const int nx[4][8] = {{0, 0, 2, 0}, {2, 1, 3, 2}, {0, 0, 2, 0}, {1, 1, 2, 1}};
    static const int tg[4][8] = {{TAG_R, TAG_R, TAG_D, TAG_R},
                                 {TAG_C, TAG_D, TAG_C, TAG_D},
                                 {TAG_F, TAG_F, TAG_D, TAG_F},
                                 {TAG_D, TAG_D, TAG_D, TAG_D}};
    make_dfa(d, 4, nx, tg, (1u << 0) | (1u << 1) | (1u << 3), -1);
}

static void dfa_paper6(orc_dfa* d) /* EOR ENC FLD EOF ESC INV (Table 1) */
{
    static const int nx[4][8] = {{0, 1, 0, 0, 0, 5}, {1, 4, 5, 1, 1, 5}, {3, 1, 3, 3, 3, 5}, {2, 1, 2, 2, 5, 5}};
    static const int tg[4][8] = {{TAG_R, TAG_D, TAG_R, TAG_R, TAG_R, TAG_D},
                                 {TAG_C, TAG_C, TAG_D, TAG_C, TAG_D, TAG_D},
                                 {TAG_F, TAG_D, TAG_F, TAG_F, TAG_F, TAG_D},
                                 {TAG_D, TAG_D, TAG_D, TAG_D, TAG_D, TAG_D}};
    make_dfa(d, 6, nx, tg, (1u << 0) | (1u << 2) | (1u << 3) | (1u << 4), 5);
}

/* ---- inputs ------------------------------------------------------------------------------ */

typedef struct {
    uint8_t* p;
    int64_t n, cap;
} buf_t;

static void put(buf_t* b, const char* s, int64_t k)
{
    if (k <= 0) return;
    if (b->n + k > b->cap) {
        b->cap = 2 * (b->n + k) + 64;
        b->p = (uint8_t*)realloc(b->p, (size_t)b->cap);
        if (!b->p) exit(3);
    }
    memcpy(b->p + b->n, s, (size_t)k);
    b->n += k;
}
static void puts_(buf_t* b, const char* s) { put(b, s, (int64_t)strlen(s)); }

static void random_bytes(buf_t* b, int64_t n)
{
    for (int64_t i = 0; i < n; ++i) {
        const char c = (char)(rnd() & 0xff);
        put(b, &c, 1);
    }
}

static void soup(buf_t* b, int64_t n)
{
    static const char alpha[] = "\n\",a1.-e+ :T0959";
    for (int64_t i = 0; i < n; ++i) put(b, &alpha[rnd_below((int64_t)sizeof alpha - 1)], 1);
}

/* A number, date, time or text field of one of many shapes, valid or not. */
static void field(buf_t* b)
{
    char t[128];
    switch (rnd_below(12)) {
    case 0: snprintf(t, sizeof t, "%lld", (long long)(int64_t)rnd()); break;
    case 1: snprintf(t, sizeof t, "%+d", (int)rnd_below(2000) - 1000); break;
    case 2: snprintf(t, sizeof t, "%.*f", (int)rnd_below(25), (double)(int64_t)rnd() / 1e6); break;
    case 3: snprintf(t, sizeof t, "%.17e", (double)(int64_t)rnd() * 1e-300); break;
    case 4: snprintf(t, sizeof t, "%d.%de%d", (int)rnd_below(100), (int)rnd_below(1000), (int)rnd_below(800) - 400); break;
    case 5:
        snprintf(t, sizeof t, "%04d-%02d-%02d", (int)rnd_below(10000), (int)rnd_below(14), (int)rnd_below(33));
        break;
    case 6:
        snprintf(t, sizeof t, "%04d-%02d-%02d%c%02d:%02d:%02d", (int)rnd_below(10000), (int)rnd_below(14),
                 (int)rnd_below(33), rnd_below(2) ? 'T' : ' ', (int)rnd_below(25), (int)rnd_below(61),
                 (int)rnd_below(61));
        break;
    case 7: { /* 20-40 digits */
        int k = 20 + (int)rnd_below(21), i;
        for (i = 0; i < k; ++i) t[i] = (char)('0' + rnd_below(10));
        t[i] = 0;
        break;
    }
    case 8: t[0] = 0; break; /* empty */
    case 9: snprintf(t, sizeof t, "\"q,%d\"\"x\n\"", (int)rnd_below(100)); break;
    case 10: snprintf(t, sizeof t, "%s", rnd_below(2) ? "-" : "."); break;
    default: {
        int k = (int)rnd_below(30), i;
        for (i = 0; i < k; ++i) t[i] = (char)('a' + rnd_below(26));
        t[i] = 0;
    }
    }
    puts_(b, t);
}

static void records(buf_t* b, int nrec)
{
    for (int r = 0; r < nrec; ++r) {
        const int nf = 1 + (int)rnd_below(12); /* ragged */
        for (int f = 0; f < nf; ++f) {
            if (f) puts_(b, ",");
            field(b);
        }
        if (r + 1 < nrec || rnd_below(2)) puts_(b, "\n");
    }
}

static void long_field(buf_t* b, int64_t len)
{
    puts_(b, "1,\"");
    for (int64_t i = 0; i < len; ++i) {
        const int64_t k = rnd_below(50);
        puts_(b, k == 0 ? "\"\"" : k == 1 ? "," : k == 2 ? "\n" : "z");
    }
    puts_(b, "\",2\n3,4");
}

/* ---- one input through every entry point ---------------------------------------------------- */

static void run(const uint8_t* buf, int64_t n, const orc_dfa* d, int64_t under)
{
    static const int32_t kinds[8] = {T_INT64, T_FLOAT64, T_STRING, T_TIMESTAMP, T_DATE, T_SKIP, T_STRING, T_INT64};
    const int32_t ncols = 1 + (int32_t)rnd_below(8);
    int32_t types[8];
    for (int c = 0; c < ncols; ++c) types[c] = kinds[(c + rnd_below(8)) % 8];

    orc_result cnt;
    CHECK(orc_parse(buf, n, d, 0, NULL, 0, 0, NULL, NULL, NULL, NULL, NULL, NULL, &cnt) == 0);
    const int64_t R = cnt.num_records, F = cnt.num_fields;
    CHECK(R >= 0 && F >= R);
    const int64_t cr = R - under < 0 ? 0 : R - under, cf = F - under < 0 ? 0 : F - under;

    int64_t* rec = (int64_t*)xmalloc((size_t)(cr + 1) * 8);
    int64_t* fld = (int64_t*)xmalloc((size_t)(cf + 1) * 8);
    int32_t* cid = (int32_t*)xmalloc((size_t)cf * 4);
    void* values[8];
    uint8_t* valid[8];
    int64_t* ends[8];
    for (int c = 0; c < ncols; ++c) {
        values[c] = types[c] == T_SKIP ? NULL : xmalloc((size_t)cr * 8);
        valid[c] = types[c] == T_SKIP ? NULL : (uint8_t*)xmalloc((size_t)cr);
        ends[c] = types[c] == T_STRING ? (int64_t*)xmalloc((size_t)cr * 8) : NULL;
    }
    orc_result res;
    CHECK(orc_parse(buf, n, d, ncols, types, cr, cf, rec, fld, cid, values, valid, ends, &res) == 0);
    CHECK(res.num_records == R && res.num_fields == F);
    CHECK(res.first_invalid_offset == cnt.first_invalid_offset && res.final_state == cnt.final_state);
    CHECK((R > cr || F > cf) ? res.status == ORC_CAPACITY : res.status != ORC_CAPACITY);
    CHECK(res.min_record_fields == cnt.min_record_fields && res.max_record_fields == cnt.max_record_fields);
    const int64_t Rw = R < cr ? R : cr, Fw = F < cf ? F : cf;
    for (int64_t k = 0; k < Fw; ++k) CHECK(fld[k] <= fld[k + 1]);
    for (int64_t k = 0; k < Rw; ++k) CHECK(rec[k] <= rec[k + 1]);
    orc_reject_ragged(ncols, types, Rw, rec, values, valid, ends);

    for (int c = 0; c < ncols; ++c) {
        if (types[c] != T_STRING) continue;
        for (int term = -1; term <= 0; ++term) {
            int64_t* offs = (int64_t*)xmalloc((size_t)(R + 1) * 8);
            const int64_t total = orc_materialize(buf, n, d, c, R, offs, NULL, 0, term);
            CHECK(total >= 0 && offs[R] == total);
            uint8_t* chars = (uint8_t*)xmalloc((size_t)total);
            CHECK(orc_materialize(buf, n, d, c, R, offs, chars, total, term) == total);
            const int64_t half = total / 2; /* a capacity below the total */
            uint8_t* part = (uint8_t*)xmalloc((size_t)half);
            CHECK(orc_materialize(buf, n, d, c, R, offs, part, half, term) == total);
            CHECK(memcmp(part, chars, (size_t)half) == 0);
            free(part);
            free(chars);
            free(offs);
        }
    }
    int32_t inferred[8];
    int64_t nonempty[8];
    orc_infer_types(buf, n, d, ncols, inferred, nonempty);
    for (int c = 0; c < ncols; ++c) CHECK(inferred[c] >= T_INT64 && inferred[c] <= T_STRING && nonempty[c] >= 0);

    for (int c = 0; c < ncols; ++c) {
        free(values[c]);
        free(valid[c]);
        free(ends[c]);
    }
    free(rec);
    free(fld);
    free(cid);
}

/* The UTF-16 entry point: the same bytes widened to code units, some of them
 * replaced by units outside ASCII (and surrogates), with exactly sized
 * buffers. */
static void run_utf16(const uint8_t* buf, int64_t n, const orc_dfa* d)
{
    uint16_t* u = (uint16_t*)xmalloc((size_t)n * 2);
    for (int64_t i = 0; i < n; ++i) {
        const int64_t k = rnd_below(10);
        u[i] = k == 0 ? (uint16_t)(0x80 + rnd_below(0xff80)) : k == 1 ? (uint16_t)(0xd800 + rnd_below(0x800)) : buf[i];
    }
    static const int32_t types[6] = {T_INT64, T_FLOAT64, T_STRING, T_TIMESTAMP, T_DATE, T_STRING};
    orc_result cnt, res;
    CHECK(orc_parse_utf16(u, n, d, 0, NULL, 0, 0, NULL, NULL, NULL, NULL, NULL, NULL, &cnt) == 0);
    const int64_t R = cnt.num_records, F = cnt.num_fields;
    int64_t* rec = (int64_t*)xmalloc((size_t)(R + 1) * 8);
    int64_t* fld = (int64_t*)xmalloc((size_t)(F + 1) * 8);
    int32_t* cid = (int32_t*)xmalloc((size_t)F * 4);
    void* values[6];
    uint8_t* valid[6];
    int64_t* ends[6];
    for (int c = 0; c < 6; ++c) {
        values[c] = xmalloc((size_t)R * 8);
        valid[c] = (uint8_t*)xmalloc((size_t)R);
        ends[c] = types[c] == T_STRING ? (int64_t*)xmalloc((size_t)R * 8) : NULL;
    }
    CHECK(orc_parse_utf16(u, n, d, 6, types, R, F, rec, fld, cid, values, valid, ends, &res) == 0);
    CHECK(res.num_records == R && res.num_fields == F && res.status != ORC_CAPACITY);
    for (int64_t k = 0; k + 1 <= F; ++k) CHECK(fld[k] % 2 == 0 && fld[k] <= fld[k + 1]);
    for (int32_t term = -1; term <= 0x2028; term += 0x2029) {
        int64_t* offs = (int64_t*)xmalloc((size_t)(R + 1) * 8);
        const int64_t total = orc_materialize_utf16(u, n, d, 2, R, offs, NULL, 0, term);
        CHECK(total >= 0 && offs[R] == total);
        uint16_t* chars = (uint16_t*)xmalloc((size_t)total * 2);
        CHECK(orc_materialize_utf16(u, n, d, 2, R, offs, chars, total, term) == total);
        free(chars);
        free(offs);
    }
    for (int c = 0; c < 6; ++c) {
        free(values[c]);
        free(valid[c]);
        free(ends[c]);
    }
    free(rec);
    free(fld);
    free(cid);
    free(u);
}

static void run_skip_rows(const uint8_t* buf, int64_t n)
{
    int64_t lines = 1;
    for (int64_t i = 0; i < n; ++i) lines += buf[i] == '\n';
    int64_t ranges[8];
    int32_t nr = 0;
    int64_t at = 0;
    while (nr < 4 && at < lines) {
        const int64_t a = at + rnd_below(3), b = a + rnd_below(4);
        ranges[2 * nr] = a;
        ranges[2 * nr + 1] = b;
        ++nr;
        at = b + 1;
    }
    uint8_t* out = (uint8_t*)xmalloc((size_t)n);
    const int64_t m = orc_skip_rows(buf, n, ranges, nr, out);
    CHECK(m >= 0 && m <= n);
    free(out);
}

static void run_conv(void)
{
    for (int k = 0; k < 4000; ++k) {
        buf_t b = {0, 0, 0};
        if (rnd_below(3) == 0) random_bytes(&b, rnd_below(40));
        else field(&b);
        /* exactly sized: a read one past the field is caught */
        uint8_t* p = (uint8_t*)xmalloc((size_t)b.n);
        if (b.n) memcpy(p, b.p, (size_t)b.n);
        int64_t iv;
        double dv;
        for (int t = T_INT64; t <= T_DATE; ++t) {
            const int r = orc_conv(t, p, b.n, &iv, &dv);
            CHECK(r == 0 || r == 1);
        }
        free(p);
        free(b.p);
    }
}

int main(void)
{
    orc_dfa dfas[2];
    dfa_csv4(&dfas[0]);
    dfa_paper6(&dfas[1]);
    for (int it = 0; it < 600; ++it) {
        buf_t b = {0, 0, 0};
        switch (it % 4) {
        case 0: random_bytes(&b, rnd_below(3000)); break;
        case 1: soup(&b, rnd_below(3000)); break;
        case 2: records(&b, 1 + (int)rnd_below(60)); break;
        default:
            if (it % 40 == 3) long_field(&b, 200000);
            else records(&b, 1 + (int)rnd_below(8));
        }
        /* exactly sized input: a read one past the end is caught */
        uint8_t* in = (uint8_t*)xmalloc((size_t)b.n);
        if (b.n) memcpy(in, b.p, (size_t)b.n);
        for (int d = 0; d < 2; ++d) {
            run(in, b.n, &dfas[d], 0);
            run(in, b.n, &dfas[d], 1 + rnd_below(5));
            run_utf16(in, b.n, &dfas[d]);
        }
        run_skip_rows(in, b.n);
        free(in);
        free(b.p);
    }
    run_conv();
    printf("ok %ld\n", g_checks);
    return 0;
}
