/*
 * Sequential reference parser: the oracle for the parallel parse.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product library links, loads or
 * calls this file; only the test suite, the smoke check and the CPU baseline
 * of the benchmark do. It shares no code, header or table with the GPU path.
 *
 * What it computes is the plain definition that the parallel method reaches
 * exactly: one DFA instance started in the start state reads the input from
 * the first symbol to the last (the sequential baseline that Sec. 3.1 sets
 * the parallel method against).
 * The multi-start-state simulation and the composition scan of Sec. 3.1 only
 * let that same run be split across threads, so they do not appear here.
 *
 * Per symbol, the DFA's tag marks it as a record delimiter, a field
 * delimiter, a control symbol or data (the three bitmap indexes of Sec. 3.1).
 * Record and column of every field follow from counting delimiters in order
 * (Sec. 3.2). Each field is then converted to its column's type (Sec. 3.3),
 * empty fields take the column default (Sec. 4.3, default values), and a
 * transition into the invalid state or a non-accepting end state is reported
 * (Sec. 4.3, validating format). The fewest and most fields over all records
 * are reported for inferring or validating the number of columns (Sec. 4.3):
 * the largest count is the inferred column count, and equal counts mean
 * every record has the same number of columns.
 *
 * Readings where the paper is silent (all listed in the design notes):
 *  - a final record without a trailing record delimiter still counts, and a
 *    trailing field delimiter closes an empty last field;
 *  - field_offsets[k] is field k's first byte; field_offsets[F] is one past
 *    the last field's end plus one (the position after its delimiter, real or
 *    virtual at n);
 *  - a string value is the (begin, end) byte span of the field with one
 *    leading and one trailing control symbol removed (the enclosing quotes);
 *  - ragged records: missing columns get value 0 with valid = 0, extra
 *    fields are kept in the field arrays and dropped from typed columns;
 *  - a record's column count is its number of fields (a blank line is one
 *    empty field); without records the fewest is -1 and the most 0;
 *  - numbers follow a strict grammar (no blanks, no locale); floats are the
 *    binary64 value nearest to the decimal, ties to even (strtod's result).
 */
#define _GNU_SOURCE
#include <errno.h>
#include <locale.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

enum { TAG_DATA = 0, TAG_CONTROL = 1, TAG_FIELD = 2, TAG_RECORD = 3 };
enum { TY_INT64 = 0, TY_FLOAT64 = 1, TY_TIMESTAMP_S = 2, TY_DATE_DAYS = 3,
       TY_STRING = 4, TY_SKIP = 5 };

static int is_digit(uint8_t c) { return c >= '0' && c <= '9'; }

/* ---- conversions (Sec. 3.3: a thread converts a field's symbols to the
 * column's type; the paper fixes no grammar, the one below is a reading) --- */

/* [+-]?[0-9]+, must fit in int64. Returns 1 if valid. */
static int conv_int64(const uint8_t* p, int64_t len, int64_t* out)
{
    int64_t i = 0;
    int neg = 0;
    if (len > 0 && (p[0] == '+' || p[0] == '-')) { neg = p[0] == '-'; i = 1; }
    if (i == len) return 0;
    /* magnitude limit: 2^63 - 1 for positive, 2^63 for negative */
    uint64_t limit = neg ? (uint64_t)1 << 63 : ((uint64_t)1 << 63) - 1;
    uint64_t mag = 0;
    for (; i < len; i++) {
        if (!is_digit(p[i])) return 0;
        uint64_t d = (uint64_t)(p[i] - '0');
        if (mag > (limit - d) / 10) return 0; /* mag*10 + d > limit */
        mag = mag * 10 + d;
    }
    if (neg) *out = (mag == ((uint64_t)1 << 63)) ? INT64_MIN : -(int64_t)mag;
    else *out = (int64_t)mag;
    return 1;
}

/* [+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+)([eE][+-]?[0-9]+)? -- grammar check only. */
static int float_grammar(const uint8_t* p, int64_t len)
{
    int64_t i = 0, nint = 0, nfrac = 0;
    if (i < len && (p[i] == '+' || p[i] == '-')) i++;
    while (i < len && is_digit(p[i])) { i++; nint++; }
    if (i < len && p[i] == '.') {
        i++;
        while (i < len && is_digit(p[i])) { i++; nfrac++; }
    }
    if (nint == 0 && nfrac == 0) return 0;
    if (i < len && (p[i] == 'e' || p[i] == 'E')) {
        int64_t nexp = 0;
        i++;
        if (i < len && (p[i] == '+' || p[i] == '-')) i++;
        while (i < len && is_digit(p[i])) { i++; nexp++; }
        if (nexp == 0) return 0;
    }
    return i == len;
}

/* Correctly rounded decimal -> binary64: a library routine serves this step
 * (glibc's strtod rounds to nearest, ties to even, including subnormals). */
static int conv_float64(const uint8_t* p, int64_t len, double* out, locale_t cloc)
{
    if (!float_grammar(p, len)) return 0;
    char small[128];
    char* s = len < (int64_t)sizeof small ? small : (char*)malloc((size_t)len + 1);
    if (!s) return 0;
    memcpy(s, p, (size_t)len);
    s[len] = 0;
    char* end = NULL;
    errno = 0;
    *out = strtod_l(s, &end, cloc); /* overflow gives +-inf, which is kept */
    int ok = end == s + len;
    if (s != small) free(s);
    return ok;
}

static int is_leap(int64_t y) { return (y % 4 == 0 && y % 100 != 0) || y % 400 == 0; }

static int days_in_month(int64_t y, int64_t m)
{
    static const int dm[12] = {31, 28, 31, 30, 31, 30, 31, 31, 30, 31, 30, 31};
    return dm[m - 1] + (m == 2 && is_leap(y));
}

/* Number of days from 0000-01-01 to y-01-01 in the proleptic Gregorian
 * calendar: 365 per year plus one per leap year in [0, y-1]. */
static int64_t days_before_year(int64_t y)
{
    return 365 * y + (y + 3) / 4 - (y + 99) / 100 + (y + 399) / 400;
}

/* Days since 1970-01-01 (negative before). */
static int64_t epoch_days(int64_t y, int64_t m, int64_t d)
{
    int64_t doy = d - 1;
    for (int64_t k = 1; k < m; k++) doy += days_in_month(y, k);
    return days_before_year(y) - days_before_year(1970) + doy;
}

static int dig(const uint8_t* p, int n, int64_t* v)
{
    int64_t x = 0;
    for (int i = 0; i < n; i++) {
        if (!is_digit(p[i])) return 0;
        x = x * 10 + (p[i] - '0');
    }
    *v = x;
    return 1;
}

/* YYYY-MM-DD */
static int conv_date(const uint8_t* p, int64_t len, int64_t* out)
{
    int64_t y, m, d;
    if (len != 10 || p[4] != '-' || p[7] != '-') return 0;
    if (!dig(p, 4, &y) || !dig(p + 5, 2, &m) || !dig(p + 8, 2, &d)) return 0;
    if (m < 1 || m > 12 || d < 1 || d > days_in_month(y, m)) return 0;
    *out = epoch_days(y, m, d);
    return 1;
}

/* YYYY-MM-DD hh:mm:ss or YYYY-MM-DDThh:mm:ss, UTC, seconds 0..59 */
static int conv_timestamp(const uint8_t* p, int64_t len, int64_t* out)
{
    int64_t days, h, mi, s;
    if (len != 19 || (p[10] != ' ' && p[10] != 'T') || p[13] != ':' || p[16] != ':') return 0;
    if (!conv_date(p, 10, &days)) return 0;
    if (!dig(p + 11, 2, &h) || !dig(p + 14, 2, &mi) || !dig(p + 17, 2, &s)) return 0;
    if (h > 23 || mi > 59 || s > 59) return 0;
    *out = days * 86400 + h * 3600 + mi * 60 + s;
    return 1;
}

/* ---- the sequential run -------------------------------------------------- */

typedef struct {
    const orc_dfa* dfa;
    int32_t ncols;
    const int32_t* types;
    int64_t cap_records, cap_fields;
    int64_t* record_offsets;
    int64_t* field_offsets;
    int32_t* column_ids;
    void** values;
    uint8_t** valid;
    int64_t** str_end;
    locale_t cloc;
    int64_t R, F, col, conv_errors, ragged;
    int64_t min_fields, max_fields; /* over the records closed so far */
    /* UTF-16 input (Sec. 4.2): the symbols are 16-bit code units, u16[i]; a
     * unit below 0x80 is the ASCII character of the same value and every
     * other unit reads as the non-ASCII byte 0x80 (data of the catch-all
     * group in DFAs whose structural symbols are ASCII). Positions in the
     * outputs are byte offsets, unit_bytes per symbol. */
    const uint16_t* u16;
    int64_t unit_bytes;
    uint8_t* text; /* a field's symbols as bytes, for its conversion */
    int64_t text_cap;
} run_t;

static uint8_t sym_at(const run_t* r, const uint8_t* buf, int64_t i)
{
    if (!r->u16) return buf[i];
    return r->u16[i] < 0x80 ? (uint8_t)r->u16[i] : (uint8_t)0x80;
}

static void write_default(run_t* r, int64_t rec, int64_t c)
{
    if (!r->values || c >= r->ncols || rec >= r->cap_records) return;
    int32_t ty = r->types[c];
    if (ty == TY_SKIP) return;
    if (ty == TY_FLOAT64) ((double*)r->values[c])[rec] = 0.0;
    else ((int64_t*)r->values[c])[rec] = 0;
    if (ty == TY_STRING) r->str_end[c][rec] = 0;
    r->valid[c][rec] = 0;
}

/* Convert field [b, e) of record rec, column c. first_tag/last_tag are the
 * tags of its first and last symbol (meaningful when b < e). */
static void convert_field(run_t* r, const uint8_t* buf, int64_t b, int64_t e,
                          int first_tag, int last_tag, int64_t rec, int64_t c)
{
    if (c >= r->ncols) return;
    int32_t ty = r->types[c];
    if (ty == TY_SKIP) return;
    /* Strip one leading and one trailing control symbol (enclosing quotes). */
    int64_t begin = b, end = e;
    if (end > begin && first_tag == TAG_CONTROL) begin++;
    if (end - 1 >= begin && last_tag == TAG_CONTROL) end--;
    int64_t len = end - begin;
    const uint8_t* p = r->u16 ? NULL : buf + begin;
    if (r->u16 && ty != TY_STRING && len > 0) { /* the field's symbols as bytes */
        if (len > r->text_cap) {
            free(r->text);
            r->text = (uint8_t*)malloc((size_t)len);
            r->text_cap = r->text ? len : 0;
        }
        if (!r->text) abort();
        for (int64_t k = 0; k < len; k++) r->text[k] = sym_at(r, buf, begin + k);
        p = r->text;
    }
    int ok = 1;
    int64_t iv = 0;
    double dv = 0.0;
    if (ty == TY_STRING) {
        iv = begin * r->unit_bytes;
    } else if (len == 0) {
        ok = 0; /* empty: the column default, not an error (Sec. 4.3) */
    } else {
        if (ty == TY_INT64) ok = conv_int64(p, len, &iv);
        else if (ty == TY_FLOAT64) ok = conv_float64(p, len, &dv, r->cloc);
        else if (ty == TY_TIMESTAMP_S) ok = conv_timestamp(p, len, &iv);
        else ok = conv_date(p, len, &iv);
        if (!ok) { r->conv_errors++; iv = 0; dv = 0.0; }
    }
    if (!r->values || rec >= r->cap_records) return;
    if (ty == TY_FLOAT64) ((double*)r->values[c])[rec] = dv;
    else ((int64_t*)r->values[c])[rec] = iv;
    if (ty == TY_STRING) r->str_end[c][rec] = end * r->unit_bytes;
    r->valid[c][rec] = (uint8_t)ok;
}

/* Close field [b, e): index F, column r->col of record r->R. */
static void close_field(run_t* r, const uint8_t* buf, int64_t b, int64_t e,
                        int first_tag, int last_tag, int is_record)
{
    /* field_offsets holds cap_fields + 1 entries, column_ids cap_fields */
    if (r->field_offsets && r->F <= r->cap_fields) r->field_offsets[r->F] = b * r->unit_bytes;
    if (r->column_ids && r->F < r->cap_fields) r->column_ids[r->F] = (int32_t)r->col;
    convert_field(r, buf, b, e, first_tag, last_tag, r->R, r->col);
    r->F++;
    if (is_record) {
        int64_t nf = r->col + 1;
        if (nf != r->ncols) r->ragged++;
        if (r->R == 0 || nf < r->min_fields) r->min_fields = nf;
        if (nf > r->max_fields) r->max_fields = nf;
        for (int64_t c = nf; c < r->ncols; c++) write_default(r, r->R, c);
        r->R++;
        if (r->record_offsets && r->R <= r->cap_records) r->record_offsets[r->R] = r->F;
        r->col = 0;
    } else {
        r->col++;
    }
}

static int parse_run(const uint8_t* buf, const uint16_t* u16, int64_t n, const orc_dfa* dfa,
                     int32_t ncols, const int32_t* types,
                     int64_t cap_records, int64_t cap_fields,
                     int64_t* record_offsets, int64_t* field_offsets, int32_t* column_ids,
                     void** values, uint8_t** valid, int64_t** str_end,
                     orc_result* res)
{
    if (!dfa || !res || n < 0 || ncols < 0) return -1;
    /* a run that starts in the invalid state has no transition into it to
     * report (Sec. 4.3 flags the transition), so such a DFA is rejected */
    if (dfa->invalid_state >= 0 && dfa->invalid_state == dfa->start_state) return -1;
    run_t r;
    memset(&r, 0, sizeof r);
    r.dfa = dfa;
    r.ncols = ncols;
    r.types = types;
    r.cap_records = cap_records;
    r.cap_fields = cap_fields;
    r.record_offsets = record_offsets;
    r.field_offsets = field_offsets;
    r.column_ids = column_ids;
    r.values = values;
    r.valid = valid;
    r.str_end = str_end;
    r.cloc = newlocale(LC_ALL_MASK, "C", (locale_t)0);
    r.u16 = u16;
    r.unit_bytes = u16 ? 2 : 1;

    if (record_offsets && cap_records >= 0) record_offsets[0] = 0;

    int32_t s = dfa->start_state;
    int64_t first_inv = -1;
    int64_t fbeg = 0;          /* first byte of the open field */
    int first_tag = TAG_DATA;  /* tag of the open field's first symbol */
    int prev_tag = TAG_DATA;   /* tag of the previous symbol */
    int last_tag = -1;         /* tag of the last symbol read (-1: none) */
    int64_t last_end = 0;      /* end + 1 of the last closed field */

    for (int64_t i = 0; i < n; i++) {
        int g = dfa->group_of[sym_at(&r, buf, i)];
        int t = dfa->tag[g][s];
        int32_t s2 = dfa->next[g][s];
        if (dfa->invalid_state >= 0 && s2 == dfa->invalid_state &&
            s != dfa->invalid_state && first_inv < 0)
            first_inv = i;
        if (i == fbeg) first_tag = t;
        if (t == TAG_FIELD || t == TAG_RECORD) {
            close_field(&r, buf, fbeg, i, first_tag, prev_tag, t == TAG_RECORD);
            fbeg = i + 1;
            last_end = i + 1;
        }
        prev_tag = t;
        last_tag = t;
        s = s2;
    }
    /* End of input acts as a record delimiter unless the last symbol was one
     * (a final record without a trailing newline still counts). */
    if (n > 0 && last_tag != TAG_RECORD) {
        close_field(&r, buf, fbeg, n, first_tag, prev_tag, 1);
        last_end = n + 1;
    }
    if (field_offsets && r.F <= cap_fields) field_offsets[r.F] = r.F ? last_end * r.unit_bytes : 0;

    res->num_records = r.R;
    res->num_fields = r.F;
    res->first_invalid_offset = first_inv >= 0 ? first_inv * r.unit_bytes : -1;
    res->final_state = s;
    res->num_conversion_errors = r.conv_errors;
    res->num_ragged_records = r.ragged;
    res->min_record_fields = r.R ? r.min_fields : -1;
    res->max_record_fields = r.max_fields;
    if (r.R > cap_records || r.F > cap_fields) res->status = ORC_CAPACITY;
    else if (first_inv >= 0) res->status = ORC_INVALID_INPUT;
    else if (!((dfa->accept_mask >> s) & 1u)) res->status = ORC_NON_ACCEPTING_END;
    else res->status = ORC_OK;
    freelocale(r.cloc);
    free(r.text);
    return 0;
}

int orc_parse(const uint8_t* buf, int64_t n, const orc_dfa* dfa,
              int32_t ncols, const int32_t* types,
              int64_t cap_records, int64_t cap_fields,
              int64_t* record_offsets, int64_t* field_offsets, int32_t* column_ids,
              void** values, uint8_t** valid, int64_t** str_end,
              orc_result* res)
{
    return parse_run(buf, NULL, n, dfa, ncols, types, cap_records, cap_fields, record_offsets, field_offsets,
                     column_ids, values, valid, str_end, res);
}

int orc_parse_utf16(const uint16_t* units, int64_t n_units, const orc_dfa* dfa,
                    int32_t ncols, const int32_t* types,
                    int64_t cap_records, int64_t cap_fields,
                    int64_t* record_offsets, int64_t* field_offsets, int32_t* column_ids,
                    void** values, uint8_t** valid, int64_t** str_end,
                    orc_result* res)
{
    if (n_units > 0 && !units) return -1;
    return parse_run(NULL, units, n_units, dfa, ncols, types, cap_records, cap_fields, record_offsets,
                     field_offsets, column_ids, values, valid, str_end, res);
}

/* Rejecting the records that do not conform to the expected number of
 * columns (Sec. 4.3, inferring or validating the number of columns): every
 * record among the first R whose field count differs from ncols loses its
 * typed values (value 0, valid 0, empty span in every column); its fields
 * stay in the field arrays and in the counters. */
void orc_reject_ragged(int32_t ncols, const int32_t* types, int64_t R, const int64_t* record_offsets,
                       void** values, uint8_t** valid, int64_t** str_end)
{
    for (int64_t rec = 0; rec < R; rec++) {
        if (record_offsets[rec + 1] - record_offsets[rec] == ncols) continue;
        for (int32_t c = 0; c < ncols; c++) {
            if (types[c] == TY_SKIP) continue;
            if (types[c] == TY_FLOAT64) ((double*)values[c])[rec] = 0.0;
            else ((int64_t*)values[c])[rec] = 0;
            if (types[c] == TY_STRING) str_end[c][rec] = 0;
            valid[c][rec] = 0;
        }
    }
}

/* A string column's materialised values (Sec. 3.3: a column's symbol string
 * holds the fields' symbols without the control symbols): one sequential DFA
 * run from the start state; every DATA symbol of a field in column `column`
 * of a record r < cap_records is appended to record r's value. offsets[r] is
 * where record r's value begins in chars, offsets[R'] (R' = min(R,
 * cap_records)) the total length; chars beyond cap_chars are not written.
 * A record without that column has an empty value. With terminator >= 0
 * every value is followed by that byte (the inline-terminated form of
 * Sec. 4.1; the offsets then include it). Returns the total. */
int64_t orc_materialize(const uint8_t* buf, int64_t n, const orc_dfa* dfa, int32_t column, int64_t cap_records,
                        int64_t* offsets, uint8_t* chars, int64_t cap_chars, int32_t terminator)
{
    int32_t s = dfa->start_state;
    int64_t rec = 0, col = 0, total = 0;
    int last_tag = -1;
    if (cap_records >= 0 && offsets) offsets[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        const int g = dfa->group_of[buf[i]];
        const int t = dfa->tag[g][s];
        s = dfa->next[g][s];
        last_tag = t;
        if (t == TAG_RECORD) {
            if (terminator >= 0 && rec < cap_records) {  /* inline-terminated values (Sec. 4.1) */
                if (chars && total < cap_chars) chars[total] = (uint8_t)terminator;
                total++;
            }
            rec++;
            col = 0;
            if (rec <= cap_records && offsets) offsets[rec] = total;
        } else if (t == TAG_FIELD) {
            col++;
        } else if (t == TAG_DATA && col == column && rec < cap_records) {
            if (chars && total < cap_chars) chars[total] = buf[i];
            total++;
        }
    }
    /* end of input closes the last record unless a record delimiter did */
    if (n > 0 && last_tag != TAG_RECORD) {
        if (terminator >= 0 && rec < cap_records) {
            if (chars && total < cap_chars) chars[total] = (uint8_t)terminator;
            total++;
        }
        rec++;
        if (rec <= cap_records && offsets) offsets[rec] = total;
    }
    return total;
}

/* The same over UTF-16 text (Sec. 4.2): symbols are code units (a unit below
 * 0x80 is that ASCII symbol, any other reads as byte 0x80), the values'
 * data units are copied as they are, offsets count code units, and the
 * terminator is a code unit. */
int64_t orc_materialize_utf16(const uint16_t* units, int64_t n, const orc_dfa* dfa, int32_t column,
                              int64_t cap_records, int64_t* offsets, uint16_t* chars, int64_t cap_chars,
                              int32_t terminator)
{
    int32_t s = dfa->start_state;
    int64_t rec = 0, col = 0, total = 0;
    int last_tag = -1;
    if (cap_records >= 0 && offsets) offsets[0] = 0;
    for (int64_t i = 0; i < n; i++) {
        const int g = dfa->group_of[units[i] < 0x80 ? units[i] : 0x80];
        const int t = dfa->tag[g][s];
        s = dfa->next[g][s];
        last_tag = t;
        if (t == TAG_RECORD) {
            if (terminator >= 0 && rec < cap_records) {
                if (chars && total < cap_chars) chars[total] = (uint16_t)terminator;
                total++;
            }
            rec++;
            col = 0;
            if (rec <= cap_records && offsets) offsets[rec] = total;
        } else if (t == TAG_FIELD) {
            col++;
        } else if (t == TAG_DATA && col == column && rec < cap_records) {
            if (chars && total < cap_chars) chars[total] = units[i];
            total++;
        }
    }
    if (n > 0 && last_tag != TAG_RECORD) {
        if (terminator >= 0 && rec < cap_records) {
            if (chars && total < cap_chars) chars[total] = (uint16_t)terminator;
            total++;
        }
        rec++;
        if (rec <= cap_records && offsets) offsets[rec] = total;
    }
    return total;
}

/* Type inference (Sec. 4.3): a field's symbols (its enclosing control
 * symbols stripped, as for conversion) admit a set of types -- INT64 if they
 * convert as one, FLOAT64 if they follow the float grammar, DATE_DAYS and
 * TIMESTAMP_S if they convert as those; a column's inferred type is the
 * narrowest type every non-empty field of the column admits, in the order
 * INT64, FLOAT64, DATE_DAYS, TIMESTAMP_S, else STRING (also for a column
 * without non-empty fields). One sequential DFA run; columns >= ncols are
 * ignored. nonempty[c] receives the number of non-empty fields. */
void orc_infer_types(const uint8_t* buf, int64_t n, const orc_dfa* dfa, int32_t ncols, int32_t* types,
                     int64_t* nonempty)
{
    enum { OK_INT = 1, OK_FLOAT = 2, OK_DATE = 4, OK_TS = 8 };
    uint32_t* mask = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(ncols > 0 ? ncols : 1));
    for (int32_t c = 0; c < ncols; c++) { mask[c] = OK_INT | OK_FLOAT | OK_DATE | OK_TS; nonempty[c] = 0; }
    int32_t s = dfa->start_state;
    int64_t col = 0, fbeg = 0;
    int first_tag = TAG_DATA, prev_tag = TAG_DATA, last_tag = -1;
    for (int64_t i = 0; i <= n; i++) {
        int t, closes;
        if (i < n) {
            const int g = dfa->group_of[buf[i]];
            t = dfa->tag[g][s];
            s = dfa->next[g][s];
            if (i == fbeg) first_tag = t;
            closes = t == TAG_FIELD || t == TAG_RECORD;
        } else {  /* end of input closes the last field unless a record delimiter did */
            t = TAG_RECORD;
            closes = n > 0 && last_tag != TAG_RECORD;
        }
        if (closes) {
            if (col < ncols) {
                int64_t b = fbeg, e = i;
                if (e > b && first_tag == TAG_CONTROL) b++;
                if (e - 1 >= b && prev_tag == TAG_CONTROL) e--;
                if (e > b) {
                    int64_t iv;
                    uint32_t m = 0;
                    if (conv_int64(buf + b, e - b, &iv)) m |= OK_INT;
                    if (float_grammar(buf + b, e - b)) m |= OK_FLOAT;
                    if (conv_date(buf + b, e - b, &iv)) m |= OK_DATE;
                    if (conv_timestamp(buf + b, e - b, &iv)) m |= OK_TS;
                    mask[col] &= m;
                    nonempty[col]++;
                }
            }
            col = t == TAG_RECORD ? 0 : col + 1;
            fbeg = i + 1;
        }
        if (i < n) { prev_tag = t; last_tag = t; }
    }
    for (int32_t c = 0; c < ncols; c++) {
        const uint32_t m = nonempty[c] ? mask[c] : 0;
        types[c] = (m & OK_INT) ? TY_INT64 : (m & OK_FLOAT) ? TY_FLOAT64 : (m & OK_DATE) ? TY_DATE_DAYS
                 : (m & OK_TS) ? TY_TIMESTAMP_S : TY_STRING;
    }
    free(mask);
}

/* Skipping rows (Sec. 4.3): rows are the input's line-feed separated lines
 * (a record may span several, so this is not the DFA's record structure);
 * row k is the bytes after the k-th line feed up to and including the next
 * one. The bytes of every row in one of the half-open ranges [first, last)
 * (ranges[2i], ranges[2i+1]) are dropped; the rest is copied to out in
 * order. Returns the number of bytes kept. */
int64_t orc_skip_rows(const uint8_t* buf, int64_t n, const int64_t* ranges, int32_t nranges, uint8_t* out)
{
    int64_t row = 0, m = 0;
    for (int64_t i = 0; i < n; i++) {
        int skip = 0;
        for (int32_t k = 0; k < nranges; k++)
            if (row >= ranges[2 * k] && row < ranges[2 * k + 1]) skip = 1;
        if (!skip) out[m++] = buf[i];
        if (buf[i] == '\n') row++;
    }
    return m;
}

/* Single conversions, exposed so that tests can pin them against Python's
 * int(), float() and calendar arithmetic on hand-picked cases. */
int orc_conv(int32_t type, const uint8_t* p, int64_t len, int64_t* iv, double* dv)
{
    locale_t cloc = newlocale(LC_ALL_MASK, "C", (locale_t)0);
    int ok = 0;
    *iv = 0;
    *dv = 0.0;
    if (type == TY_INT64) ok = conv_int64(p, len, iv);
    else if (type == TY_FLOAT64) ok = conv_float64(p, len, dv, cloc);
    else if (type == TY_TIMESTAMP_S) ok = conv_timestamp(p, len, iv);
    else if (type == TY_DATE_DAYS) ok = conv_date(p, len, iv);
    freelocale(cloc);
    return ok;
}
