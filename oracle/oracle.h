/*
 * Sequential reference parser (oracle) -- TEST INFRASTRUCTURE ONLY.
 * Private to oracle/; the GPU library neither includes nor links it.
 */
#ifndef PARPARAW_ORACLE_H
#define PARPARAW_ORACLE_H
#include <stdint.h>

typedef struct {
    int32_t num_states;
    int32_t num_groups;
    int32_t start_state;
    int32_t invalid_state; /* -1: none */
    uint32_t accept_mask;  /* bit s set: state s is accepting */
    uint8_t group_of[256];
    uint8_t next[16][16];  /* [group][state] */
    uint8_t tag[16][16];   /* [group][state]: 0 data, 1 control, 2 field, 3 record */
} orc_dfa;

enum { ORC_OK = 0, ORC_INVALID_INPUT = 1, ORC_NON_ACCEPTING_END = 2, ORC_CAPACITY = 3 };

typedef struct {
    int64_t status;
    int64_t num_records;
    int64_t num_fields;
    int64_t first_invalid_offset;
    int64_t final_state;
    int64_t num_conversion_errors;
    int64_t num_ragged_records;
    int64_t min_record_fields; /* fewest fields in a record; -1 without records */
    int64_t max_record_fields; /* most fields in a record; 0 without records */
} orc_result;

int orc_parse(const uint8_t* buf, int64_t n, const orc_dfa* dfa,
              int32_t ncols, const int32_t* types,
              int64_t cap_records, int64_t cap_fields,
              int64_t* record_offsets, int64_t* field_offsets, int32_t* column_ids,
              void** values, uint8_t** valid, int64_t** str_end,
              orc_result* res);

/* The same run over UTF-16 text (Sec. 4.2): n_units 16-bit code units (host
 * byte order); a unit below 0x80 is that ASCII symbol, any other unit reads
 * as byte 0x80. Every output position is a byte offset (twice the unit
 * index). */
int orc_parse_utf16(const uint16_t* units, int64_t n_units, const orc_dfa* dfa,
                    int32_t ncols, const int32_t* types,
                    int64_t cap_records, int64_t cap_fields,
                    int64_t* record_offsets, int64_t* field_offsets, int32_t* column_ids,
                    void** values, uint8_t** valid, int64_t** str_end,
                    orc_result* res);

void orc_reject_ragged(int32_t ncols, const int32_t* types, int64_t R, const int64_t* record_offsets,
                       void** values, uint8_t** valid, int64_t** str_end);

int64_t orc_materialize(const uint8_t* buf, int64_t n, const orc_dfa* dfa, int32_t column, int64_t cap_records,
                        int64_t* offsets, uint8_t* chars, int64_t cap_chars, int32_t terminator);

int64_t orc_materialize_utf16(const uint16_t* units, int64_t n, const orc_dfa* dfa, int32_t column,
                              int64_t cap_records, int64_t* offsets, uint16_t* chars, int64_t cap_chars,
                              int32_t terminator);

void orc_infer_types(const uint8_t* buf, int64_t n, const orc_dfa* dfa, int32_t ncols, int32_t* types,
                     int64_t* nonempty);

int64_t orc_skip_rows(const uint8_t* buf, int64_t n, const int64_t* ranges, int32_t nranges, uint8_t* out);

int orc_conv(int32_t type, const uint8_t* p, int64_t len, int64_t* iv, double* dv);

#endif
