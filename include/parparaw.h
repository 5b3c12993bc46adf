/*
 * parparaw.h -- C ABI of the MI355X (gfx950) parallel parser for
 * delimiter-separated text.
 *
 * The method is that of "ParPaRaw: Massively Parallel Parsing of
 * Delimiter-Separated Raw Data" (Stehle & Jacobsen, PVLDB 13(5), 2020):
 *  - Sec. 3.1: every chunk of the input is simulated from every DFA state,
 *    giving a state-transition vector; an exclusive scan of the vectors under
 *    composition gives every chunk its start state; a second pass from that
 *    state tags record delimiters, field delimiters and control symbols;
 *  - Sec. 3.2: record counts are prefix-summed into record offsets, column
 *    carries are scanned with the abs/rel operator into column offsets;
 *  - Sec. 3.3: fields are grouped by column and converted to typed columns;
 *  - Sec. 4.3: invalid transitions and non-accepting end states are
 *    reported, empty fields take the column default.
 *
 * All pointers named d_* are device pointers (HBM of the GPU that is
 * current when the call is made); everything else is host memory. Nothing
 * here allocates device memory: the caller owns inputs, outputs and
 * workspace. Calls are asynchronous on the given HIP stream and do no host
 * synchronisation, so they may be captured into a HIP graph. Errors in the
 * arguments are returned synchronously before any launch; outcomes that
 * depend on the data (invalid input, capacity) are written to the device
 * result record and are not errors.
 *
 * No function prints, aborts or throws. Functions are thread-safe as long as
 * concurrent calls use distinct workspaces and outputs.
 */
#ifndef PARPARAW_H
#define PARPARAW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pp_status_t;
#define PP_OK 0
#define PP_ERR_ARG (-1)         /* null pointer, negative size, bad option, misaligned workspace */
#define PP_ERR_DFA (-2)         /* DFA out of range, invalid state not absorbing or = start */
#define PP_ERR_SCHEMA (-3)      /* too many columns or unknown type */
#define PP_ERR_WORKSPACE (-4)   /* workspace smaller than pp_workspace_size() */
#define PP_ERR_HIP (-5)         /* a HIP launch failed */
#define PP_ERR_UNSUPPORTED (-6) /* a size or combination the library does not support */
#define PP_ERR_BUDGET (-7)      /* a request larger than the server's whole device budget */

/* Symbol tags (Sec. 3.1: record delimiter, field delimiter, control symbol,
 * or part of a field's value). */
#define PP_TAG_DATA 0
#define PP_TAG_CONTROL 1
#define PP_TAG_FIELD 2
#define PP_TAG_RECORD 3

/* Column types (Sec. 3.3 names integer, float and temporal conversions). */
#define PP_INT64 0       /* [+-]?[0-9]+ fitting int64 */
#define PP_FLOAT64 1     /* decimal, correctly rounded to nearest, ties to even */
#define PP_TIMESTAMP_S 2 /* YYYY-MM-DD hh:mm:ss or YYYY-MM-DDThh:mm:ss -> int64 s since 1970 UTC */
#define PP_DATE_DAYS 3   /* YYYY-MM-DD -> int64 days since 1970-01-01 */
#define PP_STRING 4      /* (begin, end) int64 byte span, enclosing control symbols stripped */
#define PP_SKIP 5        /* no typed output */

#define PP_MAX_STATES 8
#define PP_MAX_GROUPS 16
#define PP_MAX_COLUMNS 64

/* A DFA with a Mealy tag table. Tables are indexed [group][state], with
 * symbol groups as rows and states as columns (Table 1, Sec. 4.5).
 * Copied during the call. */
typedef struct {
    int32_t num_states;    /* 1..PP_MAX_STATES */
    int32_t num_groups;    /* 1..PP_MAX_GROUPS */
    int32_t start_state;   /* state before the first byte */
    int32_t invalid_state; /* -1: none; else absorbing (all next = itself) and not start_state */
    uint32_t accept_mask;  /* bit s set: ending in state s is accepted */
    uint8_t group_of[256]; /* symbol -> group */
    uint8_t next[16][16];  /* [group][state] -> next state */
    uint8_t tag[16][16];   /* [group][state] -> PP_TAG_* */
} pp_dfa_t;

/* Result record, written by the device (asynchronously). */
#define PP_RESULT_OK 0
#define PP_RESULT_INVALID_INPUT 1     /* a transition entered invalid_state */
#define PP_RESULT_NON_ACCEPTING_END 2 /* final state not in accept_mask */
#define PP_RESULT_CAPACITY 3          /* R > cap_records or F > cap_fields */
typedef struct {
    int64_t status;               /* CAPACITY, else INVALID_INPUT, else NON_ACCEPTING_END, else OK */
    int64_t num_records;          /* R (required size, even beyond capacity) */
    int64_t num_fields;           /* F */
    int64_t first_invalid_offset; /* byte of the transition into invalid_state, or -1 */
    int64_t final_state;
    int64_t num_conversion_errors; /* non-empty numeric fields that failed to convert */
    int64_t num_ragged_records;    /* records whose field count differs from ncols */
    /* Column counts for inferring or validating the number of columns
     * (Sec. 4.3): the fewest and the most fields in any record (a record's
     * fields include those beyond ncols; a blank line is one empty field).
     * The most is the inferred column count; equal values mean every record
     * has that many. Without records: -1 and 0. */
    int64_t min_record_fields;
    int64_t max_record_fields;
} pp_result_t;

/*
 * Outputs, all caller-allocated device memory (host struct of device pointers).
 *  d_record_offsets[cap_records + 1]: record r's first field index; [R] = F.
 *  d_field_offsets[cap_fields + 1]: field f's first byte; [F] = one past the
 *      last field's terminating delimiter (n + 1 when the input does not end
 *      in a record delimiter, since end of input then closes the last record).
 *  d_column_ids[cap_fields]: field f's position within its record.
 *  Per column c < ncols (by type):
 *      d_values[c][cap_records]: int64 (INT64, TIMESTAMP_S, DATE_DAYS, and
 *          the span begin for STRING) or double (FLOAT64);
 *      d_valid[c][cap_records]: 1 if present and converted, else 0 (value 0);
 *      d_str_end[c][cap_records]: span end, STRING columns only.
 *  Entries beyond a capacity are never written. d_values/d_valid/d_str_end
 *  are host arrays of ncols device pointers (NULL entries for SKIP).
 */
typedef struct {
    int64_t cap_records;
    int64_t cap_fields;
    int64_t* d_record_offsets;
    int64_t* d_field_offsets;
    int32_t* d_column_ids;
    void* const* d_values;
    uint8_t* const* d_valid;
    int64_t* const* d_str_end;
    pp_result_t* d_result;
    /* Optional (NULL: not written): the control-symbol bitmap, bit i%32 of
     * word i/32 set when byte i is a control symbol ((n + 31) / 32 words);
     * pp_materialize_strings reads it. */
    uint32_t* d_control_bitmap;
} pp_outputs_t;

/* Schema flags. PP_SCHEMA_REJECT_RAGGED: reject the records that do not
 * conform to the expected number of columns (Sec. 4.3, validating the number
 * of columns): a record whose field count differs from ncols gets the column
 * defaults (value 0, valid 0, empty span) in every typed column; its fields
 * stay in the offsets and column ids, and it is counted in
 * num_ragged_records. */
#define PP_SCHEMA_REJECT_RAGGED 1

typedef struct {
    int32_t ncols;        /* 0..PP_MAX_COLUMNS */
    int32_t flags;        /* PP_SCHEMA_* (0: none) */
    const int32_t* types; /* host array of ncols PP_* types */
} pp_schema_t;

/* Launch shape: a workgroup of block_threads threads parses a tile of
 * block_threads * bytes_per_thread bytes; bytes_per_thread is the chunk size
 * of Sec. 3.1. Supported (threads x bytes): 512x64 (the default), 256x64,
 * 512x32, 256x32, 256x16. Zero fields take the default. Any shape gives
 * identical outputs.
 * tile_order: 0 parses the tiles in input order. A value k > 0 (a
 * diagnostic for the single-pass scans, whose lookbacks then meet
 * predecessors in other states of completion) permutes each complete block
 * of 64 consecutive tiles: the block's i-th workgroup takes tile
 * ((2k+1) i + 37k) mod 64 of the block. Outputs are identical. Honoured by
 * pp_parse, pp_parse_noalloc, pp_parse_utf16, pp_infer_columns and the
 * streaming form;
 * pp_batch_create and pp_server_create reject k != 0; k < 0 is PP_ERR_ARG. */
typedef struct {
    int32_t bytes_per_thread;
    int32_t block_threads;
    int32_t tile_order;
} pp_options_t;

/* Device scratch that pp_parse needs for an input of n bytes (tile counter
 * and the per-tile lookback words of the single-pass scans). Every d_ws
 * argument of this library is device memory aligned to 256 bytes (as
 * hipMalloc returns it); a misaligned one is PP_ERR_ARG. */
size_t pp_workspace_size(int64_t n, const pp_options_t* opts);

/*
 * Parse d_in[0..n) under dfa into the outputs (Sec. 3.1-3.3, 4.3).
 * d_in: device bytes, read only, any alignment (16-byte alignment is faster).
 * d_ws: device workspace of at least pp_workspace_size(n, opts) bytes,
 *       owned by the caller and not shared with a concurrent call.
 * opts: NULL for defaults. stream: a hipStream_t, or NULL for the null stream.
 * Returns PP_OK once the work is enqueued.
 */
pp_status_t pp_parse(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa,
                     const pp_schema_t* schema, const pp_outputs_t* out,
                     void* d_ws, size_t ws_bytes, const pp_options_t* opts,
                     void* stream);

/*
 * pp_parse without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, hosts
 * that forbid allocation). Same arguments, outputs and errors as pp_parse,
 * minus d_ws/ws_bytes: the workspace is a static array of
 * PP_NOALLOC_SCRATCH_BYTES in the library's device code, one per GPU,
 * resident until the process ends. Its device address is looked up on the
 * first call on each device (the only set-up; nothing is allocated, by this
 * call or later ones). Returns PP_ERR_WORKSPACE when the input needs more
 * than that (pp_workspace_size(n, opts) > PP_NOALLOC_SCRATCH_BYTES: about
 * 8 GiB of input at the default launch shape, 1 GiB at 256x16), PP_ERR_HIP
 * if the address lookup fails.
 * Every call on one GPU shares that GPU's array: calls that overlap in time
 * on one GPU (other streams, other host threads) race and give wrong
 * results; serialise them, e.g. on one stream. Calls on different GPUs are
 * independent.
 */
#define PP_NOALLOC_SCRATCH_BYTES ((size_t)16 << 20)
pp_status_t pp_parse_noalloc(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa,
                             const pp_schema_t* schema, const pp_outputs_t* out,
                             const pp_options_t* opts, void* stream);

/*
 * Inferring the number of columns without a schema (Sec. 4.3): d_in[0..n)
 * is parsed for its structure only (no offsets, column ids or typed values
 * are written) and *d_result receives the result record, whose
 * max_record_fields is the inferred column count; min_record_fields ==
 * max_record_fields tells that every record has it, and num_records /
 * num_fields size the outputs of a following pp_parse. Status is never
 * CAPACITY. d_ws as for pp_parse (pp_workspace_size(n, opts) bytes).
 * Asynchronous on stream, no allocation.
 */
pp_status_t pp_infer_columns(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa, pp_result_t* d_result,
                             void* d_ws, size_t ws_bytes, const pp_options_t* opts, void* stream);

/*
 * Materialised string column (Sec. 3.3: a column's symbol string without its
 * control symbols). After pp_parse of d_in[0..n) with `parsed` as its
 * outputs, d_control_bitmap given, and the work of that parse ordered before
 * this call (e.g. the same stream): string column `column`'s values -- the
 * bytes of each record's span that are not control symbols (so enclosing
 * quotes, the first quote of a doubled pair and escape characters are
 * removed) -- back to back in d_chars, the Arrow large-string layout:
 * d_offsets[r] is where record r's value begins and d_offsets[R'] the total
 * length, R' = min(num_records, cap_records) (d_offsets holds cap_records + 1
 * entries). A record without the column, or rejected, has an empty value.
 * Bytes beyond cap_chars are not written (compare d_offsets[R'] with it).
 * terminator: -1 for the values alone (the offsets delimit them, the
 * vector-delimited form of Sec. 4.1), or a byte 0..255 written after every
 * value (the inline-terminated form; the offsets then include it).
 * Fields of any length are split over many wavefronts. d_ws: device scratch
 * of pp_materialize_workspace_size(n, cap_records) bytes. Asynchronous on
 * stream; no allocation. PP_ERR_ARG if the bitmap or the column's span
 * arrays are missing.
 */
size_t pp_materialize_workspace_size(int64_t n, int64_t cap_records);
pp_status_t pp_materialize_strings(const uint8_t* d_in, int64_t n, const pp_outputs_t* parsed, int32_t column,
                                   int32_t terminator, int64_t* d_offsets, uint8_t* d_chars, int64_t cap_chars,
                                   void* d_ws, size_t ws_bytes, void* stream);

/*
 * UTF-16 text (Sec. 4.2, multi-byte symbols). d_in holds n_units 16-bit code
 * units in the device's byte order (little-endian: UTF-16LE), any alignment
 * of 2. Parsed as pp_parse parses bytes, one symbol per code unit: a unit
 * below 0x80 is that ASCII symbol, every other unit (including surrogate
 * halves) reads as byte 0x80, so the DFA's structural symbols are ASCII and
 * all other characters are data of the group of 0x80. Every position in the
 * outputs (field offsets, string spans, the first invalid offset) is a byte
 * offset into d_in (twice the unit index); the control-symbol bitmap, when
 * requested, has one bit per code unit. Numbers, dates and times follow the
 * same grammars (ASCII digits). One launch, as pp_parse: each tile's code
 * units are narrowed to bytes as the tile is staged. d_ws:
 * pp_workspace_size_utf16(n_units, opts) bytes (pp_parse's workspace for
 * n_units symbols). Errors as pp_parse, returned before any work is queued;
 * also PP_ERR_ARG for a d_in at an odd address. Asynchronous on stream; no
 * allocation.
 */
size_t pp_workspace_size_utf16(int64_t n_units, const pp_options_t* opts);
/* Materialised string column of a pp_parse_utf16 parse (which wrote the
 * control-symbol bitmap, one bit per code unit): as pp_materialize_strings,
 * with code units for bytes -- d_chars receives the values' data code units
 * (cap_chars of them), d_offsets counts code units, the terminator is -1 or
 * a code unit 0..0xffff, and the workspace is
 * pp_materialize_workspace_size(n_units, cap_records). */
pp_status_t pp_materialize_strings_utf16(const uint16_t* d_in, int64_t n_units, const pp_outputs_t* parsed,
                                         int32_t column, int32_t terminator, int64_t* d_offsets, uint16_t* d_chars,
                                         int64_t cap_chars, void* d_ws, size_t ws_bytes, void* stream);
pp_status_t pp_parse_utf16(const uint16_t* d_in, int64_t n_units, const pp_dfa_t* dfa, const pp_schema_t* schema,
                           const pp_outputs_t* out, void* d_ws, size_t ws_bytes, const pp_options_t* opts,
                           void* stream);

/*
 * Type inference (Sec. 4.3). After pp_parse of d_in[0..n) with `parsed` as
 * its outputs, whose first ncols columns are STRING (e.g. the schema-less
 * parse of as many string columns as pp_infer_columns reports), ordered
 * before this call: for each of those columns, the narrowest type that every
 * non-empty field (enclosing control symbols stripped) admits, in the order
 * INT64 (converts without overflow), FLOAT64 (the float grammar), DATE_DAYS,
 * TIMESTAMP_S (valid calendar values), else STRING; a column without
 * non-empty fields is STRING. d_types[ncols] (int32) and d_nonempty[ncols]
 * (int64, non-empty fields per column) are device arrays; d_ws holds
 * pp_infer_types_workspace_size(ncols) bytes. Asynchronous; no allocation.
 */
size_t pp_infer_types_workspace_size(int32_t ncols);
pp_status_t pp_infer_types(const uint8_t* d_in, int64_t n, const pp_outputs_t* parsed, int32_t ncols,
                           int32_t* d_types, int64_t* d_nonempty, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Skipping rows (Sec. 4.3): rows are the input's line-feed separated lines
 * (row k: the bytes after the k-th line feed up to and including the next;
 * a quoted record may span several rows), so they are dropped before the
 * parse, by a parallel stream compaction. The bytes of every row in one of
 * the nranges half-open ranges [ranges[2i], ranges[2i+1]) (host array,
 * sorted, disjoint, non-empty, at most PP_MAX_SKIP_RANGES) are removed;
 * the rest of d_in[0..n) is written to d_out (n bytes of room) in order and
 * its length to *d_out_len (device). d_ws: pp_skip_rows_workspace_size(n)
 * bytes. Asynchronous; no allocation. The ranges are copied during the call.
 */
#define PP_MAX_SKIP_RANGES 64
size_t pp_skip_rows_workspace_size(int64_t n);
pp_status_t pp_skip_rows(const uint8_t* d_in, int64_t n, const int64_t* ranges, int32_t nranges, uint8_t* d_out,
                         int64_t* d_out_len, void* d_ws, size_t ws_bytes, void* stream);

/*
 * Skipping records (Sec. 4.3), after pp_parse with `parsed` as outputs and
 * `types` its schema (ncols entries), ordered before this call: the typed
 * values of every record in the nranges half-open ranges of record indices
 * (host array as for pp_skip_rows) get the column defaults (value 0, valid
 * 0, empty span), so consumers read them as ignored; their fields stay in the
 * offsets and column ids, and the counters of the result are unchanged.
 * Asynchronous; no allocation. (Selecting columns is the PP_SKIP type.)
 */
pp_status_t pp_skip_records(const pp_outputs_t* parsed, int32_t ncols, const int32_t* types, const int64_t* ranges,
                            int32_t nranges, void* stream);

/* Static text for a pp_status_t. */
const char* pp_status_str(pp_status_t s);

/* Device-to-device copy of n bytes with 16-byte nontemporal vector loads
 * and stores (bytes at unaligned ends), asynchronous on stream. The ranges
 * must not overlap (PP_ERR_ARG). It measures the practical HBM ceiling the
 * parse kernels are priced against, and moves a partition's unfinished
 * record in the streaming form. */
pp_status_t pp_copy(void* d_dst, const void* d_src, size_t n, void* stream);

/* ---- batched form ---------------------------------------------------------
 * Many independent buffers, each with its own DFA (dialect), schema and
 * outputs, parsed by one kernel launch: workgroups take (buffer, tile) work
 * items from one ticket counter in buffer-then-tile order, and each
 * buffer's tiles run the same pipeline as pp_parse (Sec. 3.1-3.3) with their
 * own lookback words. Results per buffer are identical to pp_parse's.
 *
 * Lifecycle: pp_batch_create (host only: validates, builds descriptor tables)
 * -> pp_batch_workspace_size -> pp_batch_bind (uploads the descriptors into
 * the caller's device workspace on a stream) -> pp_batch_launch any number of
 * times, or capture it once with pp_batch_graph_create and replay with
 * pp_batch_graph_launch. Launches allocate nothing and do not synchronise the
 * host. Inputs, outputs and workspace must stay valid while launches run; a
 * launch overwrites every output of every buffer. */
typedef struct {
    const uint8_t* d_in;   /* device bytes of this buffer (any alignment) */
    int64_t n;             /* its length */
    int32_t dialect;       /* index into the dfas array of pp_batch_create */
    int32_t ncols;         /* 0..PP_MAX_COLUMNS */
    const int32_t* types;  /* host array of ncols PP_* types (copied) */
    pp_outputs_t out;      /* its device outputs (pointer arrays are copied) */
} pp_batch_item_t;

typedef struct pp_batch pp_batch_t;
typedef struct pp_batch_graph pp_batch_graph_t;

pp_status_t pp_batch_create(const pp_dfa_t* dfas, int32_t ndfas, const pp_batch_item_t* items,
                            int32_t count, const pp_options_t* opts, pp_batch_t** batch);
size_t pp_batch_workspace_size(const pp_batch_t* batch);
/* Number of (buffer, tile) work items of the batch. */
int64_t pp_batch_num_tiles(const pp_batch_t* batch);
pp_status_t pp_batch_bind(pp_batch_t* batch, void* d_ws, size_t ws_bytes, void* stream);
pp_status_t pp_batch_launch(const pp_batch_t* batch, void* stream);
pp_status_t pp_batch_graph_create(const pp_batch_t* batch, pp_batch_graph_t** graph);
pp_status_t pp_batch_graph_launch(pp_batch_graph_t* graph, void* stream);
void pp_batch_graph_destroy(pp_batch_graph_t* graph);
void pp_batch_destroy(pp_batch_t* batch);

/* ---- launch-shape autotuner -------------------------------------------------
 * The launch shape fixes the chunk of Sec. 3.1 (bytes per thread) and the
 * scan tile (threads x bytes). These calls time every supported shape on the
 * caller's own inputs and outputs with HIP events (one untimed launch, then
 * reps timed ones per shape), synchronise the host on `stream`, and return
 * the fastest shape in *best; ms (optional, PP_NUM_SHAPES floats) receives
 * each shape's mean milliseconds, -1 for shapes skipped because the
 * workspace is too small for them. Outputs are overwritten with the results
 * of the last shape timed (identical for every shape). */
#define PP_NUM_SHAPES 5
/* The i-th supported shape, 0 <= i < PP_NUM_SHAPES. */
pp_status_t pp_shape(int32_t i, pp_options_t* out);
/* A workspace size that serves pp_parse of n bytes under every shape. */
size_t pp_autotune_workspace_size(int64_t n);
pp_status_t pp_parse_autotune(const uint8_t* d_in, int64_t n, const pp_dfa_t* dfa, const pp_schema_t* schema,
                              const pp_outputs_t* out, void* d_ws, size_t ws_bytes, int32_t reps, void* stream,
                              pp_options_t* best, float* ms);
/* A workspace size that serves the batch under every shape. */
size_t pp_batch_autotune_workspace_size(const pp_dfa_t* dfas, int32_t ndfas, const pp_batch_item_t* items,
                                        int32_t count);
pp_status_t pp_batch_autotune(const pp_dfa_t* dfas, int32_t ndfas, const pp_batch_item_t* items, int32_t count,
                              void* d_ws, size_t ws_bytes, int32_t reps, void* stream, pp_options_t* best,
                              float* ms);

/* ---- serving form ---------------------------------------------------------
 * A request loop in front of the batched form, for host-resident inputs: the
 * streaming setting of Sec. 4.4 (transfers overlapped with parsing) with
 * continuous batching. pp_server_create carves one device allocation of
 * hbm_budget_bytes (the only allocation the server makes) and starts a
 * scheduler thread. Requests are admitted in arrival order while a slot is
 * free and their input plus output blocks fit; admitted inputs are copied
 * from the caller's pinned host memory on copy streams; whenever a compute
 * stream is free, every request whose copy has finished joins one batched
 * launch there, so requests that arrive while others are on the device join
 * the next launch. A request whose outputs overflow the capacities it gave is
 * parsed again with the exact sizes (once). Outputs stay in device memory
 * until pp_server_release. Outputs of a request are identical to pp_parse's
 * on the same bytes, whatever else is in flight.
 *
 * Thread-safety: submit, poll, wait, release and get_stats may be called from
 * any thread; destroy must not race with the others. */
typedef struct pp_server pp_server_t;

typedef struct {
    size_t hbm_budget_bytes; /* device memory the server holds (>= 64 MiB) */
    int32_t max_slots;       /* admitted and not yet released requests, at most (>= 1) */
    int32_t copy_streams;    /* 1..4 host-to-device copy streams (0: 4) */
    int32_t compute_streams; /* 1..2 streams running batched launches (0: 2) */
    int32_t max_batch;       /* requests per batched launch (0: max_slots) */
    pp_options_t opts;       /* launch shape (zeros: default) */
} pp_server_config_t;

typedef struct {
    const uint8_t* h_in;   /* host bytes, pinned (hipHostMalloc); the caller keeps
                              them unchanged until the request completes */
    int64_t n;
    int32_t dialect;       /* index into the dfas of pp_server_create */
    int32_t ncols;         /* 0..PP_MAX_COLUMNS */
    const int32_t* types;  /* host array of ncols PP_* types (copied) */
    int64_t cap_records;   /* output capacities of the first attempt */
    int64_t cap_fields;
} pp_server_request_t;

typedef struct {
    uint64_t id;
    int64_t n;
    pp_result_t result;  /* status CAPACITY only if the exact sizes exceed the budget */
    pp_outputs_t out;    /* device pointers into the server's memory, valid until
                            pp_server_release; all NULL if no outputs were kept */
    int64_t t_arrival_ns;     /* host steady clock: submit */
    int64_t t_admit_ns;       /* admitted (memory carved, copy enqueued) */
    int64_t t_h2d_done_ns;    /* copy finished on the device */
    int64_t t_parse_done_ns;  /* its batched launch finished on the device */
} pp_server_completion_t;

typedef struct {
    int64_t submitted, completed, reparsed;
    int64_t batches, batched_requests, max_batch;
    int64_t bytes_completed;
    int64_t arena_bytes, arena_used_bytes, arena_peak_bytes;
    int64_t pending;
    int64_t hip_error; /* nonzero: a HIP call failed; the server has stopped */
} pp_server_stats_t;

pp_status_t pp_server_create(const pp_server_config_t* cfg, const pp_dfa_t* dfas, int32_t ndfas,
                             pp_server_t** server);
/* PP_ERR_BUDGET: the request's input plus outputs exceed the whole budget. */
pp_status_t pp_server_submit(pp_server_t* server, const pp_server_request_t* req, uint64_t* id);
/* Copies up to max completions, oldest first, into out; *got = how many. */
pp_status_t pp_server_poll(pp_server_t* server, pp_server_completion_t* out, int32_t max, int32_t* got);
/* Blocks until a completion is waiting or timeout_us passes. */
pp_status_t pp_server_wait(pp_server_t* server, int64_t timeout_us);
/* Frees a completed request's outputs and slot. */
pp_status_t pp_server_release(pp_server_t* server, uint64_t id);
pp_status_t pp_server_get_stats(pp_server_t* server, pp_server_stats_t* stats);
/* Waits for the device work in flight, then frees everything. */
void pp_server_destroy(pp_server_t* server);

/* ---- end-to-end streaming form (Sec. 4.4) -----------------------------------
 * A host-resident input of any size parsed partition by partition: each
 * partition's new bytes are copied to the device while the previous one is
 * parsed and its columns are copied back, on separate streams. The record a
 * partition leaves unfinished is carried over in front of the next
 * partition's bytes (the carry-over region of Sec. 4.4), and the next
 * transfer into a device buffer waits until that record has been moved out
 * of it. A structure pass (no typed columns) finds where a partition's last
 * complete record ends; the full parse then covers the complete records only,
 * so every record is parsed once with its whole bytes. Outputs are rebased
 * to global byte, field and record indices and written to host arrays.
 * Outputs and result equal pp_parse's on the whole input, with two
 * exceptions: a record longer than max_record_bytes fails the call
 * (PP_ERR_UNSUPPORTED), and on invalid input the stream stops after the
 * partition holding the first invalid transition (status INVALID_INPUT,
 * first_invalid_offset exact; records up to that partition's last record
 * delimiter are returned).
 * The DFA must enter its start state after every record delimiter (a
 * carried record restarts there); others get PP_ERR_DFA. */
typedef struct {
    int64_t partition_bytes;  /* new input bytes per partition (>= 4096; 0: 256 MiB) */
    int64_t max_record_bytes; /* longest record that may span partitions (0: 16 MiB) */
    int64_t cap_records;      /* device output capacity per partition (0: (P + M) / 32 + 1) */
    int64_t cap_fields;       /* (0: (P + M) / 4 + 1) */
    pp_options_t opts;        /* launch shape (zeros: default) */
} pp_stream_config_t;

/* Host output arrays, caller-allocated (pinned memory, hipHostMalloc, gives
 * the full transfer rate), with the layout of pp_outputs_t. */
typedef struct {
    int64_t cap_records;
    int64_t cap_fields;
    int64_t* h_record_offsets;      /* [cap_records + 1] */
    int64_t* h_field_offsets;       /* [cap_fields + 1] */
    int32_t* h_column_ids;          /* [cap_fields] */
    void* const* h_values;          /* per column, [cap_records] */
    uint8_t* const* h_valid;
    int64_t* const* h_str_end;
} pp_host_outputs_t;

typedef struct {
    int64_t partitions;        /* full parses run */
    int64_t structure_passes;  /* structure passes run (every partition but the last) */
    int64_t carried_bytes;     /* bytes moved into the next partition's carry-over region */
    int64_t max_carry;
    int64_t bytes_returned;    /* offset bytes copied back (typed columns not counted) */
} pp_stream_stats_t;

typedef struct pp_stream pp_stream_t;

/* Allocates the device buffers: two input buffers of max_record_bytes +
 * partition_bytes, two output sets of the per-partition capacities and a
 * workspace (the only allocations; parses allocate nothing). The DFA and
 * schema are copied. */
pp_status_t pp_stream_create(const pp_stream_config_t* cfg, const pp_dfa_t* dfa, const pp_schema_t* schema,
                             pp_stream_t** stream);
/* Parses h_in[0..n) (host memory; pinned gives the full rate) into the host
 * outputs and returns when everything is back in host memory (*result
 * holds the pp_result_t of the whole input; stats optional). Status
 * CAPACITY in *result: a partition exceeded the device capacities or the
 * input exceeded the host capacities (counts are those reached so far).
 * One call at a time per stream object. */
pp_status_t pp_stream_parse(pp_stream_t* stream, const uint8_t* h_in, int64_t n, const pp_host_outputs_t* out,
                            pp_result_t* result, pp_stream_stats_t* stats);
void pp_stream_destroy(pp_stream_t* stream);

#ifdef __cplusplus
}
#endif
#endif
