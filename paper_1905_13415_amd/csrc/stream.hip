// End-to-end streaming form (Sec. 4.4): a host-resident input, larger than
// what the device holds at once, parsed partition by partition with the
// transfers overlapped with the parsing, and the parsed columns returned to
// host memory.
//
// Pipeline, for partitions k = 0, 1, ... of P new bytes each, over two device
// input buffers laid out as [carry region of M bytes | P bytes]:
//   - copy stream: host-to-device transfer of partition k's new bytes into
//     buffer k%2 behind its carry region;
//   - parse stream: the record that partition k-1 left unfinished (its carry-
//     over) is copied in front of them; a first pass over the partition
//     (structure only, no typed columns) finds where its last complete record
//     ends; the full parse then runs over the complete records only, and the
//     outputs are rebased to global byte, field and record indices;
//   - return stream: the rebased outputs go back to the caller's host arrays.
// The ordering constraint of Sec. 4.4: the next transfer into a buffer waits
// until that buffer's unfinished record has been copied out (and its parse
// has finished). The unfinished record restarts in the next partition from
// the DFA's start state, which is the state after every record delimiter
// (checked at create).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "dfa_check.h"
#include "parparaw.h"

namespace {

// Where a partition's complete records end, from the structure pass.
struct Boundary {
    int64_t status;       // the structure pass's result status
    int64_t records;      // complete records (closed by a record delimiter), or all at end of input
    int64_t fields;       // their fields
    int64_t end;          // one past the last complete record's delimiter (partition-relative)
    int64_t first_invalid;
    int64_t total_records, total_fields;  // of the structure pass (the last one closed by end of input)
};

// One thread: reads the structure pass's result and offsets. A partition
// that does not end in a record delimiter has its last record closed by end
// of input; that record is unfinished and is carried over.
__global__ void find_boundary(const pp_result_t* res, const int64_t* ro, const int64_t* fo, int64_t n,
                              int64_t cap_records, int64_t cap_fields, Boundary* out)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    Boundary b;
    b.status = res->status;
    b.first_invalid = res->first_invalid_offset;
    b.total_records = res->num_records;
    b.total_fields = res->num_fields;
    const int64_t R = res->num_records, F = res->num_fields;
    if (R > cap_records || F > cap_fields) {  // offsets not all written: the caller stops
        b.records = b.fields = b.end = -1;
        *out = b;
        return;
    }
    const bool ends_in_record = F == 0 || fo[F] == n;
    const int64_t rc = ends_in_record ? R : R - 1;
    b.records = rc;
    b.fields = ro[rc];
    b.end = fo[b.fields];
    *out = b;
}

// Adds the partition's global bases: byte offsets of fields and string
// spans, field indices of records.
__global__ void rebase(int64_t* fo, int64_t nf, int64_t* ro, int64_t nr, int64_t byte_base, int64_t field_base)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride) fo[i] += byte_base;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride) ro[i] += field_base;
}

__global__ void rebase_spans(int64_t* begin, int64_t* end, const uint8_t* valid, int64_t nr, int64_t byte_base)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nr; i += stride)
        if (valid[i]) {  // absent columns keep their (0, 0) default
            begin[i] += byte_base;
            end[i] += byte_base;
        }
}

static unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 255) / 256)); }

struct DevOut {  // one partition's device outputs
    int64_t *ro = nullptr, *fo = nullptr;
    int32_t* ci = nullptr;
    std::vector<void*> values;
    std::vector<uint8_t*> valid;
    std::vector<int64_t*> ends;
    pp_result_t* res = nullptr;
};

}  // namespace

struct pp_stream {
    pp_stream_config_t cfg;
    pp_dfa_t dfa;
    std::vector<int32_t> types;
    int32_t schema_flags = 0;
    int64_t P = 0, M = 0;
    uint8_t* buf[2] = {nullptr, nullptr};
    DevOut out[2];
    void* ws = nullptr;
    size_t ws_bytes = 0;
    Boundary* d_bound = nullptr;
    Boundary* h_bound = nullptr;       // pinned
    pp_result_t* h_res = nullptr;      // pinned, one per output set
    hipStream_t s_copy = nullptr, s_parse = nullptr, s_ret = nullptr;
    hipEvent_t ev_h2d[2] = {nullptr, nullptr}, ev_free[2] = {nullptr, nullptr};
    hipEvent_t ev_parsed[2] = {nullptr, nullptr}, ev_ret[2] = {nullptr, nullptr}, ev_bound = nullptr;
    std::vector<void*> allocs;
};

static void stream_free(pp_stream* s)
{
    if (!s) return;
    for (hipStream_t* st : {&s->s_copy, &s->s_parse, &s->s_ret})
        if (*st) (void)hipStreamSynchronize(*st);
    for (void* p : s->allocs) (void)hipFree(p);
    if (s->h_bound) (void)hipHostFree(s->h_bound);
    if (s->h_res) (void)hipHostFree(s->h_res);
    for (hipEvent_t e : {s->ev_h2d[0], s->ev_h2d[1], s->ev_free[0], s->ev_free[1], s->ev_parsed[0], s->ev_parsed[1],
                         s->ev_ret[0], s->ev_ret[1], s->ev_bound})
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t st : {s->s_copy, s->s_parse, s->s_ret})
        if (st) (void)hipStreamDestroy(st);
    delete s;
}

static bool dev_alloc(pp_stream* s, void** p, size_t bytes)
{
    *p = nullptr;
    if (hipMalloc(p, std::max<size_t>(bytes, 256)) != hipSuccess) return false;
    s->allocs.push_back(*p);
    return true;
}

extern "C" pp_status_t pp_stream_create(const pp_stream_config_t* cfg, const pp_dfa_t* dfa,
                                        const pp_schema_t* schema, pp_stream_t** out)
{
    if (!cfg || !dfa || !schema || !out) return PP_ERR_ARG;
    *out = nullptr;
    if (schema->ncols < 0 || schema->ncols > PP_MAX_COLUMNS || (schema->ncols > 0 && !schema->types))
        return PP_ERR_SCHEMA;
    for (int c = 0; c < schema->ncols; ++c)
        if (schema->types[c] < PP_INT64 || schema->types[c] > PP_SKIP) return PP_ERR_SCHEMA;
    if (schema->flags & ~PP_SCHEMA_REJECT_RAGGED) return PP_ERR_SCHEMA;
    const pp_status_t dst = pp::check_dfa_tables(dfa);
    if (dst != PP_OK) return dst;
    // a carried record restarts from the start state: every record delimiter
    // must lead there
    for (int g = 0; g < dfa->num_groups; ++g)
        for (int st = 0; st < dfa->num_states; ++st)
            if (dfa->tag[g][st] == PP_TAG_RECORD && dfa->next[g][st] != dfa->start_state) return PP_ERR_DFA;
    const int64_t P = cfg->partition_bytes ? cfg->partition_bytes : (int64_t)256 << 20;
    const int64_t M0 = cfg->max_record_bytes ? cfg->max_record_bytes : (int64_t)16 << 20;
    if (P < 4096 || M0 < 1 || P + M0 >= ((int64_t)1 << 40)) return PP_ERR_ARG;
    const int64_t M = (M0 + 255) / 256 * 256;  // the carry region, 256-byte aligned
    const int64_t cap_r = cfg->cap_records ? cfg->cap_records : (P + M) / 32 + 1;
    const int64_t cap_f = cfg->cap_fields ? cfg->cap_fields : (P + M) / 4 + 1;
    if (cap_r < 1 || cap_f < 1) return PP_ERR_ARG;
    const size_t ws_bytes = pp_workspace_size(P + M, &cfg->opts);
    if (ws_bytes == 0) return PP_ERR_ARG;

    pp_stream* s = new (std::nothrow) pp_stream();
    if (!s) return PP_ERR_ARG;
    s->cfg = *cfg;
    s->cfg.partition_bytes = P;
    s->cfg.max_record_bytes = M0;
    s->cfg.cap_records = cap_r;
    s->cfg.cap_fields = cap_f;
    s->dfa = *dfa;
    s->types.assign(schema->types, schema->types + schema->ncols);
    s->schema_flags = schema->flags;
    s->P = P;
    s->M = M;
    s->ws_bytes = ws_bytes;
    bool ok = true;
    for (int b = 0; b < 2 && ok; ++b) {
        ok = dev_alloc(s, (void**)&s->buf[b], (size_t)(s->M + P));
        DevOut& o = s->out[b];
        ok = ok && dev_alloc(s, (void**)&o.ro, (size_t)(cap_r + 1) * 8) && dev_alloc(s, (void**)&o.fo, (size_t)(cap_f + 1) * 8) &&
             dev_alloc(s, (void**)&o.ci, (size_t)cap_f * 4) && dev_alloc(s, (void**)&o.res, sizeof(pp_result_t));
        o.values.assign(s->types.size(), nullptr);
        o.valid.assign(s->types.size(), nullptr);
        o.ends.assign(s->types.size(), nullptr);
        for (size_t c = 0; c < s->types.size() && ok; ++c) {
            if (s->types[c] == PP_SKIP) continue;
            ok = dev_alloc(s, &o.values[c], (size_t)cap_r * 8) && dev_alloc(s, (void**)&o.valid[c], (size_t)cap_r);
            if (ok && s->types[c] == PP_STRING) ok = dev_alloc(s, (void**)&o.ends[c], (size_t)cap_r * 8);
        }
    }
    ok = ok && dev_alloc(s, &s->ws, ws_bytes) && dev_alloc(s, (void**)&s->d_bound, sizeof(Boundary));
    ok = ok && hipHostMalloc((void**)&s->h_bound, sizeof(Boundary), hipHostMallocDefault) == hipSuccess;
    ok = ok && hipHostMalloc((void**)&s->h_res, 2 * sizeof(pp_result_t), hipHostMallocDefault) == hipSuccess;
    for (hipStream_t* st : {&s->s_copy, &s->s_parse, &s->s_ret})
        ok = ok && hipStreamCreateWithFlags(st, hipStreamNonBlocking) == hipSuccess;
    for (hipEvent_t* e : {&s->ev_h2d[0], &s->ev_h2d[1], &s->ev_free[0], &s->ev_free[1], &s->ev_parsed[0],
                          &s->ev_parsed[1], &s->ev_ret[0], &s->ev_ret[1], &s->ev_bound})
        ok = ok && hipEventCreateWithFlags(e, hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        stream_free(s);
        return PP_ERR_HIP;
    }
    *out = s;
    return PP_OK;
}

extern "C" void pp_stream_destroy(pp_stream_t* s) { stream_free(s); }

namespace {

// Parse buf[0, n) into output set o (asynchronous on the parse stream);
// ncols = 0 for the structure pass.
pp_status_t run_parse(pp_stream* s, const uint8_t* d_in, int64_t n, DevOut& o, bool typed)
{
    pp_outputs_t po;
    memset(&po, 0, sizeof po);
    po.cap_records = s->cfg.cap_records;
    po.cap_fields = s->cfg.cap_fields;
    po.d_record_offsets = o.ro;
    po.d_field_offsets = o.fo;
    po.d_column_ids = o.ci;
    po.d_values = o.values.data();
    po.d_valid = o.valid.data();
    po.d_str_end = o.ends.data();
    po.d_result = o.res;
    pp_schema_t sch;
    sch.flags = typed ? s->schema_flags : 0;
    sch.ncols = typed ? (int32_t)s->types.size() : 0;
    sch.types = typed ? s->types.data() : nullptr;
    return pp_parse(d_in, n, &s->dfa, &sch, &po, s->ws, s->ws_bytes, &s->cfg.opts, s->s_parse);
}

bool copy_back(void* dst, const void* src, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return true;
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st) == hipSuccess;
}

}  // namespace

extern "C" pp_status_t pp_stream_parse(pp_stream_t* s, const uint8_t* h_in, int64_t n,
                                       const pp_host_outputs_t* out, pp_result_t* result,
                                       pp_stream_stats_t* stats)
{
    if (!s || n < 0 || (n > 0 && !h_in) || !out || !result) return PP_ERR_ARG;
    if (out->cap_records < 0 || out->cap_fields < 0 || !out->h_record_offsets || !out->h_field_offsets ||
        (out->cap_fields > 0 && !out->h_column_ids))
        return PP_ERR_ARG;
    const int nc = (int)s->types.size();
    for (int c = 0; c < nc; ++c) {
        if (s->types[c] == PP_SKIP || out->cap_records == 0) continue;
        if (!out->h_values || !out->h_valid || !out->h_values[c] || !out->h_valid[c] ||
            (s->types[c] == PP_STRING && (!out->h_str_end || !out->h_str_end[c])))
            return PP_ERR_ARG;
    }
    const int64_t P = s->P, M = s->M;
    const int64_t K = n == 0 ? 1 : (n + P - 1) / P;
    pp_stream_stats_t st;
    memset(&st, 0, sizeof st);
    pp_result_t acc;
    memset(&acc, 0, sizeof acc);
    acc.first_invalid_offset = -1;
    acc.min_record_fields = -1;
    acc.max_record_fields = 0;
    int64_t rbase = 0, fbase = 0;   // global records and fields before the current partition
    int64_t byte_base = 0;          // global offset of the current partition's first byte (its carry)
    int64_t carry = 0;              // bytes carried into the current partition
    int64_t prev_start = 0;         // where the previous partition's bytes begin in its buffer
    int64_t prev_end = 0;           // where its complete records end (relative to prev_start)
    bool stop = false;
    pp_status_t rc = PP_OK;
    int64_t final_status = PP_RESULT_OK, final_state = s->dfa.start_state;
    bool have_final = false;

#define PP_HIP(x)                 \
    do {                          \
        if ((x) != hipSuccess) { \
            rc = PP_ERR_HIP;      \
            goto done;            \
        }                         \
    } while (0)

    // the first two transfers need no wait (both buffers are free)
    for (int64_t k = 0; k < std::min<int64_t>(K, 2); ++k) {
        const int64_t nb = std::min<int64_t>(P, n - k * P);
        if (nb > 0) PP_HIP(hipMemcpyAsync(s->buf[k % 2] + M, h_in + k * P, (size_t)nb, hipMemcpyHostToDevice, s->s_copy));
        PP_HIP(hipEventRecord(s->ev_h2d[k % 2], s->s_copy));
    }
    for (int64_t k = 0; k < K && !stop; ++k) {
        const int b = (int)(k % 2);
        const int64_t nb = std::min<int64_t>(P, n - k * P);  // new bytes of partition k
        const bool last = k == K - 1;
        const int64_t start = M - carry;                     // partition k's bytes: buf[b][start, M + nb)
        const int64_t len = carry + std::max<int64_t>(nb, 0);
        DevOut& o = s->out[b];
        PP_HIP(hipStreamWaitEvent(s->s_parse, s->ev_h2d[b], 0));
        if (k >= 2) PP_HIP(hipStreamWaitEvent(s->s_parse, s->ev_ret[b], 0));  // output set b returned
        if (carry) {
            // the previous partition's unfinished record, in front of the new bytes
            const uint8_t* src = s->buf[1 - b] + prev_start + prev_end;
            if (pp_copy(s->buf[b] + start, src, (size_t)carry, s->s_parse) != PP_OK) { rc = PP_ERR_HIP; goto done; }
        }
        // the previous buffer may now take the next transfer (Sec. 4.4's ordering constraint)
        PP_HIP(hipEventRecord(s->ev_free[1 - b], s->s_parse));
        if (k + 1 < K && k >= 1) {
            const int64_t nb1 = std::min<int64_t>(P, n - (k + 1) * P);
            PP_HIP(hipStreamWaitEvent(s->s_copy, s->ev_free[1 - b], 0));
            PP_HIP(hipMemcpyAsync(s->buf[1 - b] + M, h_in + (k + 1) * P, (size_t)nb1, hipMemcpyHostToDevice, s->s_copy));
            PP_HIP(hipEventRecord(s->ev_h2d[1 - b], s->s_copy));
        }
        int64_t rc_k, fc_k, end_k;  // complete records, their fields, where they end
        if (!last) {
            // structure pass: where do the complete records end?
            if ((rc = run_parse(s, s->buf[b] + start, len, o, false)) != PP_OK) goto done;
            hipLaunchKernelGGL(find_boundary, dim3(1), dim3(64), 0, s->s_parse, o.res, o.ro, o.fo, len,
                               s->cfg.cap_records, s->cfg.cap_fields, s->d_bound);
            PP_HIP(hipMemcpyAsync(s->h_bound, s->d_bound, sizeof(Boundary), hipMemcpyDeviceToHost, s->s_parse));
            PP_HIP(hipEventRecord(s->ev_bound, s->s_parse));
            PP_HIP(hipEventSynchronize(s->ev_bound));
            const Boundary bd = *s->h_bound;
            if (bd.records < 0) {  // more records or fields than the device capacities
                acc.status = PP_RESULT_CAPACITY;
                acc.num_records = rbase + bd.total_records;
                acc.num_fields = fbase + bd.total_fields;
                stop = true;
                break;
            }
            rc_k = bd.records;
            fc_k = bd.fields;
            end_k = bd.end;
            if (bd.status == PP_RESULT_INVALID_INPUT) {
                // the rest of the input belongs to one field (the invalid state
                // absorbs): stop after this partition's complete records
                acc.first_invalid_offset = byte_base + bd.first_invalid;
                final_status = PP_RESULT_INVALID_INPUT;
                final_state = s->dfa.invalid_state;  // it absorbs the rest of the input
                have_final = true;
                stop = true;
            } else if (len - end_k > s->cfg.max_record_bytes) {
                rc = PP_ERR_UNSUPPORTED;  // a record longer than max_record_bytes
                goto done;
            }
            ++st.structure_passes;
        } else {
            rc_k = fc_k = end_k = -1;  // known from the parse itself
        }
        // the full parse over the complete records (the whole rest at the end)
        const int64_t plen = last ? len : end_k;
        if ((rc = run_parse(s, s->buf[b] + start, plen, o, true)) != PP_OK) goto done;
        PP_HIP(hipMemcpyAsync(&s->h_res[b], o.res, sizeof(pp_result_t), hipMemcpyDeviceToHost, s->s_parse));
        PP_HIP(hipEventRecord(s->ev_parsed[b], s->s_parse));
        ++st.partitions;
        if (last) {
            PP_HIP(hipEventSynchronize(s->ev_parsed[b]));
            rc_k = s->h_res[b].num_records;
            fc_k = s->h_res[b].num_fields;
            if (rc_k > s->cfg.cap_records || fc_k > s->cfg.cap_fields) {
                acc.status = PP_RESULT_CAPACITY;
                acc.num_records = rbase + rc_k;
                acc.num_fields = fbase + fc_k;
                stop = true;
                break;
            }
            final_status = s->h_res[b].status;
            final_state = s->h_res[b].final_state;
            if (s->h_res[b].first_invalid_offset >= 0 && acc.first_invalid_offset < 0)
                acc.first_invalid_offset = byte_base + s->h_res[b].first_invalid_offset;
            have_final = true;
        }
        if (rbase + rc_k > out->cap_records || fbase + fc_k > out->cap_fields) {
            acc.status = PP_RESULT_CAPACITY;
            acc.num_records = rbase + rc_k;
            acc.num_fields = fbase + fc_k;
            stop = true;
            break;
        }
        // rebase to global indices, then return the complete records
        hipLaunchKernelGGL(rebase, dim3(grid_for(fc_k + 1)), dim3(256), 0, s->s_parse, o.fo, fc_k + 1, o.ro, rc_k + 1,
                           byte_base, fbase);
        for (int c = 0; c < nc; ++c)
            if (s->types[c] == PP_STRING && rc_k > 0)
                hipLaunchKernelGGL(rebase_spans, dim3(grid_for(rc_k)), dim3(256), 0, s->s_parse, (int64_t*)o.values[c],
                                   o.ends[c], o.valid[c], rc_k, byte_base);
        PP_HIP(hipGetLastError());
        PP_HIP(hipEventRecord(s->ev_parsed[b], s->s_parse));
        PP_HIP(hipStreamWaitEvent(s->s_ret, s->ev_parsed[b], 0));
        if (!copy_back(out->h_field_offsets + fbase, o.fo, (size_t)(fc_k + 1) * 8, s->s_ret) ||
            !copy_back(out->h_record_offsets + rbase, o.ro, (size_t)(rc_k + 1) * 8, s->s_ret) ||
            !copy_back(out->h_column_ids + fbase, o.ci, (size_t)fc_k * 4, s->s_ret)) {
            rc = PP_ERR_HIP;
            goto done;
        }
        for (int c = 0; c < nc; ++c) {
            if (s->types[c] == PP_SKIP) continue;
            if (!copy_back((char*)out->h_values[c] + rbase * 8, o.values[c], (size_t)rc_k * 8, s->s_ret) ||
                !copy_back(out->h_valid[c] + rbase, o.valid[c], (size_t)rc_k, s->s_ret) ||
                (s->types[c] == PP_STRING &&
                 !copy_back(out->h_str_end[c] + rbase, o.ends[c], (size_t)rc_k * 8, s->s_ret))) {
                rc = PP_ERR_HIP;
                goto done;
            }
        }
        PP_HIP(hipEventRecord(s->ev_ret[b], s->s_ret));
        st.bytes_returned += (fc_k + 1) * 12 + (rc_k + 1) * 8;
        // counters of this partition's complete records (read once it is done)
        PP_HIP(hipEventSynchronize(s->ev_parsed[b]));
        {
            const pp_result_t& r = s->h_res[b];
            acc.num_conversion_errors += r.num_conversion_errors;
            acc.num_ragged_records += r.num_ragged_records;
            if (r.num_records > 0) {
                acc.min_record_fields = (uint64_t)r.min_record_fields < (uint64_t)acc.min_record_fields
                                            ? r.min_record_fields : acc.min_record_fields;
                acc.max_record_fields = std::max(acc.max_record_fields, r.max_record_fields);
            }
        }
        rbase += rc_k;
        fbase += fc_k;
        if (!last) {
            carry = len - end_k;
            st.carried_bytes += carry;
            st.max_carry = std::max(st.max_carry, carry);
            byte_base += end_k;
            prev_start = start;
            prev_end = end_k;
        }
    }
    if (acc.status != PP_RESULT_CAPACITY) {
        acc.status = have_final ? final_status : PP_RESULT_OK;
        acc.num_records = rbase;
        acc.num_fields = fbase;
    }
    acc.final_state = final_state;
    for (hipStream_t x : {s->s_copy, s->s_parse, s->s_ret}) PP_HIP(hipStreamSynchronize(x));
    *result = acc;
    if (stats) *stats = st;
done:
#undef PP_HIP
    if (rc != PP_OK)
        for (hipStream_t x : {s->s_copy, s->s_parse, s->s_ret}) (void)hipStreamSynchronize(x);
    return rc;
}
