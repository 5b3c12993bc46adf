// Host-side validation of a pp_dfa_t, shared by the entry points that take
// DFAs (single buffer, batch, stream).
#pragma once
#include "parparaw.h"

namespace pp {

// Workspaces hold 64-bit atomics and 16-byte vectors: 256-byte alignment
// (what hipMalloc returns) is required of every d_ws argument.
inline bool ws_aligned(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

// States and groups in range, every transition and tag in range, and an
// invalid state (if any) that absorbs every symbol and is not the start state
// (a run that starts there has no transition into it to report).
inline pp_status_t check_dfa_tables(const pp_dfa_t* d)
{
    if (!d) return PP_ERR_ARG;
    if (d->num_states < 1 || d->num_states > PP_MAX_STATES) return PP_ERR_DFA;
    if (d->num_groups < 1 || d->num_groups > PP_MAX_GROUPS) return PP_ERR_DFA;
    if (d->start_state < 0 || d->start_state >= d->num_states) return PP_ERR_DFA;
    if (d->invalid_state < -1 || d->invalid_state >= d->num_states) return PP_ERR_DFA;
    if (d->invalid_state == d->start_state) return PP_ERR_DFA;
    for (int b = 0; b < 256; ++b)
        if (d->group_of[b] >= d->num_groups) return PP_ERR_DFA;
    for (int g = 0; g < d->num_groups; ++g)
        for (int s = 0; s < d->num_states; ++s) {
            if (d->next[g][s] >= d->num_states || d->tag[g][s] > PP_TAG_RECORD) return PP_ERR_DFA;
            if (s == d->invalid_state && d->next[g][s] != s) return PP_ERR_DFA;  // must absorb
        }
    return PP_OK;
}

}  // namespace pp
