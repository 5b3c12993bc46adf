"""The paper's chunked formulation, written plainly for small inputs --
TEST INFRASTRUCTURE ONLY.

Sec. 3.1: each chunk runs one DFA instance per state; the end state of the
instance that started in state i is entry i of the chunk's state-transition
vector. Vectors compose as (a o b)_i = b[a_i]; an exclusive scan of the
vectors under o, seeded with the identity, gives each chunk a vector whose
entry at the sequential start state is the chunk's true start state.

Sec. 3.2: given its start state, a chunk counts its record delimiters
(summed by an exclusive prefix sum into record offsets) and derives a column
carry: absolute when it contains a record delimiter (the number of field
delimiters after the last one), relative otherwise (its number of field
delimiters). Carries combine by the operator (+) of Sec. 3.2: the right
operand wins when absolute, otherwise the offsets add.

The printed bit formula for the carry masks fields before the *lowest* set
record bit, which contradicts the surrounding prose ("zero all bits ...
that precede the last set bit"); the prose is followed here.
"""
from __future__ import annotations

from typing import Callable, List, Sequence, Tuple

DATA, CONTROL, FIELD, RECORD = 0, 1, 2, 3
ABS, REL = 1, 0


def identity_vector(num_states: int) -> Tuple[int, ...]:
    return tuple(range(num_states))


def transition_vector(dfa, chunk: bytes) -> Tuple[int, ...]:
    """One DFA instance per start state, all advanced over the chunk."""
    v = list(range(dfa.num_states))
    for b in chunk:
        g = dfa.group_of[b]
        v = [dfa.next_state[g][s] for s in v]
    return tuple(v)


def compose(a: Sequence[int], b: Sequence[int]) -> Tuple[int, ...]:
    """(a o b)_i = b[a_i]: run a's chunk, then b's."""
    return tuple(b[x] for x in a)


def exclusive_scan(xs: Sequence, op: Callable, seed) -> List:
    out, acc = [], seed
    for x in xs:
        out.append(acc)
        acc = op(acc, x)
    return out


def inclusive_scan(xs: Sequence, op: Callable) -> List:
    out = []
    for i, x in enumerate(xs):
        out.append(x if i == 0 else op(out[-1], x))
    return out


def tag_chunk(dfa, chunk: bytes, start: int) -> Tuple[List[int], int]:
    """A single instance from the known start state: per-symbol tags."""
    s, tags = start, []
    for b in chunk:
        g = dfa.group_of[b]
        tags.append(dfa.tag[g][s])
        s = dfa.next_state[g][s]
    return tags, s


def column_carry(tags: Sequence[int]) -> Tuple[int, int]:
    """(ABS, field delimiters after the last record delimiter) if the chunk
    has a record delimiter, else (REL, field delimiters)."""
    if RECORD in tags:
        last = len(tags) - 1 - list(reversed(tags)).index(RECORD)
        return ABS, sum(1 for t in tags[last + 1:] if t == FIELD)
    return REL, sum(1 for t in tags if t == FIELD)


def oplus(a: Tuple[int, int], b: Tuple[int, int]) -> Tuple[int, int]:
    """The column-offset operator of Sec. 3.2."""
    if b[0] == ABS:
        return b
    return a[0], a[1] + b[1]


def parse_chunked(dfa, buf: bytes, cuts: Sequence[int]):
    """Run the chunked method over ``buf`` split before every index in
    ``cuts`` (sorted, inside (0, n)). Returns per-chunk start states, record
    and column prefixes, and the field structure assembled chunk by chunk:
    (record_offsets, field_offsets, column_ids)."""
    n = len(buf)
    bounds = [0] + list(cuts) + [n]
    chunks = [bytes(buf[bounds[i]:bounds[i + 1]]) for i in range(len(bounds) - 1)]
    if n == 0:
        chunks = []
    vecs = [transition_vector(dfa, c) for c in chunks]
    prefixes = exclusive_scan(vecs, compose, identity_vector(dfa.num_states))
    starts = [p[dfa.start_state] for p in prefixes]

    tags_per_chunk = []
    for c, s in zip(chunks, starts):
        tags, _ = tag_chunk(dfa, c, s)
        tags_per_chunk.append(tags)
    # End of input acts as a record delimiter unless the last symbol is one.
    virtual_end = n > 0 and tags_per_chunk[-1][-1] != RECORD

    rec_counts = [sum(1 for t in tg if t == RECORD) for tg in tags_per_chunk]
    fld_counts = [sum(1 for t in tg if t in (FIELD, RECORD)) for tg in tags_per_chunk]
    carries = [column_carry(tg) for tg in tags_per_chunk]
    if virtual_end:
        rec_counts[-1] += 1
        fld_counts[-1] += 1
        carries[-1] = (ABS, 0)
    rec_prefix = exclusive_scan(rec_counts, lambda a, b: a + b, 0)
    fld_prefix = exclusive_scan(fld_counts, lambda a, b: a + b, 0)
    col_prefix = exclusive_scan(carries, oplus, (ABS, 0))

    R = sum(rec_counts)
    F = sum(fld_counts)
    record_offsets = [0] * (R + 1)
    field_offsets = [0] * (F + 1)
    column_ids = [0] * F
    for j, tg in enumerate(tags_per_chunk):
        f = fld_prefix[j]
        r = rec_prefix[j]
        col = col_prefix[j][1]
        delims = [(bounds[j] + i, t) for i, t in enumerate(tg) if t in (FIELD, RECORD)]
        if virtual_end and j == len(tags_per_chunk) - 1:
            delims.append((n, RECORD))
        for pos, t in delims:
            # delimiter at pos closes field f (column col) and opens field f+1
            column_ids[f] = col
            field_offsets[f + 1] = pos + 1
            f += 1
            if t == RECORD:
                r += 1
                record_offsets[r] = f
                col = 0
            else:
                col += 1
    end_state = compose(prefixes[-1], vecs[-1])[dfa.start_state] if chunks else dfa.start_state
    return {
        "starts": starts, "vectors": vecs, "prefixes": prefixes,
        "rec_prefix": rec_prefix, "fld_prefix": fld_prefix, "col_prefix": col_prefix,
        "carries": carries, "tags": [t for tg in tags_per_chunk for t in tg],
        "record_offsets": record_offsets, "field_offsets": field_offsets,
        "column_ids": column_ids, "final_state": end_state,
    }
