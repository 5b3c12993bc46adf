"""Dialects: the DFAs and schemas that a parse call is given as input.

A dialect is user-supplied format data, not part of the parsing method: the
method takes any DFA whose transition table has symbol groups as rows and
states as columns (Sec. 3.1; the row layout of Table 1 in Sec. 4.5). Both the
oracle and the GPU library receive these tables as inputs, so they live here,
beside the seeded input generators, and hold no parsing arithmetic.

Each cell of a table is a (next state, tag) pair. Tags mark what a symbol is
when read in a given state (Sec. 3.1: record delimiter, field delimiter,
control symbol, or part of a field's value):

    DATA = 0, CONTROL = 1, FIELD = 2, RECORD = 3
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Sequence

DATA, CONTROL, FIELD, RECORD = 0, 1, 2, 3
TAG_CHARS = {"D": DATA, "C": CONTROL, "F": FIELD, "R": RECORD}

# Column types of a schema.
INT64, FLOAT64, TIMESTAMP_S, DATE_DAYS, STRING, SKIP = 0, 1, 2, 3, 4, 5
TYPE_NAMES = ["INT64", "FLOAT64", "TIMESTAMP_S", "DATE_DAYS", "STRING", "SKIP"]

NO_STATE = -1


@dataclass
class Dfa:
    """A deterministic finite automaton over bytes, with a Mealy tag table.

    ``next_state[g][s]`` and ``tag[g][s]`` are indexed [group][state], the
    layout of Table 1. ``group_of[b]`` maps every byte value to its symbol
    group; symbols with identical transitions share a group (Sec. 4.5).
    ``invalid_state`` is the absorbing state that flags malformed input
    (Sec. 4.3, validating format), or NO_STATE when the dialect is lenient.
    """

    name: str
    state_names: List[str]
    group_symbols: List[bytes]  # explicit symbols of groups 0..G-2; last group is catch-all
    next_state: List[List[int]]
    tag: List[List[int]]
    start_state: int
    accept: List[int]
    invalid_state: int = NO_STATE
    group_of: bytes = field(default=b"", repr=False)

    def __post_init__(self):
        g = len(self.next_state)
        if not self.group_of:
            gm = bytearray([g - 1] * 256)
            for gi, syms in enumerate(self.group_symbols):
                for b in syms:
                    gm[b] = gi
            self.group_of = bytes(gm)

    @property
    def num_states(self) -> int:
        return len(self.state_names)

    @property
    def num_groups(self) -> int:
        return len(self.next_state)

    @property
    def accept_mask(self) -> int:
        m = 0
        for s in self.accept:
            m |= 1 << s
        return m


def _table(rows: Sequence[str], states: Sequence[str]):
    """Parse rows of 'NEXT/T' cells (one row per group) into next/tag lists."""
    idx = {n: i for i, n in enumerate(states)}
    nxt, tg = [], []
    for row in rows:
        cells = row.split()
        assert len(cells) == len(states), row
        nxt.append([idx[c.split("/")[0]] for c in cells])
        tg.append([TAG_CHARS[c.split("/")[1]] for c in cells])
    return nxt, tg


def paper6(delim: bytes = b",") -> Dfa:
    """The CSV DFA of Table 1 (states EOR, ENC, FLD, EOF, ESC, INV); the field
    delimiter group holds ',' as printed, or another delimiter byte.

    Next states are Table 1 verbatim. The paper gives no tag table, only that
    tags follow the format's rules (Sec. 3.1); the reading used here: a
    transition into EOR from a valid state is a record delimiter, into EOF a
    field delimiter; an opening quote (EOR/EOF -> ENC) and the quote that
    leaves an enclosure (ENC -> ESC) are control symbols; the second quote of
    a doubled pair (ESC -> ENC) is a literal, hence data.
    """
    states = ["EOR", "ENC", "FLD", "EOF", "ESC", "INV"]
    rows = [
        # EOR     ENC    FLD    EOF    ESC    INV
        "EOR/R ENC/D EOR/R EOR/R EOR/R INV/D",  # 0: \n
        "ENC/C ESC/C INV/D ENC/C ENC/D INV/D",  # 1: "
        "EOF/F ENC/D EOF/F EOF/F EOF/F INV/D",  # 2: ,
        "FLD/D ENC/D FLD/D FLD/D INV/D INV/D",  # 3: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("paper6", states, [b"\n", b'"', delim], nxt, tg, start_state=0,
               accept=[0, 2, 3, 4], invalid_state=5)


def csv4(delim: bytes = b",") -> Dfa:
    """Four-state quote-aware CSV DFA: paper6 with EOR and EOF merged.

    EOR and EOF have identical columns in Table 1, so they are one state (FB,
    field begin); the invalid state is dropped and its two entry cells become
    lenient data transitions. On valid RFC-4180 input the tags equal paper6's.
    """
    states = ["FB", "UQ", "QT", "QE"]
    rows = [
        # FB     UQ     QT     QE
        "FB/R FB/R QT/D FB/R",  # 0: \n
        "QT/C UQ/D QE/C QT/D",  # 1: "
        "FB/F FB/F QT/D FB/F",  # 2: delimiter
        "UQ/D UQ/D QT/D UQ/D",  # 3: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("csv4" + ("" if delim == b"," else repr(delim)), states,
               [b"\n", b'"', delim], nxt, tg, start_state=0, accept=[0, 1, 3])


def log6() -> Dfa:
    """Six-state extended-log DFA: space-delimited, "..." with backslash
    escapes, [...] brackets (FB, UQ, QT, QB, BR, AC)."""
    states = ["FB", "UQ", "QT", "QB", "BR", "AC"]
    rows = [
        # FB    UQ    QT    QB    BR    AC
        "FB/R FB/R QT/D QT/D FB/R FB/R",  # 0: \n
        "FB/F FB/F QT/D QT/D BR/D FB/F",  # 1: space
        "QT/C UQ/D AC/C QT/D BR/D UQ/D",  # 2: "
        "UQ/D UQ/D QB/C QT/D BR/D UQ/D",  # 3: backslash
        "BR/C UQ/D QT/D QT/D BR/D UQ/D",  # 4: [
        "UQ/D UQ/D QT/D QT/D AC/C UQ/D",  # 5: ]
        "UQ/D UQ/D QT/D QT/D BR/D UQ/D",  # 6: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("log6", states, [b"\n", b" ", b'"', b"\\", b"[", b"]"], nxt, tg,
               start_state=0, accept=[0, 1, 5])


def s3(delim: bytes = b",") -> Dfa:
    """Three states, unquoted fields with backslash escapes (FB, UQ, BS).

    The backslash is tagged data: it only moves the DFA to BS, where the next
    byte is data whatever it is. A string's span therefore stays raw."""
    states = ["FB", "UQ", "BS"]
    rows = [
        "FB/R FB/R UQ/D",  # 0: \n
        "FB/F FB/F UQ/D",  # 1: delimiter
        "BS/D BS/D UQ/D",  # 2: backslash (data; it only changes state)
        "UQ/D UQ/D UQ/D",  # 3: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("s3", states, [b"\n", delim, b"\\"], nxt, tg, start_state=0, accept=[0, 1])


def s5(delim: bytes = b",") -> Dfa:
    """csv4 made strict: a quote inside an unquoted field, or data after a
    closing quote, enters the absorbing invalid state."""
    states = ["FB", "UQ", "QT", "QE", "INV"]
    rows = [
        "FB/R FB/R QT/D FB/R INV/D",   # 0: \n
        "QT/C INV/D QE/C QT/D INV/D",  # 1: "
        "FB/F FB/F QT/D FB/F INV/D",   # 2: delimiter
        "UQ/D UQ/D QT/D INV/D INV/D",  # 3: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("s5", states, [b"\n", b'"', delim], nxt, tg, start_state=0,
               accept=[0, 1, 3], invalid_state=4)


def s7(delim: bytes = b",") -> Dfa:
    """Seven states: csv4 plus a backslash escape inside quotes (QB) and in
    unquoted fields (UB), plus the absorbing invalid state."""
    states = ["FB", "UQ", "QT", "QE", "QB", "UB", "INV"]
    rows = [
        # FB    UQ     QT    QE     QB    UB    INV
        "FB/R FB/R QT/D FB/R QT/D UQ/D INV/D",    # 0: \n
        "QT/C INV/D QE/C QT/D QT/D UQ/D INV/D",   # 1: "
        "FB/F FB/F QT/D FB/F QT/D UQ/D INV/D",    # 2: delimiter
        "UB/D UB/D QB/C INV/D QT/D UQ/D INV/D",   # 3: backslash
        "UQ/D UQ/D QT/D INV/D QT/D UQ/D INV/D",   # 4: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("s7", states, [b"\n", b'"', delim, b"\\"], nxt, tg, start_state=0,
               accept=[0, 1, 3], invalid_state=6)


def s8(delim: bytes = b" ") -> Dfa:
    """Eight states: log6 plus a backslash escape in unquoted fields (UB) and
    the absorbing invalid state (a quote or bracket inside an unquoted field)."""
    states = ["FB", "UQ", "QT", "QB", "BR", "AC", "UB", "INV"]
    rows = [
        # FB    UQ     QT    QB    BR    AC     UB    INV
        "FB/R FB/R QT/D QT/D FB/R FB/R UQ/D INV/D",    # 0: \n
        "FB/F FB/F QT/D QT/D BR/D FB/F UQ/D INV/D",    # 1: delimiter
        "QT/C INV/D AC/C QT/D BR/D INV/D UQ/D INV/D",  # 2: "
        "UB/D UB/D QB/C QT/D BR/D INV/D UQ/D INV/D",   # 3: backslash
        "BR/C INV/D QT/D QT/D BR/D INV/D UQ/D INV/D",  # 4: [
        "UQ/D UQ/D QT/D QT/D AC/C INV/D UQ/D INV/D",   # 5: ]
        "UQ/D UQ/D QT/D QT/D BR/D INV/D UQ/D INV/D",   # 6: other
    ]
    nxt, tg = _table(rows, states)
    return Dfa("s8", states, [b"\n", delim, b'"', b"\\", b"[", b"]"], nxt, tg,
               start_state=0, accept=[0, 1, 5], invalid_state=7)


def relabel(dfa: Dfa, perm: Sequence[int]) -> Dfa:
    """The same automaton with its states renumbered: old state s becomes
    perm[s]. Tables, start, invalid and accepting states are permuted
    together, so every input is tagged exactly as before; only the state
    numbers (the final state reported) change. Used to exercise start states
    other than 0."""
    k = dfa.num_states
    assert sorted(perm) == list(range(k)), perm
    inv = [0] * k
    for s, t in enumerate(perm):
        inv[t] = s
    nxt = [[perm[row[inv[t]]] for t in range(k)] for row in dfa.next_state]
    tg = [[row[inv[t]] for t in range(k)] for row in dfa.tag]
    return Dfa(dfa.name + "~" + "".join(map(str, perm)), [dfa.state_names[inv[t]] for t in range(k)],
               list(dfa.group_symbols), nxt, tg, start_state=perm[dfa.start_state],
               accept=sorted(perm[a] for a in dfa.accept),
               invalid_state=perm[dfa.invalid_state] if dfa.invalid_state != NO_STATE else NO_STATE,
               group_of=dfa.group_of)


@dataclass
class Schema:
    types: List[int]

    @property
    def ncols(self) -> int:
        return len(self.types)


# Schemas of the synthetic workloads (see datagen.workloads).
SCHEMA_C1 = Schema([INT64, INT64, FLOAT64, FLOAT64, TIMESTAMP_S, STRING, STRING, STRING])
SCHEMA_C2 = Schema([INT64] * 4 + [TIMESTAMP_S] * 2 + [FLOAT64] * 8 + [STRING] * 4)
SCHEMA_C3 = Schema([STRING] * 3 + [INT64] * 3 + [DATE_DAYS] + [STRING] * 2)
SCHEMA_LOG12 = Schema([STRING, STRING, STRING, STRING, STRING, INT64, INT64,
                       STRING, STRING, FLOAT64, INT64, STRING])

ALL_DFAS: Dict[str, callable] = {
    "paper6": paper6, "csv4": csv4, "log6": log6, "s3": s3, "s5": s5, "s7": s7, "s8": s8,
}
