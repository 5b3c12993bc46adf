"""Pins of the oracle against what the paper and mathematics fix.

Nothing here touches the GPU library. Each test pins the oracle (oracle.c,
via ctypes) or the plain chunked model (oracle/method_model.py) to something
other than itself: the paper's printed tables and examples, hand-derived
worked examples, closed forms (Python's exact integer, rational and calendar
arithmetic), invariants, and brute force over every split of tiny inputs.
"""
import calendar
import itertools
import random
from fractions import Fraction

import numpy as np
import pytest

import datagen
import oracle
from datagen import dialects as D
from oracle import method_model as M
from conftest import ints, read_golden


# ---- the paper's printed tables and examples ------------------------------

def test_table1_transitions_verbatim():
    """paper6's next-state table equals Table 1 cell by cell."""
    g = read_golden("table1_transitions.txt")
    states = g["states"].split()
    dfa = D.paper6()
    assert dfa.state_names == states
    rows = [v for k, v in g.items() if k.startswith("group")]
    assert len(rows) == dfa.num_groups
    for gi, row in enumerate(rows):
        cells = row.split()
        assert [states[s] for s in dfa.next_state[gi]] == cells
    # symbols -> groups as printed: \n 0, " 1, , 2, everything else 3
    assert dfa.group_of[ord("\n")] == 0 and dfa.group_of[ord('"')] == 1
    assert dfa.group_of[ord(",")] == 2
    assert all(dfa.group_of[b] == 3 for b in range(256) if b not in (10, 34, 44))


def test_prefix_sum_example():
    g = read_golden("prefix_sum_example.txt")
    x = ints(g["x"])
    assert M.inclusive_scan(x, lambda a, b: a + b) == ints(g["inclusive"])
    assert M.exclusive_scan(x, lambda a, b: a + b, 0) == ints(g["exclusive"])


@pytest.mark.parametrize("dfa", [D.paper6(), D.csv4()], ids=["paper6", "csv4"])
def test_ragged_example(dfa):
    g = read_golden("ragged_example.txt")
    buf = bytes.fromhex(g["input_hex"])
    r = oracle.parse(buf, dfa, [D.INT64, D.STRING])
    assert r.status == oracle.STATUS_OK
    assert r.num_records == int(g["num_records"]) and r.num_fields == int(g["num_fields"])
    assert list(r.record_offsets) == ints(g["record_offsets"])
    assert list(r.field_offsets) == ints(g["field_offsets"])
    assert list(r.column_ids) == ints(g["column_ids"])
    assert list(r.values[0]) == ints(g["col0_values"])
    assert list(r.valid[0]) == ints(g["col0_valid"])
    assert list(r.values[1]) == ints(g["col1_begin"])
    assert list(r.str_end[1]) == ints(g["col1_end"])
    assert list(r.valid[1]) == ints(g["col1_valid"])
    assert r.num_ragged_records == int(g["num_ragged_records"])
    assert r.min_record_fields == int(g["min_record_fields"])
    assert r.max_record_fields == int(g["max_record_fields"])


def _quoted():
    g = read_golden("quoted_example.txt")
    return g, bytes.fromhex(g["input_hex"])


def test_quoted_example_sequential():
    g, buf = _quoted()
    dfa = D.paper6()
    r = oracle.parse(buf, dfa, [D.STRING, D.STRING])
    assert r.status == oracle.STATUS_OK and r.final_state == int(g["final_state"])
    assert r.num_records == int(g["num_records"]) and r.num_fields == int(g["num_fields"])
    assert list(r.record_offsets) == ints(g["record_offsets"])
    assert list(r.field_offsets) == ints(g["field_offsets"])
    assert list(r.column_ids) == ints(g["column_ids"])
    spans = [tuple(int(v) for v in s.split("-")) for s in g["string_spans"].split()]
    got = []
    for rec in range(r.num_records):
        for c in range(2):
            got.append((int(r.values[c][rec]), int(r.str_end[c][rec])))
    assert got == spans
    # per-symbol tags of the sequential run
    tags, _ = M.tag_chunk(dfa, buf, dfa.start_state)
    assert [i for i, t in enumerate(tags) if t == M.RECORD] == ints(g["record_tags"])
    assert [i for i, t in enumerate(tags) if t == M.FIELD] == ints(g["field_tags"])
    assert [i for i, t in enumerate(tags) if t == M.CONTROL] == ints(g["control_tags"])


def test_quoted_example_chunked():
    """The chunked method on the worked example, step by step."""
    g, buf = _quoted()
    dfa = D.paper6()
    B = int(g["chunk_size"])
    out = M.parse_chunked(dfa, buf, list(range(B, len(buf), B)))
    for j, v in enumerate(out["vectors"]):
        assert list(v) == ints(g[f"vector {j}"])
    for j, p in enumerate(out["prefixes"]):
        assert list(p) == ints(g[f"prefix {j}"])
    assert out["starts"] == ints(g["chunk_starts"])
    want = [(M.ABS if c.startswith("abs") else M.REL, int(c[3:])) for c in g["carries"].split()]
    assert out["carries"] == want
    assert [c[1] for c in out["col_prefix"]] == ints(g["column_prefix"])
    assert all(c[0] == M.ABS for c in out["col_prefix"])
    assert out["rec_prefix"] == ints(g["record_prefix"])
    assert out["record_offsets"] == ints(g["record_offsets"])
    assert out["field_offsets"] == ints(g["field_offsets"])


# ---- algebra ---------------------------------------------------------------

@pytest.mark.parametrize("ns", [2, 3, 4])
def test_composition_associative_exhaustive(ns):
    """(a o b) o c == a o (b o c) over all ns^ns vectors, and the identity."""
    vecs = np.array(list(itertools.product(range(ns), repeat=ns)), dtype=np.int64)
    code = {tuple(v): i for i, v in enumerate(vecs.tolist())}
    k = len(vecs)
    table = np.empty((k, k), dtype=np.int64)
    for i in range(k):
        comp = vecs[:, :][:, vecs[i]] if False else None  # noqa
        for j in range(k):
            table[i, j] = code[M.compose(vecs[i], vecs[j])]
    ii, jj, kk = np.meshgrid(np.arange(k), np.arange(k), np.arange(k), indexing="ij")
    assert np.array_equal(table[table[ii, jj], kk], table[ii, table[jj, kk]])
    e = code[M.identity_vector(ns)]
    assert np.array_equal(table[e, :], np.arange(k)) and np.array_equal(table[:, e], np.arange(k))


def test_compose_matches_function_composition():
    """Composition is 'apply a, then b': (a o b)_i = b[a_i], not a[b_i]."""
    a, b = (1, 2, 0), (2, 2, 1)
    assert M.compose(a, b) == (2, 1, 2)
    assert M.compose(b, a) == (0, 0, 2)


def test_oplus_associative_and_identity():
    vals = [(t, o) for t in (M.ABS, M.REL) for o in range(4)]
    for a in vals:
        assert M.oplus((M.REL, 0), a) == a or a[0] == M.REL and M.oplus((M.REL, 0), a) == a
        assert M.oplus(a, (M.REL, 0)) == a
        for b in vals:
            for c in vals:
                assert M.oplus(M.oplus(a, b), c) == M.oplus(a, M.oplus(b, c))
    # Sec. 3.2's two cases
    assert M.oplus((M.REL, 3), (M.ABS, 1)) == (M.ABS, 1)
    assert M.oplus((M.ABS, 3), (M.REL, 2)) == (M.ABS, 5)


def test_column_carry_prose_reading():
    """Carry = field delimiters after the LAST record delimiter (prose of
    Sec. 3.2), not after the first as the printed BLSMSK formula would give."""
    F, R, D_ = M.FIELD, M.RECORD, M.DATA
    assert M.column_carry([F, R, F, F, R, F]) == (M.ABS, 1)
    assert M.column_carry([F, D_, F]) == (M.REL, 2)
    assert M.column_carry([R]) == (M.ABS, 0)


@pytest.mark.parametrize("dfa", [D.paper6(), D.csv4(), D.log6(), D.s7(), D.s8()],
                         ids=lambda d: d.name)
def test_homomorphism(dfa):
    """vec(xy) = vec(x) o vec(y) on random strings of the dialect's symbols."""
    rnd = random.Random(7)
    alphabet = [syms[0] for syms in dfa.group_symbols] + [ord("a")]
    for _ in range(300):
        x = bytes(rnd.choice(alphabet) for _ in range(rnd.randint(0, 12)))
        y = bytes(rnd.choice(alphabet) for _ in range(rnd.randint(0, 12)))
        assert M.transition_vector(dfa, x + y) == M.compose(M.transition_vector(dfa, x),
                                                            M.transition_vector(dfa, y))


# ---- brute force: every split of every tiny input ---------------------------

def _all_splits(n):
    for mask in range(1 << max(n - 1, 0)):
        yield [i + 1 for i in range(n - 1) if mask >> i & 1]


def _check_all_splits(dfa, buf):
    ref = oracle.parse(buf, dfa, [])
    seq_tags, _ = M.tag_chunk(dfa, buf, dfa.start_state)
    for cuts in _all_splits(len(buf)):
        out = M.parse_chunked(dfa, buf, cuts)
        assert out["tags"] == seq_tags
        assert out["final_state"] == ref.final_state
        assert out["record_offsets"] == list(ref.record_offsets), (buf, cuts)
        assert out["field_offsets"] == list(ref.field_offsets), (buf, cuts)
        assert out["column_ids"] == list(ref.column_ids), (buf, cuts)


@pytest.mark.parametrize("dfa", [D.paper6(), D.csv4()], ids=lambda d: d.name)
def test_brute_force_all_splits_csv(dfa):
    """Every string of length <= 6 over {LF, quote, comma, a}, every split."""
    alphabet = b'\n",a'
    for n in range(0, 7):
        for tup in itertools.product(alphabet, repeat=n):
            _check_all_splits(dfa, bytes(tup))


def test_brute_force_all_splits_log6():
    dfa = D.log6()
    alphabet = b'\n "\\[]a'
    for n in range(0, 5):
        for tup in itertools.product(alphabet, repeat=n):
            _check_all_splits(dfa, bytes(tup))


def test_csv4_equals_paper6_on_valid_input():
    """csv4 merges Table 1's EOR/EOF columns and drops INV; on every input
    that paper6 accepts, the two give identical outputs."""
    p6, c4 = D.paper6(), D.csv4()
    alphabet = b'\n",a'
    checked = 0
    for n in range(0, 8):
        for tup in itertools.product(alphabet, repeat=n):
            buf = bytes(tup)
            a = oracle.parse(buf, p6, [D.STRING, D.STRING, D.STRING])
            if a.status != oracle.STATUS_OK:
                continue
            b = oracle.parse(buf, c4, [D.STRING, D.STRING, D.STRING])
            checked += 1
            assert b.status == oracle.STATUS_OK
            assert np.array_equal(a.record_offsets, b.record_offsets)
            assert np.array_equal(a.field_offsets, b.field_offsets)
            assert np.array_equal(a.column_ids, b.column_ids)
            for c in range(3):
                assert np.array_equal(a.values[c], b.values[c])
                assert np.array_equal(a.str_end[c], b.str_end[c])
                assert np.array_equal(a.valid[c], b.valid[c])
    assert checked > 1000


# ---- status, validation, capacity ----------------------------------------

def test_invalid_quote_in_unquoted_field():
    """Sec. 4.3 (validating format): a quote read in FLD enters INV (Table 1);
    the offset of that transition is reported and INV absorbs the rest."""
    buf = b'ab,c"d,e\nf\n'
    r = oracle.parse(buf, D.paper6(), [])
    assert r.status == oracle.STATUS_INVALID_INPUT
    assert r.first_invalid_offset == 4
    assert r.final_state == 5
    assert r.num_records == 1 and r.num_fields == 2  # one field after byte 2: INV absorbs


def test_unterminated_quote_is_non_accepting():
    for dfa in (D.paper6(), D.csv4()):
        r = oracle.parse(b'a,"bc\n', dfa, [])
        assert r.status == oracle.STATUS_NON_ACCEPTING_END
        assert r.first_invalid_offset == -1


def test_capacity_reports_required_sizes():
    buf = b"1,2\n3,4\n5,6\n"
    r = oracle.parse(buf, D.csv4(), [D.INT64, D.INT64], cap_records=2, cap_fields=3)
    assert r.status == oracle.STATUS_CAPACITY
    assert r.num_records == 3 and r.num_fields == 6
    assert list(r.field_offsets) == [0, 2, 4, 6]
    assert list(r.record_offsets) == [0, 2, 4]


def test_empty_and_edge_inputs():
    dfa = D.csv4()
    r = oracle.parse(b"", dfa, [D.INT64])
    assert (r.num_records, r.num_fields, r.status) == (0, 0, oracle.STATUS_OK)
    assert list(r.field_offsets) == [0] and list(r.record_offsets) == [0]
    assert (r.min_record_fields, r.max_record_fields) == (-1, 0)
    # no trailing LF: the last record still counts; field_offsets[F] = n + 1
    r = oracle.parse(b"1,2", dfa, [D.INT64, D.INT64])
    assert list(r.field_offsets) == [0, 2, 4] and list(r.values[1]) == [2]
    # trailing field delimiter: an empty last field
    r = oracle.parse(b"1,", dfa, [D.INT64, D.INT64])
    assert r.num_fields == 2 and list(r.valid[1]) == [0] and r.num_conversion_errors == 0
    # blank line: a record with one empty field
    r = oracle.parse(b"\n\n", dfa, [D.INT64])
    assert r.num_records == 2 and r.num_fields == 2 and list(r.field_offsets) == [0, 1, 2]
    assert (r.min_record_fields, r.max_record_fields) == (1, 1)
    # extra fields are kept in the field arrays and dropped from typed output
    r = oracle.parse(b"1,2,3\n", dfa, [D.INT64])
    assert r.num_fields == 3 and r.num_ragged_records == 1 and list(r.values[0]) == [1]
    assert (r.min_record_fields, r.max_record_fields) == (3, 3)


@pytest.mark.parametrize("seed", range(6))
def test_column_counts_against_csv_module(seed):
    """Fewest and most fields per record (Sec. 4.3, inferring or validating
    the number of columns) against Python's csv module on random RFC-4180
    text: quoted fields with delimiters, line breaks and doubled quotes,
    empty fields, blank lines, with and without a final line break."""
    import csv
    import io
    rng = random.Random(seed)
    pieces = ["", "7", "abc", '"x,y"', '"a\nb"', '"say ""hi"""', '""', "-1.5"]
    recs = []
    for _ in range(rng.randrange(1, 60)):
        k = rng.choice([1, 1, 2, 3, 5, 8, 13]) if seed % 2 else rng.choice([4, 4, 4, 5])
        recs.append(",".join(rng.choice(pieces) for _ in range(k)))
    text = "\n".join(recs) + ("\n" if seed % 3 else "")
    rows = list(csv.reader(io.StringIO(text, newline="")))
    counts = [max(len(row), 1) for row in rows]  # the module gives [] for a blank line
    r = oracle.parse(text.encode(), D.csv4(), [D.STRING] * 4)
    assert r.status == oracle.STATUS_OK and r.num_records == len(rows)
    assert (r.min_record_fields, r.max_record_fields) == (min(counts), max(counts))
    assert r.num_ragged_records == sum(c != 4 for c in counts)


def test_reject_ragged_hand_examples():
    """Rejecting records whose column count differs from the schema's
    (Sec. 4.3): their typed values become the defaults, their fields stay."""
    t = b"1,Apples\n2\n"
    keep = oracle.parse(t, D.csv4(), [D.INT64, D.STRING])
    r = oracle.parse(t, D.csv4(), [D.INT64, D.STRING], reject_ragged=True)
    assert list(keep.values[0]) == [1, 2] and list(keep.valid[0]) == [1, 1]
    assert list(r.values[0]) == [1, 0] and list(r.valid[0]) == [1, 0]
    assert list(r.values[1]) == [2, 0] and list(r.str_end[1]) == [8, 0] and list(r.valid[1]) == [1, 0]
    assert list(r.field_offsets) == list(keep.field_offsets) and r.num_ragged_records == 1
    t = b"a,b,c\nd,e\n"
    r = oracle.parse(t, D.csv4(), [D.STRING, D.STRING], reject_ragged=True)
    assert list(r.values[0]) == [0, 6] and list(r.str_end[0]) == [0, 7] and list(r.valid[0]) == [0, 1]
    assert list(r.values[1]) == [0, 8] and list(r.str_end[1]) == [0, 9] and list(r.valid[1]) == [0, 1]
    assert list(r.record_offsets) == [0, 3, 5] and list(r.column_ids) == [0, 1, 2, 0, 1]


@pytest.mark.parametrize("seed", range(4))
def test_reject_ragged_against_csv_module(seed):
    """The records kept under rejection are exactly those Python's csv module
    reads with four fields, and their string spans (quotes stripped, doubled
    quotes undone) are the module's values."""
    import csv
    import io
    rng = random.Random(100 + seed)
    pieces = ["", "7", "abc", '"x,y"', '"a\nb"', '"say ""hi"""', '""', "-1.5"]
    recs = [",".join(rng.choice(pieces) for _ in range(rng.choice([3, 4, 4, 4, 5])))
            for _ in range(rng.randrange(5, 80))]
    text = ("\n".join(recs) + "\n").encode()
    rows = list(csv.reader(io.StringIO(text.decode(), newline="")))
    r = oracle.parse(text, D.csv4(), [D.STRING] * 4, reject_ragged=True)
    assert r.num_records == len(rows)
    for i, row in enumerate(rows):
        for c in range(4):
            if len(row) != 4:
                assert r.valid[c][i] == 0 and r.values[c][i] == 0 and r.str_end[c][i] == 0
                continue
            b, e = int(r.values[c][i]), int(r.str_end[c][i])
            raw_begin = int(r.field_offsets[r.record_offsets[i] + c])
            span = text[b:e].decode()
            if text[raw_begin:raw_begin + 1] == b'"':
                span = span.replace('""', '"')
            assert r.valid[c][i] == 1 and span == row[c], (i, c)


def test_materialize_quoted_example():
    """The hand-worked quoted example: control symbols (enclosing quotes and
    the first quote of a doubled pair) leave the values."""
    g = read_golden("quoted_example.txt")
    data = bytes.fromhex(g["input_hex"])
    for c in (0, 1):
        want = [bytes.fromhex(h) for h in g[f"materialized_col{c}_hex"].split("|")]
        for dfa in (D.paper6(), D.csv4()):
            offs, chars = oracle.materialize(data, dfa, c)
            got = [bytes(chars[offs[r]:offs[r + 1]]) for r in range(len(offs) - 1)]
            assert got == want, (c, dfa.name)


def test_materialize_inline_terminated():
    """The inline-terminated form (Sec. 4.1): every value followed by a
    terminator byte (here the ASCII unit separator), worked by hand for the
    quoted example; on random text, the vector-delimited values with the
    terminator after each."""
    data = bytes.fromhex(read_golden("quoted_example.txt")["input_hex"])
    offs, chars = oracle.materialize(data, D.paper6(), 0, terminator=0x1F)
    assert bytes(chars) == b'a\x1fd"e\x1f' and list(offs) == [0, 2, 6]
    offs, chars = oracle.materialize(data, D.paper6(), 1, terminator=0x1F)
    assert bytes(chars) == b"b,c\x1ff\x1f" and list(offs) == [0, 4, 6]
    text = bytes(datagen.c1().data[:30000])
    o, c = oracle.materialize(text, D.csv4(), 6)
    ot, ct = oracle.materialize(text, D.csv4(), 6, terminator=0x1E)
    assert bytes(ct) == b"".join(bytes(c[o[r]:o[r + 1]]) + b"\x1e" for r in range(len(o) - 1))
    assert list(ot) == [x + i for i, x in enumerate(o)]


@pytest.mark.parametrize("seed", range(4))
def test_materialize_against_csv_module(seed):
    """Materialised values of every column equal Python's csv module's
    fields on random RFC-4180 text (empty for records without the column)."""
    import csv
    import io
    rng = random.Random(200 + seed)
    pieces = ["", "7", "abc", '"x,y"', '"a\nb"', '"say ""hi"""', '""', '""""', "-1.5", "z z"]
    recs = [",".join(rng.choice(pieces) for _ in range(rng.choice([1, 2, 3, 4, 4, 6])))
            for _ in range(rng.randrange(5, 80))]
    text = ("\n".join(recs) + ("\n" if seed % 2 else "")).encode()
    rows = list(csv.reader(io.StringIO(text.decode(), newline="")))
    for c in range(6):
        offs, chars = oracle.materialize(text, D.csv4(), c)
        assert len(offs) == len(rows) + 1
        for r, row in enumerate(rows):
            want = row[c] if c < len(row) else ""
            assert bytes(chars[offs[r]:offs[r + 1]]).decode() == want, (seed, c, r)


def test_materialize_log_escapes():
    """The log dialect: backslash escapes inside quotes keep the escaped
    character, brackets enclose a field with spaces; checked against a
    regular-expression decoder of the same format."""
    import re
    rng = random.Random(5)
    lines, want = [], []
    for _ in range(200):
        req = "".join(rng.choice(['a', ' ', '\\"', '\\\\', 'x', '/']) for _ in range(rng.randrange(0, 12)))
        lines.append(f'h{rng.randrange(9)} [d t] "{req}" 200')
        want.append(re.sub(r'\\(.)', r'\1', req))
    text = ("\n".join(lines) + "\n").encode()
    offs, chars = oracle.materialize(text, D.log6(), 2)
    assert [bytes(chars[offs[r]:offs[r + 1]]).decode() for r in range(len(lines))] == want
    offs, chars = oracle.materialize(text, D.log6(), 1)
    assert all(bytes(chars[offs[r]:offs[r + 1]]) == b"d t" for r in range(len(lines)))


def test_infer_types_hand_example():
    """Type inference (Sec. 4.3): the narrowest type every non-empty field of
    a column admits; empty fields do not constrain; a column of empty fields
    is a string column."""
    t = (b'1,1.5,2020-01-01,2020-01-01 10:00:00,abc,"42",,x\n'
         b'-3,7,2020-02-29,2020-01-01T00:00:00,12,"",,1\n')
    types, nonempty = oracle.infer_types(t, D.csv4(), 9)
    assert types == [D.INT64, D.FLOAT64, D.DATE_DAYS, D.TIMESTAMP_S, D.STRING, D.INT64, D.STRING, D.STRING,
                     D.STRING]
    assert list(nonempty) == [2, 2, 2, 2, 2, 1, 0, 2, 0]


def _py_admits(text):
    """The types a field admits, decided with Python's own parsers."""
    import datetime
    import re
    out = set()
    if re.fullmatch(r"[+-]?[0-9]+", text) and -2 ** 63 <= int(text) < 2 ** 63:
        out.add(D.INT64)
    if re.fullmatch(r"[+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+)([eE][+-]?[0-9]+)?", text):
        out.add(D.FLOAT64)
    if re.fullmatch(r"[0-9]{4}-[0-9]{2}-[0-9]{2}", text):
        try:
            datetime.date(int(text[:4]), int(text[5:7]), int(text[8:10]))
            out.add(D.DATE_DAYS)
        except ValueError:
            pass
    if re.fullmatch(r"[0-9]{4}-[0-9]{2}-[0-9]{2}[ T][0-9]{2}:[0-9]{2}:[0-9]{2}", text):
        try:
            datetime.datetime(int(text[:4]), int(text[5:7]), int(text[8:10]), int(text[11:13]), int(text[14:16]),
                              int(text[17:19]))
            out.add(D.TIMESTAMP_S)
        except ValueError:
            pass
    return out


@pytest.mark.parametrize("seed", range(5))
def test_infer_types_against_python(seed):
    rng = random.Random(300 + seed)
    kinds = {
        "int": lambda: str(rng.randrange(-10 ** 6, 10 ** 6)),
        "big": lambda: rng.choice(["9223372036854775807", "9223372036854775808", "-9223372036854775808"]),
        "float": lambda: f"{rng.uniform(-1e4, 1e4):.{rng.randrange(0, 4)}f}",
        "exp": lambda: f"{rng.uniform(1, 9):.2f}e{rng.randrange(-5, 5)}",
        "date": lambda: f"{rng.randrange(1900, 2100):04d}-{rng.randrange(1, 13):02d}-{rng.randrange(1, 32):02d}",
        "ts": lambda: f"2020-{rng.randrange(1, 13):02d}-{rng.randrange(1, 29):02d} "
                      f"{rng.randrange(0, 25):02d}:{rng.randrange(0, 60):02d}:{rng.randrange(0, 61):02d}",
        "word": lambda: rng.choice(["abc", "x1", "1x", "--", "1.2.3", "+", "."]),
        "empty": lambda: "",
    }
    ncols = 8
    colkinds = [[rng.choice(list(kinds)) for _ in range(rng.choice([1, 2]))] for _ in range(ncols)]
    rows = [[kinds[rng.choice(colkinds[c])]() for c in range(ncols)] for _ in range(rng.randrange(1, 40))]
    text = ("\n".join(",".join(r) for r in rows) + "\n").encode()
    types, nonempty = oracle.infer_types(text, D.csv4(), ncols)
    for c in range(ncols):
        vals = [r[c] for r in rows if r[c] != ""]
        admitted = {D.INT64, D.FLOAT64, D.DATE_DAYS, D.TIMESTAMP_S}
        for v in vals:
            admitted &= _py_admits(v)
        want = D.STRING if not vals else next((t for t in (D.INT64, D.FLOAT64, D.DATE_DAYS, D.TIMESTAMP_S)
                                               if t in admitted), D.STRING)
        assert types[c] == want and nonempty[c] == len(vals), (seed, c, colkinds[c], vals[:5])


@pytest.mark.parametrize("seed", range(4))
def test_skip_rows_against_splitlines(seed):
    """Skipping rows (Sec. 4.3): the same as dropping the listed lines of
    Python's line split (line feeds kept), quotes notwithstanding."""
    rng = random.Random(400 + seed)
    lines = [rng.choice(["a,b", '"x', 'y"', "", "1,2,3", '""']) for _ in range(rng.randrange(0, 50))]
    text = "\n".join(lines) + ("\n" if seed % 2 else "")
    rows = text.encode().split(b"\n")
    rows = [r + b"\n" for r in rows[:-1]] + ([rows[-1]] if rows[-1] else [])
    ranges, k = [], 0
    while k < len(rows) + 3:
        a = k + rng.randrange(0, 4)
        b = a + rng.randrange(1, 4)
        ranges.append((a, b))
        k = b + 1
    want = b"".join(r for i, r in enumerate(rows) if not any(a <= i < b for a, b in ranges))
    assert bytes(oracle.skip_rows(text.encode(), ranges)) == want
    assert bytes(oracle.skip_rows(text.encode(), [])) == text.encode()


# ---- conversions against Python's exact arithmetic -------------------------

INT_CASES = ["0", "-0", "+7", "123", "-123", "9223372036854775807", "-9223372036854775808",
             "9223372036854775808", "-9223372036854775809", "00000000000000000000042",
             "", "+", "-", "1 ", " 1", "1.0", "0x10", "12a", "99999999999999999999"]


@pytest.mark.parametrize("text", INT_CASES)
def test_int64_conversion(text):
    ok, iv, _ = oracle.convert(D.INT64, text.encode())
    try:
        want = int(text, 10) if text.strip() == text and text and text.lstrip("+-").isdigit() else None
    except ValueError:
        want = None
    if want is not None and not (-(1 << 63) <= want < (1 << 63)):
        want = None
    assert ok == (want is not None)
    if ok:
        assert iv == want


FLOAT_CASES = ["0", "-0.0", "1", "1.5", ".5", "5.", "-.25", "1e10", "1E-5", "+3.25e+2",
               "123456.789012", "0.1", "0.2", "0.3", "9007199254740993", "1e308", "1.8e308",
               "-1e400", "4.9406564584124654e-324", "2.4703282292062327e-324",
               "2.4703282292062328e-324", "1e-320", "2.2250738585072011e-308",
               "1.7976931348623157e308", "1.00000000000000011102230246251565404236316680908203125",
               "1.00000000000000011102230246251565404236316680908203124",
               "1.00000000000000011102230246251565404236316680908203126",
               "12345678901234567890123", "0.000000000000000000000000000000123456789",
               "", ".", "e5", "1e", "1e+", "--1", "inf", "nan", "0x1p3", " 1", "1,0"]


def _py_float(text):
    """Grammar-checked exact value of the decimal, rounded by Python."""
    import re
    if not re.fullmatch(r"[+-]?([0-9]+(\.[0-9]*)?|\.[0-9]+)([eE][+-]?[0-9]+)?", text):
        return None
    return float(text)


@pytest.mark.parametrize("text", FLOAT_CASES)
def test_float64_conversion(text):
    ok, _, dv = oracle.convert(D.FLOAT64, text.encode())
    want = _py_float(text)
    assert ok == (want is not None)
    if ok:
        assert np.float64(dv).tobytes() == np.float64(want).tobytes()


def test_float64_against_exact_rationals():
    """Random decimals: the oracle equals the binary64 nearest to the exact
    rational value (Python's Fraction -> float rounds correctly)."""
    rnd = random.Random(11)
    for _ in range(3000):
        digits = "".join(rnd.choice("0123456789") for _ in range(rnd.randint(1, 25)))
        point = rnd.randint(0, len(digits))
        exp = rnd.randint(-30, 30)
        text = digits[:point] + "." + digits[point:] + f"e{exp}"
        ok, _, dv = oracle.convert(D.FLOAT64, text.encode())
        assert ok
        frac = Fraction(int(digits), 10 ** (len(digits) - point)) * Fraction(10) ** exp
        assert dv == float(frac)


def _epoch(y, m, d, hh=0, mi=0, ss=0):
    return calendar.timegm((y, m, d, hh, mi, ss, 0, 0, 0))


TS_CASES = [("1970-01-01 00:00:00", _epoch(1970, 1, 1)), ("1970-01-01T00:00:01", 1),
            ("1969-12-31 23:59:59", -1), ("2000-02-29 12:00:00", _epoch(2000, 2, 29, 12)),
            ("1900-02-28 00:00:00", _epoch(1900, 2, 28)), ("2018-12-31 23:59:59", _epoch(2018, 12, 31, 23, 59, 59)),
            ("0001-01-01 00:00:00", _epoch(1, 1, 1)), ("9999-12-31 23:59:59", _epoch(9999, 12, 31, 23, 59, 59)),
            ("1900-02-29 00:00:00", None), ("2001-02-29 00:00:00", None), ("2018-13-01 00:00:00", None),
            ("2018-00-10 00:00:00", None), ("2018-01-32 00:00:00", None), ("2018-01-01 24:00:00", None),
            ("2018-01-01 00:60:00", None), ("2018-01-01 00:00:60", None), ("2018-01-01 00:00", None),
            ("2018/01/01 00:00:00", None), ("2018-01-01x00:00:00", None)]


@pytest.mark.parametrize("text,want", TS_CASES)
def test_timestamp_conversion(text, want):
    ok, iv, _ = oracle.convert(D.TIMESTAMP_S, text.encode())
    assert ok == (want is not None)
    if ok:
        assert iv == want


def test_date_conversion_all_days():
    """Every day from 1600 to 2400 against Python's calendar arithmetic."""
    import datetime
    d = datetime.date(1600, 1, 1)
    base = datetime.date(1970, 1, 1)
    while d.year < 2400:
        ok, iv, _ = oracle.convert(D.DATE_DAYS, d.isoformat().encode())
        assert ok and iv == (d - base).days
        d += datetime.timedelta(days=1)


# ---- generator round trip ----------------------------------------------------

def _check_truth(g, dfa, schema):
    r = oracle.parse(g.data, dfa, schema.types)
    t = g.truth
    R, C = g.nrecords, g.ncols
    assert r.status == oracle.STATUS_OK
    assert r.num_records == R and r.num_fields == R * C
    assert r.num_ragged_records == 0
    assert np.array_equal(r.record_offsets, np.arange(R + 1) * C)
    assert np.array_equal(r.field_offsets[:-1], t.fbeg.reshape(-1))
    assert np.array_equal(r.column_ids, np.tile(np.arange(C, dtype=np.int32), R))
    for c, ty in enumerate(schema.types):
        kind = t.kind[:, c]
        if ty == D.STRING:
            assert np.array_equal(r.values[c], t.vbeg[:, c])
            assert np.array_equal(r.str_end[c], t.vend[:, c])
            assert r.valid[c].all()
        elif ty == D.FLOAT64:
            want = np.array([float(Fraction(int(m), 10 ** int(k))) for m, k in zip(t.ival[:, c], t.aux[:, c])])
            assert np.array_equal(r.values[c], want)
        elif ty in (D.INT64, D.TIMESTAMP_S, D.DATE_DAYS):
            ok = kind == 1
            assert np.array_equal(r.valid[c].astype(bool), ok)
            assert np.array_equal(r.values[c][ok], t.ival[ok, c])
    return r


def test_generator_round_trip_c1():
    g = datagen.c1(with_truth=True)
    assert g.nrecords == 10000
    r = _check_truth(g, D.csv4(), D.SCHEMA_C1)
    assert r.num_conversion_errors == 0
    # same outputs under Table 1's DFA (the input is valid RFC-4180)
    r6 = oracle.parse(g.data, D.paper6(), D.SCHEMA_C1.types)
    assert r6.status == oracle.STATUS_OK and np.array_equal(r6.field_offsets, r.field_offsets)


def test_generator_round_trip_c2_c3_sample():
    _check_truth(datagen.c2(nbytes=4 << 20, with_truth=True), D.csv4(), D.SCHEMA_C2)
    _check_truth(datagen.c3(nbytes=8 << 20, with_truth=True), D.csv4(), D.SCHEMA_C3)


def test_generator_round_trip_log():
    g = datagen.log(5, 2 << 20, with_truth=True)
    r = _check_truth(g, D.log6(), D.SCHEMA_LOG12)
    # "-" in the bytes column is a conversion failure (null), counted
    assert r.num_conversion_errors == int((g.truth.kind[:, 6] == 0).sum())


@pytest.mark.parametrize("name,delim,qstyle", [("csv4", b",", 1), ("csv4", b"\t", 1),
                                               ("paper6", b",", 1), ("s5", b"|", 1),
                                               ("s3", b",", 3), ("s7", b",", 2)])
def test_generator_round_trip_mixed(name, delim, qstyle):
    dfa = D.ALL_DFAS[name](delim) if name != "paper6" else D.paper6()
    g = datagen.mixed(3, 1 << 20, delim=delim, qstyle=qstyle, with_truth=True)
    _check_truth(g, dfa, D.SCHEMA_C1)


def test_generator_round_trip_s8_log():
    g = datagen.log(9, 1 << 20, with_truth=True)
    _check_truth(g, D.s8(), D.SCHEMA_LOG12)


# ---- start states other than 0 ---------------------------------------------------

RELABEL = [("csv4", [2, 0, 3, 1]), ("paper6", [3, 5, 0, 1, 4, 2]), ("log6", [5, 3, 0, 1, 2, 4]),
           ("s8", [6, 0, 1, 2, 3, 4, 5, 7]), ("s5", [1, 2, 3, 0, 4]), ("s3", [2, 1, 0])]


@pytest.mark.parametrize("name,perm", RELABEL, ids=[r[0] for r in RELABEL])
def test_relabelled_dfa_same_outputs(name, perm):
    """Renumbering the states (start state no longer 0) changes no tag, so
    every output except the final state's number is unchanged; a run that
    took state 0 instead of the DFA's start state would differ here (a quoted
    field at byte 0 would keep its opening quote)."""
    base = D.ALL_DFAS[name]()
    rel = D.relabel(base, perm)
    assert rel.start_state != 0
    alphabet = b"".join(base.group_symbols) + b"a1.-"
    rnd = random.Random(7)
    types = [D.STRING, D.INT64, D.FLOAT64, D.STRING]
    quote = b'"' if b'"' in alphabet else (b"\\" if b"\\" in alphabet else b"")
    texts = [b'"12",x\n', quote + b"7,a\nb" + quote + b",3\n"]
    texts += [bytes(rnd.choice(alphabet) for _ in range(rnd.randint(0, 300))) for _ in range(200)]
    for t in texts:
        a = oracle.parse(t, base, types)
        b = oracle.parse(t, rel, types)
        assert b.final_state == perm[a.final_state]
        for k in ("status", "num_records", "num_fields", "first_invalid_offset", "num_conversion_errors",
                  "num_ragged_records", "min_record_fields", "max_record_fields"):
            assert getattr(a, k) == getattr(b, k), (t, k)
        for k in ("record_offsets", "field_offsets", "column_ids"):
            np.testing.assert_array_equal(getattr(a, k), getattr(b, k))
        for c in range(len(types)):
            np.testing.assert_array_equal(a.values[c].view(np.int64), b.values[c].view(np.int64))
            np.testing.assert_array_equal(a.valid[c], b.valid[c])


def test_quoted_first_field_under_relabelled_csv4():
    """Hand case: under csv4 with FB renumbered to 2, "12" at byte 0 is the
    integer 12 (both quotes are control symbols read from the start state)."""
    rel = D.relabel(D.csv4(), [2, 0, 3, 1])
    r = oracle.parse(b'"12",x\n', rel, [D.INT64, D.STRING])
    assert r.status == oracle.STATUS_OK and r.values[0].tolist() == [12] and r.valid[0].tolist() == [1]
    assert (r.values[1].tolist(), r.str_end[1].tolist()) == ([5], [6])


def test_start_in_invalid_state_rejected():
    d = D.s5()
    d.invalid_state = d.start_state
    with pytest.raises(ValueError):
        oracle.parse(b"1,2\n", d, [D.INT64])


# ---- UTF-16 input (Sec. 4.2, multi-byte symbols) ---------------------------------

def _same_doubled(r8, r16, types):
    """The UTF-16 parse of ASCII text equals the byte parse with every
    position doubled."""
    assert (r16.status, r16.num_records, r16.num_fields) == (r8.status, r8.num_records, r8.num_fields)
    assert r16.first_invalid_offset == (2 * r8.first_invalid_offset if r8.first_invalid_offset >= 0 else -1)
    assert (r16.final_state, r16.num_conversion_errors, r16.num_ragged_records) == \
        (r8.final_state, r8.num_conversion_errors, r8.num_ragged_records)
    assert list(r16.record_offsets) == list(r8.record_offsets)
    assert list(r16.field_offsets) == [2 * x for x in r8.field_offsets]
    assert list(r16.column_ids) == list(r8.column_ids)
    for c, ty in enumerate(types):
        if ty == D.SKIP:
            continue
        if ty == D.STRING:
            assert list(r16.values[c]) == [2 * x for x in r8.values[c]]
            assert list(r16.str_end[c]) == [2 * x for x in r8.str_end[c]]
        else:
            assert r16.values[c].tobytes() == r8.values[c].tobytes()
        assert list(r16.valid[c]) == list(r8.valid[c])


@pytest.mark.parametrize("name", ["csv4", "paper6", "log6"])
def test_utf16_ascii_text_is_the_byte_parse_doubled(name):
    dfa = D.ALL_DFAS[name]()
    rnd = random.Random(31)
    alphabet = b"".join(dfa.group_symbols) + b"a1.-e9"
    types = [D.STRING, D.INT64, D.FLOAT64, D.STRING, D.SKIP, D.INT64]
    for n in (0, 1, 2, 57, 3000):
        text = bytes(rnd.choice(alphabet) for _ in range(n))
        r8 = oracle.parse(text, dfa, types)
        r16 = oracle.parse(text.decode("latin-1").encode("utf-16-le"), dfa, types, utf16=True)
        _same_doubled(r8, r16, types)
    g = datagen.c1()
    data = bytes(g.data[:200000])
    _same_doubled(oracle.parse(data, D.csv4(), D.SCHEMA_C1.types),
                  oracle.parse(data.decode("latin-1").encode("utf-16-le"), D.csv4(), D.SCHEMA_C1.types, utf16=True),
                  D.SCHEMA_C1.types)


@pytest.mark.parametrize("seed", range(4))
def test_utf16_against_csv_module(seed):
    """Random RFC-4180 text with non-ASCII characters (Latin, CJK, characters
    outside the BMP as surrogate pairs, a fullwidth comma that is data) in
    UTF-16LE: every string field, read from its byte span and with its
    doubled quotes undone, equals Python's csv module's field."""
    import csv
    import io
    rng = random.Random(400 + seed)
    pieces = ["", "7", "é", "漢字", "😀x", '"x,y"', '"a\nb"', '"say ""hi"""', '""', "a，b", "-1.5"]
    recs = [",".join(rng.choice(pieces) for _ in range(rng.choice([1, 2, 3, 4, 4, 6])))
            for _ in range(rng.randrange(5, 80))]
    text = "\n".join(recs) + ("\n" if seed % 2 else "")
    rows = list(csv.reader(io.StringIO(text, newline="")))
    b16 = text.encode("utf-16-le")
    r = oracle.parse(b16, D.csv4(), [D.STRING] * 6, utf16=True)
    assert r.status == oracle.STATUS_OK and r.num_records == len(rows)
    for k, row in enumerate(rows):
        for c in range(6):
            want = row[c] if c < len(row) else ""
            got = b16[r.values[c][k]:r.str_end[c][k]].decode("utf-16-le")
            quoted = r.str_end[c][k] < len(b16) and b16[r.str_end[c][k]:r.str_end[c][k] + 2] == '"'.encode("utf-16-le")
            assert (got.replace('""', '"') if quoted else got) == want, (seed, k, c)


def test_utf16_numbers_and_non_ascii_digits():
    """ASCII numerals convert as in byte text; digits outside ASCII (here
    Arabic-Indic) are not digits of the grammar: a conversion error."""
    text = "12,2.5,2020-01-02\n٣,3.0,2020-01-0٣\n"
    r = oracle.parse(text.encode("utf-16-le"), D.csv4(), [D.INT64, D.FLOAT64, D.DATE_DAYS], utf16=True)
    assert r.num_records == 2 and r.num_conversion_errors == 2
    assert list(r.values[0]) == [12, 0] and list(r.valid[0]) == [1, 0]
    assert list(r.values[1]) == [2.5, 3.0]
    assert list(r.valid[2]) == [1, 0] and r.values[2][0] == 18263


@pytest.mark.parametrize("seed", range(3))
def test_utf16_materialize_against_csv_module(seed):
    """Materialised UTF-16 values (control symbols removed, code units kept)
    equal Python's csv module's fields on text with non-ASCII characters;
    with a terminator, every value is followed by that code unit."""
    import csv
    import io
    rng = random.Random(600 + seed)
    pieces = ["", "7", "é", "漢字", "😀x", '"x,y"', '"a\nb"', '"say ""hi"""', '""', '""""', "a，b"]
    recs = [",".join(rng.choice(pieces) for _ in range(rng.choice([1, 2, 3, 4, 4, 6])))
            for _ in range(rng.randrange(5, 80))]
    text = "\n".join(recs) + ("\n" if seed % 2 else "")
    rows = list(csv.reader(io.StringIO(text, newline="")))
    b16 = text.encode("utf-16-le")
    for c in range(6):
        offs, chars = oracle.materialize(b16, D.csv4(), c, utf16=True)
        assert len(offs) == len(rows) + 1
        for r, row in enumerate(rows):
            want = row[c] if c < len(row) else ""
            assert chars[offs[r]:offs[r + 1]].tobytes().decode("utf-16-le") == want, (seed, c, r)
        toffs, tchars = oracle.materialize(b16, D.csv4(), c, terminator=0x2028, utf16=True)
        assert list(toffs) == [o + k for k, o in enumerate(offs)]
        assert all(tchars[toffs[r + 1] - 1] == 0x2028 for r in range(len(rows)))
