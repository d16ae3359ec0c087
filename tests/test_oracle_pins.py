"""Pins of the CPU oracle (CPU only) and a mutation test that plants plausible
mistakes in copies of the oracle source and checks that the pins catch each."""
from __future__ import annotations

import os
import re
import subprocess

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from tests import oracle_pins as P

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def impl():
    oracle.build()
    return P.OracleLib(oracle.lib_path())


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(impl, pin):
    pin(impl)


# ------------------------------------------------------------ invariants

units = st.one_of(
    st.sampled_from([0x41, 0x7F, 0xD7FF, 0xE000, 0xFFFD, 0xFFFF, 0x0000]),
    st.integers(0xD800, 0xDBFF),
    st.integers(0xDC00, 0xDFFF),
    st.integers(0, 0xFFFF),
)
strings = st.lists(units, min_size=0, max_size=64).map(lambda xs: np.array(xs, dtype=np.uint16))


@settings(max_examples=400, deadline=None)
@given(strings)
def test_invariants(impl, s):
    t, cnt = impl.to_count(s)
    # length is preserved and the output is well-formed
    assert t.size == s.size
    assert impl.is_(t) and P.codec_strict_ok(t)
    # only surrogate units change, and they become U+FFFD
    changed = t != s
    assert np.all((s[changed] >= 0xD800) & (s[changed] <= 0xDFFF))
    assert np.all(t[changed] == P.REPL)
    assert cnt == int(changed.sum())
    # idempotence and fixed points
    assert np.array_equal(impl.to(t), t)
    assert impl.is_(s) == (cnt == 0) == np.array_equal(t, s)
    # decode with the code-point formula and re-encode
    assert np.array_equal(P.encode_codepoints(P.decode_codepoints(t)), t)
    # in place == copy
    assert np.array_equal(impl.to_inplace(s), t)


@settings(max_examples=200, deadline=None)
@given(strings, st.integers(0, 64), st.integers(0, 64))
def test_slicing_and_locality(impl, s, a, b):
    a, b = sorted((min(a, s.size), min(b, s.size)))
    whole = impl.to(s)
    part = impl.to(s[a:b])
    if b - a >= 3:
        # only the two end units of a slice can differ from the whole
        assert np.array_equal(part[1:-1], whole[a + 1:b - 1])
    # a unit's output depends on its neighbours only: changing a unit two
    # places away never changes it
    if s.size >= 5:
        i = s.size // 2
        s2 = s.copy()
        s2[i + 2] ^= 0x0400
        s2[i - 2] ^= 0x0400
        assert impl.to(s2)[i] == whole[i]


def test_well_formed_inputs_are_fixed_points(impl):
    rng = np.random.default_rng(1)
    cps = rng.integers(0, 0x110000, size=5000)
    cps = cps[(cps < 0xD800) | (cps > 0xDFFF)]
    s = P.encode_codepoints(cps.tolist())
    assert impl.is_(s)
    assert np.array_equal(impl.to(s), s)
    assert P.decode_codepoints(impl.to(s)) == cps.tolist()


def test_edges_and_short(impl):
    assert impl.to(np.zeros(0, np.uint16)).size == 0 and impl.is_(np.zeros(0, np.uint16))
    for u in range(0xD800, 0xE000, 0x7F):
        assert impl.to([u])[0] == P.REPL
    assert list(impl.to([0xDC00, 0x41, 0xD800])) == [P.REPL, 0x41, P.REPL]
    assert list(impl.to([0xFFFD])) == [0xFFFD] and impl.is_([0xFFFD])


# ------------------------------------------------------------ mutation test

SRC = os.path.join(ROOT, "oracle", "utf16_oracle.c")

# (description, regex, replacement): each is a mistake a careful reader could
# make when writing the oracle from the paper.
MUTANTS = [
    ("high range one short", r"u <= 0xDBFFu", "u <= 0xDBFEu"),
    ("low range starts late", r"u >= 0xDC00u", "u >= 0xDC01u"),
    ("wrong replacement value", r"0xFFFDu", "0xFFFEu"),
    ("pair not stepped over", r"i \+= 2; /\* a valid pair", "i += 1; /* a valid pair"),
    ("lone lows kept", r"\} else if \(is_high\(u\) \|\| is_low\(u\)\) \{", "} else if (is_high(u)) {"),
    ("lone highs kept", r"\} else if \(is_high\(u\) \|\| is_low\(u\)\) \{", "} else if (is_low(u)) {"),
    ("pair at the end dropped", r"if \(is_high\(u\) && i \+ 1 < n && is_low\(s\[i \+ 1\]\)\) \{",
     "if (is_high(u) && i + 2 < n && is_low(s[i + 1])) {"),
    ("order of pair reversed", r"if \(is_high\(u\) && i \+ 1 < n && is_low\(s\[i \+ 1\]\)\) \{",
     "if (is_low(u) && i + 1 < n && is_high(s[i + 1])) {"),
    ("is: lone low accepted", r"else if \(is_high\(u\) \|\| is_low\(u\)\)\n            return 0;",
     "else if (is_high(u))\n            return 0;"),
    ("batch pairs across strings", r"replaced \+= wf_to_seq\(buf \+ a, t \+ a, len\);",
     "replaced += wf_to_seq(buf + a, t + a, len); if (k + 1 < num_strings && len > 0 && "
     "off[k+1] < off[num_strings] && (buf[a+len-1] & 0xFC00u) == 0xD800u && "
     "(buf[a+len] & 0xFC00u) == 0xDC00u) t[a+len-1] = buf[a+len-1];"),
    ("chunk context reads wrong side", r"is_high\(s\[lo - 1\]\)", "is_low(s[lo - 1])"),
    ("first-bad off by one", r"            return i;\n", "            return i + 1;\n"),
    ("count misses lone lows", r"if \(is_high\(u\) \|\| is_low\(u\)\)\n                    c\+\+;",
     "if (is_high(u))\n                    c++;"),
]


def _build_mutant(tmp_path, idx, pattern, repl):
    text = open(SRC).read()
    new, k = re.subn(pattern, repl, text, count=1)
    assert k == 1, f"mutation pattern not found: {pattern}"
    src = tmp_path / f"mut{idx}.c"
    src.write_text(new)
    so = tmp_path / f"mut{idx}.so"
    subprocess.run(["gcc", "-std=c11", "-O1", "-fPIC", "-shared", "-pthread", "-w", "-o", str(so), str(src)],
                   check=True)
    return str(so)


@pytest.mark.parametrize("idx", range(len(MUTANTS)), ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(tmp_path, idx):
    _, pattern, repl = MUTANTS[idx]
    impl = P.OracleLib(_build_mutant(tmp_path, idx, pattern, repl))
    caught = []
    for pin in P.ALL_PINS:
        try:
            pin(impl)
        except AssertionError:
            caught.append(pin.__name__)
    assert caught, f"no pin catches mutant {MUTANTS[idx][0]!r}"
