"""Planted mistakes in the oracle are caught by its pins.

Each mutant is the C oracle with one plausible mistake: a flipped
comparison, an off-by-one, a dropped or transposed term, a missing mask, a
wrong marker field, a missing format check.  It is built with gcc into a
temporary library, and the pins of test_oracle_pins are run against it in a
subprocess (oracle_battery.py): at least one pin must fail, crash or time
out.  The unmodified source, built the same way, must pass them all, also
when built with UBSan (undefined behaviour aborts).  CPU only; nothing here
touches the library under test.
"""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "tq_oracle.c")
RUNNER = os.path.join(HERE, "oracle_battery.py")

# (name, text, replacement, which occurrence of the text)
MUTANTS = [
    ("threshold compares with >", "if (count[b] >= theta) o |= (uint64_t)1 << b;\n    out[w]",
     "if (count[b] > theta) o |= (uint64_t)1 << b;\n    out[w]", 0),
    ("threshold skips the last input", "for (uint32_t j = 0; j < n; ++j) {\n      uint64_t x = bitmaps[j][w] & mask;",
     "for (uint32_t j = 0; j + 1 < n; ++j) {\n      uint64_t x = bitmaps[j][w] & mask;", 0),
    ("threshold counts a neighbouring bit", "count[b] += (uint32_t)((x >> b) & 1);",
     "count[b] += (uint32_t)((x >> (b ^ 1)) & 1);", 2),
    ("threshold output keeps bits past r", "if (count[b] >= theta) o |= (uint64_t)1 << b;\n    out[w] = o & mask;",
     "if (count[b] >= theta) o |= (uint64_t)1 << b;\n    out[w] = o;", 0),
    ("symmetric looks up f(c - 1)", "if (f[count[b]]) o |= (uint64_t)1 << b;\n    out[w]",
     "if (f[count[b] ? count[b] - 1 : 0]) o |= (uint64_t)1 << b;\n    out[w]", 0),
    ("symmetric output keeps bits past r", "if (f[count[b]]) o |= (uint64_t)1 << b;\n    out[w] = o & mask;",
     "if (f[count[b]]) o |= (uint64_t)1 << b;\n    out[w] = o;", 0),
    ("sampled threshold compares with >", "if (count[b] >= theta) o |= (uint64_t)1 << b;\n    out[c]",
     "if (count[b] > theta) o |= (uint64_t)1 << b;\n    out[c]", 0),
    ("sampled symmetric looks up f(c + 1)", "if (f[count[b]]) o |= (uint64_t)1 << b;\n    out[c]",
     "if (f[count[b] < n ? count[b] + 1 : n]) o |= (uint64_t)1 << b;\n    out[c]", 0),
    ("tail mask one bit short", "return ((uint64_t)1 << (r_bits - first)) - 1;",
     "return ((uint64_t)1 << (r_bits - first - 1)) - 1;", 0),
    ("full words taken for partial", "if (r_bits - first >= 64) return ~(uint64_t)0;",
     "if (r_bits - first >= 63) return ~(uint64_t)0;", 0),
    ("weighted adds 1 per input", "if ((x >> b) & 1) sum[b] += weights[j];",
     "if ((x >> b) & 1) sum[b] += 1;", 0),
    ("weighted compares with >", "if (sum[b] >= theta)", "if (sum[b] > theta)", 0),
    ("count stops one position early", "for (uint64_t p = 0; p < r_bits; ++p) c +=",
     "for (uint64_t p = 0; p + 1 < r_bits; ++p) c +=", 0),
    ("decode writes zero fills only", "out[w++] = fill ? ~(uint64_t)0 : 0;", "out[w++] = 0;", 0),
    ("run field not masked", "return (m >> 1) & 0xFFFFFFFFull;", "return m >> 1;", 0),
    ("literal count field off by a bit", "return m >> 33;", "return m >> 32;", 0),
    ("decode does not check the stream end", "    if (lits > len - pos) return ORACLE_EFORMAT;\n", "", 0),
    ("decode accepts short coverage", "if (w != nwords) return ORACLE_EFORMAT;", "", 0),
    ("encode keeps bits past r in literals",
     "out[len] = dense[lit_start + k] & valid_mask(lit_start + k, r_bits);",
     "out[len] = dense[lit_start + k];", 0),
    ("encode writes the fill bit inverted", "return (fill & 1) | (run << 1) | (lits << 33);",
     "return ((fill ^ 1) & 1) | (run << 1) | (lits << 33);", 0),
    ("run count keeps the first bit", "if (b != prev) { ++runs; prev = b; }", "if (b != prev) { ++runs; }", 0),
]


UBSAN = ["-g", "-fsanitize=undefined", "-fno-sanitize-recover=all"]


def _build(src_text, path, extra=()):
    c = path + ".c"
    with open(c, "w") as fh:
        fh.write(src_text)
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC", *extra, "-o", path, c], check=True)


def _battery(lib):
    env = dict(os.environ, OMP_NUM_THREADS="2")
    try:
        r = subprocess.run([sys.executable, RUNNER, lib], capture_output=True, text=True, timeout=120, env=env)
    except subprocess.TimeoutExpired:
        return 124, "timed out"
    return r.returncode, (r.stdout + r.stderr).strip()[-300:]


def _mutate(text, old, new, which):
    start = -1
    for _ in range(which + 1):
        start = text.find(old, start + 1)
        assert start >= 0, "mutation site not found: %r (occurrence %d)" % (old[:50], which)
    return text[:start] + new + text[start + len(old):]


@pytest.fixture(scope="module")
def source():
    with open(SRC) as fh:
        return fh.read()


def test_unmodified_oracle_passes(source, tmp_path):
    lib = str(tmp_path / "liboracle_ref.so")
    _build(source, lib)
    rc, out = _battery(lib)
    assert rc == 0, out


@pytest.mark.parametrize("name,old,new,which", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(source, tmp_path, name, old, new, which):
    mutated = _mutate(source, old, new, which)
    assert mutated != source
    lib = str(tmp_path / "liboracle_mutant.so")
    _build(mutated, lib)
    rc, out = _battery(lib)
    assert rc != 0, "no pin catches the planted mistake '%s'" % name


def test_oracle_has_no_undefined_behaviour(source, tmp_path):
    """The pins pass with the oracle built under UBSan (undefined behaviour
    aborts the run); the same build of a copy whose tail mask shifts by 64
    aborts, so the sanitizer is live."""
    lib = str(tmp_path / "liboracle_ubsan.so")
    _build(source, lib, UBSAN)
    rc, out = _battery(lib)
    assert rc == 0, out
    bad = _mutate(source, "if (r_bits - first >= 64) return ~(uint64_t)0;",
                  "if (r_bits - first > 64) return ~(uint64_t)0;", 0)
    lib = str(tmp_path / "liboracle_ubsan_bad.so")
    _build(bad, lib, UBSAN)
    rc, out = _battery(lib)
    assert rc != 0 and "runtime error" in out, out
