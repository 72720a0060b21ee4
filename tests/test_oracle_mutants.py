"""Planted mistakes in the oracle must be caught by its pins.

Each case copies the oracle source, applies one plausible slip (a dropped
term, a wrong comparison, a wrong index, a missed bookkeeping step), builds it
on the CPU and runs the pin suite against that build.  The suite has to fail
for every mutant."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "hda_oracle.cpp")

# (name, text, replacement, occurrence)
MUTANTS = [
    ("ff_strict_fit", "if (it->second >= s) { pick = it; break; }",
     "if (it->second > s) { pick = it; break; }", 0),
    ("nf_strict_fit", "if (it->second >= s) { pick = it; break; }",
     "if (it->second > s) { pick = it; break; }", 1),
    ("bf_tie_highest_address", "it->second < pick->second", "it->second <= pick->second", 0),
    ("nf_start_rule", "start->first + start->second <= rover",
     "start->first + start->second < rover", 0),
    ("nf_rover_at_start", "rover = a + s;", "rover = a;", 0),
    ("split_size_dropped", "fl[a + s] = bsize - s;", "fl[a + s] = bsize;", 0),
    ("three_way_merge_drops_right", "pred->second += s + succ->second;",
     "pred->second += s;", 0),
    ("right_merge_drops_size", "fl[x] = s + sz;", "fl[x] = s;", 0),
    ("right_adjacency_index", "succ->first == x + s", "succ->first == x", 0),
    ("sf_request_class_floor", "int k = ceil_log2(uint64_t(s));",
     "int k = floor_log2(uint64_t(s));", 0),
    ("sf_highest_class", "return m == 0 ? -1 : __builtin_ctzll(m);",
     "return m == 0 ? -1 : 63 - __builtin_clzll(m);", 0),
    ("sf_bit_not_cleared", "            bitmap &= ~(uint64_t(1) << c);", "", 0),
    ("sf_push_class_ceil", ": floor_log2(uint64_t(size));", ": ceil_log2(uint64_t(size));", 0),
    ("sf_unlink_drops_tail", "else head[c] = r.next_free;", "else head[c] = NIL;", 0),
    # (Writing l instead of l's own left link into the merged record is NOT a
    # mistake the state can show: that link is rewritten before it is ever read
    # while the left neighbour is free, so it is not listed.)
    ("sf_merge_right_link_not_fixed", "if (end < A) { ht.at(end).prev_adj = start; ++touched; }",
     "", 0),
    ("sf_split_prev_adj_not_fixed", "if (old_end < A) { ht.at(old_end).prev_adj = b; ++touched; }",
     "", 0),
    ("driver_modulo_index", "uint64_t idx = (r * uint64_t(h.live.size())) >> 32;",
     "uint64_t idx = r % uint64_t(h.live.size());", 0),
    ("driver_no_swap", "*lv = live.back();\n        live.pop_back();", "live.erase(lv);", 0),
    ("size_not_rounded", "int64_t s = (req + g - 1) / g * g;", "int64_t s = req;", 0),
    # partial deallocation (Alg. 2)
    ("partial_keeps_extra_granule", "u->second = x - b;", "u->second = x - b + g;", 0),
    ("partial_frees_whole_size", "dealloc_seq(x, b + s - x);", "dealloc_seq(x, s);", 0),
    ("partial_cut_scale", "h.g)) >> 31) * h.g;", "h.g)) >> 32) * h.g;", 0),
    ("partial_result_is_block_start", "res[i] = x + keep;", "res[i] = x;", 0),
    ("partial_unaligned_accepted", "if (segregated() || x % g != 0) return E_BADFREE;",
     "if (segregated()) return E_BADFREE;", 0),
    ("partial_on_seg_fit", "if (segregated() || x % g != 0) return E_BADFREE;",
     "if (x % g != 0) return E_BADFREE;", 0),
    ("partial_cut_on_wrong_algos", "if (!h.segregated()) keep", "if (h.segregated()) keep", 0),
    # TLSF (checked by its own pin file)
    ("tlsf_no_round_up", "uint64_t r = uint64_t(s) + (f0 >= SLI ? (uint64_t(1) << (f0 - SLI)) - 1 : 0);",
     "uint64_t r = uint64_t(s);", 0, "tlsf"),
    ("tlsf_skips_a_level", "(bitmap & (~uint64_t(0) << (fl + 1)))", "(bitmap & (~uint64_t(0) << (fl + 2)))",
     0, "tlsf"),
    ("tlsf_sl_bit_not_cleared", "sl_bitmap[c / NSL] &= ~(uint32_t(1) << (c % NSL));", "", 0, "tlsf"),
    ("tlsf_fl_bit_not_cleared",
     "if (sl_bitmap[c / NSL] == 0) bitmap &= ~(uint64_t(1) << (c / NSL));", "", 0, "tlsf"),
    ("tlsf_sub_class_from_low_bits", "(b >> (fl - SLI)) - NSL", "(b & (NSL - 1))", 0, "tlsf"),
    # bitmask allocator (checked by its own pin file)
    ("bm_from_block_start", "int64_t from = std::max(it->first, rover);",
     "int64_t from = it->first;", 0, "bitmap"),
    ("bm_no_wrap", "if (it->second >= s) { pick = it; p = it->first; }", "", 0, "bitmap"),
    ("bm_left_part_dropped", "if (p > a) fl[a] = p - a;", "", 0, "bitmap"),
    ("bm_rover_at_start", "rover = p + s;\n        return p;", "rover = p;\n        return p;", 0,
     "bitmap"),
    # instrumentation counters (checked by their own pin file)
    ("ff_examined_not_counted", "                ++examined;\n                if (it->second >= s) { pick = it; break; }",
     "                if (it->second >= s) { pick = it; break; }", 0, "counters"),
    ("bf_examined_past_exact", "if (it->second == s) break;", "", 0, "counters"),
    ("sf_push_old_head_not_counted",
     "if (head[c] != NIL) { ht.at(head[c]).prev_free = a; ++touched; }",
     "if (head[c] != NIL) { ht.at(head[c]).prev_free = a; }", 0, "counters"),
]

PINS = {"seq": [os.path.join(ROOT, "tests", f)
                for f in ("test_oracle_pins.py", "test_oracle_partial.py")],
        "tlsf": [os.path.join(ROOT, "tests", "test_oracle_tlsf.py")],
        "bitmap": [os.path.join(ROOT, "tests", "test_oracle_bitmap.py")],
        "counters": [os.path.join(ROOT, "tests", "test_oracle_counters.py")]}


def _replace_nth(text, old, new, n):
    idx = -1
    for _ in range(n + 1):
        idx = text.find(old, idx + 1)
        assert idx >= 0, f"mutation anchor not found: {old!r}"
    return text[:idx] + new + text[idx + len(old):]


def _run(m, tmp):
    name, old, new, n = m[:4]
    pins = PINS[m[4] if len(m) > 4 else "seq"]
    src = open(SRC).read()
    mutated = _replace_nth(src, old, new, n)
    assert mutated != src
    cpp = os.path.join(tmp, f"{name}.cpp")
    so = os.path.join(tmp, f"{name}.so")
    with open(cpp, "w") as f:
        f.write(mutated)
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-pthread",
                           cpp, "-o", so])
    env = dict(os.environ, HDA_ORACLE_LIB=so)
    p = subprocess.run([sys.executable, "-m", "pytest", *pins, "-x", "-q",
                        "-p", "no:cacheprovider", "--timeout", "120",
                        "-k", "not depth6"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    return name, p.returncode


def test_every_anchor_is_unique_enough():
    src = open(SRC).read()
    for name, old, _, n, *_ in MUTANTS:
        assert src.count(old) > n, name


def test_pins_catch_planted_mistakes():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max(1, min(8, os.cpu_count() or 1))) as ex:
            results = list(ex.map(lambda m: _run(m, tmp), MUTANTS))
    survivors = [name for name, rc in results if rc == 0]
    assert not survivors, f"pins did not catch: {survivors}"
