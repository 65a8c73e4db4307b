"""The 32-bit partial counters of the device path stay below 2^32 by construction, so the int64
outputs are exact (Algorithm 1's counters are integers that can pass 2^32: the R-MAT scale-24
stream's exact tau is 10,286,644,549).  The bounds, read from the kernel sources:

* a wavefront's LDS histogram of global counts gains at most one per drained hit for any
  processor (a triangle is a semi-triangle of at most one processor per group); it is flushed
  once the hits since its last flush reach kHistFlushHits, and one drain handles at most kQueue
  hits, so a counter never exceeds kHistFlushHits - 1 + kQueue;
* the incremental count's per-workgroup histogram gains at most one per item; it is flushed
  before the items since the last flush would pass 2^31, with at most kRun items per run;
* a staged entry's local counter gains at most one per list walked against it (fewer than
  2 * 2^31 lists: streams hold fewer than 2^31 edges) or per entry of its table chunk (<= 4096),
  and a unit's own count is summed in 64 bits: for a light unit in one 32-bit pass when the
  chunk's W entries times the unit's lists is below 2^32 (each W entry gains at most one per
  list), else in pieces of 26, 26 and 12 bits whose 64-lane sums stay below 2^32.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1811_09136_amd", "csrc")


def _src(name):
    with open(os.path.join(CSRC, name)) as f:
        return f.read()


def _const(src, name):
    m = re.search(r"constexpr uint32_t " + name + r" = ([^;]+);", src)
    assert m, name
    expr = m.group(1).replace("u", "")
    return expr


def test_wave_histogram_bound():
    s = _src("count.hip")
    k_walk = int(_const(s, "kWalk").split()[0])
    assert _const(s, "kQueue").startswith("64 * (kWalk + 1)")
    k_queue = 64 * (k_walk + 1)
    flush = eval(_const(s, "kHistFlushHits"))  # "1 << 31"
    assert flush - 1 + k_queue < 2**32
    # every drain goes through the wrapper that counts hits and flushes
    assert "if (h >= kHistFlushHits)" in s
    assert s.count("drain_hits<ETA>(") == 2


def test_incremental_histogram_bound():
    s = _src("stream.hip")
    k_run = int(_const(s, "kRun").split()[0])
    assert "since + (i1 - i0) > (1ull << 31)" in s
    assert 2**31 + k_run < 2**32


def test_unit_total_is_64_bit():
    s = _src("count.hip")
    assert "const uint64_t tot = team_sum64<BLOCK>(part, T.red, narrow);" in s
    assert "const bool narrow = !BLOCK && (uint64_t)wn * nbtot < (1ull << 32);" in s
    assert "uint32_t team_sum(" not in s
    # the wide path's pieces: 26, 26 and 12 bits of a 64-bit part, each summed over 64 lanes in 32 bits
    assert "wave_sum((uint32_t)v & 0x3ffffffu)" in s
    assert "wave_sum((uint32_t)(v >> 26) & 0x3ffffffu) << 26" in s
    assert "wave_sum((uint32_t)(v >> 52)) << 52" in s
    assert 64 * (2**26 - 1) < 2**32 and 64 * (2**12 - 1) < 2**32
    assert 26 + 26 + 12 == 64
