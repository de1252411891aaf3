"""The Relax filter's 16-bit key-bound codes (csrc/hint_code.h), compiled
for the host: every code's value is at least the key it was made from, the
code is the smallest such, codes and values grow together, and keys beyond
the range get no bound. CPU only (a host build of the kernel's own header)."""

import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2105_06145_amd", "csrc")

PROBE = r"""
#include <cstdio>
#include <cstdint>
#include "hint_code.h"
using namespace sssp_impl;
int main() {
  // Every code's value, in code order.
  for (uint32_t c = 0; c < 0xFFFFu; ++c) std::printf("v %u %llu\n", c, (unsigned long long)hint_value(c));
  unsigned long long d;
  while (std::scanf("%llu", &d) == 1) std::printf("h %llu %u\n", d, (unsigned)as_hint(d));
  return 0;
}
"""


@pytest.fixture(scope="module")
def probe(tmp_path_factory):
    d = tmp_path_factory.mktemp("hint")
    src = d / "probe.hip"
    src.write_text(PROBE)
    exe = d / "probe"
    subprocess.check_call(["hipcc", "-O2", "-std=c++17", f"-I{CSRC}", str(src), "-o", str(exe)],
                          stderr=subprocess.DEVNULL)
    return exe


def run(probe, keys):
    out = subprocess.run([str(probe)], input="\n".join(str(int(k)) for k in keys), capture_output=True, text=True,
                         check=True).stdout.split("\n")
    values, codes = [], {}
    for line in out:
        if line.startswith("v "):
            values.append(int(line.split()[2]))
        elif line.startswith("h "):
            _, k, c = line.split()
            codes[int(k)] = int(c)
    return values, codes


def test_hint_codes_round_up_and_keep_order(probe):
    top = (2048 + 2046) << 30  # the largest value with a code
    keys = {0, 1, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, top - 1, top, top + 1,
            (4095 << 30) - 1, 4095 << 30, (4095 << 30) + 1, 1 << 42, (1 << 42) + 1, (1 << 63) + 5, 2**64 - 1}
    for k in range(11, 64):
        keys |= {(1 << k) - 1, 1 << k, (1 << k) + 1}
    rng = np.random.default_rng(7)
    keys |= set(int(x) for x in rng.integers(0, 1 << 45, 5000, dtype=np.int64))
    keys |= set(int(x) for x in rng.integers(0, 1 << 20, 5000, dtype=np.int64))
    keys = sorted(k for k in keys if k < 2**64)
    values, codes = run(probe, keys)
    assert len(values) == 0xFFFF
    # Values grow strictly with codes, and codes below 2048 are the values themselves.
    assert all(values[c] < values[c + 1] for c in range(len(values) - 1))
    assert values[:2048] == list(range(2048)) and values[-1] == top
    for k in keys:
        c = codes[k]
        if k > top:
            assert c == 0xFFFF, k  # no bound known
            continue
        assert c < 0xFFFF, k
        assert values[c] >= k, (k, c)          # an upper bound
        assert c == 0 or values[c - 1] < k, (k, c)  # the smallest one
    # Order: a larger key never gets a smaller code.
    cs = [codes[k] for k in keys]
    assert all(a <= b for a, b in zip(cs, cs[1:]))
