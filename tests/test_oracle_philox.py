"""Pins for the oracle's Philox4x32-10 (Salmon et al., SC 2011).

Three independent checks: the published known-answer vectors, PyTorch's
header-only engine (ATen/core/PhiloxRNGEngine.h) and rocRAND's
(rocrand/rocrand_philox4x32_10.h), both compiled here on the host.  The last
two also pin the counter layout (k, t, qid_lo, qid_hi) and key = seed,
through each library's documented (seed, subsequence, offset) interface.
"""
import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

import oracle
from helpers import golden_path

TORCH_PROG = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
int main() {
  unsigned long long seed, qid, k, t;
  while (std::scanf("%llu %llu %llu %llu", &seed, &qid, &k, &t) == 4) {
    at::philox_engine e(seed, qid, (t << 32) | k);   // counter = (k, t, qid_lo, qid_hi)
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""

ROCRAND_PROG = r"""
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
  unsigned long long seed, qid, k, t;
  while (std::scanf("%llu %llu %llu %llu", &seed, &qid, &k, &t) == 4) {
    // offset counts 32-bit outputs: 4 per block
    rocrand_device::philox4x32_10_engine e(seed, qid, 4ull * ((t << 32) | k));
    unsigned a = e(), b = e(), c = e(), d = e();
    std::printf("%u %u %u %u\n", a, b, c, d);
  }
}
"""


def _grid():
    rng = np.random.default_rng(12345)
    rows = []
    for seed in [0, 1, 0x5EED000002, 0xFFFFFFFFFFFFFFFF, int(rng.integers(0, 2**63))]:
        for qid in [0, 1, 9_999_999, 2**32 - 1, 2**32, (7 << 32) | 123, int(rng.integers(0, 2**62))]:
            for k in [0, 1, 79, 255, 65535]:
                for t in [0, 1, 3, 2**20]:
                    rows.append((seed, qid, k, t))
    return rows


def _oracle_block(seed, qid, k, t):
    return oracle.philox4x32_10([k, t, qid & 0xFFFFFFFF, qid >> 32],
                                [seed & 0xFFFFFFFF, seed >> 32])


def test_known_answer_vectors(oracle_lib):
    n = 0
    for line in open(golden_path("philox4x32_10_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        out = oracle.philox4x32_10(v[0:4], v[4:6])
        assert list(out) == v[6:10]
        n += 1
    assert n == 3


def _run_prog(tmp_path, src, compiler_cmd, name):
    cpp = tmp_path / f"{name}.cpp"
    exe = tmp_path / name
    cpp.write_text(src)
    subprocess.check_call(compiler_cmd(str(cpp), str(exe)), stdout=subprocess.DEVNULL,
                          stderr=subprocess.DEVNULL)
    rows = _grid()
    inp = "".join(f"{s} {q} {k} {t}\n" for s, q, k, t in rows)
    out = subprocess.run([str(exe)], input=inp, capture_output=True, text=True, check=True).stdout
    got = [tuple(int(x) for x in l.split()) for l in out.strip().splitlines()]
    assert len(got) == len(rows)
    for (s, q, k, t), ref in zip(rows, got):
        assert tuple(int(x) for x in _oracle_block(s, q, k, t)) == ref, (s, q, k, t)


def test_matches_pytorch_engine(tmp_path, oracle_lib):
    import torch
    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("PyTorch headers not present")
    _run_prog(tmp_path, TORCH_PROG,
              lambda c, e: ["g++", "-std=c++17", "-O1", "-I", inc, c, "-o", e], "torch_philox")


def test_matches_rocrand_engine(tmp_path, oracle_lib):
    hipcc = shutil.which("hipcc")
    if hipcc is None or not os.path.exists("/opt/rocm/include/rocrand/rocrand_philox4x32_10.h"):
        pytest.skip("rocRAND headers / hipcc not present")
    _run_prog(tmp_path, ROCRAND_PROG,
              lambda c, e: [hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", c, "-o", e],
              "rocrand_philox")
