"""Host build of the group step's search block: philox10_late_loc, taken verbatim from the
library source and compiled with the host compiler, equals the oracle's Philox4x32-10 of the
counter (loc, kk, 0, c3) -- words 1:0, or words 3:2 for the second draw -- on random counters
under several keys and on the extreme words.  The function splits the block so that the
parts that do not depend on the location can be computed before it is known, and forms only
one product in the last round; a slip in that split (a key bump, a product or a word out of
place) changes the draw."""
import ctypes as C
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_2108_05815_amd", "csrc", "necsim_hip.hip")

HARNESS = r"""
#include <cstdint>
#define __device__
#define __forceinline__ inline
static inline uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) { return a ^ b ^ c; }
%s
extern "C" void late_loc_array(const uint32_t *loc, const uint32_t *kk, const uint32_t *c3, uint64_t n,
                               uint32_t k0, uint32_t k1, uint32_t second, uint64_t *out) {
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t n0 = kk[i] ^ k0;
        const uint64_t m = (uint64_t)0xD2511F53u * n0;
        out[i] = philox10_late_loc(loc[i], n0, m, c3[i], k0, k1, second != 0);
    }
}
"""


def _function_text() -> str:
    text = open(SRC).read()
    m = re.search(r"__device__ __forceinline__ uint64_t philox10_late_loc\(.*?\n}\n", text, flags=re.S)
    assert m, "philox10_late_loc not found in the library source"
    return m.group(0)


@pytest.fixture(scope="module")
def late_loc(tmp_path_factory):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    d = tmp_path_factory.mktemp("late_loc")
    src, lib = d / "late_loc.cpp", d / "late_loc.so"
    src.write_text(HARNESS % _function_text())
    subprocess.run([cxx, "-O2", "-std=c++17", "-Wno-unknown-pragmas", "-shared", "-fPIC", str(src), "-o", str(lib)],
                   check=True)
    h = C.CDLL(str(lib))
    u32p, u64p = C.POINTER(C.c_uint32), C.POINTER(C.c_uint64)
    h.late_loc_array.argtypes = [u32p, u32p, u32p, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint32, u64p]
    h.late_loc_array.restype = None

    def run(loc, kk, c3, key, second):
        loc, kk, c3 = (np.ascontiguousarray(a, dtype=np.uint32) for a in (loc, kk, c3))
        out = np.zeros(len(loc), dtype=np.uint64)
        h.late_loc_array(loc.ctypes.data_as(u32p), kk.ctypes.data_as(u32p), c3.ctypes.data_as(u32p), len(loc),
                         int(key[0]), int(key[1]), int(second), out.ctypes.data_as(u64p))
        return out
    return run


def _expected(loc, kk, c3, key):
    ctr = np.stack([loc, kk, np.zeros_like(loc), c3], axis=1).astype(np.uint32)
    w = oracle.philox_array(ctr, np.asarray(key, dtype=np.uint32)).astype(np.uint64)
    first = (w[:, 1] << np.uint64(32)) | w[:, 0]
    second = (w[:, 3] << np.uint64(32)) | w[:, 2]
    return first, second


def _check(late_loc, loc, kk, c3, key):
    first, second = _expected(loc, kk, c3, key)
    assert np.array_equal(late_loc(loc, kk, c3, key, False), first)
    assert np.array_equal(late_loc(loc, kk, c3, key, True), second)


@pytest.mark.parametrize("key", [(0, 0), (0x9E3779B9, 0xBB67AE85), (0xFFFFFFFF, 1), (123456789, 987654321)])
def test_search_block_equals_philox_on_random_counters(late_loc, key):
    rng = np.random.default_rng(2108 + key[0] % 97)
    n = 200_000
    loc = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    kk = rng.integers(0, 2**32, n, dtype=np.uint64).astype(np.uint32)
    c3 = rng.integers(0, 4, n, dtype=np.uint64).astype(np.uint32)
    _check(late_loc, loc, kk, c3, key)


def test_search_block_equals_philox_on_extreme_words(late_loc):
    words = np.array([0, 1, 2, 3, 0x7FFFFFFF, 0x80000000, 0xFFFFFFFE, 0xFFFFFFFF], dtype=np.uint32)
    loc, kk, c3 = (a.ravel() for a in np.meshgrid(words, words, np.arange(4, dtype=np.uint32), indexing="ij"))
    for k0 in words:
        for k1 in words:
            _check(late_loc, loc, kk, c3, (k0, k1))
