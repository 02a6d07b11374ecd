"""The batch work lists (paper_2409_07563_amd/csrc/worklist.h) and their
host-side check, without a GPU: the library builds every table with these
functions and refuses to upload one the check rejects.  A small harness is
compiled with g++ against the same header."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_2409_07563_amd", "csrc")

HARNESS = r'''
#include "worklist.h"
#include <string.h>
using namespace mppi;
extern "C" {
int build_samples(const int32_t* K, const int32_t* T, int n, int tile, int32_t* out, int cap) {
  std::vector<WorkItem> v = build_sample_tiles(K, T, n, tile);
  if ((int)v.size() > cap) return -1;
  memcpy(out, v.data(), v.size() * sizeof(WorkItem));
  return (int)v.size();
}
int build_rows(const int32_t* TM, int n, int rpb, int32_t* out, int cap) {
  std::vector<WorkItem> v = build_row_tiles(TM, n, rpb);
  if ((int)v.size() > cap) return -1;
  memcpy(out, v.data(), v.size() * sizeof(WorkItem));
  return (int)v.size();
}
int check(const int32_t* items, long long n, long long cap, int unit, const int32_t* extent,
          int n_inst, char* msg, int len) {
  std::string s = check_work_list(reinterpret_cast<const WorkItem*>(items), n, cap, unit,
                                  extent, n_inst);
  snprintf(msg, len, "%s", s.c_str());
  return s.empty() ? 0 : 1;
}
}
'''


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    d = tmp_path_factory.mktemp("worklist")
    src = d / "harness.cpp"
    src.write_text(HARNESS)
    lib = d / "harness.so"
    subprocess.run(["g++", "-std=c++17", "-O1", "-shared", "-fPIC", f"-I{HDR}", str(src), "-o",
                    str(lib)], check=True)
    L = C.CDLL(str(lib))
    i32 = np.ctypeslib.ndpointer(np.int32, flags="C")
    L.build_samples.argtypes = [i32, i32, C.c_int, C.c_int, i32, C.c_int]
    L.build_rows.argtypes = [i32, C.c_int, C.c_int, i32, C.c_int]
    L.check.argtypes = [i32, C.c_longlong, C.c_longlong, C.c_int, i32, C.c_int, C.c_char_p,
                        C.c_int]
    return L


def _check(L, items, cap, unit, extent):
    msg = C.create_string_buffer(200)
    items = np.ascontiguousarray(np.asarray(items, np.int32).reshape(-1, 2))
    rc = L.check(items, len(items), cap, unit, np.asarray(extent, np.int32), len(extent), msg, 200)
    return rc, msg.value.decode()


def _samples(L, K, T, tile):
    out = np.zeros((sum(-(-k // 64) for k in K), 2), np.int32)
    n = L.build_samples(np.asarray(K, np.int32), np.asarray(T, np.int32), len(K), tile, out,
                        len(out))
    assert n >= 0
    return out[:n]


K = [1024, 700, 16384, 1, 65, 2048]
T = [50, 200, 100, 200, 150, 50]


@pytest.mark.parametrize("tile", [64, 128, 256])
def test_built_sample_tiles_pass_and_are_ordered(harness, tile):
    tiles = _samples(harness, K, T, tile)
    cap = sum(-(-k // 64) for k in K)          # the workspace table holds 64-sample tiles
    assert _check(harness, tiles, cap, tile, K) == (0, "")
    horizons = [T[i] for i, _ in tiles]
    assert horizons == sorted(horizons, reverse=True)


def test_built_row_tiles_pass(harness):
    TM = np.asarray([100, 400, 200, 1, 300], np.int32)
    out = np.zeros((int(TM.sum()), 2), np.int32)
    n = harness.build_rows(TM, len(TM), 1, out, len(out))
    assert n == TM.sum()
    assert _check(harness, out[:n], len(out), 1, TM) == (0, "")


def test_check_rejects_a_mismatched_grouping(harness):
    # a table built for 64-sample tiles checked (launched) as 256-sample
    # tiles: entries start past their instance's samples
    tiles64 = _samples(harness, K, T, 64)
    rc, msg = _check(harness, tiles64, len(tiles64), 256, K)
    assert rc == 1 and msg
    # a table built for 256-sample tiles launched with 64: samples uncovered
    tiles256 = _samples(harness, K, T, 256)
    rc, msg = _check(harness, tiles256, len(tiles64), 64, K)
    assert rc == 1 and "need" in msg


def test_check_rejects_bad_entries(harness):
    tiles = _samples(harness, K, T, 128)
    cap = len(tiles)
    bad = tiles.copy()
    bad[3, 0] = len(K)                         # instance past the descriptor table
    assert _check(harness, bad, cap, 128, K)[0] == 1
    bad = tiles.copy()
    bad[0, 1] = -1                             # negative index
    assert _check(harness, bad, cap, 128, K)[0] == 1
    bad = tiles.copy()
    bad[1] = bad[0]                            # duplicate (and a tile missing)
    assert "twice" in _check(harness, bad, cap, 128, K)[1]
    # more entries than the workspace table holds
    assert "table" in _check(harness, tiles, cap - 1, 128, K)[1]
    # a row tile past T*m: the fault the device-side guard also stops
    TM = [10, 20]
    rows = [[0, i] for i in range(10)] + [[1, i] for i in range(19)] + [[1, 20]]
    assert "outside" in _check(harness, rows, 40, 1, TM)[1]
