"""Host replay of the spread pass's record cursor (csrc/alp_reccursor.h).

The spread kernel walks the pair records of its work items (item, item +
stride, ...; the first item of each wave is chosen so that the waves of one
XCD start on neighbouring items) as one stream of chunks of up to 64 records,
every item giving at
least one chunk (the cells of an item without records are written too), with
two chunks in flight: a chunk's loads are issued two passes before it is
summed, and the next item's count and base are read one item ahead.  A C++
program compiled on the host from the same header replays that walk for every
wave of a grid over random record layouts (items without records, 12-, 16-
and 24-byte records, grouped items, gaps between reservations, grids larger
than the item count) and checks that every chunk comes in item order with the
right first record, that every lane's read of kRecReadBytes from its record
lies inside its own item's records or, for its tail, inside the record area
and its slack, that lanes past an item's records read nothing, that no
item's count or base is read past the item count, that the waves' first items
are a permutation of the grid, and that every item is summed exactly once.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2609_39443_amd", "csrc")

PROG = r'''
#define ALP_HD inline
#include "alp_reccursor.h"
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>
using namespace alp;

struct Src {
  const std::vector<uint32_t> *c;
  const std::vector<uint64_t> *b;
  mutable long bad = 0;
  uint32_t cnt(uint32_t i) const { if (i >= c->size()) { ++bad; return 0; } return (*c)[i]; }
  uint64_t base(uint32_t i) const { if (i >= b->size()) { ++bad; return 0; } return (*b)[i]; }
};

#define CHECK(cond, ...) do { if (!(cond)) { std::printf(__VA_ARGS__); std::printf("\n"); return 1; } } while (0)

int main() {
  std::mt19937_64 rng(12345);
  long checked = 0;
  for (int trial = 0; trial < 400; ++trial) {
    const uint32_t n = (uint32_t)(rng() % 3000);
    // grids of any size, and multiples of 8 (whose waves start XCD-wise)
    const uint32_t grid = trial % 2 ? 8 * (1 + (uint32_t)(rng() % 90)) : 1 + (uint32_t)(rng() % 700);
    std::vector<uint32_t> cnt(n);
    std::vector<uint64_t> base(n);
    // reservations in a random order, 16-byte aligned, with gaps
    std::vector<uint32_t> order(n);
    for (uint32_t i = 0; i < n; ++i) order[i] = i;
    for (uint32_t i = n; i > 1; --i) std::swap(order[i - 1], order[rng() % i]);
    uint64_t top = 0;
    const int mode = trial % 4;  // 0 mixed, 1 all empty, 2 large counts, 3 few records
    for (uint32_t q = 0; q < n; ++q) {
      const uint32_t i = order[q];
      uint32_t c = 0;
      if (mode == 0) c = (rng() % 3 == 0) ? 0 : (uint32_t)(rng() % 200);
      else if (mode == 2) c = (uint32_t)(rng() % 1000);
      else if (mode == 3) c = (rng() % 10 == 0) ? 1 + (uint32_t)(rng() % 70) : 0;
      const int kind = (int)(rng() % 3);  // 24-, 16- or 12-byte records
      const bool grouped = rng() % 5 == 0;
      const uint32_t size = kind == 0 ? 24 : (kind == 1 ? 16 : 12);
      top += 16 * (rng() % 4);  // a gap
      base[i] = top | (kind == 0 ? 1ull : 0ull) | (kind == 2 ? 4ull : 0ull) | (grouped ? 2ull : 0ull);
      top += ((uint64_t)c * size + 15) & ~15ull;
      cnt[i] = c;
    }
    const uint64_t cap = top;
    Src src{&cnt, &base};
    std::vector<uint32_t> seen(n, 0u), firsts(grid, 0u);
    for (uint32_t b = 0; b < grid; ++b) {
      const uint32_t first = rec_first_item(b, grid);
      CHECK(first < grid, "trial %d wave %u: first item %u outside the grid", trial, b, first);
      ++firsts[first];
      if (first >= n) continue;
      RecCursor cur = rec_start(src, first, n, grid);
      RecChunk A = rec_take(src, cur, n, grid), B = rec_take(src, cur, n, grid);
      // the chunks the summation must see, in order
      uint32_t item = first, p0 = 0;
      auto pass = [&](RecChunk &X) -> int {
        if (X.item >= n) return 0;
        if (X.item != item || X.p0 != p0) return -1;
        const uint32_t rn = cnt[item];
        if (X.rn != rn || X.rb != base[item]) return -1;
        if (p0 == 0) ++seen[item];
        for (int l = 0; l < 64; ++l) {
          const uint64_t at = rec_lane(X, n, l);
          const uint32_t j = p0 + (uint32_t)l;
          if (j < rn) {
            const uint64_t a0 = rec_addr(base[item]), sz = rec_bytes(base[item]);
            if (at != a0 + (uint64_t)j * sz) return -2;
            if (at + sz > a0 + (uint64_t)rn * sz) return -3;       // the record is the item's
            if (at + kRecReadBytes > cap + kRecSlack) return -4;   // the read stays in the area
            ++checked;
          } else if (at != kRecNone) {
            return -5;
          }
        }
        p0 += kSpreadChunk;
        if (p0 >= (rn > 0 ? rn : 1u)) {
          item += grid;
          p0 = 0;
        }
        X = rec_take(src, cur, n, grid);
        return 1;
      };
      for (;;) {
        int r = pass(A);
        if (r == 1) r = pass(B);
        CHECK(r >= 0, "trial %d wave %u item %u p0 %u: chunk check %d", trial, b, item, p0, r);
        if (r == 0) break;
      }
      CHECK(item >= n, "trial %d wave %u: the stream ended before item %u", trial, b, item);
      CHECK(A.item >= n && B.item >= n, "trial %d wave %u: chunks after the last item", trial, b);
    }
    CHECK(src.bad == 0, "trial %d: %ld count/base reads past the item count", trial, src.bad);
    for (uint32_t b = 0; b < grid; ++b) CHECK(firsts[b] == 1, "trial %d: %u waves start at %u", trial, firsts[b], b);
    for (uint32_t i = 0; i < n; ++i) CHECK(seen[i] == 1, "trial %d: item %u summed %u times", trial, i, seen[i]);
  }
  std::printf("ok %ld\n", checked);
  return 0;
}
'''


def test_record_cursor_reads_stay_inside_each_items_records(tmp_path):
    src = tmp_path / "replay.cpp"
    src.write_text(PROG)
    exe = tmp_path / "replay"
    subprocess.check_call(["g++", "-std=c++17", "-O2", "-I", CSRC, str(src), "-o", str(exe)])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=240)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
    assert int(out.stdout.split()[1]) > 100000
