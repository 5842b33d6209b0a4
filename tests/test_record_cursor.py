"""Host replay of the spread pass's record cursor (csrc/alp_reccursor.h).

The spread kernel walks the pair records of its work items (item, item +
stride, ...) as one stream of 64-record chunks, with the cursor two chunks
ahead of the summation and the next item's count and base read one item
ahead.  A C++ program compiled on the host from the same header replays that
walk for every wave of a grid over random record layouts (items without
records, 12-, 16- and 24-byte records, grouped items, gaps between reservations,
grids larger than the item count) and checks that every record read lies
inside its own item's records and inside the record area, that no item's
count or base is read past the item count, and that the chunk each lane sums
is the record the summation expects.
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
    const uint32_t grid = 1 + (uint32_t)(rng() % 700);
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
    // one wave per block: each call of rec_next by the 64 lanes starts from the
    // same (wave-uniform) cursor; the cursor after a chunk is any lane's
    auto chunk = [&](RecCursor &cur, uint64_t (*out)[2]) {
      RecCursor after = cur;
      for (int l = 0; l < 64; ++l) {
        RecCursor t = cur;
        uint32_t bytes;
        out[l][0] = rec_next(src, t, n, grid, l, &bytes);
        out[l][1] = bytes;
        after = t;
      }
      cur = after;
    };
    for (uint32_t b = 0; b < grid; ++b) {
      uint32_t item = b;
      if (item >= n) continue;
      uint32_t rn = src.cnt(item);
      uint64_t rb = src.base(item);
      RecCursor cur = rec_start(src, item, rn, rb, n, grid);
      uint64_t R1[64][2], R2[64][2];
      chunk(cur, R1);  // the cursor runs two chunks ahead of the summation
      chunk(cur, R2);
      for (;;) {
        for (uint32_t p0 = 0; p0 < rn; p0 += kSpreadChunk) {
          // the chunk summed now must be records p0 .. p0 + 63 of this item
          for (int l = 0; l < 64; ++l) {
            const uint32_t j = p0 + (uint32_t)l;
            if (j < rn) {
              const uint64_t want = rec_addr(rb) + (uint64_t)j * rec_bytes(rb);
              CHECK(R1[l][0] == want && R1[l][1] == rec_bytes(rb),
                    "trial %d wave %u item %u record %u: read %llu, want %llu", trial, b, item, j,
                    (unsigned long long)R1[l][0], (unsigned long long)want);
              CHECK(R1[l][0] + R1[l][1] <= cap, "record outside the record area");
              ++checked;
            } else {
              CHECK(R1[l][0] == kRecNone, "trial %d wave %u item %u: lane %d past the item's records reads %llu",
                    trial, b, item, l, (unsigned long long)R1[l][0]);
            }
          }
          std::memcpy(R1, R2, sizeof(R1));
          chunk(cur, R2);
          for (int l = 0; l < 64; ++l)
            if (R2[l][0] != kRecNone) CHECK(R2[l][0] + R2[l][1] <= cap, "prefetch outside the record area");
        }
        item += grid;
        if (item >= n) break;
        rn = src.cnt(item);
        rb = src.base(item);
      }
      CHECK(cur.done, "trial %d wave %u: the cursor still has records after the last item", trial, b);
    }
    CHECK(src.bad == 0, "trial %d: %ld count/base reads past the item count", trial, src.bad);
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
