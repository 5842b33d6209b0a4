"""Host replay of the spread pass's record cursor (csrc/alp_reccursor.h).

The spread kernel runs workgroups of 16 waves; every workgroup owns 16
consecutive work items of each window of g items (g = 16 x the workgroups;
the workgroups of one XCD own one block of each window), and its waves take
the workgroup's items in window order from a counter in its LDS.  A wave walks
its items as one stream of chunks of up to 64 records, every item giving at
least one chunk (the cells of an item without records are written too), with
two chunks in flight: a chunk's loads are issued two passes before it is
summed, and the next item's count and base are read one item ahead.  A C++
program compiled on the host from the same header replays every wave of a
grid, one pass at a time in a random order over the workgroups' counters,
over random record layouts (items without records, 12-, 16- and 24-byte
records, grouped items, gaps between reservations, grids larger than the item
count and workgroup counts that are not multiples of 8), and checks that
every chunk comes in item order with the right first record, that a wave's
items increase and lie in its workgroup's block of each window, that every
lane's read of kRecReadBytes from its record lies inside its own item's
records or, for its tail, inside the record area and its slack, that lanes
past an item's records read nothing, that no item's count or base is read
past the item count, that the workgroups' blocks tile every window with each
XCD's inside its part, and that every item is summed exactly once.
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
  uint32_t *ctr;  // the workgroup's counter
  long *bad;
  uint32_t cnt(uint32_t i) const { if (i >= c->size()) { ++*bad; return 0; } return (*c)[i]; }
  uint64_t base(uint32_t i) const { if (i >= b->size()) { ++*bad; return 0; } return (*b)[i]; }
  uint32_t ticket() const { return (*ctr)++; }
};

#define CHECK(cond, ...) do { if (!(cond)) { std::printf(__VA_ARGS__); std::printf("\n"); return 1; } } while (0)

struct Wave {
  Src src;
  RecCursor cur;
  RecChunk A, B;
  bool onA = true;
  uint32_t item = 0, p0 = 0, grp = 0;
};

int main() {
  std::mt19937_64 rng(12345);
  long checked = 0;
  const uint32_t Wg = kSpreadGroupWaves;
  for (int trial = 0; trial < 400; ++trial) {
    const uint32_t n = (uint32_t)(rng() % 3000);
    // workgroup counts of any size, and multiples of 8 (whose workgroups own XCD blocks)
    const uint32_t ngroups = trial % 2 ? 8 * (1 + (uint32_t)(rng() % 12)) : 1 + (uint32_t)(rng() % 40);
    const uint32_t g = ngroups * Wg;
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
    // the workgroups' blocks tile the window, each XCD's inside its eighth
    std::vector<uint32_t> cover(g, 0u);
    const uint32_t nx = ngroups % 8 == 0 ? 8 : 1;
    for (uint32_t w = 0; w < ngroups; ++w) {
      const uint32_t b0 = rec_group_base(w, ngroups);
      CHECK(b0 + Wg <= g, "trial %d group %u: block at %u outside the window %u", trial, w, b0, g);
      CHECK(b0 / (g / nx) == w % nx, "trial %d group %u: block at %u outside its XCD's part", trial, w, b0);
      for (uint32_t j = 0; j < Wg; ++j) ++cover[b0 + j];
    }
    for (uint32_t i = 0; i < g; ++i) CHECK(cover[i] == 1, "trial %d: window place %u owned %u times", trial, i, cover[i]);
    std::vector<uint32_t> ctrs(ngroups, 0u), seen(n, 0u);
    long bad = 0;
    std::vector<Wave> waves(ngroups * Wg);
    std::vector<uint32_t> live;
    // waves start in a random order too
    std::vector<uint32_t> start(waves.size());
    for (uint32_t i = 0; i < start.size(); ++i) start[i] = i;
    for (uint32_t i = (uint32_t)start.size(); i > 1; --i) std::swap(start[i - 1], start[rng() % i]);
    for (uint32_t id : start) {
      Wave &v = waves[id];
      v.grp = id / Wg;
      v.src = Src{&cnt, &base, &ctrs[v.grp], &bad};
      v.cur = rec_start(v.src, rec_group_base(v.grp, ngroups), g, n);
      v.item = v.cur.c.item;
      if (v.item >= n) continue;
      v.A = rec_take(v.src, v.cur, n);
      v.B = rec_take(v.src, v.cur, n);
      live.push_back(id);
    }
    auto pass = [&](Wave &v) -> int {
      RecChunk &X = v.onA ? v.A : v.B;
      if (X.item >= n) return 0;
      if (X.item != v.item || X.p0 != v.p0) return -1;
      const uint32_t b0 = rec_group_base(v.grp, ngroups);
      if ((v.item % g) < b0 || (v.item % g) >= b0 + Wg) return -6;  // the workgroup's block
      const uint32_t rn = cnt[v.item];
      if (X.rn != rn || X.rb != base[v.item]) return -1;
      if (v.p0 == 0) ++seen[v.item];
      for (int l = 0; l < 64; ++l) {
        const uint64_t at = rec_lane(X, n, l);
        const uint32_t j = v.p0 + (uint32_t)l;
        if (j < rn) {
          const uint64_t a0 = rec_addr(base[v.item]), sz = rec_bytes(base[v.item]);
          if (at != a0 + (uint64_t)j * sz) return -2;
          if (at + sz > a0 + (uint64_t)rn * sz) return -3;       // the record is the item's
          if (at + kRecReadBytes > cap + kRecSlack) return -4;   // the read stays in the area
          ++checked;
        } else if (at != kRecNone) {
          return -5;
        }
      }
      v.p0 += kSpreadChunk;
      if (v.p0 >= (rn > 0 ? rn : 1u)) {
        // the next item is the one the other chunk in flight names (or past the end)
        const RecChunk &Y = v.onA ? v.B : v.A;
        if (Y.item < n && Y.item <= v.item) return -7;  // a wave's items increase
        v.item = Y.item < n ? Y.item : n;
        v.p0 = 0;
      }
      X = rec_take(v.src, v.cur, n);
      v.onA = !v.onA;
      return 1;
    };
    while (!live.empty()) {
      const size_t k = (size_t)(rng() % live.size());
      Wave &v = waves[live[k]];
      const int r = pass(v);
      CHECK(r >= 0, "trial %d wave %u item %u p0 %u: chunk check %d", trial, live[k], v.item, v.p0, r);
      if (r == 0) {
        CHECK(v.A.item >= n && v.B.item >= n, "trial %d wave %u: chunks after the last item", trial, live[k]);
        live[k] = live.back();
        live.pop_back();
      }
    }
    CHECK(bad == 0, "trial %d: %ld count/base reads past the item count", trial, bad);
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
