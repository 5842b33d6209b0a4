// alp_reccursor.h -- the spread pass's walk over the pair records of a wave's
// work items, as index arithmetic only: which chunk of which item comes next,
// and which byte offset of the record area each lane reads for it.  The
// spread kernel loads through it; a host program compiled from the same
// source replays it over record layouts with bounds checks (no HIP header
// here, so a host compiler can include it with ALP_HD defined empty).
#pragma once
#include <stdint.h>

#ifndef ALP_HD
#define ALP_HD __host__ __device__ __forceinline__
#endif

namespace alp {

constexpr int kSpreadChunk = 64;          // records summed per pass, one per lane
constexpr uint64_t kRecNone = ~0ull;      // no record for this lane
constexpr uint32_t kRecReadBytes = 24;    // bytes a lane loads from a record's start, whatever its size
constexpr uint64_t kRecSlack = 256;       // readable bytes the record area has beyond its capacity

// An item's record base carries flags in its low bits (bases are 16-byte
// aligned): bit 0 for 24-byte records (FP64 weights), bit 2 for 12-byte
// records (FP32 weights, packed node index), else 16 bytes; bit 1 for an item
// whose cells have one run of records per entry group.
ALP_HD uint64_t rec_addr(uint64_t rb) { return rb & ~15ull; }
ALP_HD uint32_t rec_bytes(uint64_t rb) { return (rb & 1ull) ? 24u : ((rb & 4ull) ? 12u : 16u); }

// One chunk of the stream: records p0 .. p0 + 63 (those below rn) of `item`,
// whose record count and base are rn and rb.  item >= n_items: past the end.
struct RecChunk {
  uint32_t item, p0, rn;
  uint64_t rb;
};

// The chunks of a wave's items (item, item + stride, ...) in order.  Every
// item gives ceil(rn / 64) chunks and at least one, since the cells of an
// item without records are written too.  The cursor holds the chunk it hands
// out next and the count and base of the item after that chunk's item, read
// one item ahead.
struct RecCursor {
  RecChunk c;
  uint32_t gitem, grn;
  uint64_t grb;
};

// The first item of wave b in a grid of g waves (the wave then takes every
// g-th item).  Workgroups are handed to the device's eight XCDs in turn (b mod
// 8) and each XCD has its own L2: for g a multiple of 8 the waves of one XCD
// start on one contiguous eighth of every g consecutive items, rather than on
// every eighth item, so the items an L2 serves at a time lie closer together
// and share more of the beams whose forces their records read.  A permutation
// of 0 .. g-1.
constexpr uint32_t kXcds = 8;
ALP_HD uint32_t rec_first_item(uint32_t b, uint32_t g) {
  if (g % kXcds != 0u) return b;
  return (b % kXcds) * (g / kXcds) + b / kXcds;
}

// Src provides cnt(i) and base(i) for items i < n_items.
template <class Src>
ALP_HD RecCursor rec_start(const Src &src, uint32_t item, uint32_t n_items, uint32_t stride) {
  RecCursor k;
  k.c.item = item;
  k.c.p0 = 0;
  k.c.rn = 0;
  k.c.rb = 0;
  if (item < n_items) {
    k.c.rn = src.cnt(item);
    k.c.rb = src.base(item);
  }
  k.gitem = item + stride;
  k.grn = 0;
  k.grb = 0;
  if (item < n_items && k.gitem < n_items) {
    k.grn = src.cnt(k.gitem);
    k.grb = src.base(k.gitem);
  }
  return k;
}

// The next chunk; the cursor moves past it.
template <class Src>
ALP_HD RecChunk rec_take(const Src &src, RecCursor &k, uint32_t n_items, uint32_t stride) {
  const RecChunk out = k.c;
  if (out.item < n_items) {
    k.c.p0 += kSpreadChunk;
    if (k.c.p0 >= (k.c.rn > 0u ? k.c.rn : 1u)) {
      k.c.item = k.gitem;
      k.c.p0 = 0;
      k.c.rn = k.grn;
      k.c.rb = k.grb;
      k.grn = 0;
      k.grb = 0;
      if (k.gitem < n_items) {
        k.gitem += stride;
        if (k.gitem < n_items) {
          k.grn = src.cnt(k.gitem);
          k.grb = src.base(k.gitem);
        }
      }
    }
  }
  return out;
}

// Byte offset (into the record area) of this lane's record of chunk c, or
// kRecNone: a lane reads only records j < rn of the chunk's item.
ALP_HD uint64_t rec_lane(const RecChunk &c, uint32_t n_items, int lane) {
  const uint32_t j = c.p0 + (uint32_t)lane;
  if (c.item >= n_items || j >= c.rn) return kRecNone;
  return rec_addr(c.rb) + (uint64_t)j * rec_bytes(c.rb);
}

}  // namespace alp
