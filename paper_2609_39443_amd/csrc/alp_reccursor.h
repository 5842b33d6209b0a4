// alp_reccursor.h -- the spread pass's walk over the pair records of a wave's
// work items, as index arithmetic only: which byte offset of the record area
// each lane reads for each 64-record chunk.  The spread kernel loads through
// it; a host program compiled from the same source replays it over record
// layouts with bounds checks (no HIP header here, so a host compiler can
// include it with ALP_HD defined empty).
#pragma once
#include <stdint.h>

#ifndef ALP_HD
#define ALP_HD __host__ __device__ __forceinline__
#endif

namespace alp {

constexpr int kSpreadChunk = 64;          // records summed per pass, one per lane
constexpr uint64_t kRecNone = ~0ull;      // no record for this lane

// An item's record base carries flags in its low bits (bases are 16-byte
// aligned): bit 0 for 24-byte records (FP64 weights), bit 2 for 12-byte
// records (FP32 weights, packed node index), else 16 bytes; bit 1 for an item
// whose cells have one run of records per entry group.
ALP_HD uint64_t rec_addr(uint64_t rb) { return rb & ~15ull; }
ALP_HD uint32_t rec_bytes(uint64_t rb) { return (rb & 1ull) ? 24u : ((rb & 4ull) ? 12u : 16u); }

// The records of a wave's items (item, item + stride, ...), taken as one
// stream of 64-record chunks.  The cursor runs ahead of the summation; it
// holds the count and base of the item after its own, read ahead as well.
struct RecCursor {
  uint32_t item, p0, rn;  // item, first record of the chunk to fetch, item's record count
  uint64_t rb;            // item's record base (with the flag bits)
  uint32_t gitem, grn;    // the item after it
  uint64_t grb;
  bool done;
};

// Src provides cnt(i) and base(i) for items i < n_items.
template <class Src>
ALP_HD void rec_settle(const Src &src, RecCursor &c, uint32_t n_items, uint32_t stride) {
  while (!c.done && c.p0 >= c.rn) {  // skip to the next chunk that has records
    if (c.gitem >= n_items) {
      c.done = true;
      break;
    }
    c.item = c.gitem;
    c.rn = c.grn;
    c.rb = c.grb;
    c.p0 = 0;
    c.gitem += stride;
    if (c.gitem < n_items) {
      c.grn = src.cnt(c.gitem);
      c.grb = src.base(c.gitem);
    }
  }
}

// A cursor at the first chunk with records of the wave's items, the first
// being `item` (< n_items) with count rn and base rb.
template <class Src>
ALP_HD RecCursor rec_start(const Src &src, uint32_t item, uint32_t rn, uint64_t rb, uint32_t n_items,
                           uint32_t stride) {
  RecCursor c;
  c.item = item;
  c.p0 = 0;
  c.rn = rn;
  c.rb = rb;
  c.gitem = item + stride;
  c.grn = 0;
  c.grb = 0;
  c.done = false;
  if (c.gitem < n_items) {
    c.grn = src.cnt(c.gitem);
    c.grb = src.base(c.gitem);
  }
  rec_settle(src, c, n_items, stride);
  return c;
}

// Byte offset (into the record area) of this lane's record of the cursor's
// chunk, or kRecNone, with the record size in *bytes; then the cursor moves
// to its next chunk.  A lane reads only records j < rn of the cursor's item.
template <class Src>
ALP_HD uint64_t rec_next(const Src &src, RecCursor &c, uint32_t n_items, uint32_t stride, int lane,
                         uint32_t *bytes) {
  uint64_t at = kRecNone;
  *bytes = 16u;
  if (!c.done) {
    const uint32_t j = c.p0 + (uint32_t)lane;
    if (j < c.rn) {
      *bytes = rec_bytes(c.rb);
      at = rec_addr(c.rb) + (uint64_t)j * *bytes;
    }
    c.p0 += kSpreadChunk;
    rec_settle(src, c, n_items, stride);
  }
  return at;
}

}  // namespace alp
