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

// The spread runs workgroups of kSpreadGroupWaves waves, and the items are
// dealt in windows of g = (workgroups) x kSpreadGroupWaves consecutive items:
// every workgroup owns kSpreadGroupWaves consecutive items of each window,
// and its waves take the workgroup's items in window order from a counter in
// its LDS, so a wave that finishes an item early takes the next one instead
// of a fixed share, while all waves move through the windows together.
// Workgroups are handed to the device's eight XCDs in turn (workgroup index
// mod 8) and each XCD has its own L2: for a workgroup count that is a
// multiple of 8, the workgroups of one XCD own one contiguous block of each
// window, so the items an L2 serves at a time lie close together and share
// more of the beams whose forces their records read.  Ticket t of a workgroup
// whose first item is `base` is item (t / W) g + base + t mod W (W the waves
// per workgroup).
constexpr uint32_t kXcds = 8;
constexpr uint32_t kSpreadGroupWaves = 16;
ALP_HD uint32_t rec_group_base(uint32_t grp, uint32_t ngroups) {
  const uint32_t nx = ngroups % kXcds == 0u ? kXcds : 1u;
  const uint32_t per_xcd = ngroups / nx;  // workgroups per XCD
  return (grp % nx) * per_xcd * kSpreadGroupWaves + (grp / nx) * kSpreadGroupWaves;
}
ALP_HD uint32_t rec_ticket_item(uint32_t t, uint32_t base, uint32_t g) {
  const uint64_t it = (uint64_t)(t / kSpreadGroupWaves) * g + base + t % kSpreadGroupWaves;
  return it > 0xffffffffull ? 0xffffffffu : (uint32_t)it;
}

// The chunks of a wave's items in order.  Every item gives ceil(rn / 64)
// chunks and at least one, since the cells of an item without records are
// written too.  The cursor holds the chunk it hands out next and the item
// after that chunk's item, with its count and base (read one item ahead).  A
// wave takes a ticket only while it holds a valid next item and uses every
// ticket it takes; a workgroup's tickets come in increasing order and map to
// increasing items, so each of its items is summed by exactly one wave.
struct RecCursor {
  RecChunk c;
  uint32_t gitem, grn;
  uint64_t grb;
  uint32_t base, g;  // the workgroup's first item and the window length
};

// Src provides cnt(i) and base(i) for items i < n_items and ticket(), the
// workgroup counter's next value.
template <class Src>
ALP_HD RecCursor rec_start(const Src &src, uint32_t base, uint32_t g, uint32_t n_items) {
  RecCursor k;
  k.base = base;
  k.g = g;
  k.c.item = rec_ticket_item(src.ticket(), base, g);
  k.c.p0 = 0;
  k.c.rn = 0;
  k.c.rb = 0;
  k.gitem = n_items;
  k.grn = 0;
  k.grb = 0;
  if (k.c.item < n_items) {
    k.c.rn = src.cnt(k.c.item);
    k.c.rb = src.base(k.c.item);
    k.gitem = rec_ticket_item(src.ticket(), base, g);
    if (k.gitem < n_items) {
      k.grn = src.cnt(k.gitem);
      k.grb = src.base(k.gitem);
    }
  }
  return k;
}

// The next chunk; the cursor moves past it.
template <class Src>
ALP_HD RecChunk rec_take(const Src &src, RecCursor &k, uint32_t n_items) {
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
        k.gitem = rec_ticket_item(src.ticket(), k.base, k.g);
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
