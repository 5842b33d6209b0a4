// alp_internal.h -- device-side data layout and helpers shared by the libalp
// kernels (gfx950).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "alp.h"

namespace alp {

constexpr int kWave = 64;
constexpr int kChunkSegs = 16;      // segments per chunk in the segment binning
constexpr int kMaxEmitTile = 256;   // (chunk, tile) windows of a tile merged by k_tile_merge
constexpr int kMaxEmitBig = 4096;   // windows of a tile merged by k_tile_merge_big (the limit)
constexpr int kBigTileCounter = 4;  // step counter word: tiles listed for k_tile_merge_big
constexpr int kMultiItemCounter = 5;  // step counter word: items listed for the grouped weights kernels
constexpr int kQueueStripes = 16;  // counters per work queue
constexpr int kLineWords = 32;                    // uint32 words per 128-byte line
// step counters: a line of flags, then eight work queues (the four common
// weights kernels' and their grouped kernels') whose counters each sit on a
// line of their own (atomics on one line serialise)
constexpr int kCounters = kLineWords + 8 * kQueueStripes * kLineWords;
__host__ __device__ constexpr int queue_words(int q) { return kLineWords + q * kQueueStripes * kLineWords; }
constexpr int kMaxEntries = 128;    // merged (tile, beam) entries the weights pass takes at once
constexpr int kMaskWords = kMaxEntries / 32;
constexpr int kStagePts = 160;      // window points (and node accumulators) staged in LDS
// flag on a tile's entry count: its entries' windows hold more points than
// the staging area, so its items are taken in groups by the grouped kernels
constexpr uint32_t kNentGrouped = 1u << 31;
constexpr int kHiShift = 46;        // fixed-point: hi word holds v * 2^(46-E)
constexpr int kLoBits = 40;         // lo word holds the next 40 bits
constexpr int kSampleLanes = 4;  // lanes per actuator point in the sampler
constexpr unsigned long long kRecBlock = 64ull << 10;  // pair-record bytes a wave reserves at once
constexpr int kCnt = 16;            // per-case counters (see Work::cnt)

// Binned mesh, device view (built by alp_bin_cells).
struct MeshDev {
  int32_t n_cells;
  int32_t T;        // bins per tile edge
  int32_t nb[3];    // bins per axis (multiple of T)
  int32_t nt[3];    // tiles per axis
  int64_t n_bins, n_tiles;
  double lo[3];     // grid origin
  double bin, inv_bin, tile_len;
  double box[6];    // domain box (outside -> no load)
  double vmax;      // largest cell volume
  const uint32_t *bin_start;  // [n_bins+1] sorted-cell ranges, bins in tile-major order
  const double *cx, *cy, *cz; // [n] sorted centres (FP64, absolute)
  const double *cxyz;         // [n][4] the same centres interleaved with the caller index
                              // (x, y, z, index as a double): point location reads a
                              // cell's coordinates and index from one 32-byte record
  const double *vs;           // [n] sorted volumes
  const uint32_t *perm;       // [n] sorted -> caller index
};

// One case of a step, device view.  Points, beams and tiles of all cases are
// concatenated into global index spaces (the *_base fields).
struct CaseDev {
  MeshDev m;
  int64_t point_base, beam_base, tile_base;
  int64_t n_points;
  int32_t n_beams;
  int32_t prec, drag_form;
  int32_t has_fprev;
  double rho, alpha_f, tau;
  const int64_t *offsets;
  const double *P, *Psp, *e_t, *Pdot, *d, *L, *eps, *Cdn, *Cdt, *ls, *n_p, *e_up;
  const double *A, *CMn, *CMt, *a_b;  // Morison inertia (A == nullptr: none)
  const double *dUdt;                  // fluid acceleration field, or nullptr
  const double *U;
  const double *f_prev;
  double *S, *f, *U_s, *P_s, *w, *fhat;
  int64_t *cell_a, *cell_s;
  uint8_t *tile_prev;   // [n_tiles] tiles written at the previous step of this mesh
  int32_t write_S;      // spread writes S (0 for sample/drag-only calls)
  int32_t sample_mode;  // alp_sample_mode
  int32_t proj_mode;    // alp_proj_mode
};

// A (chunk, tile) window: the candidate segments lo..hi of one chunk of a
// beam for one tile (segment binning output, grouped by tile).
struct Emit {
  int32_t beam;   // global beam index
  int32_t lo, hi; // candidate segments (beam-local); 0..0 for a single-point beam
  int32_t tile;   // global tile index
};

// Pair record written by the weights pass and read by the spread pass.  Split
// precision: one word holding the cell lane in the work item (bits 0-5), 1 in
// bit 6 for a single-point beam and the global index of the first node above
// bit 6, then a0 and a1 as float: 12 bytes, while a batch has fewer than 2^25
// points; else the 16-byte form below with a0, a1 as float.  FP64: meta = cell
// lane | 0x80 for a single-point beam, node = the global index of the first
// node, then a0, a1 as double: 24 bytes.  The spread reads every form into
// the 16-byte layout (meta, node, a0 bits, a1 bits or the FP64 a0).
constexpr uint32_t kRecSingle = 0x80u;
constexpr int kRecNodeShift = 7;                    // node above the lane and single bit (12-byte form)
constexpr int64_t kRecCompactPoints = 1ll << 25;    // the 12-byte form holds node indices below this
__host__ __device__ inline int rec_size(int prec, bool compact) {
  return prec == ALP_PREC_FP32_SPLIT ? (compact ? 12 : 16) : 24;
}

// A window grouped by tile: the tile is implied by the position; k0 is the
// beam's first point (case-local) and hi < 0 marks a single-point beam.
struct Win {
  int32_t beam;   // global beam index
  int32_t lo, hi; // candidate segments (beam-local)
  int32_t k0;
};

// A merged window: the candidate segments i0..i1 of one beam for one tile
// (every window of that beam in the tile joined), written by the tile merge.
struct Entry {
  int32_t k0;      // first point of the beam (case-local point index)
  int32_t i0, i1;  // beam-local segment range
  int32_t single;  // 1: single-point beam (point kernel about its only node)
};

struct Item {
  int32_t tile;   // global tile index
  int32_t c0, c1; // sorted cell range
  int32_t cs;     // case index
  uint32_t eoff;  // first entry of the tile
  uint32_t nent;  // entries of the tile (beam order)
};

// Per-step workspace (device pointers), sized by the host.
struct Work {
  // points (global index)
  int32_t *pbeam;       // point -> global beam
  int32_t *pflags;      // sampling flags
  int32_t *wexp;        // per-node fixed-point exponent
  long long *w_hi;      // per-node fixed-point accumulators
  unsigned long long *w_lo;
  double *fhat;         // [N_P][3]
  double *Us;           // [N_P][3] internal sampled velocity
  double *Ps;           // [N_P][3] internal sampling point
  double *As;           // [N_P][3] fluid acceleration sampled at P_s (eq. 8)
  double *f;            // [N_P][3] internal force (when the case has none)
  // beams (global)
  int32_t *bcase;       // beam -> case
  double *beps_max;     // beam max eps
  uint32_t *bchunks;    // chunks per beam, then exclusive scan ([N_B+1])
  // chunks
  int32_t *chunk_beam, *chunk_s0, *chunk_s1;
  uint32_t *chunk_box;  // tiles in each chunk's box, scanned into slot offsets ([cap_chunk+1])
  int32_t *chunk_bx;    // each chunk's tile box: lo x, y, z, hi x, y, z ([cap_chunk][6])
  // tiles (global)
  uint32_t *tile_cnt;   // windows per tile ([N_T+1])
  uint32_t *tile_off;   // exclusive scan of tile_cnt ([N_T+1])
  uint32_t *tile_fill;
  uint32_t *tile_nent;  // merged entries per tile ([N_T+1])
  uint32_t *tile_items; // work items per tile ([N_T+1])
  uint32_t *tile_itoff; // exclusive scan of tile_items ([N_T+1])
  uint32_t *big_tiles;  // tiles for k_tile_merge_big ([N_T]; count in counters[kBigTileCounter])
  // lists
  Emit *emit_raw;       // [cap_emit] one slot per (chunk, box tile); beam < 0 = empty
  Win *emit;            // [cap_emit] windows grouped by tile
  Entry *entry;         // [cap_emit] merged windows, at the tile's window offset
  Item *item;           // [cap_item]
  uint32_t *multi_items; // [cap_item] items taken in entry groups (more than kMaxEntries entries,
                         // or more window points than the staging area)
  unsigned long long *rec_base;  // per item, byte offset into rec
  uint32_t *rec_cnt;    // per item
  unsigned char *rec;   // [cap_rec bytes] pair records
  unsigned long long *rec_alloc; // byte allocator
  // per-case reductions
  long long *F_hi;      // [n_cases][3]
  unsigned long long *F_lo;
  int32_t *F_exp;       // [n_cases]
  double *beam_part;    // [n_pblocks][4] (F_beam xyz, sum |f L|)
  int32_t *pblock_case; // [n_pblocks]
  int64_t *pblock_range;// [n_pblocks][2]
  long long *cnt;       // [n_cases][kCnt] counters: outside, fallback, degenerate, zero w, band, pairs,
                        // invalid, empty kernel sample, FP64 guard
  double *diag_out;     // [n_cases][16] finalised diagnostics
  // scalars
  uint32_t *counters;   // [kCounters]: [3] overflow flags; from queue_words(q) the weights work
                        // queues q = 0 nearest split, 1 integrated split, 2 integrated FP64,
                        // 3 nearest FP64 (counter x of a queue at word x * kLineWords)
  uint32_t *scan_tmp;   // scan block totals (host-side launch use only)
  int64_t cap_emit, cap_item, cap_rec, cap_chunk;
  int64_t n_points, n_beams, n_tiles;
  int32_t rec_compact;  // split-precision pair records in the 12-byte form (n_points < 2^25)
  int32_t n_cases, n_pblocks;
};

// ----------------------------------------------------------------- helpers --
// Decision arithmetic (nearest cell, nearest segment, cutoff): the one
// evaluation order dot(a,b) = (ax bx + ay by) + az bz, IEEE operations, no
// contraction into fused multiply-adds, so that every decision is bitwise
// reproducible on any IEEE FP64 machine.
__device__ __forceinline__ double dot3_exact(double ax, double ay, double az, double bx, double by,
                                             double bz) {
#pragma clang fp contract(off)
  return (ax * bx + ay * by) + az * bz;
}

// Closest point of segment [A, B] to C (eq. 21): foot parameter s in [0, 1]
// (0 for a zero-length segment) and squared distance r2.
__device__ __forceinline__ void seg_foot(double cx, double cy, double cz, double ax, double ay,
                                         double az, double bx, double by, double bz, double &s,
                                         double &r2) {
#pragma clang fp contract(off)
  double ex = bx - ax, ey = by - ay, ez = bz - az;
  double qx = cx - ax, qy = cy - ay, qz = cz - az;
  double t = (qx * ex + qy * ey) + qz * ez;
  double ee = (ex * ex + ey * ey) + ez * ez;
  double u = 0.0;
  if (ee > 0.0) {
    u = t / ee;
    if (u < 0.0) u = 0.0;
    if (u > 1.0) u = 1.0;
  }
  double px = qx - u * ex, py = qy - u * ey, pz = qz - u * ez;
  r2 = (px * px + py * py) + pz * pz;
  s = u;
}

__device__ __forceinline__ double sqdist_exact(double cx, double cy, double cz, double ax, double ay,
                                               double az) {
#pragma clang fp contract(off)
  double qx = cx - ax, qy = cy - ay, qz = cz - az;
  return (qx * qx + qy * qy) + qz * qz;
}

// Kernel width at the foot point (per-point eps interpolated with the linear
// weights) and the inclusive 3 eps cutoff, evaluated in FP64.
__device__ __forceinline__ double eps_at(double s, double e0, double e1) {
#pragma clang fp contract(off)
  return (1.0 - s) * e0 + s * e1;
}
__device__ __forceinline__ bool inside_cutoff(double r2, double ej) {
#pragma clang fp contract(off)
  return r2 <= 9.0 * (ej * ej);
}

// Truncated 2D Gaussian of eq. (22) times the linear weights of Sec. 3.2.4:
// a0 = (1 - s) eta, a1 = s eta.  In the split precision eta and the weights
// are FP32 (the values are then widened to FP64 for every product and sum).
// Both projection passes call this with identical arguments, so the weights
// that build w_k and the ones that build S are bit-identical.
__device__ __forceinline__ void pair_weights(int prec, double s, double r2, double ej, double &a0,
                                             double &a1) {
  if (prec == ALP_PREC_FP32_SPLIT) {
    const float e2 = (float)(ej * ej);
    const float ie2 = __builtin_amdgcn_rcpf(e2);  // one reciprocal (1 ulp) serves both quotients
    const float x = (float)r2 * ie2;
    // exp(-x) as the hardware 2^y of y = -x log2(e): with 0 <= x <= 9 inside
    // the cutoff, the rounding of y (|y| < 13) moves the result by at most
    // 13 ln2 2^-24 < 6e-7 relative, and the instruction adds about one ulp
    const float eta = __builtin_amdgcn_exp2f(x * -1.44269504088896340736f) *
                      (ie2 * 0.318309886183790671538f);  // 1/pi
    float sf = (float)s;
    a0 = (double)((1.0f - sf) * eta);
    a1 = (double)(sf * eta);
  } else {
    double e2 = ej * ej;
    double eta = exp(-(r2 / e2)) / (3.14159265358979323846 * e2);
    a0 = (1.0 - s) * eta;
    a1 = s * eta;
  }
}

// Segment-integrated weights (ALP_PROJ_INTEGRATED): the 3D Gaussian
// g(x) = exp(-|x|^2/eps^2) / (pi^1.5 eps^3) integrated along the segment
// [A, B] (length l > 0) against the linear weights 1 - u/l (node i, a0) and
// u/l (node i+1, a1).  With tau the unclamped foot parameter, r_p the distance
// to the line and t = tau l, the Gaussian factors into a radial and an axial
// part; with x0 = -t/eps, x1 = (l - t)/eps and lam = l/eps,
//   a0 = Q (x1 E - M) / lam,  a1 = Q (M - x0 E) / lam,
//   E = (sqrt(pi)/2)(erf x1 - erf x0),  M = (exp(-x0^2) - exp(-x1^2)) / 2,
//   Q = exp(-r_p^2/eps^2) / (pi^1.5 eps^2).
// The erf difference is taken through erfc on the side where both arguments
// share a sign, the exponential difference through expm1.  Below lam = 1/8 the
// two terms of each bracket nearly cancel, and the integral is taken instead
// by 8-point Gauss-Legendre quadrature in s = u/l, whose error there is far
// below rounding.  Always FP64; the split precision narrows the results.
namespace gl8 {
// Gauss-Legendre abscissae and weights for n = 8 on [-1, 1] (the tabulated
// values of the rule, Abramowitz and Stegun Table 25.4), mapped to [0, 1].
constexpr double kX[4] = {0.1834346424956498049, 0.5255324099163289858, 0.7966664774136267396,
                          0.9602898564975362317};
constexpr double kW[4] = {0.3626837833783619830, 0.3137066458778872873, 0.2223810344533744706,
                          0.1012285362903762592};
}  // namespace gl8

__device__ __forceinline__ void seg_int_weights(double cx, double cy, double cz, double ax, double ay,
                                                double az, double bx, double by, double bz, double eps,
                                                double &a0, double &a1) {
#pragma clang fp contract(off)
  const double ex = bx - ax, ey = by - ay, ez = bz - az;
  const double qx = cx - ax, qy = cy - ay, qz = cz - az;
  const double ee = (ex * ex + ey * ey) + ez * ez, l = sqrt(ee);
  const double tau = ((qx * ex + qy * ey) + qz * ez) / ee;
  const double px = qx - tau * ex, py = qy - tau * ey, pz = qz - tau * ez;
  const double rp2 = (px * px + py * py) + pz * pz, t = tau * l;
  // one reciprocal for the four quotients by eps (last-ulp differences only)
  const double ie = 1.0 / eps;
  const double x0 = -t * ie, x1 = (l - t) * ie, lam = l * ie;
  const double kPi = 3.14159265358979323846, kSqrtPi = 1.77245385090551602730;
  const double Q = exp(-(rp2 * (ie * ie))) * (ie * ie) * (1.0 / (kPi * kSqrtPi));
  double W0 = 0.0, W1 = 0.0;
  if (lam < 0.125) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double x = k < 4 ? -gl8::kX[3 - k] : gl8::kX[k - 4];
      const double w = 0.5 * (k < 4 ? gl8::kW[3 - k] : gl8::kW[k - 4]);
      const double sq = 0.5 * (1.0 + x);
      const double y = sq * lam + x0, g = w * exp(-(y * y));
      W0 += (1.0 - sq) * g;
      W1 += sq * g;
    }
    W0 *= lam;
    W1 *= lam;
  } else {
    double D;
    if (x0 >= 0.0) D = erfc(x0) - erfc(x1);
    else if (x1 <= 0.0) D = erfc(-x1) - erfc(-x0);
    else D = erf(x1) - erf(x0);
    const double d = (x1 - x0) * (x1 + x0);  // x1^2 - x0^2
    const double dexp = d >= 0.0 ? -exp(-(x0 * x0)) * expm1(-d) : exp(-(x1 * x1)) * expm1(d);
    const double E = 0.5 * kSqrtPi * D, M = 0.5 * dexp;
    W0 = (x1 * E - M) / lam;
    W1 = (M - x0 * E) / lam;
  }
  a0 = Q * W0;
  a1 = Q * W1;
}

// The same weights under the split precision: the geometry (foot, axial and
// radial distances, each divided by eps) in FP64, the Gaussian integrals in
// FP32.  Below lam = 2 the 8-point Gauss-Legendre rule is exact to FP32
// rounding and avoids the cancellation of the closed form; above it the
// closed form loses at most a few FP32 ulps.  x1 is formed in FP64 so the
// cancellation in x0 + lam never reaches the far-end erf.  Relative error
// against the FP64 evaluation: below 2e-6 of a0 + a1.
__device__ __forceinline__ void seg_int_weights_split(double cx, double cy, double cz, double ax, double ay,
                                                      double az, double bx, double by, double bz, double eps,
                                                      double &a0, double &a1) {
#pragma clang fp contract(off)
  const double ex = bx - ax, ey = by - ay, ez = bz - az;
  const double qx = cx - ax, qy = cy - ay, qz = cz - az;
  const double ee = (ex * ex + ey * ey) + ez * ez, l = sqrt(ee);
  const double tau = ((qx * ex + qy * ey) + qz * ez) / ee;
  const double px = qx - tau * ex, py = qy - tau * ey, pz = qz - tau * ez;
  const double rp2 = (px * px + py * py) + pz * pz, t = tau * l;
  const double ie = 1.0 / eps;  // one reciprocal for the quotients by eps
  const float x0 = (float)(-t * ie), x1 = (float)((l - t) * ie), lam = (float)(l * ie);
  const float rr = (float)(rp2 * (ie * ie));
  const float Q = expf(-rr) * (float)((ie * ie) * (1.0 / (3.14159265358979323846 * 1.77245385090551602730)));
  float W0 = 0.0f, W1 = 0.0f;
  if (lam < 2.0f) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float w = (float)(0.5 * (k < 4 ? gl8::kW[3 - k] : gl8::kW[k - 4]));
      const float sq = (float)(0.5 * (1.0 + (k < 4 ? -gl8::kX[3 - k] : gl8::kX[k - 4])));
      const float y = sq * lam + x0, g = w * expf(-(y * y));
      W0 += (1.0f - sq) * g;
      W1 += sq * g;
    }
    W0 *= lam;
    W1 *= lam;
  } else {
    float D;
    if (x0 >= 0.0f) D = erfcf(x0) - erfcf(x1);
    else if (x1 <= 0.0f) D = erfcf(-x1) - erfcf(-x0);
    else D = erff(x1) - erff(x0);
    const float d = (x1 - x0) * (x1 + x0);
    const float dexp = d >= 0.0f ? -expf(-(x0 * x0)) * expm1f(-d) : expf(-(x1 * x1)) * expm1f(d);
    const float E = 0.88622692545275801365f * D, M = 0.5f * dexp;
    W0 = (x1 * E - M) / lam;
    W1 = (M - x0 * E) / lam;
  }
  a0 = (double)(Q * W0);
  a1 = (double)(Q * W1);
}

// Exact fixed-point accumulation (order independent, so deterministic under
// any work distribution or atomic order).  A non-negative or signed value v
// with |v| < 2^E is split into hi = floor(v 2^(46-E)) and
// lo = floor(frac * 2^40); both are summed as 64-bit integers.
// Both parts are integers below 2^51 in magnitude, so adding 1.5 * 2^52 puts
// them in the low mantissa bits exactly and an integer subtraction of the
// constant's bit pattern converts them.
__device__ __forceinline__ void fx_encode(double v, int E, long long &hi, unsigned long long &lo) {
  const double kMagic = 6755399441055744.0;  // 1.5 * 2^52
  const long long kMagicBits = 0x4338000000000000ll;
  double t = ldexp(v, kHiShift - E);
  double th = floor(t);
  double r = t - th;  // exact, in [0, 1)
  double tl = floor(ldexp(r, kLoBits));
  hi = __double_as_longlong(th + kMagic) - kMagicBits;
  lo = (unsigned long long)(__double_as_longlong(tl + kMagic) - kMagicBits);
}
__device__ __host__ inline double fx_decode(long long hi, unsigned long long lo, int E) {
  hi += (long long)(lo >> kLoBits);
  lo &= ((1ull << kLoBits) - 1ull);
  return ldexp((double)hi, E - kHiShift) + ldexp((double)lo, E - kHiShift - kLoBits);
}

// Loads of values that no kernel of the pass writes (work-item tables, the
// case table) through the scalar unit: a wave-uniform address then costs no
// vector-memory slot, and the wait for it does not also wait for vector
// loads, stores or atomics in flight.
template <class T>
__device__ __forceinline__ T sload(const T *p) {
  return *(const __attribute__((address_space(4))) T *)(p);
}
__device__ __forceinline__ Item sload_item(const Item *p) {
  Item it;
  it.tile = sload(&p->tile);
  it.c0 = sload(&p->c0);
  it.c1 = sload(&p->c1);
  it.cs = sload(&p->cs);
  it.eoff = sload(&p->eoff);
  it.nent = sload(&p->nent);
  return it;
}
// the mesh fields of the tile geometry and the sorted cell arrays (the other
// fields are left zero)
__device__ __forceinline__ MeshDev sload_mesh_geometry(const MeshDev *p) {
  MeshDev m = {};
  m.T = sload(&p->T);
  for (int a = 0; a < 3; ++a) {
    m.nb[a] = sload(&p->nb[a]);
    m.nt[a] = sload(&p->nt[a]);
    m.lo[a] = sload(&p->lo[a]);
  }
  m.tile_len = sload(&p->tile_len);
  m.cx = sload(&p->cx);
  m.cy = sload(&p->cy);
  m.cz = sload(&p->cz);
  m.vs = sload(&p->vs);
  return m;
}

// Centre of tile (tx, ty, tz): (lo + t tile_len) + tile_len / 2 per axis, in
// this one evaluation order (no contraction), so that every kernel that
// forms coordinates relative to it gets the same FP64 value.
__device__ __host__ inline void tile_centre(const MeshDev &m, int tx, int ty, int tz, double *c) {
#pragma clang fp contract(off)
  const double h = 0.5 * m.tile_len;
  c[0] = (m.lo[0] + (double)tx * m.tile_len) + h;
  c[1] = (m.lo[1] + (double)ty * m.tile_len) + h;
  c[2] = (m.lo[2] + (double)tz * m.tile_len) + h;
}

// bin key: tiles in x-fastest order, then bins inside the tile x-fastest
__device__ __host__ inline uint32_t bin_key(const MeshDev &m, int ix, int iy, int iz) {
  int T = m.T;
  int tx = ix / T, ty = iy / T, tz = iz / T;
  int lx = ix - tx * T, ly = iy - ty * T, lz = iz - tz * T;
  uint32_t tile = (uint32_t)((tz * m.nt[1] + ty) * m.nt[0] + tx);
  return tile * (uint32_t)(T * T * T) + (uint32_t)((lz * T + ly) * T + lx);
}

// A read-only pointer into device global memory.  Loads through it compile to
// global memory instructions rather than flat ones, so that waits for them
// and waits for LDS operations stay independent.
template <class T>
using gptr = const __attribute__((address_space(1))) T *;
template <class T>
__device__ __forceinline__ gptr<T> to_global(const T *p) {
  return (gptr<T>)p;
}

__device__ __forceinline__ int case_of(const int64_t *bases, int n, int64_t idx) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (bases[mid] <= idx) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// ------------------------------------------------------------- launchers --
// (defined in the kernel translation units)
void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t st);
int64_t scan_tmp_words(int64_t n);
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t st);
void launch_fill_i64(long long *p, long long v, int64_t n, hipStream_t st);

// mesh binning
void launch_mesh_bounds(const double *C, const double *V, int64_t n, double *part, int nblk,
                        hipStream_t st);
int mesh_bounds_blocks(int64_t n);
void launch_bin_keys(const MeshDev &m, const double *C, int64_t n, uint32_t *key, uint32_t *count,
                     hipStream_t st);
int64_t radix_scratch_words(int64_t n);
void launch_radix_sort(const uint32_t *key, int64_t n, int64_t n_bins, uint32_t *perm, uint32_t *ksorted,
                       uint32_t *k2, uint32_t *v2, uint32_t *cnt, uint32_t *tmp, hipStream_t st);
void launch_bin_check(const uint32_t *key, const uint32_t *ksorted, const uint32_t *perm, const uint32_t *start,
                      int64_t n, uint32_t *bad, hipStream_t st);
void launch_bin_reorder(const double *C, const double *V, const uint32_t *sorted, int64_t n, double *cxyz,
                        double *cx, double *cy, double *cz, double *vs, hipStream_t st);

// step
struct StepLaunch {
  const CaseDev *cases;    // device
  const int64_t *pbase;    // device [n_cases+1] point bases
  const int64_t *bbase;    // device [n_cases+1] beam bases
  const int64_t *tbase;    // device [n_cases+1] tile bases
  Work w;
  int n_cases;
  int grid_persistent;     // blocks for persistent wave kernels
  int grid_spread;         // blocks of the spread pass: one per resident wave slot
  int kernel_sample;       // some case uses ALP_SAMPLE_KERNEL
  int sample_waves;        // sampler waves per CU (0: one wave per 64 / lanes points, no cap)
  int sample_lanes;        // lanes per point in the sampler (2, 4 or 8)
  int weights_grab;        // work items a weights wave takes from its queue at once
  int grid_weights;        // blocks (one wave each) of the weights kernels
  int near_split, near_fp64;  // some case projects with ALP_PROJ_NEAREST in that precision
  int int_split, int_fp64;    // some case projects with ALP_PROJ_INTEGRATED in that precision
};
void launch_step_reset(const StepLaunch &L, hipStream_t st);
void launch_step_reset_sample(const StepLaunch &L, hipStream_t st);
void launch_step_reset_project(const StepLaunch &L, hipStream_t st);
void launch_drag_mode(const StepLaunch &L, int use_cell_s, hipStream_t st);
void launch_points_prep(const StepLaunch &L, hipStream_t st);
void launch_beams_prep(const StepLaunch &L, hipStream_t st);
void launch_chunks(const StepLaunch &L, hipStream_t st);
void launch_chunk_boxes(const StepLaunch &L, hipStream_t st);
void launch_chunk_tiles(const StepLaunch &L, hipStream_t st);
void launch_emit_scatter(const StepLaunch &L, hipStream_t st);
void launch_tile_merge(const StepLaunch &L, hipStream_t st);
void launch_items(const StepLaunch &L, hipStream_t st);
void launch_sample(const StepLaunch &L, hipStream_t st);
// Point-wise beam geometry ahead of a step (alp_beam_geometry).
struct GeomLaunch {
  MeshDev m;
  int32_t n_beams, reserved;
  int64_t n_points;
  const int64_t *offsets;
  const double *Cb, *Wref, *W, *eps_phys;
  double factor;
  double *P, *e_t, *eps;
  unsigned long long *counts;  // [2]: zero tangents, points outside (or null)
};
void launch_beam_geometry(const GeomLaunch &G, hipStream_t st);
void launch_sample_kernel(const StepLaunch &L, hipStream_t st);
void launch_drag(const StepLaunch &L, hipStream_t st);
void launch_weights_main(const StepLaunch &L, hipStream_t st);
void launch_weights_grouped(const StepLaunch &L, hipStream_t st);
void launch_norm(const StepLaunch &L, hipStream_t st);
void launch_beam_sums(const StepLaunch &L, hipStream_t st);
void launch_spread(const StepLaunch &L, hipStream_t st);
int spread_blocks_per_cu();  // resident k_spread blocks per CU (0 if the query fails)
void launch_step_end(const StepLaunch &L, uint32_t *ovf_dst, hipStream_t st);
// copy the step's overflow word to a device-visible host word

}  // namespace alp
