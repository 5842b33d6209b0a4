// alp_step.hip -- the per-step kernels of the coupling operator (gfx950).
//
// One step of a batch runs, over the concatenated work of every case:
//   reset, points_prep, beams_prep, chunks, chunk_tiles, scan, emit_scatter,
//   tile_merge, scan, items                       [segment binning]
//   sample, drag                                    [eq. 16-20]
//   weights, norm, beam_sums                        [eq. 21-22, nodal weights]
//   spread, zero_dirty, finalize                    [eq. 23, eq. 14 check]
//
// Work lists live on the device; the kernels that walk them are persistent
// (fixed grids that loop), so a step can be captured in a hipGraph once and
// replayed.  No floating-point atomics are used: nodal weights and the force
// balance are accumulated as exact fixed-point integers, and every source
// value is summed by one lane in beam order.
#include "alp_internal.h"
#include "alp_keys.h"
#include "alp_reccursor.h"

namespace alp {

// ------------------------------------------------------------------ utils --
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

__device__ __forceinline__ uint32_t lanemask_lt_popc(uint64_t m) {
  int lane = lane_id();
  uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  return (uint32_t)__popcll(m & lt);
}

__device__ __forceinline__ uint32_t wave_excl_scan_u32(uint32_t v, uint32_t &total) {
  int lane = lane_id();
  uint32_t inc = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(inc, d, 64);
    if (lane >= d) inc += t;
  }
  total = __shfl(inc, 63, 64);
  return inc - v;
}

// lane 0's value in a scalar register (the value is the same for the wave)
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// deterministic wave sum (fixed butterfly order)
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__device__ __forceinline__ void wave_count_add(long long *dst, bool pred) {
  uint64_t m = ballot64(pred);
  if (lane_id() == 0 && m) atomicAdd((unsigned long long *)dst, (unsigned long long)__popcll(m));
}

__device__ __forceinline__ void set_overflow(Work &W, uint32_t bit) { atomicOr(&W.counters[3], bit); }

// Dynamic work distribution for a persistent kernel: work items are cut into
// chunks of `grab` consecutive items.  A wave's first chunk is its block index
// (no atomic, so idle waves of a small step leave at once); later chunks come
// from one of kQueueStripes counters (block index mod kQueueStripes, so the
// counters share the load; each sits on its own cache line): chunk
// G + S q + x for the q-th grab on counter x, G the grid size and S the
// number of counters.  The counters start at zero every step; a wave leaves
// once a chunk past the end comes back.
struct WorkQueue {
  uint32_t *ctr;  // counter x at ctr[x * kLineWords]
  uint32_t n, grab, x, item, end;
  bool started;
  __device__ bool next(int lane) {
    if (item + 1 < end) {
      ++item;
      return true;
    }
    uint64_t chunk;
    if (!started) {
      started = true;
      chunk = blockIdx.x;
    } else {
      uint32_t q = 0;
      if (lane == 0) q = atomicAdd(&ctr[x * kLineWords], 1u);
      q = __shfl(q, 0, 64);
      chunk = (uint64_t)gridDim.x + (uint64_t)q * kQueueStripes + x;
    }
    const uint64_t first = chunk * grab;
    if (first >= n) return false;
    item = (uint32_t)first;
    end = (uint32_t)min((uint64_t)n, first + grab);
    return true;
  }
};
__device__ __forceinline__ WorkQueue work_queue(uint32_t *ctr, uint32_t n, uint32_t grab) {
  WorkQueue q;
  q.ctr = ctr;
  q.n = n;
  q.grab = grab;
  q.x = blockIdx.x % (uint32_t)kQueueStripes;
  q.item = 0;
  q.end = 0;
  q.started = false;
  return q;
}

// tile (tx, ty, tz) of a case-local linear tile index
__device__ __forceinline__ void tile_xyz(const MeshDev &m, int64_t tl, int &tx, int &ty, int &tz) {
  // tile counts are below 2^32 (bin keys are 32-bit)
  const uint32_t t = (uint32_t)tl, nx = (uint32_t)m.nt[0], ny = (uint32_t)m.nt[1];
  const uint32_t r = t / nx;
  tx = (int)(t - r * nx);
  tz = (int)(r / ny);
  ty = (int)(r - (uint32_t)tz * ny);
}

__device__ __forceinline__ uint32_t tile_cell_start(const MeshDev &m, int64_t tl) {
  return m.bin_start[tl * (int64_t)(m.T * m.T * m.T)];
}

// ------------------------------------------------------------------ reset --
enum { RESET_SAMPLE = 1, RESET_PROJECT = 2 };

__global__ void k_step_reset(StepLaunch L, int what) {
  Work W = L.w;
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid < kCounters && (what & RESET_PROJECT)) W.counters[tid] = 0;
  if (tid == 0 && (what & RESET_PROJECT)) *W.rec_alloc = 0;
  for (int64_t c = tid; c < (int64_t)L.n_cases * kCnt; c += stride) {
    int k = (int)(c % kCnt);
    bool samp = k < 3 || k == 7;
    if ((samp && (what & RESET_SAMPLE)) || (!samp && (what & RESET_PROJECT))) W.cnt[c] = 0;
  }
  if (!(what & RESET_PROJECT)) return;
  for (int64_t c = tid; c < (int64_t)L.n_cases * 3; c += stride) {
    W.F_hi[c] = 0;
    W.F_lo[c] = 0;
  }
  for (int64_t i = tid; i < W.n_points; i += stride) {
    W.w_hi[i] = 0;
    W.w_lo[i] = 0;
  }
  for (int64_t i = tid; i < W.n_tiles; i += stride) {
    W.tile_cnt[i] = 0;
    W.tile_fill[i] = 0;
  }
}

void launch_step_reset(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_step_reset, dim3(1024), dim3(256), 0, st, L, (int)(RESET_SAMPLE | RESET_PROJECT));
}
void launch_step_reset_sample(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(256), 0, st, L, (int)RESET_SAMPLE);
}
void launch_step_reset_project(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_step_reset, dim3(1024), dim3(256), 0, st, L, (int)RESET_PROJECT);
}

// ------------------------------------------------------------ points prep --
// point -> beam map and the per-node fixed-point exponent: every contribution
// a V to node k is below V_max / (pi eps_min^2), eps_min over the node and its
// neighbours on the beam (the kernel width at a foot point interpolates them).
__global__ void k_points_prep(StepLaunch L) {
  Work W = L.w;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= W.n_points) return;
  int c = case_of(L.pbase, L.n_cases, g);
  const CaseDev &cs = L.cases[c];
  int64_t k = g - cs.point_base;
  int lo = 0, hi = cs.n_beams - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (cs.offsets[mid] <= k) lo = mid;
    else hi = mid - 1;
  }
  W.pbeam[g] = (int32_t)(cs.beam_base + lo);
  int64_t k0 = cs.offsets[lo], k1 = cs.offsets[lo + 1];
  double em = cs.eps[k];
  if (k > k0) em = fmin(em, cs.eps[k - 1]);
  if (k + 1 < k1) em = fmin(em, cs.eps[k + 1]);
  double bound = cs.m.vmax / (3.14159265358979323846 * em * em);
  W.wexp[g] = (bound > 0.0 && bound < INFINITY) ? ilogb(bound) + 2 : 0;
  const double *et = cs.e_t + 3 * k;
  double tt = et[0] * et[0] + et[1] * et[1] + et[2] * et[2];
  if (!(cs.eps[k] > 0.0 && cs.eps[k] < INFINITY) || !(tt > 0.0 && tt < INFINITY))
    atomicAdd((unsigned long long *)(W.cnt + kCnt * c + 6), 1ull);
}

void launch_points_prep(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_points == 0) return;
  hipLaunchKernelGGL(k_points_prep, dim3((unsigned)((L.w.n_points + 255) / 256)), dim3(256), 0, st, L);
}

// ------------------------------------------------------------- beams prep --
// One wave per beam: case index, chunk count and the largest kernel width of
// the beam (a max is exact in any order).
__global__ __launch_bounds__(256) void k_beams_prep(StepLaunch L) {
  Work W = L.w;
  const int lane = lane_id();
  const int64_t gb = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (gb >= W.n_beams) return;  // uniform per wave
  const int c = case_of(L.bbase, L.n_cases, gb);
  const CaseDev &cs = L.cases[c];
  const int64_t b = gb - cs.beam_base;
  const int64_t k0 = cs.offsets[b], k1 = cs.offsets[b + 1];
  double em = 0.0;
  for (int64_t k = k0 + lane; k < k1; k += 64) em = fmax(em, cs.eps[k]);
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) em = fmax(em, __shfl_xor(em, d, 64));
  if (lane == 0) {
    const int64_t n = k1 - k0;
    const int64_t nseg = n >= 2 ? n - 1 : n;
    W.bcase[gb] = c;
    W.beps_max[gb] = em;
    W.bchunks[gb] = (uint32_t)((nseg + kChunkSegs - 1) / kChunkSegs);
  }
}

void launch_beams_prep(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_beams == 0) return;
  hipLaunchKernelGGL(k_beams_prep, dim3((unsigned)((L.w.n_beams + 3) / 4)), dim3(256), 0, st, L);
}

// ----------------------------------------------------------------- chunks --
__global__ void k_chunks(StepLaunch L, const uint32_t *choff) {
  Work W = L.w;
  int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gb >= W.n_beams) return;
  const CaseDev &cs = L.cases[W.bcase[gb]];
  int64_t b = gb - cs.beam_base;
  int64_t n = cs.offsets[b + 1] - cs.offsets[b];
  int64_t nseg = n >= 2 ? n - 1 : n;
  uint32_t o = choff[gb];
  for (int64_t s0 = 0, j = 0; s0 < nseg; s0 += kChunkSegs, ++j) {
    int64_t id = (int64_t)o + j;
    if (id >= W.cap_chunk) {
      set_overflow(W, 16u);
      return;
    }
    W.chunk_beam[id] = (int32_t)gb;
    W.chunk_s0[id] = (int32_t)s0;
    W.chunk_s1[id] = (int32_t)(s0 + kChunkSegs - 1 < nseg - 1 ? s0 + kChunkSegs - 1 : nseg - 1);
  }
}

void launch_chunks(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_beams == 0) return;
  hipLaunchKernelGGL(k_chunks, dim3((unsigned)((L.w.n_beams + 255) / 256)), dim3(256), 0, st, L,
                     (const uint32_t *)L.w.bchunks);
}

// ------------------------------------------------------------ chunk tiles --
// For every chunk of consecutive segments, the tiles for which one of its
// segments can be the closest segment of the beam for some point of the tile
// and lies within 3 eps_max of it:
//   (a) the segment's AABB inflated by 3 eps_max(beam) overlaps the tile, and
//   (b) slab rule: segment i is never the closest segment of a point that is
//       behind its start plane while in front of the previous segment's end
//       plane (the previous segment is strictly closer), nor of a point beyond
//       its end plane while in front of the next segment's start plane (the
//       next segment is strictly closer).  Where both neighbouring segments
//       clamp to their shared vertex the two distances are equal in exact
//       arithmetic and the FP64 rounding of eq. (21) decides, so both stay
//       candidates there; the planes carry a margin of 1e-7 (tile + R) so that
//       "strictly closer" survives rounding.
// The window [first, last] candidate segment of the chunk is appended for
// every such tile, and counted per tile for the grouping scatter.
struct SegInfo {
  double lo[3], hi[3];  // inflated AABB
  double a[3];          // start point
  double u[3];          // unit direction (0 for a zero-length segment)
  double len, su;       // length, |ux| + |uy| + |uz|
};

// reach of a chunk's beam: 3 eps_max, widened by 1e-7 (tile + reach) so that
// the tile tests below survive rounding
__device__ __forceinline__ double chunk_reach(const Work &W, int gb, double tl) {
  const double R = 3.0 * W.beps_max[gb];
  return R + 1e-7 * (tl + R);
}

// tile box of a chunk: tiles overlapped by the union of its segments' AABBs
// inflated by the reach; returns false when the box misses the tile grid.
// The points are read one after another: this keeps the kernel small in
// registers, so that it finds room beside the sampling kernel, which runs
// concurrently on the other stream (loading them all at once made the
// overlapped step slower).
__device__ bool chunk_box(const StepLaunch &L, int64_t ch, int32_t *box) {
  const Work &W = L.w;
  const int gb = W.chunk_beam[ch];
  const CaseDev &cs = L.cases[W.bcase[gb]];
  const MeshDev &m = cs.m;
  const int64_t b = gb - cs.beam_base;
  const int64_t k0 = cs.offsets[b];
  const int nb = (int)(cs.offsets[b + 1] - k0);
  const int s0 = W.chunk_s0[ch], s1 = W.chunk_s1[ch];
  const double *X = cs.Psp + 3 * k0;
  const double tl = m.tile_len;
  const double R = chunk_reach(W, gb, tl);
  const int pfirst = nb >= 2 ? s0 : 0, plast = nb >= 2 ? s1 + 1 : 0;
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int p = pfirst; p <= plast; ++p)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], X[3 * p + a]);
      hi[a] = fmax(hi[a], X[3 * p + a]);
    }
  bool ok = true;
  for (int a = 0; a < 3; ++a) {
    double f0 = floor((lo[a] - R - m.lo[a]) / tl), f1 = floor((hi[a] + R - m.lo[a]) / tl);
    if (!(f1 >= 0.0) || !(f0 <= (double)(m.nt[a] - 1))) ok = false;  // also rejects NaN
    box[a] = !(f0 > 0.0) ? 0 : (int)f0;
    box[3 + a] = f1 > (double)(m.nt[a] - 1) ? m.nt[a] - 1 : (f1 > 0.0 ? (int)f1 : 0);
  }
  return ok;
}

// tiles in each chunk's box (0 when it misses the grid), and the box itself
__global__ void k_chunk_boxes(StepLaunch L) {
  const Work &W = L.w;
  const int64_t ch = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ch >= W.cap_chunk) return;
  uint32_t n = 0;
  if (ch < (int64_t)W.bchunks[W.n_beams]) {
    int32_t box[6];
    if (chunk_box(L, ch, box)) {
      n = (uint32_t)((box[3] - box[0] + 1) * (box[4] - box[1] + 1) * (box[5] - box[2] + 1));
      int32_t *o = W.chunk_bx + 6 * ch;
      for (int a = 0; a < 6; ++a) o[a] = box[a];
    }
  }
  W.chunk_box[ch] = n;
}

void launch_chunk_boxes(const StepLaunch &L, hipStream_t st) {
  if (L.w.cap_chunk == 0) return;
  hipLaunchKernelGGL(k_chunk_boxes, dim3((unsigned)((L.w.cap_chunk + 255) / 256)), dim3(256), 0, st, L);
}

__global__ __launch_bounds__(64) void k_chunk_tiles(StepLaunch L) {
  Work W = L.w;
  __shared__ SegInfo sg[kChunkSegs + 2];  // [0]: the segment before the chunk, [nsg + 1]: after
  const int lane = threadIdx.x;
  const uint32_t n_chunks = W.bchunks[W.n_beams];
  const uint32_t *box_off = W.chunk_box;  // exclusive scan of the box sizes
  for (int64_t ch = blockIdx.x; ch < (int64_t)n_chunks && ch < W.cap_chunk; ch += gridDim.x) {
    const uint32_t slot0 = box_off[ch];
    const int64_t ntile = (int64_t)box_off[ch + 1] - slot0;
    if (ntile == 0) continue;
    int32_t box[6];
    for (int a = 0; a < 6; ++a) box[a] = W.chunk_bx[6 * ch + a];
    const int gb = __builtin_amdgcn_readfirstlane(W.chunk_beam[ch]);  // uniform: scalar case loads
    const CaseDev &cs = L.cases[W.bcase[gb]];
    const MeshDev &m = cs.m;
    const int64_t b = gb - cs.beam_base;
    const int64_t k0 = cs.offsets[b];
    const int nb = (int)(cs.offsets[b + 1] - k0);
    const int s0 = W.chunk_s0[ch], s1 = W.chunk_s1[ch];
    const int nseg = nb >= 2 ? nb - 1 : 1;
    const int nsg = s1 - s0 + 1;
    const gptr<double> X = to_global(cs.Psp) + 3 * k0;
    const double tl = m.tile_len;
    const double R = chunk_reach(W, gb, tl);
    const double mrg = 1e-7 * (tl + R);
    // segment data: the chunk's segments and the ones before and after it
    for (int jj = lane; jj <= nsg + 1; jj += 64) {
      const int j = jj - 1;
      int i = s0 + j;
      SegInfo q;
      bool exists = (nb == 1) ? (j == 0) : (i >= 0 && i <= nb - 2);
      if (exists) {
        const gptr<double> A = X + 3 * (nb == 1 ? 0 : i), B = X + 3 * (nb == 1 ? 0 : i + 1);
        double e[3];
        for (int a = 0; a < 3; ++a) {
          q.lo[a] = fmin(A[a], B[a]) - R;
          q.hi[a] = fmax(A[a], B[a]) + R;
          q.a[a] = A[a];
          e[a] = B[a] - A[a];
        }
        q.len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        q.su = 0.0;
        for (int a = 0; a < 3; ++a) {
          q.u[a] = q.len > 0.0 ? e[a] / q.len : 0.0;
          q.su += fabs(q.u[a]);
        }
      } else {
        for (int a = 0; a < 3; ++a) {
          q.lo[a] = INFINITY;
          q.hi[a] = -INFINITY;
          q.a[a] = 0.0;
          q.u[a] = 0.0;
        }
        q.len = 0.0;
        q.su = 0.0;
      }
      sg[jj] = q;
    }
    __syncthreads();
    // case fields used in the tile loop, held in registers (the loop's
    // stores would otherwise make the compiler read them again)
    const bool slab = nb >= 2 && cs.proj_mode == ALP_PROJ_NEAREST;
    const int64_t tbase = cs.tile_base;
    const int ntx = m.nt[0], nty = m.nt[1];
    const double mlo0 = m.lo[0], mlo1 = m.lo[1], mlo2 = m.lo[2];
    // box offsets in 32 bits (the scanned box sizes are 32-bit counts)
    const uint32_t nx = (uint32_t)(box[3] - box[0] + 1), ny = (uint32_t)(box[4] - box[1] + 1);
    for (uint32_t q = lane; q < (uint32_t)ntile; q += 64) {
      int wlo = -1, whi = -1;
      const uint32_t qy = q / nx, qz = qy / ny;
      const int tx = box[0] + (int)(q - qy * nx), ty = box[1] + (int)(qy - qz * ny), tz = box[2] + (int)qz;
      double tlo[3] = {mlo0 + tx * tl, mlo1 + ty * tl, mlo2 + tz * tl};
      double tc[3] = {tlo[0] + 0.5 * tl, tlo[1] + 0.5 * tl, tlo[2] + 0.5 * tl};
      double half = 0.5 * tl + mrg;
      for (int j = 0; j < nsg; ++j) {
        const SegInfo &g = sg[j + 1];
        bool ov = true;
        for (int a = 0; a < 3; ++a)  // all six bounds, no early exit
          ov = ov & !(g.hi[a] < tlo[a] - mrg) & !(g.lo[a] > tlo[a] + tl + mrg);
        if (!ov) continue;
        const int i = s0 + j;
        // the slab rule keeps only segments that can be a cell's nearest one;
        // the segment-integrated rule needs every segment within reach
        if (slab && g.len > 0.0) {
          double ac = (tc[0] - g.a[0]) * g.u[0] + (tc[1] - g.a[1]) * g.u[1] + (tc[2] - g.a[2]) * g.u[2];
          double hw = half * g.su;
          if (i > 0 && !(ac + hw > -mrg)) {
            const SegInfo &gp = sg[j];
            if (gp.len > 0.0) {
              double acp = (tc[0] - gp.a[0]) * gp.u[0] + (tc[1] - gp.a[1]) * gp.u[1] +
                           (tc[2] - gp.a[2]) * gp.u[2];
              if (acp + half * gp.su < gp.len - mrg) continue;
            }
          }
          if (i < nseg - 1 && !(ac - hw < g.len + mrg)) {
            const SegInfo &gn = sg[j + 2];
            if (gn.len > 0.0) {
              double acn = (tc[0] - gn.a[0]) * gn.u[0] + (tc[1] - gn.a[1]) * gn.u[1] +
                           (tc[2] - gn.a[2]) * gn.u[2];
              if (!(acn - half * gn.su < mrg)) continue;
            }
          }
        }
        if (wlo < 0) wlo = i;
        whi = i;
      }
      const int64_t slot = (int64_t)slot0 + q;
      if (slot >= W.cap_emit) {
        set_overflow(W, 1u);
        continue;
      }
      Emit e;
      e.beam = wlo >= 0 ? gb : -1;
      e.lo = nb == 1 ? 0 : wlo;
      e.hi = nb == 1 ? 0 : whi;
      e.tile = (int32_t)(tbase + ((int64_t)tz * nty + ty) * ntx + tx);
      W.emit_raw[slot] = e;
      if (wlo >= 0) atomicAdd(&W.tile_cnt[e.tile], 1u);
    }
    __syncthreads();
  }
}

void launch_chunk_tiles(const StepLaunch &L, hipStream_t st) {
  if (L.w.cap_chunk == 0) return;
  int64_t g = L.w.cap_chunk < 65536 ? L.w.cap_chunk : 65536;
  hipLaunchKernelGGL(k_chunk_tiles, dim3((unsigned)g), dim3(64), 0, st, L);
}

// windows -> grouped by tile (counting sort; order inside a tile is fixed by
// the weights pass, which sorts each tile's windows by beam)
__global__ void k_emit_scatter(StepLaunch L) {
  Work W = L.w;
  int64_t n = W.chunk_box[W.cap_chunk];
  if (n > W.cap_emit) n = W.cap_emit;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Emit e = W.emit_raw[i];
    if (e.beam < 0) continue;
    const int c = case_of(L.tbase, L.n_cases, e.tile);
    const CaseDev &cs = L.cases[c];
    const int64_t b = e.beam - cs.beam_base;
    const int64_t k0 = cs.offsets[b];
    Win w;
    w.beam = e.beam;
    w.lo = e.lo;
    w.hi = (cs.offsets[b + 1] - k0) == 1 ? -1 : e.hi;
    w.k0 = (int32_t)k0;
    const uint32_t slot = W.tile_off[e.tile] + atomicAdd(&W.tile_fill[e.tile], 1u);
    W.emit[slot] = w;
  }
}

void launch_emit_scatter(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_emit_scatter, dim3(L.grid_persistent), dim3(256), 0, st, L);
}

// Tile merge: join the windows of one beam into one entry (entries in beam
// order; a beam's entry spans its windows' segments) and count the work items
// of the tile (64 cells each; none without entries).  Up to 16 windows are
// merged by a group of 16 lanes (four tiles per wave), up to 64 by the whole
// wave in registers, more by a sort in LDS.
template <int kCap>
struct MergeScratch {
  unsigned long long key[kCap];  // (beam << 32) | first segment
  int32_t hi[kCap];
  int32_t k0[kCap];
};

// window points an entry stages (its segments' end points, or the point of a
// single-CV beam)
__device__ __forceinline__ uint32_t entry_points(const Entry &en) {
  return en.single ? 1u : (uint32_t)(en.i1 - en.i0 + 2);
}
__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += (uint32_t)__shfl_xor((int)v, d, 64);
  return v;
}

// Tiles with more than 64 windows: sort the (beam, first segment) keys in
// LDS (bitonic), then join each beam's run.  Returns the number of entries.
template <int kCap>
__device__ uint32_t tile_merge_lds(const Work &W, MergeScratch<kCap> &sh, int lane, uint32_t eoff, uint32_t n_emit,
                                   uint32_t &npts) {
  // the scratch may still be read for the wave's previous tile
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t np2 = 1;
  while (np2 < n_emit) np2 <<= 1;
  for (uint32_t i = lane; i < np2; i += 64) {
    if (i < n_emit) {
      const Win e = W.emit[eoff + i];
      sh.key[i] = ((unsigned long long)(uint32_t)e.beam << 32) | (uint32_t)e.lo;
      sh.hi[i] = e.hi;
      sh.k0[i] = e.k0;
    } else {
      sh.key[i] = ~0ull;
      sh.hi[i] = 0;
      sh.k0[i] = 0;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  for (uint32_t k = 2; k <= np2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = lane; i < np2; i += 64) {
        const uint32_t p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const unsigned long long a = sh.key[i], bk = sh.key[p];
          if ((a > bk) == up) {
            sh.key[i] = bk;
            sh.key[p] = a;
            const int32_t t = sh.hi[i];
            sh.hi[i] = sh.hi[p];
            sh.hi[p] = t;
            const int32_t u = sh.k0[i];
            sh.k0[i] = sh.k0[p];
            sh.k0[p] = u;
          }
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
  }
  uint32_t ne = 0, pts = 0;
  for (uint32_t r0 = 0; r0 < n_emit; r0 += 64) {
    const uint32_t i = r0 + lane;
    bool head = false;
    uint32_t beam = 0;
    if (i < n_emit) {
      beam = (uint32_t)(sh.key[i] >> 32);
      head = (i == 0) || ((uint32_t)(sh.key[i - 1] >> 32) != beam);
    }
    const uint64_t bal = ballot64(head);
    if (head) {
      const uint32_t idx = ne + lanemask_lt_popc(bal);
      int32_t hi = sh.hi[i];
      for (uint32_t j = i + 1; j < n_emit && (uint32_t)(sh.key[j] >> 32) == beam; ++j)
        hi = max(hi, sh.hi[j]);
      Entry en;
      en.k0 = sh.k0[i];
      en.i0 = (int32_t)(sh.key[i] & 0xffffffffu);
      en.i1 = hi < 0 ? 0 : hi;
      en.single = hi < 0 ? 1 : 0;
      W.entry[eoff + idx] = en;  // idx < beams of the tile <= windows of the tile
      pts += entry_points(en);
    }
    ne += (uint32_t)__popcll(bal);
  }
  npts = wave_sum_u32(pts);
  return ne;
}

// Tiles with at most 64 windows, one window per lane: the head of a beam is
// its window with the smallest first segment, the entry's last segment the
// largest over the beam's windows, and its place the number of smaller beams
// in the tile.  Returns the number of entries.
__device__ uint32_t tile_merge_regs(const Work &W, int lane, uint32_t eoff, uint32_t n_emit, uint32_t &npts) {
  uint32_t beam = ~0u, lo = 0;
  int32_t hi = 0, k0 = 0;
  if ((uint32_t)lane < n_emit) {
    const Win e = W.emit[eoff + lane];
    beam = (uint32_t)e.beam;
    lo = (uint32_t)e.lo;
    hi = e.hi;
    k0 = e.k0;
  }
  bool head = (uint32_t)lane < n_emit;
  int32_t mhi = hi;
  for (uint32_t j = 0; j < n_emit; ++j) {
    const uint32_t bj = (uint32_t)__builtin_amdgcn_readlane((int)beam, (int)j);
    const uint32_t lj = (uint32_t)__builtin_amdgcn_readlane((int)lo, (int)j);
    const int32_t hj = __builtin_amdgcn_readlane(hi, (int)j);
    if (bj == beam) {
      mhi = max(mhi, hj);
      if (lj < lo || (lj == lo && j < (uint32_t)lane)) head = false;
    }
  }
  const uint64_t hb = ballot64(head);
  uint32_t idx = 0;
  for (uint64_t mm = hb; mm; mm &= mm - 1) {
    const int j = __builtin_ctzll(mm);
    idx += (uint32_t)__builtin_amdgcn_readlane((int)beam, j) < beam ? 1u : 0u;
  }
  uint32_t pts = 0;
  if (head) {
    Entry en;
    en.k0 = k0;
    en.i0 = (int32_t)lo;
    en.i1 = mhi < 0 ? 0 : mhi;
    en.single = mhi < 0 ? 1 : 0;
    W.entry[eoff + idx] = en;
    pts = entry_points(en);
  }
  npts = wave_sum_u32(pts);
  return (uint32_t)__popcll(hb);
}

// The tile's item count and entry count, written once its merge is done;
// the count carries kNentGrouped when the entries' windows hold more points
// than the weights pass stages at once.
__device__ __forceinline__ void tile_done(Work &W, int64_t t, uint32_t ne, uint32_t npts, uint32_t ncell) {
  const uint32_t ni = (ncell + 63u) / 64u;
  W.tile_nent[t] = ni ? (ne | (npts > (uint32_t)kStagePts ? kNentGrouped : 0u)) : 0u;
  W.tile_items[t] = ni;
}

// One wave takes kMergeTiles consecutive tiles, a group of kMergeGroup lanes
// each.  A tile with at most kMergeGroup windows is merged by its group (one
// window per lane, the same rule as tile_merge_regs, within the group); fuller
// tiles are merged afterwards by the whole wave, one at a time.
constexpr int kMergeGroup = 16;
constexpr int kMergeTiles = 64 / kMergeGroup;

__global__ __launch_bounds__(64) void k_tile_merge(StepLaunch L) {
  Work W = L.w;
  __shared__ MergeScratch<kMaxEmitTile> sh;
  const int lane = threadIdx.x;
  const int gl = lane & (kMergeGroup - 1), gbase = lane & ~(kMergeGroup - 1);
  const int64_t tg = (int64_t)blockIdx.x * kMergeTiles + lane / kMergeGroup;
  const bool have = tg < W.n_tiles;
  uint32_t eoff = 0, n_emit = 0, ncell = 0;
  if (have) {
    eoff = W.tile_off[tg];
    n_emit = W.tile_off[tg + 1] - eoff;
    const int c = case_of(L.tbase, L.n_cases, tg);
    const CaseDev &cs = L.cases[c];
    const int64_t tl = tg - cs.tile_base;
    ncell = tile_cell_start(cs.m, tl + 1) - tile_cell_start(cs.m, tl);
  }
  const bool small = have && n_emit > 0 && n_emit <= (uint32_t)kMergeGroup;
  const bool mine = small && (uint32_t)gl < n_emit;
  uint32_t beam = ~0u, lo = 0;
  int32_t hi = 0, k0 = 0;
  if (mine) {
    const Win e = W.emit[eoff + gl];
    beam = (uint32_t)e.beam;
    lo = (uint32_t)e.lo;
    hi = e.hi;
    k0 = e.k0;
  }
  bool head = mine;
  int32_t mhi = hi;
#pragma unroll
  for (int j = 0; j < kMergeGroup; ++j) {
    const int src = gbase | j;
    const uint32_t bj = (uint32_t)__shfl((int)beam, src, 64);
    const uint32_t lj = (uint32_t)__shfl((int)lo, src, 64);
    const int32_t hj = __shfl(hi, src, 64);
    if ((uint32_t)j < n_emit && bj == beam) {
      mhi = max(mhi, hj);
      if (lj < lo || (lj == lo && j < gl)) head = false;
    }
  }
  const uint32_t gheads = (uint32_t)(ballot64(head) >> gbase) & 0xffffu;
  uint32_t idx = 0;
#pragma unroll
  for (int j = 0; j < kMergeGroup; ++j) {
    const uint32_t bj = (uint32_t)__shfl((int)beam, gbase | j, 64);
    idx += (((gheads >> j) & 1u) != 0u && bj < beam) ? 1u : 0u;
  }
  uint32_t gpts = 0;
  if (head) {
    Entry en;
    en.k0 = k0;
    en.i0 = (int32_t)lo;
    en.i1 = mhi < 0 ? 0 : mhi;
    en.single = mhi < 0 ? 1 : 0;
    W.entry[eoff + idx] = en;
    gpts = entry_points(en);
  }
  // the group's staged points (xor steps below 16 stay inside the group)
#pragma unroll
  for (int d = kMergeGroup / 2; d > 0; d >>= 1) gpts += (uint32_t)__shfl_xor((int)gpts, d, 64);
  if (gl == 0 && have) {
    if (small) {
      tile_done(W, tg, (uint32_t)__popc(gheads), gpts, ncell);
    } else if (n_emit == 0 || n_emit > (uint32_t)kMaxEmitBig) {
      if (n_emit) set_overflow(W, 4u);
      W.tile_nent[tg] = 0;
      W.tile_items[tg] = 0;
    } else if (n_emit > (uint32_t)kMaxEmitTile) {
      // merged by k_tile_merge_big, which sorts in a larger LDS area
      const uint32_t slot = atomicAdd(&W.counters[kBigTileCounter], 1u);
      W.big_tiles[slot] = (uint32_t)tg;
    }
  }
  for (uint64_t big = ballot64(gl == 0 && have && n_emit > (uint32_t)kMergeGroup && n_emit <= (uint32_t)kMaxEmitTile);
       big; big &= big - 1) {
    const int l = __builtin_ctzll(big);
    const int64_t t = (int64_t)blockIdx.x * kMergeTiles + l / kMergeGroup;
    const uint32_t te = (uint32_t)__builtin_amdgcn_readlane((int)eoff, l);
    const uint32_t tn = (uint32_t)__builtin_amdgcn_readlane((int)n_emit, l);
    const uint32_t tc = (uint32_t)__builtin_amdgcn_readlane((int)ncell, l);
    uint32_t npts = 0;
    const uint32_t ne = tn <= 64u ? tile_merge_regs(W, lane, te, tn, npts) : tile_merge_lds(W, sh, lane, te, tn, npts);
    if (lane == 0) tile_done(W, t, ne, npts, tc);
  }
}

// Tiles with more than kMaxEmitTile windows (up to kMaxEmitBig), listed by
// k_tile_merge: one wave per tile with a 64 KB sort area.
__global__ __launch_bounds__(64) void k_tile_merge_big(StepLaunch L) {
  Work W = L.w;
  __shared__ MergeScratch<kMaxEmitBig> sh;
  const int lane = threadIdx.x;
  const uint32_t n_big = W.counters[kBigTileCounter];
  for (uint32_t i = blockIdx.x; i < n_big; i += gridDim.x) {
    const int64_t t = W.big_tiles[i];
    const uint32_t eoff = W.tile_off[t], n_emit = W.tile_off[t + 1] - eoff;
    const int c = case_of(L.tbase, L.n_cases, t);
    const CaseDev &cs = L.cases[c];
    const int64_t tl = t - cs.tile_base;
    const uint32_t ncell = tile_cell_start(cs.m, tl + 1) - tile_cell_start(cs.m, tl);
    uint32_t npts = 0;
    const uint32_t ne = tile_merge_lds(W, sh, lane, eoff, n_emit, npts);
    if (lane == 0) tile_done(W, t, ne, npts, ncell);
  }
}

void launch_tile_merge(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_tiles == 0) return;
  hipLaunchKernelGGL(k_tile_merge, dim3((unsigned)((L.w.n_tiles + kMergeTiles - 1) / kMergeTiles)), dim3(64), 0,
                     st, L);
  hipLaunchKernelGGL(k_tile_merge_big, dim3(64), dim3(64), 0, st, L);
}

__global__ void k_items(StepLaunch L) {
  Work W = L.w;
  int64_t tg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= W.n_tiles) return;
  uint32_t ni = W.tile_items[tg];
  if (ni == 0) return;
  int c = case_of(L.tbase, L.n_cases, tg);
  const CaseDev &cs = L.cases[c];
  int64_t tl = tg - cs.tile_base;
  uint32_t c0 = tile_cell_start(cs.m, tl), c1 = tile_cell_start(cs.m, tl + 1);
  uint32_t o = W.tile_itoff[tg];
  for (uint32_t j = 0; j < ni; ++j) {
    int64_t id = (int64_t)o + j;
    if (id >= W.cap_item) {
      set_overflow(W, 8u);
      return;
    }
    Item it;
    it.tile = (int32_t)tg;
    it.c0 = (int32_t)(c0 + 64u * j);
    it.c1 = (int32_t)(c0 + 64u * (j + 1) < c1 ? c0 + 64u * (j + 1) : c1);
    it.cs = c;
    it.eoff = W.tile_off[tg];
    it.nent = W.tile_nent[tg];
    W.item[id] = it;
    if (it.nent > (uint32_t)kMaxEntries) W.multi_items[atomicAdd(&W.counters[kMultiItemCounter], 1u)] = (uint32_t)id;
  }
}

void launch_items(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_tiles == 0) return;
  hipLaunchKernelGGL(k_items, dim3((unsigned)((L.w.n_tiles + 255) / 256)), dim3(256), 0, st, L);
}

// ----------------------------------------------------------------- sample --
// c(x): nearest cell centre (ties: smaller (x, y, z), then smaller caller
// index), searched over Chebyshev shells of bins until no unvisited bin can
// hold a centre as close as the best found.  A group of kSampleLanes lanes
// searches each shell together.  Returns the sorted index (the same on every
// lane of the group) or -1 when x is outside the domain box.
__device__ __forceinline__ bool closer_cell(const MeshDev &m, double D, int64_t j, double bD,
                                            int64_t best) {
  if (j < 0) return false;
  if (best < 0) return true;
  if (D < bD) return true;
  if (D > bD) return false;
  const gptr<double> a = to_global(m.cxyz) + 4 * j, b = to_global(m.cxyz) + 4 * best;
  if (a[0] != b[0]) return a[0] < b[0];
  if (a[1] != b[1]) return a[1] < b[1];
  if (a[2] != b[2]) return a[2] < b[2];
  return a[3] < b[3];  // caller index
}

// Search state of one lane: the best sorted index, its squared distance and
// its caller index.
struct Nearest {
  int64_t best = -1;
  double bD = INFINITY;
  int32_t caller = -1;
  __device__ __forceinline__ void consider(const MeshDev &m, double x, double y, double z, int64_t j,
                                           const double4 &c) {
    const double D = sqdist_exact(x, y, z, c.x, c.y, c.z);
    if (closer_cell(m, D, j, bD, best)) {
      best = j;
      bD = D;
      caller = (int32_t)c.w;
    }
  }
};

__device__ __forceinline__ double4 loc_record(const MeshDev &m, int64_t j) {
  const gptr<double> r = to_global(m.cxyz) + 4 * j;
  return make_double4(r[0], r[1], r[2], r[3]);
}

// Returns the sorted index (the same on every lane of the group) and, in
// *caller, the caller's index of that cell; -1 for both when x is outside the
// domain box.
template <int kLanes = kSampleLanes>
__device__ int64_t locate_group(const MeshDev &m, double x, double y, double z, int sub, int32_t *caller) {
  *caller = -1;
  if (!(x >= m.box[0] && x <= m.box[3] && y >= m.box[1] && y <= m.box[4] && z >= m.box[2] &&
        z <= m.box[5]))
    return -1;
  const double q[3] = {x, y, z};
  int qi[3];
  for (int a = 0; a < 3; ++a) {
    double f = floor((q[a] - m.lo[a]) / m.bin);
    qi[a] = !(f > 0.0) ? 0 : (f > (double)(m.nb[a] - 1) ? m.nb[a] - 1 : (int)f);
  }
  const double slack = 1e-9 * (m.bin * (double)(m.nb[0] + m.nb[1] + m.nb[2]) + fabs(m.lo[0]) +
                               fabs(m.lo[1]) + fabs(m.lo[2]));
  Nearest nr;
  // The first pass covers the whole 3x3x3 block of bins (with bins about one
  // cell wide it nearly always settles the search): each lane takes
  // kFirstBins bins, in batches of kFirstBatch whose loads are issued
  // together (bin ranges, then the first cell of each).  Later passes add one
  // Chebyshev shell each.
  constexpr int kFirstBins = (27 + kLanes - 1) / kLanes;
  constexpr int kFirstBatch = 4;
  for (int r = 1;; ++r) {
    if (r == 1) {
      for (int h0 = 0; h0 < kFirstBins; h0 += kFirstBatch) {
        uint32_t kb[kFirstBatch], st[kFirstBatch], en[kFirstBatch];
        bool ok[kFirstBatch];
#pragma unroll
        for (int hh = 0; hh < kFirstBatch; ++hh) {
          const int h = h0 + hh;
          const int c = sub + h * kLanes;
          const int ix = qi[0] - 1 + c % 3, iy = qi[1] - 1 + (c / 3) % 3, iz = qi[2] - 1 + c / 9;
          ok[hh] = h < kFirstBins && c < 27 && ix >= 0 && iy >= 0 && iz >= 0 && ix < m.nb[0] && iy < m.nb[1] &&
                   iz < m.nb[2];
          kb[hh] = ok[hh] ? bin_key(m, ix, iy, iz) : 0u;
        }
#pragma unroll
        for (int hh = 0; hh < kFirstBatch; ++hh) {
          st[hh] = to_global(m.bin_start)[kb[hh]];
          en[hh] = to_global(m.bin_start)[kb[hh] + 1];
        }
        double4 f[kFirstBatch];
#pragma unroll
        for (int hh = 0; hh < kFirstBatch; ++hh) {
          if (!ok[hh]) en[hh] = st[hh];
          f[hh] = loc_record(m, st[hh] < en[hh] ? st[hh] : 0);
        }
#pragma unroll
        for (int hh = 0; hh < kFirstBatch; ++hh)
          if (st[hh] < en[hh]) nr.consider(m, x, y, z, st[hh], f[hh]);
#pragma unroll
        for (int hh = 0; hh < kFirstBatch; ++hh)
          for (uint32_t j = st[hh] + 1; j < en[hh]; ++j) nr.consider(m, x, y, z, j, loc_record(m, j));
      }
    } else {
      const int side = 2 * r + 1;
      const int ncube = side * side * side;
      for (int c = sub; c < ncube; c += kLanes) {
        int dz = c / (side * side), dy = (c / side) % side, dx = c % side;
        int ix = qi[0] - r + dx, iy = qi[1] - r + dy, iz = qi[2] - r + dz;
        int ch = max(abs(dx - r), max(abs(dy - r), abs(dz - r)));
        if (ch != r || ix < 0 || iy < 0 || iz < 0 || ix >= m.nb[0] || iy >= m.nb[1] || iz >= m.nb[2])
          continue;
        uint32_t k = bin_key(m, ix, iy, iz);
        uint32_t e = to_global(m.bin_start)[k + 1];
        for (uint32_t j = to_global(m.bin_start)[k]; j < e; ++j) nr.consider(m, x, y, z, j, loc_record(m, j));
      }
    }
    // group reduction (all lanes of the group end with the same best)
#pragma unroll
    for (int o = kLanes / 2; o > 0; o >>= 1) {
      const double oD = __shfl_xor(nr.bD, o, 64);
      const long long ob = __shfl_xor((long long)nr.best, o, 64);
      const int oc = __shfl_xor(nr.caller, o, 64);
      if (closer_cell(m, oD, ob, nr.bD, nr.best)) {
        nr.best = ob;
        nr.bD = oD;
        nr.caller = oc;
      }
    }
    bool all = true;
    double bound = INFINITY;
    for (int a = 0; a < 3; ++a) {
      if (qi[a] - r > 0) {
        all = false;
        bound = fmin(bound, q[a] - (m.lo[a] + (double)(qi[a] - r) * m.bin));
      }
      if (qi[a] + r < m.nb[a] - 1) {
        all = false;
        bound = fmin(bound, (m.lo[a] + (double)(qi[a] + r + 1) * m.bin) - q[a]);
      }
    }
    if (all) break;
    bound -= slack;
    if (nr.best >= 0 && bound > 0.0 && nr.bD < bound * bound) break;
  }
  *caller = nr.caller;
  return nr.best;
}

// Eq. (16)-(18) per actuator point, in the paper's order.  Every lane of a
// group computes the same values; lane 0 of the group writes them.
template <int kLanes>
__global__ __launch_bounds__(64) void k_sample(StepLaunch L) {
#pragma clang fp contract(off)
  Work W = L.w;
  const int sub = threadIdx.x % kLanes;
  constexpr int kPts = 64 / kLanes;  // points per wave and pass
  for (int64_t g0 = (int64_t)blockIdx.x * kPts; g0 < W.n_points; g0 += (int64_t)gridDim.x * kPts) {
  const int64_t g = g0 + threadIdx.x / kLanes;
  const bool act = g < W.n_points;
  bool out = false, fb = false, dg = false;
  int c = 0;
  if (act) {
    c = case_of(L.pbase, L.n_cases, g);
    const CaseDev &cs = L.cases[c];
    const MeshDev &m = cs.m;
    const int64_t k = g - cs.point_base;
    const int64_t b = to_global(W.pbeam)[g] - cs.beam_base;
    const gptr<double> Pa = to_global(cs.P) + 3 * k, Pd = to_global(cs.Pdot) + 3 * k, et = to_global(cs.e_t) + 3 * k;
    double nrm = sqrt(dot3_exact(et[0], et[1], et[2], et[0], et[1], et[2]));
    double e[3] = {et[0] / nrm, et[1] / nrm, et[2] / nrm};
    double ps[3] = {Pa[0], Pa[1], Pa[2]}, us[3] = {0.0, 0.0, 0.0}, as[3] = {0.0, 0.0, 0.0};
    int32_t ca_c = -1, cs_c = -1;  // caller indices of the two cells
    int64_t ca = locate_group<kLanes>(m, Pa[0], Pa[1], Pa[2], sub, &ca_c), cs_ = -1;
    if (ca < 0) {
      out = true;
    } else {
      const gptr<double> Ua = to_global(cs.U) + 3 * (int64_t)ca_c;
      double u0[3] = {Ua[0] - Pd[0], Ua[1] - Pd[1], Ua[2] - Pd[2]};
      double ut = dot3_exact(u0[0], u0[1], u0[2], e[0], e[1], e[2]);
      double un[3] = {u0[0] - ut * e[0], u0[1] - ut * e[1], u0[2] - ut * e[2]};
      double mag = sqrt(dot3_exact(un[0], un[1], un[2], un[0], un[1], un[2]));
      double es[3];
      if (mag >= cs.tau && mag > 0.0) {
        es[0] = -un[0] / mag;
        es[1] = -un[1] / mag;
        es[2] = -un[2] / mag;
      } else {
        const gptr<double> eu = to_global(cs.e_up) + 3 * b;
        double ge = dot3_exact(eu[0], eu[1], eu[2], e[0], e[1], e[2]);
        double gv[3] = {eu[0] - ge * e[0], eu[1] - ge * e[1], eu[2] - ge * e[2]};
        double gn = sqrt(dot3_exact(gv[0], gv[1], gv[2], gv[0], gv[1], gv[2]));
        if (gn > 0.0) {
          es[0] = gv[0] / gn;
          es[1] = gv[1] / gn;
          es[2] = gv[2] / gn;
          fb = true;
        } else {
          es[0] = es[1] = es[2] = 0.0;
          dg = true;
        }
      }
      const gptr<double> np = to_global(cs.n_p) + 3 * b;
      double dn = dot3_exact(np[0], np[1], np[2], es[0], es[1], es[2]);
      double ls = to_global(cs.ls)[b];
      for (int a = 0; a < 3; ++a) ps[a] = Pa[a] + ls * (es[a] - dn * np[a]);
      cs_ = locate_group<kLanes>(m, ps[0], ps[1], ps[2], sub, &cs_c);
      if (cs_ < 0) {
        out = true;
      } else {
        const gptr<double> Us = to_global(cs.U) + 3 * (int64_t)cs_c;
        us[0] = Us[0];
        us[1] = Us[1];
        us[2] = Us[2];
        if (cs.dUdt) {
          const gptr<double> As = to_global(cs.dUdt) + 3 * (int64_t)cs_c;
          as[0] = As[0];
          as[1] = As[1];
          as[2] = As[2];
        }
      }
    }
    if (sub == 0) {
      W.Ps[3 * g] = ps[0];
      W.Ps[3 * g + 1] = ps[1];
      W.Ps[3 * g + 2] = ps[2];
      W.As[3 * g] = as[0];
      W.As[3 * g + 1] = as[1];
      W.As[3 * g + 2] = as[2];
      W.Us[3 * g] = us[0];
      W.Us[3 * g + 1] = us[1];
      W.Us[3 * g + 2] = us[2];
      if (cs.U_s)
        for (int a = 0; a < 3; ++a) cs.U_s[3 * k + a] = us[a];
      if (cs.P_s)
        for (int a = 0; a < 3; ++a) cs.P_s[3 * k + a] = ps[a];
      if (cs.cell_a) cs.cell_a[k] = ca < 0 ? -1 : (int64_t)ca_c;
      if (cs.cell_s) cs.cell_s[k] = cs_ < 0 ? -1 : (int64_t)cs_c;
      W.pflags[g] = (out ? 1 : 0) | (fb ? 2 : 0) | (dg ? 4 : 0);
    }
  }
  // counters: group leaders only (a wave may straddle two cases)
  const bool lead = act && sub == 0;
  int c0 = __shfl(c, 0, 64);
  bool same = __all(!act || c == c0);
  if (same) {
    long long *cnt = W.cnt + kCnt * c0;
    wave_count_add(cnt + 0, lead && out);
    wave_count_add(cnt + 1, lead && fb);
    wave_count_add(cnt + 2, lead && dg);
  } else if (lead) {
    long long *cnt = W.cnt + kCnt * c;
    if (out) atomicAdd((unsigned long long *)(cnt + 0), 1ull);
    if (fb) atomicAdd((unsigned long long *)(cnt + 1), 1ull);
    if (dg) atomicAdd((unsigned long long *)(cnt + 2), 1ull);
  }
  }
}

// One wave per 64 / lanes points, or (sample_waves > 0) at most that many
// waves per CU walking the points with a stride.  2, 4 or 8 lanes per point
// (the tuning chooses; 4 otherwise).
void launch_sample(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_points == 0) return;
  const int lanes = L.sample_lanes == 2 || L.sample_lanes == 8 ? L.sample_lanes : 4;
  int64_t blocks = (L.w.n_points * lanes + 63) / 64;
  const int64_t cap = (int64_t)(L.grid_persistent / 8) * L.sample_waves;
  if (cap > 0 && blocks > cap) blocks = cap;
  if (lanes == 2) hipLaunchKernelGGL(k_sample<2>, dim3((unsigned)blocks), dim3(64), 0, st, L);
  else if (lanes == 8) hipLaunchKernelGGL(k_sample<8>, dim3((unsigned)blocks), dim3(64), 0, st, L);
  else hipLaunchKernelGGL(k_sample<4>, dim3((unsigned)blocks), dim3(64), 0, st, L);
}

// ---------------------------------------------------------- kernel sample --
// ALP_SAMPLE_KERNEL: the volume average of U about P_s with the profile of
// eq. (22), U_s = sum_j g_j V_j U_j / sum_j g_j V_j over the cells within
// 3 eps_k, g_j = exp(-|C_j - P_s|^2 / eps_k^2).  One wave per point: the
// lanes share the bins around P_s, each keeps FP64 partial sums, and a fixed
// butterfly joins them.  The cutoff test uses the same FP64 expressions as
// every other distance decision.  With no cell in reach the single-cell value
// written by k_sample stays and the point is counted.
// ------------------------------------------------------- beam geometry --
// Helpers ahead of a step, one group of kSampleLanes lanes per point: the
// actuator point of eq. (15), P = (C^b + W^ref) + W; the unit tangent from
// the spline through the current cell centres x = C^b + W, whose node
// derivative is the derivative of the parabola through three consecutive
// centres parameterised by chord length (the first or last three at the
// ends; the chord for two-point beams; a zero chord falls back to its
// neighbour; no chord at all leaves a zero tangent, counted); and the local
// kernel width max(factor V_c^(1/3), eps_phys) with c the cell of P (a point
// outside the domain keeps eps_phys, counted).
__device__ __forceinline__ void cur_centre(const GeomLaunch &G, int64_t k, double *x) {
#pragma clang fp contract(off)
  for (int a = 0; a < 3; ++a) x[a] = G.Cb[3 * k + a] + G.W[3 * k + a];
}

__device__ __forceinline__ double unit_chord(const double *a, const double *b, double *u) {
#pragma clang fp contract(off)
  const double e0 = b[0] - a[0], e1 = b[1] - a[1], e2 = b[2] - a[2];
  const double l = sqrt((e0 * e0 + e1 * e1) + e2 * e2);
  u[0] = l > 0.0 ? e0 / l : 0.0;
  u[1] = l > 0.0 ? e1 / l : 0.0;
  u[2] = l > 0.0 ? e2 / l : 0.0;
  return l;
}

__global__ __launch_bounds__(64) void k_beam_geometry(GeomLaunch G) {
#pragma clang fp contract(off)
  const int sub = threadIdx.x % kSampleLanes;
  const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kSampleLanes;
  if (k >= G.n_points) return;  // whole groups leave together
  double P[3];
  for (int a = 0; a < 3; ++a)
    P[a] = (G.Cb[3 * k + a] + (G.Wref ? G.Wref[3 * k + a] : 0.0)) + G.W[3 * k + a];
  bool zero = false;
  double et[3] = {0.0, 0.0, 0.0};
  if (G.e_t) {
    // the beam of the point: the last b with offsets[b] <= k
    int lo = 0, hi = G.n_beams - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (G.offsets[mid] <= k) lo = mid;
      else hi = mid - 1;
    }
    const int64_t k0 = G.offsets[lo], n = G.offsets[lo + 1] - k0, i = k - k0;
    double m[3] = {0.0, 0.0, 0.0};
    if (n == 2) {
      double xa[3], xb[3];
      cur_centre(G, k0, xa);
      cur_centre(G, k0 + 1, xb);
      unit_chord(xa, xb, m);
    } else if (n >= 3) {
      const int64_t a = i == 0 ? 0 : (i == n - 1 ? n - 3 : i - 1);
      const int j = (int)(i - a);
      double x0[3], x1[3], x2[3], u0[3], u1[3];
      cur_centre(G, k0 + a, x0);
      cur_centre(G, k0 + a + 1, x1);
      cur_centre(G, k0 + a + 2, x2);
      const double d0 = unit_chord(x0, x1, u0), d1 = unit_chord(x1, x2, u1);
      if (d0 > 0.0 && d1 > 0.0) {
        double w0, w1;
        if (j == 0) {
          w0 = 2.0 * d0 + d1;
          w1 = -d0;
        } else if (j == 1) {
          w0 = d1;
          w1 = d0;
        } else {
          w0 = -d1;
          w1 = d0 + 2.0 * d1;
        }
        for (int c = 0; c < 3; ++c) m[c] = (w0 * u0[c] + w1 * u1[c]) / (d0 + d1);
      } else if (d0 > 0.0 && j <= 1) {
        for (int c = 0; c < 3; ++c) m[c] = u0[c];
      } else if (d1 > 0.0 && j >= 1) {
        for (int c = 0; c < 3; ++c) m[c] = u1[c];
      } else if (d0 > 0.0) {
        for (int c = 0; c < 3; ++c) m[c] = u0[c];
      } else if (d1 > 0.0) {
        for (int c = 0; c < 3; ++c) m[c] = u1[c];
      }
    }
    const double l = sqrt((m[0] * m[0] + m[1] * m[1]) + m[2] * m[2]);
    zero = !(l > 0.0);
    for (int c = 0; c < 3; ++c) et[c] = zero ? 0.0 : m[c] / l;
  }
  double ek = 0.0;
  bool out = false;
  if (G.eps) {
    int32_t c_caller;
    const int64_t c = locate_group(G.m, P[0], P[1], P[2], sub, &c_caller);
    ek = G.eps_phys[k];
    if (c < 0) {
      out = true;
    } else {
      const double dx = G.factor * cbrt(G.m.vs[c]);
      if (dx > ek) ek = dx;
    }
  }
  if (sub == 0) {
    if (G.P)
      for (int a = 0; a < 3; ++a) G.P[3 * k + a] = P[a];
    if (G.e_t)
      for (int a = 0; a < 3; ++a) G.e_t[3 * k + a] = et[a];
    if (G.eps) G.eps[k] = ek;
    if (G.counts && zero) atomicAdd(&G.counts[0], 1ull);
    if (G.counts && out) atomicAdd(&G.counts[1], 1ull);
  }
}

void launch_beam_geometry(const GeomLaunch &G, hipStream_t st) {
  if (G.n_points == 0) return;
  const int64_t threads = G.n_points * kSampleLanes;
  hipLaunchKernelGGL(k_beam_geometry, dim3((unsigned)((threads + 63) / 64)), dim3(64), 0, st, G);
}

__global__ __launch_bounds__(64) void k_sample_kernel(StepLaunch L) {
#pragma clang fp contract(off)
  Work W = L.w;
  const int lane = threadIdx.x;
  for (int64_t g = blockIdx.x; g < W.n_points; g += gridDim.x) {
    const int c = case_of(L.pbase, L.n_cases, g);
    const CaseDev &cs = L.cases[c];
    if (cs.sample_mode != ALP_SAMPLE_KERNEL || (W.pflags[g] & 1)) continue;  // uniform per wave
    const MeshDev &m = cs.m;
    const int64_t k = g - cs.point_base;
    const double p[3] = {W.Ps[3 * g], W.Ps[3 * g + 1], W.Ps[3 * g + 2]};
    const double ep = cs.eps[k];
    const double e2 = ep * ep, cut = 9.0 * e2, r = 3.0 * ep;
    int lo[3], hi[3];
    bool ok = true;
    for (int a = 0; a < 3; ++a) {
      // one extra bin on each side absorbs the rounding of p -/+ r
      const double f0 = floor((p[a] - r - m.lo[a]) / m.bin) - 1.0, f1 = floor((p[a] + r - m.lo[a]) / m.bin) + 1.0;
      ok = ok && f0 <= f1;  // false for non-finite input
      lo[a] = !(f0 > 0.0) ? 0 : (f0 > (double)(m.nb[a] - 1) ? m.nb[a] - 1 : (int)f0);
      hi[a] = !(f1 > 0.0) ? 0 : (f1 > (double)(m.nb[a] - 1) ? m.nb[a] - 1 : (int)f1);
    }
    double den = 0.0, n0 = 0.0, n1 = 0.0, n2 = 0.0, m0 = 0.0, m1 = 0.0, m2 = 0.0;
    const bool acc = cs.dUdt != nullptr;
    // mesh and field arrays as global pointers, read once per point
    const gptr<uint32_t> bs = to_global(m.bin_start), gp = to_global(m.perm);
    const gptr<double> gx = to_global(m.cx), gy = to_global(m.cy), gz = to_global(m.cz), gv = to_global(m.vs);
    const gptr<double> gU = to_global(cs.U);
    if (ok) {
      const int nx = hi[0] - lo[0] + 1, ny = hi[1] - lo[1] + 1, nz = hi[2] - lo[2] + 1;
      const int64_t total = (int64_t)nx * ny * nz;
      for (int64_t q = lane; q < total; q += 64) {
        const int ix = lo[0] + (int)(q % nx), iy = lo[1] + (int)((q / nx) % ny),
                  iz = lo[2] + (int)(q / ((int64_t)nx * ny));
        const uint32_t key = bin_key(m, ix, iy, iz);
        const uint32_t e = bs[key + 1];
        for (uint32_t j = bs[key]; j < e; ++j) {
          const double r2 = sqdist_exact(p[0], p[1], p[2], gx[j], gy[j], gz[j]);
          if (!(r2 <= cut)) continue;
          const double gw = exp(-(r2 / e2)) * gv[j];
          const gptr<double> Uj = gU + 3 * (int64_t)gp[j];
          den += gw;
          n0 += gw * Uj[0];
          n1 += gw * Uj[1];
          n2 += gw * Uj[2];
          if (acc) {
            const gptr<double> Aj = to_global(cs.dUdt) + 3 * (int64_t)gp[j];
            m0 += gw * Aj[0];
            m1 += gw * Aj[1];
            m2 += gw * Aj[2];
          }
        }
      }
    }
    den = wave_sum_f64(den);
    n0 = wave_sum_f64(n0);
    n1 = wave_sum_f64(n1);
    n2 = wave_sum_f64(n2);
    if (acc) {
      m0 = wave_sum_f64(m0);
      m1 = wave_sum_f64(m1);
      m2 = wave_sum_f64(m2);
    }
    if (lane == 0) {
      if (den > 0.0) {
        const double us[3] = {n0 / den, n1 / den, n2 / den};
        for (int a = 0; a < 3; ++a) W.Us[3 * g + a] = us[a];
        if (acc) {
          W.As[3 * g] = m0 / den;
          W.As[3 * g + 1] = m1 / den;
          W.As[3 * g + 2] = m2 / den;
        }
        if (cs.U_s)
          for (int a = 0; a < 3; ++a) cs.U_s[3 * k + a] = us[a];
      } else {
        atomicAdd((unsigned long long *)(W.cnt + kCnt * c + 7), 1ull);
      }
    }
  }
}

void launch_sample_kernel(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_points == 0 || !L.kernel_sample) return;
  const int64_t g = L.w.n_points < (int64_t)L.grid_persistent * 4 ? L.w.n_points : (int64_t)L.grid_persistent * 4;
  hipLaunchKernelGGL(k_sample_kernel, dim3((unsigned)g), dim3(64), 0, st, L);
}

// ------------------------------------------------------------------- drag --
// Eq. (19) with the force acting on the beam (or eq. 6), then eq. (20).
__global__ void k_drag(StepLaunch L, int use_cell_s) {
#pragma clang fp contract(off)
  Work W = L.w;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= W.n_points) return;
  int c = case_of(L.pbase, L.n_cases, g);
  const CaseDev &cs = L.cases[c];
  int64_t k = g - cs.point_base;
  int64_t b = W.pbeam[g] - cs.beam_base;
  bool out = use_cell_s ? (cs.cell_s != nullptr && cs.cell_s[k] < 0) : ((W.pflags[g] & 1) != 0);
  const double *Us = use_cell_s ? cs.U_s + 3 * k : W.Us + 3 * g;
  double fs[3] = {0.0, 0.0, 0.0};
  if (!out) {
    const double *et = cs.e_t + 3 * k, *Pd = cs.Pdot + 3 * k;
    double nrm = sqrt(dot3_exact(et[0], et[1], et[2], et[0], et[1], et[2]));
    double e[3] = {et[0] / nrm, et[1] / nrm, et[2] / nrm};
    double ur[3] = {Us[0] - Pd[0], Us[1] - Pd[1], Us[2] - Pd[2]};
    double t = dot3_exact(ur[0], ur[1], ur[2], e[0], e[1], e[2]);
    double ut[3] = {t * e[0], t * e[1], t * e[2]};
    double un[3] = {ur[0] - ut[0], ur[1] - ut[1], ur[2] - ut[2]};
    double half = 0.5 * cs.rho * cs.d[k];
    double cdn = cs.Cdn[b], cdt = cs.Cdt[b];
    if (cs.drag_form == ALP_DRAG_COMPONENTWISE) {
      double mn = sqrt(dot3_exact(un[0], un[1], un[2], un[0], un[1], un[2]));
      double mt = sqrt(dot3_exact(ut[0], ut[1], ut[2], ut[0], ut[1], ut[2]));
      for (int a = 0; a < 3; ++a) fs[a] = half * (cdn * mn * un[a] + cdt * mt * ut[a]);
    } else {
      double mr = sqrt(dot3_exact(ur[0], ur[1], ur[2], ur[0], ur[1], ur[2]));
      for (int a = 0; a < 3; ++a) fs[a] = half * mr * (cdn * un[a] + cdt * ut[a]);
    }
    if (cs.A && cs.dUdt && !use_cell_s) {
      // eq. (8) with the relative acceleration fluid minus beam
      const double *af = W.As + 3 * g;
      double ar[3];
      for (int a = 0; a < 3; ++a) ar[a] = af[a] - (cs.a_b ? cs.a_b[3 * k + a] : 0.0);
      const double ta = dot3_exact(ar[0], ar[1], ar[2], e[0], e[1], e[2]);
      const double ra = cs.rho * cs.A[k], cmn = cs.CMn[b], cmt = cs.CMt[b];
      for (int a = 0; a < 3; ++a) {
        const double art = ta * e[a], arn = ar[a] - art;
        fs[a] += ra * ((cmt * art + cmn * arn) + af[a]);
      }
    }
  }
  double *f = cs.f ? cs.f + 3 * k : W.f + 3 * g;
  for (int a = 0; a < 3; ++a)
    f[a] = cs.has_fprev ? cs.alpha_f * fs[a] + (1.0 - cs.alpha_f) * cs.f_prev[3 * k + a] : fs[a];
}

void launch_drag_mode(const StepLaunch &L, int use_cell_s, hipStream_t st) {
  if (L.w.n_points == 0) return;
  hipLaunchKernelGGL(k_drag, dim3((unsigned)((L.w.n_points + 255) / 256)), dim3(256), 0, st, L,
                     use_cell_s);
}
void launch_drag(const StepLaunch &L, hipStream_t st) { launch_drag_mode(L, 0, st); }

// ---------------------------------------------------------------- weights --
// Eq. (21)-(22) and the nodal weights of Sec. 3.2.4.  One wave per work item
// (up to 64 cells of one tile, with the tile's merged entries in beam order):
//   1. stage each entry's window in LDS as FP32 points relative to the tile
//      centre, with the node exponents and node accumulators, and build a
//      screening box (window AABB inflated by 3 eps_max, in registers);
//   2. screen every (cell, entry) combination and list the candidate pairs in
//      (cell, entry) order;
//   3. for each candidate (64 at a time) find the closest segment of the
//      window: an FP32 pass ranks the segments, and every segment whose FP32
//      distance lies within a proven error band of the best one is evaluated
//      again exactly in FP64 (from the beam arrays) with the same expressions
//      as a plain scan, so the chosen segment, s and r^2 are exactly those of a
//      full FP64 scan; then the inclusive 3 eps cutoff and the weights a0, a1;
//   4. add a V into the node accumulators (exact fixed point: LDS integer
//      atomics, then one global integer atomic per touched node);
//   5. write one record per surviving pair (cell, node, a0, a1) for the
//      spread pass.
// Entries whose windows do not fit the staging area are scanned exactly from
// the beam arrays.
constexpr uint32_t kSegIdxMask = 0xffu;  // segment index packed below the FP32 distance
static_assert(kStagePts <= 256, "segment index must fit the key");

struct WeightsScratch {
  float4 sa[kStagePts];  // window point relative to the tile centre; w: 1/|e|^2 of the segment it starts
  // the node's fixed-point exponent times 256 plus the index of the entry
  // the point belongs to (staged_exp, staged_entry)
  int32_t wx[kStagePts];
  int32_t e_k0[kMaxEntries], e_i0[kMaxEntries], e_i1[kMaxEntries];  // e_i1 < 0: single point
  int32_t e_pt0[kMaxEntries + 1];
  uint32_t e_em[kMaxEntries];  // bits of the window's largest eps (FP32, rounded up)
  float e_dabs[kMaxEntries];   // absolute error allowance of the FP32 ranking
  union {
    // screening frames of up to 64 entries (three float4 each), read by all
    // lanes at one address; live only during the screening
    float4 frm[3 * 64];
    // while the frames are built: each staged window's unit chord axis and
    // the extremes over its points (ordered keys of the smallest and largest
    // axial coordinate, bits of the largest squared deviation from the chord
    // line and of the largest squared distance from the tile centre)
    struct {
      float fax[3][kMaxEntries];
      uint32_t fred[4][kMaxEntries];
    };
    struct {
      // node accumulators of the staged points
      long long ahi[kStagePts];
      unsigned long long alo[kStagePts];
      // the item's candidates: listed in order as (cell lane | entry << 6)
      // when they fit, else as per-lane hit masks searched by candidate()
      union {
        uint32_t mask[64 * kMaskWords];
        uint16_t cand[64 * kMaskWords * 2];
      };
    };
  };
  uint32_t off[65];
};
static_assert(sizeof(float4) * 3 * 64 <= 2 * 8 * kStagePts + 4 * 64 * kMaskWords,
              "screening frames overlay the accumulators and the candidate list");
static_assert(7 * 4 * kMaxEntries <= 2 * 8 * kStagePts + 4 * 64 * kMaskWords,
              "the frame reductions overlay the accumulators and the candidate list");

// median of three (one v_med3_u32)
__device__ __forceinline__ uint32_t umed3(uint32_t a, uint32_t b, uint32_t c) {
  return max(min(a, b), min(max(a, b), c));
}


// exact FP64 scan of window segments j0..j1 (local indices; points read from
// the beam array at X), strict '<' so the lowest index wins a tie
template <class Ptr>
__device__ __forceinline__ void exact_scan(Ptr X, int j0, int j1, double cx, double cy, double cz, int &bj,
                                           double &bs, double &br2) {
  double ax = X[3 * j0], ay = X[3 * j0 + 1], az = X[3 * j0 + 2];
  for (int j = j0; j <= j1; ++j) {
    const double bx = X[3 * j + 3], by = X[3 * j + 4], bz = X[3 * j + 5];
    double s, r2;
    seg_foot(cx, cy, cz, ax, ay, az, bx, by, bz, s, r2);
    if (r2 < br2) {
      br2 = r2;
      bj = j;
      bs = s;
    }
    ax = bx;
    ay = by;
    az = bz;
  }
}

static_assert(kMaxEntries <= 256, "the entry index of a staged point takes the low 8 bits");
__device__ __forceinline__ int32_t staged_exp(int32_t wx) { return wx >> 8; }  // floor(wx / 256)
__device__ __forceinline__ int staged_entry(int32_t wx) { return wx & 255; }

__device__ __forceinline__ int entry_of_point(const WeightsScratch &sh, int n_staged, int q) {
  int lo = 0, hi = n_staged - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sh.e_pt0[mid] <= q) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// Scratch of the integrated rule's weights pass: the candidates of a round
// (cell lane, entry, first pair index) and a ring of pairs in reach waiting
// for their weights (descriptor: cell lane | entry << 6 | segment << 14, and
// the record index).
constexpr uint32_t kIntRing = 128;
struct IntScratch {
  uint8_t lc[64], ent[64];
  uint32_t pre[64];
  uint32_t qd[kIntRing], qp[kIntRing];
  uint32_t emin[kMaxEntries];  // smallest eps of each staged window (FP32, rounded down)
};
constexpr uint32_t kIntMaxSeg = 1u << 18;  // window segments a descriptor can name
static_assert(kMaxEntries <= 256, "entry field of the ring descriptor");

// Candidate p of a work item (in cell-lane order, then entry order): its
// cell lane Lc and entry e, from the per-lane prefix counts and hit masks.
__device__ __forceinline__ void candidate(const WeightsScratch &sh, int nwords, uint32_t p, int &Lc, int &e) {
  int lo = 0, hi = 63;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sh.off[mid] <= p) lo = mid;
    else hi = mid - 1;
  }
  Lc = lo;
  uint32_t r = p - sh.off[Lc];
  for (int wd = 0; wd < nwords; ++wd) {
    uint32_t mw = sh.mask[Lc * kMaskWords + wd];
    const uint32_t pc = __popc(mw);
    if (r < pc) {
      for (uint32_t q = 0; q < r; ++q) mw &= mw - 1u;
      e = wd * 32 + __ffs(mw) - 1;
      return;
    }
    r -= pc;
  }
}

// Segment-integrated rule: is the segment starting at A (end A + 3) within
// 3 eps_seg of the cell, eps_seg = (eps_a + eps_b) / 2?  Zero-length segments
// never are.  FP64, in the decision order of the nearest rule's cutoff.
template <class Ptr>
__device__ __forceinline__ bool seg_in_reach(Ptr A, double ea, double eb, double cx, double cy, double cz,
                                             double &es) {
#pragma clang fp contract(off)
  const double ex = A[3] - A[0], ey = A[4] - A[1], ez = A[5] - A[2];
  if (!(((ex * ex + ey * ey) + ez * ez) > 0.0)) return false;
  double s, r2;
  seg_foot(cx, cy, cz, A[0], A[1], A[2], A[3], A[4], A[5], s, r2);
  es = 0.5 * (ea + eb);
  return inside_cutoff(r2, es);
}

// Records of one (cell, entry) candidate under the segment-integrated rule:
// one per segment within reach, or one for a single-CV beam within 3 eps.
__device__ __forceinline__ uint32_t int_count(const CaseDev &cs, int k0, int i0, int i1, double cx, double cy,
                                              double cz) {
  if (i1 < 0) {
    const double *P = cs.Psp + 3 * (int64_t)k0;
    return inside_cutoff(sqdist_exact(cx, cy, cz, P[0], P[1], P[2]), cs.eps[k0]) ? 1u : 0u;
  }
  const double *X = cs.Psp + 3 * ((int64_t)k0 + i0);
  const double *E = cs.eps + (int64_t)k0 + i0;
  uint32_t n = 0;
  for (int j = 0; j <= i1 - i0; ++j) {
    double es;
    n += seg_in_reach(X + 3 * j, E[j], E[j + 1], cx, cy, cz, es) ? 1u : 0u;
  }
  return n;
}

__device__ __forceinline__ void write_record(unsigned char *r, int rsz, uint32_t meta, uint32_t node, double a0,
                                             double a1) {
  if (rsz == 12) {
    // lane and single bit below the node index
    const uint32_t w0 = (meta & 63u) | ((meta & kRecSingle) ? 64u : 0u) | (node << kRecNodeShift);
    uint32_t *q = (uint32_t *)r;
    q[0] = w0;
    q[1] = __float_as_uint((float)a0);
    q[2] = __float_as_uint((float)a1);
  } else if (rsz == 16) {
    uint4 q;
    q.x = meta;
    q.y = node;
    q.z = __float_as_uint((float)a0);
    q.w = __float_as_uint((float)a1);
    *(uint4 *)r = q;
  } else {
    uint2 q;
    q.x = meta;
    q.y = node;
    *(uint2 *)r = q;
    *(double2 *)(r + 8) = make_double2(a0, a1);
  }
}

// One kernel per projection rule (kInt: segment-integrated) and precision,
// so that each keeps its own register allocation; each takes only the items
// of its own cases, from its own work-queue counters.  Items of tiles with
// more than kMaxEntries entries are left to a kernel of their own (kMulti),
// which takes the entries in groups of kMaxEntries; the group loop would
// otherwise cost the common kernels registers.
template <bool kInt, bool kSplit, bool kMulti>
__device__ __forceinline__ void weights_pass(const StepLaunch &L) {
  // The sampling stream's last waves can still be resident beside this pass,
  // which is on the step's critical path: its waves take a higher issue
  // priority, so the sampler's waves use the issue slots these leave free.
  __builtin_amdgcn_s_setprio(3);
  Work W = L.w;
  __shared__ WeightsScratch sh;
  const int lane = threadIdx.x;
  const uint32_t n_items = W.tile_itoff[W.n_tiles];
  // record space is reserved in blocks per wave; pair counts are flushed per case
  unsigned long long blk_cur = 0, blk_end = 0;
  int acc_case = -1;
  unsigned long long acc_pairs = 0, acc_guard = 0;
  // the grouped kernels take the list of grouped items from queues of their
  // own, one item at a time (such items are long and vary widely)
  const uint32_t n_multi = kMulti ? min(W.counters[kMultiItemCounter], (uint32_t)min((int64_t)n_items, W.cap_item)) : 0u;
  WorkQueue wq = work_queue(W.counters + queue_words((kMulti ? 4 : 0) + (kInt ? (kSplit ? 1 : 2) : (kSplit ? 0 : 3))),
                            kMulti ? n_multi : (uint32_t)min((int64_t)n_items, W.cap_item),
                            kMulti ? 1u : (uint32_t)L.weights_grab);
  for (;;) {
    uint32_t item;
    if constexpr (kMulti) {
      if (!wq.next(lane)) break;
      item = W.multi_items[wq.item];
    } else {
      if (!wq.next(lane)) break;
      item = wq.item;
    }
    // the item index is wave-uniform: read it into a scalar register so that
    // the descriptor and the case fields are scalar loads
    item = (uint32_t)__builtin_amdgcn_readfirstlane((int)item);
    const Item it = sload_item(W.item + item);
    if (!kMulti && it.nent > (uint32_t)kMaxEntries) continue;
    const CaseDev *cp = L.cases + it.cs;
    const int cprec = sload(&cp->prec);
    if ((sload(&cp->proj_mode) == ALP_PROJ_INTEGRATED) != kInt) continue;
    if ((cprec == ALP_PREC_FP32_SPLIT) != kSplit) continue;
    if (it.cs != acc_case) {
      if (lane == 0 && acc_case >= 0 && acc_pairs)
        atomicAdd((unsigned long long *)(W.cnt + kCnt * acc_case + 5), acc_pairs);
      if (lane == 0 && acc_case >= 0 && acc_guard)
        atomicAdd((unsigned long long *)(W.cnt + kCnt * acc_case + 8), acc_guard);
      acc_case = it.cs;
      acc_pairs = 0;
      acc_guard = 0;
    }
    // case fields held in registers for the whole item, read by scalar
    // loads (the loops below store and update atomically, after which the
    // compiler would read them again; and a vector load here would first
    // wait for the previous item's node-sum atomics)
    const MeshDev m = sload_mesh_geometry(&cp->m);
    const gptr<double> Psp = to_global(sload(&cp->Psp));
    const gptr<double> Eps = to_global(sload(&cp->eps));
    const int64_t pbase = sload(&cp->point_base);
    const int64_t tl = it.tile - sload(&cp->tile_base);
    const int rsz = rec_size(cprec, W.rec_compact != 0);
    // the tile's entries, in beam order.  The grouped kernels take them in
    // groups, one after another: each group is the run of entries whose
    // windows fit the staging area together (at most kMaxEntries; a window
    // that does not fit alone is a group of its own, read from global
    // memory).  A cell then has one run of records per group.
    const uint32_t ne_all = it.nent & ~kNentGrouped;
    constexpr bool multi = kMulti;
    // cells of the item, and their FP32 coordinates relative to the tile centre
    const int c = it.c0 + lane;
    const bool valid = c < it.c1;
    double cx = 0, cy = 0, cz = 0, v = 0;
    float lx = 0.f, ly = 0.f, lz = 0.f;
    int tx, ty, tz;
    tile_xyz(m, tl, tx, ty, tz);
    double tcen[3];
    tile_centre(m, tx, ty, tz, tcen);
    const double ctx = tcen[0], cty = tcen[1], ctz = tcen[2];
    const double hl = 0.5 * m.tile_len;
    if (valid) {
      cx = to_global(m.cx)[c];
      cy = to_global(m.cy)[c];
      cz = to_global(m.cz)[c];
      v = to_global(m.vs)[c];
      lx = (float)(cx - ctx);
      ly = (float)(cy - cty);
      lz = (float)(cz - ctz);
    }

    unsigned long long rbase = 0;
    bool rec_ok = true;
    // record space for n pairs, carved from the wave's block
    auto reserve = [&](uint64_t n) {
      const unsigned long long need = ((unsigned long long)n * rsz + 15ull) & ~15ull;
      if (blk_cur + need > blk_end) {
        const unsigned long long take = need > kRecBlock ? need : kRecBlock;
        unsigned long long got = 0;
        if (lane == 0) got = atomicAdd(W.rec_alloc, take);
        blk_cur = uniform_u64(got);
        blk_end = blk_cur + take;
      }
      rbase = blk_cur;
      blk_cur += need;
      rec_ok = (int64_t)(rbase + need) <= W.cap_rec;
      if (!rec_ok && lane == 0) set_overflow(W, 2u);
    };
    uint32_t nreal = 0;  // records of the item so far
    if (multi) {
      // the records of every group follow each other: reserve for the most
      // the item can have (each cell with every entry, or with every window
      // segment under the integrated rule), and give the rest back at the end
      uint64_t per_cell = 0;
      for (uint32_t e = lane; e < ne_all; e += 64) {
        const Entry en = W.entry[it.eoff + e];
        per_cell += kInt && !en.single ? (uint64_t)(en.i1 - en.i0 + 1) : 1u;
      }
#pragma unroll
      for (int d = 32; d > 0; d >>= 1) per_cell += __shfl_xor(per_cell, d, 64);
      reserve(per_cell * (uint64_t)(it.c1 - it.c0));
    }
    for (uint32_t g0 = 0;;) {
    const uint32_t ne_plan = kMulti ? min(ne_all - g0, (uint32_t)kMaxEntries) : ne_all;
    const uint32_t eoff = it.eoff + g0;
    // 1. entries and the staging plan: the leading entries whose windows fit
    uint32_t carry = 0;
    int nst = 0;
    for (uint32_t e0 = 0; e0 < ne_plan; e0 += 64) {
      const uint32_t e = e0 + lane;
      uint32_t cntp = 0;
      if (e < ne_plan) {
        const Entry en = W.entry[eoff + e];
        sh.e_k0[e] = en.k0;
        sh.e_i0[e] = en.i0;
        sh.e_i1[e] = en.single ? -1 : en.i1;
        sh.e_em[e] = 0u;
        cntp = en.single ? 1u : (uint32_t)(en.i1 - en.i0 + 2);
      }
      uint32_t tot;
      const uint32_t ex = wave_excl_scan_u32(cntp, tot) + carry;
      const bool fits = e < ne_plan && ex + cntp <= (uint32_t)kStagePts;
      if (e < ne_plan) sh.e_pt0[e] = fits ? (int32_t)ex : -1;
      nst += __popcll(ballot64(fits));
      carry += tot;
    }
    __syncthreads();
    const int n_staged = nst;
    // the entries of this group: all of them in the common kernels; in the
    // grouped ones the staged prefix, or the first entry alone
    const uint32_t ne = !kMulti ? ne_all : (n_staged > 0 ? (uint32_t)n_staged : 1u);
    int npts = 0;
    if (nst > 0) {
      const int last = nst - 1;
      npts = sh.e_pt0[last] + (sh.e_i1[last] < 0 ? 1 : sh.e_i1[last] - sh.e_i0[last] + 2);
    }
    for (int q = lane; q < npts; q += 64) {
      const int e = entry_of_point(sh, n_staged, q);
      const int64_t k = sh.e_k0[e] + (sh.e_i1[e] < 0 ? 0 : sh.e_i0[e]) + (q - sh.e_pt0[e]);
      const gptr<double> P = Psp + 3 * k;
      sh.sa[q] = make_float4((float)(P[0] - ctx), (float)(P[1] - cty), (float)(P[2] - ctz), 0.f);
      sh.wx[q] = W.wexp[pbase + k] * 256 + e;
      // eps rounded up to FP32 (positive floats order like their bits)
      const double ep = Eps[k];
      float ef = (float)ep;
      if ((double)ef < ep) ef = __uint_as_float(__float_as_uint(ef) + 1u);  // next float up (ef > 0 is all that is used)
      if (ef > 0.f) atomicMax(&sh.e_em[e], __float_as_uint(ef));
    }
    __syncthreads();
    // Screening capsules, in registers (lane l holds entry 64 b + l).  Each
    // window gets a chord frame: origin P0 (its first point), unit axis u (to
    // its last point), the axial extent [amin, amax] of its points along u and
    // dev, the largest distance of its points from the chord line.  Every
    // point x of the window's segments then has its axial coordinate inside
    // [amin, amax] and lies within dev of the line, so for a cell at distance
    // rho from the line and axial gap g from [amin, amax],
    //   |c - x|^2 >= max(rho - dev, 0)^2 + g^2,
    // and a pair needs |c - x| <= 3 eps_j <= 3 eps_max of the window.
    // The axis comes from one lane per entry; the extremes over a staged
    // window's points from one lane per point (LDS min / max), those of a
    // window read from the beam arrays from its entry's lane.
    float fr[2][10];
    // the frame's extent, radius and error allowance from the extremes over
    // its points (rr: largest squared distance of a point from the tile
    // centre; em: the window's largest eps, rounded up)
    auto frame_finish = [&](float *F, uint32_t e, float amin, float amax, float dev2, float rr, float em) {
      // coordinates of points and cells lie within Rmax of the tile centre;
      // rho and dev computed in FP32 are each within 2^-9 Rmax of their true
      // values (|d| <= 2 Rmax), the axial gap within 2^-18 Rmax: the radius
      // is widened by 2^-7 Rmax
      const float r2max = fmaxf(rr, (float)(3.0 * hl * hl));
      // (the square roots below and in the screening are the hardware's,
      // within 1 ulp: far inside these allowances)
      const float Rc = 3.0f * em * (1.0f + 1e-5f) + ldexpf(__builtin_amdgcn_sqrtf(r2max), -7);
      F[6] = amin;
      F[7] = amax;
      F[8] = __builtin_amdgcn_sqrtf(fmaxf(dev2, 0.f));
      F[9] = Rc * Rc;
      // |FP32 distance^2 - exact distance^2| stays below ~80 u Rmax^2
      // (u = 2^-24) for coordinates within Rmax of the tile centre: rounding
      // of the inputs moves the distance by at most 2 sqrt(3) u Rmax, and the
      // clamped projection adds at most ~64 u Rmax^2.  The allowance takes
      // 2^-14 Rmax^2 (256 u Rmax^2).
      sh.e_dabs[e] = ldexpf(r2max, -14) * (1.0f + 1e-5f);
    };
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const uint32_t e = 64u * bb + lane;
#pragma unroll
      for (int q = 0; q < 10; ++q) fr[bb][q] = 0.f;
      if (bb == 1 && ne <= 64u) break;  // wave-uniform: no second batch of entries
      fr[bb][6] = INFINITY;   // amin > amax: empty capsule
      fr[bb][7] = -INFINITY;
      if (e < ne) {
        const int pt0 = (int)e < n_staged ? sh.e_pt0[e] : -1;
        const bool sgl = sh.e_i1[e] < 0;
        const int np = sgl ? 1 : sh.e_i1[e] - sh.e_i0[e] + 2;
        const int64_t k = sh.e_k0[e] + (sgl ? 0 : sh.e_i0[e]);
        auto point = [&](int p) {
          if (pt0 >= 0) {
            const float4 A = sh.sa[pt0 + p];
            return make_float3(A.x, A.y, A.z);
          }
          const gptr<double> P = Psp + 3 * (k + p);
          return make_float3((float)(P[0] - ctx), (float)(P[1] - cty), (float)(P[2] - ctz));
        };
        const float3 P0 = point(0), P1 = point(np - 1);
        float ux = P1.x - P0.x, uy = P1.y - P0.y, uz = P1.z - P0.z;
        const float len = sqrtf(ux * ux + uy * uy + uz * uz);
        if (len > 0.f) {
          const float il = 1.0f / len;
          ux *= il;
          uy *= il;
          uz *= il;
        } else {
          ux = 1.f;
          uy = 0.f;
          uz = 0.f;
        }
        fr[bb][0] = P0.x;
        fr[bb][1] = P0.y;
        fr[bb][2] = P0.z;
        fr[bb][3] = ux;
        fr[bb][4] = uy;
        fr[bb][5] = uz;
        if (pt0 >= 0) {
          sh.fax[0][e] = ux;
          sh.fax[1][e] = uy;
          sh.fax[2][e] = uz;
          sh.fred[0][e] = 0xffffffffu;  // no point yet: amin = +inf
          sh.fred[1][e] = 0u;           // amax = -inf
          sh.fred[2][e] = 0u;           // dev^2 = 0
          sh.fred[3][e] = 0u;           // rr = 0
        } else {
          float amin = INFINITY, amax = -INFINITY, dev2 = 0.f, rr = 0.f;
          double dem = 0.0;
          for (int p = 0; p < np; ++p) {
            const float3 A = p == 0 ? P0 : point(p);
            const float dx = A.x - P0.x, dy = A.y - P0.y, dz = A.z - P0.z;
            const float a = dx * ux + dy * uy + dz * uz;
            amin = fminf(amin, a);
            amax = fmaxf(amax, a);
            dev2 = fmaxf(dev2, dx * dx + dy * dy + dz * dz - a * a);
            rr = fmaxf(rr, A.x * A.x + A.y * A.y + A.z * A.z);
            dem = fmax(dem, Eps[k + p]);
          }
          frame_finish(fr[bb], e, amin, amax, dev2, rr, (float)(dem * (1.0 + 1e-6)));
        }
      }
    }
    __syncthreads();
    // one lane per staged point: 1/|e|^2 of the segment it starts, and its
    // window's extremes
    for (int q = lane; q < npts; q += 64) {
      const int e = staged_entry(sh.wx[q]);
      const int np = sh.e_i1[e] < 0 ? 1 : sh.e_i1[e] - sh.e_i0[e] + 2;
      const int pt0 = sh.e_pt0[e];
      const float4 A = sh.sa[q], O = sh.sa[pt0];
      if (q - pt0 < np - 1) {
        const float4 B = sh.sa[q + 1];
        const float ex = B.x - A.x, ey = B.y - A.y, ez = B.z - A.z;
        const float ee = ex * ex + ey * ey + ez * ez;
        sh.sa[q].w = ee > 0.f ? 1.0f / ee : 0.f;
      }
      const float dx = A.x - O.x, dy = A.y - O.y, dz = A.z - O.z;
      const float a = dx * sh.fax[0][e] + dy * sh.fax[1][e] + dz * sh.fax[2][e];
      atomicMin(&sh.fred[0][e], f32_key(a));
      atomicMax(&sh.fred[1][e], f32_key(a));
      atomicMax(&sh.fred[2][e], __float_as_uint(fmaxf(dx * dx + dy * dy + dz * dz - a * a, 0.f)));
      atomicMax(&sh.fred[3][e], __float_as_uint(A.x * A.x + A.y * A.y + A.z * A.z));
    }
    __syncthreads();
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      const uint32_t e = 64u * bb + lane;
      if (bb == 1 && ne <= 64u) break;  // wave-uniform
      if (e < ne && (int)e < n_staged && sh.e_pt0[e] >= 0)
        frame_finish(fr[bb], e, f32_of_key(sh.fred[0][e]), f32_of_key(sh.fred[1][e]),
                     __uint_as_float(sh.fred[2][e]), __uint_as_float(sh.fred[3][e]),
                     __uint_as_float(sh.e_em[e]));
    }
    __syncthreads();
    // 2. screening
    uint32_t cnt = 0;
    uint32_t mw[kMaskWords];
#pragma unroll
    for (int w = 0; w < kMaskWords; ++w) mw[w] = 0u;
    // the frames go to LDS 64 entries at a time and every lane reads entry e
    // at the same address (a broadcast), one pass per mask word
#pragma unroll
    for (int bb = 0; bb < 2; ++bb) {
      if (64u * bb >= ne) break;  // wave-uniform
      if (bb > 0) __syncthreads();
      sh.frm[3 * lane] = make_float4(fr[bb][0], fr[bb][1], fr[bb][2], fr[bb][3]);
      sh.frm[3 * lane + 1] = make_float4(fr[bb][4], fr[bb][5], fr[bb][6], fr[bb][7]);
      sh.frm[3 * lane + 2] = make_float4(fr[bb][8], fr[bb][9], 0.f, 0.f);
      __syncthreads();
#pragma unroll
      for (int ww = 0; ww < 2; ++ww) {
        const int w = 2 * bb + ww;
        const uint32_t e0 = 32u * (uint32_t)w;
        if (e0 >= ne) break;  // wave-uniform
        const uint32_t e1 = min(ne, e0 + 32u);
        uint32_t word = 0;
        for (uint32_t e = e0; e < e1; ++e) {
          const int l = (int)(e & 63);
          const float4 F0 = sh.frm[3 * l], F1 = sh.frm[3 * l + 1], F2 = sh.frm[3 * l + 2];
          const float dx = lx - F0.x, dy = ly - F0.y, dz = lz - F0.z;
          const float a = dx * F0.w + dy * F1.x + dz * F1.y;
          const float rho = __builtin_amdgcn_sqrtf(fmaxf(dx * dx + dy * dy + dz * dz - a * a, 0.f));
          const float re = fmaxf(rho - F2.x, 0.f);
          const float g = fmaxf(fmaxf(F1.z - a, a - F1.w), 0.f);
          if (re * re + g * g <= F2.y) word |= 1u << (e - e0);
        }
        if (!valid) word = 0u;
        mw[w] = word;
        cnt += __popc(word);
      }
    }
    // the frames' space now holds the node accumulators and the candidates
    __syncthreads();
    for (int q = lane; q < npts; q += 64) {
      sh.ahi[q] = 0;
      sh.alo[q] = 0;
    }
    uint32_t total;
    const uint32_t myoff = wave_excl_scan_u32(cnt, total);
    sh.off[lane] = myoff;
    if (lane == 63) sh.off[64] = myoff + cnt;
    const int nwords = (int)((ne + 31) >> 5);
    // candidate p of the item: one LDS read from the list, or a search of
    // the per-lane counts and masks when the list does not fit
    const bool listed = total <= (uint32_t)(64 * kMaskWords * 2);
    if (listed) {
      uint32_t pos = myoff;
#pragma unroll
      for (int w = 0; w < kMaskWords; ++w)
        for (uint32_t m = mw[w]; m; m &= m - 1u)
          sh.cand[pos++] = (uint16_t)((uint32_t)lane | ((uint32_t)(w * 32 + __ffs(m) - 1) << 6));
    } else {
#pragma unroll
      for (int w = 0; w < kMaskWords; ++w) sh.mask[lane * kMaskWords + w] = mw[w];
    }
    __syncthreads();
    auto cand_of = [&](uint32_t p, int &Lc, int &e) {
      if (listed) {
        const uint32_t c = sh.cand[p];
        Lc = (int)(c & 63u);
        e = (int)(c >> 6);
      } else {
        candidate(sh, nwords, p, Lc, e);
      }
    };
    if constexpr (kInt) {
      // 3.-5. segment-integrated kernel: every window segment within the
      // cutoff of the cell gives one record (cell, segment).  The (candidate,
      // segment) pairs are spread over the lanes, 64 at a time; the pairs in
      // reach go, in order, to a ring of descriptors whose weights are then
      // evaluated 64 at a time.  Records follow candidate order, so they stay
      // sorted by cell.
      __shared__ IntScratch si;
      // smallest eps of each staged window, rounded down to FP32: with the
      // largest (rounded up) it brackets eps_seg of every segment
      for (uint32_t e = lane; e < ne; e += 64) si.emin[e] = 0x7f7fffffu;  // FLT_MAX
      __syncthreads();
      for (int q = lane; q < npts; q += 64) {
        const int e = staged_entry(sh.wx[q]);
        const int64_t k = sh.e_k0[e] + (sh.e_i1[e] < 0 ? 0 : sh.e_i0[e]) + (q - sh.e_pt0[e]);
        const double ep = Eps[k];
        float ef = (float)ep;
        if ((double)ef > ep) ef = nextafterf(ef, 0.f);
        atomicMin(&si.emin[e], __float_as_uint(fmaxf(ef, 0.f)));
      }
      __syncthreads();
      // upper bound of the item's records (every window segment of every
      // candidate); the unused tail goes back to the wave's block at the end
      uint32_t ub = 0;
      for (uint32_t p0 = 0; p0 < total; p0 += 64) {
        const uint32_t p = p0 + lane;
        int Lc = lane, e = 0;
        uint32_t n = 0;
        if (p < total) {
          cand_of(p, Lc, e);
          n = sh.e_i1[e] < 0 ? 1u : (uint32_t)(sh.e_i1[e] - sh.e_i0[e] + 1);
          if (n > kIntMaxSeg) {
            set_overflow(W, 16u);  // reported as a per-tile limit
            n = 0;
          }
        }
        uint32_t tot;
        wave_excl_scan_u32(n, tot);
        ub += tot;
      }
      if (!multi) reserve(ub);
      uint32_t qh = 0, qt = 0;  // ring head and tail (wave-uniform)
      // weights of ring entries qh .. qh + n - 1, one per lane
      auto drain = [&](uint32_t n) {
        const bool on = (uint32_t)lane < n;
        uint32_t d = 0, pos = 0;
        if (on) {
          d = si.qd[(qh + lane) & (kIntRing - 1)];
          pos = si.qp[(qh + lane) & (kIntRing - 1)];
        }
        const int Lc = (int)(d & 63u), e = (int)((d >> 6) & 255u), j = (int)(d >> 14);
        const double pcx = __shfl(cx, Lc, 64), pcy = __shfl(cy, Lc, 64), pcz = __shfl(cz, Lc, 64);
        const double pv = __shfl(v, Lc, 64);
        if (on) {
          const int k0 = sh.e_k0[e], i0 = sh.e_i0[e], i1 = sh.e_i1[e];
          const int pt0 = e < n_staged ? sh.e_pt0[e] : -1;
          auto acc = [&](int q, double av) {
            long long h;
            unsigned long long l;
            if (pt0 >= 0) {
              fx_encode(av, staged_exp(sh.wx[pt0 + q]), h, l);
              atomicAdd((unsigned long long *)&sh.ahi[pt0 + q], (unsigned long long)h);
              atomicAdd(&sh.alo[pt0 + q], l);
            } else {
              const int64_t node = pbase + k0 + (i1 < 0 ? 0 : i0) + q;
              fx_encode(av, W.wexp[node], h, l);
              atomicAdd((unsigned long long *)&W.w_hi[node], (unsigned long long)h);
              atomicAdd(&W.w_lo[node], l);
            }
          };
          unsigned char *r = W.rec + rbase + (unsigned long long)pos * rsz;
          if (i1 < 0) {
            // single-CV beam: the point kernel of the nearest rule
            const gptr<double> P = Psp + 3 * (int64_t)k0;
            double a0, a1;
            pair_weights(kSplit ? ALP_PREC_FP32_SPLIT : ALP_PREC_FP64, 0.0, sqdist_exact(pcx, pcy, pcz, P[0], P[1], P[2]), Eps[k0], a0, a1);
            acc(0, a0 * pv);
            if (rec_ok) write_record(r, rsz, (uint32_t)Lc | kRecSingle, (uint32_t)(pbase + k0), a0, 0.0);
          } else {
            const gptr<double> A = Psp + 3 * ((int64_t)k0 + i0 + j);
            const gptr<double> E = Eps + (int64_t)k0 + i0 + j;
            double a0, a1;
            if constexpr (kSplit)
              seg_int_weights_split(pcx, pcy, pcz, A[0], A[1], A[2], A[3], A[4], A[5], 0.5 * (E[0] + E[1]), a0, a1);
            else
              seg_int_weights(pcx, pcy, pcz, A[0], A[1], A[2], A[3], A[4], A[5], 0.5 * (E[0] + E[1]), a0, a1);
            acc(j, a0 * pv);
            acc(j + 1, a1 * pv);
            if (rec_ok) write_record(r, rsz, (uint32_t)Lc, (uint32_t)(pbase + k0 + i0 + j), a0, a1);
          }
        }
        qh += n;
      };
      for (uint32_t p0 = 0; p0 < total; p0 += 64) {
        const uint32_t p = p0 + lane;
        int Lc = lane, e = 0;
        uint32_t n = 0;
        if (p < total) {
          cand_of(p, Lc, e);
          n = sh.e_i1[e] < 0 ? 1u : (uint32_t)(sh.e_i1[e] - sh.e_i0[e] + 1);
          if (n > kIntMaxSeg) {
            set_overflow(W, 16u);  // reported as a per-tile limit
            n = 0;
          }
        }
        uint32_t T;
        const uint32_t pre = wave_excl_scan_u32(n, T);
        si.lc[lane] = (uint8_t)Lc;
        si.ent[lane] = (uint8_t)e;
        si.pre[lane] = pre;
        __syncthreads();
        for (uint32_t t0 = 0; t0 < T; t0 += 64) {
          const uint32_t t = t0 + lane;
          const bool on = t < T;
          // the candidate owning pair t: the last o with pre[o] <= t
          int o = 0;
          if (on) {
            int lo = 0, hi = 63;
            while (lo < hi) {
              const int mid = (lo + hi + 1) >> 1;
              if (si.pre[mid] <= t) lo = mid;
              else hi = mid - 1;
            }
            o = lo;
          }
          const int cl = si.lc[o], ce = si.ent[o];
          const int j = (int)(t - si.pre[o]);
          const double pcx = __shfl(cx, cl, 64), pcy = __shfl(cy, cl, 64), pcz = __shfl(cz, cl, 64);
          bool in = false;
          if (on) {
            const int k0 = sh.e_k0[ce], i0 = sh.e_i0[ce], i1 = sh.e_i1[ce];
            if (i1 < 0) {
              const gptr<double> P = Psp + 3 * (int64_t)k0;
              in = inside_cutoff(sqdist_exact(pcx, pcy, pcz, P[0], P[1], P[2]), Eps[k0]);
            } else {
              const gptr<double> E = Eps + (int64_t)k0 + i0 + j;
              const int pt0 = ce < n_staged ? sh.e_pt0[ce] : -1;
              bool out = false, sure_in = false;
              if (pt0 >= 0) {
                // FP32 distance from the staged points: a segment clearly
                // beyond the cutoff (by more than the FP32 error allowance)
                // is out, one clearly inside it is in (a non-zero FP32 length
                // implies distinct FP64 end points); the rest take the exact
                // FP64 test, whose decision both shortcuts reproduce
                const float4 A = sh.sa[pt0 + j], B = sh.sa[pt0 + j + 1];
                const float qx = (float)(pcx - ctx), qy = (float)(pcy - cty), qz = (float)(pcz - ctz);
                const float ex = B.x - A.x, ey = B.y - A.y, ez = B.z - A.z;
                float dx = qx - A.x, dy = qy - A.y, dz = qz - A.z;
                const float sg = __saturatef((dx * ex + dy * ey + dz * ez) * A.w);
                dx -= sg * ex;
                dy -= sg * ey;
                dz -= sg * ez;
                const float d2 = dx * dx + dy * dy + dz * dz;
                // eps_seg lies between the window's smallest and largest eps
                const float eh = __uint_as_float(sh.e_em[ce]), el = __uint_as_float(si.emin[ce]);
                out = d2 > 9.0f * eh * eh * (1.0f + 0x1p-20f) + sh.e_dabs[ce];
                sure_in = A.w > 0.f && d2 < 9.0f * el * el * (1.0f - 0x1p-20f) - sh.e_dabs[ce];
              }
              double es64;
              in = sure_in ||
                   (!out && seg_in_reach(Psp + 3 * ((int64_t)k0 + i0 + j), E[0], E[1], pcx, pcy, pcz, es64));
            }
          }
          const uint64_t bal = ballot64(in);
          if (in) {
            const uint32_t rank = lanemask_lt_popc(bal);
            si.qd[(qt + rank) & (kIntRing - 1)] = (uint32_t)cl | ((uint32_t)ce << 6) | ((uint32_t)j << 14);
            si.qp[(qt + rank) & (kIntRing - 1)] = nreal + rank;
          }
          const uint32_t nin = (uint32_t)__popcll(bal);
          nreal += nin;
          qt += nin;
          __syncthreads();
          if (qt - qh >= 64) drain(64);
        }
        __syncthreads();
      }
      if (qt > qh) drain(qt - qh);
      // give back the unused tail of the reservation
      if (!multi) blk_cur = rbase + (((unsigned long long)nreal * rsz + 15ull) & ~15ull);
    } else {
      // record space for up to `total` pairs (one per candidate)
      if (!multi) reserve(total);
      // 3.-5. candidate pairs, 64 per round
      for (uint32_t p0 = 0; p0 < total; p0 += 64) {
        const uint32_t p = p0 + lane;
        const bool act = p < total;
        int Lc = lane, e = 0;
        if (act) cand_of(p, Lc, e);
        // the candidate's cell, from the lane that holds it
        const double pcx = __shfl(cx, Lc, 64), pcy = __shfl(cy, Lc, 64), pcz = __shfl(cz, Lc, 64);
        const double pv = __shfl(v, Lc, 64);
        bool in = false, guard = false;
        int bi = 0, single = 0;
        double a0 = 0.0, a1 = 0.0;
        if (act) {
          const int pt0 = (int)e < n_staged ? sh.e_pt0[e] : -1;
          const int k0 = sh.e_k0[e], i0 = sh.e_i0[e], i1 = sh.e_i1[e];
          double bs = 0.0, br2 = INFINITY, ej = 1.0;
          int bj = 0;
          if (i1 < 0) {
            single = 1;
            const gptr<double> P = Psp + 3 * (int64_t)k0;
            br2 = sqdist_exact(pcx, pcy, pcz, P[0], P[1], P[2]);
            ej = Eps[k0];
          } else {
            const int nseg = i1 - i0 + 1;
            const gptr<double> X = Psp + 3 * ((int64_t)k0 + i0);
            bool full = pt0 < 0;
            if (!full) {
              // FP32 ranking: the three smallest (distance, index) keys
              const float qx = (float)(pcx - ctx), qy = (float)(pcy - cty), qz = (float)(pcz - ctz);
              uint32_t k1 = ~0u, k2 = ~0u, k3 = ~0u;
              for (int j = 0; j < nseg; ++j) {
                // both end points from LDS (carrying B over as the next A
                // costs register moves; LDS reads are not the binding resource)
                const float4 A = sh.sa[pt0 + j], B = sh.sa[pt0 + j + 1];
                const float ex = B.x - A.x, ey = B.y - A.y, ez = B.z - A.z;
                float dx = qx - A.x, dy = qy - A.y, dz = qz - A.z;
                const float t = dx * ex + dy * ey + dz * ez;
                const float sg = __builtin_amdgcn_fmed3f(t * A.w, 0.f, 1.f);  // clamp to [0, 1]
                dx -= sg * ex;
                dy -= sg * ey;
                dz -= sg * ez;
                const float d2 = dx * dx + dy * dy + dz * dz;
                // (the high three bytes of d2 and j as the low byte: one
                // v_perm_b32, equal to (d2 & ~kSegIdxMask) | j)
                const uint32_t key = __builtin_amdgcn_perm(__float_as_uint(d2), (uint32_t)j, 0x07060500u);
                // insert into k1 <= k2 <= k3: the median of (k_i, k_i+1, key)
                // is the new i+1-th smallest
                k3 = umed3(k2, k3, key);
                k2 = umed3(k1, k2, key);
                k1 = min(k1, key);
              }
              // keys drop 8 mantissa bits (relative 2^-15): the band below holds
              // every segment whose exact distance can reach the best one
              const float b1 = __uint_as_float(k1 & ~kSegIdxMask);
              const float dl = b1 * 0x1p-14f + sh.e_dabs[e];
              const float band = (b1 + 2.0f * dl) * (1.0f + 0x1p-20f);
              full = k3 != ~0u && __uint_as_float(k3 & ~kSegIdxMask) <= band;
              guard = full;
              if (!full) {
                // the one or two segments in the band are evaluated exactly;
                // their node widths are loaded with their end points, not
                // after the choice
                int j1 = (int)(k1 & kSegIdxMask);
                bool two = k2 != ~0u && __uint_as_float(k2 & ~kSegIdxMask) <= band;
                if (two) {
                  const int j2 = (int)(k2 & kSegIdxMask);
                  if (j2 == j1 + 1 || j2 + 1 == j1) {
                    // Neighbouring segments a (A -> V) and b (V -> B) meet at V.
                    // If the cell's projection falls before V on a's line
                    // (t_a < 1) and not after V on b's (t_b <= 0), a's closest
                    // point lies strictly closer than V, which is b's closest
                    // point: a wins; mirrored for b.  The FP32 parameters are
                    // trusted only beyond 2^-19 ((R/|e|)^2 + R/|e|) + 2^-20 of
                    // the thresholds, R the largest coordinate of the window:
                    // a bound, with a margin of 16 and more, on their error from
                    // rounding and on the zone where the exact squared
                    // distances differ by less than their FP64 rounding.
                    const int ja = min(j1, j2);
                    const float4 Aa = sh.sa[pt0 + ja], Vv = sh.sa[pt0 + ja + 1], Bb = sh.sa[pt0 + ja + 2];
                    if (Aa.w > 0.f && Vv.w > 0.f) {
                      const float qx = (float)(pcx - ctx), qy = (float)(pcy - cty), qz = (float)(pcz - ctz);
                      const float R2 = sh.e_dabs[e] * 0x1p14f;  // R^2 of the window (the allowance is 2^-14 R^2)
                      const float ax = Vv.x - Aa.x, ay = Vv.y - Aa.y, az = Vv.z - Aa.z;
                      const float bx = Bb.x - Vv.x, by = Bb.y - Vv.y, bz = Bb.z - Vv.z;
                      // t_a - 1 and t_b times |e|^2 (1/|e|^2 is each segment's staged
                      // w; its hardware reciprocal is within 1 ulp, far inside the
                      // 2^-20 |e|^2 term of the margins)
                      const float la = __builtin_amdgcn_rcpf(Aa.w), lb = __builtin_amdgcn_rcpf(Vv.w);
                      const float ga = (qx - Aa.x) * ax + (qy - Aa.y) * ay + (qz - Aa.z) * az - la;
                      const float gb = (qx - Vv.x) * bx + (qy - Vv.y) * by + (qz - Vv.z) * bz;
                      const float ra = R2 * Aa.w, rb = R2 * Vv.w;  // (R/|e|)^2
                      const float da = (0x1p-19f * (ra + __builtin_amdgcn_sqrtf(ra)) + 0x1p-20f) * la;
                      const float db = (0x1p-19f * (rb + __builtin_amdgcn_sqrtf(rb)) + 0x1p-20f) * lb;
                      if (ga < -da && gb < -db) {
                        j1 = ja;
                        two = false;
                      } else if (ga > da && gb > db) {
                        j1 = ja + 1;
                        two = false;
                      }
                    }
                  }
                }
                guard = two;
                const gptr<double> E = Eps + (int64_t)k0 + i0;
                double e0 = E[j1], e1 = E[j1 + 1];
                exact_scan(X, j1, j1, pcx, pcy, pcz, bj, bs, br2);
                if (two) {
                  const int j2 = (int)(k2 & kSegIdxMask);
                  const double f0 = E[j2], f1 = E[j2 + 1];
                  int cj = j2;
                  double cs2 = 0.0, cr2 = INFINITY;
                  exact_scan(X, j2, j2, pcx, pcy, pcz, cj, cs2, cr2);
                  if (cr2 < br2 || (cr2 == br2 && j2 < bj)) {
                    br2 = cr2;
                    bj = j2;
                    bs = cs2;
                    e0 = f0;
                    e1 = f1;
                  }
                }
                ej = eps_at(bs, e0, e1);
              }
            }
            if (full) {
              br2 = INFINITY;
              bj = 0;
              bs = 0.0;
              exact_scan(X, 0, nseg - 1, pcx, pcy, pcz, bj, bs, br2);
              const gptr<double> E = Eps + (int64_t)k0 + i0;
              ej = eps_at(bs, E[bj], E[bj + 1]);
            }
          }
          in = inside_cutoff(br2, ej);
          if (in) {
            pair_weights(kSplit ? ALP_PREC_FP32_SPLIT : ALP_PREC_FP64, bs, br2, ej, a0, a1);
            const int64_t node = pbase + k0 + (single ? 0 : i0 + bj);
            long long h0, h1 = 0;
            unsigned long long l0, l1 = 0;
            if (pt0 >= 0) {
              fx_encode(a0 * pv, staged_exp(sh.wx[pt0 + bj]), h0, l0);
              atomicAdd((unsigned long long *)&sh.ahi[pt0 + bj], (unsigned long long)h0);
              atomicAdd(&sh.alo[pt0 + bj], l0);
              if (!single) {
                fx_encode(a1 * pv, staged_exp(sh.wx[pt0 + bj + 1]), h1, l1);
                atomicAdd((unsigned long long *)&sh.ahi[pt0 + bj + 1], (unsigned long long)h1);
                atomicAdd(&sh.alo[pt0 + bj + 1], l1);
              }
            } else {
              fx_encode(a0 * pv, W.wexp[node], h0, l0);
              atomicAdd((unsigned long long *)&W.w_hi[node], (unsigned long long)h0);
              atomicAdd(&W.w_lo[node], l0);
              if (!single) {
                fx_encode(a1 * pv, W.wexp[node + 1], h1, l1);
                atomicAdd((unsigned long long *)&W.w_hi[node + 1], (unsigned long long)h1);
                atomicAdd(&W.w_lo[node + 1], l1);
              }
            }
            bi = (int)node;  // global node index for the record
          }
        }
        const uint64_t bal = ballot64(act && in);
        if (act && in && rec_ok) {
          const unsigned long long at = rbase + (unsigned long long)(nreal + lanemask_lt_popc(bal)) * rsz;
          unsigned char *r = W.rec + at;
          write_record(r, rsz, (uint32_t)Lc | (single ? kRecSingle : 0u), (uint32_t)bi, a0, a1);
        }
        nreal += (uint32_t)__popcll(bal);
        acc_guard += (unsigned long long)__popcll(ballot64(act && guard));
      }
    }
    __syncthreads();
    // flush the staged node accumulators
    for (int q = lane; q < npts; q += 64) {
      long long h = sh.ahi[q];
      unsigned long long l = sh.alo[q];
      if (h == 0 && l == 0) continue;
      const int e = staged_entry(sh.wx[q]);
      const int64_t node = pbase + sh.e_k0[e] + (sh.e_i1[e] < 0 ? 0 : sh.e_i0[e]) + (q - sh.e_pt0[e]);
      h += (long long)(l >> kLoBits);
      l &= (1ull << kLoBits) - 1ull;
      atomicAdd((unsigned long long *)&W.w_hi[node], (unsigned long long)h);
      atomicAdd(&W.w_lo[node], l);
    }
    if constexpr (!kMulti) break;
    g0 += ne;
    if (g0 >= ne_all) break;
    __syncthreads();  // the previous group's scratch is done with
    }  // entry groups
    if (multi) blk_cur = rbase + (((unsigned long long)nreal * rsz + 15ull) & ~15ull);
    if (lane == 0) {
      // bases are 16-byte aligned: bits 0 and 2 carry the record size (24
      // and 12 bytes), bit 1 marks an item whose cells have records in
      // several runs (one per entry group)
      W.rec_base[item] = rbase | (rsz == 24 ? 1ull : 0ull) | (rsz == 12 ? 4ull : 0ull) | (multi ? 2ull : 0ull);
      W.rec_cnt[item] = rec_ok ? nreal : 0u;
    }
    acc_pairs += nreal;
    __syncthreads();
  }
  if (lane == 0 && acc_case >= 0 && acc_pairs)
    atomicAdd((unsigned long long *)(W.cnt + kCnt * acc_case + 5), acc_pairs);
  if (lane == 0 && acc_case >= 0 && acc_guard)
    atomicAdd((unsigned long long *)(W.cnt + kCnt * acc_case + 8), acc_guard);
}

__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(4)))
void k_weights(StepLaunch L) {
  weights_pass<false, true, false>(L);
}
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(4)))
void k_weights64(StepLaunch L) {
  weights_pass<false, false, false>(L);
}
// the items taken in entry groups (tiles with more than kMaxEntries entries,
// or whose windows hold more points than the staging area), one kernel per
// rule and precision with the register budgets of the common kernels; they
// take the list of such items from a work queue of their own, so a step
// without any launches waves that return at once
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(4)))
void k_weights_grp(StepLaunch L) {
  weights_pass<false, true, true>(L);
}
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(4)))
void k_weights_grp64(StepLaunch L) {
  weights_pass<false, false, true>(L);
}
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(4)))
void k_weights_grp_int(StepLaunch L) {
  weights_pass<true, true, true>(L);
}
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(2)))
void k_weights_grp_int64(StepLaunch L) {
  weights_pass<true, false, true>(L);
}

// the integrated rule, one kernel per precision: the split one (FP32
// Gaussian integrals) runs at four waves per SIMD; the FP64 one (erf, erfc,
// expm1 in FP64) needs more registers, two waves per SIMD
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(4)))
void k_weights_int(StepLaunch L) {
  weights_pass<true, true, false>(L);
}
__global__ __attribute__((amdgpu_flat_work_group_size(64, 64), amdgpu_waves_per_eu(2)))
void k_weights_int64(StepLaunch L) {
  weights_pass<true, false, false>(L);
}

// The common kernels and the grouped ones take disjoint items from their own
// queues and share only the record allocator, the node sums and the
// counters, all updated atomically, so the two sets may run on two streams.
void launch_weights_main(const StepLaunch &L, hipStream_t st) {
  const dim3 g((unsigned)L.grid_weights);
  if (L.near_split) hipLaunchKernelGGL(k_weights, g, dim3(64), 0, st, L);
  if (L.near_fp64) hipLaunchKernelGGL(k_weights64, g, dim3(64), 0, st, L);
  if (L.int_split) hipLaunchKernelGGL(k_weights_int, g, dim3(64), 0, st, L);
  if (L.int_fp64) hipLaunchKernelGGL(k_weights_int64, g, dim3(64), 0, st, L);
}
void launch_weights_grouped(const StepLaunch &L, hipStream_t st) {
  const dim3 g((unsigned)L.grid_weights);
  if (L.near_split) hipLaunchKernelGGL(k_weights_grp, g, dim3(64), 0, st, L);
  if (L.near_fp64) hipLaunchKernelGGL(k_weights_grp64, g, dim3(64), 0, st, L);
  if (L.int_split) hipLaunchKernelGGL(k_weights_grp_int, g, dim3(64), 0, st, L);
  if (L.int_fp64) hipLaunchKernelGGL(k_weights_grp_int64, g, dim3(64), 0, st, L);
}

// ------------------------------------------------------------------- norm --
// w_k from the exact accumulators, f_hat_k = f_k L_k / w_k (0 and counted
// when w_k = 0).
__global__ void k_norm(StepLaunch L) {
  Work W = L.w;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool act = g < W.n_points;
  bool zero = false;
  int c = 0;
  if (act) {
    c = case_of(L.pbase, L.n_cases, g);
    const CaseDev &cs = L.cases[c];
    int64_t k = g - cs.point_base;
    double w = fx_decode(W.w_hi[g], W.w_lo[g], W.wexp[g]);
    const double *f = cs.f ? cs.f + 3 * k : W.f + 3 * g;
    double Lk = cs.L[k];
    double fh[3];
    zero = !(w != 0.0);
    for (int a = 0; a < 3; ++a) fh[a] = zero ? 0.0 : (f[a] * Lk) / w;
    for (int a = 0; a < 3; ++a) W.fhat[3 * g + a] = fh[a];
    if (cs.w) cs.w[k] = w;
    if (cs.fhat)
      for (int a = 0; a < 3; ++a) cs.fhat[3 * k + a] = fh[a];
  }
  int c0 = __shfl(c, 0, 64);
  if (__all(!act || c == c0)) wave_count_add(W.cnt + kCnt * c0 + 3, act && zero);
  else if (act && zero) atomicAdd((unsigned long long *)(W.cnt + kCnt * c + 3), 1ull);
}

void launch_norm(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_points == 0) return;
  hipLaunchKernelGGL(k_norm, dim3((unsigned)((L.w.n_points + 63) / 64)), dim3(64), 0, st, L);
}

// -------------------------------------------------------------- beam sums --
// F_beam = sum_k f_k L_k and sum_k |f_k L_k| per case, by blocks of points of
// one case with a fixed reduction order.
constexpr int kSumBlock = 256;
__global__ __launch_bounds__(kSumBlock) void k_beam_sums(StepLaunch L) {
  Work W = L.w;
  __shared__ double s[4][kSumBlock];
  int pb = blockIdx.x;
  int c = W.pblock_case[pb];
  const CaseDev &cs = L.cases[c];
  int64_t k0 = W.pblock_range[2 * pb], k1 = W.pblock_range[2 * pb + 1];
  double r[4] = {0, 0, 0, 0};
  for (int64_t k = k0 + threadIdx.x; k < k1; k += kSumBlock) {
    const double *f = cs.f ? cs.f + 3 * k : W.f + 3 * (cs.point_base + k);
    double Lk = cs.L[k];
    double fl[3] = {f[0] * Lk, f[1] * Lk, f[2] * Lk};
    r[0] += fl[0];
    r[1] += fl[1];
    r[2] += fl[2];
    r[3] += sqrt(fl[0] * fl[0] + fl[1] * fl[1] + fl[2] * fl[2]);
  }
  for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = r[q];
  __syncthreads();
  for (int w = kSumBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) W.beam_part[4 * pb + q] = s[q][0];
}

// per case: F_beam, sum |f L| and the fixed-point exponent of the fluid-side
// sum (every partial of sum_j S_j V_j is bounded by sum_k |f_k L_k|); one
// block per case, each thread sums a fixed stride of the case's point blocks,
// then a fixed tree
__global__ __launch_bounds__(kSumBlock) void k_finalize_beam(StepLaunch L) {
  Work W = L.w;
  __shared__ double s[4][kSumBlock];
  const int c = blockIdx.x;
  double r[4] = {0, 0, 0, 0};
  for (int pb = threadIdx.x; pb < W.n_pblocks; pb += kSumBlock)
    if (W.pblock_case[pb] == c)
      for (int q = 0; q < 4; ++q) r[q] += W.beam_part[4 * pb + q];
  for (int q = 0; q < 4; ++q) s[q][threadIdx.x] = r[q];
  __syncthreads();
  for (int w = kSumBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int q = 0; q < 4; ++q) s[q][threadIdx.x] += s[q][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    double *d = W.diag_out + 16 * c;
    for (int q = 0; q < 4; ++q) d[q] = s[q][0];
    W.F_exp[c] = s[3][0] > 0.0 ? ilogb(s[3][0]) + 2 : 0;
  }
}

void launch_beam_sums(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_pblocks > 0)
    hipLaunchKernelGGL(k_beam_sums, dim3(L.w.n_pblocks), dim3(kSumBlock), 0, st, L);
  hipLaunchKernelGGL(k_finalize_beam, dim3(L.n_cases), dim3(kSumBlock), 0, st, L);
}

// ----------------------------------------------------------------- spread --
// Eq. (23): S_j = -sum over the cell's pairs (beam order) of
// a0 f_hat_i + a1 f_hat_i+1, from the records of the weights pass (the same
// a0, a1 that built w_k, so the transferred force balances exactly).  The
// records of a work item are sorted by cell, so each cell owns one contiguous
// run; its lane sums the run in record order.  Every cell of an active tile
// is written.
// s_waitcnt operand waiting for vmcnt 0 only (expcnt 7 and lgkmcnt 15 are
// the fields' maxima, i.e. no wait on them)
constexpr unsigned kWaitVmcnt0 = 0x0F70u;

// The record counts and bases of the work items, and the workgroup's item
// counter in LDS, for the record cursor (lane 0 takes the ticket; an LDS
// atomic waits on the LDS counter only, not on the wave's global loads).
struct ItemRecs {
  const uint32_t *c;
  const unsigned long long *b;
  uint32_t *ctr;
  int lane;
  __device__ __forceinline__ uint32_t cnt(uint32_t i) const { return sload(c + i); }
  __device__ __forceinline__ uint64_t base(uint32_t i) const { return sload(b + i); }
  __device__ __forceinline__ uint32_t ticket() const {
    uint32_t t = 0;
    if (lane == 0) t = atomicAdd(ctr, 1u);
    return (uint32_t)__builtin_amdgcn_readfirstlane((int)t);
  }
};

// Order of one wave's own LDS accesses across lanes (each wave has its own
// scratch; a workgroup barrier would hold waves that are at other items).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct SpreadScratch {
  // per-record contributions; at an item's end, its cells' source rows in
  // sorted order (64 rows of 24 bytes), read back in 16-byte pieces
  alignas(16) double cc[3][kSpreadChunk];
  uint16_t first[64], last[64];  // run of each cell inside the chunk (last exclusive)
  uint32_t pc[64];               // caller index of each cell of the item (at its end)
};
static_assert(sizeof(double) * 3 * kSpreadChunk == 24 * 64, "one 24-byte source row per cell");

// A chunk in flight: its place in the stream, its item's descriptor and the
// first 24 bytes of this lane's record (every record size is read the same
// way, so every pass issues the same loads and the waits for one chunk leave
// the next chunk's loads in flight; a shorter record's tail words belong to
// the next record or to the slack of the record area, and are not used).
struct SpreadChunk {
  RecChunk k;
  Item it;
  uint32_t d[6];
};

__device__ __forceinline__ void spread_issue(const Work &W, const ItemRecs &src, RecCursor &cur, uint32_t n_items,
                                             int lane, SpreadChunk &o) {
  o.k = rec_take(src, cur, n_items);
  if (o.k.item < n_items) {
    const Item *ip = W.item + o.k.item;
    o.it.c0 = sload(&ip->c0);
    o.it.c1 = sload(&ip->c1);
    o.it.cs = sload(&ip->cs);
  }
  const uint64_t at = rec_lane(o.k, n_items, lane);
  const uint32_t *p = (const uint32_t *)(W.rec + (at == kRecNone ? 0ull : at));
#pragma unroll
  for (int q = 0; q < 6; ++q) o.d[q] = to_global(p)[q];
}

// A chunk's records decoded: what the pass that sums it needs (a lane
// without a record has cl = ~0 and node 0).
struct SpreadDec {
  RecChunk k;
  Item it;
  uint32_t nch, cl, node, sgl;
  double a0, a1;
};

__device__ __forceinline__ void spread_decode(SpreadChunk &X, int lane, SpreadDec &D) {
  // every word is taken, whatever the record size, so that no register of X
  // is left with its load counted as in flight
  asm volatile("" : "+v"(X.d[0]), "+v"(X.d[1]), "+v"(X.d[2]), "+v"(X.d[3]), "+v"(X.d[4]), "+v"(X.d[5]));
  D.k = X.k;
  D.it = X.it;
  const uint32_t p0 = X.k.p0, rn = X.k.rn;
  D.nch = rn > p0 ? min(rn - p0, (uint32_t)kSpreadChunk) : 0u;
  const uint32_t bytes = rec_bytes(X.k.rb);
  uint32_t cl = X.d[0] & 63u, node, sgl;
  double a0, a1;
  if (bytes == 12u) {
    sgl = (X.d[0] & 64u) ? 1u : 0u;
    node = X.d[0] >> kRecNodeShift;
    a0 = (double)__uint_as_float(X.d[1]);
    a1 = (double)__uint_as_float(X.d[2]);
  } else {
    sgl = (X.d[0] & kRecSingle) ? 1u : 0u;
    node = X.d[1];
    if (bytes == 24u) {
      a0 = __hiloint2double((int)X.d[3], (int)X.d[2]);
      a1 = __hiloint2double((int)X.d[5], (int)X.d[4]);
    } else {
      a0 = (double)__uint_as_float(X.d[2]);
      a1 = (double)__uint_as_float(X.d[3]);
    }
  }
  if ((uint32_t)lane >= D.nch) {
    cl = ~0u;
    node = 0;
    sgl = 1u;
    a0 = 0.0;
    a1 = 0.0;
  }
  D.cl = cl;
  D.node = node;
  D.sgl = sgl;
  D.a0 = a0;
  D.a1 = a1;
}

constexpr int kSpreadThreads = 64 * (int)kSpreadGroupWaves;
__global__ __attribute__((amdgpu_flat_work_group_size(kSpreadThreads, kSpreadThreads), amdgpu_waves_per_eu(8)))
void k_spread(StepLaunch L) {
  Work W = L.w;
  __shared__ SpreadScratch shs[kSpreadGroupWaves];
  __shared__ uint32_t group_ctr;
  const int lane = threadIdx.x & 63;
  SpreadScratch &sh = shs[threadIdx.x >> 6];
  if (threadIdx.x == 0) group_ctr = 0u;
  __syncthreads();  // the workgroup's only barrier: its waves then go their own ways
  const uint32_t n_items = (uint32_t)min((int64_t)W.tile_itoff[W.n_tiles], W.cap_item);
  const ItemRecs src{W.rec_cnt, W.rec_base, &group_ctr, lane};
  RecCursor cur = rec_start(src, rec_group_base(blockIdx.x, gridDim.x), gridDim.x * kSpreadGroupWaves, n_items);
  if (cur.c.item >= n_items) return;
  // per-wave accumulation (exact fixed point, flushed when the case changes)
  int acc_case = -1;
  unsigned long long acc_band = 0;
  long long fh = 0;  // lanes 0..2 hold x, y, z
  unsigned long long fl = 0;
  auto flush = [&]() {
    if (acc_case < 0) return;
    if (lane == 0 && acc_band) atomicAdd((unsigned long long *)(W.cnt + kCnt * acc_case + 4), acc_band);
    if (lane < 3 && (fh || fl)) {
      fh += (long long)(fl >> kLoBits);
      fl &= (1ull << kLoBits) - 1ull;
      atomicAdd((unsigned long long *)&W.F_hi[3 * acc_case + lane], (unsigned long long)fh);
      atomicAdd(&W.F_lo[3 * acc_case + lane], fl);
    }
  };
  sh.first[lane] = 0;
  sh.last[lane] = 0;
  // the chunk stream, one chunk ahead of the one being summed.  The record
  // registers A and B alternate: a chunk's loads fill its registers, which
  // are decoded at the end of the pass before the one that sums it (after
  // that pass has waited for its own force loads, issued after these) and
  // refilled by the pass that sums it.  So no record register is read or
  // copied while its load is in flight.
  SpreadChunk A, B;
  spread_issue(W, src, cur, n_items, lane, A);
  spread_issue(W, src, cur, n_items, lane, B);
  SpreadDec D;
  spread_decode(A, lane, D);
  wave_sync();
  double S0 = 0.0, S1 = 0.0, S2 = 0.0;  // the lane's cell, over the item's chunks so far
  bool any = false;
  // sum the chunk decoded in D (it came from X), refill X with the chunk
  // after Y's, then decode Y
  auto pass = [&](SpreadChunk &X, SpreadChunk &Y) -> bool {
    if (D.k.item >= n_items) return false;
    const Item it = D.it;
    const uint32_t p0 = D.k.p0, rn = D.k.rn;
    const uint64_t rb = D.k.rb;
    if (p0 == 0 && it.cs != acc_case) {
      flush();
      // (the compiler cannot wait for one load while atomics of unknown
      // order are in flight: the rare path that issues them waits for them)
      __builtin_amdgcn_s_waitcnt(kWaitVmcnt0);
      acc_case = it.cs;
      acc_band = 0;
      fh = 0;
      fl = 0;
    }
    const uint32_t nch = D.nch;
    const bool last = p0 + (uint32_t)kSpreadChunk >= rn;
    const CaseDev *cp = L.cases + it.cs;
    const double *vs = sload(&cp->m.vs);
    const uint32_t *perm = sload(&cp->m.perm);
    // this lane's record
    const uint32_t j = (uint32_t)lane;
    const bool has = j < nch;
    const uint32_t cl = D.cl;
    const bool single = D.sgl != 0u;
    const double a0 = D.a0, a1 = D.a1;
    // f_hat of the record's nodes (the force array has two nodes of slack,
    // so the second node's address is valid for single-CV records as well),
    // and, in the item's last pass, the volume and caller index of the
    // lane's cell.  Every load of a pass is used in that pass: a register
    // with a load in flight is never left for the compiler to wait on later.
    const gptr<double> fp = to_global(W.fhat) + 3 * (int64_t)D.node;
    double fq[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) fq[q] = fp[q];
    const int c = it.c0 + lane;
    const bool valid = c < it.c1;
    double v = 0.0;
    uint32_t pc = 0;
    if (last) {
      const int cr = valid ? c : it.c0;
      v = to_global(vs)[cr];
      pc = to_global(perm)[cr];
    }
    // the next chunk's loads go out before this chunk's forces are used
    // (the empty statement keeps every use of the forces, the volume and
    // the index after them)
    spread_issue(W, src, cur, n_items, lane, X);
    double f0 = fq[0], f1 = fq[1], f2 = fq[2], f3 = fq[3], f4 = fq[4], f5 = fq[5];
    asm volatile("" : "+v"(f0), "+v"(f1), "+v"(f2), "+v"(f3), "+v"(f4), "+v"(f5), "+v"(v), "+v"(pc));
    {
      // (a lane without a record has a0 = a1 = 0 and node 0: it writes a
      // zero that no run reads)
      double q0 = a0 * f0, q1 = a0 * f1, q2 = a0 * f2;
      if (!single) {
        q0 += a1 * f3;
        q1 += a1 * f4;
        q2 += a1 * f5;
      }
      sh.cc[0][j] = -q0;
      sh.cc[1][j] = -q1;
      sh.cc[2][j] = -q2;
    }
    if ((rb & 2ull) != 0ull) {
      // an item whose entries were taken in groups holds one run per group
      // for a cell.  The chunk splits into segments where the cell index
      // falls (a group starts); inside a segment the records are sorted by
      // cell, so each segment is summed like the chunk of a one-group item,
      // one segment after the other: a cell still adds its records in record
      // order (group after group, beam order inside a group).
      const uint32_t up = (uint32_t)__shfl((int)cl, lane - 1, 64);
      const uint32_t dn = (uint32_t)__shfl((int)cl, lane + 1, 64);
      const bool head = has && (j == 0 || up > cl);
      const uint64_t heads = ballot64(head);
      const uint32_t nseg = (uint32_t)__popcll(heads);
      const uint32_t seg = lanemask_lt_popc(heads) + (head ? 1u : 0u) - 1u;
      for (uint32_t sg = 0; sg < nseg; ++sg) {
        if (has && seg == sg) {
          if (j == 0 || up != cl) sh.first[cl] = (uint16_t)j;
          if (j + 1 == nch || dn != cl) sh.last[cl] = (uint16_t)(j + 1);
        }
        wave_sync();
        const uint32_t lo = sh.first[lane], hi = sh.last[lane];
        sh.first[lane] = 0;
        sh.last[lane] = 0;
        any = any || hi > lo;
        for (uint32_t q = lo; q < hi; ++q) {
          S0 += sh.cc[0][q];
          S1 += sh.cc[1][q];
          S2 += sh.cc[2][q];
        }
        wave_sync();
      }
    } else {
      // run boundaries of each cell (records are sorted by cell): the
      // neighbouring records' cells come from the neighbouring lanes
      const uint32_t up = (uint32_t)__shfl((int)cl, lane - 1, 64);
      const uint32_t dn = (uint32_t)__shfl((int)cl, lane + 1, 64);
      if (has) {
        if (j == 0 || up != cl) sh.first[cl] = (uint16_t)j;
        if (j + 1 == nch || dn != cl) sh.last[cl] = (uint16_t)(j + 1);
      }
      wave_sync();
      const uint32_t lo = sh.first[lane], hi = sh.last[lane];
      sh.first[lane] = 0;
      sh.last[lane] = 0;
      any = any || hi > lo;
      for (uint32_t q = lo; q < hi; ++q) {
        S0 += sh.cc[0][q];
        S1 += sh.cc[1][q];
        S2 += sh.cc[2][q];
      }
      wave_sync();
    }
    if (last) {
      // the item's cells are complete: write them, count the band cells and
      // add the force on the fluid (deterministic wave sum, then exact
      // accumulation)
      if (sload(&cp->write_S)) {
        // The rows go out as 16-byte pieces of the item's rows in sorted
        // order: cells that are consecutive in the caller's numbering (runs
        // along the fastest mesh axis) then take whole pieces, and one store
        // instruction covers whole runs instead of a part of every run.  A
        // piece that spans two rows which are not neighbours in the caller's
        // order is written as two words.
        double *rows = &sh.cc[0][0];
        rows[3 * lane] = S0;
        rows[3 * lane + 1] = S1;
        rows[3 * lane + 2] = S2;
        sh.pc[lane] = pc;
        wave_sync();
        double *S = sload(&cp->S);
        // a row starts on an 8-byte boundary: the pieces are two doubles
        // with that alignment
        typedef double d2a8 __attribute__((ext_vector_type(2), aligned(8)));
        const uint32_t nv = (uint32_t)(it.c1 - it.c0);
        const uint32_t npiece = (24u * nv + 15u) / 16u;
        for (uint32_t q = (uint32_t)lane; q < npiece; q += 64u) {
          const uint32_t j = (16u * q) / 24u, word = (16u * q - 24u * j) / 8u;  // row, first word (0, 1, 2)
          const d2a8 val = *reinterpret_cast<const d2a8 *>(rows + 2 * q);
          const uint32_t pj = sh.pc[j];
          const bool two_rows = word == 2u, has_next = two_rows && j + 1u < nv;
          const uint32_t pn = has_next ? sh.pc[j + 1u] : 0u;
          double *at = S + 3 * (int64_t)pj + word;
          if (!two_rows || (has_next && pn == pj + 1u)) {
            *reinterpret_cast<d2a8 *>(at) = val;
          } else {
            at[0] = val.x;
            if (has_next) S[3 * (int64_t)pn] = val.y;
          }
        }
        wave_sync();
      }
      acc_band += (unsigned long long)__popcll(ballot64(valid && any));
      const double fx = wave_sum_f64(S0 * v), fy = wave_sum_f64(S1 * v), fz = wave_sum_f64(S2 * v);
      const int fe = sload(W.F_exp + it.cs);
      if (lane < 3) {
        const double val = lane == 0 ? fx : (lane == 1 ? fy : fz);
        if (val != 0.0) {
          long long h;
          unsigned long long l;
          fx_encode(val, fe, h, l);
          fh += h;
          fl += l;
        }
      }
      S0 = 0.0;
      S1 = 0.0;
      S2 = 0.0;
      any = false;
    }
    spread_decode(Y, lane, D);
    return true;
  };
  for (;;) {
    if (!pass(A, B)) break;
    if (!pass(B, A)) break;
  }
  flush();
}

// The spread's waves take their items window by window, so its grid is
// exactly the number of workgroups the device holds at once: none waits for
// a slot.
int spread_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void *>(k_spread), kSpreadThreads, 0) !=
      hipSuccess)
    return 0;
  return nb;
}

void launch_spread(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_spread, dim3(L.grid_spread), dim3(kSpreadThreads), 0, st, L);
}

// ---------------------------------------------------------------- step end --
// One launch after the spread: the cells of tiles written at the previous
// step but not now return to zero and the tile activity becomes the new
// previous state (every block but the last, one thread per tile); the last
// block decodes each case's fluid-side force and the balance check and, in a
// captured step, writes the step's overflow word to mapped host memory, so
// that a later call can see that a replay overflowed without synchronising.
constexpr int kEndBlock = 256;
__global__ __launch_bounds__(kEndBlock) void k_step_end(StepLaunch L, uint32_t *ovf_dst) {
  Work W = L.w;
  if (blockIdx.x + 1 < gridDim.x) {
    const int64_t tg = (int64_t)blockIdx.x * kEndBlock + threadIdx.x;
    if (tg >= W.n_tiles) return;
    const int c = case_of(L.tbase, L.n_cases, tg);
    const CaseDev &cs = L.cases[c];
    if (!cs.write_S || !cs.tile_prev) return;
    const int64_t tl = tg - cs.tile_base;
    const uint8_t now = W.tile_items[tg] > 0 ? 1 : 0;
    if (cs.tile_prev[tl] && !now) {
      const uint32_t c0 = tile_cell_start(cs.m, tl), c1 = tile_cell_start(cs.m, tl + 1);
      for (uint32_t j = c0; j < c1; ++j) {
        double *S = cs.S + 3 * (int64_t)cs.m.perm[j];
        S[0] = 0.0;
        S[1] = 0.0;
        S[2] = 0.0;
      }
    }
    cs.tile_prev[tl] = now;
    return;
  }
  for (int c = threadIdx.x; c < L.n_cases; c += kEndBlock) {
    double *d = W.diag_out + 16 * c;
    const int E = W.F_exp[c];
    double F[3];
    for (int a = 0; a < 3; ++a) F[a] = fx_decode(W.F_hi[3 * c + a], W.F_lo[3 * c + a], E);
    d[4] = F[0];
    d[5] = F[1];
    d[6] = F[2];
    const double r0 = F[0] + d[0], r1 = F[1] + d[1], r2 = F[2] + d[2];
    d[7] = d[3] > 0.0 ? sqrt(r0 * r0 + r1 * r1 + r2 * r2) / d[3] : 0.0;
    d[8] = (double)W.counters[3];
  }
  if (ovf_dst && threadIdx.x == 0) {
    __atomic_store_n(ovf_dst, W.counters[3], __ATOMIC_RELEASE);
    __threadfence_system();
  }
}

void launch_step_end(const StepLaunch &L, uint32_t *ovf_dst, hipStream_t st) {
  const unsigned nz = (unsigned)((L.w.n_tiles + kEndBlock - 1) / kEndBlock);
  hipLaunchKernelGGL(k_step_end, dim3(nz + 1), dim3(kEndBlock), 0, st, L, ovf_dst);
}

}  // namespace alp
