// alp_step.hip -- the per-step kernels of the coupling operator (gfx950).
//
// One step of a batch runs, over the concatenated work of every case:
//   reset -> points_prep / beams_prep -> chunks -> chunk_tiles (count) -> scan
//   -> chunk_tiles (emit) -> tile_merge -> items     [segment binning]
//   sample -> drag                                    [eq. 16-20]
//   weights -> norm -> beam_sums -> finalize_beam      [eq. 21-22, nodal weights]
//   spread -> zero_dirty -> finalize                   [eq. 23, eq. 14 check]
//
// Work lists live on the device; the kernels that walk them are persistent
// (fixed grids that loop), so a step can be captured in a hipGraph once and
// replayed.  No floating-point atomics are used: nodal weights and the force
// balance are accumulated as exact fixed-point integers, and every source
// value is summed by one lane in beam order.
#include "alp_internal.h"

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

__device__ __forceinline__ void tile_origin(const MeshDev &m, int64_t tl, double &ox, double &oy,
                                            double &oz, int &tx, int &ty, int &tz) {
  tx = (int)(tl % m.nt[0]);
  int64_t r = tl / m.nt[0];
  ty = (int)(r % m.nt[1]);
  tz = (int)(r / m.nt[1]);
  ox = m.lo[0] + (double)tx * m.tile_len;
  oy = m.lo[1] + (double)ty * m.tile_len;
  oz = m.lo[2] + (double)tz * m.tile_len;
}

__device__ __forceinline__ uint32_t tile_cell_start(const MeshDev &m, int64_t tl) {
  return m.bin_start[tl * (int64_t)(m.T * m.T * m.T)];
}

// ------------------------------------------------------------------ reset --
// stage masks for the reset
enum { RESET_SAMPLE = 1, RESET_PROJECT = 2 };

__global__ void k_step_reset(StepLaunch L, int what) {
  Work W = L.w;
  int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (tid < 16 && (what & RESET_PROJECT)) W.counters[tid] = 0;
  for (int64_t c = tid; c < (int64_t)L.n_cases * 8; c += stride) {
    int k = (int)(c & 7);
    bool samp = k < 3;
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
  hipLaunchKernelGGL(k_step_reset, dim3(2048), dim3(256), 0, st, L, (int)(RESET_SAMPLE | RESET_PROJECT));
}
void launch_step_reset_sample(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(256), 0, st, L, (int)RESET_SAMPLE);
}
void launch_step_reset_project(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_step_reset, dim3(2048), dim3(256), 0, st, L, (int)RESET_PROJECT);
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
    atomicAdd((unsigned long long *)(W.cnt + 8 * c + 6), 1ull);
}

void launch_points_prep(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_points == 0) return;
  hipLaunchKernelGGL(k_points_prep, dim3((unsigned)((L.w.n_points + 255) / 256)), dim3(256), 0, st, L);
}

// ------------------------------------------------------------- beams prep --
__global__ void k_beams_prep(StepLaunch L) {
  Work W = L.w;
  int64_t gb = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gb >= W.n_beams) return;
  int c = case_of(L.bbase, L.n_cases, gb);
  const CaseDev &cs = L.cases[c];
  int64_t b = gb - cs.beam_base;
  int64_t k0 = cs.offsets[b], k1 = cs.offsets[b + 1];
  int64_t n = k1 - k0;
  double em = 0.0;
  for (int64_t k = k0; k < k1; ++k) em = fmax(em, cs.eps[k]);
  W.bcase[gb] = c;
  W.beps_max[gb] = em;
  int64_t nseg = n >= 2 ? n - 1 : n;
  W.bchunks[gb] = (uint32_t)((nseg + kChunkSegs - 1) / kChunkSegs);
}

void launch_beams_prep(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_beams == 0) return;
  hipLaunchKernelGGL(k_beams_prep, dim3((unsigned)((L.w.n_beams + 255) / 256)), dim3(256), 0, st, L);
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
//   (b) slab rule: a segment i is never the (lowest-index) closest segment of a
//       point X that lies behind its start plane (the previous segment ends at
//       the same vertex) or beyond its end plane while in front of the next
//       segment's start plane (the next segment is strictly closer).
// The chunk's window for a tile is [first, last] candidate segment.
__device__ __forceinline__ bool seg_candidate(const double *A, const double *B, const double *An,
                                              bool first, bool last, double R, const double *tlo,
                                              double tl, double m) {
  // (a) inflated AABB against the tile box
  for (int a = 0; a < 3; ++a) {
    double lo = fmin(A[a], B[a]) - R, hi = fmax(A[a], B[a]) + R;
    if (hi < tlo[a] - m || lo > tlo[a] + tl + m) return false;
  }
  double e[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
  double len = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
  if (!(len > 0.0)) return true;
  double half = 0.5 * tl + m;
  double ac = 0.0, hw = 0.0;
  for (int a = 0; a < 3; ++a) {
    double u = e[a] / len;
    ac += (tlo[a] + 0.5 * tl - A[a]) * u;
    hw += half * fabs(u);
  }
  double amin = ac - hw, amax = ac + hw;
  if (!first && !(amax > -m)) return false;
  if (!last && !(amin < len + m)) {
    // the point could still sit in the wedge behind the next segment's start
    if (!An) return false;
    double en[3] = {An[0] - B[0], An[1] - B[1], An[2] - B[2]};
    double ln = sqrt(en[0] * en[0] + en[1] * en[1] + en[2] * en[2]);
    if (!(ln > 0.0)) return true;
    double acn = 0.0, hwn = 0.0;
    for (int a = 0; a < 3; ++a) {
      double u = en[a] / ln;
      acn += (tlo[a] + 0.5 * tl - B[a]) * u;
      hwn += half * fabs(u);
    }
    if (!(acn - hwn < m)) return false;
  }
  return true;
}

__global__ __launch_bounds__(64) void k_chunk_tiles(StepLaunch L, int emit) {
  Work W = L.w;
  int64_t ch = blockIdx.x;
  uint32_t n_chunks = W.bchunks[W.n_beams];
  if (ch >= (int64_t)n_chunks || ch >= W.cap_chunk) return;
  int lane = threadIdx.x;
  int gb = W.chunk_beam[ch];
  const CaseDev &cs = L.cases[W.bcase[gb]];
  const MeshDev &m = cs.m;
  int64_t b = gb - cs.beam_base;
  int64_t k0 = cs.offsets[b];
  int64_t nb = cs.offsets[b + 1] - k0;
  int s0 = W.chunk_s0[ch], s1 = W.chunk_s1[ch];
  int nseg = nb >= 2 ? (int)nb - 1 : 1;
  const double *X = cs.Psp + 3 * k0;
  double R = 3.0 * W.beps_max[gb];
  double tl = m.tile_len;
  double mrg = 1e-7 * (tl + R);
  R += mrg;
  // chunk AABB
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int plast = nb >= 2 ? s1 + 1 : 0;
  for (int p = s0; p <= plast; ++p)
    for (int a = 0; a < 3; ++a) {
      lo[a] = fmin(lo[a], X[3 * p + a]);
      hi[a] = fmax(hi[a], X[3 * p + a]);
    }
  int t0[3], t1[3];
  int64_t ntile = 1;
  for (int a = 0; a < 3; ++a) {
    double f0 = floor((lo[a] - R - m.lo[a]) / tl), f1 = floor((hi[a] + R - m.lo[a]) / tl);
    if (!(f1 >= 0.0) || !(f0 <= (double)(m.nt[a] - 1))) return;  // also rejects NaN
    t0[a] = !(f0 > 0.0) ? 0 : (int)f0;
    t1[a] = f1 > (double)(m.nt[a] - 1) ? m.nt[a] - 1 : (int)f1;
    ntile *= (t1[a] - t0[a] + 1);
  }
  int nx = t1[0] - t0[0] + 1, ny = t1[1] - t0[1] + 1;
  for (int64_t q = lane; q < ntile; q += 64) {
    int tx = t0[0] + (int)(q % nx), ty = t0[1] + (int)((q / nx) % ny), tz = t0[2] + (int)(q / ((int64_t)nx * ny));
    double tlo[3] = {m.lo[0] + tx * tl, m.lo[1] + ty * tl, m.lo[2] + tz * tl};
    int wlo = -1, whi = -1;
    if (nb == 1) {
      if (seg_candidate(X, X, nullptr, true, true, R, tlo, tl, mrg)) wlo = whi = 0;
    } else {
      for (int i = s0; i <= s1; ++i) {
        const double *A = X + 3 * i, *B = X + 3 * (i + 1);
        const double *An = (i + 2 < nb) ? X + 3 * (i + 2) : nullptr;
        if (seg_candidate(A, B, An, i == 0, i == nseg - 1, R, tlo, tl, mrg)) {
          if (wlo < 0) wlo = i;
          whi = i;
        }
      }
    }
    if (wlo < 0) continue;
    int64_t tg = cs.tile_base + ((int64_t)tz * m.nt[1] + ty) * m.nt[0] + tx;
    if (!emit) {
      atomicAdd(&W.tile_cnt[tg], 1u);
    } else {
      uint32_t slot = W.tile_off[tg] + atomicAdd(&W.tile_fill[tg], 1u);
      if ((int64_t)slot < W.cap_emit) {
        Emit e;
        e.beam = gb;
        e.lo = wlo;
        e.hi = whi;
        e.pad = 0;
        W.emit[slot] = e;
      } else {
        set_overflow(W, 1u);
      }
    }
  }
}

void launch_chunk_tiles(const StepLaunch &L, int emit, hipStream_t st) {
  if (L.w.cap_chunk == 0) return;
  hipLaunchKernelGGL(k_chunk_tiles, dim3((unsigned)L.w.cap_chunk), dim3(64), 0, st, L, emit);
}

// ------------------------------------------------------------- tile merge --
// Per tile: sort the emissions by (beam, first segment), merge those of one
// beam into a single window, and build the screening capsule of each entry:
// the chord from the window's first to last point, inflated by the largest
// distance of a window point from it plus 3 eps_max of the window.
__global__ __launch_bounds__(64) void k_tile_merge(StepLaunch L) {
  Work W = L.w;
  __shared__ unsigned long long s_key[kMaxEmit];
  __shared__ int32_t s_hi[kMaxEmit];
  __shared__ int32_t s_cnt;
  int lane = threadIdx.x;
  int64_t nw = (int64_t)gridDim.x;
  for (int64_t tg = blockIdx.x; tg < W.n_tiles; tg += nw) {
    uint32_t off = W.tile_off[tg];
    uint32_t n = W.tile_off[tg + 1] - off;
    if (n == 0) {
      if (lane == 0) {
        W.tile_nent[tg] = 0;
        W.tile_items[tg] = 0;
      }
      continue;
    }
    int c = case_of(L.tbase, L.n_cases, tg);
    const CaseDev &cs = L.cases[c];
    const MeshDev &m = cs.m;
    int64_t tl = tg - cs.tile_base;
    if (n > (uint32_t)kMaxEmit || (int64_t)off + n > W.cap_emit) {
      if (lane == 0) {
        W.tile_nent[tg] = 0;
        W.tile_items[tg] = 0;
        set_overflow(W, n > (uint32_t)kMaxEmit ? 4u : 1u);
      }
      continue;
    }
    uint32_t np2 = 1;
    while (np2 < n) np2 <<= 1;
    for (uint32_t i = lane; i < np2; i += 64) {
      if (i < n) {
        Emit e = W.emit[off + i];
        s_key[i] = ((unsigned long long)(uint32_t)e.beam << 32) | (uint32_t)e.lo;
        s_hi[i] = e.hi;
      } else {
        s_key[i] = ~0ull;
        s_hi[i] = 0;
      }
    }
    __syncthreads();
    // bitonic sort of (key, hi) pairs in LDS
    for (uint32_t k = 2; k <= np2; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t i = lane; i < np2; i += 64) {
          uint32_t p = i ^ j;
          if (p > i) {
            bool up = (i & k) == 0;
            unsigned long long a = s_key[i], bk = s_key[p];
            if ((a > bk) == up) {
              s_key[i] = bk;
              s_key[p] = a;
              int32_t t = s_hi[i];
              s_hi[i] = s_hi[p];
              s_hi[p] = t;
            }
          }
        }
        __syncthreads();
      }
    }
    // merge windows of the same beam (lane 0; tiles hold a few dozen emissions)
    if (lane == 0) {
      int ne = 0;
      for (uint32_t i = 0; i < n; ++i) {
        uint32_t beam = (uint32_t)(s_key[i] >> 32);
        int32_t lo = (int32_t)(s_key[i] & 0xffffffffu);
        if (ne > 0 && (uint32_t)(s_key[ne - 1] >> 32) == beam) {
          if (s_hi[i] > s_hi[ne - 1]) s_hi[ne - 1] = s_hi[i];
        } else {
          s_key[ne] = ((unsigned long long)beam << 32) | (uint32_t)lo;
          s_hi[ne] = s_hi[i];
          ++ne;
        }
      }
      s_cnt = ne;
    }
    __syncthreads();
    int ne = s_cnt;
    double ox, oy, oz;
    int tx, ty, tz;
    tile_origin(m, tl, ox, oy, oz, tx, ty, tz);
    for (int e = lane; e < ne; e += 64) {
      int gb = (int)(s_key[e] >> 32);
      int i0 = (int)(s_key[e] & 0xffffffffu), i1 = s_hi[e];
      int64_t b = gb - cs.beam_base;
      int64_t k0 = cs.offsets[b];
      int nb = (int)(cs.offsets[b + 1] - k0);
      const double *X = cs.Psp + 3 * k0;
      int plast = nb >= 2 ? i1 + 1 : 0;
      const double *A = X + 3 * i0, *B = X + 3 * plast;
      double ab[3] = {B[0] - A[0], B[1] - A[1], B[2] - A[2]};
      double ll = ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2];
      double dev = 0.0, em = 0.0;
      for (int p = i0; p <= plast; ++p) {
        const double *Q = X + 3 * p;
        double q[3] = {Q[0] - A[0], Q[1] - A[1], Q[2] - A[2]};
        double t = ll > 0.0 ? (q[0] * ab[0] + q[1] * ab[1] + q[2] * ab[2]) / ll : 0.0;
        t = fmin(fmax(t, 0.0), 1.0);
        double r[3] = {q[0] - t * ab[0], q[1] - t * ab[1], q[2] - t * ab[2]};
        dev = fmax(dev, sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]));
        em = fmax(em, cs.eps[k0 + p]);
      }
      double R = (3.0 * em + dev) * (1.0 + 1e-5) + 1e-6 * (m.tile_len + 3.0 * em + dev);
      if (nb >= 2 && i1 - i0 + 1 > 0xffff) set_overflow(W, 4u);  // record field width
      Entry en;
      en.kp = (int32_t)k0;
      en.nb = nb;
      en.i0 = i0;
      en.i1 = nb >= 2 ? i1 : 0;
      en.ax = (float)(A[0] - ox);
      en.ay = (float)(A[1] - oy);
      en.az = (float)(A[2] - oz);
      en.bx = (float)(B[0] - ox);
      en.by = (float)(B[1] - oy);
      en.bz = (float)(B[2] - oz);
      float Rf = (float)R;
      en.r2 = Rf * Rf * (1.0f + 1e-5f);
      en.beam = (int32_t)b;
      W.entry[off + e] = en;
    }
    if (lane == 0) {
      if (ne > kMaxEntries) {
        set_overflow(W, 4u);
        ne = 0;
      }
      W.tile_nent[tg] = (uint32_t)ne;
      uint32_t ncell = tile_cell_start(m, tl + 1) - tile_cell_start(m, tl);
      W.tile_items[tg] = ne > 0 ? (ncell + 63u) / 64u : 0u;
    }
    __syncthreads();
  }
}

void launch_tile_merge(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_tiles == 0) return;
  int64_t g = L.w.n_tiles < 16384 ? L.w.n_tiles : 16384;
  hipLaunchKernelGGL(k_tile_merge, dim3((unsigned)g), dim3(64), 0, st, L);
}

// ------------------------------------------------------------------ items --
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
    W.item[id] = it;
  }
}

void launch_items(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_tiles == 0) return;
  hipLaunchKernelGGL(k_items, dim3((unsigned)((L.w.n_tiles + 255) / 256)), dim3(256), 0, st, L);
}

// ----------------------------------------------------------------- sample --
// c(x): nearest cell centre (ties: smaller (x, y, z), then smaller caller
// index), searched over Chebyshev shells of bins until no unvisited bin can
// hold a centre as close as the best found.  Returns the sorted index or -1
// when x is outside the domain box.
__device__ __forceinline__ bool closer_cell(const MeshDev &m, double D, uint32_t j, double bD,
                                            int64_t best) {
  if (best < 0) return true;
  if (D < bD) return true;
  if (D > bD) return false;
  double a0 = m.cx[j], b0 = m.cx[best];
  if (a0 != b0) return a0 < b0;
  double a1 = m.cy[j], b1 = m.cy[best];
  if (a1 != b1) return a1 < b1;
  double a2 = m.cz[j], b2 = m.cz[best];
  if (a2 != b2) return a2 < b2;
  return m.perm[j] < m.perm[best];
}

__device__ int64_t locate_cell(const MeshDev &m, double x, double y, double z) {
  if (!(x >= m.box[0] && x <= m.box[3] && y >= m.box[1] && y <= m.box[4] && z >= m.box[2] &&
        z <= m.box[5]))
    return -1;
  double q[3] = {x, y, z};
  int qi[3];
  for (int a = 0; a < 3; ++a) {
    double f = floor((q[a] - m.lo[a]) / m.bin);
    qi[a] = !(f > 0.0) ? 0 : (f > (double)(m.nb[a] - 1) ? m.nb[a] - 1 : (int)f);
  }
  double slack = 1e-9 * (m.bin * (double)(m.nb[0] + m.nb[1] + m.nb[2]) + fabs(m.lo[0]) +
                         fabs(m.lo[1]) + fabs(m.lo[2]));
  int64_t best = -1;
  double bD = INFINITY;
  for (int r = 0;; ++r) {
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = qi[a] - r < 0 ? 0 : qi[a] - r;
      hi[a] = qi[a] + r > m.nb[a] - 1 ? m.nb[a] - 1 : qi[a] + r;
    }
    for (int iz = lo[2]; iz <= hi[2]; ++iz)
      for (int iy = lo[1]; iy <= hi[1]; ++iy)
        for (int ix = lo[0]; ix <= hi[0]; ++ix) {
          int ch = abs(ix - qi[0]);
          ch = max(ch, abs(iy - qi[1]));
          ch = max(ch, abs(iz - qi[2]));
          if (ch != r) continue;
          uint32_t k = bin_key(m, ix, iy, iz);
          uint32_t e = m.bin_start[k + 1];
          for (uint32_t j = m.bin_start[k]; j < e; ++j) {
            double D = sqdist_exact(x, y, z, m.cx[j], m.cy[j], m.cz[j]);
            if (closer_cell(m, D, j, bD, best)) {
              best = j;
              bD = D;
            }
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
    if (best >= 0 && bound > 0.0 && bD < bound * bound) break;
  }
  return best;
}

// Eq. (16)-(18) per actuator point, in the paper's order.
__global__ void k_sample(StepLaunch L) {
#pragma clang fp contract(off)
  Work W = L.w;
  int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool act = g < W.n_points;
  bool out = false, fb = false, dg = false;
  int c = 0;
  if (act) {
    c = case_of(L.pbase, L.n_cases, g);
    const CaseDev &cs = L.cases[c];
    const MeshDev &m = cs.m;
    int64_t k = g - cs.point_base;
    int64_t b = W.pbeam[g] - cs.beam_base;
    const double *Pa = cs.P + 3 * k, *Pd = cs.Pdot + 3 * k, *et = cs.e_t + 3 * k;
    double nrm = sqrt(dot3_exact(et[0], et[1], et[2], et[0], et[1], et[2]));
    double e[3] = {et[0] / nrm, et[1] / nrm, et[2] / nrm};
    double ps[3] = {Pa[0], Pa[1], Pa[2]}, us[3] = {0.0, 0.0, 0.0};
    int64_t ca = locate_cell(m, Pa[0], Pa[1], Pa[2]), cs_ = -1;
    if (ca < 0) {
      out = true;
    } else {
      const double *Ua = cs.U + 3 * (int64_t)m.perm[ca];
      double u0[3] = {Ua[0] - Pd[0], Ua[1] - Pd[1], Ua[2] - Pd[2]};
      double ut = dot3_exact(u0[0], u0[1], u0[2], e[0], e[1], e[2]);
      double un[3] = {u0[0] - ut * e[0], u0[1] - ut * e[1], u0[2] - ut * e[2]};
      double mag = sqrt(dot3_exact(un[0], un[1], un[2], un[0], un[1], un[2]));
      double es[3];
      if (mag >= cs.tau) {
        es[0] = -un[0] / mag;
        es[1] = -un[1] / mag;
        es[2] = -un[2] / mag;
      } else {
        const double *eu = cs.e_up + 3 * b;
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
      const double *np = cs.n_p + 3 * b;
      double dn = dot3_exact(np[0], np[1], np[2], es[0], es[1], es[2]);
      double ls = cs.ls[b];
      for (int a = 0; a < 3; ++a) ps[a] = Pa[a] + ls * (es[a] - dn * np[a]);
      cs_ = locate_cell(m, ps[0], ps[1], ps[2]);
      if (cs_ < 0) {
        out = true;
      } else {
        const double *Us = cs.U + 3 * (int64_t)m.perm[cs_];
        us[0] = Us[0];
        us[1] = Us[1];
        us[2] = Us[2];
      }
    }
    double *Uout = cs.U_s ? cs.U_s + 3 * k : W.Us + 3 * g;
    Uout[0] = us[0];
    Uout[1] = us[1];
    Uout[2] = us[2];
    if (cs.U_s) {
      W.Us[3 * g] = us[0];
      W.Us[3 * g + 1] = us[1];
      W.Us[3 * g + 2] = us[2];
    }
    if (cs.P_s)
      for (int a = 0; a < 3; ++a) cs.P_s[3 * k + a] = ps[a];
    if (cs.cell_a) cs.cell_a[k] = ca < 0 ? -1 : (int64_t)m.perm[ca];
    if (cs.cell_s) cs.cell_s[k] = cs_ < 0 ? -1 : (int64_t)m.perm[cs_];
    W.pflags[g] = (out ? 1 : 0) | (fb ? 2 : 0) | (dg ? 4 : 0);
  }
  // counters (one atomic per wave and case; a wave may straddle two cases)
  int c0 = __shfl(c, 0, 64);
  bool same = __all(!act || c == c0);
  if (same) {
    long long *cnt = W.cnt + 8 * c0;
    wave_count_add(cnt + 0, act && out);
    wave_count_add(cnt + 1, act && fb);
    wave_count_add(cnt + 2, act && dg);
  } else if (act) {
    long long *cnt = W.cnt + 8 * c;
    if (out) atomicAdd((unsigned long long *)(cnt + 0), 1ull);
    if (fb) atomicAdd((unsigned long long *)(cnt + 1), 1ull);
    if (dg) atomicAdd((unsigned long long *)(cnt + 2), 1ull);
  }
}

void launch_sample(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_points == 0) return;
  hipLaunchKernelGGL(k_sample, dim3((unsigned)((L.w.n_points + 63) / 64)), dim3(64), 0, st, L);
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
// (up to 64 cells of one tile):
//   1. screen every (cell, entry) combination against the entry's capsule and
//      list the candidate pairs in (cell, entry) order;
//   2. for each candidate pair (64 at a time, full lanes) find the closest
//      segment of the entry's window exactly in FP64, apply the inclusive 3 eps
//      cutoff and compute the weights a0, a1;
//   3. add a V into per-node fixed-point accumulators (LDS integer atomics,
//      then one global integer atomic per touched node);
//   4. store the surviving pairs as 32-bit records (cell, entry, segment) for
//      the spread pass.
constexpr int kMaskWords = kMaxEntries / 32;

struct WaveScratch {
  double cx[64], cy[64], cz[64], v[64];
  float lx[64], ly[64], lz[64];
  uint32_t mask[64 * kMaskWords];
  uint32_t off[65];
  uint32_t slot0[kMaxEntries + 1];
  long long acc_hi[kNodeSlots];
  unsigned long long acc_lo[kNodeSlots];
  uint32_t item;
};

__device__ __forceinline__ float seg_dist2_f32(float px, float py, float pz, float ax, float ay,
                                               float az, float bx, float by, float bz) {
  float ex = bx - ax, ey = by - ay, ez = bz - az;
  float qx = px - ax, qy = py - ay, qz = pz - az;
  float ee = ex * ex + ey * ey + ez * ez;
  float t = qx * ex + qy * ey + qz * ez;
  float u = ee > 0.0f ? fminf(fmaxf(t / ee, 0.0f), 1.0f) : 0.0f;
  float rx = qx - u * ex, ry = qy - u * ey, rz = qz - u * ez;
  return rx * rx + ry * ry + rz * rz;
}

// closest segment of the entry's window to C (FP64, lowest index on ties)
__device__ __forceinline__ void window_argmin(const double *X, const Entry &en, double cx, double cy,
                                              double cz, int &bi, double &bs, double &br2) {
  if (en.nb == 1) {
    bi = 0;
    bs = 0.0;
    br2 = sqdist_exact(cx, cy, cz, X[0], X[1], X[2]);
    return;
  }
  br2 = INFINITY;
  bi = en.i0;
  bs = 0.0;
  double ax = X[3 * en.i0], ay = X[3 * en.i0 + 1], az = X[3 * en.i0 + 2];
  for (int i = en.i0; i <= en.i1; ++i) {
    double bx = X[3 * i + 3], by = X[3 * i + 4], bz = X[3 * i + 5];
    double s, r2;
    seg_foot(cx, cy, cz, ax, ay, az, bx, by, bz, s, r2);
    if (r2 < br2) {
      br2 = r2;
      bi = i;
      bs = s;
    }
    ax = bx;
    ay = by;
    az = bz;
  }
}

__device__ __forceinline__ void acc_add(WaveScratch &sh, bool lds, Work &W, uint32_t slot,
                                        int64_t node, double v) {
  long long h;
  unsigned long long l;
  fx_encode(v, W.wexp[node], h, l);
  if (lds) {
    atomicAdd((unsigned long long *)&sh.acc_hi[slot], (unsigned long long)h);
    atomicAdd(&sh.acc_lo[slot], l);
  } else {
    atomicAdd((unsigned long long *)&W.w_hi[node], (unsigned long long)h);
    atomicAdd(&W.w_lo[node], l);
  }
}

__global__ __launch_bounds__(64) void k_weights(StepLaunch L) {
  Work W = L.w;
  __shared__ WaveScratch sh;
  const int lane = threadIdx.x;
  const uint32_t n_items = W.tile_itoff[W.n_tiles];
  for (;;) {
    if (lane == 0) sh.item = atomicAdd(&W.counters[0], 1u);
    __syncthreads();
    const uint32_t item = sh.item;
    __syncthreads();
    if (item >= n_items || (int64_t)item >= W.cap_item) break;
    const Item it = W.item[item];
    const CaseDev &cs = L.cases[it.cs];
    const MeshDev &m = cs.m;
    const int64_t tl = it.tile - cs.tile_base;
    double ox, oy, oz;
    int tx, ty, tz;
    tile_origin(m, tl, ox, oy, oz, tx, ty, tz);
    const int c = it.c0 + lane;
    const bool valid = c < it.c1;
    double cx = 0, cy = 0, cz = 0, v = 0;
    float lx = 3e30f, ly = 3e30f, lz = 3e30f;
    if (valid) {
      cx = m.cx[c];
      cy = m.cy[c];
      cz = m.cz[c];
      v = m.vs[c];
      lx = (float)(cx - ox);
      ly = (float)(cy - oy);
      lz = (float)(cz - oz);
    }
    sh.cx[lane] = cx;
    sh.cy[lane] = cy;
    sh.cz[lane] = cz;
    sh.v[lane] = v;
    const uint32_t ent0 = W.tile_off[it.tile];
    const int ne = (int)W.tile_nent[it.tile];
    const Entry *E = W.entry + ent0;
    const double *X = cs.Psp;
    // node-slot bases per entry
    uint32_t carry = 0;
    for (int e0 = 0; e0 < ne; e0 += 64) {
      int e = e0 + lane;
      uint32_t ns = 0;
      if (e < ne) {
        Entry en = E[e];
        ns = en.nb == 1 ? 1u : (uint32_t)(en.i1 - en.i0 + 2);
      }
      uint32_t tot;
      uint32_t ex = wave_excl_scan_u32(ns, tot);
      if (e < ne) sh.slot0[e] = carry + ex;
      carry += tot;
    }
    if (lane == 0) sh.slot0[ne] = carry;
    const uint32_t nslot = carry;
    const bool lds = nslot <= (uint32_t)kNodeSlots;
    if (lds)
      for (uint32_t s = lane; s < nslot; s += 64) {
        sh.acc_hi[s] = 0;
        sh.acc_lo[s] = 0;
      }
    // 1. screening
    uint32_t word = 0, cnt = 0;
    for (int e = 0; e < ne; ++e) {
      const Entry en = E[e];
      float d2 = seg_dist2_f32(lx, ly, lz, en.ax, en.ay, en.az, en.bx, en.by, en.bz);
      if (valid && d2 <= en.r2) word |= 1u << (e & 31);
      if ((e & 31) == 31 || e == ne - 1) {
        sh.mask[lane * kMaskWords + (e >> 5)] = word;
        cnt += __popc(word);
        word = 0;
      }
    }
    uint32_t total;
    uint32_t myoff = wave_excl_scan_u32(cnt, total);
    sh.off[lane] = myoff;
    if (lane == 63) sh.off[64] = myoff + cnt;
    __syncthreads();
    // record space for up to `total` pairs
    uint32_t rbase = 0;
    if (lane == 0) rbase = atomicAdd(&W.counters[2], total);
    rbase = __shfl(rbase, 0, 64);
    const bool rec_ok = (int64_t)rbase + total <= W.cap_rec;
    if (!rec_ok && lane == 0) set_overflow(W, 2u);
    uint32_t nreal = 0;
    const int nwords = (ne + 31) >> 5;
    // 2.-4. candidate pairs, 64 per round
    for (uint32_t p0 = 0; p0 < total; p0 += 64) {
      const uint32_t p = p0 + lane;
      const bool act = p < total;
      bool in = false;
      int L_ = 0, e = 0, bi = 0;
      if (act) {
        int lo = 0, hi = 63;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (sh.off[mid] <= p) lo = mid;
          else hi = mid - 1;
        }
        L_ = lo;
        uint32_t r = p - sh.off[L_];
        for (int wd = 0; wd < nwords; ++wd) {
          uint32_t mw = sh.mask[L_ * kMaskWords + wd];
          uint32_t pc = __popc(mw);
          if (r < pc) {
            for (uint32_t q = 0; q < r; ++q) mw &= mw - 1u;
            e = wd * 32 + __ffs(mw) - 1;
            break;
          }
          r -= pc;
        }
        const Entry en = E[e];
        const double *Xb = X + 3 * (int64_t)en.kp;
        const double pcx = sh.cx[L_], pcy = sh.cy[L_], pcz = sh.cz[L_];
        double bs, br2;
        window_argmin(Xb, en, pcx, pcy, pcz, bi, bs, br2);
        const double *epsb = cs.eps + en.kp;
        double ej = en.nb == 1 ? epsb[0] : eps_at(bs, epsb[bi], epsb[bi + 1]);
        in = inside_cutoff(br2, ej);
        if (in) {
          double a0, a1;
          pair_weights(cs.prec, bs, br2, ej, a0, a1);
          const double vv = sh.v[L_];
          const int64_t node = cs.point_base + en.kp + bi;
          const uint32_t slot = sh.slot0[e] + (uint32_t)(en.nb == 1 ? 0 : bi - en.i0);
          acc_add(sh, lds, W, slot, node, a0 * vv);
          if (en.nb > 1) acc_add(sh, lds, W, slot + 1, node + 1, a1 * vv);
        }
      }
      const uint64_t bal = ballot64(act && in);
      if (act && in && rec_ok) {
        uint32_t rank = lanemask_lt_popc(bal);
        const Entry en = E[e];
        uint32_t seg = (uint32_t)(en.nb == 1 ? 0 : bi - en.i0);
        W.rec[rbase + nreal + rank] = ((uint32_t)L_ << 26) | ((uint32_t)e << 16) | seg;
      }
      nreal += (uint32_t)__popcll(bal);
    }
    __syncthreads();
    // flush node accumulators
    if (lds) {
      for (uint32_t s = lane; s < nslot; s += 64) {
        long long h = sh.acc_hi[s];
        unsigned long long l = sh.acc_lo[s];
        if (h == 0 && l == 0) continue;
        int lo = 0, hi = ne - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (sh.slot0[mid] <= s) lo = mid;
          else hi = mid - 1;
        }
        const Entry en = E[lo];
        int64_t node = cs.point_base + en.kp + (en.nb == 1 ? 0 : en.i0) + (s - sh.slot0[lo]);
        h += (long long)(l >> kLoBits);
        l &= (1ull << kLoBits) - 1ull;
        atomicAdd((unsigned long long *)&W.w_hi[node], (unsigned long long)h);
        atomicAdd(&W.w_lo[node], l);
      }
    }
    if (lane == 0) {
      W.rec_base[item] = rbase;
      W.rec_cnt[item] = rec_ok ? nreal : 0u;
      atomicAdd((unsigned long long *)(W.cnt + 8 * it.cs + 5), (unsigned long long)nreal);
    }
    __syncthreads();
  }
}

void launch_weights(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_weights, dim3(L.grid_persistent), dim3(64), 0, st, L);
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
  if (__all(!act || c == c0)) wave_count_add(W.cnt + 8 * c0 + 3, act && zero);
  else if (act && zero) atomicAdd((unsigned long long *)(W.cnt + 8 * c + 3), 1ull);
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

// per case: F_beam, sum |f L| and the fixed-point exponent of the fluid-side sum
__global__ void k_finalize_beam(StepLaunch L) {
  Work W = L.w;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L.n_cases) return;
  double r[4] = {0, 0, 0, 0};
  for (int pb = 0; pb < W.n_pblocks; ++pb)
    if (W.pblock_case[pb] == c)
      for (int q = 0; q < 4; ++q) r[q] += W.beam_part[4 * pb + q];
  double *d = W.diag_out + 16 * c;
  d[0] = r[0];
  d[1] = r[1];
  d[2] = r[2];
  d[3] = r[3];
  W.F_exp[c] = r[3] > 0.0 ? ilogb(r[3]) + 2 : 0;
}

void launch_beam_sums(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_pblocks > 0)
    hipLaunchKernelGGL(k_beam_sums, dim3(L.w.n_pblocks), dim3(kSumBlock), 0, st, L);
  hipLaunchKernelGGL(k_finalize_beam, dim3((L.n_cases + 63) / 64), dim3(64), 0, st, L);
}

// ----------------------------------------------------------------- spread --
// Eq. (23): S_j = -sum over the cell's pairs (beam order) of
// a0 f_hat_i + a1 f_hat_i+1, with a0, a1 recomputed bit-identically from the
// stored pair records.  Each cell is summed by one lane in record order, so
// the source needs no atomics; every cell of an active tile is written.
struct SpreadScratch {
  double cx[64], cy[64], cz[64];
  double cc[3][64];
  uint32_t cnt[64];
  uint32_t off[65];
  uint32_t item;
};

__global__ __launch_bounds__(64) void k_spread(StepLaunch L) {
  Work W = L.w;
  __shared__ SpreadScratch sh;
  const int lane = threadIdx.x;
  const uint32_t n_items = W.tile_itoff[W.n_tiles];
  for (;;) {
    if (lane == 0) sh.item = atomicAdd(&W.counters[1], 1u);
    __syncthreads();
    const uint32_t item = sh.item;
    __syncthreads();
    if (item >= n_items || (int64_t)item >= W.cap_item) break;
    const Item it = W.item[item];
    const CaseDev &cs = L.cases[it.cs];
    const MeshDev &m = cs.m;
    const int c = it.c0 + lane;
    const bool valid = c < it.c1;
    double v = 0.0;
    if (valid) {
      sh.cx[lane] = m.cx[c];
      sh.cy[lane] = m.cy[c];
      sh.cz[lane] = m.cz[c];
      v = m.vs[c];
    }
    sh.cnt[lane] = 0;
    __syncthreads();
    const uint32_t rb = W.rec_base[item], rn = W.rec_cnt[item];
    const uint32_t ent0 = W.tile_off[it.tile];
    const Entry *E = W.entry + ent0;
    for (uint32_t j = lane; j < rn; j += 64) atomicAdd(&sh.cnt[W.rec[rb + j] >> 26], 1u);
    __syncthreads();
    uint32_t tot;
    uint32_t myoff = wave_excl_scan_u32(sh.cnt[lane], tot);
    sh.off[lane] = myoff;
    if (lane == 63) sh.off[64] = tot;
    __syncthreads();
    double S0 = 0.0, S1 = 0.0, S2 = 0.0;
    for (uint32_t p0 = 0; p0 < rn; p0 += 64) {
      const uint32_t p = p0 + lane;
      if (p < rn) {
        const uint32_t r = W.rec[rb + p];
        const int L_ = (int)(r >> 26), e = (int)((r >> 16) & 1023u), seg = (int)(r & 0xffffu);
        const Entry en = E[e];
        const double *Xb = cs.Psp + 3 * (int64_t)en.kp;
        const double *epsb = cs.eps + en.kp;
        const double pcx = sh.cx[L_], pcy = sh.cy[L_], pcz = sh.cz[L_];
        double s, r2, ej;
        int i;
        if (en.nb == 1) {
          i = 0;
          s = 0.0;
          r2 = sqdist_exact(pcx, pcy, pcz, Xb[0], Xb[1], Xb[2]);
          ej = epsb[0];
        } else {
          i = en.i0 + seg;
          seg_foot(pcx, pcy, pcz, Xb[3 * i], Xb[3 * i + 1], Xb[3 * i + 2], Xb[3 * i + 3],
                   Xb[3 * i + 4], Xb[3 * i + 5], s, r2);
          ej = eps_at(s, epsb[i], epsb[i + 1]);
        }
        double a0, a1;
        pair_weights(cs.prec, s, r2, ej, a0, a1);
        const double *fh = W.fhat + 3 * (cs.point_base + en.kp + i);
        double q0 = a0 * fh[0], q1 = a0 * fh[1], q2 = a0 * fh[2];
        if (en.nb > 1) {
          q0 += a1 * fh[3];
          q1 += a1 * fh[4];
          q2 += a1 * fh[5];
        }
        sh.cc[0][lane] = -q0;
        sh.cc[1][lane] = -q1;
        sh.cc[2][lane] = -q2;
      }
      __syncthreads();
      const uint32_t lo = sh.off[lane] > p0 ? sh.off[lane] : p0;
      const uint32_t hi = sh.off[lane + 1] < p0 + 64 ? sh.off[lane + 1] : p0 + 64;
      for (uint32_t j = lo; j < hi; ++j) {
        S0 += sh.cc[0][j - p0];
        S1 += sh.cc[1][j - p0];
        S2 += sh.cc[2][j - p0];
      }
      __syncthreads();
    }
    if (valid && cs.write_S) {
      double *S = cs.S + 3 * (int64_t)m.perm[c];
      S[0] = S0;
      S[1] = S1;
      S[2] = S2;
    }
    wave_count_add(W.cnt + 8 * it.cs + 4, valid && sh.cnt[lane] > 0);
    // force on the fluid: deterministic wave sum, then exact accumulation
    double fx = wave_sum_f64(S0 * v), fy = wave_sum_f64(S1 * v), fz = wave_sum_f64(S2 * v);
    if (lane < 3) {
      double val = lane == 0 ? fx : (lane == 1 ? fy : fz);
      if (val != 0.0) {
        long long h;
        unsigned long long l;
        fx_encode(val, W.F_exp[it.cs], h, l);
        atomicAdd((unsigned long long *)&W.F_hi[3 * it.cs + lane], (unsigned long long)h);
        atomicAdd(&W.F_lo[3 * it.cs + lane], l);
      }
    }
    __syncthreads();
  }
}

void launch_spread(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_spread, dim3(L.grid_persistent), dim3(64), 0, st, L);
}

// ------------------------------------------------------------- zero dirty --
// Cells of tiles written at the previous step but not now return to zero;
// the tile activity becomes the new previous state.
__global__ void k_zero_dirty(StepLaunch L) {
  Work W = L.w;
  int64_t tg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tg >= W.n_tiles) return;
  int c = case_of(L.tbase, L.n_cases, tg);
  const CaseDev &cs = L.cases[c];
  if (!cs.write_S || !cs.tile_prev) return;
  int64_t tl = tg - cs.tile_base;
  uint8_t now = W.tile_nent[tg] > 0 ? 1 : 0;
  if (cs.tile_prev[tl] && !now) {
    uint32_t c0 = tile_cell_start(cs.m, tl), c1 = tile_cell_start(cs.m, tl + 1);
    for (uint32_t j = c0; j < c1; ++j) {
      double *S = cs.S + 3 * (int64_t)cs.m.perm[j];
      S[0] = 0.0;
      S[1] = 0.0;
      S[2] = 0.0;
    }
  }
  cs.tile_prev[tl] = now;
}

void launch_zero_dirty(const StepLaunch &L, hipStream_t st) {
  if (L.w.n_tiles == 0) return;
  hipLaunchKernelGGL(k_zero_dirty, dim3((unsigned)((L.w.n_tiles + 255) / 256)), dim3(256), 0, st, L);
}

// --------------------------------------------------------------- finalize --
__global__ void k_finalize(StepLaunch L) {
  Work W = L.w;
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= L.n_cases) return;
  double *d = W.diag_out + 16 * c;
  int E = W.F_exp[c];
  double F[3];
  for (int a = 0; a < 3; ++a) F[a] = fx_decode(W.F_hi[3 * c + a], W.F_lo[3 * c + a], E);
  d[4] = F[0];
  d[5] = F[1];
  d[6] = F[2];
  double r0 = F[0] + d[0], r1 = F[1] + d[1], r2 = F[2] + d[2];
  d[7] = d[3] > 0.0 ? sqrt(r0 * r0 + r1 * r1 + r2 * r2) / d[3] : 0.0;
  d[8] = (double)W.counters[3];
}

void launch_finalize(const StepLaunch &L, hipStream_t st) {
  hipLaunchKernelGGL(k_finalize, dim3((L.n_cases + 63) / 64), dim3(64), 0, st, L);
}

}  // namespace alp
