// alp_mesh.hip -- scans, fills and the once-per-mesh binning of cell centres
// (the static search structure the paper builds once at the start of a run,
// Sec. 3.2.5): a uniform spatial hash whose bins are numbered tile-major, the
// bin CSR from the exclusive scan of the bin histogram, an LDS radix sort of
// the cell ids by bin key (stable, so a bin's cells stay in caller order),
// and bin-sorted FP64 copies of the centres and volumes.
#include "alp_internal.h"

namespace alp {

// ------------------------------------------------------------------ scan --
// Exclusive scan of n uint32 values: out[i] = sum_{j<i} in[j], out[n] = total.
// Three passes (block totals, scan of totals, block scan + offset); integer
// arithmetic, so the result is independent of scheduling.
constexpr int kScanBlock = 256;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanBlock * kScanPer;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    uint32_t t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// block-wide exclusive scan of one value per thread (blockDim = kScanBlock)
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *total) {
  __shared__ uint32_t s_w[kScanBlock / 64];
  int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) s_w[wid] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int i = 0; i < kScanBlock / 64; ++i) {
    if (i < wid) off += s_w[i];
    tot += s_w[i];
  }
  __syncthreads();
  if (total) *total = tot;
  return off + inc - v;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_totals(const uint32_t *in, int64_t n,
                                                            uint32_t *tot) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  uint32_t s = 0;
  for (int k = 0; k < kScanPer; ++k)
    if (base + k < n) s += in[base + k];
  uint32_t t;
  block_excl_scan(s, &t);
  if (threadIdx.x == 0) tot[blockIdx.x] = t;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_tops(uint32_t *tot, int64_t nblk) {
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblk; b0 += kScanBlock) {
    int64_t i = b0 + threadIdx.x;
    uint32_t v = i < nblk ? tot[i] : 0u, t;
    uint32_t ex = block_excl_scan(v, &t);
    if (i < nblk) tot[i] = carry + ex;
    carry += t;
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[nblk] = carry;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const uint32_t *in, uint32_t *out,
                                                           int64_t n, const uint32_t *tot,
                                                           int64_t nblk) {
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer], s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t ex = block_excl_scan(s, nullptr) + tot[blockIdx.x];
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = tot[nblk];
}

// Second pass for up to kScanDirect blocks: each block adds the totals of
// the blocks before it itself, so the scan of the totals needs no launch of
// its own.
constexpr int64_t kScanDirect = 1024;

__global__ __launch_bounds__(kScanBlock) void k_scan_final_direct(const uint32_t *in, uint32_t *out, int64_t n,
                                                                  const uint32_t *tot, int64_t nblk) {
  uint32_t before = 0, all = 0;
  for (int64_t b = threadIdx.x; b < nblk; b += kScanBlock) {
    const uint32_t t = tot[b];
    all += t;
    if (b < (int64_t)blockIdx.x) before += t;
  }
  // block sums of `before` and `all` (integer, so the order does not matter)
  uint32_t sb, sa;
  block_excl_scan(before, &sb);
  block_excl_scan(all, &sa);
  int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer], s = 0;
  for (int k = 0; k < kScanPer; ++k) {
    v[k] = (base + k < n) ? in[base + k] : 0u;
    s += v[k];
  }
  uint32_t ex = block_excl_scan(s, nullptr) + sb;
  for (int k = 0; k < kScanPer; ++k) {
    if (base + k < n) out[base + k] = ex;
    ex += v[k];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sa;
}

int64_t scan_tmp_words(int64_t n) { return (n + kScanTile - 1) / kScanTile + 2; }

void launch_scan_u32(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *tmp, hipStream_t st) {
  int64_t nblk = (n + kScanTile - 1) / kScanTile;
  if (nblk == 0) nblk = 1;
  hipLaunchKernelGGL(k_scan_totals, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, in, n, tmp);
  if (nblk <= kScanDirect) {
    hipLaunchKernelGGL(k_scan_final_direct, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, in, out, n, tmp, nblk);
    return;
  }
  hipLaunchKernelGGL(k_scan_tops, dim3(1), dim3(kScanBlock), 0, st, tmp, nblk);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)nblk), dim3(kScanBlock), 0, st, in, out, n, tmp,
                     nblk);
}

// ----------------------------------------------------------------- fills --
template <typename T>
__global__ void k_fill(T *p, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (; i < n; i += stride) p[i] = v;
}
template <typename T>
static void fill(T *p, T v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill<T>, dim3((unsigned)blocks), dim3(256), 0, st, p, v, n);
}
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st) { fill(p, v, n, st); }
void launch_fill_u8(uint8_t *p, uint8_t v, int64_t n, hipStream_t st) { fill(p, v, n, st); }
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t st) { fill(p, v, n, st); }
void launch_fill_i64(long long *p, long long v, int64_t n, hipStream_t st) { fill(p, v, n, st); }

// ---------------------------------------------------------------- bounds --
// per block: min xyz, max xyz, max V (7 doubles); the host reduces the blocks
constexpr int kBoundsBlock = 256;
int mesh_bounds_blocks(int64_t n) {
  int64_t b = (n + kBoundsBlock * 16 - 1) / (kBoundsBlock * 16);
  return (int)(b < 1 ? 1 : (b > 4096 ? 4096 : b));
}

__global__ __launch_bounds__(kBoundsBlock) void k_mesh_bounds(const double *C, const double *V,
                                                              int64_t n, double *part) {
  __shared__ double s[7][kBoundsBlock];
  double r[7] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY, 0.0};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    for (int a = 0; a < 3; ++a) {
      double x = C[3 * i + a];
      r[a] = fmin(r[a], x);
      r[3 + a] = fmax(r[3 + a], x);
    }
    r[6] = fmax(r[6], V[i]);
  }
  for (int k = 0; k < 7; ++k) s[k][threadIdx.x] = r[k];
  __syncthreads();
  for (int w = kBoundsBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 7; ++k) {
        double a = s[k][threadIdx.x], b = s[k][threadIdx.x + w];
        s[k][threadIdx.x] = (k < 3) ? fmin(a, b) : fmax(a, b);
      }
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 7; ++k) part[7 * blockIdx.x + k] = s[k][0];
}

void launch_mesh_bounds(const double *C, const double *V, int64_t n, double *part, int nblk,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_mesh_bounds, dim3(nblk), dim3(kBoundsBlock), 0, st, C, V, n, part);
}

// ------------------------------------------------------------ bin + sort --
__device__ __forceinline__ int bin_axis(double x, double lo, double bin, int nb) {
  double f = floor((x - lo) / bin);
  return !(f > 0.0) ? 0 : (f > (double)(nb - 1) ? nb - 1 : (int)f);  // NaN -> 0
}

__global__ void k_bin_keys(MeshDev m, const double *C, int64_t n, uint32_t *key, uint32_t *count) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int ix = bin_axis(C[3 * i + 0], m.lo[0], m.bin, m.nb[0]);
  int iy = bin_axis(C[3 * i + 1], m.lo[1], m.bin, m.nb[1]);
  int iz = bin_axis(C[3 * i + 2], m.lo[2], m.bin, m.nb[2]);
  uint32_t k = bin_key(m, ix, iy, iz);
  key[i] = k;
  atomicAdd(&count[k], 1u);
}

void launch_bin_keys(const MeshDev &m, const double *C, int64_t n, uint32_t *key, uint32_t *count,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_bin_keys, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, m, C, n, key,
                     count);
}

// LSD radix sort of the cell ids by bin key, eight bits a pass.  The ids
// start in caller order and every pass is stable, so the cells of a bin end
// in caller order: the layout depends only on the centres and their
// numbering, not on scheduling.  A pass: per-tile digit counts in LDS,
// one exclusive scan of the counts laid out digit-major (which gives every
// (digit, tile) its first output place), then a scatter in which each tile
// ranks its keys in LDS, 256 at a time, and writes them in order.
constexpr int kRadixBits = 8;
constexpr int kRadixDigits = 1 << kRadixBits;
constexpr int kRadixBlock = 256;  // one thread per digit in the LDS tables
constexpr int kRadixPer = 16;     // keys per thread and tile
constexpr int kRadixTile = kRadixBlock * kRadixPer;
static_assert(kRadixBlock == kRadixDigits, "one thread per digit");

int64_t radix_tiles(int64_t n) { return n > 0 ? (n + kRadixTile - 1) / kRadixTile : 1; }
int radix_passes(int64_t n_bins) {
  int bits = 0;
  while (bits < 32 && ((uint64_t)(n_bins - 1) >> bits) != 0u) ++bits;
  return (bits + kRadixBits - 1) / kRadixBits;
}

__global__ __launch_bounds__(kRadixBlock) void k_radix_count(const uint32_t *key, int64_t n, int shift,
                                                             uint32_t *cnt, int64_t n_tiles) {
  __shared__ uint32_t h[kRadixDigits];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  for (int r = 0; r < kRadixPer; ++r) {
    const int64_t i = base + (int64_t)r * kRadixBlock + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & (kRadixDigits - 1)], 1u);
  }
  __syncthreads();
  cnt[(int64_t)threadIdx.x * n_tiles + blockIdx.x] = h[threadIdx.x];
}

// vin == nullptr: the ids are the input positions (the first pass)
__global__ __launch_bounds__(kRadixBlock) void k_radix_scatter(const uint32_t *kin, const uint32_t *vin,
                                                               uint32_t *kout, uint32_t *vout, int64_t n,
                                                               int shift, const uint32_t *off,
                                                               int64_t n_tiles) {
  __shared__ uint32_t run[kRadixDigits];                     // next place of each digit
  __shared__ uint32_t wc[kRadixBlock / 64][kRadixDigits];    // this round's count per wave and digit
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  run[t] = off[(int64_t)t * n_tiles + blockIdx.x];
  for (int w = 0; w < kRadixBlock / 64; ++w) wc[w][t] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kRadixTile;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int r = 0; r < kRadixPer; ++r) {
    const int64_t i = base + (int64_t)r * kRadixBlock + t;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u;
    const uint32_t v = valid ? (vin ? vin[i] : (uint32_t)i) : 0u;
    const uint32_t d = (k >> shift) & (kRadixDigits - 1);
    // lanes of this wave holding the same digit: one ballot per digit bit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & below);
    if (valid && rank == 0u) wc[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wc[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t add = 0u;
    for (int w = 0; w < kRadixBlock / 64; ++w) {
      add += wc[w][t];
      wc[w][t] = 0u;
    }
    run[t] += add;
    __syncthreads();
  }
}

__global__ void k_iota(uint32_t *p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = (uint32_t)i;
}

int64_t radix_scratch_words(int64_t n) { return (int64_t)kRadixDigits * radix_tiles(n) + 1; }

// Sorts the ids 0 .. n-1 by key (stable) into perm; ksorted receives the
// sorted keys.  k2, v2: n words each; cnt: radix_scratch_words(n) words; tmp:
// scan_tmp_words(radix_scratch_words(n)) words.  key is left unchanged.
void launch_radix_sort(const uint32_t *key, int64_t n, int64_t n_bins, uint32_t *perm, uint32_t *ksorted,
                       uint32_t *k2, uint32_t *v2, uint32_t *cnt, uint32_t *tmp, hipStream_t st) {
  if (n <= 0) return;
  const int passes = radix_passes(n_bins);
  if (passes == 0) {
    // one bin: every key is 0 and the order is the caller's
    hipLaunchKernelGGL(k_iota, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, perm, n);
    launch_fill_u32(ksorted, 0u, n, st);
    return;
  }
  const int64_t nt = radix_tiles(n);
  const uint32_t *kin = key, *vin = nullptr;
  for (int p = 0; p < passes; ++p) {
    // the last pass writes perm and ksorted
    const bool to_out = ((passes - 1 - p) & 1) == 0;
    uint32_t *kout = to_out ? ksorted : k2, *vout = to_out ? perm : v2;
    const int shift = p * kRadixBits;
    hipLaunchKernelGGL(k_radix_count, dim3((unsigned)nt), dim3(kRadixBlock), 0, st, kin, n, shift, cnt, nt);
    launch_scan_u32(cnt, cnt, (int64_t)kRadixDigits * nt, tmp, st);
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nt), dim3(kRadixBlock), 0, st, kin, vin, kout, vout, n,
                       shift, cnt, nt);
    kin = kout;
    vin = vout;
  }
}

// The binned layout checked against its definition: every sorted cell lies
// in its own bin's range, carries its own key, and follows the one before it
// in (key, caller index) order.  Any violation sets *bad.
__global__ void k_bin_check(const uint32_t *key, const uint32_t *ksorted, const uint32_t *perm,
                            const uint32_t *start, int64_t n, uint32_t *bad) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t k = ksorted[p], c = perm[p];
  bool ok = c < (uint64_t)n && key[c] == k && start[k] <= (uint64_t)p && (uint64_t)p < start[k + 1];
  if (p > 0) {
    const uint32_t kp = ksorted[p - 1];
    ok = ok && (kp < k || (kp == k && perm[p - 1] < c));
  }
  if (!ok) atomicOr(bad, 1u);
}

void launch_bin_check(const uint32_t *key, const uint32_t *ksorted, const uint32_t *perm, const uint32_t *start,
                      int64_t n, uint32_t *bad, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(k_bin_check, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, ksorted, perm,
                     start, n, bad);
}

__global__ void k_bin_reorder(const double *C, const double *V, const uint32_t *sorted, int64_t n,
                              double *cxyz, double *cx, double *cy, double *cz, double *vs) {
  int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  uint32_t c = sorted[p];
  const double x = C[3 * (int64_t)c + 0], y = C[3 * (int64_t)c + 1], z = C[3 * (int64_t)c + 2];
  cx[p] = x;
  cy[p] = y;
  cz[p] = z;
  *(double4 *)(cxyz + 4 * p) = make_double4(x, y, z, (double)c);
  vs[p] = V[c];
}

void launch_bin_reorder(const double *C, const double *V, const uint32_t *sorted, int64_t n, double *cxyz,
                        double *cx, double *cy, double *cz, double *vs, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_reorder, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, C, V,
                     sorted, n, cxyz, cx, cy, cz, vs);
}

}  // namespace alp
