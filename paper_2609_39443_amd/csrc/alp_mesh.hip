// alp_mesh.hip -- scans, fills and the once-per-mesh binning of cell centres
// (the static search structure the paper builds once at the start of a run,
// Sec. 3.2.5): a uniform spatial hash whose bins are numbered tile-major, a
// counting sort of the cells by bin (the histogram's exclusive scan is the
// bin CSR), a per-bin sort by caller index for a deterministic layout, and
// bin-sorted FP64 copies of the centres and volumes.
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

__global__ void k_bin_scatter(const uint32_t *key, int64_t n, const uint32_t *start, uint32_t *fill,
                              uint32_t *sorted) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t k = key[i];
  uint32_t pos = start[k] + atomicAdd(&fill[k], 1u);
  sorted[pos] = (uint32_t)i;
}

void launch_bin_scatter(const uint32_t *key, int64_t n, const uint32_t *start, uint32_t *fill,
                        uint32_t *sorted, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_scatter, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, key, n,
                     start, fill, sorted);
}

// insertion sort of each bin's cells by caller index (bins hold a handful of
// cells; the order only fixes a deterministic layout)
__global__ void k_bin_sort(const uint32_t *start, int64_t n_bins, uint32_t *sorted) {
  int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= n_bins) return;
  uint32_t s0 = start[b], s1 = start[b + 1];
  for (uint32_t i = s0 + 1; i < s1; ++i) {
    uint32_t v = sorted[i];
    uint32_t j = i;
    while (j > s0 && sorted[j - 1] > v) {
      sorted[j] = sorted[j - 1];
      --j;
    }
    sorted[j] = v;
  }
}

void launch_bin_sort(const uint32_t *start, int64_t n_bins, uint32_t *sorted, hipStream_t st) {
  hipLaunchKernelGGL(k_bin_sort, dim3((unsigned)((n_bins + 255) / 256)), dim3(256), 0, st, start,
                     n_bins, sorted);
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
