// alp_api.hip -- host side of libalp: contexts, mesh binning, argument
// validation, workspace sizing, the launch sequence of a coupling step,
// hipGraph capture and replay, and diagnostics read-back.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <chrono>
#include <mutex>
#include <vector>

#include "alp_internal.h"
#include "alp_reccursor.h"

using namespace alp;

struct alp_mesh {
  int device = 0;
  MeshDev d{};
  uint32_t *bin_start = nullptr;
  double *cx = nullptr, *cy = nullptr, *cz = nullptr, *vs = nullptr, *cxyz = nullptr;
  uint32_t *perm = nullptr;
  uint8_t *tile_prev = nullptr;
  const double *last_S = nullptr;  // output array the band state refers to
};

struct alp_context {
  int device = 0;
  hipStream_t user = nullptr;
  hipStream_t st = nullptr;
  hipStream_t st2 = nullptr;  // second stream: sampling and drag run beside the projection
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_fork = nullptr, ev_join = nullptr, ev_items = nullptr;
  std::string err;
  int n_cu = 256;
  int spread_per_cu = 8;  // resident spread blocks per CU
  // workspace
  Work w{};
  std::vector<void *> wallocs;
  int64_t have_points = -1, have_beams = -1, have_tiles = -1, have_cases = -1, have_pblocks = -1;
  int64_t have_emit = -1, have_item = -1, have_rec = -1, have_chunk = -1;
  uint32_t *scan_tmp = nullptr;
  int64_t have_scan = -1;
  // case tables
  CaseDev *d_cases = nullptr;
  int64_t *d_bases = nullptr;  // [3][cap_cases+1]: points, beams, tiles
  int cap_cases = 0;
  std::vector<CaseDev> h_cases;
  std::vector<int64_t> h_bases;
  std::vector<int32_t> h_pbcase;
  std::vector<int64_t> h_pbrange;
  // graph
  hipGraphExec_t gexec = nullptr;
  // overflow word of the last replay, copied by the graph's last node into
  // mapped host memory, and an event recorded after each replay
  uint32_t *h_ovf = nullptr, *d_ovf = nullptr;
  hipEvent_t ev_replay = nullptr;
  bool replay_pending = false;
  std::vector<alp_case> gkey;
  uint32_t gflags = 0;
  int last_cases = 0;
  // where the last step left its counters and diagnostics (the workspace of
  // the allocation-free entry point lives in the device scratch array)
  const long long *dg_cnt = nullptr;
  const double *dg_out = nullptr;
  const uint32_t *dg_counters = nullptr;
  unsigned char *scratch = nullptr;  // this device's scratch array (device address)
  int any_kernel_sample = 0;  // some case of the uploaded batch samples with the kernel
  int any_proj[4] = {0, 0, 0, 0};  // the uploaded batch has cases of each (rule, precision)
  // launch shape of the step's kernels, and the cases ALP_AUTOTUNE chose it for
  alp_tuning tun{4, 0, 4, 16, 0};
  std::vector<alp_case> tkey;
};

// Workspace of alp_step_noalloc: every per-step list, the case table and
// the scan temporaries of a step, carved from one static device array.  Each
// device the library runs on holds its own copy until the process ends.  In
// host code `scratch` names a host-side stand-in: its device address comes
// from hipGetSymbolAddress, once per device with that device current, and
// only that address is ever passed to a kernel or a copy.
constexpr size_t kScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
std::mutex g_scratch_mu;
constexpr int kMaxDevices = 64;
unsigned char *g_scratch_ptr[kMaxDevices] = {};

// the device address of this device's scratch array (the device must be current)
hipError_t scratch_address(int device, unsigned char **out) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = (unsigned char *)p;
  }
  *out = g_scratch_ptr[device];
  return hipSuccess;
}
}  // namespace

namespace {

alp_status fail(alp_context *ctx, alp_status code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (ctx) ctx->err = buf;
  return code;
}

#define HIPCHK(ctx, call)                                                                      \
  do {                                                                                         \
    hipError_t e_ = (call);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return fail(ctx, e_ == hipErrorOutOfMemory ? ALP_ERR_OOM : ALP_ERR_HIP, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                           \
  } while (0)

template <typename T>
alp_status dalloc(alp_context *ctx, T **p, int64_t n) {
  *p = nullptr;
  size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(T);
  HIPCHK(ctx, hipMalloc((void **)p, bytes));
  return ALP_OK;
}

void free_work(alp_context *ctx) {
  for (void *p : ctx->wallocs) (void)hipFree(p);
  ctx->wallocs.clear();
  std::memset(&ctx->w, 0, sizeof(ctx->w));
  ctx->have_points = ctx->have_beams = ctx->have_tiles = ctx->have_cases = ctx->have_pblocks = -1;
  ctx->have_emit = ctx->have_item = ctx->have_rec = ctx->have_chunk = -1;
  if (ctx->scan_tmp) (void)hipFree(ctx->scan_tmp);
  ctx->scan_tmp = nullptr;
  ctx->have_scan = -1;
}

void drop_graph(alp_context *ctx) {
  if (ctx->gexec) (void)hipGraphExecDestroy(ctx->gexec);
  ctx->gexec = nullptr;
  ctx->gkey.clear();
  ctx->replay_pending = false;
  if (ctx->h_ovf) *ctx->h_ovf = 0u;
}

bool is_capturing(alp_context *ctx) {
  hipStreamCaptureStatus s = hipStreamCaptureStatusNone;
  if (ctx->user && hipStreamIsCapturing(ctx->user, &s) == hipSuccess &&
      s != hipStreamCaptureStatusNone)
    return true;
  return false;
}

// event ordering between the caller's stream and the internal stream
alp_status enter(alp_context *ctx) {
  HIPCHK(ctx, hipSetDevice(ctx->device));
  HIPCHK(ctx, hipEventRecord(ctx->ev_in, ctx->user));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->st, ctx->ev_in, 0));
  return ALP_OK;
}
alp_status leave(alp_context *ctx) {
  HIPCHK(ctx, hipEventRecord(ctx->ev_out, ctx->st));
  HIPCHK(ctx, hipStreamWaitEvent(ctx->user, ctx->ev_out, 0));
  return ALP_OK;
}
// wait for everything enqueued so far on the caller's stream (graph replays
// run there) and on the internal stream
alp_status settle(alp_context *ctx) {
  alp_status rc = enter(ctx);
  if (rc != ALP_OK) return rc;
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return ALP_OK;
}


// Work-list capacities and per-case sizes for one step.
struct StepShape {
  int n_cases = 0;
  int64_t n_points = 0, n_beams = 0, n_tiles = 0, n_cells = 0;
  int64_t cap_chunk = 0, cap_item = 0;
  int n_pblocks = 0;
};

alp_status ensure_work(alp_context *ctx, const StepShape &sh, int64_t want_emit, int64_t want_rec) {
  Work &w = ctx->w;
  bool grow = sh.n_points > ctx->have_points || sh.n_beams > ctx->have_beams ||
              sh.n_tiles > ctx->have_tiles || sh.n_cases > ctx->have_cases ||
              sh.n_pblocks > ctx->have_pblocks || want_emit > ctx->have_emit ||
              sh.cap_item > ctx->have_item || want_rec > ctx->have_rec ||
              sh.cap_chunk > ctx->have_chunk;
  if (!grow) {
    w.rec_compact = sh.n_points < kRecCompactPoints ? 1 : 0;
    w.n_points = sh.n_points;
    w.n_beams = sh.n_beams;
    w.n_tiles = sh.n_tiles;
    w.n_cases = sh.n_cases;
    w.n_pblocks = sh.n_pblocks;
    return ALP_OK;
  }
  (void)hipStreamSynchronize(ctx->st);
  drop_graph(ctx);
  // keep every dimension at least as large as before
  int64_t P = std::max(sh.n_points, ctx->have_points), B = std::max(sh.n_beams, ctx->have_beams);
  int64_t T = std::max(sh.n_tiles, ctx->have_tiles);
  int64_t NC = std::max<int64_t>(sh.n_cases, ctx->have_cases);
  int64_t PB = std::max<int64_t>(sh.n_pblocks, ctx->have_pblocks);
  int64_t EM = std::max(want_emit, ctx->have_emit), IT = std::max(sh.cap_item, ctx->have_item);
  int64_t RC = std::max(want_rec, ctx->have_rec), CH = std::max(sh.cap_chunk, ctx->have_chunk);
  free_work(ctx);
  std::vector<void *> &A = ctx->wallocs;
  alp_status rc;
#define WALLOC(field, n)                                  \
  do {                                                    \
    if ((rc = dalloc(ctx, &w.field, (n))) != ALP_OK) return rc; \
    A.push_back((void *)w.field);                         \
  } while (0)
  WALLOC(pbeam, P);
  WALLOC(pflags, P);
  WALLOC(wexp, P);
  WALLOC(w_hi, P);
  WALLOC(w_lo, P);
  WALLOC(fhat, 3 * (P + 2));  // two nodes of slack: the spread reads both nodes of every record
  WALLOC(Us, 3 * P);
  WALLOC(Ps, 3 * P);
  WALLOC(As, 3 * P);
  WALLOC(f, 3 * P);
  WALLOC(bcase, B);
  WALLOC(beps_max, B);
  WALLOC(bchunks, B + 1);
  WALLOC(chunk_beam, CH);
  WALLOC(chunk_s0, CH);
  WALLOC(chunk_s1, CH);
  WALLOC(chunk_box, CH + 1);
  WALLOC(chunk_bx, 6 * CH);
  WALLOC(tile_cnt, T + 1);
  WALLOC(tile_off, T + 1);
  WALLOC(tile_fill, T + 1);
  WALLOC(tile_nent, T + 1);
  WALLOC(tile_items, T + 1);
  WALLOC(tile_itoff, T + 1);
  WALLOC(big_tiles, T + 1);
  WALLOC(emit_raw, EM);
  WALLOC(emit, EM);
  WALLOC(entry, EM);
  WALLOC(item, IT);
  WALLOC(multi_items, IT);
  WALLOC(rec_base, IT);
  WALLOC(rec_cnt, IT);
  WALLOC(rec, RC + (int64_t)kRecSlack);  // the spread reads 24 bytes from every record's start
  WALLOC(rec_alloc, 1);
  WALLOC(F_hi, 3 * NC);
  WALLOC(F_lo, 3 * NC);
  WALLOC(F_exp, NC);
  WALLOC(beam_part, 4 * PB);
  WALLOC(pblock_case, PB);
  WALLOC(pblock_range, 2 * PB);
  WALLOC(cnt, kCnt * NC);
  WALLOC(diag_out, 16 * NC);
  WALLOC(counters, kCounters);
#undef WALLOC
  int64_t sc = scan_tmp_words(std::max({B + 1, T + 1, CH + 1, (int64_t)1}));
  if ((rc = dalloc(ctx, &ctx->scan_tmp, sc)) != ALP_OK) return rc;
  ctx->have_scan = sc;
  w.scan_tmp = ctx->scan_tmp;
  HIPCHK(ctx, hipMemsetAsync(w.counters, 0, kCounters * sizeof(uint32_t), ctx->st));
  HIPCHK(ctx, hipMemsetAsync(w.cnt, 0, kCnt * NC * sizeof(long long), ctx->st));
  HIPCHK(ctx, hipMemsetAsync(w.diag_out, 0, 16 * NC * sizeof(double), ctx->st));
  w.cap_emit = EM;
  w.cap_item = IT;
  w.cap_rec = RC;
  w.cap_chunk = CH;
  ctx->have_points = P;
  ctx->have_beams = B;
  ctx->have_tiles = T;
  ctx->have_cases = NC;
  ctx->have_pblocks = PB;
  ctx->have_emit = EM;
  ctx->have_item = IT;
  ctx->have_rec = RC;
  ctx->have_chunk = CH;
  w.n_points = sh.n_points;
  w.n_beams = sh.n_beams;
  w.n_tiles = sh.n_tiles;
  w.n_cases = sh.n_cases;
  w.n_pblocks = sh.n_pblocks;
  w.rec_compact = sh.n_points < kRecCompactPoints ? 1 : 0;
  return ALP_OK;
}

alp_status ensure_cases(alp_context *ctx, int n) {
  if (n <= ctx->cap_cases) return ALP_OK;
  (void)hipStreamSynchronize(ctx->st);
  drop_graph(ctx);
  if (ctx->d_cases) (void)hipFree(ctx->d_cases);
  if (ctx->d_bases) (void)hipFree(ctx->d_bases);
  ctx->d_cases = nullptr;
  ctx->d_bases = nullptr;
  int cap = std::max(n, 8);
  alp_status rc;
  if ((rc = dalloc(ctx, &ctx->d_cases, cap)) != ALP_OK) return rc;
  if ((rc = dalloc(ctx, &ctx->d_bases, 3 * (cap + 1))) != ALP_OK) return rc;
  ctx->cap_cases = cap;
  return ALP_OK;
}

alp_status check_beams(alp_context *ctx, const alp_beams *b, bool need_spread_fields,
                       bool need_sample_fields, bool copy_offsets) {
  if (!b) return fail(ctx, ALP_ERR_INVALID_ARG, "beams is NULL");
  if (b->n_beams < 0 || b->n_points < 0 || b->n_points >= (int64_t)INT32_MAX)
    return fail(ctx, ALP_ERR_INVALID_ARG, "bad beam counts (n_beams=%d, n_points=%lld)",
                b->n_beams, (long long)b->n_points);
  if (b->n_beams > 0 && !b->offsets) return fail(ctx, ALP_ERR_INVALID_ARG, "beams.offsets is NULL");
  if (b->n_points > 0) {
    if (!b->P || !b->e_t || !b->Pdot || !b->d || !b->L || !b->eps)
      return fail(ctx, ALP_ERR_INVALID_ARG, "a per-point beam array is NULL");
  }
  if (b->n_beams > 0 && (!b->Cdn || !b->Cdt || !b->ls || !b->n_p || !b->e_up))
    return fail(ctx, ALP_ERR_INVALID_ARG, "a per-beam array is NULL");
  if (b->A && b->n_beams > 0 && (!b->CMn || !b->CMt))
    return fail(ctx, ALP_ERR_INVALID_ARG, "beams.A needs beams.CMn and beams.CMt");
  (void)need_spread_fields;
  (void)need_sample_fields;
  if (copy_offsets && b->n_beams > 0) {
    // read on the caller's stream, which produced the array
    std::vector<int64_t> off((size_t)b->n_beams + 1);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipMemcpyAsync(off.data(), b->offsets, off.size() * sizeof(int64_t),
                               hipMemcpyDeviceToHost, ctx->user));
    HIPCHK(ctx, hipStreamSynchronize(ctx->user));
    if (off[0] != 0 || off[b->n_beams] != b->n_points)
      return fail(ctx, ALP_ERR_INVALID_ARG, "beams.offsets must start at 0 and end at n_points");
    for (int32_t i = 0; i < b->n_beams; ++i)
      if (off[i + 1] < off[i]) return fail(ctx, ALP_ERR_INVALID_ARG, "beams.offsets decreases at %d", i);
  }
  if (b->n_beams == 0 && b->n_points != 0)
    return fail(ctx, ALP_ERR_INVALID_ARG, "points without beams");
  return ALP_OK;
}

alp_status check_params(alp_context *ctx, const alp_params *p, bool relax) {
  if (!p) return fail(ctx, ALP_ERR_INVALID_ARG, "params is NULL");
  if (!(p->rho > 0.0) || !std::isfinite(p->rho)) return fail(ctx, ALP_ERR_INVALID_ARG, "rho must be > 0");
  if (relax && !(p->alpha_f > 0.0 && p->alpha_f <= 1.0))
    return fail(ctx, ALP_ERR_INVALID_ARG, "alpha_f must be in (0, 1]");
  if (!(p->tau >= 0.0) || !std::isfinite(p->tau)) return fail(ctx, ALP_ERR_INVALID_ARG, "tau must be >= 0");
  if (p->prec != ALP_PREC_FP64 && p->prec != ALP_PREC_FP32_SPLIT)
    return fail(ctx, ALP_ERR_INVALID_ARG, "unknown precision %d", p->prec);
  if (p->drag_form != ALP_DRAG_FULLMAG && p->drag_form != ALP_DRAG_COMPONENTWISE)
    return fail(ctx, ALP_ERR_INVALID_ARG, "unknown drag form %d", p->drag_form);
  if (p->sample_mode != ALP_SAMPLE_CELL && p->sample_mode != ALP_SAMPLE_KERNEL)
    return fail(ctx, ALP_ERR_INVALID_ARG, "unknown sample mode %d", p->sample_mode);
  if (p->proj_mode != ALP_PROJ_NEAREST && p->proj_mode != ALP_PROJ_INTEGRATED)
    return fail(ctx, ALP_ERR_INVALID_ARG, "unknown projection mode %d", p->proj_mode);
  return ALP_OK;
}

void fill_case(CaseDev &c, const alp_mesh *m, const alp_beams *b, const alp_params *p) {
  std::memset(&c, 0, sizeof(c));
  if (m) c.m = m->d;
  c.n_points = b->n_points;
  c.n_beams = b->n_beams;
  c.prec = p->prec;
  c.drag_form = p->drag_form;
  c.sample_mode = p->sample_mode;
  c.proj_mode = p->proj_mode;
  c.rho = p->rho;
  c.alpha_f = p->alpha_f;
  c.tau = p->tau;
  c.offsets = b->offsets;
  c.P = b->P;
  c.Psp = b->P_spread ? b->P_spread : b->P;
  c.e_t = b->e_t;
  c.Pdot = b->Pdot;
  c.d = b->d;
  c.L = b->L;
  c.eps = b->eps;
  c.Cdn = b->Cdn;
  c.Cdt = b->Cdt;
  c.ls = b->ls;
  c.n_p = b->n_p;
  c.e_up = b->e_up;
  c.A = b->A;
  c.CMn = b->CMn;
  c.CMt = b->CMt;
  c.a_b = b->a_b;
  if (m) c.tile_prev = m->tile_prev;
}

// global bases, point blocks for the beam-side sums, capacities
StepShape shape_cases(alp_context *ctx, std::vector<CaseDev> &cs) {
  StepShape sh;
  sh.n_cases = (int)cs.size();
  ctx->h_bases.assign(3 * (cs.size() + 1), 0);
  ctx->h_pbcase.clear();
  ctx->h_pbrange.clear();
  int64_t P = 0, B = 0, T = 0, NC = 0, CH = 0, IT = 0;
  for (size_t i = 0; i < cs.size(); ++i) {
    CaseDev &c = cs[i];
    c.point_base = P;
    c.beam_base = B;
    c.tile_base = T;
    ctx->h_bases[i] = P;
    ctx->h_bases[(cs.size() + 1) + i] = B;
    ctx->h_bases[2 * (cs.size() + 1) + i] = T;
    for (int64_t k0 = 0; k0 < c.n_points; k0 += 1024) {
      ctx->h_pbcase.push_back((int32_t)i);
      ctx->h_pbrange.push_back(k0);
      ctx->h_pbrange.push_back(std::min<int64_t>(k0 + 1024, c.n_points));
    }
    P += c.n_points;
    B += c.n_beams;
    T += c.m.n_tiles;
    NC += c.m.n_cells;
    CH += c.n_beams + (c.n_points + kChunkSegs - 1) / kChunkSegs + 1;
    IT += c.m.n_tiles + (c.m.n_cells + 63) / 64;
  }
  ctx->h_bases[cs.size()] = P;
  ctx->h_bases[2 * cs.size() + 1] = B;
  ctx->h_bases[3 * cs.size() + 2] = T;
  sh.n_points = P;
  sh.n_beams = B;
  sh.n_tiles = T;
  sh.n_cells = NC;
  sh.cap_chunk = CH;
  sh.cap_item = IT;
  sh.n_pblocks = (int)ctx->h_pbcase.size();
  return sh;
}

// which optional kernels the batch needs (sampling rule, projection rule and
// precision of each case)
void upload_flags(alp_context *ctx, const std::vector<CaseDev> &cs) {
  ctx->any_kernel_sample = 0;
  ctx->any_proj[0] = ctx->any_proj[1] = ctx->any_proj[2] = ctx->any_proj[3] = 0;
  for (const CaseDev &c : cs) {
    if (c.sample_mode == ALP_SAMPLE_KERNEL) ctx->any_kernel_sample = 1;
    ctx->any_proj[(c.proj_mode == ALP_PROJ_INTEGRATED ? 2 : 0) + (c.prec == ALP_PREC_FP32_SPLIT ? 0 : 1)] = 1;
  }
}

alp_status upload_cases(alp_context *ctx, const std::vector<CaseDev> &cs, const StepShape &sh) {
  alp_status rc;
  upload_flags(ctx, cs);
  if ((rc = ensure_cases(ctx, (int)cs.size())) != ALP_OK) return rc;
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_cases, cs.data(), cs.size() * sizeof(CaseDev),
                             hipMemcpyHostToDevice, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(ctx->d_bases, ctx->h_bases.data(), ctx->h_bases.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, ctx->st));
  if (sh.n_pblocks > 0) {
    HIPCHK(ctx, hipMemcpyAsync(ctx->w.pblock_case, ctx->h_pbcase.data(),
                               ctx->h_pbcase.size() * sizeof(int32_t), hipMemcpyHostToDevice, ctx->st));
    HIPCHK(ctx, hipMemcpyAsync(ctx->w.pblock_range, ctx->h_pbrange.data(),
                               ctx->h_pbrange.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->st));
  }
  // the host copies must outlive the asynchronous transfer
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  return ALP_OK;
}

// Sampler waves per CU while it runs beside the segment binning: four, which
// leaves the binning's small kernels the most room, unless the sampler would
// then need more than 16 passes over the CUs (a wave takes 64 / lanes points
// per pass), in which case eight, so that it still ends near the binning.
int sample_waves_beside(int64_t n_points, int n_cu, int lanes) {
  const int64_t pass4 = (int64_t)n_cu * 4 * (64 / lanes);  // points per pass at four waves per CU
  return n_points <= 16 * pass4 ? 4 : 8;
}

StepLaunch make_launch_from(alp_context *ctx, const Work &w, const CaseDev *d_cases, const int64_t *d_bases,
                            int n_cases) {
  StepLaunch L;
  L.cases = d_cases;
  L.pbase = d_bases;
  L.bbase = d_bases + (n_cases + 1);
  L.tbase = d_bases + 2 * (n_cases + 1);
  L.w = w;
  L.n_cases = n_cases;
  L.grid_persistent = ctx->n_cu * 8;
  const alp_tuning &t = ctx->tun;
  const int spw = t.spread_waves > 0 ? std::min(t.spread_waves, ctx->spread_per_cu) : ctx->spread_per_cu;
  L.grid_spread = ctx->n_cu * spw;
  L.grid_weights = ctx->n_cu * t.weights_waves;
  L.weights_grab = t.weights_grab;
  L.sample_lanes = t.sample_lanes;
  L.sample_waves = 0;
  L.kernel_sample = ctx->any_kernel_sample;
  L.near_split = ctx->any_proj[0];
  L.near_fp64 = ctx->any_proj[1];
  L.int_split = ctx->any_proj[2];
  L.int_fp64 = ctx->any_proj[3];
  return L;
}

StepLaunch make_launch(alp_context *ctx, int n_cases) {
  return make_launch_from(ctx, ctx->w, ctx->d_cases, ctx->d_bases, n_cases);
}

enum { ST_SAMPLE = 1, ST_DRAG = 2, ST_PROJECT = 4, ST_ALL = 7 };

const char *const kStageNames[] = {"prep", "sample", "drag", "segment_binning", "weights",
                                   "normalise", "spread", "finalise"};
constexpr int kNumStages = 8;

// the launch sequence of one step (no host synchronisation inside); when ev is
// given, ev[i+1] is recorded after stage i (ev[0] before the first)
void launch_sequence(alp_context *ctx, const StepLaunch &L, int stages, hipEvent_t *ev = nullptr,
                     uint32_t *ovf_dst = nullptr) {
  hipStream_t st = ctx->st;
  const Work &w = L.w;
  auto mark = [&](int i) {
    if (ev) (void)hipEventRecord(ev[i], st);
  };
  mark(0);
  if ((stages & ST_PROJECT) && (stages & ST_SAMPLE)) launch_step_reset(L, st);
  else if (stages & ST_PROJECT) launch_step_reset_project(L, st);
  else if (stages & ST_SAMPLE) launch_step_reset_sample(L, st);
  launch_points_prep(L, st);
  mark(1);
  // Sampling and drag (eq. 16-20) do not depend on the segment binning or the
  // weights pass (eq. 21-22): in a full step they run on the second stream and
  // join before the normalisation, which needs f.  The profiled step keeps
  // everything on one stream so that each stage is timed on its own.  (A fork
  // happens only in a full step, so the join below is always reached.)
  const bool fork = (stages == ST_ALL) && !ev;
  hipStream_t sd = fork ? ctx->st2 : st;
  if (fork) {
    (void)hipEventRecord(ctx->ev_fork, st);
    (void)hipStreamWaitEvent(sd, ctx->ev_fork, 0);
  }
  if (stages & ST_SAMPLE) {
    // beside the segment binning the sampler keeps to a few waves per CU,
    // which leaves the binning's small kernels room on every CU
    StepLaunch Ls = L;
    Ls.sample_waves = !fork ? 0
                      : (ctx->tun.sample_waves > 0 ? ctx->tun.sample_waves
                                                   : sample_waves_beside(L.w.n_points, ctx->n_cu, L.sample_lanes));
    launch_sample(Ls, sd);
    launch_sample_kernel(L, sd);
  }
  mark(2);
  if (stages & ST_DRAG) launch_drag(L, sd);
  // the beam-side sums need only f: with the drag, they stay on its stream
  if ((stages & ST_DRAG) && (stages & ST_PROJECT)) launch_beam_sums(L, sd);
  mark(3);
  if (!(stages & ST_PROJECT)) return;
  launch_beams_prep(L, st);
  launch_scan_u32(w.bchunks, w.bchunks, w.n_beams, w.scan_tmp, st);
  launch_chunks(L, st);
  launch_chunk_boxes(L, st);
  launch_scan_u32(w.chunk_box, w.chunk_box, w.cap_chunk, w.scan_tmp, st);
  launch_chunk_tiles(L, st);
  launch_scan_u32(w.tile_cnt, w.tile_off, w.n_tiles, w.scan_tmp, st);
  launch_emit_scatter(L, st);
  launch_tile_merge(L, st);
  launch_scan_u32(w.tile_items, w.tile_itoff, w.n_tiles, w.scan_tmp, st);
  launch_items(L, st);
  mark(4);
  // the grouped weights kernels need only the work items: in a full step they
  // follow the drag on the second stream, beside the common weights kernels,
  // and both streams join before the normalisation
  if (fork) {
    (void)hipEventRecord(ctx->ev_items, st);
    (void)hipStreamWaitEvent(sd, ctx->ev_items, 0);
    launch_weights_grouped(L, sd);
    (void)hipEventRecord(ctx->ev_join, sd);
    launch_weights_main(L, st);
  } else {
    launch_weights_main(L, st);
    launch_weights_grouped(L, st);
  }
  mark(5);
  if (fork) (void)hipStreamWaitEvent(st, ctx->ev_join, 0);
  launch_norm(L, st);
  if (!(stages & ST_DRAG)) launch_beam_sums(L, st);
  mark(6);
  launch_spread(L, st);
  mark(7);
  launch_step_end(L, ovf_dst, st);
  mark(8);
}

// Clear S and the band state when an output array is used with a mesh for
// the first time (the incremental zeroing assumes S held the last source).
alp_status prepare_outputs(alp_context *ctx, const std::vector<alp_mesh *> &meshes,
                           const std::vector<double *> &S) {
  for (size_t i = 0; i < meshes.size(); ++i) {
    alp_mesh *m = meshes[i];
    if (!m || !S[i]) continue;
    if (m->last_S != S[i]) {
      launch_fill_f64(S[i], 0.0, 3 * (int64_t)m->d.n_cells, ctx->st);
      launch_fill_u8(m->tile_prev, 0, m->d.n_tiles, ctx->st);
      m->last_S = S[i];
    }
  }
  HIPCHK(ctx, hipGetLastError());
  return ALP_OK;
}

// read the overflow word and the sizes the lists needed (synchronises)
alp_status read_needs(alp_context *ctx, uint32_t &ovf, int64_t &need_emit, int64_t &need_rec) {
  uint32_t cnt[16];
  unsigned long long rb = 0;
  uint32_t em = 0;
  HIPCHK(ctx, hipMemcpyAsync(cnt, ctx->w.counters, sizeof(cnt), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(&rb, ctx->w.rec_alloc, sizeof(rb), hipMemcpyDeviceToHost, ctx->st));
  if (ctx->w.cap_chunk > 0)
    HIPCHK(ctx, hipMemcpyAsync(&em, ctx->w.chunk_box + ctx->w.cap_chunk, sizeof(em),
                               hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  ovf = cnt[3];
  need_emit = em;
  need_rec = (int64_t)rb;
  return ALP_OK;
}

// ALP_CHECKED: the record layout the weights pass left, checked on the host
// (synchronises).  Every item's records must lie inside the record area the
// wave allocator handed out, item ranges must not overlap, and a base may
// carry only its flag bits (record size, grouped item) below 16 bytes.  The
// spread reads records j < count of each item from its base and nothing else,
// so these invariants bound every record read of the step.
alp_status verify_records(alp_context *ctx) {
  const Work &w = ctx->w;
  uint32_t n_items = 0;
  unsigned long long used = 0;
  HIPCHK(ctx, hipMemcpyAsync(&n_items, w.tile_itoff + w.n_tiles, sizeof(n_items), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(&used, w.rec_alloc, sizeof(used), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  const size_t n = (size_t)std::min<int64_t>(n_items, w.cap_item);
  std::vector<uint32_t> cnt(n);
  std::vector<unsigned long long> base(n);
  if (n > 0) {
    HIPCHK(ctx, hipMemcpyAsync(cnt.data(), w.rec_cnt, n * sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->st));
    HIPCHK(ctx, hipMemcpyAsync(base.data(), w.rec_base, n * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               ctx->st));
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  }
  const unsigned long long limit = std::min<unsigned long long>(used, (unsigned long long)w.cap_rec);
  std::vector<std::pair<unsigned long long, unsigned long long>> r;
  r.reserve(n);
  for (size_t i = 0; i < n; ++i) {
    if (cnt[i] == 0) continue;
    if ((base[i] & 8ull) || (base[i] & 5ull) == 5ull)
      return fail(ctx, ALP_ERR_HIP, "record invariant: item %zu base 0x%llx", i, base[i]);
    const unsigned long long a = base[i] & ~15ull,
                             e = a + (unsigned long long)cnt[i] * ((base[i] & 1ull) ? 24 : ((base[i] & 4ull) ? 12 : 16));
    if (e > limit)
      return fail(ctx, ALP_ERR_HIP, "record invariant: item %zu records end at %llu beyond %llu", i, e, limit);
    // the spread reads kRecReadBytes from the start of every record
    if (e - (e - a) / cnt[i] + kRecReadBytes > (unsigned long long)w.cap_rec + kRecSlack)
      return fail(ctx, ALP_ERR_HIP, "record invariant: item %zu: a record read passes the record area", i);
    r.emplace_back(a, e);
  }
  std::sort(r.begin(), r.end());
  for (size_t i = 1; i < r.size(); ++i)
    if (r[i].first < r[i - 1].second)
      return fail(ctx, ALP_ERR_HIP, "record invariant: overlapping item records at %llu", r[i].first);
  return ALP_OK;
}

alp_status run_checked(alp_context *ctx, std::vector<CaseDev> &cs, int stages,
                       const std::vector<alp_mesh *> &meshes, const std::vector<double *> &S,
                       bool verify = false) {
  StepShape sh = shape_cases(ctx, cs);
  int64_t want_emit = std::max<int64_t>(ctx->have_emit, 16 * sh.n_points + 4096);
  int64_t want_rec = std::max<int64_t>(ctx->have_rec, 24 * (3 * sh.n_cells + (1 << 16)) +
                                                        (int64_t)ctx->n_cu * 8 * (int64_t)kRecBlock);
  for (int attempt = 0; attempt < 4; ++attempt) {
    alp_status rc = ensure_work(ctx, sh, want_emit, want_rec);
    if (rc != ALP_OK) return rc;
    if ((rc = upload_cases(ctx, cs, sh)) != ALP_OK) return rc;
    if ((rc = prepare_outputs(ctx, meshes, S)) != ALP_OK) return rc;
    StepLaunch L = make_launch(ctx, (int)cs.size());
    launch_sequence(ctx, L, stages);
    HIPCHK(ctx, hipGetLastError());
    if (!(stages & ST_PROJECT)) return ALP_OK;
    uint32_t ovf;
    int64_t ne, nr;
    if ((rc = read_needs(ctx, ovf, ne, nr)) != ALP_OK) return rc;
    if (ovf == 0) return verify ? verify_records(ctx) : ALP_OK;
    if (ovf & (4u | 8u | 16u))
      return fail(ctx, ALP_ERR_CAPACITY,
                  "per-tile limits exceeded (flags 0x%x): more than %d segment windows in one tile",
                  ovf, kMaxEmitBig);
    want_emit = std::max(want_emit, ne + ne / 2 + 1024);
    want_rec = std::max(want_rec, nr + nr / 2 + (int64_t)ctx->n_cu * 8 * (int64_t)kRecBlock);
    // the band state was updated by the failed attempt: force a full clear
    for (alp_mesh *m : meshes)
      if (m) m->last_S = nullptr;
  }
  return fail(ctx, ALP_ERR_CAPACITY, "work lists kept overflowing");
}

// Validate a batch and fill its device case table (host copy), the meshes and
// the source arrays, in case order.
alp_status build_batch(alp_context *ctx, int32_t n_cases, const alp_case *cases, std::vector<CaseDev> &cs,
                       std::vector<alp_mesh *> &meshes, std::vector<double *> &S) {
  alp_status rc;
  cs.assign((size_t)n_cases, CaseDev{});
  meshes.assign((size_t)n_cases, nullptr);
  S.assign((size_t)n_cases, nullptr);
  for (int i = 0; i < n_cases; ++i) {
    const alp_case &c = cases[i];
    if (!c.mesh || !c.U || !c.S || (!c.f && c.beams.n_points > 0))
      return fail(ctx, ALP_ERR_INVALID_ARG, "case %d: mesh, U, f and S are required (f only with points)", i);
    for (int j = 0; j < i; ++j)
      if (cases[j].mesh == c.mesh)
        return fail(ctx, ALP_ERR_INVALID_ARG, "case %d: a mesh may appear in one case per batch", i);
    if ((rc = check_beams(ctx, &c.beams, true, true, true)) != ALP_OK) return rc;
    if ((rc = check_params(ctx, &c.params, c.f_prev != nullptr)) != ALP_OK) return rc;
    alp_mesh *m = const_cast<alp_mesh *>(c.mesh);
    fill_case(cs[i], m, &c.beams, &c.params);
    cs[i].U = c.U;
    cs[i].f_prev = c.f_prev;
    cs[i].has_fprev = c.f_prev != nullptr;
    cs[i].f = c.f;
    cs[i].S = c.S;
    cs[i].U_s = c.U_s;
    cs[i].w = c.w;
    cs[i].P_s = c.P_s;
    cs[i].cell_a = c.cell_a;
    cs[i].cell_s = c.cell_s;
    cs[i].dUdt = c.dUdt;
    cs[i].write_S = 1;
    meshes[i] = m;
    S[i] = c.S;
  }
  return ALP_OK;
}


// Carves 256-byte aligned arrays out of the scratch array, front to back.
struct Carver {
  unsigned char *base;
  size_t size, off = 0;
  bool ok = true;
  template <typename T>
  T *take(int64_t n) {
    const size_t bytes = (size_t)(n > 0 ? n : 1) * sizeof(T);
    const size_t o = (off + 255) & ~(size_t)255;
    if (o + bytes > size) {
      ok = false;
      return nullptr;
    }
    off = o + bytes;
    return reinterpret_cast<T *>(base + o);
  }
};

// The fixed part of a step's workspace (every list whose length the host
// knows), the case table and the scan temporaries, carved in that order.
// Returns false if they do not fit.
bool carve_fixed(Carver &cv, Work &w, const StepShape &sh, CaseDev **d_cases, int64_t **d_bases) {
  const int64_t P = sh.n_points, B = sh.n_beams, T = sh.n_tiles, NC = sh.n_cases, PB = sh.n_pblocks;
  const int64_t IT = sh.cap_item, CH = sh.cap_chunk;
  std::memset(&w, 0, sizeof(w));
  w.counters = cv.take<uint32_t>(kCounters);
  w.cnt = cv.take<long long>(kCnt * NC);
  w.diag_out = cv.take<double>(16 * NC);
  w.pbeam = cv.take<int32_t>(P);
  w.pflags = cv.take<int32_t>(P);
  w.wexp = cv.take<int32_t>(P);
  w.w_hi = cv.take<long long>(P);
  w.w_lo = cv.take<unsigned long long>(P);
  w.fhat = cv.take<double>(3 * (P + 2));
  w.Us = cv.take<double>(3 * P);
  w.Ps = cv.take<double>(3 * P);
  w.As = cv.take<double>(3 * P);
  w.f = cv.take<double>(3 * P);
  w.bcase = cv.take<int32_t>(B);
  w.beps_max = cv.take<double>(B);
  w.bchunks = cv.take<uint32_t>(B + 1);
  w.chunk_beam = cv.take<int32_t>(CH);
  w.chunk_s0 = cv.take<int32_t>(CH);
  w.chunk_s1 = cv.take<int32_t>(CH);
  w.chunk_box = cv.take<uint32_t>(CH + 1);
  w.chunk_bx = cv.take<int32_t>(6 * CH);
  w.tile_cnt = cv.take<uint32_t>(T + 1);
  w.tile_off = cv.take<uint32_t>(T + 1);
  w.tile_fill = cv.take<uint32_t>(T + 1);
  w.tile_nent = cv.take<uint32_t>(T + 1);
  w.tile_items = cv.take<uint32_t>(T + 1);
  w.tile_itoff = cv.take<uint32_t>(T + 1);
  w.big_tiles = cv.take<uint32_t>(T + 1);
  w.item = cv.take<Item>(IT);
  w.multi_items = cv.take<uint32_t>(IT);
  w.rec_base = cv.take<unsigned long long>(IT);
  w.rec_cnt = cv.take<uint32_t>(IT);
  w.rec_alloc = cv.take<unsigned long long>(1);
  w.F_hi = cv.take<long long>(3 * NC);
  w.F_lo = cv.take<unsigned long long>(3 * NC);
  w.F_exp = cv.take<int32_t>(NC);
  w.beam_part = cv.take<double>(4 * PB);
  w.pblock_case = cv.take<int32_t>(PB);
  w.pblock_range = cv.take<int64_t>(2 * PB);
  w.scan_tmp = cv.take<uint32_t>(scan_tmp_words(std::max({B + 1, T + 1, CH + 1, (int64_t)1})));
  *d_cases = cv.take<CaseDev>(NC);
  *d_bases = cv.take<int64_t>(3 * (NC + 1));
  w.cap_item = IT;
  w.cap_chunk = CH;
  w.n_points = P;
  w.n_beams = B;
  w.n_tiles = T;
  w.n_cases = (int32_t)NC;
  w.n_pblocks = PB;
  w.rec_compact = P < kRecCompactPoints ? 1 : 0;
  return cv.ok;
}

// ALP_AUTOTUNE: the launch shape of a batch by coordinate descent over the
// sampler (lanes per point, waves per CU), the weights pass (queue grab,
// waves per CU) and the spread (waves per CU), each candidate timed over
// graph replays of the step (the caller's outputs are overwritten).  A
// candidate is kept only if it is faster by more than 1%.
alp_status tune_launch(alp_context *ctx, int32_t n, const alp_case *cases, uint32_t flags) {
  flags = (flags & ~(ALP_AUTOTUNE | ALP_CHECKED)) | ALP_USE_GRAPH;
  constexpr int kReps = 5;
  hipEvent_t ea = nullptr, eb = nullptr;
  HIPCHK(ctx, hipEventCreate(&ea));
  HIPCHK(ctx, hipEventCreate(&eb));
  auto timed = [&](const alp_tuning &t, double &ms) -> alp_status {
    ctx->tun = t;
    drop_graph(ctx);
    alp_status rc = alp_step_batched(ctx, n, cases, flags);  // sizes, runs and captures
    for (int r = 0; r < 1 && rc == ALP_OK; ++r) rc = alp_step_batched(ctx, n, cases, flags);
    if (rc != ALP_OK) return rc;
    if (hipEventRecord(ea, ctx->user) != hipSuccess) return fail(ctx, ALP_ERR_HIP, "event record failed");
    for (int r = 0; r < kReps && rc == ALP_OK; ++r) rc = alp_step_batched(ctx, n, cases, flags);
    if (rc != ALP_OK) return rc;
    float e = 0.f;
    if (hipEventRecord(eb, ctx->user) != hipSuccess || hipEventSynchronize(eb) != hipSuccess ||
        hipEventElapsedTime(&e, ea, eb) != hipSuccess)
      return fail(ctx, ALP_ERR_HIP, "timing the candidate failed");
    ms = e / kReps;
    return ALP_OK;
  };
  alp_tuning best = ctx->tun;
  double best_ms = INFINITY;
  alp_status rc = timed(best, best_ms);
  const int samp[][2] = {{4, 0}, {4, 4}, {4, 8}, {4, 16}, {2, 4}, {2, 8}, {8, 4}, {8, 8}};
  const int grab[] = {2, 4, 8};
  const int wwav[] = {8, 12, 16, 24};
  const int swav[] = {0, 1};  // spread workgroups (16 waves each) per CU: all a CU holds, or one
  auto consider = [&](const alp_tuning &t) {
    if (rc != ALP_OK) return;
    double ms = INFINITY;
    rc = timed(t, ms);
    if (rc == ALP_OK && ms < 0.99 * best_ms) {
      best = t;
      best_ms = ms;
    }
  };
  for (const auto &c : samp) {
    alp_tuning t = best;
    t.sample_lanes = c[0];
    t.sample_waves = c[1];
    if (t.sample_lanes != best.sample_lanes || t.sample_waves != best.sample_waves) consider(t);
  }
  for (int g : grab) {
    alp_tuning t = best;
    t.weights_grab = g;
    if (g != best.weights_grab) consider(t);
  }
  for (int w : wwav) {
    alp_tuning t = best;
    t.weights_waves = w;
    if (w != best.weights_waves) consider(t);
  }
  for (int w : swav) {
    alp_tuning t = best;
    t.spread_waves = w;
    if (w != best.spread_waves) consider(t);
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  ctx->tun = best;
  drop_graph(ctx);
  return rc;
}

bool tuning_valid(const alp_tuning &t) {
  return (t.sample_lanes == 2 || t.sample_lanes == 4 || t.sample_lanes == 8) && t.sample_waves >= 0 &&
         t.sample_waves <= 32 && t.weights_grab >= 1 && t.weights_grab <= 16 && t.weights_waves >= 1 &&
         t.weights_waves <= 32 && t.spread_waves >= 0 && t.spread_waves <= 32;
}

}  // namespace

// ================================================================= C ABI ==
extern "C" {

const char *alp_version(void) { return "libalp 0.1 (gfx950)"; }

alp_status alp_create(int device, void *hip_stream, alp_context **out) {
  if (!out) return ALP_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return ALP_ERR_HIP;
  if (device < 0 || device >= ndev) return ALP_ERR_INVALID_ARG;
  alp_context *ctx = new alp_context();
  ctx->device = device;
  ctx->user = (hipStream_t)hip_stream;
  if (hipSetDevice(device) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->st, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipStreamCreateWithFlags(&ctx->st2, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_fork, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_join, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_items, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&ctx->ev_replay, hipEventDisableTiming) != hipSuccess ||
      hipHostMalloc((void **)&ctx->h_ovf, sizeof(uint32_t), hipHostMallocMapped) != hipSuccess ||
      hipHostGetDevicePointer((void **)&ctx->d_ovf, ctx->h_ovf, 0) != hipSuccess) {
    delete ctx;
    return ALP_ERR_HIP;
  }
  *ctx->h_ovf = 0u;
  if (scratch_address(device, &ctx->scratch) != hipSuccess) {
    alp_destroy(ctx);
    return ALP_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->n_cu = prop.multiProcessorCount;
  const int spc = spread_blocks_per_cu();
  if (spc > 0) ctx->spread_per_cu = spc;
  *out = ctx;
  return ALP_OK;
}

alp_status alp_destroy(alp_context *ctx) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  (void)hipSetDevice(ctx->device);
  (void)settle(ctx);
  drop_graph(ctx);
  free_work(ctx);
  if (ctx->d_cases) (void)hipFree(ctx->d_cases);
  if (ctx->d_bases) (void)hipFree(ctx->d_bases);
  (void)hipEventDestroy(ctx->ev_in);
  (void)hipEventDestroy(ctx->ev_out);
  (void)hipEventDestroy(ctx->ev_fork);
  (void)hipEventDestroy(ctx->ev_join);
  (void)hipEventDestroy(ctx->ev_items);
  (void)hipEventDestroy(ctx->ev_replay);
  if (ctx->h_ovf) (void)hipHostFree(ctx->h_ovf);
  (void)hipStreamDestroy(ctx->st2);
  (void)hipStreamDestroy(ctx->st);
  delete ctx;
  return ALP_OK;
}

const char *alp_last_error(const alp_context *ctx) { return ctx ? ctx->err.c_str() : "no context"; }

alp_status alp_bin_cells(alp_context *ctx, int64_t n_cells, const double *C, const double *V,
                         const double *domain_box, double bin_size, int32_t tile_bins,
                         alp_mesh **out) {
  if (!ctx || !out) return fail(ctx, ALP_ERR_INVALID_ARG, "NULL context or output");
  *out = nullptr;
  if (n_cells < 1 || n_cells >= (int64_t)INT32_MAX)
    return fail(ctx, ALP_ERR_INVALID_ARG, "n_cells must be in [1, 2^31)");
  if (!C || !V) return fail(ctx, ALP_ERR_INVALID_ARG, "C or V is NULL");
  if (tile_bins == 0) tile_bins = 4;
  if (tile_bins < 1 || tile_bins > 8) return fail(ctx, ALP_ERR_INVALID_ARG, "tile_bins must be in 1..8");
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "alp_bin_cells cannot run under capture");
  if (domain_box) {
    for (int a = 0; a < 3; ++a)
      if (!(domain_box[a] <= domain_box[3 + a]) || !std::isfinite(domain_box[a]) ||
          !std::isfinite(domain_box[3 + a]))
        return fail(ctx, ALP_ERR_INVALID_ARG, "domain_box must satisfy lo <= hi and be finite");
  }
  alp_status rc = enter(ctx);
  if (rc != ALP_OK) return rc;
  hipStream_t st = ctx->st;
  // bounds of the centres and the largest volume
  int nblk = mesh_bounds_blocks(n_cells);
  double *part = nullptr;
  if ((rc = dalloc(ctx, &part, 7 * nblk)) != ALP_OK) return rc;
  launch_mesh_bounds(C, V, n_cells, part, nblk, st);
  std::vector<double> hp(7 * (size_t)nblk);
  HIPCHK(ctx, hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(ctx, hipStreamSynchronize(st));
  (void)hipFree(part);
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY}, vmax = 0;
  for (int b = 0; b < nblk; ++b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::fmin(lo[a], hp[7 * b + a]);
      hi[a] = std::fmax(hi[a], hp[7 * b + 3 + a]);
    }
    vmax = std::fmax(vmax, hp[7 * b + 6]);
  }
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]))
      return fail(ctx, ALP_ERR_INVALID_ARG, "cell centres must be finite");
  if (!(vmax > 0.0) || !std::isfinite(vmax))
    return fail(ctx, ALP_ERR_INVALID_ARG, "cell volumes must be positive and finite");
  alp_mesh *m = new alp_mesh();
  m->device = ctx->device;
  MeshDev &d = m->d;
  d.n_cells = (int32_t)n_cells;
  d.T = tile_bins;
  d.vmax = vmax;
  double pad = 0.5 * std::cbrt(vmax);
  for (int a = 0; a < 3; ++a) {
    d.box[a] = domain_box ? domain_box[a] : lo[a] - pad;
    d.box[3 + a] = domain_box ? domain_box[3 + a] : hi[a] + pad;
  }
  double ext = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]});
  double b = bin_size;
  if (!(b > 0.0) || !std::isfinite(b)) {
    // cube root of the mean cell volume of the AABB (the cell size for a uniform mesh)
    double vol = 1.0;
    for (int a = 0; a < 3; ++a) vol *= std::max(hi[a] - lo[a] + 2 * pad, 1e-3 * (ext + 2 * pad));
    b = std::cbrt(vol / (double)n_cells);
  }
  if (!(b > 0.0)) b = 1.0;
  // keep the number of bins bounded (<= 4 n + 512 before tiling)
  for (;;) {
    double nbins = 1;
    for (int a = 0; a < 3; ++a) nbins *= std::floor((hi[a] - lo[a]) / b) + 1;
    if (nbins <= 4.0 * (double)n_cells + 512.0) break;
    b *= 1.25;
  }
  d.bin = b;
  d.inv_bin = 1.0 / b;
  d.tile_len = b * tile_bins;
  int64_t nbins = 1, ntiles = 1;
  for (int a = 0; a < 3; ++a) {
    d.lo[a] = lo[a];
    int64_t n = (int64_t)std::floor((hi[a] - lo[a]) / b) + 1;
    int64_t t = (n + tile_bins - 1) / tile_bins;
    d.nt[a] = (int32_t)t;
    d.nb[a] = (int32_t)(t * tile_bins);
    nbins *= d.nb[a];
    ntiles *= t;
  }
  if (nbins >= (int64_t)UINT32_MAX - 1) {
    delete m;
    return fail(ctx, ALP_ERR_INVALID_ARG, "mesh needs too many bins (%lld)", (long long)nbins);
  }
  d.n_bins = nbins;
  d.n_tiles = ntiles;
  uint32_t *key = nullptr, *count = nullptr, *tmp = nullptr, *ks = nullptr, *k2 = nullptr, *v2 = nullptr,
           *rcnt = nullptr, *bad = nullptr;
  auto free_scratch = [&]() {
    void *ps[] = {key, count, tmp, ks, k2, v2, rcnt, bad};
    for (void *p : ps)
      if (p) (void)hipFree(p);
  };
#define MALLOC_OR_FAIL(p, n)                      \
  if ((rc = dalloc(ctx, &(p), (n))) != ALP_OK) { \
    free_scratch();                               \
    alp_mesh_destroy(m);                          \
    return rc;                                    \
  }
  MALLOC_OR_FAIL(m->bin_start, nbins + 1);
  MALLOC_OR_FAIL(m->cxyz, 4 * n_cells);
  MALLOC_OR_FAIL(m->cx, n_cells);
  MALLOC_OR_FAIL(m->cy, n_cells);
  MALLOC_OR_FAIL(m->cz, n_cells);
  MALLOC_OR_FAIL(m->vs, n_cells);
  MALLOC_OR_FAIL(m->perm, n_cells);
  MALLOC_OR_FAIL(m->tile_prev, ntiles);
  MALLOC_OR_FAIL(key, n_cells);
  MALLOC_OR_FAIL(ks, n_cells);
  MALLOC_OR_FAIL(k2, n_cells);
  MALLOC_OR_FAIL(v2, n_cells);
  MALLOC_OR_FAIL(count, nbins + 1);
  MALLOC_OR_FAIL(rcnt, radix_scratch_words(n_cells));
  MALLOC_OR_FAIL(tmp, scan_tmp_words(std::max(nbins + 1, radix_scratch_words(n_cells))));
  MALLOC_OR_FAIL(bad, 1);
#undef MALLOC_OR_FAIL
  launch_fill_u32(count, 0u, nbins + 1, st);
  launch_fill_u32(bad, 0u, 1, st);
  launch_fill_u8(m->tile_prev, 0, ntiles, st);
  // bin keys and the bin CSR (exclusive scan of the histogram), then the
  // cell ids radix-sorted by key, the layout checked against both
  launch_bin_keys(d, C, n_cells, key, count, st);
  launch_scan_u32(count, m->bin_start, nbins, tmp, st);
  launch_radix_sort(key, n_cells, nbins, m->perm, ks, k2, v2, rcnt, tmp, st);
  launch_bin_check(key, ks, m->perm, m->bin_start, n_cells, bad, st);
  launch_bin_reorder(C, V, m->perm, n_cells, m->cxyz, m->cx, m->cy, m->cz, m->vs, st);
  uint32_t hbad = 0;
  hipError_t e = hipMemcpyAsync(&hbad, bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  free_scratch();
  if (e != hipSuccess) {
    alp_mesh_destroy(m);
    return fail(ctx, ALP_ERR_HIP, "binning failed: %s", hipGetErrorString(e));
  }
  if (hbad) {
    alp_mesh_destroy(m);
    return fail(ctx, ALP_ERR_HIP, "binned cell layout failed its check");
  }
  d.bin_start = m->bin_start;
  d.cxyz = m->cxyz;
  d.cx = m->cx;
  d.cy = m->cy;
  d.cz = m->cz;
  d.vs = m->vs;
  d.perm = m->perm;
  *out = m;
  return leave(ctx);
}

alp_status alp_mesh_destroy(alp_mesh *m) {
  if (!m) return ALP_ERR_INVALID_ARG;
  (void)hipSetDevice(m->device);
  (void)hipDeviceSynchronize();
  void *ps[] = {m->bin_start, m->cxyz, m->cx, m->cy, m->cz, m->vs, m->perm, m->tile_prev};
  for (void *p : ps)
    if (p) (void)hipFree(p);
  delete m;
  return ALP_OK;
}

alp_status alp_sample(alp_context *ctx, const alp_mesh *mesh, const double *U,
                      const alp_beams *beams, const alp_params *params, double *U_s, double *P_s,
                      int64_t *cell_a, int64_t *cell_s) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!mesh || !U) return fail(ctx, ALP_ERR_INVALID_ARG, "mesh or U is NULL");
  alp_status rc;
  if ((rc = check_beams(ctx, beams, false, true, true)) != ALP_OK) return rc;
  if (!U_s && beams->n_points > 0) return fail(ctx, ALP_ERR_INVALID_ARG, "U_s is NULL");
  if ((rc = check_params(ctx, params, false)) != ALP_OK) return rc;
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "use alp_step_batched under capture");
  if (beams->n_points == 0) return ALP_OK;
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  std::vector<CaseDev> cs(1);
  fill_case(cs[0], mesh, beams, params);
  cs[0].U = U;
  cs[0].U_s = U_s;
  cs[0].P_s = P_s;
  cs[0].cell_a = cell_a;
  cs[0].cell_s = cell_s;
  cs[0].tile_prev = nullptr;
  if ((rc = run_checked(ctx, cs, ST_SAMPLE, {}, {})) != ALP_OK) return rc;
  ctx->last_cases = 1;
  ctx->dg_cnt = nullptr;
  ctx->dg_out = nullptr;
  ctx->dg_counters = nullptr;
  return leave(ctx);
}

alp_status alp_drag(alp_context *ctx, const alp_beams *beams, const alp_params *params,
                    const double *U_s, const int64_t *cell_s, const double *f_prev, double *f) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  alp_status rc;
  if ((rc = check_beams(ctx, beams, false, true, true)) != ALP_OK) return rc;
  if ((!U_s || !f) && beams->n_points > 0) return fail(ctx, ALP_ERR_INVALID_ARG, "U_s or f is NULL");
  if ((rc = check_params(ctx, params, f_prev != nullptr)) != ALP_OK) return rc;
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "use alp_step_batched under capture");
  if (beams->n_points == 0) return ALP_OK;
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  std::vector<CaseDev> cs(1);
  fill_case(cs[0], nullptr, beams, params);
  cs[0].U_s = const_cast<double *>(U_s);
  cs[0].cell_s = const_cast<int64_t *>(cell_s);
  cs[0].f_prev = f_prev;
  cs[0].has_fprev = f_prev != nullptr;
  cs[0].f = f;
  StepShape sh = shape_cases(ctx, cs);
  if ((rc = ensure_work(ctx, sh, std::max<int64_t>(ctx->have_emit, 1), std::max<int64_t>(ctx->have_rec, 1))) != ALP_OK)
    return rc;
  if ((rc = upload_cases(ctx, cs, sh)) != ALP_OK) return rc;
  StepLaunch L = make_launch(ctx, 1);
  launch_points_prep(L, ctx->st);
  launch_drag_mode(L, 1, ctx->st);
  HIPCHK(ctx, hipGetLastError());
  return leave(ctx);
}

alp_status alp_spread(alp_context *ctx, const alp_mesh *mesh, const alp_beams *beams,
                      const alp_params *params, const double *f, double *S, double *w,
                      double *fhat) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!mesh || !S) return fail(ctx, ALP_ERR_INVALID_ARG, "mesh or S is NULL");
  alp_status rc;
  if ((rc = check_beams(ctx, beams, true, false, true)) != ALP_OK) return rc;
  if (!f && beams->n_points > 0) return fail(ctx, ALP_ERR_INVALID_ARG, "f is NULL");
  if ((rc = check_params(ctx, params, false)) != ALP_OK) return rc;
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "use alp_step_batched under capture");
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  std::vector<CaseDev> cs(1);
  alp_mesh *m = const_cast<alp_mesh *>(mesh);
  fill_case(cs[0], m, beams, params);
  cs[0].f = const_cast<double *>(f);
  cs[0].S = S;
  cs[0].w = w;
  cs[0].fhat = fhat;
  cs[0].write_S = 1;
  if ((rc = run_checked(ctx, cs, ST_PROJECT, {m}, {S})) != ALP_OK) return rc;
  ctx->last_cases = 1;
  ctx->dg_cnt = nullptr;
  ctx->dg_out = nullptr;
  ctx->dg_counters = nullptr;
  return leave(ctx);
}

alp_status alp_step_batched(alp_context *ctx, int32_t n_cases, const alp_case *cases,
                            uint32_t flags) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (n_cases < 1 || !cases) return fail(ctx, ALP_ERR_INVALID_ARG, "need n_cases >= 1 and cases");
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "the stream is capturing");
  alp_status rc;
  if (flags & ALP_AUTOTUNE) {
    // choose the launch shape once per set of case descriptors
    flags &= ~ALP_AUTOTUNE;
    if (!((int)ctx->tkey.size() == n_cases &&
          std::memcmp(ctx->tkey.data(), cases, sizeof(alp_case) * (size_t)n_cases) == 0)) {
      if ((rc = tune_launch(ctx, n_cases, cases, flags)) != ALP_OK) return rc;
      ctx->tkey.assign(cases, cases + n_cases);
    }
  }
  bool use_graph = (flags & ALP_USE_GRAPH) != 0;
  // replay an existing graph for identical case descriptors
  if (use_graph && ctx->gexec && (int)ctx->gkey.size() == n_cases && ctx->gflags == flags &&
      std::memcmp(ctx->gkey.data(), cases, sizeof(alp_case) * (size_t)n_cases) == 0) {
    // an earlier replay whose work lists overflowed (the arrays may have been
    // updated in place past the captured capacities): report it, drop the
    // graph, and let the next call size the lists again
    if (ctx->replay_pending && hipEventQuery(ctx->ev_replay) == hipSuccess) {
      ctx->replay_pending = false;
      const uint32_t ovf = __atomic_load_n(ctx->h_ovf, __ATOMIC_ACQUIRE);
      if (ovf) {
        drop_graph(ctx);
        return fail(ctx, ALP_ERR_CAPACITY,
                    "an earlier graph replay overflowed its work lists (0x%x); its results are invalid "
                    "and the graph was dropped",
                    ovf);
      }
    }
    // the replay runs on the caller's stream itself: it is ordered after the
    // caller's earlier work and before its later work with no event hand-over
    // (every other call orders the internal stream after the caller's first)
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipGraphLaunch(ctx->gexec, ctx->user));
    HIPCHK(ctx, hipEventRecord(ctx->ev_replay, ctx->user));
    ctx->replay_pending = true;
    ctx->last_cases = n_cases;
    ctx->dg_cnt = nullptr;
    ctx->dg_out = nullptr;
    ctx->dg_counters = nullptr;
    if (flags & ALP_CHECKED) {
      uint32_t ovf;
      int64_t ne, nr;
      if ((rc = enter(ctx)) != ALP_OK) return rc;
      if ((rc = read_needs(ctx, ovf, ne, nr)) != ALP_OK) return rc;
      if (ovf) return fail(ctx, ALP_ERR_CAPACITY, "work list overflow in graph replay (0x%x); call alp_invalidate", ovf);
      if ((rc = verify_records(ctx)) != ALP_OK) return rc;
    }
    return ALP_OK;
  }
  std::vector<CaseDev> cs;
  std::vector<alp_mesh *> meshes;
  std::vector<double *> S;
  if ((rc = build_batch(ctx, n_cases, cases, cs, meshes, S)) != ALP_OK) return rc;
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  // size the work lists with a checked run (this also produces this step's result)
  if ((rc = run_checked(ctx, cs, ST_ALL, meshes, S, (flags & ALP_CHECKED) != 0)) != ALP_OK) return rc;
  ctx->last_cases = n_cases;
  ctx->dg_cnt = nullptr;
  ctx->dg_out = nullptr;
  ctx->dg_counters = nullptr;
  if (use_graph) {
    drop_graph(ctx);
    HIPCHK(ctx, hipStreamSynchronize(ctx->st));
    StepLaunch L = make_launch(ctx, n_cases);
    hipGraph_t g = nullptr;
    HIPCHK(ctx, hipStreamBeginCapture(ctx->st, hipStreamCaptureModeThreadLocal));
    launch_sequence(ctx, L, ST_ALL, nullptr, ctx->d_ovf);
    hipError_t e = hipStreamEndCapture(ctx->st, &g);
    if (e != hipSuccess) return fail(ctx, ALP_ERR_HIP, "graph capture failed: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&ctx->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      ctx->gexec = nullptr;
      return fail(ctx, ALP_ERR_HIP, "graph instantiate failed: %s", hipGetErrorString(e));
    }
    ctx->gkey.assign(cases, cases + n_cases);
    ctx->gflags = flags;
  }
  return leave(ctx);
}

alp_status alp_step_noalloc(alp_context *ctx, int32_t n_cases, const alp_case *cases) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (n_cases < 1 || !cases) return fail(ctx, ALP_ERR_INVALID_ARG, "need n_cases >= 1 and cases");
  if (!ctx->scratch) return fail(ctx, ALP_ERR_HIP, "no scratch array on device %d", ctx->device);
  alp_status rc;
  std::vector<CaseDev> cs;
  std::vector<alp_mesh *> meshes;
  std::vector<double *> S;
  if ((rc = build_batch(ctx, n_cases, cases, cs, meshes, S)) != ALP_OK) return rc;
  StepShape sh = shape_cases(ctx, cs);
  // the fixed part first, then the window lists, then the pair records
  Carver cv{ctx->scratch, kScratchBytes};
  Work w;
  CaseDev *d_cases = nullptr;
  int64_t *d_bases = nullptr;
  if (!carve_fixed(cv, w, sh, &d_cases, &d_bases))
    return fail(ctx, ALP_ERR_CAPACITY,
                "the step needs %zu bytes of fixed workspace (%lld points, %lld beams, %lld tiles); the "
                "allocation-free entry point holds %zu",
                cv.off, (long long)sh.n_points, (long long)sh.n_beams, (long long)sh.n_tiles,
                (size_t)kScratchBytes);
  const size_t left = cv.size - ((cv.off + 255) & ~(size_t)255);
  // windows: three 16-byte lists per slot, up to 16 per point plus a margin,
  // and at most half of what is left; the pair records take the rest
  int64_t em = std::min<int64_t>(16 * sh.n_points + 4096, (int64_t)(left / 2 / 48));
  w.emit_raw = cv.take<Emit>(em);
  w.emit = cv.take<Win>(em);
  w.entry = cv.take<Entry>(em);
  const size_t rec_off = (cv.off + 255) & ~(size_t)255;
  const int64_t rc_bytes = cv.ok && rec_off < cv.size ? (int64_t)((cv.size - rec_off) & ~(size_t)255) : 0;
  w.rec = cv.take<unsigned char>(rc_bytes);
  if (!cv.ok || em <= 0 || rc_bytes <= (int64_t)kRecSlack)
    return fail(ctx, ALP_ERR_CAPACITY, "no room left for the window and pair lists in %zu bytes",
                (size_t)kScratchBytes);
  w.cap_emit = em;
  w.cap_rec = rc_bytes - (int64_t)kRecSlack;
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  // case table, bases and point blocks (from host arrays the context keeps);
  // the transfers complete before the host arrays can change
  upload_flags(ctx, cs);
  HIPCHK(ctx, hipMemcpyAsync(d_cases, cs.data(), cs.size() * sizeof(CaseDev), hipMemcpyHostToDevice, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(d_bases, ctx->h_bases.data(), ctx->h_bases.size() * sizeof(int64_t),
                             hipMemcpyHostToDevice, ctx->st));
  if (sh.n_pblocks > 0) {
    HIPCHK(ctx, hipMemcpyAsync(w.pblock_case, ctx->h_pbcase.data(), ctx->h_pbcase.size() * sizeof(int32_t),
                               hipMemcpyHostToDevice, ctx->st));
    HIPCHK(ctx, hipMemcpyAsync(w.pblock_range, ctx->h_pbrange.data(), ctx->h_pbrange.size() * sizeof(int64_t),
                               hipMemcpyHostToDevice, ctx->st));
  }
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  if ((rc = prepare_outputs(ctx, meshes, S)) != ALP_OK) return rc;
  StepLaunch L = make_launch_from(ctx, w, d_cases, d_bases, n_cases);
  // the step's reset kernel clears the counters, accumulators and tile
  // counts that must start at zero (the array keeps the last call's contents)
  launch_sequence(ctx, L, ST_ALL);
  HIPCHK(ctx, hipGetLastError());
  uint32_t ovf = 0;
  HIPCHK(ctx, hipMemcpyAsync(&ovf, w.counters + 3, sizeof(ovf), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  ctx->last_cases = n_cases;
  ctx->dg_cnt = w.cnt;
  ctx->dg_out = w.diag_out;
  ctx->dg_counters = w.counters;
  if (ovf) {
    // the band state of the meshes no longer matches their source arrays
    for (alp_mesh *m : meshes)
      if (m) m->last_S = nullptr;
    return fail(ctx, ALP_ERR_CAPACITY,
                "the step's window or pair lists exceed the allocation-free workspace (flags 0x%x, %lld "
                "window slots, %lld record bytes); use alp_step_batched",
                ovf, (long long)w.cap_emit, (long long)w.cap_rec);
  }
  return leave(ctx);
}

alp_status alp_beam_geometry(alp_context *ctx, const alp_mesh *mesh, const alp_beam_state *st, double *P,
                             double *e_t, double *eps, int64_t *counts) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!st) return fail(ctx, ALP_ERR_INVALID_ARG, "state is NULL");
  if (st->n_beams < 0 || st->n_points < 0 || st->n_points >= (int64_t)INT32_MAX || st->reserved0 != 0)
    return fail(ctx, ALP_ERR_INVALID_ARG, "bad beam counts (n_beams=%d, n_points=%lld)", st->n_beams,
                (long long)st->n_points);
  if (st->n_beams == 0 && st->n_points != 0) return fail(ctx, ALP_ERR_INVALID_ARG, "points without beams");
  if (st->n_beams > 0 && !st->offsets) return fail(ctx, ALP_ERR_INVALID_ARG, "state.offsets is NULL");
  if (st->n_points > 0 && (!st->Cb || !st->W)) return fail(ctx, ALP_ERR_INVALID_ARG, "state.Cb or state.W is NULL");
  if (!P && !e_t && !eps) return fail(ctx, ALP_ERR_INVALID_ARG, "nothing requested");
  if (eps && (!mesh || !st->eps_phys || !(st->eps_factor > 0.0) || !std::isfinite(st->eps_factor)))
    return fail(ctx, ALP_ERR_INVALID_ARG, "eps needs a mesh, state.eps_phys and eps_factor > 0");
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "alp_beam_geometry is not capturable");
  if (st->n_beams > 0) {
    std::vector<int64_t> off((size_t)st->n_beams + 1);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    HIPCHK(ctx, hipMemcpyAsync(off.data(), st->offsets, off.size() * sizeof(int64_t), hipMemcpyDeviceToHost,
                               ctx->user));
    HIPCHK(ctx, hipStreamSynchronize(ctx->user));
    if (off[0] != 0 || off[st->n_beams] != st->n_points)
      return fail(ctx, ALP_ERR_INVALID_ARG, "state.offsets must start at 0 and end at n_points");
    for (int32_t i = 0; i < st->n_beams; ++i)
      if (off[i + 1] < off[i]) return fail(ctx, ALP_ERR_INVALID_ARG, "state.offsets decreases at %d", i);
  }
  alp_status rc;
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  if (counts) HIPCHK(ctx, hipMemsetAsync(counts, 0, 2 * sizeof(int64_t), ctx->st));
  GeomLaunch G{};
  if (mesh) G.m = mesh->d;
  G.n_beams = st->n_beams;
  G.n_points = st->n_points;
  G.offsets = st->offsets;
  G.Cb = st->Cb;
  G.Wref = st->Wref;
  G.W = st->W;
  G.eps_phys = st->eps_phys;
  G.factor = st->eps_factor;
  G.P = P;
  G.e_t = e_t;
  G.eps = eps;
  G.counts = (unsigned long long *)counts;
  launch_beam_geometry(G, ctx->st);
  HIPCHK(ctx, hipGetLastError());
  return leave(ctx);
}

alp_status alp_autotune(alp_context *ctx, int64_t n_cells, const double *C, const double *V,
                        const double *domain_box, int32_t n_cases, const alp_case *cases,
                        int32_t tuned_case, uint32_t flags, int32_t reps, double *out_bin_size,
                        int32_t *out_tile_bins, double *out_ms) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!cases || n_cases < 1 || tuned_case < 0 || tuned_case >= n_cases || !out_bin_size ||
      !out_tile_bins)
    return fail(ctx, ALP_ERR_INVALID_ARG, "need cases, 0 <= tuned_case < n_cases and outputs");
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "alp_autotune cannot run under capture");
  if (reps <= 0) reps = 3;
  alp_status rc;
  // the default bin size of alp_bin_cells is the reference of the search
  alp_mesh *m0 = nullptr;
  if ((rc = alp_bin_cells(ctx, n_cells, C, V, domain_box, 0.0, 4, &m0)) != ALP_OK) return rc;
  const double base = m0->d.bin;
  alp_mesh_destroy(m0);
  const double scales[] = {0.75, 1.0, 1.5, 2.0};
  const int32_t tiles[] = {2, 3, 4, 5, 6};
  std::vector<alp_case> cs(cases, cases + n_cases);
  double best_ms = INFINITY, best_bin = base;
  int32_t best_t = 4;
  for (int32_t T : tiles) {
    for (double sc : scales) {
      alp_mesh *m = nullptr;
      if (alp_bin_cells(ctx, n_cells, C, V, domain_box, base * sc, T, &m) != ALP_OK) continue;
      cs[tuned_case].mesh = m;
      (void)alp_invalidate(ctx);
      rc = alp_step_batched(ctx, n_cases, cs.data(), flags | ALP_CHECKED);
      if (rc == ALP_OK) rc = alp_step_batched(ctx, n_cases, cs.data(), flags);
      if (rc == ALP_OK && hipStreamSynchronize(ctx->user) != hipSuccess) rc = ALP_ERR_HIP;
      double ms = INFINITY;
      if (rc == ALP_OK) {
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; r < reps && rc == ALP_OK; ++r) rc = alp_step_batched(ctx, n_cases, cs.data(), flags);
        if (rc == ALP_OK && hipStreamSynchronize(ctx->user) != hipSuccess) rc = ALP_ERR_HIP;
        const auto t1 = std::chrono::steady_clock::now();
        ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / reps;
      }
      (void)alp_invalidate(ctx);
      alp_mesh_destroy(m);
      if (rc == ALP_ERR_CAPACITY) continue;  // this binning exceeds a per-tile limit: skip it
      if (rc != ALP_OK) return rc;
      if (ms < best_ms) {
        best_ms = ms;
        best_bin = base * sc;
        best_t = T;
      }
    }
  }
  if (!(best_ms < INFINITY)) return fail(ctx, ALP_ERR_INVALID_ARG, "no binning setting could be built");
  *out_bin_size = best_bin;
  *out_tile_bins = best_t;
  if (out_ms) *out_ms = best_ms;
  return ALP_OK;
}

alp_status alp_autotune_binning(alp_context *ctx, int32_t n_cases, alp_case *cases, const double *const *C,
                                const double *const *V, const double *const *boxes, uint32_t flags, int32_t reps,
                                double *out_scale, int32_t *out_tile_bins, double *out_ms) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  ctx->err.clear();
  if (!cases || n_cases < 1 || !C || !V || !out_scale || !out_tile_bins)
    return fail(ctx, ALP_ERR_INVALID_ARG, "need cases, C, V and outputs");
  if (is_capturing(ctx)) return fail(ctx, ALP_ERR_CAPTURE, "alp_autotune_binning cannot run under capture");
  if (reps <= 0) reps = 3;
  flags &= ~ALP_AUTOTUNE;
  alp_status rc;
  // each case's default bin size is the reference of its candidates
  std::vector<double> base((size_t)n_cases);
  std::vector<int64_t> ncell((size_t)n_cases);
  for (int i = 0; i < n_cases; ++i) {
    if (!cases[i].mesh || !C[i] || !V[i]) return fail(ctx, ALP_ERR_INVALID_ARG, "case %d: mesh, C or V is NULL", i);
    ncell[i] = cases[i].mesh->d.n_cells;
    alp_mesh *m0 = nullptr;
    if ((rc = alp_bin_cells(ctx, ncell[i], C[i], V[i], boxes ? boxes[i] : nullptr, 0.0, 4, &m0)) != ALP_OK)
      return rc;
    base[i] = m0->d.bin;
    alp_mesh_destroy(m0);
  }
  const double scales[] = {0.75, 1.0, 1.5};
  const int32_t tiles[] = {2, 3, 4, 5};
  std::vector<alp_case> cs(cases, cases + n_cases);
  std::vector<alp_mesh *> best_m, cur((size_t)n_cases, nullptr);
  double best_ms = INFINITY, best_sc = 1.0;
  int32_t best_t = 4;
  auto drop = [](std::vector<alp_mesh *> &v) {
    for (alp_mesh *m : v)
      if (m) alp_mesh_destroy(m);
    v.clear();
  };
  for (int32_t T : tiles) {
    for (double sc : scales) {
      rc = ALP_OK;
      cur.assign((size_t)n_cases, nullptr);
      for (int i = 0; i < n_cases && rc == ALP_OK; ++i) {
        rc = alp_bin_cells(ctx, ncell[i], C[i], V[i], boxes ? boxes[i] : nullptr, base[i] * sc, T, &cur[i]);
        cs[i].mesh = cur[i];
      }
      double ms = INFINITY;
      if (rc == ALP_OK) {
        (void)alp_invalidate(ctx);
        rc = alp_step_batched(ctx, n_cases, cs.data(), flags | ALP_CHECKED);
        if (rc == ALP_OK) rc = alp_step_batched(ctx, n_cases, cs.data(), flags);
        if (rc == ALP_OK && hipStreamSynchronize(ctx->user) != hipSuccess) rc = ALP_ERR_HIP;
        if (rc == ALP_OK) {
          const auto t0 = std::chrono::steady_clock::now();
          for (int r = 0; r < reps && rc == ALP_OK; ++r) rc = alp_step_batched(ctx, n_cases, cs.data(), flags);
          if (rc == ALP_OK && hipStreamSynchronize(ctx->user) != hipSuccess) rc = ALP_ERR_HIP;
          ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count() / reps;
        }
        (void)alp_invalidate(ctx);
      }
      if (rc == ALP_OK && ms < best_ms) {
        drop(best_m);
        best_m = cur;
        best_ms = ms;
        best_sc = sc;
        best_t = T;
      } else {
        drop(cur);
      }
      if (rc == ALP_ERR_CAPACITY) continue;  // a per-tile limit: skip this candidate
      if (rc != ALP_OK) {
        drop(best_m);
        return rc;
      }
    }
  }
  if (!(best_ms < INFINITY)) return fail(ctx, ALP_ERR_INVALID_ARG, "no binning setting could be built");
  for (int i = 0; i < n_cases; ++i) cases[i].mesh = best_m[i];
  *out_scale = best_sc;
  *out_tile_bins = best_t;
  if (out_ms) *out_ms = best_ms;
  return ALP_OK;
}

const char *alp_stage_name(int32_t i) { return (i >= 0 && i < kNumStages) ? kStageNames[i] : ""; }

alp_status alp_step_profile(alp_context *ctx, int32_t n_cases, const alp_case *cases,
                            double *stage_ms, int32_t max_stages, int32_t *n_stages) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  if (!stage_ms || !n_stages || max_stages < 1)
    return fail(ctx, ALP_ERR_INVALID_ARG, "stage_ms, n_stages and max_stages >= 1 are required");
  // validate, size and warm the work lists exactly like an uncaptured batched step
  alp_status rc = alp_step_batched(ctx, n_cases, cases, 0);
  if (rc != ALP_OK) return rc;
  hipEvent_t ev[kNumStages + 1];
  for (int i = 0; i <= kNumStages; ++i) HIPCHK(ctx, hipEventCreate(&ev[i]));
  StepLaunch L = make_launch(ctx, n_cases);
  if ((rc = enter(ctx)) != ALP_OK) return rc;
  launch_sequence(ctx, L, ST_ALL, ev);
  HIPCHK(ctx, hipGetLastError());
  HIPCHK(ctx, hipEventSynchronize(ev[kNumStages]));
  int n = std::min<int>(max_stages, kNumStages);
  for (int i = 0; i < n; ++i) {
    float ms = 0.f;
    HIPCHK(ctx, hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
    stage_ms[i] = ms;
  }
  for (int i = 0; i <= kNumStages; ++i) (void)hipEventDestroy(ev[i]);
  *n_stages = n;
  return leave(ctx);
}

alp_status alp_get_diag(alp_context *ctx, int32_t case_index, alp_diag *out) {
  if (!ctx || !out) return fail(ctx, ALP_ERR_INVALID_ARG, "NULL argument");
  if (case_index < 0 || case_index >= ctx->last_cases || (!ctx->w.cnt && !ctx->dg_cnt))
    return fail(ctx, ALP_ERR_INVALID_ARG, "no diagnostics for case %d", case_index);
  alp_status rc = enter(ctx);  // after a replay on the caller's stream
  if (rc != ALP_OK) return rc;
  long long cnt[kCnt];
  double d[16];
  uint32_t counters[16];
  const long long *src_cnt = ctx->dg_cnt ? ctx->dg_cnt : ctx->w.cnt;
  const double *src_out = ctx->dg_out ? ctx->dg_out : ctx->w.diag_out;
  const uint32_t *src_ctr = ctx->dg_counters ? ctx->dg_counters : ctx->w.counters;
  HIPCHK(ctx, hipMemcpyAsync(cnt, src_cnt + kCnt * case_index, sizeof(cnt), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(d, src_out + 16 * case_index, sizeof(d), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipMemcpyAsync(counters, src_ctr, sizeof(counters), hipMemcpyDeviceToHost, ctx->st));
  HIPCHK(ctx, hipStreamSynchronize(ctx->st));
  std::memset(out, 0, sizeof(*out));
  out->n_outside = cnt[0];
  out->n_fallback = cnt[1];
  out->n_fallback_degenerate = cnt[2];
  out->n_zero_weight = cnt[3];
  out->n_band_cells = cnt[4];
  out->n_pairs = cnt[5];
  out->n_invalid = cnt[6];
  out->n_overflow = counters[3];
  for (int a = 0; a < 3; ++a) {
    out->F_beam[a] = d[a];
    out->F_fluid[a] = d[4 + a];
  }
  out->cons_rel_err = d[7];
  out->n_sample_empty = cnt[7];
  out->n_guard_fp64 = cnt[8];
  return ALP_OK;
}

alp_status alp_invalidate(alp_context *ctx) {
  if (!ctx) return ALP_ERR_INVALID_ARG;
  (void)settle(ctx);
  drop_graph(ctx);
  ctx->tkey.clear();  // the next ALP_AUTOTUNE call chooses again (the shape stays until then)
  return ALP_OK;
}

alp_status alp_get_tuning(alp_context *ctx, alp_tuning *out) {
  if (!ctx || !out) return fail(ctx, ALP_ERR_INVALID_ARG, "NULL argument");
  *out = ctx->tun;
  return ALP_OK;
}

alp_status alp_set_tuning(alp_context *ctx, const alp_tuning *t) {
  if (!ctx || !t) return fail(ctx, ALP_ERR_INVALID_ARG, "NULL argument");
  if (!tuning_valid(*t))
    return fail(ctx, ALP_ERR_INVALID_ARG, "tuning out of range (lanes 2/4/8, waves 0..32, grab 1..16)");
  (void)settle(ctx);
  drop_graph(ctx);
  ctx->tun = *t;
  ctx->tkey.clear();
  return ALP_OK;
}

}  // extern "C"
