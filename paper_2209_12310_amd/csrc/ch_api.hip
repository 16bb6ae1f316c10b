// Host side of the C ABI declared in include/convhull.h: argument checks,
// workspace layout, kernel sequencing, result staging and profiling.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/convhull.h"
#include "ch_internal.hpp"

namespace chk {
hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t st);
uint32_t reduce_blocks(uint32_t n, uint32_t max_blocks);
uint32_t filter_blocks(uint32_t n, uint32_t max_blocks);
hipError_t launch_reduce8(const float* xy, uint32_t n, uint32_t head, double* partials,
                          uint32_t* part_bad, uint32_t blocks, hipStream_t st);
hipError_t launch_oct_build(const double* partials, const uint32_t* part_bad, uint32_t nparts,
                            Header* hdr, Result* res, uint64_t* tstat, uint32_t ntstat,
                            hipStream_t st);
hipError_t launch_sample_poly(const float* xy, uint32_t n, void* scratch, SamplePoly* poly,
                              uint32_t* count0, RefineState* rs, hipStream_t st);
hipError_t launch_refine(const Rec* in, const uint32_t* count_in, uint32_t max_in,
                         const SamplePoly* poly, const Octagon* oct, RefineState* rs, Rec* out,
                         uint32_t max_blocks, hipStream_t st, LaunchHook* hk);
hipError_t launch_pass_hull(const float* xy, uint32_t n, uint32_t head, double* partials,
                            uint32_t* part_bad, const SamplePoly* poly, Rec* cand, void* scratch,
                            uint32_t blocks, uint32_t narrow_blocks, hipStream_t st);
hipError_t launch_filter(const float* xy, uint32_t n, uint32_t head, Header* hdr, uint64_t* tstat,
                         uint32_t blocks, uint32_t* surv, uint32_t* count_out, uint8_t* labels,
                         uint32_t* staging, hipStream_t st);
hipError_t launch_oct_out(const Header* hdr, void* d_oct, hipStream_t st);
hipError_t launch_filter_rec(const float* xy, uint32_t n, uint32_t head, Header* hdr,
                             uint32_t blocks, Rec* surv, uint32_t* count_out,
                             const SamplePoly* gate, const Rec* cand, const void* scratch,
                             uint32_t* ncand_out, uint32_t* mode_out, const double* partials,
                             const uint32_t* part_bad, uint32_t nparts, Result* res,
                             hipStream_t st);
hipError_t launch_hull_final(const Rec* in_rec, const uint32_t* in_count, Result* res,
                             uint32_t* res_idx, const Octagon* oct, Result* host,
                             uint32_t* host_idx, uint32_t host_n, hipStream_t st);
hipError_t launch_hull_round(uint32_t grid, const Rec* in_rec, const uint32_t* in_count,
                             Rec* out_rec, uint32_t* out_count, uint32_t* tile_ctr,
                             hipStream_t st);
hipError_t launch_large_path(const Rec* in, const uint32_t* in_count, uint32_t max_in, Rec* part,
                             uint32_t* phist, uint32_t* ptot, Rec* lstA, Rec* lstB,
                             uint32_t* wcnt, const Octagon* oct, Result* res, uint32_t* res_idx,
                             Result* host, uint32_t* host_idx, uint32_t host_n, hipStream_t st,
                             LaunchHook* hk);
hipError_t launch_read_stream(const void* d_buf, size_t bytes, uint32_t blocks, float* sink,
                              hipStream_t st);
hipError_t launch_batch_filter_side(const float* xy, const uint64_t* off, uint32_t nsets,
                                    uint64_t total_points, uint32_t tile, BatchHdr* bh,
                                    SetState* sets, SamplePoly* polys, SetTile* tiles, Rec* recs,
                                    Rec* cand, uint32_t grid, uint32_t sample_min,
                                    uint32_t sample_grid, uint32_t* slist, uint32_t* luts,
                                    hipStream_t st, LaunchHook* hk);
hipError_t launch_batch_hull_side(const uint64_t* off, uint32_t nsets, uint64_t total_points,
                                  BatchHdr* bh, SetState* sets, SetTile* rtiles, Rec* recA, Rec* recB,
                                  uint32_t* hull_idx, uint32_t* hull_count, uint32_t grid,
                                  uint32_t* order, hipStream_t st, LaunchHook* hk);
hipError_t launch_axis_extremes(const float* xy, uint32_t n, uint32_t head, double* partials,
                                uint32_t* part_bad, uint32_t blocks, Header* hdr, hipStream_t st);
hipError_t launch_corner_extremes(const float* xy, uint32_t n, uint32_t head, double* partials,
                                  uint32_t blocks, const Header* hdr, hipStream_t st);
hipError_t launch_list_chains(int NL, Rec* A, Rec* B, size_t cap, const uint32_t* begin,
                              const uint32_t* len, uint32_t lower_mask, uint32_t* wcnt,
                              uint32_t* pack, uint32_t* fold, hipStream_t st, LaunchHook* hk);
hipError_t launch_queue_split(const uint8_t* labels, uint32_t n, const Header* hdr, uint32_t* qblk,
                              QState* qs, uint32_t* qidx, hipStream_t st);
hipError_t launch_queue_order(const float* xy, uint32_t n, const uint32_t* qidx, const QState* qs,
                              const Header* hdr, uint64_t* bot, uint64_t* top, hipStream_t st);
hipError_t launch_queue_lists(const uint64_t* bot, const uint64_t* top, uint32_t* colcnt,
                              Rec* lists, size_t cap, const Header* hdr, QState* qs,
                              hipStream_t st);
hipError_t launch_queue_union(const Rec* lists, size_t cap, const QState* qs, const Header* hdr,
                              Result* res, uint32_t* res_idx, uint32_t res_cap, Result* host,
                              uint32_t* host_idx, uint32_t host_n, hipStream_t st);
}  // namespace chk

using namespace chk;

namespace {

constexpr uint32_t kPinIdx = 16384;  // hull indices the device writes to pinned host memory

// Library-owned scratch of ch_filter_noalloc: the ch_filter workspace for
// CH_FILTER_NOALLOC_MAX_POINTS points, one copy per device, loaded with the
// code object and held until the process ends. Host code never uses this
// name as an address: ch_ctx_create looks up the device address with the
// context's device current and keeps it in the context.
constexpr size_t kNoAllocBytes = layout(CH_FILTER_NOALLOC_MAX_POINTS).filter_end;
__device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct KStat {
  const char* name;
  uint64_t launches;
  double ms;
};

}  // namespace

struct ch_ctx {
  int device = 0;
  int cu_count = 0;
  uint32_t reduce_max_blocks = 1024;  // persistent grid sizes, from the CU count
  uint32_t filter_max_blocks = 1024;
  uint32_t fused_max_blocks = 512;
  uint32_t narrow_blocks = 256;
  uint32_t large_direct = kLargeDirect;  // survivors from which ch_hull skips the tile rounds
  bool poll = true;  // watch the published status instead of waiting for the stream
  bool second_poly = true;  // ch_hull: the second polygon when one workgroup cannot take the survivors
  unsigned char* pinned = nullptr;  // kResBytes + 4 * kPinIdx
  unsigned char* pinned_dev = nullptr;  // its device address (null: copied, not written directly)
  void* noalloc_ws = nullptr;           // device address of `scratch` on this context's device
  std::string err;
  ch_hull_info last{};  // counts of the last successful ch_hull
  // Batch-mode parameters: fixed ones (ch_batch_params_set), else the tuned
  // entry nearest to the call's shape, else the defaults.
  ch_batch_params batch{};
  bool batch_fixed = false;
  struct TuneEntry { int lg_sets, lg_points; ch_batch_params p; };
  std::vector<TuneEntry> tuned;
  std::string arch;
  std::string tune_path;
  bool prof = false;
  std::vector<KStat> stats;
  struct Pending { int stat; hipEvent_t a, b; };
  std::vector<Pending> pending;
  std::vector<hipEvent_t> pool;
};

namespace chk {
int ctx_device(const ch_ctx* ctx) { return ctx->device; }
}  // namespace chk

namespace {

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

ch_status fail(ch_ctx* ctx, ch_status s, const char* fmt, ...) __attribute__((format(printf, 3, 4)));
ch_status fail(ch_ctx* ctx, ch_status s, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return s;
}

ch_status hip_fail(ch_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, CH_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

int stat_index(ch_ctx* ctx, const char* name) {
  for (size_t i = 0; i < ctx->stats.size(); ++i)
    if (std::strcmp(ctx->stats[i].name, name) == 0) return (int)i;
  ctx->stats.push_back({name, 0, 0.0});
  return (int)ctx->stats.size() - 1;
}

hipEvent_t take_event(ch_ctx* ctx) {
  if (!ctx->pool.empty()) {
    hipEvent_t e = ctx->pool.back();
    ctx->pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets one kernel launch with events when profiling is on.
struct ProfScope {
  ch_ctx* ctx;
  hipStream_t st;
  int stat = -1;
  hipEvent_t a = nullptr, b = nullptr;
  ProfScope(ch_ctx* c, hipStream_t s, const char* name) : ctx(c), st(s) {
    if (!ctx->prof) return;
    stat = stat_index(ctx, name);
    a = take_event(ctx);
    b = take_event(ctx);
    if (a) (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!ctx->prof || !a || !b) return;
    (void)hipEventRecord(b, st);
    ctx->pending.push_back({stat, a, b});
  }
};

// The same events per kernel of a multi-kernel launcher.
struct ProfHook final : LaunchHook {
  ch_ctx* ctx;
  hipStream_t st;
  int stat = -1;
  hipEvent_t a = nullptr, b = nullptr;
  ProfHook(ch_ctx* c, hipStream_t s) : ctx(c), st(s) {}
  void begin(const char* name) override {
    stat = stat_index(ctx, name);
    a = take_event(ctx);
    b = take_event(ctx);
    if (a) (void)hipEventRecord(a, st);
  }
  void end() override {
    if (!a || !b) return;
    (void)hipEventRecord(b, st);
    ctx->pending.push_back({stat, a, b});
    a = b = nullptr;
  }
};

void prof_collect(ch_ctx* ctx, hipStream_t st) {
  if (!ctx->prof || ctx->pending.empty()) return;
  (void)hipStreamSynchronize(st);
  for (auto& p : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      ctx->stats[p.stat].launches += 1;
      ctx->stats[p.stat].ms += ms;
    }
    ctx->pool.push_back(p.a);
    ctx->pool.push_back(p.b);
  }
  ctx->pending.clear();
}

template <class T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<unsigned char*>(ws) + off);
}

// Enqueues the filtering stage. ch_filter (surv_rec null): pass 1 (extreme
// reduction, octagon build) and the ordered pass 2. Hull path (records into
// surv_rec): below kSampleMin points, pass 1 and the unordered pass 2; from
// kSampleMin on, the sample polygon first, then one fused read (pass 1 plus
// the polygon test) and the octagon test on the candidates, whose
// workgroups build the octagon from the pass's partials themselves (or,
// without a usable polygon, the unordered pass 2 with that octagon).
ch_status run_filter(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* surv,
                     uint32_t* count_out, uint8_t* labels, void* ws, const Layout& L,
                     hipStream_t st, Rec* surv_rec = nullptr, Rec* cand = nullptr) {
  const bool fused = surv_rec && n >= kSampleMin;
  SamplePoly* poly = fused ? at<SamplePoly>(ws, L.poly) : nullptr;
  void* scratch = fused ? at<void>(ws, L.samp) : nullptr;
  const uint32_t head = (reinterpret_cast<uintptr_t>(d_xy) & 15u) ? 1u : 0u;
  Header* hdr = at<Header>(ws, L.hdr);
  Result* res = at<Result>(ws, L.res);
  const uint32_t g1 = reduce_blocks(n, fused ? ctx->fused_max_blocks : ctx->reduce_max_blocks);
  const uint32_t g2 = filter_blocks(n, ctx->filter_max_blocks);
  double* partials = at<double>(ws, L.partials);
  uint32_t* part_bad = at<uint32_t>(ws, L.part_bad);
  hipError_t e;
  if (fused) {
    {
      ProfScope p(ctx, st, "sample_poly");
      e = launch_sample_poly(d_xy, n, scratch, poly, count_out, at<RefineState>(ws, L.refine), st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "sample polygon launch");
    {
      ProfScope p(ctx, st, "pass_fused");
      e = launch_pass_hull(d_xy, n, head, partials, part_bad, poly, cand, scratch, g1,
                           ctx->narrow_blocks, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "fused pass launch");
  } else {
    ProfScope p(ctx, st, "reduce8");
    e = launch_reduce8(d_xy, n, head, partials, part_bad, g1, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "reduce8 launch");
  }
  if (!fused) {  // after a fused pass the candidate test builds the octagon itself
    ProfScope p(ctx, st, "oct_build");
    e = launch_oct_build(partials, part_bad, g1, hdr, res, at<uint64_t>(ws, L.tstat), g2, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "oct_build launch");
  }
  {
    ProfScope p(ctx, st, fused ? "cand_filter" : "filter_compact");
    if (surv_rec)
      e = launch_filter_rec(d_xy, n, head, hdr, g1, surv_rec, count_out, poly, cand, scratch,
                            &res->ncand, &res->mode, fused ? partials : nullptr, part_bad, g1,
                            res, st);
    else
      e = launch_filter(d_xy, n, head, hdr, at<uint64_t>(ws, L.tstat), g2, surv, count_out, labels,
                        at<uint32_t>(ws, L.staging), st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "filter launch");
  return CH_OK;
}

// Alg. 2 with the chosen extreme search: the octagon in the header, the
// ordered survivor indices, their count and (labels non-null) the label of
// every point. CH_EXTREMES_FUSED is ch_filter's path; the two-kernel search
// (Sec. III) replaces pass 1 by its two reductions on the same grid.
ch_status run_gpufilter(ch_ctx* ctx, const float* d_xy, uint32_t n, int mode, uint32_t* surv,
                        uint32_t* count_out, uint8_t* labels, void* ws, const Layout& L,
                        hipStream_t st) {
  if (mode == CH_EXTREMES_FUSED) return run_filter(ctx, d_xy, n, surv, count_out, labels, ws, L, st);
  const uint32_t head = (reinterpret_cast<uintptr_t>(d_xy) & 15u) ? 1u : 0u;
  Header* hdr = at<Header>(ws, L.hdr);
  Result* res = at<Result>(ws, L.res);
  const uint32_t g1 = reduce_blocks(n, ctx->reduce_max_blocks);
  const uint32_t g2 = filter_blocks(n, ctx->filter_max_blocks);
  double* partials = at<double>(ws, L.partials);
  uint32_t* part_bad = at<uint32_t>(ws, L.part_bad);
  hipError_t e;
  {
    ProfScope p(ctx, st, "axis_extremes");
    e = launch_axis_extremes(d_xy, n, head, partials, part_bad, g1, hdr, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "axis extremes launch");
  {
    ProfScope p(ctx, st, "corner_extremes");
    e = launch_corner_extremes(d_xy, n, head, partials, g1, hdr, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "corner extremes launch");
  {
    ProfScope p(ctx, st, "oct_build");
    e = launch_oct_build(partials, part_bad, g1, hdr, res, at<uint64_t>(ws, L.tstat), g2, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "oct_build launch");
  {
    ProfScope p(ctx, st, "filter_compact");
    e = launch_filter(d_xy, n, head, hdr, at<uint64_t>(ws, L.tstat), g2, surv, count_out, labels,
                      at<uint32_t>(ws, L.staging), st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "filter launch");
  return CH_OK;
}

ch_status check_points(ch_ctx* ctx, const float* d_xy, uint32_t n) {
  if (n > CH_MAX_POINTS) return fail(ctx, CH_E_INVALID_ARG, "n = %u exceeds CH_MAX_POINTS", n);
  if (n && !d_xy) return fail(ctx, CH_E_INVALID_ARG, "d_xy is NULL");
  if (reinterpret_cast<uintptr_t>(d_xy) & 7u)
    return fail(ctx, CH_E_INVALID_ARG, "d_xy must be 8-byte aligned");
  return CH_OK;
}

ch_batch_params default_batch_params(int cu) {
  ch_batch_params p;
  p.tile_points = kBatchTile;
  p.pass_blocks = (uint32_t)cu * 8;
  p.hull_blocks = (uint32_t)cu * 9;  // three tile-hull workgroups per CU, three waves of them
  p.sample_min = kBatchSampleMin;
  return p;
}

bool valid_batch_params(const ch_batch_params& p) {
  const uint32_t t = p.tile_points;
  return t >= kBatchTileMin && t <= kBatchTileMax && (t & (t - 1)) == 0 && p.pass_blocks >= 1 &&
         p.pass_blocks <= 65535 && p.hull_blocks >= 1 && p.hull_blocks <= 65535;
}

int lg_bucket(uint64_t v) { return v ? 63 - __builtin_clzll(v) : -1; }

// Tune cache: text lines "convhull-tune 1 <arch> <cu> <lg_sets> <lg_points>
// <tile> <pass> <hull> <sample_min>"; lines for other devices are kept.
void load_tune_cache(ch_ctx* ctx) {
  std::ifstream f(ctx->tune_path);
  std::string line;
  while (std::getline(f, line)) {
    std::istringstream in(line);
    std::string tag, arch;
    int ver = 0, cu = 0;
    ch_ctx::TuneEntry e{};
    if (!(in >> tag >> ver >> arch >> cu >> e.lg_sets >> e.lg_points >> e.p.tile_points >>
          e.p.pass_blocks >> e.p.hull_blocks >> e.p.sample_min))
      continue;
    if (tag != "convhull-tune" || ver != 1 || arch != ctx->arch || cu != ctx->cu_count) continue;
    if (!valid_batch_params(e.p)) continue;
    ctx->tuned.push_back(e);
  }
}

bool save_tune_cache(const ch_ctx* ctx) {
  std::vector<std::string> keep;
  {
    std::ifstream f(ctx->tune_path);
    std::string line;
    while (std::getline(f, line)) {
      std::istringstream in(line);
      std::string tag, arch;
      int ver = 0, cu = 0;
      if ((in >> tag >> ver >> arch >> cu) && tag == "convhull-tune" && arch == ctx->arch &&
          cu == ctx->cu_count)
        continue;  // rewritten below
      if (!line.empty()) keep.push_back(line);
    }
  }
  const std::string tmp = ctx->tune_path + ".tmp";
  {
    std::ofstream o(tmp, std::ios::trunc);
    if (!o) return false;
    for (const auto& l : keep) o << l << "\n";
    for (const auto& e : ctx->tuned)
      o << "convhull-tune 1 " << ctx->arch << ' ' << ctx->cu_count << ' ' << e.lg_sets << ' '
        << e.lg_points << ' ' << e.p.tile_points << ' ' << e.p.pass_blocks << ' ' << e.p.hull_blocks
        << ' ' << e.p.sample_min << "\n";
    if (!o) return false;
  }
  return std::rename(tmp.c_str(), ctx->tune_path.c_str()) == 0;
}

ch_batch_params batch_params_for(const ch_ctx* ctx, uint32_t nsets, uint64_t total) {
  if (ctx->batch_fixed || ctx->tuned.empty()) return ctx->batch;
  const int ls = lg_bucket(nsets), lp = lg_bucket(total);
  const ch_ctx::TuneEntry* best = nullptr;
  int bd = 1 << 30;
  for (const auto& e : ctx->tuned) {
    const int d = std::abs(e.lg_sets - ls) + std::abs(e.lg_points - lp);
    if (d < bd) { bd = d; best = &e; }
  }
  return best->p;
}

ch_status check_batch(ch_ctx* ctx, const float* d_xy, const uint64_t* d_off, uint32_t nsets,
                      uint64_t total_points, const uint32_t* d_hull_idx,
                      const uint32_t* d_hull_count, void* d_ws, size_t ws_bytes) {
  if (!d_off || !d_hull_count) return fail(ctx, CH_E_INVALID_ARG, "d_off / d_hull_count is NULL");
  if (total_points >= 0xFFFFFFFFull)
    return fail(ctx, CH_E_INVALID_ARG, "total_points must stay below 2^32");
  if (total_points && (!d_xy || !d_hull_idx))
    return fail(ctx, CH_E_INVALID_ARG, "d_xy / d_hull_idx is NULL");
  if (reinterpret_cast<uintptr_t>(d_xy) & 15u)
    return fail(ctx, CH_E_INVALID_ARG, "d_xy must be 16-byte aligned in batch mode");
  const size_t need = batch_layout(nsets, total_points).total;
  if (!d_ws || ws_bytes < need)
    return fail(ctx, CH_E_INVALID_ARG, "workspace needs %zu bytes, got %zu", need, ws_bytes);
  if (reinterpret_cast<uintptr_t>(d_ws) & 255u)
    return fail(ctx, CH_E_INVALID_ARG, "workspace must be 256-byte aligned");
  return CH_OK;
}

// Enqueues one batch with parameters p (arguments already checked).
ch_status run_batch(ch_ctx* ctx, const ch_batch_params& p, const float* d_xy,
                    const uint64_t* d_off, uint32_t nsets, uint64_t total_points,
                    uint32_t* d_hull_idx, uint32_t* d_hull_count, void* d_ws, hipStream_t st) {
  const BatchLayout L = batch_layout(nsets, total_points);
  BatchHdr* bh = at<BatchHdr>(d_ws, L.hdr);
  SetState* sets = at<SetState>(d_ws, L.sets);
  Rec* recA = at<Rec>(d_ws, L.recA);
  Rec* recB = at<Rec>(d_ws, L.recB);
  ProfHook hook(ctx, st);
  LaunchHook* hk = ctx->prof ? &hook : nullptr;
  hipError_t e = launch_batch_filter_side(d_xy, d_off, nsets, total_points, p.tile_points, bh, sets,
                                          at<SamplePoly>(d_ws, L.polys), at<SetTile>(d_ws, L.tiles),
                                          recA, recB, p.pass_blocks, p.sample_min,
                                          (uint32_t)ctx->cu_count * 4, at<uint32_t>(d_ws, L.slist),
                                          at<uint32_t>(d_ws, L.luts), st, hk);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch filter launch");
  e = launch_batch_hull_side(d_off, nsets, total_points, bh, sets, at<SetTile>(d_ws, L.rtiles), recA, recB,
                             d_hull_idx, d_hull_count, p.hull_blocks, at<uint32_t>(d_ws, L.slist), st,
                             hk);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch hull launch");
  return CH_OK;
}

}  // namespace

extern "C" {

const char* ch_status_string(ch_status s) {
  switch (s) {
    case CH_OK: return "ok";
    case CH_E_INVALID_ARG: return "invalid argument";
    case CH_E_DOMAIN: return "coordinate outside the 2^-20 grid on [0,1)";
    case CH_E_CAPACITY: return "output capacity too small";
    case CH_E_NOMEM: return "out of memory";
    case CH_E_DEVICE: return "HIP runtime error";
    case CH_E_BUSY: return "busy";
    case CH_E_TIMEOUT: return "timed out";
    case CH_E_CANCELLED: return "cancelled";
    case CH_E_SHUTDOWN: return "shut down";
    case CH_E_NOT_FOUND: return "not found";
  }
  return "unknown status";
}

ch_status ch_ctx_create(int hip_device, const char* tune_cache_path, ch_ctx** out) {
  if (!out) return CH_E_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev)
    return CH_E_DEVICE;
  DeviceGuard g(hip_device);
  if (!g.ok) return CH_E_DEVICE;
  ch_ctx* ctx = new (std::nothrow) ch_ctx();
  if (!ctx) return CH_E_NOMEM;
  ctx->device = hip_device;
  if (hipDeviceGetAttribute(&ctx->cu_count, hipDeviceAttributeMultiprocessorCount, hip_device) !=
      hipSuccess)
    ctx->cu_count = 256;
  ctx->reduce_max_blocks = (uint32_t)ctx->cu_count * 4;
  if (ctx->reduce_max_blocks > (uint32_t)kReduceMaxBlocks) ctx->reduce_max_blocks = kReduceMaxBlocks;
  ctx->filter_max_blocks = (uint32_t)ctx->cu_count * 4;
  if (ctx->filter_max_blocks > (uint32_t)kFilterMaxBlocks) ctx->filter_max_blocks = kFilterMaxBlocks;
  // The fused hull pass: two workgroups per CU when many points go to the
  // exact test, one per CU (fewer, longer streams) when few do.
  ctx->fused_max_blocks = (uint32_t)ctx->cu_count * 2;
  if (ctx->fused_max_blocks > (uint32_t)kReduceMaxBlocks) ctx->fused_max_blocks = kReduceMaxBlocks;
  ctx->narrow_blocks = (uint32_t)ctx->cu_count;
  // Overrides for tuning sweeps.
  if (const char* e = std::getenv("CH_REDUCE_BLOCKS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= kReduceMaxBlocks) ctx->reduce_max_blocks = (uint32_t)v;
  }
  if (const char* e = std::getenv("CH_FILTER_BLOCKS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= kFilterMaxBlocks) ctx->filter_max_blocks = (uint32_t)v;
  }
  if (const char* e = std::getenv("CH_FUSED_BLOCKS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= kReduceMaxBlocks) ctx->fused_max_blocks = (uint32_t)v;
  }
  if (const char* e = std::getenv("CH_NARROW_BLOCKS")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= 1 && v <= kReduceMaxBlocks) ctx->narrow_blocks = (uint32_t)v;
  }
  if (const char* e = std::getenv("CH_HULL_WAIT")) ctx->poll = std::strcmp(e, "stream") != 0;
  if (const char* e = std::getenv("CH_SECOND_POLY")) ctx->second_poly = std::strcmp(e, "0") != 0;
  if (const char* e = std::getenv("CH_LARGE_DIRECT")) {
    const long v = std::strtol(e, nullptr, 10);
    if (v >= kFinalTile && v <= (long)CH_MAX_POINTS) ctx->large_direct = (uint32_t)v;
  }
  if (hipHostMalloc(reinterpret_cast<void**>(&ctx->pinned), kResBytes + 4 * kPinIdx,
                    hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
    delete ctx;
    return CH_E_NOMEM;
  }
  {
    // The block hull writes the result block straight into this buffer.
    void* dp = nullptr;
    if (hipHostGetDevicePointer(&dp, ctx->pinned, 0) == hipSuccess) ctx->pinned_dev = static_cast<unsigned char*>(dp);
    else (void)hipGetLastError();
  }
  {
    // The no-allocation filter's scratch on this device (device current).
    void* sp = nullptr;
    if (hipGetSymbolAddress(&sp, HIP_SYMBOL(scratch)) != hipSuccess || !sp) {
      (void)hipGetLastError();
      (void)hipHostFree(ctx->pinned);
      delete ctx;
      return CH_E_DEVICE;
    }
    ctx->noalloc_ws = sp;
  }
  ctx->batch = default_batch_params(ctx->cu_count);
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) == hipSuccess) ctx->arch = prop.gcnArchName;
    const size_t colon = ctx->arch.find(':');
    if (colon != std::string::npos) ctx->arch.resize(colon);
    if (ctx->arch.empty()) ctx->arch = "unknown";
  }
  if (tune_cache_path && *tune_cache_path) {
    ctx->tune_path = tune_cache_path;
    load_tune_cache(ctx);
  }
  *out = ctx;
  return CH_OK;
}

void ch_ctx_destroy(ch_ctx* ctx) {
  if (!ctx) return;
  DeviceGuard g(ctx->device);
  for (auto& p : ctx->pending) {
    (void)hipEventDestroy(p.a);
    (void)hipEventDestroy(p.b);
  }
  for (auto e : ctx->pool) (void)hipEventDestroy(e);
  if (ctx->pinned) (void)hipHostFree(ctx->pinned);
  delete ctx;
}

const char* ch_last_error(const ch_ctx* ctx) { return ctx ? ctx->err.c_str() : "no context"; }

size_t ch_filter_workspace_bytes(uint32_t n) { return layout(n).filter_end; }
size_t ch_hull_workspace_bytes(uint32_t n) { return layout(n).total; }

size_t ch_filter_noalloc_scratch_bytes(void) { return kNoAllocBytes; }

ch_status ch_filter(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* d_survivors,
                    uint32_t* d_count, uint8_t* d_label, ch_octagon* d_oct, void* d_ws,
                    size_t ws_bytes, void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (ch_status s = check_points(ctx, d_xy, n)) return s;
  if (!d_count) return fail(ctx, CH_E_INVALID_ARG, "d_count is NULL");
  if (n && !d_survivors) return fail(ctx, CH_E_INVALID_ARG, "d_survivors is NULL");
  const Layout L = layout(n);
  if (!d_ws || ws_bytes < L.filter_end)
    return fail(ctx, CH_E_INVALID_ARG, "workspace needs %zu bytes, got %zu", L.filter_end, ws_bytes);
  if (reinterpret_cast<uintptr_t>(d_ws) & 255u)
    return fail(ctx, CH_E_INVALID_ARG, "workspace must be 256-byte aligned");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (n == 0) {
    hipError_t e = launch_set_u32(d_count, 0u, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "set count");
    return CH_OK;
  }
  if (ch_status s = run_filter(ctx, d_xy, n, d_survivors, d_count, d_label, d_ws, L, st)) return s;
  if (d_oct) {
    ProfScope p(ctx, st, "oct_out");
    hipError_t e = launch_oct_out(at<Header>(d_ws, L.hdr), d_oct, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "oct_out launch");
  }
  prof_collect(ctx, st);
  return CH_OK;
}

ch_status ch_filter_noalloc(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* d_survivors,
                            uint32_t* d_count, uint8_t* d_label, ch_octagon* d_oct, void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (n > CH_FILTER_NOALLOC_MAX_POINTS)
    return fail(ctx, CH_E_INVALID_ARG,
                "ch_filter_noalloc takes at most %u points (its scratch is fixed), got %u",
                (unsigned)CH_FILTER_NOALLOC_MAX_POINTS, n);
  if (!ctx->noalloc_ws) return fail(ctx, CH_E_DEVICE, "no device scratch on this context");
  // Same kernels as ch_filter; every per-call counter in the scratch is reset
  // by the kernels of the call itself, so no clearing is needed here.
  return ch_filter(ctx, d_xy, n, d_survivors, d_count, d_label, d_oct, ctx->noalloc_ws,
                   kNoAllocBytes, stream);
}

ch_status ch_hull(ch_ctx* ctx, const float* d_xy, uint32_t n, uint32_t* h_hull_idx, uint32_t cap,
                  uint32_t* h_out, void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (ch_status s = check_points(ctx, d_xy, n)) return s;
  if (!h_out) return fail(ctx, CH_E_INVALID_ARG, "h_out is NULL");
  if (cap && !h_hull_idx) return fail(ctx, CH_E_INVALID_ARG, "h_hull_idx is NULL");
  const Layout L = layout(n);
  if (n && (!d_ws || ws_bytes < L.total))
    return fail(ctx, CH_E_INVALID_ARG, "workspace needs %zu bytes, got %zu", L.total, ws_bytes);
  if (reinterpret_cast<uintptr_t>(d_ws) & 255u)
    return fail(ctx, CH_E_INVALID_ARG, "workspace must be 256-byte aligned");
  if (n == 0) {
    *h_out = 0;
    return CH_OK;
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  Header* hdr = at<Header>(d_ws, L.hdr);
  Result* res = at<Result>(d_ws, L.res);
  uint32_t* res_idx = at<uint32_t>(d_ws, L.res_idx);
  Rec* srec = at<Rec>(d_ws, L.surv);
  Rec* rec[2] = {at<Rec>(d_ws, L.recA), at<Rec>(d_ws, L.recB)};
  // Candidates of the fused pass go to list B (first written again by the second tile-hull round).
  if (ch_status s = run_filter(ctx, d_xy, n, nullptr, &hdr->count, nullptr, d_ws, L, st, srec,
                               rec[1]))
    return s;

  const Result* hres = reinterpret_cast<const Result*>(ctx->pinned);
  const uint32_t* hidx = reinterpret_cast<const uint32_t*>(ctx->pinned + kResBytes);
  const uint32_t pin_n = hull_cap(n) < kPinIdx ? hull_cap(n) : kPinIdx;
  auto fetch = [&]() -> hipError_t {
    hipError_t e = hipMemcpyAsync(ctx->pinned, res, kResBytes + 4 * size_t(pin_n),
                                  hipMemcpyDeviceToHost, st);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(st);
  };
  // After the block hull: it wrote the result block to the pinned buffer
  // itself when that buffer is device-mapped.
  Result* dres_host = reinterpret_cast<Result*>(ctx->pinned_dev);
  uint32_t* didx_host = ctx->pinned_dev ? reinterpret_cast<uint32_t*>(ctx->pinned_dev + kResBytes) : nullptr;
  auto fetch_final = [&]() -> hipError_t {
    if (!ctx->pinned_dev) return fetch();
    return hipStreamSynchronize(st);
  };
  // The block hull publishes its result block with the status word last
  // (system-scope release): mark it pending before the launch, then watch
  // it instead of waiting for the stream (a stream wait adds its own wake-up
  // latency). A stream that ends with the status still pending is reported
  // by the status check that follows.
  Result* hres_w = reinterpret_cast<Result*>(ctx->pinned);
  auto arm_final = [&]() {
    if (ctx->pinned_dev) __atomic_store_n(&hres_w->status, (uint32_t)RES_PENDING, __ATOMIC_RELEASE);
  };
  auto wait_final = [&]() -> hipError_t {
    if (!ctx->pinned_dev || ctx->prof || !ctx->poll) return fetch_final();
    for (uint32_t spins = 1;; ++spins) {
      if (__atomic_load_n(&hres_w->status, __ATOMIC_ACQUIRE) != RES_PENDING) return hipSuccess;
      if ((spins & 1023u) == 0) {
        const hipError_t q = hipStreamQuery(st);
        if (q == hipSuccess) return hipSuccess;
        if (q != hipErrorNotReady) return q;
      }
      __builtin_ia32_pause();
    }
  };

  hipError_t e;
  arm_final();
  {
    ProfScope p(ctx, st, "hull_final");
    e = launch_hull_final(srec, &hdr->count, res, res_idx, &hdr->oct, dres_host, didx_host, pin_n, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "hull final launch");
  if ((e = wait_final()) != hipSuccess) return hip_fail(ctx, e, "hull final");
  prof_collect(ctx, st);
  if (hres->status == RES_DOMAIN) return fail(ctx, CH_E_DOMAIN, "input outside the 2^-20 grid");
  ch_hull_info info{};
  info.n = n;
  info.candidates = hres->ncand;
  info.single_read = hres->mode;
  info.survivors = hres->cin;
  bool large = false;
  int round = 0;
  int last_list = -1;  // record list holding the latest round's output (-1: the survivors)
  // The survivors: the octagon test's output, or the candidate records
  // themselves (list B) when the test was skipped.
  const Rec* surv0 = hres->cand_surv ? rec[1] : srec;
  const uint32_t* cnt0 = &hdr->count;
  // Too many survivors for one workgroup after the refined filter, but not
  // so many that the large-hull path (whose cost is mostly fixed) would
  // beat the extra steps: the second polygon from the survivors themselves
  // (k_refine_bins), the survivors strictly inside it dropped, and the block
  // hull again. The kept records go to whichever of the survivor and
  // candidate lists the survivors do not occupy (list A stays free for the
  // rounds).
  if (hres->status == RES_MORE && hres->cin <= kRefineMaxSingle && n >= kSampleMin &&
      ctx->second_poly) {
    RefineState* rs = at<RefineState>(d_ws, L.refine);
    Rec* kept = surv0 == srec ? rec[1] : srec;
    {
      ProfHook hook(ctx, st);
      e = launch_refine(surv0, cnt0, hres->cin, at<SamplePoly>(d_ws, L.poly), &hdr->oct, rs, kept,
                        (uint32_t)ctx->cu_count * 2, st, ctx->prof ? &hook : nullptr);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "second polygon launch");
    arm_final();
    {
      ProfScope p(ctx, st, "hull_final");
      e = launch_hull_final(kept, &rs->cnt, res, res_idx, &hdr->oct, dres_host, didx_host, pin_n, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hull final launch");
    if ((e = wait_final()) != hipSuccess) return hip_fail(ctx, e, "hull final");
    prof_collect(ctx, st);
    surv0 = kept;
    cnt0 = &rs->cnt;
    info.refined = hres->cin;
  }
  // Many survivors (points near a smooth boundary keep about half of every
  // tile hull): straight to the large-hull path.
  if (hres->status == RES_MORE && hres->cin > ctx->large_direct) large = true;
  while (!large && hres->status != RES_DONE) {
    if (hres->status != RES_MORE) return fail(ctx, CH_E_DEVICE, "hull status %u", hres->status);
    const uint32_t cin = hres->cin;
    uint32_t grid = (cin + kHullTile - 1) / kHullTile;
    const uint32_t gmax = (uint32_t)ctx->cu_count * 3;
    if (grid > gmax) grid = gmax;
    if (grid < 1) grid = 1;
    const uint32_t* in_count = round == 0 ? cnt0 : &res->round_cnt[round];
    {
      ProfScope p(ctx, st, round == 0 ? "hull_round0" : "hull_round");
      e = launch_hull_round(grid, round ? rec[(round - 1) & 1] : surv0, in_count, rec[round & 1],
                            &res->round_cnt[round + 1], &res->round_tile[round], st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hull round launch");
    arm_final();
    {
      ProfScope p(ctx, st, "hull_final");
      e = launch_hull_final(rec[round & 1], &res->round_cnt[round + 1], res, res_idx, &hdr->oct,
                            dres_host, didx_host, pin_n, st);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "hull final launch");
    if ((e = wait_final()) != hipSuccess) return hip_fail(ctx, e, "hull round");
    prof_collect(ctx, st);
    last_list = round & 1;
    ++round;
    if (hres->status == RES_DONE) break;
    // A round that keeps more than half of its input hands over to the
    // large-hull path.
    const uint32_t cout = hres->cin;
    if (uint64_t(cout) * 2 > cin || round + 1 >= kMaxRounds) {
      large = true;
      break;
    }
  }

  if (large) {
    // input: the last round's output, or the survivors when no round ran
    const uint32_t cin = round ? hres->round_cnt[round] : hres->cin;
    const Rec* lin = round ? rec[last_list] : surv0;
    const uint32_t* lcnt = round ? &res->round_cnt[round] : cnt0;
    {
      // Per-kernel events of the large-hull path when profiling is on.
      ProfHook hook(ctx, st);
      // The partition goes to a record list the input does not occupy.
      Rec* part = lin == srec ? rec[0] : (lin == rec[0] ? srec : rec[0]);
      e = launch_large_path(lin, lcnt, cin, part, at<uint32_t>(d_ws, L.phist),
                            at<uint32_t>(d_ws, L.ptot), at<Rec>(d_ws, L.lstA),
                            at<Rec>(d_ws, L.lstB), at<uint32_t>(d_ws, L.wcnt), &hdr->oct, res,
                            res_idx, dres_host, didx_host, pin_n, st, ctx->prof ? &hook : nullptr);
    }
    if (e != hipSuccess) return hip_fail(ctx, e, "large path launch");
    if ((e = fetch_final()) != hipSuccess) return hip_fail(ctx, e, "large path");
    prof_collect(ctx, st);
    if (hres->status != RES_DONE) return fail(ctx, CH_E_DEVICE, "large hull status %u", hres->status);
  }

  const uint32_t h = hres->h;
  *h_out = h;
  info.rounds = (uint32_t)round;
  info.large_path = large ? 1u : 0u;
  info.h = h;
  ctx->last = info;
  if (h > cap) return fail(ctx, CH_E_CAPACITY, "hull has %u vertices, capacity %u", h, cap);
  if (h <= pin_n) {
    std::memcpy(h_hull_idx, hidx, size_t(h) * 4);
  } else {
    hipError_t e = hipMemcpyAsync(h_hull_idx, res_idx, size_t(h) * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hull copy");
  }
  return CH_OK;
}

size_t ch_gpufilter_workspace_bytes(uint32_t n) { return qlayout(n).gpufilter_end; }
size_t ch_hull_queues_workspace_bytes(uint32_t n) { return qlayout(n).total; }

ch_status ch_gpufilter(ch_ctx* ctx, const float* d_xy, uint32_t n, int extremes_mode,
                       uint8_t* d_label, ch_octagon* d_oct, uint32_t* d_count, void* d_ws,
                       size_t ws_bytes, void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (ch_status s = check_points(ctx, d_xy, n)) return s;
  if (extremes_mode != CH_EXTREMES_FUSED && extremes_mode != CH_EXTREMES_TWO_KERNELS)
    return fail(ctx, CH_E_INVALID_ARG, "unknown extremes mode %d", extremes_mode);
  if (n && !d_label) return fail(ctx, CH_E_INVALID_ARG, "d_label is NULL");
  const QLayout Q = qlayout(n);
  if (!d_ws || ws_bytes < Q.gpufilter_end)
    return fail(ctx, CH_E_INVALID_ARG, "workspace needs %zu bytes, got %zu", Q.gpufilter_end, ws_bytes);
  if (reinterpret_cast<uintptr_t>(d_ws) & 255u)
    return fail(ctx, CH_E_INVALID_ARG, "workspace must be 256-byte aligned");
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(n);
  uint32_t* count = d_count ? d_count : &at<Header>(d_ws, L.hdr)->count;
  if (n == 0) {
    if (d_count) {
      hipError_t e = launch_set_u32(d_count, 0u, st);
      if (e != hipSuccess) return hip_fail(ctx, e, "set count");
    }
    return CH_OK;
  }
  if (ch_status s = run_gpufilter(ctx, d_xy, n, extremes_mode, at<uint32_t>(d_ws, Q.surv), count,
                                  d_label, d_ws, L, st))
    return s;
  if (d_oct) {
    ProfScope p(ctx, st, "oct_out");
    hipError_t e = launch_oct_out(at<Header>(d_ws, L.hdr), d_oct, st);
    if (e != hipSuccess) return hip_fail(ctx, e, "oct_out launch");
  }
  prof_collect(ctx, st);
  return CH_OK;
}

ch_status ch_hull_queues(ch_ctx* ctx, const float* d_xy, uint32_t n, int extremes_mode,
                         uint32_t* h_hull_idx, uint32_t cap, uint32_t* h_out, uint32_t* h_qcount,
                         void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (ch_status s = check_points(ctx, d_xy, n)) return s;
  if (extremes_mode != CH_EXTREMES_FUSED && extremes_mode != CH_EXTREMES_TWO_KERNELS)
    return fail(ctx, CH_E_INVALID_ARG, "unknown extremes mode %d", extremes_mode);
  if (!h_out) return fail(ctx, CH_E_INVALID_ARG, "h_out is NULL");
  if (cap && !h_hull_idx) return fail(ctx, CH_E_INVALID_ARG, "h_hull_idx is NULL");
  const QLayout Q = qlayout(n);
  if (n && (!d_ws || ws_bytes < Q.total))
    return fail(ctx, CH_E_INVALID_ARG, "workspace needs %zu bytes, got %zu", Q.total, ws_bytes);
  if (reinterpret_cast<uintptr_t>(d_ws) & 255u)
    return fail(ctx, CH_E_INVALID_ARG, "workspace must be 256-byte aligned");
  if (n == 0) {
    *h_out = 0;
    if (h_qcount) std::memset(h_qcount, 0, 4 * sizeof(uint32_t));
    return CH_OK;
  }
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const Layout L = layout(n);
  Header* hdr = at<Header>(d_ws, L.hdr);
  Result* res = at<Result>(d_ws, L.res);
  uint32_t* res_idx = at<uint32_t>(d_ws, L.res_idx);
  uint8_t* labels = at<uint8_t>(d_ws, Q.labels);
  QState* qs = at<QState>(d_ws, Q.qstate);
  const size_t lcap = size_t(kColumns) + 2;
  Rec* lstA = at<Rec>(d_ws, Q.lstA);
  const uint32_t pin_n = hull_cap(n) < kPinIdx ? hull_cap(n) : kPinIdx;
  Result* dres_host = reinterpret_cast<Result*>(ctx->pinned_dev);
  uint32_t* didx_host = ctx->pinned_dev ? reinterpret_cast<uint32_t*>(ctx->pinned_dev + kResBytes) : nullptr;
  if (ch_status s = run_gpufilter(ctx, d_xy, n, extremes_mode, at<uint32_t>(d_ws, Q.surv),
                                  &hdr->count, labels, d_ws, L, st))
    return s;
  hipError_t e;
  {
    ProfScope p(ctx, st, "queue_split");
    e = launch_queue_split(labels, n, hdr, at<uint32_t>(d_ws, Q.qblk), qs, at<uint32_t>(d_ws, Q.qidx),
                           st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "queue split launch");
  {
    ProfScope p(ctx, st, "queue_order");
    e = launch_queue_order(d_xy, n, at<uint32_t>(d_ws, Q.qidx), qs, hdr, at<uint64_t>(d_ws, Q.colbot),
                           at<uint64_t>(d_ws, Q.coltop), st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "queue order launch");
  {
    ProfScope p(ctx, st, "queue_lists");
    e = launch_queue_lists(at<uint64_t>(d_ws, Q.colbot), at<uint64_t>(d_ws, Q.coltop),
                           at<uint32_t>(d_ws, Q.colcnt), lstA, lcap, hdr, qs, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "queue lists launch");
  {
    // Queues 1, 2 feed the upper arcs, 3, 4 the lower ones.
    ProfScope p(ctx, st, "queue_hulls");
    e = launch_list_chains(4, lstA, at<Rec>(d_ws, Q.lstB), lcap, qs->begin, qs->len, 0xCu,
                           at<uint32_t>(d_ws, Q.wcnt), qs->pack, qs->fold, st, nullptr);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "queue hulls launch");
  {
    ProfScope p(ctx, st, "queue_union");
    e = launch_queue_union(lstA, lcap, qs, hdr, res, res_idx, hull_cap(n), dres_host, didx_host,
                           pin_n, st);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "queue union launch");
  const Result* hres = reinterpret_cast<const Result*>(ctx->pinned);
  const uint32_t* hidx = reinterpret_cast<const uint32_t*>(ctx->pinned + kResBytes);
  if (!ctx->pinned_dev) e = hipMemcpyAsync(ctx->pinned, res, kResBytes + 4 * size_t(pin_n),
                                           hipMemcpyDeviceToHost, st);
  uint32_t qc[4] = {0, 0, 0, 0};
  if (e == hipSuccess && h_qcount) e = hipMemcpyAsync(qc, qs->count, sizeof qc, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_fail(ctx, e, "queue hull");
  prof_collect(ctx, st);
  if (hres->status == RES_DOMAIN) return fail(ctx, CH_E_DOMAIN, "input outside the 2^-20 grid");
  if (hres->status != RES_DONE) return fail(ctx, CH_E_DEVICE, "queue hull status %u", hres->status);
  const uint32_t h = hres->h;
  if (h > hull_cap(n)) return fail(ctx, CH_E_DEVICE, "queue hull of %u vertices from %u points", h, n);
  *h_out = h;
  if (h_qcount) std::memcpy(h_qcount, qc, sizeof qc);
  if (h > cap) return fail(ctx, CH_E_CAPACITY, "hull has %u vertices, capacity %u", h, cap);
  if (h <= pin_n) {
    std::memcpy(h_hull_idx, hidx, size_t(h) * 4);
  } else {
    e = hipMemcpyAsync(h_hull_idx, res_idx, size_t(h) * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) return hip_fail(ctx, e, "hull copy");
  }
  return CH_OK;
}

size_t ch_hull_batch_workspace_bytes(uint32_t nsets, uint64_t total_points) {
  return batch_layout(nsets, total_points).total;
}

ch_status ch_hull_batch(ch_ctx* ctx, const float* d_xy, const uint64_t* d_off, uint32_t nsets,
                        uint64_t total_points, uint32_t* d_hull_idx, uint32_t* d_hull_count,
                        void* d_ws, size_t ws_bytes, void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (nsets == 0) return CH_OK;
  if (ch_status s = check_batch(ctx, d_xy, d_off, nsets, total_points, d_hull_idx, d_hull_count,
                                d_ws, ws_bytes))
    return s;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (ch_status s = run_batch(ctx, batch_params_for(ctx, nsets, total_points), d_xy, d_off, nsets,
                              total_points, d_hull_idx, d_hull_count, d_ws, st))
    return s;
  prof_collect(ctx, st);
  return CH_OK;
}

ch_status ch_batch_params_get(const ch_ctx* ctx, uint32_t nsets, uint64_t total_points,
                              ch_batch_params* out) {
  if (!ctx || !out) return CH_E_INVALID_ARG;
  *out = batch_params_for(ctx, nsets, total_points);
  return CH_OK;
}

ch_status ch_batch_params_set(ch_ctx* ctx, const ch_batch_params* p) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (!p) {
    ctx->batch = default_batch_params(ctx->cu_count);
    ctx->batch_fixed = false;
    return CH_OK;
  }
  if (!valid_batch_params(*p)) return fail(ctx, CH_E_INVALID_ARG, "batch parameters out of range");
  ctx->batch = *p;
  ctx->batch_fixed = true;
  return CH_OK;
}

ch_status ch_tune_batch(ch_ctx* ctx, const float* d_xy, const uint64_t* d_off, uint32_t nsets,
                        uint64_t total_points, uint32_t* d_hull_idx, uint32_t* d_hull_count,
                        void* d_ws, size_t ws_bytes, void* stream, ch_batch_params* best_out) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (nsets == 0) return fail(ctx, CH_E_INVALID_ARG, "nothing to tune on");
  if (ch_status s = check_batch(ctx, d_xy, d_off, nsets, total_points, d_hull_idx, d_hull_count,
                                d_ws, ws_bytes))
    return s;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const bool prof = ctx->prof;
  ctx->prof = false;
  hipEvent_t ea = nullptr, eb = nullptr;
  if (hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess) {
    if (ea) (void)hipEventDestroy(ea);
    ctx->prof = prof;
    return fail(ctx, CH_E_DEVICE, "event creation failed");
  }
  // Median of three timed runs after one warm-up.
  auto time_of = [&](const ch_batch_params& p, float& ms) -> ch_status {
    float t[3];
    for (int r = -1; r < 3; ++r) {
      hipError_t e = hipEventRecord(ea, st);
      if (e != hipSuccess) return hip_fail(ctx, e, "tune event");
      if (ch_status s = run_batch(ctx, p, d_xy, d_off, nsets, total_points, d_hull_idx,
                                  d_hull_count, d_ws, st))
        return s;
      e = hipEventRecord(eb, st);
      if (e == hipSuccess) e = hipEventSynchronize(eb);
      if (e == hipSuccess && r >= 0) e = hipEventElapsedTime(&t[r], ea, eb);
      if (e != hipSuccess) return hip_fail(ctx, e, "tune timing");
    }
    std::sort(t, t + 3);
    ms = t[1];
    return CH_OK;
  };
  // Coordinate descent from the defaults: tile size, pass grid, hull grid,
  // then the set size from which sets get a sample polygon.
  const uint32_t cu = (uint32_t)ctx->cu_count;
  ch_batch_params best = default_batch_params(ctx->cu_count);
  float best_ms = 0.f;
  ch_status st_all = time_of(best, best_ms);
  const uint32_t tiles[] = {4096, 8192, 16384, 32768};
  const uint32_t passm[] = {2, 4, 8, 16};
  const uint32_t hullm[] = {3, 6, 9, 12};
  const uint32_t smins[] = {1u << 13, 1u << 15, 1u << 17, 0xFFFFFFFFu};
  for (int dim = 0; dim < 4 && st_all == CH_OK; ++dim) {
    const int nv = 4;
    for (int i = 0; i < nv && st_all == CH_OK; ++i) {
      ch_batch_params c = best;
      if (dim == 0) c.tile_points = tiles[i];
      if (dim == 1) c.pass_blocks = passm[i] * cu;
      if (dim == 2) c.hull_blocks = hullm[i] * cu;
      if (dim == 3) c.sample_min = smins[i];
      if (std::memcmp(&c, &best, sizeof c) == 0) continue;
      float ms = 0.f;
      st_all = time_of(c, ms);
      if (st_all == CH_OK && ms < best_ms) { best_ms = ms; best = c; }
    }
  }
  (void)hipEventDestroy(ea);
  (void)hipEventDestroy(eb);
  ctx->prof = prof;
  if (st_all != CH_OK) return st_all;
  // The outputs hold the last run's (correct) result; record the winner.
  const int ls = lg_bucket(nsets), lp = lg_bucket(total_points);
  bool replaced = false;
  for (auto& e : ctx->tuned)
    if (e.lg_sets == ls && e.lg_points == lp) { e.p = best; replaced = true; }
  if (!replaced) ctx->tuned.push_back({ls, lp, best});
  ctx->batch_fixed = false;
  if (best_out) *best_out = best;
  if (!ctx->tune_path.empty() && !save_tune_cache(ctx))
    return fail(ctx, CH_E_INVALID_ARG, "cannot write the tune cache %s", ctx->tune_path.c_str());
  return CH_OK;
}

ch_status ch_last_hull_info(const ch_ctx* ctx, ch_hull_info* out) {
  if (!ctx || !out) return CH_E_INVALID_ARG;
  *out = ctx->last;
  return CH_OK;
}

ch_status ch_profile_enable(ch_ctx* ctx, int on) {
  if (!ctx) return CH_E_INVALID_ARG;
  ctx->prof = on != 0;
  return CH_OK;
}

ch_status ch_profile_reset(ch_ctx* ctx) {
  if (!ctx) return CH_E_INVALID_ARG;
  for (auto& s : ctx->stats) { s.launches = 0; s.ms = 0.0; }
  return CH_OK;
}

ch_status ch_diag_read_stream(ch_ctx* ctx, const void* d_buf, size_t bytes, uint32_t blocks,
                              void* stream) {
  if (!ctx) return CH_E_INVALID_ARG;
  if (!d_buf) return fail(ctx, CH_E_INVALID_ARG, "d_buf is NULL");
  if ((bytes & 15u) || (reinterpret_cast<uintptr_t>(d_buf) & 15u))
    return fail(ctx, CH_E_INVALID_ARG, "bytes and d_buf must be multiples of 16");
  if (blocks == 0) blocks = (uint32_t)ctx->cu_count * 2;
  if (blocks > 65535) return fail(ctx, CH_E_INVALID_ARG, "blocks above 65535");
  if (bytes == 0) return CH_OK;
  DeviceGuard g(ctx->device);
  if (!g.ok) return fail(ctx, CH_E_DEVICE, "hipSetDevice failed");
  const hipError_t e =
      launch_read_stream(d_buf, bytes, blocks, nullptr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(ctx, e, "read stream launch");
  return CH_OK;
}

ch_status ch_profile_read(ch_ctx* ctx, ch_kernel_stat* out, int cap, int* n_out) {
  if (!ctx || !n_out || (cap > 0 && !out)) return CH_E_INVALID_ARG;
  const int n = (int)ctx->stats.size();
  for (int i = 0; i < n && i < cap; ++i) {
    out[i].name = ctx->stats[i].name;
    out[i].launches = ctx->stats[i].launches;
    out[i].total_ms = ctx->stats[i].ms;
  }
  *n_out = n;
  return CH_OK;
}

}  // extern "C"
