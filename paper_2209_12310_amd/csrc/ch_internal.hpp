// Internal layout shared by the HIP kernels and the host side of libconvhull.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace chk {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;

// Pass 1 (extreme-key reduction) and pass 2 (filter): persistent grids.
constexpr int kReduceMaxBlocks = 4096;
constexpr int kFilterMaxBlocks = 1024;   // the look-back reads at most 1024 words

// Hull rounds.
constexpr int kHullTile = 2048;        // items per tile hull (LDS resident)
constexpr int kFinalTile = 4096;       // items the single-workgroup final hull takes
constexpr int kHullGridMax = 1024;
constexpr int kMaxRounds = 48;
constexpr uint32_t kLargeDirect = 4096;  // survivors above which ch_hull skips the tile rounds
constexpr uint32_t kHullCapMax = 1u << 21;  // strict vertices of a hull on the grid

// Column table for large hulls: one bottom and one top entry per grid column.
constexpr uint32_t kColumns = 1u << 20;
constexpr uint32_t kColChunk = 4096;   // columns per compaction block
constexpr uint32_t kColBlocks = kColumns / kColChunk;

// Large-hull path of ch_hull: the records are partitioned by column chunk
// (kChunkCols columns each, kChunks chunks) by kPartMax workgroups at most;
// one workgroup per chunk keeps the bottom and top point of each of its
// columns in LDS and chains them; the chunk chains are packed and folded.
constexpr uint32_t kChunkCols = 1024;
constexpr uint32_t kChunks = kColumns / kChunkCols;
constexpr uint32_t kChunkStride = kChunkCols + 2;  // list slots per chunk (a chain holds <= kChunkCols + 1)
constexpr uint32_t kPartMax = 512;
constexpr size_t kLargeListCap = size_t(kChunks) * kChunkStride;  // records per list
constexpr uint32_t kGroupChunks = 32;                  // chunk chains chained together
constexpr uint32_t kGroups = kChunks / kGroupChunks;
constexpr size_t kGroupStride = size_t(kGroupChunks) * kChunkStride;

constexpr uint32_t kCountDomain = 0xFFFFFFFFu;

// Host-side bracket around the kernel launches of a multi-kernel launcher
// (per-kernel timing on the launch stream); launchers take it as null when
// timing is off.
struct LaunchHook {
  virtual void begin(const char* name) = 0;
  virtual void end() = 0;
  virtual ~LaunchHook() = default;
};

template <class F>
inline void hooked(LaunchHook* hk, const char* name, F&& launch) {
  if (hk) hk->begin(name);
  launch();
  if (hk) hk->end();
}

enum : uint32_t { RES_PENDING = 0, RES_DONE = 1, RES_MORE = 2, RES_DOMAIN = 3 };

// The octagon and its edge forms, written once per call by the last block of
// pass 1. Edge i runs from slot i to slot i+1 (slot order E NE N NW W SW S SE).
// L_i(x, y) = A[i]*x + B[i]*y + C[i] with x, y in float units (A, B carry the
// 2^20 grid scale) equals the exact integer orientation of (v_i, v_i+1, p).
struct Octagon {
  double A[8], B[8], C[8];
  int32_t vx[8], vy[8];
  float box[4];        // open box xl < x < xh, yl < y < yh lying inside
  uint32_t status;     // 0 ok, 1 domain error
  uint32_t box_ok;
  uint32_t pad[2];
};

// The axis extremes of the two-kernel extreme search (the first of its two
// reductions), read by every workgroup of the second: the combined keys and
// the box the four points span (float units).
struct AxisBox {
  double kE_max, kE_min, kN_max, kN_min;
  double ex, wx, ny, sy;  // E.x, W.x, N.y, S.y
  uint32_t bad;           // the keys did not decode (domain error)
  uint32_t pad[7];
};

struct Header {
  uint32_t arrive;     // pass-1 blocks finished (reset by the last one)
  uint32_t tile_ctr;   // pass-2 dynamic tile ids (reset by pass 1)
  uint32_t dom_bad;    // a pass-1 block saw an off-grid / NaN value
  uint32_t count;      // survivor count (ch_hull path)
  uint32_t vidx[8];    // smallest index per octagon slot (atomicMin in pass 2)
  uint32_t col_arrive; // column-table bookkeeping
  uint32_t pad[7];
  Octagon oct;
  AxisBox axis;
};

// Followed directly in memory by the hull index array, so that one small
// device-to-host copy returns status, h and a short hull.
struct Result {
  uint32_t status;
  uint32_t h;
  uint32_t lcount;     // large-hull path: lower / upper chain lengths
  uint32_t ucount;
  uint32_t cin;        // input count of the latest hull round
  uint32_t ncand;      // candidate records of the fused pass (0 without one)
  uint32_t mode;       // how the fused pass ran (ch_hull_info.single_read)
  uint32_t cand_surv;  // 1: the octagon test was skipped, the survivors are the candidate records
  uint32_t round_cnt[kMaxRounds];   // records written by round r (index r+1 = output of round r)
  uint32_t round_tile[kMaxRounds];  // dynamic tile counter of round r
  uint32_t pack_cnt[2];             // large-hull path: window chains packed (lower, upper)
  uint32_t fold_cnt[2];             // large-hull path: final chain lengths (lower, upper)
};

struct Rec {           // a candidate hull point: grid coordinates + index
  int32_t x, y;
  uint32_t i, pad;
};

// Refined filter of the hull path: a second inner polygon whose vertices are
// input points -- the extreme points of a strided sample of the input in
// kPolyMax (or kBatchDirs) directions -- so a point strictly inside it is not
// a hull vertex. Tested after the octagon's box through a disc around an
// inner grid point, then exactly.
constexpr int kPolyMax = 512;              // directions (and at most vertices), single set
constexpr uint32_t kLutBins = 2048;        // single set: pseudo-angle bins of the wedge table
constexpr uint32_t kBatchLutBins = 1024;   // batch: wedge-table bins of a set's second polygon
constexpr uint32_t kSampleN = 65536;       // single set: sample points
constexpr uint32_t kSamplePer = 256;       // sample points per direction workgroup
constexpr uint32_t kSampleRun = 16;        // batch: consecutive points per sample run (128 bytes)
constexpr uint32_t kSampleBlocks = kSampleN / kSamplePer;
constexpr uint32_t kSampleMin = 1u << 17;  // ch_hull samples from this many points on
constexpr uint32_t kBatchDirs = 256;       // batch: directions per set
constexpr uint32_t kBatchSample = 2048;    // batch: sample points per chunk
static_assert(kBatchSample % kSampleRun == 0, "whole runs");
constexpr uint32_t kBatchChunkPoints = 131072;  // batch: one sample chunk per this many points
constexpr uint32_t kBatchChunksMax = 4;
constexpr uint32_t kBatchSampleMin = 1u << 15;

template <uint32_t V>
struct SamplePolyT {
  uint32_t nv;         // vertex count; below 3 the polygon is not used
  int32_t cx, cy;      // grid point strictly inside the polygon
  float r2;            // squared radius (float units) of a disc about (cx, cy) inside
                       // the polygon, rounded down with a margin for fp32 tests
  float os, ot;        // octagon |dx| <= os, |dy| <= os, |dx| + |dy| <= ot (float
                       // units) about (cx, cy) inside the polygon; 0 when none
  int32_t vx[V], vy[V];  // counter-clockwise, strictly convex
};
using SamplePoly = SamplePolyT<kPolyMax>;

// Single set, second polygon from the survivors (see k_refine_bins):
// bins, vertex capacity, wedge-table bins.
constexpr uint32_t kRefineBins = 1024;
constexpr uint32_t kRefineLut = 2048;
constexpr uint32_t kRefineMaxSingle = 1u << 18;  // more survivors: straight to the large-hull path
struct RefineState {
  uint64_t bin[kRefineBins];  // (dot product, record) maxima per bin; zero between calls
  uint32_t arrive;            // workgroups of k_refine_bins done; zero between calls
  uint32_t cnt;               // records kept by k_refine_filter
  uint32_t pad[62];
  SamplePolyT<kRefineBins> poly;
  uint32_t lut[kRefineLut];
};

constexpr size_t kHdrBytes = 1024;
constexpr size_t kResBytes = 1024;
static_assert(sizeof(Header) <= kHdrBytes, "header too large");
static_assert(sizeof(Result) <= kResBytes, "result too large");

constexpr size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr uint32_t hull_cap(uint32_t n) { return n < kHullCapMax ? (n ? n : 1u) : kHullCapMax; }

// Workspace layout. ch_filter uses the prefix up to `filter_end`.
struct Layout {
  size_t hdr, res, res_idx, partials, part_bad, tstat, staging, filter_end;
  size_t surv, recA, recB, phist, ptot, lstA, lstB, wcnt, poly, samp, refine, total;
};

constexpr Layout layout(uint32_t n) {
  Layout L{};
  size_t o = 0;
  L.hdr = o;       o += kHdrBytes;
  L.res = o;       o += kResBytes;
  L.res_idx = o;   o = align_up(o + size_t(hull_cap(n)) * 4, 256);
  L.partials = o;  o = align_up(o + size_t(kReduceMaxBlocks) * 8 * sizeof(double), 256);
  L.part_bad = o;  o = align_up(o + size_t(kReduceMaxBlocks) * 4, 256);
  L.tstat = o;     o = align_up(o + size_t(kFilterMaxBlocks) * 8, 256);
  size_t m = n ? n : 1;
  L.staging = o;   o = align_up(o + m * 4, 256);
  L.filter_end = o;
  // ch_hull: survivor records, then two record lists for the rounds (list B
  // doubles as the filter's overflow staging for the survivor records).
  L.surv = o;      o = align_up(o + m * sizeof(Rec), 256);
  L.recA = o;      o = align_up(o + m * sizeof(Rec), 256);
  L.recB = o;      o = align_up(o + m * sizeof(Rec), 256);
  if (n <= (uint32_t)kFinalTile) {  // one workgroup: no rounds, no large-hull path
    L.phist = L.ptot = L.lstA = L.lstB = L.wcnt = L.poly = L.samp = L.refine = o;
    L.total = o;
    return L;
  }
  // Large-hull path: the partition's count table (chunk-major) and chunk
  // totals, then the lower and upper lists (kLargeListCap records each) in
  // two buffers, and the chain length of every chunk of both lists.
  L.phist = o;     o = align_up(o + size_t(kChunks) * kPartMax * 4, 256);
  L.ptot = o;      o = align_up(o + size_t(kChunks) * 4, 256);
  L.lstA = o;      o = align_up(o + 2 * kLargeListCap * sizeof(Rec), 256);
  L.lstB = o;      o = align_up(o + 2 * kLargeListCap * sizeof(Rec), 256);
  L.wcnt = o;      o = align_up(o + 2 * size_t(kChunks + kGroups) * 4, 256);
  // Refined filter: the sample polygon and the direction maxima, then the
  // second polygon's state.
  L.poly = o;      o = align_up(o + sizeof(SamplePoly), 256);
  L.samp = o;      o = align_up(o + size_t(kPolyMax) * 8 + 256 + size_t(kLutBins) * 4 +
                                       size_t(kSampleBlocks) * kPolyMax * 16, 256);
  L.refine = o;    o = align_up(o + sizeof(RefineState), 256);
  L.total = o;
  return L;
}

// ------------------------------------------------- Alg. 1 with its four queues
// (ch_gpufilter, ch_hull_queues). Queue q (0..3 here, the paper's 1..4)
// holds the points labelled q + 1 by Alg. 2's array.
constexpr uint32_t kQBlocksMax = 1024;   // label-split workgroups
constexpr uint32_t kQChunkMin = 4096;    // labels per split workgroup at least

struct QState {
  uint32_t count[4];   // queue sizes
  uint32_t base[4];    // start of queue q in the queue array
  uint32_t emit[4];    // column entries emitted into list q
  uint32_t begin[4];   // first record of list q (1 when its start end was already there)
  uint32_t len[4];     // records of list q, both arc ends included
  uint32_t pack[4];    // packed window chains of list q
  uint32_t fold[4];    // chain length of list q
  uint32_t pad[4];
};

// Workspace of ch_gpufilter (prefix) and ch_hull_queues: the filter's layout
// up to filter_end, the ordered survivor indices, then (queues) the label
// array, the split counts, the queue array, the column tables and four
// record lists in each of two buffers.
struct QLayout {
  size_t surv, gpufilter_end, labels, qblk, qstate, qidx, colbot, coltop, colcnt, lstA, lstB, wcnt,
      total;
};

inline QLayout qlayout(uint32_t n) {
  QLayout Q{};
  const Layout L = layout(n);
  const size_t m = n ? n : 1;
  size_t o = L.filter_end;
  Q.surv = o;      o = align_up(o + m * 4, 256);
  Q.gpufilter_end = o;
  Q.labels = o;    o = align_up(o + m + 16, 256);
  Q.qblk = o;      o = align_up(o + size_t(kQBlocksMax) * 4 * 4, 256);
  Q.qstate = o;    o = align_up(o + sizeof(QState), 256);
  Q.qidx = o;      o = align_up(o + m * 4, 256);
  Q.colbot = o;    o = align_up(o + size_t(kColumns) * 8, 256);
  Q.coltop = o;    o = align_up(o + size_t(kColumns) * 8, 256);
  Q.colcnt = o;    o = align_up(o + size_t(kColBlocks) * 4 * 4, 256);
  const size_t cap = size_t(kColumns) + 2;
  Q.lstA = o;      o = align_up(o + 4 * cap * sizeof(Rec), 256);
  Q.lstB = o;      o = align_up(o + 4 * cap * sizeof(Rec), 256);
  Q.wcnt = o;      o = align_up(o + 4 * (cap / 4096 + 2) * 4, 256);
  Q.total = o;
  return Q;
}

// ---------------------------------------------------------------- batch mode
constexpr uint32_t kBatchTile = 8192;     // default points per pass-1/pass-2 tile of one set
constexpr uint32_t kBatchTileMin = 4096;  // smallest tile the workspace is sized for
constexpr uint32_t kBatchTileMax = 65536;
constexpr int kBatchRounds = 4;           // tile-hull rounds for sets with many survivors
constexpr uint32_t kCountInvalid = 0xFFFFFFFDu;

struct SetTile {       // points [begin, end) of set `set` (global indices)
  uint32_t set, begin, end, pad;
};

struct BatchHdr {
  uint32_t ntiles;                   // pass tiles (plan kernel)
  uint32_t bad_offsets;              // offsets not non-decreasing or not ending at the total
  uint32_t nround[kBatchRounds + 1]; // hull-round tiles per round
  uint32_t nsampled;                 // sets in the sampler's list (plan kernel)
  uint32_t sample_next;              // next list entry a sampler workgroup takes
  uint32_t refine_next;              // next set a second-polygon workgroup takes
  uint32_t ncand_tiles;              // tiles of the candidates' octagon test
  uint32_t final_next;               // next entry of the first block-hull list
  uint32_t pass_next;                // next pass tile a workgroup takes
  uint32_t pad[4];
};

// Per-set state, one struct per set.
struct SetState {
  uint64_t key[8];     // order-preserving encodings of the 8 slot keys (max)
  uint32_t bad;        // domain flag
  uint32_t done;       // hull written
  uint32_t cnt[kBatchRounds + 1];  // candidates after the filter / after round r
  uint32_t vidx[8];    // smallest index per octagon slot (kept for the shared classifier)
  uint32_t ncand;       // candidate records of the single read (fused pass)
  Octagon oct;
};

struct BatchLayout {
  size_t hdr, sets, polys, luts, slist, tiles, rtiles, recA, recB, total;
};

// Sample chunks of a set of n points in batch mode (0: no sample polygon).
__host__ __device__ inline uint32_t batch_chunks(uint64_t n, uint32_t sample_min) {
  if (n < sample_min || n < kBatchSample) return 0;
  const uint64_t c = n / kBatchChunkPoints;
  return c < 1 ? 1u : (c > kBatchChunksMax ? kBatchChunksMax : (uint32_t)c);
}

inline BatchLayout batch_layout(uint32_t nsets, uint64_t total_points) {
  BatchLayout L{};
  size_t o = 0;
  const size_t ntiles = total_points / kBatchTileMin + nsets + 1;
  const size_t nrt = total_points / 2048 + nsets + 1;
  L.hdr = o;    o = align_up(o + sizeof(BatchHdr), 256);
  L.sets = o;   o = align_up(o + size_t(nsets ? nsets : 1) * sizeof(SetState), 256);
  L.polys = o;  o = align_up(o + size_t(nsets ? nsets : 1) * sizeof(SamplePoly), 256);
  L.luts = o;   o = align_up(o + size_t(nsets ? nsets : 1) * kBatchLutBins * sizeof(uint32_t), 256);
  L.slist = o;  o = align_up(o + size_t(nsets ? nsets : 1) * sizeof(uint32_t), 256);
  L.tiles = o;  o = align_up(o + ntiles * sizeof(SetTile), 256);
  L.rtiles = o; o = align_up(o + nrt * sizeof(SetTile), 256);
  const size_t m = total_points ? total_points : 1;
  L.recA = o;   o = align_up(o + m * sizeof(Rec), 256);
  L.recB = o;   o = align_up(o + m * sizeof(Rec), 256);
  L.total = o;
  return L;
}

}  // namespace chk
