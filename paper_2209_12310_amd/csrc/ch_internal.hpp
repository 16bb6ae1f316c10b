// Internal layout shared by the HIP kernels and the host side of libconvhull.
// Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace chk {

constexpr int kBlock = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kBlock / 64;

// Pass 1 (extreme-key reduction).
constexpr int kReduceMaxBlocks = 2048;

// Pass 2 (octagon test + ordered compaction): 8 float4 loads = 16 points per
// thread per tile.
constexpr int kPairsPerThread = 8;
constexpr uint32_t kTilePairs = kBlock * kPairsPerThread;  // 2048 pairs
constexpr uint32_t kTilePoints = 2 * kTilePairs;           // 4096 points

// Hull rounds.
constexpr int kHullTile = 2048;        // items per tile hull (LDS resident)
constexpr int kHullGridMax = 1024;
constexpr int kMaxRounds = 48;
constexpr uint32_t kHullCapMax = 1u << 21;  // strict vertices of a hull on the grid

// Column table for large hulls: one bottom and one top entry per grid column.
constexpr uint32_t kColumns = 1u << 20;
constexpr uint32_t kColChunk = 4096;   // columns per compaction block
constexpr uint32_t kColBlocks = kColumns / kColChunk;

constexpr uint32_t kCountDomain = 0xFFFFFFFFu;

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

struct Header {
  uint32_t arrive;     // pass-1 blocks finished (reset by the last one)
  uint32_t tile_ctr;   // pass-2 dynamic tile ids (reset by pass 1)
  uint32_t dom_bad;    // a pass-1 block saw an off-grid / NaN value
  uint32_t count;      // survivor count (ch_hull path)
  uint32_t vidx[8];    // smallest index per octagon slot (atomicMin in pass 2)
  uint32_t col_arrive; // column-table bookkeeping
  uint32_t pad[7];
  Octagon oct;
};

// Followed directly in memory by the hull index array, so that one small
// device-to-host copy returns status, h and a short hull.
struct Result {
  uint32_t status;
  uint32_t h;
  uint32_t lcount;     // large-hull path: lower / upper chain lengths
  uint32_t ucount;
  uint32_t cin;        // input count of the latest hull round
  uint32_t pad[3];
  uint32_t round_cnt[kMaxRounds];   // records written by round r (index r+1 = output of round r)
  uint32_t round_tile[kMaxRounds];  // dynamic tile counter of round r
  uint32_t win_cnt[4];              // window-round outputs (lower, upper) per parity
};

struct Rec {           // a candidate hull point: grid coordinates + index
  int32_t x, y;
  uint32_t i, pad;
};

constexpr size_t kHdrBytes = 1024;
constexpr size_t kResBytes = 1024;
static_assert(sizeof(Header) <= kHdrBytes, "header too large");
static_assert(sizeof(Result) <= kResBytes, "result too large");

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

inline uint32_t filter_tiles(uint32_t n) {
  // Pairs after the (optional) unaligned head point, half pair included.
  uint64_t pairs = (uint64_t(n) + 1) / 2;
  uint64_t t = (pairs + kTilePairs - 1) / kTilePairs;
  return t ? uint32_t(t) : 1u;
}

inline uint32_t hull_cap(uint32_t n) { return n < kHullCapMax ? (n ? n : 1u) : kHullCapMax; }

// Workspace layout. ch_filter uses the prefix up to `filter_end`.
struct Layout {
  size_t hdr, res, res_idx, partials, tstat, filter_end;
  size_t surv, recA, recB, colbot, coltop, colcnt, lstA, lstB, wcnt, total;
};

inline Layout layout(uint32_t n) {
  Layout L{};
  size_t o = 0;
  L.hdr = o;       o += kHdrBytes;
  L.res = o;       o += kResBytes;
  L.res_idx = o;   o = align_up(o + size_t(hull_cap(n)) * 4, 256);
  L.partials = o;  o = align_up(o + size_t(kReduceMaxBlocks) * 8 * sizeof(double), 256);
  L.tstat = o;     o = align_up(o + size_t(filter_tiles(n)) * 8, 256);
  L.filter_end = o;
  size_t m = n ? n : 1;
  L.surv = o;      o = align_up(o + m * 4, 256);
  if (n <= (uint32_t)kHullTile) {  // one tile: no further rounds, no large-hull path
    L.recA = L.recB = L.colbot = L.coltop = L.colcnt = L.lstA = L.lstB = L.wcnt = o;
    L.total = o;
    return L;
  }
  L.recA = o;      o = align_up(o + m * sizeof(Rec), 256);
  L.recB = o;      o = align_up(o + m * sizeof(Rec), 256);
  L.colbot = o;    o = align_up(o + size_t(kColumns) * 8, 256);
  L.coltop = o;    o = align_up(o + size_t(kColumns) * 8, 256);
  L.colcnt = o;    o = align_up(o + size_t(kColBlocks) * 2 * 4, 256);
  // Lower / upper candidate chains: at most 2 per column (+1).
  const size_t chain_cap = size_t(kColumns) + 2;
  L.lstA = o;      o = align_up(o + 2 * chain_cap * sizeof(Rec), 256);
  L.lstB = o;      o = align_up(o + 2 * chain_cap * sizeof(Rec), 256);
  L.wcnt = o;      o = align_up(o + 2 * (chain_cap / kHullTile + 4) * 4, 256);
  L.total = o;
  return L;
}

}  // namespace chk
