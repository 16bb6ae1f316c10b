// Alg. 1 stage by stage, with the four queues the paper builds from Alg. 2's
// label array (Sec. III: on the CPU there; on the device here).
//
//   split   the label array Q (one byte per point: 0 discarded, else the
//           queue 1..4) becomes four index queues, each in ascending index
//           order: per-workgroup counts, one scan, an ordered scatter.
//   order   stage (3), the partial order of a queue: its points are bucketed
//           by grid column. A strict vertex of the arc a queue feeds is the
//           top point of its column (queues 1, 2: the arcs E -> N -> W, on
//           the upper hull) or the bottom point (queues 3, 4: W -> S -> E),
//           so each column keeps one point and the occupied columns, read
//           in x order, are the queue's sorted candidates.
//   lists   per queue, its columns' points between the arc's two axis
//           extremes, with those two extremes added at the ends.
//   hull    stage (4): Andrew's chain of each list (the upper one for
//           queues 1, 2, the lower one for 3, 4), then the union of the four
//           arcs counter-clockwise from W, the lexicographic minimum.
//
// Why the four queues can share one top and one bottom table: with the
// label rule (first octagon edge a point lies strictly outside of; a vertex
// by its first slot), a point of queue 1 lies in the region outside edge
// E->NE or NE->N, whose columns are [N.x, E.x]; queue 2 in [W.x, N.x];
// queue 3 in [W.x, S.x]; queue 4 in [S.x, E.x]. Queues 1 and 2 meet only in
// column N.x, where the only point of either is N itself (a point below N in
// that column is outside none of the edges E->NE, NE->N, N->NW), and
// likewise queues 3 and 4 only in column S.x, at S.
#include "ch_device.hpp"

namespace chk {

// ------------------------------------------------------------------ split

// Labels of workgroup b: [b * chunk, min((b + 1) * chunk, n)), chunk a
// multiple of 16. Counts of labels 1..4 to qblk[4 b + q].
__global__ __launch_bounds__(kBlock) void k_qcount(const uint8_t* __restrict__ labels, uint32_t n,
                                                   uint32_t chunk, const Header* __restrict__ hdr,
                                                   uint32_t* __restrict__ qblk) {
  if (hdr->oct.status != 0) return;  // no labels were written
  const uint32_t a = blockIdx.x * chunk < n ? blockIdx.x * chunk : n;
  const uint32_t e = a + chunk < n ? a + chunk : n;
  uint32_t c[4] = {0, 0, 0, 0};
  for (uint32_t p = a + threadIdx.x * 16; p < e; p += kBlock * 16) {
    uint4 w;
    if (p + 16 <= e) {
      w = *reinterpret_cast<const uint4*>(labels + p);
    } else {
      uint32_t t[4] = {0, 0, 0, 0};
      for (uint32_t i = 0; p + i < e; ++i) t[i >> 2] |= (uint32_t)labels[p + i] << (8 * (i & 3));
      w = make_uint4(t[0], t[1], t[2], t[3]);
    }
    if ((w.x | w.y | w.z | w.w) == 0) continue;
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t l = (ws[k] >> (8 * j)) & 0xFFu;
#pragma unroll
        for (int q = 0; q < 4; ++q) c[q] += l == (uint32_t)(q + 1) ? 1u : 0u;
      }
  }
  // Two 16-bit fields per scan would overflow for large chunks: four scans.
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t tot;
    block_excl_scan(c[q], tot);
    if (threadIdx.x == 0) qblk[4 * blockIdx.x + q] = tot;
  }
}

// One workgroup: queue sizes and bases, and each workgroup's first position
// in each queue (written over its counts). Also clears the per-call list
// state that later kernels read (all four queues empty on a domain error).
__global__ __launch_bounds__(kBlock) void k_qscan(uint32_t* __restrict__ qblk, uint32_t G,
                                                  const Header* __restrict__ hdr,
                                                  QState* __restrict__ qs) {
  if (threadIdx.x < 4) {
    const uint32_t q = threadIdx.x;
    qs->emit[q] = qs->begin[q] = qs->len[q] = qs->pack[q] = qs->fold[q] = 0;
  }
  if (hdr->oct.status != 0) {
    if (threadIdx.x < 4) qs->count[threadIdx.x] = qs->base[threadIdx.x] = 0;
    return;
  }
  const uint32_t per = (G + kBlock - 1) / kBlock;
  const uint32_t b0 = threadIdx.x * per;
  const uint32_t b1 = b0 + per < G ? b0 + per : G;
  uint32_t run[4];
  uint32_t total[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t mine = 0;
    for (uint32_t b = b0; b < b1; ++b) mine += qblk[4 * b + q];
    run[q] = block_excl_scan(mine, total[q]);
  }
  uint32_t base[4];
  base[0] = 0;
  for (int q = 1; q < 4; ++q) base[q] = base[q - 1] + total[q - 1];
  __syncthreads();
  for (uint32_t b = b0; b < b1; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t v = qblk[4 * b + q];
      qblk[4 * b + q] = base[q] + run[q];
      run[q] += v;
    }
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) {
      qs->count[q] = total[q];
      qs->base[q] = base[q];
    }
}

// The ordered scatter: workgroup b walks its labels 4096 at a time (16 per
// thread, in index order across threads), ranks them per queue with a block
// scan and appends their indices to the queues.
__global__ __launch_bounds__(kBlock) void k_qscatter(const uint8_t* __restrict__ labels,
                                                     uint32_t n, uint32_t chunk,
                                                     const Header* __restrict__ hdr,
                                                     const uint32_t* __restrict__ qblk,
                                                     uint32_t* __restrict__ qidx) {
  if (hdr->oct.status != 0) return;
  const uint32_t a = blockIdx.x * chunk < n ? blockIdx.x * chunk : n;
  const uint32_t e = a + chunk < n ? a + chunk : n;
  uint32_t pos[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) pos[q] = qblk[4 * blockIdx.x + q];
  for (uint32_t s = a; s < e; s += kBlock * 16) {
    const uint32_t p = s + threadIdx.x * 16;
    uint4 w = make_uint4(0, 0, 0, 0);
    if (p + 16 <= e) {
      w = *reinterpret_cast<const uint4*>(labels + p);
    } else if (p < e) {
      uint32_t t[4] = {0, 0, 0, 0};
      for (uint32_t i = 0; p + i < e; ++i) t[i >> 2] |= (uint32_t)labels[p + i] << (8 * (i & 3));
      w = make_uint4(t[0], t[1], t[2], t[3]);
    }
    const bool any = (w.x | w.y | w.z | w.w) != 0;
    if (!__syncthreads_or(any)) continue;
    const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
    // Counts of this thread's 16 labels, two queues per 32-bit word (a
    // workgroup step holds at most 4096 labels, so 16-bit fields suffice).
    uint32_t c01 = 0, c23 = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t l = (ws[k] >> (8 * j)) & 0xFFu;
        c01 += (l == 1u ? 1u : 0u) + (l == 2u ? 0x10000u : 0u);
        c23 += (l == 3u ? 1u : 0u) + (l == 4u ? 0x10000u : 0u);
      }
    uint32_t t01, t23;
    const uint32_t x01 = block_excl_scan(c01, t01);
    const uint32_t x23 = block_excl_scan(c23, t23);
    uint32_t o[4] = {pos[0] + (x01 & 0xFFFFu), pos[1] + (x01 >> 16), pos[2] + (x23 & 0xFFFFu),
                     pos[3] + (x23 >> 16)};
    if (any) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const uint32_t l = (ws[k] >> (8 * j)) & 0xFFu;
          if (l >= 1u && l <= 4u) qidx[o[l - 1]++] = p + (uint32_t)(4 * k + j);
        }
    }
    pos[0] += t01 & 0xFFFFu;
    pos[1] += t01 >> 16;
    pos[2] += t23 & 0xFFFFu;
    pos[3] += t23 >> 16;
  }
}

// ------------------------------------------------------------ partial order

// Every queued point into its column: the top table (queues 1, 2) keeps per
// column the largest (y, -index), the bottom table (queues 3, 4) the smallest
// (y, index), with the encodings of the large-hull path's column table.
__global__ __launch_bounds__(kBlock) void k_qbucket(const float* __restrict__ xy,
                                                    const uint32_t* __restrict__ qidx,
                                                    const QState* __restrict__ qs,
                                                    const Header* __restrict__ hdr,
                                                    uint64_t* __restrict__ bot,
                                                    uint64_t* __restrict__ top) {
  if (hdr->oct.status != 0) return;
  const uint32_t upper_end = qs->base[2];
  const uint32_t m = qs->base[3] + qs->count[3];
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < m; k += gridDim.x * kBlock) {
    const uint32_t j = qidx[k];
    const float2 p = reinterpret_cast<const float2*>(xy)[j];
    const uint32_t x = (uint32_t)(p.x * kGridF), y = (uint32_t)(p.y * kGridF);
    if (k < upper_end)
      atomicMax((unsigned long long*)&top[x], ((unsigned long long)(y + 1) << 32) | (0xFFFFFFFFu - j));
    else
      atomicMin((unsigned long long*)&bot[x], ((unsigned long long)y << 32) | j);
  }
}

// ------------------------------------------------------------------ lists

__device__ __forceinline__ Rec col_bot(uint32_t x, uint64_t b) {
  Rec r;
  r.x = (int32_t)x; r.y = (int32_t)(b >> 32); r.i = (uint32_t)b; r.pad = 0;
  return r;
}
__device__ __forceinline__ Rec col_top(uint32_t x, uint64_t t) {
  Rec r;
  r.x = (int32_t)x; r.y = (int32_t)(t >> 32) - 1; r.i = 0xFFFFFFFFu - (uint32_t)t; r.pad = 0;
  return r;
}

// The column entries of the four lists in x order: list 0 (queue 1) the tops
// of columns [N.x, E.x], list 1 the tops of [W.x, N.x], list 2 the bottoms of
// [W.x, S.x], list 3 the bottoms of [S.x, E.x]. Slot 0 of each list is kept
// for its start end. PASS 0 counts per chunk of kColChunk columns, PASS 1
// writes.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_qemit(const uint64_t* __restrict__ bot,
                                                  const uint64_t* __restrict__ top,
                                                  uint32_t* __restrict__ cnt,
                                                  Rec* __restrict__ lists, size_t cap,
                                                  const Header* __restrict__ hdr,
                                                  QState* __restrict__ qs) {
  if (hdr->oct.status != 0) return;
  constexpr uint32_t PER = kColChunk / kBlock;
  const uint32_t ex = (uint32_t)hdr->oct.vx[0], nx = (uint32_t)hdr->oct.vx[2];
  const uint32_t wx = (uint32_t)hdr->oct.vx[4], sx = (uint32_t)hdr->oct.vx[6];
  const uint32_t x0 = blockIdx.x * kColChunk + threadIdx.x * PER;
  auto in_list = [&](uint32_t x, int q) -> bool {
    switch (q) {
      case 0: return x >= nx && x <= ex;
      case 1: return x >= wx && x <= nx;
      case 2: return x >= wx && x <= sx;
      default: return x >= sx && x <= ex;
    }
  };
  uint32_t c01 = 0, c23 = 0;  // 16 columns per thread at most: 16-bit fields
  for (uint32_t e = 0; e < PER; ++e) {
    const uint32_t x = x0 + e;
    if (top[x] != 0ull) c01 += (in_list(x, 0) ? 1u : 0u) + (in_list(x, 1) ? 0x10000u : 0u);
    if (bot[x] != ~0ull) c23 += (in_list(x, 2) ? 1u : 0u) + (in_list(x, 3) ? 0x10000u : 0u);
  }
  uint32_t t01, t23;
  const uint32_t x01 = block_excl_scan(c01, t01);
  const uint32_t x23 = block_excl_scan(c23, t23);
  if (PASS == 0) {
    if (threadIdx.x == 0) {
      cnt[4 * blockIdx.x + 0] = t01 & 0xFFFFu;
      cnt[4 * blockIdx.x + 1] = t01 >> 16;
      cnt[4 * blockIdx.x + 2] = t23 & 0xFFFFu;
      cnt[4 * blockIdx.x + 3] = t23 >> 16;
    }
    return;
  }
  // Entries of the earlier chunks, summed by the whole workgroup.
  uint32_t before[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    uint32_t part = 0;
    for (uint32_t b = threadIdx.x; b < blockIdx.x; b += kBlock) part += cnt[4 * b + q];
    block_excl_scan(part, before[q]);
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    qs->emit[0] = before[0] + (t01 & 0xFFFFu);
    qs->emit[1] = before[1] + (t01 >> 16);
    qs->emit[2] = before[2] + (t23 & 0xFFFFu);
    qs->emit[3] = before[3] + (t23 >> 16);
  }
  uint32_t o[4] = {1 + before[0] + (x01 & 0xFFFFu), 1 + before[1] + (x01 >> 16),
                   1 + before[2] + (x23 & 0xFFFFu), 1 + before[3] + (x23 >> 16)};
  for (uint32_t e = 0; e < PER; ++e) {
    const uint32_t x = x0 + e;
    const uint64_t t = top[x], b = bot[x];
    if (t != 0ull) {
      if (in_list(x, 0)) lists[0 * cap + o[0]++] = col_top(x, t);
      if (in_list(x, 1)) lists[1 * cap + o[1]++] = col_top(x, t);
    }
    if (b != ~0ull) {
      if (in_list(x, 2)) lists[2 * cap + o[2]++] = col_bot(x, b);
      if (in_list(x, 3)) lists[3 * cap + o[3]++] = col_bot(x, b);
    }
  }
}

// One wave, lane q < 4: the arc ends of list q (1: N then E; 2: W then N;
// 3: W then S; 4: S then E, each with its smallest index). The start goes to
// slot 0 unless the first entry already is that point; the end is appended
// unless the last record is that point. Sets begin[q] and len[q].
__global__ void k_qends(Rec* __restrict__ lists, size_t cap, const Header* __restrict__ hdr,
                        QState* __restrict__ qs) {
  const uint32_t q = threadIdx.x;
  if (q >= 4 || hdr->oct.status != 0) return;  // lists stay empty (k_qscan)
  const int ss[4] = {2, 4, 4, 6}, es[4] = {0, 2, 6, 0};
  const int a = ss[q], z = es[q];
  Rec* L = lists + q * cap;
  const uint32_t c = qs->emit[q];
  Rec s;
  s.x = hdr->oct.vx[a]; s.y = hdr->oct.vy[a]; s.i = hdr->vidx[a]; s.pad = 0;
  Rec t;
  t.x = hdr->oct.vx[z]; t.y = hdr->oct.vy[z]; t.i = hdr->vidx[z]; t.pad = 0;
  uint32_t begin = 1;
  if (c == 0 || L[1].x != s.x || L[1].y != s.y) {
    L[0] = s;
    begin = 0;
  }
  uint32_t end = 1 + c;  // one past the last record
  const Rec last = L[end - 1];
  if (last.x != t.x || last.y != t.y) L[end++] = t;
  qs->begin[q] = begin;
  qs->len[q] = end - begin;
}

__global__ void k_col_clear(uint64_t* __restrict__ bot, uint64_t* __restrict__ top) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t x = g; x < kColumns; x += gridDim.x * blockDim.x) {
    bot[x] = ~0ull;
    top[x] = 0ull;
  }
}

// ------------------------------------------------------------------ union

// One workgroup: the counter-clockwise hull from W as the union of the four
// arcs: list 2's chain W..S, list 3's S..E, list 0's N..E backwards (E..N),
// list 1's W..N backwards (N..W), each without its last point (the next arc
// starts there). All axis extremes equal: the one point W. Writes res_idx,
// the result block and (pinned, device-mapped `host`) the first host_n
// indices and the result block in host memory.
__global__ __launch_bounds__(kBlock) void k_qunion(const Rec* __restrict__ lists, size_t cap,
                                                   const QState* __restrict__ qs,
                                                   const Header* __restrict__ hdr,
                                                   Result* __restrict__ res,
                                                   uint32_t* __restrict__ res_idx,
                                                   Result* __restrict__ host,
                                                   uint32_t* __restrict__ host_idx,
                                                   uint32_t host_n, uint32_t res_cap) {
  const bool bad = hdr->oct.status != 0;
  uint32_t f[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) f[q] = bad ? 1u : qs->fold[q];
  const uint32_t n2 = f[2] - 1, n3 = f[3] - 1, n0 = f[0] - 1, n1 = f[1] - 1;
  uint32_t h = n2 + n3 + n0 + n1;
  const bool single = !bad && h == 0;
  if (single) h = 1;
  if (bad) h = 0;
  const uint32_t hw = h < res_cap ? h : res_cap;  // res_idx holds res_cap entries
  for (uint32_t k = threadIdx.x; k < hw; k += kBlock) {
    uint32_t v;
    if (single) v = hdr->vidx[4];
    else if (k < n2) v = lists[2 * cap + k].i;
    else if (k < n2 + n3) v = lists[3 * cap + (k - n2)].i;
    else if (k < n2 + n3 + n0) v = lists[0 * cap + (f[0] - 1 - (k - n2 - n3))].i;
    else v = lists[1 * cap + (f[1] - 1 - (k - n2 - n3 - n0))].i;
    res_idx[k] = v;
    if (host && k < host_n) host_idx[k] = v;
  }
  __syncthreads();
  const uint32_t status = bad ? (uint32_t)RES_DOMAIN : (uint32_t)RES_DONE;
  if (threadIdx.x == 0) {
    res->h = h;
    res->status = status;
  }
  if (host) {
    constexpr uint32_t kWords = sizeof(Result) / 4;
    for (uint32_t t = threadIdx.x; t < kWords; t += kBlock) {
      uint32_t v = reinterpret_cast<const uint32_t*>(res)[t];
      if (t == offsetof(Result, status) / 4) v = status;
      else if (t == offsetof(Result, h) / 4) v = h;
      reinterpret_cast<uint32_t*>(host)[t] = v;
    }
  }
}

// ---------------------------------------------------------------- launchers

uint32_t queue_split_blocks(uint32_t n, uint32_t& chunk) {
  uint32_t G = (n + kQChunkMin - 1) / kQChunkMin;
  if (G < 1) G = 1;
  if (G > kQBlocksMax) G = kQBlocksMax;
  chunk = (uint32_t)((((uint64_t)n + G - 1) / G + 15) / 16 * 16);
  if (chunk == 0) chunk = 16;
  return G;
}

hipError_t launch_queue_split(const uint8_t* labels, uint32_t n, const Header* hdr, uint32_t* qblk,
                              QState* qs, uint32_t* qidx, hipStream_t st) {
  uint32_t chunk = 0;
  const uint32_t G = queue_split_blocks(n, chunk);
  hipLaunchKernelGGL(k_qcount, dim3(G), dim3(kBlock), 0, st, labels, n, chunk, hdr, qblk);
  hipLaunchKernelGGL(k_qscan, dim3(1), dim3(kBlock), 0, st, qblk, G, hdr, qs);
  hipLaunchKernelGGL(k_qscatter, dim3(G), dim3(kBlock), 0, st, labels, n, chunk, hdr, qblk, qidx);
  return hipGetLastError();
}

hipError_t launch_queue_order(const float* xy, uint32_t n, const uint32_t* qidx, const QState* qs,
                              const Header* hdr, uint64_t* bot, uint64_t* top, hipStream_t st) {
  hipLaunchKernelGGL(k_col_clear, dim3(1024), dim3(kBlock), 0, st, bot, top);
  uint32_t g = (n + kBlock - 1) / kBlock;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  hipLaunchKernelGGL(k_qbucket, dim3(g), dim3(kBlock), 0, st, xy, qidx, qs, hdr, bot, top);
  return hipGetLastError();
}

hipError_t launch_queue_lists(const uint64_t* bot, const uint64_t* top, uint32_t* colcnt,
                              Rec* lists, size_t cap, const Header* hdr, QState* qs,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_qemit<0>, dim3(kColBlocks), dim3(kBlock), 0, st, bot, top, colcnt, lists,
                     cap, hdr, qs);
  hipLaunchKernelGGL(k_qemit<1>, dim3(kColBlocks), dim3(kBlock), 0, st, bot, top, colcnt, lists,
                     cap, hdr, qs);
  hipLaunchKernelGGL(k_qends, dim3(1), dim3(64), 0, st, lists, cap, hdr, qs);
  return hipGetLastError();
}

hipError_t launch_queue_union(const Rec* lists, size_t cap, const QState* qs, const Header* hdr,
                              Result* res, uint32_t* res_idx, uint32_t res_cap, Result* host,
                              uint32_t* host_idx, uint32_t host_n, hipStream_t st) {
  hipLaunchKernelGGL(k_qunion, dim3(1), dim3(kBlock), 0, st, lists, cap, qs, hdr, res, res_idx, host,
                     host_idx, host_n, res_cap);
  return hipGetLastError();
}

}  // namespace chk
