// Device hull pass over the filter's survivors (Alg. 1's per-queue hull,
// done here on the GPU with Andrew's monotone chain, Table I).
//
// Main path -- hull of hulls. The candidate list is cut into tiles of
// kHullTile items; each workgroup sorts its tile in LDS by (x, y), keeps one
// entry per distinct coordinate (the smallest index), runs the lower and
// upper monotone chains and appends the tile's hull to the next round's list.
// CH(S) = CH(union of the tile hulls), so rounds repeat until one tile holds
// everything; that tile's hull is the answer.
//
// Large-hull path -- used when a round stops shrinking the list (a hull with
// more vertices than a tile holds, or many points in convex position). Only
// the lowest and the highest point of a grid column can be a strict hull
// vertex, so 64-bit atomics keep per column the bottom and top point; the
// occupied columns, read in x order, give two x-sorted candidate lists
// (lower and upper) without any sort. The chains over these lists are
// computed in windows; windows alternate between two offsets until no window
// removes anything, at which point every consecutive triple turns the right
// way and the lists are the chains themselves.
//
// Every orientation test is exact: coordinate differences are below 2^20, so
// the products are below 2^40 and fp64 holds them and their difference.
#include "ch_internal.hpp"

namespace chk {

__device__ __forceinline__ double cross3(int32_t ax, int32_t ay, int32_t bx, int32_t by, int32_t cx,
                                         int32_t cy) {
  const double t = (double)(by - ay) * (double)(cx - ax);
  return __builtin_fma((double)(bx - ax), (double)(cy - ay), -t);
}

// Block-wide exclusive scan of one value per thread (all threads call it).
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t& total) {
  __shared__ uint32_t s_w[kWaves];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t u = __shfl_up(incl, d);
    if (lane >= d) incl += u;
  }
  if (lane == 63) s_w[w] = incl;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < kWaves; ++i) {
    const uint32_t x = s_w[i];
    if (i < w) off += x;
    tot += x;
  }
  __syncthreads();
  total = tot;
  return off + incl - v;
}

// One monotone chain over `nparts` consecutive parts; part p holds len[p]
// points (1 when len is null) at src[start0 + p*stride ...]. The stack goes to
// dst starting at start0; src may equal dst because the stack never runs
// ahead of the points already read. LOWER keeps strict left turns (the lower
// chain, left to right), otherwise strict right turns (the upper chain, left
// to right). Returns the stack height.
template <bool LOWER>
__device__ int chain_parts(const int32_t* sx, const int32_t* sy, const uint32_t* si, int32_t* dx,
                           int32_t* dy, uint32_t* di, uint32_t start0, uint32_t stride, int nparts,
                           const uint16_t* len) {
  int top = 0;
  int32_t ax = 0, ay = 0, bx = 0, by = 0;  // the two topmost stack points
  for (int p = 0; p < nparts; ++p) {
    const uint32_t pos = start0 + (uint32_t)p * stride;
    const int L = len ? (int)len[p] : 1;
    for (int k = 0; k < L; ++k) {
      const int32_t x = sx[pos + k], y = sy[pos + k];
      const uint32_t id = si[pos + k];
      while (top >= 2) {
        const double cr = cross3(ax, ay, bx, by, x, y);
        if (LOWER ? (cr <= 0.0) : (cr >= 0.0)) {
          --top;
          bx = ax; by = ay;
          if (top >= 2) { ax = dx[start0 + top - 2]; ay = dy[start0 + top - 2]; }
        } else {
          break;
        }
      }
      dx[start0 + top] = x; dy[start0 + top] = y; di[start0 + top] = id;
      ++top;
      ax = bx; ay = by; bx = x; by = y;
    }
  }
  return top;
}

template <int T>
struct HullSmem {
  union {
    uint64_t key[T];                 // sort keys: x<<44 | y<<24 | position
    struct { int32_t ux[T], uy[T]; } u;  // upper chains (after compaction)
  } a;
  union {
    uint32_t pidx[T];                // point index per input position
    uint32_t ui[T];
  } b;
  int32_t px[T], py[T];              // distinct sorted points, then lower chains
  uint32_t pi[T];
  uint16_t n1[kBlock], n2[16];
  uint32_t misc[4];
};

// LDS of the window kernels: one x-sorted window and the chain bookkeeping.
template <int T>
struct WinSmem {
  int32_t px[T], py[T];
  uint32_t pi[T];
  uint16_t n1[kBlock], n2[16];
  uint32_t misc[4];
};

// One side's chain over u x-sorted distinct points in three levels: 256
// segments (one per thread), 16 groups of 16 segments, one group of groups.
// Level 1 reads (sx, sy, si) and writes the segment chains to (dx, dy, di);
// levels 2 and 3 work in place in (dx, dy, di). All threads must call it.
// Returns the chain length; the chain is (dx, dy, di)[0..len).
template <bool LOWER>
__device__ uint32_t chain3(const int32_t* sx, const int32_t* sy, const uint32_t* si, int32_t* dx,
                           int32_t* dy, uint32_t* di, uint32_t u, uint16_t* n1, uint16_t* n2,
                           uint32_t* out) {
  const uint32_t S = (u + kBlock - 1) / kBlock;
  {
    const uint32_t s0 = threadIdx.x * S;
    const uint32_t s1 = s0 + S < u ? s0 + S : u;
    const int len = s1 > s0 ? (int)(s1 - s0) : 0;
    n1[threadIdx.x] = (uint16_t)chain_parts<LOWER>(sx, sy, si, dx, dy, di, s0, 1, len, nullptr);
  }
  __syncthreads();
  if (threadIdx.x < 16) {
    const int g = threadIdx.x;
    n2[g] = (uint16_t)chain_parts<LOWER>(dx, dy, di, dx, dy, di, 16u * g * S, S, 16, &n1[16 * g]);
  }
  __syncthreads();
  if (threadIdx.x == 0) *out = (uint32_t)chain_parts<LOWER>(dx, dy, di, dx, dy, di, 0, 16u * S, 16, n2);
  __syncthreads();
  return *out;
}

// Lower and upper chains of the u distinct sorted points in sm.px/py/pi. On
// return the lower chain is px/py/pi[0..nl) and the upper chain is
// a.u.ux/uy, b.ui[0..nu). The upper chain is built first because the lower
// one overwrites its input.
template <int T>
__device__ void block_chains(HullSmem<T>& sm, uint32_t u, uint32_t& nl, uint32_t& nu) {
  nu = chain3<false>(sm.px, sm.py, sm.pi, sm.a.u.ux, sm.a.u.uy, sm.b.ui, u, sm.n1, sm.n2, &sm.misc[1]);
  nl = chain3<true>(sm.px, sm.py, sm.pi, sm.px, sm.py, sm.pi, u, sm.n1, sm.n2, &sm.misc[0]);
}

// Hull of `cnt` items starting at `base`. MODE 0: items are point indices
// (coordinates gathered from xy); MODE 1: items are records. Returns h; the
// counter-clockwise hull is element k of hull_elem().
template <int T, int MODE>
__device__ uint32_t tile_hull(HullSmem<T>& sm, const float* __restrict__ xy,
                              const uint32_t* __restrict__ in_idx, const Rec* __restrict__ in_rec,
                              uint32_t base, uint32_t cnt, uint32_t& nl, uint32_t& nu) {
  uint32_t P2 = kBlock;
  while (P2 < cnt) P2 <<= 1;
  for (uint32_t i = threadIdx.x; i < P2; i += kBlock) {
    if (i < cnt) {
      int32_t kx, ky;
      uint32_t id;
      if (MODE == 0) {
        id = in_idx[base + i];
        const float2 p = reinterpret_cast<const float2*>(xy)[id];
        kx = (int32_t)(p.x * 1048576.0f);
        ky = (int32_t)(p.y * 1048576.0f);
      } else {
        const Rec r = in_rec[base + i];
        kx = r.x; ky = r.y; id = r.i;
      }
      sm.a.key[i] = ((uint64_t)(uint32_t)kx << 44) | ((uint64_t)(uint32_t)ky << 24) | i;
      sm.b.pidx[i] = id;
    } else {
      sm.a.key[i] = ~0ull;
    }
  }
  __syncthreads();
  // Bitonic sort of P2 keys.
  for (uint32_t k = 2; k <= P2; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < P2 / 2; i += kBlock) {
        const uint32_t a = ((i & ~(j - 1)) << 1) | (i & (j - 1));
        const uint32_t b = a | j;
        const uint64_t ka = sm.a.key[a], kb = sm.a.key[b];
        const bool up = (a & k) == 0;
        if ((ka > kb) == up) { sm.a.key[a] = kb; sm.a.key[b] = ka; }
      }
      __syncthreads();
    }
  }
  // One entry per distinct coordinate, carrying the smallest index.
  const uint32_t E = P2 / kBlock;
  const uint32_t i0 = threadIdx.x * E;
  uint32_t nfirst = 0;
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t i = i0 + e;
    if (i < cnt && (i == 0 || (sm.a.key[i - 1] >> 24) != (sm.a.key[i] >> 24))) ++nfirst;
  }
  uint32_t u;
  uint32_t pos = block_excl_scan(nfirst, u);
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t i = i0 + e;
    if (i < cnt && (i == 0 || (sm.a.key[i - 1] >> 24) != (sm.a.key[i] >> 24))) {
      const uint64_t kk = sm.a.key[i];
      const uint64_t c = kk >> 24;
      uint32_t mi = sm.b.pidx[kk & 0xFFFFFFu];
      for (uint32_t j = i + 1; j < cnt && (sm.a.key[j] >> 24) == c; ++j) {
        const uint32_t o = sm.b.pidx[sm.a.key[j] & 0xFFFFFFu];
        mi = o < mi ? o : mi;
      }
      sm.px[pos] = (int32_t)(kk >> 44);
      sm.py[pos] = (int32_t)((kk >> 24) & 0xFFFFFu);
      sm.pi[pos] = mi;
      ++pos;
    }
  }
  __syncthreads();
  if (u == 0) { nl = nu = 0; return 0; }
  block_chains<T>(sm, u, nl, nu);
  return nl + (nu > 2 ? nu - 2 : 0);
}

// Element k of the counter-clockwise hull: the lower chain, then the upper
// chain backwards without its two end points.
template <int T>
__device__ __forceinline__ Rec hull_elem(const HullSmem<T>& sm, uint32_t k, uint32_t nl, uint32_t nu) {
  Rec r;
  if (k < nl) {
    r.x = sm.px[k]; r.y = sm.py[k]; r.i = sm.pi[k];
  } else {
    const uint32_t j = nu - 2 - (k - nl);
    r.x = sm.a.u.ux[j]; r.y = sm.a.u.uy[j]; r.i = sm.b.ui[j];
  }
  r.pad = 0;
  return r;
}

template <int MODE>
__global__ __launch_bounds__(kBlock) void k_hull_round(const float* __restrict__ xy,
                                                       const uint32_t* __restrict__ in_idx,
                                                       const Rec* __restrict__ in_rec,
                                                       const uint32_t* __restrict__ in_count,
                                                       Rec* __restrict__ out_rec,
                                                       uint32_t* __restrict__ out_count,
                                                       uint32_t* __restrict__ tile_ctr,
                                                       Result* __restrict__ res,
                                                       uint32_t* __restrict__ res_idx,
                                                       const Octagon* __restrict__ oct) {
  __shared__ HullSmem<kHullTile> sm;
  __shared__ uint32_t s_tile, s_base;
  if (oct->status != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) res->status = RES_DOMAIN;
    return;
  }
  const uint32_t c = *in_count;
  if (blockIdx.x == 0 && threadIdx.x == 0) res->cin = c;
  uint32_t nl, nu;
  if (c <= (uint32_t)kHullTile) {
    if (blockIdx.x != 0) return;
    const uint32_t h = tile_hull<kHullTile, MODE>(sm, xy, in_idx, in_rec, 0, c, nl, nu);
    for (uint32_t k = threadIdx.x; k < h; k += kBlock) res_idx[k] = hull_elem(sm, k, nl, nu).i;
    if (threadIdx.x == 0) {
      res->h = h;
      res->status = RES_DONE;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) res->status = RES_MORE;
  const uint32_t ntiles = (c + kHullTile - 1) / kHullTile;
  while (true) {
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint32_t base = tile * kHullTile;
    const uint32_t cnt = c - base < (uint32_t)kHullTile ? c - base : (uint32_t)kHullTile;
    const uint32_t h = tile_hull<kHullTile, MODE>(sm, xy, in_idx, in_rec, base, cnt, nl, nu);
    if (threadIdx.x == 0) s_base = atomicAdd(out_count, h);
    __syncthreads();
    const uint32_t ob = s_base;
    for (uint32_t k = threadIdx.x; k < h; k += kBlock) out_rec[ob + k] = hull_elem(sm, k, nl, nu);
    __syncthreads();
  }
}

// ------------------------------------------------------ large-hull path

__global__ void k_col_init(uint64_t* __restrict__ bot, uint64_t* __restrict__ top) {
  const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t x = g; x < kColumns; x += gridDim.x * blockDim.x) {
    bot[x] = ~0ull;
    top[x] = 0ull;
  }
}

// Per column: bottom = min (y, index), top = max (y, -index). An empty top
// column reads 0 (y is stored plus one).
__global__ void k_col_scatter(const Rec* __restrict__ in, const uint32_t* __restrict__ in_count,
                              uint64_t* __restrict__ bot, uint64_t* __restrict__ top) {
  const uint32_t c = *in_count;
  for (uint32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < c; k += gridDim.x * blockDim.x) {
    const Rec r = in[k];
    atomicMin((unsigned long long*)&bot[r.x], ((unsigned long long)(uint32_t)r.y << 32) | r.i);
    atomicMax((unsigned long long*)&top[r.x],
              ((unsigned long long)(uint32_t)(r.y + 1) << 32) | (0xFFFFFFFFu - r.i));
  }
}

__device__ __forceinline__ Rec bot_rec(uint32_t x, uint64_t b) {
  Rec r;
  r.x = (int32_t)x; r.y = (int32_t)(b >> 32); r.i = (uint32_t)b; r.pad = 0;
  return r;
}
__device__ __forceinline__ Rec top_rec(uint32_t x, uint64_t t) {
  Rec r;
  r.x = (int32_t)x; r.y = (int32_t)(t >> 32) - 1; r.i = 0xFFFFFFFFu - (uint32_t)t; r.pad = 0;
  return r;
}

// Emission rule per occupied column x: lower list gets bottom(x), plus top(x)
// after it when x is the last column and top != bottom; upper list gets
// top(x), preceded by bottom(x) when x is the first column and top != bottom.
// PASS 0 counts per chunk, PASS 1 writes in column order.
template <int PASS>
__global__ __launch_bounds__(kBlock) void k_col_emit(const uint64_t* __restrict__ bot,
                                                     const uint64_t* __restrict__ top,
                                                     uint32_t* __restrict__ cnt,
                                                     Rec* __restrict__ lst_lo,
                                                     Rec* __restrict__ lst_up,
                                                     const Octagon* __restrict__ oct,
                                                     Result* __restrict__ res) {
  constexpr uint32_t PER = kColChunk / kBlock;  // 16 columns per thread
  const uint32_t xmin = (uint32_t)oct->vx[4], xmax = (uint32_t)oct->vx[0];
  const uint32_t x0 = blockIdx.x * kColChunk + threadIdx.x * PER;
  uint32_t nlo = 0, nup = 0;
  for (uint32_t e = 0; e < PER; ++e) {
    const uint32_t x = x0 + e;
    const uint64_t b = bot[x];
    if (b == ~0ull) continue;
    const bool two = (uint32_t)(top[x] >> 32) - 1 != (uint32_t)(b >> 32);
    nlo += 1 + ((x == xmax && two) ? 1 : 0);
    nup += 1 + ((x == xmin && two) ? 1 : 0);
  }
  uint32_t tlo, tup;
  uint32_t olo = block_excl_scan(nlo, tlo);
  uint32_t oup = block_excl_scan(nup, tup);
  if (PASS == 0) {
    if (threadIdx.x == 0) { cnt[2 * blockIdx.x] = tlo; cnt[2 * blockIdx.x + 1] = tup; }
    return;
  }
  __shared__ uint32_t s_base[2];
  if (threadIdx.x < 2) {
    uint32_t s = 0;
    for (uint32_t b = 0; b < blockIdx.x; ++b) s += cnt[2 * b + threadIdx.x];
    s_base[threadIdx.x] = s;
    if (blockIdx.x == gridDim.x - 1) {
      if (threadIdx.x == 0) res->lcount = s + tlo; else res->ucount = s + tup;
    }
  }
  __syncthreads();
  olo += s_base[0];
  oup += s_base[1];
  for (uint32_t e = 0; e < PER; ++e) {
    const uint32_t x = x0 + e;
    const uint64_t b = bot[x];
    if (b == ~0ull) continue;
    const uint64_t t = top[x];
    const bool two = (uint32_t)(t >> 32) - 1 != (uint32_t)(b >> 32);
    lst_lo[olo++] = bot_rec(x, b);
    if (x == xmax && two) lst_lo[olo++] = top_rec(x, t);
    if (x == xmin && two) lst_up[oup++] = bot_rec(x, b);
    lst_up[oup++] = top_rec(x, t);
  }
}

// Chain of one x-sorted, distinct window held in LDS (px/py/pi), in place.
template <int T, bool LOWER>
__device__ uint32_t window_chain(WinSmem<T>& sm, uint32_t u) {
  return chain3<LOWER>(sm.px, sm.py, sm.pi, sm.px, sm.py, sm.pi, u, sm.n1, sm.n2, &sm.misc[0]);
}

constexpr int kWin = 4096;

// One window round over the lower list (blocks [0, nwl)) and the upper list
// (blocks [nwl, nwl + nwu)). Window k covers [k*W - shift, (k+1)*W - shift).
// Its chain is written back at the window's start in dst; its length in wcnt.
__global__ __launch_bounds__(kBlock) void k_window(const Rec* __restrict__ src_lo,
                                                   const Rec* __restrict__ src_up, uint32_t cl,
                                                   uint32_t cu, uint32_t shift, uint32_t nwl,
                                                   Rec* __restrict__ dst_lo,
                                                   Rec* __restrict__ dst_up,
                                                   uint32_t* __restrict__ wcnt_lo,
                                                   uint32_t* __restrict__ wcnt_up) {
  __shared__ WinSmem<kWin> sm;
  const bool lower = blockIdx.x < nwl;
  const uint32_t k = lower ? blockIdx.x : blockIdx.x - nwl;
  const uint32_t c = lower ? cl : cu;
  const Rec* src = lower ? src_lo : src_up;
  Rec* dst = lower ? dst_lo : dst_up;
  const int64_t s = (int64_t)k * kWin - shift;
  const uint32_t lo = s < 0 ? 0u : (uint32_t)s;
  const uint64_t e = (uint64_t)(s + kWin);
  const uint32_t hi = e > c ? c : (uint32_t)e;
  const uint32_t u = hi > lo ? hi - lo : 0;
  for (uint32_t i = threadIdx.x; i < u; i += kBlock) {
    const Rec r = src[lo + i];
    sm.px[i] = r.x; sm.py[i] = r.y; sm.pi[i] = r.i;
  }
  __syncthreads();
  const uint32_t h = lower ? window_chain<kWin, true>(sm, u) : window_chain<kWin, false>(sm, u);
  for (uint32_t i = threadIdx.x; i < h; i += kBlock) {
    Rec r;
    r.x = sm.px[i]; r.y = sm.py[i]; r.i = sm.pi[i]; r.pad = 0;
    dst[lo + i] = r;
  }
  if (threadIdx.x == 0) (lower ? wcnt_lo : wcnt_up)[k] = h;
}

// Concatenate the window chains in order: window k's chain moves to the sum
// of the lengths before it.
__global__ __launch_bounds__(kBlock) void k_window_pack(const Rec* __restrict__ src_lo,
                                                        const Rec* __restrict__ src_up,
                                                        uint32_t shift, uint32_t nwl,
                                                        const uint32_t* __restrict__ wcnt_lo,
                                                        const uint32_t* __restrict__ wcnt_up,
                                                        Rec* __restrict__ dst_lo,
                                                        Rec* __restrict__ dst_up,
                                                        Result* __restrict__ res, uint32_t nwu) {
  __shared__ uint32_t s_off;
  const bool lower = blockIdx.x < nwl;
  const uint32_t k = lower ? blockIdx.x : blockIdx.x - nwl;
  const uint32_t* wc = lower ? wcnt_lo : wcnt_up;
  if (threadIdx.x == 0) {
    uint32_t o = 0;
    for (uint32_t i = 0; i < k; ++i) o += wc[i];
    s_off = o;
    const uint32_t nw = lower ? nwl : nwu;
    if (k == nw - 1) (lower ? res->lcount : res->ucount) = o + wc[k];
  }
  __syncthreads();
  const int64_t s = (int64_t)k * kWin - shift;
  const uint32_t lo = s < 0 ? 0u : (uint32_t)s;
  const uint32_t h = wc[k];
  const Rec* src = lower ? src_lo : src_up;
  Rec* dst = lower ? dst_lo : dst_up;
  for (uint32_t i = threadIdx.x; i < h; i += kBlock) dst[s_off + i] = src[lo + i];
}

// Final output of the large-hull path. When both lists fit one window the
// chains are computed here (single=1); otherwise the lists already are the
// chains. Writes the counter-clockwise hull to res_idx.
__global__ __launch_bounds__(kBlock) void k_large_final(const Rec* __restrict__ lo_lst,
                                                        const Rec* __restrict__ up_lst,
                                                        uint32_t cl, uint32_t cu, int single,
                                                        Result* __restrict__ res,
                                                        uint32_t* __restrict__ res_idx) {
  __shared__ WinSmem<kWin> sm;
  uint32_t nl = cl, nu = cu;
  if (single) {
    for (uint32_t i = threadIdx.x; i < cl; i += kBlock) {
      const Rec r = lo_lst[i];
      sm.px[i] = r.x; sm.py[i] = r.y; sm.pi[i] = r.i;
    }
    __syncthreads();
    nl = window_chain<kWin, true>(sm, cl);
    for (uint32_t i = threadIdx.x; i < nl; i += kBlock) res_idx[i] = sm.pi[i];
    __syncthreads();
    for (uint32_t i = threadIdx.x; i < cu; i += kBlock) {
      const Rec r = up_lst[i];
      sm.px[i] = r.x; sm.py[i] = r.y; sm.pi[i] = r.i;
    }
    __syncthreads();
    nu = window_chain<kWin, false>(sm, cu);
    for (uint32_t k = threadIdx.x; k + 2 < nu; k += kBlock) res_idx[nl + k] = sm.pi[nu - 2 - k];
  } else {
    for (uint32_t i = threadIdx.x; i < nl; i += kBlock) res_idx[i] = lo_lst[i].i;
    for (uint32_t k = threadIdx.x; k + 2 < nu; k += kBlock) res_idx[nl + k] = up_lst[nu - 2 - k].i;
  }
  if (threadIdx.x == 0) {
    res->h = nl + (nu > 2 ? nu - 2 : 0);
    res->status = RES_DONE;
  }
}

// ------------------------------------------------------------- launchers

hipError_t launch_hull_round(int mode, uint32_t grid, const float* xy, const uint32_t* in_idx,
                             const Rec* in_rec, const uint32_t* in_count, Rec* out_rec,
                             uint32_t* out_count, uint32_t* tile_ctr, Result* res,
                             uint32_t* res_idx, const Octagon* oct, hipStream_t st) {
  if (mode == 0)
    hipLaunchKernelGGL(k_hull_round<0>, dim3(grid), dim3(kBlock), 0, st, xy, in_idx, in_rec,
                       in_count, out_rec, out_count, tile_ctr, res, res_idx, oct);
  else
    hipLaunchKernelGGL(k_hull_round<1>, dim3(grid), dim3(kBlock), 0, st, xy, in_idx, in_rec,
                       in_count, out_rec, out_count, tile_ctr, res, res_idx, oct);
  return hipGetLastError();
}

hipError_t launch_col_build(const Rec* in, const uint32_t* in_count, uint32_t max_in,
                            uint64_t* bot, uint64_t* top, uint32_t* cnt, Rec* lst_lo, Rec* lst_up,
                            const Octagon* oct, Result* res, hipStream_t st) {
  hipLaunchKernelGGL(k_col_init, dim3(1024), dim3(kBlock), 0, st, bot, top);
  uint32_t g = (max_in + kBlock - 1) / kBlock;
  if (g < 1) g = 1;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_col_scatter, dim3(g), dim3(kBlock), 0, st, in, in_count, bot, top);
  hipLaunchKernelGGL(k_col_emit<0>, dim3(kColBlocks), dim3(kBlock), 0, st, bot, top, cnt, lst_lo,
                     lst_up, oct, res);
  hipLaunchKernelGGL(k_col_emit<1>, dim3(kColBlocks), dim3(kBlock), 0, st, bot, top, cnt, lst_lo,
                     lst_up, oct, res);
  return hipGetLastError();
}

uint32_t window_count(uint32_t c, uint32_t shift) {
  if (c == 0) return 0;
  return (c + shift + kWin - 1) / kWin;
}

hipError_t launch_window_round(const Rec* src_lo, const Rec* src_up, uint32_t cl, uint32_t cu,
                               uint32_t shift, Rec* tmp_lo, Rec* tmp_up, uint32_t* wcnt_lo,
                               uint32_t* wcnt_up, Rec* dst_lo, Rec* dst_up, Result* res,
                               hipStream_t st) {
  const uint32_t nwl = window_count(cl, shift), nwu = window_count(cu, shift);
  if (nwl + nwu == 0) return hipSuccess;
  hipLaunchKernelGGL(k_window, dim3(nwl + nwu), dim3(kBlock), 0, st, src_lo, src_up, cl, cu, shift,
                     nwl, tmp_lo, tmp_up, wcnt_lo, wcnt_up);
  hipLaunchKernelGGL(k_window_pack, dim3(nwl + nwu), dim3(kBlock), 0, st, tmp_lo, tmp_up, shift,
                     nwl, wcnt_lo, wcnt_up, dst_lo, dst_up, res, nwu);
  return hipGetLastError();
}

hipError_t launch_large_final(const Rec* lo, const Rec* up, uint32_t cl, uint32_t cu, int single,
                              Result* res, uint32_t* res_idx, hipStream_t st) {
  hipLaunchKernelGGL(k_large_final, dim3(1), dim3(kBlock), 0, st, lo, up, cl, cu, single, res,
                     res_idx);
  return hipGetLastError();
}

}  // namespace chk
