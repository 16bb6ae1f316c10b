// Device hull pass over the filter's survivors (Alg. 1's per-queue hull,
// done here on the GPU with Andrew's monotone chain, Table I).
//
// Block hull: a workgroup sorts up to T candidates in LDS by (x, y, position),
// keeps one entry per distinct coordinate (the smallest index), and builds
// the lower and upper chains in parallel: every thread chains its own short
// segment, then log2(256) levels merge neighbouring chains pairwise. A merge
// pops the left chain's tail and the right chain's head exactly as Andrew's
// scan would at the junction (both chains are already convex, so no other
// point can pop), then shifts the right remainder next to the left one.
//
// Main path -- hull of hulls. When there are more candidates than one block
// holds, tiles of kHullTile candidates are reduced to their hulls by many
// workgroups and the union goes round again: CH(S) = CH(union of tile hulls).
//
// Large-hull path -- used when a round stops shrinking the list (a hull with
// more vertices than a block holds, or many points in convex position). Only
// the lowest and the highest point of a grid column can be a strict hull
// vertex, so 64-bit atomics keep per column the bottom and top point; the
// occupied columns, read in x order, give two x-sorted candidate lists
// (lower and upper) without any sort. Their chains are computed in windows
// that alternate between two offsets until no window removes anything; then
// every consecutive triple turns the right way and the lists are the chains.
//
// Every orientation test is exact: coordinate differences are below 2^20, so
// the products are below 2^40 and fp64 holds them and their difference.
#include <cstddef>

#include "ch_device.hpp"

namespace chk {

// Sequential monotone chain of src[s0, s0+len) onto a stack at dst[s0...];
// src may equal dst (the stack never overtakes the read position).
template <bool LOWER>
__device__ int seg_chain(const int32_t* sx, const int32_t* sy, const uint32_t* si, int32_t* dx,
                         int32_t* dy, uint32_t* di, uint32_t s0, int len) {
  int top = 0;
  int32_t ax = 0, ay = 0, bx = 0, by = 0;  // the two topmost stack points
  for (int k = 0; k < len; ++k) {
    const int32_t x = sx[s0 + k], y = sy[s0 + k];
    const uint32_t id = si[s0 + k];
    while (top >= 2 && bad_turn<LOWER>(ax, ay, bx, by, x, y)) {
      --top;
      bx = ax; by = ay;
      if (top >= 2) { ax = dx[s0 + top - 2]; ay = dy[s0 + top - 2]; }
    }
    dx[s0 + top] = x; dy[s0 + top] = y; di[s0 + top] = id;
    ++top;
    ax = bx; ay = by; bx = x; by = y;
  }
  return top;
}

// Exact pre-sieve of an x-sorted list of distinct points before its chain.
// For such a list, p_i is a strict vertex of the lower chain exactly when
// orient(p_a, p_i, p_b) > 0 for every a < i < b (the upper chain mirrors the
// sign), so p_i can go as soon as one pair fails; the chain of what is left
// is the same, since no vertex ever fails a pair. Every inner point tests the
// pairs (i - k, i + k) for a few spreads k (clamped to the list), all points
// at once; the survivors are compacted in place (order kept) and their
// count returned. Whole workgroup; MAXE >= ceil(u / kBlock).
template <bool LOWER, int MAXE>
__device__ uint32_t presieve(int32_t* px, int32_t* py, uint32_t* pi, uint32_t u) {
  if (u <= 64) return u;  // (u is uniform: every thread returns here or none)
  constexpr int kSpreads = 8;
  constexpr uint32_t spread[kSpreads] = {1, 2, 4, 7, 12, 20, 33, 54};
  const uint32_t E = (u + kBlock - 1) / kBlock;
  const uint32_t i0 = threadIdx.x * E;
  int32_t x[MAXE], y[MAXE];
  uint32_t id[MAXE], keep = 0, nk = 0;
#pragma unroll
  for (int e = 0; e < MAXE; ++e) {
    const uint32_t i = i0 + (uint32_t)e;
    if ((uint32_t)e < E && i < u) {
      x[e] = px[i]; y[e] = py[i]; id[e] = pi[i];
      bool k = true;
      if (i > 0 && i + 1 < u) {
#pragma unroll
        for (int s = 0; s < kSpreads; ++s) {
          const uint32_t a = i >= spread[s] ? i - spread[s] : 0u;
          const uint32_t b = i + spread[s] < u ? i + spread[s] : u - 1;
          k &= !bad_turn<LOWER>(px[a], py[a], x[e], y[e], px[b], py[b]);
        }
      }
      if (k) { keep |= 1u << e; ++nk; }
    }
  }
  uint32_t total;
  uint32_t pos = block_excl_scan(nk, total);  // its barriers end every read above
#pragma unroll
  for (int e = 0; e < MAXE; ++e) {
    if (keep & (1u << e)) { px[pos] = x[e]; py[pos] = y[e]; pi[pos] = id[e]; ++pos; }
  }
  __syncthreads();
  return total;
}

// One side's chain of u x-sorted distinct points (src), written to dst[0..len):
// per-thread segment chains, then pairwise merges up a binary tree. MAXC
// bounds the elements one thread moves per merge (ceil(S/2), S = u/256).
// All threads must call it; returns the chain length.
template <bool LOWER, int MAXC>
__device__ uint32_t par_chain(const int32_t* sx, const int32_t* sy, const uint32_t* si, int32_t* dx,
                              int32_t* dy, uint32_t* di, uint32_t u, uint16_t* cnt, int32_t* wij) {
  // Segments of at least kMinSeg points: fewer merge levels for small inputs.
  constexpr uint32_t kMinSeg = 2 * MAXC < 8 ? 2 * MAXC : 8;
  uint32_t S = (u + kBlock - 1) / kBlock;
  if (S < kMinSeg) S = kMinSeg;
  const uint32_t nseg = (u + S - 1) / S;
  const uint32_t t = threadIdx.x;
  {
    const uint32_t s0 = t * S;
    const uint32_t s1 = s0 + S < u ? s0 + S : u;
    cnt[t] = (uint16_t)seg_chain<LOWER>(sx, sy, si, dx, dy, di, s0, s1 > s0 ? (int)(s1 - s0) : 0);
  }
  __syncthreads();
  for (uint32_t half = 1; half < nseg; half <<= 1) {
    const uint32_t npairs = kBlock / (2 * half);
    if (t < npairs) {
      const uint32_t ls = 2 * t * half * S, rs = (2 * t + 1) * half * S;
      const int nl = cnt[2 * t * half], nr = cnt[(2 * t + 1) * half];
      int i = nl - 1, j = 0;
      if (nl > 0 && nr > 0) {
        int32_t a1x = dx[ls + i], a1y = dy[ls + i];
        int32_t a0x = i > 0 ? dx[ls + i - 1] : 0, a0y = i > 0 ? dy[ls + i - 1] : 0;
        int32_t b0x = dx[rs], b0y = dy[rs];
        int32_t b1x = nr > 1 ? dx[rs + 1] : 0, b1y = nr > 1 ? dy[rs + 1] : 0;
        while (true) {
          bool ch = false;
          while (i > 0 && bad_turn<LOWER>(a0x, a0y, a1x, a1y, b0x, b0y)) {
            --i;
            a1x = a0x; a1y = a0y;
            if (i > 0) { a0x = dx[ls + i - 1]; a0y = dy[ls + i - 1]; }
            ch = true;
          }
          while (j + 1 < nr && bad_turn<LOWER>(a1x, a1y, b0x, b0y, b1x, b1y)) {
            ++j;
            b0x = b1x; b0y = b1y;
            if (j + 1 < nr) { b1x = dx[rs + j + 1]; b1y = dy[rs + j + 1]; }
            ch = true;
          }
          if (!ch) break;
        }
      }
      wij[2 * t] = i;
      wij[2 * t + 1] = j;
    }
    __syncthreads();
    const uint32_t tpp = 2 * half;  // threads per pair
    const uint32_t m = t / tpp, tl = t % tpp;
    const uint32_t ls = 2 * m * half * S, rs = (2 * m + 1) * half * S;
    const int nl = cnt[2 * m * half], nr = cnt[(2 * m + 1) * half];
    const int i = wij[2 * m], j = wij[2 * m + 1];
    const int ncopy = (nl > 0 && nr > 0) ? nr - j : 0;
    int32_t vx[MAXC], vy[MAXC];
    uint32_t vi[MAXC];
#pragma unroll
    for (int e = 0; e < MAXC; ++e) {
      const int p = (int)tl + e * (int)tpp;
      if (p < ncopy) { vx[e] = dx[rs + j + p]; vy[e] = dy[rs + j + p]; vi[e] = di[rs + j + p]; }
    }
    __syncthreads();
#pragma unroll
    for (int e = 0; e < MAXC; ++e) {
      const int p = (int)tl + e * (int)tpp;
      if (p < ncopy) { dx[ls + i + 1 + p] = vx[e]; dy[ls + i + 1 + p] = vy[e]; di[ls + i + 1 + p] = vi[e]; }
    }
    if (tl == 0 && nl > 0) cnt[2 * m * half] = (uint16_t)(i + 1 + ncopy);
    __syncthreads();
  }
  return cnt[0];
}

// Lower chain of (px, py, pi)[0..ul) and upper chain of (ux, uy, ui)[0..uu),
// both x-sorted, each built in place: level 0 chains one segment of each side
// per thread; each merge level walks lower pairs on threads [0, 128) and upper
// pairs on threads [128, 256), sharing the barriers.
template <int MAXC>
__device__ void dual_chain(int32_t* px, int32_t* py, uint32_t* pi, uint32_t ul, int32_t* ux,
                           int32_t* uy, uint32_t* ui, uint32_t uu, uint16_t* cnt_l,
                           uint16_t* cnt_u, int32_t* wij_l, int32_t* wij_u, uint32_t& nl,
                           uint32_t& nu) {
  ul = presieve<true, 2 * MAXC>(px, py, pi, ul);
  uu = presieve<false, 2 * MAXC>(ux, uy, ui, uu);
  constexpr uint32_t kMinSeg = 2 * MAXC < 8 ? 2 * MAXC : 8;
  uint32_t SL = (ul + kBlock - 1) / kBlock, SU = (uu + kBlock - 1) / kBlock;
  if (SL < kMinSeg) SL = kMinSeg;
  if (SU < kMinSeg) SU = kMinSeg;
  const uint32_t nseg_l = (ul + SL - 1) / SL, nseg_u = (uu + SU - 1) / SU;
  const uint32_t nseg = nseg_l > nseg_u ? nseg_l : nseg_u;
  const uint32_t t = threadIdx.x;
  {
    uint32_t s0 = t * SL, s1 = s0 + SL < ul ? s0 + SL : ul;
    cnt_l[t] = (uint16_t)seg_chain<true>(px, py, pi, px, py, pi, s0, s1 > s0 ? (int)(s1 - s0) : 0);
    s0 = t * SU;
    s1 = s0 + SU < uu ? s0 + SU : uu;
    cnt_u[t] = (uint16_t)seg_chain<false>(ux, uy, ui, ux, uy, ui, s0, s1 > s0 ? (int)(s1 - s0) : 0);
  }
  __syncthreads();
  for (uint32_t half = 1; half < nseg; half <<= 1) {
    const uint32_t npairs = kBlock / (2 * half);
    {
      const bool lower = t < 128;
      const uint32_t m = lower ? t : t - 128;
      if (m < npairs) {
        int32_t* dx = lower ? px : ux;
        int32_t* dy = lower ? py : uy;
        const uint16_t* cnt = lower ? cnt_l : cnt_u;
        const uint32_t S = lower ? SL : SU;
        const uint32_t ls = 2 * m * half * S, rs = (2 * m + 1) * half * S;
        const int nl2 = cnt[2 * m * half], nr = cnt[(2 * m + 1) * half];
        int i = nl2 - 1, j = 0;
        if (nl2 > 0 && nr > 0) {
          // Two left points and two right points stay in registers.
          int32_t a1x = dx[ls + i], a1y = dy[ls + i];
          int32_t a0x = i > 0 ? dx[ls + i - 1] : 0, a0y = i > 0 ? dy[ls + i - 1] : 0;
          int32_t b0x = dx[rs], b0y = dy[rs];
          int32_t b1x = nr > 1 ? dx[rs + 1] : 0, b1y = nr > 1 ? dy[rs + 1] : 0;
          while (true) {
            bool ch = false;
            while (i > 0 && (lower ? bad_turn<true>(a0x, a0y, a1x, a1y, b0x, b0y)
                                   : bad_turn<false>(a0x, a0y, a1x, a1y, b0x, b0y))) {
              --i;
              a1x = a0x; a1y = a0y;
              if (i > 0) { a0x = dx[ls + i - 1]; a0y = dy[ls + i - 1]; }
              ch = true;
            }
            while (j + 1 < nr && (lower ? bad_turn<true>(a1x, a1y, b0x, b0y, b1x, b1y)
                                        : bad_turn<false>(a1x, a1y, b0x, b0y, b1x, b1y))) {
              ++j;
              b0x = b1x; b0y = b1y;
              if (j + 1 < nr) { b1x = dx[rs + j + 1]; b1y = dy[rs + j + 1]; }
              ch = true;
            }
            if (!ch) break;
          }
        }
        int32_t* wij = lower ? wij_l : wij_u;
        wij[2 * m] = i;
        wij[2 * m + 1] = j;
      }
    }
    __syncthreads();
    const uint32_t tpp = 2 * half;  // threads per pair
    const uint32_t m = t / tpp, tl = t % tpp;
    int ncopy[2], ii[2], nlv[2];
    uint32_t dst0[2];
    int32_t vx[2][MAXC], vy[2][MAXC];
    uint32_t vi[2][MAXC];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const uint16_t* cnt = side == 0 ? cnt_l : cnt_u;
      const int32_t* wij = side == 0 ? wij_l : wij_u;
      const int32_t* dx = side == 0 ? px : ux;
      const int32_t* dy = side == 0 ? py : uy;
      const uint32_t* di = side == 0 ? pi : ui;
      const uint32_t S = side == 0 ? SL : SU;
      const uint32_t ls = 2 * m * half * S, rs = (2 * m + 1) * half * S;
      nlv[side] = cnt[2 * m * half];
      const int nr = cnt[(2 * m + 1) * half];
      ii[side] = wij[2 * m];
      const int jj = wij[2 * m + 1];
      ncopy[side] = (nlv[side] > 0 && nr > 0) ? nr - jj : 0;
      dst0[side] = ls + ii[side] + 1;
#pragma unroll
      for (int e = 0; e < MAXC; ++e) {
        const int p = (int)tl + e * (int)tpp;
        if (p < ncopy[side]) {
          vx[side][e] = dx[rs + jj + p];
          vy[side][e] = dy[rs + jj + p];
          vi[side][e] = di[rs + jj + p];
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      int32_t* dx = side == 0 ? px : ux;
      int32_t* dy = side == 0 ? py : uy;
      uint32_t* di = side == 0 ? pi : ui;
#pragma unroll
      for (int e = 0; e < MAXC; ++e) {
        const int p = (int)tl + e * (int)tpp;
        if (p < ncopy[side]) {
          dx[dst0[side] + p] = vx[side][e]; dy[dst0[side] + p] = vy[side][e]; di[dst0[side] + p] = vi[side][e];
        }
      }
      if (tl == 0 && nlv[side] > 0)
        (side == 0 ? cnt_l : cnt_u)[2 * m * half] = (uint16_t)(ii[side] + 1 + ncopy[side]);
    }
    __syncthreads();
  }
  nl = cnt_l[0];
  nu = cnt_u[0];
}

template <int T>
struct HullSmem {
  union {
    uint64_t key[T];                     // sort keys: x<<44 | y<<24 | position
    struct { int32_t ux[T], uy[T]; } u;  // upper chain (after compaction)
  } a;
  union {
    uint32_t pidx[T];                    // point index per input position
    uint32_t ui[T];
  } b;
  int32_t px[T], py[T];                  // distinct sorted points, then the lower chain
  uint32_t pi[T];
  uint16_t cnt[kBlock], cnt2[kBlock];
  int32_t wij[kBlock], wij2[kBlock];
};

template <int T>
struct WinSmem {
  int32_t px[T], py[T];
  uint32_t pi[T];
  uint16_t cnt[kBlock];
  int32_t wij[kBlock];
};

template <int T>
constexpr int maxc() { return (T / kBlock + 1) / 2; }

// A 64-bit lane move through DPP (all 64 lanes active).
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)v, (int)(uint32_t)v, CTRL, 0xF, 0xF, false);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(v >> 32), (int)(uint32_t)(v >> 32), CTRL,
                                                            0xF, 0xF, false);
  return ((uint64_t)hi << 32) | lo;
}

// One halving step of wave_max16_t: partners (the DPP pattern CTRL) differ in
// lane bit B and hold the same 2H values; the lane with bit B set keeps the
// upper H, its partner the lower H, and each takes the maximum with the half
// the other sends.
template <int CTRL, int B, int H>
__device__ __forceinline__ void max_half(const uint64_t (&in)[2 * H], uint64_t (&out)[H], int lane) {
  const bool up = (lane >> B) & 1;
#pragma unroll
  for (int j = 0; j < H; ++j) {
    const uint64_t keep = up ? in[j + H] : in[j];
    const uint64_t send = up ? in[j] : in[j + H];
    const uint64_t got = dpp_u64<CTRL>(send);
    out[j] = got > keep ? got : keep;
  }
}

// Wave-wide maxima of 16 values per lane, transposed: lane l returns the
// maximum of value l mod 16 over all 64 lanes. Row mirror (bit 3), half-row
// mirror (bit 2) and the two quad swaps (bits 1, 0) pair lanes that hold the
// same values at each step, so one row ends with one value per lane; two
// cross-row exchanges finish. All 64 lanes must be active.
__device__ __forceinline__ uint64_t wave_max16_t(const uint64_t (&b)[16], int lane) {
  uint64_t c8[8], c4[4], c2[2], c1[1];
  max_half<0x140, 3, 8>(b, c8, lane);   // row_mirror
  max_half<0x141, 2, 4>(c8, c4, lane);  // row_half_mirror
  max_half<0x4E, 1, 2>(c4, c2, lane);   // quad_perm [2,3,0,1]
  max_half<0xB1, 0, 1>(c2, c1, lane);   // quad_perm [1,0,3,2]
  uint64_t v = c1[0];
  uint64_t o = __shfl_xor(v, 16);
  v = o > v ? o : v;
  o = __shfl_xor(v, 32);
  return o > v ? o : v;
}

// ------------------------------------------------ small inputs: two waves per chain
//
// When the pre-filter leaves few candidates (at most kSmallChain per chain),
// each chain is built without a sort. For distinct points in (x, y) order, p
// is a strict lower-chain vertex exactly when orient(a, p, b) > 0 for every a
// before p and every b after it: when every slope a -> p is below every slope
// p -> b (a point straight above or below counts as slope +infinity in the
// direction of increasing order); the upper chain mirrors the signs. Each
// point's largest slope to the left and smallest to the right come from one
// pass over the chain. The slopes are quotients of integers below 2^21, so
// two different ones differ by at least 2^-42 of their size, far above an
// fp64 rounding: correctly rounded fp64 quotients keep every strict order and
// every equality, and the comparison of the two bounds is exact. Two waves
// share a chain (each takes half the pairs); equal points keep the smallest
// index; the vertices are placed by rank.
constexpr uint32_t kSmallChain = 128;

// Points per lane of a chain scan (1 or 2), as a compile-time tag.
template <int N>
struct Slots {
  static constexpr int value = N;
};

// Lexicographic minimum and maximum of a 64-bit key over the wave
// (wave-uniform). All 64 lanes must be active.
__device__ __forceinline__ void wave_minmax_u64(uint64_t& mn, uint64_t& mx) {
  mn = wave_allreduce(mn, [](uint64_t a, uint64_t b) { return a < b ? a : b; });
  mx = wave_allreduce(mx, [](uint64_t a, uint64_t b) { return a > b ? a : b; });
}

// Whole workgroup. The `kept` (1..2 kSmallChain) candidates are in sm.a.key
// (x<<44 | y<<24 | position) with their indices in sm.b.pidx. The lower chain
// goes to px/py/pi, the upper chain to a.u / b.ui (both from the
// lexicographic minimum to the maximum, ends included). Waves 0-1 take the
// lower chain, waves 2-3 the upper one. Returns false, with sm untouched,
// when a chain has more than kSmallChain candidates.
template <int T>
__device__ bool small_chains(HullSmem<T>& sm, uint32_t kept, uint32_t& nl, uint32_t& nu) {
  static_assert(kWaves == 4, "two waves per chain");
  static_assert(T >= 4 * kSmallChain, "scratch laid over px / py");
  static_assert(sizeof(sm.cnt) + sizeof(sm.cnt2) + sizeof(sm.wij) + sizeof(sm.wij2) >=
                    2 * kSmallChain * sizeof(uint64_t),
                "chain vertices laid over the merge scratch");
  __shared__ uint32_t s_n[2], s_vc[2][2];
  // Scratch laid over storage that is dead while this runs (fewer bytes of
  // LDS per workgroup, so more workgroups per CU): px / py (written only by
  // the final placement, after every read of the scratch) and the chain
  // builders' merge tables (unused on this path).
  int32_t (*s_x)[kSmallChain] = reinterpret_cast<int32_t (*)[kSmallChain]>(sm.px);
  int32_t (*s_y)[kSmallChain] = reinterpret_cast<int32_t (*)[kSmallChain]>(sm.px + 2 * kSmallChain);
  uint32_t (*s_ui)[kSmallChain] = reinterpret_cast<uint32_t (*)[kSmallChain]>(sm.px + 4 * kSmallChain);
  double (*s_pl)[64] = reinterpret_cast<double (*)[64]>(sm.py);
  double (*s_pr)[64] = reinterpret_cast<double (*)[64]>(sm.py + 256);
  uint32_t (*s_pf)[64] = reinterpret_cast<uint32_t (*)[64]>(sm.py + 512);
  uint64_t (*s_vt)[kSmallChain] = reinterpret_cast<uint64_t (*)[kSmallChain]>(sm.cnt);  // chain vertices (x<<20 | y)
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t lt = (1ull << lane) - 1ull;
  // Waves 0 and 1 select the candidates of the lower / upper chain: the ends
  // (lexicographic minimum and maximum) and the points strictly below /
  // above the line through them.
  uint64_t sel[4] = {0, 0, 0, 0};
  uint64_t kin[4];
  if (w < 2) {
    bool v[4];
    uint64_t mn = ~0ull, mx = 0ull;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      v[e] = (uint32_t)(lane + 64 * e) < kept;
      kin[e] = v[e] ? sm.a.key[lane + 64 * e] : ~0ull;
      mn = kin[e] < mn ? kin[e] : mn;
      mx = v[e] && kin[e] > mx ? kin[e] : mx;
    }
    wave_minmax_u64(mn, mx);
    const int32_t ax = (int32_t)(mn >> 44), ay = (int32_t)((mn >> 24) & 0xFFFFFu);
    const int32_t bx = (int32_t)(mx >> 44), by = (int32_t)((mx >> 24) & 0xFFFFFu);
    uint32_t c = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      bool in = false;
      if (v[e]) {
        const int32_t x = (int32_t)(kin[e] >> 44), y = (int32_t)((kin[e] >> 24) & 0xFFFFFu);
        const double cr = cross3(ax, ay, bx, by, x, y);
        in = (x == ax && y == ay) || (x == bx && y == by) || (w == 0 ? cr < 0.0 : cr > 0.0);
      }
      sel[e] = __builtin_amdgcn_ballot_w64(in);
      c += popc64(sel[e]);
    }
    if (lane == 0) s_n[w] = c;
  }
  __syncthreads();
  if (s_n[0] > kSmallChain || s_n[1] > kSmallChain) return false;
  if (w < 2) {  // compact the chain's candidates (unordered)
    uint32_t base = 0;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      if ((sel[e] >> lane) & 1ull) {
        const uint32_t pos = base + popc64(sel[e] & lt);
        s_x[w][pos] = (int32_t)(kin[e] >> 44);
        s_y[w][pos] = (int32_t)((kin[e] >> 24) & 0xFFFFFu);
        s_ui[w][pos] = sm.b.pidx[kin[e] & 0xFFFFFFu];
      }
      base += popc64(sel[e]);
    }
  }
  __syncthreads();
  // Chain ch = w / 2, half hf = w % 2. Up to 64 points: both halves take
  // point `lane`, each over half of the chain; more: half hf takes point
  // lane + 64 hf over the whole chain.
  const int ch = w >> 1, hf = w & 1;
  const uint32_t c = __builtin_amdgcn_readfirstlane(s_n[ch]);
  const bool split = c <= 64;
  const uint32_t i = split ? (uint32_t)lane : (uint32_t)lane + 64 * hf;
  const uint32_t q0 = split && hf ? (c + 1) / 2 : 0;
  const uint32_t q1 = split && !hf ? (c + 1) / 2 : c;
  const bool has = i < c;
  const int32_t px = has ? s_x[ch][i] : 0, py = has ? s_y[ch][i] : 0;
  const uint32_t pid = has ? s_ui[ch][i] : 0u;
  double lmax = -__builtin_inf(), rmin = __builtin_inf();
  bool dup = false, hl = false, hr = false;
  auto scan = [&](auto up_tag) {
    constexpr bool UP = decltype(up_tag)::value == 1;  // mirrored slopes for the upper chain
#pragma unroll 4
    for (uint32_t q = q0; q < q1; ++q) {
      const int32_t qx = s_x[ch][q], qy = s_y[ch][q];  // one address: an LDS broadcast
      const uint32_t qi = s_ui[ch][q];
      const bool same = (qx == px) & (qy == py);
      const bool left = (qx < px) | ((qx == px) & (qy < py));
      const bool right = !left & !same;
      const int32_t dx = left ? px - qx : qx - px;
      const int32_t dy = left ? py - qy : qy - py;
      const double t = (double)(UP ? -dy : dy) / (double)dx;
      dup |= same & (qi < pid);
      lmax = left && t > lmax ? t : lmax;
      rmin = right && t < rmin ? t : rmin;
      hl |= left;
      hr |= right;
    }
  };
  if (ch == 0) scan(Slots<0>{});
  else scan(Slots<1>{});
  if (split && hf) {
    s_pl[ch][lane] = lmax;
    s_pr[ch][lane] = rmin;
    s_pf[ch][lane] = (dup ? 1u : 0u) | (hl ? 2u : 0u) | (hr ? 4u : 0u);
  }
  __syncthreads();
  bool vert = false;
  if (!(split && hf)) {
    if (split) {
      const double l2 = s_pl[ch][lane], r2 = s_pr[ch][lane];
      const uint32_t f2 = s_pf[ch][lane];
      lmax = l2 > lmax ? l2 : lmax;
      rmin = r2 < rmin ? r2 : rmin;
      dup |= (f2 & 1u) != 0;
      hl |= (f2 & 2u) != 0;
      hr |= (f2 & 4u) != 0;
    }
    vert = has && !dup && (!hl || !hr || lmax < rmin);
  }
  // place the vertices by rank in (x, y) order
  const uint64_t vm = __builtin_amdgcn_ballot_w64(vert);
  if (lane == 0) s_vc[ch][hf] = popc64(vm);
  __syncthreads();
  const uint32_t n0 = s_vc[ch][0], nv = n0 + s_vc[ch][1];
  const uint64_t key = ((uint64_t)(uint32_t)px << 20) | (uint32_t)py;
  if (vert) s_vt[ch][(hf ? n0 : 0u) + popc64(vm & lt)] = key;
  __syncthreads();
  uint32_t rank = 0;
  if (vert)
    for (uint32_t v = 0; v < nv; ++v) rank += s_vt[ch][v] < key;
  // every read of a.key / b.pidx is long done: the upper chain may overwrite them
  if (vert) {
    if (ch == 0) { sm.px[rank] = px; sm.py[rank] = py; sm.pi[rank] = pid; }
    else { sm.a.u.ux[rank] = px; sm.a.u.uy[rank] = py; sm.b.ui[rank] = pid; }
  }
  __syncthreads();
  nl = s_vc[0][0] + s_vc[0][1];
  nu = s_vc[1][0] + s_vc[1][1];
  return true;
}

// Directions of the pre-filter polygon: 16 small-integer vectors in
// counter-clockwise order (0, 22, 45, 68, 90, ... degrees). Dot products with
// grid points stay below 7 * 2^20, exact in int32.
// (Compile-time constants: the products fold into shifts and adds.)
__device__ __forceinline__ constexpr int dir_x(int d) {
  constexpr int8_t v[16] = {1, 5, 1, 2, 0, -2, -1, -5, -1, -5, -1, -2, 0, 2, 1, 5};
  return v[d];
}
__device__ __forceinline__ constexpr int dir_y(int d) {
  constexpr int8_t v[16] = {0, 2, 1, 5, 1, 5, 1, 2, 0, -2, -1, -5, -1, -5, -1, -2};
  return v[d];
}

// Hull of the `cnt` records starting at in_rec[base]. Returns h; the
// counter-clockwise hull is element k of hull_elem().
//
// Before sorting, the candidates are filtered once more by the rule of the
// octagon stage, with a finer polygon: the candidates' own extreme points in
// 16 directions. Every vertex of that polygon is a candidate, so a candidate
// inside it (or on a side without being a vertex) is not a strict hull vertex
// of the candidates and can be dropped.
//
// tile_hull_core expects the `cnt` candidates in sm.px/py/pi (visible to the
// whole workgroup); tile_hull loads them from records first.
template <int T>
__device__ uint32_t tile_hull_core(HullSmem<T>& sm, uint32_t cnt, uint32_t& nl, uint32_t& nu) {
  constexpr uint32_t E = T / kBlock;  // items per thread: i = threadIdx.x + e * kBlock
  // The pre-filter's scratch lies over the sort keys, written only after
  // its last read (the keys follow the compaction scan's barriers).
  static_assert(T >= 256, "pre-filter scratch laid over the keys");
  uint64_t (*s_ext)[16] = reinterpret_cast<uint64_t (*)[16]>(sm.a.key);
  int32_t* s_vx = reinterpret_cast<int32_t*>(sm.a.key + 64);
  int32_t* s_vy = reinterpret_cast<int32_t*>(sm.a.key + 72);
  double* s_ex = reinterpret_cast<double*>(sm.a.key + 80);
  double* s_ney = reinterpret_cast<double*>(sm.a.key + 96);
  double* s_c = reinterpret_cast<double*>(sm.a.key + 112);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // Extreme position per direction: max of (dot, -position) per thread, then
  // per wave (transposed DPP exchange: lane l ends with direction l mod 16),
  // then over the waves.
  {
    uint64_t best[16];
#pragma unroll
    for (int d = 0; d < 16; ++d) best[d] = 0ull;
    for (uint32_t i = threadIdx.x; i < cnt; i += kBlock) {
      const int32_t x = sm.px[i], y = sm.py[i];
#pragma unroll
      for (int d = 0; d < 16; ++d) {
        const int32_t dot = dir_x(d) * x + dir_y(d) * y + (1 << 23);
        const uint64_t key = ((uint64_t)(uint32_t)dot << 32) | (0xFFFFFFFFu - i);
        best[d] = key > best[d] ? key : best[d];
      }
    }
    const uint64_t m = wave_max16_t(best, lane);
    if (lane < 16) s_ext[w][lane] = m;
  }
  __syncthreads();
  // Thread d takes vertices d and d+1 and writes side d as
  // orient(v_d, v_(d+1), p) = ex * py + ney * px + c, exact in fp64 (each
  // product below 2^42, each partial sum below 2^43).
  if (threadIdx.x < 16) {
    const int d = threadIdx.x, d2 = (d + 1) & 15;
    uint64_t b = s_ext[0][d], b2 = s_ext[0][d2];
#pragma unroll
    for (int q = 1; q < kWaves; ++q) {
      b = s_ext[q][d] > b ? s_ext[q][d] : b;
      b2 = s_ext[q][d2] > b2 ? s_ext[q][d2] : b2;
    }
    const uint32_t p = 0xFFFFFFFFu - (uint32_t)b, p2 = 0xFFFFFFFFu - (uint32_t)b2;
    const int32_t ax = cnt ? sm.px[p] : 0, ay = cnt ? sm.py[p] : 0;
    const int32_t bx = cnt ? sm.px[p2] : 0, by = cnt ? sm.py[p2] : 0;
    s_vx[d] = ax;
    s_vy[d] = ay;
    const double ex = (double)(bx - ax), ey = (double)(by - ay);
    s_ex[d] = ex;
    s_ney[d] = -ey;
    s_c[d] = ey * (double)ax - ex * (double)ay;
  }
  __syncthreads();
  // Keep a candidate outside some polygon side, or equal to a vertex. The
  // vertices are wave-uniform (scalar registers): the equality test needs
  // no branch and no LDS read.
  int32_t cvx[16], cvy[16];
#pragma unroll
  for (int d = 0; d < 16; ++d) {
    cvx[d] = __builtin_amdgcn_readfirstlane(s_vx[d]);
    cvy[d] = __builtin_amdgcn_readfirstlane(s_vy[d]);
  }
  // Items go in groups of up to four (independent chains side by side); a
  // group starts only when some item of it exists in the workgroup.
  constexpr uint32_t kG = E < 4 ? E : 4;
  const uint32_t ea = (cnt + kBlock - 1) / kBlock;  // items per thread in use (uniform)
  uint32_t keepmask = 0, nkeep = 0;
#pragma unroll
  for (uint32_t e0 = 0; e0 < E; e0 += kG) {
    if (e0 >= ea) break;
    int32_t x[kG], y[kG];
    double fx[kG], fy[kG], mn[kG];
    bool eq[kG];
#pragma unroll
    for (uint32_t u = 0; u < kG; ++u) {
      const uint32_t i = threadIdx.x + (e0 + u) * kBlock;
      const uint32_t ii = i < cnt ? i : cnt - 1;
      x[u] = sm.px[ii];
      y[u] = sm.py[ii];
      fx[u] = (double)x[u];
      fy[u] = (double)y[u];
      mn[u] = __builtin_inf();
      eq[u] = false;
    }
#pragma unroll
    for (int d = 0; d < 16; ++d) {
      const double ex = s_ex[d], ney = s_ney[d], c = s_c[d];
#pragma unroll
      for (uint32_t u = 0; u < kG; ++u) {
        mn[u] = __builtin_fmin(mn[u], __builtin_fma(ex, fy[u], __builtin_fma(ney, fx[u], c)));
        eq[u] |= (x[u] == cvx[d]) & (y[u] == cvy[d]);
      }
    }
#pragma unroll
    for (uint32_t u = 0; u < kG; ++u) {
      const uint32_t i = threadIdx.x + (e0 + u) * kBlock;
      if (i < cnt && ((mn[u] < 0.0) | eq[u])) { keepmask |= 1u << (e0 + u); ++nkeep; }
    }
  }
  uint32_t kept;
  uint32_t kpos = block_excl_scan(nkeep, kept);
  uint32_t P2 = kBlock;
  while (P2 < kept) P2 <<= 1;
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    if (keepmask & (1u << e)) {
      const uint32_t i = threadIdx.x + e * kBlock;
      sm.a.key[kpos] = ((uint64_t)(uint32_t)sm.px[i] << 44) | ((uint64_t)(uint32_t)sm.py[i] << 24) | kpos;
      sm.b.pidx[kpos] = sm.pi[i];
      ++kpos;
    }
  }
  for (uint32_t i = kept + threadIdx.x; i < P2; i += kBlock) sm.a.key[i] = ~0ull;
  cnt = kept;
  __syncthreads();
  if (kept >= 1 && kept <= 2 * kSmallChain && small_chains<T>(sm, kept, nl, nu)) {
    return nl + (nu > 2 ? nu - 2 : 0);
  }
  bitonic_sort(sm.a.key, P2);
  // One entry per distinct coordinate, carrying the smallest index.
  const uint32_t E2 = P2 / kBlock;
  const uint32_t j0 = threadIdx.x * E2;
  uint32_t nfirst = 0;
  for (uint32_t e = 0; e < E2; ++e) {
    const uint32_t i = j0 + e;
    if (i < cnt && (i == 0 || (sm.a.key[i - 1] >> 24) != (sm.a.key[i] >> 24))) ++nfirst;
  }
  uint32_t u;
  uint32_t pos = block_excl_scan(nfirst, u);
  for (uint32_t e = 0; e < E2; ++e) {
    const uint32_t i = j0 + e;
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
  // Split by the line from the lexicographic minimum to the maximum: a point
  // strictly above it cannot be on the lower chain, one strictly below cannot
  // be on the upper chain (Andrew's chains both run between these two ends).
  // Lower candidates stay in px/py/pi, upper ones move to ux/uy/ui.
  uint32_t ul, uu;
  {
    constexpr uint32_t EM = T / kBlock;
    const uint32_t Eu = (u + kBlock - 1) / kBlock;
    const uint32_t q0 = threadIdx.x * Eu;
    const int32_t x0 = sm.px[0], y0 = sm.py[0], x1 = sm.px[u - 1], y1 = sm.py[u - 1];
    int32_t rx[EM], ry[EM];
    uint32_t ri[EM], side = 0;  // bit 2e: lower candidate, bit 2e+1: upper candidate
    uint32_t nlo = 0, nup = 0;
#pragma unroll
    for (uint32_t e = 0; e < EM; ++e) {
      const uint32_t q = q0 + e;
      if (e < Eu && q < u) {
        rx[e] = sm.px[q]; ry[e] = sm.py[q]; ri[e] = sm.pi[q];
        const double c = cross3(x0, y0, x1, y1, rx[e], ry[e]);
        const bool end = q == 0 || q == u - 1;
        const bool lo = end || c < 0.0, up = end || c > 0.0;
        side |= (lo ? 1u : 0u) << (2 * e);
        side |= (up ? 1u : 0u) << (2 * e + 1);
        nlo += lo; nup += up;
      }
    }
    uint32_t plo = block_excl_scan(nlo, ul);
    uint32_t pup = block_excl_scan(nup, uu);
#pragma unroll
    for (uint32_t e = 0; e < EM; ++e) {
      if (side & (1u << (2 * e))) { sm.px[plo] = rx[e]; sm.py[plo] = ry[e]; sm.pi[plo] = ri[e]; ++plo; }
      if (side & (2u << (2 * e))) { sm.a.u.ux[pup] = rx[e]; sm.a.u.uy[pup] = ry[e]; sm.b.ui[pup] = ri[e]; ++pup; }
    }
    __syncthreads();
  }
  dual_chain<maxc<T>()>(sm.px, sm.py, sm.pi, ul, sm.a.u.ux, sm.a.u.uy, sm.b.ui, uu, sm.cnt,
                        sm.cnt2, sm.wij, sm.wij2, nl, nu);
  return nl + (nu > 2 ? nu - 2 : 0);
}

template <int T>
__device__ uint32_t tile_hull(HullSmem<T>& sm, const Rec* __restrict__ in_rec, uint32_t base,
                              uint32_t cnt, uint32_t& nl, uint32_t& nu) {
  // four loads in flight per thread (clamped to the last record), then the stores
  constexpr uint32_t kLd = 4;
  for (uint32_t i0 = 0; i0 < cnt; i0 += kLd * kBlock) {
    Rec r[kLd];
#pragma unroll
    for (uint32_t u = 0; u < kLd; ++u) {
      const uint32_t i = i0 + u * kBlock + threadIdx.x;
      r[u] = in_rec[base + (i < cnt ? i : cnt - 1)];
    }
#pragma unroll
    for (uint32_t u = 0; u < kLd; ++u) {
      const uint32_t i = i0 + u * kBlock + threadIdx.x;
      if (i < cnt) { sm.px[i] = r[u].x; sm.py[i] = r[u].y; sm.pi[i] = r[u].i; }
    }
  }
  __syncthreads();
  return tile_hull_core<T>(sm, cnt, nl, nu);
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

// The result block for the host, written straight into pinned host memory
// mapped for the device (no copy launch): the device Result with this
// call's status, h and input count.
// The status word goes last, after a system-scope fence of every thread
// (this workgroup's earlier writes to host memory, the hull indices
// included, are visible first): the host may read the block as soon as it
// sees the status change. Whole workgroup.
__device__ void publish_result(const Result* __restrict__ res, Result* __restrict__ host,
                               uint32_t status, uint32_t h, uint32_t cin) {
  constexpr uint32_t kWords = sizeof(Result) / 4;
  constexpr uint32_t kStatus = offsetof(Result, status) / 4;
  for (uint32_t t = threadIdx.x; t < kWords; t += kBlock) {
    if (t == kStatus) continue;
    uint32_t v = reinterpret_cast<const uint32_t*>(res)[t];
    if (t == offsetof(Result, h) / 4) v = h;
    else if (t == offsetof(Result, cin) / 4) v = cin;
    reinterpret_cast<uint32_t*>(host)[t] = v;
  }
  __threadfence_system();
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(&host->status, status, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// One workgroup: the hull of all candidates when they fit (status DONE),
// otherwise status MORE with the candidate count in res->cin. With `host`
// (pinned, device-mapped) the result block and the first `host_n` hull
// indices also go to host memory.
__global__ __launch_bounds__(kBlock) void k_hull_final(const Rec* __restrict__ in_rec,
                                                       const uint32_t* __restrict__ in_count,
                                                       Result* __restrict__ res,
                                                       uint32_t* __restrict__ res_idx,
                                                       const Octagon* __restrict__ oct,
                                                       Result* __restrict__ host,
                                                       uint32_t* __restrict__ host_idx,
                                                       uint32_t host_n) {
  __shared__ HullSmem<kFinalTile> sm;
  if (oct->status != 0) {
    if (threadIdx.x == 0) res->status = RES_DOMAIN;
    if (host) publish_result(res, host, RES_DOMAIN, 0, 0);
    return;
  }
  const uint32_t c = *in_count;
  if (threadIdx.x == 0) res->cin = c;
  if (c > (uint32_t)kFinalTile) {
    if (threadIdx.x == 0) res->status = RES_MORE;
    if (host) publish_result(res, host, RES_MORE, 0, c);
    return;
  }
  uint32_t nl, nu;
  const uint32_t h = tile_hull<kFinalTile>(sm, in_rec, 0, c, nl, nu);
  for (uint32_t k = threadIdx.x; k < h; k += kBlock) {
    const uint32_t v = hull_elem(sm, k, nl, nu).i;
    res_idx[k] = v;
    if (host && k < host_n) host_idx[k] = v;
  }
  if (threadIdx.x == 0) {
    res->h = h;
    res->status = RES_DONE;
  }
  if (host) publish_result(res, host, RES_DONE, h, c);
}

// Many workgroups: tiles of kHullTile candidates to tile hulls, appended to
// out_rec (order between tiles is immaterial: the next round sorts again).
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_hull_round(const Rec* __restrict__ in_rec,
                                                       const uint32_t* __restrict__ in_count,
                                                       Rec* __restrict__ out_rec,
                                                       uint32_t* __restrict__ out_count,
                                                       uint32_t* __restrict__ tile_ctr) {
  __shared__ HullSmem<kHullTile> sm;
  __shared__ uint32_t s_tile, s_base;
  const uint32_t c = *in_count;
  const uint32_t ntiles = (c + kHullTile - 1) / kHullTile;
  uint32_t nl, nu;
  while (true) {
    if (threadIdx.x == 0) s_tile = atomicAdd(tile_ctr, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    if (tile >= ntiles) break;
    const uint32_t base = tile * kHullTile;
    const uint32_t cnt = c - base < (uint32_t)kHullTile ? c - base : (uint32_t)kHullTile;
    const uint32_t h = tile_hull<kHullTile>(sm, in_rec, base, cnt, nl, nu);
    if (threadIdx.x == 0) s_base = atomicAdd(out_count, h);
    __syncthreads();
    const uint32_t ob = s_base;
    for (uint32_t k = threadIdx.x; k < h; k += kBlock) out_rec[ob + k] = hull_elem(sm, k, nl, nu);
    __syncthreads();
  }
}

// ------------------------------------------------------ large-hull path

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

// Large-hull path. Only the lowest and the highest point of a grid column can
// be a strict hull vertex (the lexicographic ends aside), so the records are
// reduced per column and read in x order -- two x-sorted lists, the lower and
// the upper one, with no sort. The records are first partitioned by chunk of
// kChunkCols columns (counts per workgroup in LDS, a scan per chunk, then a
// scatter through LDS cursors); one workgroup per chunk then keeps the bottom
// and top point of each of its columns with LDS atomics and builds the
// chunk's two chains in LDS. No global atomics are involved.
//
// Emission rule per occupied column x: the lower list gets bottom(x), plus
// top(x) after it when x is the last column (xmax) and top != bottom; the
// upper list gets top(x), preceded by bottom(x) when x is the first column
// (xmin) and top != bottom. Andrew's chains run from the lexicographic
// minimum (bottom of xmin) to the maximum (top of xmax).

// Partition slice of workgroup g of G: records [g * per, min((g+1) * per, c)).
__device__ __forceinline__ void part_slice(uint32_t c, uint32_t& a, uint32_t& b) {
  const uint32_t per = (c + gridDim.x - 1) / gridDim.x;
  a = blockIdx.x * per;
  b = a + per < c ? a + per : c;
  if (a > c) a = c;
}

__device__ __forceinline__ uint32_t chunk_of(int32_t x) { return (uint32_t)x / kChunkCols; }

// Counts of the slice's records per chunk: hist[k * G + g].
__global__ __launch_bounds__(kBlock) void k_lg_count(const Rec* __restrict__ in,
                                                     const uint32_t* __restrict__ in_count,
                                                     uint32_t* __restrict__ hist) {
  __shared__ uint32_t s_h[kChunks];
  for (uint32_t k = threadIdx.x; k < kChunks; k += kBlock) s_h[k] = 0;
  __syncthreads();
  uint32_t a, b;
  part_slice(*in_count, a, b);
  constexpr uint32_t kLd = 4;  // loads in flight per thread
  for (uint32_t i0 = a; i0 < b; i0 += kLd * kBlock) {
    int32_t x[kLd];
#pragma unroll
    for (uint32_t v = 0; v < kLd; ++v) {
      const uint32_t i = i0 + v * kBlock + threadIdx.x;
      x[v] = in[i < b ? i : b - 1].x;
    }
#pragma unroll
    for (uint32_t v = 0; v < kLd; ++v)
      if (i0 + v * kBlock + threadIdx.x < b) atomicAdd(&s_h[chunk_of(x[v])], 1u);
  }
  __syncthreads();
  for (uint32_t k = threadIdx.x; k < kChunks; k += kBlock) hist[k * gridDim.x + blockIdx.x] = s_h[k];
}

// One workgroup per chunk k: exclusive scan of hist[k * G .. k * G + G) in
// place, the chunk's total to tot[k].
__global__ __launch_bounds__(kBlock) void k_lg_scan(uint32_t* __restrict__ hist, uint32_t G,
                                                    uint32_t* __restrict__ tot) {
  constexpr uint32_t E = kPartMax / kBlock;
  uint32_t* row = hist + blockIdx.x * G;
  uint32_t v[E], sum = 0;
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t j = threadIdx.x * E + e;
    v[e] = j < G ? row[j] : 0u;
    sum += v[e];
  }
  uint32_t total;
  uint32_t run = block_excl_scan(sum, total);
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    const uint32_t j = threadIdx.x * E + e;
    if (j < G) row[j] = run;
    run += v[e];
  }
  if (threadIdx.x == 0) tot[blockIdx.x] = total;
}

// First record of every chunk: exclusive scan of the chunk totals into s_base.
__device__ __forceinline__ void chunk_bases(const uint32_t* __restrict__ tot, uint32_t* s_base) {
  constexpr uint32_t E = kChunks / kBlock;  // chunks per thread
  static_assert(E * kBlock == kChunks, "whole chunks per thread");
  uint32_t t[E], sum = 0;
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    t[e] = tot[E * threadIdx.x + e];
    sum += t[e];
  }
  uint32_t all;
  uint32_t run = block_excl_scan(sum, all);
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    s_base[E * threadIdx.x + e] = run;
    run += t[e];
  }
  if (threadIdx.x == 0) s_base[kChunks] = all;
  __syncthreads();
}

// The slice's records to their chunk's range (order within a chunk is
// immaterial: the column reduction does not depend on it).
__global__ __launch_bounds__(kBlock) void k_lg_scatter(const Rec* __restrict__ in,
                                                       const uint32_t* __restrict__ in_count,
                                                       const uint32_t* __restrict__ hist,
                                                       const uint32_t* __restrict__ tot,
                                                       Rec* __restrict__ out) {
  __shared__ uint32_t s_cur[kChunks + 1];
  chunk_bases(tot, s_cur);
  for (uint32_t k = threadIdx.x; k < kChunks; k += kBlock) s_cur[k] += hist[k * gridDim.x + blockIdx.x];
  __syncthreads();
  uint32_t a, b;
  part_slice(*in_count, a, b);
  constexpr uint32_t kLd = 4;  // loads in flight per thread
  for (uint32_t i0 = a; i0 < b; i0 += kLd * kBlock) {
    Rec r[kLd];
#pragma unroll
    for (uint32_t v = 0; v < kLd; ++v) {
      const uint32_t i = i0 + v * kBlock + threadIdx.x;
      r[v] = in[i < b ? i : b - 1];
    }
#pragma unroll
    for (uint32_t v = 0; v < kLd; ++v)
      if (i0 + v * kBlock + threadIdx.x < b) out[atomicAdd(&s_cur[chunk_of(r[v].x)], 1u)] = r[v];
  }
}

constexpr uint32_t kChunkList = kChunkCols + 1;  // records of a chunk's list at most
constexpr int kChunkMaxc = ((kChunkList + kBlock - 1) / kBlock + 1) / 2;

struct ChunkSmem {
  union {
    struct { uint64_t bot[kChunkCols], top[kChunkCols]; } t;  // column table
    struct {                                                  // the two lists, then chains
      int32_t lx[kChunkList], ly[kChunkList];
      uint32_t li[kChunkList];
      int32_t ux[kChunkList], uy[kChunkList];
      uint32_t ui[kChunkList];
    } l;
  } u;
  uint16_t cnt_l[kBlock], cnt_u[kBlock];
  int32_t wij_l[kBlock], wij_u[kBlock];
  uint32_t base[kChunks + 1];
};

// One workgroup per chunk: its records' bottom and top per column, the lower
// and upper lists in x order, their chains; chain k of list q goes to
// dst + q * cap + k * kChunkStride, its length to wcnt[q * kChunks + k].
__global__ __launch_bounds__(kBlock) void k_lg_chunk(const Rec* __restrict__ part,
                                                     const uint32_t* __restrict__ tot,
                                                     const Octagon* __restrict__ oct,
                                                     Rec* __restrict__ dst, size_t cap,
                                                     uint32_t* __restrict__ wcnt) {
  __shared__ ChunkSmem sm;
  constexpr uint32_t PER = kChunkCols / kBlock;  // columns per thread
  const uint32_t k = blockIdx.x;
  chunk_bases(tot, sm.base);
  const uint32_t r0 = sm.base[k], r1 = sm.base[k + 1];
  if (r0 == r1) {
    if (threadIdx.x == 0) { wcnt[k] = 0; wcnt[kChunks + k] = 0; }
    return;
  }
  for (uint32_t c = threadIdx.x; c < kChunkCols; c += kBlock) {
    sm.u.t.bot[c] = ~0ull;
    sm.u.t.top[c] = 0ull;
  }
  __syncthreads();
  const int32_t x0 = (int32_t)(k * kChunkCols);
  constexpr uint32_t kLd = 4;  // loads in flight per thread
  for (uint32_t i0 = r0; i0 < r1; i0 += kLd * kBlock) {
    Rec q[kLd];
#pragma unroll
    for (uint32_t v = 0; v < kLd; ++v) {
      const uint32_t i = i0 + v * kBlock + threadIdx.x;
      q[v] = part[i < r1 ? i : r1 - 1];
    }
#pragma unroll
    for (uint32_t v = 0; v < kLd; ++v) {
      if (i0 + v * kBlock + threadIdx.x >= r1) continue;
      const uint32_t c = (uint32_t)(q[v].x - x0);
      atomicMin(&sm.u.t.bot[c], ((unsigned long long)(uint32_t)q[v].y << 32) | q[v].i);
      atomicMax(&sm.u.t.top[c],
                ((unsigned long long)(uint32_t)(q[v].y + 1) << 32) | (0xFFFFFFFFu - q[v].i));
    }
  }
  __syncthreads();
  // Thread t owns columns [PER t, PER (t + 1)): read them, then (the lists
  // overwrite the table) place its list entries.
  const int32_t xmin = oct->vx[4], xmax = oct->vx[0];
  uint64_t cb[PER], ct[PER];
  uint32_t nlo = 0, nup = 0;
#pragma unroll
  for (uint32_t e = 0; e < PER; ++e) {
    const uint32_t c = threadIdx.x * PER + e;
    cb[e] = sm.u.t.bot[c];
    ct[e] = sm.u.t.top[c];
    if (cb[e] == ~0ull) continue;
    const int32_t x = x0 + (int32_t)c;
    const bool two = (uint32_t)(ct[e] >> 32) - 1 != (uint32_t)(cb[e] >> 32);
    nlo += 1 + ((x == xmax && two) ? 1 : 0);
    nup += 1 + ((x == xmin && two) ? 1 : 0);
  }
  uint32_t ul, uu;
  uint32_t olo = block_excl_scan(nlo, ul);
  uint32_t oup = block_excl_scan(nup, uu);  // (its barriers also end the table reads)
#pragma unroll
  for (uint32_t e = 0; e < PER; ++e) {
    if (cb[e] == ~0ull) continue;
    const uint32_t x = (uint32_t)(x0 + (int32_t)(threadIdx.x * PER + e));
    const bool two = (uint32_t)(ct[e] >> 32) - 1 != (uint32_t)(cb[e] >> 32);
    const Rec b = bot_rec(x, cb[e]), t = top_rec(x, ct[e]);
    sm.u.l.lx[olo] = b.x; sm.u.l.ly[olo] = b.y; sm.u.l.li[olo] = b.i; ++olo;
    if ((int32_t)x == xmax && two) { sm.u.l.lx[olo] = t.x; sm.u.l.ly[olo] = t.y; sm.u.l.li[olo] = t.i; ++olo; }
    if ((int32_t)x == xmin && two) { sm.u.l.ux[oup] = b.x; sm.u.l.uy[oup] = b.y; sm.u.l.ui[oup] = b.i; ++oup; }
    sm.u.l.ux[oup] = t.x; sm.u.l.uy[oup] = t.y; sm.u.l.ui[oup] = t.i; ++oup;
  }
  __syncthreads();
  uint32_t nl, nu;
  dual_chain<kChunkMaxc>(sm.u.l.lx, sm.u.l.ly, sm.u.l.li, ul, sm.u.l.ux, sm.u.l.uy, sm.u.l.ui, uu,
                         sm.cnt_l, sm.cnt_u, sm.wij_l, sm.wij_u, nl, nu);
  Rec* dl = dst + (size_t)k * kChunkStride;
  Rec* du = dst + cap + (size_t)k * kChunkStride;
  for (uint32_t i = threadIdx.x; i < nl; i += kBlock) {
    Rec r;
    r.x = sm.u.l.lx[i]; r.y = sm.u.l.ly[i]; r.i = sm.u.l.li[i]; r.pad = 0;
    dl[i] = r;
  }
  for (uint32_t i = threadIdx.x; i < nu; i += kBlock) {
    Rec r;
    r.x = sm.u.l.ux[i]; r.y = sm.u.l.uy[i]; r.i = sm.u.l.ui[i]; r.pad = 0;
    du[i] = r;
  }
  if (threadIdx.x == 0) { wcnt[k] = nl; wcnt[kChunks + k] = nu; }
}

// Concatenate the pieces of both lists in order (grid 2 x nper): piece k of
// list q (cnt[q * nper + k] records at src + q * cap + k * stride) moves to
// the sum of the piece lengths before it; the last piece records the
// packed length in pack[q].
__global__ __launch_bounds__(kBlock) void k_lg_pack(const Rec* __restrict__ src,
                                                    Rec* __restrict__ dst, size_t cap,
                                                    size_t stride, uint32_t nper,
                                                    const uint32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ pack) {
  const uint32_t q = blockIdx.x / nper, k = blockIdx.x % nper;
  const uint32_t* wc = cnt + q * nper;
  uint32_t part = 0;
  for (uint32_t i = threadIdx.x; i < k; i += kBlock) part += wc[i];
  uint32_t off;
  block_excl_scan(part, off);
  const uint32_t h = wc[k];
  if (threadIdx.x == 0 && k == nper - 1) pack[q] = off + h;
  const Rec* s = src + q * cap + (size_t)k * stride;
  Rec* d = dst + q * cap;
  for (uint32_t i = threadIdx.x; i < h; i += kBlock) d[off + i] = s[i];
}

constexpr int kWin = 4096;
// Windows per column list (a list holds at most kColumns + 2 records).
constexpr uint32_t kWinPerList = (kColumns + 2 + kWin - 1) / kWin;

template <bool LOWER>
__device__ uint32_t window_chain(WinSmem<kWin>& sm, uint32_t u) {
  return par_chain<LOWER, maxc<kWin>()>(sm.px, sm.py, sm.pi, sm.px, sm.py, sm.pi, u, sm.cnt, sm.wij);
}

// Window chains of NL x-sorted lists (list q holds len[q] records from
// src + q * cap + begin[q]; begin may be null for 0; bit q of lower_mask
// selects its lower chain, else the upper one). Workgroup b takes window
// b % kWinPerList of list b / kWinPerList; past its list's end it returns at
// once. Window k covers [k*kWin, (k+1)*kWin); its chain goes to the window's
// start in dst + q * cap, its length to wcnt[b].
__global__ __launch_bounds__(kBlock) void k_window(const Rec* __restrict__ src,
                                                   Rec* __restrict__ dst, size_t cap,
                                                   const uint32_t* __restrict__ begin,
                                                   const uint32_t* __restrict__ len,
                                                   uint32_t lower_mask,
                                                   uint32_t* __restrict__ wcnt) {
  __shared__ WinSmem<kWin> sm;
  const uint32_t q = blockIdx.x / kWinPerList, k = blockIdx.x % kWinPerList;
  const bool lower = (lower_mask >> q) & 1u;
  const uint32_t c = len[q];
  const uint32_t lo = k * (uint32_t)kWin;
  if (lo >= c) return;
  const uint32_t u = c - lo < (uint32_t)kWin ? c - lo : (uint32_t)kWin;
  const Rec* s = src + q * cap + (begin ? begin[q] : 0u) + lo;
  Rec* d = dst + q * cap + lo;
  for (uint32_t i = threadIdx.x; i < u; i += kBlock) {
    const Rec r = s[i];
    sm.px[i] = r.x; sm.py[i] = r.y; sm.pi[i] = r.i;
  }
  __syncthreads();
  const uint32_t h = lower ? window_chain<true>(sm, u) : window_chain<false>(sm, u);
  for (uint32_t i = threadIdx.x; i < h; i += kBlock) {
    Rec r;
    r.x = sm.px[i]; r.y = sm.py[i]; r.i = sm.pi[i]; r.pad = 0;
    d[i] = r;
  }
  if (threadIdx.x == 0) wcnt[blockIdx.x] = h;
}

// Concatenate the window chains of each list in order (same grid as
// k_window): window k's chain moves to the sum of the chain lengths before
// it; the last window of list q records the packed length in pack[q].
__global__ __launch_bounds__(kBlock) void k_window_pack(const Rec* __restrict__ src,
                                                        Rec* __restrict__ dst, size_t cap,
                                                        const uint32_t* __restrict__ len,
                                                        const uint32_t* __restrict__ wcnt,
                                                        uint32_t* __restrict__ pack) {
  const uint32_t q = blockIdx.x / kWinPerList, k = blockIdx.x % kWinPerList;
  const uint32_t c = len[q];
  const uint32_t lo = k * (uint32_t)kWin;
  if (lo >= c) return;
  const uint32_t* wc = wcnt + q * kWinPerList;
  uint32_t part = 0;
  for (uint32_t i = threadIdx.x; i < k; i += kBlock) part += wc[i];
  uint32_t off;
  block_excl_scan(part, off);
  const uint32_t h = wc[k];
  if (threadIdx.x == 0 && c - lo <= (uint32_t)kWin) pack[q] = off + h;
  const Rec* s = src + q * cap + lo;
  Rec* d = dst + q * cap;
  for (uint32_t i = threadIdx.x; i < h; i += kBlock) d[off + i] = s[i];
}

// ------------------------------------------------ the chain of a long list
//
// One workgroup computes Andrew's chain (the lower one for LOWER, else the
// upper one) of the m records in[0..m), sorted by (x, y) with distinct
// coordinates, as a stack in out[0..r), and returns r. The list is read in
// batches of up to kWin records; each batch is chained in LDS (par_chain),
// then joined to the stack: wave 0 walks from the junction, popping the
// stack's tail and the batch chain's head exactly as Andrew's scan pops when
// it reaches the batch (both sides are chains already, so only their ends
// can pop), 64 candidate positions per step; the rest of the batch chain is
// appended. out may equal in: the stack never holds more records than have
// been read.
template <bool LOWER>
__device__ uint32_t fold_chain(WinSmem<kWin>& sm, const Rec* in, uint32_t m, Rec* out) {
  __shared__ uint32_t s_keep, s_from;
  const int lane = threadIdx.x & 63;
  uint32_t r = 0;
  for (uint32_t pos = 0; pos < m; pos += kWin) {
    const uint32_t t = m - pos < (uint32_t)kWin ? m - pos : (uint32_t)kWin;
    __syncthreads();  // the previous batch is appended; sm is free
    for (uint32_t i = threadIdx.x; i < t; i += kBlock) {
      const Rec q = in[pos + i];
      sm.px[i] = q.x; sm.py[i] = q.y; sm.pi[i] = q.i;
    }
    __syncthreads();
    const uint32_t nc = window_chain<LOWER>(sm, t);
    if (threadIdx.x < 64) {
      int i = (int)r - 1;  // stack top
      uint32_t j = 0;      // head of the batch chain
      if (r > 0) {
        bool moved = true;
        while (moved) {
          moved = false;
          // Pop the stack's top while it does not turn the right way
          // towards the batch chain's head (stack positions i, i-1, ...).
          const int32_t cx = sm.px[j], cy = sm.py[j];
          while (i >= 1) {
            const int q = i - lane;
            bool good = true;  // position 0 is never popped
            if (q >= 1) {
              const Rec a = out[q - 1], b = out[q];
              good = !bad_turn<LOWER>(a.x, a.y, b.x, b.y, cx, cy);
            }
            const uint64_t gm = __ballot(good);
            if (gm) {
              const int f = __builtin_ctzll(gm);
              if (f) { i -= f; moved = true; }
              break;
            }
            i -= 64;
            moved = true;
          }
          // Pop the batch chain's head while the stack top, it and its
          // successor do not turn the right way.
          const Rec s = out[i];
          while (j + 1 < nc) {
            const uint32_t q = j + (uint32_t)lane;
            bool good = true;  // the batch chain's last point is never popped
            if (q + 1 < nc) good = !bad_turn<LOWER>(s.x, s.y, sm.px[q], sm.py[q], sm.px[q + 1], sm.py[q + 1]);
            const uint64_t gm = __ballot(good);
            if (gm) {
              const int f = __builtin_ctzll(gm);
              if (f) { j += (uint32_t)f; moved = true; }
              break;
            }
            j += 64;
            moved = true;
          }
        }
      }
      if (lane == 0) { s_keep = (uint32_t)(i + 1); s_from = j; }
    }
    __syncthreads();
    const uint32_t keep = s_keep, from = s_from;
    for (uint32_t k = threadIdx.x; from + k < nc; k += kBlock) {
      Rec q;
      q.x = sm.px[from + k]; q.y = sm.py[from + k]; q.i = sm.pi[from + k]; q.pad = 0;
      out[keep + k] = q;
    }
    r = keep + (nc - from);
  }
  __syncthreads();
  return r;
}

// One workgroup per list: the chain of packed list q (pack[q] records at
// lists + q * cap; lower when bit q of lower_mask is set), in place; its
// length to fold[q].
__global__ __launch_bounds__(kBlock) void k_fold(Rec* __restrict__ lists, size_t cap,
                                                 const uint32_t* __restrict__ pack,
                                                 uint32_t lower_mask, uint32_t* __restrict__ fold) {
  __shared__ WinSmem<kWin> sm;
  const uint32_t q = blockIdx.x;
  Rec* l = lists + q * cap;
  const uint32_t m = pack[q];
  const uint32_t r = ((lower_mask >> q) & 1u) ? fold_chain<true>(sm, l, m, l)
                                               : fold_chain<false>(sm, l, m, l);
  if (threadIdx.x == 0) fold[q] = r;
}

// Groups of kGroupChunks consecutive chunk chains of both lists (grid 2 x
// kGroups): up to kWin records are chained together in LDS (the chain of
// x-ordered pieces is the chain of all their points, and each piece already
// holds every vertex of its own range), so the fold sees few records; a
// larger group is passed on unchanged. Group g of list q goes to
// dst + q * cap + g * kGroupStride, its length to gcnt[q * kGroups + g].
__global__ __launch_bounds__(kBlock) void k_lg_group(const Rec* __restrict__ src,
                                                     Rec* __restrict__ dst, size_t cap,
                                                     const uint32_t* __restrict__ wcnt,
                                                     uint32_t* __restrict__ gcnt) {
  __shared__ WinSmem<kWin> sm;
  __shared__ uint32_t s_off[kGroupChunks + 1];
  const uint32_t q = blockIdx.x / kGroups, g = blockIdx.x % kGroups;
  const uint32_t* wl = wcnt + q * kChunks;
  const uint32_t* wc = wl + g * kGroupChunks;
  if (threadIdx.x == 0) {
    uint32_t o = 0;
    for (uint32_t j = 0; j < kGroupChunks; ++j) {
      s_off[j] = o;
      o += wc[j];
    }
    s_off[kGroupChunks] = o;
  }
  // The whole list's length: a list the fold takes in one batch anyway is
  // passed on unchanged.
  uint32_t part = 0;
  for (uint32_t k = threadIdx.x; k < kChunks; k += kBlock) part += wl[k];
  uint32_t list_len;
  block_excl_scan(part, list_len);  // (its barriers also publish s_off)
  const uint32_t total = s_off[kGroupChunks];
  const Rec* sg = src + q * cap + (size_t)(g * kGroupChunks) * kChunkStride;
  Rec* d = dst + q * cap + (size_t)g * kGroupStride;
  if (total > (uint32_t)kWin || list_len <= (uint32_t)kWin) {
    for (uint32_t j = 0; j < kGroupChunks; ++j) {
      const uint32_t c = s_off[j + 1] - s_off[j];
      for (uint32_t i = threadIdx.x; i < c; i += kBlock) d[s_off[j] + i] = sg[(size_t)j * kChunkStride + i];
    }
    if (threadIdx.x == 0) gcnt[q * kGroups + g] = total;
    return;
  }
  for (uint32_t j = 0; j < kGroupChunks; ++j) {
    const uint32_t c = s_off[j + 1] - s_off[j];
    for (uint32_t i = threadIdx.x; i < c; i += kBlock) {
      const Rec r = sg[(size_t)j * kChunkStride + i];
      sm.px[s_off[j] + i] = r.x; sm.py[s_off[j] + i] = r.y; sm.pi[s_off[j] + i] = r.i;
    }
  }
  __syncthreads();
  const uint32_t h = q == 0 ? window_chain<true>(sm, total) : window_chain<false>(sm, total);
  for (uint32_t i = threadIdx.x; i < h; i += kBlock) {
    Rec r;
    r.x = sm.px[i]; r.y = sm.py[i]; r.i = sm.pi[i]; r.pad = 0;
    d[i] = r;
  }
  if (threadIdx.x == 0) gcnt[q * kGroups + g] = h;
}

// Window chains, packing and one fold per list, for NL lists as k_window
// describes them: the chains end up packed at the start of each list of A.
hipError_t launch_list_chains(int NL, Rec* A, Rec* B, size_t cap, const uint32_t* begin,
                              const uint32_t* len, uint32_t lower_mask, uint32_t* wcnt,
                              uint32_t* pack, uint32_t* fold, hipStream_t st, LaunchHook* hk) {
  hooked(hk, "lg_window", [&] {
    hipLaunchKernelGGL(k_window, dim3(NL * kWinPerList), dim3(kBlock), 0, st, A, B, cap, begin, len,
                       lower_mask, wcnt);
  });
  hooked(hk, "lg_window_pack", [&] {
    hipLaunchKernelGGL(k_window_pack, dim3(NL * kWinPerList), dim3(kBlock), 0, st, B, A, cap, len,
                       wcnt, pack);
  });
  hooked(hk, "lg_fold", [&] {
    hipLaunchKernelGGL(k_fold, dim3(NL), dim3(kBlock), 0, st, A, cap, pack, lower_mask, fold);
  });
  return hipGetLastError();
}

// Final output of the large-hull path: the counter-clockwise hull (the lower
// chain, then the upper chain backwards without its end points) to res_idx,
// status and h to the result block; with `host` (pinned, device-mapped) the
// result block and the first host_n indices also go to host memory.
__global__ __launch_bounds__(kBlock) void k_large_out(const Rec* __restrict__ lo,
                                                      const Rec* __restrict__ up,
                                                      Result* __restrict__ res,
                                                      uint32_t* __restrict__ res_idx,
                                                      Result* __restrict__ host,
                                                      uint32_t* __restrict__ host_idx,
                                                      uint32_t host_n) {
  const uint32_t nl = res->fold_cnt[0], nu = res->fold_cnt[1], cin = res->cin;
  const uint32_t h = nl + (nu > 2 ? nu - 2 : 0);
  // Every workgroup writes its share of the indices (the writes to host
  // memory are latency-bound); workgroup 0 the result block. The host reads
  // them after the kernel has completed.
  for (uint32_t k = blockIdx.x * kBlock + threadIdx.x; k < h; k += gridDim.x * kBlock) {
    const uint32_t v = k < nl ? lo[k].i : up[nu - 2 - (k - nl)].i;
    res_idx[k] = v;
    if (host && k < host_n) host_idx[k] = v;
  }
  if (blockIdx.x != 0) return;
  if (threadIdx.x == 0) {
    res->h = h;
    res->status = RES_DONE;
  }
  if (host) publish_result(res, host, RES_DONE, h, cin);
}

// ------------------------------------- batch: sets with many candidates left
//
// A set whose candidates did not shrink to one workgroup within the tile-hull
// rounds (thousands of points in convex position, or close to a smooth curve)
// gets its hull from one workgroup here, by the column rule of the large-hull
// path: only the lowest and the highest candidate of a grid column can be a
// strict hull vertex. The set's columns [xmin, xmax] are taken in chunks of
// kLdsCols: the candidates are bucketed by chunk (a counting sort into the
// set's free record slice), each chunk's bottom and top per column come from
// LDS atomics and are emitted in column order -- the x-sorted lower and upper
// lists, written over consumed input -- and both chains are folded.
constexpr uint32_t kLdsCols = 4096;
constexpr uint32_t kLdsChunksMax = kColumns / kLdsCols;

struct BigSmem {
  union {
    struct {
      uint64_t bot[kLdsCols], top[kLdsCols];
    } col;
    WinSmem<kWin> win;
  } u;
  uint32_t start[kLdsChunksMax];  // first bucketed record of each chunk
  uint32_t cur[kLdsChunksMax];    // scatter cursors (counts first)
};

// The hull of the c candidate records X[0..c) (set-local indices, columns
// within [xmin, xmax]), using Y[0..c) as scratch; writes the counter-
// clockwise hull to hull_out and returns h. Whole workgroup; X and Y are
// overwritten.
__device__ uint32_t big_set_hull(BigSmem& sm, Rec* X, Rec* Y, uint32_t c, int32_t xmin,
                                 int32_t xmax, uint32_t* __restrict__ hull_out) {
  const uint32_t nch = ((uint32_t)(xmax - xmin) / kLdsCols) + 1;
  for (uint32_t k = threadIdx.x; k < nch; k += kBlock) sm.cur[k] = 0;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < c; i += kBlock)
    atomicAdd(&sm.cur[(uint32_t)(X[i].x - xmin) / kLdsCols], 1u);
  __syncthreads();
  {
    const uint32_t v = threadIdx.x < nch ? sm.cur[threadIdx.x] : 0u;
    uint32_t tot;
    const uint32_t st = block_excl_scan(v, tot);
    if (threadIdx.x < nch) { sm.start[threadIdx.x] = st; sm.cur[threadIdx.x] = st; }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < c; i += kBlock) {
    const Rec q = X[i];
    const uint32_t p = atomicAdd(&sm.cur[(uint32_t)(q.x - xmin) / kLdsCols], 1u);
    Y[p] = q;
  }
  __syncthreads();
  constexpr uint32_t PER = kLdsCols / kBlock;
  uint32_t nlo = 0, nup = 0;
  for (uint32_t k = 0; k < nch; ++k) {
    const uint32_t b0 = sm.start[k], b1 = k + 1 < nch ? sm.start[k + 1] : c;
    if (b0 == b1) continue;
    for (uint32_t i = threadIdx.x; i < kLdsCols; i += kBlock) {
      sm.u.col.bot[i] = ~0ull;
      sm.u.col.top[i] = 0ull;
    }
    __syncthreads();
    const int32_t x0 = xmin + (int32_t)(k * kLdsCols);
    for (uint32_t i = b0 + threadIdx.x; i < b1; i += kBlock) {
      const Rec q = Y[i];
      const uint32_t cc = (uint32_t)(q.x - x0);
      atomicMin(&sm.u.col.bot[cc], ((unsigned long long)(uint32_t)q.y << 32) | q.i);
      atomicMax(&sm.u.col.top[cc],
                ((unsigned long long)(uint32_t)(q.y + 1) << 32) | (0xFFFFFFFFu - q.i));
    }
    __syncthreads();
    // Emission in column order: thread t owns columns [PER*t, PER*(t+1)).
    uint32_t clo = 0, cup = 0;
    for (uint32_t e = 0; e < PER; ++e) {
      const uint32_t cc = threadIdx.x * PER + e;
      const uint64_t b = sm.u.col.bot[cc];
      if (b == ~0ull) continue;
      const int32_t x = x0 + (int32_t)cc;
      const bool two = (uint32_t)(sm.u.col.top[cc] >> 32) - 1 != (uint32_t)(b >> 32);
      clo += 1 + ((x == xmax && two) ? 1 : 0);
      cup += 1 + ((x == xmin && two) ? 1 : 0);
    }
    uint32_t tlo, tup;
    uint32_t olo = nlo + block_excl_scan(clo, tlo);
    uint32_t oup = nup + block_excl_scan(cup, tup);
    for (uint32_t e = 0; e < PER; ++e) {
      const uint32_t cc = threadIdx.x * PER + e;
      const uint64_t b = sm.u.col.bot[cc];
      if (b == ~0ull) continue;
      const uint64_t t = sm.u.col.top[cc];
      const uint32_t x = (uint32_t)(x0 + (int32_t)cc);
      const bool two = (uint32_t)(t >> 32) - 1 != (uint32_t)(b >> 32);
      Y[olo++] = bot_rec(x, b);
      if ((int32_t)x == xmax && two) Y[olo++] = top_rec(x, t);
      if ((int32_t)x == xmin && two) X[oup++] = bot_rec(x, b);
      X[oup++] = top_rec(x, t);
    }
    nlo += tlo;
    nup += tup;
    __syncthreads();
  }
  const uint32_t nl = fold_chain<true>(sm.u.win, Y, nlo, Y);
  for (uint32_t k = threadIdx.x; k < nl; k += kBlock) hull_out[k] = Y[k].i;
  const uint32_t nu = fold_chain<false>(sm.u.win, X, nup, X);
  for (uint32_t k = threadIdx.x; k + 2 < nu; k += kBlock) hull_out[nl + k] = X[nu - 2 - k].i;
  return nl + (nu > 2 ? nu - 2 : 0);
}

// ------------------------------------------------------------- batch mode

// The first block-hull list: every set, those with the most survivors of
// the candidates' test first (buckets of more than 1024, 257-1024, 65-256
// and at most 64, each in set order), so that the longest block hulls start
// first. Workgroup b ranks sets b kBlock .. b kBlock + kBlock - 1 after
// counting every set's bucket (a strided pass over the set states, from L2).
__global__ __launch_bounds__(kBlock) void k_batch_final_plan(uint32_t nsets,
                                                             BatchHdr* __restrict__ bh,
                                                             const SetState* __restrict__ sets,
                                                             uint32_t* __restrict__ order) {
  constexpr int kVals = 8;  // 4 buckets before this workgroup's sets, 4 in all
  __shared__ uint32_t s_red[kWaves][kVals];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t first = blockIdx.x * kBlock;
  auto bucket = [&](uint32_t s) {
    const uint32_t c = sets[s].cnt[0];
    return c > 1024 ? 0u : (c > 256 ? 1u : (c > 64 ? 2u : 3u));
  };
  uint32_t v[kVals] = {};
  for (uint32_t s = threadIdx.x; s < nsets; s += kBlock) {
    const uint32_t b = bucket(s);
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t hit = b == k ? 1u : 0u;
      v[4 + k] += hit;
      v[k] += s < first ? hit : 0u;
    }
  }
#pragma unroll
  for (int k = 0; k < kVals; ++k) {
    const uint32_t r = wave_allreduce(v[k], [](uint32_t a, uint32_t b) { return a + b; });
    if (lane == 0) s_red[w][k] = r;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < kVals; ++k) {
    v[k] = 0;
#pragma unroll
    for (int q = 0; q < kWaves; ++q) v[k] += s_red[q][k];
  }
  const uint32_t s = first + threadIdx.x;
  const bool own = s < nsets;
  const uint32_t b = own ? bucket(s) : 4u;
  uint32_t unused;
  const uint32_t e01 = block_excl_scan(own && b < 2 ? 1u << (16 * b) : 0u, unused);
  const uint32_t e23 = block_excl_scan(own && b >= 2 && b < 4 ? 1u << (16 * (b - 2)) : 0u, unused);
  if (own) {
    const uint32_t rank = ((b < 2 ? e01 : e23) >> (16 * (b & 1))) & 0xFFFFu;
    uint32_t start = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) start += j < b ? v[4 + j] : (j == b ? v[j] : 0u);
    order[start + rank] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) bh->final_next = 0;
}

// Hull of every set whose candidates fit one block (<= T); a set still above
// that waits for the next tile-hull round (or, after the last one, for
// k_batch_large). With `order` the workgroups take the sets of that list
// through a shared counter (the first stage), else with a fixed stride.
template <int T>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_batch_final(const uint64_t* __restrict__ off,
                                                        uint32_t nsets,
                                                        BatchHdr* __restrict__ bh,
                                                        SetState* __restrict__ sets, int stage,
                                                        const Rec* __restrict__ recs,
                                                        uint32_t* __restrict__ hull_idx,
                                                        uint32_t* __restrict__ hull_count,
                                                        const uint32_t* __restrict__ order) {
  __shared__ HullSmem<T> sm;
  __shared__ uint32_t s_item;
  const bool bad_off = bh->bad_offsets != 0;
  for (uint32_t it = blockIdx.x;; it += gridDim.x) {
    uint32_t s = it;
    if (order) {
      __syncthreads();  // every thread has read s_item
      if (threadIdx.x == 0) s_item = atomicAdd(&bh->final_next, 1u);
      __syncthreads();
      s = s_item < nsets ? order[s_item] : nsets;
    }
    if (s >= nsets) break;
    SetState& ss = sets[s];
    if (ss.done) continue;
    if (bad_off) {
      if (threadIdx.x == 0) { hull_count[s] = kCountInvalid; ss.done = 1; }
      continue;
    }
    const uint32_t a = (uint32_t)off[s];
    const uint32_t n = (uint32_t)(off[s + 1] - off[s]);
    if (n == 0 || ss.oct.status != 0) {
      if (threadIdx.x == 0) { hull_count[s] = n == 0 ? 0u : kCountDomain; ss.done = 1; }
      continue;
    }
    const uint32_t c = ss.cnt[stage];
    if (c > (uint32_t)T) continue;
    uint32_t nl, nu;
    const uint32_t h = tile_hull<T>(sm, recs + a, 0, c, nl, nu);
    for (uint32_t k = threadIdx.x; k < h; k += kBlock) hull_idx[a + k] = hull_elem(sm, k, nl, nu).i;
    if (threadIdx.x == 0) { hull_count[s] = h; ss.done = 1; }
    __syncthreads();
  }
}

// Tiles of kHullTile candidates for every unfinished set, in set order.
// Workgroup b owns sets b kBlock .. b kBlock + kBlock - 1, one per thread;
// every workgroup first counts the tiles of all sets (a strided pass over
// the set states, from L2) for the first tile of its own and the round's
// total.
__global__ __launch_bounds__(kBlock) void k_batch_round_plan(const uint64_t* __restrict__ off,
                                                             uint32_t nsets,
                                                             BatchHdr* __restrict__ bh,
                                                             SetState* __restrict__ sets,
                                                             int stage,
                                                             SetTile* __restrict__ rtiles) {
  __shared__ uint32_t s_red[kWaves][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t first = blockIdx.x * kBlock;
  auto tiles_of = [](uint32_t c) { return c / kHullTile + (c % kHullTile ? 1u : 0u); };
  uint32_t before = 0, all = 0;
  for (uint32_t s = threadIdx.x; s < nsets; s += kBlock) {
    const uint32_t t = sets[s].done ? 0u : tiles_of(sets[s].cnt[stage]);
    all += t;
    before += s < first ? t : 0u;
  }
  auto add = [](uint32_t a, uint32_t b) { return a + b; };
  before = wave_allreduce(before, add);
  all = wave_allreduce(all, add);
  if (lane == 0) { s_red[w][0] = before; s_red[w][1] = all; }
  __syncthreads();
  before = all = 0;
#pragma unroll
  for (int q = 0; q < kWaves; ++q) { before += s_red[q][0]; all += s_red[q][1]; }
  const uint32_t s = first + threadIdx.x;
  const bool live = s < nsets && !sets[s].done;
  const uint32_t c = live ? sets[s].cnt[stage] : 0u;
  uint32_t unused;
  uint32_t t = before + block_excl_scan(tiles_of(c), unused);
  const uint32_t a = live ? (uint32_t)off[s] : 0u;
  for (uint32_t p = 0; p < c; p += kHullTile) {
    SetTile st;
    st.set = s; st.begin = a + p; st.end = a + (p + kHullTile < c ? p + kHullTile : c); st.pad = 0;
    rtiles[t++] = st;
  }
  if (live) sets[s].cnt[stage + 1] = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) bh->nround[stage] = all;
}

// Tile hulls of one round, appended to the set's slice of the next buffer.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void k_batch_round(const uint64_t* __restrict__ off,
                                                        const BatchHdr* __restrict__ bh, int stage,
                                                        const SetTile* __restrict__ rtiles,
                                                        SetState* __restrict__ sets,
                                                        const Rec* __restrict__ in,
                                                        Rec* __restrict__ out) {
  __shared__ HullSmem<kHullTile> sm;
  __shared__ uint32_t s_base;
  const uint32_t nt = bh->nround[stage];
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const SetTile st = rtiles[t];
    uint32_t nl, nu;
    const uint32_t h = tile_hull<kHullTile>(sm, in, st.begin, st.end - st.begin, nl, nu);
    if (threadIdx.x == 0) s_base = (uint32_t)off[st.set] + atomicAdd(&sets[st.set].cnt[stage + 1], h);
    __syncthreads();
    const uint32_t ob = s_base;
    for (uint32_t k = threadIdx.x; k < h; k += kBlock) out[ob + k] = hull_elem(sm, k, nl, nu);
    __syncthreads();
  }
}

// Every set still unfinished after the rounds: its hull by big_set_hull,
// one workgroup per set (sets with a fixed stride). The last round's output
// (the candidates) is in `cand`; the set's slice of `spare` is free.
__global__ __launch_bounds__(kBlock) void k_batch_large(const uint64_t* __restrict__ off,
                                                        uint32_t nsets,
                                                        const BatchHdr* __restrict__ bh,
                                                        SetState* __restrict__ sets,
                                                        Rec* __restrict__ cand,
                                                        Rec* __restrict__ spare,
                                                        uint32_t* __restrict__ hull_idx,
                                                        uint32_t* __restrict__ hull_count) {
  __shared__ BigSmem sm;
  if (bh->bad_offsets) return;
  for (uint32_t s = blockIdx.x; s < nsets; s += gridDim.x) {
    SetState& ss = sets[s];
    if (ss.done) continue;
    const uint32_t a = (uint32_t)off[s];
    const uint32_t h = big_set_hull(sm, cand + a, spare + a, ss.cnt[kBatchRounds], ss.oct.vx[4],
                                    ss.oct.vx[0], hull_idx + a);
    if (threadIdx.x == 0) {
      hull_count[s] = h;
      ss.done = 1;
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------- launchers

hipError_t launch_hull_final(const Rec* in_rec, const uint32_t* in_count, Result* res,
                             uint32_t* res_idx, const Octagon* oct, Result* host,
                             uint32_t* host_idx, uint32_t host_n, hipStream_t st) {
  hipLaunchKernelGGL(k_hull_final, dim3(1), dim3(kBlock), 0, st, in_rec, in_count, res, res_idx, oct,
                     host, host_idx, host_n);
  return hipGetLastError();
}

hipError_t launch_hull_round(uint32_t grid, const Rec* in_rec, const uint32_t* in_count,
                             Rec* out_rec, uint32_t* out_count, uint32_t* tile_ctr,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_hull_round, dim3(grid), dim3(kBlock), 0, st, in_rec, in_count, out_rec,
                     out_count, tile_ctr);
  return hipGetLastError();
}

// The large-hull path from the records in[0..*in_count) (at most max_in)
// to the hull in res_idx, with no host round trip: partition by column
// chunk into `part` (max_in records), chunk chains into lstB, groups of them
// chained into lstA, packed into lstB, one fold per list, output. lstA /
// lstB hold two lists of kLargeListCap records each (lower, then upper);
// phist holds kChunks x kPartMax counts, ptot kChunks totals, wcnt
// 2 x (kChunks + kGroups) chain lengths.
hipError_t launch_large_path(const Rec* in, const uint32_t* in_count, uint32_t max_in, Rec* part,
                             uint32_t* phist, uint32_t* ptot, Rec* lstA, Rec* lstB,
                             uint32_t* wcnt, const Octagon* oct, Result* res, uint32_t* res_idx,
                             Result* host, uint32_t* host_idx, uint32_t host_n, hipStream_t st,
                             LaunchHook* hk) {
  const size_t cap = kLargeListCap;
  uint32_t G = (max_in + 2047) / 2048;
  if (G < 1) G = 1;
  if (G > kPartMax) G = kPartMax;
  hooked(hk, "lg_count", [&] {
    hipLaunchKernelGGL(k_lg_count, dim3(G), dim3(kBlock), 0, st, in, in_count, phist);
  });
  hooked(hk, "lg_scan", [&] {
    hipLaunchKernelGGL(k_lg_scan, dim3(kChunks), dim3(kBlock), 0, st, phist, G, ptot);
  });
  hooked(hk, "lg_scatter", [&] {
    hipLaunchKernelGGL(k_lg_scatter, dim3(G), dim3(kBlock), 0, st, in, in_count, phist, ptot, part);
  });
  hooked(hk, "lg_chunk", [&] {
    hipLaunchKernelGGL(k_lg_chunk, dim3(kChunks), dim3(kBlock), 0, st, part, ptot, oct, lstB, cap,
                       wcnt);
  });
  uint32_t* gcnt = wcnt + 2 * kChunks;
  hooked(hk, "lg_group", [&] {
    hipLaunchKernelGGL(k_lg_group, dim3(2 * kGroups), dim3(kBlock), 0, st, lstB, lstA, cap, wcnt,
                       gcnt);
  });
  hooked(hk, "lg_pack", [&] {
    hipLaunchKernelGGL(k_lg_pack, dim3(2 * kGroups), dim3(kBlock), 0, st, lstA, lstB, cap,
                       kGroupStride, kGroups, gcnt, res->pack_cnt);
  });
  hooked(hk, "lg_fold", [&] {
    hipLaunchKernelGGL(k_fold, dim3(2), dim3(kBlock), 0, st, lstB, cap, res->pack_cnt, 1u,
                       res->fold_cnt);
  });
  hooked(hk, "lg_out", [&] {
    hipLaunchKernelGGL(k_large_out, dim3(16), dim3(kBlock), 0, st, lstB, lstB + cap, res, res_idx,
                       host, host_idx, host_n);
  });
  return hipGetLastError();
}

}  // namespace chk

namespace chk {

hipError_t launch_batch_hull_side(const uint64_t* off, uint32_t nsets, uint64_t total_points,
                                  BatchHdr* bh, SetState* sets, SetTile* rtiles, Rec* recA, Rec* recB,
                                  uint32_t* hull_idx, uint32_t* hull_count, uint32_t grid,
                                  uint32_t* order, hipStream_t st, LaunchHook* hk) {
  Rec* buf[2] = {recA, recB};
  // Grids above the most workgroups with work (sets, or round tiles) only
  // add dispatch time, which small batches feel.
  auto cap = [](uint64_t g, uint64_t most) { return (uint32_t)(most < 1 ? 1 : (g < most ? g : most)); };
  const uint32_t g_sets = cap(grid, nsets);
  const uint32_t g_tiles = cap(grid, total_points / kHullTile + nsets);
  hooked(hk, "batch_final_plan", [&] {
    hipLaunchKernelGGL(k_batch_final_plan, dim3(nsets / kBlock + 1), dim3(kBlock), 0, st, nsets, bh,
                       sets, order);
  });
  hooked(hk, "batch_final", [&] {
    hipLaunchKernelGGL(k_batch_final<kHullTile>, dim3(g_sets), dim3(kBlock), 0, st, off, nsets, bh,
                       sets, 0, recA, hull_idx, hull_count, order);
  });
  for (int r = 0; r < kBatchRounds; ++r) {
    hooked(hk, "batch_round_plan", [&] {
      hipLaunchKernelGGL(k_batch_round_plan, dim3(nsets / kBlock + 1), dim3(kBlock), 0, st, off,
                         nsets, bh, sets, r, rtiles);
    });
    hooked(hk, "batch_round", [&] {
      hipLaunchKernelGGL(k_batch_round, dim3(g_tiles), dim3(kBlock), 0, st, off, bh, r, rtiles, sets,
                         buf[r & 1], buf[(r + 1) & 1]);
    });
    hooked(hk, "batch_final", [&] {
      if (r + 1 < kBatchRounds)
        hipLaunchKernelGGL(k_batch_final<kHullTile>, dim3(g_sets), dim3(kBlock), 0, st, off, nsets, bh,
                           sets, r + 1, buf[(r + 1) & 1], hull_idx, hull_count, nullptr);
      else
        hipLaunchKernelGGL(k_batch_final<kFinalTile>, dim3(g_sets), dim3(kBlock), 0, st, off, nsets, bh,
                           sets, r + 1, buf[(r + 1) & 1], hull_idx, hull_count, nullptr);
    });
  }
  // Sets whose candidates did not shrink to one workgroup: the last round
  // wrote them to buf[kBatchRounds & 1].
  hooked(hk, "batch_large", [&] {
    hipLaunchKernelGGL(k_batch_large, dim3(g_sets), dim3(kBlock), 0, st, off, nsets, bh, sets,
                       buf[kBatchRounds & 1], buf[(kBatchRounds + 1) & 1], hull_idx, hull_count);
  });
  return hipGetLastError();
}

}  // namespace chk
