// Filtering stage of the heaphull method on gfx950 (CDNA4, wave64).
//
// Pass 1 (k_reduce8): one streaming read of the points. Each lane keeps eight
// running extremes; the four axis extremes and the four Manhattan corners of
// Sec. III collapse into max/min of four exact fp64 keys, because for points
// inside the box of the axis extremes the Manhattan distance to a box corner
// is an affine function of x+y or x-y. The last block to finish builds the
// octagon (slot order E NE N NW W SW S SE), its exact edge forms and an
// axis-aligned box inside it for a cheap first test.
//
// Pass 2 (k_filter): a second streaming read. Each point is tested against the
// octagon (Alg. 1/2: keep what lies outside; Sec. I: a point on a side that is
// not a vertex is discarded). Survivors are compacted in ascending index order
// in the same pass: ballot + popcount ranks inside a wave, an LDS scan across
// the waves of a tile, and a decoupled look-back across tiles with tile ids
// handed out in launch order so that every tile waited on is already running.
//
// All predicates are exact: coordinates are multiples of 2^-20 below 1, so the
// keys (< 2^45 in units of 2^-20) and the edge forms (< 2^42) are integers that
// fp64 represents exactly, and every fma below rounds nothing.
#include "ch_internal.hpp"

namespace chk {

static constexpr double kShift = 4194304.0;  // 2^22: primary key weight
static constexpr float kGridF = 1048576.0f;  // 2^20

struct Keys {
  double mxE, mnE, mxN, mnN, mxNE, mnNE, mxSE, mnSE;
};

__device__ __forceinline__ void keys_init(Keys& k) {
  const double inf = __builtin_inf();
  k.mxE = k.mxN = k.mxNE = k.mxSE = -inf;
  k.mnE = k.mnN = k.mnNE = k.mnSE = inf;
}

// Slot keys, each maximised (mx) and minimised (mn):
//   kE  = (x,   y)    -> max: E,  min: W
//   kN  = (y,  -x)    -> max: N,  min: S
//   kNE = (x+y, y-x)  -> max: NE, min: SW
//   kSE = (x-y, x+y)  -> max: SE, min: NW
// The pair (f, g) is packed as f*2^22 + g; the secondary term is the slot's
// direction turned counter-clockwise, which breaks ties towards the
// counter-clockwise end of a supporting side.
__device__ __forceinline__ void keys_add(Keys& k, float x, float y, bool& bad) {
  const float tx = x * kGridF, ty = y * kGridF;
  bad |= (tx != __builtin_rintf(tx)) | (ty != __builtin_rintf(ty));
  const double dx = x, dy = y;
  const double s = dx + dy, d = dx - dy;
  const double kE = __builtin_fma(dx, kShift, dy);
  const double kN = __builtin_fma(dy, kShift, -dx);
  const double kNE = __builtin_fma(s, kShift, -d);
  const double kSE = __builtin_fma(d, kShift, s);
  k.mxE = __builtin_fmax(k.mxE, kE);   k.mnE = __builtin_fmin(k.mnE, kE);
  k.mxN = __builtin_fmax(k.mxN, kN);   k.mnN = __builtin_fmin(k.mnN, kN);
  k.mxNE = __builtin_fmax(k.mxNE, kNE); k.mnNE = __builtin_fmin(k.mnNE, kNE);
  k.mxSE = __builtin_fmax(k.mxSE, kSE); k.mnSE = __builtin_fmin(k.mnSE, kSE);
}

__device__ __forceinline__ void keys_merge(Keys& k, const Keys& o) {
  k.mxE = __builtin_fmax(k.mxE, o.mxE);   k.mnE = __builtin_fmin(k.mnE, o.mnE);
  k.mxN = __builtin_fmax(k.mxN, o.mxN);   k.mnN = __builtin_fmin(k.mnN, o.mnN);
  k.mxNE = __builtin_fmax(k.mxNE, o.mxNE); k.mnNE = __builtin_fmin(k.mnNE, o.mnNE);
  k.mxSE = __builtin_fmax(k.mxSE, o.mxSE); k.mnSE = __builtin_fmin(k.mnSE, o.mnSE);
}

__device__ __forceinline__ void keys_to_array(const Keys& k, double* a) {
  a[0] = k.mxE; a[1] = k.mnE; a[2] = k.mxN; a[3] = k.mnN;
  a[4] = k.mxNE; a[5] = k.mnNE; a[6] = k.mxSE; a[7] = k.mnSE;
}

__device__ __forceinline__ void keys_from_array(Keys& k, const double* a) {
  k.mxE = a[0]; k.mnE = a[1]; k.mxN = a[2]; k.mnN = a[3];
  k.mxNE = a[4]; k.mnNE = a[5]; k.mxSE = a[6]; k.mnSE = a[7];
}

__device__ __forceinline__ double wmax(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = __builtin_fmax(v, __shfl_xor(v, o));
  return v;
}
__device__ __forceinline__ double wmin(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = __builtin_fmin(v, __shfl_xor(v, o));
  return v;
}

// Reduce a block's keys; the result is valid in thread 0.
__device__ void block_keys(Keys& k) {
  __shared__ double s[kWaves][8];
  k.mxE = wmax(k.mxE); k.mnE = wmin(k.mnE); k.mxN = wmax(k.mxN); k.mnN = wmin(k.mnN);
  k.mxNE = wmax(k.mxNE); k.mnNE = wmin(k.mnNE); k.mxSE = wmax(k.mxSE); k.mnSE = wmin(k.mnSE);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) keys_to_array(k, s[w]);
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int i = 1; i < kWaves; ++i) {
      Keys o;
      keys_from_array(o, s[i]);
      keys_merge(k, o);
    }
  }
  __syncthreads();
}

// Decode one slot key into grid coordinates. type 0: (x, y); 1: (y, -x);
// 2: (x+y, y-x); 3: (x-y, x+y). Returns false for values no valid input
// produces (infinite, non-integral, wrong parity, outside the grid).
__device__ bool decode_slot(double K, int type, int64_t& x, int64_t& y) {
  if (!(__builtin_fabs(K) < 1.0e15)) return false;
  const double kf = __builtin_rint(K * 0.25);            // primary, grid units
  const double kg = (K - 4.0 * kf) * 1048576.0;          // secondary, grid units
  if (kg != __builtin_rint(kg)) return false;
  const int64_t f = (int64_t)kf, g = (int64_t)kg;
  switch (type) {
    case 0: x = f; y = g; break;
    case 1: y = f; x = -g; break;
    case 2:
      if ((f - g) & 1) return false;
      x = (f - g) / 2; y = (f + g) / 2; break;
    default:
      if ((f + g) & 1) return false;
      x = (f + g) / 2; y = (g - f) / 2; break;
  }
  return x >= 0 && x < 1048576 && y >= 0 && y < 1048576;
}

__device__ __forceinline__ int64_t orient_i64(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                                              int64_t px, int64_t py) {
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

__device__ bool box_inside(const int64_t* vx, const int64_t* vy, int64_t xl, int64_t xh,
                           int64_t yl, int64_t yh) {
  if (!(xl < xh && yl < yh)) return false;
  const int64_t cx[4] = {xl, xh, xh, xl}, cy[4] = {yl, yl, yh, yh};
  for (int i = 0; i < 8; ++i) {
    const int j = (i + 1) & 7;
    for (int c = 0; c < 4; ++c)
      if (orient_i64(vx[i], vy[i], vx[j], vy[j], cx[c], cy[c]) < 0) return false;
  }
  return true;
}

// Single-thread tail of pass 1: decode the octagon, check the domain, build
// the edge forms and an inscribed box, and reset the per-call counters.
__device__ void build_octagon(const Keys& k, Header* hdr, Result* res, uint32_t dom_bad) {
  Octagon& o = hdr->oct;
  const double K[8] = {k.mxE, k.mxNE, k.mxN, k.mnSE, k.mnE, k.mnNE, k.mnN, k.mxSE};
  const int type[8] = {0, 2, 1, 3, 0, 2, 1, 3};
  int64_t vx[8], vy[8];
  bool ok = dom_bad == 0;
  for (int s = 0; s < 8; ++s) {
    if (!decode_slot(K[s], type[s], vx[s], vy[s])) { ok = false; vx[s] = vy[s] = 0; }
  }
  o.status = ok ? 0u : 1u;
  for (int s = 0; s < 8; ++s) {
    const int t = (s + 1) & 7;
    const int64_t ddx = vx[t] - vx[s], ddy = vy[t] - vy[s];
    o.A[s] = (double)(-ddy) * 1048576.0;
    o.B[s] = (double)ddx * 1048576.0;
    o.C[s] = (double)(ddy * vx[s] - ddx * vy[s]);
    o.vx[s] = (int32_t)vx[s];
    o.vy[s] = (int32_t)vy[s];
    hdr->vidx[s] = 0xFFFFFFFFu;
  }
  // Inscribed box: centred on the octagon's bounding box with the same aspect
  // ratio, scaled by the largest factor that keeps all four corners inside
  // every edge (solved in fp64), then rounded inwards and verified exactly.
  bool box_ok = false;
  int64_t xl = 0, xh = 0, yl = 0, yh = 0;
  if (ok) {
    const double cx = 0.5 * (double)(vx[0] + vx[4]), cy = 0.5 * (double)(vy[2] + vy[6]);
    const double wx = 0.5 * (double)(vx[0] - vx[4]), wy = 0.5 * (double)(vy[2] - vy[6]);
    double t = 1.0;
    for (int i = 0; i < 8; ++i) {
      const int j = (i + 1) & 7;
      const double ex = (double)(vx[j] - vx[i]), ey = (double)(vy[j] - vy[i]);
      const double Lc = ex * (cy - (double)vy[i]) - ey * (cx - (double)vx[i]);
      for (int sx = -1; sx <= 1; sx += 2)
        for (int sy = -1; sy <= 1; sy += 2) {
          const double kk = ex * sy * wy - ey * sx * wx;
          if (kk < 0) t = __builtin_fmin(t, Lc / -kk);
          else if (Lc < 0) t = -1.0;
        }
    }
    if (t > 0 && wx > 0 && wy > 0) {
      t *= 0.999999;
      xl = (int64_t)__builtin_ceil(cx - t * wx);
      xh = (int64_t)__builtin_floor(cx + t * wx);
      yl = (int64_t)__builtin_ceil(cy - t * wy);
      yh = (int64_t)__builtin_floor(cy + t * wy);
      for (int it = 0; it < 4 && !box_ok; ++it) {
        box_ok = box_inside(vx, vy, xl, xh, yl, yh);
        if (!box_ok) { ++xl; --xh; ++yl; --yh; }
      }
    }
  }
  o.box_ok = box_ok ? 1u : 0u;
  if (box_ok) {
    o.box[0] = (float)xl * (1.0f / kGridF);
    o.box[1] = (float)xh * (1.0f / kGridF);
    o.box[2] = (float)yl * (1.0f / kGridF);
    o.box[3] = (float)yh * (1.0f / kGridF);
  } else {
    o.box[0] = 1.0f; o.box[1] = 0.0f; o.box[2] = 1.0f; o.box[3] = 0.0f;  // empty
  }
  // Per-call counters used by the kernels that follow in stream order.
  hdr->tile_ctr = 0;
  hdr->dom_bad = 0;
  hdr->count = 0;
  hdr->col_arrive = 0;
  res->status = RES_PENDING;
  res->h = 0;
  res->lcount = res->ucount = 0;
  for (int r = 0; r < kMaxRounds; ++r) { res->round_cnt[r] = 0; res->round_tile[r] = 0; }
  for (int r = 0; r < 4; ++r) res->win_cnt[r] = 0;
}

// Pass 1. head = 1 when xy is 8 mod 16 bytes aligned: point 0 is then handled
// on its own and the float4 stream starts at point 1.
__global__ __launch_bounds__(kBlock) void k_reduce8(const float* __restrict__ xy, uint32_t n,
                                                    uint32_t head, Header* __restrict__ hdr,
                                                    Result* __restrict__ res,
                                                    double* __restrict__ partials,
                                                    uint64_t* __restrict__ tstat, uint32_t ntiles2) {
  const uint32_t gsize = gridDim.x * blockDim.x;
  const uint32_t gtid = blockIdx.x * blockDim.x + threadIdx.x;
  for (uint32_t i = gtid; i < ntiles2; i += gsize) tstat[i] = 0ull;  // pass-2 look-back state

  Keys k;
  keys_init(k);
  bool bad = false;
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * head);
  const uint32_t npairs = (n - head) >> 1;
  uint32_t p = gtid;
  for (; p + 3 * gsize < npairs; p += 4 * gsize) {
    const float4 a = p4[p], b = p4[p + gsize], c = p4[p + 2 * gsize], d = p4[p + 3 * gsize];
    keys_add(k, a.x, a.y, bad); keys_add(k, a.z, a.w, bad);
    keys_add(k, b.x, b.y, bad); keys_add(k, b.z, b.w, bad);
    keys_add(k, c.x, c.y, bad); keys_add(k, c.z, c.w, bad);
    keys_add(k, d.x, d.y, bad); keys_add(k, d.z, d.w, bad);
  }
  for (; p < npairs; p += gsize) {
    const float4 a = p4[p];
    keys_add(k, a.x, a.y, bad); keys_add(k, a.z, a.w, bad);
  }
  if (gtid == 0) {
    if (head) keys_add(k, xy[0], xy[1], bad);
    if ((n - head) & 1) keys_add(k, xy[2 * (n - 1)], xy[2 * (n - 1) + 1], bad);
  }
  if (bad) atomicOr(&hdr->dom_bad, 1u);

  block_keys(k);
  __shared__ int s_last;
  if (threadIdx.x == 0) {
    double a[8];
    keys_to_array(k, a);
    uint64_t* dst = reinterpret_cast<uint64_t*>(partials) + size_t(blockIdx.x) * 8;
    for (int i = 0; i < 8; ++i)
      __hip_atomic_store(dst + i, (uint64_t)__double_as_longlong(a[i]), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    __threadfence();
    const uint32_t prev = __hip_atomic_fetch_add(&hdr->arrive, 1u, __ATOMIC_ACQ_REL,
                                                 __HIP_MEMORY_SCOPE_AGENT);
    s_last = prev == gridDim.x - 1;
  }
  __syncthreads();
  if (!s_last) return;
  __threadfence();
  keys_init(k);
  const uint64_t* src = reinterpret_cast<const uint64_t*>(partials);
  for (uint32_t b = threadIdx.x; b < gridDim.x; b += blockDim.x) {
    double a[8];
    for (int i = 0; i < 8; ++i)
      a[i] = __longlong_as_double((long long)__hip_atomic_load(src + size_t(b) * 8 + i,
                                                               __ATOMIC_RELAXED,
                                                               __HIP_MEMORY_SCOPE_AGENT));
    Keys o;
    keys_from_array(o, a);
    keys_merge(k, o);
  }
  block_keys(k);
  if (threadIdx.x == 0) {
    const uint32_t db = __hip_atomic_load(&hdr->dom_bad, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    build_octagon(k, hdr, res, db);
    hdr->arrive = 0;
  }
}

// ---------------------------------------------------------------- pass 2

struct Verdict {
  bool keep;
  uint8_t label;
};

// Exact classification of one point against the octagon (outside some edge,
// or equal to a vertex). Records the smallest index per vertex.
template <bool LABELS>
__device__ __forceinline__ Verdict classify(float x, float y, uint32_t gidx,
                                            const Octagon* __restrict__ o,
                                            uint32_t* __restrict__ vidx) {
  const double dx = x, dy = y;
  double mn = __builtin_inf();
  int first = 8;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const double L = __builtin_fma(o->A[i], dx, __builtin_fma(o->B[i], dy, o->C[i]));
    if (LABELS) {
      if (L < 0.0 && first == 8) first = i;
    }
    mn = __builtin_fmin(mn, L);
  }
  Verdict v{mn < 0.0, 0};
  if (LABELS && v.keep) v.label = (uint8_t)(1 + (first >> 1));
  if (mn == 0.0) {  // on the boundary: kept only when it is a vertex
    const int32_t ix = (int32_t)(x * kGridF), iy = (int32_t)(y * kGridF);
    int slot = 8;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      if (ix == o->vx[s] && iy == o->vy[s]) {
        atomicMin(&vidx[s], gidx);
        if (slot == 8) slot = s;
      }
    }
    if (slot < 8) {
      v.keep = true;
      if (LABELS) v.label = (uint8_t)(1 + (slot >> 1));
    }
  }
  return v;
}

__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

// Pass 2. Grid = filter_tiles(n) blocks; tile ids come from hdr->tile_ctr.
template <bool LABELS>
__global__ __launch_bounds__(kBlock) void k_filter(const float* __restrict__ xy, uint32_t n,
                                                   uint32_t head, Header* __restrict__ hdr,
                                                   uint64_t* __restrict__ tstat, uint32_t ntiles,
                                                   uint32_t* __restrict__ surv,
                                                   uint32_t* __restrict__ count_out,
                                                   uint8_t* __restrict__ labels) {
  __shared__ uint32_t s_tile, s_head, s_total, s_prefix;
  __shared__ uint32_t s_off[kPairsPerThread * kWaves];
  const Octagon* __restrict__ o = &hdr->oct;
  uint32_t* __restrict__ vidx = hdr->vidx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  if (threadIdx.x == 0) s_tile = atomicAdd(&hdr->tile_ctr, 1u);
  __syncthreads();
  const uint32_t t = s_tile;
  if (o->status != 0) {
    if (t == ntiles - 1 && threadIdx.x == 0) *count_out = kCountDomain;
    return;
  }
  const float bxl = o->box[0], bxh = o->box[1], byl = o->box[2], byh = o->box[3];
  const uint32_t nfull = (n - head) >> 1;
  const bool half = ((n - head) & 1) != 0;
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * head);

  float4 v[kPairsPerThread];
#pragma unroll
  for (int j = 0; j < kPairsPerThread; ++j) {
    const uint32_t q = t * kTilePairs + j * kBlock + threadIdx.x;
    if (q < nfull) {
      v[j] = p4[q];
    } else if (q == nfull && half) {
      const float2 u = reinterpret_cast<const float2*>(xy)[head + 2 * q];
      v[j] = make_float4(u.x, u.y, 0.f, 0.f);
    } else {
      v[j] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  }

  uint64_t b0[kPairsPerThread], b1[kPairsPerThread];
#pragma unroll
  for (int j = 0; j < kPairsPerThread; ++j) {
    const uint32_t q = t * kTilePairs + j * kBlock + threadIdx.x;
    const bool val1 = q < nfull;
    const bool val0 = val1 || (q == nfull && half);
    const uint32_t g = head + 2 * q;
    const float x0 = v[j].x, y0 = v[j].y, x1 = v[j].z, y1 = v[j].w;
    const bool in0 = (x0 > bxl) & (x0 < bxh) & (y0 > byl) & (y0 < byh);
    const bool in1 = (x1 > bxl) & (x1 < bxh) & (y1 > byl) & (y1 < byh);
    const bool need0 = val0 & !in0, need1 = val1 & !in1;
    Verdict r0{false, 0}, r1{false, 0};
    if (__ballot(need0 | need1)) {
      if (need0) r0 = classify<LABELS>(x0, y0, g, o, vidx);
      if (need1) r1 = classify<LABELS>(x1, y1, g + 1, o, vidx);
    }
    b0[j] = __ballot(r0.keep);
    b1[j] = __ballot(r1.keep);
    if (LABELS) {
      if (val0) labels[g] = r0.label;
      if (val1) labels[g + 1] = r1.label;
    }
  }

  // Tile 0 also owns the unaligned head point (index 0), ranked first.
  if (threadIdx.x == 0) {
    uint32_t hk = 0;
    if (t == 0 && head) {
      const Verdict r = classify<LABELS>(xy[0], xy[1], 0u, o, vidx);
      hk = r.keep ? 1u : 0u;
      if (LABELS) labels[0] = r.label;
    }
    s_head = hk;
  }
  if (lane == 0) {
#pragma unroll
    for (int j = 0; j < kPairsPerThread; ++j) s_off[j * kWaves + w] = popc64(b0[j]) + popc64(b1[j]);
  }
  __syncthreads();

  // Exclusive scan of the (j, wave) group counts in index order, then the
  // look-back for the tile's global offset; both by wave 0.
  if (w == 0) {
    constexpr int kGroups = kPairsPerThread * kWaves;
    static_assert(kGroups <= 64, "group scan fits one wave");
    const uint32_t c = lane < kGroups ? s_off[lane] : 0u;
    uint32_t incl = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t u = __shfl_up(incl, d);
      if (lane >= d) incl += u;
    }
    const uint32_t hk = s_head;
    if (lane < kGroups) s_off[lane] = incl - c + hk;
    const uint32_t total = __shfl(incl, 63) + hk;

    uint64_t excl = 0;
    if (t == 0) {
      if (lane == 0)
        __hip_atomic_store(&tstat[0], (2ull << 32) | total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    } else {
      if (lane == 0)
        __hip_atomic_store(&tstat[t], (1ull << 32) | total, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
      int64_t base = (int64_t)t - 1;
      while (true) {
        const int64_t idx = base - lane;
        uint64_t s = 2ull << 32;  // beyond tile 0: an inclusive zero
        if (idx >= 0) {
          s = __hip_atomic_load(&tstat[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          while ((s >> 32) == 0) {
            __builtin_amdgcn_s_sleep(1);
            s = __hip_atomic_load(&tstat[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        const uint64_t pm = __ballot((s >> 32) == 2);
        const int first = pm ? (__ffsll((long long)pm) - 1) : 63;
        uint64_t contrib = lane <= first ? (uint64_t)(uint32_t)s : 0ull;
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) contrib += __shfl_xor(contrib, d);
        excl += contrib;
        if (pm) break;
        base -= 64;
      }
      if (lane == 0)
        __hip_atomic_store(&tstat[t], (2ull << 32) | (uint32_t)(excl + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_prefix = (uint32_t)excl;
      s_total = total;
    }
  }
  __syncthreads();

  const uint32_t prefix = s_prefix;
  if (t == ntiles - 1 && threadIdx.x == 0) *count_out = prefix + s_total;
  if (threadIdx.x == 0 && s_head) surv[prefix] = 0u;
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int j = 0; j < kPairsPerThread; ++j) {
    if ((b0[j] | b1[j]) == 0ull) continue;
    const uint32_t q = t * kTilePairs + j * kBlock + threadIdx.x;
    const uint32_t g = head + 2 * q;
    const uint32_t base = prefix + s_off[j * kWaves + w] + popc64(b0[j] & lt) + popc64(b1[j] & lt);
    const uint32_t k0 = (uint32_t)(b0[j] >> lane) & 1u, k1 = (uint32_t)(b1[j] >> lane) & 1u;
    if (k0) surv[base] = g;
    if (k1) surv[base + k0] = g + 1;
  }
}

// Copies the octagon (coordinates and smallest indices) to a caller buffer.
__global__ void k_oct_out(const Header* __restrict__ hdr, int32_t* __restrict__ out) {
  const int s = threadIdx.x;
  if (s < 8) {
    out[s] = hdr->oct.vx[s];
    out[8 + s] = hdr->oct.vy[s];
    out[16 + s] = (int32_t)hdr->vidx[s];
  }
}

__global__ void k_ws_init(uint32_t* __restrict__ hdr_words, uint32_t nwords) {
  for (uint32_t i = threadIdx.x; i < nwords; i += blockDim.x) hdr_words[i] = 0u;
}

__global__ void k_set_u32(uint32_t* __restrict__ p, uint32_t v) {
  if (threadIdx.x == 0) *p = v;
}

// ------------------------------------------------------------- launchers

hipError_t launch_ws_init(void* ws, hipStream_t st) {
  hipLaunchKernelGGL(k_ws_init, dim3(1), dim3(kBlock), 0, st, static_cast<uint32_t*>(ws),
                     uint32_t((kHdrBytes + kResBytes) / 4));
  return hipGetLastError();
}

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

uint32_t reduce_blocks(uint32_t n) {
  const uint32_t per = kBlock * 16;  // aim for >= 16 points per thread
  uint32_t b = (n + per - 1) / per;
  if (b < 1) b = 1;
  if (b > (uint32_t)kReduceMaxBlocks) b = kReduceMaxBlocks;
  return b;
}

hipError_t launch_reduce8(const float* xy, uint32_t n, uint32_t head, Header* hdr, Result* res,
                          double* partials, uint64_t* tstat, uint32_t ntiles2, uint32_t blocks,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_reduce8, dim3(blocks), dim3(kBlock), 0, st, xy, n, head, hdr, res, partials,
                     tstat, ntiles2);
  return hipGetLastError();
}

hipError_t launch_filter(const float* xy, uint32_t n, uint32_t head, Header* hdr, uint64_t* tstat,
                         uint32_t ntiles, uint32_t* surv, uint32_t* count_out, uint8_t* labels,
                         hipStream_t st) {
  if (labels)
    hipLaunchKernelGGL(k_filter<true>, dim3(ntiles), dim3(kBlock), 0, st, xy, n, head, hdr, tstat,
                       ntiles, surv, count_out, labels);
  else
    hipLaunchKernelGGL(k_filter<false>, dim3(ntiles), dim3(kBlock), 0, st, xy, n, head, hdr, tstat,
                       ntiles, surv, count_out, labels);
  return hipGetLastError();
}

hipError_t launch_oct_out(const Header* hdr, void* d_oct, hipStream_t st) {
  hipLaunchKernelGGL(k_oct_out, dim3(1), dim3(64), 0, st, hdr, static_cast<int32_t*>(d_oct));
  return hipGetLastError();
}

}  // namespace chk
