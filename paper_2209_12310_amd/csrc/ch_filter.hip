// Filtering stage of the heaphull method on gfx950 (CDNA4, wave64).
//
// Pass 1 (k_reduce8 + k_oct_build): one streaming read of the points. Each
// lane keeps eight running extremes; the four axis extremes and the four
// Manhattan corners of Sec. III collapse into max/min of four exact fp64 keys,
// because for points inside the box of the axis extremes the Manhattan
// distance to a box corner is an affine function of x+y or x-y. One workgroup
// then builds the octagon (slot order E NE N NW W SW S SE), its exact edge
// forms and an axis-aligned box inside it for a cheap first test.
//
// Pass 2 (k_filter): a second streaming read. Each point is tested against the
// octagon (Alg. 1/2: keep what lies outside; Sec. I: a point on a side that is
// not a vertex is discarded). Survivors are compacted in ascending index order
// in the same pass: ballot + popcount ranks inside a wave, contiguous ranges
// per wave, and one look-back per workgroup over the counts of the earlier
// workgroups.
//
// All predicates are exact: coordinates are multiples of 2^-20 below 1, so the
// keys (< 2^45 in units of 2^-20) and the edge forms (< 2^42) are integers that
// fp64 represents exactly, and every fma below rounds nothing.
#include "ch_refine.hpp"

namespace chk {

static constexpr double kShift = 4194304.0;  // 2^22: primary key weight

// Waits for every outstanding memory operation. Called once after a streaming
// loop's first batch of loads: without it the wait-count insertion treats the
// loop-carried current batch as possibly still in flight at the loop head and
// waits for the prefetched batch too, which serialises the pipeline.
__device__ __forceinline__ void wait_all_loads() { __builtin_amdgcn_s_waitcnt(0); }

// Streaming loads of two points (16 B) that bypass cache retention: the
// points are read once per pass.
typedef float f4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float4 ld_stream(const float4* p) {
  const f4v v = __builtin_nontemporal_load(reinterpret_cast<const f4v*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

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
  return wave_allreduce(v, [](double a, double b) { return __builtin_fmax(a, b); });
}
__device__ __forceinline__ double wmin(double v) {
  return wave_allreduce(v, [](double a, double b) { return __builtin_fmin(a, b); });
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

// The inscribed box is centred on the octagon's bounding box, keeps its aspect
// ratio, and is scaled by the largest factor t <= 1 that keeps all four
// corners inside every edge. Lane 4*i + c solves the bound of edge i and
// corner c in fp64; a wave-wide minimum follows. The result is a candidate
// only: it is rounded inwards and verified exactly.
__device__ double box_scale_lane(const int64_t* vx, const int64_t* vy, int lane) {
  double t = 1.0;
  if (lane < 32) {
    const int i = lane >> 2, j = (i + 1) & 7;
    const int sx = (lane & 1) ? 1 : -1, sy = (lane & 2) ? 1 : -1;
    const double cx = 0.5 * (double)(vx[0] + vx[4]), cy = 0.5 * (double)(vy[2] + vy[6]);
    const double wx = 0.5 * (double)(vx[0] - vx[4]), wy = 0.5 * (double)(vy[2] - vy[6]);
    const double ex = (double)(vx[j] - vx[i]), ey = (double)(vy[j] - vy[i]);
    const double Lc = ex * (cy - (double)vy[i]) - ey * (cx - (double)vx[i]);
    const double kk = ex * sy * wy - ey * sx * wx;
    if (kk < 0) t = Lc / -kk;
    else if (Lc < 0) t = -1.0;
  }
  return wmin(t);
}

// One wave: decode the octagon from the slot keys, check the domain, write
// the edge forms and (BOX) the inscribed box to `o`, and reset vidx (may be
// null). Lanes 0-7 decode one slot each; lanes 0-31 test one (edge, corner)
// pair each.
template <bool BOX = true>
__device__ void octagon_wave(const Keys& k, Octagon& o, uint32_t* vidx, uint32_t dom_bad) {
  const int lane = threadIdx.x & 63;
  const double K[8] = {k.mxE, k.mxNE, k.mxN, k.mnSE, k.mnE, k.mnNE, k.mnN, k.mxSE};
  int64_t mx = 0, my = 0;
  bool good = true;
  if (lane < 8) {
    const int type = (lane == 0 || lane == 4) ? 0 : (lane == 2 || lane == 6) ? 1
                     : (lane == 1 || lane == 5) ? 2 : 3;
    double kv = K[0];
#pragma unroll
    for (int s = 1; s < 8; ++s) kv = lane == s ? K[s] : kv;
    good = decode_slot(kv, type, mx, my);
    if (!good) mx = my = 0;
  }
  const bool ok = __ballot(!good) == 0 && dom_bad == 0;
  int64_t vx[8], vy[8];
#pragma unroll
  for (int s = 0; s < 8; ++s) {
    vx[s] = read_lane(mx, s);
    vy[s] = read_lane(my, s);
  }
  if (lane < 8) {
    const int t = (lane + 1) & 7;
    const int64_t ddx = vx[t] - mx, ddy = vy[t] - my;
    o.A[lane] = (double)(-ddy) * 1048576.0;
    o.B[lane] = (double)ddx * 1048576.0;
    o.C[lane] = (double)(ddy * mx - ddx * my);
    o.vx[lane] = (int32_t)mx;
    o.vy[lane] = (int32_t)my;
    if (vidx) vidx[lane] = 0xFFFFFFFFu;
  }
  if (!BOX) {
    if (lane == 0) o.status = ok ? 0u : 1u;
    return;
  }
  const double t0 = box_scale_lane(vx, vy, lane);
  bool box_ok = false;
  int64_t xl = 0, xh = 0, yl = 0, yh = 0;
  const double cx = 0.5 * (double)(vx[0] + vx[4]), cy = 0.5 * (double)(vy[2] + vy[6]);
  const double wx = 0.5 * (double)(vx[0] - vx[4]), wy = 0.5 * (double)(vy[2] - vy[6]);
  if (ok && t0 > 0 && wx > 0 && wy > 0) {
    const double t = t0 * 0.999999;
    xl = (int64_t)__builtin_ceil(cx - t * wx);
    xh = (int64_t)__builtin_floor(cx + t * wx);
    yl = (int64_t)__builtin_ceil(cy - t * wy);
    yh = (int64_t)__builtin_floor(cy + t * wy);
    for (int it = 0; it < 4; ++it) {
      bool in = true;
      if (lane < 32) {
        const int i = lane >> 2, j = (i + 1) & 7;
        const int64_t px = (lane & 1) ? xh : xl, py = (lane & 2) ? yh : yl;
        in = orient_i64(vx[i], vy[i], vx[j], vy[j], px, py) >= 0;
      }
      box_ok = xl < xh && yl < yh && __ballot(!in) == 0;
      if (box_ok) break;
      ++xl; --xh; ++yl; --yh;
    }
  }
  if (lane == 0) {
    o.status = ok ? 0u : 1u;
    o.box_ok = box_ok ? 1u : 0u;
    if (box_ok) {
      o.box[0] = (float)xl * (1.0f / kGridF);
      o.box[1] = (float)xh * (1.0f / kGridF);
      o.box[2] = (float)yl * (1.0f / kGridF);
      o.box[3] = (float)yh * (1.0f / kGridF);
    } else {
      o.box[0] = 1.0f; o.box[1] = 0.0f; o.box[2] = 1.0f; o.box[3] = 0.0f;  // empty
    }
  }
}

// One wave: the per-call counters used by the kernels that follow in stream
// order (the survivor count too when `count`).
__device__ void reset_call_state(Header* hdr, Result* res, bool count) {
  const int lane = threadIdx.x & 63;
  if (lane == 0) {
    hdr->tile_ctr = 0;
    hdr->dom_bad = 0;
    if (count) hdr->count = 0;
    hdr->col_arrive = 0;
    res->status = RES_PENDING;
    res->h = 0;
    res->lcount = res->ucount = 0;
    res->ncand = 0;
    res->cand_surv = 0;
  }
  for (int r = lane; r < kMaxRounds; r += 64) { res->round_cnt[r] = 0; res->round_tile[r] = 0; }
  if (lane < 2) { res->pack_cnt[lane] = 0; res->fold_cnt[lane] = 0; }
}

// Wave 0 of k_oct_build: the octagon of the single set, then the per-call
// counters.
__device__ void build_octagon_wave(const Keys& k, Header* hdr, Result* res, uint32_t dom_bad) {
  octagon_wave(k, hdr->oct, hdr->vidx, dom_bad);
  reset_call_state(hdr, res, true);
}

// Rows of 64 pairs per streaming batch of passes 1 and 2 (kU coalesced 1 KiB
// loads; with the next batch in flight every wave keeps 4-8 KiB outstanding).
constexpr int kU = 4;
// Rows per batch of the fused hull pass, which runs with fewer workgroups
// (it is launched with about one per CU: fewer, longer streams keep the
// HBM reads closer together).
constexpr int kUF = 8;
// The fused pass runs on its whole grid when more than 1 in kWideRatio of
// its estimate's points (kEstPer per thread) fall outside the polygon's
// inner region.
constexpr uint32_t kWideRatio = 300;
constexpr uint32_t kEstPer = 4;

// Compile-time mode passed to generic lambdas (one instantiation per mode).
template <int M>
struct IntC {
  static constexpr int value = M;
};

// One streaming read of all n points by a persistent grid, handing every
// point to acc.add(x, y, bad). Each wave streams batches of kU rows of 64
// pairs and issues the next batch's loads before reducing the current one.
// Lanes past the end re-read the last pair (duplicates move no extreme).
template <class Acc>
__device__ __forceinline__ void stream_points(const float* __restrict__ xy, uint32_t n,
                                              uint32_t head, Acc& acc, bool& bad) {
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * head);
  const uint32_t nfull = (n - head) >> 1;
  const int lane = threadIdx.x & 63;
  const uint32_t gw = blockIdx.x * kWaves + (threadIdx.x >> 6);
  const uint32_t nw = gridDim.x * kWaves;
  const uint32_t per_batch = kU * 64;
  const uint32_t nbatch = (nfull + per_batch - 1) / per_batch;
  if (gw < nbatch) {
    float4 cur[kU], nxt[kU];
    uint32_t b = gw;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t q = b * per_batch + u * 64 + lane;
      cur[u] = ld_stream(&p4[q < nfull ? q : nfull - 1]);
    }
    wait_all_loads();
    while (true) {
      const uint32_t bn = b + nw;
      const bool more = bn < nbatch;
      if (more) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const uint32_t q = bn * per_batch + u * 64 + lane;
          nxt[u] = ld_stream(&p4[q < nfull ? q : nfull - 1]);
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        acc.add(cur[u].x, cur[u].y, bad);
        acc.add(cur[u].z, cur[u].w, bad);
      }
      if (!more) break;
#pragma unroll
      for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
      b = bn;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (head) acc.add(xy[0], xy[1], bad);
    if ((n - head) & 1) acc.add(xy[2 * (n - 1)], xy[2 * (n - 1) + 1], bad);
  }
}

// The block's domain flag (any lane saw a bad value), valid in every thread.
__device__ __forceinline__ uint32_t block_any(bool bad) {
  const uint64_t badmask = __ballot(bad);
  __shared__ uint32_t s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && badmask) s_bad = 1;
  __syncthreads();
  return s_bad;
}

// Accumulator of the one-read search: all eight slot keys.
struct AccAll {
  Keys k;
  __device__ __forceinline__ void add(float x, float y, bool& bad) { keys_add(k, x, y, bad); }
};

// Pass 1: persistent grid. Each block writes its 8 keys and a domain flag;
// k_oct_build combines them. head = 1 when xy is 8 mod 16 bytes aligned:
// point 0 is then read on its own and the float4 stream starts at point 1.
__global__ __launch_bounds__(kBlock) void k_reduce8(const float* __restrict__ xy, uint32_t n,
                                                    uint32_t head, double* __restrict__ partials,
                                                    uint32_t* __restrict__ part_bad) {
  AccAll acc;
  keys_init(acc.k);
  bool bad = false;
  stream_points(xy, n, head, acc, bad);
  const uint32_t bflag = block_any(bad);
  block_keys(acc.k);
  if (threadIdx.x == 0) {
    keys_to_array(acc.k, partials + size_t(blockIdx.x) * 8);
    part_bad[blockIdx.x] = bflag;
  }
}

// Combines the pass-1 partials of nparts workgroups (all loads issued up
// front). Every thread calls it; on return the keys are valid in every lane
// of wave 0, and the domain flag in every thread.
__device__ uint32_t combine_partials(const double* __restrict__ partials,
                                     const uint32_t* __restrict__ part_bad, uint32_t nparts,
                                     Keys& k) {
  constexpr int kPer = kReduceMaxBlocks / kBlock;
  constexpr int kChunk = 4;  // partials in flight per thread (register budget)
  keys_init(k);
  uint32_t bad = 0;
  const double4* __restrict__ p4 = reinterpret_cast<const double4*>(partials);
  for (int r0 = 0; r0 < kPer; r0 += kChunk) {
    if (threadIdx.x + r0 * kBlock >= nparts) break;
    double4 a[kChunk][2];
    uint32_t bb[kChunk];
#pragma unroll
    for (int r = 0; r < kChunk; ++r) {
      const uint32_t b = threadIdx.x + (r0 + r) * kBlock;
      if (b < nparts) {
        a[r][0] = p4[2 * b];
        a[r][1] = p4[2 * b + 1];
        bb[r] = part_bad[b];
      }
    }
#pragma unroll
    for (int r = 0; r < kChunk; ++r) {
      const uint32_t b = threadIdx.x + (r0 + r) * kBlock;
      if (b < nparts) {
        const double v[8] = {a[r][0].x, a[r][0].y, a[r][0].z, a[r][0].w,
                             a[r][1].x, a[r][1].y, a[r][1].z, a[r][1].w};
        Keys o;
        keys_from_array(o, v);
        keys_merge(k, o);
        bad |= bb[r];
      }
    }
  }
  const uint64_t badmask = __ballot(bad != 0);
  __shared__ uint32_t s_bad;
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();
  if ((threadIdx.x & 63) == 0 && badmask) s_bad = 1;
  block_keys(k);
  if (threadIdx.x < 64) {
    double v[8];
    keys_to_array(k, v);
#pragma unroll
    for (int i = 0; i < 8; ++i) v[i] = read_lane(v[i], 0);
    keys_from_array(k, v);
  }
  return s_bad;
}

// One workgroup: combine the pass-1 partials, build the octagon, and reset
// every per-call counter and look-back word used by the kernels that follow.
__global__ __launch_bounds__(kBlock) void k_oct_build(const double* __restrict__ partials,
                                                      const uint32_t* __restrict__ part_bad,
                                                      uint32_t nparts, Header* __restrict__ hdr,
                                                      Result* __restrict__ res,
                                                      uint64_t* __restrict__ tstat,
                                                      uint32_t ntstat) {
  Keys k;
  const uint32_t bad = combine_partials(partials, part_bad, nparts, k);
  for (uint32_t i = threadIdx.x; i < ntstat; i += blockDim.x) tstat[i] = 0ull;
  if (threadIdx.x < 64) build_octagon_wave(k, hdr, res, bad);
}

// ------------------------------------------- the extreme search in two kernels
//
// Sec. III runs findExtremes on the GPU as two reductions in succession: one
// for the four axis extremes, then one for the point of least Manhattan
// distance to each corner of the box those four span (it needs the first
// result). ch_gpufilter and ch_hull_queues can run it that way, beside the
// one-read search above:
//   k_axis4    max/min of kE = (x, y) and kN = (y, -x): E, W, N, S, and the
//              domain check (the same keys and tie-breaks as pass 1);
//   k_axis_box one workgroup: combine, decode the four points, keep the box;
//   k_corner4  per corner c, the largest (-d_c, g): d_c = |c.x - x| + |c.y - y|
//              the Manhattan distance, g the slot's counter-clockwise
//              tie-break. On output each key is moved to pass 1's form by the
//              corner's constant (inside the box, -d_c is +-x +-y minus a
//              constant), so k_oct_build and every later stage see the
//              same partials either way and the octagon is identical.
struct AccAxis {
  double mxE, mnE, mxN, mnN;
  __device__ __forceinline__ void add(float x, float y, bool& bad) {
    const float tx = x * kGridF, ty = y * kGridF;
    bad |= (tx != __builtin_rintf(tx)) | (ty != __builtin_rintf(ty));
    const double dx = x, dy = y;
    const double kE = __builtin_fma(dx, kShift, dy);
    const double kN = __builtin_fma(dy, kShift, -dx);
    mxE = __builtin_fmax(mxE, kE); mnE = __builtin_fmin(mnE, kE);
    mxN = __builtin_fmax(mxN, kN); mnN = __builtin_fmin(mnN, kN);
  }
};

struct AccCorner {
  double ex, wx, ny, sy;          // the box (E.x, W.x, N.y, S.y)
  double kNE, kNW, kSW, kSE;      // max of -d * 2^22 + g per corner
  __device__ __forceinline__ void add(float x, float y, bool&) {
    const double dx = x, dy = y;
    const double dNE = __builtin_fabs(ex - dx) + __builtin_fabs(ny - dy);
    const double dNW = __builtin_fabs(wx - dx) + __builtin_fabs(ny - dy);
    const double dSW = __builtin_fabs(wx - dx) + __builtin_fabs(sy - dy);
    const double dSE = __builtin_fabs(ex - dx) + __builtin_fabs(sy - dy);
    kNE = __builtin_fmax(kNE, __builtin_fma(-dNE, kShift, dy - dx));
    kNW = __builtin_fmax(kNW, __builtin_fma(-dNW, kShift, -(dx + dy)));
    kSW = __builtin_fmax(kSW, __builtin_fma(-dSW, kShift, dx - dy));
    kSE = __builtin_fmax(kSE, __builtin_fma(-dSE, kShift, dx + dy));
  }
};

// First reduction: the axis keys, written as 8-slot partials whose corner
// slots hold the neutral values, and the domain flags.
__global__ __launch_bounds__(kBlock) void k_axis4(const float* __restrict__ xy, uint32_t n,
                                                  uint32_t head, double* __restrict__ partials,
                                                  uint32_t* __restrict__ part_bad) {
  const double inf = __builtin_inf();
  AccAxis acc{-inf, inf, -inf, inf};
  bool bad = false;
  stream_points(xy, n, head, acc, bad);
  const uint32_t bflag = block_any(bad);
  Keys k;
  keys_init(k);
  k.mxE = acc.mxE; k.mnE = acc.mnE; k.mxN = acc.mxN; k.mnN = acc.mnN;
  block_keys(k);
  if (threadIdx.x == 0) {
    keys_to_array(k, partials + size_t(blockIdx.x) * 8);
    part_bad[blockIdx.x] = bflag;
  }
}

// One workgroup between the two reductions: the four axis extremes and
// their box.
__global__ __launch_bounds__(kBlock) void k_axis_box(const double* __restrict__ partials,
                                                     const uint32_t* __restrict__ part_bad,
                                                     uint32_t nparts, Header* __restrict__ hdr) {
  Keys k;
  const uint32_t bad = combine_partials(partials, part_bad, nparts, k);
  if (threadIdx.x != 0) return;
  int64_t ex, ey, wx, wy, nx, ny, sx, sy;
  const bool ok = decode_slot(k.mxE, 0, ex, ey) && decode_slot(k.mnE, 0, wx, wy) &&
                  decode_slot(k.mxN, 1, nx, ny) && decode_slot(k.mnN, 1, sx, sy);
  AxisBox& a = hdr->axis;
  a.kE_max = k.mxE; a.kE_min = k.mnE; a.kN_max = k.mxN; a.kN_min = k.mnN;
  a.bad = (ok && !bad) ? 0u : 1u;
  const double g = 1.0 / 1048576.0;
  a.ex = ok ? (double)ex * g : 0.0;
  a.wx = ok ? (double)wx * g : 0.0;
  a.ny = ok ? (double)ny * g : 0.0;
  a.sy = ok ? (double)sy * g : 0.0;
}

// Second reduction: the corner keys, moved to pass 1's form and written with
// the combined axis keys as full 8-slot partials (the domain flags stay
// those of the first reduction, which ran on the same grid).
__global__ __launch_bounds__(kBlock) void k_corner4(const float* __restrict__ xy, uint32_t n,
                                                    uint32_t head, const Header* __restrict__ hdr,
                                                    double* __restrict__ partials) {
  const AxisBox& a = hdr->axis;
  const double inf = __builtin_inf();
  AccCorner acc{a.ex, a.wx, a.ny, a.sy, -inf, -inf, -inf, -inf};
  bool unused = false;
  stream_points(xy, n, head, acc, unused);
  Keys k;
  keys_init(k);
  k.mxNE = acc.kNE; k.mxSE = acc.kSE;
  k.mnNE = -acc.kSW;  // block_keys maximises mx* and minimises mn*
  k.mnSE = -acc.kNW;
  block_keys(k);
  if (threadIdx.x == 0) {
    // -d_NE = (x+y) - (E.x + N.y); -d_SW = (W.x + S.y) - (x+y);
    // -d_SE = (x-y) - (E.x - S.y); -d_NW = (W.x - N.y) - (x-y). Every term is
    // a multiple of 2^-20 below 2^24, so these sums are exact.
    Keys o;
    o.mxE = a.kE_max; o.mnE = a.kE_min; o.mxN = a.kN_max; o.mnN = a.kN_min;
    o.mxNE = k.mxNE + (a.ex + a.ny) * kShift;
    o.mnNE = k.mnNE + (a.wx + a.sy) * kShift;
    o.mxSE = k.mxSE + (a.ex - a.sy) * kShift;
    o.mnSE = k.mnSE + (a.wx - a.ny) * kShift;
    keys_to_array(o, partials + size_t(blockIdx.x) * 8);
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


// Pass 2 of ch_filter (the survivor list in ascending index order; the hull
// path uses k_filter_hull below): persistent grid of G2 workgroups. Workgroup ids come from
// hdr->tile_ctr in start order; workgroup c owns waves 4c..4c+3 and wave k
// streams the contiguous rows [k*RW, (k+1)*RW) of 64 pairs, so the survivors
// of the waves, concatenated in wave order, are in ascending index order.
// A wave stages its survivors in LDS (overflow: in `staging` at the wave's
// own point range). When the workgroup is done it publishes its count, reads
// the counts of all earlier workgroups (look-back over at most G2 words, all
// loaded at once), and copies its survivors to their final place.
// Survivor payloads: the index alone (ch_filter), or a record with the grid
// coordinates (hull path and batch mode: the hull pass then never gathers
// from the point array).
template <class P>
__device__ __forceinline__ P make_payload(uint32_t g, float x, float y);
template <>
__device__ __forceinline__ uint32_t make_payload<uint32_t>(uint32_t g, float, float) {
  return g;
}
template <>
__device__ __forceinline__ Rec make_payload<Rec>(uint32_t g, float x, float y) {
  Rec r;
  r.x = (int32_t)(x * kGridF);
  r.y = (int32_t)(y * kGridF);
  r.i = g;
  r.pad = 0;
  return r;
}

template <class P>
struct StageCap {
  static constexpr int value = 8192 / (int)sizeof(P);  // 8 KiB of LDS per wave
};
// Records (k_pass_hull, k_filter_hull) leave room for the sample polygon,
// its wedge table and the exact-test queue within 40 KiB per workgroup.
template <>
struct StageCap<Rec> {
  static constexpr int value = 320;
};

// Exact-test queue of the hull path: points that pass neither cheap test
// wait in LDS until a whole wave's worth (64) can be tested together, so the
// exact tests run with full waves however rare those points are. The fused
// pass of a single set (queue kQueueF) appends a whole batch's points with
// one wave sync when they fit.
constexpr int kQueue = 128;
constexpr int kQueueF = 256;
// Candidate records the fused pass stages per wave before one reservation
// in the shared list (a device-scope atomic on one counter, whose round
// trips serialise: many candidates want few, large flushes). Sized so that
// two workgroups still fit a CU's LDS with the polygon, wedge table and queue.
constexpr int kCapF = 832;
// Candidate records the batch pass stages per wave (its grid runs eight
// workgroups per CU, so its LDS stays small).
constexpr int kCapB = 128;

// The candidates' octagon test is skipped when it removes fewer than 1 in
// kSkipRatio of the first kSkipEst candidate records.
constexpr uint32_t kSkipEst = 1024;
constexpr uint32_t kSkipRatio = 8;
constexpr uint32_t kSkipMin = 1u << 17;  // candidates from which the estimate runs (> kFinalTile)

template <bool LABELS, class P>
__global__ __launch_bounds__(kBlock) void k_filter(const float* __restrict__ xy, uint32_t n,
                                                   uint32_t head, Header* __restrict__ hdr,
                                                   uint64_t* __restrict__ tstat, uint32_t G2,
                                                   P* __restrict__ surv,
                                                   uint32_t* __restrict__ count_out,
                                                   uint8_t* __restrict__ labels,
                                                   P* __restrict__ staging) {
  constexpr int kCapW = StageCap<P>::value;
  __shared__ P s_buf[kWaves][kCapW];
  __shared__ uint32_t s_chunk, s_prefix, s_total;
  __shared__ uint32_t s_cnt[kWaves];
  const Octagon* __restrict__ o = &hdr->oct;
  uint32_t* __restrict__ vidx = hdr->vidx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;

  if (threadIdx.x == 0) s_chunk = atomicAdd(&hdr->tile_ctr, 1u);
  __syncthreads();
  const uint32_t c = s_chunk;
  if (o->status != 0) {
    if (c == G2 - 1 && threadIdx.x == 0) *count_out = kCountDomain;
    return;
  }
  const float bxl = o->box[0], bxh = o->box[1], byl = o->box[2], byh = o->box[3];
  const uint32_t nfull = (n - head) >> 1;
  const bool half = ((n - head) & 1) != 0;
  const uint32_t npt = nfull + (half ? 1u : 0u);        // pairs including the half pair
  const uint32_t rows = (npt + 63) / 64;
  const uint32_t nwaves = G2 * kWaves;
  const uint32_t rw = (rows + nwaves - 1) / nwaves;     // rows per wave
  const uint32_t k = c * kWaves + w;
  const uint32_t r0 = k * rw < rows ? k * rw : rows;
  const uint32_t r1 = r0 + rw < rows ? r0 + rw : rows;
  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * head);
  const float2* __restrict__ p2 = reinterpret_cast<const float2*>(xy);
  // Staging slot 0 of wave k is the first point index it owns (0 for wave 0,
  // which also owns the head point).
  const uint32_t sbase = k == 0 ? 0u : head + 2u * r0 * 64u;
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t cw = 0;  // survivors of this wave so far (wave-uniform)

  auto put = [&](uint32_t pos, const P& v) {
    if (pos < (uint32_t)kCapW) s_buf[w][pos] = v;
    else staging[sbase + pos] = v;
  };

  if (k == 0 && head && lane == 0) {
    const Verdict r = classify<LABELS>(xy[0], xy[1], 0u, o, vidx);
    if (LABELS) labels[0] = r.label;
    if (r.keep) s_buf[0][0] = make_payload<P>(0u, xy[0], xy[1]);
    cw = r.keep ? 1u : 0u;
  }
  cw = __shfl(cw, 0);

  auto load_row = [&](uint32_t r, float4& v) {
    const uint32_t q = r * 64 + lane;
    if (q < nfull) {
      v = ld_stream(&p4[q]);
    } else if (q == nfull && half) {
      const float2 u = p2[head + 2 * q];
      v = make_float4(u.x, u.y, 0.f, 0.f);
    } else {
      v = make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };

  float4 cur[kU], nxt[kU];
  uint32_t r = r0;
  if (r < r1) {
#pragma unroll
    for (int u = 0; u < kU; ++u) load_row(r + u < r1 ? r + u : r1 - 1, cur[u]);
    wait_all_loads();
  }
  while (r < r1) {
    const uint32_t rn = r + kU;
    const bool more = rn < r1;
    if (more) {
#pragma unroll
      for (int u = 0; u < kU; ++u) load_row(rn + u < r1 ? rn + u : r1 - 1, nxt[u]);
    }
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t row = r + u;
      if (row < r1) {  // wave-uniform
        const uint32_t q = row * 64 + lane;
        const bool val1 = q < nfull;
        const bool val0 = val1 || (q == nfull && half);
        const uint32_t g = head + 2 * q;
        const float x0 = cur[u].x, y0 = cur[u].y, x1 = cur[u].z, y1 = cur[u].w;
        const bool in0 = (x0 > bxl) & (x0 < bxh) & (y0 > byl) & (y0 < byh);
        const bool in1 = (x1 > bxl) & (x1 < bxh) & (y1 > byl) & (y1 < byh);
        const bool need0 = val0 & !in0, need1 = val1 & !in1;
        Verdict v0{false, 0}, v1{false, 0};
        if (__ballot(need0 | need1)) {
          if (need0) v0 = classify<LABELS>(x0, y0, g, o, vidx);
          if (need1) v1 = classify<LABELS>(x1, y1, g + 1, o, vidx);
        }
        if (LABELS) {
          if (val0) labels[g] = v0.label;
          if (val1) labels[g + 1] = v1.label;
        }
        const uint64_t b0 = __ballot(v0.keep), b1 = __ballot(v1.keep);
        if (b0 | b1) {
          const uint32_t rank = cw + popc64(b0 & lt) + popc64(b1 & lt);
          if (v0.keep) put(rank, make_payload<P>(g, x0, y0));
          if (v1.keep) put(rank + (v0.keep ? 1u : 0u), make_payload<P>(g + 1, x1, y1));
          cw += popc64(b0) + popc64(b1);
        }
      }
    }
    if (!more) break;
#pragma unroll
    for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
    r = rn;
  }
  if (lane == 0) s_cnt[w] = cw;
  __syncthreads();

  // Look-back: publish this workgroup's count, then add up every earlier
  // workgroup's count, stopping at the nearest one that already published
  // its inclusive prefix.
  if (w == 0) {
    uint32_t total = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) total += s_cnt[i];
    if (lane == 0)
      __hip_atomic_store(&tstat[c], ((c == 0 ? 2ull : 1ull) << 32) | total, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    if (c > 0) {
      constexpr int kSlots = 16;  // 16 * 64 = 1024 >= G2
      uint64_t word[kSlots];
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        const int64_t idx = (int64_t)c - 1 - lane - 64 * i;
        word[i] = idx >= 0 ? __hip_atomic_load(&tstat[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                           : (2ull << 32);
      }
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        const int64_t idx = (int64_t)c - 1 - lane - 64 * i;
        if (idx >= 0) {
          while ((word[i] >> 32) == 0) {
            __builtin_amdgcn_s_sleep(2);
            word[i] = __hip_atomic_load(&tstat[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
      }
      // Distance (in workgroups) to the nearest inclusive word.
      int near = 1 << 30;
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        const int d = lane + 64 * i;
        if ((word[i] >> 32) == 2 && d < near) near = d;
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const int o2 = __shfl_xor(near, off);
        near = o2 < near ? o2 : near;
      }
      uint64_t sum = 0;
#pragma unroll
      for (int i = 0; i < kSlots; ++i) {
        const int d = lane + 64 * i;
        if (d <= near) sum += (uint32_t)word[i];
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
      excl = sum;
      if (lane == 0)
        __hip_atomic_store(&tstat[c], (2ull << 32) | (uint32_t)(excl + total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_prefix = (uint32_t)excl;
      s_total = total;
    }
  }
  __syncthreads();
  const uint32_t prefix = s_prefix;
  if (c == G2 - 1 && threadIdx.x == 0) *count_out = prefix + s_total;
  uint32_t off = prefix;
  for (int i = 0; i < w; ++i) off += s_cnt[i];
  const uint32_t nb = cw < (uint32_t)kCapW ? cw : (uint32_t)kCapW;
  for (uint32_t i = lane; i < nb; i += 64) surv[off + i] = s_buf[w][i];
  for (uint32_t i = kCapW + lane; i < cw; i += 64) surv[off + i] = staging[sbase + i];
}

// The octagon test (Alg. 1/2 with Sec. I's boundary rule) on the fused
// pass's candidate records; survivors are appended to `surv` (one atomic per
// wave and 64 candidates). Run by k_filter_hull's grid after a fused pass
// with a usable sample polygon.
__device__ void cand_filter(const Rec* __restrict__ cand, const uint32_t* __restrict__ cand_count,
                            const Octagon* __restrict__ o, uint32_t* __restrict__ vidx,
                            Rec* __restrict__ surv, uint32_t* __restrict__ count_out,
                            uint32_t* __restrict__ ncand_out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *ncand_out = *cand_count;
  if (o->status != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_out = kCountDomain;
    return;
  }
  // Each round a workgroup tests KR records per thread and reserves room for
  // all its survivors with one atomic (a counter shared by the whole grid
  // serialises, so reservations are kept few: many candidates take 16 per
  // thread, few take 4 and spread over more workgroups).
  __shared__ uint32_t s_base;
  const uint32_t m = *cand_count;
  if (blockIdx.x * kBlock * 4 >= m) return;  // no records for this workgroup
  auto rounds = [&](auto kr_tag) {
    constexpr uint32_t KR = decltype(kr_tag)::value;
    constexpr uint32_t kChunk = kBlock * KR;
    for (uint32_t s0 = blockIdx.x * kChunk; s0 < m; s0 += gridDim.x * kChunk) {
      Rec r[KR];
      uint32_t km = 0, cnt = 0;
      // all loads first (clamped to the last record), then the tests
#pragma unroll
      for (uint32_t j = 0; j < KR; ++j) {
        const uint32_t i = s0 + j * kBlock + threadIdx.x;
        r[j] = cand[i < m ? i : m - 1];
      }
#pragma unroll
      for (uint32_t j = 0; j < KR; ++j) {
        const uint32_t i = s0 + j * kBlock + threadIdx.x;
        if (i < m && classify<false>((float)r[j].x * (1.0f / kGridF), (float)r[j].y * (1.0f / kGridF),
                                     r[j].i, o, vidx).keep) {
          km |= 1u << j;
          ++cnt;
        }
      }
      uint32_t total;
      const uint32_t off = block_excl_scan(cnt, total);
      if (threadIdx.x == 0 && total) s_base = atomicAdd(count_out, total);
      __syncthreads();
      uint32_t q = s_base + off;
#pragma unroll
      for (uint32_t j = 0; j < KR; ++j)
        if (km & (1u << j)) surv[q++] = r[j];
      __syncthreads();  // s_base is rewritten next round
    }
  };
  if (m >= (1u << 18)) rounds(IntC<16>{});
  else rounds(IntC<4>{});
}

// Pass 2 of the hull path when there is no fused pass (fewer than kSampleMin
// points, or no usable sample polygon). The hull pass sorts its candidates,
// so their order is free: the grid walks the points exactly as pass 1 does
// (each wave takes every nw-th batch of kU rows, next batch's loads issued
// before the current one is tested), tests them (octagon box, then the
// per-wave queue of exact tests), stages survivor records per wave in LDS and
// flushes them to `surv` with one atomic reservation per flush -- no ordering
// and no look-back. The head point and an odd last point go to workgroup 0.
__global__ __launch_bounds__(kBlock) void k_filter_hull(const float* __restrict__ xy, uint32_t n,
                                                        uint32_t head, Header* __restrict__ hdr,
                                                        Rec* __restrict__ surv,
                                                        uint32_t* __restrict__ count_out,
                                                        const SamplePoly* __restrict__ gate,
                                                        const Rec* __restrict__ cand,
                                                        const uint32_t* __restrict__ cand_count,
                                                        uint32_t* __restrict__ ncand_out,
                                                        const uint32_t* __restrict__ mode_in,
                                                        uint32_t* __restrict__ mode_out,
                                                        const double* __restrict__ partials,
                                                        const uint32_t* __restrict__ part_bad,
                                                        uint32_t nparts, Result* __restrict__ res) {
  // The octagon lives in LDS: one read (or one build) per workgroup, not a
  // global read per tested point. The smallest index per vertex is not used
  // on the hull path (the hull keeps the smallest index of equal points
  // itself), so vidx is workgroup-local.
  __shared__ Octagon s_oct;
  __shared__ uint32_t s_vidx[8];
  const bool use_cand = gate && gate->nv >= 3;
  if (partials) {
    // After a fused pass every workgroup with work combines the pass's
    // partials and builds the octagon itself (no separate launch);
    // workgroup 0 publishes it (later kernels check its status) and resets
    // the per-call counters; the survivor count was reset before the pass.
    if (use_cand && blockIdx.x != 0 && blockIdx.x * kBlock * 4 >= *cand_count) return;
    Keys k;
    const uint32_t bad = combine_partials(partials, part_bad, nparts, k);
    if (threadIdx.x < 64) octagon_wave(k, s_oct, s_vidx, bad);
    __syncthreads();
    if (blockIdx.x == 0) {
      if (threadIdx.x < sizeof(Octagon) / 4)
        reinterpret_cast<uint32_t*>(&hdr->oct)[threadIdx.x] = reinterpret_cast<const uint32_t*>(&s_oct)[threadIdx.x];
      if (threadIdx.x < 64) reset_call_state(hdr, res, false);
    }
  } else {
    if (threadIdx.x < sizeof(Octagon) / 4)
      reinterpret_cast<uint32_t*>(&s_oct)[threadIdx.x] = reinterpret_cast<const uint32_t*>(&hdr->oct)[threadIdx.x];
    if (threadIdx.x < 8) s_vidx[threadIdx.x] = 0xFFFFFFFFu;
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *mode_out = mode_in ? *mode_in : 0u;
  // After a fused pass with a usable sample polygon only its candidates need
  // the octagon test; otherwise this is the second read of the points.
  if (use_cand) {
    // Many candidates that the octagon barely thins (points near a smooth
    // curve, whose sample polygon already holds most of the octagon): the
    // test is skipped and the candidate records are the survivors. Every
    // workgroup estimates on the same first records, so all decide alike;
    // only when the hull path will not read the survivor records (more than
    // one block of them) -- the hull is the same either way, the candidates
    // containing every hull vertex.
    const uint32_t m = *cand_count;
    if (m >= kSkipMin && s_oct.status == 0) {
      __shared__ uint32_t s_rm[kWaves];
      uint32_t rm = 0;
#pragma unroll
      for (uint32_t e = 0; e < kSkipEst / kBlock; ++e) {
        const Rec r = cand[threadIdx.x + e * kBlock];
        rm += classify<false>((float)r.x * (1.0f / kGridF), (float)r.y * (1.0f / kGridF), r.i, &s_oct,
                              s_vidx).keep ? 0u : 1u;
      }
      rm = wave_allreduce(rm, [](uint32_t a, uint32_t b) { return a + b; });
      if ((threadIdx.x & 63) == 0) s_rm[threadIdx.x >> 6] = rm;
      __syncthreads();
      uint32_t removed = 0;
#pragma unroll
      for (int i = 0; i < kWaves; ++i) removed += s_rm[i];
      if (removed * kSkipRatio < kSkipEst) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
          *ncand_out = m;
          *count_out = m;
          res->cand_surv = 1;
        }
        return;
      }
    }
    cand_filter(cand, cand_count, &s_oct, s_vidx, surv, count_out, ncand_out);
    return;
  }
  constexpr int kCapW = StageCap<Rec>::value;
  __shared__ Rec s_buf[kWaves][kCapW];
  __shared__ float s_qx[kWaves][kQueue], s_qy[kWaves][kQueue];
  __shared__ uint32_t s_qg[kWaves][kQueue];
  const Octagon* __restrict__ o = &s_oct;
  uint32_t* __restrict__ vidx = s_vidx;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  if (o->status != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *count_out = kCountDomain;
    return;
  }
  const float bxl = o->box[0], bxh = o->box[1], byl = o->box[2], byh = o->box[3];

  uint32_t cw = 0, qn = 0;  // staged survivors, queued points (wave-uniform)
  auto flush = [&]() {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(count_out, cw);
    base = __shfl(base, 0);
    for (uint32_t i = lane; i < cw; i += 64) surv[base + i] = s_buf[w][i];
    wave_sync();
    cw = 0;
  };
  auto exact_keep = [&](float x, float y, uint32_t g) {
    return classify<false>(x, y, g, o, vidx).keep;
  };
  auto drain = [&](uint32_t base, uint32_t cnt) {
    float x = 0.f, y = 0.f;
    uint32_t g = 0;
    if (lane < (int)cnt) { x = s_qx[w][base + lane]; y = s_qy[w][base + lane]; g = s_qg[w][base + lane]; }
    wave_sync();
    const bool keep = lane < (int)cnt && exact_keep(x, y, g);
    const uint64_t b = __ballot(keep);
    if (!b) return;
    if (cw + popc64(b) > (uint32_t)kCapW) flush();
    if (keep) s_buf[w][cw + popc64(b & lt)] = make_payload<Rec>(g, x, y);
    cw += popc64(b);
  };
  auto push = [&](bool q, float x, float y, uint32_t g) {
    const uint64_t m = __ballot(q);
    if (!m) return;
    if (q) {
      const uint32_t pos = qn + popc64(m & lt);
      s_qx[w][pos] = x; s_qy[w][pos] = y; s_qg[w][pos] = g;
    }
    qn += popc64(m);
    wave_sync();
    if (qn >= 64) {
      qn -= 64;
      drain(qn, 64);
    }
  };
  auto test_pair = [&](const float4& v, uint32_t q, bool val) {
    const uint32_t g = head + 2 * q;
    const bool in0 = (v.x > bxl) & (v.x < bxh) & (v.y > byl) & (v.y < byh);
    const bool in1 = (v.z > bxl) & (v.z < bxh) & (v.w > byl) & (v.w < byh);
    const bool t0 = val & !in0, t1 = val & !in1;
    if (__ballot(t0 | t1)) {
      push(t0, v.x, v.y, g);
      push(t1, v.z, v.w, g + 1);
    }
  };

  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * head);
  const uint32_t nfull = (n - head) >> 1;
  const uint32_t gw = blockIdx.x * kWaves + w;
  const uint32_t nw = gridDim.x * kWaves;
  const uint32_t per_batch = kU * 64;
  const uint32_t nbatch = (nfull + per_batch - 1) / per_batch;
  if (gw < nbatch) {
    float4 cur[kU], nxt[kU];
    uint32_t b = gw;
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const uint32_t q = b * per_batch + u * 64 + lane;
      cur[u] = ld_stream(&p4[q < nfull ? q : nfull - 1]);
    }
    wait_all_loads();
    while (true) {
      const uint32_t bn = b + nw;
      const bool more = bn < nbatch;
      if (more) {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const uint32_t q = bn * per_batch + u * 64 + lane;
          nxt[u] = ld_stream(&p4[q < nfull ? q : nfull - 1]);
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint32_t q = b * per_batch + u * 64 + lane;
        test_pair(cur[u], q, q < nfull);
      }
      if (!more) break;
#pragma unroll
      for (int u = 0; u < kU; ++u) cur[u] = nxt[u];
      b = bn;
    }
  }
  if (qn) drain(0, qn);
  if (cw) flush();
  // The head point (xy 8 mod 16 bytes aligned) and an odd last point.
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t single[2];
    int ns = 0;
    if (head) single[ns++] = 0;
    if ((n - head) & 1) single[ns++] = n - 1;
    for (int i = 0; i < ns; ++i) {
      const uint32_t g = single[i];
      const float x = xy[2 * (size_t)g], y = xy[2 * (size_t)g + 1];
      if (exact_keep(x, y, g)) surv[atomicAdd(count_out, 1u)] = make_payload<Rec>(g, x, y);
    }
  }
}

// Hull path from kSampleMin points, with the sample polygon built first: one
// read of the points does pass 1 -- the exact 8-way extremes, per-workgroup
// partials and the domain flag, as k_reduce8 -- and in the same pass keeps the
// points not strictly inside the sample polygon as candidate records (inner
// region test, then the exact wedge test through the per-wave queue). The
// octagon test then runs on the candidates alone (cand_filter): every point
// it would keep is either a candidate or strictly inside a polygon of input
// points, which no hull vertex is. Without a usable polygon this is pass 1
// only, and k_filter_hull makes the second read.
//
// With a polygon, the extremes are taken over the points outside its inner
// region (disc or octagon, see in_inner) only: a point strictly inside the
// convex hull of other input points is not extreme in any direction, so no
// key it would give can win. Points inside the region are finite and inside
// the grid square, so their domain check is
// the grid test alone, done as the largest fractional part of the scaled
// coordinates (zero exactly when every one is a grid value); points outside
// get their keys and the full check of keys_add (NaN, infinities, range
// through the keys) when the exact-test queue drains, a wave at a time.
__global__ __launch_bounds__(kBlock) void k_pass_hull(const float* __restrict__ xy, uint32_t n,
                                                      uint32_t head, double* __restrict__ partials,
                                                      uint32_t* __restrict__ part_bad,
                                                      const SamplePoly* __restrict__ poly,
                                                      SampleDirs* __restrict__ sd,
                                                      Rec* __restrict__ cand,
                                                      uint32_t narrow_blocks) {
  constexpr int kCapW = kCapF;
  __shared__ Rec s_buf[kWaves][kCapW];
  __shared__ int32_t s_pvx[kPolyMax], s_pvy[kPolyMax];
  __shared__ uint32_t s_lut[kLutBins];
  __shared__ float s_qx[kWaves][kQueueF], s_qy[kWaves][kQueueF];
  __shared__ uint32_t s_qg[kWaves][kQueueF];
  __shared__ uint32_t s_bad;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t pnv = min(poly->nv, (uint32_t)kPolyMax);
  const bool use_sp = pnv >= 3;
  const uint32_t* __restrict__ lut = sd->lut;
  uint32_t* __restrict__ cand_count = &sd->cand;
  __shared__ uint32_t s_est[kWaves];
  // Inner region in grid units (scaled coordinates t = 2^20 x are exact):
  // the disc, or the octagon when its area is larger (one test per point).
  float gcx = 0.f, gcy = 0.f, gr2 = 0.f, gos = 0.f, got = 0.f;
  int32_t pcxi = 0, pcyi = 0;
  bool use_oct = false;
  uint32_t act = gridDim.x;
  auto in_oct = [&](float dx, float dy) {
    const float ax = __builtin_fabsf(dx), ay = __builtin_fabsf(dy);
    return (ax < gos) & (ay < gos) & (ax + ay < got);
  };
  auto inner = [&](float tx, float ty) {
    const float dx = tx - gcx, dy = ty - gcy;
    return use_oct ? in_oct(dx, dy) : __builtin_fmaf(dx, dx, dy * dy) < gr2;
  };
  if (use_sp) {
    pcxi = poly->cx;
    pcyi = poly->cy;
    gcx = (float)pcxi;
    gcy = (float)pcyi;
    gr2 = poly->r2 * 0x1p40f;
    gos = poly->os * kGridF;
    got = poly->ot * kGridF;
    const float cut = __builtin_fmaxf(2.0f * gos - got, 0.0f);
    use_oct = 4.0f * gos * gos - 2.0f * cut * cut > 3.14159265f * gr2;
    // Share of points outside the inner region, estimated on kEstPer kBlock
    // points spread over the input (the same ones in every workgroup, so all take
    // the same decision). Few: stream with narrow_blocks workgroups (fewer
    // concurrent streams read HBM faster); the rest only write empty
    // partials. Many: the whole grid, whose waves hide the exact tests.
    float ex[kEstPer], ey[kEstPer];
#pragma unroll
    for (uint32_t e = 0; e < kEstPer; ++e) {
      const size_t q = (size_t)((uint64_t(threadIdx.x + e * kBlock) * n) / (kBlock * kEstPer));
      ex[e] = xy[2 * q];
      ey[e] = xy[2 * q + 1];
    }
    uint32_t nout = 0;
#pragma unroll
    for (uint32_t e = 0; e < kEstPer; ++e) {
      const uint64_t ob = __builtin_amdgcn_ballot_w64(!inner(ex[e] * kGridF, ey[e] * kGridF));
      nout += popc64(ob);
    }
    if (lane == 0) s_est[w] = nout;
    __syncthreads();
    uint32_t est = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) est += s_est[i];
    if (est * kWideRatio <= kBlock * kEstPer) act = min(narrow_blocks, gridDim.x);
  }
  if (blockIdx.x == 0 && threadIdx.x == 0)
    sd->mode = (use_sp ? 1u : 0u) | (use_oct ? 2u : 0u) | (use_sp && act == gridDim.x ? 4u : 0u);
  if (blockIdx.x >= act) {
    if (threadIdx.x == 0) {
      Keys e;
      keys_init(e);
      keys_to_array(e, partials + size_t(blockIdx.x) * 8);
      part_bad[blockIdx.x] = 0;
    }
    return;
  }
  if (use_sp) {
    for (uint32_t i = threadIdx.x; i < pnv; i += kBlock) { s_pvx[i] = poly->vx[i]; s_pvy[i] = poly->vy[i]; }
    for (uint32_t i = threadIdx.x; i < kLutBins; i += kBlock) s_lut[i] = lut[i];
  }
  if (threadIdx.x == 0) s_bad = 0;
  __syncthreads();

  Keys k;
  keys_init(k);
  bool bad = false;
  float frac = 0.f;         // largest fractional part of a scaled coordinate (inner points)
  uint32_t cw = 0, qn = 0;  // staged candidates, queued points (wave-uniform)
  auto flush = [&]() {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(cand_count, cw);
    base = __shfl(base, 0);
    for (uint32_t i = lane; i < cw; i += 64) cand[base + i] = s_buf[w][i];
    wave_sync();
    cw = 0;
  };
  auto outside = [&](float x, float y) {
    return !poly_lut_inside(s_pvx, s_pvy, pnv, s_lut, pcxi, pcyi, (int32_t)(x * kGridF),
                            (int32_t)(y * kGridF));
  };
  // Queued points (all outside the inner region): their keys, then the exact test.
  auto drain = [&](uint32_t base, uint32_t cnt) {
    float x = 0.f, y = 0.f;
    uint32_t g = 0;
    if (lane < (int)cnt) {
      x = s_qx[w][base + lane]; y = s_qy[w][base + lane]; g = s_qg[w][base + lane];
      keys_add(k, x, y, bad);
    }
    wave_sync();
    const bool keep = lane < (int)cnt && outside(x, y);
    const uint64_t b = __ballot(keep);
    if (!b) return;
    if (cw + popc64(b) > (uint32_t)kCapW) flush();
    if (keep) s_buf[w][cw + popc64(b & lt)] = make_payload<Rec>(g, x, y);
    cw += popc64(b);
  };
  // Points outside the inner region (mask = the wave's ballot) join the queue.
  auto push = [&](uint64_t m, float x, float y, uint32_t g) {
    if (!m) return;
    if ((m >> lane) & 1ull) {
      const uint32_t pos = qn + popc64(m & lt);
      s_qx[w][pos] = x; s_qy[w][pos] = y; s_qg[w][pos] = g;
    }
    qn += popc64(m);
    wave_sync();
    if (qn >= 64) {
      qn -= 64;
      drain(qn, 64);
    }
  };

  const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * head);
  const uint32_t nfull = (n - head) >> 1;
  const uint32_t gw = blockIdx.x * kWaves + w;
  const uint32_t nw = act * kWaves;
  const uint32_t per_batch = kUF * 64;
  const uint32_t nbatch = (nfull + per_batch - 1) / per_batch;
  // One streaming loop per mode, uniform over the grid: no polygon (keys of
  // every point), inner disc, inner octagon.
  auto stream = [&](auto mode_tag) {
    constexpr int MODE = decltype(mode_tag)::value;
    constexpr bool SP = MODE != 0;
    float4 cur[kUF], nxt[kUF];
    uint32_t b = gw;
#pragma unroll
    for (int u = 0; u < kUF; ++u) {
      const uint32_t q = b * per_batch + u * 64 + lane;
      cur[u] = ld_stream(&p4[q < nfull ? q : nfull - 1]);
    }
    wait_all_loads();
    while (true) {
      const uint32_t bn = b + nw;
      const bool more = bn < nbatch;
      if (more) {
#pragma unroll
        for (int u = 0; u < kUF; ++u) {
          const uint32_t q = bn * per_batch + u * 64 + lane;
          nxt[u] = ld_stream(&p4[q < nfull ? q : nfull - 1]);
        }
      }
      if constexpr (!SP) {
#pragma unroll
        for (int u = 0; u < kUF; ++u) {
          // Lanes past the end hold a copy of the last pair: harmless for
          // the extremes.
          keys_add(k, cur[u].x, cur[u].y, bad);
          keys_add(k, cur[u].z, cur[u].w, bad);
        }
      } else {
        // Grid check and inner-region votes for the whole batch, then one branch:
        // a branch on each row's vote stalls the wave on every row. Lanes
        // past the end hold a copy of the last pair and vote no.
        uint64_t mk[2 * kUF];
        uint64_t any = 0;
#pragma unroll
        for (int u = 0; u < kUF; ++u) {
          const float4 v = cur[u];
          const float t0 = v.x * kGridF, t1 = v.y * kGridF, t2 = v.z * kGridF, t3 = v.w * kGridF;
          frac = __builtin_fmaxf(frac, __builtin_fmaxf(__builtin_amdgcn_fractf(t0),
                                                       __builtin_amdgcn_fractf(t1)));
          frac = __builtin_fmaxf(frac, __builtin_fmaxf(__builtin_amdgcn_fractf(t2),
                                                       __builtin_amdgcn_fractf(t3)));
          bool i0, i1;
          if constexpr (MODE == 1) {
            const float dx0 = t0 - gcx, dy0 = t1 - gcy, dx1 = t2 - gcx, dy1 = t3 - gcy;
            i0 = __builtin_fmaf(dx0, dx0, dy0 * dy0) < gr2;
            i1 = __builtin_fmaf(dx1, dx1, dy1 * dy1) < gr2;
          } else {
            i0 = in_oct(t0 - gcx, t1 - gcy);
            i1 = in_oct(t2 - gcx, t3 - gcy);
          }
          const uint64_t val = __builtin_amdgcn_ballot_w64(b * per_batch + u * 64 + lane < nfull);
          mk[2 * u] = __builtin_amdgcn_ballot_w64(!i0) & val;
          mk[2 * u + 1] = __builtin_amdgcn_ballot_w64(!i1) & val;
          any |= mk[2 * u] | mk[2 * u + 1];
        }
        if (any) {
          uint32_t tot = 0;
#pragma unroll
          for (int j = 0; j < 2 * kUF; ++j) tot += popc64(mk[j]);
          if (qn + tot <= (uint32_t)kQueueF) {
            // The whole batch's outside points join the queue at once (one
            // wave sync), then full waves of them are drained.
            uint32_t pos = qn;
#pragma unroll
            for (int u = 0; u < kUF; ++u) {
              const uint32_t g = head + 2 * (b * per_batch + u * 64 + lane);
              const uint64_t m0 = mk[2 * u], m1 = mk[2 * u + 1];
              if ((m0 >> lane) & 1ull) {
                const uint32_t p0 = pos + popc64(m0 & lt);
                s_qx[w][p0] = cur[u].x; s_qy[w][p0] = cur[u].y; s_qg[w][p0] = g;
              }
              pos += popc64(m0);
              if ((m1 >> lane) & 1ull) {
                const uint32_t p1 = pos + popc64(m1 & lt);
                s_qx[w][p1] = cur[u].z; s_qy[w][p1] = cur[u].w; s_qg[w][p1] = g + 1;
              }
              pos += popc64(m1);
            }
            qn = pos;
            wave_sync();
            while (qn >= 64) {
              qn -= 64;
              drain(qn, 64);
            }
          } else {
#pragma unroll
            for (int u = 0; u < kUF; ++u) {
              const uint32_t g = head + 2 * (b * per_batch + u * 64 + lane);
              push(mk[2 * u], cur[u].x, cur[u].y, g);
              push(mk[2 * u + 1], cur[u].z, cur[u].w, g + 1);
            }
          }
        }
      }
      if (!more) break;
#pragma unroll
      for (int u = 0; u < kUF; ++u) cur[u] = nxt[u];
      b = bn;
    }
  };
  if (gw < nbatch) {
    if (!use_sp) stream(IntC<0>{});
    else if (!use_oct) stream(IntC<1>{});
    else stream(IntC<2>{});
  }
  bad |= frac != 0.f;
  if (use_sp) {
    if (qn) drain(0, qn);
    if (cw) flush();
  }
  // The head point (xy 8 mod 16 bytes aligned) and an odd last point.
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    uint32_t single[2];
    int ns = 0;
    if (head) single[ns++] = 0;
    if ((n - head) & 1) single[ns++] = n - 1;
    for (int i = 0; i < ns; ++i) {
      const uint32_t g = single[i];
      const float x = xy[2 * (size_t)g], y = xy[2 * (size_t)g + 1];
      keys_add(k, x, y, bad);
      if (use_sp && outside(x, y)) cand[atomicAdd(cand_count, 1u)] = make_payload<Rec>(g, x, y);
    }
  }
  const uint64_t badmask = __ballot(bad);
  if (lane == 0 && badmask) s_bad = 1;
  block_keys(k);
  if (threadIdx.x == 0) {
    keys_to_array(k, partials + size_t(blockIdx.x) * 8);
    part_bad[blockIdx.x] = s_bad;
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

__global__ void k_set_u32(uint32_t* __restrict__ p, uint32_t v) {
  if (threadIdx.x == 0) *p = v;
}

// ------------------------------------------------------------- batch mode
//
// Thousands of independent sets in one stream-ordered sequence of kernels
// (capturable in a graph, no host synchronisation): a plan kernel cuts every
// set into tiles of `tile` points; pass 1 reduces tiles (workgroups take
// tiles with a fixed stride, no shared counter) and folds them into the set's
// keys with 64-bit atomic max on an order-preserving encoding; one wave per
// set builds its octagon; pass 2 filters tiles and appends survivor records
// (set-local indices) to the set's own slice of a record buffer.

// Order-preserving map from fp64 to uint64 (for atomic max on keys).
__device__ __forceinline__ uint64_t enc_f64(double d) {
  const uint64_t b = (uint64_t)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double dec_f64(uint64_t e) {
  const uint64_t b = (e >> 63) ? (e & 0x7FFFFFFFFFFFFFFFull) : ~e;
  return __longlong_as_double((long long)b);
}

// Tile lists, per-set state and the sampler's list. Workgroup b owns sets
// b kBlock .. b kBlock + kBlock - 1, one per thread. Every workgroup first
// reads all offsets (a few KB, from L2) for the batch-wide facts: whether
// they are valid (else every set is empty), the pass tiles of the sets before
// its own and in all, and the sampled sets (batch_chunks > 0) per chunk count,
// before its own and in all. It then writes its sets' pass tiles in set
// order, resets their SetState, clears the polygon of each set without a
// sample, and enters its sampled sets in the sampler's list, ordered by chunk
// count from 4 down to 1 and by set within a count, so that the longest
// sampler jobs are taken first.
__global__ __launch_bounds__(kBlock) void k_batch_plan(const uint64_t* __restrict__ off,
                                                       uint32_t nsets, uint64_t total_points,
                                                       uint32_t tile, uint32_t sample_min,
                                                       BatchHdr* __restrict__ bh,
                                                       SetState* __restrict__ sets,
                                                       SetTile* __restrict__ tiles,
                                                       SamplePoly* __restrict__ polys,
                                                       uint32_t* __restrict__ slist) {
  static_assert(kBatchChunksMax == 4, "one list bucket per chunk count 4, 3, 2, 1");
  constexpr int kVals = 10;  // tiles before, tiles in all, 4 buckets before, 4 in all
  __shared__ uint32_t s_bad;
  __shared__ uint32_t s_red[kWaves][kVals];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t first = blockIdx.x * kBlock;
  if (threadIdx.x == 0) s_bad = (off[0] != 0 || off[nsets] != total_points) ? 1u : 0u;
  __syncthreads();
  for (uint32_t s = threadIdx.x; s < nsets; s += kBlock)
    if (off[s + 1] < off[s]) s_bad = 1u;
  __syncthreads();
  const bool bad = s_bad != 0;
  // Sizes below 2^32 (the batch total is), so 32-bit divisions.
  uint32_t v[kVals] = {};
  for (uint32_t s = threadIdx.x; s < nsets && !bad; s += kBlock) {
    const uint32_t n = (uint32_t)(off[s + 1] - off[s]);
    const uint32_t t = n / tile + (n % tile ? 1u : 0u), c = batch_chunks(n, sample_min);
    v[1] += t;
    if (s < first) v[0] += t;
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
      const uint32_t hit = c == 4 - k ? 1u : 0u;  // bucket k: chunk count 4 - k
      v[6 + k] += hit;
      v[2 + k] += s < first ? hit : 0u;
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
  const uint32_t a = own ? (uint32_t)off[s] : 0u;
  const uint32_t b = own && !bad ? (uint32_t)off[s + 1] : a;
  const uint32_t c = own && !bad ? batch_chunks(b - a, sample_min) : 0u;
  uint32_t unused;
  uint32_t t = v[0] + block_excl_scan((b - a) / tile + ((b - a) % tile ? 1u : 0u), unused);
  for (uint32_t p = a; p < b; p += tile) {
    SetTile st;
    st.set = s; st.begin = p; st.end = b - p > tile ? p + tile : b; st.pad = 0;
    tiles[t++] = st;
  }
  if (own) {
    SetState& ss = sets[s];
    for (int k = 0; k < 8; ++k) ss.key[k] = 0ull;
    ss.bad = 0;
    ss.done = 0;
    ss.ncand = 0;
    for (int r = 0; r <= kBatchRounds; ++r) ss.cnt[r] = 0;
    if (!c) polys[s].nv = 0;
  }
  // Rank among this workgroup's sets of the same chunk count: two scans of
  // two 16-bit counters each (at most kBlock per bucket).
  const uint32_t k = 4 - c;  // bucket (4 = none)
  const uint32_t e01 = block_excl_scan(c && k < 2 ? 1u << (16 * k) : 0u, unused);
  const uint32_t e23 = block_excl_scan(c && k >= 2 ? 1u << (16 * (k - 2)) : 0u, unused);
  if (c) {
    const uint32_t rank = ((k < 2 ? e01 : e23) >> (16 * (k & 1))) & 0xFFFFu;
    uint32_t start = 0;
#pragma unroll
    for (uint32_t j = 0; j < 4; ++j) start += j < k ? v[6 + j] : (j == k ? v[2 + j] : 0u);
    slist[start + rank] = s;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    bh->ntiles = v[1];
    bh->bad_offsets = bad ? 1u : 0u;
    for (int r = 0; r <= kBatchRounds; ++r) bh->nround[r] = 0;
    bh->nsampled = v[6] + v[7] + v[8] + v[9];
    bh->sample_next = 0;
    bh->refine_next = 0;
    bh->pass_next = 0;
  }
}

// One wave per set: decode the set's keys and build its octagon.
__global__ __launch_bounds__(kBlock) void k_batch_octagon(const uint64_t* __restrict__ off,
                                                          uint32_t nsets,
                                                          const BatchHdr* __restrict__ bh,
                                                          SetState* __restrict__ sets) {
  const uint32_t s = blockIdx.x * kWaves + (threadIdx.x >> 6);
  if (s >= nsets || bh->bad_offsets) return;
  if (off[s + 1] <= off[s]) return;
  SetState& ss = sets[s];
  Keys k;
  k.mxE = dec_f64(ss.key[0]); k.mxN = dec_f64(ss.key[1]);
  k.mxNE = dec_f64(ss.key[2]); k.mxSE = dec_f64(ss.key[3]);
  k.mnE = -dec_f64(ss.key[4]); k.mnN = -dec_f64(ss.key[5]);
  k.mnNE = -dec_f64(ss.key[6]); k.mnSE = -dec_f64(ss.key[7]);
  octagon_wave(k, ss.oct, ss.vidx, ss.bad);
}

// The single read of a tile (pass 1 and the polygon test, as k_pass_hull
// for one set): with the set's sample polygon, the grid check of every point
// (fractional parts) and the inner-region test; points outside the region
// get their keys and the exact polygon test through the wave's queue, and
// those not strictly inside become candidate records in the set's slice of
// `cand` (set-local indices). Without a polygon (small sets) every point
// gets its keys and becomes a candidate. The tile's keys go into the set's
// with 64-bit atomic max on an order-preserving encoding.
__global__ __launch_bounds__(kBlock) void k_batch_pass(const float* __restrict__ xy,
                                                       const uint64_t* __restrict__ off,
                                                       BatchHdr* __restrict__ bh,
                                                       const SetTile* __restrict__ tiles,
                                                       SetState* __restrict__ sets,
                                                       const SamplePoly* __restrict__ polys,
                                                       Rec* __restrict__ cand) {
  __shared__ int32_t s_pvx[kBatchDirs], s_pvy[kBatchDirs];
  __shared__ float s_qx[kWaves][kQueue], s_qy[kWaves][kQueue];
  __shared__ uint32_t s_qg[kWaves][kQueue];
  __shared__ Rec s_cb[kWaves][kCapB];  // staged candidate records of the wave
  const uint32_t ntiles = bh->ntiles;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint64_t lt = (1ull << lane) - 1ull;
  __shared__ uint32_t s_t;
  for (;;) {
    // Tiles through a shared counter: a workgroup that drew short tiles
    // takes more instead of waiting on a fixed share.
    __syncthreads();  // every thread has read s_t
    if (threadIdx.x == 0) s_t = atomicAdd(&bh->pass_next, 1u);
    __syncthreads();
    const uint32_t t = s_t;
    if (t >= ntiles) break;
    const SetTile st = tiles[t];
    SetState& ss = sets[st.set];
    // The set's sample polygon, if it has one (block-uniform).
    const SamplePoly* __restrict__ sp = &polys[st.set];
    const uint32_t pnv = min(sp->nv, (uint32_t)kBatchDirs);
    const bool use_sp = pnv >= 3;
    float pcx = 0.f, pcy = 0.f, pr2 = 0.f, pos = 0.f, pot = 0.f;
    __syncthreads();  // the previous tile is done with s_pvx / s_pvy
    if (use_sp) {
      for (uint32_t i = threadIdx.x; i < pnv; i += kBlock) { s_pvx[i] = sp->vx[i]; s_pvy[i] = sp->vy[i]; }
      pcx = (float)sp->cx * (1.0f / kGridF);
      pcy = (float)sp->cy * (1.0f / kGridF);
      pr2 = sp->r2;
      pos = sp->os;
      pot = sp->ot;
    }
    __syncthreads();
    const uint32_t base = (uint32_t)off[st.set];
    const uint32_t a = st.begin, b = st.end;
    const uint32_t a2 = a + (a & 1u);
    const uint32_t npairs = b > a2 ? (b - a2) >> 1 : 0;
    const uint32_t nrows = (npairs + 63) / 64;
    const float4* __restrict__ p4 = reinterpret_cast<const float4*>(xy + 2 * (size_t)a2);
    Keys k;
    keys_init(k);
    bool bad = false;
    float frac = 0.f;  // largest fractional part of a scaled coordinate (inner points)
    uint32_t qn = 0, cw = 0;
    // Staged candidates go to the set's slice with one reservation per
    // flush (a full buffer, or the end of the tile).
    auto flush = [&]() {
      uint32_t p = 0;
      if (lane == 0) p = atomicAdd(&ss.ncand, cw);
      p = __shfl(p, 0);
      for (uint32_t i = lane; i < cw; i += 64) cand[base + p + i] = s_cb[w][i];
      wave_sync();
      cw = 0;
    };
    auto emit = [&](bool keep, float x, float y, uint32_t gl) {
      const uint64_t bk = __ballot(keep);
      if (!bk) return;
      if (cw + popc64(bk) > (uint32_t)kCapB) flush();
      if (keep) s_cb[w][cw + popc64(bk & lt)] = make_payload<Rec>(gl, x, y);
      cw += popc64(bk);
    };
    // Queued points (outside the inner region): keys, then the exact test.
    auto drain = [&](uint32_t qb, uint32_t cnt) {
      float x = 0.f, y = 0.f;
      uint32_t gl = 0;
      if (lane < (int)cnt) {
        x = s_qx[w][qb + lane]; y = s_qy[w][qb + lane]; gl = s_qg[w][qb + lane];
        keys_add(k, x, y, bad);
      }
      wave_sync();
      const bool keep = lane < (int)cnt &&
                        !poly_strict_inside(s_pvx, s_pvy, pnv, (int32_t)(x * kGridF), (int32_t)(y * kGridF));
      emit(keep, x, y, gl);
    };
    auto push = [&](bool qq, float x, float y, uint32_t gl) {
      const uint64_t m = __ballot(qq);
      if (!m) return;
      if (qq) {
        const uint32_t p = qn + popc64(m & lt);
        s_qx[w][p] = x; s_qy[w][p] = y; s_qg[w][p] = gl;
      }
      qn += popc64(m);
      wave_sync();
      if (qn >= 64) {
        qn -= 64;
        drain(qn, 64);
      }
    };
    // kU rows of the wave per step (rows r + u kWaves), loaded together;
    // the next step's rows are requested before this step is tested.
    auto load = [&](float4 (&dst)[kU], uint32_t r) {
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const uint32_t q = (r + u * kWaves) * 64 + lane;
        dst[u] = q < npairs ? ld_stream(&p4[q]) : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
    float4 v[kU], nx[kU];
    if ((uint32_t)w < nrows) load(v, w);
    for (uint32_t r = w; r < nrows; r += kU * kWaves) {
      const uint32_t rn = r + kU * kWaves;
      if (rn < nrows) load(nx, rn);
      if (use_sp) {
        uint32_t tm = 0;  // bit 2u: first point of row u is queued, 2u+1: the second
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const bool val = (r + u * kWaves) * 64 + lane < npairs;
          frac = __builtin_fmaxf(frac, __builtin_fmaxf(__builtin_amdgcn_fractf(v[u].x * kGridF),
                                                       __builtin_amdgcn_fractf(v[u].y * kGridF)));
          frac = __builtin_fmaxf(frac, __builtin_fmaxf(__builtin_amdgcn_fractf(v[u].z * kGridF),
                                                       __builtin_amdgcn_fractf(v[u].w * kGridF)));
          const bool t0 = val & !in_inner(v[u].x, v[u].y, pcx, pcy, pr2, pos, pot);
          const bool t1 = val & !in_inner(v[u].z, v[u].w, pcx, pcy, pr2, pos, pot);
          tm |= (t0 ? 1u : 0u) << (2 * u);
          tm |= (t1 ? 2u : 0u) << (2 * u);
        }
        if (__ballot(tm != 0)) {
#pragma unroll
          for (int u = 0; u < kU; ++u) {
            const uint32_t g = a2 + 2 * ((r + u * kWaves) * 64 + lane);
            push((tm >> (2 * u)) & 1u, v[u].x, v[u].y, g - base);
            push((tm >> (2 * u)) & 2u, v[u].z, v[u].w, g + 1 - base);
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const bool val = (r + u * kWaves) * 64 + lane < npairs;
          if (val) {
            keys_add(k, v[u].x, v[u].y, bad);
            keys_add(k, v[u].z, v[u].w, bad);
          }
          const uint32_t g = a2 + 2 * ((r + u * kWaves) * 64 + lane);
          emit(val, v[u].x, v[u].y, g - base);
          emit(val, v[u].z, v[u].w, g + 1 - base);
        }
      }
#pragma unroll
      for (int u = 0; u < kU; ++u) v[u] = nx[u];
    }
    if (qn) drain(0, qn);
    if (cw) flush();
    bad |= frac != 0.f;
    if (threadIdx.x == 0) {
      const uint32_t last = a2 + 2 * npairs;
      uint32_t singles[2];
      int ns = 0;
      if ((a & 1u) && a < b) singles[ns++] = a;
      if (last < b) singles[ns++] = last;
      for (int i = 0; i < ns; ++i) {
        const uint32_t g = singles[i];
        const float x = xy[2 * (size_t)g], y = xy[2 * (size_t)g + 1];
        keys_add(k, x, y, bad);
        if (!use_sp ||
            !poly_strict_inside(s_pvx, s_pvy, pnv, (int32_t)(x * kGridF), (int32_t)(y * kGridF)))
          cand[base + atomicAdd(&ss.ncand, 1u)] = make_payload<Rec>(g - base, x, y);
      }
    }
    const uint64_t badmask = __ballot(bad);
    block_keys(k);
    if (threadIdx.x == 0) {
      const double mx[4] = {k.mxE, k.mxN, k.mxNE, k.mxSE};
      const double mn[4] = {k.mnE, k.mnN, k.mnNE, k.mnSE};
      for (int i = 0; i < 4; ++i) {
        atomicMax((unsigned long long*)&ss.key[i], (unsigned long long)enc_f64(mx[i]));
        atomicMax((unsigned long long*)&ss.key[4 + i], (unsigned long long)enc_f64(-mn[i]));
      }
    }
    if (lane == 0 && badmask) atomicOr(&ss.bad, 1u);
  }
}

// Candidates per set from which the batch candidates get a second polygon,
// and its bins.
constexpr uint32_t kRefineMin = 1024;
constexpr uint32_t kRefineBatchBins = 512;

// Whole workgroup, one set's m >= kRefineMin candidates (every point not
// strictly inside its sample polygon, or all its points) and a point c
// inside its hull: a second polygon from the candidates themselves. The plane around c is cut
// into kRefineBatchBins bins of pseudo-angle; in each bin the candidate of largest
// dot product with the bin's middle direction is kept (a 64-bit LDS max of
// (dot product, position)), and the kept points, in bin order, go through
// build_poly (repeats and reflex points dropped until none is left, then the
// same exact checks as any polygon), which overwrites the set's SamplePoly
// and wedge table. Every vertex is an input point, so a candidate strictly
// inside the result is not a hull vertex whichever points were picked; a
// failed check leaves nv = 0. When the candidates hold most of the set's
// points near the hull (points close to a circle), the kept points are the
// set's extreme points in the bins' directions, and the second polygon is
// as close to the hull as its number of sides allows.
__device__ void refine_poly(const Rec* __restrict__ cand, uint32_t m, int32_t cx, int32_t cy,
                            SamplePoly* __restrict__ out, uint32_t* __restrict__ lut) {
  constexpr uint32_t B = kRefineBatchBins, E = B / kBlock;
  static_assert(B % kBlock == 0 && B <= kPolyMax, "whole bins per thread, within the polygon");
  __shared__ uint64_t s_bin[B];
  __shared__ int32_t s_da[B], s_db[B];
  __shared__ int32_t s_px[B], s_py[B];
  for (uint32_t k = threadIdx.x; k < B; k += kBlock) {
    // Bin k: pseudo-angles [4k, 4k + 4) / B; its middle direction as an
    // integer vector with |a| + |b| = 1024 (dot products below 2^30).
    const float pa = ((float)k + 0.5f) * (4.0f / (float)B);
    const uint32_t q = (uint32_t)pa;
    const int32_t f = (int32_t)__builtin_rintf((pa - (float)q) * 1024.0f);
    const int32_t u = 1024 - f, v = f;
    s_da[k] = q == 0 ? u : (q == 1 ? -v : (q == 2 ? -u : v));
    s_db[k] = q == 0 ? v : (q == 1 ? u : (q == 2 ? -v : -u));
    s_bin[k] = 0ull;
  }
  __syncthreads();
  constexpr int kR = 8;  // records per thread and step, loaded together
  for (uint32_t i0 = threadIdx.x; i0 < m; i0 += kBlock * kR) {
    Rec r[kR];
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const uint32_t i = i0 + j * kBlock;
      r[j] = cand[i < m ? i : m - 1];
    }
#pragma unroll
    for (int j = 0; j < kR; ++j) {
      const uint32_t i = i0 + j * kBlock;
      const float dx = (float)(r[j].x - cx), dy = (float)(r[j].y - cy);
      if (i >= m || (dx == 0.f && dy == 0.f)) continue;
      const uint32_t k = min((uint32_t)(pangle32(dx, dy) * (float)(B / 4)), B - 1);
      const int32_t dot = __mul24(s_da[k], r[j].x) + __mul24(s_db[k], r[j].y) + (1 << 30);
      atomicMax(&s_bin[k], ((uint64_t)(uint32_t)dot << 32) | i);
    }
  }
  __syncthreads();
  // Thread t takes bins tE .. tE + E - 1 (bin order kept by the scan).
  uint64_t key[E];
  uint32_t nk = 0;
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    key[e] = s_bin[threadIdx.x * E + e];
    nk += key[e] ? 1u : 0u;
  }
  uint32_t mp;
  uint32_t pos = block_excl_scan(nk, mp);
#pragma unroll
  for (uint32_t e = 0; e < E; ++e) {
    if (key[e]) {
      const Rec r = cand[(uint32_t)key[e]];
      s_px[pos] = r.x;
      s_py[pos] = r.y;
      ++pos;
    }
  }
  __syncthreads();
  build_poly<kBatchLutBins, 16>(s_px, s_py, mp, out, lut);
}

// Tiles of the candidates' octagon test.
constexpr uint32_t kCandTile = 8192;

// After the per-set octagons: the second polygon of every set with at least
// kRefineMin candidates (refine_poly), one workgroup per set, the sets taken
// through a shared counter. Its centre for the bins: the sample polygon's
// centre, else the mean of the octagon's vertices (any point does for
// exactness; one inside the hull gives good bins).
__global__ __launch_bounds__(kBlock) void k_batch_refine(const uint64_t* __restrict__ off,
                                                         uint32_t nsets, BatchHdr* __restrict__ bh,
                                                         const SetState* __restrict__ sets,
                                                         const Rec* __restrict__ cand,
                                                         SamplePoly* __restrict__ polys,
                                                         uint32_t* __restrict__ luts) {
  __shared__ uint32_t s_item;
  if (bh->bad_offsets) return;
  for (;;) {
    __syncthreads();  // the previous set is done with s_item and refine_poly's arrays
    if (threadIdx.x == 0) s_item = atomicAdd(&bh->refine_next, 1u);
    __syncthreads();
    const uint32_t s = s_item;
    if (s >= nsets) break;
    const SetState& ss = sets[s];
    const Octagon* __restrict__ o = &ss.oct;
    if (off[s + 1] <= off[s] || o->status != 0 || ss.ncand < kRefineMin) continue;
    int32_t cx = polys[s].cx, cy = polys[s].cy;
    if (polys[s].nv < 3) {
      int64_t sx = 0, sy = 0;
      for (int v = 0; v < 8; ++v) { sx += o->vx[v]; sy += o->vy[v]; }
      cx = (int32_t)(sx / 8);
      cy = (int32_t)(sy / 8);
    }
    refine_poly(cand + (uint32_t)off[s], ss.ncand, cx, cy, &polys[s], luts + size_t(s) * kBatchLutBins);
  }
}

// Tiles of kCandTile candidates of every set with a usable octagon, in set
// order (the layout of k_batch_round_plan; the pass tiles' buffer is free
// by now).
__global__ __launch_bounds__(kBlock) void k_batch_cand_plan(const uint64_t* __restrict__ off,
                                                            uint32_t nsets, BatchHdr* __restrict__ bh,
                                                            const SetState* __restrict__ sets,
                                                            SetTile* __restrict__ ctiles) {
  __shared__ uint32_t s_red[kWaves][2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const uint32_t first = blockIdx.x * kBlock;
  const bool bad = bh->bad_offsets != 0;
  auto count = [&](uint32_t s) {
    return bad || off[s + 1] <= off[s] || sets[s].oct.status != 0 ? 0u : sets[s].ncand;
  };
  auto tiles_of = [](uint32_t c) { return c / kCandTile + (c % kCandTile ? 1u : 0u); };
  uint32_t before = 0, all = 0;
  for (uint32_t s = threadIdx.x; s < nsets; s += kBlock) {
    const uint32_t t = tiles_of(count(s));
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
  const uint32_t c = s < nsets ? count(s) : 0u;
  uint32_t unused;
  uint32_t t = before + block_excl_scan(tiles_of(c), unused);
  for (uint32_t p = 0; p < c; p += kCandTile) {
    SetTile st;
    st.set = s; st.begin = p; st.end = p + kCandTile < c ? p + kCandTile : c; st.pad = 0;
    ctiles[t++] = st;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) bh->ncand_tiles = all;
}

// The octagon test of the candidates, a tile of them per workgroup at a
// time; survivors appended as records to the set's slice of `surv`, their
// count in cnt[0]. In a set with a second polygon (at least kRefineMin
// candidates) a candidate strictly inside it is dropped too. Five waves per
// SIMD (at most 96 VGPRs) rather than four: more tiles' record loads in flight.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_batch_cand(const uint64_t* __restrict__ off,
                                                       const BatchHdr* __restrict__ bh,
                                                       SetState* __restrict__ sets,
                                                       const SetTile* __restrict__ ctiles,
                                                       const Rec* __restrict__ cand,
                                                       Rec* __restrict__ surv,
                                                       const SamplePoly* __restrict__ polys,
                                                       const uint32_t* __restrict__ luts) {
  __shared__ int32_t s_pvx[kPolyMax], s_pvy[kPolyMax];
  __shared__ uint32_t s_lut[kBatchLutBins];
  const int lane = threadIdx.x & 63;
  const uint64_t lt = (1ull << lane) - 1ull;
  const uint32_t nt = bh->ncand_tiles;
  for (uint32_t t = blockIdx.x; t < nt; t += gridDim.x) {
    const SetTile st = ctiles[t];
    const uint32_t s = st.set;
    SetState& ss = sets[s];
    const Octagon* __restrict__ o = &ss.oct;
    const uint32_t base = (uint32_t)off[s];
    // Second polygon (block-uniform decision).
    const uint32_t nv2 = ss.ncand >= kRefineMin ? min(polys[s].nv, (uint32_t)kPolyMax) : 0u;
    const int32_t cx2 = polys[s].cx, cy2 = polys[s].cy;
    __syncthreads();  // the previous tile is done with s_pvx / s_pvy / s_lut
    if (nv2 >= 3) {
      for (uint32_t i = threadIdx.x; i < nv2; i += kBlock) { s_pvx[i] = polys[s].vx[i]; s_pvy[i] = polys[s].vy[i]; }
      const uint32_t* __restrict__ lut = luts + size_t(s) * kBatchLutBins;
      for (uint32_t i = threadIdx.x; i < kBatchLutBins; i += kBlock) s_lut[i] = lut[i];
    }
    __syncthreads();
    const uint32_t m = st.end;
    // kR records per lane and step, loaded together; one reservation per
    // wave and step.
    constexpr int kR = 8;
    for (uint32_t i0 = st.begin + (threadIdx.x - lane) * kR; i0 < m; i0 += kBlock * kR) {
      Rec r[kR];
      uint64_t bk[kR];
      uint32_t tot = 0;
#pragma unroll
      for (int j = 0; j < kR; ++j) {
        const uint32_t i = i0 + j * 64 + lane;
        r[j] = i < m ? cand[base + i] : Rec{};
      }
#pragma unroll
      for (int j = 0; j < kR; ++j) {
        const uint32_t i = i0 + j * 64 + lane;
        const bool keep = i < m &&
                          classify<false>((float)r[j].x * (1.0f / kGridF), (float)r[j].y * (1.0f / kGridF),
                                          r[j].i, o, ss.vidx).keep &&
                          !(nv2 >= 3 && poly_lut_inside<kBatchLutBins>(s_pvx, s_pvy, nv2, s_lut, cx2, cy2,
                                                                       r[j].x, r[j].y));
        bk[j] = __ballot(keep);
        tot += popc64(bk[j]);
      }
      if (!tot) continue;
      uint32_t p = 0;
      if (lane == 0) p = atomicAdd(&ss.cnt[0], tot);
      p = __shfl(p, 0);
#pragma unroll
      for (int j = 0; j < kR; ++j) {
        if ((bk[j] >> lane) & 1ull) surv[base + p + popc64(bk[j] & lt)] = r[j];
        p += popc64(bk[j]);
      }
    }
  }
}

// ------------------------------------------------------------- launchers

hipError_t launch_set_u32(uint32_t* p, uint32_t v, hipStream_t st) {
  hipLaunchKernelGGL(k_set_u32, dim3(1), dim3(64), 0, st, p, v);
  return hipGetLastError();
}

// Persistent grid of pass 1: at most `max_blocks`, and no more than needed
// for one batch per wave.
uint32_t reduce_blocks(uint32_t n, uint32_t max_blocks) {
  const uint64_t pairs = (uint64_t(n) + 1) / 2;
  const uint64_t per_block = uint64_t(kWaves) * kU * 64;
  uint64_t b = (pairs + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  return (uint32_t)b;
}

// Persistent grid of pass 2: at most `max_blocks` (and at most 1024, the
// look-back reach), each wave getting at least one row.
uint32_t filter_blocks(uint32_t n, uint32_t max_blocks) {
  const uint64_t rows = ((uint64_t(n) + 1) / 2 + 63) / 64;
  uint64_t b = (rows + kWaves - 1) / kWaves;
  if (b < 1) b = 1;
  if (b > max_blocks) b = max_blocks;
  if (b > 1024) b = 1024;
  return (uint32_t)b;
}

hipError_t launch_reduce8(const float* xy, uint32_t n, uint32_t head, double* partials,
                          uint32_t* part_bad, uint32_t blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce8, dim3(blocks), dim3(kBlock), 0, st, xy, n, head, partials, part_bad);
  return hipGetLastError();
}

hipError_t launch_axis_extremes(const float* xy, uint32_t n, uint32_t head, double* partials,
                                uint32_t* part_bad, uint32_t blocks, Header* hdr, hipStream_t st) {
  hipLaunchKernelGGL(k_axis4, dim3(blocks), dim3(kBlock), 0, st, xy, n, head, partials, part_bad);
  hipLaunchKernelGGL(k_axis_box, dim3(1), dim3(kBlock), 0, st, partials, part_bad, blocks, hdr);
  return hipGetLastError();
}
hipError_t launch_corner_extremes(const float* xy, uint32_t n, uint32_t head, double* partials,
                                  uint32_t blocks, const Header* hdr, hipStream_t st) {
  hipLaunchKernelGGL(k_corner4, dim3(blocks), dim3(kBlock), 0, st, xy, n, head, hdr, partials);
  return hipGetLastError();
}
hipError_t launch_oct_build(const double* partials, const uint32_t* part_bad, uint32_t nparts,
                            Header* hdr, Result* res, uint64_t* tstat, uint32_t ntstat,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_oct_build, dim3(1), dim3(kBlock), 0, st, partials, part_bad, nparts, hdr, res,
                     tstat, ntstat);
  return hipGetLastError();
}

hipError_t launch_pass_hull(const float* xy, uint32_t n, uint32_t head, double* partials,
                            uint32_t* part_bad, const SamplePoly* poly, Rec* cand, void* scratch,
                            uint32_t blocks, uint32_t narrow_blocks, hipStream_t st) {
  hipLaunchKernelGGL(k_pass_hull, dim3(blocks), dim3(kBlock), 0, st, xy, n, head, partials, part_bad,
                     poly, static_cast<SampleDirs*>(scratch), cand, narrow_blocks);
  return hipGetLastError();
}



hipError_t launch_filter(const float* xy, uint32_t n, uint32_t head, Header* hdr, uint64_t* tstat,
                         uint32_t blocks, uint32_t* surv, uint32_t* count_out, uint8_t* labels,
                         uint32_t* staging, hipStream_t st) {
  if (labels)
    hipLaunchKernelGGL((k_filter<true, uint32_t>), dim3(blocks), dim3(kBlock), 0, st, xy, n, head,
                       hdr, tstat, blocks, surv, count_out, labels, staging);
  else
    hipLaunchKernelGGL((k_filter<false, uint32_t>), dim3(blocks), dim3(kBlock), 0, st, xy, n, head,
                       hdr, tstat, blocks, surv, count_out, labels, staging);
  return hipGetLastError();
}

// gate/cand/scratch non-null: after a fused pass (see k_filter_hull).
hipError_t launch_filter_rec(const float* xy, uint32_t n, uint32_t head, Header* hdr,
                             uint32_t blocks, Rec* surv, uint32_t* count_out,
                             const SamplePoly* gate, const Rec* cand, const void* scratch,
                             uint32_t* ncand_out, uint32_t* mode_out, const double* partials,
                             const uint32_t* part_bad, uint32_t nparts, Result* res,
                             hipStream_t st) {
  const SampleDirs* sd = static_cast<const SampleDirs*>(scratch);
  hipLaunchKernelGGL(k_filter_hull, dim3(blocks), dim3(kBlock), 0, st, xy, n, head, hdr, surv,
                     count_out, gate, cand, sd ? &sd->cand : nullptr, ncand_out,
                     sd ? &sd->mode : nullptr, mode_out, partials, part_bad, nparts, res);
  return hipGetLastError();
}

hipError_t launch_oct_out(const Header* hdr, void* d_oct, hipStream_t st) {
  hipLaunchKernelGGL(k_oct_out, dim3(1), dim3(64), 0, st, hdr, static_cast<int32_t*>(d_oct));
  return hipGetLastError();
}

}  // namespace chk

namespace chk {

hipError_t launch_batch_sample(const float* xy, const uint64_t* off, BatchHdr* bh,
                               const uint32_t* slist, SamplePoly* polys, uint32_t sample_min,
                               uint32_t grid, hipStream_t st);

hipError_t launch_batch_filter_side(const float* xy, const uint64_t* off, uint32_t nsets,
                                    uint64_t total_points, uint32_t tile, BatchHdr* bh,
                                    SetState* sets, SamplePoly* polys, SetTile* tiles, Rec* recs,
                                    Rec* cand, uint32_t grid, uint32_t sample_min,
                                    uint32_t sample_grid, uint32_t* slist, uint32_t* luts,
                                    hipStream_t st, LaunchHook* hk) {
  // Grids above the most workgroups with work (sets, or tiles: at most one
  // partial tile per set) only add dispatch time, which small batches feel.
  auto cap = [](uint64_t g, uint64_t most) { return (uint32_t)(most < 1 ? 1 : (g < most ? g : most)); };
  const uint32_t g_sets = cap(sample_grid, nsets);
  const uint32_t g_pass = cap(grid, total_points / tile + nsets);
  const uint32_t g_cand = cap(4ull * sample_grid, total_points / kCandTile + nsets);
  hooked(hk, "batch_plan", [&] {
    hipLaunchKernelGGL(k_batch_plan, dim3(nsets / kBlock + 1), dim3(kBlock), 0, st, off, nsets,
                       total_points, tile, sample_min, bh, sets, tiles, polys, slist);
  });
  hipError_t e = hipSuccess;
  hooked(hk, "batch_sample",
         [&] { e = launch_batch_sample(xy, off, bh, slist, polys, sample_min, g_sets, st); });
  if (e != hipSuccess) return e;
  hooked(hk, "batch_pass", [&] {
    hipLaunchKernelGGL(k_batch_pass, dim3(g_pass), dim3(kBlock), 0, st, xy, off, bh, tiles, sets, polys,
                       cand);
  });
  hooked(hk, "batch_octagon", [&] {
    hipLaunchKernelGGL(k_batch_octagon, dim3((nsets + kWaves - 1) / kWaves), dim3(kBlock), 0, st, off,
                       nsets, bh, sets);
  });
  hooked(hk, "batch_refine", [&] {
    hipLaunchKernelGGL(k_batch_refine, dim3(g_sets), dim3(kBlock), 0, st, off, nsets, bh, sets,
                       cand, polys, luts);
  });
  hooked(hk, "batch_cand_plan", [&] {
    hipLaunchKernelGGL(k_batch_cand_plan, dim3(nsets / kBlock + 1), dim3(kBlock), 0, st, off, nsets,
                       bh, sets, tiles);
  });
  hooked(hk, "batch_cand", [&] {
    // its own grid (16 workgroups per CU): the candidate tiles are short
    // latency chains, which more workgroups than the pass's overlap better
    hipLaunchKernelGGL(k_batch_cand, dim3(g_cand), dim3(kBlock), 0, st, off, bh, sets, tiles,
                       cand, recs, polys, luts);
  });
  return hipGetLastError();
}

}  // namespace chk
