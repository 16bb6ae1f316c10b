/*
 * CPU oracle for the heaphull-style convex hull: octagon filter followed by
 * Andrew's monotone chain.
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU library shares
 * no code, header, table or helper with it.
 *
 * Paper: A. Keith, H. Ferrada, C. A. Navarro, "Accelerating the Convex Hull
 * Computation with a Parallel GPU Algorithm" (arXiv 2209.12310).
 *   - Alg. 1 (heaphull): extremes -> octagon -> outside test -> per-queue hull.
 *   - Sec. III: the four axis extremes N, S, E, W come first; the four corner
 *     points are then the input points of least Manhattan distance to the
 *     corners of the box those four span.
 *   - Alg. 2 (GPUfilter): a label per point, 0 for a discarded point.
 *   - Sec. I, stage 1 of the two-stage scheme: a point lying on a side of the
 *     filter polygon without being one of its vertices is discarded.
 *   - Table I: Andrew's monotone chain (1979) is the hull algorithm used here.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *   - Input: float32 coordinates x, y with x*2^20 and y*2^20 integers in
 *     [0, 2^20). kx = x*2^20, ky = y*2^20. All predicates are exact integer
 *     arithmetic on (kx, ky).
 *   - Tie-breaks for an extreme: among equal primary values, the point that
 *     lies further counter-clockwise along the support line; among equal
 *     coordinates, the smallest index.
 *   - The hull: strict vertices only (collinear boundary points excluded),
 *     counter-clockwise, starting at the lexicographic minimum (min kx, then
 *     min ky). A vertex reported for duplicated coordinates carries the
 *     smallest index holding them. Indices are 0-based.
 *   - Queue label of a surviving point: 1 + floor(i/2) for the first octagon
 *     edge i it lies strictly outside of; for a vertex lying outside no edge,
 *     1 + floor(k/2) for the first octagon slot k it occupies.
 *     This rule is our own: parity unpinned by the paper.
 *
 * Floating point never decides anything here: every product is of integers
 * below 2^21 and is formed in int64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* Planted-mistake switch used only by the test that shows the pins bite.
 * 0 = the oracle as written. Any other value injects one known mistake.
 * The timed CPU-baseline build (OR_NO_MUTATION) compiles the switch out. */
#ifdef OR_NO_MUTATION
#define g_mutation 0
void or_set_mutation(int m) { (void)m; }
int or_get_mutation(void) { return 0; }
#else
static int g_mutation = 0;
void or_set_mutation(int m) { g_mutation = m; }
int or_get_mutation(void) { return g_mutation; }
#endif

int or_version(void) { return 1; }

int or_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* ---------------------------------------------------------------- domain */

/* Convert the n interleaved float32 pairs to grid integers.
 * Returns -1 when every coordinate is a value k*2^-20 with integer k in
 * [0, 2^20); otherwise the index of the first offending point. */
int64_t or_to_grid(const float* xy, int64_t n, int32_t* kx, int32_t* ky) {
  for (int64_t j = 0; j < n; ++j) {
    for (int c = 0; c < 2; ++c) {
      double v = (double)xy[2 * j + c];
      if (!(v >= 0.0 && v < 1.0)) return j; /* NaN fails both tests */
      double s = v * 1048576.0;             /* exact: power-of-two scale */
      double f = floor(s);
      if (f != s) return j;
      if (c == 0) kx[j] = (int32_t)f; else ky[j] = (int32_t)f;
    }
  }
  return -1;
}

/* -------------------------------------------------------------- extremes */

/* orient(a, b, p): twice the signed area of (a, b, p); > 0 when p lies to the
 * left of the directed line a -> b. Exact: |terms| < 2^41. */
static int64_t orient(int64_t ax, int64_t ay, int64_t bx, int64_t by,
                      int64_t px, int64_t py) {
  if (g_mutation == 2) /* planted: transposed operand */
    return (bx - ax) * (py - ay) - (by - ay) * (px - ay);
  return (bx - ax) * (py - ay) - (by - ay) * (px - ax);
}

/* Octagon slot order (counter-clockwise): E, NE, N, NW, W, SW, S, SE. */
enum { S_E = 0, S_NE, S_N, S_NW, S_W, S_SW, S_S, S_SE };

/* findExtremes as the paper describes it for the GPU (Sec. III):
 *   first reduction: the axis extremes E (max x), N (max y), W (min x),
 *   S (min y); second reduction: for each corner of the box
 *   [W.x, E.x] x [S.y, N.y], the point of least Manhattan distance to it.
 * out[8] receives point indices in slot order. n must be >= 1. */
void or_extremes(const int32_t* kx, const int32_t* ky, int64_t n, int64_t out[8]) {
  int64_t e = 0, nn = 0, w = 0, s = 0;
  for (int64_t j = 1; j < n; ++j) {
    /* E: larger x; on a tie the point further counter-clockwise (larger y). */
    if (kx[j] > kx[e] || (kx[j] == kx[e] && ky[j] > ky[e])) e = j;
    /* N: larger y; on a tie, smaller x. */
    if (ky[j] > ky[nn] || (ky[j] == ky[nn] && kx[j] < kx[nn])) nn = j;
    /* W: smaller x; on a tie, smaller y. */
    if (kx[j] < kx[w] || (kx[j] == kx[w] && ky[j] < ky[w])) w = j;
    /* S: smaller y; on a tie, larger x. */
    if (ky[j] < ky[s] || (ky[j] == ky[s] && kx[j] > kx[s])) s = j;
  }
  if (g_mutation == 4) { /* planted: E tie-break reversed (smaller y wins) */
    e = 0;
    for (int64_t j = 1; j < n; ++j)
      if (kx[j] > kx[e] || (kx[j] == kx[e] && ky[j] < ky[e])) e = j;
  }
  /* Box corners spanned by the first four points. */
  const int64_t xmax = kx[e], ymax = ky[nn], xmin = kx[w], ymin = ky[s];
  const int64_t cx[4] = {xmax, xmin, xmin, xmax}; /* NE, NW, SW, SE */
  const int64_t cy[4] = {ymax, ymax, ymin, ymin};
  int64_t best[4] = {0, 0, 0, 0};
  int64_t bd[4];
  for (int c = 0; c < 4; ++c) bd[c] = llabs(kx[0] - cx[c]) + llabs(ky[0] - cy[c]);
  for (int64_t j = 1; j < n; ++j) {
    for (int c = 0; c < 4; ++c) {
      int64_t d = llabs(kx[j] - cx[c]) + llabs(ky[j] - cy[c]);
      if (g_mutation == 5 && c == 0) d = llabs(kx[j] - cx[c]); /* planted: dropped term */
      int64_t b = best[c];
      int better = d < bd[c];
      if (d == bd[c]) {
        /* Equal distance: the points lie on one line of slope -1 (NE, SW) or
         * +1 (NW, SE); take the end further counter-clockwise. */
        switch (c) {
          case 0: better = ky[j] > ky[b]; break; /* NE: towards N, larger y */
          case 1: better = ky[j] < ky[b]; break; /* NW: towards W, smaller y */
          case 2: better = kx[j] > kx[b]; break; /* SW: towards S, larger x */
          default: better = ky[j] > ky[b]; break; /* SE: towards E, larger y */
        }
      }
      if (better) { best[c] = j; bd[c] = d; }
    }
  }
  out[S_E] = e;  out[S_NE] = best[0]; out[S_N] = nn; out[S_NW] = best[1];
  out[S_W] = w;  out[S_SW] = best[2]; out[S_S] = s;  out[S_SE] = best[3];
}

/* ---------------------------------------------------------------- filter */

/* Classify one point against the octagon with vertices (vx[k], vy[k]).
 * Returns 0 when the point is discarded (inside the closed octagon and not a
 * vertex), else its queue label in 1..4. */
static int classify(int64_t px, int64_t py, const int64_t vx[8], const int64_t vy[8]) {
  for (int i = 0; i < 8; ++i) {
    int i2 = (i + 1) & 7;
    int64_t o = orient(vx[i], vy[i], vx[i2], vy[i2], px, py);
    if (g_mutation == 1 ? (o <= 0 && !(vx[i] == vx[i2] && vy[i] == vy[i2]))
                        : (o < 0))
      return 1 + i / 2;
  }
  if (g_mutation == 3) return 0; /* planted: vertices not kept */
  for (int k = 0; k < 8; ++k)
    if (px == vx[k] && py == vy[k]) return 1 + k / 2;
  return 0;
}

static void load_octagon(const int32_t* kx, const int32_t* ky, const int64_t oct[8],
                         int64_t vx[8], int64_t vy[8]) {
  for (int k = 0; k < 8; ++k) { vx[k] = kx[oct[k]]; vy[k] = ky[oct[k]]; }
}

/* Outside test and queue labels of Alg. 1 / Alg. 2 over all n points.
 * survivors (may be NULL) receives the kept indices in ascending order;
 * labels (may be NULL) receives one byte per point. Returns the count. */
int64_t or_filter(const int32_t* kx, const int32_t* ky, int64_t n, const int64_t oct[8],
                  uint32_t* survivors, uint8_t* labels) {
  int64_t vx[8], vy[8];
  load_octagon(kx, ky, oct, vx, vy);
  int64_t m = 0;
  for (int64_t j = 0; j < n; ++j) {
    int q = classify(kx[j], ky[j], vx, vy);
    if (labels) labels[j] = (uint8_t)q;
    if (q) { if (survivors) survivors[m] = (uint32_t)j; ++m; }
  }
  return m;
}

/* The CPU-parallel variant the paper compares against (Sec. III, last
 * paragraph): the input is split into one contiguous chunk per thread; each
 * thread finds its chunk's extremes and filters its chunk; the partial
 * results are combined in chunk order. Same outputs as the sequential path. */
int64_t or_filter_parallel(const int32_t* kx, const int32_t* ky, int64_t n,
                           int64_t oct_out[8], uint32_t* survivors, int nthreads) {
#ifndef _OPENMP
  (void)nthreads;
  or_extremes(kx, ky, n, oct_out);
  return or_filter(kx, ky, n, oct_out, survivors, NULL);
#else
  if (nthreads <= 0) nthreads = omp_get_max_threads();
  if (n < 2 * (int64_t)nthreads) nthreads = 1;
  int64_t* part = (int64_t*)malloc(sizeof(int64_t) * 8 * (size_t)nthreads);
  int64_t* cnt = (int64_t*)calloc((size_t)nthreads + 1, sizeof(int64_t));
  /* Stage 1: chunk extremes; combined with the same comparisons as above,
   * scanning the chunk winners in chunk (= index) order. */
#pragma omp parallel num_threads(nthreads)
  {
    int t = omp_get_thread_num();
    int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
    int64_t e = lo, nn = lo, w = lo, s = lo;
    for (int64_t j = lo + 1; j < hi; ++j) {
      if (kx[j] > kx[e] || (kx[j] == kx[e] && ky[j] > ky[e])) e = j;
      if (ky[j] > ky[nn] || (ky[j] == ky[nn] && kx[j] < kx[nn])) nn = j;
      if (kx[j] < kx[w] || (kx[j] == kx[w] && ky[j] < ky[w])) w = j;
      if (ky[j] < ky[s] || (ky[j] == ky[s] && kx[j] > kx[s])) s = j;
    }
    part[8 * t + 0] = e; part[8 * t + 1] = nn; part[8 * t + 2] = w; part[8 * t + 3] = s;
  }
  int64_t e = part[0], nn = part[1], w = part[2], s = part[3];
  for (int t = 1; t < nthreads; ++t) {
    int64_t j;
    j = part[8 * t + 0]; if (kx[j] > kx[e] || (kx[j] == kx[e] && ky[j] > ky[e])) e = j;
    j = part[8 * t + 1]; if (ky[j] > ky[nn] || (ky[j] == ky[nn] && kx[j] < kx[nn])) nn = j;
    j = part[8 * t + 2]; if (kx[j] < kx[w] || (kx[j] == kx[w] && ky[j] < ky[w])) w = j;
    j = part[8 * t + 3]; if (ky[j] < ky[s] || (ky[j] == ky[s] && kx[j] > kx[s])) s = j;
  }
  const int64_t cx[4] = {kx[e], kx[w], kx[w], kx[e]};
  const int64_t cy[4] = {ky[nn], ky[nn], ky[s], ky[s]};
#pragma omp parallel num_threads(nthreads)
  {
    int t = omp_get_thread_num();
    int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads;
    for (int c = 0; c < 4; ++c) {
      int64_t b = lo, bd = llabs(kx[lo] - cx[c]) + llabs(ky[lo] - cy[c]);
      for (int64_t j = lo + 1; j < hi; ++j) {
        int64_t d = llabs(kx[j] - cx[c]) + llabs(ky[j] - cy[c]);
        int better = d < bd;
        if (d == bd) better = (c == 0) ? ky[j] > ky[b] : (c == 1) ? ky[j] < ky[b]
                              : (c == 2) ? kx[j] > kx[b] : ky[j] > ky[b];
        if (better) { b = j; bd = d; }
      }
      part[8 * t + 4 + c] = b;
    }
  }
  int64_t best[4];
  for (int c = 0; c < 4; ++c) {
    int64_t b = part[4 + c];
    int64_t bd = llabs(kx[b] - cx[c]) + llabs(ky[b] - cy[c]);
    for (int t = 1; t < nthreads; ++t) {
      int64_t j = part[8 * t + 4 + c];
      int64_t d = llabs(kx[j] - cx[c]) + llabs(ky[j] - cy[c]);
      int better = d < bd;
      if (d == bd) better = (c == 0) ? ky[j] > ky[b] : (c == 1) ? ky[j] < ky[b]
                            : (c == 2) ? kx[j] > kx[b] : ky[j] > ky[b];
      if (better) { b = j; bd = d; }
    }
    best[c] = b;
  }
  oct_out[S_E] = e;  oct_out[S_NE] = best[0]; oct_out[S_N] = nn; oct_out[S_NW] = best[1];
  oct_out[S_W] = w;  oct_out[S_SW] = best[2]; oct_out[S_S] = s;  oct_out[S_SE] = best[3];
  /* Stage 2: each thread filters its chunk into its own ordered list (count
   * first, then an exclusive scan of the counts gives each list its place). */
  int64_t vx[8], vy[8];
  load_octagon(kx, ky, oct_out, vx, vy);
#pragma omp parallel num_threads(nthreads)
  {
    int t = omp_get_thread_num();
    int64_t lo = n * t / nthreads, hi = n * (t + 1) / nthreads, c = 0;
    for (int64_t j = lo; j < hi; ++j) c += classify(kx[j], ky[j], vx, vy) != 0;
    cnt[t + 1] = c;
#pragma omp barrier
#pragma omp single
    for (int u = 0; u < nthreads; ++u) cnt[u + 1] += cnt[u];
    if (survivors) {
      int64_t o = cnt[t];
      for (int64_t j = lo; j < hi; ++j)
        if (classify(kx[j], ky[j], vx, vy)) survivors[o++] = (uint32_t)j;
    }
  }
  int64_t m = cnt[nthreads];
  free(part);
  free(cnt);
  return m;
#endif
}

/* ------------------------------------------------------------------ hull */

typedef struct { int32_t x, y; uint32_t i; } rec_t;

static int rec_cmp(const void* a, const void* b) {
  const rec_t* p = (const rec_t*)a;
  const rec_t* q = (const rec_t*)b;
  if (p->x != q->x) return p->x < q->x ? -1 : 1;
  if (p->y != q->y) return p->y < q->y ? -1 : 1;
  if (p->i != q->i) return p->i < q->i ? -1 : 1;
  return 0;
}

/* Andrew's scan over records already sorted by (kx, ky, index): keep the
 * first of each run of equal coordinates (the smallest index); lower chain
 * left to right and upper chain right to left, each popping while the last
 * turn is not strictly counter-clockwise. r is compacted in place; hull
 * receives the counter-clockwise hull from the lexicographic minimum.
 * Returns h (m >= 1). */
static int64_t chain_sorted(rec_t* r, int64_t m, uint32_t* hull) {
  int64_t u = 0;
  for (int64_t t = 0; t < m; ++t) {
    if (u > 0 && r[u - 1].x == r[t].x && r[u - 1].y == r[t].y) {
      if (g_mutation == 6) r[u - 1].i = r[t].i; /* planted: keeps the largest index */
      continue;
    }
    r[u++] = r[t];
  }
  if (u == 1) { hull[0] = r[0].i; return 1; }
  rec_t** st = (rec_t**)malloc(sizeof(rec_t*) * (size_t)(2 * u + 1));
  int64_t k = 0;
  for (int64_t t = 0; t < u; ++t) { /* lower chain */
    while (k >= 2) {
      int64_t c = orient(st[k - 2]->x, st[k - 2]->y, st[k - 1]->x, st[k - 1]->y, r[t].x, r[t].y);
      if (g_mutation == 7 ? c < 0 : c <= 0) --k; else break; /* 7: collinear kept */
    }
    st[k++] = &r[t];
  }
  int64_t lower = k + 1;
  for (int64_t t = u - 2; t >= 0; --t) { /* upper chain */
    while (k >= lower) {
      int64_t c = orient(st[k - 2]->x, st[k - 2]->y, st[k - 1]->x, st[k - 1]->y, r[t].x, r[t].y);
      if (g_mutation == 7 ? c < 0 : c <= 0) --k; else break;
    }
    st[k++] = &r[t];
  }
  int64_t h = k - 1; /* the last point repeats the first */
  for (int64_t t = 0; t < h; ++t) hull[t] = st[t]->i;
  if (g_mutation == 8 && h > 2) { /* planted: clockwise order */
    for (int64_t a = 1, b = h - 1; a < b; ++a, --b) { uint32_t x = hull[a]; hull[a] = hull[b]; hull[b] = x; }
  }
  free(st);
  return h;
}

static rec_t* gather_recs(const int32_t* kx, const int32_t* ky, const uint32_t* cand, int64_t m) {
  rec_t* r = (rec_t*)malloc(sizeof(rec_t) * (size_t)m);
  for (int64_t t = 0; t < m; ++t) {
    uint32_t j = cand ? cand[t] : (uint32_t)t;
    r[t].x = kx[j]; r[t].y = ky[j]; r[t].i = j;
  }
  return r;
}

/* Andrew's monotone chain over a candidate subset of the points.
 * cand == NULL means all n points; otherwise cand[0..m) lists point indices.
 * hull receives at most (m) indices, counter-clockwise from the
 * lexicographic minimum; returns h. Steps: sort by (kx, ky, index), then the
 * scan of chain_sorted. */
int64_t or_chain(const int32_t* kx, const int32_t* ky, int64_t n,
                 const uint32_t* cand, int64_t m, uint32_t* hull) {
  if (!cand) m = n;
  if (m <= 0) return 0;
  rec_t* r = gather_recs(kx, ky, cand, m);
  qsort(r, (size_t)m, sizeof(rec_t), rec_cmp);
  int64_t h = chain_sorted(r, m, hull);
  free(r);
  return h;
}

/* Multi-core sort for the CPU baseline: each thread sorts one contiguous
 * chunk with qsort, then neighbouring sorted runs are merged pairwise (the
 * merges of a round in parallel) until one run is left. Same order as one
 * qsort: the (kx, ky, index) keys are distinct. */
static void sort_recs_parallel(rec_t* r, int64_t m, int nthreads) {
#ifdef _OPENMP
  if (nthreads <= 1 || m < 4096) {
    qsort(r, (size_t)m, sizeof(rec_t), rec_cmp);
    return;
  }
  int64_t* b = (int64_t*)malloc(sizeof(int64_t) * ((size_t)nthreads + 1));
  for (int t = 0; t <= nthreads; ++t) b[t] = m * t / nthreads;
#pragma omp parallel for num_threads(nthreads) schedule(static, 1)
  for (int t = 0; t < nthreads; ++t)
    qsort(r + b[t], (size_t)(b[t + 1] - b[t]), sizeof(rec_t), rec_cmp);
  rec_t* tmp = (rec_t*)malloc(sizeof(rec_t) * (size_t)m);
  for (int w = 1; w < nthreads; w *= 2) {
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 1)
    for (int t = 0; t < nthreads; t += 2 * w) {
      if (t + w >= nthreads) continue;
      const int64_t lo = b[t], mid = b[t + w], hi = b[t + 2 * w < nthreads ? t + 2 * w : nthreads];
      int64_t i = lo, j = mid, o = lo;
      while (i < mid && j < hi) tmp[o++] = rec_cmp(&r[j], &r[i]) < 0 ? r[j++] : r[i++];
      while (i < mid) tmp[o++] = r[i++];
      while (j < hi) tmp[o++] = r[j++];
      memcpy(r + lo, tmp + lo, sizeof(rec_t) * (size_t)(hi - lo));
    }
  }
  free(tmp);
  free(b);
#else
  (void)nthreads;
  qsort(r, (size_t)m, sizeof(rec_t), rec_cmp);
#endif
}

/* or_chain on nthreads threads (the sort in parallel, then the scan). */
int64_t or_chain_parallel(const int32_t* kx, const int32_t* ky, int64_t n,
                          const uint32_t* cand, int64_t m, uint32_t* hull, int nthreads) {
  if (!cand) m = n;
  if (m <= 0) return 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#endif
  rec_t* r = gather_recs(kx, ky, cand, m);
  sort_recs_parallel(r, m, nthreads);
  int64_t h = chain_sorted(r, m, hull);
  free(r);
  return h;
}

/* ------------------------------------------------------- the four queues */

/* Alg. 1, stages (2)-(4): the surviving points go to four queues by their
 * label (Alg. 2's array Q: 0 for a discarded point, else the queue), each
 * queue gets its own hull, and the hull of the set is the union of the
 * pieces. Queue q (1..4) holds the quadrant between the axis extremes
 * A_q and A_{q+1} (A = E, N, W, S, then E again: octagon slots 0, 2, 4, 6);
 * its piece is the counter-clockwise arc from A_q to A_{q+1} of the hull of
 * the queue's points together with A_q and A_{q+1} (an axis extreme that
 * coincides with a corner vertex carries that corner's label, so it may sit
 * in the neighbouring queue).
 * Each axis extreme, with the tie-breaks of the extremes, is a strict
 * vertex of every subset containing it, so the arcs meet at them; the union
 * starts at the lexicographic minimum (W).
 * oct: the octagon's point indices in slot order; labels: n bytes; qcount
 * (may be NULL) receives the queue sizes. The queue hulls run one after the
 * other, each on nthreads threads. Returns h. */
int64_t or_heaphull_queues(const int32_t* kx, const int32_t* ky, int64_t n,
                           const int64_t oct[8], const uint8_t* labels, uint32_t* hull,
                           int64_t qcount[4], int nthreads) {
  if (n <= 0) return 0;
  /* Queue build: one pass over the labels, indices in ascending order. */
  int64_t cnt[5] = {0, 0, 0, 0, 0};
  for (int64_t j = 0; j < n; ++j) cnt[labels[j] <= 4 ? labels[j] : 0]++;
  uint32_t* q[5];
  for (int k = 1; k <= 4; ++k) q[k] = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(cnt[k] + 2));
  int64_t fill[5] = {0, 0, 0, 0, 0};
  for (int64_t j = 0; j < n; ++j) {
    const int k = labels[j];
    if (k >= 1 && k <= 4) q[k][fill[k]++] = (uint32_t)j;
  }
  if (qcount)
    for (int k = 0; k < 4; ++k) qcount[k] = cnt[k + 1];
  /* The axis extremes, each by its smallest index. */
  uint32_t ax[5];
  for (int k = 0; k < 4; ++k) {
    const int64_t v = oct[2 * k];
    int64_t best = v;
    for (int64_t j = 0; j < v; ++j)
      if (kx[j] == kx[v] && ky[j] == ky[v]) { best = j; break; }
    ax[k] = (uint32_t)best;
  }
  ax[4] = ax[0];
  /* Per-queue hulls and their arcs. */
  uint32_t* out = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n + 4));
  int64_t h = 0;
  for (int k = 1; k <= 4; ++k) {
    const uint32_t a = ax[k - 1], b = ax[k];
    const int64_t m = cnt[k];
    q[k][m] = a; /* the arc's end points join the queue */
    q[k][m + 1] = g_mutation == 9 ? a : b; /* 9 (planted): A_{q+1} left out */
    uint32_t* hk = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(m + 2));
    const int64_t hq = nthreads > 1 ? or_chain_parallel(kx, ky, n, q[k], m + 2, hk, nthreads)
                                    : or_chain(kx, ky, n, q[k], m + 2, hk);
    int64_t pa = -1, pb = -1;
    for (int64_t t = 0; t < hq; ++t) {
      if (kx[hk[t]] == kx[a] && ky[hk[t]] == ky[a]) pa = t;
      if (kx[hk[t]] == kx[b] && ky[hk[t]] == ky[b]) pb = t;
    }
    /* The arc from A_q up to (not including) A_{q+1}: the next arc starts
     * there. pa and pb always exist (extremes of the queue's hull). */
    if (pa >= 0 && pb >= 0)
      for (int64_t t = pa; t != pb; t = (t + 1) % hq) out[h++] = hk[t];
    free(hk);
  }
  if (h == 0) { /* every axis extreme is the same point */
    out[h++] = ax[0];
  }
  /* Start at the lexicographic minimum, the west extreme. */
  int64_t s = 0;
  for (int64_t t = 0; t < h; ++t)
    if (kx[out[t]] == kx[ax[2]] && ky[out[t]] == ky[ax[2]]) { s = t; break; }
  for (int64_t t = 0; t < h; ++t) hull[t] = out[(s + t) % h];
  free(out);
  for (int k = 1; k <= 4; ++k) free(q[k]);
  return h;
}

/* The full heaphull on the CPU's cores (the paper's divide-and-conquer
 * variant, Sec. III): chunked extremes and filter per thread, the labels of
 * the survivors, then the four queues, each hulled on every thread. */
int64_t or_heaphull_parallel(const int32_t* kx, const int32_t* ky, int64_t n, uint32_t* hull,
                             int nthreads) {
  if (n <= 0) return 0;
#ifdef _OPENMP
  if (nthreads <= 0) nthreads = omp_get_max_threads();
#else
  nthreads = 1;
#endif
  int64_t oct[8];
  uint32_t* surv = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
  const int64_t m = or_filter_parallel(kx, ky, n, oct, surv, nthreads);
  uint8_t* labels = (uint8_t*)calloc((size_t)n, 1);
  int64_t vx[8], vy[8];
  load_octagon(kx, ky, oct, vx, vy);
#pragma omp parallel for num_threads(nthreads) schedule(static)
  for (int64_t t = 0; t < m; ++t) labels[surv[t]] = (uint8_t)classify(kx[surv[t]], ky[surv[t]], vx, vy);
  const int64_t h = or_heaphull_queues(kx, ky, n, oct, labels, hull, NULL, nthreads);
  free(labels);
  free(surv);
  return h;
}

/* The heaphull pipeline: extremes -> octagon filter -> chain over survivors.
 * Returns h, or -1 when n == 0 is passed with a NULL hull (never fails
 * otherwise). survivors must hold n entries. */
int64_t or_heaphull(const int32_t* kx, const int32_t* ky, int64_t n,
                    uint32_t* survivors, uint32_t* hull) {
  if (n <= 0) return 0;
  int64_t oct[8];
  or_extremes(kx, ky, n, oct);
  int64_t m = or_filter(kx, ky, n, oct, survivors, NULL);
  return or_chain(kx, ky, n, survivors, m, hull);
}
