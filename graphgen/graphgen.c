/*
 * graphgen.c -- seeded synthetic input graphs (R-MAT and 2D random geometric).
 *
 * This module is input preparation only.  It holds none of the partitioning
 * method's arithmetic: it draws random graphs and writes them as symmetric CSR
 * (int64 row offsets, int32 neighbour ids, rows sorted ascending, no
 * self-loops, no duplicate entries).  Both the oracle side and the device
 * side read the graphs it produces.
 *
 * Random numbers come from a counter-based SplitMix64: draw j of stream `key`
 * is mix(key + (j+1) * 0x9E3779B97F4A7C15), with mix the SplitMix64 output
 * function (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  Every sample owns its own stream, so the result
 * does not depend on the number of threads.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GG_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t gg_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t gg_draw(uint64_t key, uint64_t j) { return gg_mix(key + (j + 1) * GG_GOLDEN); }
static inline uint64_t gg_stream(uint64_t seed, uint64_t tag, uint64_t i) {
  return gg_mix(gg_mix(seed * GG_GOLDEN + tag) + i * GG_GOLDEN);
}

typedef struct gg_csr {
  int64_t n;
  int64_t m;        /* directed entries = 2 |E| */
  int64_t* rp;      /* n + 1 */
  int32_t* col;     /* m */
} gg_csr;

void gg_free(void* p) { free(p); }

/* When on, every finished phase of a generation prints a line to stderr. */
static int gg_progress = 0;
void gg_set_progress(int on) { gg_progress = on; }
static void gg_phase(const char* what, int64_t count) {
  if (gg_progress) {
    fprintf(stderr, "graphgen: %s (%lld)\n", what, (long long)count);
    fflush(stderr);
  }
}

/* Exposed for tests: raw draw and stream key. */
uint64_t gg_draw_u64(uint64_t seed, uint64_t tag, uint64_t i, uint64_t j) {
  return gg_draw(gg_stream(seed, tag, i), j);
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Sort non-negative int32 values: qsort for short rows, two 16-bit LSD
 * counting passes for long ones. */
static void sort_row(int32_t* row, int64_t d) {
  if (d < 2) return;
  if (d <= 512) { qsort(row, (size_t)d, sizeof(int32_t), cmp_i32); return; }
  int32_t* tmp = (int32_t*)malloc((size_t)d * sizeof(int32_t));
  int64_t* cnt = (int64_t*)malloc(65537 * sizeof(int64_t));
  if (!tmp || !cnt) { free(tmp); free(cnt); qsort(row, (size_t)d, sizeof(int32_t), cmp_i32); return; }
  for (int pass = 0; pass < 2; ++pass) {
    int32_t* src = pass ? tmp : row;
    int32_t* dst = pass ? row : tmp;
    int shift = pass * 16;
    memset(cnt, 0, 65537 * sizeof(int64_t));
    for (int64_t e = 0; e < d; ++e) cnt[(((uint32_t)src[e]) >> shift & 0xFFFF) + 1]++;
    for (int b = 0; b < 65536; ++b) cnt[b + 1] += cnt[b];
    for (int64_t e = 0; e < d; ++e) dst[cnt[((uint32_t)src[e]) >> shift & 0xFFFF]++] = src[e];
  }
  free(tmp);
  free(cnt);
}

/* Build symmetric CSR from sample pairs (u[i], v[i]); drops self-loops and
 * duplicates; rows sorted ascending. */
static int build_sym_csr(int64_t n, int64_t ns, const int32_t* su, const int32_t* sv, gg_csr* out) {
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ns; ++i) {
    if (su[i] == sv[i]) continue;
    __atomic_fetch_add(&cnt[su[i] + 1], 1, __ATOMIC_RELAXED);
    __atomic_fetch_add(&cnt[sv[i] + 1], 1, __ATOMIC_RELAXED);
  }
  for (int64_t v = 0; v < n; ++v) cnt[v + 1] += cnt[v];
  int64_t tot = cnt[n];
  gg_phase("degrees counted", tot);
  int32_t* tmp = (int32_t*)malloc((size_t)(tot > 0 ? tot : 1) * sizeof(int32_t));
  int64_t* pos = (int64_t*)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
  if (!tmp || !pos) { free(cnt); free(tmp); free(pos); return -1; }
  memcpy(pos, cnt, (size_t)n * sizeof(int64_t));
  /* order inside a row is arbitrary here; rows are sorted below */
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ns; ++i) {
    int32_t a = su[i], b = sv[i];
    if (a == b) continue;
    tmp[__atomic_fetch_add(&pos[a], 1, __ATOMIC_RELAXED)] = b;
    tmp[__atomic_fetch_add(&pos[b], 1, __ATOMIC_RELAXED)] = a;
  }
  free(pos);
  gg_phase("entries scattered", tot);
  int64_t* deg = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!deg) { free(cnt); free(tmp); return -1; }
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t v = 0; v < n; ++v) {
    int32_t* row = tmp + cnt[v];
    int64_t d = cnt[v + 1] - cnt[v];
    sort_row(row, d);
    int64_t w = 0;
    for (int64_t e = 0; e < d; ++e)
      if (w == 0 || row[w - 1] != row[e]) row[w++] = row[e];
    deg[v + 1] = w;
  }
  for (int64_t v = 0; v < n; ++v) deg[v + 1] += deg[v];
  int64_t m = deg[n];
  gg_phase("rows sorted and deduplicated", m);
  int32_t* col = (int32_t*)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
  if (!col) { free(cnt); free(tmp); free(deg); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t v = 0; v < n; ++v)
    memcpy(col + deg[v], tmp + cnt[v], (size_t)(deg[v + 1] - deg[v]) * sizeof(int32_t));
  free(cnt);
  free(tmp);
  out->n = n;
  out->m = m;
  out->rp = deg;
  out->col = col;
  return 0;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos, SDM 2004).  Each sample descends
 * `scale` levels, most significant bit first; at each level a 32-bit draw r
 * picks a quadrant: r < ta -> (0,0), r < tab -> (0,1), r < tabc -> (1,0),
 * else (1,1), where ta, tab, tabc are floor(cumulative probability * 2^32).
 * One 64-bit draw serves two levels (high half first).  If n < 2^scale an
 * endpoint >= n rejects the whole sample, which is redrawn from the same
 * stream.  No vertex permutation is applied.
 */
int gg_rmat(int32_t scale, int64_t n, int64_t nsamples, uint64_t seed,
            uint32_t ta, uint32_t tab, uint32_t tabc, gg_csr* out) {
  if (scale < 1 || scale > 31 || n < 1 || n > ((int64_t)1 << scale) || nsamples < 0) return -2;
  int32_t* su = (int32_t*)malloc((size_t)(nsamples > 0 ? nsamples : 1) * sizeof(int32_t));
  int32_t* sv = (int32_t*)malloc((size_t)(nsamples > 0 ? nsamples : 1) * sizeof(int32_t));
  if (!su || !sv) { free(su); free(sv); return -1; }
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < nsamples; ++i) {
    uint64_t key = gg_stream(seed, 0x524D4154ULL /* "RMAT" */, (uint64_t)i);
    uint64_t j = 0;
    int64_t u, v;
    for (;;) {
      u = 0;
      v = 0;
      uint64_t d = 0;
      for (int lv = 0; lv < scale; ++lv) {
        uint32_t r;
        if ((lv & 1) == 0) { d = gg_draw(key, j++); r = (uint32_t)(d >> 32); }
        else r = (uint32_t)(d & 0xFFFFFFFFULL);
        int rb, cb;
        if (r < ta) { rb = 0; cb = 0; }
        else if (r < tab) { rb = 0; cb = 1; }
        else if (r < tabc) { rb = 1; cb = 0; }
        else { rb = 1; cb = 1; }
        u = (u << 1) | rb;
        v = (v << 1) | cb;
      }
      if (u < n && v < n) break;
    }
    su[i] = (int32_t)u;
    sv[i] = (int32_t)v;
  }
  gg_phase("R-MAT samples drawn", nsamples);
  int rc = build_sym_csr(n, nsamples, su, sv, out);
  free(su);
  free(sv);
  return rc;
}

typedef struct { uint32_t y, x; int64_t idx; int64_t cell; } gg_pt;

static int cmp_pt(const void* a, const void* b) {
  const gg_pt* p = (const gg_pt*)a;
  const gg_pt* q = (const gg_pt*)b;
  if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
  if (p->y != q->y) return p->y < q->y ? -1 : 1;
  if (p->x != q->x) return p->x < q->x ? -1 : 1;
  return (p->idx > q->idx) - (p->idx < q->idx);
}

static uint64_t isqrt_ceil(uint64_t x) {
  uint64_t r = (uint64_t)sqrt((double)x);
  while (r * r < x) ++r;
  while (r > 0 && (r - 1) * (r - 1) >= x) --r;
  return r;
}

/*
 * 2D random geometric graph: n points with integer coordinates in
 * [0, 2^30)^2 (draws 0 and 1 of point i's stream, top 30 bits), an edge
 * between distinct points with dx^2 + dy^2 <= R2, R2 = floor(d * 2^60 /
 * (pi n)) so that the radius is sqrt(d / (pi n)) of the unit square and the
 * expected degree is about d away from the border.  Node ids follow a
 * row-major order of square grid cells of side 2^sh >= sqrt(R2), then
 * (y, x, draw index) inside a cell.
 */
int gg_rgg(int64_t n, double avg_degree, uint64_t seed, gg_csr* out) {
  if (n < 1 || n > ((int64_t)1 << 31) - 1 || !(avg_degree > 0.0)) return -2;
  const uint64_t R2 = (uint64_t)floor(avg_degree * 0x1p60 / (M_PI * (double)n));
  const uint64_t R = isqrt_ceil(R2);
  int lg = 0;                          /* G = 2^lg cells per side */
  while (lg < 15 && ((1ULL << (30 - (lg + 1))) >= R)) ++lg;
  const int sh = 30 - lg;
  const int64_t G = (int64_t)1 << lg;
  gg_pt* pts = (gg_pt*)malloc((size_t)n * sizeof(gg_pt));
  if (!pts) return -1;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    uint64_t key = gg_stream(seed, 0x52474721ULL /* "RGG!" */, (uint64_t)i);
    uint32_t x = (uint32_t)(gg_draw(key, 0) >> 34);
    uint32_t y = (uint32_t)(gg_draw(key, 1) >> 34);
    pts[i].x = x;
    pts[i].y = y;
    pts[i].idx = i;
    pts[i].cell = (int64_t)(y >> sh) * G + (int64_t)(x >> sh);
  }
  /* counting sort by cell, then (y, x, idx) inside each cell */
  int64_t ncell = G * G;
  int64_t* cs = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  gg_pt* srt = (gg_pt*)malloc((size_t)n * sizeof(gg_pt));
  if (!cs || !srt) { free(pts); free(cs); free(srt); return -1; }
  for (int64_t i = 0; i < n; ++i) cs[pts[i].cell + 1]++;
  for (int64_t c = 0; c < ncell; ++c) cs[c + 1] += cs[c];
  {
    int64_t* pos = (int64_t*)malloc((size_t)ncell * sizeof(int64_t));
    if (!pos) { free(pts); free(cs); free(srt); return -1; }
    memcpy(pos, cs, (size_t)ncell * sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i) srt[pos[pts[i].cell]++] = pts[i];
    free(pos);
  }
  free(pts);
#pragma omp parallel for schedule(dynamic, 256)
  for (int64_t c = 0; c < ncell; ++c) {
    int64_t d = cs[c + 1] - cs[c];
    if (d > 1) qsort(srt + cs[c], (size_t)d, sizeof(gg_pt), cmp_pt);
  }
  int64_t* rp = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!rp) { free(cs); free(srt); return -1; }
  /* pass 1: count; pass 2: fill.  Scanning the 3x3 cell block in row-major
   * order visits ids in increasing order, so rows come out sorted. */
  for (int pass = 0; pass < 2; ++pass) {
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t p = 0; p < n; ++p) {
      const int64_t cy = (int64_t)(srt[p].y >> sh), cx = (int64_t)(srt[p].x >> sh);
      int64_t w = pass ? rp[p] : 0;
      for (int64_t yy = cy - 1; yy <= cy + 1; ++yy) {
        if (yy < 0 || yy >= G) continue;
        for (int64_t xx = cx - 1; xx <= cx + 1; ++xx) {
          if (xx < 0 || xx >= G) continue;
          int64_t c = yy * G + xx;
          for (int64_t q = cs[c]; q < cs[c + 1]; ++q) {
            if (q == p) continue;
            int64_t dx = (int64_t)srt[p].x - (int64_t)srt[q].x;
            int64_t dy = (int64_t)srt[p].y - (int64_t)srt[q].y;
            uint64_t d2 = (uint64_t)(dx * dx) + (uint64_t)(dy * dy);
            if (d2 <= R2) {
              if (pass) out->col[w] = (int32_t)q;
              ++w;
            }
          }
        }
      }
      if (!pass) rp[p + 1] = w;
    }
    if (!pass) {
      for (int64_t p = 0; p < n; ++p) rp[p + 1] += rp[p];
      out->col = (int32_t*)malloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(int32_t));
      if (!out->col) { free(cs); free(srt); free(rp); return -1; }
    }
  }
  free(cs);
  free(srt);
  out->n = n;
  out->m = rp[n];
  out->rp = rp;
  return 0;
}
