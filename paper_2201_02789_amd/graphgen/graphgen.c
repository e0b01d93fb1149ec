/*
 * Seeded synthetic graph generators (host C, OpenMP).
 *
 * This module only produces inputs: it holds none of the traversal
 * arithmetic.  Both the GPU path and the CPU oracle consume what it writes.
 *
 * The paper evaluates BFS and SSSP on a Kronecker graph
 * (kron_g500-simple-logn16, Table I).  That file is not available, so the
 * same family is generated here at configurable scale:
 *
 *   R-MAT: for each of edgefactor * 2^scale edge draws and each bit level
 *   (most significant first) one quadrant is picked with probabilities
 *   a/b/c/d: a -> (row bit 0, col bit 0), b -> (0,1), c -> (1,0), d -> (1,1).
 *   The uniform variate of (draw e, level l) is
 *       (splitmix64(seed * PHI + e * 64 + l) >> 11) * 2^-53
 *   so every variate is a pure function of (seed, e, l) and generation is
 *   order-independent and parallel.
 *
 *   Then: optional relabelling by a seeded Fisher-Yates permutation,
 *   self loops dropped, every edge stored in both directions, duplicates
 *   removed, rows sorted ascending.  Output is an int32 CSR.
 *
 *   Erdos-Renyi G(n, M): uniform distinct unordered pairs u != v, drawn
 *   from the counter stream splitmix64(seed * PHI + i) until M distinct
 *   pairs are held, then stored in both directions like R-MAT.
 *
 *   Weights: one uint32 per undirected edge, identical in both directions,
 *       w(u,v) = 1 + splitmix64(wseed * PHI + (min(u,v) << 32 | max(u,v))) % 255
 *   so w is uniform on [1, 255] up to the 2^64 mod 255 bias.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define PHI 0x9E3779B97F4A7C15ULL

static inline uint64_t splitmix64(uint64_t x) {
  x += PHI;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ULL;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBULL;
  return x ^ (x >> 31);
}

uint64_t gg_splitmix64(uint64_t x) { return splitmix64(x); }

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Seeded Fisher-Yates permutation of [0, n). */
void gg_permutation(int32_t n, uint64_t seed, int32_t* perm) {
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    uint64_t r = splitmix64(seed * PHI + (uint64_t)i);
    int32_t j = (int32_t)(r % (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

/*
 * Builds a symmetric, deduplicated, loop-free CSR from ne undirected edge
 * draws (src[i], dst[i]).  Writes row_ptr[n+1] and col[<= cap].
 * Returns the number of directed entries m, or -1 if cap is too small.
 */
static int64_t build_csr(int32_t n, int64_t ne, const int32_t* src, const int32_t* dst,
                         int32_t* row_ptr, int32_t* col, int64_t cap) {
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -2;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ne; ++i) {
    int32_t u = src[i], v = dst[i];
    if (u == v) continue;
#pragma omp atomic
    cnt[u + 1]++;
#pragma omp atomic
    cnt[v + 1]++;
  }
  for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  int64_t total = cnt[n];
  int32_t* tmp = (int32_t*)malloc((size_t)(total ? total : 1) * sizeof(int32_t));
  int64_t* cur = (int64_t*)malloc((size_t)n * sizeof(int64_t));
  if (!tmp || !cur) { free(cnt); free(tmp); free(cur); return -2; }
  memcpy(cur, cnt, (size_t)n * sizeof(int64_t));
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < ne; ++i) {
    int32_t u = src[i], v = dst[i];
    if (u == v) continue;
    int64_t pu, pv;
#pragma omp atomic capture
    pu = cur[u]++;
#pragma omp atomic capture
    pv = cur[v]++;
    tmp[pu] = v;
    tmp[pv] = u;
  }
  free(cur);
  /* sort and dedup each row in place; record unique counts */
  int64_t* ucnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!ucnt) { free(cnt); free(tmp); return -2; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; ++u) {
    int32_t* r = tmp + cnt[u];
    int64_t d = cnt[u + 1] - cnt[u];
    if (d > 1) qsort(r, (size_t)d, sizeof(int32_t), cmp_i32);
    int64_t k = 0;
    for (int64_t j = 0; j < d; ++j)
      if (k == 0 || r[j] != r[k - 1]) r[k++] = r[j];
    ucnt[u + 1] = k;
  }
  for (int32_t i = 0; i < n; ++i) ucnt[i + 1] += ucnt[i];
  int64_t m = ucnt[n];
  if (m > cap || m > INT32_MAX) { free(cnt); free(tmp); free(ucnt); return -1; }
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; ++u)
    memcpy(col + ucnt[u], tmp + cnt[u], (size_t)(ucnt[u + 1] - ucnt[u]) * sizeof(int32_t));
  for (int32_t i = 0; i <= n; ++i) row_ptr[i] = (int32_t)ucnt[i];
  free(cnt); free(tmp); free(ucnt);
  return m;
}

/*
 * R-MAT graph with n = 2^scale vertices and edgefactor * n edge draws.
 * perm_seed == 0 keeps the generated ids; otherwise ids are relabelled by
 * gg_permutation(n, perm_seed).  Returns m (directed CSR entries), -1 if
 * cap is too small, -2 on allocation failure, -3 on bad arguments.
 */
int64_t gg_rmat(int32_t scale, int32_t edgefactor, double a, double b, double c, uint64_t seed,
                uint64_t perm_seed, int32_t* row_ptr, int32_t* col, int64_t cap) {
  if (scale < 1 || scale > 30 || edgefactor < 1) return -3;
  int32_t n = (int32_t)1 << scale;
  int64_t ne = (int64_t)edgefactor * n;
  int32_t* src = (int32_t*)malloc((size_t)ne * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)ne * sizeof(int32_t));
  if (!src || !dst) { free(src); free(dst); return -2; }
  const double ab = a + b, abc = a + b + c;
  const double inv53 = 1.0 / 9007199254740992.0;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < ne; ++e) {
    uint32_t r = 0, cc = 0;
    for (int32_t l = 0; l < scale; ++l) {
      double x = (double)(splitmix64(seed * PHI + (uint64_t)e * 64u + (uint64_t)l) >> 11) * inv53;
      uint32_t rb, cb;
      if (x < a) { rb = 0; cb = 0; }
      else if (x < ab) { rb = 0; cb = 1; }
      else if (x < abc) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      r |= rb << (scale - 1 - l);
      cc |= cb << (scale - 1 - l);
    }
    src[e] = (int32_t)r;
    dst[e] = (int32_t)cc;
  }
  if (perm_seed) {
    int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
    if (!perm) { free(src); free(dst); return -2; }
    gg_permutation(n, perm_seed, perm);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < ne; ++e) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
    free(perm);
  }
  int64_t m = build_csr(n, ne, src, dst, row_ptr, col, cap);
  free(src); free(dst);
  return m;
}

/* Open-addressing set of canonical pairs (u << 32 | v), u < v. */
static int set_insert(uint64_t* tab, uint64_t mask, uint64_t key) {
  uint64_t h = splitmix64(key) & mask;
  for (;;) {
    if (tab[h] == UINT64_MAX) { tab[h] = key; return 1; }
    if (tab[h] == key) return 0;
    h = (h + 1) & mask;
  }
}

/*
 * Erdos-Renyi G(n, M): M distinct undirected pairs.  Returns m = 2M, -1 if
 * cap is too small, -2 on allocation failure, -3 on bad arguments.
 */
int64_t gg_er(int32_t n, int64_t M, uint64_t seed, int32_t* row_ptr, int32_t* col, int64_t cap) {
  if (n < 2 || M < 0 || M > (int64_t)n * (n - 1) / 2) return -3;
  uint64_t sz = 1;
  while (sz < (uint64_t)M * 2 + 16) sz <<= 1;
  uint64_t* tab = (uint64_t*)malloc(sz * sizeof(uint64_t));
  int32_t* src = (int32_t*)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
  int32_t* dst = (int32_t*)malloc((size_t)(M ? M : 1) * sizeof(int32_t));
  if (!tab || !src || !dst) { free(tab); free(src); free(dst); return -2; }
  memset(tab, 0xFF, sz * sizeof(uint64_t));
  int64_t have = 0;
  for (uint64_t i = 0; have < M; ++i) {
    uint64_t r = splitmix64(seed * PHI + i);
    uint32_t u = (uint32_t)((r >> 32) % (uint64_t)n), v = (uint32_t)((r & 0xFFFFFFFFu) % (uint64_t)n);
    if (u == v) continue;
    if (u > v) { uint32_t t = u; u = v; v = t; }
    if (set_insert(tab, sz - 1, ((uint64_t)u << 32) | v)) { src[have] = (int32_t)u; dst[have] = (int32_t)v; ++have; }
  }
  free(tab);
  int64_t m = build_csr(n, M, src, dst, row_ptr, col, cap);
  free(src); free(dst);
  return m;
}

/* Per-undirected-edge weights in [1, 255], identical in both directions. */
void gg_weights(int32_t n, const int32_t* row_ptr, const int32_t* col, uint64_t wseed, uint32_t* w) {
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t u = 0; u < n; ++u)
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      uint64_t lo = (uint64_t)(u < col[e] ? u : col[e]), hi = (uint64_t)(u < col[e] ? col[e] : u);
      w[e] = 1u + (uint32_t)(splitmix64(wseed * PHI + ((lo << 32) | hi)) % 255u);
    }
}

int32_t gg_num_threads(void) { return omp_get_max_threads(); }
