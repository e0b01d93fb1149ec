/*
 * CPU oracle for nested-parallel BFS and SSSP.  TEST INFRASTRUCTURE ONLY:
 * the tests, the smoke check and the benchmark's CPU-baseline leg call it;
 * the GPU library never links or calls it, and it includes nothing from the
 * GPU path.
 *
 * The paper's three transformations (thresholding, Sec. III; coarsening,
 * Sec. IV; aggregation, Sec. V) only reschedule the child work: Sec. VI
 * states that any combination in any order yields correct code, and
 * Sec. III-D that the threshold choice cannot change the result.  The
 * optimised traversal therefore computes exactly the plain definitions,
 * which is what this file implements:
 *
 *   BFS (Table I, BFS benchmark): level[v] = fewest edges on a path from the
 *   source to v, -1 when v is unreachable.  FIFO queue, textbook order.
 *
 *   SSSP (Table I, SSSP benchmark): dist[v] = minimum total weight of a path
 *   from the source to v with non-negative integer weights, 0xFFFFFFFF when
 *   unreachable.  Dijkstra with a binary min-heap and lazy deletion,
 *   accumulating in uint64.
 */
#include <stdint.h>
#include <stdlib.h>

#define ORACLE_OK 0
#define ORACLE_ERR_ARG (-1)
#define ORACLE_ERR_MEM (-2)
#define ORACLE_ERR_RANGE (-3)

/* Returns the number of distinct levels (eccentricity of src + 1), or < 0. */
int32_t oracle_bfs(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t src,
                   int32_t* level) {
  if (n <= 0 || !row_ptr || !level || src < 0 || src >= n) return ORACLE_ERR_ARG;
  int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  if (!queue) return ORACLE_ERR_MEM;
  for (int32_t v = 0; v < n; ++v) level[v] = -1;
  int32_t head = 0, tail = 0, depth = 0;
  level[src] = 0;
  queue[tail++] = src;
  while (head < tail) {
    int32_t u = queue[head++];
    int32_t lu = level[u];
    if (lu + 1 > depth) depth = lu + 1;
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col_idx[e];
      if (level[v] == -1) {
        level[v] = lu + 1;
        queue[tail++] = v;
      }
    }
  }
  free(queue);
  return depth;
}

/* Binary min-heap of (distance, vertex) pairs. */
typedef struct { uint64_t d; int32_t v; } hitem;

static void heap_push(hitem* h, int64_t* size, uint64_t d, int32_t v) {
  int64_t i = (*size)++;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p].d <= d) break;
    h[i] = h[p];
    i = p;
  }
  h[i].d = d;
  h[i].v = v;
}

static hitem heap_pop(hitem* h, int64_t* size) {
  hitem top = h[0];
  hitem last = h[--(*size)];
  int64_t i = 0, s = *size;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, c = i;
    uint64_t cd = last.d;
    if (l < s && h[l].d < cd) { c = l; cd = h[l].d; }
    if (r < s && h[r].d < cd) { c = r; }
    if (c == i) break;
    h[i] = h[c];
    i = c;
  }
  if (s > 0) h[i] = last;
  return top;
}

/*
 * Returns the number of settled vertices, or < 0.  ORACLE_ERR_RANGE if a
 * finite distance does not fit below 0xFFFFFFFF.
 */
int64_t oracle_dijkstra(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                        const uint32_t* w, int32_t src, uint32_t* dist) {
  if (n <= 0 || !row_ptr || !dist || src < 0 || src >= n) return ORACLE_ERR_ARG;
  int64_t m = row_ptr[n];
  if (m > 0 && (!col_idx || !w)) return ORACLE_ERR_ARG;
  uint64_t* d = (uint64_t*)malloc((size_t)n * sizeof(uint64_t));
  hitem* heap = (hitem*)malloc((size_t)(m + 1) * sizeof(hitem));
  if (!d || !heap) { free(d); free(heap); return ORACLE_ERR_MEM; }
  const uint64_t INF = UINT64_MAX;
  for (int32_t v = 0; v < n; ++v) d[v] = INF;
  int64_t size = 0, settled = 0;
  d[src] = 0;
  heap_push(heap, &size, 0, src);
  while (size > 0) {
    hitem it = heap_pop(heap, &size);
    if (it.d != d[it.v]) continue; /* stale entry */
    ++settled;
    int32_t u = it.v;
    for (int32_t e = row_ptr[u]; e < row_ptr[u + 1]; ++e) {
      int32_t v = col_idx[e];
      uint64_t nd = it.d + (uint64_t)w[e];
      if (nd < d[v]) {
        d[v] = nd;
        heap_push(heap, &size, nd, v);
      }
    }
  }
  int64_t rc = settled;
  for (int32_t v = 0; v < n; ++v) {
    if (d[v] == INF) dist[v] = 0xFFFFFFFFu;
    else if (d[v] >= 0xFFFFFFFFull) { dist[v] = 0xFFFFFFFFu; rc = ORACLE_ERR_RANGE; }
    else dist[v] = (uint32_t)d[v];
  }
  free(d);
  free(heap);
  return rc;
}
