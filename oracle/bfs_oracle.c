/*
 * CPU ORACLE -- test infrastructure, not part of the product.
 *
 * Only the test-suite, the smoke entry point and the benchmark's CPU-baseline
 * leg may load this code.  It shares no code with the HIP library.
 *
 * What it computes (the paper's EDGE BFS cascade, Cascade 1, Sec. "Expressing
 * BFS with EDGE"): from F_0 = {s}, P_0 = {s}, each level sets
 *   F_{i+1} = { d : some s in F_i has an edge (s,d) } minus P_i   (Eq. advance)
 *   P_{i+1} = P_i union F_{i+1}                                  (Eq. update)
 * and stops when F_{i+1} is empty.  The depth of v is the i with v in F_i,
 * i.e. the minimum number of hops from the source; unreached vertices get -1
 * (the paper's empty value, infinity).
 *
 * The implementation is the textbook FIFO-queue BFS, which reaches exactly the
 * same depths (a vertex is first dequeued in non-decreasing depth order).  The
 * parent recorded for v is the first dequeued in-neighbour at depth(v)-1; the
 * cascade's ANY reduction allows any such vertex.
 */
#include <stdint.h>
#include <stdlib.h>

/* Returns the number of levels (1 + largest depth), or -1 on bad input.
 * level, parent: n entries each (parent may be NULL); queue: n entries. */
int32_t oracle_bfs(int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                   int32_t source, int32_t *level, int32_t *parent, int32_t *queue) {
  if (n <= 0 || source < 0 || source >= n) return -1;
  for (int64_t v = 0; v < n; ++v) level[v] = -1;
  if (parent)
    for (int64_t v = 0; v < n; ++v) parent[v] = -1;
  int64_t head = 0, tail = 0;
  level[source] = 0;
  if (parent) parent[source] = source;
  queue[tail++] = source;
  int32_t maxlev = 0;
  while (head < tail) {
    int32_t u = queue[head++];
    int32_t du = level[u];
    for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
      int32_t v = col_idx[j];
      if (level[v] == -1) {
        level[v] = du + 1;
        if (parent) parent[v] = u;
        if (du + 1 > maxlev) maxlev = du + 1;
        queue[tail++] = v;
      }
    }
  }
  return maxlev + 1;
}

/*
 * Per-level work profile of one BFS, from its depths.  For each level k in
 * [0, nlev): with F_k = {v: depth v = k}, P_k = {v: 0 <= depth v <= k} and
 * U_k = V \ P_k,
 *   nF[k]    = |F_k|
 *   eF[k]    = sum of out-degrees over F_k
 *   nU[k]    = |U_k|
 *   eU[k]    = sum of in-degrees over U_k
 *   eScan[k] = in-edges a bottom-up step examines when every v in U_k scans
 *              its in-neighbours in ascending CSC order and stops at the first
 *              one in F_k (inclusive); all of them when none is in F_k.
 */
void oracle_level_profile(int64_t n, const int32_t *row_ptr,
                          const int32_t *csc_ptr, const int32_t *csc_idx,
                          const int32_t *level, int32_t nlev,
                          int64_t *nF, int64_t *eF, int64_t *nU, int64_t *eU, int64_t *eScan) {
  for (int32_t k = 0; k < nlev; ++k) {
    int64_t a = 0, b = 0, c = 0, d = 0, e = 0;
    for (int64_t v = 0; v < n; ++v) {
      int32_t lv = level[v];
      if (lv == k) { a++; b += row_ptr[v + 1] - row_ptr[v]; }
      if (lv < 0 || lv > k) {
        c++;
        d += csc_ptr[v + 1] - csc_ptr[v];
        int64_t j = csc_ptr[v];
        for (; j < csc_ptr[v + 1]; ++j)
          if (level[csc_idx[j]] == k) { ++j; break; }
        e += j - csc_ptr[v];
      }
    }
    nF[k] = a; eF[k] = b; nU[k] = c; eU[k] = d; eScan[k] = e;
  }
}
