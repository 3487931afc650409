/* Symbolic fill of a sparse symmetric pattern in its given order.
 *
 * Input generation only: the method takes an already filled (chordal)
 * pattern V as its input, so computing V from a graph and an ordering is
 * part of building test and benchmark workloads, not of the method.
 *
 * Given the strict lower adjacency of a graph in compressed-column form
 * (rows > column, any order, duplicates allowed), compute the pattern of
 * the Cholesky factor in that order (diagonal included), column by column:
 * the rows of column j are the rows of the graph below j, merged with the
 * rows of every already-finished column whose first off-diagonal row is j.
 * Output rows are sorted ascending with the diagonal first.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* Returns nnz of the filled pattern (diagonal included), or -1 on
 * allocation failure.  *out_rowind is malloc'd; caller frees with
 * wl_free. */
int64_t wl_fill(int64_t n, const int64_t* acp, const int32_t* ari,
                int64_t* out_colptr, int32_t** out_rowind) {
  int64_t cap = (acp[n] + n) * 2 + 16, nnz = 0;
  int32_t* ri = (int32_t*)malloc(sizeof(int32_t) * cap);
  int32_t* mark = (int32_t*)malloc(sizeof(int32_t) * n);
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * n); /* child lists */
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * n);
  int32_t* buf = (int32_t*)malloc(sizeof(int32_t) * n);
  if (!ri || !mark || !head || !next || !buf) return -1;
  for (int64_t i = 0; i < n; ++i) { mark[i] = -1; head[i] = -1; }
  out_colptr[0] = 0;
  for (int64_t j = 0; j < n; ++j) {
    int64_t m = 0;
    mark[j] = (int32_t)j;
    for (int64_t p = acp[j]; p < acp[j + 1]; ++p) {
      int32_t r = ari[p];
      if (r > j && mark[r] != j) { mark[r] = (int32_t)j; buf[m++] = r; }
    }
    for (int64_t c = head[j]; c != -1; c = next[c]) {
      for (int64_t p = out_colptr[c] + 1; p < out_colptr[c + 1]; ++p) {
        int32_t r = ri[p];
        if (mark[r] != j) { mark[r] = (int32_t)j; buf[m++] = r; }
      }
    }
    qsort(buf, (size_t)m, sizeof(int32_t), cmp_i32);
    if (nnz + m + 1 > cap) {
      while (nnz + m + 1 > cap) cap *= 2;
      int32_t* nr = (int32_t*)realloc(ri, sizeof(int32_t) * cap);
      if (!nr) return -1;
      ri = nr;
    }
    ri[nnz++] = (int32_t)j;
    memcpy(ri + nnz, buf, sizeof(int32_t) * m);
    nnz += m;
    out_colptr[j + 1] = nnz;
    if (m > 0) { int32_t par = buf[0]; next[j] = head[par]; head[par] = j; }
  }
  free(mark); free(head); free(next); free(buf);
  *out_rowind = ri;
  return nnz;
}

void wl_free(void* p) { free(p); }
