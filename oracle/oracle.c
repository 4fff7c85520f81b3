/*
 * CPU oracle for the semiring sparse contraction (test infrastructure only).
 *
 * Plain, slow, obviously-correct reference code.  Only the tests, the smoke
 * check and the benchmark's CPU-baseline leg call it; the product path never
 * does.  It shares no code, header or table with the GPU library.
 *
 * What it follows (Solomonik and Hoefler, "Sparse Tensor Algebra as a Parallel
 * Programming Model"):
 *   - Section 3.1 / Table 1: a semiring is (add op, add identity, mul op,
 *     mul identity); the tropical semiring on int is (min, INT_MAX/2, +, 0).
 *   - Section 3.3.1: an indexed contraction is the nest of loops over every
 *     distinct index with the elementwise product accumulated by the output's
 *     additive operator in the innermost loop.  For C["ij"] (+)= A["ik"] (x) B["kj"]
 *     that is  C_ij = (+)_{k} A_ik (x) B_kj  over the stored entries.
 *   - Section 3.2: a new sparse tensor holds no entries; a new dense tensor is
 *     filled with the additive identity; data enters as index-value pairs.
 *   - Section 4.2: Bellman-Ford as tropical matrix-vector products
 *     P <- P (+) A (x) P until P stops changing (at most |V| rounds without a
 *     negative cycle); path doubling A <- A (+) A (x) A.
 *
 * Readings where the paper is silent (each is listed with its reason in the
 * design notes):
 *   - an operand entry equal to the additive identity is absent;
 *   - (min,+) on int32: (x) is exact integer addition, and a result at or above
 *     the identity is clamped to it (hence absent);
 *   - duplicate index-value pairs are combined with (+) in input order; float
 *     (+,x) duplicates are summed in fp64 in that order and rounded once to the
 *     stored type;
 *   - output entries equal to the additive identity are dropped; output rows
 *     list columns in ascending order;
 *   - (+,x) contractions are computed with the compensated dot product Dot2
 *     (Ogita, Rump and Oishi, "Accurate sum and dot product", SISC 2005): each
 *     product is split exactly with an fma, partial sums with TwoSum, so the
 *     fp64 result is as accurate as if computed in twice the working precision.
 *   - (max,x) and float (min,+): the product is rounded to the stored type (an
 *     fp32 product or sum formed in fp64 and rounded once is the correctly
 *     rounded fp32 result), then compared exactly.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

enum { ORC_PLUS_TIMES = 0, ORC_MIN_PLUS = 1, ORC_OR_AND = 2, ORC_MAX_TIMES = 3 };
enum { ORC_F64 = 0, ORC_F32 = 1, ORC_I32 = 2, ORC_U8 = 3 };

int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int t) { if (t > 0) omp_set_num_threads(t); }

/* ---------------------------------------------------------------- values -- */

/* Element read as a "wide" value: int64 for int32, double for floats, 0/1
 * for booleans. */
static double rd_f(const void *v, int dt, int64_t i) {
  return dt == ORC_F64 ? ((const double *)v)[i] : (double)((const float *)v)[i];
}
static int64_t rd_i(const void *v, int dt, int64_t i) {
  return dt == ORC_I32 ? (int64_t)((const int32_t *)v)[i]
                       : (int64_t)(((const uint8_t *)v)[i] != 0);
}
static int is_float(int dt) { return dt == ORC_F64 || dt == ORC_F32; }
/* (+,x) results are returned in fp64; other float semirings keep the type. */
static int out_is_double(int sr, int dt) {
  return dt == ORC_F64 || (dt == ORC_F32 && sr == ORC_PLUS_TIMES);
}

/* Round a double to the stored float type (identity for fp64). */
static double to_store(double x, int dt) { return dt == ORC_F32 ? (double)(float)x : x; }

/* Semiring product of two present entries, in the stored type. */
static double mul_f(int sr, int dt, double a, double b) {
  if (sr == ORC_MIN_PLUS) return to_store(a + b, dt);
  return to_store(a * b, dt); /* MAX_TIMES; PLUS_TIMES handled by Dot2 */
}
static double add_f(int sr, double a, double b) {
  if (sr == ORC_MIN_PLUS) return a < b ? a : b;
  if (sr == ORC_MAX_TIMES) return a > b ? a : b;
  return a + b;
}
static int64_t mul_i(int sr, int64_t a, int64_t b) {
  if (sr == ORC_MIN_PLUS) return a + b;
  return a & b; /* OR_AND */
}
static int64_t add_i(int sr, int64_t a, int64_t b) {
  if (sr == ORC_MIN_PLUS) return a < b ? a : b;
  return a | b;
}

/* Dot2 building blocks (error-free transformations). */
static void two_sum(double a, double b, double *s, double *e) {
  double x = a + b;
  double z = x - a;
  *e = (a - (x - z)) + (b - z);
  *s = x;
}
static void two_prod(double a, double b, double *p, double *e) {
  double x = a * b;
  *e = fma(a, b, -x);
  *p = x;
}

/* ------------------------------------------------------------------ fold -- */

typedef struct { int64_t r, c, i; } orc_key;
static int key_cmp(const void *pa, const void *pb) {
  const orc_key *a = pa, *b = pb;
  if (a->r != b->r) return a->r < b->r ? -1 : 1;
  if (a->c != b->c) return a->c < b->c ? -1 : 1;
  return a->i < b->i ? -1 : (a->i > b->i);
}

/* Index-value pairs (row, col, val) -> CSR with ascending columns.
 * Duplicates are combined with (+) in input order; entries equal to the
 * additive identity (before or after combining) are dropped.
 * Outputs must hold nnz entries; *out_nnz receives the kept count.
 * Float values: combined in fp64 in input order, rounded once; for
 * OR_AND any nonzero byte is "true". */
int orc_fold(int sr, int dt, const void *add_id, int64_t nnz, const int64_t *rows,
             const int64_t *cols, const void *vals, int64_t nrows, int64_t *rowptr,
             int32_t *col_out, void *val_out, int64_t *out_nnz) {
  orc_key *k = (orc_key *)malloc(sizeof(orc_key) * (size_t)(nnz > 0 ? nnz : 1));
  if (!k) return -1;
  for (int64_t i = 0; i < nnz; i++) { k[i].r = rows[i]; k[i].c = cols[i]; k[i].i = i; }
  qsort(k, (size_t)nnz, sizeof(orc_key), key_cmp);
  for (int64_t r = 0; r <= nrows; r++) rowptr[r] = 0;
  double idf = is_float(dt) ? rd_f(add_id, dt, 0) : 0.0;
  int64_t idi = is_float(dt) ? 0 : rd_i(add_id, dt, 0);
  int64_t o = 0;
  for (int64_t a = 0; a < nnz;) {
    int64_t b = a;
    while (b < nnz && k[b].r == k[a].r && k[b].c == k[a].c) b++;
    int keep;
    if (is_float(dt)) {
      double acc = idf;
      int any = 0;
      for (int64_t t = a; t < b; t++) {
        double v = rd_f(vals, dt, k[t].i);
        if (v == idf) continue; /* an identity entry is absent */
        acc = any ? add_f(sr, acc, v) : v;
        any = 1;
      }
      acc = to_store(acc, dt);
      keep = any && acc != idf;
      if (keep) {
        if (dt == ORC_F64) ((double *)val_out)[o] = acc;
        else ((float *)val_out)[o] = (float)acc;
      }
    } else {
      int64_t acc = idi;
      int any = 0;
      for (int64_t t = a; t < b; t++) {
        int64_t v = rd_i(vals, dt, k[t].i);
        if (v == idi) continue;
        acc = any ? add_i(sr, acc, v) : v;
        any = 1;
      }
      keep = any && acc != idi;
      if (keep) {
        if (dt == ORC_I32) ((int32_t *)val_out)[o] = (int32_t)acc;
        else ((uint8_t *)val_out)[o] = 1;
      }
    }
    if (keep) {
      col_out[o] = (int32_t)k[a].c;
      rowptr[k[a].r + 1]++;
      o++;
    }
    a = b;
  }
  for (int64_t r = 0; r < nrows; r++) rowptr[r + 1] += rowptr[r];
  *out_nnz = o;
  free(k);
  return 0;
}

/* --------------------------------------------------------------- SpGEMM -- */

/* One output row of C = A (x) B (optionally (+) C_old), by the definition
 * C_ij = (+)_{k:(i,k) in A,(k,j) in B} A_ik (x) B_kj.  The loop over k and j is
 * the innermost accumulation of the paper's loop nest; a dense row of
 * per-column accumulators stands in for C's row i.
 * Scratch arrays have length n.  Returns the number of entries written (or,
 * with write = 0, counted). */
typedef struct {
  double *s, *c;   /* float accumulators (sum and Dot2 correction) */
  int64_t *iv;     /* int accumulators */
  uint8_t *seen;
  int32_t *list;
} orc_row_ws;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static int64_t spgemm_row(int sr, int dt, double idf, int64_t idi, int64_t i,
                          const int64_t *ra, const int32_t *ca, const void *va,
                          const int64_t *rb, const int32_t *cb, const void *vb,
                          const int64_t *rc, const int32_t *cc, const void *vc,
                          orc_row_ws *w, int write, int32_t *oc, void *ov) {
  int64_t cnt = 0;
  int fl = is_float(dt);
  /* previous C entries join the (+) when accumulating */
  if (rc) {
    for (int64_t p = rc[i]; p < rc[i + 1]; p++) {
      int32_t j = cc[p];
      if (fl) {
        double v = rd_f(vc, dt, p);
        if (v == idf) continue;
        if (!w->seen[j]) { w->seen[j] = 1; w->list[cnt++] = j; w->s[j] = v; w->c[j] = 0.0; }
        else if (sr == ORC_PLUS_TIMES) { double s, e; two_sum(w->s[j], v, &s, &e); w->s[j] = s; w->c[j] += e; }
        else w->s[j] = add_f(sr, w->s[j], v);
      } else {
        int64_t v = rd_i(vc, dt, p);
        if (v == idi) continue;
        if (!w->seen[j]) { w->seen[j] = 1; w->list[cnt++] = j; w->iv[j] = v; }
        else w->iv[j] = add_i(sr, w->iv[j], v);
      }
    }
  }
  for (int64_t p = ra[i]; p < ra[i + 1]; p++) {
    int32_t k = ca[p];
    if (fl) {
      double a = rd_f(va, dt, p);
      if (a == idf) continue;
      for (int64_t q = rb[k]; q < rb[k + 1]; q++) {
        double b = rd_f(vb, dt, q);
        if (b == idf) continue;
        int32_t j = cb[q];
        if (sr == ORC_PLUS_TIMES) {
          double pr, ep;
          two_prod(a, b, &pr, &ep);
          if (!w->seen[j]) { w->seen[j] = 1; w->list[cnt++] = j; w->s[j] = pr; w->c[j] = ep; }
          else { double s, e; two_sum(w->s[j], pr, &s, &e); w->s[j] = s; w->c[j] += e + ep; }
        } else {
          double x = mul_f(sr, dt, a, b);
          if (!w->seen[j]) { w->seen[j] = 1; w->list[cnt++] = j; w->s[j] = x; }
          else w->s[j] = add_f(sr, w->s[j], x);
        }
      }
    } else {
      int64_t a = rd_i(va, dt, p);
      if (a == idi) continue;
      for (int64_t q = rb[k]; q < rb[k + 1]; q++) {
        int64_t b = rd_i(vb, dt, q);
        if (b == idi) continue;
        int32_t j = cb[q];
        int64_t x = mul_i(sr, a, b);
        if (!w->seen[j]) { w->seen[j] = 1; w->list[cnt++] = j; w->iv[j] = x; }
        else w->iv[j] = add_i(sr, w->iv[j], x);
      }
    }
  }
  qsort(w->list, (size_t)cnt, sizeof(int32_t), cmp_i32);
  int64_t o = 0;
  for (int64_t t = 0; t < cnt; t++) {
    int32_t j = w->list[t];
    w->seen[j] = 0;
    if (fl) {
      double v = sr == ORC_PLUS_TIMES ? w->s[j] + w->c[j] : w->s[j];
      if (v == idf) continue; /* identity results are absent */
      if (write) {
        oc[o] = j;
        if (out_is_double(sr, dt)) ((double *)ov)[o] = v;
        else ((float *)ov)[o] = (float)v;
      }
    } else {
      int64_t v = w->iv[j];
      if (sr == ORC_MIN_PLUS && v >= idi) continue; /* clamp to identity: absent */
      if (v == idi) continue;
      if (write) {
        oc[o] = j;
        if (dt == ORC_I32) ((int32_t *)ov)[o] = (int32_t)v;
        else ((uint8_t *)ov)[o] = 1;
      }
    }
    o++;
  }
  return o;
}

static int ws_alloc(orc_row_ws *w, int64_t n) {
  size_t nn = (size_t)(n > 0 ? n : 1);
  w->s = (double *)malloc(nn * sizeof(double));
  w->c = (double *)malloc(nn * sizeof(double));
  w->iv = (int64_t *)malloc(nn * sizeof(int64_t));
  w->seen = (uint8_t *)calloc(nn, 1);
  w->list = (int32_t *)malloc(nn * sizeof(int32_t));
  return w->s && w->c && w->iv && w->seen && w->list;
}
static void ws_free(orc_row_ws *w) { free(w->s); free(w->c); free(w->iv); free(w->seen); free(w->list); }

/* Count (phase 0) or write (phase 1) the selected rows of C = A (x) B
 * [(+) C_old].  rowsel lists the rows (nsel of them); counts[t] is the entry
 * count of row rowsel[t] and offs[t] where its entries go in the output
 * (phase 1 only).  Float values come back as fp64 (oc/ov), others in the
 * stored type.  Rows are processed in parallel. */
int orc_spgemm_rows(int phase, int sr, int dt, const void *add_id, int64_t n,
                    const int64_t *ra, const int32_t *ca, const void *va,
                    const int64_t *rb, const int32_t *cb, const void *vb,
                    const int64_t *rc, const int32_t *cc, const void *vc,
                    const int64_t *rowsel, int64_t nsel, int64_t *counts,
                    const int64_t *offs, int32_t *oc, void *ov) {
  double idf = is_float(dt) ? rd_f(add_id, dt, 0) : 0.0;
  int64_t idi = is_float(dt) ? 0 : rd_i(add_id, dt, 0);
  int err = 0;
#pragma omp parallel
  {
    orc_row_ws w;
    if (!ws_alloc(&w, n)) {
#pragma omp atomic write
      err = 1;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (int64_t t = 0; t < nsel; t++) {
        int64_t i = rowsel[t];
        if (phase == 0) {
          counts[t] = spgemm_row(sr, dt, idf, idi, i, ra, ca, va, rb, cb, vb, rc, cc, vc,
                                 &w, 0, NULL, NULL);
        } else {
          void *dst;
          if (out_is_double(sr, dt)) dst = (double *)ov + offs[t];
          else if (dt == ORC_F32) dst = (float *)ov + offs[t];
          else if (dt == ORC_I32) dst = (int32_t *)ov + offs[t];
          else dst = (uint8_t *)ov + offs[t];
          spgemm_row(sr, dt, idf, idi, i, ra, ca, va, rb, cb, vb, rc, cc, vc, &w, 1,
                     oc + offs[t], dst);
        }
      }
    }
    ws_free(&w);
  }
  return err ? -1 : 0;
}

/* ----------------------------------------------------------------- SpMM -- */

/* Y[i,:] = [X0[i,:] (+)] (+)_{k in A_i} A_ik (x) X[k,:] for a dense row-major X
 * of width s (n rows).  With self_term, row i of X itself joins the (+)
 * (the Bellman-Ford update P <- P (+) A (x) P).  Absent (identity) entries of
 * X are skipped.  (+,x) results are fp64 (Dot2); other semirings in the
 * stored type.  Returns in *changed whether Y differs from X (self_term). */
int orc_spmm(int sr, int dt, const void *add_id, int64_t m, int64_t s,
             const int64_t *ra, const int32_t *ca, const void *va, const void *x,
             int self_term, void *y, int *changed) {
  double idf = is_float(dt) ? rd_f(add_id, dt, 0) : 0.0;
  int64_t idi = is_float(dt) ? 0 : rd_i(add_id, dt, 0);
  int ch = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : ch)
  for (int64_t i = 0; i < m; i++) {
    for (int64_t c = 0; c < s; c++) {
      if (is_float(dt)) {
        double acc = idf, corr = 0.0;
        int any = 0;
        if (self_term) {
          double v = rd_f(x, dt, i * s + c);
          if (v != idf) { acc = v; any = 1; }
        }
        for (int64_t p = ra[i]; p < ra[i + 1]; p++) {
          double a = rd_f(va, dt, p);
          double b = rd_f(x, dt, (int64_t)ca[p] * s + c);
          if (a == idf || b == idf) continue;
          if (sr == ORC_PLUS_TIMES) {
            double pr, ep, t, e;
            two_prod(a, b, &pr, &ep);
            if (!any) { acc = pr; corr = ep; any = 1; }
            else { two_sum(acc, pr, &t, &e); acc = t; corr += e + ep; }
          } else {
            double v = mul_f(sr, dt, a, b);
            acc = any ? add_f(sr, acc, v) : v;
            any = 1;
          }
        }
        double out = sr == ORC_PLUS_TIMES ? acc + corr : acc;
        if (!any) out = idf;
        if (sr != ORC_PLUS_TIMES && dt == ORC_F32) out = (double)(float)out;
        if (sr == ORC_PLUS_TIMES || dt == ORC_F64) ((double *)y)[i * s + c] = out;
        else ((float *)y)[i * s + c] = (float)out;
        if (self_term && out != rd_f(x, dt, i * s + c)) ch = 1;
      } else {
        int64_t acc = idi;
        int any = 0;
        if (self_term) {
          int64_t v = rd_i(x, dt, i * s + c);
          if (v != idi) { acc = v; any = 1; }
        }
        for (int64_t p = ra[i]; p < ra[i + 1]; p++) {
          int64_t a = rd_i(va, dt, p);
          int64_t b = rd_i(x, dt, (int64_t)ca[p] * s + c);
          if (a == idi || b == idi) continue;
          int64_t v = mul_i(sr, a, b);
          acc = any ? add_i(sr, acc, v) : v;
          any = 1;
        }
        if (sr == ORC_MIN_PLUS && acc > idi) acc = idi;
        if (dt == ORC_I32) ((int32_t *)y)[i * s + c] = (int32_t)acc;
        else ((uint8_t *)y)[i * s + c] = (uint8_t)(acc != 0);
        if (self_term && acc != rd_i(x, dt, i * s + c)) ch = 1;
      }
    }
  }
  if (changed) *changed = ch;
  return 0;
}

/* Bellman-Ford over a semiring by repeated BSP steps P <- P (+) A (x) P
 * (Section 4.2).  P is n x s row-major, updated in place; a scratch buffer
 * of the same size is allocated here.  The loop runs until a step leaves P
 * unchanged; *iters receives the number of steps taken (including the final
 * unchanged one).  Gives up after max_iters steps (returns 1 = not
 * converged).  For (+,x) this is not meaningful and is rejected. */
int orc_bellman_ford(int sr, int dt, const void *add_id, int64_t n, int64_t s,
                     const int64_t *ra, const int32_t *ca, const void *va, void *p,
                     int64_t max_iters, int64_t *iters) {
  if (sr == ORC_PLUS_TIMES) return -2;
  size_t es = dt == ORC_F64 ? 8 : (dt == ORC_U8 ? 1 : 4);
  size_t bytes = (size_t)n * (size_t)s * es;
  void *q = malloc(bytes > 0 ? bytes : 1);
  if (!q) return -1;
  int64_t r = 0;
  int conv = 0;
  while (r < max_iters) {
    int changed = 0;
    orc_spmm(sr, dt, add_id, n, s, ra, ca, va, p, 1, q, &changed);
    memcpy(p, q, bytes);
    r++;
    if (!changed) { conv = 1; break; }
  }
  *iters = r;
  free(q);
  return conv ? 0 : 1;
}

/* ------------------------------------------------------ graph references -- */

/* Build out-edge lists (the transpose of A, whose row i holds in-edges). */
static void transpose_csr(int64_t n, const int64_t *ra, const int32_t *ca, int64_t **ro,
                          int32_t **co, int64_t **pos) {
  int64_t nnz = ra[n];
  int64_t *r = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *c = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t *ps = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  for (int64_t p = 0; p < nnz; p++) r[ca[p] + 1]++;
  for (int64_t i = 0; i < n; i++) r[i + 1] += r[i];
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) fill[i] = r[i];
  for (int64_t i = 0; i < n; i++)
    for (int64_t p = ra[i]; p < ra[i + 1]; p++) {
      int64_t o = fill[ca[p]]++;
      c[o] = (int32_t)i;
      ps[o] = p;
    }
  free(fill);
  *ro = r; *co = c; *pos = ps;
}

/* Breadth-first levels from each source over edges j -> i stored as A[i][j]:
 * levels[v * ns + t] = hop distance from sources[t], -1 if unreachable. */
int orc_bfs(int64_t n, const int64_t *ra, const int32_t *ca, const int64_t *sources,
            int64_t ns, int32_t *levels) {
  int64_t *ro; int32_t *co; int64_t *ps;
  transpose_csr(n, ra, ca, &ro, &co, &ps);
#pragma omp parallel
  {
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < ns; t++) {
      for (int64_t v = 0; v < n; v++) levels[v * ns + t] = -1;
      int64_t h = 0, e = 0;
      levels[sources[t] * ns + t] = 0;
      queue[e++] = sources[t];
      while (h < e) {
        int64_t u = queue[h++];
        for (int64_t p = ro[u]; p < ro[u + 1]; p++) {
          int64_t v = co[p];
          if (levels[v * ns + t] < 0) { levels[v * ns + t] = levels[u * ns + t] + 1; queue[e++] = v; }
        }
      }
    }
    free(queue);
  }
  free(ro); free(co); free(ps);
  return 0;
}

/* Dijkstra with a binary heap from each source; non-negative int weights
 * A[i][j] = w(j -> i).  dist[v * ns + t]; unreachable = inf_value. */
int orc_dijkstra(int64_t n, const int64_t *ra, const int32_t *ca, const int32_t *wa,
                 const int64_t *sources, int64_t ns, int64_t inf_value, int64_t *dist) {
  int64_t *ro; int32_t *co; int64_t *ps;
  transpose_csr(n, ra, ca, &ro, &co, &ps);
  int64_t nnz = ra[n];
#pragma omp parallel
  {
    int64_t cap = nnz + n + 1;
    int64_t *hk = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int64_t *hv = (int64_t *)malloc(sizeof(int64_t) * (size_t)cap);
    int64_t *d = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    uint8_t *done = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 1)
    for (int64_t t = 0; t < ns; t++) {
      for (int64_t v = 0; v < n; v++) { d[v] = inf_value; done[v] = 0; }
      int64_t hn = 0;
      d[sources[t]] = 0;
      hk[hn] = 0; hv[hn] = sources[t]; hn++;
      while (hn > 0) {
        int64_t key = hk[0], u = hv[0];
        hn--;
        /* sift down the last element from the root */
        int64_t lk = hk[hn], lv = hv[hn], x = 0;
        while (1) {
          int64_t l = 2 * x + 1, r = l + 1, m = x;
          int64_t mk = lk;
          if (l < hn && hk[l] < mk) { m = l; mk = hk[l]; }
          if (r < hn && hk[r] < mk) { m = r; mk = hk[r]; }
          if (m == x) break;
          hk[x] = hk[m]; hv[x] = hv[m]; x = m;
        }
        if (hn > 0) { hk[x] = lk; hv[x] = lv; }
        if (done[u] || key > d[u]) continue;
        done[u] = 1;
        for (int64_t p = ro[u]; p < ro[u + 1]; p++) {
          int64_t v = co[p];
          int64_t nd = key + wa[ps[p]];
          if (nd < d[v]) {
            d[v] = nd;
            int64_t y = hn++;
            while (y > 0) {
              int64_t par = (y - 1) / 2;
              if (hk[par] <= nd) break;
              hk[y] = hk[par]; hv[y] = hv[par]; y = par;
            }
            hk[y] = nd; hv[y] = v;
          }
        }
      }
      for (int64_t v = 0; v < n; v++) dist[v * ns + t] = d[v];
    }
    free(hk); free(hv); free(d); free(done);
  }
  free(ro); free(co); free(ps);
  return 0;
}

/* Floyd-Warshall on a dense n x n distance matrix (row i, col j = distance
 * from j to i, matching A's orientation); inf entries hold inf_value. */
int orc_floyd_warshall(int64_t n, int64_t *d, int64_t inf_value) {
  for (int64_t k = 0; k < n; k++)
    for (int64_t i = 0; i < n; i++) {
      int64_t dik = d[i * n + k];
      if (dik >= inf_value) continue;
      for (int64_t j = 0; j < n; j++) {
        int64_t dkj = d[k * n + j];
        if (dkj >= inf_value) continue;
        if (dik + dkj < d[i * n + j]) d[i * n + j] = dik + dkj;
      }
    }
  return 0;
}

/* Tiskin's path doubling for all-pairs shortest paths (Section 4.2).
 * A path is a (weight, hops) pair; of two paths the lighter is kept, and of
 * two equally light ones the one with fewer hops.  P starts as the identity
 * (weight 0, 0 hops on the diagonal) joined with the edges (weight, 1 hop).
 * Round l, for l = 1, 2, 4, ... while l < n: P_l = the entries of P with
 * exactly l hops, and P <- P (+) P_l (x) P, where (x) adds weights and hops
 * and both factors are the P from before the round.  Paths whose weight
 * reaches inf_value count as no path.  Orientation as A: row i, column j =
 * path j -> i.
 * d: n x n weights (inf_value where no path); h: n x n hops (-1 where none);
 * *rounds = rounds whose P_l had entries; pl_nnz[r] = entries of P_l in
 * round r (as many slots as rounds of the loop, at most 64).  Returns -1 on
 * a negative weight. */
int orc_apsp_tiskin(int64_t n, const int64_t *rowptr, const int32_t *col, const int32_t *w, int64_t inf_value,
                    int64_t *d, int64_t *h, int32_t *rounds, int64_t *pl_nnz) {
  const int64_t nn = n * n;
  for (int64_t e = 0; e < nn; e++) {
    const int diag = (e / n) == (e % n);
    d[e] = diag ? 0 : inf_value;
    h[e] = diag ? 0 : -1;
  }
  for (int64_t i = 0; i < n; i++)
    for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
      const int64_t x = w[p];
      if (x < 0) return -1;
      if (x >= inf_value) continue;
      const int64_t e = i * n + col[p];
      if (x < d[e] || (x == d[e] && 1 < h[e])) {
        d[e] = x;
        h[e] = 1;
      }
    }
  int64_t *nd = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn > 0 ? nn : 1));
  int64_t *nh = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn > 0 ? nn : 1));
  int32_t r = 0;
  for (int64_t l = 1; l < n; l <<= 1) {
    int64_t cnt = 0;
    for (int64_t e = 0; e < nn; e++) cnt += (h[e] == l);
    if (pl_nnz && r < 64) pl_nnz[r] = cnt;
    memcpy(nd, d, sizeof(int64_t) * (size_t)nn);
    memcpy(nh, h, sizeof(int64_t) * (size_t)nn);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < n; i++)
      for (int64_t k = 0; k < n; k++) {
        if (h[i * n + k] != l) continue;  /* P_l (i, k) */
        const int64_t wik = d[i * n + k], hik = h[i * n + k];
        for (int64_t j = 0; j < n; j++) {
          if (h[k * n + j] < 0) continue;
          const int64_t cw = wik + d[k * n + j], ch = hik + h[k * n + j];
          if (cw >= inf_value) continue;
          const int64_t e = i * n + j;
          if (cw < nd[e] || (cw == nd[e] && ch < nh[e])) {
            nd[e] = cw;
            nh[e] = ch;
          }
        }
      }
    memcpy(d, nd, sizeof(int64_t) * (size_t)nn);
    memcpy(h, nh, sizeof(int64_t) * (size_t)nn);
    if (cnt > 0) r++;
  }
  free(nd);
  free(nh);
  *rounds = r;
  return 0;
}
