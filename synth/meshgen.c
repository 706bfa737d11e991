/*
 * Seeded synthetic inputs for the eddy-current model problem (Sec. 1 and the
 * model problems of Sec. 6.1): a unit-cube lattice of N^3 hexahedra, each split
 * into six Kuhn tetrahedra, discretised with lowest-order (Whitney) edge
 * elements.  This file produces the edge operator A = S + M (or S, or M alone),
 * the discrete gradient D_h as (tail, head) node pairs, and the tetrahedra.
 *
 * It contains none of the multigrid method: it is the problem generator used by
 * both the CPU checker and the GPU path.
 *
 * Lattice conventions
 *   n = N + 1 nodes per side, node id = i + n*j + n*n*k.
 *   Every mesh edge joins a node v to v + d with d one of the seven offsets
 *   (1,0,0) (0,1,0) (1,1,0) (0,0,1) (1,0,1) (0,1,1) (1,1,1); it is oriented
 *   from the lower to the higher node id (tail -> head), and edges are numbered
 *   lexicographically by (tail, head).  Listed in that order the offsets have
 *   increasing id differences 1, n, n+1, n^2, n^2+1, n^2+n, n^2+n+1, so walking
 *   nodes in id order and offsets in this order yields the sorted edge list.
 *   Each hex with origin v0 holds the six tetrahedra
 *   v0, v0+e_p, v0+e_p+e_q, v0+(1,1,1) for the permutations (p,q,r) of (x,y,z).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC meshgen.c -o libsynth.so
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

static const int OFF[7][3] = {{1,0,0},{0,1,0},{1,1,0},{0,0,1},{1,0,1},{0,1,1},{1,1,1}};
static const int PERM[6][3] = {{0,1,2},{0,2,1},{1,0,2},{1,2,0},{2,0,1},{2,1,0}};

/* number of edges that leave node (i,j,k) towards a higher id */
static int node_out_mask(int n, int i, int j, int k) {
  int m = 0;
  for (int d = 0; d < 7; ++d) {
    int a = i + OFF[d][0], b = j + OFF[d][1], c = k + OFF[d][2];
    if (a < n && b < n && c < n) m |= 1 << d;
  }
  return m;
}

/* edge pointer: first edge id of every node; returns the number of edges */
int64_t synth_edge_ptr(int N, int64_t* eptr /* n^3 + 1 */) {
  int n = N + 1;
  int64_t e = 0, v = 0;
  for (int k = 0; k < n; ++k)
    for (int j = 0; j < n; ++j)
      for (int i = 0; i < n; ++i, ++v) {
        eptr[v] = e;
        e += __builtin_popcount(node_out_mask(n, i, j, k));
      }
  eptr[v] = e;
  return e;
}

/* fills tail/head (int32) for all edges, in lexicographic order */
void synth_edges(int N, const int64_t* eptr, int32_t* tail, int32_t* head) {
  int n = N + 1;
  int64_t nn = (int64_t)n * n * n;
#pragma omp parallel for schedule(static)
  for (int64_t v = 0; v < nn; ++v) {
    int i = (int)(v % n), j = (int)((v / n) % n), k = (int)(v / ((int64_t)n * n));
    int64_t e = eptr[v];
    for (int d = 0; d < 7; ++d) {
      int a = i + OFF[d][0], b = j + OFF[d][1], c = k + OFF[d][2];
      if (a < n && b < n && c < n) {
        tail[e] = (int32_t)v;
        head[e] = (int32_t)(a + (int64_t)n * b + (int64_t)n * n * c);
        ++e;
      }
    }
  }
}

/* id of the edge between nodes u < w (must exist) */
static int64_t edge_id(int n, const int64_t* eptr, int64_t u, int64_t w) {
  int i = (int)(u % n), j = (int)((u / n) % n), k = (int)(u / ((int64_t)n * n));
  int64_t diff = w - u;
  int64_t e = eptr[u];
  for (int d = 0; d < 7; ++d) {
    int a = i + OFF[d][0], b = j + OFF[d][1], c = k + OFF[d][2];
    if (a < n && b < n && c < n) {
      int64_t dd = OFF[d][0] + (int64_t)n * OFF[d][1] + (int64_t)n * n * OFF[d][2];
      if (dd == diff) return e;
      ++e;
    }
  }
  return -1;
}

/* tets (6 per hex, int32 node ids, 4 per tet) and their 6 edge ids, local edge
 * order (0,1) (0,2) (0,3) (1,2) (1,3) (2,3) over the vertex list
 * v0, v0+e_p, v0+e_p+e_q, v0+(1,1,1), whose ids increase along the list. */
void synth_tets(int N, const int64_t* eptr, int32_t* tets, int32_t* tet_edges) {
  int n = N + 1;
  int64_t nh = (int64_t)N * N * N;
#pragma omp parallel for schedule(static)
  for (int64_t h = 0; h < nh; ++h) {
    int i = (int)(h % N), j = (int)((h / N) % N), k = (int)(h / ((int64_t)N * N));
    for (int p = 0; p < 6; ++p) {
      int64_t t = h * 6 + p;
      int x[3] = {i, j, k};
      int64_t vid[4];
      vid[0] = x[0] + (int64_t)n * x[1] + (int64_t)n * n * x[2];
      for (int s = 0; s < 3; ++s) {
        x[PERM[p][s]] += 1;
        vid[s + 1] = x[0] + (int64_t)n * x[1] + (int64_t)n * n * x[2];
      }
      for (int s = 0; s < 4; ++s) tets[4 * t + s] = (int32_t)vid[s];
      int le = 0;
      for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b)
          tet_edges[6 * t + le++] = (int32_t)edge_id(n, eptr, vid[a], vid[b]);
    }
  }
}

/* gradients of the barycentric coordinates and volume of one tet */
static double tet_grads(const double* X, const int32_t* tv, double g[4][3]) {
  const double* x0 = X + 3 * (int64_t)tv[0];
  double J[3][3]; /* columns x_s - x0 */
  for (int s = 0; s < 3; ++s) {
    const double* xs = X + 3 * (int64_t)tv[s + 1];
    for (int r = 0; r < 3; ++r) J[r][s] = xs[r] - x0[r];
  }
  double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
               J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
               J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
  /* inverse of J: row s of J^{-1} is grad lambda_{s+1} */
  double inv[3][3];
  inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
  inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
  inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
  inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
  inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
  inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
  inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
  inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
  inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
  for (int r = 0; r < 3; ++r) {
    g[1][r] = inv[0][r];
    g[2][r] = inv[1][r];
    g[3][r] = inv[2][r];
    g[0][r] = -(inv[0][r] + inv[1][r] + inv[2][r]);
  }
  return fabs(det) / 6.0;
}

static double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}

static const int LE[6][2] = {{0,1},{0,2},{0,3},{1,2},{1,3},{2,3}};

/* Whitney element matrices; which: 0 -> S + sigma M, 1 -> S, 2 -> sigma M.
 * Local edge (a,b) runs from the lower to the higher node id, which is the
 * vertex-list order, so it carries the global orientation. */
static void element_matrix(const double* X, const int32_t* tv, double sigma, int which, double K[6][6]) {
  double g[4][3];
  double vol = tet_grads(X, tv, g);
  double cr[6][3];
  for (int e = 0; e < 6; ++e) cross3(g[LE[e][0]], g[LE[e][1]], cr[e]);
  for (int e = 0; e < 6; ++e) {
    int a = LE[e][0], b = LE[e][1];
    for (int f = 0; f < 6; ++f) {
      int c = LE[f][0], d = LE[f][1];
      double s = 4.0 * vol * dot3(cr[e], cr[f]);
      /* int lambda_x lambda_y = vol (1 + delta_xy) / 20 */
      double mac = vol * (1.0 + (a == c)) / 20.0, mad = vol * (1.0 + (a == d)) / 20.0;
      double mbc = vol * (1.0 + (b == c)) / 20.0, mbd = vol * (1.0 + (b == d)) / 20.0;
      double m = dot3(g[b], g[d]) * mac - dot3(g[b], g[c]) * mad - dot3(g[a], g[d]) * mbc + dot3(g[a], g[c]) * mbd;
      m *= sigma;
      K[e][f] = which == 0 ? s + m : (which == 1 ? s : m);
    }
  }
}

static int cmp_i32(const void* a, const void* b) {
  int32_t x = *(const int32_t*)a, y = *(const int32_t*)b;
  return (x > y) - (x < y);
}

/* edge -> tet incidence (CSR); returns nothing, fills ptr (ne+1) and list (6*ntet) */
void synth_edge_tets(int64_t ne, int64_t ntet, const int32_t* tet_edges, int64_t* ptr, int32_t* list) {
  memset(ptr, 0, sizeof(int64_t) * (ne + 1));
  for (int64_t t = 0; t < ntet; ++t)
    for (int s = 0; s < 6; ++s) ptr[tet_edges[6 * t + s] + 1]++;
  for (int64_t e = 0; e < ne; ++e) ptr[e + 1] += ptr[e];
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * ne);
  memcpy(cur, ptr, sizeof(int64_t) * ne);
  for (int64_t t = 0; t < ntet; ++t)
    for (int s = 0; s < 6; ++s) list[cur[tet_edges[6 * t + s]]++] = (int32_t)t;
  free(cur);
}

/* row lengths of the edge operator: union of the edges of all tets at each edge */
void synth_row_counts(int64_t ne, const int64_t* etp, const int32_t* etl, const int32_t* tet_edges, int64_t* cnt) {
#pragma omp parallel
  {
    int32_t buf[512];
#pragma omp for schedule(dynamic, 4096)
    for (int64_t e = 0; e < ne; ++e) {
      int m = 0;
      for (int64_t q = etp[e]; q < etp[e + 1]; ++q)
        for (int s = 0; s < 6; ++s) buf[m++] = tet_edges[6 * (int64_t)etl[q] + s];
      qsort(buf, m, sizeof(int32_t), cmp_i32);
      int u = 0;
      for (int r = 0; r < m; ++r)
        if (r == 0 || buf[r] != buf[r - 1]) ++u;
      cnt[e] = u;
    }
  }
}

/* fills sorted column indices and values of the edge operator */
void synth_assemble(int64_t ne, const int64_t* etp, const int32_t* etl, const int32_t* tets, const int32_t* tet_edges,
                    const double* X, const double* sigma, int which, const int64_t* rowptr, int32_t* col, double* val) {
#pragma omp parallel
  {
    int32_t buf[512];
    double K[6][6];
#pragma omp for schedule(dynamic, 4096)
    for (int64_t e = 0; e < ne; ++e) {
      int m = 0;
      for (int64_t q = etp[e]; q < etp[e + 1]; ++q)
        for (int s = 0; s < 6; ++s) buf[m++] = tet_edges[6 * (int64_t)etl[q] + s];
      qsort(buf, m, sizeof(int32_t), cmp_i32);
      int64_t r0 = rowptr[e];
      int u = 0;
      for (int r = 0; r < m; ++r)
        if (r == 0 || buf[r] != buf[r - 1]) { col[r0 + u] = buf[r]; val[r0 + u] = 0.0; ++u; }
      for (int64_t q = etp[e]; q < etp[e + 1]; ++q) {
        int64_t t = etl[q];
        const int32_t* te = tet_edges + 6 * t;
        int le = 0;
        while (te[le] != e) ++le;
        element_matrix(X, tets + 4 * t, sigma[t], which, K);
        for (int f = 0; f < 6; ++f) {
          /* binary search of te[f] in the row */
          int lo = 0, hi = u - 1;
          while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (col[r0 + mid] < te[f]) lo = mid + 1; else hi = mid;
          }
          val[r0 + lo] += K[le][f];
        }
      }
    }
  }
}

/* signed tet volumes (for the no-inversion check of jittered meshes) */
void synth_tet_volumes(int64_t ntet, const int32_t* tets, const double* X, double* vol) {
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < ntet; ++t) {
    const int32_t* tv = tets + 4 * t;
    const double* x0 = X + 3 * (int64_t)tv[0];
    double J[3][3];
    for (int s = 0; s < 3; ++s)
      for (int r = 0; r < 3; ++r) J[r][s] = X[3 * (int64_t)tv[s + 1] + r] - x0[r];
    vol[t] = (J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
              J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0])) / 6.0;
  }
}
