// Hierarchy setup (Alg. 3 on every level): nodal operator, smoothed
// aggregation, coarse gradient, Emin_Setup pattern and local systems (Alg. 2),
// constrained energy minimisation of P^(e) (Sec. 3, Sec. 4), Galerkin RAP.
#include <chrono>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <limits>

#include "mpnn.hpp"

namespace hc {

// device scalar slots (Ctx::scal)
enum { S_RHO = 0, S_GAMMA, S_ALPHA, S_RHONEW, S_BETA, S_NX2, S_NY2, S_POWRHO, S_OMEGA, S_ENERGY, S_RHO0 };
// device integer flag slots (Ctx::iscal); 0 and 1 are used by the primitives
enum { F_BAD = 2, F_DISCONNECTED, F_MAXJ, F_MAXNP, F_TOOBIG, F_NOTSPD };
// slots 8-12 serve the solve; 13: rows with an infeasible constraint, 14: the
// largest such row + 1
enum { F_INFEASIBLE = 13, F_INFEASIBLE_ROW = 14 };

// ---------------------------------------------------------------------------
// discrete gradient
// ---------------------------------------------------------------------------
// Reads a caller CSR gradient: every row one -1 and one +1, or a single +-1
// (a Dirichlet edge whose other node was eliminated, Sec. 2); the absent end
// is stored as -1.
__global__ void k_grad_from_csr(const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ val,
                                int n, int m, int* __restrict__ tail, int* __restrict__ head, long long* __restrict__ bad,
                                long long* __restrict__ single) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a = rp[i];
  const int len = rp[i + 1] - a;
  if (len == 1) {
    const int c0 = col[a];
    const double v0 = val[a];
    if (c0 < 0 || c0 >= m || (v0 != 1.0 && v0 != -1.0)) { atomicAdd((unsigned long long*)bad, 1ULL); return; }
    tail[i] = v0 < 0.0 ? c0 : -1;
    head[i] = v0 < 0.0 ? -1 : c0;
    atomicAdd((unsigned long long*)single, 1ULL);
    return;
  }
  if (len != 2) { atomicAdd((unsigned long long*)bad, 1ULL); return; }
  const int c0 = col[a], c1 = col[a + 1];
  const double v0 = val[a], v1 = val[a + 1];
  if (c0 < 0 || c1 < 0 || c0 >= m || c1 >= m || c0 == c1) { atomicAdd((unsigned long long*)bad, 1ULL); return; }
  if (v0 == -1.0 && v1 == 1.0) { tail[i] = c0; head[i] = c1; }
  else if (v0 == 1.0 && v1 == -1.0) { tail[i] = c1; head[i] = c0; }
  else atomicAdd((unsigned long long*)bad, 1ULL);
}

// D as CSR with sorted columns from the endpoint arrays (an absent end, -1,
// gives no entry).
__global__ void k_grad_count(const int* __restrict__ tail, const int* __restrict__ head, int n, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cnt[i] = (tail[i] >= 0) + (head[i] >= 0);
}
__global__ void k_grad_csr(const int* __restrict__ tail, const int* __restrict__ head, int n, const int* __restrict__ rp,
                           int* __restrict__ col, double* __restrict__ val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = tail[i], h = head[i], o = rp[i];
  if (t < 0) { col[o] = h; val[o] = 1.0; return; }
  if (h < 0) { col[o] = t; val[o] = -1.0; return; }
  if (t < h) { col[o] = t; col[o + 1] = h; val[o] = -1.0; val[o + 1] = 1.0; }
  else { col[o] = h; col[o + 1] = t; val[o] = 1.0; val[o + 1] = -1.0; }
}

static void gradient_csr(Level& L, Ctx& c) {
  L.D.nrows = L.n; L.D.ncols = L.m;
  L.D.rowptr.alloc(L.n + 1, c.s);
  DBuf<int> cnt(L.n + 1, c.s);
  k_grad_count<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, L.n, cnt.p);
  HC_LAUNCH_CHECK();
  L.D.nnz = exclusive_scan(cnt.p, L.D.rowptr.p, L.n, c);
  L.D.col.alloc(std::max<int64_t>(L.D.nnz, 1), c.s);
  L.D.val.alloc(std::max<int64_t>(L.D.nnz, 1), c.s);
  c.run("grad_csr", 24.0 * L.n, [&] {
    k_grad_csr<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, L.n, L.D.rowptr.p, L.D.col.p, L.D.val.p);
  });
  transpose(L.D, L.DT, true, c);
}

// Diagonal must be positive and finite.
__global__ void k_check_diag(const double* __restrict__ dinv, int n, long long* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = dinv[i];
  if (!(v > 0.0) || !isfinite(v)) atomicAdd((unsigned long long*)bad, 1ULL);
}

static long long read_flag(int slot, Ctx& c) {
  long long h = 0;
  d2h(&h, c.iscal.p + slot, 1, c);
  return h;
}
static void clear_flag(int slot, Ctx& c) { HC_HIP(hipMemsetAsync(c.iscal.p + slot, 0, sizeof(long long), c.s)); }

// ---------------------------------------------------------------------------
// smoothed aggregation
// ---------------------------------------------------------------------------
__global__ void k_hash_unit(double* __restrict__ x, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (double)(splitmix64((uint64_t)i) >> 11) * 0x1.0p-53;
}
__global__ void k_mul(double* __restrict__ y, const double* __restrict__ d, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] *= d[i];
}
// rho = ||y|| / ||x||, x = y / ||y||
__global__ void k_power_normalise(double* __restrict__ x, const double* __restrict__ y, int n, const double* __restrict__ nx2,
                                  const double* __restrict__ ny2, double* __restrict__ rho) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double ny = sqrt(*ny2);
  if (i == 0) *rho = ny / sqrt(*nx2);
  if (i < n) x[i] = y[i] / ny;
}
__global__ void k_omega(const double* __restrict__ rho, double* __restrict__ omega) { *omega = 4.0 / (3.0 * *rho); }

__global__ void k_pbar(const int* __restrict__ agg, int m, int* __restrict__ rp, int* __restrict__ col,
                       double* __restrict__ val) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > m) return;
  rp[i] = i;
  if (i < m) { col[i] = agg[i]; val[i] = 1.0; }
}

// P^(n) = P-bar - omega D^-1 A^(n) P-bar on the pattern of A^(n) P-bar, rows
// then scaled to sum 1.  On entry val holds (A^(n) P-bar).
__global__ void k_sa_values(const int* __restrict__ rp, const int* __restrict__ col, double* __restrict__ val,
                            const int* __restrict__ agg, const double* __restrict__ dinv, const double* __restrict__ omega,
                            int m) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m) return;
  const double w = *omega * dinv[u];
  const int a = agg[u];
  double s = 0.0;
  for (int q = rp[u]; q < rp[u + 1]; ++q) {
    const double v = (col[q] == a ? 1.0 : 0.0) - w * val[q];
    val[q] = v;
    s += v;
  }
  const double inv = 1.0 / s;
  for (int q = rp[u]; q < rp[u + 1]; ++q) val[q] *= inv;
}

// ---------------------------------------------------------------------------
// caller-given P^(n): rows scaled to sum one, aggregates by Alg. 1
// ---------------------------------------------------------------------------
// Row sums in index order, one term at a time; every value divided by its
// row's sum.  Empty rows, zero or non-finite sums and non-finite values are
// flagged.
__global__ void k_scale_rows(const int* __restrict__ rp, double* __restrict__ val, int m, long long* __restrict__ bad) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m) return;
  double s = 0.0;
  bool fin = true;
  for (int q = rp[u]; q < rp[u + 1]; ++q) {
    s += val[q];
    fin = fin && isfinite(val[q]);
  }
  if (!(s != 0.0) || !isfinite(s) || !fin) { atomicAdd((unsigned long long*)bad, 1ULL); return; }
  for (int q = rp[u]; q < rp[u + 1]; ++q) val[q] = val[q] / s;
}

// Order key of |p|: the bit pattern of a non-negative finite double orders
// like its value; +1 keeps 0 free for "no proposal".
__device__ __forceinline__ unsigned long long mag_key(double v) {
  return (unsigned long long)__double_as_longlong(fabs(v)) + 1ULL;
}

// Alg. 1 passes in the order of the algorithm: one workgroup walks the
// columns (rows of P^(n)T, fine nodes increasing) in order; for each column
// its unassigned rows are gathered in LDS and those ranking below the
// column's quota (larger |p| first, then smaller fine node) are assigned to
// it before the next column starts.  Columns hold at most kAlg1Cap entries
// (checked on the host).
constexpr int kAlg1Cap = 4096;
__global__ void __launch_bounds__(1024) k_alg1_passes(const int* __restrict__ tp, const int* __restrict__ trow,
                                                      const double* __restrict__ tval, int mH, int64_t mh, int64_t nnz,
                                                      int passes, int* __restrict__ assign) {
  __shared__ unsigned long long sk[kAlg1Cap];
  __shared__ int sr[kAlg1Cap];
  __shared__ int nfree;
  for (int pass = 0; pass < passes; ++pass) {
    for (int j = 0; j < mH; ++j) {
      const int a = tp[j], b = tp[j + 1];
      const int64_t target = ((int64_t)(b - a) * mh + nnz - 1) / nnz;
      const int64_t quota = (target + passes - 1) / passes;
      if (threadIdx.x == 0) nfree = 0;
      __syncthreads();
      for (int e = a + (int)threadIdx.x; e < b; e += blockDim.x) {
        const int r = trow[e];
        if (assign[r] < 0) {
          const int s = atomicAdd(&nfree, 1);
          sk[s] = mag_key(tval[e]);
          sr[s] = r;
        }
      }
      __syncthreads();
      const int nf = nfree;
      for (int s = threadIdx.x; s < nf; s += blockDim.x) {
        const unsigned long long k = sk[s];
        const int r = sr[s];
        int64_t better = 0;
        for (int t = 0; t < nf && better < quota; ++t) better += (sk[t] > k) || (sk[t] == k && sr[t] < r);
        if (better < quota) assign[r] = j;
      }
      __syncthreads();
    }
  }
}

__global__ void k_alg1_count(const int* __restrict__ assign, int m, int* __restrict__ cnt) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < m) atomicAdd(&cnt[assign[u]], 1);
}

// Safeguard for empty columns, in column order: the column takes its row of
// largest |p| (ties: smaller fine node) among rows whose column keeps another
// row; a column with no such row is flagged.  Moves never empty a column, so
// the empty set is known before the walk; only the order matters.
__global__ void __launch_bounds__(1024) k_alg1_safeguard(const int* __restrict__ tp, const int* __restrict__ trow,
                                                         const double* __restrict__ tval, int mH,
                                                         int* __restrict__ assign, int* __restrict__ cnt,
                                                         long long* __restrict__ bad) {
  __shared__ unsigned char empty[1024];
  __shared__ unsigned long long bk;
  __shared__ int br;
  for (int c0 = 0; c0 < mH; c0 += 1024) {
    const int jt = c0 + (int)threadIdx.x;
    empty[threadIdx.x] = jt < mH && cnt[jt] == 0;
    __syncthreads();
    const int nt = min(1024, mH - c0);
    for (int t = 0; t < nt; ++t) {
      if (!empty[t]) continue;  // uniform across the workgroup
      const int j = c0 + t;
      if (threadIdx.x == 0) { bk = 0ULL; br = 0x7fffffff; }
      __syncthreads();
      for (int e = tp[j] + (int)threadIdx.x; e < tp[j + 1]; e += blockDim.x)
        if (cnt[assign[trow[e]]] >= 2) atomicMax(&bk, mag_key(tval[e]));
      __syncthreads();
      for (int e = tp[j] + (int)threadIdx.x; e < tp[j + 1]; e += blockDim.x)
        if (cnt[assign[trow[e]]] >= 2 && mag_key(tval[e]) == bk) atomicMin(&br, trow[e]);
      __syncthreads();
      if (threadIdx.x == 0) {
        if (bk == 0ULL) {
          atomicAdd((unsigned long long*)bad, 1ULL);
        } else {
          cnt[assign[br]] -= 1;
          assign[br] = j;
          cnt[j] += 1;
        }
      }
      __syncthreads();
    }
    __syncthreads();
  }
}

// Fine nodes no pass assigned: the coarse node of the row's largest |p|
// (columns increase along the row, so the first maximum is the smallest).
__global__ void k_alg1_leftover(const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ val,
                                int m, int* __restrict__ assign) {
  int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= m || assign[u] >= 0) return;
  unsigned long long bk = 0ULL;
  int bc = -1;
  for (int q = rp[u]; q < rp[u + 1]; ++q) {
    const unsigned long long k = mag_key(val[q]);
    if (k > bk) { bk = k; bc = col[q]; }
  }
  assign[u] = bc;
}

// ---------------------------------------------------------------------------
// coarse gradient by the RS rule on P-bar
// ---------------------------------------------------------------------------
__global__ void k_cross_count(const int* __restrict__ tail, const int* __restrict__ head, const int* __restrict__ agg,
                              int n, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = tail[i], h = head[i];
  cnt[i] = (t >= 0 && h >= 0 && agg[t] != agg[h]) ? 2 : 0;
}
__global__ void k_cross_fill(const int* __restrict__ tail, const int* __restrict__ head, const int* __restrict__ agg,
                             int n, const int* __restrict__ rp, int* __restrict__ col) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = tail[i], h = head[i];
  if (t < 0 || h < 0) return;
  const int I = agg[t], K = agg[h];
  if (I == K) return;
  col[rp[i]] = min(I, K);
  col[rp[i] + 1] = max(I, K);
}
// Dirichlet edges: the coarse node their remaining node belongs to gets one
// single-node coarse edge (Sec. 2)
__global__ void k_single_mark(const int* __restrict__ tail, const int* __restrict__ head, const int* __restrict__ agg,
                              int n, int* __restrict__ mark) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t = tail[i], h = head[i];
  if (t < 0 && h >= 0) mark[agg[h]] = 1;
  else if (h < 0 && t >= 0) mark[agg[t]] = 1;
}
// sne[I] = id of node I's single-node coarse edge (after the nTwo two-node
// edges, in node order) or -1; also writes the edges' ends
__global__ void k_single_ids(int mH, const int* __restrict__ mark, const int* __restrict__ pos, int nTwo,
                             int* __restrict__ sne, int* __restrict__ ctail, int* __restrict__ chead) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= mH) return;
  if (!mark[I]) { sne[I] = -1; return; }
  const int e = nTwo + pos[I];
  sne[I] = e;
  if (ctail) { ctail[e] = -1; chead[e] = I; }
}
__global__ void k_upper_count(const int* __restrict__ rp, const int* __restrict__ col, int n, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int c = 0;
  for (int q = rp[i]; q < rp[i + 1]; ++q) c += col[q] > i;
  cnt[i] = c;
}
__global__ void k_upper_fill(const int* __restrict__ rp, const int* __restrict__ col, int n, const int* __restrict__ up,
                             int* __restrict__ ctail, int* __restrict__ chead) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int o = up[i];
  for (int q = rp[i]; q < rp[i + 1]; ++q)
    if (col[q] > i) { ctail[o] = i; chead[o] = col[q]; ++o; }
}

// ---------------------------------------------------------------------------
// pattern N of P^(e) (Alg. 2): for fine edge i, the coarse edges whose two end
// points both lie in T_i (B_ij = 2 with W = 1 for two-node coarse edges).
// Coarse edges are ordered by (tail, head), so walking T_i in increasing order
// and each node's outgoing edges yields sorted columns.
// ---------------------------------------------------------------------------
static constexpr int kMaxJ = 32;

template <bool FILL>
__global__ void k_pattern(int n, const int* __restrict__ Trp, const int* __restrict__ Tcol, const int* __restrict__ tptr,
                          const int* __restrict__ chead, const int* __restrict__ sne, int* __restrict__ cnt,
                          const int* __restrict__ Nrp, int* __restrict__ Ncol, uint16_t* __restrict__ lpair,
                          long long* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int t0 = Trp[i];
  const int nJ = Trp[i + 1] - t0;
  if (nJ > kMaxJ) { atomicAdd((unsigned long long*)&flags[F_TOOBIG], 1ULL); if (!FILL) cnt[i] = 0; return; }
  unsigned adj[kMaxJ];
  for (int a = 0; a < nJ; ++a) adj[a] = 0u;
  int c = 0;
  const int o = FILL ? Nrp[i] : 0;
  for (int a = 0; a < nJ; ++a) {
    const int I = Tcol[t0 + a];
    for (int e = tptr[I]; e < tptr[I + 1]; ++e) {
      const int K = chead[e];
      int lo = a + 1, hi = nJ - 1, b = -1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = Tcol[t0 + mid];
        if (v == K) { b = mid; break; }
        if (v < K) lo = mid + 1; else hi = mid - 1;
      }
      if (b >= 0) {
        if (FILL) {
          Ncol[o + c] = e;
          lpair[o + c] = (uint16_t)(a | (b << 8));
        }
        adj[a] |= 1u << b;
        adj[b] |= 1u << a;
        ++c;
      }
    }
  }
  // single-node coarse edges of T_i's nodes (W = 2 in Alg. 2); their ids
  // follow every two-node id and increase with the node
  if (sne)
    for (int a = 0; a < nJ; ++a) {
      const int e = sne[Tcol[t0 + a]];
      if (e < 0) continue;
      if (FILL) {
        Ncol[o + c] = e;
        lpair[o + c] = (uint16_t)(255 | (a << 8));
      }
      ++c;
    }
  if (!FILL) {
    cnt[i] = c;
    atomicMax((unsigned long long*)&flags[F_MAXJ], (unsigned long long)nJ);
    atomicMax((unsigned long long*)&flags[F_MAXNP], (unsigned long long)c);
    if (nJ >= 2) {
      unsigned reach = 1u, prev = 0u;
      while (reach != prev) {
        prev = reach;
        for (int a = 0; a < nJ; ++a)
          if (reach >> a & 1u) reach |= adj[a];
      }
      const unsigned all = nJ == 32 ? 0xffffffffu : ((1u << nJ) - 1u);
      if (reach != all) atomicAdd((unsigned long long*)&flags[F_DISCONNECTED], 1ULL);
    }
  }
}

// ---------------------------------------------------------------------------
// make_irreducible (Alg. 2; reading R15).  For every fine edge whose local
// graph is disconnected: the component of the row's smallest coarse node is
// joined to the rest by the pair (I, K), I inside, K outside, of largest
// |(P^(n)T D^T D P^(n))_IK| (ties: smallest (min, max) pair).  The new coarse
// edges are merged into the lexicographic edge order, and the pattern is
// rebuilt until every row is connected.
// ---------------------------------------------------------------------------
__global__ void k_irreducible_pick(int n, const int* __restrict__ Trp, const int* __restrict__ Tcol,
                                   const int* __restrict__ tptr, const int* __restrict__ chead,
                                   const int* __restrict__ Zrp, const int* __restrict__ Zcol,
                                   const double* __restrict__ Zval, unsigned long long* __restrict__ cand) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  cand[i] = ~0ULL;
  const int t0 = Trp[i];
  const int nJ = Trp[i + 1] - t0;
  if (nJ < 2 || nJ > kMaxJ) return;
  unsigned adj[kMaxJ];
  for (int a = 0; a < nJ; ++a) adj[a] = 0u;
  for (int a = 0; a < nJ; ++a) {
    const int I = Tcol[t0 + a];
    for (int e = tptr[I]; e < tptr[I + 1]; ++e) {
      const int K = chead[e];
      int lo = a + 1, hi = nJ - 1;
      while (lo <= hi) {
        const int mid = (lo + hi) >> 1;
        const int v = Tcol[t0 + mid];
        if (v == K) { adj[a] |= 1u << mid; adj[mid] |= 1u << a; break; }
        if (v < K) lo = mid + 1; else hi = mid - 1;
      }
    }
  }
  unsigned reach = 1u, prev = 0u;
  while (reach != prev) {
    prev = reach;
    for (int a = 0; a < nJ; ++a)
      if (reach >> a & 1u) reach |= adj[a];
  }
  const unsigned all = nJ == 32 ? 0xffffffffu : ((1u << nJ) - 1u);
  if (reach == all) return;
  double bw = -1.0;
  int blo = 0, bhi = 0;
  for (int p = 0; p < nJ; ++p) {
    if (!(reach >> p & 1u)) continue;
    for (int q = 0; q < nJ; ++q) {
      if (reach >> q & 1u) continue;
      const int I = Tcol[t0 + p], K = Tcol[t0 + q];
      const int lo = I < K ? I : K, hi = I < K ? K : I;
      double w = 0.0;
      int l = Zrp[lo], h = Zrp[lo + 1] - 1;
      while (l <= h) {
        const int mid = (l + h) >> 1;
        const int v = Zcol[mid];
        if (v == hi) { w = fabs(Zval[mid]); break; }
        if (v < hi) l = mid + 1; else h = mid - 1;
      }
      const bool better = w > bw || (w == bw && (lo < blo || (lo == blo && hi < bhi)));
      if (better) { bw = w; blo = lo; bhi = hi; }
    }
  }
  cand[i] = ((unsigned long long)(unsigned)blo << 32) | (unsigned)bhi;
}
__global__ void k_cand_count(int n, const unsigned long long* __restrict__ cand, int* __restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && cand[i] != ~0ULL) atomicAdd(&cnt[(int)(cand[i] >> 32)], 1);
}
__global__ void k_cand_fill(int n, const unsigned long long* __restrict__ cand, int* __restrict__ cursor,
                            int* __restrict__ xcol) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && cand[i] != ~0ULL) xcol[atomicAdd(&cursor[(int)(cand[i] >> 32)], 1)] = (int)(cand[i] & 0xffffffffu);
}
// Per coarse node I: the union of its present upper neighbours (sorted) and
// the new ones (sorted here, duplicates dropped); FILL writes the merged edges.
template <bool FILL>
__global__ void k_edge_union(int mH, const int* __restrict__ tptr, const int* __restrict__ chead,
                             const int* __restrict__ xptr, int* __restrict__ xcol, int* __restrict__ cnt,
                             const int* __restrict__ nptr, int* __restrict__ ntail, int* __restrict__ nhead) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= mH) return;
  const int xa = xptr[I], xb = xptr[I + 1];
  if (!FILL)
    for (int q = xa + 1; q < xb; ++q) {
      const int key = xcol[q];
      int r = q - 1;
      while (r >= xa && xcol[r] > key) { xcol[r + 1] = xcol[r]; --r; }
      xcol[r + 1] = key;
    }
  int a = tptr[I];
  const int b = tptr[I + 1];
  int x = xa, c = 0, last = -1;
  const int o = FILL ? nptr[I] : 0;
  while (a < b || x < xb) {
    int v;
    if (x >= xb || (a < b && chead[a] <= xcol[x])) v = chead[a++];
    else v = xcol[x++];
    if (v == last) continue;
    last = v;
    if (FILL) { ntail[o + c] = I; nhead[o + c] = v; }
    ++c;
  }
  if (!FILL) cnt[I] = c;
}

// ---------------------------------------------------------------------------
// local constraint systems (Sec. 4.2).  For row i with coarse nodes T_i
// (|J| = nJ) and pattern entries e = (local tail t_e, local head h_e), the
// transposed sub-matrix G~ keeps all nodes but the last (largest id); its
// normal matrix L~ = G~^T G~ is the reduced graph Laplacian of the local
// graph, SPD when the graph is connected (k = nJ - 1 unknowns).
//   project:     x <- x - G~ L~^-1 G~^T x
//   affine:      x <- x + G~ L~^-1 (r~ - G~^T x)
// ---------------------------------------------------------------------------
template <int MAXJ>
__device__ __forceinline__ bool local_solve(double* x, const uint16_t* __restrict__ lp, int np, int nJ,
                                            const double* __restrict__ rrow) {
  constexpr int MK = MAXJ - 1;
  constexpr int NL = MK * (MK + 1) / 2;
  // a Dirichlet (single-node) coarse edge, marked by the local index 255 at
  // its absent end, makes G~ full rank: no column is dropped (Alg. 2)
  int miss = 0;
  for (int e = 0; e < np; ++e) miss |= ((lp[e] & 255) == 255) | ((lp[e] >> 8) == 255);
  const int k = nJ - 1 + miss;
  if (k <= 0 || np == 0) return true;
  double L[NL];
  double y[MK];
#pragma unroll
  for (int a = 0; a < NL; ++a) L[a] = 0.0;
#pragma unroll
  for (int a = 0; a < MK; ++a) y[a] = 0.0;
  for (int e = 0; e < np; ++e) {
    const int t = lp[e] & 255, h = lp[e] >> 8;
    const double xe = x[e];
    const int hi = t > h ? t : h, lo = t > h ? h : t;
#pragma unroll
    for (int a = 0; a < MK; ++a) {
      if (a == t) { L[a * (a + 1) / 2 + a] += 1.0; y[a] -= xe; }
      if (a == h) { L[a * (a + 1) / 2 + a] += 1.0; y[a] += xe; }
#pragma unroll
      for (int b = 0; b < a; ++b)
        if (a == hi && b == lo) L[a * (a + 1) / 2 + b] -= 1.0;
    }
  }
  if (rrow) {
#pragma unroll
    for (int a = 0; a < MK; ++a)
      if (a < k) y[a] = rrow[a] - y[a];
  }
  bool ok = true;
  // Cholesky, packed lower triangle
#pragma unroll
  for (int i = 0; i < MK; ++i) {
    if (i < k) {
#pragma unroll
      for (int j = 0; j <= i; ++j) {
        double s = L[i * (i + 1) / 2 + j];
#pragma unroll
        for (int q = 0; q < j; ++q) s -= L[i * (i + 1) / 2 + q] * L[j * (j + 1) / 2 + q];
        if (i == j) {
          ok = ok && (s > 0.0);
          L[i * (i + 1) / 2 + i] = sqrt(s);
        } else {
          L[i * (i + 1) / 2 + j] = s / L[j * (j + 1) / 2 + j];
        }
      }
    }
  }
  // forward L w = y, backward L^T z = w (in y)
#pragma unroll
  for (int i = 0; i < MK; ++i) {
    if (i < k) {
      double s = y[i];
#pragma unroll
      for (int q = 0; q < i; ++q) s -= L[i * (i + 1) / 2 + q] * y[q];
      y[i] = s / L[i * (i + 1) / 2 + i];
    }
  }
#pragma unroll
  for (int i = MK - 1; i >= 0; --i) {
    if (i < k) {
      double s = y[i];
#pragma unroll
      for (int q = i + 1; q < MK; ++q)
        if (q < k) s -= L[q * (q + 1) / 2 + i] * y[q];
      y[i] = s / L[i * (i + 1) / 2 + i];
    }
  }
#pragma unroll
  for (int a = 0; a < MK; ++a)
    if (a >= k) y[a] = 0.0;
  for (int e = 0; e < np; ++e) {
    const int t = lp[e] & 255, h = lp[e] >> 8;
    double zt = 0.0, zh = 0.0;
#pragma unroll
    for (int a = 0; a < MK; ++a) {
      if (a == t) zt = y[a];
      if (a == h) zh = y[a];
    }
    const double dz = zh - zt;
    x[e] = rrow ? x[e] + dz : x[e] - dz;
  }
  return ok;
}

// Runs each row in the smallest register layout that holds it: the unknowns
// a >= k never enter the arithmetic, so a row with k unknowns gives the same
// bits in every layout with MAXJ - 1 >= k, and a level whose largest rows need
// a wide layout does not make every row pay for it.
template <int MAXJ>
__device__ __forceinline__ bool local_solve_fit(double* x, const uint16_t* __restrict__ lp, int np, int nJ,
                                                const double* __restrict__ rrow) {
  if constexpr (MAXJ > 8) {
    int miss = 0;
    for (int e = 0; e < np; ++e) miss |= ((lp[e] & 255) == 255) | ((lp[e] >> 8) == 255);
    const int k = nJ - 1 + miss;
    if (k <= 7) return local_solve<8>(x, lp, np, nJ, rrow);
    if constexpr (MAXJ > 16) {
      if (k <= 15) return local_solve<16>(x, lp, np, nJ, rrow);
    }
  }
  return local_solve<MAXJ>(x, lp, np, nJ, rrow);
}

// Affine step on every row: x <- x + G~ L~^-1 (r~ - G~^T x).  With `ones` the
// row is first set to ones (the plain initial guess of Sec. 6.1).
template <int MAXJ>
__global__ void k_make_feasible(int n, const int* __restrict__ Prp, double* __restrict__ x, const uint16_t* __restrict__ lp,
                                const int* __restrict__ Trp, const double* __restrict__ Rval, int ones,
                                long long* __restrict__ flags) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = Prp[i], np = Prp[i + 1] - p0;
  if (ones)
    for (int e = 0; e < np; ++e) x[p0 + e] = 1.0;
  const int t0 = Trp[i], nJ = Trp[i + 1] - t0;
  // Solvability (Sec. 4.2): the columns of G_i = [D_H]_{N_i,T_i} sum to zero
  // when no coarse edge of the row has a single node, so G_i^T p = r_i needs
  // sum_k r_ik = 0.  With rows of P^(n) summing to one, sum_k r_ik is the
  // difference of two such sums, zero up to their rounding; the bound is
  // absolute (r_i itself may be zero up to rounding) unless r_i is larger
  // than one.  With a single-node edge G_i has full column rank.  Either way
  // r_i must be finite.
  int miss = 0;
  for (int e = 0; e < np; ++e) miss |= ((lp[p0 + e] & 255) == 255) | ((lp[p0 + e] >> 8) == 255);
  double rs = 0.0, ra = 0.0;
  for (int k = 0; k < nJ; ++k) {
    rs += Rval[t0 + k];
    ra += fabs(Rval[t0 + k]);
  }
  if (!(ra <= DBL_MAX) || (!miss && !(fabs(rs) <= 1e-10 * fmax(1.0, ra)))) {
    atomicAdd((unsigned long long*)&flags[F_INFEASIBLE], 1ULL);
    atomicMax((unsigned long long*)&flags[F_INFEASIBLE_ROW], (unsigned long long)i + 1);
    return;
  }
  if (!local_solve_fit<MAXJ>(x + p0, lp + p0, np, nJ, Rval + t0)) atomicAdd((unsigned long long*)&flags[F_NOTSPD], 1ULL);
}

// ---------------------------------------------------------------------------
// masked SpGEMM on P's pattern:  Y = dscale * mask_N(A X)
// One 64-lane workgroup takes a block of R consecutive rows.  The products of
// the block are flattened over the lanes (prefix sum of the pattern lengths
// of the A-columns of each chunk of 64 A entries); each product finds its
// owner (the chunk's A entry) and its slot in the owner row's pattern (binary
// searches in LDS) and accumulates there with an LDS atomic.  Two products
// per lane are in flight at a time (kMapBatch when reading codes back).  With
// EM_DOT the block also sums X * Y (the energy <P, A P>).
//
// The pattern stays fixed over the iterations of an energy minimisation, so
// the first launch can record both searches per product (MAP = 1) and the
// later ones read them back (MAP = 2): a 16-bit code per product, in the
// kernel's enumeration order, block after block (offsets from
// k_emin_map_count and k_emin_map_offsets); bits 0-5 hold the owner lane and
// bits 6-15 the slot among the row block's pattern entries (fewer than
// kPatCap), kNoSlot marks a product whose column is not in the owner row's
// pattern.
// ---------------------------------------------------------------------------
static constexpr int kPatCap = 512;
static constexpr int kRowsCap = 64;
enum { EM_PROJECT = 1, EM_NEGATE = 2, EM_DOT = 4 };

struct RowBlocks {
  // contiguous row-block ranges per XCD (workgroup b runs on XCD b % 8)
  int nbr, chunk, xcd, wi, nw;
  __device__ RowBlocks(int nrows, int R) {
    nbr = (nrows + R - 1) / R;
    nw = gridDim.x / 8;
    xcd = blockIdx.x % 8;
    wi = blockIdx.x / 8;
    chunk = (nbr + 7) / 8;
  }
  __device__ int first() const { return xcd * chunk + wi; }
  __device__ int end() const { return min(nbr, (xcd + 1) * chunk); }
};

// code of a product whose column is not in its owner row's pattern (owner
// lane 63 with slot 1023, which no row block reaches: slots stay below kPatCap)
static constexpr unsigned kNoSlot = 0xFFFFu;

template <bool BUILD>
__device__ __forceinline__ void emin_product(int p, const int* pre, const int* kst, const int* arow, const double* av,
                                             const int* pofs, const int* pcol, double* acc, const int* __restrict__ Pcol,
                                             const double* __restrict__ X, uint16_t* __restrict__ mp) {
  int lo = 0, hi = 63;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (pre[mid] <= p) lo = mid; else hi = mid - 1;
  }
  const int pos = kst[lo] + (p - pre[lo]);
  const int key = Pcol[pos];
  const double v = av[lo] * X[pos];
  const int rr = arow[lo];
  int s = pofs[rr], e = pofs[rr + 1] - 1;
  while (s < e) {
    const int mid = (s + e) >> 1;
    if (pcol[mid] < key) s = mid + 1; else e = mid;
  }
  const bool hit = s <= e && pcol[s] == key;
  if (hit) atomicAdd(&acc[s], v);
  if (BUILD) mp[p] = hit ? (uint16_t)(lo | (s << 6)) : (uint16_t)kNoSlot;
}

// products per lane in flight in the read-back launches: four keep eight
// waves per SIMD; eight need more registers and ran slower
static constexpr int kMapBatch = 4;

// Products per workgroup of k_emin_masked (same grid, same row blocks): the
// pattern lengths of the A-columns of every A entry of its row blocks.
__global__ void __launch_bounds__(64) k_emin_map_count(int nrows, int R, const int* __restrict__ Arp,
                                                       const int* __restrict__ Acol, const int* __restrict__ Prp,
                                                       long long* __restrict__ cnt) {
  const int l = threadIdx.x;
  const RowBlocks B(nrows, R);
  long long t = 0;
  for (int rb = B.first(); rb < B.end(); rb += B.nw) {
    const int r0 = rb * R, r1 = min(r0 + R, nrows);
    for (int q = Arp[r0] + l; q < Arp[r1]; q += 64) {
      const int k = Acol[q];
      t += Prp[k + 1] - Prp[k];
    }
  }
  t = wave_sum(t);
  if (l == 0) cnt[blockIdx.x] = t;
}

// Exclusive prefix sum of the per-workgroup counts (one 1024-thread
// workgroup, n <= 8192); off[n] receives the total.
__global__ void __launch_bounds__(1024) k_emin_map_offsets(const long long* __restrict__ cnt, int n,
                                                           long long* __restrict__ off) {
  __shared__ long long sh[1024];
  const int t = threadIdx.x, per = (n + 1023) / 1024, b0 = t * per;
  long long s = 0;
  for (int i = b0; i < min(n, b0 + per); ++i) s += cnt[i];
  sh[t] = s;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const long long v = t >= o ? sh[t - o] : 0;
    __syncthreads();
    sh[t] += v;
    __syncthreads();
  }
  long long run = sh[t] - s;
  for (int i = b0; i < min(n, b0 + per); ++i) {
    off[i] = run;
    run += cnt[i];
  }
  if (t == 1023) off[n] = sh[t];
}

template <int CAP, int MAP>
__global__ void __launch_bounds__(64) k_emin_masked(int nrows, int R, const int* __restrict__ Arp,
                                                    const int* __restrict__ Acol, const double* __restrict__ Aval,
                                                    const double* __restrict__ dscale, const int* __restrict__ Prp,
                                                    const int* __restrict__ Pcol, const double* __restrict__ X,
                                                    double* __restrict__ Y, int flags, double* __restrict__ part,
                                                    uint16_t* __restrict__ pmap, const long long* __restrict__ moff,
                                                    int2* __restrict__ asl) {
  static_assert(MAP == 0 || MAP == 1, "the read-back launches use k_emin_masked_codes");
  __shared__ int pcol[CAP];
  __shared__ double acc[CAP];
  __shared__ int pofs[kRowsCap + 1];
  __shared__ int arp[kRowsCap + 1];
  __shared__ int kst[64], pre[64], arow[64];
  __shared__ double av[64];
  const int l = threadIdx.x;
  const RowBlocks B(nrows, R);
  long long mb = MAP ? moff[blockIdx.x] : 0;
  double dsum = 0.0;
  for (int rb = B.first(); rb < B.end(); rb += B.nw) {
    const int r0 = rb * R, r1 = min(r0 + R, nrows), nr = r1 - r0;
    const int p0 = Prp[r0], pn = Prp[r1] - p0;
    for (int t = l; t < pn; t += 64) {
      pcol[t] = Pcol[p0 + t];
      acc[t] = 0.0;
    }
    for (int t = l; t <= nr; t += 64) { pofs[t] = Prp[r0 + t] - p0; arp[t] = Arp[r0 + t]; }
    __syncthreads();
    const int a0 = arp[0], a1 = arp[nr];
    for (int c0 = a0; c0 < a1; c0 += 64) {
      const int q = c0 + l;
      int st = 0, len = 0, rl = 0;
      double a = 0.0;
      if (q < a1) {
        // the owner row of A entry q, for the slot search (a row with an
        // empty pattern gets no hits)
        int lo = 0, hi = nr - 1;
        while (lo < hi) {  // largest rl with arp[rl] <= q
          const int mid = (lo + hi + 1) >> 1;
          if (arp[mid] <= q) lo = mid; else hi = mid - 1;
        }
        rl = lo;
        const int k = Acol[q];
        a = Aval[q];
        st = Prp[k];
        len = Prp[k + 1] - st;
        if (MAP == 1) asl[q] = make_int2(st, len);
      }
      const int incl = wave_incl_scan(len);
      const int total = __shfl(incl, 63, 64);
      kst[l] = st; pre[l] = incl - len; arow[l] = rl; av[l] = a;
      __syncthreads();
      int p = l;
      uint16_t* mp = MAP ? pmap + mb : nullptr;
      for (; p + 64 < total; p += 128) {
        emin_product<MAP == 1>(p, pre, kst, arow, av, pofs, pcol, acc, Pcol, X, mp);
        emin_product<MAP == 1>(p + 64, pre, kst, arow, av, pofs, pcol, acc, Pcol, X, mp);
      }
      if (p < total) emin_product<MAP == 1>(p, pre, kst, arow, av, pofs, pcol, acc, Pcol, X, mp);
      mb += total;
      __syncthreads();
    }
    for (int t = l; t < pn; t += 64) {
      double v = acc[t];
      if (dscale) {
        int lo = 0, hi = nr - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pofs[mid] <= t) lo = mid; else hi = mid - 1;
        }
        v *= dscale[r0 + lo];
      }
      Y[p0 + t] = v;
      if (flags & EM_DOT) dsum += X[p0 + t] * v;
    }
    __syncthreads();
  }
  dsum = wave_sum(dsum);
  if (l == 0) part[blockIdx.x] = dsum;
}

// LDS-only barrier for single-wave workgroups: waits for this wave's LDS
// operations, not its global loads, so loads issued before it stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The read-back launches of the masked product (codes recorded by
// k_emin_masked<CAP, 1>, which also stored every A entry's pattern start and
// length of its column in asl).  The same products, in the same order, go to
// the same LDS sums; the next chunk's A entries are loaded while the current
// chunk's products run.
template <int CAP>
__global__ void __launch_bounds__(64) k_emin_masked_codes(int nrows, int R, const int* __restrict__ Arp,
                                                          const double* __restrict__ Aval, const int2* __restrict__ asl,
                                                          const double* __restrict__ dscale, const int* __restrict__ Prp,
                                                          const double* __restrict__ X, double* __restrict__ Y, int flags,
                                                          double* __restrict__ part, const uint16_t* __restrict__ codes,
                                                          const long long* __restrict__ moff) {
  __shared__ double acc[CAP];
  __shared__ int pofs[kRowsCap + 1];
  __shared__ int kst[64], pre[64];
  __shared__ double av[64];
  const int l = threadIdx.x;
  const RowBlocks B(nrows, R);
  long long mb = moff[blockIdx.x];
  double dsum = 0.0;
  for (int rb = B.first(); rb < B.end(); rb += B.nw) {
    const int r0 = rb * R, r1 = min(r0 + R, nrows), nr = r1 - r0;
    const int p0 = Prp[r0], pn = Prp[r1] - p0;
    const int a0 = Arp[r0], a1 = Arp[r1];
    int2 nsl = make_int2(0, 0);
    double na = 0.0;
    if (a0 + l < a1) { nsl = asl[a0 + l]; na = Aval[a0 + l]; }
    for (int t = l; t < pn; t += 64) acc[t] = 0.0;
    for (int t = l; t <= nr; t += 64) pofs[t] = Prp[r0 + t] - p0;
    lds_barrier();
    for (int c0 = a0; c0 < a1; c0 += 64) {
      const int st = nsl.x, len = nsl.y;
      const double a = na;
      nsl = make_int2(0, 0);
      na = 0.0;
      if (c0 + 64 + l < a1) { nsl = asl[c0 + 64 + l]; na = Aval[c0 + 64 + l]; }
      const int incl = wave_incl_scan(len);
      const int total = __shfl(incl, 63, 64);
      kst[l] = st; pre[l] = incl - len; av[l] = a;
      lds_barrier();
      // kMapBatch products per lane: their codes, then their X gathers,
      // then their LDS sums, so the loads of a batch are in flight together
      const uint16_t* mp = codes + mb;
      for (int p = l; p < total; p += 64 * kMapBatch) {
        unsigned m[kMapBatch];
#pragma unroll
        for (int u = 0; u < kMapBatch; ++u) m[u] = p + 64 * u < total ? mp[p + 64 * u] : kNoSlot;
        double xv[kMapBatch];
        int sl[kMapBatch];
#pragma unroll
        for (int u = 0; u < kMapBatch; ++u) {
          const int o = m[u] & 63;
          sl[u] = (int)(m[u] >> 6);
          xv[u] = m[u] != kNoSlot ? av[o] * X[kst[o] + (p + 64 * u - pre[o])] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kMapBatch; ++u)
          if (m[u] != kNoSlot) atomicAdd(&acc[sl[u]], xv[u]);
      }
      mb += total;
      lds_barrier();
    }
    for (int t = l; t < pn; t += 64) {
      double v = acc[t];
      if (dscale) {
        int lo = 0, hi = nr - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (pofs[mid] <= t) lo = mid; else hi = mid - 1;
        }
        v *= dscale[r0 + lo];
      }
      Y[p0 + t] = v;
      if (flags & EM_DOT) dsum += X[p0 + t] * v;
    }
    lds_barrier();
  }
  dsum = wave_sum(dsum);
  if (l == 0) part[blockIdx.x] = dsum;
}

// Row projection of a vector on the pattern: Out = s * Pi(Y), with the
// block's values staged through LDS (coalesced load and store) and one
// thread per row solving its local system; with EM_DOT, part[block] = sum X*Out.
template <int MAXJ, int CAP>
__global__ void __launch_bounds__(64) k_emin_project(int nrows, int R, const int* __restrict__ Prp,
                                                     const double* __restrict__ Y, const uint16_t* __restrict__ lpair,
                                                     const int* __restrict__ Trp, const double* __restrict__ X,
                                                     double* __restrict__ Out, int flags, double* __restrict__ part,
                                                     long long* __restrict__ iflags) {
  __shared__ double acc[CAP];
  __shared__ uint16_t lps[CAP];
  __shared__ int pofs[kRowsCap + 1];
  const int l = threadIdx.x;
  const RowBlocks B(nrows, R);
  double dsum = 0.0;
  for (int rb = B.first(); rb < B.end(); rb += B.nw) {
    const int r0 = rb * R, r1 = min(r0 + R, nrows), nr = r1 - r0;
    const int p0 = Prp[r0], pn = Prp[r1] - p0;
    // values and local endpoint pairs staged together: the row solves then
    // read only LDS
    for (int t = l; t < pn; t += 64) { acc[t] = Y[p0 + t]; lps[t] = lpair[p0 + t]; }
    for (int t = l; t <= nr; t += 64) pofs[t] = Prp[r0 + t] - p0;
    __syncthreads();
    if (l < nr) {
      const int i = r0 + l;
      const int t0 = Trp[i];
      if (!local_solve_fit<MAXJ>(acc + pofs[l], lps + pofs[l], pofs[l + 1] - pofs[l], Trp[i + 1] - t0, nullptr))
        atomicAdd((unsigned long long*)&iflags[F_NOTSPD], 1ULL);
    }
    __syncthreads();
    for (int t = l; t < pn; t += 64) {
      double v = acc[t];
      if (flags & EM_NEGATE) v = -v;
      Out[p0 + t] = v;
      if (flags & EM_DOT) dsum += X[p0 + t] * v;
    }
    __syncthreads();
  }
  dsum = wave_sum(dsum);
  if (l == 0) part[blockIdx.x] = dsum;
}

// CG vector updates on the pattern values.
__global__ void __launch_bounds__(256) k_cg_update(int64_t n, double* __restrict__ P, double* __restrict__ R,
                                                   const double* __restrict__ D, const double* __restrict__ Q,
                                                   const double* __restrict__ alpha, double* __restrict__ part) {
  __shared__ double sh[4];
  const double a = *alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    P[i] += a * D[i];
    const double r = R[i] - a * Q[i];
    R[i] = r;
    s += r * r;
  }
  double t = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}
__global__ void k_cg_dir(int64_t n, double* __restrict__ D, const double* __restrict__ R, const double* __restrict__ beta) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) D[i] = R[i] + *beta * D[i];
}
// alpha = rho / gamma (0 when rho = 0); flags gamma <= 0 with rho > 0
// Once the projected gradient has fallen to 1e-12 of its first norm the
// minimiser is reached to rounding: the curvature is then rounding noise
// (either sign) and the iterate is left as it is.
__global__ void k_cg_alpha(double* __restrict__ sc, long long* __restrict__ iflags) {
  const double rho = sc[S_RHO], gamma = sc[S_GAMMA];
  const bool converged = rho <= 1e-24 * sc[S_RHO0];
  if (rho > 0.0 && !converged && !(gamma > 0.0)) iflags[F_NOTSPD] += 1;
  sc[S_ALPHA] = (gamma > 0.0 && !converged) ? rho / gamma : 0.0;
}
__global__ void k_copy_scalar(const double* __restrict__ a, double* __restrict__ b) { *b = *a; }
__global__ void k_cg_beta(double* __restrict__ sc) {
  const double rho = sc[S_RHO], rn = sc[S_RHONEW];
  sc[S_BETA] = rho > 0.0 ? rn / rho : 0.0;
  sc[S_RHO] = rn;
}
__global__ void k_axpy_scalar(int64_t n, double* __restrict__ y, const double* __restrict__ x, double a) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] += a * x[i];
}

// ---------------------------------------------------------------------------
// coarsest level: explicit dense inverse
// ---------------------------------------------------------------------------
__global__ void k_to_dense(const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ val, int n,
                           double* __restrict__ M) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = rp[i]; q < rp[i + 1]; ++q) M[(size_t)i * n + col[q]] = val[q];
}
// In-place Gauss-Jordan inversion of the dense SPD matrix (no pivoting: the
// pivots are the diagonals of successive Schur complements, positive for an
// SPD matrix).  Step k: save column k, scale row k by 1/a_kk (with a_kk
// replaced by 1), then a_ij -= a_ik a_kj for i != k (with a_ik replaced by 0).
// After the n steps the matrix holds its inverse.
__global__ void __launch_bounds__(1024) k_gj_pivot(double* __restrict__ M, int n, int k, double* __restrict__ colk,
                                                   long long* __restrict__ iflags) {
  const int t = threadIdx.x;
  const double p = M[(size_t)k * n + k];
  double rowv = 0.0, colv = 0.0;
  if (t < n) {
    colv = M[(size_t)t * n + k];
    rowv = M[(size_t)k * n + t];
  }
  __syncthreads();  // row and column k are read before either is written
  const bool ok = p > 0.0;
  if (t < n) {
    colk[t] = colv;
    M[(size_t)k * n + t] = (t == k ? 1.0 : rowv) / (ok ? p : 1.0);
  }
  if (t == 0 && !ok) iflags[F_NOTSPD] += 1;
}
__global__ void __launch_bounds__(256) k_gj_eliminate(double* __restrict__ M, int n, int k, const double* __restrict__ colk) {
  const int i = blockIdx.y;
  const int j = blockIdx.x * 256 + threadIdx.x;
  if (i == k || j >= n) return;
  const size_t t = (size_t)i * n + j;
  M[t] = (j == k ? 0.0 : M[t]) - colk[i] * M[(size_t)k * n + j];
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------
static int pick_maxj(int maxJ) {
  if (maxJ <= 8) return 8;
  if (maxJ <= 16) return 16;
  return 32;
}

template <class F>
static void with_maxj(int maxJ, F&& f) {
  switch (pick_maxj(maxJ)) {
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 16: f(std::integral_constant<int, 16>{}); break;
    default: f(std::integral_constant<int, 32>{}); break;
  }
}

struct EminWork {
  DBuf<double> P, Rv, Dir, Q, Y, part;
};

static int emin_grid(int nrows, int R) {
  const int nbr = (nrows + R - 1) / R;
  int g = std::min(nbr, 8192);
  g = std::max(8, (g + 7) / 8 * 8);
  return g;
}

// Out = s Pi(dscale mask(A X)) (projection with EM_PROJECT); returns the
// grid whose partial sums X . Out are in part (EM_DOT).  Y is scratch of the
// pattern's length, used when projecting.
static constexpr int kPatSmall = 256;

static int emin_rows_per_block(const Level& L) {
  const int cap = L.maxNp * 4 <= kPatSmall ? kPatSmall : kPatCap;
  return std::max(1, std::min(kRowsCap, cap / std::max(1, L.maxNp)));
}

// The product codes of one energy minimisation (see k_emin_masked).
struct EminMap {
  DBuf<uint16_t> codes;
  DBuf<int2> asl;  // per A entry: pattern start and length of its column
  DBuf<long long> off;
  long long nprod = 0;
  bool on = false, built = false;
};

// Codes take 2 bytes per product and the A-entry records 8 bytes per entry;
// above this size the searches are repeated.
static constexpr double kEminMapMaxBytes = 16.0 * (1 << 30);

static void emin_map_prepare(Level& L, EminMap& m, Ctx& c) {
  const int R = emin_rows_per_block(L);
  const int grid = emin_grid(L.n, R);
  DBuf<long long> cnt(grid, c.s);
  m.off.alloc(grid + 1, c.s);
  c.run(L.fine ? "emin_map_count_l0" : "emin_map_count", 8.0 * (L.n + 1) + 4.0 * L.A.nnz, [&] {
    k_emin_map_count<<<grid, 64, 0, c.s>>>(L.n, R, L.A.rowptr.p, L.A.col.p, L.Pe.rowptr.p, cnt.p);
  });
  c.run("emin_map_offsets", 16.0 * grid, [&] { k_emin_map_offsets<<<1, 1024, 0, c.s>>>(cnt.p, grid, m.off.p); });
  d2h(&m.nprod, m.off.p + grid, 1, c);
  m.built = false;
  const double need = 2.0 * (double)m.nprod + 8.0 * (double)L.A.nnz;
  m.on = m.nprod > 0 && need <= kEminMapMaxBytes;
  // the codes are an optimisation: without room for them every launch searches
  size_t free_b = 0, total_b = 0;
  if (m.on && hipMemGetInfo(&free_b, &total_b) == hipSuccess && need > 0.5 * (double)free_b) m.on = false;
  if (m.on) {
    try {
      m.codes.alloc((size_t)m.nprod, c.s);
      m.asl.alloc((size_t)L.A.nnz, c.s);
    } catch (const Error& e) {
      if (e.code != HCURL_ENOMEM) throw;
      (void)hipGetLastError();
      m.on = false;
    }
  }
  if (!m.on) { m.codes.release(); m.asl.release(); m.off.release(); }
}

static int emin_apply(Level& L, const double* dscale, const double* X, double* Out, int flags, double* part, double* Y,
                      Ctx& c, EminMap* em = nullptr) {
  const int R = emin_rows_per_block(L);
  const bool small = L.maxNp * 4 <= kPatSmall;
  const int grid = emin_grid(L.n, R);
  const int mode = em && em->on ? (em->built ? 2 : 1) : 0;
  // the read-back launch reads the A entries' recorded pattern starts and
  // lengths (8 bytes) in place of their columns, and not the pattern's columns
  const double abytes = mode == 2 ? 16.0 * L.A.nnz : 12.0 * L.A.nnz + (mode == 1 ? 8.0 * L.A.nnz : 0.0);
  const double pbytes = mode == 2 ? 16.0 * L.Pe.nnz : 20.0 * L.Pe.nnz;
  const double mbytes = mode ? 2.0 * (double)em->nprod : 0.0;
  const double bytes = abytes + 4.0 * (L.n + 1) * 2 + pbytes + mbytes;
  const bool proj = flags & EM_PROJECT;
  double* tgt = proj ? Y : Out;
  uint16_t* codes = mode ? em->codes.p : nullptr;
  int2* asl = mode ? em->asl.p : nullptr;
  const long long* moff = mode ? em->off.p : nullptr;
  const char* tag = mode == 1 ? (L.fine ? "emin_masked_build_l0" : "emin_masked_build")
                              : (L.fine ? "emin_masked_spgemm_l0" : "emin_masked_spgemm");
  auto launch = [&](auto cap, auto md) {
    constexpr int CAPV = decltype(cap)::value, MD = decltype(md)::value;
    if constexpr (MD == 2)
      k_emin_masked_codes<CAPV><<<grid, 64, 0, c.s>>>(L.n, R, L.A.rowptr.p, L.A.val.p, asl, dscale, L.Pe.rowptr.p, X, tgt,
                                                      proj ? 0 : flags, part, codes, moff);
    else
      k_emin_masked<CAPV, MD><<<grid, 64, 0, c.s>>>(L.n, R, L.A.rowptr.p, L.A.col.p, L.A.val.p, dscale, L.Pe.rowptr.p,
                                                    L.Pe.col.p, X, tgt, proj ? 0 : flags, part, codes, moff, asl);
  };
  using SmallCap = std::integral_constant<int, kPatSmall>;
  using BigCap = std::integral_constant<int, kPatCap>;
  c.run(tag, bytes, [&] {
    switch (mode * 2 + (small ? 0 : 1)) {
      case 0: launch(SmallCap{}, std::integral_constant<int, 0>{}); break;
      case 1: launch(BigCap{}, std::integral_constant<int, 0>{}); break;
      case 2: launch(SmallCap{}, std::integral_constant<int, 1>{}); break;
      case 3: launch(BigCap{}, std::integral_constant<int, 1>{}); break;
      case 4: launch(SmallCap{}, std::integral_constant<int, 2>{}); break;
      default: launch(BigCap{}, std::integral_constant<int, 2>{}); break;
    }
  });
  if (mode == 1) em->built = true;
  if (proj) {
    // one row per lane: blocks of up to 64 rows, LDS sized for them
    constexpr int kProjCap = 1536;
    const int RP = std::max(1, std::min(kRowsCap, kProjCap / std::max(1, L.maxNp)));
    const int pgrid = emin_grid(L.n, RP);
    with_maxj(L.maxJ + (L.nsingle_coarse ? 1 : 0), [&](auto mj) {
      c.run(L.fine ? "emin_projection_l0" : "emin_projection", 26.0 * L.Pe.nnz, [&] {
        k_emin_project<decltype(mj)::value, kProjCap><<<pgrid, 64, 0, c.s>>>(L.n, RP, L.Pe.rowptr.p, Y, L.lpair.p,
                                                                             L.R.rowptr.p, X, Out, flags, part, c.iscal.p);
      });
    });
    return pgrid;
  }
  return grid;
}

static void make_feasible(Level& L, double* x, bool ones, Ctx& c) {
  with_maxj(L.maxJ + (L.nsingle_coarse ? 1 : 0), [&](auto mj) {
    c.run(L.fine ? "emin_affine_l0" : "emin_affine", 26.0 * L.Pe.nnz, [&] {
      k_make_feasible<decltype(mj)::value><<<ceil_div(L.n, 128), 128, 0, c.s>>>(
          L.n, L.Pe.rowptr.p, x, L.lpair.p, L.R.rowptr.p, L.R.val.p, ones ? 1 : 0, c.iscal.p);
    });
  });
}

void emin_make_feasible(Level& L, double* x, bool ones, Ctx& c) { make_feasible(L, x, ones, c); }

// Commuting residual of a level (Sec. 4.2: P^(e) D_H = D_h P^(n)).  Row i of
// P^(e) D_H lies on the coarse nodes T_i: pattern entry (i, e) adds -p at the
// local tail and +p at the local head of coarse edge e (an end with local
// index 255 is absent: a single-node coarse edge).  One single-wave
// workgroup per row accumulates the row in LDS, subtracts R_i = (D_h P^(n))_i
// on T_i and keeps the largest |difference| and |R|; out holds their bit
// patterns (non-negative doubles order like their bits) and a NaN count.
__global__ void __launch_bounds__(64) k_commute_residual(int n, const int* __restrict__ Prp, const double* __restrict__ pv,
                                                         const uint16_t* __restrict__ lp, const int* __restrict__ Trp,
                                                         const double* __restrict__ Rv,
                                                         unsigned long long* __restrict__ out) {
  __shared__ double b[256];
  const int l = threadIdx.x;
  double cmax = 0.0, rmax = 0.0;
  unsigned long long nan = 0;
  for (int i = blockIdx.x; i < n; i += gridDim.x) {
    const int t0 = Trp[i], nt = Trp[i + 1] - t0;
    const int p0 = Prp[i], np = Prp[i + 1] - p0;
    if (nt > 255) {  // local indices are 8-bit: cannot occur
      nan += l == 0;
      continue;
    }
    for (int k = l; k < nt; k += 64) b[k] = 0.0;
    __syncthreads();
    for (int e = l; e < np; e += 64) {
      const int q = lp[p0 + e], t = q & 255, h = q >> 8;
      const double p = pv[p0 + e];
      if (t < nt) atomicAdd(&b[t], -p);
      if (h < nt) atomicAdd(&b[h], p);
    }
    __syncthreads();
    for (int k = l; k < nt; k += 64) {
      const double r = Rv[t0 + k], d = fabs(b[k] - r);
      nan += (d != d) || (r != r);
      cmax = d > cmax ? d : cmax;
      rmax = fabs(r) > rmax ? fabs(r) : rmax;
    }
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cmax = fmax(cmax, __shfl_xor(cmax, o, 64));
    rmax = fmax(rmax, __shfl_xor(rmax, o, 64));
  }
  nan = wave_sum(nan);
  if (l == 0) {
    atomicMax(out + 0, (unsigned long long)__double_as_longlong(cmax));
    atomicMax(out + 1, (unsigned long long)__double_as_longlong(rmax));
    if (nan) atomicAdd(out + 2, nan);
  }
}

void commute_residual(Level& L, double* abs_max, double* ref_max, Ctx& c) {
  if (!L.has_transfer) fail(HCURL_EINVAL, "level has no transfer");
  DBuf<unsigned long long> r(3, c.s);
  HC_HIP(hipMemsetAsync(r.p, 0, 3 * sizeof(unsigned long long), c.s));
  if (L.n > 0) {
    const int grid = std::min(L.n, 65536);
    c.run("commute_residual", 14.0 * L.Pe.nnz + 8.0 * L.R.nnz, [&] {
      k_commute_residual<<<grid, 64, 0, c.s>>>(L.n, L.Pe.rowptr.p, L.Pe.val.p, L.lpair.p, L.R.rowptr.p, L.R.val.p, r.p);
    });
  }
  unsigned long long h[3];
  d2h(h, r.p, 3, c);
  double a, b;
  std::memcpy(&a, &h[0], sizeof a);
  std::memcpy(&b, &h[1], sizeof b);
  *abs_max = h[2] ? std::numeric_limits<double>::quiet_NaN() : a;
  *ref_max = b;
}

// Sizes of the local least-squares problems (Table 4): the number of rows i
// with |T_i| = J and n_p pattern entries, binned at [min(J, HJ-1) * HNP +
// min(n_p, HNP-1)].  Small keys are counted in an LDS histogram per block.
constexpr int kHistJ = HCURL_LS_HIST_J, kHistNP = HCURL_LS_HIST_NP;
constexpr int kLdsJ = 32, kLdsNP = 64;
__global__ void __launch_bounds__(256) k_ls_histogram(int n, const int* __restrict__ Trp, const int* __restrict__ Prp,
                                                      unsigned long long* __restrict__ hist) {
  __shared__ unsigned int h[kLdsJ * kLdsNP];
  for (int k = threadIdx.x; k < kLdsJ * kLdsNP; k += 256) h[k] = 0;
  __syncthreads();
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const int J = min(Trp[i + 1] - Trp[i], kHistJ - 1), np = min(Prp[i + 1] - Prp[i], kHistNP - 1);
    if (J < kLdsJ && np < kLdsNP) atomicAdd(&h[J * kLdsNP + np], 1u);
    else atomicAdd(&hist[J * kHistNP + np], 1ULL);
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kLdsJ * kLdsNP; k += 256)
    if (h[k]) atomicAdd(&hist[(k / kLdsNP) * kHistNP + k % kLdsNP], (unsigned long long)h[k]);
}

__global__ void k_zero_u64(unsigned long long* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0;
}

void ls_histogram(Level& L, int64_t* out, Ctx& c) {
  if (!L.has_transfer) fail(HCURL_EINVAL, "level has no transfer");
  DBuf<unsigned long long> h((size_t)kHistJ * kHistNP, c.s);
  k_zero_u64<<<ceil_div(kHistJ * kHistNP, 256), 256, 0, c.s>>>(h.p, kHistJ * kHistNP);
  HC_LAUNCH_CHECK();
  if (L.n > 0)
    c.run("ls_histogram", 8.0 * L.n, [&] {
      k_ls_histogram<<<std::min(ceil_div(L.n, 256), 2048), 256, 0, c.s>>>(L.n, L.R.rowptr.p, L.Pe.rowptr.p, h.p);
    });
  d2h((unsigned long long*)out, h.p, (size_t)kHistJ * kHistNP, c);
}

// max |x_i| over a value array (non-negative doubles order like their bits);
// a NaN counts in out[1]
__global__ void k_absmax(int64_t n, const double* __restrict__ v, unsigned long long* __restrict__ out) {
  double m = 0.0;
  unsigned long long nan = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double a = fabs(v[i]);
    nan += a != a;
    m = a > m ? a : m;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  nan = wave_sum(nan);
  if ((threadIdx.x & 63) == 0) {
    atomicMax(out, (unsigned long long)__double_as_longlong(m));
    if (nan) atomicAdd(out + 1, nan);
  }
}

static double abs_max(const Csr& M, Ctx& c) {
  DBuf<unsigned long long> r(2, c.s);
  k_zero_u64<<<1, 64, 0, c.s>>>(r.p, 2);
  HC_LAUNCH_CHECK();
  if (M.nnz > 0)
    c.run("absmax", 8.0 * M.nnz, [&] {
      k_absmax<<<std::min<int64_t>(ceil_div(M.nnz, 256), 2048), 256, 0, c.s>>>(M.nnz, M.val.p, r.p);
    });
  unsigned long long h[2];
  d2h(h, r.p, 2, c);
  double a;
  std::memcpy(&a, &h[0], sizeof a);
  return h[1] ? std::numeric_limits<double>::quiet_NaN() : a;
}

// S_l D_l on every level l < nlev, with S_0 = S and S_{l+1} = P^(e)T S_l P^(e)
// formed on the device by the Galerkin products of the setup.
void curl_residual(Hierarchy& H, const hcurl_csr& S, int nlev, double* absmax, double* refmax) {
  Ctx& c = H.ctx;
  const Level& L0 = *H.lv[0];
  if (S.nrows != L0.n || S.ncols != L0.n || !S.val) fail(HCURL_EINVAL, "S must be n_0 x n_0 with values");
  if (nlev < 1 || nlev > (int)H.lv.size()) fail(HCURL_EINVAL, "nlev out of range");
  Csr Sl;
  upload_csr(S, H.opts.mem_space == HCURL_MEM_DEVICE, Sl, true, c);
  for (int l = 0; l < nlev; ++l) {
    Level& L = *H.lv[l];
    if (L.D.nrows != L.n || !L.D.rowptr.p) gradient_csr(L, c);  // the coarsest level keeps none
    Csr SD;
    spgemm(Sl, L.D, SD, true, c, "spgemm_curl_SD");
    absmax[l] = abs_max(SD, c);
    refmax[l] = abs_max(Sl, c);
    if (l + 1 < nlev) {
      Csr SP, Sn;
      spgemm(Sl, L.Pe, SP, true, c, "spgemm_curl_SP");
      spgemm(L.PeT, SP, Sn, true, c, "spgemm_curl_PtSP");
      Sl = std::move(Sn);
    }
  }
}

__global__ void k_add2(int64_t n, const double* __restrict__ a, const double* __restrict__ b, double* __restrict__ y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a[i] + b[i];
}

static double energy_of(Level& L, const double* P, EminWork& w, Ctx& c, EminMap* em) {
  int g = emin_apply(L, nullptr, P, w.Q.p, EM_DOT, w.part.p, nullptr, c, em);
  // sum of partials (g may exceed kRedBlocks: reduce on host deterministically)
  std::vector<double> h(g);
  d2h(h.data(), w.part.p, g, c);
  double s = 0.0;
  for (double v : h) s += v;
  return 0.5 * s;
}

__global__ void k_sum_partials(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  double r = block_sum256(s, sh);
  if (threadIdx.x == 0) *out = r;
}
static void sum_partials(const double* part, int nb, double* out, Ctx& c) {
  c.run("reduce", 8.0 * nb, [&] { k_sum_partials<<<1, 256, 0, c.s>>>(part, nb, out); });
}

static void energy_minimisation(Hierarchy& H, Level& L, const Level* next, int iters, bool given_init, const double* init,
                                bool init_dev, bool learned) {
  Ctx& c = H.ctx;
  const int64_t np = L.Pe.nnz;
  EminWork w;
  w.P.alloc(np, c.s);
  w.Rv.alloc(np, c.s);
  w.Dir.alloc(np, c.s);
  w.Q.alloc(np, c.s);
  w.Y.alloc(np, c.s);
  w.part.alloc(8192, c.s);
  clear_flag(F_NOTSPD, c);
  clear_flag(F_INFEASIBLE, c);
  clear_flag(F_INFEASIBLE_ROW, c);
  // initial guess
  if (learned) {
    // plain guess plus the network's correction, then the min-norm correction
    DBuf<double> p0plain(np, c.s), pmin(np, c.s);
    make_feasible(L, p0plain.p, true, c);
    fill(pmin.p, 0.0, np, c);
    make_feasible(L, pmin.p, false, c);
    Sample S;
    mpnn_build_sample(H, L, *next, p0plain.p, pmin.p, S);
    Net& net = ((hcurl_mpnn_s*)H.opts.mpnn)->net;
    net.ctx.sync();
    mpnn_forward(net, S, c, false);
    c.run("mpnn_add", 24.0 * np, [&] { k_add2<<<ceil_div(np, 256), 256, 0, c.s>>>(np, p0plain.p, S.delta.p, w.P.p); });
    make_feasible(L, w.P.p, false, c);
  } else {
    if (given_init)
      HC_HIP(hipMemcpyAsync(w.P.p, init, sizeof(double) * np, init_dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c.s));
    make_feasible(L, w.P.p, !given_init, c);
  }
  if (const long long bad = read_flag(F_INFEASIBLE, c))
    fail(HCURL_EINFEASIBLE, std::to_string(bad) + " rows of P^(e) have a commuting constraint without finite solution "
                                                 "(largest: row " + std::to_string(read_flag(F_INFEASIBLE_ROW, c) - 1) + ")");
  L.p0.alloc(np, c.s);
  d2d(L.p0.p, w.P.p, np, c);
  double* sc = c.scal.p;
  L.energy.clear();
  const bool rec = H.opts.record_energy != 0;
  const bool jac = H.opts.emin_method == HCURL_EMIN_JACOBI;
  // masked products of this minimisation: codes pay off from the second one
  EminMap em;
  if (H.opts.emin_codes && (jac ? iters : iters + 1) + (rec ? iters + 1 : 0) >= 2) emin_map_prepare(L, em, c);
  if (rec) L.energy.push_back(energy_of(L, w.P.p, w, c, &em));
  if (jac) {
    DBuf<double> dinv(L.n, c.s);
    diagonal(L.A, dinv.p, true, c);
    for (int it = 0; it < iters; ++it) {
      emin_apply(L, dinv.p, w.P.p, w.Q.p, EM_PROJECT, w.part.p, w.Y.p, c, &em);
      c.run("emin_axpy", 24.0 * np, [&] { k_axpy_scalar<<<ceil_div(np, 256), 256, 0, c.s>>>(np, w.P.p, w.Q.p, -H.opts.emin_omega); });
      if (rec) L.energy.push_back(energy_of(L, w.P.p, w, c, &em));
    }
  } else {
    // R = -Pi(mask(A P)), Dir = R, rho = <R, R>
    emin_apply(L, nullptr, w.P.p, w.Rv.p, EM_PROJECT | EM_NEGATE, w.part.p, w.Y.p, c, &em);
    d2d(w.Dir.p, w.Rv.p, np, c);
    dot(w.Rv.p, w.Rv.p, np, sc + S_RHO, c, 0);
    c.run("cg_scalar", 0.0, [&] { k_copy_scalar<<<1, 1, 0, c.s>>>(sc + S_RHO, sc + S_RHO0); });
    const int ub = Ctx::kRedBlocks;
    const int nbu = (int)std::min<int64_t>(ub, std::max<int64_t>(1, (np + 255) / 256));
    for (int it = 0; it < iters; ++it) {
      int g = emin_apply(L, nullptr, w.Dir.p, w.Q.p, EM_PROJECT | EM_DOT, w.part.p, w.Y.p, c, &em);
      sum_partials(w.part.p, g, sc + S_GAMMA, c);
      c.run("cg_scalar", 0.0, [&] { k_cg_alpha<<<1, 1, 0, c.s>>>(sc, c.iscal.p); });
      c.run("emin_cg_update", 48.0 * np, [&] {
        k_cg_update<<<nbu, 256, 0, c.s>>>(np, w.P.p, w.Rv.p, w.Dir.p, w.Q.p, sc + S_ALPHA, c.red.p);
      });
      reduce_partials(nbu, 0, sc + S_RHONEW, c);
      c.run("cg_scalar", 0.0, [&] { k_cg_beta<<<1, 1, 0, c.s>>>(sc); });
      c.run("emin_cg_dir", 24.0 * np, [&] { k_cg_dir<<<ceil_div(np, 256), 256, 0, c.s>>>(np, w.Dir.p, w.Rv.p, sc + S_BETA); });
      if (rec) L.energy.push_back(energy_of(L, w.P.p, w, c, &em));
    }
  }
  // rounding cleanup: re-apply the affine step
  make_feasible(L, w.P.p, false, c);
  L.Pe.val = std::move(w.P);
  if (read_flag(F_NOTSPD, c)) fail(HCURL_ENOTSPD, "non-positive curvature or local Cholesky failure in the energy minimisation");
}

static void coarsest_factor(Hierarchy& H, Level& L) {
  Ctx& c = H.ctx;
  const int n = L.n;
  if (n > 1024) fail(HCURL_EUNSUPPORTED, "coarsest level has " + std::to_string(n) + " rows (limit 1024): provide more aggregate levels");
  H.co.n = n;
  if (n == 0) return;
  clear_flag(F_NOTSPD, c);
  H.co.inv.alloc((size_t)n * n, c.s);
  DBuf<double> colk(n, c.s);
  double* M = H.co.inv.p;
  HC_HIP(hipMemsetAsync(M, 0, sizeof(double) * n * n, c.s));
  c.run("coarse_dense", 12.0 * L.A.nnz, [&] { k_to_dense<<<ceil_div(n, 64), 64, 0, c.s>>>(L.A.rowptr.p, L.A.col.p, L.A.val.p, n, M); });
  c.run("coarse_inverse", 16.0 * n * n * n, [&] {
    for (int k = 0; k < n; ++k) {
      k_gj_pivot<<<1, 1024, 0, c.s>>>(M, n, k, colk.p, c.iscal.p);
      k_gj_eliminate<<<dim3(ceil_div(n, 256), n), 256, 0, c.s>>>(M, n, k, colk.p);
    }
  });
  if (read_flag(F_NOTSPD, c)) fail(HCURL_ENOTSPD, "coarsest operator is not positive definite");
}

// nodal operator, diagonals, colourings of one level (all levels)
// A^(n) = D^T A D, (A D)^T and the diagonals, from the level's current A
// A product's row pointers kept for spgemm_refill, and taken back.
static void keep_shape(Csr& M, Csr& shape) {
  shape.nrows = M.nrows;
  shape.ncols = M.ncols;
  shape.nnz = M.nnz;
  shape.rowptr = std::move(M.rowptr);
}
static bool take_shape(Csr& shape, Csr& M) {
  if (!shape.rowptr.p) return false;
  M.nrows = shape.nrows;
  M.ncols = shape.ncols;
  M.nnz = shape.nnz;
  M.rowptr = std::move(shape.rowptr);
  return true;
}

// reuse: A has the pattern of the setup's A, so A D and D^T (A D) keep
// theirs and only their numeric passes run
static void nodal_operators(Hierarchy& H, Level& L, bool reuse = false) {
  Ctx& c = H.ctx;
  const char* tAD = L.fine ? "spgemm_AD_l0" : "spgemm_AD";
  const char* tDtAD = L.fine ? "spgemm_DtAD_l0" : "spgemm_DtAD";
  Csr AD;
  if (reuse && L.An.rowptr.p && L.DTA.rowptr.p && take_shape(L.ADshape, AD)) {
    spgemm_refill(L.A, L.D, AD, c, tAD);
    spgemm_refill(L.DT, AD, L.An, c, tDtAD);
    transpose_refill(AD, L.DTA, c);
  } else {
    spgemm(L.A, L.D, AD, true, c, tAD);
    spgemm(L.DT, AD, L.An, true, c, tDtAD);
    transpose(AD, L.DTA, true, c);
  }
  keep_shape(AD, L.ADshape);
  L.dinvA.alloc(L.n, c.s);
  L.dinvAn.alloc(L.m, c.s);
  diagonal(L.A, L.dinvA.p, true, c);
  diagonal(L.An, L.dinvAn.p, true, c);
  clear_flag(F_BAD, c);
  k_check_diag<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.dinvA.p, L.n, c.iscal.p + F_BAD);
  HC_LAUNCH_CHECK();
  if (read_flag(F_BAD, c)) fail(HCURL_EINVAL, "edge operator has a non-positive or non-finite diagonal entry");
}

static void level_operators(Hierarchy& H, Level& L) {
  gradient_csr(L, H.ctx);
  nodal_operators(H, L);
}

// Smoothed aggregation P^(n) = (I - omega D^-1 A^(n)) P-bar on the symbolic
// pattern, rows scaled to sum one; omega = 4 / (3 rho(D^-1 A^(n))).
static void smoothed_aggregation(Hierarchy& H, Level& L, const int* agg, int mH) {
  Ctx& c = H.ctx;
  DBuf<double> x(L.m, c.s), y(L.m, c.s);
  c.run("power_init", 8.0 * L.m, [&] { k_hash_unit<<<ceil_div(L.m, 256), 256, 0, c.s>>>(x.p, L.m); });
  for (int it = 0; it < H.opts.power_iters; ++it) {
    spmv(L.An, x.p, y.p, nullptr, 0, c, "power_spmv");
    c.run("power_scale", 24.0 * L.m, [&] { k_mul<<<ceil_div(L.m, 256), 256, 0, c.s>>>(y.p, L.dinvAn.p, L.m); });
    dot(x.p, x.p, L.m, c.scal.p + S_NX2, c, 1);
    dot(y.p, y.p, L.m, c.scal.p + S_NY2, c, 2);
    c.run("power_norm", 16.0 * L.m, [&] {
      k_power_normalise<<<ceil_div(L.m, 256), 256, 0, c.s>>>(x.p, y.p, L.m, c.scal.p + S_NX2, c.scal.p + S_NY2,
                                                             c.scal.p + S_POWRHO);
    });
  }
  k_omega<<<1, 1, 0, c.s>>>(c.scal.p + S_POWRHO, c.scal.p + S_OMEGA);
  HC_LAUNCH_CHECK();
  double hs[2];
  d2h(hs, c.scal.p + S_POWRHO, 2, c);
  L.rho = hs[0];
  L.omega = hs[1];
  Csr Pbar;
  Pbar.nrows = L.m; Pbar.ncols = mH; Pbar.nnz = L.m;
  Pbar.rowptr.alloc(L.m + 1, c.s); Pbar.col.alloc(L.m, c.s); Pbar.val.alloc(L.m, c.s);
  k_pbar<<<ceil_div(L.m + 1, 256), 256, 0, c.s>>>(agg, L.m, Pbar.rowptr.p, Pbar.col.p, Pbar.val.p);
  HC_LAUNCH_CHECK();
  spgemm(L.An, Pbar, L.Pn, true, c, "spgemm_AnPbar");
  c.run("sa_values", 12.0 * L.Pn.nnz, [&] {
    k_sa_values<<<ceil_div(L.m, 256), 256, 0, c.s>>>(L.Pn.rowptr.p, L.Pn.col.p, L.Pn.val.p, agg, L.dinvAn.p,
                                                     c.scal.p + S_OMEGA, L.m);
  });
}

// Alg. 1: every fine node of the (row-scaled) P^(n) is assigned to one
// coarse node, which defines the piecewise-constant P-bar.
static void alg1_aggregates(Hierarchy& H, Level& L, DBuf<int>& assign) {
  Ctx& c = H.ctx;
  const int mH = L.Pn.ncols;
  Csr PT;
  transpose(L.Pn, PT, true, c);
  {
    std::vector<int> hp(mH + 1);
    d2h(hp.data(), PT.rowptr.p, mH + 1, c);
    for (int j = 0; j < mH; ++j)
      if (hp[j + 1] - hp[j] > kAlg1Cap) fail(HCURL_EUNSUPPORTED, "a column of P^(n) has more than 4096 entries (Alg. 1)");
  }
  HC_HIP(hipMemsetAsync(assign.p, 0xff, sizeof(int) * L.m, c.s));  // every node unassigned (-1)
  c.run("alg1_passes", 12.0 * PT.nnz * H.opts.alg1_passes, [&] {
    k_alg1_passes<<<1, 1024, 0, c.s>>>(PT.rowptr.p, PT.col.p, PT.val.p, mH, L.m, L.Pn.nnz, H.opts.alg1_passes,
                                       assign.p);
  });
  c.run("alg1_leftover", 16.0 * L.Pn.nnz, [&] {
    k_alg1_leftover<<<ceil_div(L.m, 256), 256, 0, c.s>>>(L.Pn.rowptr.p, L.Pn.col.p, L.Pn.val.p, L.m, assign.p);
  });
  DBuf<int> cnt(mH, c.s);
  HC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * mH, c.s));
  k_alg1_count<<<ceil_div(L.m, 256), 256, 0, c.s>>>(assign.p, L.m, cnt.p);
  HC_LAUNCH_CHECK();
  clear_flag(F_BAD, c);
  c.run("alg1_safeguard", 4.0 * mH, [&] {
    k_alg1_safeguard<<<1, 1024, 0, c.s>>>(PT.rowptr.p, PT.col.p, PT.val.p, mH, assign.p, cnt.p, c.iscal.p + F_BAD);
  });
  if (read_flag(F_BAD, c))
    fail(HCURL_EINVAL, "Alg. 1 left a coarse node without fine nodes and no row can move to it");
}

// Everything that builds the transfer from level L to a new level.
// ---------------------------------------------------------------------------
// MIS-2 aggregation from the nodal graph when the caller gives no aggregates
// (not in the paper; reading R26).  Roots: distance-2 maximal independent set
// in Luby rounds on tuples (state, key); every other node joins the root next
// to it, or, two steps away, the aggregate of its neighbour of largest key
// among those next to a root.  Aggregate ids follow the roots' node order.
// ---------------------------------------------------------------------------
enum { MIS_OUT = 0, MIS_UND = 1, MIS_IN = 2 };
__device__ __forceinline__ unsigned long long mis_key(int i) {
  return ((splitmix64((uint64_t)i) >> 34) << 32) | (unsigned long long)(unsigned)i;
}
__global__ void k_mis_tuple(const int* __restrict__ state, int n, unsigned long long* __restrict__ t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) t[i] = ((unsigned long long)state[i] << 62) | mis_key(i);
}
// out_i = max over i and its neighbours of in
__global__ void k_closed_max(const int* __restrict__ rp, const int* __restrict__ col, int n,
                             const unsigned long long* __restrict__ in, unsigned long long* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long m = in[i];
  for (int q = rp[i]; q < rp[i + 1]; ++q) {
    const unsigned long long v = in[col[q]];
    m = v > m ? v : m;
  }
  out[i] = m;
}
__global__ void k_mis_update(int n, const unsigned long long* __restrict__ t, const unsigned long long* __restrict__ m2,
                             int* __restrict__ state, long long* __restrict__ undecided) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || state[i] != MIS_UND) return;
  if (m2[i] == t[i]) state[i] = MIS_IN;
  else if ((m2[i] >> 62) == (unsigned long long)MIS_IN) state[i] = MIS_OUT;
  else atomicAdd((unsigned long long*)undecided, 1ULL);
}
__global__ void k_mis_rootflag(const int* __restrict__ state, int n, int* __restrict__ flag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flag[i] = state[i] == MIS_IN;
}
__global__ void k_mis_first(const int* __restrict__ rp, const int* __restrict__ col, int n, const int* __restrict__ state,
                            const int* __restrict__ rid, int* __restrict__ first) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (state[i] == MIS_IN) { first[i] = rid[i]; return; }
  int a = -1;
  for (int q = rp[i]; q < rp[i + 1]; ++q) {
    const int j = col[q];
    if (j != i && state[j] == MIS_IN) a = rid[j];  // roots are three or more steps apart: at most one
  }
  first[i] = a;
}
__global__ void k_mis_second(const int* __restrict__ rp, const int* __restrict__ col, int n, const int* __restrict__ state,
                             const int* __restrict__ first, int* __restrict__ agg, long long* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (first[i] >= 0) { agg[i] = first[i]; return; }
  unsigned long long best = 0ULL;
  int a = -1;
  for (int q = rp[i]; q < rp[i + 1]; ++q) {
    const int j = col[q];
    if (j == i || first[j] < 0 || state[j] == MIS_IN) continue;
    const unsigned long long k = mis_key(j) + 1ULL;
    if (k > best) { best = k; a = first[j]; }
  }
  agg[i] = a;
  if (a < 0) atomicAdd((unsigned long long*)bad, 1ULL);
}

// Writes L.agg from the graph of L.An; returns the number of aggregates.
static int mis2_aggregates(Hierarchy& H, Level& L) {
  Ctx& c = H.ctx;
  const int n = L.m;
  const Csr& G = L.An;
  DBuf<int> state(n, c.s), flag(n + 1, c.s), rid(n + 1, c.s), first(n, c.s);
  DBuf<unsigned long long> t(n, c.s), m1(n, c.s), m2(n, c.s);
  fill_int(state.p, MIS_UND, n, c);
  for (int round = 0;; ++round) {
    if (round > n + 1) fail(HCURL_EHIP, "MIS-2 rounds did not terminate");
    clear_flag(F_BAD, c);
    c.run("mis2_round", 8.0 * n + 24.0 * G.nnz, [&] {
      k_mis_tuple<<<ceil_div(n, 256), 256, 0, c.s>>>(state.p, n, t.p);
      k_closed_max<<<ceil_div(n, 256), 256, 0, c.s>>>(G.rowptr.p, G.col.p, n, t.p, m1.p);
      k_closed_max<<<ceil_div(n, 256), 256, 0, c.s>>>(G.rowptr.p, G.col.p, n, m1.p, m2.p);
      k_mis_update<<<ceil_div(n, 256), 256, 0, c.s>>>(n, t.p, m2.p, state.p, c.iscal.p + F_BAD);
    });
    if (read_flag(F_BAD, c) == 0) break;
  }
  k_mis_rootflag<<<ceil_div(n, 256), 256, 0, c.s>>>(state.p, n, flag.p);
  HC_LAUNCH_CHECK();
  const int nroots = (int)exclusive_scan(flag.p, rid.p, n, c);
  L.agg.alloc(n, c.s);
  clear_flag(F_BAD, c);
  c.run("mis2_attach", 16.0 * G.nnz, [&] {
    k_mis_first<<<ceil_div(n, 256), 256, 0, c.s>>>(G.rowptr.p, G.col.p, n, state.p, rid.p, first.p);
    k_mis_second<<<ceil_div(n, 256), 256, 0, c.s>>>(G.rowptr.p, G.col.p, n, state.p, first.p, L.agg.p, c.iscal.p + F_BAD);
  });
  if (read_flag(F_BAD, c)) fail(HCURL_EHIP, "MIS-2 aggregation left a node unassigned");
  return nroots;
}

static std::unique_ptr<Level> coarsen(Hierarchy& H, Level& L, const int32_t* agg_in, bool level0, bool agg_ready) {
  Ctx& c = H.ctx;
  const bool dev = H.opts.mem_space == HCURL_MEM_DEVICE;
  // a caller-given nodal prolongator replaces smoothed aggregation on level 0
  const hcurl_csr* Pgiven = level0 ? H.opts.nodal_prolongator : nullptr;
  if (Pgiven) {
    if (Pgiven->nrows != L.m || Pgiven->ncols < 1)
      fail(HCURL_EINVAL, "the given P^(n) must have one row per level-0 node and at least one column");
    upload_csr(*Pgiven, dev, L.Pn, true, c);
    clear_flag(F_BAD, c);
    k_scale_rows<<<ceil_div(L.m, 256), 256, 0, c.s>>>(L.Pn.rowptr.p, L.Pn.val.p, L.m, c.iscal.p + F_BAD);
    HC_LAUNCH_CHECK();
    if (read_flag(F_BAD, c))
      fail(HCURL_EINVAL, "a row of the given P^(n) is empty, sums to zero or holds a non-finite value");
  } else if (!agg_in && !agg_ready) {
    fail(HCURL_EINVAL, "aggregates missing for a level");
  }
  // aggregates: the caller's, MIS-2's (already in L.agg), or Alg. 1 on the given P^(n)
  DBuf<int>& agg = L.agg;
  if (!agg_ready) {
    L.agg.alloc(L.m, c.s);
    if (agg_in)
      HC_HIP(hipMemcpyAsync(agg.p, agg_in, sizeof(int) * L.m, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c.s));
    else
      alg1_aggregates(H, L, agg);
  }
  std::vector<int> hagg(L.m);
  d2h(hagg.data(), agg.p, L.m, c);
  int mH = 0;
  {
    std::vector<char> seen;
    for (int v : hagg) {
      if (v < 0) fail(HCURL_EINVAL, "negative aggregate id");
      mH = std::max(mH, v + 1);
    }
    if (Pgiven && mH > L.Pn.ncols) fail(HCURL_EINVAL, "an aggregate id exceeds the columns of the given P^(n)");
    if (Pgiven) mH = L.Pn.ncols;
    seen.assign(mH, 0);
    for (int v : hagg) seen[v] = 1;
    for (char s : seen)
      if (!s)
        fail(HCURL_EINVAL, agg_in || agg_ready ? "aggregate ids are not contiguous (an id is unused)"
                                               : "Alg. 1 left a coarse node of the given P^(n) without fine nodes");
  }
  if (mH < 2 && L.nsingle == 0)
    fail(HCURL_EINVAL, "the aggregates leave no coarse edge (every fine edge inside one aggregate)");
  // smoothed aggregation P^(n)
  if (!Pgiven) smoothed_aggregation(H, L, agg.p, mH);
  // P-bar from Alg. 1 on the smoothed P^(n) instead of the aggregates
  if (!Pgiven && H.opts.pbar_alg1) {
    L.pbar.alloc(L.m, c.s);
    alg1_aggregates(H, L, L.pbar);
    std::vector<int> hp(L.m);
    d2h(hp.data(), L.pbar.p, L.m, c);
    std::vector<char> seen(mH, 0);
    for (int v : hp) seen[v] = 1;
    for (char s : seen)
      if (!s) fail(HCURL_EINVAL, "Alg. 1 left a coarse node of the smoothed P^(n) without fine nodes");
  }
  const int* pbar = L.pbar.p ? L.pbar.p : agg.p;
  // coarse gradient: Z = E^T E with E the aggregate pairs of crossing edges
  auto next = std::make_unique<Level>();
  DBuf<int> tptr;
  {
    Csr E, ET, Z;
    E.nrows = L.n; E.ncols = mH;
    E.rowptr.alloc(L.n + 1, c.s);
    DBuf<int> cnt(L.n + 1, c.s);
    k_cross_count<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, pbar, L.n, cnt.p);
    HC_LAUNCH_CHECK();
    E.nnz = exclusive_scan(cnt.p, E.rowptr.p, L.n, c);
    E.col.alloc(E.nnz, c.s);
    k_cross_fill<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, pbar, L.n, E.rowptr.p, E.col.p);
    HC_LAUNCH_CHECK();
    transpose(E, ET, false, c);
    spgemm(ET, E, Z, false, c, "spgemm_EtE");
    DBuf<int> ucnt(mH + 1, c.s);
    tptr.alloc(mH + 1, c.s);
    k_upper_count<<<ceil_div(mH, 256), 256, 0, c.s>>>(Z.rowptr.p, Z.col.p, mH, ucnt.p);
    HC_LAUNCH_CHECK();
    const int64_t nH = exclusive_scan(ucnt.p, tptr.p, mH, c);
    next->n = (int)nH;
    next->m = mH;
    next->tail.alloc(nH, c.s);
    next->head.alloc(nH, c.s);
    k_upper_fill<<<ceil_div(mH, 256), 256, 0, c.s>>>(Z.rowptr.p, Z.col.p, mH, tptr.p, next->tail.p, next->head.p);
    HC_LAUNCH_CHECK();
  }
  // Dirichlet edges (Sec. 2): one single-node coarse edge for every coarse
  // node that a fine Dirichlet edge's remaining node belongs to, placed after
  // the two-node edges in node order, +1 at the node
  DBuf<int> smark, spos, sne;
  int nsingle = 0;
  if (L.nsingle > 0) {
    smark.alloc(mH + 1, c.s);
    spos.alloc(mH + 1, c.s);
    sne.alloc(mH, c.s);
    HC_HIP(hipMemsetAsync(smark.p, 0, sizeof(int) * (mH + 1), c.s));
    k_single_mark<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, pbar, L.n, smark.p);
    HC_LAUNCH_CHECK();
    nsingle = (int)exclusive_scan(smark.p, spos.p, mH, c);
  }
  if (next->n == 0 && nsingle == 0)
    fail(HCURL_EINVAL, "the aggregates leave no coarse edge (every fine edge inside one aggregate)");
  L.n_coarse = next->n;
  // T and R = D P^(n) on T
  gradient_product(L.D, L.Pn, L.R, c, L.fine ? "grad_DPn_l0" : "grad_DPn");
  // pattern N, with make_irreducible while a local graph is disconnected
  {
    DBuf<int> cnt(L.n + 1, c.s);
    long long fl[F_NOTSPD + 1];
    Csr Zw;  // P^(n)T D^T D P^(n) = R^T R, formed on the first repair
    L.irreducible_added = 0;
    for (int round = 0;; ++round) {
      for (int f = F_DISCONNECTED; f <= F_TOOBIG; ++f) clear_flag(f, c);
      if (nsingle) {
        k_single_ids<<<ceil_div(mH, 256), 256, 0, c.s>>>(mH, smark.p, spos.p, next->n, sne.p, nullptr, nullptr);
        HC_LAUNCH_CHECK();
      }
      c.run("pattern", 8.0 * L.R.nnz, [&] {
        k_pattern<false><<<ceil_div(L.n, 128), 128, 0, c.s>>>(L.n, L.R.rowptr.p, L.R.col.p, tptr.p, next->head.p,
                                                              nsingle ? sne.p : nullptr, cnt.p, nullptr, nullptr,
                                                              nullptr, c.iscal.p);
      });
      d2h(fl, c.iscal.p, F_NOTSPD + 1, c);
      if (fl[F_TOOBIG]) fail(HCURL_EUNSUPPORTED, "a fine edge touches more than 32 coarse nodes");
      if (!fl[F_DISCONNECTED]) break;
      if (round == 64)
        fail(HCURL_EREDUCIBLE, std::to_string(fl[F_DISCONNECTED]) + " rows stay disconnected after 64 repair rounds");
      if (!Zw.rowptr.p) {
        Csr RT;
        transpose(L.R, RT, true, c);
        spgemm(RT, L.R, Zw, true, c, "spgemm_RtR");
      }
      DBuf<unsigned long long> cand(L.n, c.s);
      DBuf<int> xcnt(mH + 1, c.s), xptr(mH + 1, c.s), cursor(mH + 1, c.s), ucnt(mH + 1, c.s);
      c.run("irreducible_pick", 8.0 * L.R.nnz, [&] {
        k_irreducible_pick<<<ceil_div(L.n, 128), 128, 0, c.s>>>(L.n, L.R.rowptr.p, L.R.col.p, tptr.p, next->head.p,
                                                               Zw.rowptr.p, Zw.col.p, Zw.val.p, cand.p);
      });
      HC_HIP(hipMemsetAsync(xcnt.p, 0, sizeof(int) * (mH + 1), c.s));
      k_cand_count<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.n, cand.p, xcnt.p);
      HC_LAUNCH_CHECK();
      const int64_t nx = exclusive_scan(xcnt.p, xptr.p, mH, c);
      DBuf<int> xcol(std::max<int64_t>(nx, 1), c.s);
      d2d(cursor.p, xptr.p, mH + 1, c);
      k_cand_fill<<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.n, cand.p, cursor.p, xcol.p);
      HC_LAUNCH_CHECK();
      k_edge_union<false><<<ceil_div(mH, 256), 256, 0, c.s>>>(mH, tptr.p, next->head.p, xptr.p, xcol.p, ucnt.p,
                                                              nullptr, nullptr, nullptr);
      HC_LAUNCH_CHECK();
      DBuf<int> nptr(mH + 1, c.s);
      const int64_t nH = exclusive_scan(ucnt.p, nptr.p, mH, c);
      DBuf<int> ntail(nH, c.s), nhead(nH, c.s);
      k_edge_union<true><<<ceil_div(mH, 256), 256, 0, c.s>>>(mH, tptr.p, next->head.p, xptr.p, xcol.p, nullptr, nptr.p,
                                                             ntail.p, nhead.p);
      HC_LAUNCH_CHECK();
      L.irreducible_added += nH - next->n;
      next->n = (int)nH;
      next->tail = std::move(ntail);
      next->head = std::move(nhead);
      tptr = std::move(nptr);
    }
    if (nsingle) {
      const int nTwo = next->n;
      DBuf<int> nt(nTwo + nsingle, c.s), nh(nTwo + nsingle, c.s);
      d2d(nt.p, next->tail.p, nTwo, c);
      d2d(nh.p, next->head.p, nTwo, c);
      k_single_ids<<<ceil_div(mH, 256), 256, 0, c.s>>>(mH, smark.p, spos.p, nTwo, sne.p, nt.p, nh.p);
      HC_LAUNCH_CHECK();
      next->tail = std::move(nt);
      next->head = std::move(nh);
      next->n = nTwo + nsingle;
    }
    next->nsingle = nsingle;
    L.nsingle_coarse = nsingle;
    L.n_coarse = next->n;
    L.maxJ = (int)fl[F_MAXJ];
    if (nsingle && L.maxJ + 1 > kMaxJ)
      fail(HCURL_EUNSUPPORTED, "a fine edge with a Dirichlet coarse edge touches 32 coarse nodes");
    L.maxNp = (int)fl[F_MAXNP];
    if (L.maxNp > kPatCap) fail(HCURL_EUNSUPPORTED, "a row of P^(e) has more than 512 pattern entries");
    L.Pe.nrows = L.n;
    L.Pe.ncols = next->n;
    L.Pe.rowptr.alloc(L.n + 1, c.s);
    L.Pe.nnz = exclusive_scan(cnt.p, L.Pe.rowptr.p, L.n, c);
    L.Pe.col.alloc(L.Pe.nnz, c.s);
    L.lpair.alloc(L.Pe.nnz, c.s);
    c.run("pattern", 14.0 * L.R.nnz, [&] {
      k_pattern<true><<<ceil_div(L.n, 128), 128, 0, c.s>>>(L.n, L.R.rowptr.p, L.R.col.p, tptr.p, next->head.p,
                                                           nsingle ? sne.p : nullptr, nullptr,
                                                           L.Pe.rowptr.p, L.Pe.col.p, L.lpair.p, c.iscal.p);
    });
  }
  // energy minimisation of P^(e)
  const bool given = level0 && H.opts.init_guess == HCURL_INIT_GIVEN;
  const bool learned = level0 && H.opts.init_guess == HCURL_INIT_MPNN;
  const int iters = (given || learned) ? H.opts.emin_iters_given : H.opts.emin_iters;
  energy_minimisation(H, L, next.get(), iters, given, H.opts.init_values, dev, learned);
  transpose(L.Pe, L.PeT, true, c);
  // Galerkin A_H = P^T A P
  {
    Csr AP;
    spgemm(L.A, L.Pe, AP, true, c, L.fine ? "spgemm_AP_l0" : "spgemm_AP");
    spgemm(L.PeT, AP, next->A, true, c, L.fine ? "spgemm_PtAP_l0" : "spgemm_PtAP");
    keep_shape(AP, L.APshape);
  }
  L.has_transfer = true;
  return next;
}

void build_hierarchy(Hierarchy& H, const hcurl_csr& A, const hcurl_csr& Dh, const double* coords, const int32_t* const* aggs,
                     int nagg) {
  Ctx& c = H.ctx;
  const bool dev = H.opts.mem_space == HCURL_MEM_DEVICE;
  if (A.nrows != A.ncols) fail(HCURL_EINVAL, "A must be square");
  if (A.nrows == 0 || Dh.ncols == 0) fail(HCURL_EINVAL, "empty problem: A and D_h need at least one edge and one node");
  if (Dh.nrows != A.nrows) fail(HCURL_EINVAL, "D_h must have one row per edge");
  if (nagg < 0 || (nagg > 0 && !aggs)) fail(HCURL_EINVAL, "aggregates missing");
  auto L0 = std::make_unique<Level>();
  L0->fine = true;
  L0->n = (int)A.nrows;
  L0->m = (int)Dh.ncols;
  upload_csr(A, dev, L0->A, true, c);
  {
    Csr Du;
    upload_csr(Dh, dev, Du, true, c);
    L0->tail.alloc(L0->n, c.s);
    L0->head.alloc(L0->n, c.s);
    clear_flag(F_BAD, c);
    clear_flag(F_TOOBIG, c);
    if (L0->n)
      k_grad_from_csr<<<ceil_div(L0->n, 256), 256, 0, c.s>>>(Du.rowptr.p, Du.col.p, Du.val.p, L0->n, L0->m, L0->tail.p,
                                                             L0->head.p, c.iscal.p + F_BAD, c.iscal.p + F_TOOBIG);
    HC_LAUNCH_CHECK();
    if (read_flag(F_BAD, c))
      fail(HCURL_EINVAL, "every row of D_h must hold one -1 and one +1, or a single +-1 (a Dirichlet edge)");
    L0->nsingle = (int)read_flag(F_TOOBIG, c);
    if (L0->nsingle && H.opts.init_guess == HCURL_INIT_MPNN)
      fail(HCURL_EUNSUPPORTED, "the learned initial guess does not take Dirichlet edges");
  }
  if (H.opts.init_guess == HCURL_INIT_GIVEN && !H.opts.init_values)
    fail(HCURL_EINVAL, "init_guess = HCURL_INIT_GIVEN needs init_values");
  if (H.opts.init_guess == HCURL_INIT_MPNN && (!H.opts.mpnn || !coords))
    fail(HCURL_EINVAL, "init_guess = HCURL_INIT_MPNN needs opts.mpnn and coords");
  if (coords) {
    H.coords.alloc(3 * (size_t)Dh.ncols, c.s);
    HC_HIP(hipMemcpyAsync(H.coords.p, coords, sizeof(double) * 3 * Dh.ncols,
                          dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c.s));
  }
  H.lv.clear();
  H.lv.push_back(std::move(L0));
  const int maxl = H.opts.max_levels > 0 ? H.opts.max_levels : 1 << 20;
  for (int l = 0;; ++l) {
    Level& L = *H.lv.back();
    const int32_t* amap = l < nagg ? aggs[l] : nullptr;
    const bool given_pn = l == 0 && H.opts.nodal_prolongator != nullptr;
    const bool auto_agg = !amap && !given_pn && H.opts.aggregation == HCURL_AGG_MIS2;
    const bool stop = (l >= nagg && !auto_agg) || (int)H.lv.size() >= maxl ||
                      (H.opts.coarse_max_rows > 0 && L.n <= H.opts.coarse_max_rows);
    if (stop) break;
    level_operators(H, L);
    // a level whose MIS-2 aggregation does not reduce it stays the coarsest
    if (auto_agg && mis2_aggregates(H, L) >= L.m) {
      L.agg.release();
      break;
    }
    color_rows(L.A, L.colorA, L.rowsA, L.cptrA, L.ncolA, c);
    color_rows(L.An, L.colorAn, L.rowsAn, L.cptrAn, L.ncolAn, c);
    H.lv.push_back(coarsen(H, L, amap, l == 0, auto_agg));
  }
  H.pn_given = H.opts.nodal_prolongator != nullptr;
  coarsest_factor(H, *H.lv.back());
  prepare_solve(H);
  c.sync();
}

// Same row pointers and columns as the stored pattern.
__global__ void k_same_pattern(const int* __restrict__ rp0, const int* __restrict__ col0, const int* __restrict__ rp1,
                               const int* __restrict__ col1, int n, long long* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > n) return;
  if (rp0[i] != rp1[i]) { atomicAdd((unsigned long long*)bad, 1ULL); return; }
  if (i == n) return;
  for (int q = rp0[i]; q < rp0[i + 1]; ++q)
    if (col0[q] != col1[q]) { atomicAdd((unsigned long long*)bad, 1ULL); return; }
}

void update_hierarchy(Hierarchy& H, const hcurl_csr& A, int mode, int iters) {
  Ctx& c = H.ctx;
  const bool dev = H.opts.mem_space == HCURL_MEM_DEVICE;
  Level& L0 = *H.lv[0];
  if (A.nrows != L0.n || A.ncols != L0.n || A.nnz != L0.A.nnz)
    fail(HCURL_EINVAL, "the new matrix must keep the sparsity pattern of the setup's");
  Csr Anew;
  upload_csr(A, dev, Anew, true, c);
  clear_flag(F_BAD, c);
  k_same_pattern<<<ceil_div(L0.n + 1, 256), 256, 0, c.s>>>(L0.A.rowptr.p, L0.A.col.p, Anew.rowptr.p, Anew.col.p, L0.n,
                                                          c.iscal.p + F_BAD);
  HC_LAUNCH_CHECK();
  if (read_flag(F_BAD, c)) fail(HCURL_EINVAL, "the new matrix must keep the sparsity pattern of the setup's");
  // captured graphs hold the addresses of buffers rebuilt below
  if (H.vgraph) { HC_HIP(hipGraphExecDestroy(H.vgraph)); H.vgraph = nullptr; }
  if (H.cgraph) { HC_HIP(hipGraphExecDestroy(H.cgraph)); H.cgraph = nullptr; }
  H.valid = false;
  L0.A.val = std::move(Anew.val);
  const int K = iters < 0 ? H.opts.emin_iters : iters;
  for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
    Level& L = *H.lv[l];
    Level& N = *H.lv[l + 1];
    nodal_operators(H, L, true);
    if (mode == HCURL_REUSE_WARM) {
      if (!(l == 0 && H.pn_given)) smoothed_aggregation(H, L, L.agg.p, L.Pn.ncols);
      gradient_product(L.D, L.Pn, L.R, c, L.fine ? "grad_DPn_l0" : "grad_DPn");
      energy_minimisation(H, L, &N, K, true, L.Pe.val.p, true, false);
      transpose_refill(L.Pe, L.PeT, c);
    } else {
      L.energy.clear();
    }
    // P^(e) keeps its pattern in both modes: A P^(e) and the Galerkin
    // product keep theirs
    Csr AP;
    const char* tAP = L.fine ? "spgemm_AP_l0" : "spgemm_AP";
    const char* tPtAP = L.fine ? "spgemm_PtAP_l0" : "spgemm_PtAP";
    if (N.A.rowptr.p && take_shape(L.APshape, AP)) {
      spgemm_refill(L.A, L.Pe, AP, c, tAP);
      spgemm_refill(L.PeT, AP, N.A, c, tPtAP);
    } else {
      spgemm(L.A, L.Pe, AP, true, c, tAP);
      spgemm(L.PeT, AP, N.A, true, c, tPtAP);
    }
    keep_shape(AP, L.APshape);
  }
  coarsest_factor(H, *H.lv.back());
  prepare_solve(H);
  c.sync();
  H.valid = true;
}

}  // namespace hc
