// Solve phase (Sec. 6.1): multicolour symmetric Gauss-Seidel, Hiptmair
// smoothing, V-cycle with a direct coarsest solve, preconditioned CG.
#include <chrono>
#include <cmath>
#include <algorithm>
#include <cstring>

#include "amg.hpp"

namespace hc {

enum { P_RZ = 16, P_PQ, P_ALPHA, P_RR, P_RZNEW, P_RZOLD, P_BETA, P_FF };

// ---------------------------------------------------------------------------
// Jones-Plassmann colouring with priorities (splitmix64(i), i): every round,
// an uncoloured vertex whose priority beats all uncoloured neighbours takes
// the smallest colour absent from its coloured neighbours.  color < 0 means
// uncoloured (-1) or selected in this round (-2).
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool prio_greater(int u, int v) {
  const uint64_t hu = splitmix64((uint64_t)u), hv = splitmix64((uint64_t)v);
  return hu > hv || (hu == hv && u > v);
}

__global__ void k_jp_select(const int* __restrict__ rp, const int* __restrict__ col, int n, int* __restrict__ color) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || color[v] >= 0) return;
  for (int q = rp[v]; q < rp[v + 1]; ++q) {
    const int u = col[q];
    if (u != v && color[u] < 0 && prio_greater(u, v)) return;
  }
  color[v] = -2;
}

__global__ void k_jp_assign(const int* __restrict__ rp, const int* __restrict__ col, int n, int* __restrict__ color,
                            unsigned long long* __restrict__ remaining) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  const int cv = v < n ? color[v] : 0;
  // only "any vertex left" matters: one store per wave that has one
  if (__any(cv == -1) && (threadIdx.x & 63) == 0) *remaining = 1ULL;
  if (cv != -2) return;
  for (int base = 0;; base += 64) {
    unsigned long long used = 0ull;
    for (int q = rp[v]; q < rp[v + 1]; ++q) {
      const int c = color[col[q]];
      if (c >= base && c < base + 64) used |= 1ull << (c - base);
    }
    if (used != ~0ull) {
      color[v] = base + __ffsll((long long)~used) - 1;
      return;
    }
  }
}

// Rows are grouped by colour, in increasing row index inside a colour: the
// rows of one launch then follow the lattice order, so neighbouring waves
// gather overlapping parts of x (grouping by row length as well was measured
// 20% slower on the finest level, because every length class sweeps the whole
// domain again).
// Rows per colour: a histogram in LDS per block (few colours would make
// global atomics contend), added to the global counts once per block.
static constexpr int kHistLds = 4096;
__global__ void __launch_bounds__(256) k_group_key(const int* __restrict__ color, int n, int ncol, int* __restrict__ key,
                                                   int* __restrict__ hist) {
  __shared__ int h[kHistLds];
  const bool lds = ncol <= kHistLds;
  if (lds)
    for (int k = threadIdx.x; k < ncol; k += 256) h[k] = 0;
  __syncthreads();
  for (int v = blockIdx.x * 256 + threadIdx.x; v < n; v += gridDim.x * 256) {
    const int k = color[v];
    key[v] = k;
    if (lds) atomicAdd(&h[k], 1);
    else atomicAdd(&hist[k], 1);
  }
  __syncthreads();
  if (lds)
    for (int k = threadIdx.x; k < ncol; k += 256)
      if (h[k]) atomicAdd(&hist[k], h[k]);
}
__global__ void k_flag_eq(const int* __restrict__ key, int n, int k, int* __restrict__ flag) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) flag[v] = key[v] == k;
}
__global__ void k_scatter_eq(const int* __restrict__ key, int n, int k, const int* __restrict__ pos, int base,
                             int* __restrict__ rows) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n && key[v] == k) rows[base + pos[v]] = v;
}

// Stable grouping of the rows by colour in two passes over blocks of 256
// rows: per-block counts of every colour (stored colour-major, so that one
// exclusive scan gives every (colour, block) its first slot), then every row
// goes to its slot plus its rank among the block's earlier rows of its colour
// (wave ballots per colour present in the wave, then the counts of the
// block's earlier waves).
static constexpr int kGroupLds = 1024;
__global__ void __launch_bounds__(256) k_block_colour_count(const int* __restrict__ color, int n, int ncol, int nb,
                                                            int* __restrict__ cnt) {
  __shared__ int h[kGroupLds];
  for (int k = threadIdx.x; k < ncol; k += 256) h[k] = 0;
  __syncthreads();
  const int v = blockIdx.x * 256 + threadIdx.x;
  if (v < n) atomicAdd(&h[color[v]], 1);
  __syncthreads();
  for (int k = threadIdx.x; k < ncol; k += 256) cnt[(int64_t)k * nb + blockIdx.x] = h[k];
}

__global__ void __launch_bounds__(256) k_block_colour_scatter(const int* __restrict__ color, int n, int ncol, int nb,
                                                              const int* __restrict__ off, int* __restrict__ rows) {
  __shared__ int wc[4][kGroupLds];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  for (int k = l; k < ncol; k += 64) wc[w][k] = 0;
  const int v = blockIdx.x * 256 + threadIdx.x;
  const int k = v < n ? color[v] : -1;
  // rank among the wave's earlier lanes of the same colour
  int rank = 0;
  unsigned long long todo = __ballot(k >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int kc = __shfl(k, leader, 64);
    const unsigned long long m = __ballot(k == kc);
    if (k == kc) rank = __popcll(m & ((1ull << l) - 1ull));
    if (l == leader) wc[w][kc] = __popcll(m);
    todo &= ~m;
  }
  __syncthreads();
  if (k >= 0) {
    int base = off[(int64_t)k * nb + blockIdx.x];
    for (int u = 0; u < w; ++u) base += wc[u][k];
    rows[base + rank] = v;
  }
}

void color_rows(const Csr& A, DBuf<int>& color, DBuf<int>& rows, std::vector<int>& cptr, int& ncol, Ctx& c) {
  const int n = A.nrows;
  color.alloc(n, c.s);
  rows.alloc(n, c.s);
  fill_int(color.p, -1, n, c);
  unsigned long long* rem = (unsigned long long*)(c.iscal.p + 8);
  for (int round = 0;; ++round) {
    if (round > n + 1) fail(HCURL_EHIP, "colouring did not terminate");
    // booked bytes: every vertex's colour; the rows still uncoloured (read
    // in full) shrink every round and are not counted, so this is a lower bound
    c.run("jp_select", 4.0 * n, [&] { k_jp_select<<<ceil_div(n, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, n, color.p); });
    HC_HIP(hipMemsetAsync(rem, 0, sizeof(unsigned long long), c.s));
    c.run("jp_assign", 4.0 * n, [&] { k_jp_assign<<<ceil_div(n, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, n, color.p, rem); });
    unsigned long long h = 0;
    d2h(&h, rem, 1, c);
    if (h == 0) break;
  }
  std::vector<int> hc_(n);
  d2h(hc_.data(), color.p, n, c);
  ncol = 0;
  for (int v : hc_) ncol = std::max(ncol, v + 1);
  const int nk = ncol;
  DBuf<int> key(n + 1, c.s), hist(nk, c.s);
  HC_HIP(hipMemsetAsync(hist.p, 0, sizeof(int) * nk, c.s));
  if (n) k_group_key<<<(int)std::min<int64_t>(ceil_div(n, 256), 2048), 256, 0, c.s>>>(color.p, n, ncol, key.p, hist.p);
  HC_LAUNCH_CHECK();
  std::vector<int> hh(nk);
  d2h(hh.data(), hist.p, nk, c);
  cptr.assign(ncol + 1, 0);
  const int nb = ceil_div(n, 256);
  if (nk <= kGroupLds && (int64_t)nk * nb < (int64_t)1 << 31) {
    DBuf<int> bcnt((int64_t)nk * nb, c.s), boff((int64_t)nk * nb + 1, c.s);
    c.run("colour_group", 4.0 * n + 4.0 * nk * nb, [&] {
      k_block_colour_count<<<nb, 256, 0, c.s>>>(color.p, n, nk, nb, bcnt.p);
    });
    exclusive_scan(bcnt.p, boff.p, (int64_t)nk * nb, c);
    c.run("colour_group", 8.0 * n + 4.0 * nk * nb, [&] {
      k_block_colour_scatter<<<nb, 256, 0, c.s>>>(color.p, n, nk, nb, boff.p, rows.p);
    });
  } else {
    DBuf<int> flag(n + 1, c.s), pos(n + 1, c.s);
    int base = 0;
    for (int k = 0; k < nk; ++k) {
      if (hh[k] == 0) continue;
      k_flag_eq<<<ceil_div(n, 256), 256, 0, c.s>>>(key.p, n, k, flag.p);
      HC_LAUNCH_CHECK();
      exclusive_scan(flag.p, pos.p, n, c);
      k_scatter_eq<<<ceil_div(n, 256), 256, 0, c.s>>>(key.p, n, k, pos.p, base, rows.p);
      HC_LAUNCH_CHECK();
      base += hh[k];
    }
  }
  for (int k = 0; k < nk; ++k) cptr[k + 1] += hh[k];
  for (int k = 0; k < ncol; ++k) cptr[k + 1] += cptr[k];
}

__global__ void k_perm_len(const int* __restrict__ rp, const int* __restrict__ rows, int n, int* __restrict__ len) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) len[g] = rp[rows[g] + 1] - rp[rows[g]];
}
__global__ void __launch_bounds__(256) k_perm_copy(const int* __restrict__ rp, const int* __restrict__ col,
                                                   const double* __restrict__ val, const int* __restrict__ rows, int n,
                                                   const int* __restrict__ nrp, int* __restrict__ ncol,
                                                   double* __restrict__ nval) {
  const int g = (blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int l = threadIdx.x & 15;
  if (g >= n) return;
  const int a = rp[rows[g]], len = rp[rows[g] + 1] - a, o = nrp[g];
  for (int q = l; q < len; q += 16) {
    ncol[o + q] = col[a + q];
    nval[o + q] = val[a + q];
  }
}

void colour_major(const Csr& A, const DBuf<int>& rows, Csr& Acm, Ctx& c) {
  const int n = A.nrows;
  Acm.nrows = n;
  Acm.ncols = A.ncols;
  Acm.nnz = A.nnz;
  Acm.rowptr.alloc(n + 1, c.s);
  Acm.col.alloc(A.nnz, c.s);
  Acm.val.alloc(A.nnz, c.s);
  DBuf<int> len(n + 1, c.s);
  k_perm_len<<<ceil_div(n, 256), 256, 0, c.s>>>(A.rowptr.p, rows.p, n, len.p);
  HC_LAUNCH_CHECK();
  exclusive_scan(len.p, Acm.rowptr.p, n, c);
  c.run("colour_major", 24.0 * A.nnz, [&] {
    k_perm_copy<<<ceil_div((int64_t)n * 16, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, A.val.p, rows.p, n, Acm.rowptr.p,
                                                               Acm.col.p, Acm.val.p);
  });
}

__global__ void k_gather(const double* __restrict__ x, const int* __restrict__ rows, double* __restrict__ y, int n) {
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) y[g] = x[rows[g]];
}
void gather_vec(const double* x, const int* rows, double* y, int n, Ctx& c) {
  if (n) c.run("gather", 16.0 * n, [&] { k_gather<<<ceil_div(n, 256), 256, 0, c.s>>>(x, rows, y, n); });
}

// ---------------------------------------------------------------------------
// Gauss-Seidel on the rows of one colour: x_i += (b_i - A_i x) / a_ii.
// Rows of one colour are not coupled, so they update in parallel.  The
// matrix is the colour-major copy: the colour's rows are contiguous (g) and
// rows[g] is the original row index, used for b and x.
// ---------------------------------------------------------------------------
// One row by a group of LPR lanes; every kernel below sums a row this way, so
// a row gives the same bits whichever kernel updates it.
template <class V, class T, int LPR>
__device__ __forceinline__ void gs_row(int g, int l, const int* __restrict__ rows, const int* __restrict__ rp,
                                       const int* __restrict__ col, const V* __restrict__ val,
                                       const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x) {
  T s = 0;
  const int a = rp[g], e = rp[g + 1];
  const int i = rows[g];
  const T bi = b[i], di = dinv[g];
  // Up to four entries per lane are loaded before they are summed, so their
  // gathers overlap; padding slots gather the row's own x entry (a local
  // line).  Plain loads: non-temporal ones measured no faster here.
  int q = a + l;
  for (; q + 3 * LPR < e; q += 4 * LPR) {
    const int c0 = col[q], c1 = col[q + LPR], c2 = col[q + 2 * LPR], c3 = col[q + 3 * LPR];
    const V v0 = val[q], v1 = val[q + LPR], v2 = val[q + 2 * LPR], v3 = val[q + 3 * LPR];
    s += (T)v0 * x[c0] + (T)v1 * x[c1] + (T)v2 * x[c2] + (T)v3 * x[c3];
  }
  int cc[3];
  V vv[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int qq = q + u * LPR;
    cc[u] = qq < e ? col[qq] : i;
    vv[u] = qq < e ? val[qq] : V(0);
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) s += (T)vv[u] * x[cc[u]];
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
  if (l == 0) x[i] += (bi - s) * di;
}

template <class V, class T, int LPR, int TAG>
__global__ void __launch_bounds__(256) k_gs_color(int g0, int nr, const int* __restrict__ rows, const int* __restrict__ rp,
                                                  const int* __restrict__ col, const V* __restrict__ val,
                                                  const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x) {
  // neighbouring row blocks share gathered x entries: give every XCD a
  // contiguous range of blocks so they meet in the same L2
  const int g = g0 + (xcd_block(gridDim.x) * blockDim.x + threadIdx.x) / LPR;
  const int l = threadIdx.x & (LPR - 1);
  if (g >= g0 + nr) return;
  gs_row<V, T, LPR>(g, l, rows, rp, col, val, dinv, b, x);
}

// Colours k0, k0 + dir, ..., nk of them, in one workgroup with a barrier
// between colours: for runs of small colour classes, whose launches would
// cost more than their rows.  The coarse levels' colour classes have a long
// tail: the densest rows of a Galerkin operator can form a clique, which takes
// one colour per row.
template <class V, class T, int LPR>
__global__ void __launch_bounds__(1024) k_gs_chain(int k0, int nk, int dir, const int* __restrict__ cptr,
                                                   const int* __restrict__ rows, const int* __restrict__ rp,
                                                   const int* __restrict__ col, const V* __restrict__ val,
                                                   const T* __restrict__ dinv, const T* __restrict__ b,
                                                   T* __restrict__ x) {
  const int l = threadIdx.x & (LPR - 1);
  const int grp = threadIdx.x / LPR;
  constexpr int NG = 1024 / LPR;
  for (int t = 0; t < nk; ++t) {
    const int k = k0 + dir * t;
    for (int g = cptr[k] + grp; g < cptr[k + 1]; g += NG) gs_row<V, T, LPR>(g, l, rows, rp, col, val, dinv, b, x);
    __syncthreads();
  }
}

// gs_row on a run's LDS copy of x: lcol[q - e_lo] is the slot of entry q's
// column, lrow[g - g_lo] the slot of row g's own entry; b and 1/a_ii are read
// as in gs_row.  Same arithmetic in the same order as gs_row.
template <class V, class T, int LPR>
__device__ __forceinline__ void gs_row_lds(int g, int l, int g_lo, int e_lo, const int* __restrict__ lcol,
                                           const int* __restrict__ lrow, const int* __restrict__ rows,
                                           const int* __restrict__ rp, const V* __restrict__ val,
                                           const T* __restrict__ dinv, const T* __restrict__ b, T* xs) {
  T s = 0;
  const int a = rp[g], e = rp[g + 1];
  const int i = rows[g];
  const int il = lrow[g - g_lo];
  const T bi = b[i], di = dinv[g];
  int q = a + l;
  for (; q + 3 * LPR < e; q += 4 * LPR) {
    const int c0 = lcol[q - e_lo], c1 = lcol[q + LPR - e_lo], c2 = lcol[q + 2 * LPR - e_lo],
              c3 = lcol[q + 3 * LPR - e_lo];
    const V v0 = val[q], v1 = val[q + LPR], v2 = val[q + 2 * LPR], v3 = val[q + 3 * LPR];
    s += (T)v0 * xs[c0] + (T)v1 * xs[c1] + (T)v2 * xs[c2] + (T)v3 * xs[c3];
  }
  int cc[3];
  V vv[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int qq = q + u * LPR;
    cc[u] = qq < e ? lcol[qq - e_lo] : il;
    vv[u] = qq < e ? val[qq] : V(0);
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) s += (T)vv[u] * xs[cc[u]];
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
  if (l == 0) xs[il] += (bi - s) * di;
}

// k_gs_chain with the x entries the run touches (nU <= kChainSlots of them,
// listed in U) copied to LDS first: each chained colour then gathers from LDS
// instead of L2.  The run's own rows are written back at the end; the other
// entries of U do not change during the run.
static constexpr int kChainSlots = 16384;
template <class V, class T, int LPR>
__global__ void __launch_bounds__(1024) k_gs_chain_lds(int k0, int nk, int dir, const int* __restrict__ cptr, int g_lo,
                                                       int g_hi, int e_lo, int nU, const int* __restrict__ U,
                                                       const int* __restrict__ lcol, const int* __restrict__ lrow,
                                                       const int* __restrict__ rows, const int* __restrict__ rp,
                                                       const V* __restrict__ val, const T* __restrict__ dinv,
                                                       const T* __restrict__ b, T* __restrict__ x) {
  __shared__ T xs[kChainSlots];
  const int l = threadIdx.x & (LPR - 1);
  const int grp = threadIdx.x / LPR;
  constexpr int NG = 1024 / LPR;
  for (int j = threadIdx.x; j < nU; j += 1024) xs[j] = x[U[j]];
  __syncthreads();
  for (int t = 0; t < nk; ++t) {
    const int k = k0 + dir * t;
    for (int g = cptr[k] + grp; g < cptr[k + 1]; g += NG)
      gs_row_lds<V, T, LPR>(g, l, g_lo, e_lo, lcol, lrow, rows, rp, val, dinv, b, xs);
    __syncthreads();
  }
  for (int g = g_lo + (int)threadIdx.x; g < g_hi; g += 1024) x[rows[g]] = xs[lrow[g - g_lo]];
}

// The whole symmetric sweep (all colours forward, then backward) in one
// workgroup, for levels small enough that launches would dominate.  The
// level's x (at most kSmallRows entries) lives in LDS for the sweep: one CU
// would otherwise fetch a cache line per gathered entry.
static constexpr int kSmallRows = 8192;
template <class V, class T, int LPR>
__global__ void __launch_bounds__(1024) k_gs_sweep_small(int n, int ncol, const int* __restrict__ cptr,
                                                         const int* __restrict__ rows, const int* __restrict__ rp,
                                                         const int* __restrict__ col, const V* __restrict__ val,
                                                         const T* __restrict__ dinv, const T* __restrict__ b,
                                                         T* __restrict__ x) {
  __shared__ T xs[kSmallRows];
  const int l = threadIdx.x & (LPR - 1);
  const int grp = threadIdx.x / LPR;
  constexpr int NG = 1024 / LPR;
  for (int i = threadIdx.x; i < n; i += 1024) xs[i] = x[i];
  __syncthreads();
  // forward over the colours, then backward from the second-to-last: the
  // last colour's rows already solve their equations after the forward pass
  // (rows of one colour do not couple), so repeating it changes nothing
  for (int step = 0; step < 2 * ncol - 1; ++step) {
    const int k = step < ncol ? step : 2 * ncol - 2 - step;
    for (int g = cptr[k] + grp; g < cptr[k + 1]; g += NG) gs_row<V, T, LPR>(g, l, rows, rp, col, val, dinv, b, xs);
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += 1024) x[i] = xs[i];
}

static constexpr int kSmallLevel = kSmallRows;

// Algorithmic bytes of one colour launch: the rows' CSR data (column and
// value per entry, row pointer and original row index per row), their b,
// 1/a_ii and x written, and every x entry gathered once per sweep (ideal reuse
// of the gathered neighbours): nnz_c (4 + sizeof V) + rows_c (8 + 4 sizeof T).
static int gs_lpr(double avg) { return avg <= 20 ? 8 : avg <= 48 ? 16 : 32; }

// Launch plan of one symmetric sweep: colours in sweep order, forward, then
// backward from the second-to-last (the last colour's rows already solve
// their equations after the forward pass, so repeating it is a no-op); a run
// of two or more consecutive colours in one direction whose classes have at
// most `tiny` rows goes to one chain launch.
// Colour classes of at most this many rows go into single-workgroup chain
// launches: one pass of the workgroup per class.  (Classes of up to four
// passes measured no faster at 128^3: 4.01 against 3.95 ms for the coarse
// levels of a V-cycle.)
static constexpr int kChainPasses = 1;
static int chain_rows(int lpr) { return kChainPasses * 1024 / lpr; }

template <class F, class G>
static void sweep_plan(const std::vector<int>& cptr, int ncol, int tiny, F&& single, G&& chain, int first = 0) {
  auto pass = [&](int first, int last, int dir) {
    for (int k = first; k != last + dir;) {
      int n = 0;
      while (k + dir * n != last + dir && cptr[k + dir * n + 1] - cptr[k + dir * n] <= tiny) ++n;
      if (n >= 2) {
        chain(k, n, dir);
        k += dir * n;
      } else {
        single(k);
        k += dir;
      }
    }
  };
  pass(first, ncol - 1, 1);
  if (ncol >= 2) pass(ncol - 2, 0, -1);
}

// LDS plans of the chain runs of a colour-major matrix (levels swept by
// launches only): the x entries each run touches, and every entry's and row's
// slot among them.
void plan_chains(const Csr& Acm, const DBuf<int>& rows, const std::vector<int>& cptr, int ncol,
                 std::vector<ChainRun>& out, Ctx& c) {
  out.clear();
  if (Acm.nrows <= kSmallRows || Acm.nrows == 0) return;
  const int tiny = chain_rows(gs_lpr((double)Acm.nnz / Acm.nrows));
  // the runs of a sweep from colour 0 and of one whose first colour was
  // written by k_gs_first_colour (forward pass from colour 1)
  auto add_run = [&](int k0, int nk, int dir) {
    for (const ChainRun& r : out)
      if (r.k0 == k0 && r.nk == nk && r.dir == dir) return;
    ChainRun R;
    R.k0 = k0;
    R.nk = nk;
    R.dir = dir;
    const int klo = dir > 0 ? k0 : k0 - (nk - 1), khi = dir > 0 ? k0 + nk - 1 : k0;
    R.g_lo = cptr[klo];
    R.g_hi = cptr[khi + 1];
    const int nr = R.g_hi - R.g_lo;
    std::vector<int> rp(nr + 1), rw(std::max(nr, 1));
    d2h(rp.data(), Acm.rowptr.p + R.g_lo, nr + 1, c);
    if (nr) d2h(rw.data(), rows.p + R.g_lo, nr, c);
    R.e_lo = rp[0];
    const int ne = rp[nr] - rp[0];
    std::vector<int> cl(std::max(ne, 1));
    if (ne) d2h(cl.data(), Acm.col.p + R.e_lo, ne, c);
    std::vector<int> U(cl.begin(), cl.begin() + ne);
    U.insert(U.end(), rw.begin(), rw.begin() + nr);
    std::sort(U.begin(), U.end());
    U.erase(std::unique(U.begin(), U.end()), U.end());
    R.nU = (int)U.size();
    if (R.nU <= kChainSlots && nr > 0) {
      auto slot = [&](int v) { return (int)(std::lower_bound(U.begin(), U.end(), v) - U.begin()); };
      std::vector<int> lc(std::max(ne, 1)), lr(nr);
      for (int q = 0; q < ne; ++q) lc[q] = slot(cl[q]);
      for (int g = 0; g < nr; ++g) lr[g] = slot(rw[g]);
      R.U.alloc(R.nU, c.s);
      R.lcol.alloc(std::max(ne, 1), c.s);
      R.lrow.alloc(nr, c.s);
      h2d(R.U.p, U.data(), R.nU, c);
      h2d(R.lcol.p, lc.data(), std::max(ne, 1), c);
      h2d(R.lrow.p, lr.data(), nr, c);
    }
    out.push_back(std::move(R));
  };
  sweep_plan(cptr, ncol, tiny, [](int) {}, add_run, 0);
  sweep_plan(cptr, ncol, tiny, [](int) {}, add_run, 1);
}

// Algorithmic bytes of one colour launch: the rows' CSR data (column and
// value per entry, row pointer and original row index per row), their b,
// 1/a_ii and x written, and every x entry gathered once per sweep (ideal reuse
// of the gathered neighbours): nnz_c (4 + sizeof V) + rows_c (8 + 4 sizeof T).
template <class V, class T, int TAG>
static void sgs_t(const Csr& A, const V* val, const T* dinv, const DBuf<int>& rows, const std::vector<int>& cptr,
                  const DBuf<int>& cptr_d, int ncol, const std::vector<ChainRun>& runs, const T* b, T* x, Ctx& c,
                  const char* tag, int first = 0) {
  const double avg = A.nrows ? (double)A.nnz / A.nrows : 0.0;
  if (A.nrows <= kSmallLevel) {
    const double bytes = 2.0 * ((double)A.nnz * (4 + sizeof(V)) + (double)A.nrows * (8 + 4 * sizeof(T)));
    c.run("sgs_small", bytes, [&] { k_gs_sweep_small<V, T, 8><<<1, 1024, 0, c.s>>>(A.nrows, ncol, cptr_d.p, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
    return;
  }
  const int lpr = gs_lpr(avg);
  auto launch = [&](int k) {
    const int g0 = cptr[k], nr = cptr[k + 1] - cptr[k];
    if (!nr) return;
    const double bytes = (double)nr * avg * (4 + sizeof(V)) + (double)nr * (8 + 4 * sizeof(T));
    if (lpr == 8)
      c.run(tag, bytes, [&] { k_gs_color<V, T, 8, TAG><<<ceil_div((int64_t)nr * 8, 256), 256, 0, c.s>>>(g0, nr, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
    else if (lpr == 16)
      c.run(tag, bytes, [&] { k_gs_color<V, T, 16, TAG><<<ceil_div((int64_t)nr * 16, 256), 256, 0, c.s>>>(g0, nr, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
    else
      c.run(tag, bytes, [&] { k_gs_color<V, T, 32, TAG><<<ceil_div((int64_t)nr * 32, 256), 256, 0, c.s>>>(g0, nr, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
  };
  auto chain = [&](int k0, int nk, int dir) {
    double nr = 0.0;
    for (int t = 0; t < nk; ++t) nr += cptr[k0 + dir * t + 1] - cptr[k0 + dir * t];
    const double bytes = nr * avg * (4 + sizeof(V)) + nr * (8 + 4 * sizeof(T));
    const ChainRun* R = nullptr;
    for (const ChainRun& r : runs)
      if (r.k0 == k0 && r.nk == nk && r.dir == dir && r.U.p) R = &r;
    if (R) {
      if (lpr == 8)
        c.run(tag, bytes, [&] { k_gs_chain_lds<V, T, 8><<<1, 1024, 0, c.s>>>(k0, nk, dir, cptr_d.p, R->g_lo, R->g_hi, R->e_lo, R->nU, R->U.p, R->lcol.p, R->lrow.p, rows.p, A.rowptr.p, val, dinv, b, x); });
      else if (lpr == 16)
        c.run(tag, bytes, [&] { k_gs_chain_lds<V, T, 16><<<1, 1024, 0, c.s>>>(k0, nk, dir, cptr_d.p, R->g_lo, R->g_hi, R->e_lo, R->nU, R->U.p, R->lcol.p, R->lrow.p, rows.p, A.rowptr.p, val, dinv, b, x); });
      else
        c.run(tag, bytes, [&] { k_gs_chain_lds<V, T, 32><<<1, 1024, 0, c.s>>>(k0, nk, dir, cptr_d.p, R->g_lo, R->g_hi, R->e_lo, R->nU, R->U.p, R->lcol.p, R->lrow.p, rows.p, A.rowptr.p, val, dinv, b, x); });
      return;
    }
    if (lpr == 8)
      c.run(tag, bytes, [&] { k_gs_chain<V, T, 8><<<1, 1024, 0, c.s>>>(k0, nk, dir, cptr_d.p, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
    else if (lpr == 16)
      c.run(tag, bytes, [&] { k_gs_chain<V, T, 16><<<1, 1024, 0, c.s>>>(k0, nk, dir, cptr_d.p, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
    else
      c.run(tag, bytes, [&] { k_gs_chain<V, T, 32><<<1, 1024, 0, c.s>>>(k0, nk, dir, cptr_d.p, rows.p, A.rowptr.p, A.col.p, val, dinv, b, x); });
  };
  // first = 1: the caller has swept colour 0 already (k_gs_first_colour)
  sweep_plan(cptr, ncol, chain_rows(lpr), launch, chain, first);
}

// x += D c  with D given by its endpoints: x_e += c[head] - c[tail]
template <class T>
__global__ void k_grad_add(const int* __restrict__ tail, const int* __restrict__ head, int n, const T* __restrict__ cn,
                           T* __restrict__ x) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int h = head[e], t = tail[e];  // -1: the eliminated end of a Dirichlet edge
  x[e] += (h >= 0 ? cn[h] : T(0)) - (t >= 0 ? cn[t] : T(0));
}

// dense coarsest solve x = A^-1 b (one wave per row)
template <class T>
__global__ void __launch_bounds__(256) k_dense_apply(const double* __restrict__ inv, int n, const T* __restrict__ b,
                                                     T* __restrict__ x) {
  const int row = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int l = threadIdx.x & 63;
  if (row >= n) return;
  double s = 0.0;
  for (int j = l; j < n; j += 64) s += inv[(size_t)row * n + j] * (double)b[j];
  s = wave_sum(s);
  if (l == 0) x[row] = (T)s;
}

// ---------------------------------------------------------------------------
// Hiptmair smoother and V-cycle
// ---------------------------------------------------------------------------
// Level 0 gets its own kernel instances (TAG 1, 2) so that profiles separate
// the fine-level sweeps from the launch-bound coarse ones.
// The first colour of a sweep that starts from x = 0 gathers only zeros, so
// its rows become 0 + (b_i - 0) / a_ii (gs_row's value, bit for bit) and
// every other row stays zero: one pass over the level in place of the fill
// and that colour's launch.  color and dinv are in original row order; dinv
// is rounded to T as the sweeps' copies of it are.
template <class T>
__global__ void k_gs_first_colour(int n, const int* __restrict__ color, const double* __restrict__ dinv,
                                  const T* __restrict__ b, T* __restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T v = 0;
  if (color[i] == 0) v += (b[i] - T(0)) * (T)dinv[i];
  x[i] = v;
}

// Levels that sweep by launches; the others sweep in one workgroup
static bool swept_by_launches(const Level& L) { return L.Acm.nrows > kSmallLevel; }
static bool nodes_swept_by_launches(const Level& L) { return L.Ancm.nrows > kSmallLevel; }

// x_zero: x is to start from zero (the pre-smoother of a V-cycle visit); on
// levels swept by launches the first sweep then writes x itself.
static void hiptmair64(Level& L, bool fine, double* x, const double* b, const double* dtb, Ctx& c, bool x_zero) {
  auto edge = [&](int first) {
    if (fine) sgs_t<double, double, 1>(L.Acm, L.Acm.val.p, L.dinvAcm.p, L.rowsA, L.cptrA, L.cptrA_d, L.ncolA, L.chainsA, b, x, c, "sgs_edge_l0", first);
    else sgs_t<double, double, 0>(L.Acm, L.Acm.val.p, L.dinvAcm.p, L.rowsA, L.cptrA, L.cptrA_d, L.ncolA, L.chainsA, b, x, c, "sgs_edge", first);
  };
  if (x_zero && swept_by_launches(L)) {
    c.run(fine ? "sgs_first_l0" : "sgs_first", 28.0 * L.n, [&] {
      k_gs_first_colour<double><<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.n, L.colorA.p, L.dinvA.p, b, x);
    });
    edge(1);
  } else {
    if (x_zero) fill(x, 0.0, L.n, c);
    edge(0);
  }
  // nodal right-hand side D^T (b - A x) = D^T b - (D^T A) x
  spmv(L.DTA, x, L.rn.p, dtb, 1, c, fine ? "nodal_residual_l0" : "nodal_residual");
  // the nodal sweep starts from c = 0: its first colour is written in one pass
  // with the zero fill where the level is swept by launches
  int nfirst = 0;
  if (nodes_swept_by_launches(L)) {
    c.run(fine ? "sgs_node_first_l0" : "sgs_node_first", 28.0 * L.m, [&] {
      k_gs_first_colour<double><<<ceil_div(L.m, 256), 256, 0, c.s>>>(L.m, L.colorAn.p, L.dinvAn.p, L.rn.p, L.cn.p);
    });
    nfirst = 1;
  } else {
    fill(L.cn.p, 0.0, L.m, c);
  }
  if (fine) sgs_t<double, double, 2>(L.Ancm, L.Ancm.val.p, L.dinvAncm.p, L.rowsAn, L.cptrAn, L.cptrAn_d, L.ncolAn, L.chainsAn, L.rn.p, L.cn.p, c, "sgs_node_l0", nfirst);
  else sgs_t<double, double, 0>(L.Ancm, L.Ancm.val.p, L.dinvAncm.p, L.rowsAn, L.cptrAn, L.cptrAn_d, L.ncolAn, L.chainsAn, L.rn.p, L.cn.p, c, "sgs_node", nfirst);
  c.run("grad_add", 24.0 * L.n, [&] { k_grad_add<double><<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, L.n, L.cn.p, x); });
  edge(0);
}

// FP32 form of the V-cycle: smoothers and transfers read the FP32 copies of
// the operators; vectors are FP64 on level 0 (T = double) and FP32 below
// (T = float); residuals are formed with the FP64 operator (spmv_v64), since
// the FP32 copy of A breaks S D = 0 by more than sigma M in low-conductivity
// regions.  The V-cycle's output stays FP64.
static inline void fill_t(double* x, double v, int64_t n, Ctx& c) { fill(x, v, n, c); }
static inline void fill_t(float* x, float v, int64_t n, Ctx& c) { fill32(x, v, n, c); }

template <class T>
struct Vec32Form;
template <>
struct Vec32Form<double> {
  static double* r(Level& L) { return L.r.p; }
  static double* rn(Level& L) { return L.rn.p; }
  static double* cn(Level& L) { return L.cn.p; }
  static double* dtb(Level& L) { return L.dtb.p; }
  static const double* dA(Level& L) { return L.dinvAcm.p; }
  static const double* dAn(Level& L) { return L.dinvAncm.p; }
};
template <>
struct Vec32Form<float> {
  static float* r(Level& L) { return L.r32.p; }
  static float* rn(Level& L) { return L.rn32.p; }
  static float* cn(Level& L) { return L.cn32.p; }
  static float* dtb(Level& L) { return L.dtb32.p; }
  static const float* dA(Level& L) { return L.dinvAcm32.p; }
  static const float* dAn(Level& L) { return L.dinvAncm32.p; }
};

template <class T>
static void hiptmair32(Level& L, bool fine, T* x, const T* b, const T* dtb, Ctx& c, bool x_zero) {
  using F = Vec32Form<T>;
  auto edge = [&](int first) {
    if (fine) sgs_t<float, T, 1>(L.Acm, L.Acm.val32.p, F::dA(L), L.rowsA, L.cptrA, L.cptrA_d, L.ncolA, L.chainsA, b, x, c, "sgs_edge32_l0", first);
    else sgs_t<float, T, 0>(L.Acm, L.Acm.val32.p, F::dA(L), L.rowsA, L.cptrA, L.cptrA_d, L.ncolA, L.chainsA, b, x, c, "sgs_edge32", first);
  };
  if (x_zero && swept_by_launches(L)) {
    c.run(fine ? "sgs_first32_l0" : "sgs_first32", (12.0 + 2.0 * sizeof(T)) * L.n, [&] {
      k_gs_first_colour<T><<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.n, L.colorA.p, L.dinvA.p, b, x);
    });
    edge(1);
  } else {
    if (x_zero) fill_t(x, T(0), L.n, c);
    edge(0);
  }
  // nodal right-hand side D^T b - (D^T A) x with the FP64 operator
  spmv_v64<T, T>(L.DTA, x, F::rn(L), dtb, 1, c, fine ? "nodal_residual32_l0" : "nodal_residual32");
  int nfirst = 0;
  if (nodes_swept_by_launches(L)) {
    c.run(fine ? "sgs_node_first32_l0" : "sgs_node_first32", (12.0 + 2.0 * sizeof(T)) * L.m, [&] {
      k_gs_first_colour<T><<<ceil_div(L.m, 256), 256, 0, c.s>>>(L.m, L.colorAn.p, L.dinvAn.p, F::rn(L), F::cn(L));
    });
    nfirst = 1;
  } else {
    fill_t(F::cn(L), T(0), L.m, c);
  }
  if (fine) sgs_t<float, T, 2>(L.Ancm, L.Ancm.val32.p, F::dAn(L), L.rowsAn, L.cptrAn, L.cptrAn_d, L.ncolAn, L.chainsAn, F::rn(L), F::cn(L), c, "sgs_node32_l0", nfirst);
  else sgs_t<float, T, 0>(L.Ancm, L.Ancm.val32.p, F::dAn(L), L.rowsAn, L.cptrAn, L.cptrAn_d, L.ncolAn, L.chainsAn, F::rn(L), F::cn(L), c, "sgs_node32", nfirst);
  c.run("grad_add32", (8.0 + 3.0 * sizeof(T)) * L.n, [&] { k_grad_add<T><<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, L.n, F::cn(L), x); });
  edge(0);
}

static void coarse_cycle(Hierarchy& H);

static void vcycle64(Hierarchy& H, int l, const double* b, double* x) {
  Ctx& c = H.ctx;
  if (l == (int)H.lv.size() - 1) {
    c.run("coarse_solve", 8.0 * H.co.n * H.co.n, [&] {
      k_dense_apply<double><<<ceil_div((int64_t)H.co.n * 64, 256), 256, 0, c.s>>>(H.co.inv.p, H.co.n, b, x);
    });
    return;
  }
  Level& L = *H.lv[l];
  Level& N = *H.lv[l + 1];
  spmv(L.DT, b, L.dtb.p, nullptr, 0, c, "grad_transpose");
  hiptmair64(L, l == 0, x, b, L.dtb.p, c, true);
  spmv(L.A, x, L.r.p, b, 1, c, l == 0 ? "residual_l0" : "residual");
  spmv(L.PeT, L.r.p, N.b.p, nullptr, 0, c, "restrict");
  if (l == 0) coarse_cycle(H);
  else vcycle64(H, l + 1, N.b.p, N.x.p);
  spmv(L.Pe, N.x.p, x, nullptr, 2, c, "prolong");
  hiptmair64(L, l == 0, x, b, L.dtb.p, c, false);
}

// Level l of the FP32 form (T = double on level 0, float below).
template <class T>
static void vcycle32(Hierarchy& H, int l, const T* b, T* x) {
  Ctx& c = H.ctx;
  if (l == (int)H.lv.size() - 1) {
    c.run("coarse_solve32", 8.0 * H.co.n * H.co.n, [&] {
      k_dense_apply<T><<<ceil_div((int64_t)H.co.n * 64, 256), 256, 0, c.s>>>(H.co.inv.p, H.co.n, b, x);
    });
    return;
  }
  Level& L = *H.lv[l];
  Level& N = *H.lv[l + 1];
  using F = Vec32Form<T>;
  spmv_v32<T, T>(L.DT, b, F::dtb(L), nullptr, 0, c, "grad_transpose32");
  hiptmair32<T>(L, l == 0, x, b, F::dtb(L), c, true);
  spmv_v64<T, T>(L.A, x, F::r(L), b, 1, c, l == 0 ? "residual32_l0" : "residual32");
  spmv_v32<T, float>(L.PeT, F::r(L), N.b32.p, nullptr, 0, c, "restrict32");
  if (l == 0) coarse_cycle(H);
  else vcycle32<float>(H, l + 1, N.b32.p, N.x32.p);
  spmv_v32<float, T>(L.Pe, N.x32.p, x, nullptr, 2, c, "prolong32");
  hiptmair32<T>(L, l == 0, x, b, F::dtb(L), c, false);
}

static void vcycle_direct(Hierarchy& H, const double* r, double* z) {
  if (H.fp32 && H.lv.size() > 1) {
    vcycle32<double>(H, 0, r, z);
  } else {
    vcycle64(H, 0, r, z);
  }
}

// Captures what `body` enqueues on the handle's stream as a graph (no
// per-kernel events inside a capture).
template <class F>
static void capture_graph(Hierarchy& H, hipGraphExec_t* out, F&& body) {
  Ctx& c = H.ctx;
  const bool prof = c.profile;
  hipGraph_t g = nullptr;
  HC_HIP(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
  c.profile = false;
  H.capturing = true;
  try {
    body();
  } catch (...) {
    c.profile = prof;
    H.capturing = false;
    (void)hipStreamEndCapture(c.s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  c.profile = prof;
  H.capturing = false;
  HC_HIP(hipStreamEndCapture(c.s, &g));
  hipError_t e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  HC_HIP(e);
}

static bool graphs_allowed(const Hierarchy& H) { return H.ctx.s != nullptr && H.opts.profile != 2; }

// Levels >= 1 of the V-cycle (from lv[1].b into lv[1].x).  The coarse levels
// are launch-bound (hundreds of short colour sweeps), and their kernels and
// buffers are the same on every call, so on a non-null stream they are
// captured once and replayed as one graph; the finest level stays eager.
static void coarse_cycle(Hierarchy& H) {
  Level& N = *H.lv[1];
  const bool f32 = H.fp32;
  auto body = [&] {
    if (f32) vcycle32<float>(H, 1, N.b32.p, N.x32.p);
    else vcycle64(H, 1, N.b.p, N.x.p);
  };
  if (H.capturing || !graphs_allowed(H) || H.lv.size() < 3) {
    body();
    return;
  }
  if (!H.cgraph) capture_graph(H, &H.cgraph, body);
  Ctx& c = H.ctx;
  c.run("graph_coarse_levels", 0.0, [&] { HC_HIP(hipGraphLaunch(H.cgraph, c.s)); });
}

// Without per-kernel profiling on a non-null stream, the whole V-cycle of the
// PCG workspace (pr -> pz) is captured once and replayed; otherwise level 0
// runs eagerly and the coarse levels replay as a graph.
void apply_vcycle(Hierarchy& H, const double* r, double* z) {
  Ctx& c = H.ctx;
  const bool whole = graphs_allowed(H) && !c.profile && r == H.pr.p && z == H.pz.p;
  if (!whole) {
    vcycle_direct(H, r, z);
    return;
  }
  if (!H.vgraph) capture_graph(H, &H.vgraph, [&] { vcycle_direct(H, r, z); });
  HC_HIP(hipGraphLaunch(H.vgraph, c.s));
}

// ---------------------------------------------------------------------------
// preparation: workspace and FP32 copies
// ---------------------------------------------------------------------------
static void make32(Csr& A, Ctx& c) {
  if (!A.val.p) return;
  A.val32.alloc(A.nnz, c.s);
  cast_d2f(A.val.p, A.val32.p, A.nnz, c);
}

// Cancellation ratio of D^T A D at node u: (|D|^T |A| |D| 1)_u / (D^T A D)_uu
// = sum over the edges e at u of s_e, over A^(n)_uu.  For a
// gradient field x, A x = sigma M x while the terms summed are of size
// |S||x|: an operator rounded with relative error u leaves an error of about
// u times this ratio relative to the result.
// s_e = sum_f |a_ef| (|D| 1)_f: two per edge, one per Dirichlet edge
// eight lanes per row (coalesced loads of the row's entries), shuffle sum
__global__ void __launch_bounds__(256) k_abs_rowsum(const int* __restrict__ rp, const int* __restrict__ col,
                                                    const double* __restrict__ val, const int* __restrict__ drp, int n,
                                                    double* __restrict__ s) {
  const int i = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3);
  const int l = threadIdx.x & 7;
  double t = 0.0;
  if (i < n)
    for (int q = rp[i] + l; q < rp[i + 1]; q += 8) {
      const int f = col[q];
      t += fabs(val[q]) * (double)(drp[f + 1] - drp[f]);
    }
#pragma unroll
  for (int o = 4; o > 0; o >>= 1) t += __shfl_xor(t, o, 8);
  if (i < n && l == 0) s[i] = t;
}
__global__ void __launch_bounds__(256) k_cancel_max(const int* __restrict__ rp, const int* __restrict__ col, int m,
                                                    const double* __restrict__ s, const double* __restrict__ dinv,
                                                    unsigned long long* __restrict__ out) {
  __shared__ double sh[4];
  const int u = blockIdx.x * 256 + threadIdx.x;
  double r = 0.0;
  if (u < m) {
    double t = 0.0;
    for (int q = rp[u]; q < rp[u + 1]; ++q) t += s[col[q]];
    const double d = dinv[u];
    if (d > 0.0) r = t * d;
  }
  for (int o = 32; o > 0; o >>= 1) r = fmax(r, __shfl_xor(r, o, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = r;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double b = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
    // non-negative doubles order like their bit patterns
    atomicMax(out, (unsigned long long)__double_as_longlong(b));
  }
}

static double cancellation_ratio(Level& L, Ctx& c) {
  if (L.n == 0 || L.m == 0) return 0.0;
  constexpr int kSlot = 10;
  unsigned long long* out = (unsigned long long*)(c.iscal.p + kSlot);
  DBuf<double> s;
  s.alloc(L.n, c.s);
  HC_HIP(hipMemsetAsync(out, 0, sizeof(unsigned long long), c.s));
  c.run("cancel_rowsum", 16.0 * L.A.nnz, [&] {
    k_abs_rowsum<<<ceil_div((int64_t)L.n * 8, 256), 256, 0, c.s>>>(L.A.rowptr.p, L.A.col.p, L.A.val.p, L.D.rowptr.p,
                                                                  L.n, s.p);
  });
  c.run("cancel_max", 12.0 * L.DT.nnz, [&] {
    k_cancel_max<<<ceil_div(L.m, 256), 256, 0, c.s>>>(L.DT.rowptr.p, L.DT.col.p, L.m, s.p, L.dinvAn.p, out);
  });
  unsigned long long bits = 0;
  d2h(&bits, out, 1, c);
  double r;
  std::memcpy(&r, &bits, sizeof r);
  s.release();
  return r;
}

// The FP32 form rounds every operator of the smoothers to FP32; it is used
// (opts.vcycle_fp32 = 1) only if FP32 machine epsilon (2^-23) times the
// cancellation ratio stays at most kFp32Guard on every smoothed level, else
// the V-cycle stays FP64.  opts.vcycle_fp32 = 2 uses it unconditionally.
static constexpr double kFp32Guard = 10.0;

void prepare_solve(Hierarchy& H) {
  Ctx& c = H.ctx;
  for (size_t l = 0; l + 1 < H.lv.size(); ++l) H.lv[l]->cancel = cancellation_ratio(*H.lv[l], c);
  bool ok = H.lv.size() > 1;
  for (size_t l = 0; l + 1 < H.lv.size(); ++l) ok = ok && 0x1p-23 * H.lv[l]->cancel <= kFp32Guard;
  H.fp32 = H.opts.vcycle_fp32 == 2 || (H.opts.vcycle_fp32 == 1 && ok);
  const bool f32 = H.fp32;
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = *H.lv[l];
    L.x.alloc(L.n, c.s);
    L.b.alloc(L.n, c.s);
    if (l + 1 == H.lv.size()) {
      if (f32) { L.x32.alloc(L.n, c.s); L.b32.alloc(L.n, c.s); }
      continue;
    }
    colour_major(L.A, L.rowsA, L.Acm, c);
    colour_major(L.An, L.rowsAn, L.Ancm, c);
    L.cptrA_d.alloc(L.ncolA + 1, c.s);
    L.cptrAn_d.alloc(L.ncolAn + 1, c.s);
    h2d(L.cptrA_d.p, L.cptrA.data(), L.ncolA + 1, c);
    h2d(L.cptrAn_d.p, L.cptrAn.data(), L.ncolAn + 1, c);
    plan_chains(L.Acm, L.rowsA, L.cptrA, L.ncolA, L.chainsA, c);
    plan_chains(L.Ancm, L.rowsAn, L.cptrAn, L.ncolAn, L.chainsAn, c);
    L.dinvAcm.alloc(L.n, c.s);
    L.dinvAncm.alloc(L.m, c.s);
    gather_vec(L.dinvA.p, L.rowsA.p, L.dinvAcm.p, L.n, c);
    gather_vec(L.dinvAn.p, L.rowsAn.p, L.dinvAncm.p, L.m, c);
    L.r.alloc(L.n, c.s);
    L.rn.alloc(L.m, c.s);
    L.cn.alloc(L.m, c.s);
    L.dtb.alloc(L.m, c.s);
    if (f32) {
      // FP32 operator copies on every level; FP32 vectors below level 0
      make32(L.Acm, c); make32(L.Ancm, c);
      make32(L.Pe, c); make32(L.PeT, c); make32(L.DT, c);
      if (l > 0) {
        L.x32.alloc(L.n, c.s); L.b32.alloc(L.n, c.s); L.r32.alloc(L.n, c.s);
        L.rn32.alloc(L.m, c.s); L.cn32.alloc(L.m, c.s); L.dtb32.alloc(L.m, c.s);
        L.dinvAcm32.alloc(L.n, c.s); L.dinvAncm32.alloc(L.m, c.s);
        cast_d2f(L.dinvAcm.p, L.dinvAcm32.p, L.n, c);
        cast_d2f(L.dinvAncm.p, L.dinvAncm32.p, L.m, c);
      }
    }
  }
  const int n = H.lv[0]->n;
  H.px.alloc(n, c.s); H.pr.alloc(n, c.s); H.pz.alloc(n, c.s); H.pp.alloc(n, c.s); H.pq.alloc(n, c.s);
  if (f32) H.pzold.alloc(n, c.s);
}

// ---------------------------------------------------------------------------
// PCG (FP64 vectors and inner products, device scalars)
// ---------------------------------------------------------------------------
// flags[0]: breakdown count; flags[3]: set by the update when any entry of x
// changed (cleared here, before the update of the same iteration)
__global__ void k_pcg_alpha(double* __restrict__ sc, unsigned long long* __restrict__ flags) {
  flags[3] = 0;
  const double pq = sc[P_PQ];
  if (!(pq > 0.0)) { flags[0] += 1; sc[P_ALPHA] = 0.0; return; }
  sc[P_ALPHA] = sc[P_RZ] / pq;
}
__global__ void __launch_bounds__(256) k_pcg_update(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* __restrict__ alpha, double* __restrict__ part,
                                                    unsigned long long* __restrict__ flags) {
  __shared__ double sh[4];
  const double a = *alpha;
  double s = 0.0;
  int changed = 0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const double xo = x[i], xn = xo + a * p[i];
    changed |= xn != xo;
    x[i] = xn;
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  double t = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
  // every block that changed an entry stores the same value
  if (__syncthreads_or(changed) && threadIdx.x == 0) flags[3] = 1;
}

// Extreme eigenvalues of the Lanczos matrix of the preconditioned operator
// that CG builds from its own coefficients (the CG-Lanczos relation): T is
// symmetric tridiagonal with T_00 = 1/alpha_0, T_jj = 1/alpha_j +
// beta_{j-1}/alpha_{j-1}, T_j,j+1 = sqrt(beta_j)/alpha_j.  Its extreme
// eigenvalues approach those of V A from inside; they are found by bisection
// on the Sturm count (the number of negative pivots of T - x I).
static void lanczos_extremes(const std::vector<double>& alpha, const std::vector<double>& beta, double* lmin,
                             double* lmax) {
  const size_t k = alpha.size();
  *lmin = *lmax = 0.0;
  if (k == 0) return;
  std::vector<double> d(k), e(k, 0.0);
  for (size_t j = 0; j < k; ++j) {
    d[j] = 1.0 / alpha[j] + (j > 0 ? beta[j - 1] / alpha[j - 1] : 0.0);
    if (j + 1 < k) e[j] = std::sqrt(std::max(beta[j], 0.0)) / alpha[j];
  }
  for (size_t j = 0; j < k; ++j)
    if (!std::isfinite(d[j]) || !std::isfinite(e[j])) return;
  double lo = d[0], hi = d[0];
  for (size_t j = 0; j < k; ++j) {
    const double rad = std::fabs(e[j]) + (j > 0 ? std::fabs(e[j - 1]) : 0.0);
    lo = std::min(lo, d[j] - rad);
    hi = std::max(hi, d[j] + rad);
  }
  auto below = [&](double x) {  // eigenvalues of T smaller than x
    size_t cnt = 0;
    double q = 1.0;
    for (size_t j = 0; j < k; ++j) {
      const double off = j > 0 ? e[j - 1] * e[j - 1] : 0.0;
      q = (d[j] - x) - (j > 0 ? off / q : 0.0);
      if (q == 0.0) q = -1e-300;
      cnt += q < 0.0;
    }
    return cnt;
  };
  auto bisect = [&](size_t target) {  // smallest x with below(x) >= target
    double a = lo, b = hi;
    for (int it = 0; it < 200 && b - a > 1e-15 * std::max(std::fabs(a), std::fabs(b)); ++it) {
      const double mid = 0.5 * (a + b);
      if (below(mid) >= target) b = mid; else a = mid;
    }
    return 0.5 * (a + b);
  };
  *lmin = bisect(1);
  *lmax = bisect(k);
}
// beta = <r,z> / rz (FP64 form) or (<r,z> - <r,zold>) / rz (flexible)
__global__ void k_pcg_beta(double* __restrict__ sc, int flexible) {
  const double rz = sc[P_RZ], rznew = sc[P_RZNEW];
  sc[P_BETA] = (flexible ? (rznew - sc[P_RZOLD]) : rznew) / rz;
  sc[P_RZ] = rznew;
}
__global__ void k_pcg_dir(int64_t n, double* __restrict__ p, const double* __restrict__ z, const double* __restrict__ beta) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = z[i] + *beta * p[i];
}
__global__ void k_sub(int64_t n, const double* __restrict__ a, double* __restrict__ b) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = a[i] - b[i];
}

int pcg_solve(Hierarchy& H, const double* f, double* u, double rtol, int maxit, int* iters, double* relres) {
  Ctx& c = H.ctx;
  Level& L = *H.lv[0];
  const int64_t n = L.n;
  const bool flex = H.fp32;
  double* sc = c.scal.p;
  // iscal[9] breakdown count, iscal[12] "x changed" (see k_pcg_alpha)
  unsigned long long* flags = (unsigned long long*)(c.iscal.p + 9);
  HC_HIP(hipMemsetAsync(flags, 0, 4 * sizeof(unsigned long long), c.s));
  H.pcg_alpha.clear();
  H.pcg_beta.clear();
  H.lanczos_min = H.lanczos_max = 0.0;
  H.stagnated = false;
  const int nbu = (int)std::min<int64_t>(Ctx::kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
  // x = 0, r = f, z = V(r), p = z
  fill(H.px.p, 0.0, n, c);
  d2d(H.pr.p, f, n, c);
  dot(f, f, n, sc + P_FF, c, 3);
  double ff = 0.0;
  d2h(&ff, sc + P_FF, 1, c);
  const double nf = std::sqrt(ff);
  int it = 0;
  double rel = 1.0;
  H.pcg_hist.assign(1, nf == 0.0 ? 0.0 : 1.0);
  if (nf == 0.0) {
    d2d(u, H.px.p, n, c);
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    c.sync();
    return HCURL_OK;
  }
  // profile 3: per-kernel events on every kSampleEvery-th iteration only; the
  // others run like an unprofiled solve (whole V-cycle graph, no events)
  const bool prof = c.profile;
  const bool sampled = prof && H.opts.profile == 3;
  constexpr int kSampleEvery = 16;
  struct Restore {
    Ctx& c;
    bool v;
    ~Restore() { c.profile = v; }
  } restore{c, prof};
  apply_vcycle(H, H.pr.p, H.pz.p);
  d2d(H.pp.p, H.pz.p, n, c);
  dot(H.pr.p, H.pz.p, n, sc + P_RZ, c, 3);
  while (it < maxit) {
    if (sampled) c.profile = it % kSampleEvery == 0;
    spmv(L.A, H.pp.p, H.pq.p, nullptr, 0, c, "pcg_spmv");
    dot(H.pp.p, H.pq.p, n, sc + P_PQ, c, 3);
    c.run("pcg_scalar", 0.0, [&] { k_pcg_alpha<<<1, 1, 0, c.s>>>(sc, flags); });
    c.run("pcg_update", 48.0 * n, [&] {
      k_pcg_update<<<nbu, 256, 0, c.s>>>(n, H.px.p, H.pr.p, H.pp.p, H.pq.p, sc + P_ALPHA, c.red.p + 4 * (size_t)Ctx::kRedBlocks,
                                         flags);
    });
    reduce_partials(nbu, 4, sc + P_RR, c);
    double scv[P_FF - P_RZ + 1];
    d2h(scv, sc + P_RZ, P_FF - P_RZ + 1, c);
    ++it;
    unsigned long long hf[4];
    d2h(hf, flags, 4, c);
    if (hf[0]) fail(HCURL_ENOTSPD, "PCG breakdown: <p, A p> <= 0");
    if (it > 1) H.pcg_beta.push_back(scv[P_BETA - P_RZ]);  // beta of the previous iteration
    H.pcg_alpha.push_back(scv[P_ALPHA - P_RZ]);
    rel = std::sqrt(scv[P_RR - P_RZ]) / nf;
    H.pcg_hist.push_back(rel);
    if (rel <= rtol) break;
    // the stagnation the paper reports for its hardest cases (Sec. 6.2): two
    // consecutive iterates equal in every entry
    if (!hf[3]) {
      H.stagnated = true;
      break;
    }
    if (flex) d2d(H.pzold.p, H.pz.p, n, c);
    apply_vcycle(H, H.pr.p, H.pz.p);
    dot(H.pr.p, H.pz.p, n, sc + P_RZNEW, c, 3);
    if (flex) dot(H.pr.p, H.pzold.p, n, sc + P_RZOLD, c, 5);
    c.run("pcg_scalar", 0.0, [&] { k_pcg_beta<<<1, 1, 0, c.s>>>(sc, flex ? 1 : 0); });
    c.run("pcg_dir", 24.0 * n, [&] { k_pcg_dir<<<ceil_div(n, 256), 256, 0, c.s>>>(n, H.pp.p, H.pz.p, sc + P_BETA); });
  }
  c.profile = prof;
  // true residual
  spmv(L.A, H.px.p, H.pq.p, f, 1, c, "pcg_spmv");
  dot(H.pq.p, H.pq.p, n, sc + P_RR, c, 3);
  double tr = 0.0;
  d2h(&tr, sc + P_RR, 1, c);
  d2d(u, H.px.p, n, c);
  c.sync();
  if (iters) *iters = it;
  if (relres) *relres = std::sqrt(tr) / nf;
  H.last_iters = it;
  H.last_relres = std::sqrt(tr) / nf;
  lanczos_extremes(H.pcg_alpha, H.pcg_beta, &H.lanczos_min, &H.lanczos_max);
  if (rel <= rtol) return HCURL_OK;
  return H.stagnated ? HCURL_ESTAGNATE : HCURL_EMAXIT;
}

}  // namespace hc
