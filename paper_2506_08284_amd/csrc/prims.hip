// Sparse and vector primitives: prefix sums, CSR transpose, hashed SpGEMM
// with symbolic patterns, SpMV, deterministic reductions.
#include "prims.hpp"

namespace hc {

// ---------------------------------------------------------------------------
// exclusive scan (three passes: block sums, scan of block sums, apply)
// ---------------------------------------------------------------------------
static constexpr int kScanThreads = 256;
static constexpr int kScanItems = 8;
static constexpr int kScanTile = kScanThreads * kScanItems;

__global__ void __launch_bounds__(256) k_scan_sums(const int* __restrict__ in, int64_t n, long long* __restrict__ bsum) {
  __shared__ long long sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + (int64_t)j * kScanThreads + threadIdx.x;
    if (i < n) s += in[i];
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) bsum[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ void __launch_bounds__(1024) k_scan_partials(long long* __restrict__ bsum, int nb, long long* __restrict__ total) {
  __shared__ long long sh[16];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int c0 = 0; c0 < nb; c0 += 1024) {
    int i = c0 + threadIdx.x;
    long long v = i < nb ? bsum[i] : 0;
    // inclusive scan in wave
    long long x = v;
    const int l = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      long long t = __shfl_up(x, o, 64);
      if (l >= o) x += t;
    }
    if (l == 63) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x < 16) {
      long long y = sh[threadIdx.x];
      for (int o = 1; o < 16; o <<= 1) {
        long long t = __shfl_up(y, o, 16);
        if ((int)threadIdx.x >= o) y += t;
      }
      sh[threadIdx.x] = y;
    }
    __syncthreads();
    long long woff = (threadIdx.x >> 6) ? sh[(threadIdx.x >> 6) - 1] : 0;
    long long excl = carry + woff + x - v;
    if (i < nb) bsum[i] = excl;
    __syncthreads();
    if (threadIdx.x == 1023) carry = excl + v;
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}

__global__ void __launch_bounds__(256) k_scan_apply(const int* __restrict__ in, int* __restrict__ out, int64_t n,
                                                    const long long* __restrict__ boff, const long long* __restrict__ total) {
  __shared__ long long sh[4];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  long long s = 0;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    v[j] = i < n ? in[i] : 0;
    s += v[j];
  }
  long long x = s;
  const int l = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    long long t = __shfl_up(x, o, 64);
    if (l >= o) x += t;
  }
  if (l == 63) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  long long woff = 0;
  for (int w = 0; w < (int)(threadIdx.x >> 6); ++w) woff += sh[w];
  long long run = boff[blockIdx.x] + woff + x - s;
#pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    int64_t i = base + j;
    if (i < n) out[i] = (int)run;
    run += v[j];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = (int)*total;
}

int64_t exclusive_scan(const int* in, int* out, int64_t n, Ctx& c) {
  if (n == 0) {
    int z = 0;
    HC_HIP(hipMemcpyAsync(out, &z, sizeof(int), hipMemcpyHostToDevice, c.s));
    HC_HIP(hipStreamSynchronize(c.s));
    return 0;
  }
  int nb = ceil_div(n, kScanTile);
  DBuf<long long> bsum(nb + 1, c.s);
  c.run("scan", 4.0 * n, [&] { k_scan_sums<<<nb, 256, 0, c.s>>>(in, n, bsum.p); });
  c.run("scan", 8.0 * nb, [&] { k_scan_partials<<<1, 1024, 0, c.s>>>(bsum.p, nb, bsum.p + nb); });
  long long total = 0;
  d2h(&total, bsum.p + nb, 1, c);
  if (total > 0x7fffffffLL) fail(HCURL_EUNSUPPORTED, "a matrix would exceed 2^31-1 nonzeros");
  c.run("scan", 8.0 * n, [&] { k_scan_apply<<<nb, 256, 0, c.s>>>(in, out, n, bsum.p, bsum.p + nb); });
  return total;
}

// ---------------------------------------------------------------------------
// upload / copy
// ---------------------------------------------------------------------------
__global__ void k_i64_to_i32(const int64_t* __restrict__ a, int* __restrict__ b, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (int)a[i];
}

// Caller CSR check: row pointers rise from 0 to nnz, columns lie in range and
// increase strictly within a row.
__global__ void k_check_csr(const int64_t* __restrict__ rp, const int* __restrict__ col, int64_t n, int64_t ncols,
                            int64_t nnz, int* __restrict__ bad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0 && (rp[0] != 0 || rp[n] != nnz)) atomicOr(bad, 1);
  if (i >= n) return;
  const int64_t a = rp[i], b = rp[i + 1];
  if (a < 0 || b < a || b > nnz) { atomicOr(bad, 1); return; }
  int prev = -1;
  for (int64_t k = a; k < b; ++k) {
    const int j = col[k];
    if (j <= prev || j >= ncols) { atomicOr(bad, 1); return; }
    prev = j;
  }
}

void upload_csr(const hcurl_csr& in, bool device_ptrs, Csr& out, bool values, Ctx& c) {
  if (in.nrows < 0 || in.ncols < 0 || in.nnz < 0 || in.nnz > 0x7fffffffLL || in.nrows > 0x7fffffffLL)
    fail(HCURL_EINVAL, "CSR sizes out of range");
  if (!in.rowptr || (in.nnz && !in.col) || (values && in.nnz && !in.val)) fail(HCURL_EINVAL, "CSR pointer is NULL");
  out.nrows = (int)in.nrows;
  out.ncols = (int)in.ncols;
  out.nnz = in.nnz;
  out.rowptr.alloc(in.nrows + 1, c.s);
  out.col.alloc(in.nnz, c.s);
  if (values) out.val.alloc(in.nnz, c.s);
  DBuf<int64_t> rp(in.nrows + 1, c.s);
  auto kind = device_ptrs ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
  HC_HIP(hipMemcpyAsync(rp.p, in.rowptr, (in.nrows + 1) * sizeof(int64_t), kind, c.s));
  if (in.nnz) HC_HIP(hipMemcpyAsync(out.col.p, in.col, in.nnz * sizeof(int), kind, c.s));
  if (values && in.nnz) HC_HIP(hipMemcpyAsync(out.val.p, in.val, in.nnz * sizeof(double), kind, c.s));
  {
    DBuf<int> bad(1, c.s);
    HC_HIP(hipMemsetAsync(bad.p, 0, sizeof(int), c.s));
    k_check_csr<<<ceil_div(in.nrows + 1, 256), 256, 0, c.s>>>(rp.p, out.col.p, in.nrows, in.ncols, in.nnz, bad.p);
    HC_LAUNCH_CHECK();
    int hb = 0;
    d2h(&hb, bad.p, 1, c);
    if (hb)
      fail(HCURL_EINVAL, "malformed CSR: row pointers must rise from 0 to nnz and column indices must lie in "
                         "[0, ncols) and increase within each row");
  }
  int64_t n1 = in.nrows + 1;
  k_i64_to_i32<<<ceil_div(n1, 256), 256, 0, c.s>>>(rp.p, out.rowptr.p, n1);
  HC_LAUNCH_CHECK();
  HC_HIP(hipStreamSynchronize(c.s));
}

void copy_csr(const Csr& A, Csr& B, Ctx& c) {
  B.nrows = A.nrows; B.ncols = A.ncols; B.nnz = A.nnz;
  B.rowptr.alloc(A.nrows + 1, c.s);
  B.col.alloc(A.nnz, c.s);
  d2d(B.rowptr.p, A.rowptr.p, A.nrows + 1, c);
  d2d(B.col.p, A.col.p, A.nnz, c);
  if (A.val.p) { B.val.alloc(A.nnz, c.s); d2d(B.val.p, A.val.p, A.nnz, c); }
}

// ---------------------------------------------------------------------------
// transpose: count, scan, scatter with cursors, then sort every output row
// ---------------------------------------------------------------------------
// One wave takes 64 consecutive rows and walks their entries slot by slot;
// the lanes whose rows hold the same column in a slot share one atomic (the
// rows of a mesh operator's neighbourhood repeat each other's columns).
// Positions inside an output row are in no particular order: sort_rows
// orders them.
template <bool SCATTER>
__global__ void __launch_bounds__(256) k_transpose_pass(const int* __restrict__ rowptr, const int* __restrict__ col,
                                                        const double* __restrict__ val, int nrows,
                                                        int* __restrict__ cursor, int* __restrict__ tcol,
                                                        double* __restrict__ tval) {
  const int i = (int)((int64_t)blockIdx.x * blockDim.x + threadIdx.x);
  const int l = threadIdx.x & 63;
  const int a = i < nrows ? rowptr[i] : 0, len = i < nrows ? rowptr[i + 1] - a : 0;
  int maxlen = len;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) maxlen = max(maxlen, __shfl_xor(maxlen, o, 64));
  for (int j = 0; j < maxlen; ++j) {
    const int c = j < len ? col[a + j] : -1;
    unsigned long long todo = __ballot(c >= 0);
    int pos = 0;
    while (todo) {
      const int leader = __ffsll((long long)todo) - 1;
      const int cc = __shfl(c, leader, 64);
      const unsigned long long m = __ballot(c == cc);
      if (SCATTER) {
        int base = 0;
        if (l == leader) base = atomicAdd(&cursor[cc], __popcll(m));
        base = __shfl(base, leader, 64);
        if (c == cc) pos = base + __popcll(m & ((1ull << l) - 1ull));
      } else if (l == leader) {
        atomicAdd(&cursor[cc], __popcll(m));
      }
      todo &= ~m;
    }
    if (SCATTER && c >= 0) {
      tcol[pos] = i;
      if (val) tval[pos] = val[a + j];
    }
  }
}

// Sorts the column indices (unique within a row) of every row, carrying
// values, by rank counting in LDS: one wave per row, rows up to kSortCap.
// Longer rows are listed in long_rows (count in *n_long) for k_sort_rows_wg.
static constexpr int kSortCap = 1024;
__global__ void __launch_bounds__(64) k_sort_rows(const int* __restrict__ rowptr, int nrows, int* __restrict__ col,
                                                  double* __restrict__ val, int* __restrict__ n_long,
                                                  int* __restrict__ long_rows) {
  __shared__ int kk[kSortCap];
  __shared__ double vv[kSortCap];
  for (int i = blockIdx.x; i < nrows; i += gridDim.x) {
    const int a = rowptr[i], len = rowptr[i + 1] - a;
    if (len <= 1) continue;
    if (len > kSortCap) {
      if (threadIdx.x == 0) long_rows[atomicAdd(n_long, 1)] = i;
      continue;
    }
    for (int t = threadIdx.x; t < len; t += 64) {
      kk[t] = col[a + t];
      if (val) vv[t] = val[a + t];
    }
    __syncthreads();
    // up to four keys per lane ranked in one pass over the row
    for (int t0 = threadIdx.x; t0 < len; t0 += 256) {
      int key[4], r[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        key[j] = t0 + 64 * j < len ? kk[t0 + 64 * j] : 0x7fffffff;
        r[j] = 0;
      }
      for (int u = 0; u < len; ++u) {
        const int kv = kk[u];
#pragma unroll
        for (int j = 0; j < 4; ++j) r[j] += kv < key[j];
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int t = t0 + 64 * j;
        if (t < len) {
          col[a + r[j]] = key[j];
          if (val) val[a + r[j]] = vv[t];
        }
      }
    }
    __syncthreads();
  }
}

// Rows longer than kSortCap, one workgroup per listed row.  Every thread
// takes kLongPer of the row's entries at a time and ranks them against the
// whole row, staged through LDS in chunks of kLongChunk keys; entries go to
// their ranks in tcol/tval (same offsets as col), and after a barrier the
// row is copied back.  The row is only read before the barrier and only
// written after it.
static constexpr int kLongPer = 8;
static constexpr int kLongChunk = 8192;
__global__ void __launch_bounds__(1024) k_sort_rows_wg(const int* __restrict__ rowptr, const int* __restrict__ long_rows,
                                                       int* __restrict__ col, double* __restrict__ val,
                                                       int* __restrict__ tcol, double* __restrict__ tval) {
  __shared__ int sk[kLongChunk];
  const int i = long_rows[blockIdx.x];
  const int a = rowptr[i], len = rowptr[i + 1] - a;
  const int tid = threadIdx.x;
  for (int base = 0; base < len; base += 1024 * kLongPer) {
    int key[kLongPer], rk[kLongPer];
#pragma unroll
    for (int u = 0; u < kLongPer; ++u) {
      const int t = base + u * 1024 + tid;
      key[u] = t < len ? col[a + t] : 0x7fffffff;
      rk[u] = 0;
    }
    for (int c0 = 0; c0 < len; c0 += kLongChunk) {
      const int nc = min(kLongChunk, len - c0);
      __syncthreads();  // the previous chunk has been consumed
      for (int t = tid; t < nc; t += 1024) sk[t] = col[a + c0 + t];
      __syncthreads();
      for (int v = 0; v < nc; ++v) {
        const int kv = sk[v];
#pragma unroll
        for (int u = 0; u < kLongPer; ++u) rk[u] += kv < key[u];
      }
    }
#pragma unroll
    for (int u = 0; u < kLongPer; ++u) {
      const int t = base + u * 1024 + tid;
      if (t < len) {
        tcol[a + rk[u]] = key[u];
        if (val) tval[a + rk[u]] = val[a + t];
      }
    }
  }
  __syncthreads();
  for (int t = tid; t < len; t += 1024) {
    col[a + t] = tcol[a + t];
    if (val) val[a + t] = tval[a + t];
  }
}

static void sort_rows(Csr& C, Ctx& c) {
  if (C.nrows == 0 || C.nnz == 0) return;
  long long* flag = c.iscal.p + 0;
  HC_HIP(hipMemsetAsync(flag, 0, sizeof(long long), c.s));
  // at most nnz / (kSortCap + 1) rows are longer than kSortCap
  DBuf<int> long_rows(C.nnz / (kSortCap + 1) + 1, c.s);
  int nb = std::min(C.nrows, 65536);
  c.run("sort_rows", 16.0 * C.nnz,
        [&] { k_sort_rows<<<nb, 64, 0, c.s>>>(C.rowptr.p, C.nrows, C.col.p, C.val.p, (int*)flag, long_rows.p); });
  long long h = 0;
  d2h(&h, flag, 1, c);
  const int nlong = (int)h;
  if (nlong > 0) {
    DBuf<int> tcol(C.nnz, c.s);
    DBuf<double> tval(C.val.p ? C.nnz : 0, c.s);
    c.run("sort_rows_long", 32.0 * C.nnz, [&] {
      k_sort_rows_wg<<<nlong, 1024, 0, c.s>>>(C.rowptr.p, long_rows.p, C.col.p, C.val.p, tcol.p, tval.p);
    });
  }
}

void transpose(const Csr& A, Csr& AT, bool values, Ctx& c) {
  values = values && A.val.p;
  AT.nrows = A.ncols;
  AT.ncols = A.nrows;
  AT.nnz = A.nnz;
  AT.rowptr.alloc(AT.nrows + 1, c.s);
  AT.col.alloc(A.nnz, c.s);
  if (values) AT.val.alloc(A.nnz, c.s); else AT.val.release();
  DBuf<int> cnt(AT.nrows + 1, c.s);
  HC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (AT.nrows + 1), c.s));
  if (A.nnz)
    c.run("transpose", 8.0 * A.nnz, [&] {
      k_transpose_pass<false><<<ceil_div(A.nrows, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, nullptr, A.nrows, cnt.p,
                                                                     nullptr, nullptr);
    });
  exclusive_scan(cnt.p, AT.rowptr.p, AT.nrows, c);
  d2d(cnt.p, AT.rowptr.p, AT.nrows, c);
  if (A.nrows)
    c.run("transpose", 24.0 * A.nnz, [&] {
      k_transpose_pass<true><<<ceil_div(A.nrows, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, values ? A.val.p : nullptr,
                                                                    A.nrows, cnt.p, AT.col.p,
                                                                    values ? AT.val.p : nullptr);
    });
  sort_rows(AT, c);
}

// AT's values from A on AT's kept pattern: entry (j, i) of AT is A(i, j),
// found by a binary search of column j in row i of A (sorted columns).  One
// wave per row of AT.
__global__ void __launch_bounds__(256) k_transpose_values(int nT, const int* __restrict__ Trp,
                                                          const int* __restrict__ Tcol, double* __restrict__ Tval,
                                                          const int* __restrict__ Arp, const int* __restrict__ Acol,
                                                          const double* __restrict__ Aval) {
  const int j = (int)(((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6);
  if (j >= nT) return;
  for (int q = Trp[j] + lane_id(); q < Trp[j + 1]; q += 64) {
    const int i = Tcol[q];
    int lo = Arp[i], hi = Arp[i + 1] - 1;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (Acol[mid] < j) lo = mid + 1; else hi = mid;
    }
    Tval[q] = Aval[lo];
  }
}

void transpose_refill(const Csr& A, Csr& AT, Ctx& c) {
  if (AT.nrows != A.ncols || AT.ncols != A.nrows || AT.nnz != A.nnz || !A.val.p || !AT.rowptr.p)
    fail(HCURL_EINVAL, "transpose_refill: the kept transpose does not match");
  if (AT.val.n < (size_t)AT.nnz) AT.val.alloc(AT.nnz, c.s);
  if (AT.nrows && AT.nnz)
    c.run("transpose_values", 36.0 * A.nnz, [&] {
      k_transpose_values<<<ceil_div(AT.nrows, 4), 256, 0, c.s>>>(AT.nrows, AT.rowptr.p, AT.col.p, AT.val.p, A.rowptr.p,
                                                                 A.col.p, A.val.p);
    });
}

// ---------------------------------------------------------------------------
// SpGEMM: one wave per row; the products of a row are flattened over 64
// lanes (prefix sum of the B-row lengths of each chunk of 64 A entries) and
// inserted into an LDS open-addressing hash table (symbolic pattern: every
// product inserts its column whatever its value).  Overflowing rows are
// redone with a larger table; the fill pass ranks the unique columns to
// write them sorted.
// ---------------------------------------------------------------------------
template <int HT>
struct HashWave {
  int keys[HT];
  double vals[HT];
  int ck[HT * 3 / 4];
  double cv[HT * 3 / 4];
  int kst[64];
  int pre[64];
  double av[64];
  int count;
  int overflow;
};

__device__ __forceinline__ unsigned hash_slot(int key, unsigned mask) {
  return ((unsigned)key * 2654435761u) & mask;
}

// Inserts all products of row i; returns unique count or -1 on overflow.
template <int HT, bool NUMERIC>
__device__ int hash_row(HashWave<HT>& H, int i, const int* __restrict__ Arp, const int* __restrict__ Acol,
                        const double* __restrict__ Aval, const int* __restrict__ Brp, const int* __restrict__ Bcol,
                        const double* __restrict__ Bval) {
  const int l = lane_id();
  constexpr int CAP = HT * 3 / 4;
  for (int s = l; s < HT; s += 64) {
    H.keys[s] = -1;
    if (NUMERIC) H.vals[s] = 0.0;
  }
  if (l == 0) { H.count = 0; H.overflow = 0; }
  __syncthreads();
  const int a0 = Arp[i], a1 = Arp[i + 1];
  for (int c0 = a0; c0 < a1; c0 += 64) {
    const int j = c0 + l;
    int k = 0, st = 0, len = 0;
    double a = 0.0;
    if (j < a1) {
      k = Acol[j];
      if (NUMERIC) a = Aval[j];
      st = Brp[k];
      len = Brp[k + 1] - st;
    }
    const int incl = wave_incl_scan(len);
    const int total = __shfl(incl, 63, 64);
    H.kst[l] = st;
    H.pre[l] = incl - len;
    H.av[l] = a;
    __syncthreads();
    for (int p = l; p < total; p += 64) {
      // largest q with pre[q] <= p
      int lo = 0, hi = 63;
      while (lo < hi) {
        int mid = (lo + hi + 1) >> 1;
        if (H.pre[mid] <= p) lo = mid; else hi = mid - 1;
      }
      const int q = lo;
      const int pos = H.kst[q] + (p - H.pre[q]);
      const int key = Bcol[pos];
      unsigned h = hash_slot(key, HT - 1);
      int slot = -1;
      for (int probe = 0; probe < HT; ++probe) {
        int old = atomicCAS(&H.keys[h], -1, key);
        if (old == -1) {
          int cnt = atomicAdd(&H.count, 1);
          if (cnt >= CAP) H.overflow = 1;
          slot = (int)h;
          break;
        }
        if (old == key) { slot = (int)h; break; }
        h = (h + 1) & (HT - 1);
      }
      if (slot < 0) { H.overflow = 1; continue; }
      if (NUMERIC) atomicAdd(&H.vals[slot], H.av[q] * Bval[pos]);
    }
    __syncthreads();
    if (H.overflow) break;
  }
  __syncthreads();
  return H.overflow ? -1 : H.count;
}

template <int HT>
__global__ void __launch_bounds__(64) k_spgemm_count(const int* __restrict__ rows, int nrows_list, int nrows,
                                                     const int* __restrict__ Arp, const int* __restrict__ Acol,
                                                     const int* __restrict__ Brp, const int* __restrict__ Bcol,
                                                     int* __restrict__ cnt) {
  __shared__ HashWave<HT> H;
  const int n = rows ? nrows_list : nrows;
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const int i = rows ? rows[t] : t;
    int u = hash_row<HT, false>(H, i, Arp, Acol, nullptr, Brp, Bcol, nullptr);
    if (lane_id() == 0) cnt[i] = u;
    __syncthreads();
  }
}

template <int HT, bool NUMERIC>
__global__ void __launch_bounds__(64) k_spgemm_fill(const int* __restrict__ rows, int nrows_list, int nrows,
                                                    const int* __restrict__ Arp, const int* __restrict__ Acol,
                                                    const double* __restrict__ Aval, const int* __restrict__ Brp,
                                                    const int* __restrict__ Bcol, const double* __restrict__ Bval,
                                                    const int* __restrict__ Crp, int* __restrict__ Ccol,
                                                    double* __restrict__ Cval) {
  __shared__ HashWave<HT> H;
  const int n = rows ? nrows_list : nrows;
  const int l = lane_id();
  for (int t = blockIdx.x; t < n; t += gridDim.x) {
    const int i = rows ? rows[t] : t;
    int u = hash_row<HT, NUMERIC>(H, i, Arp, Acol, Aval, Brp, Bcol, Bval);
    if (u < 0) continue;  // an overflowing row: the large table's pass writes it
    // compact occupied slots
    int base = 0;
    for (int s0 = 0; s0 < HT; s0 += 64) {
      const int s = s0 + l;
      const bool occ = H.keys[s] >= 0;
      const int incl = wave_incl_scan(occ ? 1 : 0);
      if (occ) {
        H.ck[base + incl - 1] = H.keys[s];
        if (NUMERIC) H.cv[base + incl - 1] = H.vals[s];
      }
      base += __shfl(incl, 63, 64);
    }
    __syncthreads();
    const int off = Crp[i];
    for (int t2 = l; t2 < u; t2 += 64) {
      const int key = H.ck[t2];
      int r = 0;
      for (int v = 0; v < u; ++v) r += H.ck[v] < key;
      Ccol[off + r] = key;
      if (NUMERIC) Cval[off + r] = H.cv[t2];
    }
    __syncthreads();
  }
}

__global__ void k_collect_overflow(const int* __restrict__ cnt, int n, int* __restrict__ list, int* __restrict__ nlist) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && cnt[i] < 0) list[atomicAdd(nlist, 1)] = i;
}

// Short rows: when every row of A has at most 64 entries and at most 64
// products, one wave handles a row with one product per lane.  The (column,
// value) pairs are sorted over the wave by a bitonic network of lane
// exchanges and equal columns are summed by a segmented scan, so no LDS table
// is cleared or compacted per row and the sums run in a fixed order.
__global__ void k_row_products(int nrows, const int* __restrict__ Arp, const int* __restrict__ Acol,
                               const int* __restrict__ Brp, unsigned long long* __restrict__ maxes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int prod = 0, len = 0;
  if (i < nrows) {
    const int a = Arp[i], e = Arp[i + 1];
    len = e - a;
    for (int q = a; q < e; ++q) {
      const int k = Acol[q];
      prod += Brp[k + 1] - Brp[k];
    }
  }
  const int m = max(prod, len);
  // one atomic per wave
  int w = m;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) w = max(w, __shfl_xor(w, o, 64));
  if ((threadIdx.x & 63) == 0 && w > 0) atomicMax(maxes, (unsigned long long)w);
}

template <bool FILL, bool NUMERIC>
__global__ void __launch_bounds__(256) k_spgemm_wave(int nrows, const int* __restrict__ Arp, const int* __restrict__ Acol,
                                                     const double* __restrict__ Aval, const int* __restrict__ Brp,
                                                     const int* __restrict__ Bcol, const double* __restrict__ Bval,
                                                     int* __restrict__ cnt, const int* __restrict__ Crp,
                                                     int* __restrict__ Ccol, double* __restrict__ Cval) {
  const int l = threadIdx.x & 63;
  const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= nrows) return;  // whole waves leave together
  const int a0 = Arp[i], na = Arp[i + 1] - a0;  // na <= 64
  int st = 0, len = 0;
  double av = 0.0;
  if (l < na) {
    const int k = Acol[a0 + l];
    if (NUMERIC) av = Aval[a0 + l];
    st = Brp[k];
    len = Brp[k + 1] - st;
  }
  const int incl = wave_incl_scan(len);
  const int total = __shfl(incl, 63, 64);  // <= 64
  const int pre = incl - len;
  // owner of product l: the last lane q with pre[q] <= l (six halvings of 0..63)
  int lo = 0, hi = 63;
#pragma unroll
  for (int it = 0; it < 6; ++it) {
    const int mid = (lo + hi + 1) >> 1;
    const int pm = __shfl(pre, mid, 64);
    if (pm <= l) lo = mid; else hi = mid - 1;
  }
  const int stq = __shfl(st, lo, 64), preq = __shfl(pre, lo, 64);
  const double aq = __shfl(av, lo, 64);
  int key = 0x7fffffff;
  double v = 0.0;
  if (l < total) {
    const int pos = stq + (l - preq);
    key = Bcol[pos];
    if (NUMERIC) v = aq * Bval[pos];
  }
  // bitonic sort of (key, v) ascending over the 64 lanes
#pragma unroll
  for (int size = 2; size <= 64; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      const int pk = __shfl_xor(key, stride, 64);
      const double pv = NUMERIC ? __shfl_xor(v, stride, 64) : 0.0;
      const bool asc = (l & size) == 0;
      const bool lower = (l & stride) == 0;
      const bool take = (lower == asc) ? (pk < key) : (pk > key);
      if (take) { key = pk; v = pv; }
    }
  }
  // sum equal keys (contiguous after the sort): segmented inclusive scan
  if (NUMERIC) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int pk = __shfl_up(key, o, 64);
      const double pv = __shfl_up(v, o, 64);
      if (l >= o && pk == key) v += pv;
    }
  }
  const int nk = __shfl_down(key, 1, 64);
  const bool tail = key != 0x7fffffff && (l == 63 || nk != key);
  const unsigned long long tails = __ballot(tail);
  if (!FILL) {
    if (l == 0) cnt[i] = __popcll(tails);
    return;
  }
  if (tail) {
    const int r = Crp[i] + __popcll(tails & ((1ull << l) - 1ull));
    Ccol[r] = key;
    if (NUMERIC) Cval[r] = v;
  }
}

static constexpr int kHtSmall = 512;
static constexpr int kHtLarge = 2048;

// C = D B for a D whose rows hold at most two entries, each +-1 (a discrete
// gradient): row i of C is the signed merge of at most two sorted rows of B,
// a shared column summing the two products (one addition, whose order does not
// matter), a lone column keeping its product.  The same pattern (structural
// zeros kept) and values as spgemm; one thread per row.  A row of D outside
// that form sets *bad, and the caller falls back to spgemm.
template <bool FILL>
__global__ void k_grad_rows(int n, const int* __restrict__ Drp, const int* __restrict__ Dcol,
                            const double* __restrict__ Dval, const int* __restrict__ Brp, const int* __restrict__ Bcol,
                            const double* __restrict__ Bval, int* __restrict__ cnt, const int* __restrict__ Crp,
                            int* __restrict__ Ccol, double* __restrict__ Cval, int* __restrict__ bad) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d0 = Drp[i], nd = Drp[i + 1] - d0;
  int r0 = 0, r1 = 0;
  double s0 = 0.0, s1 = 0.0;
  if (nd >= 1) { r0 = Dcol[d0]; s0 = Dval[d0]; }
  if (nd >= 2) { r1 = Dcol[d0 + 1]; s1 = Dval[d0 + 1]; }
  if (!FILL && (nd > 2 || (nd >= 1 && fabs(s0) != 1.0) || (nd == 2 && (fabs(s1) != 1.0 || r1 <= r0)))) {
    atomicOr(bad, 1);
    cnt[i] = 0;
    return;
  }
  int p = nd >= 1 ? Brp[r0] : 0, pe = nd >= 1 ? Brp[r0 + 1] : 0;
  int q = nd >= 2 ? Brp[r1] : 0, qe = nd >= 2 ? Brp[r1 + 1] : 0;
  int w = FILL ? Crp[i] : 0, m = 0;
  while (p < pe || q < qe) {
    const int cp = p < pe ? Bcol[p] : 0x7fffffff, cq = q < qe ? Bcol[q] : 0x7fffffff;
    const int cmin = cp < cq ? cp : cq;
    if (FILL) {
      double v;
      if (cp == cq) v = s0 * Bval[p] + s1 * Bval[q];
      else if (cp < cq) v = s0 * Bval[p];
      else v = s1 * Bval[q];
      Ccol[w] = cmin;
      Cval[w] = v;
      ++w;
    }
    ++m;
    if (cp == cmin) ++p;
    if (cq == cmin) ++q;
  }
  if (!FILL) cnt[i] = m;
}

void gradient_product(const Csr& D, const Csr& B, Csr& C, Ctx& c, const char* tag) {
  if (D.ncols != B.nrows) fail(HCURL_EINVAL, "gradient_product: inner dimensions differ");
  if (!D.val.p || !B.val.p) {
    spgemm(D, B, C, true, c, tag);
    return;
  }
  C.nrows = D.nrows;
  C.ncols = B.ncols;
  C.rowptr.alloc(C.nrows + 1, c.s);
  DBuf<int> cnt(C.nrows + 1, c.s);
  int* bad = (int*)(c.iscal.p + 15);  // a slot no other primitive uses
  HC_HIP(hipMemsetAsync(bad, 0, sizeof(int), c.s));
  const std::string t = tag ? std::string(tag) : std::string("gradient_product");
  const int nb = ceil_div(std::max(C.nrows, 1), 256);
  if (C.nrows)
    c.run((t + "_sym").c_str(), 20.0 * D.nrows + 4.0 * B.nnz, [&] {
      k_grad_rows<false><<<nb, 256, 0, c.s>>>(C.nrows, D.rowptr.p, D.col.p, D.val.p, B.rowptr.p, B.col.p, B.val.p, cnt.p,
                                             nullptr, nullptr, nullptr, bad);
    });
  int hbad = 0;
  d2h(&hbad, bad, 1, c);
  if (hbad) {
    spgemm(D, B, C, true, c, tag);
    return;
  }
  C.nnz = exclusive_scan(cnt.p, C.rowptr.p, C.nrows, c);
  C.col.alloc(C.nnz, c.s);
  C.val.alloc(C.nnz, c.s);
  if (C.nrows)
    c.run((t + "_num").c_str(), 20.0 * D.nrows + 12.0 * C.nnz, [&] {
      k_grad_rows<true><<<nb, 256, 0, c.s>>>(C.nrows, D.rowptr.p, D.col.p, D.val.p, B.rowptr.p, B.col.p, B.val.p, nullptr,
                                            C.rowptr.p, C.col.p, C.val.p, bad);
    });
}

void spgemm(const Csr& A, const Csr& B, Csr& C, bool numeric, Ctx& c, const char* tag) {
  if (A.ncols != B.nrows) fail(HCURL_EINVAL, "spgemm: inner dimensions differ");
  numeric = numeric && A.val.p && B.val.p;
  C.nrows = A.nrows;
  C.ncols = B.ncols;
  C.rowptr.alloc(C.nrows + 1, c.s);
  DBuf<int> cnt(C.nrows + 1, c.s);
  if (C.nrows) {
    // short rows everywhere: the wave-sort path
    unsigned long long* mx = (unsigned long long*)(c.iscal.p + 11);
    HC_HIP(hipMemsetAsync(mx, 0, sizeof(unsigned long long), c.s));
    k_row_products<<<ceil_div(A.nrows, 256), 256, 0, c.s>>>(A.nrows, A.rowptr.p, A.col.p, B.rowptr.p, mx);
    HC_LAUNCH_CHECK();
    unsigned long long hmax = 0;
    d2h(&hmax, mx, 1, c);
    if (hmax <= 64) {
      const int nb = ceil_div(C.nrows, 4);
      const std::string t = tag ? std::string(tag) : std::string("spgemm");
      c.run((t + "_sym").c_str(), 12.0 * A.nnz, [&] {
        k_spgemm_wave<false, false><<<nb, 256, 0, c.s>>>(C.nrows, A.rowptr.p, A.col.p, nullptr, B.rowptr.p, B.col.p, nullptr,
                                                         cnt.p, nullptr, nullptr, nullptr);
      });
      C.nnz = exclusive_scan(cnt.p, C.rowptr.p, C.nrows, c);
      C.col.alloc(C.nnz, c.s);
      if (numeric) C.val.alloc(C.nnz, c.s); else C.val.release();
      c.run((t + "_num").c_str(), 12.0 * A.nnz + 12.0 * C.nnz, [&] {
        if (numeric)
          k_spgemm_wave<true, true><<<nb, 256, 0, c.s>>>(C.nrows, A.rowptr.p, A.col.p, A.val.p, B.rowptr.p, B.col.p, B.val.p,
                                                         nullptr, C.rowptr.p, C.col.p, C.val.p);
        else
          k_spgemm_wave<true, false><<<nb, 256, 0, c.s>>>(C.nrows, A.rowptr.p, A.col.p, nullptr, B.rowptr.p, B.col.p, nullptr,
                                                          nullptr, C.rowptr.p, C.col.p, nullptr);
      });
      return;
    }
  }
  const int nb = std::max(1, std::min(C.nrows, 1 << 17));
  const double est_bytes = 12.0 * A.nnz + 8.0 * B.nnz;
  if (C.nrows)
    c.run(tag ? (std::string(tag) + "_sym").c_str() : "spgemm_symbolic", est_bytes, [&] {
      k_spgemm_count<kHtSmall><<<nb, 64, 0, c.s>>>(nullptr, 0, A.nrows, A.rowptr.p, A.col.p, B.rowptr.p, B.col.p, cnt.p);
    });
  // rows that overflowed the small table
  DBuf<int> olist(C.nrows + 1, c.s);
  int* nover = (int*)(c.iscal.p + 1);
  HC_HIP(hipMemsetAsync(nover, 0, sizeof(int), c.s));
  if (C.nrows) {
    k_collect_overflow<<<ceil_div(C.nrows, 256), 256, 0, c.s>>>(cnt.p, C.nrows, olist.p, nover);
    HC_LAUNCH_CHECK();
  }
  int hover = 0;
  d2h(&hover, nover, 1, c);
  if (hover > 0) {
    c.run("spgemm_symbolic_large", est_bytes, [&] {
      k_spgemm_count<kHtLarge><<<std::min(hover, 65536), 64, 0, c.s>>>(olist.p, hover, A.nrows, A.rowptr.p, A.col.p,
                                                                        B.rowptr.p, B.col.p, cnt.p);
    });
    std::vector<int> hc_(C.nrows);
    d2h(hc_.data(), cnt.p, C.nrows, c);
    for (int v : hc_)
      if (v < 0) fail(HCURL_EUNSUPPORTED, "spgemm: a product row has more than 1536 nonzeros");
  }
  C.nnz = exclusive_scan(cnt.p, C.rowptr.p, C.nrows, c);
  C.col.alloc(C.nnz, c.s);
  if (numeric) C.val.alloc(C.nnz, c.s); else C.val.release();
  if (C.nrows) {
    if (numeric)
      c.run(tag ? (std::string(tag) + "_num").c_str() : "spgemm_numeric", est_bytes + 12.0 * C.nnz, [&] {
        k_spgemm_fill<kHtSmall, true><<<nb, 64, 0, c.s>>>(nullptr, 0, A.nrows, A.rowptr.p, A.col.p, A.val.p, B.rowptr.p,
                                                          B.col.p, B.val.p, C.rowptr.p, C.col.p, C.val.p);
      });
    else
      c.run("spgemm_numeric", est_bytes + 4.0 * C.nnz, [&] {
        k_spgemm_fill<kHtSmall, false><<<nb, 64, 0, c.s>>>(nullptr, 0, A.nrows, A.rowptr.p, A.col.p, nullptr,
                                                           B.rowptr.p, B.col.p, nullptr, C.rowptr.p, C.col.p, nullptr);
      });
    if (hover > 0) {
      if (numeric)
        c.run("spgemm_numeric_large", est_bytes, [&] {
          k_spgemm_fill<kHtLarge, true><<<std::min(hover, 65536), 64, 0, c.s>>>(
              olist.p, hover, A.nrows, A.rowptr.p, A.col.p, A.val.p, B.rowptr.p, B.col.p, B.val.p, C.rowptr.p, C.col.p,
              C.val.p);
        });
      else
        c.run("spgemm_numeric_large", est_bytes, [&] {
          k_spgemm_fill<kHtLarge, false><<<std::min(hover, 65536), 64, 0, c.s>>>(
              olist.p, hover, A.nrows, A.rowptr.p, A.col.p, nullptr, B.rowptr.p, B.col.p, nullptr, C.rowptr.p, C.col.p,
              nullptr);
        });
    }
  }
}

// Rows whose product has more distinct columns than the small table holds
// (hash_row overflows exactly then), from the product's row pointers.
__global__ void k_rows_longer(const int* __restrict__ rp, int n, int limit, int* __restrict__ list,
                              int* __restrict__ nlist) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && rp[i + 1] - rp[i] > limit) list[atomicAdd(nlist, 1)] = i;
}

void spgemm_refill(const Csr& A, const Csr& B, Csr& C, Ctx& c, const char* tag) {
  if (A.ncols != B.nrows || C.nrows != A.nrows || C.ncols != B.ncols || !A.val.p || !B.val.p)
    fail(HCURL_EINVAL, "spgemm_refill: operands do not match the kept product");
  if (!C.nrows) return;
  if (C.col.n < (size_t)C.nnz) C.col.alloc(C.nnz, c.s);
  if (C.val.n < (size_t)C.nnz) C.val.alloc(C.nnz, c.s);
  const std::string t = std::string(tag ? tag : "spgemm") + "_num";
  unsigned long long* mx = (unsigned long long*)(c.iscal.p + 11);
  HC_HIP(hipMemsetAsync(mx, 0, sizeof(unsigned long long), c.s));
  k_row_products<<<ceil_div(A.nrows, 256), 256, 0, c.s>>>(A.nrows, A.rowptr.p, A.col.p, B.rowptr.p, mx);
  HC_LAUNCH_CHECK();
  unsigned long long hmax = 0;
  d2h(&hmax, mx, 1, c);
  if (hmax <= 64) {
    c.run(t.c_str(), 12.0 * A.nnz + 12.0 * C.nnz, [&] {
      k_spgemm_wave<true, true><<<ceil_div(C.nrows, 4), 256, 0, c.s>>>(C.nrows, A.rowptr.p, A.col.p, A.val.p, B.rowptr.p,
                                                                       B.col.p, B.val.p, nullptr, C.rowptr.p, C.col.p,
                                                                       C.val.p);
    });
    return;
  }
  const int nb = std::max(1, std::min(C.nrows, 1 << 17));
  const double est_bytes = 12.0 * A.nnz + 8.0 * B.nnz;
  c.run(t.c_str(), est_bytes + 12.0 * C.nnz, [&] {
    k_spgemm_fill<kHtSmall, true><<<nb, 64, 0, c.s>>>(nullptr, 0, A.nrows, A.rowptr.p, A.col.p, A.val.p, B.rowptr.p,
                                                      B.col.p, B.val.p, C.rowptr.p, C.col.p, C.val.p);
  });
  DBuf<int> olist(C.nrows, c.s);
  int* nover = (int*)(c.iscal.p + 1);
  HC_HIP(hipMemsetAsync(nover, 0, sizeof(int), c.s));
  k_rows_longer<<<ceil_div(C.nrows, 256), 256, 0, c.s>>>(C.rowptr.p, C.nrows, kHtSmall * 3 / 4, olist.p, nover);
  HC_LAUNCH_CHECK();
  int hover = 0;
  d2h(&hover, nover, 1, c);
  if (hover > 0)
    c.run("spgemm_numeric_large", est_bytes, [&] {
      k_spgemm_fill<kHtLarge, true><<<std::min(hover, 65536), 64, 0, c.s>>>(olist.p, hover, A.nrows, A.rowptr.p, A.col.p,
                                                                            A.val.p, B.rowptr.p, B.col.p, B.val.p,
                                                                            C.rowptr.p, C.col.p, C.val.p);
    });
}

// ---------------------------------------------------------------------------
// SpMV: LPR lanes per row, shuffle reduction inside the lane group
// ---------------------------------------------------------------------------
// V: matrix value type, X: input vector type, Y: output (and b) type; sums in
// FP64.  mode 0: y = A x, 1: y = b - A x, 2: y += A x.
template <class V, class X, class Y, int LPR>
__global__ void __launch_bounds__(256) k_spmv(const int* __restrict__ rp, const int* __restrict__ col,
                                              const V* __restrict__ val, const X* __restrict__ x, Y* __restrict__ y,
                                              const Y* __restrict__ b, int n, int mode) {
  const int g = (xcd_block(gridDim.x) * blockDim.x + threadIdx.x) / LPR;
  const int l = threadIdx.x & (LPR - 1);
  if (g >= n) return;
  double s = 0;
  const int a = rp[g], e = rp[g + 1];
  // padding slots gather x at the row's first column (a cached, local line);
  // a fixed column would make one address hot for every wave of the grid
  const int cpad = a < e ? col[a] : 0;
  // up to four entries per lane are loaded before they are summed, so their
  // gathers overlap (plain loads measured faster than non-temporal ones here)
  int q = a + l;
  for (; q + 3 * LPR < e; q += 4 * LPR) {
    const int c0 = col[q], c1 = col[q + LPR], c2 = col[q + 2 * LPR], c3 = col[q + 3 * LPR];
    const V v0 = val[q], v1 = val[q + LPR], v2 = val[q + 2 * LPR], v3 = val[q + 3 * LPR];
    s += (double)v0 * (double)x[c0] + (double)v1 * (double)x[c1] + (double)v2 * (double)x[c2] +
         (double)v3 * (double)x[c3];
  }
  int cc[3];
  V vv[3];
#pragma unroll
  for (int u = 0; u < 3; ++u) {
    const int qq = q + u * LPR;
    cc[u] = qq < e ? col[qq] : cpad;
    vv[u] = qq < e ? val[qq] : V(0);
  }
#pragma unroll
  for (int u = 0; u < 3; ++u) s += (double)vv[u] * (double)x[cc[u]];
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
  if (l == 0) {
    if (mode == 0) y[g] = (Y)s;
    else if (mode == 1) y[g] = (Y)((double)b[g] - s);
    else y[g] = (Y)((double)y[g] + s);
  }
}

template <class V, class X, class Y>
static void spmv_t(const int* rp, const int* col, const V* val, int n, int64_t nnz, const X* x, Y* y, const Y* b, int mode,
                   Ctx& c, const char* tag) {
  if (n == 0) return;
  const double avg = (double)nnz / n;
  const double bytes = (double)nnz * (4 + sizeof(V)) + 4.0 * (n + 1) + (double)n * (sizeof(X) + sizeof(Y)) +
                       (mode ? (double)n * sizeof(Y) : 0.0);
  const int64_t nb = n;
  // lanes per row: measured at 128^3 (A^(e) ~16, P^(e) ~8, D^T A ~69,
  // A_1 ~40, P^(e)T ~230 entries per row), wider rows run fastest with
  // four or more entries per lane, so each lane has independent gathers in
  // flight; rows of 13-20 entries (A^(e), D^T) keep two per lane
  if (avg <= 12)
    c.run(tag, bytes, [&] { k_spmv<V, X, Y, 2><<<ceil_div(nb * 2, 256), 256, 0, c.s>>>(rp, col, val, x, y, b, n, mode); });
  else if (avg <= 48)
    c.run(tag, bytes, [&] { k_spmv<V, X, Y, 8><<<ceil_div(nb * 8, 256), 256, 0, c.s>>>(rp, col, val, x, y, b, n, mode); });
  else if (avg <= 96)
    c.run(tag, bytes, [&] { k_spmv<V, X, Y, 16><<<ceil_div(nb * 16, 256), 256, 0, c.s>>>(rp, col, val, x, y, b, n, mode); });
  else
    c.run(tag, bytes, [&] { k_spmv<V, X, Y, 64><<<ceil_div(nb * 64, 256), 256, 0, c.s>>>(rp, col, val, x, y, b, n, mode); });
}

template <class X, class Y>
void spmv_v64(const Csr& A, const X* x, Y* y, const Y* b, int mode, Ctx& c, const char* tag) {
  spmv_t<double, X, Y>(A.rowptr.p, A.col.p, A.val.p, A.nrows, A.nnz, x, y, b, mode, c, tag);
}
template <class X, class Y>
void spmv_v32(const Csr& A, const X* x, Y* y, const Y* b, int mode, Ctx& c, const char* tag) {
  spmv_t<float, X, Y>(A.rowptr.p, A.col.p, A.val32.p, A.nrows, A.nnz, x, y, b, mode, c, tag);
}
template void spmv_v64<double, double>(const Csr&, const double*, double*, const double*, int, Ctx&, const char*);
template void spmv_v64<float, float>(const Csr&, const float*, float*, const float*, int, Ctx&, const char*);
template void spmv_v32<float, float>(const Csr&, const float*, float*, const float*, int, Ctx&, const char*);
template void spmv_v32<double, float>(const Csr&, const double*, float*, const float*, int, Ctx&, const char*);
template void spmv_v32<float, double>(const Csr&, const float*, double*, const double*, int, Ctx&, const char*);
template void spmv_v32<double, double>(const Csr&, const double*, double*, const double*, int, Ctx&, const char*);

void spmv(const Csr& A, const double* x, double* y, const double* b, int mode, Ctx& c, const char* tag) {
  spmv_v64<double, double>(A, x, y, b, mode, c, tag);
}

// ---------------------------------------------------------------------------
// deterministic dot products: fixed grid of kRedBlocks blocks, then one block
// ---------------------------------------------------------------------------
template <class T>
__global__ void __launch_bounds__(256) k_dot_partial(const T* __restrict__ x, const T* __restrict__ y, int64_t n,
                                                     double* __restrict__ part) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    s += (double)x[i] * (double)y[i];
  double r = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256) k_reduce_partials(const double* __restrict__ part, int nb, double* __restrict__ out) {
  __shared__ double sh[4];
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) s += part[i];
  double r = block_sum256(s, sh);
  if (threadIdx.x == 0) *out = r;
}

void reduce_partials(int nblocks, int slot, double* out, Ctx& c) {
  c.run("reduce", 8.0 * nblocks, [&] {
    k_reduce_partials<<<1, 256, 0, c.s>>>(c.red.p + (size_t)slot * Ctx::kRedBlocks, nblocks, out);
  });
}

void dot(const double* x, const double* y, int64_t n, double* out, Ctx& c, int slot) {
  int nb = (int)std::min<int64_t>(Ctx::kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
  c.run("dot", 16.0 * n, [&] { k_dot_partial<double><<<nb, 256, 0, c.s>>>(x, y, n, c.red.p + (size_t)slot * Ctx::kRedBlocks); });
  reduce_partials(nb, slot, out, c);
}
void dot32(const float* x, const float* y, int64_t n, double* out, Ctx& c, int slot) {
  int nb = (int)std::min<int64_t>(Ctx::kRedBlocks, std::max<int64_t>(1, (n + 255) / 256));
  c.run("dot32", 8.0 * n, [&] { k_dot_partial<float><<<nb, 256, 0, c.s>>>(x, y, n, c.red.p + (size_t)slot * Ctx::kRedBlocks); });
  reduce_partials(nb, slot, out, c);
}

// ---------------------------------------------------------------------------
// small elementwise kernels
// ---------------------------------------------------------------------------
__global__ void k_diag(const int* __restrict__ rp, const int* __restrict__ col, const double* __restrict__ val, int n,
                       double* __restrict__ d, int inv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double v = 0.0;
  for (int q = rp[i]; q < rp[i + 1]; ++q)
    if (col[q] == i) v = val[q];
  d[i] = inv ? 1.0 / v : v;
}
void diagonal(const Csr& A, double* d, bool inv, Ctx& c) {
  if (!A.nrows) return;
  c.run("diag", 12.0 * A.nnz, [&] { k_diag<<<ceil_div(A.nrows, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, A.val.p, A.nrows, d, inv); });
}

template <class T>
__global__ void k_fill(T* __restrict__ x, T v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
void fill(double* x, double v, int64_t n, Ctx& c) {
  if (n) c.run("fill", 8.0 * n, [&] { k_fill<double><<<ceil_div(n, 256), 256, 0, c.s>>>(x, v, n); });
}
void fill32(float* x, float v, int64_t n, Ctx& c) {
  if (n) c.run("fill", 4.0 * n, [&] { k_fill<float><<<ceil_div(n, 256), 256, 0, c.s>>>(x, v, n); });
}
void fill_int(int* x, int v, int64_t n, Ctx& c) {
  if (n) c.run("fill", 4.0 * n, [&] { k_fill<int><<<ceil_div(n, 256), 256, 0, c.s>>>(x, v, n); });
}

template <class A, class B>
__global__ void k_cast(const A* __restrict__ x, B* __restrict__ y, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = (B)x[i];
}
void cast_d2f(const double* x, float* y, int64_t n, Ctx& c) {
  if (n) c.run("cast", 12.0 * n, [&] { k_cast<double, float><<<ceil_div(n, 256), 256, 0, c.s>>>(x, y, n); });
}
void cast_f2d(const float* x, double* y, int64_t n, Ctx& c) {
  if (n) c.run("cast", 12.0 * n, [&] { k_cast<float, double><<<ceil_div(n, 256), 256, 0, c.s>>>(x, y, n); });
}

}  // namespace hc
