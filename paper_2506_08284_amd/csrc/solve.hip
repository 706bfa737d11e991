// Solve phase (Sec. 6.1): multicolour symmetric Gauss-Seidel, Hiptmair
// smoothing, V-cycle with a direct coarsest solve, preconditioned CG.
#include <chrono>
#include <cmath>

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
  if (v >= n) return;
  const int cv = color[v];
  if (cv == -1) { atomicAdd(remaining, 1ULL); return; }
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

__global__ void k_color_count(const int* __restrict__ color, int n, int* __restrict__ cnt) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) atomicAdd(&cnt[color[v]], 1);
}
__global__ void k_color_fill(const int* __restrict__ color, int n, int* __restrict__ cursor, int* __restrict__ rows) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v < n) rows[atomicAdd(&cursor[color[v]], 1)] = v;
}

void color_rows(const Csr& A, DBuf<int>& color, DBuf<int>& rows, std::vector<int>& cptr, int& ncol, Ctx& c) {
  const int n = A.nrows;
  color.alloc(n, c.s);
  rows.alloc(n, c.s);
  fill_int(color.p, -1, n, c);
  unsigned long long* rem = (unsigned long long*)(c.iscal.p + 8);
  for (int round = 0;; ++round) {
    if (round > n + 1) fail(HCURL_EHIP, "colouring did not terminate");
    c.run("jp_select", 12.0 * A.nnz, [&] { k_jp_select<<<ceil_div(n, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, n, color.p); });
    HC_HIP(hipMemsetAsync(rem, 0, sizeof(unsigned long long), c.s));
    c.run("jp_assign", 12.0 * A.nnz, [&] { k_jp_assign<<<ceil_div(n, 256), 256, 0, c.s>>>(A.rowptr.p, A.col.p, n, color.p, rem); });
    unsigned long long h = 0;
    d2h(&h, rem, 1, c);
    if (h == 0) break;
  }
  // group rows by colour
  std::vector<int> hc_(n);
  d2h(hc_.data(), color.p, n, c);
  ncol = 0;
  for (int v : hc_) ncol = std::max(ncol, v + 1);
  DBuf<int> cnt(ncol + 1, c.s);
  HC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(int) * (ncol + 1), c.s));
  k_color_count<<<ceil_div(n, 256), 256, 0, c.s>>>(color.p, n, cnt.p);
  HC_LAUNCH_CHECK();
  std::vector<int> hcnt(ncol + 1);
  d2h(hcnt.data(), cnt.p, ncol, c);
  cptr.assign(ncol + 1, 0);
  for (int k = 0; k < ncol; ++k) cptr[k + 1] = cptr[k] + hcnt[k];
  h2d(cnt.p, cptr.data(), ncol, c);
  k_color_fill<<<ceil_div(n, 256), 256, 0, c.s>>>(color.p, n, cnt.p, rows.p);
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// Gauss-Seidel on the rows of one colour: x_i += (b_i - A_i x) / a_ii.
// Rows of one colour are not coupled, so they update in parallel.
// ---------------------------------------------------------------------------
template <class T, int LPR, int TAG>
__global__ void __launch_bounds__(256) k_gs_color(const int* __restrict__ rows, int nr, const int* __restrict__ rp,
                                                  const int* __restrict__ col, const T* __restrict__ val,
                                                  const T* __restrict__ dinv, const T* __restrict__ b, T* __restrict__ x) {
  const int g = (blockIdx.x * blockDim.x + threadIdx.x) / LPR;
  const int l = threadIdx.x & (LPR - 1);
  if (g >= nr) return;
  const int i = rows[g];
  T s = 0;
  const int e = rp[i + 1];
  for (int q = rp[i] + l; q < e; q += LPR) s += val[q] * x[col[q]];
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, LPR);
  if (l == 0) x[i] += (b[i] - s) * dinv[i];
}

// Algorithmic bytes of one colour launch: the rows' CSR data, their b, 1/a_ii
// and x (read and write), counting every x entry once per sweep (ideal reuse
// of the gathered neighbours).
template <class T, int TAG>
static void sgs_t(const Csr& A, const T* val, const T* dinv, const DBuf<int>& rows, const std::vector<int>& cptr, int ncol,
                  const T* b, T* x, Ctx& c, const char* tag) {
  const double avg = A.nrows ? (double)A.nnz / A.nrows : 0.0;
  auto launch = [&](int k) {
    const int nr = cptr[k + 1] - cptr[k];
    if (!nr) return;
    const int* r = rows.p + cptr[k];
    const double bytes = (double)nr * avg * (4 + sizeof(T)) + (double)nr * (8 + 4 + 4 * sizeof(T));
    if (avg <= 12)
      c.run(tag, bytes, [&] { k_gs_color<T, 8, TAG><<<ceil_div((int64_t)nr * 8, 256), 256, 0, c.s>>>(r, nr, A.rowptr.p, A.col.p, val, dinv, b, x); });
    else if (avg <= 40)
      c.run(tag, bytes, [&] { k_gs_color<T, 16, TAG><<<ceil_div((int64_t)nr * 16, 256), 256, 0, c.s>>>(r, nr, A.rowptr.p, A.col.p, val, dinv, b, x); });
    else
      c.run(tag, bytes, [&] { k_gs_color<T, 64, TAG><<<ceil_div((int64_t)nr * 64, 256), 256, 0, c.s>>>(r, nr, A.rowptr.p, A.col.p, val, dinv, b, x); });
  };
  for (int k = 0; k < ncol; ++k) launch(k);
  for (int k = ncol - 1; k >= 0; --k) launch(k);
}

// x += D c  with D given by its endpoints: x_e += c[head] - c[tail]
template <class T>
__global__ void k_grad_add(const int* __restrict__ tail, const int* __restrict__ head, int n, const T* __restrict__ cn,
                           T* __restrict__ x) {
  int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) x[e] += cn[head[e]] - cn[tail[e]];
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
// Level 0 gets its own kernel instances (TAG 1) so that profiles separate the
// fine-level sweeps from the launch-bound coarse ones.
static void hiptmair64(Level& L, bool fine, double* x, const double* b, Ctx& c) {
  auto edge = [&] {
    if (fine) sgs_t<double, 1>(L.A, L.A.val.p, L.dinvA.p, L.rowsA, L.cptrA, L.ncolA, b, x, c, "sgs_edge_l0");
    else sgs_t<double, 0>(L.A, L.A.val.p, L.dinvA.p, L.rowsA, L.cptrA, L.ncolA, b, x, c, "sgs_edge");
  };
  edge();
  spmv(L.A, x, L.r.p, b, 1, c, fine ? "residual_l0" : "residual");
  spmv(L.DT, L.r.p, L.rn.p, nullptr, 0, c, "grad_transpose");
  fill(L.cn.p, 0.0, L.m, c);
  if (fine) sgs_t<double, 2>(L.An, L.An.val.p, L.dinvAn.p, L.rowsAn, L.cptrAn, L.ncolAn, L.rn.p, L.cn.p, c, "sgs_node_l0");
  else sgs_t<double, 0>(L.An, L.An.val.p, L.dinvAn.p, L.rowsAn, L.cptrAn, L.ncolAn, L.rn.p, L.cn.p, c, "sgs_node");
  c.run("grad_add", 24.0 * L.n, [&] { k_grad_add<double><<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, L.n, L.cn.p, x); });
  edge();
}

static void hiptmair32(Level& L, bool fine, float* x, const float* b, Ctx& c) {
  auto edge = [&] {
    if (fine) sgs_t<float, 1>(L.A, L.A.val32.p, L.dinvA32.p, L.rowsA, L.cptrA, L.ncolA, b, x, c, "sgs_edge32_l0");
    else sgs_t<float, 0>(L.A, L.A.val32.p, L.dinvA32.p, L.rowsA, L.cptrA, L.ncolA, b, x, c, "sgs_edge32");
  };
  edge();
  spmv32(L.A, x, L.r32.p, b, 1, c, fine ? "residual32_l0" : "residual32");
  spmv32(L.DT, L.r32.p, L.rn32.p, nullptr, 0, c, "grad_transpose32");
  fill32(L.cn32.p, 0.0f, L.m, c);
  if (fine) sgs_t<float, 2>(L.An, L.An.val32.p, L.dinvAn32.p, L.rowsAn, L.cptrAn, L.ncolAn, L.rn32.p, L.cn32.p, c, "sgs_node32_l0");
  else sgs_t<float, 0>(L.An, L.An.val32.p, L.dinvAn32.p, L.rowsAn, L.cptrAn, L.ncolAn, L.rn32.p, L.cn32.p, c, "sgs_node32");
  c.run("grad_add32", 12.0 * L.n, [&] { k_grad_add<float><<<ceil_div(L.n, 256), 256, 0, c.s>>>(L.tail.p, L.head.p, L.n, L.cn32.p, x); });
  edge();
}

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
  fill(x, 0.0, L.n, c);
  hiptmair64(L, l == 0, x, b, c);
  spmv(L.A, x, L.r.p, b, 1, c, "residual");
  spmv(L.PeT, L.r.p, N.b.p, nullptr, 0, c, "restrict");
  vcycle64(H, l + 1, N.b.p, N.x.p);
  spmv(L.Pe, N.x.p, x, nullptr, 2, c, "prolong");
  hiptmair64(L, l == 0, x, b, c);
}

static void vcycle32(Hierarchy& H, int l, const float* b, float* x) {
  Ctx& c = H.ctx;
  if (l == (int)H.lv.size() - 1) {
    c.run("coarse_solve32", 8.0 * H.co.n * H.co.n, [&] {
      k_dense_apply<float><<<ceil_div((int64_t)H.co.n * 64, 256), 256, 0, c.s>>>(H.co.inv.p, H.co.n, b, x);
    });
    return;
  }
  Level& L = *H.lv[l];
  Level& N = *H.lv[l + 1];
  fill32(x, 0.0f, L.n, c);
  hiptmair32(L, l == 0, x, b, c);
  spmv32(L.A, x, L.r32.p, b, 1, c, "residual32");
  spmv32(L.PeT, L.r32.p, N.b32.p, nullptr, 0, c, "restrict32");
  vcycle32(H, l + 1, N.b32.p, N.x32.p);
  spmv32(L.Pe, N.x32.p, x, nullptr, 2, c, "prolong32");
  hiptmair32(L, l == 0, x, b, c);
}

void apply_vcycle(Hierarchy& H, const double* r, double* z) {
  Ctx& c = H.ctx;
  if (H.opts.vcycle_fp32) {
    Level& L = *H.lv[0];
    if (H.lv.size() == 1) {
      vcycle64(H, 0, r, z);
      return;
    }
    cast_d2f(r, L.b32.p, L.n, c);
    vcycle32(H, 0, L.b32.p, L.x32.p);
    cast_f2d(L.x32.p, z, L.n, c);
  } else {
    vcycle64(H, 0, r, z);
  }
}

// ---------------------------------------------------------------------------
// preparation: workspace and FP32 copies
// ---------------------------------------------------------------------------
static void make32(Csr& A, Ctx& c) {
  if (!A.val.p) return;
  A.val32.alloc(A.nnz, c.s);
  cast_d2f(A.val.p, A.val32.p, A.nnz, c);
}

void prepare_solve(Hierarchy& H) {
  Ctx& c = H.ctx;
  const bool f32 = H.opts.vcycle_fp32 != 0;
  for (size_t l = 0; l < H.lv.size(); ++l) {
    Level& L = *H.lv[l];
    L.x.alloc(L.n, c.s);
    L.b.alloc(L.n, c.s);
    if (l + 1 == H.lv.size()) {
      if (f32) { L.x32.alloc(L.n, c.s); L.b32.alloc(L.n, c.s); }
      continue;
    }
    L.r.alloc(L.n, c.s);
    L.rn.alloc(L.m, c.s);
    L.cn.alloc(L.m, c.s);
    if (f32) {
      L.x32.alloc(L.n, c.s); L.b32.alloc(L.n, c.s); L.r32.alloc(L.n, c.s);
      L.rn32.alloc(L.m, c.s); L.cn32.alloc(L.m, c.s);
      make32(L.A, c); make32(L.An, c); make32(L.Pe, c); make32(L.PeT, c); make32(L.D, c); make32(L.DT, c);
      L.dinvA32.alloc(L.n, c.s); L.dinvAn32.alloc(L.m, c.s);
      cast_d2f(L.dinvA.p, L.dinvA32.p, L.n, c);
      cast_d2f(L.dinvAn.p, L.dinvAn32.p, L.m, c);
    }
  }
  const int n = H.lv[0]->n;
  H.px.alloc(n, c.s); H.pr.alloc(n, c.s); H.pz.alloc(n, c.s); H.pp.alloc(n, c.s); H.pq.alloc(n, c.s);
  if (f32) H.pzold.alloc(n, c.s);
}

// ---------------------------------------------------------------------------
// PCG (FP64 vectors and inner products, device scalars)
// ---------------------------------------------------------------------------
__global__ void k_pcg_alpha(double* __restrict__ sc, unsigned long long* __restrict__ bad) {
  const double pq = sc[P_PQ];
  if (!(pq > 0.0)) { *bad += 1; sc[P_ALPHA] = 0.0; return; }
  sc[P_ALPHA] = sc[P_RZ] / pq;
}
__global__ void __launch_bounds__(256) k_pcg_update(int64_t n, double* __restrict__ x, double* __restrict__ r,
                                                    const double* __restrict__ p, const double* __restrict__ q,
                                                    const double* __restrict__ alpha, double* __restrict__ part) {
  __shared__ double sh[4];
  const double a = *alpha;
  double s = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    x[i] += a * p[i];
    const double ri = r[i] - a * q[i];
    r[i] = ri;
    s += ri * ri;
  }
  double t = block_sum256(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
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
  const bool flex = H.opts.vcycle_fp32 != 0;
  double* sc = c.scal.p;
  unsigned long long* bad = (unsigned long long*)(c.iscal.p + 9);
  HC_HIP(hipMemsetAsync(bad, 0, sizeof(unsigned long long), c.s));
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
  if (nf == 0.0) {
    d2d(u, H.px.p, n, c);
    if (iters) *iters = 0;
    if (relres) *relres = 0.0;
    c.sync();
    return HCURL_OK;
  }
  apply_vcycle(H, H.pr.p, H.pz.p);
  d2d(H.pp.p, H.pz.p, n, c);
  dot(H.pr.p, H.pz.p, n, sc + P_RZ, c, 3);
  while (it < maxit) {
    spmv(L.A, H.pp.p, H.pq.p, nullptr, 0, c, "pcg_spmv");
    dot(H.pp.p, H.pq.p, n, sc + P_PQ, c, 3);
    c.run("pcg_scalar", 0.0, [&] { k_pcg_alpha<<<1, 1, 0, c.s>>>(sc, bad); });
    c.run("pcg_update", 48.0 * n, [&] {
      k_pcg_update<<<nbu, 256, 0, c.s>>>(n, H.px.p, H.pr.p, H.pp.p, H.pq.p, sc + P_ALPHA, c.red.p + 4 * (size_t)Ctx::kRedBlocks);
    });
    reduce_partials(nbu, 4, sc + P_RR, c);
    double rr[1];
    d2h(rr, sc + P_RR, 1, c);
    ++it;
    unsigned long long hb = 0;
    d2h(&hb, bad, 1, c);
    if (hb) fail(HCURL_ENOTSPD, "PCG breakdown: <p, A p> <= 0");
    rel = std::sqrt(rr[0]) / nf;
    if (rel <= rtol) break;
    if (flex) d2d(H.pzold.p, H.pz.p, n, c);
    apply_vcycle(H, H.pr.p, H.pz.p);
    dot(H.pr.p, H.pz.p, n, sc + P_RZNEW, c, 3);
    if (flex) dot(H.pr.p, H.pzold.p, n, sc + P_RZOLD, c, 5);
    c.run("pcg_scalar", 0.0, [&] { k_pcg_beta<<<1, 1, 0, c.s>>>(sc, flex ? 1 : 0); });
    c.run("pcg_dir", 24.0 * n, [&] { k_pcg_dir<<<ceil_div(n, 256), 256, 0, c.s>>>(n, H.pp.p, H.pz.p, sc + P_BETA); });
  }
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
  return rel <= rtol ? HCURL_OK : HCURL_EMAXIT;
}

}  // namespace hc
