// extern "C" entry points (include/hcurl_amg.h).  Every call catches the
// library's errors and turns them into return codes.
#include <algorithm>
#include <chrono>
#include <cstring>
#include <mutex>

#include "mpnn.hpp"

struct hcurl_amg_s {
  hc::Allocator alloc;  // declared first: outlives every buffer of H
  hc::Hierarchy H;
  int device = -1;      // current device at setup
};

// Staging area of hcurl_amg_solve_noalloc: f in the first half, u in the
// second.  Host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (scratch_address).
static __device__ __align__(256) double scratch[2 * (size_t)HCURL_NOALLOC_MAX_ROWS];

namespace {
thread_local std::string g_last_error;

int guard_error(const hc::Error& e) {
  g_last_error = e.msg;
  return e.code;
}

template <class F>
int guarded(F&& f) {
  try {
    g_last_error.clear();
    return f();
  } catch (const hc::Error& e) {
    return guard_error(e);
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HCURL_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HCURL_EHIP;
  } catch (...) {
    g_last_error = "unknown error";
    return HCURL_EHIP;
  }
}

// the handle's allocator for the scope of an entry point (null: the default)
const hc::Allocator* alloc_of(hcurl_amg h) { return h && h->alloc.alloc ? &h->alloc : nullptr; }

hc::Level* level_of(hcurl_amg h, int level) {
  if (!h || level < 0 || level >= (int)h->H.lv.size()) hc::fail(HCURL_EINVAL, "level out of range");
  return h->H.lv[level].get();
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per device.
double* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) hc::fail(HCURL_EUNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      hc::fail(HCURL_EHIP, std::string("hipGetSymbolAddress(scratch) -> ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = (double*)p;
  }
  return g_scratch_ptr[dev];
}

// Installed for the duration of hcurl_amg_solve_noalloc: any device buffer
// requested inside it fails the call instead of allocating.
const hc::Allocator kNoAllocation{nullptr, nullptr, nullptr, "hcurl_amg_solve_noalloc allocates no device memory"};

void export_csr(const hc::Csr& A, int64_t* rowptr, int32_t* col, double* val, hc::Ctx& c) {
  std::vector<int> rp(A.nrows + 1);
  hc::d2h(rp.data(), A.rowptr.p, A.nrows + 1, c);
  if (rowptr)
    for (int i = 0; i <= A.nrows; ++i) rowptr[i] = rp[i];
  if (col) hc::d2h(col, A.col.p, A.nnz, c);
  if (val) {
    if (!A.val.p) hc::fail(HCURL_EINVAL, "matrix has no values");
    hc::d2h(val, A.val.p, A.nnz, c);
  }
}
}  // namespace

extern "C" {

void hcurl_amg_default_opts(hcurl_amg_opts* o) {
  std::memset(o, 0, sizeof(*o));
  o->max_levels = 0;
  o->coarse_max_rows = 0;
  o->emin_iters = 10;
  o->emin_method = HCURL_EMIN_CG;
  o->emin_omega = 0.5;
  o->init_guess = HCURL_INIT_ONES;
  o->init_values = nullptr;
  o->emin_iters_given = 3;
  o->mpnn = nullptr;
  o->vcycle_fp32 = 0;
  o->nodal_prolongator = nullptr;
  o->alg1_passes = 2;
  o->pbar_alg1 = 0;
  o->aggregation = HCURL_AGG_GIVEN;
  o->power_iters = 20;
  o->record_energy = 0;
  o->emin_codes = 1;
  o->profile = 0;
  o->mem_space = HCURL_MEM_HOST;
  o->stream = nullptr;
}

int hcurl_amg_setup(const hcurl_csr* A, const hcurl_csr* Dh, const double* coords, const int32_t* const* aggregates,
                    int n_agg_levels, const hcurl_amg_opts* opts, hcurl_amg* out) {
  if (!out) return HCURL_EINVAL;
  *out = nullptr;
  if (!A || !Dh) return HCURL_EINVAL;
  auto* h = new (std::nothrow) hcurl_amg_s();
  if (!h) return HCURL_ENOMEM;
  int rc = guarded([&]() -> int {
    if (opts) h->H.opts = *opts; else hcurl_amg_default_opts(&h->H.opts);
    if (h->H.opts.emin_iters < 0 || h->H.opts.power_iters < 1) hc::fail(HCURL_EINVAL, "bad iteration counts");
    if (h->H.opts.profile < 0 || h->H.opts.profile > 3) hc::fail(HCURL_EINVAL, "profile must be 0, 1, 2 or 3");
    if (h->H.opts.emin_codes != 0 && h->H.opts.emin_codes != 1) hc::fail(HCURL_EINVAL, "emin_codes must be 0 or 1");
    if (h->H.opts.aggregation != HCURL_AGG_GIVEN && h->H.opts.aggregation != HCURL_AGG_MIS2)
      hc::fail(HCURL_EINVAL, "unknown aggregation");
    if ((h->H.opts.nodal_prolongator || h->H.opts.pbar_alg1) && h->H.opts.alg1_passes < 1)
      hc::fail(HCURL_EINVAL, "alg1_passes must be >= 1");
    if (!h->H.opts.dev_alloc != !h->H.opts.dev_free) hc::fail(HCURL_EINVAL, "dev_alloc and dev_free go together");
    h->alloc.alloc = h->H.opts.dev_alloc;
    h->alloc.free = h->H.opts.dev_free;
    h->alloc.ctx = h->H.opts.alloc_ctx;
    hc::AllocatorScope scope(alloc_of(h));
    HC_HIP(hipGetDevice(&h->device));
    h->H.ctx.init((hipStream_t)h->H.opts.stream, h->H.opts.profile != 0);
    auto t0 = std::chrono::steady_clock::now();
    hc::build_hierarchy(h->H, *A, *Dh, coords, aggregates, n_agg_levels);
    h->H.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return HCURL_OK;
  });
  if (rc != HCURL_OK) {
    std::string msg = g_last_error;
    try { (void)hipStreamSynchronize(h->H.ctx.s); } catch (...) {}
    delete h;
    g_last_error = msg;
    return rc;
  }
  *out = h;
  return HCURL_OK;
}

int hcurl_amg_solve(hcurl_amg h, const double* f, double* u, double rtol, int maxit, int* iters, double* relres) {
  if (!h || !f || !u || maxit < 0) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    auto& H = h->H;
    auto& c = H.ctx;
    if (!H.valid) hc::fail(HCURL_EINVAL, "the handle is unusable after a failed hcurl_amg_update");
    const int64_t n = H.lv[0]->n;
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    if (H.opts.mem_space == HCURL_MEM_DEVICE) {
      rc = hc::pcg_solve(H, f, u, rtol, maxit, iters, relres);
    } else {
      hc::DBuf<double> df(n, c.s), du(n, c.s);
      hc::h2d(df.p, f, n, c);
      rc = hc::pcg_solve(H, df.p, du.p, rtol, maxit, iters, relres);
      hc::d2h(u, du.p, n, c);
    }
    H.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
  });
}

int hcurl_amg_solve_noalloc(hcurl_amg h, const double* f, double* u, double rtol, int maxit, int* iters,
                            double* relres) {
  if (!h || !f || !u || maxit < 0) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::AllocatorScope scope(&kNoAllocation);
    auto& H = h->H;
    auto& c = H.ctx;
    if (!H.valid) hc::fail(HCURL_EINVAL, "the handle is unusable after a failed hcurl_amg_update");
    int dev = -1;
    HC_HIP(hipGetDevice(&dev));
    if (dev != h->device)
      hc::fail(HCURL_EINVAL, "the current device (" + std::to_string(dev) + ") is not the handle's (" +
                                 std::to_string(h->device) + ")");
    const int64_t n = H.lv[0]->n;
    const bool host = H.opts.mem_space != HCURL_MEM_DEVICE;
    if (host && n > HCURL_NOALLOC_MAX_ROWS)
      hc::fail(HCURL_EUNSUPPORTED, "hcurl_amg_solve_noalloc stages at most " + std::to_string(HCURL_NOALLOC_MAX_ROWS) +
                                       " rows; this handle has " + std::to_string(n));
    auto t0 = std::chrono::steady_clock::now();
    int rc;
    if (!host) {
      rc = hc::pcg_solve(H, f, u, rtol, maxit, iters, relres);
    } else {
      double* df = scratch_address(dev);
      double* du = df + HCURL_NOALLOC_MAX_ROWS;
      hc::h2d(df, f, n, c);
      rc = hc::pcg_solve(H, df, du, rtol, maxit, iters, relres);
      hc::d2h(u, du, n, c);
    }
    H.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return rc;
  });
}

int hcurl_amg_vcycle(hcurl_amg h, const double* r, double* z) {
  if (!h || !r || !z) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    auto& H = h->H;
    auto& c = H.ctx;
    if (!H.valid) hc::fail(HCURL_EINVAL, "the handle is unusable after a failed hcurl_amg_update");
    const int64_t n = H.lv[0]->n;
    if (H.opts.mem_space == HCURL_MEM_DEVICE) {
      hc::apply_vcycle(H, r, z);
      c.sync();
    } else {
      hc::DBuf<double> dr(n, c.s), dz(n, c.s);
      hc::h2d(dr.p, r, n, c);
      hc::apply_vcycle(H, dr.p, dz.p);
      hc::d2h(z, dz.p, n, c);
    }
    return HCURL_OK;
  });
}

void hcurl_amg_destroy(hcurl_amg h) {
  if (!h) return;
  try {
    (void)hipStreamSynchronize(h->H.ctx.s);
  } catch (...) {
  }
  delete h;
}

int hcurl_amg_num_levels(hcurl_amg h) { return h ? (int)h->H.lv.size() : HCURL_EINVAL; }

int hcurl_amg_level_info(hcurl_amg h, int level, hcurl_level_info* info) {
  if (!info) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::Level* L = level_of(h, level);
    std::memset(info, 0, sizeof(*info));
    info->n_edges = L->n;
    info->n_nodes = L->m;
    info->nnz_A = L->A.nnz;
    info->nnz_An = L->An.nnz;
    info->nnz_Pe = L->Pe.nnz;
    info->nnz_Pn = L->Pn.nnz;
    info->nnz_T = L->R.nnz;
    info->n_coarse_edges = L->n_coarse;
    info->irreducible_added = L->irreducible_added;
    info->n_colors_A = L->ncolA;
    info->n_colors_An = L->ncolAn;
    info->rho = L->rho;
    info->omega = L->omega;
    info->cancellation_ratio = L->cancel;
    return HCURL_OK;
  });
}

int hcurl_amg_commute_residual(hcurl_amg h, int level, double* abs_max, double* ref_max) {
  if (!abs_max || !ref_max) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    hc::Level* L = level_of(h, level);
    if (!h->H.valid) hc::fail(HCURL_EINVAL, "the handle is unusable after a failed hcurl_amg_update");
    hc::commute_residual(*L, abs_max, ref_max, h->H.ctx);
    return HCURL_OK;
  });
}

int hcurl_amg_curl_residual(hcurl_amg h, const hcurl_csr* S, int nlev, double* abs_max, double* ref_max) {
  if (!h || !S || !abs_max || !ref_max) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    if (!h->H.valid) hc::fail(HCURL_EINVAL, "the handle is unusable after a failed hcurl_amg_update");
    hc::curl_residual(h->H, *S, nlev, abs_max, ref_max);
    return HCURL_OK;
  });
}

int hcurl_amg_export_csr(hcurl_amg h, int level, int which, int64_t* rowptr, int32_t* col, double* val) {
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    hc::Level* L = level_of(h, level);
    auto& c = h->H.ctx;
    switch (which) {
      case HCURL_EXPORT_A: export_csr(L->A, rowptr, col, val, c); break;
      case HCURL_EXPORT_AN: export_csr(L->An, rowptr, col, val, c); break;
      case HCURL_EXPORT_PN: export_csr(L->Pn, rowptr, col, val, c); break;
      case HCURL_EXPORT_PE: export_csr(L->Pe, rowptr, col, val, c); break;
      case HCURL_EXPORT_R: export_csr(L->R, rowptr, col, val, c); break;
      case HCURL_EXPORT_P0: {
        if (!L->has_transfer) hc::fail(HCURL_EINVAL, "level has no transfer");
        export_csr(L->Pe, rowptr, col, nullptr, c);
        if (val) hc::d2h(val, L->p0.p, L->Pe.nnz, c);
        break;
      }
      case HCURL_EXPORT_DH: {
        if (!L->has_transfer) hc::fail(HCURL_EINVAL, "level has no transfer");
        hc::Level* N = level_of(h, level + 1);
        std::vector<int> t(N->n), hd(N->n);
        hc::d2h(t.data(), N->tail.p, N->n, c);
        hc::d2h(hd.data(), N->head.p, N->n, c);
        // a single-node (Dirichlet) coarse edge has one entry; call with col
        // and val NULL to read the entry count from rowptr first
        int64_t o = 0;
        for (int e = 0; e < N->n; ++e) {
          if (rowptr) rowptr[e] = o;
          if (t[e] < 0 || hd[e] < 0) {
            const bool at_head = t[e] < 0;
            if (col) col[o] = at_head ? hd[e] : t[e];
            if (val) val[o] = at_head ? 1.0 : -1.0;
            o += 1;
            continue;
          }
          const bool up = t[e] < hd[e];
          if (col) { col[o] = up ? t[e] : hd[e]; col[o + 1] = up ? hd[e] : t[e]; }
          if (val) { val[o] = up ? -1.0 : 1.0; val[o + 1] = up ? 1.0 : -1.0; }
          o += 2;
        }
        if (rowptr) rowptr[N->n] = o;
        break;
      }
      default: hc::fail(HCURL_EINVAL, "unknown export");
    }
    return HCURL_OK;
  });
}

int hcurl_amg_export_vec(hcurl_amg h, int level, int which, void* out, int64_t capacity) {
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    hc::Level* L = level_of(h, level);
    auto& c = h->H.ctx;
    auto need = [&](int64_t b) {
      if (capacity < b) hc::fail(HCURL_EINVAL, "output buffer too small");
    };
    switch (which) {
      case HCURL_VEC_COLORS_A: need(4LL * L->n); hc::d2h((int*)out, L->colorA.p, L->n, c); break;
      case HCURL_VEC_COLORS_AN: need(4LL * L->m); hc::d2h((int*)out, L->colorAn.p, L->m, c); break;
      case HCURL_VEC_ENERGY: {
        need(8LL * (int64_t)L->energy.size());
        std::memcpy(out, L->energy.data(), 8 * L->energy.size());
        return (int)L->energy.size();
      }
      case HCURL_VEC_LOCAL_PAIRS: need(2LL * L->Pe.nnz); hc::d2h((uint16_t*)out, L->lpair.p, L->Pe.nnz, c); break;
      case HCURL_VEC_PCG_HISTORY: {
        if (level != 0) hc::fail(HCURL_EINVAL, "the PCG history belongs to level 0");
        const auto& v = h->H.pcg_hist;
        need(8LL * (int64_t)v.size());
        std::memcpy(out, v.data(), 8 * v.size());
        return (int)v.size();
      }
      case HCURL_VEC_AGGREGATES:
        if (!L->agg.p) hc::fail(HCURL_EINVAL, "the coarsest level has no aggregates");
        need(4LL * L->m);
        hc::d2h((int*)out, L->pbar.p ? L->pbar.p : L->agg.p, L->m, c);
        break;
      case HCURL_VEC_LS_HISTOGRAM:
        need(8LL * HCURL_LS_HIST_J * HCURL_LS_HIST_NP);
        hc::ls_histogram(*L, (int64_t*)out, c);
        break;
      case HCURL_VEC_PCG_ALPHA:
      case HCURL_VEC_PCG_BETA: {
        if (level != 0) hc::fail(HCURL_EINVAL, "the PCG coefficients belong to level 0");
        const auto& v = which == HCURL_VEC_PCG_ALPHA ? h->H.pcg_alpha : h->H.pcg_beta;
        need(8LL * (int64_t)v.size());
        std::memcpy(out, v.data(), 8 * v.size());
        return (int)v.size();
      }
      default: hc::fail(HCURL_EINVAL, "unknown vector");
    }
    return HCURL_OK;
  });
}

int hcurl_amg_update(hcurl_amg h, const hcurl_csr* A, int mode, int iters) {
  if (!h || !A) return HCURL_EINVAL;
  if (mode != HCURL_REUSE_TRANSFERS && mode != HCURL_REUSE_WARM) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::AllocatorScope scope(alloc_of(h));
    auto& H = h->H;
    if (!H.valid) hc::fail(HCURL_EINVAL, "the handle is unusable after a failed hcurl_amg_update");
    if (H.lv.size() < 2) hc::fail(HCURL_EINVAL, "a single-level hierarchy has no transfers to reuse");
    auto t0 = std::chrono::steady_clock::now();
    hc::update_hierarchy(H, *A, mode, iters);
    H.update_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return HCURL_OK;
  });
}

int hcurl_amg_stats(hcurl_amg h, hcurl_amg_stats_t* s) {
  if (!h || !s) return HCURL_EINVAL;
  auto& H = h->H;
  s->num_levels = (int)H.lv.size();
  double tot = 0.0;
  for (auto& L : H.lv) tot += (double)L->A.nnz;
  s->operator_complexity = H.lv.empty() ? 0.0 : tot / (double)H.lv[0]->A.nnz;
  s->setup_ms = H.setup_ms;
  s->solve_ms = H.solve_ms;
  s->last_iters = H.last_iters;
  s->last_relres = H.last_relres;
  s->vcycle_fp32 = H.fp32 ? 1 : 0;
  s->update_ms = H.update_ms;
  s->lanczos_lambda_min = H.lanczos_min;
  s->lanczos_lambda_max = H.lanczos_max;
  s->last_stagnated = H.stagnated ? 1 : 0;
  s->max_local_J = s->max_local_np = 0;
  for (auto& L : H.lv) {
    if (!L->has_transfer) continue;
    s->max_local_J = std::max(s->max_local_J, L->maxJ);
    s->max_local_np = std::max(s->max_local_np, L->maxNp);
  }
  return HCURL_OK;
}

int hcurl_amg_kernel_stats(hcurl_amg h, int max_kernels, char (*names)[48], int64_t* launches, double* ms, double* bytes) {
  if (!h) return HCURL_EINVAL;
  return guarded([&]() -> int {
    auto& c = h->H.ctx;
    c.drain();
    const int n = (int)c.stats.size();
    for (int k = 0; k < n && k < max_kernels; ++k) {
      if (names) {
        std::strncpy(names[k], c.stats[k].name.c_str(), 47);
        names[k][47] = 0;
      }
      if (launches) launches[k] = c.stats[k].launches;
      if (ms) ms[k] = c.stats[k].ms;
      if (bytes) bytes[k] = c.stats[k].bytes;
    }
    return n;
  });
}

void hcurl_amg_reset_kernel_stats(hcurl_amg h) {
  if (!h) return;
  try {
    h->H.ctx.drain();
  } catch (...) {
  }
  h->H.ctx.stats.clear();
}

// ---------------------------------------------------------------------------
// learned initial guess
// ---------------------------------------------------------------------------
int64_t hcurl_mpnn_num_params(void) { return hc::kNParam; }

int hcurl_mpnn_create(const float* params, void* stream, hcurl_mpnn* out) {
  if (!out || !params) return HCURL_EINVAL;
  *out = nullptr;
  auto* n = new (std::nothrow) hcurl_mpnn_s();
  if (!n) return HCURL_ENOMEM;
  int rc = guarded([&]() -> int {
    hc::Net& net = n->net;
    hc::Ctx& c = net.ctx;
    c.init((hipStream_t)stream, false);
    net.w.alloc(hc::kNParam, c.s);
    net.m.alloc(hc::kNParam, c.s);
    net.v.alloc(hc::kNParam, c.s);
    net.g.alloc(hc::kNParam, c.s);
    HC_HIP(hipMemsetAsync(net.m.p, 0, sizeof(float) * hc::kNParam, c.s));
    HC_HIP(hipMemsetAsync(net.v.p, 0, sizeof(float) * hc::kNParam, c.s));
    HC_HIP(hipMemsetAsync(net.g.p, 0, sizeof(float) * hc::kNParam, c.s));
    hc::h2d(net.w.p, params, hc::kNParam, c);
    net.wt_in.alloc(hc::kNF * hc::kHD, c.s);
    for (int l = 0; l < hc::kNL; ++l) {
      net.wt[l].alloc(hc::kKZ * hc::kHD, c.s);
      net.wr[l].alloc(hc::kKZ * hc::kHD, c.s);
    }
    net.refresh_bf16(c);
    c.sync();
    return HCURL_OK;
  });
  if (rc != HCURL_OK) { delete n; return rc; }
  *out = n;
  return HCURL_OK;
}

int hcurl_mpnn_get_params(hcurl_mpnn net, float* params) {
  if (!net || !params) return HCURL_EINVAL;
  return guarded([&]() -> int {
    hc::d2h(params, net->net.w.p, hc::kNParam, net->net.ctx);
    return HCURL_OK;
  });
}

int hcurl_mpnn_set_fp32_products(hcurl_mpnn net, int on) {
  if (!net || (on != 0 && on != 1)) return HCURL_EINVAL;
  net->net.fp32_products = on == 1;
  return HCURL_OK;
}

void hcurl_mpnn_destroy(hcurl_mpnn net) {
  if (!net) return;
  try { (void)hipStreamSynchronize(net->net.ctx.s); } catch (...) {}
  delete net;
}

int hcurl_amg_mpnn_sample(hcurl_amg h, hcurl_mpnn_sample* out) {
  if (!h || !out) return HCURL_EINVAL;
  *out = nullptr;
  auto* smp = new (std::nothrow) hcurl_mpnn_sample_s();
  if (!smp) return HCURL_ENOMEM;
  int rc = guarded([&]() -> int {
    auto& H = h->H;
    if (H.lv.size() < 2) hc::fail(HCURL_EINVAL, "hierarchy has a single level");
    if (H.opts.init_guess != HCURL_INIT_ONES) hc::fail(HCURL_EINVAL, "samples come from hierarchies with the plain initial guess");
    hc::Level& L0 = *H.lv[0];
    const int64_t np = L0.Pe.nnz;
    hc::DBuf<double> pmin(np, H.ctx.s);
    hc::fill(pmin.p, 0.0, np, H.ctx);
    hc::emin_make_feasible(L0, pmin.p, false, H.ctx);
    hc::mpnn_build_sample(H, L0, *H.lv[1], L0.p0.p, pmin.p, smp->S);
    smp->S.target.alloc(np, H.ctx.s);
    hc::d2d(smp->S.target.p, L0.Pe.val.p, np, H.ctx);
    H.ctx.sync();
    smp->ctx.init(H.ctx.s, false);
    return HCURL_OK;
  });
  if (rc != HCURL_OK) { delete smp; return rc; }
  *out = smp;
  return HCURL_OK;
}

int64_t hcurl_mpnn_sample_entries(hcurl_mpnn_sample s) { return s ? s->S.E : HCURL_EINVAL; }

int hcurl_mpnn_sample_export(hcurl_mpnn_sample s, float* features, double* p0, double* target) {
  if (!s) return HCURL_EINVAL;
  return guarded([&]() -> int {
    if (features) hc::d2h(features, s->S.X.p, s->S.E * hc::kNF, s->ctx);
    if (p0) hc::d2h(p0, s->S.p0.p, s->S.E, s->ctx);
    if (target) hc::d2h(target, s->S.target.p, s->S.E, s->ctx);
    return HCURL_OK;
  });
}

void hcurl_mpnn_sample_destroy(hcurl_mpnn_sample s) {
  if (!s) return;
  try { (void)hipStreamSynchronize(s->ctx.s); } catch (...) {}
  delete s;
}

int hcurl_mpnn_forward(hcurl_mpnn net, hcurl_mpnn_sample s, double* delta) {
  if (!net || !s || !delta) return HCURL_EINVAL;
  return guarded([&]() -> int {
    net->net.ctx.sync();
    hc::mpnn_forward(net->net, s->S, s->ctx, false);
    hc::d2h(delta, s->S.delta.p, s->S.E, s->ctx);
    s->S.release_workspace();
    return HCURL_OK;
  });
}

int hcurl_mpnn_loss_grad(hcurl_mpnn net, hcurl_mpnn_sample s, double* loss, float* grad) {
  if (!net || !s) return HCURL_EINVAL;
  return guarded([&]() -> int {
    net->net.ctx.sync();
    const double l = hc::mpnn_loss_grad(net->net, s->S, s->ctx);
    if (loss) *loss = l;
    if (grad) hc::d2h(grad, net->net.g.p, hc::kNParam, s->ctx);
    s->S.release_workspace();
    return HCURL_OK;
  });
}

int hcurl_mpnn_train_step(hcurl_mpnn net, hcurl_mpnn_sample s, float lr, float beta1, float beta2, float eps, int step,
                          double* loss) {
  if (!net || !s || step < 1) return HCURL_EINVAL;
  return guarded([&]() -> int {
    net->net.ctx.sync();
    const double l = hc::mpnn_loss_grad(net->net, s->S, s->ctx);
    hc::mpnn_adam(net->net, lr, beta1, beta2, eps, step, s->ctx);
    s->S.release_workspace();
    s->ctx.sync();
    if (loss) *loss = l;
    return HCURL_OK;
  });
}

const char* hcurl_last_error(void) { return g_last_error.c_str(); }

const char* hcurl_error_string(int code) {
  switch (code) {
    case HCURL_OK: return "ok";
    case HCURL_EINVAL: return "invalid argument";
    case HCURL_EHIP: return "HIP runtime error";
    case HCURL_ENOMEM: return "out of device memory";
    case HCURL_EREDUCIBLE: return "disconnected local coarse-edge graph";
    case HCURL_ENOTSPD: return "not positive definite";
    case HCURL_EMAXIT: return "maximum iterations reached";
    case HCURL_EUNSUPPORTED: return "size limit exceeded";
    case HCURL_ESTAGNATE: return "PCG stagnated: an iteration left the iterate unchanged";
    case HCURL_EINFEASIBLE: return "commuting constraint without finite solution";
    default: return "unknown error";
  }
}

}  // extern "C"
