// Message-passing network for the learned P^(e) initial guess: per-entry
// features, BF16 matrix-core (MFMA 32x32x16) dense layers with FP32
// accumulation, segment means over pattern rows and columns, MSE loss,
// backward pass and Adam.
#include <cmath>
#include <cstring>
#include <type_traits>

#include "mpnn.hpp"

namespace hc {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

// one 32x32x16 matrix-core product (gfx950): lane l supplies A[l % 32][k]
// and B[k][l % 32] for the eight k = k0 + 8 (l / 32) + v, v < 8, read as 16
// bytes from LDS rows of bf16; any fixed assignment of the k values works as
// long as A and B use the same one
__device__ __forceinline__ f32x16 mfma16(const uint16_t* a, const uint16_t* b, f32x16 acc) {
  return __builtin_amdgcn_mfma_f32_32x32x16_bf16(*(const bf16x8*)a, *(const bf16x8*)b, acc, 0, 0, 0);
}
__device__ __forceinline__ float bf2f(uint16_t v) { return __uint_as_float((uint32_t)v << 16); }

__device__ __forceinline__ uint16_t f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float silu_f(float x) { return x / (1.0f + expf(-x)); }
__device__ __forceinline__ float dsilu_f(float x) {
  const float s = 1.0f / (1.0f + expf(-x));
  return s * (1.0f + x * (1.0f - s));
}

// ---------------------------------------------------------------------------
// features of pattern entry e = (i, j); see the feature list in the header
// of the FP64 reference (same definitions)
// ---------------------------------------------------------------------------
__global__ void k_expand_rows(const int* __restrict__ rp, int n, int* __restrict__ row_of) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  for (int q = rp[i]; q < rp[i + 1]; ++q) row_of[q] = i;
}
__global__ void k_iota_d(double* __restrict__ v, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = (double)i;
}
__global__ void k_d2i(const double* __restrict__ v, int* __restrict__ o, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) o[i] = (int)v[i];
}
__global__ void k_centroid_sum(const double* __restrict__ x, const int* __restrict__ agg, int m, double* __restrict__ cen,
                               double* __restrict__ cnt) {
  int a = blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= m) return;
  const int I = agg[a];
  atomicAdd(&cen[3 * I + 0], x[3 * a + 0]);
  atomicAdd(&cen[3 * I + 1], x[3 * a + 1]);
  atomicAdd(&cen[3 * I + 2], x[3 * a + 2]);
  atomicAdd(&cnt[I], 1.0);
}
__global__ void k_centroid_div(double* __restrict__ cen, const double* __restrict__ cnt, int mH) {
  int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= mH) return;
  for (int d = 0; d < 3; ++d) cen[3 * I + d] /= cnt[I];
}

__device__ __forceinline__ double r_at(const int* __restrict__ Rrp, const int* __restrict__ Rcol,
                                       const double* __restrict__ Rval, int i, int I) {
  int lo = Rrp[i], hi = Rrp[i + 1] - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int c = Rcol[mid];
    if (c == I) return Rval[mid];
    if (c < I) lo = mid + 1; else hi = mid - 1;
  }
  return 0.0;
}

__global__ void k_features(int64_t E, const int* __restrict__ row_of, const int* __restrict__ col_of,
                           const int* __restrict__ Prp, const int* __restrict__ colptr, const int* __restrict__ tail,
                           const int* __restrict__ head, const int* __restrict__ ctail, const int* __restrict__ chead,
                           const double* __restrict__ x, const double* __restrict__ cen, const double* __restrict__ p0,
                           const double* __restrict__ pmin, const int* __restrict__ Rrp, const int* __restrict__ Rcol,
                           const double* __restrict__ Rval, const double* __restrict__ dinvA, const int* __restrict__ agg,
                           float* __restrict__ X) {
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int i = row_of[e], j = col_of[e];
  const int a = tail[i], b = head[i], I = ctail[j], K = chead[j];
  double t[3], mid[3], T[3], Mid[3];
  for (int d = 0; d < 3; ++d) {
    t[d] = x[3 * b + d] - x[3 * a + d];
    mid[d] = 0.5 * (x[3 * b + d] + x[3 * a + d]);
    T[d] = cen[3 * K + d] - cen[3 * I + d];
    Mid[d] = 0.5 * (cen[3 * K + d] + cen[3 * I + d]);
  }
  const double lt = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
  const double LT = sqrt(T[0] * T[0] + T[1] * T[1] + T[2] * T[2]);
  const double dm = sqrt((mid[0] - Mid[0]) * (mid[0] - Mid[0]) + (mid[1] - Mid[1]) * (mid[1] - Mid[1]) +
                         (mid[2] - Mid[2]) * (mid[2] - Mid[2]));
  float* f = X + e * kNF;
  f[0] = (float)p0[e];
  f[1] = (float)pmin[e];
  f[2] = (float)((t[0] * T[0] + t[1] * T[1] + t[2] * T[2]) / (lt * LT));
  f[3] = (float)(lt / LT);
  f[4] = (float)(dm / LT);
  f[5] = (float)((Prp[i + 1] - Prp[i]) / 16.0);
  f[6] = (float)((Rrp[i + 1] - Rrp[i]) / 8.0);
  f[7] = (float)((colptr[j + 1] - colptr[j]) / 256.0);
  f[8] = (float)r_at(Rrp, Rcol, Rval, i, I);
  f[9] = (float)r_at(Rrp, Rcol, Rval, i, K);
  const int ai = agg[a], bi = agg[b];
  f[10] = (ai == I || ai == K) ? 1.0f : 0.0f;
  f[11] = (bi == I || bi == K) ? 1.0f : 0.0f;
  f[12] = (float)(log10(1.0 / dinvA[i]) / 8.0);
  f[13] = 0.0f;
  f[14] = 0.0f;
  f[15] = 0.0f;
}

void mpnn_build_sample(Hierarchy& H, Level& L0, const Level& L1, const double* p0plain, const double* pmin, Sample& S) {
  if (L0.nsingle > 0) fail(HCURL_EUNSUPPORTED, "the learned initial guess does not take Dirichlet edges");
  Ctx& c = H.ctx;
  if (!H.coords.p) fail(HCURL_EINVAL, "the learned initial guess needs node coordinates at setup");
  S.s = c.s;
  S.E = L0.Pe.nnz;
  S.nrow = L0.n;
  S.ncol = L0.Pe.ncols;
  const int64_t E = S.E;
  S.rowptr.alloc(L0.n + 1, c.s);
  d2d(S.rowptr.p, L0.Pe.rowptr.p, L0.n + 1, c);
  S.row_of.alloc(E, c.s);
  S.col_of.alloc(E, c.s);
  d2d(S.col_of.p, L0.Pe.col.p, E, c);
  k_expand_rows<<<ceil_div(L0.n, 256), 256, 0, c.s>>>(L0.Pe.rowptr.p, L0.n, S.row_of.p);
  HC_LAUNCH_CHECK();
  {  // entries grouped by column: transpose of the pattern carrying entry ids
    Csr P, PT;
    P.nrows = L0.n; P.ncols = S.ncol; P.nnz = E;
    P.rowptr.alloc(L0.n + 1, c.s); P.col.alloc(E, c.s); P.val.alloc(E, c.s);
    d2d(P.rowptr.p, L0.Pe.rowptr.p, L0.n + 1, c);
    d2d(P.col.p, L0.Pe.col.p, E, c);
    k_iota_d<<<ceil_div(E, 256), 256, 0, c.s>>>(P.val.p, E);
    HC_LAUNCH_CHECK();
    transpose(P, PT, true, c);
    S.colptr = std::move(PT.rowptr);
    S.colidx.alloc(E, c.s);
    k_d2i<<<ceil_div(E, 256), 256, 0, c.s>>>(PT.val.p, S.colidx.p, E);
    HC_LAUNCH_CHECK();
  }
  const int mH = L1.m;
  DBuf<double> cen(3 * (size_t)mH, c.s), cnt(mH, c.s);
  fill(cen.p, 0.0, 3 * (int64_t)mH, c);
  fill(cnt.p, 0.0, mH, c);
  k_centroid_sum<<<ceil_div(L0.m, 256), 256, 0, c.s>>>(H.coords.p, L0.agg.p, L0.m, cen.p, cnt.p);
  HC_LAUNCH_CHECK();
  k_centroid_div<<<ceil_div(mH, 256), 256, 0, c.s>>>(cen.p, cnt.p, mH);
  HC_LAUNCH_CHECK();
  S.X.alloc(E * kNF, c.s);
  c.run("mpnn_features", 100.0 * E, [&] {
    k_features<<<ceil_div(E, 256), 256, 0, c.s>>>(E, S.row_of.p, S.col_of.p, L0.Pe.rowptr.p, S.colptr.p, L0.tail.p,
                                                  L0.head.p, L1.tail.p, L1.head.p, H.coords.p, cen.p, p0plain, pmin,
                                                  L0.R.rowptr.p, L0.R.col.p, L0.R.val.p, L0.dinvA.p, L0.agg.p, S.X.p);
  });
  S.p0.alloc(E, c.s);
  d2d(S.p0.p, p0plain, E, c);
}

// ---------------------------------------------------------------------------
// dense layers on the matrix cores.  Tiles of 64 entries x 64 outputs, four
// waves each computing a 32x32 block with v_mfma_f32_32x32x16_bf16 (mfma16);
// accumulator r of lane l is element (8(r/4) + 4(l/32) + r%4, l%32).
// ---------------------------------------------------------------------------
// Z row of entry e for layer input: MODE 0 the features, MODE 1 the
// concatenation [h_e, mean_row(i(e)), mean_col(j(e))].
template <int K, int MODE>
__device__ __forceinline__ float z_value(int64_t e, int k, const float* __restrict__ X, const float* __restrict__ hin,
                                         const float* __restrict__ mr, const float* __restrict__ mc,
                                         const int* __restrict__ row_of, const int* __restrict__ col_of) {
  if (MODE == 0) return X[e * K + k];
  if (k < kHD) return hin[e * kHD + k];
  if (k < 2 * kHD) return mr[(int64_t)row_of[e] * kHD + (k - kHD)];
  return mc[(int64_t)col_of[e] * kHD + (k - 2 * kHD)];
}

// Storage of the activations: FP32 (training keeps them for the backward
// pass) or BF16 (inference: the products take BF16 operands anyway, and the
// layer moves half the bytes).
__device__ __forceinline__ uint16_t to_store(float v, uint16_t*) { return f2bf(v); }
__device__ __forceinline__ float to_store(float v, float*) { return v; }

// The Z row of an entry is staged in 16-byte pieces: 4 FP32 or 8 BF16 values
// of the features (MODE 0) or of [h, mean_row, mean_col] (MODE 1, 2).
template <int K, int MODE, class IT>
__device__ __forceinline__ void layer_load(int64_t E, int64_t e0, int t, const IT* __restrict__ zin,
                                           const IT* __restrict__ mr, const IT* __restrict__ mc,
                                           const int* __restrict__ row_of, const int* __restrict__ col_of, uint4* v) {
  constexpr int PW = 16 / sizeof(IT);
  constexpr int NP = K / PW;
  constexpr int PER = 64 * NP / 256;
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int j = t + 256 * u;
    const int r = j / NP, kz = (j - r * NP) * PW;
    const int64_t e = e0 + r;
    v[u] = make_uint4(0u, 0u, 0u, 0u);
    if (e < E) {
      const IT* src;
      if (MODE == 0) {
        src = zin + e * K + kz;
      } else {
        const int seg = kz / kHD, f = kz % kHD;
        src = seg == 0 ? zin + e * kHD + f
                       : seg == 1 ? mr + (int64_t)row_of[e] * kHD + f : mc + (int64_t)col_of[e] * kHD + f;
      }
      v[u] = *(const uint4*)src;
    }
  }
}

// Persistent form of the dense layer: every block loads W^T into LDS once and
// then takes 64-entry tiles in turn.  Each thread stages whole 16-byte pieces
// of the Z rows in LDS; the pieces of the next tile are loaded while the
// current one is multiplied; the residual term reads the tile's h rows (FP32
// inputs keep an FP32 copy in LDS).  MODE 0: Z = features (K = 16, FP32).  MODE 1: Z = [h, mean_row,
// mean_col] (K = 192), output h + silu(Z W + b).  MODE 2: as MODE 1, and the
// head delta = h_out . w_out + b_out is formed in place of writing h_out.
// HT: storage type of h and the means (float, or uint16_t holding BF16).
template <int K, int MODE, class HT>
__global__ void __launch_bounds__(256) k_mpnn_layer(int64_t E, const float* __restrict__ X, const HT* __restrict__ hin,
                                                    const HT* __restrict__ mr, const HT* __restrict__ mc,
                                                    const int* __restrict__ row_of, const int* __restrict__ col_of,
                                                    const uint16_t* __restrict__ Wt, const float* __restrict__ bias,
                                                    const float* __restrict__ wout, float* __restrict__ U,
                                                    HT* __restrict__ hout, double* __restrict__ delta) {
  using IT = typename std::conditional<MODE == 0, float, HT>::type;
  constexpr bool IBF = sizeof(IT) == 2;
  constexpr int PW = 16 / sizeof(IT);
  constexpr int NP = K / PW;
  constexpr int PER = 64 * NP / 256;
  static_assert((64 * NP) % 256 == 0 && K % 16 == 0, "tile staging");
  constexpr int KP = K + 8;
  // FP32 inputs keep their h rows in LDS for the residual; BF16 inputs read
  // them back from the staged tile (the stored values themselves)
  constexpr int HR = (MODE && !IBF) ? 64 : 1;
  __shared__ __attribute__((aligned(16))) uint16_t Zs[64][KP];
  __shared__ __attribute__((aligned(16))) uint16_t Ws[64][KP];
  __shared__ __attribute__((aligned(16))) float Hs[HR][kHD + 4];
  __shared__ float red[64][2];
  const int t = threadIdx.x;
  for (int q = t; q < 64 * K; q += 256) Ws[q / K][q % K] = Wt[q];
  const int w = t >> 6, l = t & 63;
  const int mt = w >> 1, nt = w & 1;
  const int col = nt * 32 + (l & 31);
  const float bcol = bias[col];
  const float wcol = MODE == 2 ? wout[col] : 0.0f;
  const float bout = MODE == 2 ? wout[kHD] : 0.0f;
  const IT* zin;
  if constexpr (MODE == 0) zin = X; else zin = hin;
  const int64_t ntiles = (E + 63) / 64;
  uint4 v[PER];
  int64_t tile = blockIdx.x;
  const IT* mri = reinterpret_cast<const IT*>(mr);
  const IT* mci = reinterpret_cast<const IT*>(mc);
  if (tile < ntiles) layer_load<K, MODE, IT>(E, tile * 64, t, zin, mri, mci, row_of, col_of, v);
  for (; tile < ntiles; tile += gridDim.x) {
    const int64_t e0 = tile * 64;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int j = t + 256 * u;
      const int r = j / NP, kz = (j - r * NP) * PW;
      if constexpr (IBF) {
        *(uint4*)&Zs[r][kz] = v[u];
      } else {
        const float* fv = (const float*)&v[u];
        uint2 packed;
        packed.x = (uint32_t)f2bf(fv[0]) | ((uint32_t)f2bf(fv[1]) << 16);
        packed.y = (uint32_t)f2bf(fv[2]) | ((uint32_t)f2bf(fv[3]) << 16);
        *(uint2*)&Zs[r][kz] = packed;
        if (HR > 1 && kz < kHD) *(float4*)&Hs[r][kz] = *(const float4*)fv;
      }
    }
    __syncthreads();
    // next tile's pieces are in flight during the products and the epilogue
    const int64_t next = tile + gridDim.x;
    if (next < ntiles) layer_load<K, MODE, IT>(E, next * 64, t, zin, mri, mci, row_of, col_of, v);
    f32x16 acc;
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
    for (int kk = 0; kk < K; kk += 16)
      acc = mfma16(&Zs[mt * 32 + (l & 31)][kk + 8 * (l >> 5)], &Ws[col][kk + 8 * (l >> 5)], acc);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int row = mt * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
      const int64_t e = e0 + row;
      const bool ok = e < E;
      const float u = acc[r] + bcol;
      float hres = 0.0f;
      if constexpr (MODE != 0) hres = HR > 1 ? Hs[HR > 1 ? row : 0][col] : bf2f(Zs[row][col]);
      const float hv = hres + silu_f(u);
      if (MODE == 2) {
        float d = ok ? hv * wcol : 0.0f;
#pragma unroll
        for (int o = 16; o > 0; o >>= 1) d += __shfl_xor(d, o, 32);
        if ((l & 31) == 0) red[row][nt] = d;
      } else if (ok) {
        if (U) U[e * kHD + col] = u;
        hout[e * kHD + col] = to_store(hv, hout);
      }
    }
    if (MODE == 2) {
      __syncthreads();
      if (t < 64 && e0 + t < E) delta[e0 + t] = (double)(red[t][0] + red[t][1] + bout);
    }
    __syncthreads();
  }
}

// up to three resident blocks per CU (LDS: two 64-row tiles of bf16)
static int layer_grid(int64_t E) {
  const int64_t tiles = (E + 63) / 64;
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, 256 * 3));
}

// dZ = du W^T: du (E x 64), W (192 x 64) bf16 row-major, dz (E x 192); grid.y
// picks the 64-column slice of dz.
__global__ void __launch_bounds__(256) k_mpnn_dz(int64_t E, const float* __restrict__ du, const uint16_t* __restrict__ Wr,
                                                 float* __restrict__ dz) {
  __shared__ __attribute__((aligned(16))) uint16_t As[64][kHD + 8];
  __shared__ __attribute__((aligned(16))) uint16_t Bs[64][kHD + 8];
  const int t = threadIdx.x;
  const int64_t e0 = (int64_t)blockIdx.x * 64;
  const int n0 = blockIdx.y * 64;
  for (int q = t; q < 64 * kHD; q += 256) {
    const int r = q / kHD, k = q % kHD;
    const int64_t e = e0 + r;
    As[r][k] = f2bf(e < E ? du[e * kHD + k] : 0.0f);
    Bs[r][k] = Wr[(int64_t)(n0 + r) * kHD + k];
  }
  __syncthreads();
  const int w = t >> 6, l = t & 63;
  const int mt = w >> 1, nt = w & 1;
  f32x16 acc;
#pragma unroll
  for (int r = 0; r < 16; ++r) acc[r] = 0.0f;
#pragma unroll
  for (int kk = 0; kk < kHD; kk += 16)
    acc = mfma16(&As[mt * 32 + (l & 31)][kk + 8 * (l >> 5)], &Bs[nt * 32 + (l & 31)][kk + 8 * (l >> 5)], acc);
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int row = mt * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
    const int col = nt * 32 + (l & 31);
    const int64_t e = e0 + row;
    if (e < E) dz[e * kKZ + n0 + col] = acc[r];
  }
}

// Partial weight gradient over a run of entries: dW (K x 64) += Z^T du,
// db (64) += sum du.  The entry dimension is the MFMA reduction dimension.
template <int K, int MODE>
__global__ void __launch_bounds__(256) k_mpnn_wgrad(int64_t E, int chunks, const float* __restrict__ X,
                                                    const float* __restrict__ hin, const float* __restrict__ mr,
                                                    const float* __restrict__ mc, const int* __restrict__ row_of,
                                                    const int* __restrict__ col_of, const float* __restrict__ du,
                                                    float* __restrict__ part) {
  constexpr int MP = (K + 31) / 32 * 32;
  constexpr int NT = (MP / 32) * 2;  // 32x32 output tiles
  constexpr int PER = (NT + 3) / 4;  // tiles per wave
  __shared__ __attribute__((aligned(16))) uint16_t Zt[MP][64 + 8];
  __shared__ __attribute__((aligned(16))) uint16_t Dt[kHD][64 + 8];
  const int t = threadIdx.x;
  const int w = t >> 6, l = t & 63;
  f32x16 acc[PER];
#pragma unroll
  for (int s = 0; s < PER; ++s)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[s][r] = 0.0f;
  float bsum = 0.0f;
  for (int cidx = 0; cidx < chunks; ++cidx) {
    const int64_t e0 = ((int64_t)blockIdx.x * chunks + cidx) * 64;
    if (e0 >= E) break;
    for (int q = t; q < 64 * MP; q += 256) {
      const int el = q / MP, zf = q % MP;
      const int64_t e = e0 + el;
      Zt[zf][el] = f2bf((zf < K && e < E) ? z_value<K, MODE>(e, zf, X, hin, mr, mc, row_of, col_of) : 0.0f);
    }
    for (int q = t; q < 64 * kHD; q += 256) {
      const int el = q / kHD, hid = q % kHD;
      const int64_t e = e0 + el;
      Dt[hid][el] = f2bf(e < E ? du[e * kHD + hid] : 0.0f);
    }
    if (t < kHD)
      for (int el = 0; el < 64 && e0 + el < E; ++el) bsum += du[(e0 + el) * kHD + t];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int ti = w + 4 * s;
      if (ti < NT) {
        const int tm = ti >> 1, tn = ti & 1;
#pragma unroll
        for (int kk = 0; kk < 64; kk += 16)
          acc[s] = mfma16(&Zt[tm * 32 + (l & 31)][kk + 8 * (l >> 5)], &Dt[tn * 32 + (l & 31)][kk + 8 * (l >> 5)], acc[s]);
      }
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * (K * kHD + kHD);
#pragma unroll
  for (int s = 0; s < PER; ++s) {
    const int ti = w + 4 * s;
    if (ti < NT) {
      const int tm = ti >> 1, tn = ti & 1;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int i = tm * 32 + 8 * (r >> 2) + 4 * (l >> 5) + (r & 3);
        const int j = tn * 32 + (l & 31);
        if (i < K) out[i * kHD + j] = acc[s][r];
      }
    }
  }
  if (t < kHD) out[K * kHD + t] = bsum;
}

// out[k] = sum over blocks of part[b * stride + k] (fixed order)
__global__ void k_sum_blocks(const float* __restrict__ part, int nb, int stride, float* __restrict__ out) {
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= stride) return;
  float s = 0.0f;
  for (int b = 0; b < nb; ++b) s += part[(int64_t)b * stride + k];
  out[k] = s;
}

// mean over segments: dst[s][f] = mean of src[e][off + f] over the segment's
// entries (idx maps positions to entries, NULL = identity); one wave per
// segment, sums in FP32 whatever the storage type T.  The wave reads four
// entries at a time, a quarter-wave per entry and four features per lane (8
// or 16 bytes), so quarter g holds the partial sum of the entries at
// positions g mod 4 of every complete group of four (the remainder goes to
// quarter 0); the quarters combine as (s0 + s1) + (s2 + s3).
template <class T> struct Vec4;
template <> struct Vec4<float> {
  using V = float4;
  static __device__ __forceinline__ void add(float* acc, V v) { acc[0] += v.x; acc[1] += v.y; acc[2] += v.z; acc[3] += v.w; }
  static __device__ __forceinline__ V pack(const float* r) { return make_float4(r[0], r[1], r[2], r[3]); }
};
template <> struct Vec4<uint16_t> {
  using V = uint2;
  static __device__ __forceinline__ void add(float* acc, V v) {
    acc[0] += bf2f((uint16_t)(v.x & 0xffffu)); acc[1] += bf2f((uint16_t)(v.x >> 16));
    acc[2] += bf2f((uint16_t)(v.y & 0xffffu)); acc[3] += bf2f((uint16_t)(v.y >> 16));
  }
  static __device__ __forceinline__ V pack(const float* r) {
    return make_uint2((uint32_t)f2bf(r[0]) | ((uint32_t)f2bf(r[1]) << 16), (uint32_t)f2bf(r[2]) | ((uint32_t)f2bf(r[3]) << 16));
  }
};
template <class T>
__global__ void __launch_bounds__(256) k_seg_mean(int nseg, const int* __restrict__ ptr, const int* __restrict__ idx,
                                                  const T* __restrict__ src, int stride, int off,
                                                  T* __restrict__ dst) {
  using W = Vec4<T>;
  const int sgi = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4;
  const int f0 = (lane & 15) * 4;
  if (sgi >= nseg) return;
  const int a = ptr[sgi], b = ptr[sgi + 1];
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  int q = a;
#pragma unroll 4
  for (; q + 3 < b; q += 4) {
    const int64_t e = idx ? idx[q + g] : q + g;
    W::add(acc, *(const typename W::V*)(src + e * stride + off + f0));
  }
  if (g == 0)
    for (; q < b; ++q) {
      const int64_t e = idx ? idx[q] : q;
      W::add(acc, *(const typename W::V*)(src + e * stride + off + f0));
    }
  float r[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const float s = acc[i] + __shfl_xor(acc[i], 16, 64);  // quarters 0+1 and 2+3
    const float t = s + __shfl_xor(s, 32, 64);            // (0+1) + (2+3)
    r[i] = b > a ? t / (float)(b - a) : 0.0f;
  }
  if (g == 0) *(typename W::V*)(dst + (int64_t)sgi * kHD + f0) = W::pack(r);
}

// delta_e = h_e . w_out + b_out; with training: residual, loss, dh = dd w_out,
// and partial sums of the head gradient (one wave per entry, lane = feature)
__global__ void __launch_bounds__(256) k_head(int64_t E, const float* __restrict__ h, const float* __restrict__ w,
                                              const double* __restrict__ p0, const double* __restrict__ target,
                                              double* __restrict__ delta, float* __restrict__ dh,
                                              float* __restrict__ part /* per block: 64 gw, gb, loss */) {
  __shared__ float sg[4][kHD + 2];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const float wf = w[lane];
  const float bo = w[kHD];
  float gw = 0.0f, gb = 0.0f, ls = 0.0f;
  const int64_t nw = (int64_t)gridDim.x * 4;
  for (int64_t e = (int64_t)blockIdx.x * 4 + wv; e < E; e += nw) {
    const float hv = h[e * kHD + lane];
    const float d = wave_sum(hv * wf) + bo;
    if (lane == 0) delta[e] = (double)d;
    if (target) {
      const double res = p0[e] + (double)d - target[e];
      const float dd = (float)(2.0 * res / (double)E);
      dh[e * kHD + lane] = dd * wf;
      gw += dd * hv;
      gb += dd;
      ls += (float)(res * res);
    }
  }
  if (!target) return;
  sg[wv][lane] = gw;
  if (lane == 0) { sg[wv][kHD] = gb; sg[wv][kHD + 1] = ls; }
  __syncthreads();
  if (threadIdx.x < kHD + 2) {
    const int k = threadIdx.x;
    part[(int64_t)blockIdx.x * (kHD + 2) + k] = (sg[0][k] + sg[1][k]) + (sg[2][k] + sg[3][k]);
  }
}

__global__ void k_du(int64_t n, const float* __restrict__ dh, const float* __restrict__ u, float* __restrict__ du) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) du[i] = dh[i] * dsilu_f(u[i]);
}

// dh_e += dz_e[0:64] + mdr[i(e)] + mdc[j(e)]
__global__ void k_dh_combine(int64_t E, float* __restrict__ dh, const float* __restrict__ dz, const float* __restrict__ mdr,
                             const float* __restrict__ mdc, const int* __restrict__ row_of,
                             const int* __restrict__ col_of) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= E * kHD) return;
  const int64_t e = q / kHD;
  const int f = (int)(q % kHD);
  dh[q] += dz[e * kKZ + f] + mdr[(int64_t)row_of[e] * kHD + f] + mdc[(int64_t)col_of[e] * kHD + f];
}

__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// bf16 copies: transposed (out x in) for forward products, plain for dZ
__global__ void k_to_bf16_t(const float* __restrict__ W, int rows, int cols, uint16_t* __restrict__ Wt) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= rows * cols) return;
  const int r = q / cols, c = q % cols;
  Wt[(int64_t)c * rows + r] = f2bf(W[q]);
}
__global__ void k_to_bf16(const float* __restrict__ W, int n, uint16_t* __restrict__ Wb) {
  int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) Wb[q] = f2bf(W[q]);
}

void Net::refresh_bf16(Ctx& c) {
  k_to_bf16_t<<<ceil_div(kNF * kHD, 256), 256, 0, c.s>>>(w.p + kOffWin, kNF, kHD, wt_in.p);
  for (int l = 0; l < kNL; ++l) {
    k_to_bf16_t<<<ceil_div(kKZ * kHD, 256), 256, 0, c.s>>>(w.p + off_W(l), kKZ, kHD, wt[l].p);
    k_to_bf16<<<ceil_div(kKZ * kHD, 256), 256, 0, c.s>>>(w.p + off_W(l), kKZ * kHD, wr[l].p);
  }
  HC_LAUNCH_CHECK();
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static void check_mean_layout(int stride, int off) {
  // k_seg_mean reads four features per lane with one 8- or 16-byte load
  if (stride % 4 || off % 4) fail(HCURL_EINVAL, "segment mean: feature stride and offset must be multiples of 4");
}
template <class T>
static void row_mean(Sample& S, const T* src, int stride, int off, T* mr, Ctx& c) {
  check_mean_layout(stride, off);
  // the entries' features once, the means written, the row pointers
  const double bytes = (double)sizeof(T) * kHD * ((double)S.E + S.nrow) + 4.0 * (S.nrow + 1);
  c.run("mpnn_segment_mean", bytes, [&] {
    k_seg_mean<T><<<ceil_div((int64_t)S.nrow * 64, 256), 256, 0, c.s>>>(S.nrow, S.rowptr.p, nullptr, src, stride, off, mr);
  });
}
template <class T>
static void col_mean(Sample& S, const T* src, int stride, int off, T* mc, Ctx& c) {
  check_mean_layout(stride, off);
  // the entries' features once (gathered through colidx), the means written
  const double bytes = (double)sizeof(T) * kHD * ((double)S.E + S.ncol) + 4.0 * (S.E + S.ncol + 1);
  c.run("mpnn_segment_mean", bytes, [&] {
    k_seg_mean<T><<<ceil_div((int64_t)S.ncol * 64, 256), 256, 0, c.s>>>(S.ncol, S.colptr.p, S.colidx.p, src, stride, off, mc);
  });
}

// Debug form of the dense products (Net::fp32_products): FP32 operands and
// master weights, no BF16 rounding, plain FMAs; the long reductions over the
// entries (weight gradients) accumulate in FP64.  One thread per output.
template <int K, int MODE>
__global__ void k_dense_f32(int64_t E, const float* __restrict__ X, const float* __restrict__ hin,
                            const float* __restrict__ mr, const float* __restrict__ mc, const int* __restrict__ row_of,
                            const int* __restrict__ col_of, const float* __restrict__ W, const float* __restrict__ bias,
                            float* __restrict__ U, float* __restrict__ hout) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= E * kHD) return;
  const int64_t e = q / kHD;
  const int col = (int)(q % kHD);
  float u = bias[col];
  for (int k = 0; k < K; ++k) u += z_value<K, MODE>(e, k, X, hin, mr, mc, row_of, col_of) * W[k * kHD + col];
  U[q] = u;
  hout[q] = (MODE ? hin[q] : 0.0f) + silu_f(u);
}
// dz[e][k] = sum_h du[e][h] W[k][h], k < 192
__global__ void k_dz_f32(int64_t E, const float* __restrict__ du, const float* __restrict__ W, float* __restrict__ dz) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= E * kKZ) return;
  const int64_t e = q / kKZ;
  const int k = (int)(q % kKZ);
  float s = 0.0f;
  for (int h = 0; h < kHD; ++h) s += du[e * kHD + h] * W[k * kHD + h];
  dz[q] = s;
}
// g[k][h] = sum_e Z[e][k] du[e][h] for k < K, and g[K][h] = sum_e du[e][h]
template <int K, int MODE>
__global__ void k_wgrad_f32(int64_t E, const float* __restrict__ X, const float* __restrict__ hin,
                            const float* __restrict__ mr, const float* __restrict__ mc, const int* __restrict__ row_of,
                            const int* __restrict__ col_of, const float* __restrict__ du, float* __restrict__ g) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (K + 1) * kHD) return;
  const int k = q / kHD, h = q % kHD;
  double s = 0.0;
  for (int64_t e = 0; e < E; ++e)
    s += (double)(k < K ? z_value<K, MODE>(e, k, X, hin, mr, mc, row_of, col_of) : 1.0f) * (double)du[e * kHD + h];
  g[q] = (float)s;
}

// The layers on activation buffers of storage type HT: h[l] / h[l + 1] are
// the input and output of layer l, mr[l] / mc[l] its row and column means.
// With `keep` (training) every buffer is distinct and the pre-activations go
// to S.u; otherwise buffers alternate and the head is fused into the last
// layer.
template <class HT>
static void forward_layers(Net& net, Sample& S, Ctx& c, bool keep, HT* const* h, HT* const* mr, HT* const* mc) {
  const int64_t E = S.E;
  const int lg = layer_grid(E);
  c.run("mpnn_dense_in_flop", 2.0 * E * kNF * kHD, [&] {
    k_mpnn_layer<kNF, 0, HT><<<lg, 256, 0, c.s>>>(E, S.X.p, nullptr, nullptr, nullptr, nullptr, nullptr, net.wt_in.p,
                                                  net.w.p + kOffBin, nullptr, keep ? S.u[0].p : nullptr, h[0], nullptr);
  });
  for (int l = 0; l < kNL; ++l) {
    HT* hin = h[l];
    HT* hout = h[l + 1];
    row_mean(S, (const HT*)hin, kHD, 0, mr[l], c);
    col_mean(S, (const HT*)hin, kHD, 0, mc[l], c);
    const bool last_fused = !keep && l == kNL - 1;  // inference: the head is formed in the last layer
    c.run("mpnn_dense_flop", 2.0 * E * kKZ * kHD, [&] {
      if (last_fused)
        k_mpnn_layer<kKZ, 2, HT><<<lg, 256, 0, c.s>>>(E, nullptr, hin, mr[l], mc[l], S.row_of.p, S.col_of.p, net.wt[l].p,
                                                      net.w.p + off_b(l), net.w.p + kOffWout, nullptr, nullptr, S.delta.p);
      else
        k_mpnn_layer<kKZ, 1, HT><<<lg, 256, 0, c.s>>>(E, nullptr, hin, mr[l], mc[l], S.row_of.p, S.col_of.p, net.wt[l].p,
                                                      net.w.p + off_b(l), nullptr, keep ? S.u[l + 1].p : nullptr, hout,
                                                      nullptr);
    });
  }
}

void mpnn_forward(Net& net, Sample& S, Ctx& c, bool keep) {
  const int64_t E = S.E;
  if (S.delta.n != (size_t)E) S.delta.alloc(E, c.s);
  if (keep || net.fp32_products) {
    // training: FP32 activations, all kept for the backward pass
    for (int k = 0; k <= kNL; ++k) {
      if (S.h[k].n != (size_t)(E * kHD)) S.h[k].alloc(E * kHD, c.s);
      if (S.u[k].n != (size_t)(E * kHD)) S.u[k].alloc(E * kHD, c.s);
    }
    for (int l = 0; l < kNL; ++l) {
      if (S.mr[l].n != (size_t)S.nrow * kHD) S.mr[l].alloc((size_t)S.nrow * kHD, c.s);
      if (S.mc[l].n != (size_t)S.ncol * kHD) S.mc[l].alloc((size_t)S.ncol * kHD, c.s);
    }
    float* h[kNL + 1];
    float* mr[kNL];
    float* mc[kNL];
    for (int k = 0; k <= kNL; ++k) h[k] = S.h[k].p;
    for (int l = 0; l < kNL; ++l) { mr[l] = S.mr[l].p; mc[l] = S.mc[l].p; }
    if (net.fp32_products) {
      const int g = ceil_div(E * kHD, 256);
      k_dense_f32<kNF, 0><<<g, 256, 0, c.s>>>(E, S.X.p, nullptr, nullptr, nullptr, nullptr, nullptr, net.w.p + kOffWin,
                                              net.w.p + kOffBin, S.u[0].p, h[0]);
      HC_LAUNCH_CHECK();
      for (int l = 0; l < kNL; ++l) {
        row_mean(S, (const float*)h[l], kHD, 0, mr[l], c);
        col_mean(S, (const float*)h[l], kHD, 0, mc[l], c);
        k_dense_f32<kKZ, 1><<<g, 256, 0, c.s>>>(E, nullptr, h[l], mr[l], mc[l], S.row_of.p, S.col_of.p, net.w.p + off_W(l),
                                                net.w.p + off_b(l), S.u[l + 1].p, h[l + 1]);
        HC_LAUNCH_CHECK();
      }
    } else {
      forward_layers<float>(net, S, c, true, h, mr, mc);
    }
    c.run("mpnn_head", 4.0 * E * kHD, [&] {
      k_head<<<1024, 256, 0, c.s>>>(E, S.h[kNL].p, net.w.p + kOffWout, nullptr, nullptr, S.delta.p, nullptr, nullptr);
    });
    return;
  }
  // inference: BF16 activations in two alternating buffers
  for (int k = 0; k < 2; ++k)
    if (S.hb[k].n != (size_t)(E * kHD)) S.hb[k].alloc(E * kHD, c.s);
  if (S.mrb.n != (size_t)S.nrow * kHD) S.mrb.alloc((size_t)S.nrow * kHD, c.s);
  if (S.mcb.n != (size_t)S.ncol * kHD) S.mcb.alloc((size_t)S.ncol * kHD, c.s);
  uint16_t* h[kNL + 1];
  uint16_t* mr[kNL];
  uint16_t* mc[kNL];
  for (int k = 0; k <= kNL; ++k) h[k] = S.hb[k & 1].p;
  for (int l = 0; l < kNL; ++l) { mr[l] = S.mrb.p; mc[l] = S.mcb.p; }
  forward_layers<uint16_t>(net, S, c, false, h, mr, mc);
}

double mpnn_loss_grad(Net& net, Sample& S, Ctx& c) {
  if (!S.target.p) fail(HCURL_EINVAL, "sample has no target");
  const int64_t E = S.E;
  mpnn_forward(net, S, c, true);
  if (S.dh.n != (size_t)(E * kHD)) { S.dh.alloc(E * kHD, c.s); S.du.alloc(E * kHD, c.s); }
  if (S.dz.n != (size_t)(E * kKZ)) S.dz.alloc(E * kKZ, c.s);
  if (S.mdr.n != (size_t)S.nrow * kHD) S.mdr.alloc((size_t)S.nrow * kHD, c.s);
  if (S.mdc.n != (size_t)S.ncol * kHD) S.mdc.alloc((size_t)S.ncol * kHD, c.s);
  // head: loss, dh, gradient of w_out and b_out
  DBuf<float> hpart(1024 * (kHD + 2), c.s), hsum(kHD + 2, c.s);
  c.run("mpnn_head", 12.0 * E * kHD, [&] {
    k_head<<<1024, 256, 0, c.s>>>(E, S.h[kNL].p, net.w.p + kOffWout, S.p0.p, S.target.p, S.delta.p, S.dh.p, hpart.p);
  });
  k_sum_blocks<<<1, 128, 0, c.s>>>(hpart.p, 1024, kHD + 2, hsum.p);
  HC_LAUNCH_CHECK();
  d2d(net.g.p + kOffWout, hsum.p, kHD + 1, c);
  float hl[kHD + 2];
  d2h(hl, hsum.p, kHD + 2, c);
  const double loss = (double)hl[kHD + 1] / (double)E;
  // message layers, top down
  const int chunks = 16;
  const int nbw = ceil_div(E, 64 * chunks);
  DBuf<float> wpart((size_t)nbw * (kKZ * kHD + kHD), c.s);
  const int nb = ceil_div(E, 64);
  for (int l = kNL - 1; l >= 0; --l) {
    c.run("mpnn_du", 12.0 * E * kHD, [&] { k_du<<<ceil_div(E * kHD, 256), 256, 0, c.s>>>(E * kHD, S.dh.p, S.u[l + 1].p, S.du.p); });
    if (net.fp32_products) {
      k_wgrad_f32<kKZ, 1><<<ceil_div((kKZ + 1) * kHD, 256), 256, 0, c.s>>>(E, nullptr, S.h[l].p, S.mr[l].p, S.mc[l].p,
                                                                          S.row_of.p, S.col_of.p, S.du.p,
                                                                          net.g.p + off_W(l));
      k_dz_f32<<<ceil_div(E * kKZ, 256), 256, 0, c.s>>>(E, S.du.p, net.w.p + off_W(l), S.dz.p);
      HC_LAUNCH_CHECK();
    } else {
      c.run("mpnn_dense_wgrad_flop", 2.0 * E * kKZ * kHD, [&] {
        k_mpnn_wgrad<kKZ, 1><<<nbw, 256, 0, c.s>>>(E, chunks, nullptr, S.h[l].p, S.mr[l].p, S.mc[l].p, S.row_of.p,
                                                   S.col_of.p, S.du.p, wpart.p);
      });
      k_sum_blocks<<<ceil_div(kKZ * kHD + kHD, 256), 256, 0, c.s>>>(wpart.p, nbw, kKZ * kHD + kHD, net.g.p + off_W(l));
      HC_LAUNCH_CHECK();
      c.run("mpnn_dense_dz_flop", 2.0 * E * kKZ * kHD, [&] {
        k_mpnn_dz<<<dim3(nb, 3), 256, 0, c.s>>>(E, S.du.p, net.wr[l].p, S.dz.p);
      });
    }
    // adjoints of the gathered means: average the row slice over rows and
    // the column slice over columns
    row_mean(S, S.dz.p, kKZ, kHD, S.mdr.p, c);
    col_mean(S, S.dz.p, kKZ, 2 * kHD, S.mdc.p, c);
    c.run("mpnn_dh", 16.0 * E * kHD, [&] {
      k_dh_combine<<<ceil_div(E * kHD, 256), 256, 0, c.s>>>(E, S.dh.p, S.dz.p, S.mdr.p, S.mdc.p, S.row_of.p, S.col_of.p);
    });
  }
  // input layer
  c.run("mpnn_du", 12.0 * E * kHD, [&] { k_du<<<ceil_div(E * kHD, 256), 256, 0, c.s>>>(E * kHD, S.dh.p, S.u[0].p, S.du.p); });
  if (net.fp32_products) {
    k_wgrad_f32<kNF, 0><<<ceil_div((kNF + 1) * kHD, 256), 256, 0, c.s>>>(E, S.X.p, nullptr, nullptr, nullptr, nullptr,
                                                                        nullptr, S.du.p, net.g.p + kOffWin);
  } else {
    c.run("mpnn_dense_wgrad_flop", 2.0 * E * kNF * kHD, [&] {
      k_mpnn_wgrad<kNF, 0><<<nbw, 256, 0, c.s>>>(E, chunks, S.X.p, nullptr, nullptr, nullptr, nullptr, nullptr, S.du.p,
                                                 wpart.p);
    });
    k_sum_blocks<<<ceil_div(kNF * kHD + kHD, 256), 256, 0, c.s>>>(wpart.p, nbw, kNF * kHD + kHD, net.g.p + kOffWin);
  }
  HC_LAUNCH_CHECK();
  c.sync();
  return loss;
}

void mpnn_adam(Net& net, float lr, float b1, float b2, float eps, int step, Ctx& c) {
  const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
  k_adam<<<ceil_div(kNParam, 256), 256, 0, c.s>>>(kNParam, net.w.p, net.g.p, net.m.p, net.v.p, lr, b1, b2, eps, c1, c2);
  HC_LAUNCH_CHECK();
  net.refresh_bf16(c);
}

}  // namespace hc
