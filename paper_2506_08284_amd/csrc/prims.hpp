// Sparse and vector primitives used by the setup and the solve.
#pragma once
#include "common.hpp"

namespace hc {

// out[0..n] = exclusive prefix sum of in[0..n-1], out[n] = total; returns the
// total (host synchronises).  Fails with HCURL_EUNSUPPORTED if it exceeds 2^31-1.
int64_t exclusive_scan(const int* in, int* out, int64_t n, Ctx& c);

// C = A B on the symbolic pattern of |A||B| (structural zeros kept, columns
// sorted).  numeric: also the values (A and B must carry values).
void spgemm(const Csr& A, const Csr& B, Csr& C, bool numeric, Ctx& c, const char* tag = nullptr);
// C = A B again on the pattern C holds: C.rowptr (and C.nnz) must come from
// spgemm of matrices with the patterns of A and B; columns and values are
// rewritten (the same columns).
void spgemm_refill(const Csr& A, const Csr& B, Csr& C, Ctx& c, const char* tag = nullptr);

// C = D B for a discrete gradient D (rows of one or two entries +-1): the
// same pattern and values as spgemm(D, B), by merging rows of B; any other D
// goes to spgemm.
void gradient_product(const Csr& D, const Csr& B, Csr& C, Ctx& c, const char* tag = nullptr);

// AT = A^T with sorted columns; values copied when A has them and `values`.
void transpose(const Csr& A, Csr& AT, bool values, Ctx& c);
// AT's values again from A with the pattern AT already holds (A's pattern
// unchanged since the transpose, columns sorted within A's rows).
void transpose_refill(const Csr& A, Csr& AT, Ctx& c);

// Builds a device CSR from host or device arrays with int64 row pointers.
void upload_csr(const hcurl_csr& in, bool device_ptrs, Csr& out, bool values, Ctx& c);

// Pattern-and-values copy (deep).
void copy_csr(const Csr& A, Csr& B, Ctx& c);

// y = A x   (mode 0), y = b - A x   (mode 1), y += A x (mode 2)
void spmv(const Csr& A, const double* x, double* y, const double* b, int mode, Ctx& c, const char* tag = "spmv");
// Mixed-precision forms (sums in FP64): A's FP64 values (spmv_v64) or its FP32
// copy val32 (spmv_v32); instantiated for the vector types the FP32 V-cycle
// uses.  The FP32 V-cycle forms residuals with spmv_v64: A x of a large
// gradient field cancels (S D = 0), and the FP32 copy of A would leave
// rounding noise far above the result.
template <class X, class Y>
void spmv_v64(const Csr& A, const X* x, Y* y, const Y* b, int mode, Ctx& c, const char* tag);
template <class X, class Y>
void spmv_v32(const Csr& A, const X* x, Y* y, const Y* b, int mode, Ctx& c, const char* tag);

// Deterministic reductions into device scalars: scal[slot] = sum x*y.
void dot(const double* x, const double* y, int64_t n, double* out, Ctx& c, int red_slot = 0);
// sum_i x_i * y_i with x float, y float accumulated in double
void dot32(const float* x, const float* y, int64_t n, double* out, Ctx& c, int red_slot = 0);

// Diagonal of A (inverse if inv) into d.
void diagonal(const Csr& A, double* d, bool inv, Ctx& c);

void fill(double* x, double v, int64_t n, Ctx& c);
void fill32(float* x, float v, int64_t n, Ctx& c);
void fill_int(int* x, int v, int64_t n, Ctx& c);
void cast_d2f(const double* x, float* y, int64_t n, Ctx& c);
void cast_f2d(const float* x, double* y, int64_t n, Ctx& c);

// Finalise partial sums written by a kernel that used the reduction scratch:
// out = sum over blocks of red[slot * kRedBlocks + b], b < nblocks.
void reduce_partials(int nblocks, int slot, double* out, Ctx& c);

// splitmix64 finaliser of (i + golden gamma) as a device function
__device__ __forceinline__ uint64_t splitmix64(uint64_t i) {
  uint64_t z = i + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Wave-level helpers (64 lanes).
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    int t = __shfl_up(v, o, 64);
    if (l >= o) v += t;
  }
  return v;
}

// Block-wide (256 threads) deterministic sum; result valid in thread 0.
__device__ __forceinline__ double block_sum256(double v, double* sh /* 4 doubles */) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0) r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

}  // namespace hc
