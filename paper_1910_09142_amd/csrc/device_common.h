// Device helpers shared by the gfx950 kernels (update.hip, observe.hip).
#pragma once
#include "hmps_internal.h"

#include <math.h>

namespace hmps {
namespace dev {

constexpr int NT = 256;  // threads per workgroup of every kernel here

static __device__ __forceinline__ double *site_ptr(const Batch &b, int c, int p) {
  return b.sites + ((size_t)c * b.nsites + p) * b.site_cap;
}
static __device__ __forceinline__ const int32_t *chi_row(const Batch &b, int c) {
  return b.chi + (size_t)c * (b.nsites + 1);
}

// Round-robin (circle method) pairing of n (even) indices: round r in
// [0, n-1), pair i in [0, n/2).  Every unordered pair occurs exactly once
// per n-1 rounds and the pairs of one round are disjoint.
static __device__ __forceinline__ void rr_pair(int r, int i, int n, int &p, int &q) {
  const int mod = n - 1;
  if (i == 0) {
    p = r;
    q = n - 1;
  } else {
    p = (r + i) % mod;
    q = (r - i + mod) % mod;
  }
  if (p > q) {
    int t = p;
    p = q;
    q = t;
  }
}

// FP64 matrix-core product D(16x16) += A(16x4) B(4x16) of one wavefront.
// Operand layout on gfx950 (checked on the device): lane i + 16k holds
// A[i][k]; lane j + 16k holds B[k][j]; lane j + 16 (i % 4) holds D[i][j]
// in element i / 4.
typedef double v4d __attribute__((ext_vector_type(4)));
static __device__ __forceinline__ v4d mfma_f64(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Whether two vectors with squared norms a, b and inner product g still need
// a rotation.  A vector whose squared norm is at most `skip` times its
// partner's (skip <= SIGMA_FLOOR^2), or below 1e-30 absolutely (theta' has
// norm of order one: the state is normalised before every update), lies
// below the singular-value floor and is always discarded; rotating it
// would change its partner's squared norm by less than skip relative, so
// it is left alone.
static __device__ __forceinline__ bool pair_needs_rotation(double a, double b,
                                                           double g,
                                                           double tol,
                                                           double skip) {
  if (g == 0.0 || !(a > 0.0) || !(b > 0.0)) return false;
  const double lo = fmin(a, b), hi = fmax(a, b);
  if (lo <= 1e-30 || lo <= skip * hi) return false;
  // |g| > tol sqrt(a b) without square roots: a, b are squared norms of
  // columns of theta' (norm of order one) and at least 1e-30 here, so a b
  // neither overflows nor underflows
  return g * g > (tol * tol) * (a * b);
}

// Plane rotation that makes two vectors with squared norms a, b and inner
// product g orthogonal: (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q).
// Returns false when they are already orthogonal to relative tolerance tol.
static __device__ __forceinline__ bool jacobi_rotation(double a, double b, double g,
                                                double tol, double skip,
                                                double &c, double &s) {
  if (!pair_needs_rotation(a, b, g, tol, skip)) return false;
  const double zeta = (b - a) / (2.0 * g);
  double t;
  if (fabs(zeta) > 1e150)
    t = 0.5 / zeta;
  else
    t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
  c = 1.0 / sqrt(1.0 + t * t);
  s = c * t;
  return true;
}

// Stride between consecutive vectors of the vector matrix (see
// vector_stride): four consecutive rows are one aligned 32-byte load.
static __device__ __forceinline__ int vec_ld(int L) { return vector_stride(L); }


// Sum over the workgroup; every thread gets the result.
static __device__ double wg_sum(double v, double *red) {
  const int tid = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((tid & 63) == 0) red[tid >> 6] = v;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NT / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

// C = alpha op(A) op(B) + beta C, computed by one workgroup.  Row-major
// storage; op(A) is M x K: ta = 0 reads A[m*lda + k], ta = 1 reads
// A[k*lda + m].  op(B) is K x N: tb = 0 reads B[k*ldb + n], tb = 1 reads
// B[n*ldb + k].  beta == 0 never reads C.
static __device__ void wg_gemm(int M, int N, int K, double alpha, const double *A,
                        int lda, int ta, const double *B, int ldb, int tb,
                        double beta, double *C, int ldc) {
  __shared__ double As[16][65];
  __shared__ double Bs[16][65];
  const int tid = threadIdx.x;
  const int tr = tid >> 4, tc = tid & 15;
  for (int m0 = 0; m0 < M; m0 += 64) {
    for (int n0 = 0; n0 < N; n0 += 64) {
      double acc[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
      for (int k0 = 0; k0 < K; k0 += 16) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int idx = tid + NT * h;
          int mm, kk;
          double v = 0.0;
          if (!ta) {
            mm = idx >> 4;
            kk = idx & 15;
            if (m0 + mm < M && k0 + kk < K)
              v = A[(size_t)(m0 + mm) * lda + k0 + kk];
          } else {
            kk = idx >> 6;
            mm = idx & 63;
            if (m0 + mm < M && k0 + kk < K)
              v = A[(size_t)(k0 + kk) * lda + m0 + mm];
          }
          As[kk][mm] = v;
          int nn;
          v = 0.0;
          if (!tb) {
            kk = idx >> 6;
            nn = idx & 63;
            if (n0 + nn < N && k0 + kk < K)
              v = B[(size_t)(k0 + kk) * ldb + n0 + nn];
          } else {
            nn = idx >> 4;
            kk = idx & 15;
            if (n0 + nn < N && k0 + kk < K)
              v = B[(size_t)(n0 + nn) * ldb + k0 + kk];
          }
          Bs[kk][nn] = v;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 16; ++kk) {
          double a[4], bv[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) a[i] = As[kk][tr + 16 * i];
#pragma unroll
          for (int j = 0; j < 4; ++j) bv[j] = Bs[kk][tc + 16 * j];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j) acc[i][j] += a[i] * bv[j];
        }
        __syncthreads();
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int row = m0 + tr + 16 * i;
        if (row >= M) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int col = n0 + tc + 16 * j;
          if (col >= N) continue;
          double v = alpha * acc[i][j];
          if (beta != 0.0) v += beta * C[(size_t)row * ldc + col];
          C[(size_t)row * ldc + col] = v;
        }
      }
    }
  }
  __syncthreads();
}

// <A, B> (Frobenius) of two row-major M x N arrays with the same ld.
static __device__ double wg_dot(int M, int N, const double *A, const double *B,
                         int ld, double *red) {
  double v = 0.0;
  for (int idx = threadIdx.x; idx < M * N; idx += NT) {
    const int i = idx / N, j = idx - i * N;
    v += A[(size_t)i * ld + j] * B[(size_t)i * ld + j];
  }
  return wg_sum(v, red);
}

// ---------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11): first output word.
// ---------------------------------------------------------------------
static __device__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
                                 uint64_t c3, uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += W0;
      k1 += W1;
    }
    const uint64_t hi0 = __umul64hi(M0, c0), lo0 = M0 * c0;
    const uint64_t hi1 = __umul64hi(M1, c2), lo1 = M1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

}  // namespace dev
}  // namespace hmps
