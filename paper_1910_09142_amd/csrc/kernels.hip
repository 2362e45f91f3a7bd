// gfx950 kernels of the hybrid purification/sampling hot path
// (Chen & Stoudenmire, arXiv:1910.09142).
//
//   k_theta          theta'[(s1,a),(s2,c)] = sum G[(s1 s2),(t1 t2)]
//                    sum_b T_k[t1,a,b] T_{k+1}[t2,b,c]   (two-site gate on a
//                    bond; Ancilla Method subsection, Trotter gates)
//   k_jacobi_small   one-sided Jacobi SVD with the whole matrix in LDS
//   k_jacobi_round   one round of the blocked one-sided Jacobi SVD: Gram of
//                    a column-block pair, its eigenvectors by cyclic Jacobi
//                    in LDS, rotation of the block pair
//   k_truncate       sort the singular values, choose how many to keep
//                    (relative discarded weight, chi_max; Results section)
//   k_writeback_*    new site tensors from the kept singular triplets
//   k_measure_*      <S_i.S_j> by transfer matrices (step 3)
//   k_collapse       sequential projective measurement of the environment
//                    (step 4), Philox4x64-10 draws
//   k_init           environment product state x cluster Bell pairs (step 1)
#include "hmps_internal.h"

#include <math.h>

namespace hmps {

namespace {

constexpr int NT = 256;  // threads per workgroup of every kernel here

__device__ __forceinline__ double *site_ptr(const Batch &b, int c, int p) {
  return b.sites + ((size_t)c * b.nsites + p) * b.site_cap;
}
__device__ __forceinline__ const int32_t *chi_row(const Batch &b, int c) {
  return b.chi + (size_t)c * (b.nsites + 1);
}

// Round-robin (circle method) pairing of n (even) indices: round r in
// [0, n-1), pair i in [0, n/2).  Every unordered pair occurs exactly once
// per n-1 rounds and the pairs of one round are disjoint.
__device__ __forceinline__ void rr_pair(int r, int i, int n, int &p, int &q) {
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

// Plane rotation that makes two vectors with squared norms a, b and inner
// product g orthogonal: (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q).
// Returns false when they are already orthogonal to relative tolerance tol.
__device__ __forceinline__ bool jacobi_rotation(double a, double b, double g,
                                                double tol, double &c,
                                                double &s) {
  if (g == 0.0 || !(a > 0.0) || !(b > 0.0)) return false;
  if (fabs(g) <= tol * sqrt(a) * sqrt(b)) return false;
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

__device__ __forceinline__ int n_blocks_even(int n) {
  const int nb = (n + JB - 1) / JB;
  return nb + (nb & 1);
}

// Sum over the workgroup; every thread gets the result.
__device__ double wg_sum(double v, double *red) {
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
__device__ void wg_gemm(int M, int N, int K, double alpha, const double *A,
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
__device__ double wg_dot(int M, int N, const double *A, const double *B,
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
__device__ uint64_t philox_word0(uint64_t c0, uint64_t c1, uint64_t c2,
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

// Product-basis vectors: row t is the state of outcome t (eigenvalue
// +1, 0, -1) written in the S^z basis; basis 0 = S^z, 1 = S^x.
__constant__ double c_basis[2][3][3] = {
    {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}},
    {{0.5, 0.70710678118654752440, 0.5},
     {0.70710678118654752440, 0.0, -0.70710678118654752440},
     {0.5, -0.70710678118654752440, 0.5}}};

// =====================================================================
// theta' = G . (T_k T_{k+1})
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_theta(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.z;
  const int32_t *chi = chi_row(b, c);
  const int chiL = chi[u.k], chiM = chi[u.k + 1], chiR = chi[u.k + 2];
  const int a0 = blockIdx.x * 16, c0 = blockIdx.y * 16;
  if (a0 >= chiL) return;
  const int m = 3 * chiL, n = 3 * chiR;
  const int npad = n_blocks_even(n) * JB;
  const double *A = site_ptr(b, c, u.k);
  const double *Bt = site_ptr(b, c, u.k + 1);
  double *TH = s.TH + (size_t)c * s.th_stride;
  double *X = s.X + (size_t)c * s.th_stride;
  __shared__ double As[3][16][17];
  __shared__ double Bs[3][16][17];
  __shared__ double G[81];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  if (threadIdx.x < 81) G[threadIdx.x] = u.gate[threadIdx.x];
  __syncthreads();
  if (c0 < chiR) {
    double acc[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) acc[t] = 0.0;
    for (int b0 = 0; b0 < chiM; b0 += 16) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        As[t][ty][tx] = (a0 + ty < chiL && b0 + tx < chiM)
                            ? A[(size_t)t * chiL * chiM +
                                (size_t)(a0 + ty) * chiM + b0 + tx]
                            : 0.0;
        Bs[t][ty][tx] = (b0 + ty < chiM && c0 + tx < chiR)
                            ? Bt[(size_t)t * chiM * chiR +
                                 (size_t)(b0 + ty) * chiR + c0 + tx]
                            : 0.0;
      }
      __syncthreads();
#pragma unroll 4
      for (int bb = 0; bb < 16; ++bb) {
        const double a_0 = As[0][tx][bb], a_1 = As[1][tx][bb],
                     a_2 = As[2][tx][bb];
        const double b_0 = Bs[0][bb][ty], b_1 = Bs[1][bb][ty],
                     b_2 = Bs[2][bb][ty];
        acc[0] += a_0 * b_0;
        acc[1] += a_0 * b_1;
        acc[2] += a_0 * b_2;
        acc[3] += a_1 * b_0;
        acc[4] += a_1 * b_1;
        acc[5] += a_1 * b_2;
        acc[6] += a_2 * b_0;
        acc[7] += a_2 * b_1;
        acc[8] += a_2 * b_2;
      }
      __syncthreads();
    }
    const int a = a0 + tx, cc = c0 + ty;
    if (a < chiL && cc < chiR) {
#pragma unroll
      for (int s1 = 0; s1 < 3; ++s1) {
#pragma unroll
        for (int s2 = 0; s2 < 3; ++s2) {
          double v = 0.0;
#pragma unroll
          for (int t = 0; t < 9; ++t) v += G[(s1 * 3 + s2) * 9 + t] * acc[t];
          const size_t off =
              (size_t)(s2 * chiR + cc) * m + (size_t)(s1 * chiL + a);
          TH[off] = v;
          X[off] = v;
        }
      }
    }
  }
  if (blockIdx.y == 0 && a0 + tx < chiL) {
    for (int j = n + ty; j < npad; j += 16)
      for (int s1 = 0; s1 < 3; ++s1)
        X[(size_t)j * m + s1 * chiL + a0 + tx] = 0.0;
  }
}

// =====================================================================
// One-sided Jacobi SVD, whole matrix in LDS (one workgroup per chain).
// The columns of X (m x n, column-major) are rotated until every pair is
// orthogonal to relative tolerance tol; then X = U Sigma and the squared
// column norms are written to sig2.
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_jacobi_small(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.x;
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  double *X = s.X + (size_t)c * s.th_stride;
  __shared__ double xs[SMALL_LDS];
  __shared__ int flag;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < m * n; idx += NT) xs[idx] = X[idx];
  const int n_even = n + (n & 1);
  const int npairs = n_even / 2;
  int g = 64;
  while (g > 1 && g * npairs > NT) g >>= 1;
  const int lane = tid & (g - 1);
  const int per_pass = NT / g;
  bool converged = false;
  int sweep = 0;
  for (; sweep < u.max_sweeps; ++sweep) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int r = 0; r < n_even - 1; ++r) {
      for (int pi = tid / g; pi < npairs; pi += per_pass) {
        int p, q;
        rr_pair(r, pi, n_even, p, q);
        if (q < n) {
          double aa = 0.0, bb = 0.0, gg = 0.0;
          for (int i = lane; i < m; i += g) {
            const double x = xs[p * m + i], y = xs[q * m + i];
            aa += x * x;
            bb += y * y;
            gg += x * y;
          }
          for (int off = g >> 1; off > 0; off >>= 1) {
            aa += __shfl_xor(aa, off);
            bb += __shfl_xor(bb, off);
            gg += __shfl_xor(gg, off);
          }
          double cr, sr;
          if (jacobi_rotation(aa, bb, gg, u.tol, cr, sr)) {
            for (int i = lane; i < m; i += g) {
              const double x = xs[p * m + i], y = xs[q * m + i];
              xs[p * m + i] = cr * x - sr * y;
              xs[q * m + i] = sr * x + cr * y;
            }
            if (lane == 0) flag = 1;
          }
        }
      }
      __syncthreads();
    }
    const int f = flag;
    __syncthreads();
    if (f == 0) {
      converged = true;
      break;
    }
  }
  for (int idx = tid; idx < m * n; idx += NT) X[idx] = xs[idx];
  double *sig2 = s.sig2 + (size_t)c * s.n_cap;
  for (int j = tid; j < n; j += NT) {
    double v = 0.0;
    for (int i = 0; i < m; ++i) v += xs[j * m + i] * xs[j * m + i];
    sig2[j] = v;
  }
  if (tid == 0) {
    if (!converged) s.err[c] = 1;
    s.sweeps[c] += converged ? sweep + 1 : sweep;
  }
}

__global__ void k_jacobi_sweep_begin(UpdScratch s, int B, int sweep) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= B) return;
  if (sweep == 0)
    s.done[c] = 0;
  else if (s.rot_cur[c] == 0)
    s.done[c] = 1;
  s.rot_cur[c] = 0;
}

// =====================================================================
// One round of the blocked one-sided Jacobi SVD (one workgroup per
// column-block pair per chain).
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_jacobi_round(Batch b, UpdScratch s, UpdParams u, int r) {
  const int c = blockIdx.y, pi = blockIdx.x;
  if (s.done[c]) return;
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  const int NB = n_blocks_even(n);
  if (r >= NB - 1 || pi >= NB / 2) return;
  int bi, bj;
  rr_pair(r, pi, NB, bi, bj);
  double *X = s.X + (size_t)c * s.th_stride;
  __shared__ double xs[64][33];
  __shared__ double G[32][33];
  __shared__ double Q[32][33];
  __shared__ double cs[16], sn[16];
  __shared__ int flag;
  const int tid = threadIdx.x;
  const int gi = tid >> 3, gj0 = (tid & 7) * 4;
  auto colidx = [&](int t) { return t < JB ? bi * JB + t : bj * JB + t - JB; };

  // Gram matrix of the 32 columns, streamed through LDS in 64-row chunks.
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int e0 = 0; e0 < m; e0 += 64) {
#pragma unroll
    for (int h = 0; h < 8; ++h) {
      const int idx = tid + NT * h;
      const int col = idx >> 6, row = idx & 63;
      xs[row][col] = (e0 + row < m)
                         ? X[(size_t)colidx(col) * m + e0 + row]
                         : 0.0;
    }
    __syncthreads();
    for (int row = 0; row < 64; ++row) {
      const double xi = xs[row][gi];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) acc[jj] += xi * xs[row][gj0 + jj];
    }
    __syncthreads();
  }
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) G[gi][gj0 + jj] = acc[jj];
  if (tid == 0) flag = 0;
  __syncthreads();
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) {
    const int j = gj0 + jj;
    if (j == gi) continue;
    const double a = G[gi][gi], bb = G[j][j], g = G[gi][j];
    if (a > 0.0 && bb > 0.0 && fabs(g) > u.tol * sqrt(a) * sqrt(bb))
      flag = 1;
  }
  __syncthreads();
  if (!flag) {
    if (tid < 2 * JB) {
      const int col = colidx(tid);
      if (col < n) s.sig2[(size_t)c * s.n_cap + col] = G[tid][tid];
    }
    return;
  }
#pragma unroll
  for (int jj = 0; jj < 4; ++jj) Q[gi][gj0 + jj] = (gi == gj0 + jj) ? 1.0 : 0.0;
  __syncthreads();

  // Eigenvectors of G by cyclic Jacobi: G <- J^T G J, Q <- Q J.
  const double tol_in = fmax(0.125 * u.tol, 4e-16);
  for (int isw = 0; isw < 20; ++isw) {
    if (tid == 0) flag = 0;
    __syncthreads();
    for (int rr = 0; rr < 2 * JB - 1; ++rr) {
      if (tid < JB) {
        int p, q;
        rr_pair(rr, tid, 2 * JB, p, q);
        double cr = 1.0, sr = 0.0;
        if (jacobi_rotation(G[p][p], G[q][q], G[p][q], tol_in, cr, sr))
          flag = 1;
        cs[tid] = cr;
        sn[tid] = sr;
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int idx = tid + NT * h;
        const int pp = idx >> 5, col = idx & 31;
        int p, q;
        rr_pair(rr, pp, 2 * JB, p, q);
        const double cr = cs[pp], sr = sn[pp];
        const double x = G[p][col], y = G[q][col];
        G[p][col] = cr * x - sr * y;
        G[q][col] = sr * x + cr * y;
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int idx = tid + NT * h;
        const int pp = idx >> 5, row = idx & 31;
        int p, q;
        rr_pair(rr, pp, 2 * JB, p, q);
        const double cr = cs[pp], sr = sn[pp];
        double x = G[row][p], y = G[row][q];
        G[row][p] = cr * x - sr * y;
        G[row][q] = sr * x + cr * y;
        x = Q[row][p];
        y = Q[row][q];
        Q[row][p] = cr * x - sr * y;
        Q[row][q] = sr * x + cr * y;
      }
      __syncthreads();
    }
    const int f = flag;
    __syncthreads();
    if (!f) break;
  }

  // X[:, pair] <- X[:, pair] Q
  for (int e = tid; e < m; e += NT) {
    double xin[2 * JB];
#pragma unroll
    for (int t = 0; t < 2 * JB; ++t) xin[t] = X[(size_t)colidx(t) * m + e];
#pragma unroll 4
    for (int j = 0; j < 2 * JB; ++j) {
      double v = 0.0;
#pragma unroll
      for (int t = 0; t < 2 * JB; ++t) v += xin[t] * Q[t][j];
      X[(size_t)colidx(j) * m + e] = v;
    }
  }
  if (tid == 0) atomicAdd(&s.rot_cur[c], 1);
}

// =====================================================================
// Truncation: sort, choose k, bookkeeping.
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_truncate(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.x;
  int32_t *chi = b.chi + (size_t)c * (b.nsites + 1);
  const int n = 3 * chi[u.k + 2];
  __shared__ double key[2048];
  __shared__ int idx[2048];
  __shared__ int kk_s;
  const int tid = threadIdx.x;
  int N2 = 1;
  while (N2 < n) N2 <<= 1;
  const double *sig2 = s.sig2 + (size_t)c * s.n_cap;
  for (int j = tid; j < N2; j += NT) {
    key[j] = (j < n) ? sqrt(fmax(sig2[j], 0.0)) : -1.0;
    idx[j] = j;
  }
  __syncthreads();
  for (int size = 2; size <= N2; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = tid; t < N2 / 2; t += NT) {
        const int i = 2 * stride * (t / stride) + (t % stride);
        const int j = i + stride;
        const bool desc = (i & size) == 0;
        const double ki = key[i], kj = key[j];
        const int ii = idx[i], ij = idx[j];
        const bool j_first = (kj > ki) || (kj == ki && ij < ii);
        const bool i_first = (ki > kj) || (ki == kj && ii < ij);
        if (desc ? j_first : i_first) {
          key[i] = kj;
          key[j] = ki;
          idx[i] = ij;
          idx[j] = ii;
        }
      }
      __syncthreads();
    }
  }
  if (tid == 0) {
    // tail[k] = sum_{j >= k} sigma_j^2, accumulated from the smallest
    double total = 0.0;
    for (int j = n - 1; j >= 0; --j) total += key[j] * key[j];
    int kfloor = 0;
    while (kfloor < n && key[kfloor] > SIGMA_FLOOR * key[0]) ++kfloor;
    const double thr = u.cutoff * total;
    int k_eps = n;
    double tail = 0.0;
    // smallest k >= 1 with tail[k] <= thr: scan k from n down while the
    // tail stays below the threshold
    for (int k = n; k >= 1; --k) {
      if (k < n) tail += key[k] * key[k];
      if (tail <= thr)
        k_eps = k;
      else
        break;
    }
    const int m = 3 * chi[u.k];
    int k = k_eps < u.chi_max ? k_eps : u.chi_max;
    if (k > kfloor) k = kfloor;
    if (k > m) k = m;
    if (k < 1) k = 1;
    if (k < n && key[k - 1] - key[k] <= TIE_TOL * key[k - 1]) {
      int i = k - 1;
      while (i > 0 && key[i - 1] - key[i] <= TIE_TOL * key[i - 1]) --i;
      if (i > 0) k = i;
    }
    double kept = 0.0;
    for (int j = k - 1; j >= 0; --j) kept += key[j] * key[j];
    if (!(total > 0.0) || !isfinite(total) || !(kept > 0.0)) s.err[c] = 2;
    s.fac[c] = 1.0 / sqrt(kept);
    if (u.is_gate) s.logw[c] += log(total);
    s.discarded[c] += (total - kept) / total;
    s.knew[c] = k;
    chi[u.k + 1] = k;
    kk_s = k;
  }
  __syncthreads();
  const int k = kk_s;
  for (int j = tid; j < k; j += NT) {
    s.perm[(size_t)c * s.n_cap + j] = idx[j];
    s.sig[(size_t)c * s.n_cap + j] = key[j];
  }
}

// =====================================================================
// Write-back of the kept triplets.  X = U Sigma (columns perm[j]).
// right: T_k = U, T_{k+1} = fac Sigma V^T = (fac / sigma_j) X_j^T theta'
// left : T_k = fac U Sigma = fac X_j, T_{k+1} = V^T = sigma_j^-2 X_j^T theta'
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_writeback_direct(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.y;
  const int32_t *chi = chi_row(b, c);
  const int chiL = chi[u.k], k = s.knew[c];
  const int m = 3 * chiL;
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= m * k) return;
  const int i = t % m, j = t / m;
  const int col = s.perm[(size_t)c * s.n_cap + j];
  const double f = u.right ? 1.0 / s.sig[(size_t)c * s.n_cap + j] : s.fac[c];
  const double v = s.X[(size_t)c * s.th_stride + (size_t)col * m + i] * f;
  const int s1 = i / chiL, a = i - s1 * chiL;
  site_ptr(b, c, u.k)[(size_t)s1 * chiL * k + (size_t)a * k + j] = v;
}

__global__ void __launch_bounds__(NT)
    k_writeback_gemm(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.z;
  const int32_t *chi = chi_row(b, c);
  const int chiL = chi[u.k], chiR = chi[u.k + 2], k = s.knew[c];
  const int m = 3 * chiL, n = 3 * chiR;
  const int col0 = blockIdx.x * 16, j0 = blockIdx.y * 16;
  if (col0 >= n || j0 >= k) return;
  const double *X = s.X + (size_t)c * s.th_stride;
  const double *TH = s.TH + (size_t)c * s.th_stride;
  const int32_t *perm = s.perm + (size_t)c * s.n_cap;
  __shared__ double As[16][17];
  __shared__ double Bs[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int pj = (j0 + ty < k) ? perm[j0 + ty] : -1;
  double acc = 0.0;
  for (int i0 = 0; i0 < m; i0 += 16) {
    As[ty][tx] = (pj >= 0 && i0 + tx < m) ? X[(size_t)pj * m + i0 + tx] : 0.0;
    Bs[tx][ty] = (col0 + ty < n && i0 + tx < m)
                     ? TH[(size_t)(col0 + ty) * m + i0 + tx]
                     : 0.0;
    __syncthreads();
#pragma unroll
    for (int ii = 0; ii < 16; ++ii) acc += As[ty][ii] * Bs[ii][tx];
    __syncthreads();
  }
  const int j = j0 + ty, col = col0 + tx;
  if (j < k && col < n) {
    const double sg = s.sig[(size_t)c * s.n_cap + j];
    const double f = u.right ? s.fac[c] / sg : 1.0 / (sg * sg);
    const int s2 = col / chiR, cc = col - s2 * chiR;
    site_ptr(b, c, u.k + 1)[(size_t)s2 * k * chiR + (size_t)j * chiR + cc] =
        f * acc;
  }
}

// =====================================================================
// Measurement.  The centre is site 0 and sites 1.. are right-orthonormal,
// so the right environment of every site is the identity.  L_p is the
// left environment of <psi|psi> (sites < p).
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_measure_envs(Batch b, MeasureArgs ma) {
  const int c = blockIdx.x;
  const int32_t *chi = chi_row(b, c);
  double *env = ma.envs + (size_t)c * (b.nsites + 1) * ma.chi2;
  double *Y = ma.bond_scratch + (size_t)c * ma.slots * 4 * ma.chi2;
  __shared__ double red[NT / 64];
  if (threadIdx.x == 0) env[0] = 1.0;
  __syncthreads();
  for (int p = 0; p < b.nsites; ++p) {
    const int chiL = chi[p], chiR = chi[p + 1];
    const double *T = site_ptr(b, c, p);
    double *Lp = env + (size_t)p * ma.chi2;
    double *Lq = env + (size_t)(p + 1) * ma.chi2;
    double sz = 0.0;
    for (int t = 0; t < 3; ++t) {
      const double *Ts = T + (size_t)t * chiL * chiR;
      wg_gemm(chiL, chiR, chiL, 1.0, Lp, chiL, 0, Ts, chiR, 0, 0.0, Y, chiR);
      const double w = wg_dot(chiL, chiR, Ts, Y, chiR, red);
      sz += (1 - t) * w;
      wg_gemm(chiR, chiR, chiL, 1.0, Ts, chiR, 1, Y, chiR, 0, t ? 1.0 : 0.0,
              Lq, chiR);
    }
    if (threadIdx.x == 0)
      ma.wsz[(size_t)c * b.nsites + p] = ma.is_ancilla[p] ? -sz : sz;
  }
  if (threadIdx.x == 0) ma.norm[c] = env[(size_t)b.nsites * ma.chi2];
}

__global__ void __launch_bounds__(NT)
    k_measure_bonds(Batch b, MeasureArgs ma, int b0) {
  const int c = blockIdx.y, slot = blockIdx.x, bond = b0 + blockIdx.x;
  if (bond >= ma.n_bonds) return;
  const int32_t *chi = chi_row(b, c);
  const int p = ma.bond_p[bond], q = ma.bond_q[bond];
  const double *env = ma.envs + (size_t)c * (b.nsites + 1) * ma.chi2;
  double *scr = ma.bond_scratch + ((size_t)c * ma.slots + slot) * 4 * ma.chi2;
  double *E = scr, *E2 = scr + ma.chi2, *Y = scr + 2 * ma.chi2;
  __shared__ double red[NT / 64];
  const double r2 = 1.4142135623730950488;
  double total = 0.0;
  for (int str = 0; str < 2; ++str) {
    // at p: E = sum_{s,t} O[s,t] T_p[s]^T L_p T_p[t]  (O = S^z or S^+)
    {
      const int chiL = chi[p], chiR = chi[p + 1];
      const double *T = site_ptr(b, c, p);
      const double *Lp = env + (size_t)p * ma.chi2;
      bool first = true;
      for (int sb = 0; sb < 3; ++sb) {
        int tk;
        double coef;
        if (str == 0) {
          tk = sb;
          coef = 1.0 - sb;
        } else {
          tk = sb + 1;
          coef = r2;
          if (sb == 2) coef = 0.0;
        }
        if (coef == 0.0) continue;
        wg_gemm(chiL, chiR, chiL, 1.0, Lp, chiL, 0,
                T + (size_t)tk * chiL * chiR, chiR, 0, 0.0, Y, chiR);
        wg_gemm(chiR, chiR, chiL, coef, T + (size_t)sb * chiL * chiR, chiR, 1,
                Y, chiR, 0, first ? 0.0 : 1.0, E, chiR);
        first = false;
      }
    }
    for (int mid = p + 1; mid < q; ++mid) {
      const int chiL = chi[mid], chiR = chi[mid + 1];
      const double *T = site_ptr(b, c, mid);
      for (int sb = 0; sb < 3; ++sb) {
        const double *Ts = T + (size_t)sb * chiL * chiR;
        wg_gemm(chiL, chiR, chiL, 1.0, E, chiL, 0, Ts, chiR, 0, 0.0, Y, chiR);
        wg_gemm(chiR, chiR, chiL, 1.0, Ts, chiR, 1, Y, chiR, 0,
                sb ? 1.0 : 0.0, E2, chiR);
      }
      double *t = E;
      E = E2;
      E2 = t;
    }
    // at q: sum_{s,t} O'[s,t] <T_q[s], E T_q[t]>  (O' = S^z or S^-)
    {
      const int chiL = chi[q], chiR = chi[q + 1];
      const double *T = site_ptr(b, c, q);
      for (int sb = 0; sb < 3; ++sb) {
        int tk;
        double coef;
        if (str == 0) {
          tk = sb;
          coef = 1.0 - sb;
        } else {
          tk = sb - 1;
          coef = (sb == 0) ? 0.0 : r2;
        }
        if (coef == 0.0) continue;
        wg_gemm(chiL, chiR, chiL, 1.0, E, chiL, 0,
                T + (size_t)tk * chiL * chiR, chiR, 0, 0.0, Y, chiR);
        total += coef *
                 wg_dot(chiL, chiR, T + (size_t)sb * chiL * chiR, Y, chiR, red);
      }
    }
  }
  if (threadIdx.x == 0) ma.bond_ss[(size_t)c * ma.n_bonds + bond] = total;
}

__global__ void k_measure_finish(Batch b, MeasureArgs ma, double *energy,
                                 double *qn) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.B) return;
  const double nrm = ma.norm[c];
  double e = 0.0;
  for (int i = 0; i < ma.n_bonds; ++i) {
    const double v = ma.bond_ss[(size_t)c * ma.n_bonds + i] / nrm;
    ma.bond_ss[(size_t)c * ma.n_bonds + i] = v;
    e += ma.bond_J[i] * v;
  }
  energy[c] = e;
  double z = 0.0;
  for (int p = 0; p < b.nsites; ++p) z += ma.wsz[(size_t)c * b.nsites + p];
  qn[c] = z / nrm;
}

// =====================================================================
// Collapse: E is the left density matrix of the measured/traced past.
// =====================================================================
__global__ void __launch_bounds__(NT) k_collapse(Batch b, CollapseArgs a) {
  const int c = blockIdx.x;
  const int32_t *chi = chi_row(b, c);
  double *scr = a.scratch + (size_t)c * 8 * a.chi2;
  double *E = scr, *E2 = scr + a.chi2, *Z = scr + 2 * a.chi2;
  double *Yt = scr + 3 * a.chi2;  // 3 buffers
  __shared__ double red[NT / 64];
  __shared__ int pick;
  if (threadIdx.x == 0) {
    E[0] = 1.0;
    a.near[c] = 0;
  }
  __syncthreads();
  for (int k = 0; k < b.nsites; ++k) {
    const int chiL = chi[k], chiR = chi[k + 1];
    const double *T = site_ptr(b, c, k);
    if (a.is_cluster[k]) {
      for (int sb = 0; sb < 3; ++sb) {
        const double *Ts = T + (size_t)sb * chiL * chiR;
        wg_gemm(chiL, chiR, chiL, 1.0, E, chiL, 0, Ts, chiR, 0, 0.0, Z, chiR);
        wg_gemm(chiR, chiR, chiL, 1.0, Ts, chiR, 1, Z, chiR, 0,
                sb ? 1.0 : 0.0, E2, chiR);
      }
    } else {
      const int sz = chiL * chiR;
      for (int idx = threadIdx.x; idx < sz; idx += NT) {
        const double v0 = T[idx], v1 = T[sz + idx], v2 = T[2 * sz + idx];
        for (int t = 0; t < 3; ++t)
          Yt[(size_t)t * a.chi2 + idx] = c_basis[a.basis][t][0] * v0 +
                                         c_basis[a.basis][t][1] * v1 +
                                         c_basis[a.basis][t][2] * v2;
      }
      __syncthreads();
      double pr[3];
      for (int t = 0; t < 3; ++t) {
        wg_gemm(chiL, chiR, chiL, 1.0, E, chiL, 0, Yt + (size_t)t * a.chi2,
                chiR, 0, 0.0, Z, chiR);
        pr[t] = fmax(wg_dot(chiL, chiR, Yt + (size_t)t * a.chi2, Z, chiR, red),
                     0.0);
      }
      if (threadIdx.x == 0) {
        const double P = pr[0] + pr[1] + pr[2];
        const double cum0 = pr[0] / P, cum1 = (pr[0] + pr[1]) / P;
        const uint64_t x = philox_word0((uint64_t)c, (uint64_t)a.sample,
                                        (uint64_t)k, 1ull, a.seed, 0ull);
        const double uu = (double)(x >> 11) * (1.0 / 9007199254740992.0);
        int sel = 2;
        if (uu < cum0)
          sel = 0;
        else if (uu < cum1)
          sel = 1;
        double dmin = fmin(fabs(uu - cum0), fabs(uu - cum1));
        dmin = fmin(dmin, fabs(uu - 1.0));
        if (dmin < 1e-12) a.near[c] += 1;
        pick = sel;
        a.outcomes[(size_t)c * a.n_env + a.env_index[k]] = (uint8_t)sel;
      }
      __syncthreads();
      const int sel = pick;
      const double *Ys = Yt + (size_t)sel * a.chi2;
      wg_gemm(chiL, chiR, chiL, 1.0, E, chiL, 0, Ys, chiR, 0, 0.0, Z, chiR);
      wg_gemm(chiR, chiR, chiL, 1.0 / pr[sel], Ys, chiR, 1, Z, chiR, 0, 0.0,
              E2, chiR);
    }
    double *t = E;
    E = E2;
    E2 = t;
  }
}

// =====================================================================
// Initial states.
// =====================================================================
__global__ void k_init(Batch b, InitArgs a, double *logw) {
  const int p = blockIdx.x, c = blockIdx.y;
  int32_t *chi = b.chi + (size_t)c * (b.nsites + 1);
  double *T = site_ptr(b, c, p);
  const int t = threadIdx.x;
  if (a.is_cluster[p] && !a.is_ancilla[p]) {
    if (t < 9) T[t] = ((t / 3) == (t % 3)) ? 0.57735026918962576451 : 0.0;
    if (t == 0) chi[p + 1] = 3;
  } else if (a.is_ancilla[p]) {
    if (t < 9) T[t] = ((t / 3) == (t % 3)) ? 1.0 : 0.0;
    if (t == 0) chi[p + 1] = 1;
  } else {
    const int lab = a.labels[(size_t)c * a.n_env + a.env_index[p]];
    if (t < 3) T[t] = c_basis[a.basis][lab][t];
    if (t == 0) chi[p + 1] = 1;
  }
  if (p == 0 && t == 0) {
    chi[0] = 1;
    logw[c] = 0.0;
  }
}

}  // namespace

// ---- launchers ---------------------------------------------------------
void launch_theta(const Batch &b, const UpdScratch &s, const UpdParams &u,
                  int max_chiL, int max_chiR, hipStream_t st) {
  dim3 grid((max_chiL + 15) / 16, (max_chiR + 15) / 16, b.B);
  hipLaunchKernelGGL(k_theta, grid, dim3(NT), 0, st, b, s, u);
}

void launch_jacobi_small(const Batch &b, const UpdScratch &s,
                         const UpdParams &u, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_small, dim3(b.B), dim3(NT), 0, st, b, s, u);
}

void launch_jacobi_sweep_begin(const UpdScratch &s, int B, int sweep,
                               hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_sweep_begin, dim3((B + 255) / 256), dim3(256),
                     0, st, s, B, sweep);
}

void launch_jacobi_round(const Batch &b, const UpdScratch &s,
                         const UpdParams &u, int round, int max_pairs,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_round, dim3(max_pairs, b.B), dim3(NT), 0, st, b,
                     s, u, round);
}

void launch_truncate(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_truncate, dim3(b.B), dim3(NT), 0, st, b, s, u);
}

void launch_writeback(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int max_m, int max_n, int max_k, hipStream_t st) {
  const int nd = (max_m * max_k + NT - 1) / NT;
  hipLaunchKernelGGL(k_writeback_direct, dim3(nd, b.B), dim3(NT), 0, st, b, s,
                     u);
  dim3 g2((max_n + 15) / 16, (max_k + 15) / 16, b.B);
  hipLaunchKernelGGL(k_writeback_gemm, g2, dim3(NT), 0, st, b, s, u);
}

void launch_measure_envs(const Batch &b, const MeasureArgs &m,
                         hipStream_t st) {
  hipLaunchKernelGGL(k_measure_envs, dim3(b.B), dim3(NT), 0, st, b, m);
}

void launch_measure_bonds(const Batch &b, const MeasureArgs &m, int b0,
                          int nb, hipStream_t st) {
  hipLaunchKernelGGL(k_measure_bonds, dim3(nb, b.B), dim3(NT), 0, st, b, m,
                     b0);
}

void launch_measure_finish(const Batch &b, const MeasureArgs &m,
                           double *energy, double *qn, hipStream_t st) {
  hipLaunchKernelGGL(k_measure_finish, dim3((b.B + 255) / 256), dim3(256), 0,
                     st, b, m, energy, qn);
}

void launch_collapse(const Batch &b, const CollapseArgs &a, hipStream_t st) {
  hipLaunchKernelGGL(k_collapse, dim3(b.B), dim3(NT), 0, st, b, a);
}

void launch_init(const Batch &b, const InitArgs &a, double *logw,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_init, dim3(b.nsites, b.B), dim3(64), 0, st, b, a,
                     logw);
}

}  // namespace hmps
