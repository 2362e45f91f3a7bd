// Mixed-precision SVD of the QR path on gfx950 (the SVD that restores the
// MPS form after every two-site gate; Chen & Stoudenmire, arXiv:1910.09142,
// Results section: singular values kept up to chi_max and the cutoff).
//
// With M = theta' (L x N, FP64 in TH) and M = Q R (FP64), the first stage
// runs the blocked Jacobi rounds in FP32 on a copy of R^T: its converged
// vectors are sigma_j w_j, w_j the right singular vectors of M, to FP32
// accuracy, at half the bytes per pass of FP64.  The second stage is a
// Rayleigh-Ritz step in FP64 on the span of the k' = rr_vectors largest of
// them:
//   k_rr_to32      R^T (FP64, Y) -> FP32 copy in X
//   (FP32 rounds)
//   k_rr_select    the k' columns of largest norm, largest first
//   k_rr_gather    W0 = those columns, normalised, in FP64 (Y)
//   k_rr_gram      G = W^T W (Z)
//   k_rr_correct   W <- W (I + E)^{-1/2} to first order along the Cholesky
//                  order (W_j (3 - G_jj) / 2 - sum_{i<j} W_i G_ij), twice:
//                  W orthonormal to FP64 rounding (the FP32 error is
//                  squared by each pass)
//   k_rr_project   B = M W (L x k', FP64 MFMA) into X
// after which FP64 rounds on the k' columns of B give B = U Sigma_B V_B^T:
// Sigma_B are Ritz values of M (their error is of second order in the FP32
// error of the basis), U the kept left singular vectors.  Truncation,
// log-weight and write-back stay FP64 and take the rest of ||theta'||^2
// (summed in FP64 from theta') as the unresolved tail.
//
// Two-QR variant (PATH_RR2): the FP32 rounds run on R2^T (R^T = Q2 R2, in
// fewer sweeps), whose converged vectors approximate sigma_j u~_j, u~_j =
// Q^T u_j the left singular vectors in the basis of Q.  With W the
// orthonormalised basis of the k' largest, B = R^T W (N x k') is M^T (Q W):
// the FP64 rounds on its columns converge to sigma_j w_j, the right Ritz
// vectors, and the write-back is that of the QR path.  Buffers: R in the
// upper triangle of X (kept), R2^T in Z, its FP32 copy in Y, the basis in
// Z and Y, its Gram in rrG, B in Y.
#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

struct RDims {
  int L, N, ld, ldN, kp, ldK, rr, two;
};

// kp: the chain's Ritz basis size, set by k_rr_select (read after it)
__device__ __forceinline__ RDims rdims(const Batch &b, int c,
                                      const UpdParams &u,
                                      const UpdScratch &s) {
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  RDims d;
  d.L = m > n ? m : n;
  d.N = m > n ? n : m;
  d.ld = vec_ld(d.L);
  d.ldN = vec_ld(d.N);
  const int path = svd_path(d.L, d.N, u.small_max, u.precond, u.mixed);
  d.rr = path_is_rr(path);
  d.two = path == PATH_RR2;
  d.kp = d.rr ? s.rrk[c] : 0;
  d.ldK = (d.kp + 15) & ~15;
  return d;
}

__global__ void __launch_bounds__(NT) k_rr_to32(Batch b, UpdScratch s,
                                                UpdParams u) {
  const int c = blockIdx.y;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  const size_t cnt = (size_t)n_blocks_even(d.N, JB) * JB * d.ldN;
  const double *Y = (d.two ? s.Z : s.Y) + (size_t)c * s.th_stride;
  float *X = reinterpret_cast<float *>(d.two ? s.Y : s.X) +
             (size_t)c * 2 * s.th_stride;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * NT)
    X[i] = (float)Y[i];
}

// Squared norms (FP64 sums) of the N FP32 vectors into sig2: wavefront w
// of workgroup x takes vectors 16 x + 4 w .. + 3.
__global__ void __launch_bounds__(NT) k_rr_norms(Batch b, UpdScratch s,
                                                 UpdParams u) {
  const int c = blockIdx.y;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  const float *X = reinterpret_cast<const float *>(d.two ? s.Y : s.X) +
                   (size_t)c * 2 * s.th_stride;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int t = 0; t < 4; ++t) {
    const int j = 16 * blockIdx.x + 4 * w + t;
    if (j >= d.N) return;
    double v = 0.0;
    for (int e = lane; e < d.ldN; e += 64) {
      const double x = X[(size_t)j * d.ldN + e];
      v = fma(x, x, v);
    }
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane == 0) s.sig2[(size_t)c * s.n_cap + j] = v;
  }
}

// One workgroup per chain: bitonic sort of the N squared norms (descending,
// ties by index), the first k' indices into perm.
__global__ void __launch_bounds__(NT) k_rr_select(Batch b, UpdScratch s,
                                                  UpdParams u) {
  const int c = blockIdx.x;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  __shared__ double key[2048];
  __shared__ int idx[2048];
  const int tid = threadIdx.x;
  int N2 = 1;
  while (N2 < d.N) N2 <<= 1;
  const double *sig2 = s.sig2 + (size_t)c * s.n_cap;
  for (int j = tid; j < N2; j += NT) {
    key[j] = j < d.N ? sig2[j] : -1.0;
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
  // basis: the largest rr_vectors vectors whose squared norm exceeds
  // skip32 times the largest (the FP32 rounds rotate those against all
  // others; smaller ones are left unrotated and are not a basis)
  const int kmax = rr_vectors(d.N, u.chi_max);
  __shared__ int cnt;
  if (tid == 0) {
    int k = 0;
    while (k < kmax && key[k] > 0.0 && key[k] > u.skip32 * key[0]) ++k;
    cnt = k < 1 ? 1 : k;
    s.rrk[c] = cnt;
  }
  __syncthreads();
  for (int j = tid; j < cnt; j += NT) s.perm[(size_t)c * s.n_cap + j] = idx[j];
}

// W0[:, j] = v_perm(j) / ||v_perm(j)|| (FP64, Y), padding rows included.
__global__ void __launch_bounds__(NT) k_rr_gather(Batch b, UpdScratch s,
                                                  UpdParams u) {
  const int c = blockIdx.y;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  const float *X = reinterpret_cast<const float *>(d.two ? s.Y : s.X) +
                   (size_t)c * 2 * s.th_stride;
  double *W = (d.two ? s.Z : s.Y) + (size_t)c * s.th_stride;
  const int32_t *perm = s.perm + (size_t)c * s.n_cap;
  const double *sig2 = s.sig2 + (size_t)c * s.n_cap;
  const size_t cnt = (size_t)d.kp * d.ldN;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * NT) {
    const int j = (int)(i / d.ldN), e = (int)(i % d.ldN);
    const int pj = perm[j];
    const double n2 = sig2[pj];
    W[i] = n2 > 0.0 ? (double)X[(size_t)pj * d.ldN + e] / sqrt(n2) : 0.0;
  }
}

// The basis of pass p: W0 in Y (p = 0) or W1 in X (p = 1); the corrected
// basis goes to the other buffer.  Two-QR variant: Z and Y (X keeps R).
__device__ __forceinline__ double *basis_src(const UpdScratch &s, int c, int p,
                                             bool two) {
  double *a = two ? s.Z : s.Y, *bb = two ? s.Y : s.X;
  return (p == 0 ? a : bb) + (size_t)c * s.th_stride;
}
__device__ __forceinline__ double *basis_dst(const UpdScratch &s, int c, int p,
                                             bool two) {
  double *a = two ? s.Z : s.Y, *bb = two ? s.Y : s.X;
  return (p == 0 ? bb : a) + (size_t)c * s.th_stride;
}
__device__ __forceinline__ double *basis_gram(const UpdScratch &s, int c,
                                              bool two) {
  return two ? s.rrG + (size_t)c * s.rrG_stride : s.Z + (size_t)c * s.th_stride;
}

// G = W^T W, one 16 x 16 tile per wavefront, rows of W as aligned 32-byte
// loads (rows N .. ldN-1 are zero); G row-major with stride ldK, zero
// beyond k'.
__global__ void __launch_bounds__(NT) k_rr_gram(Batch b, UpdScratch s,
                                                UpdParams u, int p) {
  const int c = blockIdx.z;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int j1 = blockIdx.x * 64 + 16 * w, j2 = blockIdx.y * 16;
  if (j1 >= d.ldK || j2 >= d.ldK) return;
  const double *W = basis_src(s, c, p, d.two);
  double *G = basis_gram(s, c, d.two);
  const bool aok = j1 + li < d.kp, bok = j2 + li < d.kp;
  const double *pa = W + (size_t)(aok ? j1 + li : 0) * d.ldN;
  const double *pb = W + (size_t)(bok ? j2 + li : 0) * d.ldN;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 0; r0 < d.ldN; r0 += 16) {
    const int rb = r0 + 4 * lk;
    const v4d x = *reinterpret_cast<const v4d *>(pa + rb);
    const v4d y = *reinterpret_cast<const v4d *>(pb + rb);
    acc = mfma_f64(aok ? x.x : 0.0, bok ? y.x : 0.0, acc);
    acc = mfma_f64(aok ? x.y : 0.0, bok ? y.y : 0.0, acc);
    acc = mfma_f64(aok ? x.z : 0.0, bok ? y.z : 0.0, acc);
    acc = mfma_f64(aok ? x.w : 0.0, bok ? y.w : 0.0, acc);
  }
  // D[i][j] (j1 + i, j2 + j) in lane j + 16 (i % 4), element i / 4
#pragma unroll
  for (int q = 0; q < 4; ++q)
    G[(size_t)(j1 + lk + 4 * q) * d.ldK + j2 + li] = acc[q];
}

// W'[r][j] = W[r][j] (3 - G_jj) / 2 - sum_{i<j} W[r][i] G[i][j]: tile of 16
// rows x 16 columns per wavefront; G row j0 + li, entries i0 + 4 lk .. + 3,
// as one aligned 32-byte load (G is symmetric).
__global__ void __launch_bounds__(NT) k_rr_correct(Batch b, UpdScratch s,
                                                   UpdParams u, int p) {
  const int c = blockIdx.z;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = blockIdx.x * 64 + 16 * w, j0 = blockIdx.y * 16;
  if (r0 >= d.ldN || j0 >= d.kp) return;
  const double *W = basis_src(s, c, p, d.two);
  double *Wn = basis_dst(s, c, p, d.two);
  const double *G = basis_gram(s, c, d.two);
  const bool jok = j0 + li < d.kp;
  const int jj = j0 + li;
  const double *grow = G + (size_t)(jok ? jj : 0) * d.ldK;
  const double *wrow = W + r0 + li;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < d.ldK; i0 += 16) {
    const int ib = i0 + 4 * lk;
    const v4d g = *reinterpret_cast<const v4d *>(grow + ib);
    double wv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ii = min(ib + q, d.kp - 1);
      const double x = wrow[(size_t)ii * d.ldN];
      wv[q] = ib + q < d.kp ? x : 0.0;
    }
    acc = mfma_f64(wv[0], jok && ib < jj ? g.x : 0.0, acc);
    acc = mfma_f64(wv[1], jok && ib + 1 < jj ? g.y : 0.0, acc);
    acc = mfma_f64(wv[2], jok && ib + 2 < jj ? g.z : 0.0, acc);
    acc = mfma_f64(wv[3], jok && ib + 3 < jj ? g.w : 0.0, acc);
  }
  if (!jok) return;
  const double gjj = G[(size_t)jj * d.ldK + jj];
  // D[i][j] (row r0 + i, column j0 + j) in lane j + 16 (i % 4), element i/4
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + lk + 4 * q;
    const double x = W[(size_t)jj * d.ldN + r];
    Wn[(size_t)jj * d.ldN + r] = x * (1.5 - 0.5 * gjj) - acc[q];
  }
}

// B = M W (L x k') into X: vector j of length L, stride ld, rows L .. ld-1
// and vectors k' .. npad(k')-1 zero.  Lane (li, lk) takes row l0 + li of M
// (single coalesced loads per contraction index) and elements q0 + 4 lk ..
// + 3 of W_j as one aligned 32-byte load.
// Two-QR variant: B = R^T W (N x k') into Y, vector stride ldN: row q of
// B is column q of R (the upper part of column q of X, rows i <= q) times
// W, both operands as aligned 32-byte loads of four consecutive i.
__global__ void __launch_bounds__(NT) k_rr_project(Batch b, UpdScratch s,
                                                   UpdParams u) {
  const int c = blockIdx.z;
  const RDims d = rdims(b, c, u, s);
  if (!d.rr) return;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int l0 = blockIdx.x * 64 + 16 * w, j0 = blockIdx.y * 16;
  const int npad = n_blocks_even(d.kp, JB) * JB;
  const int out_ld = d.two ? d.ldN : d.ld, out_len = d.two ? d.N : d.L;
  if (l0 >= out_ld || j0 >= npad) return;
  const bool jok = j0 + li < d.kp;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  double *out;
  if (d.two) {
    const double *R = s.X + (size_t)c * s.th_stride;
    const double *W = s.Z + (size_t)c * s.th_stride;  // W2 (after two passes)
    out = s.Y + (size_t)c * s.th_stride;
    const double *wv = W + (size_t)(jok ? j0 + li : 0) * d.ldN;
    const int q = l0 + li;
    const bool qok = q < d.N;
    const double *rcol = R + (size_t)(qok ? q : 0) * d.ld;
    const int iend = min(d.N, l0 + 16);  // R is upper triangular
    for (int i0 = 0; i0 < iend; i0 += 16) {
      const int ib = i0 + 4 * lk;
      const v4d wq = *reinterpret_cast<const v4d *>(wv + ib);
      const v4d rq = *reinterpret_cast<const v4d *>(rcol + ib);
      const int lim = min(d.N - 1, q);
      acc = mfma_f64(qok && ib <= lim ? rq.x : 0.0, jok ? wq.x : 0.0, acc);
      acc = mfma_f64(qok && ib + 1 <= lim ? rq.y : 0.0, jok ? wq.y : 0.0, acc);
      acc = mfma_f64(qok && ib + 2 <= lim ? rq.z : 0.0, jok ? wq.z : 0.0, acc);
      acc = mfma_f64(qok && ib + 3 <= lim ? rq.w : 0.0, jok ? wq.w : 0.0, acc);
    }
  } else {
    const double *M = s.TH + (size_t)c * s.th_stride;
    const double *W = s.Y + (size_t)c * s.th_stride;  // W2 (after two passes)
    out = s.X + (size_t)c * s.th_stride;
    const double *wv = W + (size_t)(jok ? j0 + li : 0) * d.ldN;
    const bool lok = l0 + li < d.L;
    const double *mrow = M + (lok ? l0 + li : 0);
    for (int q0 = 0; q0 < d.N; q0 += 16) {
      const int qb = q0 + 4 * lk;
      const v4d wq = *reinterpret_cast<const v4d *>(wv + qb);
      double mv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int qq = min(qb + q, d.N - 1);
        const double x = mrow[(size_t)qq * d.ld];
        mv[q] = (lok && qb + q < d.N) ? x : 0.0;
      }
      acc = mfma_f64(mv[0], jok ? wq.x : 0.0, acc);
      acc = mfma_f64(mv[1], jok ? wq.y : 0.0, acc);
      acc = mfma_f64(mv[2], jok ? wq.z : 0.0, acc);
      acc = mfma_f64(mv[3], jok ? wq.w : 0.0, acc);
    }
  }
  // D[i][j] (row l0 + i, vector j0 + j) in lane j + 16 (i % 4), element i/4
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int l = l0 + lk + 4 * q;
    out[(size_t)(j0 + li) * out_ld + l] = (jok && l < out_len) ? acc[q] : 0.0;
  }
}

}  // namespace

void launch_rr_stage2(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int max_N, int max_L, hipStream_t st) {
  const int kp = rr_vectors(max_N, u.chi_max);
  const int ldK = (kp + 15) & ~15, ldN = vector_stride(max_N);
  hipLaunchKernelGGL(k_rr_norms, dim3((max_N + 15) / 16, b.B), dim3(NT), 0, st,
                     b, s, u);
  hipLaunchKernelGGL(k_rr_select, dim3(b.B), dim3(NT), 0, st, b, s, u);
  hipLaunchKernelGGL(k_rr_gather, dim3(64, b.B), dim3(NT), 0, st, b, s, u);
  for (int p = 0; p < 2; ++p) {
    hipLaunchKernelGGL(k_rr_gram, dim3((ldK + 63) / 64, ldK / 16, b.B),
                       dim3(NT), 0, st, b, s, u, p);
    hipLaunchKernelGGL(k_rr_correct, dim3((ldN + 63) / 64, ldK / 16, b.B),
                       dim3(NT), 0, st, b, s, u, p);
  }
  const int npad = n_blocks_even(kp, JB) * JB;
  hipLaunchKernelGGL(k_rr_project,
                     dim3((vector_stride(max_L) + 63) / 64, npad / 16, b.B),
                     dim3(NT), 0, st, b, s, u);
}

void launch_rr_to32(const Batch &b, const UpdScratch &s, const UpdParams &u,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_rr_to32, dim3(64, b.B), dim3(NT), 0, st, b, s, u);
}

}  // namespace hmps
