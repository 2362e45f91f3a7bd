// Householder QR preconditioning of the blocked one-sided Jacobi SVD on
// gfx950 (the SVD that restores the MPS form after every two-site gate;
// Chen & Stoudenmire, arXiv:1910.09142, Results section).
//
// The vector matrix M (L x N, column-major, stride ld; theta' or its
// transpose) is factored M = Q R by blocked Householder reflections, and
// the Jacobi rounds then run on the N columns of R^T (Drmac and Veselic,
// "New fast and accurate Jacobi SVD algorithm", SIAM J. Matrix Anal. Appl.
// 29 (2008)): R^T has the singular values of M, and its columns are much
// closer to orthogonal than those of M, so far fewer sweeps are needed.
// R^T = W Sigma U^T gives M = (Q U) Sigma W^T: the converged vectors are the
// right singular vectors W of M scaled by Sigma, and the left ones follow
// as M W / Sigma, so Q itself is never formed.
//
//   k_qr_panel      Householder reflectors of one 16-column panel, the
//                   panel held in LDS; the compact-WY factor T with
//                   H_1 ... H_16 = I - V T V^T, T^{-1} = striu(V^T V) +
//                   diag(1 / tau) (Joffrain et al., ACM TOMS 32 (2006))
//   k_qr_update     trailing columns C <- C - V T^T (V^T C) on the FP64
//                   matrix cores, one 16-column tile per workgroup
//   k_qr_to_vectors R^T into the vector buffer Y, zero padding included
#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

constexpr int PT = 256;  // threads of the QR kernels (4 wavefronts)

struct QDims {
  int L, N, ld, qr;
};

__device__ __forceinline__ QDims qdims(const Batch &b, int c, const UpdParams &u) {
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  QDims d;
  d.L = m > n ? m : n;
  d.N = m > n ? n : m;
  d.ld = vec_ld(d.L);
  d.qr = qr_path(d.L, d.N, u.small_max, u.precond);
  return d;
}

// Sum of 16 per-lane values over a wavefront: afterwards lane l holds the
// sum of value l >> 2 (every value is held by four lanes).  Each exchange
// step halves the values a lane carries (17 exchanges instead of 96).
__device__ __forceinline__ double wave_sum16(double (&v)[16]) {
  const int lane = threadIdx.x & 63;
  double u8[8], u4[4], u2[2];
  const bool b5 = lane & 32, b4 = lane & 16, b3 = lane & 8;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const double send = b5 ? v[k] : v[k + 8];
    u8[k] = (b5 ? v[k + 8] : v[k]) + __shfl_xor(send, 32);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const double send = b4 ? u8[k] : u8[k + 4];
    u4[k] = (b4 ? u8[k + 4] : u8[k]) + __shfl_xor(send, 16);
  }
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    const double send = b3 ? u4[k] : u4[k + 2];
    u2[k] = (b3 ? u4[k + 2] : u4[k]) + __shfl_xor(send, 8);
  }
  const bool b2 = lane & 4;
  double x = (b2 ? u2[1] : u2[0]) + __shfl_xor(b2 ? u2[0] : u2[1], 4);
  x += __shfl_xor(x, 2);
  x += __shfl_xor(x, 1);
  return x;
}

// Sum of one value over the workgroup, every thread gets the result; the
// four wave sums are added in a fixed order.
__device__ __forceinline__ double block_sum1(double v, double *red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  const int w = threadIdx.x >> 6;
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[w] = v;
  __syncthreads();
  return (red[0] + red[1]) + (red[2] + red[3]);
}

// Sums of 16 values over the workgroup into out[16] (LDS, every thread may
// read it after the call).
__device__ __forceinline__ void block_sum16(double (&v)[16], double *red,
                                            double *out) {
  const double x = wave_sum16(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if ((lane & 3) == 0) red[w * 16 + (lane >> 2)] = x;
  __syncthreads();
  if (threadIdx.x < 16) {
    const int t = threadIdx.x;
    out[t] = (red[t] + red[16 + t]) + (red[32 + t] + red[48 + t]);
  }
  __syncthreads();
}

// =====================================================================
// Panel p: columns j0 .. j0 + w - 1 (j0 = 16 p) of M, rows j0 .. L - 1.
// Column t of the panel (global column j = j0 + t): with x its rows j..L-1,
// alpha = x_0, beta = -sign(alpha) ||x||, v = x / (alpha - beta) with v_0 =
// 1, tau = (beta - alpha) / beta, so that (I - tau v v^T) x = beta e_0.
// R_jj = beta; v_1.. are stored below the diagonal.  The same reduction
// that applies the reflector to the later panel columns (v^T a_t', t' > t)
// yields V^T v for the earlier ones, which builds T column by column:
// T[0:t, t] = -tau_t T[0:t, 0:t] (V[:, 0:t]^T v_t), T[t][t] = tau_t.
// =====================================================================
__global__ void __launch_bounds__(PT) k_qr_panel(Batch b, UpdScratch s,
                                                 UpdParams u, int p) {
  const int c = blockIdx.x;
  const QDims d = qdims(b, c, u);
  const int j0 = QB * p;
  if (!d.qr || j0 >= d.N) return;
  const int w = min(QB, d.N - j0);
  const int rows = d.L - j0;  // panel rows j0 .. L-1
  double *X = s.X + (size_t)c * s.th_stride;
  __shared__ double P[QB * QR_MAX_L];  // column t at P + t * rows
  __shared__ double red[64];
  __shared__ double dots[QB];
  __shared__ double T[QB][QB];
  const int tid = threadIdx.x;
  for (int t = 0; t < QB; ++t)
    for (int r = tid; r < rows; r += PT)
      P[t * rows + r] = t < w ? X[(size_t)(j0 + t) * d.ld + j0 + r] : 0.0;
  if (tid < QB * QB) T[tid / QB][tid % QB] = 0.0;
  __syncthreads();
  for (int t = 0; t < w; ++t) {
    // ||x||^2 over panel rows t .. rows-1 of column t, and alpha
    double *col = P + t * rows;
    double part = 0.0;
    for (int r = t + tid; r < rows; r += PT) part += col[r] * col[r];
    const double s2 = block_sum1(part, red);
    const double alpha = col[t];
    double tau = 0.0, scale = 0.0, beta = alpha;
    if (s2 > 0.0) {
      beta = -copysign(sqrt(s2), alpha);
      tau = (beta - alpha) / beta;
      scale = 1.0 / (alpha - beta);
    }
    __syncthreads();  // every thread has read col[t] as alpha
    for (int r = t + 1 + tid; r < rows; r += PT) col[r] *= scale;
    if (tid == 0) col[t] = beta;
    __syncthreads();
    // dots[t'] = v_t^T (panel column t') over rows t.. : for t' > t the
    // current column (to be reflected), for t' < t the reflector v_t'
    // (zero above its row t', one at it)
    double acc[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) acc[q] = 0.0;
    for (int r = t + tid; r < rows; r += PT) {
      const double vr = r == t ? 1.0 : col[r];
#pragma unroll
      for (int q = 0; q < QB; ++q) {
        double a;
        if (q < t)
          a = r > q ? P[q * rows + r] : (r == q ? 1.0 : 0.0);
        else if (q > t && q < w)
          a = P[q * rows + r];
        else
          a = 0.0;
        acc[q] += vr * a;
      }
    }
    block_sum16(acc, red, dots);
    // reflect the later columns: a_t' -= tau v (v^T a_t')
    for (int r = t + tid; r < rows; r += PT) {
      const double vr = r == t ? 1.0 : col[r];
      for (int q = t + 1; q < w; ++q) P[q * rows + r] -= tau * vr * dots[q];
    }
    // T column t from the dots with the earlier reflectors, row i by
    // thread i (each reads its own row of T, columns < t)
    if (tid < t) {
      double x = 0.0;
      for (int q = tid; q < t; ++q) x += T[tid][q] * dots[q];
      T[tid][t] = -tau * x;
    }
    if (tid == 0) T[t][t] = tau;
    __syncthreads();
  }
  for (int t = 0; t < w; ++t)
    for (int r = tid; r < rows; r += PT)
      X[(size_t)(j0 + t) * d.ld + j0 + r] = P[t * rows + r];
  if (tid < QB * QB) s.qrT[(size_t)c * QB * QB + tid] = T[tid / QB][tid % QB];
}

// =====================================================================
// Trailing update of panel p: tile x holds columns c0 = j0 + 16 + 16 x ..
// c0 + 15 of M.  W = V^T C (16 x 16, FP64 MFMA over 16-row chunks, four
// wavefront partials summed in a fixed order), W' = T^T W, C -= V W' (FP64
// MFMA, computed transposed so that lanes store consecutive rows).  Only
// rows j0 .. L-1 change; rows L .. ld-1 of M are zero and V is zero there.
// =====================================================================
__global__ void __launch_bounds__(PT) k_qr_update(Batch b, UpdScratch s,
                                                  UpdParams u, int p) {
  const int c = blockIdx.y;
  const QDims d = qdims(b, c, u);
  const int j0 = QB * p;
  const int c0 = j0 + QB + QB * blockIdx.x;
  if (!d.qr || c0 >= d.N) return;
  const int wcol = min(QB, d.N - j0);  // reflectors of this panel
  double *X = s.X + (size_t)c * s.th_stride;
  const int ld = d.ld;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double Wp[4][QB][QB + 1];
  __shared__ double W2[QB][QB + 1];
  __shared__ double Ts[QB][QB + 1];
  Ts[tid / QB][tid % QB] = s.qrT[(size_t)c * QB * QB + tid];
  // reflector t at row r: 0 above its diagonal row j0 + t, 1 on it
  const bool vcol_ok = li < wcol;
  const double *vcol = X + (size_t)(j0 + (vcol_ok ? li : 0)) * ld;
  const bool ccol_ok = c0 + li < d.N;
  const double *ccol = X + (size_t)(ccol_ok ? c0 + li : c0) * ld;
  auto vval = [&](int r, double x) -> double {
    const int dr = j0 + li;
    return !vcol_ok ? 0.0 : (r < dr ? 0.0 : (r == dr ? 1.0 : x));
  };
  // ---- W = V^T C over rows j0 .. ld-1 (row order is free in the sum) ----
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int e0 = j0 + 16 * wv; e0 < ld; e0 += 64) {
    const int r0 = e0 + 4 * lk;
    const v4d xv = *reinterpret_cast<const v4d *>(vcol + r0);
    const v4d xc = *reinterpret_cast<const v4d *>(ccol + r0);
    acc = mfma_f64(vval(r0, xv.x), ccol_ok ? xc.x : 0.0, acc);
    acc = mfma_f64(vval(r0 + 1, xv.y), ccol_ok ? xc.y : 0.0, acc);
    acc = mfma_f64(vval(r0 + 2, xv.z), ccol_ok ? xc.z : 0.0, acc);
    acc = mfma_f64(vval(r0 + 3, xv.w), ccol_ok ? xc.w : 0.0, acc);
  }
  // D[i][j] (i: reflector, j: tile column) in lane j + 16 (i % 4), elem i/4
#pragma unroll
  for (int q = 0; q < 4; ++q) Wp[wv][lk + 4 * q][li] = acc[q];
  __syncthreads();
  {
    const int i = tid / QB, j = tid % QB;
    Wp[0][i][j] = (Wp[0][i][j] + Wp[1][i][j]) + (Wp[2][i][j] + Wp[3][i][j]);
  }
  __syncthreads();
  {
    // W' = T^T W (T upper triangular)
    const int i = tid / QB, j = tid % QB;
    double x = 0.0;
    for (int t = 0; t <= i; ++t) x += Ts[t][i] * Wp[0][t][j];
    W2[i][j] = x;
  }
  __syncthreads();
  // ---- C -= V W', as D^T = W'^T V^T per 16-row chunk ----------------------
  // A operand lane (li, lk): W'^T[li][4 s + lk] = W'[4 s + lk][li];
  // B operand lane (li, lk): V^T[4 s + lk][row li] = V[e0 + li][4 s + lk];
  // D'[j][i] (tile column j, row e0 + i) in lane i + 16 (j % 4), elem j / 4
  double wa[4];
#pragma unroll
  for (int sidx = 0; sidx < 4; ++sidx) wa[sidx] = W2[4 * sidx + lk][li];
  for (int e0 = j0 + 16 * wv; e0 < ld; e0 += 64) {
    const int r = e0 + li;
    v4d dd = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int sidx = 0; sidx < 4; ++sidx) {
      const int t = 4 * sidx + lk;
      const double x = X[(size_t)(j0 + (t < wcol ? t : 0)) * ld + r];
      const double v = t >= wcol ? 0.0 : (r < j0 + t ? 0.0 : (r == j0 + t ? 1.0 : x));
      dd = mfma_f64(wa[sidx], v, dd);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int col = c0 + lk + 4 * q;
      if (col < d.N && r < d.L) X[(size_t)col * ld + r] -= dd[q];
    }
  }
}

// =====================================================================
// R^T into Y: vector i (row i of R) at Y + i * ldN, R[i][j] = M[j * ld + i]
// for j >= i and 0 below; rows N .. ldN-1 and vectors N .. npad-1 zero.
// One 16 x 16 tile per thread block, through LDS.
// =====================================================================
__global__ void __launch_bounds__(PT) k_qr_to_vectors(Batch b, UpdScratch s,
                                                      UpdParams u) {
  const int c = blockIdx.z;
  const QDims d = qdims(b, c, u);
  if (!d.qr) return;
  const int ldN = vec_ld(d.N);
  const int npad = n_blocks_even(d.N, JB) * JB;
  const int i0 = 16 * blockIdx.x, jj0 = 16 * blockIdx.y;  // vector, element
  if (i0 >= npad || jj0 >= ldN) return;
  const double *X = s.X + (size_t)c * s.th_stride;
  double *Y = s.Y + (size_t)c * s.th_stride;
  __shared__ double tile[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  {
    // read R[i0 + tx][jj0 + ty] = M[(jj0 + ty) * ld + i0 + tx]
    const int i = i0 + tx, j = jj0 + ty;
    tile[ty][tx] = (i < d.N && j < d.N && j >= i) ? X[(size_t)j * d.ld + i] : 0.0;
  }
  __syncthreads();
  // Y[(i0 + ty) * ldN + jj0 + tx] = R[i0 + ty][jj0 + tx]
  Y[(size_t)(i0 + ty) * ldN + jj0 + tx] = tile[tx][ty];
}

}  // namespace

void launch_qr_panel(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     int p, hipStream_t st) {
  hipLaunchKernelGGL(k_qr_panel, dim3(b.B), dim3(PT), 0, st, b, s, u, p);
}

void launch_qr_update(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int p, int max_tiles, hipStream_t st) {
  if (max_tiles <= 0) return;
  hipLaunchKernelGGL(k_qr_update, dim3(max_tiles, b.B), dim3(PT), 0, st, b, s,
                     u, p);
}

void launch_qr_to_vectors(const Batch &b, const UpdScratch &s,
                          const UpdParams &u, int max_N, hipStream_t st) {
  const int npad = n_blocks_even(max_N, JB) * JB;
  dim3 grid(npad / 16, vector_stride(max_N) / 16, b.B);
  hipLaunchKernelGGL(k_qr_to_vectors, grid, dim3(PT), 0, st, b, s, u);
}

}  // namespace hmps
