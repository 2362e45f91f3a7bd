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
// A second factorization R^T = Q2 R2 (PATH_QR2) brings the columns of
// R2^T closer still to orthogonal; the same kernels run on R^T in Y
// (stage 1) after the first QR of the vector matrix in X (stage 0).
//
//   k_qr_panel      Householder reflectors of one 16-column panel, the
//                   panel rows held in registers (1 to 3 per thread), the
//                   columns in a loop over four groups of four; the
//                   compact-WY factor T with H_1 ... H_16 = I - V T V^T
//                   from the kept products once the panel is done (as in
//                   LAPACK's dlarft)
//   k_qr_update     trailing columns C <- C - V T^T (V^T C) on the FP64
//                   matrix cores, one 16-column tile per workgroup
//   k_qr_to_vectors R^T into the vector buffer (Y, or Z after stage 1),
//                   zero padding included
#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

constexpr int PT = 256;   // threads of the update and transpose kernels
constexpr int QPT = 512;  // threads of the panel kernel (8 wavefronts)
// panel rows per thread of the panel kernel, at most (a launch takes the
// fewest that hold its longest panel)
constexpr int RPT = (QR_MAX_L + QPT - 1) / QPT;

// The matrix a stage factors (column-major, stride ld, L x N) and where
// its transposed triangular factor goes.
struct QDims {
  int L, N, ld, qr;
  double *M;    // the matrix, factored in place
  double *out;  // R^T as N vectors of length N (stride vec_ld(N))
};

__device__ __forceinline__ QDims qdims(const Batch &b, int c,
                                       const UpdParams &u,
                                       const UpdScratch &s, int stage) {
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  const int Lt = m > n ? m : n;
  const int path = svd_path(Lt, m > n ? n : m, u.small_max, u.precond,
                            u.mixed);
  QDims d;
  d.N = m > n ? n : m;
  const size_t off = (size_t)c * s.th_stride;
  if (stage == 0) {
    d.L = Lt;
    d.qr = path_has_qr(path);
    d.M = s.X + off;
    d.out = s.Y + off;
  } else {
    d.L = d.N;
    d.qr = path_has_qr2(path);
    d.M = s.Y + off;
    d.out = s.Z + off;
  }
  d.ld = vec_ld(d.L);
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

// =====================================================================
// Panel p: columns j0 .. j0 + w - 1 (j0 = 16 p) of M, rows j0 .. L - 1.
// Column t of the panel (global column j = j0 + t): with x its rows j..L-1,
// alpha = x_0, beta = -sign(alpha) ||x||, v = (x - beta e_0) / (alpha -
// beta) (so v_0 = 1), tau = (beta - alpha) / beta, and (I - tau v v^T) x =
// beta e_0.  R_jj = beta; v_1.. are stored below the diagonal.
// Thread i holds panel rows i, i + 512, .. (R of them, the fewest that
// hold the launch's longest panel) of all 16 columns in registers.  One reduction per column gives every product the column
// needs: d_q = x^T y_q over rows t.. with y_q the later panel columns
// (q > t), the earlier reflectors (q < t) and x itself (q = t, ||x||^2).
// Since v = (x - beta e_0) / (alpha - beta), v^T y_q = (d_q - beta y_q[t])
// / (alpha - beta); sign(-beta) = sign(alpha), so nothing cancels.  These
// reflect the later columns, a_q -= tau v (v^T a_q), and, kept for the
// earlier reflectors, give T once the panel is done: T[0:t, t] = -tau
// T[0:t, 0:t] (V[:, 0:t]^T v_t), T[t][t] = tau.  The eight wavefront
// partials are summed in a fixed order.
// =====================================================================
template <int R>
__global__ void __launch_bounds__(QPT) k_qr_panel(Batch b, UpdScratch s,
                                                  UpdParams u, int stage,
                                                  int p, int cb) {
  const int c = cb + blockIdx.x;
  const QDims d = qdims(b, c, u, s, stage);
  const int j0 = QB * p;
  if (!d.qr || j0 >= d.N) return;
  const int w = min(QB, d.N - j0);
  const int rows = d.L - j0;  // panel rows j0 .. L-1
  double *M = d.M;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  __shared__ double red[(QPT / 64) * QB];
  __shared__ double dots[QB];
  __shared__ double yt[QB];        // row t of the panel (the y_q[t])
  __shared__ double VV[QB][QB + 1];  // VV[t][q] = v_t^T y_q, panel order
  __shared__ double taus[QB];
  // The columns are taken in four groups of four.  The registers hold the
  // groups in a rotating order: in quarter k, register group g holds panel
  // columns 4 ((k + g) mod 4) .. + 3, so the current group is always
  // group 0 and every register index is a constant, while the loop over
  // the quarters stays a loop (a fully unrolled panel is too long for the
  // instruction cache).  After the fourth rotation the order is the
  // panel's again.
  double a[R][QB];
  // loads with clamped addresses and a select (no branch around a load)
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = tid + QPT * i;
    const int rr = r < rows ? r : rows - 1;
#pragma unroll
    for (int q = 0; q < QB; ++q) {
      const int qq = q < w ? q : w - 1;
      const double x = M[(size_t)(j0 + qq) * d.ld + j0 + rr];
      a[i][q] = (r < rows && q < w) ? x : 0.0;
    }
  }
  static_assert(QB == 16, "four groups of four columns");
#pragma unroll 1
  for (int k = 0; k < 4; ++k) {
#pragma unroll
    for (int tl = 0; tl < 4; ++tl) {
      const int t = 4 * k + tl;  // panel column, in register slot tl
      if (t < w) {               // uniform: every thread takes it
        if (tid == t) {
#pragma unroll
          for (int q = 0; q < QB; ++q) yt[q] = a[0][q];
        }
        double acc[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q) acc[q] = 0.0;
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int r = tid + QPT * i;
          const double x = r >= t ? a[i][tl] : 0.0;
#pragma unroll
          for (int q = 0; q < QB; ++q) acc[q] = fma(x, a[i][q], acc[q]);
        }
        const double part = wave_sum16(acc);  // value lane >> 2
        if ((lane & 3) == 0) red[wv * QB + (lane >> 2)] = part;
        __syncthreads();
        if (tid < QB) {
          const double *rq = red + tid;
          dots[tid] = ((rq[0] + rq[QB]) + (rq[2 * QB] + rq[3 * QB])) +
                      ((rq[4 * QB] + rq[5 * QB]) + (rq[6 * QB] + rq[7 * QB]));
        }
        __syncthreads();
        const double s2 = dots[tl];
        const double alpha = yt[tl];
        double tau = 0.0, scale = 0.0, beta = alpha;
        if (s2 > 0.0) {
          beta = -copysign(sqrt(s2), alpha);
          tau = (beta - alpha) / beta;
          scale = 1.0 / (alpha - beta);
        }
        // v^T y_q; with x = 0 the reflector is the identity and v = e_0
        double vy[QB];
#pragma unroll
        for (int q = 0; q < QB; ++q)
          vy[q] = s2 > 0.0 ? scale * (dots[q] - beta * yt[q]) : yt[q];
        // the later columns: the rest of this group, and the groups that
        // hold columns after this quarter's (v_r = 0 above row t leaves
        // those rows unchanged)
#pragma unroll
        for (int i = 0; i < R; ++i) {
          const int r = tid + QPT * i;
          const double vr = r == t ? 1.0 : (r > t ? a[i][tl] * scale : 0.0);
          const double f = -tau * vr;
#pragma unroll
          for (int q = tl + 1; q < 4; ++q) a[i][q] = fma(f, vy[q], a[i][q]);
#pragma unroll
          for (int g = 1; g < 4; ++g) {
            if (k + g < 4) {
#pragma unroll
              for (int q = 4 * g; q < 4 * g + 4; ++q)
                a[i][q] = fma(f, vy[q], a[i][q]);
            }
          }
          a[i][tl] = r == t ? beta : (r > t ? vr : a[i][tl]);
        }
        if (tid == 0) {
          taus[t] = tau;
#pragma unroll
          for (int q = 0; q < QB; ++q)
            VV[t][4 * ((k + (q >> 2)) & 3) + (q & 3)] = vy[q];
        }
        __syncthreads();
      }
    }
    // rotate the register groups: group g <- group g + 1
#pragma unroll
    for (int i = 0; i < R; ++i) {
      double h[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) h[q] = a[i][q];
#pragma unroll
      for (int q = 0; q < QB - 4; ++q) a[i][q] = a[i][q + 4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[i][QB - 4 + q] = h[q];
    }
  }
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int r = tid + QPT * i;
    if (r < rows) {
#pragma unroll
      for (int q = 0; q < QB; ++q)
        if (q < w) M[(size_t)(j0 + q) * d.ld + j0 + r] = a[i][q];
    }
  }
  // T (H_1 ... H_w = I - V T V^T), row i by thread i: T[i][i] = tau_i and
  // T[i][t] = -tau_t sum_q T[i][q] (v_q^T v_t) for t > i; the sum runs
  // over every earlier q, the entries left of the diagonal being zero
  if (tid < QB) {
    double Tr[QB];
#pragma unroll
    for (int q = 0; q < QB; ++q) Tr[q] = 0.0;
#pragma unroll
    for (int t = 0; t < QB; ++t) {
      if (t < w) {
        if (t == tid) {
          Tr[t] = taus[t];
        } else if (t > tid) {
          double x = 0.0;
#pragma unroll
          for (int q = 0; q < t; ++q) x += Tr[q] * VV[t][q];
          Tr[t] = -taus[t] * x;
        }
      }
    }
    double *Tout = qrT_slot(s, c, stage, p) + tid * QB;
#pragma unroll
    for (int q = 0; q < QB; ++q) Tout[q] = Tr[q];
  }
}

// =====================================================================
// Trailing update of panel p: tile x holds columns c0 = j0 + 16 + 16 x ..
// c0 + 15 of M.  W = V^T C (16 x 16, FP64 MFMA over 16-row chunks, four
// wavefront partials summed in a fixed order), W' = T^T W, C -= V W' (FP64
// MFMA, computed transposed so that lanes store consecutive rows): C <-
// H_{16}^T .. H_1^T C.  Only rows j0 .. L-1 change; rows L .. ld-1 of M
// are zero and V is zero there.
// APPLY: the same block reflector, untransposed (W' = T W, C <- H_1 ..
// H_16 C), on the k unit vectors in TH of a PATH_QR2 chain (length L,
// stride ld, zero below row N): panels from last to first give Q u~.
// =====================================================================
template <bool APPLY>
__global__ void __launch_bounds__(PT) k_qr_update(Batch b, UpdScratch s,
                                                  UpdParams u, int stage,
                                                  int p, int cb) {
  const int c = cb + blockIdx.y;
  const QDims d = qdims(b, c, u, s, stage);
  const int j0 = QB * p;
  int ncols = d.N, c0 = j0 + QB + QB * blockIdx.x;
  double *C = d.M;
  if (APPLY) {
    const int path = svd_path(d.L, d.N, u.small_max, u.precond, u.mixed);
    if (path != PATH_QR2) return;
    ncols = s.knew[c];
    c0 = QB * blockIdx.x;
    C = s.TH + (size_t)c * s.th_stride;
  } else if (!d.qr) {
    return;
  }
  if (j0 >= d.N || c0 >= ncols) return;
  const int wcol = min(QB, d.N - j0);  // reflectors of this panel
  const double *X = d.M;
  const int ld = d.ld;
  const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  __shared__ double Wp[4][QB][QB + 1];
  __shared__ double W2[QB][QB + 1];
  __shared__ double Ts[QB][QB + 1];
  Ts[tid / QB][tid % QB] = qrT_slot(s, c, stage, p)[tid];
  // reflector t at row r: 0 above its diagonal row j0 + t, 1 on it
  const bool vcol_ok = li < wcol;
  const double *vcol = X + (size_t)(j0 + (vcol_ok ? li : 0)) * ld;
  const bool ccol_ok = c0 + li < ncols;
  const double *ccol = C + (size_t)(ccol_ok ? c0 + li : c0) * ld;
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
    // W' = T^T W or T W (T upper triangular)
    const int i = tid / QB, j = tid % QB;
    double x = 0.0;
    if (APPLY) {
      for (int t = i; t < QB; ++t) x += Ts[i][t] * Wp[0][t][j];
    } else {
      for (int t = 0; t <= i; ++t) x += Ts[t][i] * Wp[0][t][j];
    }
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
      if (col < ncols && r < d.L) C[(size_t)col * ld + r] -= dd[q];
    }
  }
}

// =====================================================================
// R^T into the stage's vector buffer: vector i (row i of R) at out + i *
// ldN, R[i][j] = M[j * ld + i] for j >= i and 0 below; rows N .. ldN-1 and
// vectors N .. npad-1 zero.  One 16 x 16 tile per thread block, through
// LDS.
// =====================================================================
__global__ void __launch_bounds__(PT) k_qr_to_vectors(Batch b, UpdScratch s,
                                                      UpdParams u, int stage,
                                                      int cb) {
  const int c = cb + blockIdx.z;
  const QDims d = qdims(b, c, u, s, stage);
  if (!d.qr) return;
  const int ldN = vec_ld(d.N);
  const int npad = npad_vectors(d.N);
  const int i0 = 16 * blockIdx.x, jj0 = 16 * blockIdx.y;  // vector, element
  if (i0 >= npad || jj0 >= ldN) return;
  const double *X = d.M;
  double *Y = d.out;
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
                     int stage, int p, int max_rows, int cb, int nc,
                     hipStream_t st) {
  // every chain's panel rows fit R rows per thread
  static_assert(RPT == 3, "panel variants for 1 .. 3 rows per thread");
  if (max_rows <= QPT)
    hipLaunchKernelGGL(k_qr_panel<1>, dim3(nc), dim3(QPT), 0, st, b, s, u,
                       stage, p, cb);
  else if (max_rows <= 2 * QPT)
    hipLaunchKernelGGL(k_qr_panel<2>, dim3(nc), dim3(QPT), 0, st, b, s, u,
                       stage, p, cb);
  else
    hipLaunchKernelGGL(k_qr_panel<3>, dim3(nc), dim3(QPT), 0, st, b, s, u,
                       stage, p, cb);
}

void launch_qr_update(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int stage, int p, int max_tiles, int cb, int nc,
                      hipStream_t st) {
  if (max_tiles <= 0) return;
  hipLaunchKernelGGL(k_qr_update<false>, dim3(max_tiles, nc), dim3(PT), 0, st,
                     b, s, u, stage, p, cb);
}

void launch_qr_apply(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     int p, int max_tiles, hipStream_t st) {
  if (max_tiles <= 0) return;
  hipLaunchKernelGGL(k_qr_update<true>, dim3(max_tiles, b.B), dim3(PT), 0, st,
                     b, s, u, 0, p, 0);
}

void launch_qr_to_vectors(const Batch &b, const UpdScratch &s,
                          const UpdParams &u, int stage, int max_N, int cb,
                          int nc, hipStream_t st) {
  const int npad = npad_vectors(max_N);
  dim3 grid(npad / 16, vector_stride(max_N) / 16, nc);
  hipLaunchKernelGGL(k_qr_to_vectors, grid, dim3(PT), 0, st, b, s, u, stage,
                     cb);
}

}  // namespace hmps
