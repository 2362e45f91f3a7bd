// gfx950 kernels of one two-site Trotter update on every chain of a batch
// (Chen & Stoudenmire, arXiv:1910.09142: gate on a bond, then a truncated
// SVD restores the MPS form -- Ancilla Method subsection and Results
// section, sources of error).
//
//   k_theta         theta' = G (T_k T_{k+1}), written as a matrix whose
//                   columns are the vectors the Jacobi SVD orthogonalises
//   k_pad           zero padding vectors of the blocked Jacobi path
//   k_jacobi_small  one-sided Jacobi SVD with the whole matrix in LDS
//   (the rounds of the blocked one-sided Jacobi SVD are in jacobi.hip)
//   k_truncate      sort singular values, choose how many to keep
//   k_writeback_*   new site tensors from the kept singular triplets
//
// Vector layout.  theta' is m x n with m = 3 chi_L (rows (s1,a)) and
// n = 3 chi_R (columns (s2,c)).  The Jacobi SVD orthogonalises the N =
// min(m, n) vectors of length L = max(m, n): the columns of theta' when
// n <= m, its rows when n > m ("transposed").  More vectors than their
// length could never all become orthogonal.  X and TH hold the L x N
// vector matrix column-major (vector j at offset j*L).  Vectors are
// ordered bond index first, 3 c + s2 (or 3 a + s1): the bond's basis
// comes from the previous truncations sorted by Schmidt value, so this
// order grades the vectors by norm, which is what the unpivoted QR of the
// preconditioned path needs.  Elements along a vector keep s-major order.
#include "device_common.h"
#include "small_path.h"
#include "truncate_rule.h"

namespace hmps {
namespace {
using namespace dev;

struct Dims {
  int chiL, chiM, chiR, m, n, L, N, trans;
  int ld;  // vector stride in X and TH: L rounded up to a multiple of 16
  // the side of theta' whose index is the vector index (rows when trans,
  // columns otherwise) is interleaved, 3 (bond index) + s
  int il_rows, il_cols;
};

// A chain on a QR path rotates R^T (or R2^T; N vectors of length N): its
// converged vectors lie on the other side of theta' than those of the
// plain path (see qr.hip), so the write-back swaps sides.
__device__ __forceinline__ int path_of(const Dims &d, const UpdParams &u) {
  return svd_path(d.L, d.N, u.small_max, u.precond, u.mixed);
}
__device__ __forceinline__ Dims vector_side(const Dims &d, bool qr) {
  Dims e = d;
  if (qr) e.trans = !d.trans;
  return e;
}

__device__ __forceinline__ Dims dims_of(const Batch &b, int c, int k) {
  const int32_t *chi = chi_row(b, c);
  Dims d;
  d.chiL = chi[k];
  d.chiM = chi[k + 1];
  d.chiR = chi[k + 2];
  d.m = 3 * d.chiL;
  d.n = 3 * d.chiR;
  d.trans = d.n > d.m;
  d.L = d.trans ? d.n : d.m;
  d.N = d.trans ? d.m : d.n;
  d.ld = vec_ld(d.L);
  d.il_rows = d.trans;
  d.il_cols = !d.trans;
  return d;
}

// =====================================================================
// theta'[(s1,a),(s2,c)] = sum_{t1,t2} G[(s1 s2),(t1 t2)]
//                          sum_b T_k[t1][a][b] T_{k+1}[t2][b][c]
// on the matrix cores.  One wavefront per 16 x 16 tile of (a, c): the nine
// (t1, t2) blocks of the tile are nine MFMA accumulators fed from the same
// operand loads, and the 9 x 9 gate is applied to them in registers.
// Precision T: double (FP64 mode) or float (mixed mode: the FP64 site
// tensors are rounded to FP32 on load, products and the gate are FP32 with
// FP32 accumulation, and theta' is stored as FP64 for the SVD).
// =====================================================================
typedef float v4f __attribute__((ext_vector_type(4)));

template <typename T> struct Mfma;
template <> struct Mfma<double> {
  typedef v4d V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return mfma_f64(a, b, c);
  }
  // row of D held by a lane in element e (FP64 16x16x4 layout)
  static __device__ __forceinline__ int row(int lane, int e) {
    return (lane >> 4) + 4 * e;
  }
};
template <> struct Mfma<float> {
  typedef v4f V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // FP32 16x16x4 layout: lane j + 16 (i / 4) holds D[i][j] in element i % 4
  static __device__ __forceinline__ int row(int lane, int e) {
    return 4 * (lane >> 4) + e;
  }
};

template <typename T>
__global__ void __launch_bounds__(NT) k_theta(Batch b, UpdScratch s, UpdParams u) {
  typedef Mfma<T> M;
  const int c = blockIdx.z;
  const Dims d = dims_of(b, c, u.k);
  __shared__ T G[81];
  if (threadIdx.x < 81) G[threadIdx.x] = (T)u.gate[threadIdx.x];
  __syncthreads();
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int a0 = blockIdx.x * 32 + 16 * (w & 1);
  const int c0 = blockIdx.y * 32 + 16 * (w >> 1);
  if (a0 >= d.chiL || c0 >= d.chiR) return;
  const int chiL = d.chiL, chiM = d.chiM, chiR = d.chiR;
  const double *A = site_ptr(b, c, u.k);
  const double *Bt = site_ptr(b, c, u.k + 1);
  typename M::V acc[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) acc[t] = typename M::V{0, 0, 0, 0};
  // Chunks of 16 b: lane (li, lk) holds A_t[a0 + li][b0 + 4 lk + q] and
  // B_t[b0 + 4 lk + q][c0 + li] for q < 4, and MFMA step q takes k-slot lk
  // = b0 + 4 lk + q (the contraction sums over b, so the order is free).
  // Out-of-range rows, columns and b are read at a clamped address and
  // zeroed by a select: no branch around a load, so the next chunk's loads
  // stay in flight while this chunk is multiplied.
  const int a = min(a0 + li, chiL - 1), cc = min(c0 + li, chiR - 1);
  const bool arow = a0 + li < chiL, bcol = c0 + li < chiR;
  const double *Ar = A + (size_t)a * chiM;
  const double *Bc = Bt + cc;
  const size_t As = (size_t)chiL * chiM, Bs = (size_t)chiM * chiR;
  auto load = [&](int b0, T (&av)[3][4], T (&bv)[3][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int bb = b0 + 4 * lk + q;
      const int bcl = min(bb, chiM - 1);
      const bool ok = bb < chiM;
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const double x = Ar[t * As + bcl];
        const double y = Bc[t * Bs + (size_t)bcl * chiR];
        av[t][q] = (arow && ok) ? (T)x : (T)0;
        bv[t][q] = (bcol && ok) ? (T)y : (T)0;
      }
    }
  };
  auto mult = [&](const T (&av)[3][4], const T (&bv)[3][4]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t1 = 0; t1 < 3; ++t1)
#pragma unroll
        for (int t2 = 0; t2 < 3; ++t2)
          acc[3 * t1 + t2] = M::mma(av[t1][q], bv[t2][q], acc[3 * t1 + t2]);
  };
  T a0v[3][4], b0v[3][4], a1v[3][4], b1v[3][4];
  load(0, a0v, b0v);
  for (int b0 = 0; b0 < chiM; b0 += 32) {
    load(b0 + 16, a1v, b1v);
    asm volatile("" ::: "memory");  // next chunk's loads go first
    mult(a0v, b0v);
    if (b0 + 16 >= chiM) break;
    load(b0 + 32, a0v, b0v);
    asm volatile("" ::: "memory");
    mult(a1v, b1v);
  }
  double *TH = s.TH + (size_t)c * s.th_stride;
  double *X = s.X + (size_t)c * s.th_stride;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int ai = a0 + M::row(lane, e), ci = c0 + li;
    if (ai >= chiL || ci >= chiR) continue;
    T th[9];
#pragma unroll
    for (int t = 0; t < 9; ++t) th[t] = acc[t][e];
#pragma unroll
    for (int s1 = 0; s1 < 3; ++s1)
#pragma unroll
      for (int s2 = 0; s2 < 3; ++s2) {
        T v = 0;
#pragma unroll
        for (int t = 0; t < 9; ++t) v += G[(s1 * 3 + s2) * 9 + t] * th[t];
        // the vector index interleaved (3 bond + s), the element index not
        const size_t off =
            d.trans ? (size_t)(3 * ai + s1) * d.ld + (size_t)s2 * chiR + ci
                    : (size_t)(3 * ci + s2) * d.ld + (size_t)s1 * chiL + ai;
        TH[off] = (double)v;
        X[off] = (double)v;
      }
  }
}

// ||theta'||^2 of every chain in FP64, summed over theta' as stored (before
// any rotation) in a fixed order: the gate's log-weight increment ln
// ||theta'||^2 (the sampling weight is the product of the squared norms of
// the evolution, Hybrid METTS-Ancilla subsection).
// Workgroup x of a chain sums the vectors q = x (mod NORM_SPLIT); the
// partial sums are added in a fixed order by k_truncate.
__global__ void __launch_bounds__(NT) k_theta_norm(Batch b, UpdScratch s,
                                                   UpdParams u) {
  const int c = blockIdx.y;
  const Dims d = dims_of(b, c, u.k);
  const double *TH = s.TH + (size_t)c * s.th_stride;
  __shared__ double red[NT / 64];
  double v = 0.0;
  for (int q = blockIdx.x; q < d.N; q += NORM_SPLIT)
    for (int l = threadIdx.x; l < d.L; l += NT) {
      const double x = TH[(size_t)q * d.ld + l];
      v = fma(x, x, v);
    }
  v = wg_sum(v, red);
  if (threadIdx.x == 0) s.norm2[(size_t)c * NORM_SPLIT + blockIdx.x] = v;
}

// Zero what the blocked paths read beyond theta': the padding rows
// L..ld-1 of every vector and, for the plain rounds, the padding vectors
// N..npad-1 (the QR path writes its own vectors, padding included).
__global__ void __launch_bounds__(NT) k_pad(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.y;
  const Dims d = dims_of(b, c, u.k);
  const bool qr = path_has_qr(path_of(d, u));
  const int npad = npad_vectors(d.N);
  double *X = s.X + (size_t)c * s.th_stride;
  const int tail = d.ld - d.L;
  if (tail > 0)
    for (int i = blockIdx.x * NT + threadIdx.x; i < d.N * tail;
         i += gridDim.x * NT)
      X[(size_t)(i / tail) * d.ld + d.L + i % tail] = 0.0;
  if (qr) return;
  const size_t cnt = (size_t)(npad - d.N) * d.ld;
  double *P = X + (size_t)d.N * d.ld;
  for (size_t i = (size_t)blockIdx.x * NT + threadIdx.x; i < cnt;
       i += (size_t)gridDim.x * NT)
    P[i] = 0.0;
}

// =====================================================================
// One-sided Jacobi SVD, whole matrix in LDS (one workgroup per chain).
// The N vectors are rotated in round-robin pair order until every pair is
// orthogonal to relative tolerance tol; then X = U Sigma (vector side) and
// the squared vector norms are written to sig2.
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_jacobi_small(Batch b, UpdScratch s, UpdParams u, size_t small_max) {
  const int c = blockIdx.x;
  const Dims d = dims_of(b, c, u.k);
  const int L = d.L, N = d.N;
  if ((size_t)L * N > small_max) return;  // this chain takes the blocked path
  double *X = s.X + (size_t)c * s.th_stride;
  __shared__ double xs[SMALL_LDS];
  __shared__ int flag;
  const int tid = threadIdx.x;
  for (int idx = tid; idx < L * N; idx += NT)
    xs[idx] = X[(size_t)(idx / L) * d.ld + idx % L];
  const int n_even = N + (N & 1);
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
        if (q < N) {
          double aa = 0.0, bb = 0.0, gg = 0.0;
          for (int i = lane; i < L; i += g) {
            const double x = xs[p * L + i], y = xs[q * L + i];
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
          if (jacobi_rotation(aa, bb, gg, u.tol, u.skip, cr, sr)) {
            for (int i = lane; i < L; i += g) {
              const double x = xs[p * L + i], y = xs[q * L + i];
              xs[p * L + i] = cr * x - sr * y;
              xs[q * L + i] = sr * x + cr * y;
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
  for (int idx = tid; idx < L * N; idx += NT)
    X[(size_t)(idx / L) * d.ld + idx % L] = xs[idx];
  double *sig2 = s.sig2 + (size_t)c * s.n_cap;
  for (int j = tid; j < N; j += NT) {
    double v = 0.0;
    for (int i = 0; i < L; ++i) v += xs[j * L + i] * xs[j * L + i];
    sig2[j] = v;
  }
  if (tid == 0) {
    if (!converged) s.err[c] = 1;
    s.sweeps[c] += converged ? sweep + 1 : sweep;
  }
}

// Chains whose SVD runs in LDS take no part in the blocked rounds.
__global__ void k_mark_small_done(Batch b, UpdScratch s, UpdParams u,
                                  size_t small_max) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.B) return;
  const Dims d = dims_of(b, c, u.k);
  if ((size_t)d.L * d.N <= small_max) s.done[c] = 1;
}

// =====================================================================
// Truncation: sort the singular values (bitonic, LDS), then keep the
//   number truncation_rule gives (chi_max, the relative discarded weight,
//   the numerical floor, no cut inside a run of ties).
//   ln ||theta'||^2 (k_theta_norm) goes into logw for a gate (the sampling
//   weight is the product of these norms).
// =====================================================================
__global__ void __launch_bounds__(NT)
    k_truncate(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.x;
  const Dims d = dims_of(b, c, u.k);
  // the mixed path resolves only the rr_vectors largest singular values;
  // the rest of ||theta'||^2 is the unresolved tail
  const bool rr = path_is_rr(path_of(d, u));
  const int N = rr ? s.rrk[c] : d.N;
  __shared__ double key[2048];
  __shared__ int idx[2048];
  __shared__ int kk_s;
  const int tid = threadIdx.x;
  int N2 = 1;
  while (N2 < N) N2 <<= 1;
  const double *sig2 = s.sig2 + (size_t)c * s.n_cap;
  for (int j = tid; j < N2; j += NT) {
    key[j] = (j < N) ? sqrt(fmax(sig2[j], 0.0)) : -1.0;
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
    double n2 = 0.0;  // ||theta'||^2 in FP64, summed from theta'
    if (u.is_gate || rr)
      for (int x = 0; x < NORM_SPLIT; ++x)
        n2 += s.norm2[(size_t)c * NORM_SPLIT + x];
    const TruncResult tr =
        truncation_rule(key, N, rr, n2, u.chi_max, u.cutoff);
    int k = tr.k;
    const double total = tr.total;
    double kept = tr.kept;
    if (u.zero_ok && total == 0.0) {
      k = 0;  // an empty charge block: nothing to keep
      kept = 1.0;
    } else if (!(total > 0.0) || !isfinite(total) || !(kept > 0.0)) {
      s.err[c] = 2;
    }
    s.fac[c] = 1.0 / sqrt(kept);
    if (u.is_gate) s.logw[c] += log(n2);
    if (total > 0.0) s.discarded[c] += (total - kept) / total;
    s.knew[c] = k;
    kk_s = k;
  }
  __syncthreads();
  const int k = kk_s;
  for (int j = tid; j < k; j += NT) {
    s.perm[(size_t)c * s.n_cap + j] = idx[j];
    s.sig[(size_t)c * s.n_cap + j] = key[j];
  }
  // the new bond dimension is published last: the write-back kernels read
  // the old chi of bonds k and k+2 only
  if (tid == 0) b.chi[(size_t)c * (b.nsites + 1) + u.k + 1] = k;
}

// =====================================================================
// Write-back.  X = U_v Sigma with U_v the singular vectors on the vector
// side (U for the normal layout, V for the transposed one).  The vector-
// side site takes X_j scaled by fac (if the orthogonality centre moves
// there) or by 1/sigma_j (isometry); the other site takes the projection
// X_j^T TH scaled by 1/sigma_j^2 (isometry) or fac/sigma_j (centre).
// Normal layout: vector side is site k (rows (s1,a)); transposed: site k+1
// (columns (s2,c)).  With fac = 1/||kept||, right = 1 gives T_k = U,
// T_{k+1} = fac Sigma V^T; right = 0 gives T_k = fac U Sigma, T_{k+1} = V^T.
// =====================================================================
// Element i of a row-side factor (site k, T[s1][a][j]) and element q of a
// column-side factor (site k+1, T[s2][j][c]); il: the index is interleaved.
__device__ __forceinline__ void store_row(const Batch &b, int c, int k,
                                          const Dims &d, int knew, int i,
                                          int j, double v) {
  const int s1 = d.il_rows ? i % 3 : i / d.chiL;
  const int a = d.il_rows ? i / 3 : i - s1 * d.chiL;
  site_ptr(b, c, k)[(size_t)s1 * d.chiL * knew + (size_t)a * knew + j] = v;
}
__device__ __forceinline__ void store_col(const Batch &b, int c, int k,
                                          const Dims &d, int knew, int q,
                                          int j, double v) {
  const int s2 = d.il_cols ? q % 3 : q / d.chiR;
  const int cc = d.il_cols ? q / 3 : q - s2 * d.chiR;
  site_ptr(b, c, k + 1)[(size_t)s2 * knew * d.chiR + (size_t)j * d.chiR + cc] =
      v;
}
__device__ __forceinline__ void store_vector_side(const Batch &b, int c,
                                                  int k, const Dims &d,
                                                  int knew, int l, int j,
                                                  double v) {
  if (!d.trans)
    store_row(b, c, k, d, knew, l, j, v);
  else
    store_col(b, c, k, d, knew, l, j, v);
}
__device__ __forceinline__ void store_other_side(const Batch &b, int c,
                                                 int k, const Dims &d,
                                                 int knew, int q, int j,
                                                 double v) {
  if (!d.trans)
    store_col(b, c, k, d, knew, q, j, v);
  else
    store_row(b, c, k, d, knew, q, j, v);
}

// Dims as they were before the truncation: chi[k+1] now holds knew, but
// nothing here depends on the old middle dimension.  The two-QR path
// writes both sides by projection (below).
__global__ void __launch_bounds__(NT)
    k_writeback_direct(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.y;
  const Dims d = dims_of(b, c, u.k);
  const int path = path_of(d, u);
  if (path == PATH_QR2) return;
  // the two-QR mixed path ends like the QR path: sigma_j w_j in Y
  const bool qr = path == PATH_QR || path == PATH_RR2;
  const Dims e = vector_side(d, qr);
  const int vlen = qr ? d.N : d.L, vld = qr ? vec_ld(d.N) : d.ld;
  const int k = s.knew[c];
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= vlen * k) return;
  const int l = t % vlen, j = t / vlen;
  const int col = s.perm[(size_t)c * s.n_cap + j];
  const bool vec_center = (e.trans != 0) == (u.right != 0);
  const double f =
      vec_center ? s.fac[c] : 1.0 / s.sig[(size_t)c * s.n_cap + j];
  const double *V = (qr ? s.Y : s.X) + (size_t)c * s.th_stride;
  store_vector_side(b, c, u.k, e, k, l, j, V[(size_t)col * vld + l] * f);
}

// The other side.  With X_j = sigma_j x_j the converged vectors (x_j unit
// singular vectors on the vector side) and M the vector matrix of the path
// (theta' or its transpose as stored in TH), the unit singular vectors on
// the other side are p_j = op(M) X_j / sigma_j^2: op(M) = M^T on the plain
// path (X_j of length L, p_j of length N), op(M) = M on the QR path (X_j
// = Y_j of length N, p_j of length L).  On the two-QR path the converged
// vectors (in Z) are sigma_j u~_j with u~_j the left singular vectors in
// the basis of Q (R = U~ Sigma W^T): the right ones are p_j = R^T u~_j /
// sigma_j, from the R kept in the upper triangle of X, and the left ones
// Q u~_j come from the stored reflectors (k_qr2_fill, the reflectors in
// qr.hip, k_qr2_store_left).  A second projection, M p_j / sigma_j, would
// amplify the residual error of p_j along the larger singular vectors by
// sigma_0 / sigma_j.
// The projections are orthonormal only to about eps sigma_0 / sigma_j, so
// they are corrected before they are stored, to first order in E (G = P^T
// P = I + E) along the Cholesky factor of G taken in the order of
// decreasing sigma: p_j <- p_j (1 - E_jj / 2) - sum_{i<j} p_i E_ij.
// Column j is made orthonormal against the columns of larger singular
// value and never feeds back into them, so the large rounding error of a
// tiny-sigma projection stays in that column (where the state weighs it by
// sigma_j).
//   k_other_project  P into a free buffer, column j at j * ldP, zero rows
//                    P_len .. ldP-1
//   k_other_gram     G = P^T P into a free buffer (row-major, stride
//                    round16(k), zero beyond k)
//   k_other_store    corrected, scaled P into the site tensor
// All three on the FP64 matrix cores, one 16 x 16 tile per wavefront.
enum { OM_PLAIN = 0, OM_QR, OM_QR2 };
struct Other {
  int mode, len, ldP, k, ldG;
  double *P;
  double *G;
};

__device__ __forceinline__ Other other_of(const Dims &d, const UpdParams &u,
                                          const UpdScratch &s, int c) {
  const int path = path_of(d, u);
  Other o;
  o.mode = path == PATH_QR2 ? OM_QR2
           : (path == PATH_QR || path == PATH_RR2) ? OM_QR
                                                   : OM_PLAIN;
  o.len = o.mode == OM_QR ? d.L : d.N;
  o.ldP = vec_ld(o.len);
  o.k = s.knew[c];
  o.ldG = (o.k + 15) & ~15;
  const size_t off = (size_t)c * s.th_stride;
  o.P = (o.mode == OM_QR ? s.X : s.Y) + off;
  o.G = (o.mode == OM_QR2 ? s.Z : s.TH) + off;
  return o;
}

// Two-QR path, left factor: u~_j = Z_pj / sigma_j into TH (length L, stride
// ld, zero from row N), for the reflectors to turn into Q u~_j.
__global__ void __launch_bounds__(NT)
    k_qr2_fill(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.y;
  const Dims d = dims_of(b, c, u.k);
  if (path_of(d, u) != PATH_QR2) return;
  const int k = s.knew[c];
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= d.ld * k) return;
  const int r = t % d.ld, j = t / d.ld;
  const int ldN = vec_ld(d.N);
  const int pj = s.perm[(size_t)c * s.n_cap + j];
  const double *z = s.Z + (size_t)c * s.th_stride + (size_t)pj * ldN;
  const double v = r < d.N ? z[r] / s.sig[(size_t)c * s.n_cap + j] : 0.0;
  s.TH[(size_t)c * s.th_stride + (size_t)j * d.ld + r] = v;
}

// Two-QR path: the left factor Q u~_j (in TH) into the site tensor, scaled
// like the other side of the QR path.
__global__ void __launch_bounds__(NT)
    k_qr2_store_left(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.y;
  const Dims d = dims_of(b, c, u.k);
  if (path_of(d, u) != PATH_QR2) return;
  const int k = s.knew[c];
  const int t = blockIdx.x * NT + threadIdx.x;
  if (t >= d.L * k) return;
  const int r = t % d.L, j = t / d.L;
  const Dims e = vector_side(d, true);
  const bool vec_center = (e.trans != 0) == (u.right != 0);
  const double f = vec_center
                       ? 1.0
                       : s.fac[c] * s.sig[(size_t)c * s.n_cap + j];
  store_other_side(b, c, u.k, e, k, r, j,
                   f * s.TH[(size_t)c * s.th_stride + (size_t)j * d.ld + r]);
}

// P tile (rows r0 .. r0+15, vectors j0 .. j0+15) per wavefront.
__global__ void __launch_bounds__(NT)
    k_other_project(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.z;
  const Dims d = dims_of(b, c, u.k);
  const Other o = other_of(d, u, s, c);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = blockIdx.x * 64 + 16 * w, j0 = blockIdx.y * 16;
  if (r0 >= o.ldP || j0 >= o.k) return;
  const double *M = s.TH + (size_t)c * s.th_stride;
  const int32_t *perm = s.perm + (size_t)c * s.n_cap;
  const bool jok = j0 + li < o.k;
  const int pj = perm[jok ? j0 + li : j0];
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  if (o.mode == OM_QR) {
    // D[l][j] = sum_q M[l][q] Y[q][pj]: lane (li, lk) takes row r0 + li of
    // M (single coalesced loads per q) and q = q0 + 4 lk .. + 3 of Y_pj
    const int ldN = vec_ld(d.N);
    const double *yv = s.Y + (size_t)c * s.th_stride + (size_t)pj * ldN;
    const bool lok = r0 + li < d.L;
    const double *mrow = M + (lok ? r0 + li : 0);
    for (int q0 = 0; q0 < d.N; q0 += 16) {
      const int qb = q0 + 4 * lk;
      const v4d yq = *reinterpret_cast<const v4d *>(yv + qb);
      double mv[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int qq = min(qb + q, d.N - 1);
        const double x = mrow[(size_t)qq * d.ld];
        mv[q] = (lok && qb + q < d.N) ? x : 0.0;
      }
      acc = mfma_f64(mv[0], jok ? yq.x : 0.0, acc);
      acc = mfma_f64(mv[1], jok ? yq.y : 0.0, acc);
      acc = mfma_f64(mv[2], jok ? yq.z : 0.0, acc);
      acc = mfma_f64(mv[3], jok ? yq.w : 0.0, acc);
    }
  } else {
    // D[q][j] = sum_l A[l][q] V[l][pj]: both operands as aligned 32-byte
    // loads of four consecutive l.  Plain path: A = M (column q of TH), V
    // = X (length L, rows L .. ld-1 zero).  Two-QR path: A = R (column q
    // of R is the upper part of column q of X: l <= q), V = the converged
    // vectors in Z (length N).
    const bool qr2 = o.mode == OM_QR2;
    const int vlen = qr2 ? d.N : d.L, vld = qr2 ? vec_ld(d.N) : d.ld;
    const double *xv = (qr2 ? s.Z : s.X) + (size_t)c * s.th_stride +
                       (size_t)pj * vld;
    const double *A = qr2 ? s.X + (size_t)c * s.th_stride : M;
    const int qrow = r0 + li;
    const bool qok = qrow < d.N;
    const double *acol = A + (size_t)(qok ? qrow : 0) * d.ld;
    // R is upper triangular: rows l <= r0 + 15 reach this tile
    const int lend = qr2 ? min(vlen, r0 + 16) : vlen;
    for (int l0 = 0; l0 < lend; l0 += 16) {
      const int lb = l0 + 4 * lk;
      const v4d xq = *reinterpret_cast<const v4d *>(xv + lb);
      const v4d mq = *reinterpret_cast<const v4d *>(acol + lb);
      // rows L .. ld-1 of TH are not written by the update, and X holds
      // the reflectors below the diagonal of R: mask them
      const int lim = qr2 ? min(vlen - 1, qrow) : vlen - 1;
      const bool l0ok = lb <= lim, l1ok = lb + 1 <= lim, l2ok = lb + 2 <= lim,
                 l3ok = lb + 3 <= lim;
      acc = mfma_f64(qok && l0ok ? mq.x : 0.0, jok ? xq.x : 0.0, acc);
      acc = mfma_f64(qok && l1ok ? mq.y : 0.0, jok ? xq.y : 0.0, acc);
      acc = mfma_f64(qok && l2ok ? mq.z : 0.0, jok ? xq.z : 0.0, acc);
      acc = mfma_f64(qok && l3ok ? mq.w : 0.0, jok ? xq.w : 0.0, acc);
    }
  }
  if (!jok) return;
  const double sg = s.sig[(size_t)c * s.n_cap + j0 + li];
  const double inv = 1.0 / (sg * sg);
  // D[i][j] (row r0 + i, vector j0 + j) in lane j + 16 (i % 4), element i/4
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + lk + 4 * q;
    o.P[(size_t)(j0 + li) * o.ldP + r] = r < o.len ? acc[q] * inv : 0.0;
  }
}

// G tile (j1 .. j1+15, j2 .. j2+15) per wavefront; contraction over the
// rows of P (zero beyond len) as aligned 32-byte loads.
__global__ void __launch_bounds__(NT)
    k_other_gram(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.z;
  const Dims d = dims_of(b, c, u.k);
  const Other o = other_of(d, u, s, c);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int j1 = blockIdx.x * 64 + 16 * w, j2 = blockIdx.y * 16;
  if (j1 >= o.ldG || j2 >= o.ldG) return;
  const bool aok = j1 + li < o.k, bok = j2 + li < o.k;
  const double *pa = o.P + (size_t)(aok ? j1 + li : 0) * o.ldP;
  const double *pb = o.P + (size_t)(bok ? j2 + li : 0) * o.ldP;
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int r0 = 0; r0 < o.ldP; r0 += 16) {
    const int rb = r0 + 4 * lk;
    const v4d a = *reinterpret_cast<const v4d *>(pa + rb);
    const v4d bb = *reinterpret_cast<const v4d *>(pb + rb);
    acc = mfma_f64(aok ? a.x : 0.0, bok ? bb.x : 0.0, acc);
    acc = mfma_f64(aok ? a.y : 0.0, bok ? bb.y : 0.0, acc);
    acc = mfma_f64(aok ? a.z : 0.0, bok ? bb.z : 0.0, acc);
    acc = mfma_f64(aok ? a.w : 0.0, bok ? bb.w : 0.0, acc);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q)
    o.G[(size_t)(j1 + lk + 4 * q) * o.ldG + j2 + li] = acc[q];
}

// out[r][j] = P[r][j] (3 - G[j][j]) / 2 - sum_{i<j} P[r][i] G[i][j], times
// 1 for an isometry or fac sigma_j for the centre; G is symmetric, so lane
// (li, lk) loads G[j0 + li][i0 + 4 lk .. + 3] as one aligned 32-byte load.
// The two-QR path stores this factor on its vector side.
__global__ void __launch_bounds__(NT)
    k_other_store(Batch b, UpdScratch s, UpdParams u) {
  const int c = blockIdx.z;
  const Dims d = dims_of(b, c, u.k);
  const Other o = other_of(d, u, s, c);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int r0 = blockIdx.x * 64 + 16 * w, j0 = blockIdx.y * 16;
  if (r0 >= o.len || j0 >= o.k) return;
  const bool jok = j0 + li < o.k;
  const double *grow = o.G + (size_t)(jok ? j0 + li : 0) * o.ldG;
  const double *prow = o.P + r0 + li;  // row r0 + li of every column
  v4d acc = {0.0, 0.0, 0.0, 0.0};
  for (int i0 = 0; i0 < o.ldG; i0 += 16) {
    const int ib = i0 + 4 * lk;
    const v4d g = *reinterpret_cast<const v4d *>(grow + ib);
    double pv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ii = min(ib + q, o.k - 1);
      const double x = prow[(size_t)ii * o.ldP];
      pv[q] = ib + q < o.k ? x : 0.0;
    }
    // only i < j (the strictly upper part of E)
    const int jj = j0 + li;
    acc = mfma_f64(pv[0], jok && ib < jj ? g.x : 0.0, acc);
    acc = mfma_f64(pv[1], jok && ib + 1 < jj ? g.y : 0.0, acc);
    acc = mfma_f64(pv[2], jok && ib + 2 < jj ? g.z : 0.0, acc);
    acc = mfma_f64(pv[3], jok && ib + 3 < jj ? g.w : 0.0, acc);
  }
  if (!jok) return;
  const int j = j0 + li;
  const double gjj = o.G[(size_t)j * o.ldG + j];
  const Dims e = vector_side(d, o.mode != OM_PLAIN);
  const bool vec_center = (e.trans != 0) == (u.right != 0);
  const double fsig = s.fac[c] * s.sig[(size_t)c * s.n_cap + j];
  if (o.mode == OM_QR2) {
    const double f = vec_center ? fsig : 1.0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = r0 + lk + 4 * q;
      if (r < o.len) {
        const double pr = o.P[(size_t)j * o.ldP + r];
        store_vector_side(b, c, u.k, e, o.k, r, j,
                          f * (pr * (1.5 - 0.5 * gjj) - acc[q]));
      }
    }
    return;
  }
  const double f = vec_center ? 1.0 : fsig;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + lk + 4 * q;
    if (r < o.len) {
      const double pr = o.P[(size_t)j * o.ldP + r];
      store_other_side(b, c, u.k, e, o.k, r, j,
                       f * (pr * (1.5 - 0.5 * gjj) - acc[q]));
    }
  }
}

}  // namespace

// ---- launchers ---------------------------------------------------------
void launch_theta(const Batch &b, const UpdScratch &s, const UpdParams &u,
                  int max_chiL, int max_chiR, hipStream_t st) {
  dim3 grid((max_chiL + 31) / 32, (max_chiR + 31) / 32, b.B);
  if (u.mixed)
    hipLaunchKernelGGL(k_theta<float>, grid, dim3(NT), 0, st, b, s, u);
  else
    hipLaunchKernelGGL(k_theta<double>, grid, dim3(NT), 0, st, b, s, u);
}

void launch_theta_norm(const Batch &b, const UpdScratch &s,
                       const UpdParams &u, hipStream_t st) {
  hipLaunchKernelGGL(k_theta_norm, dim3(NORM_SPLIT, b.B), dim3(NT), 0, st, b,
                     s, u);
}

void launch_pad(const Batch &b, const UpdScratch &s, const UpdParams &u,
                hipStream_t st) {
  hipLaunchKernelGGL(k_pad, dim3(16, b.B), dim3(NT), 0, st, b, s, u);
}

void launch_jacobi_small(const Batch &b, const UpdScratch &s,
                         const UpdParams &u, hipStream_t st) {
  launch_jacobi_small_upto(b, s, u, SMALL_LDS, st);
}

void launch_jacobi_small_upto(const Batch &b, const UpdScratch &s,
                              const UpdParams &u, size_t small_max,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_small, dim3(b.B), dim3(NT), 0, st, b, s, u,
                     small_max);
}

void launch_mark_small_done(const Batch &b, const UpdScratch &s,
                            const UpdParams &u, size_t small_max,
                            hipStream_t st) {
  hipLaunchKernelGGL(k_mark_small_done, dim3((b.B + NT - 1) / NT), dim3(NT),
                     0, st, b, s, u, small_max);
}

void launch_truncate(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_truncate, dim3(b.B), dim3(NT), 0, st, b, s, u);
}

void launch_writeback(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int max_L, int max_N, int max_k, int qr2_panels,
                      hipStream_t st) {
  (void)max_N;
  const int nd = (max_L * max_k + NT - 1) / NT;
  hipLaunchKernelGGL(k_writeback_direct, dim3(nd, b.B), dim3(NT), 0, st, b, s,
                     u);
  const int rows = (max_L + 15) & ~15, kk = (max_k + 15) & ~15;
  if (qr2_panels > 0) {
    // left factor of the two-QR path: Q u~ = H_1 .. H_N [u~; 0], the
    // block reflectors from the last panel to the first; Z is read here
    // and by the projection below, before the Gram overwrites it
    const int nf = (rows * max_k + NT - 1) / NT;
    hipLaunchKernelGGL(k_qr2_fill, dim3(nf, b.B), dim3(NT), 0, st, b, s, u);
    for (int p = qr2_panels - 1; p >= 0; --p)
      launch_qr_apply(b, s, u, p, kk / 16, st);
    hipLaunchKernelGGL(k_qr2_store_left, dim3(nd, b.B), dim3(NT), 0, st, b, s,
                       u);
  }
  // the other side has at most max_L rows (L on the QR path, N <= L on
  // the plain and two-QR paths), padded to 16
  dim3 gp((rows + 63) / 64, kk / 16, b.B);
  hipLaunchKernelGGL(k_other_project, gp, dim3(NT), 0, st, b, s, u);
  dim3 gg((kk + 63) / 64, kk / 16, b.B);
  hipLaunchKernelGGL(k_other_gram, gg, dim3(NT), 0, st, b, s, u);
  hipLaunchKernelGGL(k_other_store, gp, dim3(NT), 0, st, b, s, u);
}

}  // namespace hmps
