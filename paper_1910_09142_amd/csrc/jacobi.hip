// Blocked one-sided Jacobi SVD round on gfx950 matrix cores
// (the SVD that restores the MPS form after every two-site gate;
// Chen & Stoudenmire, arXiv:1910.09142, Results section).
//
// The N vectors (columns of the L x N vector matrix X, column-major) are
// split into NB (even) blocks of JB.  A sweep has NB-1 rounds; in a round
// the blocks are paired by the circle method and one workgroup handles
// one block pair of one chain:
//   1. Gram matrix G = Xp^T Xp of the 2 JB vectors: wavefronts 0, 1, 2
//      compute the tiles II, IJ, JJ with FP64 MFMA;
//   2. if every off-diagonal element is below tol sqrt(G_ii G_jj) the pair
//      is orthogonal: record the squared norms and stop;
//   3. one cyclic two-sided Jacobi sweep on G in LDS accumulating the
//      rotations in Q (one thread per 2 x 2 block of a rotation round, in
//      place);
//   4. Xp <- Xp Q (FP64 MFMA, 16-row chunks, coalesced stores).
// About 17 KB of LDS per workgroup, so many chains' block pairs share a CU.
#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

constexpr int P2 = 2 * JB;  // vectors in a block pair
constexpr int NPAIR = JB;   // disjoint pairs in one inner rotation round

__global__ void k_jacobi_sweep_begin(UpdScratch s, int B, int sweep) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= B) return;
  if (sweep == 0)
    s.done[c] = 0;
  else if (s.rot_cur[c] == 0)
    s.done[c] = 1;
  s.rot_cur[c] = 0;
}

// Rotation (x_p, x_q) <- (c x_p - s x_q, s x_p + c x_q) that zeroes the
// inner product g of two vectors with squared norms a, b (the same angle
// as tan 2phi = 2g / (b - a), smaller root), written with one square root,
// one division and one reciprocal square root.
__device__ __forceinline__ bool pair_rotation(double a, double b, double g,
                                              double tol, double skip,
                                              double &c, double &s) {
  if (!pair_needs_rotation(a, b, g, tol, skip)) return false;
  const double d = b - a;
  const double r = sqrt(d * d + 4.0 * g * g);
  const double t = copysign(1.0, d) * (2.0 * g) / (fabs(d) + r);
  c = rsqrt(1.0 + t * t);
  s = c * t;
  return true;
}

// at most 128 registers: four workgroups of this kernel fit on a CU
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4)))
    k_jacobi_round(Batch b, UpdScratch s, UpdParams u, int r) {
  const int c = blockIdx.y, pi = blockIdx.x;
  if (s.done[c]) return;
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  const int L = m > n ? m : n, N = m > n ? n : m;
  const int NB = n_blocks_even(N);
  if (r >= NB - 1 || pi >= NB / 2) return;
  int bi, bj;
  rr_pair(r, pi, NB, bi, bj);
  double *X = s.X + (size_t)c * s.th_stride;

  __shared__ double G[P2][P2 + 1];
  __shared__ double Q[P2][P2 + 1];
  __shared__ double cs[NPAIR], sn[NPAIR];
  __shared__ int flag;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;

  // ---- 1. Gram tiles: wave 0 = II, 1 = IJ, 2 = JJ; wave 3 sets Q = I ----
  if (w < 3) {
    const int ba = (w == 2) ? bj : bi, bb = (w == 0) ? bi : bj;
    const double *xa = X + (size_t)(ba * JB + li) * L;
    const double *xb = X + (size_t)(bb * JB + li) * L;
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    // software pipeline: the loads of the next GB k-steps are in flight
    // while the MFMAs of the current ones run
    constexpr int GB = 4;
    double ca[GB], cb[GB], na[GB], nb[GB];
    auto load = [&](int base, double *va, double *vb) {
#pragma unroll
      for (int t = 0; t < GB; ++t) {
        const int e = base + 4 * t + lk;
        va[t] = e < L ? xa[e] : 0.0;
        vb[t] = e < L ? xb[e] : 0.0;
      }
    };
    load(0, ca, cb);
    for (int e0 = 0; e0 < L; e0 += 4 * GB) {
      if (e0 + 4 * GB < L) load(e0 + 4 * GB, na, nb);
#pragma unroll
      for (int t = 0; t < GB; t += 2) {
        acc0 = mfma_f64(ca[t], cb[t], acc0);
        acc1 = mfma_f64(ca[t + 1], cb[t + 1], acc1);
      }
#pragma unroll
      for (int t = 0; t < GB; ++t) {
        ca[t] = na[t];
        cb[t] = nb[t];
      }
    }
    const int ro = (w == 2) ? JB : 0, co = (w == 0) ? 0 : JB;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = lk + 4 * q;
      const double v = acc0[q] + acc1[q];
      G[ro + i][co + li] = v;
      if (w == 1) G[JB + li][i] = v;  // G_JI = G_IJ^T
    }
  } else {
    for (int idx = lane; idx < P2 * P2; idx += 64)
      Q[idx / P2][idx % P2] = (idx / P2 == idx % P2) ? 1.0 : 0.0;
    if (lane == 0) flag = 0;
  }
  __syncthreads();

  // ---- 2. convergence test -----------------------------------------------
  for (int idx = tid; idx < P2 * P2; idx += NT) {
    const int i = idx / P2, j = idx % P2;
    if (i < j && pair_needs_rotation(G[i][i], G[j][j], G[i][j], u.tol, u.skip))
      flag = 1;
  }
  __syncthreads();
  const int needs_rotation = flag;
  __syncthreads();  // every wave has read flag before it is reused below
  if (!needs_rotation) {
    if (tid < P2) {
      const int col = tid < JB ? bi * JB + tid : bj * JB + tid - JB;
      if (col < N) s.sig2[(size_t)c * s.n_cap + col] = G[tid][tid];
    }
    return;
  }

  // ---- 3. inner Jacobi sweeps on G, rotations accumulated in Q ------------
  // Thread t owns the 2 x 2 block (row pair t / NPAIR, column pair
  // t % NPAIR) of G and two (row, column pair) items of Q; every element
  // belongs to exactly one owner, so the update is in place.
  const int rp = tid / NPAIR, cp = tid % NPAIR;
  const double tol_in = fmax(0.125 * u.tol, 4e-16);
  for (int isw = 0; isw < u.inner_sweeps; ++isw) {
    if (tid == 0) flag = 0;
    for (int rr = 0; rr < P2 - 1; ++rr) {
      if (tid < NPAIR) {
        int p, q;
        rr_pair(rr, tid, P2, p, q);
        double cr = 1.0, sr = 0.0;
        if (pair_rotation(G[p][p], G[q][q], G[p][q], tol_in, u.skip, cr, sr))
          flag = 1;
        cs[tid] = cr;
        sn[tid] = sr;
      }
      __syncthreads();
      {
        int p1, q1, p2, q2;
        rr_pair(rr, rp, P2, p1, q1);
        rr_pair(rr, cp, P2, p2, q2);
        const double c1 = cs[rp], s1 = sn[rp], c2 = cs[cp], s2 = sn[cp];
        const double g11 = G[p1][p2], g12 = G[p1][q2];
        const double g21 = G[q1][p2], g22 = G[q1][q2];
        // rows: J^T G
        const double h11 = c1 * g11 - s1 * g21, h12 = c1 * g12 - s1 * g22;
        const double h21 = s1 * g11 + c1 * g21, h22 = s1 * g12 + c1 * g22;
        // columns: (J^T G) J
        G[p1][p2] = c2 * h11 - s2 * h12;
        G[p1][q2] = s2 * h11 + c2 * h12;
        G[q1][p2] = c2 * h21 - s2 * h22;
        G[q1][q2] = s2 * h21 + c2 * h22;
      }
#pragma unroll
      for (int h = 0; h < P2 * NPAIR / NT; ++h) {
        const int item = tid + NT * h;
        const int row = item / NPAIR, pq = item % NPAIR;
        int p, q;
        rr_pair(rr, pq, P2, p, q);
        const double cq = cs[pq], sq = sn[pq];
        const double x = Q[row][p], y = Q[row][q];
        Q[row][p] = cq * x - sq * y;
        Q[row][q] = sq * x + cq * y;
      }
      __syncthreads();
    }
    const int rotated = flag;
    __syncthreads();  // read before the next sweep resets it
    if (!rotated) break;
  }

  // ---- 4. Xp <- Xp Q, as D = Q^T Xp^T per 16-row chunk --------------------
  // the chunk of rows e0 + 64 is loaded while chunk e0 is multiplied
  constexpr int KB = P2 / 4;
  double cur[KB], nxt[KB];
  auto load_chunk = [&](int e0, double *v) {
    const int e = e0 + li;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const int t = 4 * kk + lk;
      const int col = t < JB ? bi * JB + t : bj * JB + t - JB;
      v[kk] = e < L ? X[(size_t)col * L + e] : 0.0;
    }
  };
  if (16 * w < L) load_chunk(16 * w, cur);
  for (int e0 = 16 * w; e0 < L; e0 += 64) {
    if (e0 + 64 < L) load_chunk(e0 + 64, nxt);
    v4d d0 = {0.0, 0.0, 0.0, 0.0}, d1 = d0;
    const int e = e0 + li;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      d0 = mfma_f64(Q[4 * kk + lk][li], cur[kk], d0);
      d1 = mfma_f64(Q[4 * kk + lk][JB + li], cur[kk], d1);
    }
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) cur[kk] = nxt[kk];
    if (e < L) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int jo = lk + 4 * q;
        X[(size_t)(bi * JB + jo) * L + e] = d0[q];
        X[(size_t)(bj * JB + jo) * L + e] = d1[q];
      }
    }
  }
  if (tid == 0) atomicAdd(&s.rot_cur[c], 1);
}

}  // namespace

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

}  // namespace hmps
