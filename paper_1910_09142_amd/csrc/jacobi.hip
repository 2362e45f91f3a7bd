// Blocked one-sided Jacobi SVD round on gfx950 matrix cores
// (the SVD that restores the MPS form after every two-site gate;
// Chen & Stoudenmire, arXiv:1910.09142, Results section).
//
// The N vectors (columns of the L x N vector matrix X, column-major) are
// split into NB (even) blocks of JB.  A sweep has NB-1 rounds; in a round
// the blocks are paired by the circle method and one workgroup of eight
// wavefronts handles one block pair of one chain:
//   1. Gram matrix G = Xp^T Xp of the 2 JB vectors: six wavefronts compute
//      the tiles II, IJ, JJ over alternate 16-row chunks (FP64 MFMA fed by
//      coalesced 32-byte loads, software-pipelined), summed in LDS in a
//      fixed order;
//   2. if every off-diagonal element is below tol sqrt(G_ii G_jj) the pair
//      is orthogonal: record the squared norms and stop;
//   3. one cyclic two-sided Jacobi sweep on G in LDS accumulating the
//      rotations in Q (one thread per 2 x 2 block of G and per (row,
//      column pair) item of Q, in place);
//   4. Xp <- Xp Q (FP64 MFMA, 16-row chunks over eight wavefronts,
//      coalesced stores).
#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

constexpr int RT = 512;     // threads of the round kernel (8 wavefronts)
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

// at most 128 registers: two workgroups of this kernel fit on a CU
__global__ void __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(4)))
    k_jacobi_round(Batch b, UpdScratch s, UpdParams u, int r) {
  const int c = blockIdx.y, pi = blockIdx.x;
  if (s.done[c]) return;
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  const int L = m > n ? m : n, N = m > n ? n : m;
  const int NB = n_blocks_even(N);
  if (r >= NB - 1 || pi >= NB / 2) return;
  const int ld = vec_ld(L);
  int bi, bj;
  rr_pair(r, pi, NB, bi, bj);
  double *X = s.X + (size_t)c * s.th_stride;

  __shared__ double G[P2][P2 + 1];
  // partial Gram tiles [row half][tile][16][16]; reused as Q afterwards
  __shared__ double scratch[2 * 3 * JB * JB];
  double (*Q)[P2 + 1] = reinterpret_cast<double (*)[P2 + 1]>(scratch);
  static_assert(P2 * (P2 + 1) <= 2 * 3 * JB * JB, "Q fits in the scratch");
  __shared__ double cs[NPAIR], sn[NPAIR];
  __shared__ int flag;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;

  // ---- 1. Gram tiles: wave w < 6 computes tile w % 3 (II, IJ, JJ) over
  //         the groups of k-steps of parity w / 3 ----------------------------
  if (w < 6) {
    const int tile = w % 3, half = w / 3;
    const int ba = (tile == 2) ? bj : bi, bb = (tile == 0) ? bi : bj;
    const double *xa = X + (size_t)(ba * JB + li) * ld;
    const double *xb = X + (size_t)(bb * JB + li) * ld;
    v4d acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = acc0;
    // Chunks of 16 rows: lane (li, lk) reads rows e0 + 4 lk .. e0 + 4 lk + 3
    // of its column as one aligned 32-byte load, and MFMA step t takes row
    // e0 + 4 lk + t (the Gram sums over rows, so the row order is free).
    // The wave of parity `half` takes chunks half, half + 2, ...; the next
    // chunk is loaded while the current one is multiplied.  Rows L..ld-1
    // are zero.
    double4 ca, cb, na, nb;
    auto load = [&](int e0, double4 &va, double4 &vb) {
      const int e = e0 + 4 * lk;
      if (e < ld) {
        va = *reinterpret_cast<const double4 *>(xa + e);
        vb = *reinterpret_cast<const double4 *>(xb + e);
      } else {
        va = make_double4(0.0, 0.0, 0.0, 0.0);
        vb = va;
      }
    };
    int e0 = 16 * half;
    if (e0 < L) load(e0, ca, cb);
    for (; e0 < L; e0 += 32) {
      if (e0 + 32 < L) load(e0 + 32, na, nb);
      acc0 = mfma_f64(ca.x, cb.x, acc0);
      acc1 = mfma_f64(ca.y, cb.y, acc1);
      acc0 = mfma_f64(ca.z, cb.z, acc0);
      acc1 = mfma_f64(ca.w, cb.w, acc1);
      ca = na;
      cb = nb;
    }
    double *part = scratch + (half * 3 + tile) * JB * JB;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      part[(lk + 4 * q) * JB + li] = acc0[q] + acc1[q];
  } else if (tid == 6 * 64) {
    flag = 0;
  }
  __syncthreads();
  for (int idx = tid; idx < P2 * P2; idx += RT) {
    const int i = idx / P2, j = idx % P2;
    int t, a, bb;
    if (i < JB && j < JB) {
      t = 0; a = i; bb = j;
    } else if (i < JB) {
      t = 1; a = i; bb = j - JB;
    } else if (j < JB) {
      t = 1; a = j; bb = i - JB;   // G_JI = G_IJ^T
    } else {
      t = 2; a = i - JB; bb = j - JB;
    }
    G[i][j] = scratch[t * JB * JB + a * JB + bb] +
              scratch[(3 + t) * JB * JB + a * JB + bb];
  }
  __syncthreads();

  // ---- 2. convergence test; Q = I over the consumed partials -------------
  for (int idx = tid; idx < P2 * P2; idx += RT) {
    const int i = idx / P2, j = idx % P2;
    if (i < j && pair_needs_rotation(G[i][i], G[j][j], G[i][j], u.tol, u.skip))
      flag = 1;
    Q[i][j] = (i == j) ? 1.0 : 0.0;
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
  // Threads t < 256 own the 2 x 2 block (row pair t / NPAIR, column pair
  // t % NPAIR) of G; every thread owns one (row, column pair) item of Q.
  // Every element has exactly one owner, so the update is in place.
  const int rp = (tid & 255) / NPAIR, cp = tid % NPAIR;
  const int qrow = tid / NPAIR;
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
      if (tid < NPAIR * NPAIR) {
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
      {
        int p, q;
        rr_pair(rr, cp, P2, p, q);
        const double cq = cs[cp], sq = sn[cp];
        const double x = Q[qrow][p], y = Q[qrow][q];
        Q[qrow][p] = cq * x - sq * y;
        Q[qrow][q] = sq * x + cq * y;
      }
      __syncthreads();
    }
    const int rotated = flag;
    __syncthreads();  // read before the next sweep resets it
    if (!rotated) break;
  }

  // ---- 4. Xp <- Xp Q, as D = Q^T Xp^T per 16-row chunk --------------------
  // each wave takes every eighth chunk; the next chunk is loaded while the
  // current one is multiplied
  constexpr int KB = P2 / 4;
  double cur[KB], nxt[KB];
  auto load_chunk = [&](int e0, double *v) {
    const int e = e0 + li;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      const int t = 4 * kk + lk;
      const int col = t < JB ? bi * JB + t : bj * JB + t - JB;
      v[kk] = e < L ? X[(size_t)col * ld + e] : 0.0;
    }
  };
  constexpr int CSTEP = 16 * (RT / 64);
  if (16 * w < L) load_chunk(16 * w, cur);
  for (int e0 = 16 * w; e0 < L; e0 += CSTEP) {
    if (e0 + CSTEP < L) load_chunk(e0 + CSTEP, nxt);
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
        X[(size_t)(bi * JB + jo) * ld + e] = d0[q];
        X[(size_t)(bj * JB + jo) * ld + e] = d1[q];
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
  hipLaunchKernelGGL(k_jacobi_round, dim3(max_pairs, b.B), dim3(RT), 0, st, b,
                     s, u, round);
}

}  // namespace hmps
