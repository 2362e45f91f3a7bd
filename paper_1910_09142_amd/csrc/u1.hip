// gfx950 kernels of a U(1)-symmetric two-site update (Chen & Stoudenmire,
// arXiv:1910.09142, Exploiting Conserved Quantum Numbers subsection: each
// imaginary-time evolution conserves the total charge Q = sum_phys S^z -
// sum_anc S^z, so the MPS tensors are block sparse).
//
// Every bond index carries a charge, the Q of the sites left of it.  Row
// (s1, a) of theta' belongs to charge q_k(a) + sign_k S^z(s1) of the new
// bond and column (s2, c) to q_{k+2}(c) - sign_{k+1} S^z(s2) (sign -1 at a
// position that holds an ancilla): theta' vanishes between rows and columns
// of different charges, so it is the direct sum of one block per charge,
// and its SVD is the union of the blocks' SVDs.  The host lists the
// blocks; each is decomposed as a chain of a second batch (the blocked or
// in-LDS Jacobi SVD of the dense path).  Then
//   k_u1_gather   each block's theta' from the chain's theta' (TH), in the
//                 block batch's vector layout
//   k_u1_merge    the singular values of all blocks of a chain sorted
//                 together and truncated by the dense rule: the kept set,
//                 the new bond in block order (ascending charge), the
//                 chain's log-weight, discarded weight and spectrum
//   k_u1_scatter  the chain's new site tensors from the blocks' factors,
//                 zero outside the blocks
#include <algorithm>

#include "device_common.h"
#include "truncate_rule.h"

namespace hmps {
namespace {
using namespace dev;

// blocks of one chain that k_u1_merge holds in LDS
constexpr int U1_MAXB = 512;
// singular values k_u1_merge sorts (3 chi_cap <= 1920)
constexpr int U1_MAXV = 2048;

__global__ void __launch_bounds__(NT)
    k_u1_gather(Batch b, UpdScratch s, U1Args a) {
  const int v = blockIdx.y;
  const int32_t *bt = a.blk + (size_t)v * U1_BLK;
  const int c = a.chains[(size_t)bt[0] * U1_CH];
  const int32_t *chi = chi_row(b, c);
  const int chiL = chi[a.k], chiR = chi[a.k + 2];
  const int m = 3 * chiL, n = 3 * chiR;
  const bool trans = n > m;
  const int ld = vec_ld(trans ? n : m);
  const double *TH = s.TH + (size_t)c * s.th_stride;
  // the block as a chain: theta'_q of 3 cl x 3 cr, rows (s1, a') s-major,
  // stored as the min(m', n') vectors of length max(m', n') (interleaved
  // vector index 3 (bond index) + s), stride vec_ld, zero padding rows
  const int cl = bt[2], cr = bt[3];
  const int mp = 3 * cl, np = 3 * cr;
  const bool tp = np > mp;
  const int Lp = tp ? np : mp, Np = tp ? mp : np;
  const int ldp = vec_ld(Lp);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.bchi[3 * v] = cl;
    a.bchi[3 * v + 1] = 1;
    a.bchi[3 * v + 2] = cr;
    a.berr[v] = 0;
    a.bdisc[v] = 0.0;
    a.blogw[v] = 0.0;
  }
  double *dTH = a.bTH + (size_t)v * a.bstride;
  double *dX = a.bX + (size_t)v * a.bstride;
  const size_t total = (size_t)ldp * Np;
  for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < total;
       e += (size_t)gridDim.x * NT) {
    const int vec = (int)(e / ldp), l = (int)(e % ldp);
    double val = 0.0;
    if (l < Lp) {
      int s1, ap, s2, cp;
      if (!tp) {  // the vectors are the columns (s2, c')
        s2 = vec % 3;
        cp = vec / 3;
        s1 = l / cl;
        ap = l - s1 * cl;
      } else {    // the vectors are the rows (s1, a')
        s1 = vec % 3;
        ap = vec / 3;
        s2 = l / cr;
        cp = l - s2 * cr;
      }
      if (ap < bt[7 + s1] && cp < bt[13 + s2]) {
        const int ar = bt[4 + s1] + ap, cc = bt[10 + s2] + cp;
        const size_t off =
            trans ? (size_t)(3 * ar + s1) * ld + (size_t)s2 * chiR + cc
                  : (size_t)(3 * cc + s2) * ld + (size_t)s1 * chiL + ar;
        val = TH[off];
      }
    }
    dTH[e] = val;
    dX[e] = val;
  }
}

// One workgroup per chain of the pass.
__global__ void __launch_bounds__(NT)
    k_u1_merge(Batch b, UpdScratch s, UpdParams u, U1Args a) {
  const int32_t *ch = a.chains + (size_t)blockIdx.x * U1_CH;
  const int c = ch[0], v0 = ch[1], nv = ch[2];
  __shared__ double key[U1_MAXV];
  __shared__ int idx[U1_MAXV];
  __shared__ int start[U1_MAXB + 1];
  __shared__ int kcount[U1_MAXB];
  __shared__ int kk_s, bad_s;
  const int tid = threadIdx.x;
  if (tid == 0) {
    // candidates of block v: its kept values (all above the block's own
    // numerical floor), largest first
    int n = 0;
    bad_s = nv > U1_MAXB;
    for (int v = 0; v < nv && !bad_s; ++v) {
      start[v] = n;
      n += a.bknew[v0 + v];
    }
    if (!bad_s) start[nv] = n;
    if (n > U1_MAXV) bad_s = 1;
  }
  __syncthreads();
  if (bad_s) {
    if (tid == 0) s.err[c] = 3;
    return;
  }
  const int N = start[nv];
  int N2 = 1;
  while (N2 < N) N2 <<= 1;
  for (int j = tid; j < N2; j += NT) {
    key[j] = -1.0;
    idx[j] = 0x7fffffff;
  }
  for (int v = tid; v < nv; v += NT) kcount[v] = 0;
  __syncthreads();
  for (int v = 0; v < nv; ++v) {
    const int kb = a.bknew[v0 + v];
    const double *sg = a.bsig + (size_t)(v0 + v) * a.bn_cap;
    for (int i = tid; i < kb; i += NT) {
      key[start[v] + i] = sg[i];
      idx[start[v] + i] = (v << 16) | i;
    }
  }
  __syncthreads();
  // bitonic sort, descending; equal values by (block, index)
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
  __shared__ double kept_s;
  if (tid == 0) {
    double n2 = 0.0;  // ||theta'||^2 in FP64, summed from theta'
    if (u.is_gate)
      for (int x = 0; x < NORM_SPLIT; ++x)
        n2 += s.norm2[(size_t)c * NORM_SPLIT + x];
    const TruncResult tr =
        truncation_rule(key, N, false, 0.0, u.chi_max, u.cutoff);
    const double total = tr.total, kept = tr.kept;
    if (N == 0 || !(total > 0.0) || !isfinite(total) || !(kept > 0.0))
      s.err[c] = 2;
    if (u.is_gate) s.logw[c] += log(n2);
    if (total > 0.0) s.discarded[c] += (total - kept) / total;
    s.knew[c] = tr.k;
    kk_s = tr.k;
    kept_s = kept;
  }
  __syncthreads();
  const int K = kk_s;
  // within a block the kept values are its first kcount[v] (its values are
  // in descending order and ties go by index)
  for (int j = tid; j < K; j += NT) {
    s.sig[(size_t)c * s.n_cap + j] = key[j];
    atomicAdd(&kcount[idx[j] >> 16], 1);
  }
  __syncthreads();
  if (tid == 0) {
    int off = 0;
    for (int v = 0; v < nv; ++v) {
      start[v] = off;  // first new bond index of block v
      off += kcount[v];
    }
  }
  __syncthreads();
  for (int j = tid; j < K; j += NT) {
    const int v = idx[j] >> 16, i = idx[j] & 0xffff;
    a.jmap[(size_t)c * a.jstride + start[v] + i] = idx[j];
  }
  // the block's singular-value side carries sigma / ||its own kept||: the
  // chain's carries sigma / ||all kept||
  const double inv_kept = 1.0 / sqrt(kept_s);
  for (int v = tid; v < nv; v += NT) {
    const int kb = a.bknew[v0 + v];
    const double *sg = a.bsig + (size_t)(v0 + v) * a.bn_cap;
    double kv = 0.0;
    for (int i = kb - 1; i >= 0; --i) kv += sg[i] * sg[i];
    a.kv[v0 + v] = kcount[v];
    a.scale[v0 + v] = sqrt(kv) * inv_kept;
  }
  // the new bond dimension is published last
  __syncthreads();
  if (tid == 0) b.chi[(size_t)c * (b.nsites + 1) + u.k + 1] = K;
}

// grid (x, 2 sites, chains of the pass)
__global__ void __launch_bounds__(NT) k_u1_scatter(Batch b, U1Args a) {
  const int32_t *ch = a.chains + (size_t)blockIdx.z * U1_CH;
  const int c = ch[0], v0 = ch[1];
  const int32_t *chi = chi_row(b, c);
  const int chiL = chi[a.k], K = chi[a.k + 1], chiR = chi[a.k + 2];
  const int site = blockIdx.y;
  const int32_t *jm = a.jmap + (size_t)c * a.jstride;
  if (site == 0) {
    // T_k[s1][a][j]: the block's left factor where row (s1, a) is in it
    double *T = site_ptr(b, c, a.k);
    const int total = 3 * chiL * K;
    for (int e = blockIdx.x * NT + threadIdx.x; e < total;
         e += gridDim.x * NT) {
      const int s1 = e / (chiL * K), r = e - s1 * chiL * K;
      const int ar = r / K, j = r - ar * K;
      const int v = v0 + (jm[j] >> 16), i = jm[j] & 0xffff;
      const int32_t *bt = a.blk + (size_t)v * U1_BLK;
      const int ap = ar - bt[4 + s1];
      double val = 0.0;
      if (ap >= 0 && ap < bt[7 + s1]) {
        const int kb = a.bknew[v];
        const double *B0 = a.bsites + (size_t)(2 * v) * a.bsite_cap;
        val = B0[((size_t)s1 * bt[2] + ap) * kb + i];
        if (!a.right) val *= a.scale[v];
      }
      T[e] = val;
    }
  } else {
    // T_{k+1}[s2][j][c]
    double *T = site_ptr(b, c, a.k + 1);
    const int total = 3 * K * chiR;
    for (int e = blockIdx.x * NT + threadIdx.x; e < total;
         e += gridDim.x * NT) {
      const int s2 = e / (K * chiR), r = e - s2 * K * chiR;
      const int j = r / chiR, cc = r - j * chiR;
      const int v = v0 + (jm[j] >> 16), i = jm[j] & 0xffff;
      const int32_t *bt = a.blk + (size_t)v * U1_BLK;
      const int cp = cc - bt[10 + s2];
      double val = 0.0;
      if (cp >= 0 && cp < bt[13 + s2]) {
        const int kb = a.bknew[v];
        const double *B1 = a.bsites + (size_t)(2 * v + 1) * a.bsite_cap;
        val = B1[((size_t)s2 * kb + i) * bt[3] + cp];
        if (a.right) val *= a.scale[v];
      }
      T[e] = val;
    }
  }
}

}  // namespace

void launch_u1_gather(const Batch &b, const UpdScratch &s, const U1Args &a,
                      hipStream_t st) {
  if (a.n_blocks <= 0) return;
  hipLaunchKernelGGL(k_u1_gather, dim3(16, a.n_blocks), dim3(NT), 0, st, b, s,
                     a);
}

void launch_u1_merge(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     const U1Args &a, hipStream_t st) {
  if (a.n_chains <= 0) return;
  hipLaunchKernelGGL(k_u1_merge, dim3(a.n_chains), dim3(NT), 0, st, b, s, u,
                     a);
}

void launch_u1_scatter(const Batch &b, const U1Args &a, int max_chiL,
                       int max_chiR, int max_k, hipStream_t st) {
  if (a.n_chains <= 0) return;
  const long most = 3L * std::max(max_chiL, max_chiR) * max_k;
  const int gx = (int)std::min<long>(64, std::max<long>(1, (most + NT - 1) / NT));
  hipLaunchKernelGGL(k_u1_scatter, dim3(gx, 2, a.n_chains), dim3(NT), 0, st,
                     b, a);
}

}  // namespace hmps
