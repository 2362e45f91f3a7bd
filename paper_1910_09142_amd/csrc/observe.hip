// gfx950 kernels of steps 1, 3 and 4 of the hybrid Markov chain
// (Chen & Stoudenmire, arXiv:1910.09142, Hybrid METTS-Ancilla subsection):
// initial states, measurement by transfer matrices, sequential projective
// collapse of the environment with Philox4x64-10 draws.
#include <algorithm>

#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

// Product-basis vectors: row t is the state of outcome t (eigenvalue
// +1, 0, -1) written in the S^z basis; basis 0 = S^z, 1 = S^x.
__constant__ double c_basis[2][3][3] = {
    {{1.0, 0.0, 0.0}, {0.0, 1.0, 0.0}, {0.0, 0.0, 1.0}},
    {{0.5, 0.70710678118654752440, 0.5},
     {0.70710678118654752440, 0.0, -0.70710678118654752440},
     {0.5, -0.70710678118654752440, 0.5}}};

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

// Correlators of arbitrary site pairs: divide by the norm <psi|psi>.
__global__ void k_measure_scale(Batch b, MeasureArgs ma) {
  const int c = blockIdx.y;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= b.B || i >= ma.n_bonds) return;
  ma.bond_ss[(size_t)c * ma.n_bonds + i] /= ma.norm[c];
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
// Per-bond sample moments (the variance study of the estimators, Section
// Entanglement and Cost of Hybrid States): for every chain c and every
// bond b, and for the energy as entry n_bonds, a running count, mean and
// sum of squared deviations, updated in the order of the measurements
// (Welford's update, FP64).  One thread per (chain, entry); no atomics,
// so the result does not depend on the launch.
// =====================================================================
__global__ void k_moments_add(const double *bond_ss, const double *energy,
                              double *mom, int B, int nb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * (nb + 1)) return;
  const int c = t / (nb + 1), e = t % (nb + 1);
  const double x = e < nb ? bond_ss[(size_t)c * nb + e] : energy[c];
  double *m = mom + (size_t)t * 3;
  const double n = m[0] + 1.0;
  const double d = x - m[1];
  const double mean = m[1] + d / n;
  m[0] = n;
  m[1] = mean;
  m[2] += d * (x - mean);
}

// The chains combined in chain order (Chan, Golub and LeVeque's pairwise
// update of count, mean and squared deviations): one thread per entry.
__global__ void k_moments_reduce(const double *mom, double *out, int B,
                                 int nb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e > nb) return;
  double n = 0.0, mean = 0.0, m2 = 0.0;
  for (int c = 0; c < B; ++c) {
    const double *m = mom + ((size_t)c * (nb + 1) + e) * 3;
    const double nc = m[0];
    if (nc == 0.0) continue;
    const double tot = n + nc;
    const double d = m[1] - mean;
    mean += d * (nc / tot);
    m2 += m[2] + d * d * (n * nc / tot);
    n = tot;
  }
  out[3 * e] = n;
  out[3 * e + 1] = mean;
  out[3 * e + 2] = m2;
}

__global__ void k_fill(double *p, size_t n, double v) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (size_t)gridDim.x * blockDim.x)
    p[i] = v;
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
        // counter (global chain id, sample, MPS position, purpose 1)
        const uint64_t x = philox_word0(a.chain0 + (uint64_t)c,
                                        (uint64_t)a.sample,
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

void launch_measure_scale(const Batch &b, const MeasureArgs &m,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_measure_scale, dim3((m.n_bonds + NT - 1) / NT, b.B),
                     dim3(NT), 0, st, b, m);
}

void launch_moments_add(const double *bond_ss, const double *energy,
                        double *mom, int B, int n_bonds, hipStream_t st) {
  const int n = B * (n_bonds + 1);
  hipLaunchKernelGGL(k_moments_add, dim3((n + 255) / 256), dim3(256), 0, st,
                     bond_ss, energy, mom, B, n_bonds);
}

void launch_moments_reduce(const double *mom, double *out, int B,
                           int n_bonds, hipStream_t st) {
  hipLaunchKernelGGL(k_moments_reduce, dim3((n_bonds + 256) / 256),
                     dim3(256), 0, st, mom, out, B, n_bonds);
}

void launch_fill(double *p, size_t n, double v, hipStream_t st) {
  if (n == 0) return;
  const size_t blocks = std::min<size_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, st, p, n,
                     v);
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
