// Internal interface between the host orchestration (hmps.cpp) and the
// gfx950 kernels (update.hip, jacobi.hip, observe.hip).  Not part of the public ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace hmps {

// Jacobi column-block width of the large-matrix SVD path; a block pair is
// 2 JB vectors.
constexpr int JB = 16;
// Stride between consecutive vectors of the L x N vector matrix: L rounded
// up to a multiple of 16, so that every 16-row chunk of a vector lies
// inside it (the padding rows are zero) and the Jacobi kernels load and
// store whole chunks without bounds tests.
__host__ __device__ inline int vector_stride(int len) {
  return (len + 15) & ~15;
}

// Number of column blocks, rounded up to an even count.
__host__ __device__ constexpr int n_blocks_even(int nvec, int jb) {
  return (nvec + jb - 1) / jb + (((nvec + jb - 1) / jb) & 1);
}
// Wide rounds: blocks of JBW vectors (pairs of 64) for the chains with at
// least W32_MIN_N vectors on the FP64 blocked paths -- half the rounds per
// sweep, so half the passes over the vectors (jacobi.hip).
constexpr int JBW = 32;
constexpr int W32_MIN_N = 512;
// Vectors of the blocked paths padded with zero vectors to an even number
// of blocks of either width.
__host__ __device__ constexpr int npad_vectors(int nvec) {
  return n_blocks_even(nvec, JBW) * JBW;
}
// Largest m * n_even (doubles) handled by the single-workgroup SVD whose
// matrix lives entirely in LDS.
constexpr int SMALL_LDS = 18432;
// Relative floor below which a singular value is numerically zero (it is
// always discarded: its singular vectors are noise).
constexpr double SIGMA_FLOOR = 1e-13;
// Relative gap below which neighbouring singular values tie.
constexpr double TIE_TOL = 1e-8;

// Workgroups per chain summing ||theta'||^2.
constexpr int NORM_SPLIT = 16;

// Householder QR preconditioning of the blocked Jacobi SVD: panel width,
// and the longest vectors whose 16-column panel one workgroup of the panel
// kernel holds in registers (three rows per thread: chi <= 512).
constexpr int QB = 16;
constexpr int QR_MAX_L = 1536;

// The per-chain path of an update's SVD: the in-LDS Jacobi for L * N <=
// small_max, else the blocked rounds -- on R^T of theta' = Q R when the
// preconditioning is on and the vectors fit a QR panel, else on theta'
// itself.  The choice depends on the chain's own dimensions only, so a
// chain takes the same path alone and in a batch.
__host__ __device__ inline bool small_path(int L, int N, size_t small_max) {
  return (size_t)L * N <= small_max;
}
__host__ __device__ inline bool qr_path(int L, int N, size_t small_max,
                                        int precond) {
  return precond && !small_path(L, N, small_max) && L <= QR_MAX_L;
}
// Paths of a chain's SVD.
//   PATH_QR   Jacobi rounds on R^T of theta' = Q R (precond >= 1).
//   PATH_QR2  (precond >= 2, FP64) a second QR, R^T = Q2 R2, and the rounds
//             on R2^T: its columns are closer still to orthogonal, so fewer
//             sweeps are needed.  R2^T = (Q^T U) Sigma (Q2^T V)^T, so the
//             converged vectors are the left singular vectors in the basis
//             of Q; both factors then follow by projection (see update.hip).
//   PATH_RR   (mixed precision, on chains that take the QR) Jacobi rounds
//             on an FP32 copy of R^T, then the rr_vectors largest of its
//             converged vectors, orthonormalised in FP64, give the basis W
//             of a Rayleigh-Ritz step: FP64 rounds on the columns of
//             theta' W.
//   PATH_RR2  (mixed precision, precond >= 2) the FP32 rounds on R2^T: their
//             vectors approximate the left singular vectors u~ in the basis
//             of Q, and the FP64 rounds run on the columns of R^T W (whose
//             converged vectors are sigma_j w_j, as on the QR path).
enum {
  PATH_SMALL = 0, PATH_PLAIN = 1, PATH_QR = 2, PATH_RR = 3, PATH_QR2 = 4,
  PATH_RR2 = 5
};
// The second QR pays from this many vectors on: below it the sweeps it
// saves cost less than its launches (one chain of the 2x3 ladder, N <= 96,
// runs 12% faster per sample with one QR; the chi = 256 gate workload, N =
// 768, 16% faster with two).
constexpr int QR2_MIN_N = 160;
__host__ __device__ inline int svd_path(int L, int N, size_t small_max,
                                        int precond, int mixed) {
  if (small_path(L, N, small_max)) return PATH_SMALL;
  if (qr_path(L, N, small_max, precond)) {
    const bool two = precond >= 2 && N >= QR2_MIN_N;
    if (mixed) return two ? PATH_RR2 : PATH_RR;
    return two ? PATH_QR2 : PATH_QR;
  }
  return PATH_PLAIN;
}
// Block width of a chain's Jacobi rounds: JBW for the FP64 blocked paths
// from wide_min vectors on (wide_min >= W32_MIN_N; 0: never), JB
// otherwise.  The host sets wide_min for the whole update from the batch
// size (the width rule).
__host__ __device__ inline int round_width(int path, int nvec, int wide_min) {
  return (wide_min > 0 && nvec >= wide_min &&
          (path == PATH_PLAIN || path == PATH_QR || path == PATH_QR2))
             ? JBW
             : JB;
}
// The paths whose first step is theta' = Q R, those with a second QR, and
// the mixed-precision paths.
__host__ __device__ inline bool path_has_qr(int path) {
  return path >= PATH_QR;
}
__host__ __device__ inline bool path_has_qr2(int path) {
  return path == PATH_QR2 || path == PATH_RR2;
}
__host__ __device__ inline bool path_is_rr(int path) {
  return path == PATH_RR || path == PATH_RR2;
}
// Largest Ritz basis: chi_max plus 64 (at least 64 vectors beyond the
// cut), rounded to 32, at most N.  The basis holds only the vectors the
// FP32 stage resolves (squared norm above skip32 times the largest, which
// it rotates against every other): the chain's size is rrk <= this.
__host__ __device__ inline int rr_vectors(int N, int chi_max) {
  const int k = (chi_max + 64 + 31) / 32 * 32;
  return k < N ? k : N;
}

// Device view of one batch of chains.  Site p of chain c is the row-major
// tensor T[s][l][r] (s < 3, l < chi[c][p], r < chi[c][p+1]) stored at
// sites + (c * nsites + p) * site_cap.
struct Batch {
  double *sites;
  int32_t *chi;       // [B][nsites + 1]
  int nsites;
  size_t site_cap;    // doubles per site slot
  int B;
};

// Per-chain scratch of one two-site update.  theta' (m x n) is stored
// column-major twice: TH keeps it, X is rotated by the Jacobi sweeps
// (n_pad >= n columns, the padding columns are zero).
struct UpdScratch {
  double *TH;         // [B][th_stride]
  double *X;          // [B][th_stride]
  double *Y;          // [B][th_stride] R^T of the QR path (the vectors)
  double *qrT;        // [B][2][qr_panels][QB * QB] compact-WY factors of
                      // every panel of both QR stages
  int qr_panels;      // panels per stage: ceil(3 chi_cap / QB)
  double *Z;          // [B][th_stride] R2^T of PATH_QR2 (its vectors),
                      // Gram of the mixed path's basis, Grams of the
                      // write-back
  size_t th_stride;
  double *sig2;       // [B][n_cap] squared column norms after convergence
  int32_t *perm;      // [B][n_cap] kept columns, largest singular value first
  double *sig;        // [B][n_cap] kept singular values (sorted)
  int n_cap;
  int32_t *knew;      // [B]
  double *fac;        // [B] 1/||kept||
  double *norm2;      // [B][NORM_SPLIT] partial sums of ||theta'||^2 (FP64)
  double *logw;       // [B]
  double *discarded;  // [B] accumulated relative discarded weight
  int32_t *rot_cur;   // [B] rotations in the current sweep
  int32_t *done;      // [B] Jacobi converged
  int32_t *err;       // [B] nonzero: numerical failure
  int32_t *sweeps;    // [B] Jacobi sweeps done by the in-LDS path
  int32_t *rrk;       // [B] Ritz basis size of the mixed path (<= rr_vectors)
  double *rrG;        // [B][rrG_stride] Gram of the basis on PATH_RR2
  size_t rrG_stride;  // doubles per chain: round16(k')^2 for the largest k'
};

// T factor of panel p of QR stage `stage` of chain c.
__host__ __device__ inline double *qrT_slot(const UpdScratch &s, int c,
                                            int stage, int p) {
  return s.qrT + ((size_t)(2 * c + stage) * s.qr_panels + p) * QB * QB;
}

struct UpdParams {
  int k;              // left site of the update
  const double *gate; // 81 doubles on the device (row-major (s1 s2),(t1 t2))
  int is_gate;        // accumulate ln ||theta'||^2 into logw
  int right;          // absorb singular values to the right
  int chi_max;
  double cutoff;
  double tol;         // Jacobi relative orthogonality tolerance
  double tol32;       // the same for the FP32 rounds of the mixed path
  int max_sweeps;
  int mixed;          // FP32 contraction
  int inner_sweeps;   // cap on the inner Jacobi sweeps of a block pair
  double skip;        // relative squared norm below which a vector is zero
  double skip32;      // the same for the FP32 rounds
  int cross_inner;    // inner rotations across the two blocks only (rounds > 0)
  int wide_min;       // wide (32-vector) blocks from this many vectors on
                      // (0: none)
  int precond;        // QR preconditioning of the blocked path: 0 none,
                      // 1 one QR, 2 two (FP64)
  size_t small_max;   // largest L * N of the in-LDS SVD path
  int zero_ok;        // a zero theta' keeps no vector instead of failing
                      // (the charge blocks of a U(1) update)
};

// ---- launchers (update.hip, jacobi.hip, observe.hip) -----------------------------------------
void launch_theta(const Batch &b, const UpdScratch &s, const UpdParams &u,
                  int max_chiL, int max_chiR, hipStream_t st);
void launch_pad(const Batch &b, const UpdScratch &s, const UpdParams &u,
                hipStream_t st);
void launch_theta_norm(const Batch &b, const UpdScratch &s,
                       const UpdParams &u, hipStream_t st);
void launch_jacobi_small(const Batch &b, const UpdScratch &s,
                         const UpdParams &u, hipStream_t st);
void launch_jacobi_sweep_begin(const UpdScratch &s, int B, int sweep,
                               hipStream_t st);
// max_len: the longest vector over the chains on these (16-wide FP64)
// rounds; it and the workgroup count choose the register budget
void launch_jacobi_round(const Batch &b, const UpdScratch &s,
                         const UpdParams &u, int round, int max_pairs,
                         int max_len, hipStream_t st);
void launch_jacobi_round32(const Batch &b, const UpdScratch &s,
                           const UpdParams &u, int round, int max_pairs,
                           hipStream_t st);
// Round `round` of the wide (JBW) blocks of the chains that take them.
// chains c0 .. c0 + nc - 1 of the batch
void launch_jacobi_round_wide(const Batch &b, const UpdScratch &s,
                              const UpdParams &u, int round, int max_pairs,
                              int c0, int nc, hipStream_t st);
void launch_truncate(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     hipStream_t st);
// qr2_panels: panels of the largest PATH_QR2 chain (0: none)
void launch_writeback(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int max_L, int max_N, int max_k, int qr2_panels,
                      hipStream_t st);
// QR preconditioning (qr.hip).  Stage 0: theta' = Q R on every chain
// whose path starts with a QR (the vector matrix in X), R^T into Y.
// Stage 1: R^T = Q2 R2 on the PATH_QR2 chains (in Y), R2^T into Z.  Panel
// p, the update of its trailing columns (max_tiles 16-column tiles), and
// the transposed factor into the vector buffer.  Each launch covers the
// chains cb .. cb + nc - 1 of the batch.
void launch_qr_panel(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     int stage, int p, int max_rows, int cb, int nc,
                     hipStream_t st);
void launch_qr_update(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int stage, int p, int max_tiles, int cb, int nc,
                      hipStream_t st);
void launch_qr_to_vectors(const Batch &b, const UpdScratch &s,
                          const UpdParams &u, int stage, int max_N, int cb,
                          int nc, hipStream_t st);
// The first QR's block reflector of panel p applied to the k unit vectors
// held in TH of every PATH_QR2 chain (max_tiles 16-column tiles): panels
// from last to first give Q u~ (the left factor on the two-QR path).
void launch_qr_apply(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     int p, int max_tiles, hipStream_t st);
// Mixed path (rr.hip): R^T to FP32 before the FP32 rounds; after them the
// FP64 Ritz basis W and theta' W into X for the FP64 rounds.
void launch_rr_to32(const Batch &b, const UpdScratch &s, const UpdParams &u,
                    hipStream_t st);
void launch_rr_stage2(const Batch &b, const UpdScratch &s, const UpdParams &u,
                      int max_N, int max_L, hipStream_t st);

// U(1) updates (u1.hip).  Each charge block of an update is a chain of
// a second batch (two sites, the block's theta' placed in its vector
// layout).  Block table, U1_BLK ints per block:
//   [0] index of the block's chain in the chain list of the pass,
//   [1] charge, [2] chi_l', [3] chi_r' (block theta' is 3 chi_l' x 3 chi_r',
//   rows (s1, a'), columns (s2, c'), zero outside the pieces below),
//   [4 + s] first index a of the left bond whose row (s, a) falls in the
//   block, [7 + s] their count, [10 + s], [13 + s] the same for the
//   columns (s, c) and the right bond.
// Chain list, U1_CH ints per chain: [0] chain, [1] first block, [2] blocks.
constexpr int U1_BLK = 16;
constexpr int U1_CH = 4;
struct U1Args {
  const int32_t *blk;   // [blocks][U1_BLK]
  const int32_t *chains;  // [chains of the pass][U1_CH]
  int n_chains;           // chains of the pass
  int n_blocks;           // blocks of the pass
  int k;                  // left site of the update
  int right;              // the singular values go right
  // the block batch: its dimensions and flags (set by k_u1_gather), its
  // sites (two per block), TH and X, sig, knew
  int32_t *bchi, *berr;
  double *bdisc, *blogw;
  double *bsites;
  size_t bsite_cap;
  double *bTH, *bX;
  size_t bstride;
  const double *bsig;
  const int32_t *bknew;
  int bn_cap;
  // merge results
  int32_t *kv;          // [blocks] vectors of each block kept
  double *scale;        // [blocks] norm factor of the singular-value side
  int32_t *jmap;        // [chain][jstride] new bond index -> block << 16 | i
  int jstride;
};
// theta' blocks of every block of the pass (from the chains' TH), and the
// block batch's dimensions {chi_l', 1, chi_r'} with its flags cleared
void launch_u1_gather(const Batch &b, const UpdScratch &s, const U1Args &a,
                      hipStream_t st);
// the kept set over all blocks of each chain (rule of k_truncate), the
// chain's logw, discarded weight, kept spectrum and new bond dimension
void launch_u1_merge(const Batch &b, const UpdScratch &s, const UpdParams &u,
                     const U1Args &a, hipStream_t st);
// the chains' new site tensors k and k+1 from the blocks' factors
void launch_u1_scatter(const Batch &b, const U1Args &a, int max_chiL,
                       int max_chiR, int max_k, hipStream_t st);

struct MeasureArgs {
  const int32_t *bond_p, *bond_q;  // [n_bonds] MPS positions, p < q
  const double *bond_J;
  int n_bonds;
  const int32_t *is_ancilla;       // [nsites]
  double *envs;                    // [B][nsites+1][chi_cap^2] left envs
  double *wsz;                     // [B][nsites] <S^z> per site
  double *bond_scratch;            // [B][slots][4 chi_cap^2]
  int slots;
  size_t chi2;                     // chi_cap^2
  double *norm;                    // [B]
  double *bond_ss;                 // [B][n_bonds]
};
void launch_measure_envs(const Batch &b, const MeasureArgs &m,
                         hipStream_t st);
void launch_measure_bonds(const Batch &b, const MeasureArgs &m, int b0,
                          int nb, hipStream_t st);
void launch_measure_finish(const Batch &b, const MeasureArgs &m,
                           double *energy, double *qn, hipStream_t st);
// bond_ss[c][i] /= norm[c] for i < n_bonds (correlators of arbitrary pairs)
void launch_measure_scale(const Batch &b, const MeasureArgs &m,
                          hipStream_t st);
// site pairs measured per pass by hmps_measure_pairs
constexpr int PAIR_CHUNK = 256;

// Per-bond sample moments (observe.hip): mom is [B][n_bonds + 1][3]
// (count, mean, sum of squared deviations; the energy is entry n_bonds),
// out is [n_bonds + 1][3] over all chains.
void launch_moments_add(const double *bond_ss, const double *energy,
                        double *mom, int B, int n_bonds, hipStream_t st);
void launch_moments_reduce(const double *mom, double *out, int B,
                           int n_bonds, hipStream_t st);
// p[0 .. n) = v (a kernel, so that a captured stream records no memset)
void launch_fill(double *p, size_t n, double v, hipStream_t st);

struct CollapseArgs {
  const int32_t *is_cluster;  // [nsites]
  const int32_t *env_index;   // [nsites] index among env sites or -1
  int n_env;
  double *scratch;            // [B][8 chi_cap^2]
  size_t chi2;
  uint8_t *outcomes;          // [B][n_env]
  int32_t *near;              // [B] draws within 1e-12 of a threshold
  int basis;
  uint64_t seed;
  uint64_t chain0;            // global id of chain 0 of the batch
  int64_t sample;
};
void launch_collapse(const Batch &b, const CollapseArgs &a, hipStream_t st);

struct InitArgs {
  const int32_t *is_cluster;   // [nsites]
  const int32_t *is_ancilla;   // [nsites]
  const int32_t *env_index;    // [nsites]
  const uint8_t *labels;       // [B][n_env]
  int n_env;
  int basis;
};
void launch_init(const Batch &b, const InitArgs &a, double *logw,
                 hipStream_t st);

}  // namespace hmps
