// Blocked one-sided Jacobi SVD round on gfx950 matrix cores
// (the SVD that restores the MPS form after every two-site gate;
// Chen & Stoudenmire, arXiv:1910.09142, Results section).
//
// The N vectors (columns of the L x N vector matrix X -- or, on the QR
// paths, of the N x N matrix R^T in Y or R2^T in Z -- stride ld = L
// rounded up to 16, column-major) are split into NB (even) blocks of
// JB = 16 vectors.  A sweep has NB-1 rounds; in a round the blocks are
// paired by the circle method and one workgroup of eight wavefronts handles
// one block pair of one chain:
//   1. Gram matrix G = Xp^T Xp of the 2 JB vectors: its three upper 16 x 16
//      tiles by FP64 MFMA from coalesced 32-byte loads of four rows, the
//      next chunk in flight while the current one is multiplied; the eight
//      wavefront partials are summed in LDS in a fixed order;
//   2. if every pair the round rotates is orthogonal to tol sqrt(G_ii G_jj),
//      record the squared norms and stop;
//   3. one cyclic two-sided Jacobi sweep on the upper triangle of G in LDS,
//      rotations accumulated in Q, one barrier per rotation round (all
//      pairs in the first round of a sweep, the pairs across the two blocks
//      afterwards, with the second block relabelled after every rotation
//      round so that their LDS offsets stay fixed);
//   4. Xp <- Xp Q (FP64 MFMA, 16-row chunks over eight wavefronts, loads
//      of the next chunk in flight, coalesced stores).
#include "device_common.h"

namespace hmps {
namespace {
using namespace dev;

constexpr int RT = 512;  // threads of the round kernel (8 wavefronts)

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
// inner product g of two vectors with squared norms a, b: the smaller root
// t = tan(phi) of tan(2 phi) = 2g / (b - a), then c = 1 / sqrt(1 + t^2),
// s = c t.  The square root and the reciprocal behind t come from the
// hardware estimates refined by Newton steps (t only has to be close to
// the optimal angle); c is refined to rounding accuracy, so c^2 + s^2 = 1
// holds to rounding for the t actually used.
__device__ __forceinline__ double rsqrt_newton(double x, int steps) {
  double y = __builtin_amdgcn_rsq(x);
  for (int i = 0; i < steps; ++i) {
    const double e = fma(-x * y, y, 1.0);  // 1 - x y^2
    y = fma(0.5 * y, e, y);
  }
  return y;
}
__device__ __forceinline__ bool pair_rotation(double a, double b, double g,
                                              double tol, double skip,
                                              double &c, double &s) {
  if (!pair_needs_rotation(a, b, g, tol, skip)) return false;
  const double d = b - a;
  const double x = fma(d, d, 4.0 * g * g);
  const double r = x * rsqrt_newton(x, 2);  // sqrt(d^2 + 4 g^2)
  const double den = fabs(d) + r;
  double inv = __builtin_amdgcn_rcp(den);
  inv = fma(inv, fma(-den, inv, 1.0), inv);
  inv = fma(inv, fma(-den, inv, 1.0), inv);
  const double t = copysign(1.0, d) * (2.0 * g * inv);
  c = rsqrt_newton(fma(t, t, 1.0), 3);
  s = c * t;
  return true;
}

// Slot of index x in round r of the circle-method pairing over n indices
// (the inverse of rr_pair): pair i, and the partner of x in that pair.
__device__ __forceinline__ void rr_slot(int r, int x, int n, int &i,
                                        int &partner) {
  const int mod = n - 1;
  if (x == n - 1) {
    i = 0;
    partner = r;
    return;
  }
  if (x == r) {
    i = 0;
    partner = n - 1;
    return;
  }
  int d = x - r;
  if (d < 0) d += mod;  // x = (r + d) mod (n - 1)
  if (d <= (mod - 1) / 2) {
    i = d;
    partner = r - d < 0 ? r - d + mod : r - d;
  } else {
    i = mod - d;
    partner = r + i >= mod ? r + i - mod : r + i;
  }
}

// Inner (in-LDS) rotation schedule of a block pair of 2 NPAIR vectors:
// the circle method over all 2 NPAIR - 1 rounds (every pair), or, with
// `cross`, NPAIR rounds of the pairs (i, NPAIR + (i + rr) mod NPAIR) that
// join one vector of each block.
__device__ __forceinline__ void inner_pair(bool cross, int rr, int i, int n,
                                           int &p, int &q) {
  if (cross) {
    p = i;
    q = n / 2 + ((i + rr) & (n / 2 - 1));
  } else {
    rr_pair(rr, i, n, p, q);
  }
}
__device__ __forceinline__ void inner_slot(bool cross, int rr, int x, int n,
                                           int &i, int &partner) {
  if (cross) {
    const int h = n / 2;
    if (x < h) {
      i = x;
      partner = h + ((x + rr) & (h - 1));
    } else {
      i = (x - h - rr) & (h - 1);
      partner = i;
    }
  } else {
    rr_slot(rr, x, n, i, partner);
  }
}

// One 2 x 2 block of J^T G J: rows (p1, q1) rotated by (c1, s1), columns
// (p2, q2) by (c2, s2); g and n are row-major [row][column].
__device__ __forceinline__ void rot_block(double c1, double s1, double c2,
                                          double s2, const double g[4],
                                          double n[4]) {
  const double h11 = c1 * g[0] - s1 * g[2], h12 = c1 * g[1] - s1 * g[3];
  const double h21 = s1 * g[0] + c1 * g[2], h22 = s1 * g[1] + c1 * g[3];
  n[0] = c2 * h11 - s2 * h12;
  n[1] = s2 * h11 + c2 * h12;
  n[2] = c2 * h21 - s2 * h22;
  n[3] = s2 * h21 + c2 * h22;
}

// a compile-time int as a value (the copy of G a cross round reads)
template <int V> struct IntC {
  static constexpr int value = V;
};

constexpr int P2 = 2 * JB;             // vectors in a block pair
constexpr int NPAIR = JB;              // disjoint pairs per rotation round
constexpr int NTILE = 3;               // upper Gram tiles: II, IJ, JJ
constexpr int NWAVE = RT / 64;
constexpr int NSLOT = 4;               // partial Gram sets summed in LDS
static_assert(P2 == 32 && RT == 512, "tiling assumes 16-wide blocks");

// Storage precision of the rounds: FP64 (every path), or FP32 (the first
// stage of the mixed-precision path).  The Gram products and the rotation
// run on the matrix cores in the storage precision; the Gram is summed,
// tested and diagonalised in FP64 in both.
typedef float v4f __attribute__((ext_vector_type(4)));
template <typename T> struct Prec;
template <> struct Prec<double> {
  typedef v4d V;
  static __device__ __forceinline__ V mma(double a, double b, V c) {
    return mfma_f64(a, b, c);
  }
  // row of the 16 x 16 product held by lane group lk in element e
  // (FP64: lane j + 16 (i % 4) holds D[i][j] in element i / 4)
  static __device__ __forceinline__ int drow(int lk, int e) { return lk + 4 * e; }
};
template <> struct Prec<float> {
  typedef v4f V;
  static __device__ __forceinline__ V mma(float a, float b, V c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  // FP32: lane j + 16 (i / 4) holds D[i][j] in element i % 4
  static __device__ __forceinline__ int drow(int lk, int e) { return 4 * lk + e; }
};

// WPE: wavefronts per SIMD the registers are budgeted for.  Four (two
// workgroups per CU) hold the rotation loop's offsets without spills; six
// (three workgroups per CU, 80 registers, a few reloads per rotation
// chunk) pay off for short vectors in launches of more than two
// workgroups per CU (launch_jacobi_round).
template <typename T, int WPE>
__global__ void __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(WPE)))
    k_jacobi_round(Batch b, UpdScratch s, UpdParams u, int r) {
  typedef Prec<T> PR;
  typedef typename PR::V V;
  constexpr bool F32 = sizeof(T) == 4;
  const int c = blockIdx.y, pi = blockIdx.x;
  if (s.done[c]) return;
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  const int Lt = m > n ? m : n, N = m > n ? n : m;
  const int path = svd_path(Lt, N, u.small_max, u.precond, u.mixed);
  // the vector matrix of the chain's path: R^T (length N) in Y on the QR
  // path, R2^T (length N) in Z on the two-QR path; on the mixed path the
  // FP32 copy of R^T in X (first stage), then the rrk columns of theta' W
  // in X (second stage); on the two-QR mixed path the FP32 copy of R2^T in
  // Y, then the rrk columns of R^T W in Y; theta' in X else
  if (F32 && !path_is_rr(path)) return;
  if (!F32 && round_width(path, N, u.wide_min) != JB) return;  // wide rounds
  const int L = (F32 || path == PATH_QR || path_has_qr2(path)) ? N : Lt;
  const int nvec = (!F32 && path_is_rr(path)) ? s.rrk[c] : N;
  const int NB = n_blocks_even(nvec, JB);
  if (r >= NB - 1 || pi >= NB / 2) return;
  const int ld = vec_ld(L);
  int bi, bj;
  rr_pair(r, pi, NB, bi, bj);
  double *base = path == PATH_QR2 ? s.Z
                 : (path == PATH_QR || path == PATH_RR2) ? s.Y
                                                         : s.X;
  T *X = reinterpret_cast<T *>(base) + (size_t)c * (F32 ? 2 : 1) * s.th_stride;
  const double tol = F32 ? u.tol32 : u.tol;
  const double skip = F32 ? u.skip32 : u.skip;
  auto colidx = [&](int t) { return t < JB ? bi * JB + t : bj * JB + t - JB; };

  // G is symmetric and only its upper triangle (i <= j) is kept.  It is
  // double-buffered: rotation round k reads G[k & 1] and writes
  // G[(k + 1) & 1], so nothing read in a round is overwritten in it.
  __shared__ double G[2][P2][P2 + 1];
  // partial Gram tiles, reused as Q once they are summed into G
  __shared__ double scratch[NSLOT * NTILE * 256];
  double (*Q)[P2 + 1] = reinterpret_cast<double (*)[P2 + 1]>(scratch);
  __shared__ double2 csn[2][NPAIR];  // (c, s) of every pair of a round
  __shared__ int flag[2];
  // per rotation round rr and pair t of round rr + 1: where that pair's
  // three Gram entries sit in round rr (see step 3), packed as bytes; built
  // for the all-pairs rounds only (the cross rounds use fixed offsets)
  __shared__ uint2 look[P2 - 1][NPAIR];
  // The first round of every outer sweep diagonalises the whole block pair
  // (all pairs, so the pairs inside each block are rotated once per
  // sweep); later rounds rotate only the pairs across the two blocks.
  const bool cross = u.cross_inner && r > 0;
  const int nrounds = cross ? NPAIR : P2 - 1;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;

  // ---- 1. Gram matrix -----------------------------------------------------
  // Wave w takes every eighth chunk of 16 rows.  Lane (li, lk) loads rows
  // e0 + 4 lk .. e0 + 4 lk + 3 of vector li of both blocks as aligned
  // 32-byte loads; MFMA step q takes row e0 + 4 lk + q of both operands
  // (the Gram sums over rows, so their order is free) and the three upper
  // tiles are accumulated from the same loads.  Rows L..ld-1 are zero and
  // ld is a multiple of 16, so chunks are loaded without bounds tests (a
  // branch around a load makes the compiler wait for every load in flight,
  // which would serialise the prefetch); past the last chunk the prefetch
  // re-reads the last one.
  if (tid == 0) {
    flag[0] = 0;
    flag[1] = 0;
  }
  for (int e = tid; !cross && e < nrounds * NPAIR; e += RT) {
    const int rr = e / NPAIR, t = e % NPAIR;
    const int rn = rr + 1 < nrounds ? rr + 1 : 0;
    int pn, qn, ia, pa, ib, pb;
    inner_pair(cross, rn, t, P2, pn, qn);
    inner_slot(cross, rr, pn, P2, ia, pa);
    inner_slot(cross, rr, qn, P2, ib, pb);
    const int ra = pn < pa ? 0 : 1, rb = qn < pb ? 0 : 1;
    const unsigned a0 = ra ? pa : pn, a1 = ra ? pn : pa;
    const unsigned b0 = rb ? pb : qn, b1 = rb ? qn : pb;
    look[rr][t] = make_uint2(a0 | a1 << 8 | b0 << 16 | b1 << 24,
                             ia | ib << 8 | ra << 16 | rb << 24);
  }
  {
    constexpr int CSTEP = 16 * NWAVE;
    V acc[NTILE];
#pragma unroll
    for (int t = 0; t < NTILE; ++t) acc[t] = V{0, 0, 0, 0};
    const T *xa = X + (size_t)colidx(li) * ld + 4 * lk;
    const T *xb = X + (size_t)colidx(JB + li) * ld + 4 * lk;
    auto load = [&](const T *x, int e0) -> V {
      return *reinterpret_cast<const V *>(x + e0);
    };
    auto gram4 = [&](const V &a, const V &b) {
      acc[0] = PR::mma(a.x, a.x, acc[0]);
      acc[1] = PR::mma(a.x, b.x, acc[1]);
      acc[2] = PR::mma(b.x, b.x, acc[2]);
      acc[0] = PR::mma(a.y, a.y, acc[0]);
      acc[1] = PR::mma(a.y, b.y, acc[1]);
      acc[2] = PR::mma(b.y, b.y, acc[2]);
      acc[0] = PR::mma(a.z, a.z, acc[0]);
      acc[1] = PR::mma(a.z, b.z, acc[1]);
      acc[2] = PR::mma(b.z, b.z, acc[2]);
      acc[0] = PR::mma(a.w, a.w, acc[0]);
      acc[1] = PR::mma(a.w, b.w, acc[1]);
      acc[2] = PR::mma(b.w, b.w, acc[2]);
    };
    // two register buffers, unrolled by two: the next chunk's loads are
    // issued before this chunk's products (the compiler barrier keeps them
    // there) and no register copy forces an early wait
    const int elast = ld - 16;
    int e0 = 16 * w;
    V a0 = load(xa, min(e0, elast)), b0 = load(xb, min(e0, elast));
    V a1, b1;
    while (e0 < L) {
      const int e1 = min(e0 + CSTEP, elast);
      a1 = load(xa, e1);
      b1 = load(xb, e1);
      asm volatile("" ::: "memory");
      gram4(a0, b0);
      if (e0 + CSTEP >= L) break;
      const int e2 = min(e0 + 2 * CSTEP, elast);
      a0 = load(xa, e2);
      b0 = load(xb, e2);
      asm volatile("" ::: "memory");
      gram4(a1, b1);
      e0 += 2 * CSTEP;
    }
    // fixed-order sum of the eight wave partials: step j adds waves
    // 4 j .. 4 j + 3 into slots 0 .. 3
    double *part = scratch + (w % NSLOT) * NTILE * 256;
#pragma unroll
    for (int step = 0; step < NWAVE / NSLOT; ++step) {
      if (w / NSLOT == step) {
#pragma unroll
        for (int t = 0; t < NTILE; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double *dst = part + t * 256 + PR::drow(lk, q) * 16 + li;
            *dst = step == 0 ? (double)acc[t][q] : *dst + (double)acc[t][q];
          }
      }
      __syncthreads();
    }
  }
  // upper triangle of G from the upper tiles (tile 0: II, 1: IJ, 2: JJ)
  for (int idx = tid; idx < P2 * P2; idx += RT) {
    const int i = idx / P2, j = idx % P2;
    if (i > j) continue;
    const int tile = (i >> 4) + (j >> 4);
    const double *src = scratch + tile * 256 + (i & 15) * 16 + (j & 15);
    double v = src[0];
#pragma unroll
    for (int sl = 1; sl < NSLOT; ++sl) v += src[sl * NTILE * 256];
    G[0][i][j] = v;
  }
  __syncthreads();

  // ---- 2. convergence test; Q = I; angles of the first rotation round -----
  const double tol_in = fmax(0.125 * tol, 4e-16);
  int needs = 0;
  for (int idx = tid; idx < P2 * P2; idx += RT) {
    const int i = idx / P2, j = idx % P2;
    // a cross round tests only the pairs it rotates; the pairs inside a
    // block are tested (and rotated) in the first round of every sweep, and
    // a sweep without any rotation leaves them as tested there
    if (i < j && (!cross || (i < NPAIR && j >= NPAIR)) &&
        pair_needs_rotation(G[0][i][i], G[0][j][j], G[0][i][j], tol, skip))
      needs = 1;
    Q[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid < NPAIR) {
    int p, q;
    inner_pair(cross, 0, tid, P2, p, q);
    double cr = 1.0, sr = 0.0;
    if (pair_rotation(G[0][p][p], G[0][q][q], G[0][p][q], tol_in, skip, cr,
                      sr))
      flag[0] = 1;
    csn[0][tid] = make_double2(cr, sr);
  }
  if (__syncthreads_or(needs) == 0) {
    if (tid < P2) {
      const int col = colidx(tid);
      if (col < nvec) s.sig2[(size_t)c * s.n_cap + col] = G[0][tid][tid];
    }
    return;
  }

  // ---- 3. inner Jacobi sweeps on G, rotations accumulated in Q ------------
  // One barrier per rotation round.  Threads 256.. own the 2 x 2 blocks
  // (pair rp, pair cp), rp <= cp, of the upper triangle of the round,
  // waves 1-7 the (row, pair) items of Q, and lanes 0-15 of wave 0 derive
  // the next round's angles: the three entries of their next pair are
  // recomputed from this round's input exactly as their block owners
  // compute them.
  constexpr int NBLK = NPAIR * (NPAIR + 1) / 2;
  auto gs = [&](double (*Gm)[P2 + 1], int x, int y) -> double & {
    return x <= y ? Gm[x][y] : Gm[y][x];
  };
  // block of the upper triangle owned by this thread (rp <= cp)
  int brp = 0, bcp = 0;
  const bool owner = tid >= 256 && tid < 256 + NBLK;
  if (owner) {
    int k = tid - 256;
    while (k >= NPAIR - brp) {
      k -= NPAIR - brp;
      ++brp;
    }
    bcp = brp + k;
  }
  // Cross rounds relabel the second block after every round: the vector
  // at label 16 + a moves to label 16 + (a - 1) mod 16 in the next round's
  // copy of G.  Pair i is then (i, 16 + i) in every round, so every G
  // offset of the angle lanes and the owners is fixed (bytes from the
  // start of a copy, computed here once).  The values, and the order of
  // the operations on them, are those of the pairing (i, 16 + (i + rr)
  // mod 16) on fixed labels; after a full inner sweep (16 rounds) the
  // labels are the original ones again.  Q keeps the original labels.
  //   owners: the four entries read (rows (rp, 16 + rp), columns (cp,
  //   16 + cp)) and the three written at new places;
  //   angle lane i: the next round's pair i is (i, 16 + (i + 1) mod 16)
  //   here, the first member from pair i and the second from pair ip =
  //   (i + 1) mod 16: both diagonal 2 x 2 blocks and the block between
  //   them, rows from the lower-numbered pair.
  int fo[10];
#pragma unroll
  for (int k = 0; k < 10; ++k) fo[k] = 0;
  bool aswap = false;
  if (cross) {
    constexpr int GROW = (P2 + 1) * (int)sizeof(double);
    auto go = [](int x, int y) {
      return x <= y ? x * GROW + 8 * y : y * GROW + 8 * x;
    };
    if (tid < NPAIR) {
      const int i = tid, ip = (tid + 1) & (NPAIR - 1);
      aswap = ip < i;
      const int ro = aswap ? ip : i, co = aswap ? i : ip;
      fo[0] = go(i, i);
      fo[1] = go(i, NPAIR + i);
      fo[2] = go(NPAIR + i, NPAIR + i);
      fo[3] = go(ip, ip);
      fo[4] = go(ip, NPAIR + ip);
      fo[5] = go(NPAIR + ip, NPAIR + ip);
      fo[6] = go(ro, co);
      fo[7] = go(ro, NPAIR + co);
      fo[8] = go(NPAIR + ro, co);
      fo[9] = go(NPAIR + ro, NPAIR + co);
    }
    if (owner) {
      const int rp = brp, cp = bcp;
      const int rpm = (rp - 1) & (NPAIR - 1), cpm = (cp - 1) & (NPAIR - 1);
      fo[0] = go(rp, cp);
      fo[1] = go(rp, NPAIR + cp);
      fo[2] = go(cp, NPAIR + rp);
      fo[3] = go(NPAIR + rp, NPAIR + cp);
      fo[4] = go(rp, NPAIR + cpm);
      fo[5] = go(cp, NPAIR + rpm);
      fo[6] = go(NPAIR + rpm, NPAIR + cpm);
    }
  }
  // one cross round; the copy of G it reads is a constant of each
  // instantiation, so every G access is a fixed offset from a constant
  // address (the rounds alternate between the copies, 16 to a sweep)
  auto cross_round = [&](auto cur_c, int rr, int isw) {
    constexpr int cur = decltype(cur_c)::value, nxt = cur ^ 1;
    const int rn = rr + 1 < NPAIR ? rr + 1 : 0;
    const char *Gc = reinterpret_cast<const char *>(&G[cur][0][0]);
    char *Gn = reinterpret_cast<char *>(&G[nxt][0][0]);
    auto gc = [&](int o) -> double {
      return *reinterpret_cast<const double *>(Gc + o);
    };
    auto gn = [&](int o) -> double & {
      return *reinterpret_cast<double *>(Gn + o);
    };
    if (tid < NPAIR) {
      const double2 ji = csn[cur][tid];
      const double2 jp = csn[cur][(tid + 1) & (NPAIR - 1)];
      double g[4], nv[4];
      g[0] = gc(fo[0]);
      g[1] = gc(fo[1]);
      g[2] = g[1];
      g[3] = gc(fo[2]);
      rot_block(ji.x, ji.y, ji.x, ji.y, g, nv);
      const double app = nv[0];
      g[0] = gc(fo[3]);
      g[1] = gc(fo[4]);
      g[2] = g[1];
      g[3] = gc(fo[5]);
      rot_block(jp.x, jp.y, jp.x, jp.y, g, nv);
      const double aqq = nv[3];
      g[0] = gc(fo[6]);
      g[1] = gc(fo[7]);
      g[2] = gc(fo[8]);
      g[3] = gc(fo[9]);
      const double2 jr = aswap ? jp : ji, jc = aswap ? ji : jp;
      rot_block(jr.x, jr.y, jc.x, jc.y, g, nv);
      const double apq = aswap ? nv[2] : nv[1];
      double cr = 1.0, sr = 0.0;
      const bool rot = pair_rotation(app, aqq, apq, tol_in, skip, cr, sr);
      if (rot) flag[(isw + (rn == 0)) & 1] = 1;
      csn[nxt][tid] = make_double2(cr, sr);
    }
    if (owner) {
      const double2 j1 = csn[cur][brp], j2 = csn[cur][bcp];
      double g[4], nv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) g[k] = gc(fo[k]);
      rot_block(j1.x, j1.y, j2.x, j2.y, g, nv);
      gn(fo[0]) = nv[0];
      gn(fo[4]) = nv[1];
      // a diagonal block holds (p, q) once: its (q, p) element is skipped
      if (brp != bcp) gn(fo[5]) = nv[2];
      gn(fo[6]) = nv[3];
    }
    // Q items go to waves 1-7 (wave 0 carries the angle lanes)
    for (int item = tid - 64; item >= 0 && item < P2 * NPAIR;
         item += RT - 64) {
      const int row = item / NPAIR, cp = item % NPAIR;
      const int p = cp, q = NPAIR + ((cp + rr) & (NPAIR - 1));
      const double2 jq = csn[cur][cp];
      const double x = Q[row][p], y = Q[row][q];
      Q[row][p] = jq.x * x - jq.y * y;
      Q[row][q] = jq.y * x + jq.x * y;
    }
    __syncthreads();
    if (rr == 0 && tid == 0) flag[(isw + 1) & 1] = 0;
  };
  if (cross) {
    for (int isw = 0; isw < u.inner_sweeps; ++isw) {
      for (int rr = 0; rr < NPAIR; rr += 2) {
        cross_round(IntC<0>(), rr, isw);
        cross_round(IntC<1>(), rr + 1, isw);
      }
      if (!flag[isw & 1]) break;
    }
  } else {
    int gr = 0;                   // rotation rounds done
    // pairing entry of the current round (angle lanes), read one round ahead
    uint2 lk2 = tid < NPAIR ? look[0][tid] : make_uint2(0u, 0u);
    for (int isw = 0; isw < u.inner_sweeps; ++isw) {
      for (int rr = 0; rr < nrounds; ++rr, ++gr) {
        const int cur = gr & 1, nxt = cur ^ 1;
        const int rn = rr + 1 < nrounds ? rr + 1 : 0;
        double (*Gc)[P2 + 1] = G[cur];
        double (*Gn)[P2 + 1] = G[nxt];
        if (tid < NPAIR) {
          // angles of pair tid of the next round from this round's G: its
          // members are row ra of pair ia = (a0, a1) and row rb of pair
          // ib = (b0, b1) of this round
          const int a0 = lk2.x & 255, a1 = (lk2.x >> 8) & 255;
          const int b0 = (lk2.x >> 16) & 255, b1 = lk2.x >> 24;
          const int ia = lk2.y & 255, ib = (lk2.y >> 8) & 255;
          const int ra = (lk2.y >> 16) & 255, rb = lk2.y >> 24;
          const double2 ja = csn[cur][ia], jb = csn[cur][ib];
          double g[4], nv[4];
          g[0] = Gc[a0][a0]; g[1] = Gc[a0][a1]; g[2] = g[1]; g[3] = Gc[a1][a1];
          rot_block(ja.x, ja.y, ja.x, ja.y, g, nv);
          // selects, not indexing: a runtime index would put nv in scratch
          const double app = ra ? nv[3] : nv[0];
          g[0] = Gc[b0][b0]; g[1] = Gc[b0][b1]; g[2] = g[1]; g[3] = Gc[b1][b1];
          rot_block(jb.x, jb.y, jb.x, jb.y, g, nv);
          const double aqq = rb ? nv[3] : nv[0];
          // the cross entry as its owner, block (min(ia,ib), max(ia,ib)),
          // computes it: rows of the smaller pair index first
          double apq;
          if (ia < ib) {
            g[0] = gs(Gc, a0, b0); g[1] = gs(Gc, a0, b1);
            g[2] = gs(Gc, a1, b0); g[3] = gs(Gc, a1, b1);
            rot_block(ja.x, ja.y, jb.x, jb.y, g, nv);
            apq = ra ? (rb ? nv[3] : nv[2]) : (rb ? nv[1] : nv[0]);
          } else {
            g[0] = gs(Gc, b0, a0); g[1] = gs(Gc, b0, a1);
            g[2] = gs(Gc, b1, a0); g[3] = gs(Gc, b1, a1);
            rot_block(jb.x, jb.y, ja.x, ja.y, g, nv);
            apq = rb ? (ra ? nv[3] : nv[2]) : (ra ? nv[1] : nv[0]);
          }
          double cr = 1.0, sr = 0.0;
          const bool rot = pair_rotation(app, aqq, apq, tol_in, skip, cr, sr);
          // the angle belongs to the next sweep when rn wraps to 0
          if (rot) flag[(isw + (rn == 0)) & 1] = 1;
          csn[nxt][tid] = make_double2(cr, sr);
          lk2 = look[rn][tid];
        }
        if (owner) {
          int p1, q1, p2, q2;
          inner_pair(cross, rr, brp, P2, p1, q1);
          inner_pair(cross, rr, bcp, P2, p2, q2);
          const double2 j1 = csn[cur][brp], j2 = csn[cur][bcp];
          double g[4], nv[4];
          g[0] = gs(Gc, p1, p2); g[1] = gs(Gc, p1, q2);
          g[2] = gs(Gc, q1, p2); g[3] = gs(Gc, q1, q2);
          rot_block(j1.x, j1.y, j2.x, j2.y, g, nv);
          gs(Gn, p1, p2) = nv[0];
          gs(Gn, p1, q2) = nv[1];
          // a diagonal block holds (p, q) once: its (q, p) element is skipped
          if (brp != bcp) gs(Gn, q1, p2) = nv[2];
          gs(Gn, q1, q2) = nv[3];
        }
        // Q items go to waves 1-7 (wave 0 carries the angle lanes)
        for (int item = tid - 64; item >= 0 && item < P2 * NPAIR;
             item += RT - 64) {
          const int row = item / NPAIR, cp = item % NPAIR;
          int p, q;
          inner_pair(cross, rr, cp, P2, p, q);
          const double2 jq = csn[cur][cp];
          const double cq = jq.x, sq = jq.y;
          const double x = Q[row][p], y = Q[row][q];
          Q[row][p] = cq * x - sq * y;
          Q[row][q] = sq * x + cq * y;
        }
        __syncthreads();
        // the flag of sweep isw + 1 is cleared once every thread has read it
        // as the flag of sweep isw - 1
        if (rr == 0 && tid == 0) flag[(isw + 1) & 1] = 0;
      }
      if (!flag[isw & 1]) break;
    }
  }

  // ---- 4. Xp <- Xp Q, as D = Q^T Xp^T per 16-row chunk --------------------
  // each wave takes every eighth chunk and loads the next chunk while the
  // current one is multiplied
  constexpr int KB = P2 / 4;
  // lane (li, lk) reads and writes vectors 4 kk + lk (kk < KB) at row
  // e0 + li: the same set on both sides, so one offset table serves both
  int coff[KB];
#pragma unroll
  for (int kk = 0; kk < KB; ++kk) coff[kk] = colidx(4 * kk + lk) * ld;
  // output vectors of lane group lk: PR::drow(lk, q) of each block
  int soff[KB];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    soff[q] = colidx(PR::drow(lk, q)) * ld;
    soff[4 + q] = colidx(JB + PR::drow(lk, q)) * ld;
  }
  T cur[KB], nxt[KB];
  // rows L..ld-1 are zero and stay zero under the rotation, and every
  // 16-row chunk lies inside ld: loads and stores need no bounds tests
  auto load_chunk = [&](int e0, T *v) {
    const int e = e0 + li;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) v[kk] = X[coff[kk] + e];
  };
  constexpr int CSTEP = 16 * NWAVE;
  auto rotate16 = [&](int e0, const T *v) {
    V d0 = {0, 0, 0, 0}, d1 = d0;
#pragma unroll
    for (int kk = 0; kk < KB; ++kk) {
      d0 = PR::mma((T)Q[4 * kk + lk][li], v[kk], d0);
      d1 = PR::mma((T)Q[4 * kk + lk][16 + li], v[kk], d1);
    }
    // D[i][j] (vector 16 t + i, row e0 + j) sits in lane j and element q
    // with i = PR::drow(lk, q)
    const int e = e0 + li;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      X[soff[q] + e] = d0[q];
      X[soff[4 + q] + e] = d1[q];
    }
  };
  // two register buffers, unrolled by two, as in the Gram loop
  int e0 = 16 * w;
  load_chunk(min(e0, ld - 16), cur);
  while (e0 < L) {
    load_chunk(min(e0 + CSTEP, ld - 16), nxt);
    asm volatile("" ::: "memory");
    rotate16(e0, cur);
    if (e0 + CSTEP >= L) break;
    load_chunk(min(e0 + 2 * CSTEP, ld - 16), cur);
    asm volatile("" ::: "memory");
    rotate16(e0 + CSTEP, nxt);
    e0 += 2 * CSTEP;
  }
  if (tid == 0) atomicAdd(&s.rot_cur[c], 1);
}


// =====================================================================
// Wide rounds: blocks of JBW = 32 vectors, one workgroup per block pair of
// 64 vectors, for the chains that take them (round_width).  A sweep has
// NB - 1 rounds of NB / 2 pairs: half the rounds, and half the passes over
// the vectors, of the 16-wide rounds.  Per round:
//   1. Gram of the 64 vectors, its ten upper 16 x 16 tiles by FP64 MFMA:
//      waves 0-3 accumulate tiles (0,0) (0,1) (0,2) (0,3) (1,1) of the four
//      16-vector sub-blocks, waves 4-7 the other five (sub-blocks 1-3 only),
//      each group over all 16-row chunks (the second load of a chunk may hit
//      L2); the partials are summed in a fixed order;
//   2. the convergence test of the 16-wide rounds;
//   3. one cyclic Jacobi sweep of the 64 x 64 Gram, its upper triangle
//      packed and double-buffered in LDS, one barrier per rotation round:
//      lanes 0-31 of wave 0 derive the next round's angles (recomputing the
//      entries they need as the block owners do), waves 1-7 own the 528
//      2 x 2 blocks; on the cross rounds every thread keeps four (row,
//      pair) items of Q in registers, the second column of a pair moving
//      one lane per round, and the second block's vectors are relabelled
//      in G after every round so that the pairs, and with them every LDS
//      offset of the angle lanes and the owners, stay fixed; on the
//      all-pairs round Q is updated in LDS;
//   4. Xp <- Xp Q by FP64 MFMA, each wave reading and writing whole 16-row
//      chunks of all 64 vectors.
// =====================================================================
constexpr int W_P2 = 2 * JBW;
constexpr int W_NPAIR = JBW;
constexpr int W_TRI = W_P2 * (W_P2 + 1) / 2;
constexpr int W_NTILE = 10;
constexpr int W_NBLK = W_NPAIR * (W_NPAIR + 1) / 2;
// waves 1.. own the blocks: wave 0 derives the angles, and a wave whose
// lanes split between the two tasks would run them one after the other
constexpr int W_OWN0 = 64;
constexpr int W_OWNERS = RT - W_OWN0;
static_assert(W_NBLK <= 2 * W_OWNERS, "two blocks per owner at most");

// packed upper triangle, i <= j
__device__ __forceinline__ int wtri(int i, int j) {
  return i * W_P2 - (i * (i - 1)) / 2 + (j - i);
}

__global__ void __launch_bounds__(RT) __attribute__((amdgpu_waves_per_eu(4)))
    k_jacobi_round_wide(Batch b, UpdScratch s, UpdParams u, int r, int c0) {
  const int c = c0 + blockIdx.y, pi = blockIdx.x;
  if (s.done[c]) return;
  const int32_t *chi = chi_row(b, c);
  const int m = 3 * chi[u.k], n = 3 * chi[u.k + 2];
  const int Lt = m > n ? m : n, N = m > n ? n : m;
  const int path = svd_path(Lt, N, u.small_max, u.precond, u.mixed);
  if (round_width(path, N, u.wide_min) != JBW) return;
  const int L = (path == PATH_QR || path == PATH_QR2) ? N : Lt;
  const int NB = n_blocks_even(N, JBW);
  if (r >= NB - 1 || pi >= NB / 2) return;
  const int ld = vec_ld(L);
  int bi, bj;
  rr_pair(r, pi, NB, bi, bj);
  double *base = path == PATH_QR2 ? s.Z : (path == PATH_QR ? s.Y : s.X);
  double *X = base + (size_t)c * s.th_stride;
  const double tol = u.tol, skip = u.skip;
  auto colidx = [&](int t) {
    return t < JBW ? bi * JBW + t : bj * JBW + t - JBW;
  };

  __shared__ double G[2][W_TRI];
  // partial Gram tiles (two slots), reused as Q once they are summed
  __shared__ double scratch[2 * W_NTILE * 256];
  static_assert(W_P2 * (W_P2 + 1) <= 2 * W_NTILE * 256, "Q fits");
  double (*Q)[W_P2 + 1] = reinterpret_cast<double (*)[W_P2 + 1]>(scratch);
  __shared__ double2 csn[2][W_NPAIR];
  __shared__ int flag[2];
  const bool cross = u.cross_inner && r > 0;
  const int nrounds = cross ? W_NPAIR : W_P2 - 1;
  const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int grp = w >> 2, wl = w & 3;
  auto gs = [&](double *Gm, int x, int y) -> double & {
    return x <= y ? Gm[wtri(x, y)] : Gm[wtri(y, x)];
  };

  // ---- 1. Gram matrix -----------------------------------------------------
  if (tid == 0) {
    flag[0] = 0;
    flag[1] = 0;
  }
  {
    constexpr int CSTEP = 16 * 4;  // four waves per group
    v4d acc[5];
#pragma unroll
    for (int t = 0; t < 5; ++t) acc[t] = v4d{0.0, 0.0, 0.0, 0.0};
    const double *xs[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      xs[k] = X + (size_t)colidx(16 * k + li) * ld + 4 * lk;
    // group 1 never uses sub-block 0 (tiles (1,2) .. (3,3))
    auto load4 = [&](int e0, v4d (&v)[4]) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        v[k] = (k > 0 || grp == 0)
                   ? *reinterpret_cast<const v4d *>(xs[k] + e0)
                   : v4d{0.0, 0.0, 0.0, 0.0};
    };
    auto mm = [&](v4d &a, const v4d &x, const v4d &y) {
      a = mfma_f64(x.x, y.x, a);
      a = mfma_f64(x.y, y.y, a);
      a = mfma_f64(x.z, y.z, a);
      a = mfma_f64(x.w, y.w, a);
    };
    auto gram = [&](const v4d (&v)[4]) {
      if (grp == 0) {
        mm(acc[0], v[0], v[0]);
        mm(acc[1], v[0], v[1]);
        mm(acc[2], v[0], v[2]);
        mm(acc[3], v[0], v[3]);
        mm(acc[4], v[1], v[1]);
      } else {
        mm(acc[0], v[1], v[2]);
        mm(acc[1], v[1], v[3]);
        mm(acc[2], v[2], v[2]);
        mm(acc[3], v[2], v[3]);
        mm(acc[4], v[3], v[3]);
      }
    };
    const int elast = ld - 16;
    int e0 = 16 * wl;
    v4d a0[4], a1[4];
    load4(min(e0, elast), a0);
    while (e0 < L) {
      load4(min(e0 + CSTEP, elast), a1);
      asm volatile("" ::: "memory");
      gram(a0);
      if (e0 + CSTEP >= L) break;
      load4(min(e0 + 2 * CSTEP, elast), a0);
      asm volatile("" ::: "memory");
      gram(a1);
      e0 += 2 * CSTEP;
    }
    // fixed-order sum of the four partials of each tile: waves wl = 0, 1
    // write slots 0, 1, then waves wl = 2, 3 add into them
    double *part = scratch + (size_t)(wl & 1) * W_NTILE * 256;
#pragma unroll
    for (int step = 0; step < 2; ++step) {
      if ((wl >> 1) == step) {
#pragma unroll
        for (int t = 0; t < 5; ++t)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            double *dst = part + (5 * grp + t) * 256 + (lk + 4 * q) * 16 + li;
            *dst = step == 0 ? acc[t][q] : *dst + acc[t][q];
          }
      }
      __syncthreads();
    }
  }
  // packed upper triangle of G from the tiles: tile (x, y), x <= y, of the
  // 16-vector sub-blocks -> partial index
  for (int idx = tid; idx < W_P2 * W_P2; idx += RT) {
    const int i = idx / W_P2, j = idx % W_P2;
    if (i > j) continue;
    const int x = i >> 4, y = j >> 4;
    const int tile = x == 0 ? y : (x == 1 ? (y == 1 ? 4 : y + 3)
                                          : (x == 2 ? (y == 2 ? 7 : 8) : 9));
    const int o = tile * 256 + (i & 15) * 16 + (j & 15);
    G[0][wtri(i, j)] = scratch[o] + scratch[W_NTILE * 256 + o];
  }
  __syncthreads();

  // ---- 2. convergence test; Q = I; angles of the first rotation round -----
  const double tol_in = fmax(0.125 * tol, 4e-16);
  int needs = 0;
  for (int idx = tid; idx < W_P2 * W_P2; idx += RT) {
    const int i = idx / W_P2, j = idx % W_P2;
    if (i < j && (!cross || (i < W_NPAIR && j >= W_NPAIR)) &&
        pair_needs_rotation(G[0][wtri(i, i)], G[0][wtri(j, j)],
                            G[0][wtri(i, j)], tol, skip))
      needs = 1;
    Q[i][j] = (i == j) ? 1.0 : 0.0;
  }
  if (tid < W_NPAIR) {
    int p, q;
    inner_pair(cross, 0, tid, W_P2, p, q);
    double cr = 1.0, sr = 0.0;
    if (pair_rotation(G[0][wtri(p, p)], G[0][wtri(q, q)], G[0][wtri(p, q)],
                      tol_in, skip, cr, sr))
      flag[0] = 1;
    csn[0][tid] = make_double2(cr, sr);
  }
  if (__syncthreads_or(needs) == 0) {
    if (tid < W_P2) {
      const int col = colidx(tid);
      if (col < N) s.sig2[(size_t)c * s.n_cap + col] = G[0][wtri(tid, tid)];
    }
    return;
  }

  // ---- 3. inner Jacobi sweep on G, rotations accumulated in Q -------------
  int brp[2] = {0, 0}, bcp[2] = {0, 0};
  bool own[2] = {false, false};
#pragma unroll
  for (int o = 0; o < 2; ++o) {
    int k = tid - W_OWN0 + W_OWNERS * o;
    own[o] = tid >= W_OWN0 && k < W_NBLK;
    if (own[o]) {
      int rp = 0;
      while (k >= W_NPAIR - rp) {
        k -= W_NPAIR - rp;
        ++rp;
      }
      brp[o] = rp;
      bcp[o] = rp + k;
    }
  }
  // Cross rounds relabel the second block after every round: the vector of
  // the second block at label 32 + a moves to label 32 + (a - 1) mod 32 in
  // the next round's copy of G.  Pair i is then (i, 32 + i) in every round,
  // so every LDS offset of the loop is fixed, and it is computed here once.
  // The values, and the order of the operations on them, are those of the
  // pairing (i, 32 + (i + rr) mod 32) on fixed labels.  After a full inner
  // sweep (32 rounds) the labels are the original ones again.
  //   block owners: per block, the four entries read (rows (rp, 32 + rp),
  //   columns (cp, 32 + cp)) and the four written in the next labels;
  //   angle lane i: the next round's pair i is (i, 32 + (i + 1) mod 32) in
  //   this round's labels, the first member from pair i and the second from
  //   pair ip = (i + 1) mod 32: the diagonal 2 x 2 blocks of both pairs and
  //   the block between them, rows from the lower-numbered pair.
  // (offsets in bytes, from the start of either copy of G)
  int fo[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) fo[k] = 0;
  bool aswap = false;
  if (cross) {
    auto gso = [](int x, int y) { return x <= y ? wtri(x, y) : wtri(y, x); };
    if (tid < W_NPAIR) {
      const int i = tid, ip = (tid + 1) & (W_NPAIR - 1);
      aswap = ip < i;
      const int ro = aswap ? ip : i, co = aswap ? i : ip;
      fo[0] = 8 * wtri(i, i);
      fo[1] = 8 * wtri(i, W_NPAIR + i);
      fo[2] = 8 * wtri(W_NPAIR + i, W_NPAIR + i);
      fo[3] = 8 * wtri(ip, ip);
      fo[4] = 8 * wtri(ip, W_NPAIR + ip);
      fo[5] = 8 * wtri(W_NPAIR + ip, W_NPAIR + ip);
      fo[6] = 8 * gso(ro, co);
      fo[7] = 8 * gso(ro, W_NPAIR + co);
      fo[8] = 8 * gso(W_NPAIR + ro, co);
      fo[9] = 8 * gso(W_NPAIR + ro, W_NPAIR + co);
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      if (own[o]) {
        const int rp = brp[o], cp = bcp[o];
        const int rpm = (rp - 1) & (W_NPAIR - 1), cpm = (cp - 1) & (W_NPAIR - 1);
        fo[8 * o + 0] = 8 * wtri(rp, cp);
        fo[8 * o + 1] = 8 * wtri(rp, W_NPAIR + cp);
        fo[8 * o + 2] = 8 * wtri(cp, W_NPAIR + rp);
        fo[8 * o + 3] = 8 * wtri(W_NPAIR + rp, W_NPAIR + cp);
        fo[8 * o + 4] = 8 * wtri(rp, W_NPAIR + cpm);
        fo[8 * o + 5] = 8 * wtri(cp, W_NPAIR + rpm);
        fo[8 * o + 6] = 8 * gso(W_NPAIR + rpm, W_NPAIR + cpm);
      }
    }
  }
  // cross rounds: thread (row, i) holds Q[row][i] and Q[row][32 + (i + rr)
  // % 32] for rows (tid >> 5) + 16 m
  const int qi = tid & 31, qrow = tid >> 5;
  double qa[4], qb[4];
#pragma unroll
  for (int mm = 0; mm < 4; ++mm) {
    const int row = qrow + 16 * mm;
    qa[mm] = row == qi ? 1.0 : 0.0;
    qb[mm] = row == W_NPAIR + qi ? 1.0 : 0.0;
  }
  // one cross round; the copy of G it reads is a constant of each
  // instantiation, so every LDS access is a fixed offset from a constant
  // address (the rounds alternate between the copies, 32 to a sweep)
  auto cross_round = [&](auto cur_c, int rr, int isw) {
    constexpr int cur = decltype(cur_c)::value, nxt = cur ^ 1;
    const int rn = rr + 1 < W_NPAIR ? rr + 1 : 0;
    const char *Gc = reinterpret_cast<const char *>(G[cur]);
    char *Gn = reinterpret_cast<char *>(G[nxt]);
    auto gc = [&](int o) -> double {
      return *reinterpret_cast<const double *>(Gc + o);
    };
    auto gn = [&](int o) -> double & {
      return *reinterpret_cast<double *>(Gn + o);
    };
    if (tid < W_NPAIR) {
      const double2 ji = csn[cur][tid];
      const double2 jp = csn[cur][(tid + 1) & (W_NPAIR - 1)];
      double g[4], nv[4];
      g[0] = gc(fo[0]);
      g[1] = gc(fo[1]);
      g[2] = g[1];
      g[3] = gc(fo[2]);
      rot_block(ji.x, ji.y, ji.x, ji.y, g, nv);
      const double app = nv[0];
      g[0] = gc(fo[3]);
      g[1] = gc(fo[4]);
      g[2] = g[1];
      g[3] = gc(fo[5]);
      rot_block(jp.x, jp.y, jp.x, jp.y, g, nv);
      const double aqq = nv[3];
      g[0] = gc(fo[6]);
      g[1] = gc(fo[7]);
      g[2] = gc(fo[8]);
      g[3] = gc(fo[9]);
      const double2 jr = aswap ? jp : ji, jc = aswap ? ji : jp;
      rot_block(jr.x, jr.y, jc.x, jc.y, g, nv);
      const double apq = aswap ? nv[2] : nv[1];
      double cr = 1.0, sr = 0.0;
      const bool rot = pair_rotation(app, aqq, apq, tol_in, skip, cr, sr);
      if (rot) flag[(isw + (rn == 0)) & 1] = 1;
      csn[nxt][tid] = make_double2(cr, sr);
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
      if (own[o]) {
        const double2 j1 = csn[cur][brp[o]], j2 = csn[cur][bcp[o]];
        double g[4], nv[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) g[k] = gc(fo[8 * o + k]);
        rot_block(j1.x, j1.y, j2.x, j2.y, g, nv);
        gn(fo[8 * o + 0]) = nv[0];
        gn(fo[8 * o + 4]) = nv[1];
        if (brp[o] != bcp[o]) gn(fo[8 * o + 5]) = nv[2];
        gn(fo[8 * o + 6]) = nv[3];
      }
    }
    const double2 jq = csn[cur][qi];
    const int src = (lane & 32) | ((lane + 1) & 31);
#pragma unroll
    for (int mm = 0; mm < 4; ++mm) {
      const double na = jq.x * qa[mm] - jq.y * qb[mm];
      const double nb = jq.y * qa[mm] + jq.x * qb[mm];
      qa[mm] = na;
      qb[mm] = __shfl(nb, src);
    }
    __syncthreads();
    if (rr == 0 && tid == 0) flag[(isw + 1) & 1] = 0;
  };
  if (cross) {
    for (int isw = 0; isw < u.inner_sweeps; ++isw) {
      for (int rr = 0; rr < W_NPAIR; rr += 2) {
        cross_round(IntC<0>(), rr, isw);
        cross_round(IntC<1>(), rr + 1, isw);
      }
      if (!flag[isw & 1]) break;
    }
  } else {
    int gr = 0;
    for (int isw = 0; isw < u.inner_sweeps; ++isw) {
      for (int rr = 0; rr < nrounds; ++rr, ++gr) {
        const int cur = gr & 1, nxt = cur ^ 1;
        const int rn = rr + 1 < nrounds ? rr + 1 : 0;
        double *Gc = G[cur];
        double *Gn = G[nxt];
        if (tid < W_NPAIR) {
          // angles of pair tid of the next round: its members are row ra of
          // pair ia = (a0, a1) and row rb of pair ib = (b0, b1) of this round
          int pn, qn, ia, pa, ib, pb;
          inner_pair(cross, rn, tid, W_P2, pn, qn);
          inner_slot(cross, rr, pn, W_P2, ia, pa);
          inner_slot(cross, rr, qn, W_P2, ib, pb);
          const int ra = pn < pa ? 0 : 1, rb = qn < pb ? 0 : 1;
          const int a0 = ra ? pa : pn, a1 = ra ? pn : pa;
          const int b0 = rb ? pb : qn, b1 = rb ? qn : pb;
          const double2 ja = csn[cur][ia], jb = csn[cur][ib];
          double g[4], nv[4];
          g[0] = Gc[wtri(a0, a0)];
          g[1] = Gc[wtri(a0, a1)];
          g[2] = g[1];
          g[3] = Gc[wtri(a1, a1)];
          rot_block(ja.x, ja.y, ja.x, ja.y, g, nv);
          const double app = ra ? nv[3] : nv[0];
          g[0] = Gc[wtri(b0, b0)];
          g[1] = Gc[wtri(b0, b1)];
          g[2] = g[1];
          g[3] = Gc[wtri(b1, b1)];
          rot_block(jb.x, jb.y, jb.x, jb.y, g, nv);
          const double aqq = rb ? nv[3] : nv[0];
          double apq;
          if (ia < ib) {
            g[0] = gs(Gc, a0, b0);
            g[1] = gs(Gc, a0, b1);
            g[2] = gs(Gc, a1, b0);
            g[3] = gs(Gc, a1, b1);
            rot_block(ja.x, ja.y, jb.x, jb.y, g, nv);
            apq = ra ? (rb ? nv[3] : nv[2]) : (rb ? nv[1] : nv[0]);
          } else {
            g[0] = gs(Gc, b0, a0);
            g[1] = gs(Gc, b0, a1);
            g[2] = gs(Gc, b1, a0);
            g[3] = gs(Gc, b1, a1);
            rot_block(jb.x, jb.y, ja.x, ja.y, g, nv);
            apq = rb ? (ra ? nv[3] : nv[2]) : (ra ? nv[1] : nv[0]);
          }
          double cr = 1.0, sr = 0.0;
          const bool rot = pair_rotation(app, aqq, apq, tol_in, skip, cr, sr);
          if (rot) flag[(isw + (rn == 0)) & 1] = 1;
          csn[nxt][tid] = make_double2(cr, sr);
        }
  #pragma unroll
        for (int o = 0; o < 2; ++o) {
          if (!cross && own[o]) {
            int p1, q1, p2, q2;
            inner_pair(cross, rr, brp[o], W_P2, p1, q1);
            inner_pair(cross, rr, bcp[o], W_P2, p2, q2);
            const double2 j1 = csn[cur][brp[o]], j2 = csn[cur][bcp[o]];
            double g[4], nv[4];
            g[0] = gs(Gc, p1, p2);
            g[1] = gs(Gc, p1, q2);
            g[2] = gs(Gc, q1, p2);
            g[3] = gs(Gc, q1, q2);
            rot_block(j1.x, j1.y, j2.x, j2.y, g, nv);
            gs(Gn, p1, p2) = nv[0];
            gs(Gn, p1, q2) = nv[1];
            if (brp[o] != bcp[o]) gs(Gn, q1, p2) = nv[2];
            gs(Gn, q1, q2) = nv[3];
          }
        }
        {
          for (int item = tid - 64; item >= 0 && item < W_P2 * W_NPAIR;
               item += RT - 64) {
            const int row = item / W_NPAIR, cp = item % W_NPAIR;
            int p, q;
            inner_pair(false, rr, cp, W_P2, p, q);
            const double2 jq = csn[cur][cp];
            const double x = Q[row][p], y = Q[row][q];
            Q[row][p] = jq.x * x - jq.y * y;
            Q[row][q] = jq.y * x + jq.x * y;
          }
        }
        __syncthreads();
        if (rr == 0 && tid == 0) flag[(isw + 1) & 1] = 0;
      }
        if (!flag[isw & 1]) break;
    }
  }
  if (cross) {
    // an inner sweep is W_NPAIR shifts: the second column is 32 + i again
#pragma unroll
    for (int mm = 0; mm < 4; ++mm) {
      Q[qrow + 16 * mm][qi] = qa[mm];
      Q[qrow + 16 * mm][W_NPAIR + qi] = qb[mm];
    }
    __syncthreads();
  }

  // ---- 4. Xp <- Xp Q, as D = Q^T Xp^T per 16-row chunk --------------------
  // each wave takes every eighth chunk; lane (li, lk) reads row e0 + li of
  // vectors 4 kk + lk (kk < 16) and writes row e0 + li of the vectors
  // 16 t + lk + 4 q of the four output tiles
  // Each chunk is loaded in two halves (the 32 vectors of block I, then of
  // block J: eight operands per lane each) into four accumulator tiles, and
  // stored once both halves are in.
  // 32-bit element offsets from one per-lane base per block: vector
  // colidx(32 g + t) = (g ? bj : bi) * 32 + t, so the offset of lane
  // group lk's vector 4 k + lk at row e is gbase[g] + 4 k ld + e, with the
  // 4 k ld part uniform (per-vector pointers hoisted out of the loop would
  // take the registers the accumulators need)
  constexpr int CSTEP = 16 * NWAVE;
  const int gbase0 = (bi * JBW + lk) * ld, gbase1 = (bj * JBW + lk) * ld;
  for (int e0 = 16 * w; e0 < L; e0 += CSTEP) {
    // keeps the Q operands inside the loop: hoisted out they would not fit
    // the registers
    asm volatile("" ::: "memory");
    const int e = e0 + li;
    v4d d[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) d[t] = v4d{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      const int o = (g ? gbase1 : gbase0) + e;
      double v[8];
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8) v[k8] = X[o + 4 * k8 * ld];
#pragma unroll
      for (int k8 = 0; k8 < 8; ++k8) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          d[t] = mfma_f64(Q[32 * g + 4 * k8 + lk][16 * t + li], v[k8], d[t]);
        // at most four Q operands in flight
        asm volatile("" ::: "memory");
      }
    }
    // D_t[i][j] (vector 16 t + i, row e0 + j) in lane j, element q with
    // i = lk + 4 q: block t >> 1, vector 16 (t & 1) + lk + 4 q of it
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int o = ((t >> 1) ? gbase1 : gbase0) + e + 16 * (t & 1) * ld;
#pragma unroll
      for (int q = 0; q < 4; ++q) X[o + 4 * q * ld] = d[t][q];
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
                         int max_len, hipStream_t st) {
  // measured at 64 chains: three workgroups per CU win 7% on theta' of
  // 384 vectors (768 workgroups: one wave of them instead of one and a
  // half) and lose 5% on 768 (the rotation loop's reloads); at one chain
  // occupancy does not matter and the reloads cost 5%
  if (max_len <= 512 && max_pairs * b.B > 2 * 256)
    hipLaunchKernelGGL((k_jacobi_round<double, 6>), dim3(max_pairs, b.B),
                       dim3(RT), 0, st, b, s, u, round);
  else
    hipLaunchKernelGGL((k_jacobi_round<double, 4>), dim3(max_pairs, b.B),
                       dim3(RT), 0, st, b, s, u, round);
}

void launch_jacobi_round_wide(const Batch &b, const UpdScratch &s,
                              const UpdParams &u, int round, int max_pairs,
                              int c0, int nc, hipStream_t st) {
  hipLaunchKernelGGL(k_jacobi_round_wide, dim3(max_pairs, nc), dim3(RT), 0,
                     st, b, s, u, round, c0);
}

void launch_jacobi_round32(const Batch &b, const UpdScratch &s,
                           const UpdParams &u, int round, int max_pairs,
                           hipStream_t st) {
  hipLaunchKernelGGL((k_jacobi_round<float, 4>), dim3(max_pairs, b.B),
                     dim3(RT), 0, st, b, s, u, round);
}

}  // namespace hmps
