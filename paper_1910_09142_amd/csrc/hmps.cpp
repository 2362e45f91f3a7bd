// Host side of the hmps C ABI: validation, the hybrid MPS layout and the
// Trotter update list, the closed-form gates, the workspace layout, and
// the orchestration of the gfx950 kernels (kernels.hip).
//
// Method: Chen & Stoudenmire, arXiv:1910.09142 -- Hybrid METTS-Ancilla
// subsection (steps 1-4 of the Markov chain), Ancilla Method subsection
// (Trotter evolution of physical sites, ancilla interleaving), Results
// section (S=1 Heisenberg Hamiltonian, second-order Trotter, truncation by
// relative discarded weight).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <string>
#include <vector>

#include "../../include/hmps.h"
#include "hmps_internal.h"
#include "small_path.h"

using namespace hmps;

namespace {

constexpr int OP_SWAP = -1;
// sweeps of the FP32 stage of the mixed path (it stops earlier once no
// pair needs a rotation at the FP32 tolerance)
constexpr int RR_FP32_SWEEPS = 40;
constexpr int OP_IDENT = -2;
constexpr size_t ALIGN = 256;
// The width rule: an update takes wide (32-vector) blocks for its chains of
// at least nvec_min vectors when the batch has at least chains_min chains
// (entries with nvec_min ascending and chains_min not increasing, so the
// entries a batch size satisfies give one threshold).  A wide block pair
// is four times the MFMA work of a 16-wide one on a single compute unit,
// in half as many workgroups: it pays once the rounds fill the chip, with
// fewer chains for larger updates.  The default is the table measured on
// MI355X by tune_width.py (width_rule_gfx950.json): gate applications on
// bonds of chi = 180, 256, 384, 512 with 1 .. 64 chains; e.g. at chi = 256
// (768 vectors) 16-wide vs wide 356.9 vs 321.1 per s at 8 chains, 515.8
// vs 602.3 at 16, 766.4 vs 983.3 at 64.  hmps_set_width_rule replaces it.
// A chain's result depends on its own input and on the width it takes.
struct WidthEntry {
  int nvec_min, chains_min;
};
constexpr int MAX_WIDTH_RULE = 16;
const WidthEntry DEFAULT_WIDTH_RULE[] = {
    {540, 16}, {768, 16}, {1152, 8}, {1536, 8}};

size_t align_up(size_t x) { return (x + ALIGN - 1) / ALIGN * ALIGN; }

// ---------------------------------------------------------------------
// two-site gate exp(-x J S_1.S_2): S.S has eigenvalues -2, -1, +1 on total
// spin 0, 1, 2; the projectors are polynomials of h = S.S.
// ---------------------------------------------------------------------
void heisenberg9(double h[81]) {
  const double r2 = std::sqrt(2.0);
  double sz[3] = {1.0, 0.0, -1.0};
  double sp[3][3] = {{0, r2, 0}, {0, 0, r2}, {0, 0, 0}};
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b)
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d) {
          // <a b| Sz Sz + (S+ S- + S- S+)/2 |c d>
          double v = (a == c && b == d) ? sz[a] * sz[b] : 0.0;
          v += 0.5 * (sp[a][c] * sp[d][b] + sp[c][a] * sp[b][d]);
          h[(a * 3 + b) * 9 + (c * 3 + d)] = v;
        }
}

void matmul9(const double *A, const double *B, double *C) {
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double v = 0.0;
      for (int k = 0; k < 9; ++k) v += A[i * 9 + k] * B[k * 9 + j];
      C[i * 9 + j] = v;
    }
}

void gate9(double J, double x, double *out) {
  double h[81], h2[81], hp2[81], hm1[81], hp1[81], t[81];
  heisenberg9(h);
  for (int i = 0; i < 81; ++i) {
    const double id = (i % 10 == 0) ? 1.0 : 0.0;
    hp2[i] = h[i] + 2.0 * id;
    hm1[i] = h[i] - id;
    hp1[i] = h[i] + id;
  }
  matmul9(h, h, h2);
  double p0[81], p1[81], p2[81];
  for (int i = 0; i < 81; ++i) p0[i] = (h2[i] - ((i % 10 == 0) ? 1.0 : 0.0)) / 3.0;
  matmul9(hp2, hm1, t);
  for (int i = 0; i < 81; ++i) p1[i] = -0.5 * t[i];
  matmul9(hp2, hp1, t);
  for (int i = 0; i < 81; ++i) p2[i] = t[i] / 6.0;
  const double e0 = std::exp(2.0 * x * J), e1 = std::exp(x * J),
               e2 = std::exp(-x * J);
  for (int i = 0; i < 81; ++i) out[i] = e0 * p0[i] + e1 * p1[i] + e2 * p2[i];
}

void swap9(double *out) {
  for (int i = 0; i < 81; ++i) out[i] = 0.0;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) out[(b * 3 + a) * 9 + (a * 3 + b)] = 1.0;
}

// ---------------------------------------------------------------------
// Philox4x64-10 (Salmon et al., SC'11), first output word.
// ---------------------------------------------------------------------
uint64_t philox0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                 uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
  for (int r = 0; r < 10; ++r) {
    if (r) {
      k0 += W0;
      k1 += W1;
    }
    const unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    const unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    const uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    const uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  return c0;
}

// ---------------------------------------------------------------------
// layout + update list
// ---------------------------------------------------------------------
struct Plan {
  int n_phys = 0, len = 0, n_env = 0, n_bonds = 0;
  std::vector<int> phys_of_pos, pos_of_phys, is_cluster, is_ancilla,
      env_index, env_pos;
  std::vector<double> couplings;       // distinct J, first-appearance order
  std::vector<int> bond_p, bond_q;     // per lattice bond, p < q
  std::vector<double> bond_J;
  std::vector<int> step_k, step_op;    // one Trotter step
};

std::string validate_and_plan(const hmps_lattice *lat, Plan &P) {
  if (!lat) return "lattice is NULL";
  if (lat->n_phys < 1) return "n_phys must be >= 1";
  if (lat->n_bonds < 0) return "n_bonds must be >= 0";
  if (lat->n_bonds > 0 && (!lat->bond_i || !lat->bond_j || !lat->bond_J))
    return "bond arrays are NULL";
  if (!lat->mps_order || !lat->in_cluster) return "order/cluster arrays NULL";
  const int n = lat->n_phys;
  std::vector<int> seen(n, 0);
  for (int t = 0; t < n; ++t) {
    const int i = lat->mps_order[t];
    if (i < 0 || i >= n || seen[i]) return "mps_order is not a permutation";
    seen[i] = 1;
  }
  for (int b = 0; b < lat->n_bonds; ++b) {
    const int i = lat->bond_i[b], j = lat->bond_j[b];
    if (i < 0 || i >= n || j < 0 || j >= n || i == j)
      return "bond endpoints out of range";
    if (!std::isfinite(lat->bond_J[b])) return "bond coupling is not finite";
  }
  P = Plan();
  P.n_phys = n;
  P.pos_of_phys.assign(n, -1);
  for (int t = 0; t < n; ++t) {
    const int i = lat->mps_order[t];
    P.pos_of_phys[i] = (int)P.phys_of_pos.size();
    P.phys_of_pos.push_back(i);
    P.is_ancilla.push_back(0);
    P.is_cluster.push_back(lat->in_cluster[i] ? 1 : 0);
    if (lat->in_cluster[i]) {
      P.phys_of_pos.push_back(-1);
      P.is_ancilla.push_back(1);
      P.is_cluster.push_back(1);
    }
  }
  P.len = (int)P.phys_of_pos.size();
  P.env_index.assign(P.len, -1);
  for (int p = 0; p < P.len; ++p)
    if (!P.is_cluster[p]) {
      P.env_index[p] = (int)P.env_pos.size();
      P.env_pos.push_back(p);
    }
  P.n_env = (int)P.env_pos.size();
  P.n_bonds = lat->n_bonds;
  struct B3 {
    int p, q, jx;
  };
  std::vector<B3> mb;
  for (int b = 0; b < lat->n_bonds; ++b) {
    const double J = lat->bond_J[b];
    int jx = -1;
    for (size_t t = 0; t < P.couplings.size(); ++t)
      if (P.couplings[t] == J) jx = (int)t;
    if (jx < 0) {
      jx = (int)P.couplings.size();
      P.couplings.push_back(J);
    }
    int p = P.pos_of_phys[lat->bond_i[b]], q = P.pos_of_phys[lat->bond_j[b]];
    if (p > q) std::swap(p, q);
    P.bond_p.push_back(p);
    P.bond_q.push_back(q);
    P.bond_J.push_back(J);
    mb.push_back({p, q, jx});
  }
  std::stable_sort(mb.begin(), mb.end(), [](const B3 &a, const B3 &b) {
    return a.p != b.p ? a.p < b.p : a.q < b.q;
  });
  // forward half-sweep: bring p next to q by swaps, gate, swap back
  std::vector<int> hk, hop;
  for (const B3 &e : mb) {
    for (int k = e.p; k < e.q - 1; ++k) {
      hk.push_back(k);
      hop.push_back(OP_SWAP);
    }
    hk.push_back(e.q - 1);
    hop.push_back(e.jx);
    for (int k = e.q - 2; k >= e.p; --k) {
      hk.push_back(k);
      hop.push_back(OP_SWAP);
    }
  }
  P.step_k = hk;
  P.step_op = hop;
  for (int t = (int)hk.size() - 1; t >= 0; --t) {
    P.step_k.push_back(hk[t]);
    P.step_op.push_back(hop[t]);
  }
  return "";
}

}  // namespace

// ---------------------------------------------------------------------
// context
// ---------------------------------------------------------------------
struct hmps_ctx {
  hmps_options opt{};
  hipStream_t stream = nullptr;
  std::string err;
  bool poisoned = false;
  bool ready = false;        // chains from hmps_init_cluster_env
  bool bond_loaded = false;  // chains from hmps_load_bond
  Plan plan;
  int B = 0;
  uint64_t seed = 0;
  uint64_t chain0 = 0;     // global id of chain 0 (Philox counters)
  int64_t sample = 0;
  int center = 0;
  // an evolution applied in parts (hmps_evolve_updates): the next update
  // of its list and the parameters it was started with
  int64_t evo_pos = 0;
  double evo_beta = 0.0, evo_tau = 0.0, evo_cutoff = 0.0;
  int evo_chi = 0;
  bool have_spectrum = false;  // d_sig / d_knew hold an update's result
  std::vector<int> h_chi;  // [B][len+1]
  hmps_stats_t stats{};
  bool sync_debug = false;  // HMPS_SYNC_DEBUG=1: check every launch
  // One inner sweep per block pair: measured on the 2x16 ladder at
  // chi = 256, capping the inner Gram Jacobi at 1 sweep instead of 4 costs
  // 2% more outer sweeps and halves the time per round.
  int inner_sweeps = 1;
  double skip = 1e-30;
  // Outer rounds after the first of a sweep rotate only the pairs across
  // their two blocks (16 inner rounds instead of 31): measured on the same
  // ladder, 4% more outer sweeps and 23% less time (one chain).
  int cross_inner = 1;
  // wide (32-vector) blocks for the large FP64 updates: -1 = by the width
  // rule, 0 = never, 1 = always (HMPS_WIDE)
  int wide = -1;
  std::vector<WidthEntry> width_rule{std::begin(DEFAULT_WIDTH_RULE),
                                    std::end(DEFAULT_WIDTH_RULE)};
  // the batch size the width rule reads, when not B: the U(1) block batch
  // reads the chain count of the whole update, so that every pass of an
  // update gives a block the same width
  int width_batch = 0;
  // largest theta' (m * n doubles) whose SVD runs in one workgroup's LDS;
  // larger ones take the blocked rounds.  The in-LDS kernel runs its pair
  // products on vector lanes, so beyond a few thousand entries the blocked
  // MFMA rounds win even at a single chain (at most SMALL_LDS).
  size_t small_max = 2048;
  // Householder QR preconditioning of the blocked rounds: 0 none, 1 one QR,
  // 2 two (FP64 chains; HMPS_QR=0/1/2, for measurements).  On the chi =
  // 256 gate workload one QR cuts the sweeps per update from about 30 to
  // about 14.
  int precond = 2;
  bool skip_theta = false;  // hmps_svd_probe: theta' is placed by the host
  bool zero_ok = false;     // an all-zero theta' keeps nothing (U(1) blocks)
  // U(1) symmetry (HMPS_SYM_U1): the charge blocks of an update are the
  // chains of `sub` (two sites each, theta' placed by k_u1_gather)
  int symmetry = HMPS_SYM_NONE;
  int max_blocks = 0;
  bool u1_live = false;  // the chains carry charges (init or collapse)
  hmps_ctx *sub = nullptr;
  // +1 where an MPS position holds a physical site, -1 an ancilla (swap
  // updates move them; every Trotter step restores the layout)
  std::vector<int> pos_sign;
  // charges of every bond of every chain as runs (charge, count) in index
  // order, one run per charge: [B][len+1]
  std::vector<std::vector<std::pair<int, int>>> h_qg;
  int32_t *d_u1_blk = nullptr, *d_u1_kv = nullptr, *d_u1_jmap = nullptr;
  double *d_u1_scale = nullptr;
  int32_t *h_u1_kv = nullptr;   // pinned [max_blocks]
  int32_t *h_u1_err = nullptr;  // pinned [max_blocks] the blocks' error flags
  int32_t *h_u1_tab = nullptr;  // pinned block and chain tables of a pass
  // the block batch leaves its ranks and flags on the device for the U(1)
  // update to read with its own; its round time is read then
  bool defer_finish = false;
  bool pending_time = false;
  double pending_svd_flops = 0.0;
  size_t u1_sub_off = 0, u1_sub_bytes = 0;
  int64_t u1_blocks = 0;
  // device buffers (carved from the workspace)
  size_t site_cap = 0, chi2 = 0, th_stride = 0;
  int n_cap = 0, slots = 0, qr_panels = 0;
  size_t rrG_stride = 0;
  double *d_sites = nullptr, *d_TH = nullptr, *d_X = nullptr,
         *d_Y = nullptr, *d_Z = nullptr, *d_qrT = nullptr, *d_norm2 = nullptr,
         *d_rrG = nullptr,
         *d_sig2 = nullptr, *d_sig = nullptr, *d_fac = nullptr,
         *d_logw = nullptr, *d_disc = nullptr, *d_gates = nullptr,
         *d_envs = nullptr, *d_wsz = nullptr, *d_bscr = nullptr,
         *d_norm = nullptr, *d_bond_ss = nullptr, *d_energy = nullptr,
         *d_pair_ss = nullptr, *d_mom = nullptr, *d_mom_out = nullptr,
         *d_qn = nullptr, *d_bond_J = nullptr;
  int32_t *d_chi = nullptr, *d_perm = nullptr, *d_knew = nullptr,
          *d_rot = nullptr, *d_done = nullptr, *d_err = nullptr,
          *d_pair_p = nullptr, *d_pair_q = nullptr,
          *d_sweeps = nullptr, *d_near = nullptr, *d_bond_p = nullptr,
          *d_rrk = nullptr,
          *d_bond_q = nullptr, *d_is_cluster = nullptr,
          *d_is_ancilla = nullptr, *d_env_index = nullptr;
  uint8_t *d_labels = nullptr, *d_outcomes = nullptr;
  // pinned host staging
  int32_t *h_stage = nullptr;  // 4 * max_chains
  hipEvent_t sweep_ev[2] = {nullptr, nullptr};
  hipEvent_t svd_ev[2] = {nullptr, nullptr};  // timed span of the rounds
  // the second half of the chains runs on stream2 for the wide rounds
  // (bit 1: one half's launches fill the compute units the other half's
  // last workgroups leave idle) and the QRs (bit 2: one half's panels run
  // beside the other half's trailing updates); HMPS_SPLIT=0..3
  hipStream_t stream2 = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  int split = 3;
};

namespace {

struct Carver {
  char *base;
  size_t off = 0;
  template <class T>
  T *take(size_t count) {
    T *p = reinterpret_cast<T *>(base ? base + off : nullptr);
    off += align_up(count * sizeof(T));
    return p;
  }
};

// Lays out every device buffer; with base == nullptr it only measures.
// svd_only: the block batch of a U(1) context, which never measures (no
// environments or bond scratch).
size_t carve(hmps_ctx *c, char *base, int max_chains, int max_sites,
             int chi_cap, int max_bonds, int max_blocks = 0,
             bool svd_only = false) {
  Carver cv{base};
  const size_t B = max_chains;
  const size_t chi2 = (size_t)chi_cap * chi_cap;
  const size_t site_cap = 3 * chi2;
  const int mc = 3 * chi_cap;
  // padded vector count: an even number of blocks of JB vectors
  const int n_cap = npad_vectors(mc);
  // vectors of length L <= 3 chi_cap are stored with stride vector_stride
  const size_t th_stride = (size_t)vector_stride(mc) * n_cap;
  const int slots = std::max(2, std::min(std::max(max_bonds, 1), 8));
  hmps_ctx tmp;
  hmps_ctx *t = c ? c : &tmp;
  t->site_cap = site_cap;
  t->chi2 = chi2;
  t->th_stride = th_stride;
  t->n_cap = n_cap;
  t->slots = slots;
  t->d_sites = cv.take<double>(B * max_sites * site_cap);
  t->d_chi = cv.take<int32_t>(B * (max_sites + 1));
  t->d_TH = cv.take<double>(B * th_stride);
  t->d_X = cv.take<double>(B * th_stride);
  t->d_Y = cv.take<double>(B * th_stride);
  t->d_Z = cv.take<double>(B * th_stride);
  // T factors of every panel of both QR stages
  t->qr_panels = (mc + QB - 1) / QB;
  t->d_qrT = cv.take<double>(B * 2 * t->qr_panels * QB * QB);
  // Gram of the Ritz basis of the two-QR mixed path (chi_max <= chi_cap)
  {
    const int kcap = std::min(n_cap, (chi_cap + 64 + 31) / 32 * 32);
    const size_t ldk = (size_t)((kcap + 15) & ~15);
    t->rrG_stride = ldk * ldk;
    t->d_rrG = cv.take<double>(B * t->rrG_stride);
  }
  t->d_sig2 = cv.take<double>(B * n_cap);
  t->d_sig = cv.take<double>(B * n_cap);
  t->d_perm = cv.take<int32_t>(B * n_cap);
  t->d_knew = cv.take<int32_t>(B);
  t->d_err = cv.take<int32_t>(B);
  t->d_rot = cv.take<int32_t>(B);
  t->d_done = cv.take<int32_t>(B);
  t->d_sweeps = cv.take<int32_t>(B);
  t->d_rrk = cv.take<int32_t>(B);
  t->d_near = cv.take<int32_t>(B);
  t->d_fac = cv.take<double>(B);
  t->d_norm2 = cv.take<double>(B * NORM_SPLIT);
  t->d_logw = cv.take<double>(B);
  t->d_disc = cv.take<double>(B);
  t->d_norm = cv.take<double>(B);
  t->d_energy = cv.take<double>(B);
  t->d_qn = cv.take<double>(B);
  t->d_gates = cv.take<double>((size_t)(max_bonds + 2) * 81);
  const size_t meas = svd_only ? 0 : 1;
  t->d_envs = cv.take<double>(meas * B * (max_sites + 1) * chi2);
  t->d_wsz = cv.take<double>(B * max_sites);
  t->d_bscr = cv.take<double>(meas * B * slots * 4 * chi2);
  t->d_bond_ss = cv.take<double>(B * std::max(max_bonds, 1));
  // per-chain moments of every bond and of the energy, and their total
  t->d_mom = cv.take<double>(B * (size_t)(max_bonds + 1) * 3);
  t->d_mom_out = cv.take<double>((size_t)(max_bonds + 1) * 3);
  t->d_bond_J = cv.take<double>(std::max(max_bonds, 1));
  t->d_bond_p = cv.take<int32_t>(std::max(max_bonds, 1));
  t->d_bond_q = cv.take<int32_t>(std::max(max_bonds, 1));
  t->d_pair_ss = cv.take<double>(B * PAIR_CHUNK);
  t->d_pair_p = cv.take<int32_t>(PAIR_CHUNK);
  t->d_pair_q = cv.take<int32_t>(PAIR_CHUNK);
  t->d_is_cluster = cv.take<int32_t>(max_sites);
  t->d_is_ancilla = cv.take<int32_t>(max_sites);
  t->d_env_index = cv.take<int32_t>(max_sites);
  t->d_labels = cv.take<uint8_t>(B * max_sites);
  t->d_outcomes = cv.take<uint8_t>(B * max_sites);
  if (max_blocks > 0) {
    // U(1): block and chain tables of a pass, the merge's results, and the
    // workspace of the block batch (two-site chains of up to chi_cap)
    // the block table of a pass and its chain table right after it: one
    // copy from the host
    t->d_u1_blk = cv.take<int32_t>((size_t)max_blocks * U1_BLK + B * U1_CH);
    t->d_u1_kv = cv.take<int32_t>(max_blocks);
    t->d_u1_scale = cv.take<double>(max_blocks);
    t->d_u1_jmap = cv.take<int32_t>(B * n_cap);
    t->u1_sub_bytes =
        carve(nullptr, nullptr, max_blocks, 2, chi_cap, 0, 0, true);
    t->u1_sub_off = cv.off;
    cv.off += align_up(t->u1_sub_bytes);
  }
  return cv.off;
}

// Records the error.  A device or numeric failure poisons the context and
// drains its stream first: entry points enqueue host-to-device copies from
// their own local buffers and the caller's arrays, and none of those may
// still be in flight once the entry point has returned.
hmps_status fail(hmps_ctx *c, hmps_status st, const std::string &msg) {
  if (c) {
    c->err = msg;
    if (st == HMPS_E_DEVICE || st == HMPS_E_NUMERIC) {
      c->poisoned = true;
      (void)hipStreamSynchronize(c->stream);  // null: the default stream
    }
  }
  return st;
}

#define LAUNCHCHK(ctx)                                                     \
  do {                                                                     \
    if ((ctx)->sync_debug) {                                               \
      HIPCHK(hipStreamSynchronize((ctx)->stream));                         \
      HIPCHK(hipGetLastError());                                           \
    }                                                                      \
  } while (0)

#define HIPCHK(call)                                                       \
  do {                                                                     \
    hipError_t e_ = (call);                                                \
    if (e_ != hipSuccess)                                                  \
      return fail(ctx, HMPS_E_DEVICE,                                      \
                  std::string(#call) + ": " + hipGetErrorString(e_));      \
  } while (0)

Batch batch_of(hmps_ctx *ctx) {
  Batch b;
  b.sites = ctx->d_sites;
  b.chi = ctx->d_chi;
  b.nsites = ctx->plan.len;
  b.site_cap = ctx->site_cap;
  b.B = ctx->B;
  return b;
}

UpdScratch scratch_of(hmps_ctx *ctx) {
  UpdScratch s;
  s.TH = ctx->d_TH;
  s.X = ctx->d_X;
  s.Y = ctx->d_Y;
  s.Z = ctx->d_Z;
  s.qrT = ctx->d_qrT;
  s.qr_panels = ctx->qr_panels;
  s.rrG = ctx->d_rrG;
  s.rrG_stride = ctx->rrG_stride;
  s.th_stride = ctx->th_stride;
  s.sig2 = ctx->d_sig2;
  s.perm = ctx->d_perm;
  s.sig = ctx->d_sig;
  s.n_cap = ctx->n_cap;
  s.knew = ctx->d_knew;
  s.fac = ctx->d_fac;
  s.norm2 = ctx->d_norm2;
  s.logw = ctx->d_logw;
  s.discarded = ctx->d_disc;
  s.rot_cur = ctx->d_rot;
  s.done = ctx->d_done;
  s.err = ctx->d_err;
  s.sweeps = ctx->d_sweeps;
  s.rrk = ctx->d_rrk;
  return s;
}

// Host copy of the bond dimensions right after an initialisation.
void init_host_chi(hmps_ctx *ctx) {
  const int L = ctx->plan.len;
  ctx->h_chi.assign((size_t)ctx->B * (L + 1), 1);
  for (int c = 0; c < ctx->B; ++c)
    for (int p = 0; p < L; ++p)
      ctx->h_chi[(size_t)c * (L + 1) + p + 1] =
          (ctx->plan.is_cluster[p] && !ctx->plan.is_ancilla[p]) ? 3 : 1;
}

// Makes the context's device current for the duration of a call and
// restores the caller's device afterwards.
struct DeviceGuard {
  int prev = -1, dev;
  explicit DeviceGuard(int d) : dev(d) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    if (prev >= 0 && prev != dev) (void)hipSetDevice(prev);
  }
};

hmps_status check_usable(hmps_ctx *ctx, bool need_init) {
  if (!ctx) return HMPS_E_INVALID;
  if (ctx->poisoned)
    return HMPS_E_STATE;
  if (need_init && !ctx->ready)
    return fail(ctx, HMPS_E_STATE, "hmps_init_cluster_env has not been called");
  return HMPS_OK;
}

// The smallest vector count that takes wide blocks in an update of this
// batch (0: none).
int wide_threshold(const hmps_ctx *ctx) {
  if (ctx->wide == 0) return 0;
  if (ctx->wide == 1) return W32_MIN_N;
  const int batch = ctx->width_batch > 0 ? ctx->width_batch : ctx->B;
  int t = 0;
  for (const WidthEntry &e : ctx->width_rule)
    if (batch >= e.chains_min && (t == 0 || e.nvec_min < t)) t = e.nvec_min;
  return t;
}

// Parameters of one two-site update on (k, k+1).
UpdParams update_params(const hmps_ctx *ctx, int k, int op, bool right,
                        int chi_max, double cutoff, int mixed,
                        int wide_min) {
  const bool is_move = (op == OP_IDENT);
  UpdParams u;
  u.k = k;
  const int ncoup = (int)ctx->plan.couplings.size();
  u.gate = ctx->d_gates +
           81 * (op >= 0 ? op : (op == OP_SWAP ? ncoup : ncoup + 1));
  u.is_gate = op >= 0;
  u.right = right ? 1 : 0;
  u.chi_max = is_move ? ctx->opt.chi_cap : chi_max;
  u.cutoff = is_move ? 0.0 : cutoff;
  u.tol = ctx->opt.jacobi_tol;
  u.max_sweeps = ctx->opt.max_sweeps;
  u.mixed = mixed;
  u.tol32 = 8.0 * std::sqrt(3.0 * ctx->opt.chi_cap) * 1.1920929e-7;
  // vectors below 1e-12 sigma_0 are left unrotated in FP32 and out of the
  // Ritz basis (the numerically null part of a rank-deficient theta');
  // every other pair is rotated to the FP32 tolerance relative to its own
  // norms, so the basis vectors are orthogonal to about tol32
  u.skip32 = 1e-24;
  u.precond = ctx->precond;
  u.small_max = ctx->small_max;
  u.inner_sweeps = ctx->inner_sweeps;
  u.skip = ctx->skip;
  u.cross_inner = ctx->cross_inner;
  u.wide_min = wide_min;
  u.zero_ok = ctx->zero_ok ? 1 : 0;
  return u;
}

hmps_status do_update_u1(hmps_ctx *ctx, int k, int op, bool right,
                         int chi_max, double cutoff);

// One two-site update on (k, k+1) for every chain.
hmps_status do_update(hmps_ctx *ctx, int k, int op, bool right, int chi_max,
                      double cutoff) {
  if (ctx->u1_live) return do_update_u1(ctx, k, op, right, chi_max, cutoff);
  const int L = ctx->plan.len;
  int max_chiL = 1, max_chiR = 1;
  // each chain's SVD runs in LDS when its theta' has at most small_max
  // entries, else on the blocked rounds; the rounds' grid is sized by the
  // blocked chains alone
  int n_small = 0, n_blocked = 0, n_qr = 0, n_rr = 0, n_qr2 = 0;
  // max_nb: 16-wide FP64 blocks, max_nbw: wide blocks (0: no chain takes
  // that width), max_nb32: the FP32 rounds of the mixed path (16-wide)
  int max_nb = 0, max_nbw = 0, max_nb32 = 2, max_vlen = 1, max_nvec = 1,
      max_qr_n = 0;
  int max_rr_n = 0, max_rr_l = 0, max_qr2_n = 0, max_qr_l = 0;
  // longest vector of the 16-wide FP64 rounds (R^T, R2^T, the Ritz basis
  // projection or theta' itself)
  int max_len16 = 0;
  double flops = 0.0, svd_flops = 0.0;
  const bool is_move = (op == OP_IDENT);
  // centre moves are exact gauge changes, and hmps_svd_probe (theta' placed
  // by the host) is the FP64 SVD: both always FP64
  const int mixed = ctx->opt.precision == HMPS_PREC_MIXED_FP32 && !is_move &&
                    !ctx->skip_theta;
  const int wide = wide_threshold(ctx);
  for (int c = 0; c < ctx->B; ++c) {
    const int *row = &ctx->h_chi[(size_t)c * (L + 1)];
    {
      // algorithmic work: theta, gate, Golub-Reinsch thin SVD (U and V)
      const double cl = row[k], cm = row[k + 1], cr = row[k + 2];
      const double lv = 3.0 * std::max(cl, cr), nv = 3.0 * std::min(cl, cr);
      const double f_svd = 14.0 * lv * nv * nv + 8.0 * nv * nv * nv;
      flops += 18.0 * cl * cm * cr + 162.0 * cl * cr + f_svd;
      svd_flops += f_svd;
    }
    max_chiL = std::max(max_chiL, row[k]);
    max_chiR = std::max(max_chiR, row[k + 2]);
    // the Jacobi SVD orthogonalises min(m, n) vectors of length max(m, n)
    const int nvec = 3 * std::min(row[k], row[k + 2]);
    max_vlen = std::max(max_vlen, 3 * std::max(row[k], row[k + 2]));
    max_nvec = std::max(max_nvec, nvec);
    const int vlen = 3 * std::max(row[k], row[k + 2]);
    const int path = svd_path(vlen, nvec, ctx->small_max, ctx->precond, mixed);
    if (path == PATH_SMALL) {
      ++n_small;
    } else {
      ++n_blocked;
      if (path_is_rr(path)) {
        // FP32 rounds on all nvec vectors, FP64 rounds on the Ritz basis
        ++n_rr;
        max_rr_n = std::max(max_rr_n, nvec);
        max_rr_l = std::max(max_rr_l, vlen);
        max_nb32 = std::max(max_nb32, n_blocks_even(nvec, JB));
        max_nb = std::max(max_nb,
                          n_blocks_even(rr_vectors(nvec, chi_max), JB));
        max_len16 = std::max(max_len16, path == PATH_RR2 ? nvec : vlen);
      } else if (round_width(path, nvec, wide) == JBW) {
        max_nbw = std::max(max_nbw, n_blocks_even(nvec, JBW));
      } else {
        max_nb = std::max(max_nb, n_blocks_even(nvec, JB));
        max_len16 = std::max(max_len16,
                             path == PATH_QR || path == PATH_QR2 ? nvec : vlen);
      }
      if (path_has_qr(path)) {
        ++n_qr;
        max_qr_n = std::max(max_qr_n, nvec);
        max_qr_l = std::max(max_qr_l, vlen);
      }
      if (path_has_qr2(path)) ++n_qr2;
      if (path == PATH_QR2) max_qr2_n = std::max(max_qr2_n, nvec);
    }
  }
  const UpdParams u = update_params(ctx, k, op, right, chi_max, cutoff, mixed, wide);
  Batch b = batch_of(ctx);
  UpdScratch s = scratch_of(ctx);
  hipStream_t st = ctx->stream;
  bool timed_svd = false;
  if (!ctx->skip_theta) {
    launch_theta(b, s, u, max_chiL, max_chiR, st);
    // ||theta'||^2: the gate's log-weight, the mixed path's unresolved tail
    if (u.is_gate || mixed) launch_theta_norm(b, s, u, st);
    LAUNCHCHK(ctx);
  }
  if (n_small > 0) {
    launch_jacobi_small_upto(b, s, u, ctx->small_max, st);
    LAUNCHCHK(ctx);
  }
  if (n_blocked > 0) {
    launch_pad(b, s, u, st);
    if (n_qr > 0) {
      // theta' = Q R panel by panel, then R^T into the vector buffer; on
      // the two-QR path R^T = Q2 R2 the same way, and R2^T into Z
      const int panels = (max_qr_n + QB - 1) / QB;
      // the two halves of a batch of 16 chains or more on two streams: one
      // half's latency-bound panel runs beside the other half's trailing
      // update, which is bound by HBM
      const bool qsplit = (ctx->split & 2) && ctx->stream2 && ctx->B >= 16;
      const int h = qsplit ? ctx->B / 2 : ctx->B;
      if (qsplit) {
        HIPCHK(hipEventRecord(ctx->fork_ev, st));
        HIPCHK(hipStreamWaitEvent(ctx->stream2, ctx->fork_ev, 0));
      }
      for (int stage = 0; stage < (n_qr2 > 0 ? 2 : 1); ++stage) {
        // rows of the longest matrix this stage factors (R^T: N x N)
        const int qrows = stage == 0 ? max_qr_l : max_qr_n;
        for (int p = 0; p < panels; ++p) {
          launch_qr_panel(b, s, u, stage, p, qrows - QB * p, 0, h, st);
          launch_qr_update(b, s, u, stage, p, panels - 1 - p, 0, h, st);
          if (qsplit) {
            launch_qr_panel(b, s, u, stage, p, qrows - QB * p, h,
                            ctx->B - h, ctx->stream2);
            launch_qr_update(b, s, u, stage, p, panels - 1 - p, h,
                             ctx->B - h, ctx->stream2);
          }
        }
        launch_qr_to_vectors(b, s, u, stage, max_qr_n, 0, h, st);
        if (qsplit)
          launch_qr_to_vectors(b, s, u, stage, max_qr_n, h, ctx->B - h,
                               ctx->stream2);
      }
      if (qsplit) {
        HIPCHK(hipEventRecord(ctx->join_ev, ctx->stream2));
        HIPCHK(hipStreamWaitEvent(st, ctx->join_ev, 0));
      }
      LAUNCHCHK(ctx);
    }
    // Sweep s is enqueued before the host waits for the rotation count of
    // sweep s-1, so the read-back overlaps the next sweep; a sweep enqueued
    // after convergence finds every chain done and exits at once.  f32:
    // the FP32 rounds of the mixed path (only its chains take part).
    auto run_sweeps = [&](bool f32, int nb_max, int cap,
                          bool &converged) -> hmps_status {
      converged = false;
      auto enqueue_sweep = [&](int sweep) -> hmps_status {
        launch_jacobi_sweep_begin(s, ctx->B, sweep, st);
        if (sweep == 0 && n_small > 0)
          launch_mark_small_done(b, s, u, ctx->small_max, st);
        for (int r = 0; r < nb_max - 1; ++r) {
          if (f32)
            launch_jacobi_round32(b, s, u, r, nb_max / 2, st);
          else
            launch_jacobi_round(b, s, u, r, nb_max / 2, max_len16, st);
        }
        ctx->stats.round_launches += std::max(0, nb_max - 1);
        // the chains on wide blocks: half the rounds per sweep
        // split only rounds of more than one workgroup per compute unit:
        // with fewer, every workgroup has a unit to itself and a second
        // dispatch per round only adds its launch (measured at 16 chains:
        // 144 and 192 workgroups lose 13% split, 288 and 384 gain 9-16%)
        if (!f32 && max_nbw > 0 && (ctx->split & 1) && ctx->stream2 &&
            ctx->B >= 2 && (max_nbw / 2) * ctx->B > 256) {
          const int h = ctx->B / 2;
          HIPCHK(hipEventRecord(ctx->fork_ev, st));
          HIPCHK(hipStreamWaitEvent(ctx->stream2, ctx->fork_ev, 0));
          for (int r = 0; r < max_nbw - 1; ++r) {
            launch_jacobi_round_wide(b, s, u, r, max_nbw / 2, 0, h, st);
            launch_jacobi_round_wide(b, s, u, r, max_nbw / 2, h,
                                     ctx->B - h, ctx->stream2);
          }
          HIPCHK(hipEventRecord(ctx->join_ev, ctx->stream2));
          HIPCHK(hipStreamWaitEvent(st, ctx->join_ev, 0));
          ctx->stats.round_launches += max_nbw - 1;
          ctx->stats.wide_launches += max_nbw - 1;
          ctx->stats.split_launches += max_nbw - 1;
        } else if (!f32 && max_nbw > 0) {
          for (int r = 0; r < max_nbw - 1; ++r)
            launch_jacobi_round_wide(b, s, u, r, max_nbw / 2, 0, ctx->B, st);
          ctx->stats.round_launches += max_nbw - 1;
          ctx->stats.wide_launches += max_nbw - 1;
        }
        ctx->stats.jacobi_sweeps += 1;
        if (f32) ctx->stats.jacobi_sweeps_fp32 += 1;
        int32_t *slot =
            ctx->h_stage + (size_t)(2 + (sweep & 1)) * ctx->opt.max_chains;
        HIPCHK(hipMemcpyAsync(slot, ctx->d_rot, sizeof(int32_t) * ctx->B,
                              hipMemcpyDeviceToHost, st));
        HIPCHK(hipEventRecord(ctx->sweep_ev[sweep & 1], st));
        return HMPS_OK;
      };
      // algorithmic bytes of the rounds: in every round a chain's block
      // pairs are read once and, in a sweep where the chain still rotates,
      // written once (its last, checking sweep only reads them)
      std::vector<double> round_bytes(ctx->B);
      std::vector<uint8_t> active(ctx->B, 1);
      for (int c = 0; c < ctx->B; ++c) {
        const int *row = &ctx->h_chi[(size_t)c * (L + 1)];
        const int nvec = 3 * std::min(row[k], row[k + 2]);
        const int len = 3 * std::max(row[k], row[k + 2]);
        const int path =
            svd_path(len, nvec, ctx->small_max, ctx->precond, mixed);
        int vlen = len, nv = nvec;
        double esz = 8.0;
        if (f32) {
          vlen = nvec;
          esz = 4.0;
        } else if (path == PATH_QR || path == PATH_QR2) {
          vlen = nvec;  // R^T or R2^T
        } else if (path_is_rr(path)) {
          nv = rr_vectors(nvec, chi_max);
          if (path == PATH_RR2) vlen = nvec;  // R^T W
        }
        const int jb = f32 ? JB : round_width(path, nv, wide);
        const int nb = n_blocks_even(nv, jb);
        const bool part = f32 ? path_is_rr(path) : path != PATH_SMALL;
        round_bytes[c] =
            part ? (double)(nb - 1) * nb * jb * vector_stride(vlen) * esz : 0.0;
      }
      hmps_status est = enqueue_sweep(0);
      if (est) return est;
      for (int sweep = 1; sweep <= cap; ++sweep) {
        if (sweep < cap) {
          est = enqueue_sweep(sweep);
          if (est) return est;
        }
        const int prev = (sweep - 1) & 1;
        HIPCHK(hipEventSynchronize(ctx->sweep_ev[prev]));
        const int32_t *slot =
            ctx->h_stage + (size_t)(2 + prev) * ctx->opt.max_chains;
        bool any = false;
        for (int c = 0; c < ctx->B; ++c) {
          if (active[c])
            ctx->stats.svd_bytes += round_bytes[c] * (slot[c] != 0 ? 2.0 : 1.0);
          active[c] = slot[c] != 0;
          any |= slot[c] != 0;
        }
        if (!any) {
          converged = true;
          break;
        }
      }
      // a sweep enqueued beyond convergence may still be in flight: the
      // next loop resets the flags it reads only after it (stream order)
      return HMPS_OK;
    };
    HIPCHK(hipEventRecord(ctx->svd_ev[0], st));
    bool converged = false;
    if (n_rr > 0) {
      // mixed path: FP32 rounds on R^T (their convergence to the FP32
      // tolerance is not required: the FP64 Ritz step takes whatever basis
      // they reach), then the FP64 Ritz basis and theta' W
      launch_rr_to32(b, s, u, st);
      hmps_status est = run_sweeps(true, max_nb32, RR_FP32_SWEEPS, converged);
      if (est) return est;
      launch_rr_stage2(b, s, u, max_rr_n, max_rr_l, st);
      LAUNCHCHK(ctx);
    }
    {
      hmps_status est = run_sweeps(false, max_nb, ctx->opt.max_sweeps,
                                   converged);
      if (est) return est;
    }
    if (!converged)
      return fail(ctx, HMPS_E_NUMERIC,
                  "Jacobi SVD did not converge within max_sweeps");
    HIPCHK(hipEventRecord(ctx->svd_ev[1], st));
    timed_svd = true;
  }
  launch_truncate(b, s, u, st);
  LAUNCHCHK(ctx);
  const int kmax = std::max(1, std::min(u.chi_max, max_nvec));
  launch_writeback(b, s, u, max_vlen, max_nvec, kmax,
                   (max_qr2_n + QB - 1) / QB, st);
  HIPCHK(hipGetLastError());
  if (ctx->defer_finish) {
    // the block batch of a U(1) update: that update reads the ranks and
    // error flags, and then the round time (finish_deferred)
    ctx->pending_time = timed_svd;
    ctx->pending_svd_flops = svd_flops;
    ctx->have_spectrum = true;
    ctx->stats.algo_flops += flops;
    ctx->stats.updates += ctx->B;
    return HMPS_OK;
  }
  HIPCHK(hipMemcpyAsync(ctx->h_stage, ctx->d_knew, sizeof(int32_t) * ctx->B,
                        hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(ctx->h_stage + ctx->opt.max_chains, ctx->d_err,
                        sizeof(int32_t) * ctx->B, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  for (int c = 0; c < ctx->B; ++c) {
    const int code = ctx->h_stage[ctx->opt.max_chains + c];
    if (code) {
      const int *row = &ctx->h_chi[(size_t)c * (L + 1)];
      const int m = 3 * row[k], n = 3 * row[k + 2];
      double sg[6] = {0, 0, 0, 0, 0, 0};
      (void)hipMemcpy(sg, ctx->d_sig2 + (size_t)c * ctx->n_cap,
                      sizeof(double) * std::min(n, 6), hipMemcpyDeviceToHost);
      char buf[512];
      std::snprintf(buf, sizeof buf,
                    "numerical failure (code %d: %s) in chain %d, update on "
                    "sites (%d,%d) op %d, theta %d x %d, update #%lld; "
                    "sigma^2[0..5] = %.3e %.3e %.3e %.3e %.3e %.3e",
                    code,
                    code == 1 ? "in-LDS Jacobi did not converge"
                              : "zero or non-finite singular values",
                    c, k, k + 1, op, m, n, (long long)ctx->stats.updates,
                    sg[0], sg[1], sg[2], sg[3], sg[4], sg[5]);
      return fail(ctx, HMPS_E_NUMERIC, buf);
    }
    const int kn = ctx->h_stage[c];
    ctx->h_chi[(size_t)c * (L + 1) + k + 1] = kn;
    ctx->stats.max_chi = std::max(ctx->stats.max_chi, kn);
  }
  if (timed_svd) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ctx->svd_ev[0], ctx->svd_ev[1]));
    ctx->stats.svd_seconds += 1e-3 * ms;
    ctx->stats.svd_flops += svd_flops;
  }
  ctx->have_spectrum = true;
  ctx->stats.algo_flops += flops;
  ctx->stats.updates += ctx->B;
  if (op >= 0) ctx->stats.gate_updates += ctx->B;
  if (is_move) ctx->stats.move_updates += ctx->B;
  return HMPS_OK;
}

// Charges of every bond after an initialisation: bond 0 carries 0; a
// cluster physical site opens its Bell pair (bond index s carries S^z(s) =
// 1 - s more), its ancilla closes it (-S^z: the pair carries 0), and an
// environment site in S^z label l adds 1 - l.  labels: [B][n_env].
void init_host_charges(hmps_ctx *ctx, const uint8_t *labels) {
  const Plan &P = ctx->plan;
  const int L = P.len;
  ctx->pos_sign.assign(L, 1);
  for (int p = 0; p < L; ++p)
    if (P.is_ancilla[p]) ctx->pos_sign[p] = -1;
  ctx->h_qg.assign((size_t)ctx->B * (L + 1), {});
  for (int c = 0; c < ctx->B; ++c) {
    auto *g = &ctx->h_qg[(size_t)c * (L + 1)];
    int q = 0;
    g[0] = {{0, 1}};
    for (int p = 0; p < L; ++p) {
      if (P.is_cluster[p] && !P.is_ancilla[p]) {
        g[p + 1] = {{q + 1, 1}, {q, 1}, {q - 1, 1}};
      } else if (P.is_ancilla[p]) {
        g[p + 1] = {{q, 1}};
      } else {
        q += 1 - labels[(size_t)c * P.n_env + P.env_index[p]];
        g[p + 1] = {{q, 1}};
      }
    }
  }
}

// The round time of a deferred update of the block batch, once its stream
// has been synchronised.
hmps_status finish_deferred(hmps_ctx *ctx, hmps_ctx *sub) {
  if (sub->pending_time) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, sub->svd_ev[0], sub->svd_ev[1]));
    sub->stats.svd_seconds += 1e-3 * ms;
    sub->stats.svd_flops += sub->pending_svd_flops;
    sub->pending_time = false;
  }
  return HMPS_OK;
}

// One U(1) update on (k, k+1) for every chain (Exploiting Conserved Quantum
// Numbers subsection): theta' of every chain as in the dense update; then
// its charge blocks, listed here from the charges of bonds k and k+2, are
// decomposed as the chains of the block batch (ctx->sub, in passes of at
// most max_blocks blocks), merged and truncated together per chain, and
// written back block by block; bond k+1 lists the kept vectors by block in
// ascending charge.
hmps_status do_update_u1(hmps_ctx *ctx, int k, int op, bool right,
                         int chi_max, double cutoff) {
  const int L = ctx->plan.len;
  const bool is_move = (op == OP_IDENT);
  hmps_ctx *sub = ctx->sub;
  // the sites at k and k+1 once the update is done (a swap exchanges them)
  int sk = ctx->pos_sign[k], sk1 = ctx->pos_sign[k + 1];
  if (op == OP_SWAP) std::swap(sk, sk1);
  struct Piece {
    int start = 0, count = 0;
  };
  struct Blk {
    int q = 0;
    Piece row[3], col[3];
  };
  std::vector<std::vector<Blk>> blocks(ctx->B);
  int max_chiL = 1, max_chiR = 1;
  double flops = 0.0;
  int64_t n_blocks = 0;
  size_t largest = 0;  // entries of the largest block theta'
  for (int c = 0; c < ctx->B; ++c) {
    const int *row = &ctx->h_chi[(size_t)c * (L + 1)];
    max_chiL = std::max(max_chiL, row[k]);
    max_chiR = std::max(max_chiR, row[k + 2]);
    flops += 18.0 * row[k] * row[k + 1] * row[k + 2] +
             162.0 * row[k] * row[k + 2];
    // rows (s1, a): charge q_k(a) + sk S^z(s1); columns (s2, c): q_{k+2}(c)
    // - sk1 S^z(s2); S^z(s) = 1 - s
    std::map<int, std::array<Piece, 3>> rows, cols;
    // each bond's runs: one per charge, covering its dimension exactly
    bool ok = true;
    int start = 0;
    for (const auto &g : ctx->h_qg[(size_t)c * (L + 1) + k]) {
      for (int s1 = 0; s1 < 3; ++s1) {
        Piece &pc = rows[g.first + sk * (1 - s1)][s1];
        ok = ok && pc.count == 0 && g.second > 0;
        pc = {start, g.second};
      }
      start += g.second;
    }
    ok = ok && start == row[k];
    start = 0;
    for (const auto &g : ctx->h_qg[(size_t)c * (L + 1) + k + 2]) {
      for (int s2 = 0; s2 < 3; ++s2) {
        Piece &pc = cols[g.first - sk1 * (1 - s2)][s2];
        ok = ok && pc.count == 0 && g.second > 0;
        pc = {start, g.second};
      }
      start += g.second;
    }
    ok = ok && start == row[k + 2];
    if (!ok)
      return fail(ctx, HMPS_E_NUMERIC,
                  "charges of bonds " + std::to_string(k) + " and " +
                      std::to_string(k + 2) + " of chain " +
                      std::to_string(c) + " do not match their dimensions");
    for (const auto &r : rows) {
      const auto it = cols.find(r.first);
      if (it == cols.end()) continue;
      Blk bk;
      bk.q = r.first;
      int mq = 0, nq = 0;
      for (int x = 0; x < 3; ++x) {
        bk.row[x] = r.second[x];
        bk.col[x] = it->second[x];
        mq += bk.row[x].count;
        nq += bk.col[x].count;
      }
      const double lq = std::max(mq, nq), nn = std::min(mq, nq);
      flops += 14.0 * lq * nn * nn + 8.0 * nn * nn * nn;
      int cl = 1, cr = 1;
      for (int x = 0; x < 3; ++x) {
        cl = std::max(cl, bk.row[x].count);
        cr = std::max(cr, bk.col[x].count);
      }
      largest = std::max(largest, (size_t)9 * cl * cr);
      blocks[c].push_back(bk);
    }
    n_blocks += (int64_t)blocks[c].size();
  }
  for (int c = 0; c < ctx->B; ++c)
    if ((int)blocks[c].size() > ctx->max_blocks)
      return fail(ctx, HMPS_E_NOMEM,
                  "chain " + std::to_string(c) + " has " +
                      std::to_string(blocks[c].size()) +
                      " charge blocks, more than max_blocks");
  const UpdParams u =
      update_params(ctx, k, op, right, chi_max, cutoff, 0, 0);
  Batch b = batch_of(ctx);
  UpdScratch s = scratch_of(ctx);
  hipStream_t st = ctx->stream;
  launch_theta(b, s, u, max_chiL, max_chiR, st);
  if (u.is_gate) launch_theta_norm(b, s, u, st);
  LAUNCHCHK(ctx);
  const int kmax = std::max(
      1, std::min(u.chi_max, 3 * std::max(max_chiL, max_chiR)));
  // The blocks take the in-LDS SVD only when all of them fit it: one
  // launch.  Otherwise every block joins the blocked rounds that the large
  // ones need anyway, where a small block costs a few more workgroups; the
  // in-LDS kernel beside them would add its own latency.  Measured with 64
  // chains on the 2x16 ladder at chi 256: 3574 -> 3817 gate applications/s;
  // on the 2x3 ladder (every block small, one chain) the in-LDS path is
  // 1.8x faster than the rounds.
  sub->small_max = largest <= ctx->small_max ? ctx->small_max : 0;
  std::vector<std::vector<std::pair<int, int>>> newg(ctx->B);
  bool single = true;  // one pass: its read-back is the update's last sync
  for (int c0 = 0; c0 < ctx->B;) {
    // the chains c0 .. c1-1 whose blocks fit one pass
    int nb = 0, c1 = c0;
    while (c1 < ctx->B && nb + (int)blocks[c1].size() <= ctx->max_blocks)
      nb += (int)blocks[c1++].size();
    if (c1 < ctx->B) single = false;
    // the block table, then the chain table, in pinned memory: one copy
    int32_t *tb = ctx->h_u1_tab;
    int32_t *tc = tb + (size_t)nb * U1_BLK;
    sub->h_chi.assign((size_t)std::max(nb, 1) * 3, 1);
    int v = 0;
    for (int c = c0; c < c1; ++c) {
      int32_t *t = &tc[(size_t)(c - c0) * U1_CH];
      t[0] = c;
      t[1] = v;
      t[2] = (int32_t)blocks[c].size();
      t[3] = 0;
      for (const Blk &bk : blocks[c]) {
        int32_t *e = &tb[(size_t)v * U1_BLK];
        int cl = 1, cr = 1;
        for (int x = 0; x < 3; ++x) {
          cl = std::max(cl, bk.row[x].count);
          cr = std::max(cr, bk.col[x].count);
          e[4 + x] = bk.row[x].start;
          e[7 + x] = bk.row[x].count;
          e[10 + x] = bk.col[x].start;
          e[13 + x] = bk.col[x].count;
        }
        e[0] = c - c0;
        e[1] = bk.q;
        e[2] = cl;
        e[3] = cr;
        sub->h_chi[(size_t)v * 3] = cl;
        sub->h_chi[(size_t)v * 3 + 2] = cr;
        ++v;
      }
    }
    const size_t n_tab = (size_t)nb * U1_BLK + (size_t)(c1 - c0) * U1_CH;
    HIPCHK(hipMemcpyAsync(ctx->d_u1_blk, tb, sizeof(int32_t) * n_tab,
                          hipMemcpyHostToDevice, st));
    U1Args a;
    a.blk = ctx->d_u1_blk;
    a.chains = ctx->d_u1_blk + (size_t)nb * U1_BLK;
    a.n_chains = c1 - c0;
    a.n_blocks = nb;
    a.k = k;
    a.right = right ? 1 : 0;
    a.bchi = sub->d_chi;
    a.berr = sub->d_err;
    a.bdisc = sub->d_disc;
    a.blogw = sub->d_logw;
    a.bsites = sub->d_sites;
    a.bsite_cap = sub->site_cap;
    a.bTH = sub->d_TH;
    a.bX = sub->d_X;
    a.bstride = sub->th_stride;
    a.bsig = sub->d_sig;
    a.bknew = sub->d_knew;
    a.bn_cap = sub->n_cap;
    a.kv = ctx->d_u1_kv;
    a.scale = ctx->d_u1_scale;
    a.jmap = ctx->d_u1_jmap;
    a.jstride = ctx->n_cap;
    launch_u1_gather(b, s, a, st);
    LAUNCHCHK(ctx);
    if (nb > 0) {
      // every block keeps all it resolves; the merge truncates
      sub->B = nb;
      sub->width_batch = ctx->B;
      sub->defer_finish = true;
      const hmps_status e =
          do_update(sub, 0, OP_SWAP, right, sub->opt.chi_cap, 0.0);
      sub->defer_finish = false;
      if (e) return fail(ctx, e, "charge block SVD: " + sub->err);
    }
    launch_u1_merge(b, s, u, a, st);
    launch_u1_scatter(b, a, max_chiL, max_chiR, kmax, st);
    HIPCHK(hipGetLastError());
    if (nb > 0) {
      HIPCHK(hipMemcpyAsync(ctx->h_u1_kv, ctx->d_u1_kv, sizeof(int32_t) * nb,
                            hipMemcpyDeviceToHost, st));
      HIPCHK(hipMemcpyAsync(ctx->h_u1_err, sub->d_err, sizeof(int32_t) * nb,
                            hipMemcpyDeviceToHost, st));
    }
    if (single) {
      HIPCHK(hipMemcpyAsync(ctx->h_stage, ctx->d_knew,
                            sizeof(int32_t) * ctx->B, hipMemcpyDeviceToHost,
                            st));
      HIPCHK(hipMemcpyAsync(ctx->h_stage + ctx->opt.max_chains, ctx->d_err,
                            sizeof(int32_t) * ctx->B, hipMemcpyDeviceToHost,
                            st));
    }
    HIPCHK(hipStreamSynchronize(st));
    if (nb > 0) {
      hmps_status e = finish_deferred(ctx, sub);
      if (e) return e;
    }
    for (int w = 0; w < nb; ++w)
      if (ctx->h_u1_err[w])
        return fail(ctx, HMPS_E_NUMERIC,
                    std::string("charge block SVD: ") +
                        (ctx->h_u1_err[w] == 1
                             ? "in-LDS Jacobi did not converge"
                             : "zero or non-finite singular values"));
    v = 0;
    for (int c = c0; c < c1; ++c)
      for (const Blk &bk : blocks[c]) {
        const int kv = ctx->h_u1_kv[v++];
        if (kv > 0) newg[c].push_back({bk.q, kv});
      }
    c0 = c1;
  }
  if (!single) {
    HIPCHK(hipMemcpyAsync(ctx->h_stage, ctx->d_knew, sizeof(int32_t) * ctx->B,
                          hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->h_stage + ctx->opt.max_chains, ctx->d_err,
                          sizeof(int32_t) * ctx->B, hipMemcpyDeviceToHost,
                          st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int c = 0; c < ctx->B; ++c) {
    const int code = ctx->h_stage[ctx->opt.max_chains + c];
    const int kn = ctx->h_stage[c];
    int sum = 0;
    for (const auto &g : newg[c]) sum += g.second;
    if (code || sum != kn)
      return fail(ctx, HMPS_E_NUMERIC,
                  "U(1) update on sites (" + std::to_string(k) + "," +
                      std::to_string(k + 1) + ") failed in chain " +
                      std::to_string(c) + ": " +
                      (code == 3 ? "more charge blocks or singular values "
                                   "than the merge holds"
                       : code    ? "zero or non-finite singular values"
                                 : "block counts do not add up"));
    ctx->h_chi[(size_t)c * (L + 1) + k + 1] = kn;
    ctx->h_qg[(size_t)c * (L + 1) + k + 1] = newg[c];
    ctx->stats.max_chi = std::max(ctx->stats.max_chi, kn);
  }
  ctx->pos_sign[k] = sk;
  ctx->pos_sign[k + 1] = sk1;
  ctx->have_spectrum = true;
  ctx->stats.algo_flops += flops;
  ctx->stats.updates += ctx->B;
  if (op >= 0) ctx->stats.gate_updates += ctx->B;
  if (is_move) ctx->stats.move_updates += ctx->B;
  ctx->u1_blocks += n_blocks;
  return HMPS_OK;
}

hmps_status move_center(hmps_ctx *ctx, int target) {
  while (ctx->center < target) {
    hmps_status st = do_update(ctx, ctx->center, OP_IDENT, true, 0, 0.0);
    if (st) return st;
    ctx->center += 1;
  }
  while (ctx->center > target) {
    hmps_status st = do_update(ctx, ctx->center - 1, OP_IDENT, false, 0, 0.0);
    if (st) return st;
    ctx->center -= 1;
  }
  return HMPS_OK;
}

}  // namespace

// =====================================================================
// ABI
// =====================================================================
extern "C" {

size_t hmps_workspace_bytes(int32_t max_chains, int32_t max_sites,
                            int32_t chi_cap, int32_t max_bonds) {
  if (max_chains < 1 || max_sites < 1 || chi_cap < 1 || max_bonds < 0)
    return 0;
  return carve(nullptr, nullptr, max_chains, max_sites, chi_cap, max_bonds);
}

}  // extern "C"

namespace {
// charge blocks the block batch holds: max_blocks, or 16 per chain and at
// least 64 (the blocks of one chain's update must fit one pass; on the
// 2x16 ladder at chi 256 an update has up to about 15 per chain, and
// every pass is a sweep loop of its own)
int u1_blocks_of(int32_t symmetry, int32_t max_chains, int32_t max_blocks) {
  if (symmetry != HMPS_SYM_U1) return 0;
  return max_blocks > 0 ? max_blocks
                        : std::min(65535, std::max(64, 16 * max_chains));
}
}  // namespace

extern "C" {

size_t hmps_workspace_bytes_sym(int32_t max_chains, int32_t max_sites,
                                int32_t chi_cap, int32_t max_bonds,
                                int32_t symmetry, int32_t max_blocks) {
  if (max_chains < 1 || max_sites < 1 || chi_cap < 1 || max_bonds < 0 ||
      (symmetry != HMPS_SYM_NONE && symmetry != HMPS_SYM_U1) ||
      max_blocks < 0 || max_blocks > 65535)
    return 0;
  return carve(nullptr, nullptr, max_chains, max_sites, chi_cap, max_bonds,
               u1_blocks_of(symmetry, max_chains, max_blocks));
}

}  // extern "C"

namespace {
hmps_status create_ctx(hmps_ctx **out, const hmps_options *opt,
                       bool svd_only) {
  if (!out || !opt) return HMPS_E_INVALID;
  *out = nullptr;
  // chi_cap >= 3: a Bell pair carries a bond of dimension 3; chi_cap <= 640:
  // the truncation sorts at most 2048 singular values (3 chi_cap <= 1920);
  // max_chains <= 65535: the chain index is grid.y or grid.z of launches
  if (opt->max_chains < 1 || opt->max_chains > 65535 || opt->max_sites < 1 ||
      opt->chi_cap < 3 ||
      opt->max_bonds < 0 || opt->chi_cap > 640 ||
      (opt->precision != HMPS_PREC_FP64 &&
       opt->precision != HMPS_PREC_MIXED_FP32))
    return HMPS_E_INVALID;  // HMPS_PREC_MIXED_BF16X3 included: not built
  if ((opt->symmetry != HMPS_SYM_NONE && opt->symmetry != HMPS_SYM_U1) ||
      (opt->symmetry == HMPS_SYM_U1 && opt->precision != HMPS_PREC_FP64) ||
      opt->max_blocks < 0 || opt->max_blocks > 65535)
    return HMPS_E_INVALID;
  const int max_blocks =
      u1_blocks_of(opt->symmetry, opt->max_chains, opt->max_blocks);
  const size_t need =
      carve(nullptr, nullptr, opt->max_chains, opt->max_sites, opt->chi_cap,
            opt->max_bonds, max_blocks, svd_only);
  if (!opt->workspace || opt->workspace_bytes < need) return HMPS_E_NOMEM;
  if (((uintptr_t)opt->workspace) % ALIGN) return HMPS_E_INVALID;
  hmps_ctx *ctx = new hmps_ctx();
  ctx->opt = *opt;
  // A dense theta' with a graded spectrum (sigma_j = exp(-j/40), 1536 x
  // 1536) needs 63 sweeps; updates of the 2x16 ladder at chi 256 average
  // about 16.
  if (ctx->opt.max_sweeps <= 0) ctx->opt.max_sweeps = 100;
  if (!(ctx->opt.jacobi_tol > 0.0)) {
    // relative orthogonality reachable with rounded inner products of
    // length 3 chi_cap: a few sqrt(m) eps
    ctx->opt.jacobi_tol = 8.0 * std::sqrt(3.0 * opt->chi_cap) * 2.220446e-16;
  }
  ctx->stream = reinterpret_cast<hipStream_t>(opt->stream);
  DeviceGuard guard(opt->device);
  if (const char *e = std::getenv("HMPS_SYNC_DEBUG")) ctx->sync_debug = e[0] == '1';
  if (const char *e = std::getenv("HMPS_INNER")) ctx->inner_sweeps = std::max(1, std::atoi(e));
  if (const char *e = std::getenv("HMPS_SKIP")) ctx->skip = std::min(1e-26, std::atof(e));
  if (const char *e = std::getenv("HMPS_CROSS")) ctx->cross_inner = e[0] == '1';
  if (const char *e = std::getenv("HMPS_SPLIT"))
    ctx->split = std::max(0, std::min(3, std::atoi(e)));
  if (const char *e = std::getenv("HMPS_WIDE"))
    ctx->wide = e[0] == '0' ? 0 : (e[0] == '1' ? 1 : -1);
  if (const char *e = std::getenv("HMPS_QR"))
    ctx->precond = std::max(0, std::min(2, std::atoi(e)));
  if (const char *e = std::getenv("HMPS_SMALL_MAX"))
    ctx->small_max = std::min<size_t>(SMALL_LDS, std::strtoull(e, nullptr, 10));
  int current = -1;
  hipError_t e = hipGetDevice(&current);
  if (e != hipSuccess || current != opt->device) {
    delete ctx;
    return HMPS_E_DEVICE;
  }
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&ctx->sweep_ev[i], hipEventDisableTiming);
  for (int i = 0; i < 2 && e == hipSuccess; ++i)
    e = hipEventCreate(&ctx->svd_ev[i]);
  if (e == hipSuccess)
    e = hipStreamCreateWithFlags(&ctx->stream2, hipStreamNonBlocking);
  if (e == hipSuccess)
    e = hipEventCreateWithFlags(&ctx->fork_ev, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipEventCreateWithFlags(&ctx->join_ev, hipEventDisableTiming);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&ctx->h_stage,
                    sizeof(int32_t) * 4 * opt->max_chains);
  if (e != hipSuccess) {
    hmps_destroy(ctx);  // releases what was created so far
    return HMPS_E_DEVICE;
  }
  carve(ctx, reinterpret_cast<char *>(opt->workspace), opt->max_chains,
        opt->max_sites, opt->chi_cap, opt->max_bonds, max_blocks, svd_only);
  if (max_blocks > 0) {
    // the block batch: a context of max_blocks two-site chains on the
    // tail of the workspace, with the same SVD settings
    ctx->symmetry = HMPS_SYM_U1;
    ctx->max_blocks = max_blocks;
    hmps_options so{};
    so.device = opt->device;
    so.stream = opt->stream;
    so.workspace = reinterpret_cast<char *>(opt->workspace) + ctx->u1_sub_off;
    so.workspace_bytes = ctx->u1_sub_bytes;
    so.max_chains = max_blocks;
    so.max_sites = 2;
    so.chi_cap = opt->chi_cap;
    so.max_bonds = 0;
    so.precision = HMPS_PREC_FP64;
    so.max_sweeps = ctx->opt.max_sweeps;
    so.jacobi_tol = ctx->opt.jacobi_tol;
    hmps_status e2 = create_ctx(&ctx->sub, &so, true);
    if (e2 == HMPS_OK &&
        (hipHostMalloc((void **)&ctx->h_u1_kv,
                       sizeof(int32_t) * max_blocks) != hipSuccess ||
         hipHostMalloc((void **)&ctx->h_u1_err,
                       sizeof(int32_t) * max_blocks) != hipSuccess ||
         hipHostMalloc((void **)&ctx->h_u1_tab,
                       sizeof(int32_t) * ((size_t)max_blocks * U1_BLK +
                                          (size_t)opt->max_chains * U1_CH)) !=
             hipSuccess))
      e2 = HMPS_E_DEVICE;
    if (e2 == HMPS_OK &&
        (hipMemsetAsync(ctx->sub->d_sweeps, 0, sizeof(int32_t) * max_blocks,
                        ctx->stream) != hipSuccess ||
         hipStreamSynchronize(ctx->stream) != hipSuccess))
      e2 = HMPS_E_DEVICE;
    if (e2 != HMPS_OK) {
      hmps_destroy(ctx);
      return e2;
    }
    Plan P;
    P.len = 2;
    ctx->sub->plan = P;
    ctx->sub->skip_theta = true;
    ctx->sub->zero_ok = true;
  }
  *out = ctx;
  return HMPS_OK;
}
}  // namespace

extern "C" {

hmps_status hmps_create(hmps_ctx **out, const hmps_options *opt) {
  return create_ctx(out, opt, false);
}

void hmps_destroy(hmps_ctx *ctx) {
  if (!ctx) return;
  DeviceGuard guard(ctx->opt.device);
  (void)hipStreamSynchronize(ctx->stream);
  if (ctx->h_stage) (void)hipHostFree(ctx->h_stage);
  if (ctx->h_u1_kv) (void)hipHostFree(ctx->h_u1_kv);
  if (ctx->h_u1_err) (void)hipHostFree(ctx->h_u1_err);
  if (ctx->h_u1_tab) (void)hipHostFree(ctx->h_u1_tab);
  if (ctx->sub) hmps_destroy(ctx->sub);
  for (hipEvent_t ev : ctx->sweep_ev)
    if (ev) (void)hipEventDestroy(ev);
  for (hipEvent_t ev : ctx->svd_ev)
    if (ev) (void)hipEventDestroy(ev);
  if (ctx->stream2) {
    (void)hipStreamSynchronize(ctx->stream2);
    (void)hipStreamDestroy(ctx->stream2);
  }
  if (ctx->fork_ev) (void)hipEventDestroy(ctx->fork_ev);
  if (ctx->join_ev) (void)hipEventDestroy(ctx->join_ev);
  delete ctx;
}

const char *hmps_last_error(const hmps_ctx *ctx) {
  return ctx ? ctx->err.c_str() : "null context";
}

hmps_status hmps_init_cluster_env(hmps_ctx *ctx, const hmps_lattice *lat,
                                  int32_t n_chains, uint64_t seed,
                                  const uint8_t *env_state, int32_t basis) {
  return hmps_init_cluster_env_at(ctx, lat, n_chains, seed, 0, 0, env_state,
                                  basis);
}

hmps_status hmps_init_cluster_env_at(hmps_ctx *ctx, const hmps_lattice *lat,
                                     int32_t n_chains, uint64_t seed,
                                     uint64_t chain_offset, int64_t sample,
                                     const uint8_t *env_state, int32_t basis) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (sample < 0)
    return fail(ctx, HMPS_E_INVALID, "sample must be >= 0");
  if (chain_offset > UINT64_MAX - (uint64_t)std::max(n_chains, 0))
    return fail(ctx, HMPS_E_INVALID, "chain_offset + n_chains overflows");
  Plan P;
  std::string why = validate_and_plan(lat, P);
  if (!why.empty()) return fail(ctx, HMPS_E_INVALID, why);
  if (n_chains < 1 || n_chains > ctx->opt.max_chains)
    return fail(ctx, HMPS_E_INVALID, "n_chains outside [1, max_chains]");
  if (P.len > ctx->opt.max_sites)
    return fail(ctx, HMPS_E_INVALID, "MPS length exceeds max_sites");
  if (P.n_bonds > ctx->opt.max_bonds)
    return fail(ctx, HMPS_E_INVALID, "n_bonds exceeds max_bonds");
  if (basis != 0 && basis != 1)
    return fail(ctx, HMPS_E_INVALID, "basis must be 0 or 1");
  if (basis != 0 && ctx->symmetry == HMPS_SYM_U1)
    return fail(ctx, HMPS_E_INVALID,
                "a U(1) context takes environment states in S^z (basis 0)");
  std::vector<uint8_t> labels((size_t)n_chains * std::max(P.n_env, 1), 0);
  if (env_state) {
    for (size_t i = 0; i < (size_t)n_chains * P.n_env; ++i) {
      if (env_state[i] > 2)
        return fail(ctx, HMPS_E_INVALID, "environment label > 2");
      labels[i] = env_state[i];
    }
  } else {
    basis = 0;
    // counter (global chain id, sample, MPS position, purpose 0)
    for (int c = 0; c < n_chains; ++c)
      for (int e = 0; e < P.n_env; ++e) {
        const uint64_t x = philox0(chain_offset + (uint64_t)c,
                                   (uint64_t)sample, (uint64_t)P.env_pos[e],
                                   0, seed, 0);
        const double u = (double)(x >> 11) * (1.0 / 9007199254740992.0);
        labels[(size_t)c * P.n_env + e] =
            (uint8_t)std::min(2, (int)std::floor(3.0 * u));
      }
  }
  ctx->plan = P;
  ctx->B = n_chains;
  ctx->seed = seed;
  ctx->chain0 = chain_offset;
  ctx->sample = sample;
  ctx->center = 0;
  ctx->evo_pos = 0;
  ctx->have_spectrum = false;
  ctx->ready = false;
  ctx->bond_loaded = false;
  std::memset(&ctx->stats, 0, sizeof(ctx->stats));
  hipStream_t s = ctx->stream;
  std::vector<int32_t> bp(P.bond_p), bq(P.bond_q);
  if (P.n_bonds > 0) {
    HIPCHK(hipMemcpyAsync(ctx->d_bond_p, bp.data(), sizeof(int32_t) * P.n_bonds,
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_bond_q, bq.data(), sizeof(int32_t) * P.n_bonds,
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_bond_J, P.bond_J.data(),
                          sizeof(double) * P.n_bonds, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipMemcpyAsync(ctx->d_is_cluster, P.is_cluster.data(),
                        sizeof(int32_t) * P.len, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_is_ancilla, P.is_ancilla.data(),
                        sizeof(int32_t) * P.len, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_env_index, P.env_index.data(),
                        sizeof(int32_t) * P.len, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_labels, labels.data(), labels.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(ctx->d_disc, 0, sizeof(double) * n_chains, s));
  HIPCHK(hipMemsetAsync(ctx->d_err, 0, sizeof(int32_t) * n_chains, s));
  HIPCHK(hipMemsetAsync(ctx->d_sweeps, 0, sizeof(int32_t) * n_chains, s));
  // new chains start with no accumulated moments
  launch_fill(ctx->d_mom, (size_t)n_chains * (P.n_bonds + 1) * 3, 0.0, s);
  Batch b = batch_of(ctx);
  InitArgs ia;
  ia.is_cluster = ctx->d_is_cluster;
  ia.is_ancilla = ctx->d_is_ancilla;
  ia.env_index = ctx->d_env_index;
  ia.labels = ctx->d_labels;
  ia.n_env = P.n_env;
  ia.basis = basis;
  launch_init(b, ia, ctx->d_logw, s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  init_host_chi(ctx);
  ctx->u1_live = ctx->symmetry == HMPS_SYM_U1;
  ctx->u1_blocks = 0;
  if (ctx->u1_live) {
    init_host_charges(ctx, labels.data());
    std::memset(&ctx->sub->stats, 0, sizeof(ctx->sub->stats));
    HIPCHK(hipMemsetAsync(ctx->sub->d_sweeps, 0,
                          sizeof(int32_t) * ctx->max_blocks, s));
    HIPCHK(hipStreamSynchronize(s));
  }
  ctx->stats.n_chains = n_chains;
  ctx->stats.n_sites = P.len;
  ctx->stats.n_env = P.n_env;
  ctx->stats.sample = sample;
  ctx->ready = true;
  return HMPS_OK;
}

// Validates the parameters of an evolution and returns its number of
// Trotter steps M = beta / (2 tau).
static hmps_status evolve_steps(hmps_ctx *ctx, double beta, double tau,
                                int32_t chi_max, double cutoff, int &M) {
  if (!(std::isfinite(beta) && beta >= 0.0))
    return fail(ctx, HMPS_E_INVALID, "beta must be finite and >= 0");
  if (chi_max < 1 || chi_max > ctx->opt.chi_cap)
    return fail(ctx, HMPS_E_INVALID, "chi_max outside [1, chi_cap]");
  if (!(cutoff >= 0.0) || !std::isfinite(cutoff))
    return fail(ctx, HMPS_E_INVALID, "cutoff must be finite and >= 0");
  M = 0;
  if (beta > 0.0) {
    if (!(tau > 0.0) || !std::isfinite(tau))
      return fail(ctx, HMPS_E_INVALID, "tau must be > 0");
    const double m = beta / (2.0 * tau);
    if (!(m < 1e9)) return fail(ctx, HMPS_E_INVALID, "beta/(2 tau) too large");
    M = (int)std::llround(m);
    if (std::fabs(m - M) > 1e-9 * std::max(1.0, m) || M < 1)
      return fail(ctx, HMPS_E_INVALID, "beta/(2 tau) must be an integer");
  }
  return HMPS_OK;
}

// Updates [first, first + count) of the update list of one evolution
// (M Trotter steps of the schedule), with the centre moves they need; the
// centre goes to site 0 once the last update of the list is done.
static hmps_status evolve_part(hmps_ctx *ctx, double beta, double tau,
                               int32_t chi_max, double cutoff, int M,
                               int64_t first, int64_t count) {
  hmps_status st = HMPS_OK;
  const auto t0 = std::chrono::steady_clock::now();
  const Plan &P = ctx->plan;
  const int ncoup = (int)P.couplings.size();
  std::vector<double> g((size_t)(ncoup + 2) * 81);
  for (int j = 0; j < ncoup; ++j) gate9(P.couplings[j], tau / 2.0, &g[81 * j]);
  swap9(&g[81 * ncoup]);
  for (int i = 0; i < 81; ++i) g[81 * (ncoup + 1) + i] = (i % 10 == 0) ? 1.0 : 0.0;
  HIPCHK(hipMemcpyAsync(ctx->d_gates, g.data(), sizeof(double) * g.size(),
                        hipMemcpyHostToDevice, ctx->stream));
  const int steplen = (int)P.step_k.size();
  const int64_t total = (int64_t)M * steplen;
  ctx->evo_beta = beta;
  ctx->evo_tau = tau;
  ctx->evo_chi = chi_max;
  ctx->evo_cutoff = cutoff;
  for (int64_t t = first; t < first + count; ++t) {
    const int k = P.step_k[t % steplen], op = P.step_op[t % steplen];
    const int kn = (t + 1 < total) ? P.step_k[(t + 1) % steplen] : 0;
    if (ctx->center < k) {
      st = move_center(ctx, k);
    } else if (ctx->center > k + 1) {
      st = move_center(ctx, k + 1);
    }
    if (st) return st;
    const bool right = kn >= k;
    st = do_update(ctx, k, op, right, chi_max, cutoff);
    if (st) return st;
    ctx->center = right ? k + 1 : k;
    ctx->evo_pos = t + 1;
    if (ctx->opt.progress && (t + 1) % steplen == 0)
      ctx->opt.progress(ctx->opt.progress_user, (t + 1) / steplen, M);
  }
  if (first + count == total) {
    st = move_center(ctx, 0);
    if (st) return st;
    ctx->evo_pos = 0;
  }
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->stats.evolve_seconds +=
      std::chrono::duration<double>(std::chrono::steady_clock::now() - t0)
          .count();
  return HMPS_OK;
}

hmps_status hmps_evolve(hmps_ctx *ctx, double beta, double tau,
                        int32_t chi_max, double cutoff) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  int M = 0;
  st = evolve_steps(ctx, beta, tau, chi_max, cutoff, M);
  if (st) return st;
  if (ctx->evo_pos != 0)
    return fail(ctx, HMPS_E_STATE,
                "an evolution applied in parts is not finished");
  const int64_t total = (int64_t)M * (int64_t)ctx->plan.step_k.size();
  return evolve_part(ctx, beta, tau, chi_max, cutoff, M, 0, total);
}

hmps_status hmps_evolve_updates(hmps_ctx *ctx, double beta, double tau,
                                int32_t chi_max, double cutoff, int64_t first,
                                int64_t count) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  int M = 0;
  st = evolve_steps(ctx, beta, tau, chi_max, cutoff, M);
  if (st) return st;
  const int64_t total = (int64_t)M * (int64_t)ctx->plan.step_k.size();
  if (first < 0 || count < 0 || first > total || count > total - first)
    return fail(ctx, HMPS_E_INVALID, "update range outside the evolution");
  if (first != ctx->evo_pos)
    return fail(ctx, HMPS_E_STATE,
                "updates must follow the last one applied (first = " +
                    std::to_string(ctx->evo_pos) + ")");
  if (first > 0 && (beta != ctx->evo_beta || tau != ctx->evo_tau ||
                    chi_max != ctx->evo_chi || cutoff != ctx->evo_cutoff))
    return fail(ctx, HMPS_E_INVALID,
                "parameters differ from those the evolution started with");
  return evolve_part(ctx, beta, tau, chi_max, cutoff, M, first, count);
}

hmps_status hmps_last_spectrum(hmps_ctx *ctx, int32_t cap, int32_t *rank,
                               double *sigma) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!ctx->have_spectrum)
    return fail(ctx, HMPS_E_STATE, "no two-site update since initialisation");
  if (!rank || cap < 0 || (cap > 0 && !sigma))
    return fail(ctx, HMPS_E_INVALID, "bad output arrays");
  hipStream_t s = ctx->stream;
  HIPCHK(hipMemcpyAsync(rank, ctx->d_knew, sizeof(int32_t) * ctx->B,
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  for (int c = 0; c < ctx->B; ++c) {
    const int n = std::min(cap, (int)rank[c]);
    if (n > 0)
      HIPCHK(hipMemcpyAsync(sigma + (size_t)c * cap,
                            ctx->d_sig + (size_t)c * ctx->n_cap,
                            sizeof(double) * n, hipMemcpyDeviceToHost, s));
  }
  HIPCHK(hipStreamSynchronize(s));
  return HMPS_OK;
}

hmps_status hmps_measure(hmps_ctx *ctx, uint32_t what, double *energy,
                         double *bond_ss, double *logw, double *qn) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (what & ~(uint32_t)(HMPS_MEASURE_ALL | HMPS_MEASURE_ACCUMULATE))
    return fail(ctx, HMPS_E_INVALID, "unknown bits in what");
  const bool accumulate = (what & HMPS_MEASURE_ACCUMULATE) != 0;
  if (!(what & HMPS_MEASURE_ENERGY)) energy = nullptr;
  if (!(what & HMPS_MEASURE_BONDS)) bond_ss = nullptr;
  if (!(what & HMPS_MEASURE_LOGW)) logw = nullptr;
  if (!(what & HMPS_MEASURE_QN)) qn = nullptr;
  const Plan &P = ctx->plan;
  hipStream_t s = ctx->stream;
  const size_t B = ctx->B;
  // the log-weights need no contraction
  if (!accumulate && !energy && !qn && !(bond_ss && P.n_bonds > 0)) {
    if (logw)
      HIPCHK(hipMemcpyAsync(logw, ctx->d_logw, sizeof(double) * B,
                            hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    return HMPS_OK;
  }
  if (ctx->center != 0) {
    st = move_center(ctx, 0);
    if (st) return st;
  }
  Batch b = batch_of(ctx);
  MeasureArgs ma;
  ma.bond_p = ctx->d_bond_p;
  ma.bond_q = ctx->d_bond_q;
  ma.bond_J = ctx->d_bond_J;
  ma.n_bonds = P.n_bonds;
  ma.is_ancilla = ctx->d_is_ancilla;
  ma.envs = ctx->d_envs;
  ma.wsz = ctx->d_wsz;
  ma.bond_scratch = ctx->d_bscr;
  ma.slots = ctx->slots;
  ma.chi2 = ctx->chi2;
  ma.norm = ctx->d_norm;
  ma.bond_ss = ctx->d_bond_ss;
  launch_measure_envs(b, ma, s);
  if (energy || bond_ss || accumulate)
    for (int b0 = 0; b0 < P.n_bonds; b0 += ctx->slots)
      launch_measure_bonds(b, ma, b0, std::min(ctx->slots, P.n_bonds - b0), s);
  launch_measure_finish(b, ma, ctx->d_energy, ctx->d_qn, s);
  if (accumulate)
    launch_moments_add(ctx->d_bond_ss, ctx->d_energy, ctx->d_mom, (int)B,
                       P.n_bonds, s);
  HIPCHK(hipGetLastError());
  if (energy)
    HIPCHK(hipMemcpyAsync(energy, ctx->d_energy, sizeof(double) * B,
                          hipMemcpyDeviceToHost, s));
  if (bond_ss && P.n_bonds > 0)
    HIPCHK(hipMemcpyAsync(bond_ss, ctx->d_bond_ss,
                          sizeof(double) * B * P.n_bonds,
                          hipMemcpyDeviceToHost, s));
  if (logw)
    HIPCHK(hipMemcpyAsync(logw, ctx->d_logw, sizeof(double) * B,
                          hipMemcpyDeviceToHost, s));
  if (qn)
    HIPCHK(hipMemcpyAsync(qn, ctx->d_qn, sizeof(double) * B,
                          hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return HMPS_OK;
}

hmps_status hmps_moments_reset(hmps_ctx *ctx) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  hipStream_t s = ctx->stream;
  launch_fill(ctx->d_mom, (size_t)ctx->B * (ctx->plan.n_bonds + 1) * 3, 0.0,
              s);
  HIPCHK(hipGetLastError());
  HIPCHK(hipStreamSynchronize(s));
  return HMPS_OK;
}

hmps_status hmps_bond_moments(hmps_ctx *ctx, int64_t *n_samples,
                              double *bond_mean, double *bond_var,
                              double *energy_mean_var) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!n_samples)
    return fail(ctx, HMPS_E_INVALID, "n_samples must not be NULL");
  const int nb = ctx->plan.n_bonds;
  if (nb > 0 && (!bond_mean || !bond_var))
    return fail(ctx, HMPS_E_INVALID, "bond_mean and bond_var must not be NULL");
  hipStream_t s = ctx->stream;
  launch_moments_reduce(ctx->d_mom, ctx->d_mom_out, ctx->B, nb, s);
  HIPCHK(hipGetLastError());
  std::vector<double> h((size_t)(nb + 1) * 3);
  HIPCHK(hipMemcpyAsync(h.data(), ctx->d_mom_out, sizeof(double) * h.size(),
                        hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double n = h[3 * nb];
  if (n < 2.0)
    return fail(ctx, HMPS_E_STATE,
                "fewer than two measurements accumulated (hmps_measure with "
                "HMPS_MEASURE_ACCUMULATE)");
  *n_samples = (int64_t)n;
  for (int e = 0; e < nb; ++e) {
    bond_mean[e] = h[3 * e + 1];
    bond_var[e] = h[3 * e + 2] / (n - 1.0);
  }
  if (energy_mean_var) {
    energy_mean_var[0] = h[3 * nb + 1];
    energy_mean_var[1] = h[3 * nb + 2] / (n - 1.0);
  }
  return HMPS_OK;
}

hmps_status hmps_collapse_resample(hmps_ctx *ctx, int32_t basis,
                                   uint8_t *env_out) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (basis != 0 && basis != 1)
    return fail(ctx, HMPS_E_INVALID, "basis must be 0 or 1");
  if (basis != 0 && ctx->u1_live)
    return fail(ctx, HMPS_E_INVALID,
                "a U(1) context collapses in S^z (basis 0): an S^x outcome "
                "has no definite charge");
  if (ctx->center != 0) {
    st = move_center(ctx, 0);
    if (st) return st;
  }
  const Plan &P = ctx->plan;
  Batch b = batch_of(ctx);
  hipStream_t s = ctx->stream;
  CollapseArgs ca;
  ca.is_cluster = ctx->d_is_cluster;
  ca.env_index = ctx->d_env_index;
  ca.n_env = P.n_env;
  ca.scratch = ctx->d_bscr;
  ca.chi2 = ctx->chi2;
  ca.outcomes = ctx->d_outcomes;
  ca.near = ctx->d_near;
  ca.basis = basis;
  ca.seed = ctx->seed;
  ca.chain0 = ctx->chain0;
  ca.sample = ctx->sample;
  launch_collapse(b, ca, s);
  HIPCHK(hipGetLastError());
  if (env_out && P.n_env > 0)
    HIPCHK(hipMemcpyAsync(env_out, ctx->d_outcomes,
                          (size_t)ctx->B * P.n_env, hipMemcpyDeviceToHost, s));
  InitArgs ia;
  ia.is_cluster = ctx->d_is_cluster;
  ia.is_ancilla = ctx->d_is_ancilla;
  ia.env_index = ctx->d_env_index;
  ia.labels = ctx->d_outcomes;
  ia.n_env = P.n_env;
  ia.basis = basis;
  launch_init(b, ia, ctx->d_logw, s);
  HIPCHK(hipGetLastError());
  std::vector<uint8_t> outcomes;
  if (ctx->u1_live) {
    outcomes.resize((size_t)ctx->B * std::max(P.n_env, 1));
    if (P.n_env > 0)
      HIPCHK(hipMemcpyAsync(outcomes.data(), ctx->d_outcomes,
                            (size_t)ctx->B * P.n_env, hipMemcpyDeviceToHost,
                            s));
  }
  HIPCHK(hipStreamSynchronize(s));
  init_host_chi(ctx);
  if (ctx->u1_live) init_host_charges(ctx, outcomes.data());
  ctx->center = 0;
  ctx->evo_pos = 0;
  ctx->sample += 1;
  ctx->stats.sample = ctx->sample;
  return HMPS_OK;
}

hmps_status hmps_stats(hmps_ctx *ctx, hmps_stats_t *out) {
  if (!ctx || !out) return HMPS_E_INVALID;
  DeviceGuard guard(ctx->opt.device);
  hmps_stats_t s = ctx->stats;
  s.center = ctx->center;
  s.evolve_pos = ctx->evo_pos;
  s.u1_blocks = ctx->u1_blocks;
  if (ctx->sub && !ctx->poisoned) {
    // the SVD work of the charge blocks
    const hmps_stats_t &b = ctx->sub->stats;
    s.jacobi_sweeps += b.jacobi_sweeps;
    s.svd_flops += b.svd_flops;
    s.svd_seconds += b.svd_seconds;
    s.round_launches += b.round_launches;
    s.svd_bytes += b.svd_bytes;
    s.wide_launches += b.wide_launches;
    s.split_launches += b.split_launches;
    std::vector<int32_t> sw(ctx->max_blocks);
    if (hipMemcpy(sw.data(), ctx->sub->d_sweeps,
                  sizeof(int32_t) * ctx->max_blocks,
                  hipMemcpyDeviceToHost) == hipSuccess)
      for (int32_t v : sw) s.jacobi_sweeps += v;
  }
  if ((ctx->ready || ctx->bond_loaded) && !ctx->poisoned) {
    std::vector<double> disc(ctx->B);
    std::vector<int32_t> sw(ctx->B);
    if (hipMemcpy(disc.data(), ctx->d_disc, sizeof(double) * ctx->B,
                  hipMemcpyDeviceToHost) == hipSuccess &&
        hipMemcpy(sw.data(), ctx->d_sweeps, sizeof(int32_t) * ctx->B,
                  hipMemcpyDeviceToHost) == hipSuccess) {
      s.discarded_weight = 0.0;
      for (double d : disc) s.discarded_weight += d;
      for (int32_t v : sw) s.jacobi_sweeps += v;
    }
  }
  *out = s;
  return HMPS_OK;
}

// <S_i.S_j> of every chain for physical-site pairs (i != j), written to
// out[c * n + t]: the transfer-matrix strings of the bond measurement on a
// list of arbitrary pairs, PAIR_CHUNK pairs per pass.
static hmps_status measure_pairs(hmps_ctx *ctx, int n, const int32_t *si,
                                 const int32_t *sj, double *out) {
  if (ctx->center != 0) {
    hmps_status st = move_center(ctx, 0);
    if (st) return st;
  }
  const Plan &P = ctx->plan;
  Batch b = batch_of(ctx);
  hipStream_t s = ctx->stream;
  MeasureArgs ma;
  ma.bond_p = ctx->d_pair_p;
  ma.bond_q = ctx->d_pair_q;
  ma.bond_J = nullptr;
  ma.is_ancilla = ctx->d_is_ancilla;
  ma.envs = ctx->d_envs;
  ma.wsz = ctx->d_wsz;
  ma.bond_scratch = ctx->d_bscr;
  ma.slots = ctx->slots;
  ma.chi2 = ctx->chi2;
  ma.norm = ctx->d_norm;
  ma.bond_ss = ctx->d_pair_ss;
  launch_measure_envs(b, ma, s);
  std::vector<int32_t> pp(PAIR_CHUNK), qq(PAIR_CHUNK);
  std::vector<double> chunk((size_t)ctx->B * PAIR_CHUNK);
  for (int t0 = 0; t0 < n; t0 += PAIR_CHUNK) {
    const int cnt = std::min(PAIR_CHUNK, n - t0);
    for (int t = 0; t < cnt; ++t) {
      const int a = P.pos_of_phys[si[t0 + t]], c = P.pos_of_phys[sj[t0 + t]];
      pp[t] = std::min(a, c);
      qq[t] = std::max(a, c);
    }
    HIPCHK(hipMemcpyAsync(ctx->d_pair_p, pp.data(), sizeof(int32_t) * cnt,
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(ctx->d_pair_q, qq.data(), sizeof(int32_t) * cnt,
                          hipMemcpyHostToDevice, s));
    ma.n_bonds = cnt;
    for (int b0 = 0; b0 < cnt; b0 += ctx->slots)
      launch_measure_bonds(b, ma, b0, std::min(ctx->slots, cnt - b0), s);
    launch_measure_scale(b, ma, s);
    HIPCHK(hipGetLastError());
    HIPCHK(hipMemcpyAsync(chunk.data(), ctx->d_pair_ss,
                          sizeof(double) * ctx->B * cnt,
                          hipMemcpyDeviceToHost, s));
    // the host arrays are reused by the next pass
    HIPCHK(hipStreamSynchronize(s));
    for (int c = 0; c < ctx->B; ++c)
      for (int t = 0; t < cnt; ++t)
        out[(size_t)c * n + t0 + t] = chunk[(size_t)c * cnt + t];
  }
  return HMPS_OK;
}

hmps_status hmps_measure_pairs(hmps_ctx *ctx, int32_t n_pairs,
                               const int32_t *site_i, const int32_t *site_j,
                               double *ss) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (n_pairs < 0 || (n_pairs > 0 && (!site_i || !site_j || !ss)))
    return fail(ctx, HMPS_E_INVALID, "bad pair arrays");
  const int np = ctx->plan.n_phys;
  std::vector<int32_t> ii, jj;
  std::vector<int> where;
  for (int t = 0; t < n_pairs; ++t) {
    if (site_i[t] < 0 || site_i[t] >= np || site_j[t] < 0 || site_j[t] >= np)
      return fail(ctx, HMPS_E_INVALID, "site id outside [0, n_phys)");
    if (site_i[t] != site_j[t]) {
      ii.push_back(site_i[t]);
      jj.push_back(site_j[t]);
      where.push_back(t);
    }
  }
  std::vector<double> vals((size_t)ctx->B * ii.size());
  if (!ii.empty()) {
    st = measure_pairs(ctx, (int)ii.size(), ii.data(), jj.data(), vals.data());
    if (st) return st;
  }
  // S_i.S_i = s(s+1) = 2 for spin 1
  for (int c = 0; c < ctx->B; ++c) {
    for (int t = 0; t < n_pairs; ++t) ss[(size_t)c * n_pairs + t] = 2.0;
    for (size_t u = 0; u < ii.size(); ++u)
      ss[(size_t)c * n_pairs + where[u]] = vals[(size_t)c * ii.size() + u];
  }
  return HMPS_OK;
}

hmps_status hmps_susceptibility(hmps_ctx *ctx, double beta, int32_t n_center,
                                const int32_t *center, double *chi) {
  hmps_status st = check_usable(ctx, true);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  const int np = ctx->plan.n_phys;
  if (n_center < 1 || !center || !chi || !(beta >= 0.0))
    return fail(ctx, HMPS_E_INVALID, "bad susceptibility arguments");
  std::vector<int32_t> ii, jj;
  for (int t = 0; t < n_center; ++t) {
    if (center[t] < 0 || center[t] >= np)
      return fail(ctx, HMPS_E_INVALID, "center site outside [0, n_phys)");
    for (int i = 0; i < np; ++i)
      if (i != center[t]) {
        ii.push_back(center[t]);
        jj.push_back(i);
      }
  }
  std::vector<double> vals((size_t)ctx->B * ii.size());
  if (!ii.empty()) {
    st = measure_pairs(ctx, (int)ii.size(), ii.data(), jj.data(), vals.data());
    if (st) return st;
  }
  for (int c = 0; c < ctx->B; ++c) {
    // the i = j terms: S_j.S_j = 2
    double sum = 2.0 * n_center;
    for (size_t u = 0; u < ii.size(); ++u) sum += vals[(size_t)c * ii.size() + u];
    chi[c] = beta / 3.0 * sum / n_center;
  }
  return HMPS_OK;
}

hmps_status hmps_svd_probe(hmps_ctx *ctx, int32_t chi_l, int32_t chi_r,
                           const double *theta, int32_t chi_max,
                           double cutoff, double *sigma, int32_t *rank,
                           double *left, double *right) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!theta || !sigma || !rank)
    return fail(ctx, HMPS_E_INVALID, "theta, sigma and rank must not be NULL");
  if (chi_l < 1 || chi_r < 1 || chi_l > ctx->opt.chi_cap ||
      chi_r > ctx->opt.chi_cap)
    return fail(ctx, HMPS_E_INVALID, "chi_l and chi_r must be in [1, chi_cap]");
  if (ctx->opt.max_sites < 2)
    return fail(ctx, HMPS_E_INVALID, "the context needs max_sites >= 2");
  if (chi_max < 1 || !(cutoff >= 0.0) || !(cutoff < 1.0))
    return fail(ctx, HMPS_E_INVALID, "chi_max >= 1 and 0 <= cutoff < 1");
  const int m = 3 * chi_l, n = 3 * chi_r;
  for (size_t i = 0; i < (size_t)m * n; ++i)
    if (!std::isfinite(theta[i]))
      return fail(ctx, HMPS_E_INVALID, "theta has a non-finite entry");
  // the context's chains are replaced by one chain of two sites whose
  // update on bond (0, 1) finds theta' already in place
  Plan P;
  P.len = 2;
  ctx->plan = P;
  ctx->B = 1;
  ctx->ready = false;
  ctx->bond_loaded = false;
  ctx->u1_live = false;
  ctx->center = 0;
  ctx->h_chi = {chi_l, 1, chi_r};
  hipStream_t s = ctx->stream;
  HIPCHK(hipMemcpyAsync(ctx->d_chi, ctx->h_chi.data(), sizeof(int32_t) * 3,
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemsetAsync(ctx->d_err, 0, sizeof(int32_t), s));
  HIPCHK(hipMemsetAsync(ctx->d_disc, 0, sizeof(double), s));
  HIPCHK(hipMemsetAsync(ctx->d_logw, 0, sizeof(double), s));
  // theta' in the vector layout of the SVD: the min(m, n) vectors of length
  // max(m, n), stride vector_stride, column-major, zero padding rows, the
  // vector index interleaved (3 bond index + s)
  const bool trans = n > m;
  const int len = trans ? n : m, nvec = trans ? m : n,
            ld = vector_stride(len);
  std::vector<double> h((size_t)ld * nvec, 0.0);
  for (int r = 0; r < m; ++r)
    for (int c = 0; c < n; ++c) {
      const size_t vr = 3 * (size_t)(r % chi_l) + r / chi_l;
      const size_t vc = 3 * (size_t)(c % chi_r) + c / chi_r;
      h[trans ? vr * ld + c : vc * ld + r] = theta[(size_t)r * n + c];
    }
  HIPCHK(hipMemcpyAsync(ctx->d_TH, h.data(), sizeof(double) * h.size(),
                        hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(ctx->d_X, h.data(), sizeof(double) * h.size(),
                        hipMemcpyHostToDevice, s));
  ctx->skip_theta = true;
  st = do_update(ctx, 0, OP_SWAP, true, chi_max, cutoff);
  ctx->skip_theta = false;
  if (st) return st;
  const int k = ctx->h_chi[1];
  *rank = k;
  HIPCHK(hipMemcpy(sigma, ctx->d_sig, sizeof(double) * k,
                   hipMemcpyDeviceToHost));
  if (left)
    HIPCHK(hipMemcpy(left, ctx->d_sites, sizeof(double) * 3 * chi_l * k,
                     hipMemcpyDeviceToHost));
  if (right)
    HIPCHK(hipMemcpy(right, ctx->d_sites + ctx->site_cap,
                     sizeof(double) * 3 * k * chi_r, hipMemcpyDeviceToHost));
  return HMPS_OK;
}

hmps_status hmps_load_bond(hmps_ctx *ctx, int32_t n_chains, int32_t chi_l,
                           int32_t chi_m, int32_t chi_r, const double *center,
                           const double *right) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!center || !right)
    return fail(ctx, HMPS_E_INVALID, "center and right must not be NULL");
  if (n_chains < 1 || n_chains > ctx->opt.max_chains)
    return fail(ctx, HMPS_E_INVALID, "n_chains outside [1, max_chains]");
  const int cap = ctx->opt.chi_cap;
  if (chi_l < 1 || chi_m < 1 || chi_r < 1 || chi_l > cap || chi_m > cap ||
      chi_r > cap)
    return fail(ctx, HMPS_E_INVALID, "bond dimensions outside [1, chi_cap]");
  if (ctx->opt.max_sites < 2)
    return fail(ctx, HMPS_E_INVALID, "the context needs max_sites >= 2");
  const size_t nc = (size_t)3 * chi_l * chi_m, nr = (size_t)3 * chi_m * chi_r;
  for (size_t i = 0; i < nc * n_chains; ++i)
    if (!std::isfinite(center[i]))
      return fail(ctx, HMPS_E_INVALID, "center has a non-finite entry");
  for (size_t i = 0; i < nr * n_chains; ++i)
    if (!std::isfinite(right[i]))
      return fail(ctx, HMPS_E_INVALID, "right has a non-finite entry");
  // every chain becomes an open two-site segment (0, 1) with outer bonds
  // chi_l and chi_r, the centre on site 0
  Plan P;
  P.len = 2;
  ctx->plan = P;
  ctx->B = n_chains;
  ctx->ready = false;
  ctx->u1_live = false;
  ctx->bond_loaded = false;
  ctx->center = 0;
  std::memset(&ctx->stats, 0, sizeof(ctx->stats));
  ctx->h_chi.resize((size_t)3 * n_chains);
  for (int c = 0; c < n_chains; ++c) {
    ctx->h_chi[3 * c] = chi_l;
    ctx->h_chi[3 * c + 1] = chi_m;
    ctx->h_chi[3 * c + 2] = chi_r;
  }
  hipStream_t s = ctx->stream;
  HIPCHK(hipMemcpyAsync(ctx->d_chi, ctx->h_chi.data(),
                        sizeof(int32_t) * 3 * n_chains, hipMemcpyHostToDevice,
                        s));
  for (int c = 0; c < n_chains; ++c) {
    double *site0 = ctx->d_sites + (size_t)2 * c * ctx->site_cap;
    HIPCHK(hipMemcpyAsync(site0, center + nc * c, sizeof(double) * nc,
                          hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(site0 + ctx->site_cap, right + nr * c,
                          sizeof(double) * nr, hipMemcpyHostToDevice, s));
  }
  HIPCHK(hipMemsetAsync(ctx->d_err, 0, sizeof(int32_t) * n_chains, s));
  HIPCHK(hipMemsetAsync(ctx->d_disc, 0, sizeof(double) * n_chains, s));
  HIPCHK(hipMemsetAsync(ctx->d_logw, 0, sizeof(double) * n_chains, s));
  HIPCHK(hipMemsetAsync(ctx->d_sweeps, 0, sizeof(int32_t) * n_chains, s));
  HIPCHK(hipStreamSynchronize(s));
  ctx->stats.n_chains = n_chains;
  ctx->stats.n_sites = 2;
  ctx->bond_loaded = true;
  return HMPS_OK;
}

hmps_status hmps_apply_gate(hmps_ctx *ctx, double J, double x,
                            int32_t chi_max, double cutoff, double *logw) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!ctx->bond_loaded)
    return fail(ctx, HMPS_E_STATE, "hmps_load_bond has not been called");
  if (!std::isfinite(J) || !std::isfinite(x))
    return fail(ctx, HMPS_E_INVALID, "J and x must be finite");
  if (chi_max < 1 || chi_max > ctx->opt.chi_cap)
    return fail(ctx, HMPS_E_INVALID, "chi_max outside [1, chi_cap]");
  if (!(cutoff >= 0.0) || !std::isfinite(cutoff))
    return fail(ctx, HMPS_E_INVALID, "cutoff must be finite and >= 0");
  // the gate takes coupling slot 0; do_update synchronises the stream
  // before g goes out of scope
  double g[81];
  gate9(J, x, g);
  ctx->plan.couplings.assign(1, J);
  HIPCHK(hipMemcpyAsync(ctx->d_gates, g, sizeof(g), hipMemcpyHostToDevice,
                        ctx->stream));
  const bool right = ctx->center == 0;
  st = do_update(ctx, 0, 0, right, chi_max, cutoff);
  if (st) return st;
  ctx->center = right ? 1 : 0;
  if (logw) {
    HIPCHK(hipMemcpyAsync(logw, ctx->d_logw, sizeof(double) * ctx->B,
                          hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  return HMPS_OK;
}

hmps_status hmps_read_site(hmps_ctx *ctx, int32_t chain, int32_t site,
                           double *out) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!ctx->ready && !ctx->bond_loaded)
    return fail(ctx, HMPS_E_STATE, "the context holds no chains");
  if (!out) return fail(ctx, HMPS_E_INVALID, "out is NULL");
  const int L = ctx->plan.len;
  if (chain < 0 || chain >= ctx->B || site < 0 || site >= L)
    return fail(ctx, HMPS_E_INVALID, "chain or site out of range");
  const int *row = &ctx->h_chi[(size_t)chain * (L + 1)];
  const size_t n = (size_t)3 * row[site] * row[site + 1];
  const double *src =
      ctx->d_sites + ((size_t)chain * L + site) * ctx->site_cap;
  HIPCHK(hipMemcpyAsync(out, src, sizeof(double) * n, hipMemcpyDeviceToHost,
                        ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HMPS_OK;
}

hmps_status hmps_bond_dims(hmps_ctx *ctx, int32_t *chi) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  DeviceGuard guard(ctx->opt.device);
  if (!ctx->ready && !ctx->bond_loaded)
    return fail(ctx, HMPS_E_STATE, "hmps_init_cluster_env has not been called");
  if (!chi) return fail(ctx, HMPS_E_INVALID, "chi is NULL");
  HIPCHK(hipMemcpyAsync(chi, ctx->d_chi,
                        sizeof(int32_t) * ctx->B * (ctx->plan.len + 1),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return HMPS_OK;
}

hmps_status hmps_set_width_rule(hmps_ctx *ctx, int32_t n,
                                const int32_t *nvec_min,
                                const int32_t *chains_min) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  if (n < 0 || n > MAX_WIDTH_RULE || (n > 0 && (!nvec_min || !chains_min)))
    return fail(ctx, HMPS_E_INVALID, "width rule: 0..16 entries");
  std::vector<WidthEntry> rule;
  for (int i = 0; i < n; ++i) {
    if (nvec_min[i] < W32_MIN_N || chains_min[i] < 1 ||
        (i > 0 && (nvec_min[i] <= nvec_min[i - 1] ||
                   chains_min[i] > chains_min[i - 1])))
      return fail(ctx, HMPS_E_INVALID,
                  "width rule: nvec_min ascending from " +
                      std::to_string(W32_MIN_N) +
                      ", chains_min >= 1 and not increasing");
    rule.push_back({nvec_min[i], chains_min[i]});
  }
  ctx->width_rule =
      n > 0 ? rule
            : std::vector<WidthEntry>{std::begin(DEFAULT_WIDTH_RULE),
                                      std::end(DEFAULT_WIDTH_RULE)};
  if (ctx->sub) ctx->sub->width_rule = ctx->width_rule;
  return HMPS_OK;
}

hmps_status hmps_bond_charges(hmps_ctx *ctx, int32_t chain, int32_t bond,
                              int32_t *q) {
  hmps_status st = check_usable(ctx, false);
  if (st) return st;
  if (!ctx->u1_live)
    return fail(ctx, HMPS_E_STATE,
                "no charges: the chains do not come from "
                "hmps_init_cluster_env on a U(1) context");
  const int L = ctx->plan.len;
  if (!q || chain < 0 || chain >= ctx->B || bond < 0 || bond > L)
    return fail(ctx, HMPS_E_INVALID, "chain or bond out of range");
  int i = 0;
  for (const auto &g : ctx->h_qg[(size_t)chain * (L + 1) + bond])
    for (int t = 0; t < g.second; ++t) q[i++] = g.first;
  return HMPS_OK;
}

hmps_status hmps_gate(double J, double x, double *out) {
  if (!out || !std::isfinite(J) || !std::isfinite(x)) return HMPS_E_INVALID;
  gate9(J, x, out);
  return HMPS_OK;
}

hmps_status hmps_schedule(const hmps_lattice *lat, int32_t *n_sites,
                          int32_t *n_updates, int32_t *k, int32_t *op,
                          int32_t cap) {
  Plan P;
  if (!validate_and_plan(lat, P).empty()) return HMPS_E_INVALID;
  if (n_sites) *n_sites = P.len;
  if (n_updates) *n_updates = (int32_t)P.step_k.size();
  if (k && op && cap >= (int32_t)P.step_k.size()) {
    for (size_t t = 0; t < P.step_k.size(); ++t) {
      k[t] = P.step_k[t];
      op[t] = P.step_op[t];
    }
  }
  return HMPS_OK;
}

}  // extern "C"
