/*
 * hmps.h -- C ABI of the MI355X (gfx950) library for the hot path of the
 * hybrid purification/sampling method for thermal quantum systems
 * (J. Chen and E.M. Stoudenmire, arXiv:1910.09142).
 *
 * The library evolves a batch of independent hybrid METTS-ancilla Markov
 * chains.  Each chain is a matrix product state (MPS) whose cluster sites
 * are physical-ancilla Bell pairs and whose environment sites are a sampled
 * product state (Hybrid METTS-Ancilla subsection, steps 1-4 of the Markov
 * Chain Sampling Algorithm).  All numerical work runs in hand-written HIP
 * kernels on the device selected at create time.
 *
 * Conventions used by every call
 *   - Spin-1 sites, physical dimension d = 3, local basis ordered
 *     m = +1, 0, -1 (S^z eigenbasis).  Product-state outcome labels 0,1,2
 *     denote the eigenvalues +1, 0, -1 of S^z (basis 0) or S^x (basis 1).
 *   - MPS layout: physical sites in the order mps_order; every cluster
 *     physical site is immediately followed by its ancilla partner (Ancilla
 *     Method subsection; Fig. "initial").  "Environment positions" are the
 *     MPS positions of non-cluster physical sites, ascending.
 *   - Ownership: the caller owns every host array (read during the call or
 *     written before it returns) and the device workspace it passes to
 *     hmps_create; the library never allocates device memory.
 *   - Streams: work is enqueued on the stream given at create time.  Calls
 *     returning host data synchronise that stream before returning.
 *   - Errors: no exception crosses the ABI.  HMPS_E_INVALID leaves the
 *     context unchanged.  HMPS_E_DEVICE and HMPS_E_NUMERIC poison the
 *     context: only hmps_last_error, hmps_stats and hmps_destroy are
 *     accepted afterwards.  hmps_last_error explains the last failure.
 *   - Thread compatibility: one context must not be used by two threads at
 *     once; distinct contexts are independent.
 */
#ifndef HMPS_H
#define HMPS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hmps_ctx hmps_ctx;
typedef int32_t hmps_status;

#define HMPS_OK 0
#define HMPS_E_INVALID 1 /* bad argument; context unchanged             */
#define HMPS_E_NOMEM 2   /* workspace too small for the request         */
#define HMPS_E_DEVICE 3  /* a HIP call failed                           */
#define HMPS_E_STATE 4   /* call out of order (e.g. evolve before init) */
#define HMPS_E_NUMERIC 5 /* SVD did not converge, NaN/Inf, zero norm    */

/* Precision of an update (Trotter gate or swap; centre moves are always
 * FP64).  HMPS_PREC_FP64: every step in FP64.  HMPS_PREC_MIXED_FP32: the
 * theta contraction and the gate in FP32 on the matrix cores (FP32
 * accumulation, FP64 site tensors rounded on load); for updates whose SVD
 * takes the QR-preconditioned blocked path, the Jacobi sweeps run in FP32
 * on the FP64 R factor rounded to FP32, and a Rayleigh-Ritz step in FP64
 * on the chi_max + 64 (rounded to 32) largest resulting vectors gives the
 * kept singular triplets.  Truncation, ||theta'||^2, the log-weight,
 * norms, observables and all accumulations are FP64 in both modes. */
#define HMPS_PREC_FP64 0
#define HMPS_PREC_MIXED_FP32 1
/* Split-bf16 (three bf16 products per FP32 product) contractions are not
 * built: hmps_create rejects this value with HMPS_E_INVALID.  The theta
 * contraction is a small share of an update; the SVD sets the cost. */
#define HMPS_PREC_MIXED_BF16X3 2

/* Symmetry of the evolution (Exploiting Conserved Quantum Numbers
 * subsection).  The gates conserve Q = sum_phys S^z - sum_ancilla S^z, the
 * Bell pairs carry Q = 0, and an environment collapsed in S^z is a
 * product state of definite Q, so every state of an evolution lies in one
 * sector of Q, which changes from sample to sample with the collapse.
 *   HMPS_SYM_NONE: dense site tensors.
 *   HMPS_SYM_U1:   every bond index carries the charge of the sites left of
 *                  it (ancillas counted with flipped sign), and each
 *                  update's theta' splits into one block per charge of the
 *                  new bond: every block is decomposed on its own, the
 *                  singular values of all blocks are truncated together
 *                  by the rule of hmps_evolve, and the new bond lists the
 *                  kept vectors block by block in ascending charge.  The
 *                  site tensors stay dense arrays whose entries outside
 *                  the blocks are zero.  Collapses and initial states must
 *                  be in S^z (basis 0); FP64 only.  Chains loaded by
 *                  hmps_load_bond or replaced by hmps_svd_probe carry no
 *                  charges and are updated densely. */
#define HMPS_SYM_NONE 0
#define HMPS_SYM_U1 1

/* Bits of the `what` mask of hmps_measure. */
#define HMPS_MEASURE_ENERGY 1u /* energy (needs every bond correlator)   */
#define HMPS_MEASURE_BONDS 2u  /* <S_i.S_j> of every Hamiltonian bond    */
#define HMPS_MEASURE_LOGW 4u   /* log-weights (no device contraction)    */
#define HMPS_MEASURE_QN 8u     /* <Q>, Q = sum_phys S^z - sum_anc S^z    */
#define HMPS_MEASURE_ALL 15u
/* Not an output: add this measurement's per-bond correlators and energy
 * of every chain to the device-side sample moments (hmps_bond_moments). */
#define HMPS_MEASURE_ACCUMULATE 16u

typedef struct {
  int32_t device;          /* HIP device ordinal                          */
  void *stream;            /* hipStream_t; NULL = the null stream         */
  void *workspace;         /* device buffer owned by the caller           */
  size_t workspace_bytes;  /* its size; see hmps_workspace_bytes          */
  int32_t max_chains;      /* largest n_chains accepted, <= 65535         */
  int32_t max_sites;       /* largest MPS length (physical + ancilla)     */
  int32_t chi_cap;         /* largest chi_max accepted by evolve          */
  int32_t max_bonds;       /* largest number of Hamiltonian bonds         */
  int32_t precision;       /* HMPS_PREC_*                                 */
  int32_t max_sweeps;      /* Jacobi sweep cap, 0 = default (100)         */
  double jacobi_tol;       /* relative orthogonality tolerance, 0 = auto  */
  /* Optional: called on the calling thread after every Trotter step of
   * hmps_evolve with (progress_user, steps done, steps in this call).  It
   * must not call back into the library with the same context. */
  void (*progress)(void *user, int64_t done, int64_t total);
  void *progress_user;
  int32_t symmetry;        /* HMPS_SYM_*                                  */
  int32_t max_blocks;      /* HMPS_SYM_U1: charge blocks one pass of an
                              update holds over all chains (an update takes
                              several passes when it has more); 0 =
                              max(64, 4 * max_chains)                      */
} hmps_options;

/* Hamiltonian H = sum_b J_b S_{i_b} . S_{j_b} on n_phys spin-1 sites
 * (Results section: the S=1 Heisenberg ladder is one instance), the
 * order of the physical sites along the MPS, and the cluster mask (sites
 * purified by an ancilla; the rest is sampled).  Host arrays, read only
 * during hmps_init_cluster_env. */
typedef struct {
  int32_t n_phys;
  int32_t n_bonds;
  const int32_t *bond_i;     /* n_bonds physical ids                       */
  const int32_t *bond_j;     /* n_bonds physical ids, != bond_i            */
  const double *bond_J;      /* n_bonds couplings (finite)                 */
  const int32_t *mps_order;  /* n_phys: a permutation of 0..n_phys-1       */
  const uint8_t *in_cluster; /* n_phys: 1 = cluster (purified) site        */
} hmps_lattice;

typedef struct {
  int64_t updates;          /* two-site updates applied (all chains)     */
  int64_t gate_updates;     /* of which Hamiltonian gates                */
  int64_t move_updates;     /* of which orthogonality-centre moves       */
  int64_t jacobi_sweeps;    /* Jacobi sweeps launched                    */
  int32_t max_chi;          /* largest bond dimension reached            */
  int32_t n_chains;
  int32_t n_sites;
  int32_t n_env;
  int64_t sample;           /* index of the current sample               */
  double discarded_weight;  /* sum of relative discarded weights         */
  double evolve_seconds;    /* wall time spent in hmps_evolve            */
  /* Algorithmic work of the updates applied, summed over chains: per
   * update 2*9*chiL*chiM*chiR (theta) + 2*81*chiL*chiR (gate) + the
   * Golub-Reinsch count of a thin SVD with both factors of the L x N
   * vector matrix, 14 L N^2 + 8 N^3 (L >= N). */
  double algo_flops;
  double svd_flops;         /* SVD part of algo_flops for the updates    */
                            /* that took the blocked (multi-workgroup)   */
                            /* Jacobi path                               */
  double svd_seconds;       /* device time (event span) of those rounds  */
  int64_t round_launches;   /* blocked Jacobi round kernels launched     */
  double svd_bytes;         /* algorithmic bytes of those rounds: each
                               vector read once per round, and written
                               once while its chain still rotates        */
  int64_t center;           /* MPS position of the orthogonality centre  */
  int64_t evolve_pos;       /* updates applied of an evolution run in
                               parts by hmps_evolve_updates (0: none)    */
  int64_t jacobi_sweeps_fp32; /* of jacobi_sweeps, the FP32 sweeps of the
                               mixed-precision SVD                        */
  int64_t wide_launches;    /* of round_launches, rounds of 32-vector
                               blocks (updates with >= 512 vectors)      */
  int64_t u1_blocks;        /* HMPS_SYM_U1: charge blocks decomposed     */
  int64_t split_launches;   /* of wide_launches, rounds issued as two
                               concurrent dispatches (the two halves of
                               the chains, on two streams; rounds of more
                               than 256 workgroups)                      */
} hmps_stats_t;

/* Bytes of device workspace needed for the given capacities. */
size_t hmps_workspace_bytes(int32_t max_chains, int32_t max_sites,
                            int32_t chi_cap, int32_t max_bonds);

/* The same for a context created with `symmetry` and `max_blocks` (the
 * hmps_options fields; HMPS_SYM_NONE gives hmps_workspace_bytes).  Every
 * charge block of an update is a two-site segment of up to 3 chi_cap x
 * 3 chi_cap entries with its own SVD buffers. */
size_t hmps_workspace_bytes_sym(int32_t max_chains, int32_t max_sites,
                                int32_t chi_cap, int32_t max_bonds,
                                int32_t symmetry, int32_t max_blocks);

/* Create a context on opt->device using the caller's workspace (device
 * memory aligned to 256 bytes, at least hmps_workspace_bytes_sym(...) long,
 * owned by the caller and not freed by the library).  E_INVALID for bad
 * capacities (max_chains outside [1, 65535]: chains are a grid dimension
 * of the launches; max_sites < 1; chi_cap outside [3, 640]; max_bonds <
 * 0; an unknown precision or symmetry; HMPS_SYM_U1 with mixed precision
 * or max_blocks outside [0, 65535]) or a misaligned workspace; E_NOMEM for
 * a NULL or too small workspace; E_DEVICE if opt->device is not usable. */
hmps_status hmps_create(hmps_ctx **out, const hmps_options *opt);

/* Step 1 of the Markov chain (Hybrid METTS-Ancilla subsection; Bell pair
 * |B_j> = d^{-1/2} sum_s |s>_P |s>_A): build n_chains initial states.
 * env_state: n_chains x n_env outcome labels (row-major, chain-major) in
 * `basis`, or NULL to draw each environment site's S^z label uniformly
 * with Philox4x64-10 (key = (seed, 0), counter = (chain, 0, MPS position,
 * 0), label = floor(3 u), u = top 53 bits / 2^53).  Resets the sample
 * counter to 0 and every log-weight to 0.  E_INVALID for a malformed
 * lattice, a label > 2, capacities exceeded, or basis 1 on a HMPS_SYM_U1
 * context.  Same as
 * hmps_init_cluster_env_at with chain_offset = 0 and sample = 0. */
hmps_status hmps_init_cluster_env(hmps_ctx *ctx, const hmps_lattice *lat,
                                  int32_t n_chains, uint64_t seed,
                                  const uint8_t *env_state, int32_t basis);

/* Step 1 for chains chain_offset .. chain_offset + n_chains - 1 of a
 * larger ensemble, starting at sample `sample` (the Markov chains of the
 * Hybrid METTS-Ancilla subsection are independent, so the ensemble splits
 * over contexts or devices, and a chain resumes from the product state its
 * last collapse produced).  Every Philox counter carries the global chain
 * id chain_offset + c and the sample index: the initial draws use
 * (chain_offset + c, sample, MPS position, 0) and the collapse of sample n
 * uses (chain_offset + c, n, MPS position, 1).  So chains split over
 * contexts with matching offsets, or resumed at sample n with the outcomes
 * of sample n - 1 (in its basis), reproduce an uninterrupted run bit for
 * bit.  E_INVALID as hmps_init_cluster_env, and for sample < 0 or an
 * offset whose chain ids overflow. */
hmps_status hmps_init_cluster_env_at(hmps_ctx *ctx, const hmps_lattice *lat,
                                     int32_t n_chains, uint64_t seed,
                                     uint64_t chain_offset, int64_t sample,
                                     const uint8_t *env_state, int32_t basis);

/* Step 2: apply (e^{-tau H})^M, M = beta/(2 tau) (Ancilla Method
 * subsection; M must be an integer to 1e-9, else E_INVALID), as a second-
 * order Trotter product of two-site gates exp(-(tau/2) J S_i.S_j) applied
 * with nearest-neighbour swaps, each followed by an SVD truncated to at
 * most chi_max values with relative discarded weight <= cutoff (Results
 * section).  The state is renormalised after every gate and ln of its
 * squared norm is added to the chain's log-weight.  On return the
 * orthogonality centre is site 0.  E_INVALID: chi_max < 1 or > chi_cap,
 * cutoff < 0, tau <= 0 with beta > 0.  E_NUMERIC: the Jacobi SVD did not
 * converge in max_sweeps or produced a non-finite value.  E_NOMEM (U(1)):
 * an update of one chain has more charge blocks than max_blocks; the
 * chains keep the updates applied before it. */
hmps_status hmps_evolve(hmps_ctx *ctx, double beta, double tau,
                        int32_t chi_max, double cutoff);

/* Part of the evolution hmps_evolve(beta, tau, chi_max, cutoff) applies:
 * its two-site updates first .. first + count - 1 (the list has M times
 * the updates of one Trotter step, see hmps_schedule), each with the
 * centre moves it needs.  Parts must follow each other (first = the
 * number already applied, hmps_stats.evolve_pos) with the same
 * parameters, else E_STATE / E_INVALID; the part that applies the last
 * update also moves the centre to site 0, as hmps_evolve does.  For
 * update-by-update comparison with a reference (teacher forcing).
 * E_INVALID for a range outside [0, M * steplen] and as hmps_evolve. */
hmps_status hmps_evolve_updates(hmps_ctx *ctx, double beta, double tau,
                                int32_t chi_max, double cutoff, int64_t first,
                                int64_t count);

/* Result of the last two-site update of every chain (a Trotter gate, a
 * swap or a centre move): rank[c] = singular values kept, sigma[c * cap +
 * j] (j < min(rank[c], cap)) the kept singular values of theta' in
 * descending order, before the kept ones are renormalised (theta' of a
 * gate has unit norm; Results section: truncated SVD).  E_STATE if no
 * update has run since the chains were created.  Synchronises. */
hmps_status hmps_last_spectrum(hmps_ctx *ctx, int32_t cap, int32_t *rank,
                               double *sigma);

/* Step 3: per-chain Monte Carlo estimators <psi|A|psi> (Markov Chain
 * Sampling Algorithm, step 3).  `what` is a mask of HMPS_MEASURE_* bits;
 * an output is written when its bit is set and its pointer is not NULL,
 * and only the contractions those outputs need run.  Outputs (host):
 *   energy  [n_chains]           sum_b J_b <S_i.S_j>
 *   bond_ss [n_chains * n_bonds] <S_i.S_j> per bond, in lattice order
 *   logw    [n_chains]           accumulated ln of squared gate norms
 *   qn      [n_chains]           <sum_phys S^z - sum_ancilla S^z> (an
 *                                expectation value: an integer only for
 *                                environments collapsed in S^z, so FP64)
 * With HMPS_MEASURE_ACCUMULATE the correlators are computed whether or
 * not they are output, and added on the device to the per-chain moments.
 * E_INVALID for unknown bits.  Synchronises the stream. */
hmps_status hmps_measure(hmps_ctx *ctx, uint32_t what, double *energy,
                         double *bond_ss, double *logw, double *qn);

/* Sample variance of the estimators, bond by bond (Entanglement and Cost
 * of Hybrid States: the variance of every bond energy <S_i.S_j> along the
 * ladder, lower inside the purified cluster than outside).  Every
 * hmps_measure call with HMPS_MEASURE_ACCUMULATE adds the n_chains values
 * of each bond correlator and of the energy to per-chain running moments
 * on the device (count, mean, sum of squared deviations: Welford's update
 * in FP64); hmps_bond_moments combines the chains in chain order (Chan,
 * Golub and LeVeque) and returns, over all accumulated chains and
 * measurements:
 *   n_samples            the number of values per bond
 *   bond_mean [n_bonds]  their mean, bond_var [n_bonds] their unbiased
 *                        sample variance (divisor n - 1)
 *   energy_mean_var [2]  (optional) the same for the energy
 * A Markov chain samples product states with probability P_i / sum_j P_j,
 * so these are plain (unweighted) sample moments; consecutive samples of
 * one chain are correlated, which a variance of the mean must account
 * for.  hmps_init_cluster_env and hmps_moments_reset clear the moments.
 * E_STATE with fewer than two values, E_INVALID for NULL outputs.
 * Synchronises. */
hmps_status hmps_moments_reset(hmps_ctx *ctx);
hmps_status hmps_bond_moments(hmps_ctx *ctx, int64_t *n_samples,
                              double *bond_mean, double *bond_var,
                              double *energy_mean_var);

/* Step 4: collapse every environment site in MPS order by a projective
 * measurement in `basis` (0 = S^z, 1 = S^x), tracing the cluster sites;
 * outcome of a site = smallest label s with u < cumulative conditional
 * probability, u from Philox4x64-10 with counter (global chain id, sample,
 * MPS position, 1) (see hmps_init_cluster_env_at).  Then re-initialise every chain to the new product state
 * (in `basis`) with fresh Bell pairs and advance the sample counter.
 * env_out (host, may be NULL): n_chains x n_env labels.  E_INVALID for
 * basis 1 on a HMPS_SYM_U1 context (an S^x outcome has no definite
 * charge).  Synchronises. */
hmps_status hmps_collapse_resample(hmps_ctx *ctx, int32_t basis,
                                   uint8_t *env_out);

/* Counters since init. */
hmps_status hmps_stats(hmps_ctx *ctx, hmps_stats_t *out);

/* Block width of the Jacobi rounds (a tuning choice: the rounds rotate
 * pairs of 16-vector blocks, or of 32-vector blocks for large FP64 updates
 * in large batches).  Entry i: updates of a batch of at least
 * chains_min[i] chains take 32-vector blocks for every chain of at least
 * nvec_min[i] vectors (the smaller dimension of theta').  nvec_min
 * ascending from 512, chains_min >= 1 and not increasing; at most 16
 * entries; n = 0 restores the default, measured on MI355X: {540 vectors:
 * 16 chains, 768: 16, 1152: 8, 1536: 8}.  The width
 * changes the rounding of an update, not its result beyond it.  The
 * environment variable HMPS_WIDE=0 or 1, read at create time, overrides
 * the rule (never or always).  E_INVALID for a malformed rule. */
hmps_status hmps_set_width_rule(hmps_ctx *ctx, int32_t n,
                                const int32_t *nvec_min,
                                const int32_t *chains_min);

/* Charges of bond `bond` (0..n_sites) of chain `chain` on a HMPS_SYM_U1
 * context (Exploiting Conserved Quantum Numbers subsection): q[i], i <
 * chi[bond], is the Q of the sites left of the bond for bond index i;
 * a site tensor T[s][a][b] at a position holding a physical site is
 * nonzero only where q_right[b] = q_left[a] + S^z(s), and -S^z(s) for an
 * ancilla.  Host array of chi[bond] int32.  E_STATE unless the chains
 * come from hmps_init_cluster_env on a HMPS_SYM_U1 context; E_INVALID for
 * an index out of range. */
hmps_status hmps_bond_charges(hmps_ctx *ctx, int32_t chain, int32_t bond,
                              int32_t *q);

/* Bond dimensions chi[c][b], b = 0..n_sites, of every chain (host array
 * of n_chains * (n_sites + 1) int32), after hmps_init_cluster_env or
 * hmps_load_bond.  Synchronises. */
hmps_status hmps_bond_dims(hmps_ctx *ctx, int32_t *chi);

/* Site tensor `site` of chain `chain` (host array out of 3 * chi[site] *
 * chi[site + 1] doubles, layout T[s][a][b], s the S^z index m = +1, 0, -1,
 * a the left and b the right bond; bond dimensions from hmps_bond_dims),
 * after hmps_init_cluster_env or hmps_load_bond.  E_INVALID for an index
 * out of range.  Synchronises. */
hmps_status hmps_read_site(hmps_ctx *ctx, int32_t chain, int32_t site,
                           double *out);

/* One bond of an MPS as the workload of a single gate application (Ancilla
 * Method subsection: a two-site gate contracts the two site tensors with
 * the bond weights, and an SVD truncated by discarded weight restores the
 * MPS form).  Every one of n_chains chains becomes an open two-site
 * segment: site 0 is the orthogonality centre C with outer bond chi_l,
 * site 1 a right-orthonormal tensor B with outer bond chi_r, and chi_m the
 * bond between them.  center: host, n_chains blocks of 3 * chi_l * chi_m
 * doubles, C[s][a][b]; right: host, n_chains blocks of 3 * chi_m * chi_r
 * doubles, B[s][b][c] (layout of hmps_read_site).  Bond dimensions in
 * [1, chi_cap], n_chains in [1, max_chains], max_sites >= 2, finite
 * entries, else E_INVALID.  The context's chains are replaced
 * (hmps_init_cluster_env must be called again before evolve); log-weights
 * and counters restart at 0.  Synchronises. */
hmps_status hmps_load_bond(hmps_ctx *ctx, int32_t n_chains, int32_t chi_l,
                           int32_t chi_m, int32_t chi_r, const double *center,
                           const double *right);

/* One application of exp(-x J S_0.S_1) to the loaded bond of every chain,
 * the update that hmps_evolve runs for each Trotter gate (Ancilla Method
 * subsection; Results section for chi_max and the cutoff): theta =
 * T_0 T_1, theta' = G theta in the context's precision, log ||theta'||^2
 * added to the chain's log-weight, theta' normalised and split by the
 * truncated SVD.  With the centre on site 0 the singular values go to
 * site 1 (the centre moves right), otherwise to site 0, so repeated calls
 * sweep the bond back and forth.  logw (host, may be NULL): n_chains
 * accumulated log-weights.  Needs hmps_load_bond (E_STATE otherwise);
 * E_INVALID for non-finite J or x, chi_max outside [1, chi_cap] or a
 * negative or non-finite cutoff; E_NUMERIC if the SVD fails.
 * Synchronises. */
hmps_status hmps_apply_gate(hmps_ctx *ctx, double J, double x,
                            int32_t chi_max, double cutoff, double *logw);

/* Correlators <S_i.S_j> of the current sample of every chain for
 * arbitrary physical-site pairs (Results section: the susceptibility is
 * built from the correlations of central spins with all spins; the same
 * transfer-matrix strings as hmps_measure, at any distance along the MPS).
 * site_i, site_j: host arrays of n_pairs physical ids in [0, n_phys);
 * i == j gives s(s+1) = 2.  ss: host array, n_chains * n_pairs,
 * ss[c * n_pairs + t].  Needs hmps_init_cluster_env; moves the
 * orthogonality centre to site 0 if needed.  E_INVALID on bad ids.
 * Synchronises. */
hmps_status hmps_measure_pairs(hmps_ctx *ctx, int32_t n_pairs,
                               const int32_t *site_i, const int32_t *site_j,
                               double *ss);

/* Susceptibility estimator of every chain (Results section, equation of
 * chi_6): chi = (beta / 3) (1 / n_center) sum_{j in center} sum_{i in all}
 * <S_j.S_i>, i running over every physical site including j.  center: host
 * array of n_center physical ids (the paper averages over the middle 6 x 2
 * sites of the ladder); chi: host array of n_chains.  beta is the inverse
 * temperature of the ensemble (the state was evolved to beta/2).  Needs
 * hmps_init_cluster_env; E_INVALID for an id outside [0, n_phys),
 * n_center < 1 or beta < 0.  Synchronises. */
hmps_status hmps_susceptibility(hmps_ctx *ctx, double beta, int32_t n_center,
                                const int32_t *center, double *chi);

/* Diagnostic: the truncated SVD that follows every two-site gate (Ancilla
 * Method subsection: the bond is restored to MPS form by an SVD truncated
 * by discarded weight; Results section: the cutoff and chi_max), applied
 * to a given theta'.  theta: host array, m x n row-major with m = 3 chi_l
 * (rows (s1, a)) and n = 3 chi_r (columns (s2, c)), 1 <= chi_l, chi_r <=
 * chi_cap, finite.  It runs the device kernels of an FP64 update of
 * hmps_evolve (whatever the context's precision: the QR-preconditioned or
 * plain blocked one-sided Jacobi, truncation with the rules of hmps_evolve,
 * write-back with the singular values absorbed to the right) on chain 0.
 * Outputs (host, caller-owned): rank = k kept; sigma[k] the kept singular
 * values of theta' (descending, not renormalised); left (optional,
 * 3*chi_l*k) = U as T[s1][a][j]; right (optional, 3*k*chi_r) =
 * Sigma V^T / ||Sigma_kept|| as T[s2][j][c].  The context's chains are
 * replaced (hmps_init_cluster_env must be called again before evolve).
 * Needs max_sites >= 2; E_INVALID on bad arguments, E_NUMERIC if the SVD
 * does not converge.  Synchronises. */
hmps_status hmps_svd_probe(hmps_ctx *ctx, int32_t chi_l, int32_t chi_r,
                           const double *theta, int32_t chi_max,
                           double cutoff, double *sigma, int32_t *rank,
                           double *left, double *right);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * truncated SVD of hmps_svd_probe without a context, on caller-owned
 * device arrays, every intermediate in one file-scope device array of the
 * library (5.4 MiB per device, held until the process ends).  It allocates
 * nothing: no device memory, no events, no pinned memory.
 *   device, stream: the HIP device ordinal and a hipStream_t on it (NULL
 *     = the null stream); work is enqueued on the stream.
 *   theta: device array, m x n row-major (m = 3 chi_l, n = 3 chi_r),
 *     1 <= chi_l, chi_r <= 128 (the array's capacity; larger sizes return
 *     HMPS_E_INVALID).
 *   chi_max >= 1, 0 <= cutoff < 1: as hmps_svd_probe.
 *   Outputs, as hmps_svd_probe: *rank (host) = k, valid on return;
 *     sigma (device, >= min(m, n) doubles): the k kept singular values;
 *     left (device, >= 3 chi_l min(m, n)): U as T[s1][a][j]; right
 *     (device, >= 3 min(m, n) chi_r): Sigma V^T / ||Sigma_kept|| as
 *     T[s2][j][c]; these are written on `stream` after the call returns.
 * It runs the kernels of hmps_svd_probe on a context with chi_cap = 128
 * and default options (max_sweeps 100), with the Jacobi sweeps as a fixed
 * launch sequence; results equal that entry point's.  Every call on a
 * device shares the device's array and leaves its contents there: calls
 * that overlap on one device (other streams or threads) race.  Returns
 * HMPS_E_INVALID for bad arguments, HMPS_E_DEVICE for a failed HIP call,
 * HMPS_E_NUMERIC if the SVD does not converge.  Synchronises the stream
 * once (to read the status and rank). */
hmps_status hmps_svd_probe_noalloc(int32_t device, void *stream,
                                   int32_t chi_l, int32_t chi_r,
                                   const double *theta, int32_t chi_max,
                                   double cutoff, double *sigma,
                                   int32_t *rank, double *left,
                                   double *right);

/* Destroy a context (NULL is accepted).  Does not free the workspace. */
void hmps_destroy(hmps_ctx *ctx);

/* Text of the last error on this context ("" if none); static storage
 * owned by the context. */
const char *hmps_last_error(const hmps_ctx *ctx);

/* ---- host-only helpers (no device work) -------------------------------
 * The 9x9 gate exp(-x J S_1.S_2), index (s1,s2) -> 3 s1 + s2, row-major,
 * written into out[81] (spectral form with the three total-spin
 * projectors; Results section Hamiltonian, d = 3). */
hmps_status hmps_gate(double J, double x, double *out);

/* The update list of one Trotter step for `lat`: entries (k, op), k the
 * left MPS site, op >= 0 an index into the distinct couplings (in order
 * of first appearance in the bond list) or -1 for a swap.  Writes
 * *n_sites, *n_updates and, when the arrays are not NULL and cap >=
 * *n_updates, the entries. */
hmps_status hmps_schedule(const hmps_lattice *lat, int32_t *n_sites,
                          int32_t *n_updates, int32_t *k, int32_t *op,
                          int32_t cap);

#ifdef __cplusplus
}
#endif
#endif /* HMPS_H */
