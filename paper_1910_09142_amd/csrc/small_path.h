// Per-chain choice between the single-workgroup in-LDS SVD and the
// blocked Jacobi rounds.  The choice depends only on the chain's own
// theta' (L * N <= small_max), so a chain takes the same path alone and in
// a batch and gives the same result.
#pragma once
#include "hmps_internal.h"

namespace hmps {

// In-LDS one-sided Jacobi SVD of the chains whose L * N <= small_max; the
// other chains are left to the blocked rounds.
void launch_jacobi_small_upto(const Batch &b, const UpdScratch &s,
                              const UpdParams &u, size_t small_max,
                              hipStream_t st);

// Marks the chains whose L * N <= small_max as converged for the blocked
// rounds (launched after the first sweep's reset of the flags).
void launch_mark_small_done(const Batch &b, const UpdScratch &s,
                            const UpdParams &u, size_t small_max,
                            hipStream_t st);

}  // namespace hmps
