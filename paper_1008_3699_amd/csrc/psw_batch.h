// psw_batch.h -- batched FP64 vector kernels (psw_batch_kernels.hip).
#pragma once

#include "psw_fast2d.h"

namespace psw {

// vector chunk length of a batch (a chunk never spans two problems)
constexpr int kBatchChunk = 2048;

hipError_t launch_b_spmv(const BChunk *c, int nc, const BProb *p, int src, int dst, bool residual, hipStream_t st);
// scal[dst] = slot a . slot b per problem (force: also for inactive problems)
hipError_t launch_b_dot(const BChunk *c, int nc, const BProb *p, int np, int a, int b, double *partials, int dst,
                        bool force, hipStream_t st);
hipError_t launch_b_cg_xr(const BChunk *c, int nc, const BProb *p, int np, int num, double *partials,
                          hipStream_t st);
hipError_t launch_b_check(const BProb *p, int np, double rtol2, int64_t maxit, hipStream_t st);
hipError_t launch_b_init(const BProb *p, int np, double rtol2, hipStream_t st);
hipError_t launch_b_activate(const BProb *p, int np, hipStream_t st);
hipError_t launch_b_count(const BProb *p, int np, int *out, hipStream_t st);
// iflags[3 b + k] = flags[k] (active, iterations, status); dscal[5 b + k] = scal[k] (dscal may be null)
hipError_t launch_b_gather(const BProb *p, int np, int *iflags, double *dscal, hipStream_t st);
hipError_t launch_b_cg_p(const BChunk *c, int nc, const BProb *p, int num, int den, hipStream_t st);
hipError_t launch_b_combine(const BChunk *c, int nc, const BProb *p, bool y_f64, hipStream_t st);
hipError_t launch_b_copy(const BChunk *c, int nc, const BProb *p, int src, int dst, hipStream_t st);

} // namespace psw
