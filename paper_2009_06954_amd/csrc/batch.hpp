// Batched lockstep solves of many systems (see batch.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/asss.h"

namespace asss {
namespace batch {

// Whether the batch engine takes these systems: all on one device, natural
// inner order, at most 16 deflation vectors and 256 low-rank columns, at
// most four right-hand sides each, FGMRES from zero without fixed inner
// steps, one inner precision for all.
bool applies(int32_t nsys, const asss_handle_t* hs, const int32_t* nrhs, const asss_solve_opts_t& o);

// Solve (the arguments of asss_solve_batched, already validated); the
// concatenated data of this set of handles is built on the first call and
// kept for later calls with the same handles and restart length.
asss_status_t run(int32_t nsys, const asss_handle_t* hs, const int32_t* nrhs, const double* const* B,
                  double* const* X, const asss_solve_opts_t& o, asss_info_t* infos, int maxr, hipStream_t s);

// Drop the kept data of every batch that contains h (called by asss_destroy).
void forget(asss_handle_t h);

}  // namespace batch
}  // namespace asss
