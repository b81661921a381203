// Setup of the general incomplete LDL^T preconditioner (definitions in
// ildl_setup.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "handle.hpp"

namespace asss {
namespace host {

// From A_hat = Abar S (CSR in Abar's index space): M_hat and J_hat, the
// Bunch-Kaufman incomplete LDL^T of M_hat with h->il.opts, the scaled factor,
// U_r and Sigma_r (host, kept in h->il), and the device data of the scaled
// system in the factorization's positions.  Throws Error / HostError.
void ildl_setup(asss_handle_s* h, const Csr& Ahat, hipStream_t s);

}  // namespace host
}  // namespace asss
