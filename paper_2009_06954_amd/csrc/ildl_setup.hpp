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

// J_tilde = Lcal^-1 J_hat_p Lcal^-T formed explicitly on the device (after
// ildl_setup): column j is the two triangular solves around J_hat_p applied
// to e_j; the stored operator is (C - C^T) / 2 of those columns C, exactly
// skew, row-major, in FP64 and FP32, with row blocks for the fused inner
// step (h->J64, h->J32 with dense set).  The outer operator A_chk = Lcal^-1
// A_hat_p Lcal^-T likewise, row-major, and its transpose (h->il.A_rows,
// AT_rows).  Sets h->il.explicit_j.
void ildl_explicit_jtilde(asss_handle_s* h, hipStream_t s);

}  // namespace host
}  // namespace asss
