// ens_lambda.h -- lambda densities given by their characteristic function, and
// the mixture with weights from a tabulated lambda density.
// Not part of the public ABI (include/ens.h is).
#pragma once

#include "ens_internal.h"

namespace ens {

// Largest table the characteristic-function inversion accepts.
constexpr int kMaxCfTable = 1 << 16;

// P_j = Re sum_k psi_k e^(-2 pi i k j / M) / (M h), psi_k = phi_k e^(-i omega_k lam0):
// the density on lam0 + j h from phi_k (interleaved complex, M values) at
// omega_k = 2 pi f_k / (M h), f_k = k for k < M/2, k - M otherwise.
hipError_t launch_cf_invert(const double *phi, int M, double lam0, double h, double *pdf, hipStream_t s);

// launch_mix with mode 4 reading member weights from a tabulated lambda
// density (M samples on lam0 + j h); other modes ignore the table.
hipError_t launch_mix_table(const MemberDev *const *members_host, const double *lambdas, int count,
                            const ens_hist_desc &h, double c, double Z, int mode, double q_sigma, const double *table,
                            int table_len, double lam0, double dlam, double *out, void *scratch, hipStream_t s);

}  // namespace ens
