// kernels_lambda.hip -- a lambda density from samples of its characteristic
// function exp(K(i omega; Z)): the cumulant generating function at imaginary
// argument, inverted by a discrete Fourier transform.
#include "ens_lambda.h"

namespace ens {

// One thread per output sample j, terms k in increasing order (deterministic).
// The phase of the DFT kernel is taken from the exact integer k j mod M, the
// shift by lam0 from omega_k lam0.
__global__ void __launch_bounds__(256) k_cf_invert(const double2 *__restrict__ phi, int M, double lam0, double h,
                                                   double *__restrict__ pdf) {
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= M) return;
    const double two_pi = 6.283185307179586476925286766559;
    double acc = 0.0;
    for (int k = 0; k < M; k++) {
        const int f = k < M / 2 ? k : k - M;                       // frequency index
        const double omega = two_pi * (double)f / ((double)M * h);
        const long long kj = ((long long)k * j) % M;
        const double th = -(omega * lam0) - two_pi * (double)kj / (double)M;
        double sn, cs;
        sincos(th, &sn, &cs);
        const double2 p = phi[k];
        acc += p.x * cs - p.y * sn;
    }
    pdf[j] = acc / ((double)M * h);
}

hipError_t launch_cf_invert(const double *phi, int M, double lam0, double h, double *pdf, hipStream_t s) {
    if (M < 2 || M > kMaxCfTable || !(h > 0) || !phi || !pdf) return hipErrorInvalidValue;
    k_cf_invert<<<(M + 255) / 256, 256, 0, s>>>(reinterpret_cast<const double2 *>(phi), M, lam0, h, pdf);
    return hipGetLastError();
}

}  // namespace ens
