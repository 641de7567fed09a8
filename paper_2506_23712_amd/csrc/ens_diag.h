// ens_diag.h -- launchers of the spectral diagnostics (kernels_diag.hip).
// Not part of the public ABI (include/ens.h is).
#pragma once

#include "ens_internal.h"

namespace ens {

// Workgroups per z-mode plane in the first passes of the spectrum and the scales.
constexpr int kDiagParts = 4;
// Shells that can hold retained modes (|m| <= sqrt(3) K): 0 .. spectrum_shells(K) - 1.
inline int spectrum_shells(int K) {
    long long r = 0;
    while ((r + 1) * (r + 1) <= 3LL * K * K) r++;
    return (int)r + 2;
}
// FP64 partial sums the spectrum needs in a member's partials area.
inline long long spectrum_partials(int K) { return (long long)(2 * K + 1) * kDiagParts * spectrum_shells(K); }
// ... and the integral scales.
inline long long scales_partials(int K) { return 2LL * (2 * K + 1) * kDiagParts; }

// Shell energy spectrum of one member into `out` (device, nshell doubles).
hipError_t launch_spectrum(int prec, const MemberDev *mem, int K, int nshell, double *out, hipStream_t s);
// E, u', integral length L and integral time T of one member into `out`
// (device, 4 doubles); uses the member's FP64 partials (scales_partials(K)).
hipError_t launch_scales(int prec, const MemberDev *mem, int K, double *out, hipStream_t s);
// Set diag.E of one member to the energy of its current field (the scales'
// passes, with DevState::pad as their output); `st` is the member's DevState.
hipError_t launch_refresh_energy(int prec, const MemberDev *mem, DevState *st, int K, hipStream_t s);
// Copy member src onto the finer grid of member dst (retained modes of src,
// zeros elsewhere), clear dst's RK register, carry time and diagnostics.
hipError_t launch_refine(int prec_src, int prec_dst, const MemberDev *src, const MemberDev *dst, int n_dst,
                         hipStream_t s);

}  // namespace ens
