"""MI355X-native ensemble DNS for the method of arXiv 2506.23712.

An ensemble of forced periodic-box Navier-Stokes simulations (Fourier
pseudo-spectral, 2/3 truncation, low-storage integrating-factor RK3), each
member injecting energy at exp(lambda) * eps_ref, with velocity-gradient
statistics (A_ij moments, joint Q-R histogram, dissipation and enstrophy
histograms) and their Gaussian-in-lambda mixture.  All arithmetic runs in
libensdns.so (hand-written HIP for gfx950); see include/ens.h for the C ABI.
"""
from ._lib import EnsError, lib
from .ensemble import Ensemble, HistSpec, Member, MemberSpec, fft_pencils, lambda_pdf_from_cf

__all__ = ["Ensemble", "HistSpec", "Member", "MemberSpec", "EnsError", "fft_pencils", "lambda_pdf_from_cf", "lib"]
