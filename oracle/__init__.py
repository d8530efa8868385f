"""FP64 CPU oracle (test infrastructure only; see fobf_oracle.py)."""
from .fobf_oracle import *  # noqa: F401,F403
from .fobf_oracle import (algorithm1, blur_weight, brute_bf, brute_bf_points,
                          conv_zero, cosine_series, design_matrix, fit, fit_E,
                          fourier_direct, gaussian_range, kernel_maxdev,
                          max_abs, prop1_bound, psnr, spatial_radius,
                          spatial_taps)
