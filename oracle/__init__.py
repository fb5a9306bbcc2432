"""CPU oracle of the FFT polyspectrum estimator -- TEST INFRASTRUCTURE ONLY.

Plain, slow, FP64 implementation of what the GPU path computes, written from
Watkinson et al. 2017 (arXiv:1705.06284), Section 2: the forward DFT of
Eq. (DeltaFFTtoDelta), the shell bins of Eq. (gen_Nspec3) and the direct sums
over closed k-vector tuples that Eqs. (Jeong_gen), (Jeong_PS) and (Jeong_BI)
evaluate with FFTs.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import, call, link or execute anything in this directory.
The product library never does, and nothing here imports the product.

Pins (each function is checked against something other than itself in
``tests/test_oracle_*.py``): brute-force DFT and numpy.fft, brute-force tuple
counts over the whole grid, plane-wave closed forms for B, P and T, the
discrete skewness identity, Parseval, translation / rotation / scaling
invariance, strict = modulo-N closure below N/3, and the Gaussian zero mean.
"""
from .polyspec import (  # noqa: F401
    Spectrum,
    bin_mask_table,
    bispectrum,
    build,
    candidate_triplets,
    closed_triplets,
    collapsed_quads,
    dft3,
    dft_matrix,
    freq,
    mode_counts,
    power_spectrum,
    prepare,
    quad_counts,
    shell_modes,
    squared_edges,
    triangle_counts,
    trispectrum,
    trispectrum_diag,
    trispectrum_diag_connected,
)
