"""FP64 CPU oracle of the meshfree likelihood (arXiv:2508.04172).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The library under
``paper_2508_04172_amd`` never imports, links or executes anything here, and
this package shares no code with it: both are written independently from the
paper's definitions and the readings recorded in the design notes.

Modules:
  physics     -- inner product, PSD, synthetic waveform family, chirp-time
                 coordinates, spin-weighted harmonics, antenna patterns
                 (Sec. II A-B, Eqs. innerProduct, h_spherical_harmonic_basis,
                 hplus_hcross_decomposed1/2, projected_h_fd, metric_coords)
  startup     -- metric ellipsoid, Halton nodes, overlap time series, mode
                 overlaps, SVD basis, RBF solve (Sec. II C, Eqs. MisMatch,
                 conjugation_symmetry, rbfcoeff, SVD)
  likelihood  -- brute-force ln L (Eq. logl_basic), mode-factorised ln L
                 (Eq. logl_complete, corrected), meshfree online evaluation
                 (Sec. II D)
  mlp         -- surrogate network forward/backward/Adam in FP64

Every function is plain numpy in float64, vectorised where it does not
obscure the definition; nothing is blocked, fused or reordered.
"""
