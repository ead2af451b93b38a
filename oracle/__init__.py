"""Plain FP64 CPU oracle for the SVGD / sSVGD full-waveform-inversion hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
this package: only the test suite, the smoke check and the CPU-baseline leg of
the benchmark do.  It shares no code with the HIP library (no kernels, headers,
helpers, tables or constants) and never imports it.

Modules
-------
fwi    -- 2-D acoustic finite-difference forward simulation, its exact discrete
          adjoint and the adjoint-state velocity gradient (paper section 4.2,
          likelihood eq:likelihood; adjoint method of section 3).
svgd   -- RBF kernel with median bandwidth, SVGD update (eq:rbf, eq:phi_mean),
          sSVGD update with Cholesky-correlated noise (eq:stochastic_svgd,
          eq:matrixDK, eq:noise_term), uniform-prior clip (section 3),
          posterior statistics (section 4).
philox -- Philox4x32-10 counter-based generator (Salmon et al., SC'11) and the
          Box-Muller transform, for noise drawn inside the library.
cpu_pool -- process-pool runner that spreads (particle, shot) pairs over host
          cores; used to time the oracle as a CPU baseline.
"""
