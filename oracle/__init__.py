"""CPU oracle for decentralized ADMM tomography with quantized exchange.

TEST INFRASTRUCTURE ONLY.  Plain, slow, float64 NumPy code written from the
paper ("Distributed Tomographic Reconstruction with Quantization",
arXiv 2410.06106) to check the GPU path.  Only the test-suite, the smoke check
and the CPU-baseline leg of the benchmark may import it; the GPU library and its
Python binding never do, and nothing here imports them.

Modules
-------
joseph    Eq. 1-4: parallel-beam forward model as a Joseph (linear interpolation)
          system matrix, its transpose, and a dense form for tiny grids.
chord     Eq. 2 with intersection lengths: the chord of each ray through each
          pixel square (a trapezoid in the ray offset), its transpose, dense form.
admm      Alg. 1 (centralized GD), Alg. 2 (local u-update), Alg. 3 (segment
          x-update), Eq. 9 (averaging x-update), Eq. 23-24 (exchange, dual),
          Alg. 4 (the outer iteration).
kmeans    Alg. 5: scalar K-means quantizer with a fully specified, bit-exact
          fixed-point centroid update.
dct       "standard JPEG" quantizer: 8x8 orthonormal DCT-II with the luminance
          table scaled to a quality factor (no entropy coding).
metrics   Eq. 25-27 (RMSE, PSNR, NSD) and Eq. 19-20 (memory and communication).
wire      the K-means message on the wire: labels packed at ceil(log2 K) bits.
entropy   the DCT message on the wire: zigzag run-length codes with Exp-Golomb
          numbers and restart intervals of 64 blocks.
stepsize  power iteration for the step size of Alg. 2.

Parity status: every function is pinned by a ``-m "not gpu"`` test in
``tests/test_oracle_*.py`` except the long-horizon trajectory of the segment
x-update iteration (its iteration map is not contractive), which is parity
unpinned beyond single-iteration checks.
"""
