"""Plain, slow FP64 CPU oracle for the DLS block encoder.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product library
never calls it, and it shares no code with the GPU path (the GPU path lives in
``paper_2601_20113_amd``; neither imports the other).

Modules:
  dls       -- the method, step by step (plan, gather, Gram, eigensolve, rank,
               projection, quantization, lattice reconstruction, residual,
               escapes), plus the decoder (Alg. 2).
  container -- the stream format (fixed header with a per-batch offset table,
               zlib-compressed batches of 1000 blocks, Sec. 2.7.2).
  mlp       -- FP64 forward/backward of the warm-start network and its
               per-block input features.
  jacobi    -- an independent cyclic Jacobi eigensolver used to cross-check
               LAPACK on small matrices.
"""
