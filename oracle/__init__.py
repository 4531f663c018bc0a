"""CPU oracle for the function-setup path (test infrastructure only).

A plain, slow, obviously-correct CPU implementation of what the GPU path
computes: block fingerprints, the deduplication partition and its byte
accounting, the refcount/eviction state, the MLP and stencil function bodies
and the setup-overlap model.  Floating point is evaluated in float64.

Only the test-suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the GPU library
(no kernels, headers, constants or helpers); the only module both sides read
is the seeded input generator ``paper_2404_14691_amd.synth``.

Parity status per function (what pins it) is listed in each module header.
"""
