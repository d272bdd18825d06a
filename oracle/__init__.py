"""FP64 CPU oracle for the time-ordered-data simulator -- TEST INFRASTRUCTURE.

This package is a plain, slow, obviously-correct NumPy implementation of
what the simulator computes, written from the paper's section 2 (source and
atmosphere, telescope and instrument, scanning, radiative-transfer cascade,
noise, output).  It exists only to check the GPU path: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it.  The
product path never calls it and shares no code with it; the only module both
sides use is `workloads`, which draws inputs and holds no simulator
arithmetic.

Modules
  physics  constants, Johnson-Nyquist power, telescope and stage efficiencies
  filters  Lorentzian, filterbank and user-matrix channel responses
  philox   Philox4x32-10 counters, uniforms and Box-Muller normals
  tod      pointing, screen and source sampling, cascade, contraction,
           photon noise, TOD assembly
  pink     Timmer-Koenig 1/f series
  skydip   brightness-temperature scale by a simulated skydip
  reduce   common-mode atmosphere subtraction and inverse-variance gridding
  inputs   aperture field, far field, source-beam and screen-footprint convolutions
"""
from . import physics, filters, philox, tod, pink, skydip, reduce, inputs  # noqa: F401,E501
