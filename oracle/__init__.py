"""CPU oracle for the FDAS hot path -- TEST INFRASTRUCTURE ONLY.

Plain, slow, double-precision implementation of what the path computes, used
to prove the GPU library right.  Only the test-suite, the smoke check and the
CPU-baseline leg of the benchmark may import, call or execute anything here;
the product library never does, and it shares no code with this package.

Contents
--------
response.py  acceleration response A(q, z) (closed form through the library
             Fresnel integrals), its derivatives by Gauss-Legendre quadrature,
             the template taps and their length-L spectra.
direct.c     direct (no-FFT) correlation of the spectrum with every template,
             i.e. the f-fdot plane by its definition, OpenMP over r.
plane.py     ctypes front-end of direct.c.
peaks.py     thresholded 3x3 local maxima with the tie-break rule.
casts.py     round-to-nearest-even bfloat16 of single-precision values.
refine.py    interpolated power at continuous (r, z) and its gradient.

Pin status (what fixes each function other than itself; the tests under
``tests/test_oracle_*.py`` check every row):
  response    quadrature of the defining integral, z = 0 Fourier
              interpolation, Parseval, known limits.
  templates   unit norm, z = 0 identity, chirp injection power.
  plane       z = 0 row equals |X|^2, linearity, shift equivariance,
              brute-force FFT overlap-save on tiny inputs, injected chirp power.
  peaks       brute force on tiny planes, hand-built fixtures.
  casts       the paper's template-conversion statistics (Table 1), exact
              representable values, ties.
  refine      central finite differences, analytic peak curvature.
"""
