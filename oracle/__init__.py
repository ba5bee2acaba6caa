"""FP64 CPU oracle for two-link staggered Gaussian smearing (test infrastructure).

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library never calls it and
shares no code with it.

* ``oracle.core``   -- ctypes wrapper over ``oracle.c`` (plain FP64 C loops).
* ``oracle.checks`` -- independent closed forms: the exact free-field
  smearing kernel (by a discrete Fourier sum and by a multinomial sum of
  +-2 walks, also in exact rational arithmetic) and dense-matrix helpers.
* ``oracle.build``  -- compiles ``oracle.c`` into ``liboracle.so`` with gcc.
"""
