"""Plain, slow, FP64 CPU oracle for the 1D/2D/3D nonuniform FFT hot path (types 1, 2, 3).

This package is TEST INFRASTRUCTURE.  Only the test-suite (``tests/``), the
smoke check in ``__graft_entry__.smoke`` and the CPU-baseline leg of
``bench.py`` may import it.  The GPU library never imports, links or calls it,
and it shares no code, header, table or constant generator with the GPU
library; only the seeded input generators in ``workloads.py`` (which hold none
of the method's arithmetic) feed both sides.

Modules
  params   kernel width/beta/fine grid selection (Sec. II), the ES kernel
           (eq. es) and its Fourier transform by Gauss-Legendre quadrature,
           correction factors (Sec. II-A step 3), density (eq. den)
  direct   exact exponential sums (Sec. I, eqs. 2d1 and 2d2; and the type 3 sum) in
           C/OpenMP
  nufft    the three-step type 1 / type 2 algorithm (Sec. II-A, II-B) in FP64, and the
           type 3 reduction built on it
  binsort  bin keys, the stable bin-sort permutation and the subproblem list
           (Sec. III-A)
  grad     reference gradients of the type 1 and type 2 sums
  mlp      reference MLP forward/backward/Adam used to check the selector
"""
