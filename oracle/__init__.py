"""CPU oracle for SFFT-based homogenization -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct FP64 implementations of what the hot path
computes, written from the paper (Hauck, Kabel, Ali, Gauger, "SFFT-based
homogenization", arXiv 2412.11566):

* ``oracle.dense``  -- the FFT-based basic scheme (Sec. 2, Alg. 1) on dense
  voxel fields, the Green operator tables (App. A: direct and staggered
  grid schemes of Table 3), the
  effective stiffness from unit load cases (Sec. 2), and gradient references
  (energy identity, central finite differences, dense adjoint).
* ``oracle.qtt``    -- a dense-vector quantized-tensor-train reference:
  TT-SVD, TTO x TT contraction, raise-to-TTO (App. C), TT-rounding (Sec. 3,
  eq. rounding_condition_tt), the SFFT operator from the reduced QFT
  (Sec. 4.1), the Green TT in the SFFT momentum convention (Sec. 4.3) and the
  SFFT-based homogenization loop (Alg. 2).
* ``oracle.amen``   -- the AMEn-adapted approximate TTO x TT product
  (App. B): Galerkin core updates, residual enrichment, QR.
* ``oracle.plane``  -- the basic scheme in plane strain (Voigt 3) on N x N
  pixels, both Green schemes, and its C_eff gradients.
* ``oracle.unrolled`` -- the exact derivative of the C_eff returned after a
  fixed number of updates (reverse mode of Alg. 1), 3D and plane strain.
* ``oracle.bounds`` -- closed forms: isotropic stiffness, laminate effective
  stiffness, Voigt/Reuss and Hashin-Shtrikman bounds.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP path
(``paper_2412_11566_amd``) and neither imports the other; both consume the
seeded inputs of ``microstructures``.

Pins: every function here is checked in ``tests/test_oracle_*.py`` against
facts fixed by the paper or by mathematics (closed forms, invariants,
brute force on tiny inputs).  Functions without such a pin say
"parity unpinned" in their docstring.
"""
