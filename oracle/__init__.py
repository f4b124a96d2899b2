"""CPU oracle for the implicit symmetric CP decomposition of moment tensors.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
calls this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the GPU path.

Everything is plain NumPy in fp64 and follows Sherman & Kolda, "Estimating
higher-order moments using symmetric tensor decomposition" (SIAM J. Matrix
Anal. Appl., 2020; arXiv 1911.03813):

* ``tensor``  - explicit d-way tensors: outer powers, inner products and
  tensor-times-same-vector (Section 2, eqs. (tensorIP), (ExpXbd),
  (ExpXbdd), (outer_product)).  Used only on tiny sizes, as brute force.
* ``fg``      - the objective and gradient: by the plain definition on
  explicit tensors (eqs. (optFunc), (gradl), (gradb)), and by the implicit
  Algorithm 2 built on Lemmas 3.1-3.5 and eq. (Y).
* ``normx``   - the constant ||X||^2 (Lemma 3.4 applied to X).
* ``lbfgs``   - the reference L-BFGS driver (Section 4 uses L-BFGS with
  memory 5; the line search and stopping tests are a stated reading).
* ``solve``   - Gaussian and randomized-range-finder starts (eq. (rrf)) and
  the restarted solve that keeps the best final f (Section 4.2).
* ``metrics`` - relative error (Section 4.2), similarity score
  (eq. (Score)) and a gauge-invariant model distance.
* ``philox``  - the Philox-4x32-10 counter-based generator and Box-Muller
  normals, written from their published definitions, for starts drawn on
  the device.
* ``stochastic`` - the sampled objective of Section 5 (Lemma 5.1) and Adam
  with the paper's epoch, learning-rate and restore schedule.
* ``corrected`` - moments corrected for spherical Gaussian noise (the
  lower-order terms of Section 4.2, left as future work in Section 6),
  derived from Isserlis' theorem for d = 3 and d = 4.

Pins (tests marked "not gpu") tie every function to something other than
itself: brute force on explicit tensors, closed forms, invariants and
textbook routines.
"""

from .fg import fg_explicit, fg_implicit, fg_bruteforce, grad_paper_explicit, magnitudes, magnitudes_explicit  # noqa: F401
from .normx import normx_implicit, normx_explicit  # noqa: F401
