"""FP64 CPU oracle for synthetic Shack-Hartmann interaction matrices.

TEST INFRASTRUCTURE ONLY.  Nothing in the library's compute path imports, calls
or links this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP implementation.

Each function is the plain, slow, obviously-correct definition of one step of
the method, evaluated in float64 on the (float32) inputs upcast:

* :mod:`oracle.geometry` - composite affine map (paper Sec. 2.1: DM and WFS
  transforms multiplied into one matrix) and its derivative maps;
* :mod:`oracle.warp`     - single bilinear resampling of an IF onto the WFS grid
  (Sec. 2.1, "interpolated exactly once"; Sec. 2.2 absolute sub-pixel alignment);
* :mod:`oracle.slopes`   - central finite differences at every pupil pixel and
  the mean over each subaperture (Sec. 2.2);
* :mod:`oracle.im`       - interaction matrix, its Jacobian with respect to the
  misregistration parameters, and the vector-Jacobian product;
* :mod:`oracle.misreg`   - probe slopes and the Gauss-Newton misregistration fit
  (the online-tracking use of Sec. 5);
* :mod:`oracle.mlp`      - FP64 forward/backward/Adam of the small estimator MLP.

Parity status: every function is pinned by closed forms, invariants or
brute-force loops in ``tests/test_oracle_*.py``.  Physical fidelity against a
diffractive model (Sec. 3) is parity unpinned: no diffractive simulator is here.
"""
from . import geometry, warp, slopes, im, misreg, mlp  # noqa: F401
