"""CPU oracle for the CS decomposition hot path (test infrastructure only).

This package is a plain, slow, obviously-correct FP64 CPU statement of what
the GPU library computes, written from Gawlik, Nakatsukasa & Sutton, "A
Backward Stable Algorithm for Computing the CS Decomposition via the Polar
Decomposition" (arXiv 1804.09002).  It exists to check the HIP path:

* only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
  ``bench.py`` may import it;
* it shares no code with the GPU library (no kernels, headers, helpers,
  coefficient generators, pre- or post-processing) and never imports it;
* the product path never calls it.

Modules
-------
``zolotarev``  Zolotarev coefficients from their elliptic-function definition
               (mpmath, 60 digits) and the degree choice (Sec. 5).
``zolo_pd``    The two Zolo-pd iterations as the rational matrix function they
               define (Sec. 5), for parity of the GPU iterates.
``csd``        Algorithm 1 / Algorithm 3 with the classical backward-stable
               polar (SVD) and symmetric eigensolver (LAPACK), Remarks (iii),
               (vi), (vii).
``grad``       Closed-form gradients of the angles and the polar factors.
``metrics``    Residual, orthogonality and distance-to-partial-isometry (Sec. 2.1).
"""
