"""FP64 CPU oracle for assembled canonical-tensor lattice summation.

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously-correct
restatement of what the GPU library computes, written from the paper
(Khoromskaia & Khoromskij, "Grid-based lattice summation of electrostatic
potentials by assembled rank-structured tensor approximation", arXiv 1405.2270).
Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import it. The product path never calls it, and it shares no
code with the HIP library: the only module both sides use is ``workloads``,
which draws seeded inputs and holds none of the method's arithmetic.

Modules
-------
quadrature  sinc rules for the Gaussian integral of 1/r (Sec. 2.1, eqs. laplace,
            sinc_Newt, hM) and the rule-S calibration against the exact tensor.
projection  1D Gaussian cell integrals b_i(t) (eq. galten_int) and their
            derivative with respect to the charge position.
prism       exact Galerkin tensor P (eq. galten) by the closed-form potential of
            a uniform box, with a Gauss-Legendre far field.
lattice     grid/lattice geometry, the direct canonical sum over every image
            (eqs. core_tens, EwaldSumE, EwaldSumP), the assembled sums
            (Theorem 3.1, eq. EwaldTensorM0, Lemma 3.2), and 3D brute force.
canonical   canonical-format operations (Appendix: eqs. CP_form, scal, had,
            conc): reconstruction, scalar product, Hadamard product.
physics     energy against a charge density, forces (adjoint and central
            finite differences), Richardson extrapolation (Sec. 3.2).
qtt         quantics-TT compression of assembled vectors (Sec. 4, eq.
            EwaldTensorQTT) by TT-SVD, and its expansion.

Parity status of every function is listed in its module header.
"""
