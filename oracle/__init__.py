"""CPU FP64 oracle for the band-limited FMM matrix-vector product.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call, link or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (``paper_1606_07652_amd``); the only common module is ``workloads``, which
draws seeded random inputs and holds none of the method's arithmetic.

Contents (each function cites the passage of Zhao & Stoll, "A Fast Multipole Method
based on Band-limited Approximations for Radial Basis Functions", arXiv 1606.07652,
that it writes out):

* ``rbf``       radial kernels (Tab. "Global functions") and the Fourier transform
                convention of eq. (5)/(6).
* ``direct``    oracle A: the plain O(N^2) sum of eq. (1), in C (OpenMP) and numpy.
* ``bandlimit`` the band-limited kernel Phi_sigma (eq. 16/28) in closed form for the
                Gaussian, the tensor quadrature of eq. (29) and its periodisation.
* ``tree``      quantisation, Morton order, adaptive boxes, neighbour (near) lists.
* ``splitref``  oracle B: the near/far split of eq. (38) evaluated by brute force.
* ``params``    the rule that turns a tolerance into (band limit, nodes, coarse level).
* ``bands``     the translation factor from kernel samples (eq. "M2Loperator"), and the
                split of the multiquadric kernels into Gaussian-mixture scale bands that
                gives them per-level band limits (section 4.1).
* ``gmres``     restarted GMRES (cited in section 1) with modified Gram-Schmidt.
* ``precond``   block-Jacobi and the FP64 forward/backward of the per-block network used as
                a right preconditioner (not in the paper).
* ``poly``      interpolation with polynomial terms for the conditionally positive
                definite kernels.
* ``lagrange``  Lagrange interpolation between frequency grids (section 4.1).

Parity status per function is listed in each module header.
"""
