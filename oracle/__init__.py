"""Plain FP64 CPU oracle for the micromagnetic hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
C ABI or its Python binding) may import, call or link anything in this
package; only the tests, the smoke check and the CPU-baseline leg of the
benchmark use it.  It shares no code with the GPU path.

It is a slow, literal implementation of the finite-difference method of
Moreels et al., "mumax+: extensible GPU-accelerated micromagnetics and
beyond" (arXiv 2411.18194), Methods section:

* ``tensor``  - cell-averaged demagnetising tensor (Methods, "Magnetostatic
  field": analytic Newell result near, asymptotic result far; a cell-pair
  quadrature bridges the two, see the module docstring).
* ``demag``   - zero-padded FFT convolution and its brute-force direct sum.
* ``fields``  - exchange (Eq. 3), interfacial DMI (Eq. 4 special case with
  the boundary condition of Eq. 5), anisotropy, Zeeman, magnetoelastic field
  (Eq. 9).
* ``elastic`` - strain, stress, elastic and magnetoelastic forces (Eq. 7, 8).
* ``torque``  - LLG torque (Eq. 2) and Zhang-Li spin-transfer torque.
* ``rk``      - Dormand-Prince 5(4) (Table 2) with step control.
* ``system``  - the assembled problem: effective field, energies, RHS, runs.

Parity status of every function is listed in the module docstrings; the
Zhang-Li prefactor and the step-controller constants are definitions of this
build ("parity unpinned": only GPU/oracle agreement is checked for them).
"""
