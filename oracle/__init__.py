"""CPU FP64 oracle for the neural-collision-operator (NCO) lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or calls
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, table or
helper with the HIP library; the two meet only through the seeded input
generators in ``paper_2412_08229_amd.inputs`` (which hold none of the method's
arithmetic) and through the tests that compare them.

Every function is a plain, slow, literal transcription of the operation the
paper defines, in float64, with the passage it follows named in its docstring:

* ``lattice``     - D3Q27 velocities and weights, the Hermite moment matrix M
                    (Sec. II.B, definition of M), the octahedral group O_h and
                    its population permutations (Sec. II.B, equivariance).
* ``collision``   - equilibrium (Eq. EquilibriumDistribution), macroscopic
                    moments, BGK, fixed-rate moment relaxation, the invariant
                    network N_Phi (Eq. gconv_m), the rate squashing and the
                    NCO collision (Eq. omegatheta), Kupershtokh forcing.
* ``step``        - pull streaming + collision (Sec. II.A, lattice Boltzmann
                    equation).
* ``observables`` - mass/momentum/kinetic-energy sums and the energy spectrum
                    E(k) (Sec. "Learning Task", loss on E(kappa)).
* ``brute``       - a second, independent scalar-loop implementation of one
                    step, for brute-force checks on tiny grids.
* ``reduced``     - the reduced Taylor-Green domain of Appendix A: the cube
                    [0, pi/2]^3 stepped by unfolding it to the periodic box
                    through the vortex's symmetry group.
* ``restrict``    - fine-to-coarse restriction by acoustic scaling (Sec.
                    "Learning Task").
* ``adjoint``     - reverse-mode derivative of an unrolled run with respect to
                    the network parameters (what Adam consumes in Sec.
                    "Learning Task").

Readings where the paper is silent or garbled are stated at each use.
"""
