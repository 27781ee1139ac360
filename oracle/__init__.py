"""CPU FP64 oracle for the spin-coherent-state Monte Carlo singlet yield.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, tables or constants); the only module both sides
read is the seeded workload generator, which holds none of the method's
arithmetic.

What it computes (Lewis, Fay & Manolopoulos, arXiv:1612.09517):

* ``spin``      -- the radical-pair Hamiltonian, Haberkorn operator and the
                   singlet/triplet projectors (Sec. II, Eqs. 1-4), as dense
                   Kronecker-product matrices.
* ``coherent``  -- spin coherent states (Sec. III, Eq. 15) and their product
                   initial wavepackets |S> x |Omega_1..Omega_N> (Eq. 18-19).
* ``philox``    -- Philox4x64-10 (Salmon et al., SC'11) and the uniform-on-the-
                   sphere sampling of each nuclear direction (Eq. 18).
* ``yields``    -- the exact finite-horizon single-wavepacket yield
                   phi_S = k_S int_0^T <S,Omega;t|P_S|S,Omega;t> dt
                   (Eq. 22 with the propagator of Eq. 13) as the quadratic form
                   of one per-field operator X_T, and the deterministic trace
                   of Eq. 14 (rho(0) = P_S / Z).
* ``large``     -- the same yield for state sizes too large for dense
                   matrices, from sparse operators and an exact augmented
                   linear system integrated by a library matrix-exponential
                   action.
* ``stats``     -- the Monte Carlo mean and its error eps = sigma/sqrt(M)
                   (Eq. 23).
* ``mlp``       -- FP64 forward/backward of the control-variate network.

Parity status of every function is stated in its docstring; all are pinned by
the ``-m "not gpu"`` tests against closed forms, invariants, library routines
or brute force.
"""
