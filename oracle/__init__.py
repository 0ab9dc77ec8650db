"""CPU FP64 oracle for tensor-network Monte Carlo (TNMC) on the 2D +-J random-bond Ising model.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously-correct reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline``
leg of ``bench.py`` may import it.  The product path (``paper_2409_06538_amd``) never imports,
calls or links anything here, and this package imports nothing from the product path: the two
share no code (no kernels, helpers, tables or constants).  Inputs that both sides consume are
either generated here from the published Philox definition (couplings, sampling and accept
uniforms; the HIP side implements the same generator independently) or come from ``synth.py``,
which holds seeded random arrays and workload sizes but none of the method's arithmetic.

Paper: T. Chen, E. Guo, W. Zhang, P. Zhang, Y. Deng, "Tensor network Monte Carlo simulations for
the two-dimensional random bond Ising model", arXiv:2409.06538.  Each module cites the section or
equation it follows.

Modules
-------
philox       Philox4x64-10 counter-based generator (Salmon et al., SC'11) and 53-bit uniforms.
instance     +-J couplings with antiferromagnetic probability p; Nishimori-line inverse temperature.
energy       E(s) = -sum J_ij s_i s_j with open boundaries (Sec. III A, Eq. (10)).
exact        Brute-force enumeration and exact row transfer matrix (independent of the TN code).
envbuild     Boundary-MPS environments: row MPO applied to an MPS, QR + SVD compression to chi.
sampler      Whole-lattice proposals from the environments with log q(s); teacher-forced log q.
accept       Independence Metropolis chain (Eq. (3) with g(s'|s) = q(s')).
observables  Energy, magnetisation, edge magnetisation and replica overlap (Sec. III C).
pbc          Periodic lattices by a frozen row and column per step; the open block and its fields.

Parity pins (what fixes each part independently of this code) live in ``tests/test_oracle_*.py``.
"""
