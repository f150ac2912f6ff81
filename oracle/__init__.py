"""Plain FP64 CPU oracle for three-site-gate TEBD on the Bose-Hubbard chain.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, as the independent checker of
the GPU library.  It shares no code with the library; both are fed from the
seeded generators in ``workloads``.

Contents
--------
model      Eq. (1) Hamiltonian, its exact split into three-site terms and
           the gates exp(-i h_j tau).
tebd       MPS in (B = Gamma Lambda, Lambda) form, the three-site gate update
           with two truncated SVDs, the second-order (Strang) step over the
           three commuting gate groups, the fourth-order step composed of
           five Strang steps (Suzuki's weights), and local measurement of n_j,
           C_j = <b_j^+ b_{j+1}> and D_j = <b_j^+ b_{j+2}> (Eqs. (4), (7)).
reference  Independent checks of the above: dense state vectors evolved by
           the same gate layers or by exp(-iHt), the single-particle
           propagator of the non-interacting chain, and the bulk closed
           form 1/2 (1 +- J0(4t)) of the free CDW quench.

Every function is written for readability, in FP64, with NumPy/SciPy
primitives (eigh, svd, expm) as its only library steps.

Parity status: every function here is pinned by a ``-m "not gpu"`` test
against brute force, closed forms, invariants or special cases (see
``tests/test_oracle_*.py``).  No function is "parity unpinned".
"""

from . import model, tebd, reference  # noqa: F401
