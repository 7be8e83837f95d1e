"""Plain, slow FP64 CPU oracle for one-site TDVP-PS (and TDVP-MU, two-site
TDVP-PS and P&C-RK4).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call or
execute anything here; only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  The oracle shares no code with the HIP path: it
builds its own Hamiltonian, its own MPO (a different channel construction
from the library's), and does every contraction with numpy, every QR with
numpy.linalg.qr (or the Cholesky QR written out in mps.py), every SVD with
numpy.linalg.svd, every small exponential through numpy.linalg.eigh or
scipy.linalg.expm, and every Runge-Kutta integration with scipy's RK45.

Modules
  model   Frenkel-Holstein Hamiltonian: dense matrix and MPO (Sec. II.C)
  mps     canonical forms, environments, local operators, observables
          (Sec. II.A, eq:QR, eq:tdvp1_h, eq:tdvp1_H, eq:tdvp2_D)
  krylov  Lanczos approximation of exp(z A) x (Sec. II.A.2, TDVP-PS)
  ps      the projector-splitting time step (eq:ps_trotter, eq:tdvp2_C/D)
  ps2     the two-site projector-splitting step (Sec. II.A.2, after
          eq:tdvp2_D; eq:SVD)
  dense   exact propagation and dense-projector forms of the one- and
          two-site PS steps
  mu      TDVP-MU with matrix-unfolding regularisation, VMF/RK45 and
          second-order CMF (eq:tdvp1_C, eq:tdvp1_mu_L, eq:reg2)
  pc      P&C-RK4 (Sec. II.A.1: eq:RK4, eq:mpo-apply, eq:mps+mps, eq:SVD)

Pins: every function above is checked in tests/test_oracle_*.py against a
closed form, a library routine on tiny inputs, brute force, or an exact
invariant.  TDVP-MU vs TDVP-PS agreement is "parity unpinned" (the paper
states it only qualitatively).
"""
