"""FP64 CPU oracle for the adaptive-multigrid Wilson-Dirac solve.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import or call anything in this package.  The GPU library never routes
through it, and it shares no code, table or helper with the HIP path: the
two meet only in the seeded inputs of ``synthetic`` and in the conventions
written out below.

Everything is plain numpy in complex128.  Each function cites the passage of
Clark et al., "The removal of critical slowing down" (Lattice 2008) it
follows.  Where the paper is silent, the reading taken is stated in the
docstring; the full list of readings is kept with the design notes.

Conventions shared with the GPU path (a specification, not code):

* dims ``(Lx, Ly, Lz, Lt)``; ``mu`` = 0,1,2,3 = x,y,z,t; canonical arrays are
  ``[t, z, y, x, ...]`` (x fastest).
* chiral gamma basis, ``gamma5 = diag(1, 1, -1, -1)``; chirality + is spins
  {0,1}, chirality - is spins {2,3}.
* ``(D psi)(x) = (4 + m) psi(x) - 1/2 sum_mu [(1 - gamma_mu) U_mu(x) psi(x+mu)
  + (1 + gamma_mu) U_mu(x-mu)^dagger psi(x-mu)]``, periodic in x, y, z and
  antiperiodic in t (a hop across the t boundary carries a factor ``t_bc``).
* a field at multigrid level ``l`` has per-site dof ``[2, n]``: chirality
  first.  At the fine level ``n = 6`` is (spin within chirality, colour), so
  a spinor ``[..., 4, 3]`` reshaped to ``[..., 2, 6]`` is its chirality split.
* coarse dof order at every level: ``(chi, k)``, index ``chi * Nv + k``.
* ``<a, b> = sum conj(a) * b``.
* 2d workload (``qed2d``): dims ``(Lx, Lt)``, arrays ``[t, x, ...]``; links
  ``[t, x, mu]`` of modulus one; spinors ``[t, x, 2]`` with ``gamma_0 = sigma_1``,
  ``gamma_1 = sigma_2``, ``gamma5 = sigma_3``; coarse stencils of 5 (D) or 9
  (``D^dagger D``) offsets ``(d_x, d_t)`` in the order of ``qed2d.OFFSETS_NORMAL``.

Parity status: every function here is pinned by a test in ``tests/`` against
a closed form, an invariant, a brute-force construction or a library routine,
except where its docstring says "parity unpinned".
"""
