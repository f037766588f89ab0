"""Plain FP64 CPU oracle of the TDA Liouville / Davidson path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import or call anything here.  The
HIP library never links, imports or calls it, and it shares no code with the
HIP library: both consume the seeded inputs of ``synth`` and nothing else.

Modules
  liouville   grid <-> sphere maps, Eq. (evp) with Eqs. (d), (k1e), (k1d)
  screening   Eq. (tau), Eq. (tau_from_tau_u) with the low-rank Eq. (pdep)
  pairs       Eq. (overlap) and the nearsighted pair list (Sec. 2)
  davidson    block Davidson (Sec. 3, Davidson 1975) with a diagonal
              preconditioner
  eh          explicit electron-hole Hamiltonian over all empty states
              (the e-h-basis formulation of Sec. 2 / Sec. 5), built with
              its own primitives, used to pin the Liouville form
  jade        Wannier localisation: the six A^(n) matrices and the JADE
              sweeps of Sec. 2 (Eq. (wannier), Eq. (spread))
  mlp         reference forward/backward of the learned preconditioner's
              network (parity unpinned against the paper: no such network
              appears there)

Everything is float64 unless stated.
"""
