"""CPU reference implementation (oracle) of linearized OSB-PD.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the GPU library never does, and
the two share no code.  The only module both sides read is ``pd_inputs``
(seeded geometry, loads and material tables; no peridynamic arithmetic).

Contents:
  pd_oracle.c  -- FP64 loop solver (family search, weighted volume, critical
                  stretch, notch cuts, dilatation, pair force, explicit
                  update, damage, energy, power iteration for the stable step)
  oracle.py    -- ctypes wrapper (class Oracle) and build()
  dense.py     -- the paper's matrix form (C_e, C_theta, K_theta, K_e and
                  K = K^v + K^d) assembled densely with numpy for tiny grids
  make_params.py -- writes pd_inputs/params.json (time steps, twist rates)
"""

from .oracle import Oracle, build, lib, critical_stretch, constants  # noqa: F401
