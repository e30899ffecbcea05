"""MI355X-native Monte Carlo geometry tracking through nested CSG universes.

* ``synth``  -- seeded synthetic geometry inputs (flattened arrays)
* ``gt``     -- binding of the HIP library ``libgt.so`` (C ABI in include/gt.h)
* ``build``  -- in-tree hipcc build of ``libgt.so`` for gfx950
"""

__all__ = ["synth", "gt", "build"]
