"""MI355X-native SIMP finite-element assembly, compliance and sensitivity
(the fast-assembly hot path of arXiv 2505.02438, SOPTX).

Submodules are imported lazily so that the seeded input generators
(``inputs``) can be used without loading the HIP library:

* ``api``      -- Pattern / Material binding of the C ABI (include/soptx.h)
* ``autograd`` -- torch.autograd.Function around assembly with the
                  hand-written backward kernel
* ``serving``  -- continuous-batching request loop
* ``inputs``   -- seeded synthetic meshes, loads, boundary conditions
"""
