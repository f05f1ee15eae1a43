"""MI355X-native quasi-Newton / L-BFGS implicit-Euler step for tetrahedral
hyperelastic meshes (Liu, Bouaziz, Kavan 2016), as a HIP library with a thin
Python binding.

    from paper_1604_07378_amd import qnsim
    sim = qnsim.Sim()
    sim.set_mesh(rest, tets); sim.set_pinned(pinned); sim.set_materials(mats)
    sim.prepare(h)
    x, v, stats = sim.step(x, v, h)
"""
from . import qnsim  # noqa: F401
from .qnsim import Sim, QnsimError, load_library, sim_from_workload  # noqa: F401
