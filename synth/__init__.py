"""Seeded synthetic inputs (atoms, grid-sampled localised functions, S, H, K^v, K^c,
the block pattern M and random initial guesses).  Holds none of the response-operator
arithmetic; both the CPU oracle and the GPU library read what it produces."""
from .system import Config, FunctionSet, System, build_system, atom_distances  # noqa: F401
from . import configs  # noqa: F401
