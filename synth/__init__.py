"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench."""
from .ncp_jacobian import CONFIGS, NCPSystem, make_config, make_poisson, make_system, random_vector  # noqa: F401
from .ncp_problem import NCPProblem, make_ncp_problem  # noqa: F401
