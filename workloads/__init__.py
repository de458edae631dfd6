"""Seeded synthetic inputs shared by the CPU oracle, the tests and the bench.

Only input data lives here (meshes, closed-form initial/boundary fields and the
workload table); none of the method's arithmetic does.
"""
from .meshes import DIRICHLET, NATURAL, unit_square, channel_cylinder, disc  # noqa: F401
from .flows import taylor_green, cavity_lid, channel_inflow, jobelin_disc  # noqa: F401
from .configs import Workload, WORKLOADS, get_workload  # noqa: F401
