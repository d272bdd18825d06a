"""Seeded synthetic inputs shared by the oracle and the GPU path.

Holds no simulator arithmetic; see workloads.gen and workloads.configs."""
from .scenario import (KID, Filters, Scan, Scenario, Screen, Source,  # noqa
                       Spectral, Stage, Telescope)
from . import gen, configs  # noqa
