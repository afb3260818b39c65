"""Seeded synthetic inputs shared by the oracle-side tests and the GPU path.

This package holds workload *data* (ranges, true parameter values, start
values, the synthetic resonance table) and seeded random sampling only.  It
contains none of the likelihood arithmetic: where a sample must follow the
model density (accept-reject for the Dalitz workloads) the caller passes the
density in as a function.
"""
from .configs import *  # noqa: F401,F403
from .generators import *  # noqa: F401,F403
