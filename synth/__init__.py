"""Seeded synthetic inputs shared by the oracle's tests and the HIP path.

This module holds none of the method's arithmetic: it only draws inputs
(initial polymer conformations, request streams) and names the workloads.
"""
from .inputs import polymer_walk, request_stream  # noqa: F401
from .workloads import PAPER_POLYMER, WORKLOADS, m_opt, sweeps_per_iteration  # noqa: F401
