"""CPU oracle for the FDFD design iteration -- test infrastructure only.

Importable by the tests, by the smoke check and by the benchmark's CPU-baseline
leg; never by the GPU library.
"""
from .fdfd_oracle import *  # noqa: F401,F403
