"""Shared pytest configuration.

Marker ``gpu``: the test needs an AMD Instinct GPU and the built HIP library;
everything else runs on the CPU.
"""
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs a GPU and the built libmfgemm")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")
