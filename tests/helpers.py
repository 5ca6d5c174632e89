"""Shared test helpers: one seeded event, seen by the oracle and the library
through the same arrays."""
import dataclasses

import numpy as np

import oracle
from paper_2509_04336_amd import inputs


def both_sides(spec):
    """Oracle event, library spec and data for one workload, with the signal
    injected by the oracle (the oracle never receives anything computed by
    the library)."""
    ev, th, data = oracle.build_event(spec)
    spec2 = dataclasses.replace(spec, fixed_theta=np.array(ev._keep["fixed_theta"]))
    return ev, spec2, data, th


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


WORKLOADS = {
    "tiny": lambda: inputs.tiny_event(),
    "paper": lambda: inputs.paper_event(seed=0),
    "long": lambda: inputs.tiny_event(duration=8.0, f_hi=2048.0),
    "toy4": lambda: inputs.toy_event(4, 0.05),
}
