"""Seeded synthetic inputs shared by the oracle and the HIP path (no method arithmetic)."""
from .connectome import CONFIGS, Config, Connectome, make, make_batch, random_coo, fibonacci_sphere

__all__ = ["CONFIGS", "Config", "Connectome", "make", "make_batch", "random_coo", "fibonacci_sphere"]
