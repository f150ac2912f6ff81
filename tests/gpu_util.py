"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys


def note(msg: str):
    """Print and flush the name of the case about to run on the GPU."""
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


def rand_c(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
