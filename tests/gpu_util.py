"""Helpers shared by the GPU parity tests."""
import numpy as np


def rel(a, b):
    """max |a - b| / max |b|"""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.abs(b).max()
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def announce(msg):
    print(f"[gpu] {msg}", flush=True)
