"""Helpers shared by the GPU parity tests (inputs from synth, references
from the oracle, results through the C ABI)."""
import numpy as np


def rel_err(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def banner(msg):
    print(f"\n[case] {msg}", flush=True)
