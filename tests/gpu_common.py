"""Shared helpers of the GPU parity tests (inputs only; no arithmetic of the
method)."""
import sys

import numpy as np
import torch


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_np_state(t: torch.Tensor) -> np.ndarray:
    return t.detach().to("cpu").numpy().astype(np.complex128)
