"""Helpers for the GPU parity tests: upload seeded inputs, run the oracle."""
import numpy as np
import torch

DEV = "cuda:0"


def dev(a, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def host(t):
    return t.detach().to("cpu").numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.linalg.norm(b)
    return np.linalg.norm(a - b) / (d if d > 0 else 1.0)


def bf16_tensor(a64):
    """FP64 array -> torch bfloat16 tensor on the GPU (round to nearest even
    through FP32, the generator's rounding)."""
    from workloads import to_bf16_bits
    bits = to_bf16_bits(a64).view(np.int16)
    return torch.from_numpy(bits.copy()).view(torch.bfloat16).to(DEV)


def bf16_values(a64):
    from workloads import to_bf16_bits, bf16_bits_to_f64
    return bf16_bits_to_f64(to_bf16_bits(a64))
