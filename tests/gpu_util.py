"""Helpers for GPU parity tests: seeded inputs to the device, oracle checks."""
import numpy as np

import oracle

FP64_TOL = 1e-12   # componentwise: |C_gpu - C_ref| <= FP64_TOL * (|A||B|)(c)


def to_dev(x, device="cuda"):
    import torch
    return torch.from_numpy(np.asarray(x)).to(device)


def colmajor_zeros(shape, device="cuda"):
    import paper_1307_2100_amd as tc
    C = tc.empty_colmajor(list(shape), device=device)
    C.zero_()
    return C


def componentwise_error(got, ref, scale):
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(got - ref) / scale)) if got.size else 0.0


def reference(A, labA, B, labB, labC, alpha=1.0, beta=0.0, C0=None):
    """Oracle result (compensated) and the componentwise error scale."""
    ref = oracle.contract(A, labA, B, labB, labC, mode="dot2")
    absr = oracle.contract(A, labA, B, labB, labC, mode="abs")
    if C0 is not None and beta != 0.0:
        ref = alpha * ref + beta * C0
        absr = abs(alpha) * absr + abs(beta) * np.abs(C0)
    else:
        ref = alpha * ref
        absr = abs(alpha) * absr
    return ref, absr
