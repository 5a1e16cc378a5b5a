"""Shared helpers of the GPU parity tests (comparison metrics and gathers)."""
import sys

import numpy as np


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def vis_to_complex(vis_np):
    """[..][2] float/int pairs -> complex128."""
    v = vis_np.astype(np.float64)
    return v[..., 0] + 1j * v[..., 1]


def tri_indices(Na):
    a, b = np.tril_indices(Na)
    return a, b


def normalised_error(V, Vref, Na):
    """|V - Vref| / sqrt(Vref_ii Vref_jj) for [.., Nbl, 2, 2] complex arrays (one channel)."""
    a, b = tri_indices(Na)
    bl_aa = a * (a + 1) // 2 + a
    bl_bb = b * (b + 1) // 2 + b
    err = np.zeros(V.shape, np.float64)
    for p in range(2):
        for q in range(2):
            vii = Vref[..., bl_aa, p, p].real
            vjj = Vref[..., bl_bb, q, q].real
            den = np.sqrt(np.maximum(vii * vjj, 1e-300))
            err[..., p, q] = np.abs(V[..., p, q] - Vref[..., p, q]) / den
    return err


def gather_rows(z, sb, ch, inputs, S):
    """Samples of the listed receivers from the block layout on the GPU -> numpy [S][R][2]."""
    import torch
    idx = torch.as_tensor(list(inputs), device=z.device, dtype=torch.long)
    sub = z[sb, ch].index_select(1, idx)                 # [Sb][R][8][2]
    sub = sub.permute(0, 2, 1, 3).reshape(-1, len(inputs), 2)[:S]
    return sub.cpu().numpy()
