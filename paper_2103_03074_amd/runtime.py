"""Torch-side helpers around the C ABI: device memory and streams only.

These allocate the caller-owned buffers of tn.h (workspace, float64
accumulator, amplitudes) as torch tensors on the current device and call the
library.  No arithmetic of the method happens here.
"""

import torch

from . import tn


def workspace(plan, device=None):
    """Workspace for tn_contract_slices (every lane the plan is set to use)
    and tn_amplitudes: the larger need."""
    s = plan.stats()
    n = max(int(s["lanes_workspace_bytes"]), int(s["tail_workspace_bytes"]), 256)
    return torch.empty(n, dtype=torch.uint8, device=device or "cuda")


def accumulator(plan, device=None):
    s = plan.stats()
    return torch.zeros(2 << int(s["acc_log2"]), dtype=torch.float64, device=device or "cuda")


def amplitudes(plan, slices=None, ws=None, acc=None, stream=None):
    """Contract the given slices (None = all; a (begin, end) pair; or a list of
    ids), sum them in float64 and return the amplitudes as a complex128 CUDA
    tensor of length 2^n_open."""
    s = plan.stats()
    ws = workspace(plan) if ws is None else ws
    acc = accumulator(plan) if acc is None else acc
    if slices is None:
        plan.contract_slices(ws, acc, 0, s["n_slices"], stream)
    elif isinstance(slices, tuple):
        plan.contract_slices(ws, acc, slices[0], slices[1], stream)
    else:
        plan.contract_slice_list(ws, acc, slices, stream)
    amps = torch.empty(2 << int(s["n_open"]), dtype=torch.float64, device=acc.device)
    plan.amplitudes(acc, amps, ws, stream)
    return torch.view_as_complex(amps.view(-1, 2))
