"""Shared helpers for the GPU parity tests (inputs go to the device, results come back as numpy)."""
import os
import sys

import numpy as np
import pytest
import torch

from paper_2005_01372_amd import lsop


def require_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(lsop.LIB_PATH):
        pytest.fail("liblsop.so is not built: GPU tests need the HIP library (run the build first)")
    lsop.load_library()


def announce(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype).cuda().contiguous()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.complex128)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def make_op(w, dtype=lsop.C128, max_vec=16):
    op = lsop.Operator(w.nx, w.nz, dtype, max_vec)
    op.set_problem(torch.as_tensor(w.vel).cuda(), w.h, w.freq, w.c0)
    return op
